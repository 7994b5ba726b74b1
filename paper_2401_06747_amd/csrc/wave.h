// Device helpers shared by the kernel files: the grid degree, DPP wavefront
// sums and the XCD-aware workgroup remap.
#pragma once
#include <hip/hip_runtime.h>

namespace hdi {

__device__ __forceinline__ int deg_of(int x, int y, int W, int H) {
    return (x > 0) + (x < W - 1) + (y > 0) + (y < H - 1);
}

// Sum over the 64 lanes of a wavefront with DPP lane moves (no LDS traffic):
// pairs and quads, then shifts by 4 and 8 inside each row of 16, then the
// row broadcasts of lane 15 and lane 31. Lane 63 ends with the total; its value
// is broadcast, so every lane returns the same bits and the order of the
// additions is fixed (deterministic).
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_i(int x) {
    return __builtin_amdgcn_update_dpp(0, x, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f(float x) {
    return __int_as_float(dpp_i<CTRL, ROWS>(__float_as_int(x)));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double x) {
    const int lo = dpp_i<CTRL, ROWS>(__double2loint(x));
    const int hi = dpp_i<CTRL, ROWS>(__double2hiint(x));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_f<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v += dpp_f<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v += dpp_f<0x114, 0xF>(v);  // row_shr:4
    v += dpp_f<0x118, 0xF>(v);  // row_shr:8
    v += dpp_f<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_f<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
// Two sums over the wavefront at once (independent DPP chains, interleaved).
__device__ __forceinline__ void wave_sum2(float &a, float &b) {
    a += dpp_f<0xB1, 0xF>(a);
    b += dpp_f<0xB1, 0xF>(b);
    a += dpp_f<0x4E, 0xF>(a);
    b += dpp_f<0x4E, 0xF>(b);
    a += dpp_f<0x114, 0xF>(a);
    b += dpp_f<0x114, 0xF>(b);
    a += dpp_f<0x118, 0xF>(a);
    b += dpp_f<0x118, 0xF>(b);
    a += dpp_f<0x142, 0xA>(a);
    b += dpp_f<0x142, 0xA>(b);
    a += dpp_f<0x143, 0xC>(a);
    b += dpp_f<0x143, 0xC>(b);
    a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a), 63));
    b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(b), 63));
}
__device__ __forceinline__ double wave_sum_d(double v) {
    v += dpp_d<0xB1, 0xF>(v);
    v += dpp_d<0x4E, 0xF>(v);
    v += dpp_d<0x114, 0xF>(v);
    v += dpp_d<0x118, 0xF>(v);
    v += dpp_d<0x142, 0xA>(v);
    v += dpp_d<0x143, 0xC>(v);
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// Map the hardware workgroup id to a block index so that each of the 8 XCDs
// (workgroups are dealt round-robin to them) works on one contiguous band of
// blocks, and neighbouring blocks share that XCD's L2 for their halos.
__device__ __forceinline__ int xcd_remap(int bid, int n) {
    const int q = n >> 3, rem = n & 7;
    const int x = bid & 7, k = bid >> 3;
    return x * q + min(x, rem) + k;
}

}  // namespace hdi
