// LDS bandwidth calibration. The block solvers keep their tiles in LDS, so
// their LDS traffic is set against what the LDS of this GPU actually moves: a
// kernel that does nothing but write and read float4s through LDS at full
// occupancy, timed with HIP events on the caller's stream.
#include <cmath>

#include "hdi_internal.h"

namespace hdi {

constexpr int PROBE_THREADS = 256;
constexpr int PROBE_SLOTS = 4;   // independent float4 streams per lane

// Each iteration: every lane writes PROBE_SLOTS float4s to its own slots and
// reads the slots of its partner lane (lane ^ 1, in the same wavefront, whose
// LDS operations complete in issue order), 128 bytes per lane. The values read
// feed the next writes, so nothing can be elided; `key` is NaN, so the final
// store never happens but keeps the loop alive.
__global__ void __launch_bounds__(PROBE_THREADS) k_lds_probe(int iters, float key, float *__restrict__ sink) {
    __shared__ float4 buf[PROBE_SLOTS][PROBE_THREADS];
    const int t = threadIdx.x, o = t ^ 1;
    float4 a[PROBE_SLOTS];
#pragma unroll
    for (int q = 0; q < PROBE_SLOTS; ++q) a[q] = make_float4((float)(t + q), (float)(t - q), (float)q, 1.f);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int q = 0; q < PROBE_SLOTS; ++q) buf[q][t] = a[q];
#pragma unroll
        for (int q = 0; q < PROBE_SLOTS; ++q) {
            const float4 b = buf[q][o];
            a[q].x += b.y;
            a[q].y += b.z;
            a[q].z += b.w;
            a[q].w += b.x;
        }
    }
    const float acc = (a[0].x + a[1].y) + (a[2].z + a[3].w);
    if (acc == key) sink[0] = acc;
}

}  // namespace hdi

using namespace hdi;

extern "C" {

int32_t hdi_lds_calibrate(int32_t iters, float *sink, double *bytes_per_s, void *stream) {
    if (iters < 1 || iters > (1 << 20) || !sink || !bytes_per_s) {
        set_error("hdi_lds_calibrate: iters must lie in 1..2^20, sink and bytes_per_s must be non-null");
        return HDI_ERR_ARG;
    }
    *bytes_per_s = 0.0;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        set_error("hdi_lds_calibrate: no device");
        return HDI_ERR_HIP;
    }
    // 16 blocks of 4 wavefronts per CU (16 KB of LDS each): full occupancy
    const int blocks = 16 * cus;
    const float key = std::nanf("");
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        set_error("hdi_lds_calibrate: event creation failed");
        return HDI_ERR_HIP;
    }
    float best = 0.f;
    hipError_t e = hipSuccess;
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {   // the first run warms up
        (void)hipEventRecord(a, s);
        hipLaunchKernelGGL(k_lds_probe, dim3(blocks), dim3(PROBE_THREADS), 0, s, iters, key, sink);
        (void)hipEventRecord(b, s);
        e = hipGetLastError();
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventSynchronize(b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e == hipSuccess && rep > 0 && (best == 0.f || ms < best)) best = ms;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess || !(best > 0.f)) {
        set_error("hdi_lds_calibrate: %s", e != hipSuccess ? hipGetErrorString(e) : "no time measured");
        return HDI_ERR_HIP;
    }
    const double bytes = (double)blocks * PROBE_THREADS * iters * PROBE_SLOTS * 2.0 * sizeof(float4);
    *bytes_per_s = bytes / (best * 1e-3);
    return HDI_OK;
}

}  // extern "C"
