// Kernels of the masked-Laplace solve (paper Sec. 2.1 and Sec. 3) for gfx950.
//
// Operator: for pixel p with in-image 4-neighbours N4(p),
//   (L v)_p = deg(p) v_p - sum_{q in N4(p)} v_q,   deg(p) = |N4(p)|   (reflecting border)
//   (A v)_p = v_p if p is known, (L v)_p otherwise                 (eq. inp-discrete-lsi)
// The correction equation A e = r with r = 0 on known pixels pins e = 0 there,
// so every FP32 kernel below works on the unknown pixels only.
#include <algorithm>
#include <cfloat>

#include "hdi_internal.h"
#include "wave.h"

namespace hdi {

// ------------------------------------------------------------------ level-0 FP64 kernels

// u = u0 (or 0) on unknown pixels, u = data exactly on known pixels.
template <typename TD>
__device__ __forceinline__ void init_u_at(int i, int N, int C, const uint8_t *__restrict__ mask,
                                          const TD *__restrict__ data, const double *__restrict__ u0,
                                          double *__restrict__ u) {
    if (i >= N) return;
    const bool known = mask[i] != 0;
    for (int c = 0; c < C; ++c) {
        const size_t j = (size_t)c * N + i;
        u[j] = known ? (data ? (double)data[j] : 0.0) : (u0 ? u0[j] : 0.0);
    }
}

// keep_unknown: leave u on unknown pixels as it is (a warm start, or a start
// that the FMG prolongation overwrites there), so only known pixels are touched.
template <typename TD>
__global__ void k_init_u(int N, int C, const uint8_t *__restrict__ mask, const TD *__restrict__ data,
                         bool keep_unknown, double *__restrict__ u) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    if (keep_unknown && !mask[i]) return;
    init_u_at<TD>(i, N, C, mask, data, nullptr, u);
}

// Fused refinement step and FP64 residual. With e != nullptr the iterate is
// first advanced, u_out = u_in + e (e is exactly 0 on known pixels, so known
// values stay bit-exact), and the residual is taken at u_out; u_out must not
// alias u_in because neighbours read u_in. A null u_in is the zero iterate
// (nothing is read for it; the values are those of a zero-filled u_in). Then r = b - A u in FP64 with
// b = data on known pixels and src (or 0) elsewhere, stored as FP32 for the
// inner solve, plus per-workgroup FP64 partial sums of r^2 and b^2 per channel.
//
// Access pattern: each wave owns 62 columns (its 64 lanes minus one halo lane
// on each side) and sweeps RES_BAND rows downwards, keeping the rows y-1, y,
// y+1 of every channel in registers and prefetching row y+2, so each element
// is read from memory once (plus two halo rows per band). Left and right
// neighbours come from the adjacent lanes by whole-wave DPP shifts. One thread
// serves all channels, so the mask is read once (Sec. 2.1: the colour channels
// share the matrix).
constexpr int RES_BAND = 32;
constexpr int RES_COLS = 62;

__device__ __forceinline__ double wave_from_left(double v) {   // value of lane - 1
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x138, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x138, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_from_right(double v) {  // value of lane + 1
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x130, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x130, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// SRC: the right-hand side off the mask is src (a source problem, data absent);
// otherwise the problem has data on the mask and zero source. Each variant
// keeps only the registers its right-hand side needs.
template <typename TD, int C, bool SRC>
__device__ __forceinline__ void residual_block(int W, int H, const uint8_t *__restrict__ mask,
                                               const double *__restrict__ u_in, const float *__restrict__ e,
                                               double *__restrict__ u_out, const TD *__restrict__ data,
                                               const double *__restrict__ src, float *__restrict__ r,
                                               double *__restrict__ partials, int nblk, int bx, int by, int gx) {
    const int N = W * H;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int x = (bx * (RED_THREADS / 64) + wid) * RES_COLS + lane - 1;
    const int xs = min(max(x, 0), W - 1);
    const bool owner = lane >= 1 && lane <= RES_COLS && x < W;
    const double wl = x > 0, wr = x < W - 1;
    const int y0 = by * RES_BAND, y1 = min(y0 + RES_BAND, H);
    const int bid = by * gx + bx;

    // Rows of u (+ e) at column xs: prev (y-1), cur (y), next (y+1), and the
    // prefetched y+2; mask rows y and y+1; src of row y. Loads are issued one
    // or two rows ahead, and everything row y needs was issued in an earlier
    // iteration, so the in-order memory counter never makes the wave wait for
    // its own prefetch. The data on known pixels is not read: there the
    // iterate holds it exactly (set at the start, and every correction is 0
    // there), so b = u on known pixels.
    auto fetch = [&](int c, int y, double &uv, float &ev) {
        const int yc = min(max(y, 0), H - 1);
        const size_t j = (size_t)c * N + (size_t)yc * W + xs;
        uv = u_in ? u_in[j] : 0.0;
        ev = e ? e[j] : 0.f;
    };
    auto fetch_mask = [&](int y) -> int { return mask[(size_t)min(y, H - 1) * W + xs]; };
    // source term of row y (source problems; 0 otherwise)
    auto fetch_b = [&](int y, double *sv) {
        const size_t i = (size_t)min(y, H - 1) * W + xs;
#pragma unroll
        for (int c = 0; c < C; ++c) sv[c] = SRC ? src[(size_t)c * N + i] : 0.0;
    };
    double pu[C], cu[C], nu[C], qu[C];
    float pe[C], ce[C], ne[C], qe[C];
    double scur[C], snxt[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        fetch(c, y0 - 1, pu[c], pe[c]);
        fetch(c, y0, cu[c], ce[c]);
        fetch(c, y0 + 1, nu[c], ne[c]);
    }
    int mcur = fetch_mask(y0), mnxt = fetch_mask(y0 + 1);
    fetch_b(y0, scur);
    double rr[C], bb[C];
#pragma unroll
    for (int c = 0; c < C; ++c) rr[c] = bb[c] = 0.0;
    for (int y = y0; y < y1; ++y) {
        // issue the loads for later rows first
#pragma unroll
        for (int c = 0; c < C; ++c) fetch(c, y + 2, qu[c], qe[c]);
        const int mq = fetch_mask(y + 2);
        fetch_b(y + 1, snxt);
        // then compute row y from registers
        const size_t i = (size_t)y * W + xs;
        const bool known = mcur != 0;
        const double wu = y > 0, wd = y < H - 1;
        const double dgv = wl + wr + wu + wd;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const size_t o = (size_t)c * N;
            const double u0 = cu[c] + (double)ce[c];
            const double ul = wave_from_left(u0), ur = wave_from_right(u0);
            const double uu = pu[c] + (double)pe[c], ud = nu[c] + (double)ne[c];
            const double au = dgv * u0 - (wl * ul + wr * ur + wu * uu + wd * ud);
            const double b = known ? u0 : scur[c];
            const double res = known ? b - u0 : b - au;
            if (owner) {
                if (e) u_out[o + i] = u0;
                r[o + i] = (float)res;
                rr[c] += res * res;
                bb[c] += b * b;
            }
            pu[c] = cu[c]; pe[c] = ce[c];
            cu[c] = nu[c]; ce[c] = ne[c];
            nu[c] = qu[c]; ne[c] = qe[c];
            scur[c] = snxt[c];
        }
        mcur = mnxt;
        mnxt = mq;
    }
    __shared__ double s_red[RED_THREADS / 64][2 * C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const double a = wave_sum_d(rr[c]);
        const double b = wave_sum_d(bb[c]);
        if (lane == 0) { s_red[wid][2 * c] = a; s_red[wid][2 * c + 1] = b; }
    }
    __syncthreads();
    if (threadIdx.x < 2 * C) {
        double acc = 0.0;
        for (int w = 0; w < RED_THREADS / 64; ++w) acc += s_red[w][threadIdx.x];
        const int c = threadIdx.x >> 1;
        partials[((size_t)c * nblk + bid) * 2 + (threadIdx.x & 1)] = acc;
    }
}

template <typename TD, int C, bool SRC>
__global__ void __launch_bounds__(RED_THREADS)
k_residual(int W, int H, const uint8_t *__restrict__ mask, const double *__restrict__ u_in,
           const float *__restrict__ e, double *__restrict__ u_out, const TD *__restrict__ data,
           const double *__restrict__ src, float *__restrict__ r, double *__restrict__ partials, int nblk) {
    residual_block<TD, C, SRC>(W, H, mask, u_in, e, u_out, data, src, r, partials, nblk, blockIdx.x, blockIdx.y,
                               gridDim.x);
}

// Second stage of the fixed-order reduction: one workgroup of 1024 threads per
// channel; thread t sums partials t, t+1024, ... in order, then waves and the
// 16 wave sums are combined in a fixed order.
__device__ __forceinline__ void reduce_partials_block(int nblk, const double *__restrict__ partials,
                                                      double *__restrict__ norms, int c) {
    double a = 0.0, b = 0.0;
    const double2 *pp = reinterpret_cast<const double2 *>(partials) + (size_t)c * nblk;
#pragma unroll 4
    for (int k = threadIdx.x; k < nblk; k += 1024) {
        const double2 v = pp[k];
        a += v.x;
        b += v.y;
    }
    a = wave_sum_d(a);
    b = wave_sum_d(b);
    __shared__ double s[16][2];
    if ((threadIdx.x & 63) == 0) { s[threadIdx.x >> 6][0] = a; s[threadIdx.x >> 6][1] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0.0, y = 0.0;
        for (int w = 0; w < 16; ++w) { x += s[w][0]; y += s[w][1]; }
        norms[c * 2 + 0] = x;
        norms[c * 2 + 1] = y;
    }
}

__global__ void __launch_bounds__(1024)
k_reduce_partials(int nblk, const double *__restrict__ partials, double *__restrict__ norms) {
    reduce_partials_block(nblk, partials, norms, blockIdx.x);
}

// u += e on unknown pixels (iterative refinement step, FP64).
__global__ void k_update(int N, int C, const uint8_t *__restrict__ mask, const float *__restrict__ e,
                         double *__restrict__ u) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N || mask[i]) return;
    for (int c = 0; c < C; ++c) u[(size_t)c * N + i] += (double)e[(size_t)c * N + i];
}

// ------------------------------------------------------------------ grid transfers

// Workgroup total of a per-thread count, added with one atomic per workgroup
// (integer atomics: exact and order independent).
__device__ __forceinline__ void block_count_add(unsigned int local, unsigned int *count) {
    __shared__ unsigned int s_cnt[4];
    for (int o = 32; o >= 1; o >>= 1) local += __shfl_xor(local, o, 64);
    if ((threadIdx.x & 63) == 0) s_cnt[threadIdx.x >> 6] = local;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int t = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
        if (t) atomicAdd(count, t);
    }
}

// Coarse mask: a coarse pixel is known if any of its (up to) four fine pixels
// is known (Sec. 3.3). Also counts the known coarse pixels. Grid-stride loop
// over coarse pixels, 256 threads per workgroup.
__device__ __forceinline__ void mask_restrict_block(int W, int H, const uint8_t *__restrict__ m, int Wc, int Hc,
                                                    uint8_t *__restrict__ mc, unsigned int *__restrict__ count,
                                                    int blk, int nblks) {
    unsigned int local = 0;
    for (int i = blk * 256 + threadIdx.x; i < Wc * Hc; i += nblks * 256) {
        const int X = i % Wc, Y = i / Wc;
        uint8_t k = 0;
        for (int j = 0; j < 2; ++j)
            for (int q = 0; q < 2; ++q) {
                const int x = 2 * X + q, y = 2 * Y + j;
                if (x < W && y < H) k |= (m[y * W + x] != 0);
            }
        mc[i] = k;
        local += k;
    }
    block_count_add(local, count);
}

__global__ void __launch_bounds__(256)
k_mask_restrict(int W, int H, const uint8_t *__restrict__ m, int Wc, int Hc, uint8_t *__restrict__ mc,
                unsigned int *__restrict__ count) {
    mask_restrict_block(W, H, m, Wc, Hc, mc, count, blockIdx.x, gridDim.x);
}

// Known pixels of the finest mask.
__device__ __forceinline__ void count_known_block(int N, const uint8_t *__restrict__ m, unsigned int *__restrict__ count,
                                                  int blk, int nblks) {
    unsigned int local = 0;
    for (int i = blk * 256 + threadIdx.x; i < N; i += nblks * 256) local += m[i] != 0;
    block_count_add(local, count);
}

__global__ void __launch_bounds__(256)
k_count_known(int N, const uint8_t *__restrict__ m, unsigned int *__restrict__ count) {
    count_known_block(N, m, count, blockIdx.x, gridDim.x);
}

__global__ void k_zero_u32(int n, unsigned int *p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Coarse right-hand side: sum over the unknown fine children of the fine
// residual r - A e (the coarse operator is the same stencil on the coarse grid,
// so summing four children scales the averaged residual by H^2/h^2 = 4).
// Zero on coarse known pixels, where the coarse correction is pinned.
// Branch-free: the thread loads the 4x4 fine neighbourhood of its 2x2 children
// (corners excluded) from clamped addresses, all loads in flight at once, and
// validity (inside the image, unknown child) enters through selects.
__device__ __forceinline__ void restrict_residual_at(int i, int W, int H, int C, const uint8_t *__restrict__ m,
                                                     const float *__restrict__ r, const float *__restrict__ e, int Wc,
                                                     int Hc, const uint8_t *__restrict__ mc, float *__restrict__ rc) {
    if (i >= Wc * Hc) return;
    const int X = i % Wc, Y = i / Wc;
    const int N = W * H, Nc = Wc * Hc;
    // fine columns 2X-1 .. 2X+2 and rows 2Y-1 .. 2Y+2: clamped index, inside flag
    int xs[4], ys[4];
    bool vx[4], vy[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int x = 2 * X - 1 + k, y = 2 * Y - 1 + k;
        vx[k] = x >= 0 && x < W;
        vy[k] = y >= 0 && y < H;
        xs[k] = min(max(x, 0), W - 1);
        ys[k] = min(max(y, 0), H - 1);
    }
    bool unk[2][2];
#pragma unroll
    for (int jc = 0; jc < 2; ++jc)
#pragma unroll
        for (int qc = 0; qc < 2; ++qc)
            unk[jc][qc] = vx[1 + qc] && vy[1 + jc] && m[ys[1 + jc] * W + xs[1 + qc]] == 0;
    const bool cknown = mc[i] != 0;
    for (int c = 0; c < C; ++c) {
        const float *ecn = e + (size_t)c * N;
        const float *rcn = r + (size_t)c * N;
        float E[4][4], R[2][2];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if ((a == 0 || a == 3) && (b == 0 || b == 3))
                    E[a][b] = 0.f;   // corners: not a neighbour of any child
                else
                    E[a][b] = ecn[ys[a] * W + xs[b]];
#pragma unroll
        for (int jc = 0; jc < 2; ++jc)
#pragma unroll
            for (int qc = 0; qc < 2; ++qc) R[jc][qc] = rcn[ys[1 + jc] * W + xs[1 + qc]];
        float acc = 0.f;
#pragma unroll
        for (int jc = 0; jc < 2; ++jc)
#pragma unroll
            for (int qc = 0; qc < 2; ++qc) {
                const int a = 1 + jc, b = 1 + qc;
                const float s = (vx[b - 1] ? E[a][b - 1] : 0.f) + (vx[b + 1] ? E[a][b + 1] : 0.f) +
                                (vy[a - 1] ? E[a - 1][b] : 0.f) + (vy[a + 1] ? E[a + 1][b] : 0.f);
                const float d = (float)((int)vx[b - 1] + (int)vx[b + 1] + (int)vy[a - 1] + (int)vy[a + 1]);
                const float res = R[jc][qc] - (d * E[a][b] - s);
                acc += unk[jc][qc] ? res : 0.f;
            }
        rc[(size_t)c * Nc + i] = cknown ? 0.f : acc;
    }
}

// Consecutive workgroups (coarse rows, in order) go to one XCD, so the fine
// rows that neighbouring coarse rows share are read from that XCD's L2.
__global__ void k_restrict_residual(int W, int H, int C, const uint8_t *__restrict__ m,
                                    const float *__restrict__ r, const float *__restrict__ e,
                                    int Wc, int Hc, const uint8_t *__restrict__ mc, float *__restrict__ rc) {
    restrict_residual_at(xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x, W, H, C, m, r, e, Wc, Hc, mc,
                         rc);
}

// Cell-centred bilinear prolongation weights: fine x maps to coarse position
// x/2 - 1/4, i.e. 3/4 of the parent and 1/4 of the next coarse cell on x's side.
__device__ __forceinline__ float prolong_at(const float *__restrict__ ec, int Wc, int Hc, int x, int y) {
    const int X = x >> 1, Y = y >> 1;
    const int Xn = min(max((x & 1) ? X + 1 : X - 1, 0), Wc - 1);
    const int Yn = min(max((y & 1) ? Y + 1 : Y - 1, 0), Hc - 1);
    const float a = ec[Y * Wc + X], b = ec[Y * Wc + Xn];
    const float c = ec[Yn * Wc + X], d = ec[Yn * Wc + Xn];
    return 0.5625f * a + 0.1875f * (b + c) + 0.0625f * d;
}

// ------------------------------------------------------------------ Schwarz block smoother

// One restricted additive Schwarz step (Sec. 3.1) on T x T blocks (T = 32 or
// 16): each block solves its local problem A_i v_i = R_i r^n with zero
// Dirichlet values outside the block (interior block boundaries) and the
// reflecting condition at the image border, by `iters` steps of conjugate
// gradients (Sec. 3.3). The correction is written back only on the pixels the
// block owns (the middle of each overlap splits ownership), which is a
// partition of unity with 0/1 weights (eq. partition-of-unity-discrete).
//
// Layout: one wavefront (64 lanes) per block; lane (bx, by) = (lane & 7,
// lane >> 3) holds the PS x PS pixels (PS bx + i, PS by + j), PS = T / 8, in
// registers. The current vector is exchanged through LDS (a (T+2)-row float
// tile with a zero halo ring), dot products use wavefront shuffles, so the
// block needs no barrier beyond its own wave. Small tiles give four times as
// many waves with a quarter of the work each, which pays on the coarse levels
// of the V-cycle, where there are few blocks and the latency of each step
// dominates.
//
// MODE 0: pre-smoothing from e = 0 (reads r only)
// MODE 1: post-smoothing of e_in + P ec (reads e_in with a 1-pixel halo and
//         the coarse correction ec around the block)
// MODE 2: FMG smoothing from the prolongated guess e_in (like MODE 1 with ec = 0)
constexpr int COL0 = 4;     // LDS column of block column 0 (columns 3 and T + 4 are the halo)

template <int T> struct TileGeom {
    static constexpr int PS = T / 8;          // pixels per lane and dimension
    static constexpr int NPX = PS * PS;       // pixels per lane
    static constexpr int LW = T + 8;          // LDS row pitch (floats; rows stay 16-byte aligned)
    static constexpr int NC = T / 2 + 4;      // coarse correction staged around the block
};

// PS consecutive floats of one LDS row, as one vector access
template <int PS>
__device__ __forceinline__ void lds_put(float *dst, const float *v) {
    if constexpr (PS == 4)
        *reinterpret_cast<float4 *>(dst) = make_float4(v[0], v[1], v[2], v[3]);
    else
        *reinterpret_cast<float2 *>(dst) = make_float2(v[0], v[1]);
}
template <int PS>
__device__ __forceinline__ void lds_get(const float *src, float *v) {
    if constexpr (PS == 4) {
        const float4 a = *reinterpret_cast<const float4 *>(src);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    } else {
        const float2 a = *reinterpret_cast<const float2 *>(src);
        v[0] = a.x; v[1] = a.y;
    }
}

// Cell-centred bilinear prolongation of a coarse correction: 3/4 of the parent
// cell, 1/4 of the next cell on each side of x and y (a = parent, b and c the
// next cells along x and along y, d the diagonal one).
__device__ __forceinline__ float bilinear(float a, float b, float c, float d) {
    return 0.5625f * a + 0.1875f * (b + c) + 0.0625f * d;
}

// P ec at a lane's PS x PS pixels from the (PS/2 + 2)^2 coarse cells around
// them, cc[0][0] being the cell left of and above the first pixel's parent;
// PX, PY: the parity of the first pixel's x and y (every lane of a block has
// the same).
template <int PS, int PX, int PY>
__device__ __forceinline__ void prolong_patch(const float (&cc)[PS / 2 + 2][PS / 2 + 2], float *out) {
#pragma unroll
    for (int j = 0; j < PS; ++j)
#pragma unroll
        for (int i = 0; i < PS; ++i) {
            const int X = ((i + PX) >> 1) + 1, Xn = ((i + PX) & 1) ? X + 1 : X - 1;
            const int Y = ((j + PY) >> 1) + 1, Yn = ((j + PY) & 1) ? Y + 1 : Y - 1;
            out[j * PS + i] = bilinear(cc[Y][X], cc[Y][Xn], cc[Yn][X], cc[Yn][Xn]);
        }
}

template <int MODE, int T>
__device__ __forceinline__ void schwarz_block(int W, int H, int ntx, int nty, int sx, int sy, int iters, float robin,
                                              float stop_sq, const uint8_t *__restrict__ mask,
                                              const float *__restrict__ r,
                                              const float *__restrict__ e_in, const float *__restrict__ ec, int Wc,
                                              int Hc, float *__restrict__ e_out, const int t, const int c) {
    using G = TileGeom<T>;
    constexpr int PS = G::PS, NPX = G::NPX, LW = G::LW, NC = G::NC;
    // s_p: the vector of the current CG step with a zero ring; before that it
    // holds the starting correction with its 1-pixel halo (MODE 1/2)
    __shared__ __attribute__((aligned(16))) float s_p[T + 2][LW];
    __shared__ uint8_t s_m[MODE == 2 ? T + 2 : 1][T + 2];
    __shared__ float s_c[MODE == 1 ? NC : 1][NC];   // coarse correction around the block (MODE 1)

    const int tx = t % ntx, ty = t / ntx;
    const int Tx = min(T, W), Ty = min(T, H);
    const int x0 = min(tx * sx, W - Tx), y0 = min(ty * sy, H - Ty);
    const int N = W * H;
    const float *rc = r + (size_t)c * N;
    const int lane = threadIdx.x;
    const int bx = lane & 7, by = lane >> 3;

    // The lane's own right-hand side goes straight to registers (8 lanes
    // cover a block row); addresses are clamped so every load is unconditional.
    // MODE 0 and 1 take the lane's own mask values (and in MODE 1 its part of
    // the pre-smoothed correction) the same way.
    float rown[NPX];
    uint8_t mown[MODE != 2 ? NPX : 1];
    float eown[MODE == 1 ? NPX : 1];
#pragma unroll
    for (int j = 0; j < PS; ++j)
#pragma unroll
        for (int i = 0; i < PS; ++i) {
            const int xc = min(x0 + PS * bx + i, W - 1), yc = min(y0 + PS * by + j, H - 1);
            rown[j * PS + i] = r ? rc[yc * W + xc] : 0.f;
            if constexpr (MODE != 2) mown[j * PS + i] = mask[yc * W + xc];
            if constexpr (MODE == 1) eown[j * PS + i] = e_in[(size_t)c * N + yc * W + xc];
        }
    // MODE 1: the coarse correction around the block, with clamped coordinates
    // so that the clamped bilinear lookup becomes plain indexing; its loads are
    // in flight together with the first staging batch.
    const int X0 = ((x0 - 1) >> 1) - 1, Y0 = ((y0 - 1) >> 1) - 1;
    constexpr int NCS = NC * NC;
    constexpr int NCV = (NCS + 63) / 64;
    // MODE 1: the block's 1-pixel halo ring (4T + 4 pixels: rows 0 and T + 1
    // of the tile, then the two halo columns of rows 1..T), loaded with the
    // rest so that every load is in flight at once.
    constexpr int NRING = 4 * T + 4;
    constexpr int NRV = (NRING + 63) / 64;
    float cv[MODE == 1 ? NCV : 1];
    int rmk[MODE == 1 ? NRV : 1];
    float rev[MODE == 1 ? NRV : 1];
    auto ring_pos = [&](int k, int &lx, int &ly) {
        if (k < 2 * (T + 2)) {
            ly = k < T + 2 ? 0 : T + 1;
            lx = k % (T + 2);
        } else {
            ly = 1 + (k - 2 * (T + 2)) / 2;
            lx = (k & 1) ? T + 1 : 0;
        }
    };
    if constexpr (MODE == 1) {
        const float *ecc = ec + (size_t)c * Wc * Hc;
#pragma unroll
        for (int h = 0; h < NCV; ++h) {
            const int k = min(lane + 64 * h, NCS - 1);
            const int X = min(max(X0 + k % NC, 0), Wc - 1), Y = min(max(Y0 + k / NC, 0), Hc - 1);
            cv[h] = ecc[Y * Wc + X];
        }
#pragma unroll
        for (int h = 0; h < NRV; ++h) {
            int lx, ly;
            ring_pos(min(lane + 64 * h, NRING - 1), lx, ly);
            const int pc = min(max(y0 + ly - 1, 0), H - 1) * W + min(max(x0 + lx - 1, 0), W - 1);
            rmk[h] = mask[pc];
            rev[h] = e_in[(size_t)c * N + pc];
        }
    }
    // MODE 1: the starting correction e_in + P ec on unknown pixels (0 on
    // known ones and outside the image). e_in is exactly 0 on known pixels.
    // The ring goes to the tile pixel by pixel; the lane's own pixels are
    // computed in registers from the coarse cells around them and published.
    float e_st[MODE == 1 ? NPX : 1];
    if constexpr (MODE == 1) {
#pragma unroll
        for (int h = 0; h < NCV; ++h) {
            const int k = lane + 64 * h;
            if (k < NCS) s_c[k / NC][k % NC] = cv[h];
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < NRV; ++h) {
            const int k = lane + 64 * h;
            if (k < NRING) {
                int lx, ly;
                ring_pos(k, lx, ly);
                const int x = x0 + lx - 1, y = y0 + ly - 1;
                float v = 0.f;
                if (x >= 0 && x < W && y >= 0 && y < H && rmk[h] == 0) {
                    const int X = (x >> 1) - X0, Y = (y >> 1) - Y0;
                    const int Xn = (x & 1) ? X + 1 : X - 1, Yn = (y & 1) ? Y + 1 : Y - 1;
                    v = rev[h] + bilinear(s_c[Y][X], s_c[Y][Xn], s_c[Yn][X], s_c[Yn][Xn]);
                }
                s_p[ly][COL0 - 1 + lx] = v;
            }
        }
        constexpr int NCC = PS / 2 + 2;
        const int xs = x0 + PS * bx, ys = y0 + PS * by;
        const int Xb = (xs >> 1) - 1 - X0, Yb = (ys >> 1) - 1 - Y0;
        float cc[NCC][NCC];
#pragma unroll
        for (int a = 0; a < NCC; ++a)
#pragma unroll
            for (int b = 0; b < NCC; ++b) cc[a][b] = s_c[Yb + a][Xb + b];
        switch ((xs & 1) | ((ys & 1) << 1)) {
            case 0: prolong_patch<PS, 0, 0>(cc, e_st); break;
            case 1: prolong_patch<PS, 1, 0>(cc, e_st); break;
            case 2: prolong_patch<PS, 0, 1>(cc, e_st); break;
            default: prolong_patch<PS, 1, 1>(cc, e_st); break;
        }
#pragma unroll
        for (int j = 0; j < PS; ++j)
#pragma unroll
            for (int i = 0; i < PS; ++i) {
                const int k = j * PS + i;
                const bool act = PS * bx + i < Tx && PS * by + j < Ty && mown[k] == 0;
                e_st[k] = act ? eown[k] + e_st[k] : 0.f;
            }
#pragma unroll
        for (int j = 0; j < PS; ++j) lds_put<PS>(&s_p[PS * by + j + 1][COL0 + PS * bx], &e_st[j * PS]);
    }

    // MODE 2: stage mask and the starting correction (the data on known
    // pixels) for the block and a 1-pixel halo, in coalesced rows of T + 2.
    // s_m: 0 unknown, 1 known, 2 outside the image.
    constexpr int NST = (T + 2) * (T + 2);
    constexpr int NIT = (NST + 63) / 64;
    constexpr int HALF = (NIT + 1) / 2;      // staged in two batches to bound register use
#pragma unroll
    for (int batch = 0; batch < (MODE == 2 ? 2 : 0); ++batch) {
        int mraw[HALF];
        float ev[HALF];
#pragma unroll
        for (int h = 0; h < HALF; ++h) {
            const int k = lane + 64 * (batch * HALF + h);
            const int ly = k / (T + 2), lx = k % (T + 2);
            const int xc = min(max(x0 + lx - 1, 0), W - 1), yc = min(max(y0 + ly - 1, 0), H - 1);
            const int pc = yc * W + xc;
            mraw[h] = mask[pc];
            ev[h] = MODE != 0 ? e_in[(size_t)c * N + pc] : 0.f;
        }
#pragma unroll
        for (int h = 0; h < HALF; ++h) {
            const int k = lane + 64 * (batch * HALF + h);
            if (k < NST) {
                const int ly = k / (T + 2), lx = k % (T + 2);
                const int x = x0 + lx - 1, y = y0 + ly - 1;
                const bool in = x >= 0 && x < W && y >= 0 && y < H;
                s_m[ly][lx] = (uint8_t)(in ? (mraw[h] != 0) : 2);
                s_p[ly][COL0 - 1 + lx] = in ? ev[h] : 0.f;
            }
        }
    }
    if constexpr (MODE != 0) __syncthreads();

    // Local right-hand side r - A e_start on the block's unknown pixels; the
    // CG iterate v starts at e_start (so it is the final correction), and the
    // local residual at the right-hand side.
    float v[NPX], rl[NPX], dg[NPX];
#pragma unroll
    for (int j = 0; j < PS; ++j)
#pragma unroll
        for (int i = 0; i < PS; ++i) {
            const int lx = PS * bx + i, ly = PS * by + j, k = j * PS + i;
            const int x = x0 + lx, y = y0 + ly;
            float res = 0.f, d = 0.f, e0 = 0.f;
            const bool inside = lx < Tx && ly < Ty;
            if constexpr (MODE == 1) e0 = e_st[k];
            if (MODE == 2 && inside) e0 = s_p[ly + 1][COL0 + lx];
            bool unknown;
            if constexpr (MODE != 2)
                unknown = inside && mown[k] == 0;
            else
                unknown = inside && s_m[ly + 1][lx + 1] == 0;
            if (unknown) {
                d = (float)deg_of(x, y, W, H);
                res = rown[k];
                if (MODE != 0) {
                    const float sn = s_p[ly][COL0 + lx] + s_p[ly + 2][COL0 + lx] +
                                     s_p[ly + 1][COL0 + lx - 1] + s_p[ly + 1][COL0 + lx + 1];
                    res -= d * e0 - sn;
                }
            }
            // local operator: an edge to a pixel outside the block (not the
            // image border) adds 1 - robin to the diagonal (Robin transmission
            // condition; robin = 0 is a zero Dirichlet value outside)
            const int cross = (lx == 0 && x > 0) + (lx == Tx - 1 && x < W - 1) + (ly == 0 && y > 0) +
                              (ly == Ty - 1 && y < H - 1);
            dg[k] = d > 0.f ? d - robin * (float)cross : 0.f;
            v[k] = e0;
            rl[k] = res;
        }
    if constexpr (MODE != 0) __syncthreads();   // every lane has read the starting correction
    // zero ring (Dirichlet values outside the block): rows 0 and T + 1, and the
    // two halo columns of rows 1..T (the first step's barrier orders it before
    // any read)
    for (int k = lane; k < 2 * (T + 2) + 2 * T; k += 64) {
        if (k < 2 * (T + 2))
            s_p[k < T + 2 ? 0 : T + 1][COL0 - 1 + k % (T + 2)] = 0.f;
        else
            s_p[1 + (k - 2 * (T + 2)) / 2][(k & 1) ? COL0 + T : COL0 - 1] = 0.f;
    }

    // Local CG in the Chronopoulos-Gear arrangement: each step applies the
    // block operator to the residual and takes both inner products, (r, r) and
    // (A r, r), in one merged wavefront reduction; the directions follow from
    // the recurrences p = r + beta p, s = A r + beta s (s = A p). It stops after
    // `iters` steps, once the block residual has fallen to the FP32 rounding
    // floor (squared norm 1e-14 of the start), or once its squared norm is at
    // most stop_sq (the global-relative stop of Sec. 3.3; 0: off); the
    // reciprocals also need normal (not denormal) divisors.
    float p[NPX], sv[NPX];
#pragma unroll
    for (int k = 0; k < NPX; ++k) p[k] = sv[k] = 0.f;
    float gamma_prev = 1.f, alpha_prev = 1.f, rr_floor = 0.f;
    for (int it = 0; it < iters; ++it) {
        // publish r
#pragma unroll
        for (int j = 0; j < PS; ++j) lds_put<PS>(&s_p[PS * by + j + 1][COL0 + PS * bx], &rl[j * PS]);
        __syncthreads();
        float upv[PS], dnv[PS], lf[PS], rt[PS];
        lds_get<PS>(&s_p[PS * by][COL0 + PS * bx], upv);
        lds_get<PS>(&s_p[PS * by + PS + 1][COL0 + PS * bx], dnv);
#pragma unroll
        for (int j = 0; j < PS; ++j) {
            lf[j] = s_p[PS * by + j + 1][COL0 + PS * bx - 1];
            rt[j] = s_p[PS * by + j + 1][COL0 + PS * bx + PS];
        }
        float w[NPX];
        float gamma = 0.f, delta = 0.f;
#pragma unroll
        for (int j = 0; j < PS; ++j)
#pragma unroll
            for (int i = 0; i < PS; ++i) {
                const int k = j * PS + i;
                const float n = (j > 0 ? rl[k - PS] : upv[i]) + (j < PS - 1 ? rl[k + PS] : dnv[i]) +
                                (i > 0 ? rl[k - 1] : lf[j]) + (i < PS - 1 ? rl[k + 1] : rt[j]);
                w[k] = dg[k] > 0.f ? dg[k] * rl[k] - n : 0.f;
                gamma += rl[k] * rl[k];
                delta += w[k] * rl[k];
            }
        wave_sum2(gamma, delta);
        if (it == 0) rr_floor = fmaxf(gamma * 1e-14f, stop_sq);
        if (!(gamma > rr_floor && gamma >= FLT_MIN)) break;
        const float beta = it == 0 ? 0.f : gamma * __builtin_amdgcn_rcpf(gamma_prev);
        const float denom = delta - beta * gamma * __builtin_amdgcn_rcpf(alpha_prev);
        if (!(denom >= FLT_MIN)) break;
        const float alpha = gamma * __builtin_amdgcn_rcpf(denom);
#pragma unroll
        for (int k = 0; k < NPX; ++k) {
            p[k] = rl[k] + beta * p[k];
            sv[k] = w[k] + beta * sv[k];
            v[k] += alpha * p[k];
            rl[k] -= alpha * sv[k];
        }
        gamma_prev = gamma;
        alpha_prev = alpha;
        __syncthreads();
    }

    // Restricted write-back on the owned part of the block.
    const int xlo = tx == 0 ? 0 : (min((tx - 1) * sx, W - Tx) + Tx + x0) / 2;
    const int xhi = tx == ntx - 1 ? W : (x0 + Tx + min((tx + 1) * sx, W - Tx)) / 2;
    const int ylo = ty == 0 ? 0 : (min((ty - 1) * sy, H - Ty) + Ty + y0) / 2;
    const int yhi = ty == nty - 1 ? H : (y0 + Ty + min((ty + 1) * sy, H - Ty)) / 2;
    // v is the starting correction plus the local CG update; on known pixels
    // it kept its start (0 in MODE 0/1, the data in MODE 2)
    float *eo = e_out + (size_t)c * N;
#pragma unroll
    for (int j = 0; j < PS; ++j)
#pragma unroll
        for (int i = 0; i < PS; ++i) {
            const int lx = PS * bx + i, ly = PS * by + j;
            const int x = x0 + lx, y = y0 + ly;
            if (lx < Tx && ly < Ty && x >= xlo && x < xhi && y >= ylo && y < yhi) eo[y * W + x] = v[j * PS + i];
        }
}

// Squared-residual level below which a block's local CG stops: the fraction
// `frac` of the channel's global squared residual norm (gnorm[c * stride],
// FP64), or 0 without one (Sec. 3.3).
__device__ __forceinline__ float local_stop_sq(const double *__restrict__ gnorm, int stride, float frac, int c) {
    return gnorm && frac > 0.f ? (float)((double)frac * gnorm[(size_t)c * stride]) : 0.f;
}

// The refinement's stopping test on the norms of a residual sweep (rr, bb per
// channel, C <= 3), squared: rr <= tol^2 bb for every channel (rr <= tol^2
// where bb = 0). A NaN fails it. The caller passes tol with a relative margin
// far above rounding, so that a met test here implies the host's test
// sqrt(rr / bb) <= its tolerance on the same norms.
__device__ __forceinline__ bool residual_met(const double *norms, int C, double tol) {
    const double t2 = tol * tol;
    double rr[3], bb[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        rr[c] = c < C ? norms[2 * c] : 0.0;
        bb[c] = c < C ? norms[2 * c + 1] : 0.0;
    }
    bool met = true;
#pragma unroll
    for (int c = 0; c < 3; ++c) met = met && (bb[c] > 0.0 ? rr[c] <= t2 * bb[c] : rr[c] <= t2);
    return met;
}

template <int MODE, int T>
__global__ void __launch_bounds__(64)
k_schwarz(int W, int H, int C, int ntx, int nty, int sx, int sy, int iters, float robin, const double *gnorm,
          float frac, double guard, const uint8_t *__restrict__ mask, const float *__restrict__ r,
          const float *__restrict__ e_in, const float *__restrict__ ec, int Wc, int Hc, float *__restrict__ e_out) {
    if (MODE == 0 && guard >= 0.0 && residual_met(gnorm, C, guard)) return;
    schwarz_block<MODE, T>(W, H, ntx, nty, sx, sy, iters, robin, local_stop_sq(gnorm, 2, frac, blockIdx.y), mask,
                           r, e_in, ec, Wc, Hc, e_out, xcd_remap(blockIdx.x, ntx * nty), blockIdx.y);
}

// ------------------------------------------------------------------ reduced FMG (Sec. 3.2)

// Data on the first coarse level: a coarse known pixel takes the mean of its
// known fine children's values (Sec. 3.3).
template <typename TD>
__device__ __forceinline__ void data_restrict_at(int i, int W, int H, int C, const uint8_t *__restrict__ m,
                                                 const TD *__restrict__ d, int Wc, int Hc,
                                                 const uint8_t *__restrict__ mc, float *__restrict__ dc) {
    if (i >= Wc * Hc) return;
    const int X = i % Wc, Y = i / Wc;
    for (int c = 0; c < C; ++c) {
        float acc = 0.f;
        int n = 0;
        if (mc[i])
            for (int j = 0; j < 2; ++j)
                for (int q = 0; q < 2; ++q) {
                    const int x = 2 * X + q, y = 2 * Y + j;
                    if (x < W && y < H && m[y * W + x]) { acc += (float)d[(size_t)c * W * H + y * W + x]; ++n; }
                }
        dc[(size_t)c * Wc * Hc + i] = n ? acc / (float)n : 0.f;
    }
}

template <typename TD>
__global__ void k_data_restrict0(int W, int H, int C, const uint8_t *__restrict__ m, const TD *__restrict__ d,
                                 int Wc, int Hc, const uint8_t *__restrict__ mc, float *__restrict__ dc) {
    data_restrict_at<TD>(blockIdx.x * blockDim.x + threadIdx.x, W, H, C, m, d, Wc, Hc, mc, dc);
}

// FMG prolongation: out = P ec on unknown pixels, the level's data on known ones.
__device__ __forceinline__ void fmg_prolong_at(int i, int W, int H, int C, const uint8_t *__restrict__ m,
                                               const float *__restrict__ data, const float *__restrict__ ec, int Wc,
                                               int Hc, float *__restrict__ out) {
    if (i >= W * H) return;
    const int x = i % W, y = i / W;
    for (int c = 0; c < C; ++c) {
        const size_t j = (size_t)c * W * H + i;
        out[j] = m[i] ? data[j] : prolong_at(ec + (size_t)c * Wc * Hc, Wc, Hc, x, y);
    }
}

__global__ void k_fmg_prolong(int W, int H, int C, const uint8_t *__restrict__ m, const float *__restrict__ data,
                              const float *__restrict__ ec, int Wc, int Hc, float *__restrict__ out) {
    fmg_prolong_at(blockIdx.x * blockDim.x + threadIdx.x, W, H, C, m, data, ec, Wc, Hc, out);
}

// Level-0 FMG prolongation into the FP64 iterate (known pixels keep the data).
__device__ __forceinline__ void fmg_prolong0_at(int i, int W, int H, int C, const uint8_t *__restrict__ m,
                                                const float *__restrict__ ec, int Wc, int Hc, double *__restrict__ u) {
    if (i >= W * H || m[i]) return;
    const int x = i % W, y = i / W;
    for (int c = 0; c < C; ++c) u[(size_t)c * W * H + i] = (double)prolong_at(ec + (size_t)c * Wc * Hc, Wc, Hc, x, y);
}

__global__ void k_fmg_prolong0(int W, int H, int C, const uint8_t *__restrict__ m, const float *__restrict__ ec,
                               int Wc, int Hc, double *__restrict__ u) {
    fmg_prolong0_at(blockIdx.x * blockDim.x + threadIdx.x, W, H, C, m, ec, Wc, Hc, u);
}

// ------------------------------------------------------------------ launchers

static inline dim3 grid1(long n, int bs) { return dim3((unsigned)((n + bs - 1) / bs)); }

void launch_mask_pyramid(const Hierarchy &h, int nlev, unsigned int *counts, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, MAX_LEVELS, counts);
    const long N = (long)h.lev[0].W * h.lev[0].H;
    auto nb = [](long n) { return (int)std::min<long>((n + 255) / 256, 1024); };
    hipLaunchKernelGGL(k_count_known, dim3(nb(N)), dim3(256), 0, s, (int)N, h.lev[0].mask, counts);
    for (int l = 1; l < nlev; ++l) {
        const Level &f = h.lev[l - 1], &c = h.lev[l];
        hipLaunchKernelGGL(k_mask_restrict, dim3(nb((long)c.W * c.H)), dim3(256), 0, s, f.W, f.H, f.mask, c.W, c.H,
                           c.mask, counts + l);
    }
}

template <typename TD>
void launch_init_u(int W, int H, int C, const uint8_t *mask, const TD *data, bool keep_unknown, double *u,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_init_u<TD>, grid1((long)W * H, 256), dim3(256), 0, s, W * H, C, mask, data, keep_unknown, u);
}

dim3 residual_grid(int W, int H) {
    const int cols = (RED_THREADS / 64) * RES_COLS;
    return dim3((W + cols - 1) / cols, (H + RES_BAND - 1) / RES_BAND);
}

template <typename TD>
void launch_residual(int W, int H, int C, const uint8_t *mask, const double *u_in, const float *e, double *u_out,
                     const TD *data, const double *src, float *r, double *partials, double *norms, hipStream_t s) {
    const dim3 g = residual_grid(W, H);
    const int nblk = g.x * g.y;
    // a problem has either data on the mask or a source off it
    if (src) {
        if (C == 3)
            hipLaunchKernelGGL((k_residual<TD, 3, true>), g, dim3(RED_THREADS), 0, s, W, H, mask, u_in, e, u_out,
                               data, src, r, partials, nblk);
        else
            hipLaunchKernelGGL((k_residual<TD, 1, true>), g, dim3(RED_THREADS), 0, s, W, H, mask, u_in, e, u_out,
                               data, src, r, partials, nblk);
    } else {
        if (C == 3)
            hipLaunchKernelGGL((k_residual<TD, 3, false>), g, dim3(RED_THREADS), 0, s, W, H, mask, u_in, e, u_out,
                               data, src, r, partials, nblk);
        else
            hipLaunchKernelGGL((k_residual<TD, 1, false>), g, dim3(RED_THREADS), 0, s, W, H, mask, u_in, e, u_out,
                               data, src, r, partials, nblk);
    }
    hipLaunchKernelGGL(k_reduce_partials, dim3(C), dim3(1024), 0, s, nblk, partials, norms);
}

void launch_update(int W, int H, int C, const uint8_t *mask, const float *e, double *u, hipStream_t s) {
    hipLaunchKernelGGL(k_update, grid1((long)W * H, 256), dim3(256), 0, s, W * H, C, mask, e, u);
}

template <int MODE>
static void launch_schwarz(const Level &L, int C, int iters, float robin, const double *gnorm, float frac,
                           double guard, const float *r, const float *e_in, const float *ec, int Wc, int Hc,
                           float *e_out, hipStream_t s) {
    const dim3 g(L.bx.count * L.by.count, C);
    if (L.tile == 16)
        hipLaunchKernelGGL((k_schwarz<MODE, 16>), g, dim3(64), 0, s, L.W, L.H, C, L.bx.count, L.by.count,
                           L.bx.stride, L.by.stride, iters, robin, gnorm, frac, guard, L.mask, r, e_in, ec, Wc, Hc,
                           e_out);
    else
        hipLaunchKernelGGL((k_schwarz<MODE, 32>), g, dim3(64), 0, s, L.W, L.H, C, L.bx.count, L.by.count,
                           L.bx.stride, L.by.stride, iters, robin, gnorm, frac, guard, L.mask, r, e_in, ec, Wc, Hc,
                           e_out);
}

void launch_smooth_pre(const Level &L, int C, int iters, float robin, const double *gnorm, float frac, float *e_out,
                       hipStream_t s, double guard) {
    if (guard >= 0.0 && !gnorm) guard = -1.0;
    launch_schwarz<0>(L, C, iters, robin, gnorm, frac, guard, L.r, nullptr, nullptr, 1, 1, e_out, s);
}

void launch_smooth_post(const Level &L, const Level &Lc, int C, int iters, float robin, const double *gnorm,
                        float frac, const float *e_in, const float *ec, float *e_out, hipStream_t s) {
    launch_schwarz<1>(L, C, iters, robin, gnorm, frac, -1.0, L.r, e_in, ec, Lc.W, Lc.H, e_out, s);
}

void launch_smooth_fmg(const Level &L, int C, int iters, float robin, const float *e_in, float *e_out,
                       hipStream_t s) {
    // the full problem A u = C d has a zero right-hand side on unknown pixels
    launch_schwarz<2>(L, C, iters, robin, nullptr, 0.f, -1.0, nullptr, e_in, nullptr, 1, 1, e_out, s);
}

void launch_restrict_residual(const Level &L, const Level &Lc, int C, const float *e, hipStream_t s) {
    hipLaunchKernelGGL(k_restrict_residual, grid1((long)Lc.W * Lc.H, 256), dim3(256), 0, s, L.W, L.H, C, L.mask,
                       L.r, e, Lc.W, Lc.H, Lc.mask, Lc.r);
}

template <typename TD>
void launch_data_restrict0(int W, int H, int C, const uint8_t *mask, const TD *data, const Level &Lc, hipStream_t s) {
    hipLaunchKernelGGL(k_data_restrict0<TD>, grid1((long)Lc.W * Lc.H, 256), dim3(256), 0, s, W, H, C, mask, data,
                       Lc.W, Lc.H, Lc.mask, Lc.aux);
}

void launch_data_restrict(const Level &L, const Level &Lc, int C, hipStream_t s) {
    hipLaunchKernelGGL(k_data_restrict0<float>, grid1((long)Lc.W * Lc.H, 256), dim3(256), 0, s, L.W, L.H, C, L.mask,
                       (const float *)L.aux, Lc.W, Lc.H, Lc.mask, Lc.aux);
}

void launch_fmg_prolong(const Level &L, const Level &Lc, int C, const float *ec, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_fmg_prolong, grid1((long)L.W * L.H, 256), dim3(256), 0, s, L.W, L.H, C, L.mask,
                       (const float *)L.aux, ec, Lc.W, Lc.H, out);
}

void launch_fmg_prolong0(int W, int H, int C, const uint8_t *mask, const Level &Lc, const float *ec, double *u,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_fmg_prolong0, grid1((long)W * H, 256), dim3(256), 0, s, W, H, C, mask, ec, Lc.W, Lc.H, u);
}

template void launch_init_u<float>(int, int, int, const uint8_t *, const float *, bool, double *, hipStream_t);
template void launch_init_u<double>(int, int, int, const uint8_t *, const double *, bool, double *, hipStream_t);
template void launch_residual<float>(int, int, int, const uint8_t *, const double *, const float *, double *,
                                     const float *, const double *, float *, double *, double *, hipStream_t);
template void launch_residual<double>(int, int, int, const uint8_t *, const double *, const float *, double *,
                                      const double *, const double *, float *, double *, double *, hipStream_t);
template void launch_data_restrict0<float>(int, int, int, const uint8_t *, const float *, const Level &, hipStream_t);
template void launch_data_restrict0<double>(int, int, int, const uint8_t *, const double *, const Level &, hipStream_t);

// ------------------------------------------------------------------ plain CG (comparator)
//
// Unpreconditioned conjugate gradients in FP64 on the unknown pixels (the
// reduced system L_UU u_U = b_U - L_UK f_K, symmetric positive definite when
// the mask is non-empty), the classical solver of Sec. 2.1 that the paper's
// GPU baseline for tonal optimisation nests inside CGNR (Sec. 6.1). Vectors
// are C x H x W with zeros on known pixels; each channel has its own step
// sizes. Every kernel runs CG_BLOCKS workgroups in a grid-stride loop, so its
// per-workgroup partial sums have a fixed order, and one workgroup per channel
// reduces them in a fixed order: results do not depend on scheduling.
// scal[c * 8 + k]: k = 0 r.r, 1 b.b, 2 alpha, 3 beta, 4 p.q.
constexpr int CG_THREADS = 256;

template <int C>
__device__ __forceinline__ void cg_block_partials(double (&a)[C], double (&b)[C], double *__restrict__ part) {
    __shared__ double s[CG_THREADS / 64][2 * C];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const double x = wave_sum_d(a[c]), y = wave_sum_d(b[c]);
        if (lane == 0) { s[wid][2 * c] = x; s[wid][2 * c + 1] = y; }
    }
    __syncthreads();
    if (threadIdx.x < C) {
        const int c = threadIdx.x;
        double x = 0.0, y = 0.0;
        for (int w = 0; w < CG_THREADS / 64; ++w) { x += s[w][2 * c]; y += s[w][2 * c + 1]; }
        part[((size_t)c * CG_BLOCKS + blockIdx.x) * 2 + 0] = x;
        part[((size_t)c * CG_BLOCKS + blockIdx.x) * 2 + 1] = y;
    }
}

// r = b - A u for every pixel (0 on known pixels in the stored r, whose row is
// the identity with u = data there), partial sums of the true residual's r.r
// and of b.b with b = data on known pixels and src (or 0) elsewhere.
template <typename TD, int C>
__global__ void __launch_bounds__(CG_THREADS)
k_cg_start(int W, int H, const uint8_t *__restrict__ mask, const double *__restrict__ u,
           const TD *__restrict__ data, const double *__restrict__ src, double *__restrict__ r,
           double *__restrict__ part) {
    const int N = W * H;
    double rr[C], bb[C];
#pragma unroll
    for (int c = 0; c < C; ++c) rr[c] = bb[c] = 0.0;
    for (int i = blockIdx.x * CG_THREADS + threadIdx.x; i < N; i += CG_BLOCKS * CG_THREADS) {
        const int x = i % W, y = i / W;
        const bool known = mask[i] != 0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const double *uc = u + (size_t)c * N;
            double b, res;
            if (known) {
                b = data ? (double)data[(size_t)c * N + i] : 0.0;
                res = b - uc[i];
            } else {
                b = src ? src[(size_t)c * N + i] : 0.0;
                double au = deg_of(x, y, W, H) * uc[i];
                if (x > 0) au -= uc[i - 1];
                if (x < W - 1) au -= uc[i + 1];
                if (y > 0) au -= uc[i - W];
                if (y < H - 1) au -= uc[i + W];
                res = b - au;
            }
            r[(size_t)c * N + i] = known ? 0.0 : res;
            rr[c] += res * res;
            bb[c] += b * b;
        }
    }
    cg_block_partials<C>(rr, bb, part);
}

// p_new = r + beta p_old (beta = 0: p_new = r, p_old unread), and the partial
// sums of p_new.(A p_new) over unknown pixels (p_new is 0 on known pixels).
// A p_new is not stored: the update recomputes it from p_new, which costs a
// stencil but saves writing and reading one vector per step.
template <int C>
__global__ void __launch_bounds__(CG_THREADS)
k_cg_direction(int W, int H, const uint8_t *__restrict__ mask, const double *__restrict__ r,
               const double *__restrict__ p_old, double *__restrict__ p_new, const double *__restrict__ scal,
               double *__restrict__ part) {
    const int N = W * H;
    double pq[C], zero[C];
#pragma unroll
    for (int c = 0; c < C; ++c) pq[c] = zero[c] = 0.0;
    for (int i = blockIdx.x * CG_THREADS + threadIdx.x; i < N; i += CG_BLOCKS * CG_THREADS) {
        const int x = i % W, y = i / W;
        const bool known = mask[i] != 0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const double beta = scal[c * 8 + 3];
            const double *rc = r + (size_t)c * N, *pc = p_old + (size_t)c * N;
            auto pn = [&](int j) { return beta != 0.0 ? rc[j] + beta * pc[j] : rc[j]; };
            const double p0 = pn(i);
            double qv = 0.0;
            if (!known) {
                qv = deg_of(x, y, W, H) * p0;
                if (x > 0) qv -= pn(i - 1);
                if (x < W - 1) qv -= pn(i + 1);
                if (y > 0) qv -= pn(i - W);
                if (y < H - 1) qv -= pn(i + W);
            }
            p_new[(size_t)c * N + i] = p0;
            pq[c] += p0 * qv;
        }
    }
    cg_block_partials<C>(pq, zero, part);
}

// q = A p, u += alpha p, r -= alpha q on unknown pixels, partial sums of the
// new r.r.
template <int C>
__global__ void __launch_bounds__(CG_THREADS)
k_cg_update(int W, int H, const uint8_t *__restrict__ mask, double *__restrict__ u, double *__restrict__ r,
            const double *__restrict__ p, const double *__restrict__ scal, double *__restrict__ part) {
    const int N = W * H;
    double rr[C], zero[C];
#pragma unroll
    for (int c = 0; c < C; ++c) rr[c] = zero[c] = 0.0;
    for (int i = blockIdx.x * CG_THREADS + threadIdx.x; i < N; i += CG_BLOCKS * CG_THREADS) {
        if (mask[i]) continue;
        const int x = i % W, y = i / W;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const size_t j = (size_t)c * N + i;
            const double *pc = p + (size_t)c * N;
            double q = deg_of(x, y, W, H) * pc[i];
            if (x > 0) q -= pc[i - 1];
            if (x < W - 1) q -= pc[i + 1];
            if (y > 0) q -= pc[i - W];
            if (y < H - 1) q -= pc[i + W];
            const double alpha = scal[c * 8 + 2];
            u[j] += alpha * pc[i];
            const double rn = r[j] - alpha * q;
            r[j] = rn;
            rr[c] += rn * rn;
        }
    }
    cg_block_partials<C>(rr, zero, part);
}

// One workgroup of 1024 threads per channel: fixed-order sum of the CG_BLOCKS
// partial pairs (thread t takes t, t + 1024, ...), then the scalar step. step 0: r.r and b.b of the start
// (beta = 0); 1: alpha = r.r / p.q; 2: beta = r.r_new / r.r, r.r = r.r_new.
// A zero denominator (exact convergence) gives a zero step.
__global__ void __launch_bounds__(1024) k_cg_scalars(int step, const double *__restrict__ part, double *__restrict__ scal) {
    const int c = blockIdx.x;
    double pa = 0.0, pb = 0.0;
#pragma unroll
    for (int k = 0; k < CG_BLOCKS / 1024; ++k) {
        const double2 v = reinterpret_cast<const double2 *>(part)[(size_t)c * CG_BLOCKS + k * 1024 + threadIdx.x];
        pa += v.x;
        pb += v.y;
    }
    const double a = wave_sum_d(pa), b = wave_sum_d(pb);
    __shared__ double s[16][2];
    if ((threadIdx.x & 63) == 0) { s[threadIdx.x >> 6][0] = a; s[threadIdx.x >> 6][1] = b; }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double x = 0.0, y = 0.0;
    for (int w = 0; w < 16; ++w) { x += s[w][0]; y += s[w][1]; }
    double *sc = scal + c * 8;
    if (step == 0) {
        sc[0] = x;
        sc[1] = y;
        sc[3] = 0.0;
    } else if (step == 1) {
        sc[4] = x;
        sc[2] = x > 0.0 ? sc[0] / x : 0.0;
    } else {
        sc[3] = sc[0] > 0.0 ? x / sc[0] : 0.0;
        sc[0] = x;
    }
}

static_assert(CG_BLOCKS % 1024 == 0, "k_cg_scalars takes CG_BLOCKS / 1024 partials per thread");

template <typename TD>
void launch_cg_start(int W, int H, int C, const uint8_t *mask, const double *u, const TD *data, const double *src,
                     double *r, double *part, double *scal, hipStream_t s) {
    if (C == 3)
        k_cg_start<TD, 3><<<CG_BLOCKS, CG_THREADS, 0, s>>>(W, H, mask, u, data, src, r, part);
    else
        k_cg_start<TD, 1><<<CG_BLOCKS, CG_THREADS, 0, s>>>(W, H, mask, u, data, src, r, part);
    k_cg_scalars<<<C, 1024, 0, s>>>(0, part, scal);
}
template void launch_cg_start<float>(int, int, int, const uint8_t *, const double *, const float *, const double *,
                                     double *, double *, double *, hipStream_t);
template void launch_cg_start<double>(int, int, int, const uint8_t *, const double *, const double *,
                                      const double *, double *, double *, double *, hipStream_t);

void launch_cg_iteration(int W, int H, int C, const uint8_t *mask, double *u, double *r, const double *p_old,
                         double *p_new, double *part, double *scal, hipStream_t s) {
    if (C == 3) {
        k_cg_direction<3><<<CG_BLOCKS, CG_THREADS, 0, s>>>(W, H, mask, r, p_old, p_new, scal, part);
        k_cg_scalars<<<C, 1024, 0, s>>>(1, part, scal);
        k_cg_update<3><<<CG_BLOCKS, CG_THREADS, 0, s>>>(W, H, mask, u, r, p_new, scal, part);
    } else {
        k_cg_direction<1><<<CG_BLOCKS, CG_THREADS, 0, s>>>(W, H, mask, r, p_old, p_new, scal, part);
        k_cg_scalars<<<C, 1024, 0, s>>>(1, part, scal);
        k_cg_update<1><<<CG_BLOCKS, CG_THREADS, 0, s>>>(W, H, mask, u, r, p_new, scal, part);
    }
    k_cg_scalars<<<C, 1024, 0, s>>>(2, part, scal);
}

// ------------------------------------------------------------------ batched kernels
// One launch serves several images: each workgroup finds its segment in the
// launch's segment table (one entry per image and level taking part), looks up
// the image and level descriptors and runs the same block function as the
// single-image kernel, so an image's result does not depend on the batch.

struct SegItem { int img, lev, a, b; };

// Segment k covers workgroups [start_k, start_{k+1}); starts ascend from 0. One
// lane per segment compares its start with the workgroup index and the ballot
// count is the segment's position, so a table of up to 64 segments costs one
// vector load. The local index splits into (local % unit, local / unit).
__device__ __forceinline__ SegItem seg_item(const int4 *__restrict__ seg, int nseg, int b) {
    const int lane = threadIdx.x & 63;
    int4 cur = make_int4(0, 0, 0, 1), prev = cur;
    int cnt = 0;
    for (int base = 0; base < nseg; base += 64) {
        prev = cur;
        const int k = base + lane;
        cur = k < nseg ? seg[k] : make_int4(0, 0, 0x7fffffff, 1);
        cnt = (int)__popcll(__ballot(cur.z <= b));
        if (cnt < 64) break;
    }
    const int4 src = cnt == 0 ? prev : cur;
    const int at = cnt == 0 ? 63 : cnt - 1;
    const int img = __builtin_amdgcn_readlane(src.x, at);
    const int lev = __builtin_amdgcn_readlane(src.y, at);
    const int start = __builtin_amdgcn_readlane(src.z, at);
    const int unit = __builtin_amdgcn_readlane(src.w, at);
    const int local = b - start;
    return SegItem{img, lev, local % unit, local / unit};
}

__global__ void __launch_bounds__(256)
kb_count(const int4 *__restrict__ seg, int nseg, const BLev *__restrict__ L, const BImg *__restrict__ I) {
    const SegItem it = seg_item(seg, nseg, blockIdx.x);
    const BImg &im = I[it.img];
    if (it.lev == 0) {
        const int N = im.W * im.H;
        count_known_block(N, im.mask, im.counts, it.a, min((N + 255) / 256, 1024));
    } else {
        const BLev &f = L[it.img * MAX_LEVELS + it.lev - 1];
        const int Nc = f.Wc * f.Hc;
        mask_restrict_block(f.W, f.H, f.mask, f.Wc, f.Hc, f.mask_c, im.counts + it.lev, it.a,
                            min((Nc + 255) / 256, 1024));
    }
}

// Starting iterate: the data (or 0 for a source problem) on known pixels;
// unknown pixels 0, or kept for a warm start.
__global__ void kb_init_u(const int4 *__restrict__ seg, int nseg, const BImg *__restrict__ I) {
    const SegItem it = seg_item(seg, nseg, blockIdx.x);
    const BImg &im = I[it.img];
    const int i = it.a * 256 + threadIdx.x, N = im.W * im.H;
    if (i >= N || (im.warm && !im.mask[i])) return;
    if (im.kind == EK_DATA_F32)
        init_u_at<float>(i, N, im.C, im.mask, im.f, nullptr, im.u);
    else
        init_u_at<double>(i, N, im.C, im.mask, im.kind == EK_DATA_F64 ? im.data_d : nullptr, nullptr, im.u);
}

// flags[img]: bit 1 = apply the last V-cycle's correction, bit 2 = the current
// iterate is in u_alt (the refinement ping-pongs between u and u_alt)
template <int C>
__global__ void __launch_bounds__(RED_THREADS)
kb_residual(const int4 *__restrict__ seg, int nseg, const BImg *__restrict__ I, const uint8_t *__restrict__ flags,
            const BLev *__restrict__ L) {
    const SegItem it = seg_item(seg, nseg, blockIdx.x);
    const BImg &im = I[it.img];
    const int fl = flags[it.img];
    const bool use_e = fl & 2, parity = fl & 4;
    const double *u_in = parity ? im.u_alt : im.u;
    double *u_out = parity ? im.u : im.u_alt;
    const BLev &l0 = L[it.img * MAX_LEVELS];
    // the last V-cycle's correction is the finest level's post-smoothing
    // output (or the single level's smoothing output)
    const float *e = use_e ? (im.nlev > 1 ? l0.eb : l0.ea) : nullptr;
    double *uo = use_e ? u_out : nullptr;
    if (im.kind == EK_DATA_F32)
        residual_block<float, C, false>(im.W, im.H, im.mask, u_in, e, uo, im.f, nullptr, l0.r, im.partials, im.nblk,
                                        it.a, it.b, im.gx);
    else if (im.kind == EK_DATA_F64)
        residual_block<double, C, false>(im.W, im.H, im.mask, u_in, e, uo, im.data_d, nullptr, l0.r, im.partials,
                                         im.nblk, it.a, it.b, im.gx);
    else
        residual_block<double, C, true>(im.W, im.H, im.mask, u_in, e, uo, (const double *)nullptr, im.src, l0.r,
                                        im.partials, im.nblk, it.a, it.b, im.gx);
}

__global__ void __launch_bounds__(1024)
kb_reduce(const int4 *__restrict__ seg, int nseg, const BImg *__restrict__ I) {
    const SegItem it = seg_item(seg, nseg, blockIdx.x);
    const BImg &im = I[it.img];
    reduce_partials_block(im.nblk, im.partials, im.norms, it.a);
}

template <int MODE, bool COARSEST, int T>
__global__ void __launch_bounds__(64)
kb_schwarz(const int4 *__restrict__ seg, int nseg, int n, const BLev *__restrict__ L, const BImg *__restrict__ I) {
    const SegItem it = seg_item(seg, nseg, xcd_remap(blockIdx.x, n));
    const BImg &im = I[it.img];
    const BLev &l = L[it.img * MAX_LEVELS + it.lev];
    const int iters = COARSEST ? im.coarse_iters : it.lev == 0 ? im.local_iters : im.mid_iters;
    // the global-relative local stop on the finest level of a V-cycle (the
    // residual sweep before it left the global norms in im.norms)
    const float stop_sq = MODE != 2 && !COARSEST && it.lev == 0 ? local_stop_sq(im.norms, 2, im.local_stop, it.b) : 0.f;
    if (MODE == 0)
        schwarz_block<0, T>(l.W, l.H, l.ntx, l.nty, l.sx, l.sy, iters, im.robin, stop_sq, l.mask, l.r, nullptr,
                            nullptr, 1, 1, l.ea, it.a, it.b);
    else if (MODE == 1)
        schwarz_block<1, T>(l.W, l.H, l.ntx, l.nty, l.sx, l.sy, iters, im.robin, stop_sq, l.mask, l.r, l.ea, l.ec,
                            l.Wc, l.Hc, l.eb, it.a, it.b);
    else
        schwarz_block<2, T>(l.W, l.H, l.ntx, l.nty, l.sx, l.sy, iters, im.robin, 0.f, l.mask, nullptr,
                            COARSEST ? l.aux : l.eb, nullptr, 1, 1, l.ea, it.a, it.b);
}

__global__ void kb_restrict(const int4 *__restrict__ seg, int nseg, const BLev *__restrict__ L,
                            const BImg *__restrict__ I) {
    const SegItem it = seg_item(seg, nseg, blockIdx.x);
    const BImg &im = I[it.img];
    const BLev &l = L[it.img * MAX_LEVELS + it.lev];
    restrict_residual_at(it.a * 256 + threadIdx.x, l.W, l.H, im.C, l.mask, l.r, l.ea, l.Wc, l.Hc, l.mask_c, l.r_c);
}

template <bool FROM_F>
__global__ void kb_data_restrict(const int4 *__restrict__ seg, int nseg, const BLev *__restrict__ L,
                                 const BImg *__restrict__ I) {
    const SegItem it = seg_item(seg, nseg, blockIdx.x);
    const BImg &im = I[it.img];
    const BLev &l = L[it.img * MAX_LEVELS + it.lev];
    if (FROM_F && im.kind == EK_DATA_F64)
        data_restrict_at<double>(it.a * 256 + threadIdx.x, l.W, l.H, im.C, l.mask, im.data_d, l.Wc, l.Hc, l.mask_c,
                                 l.aux_c);
    else
        data_restrict_at<float>(it.a * 256 + threadIdx.x, l.W, l.H, im.C, l.mask, FROM_F ? im.f : l.aux, l.Wc, l.Hc,
                                l.mask_c, l.aux_c);
}

__global__ void kb_fmg_prolong(const int4 *__restrict__ seg, int nseg, const BLev *__restrict__ L,
                               const BImg *__restrict__ I) {
    const SegItem it = seg_item(seg, nseg, blockIdx.x);
    const BImg &im = I[it.img];
    const BLev &l = L[it.img * MAX_LEVELS + it.lev];
    // the coarser level's FMG result is in its ea
    const BLev &c = L[it.img * MAX_LEVELS + it.lev + 1];
    fmg_prolong_at(it.a * 256 + threadIdx.x, l.W, l.H, im.C, l.mask, l.aux, c.ea, l.Wc, l.Hc, l.eb);
}

__global__ void kb_fmg_prolong0(const int4 *__restrict__ seg, int nseg, const BLev *__restrict__ L,
                                const BImg *__restrict__ I) {
    const SegItem it = seg_item(seg, nseg, blockIdx.x);
    const BImg &im = I[it.img];
    const BLev &l = L[it.img * MAX_LEVELS];
    const BLev &c = L[it.img * MAX_LEVELS + 1];
    fmg_prolong0_at(it.a * 256 + threadIdx.x, im.W, im.H, im.C, im.mask, c.ea, l.Wc, l.Hc, im.u);
}

#define SEG_ARGS(ph) (ph).seg, (ph).nseg
void launch_b_count(const BPhase &ph, const BLev *L, const BImg *I, hipStream_t s) {
    if (ph.n) hipLaunchKernelGGL(kb_count, dim3(ph.n), dim3(256), 0, s, SEG_ARGS(ph), L, I);
}
void launch_b_init_u(const BPhase &ph, const BImg *I, hipStream_t s) {
    if (ph.n) hipLaunchKernelGGL(kb_init_u, dim3(ph.n), dim3(256), 0, s, SEG_ARGS(ph), I);
}
void launch_b_residual(const BPhase &ph, int C, const BImg *I, const uint8_t *flags, const BLev *L, hipStream_t s) {
    if (!ph.n) return;
    if (C == 3)
        hipLaunchKernelGGL(kb_residual<3>, dim3(ph.n), dim3(RED_THREADS), 0, s, SEG_ARGS(ph), I, flags, L);
    else
        hipLaunchKernelGGL(kb_residual<1>, dim3(ph.n), dim3(RED_THREADS), 0, s, SEG_ARGS(ph), I, flags, L);
}
void launch_b_reduce(const BPhase &ph, const BImg *I, hipStream_t s) {
    if (ph.n) hipLaunchKernelGGL(kb_reduce, dim3(ph.n), dim3(1024), 0, s, SEG_ARGS(ph), I);
}
template <int T>
static void launch_b_schwarz_t(int mode, bool coarsest, const BPhase &ph, const BLev *L, const BImg *I,
                               hipStream_t s) {
    const dim3 g(ph.n), b(64);
    if (mode == 0 && !coarsest) hipLaunchKernelGGL((kb_schwarz<0, false, T>), g, b, 0, s, SEG_ARGS(ph), ph.n, L, I);
    if (mode == 0 && coarsest) hipLaunchKernelGGL((kb_schwarz<0, true, T>), g, b, 0, s, SEG_ARGS(ph), ph.n, L, I);
    if (mode == 1) hipLaunchKernelGGL((kb_schwarz<1, false, T>), g, b, 0, s, SEG_ARGS(ph), ph.n, L, I);
    if (mode == 2 && !coarsest) hipLaunchKernelGGL((kb_schwarz<2, false, T>), g, b, 0, s, SEG_ARGS(ph), ph.n, L, I);
    if (mode == 2 && coarsest) hipLaunchKernelGGL((kb_schwarz<2, true, T>), g, b, 0, s, SEG_ARGS(ph), ph.n, L, I);
}
void launch_b_schwarz(int mode, bool coarsest, int tile, const BPhase &ph, const BLev *L, const BImg *I,
                      hipStream_t s) {
    if (!ph.n) return;
    if (tile == 16)
        launch_b_schwarz_t<16>(mode, coarsest, ph, L, I, s);
    else
        launch_b_schwarz_t<32>(mode, coarsest, ph, L, I, s);
}
void launch_b_restrict(const BPhase &ph, const BLev *L, const BImg *I, hipStream_t s) {
    if (ph.n) hipLaunchKernelGGL(kb_restrict, dim3(ph.n), dim3(256), 0, s, SEG_ARGS(ph), L, I);
}
void launch_b_data_restrict(bool from_f, const BPhase &ph, const BLev *L, const BImg *I, hipStream_t s) {
    if (!ph.n) return;
    if (from_f) hipLaunchKernelGGL(kb_data_restrict<true>, dim3(ph.n), dim3(256), 0, s, SEG_ARGS(ph), L, I);
    else hipLaunchKernelGGL(kb_data_restrict<false>, dim3(ph.n), dim3(256), 0, s, SEG_ARGS(ph), L, I);
}
void launch_b_fmg_prolong(const BPhase &ph, const BLev *L, const BImg *I, hipStream_t s) {
    if (ph.n) hipLaunchKernelGGL(kb_fmg_prolong, dim3(ph.n), dim3(256), 0, s, SEG_ARGS(ph), L, I);
}
void launch_b_fmg_prolong0(const BPhase &ph, const BLev *L, const BImg *I, hipStream_t s) {
    if (ph.n) hipLaunchKernelGGL(kb_fmg_prolong0, dim3(ph.n), dim3(256), 0, s, SEG_ARGS(ph), L, I);
}
#undef SEG_ARGS

}  // namespace hdi
