// Kernels of tonal optimisation (paper Sec. 5) for gfx950.
//
// The unknowns are the values on the mask K (eq. tonal-opt-minimisation; off
// the mask g = 0), stored as compact FP64 vectors [C][m] in ascending pixel
// order. B g = A^{-1} C g is an inpainting solve; B^T y, by the symmetrised
// form of Sec. 5.1, is y_k + sum_{j in N4(k), j unknown} w_j with
// L_UU w_U = y_U (an inpainting solve with a source term and zero data).
#include <algorithm>
#include <cfloat>

#include "hdi_internal.h"
#include "wave.h"

namespace hdi {

// ------------------------------------------------------------------ mask compaction

constexpr int CMP_THREADS = 1024;

// Known pixels per workgroup chunk of CMP_THREADS pixels.
__global__ void __launch_bounds__(CMP_THREADS)
k_compact_count(int N, const uint8_t *__restrict__ m, int *__restrict__ chunk_cnt) {
    const int i = blockIdx.x * CMP_THREADS + threadIdx.x;
    const int k = (i < N && m[i]) ? 1 : 0;
    __shared__ int s[CMP_THREADS / 64];
    const unsigned long long b = __ballot(k);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = __popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < CMP_THREADS / 64; ++w) t += s[w];
        chunk_cnt[blockIdx.x] = t;
    }
}

// Exclusive scan of the chunk counts (one workgroup; sequential over blocks of
// 1024 with a workgroup scan inside), plus the total.
__global__ void __launch_bounds__(CMP_THREADS)
k_compact_scan(int nchunks, const int *__restrict__ cnt, int *__restrict__ off, int *__restrict__ total) {
    __shared__ int s[CMP_THREADS];
    int carry = 0;
    for (int base = 0; base < nchunks; base += CMP_THREADS) {
        const int i = base + threadIdx.x;
        const int v = i < nchunks ? cnt[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int d = 1; d < CMP_THREADS; d <<= 1) {
            const int t = threadIdx.x >= d ? s[threadIdx.x - d] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nchunks) off[i] = carry + s[threadIdx.x] - v;
        const int last = s[CMP_THREADS - 1];
        __syncthreads();
        carry += last;
    }
    if (threadIdx.x == 0) *total = carry;
}

// idx[j] = pixel of the j-th known pixel (ascending), pos[i] = j or -1.
__global__ void __launch_bounds__(CMP_THREADS)
k_compact_scatter(int N, const uint8_t *__restrict__ m, const int *__restrict__ off, int *__restrict__ idx,
                  int *__restrict__ pos) {
    const int i = blockIdx.x * CMP_THREADS + threadIdx.x;
    const int k = (i < N && m[i]) ? 1 : 0;
    const unsigned long long b = __ballot(k);
    const int lane = threadIdx.x & 63;
    const int before = __popcll(b & ((1ull << lane) - 1ull));
    __shared__ int s[CMP_THREADS / 64];
    if (lane == 0) s[threadIdx.x >> 6] = __popcll(b);
    __syncthreads();
    int wbase = 0;
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) wbase += s[w];
    if (i < N) {
        const int j = off[blockIdx.x] + wbase + before;
        pos[i] = k ? j : -1;
        if (k) idx[j] = i;
    }
}

// ------------------------------------------------------------------ compact <-> image

// img[c][idx[j]] = v[c][j] (only mask pixels are written).
__global__ void k_scatter_K(int m, int C, int N, const int *__restrict__ idx, const double *__restrict__ v,
                            double *__restrict__ img) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const int i = idx[j];
    for (int c = 0; c < C; ++c) img[(size_t)c * N + i] = v[(size_t)c * m + j];
}

// v[c][j] = (double) f[c][idx[j]]
__global__ void k_gather_f(int m, int C, int N, const int *__restrict__ idx, const float *__restrict__ f,
                           double *__restrict__ v) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const int i = idx[j];
    for (int c = 0; c < C; ++c) v[(size_t)c * m + j] = (double)f[(size_t)c * N + i];
}

// B^T gather (Sec. 5.1, symmetrised system): out[c][j] = y[c][k] + sum of w over
// the unknown 4-neighbours of k = idx[j]. y may be null (then y_k = yK[c][j]).
__global__ void k_gather_Bt(int W, int H, int m, int C, const int *__restrict__ idx, const uint8_t *__restrict__ mask,
                            const double *__restrict__ y, const double *__restrict__ yK, const double *__restrict__ w,
                            double *__restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const int N = W * H;
    const int k = idx[j];
    const int x = k % W, yy = k / W;
    const bool hl = x > 0 && !mask[k - 1], hr = x < W - 1 && !mask[k + 1];
    const bool hu = yy > 0 && !mask[k - W], hd = yy < H - 1 && !mask[k + W];
    for (int c = 0; c < C; ++c) {
        const double *wc = w + (size_t)c * N;
        double s = y ? y[(size_t)c * N + k] : yK[(size_t)c * m + j];
        if (hl) s += wc[k - 1];
        if (hr) s += wc[k + 1];
        if (hu) s += wc[k - W];
        if (hd) s += wc[k + W];
        out[(size_t)c * m + j] = s;
    }
}

// rho = f - u over the whole image (FP64), plus partial sums of rho^2 per channel.
__global__ void __launch_bounds__(256)
k_image_residual(int N, int C, const float *__restrict__ f, const double *__restrict__ u, double *__restrict__ rho,
                 double *__restrict__ partials, int nblk) {
    double acc[3] = {0.0, 0.0, 0.0};
    for (int i = blockIdx.x * 256 + threadIdx.x; i < N; i += nblk * 256)
        for (int c = 0; c < C; ++c) {
            const size_t o = (size_t)c * N + i;
            const double d = (double)f[o] - (u ? u[o] : 0.0);
            rho[o] = d;
            acc[c] += d * d;
        }
    __shared__ double s[4][3];
    for (int c = 0; c < C; ++c) {
        const double a = wave_sum_d(acc[c]);
        if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6][c] = a;
    }
    __syncthreads();
    if (threadIdx.x < C) {
        double a = 0.0;
        for (int w = 0; w < 4; ++w) a += s[w][threadIdx.x];
        partials[(size_t)threadIdx.x * nblk + blockIdx.x] = a;
    }
}

// ------------------------------------------------------------------ compact vector algebra (FP64)

// Partial sums of sum_j a[c][j] * b[c][j] for NP pairs at once: pairs (a_q, b_q),
// q < np; partials[q][c][blk]. Fixed grid => fixed summation order.
struct DotArgs { const double *a[4]; const double *b[4]; };

template <int NP, int C>
__global__ void __launch_bounds__(256)
k_dots(int m, DotArgs args, double *__restrict__ partials, int nblk) {
    double acc[NP][C];
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
        for (int c = 0; c < C; ++c) acc[q][c] = 0.0;
    for (int j = blockIdx.x * 256 + threadIdx.x; j < m; j += nblk * 256)
#pragma unroll
        for (int q = 0; q < NP; ++q)
#pragma unroll
            for (int c = 0; c < C; ++c) acc[q][c] += args.a[q][(size_t)c * m + j] * args.b[q][(size_t)c * m + j];
    __shared__ double s[4][12];
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const double v = wave_sum_d(acc[q][c]);
            if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6][q * 3 + c] = v;
        }
    __syncthreads();
    if (threadIdx.x < NP * 3) {
        const int q = threadIdx.x / 3, c = threadIdx.x % 3;
        if (c < C) {
            double v = 0.0;
            for (int w = 0; w < 4; ++w) v += s[w][threadIdx.x];
            partials[((size_t)q * 3 + c) * nblk + blockIdx.x] = v;
        }
    }
}

// out[k] = sum_b partials[k][b] for k < nk (one wave per value, fixed order).
__global__ void k_sum_rows(int nk, int nblk, const double *__restrict__ partials, double *__restrict__ out) {
    const int k = blockIdx.x;
    if (k >= nk) return;
    double a = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 64) a += partials[(size_t)k * nblk + b];
    a = wave_sum_d(a);
    if (threadIdx.x == 0) out[k] = a;
}

// y[c] = a[c] * x[c] + b[c] * y[c] (per-channel scalars on the device-visible arg).
struct Coef3 { double a[3], b[3]; };
__global__ void k_axpby(int m, int C, Coef3 k, const double *__restrict__ x, double *__restrict__ y) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    for (int c = 0; c < C; ++c) {
        const size_t o = (size_t)c * m + j;
        // with b = 0, y is output only: it may hold anything (a fresh direction)
        y[o] = k.b[c] != 0.0 ? k.a[c] * x[o] + k.b[c] * y[o] : k.a[c] * x[o];
    }
}

// ------------------------------------------------------------------ RAS local normal equations

// One RAS sweep of Alg. 2 step 2 on TB x TB blocks: each block solves its
// local normal equations B_i^T B_i v_i = R_i r by `nc` steps of CG on the
// normal equations (CGNR), where B_i = A_i^{-1} C_i is inpainting on the
// block's own grid graph (homogeneous Neumann at the block boundary, Sec. 5.2)
// and each local inpainting is `ni` steps of CG on L_UU of the block. The
// result is written on the mask pixels the block owns (0/1 partition of unity,
// the middle of each overlap splitting ownership). FP32 throughout (a
// preconditioner). Each lane holds 4x4 pixels: TB = 32 is one wavefront per
// block; TB = 64 (the paper's block size) is four wavefronts, one per 32x32
// quadrant, which exchange their edges through the LDS tile and combine their
// dot products through LDS, with workgroup barriers. Every loop bound and
// branch below depends only on values that all threads of the block share,
// so every thread reaches every barrier.
constexpr int TCOL0 = 4;

template <int TB>
struct LocalTile {
    static constexpr int LW = TB + 8;   // LDS row: TCOL0 zero columns, TB pixels, zero columns
    float (*s_x)[LW];
    int ox, oy;                         // the lane's 4x4 pixels start at (ox, oy) in the block
    float *s_red;                       // [2][4] partial sums of the four wavefronts (TB = 64)
    int parity = 0;
    __device__ void publish(const float *v) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            *reinterpret_cast<float4 *>(&s_x[oy + j + 1][TCOL0 + ox]) =
                make_float4(v[j * 4 + 0], v[j * 4 + 1], v[j * 4 + 2], v[j * 4 + 3]);
        __syncthreads();
    }
    // n[k] = sum of the 4 neighbours of pixel k of v (zero outside the block)
    __device__ void nbsum(const float *v, float *n) {
        publish(v);
        const float4 up = *reinterpret_cast<const float4 *>(&s_x[oy][TCOL0 + ox]);
        const float4 dn = *reinterpret_cast<const float4 *>(&s_x[oy + 5][TCOL0 + ox]);
        const float upv[4] = {up.x, up.y, up.z, up.w};
        const float dnv[4] = {dn.x, dn.y, dn.z, dn.w};
        float lf[4], rt[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            lf[j] = s_x[oy + j + 1][TCOL0 + ox - 1];
            rt[j] = s_x[oy + j + 1][TCOL0 + ox + 4];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = j * 4 + i;
                n[k] = (j > 0 ? v[k - 4] : upv[i]) + (j < 3 ? v[k + 4] : dnv[i]) + (i > 0 ? v[k - 1] : lf[j]) +
                       (i < 3 ? v[k + 1] : rt[j]);
            }
        __syncthreads();
    }
    // sum over the block: the wavefront's DPP sum, then (TB = 64) the four
    // wavefront sums in a fixed order from double-buffered LDS slots (a slot is
    // rewritten only after the next sum's barrier, when every wave has read it)
    __device__ float sum(float v) {
        v = wave_sum(v);
        if constexpr (TB == 64) {
            float *slot = s_red + 4 * parity;
            if ((threadIdx.x & 63) == 0) slot[threadIdx.x >> 6] = v;
            __syncthreads();
            v = (slot[0] + slot[1]) + (slot[2] + slot[3]);
            parity ^= 1;
        }
        return v;
    }
};

// x = (L_UU of the block)^{-1} b by `iters` CG steps from 0 (fewer once the
// residual reaches the FP32 floor); b and x are zero off U. dg[k] = block-graph
// degree on U pixels, 0 elsewhere. Returns the steps taken.
template <int TB>
__device__ __forceinline__ int local_cg(LocalTile<TB> &T, const float *dg, const float *b, float *x, int iters) {
    float r[16], p[16], q[16];
    float rr = 0.f;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        x[k] = 0.f;
        r[k] = b[k];
        p[k] = b[k];
        rr += b[k] * b[k];
    }
    rr = T.sum(rr);
    const float floor_rr = rr * 1e-14f;
    int it = 0;
    for (; it < iters && rr > floor_rr && rr >= FLT_MIN; ++it) {
        T.nbsum(p, q);
        float pq = 0.f;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            q[k] = dg[k] > 0.f ? dg[k] * p[k] - q[k] : 0.f;
            pq += p[k] * q[k];
        }
        pq = T.sum(pq);
        if (!(pq >= FLT_MIN)) break;
        const float alpha = rr * __builtin_amdgcn_rcpf(pq);
        float rr2 = 0.f;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            x[k] += alpha * p[k];
            r[k] -= alpha * q[k];
            rr2 += r[k] * r[k];
        }
        rr2 = T.sum(rr2);
        const float beta = rr2 * __builtin_amdgcn_rcpf(rr);
        rr = rr2;
#pragma unroll
        for (int k = 0; k < 16; ++k) p[k] = r[k] + beta * p[k];
    }
    return it;
}

template <int TB>
__global__ void __launch_bounds__(TB == 64 ? 256 : 64)
k_ras_local(int W, int H, int C, int m, int ntx, int nty, int sx, int sy, int nc, int ni,
            const uint8_t *__restrict__ mask, const int *__restrict__ pos, const double *__restrict__ r,
            double *__restrict__ z, unsigned int *__restrict__ steps) {
    constexpr int NT = TB == 64 ? 256 : 64;
    __shared__ __attribute__((aligned(16))) float s_x[TB + 2][LocalTile<TB>::LW];
    __shared__ __attribute__((aligned(16))) float s_t[TB][TB];   // t = B_i p between the two local solves
    __shared__ float s_red[8];
    // the C channel blocks of a tile are neighbours in the launch order and go
    // to the same XCD, so the tile's mask and compact positions come from L2
    // after the first of them
    const int b = xcd_remap(blockIdx.x, ntx * nty * C);
    const int c = b % C, t = b / C;
    const int tx = t % ntx, ty = t / ntx;
    const int Tx = min(TB, W), Ty = min(TB, H);
    const int x0 = min(tx * sx, W - Tx), y0 = min(ty * sy, H - Ty);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int k = threadIdx.x; k < (TB + 2) * LocalTile<TB>::LW; k += NT) (&s_x[0][0])[k] = 0.f;
    __syncthreads();
    // the lane's 4x4 pixels: wavefront w takes quadrant (w & 1, w >> 1) of a 64 block
    const int ox = 32 * (w & 1) + 4 * (lane & 7), oy = 32 * (w >> 1) + 4 * (lane >> 3);
    LocalTile<TB> T{s_x, ox, oy, s_red};

    // pixel classes and right-hand side (all loads first, clamped addresses)
    int pk[16];
    uint8_t mk[16];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int xx = min(x0 + ox + i, W - 1), yy = min(y0 + oy + j, H - 1);
            pk[j * 4 + i] = pos[yy * W + xx];
            mk[j * 4 + i] = mask[yy * W + xx];
        }
    // pixel class in one value: degree in the block graph on U (> 0), 0 on
    // the mask, -1 outside the image (tiles narrower than TB)
    float dgU[16], s[16];
    float ss = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = j * 4 + i;
            const int lx = ox + i, ly = oy + j;
            const bool act = lx < Tx && ly < Ty;
            const bool known = act && mk[k];
            const float d = (float)((lx > 0) + (lx < Tx - 1) + (ly > 0) + (ly < Ty - 1));
            dgU[k] = !act ? -1.f : (known ? 0.f : d);
            s[k] = known ? (float)r[(size_t)c * m + pk[k]] : 0.f;
            ss += s[k] * s[k];
        }
    ss = T.sum(ss);

    // local CGNR on the mask pixels of the block
    float v[16], p[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) { v[k] = 0.f; p[k] = s[k]; }
    const float floor_ss = ss * 1e-14f;
    int n_local = 0, n_outer = 0;   // steps taken (counted for the FLOP statistics)
    for (int it = 0; it < nc && ss > floor_ss && ss >= FLT_MIN; ++it) {
        float tmp[16], u[16];
        // t = B_i p: p on K, inpainted values on U
        T.nbsum(p, tmp);
#pragma unroll
        for (int k = 0; k < 16; ++k) tmp[k] = dgU[k] > 0.f ? tmp[k] : 0.f;
        n_local += local_cg<TB>(T, dgU, tmp, u, ni);
        // t is parked in LDS (the lane's own 4x4) while the second solve runs
#pragma unroll
        for (int k = 0; k < 16; ++k) tmp[k] = dgU[k] == 0.f ? p[k] : u[k];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            *reinterpret_cast<float4 *>(&s_t[oy + j][ox]) =
                make_float4(tmp[j * 4 + 0], tmp[j * 4 + 1], tmp[j * 4 + 2], tmp[j * 4 + 3]);
        // q = B_i^T t = t_K + sum over unknown neighbours of (L_UU^{-1} t_U)
#pragma unroll
        for (int k = 0; k < 16; ++k) tmp[k] = dgU[k] > 0.f ? tmp[k] : 0.f;
        n_local += local_cg<TB>(T, dgU, tmp, u, ni);
        ++n_outer;
        T.nbsum(u, tmp);
        float pq = 0.f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float4 t4 = *reinterpret_cast<const float4 *>(&s_t[oy + j][ox]);
            const float tv[4] = {t4.x, t4.y, t4.z, t4.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = j * 4 + i;
                tmp[k] = dgU[k] == 0.f ? tv[i] + tmp[k] : 0.f;   // q
                pq += p[k] * tmp[k];
            }
        }
        pq = T.sum(pq);
        if (!(pq >= FLT_MIN)) break;
        const float alpha = ss * __builtin_amdgcn_rcpf(pq);
        float ss2 = 0.f;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            v[k] += alpha * p[k];
            s[k] -= alpha * tmp[k];
            ss2 += s[k] * s[k];
        }
        ss2 = T.sum(ss2);
        const float beta = ss2 * __builtin_amdgcn_rcpf(ss);
        ss = ss2;
#pragma unroll
        for (int k = 0; k < 16; ++k) p[k] = s[k] + beta * p[k];
    }

    if (steps && threadIdx.x == 0) steps[blockIdx.x] = ((unsigned)n_local << 8) | (unsigned)n_outer;
    // restricted write-back on owned mask pixels
    const int xlo = tx == 0 ? 0 : (min((tx - 1) * sx, W - Tx) + Tx + x0) / 2;
    const int xhi = tx == ntx - 1 ? W : (x0 + Tx + min((tx + 1) * sx, W - Tx)) / 2;
    const int ylo = ty == 0 ? 0 : (min((ty - 1) * sy, H - Ty) + Ty + y0) / 2;
    const int yhi = ty == nty - 1 ? H : (y0 + Ty + min((ty + 1) * sy, H - Ty)) / 2;
    // the compact positions are read again rather than kept live through the solve
    asm volatile("" ::: "memory");
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = j * 4 + i;
            const int x = x0 + ox + i, y = y0 + oy + j;
            if (dgU[k] == 0.f && x >= xlo && x < xhi && y >= ylo && y < yhi)
                z[(size_t)c * m + pos[y * W + x]] = (double)v[k];
        }
}

// ------------------------------------------------------------------ launchers

static inline dim3 g1(long n, int bs) { return dim3((unsigned)((n + bs - 1) / bs)); }

void launch_compact(int N, const uint8_t *mask, int *chunk_cnt, int *chunk_off, int *total, int *idx, int *pos,
                    hipStream_t s) {
    const int nch = (N + CMP_THREADS - 1) / CMP_THREADS;
    hipLaunchKernelGGL(k_compact_count, dim3(nch), dim3(CMP_THREADS), 0, s, N, mask, chunk_cnt);
    hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(CMP_THREADS), 0, s, nch, chunk_cnt, chunk_off, total);
    hipLaunchKernelGGL(k_compact_scatter, dim3(nch), dim3(CMP_THREADS), 0, s, N, mask, chunk_off, idx, pos);
}

void launch_scatter_K(int m, int C, int N, const int *idx, const double *v, double *img, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_K, g1(m, 256), dim3(256), 0, s, m, C, N, idx, v, img);
}

void launch_gather_f(int m, int C, int N, const int *idx, const float *f, double *v, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_f, g1(m, 256), dim3(256), 0, s, m, C, N, idx, f, v);
}

void launch_gather_Bt(int W, int H, int m, int C, const int *idx, const uint8_t *mask, const double *y,
                      const double *yK, const double *w, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_Bt, g1(m, 256), dim3(256), 0, s, W, H, m, C, idx, mask, y, yK, w, out);
}

constexpr int RED_BLOCKS = 512;

void launch_image_residual(int N, int C, const float *f, const double *u, double *rho, double *partials,
                           double *sums, hipStream_t s) {
    hipLaunchKernelGGL(k_image_residual, dim3(RED_BLOCKS), dim3(256), 0, s, N, C, f, u, rho, partials, RED_BLOCKS);
    hipLaunchKernelGGL(k_sum_rows, dim3(C), dim3(64), 0, s, C, RED_BLOCKS, partials, sums);
}

void launch_dots(int m, int C, int np, const double *const *a, const double *const *b, double *partials,
                 double *sums, hipStream_t s) {
    DotArgs args;
    for (int q = 0; q < 4; ++q) {
        args.a[q] = q < np ? a[q] : nullptr;
        args.b[q] = q < np ? b[q] : nullptr;
    }
    // one instantiation per product count (1..4) and channel count keeps the
    // sums in registers
    using Kern = void (*)(int, DotArgs, double *, int);
    static const Kern k3[4] = {k_dots<1, 3>, k_dots<2, 3>, k_dots<3, 3>, k_dots<4, 3>};
    static const Kern k1[4] = {k_dots<1, 1>, k_dots<2, 1>, k_dots<3, 1>, k_dots<4, 1>};
    const Kern kern = (C == 3 ? k3 : k1)[std::min(std::max(np, 1), 4) - 1];
    hipLaunchKernelGGL(kern, dim3(RED_BLOCKS), dim3(256), 0, s, m, args, partials, RED_BLOCKS);
    // sums laid out [q][3]
    hipLaunchKernelGGL(k_sum_rows, dim3(np * 3), dim3(64), 0, s, np * 3, RED_BLOCKS, partials, sums);
}

void launch_axpby(int m, int C, const double *a, const double *b, const double *x, double *y, hipStream_t s) {
    Coef3 k;
    for (int c = 0; c < 3; ++c) {
        k.a[c] = c < C ? a[c] : 0.0;
        k.b[c] = c < C ? b[c] : 0.0;
    }
    hipLaunchKernelGGL(k_axpby, g1(m, 256), dim3(256), 0, s, m, C, k, x, y);
}

void launch_ras_local(int W, int H, int C, int m, int block, int overlap, int nc, int ni, const uint8_t *mask,
                      const int *pos, const double *r, double *z, unsigned int *steps, hipStream_t s) {
    const Blocks1D bx = make_blocks(W, overlap, block), by = make_blocks(H, overlap, block);
    const dim3 g(bx.count * by.count * C);
    if (block == 64)
        hipLaunchKernelGGL(k_ras_local<64>, g, dim3(256), 0, s, W, H, C, m, bx.count, by.count, bx.stride, by.stride,
                           nc, ni, mask, pos, r, z, steps);
    else
        hipLaunchKernelGGL(k_ras_local<32>, g, dim3(64), 0, s, W, H, C, m, bx.count, by.count, bx.stride, by.stride,
                           nc, ni, mask, pos, r, z, steps);
}

// totals[0] += local CG steps, totals[1] += local CGNR steps over the n
// per-wave counts of a sweep (integer sums: exact in any order)
__global__ void k_sum_steps(int n, const unsigned int *__restrict__ steps, unsigned long long *__restrict__ totals) {
    unsigned long long a = 0, b = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        a += steps[i] >> 8;
        b += steps[i] & 0xFF;
    }
    __shared__ unsigned long long sa[256], sb[256];
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            sa[threadIdx.x] += sa[threadIdx.x + h];
            sb[threadIdx.x] += sb[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(totals, sa[0]);
        atomicAdd(totals + 1, sb[0]);
    }
}

__global__ void k_zero_totals(int n, unsigned long long *__restrict__ p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

void launch_sum_steps(int n, const unsigned int *steps, unsigned long long *totals, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_totals, dim3(1), dim3(64), 0, s, 2, totals);
    hipLaunchKernelGGL(k_sum_steps, dim3(64), dim3(256), 0, s, n, steps, totals);
}

}  // namespace hdi
