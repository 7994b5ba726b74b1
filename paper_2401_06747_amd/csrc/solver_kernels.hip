// Kernels of the masked-Laplace solve (paper Sec. 2.1 and Sec. 3) for gfx950.
//
// Operator: for pixel p with in-image 4-neighbours N4(p),
//   (L v)_p = deg(p) v_p - sum_{q in N4(p)} v_q,   deg(p) = |N4(p)|   (reflecting border)
//   (A v)_p = v_p if p is known, (L v)_p otherwise                 (eq. inp-discrete-lsi)
// The correction equation A e = r with r = 0 on known pixels pins e = 0 there,
// so every FP32 kernel below works on the unknown pixels only.
#include "hdi_internal.h"

namespace hdi {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int deg_of(int x, int y, int W, int H) {
    return (x > 0) + (x < W - 1) + (y > 0) + (y < H - 1);
}

// Sum over the 64 lanes of a wavefront. XOR butterfly: every lane ends with the
// same bits (each step adds the same two operands in either order).
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Map the hardware workgroup id to a block index so that each of the 8 XCDs
// (workgroups are dealt round-robin to them) works on one contiguous band of
// blocks, and neighbouring blocks share that XCD's L2 for their halos.
__device__ __forceinline__ int xcd_remap(int bid, int n) {
    const int q = n >> 3, rem = n & 7;
    const int x = bid & 7, k = bid >> 3;
    return x * q + min(x, rem) + k;
}

// ------------------------------------------------------------------ level-0 FP64 kernels

// u = u0 (or 0) on unknown pixels, u = data exactly on known pixels.
template <typename TD>
__global__ void k_init_u(int N, int C, const uint8_t *__restrict__ mask, const TD *__restrict__ data,
                         const double *__restrict__ u0, double *__restrict__ u) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const bool known = mask[i] != 0;
    for (int c = 0; c < C; ++c) {
        const size_t j = (size_t)c * N + i;
        u[j] = known ? (data ? (double)data[j] : 0.0) : (u0 ? u0[j] : 0.0);
    }
}

// r = b - A u in FP64 (b = data on known pixels, src (or 0) elsewhere), stored
// as FP32 for the inner solve, plus per-block FP64 partial sums of r^2 and b^2.
// One thread per pixel serves all channels, so the mask is read once (Sec. 2.1:
// the colour channels share the matrix).
template <typename TD>
__global__ void __launch_bounds__(RED_THREADS)
k_residual(int W, int H, int C, const uint8_t *__restrict__ mask, const double *__restrict__ u,
           const TD *__restrict__ data, const double *__restrict__ src, float *__restrict__ r,
           double *__restrict__ partials, int nblk) {
    const int N = W * H;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    __shared__ double s_red[RED_THREADS / 64][2];
    for (int c = 0; c < C; ++c) {
        double rr = 0.0, bb = 0.0;
        if (i < N) {
            const int x = i % W, y = i / W;
            const size_t o = (size_t)c * N;
            const double *uc = u + o;
            double res, b;
            if (mask[i]) {
                b = data ? (double)data[o + i] : 0.0;
                res = b - uc[i];
            } else {
                b = src ? src[o + i] : 0.0;
                double s = 0.0;
                int d = 0;
                if (x > 0) { s += uc[i - 1]; ++d; }
                if (x < W - 1) { s += uc[i + 1]; ++d; }
                if (y > 0) { s += uc[i - W]; ++d; }
                if (y < H - 1) { s += uc[i + W]; ++d; }
                res = b - (d * uc[i] - s);
            }
            r[o + i] = (float)res;
            rr = res * res;
            bb = b * b;
        }
        rr = wave_sum_d(rr);
        bb = wave_sum_d(bb);
        const int wid = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) { s_red[wid][0] = rr; s_red[wid][1] = bb; }
        __syncthreads();
        if (threadIdx.x == 0) {
            double a = 0.0, bsum = 0.0;
            for (int w = 0; w < RED_THREADS / 64; ++w) { a += s_red[w][0]; bsum += s_red[w][1]; }
            partials[((size_t)c * nblk + blockIdx.x) * 2 + 0] = a;
            partials[((size_t)c * nblk + blockIdx.x) * 2 + 1] = bsum;
        }
        __syncthreads();
    }
}

// Second stage of the fixed-order reduction: one workgroup per channel.
__global__ void __launch_bounds__(RED_THREADS)
k_reduce_partials(int nblk, const double *__restrict__ partials, double *__restrict__ norms) {
    const int c = blockIdx.x;
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nblk; k += RED_THREADS) {
        a += partials[((size_t)c * nblk + k) * 2 + 0];
        b += partials[((size_t)c * nblk + k) * 2 + 1];
    }
    a = wave_sum_d(a);
    b = wave_sum_d(b);
    __shared__ double s[RED_THREADS / 64][2];
    if ((threadIdx.x & 63) == 0) { s[threadIdx.x >> 6][0] = a; s[threadIdx.x >> 6][1] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0.0, y = 0.0;
        for (int w = 0; w < RED_THREADS / 64; ++w) { x += s[w][0]; y += s[w][1]; }
        norms[c * 2 + 0] = x;
        norms[c * 2 + 1] = y;
    }
}

// u += e on unknown pixels (iterative refinement step, FP64).
__global__ void k_update(int N, int C, const uint8_t *__restrict__ mask, const float *__restrict__ e,
                         double *__restrict__ u) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N || mask[i]) return;
    for (int c = 0; c < C; ++c) u[(size_t)c * N + i] += (double)e[(size_t)c * N + i];
}

// ------------------------------------------------------------------ grid transfers

// Coarse mask: a coarse pixel is known if any of its (up to) four fine pixels
// is known (Sec. 3.3).
__global__ void k_mask_restrict(int W, int H, const uint8_t *__restrict__ m, int Wc, int Hc,
                                uint8_t *__restrict__ mc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Wc * Hc) return;
    const int X = i % Wc, Y = i / Wc;
    uint8_t k = 0;
    for (int j = 0; j < 2; ++j)
        for (int q = 0; q < 2; ++q) {
            const int x = 2 * X + q, y = 2 * Y + j;
            if (x < W && y < H) k |= (m[y * W + x] != 0);
        }
    mc[i] = k;
}

// Coarse right-hand side: sum over the unknown fine children of the fine
// residual r - A e (the coarse operator is the same stencil on the coarse grid,
// so summing four children scales the averaged residual by H^2/h^2 = 4).
// Zero on coarse known pixels, where the coarse correction is pinned.
__global__ void k_restrict_residual(int W, int H, int C, const uint8_t *__restrict__ m,
                                    const float *__restrict__ r, const float *__restrict__ e,
                                    int Wc, int Hc, const uint8_t *__restrict__ mc, float *__restrict__ rc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Wc * Hc) return;
    const int X = i % Wc, Y = i / Wc;
    const int N = W * H, Nc = Wc * Hc;
    const bool cknown = mc[i] != 0;
    for (int c = 0; c < C; ++c) {
        float acc = 0.f;
        if (!cknown) {
            const float *ec = e + (size_t)c * N;
            const float *rcn = r + (size_t)c * N;
            for (int j = 0; j < 2; ++j)
                for (int q = 0; q < 2; ++q) {
                    const int x = 2 * X + q, y = 2 * Y + j;
                    if (x >= W || y >= H) continue;
                    const int p = y * W + x;
                    if (m[p]) continue;
                    float s = 0.f;
                    int d = 0;
                    if (x > 0) { s += ec[p - 1]; ++d; }
                    if (x < W - 1) { s += ec[p + 1]; ++d; }
                    if (y > 0) { s += ec[p - W]; ++d; }
                    if (y < H - 1) { s += ec[p + W]; ++d; }
                    acc += rcn[p] - ((float)d * ec[p] - s);
                }
        }
        rc[(size_t)c * Nc + i] = acc;
    }
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

// One restricted additive Schwarz step (Sec. 3.1) on 32x32 blocks: each block
// solves its local problem A_i v_i = R_i r^n with zero Dirichlet values outside
// the block (interior block boundaries) and the reflecting condition at the
// image border, by `iters` steps of conjugate gradients (Sec. 3.3). The
// correction is written back only on the pixels the block owns (the middle of
// each overlap splits ownership), which is a partition of unity with 0/1
// weights (eq. partition-of-unity-discrete).
//
// Layout: one wavefront (64 lanes) per block; lane (bx, by) = (lane & 7,
// lane >> 3) holds the 4x4 pixels (4bx + i, 4by + j) in registers. The search
// direction is exchanged through LDS (a 34 x 40 float tile with a zero halo),
// dot products use wavefront shuffles, so the block needs no barrier beyond
// its own wave.
//
// MODE 0: pre-smoothing from e = 0 (reads r only)
// MODE 1: post-smoothing of e_in + P ec (reads e_in with a 1-pixel halo and
//         the coarse correction ec around the block)
// MODE 2: FMG smoothing from the prolongated guess e_in (like MODE 1 with ec = 0)
constexpr int LDS_W = 40;   // row pitch of the LDS tiles (floats), 16-byte aligned rows
constexpr int COL0 = 4;     // LDS column of block column 0 (col 3 and 36 are the halo)

template <int MODE>
__global__ void __launch_bounds__(64)
k_schwarz(int W, int H, int C, int ntx, int nty, int sx, int sy, int iters,
          const uint8_t *__restrict__ mask, const float *__restrict__ r, const float *__restrict__ e_in,
          const float *__restrict__ ec, int Wc, int Hc, float *__restrict__ e_out) {
    __shared__ __attribute__((aligned(16))) float s_p[TILE + 2][LDS_W];
    __shared__ __attribute__((aligned(16))) float s_e[TILE + 2][LDS_W];
    __shared__ uint8_t s_m[TILE + 2][TILE + 2];

    const int ntiles = ntx * nty;
    const int t = xcd_remap(blockIdx.x, ntiles);
    const int c = blockIdx.y;
    const int tx = t % ntx, ty = t / ntx;
    const int Tx = min(TILE, W), Ty = min(TILE, H);
    const int x0 = min(tx * sx, W - Tx), y0 = min(ty * sy, H - Ty);
    const int N = W * H;
    const float *rc = r + (size_t)c * N;
    const int lane = threadIdx.x;

    // Stage mask and (MODE 1/2) the current correction, with a 1-pixel halo.
    // s_m: 0 unknown, 1 known, 2 outside the image.
    for (int k = lane; k < (TILE + 2) * (TILE + 2); k += 64) {
        const int ly = k / (TILE + 2), lx = k % (TILE + 2);
        const int x = x0 + lx - 1, y = y0 + ly - 1;
        const bool in = (x >= 0 && x < W && y >= 0 && y < H);
        const int p = y * W + x;
        const uint8_t mk = in ? (mask[p] != 0) : 2;
        s_m[ly][lx] = mk;
        if (MODE != 0) {
            float v = 0.f;
            if (in && (mk == 0 || MODE == 2)) {
                v = e_in[(size_t)c * N + p];
                if (MODE == 1) v += prolong_at(ec + (size_t)c * Wc * Hc, Wc, Hc, x, y);
            }
            s_e[ly][COL0 - 1 + lx] = v;
        }
        // zero halo ring of the search-direction tile
        s_p[ly][COL0 - 1 + lx] = 0.f;
    }
    __syncthreads();

    const int bx = lane & 7, by = lane >> 3;
    float v[16], rl[16], p[16], dg[16];
    float rr = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int lx = 4 * bx + i, ly = 4 * by + j, k = j * 4 + i;
            const int x = x0 + lx, y = y0 + ly;
            float res = 0.f, d = 0.f;
            if (lx < Tx && ly < Ty && s_m[ly + 1][lx + 1] == 0) {
                d = (float)deg_of(x, y, W, H);
                res = r ? rc[y * W + x] : 0.f;
                if (MODE != 0) {
                    const float s = s_e[ly][COL0 + lx] + s_e[ly + 2][COL0 + lx] +
                                    s_e[ly + 1][COL0 + lx - 1] + s_e[ly + 1][COL0 + lx + 1];
                    res -= d * s_e[ly + 1][COL0 + lx] - s;
                }
            }
            dg[k] = d;
            v[k] = 0.f;
            rl[k] = res;
            p[k] = res;
            rr += res * res;
        }
    rr = wave_sum(rr);

    for (int it = 0; it < iters && rr > 0.f; ++it) {
        // publish p
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float4 w4 = make_float4(p[j * 4 + 0], p[j * 4 + 1], p[j * 4 + 2], p[j * 4 + 3]);
            *reinterpret_cast<float4 *>(&s_p[4 * by + j + 1][COL0 + 4 * bx]) = w4;
        }
        __syncthreads();
        const float4 up = *reinterpret_cast<const float4 *>(&s_p[4 * by][COL0 + 4 * bx]);
        const float4 dn = *reinterpret_cast<const float4 *>(&s_p[4 * by + 5][COL0 + 4 * bx]);
        float lf[4], rt[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            lf[j] = s_p[4 * by + j + 1][COL0 + 4 * bx - 1];
            rt[j] = s_p[4 * by + j + 1][COL0 + 4 * bx + 4];
        }
        const float upv[4] = {up.x, up.y, up.z, up.w};
        const float dnv[4] = {dn.x, dn.y, dn.z, dn.w};
        float q[16];
        float pq = 0.f;
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = j * 4 + i;
                const float n = (j > 0 ? p[k - 4] : upv[i]) + (j < 3 ? p[k + 4] : dnv[i]) +
                                (i > 0 ? p[k - 1] : lf[j]) + (i < 3 ? p[k + 1] : rt[j]);
                q[k] = dg[k] > 0.f ? dg[k] * p[k] - n : 0.f;
                pq += p[k] * q[k];
            }
        pq = wave_sum(pq);
        if (!(pq > 0.f)) break;
        const float alpha = rr / pq;
        float rr2 = 0.f;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            v[k] += alpha * p[k];
            rl[k] -= alpha * q[k];
            rr2 += rl[k] * rl[k];
        }
        rr2 = wave_sum(rr2);
        const float beta = rr2 / rr;
        rr = rr2;
#pragma unroll
        for (int k = 0; k < 16; ++k) p[k] = rl[k] + beta * p[k];
        __syncthreads();
    }

    // Restricted write-back on the owned part of the block.
    const int xlo = tx == 0 ? 0 : (min((tx - 1) * sx, W - Tx) + Tx + x0) / 2;
    const int xhi = tx == ntx - 1 ? W : (x0 + Tx + min((tx + 1) * sx, W - Tx)) / 2;
    const int ylo = ty == 0 ? 0 : (min((ty - 1) * sy, H - Ty) + Ty + y0) / 2;
    const int yhi = ty == nty - 1 ? H : (y0 + Ty + min((ty + 1) * sy, H - Ty)) / 2;
    float *eo = e_out + (size_t)c * N;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int lx = 4 * bx + i, ly = 4 * by + j;
            const int x = x0 + lx, y = y0 + ly;
            if (lx < Tx && ly < Ty && x >= xlo && x < xhi && y >= ylo && y < yhi) {
                float base = 0.f;
                if (MODE != 0) base = s_e[ly + 1][COL0 + lx];
                eo[y * W + x] = dg[j * 4 + i] > 0.f ? base + v[j * 4 + i] : (MODE == 2 ? base : 0.f);
            }
        }
}

// ------------------------------------------------------------------ reduced FMG (Sec. 3.2)

// Data on the first coarse level: a coarse known pixel takes the mean of its
// known fine children's values (Sec. 3.3).
template <typename TD>
__global__ void k_data_restrict0(int W, int H, int C, const uint8_t *__restrict__ m, const TD *__restrict__ d,
                                 int Wc, int Hc, const uint8_t *__restrict__ mc, float *__restrict__ dc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
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

// FMG prolongation: out = P ec on unknown pixels, the level's data on known ones.
__global__ void k_fmg_prolong(int W, int H, int C, const uint8_t *__restrict__ m, const float *__restrict__ data,
                              const float *__restrict__ ec, int Wc, int Hc, float *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= W * H) return;
    const int x = i % W, y = i / W;
    for (int c = 0; c < C; ++c) {
        const size_t j = (size_t)c * W * H + i;
        out[j] = m[i] ? data[j] : prolong_at(ec + (size_t)c * Wc * Hc, Wc, Hc, x, y);
    }
}

// Level-0 FMG prolongation into the FP64 iterate (known pixels keep the data).
__global__ void k_fmg_prolong0(int W, int H, int C, const uint8_t *__restrict__ m, const float *__restrict__ ec,
                               int Wc, int Hc, double *__restrict__ u) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= W * H || m[i]) return;
    const int x = i % W, y = i / W;
    for (int c = 0; c < C; ++c) u[(size_t)c * W * H + i] = (double)prolong_at(ec + (size_t)c * Wc * Hc, Wc, Hc, x, y);
}

// ------------------------------------------------------------------ launchers

static inline dim3 grid1(long n, int bs) { return dim3((unsigned)((n + bs - 1) / bs)); }

void launch_mask_restrict(const Level &f, const Level &c, hipStream_t s) {
    hipLaunchKernelGGL(k_mask_restrict, grid1((long)c.W * c.H, 256), dim3(256), 0, s, f.W, f.H, f.mask, c.W, c.H, c.mask);
}

template <typename TD>
void launch_init_u(int W, int H, int C, const uint8_t *mask, const TD *data, const double *u0, double *u, hipStream_t s) {
    hipLaunchKernelGGL(k_init_u<TD>, grid1((long)W * H, 256), dim3(256), 0, s, W * H, C, mask, data, u0, u);
}

template <typename TD>
void launch_residual(int W, int H, int C, const uint8_t *mask, const double *u, const TD *data, const double *src,
                     float *r, double *partials, int nblk, double *norms, hipStream_t s) {
    hipLaunchKernelGGL(k_residual<TD>, dim3(nblk), dim3(RED_THREADS), 0, s, W, H, C, mask, u, data, src, r, partials, nblk);
    hipLaunchKernelGGL(k_reduce_partials, dim3(C), dim3(RED_THREADS), 0, s, nblk, partials, norms);
}

void launch_update(int W, int H, int C, const uint8_t *mask, const float *e, double *u, hipStream_t s) {
    hipLaunchKernelGGL(k_update, grid1((long)W * H, 256), dim3(256), 0, s, W * H, C, mask, e, u);
}

void launch_smooth_pre(const Level &L, int C, int iters, float *e_out, hipStream_t s) {
    dim3 g(L.bx.count * L.by.count, C);
    hipLaunchKernelGGL(k_schwarz<0>, g, dim3(64), 0, s, L.W, L.H, C, L.bx.count, L.by.count, L.bx.stride,
                       L.by.stride, iters, L.mask, L.r, (const float *)nullptr, (const float *)nullptr, 1, 1, e_out);
}

void launch_smooth_post(const Level &L, const Level &Lc, int C, int iters, const float *e_in, const float *ec,
                        float *e_out, hipStream_t s) {
    dim3 g(L.bx.count * L.by.count, C);
    hipLaunchKernelGGL(k_schwarz<1>, g, dim3(64), 0, s, L.W, L.H, C, L.bx.count, L.by.count, L.bx.stride,
                       L.by.stride, iters, L.mask, L.r, e_in, ec, Lc.W, Lc.H, e_out);
}

void launch_smooth_fmg(const Level &L, int C, int iters, const float *e_in, float *e_out, hipStream_t s) {
    dim3 g(L.bx.count * L.by.count, C);
    // the full problem A u = C d has a zero right-hand side on unknown pixels
    hipLaunchKernelGGL(k_schwarz<2>, g, dim3(64), 0, s, L.W, L.H, C, L.bx.count, L.by.count, L.bx.stride,
                       L.by.stride, iters, L.mask, (const float *)nullptr, e_in, (const float *)nullptr, 1, 1, e_out);
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

template void launch_init_u<float>(int, int, int, const uint8_t *, const float *, const double *, double *, hipStream_t);
template void launch_init_u<double>(int, int, int, const uint8_t *, const double *, const double *, double *, hipStream_t);
template void launch_residual<float>(int, int, int, const uint8_t *, const double *, const float *, const double *,
                                     float *, double *, int, double *, hipStream_t);
template void launch_residual<double>(int, int, int, const uint8_t *, const double *, const double *, const double *,
                                      float *, double *, int, double *, hipStream_t);
template void launch_data_restrict0<float>(int, int, int, const uint8_t *, const float *, const Level &, hipStream_t);
template void launch_data_restrict0<double>(int, int, int, const uint8_t *, const double *, const Level &, hipStream_t);

}  // namespace hdi
