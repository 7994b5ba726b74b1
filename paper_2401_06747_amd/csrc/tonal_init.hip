// Voronoi initialisation of tonal optimisation (paper Sec. 5.3) and its C-ABI
// entry point.
//
// The surrogate problem asks the inpainting u = B g to reproduce weighted local
// averages of f around every mask pixel, C W u = C W f, and a Richardson
// iteration g_K <- g_K + tau (W (f - u))_K solves it; one inpainting per step.
// W is row-normalised over either the clipped 3x3 window of the mask pixel or
// its exact Voronoi cell (the labels of the densification step), the latter
// with constant or inverse-logarithmic distance weights. The paper stops once
// the MSE rises and keeps the best iterate.
//
// GPU layout: per step one inpainting (warm-started from the previous one),
// one scan over the image that forms f - u, its per-channel sums of squares
// (fixed-order partials) and, for Voronoi weights, the cell sums of
// round(W_j (f_j - u_j) 2^32) in 64-bit integer atomics (exact, so the result
// does not depend on the order of the atomics), and one update over the mask.
#include <algorithm>
#include <cmath>

#include "hdi_internal.h"
#include "wave.h"

namespace hdi {

bool check_image(const hdi_image &img);
int32_t fill_cfg(const hdi_solve_params *p, SolveCfg &cfg, int &overlap);

namespace {

constexpr int VI_THREADS = 256;
constexpr int VI_BLOCKS = 1024;   // scan grid (grid-stride): fixed partial order
constexpr int VI_RUN = 8;         // consecutive pixels per thread and pass of the scan
constexpr double FIX = 4294967296.0;          // 2^32
constexpr double FIX_INV = 1.0 / 4294967296.0;
constexpr double V_MAX = 1073741824.0;        // 2^30: bound on |f - u| that keeps cell sums in 64 bits

inline dim3 gd(long n) { return dim3((unsigned)std::max<long>(1, (n + 255) / 256)); }

__global__ void k_vi_fill_ll(long n, long long *__restrict__ p) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// g = f (from_f) or g itself on the mask, 0 elsewhere.
__global__ void k_vi_start(int N, int C, const uint8_t *__restrict__ mask, const float *__restrict__ f, bool from_f,
                           double *__restrict__ g) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const bool known = mask[i] != 0;
    for (int c = 0; c < C; ++c) {
        const size_t j = (size_t)c * N + i;
        g[j] = known ? (from_f ? (double)f[j] : g[j]) : 0.0;
    }
}

// Raw weight of every pixel for its cell (constant, or 1 / (1 + ln(1 + d)) at
// distance d from the cell's mask pixel) and the cell totals in fixed point.
__global__ void k_vi_weights(int W, int H, bool log_w, const int *__restrict__ labels, double *__restrict__ w,
                             long long *__restrict__ z) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= W * H) return;
    const int l = labels[i];
    const double dx = (double)(i % W - l % W), dy = (double)(i / W - l / W);
    const double v = log_w ? 1.0 / (1.0 + log1p(sqrt(dx * dx + dy * dy))) : 1.0;
    w[i] = v;
    atomicAdd(reinterpret_cast<unsigned long long *>(z + l), (unsigned long long)__double2ll_rn(v * FIX));
}

__global__ void k_vi_normalise(int N, const int *__restrict__ labels, const long long *__restrict__ z,
                               double *__restrict__ w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    w[i] = w[i] / ((double)z[labels[i]] * FIX_INV);
}

// One pass over f - u: per-workgroup sums of squares per channel into
// part[c][block], and (VOR) the fixed-point cell sums of w_j (f_j - u_j) into
// acc[c][label]. Each thread takes runs of VI_RUN consecutive pixels and adds
// one atomic per run of equal labels. flag[0] is set if |f - u| >= 2^30 or is
// not finite.
template <int C, bool VOR>
__global__ void __launch_bounds__(VI_THREADS)
k_vi_scan(int N, const float *__restrict__ f, const double *__restrict__ u, const int *__restrict__ labels,
          const double *__restrict__ w, long long *__restrict__ acc, double *__restrict__ part, int *__restrict__ flag) {
    double sq[C];
#pragma unroll
    for (int c = 0; c < C; ++c) sq[c] = 0.0;
    bool bad = false;
    for (long base = ((long)blockIdx.x * VI_THREADS + threadIdx.x) * VI_RUN; base < N;
         base += (long)VI_BLOCKS * VI_THREADS * VI_RUN) {
        const int end = (int)std::min<long>(base + VI_RUN, N);
        int cur = -1;
        long long run[C];
#pragma unroll
        for (int c = 0; c < C; ++c) run[c] = 0;
        for (int j = (int)base; j < end; ++j) {
            const int l = VOR ? labels[j] : 0;
            const double wj = VOR ? w[j] : 0.0;
            if (VOR && l != cur) {
                if (cur >= 0) {
#pragma unroll
                    for (int c = 0; c < C; ++c)
                        if (run[c]) atomicAdd(reinterpret_cast<unsigned long long *>(acc + (size_t)c * N + cur),
                                              (unsigned long long)run[c]);
                }
                cur = l;
#pragma unroll
                for (int c = 0; c < C; ++c) run[c] = 0;
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const double v = (double)f[(size_t)c * N + j] - u[(size_t)c * N + j];
                sq[c] += v * v;
                const bool ok = fabs(v) < V_MAX;   // false for NaN too
                bad |= !ok;
                if (VOR && ok) run[c] += __double2ll_rn(wj * v * FIX);
            }
        }
        if (VOR && cur >= 0) {
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (run[c]) atomicAdd(reinterpret_cast<unsigned long long *>(acc + (size_t)c * N + cur),
                                      (unsigned long long)run[c]);
        }
    }
    if (bad) atomicOr(flag, 1);
    __shared__ double s[VI_THREADS / 64][C];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const double t = wave_sum_d(sq[c]);
        if (lane == 0) s[wid][c] = t;
    }
    __syncthreads();
    if (threadIdx.x < C) {
        double t = 0.0;
        for (int k = 0; k < VI_THREADS / 64; ++k) t += s[k][threadIdx.x];
        part[(size_t)threadIdx.x * VI_BLOCKS + blockIdx.x] = t;
    }
}

// sums[c] = sum of the VI_BLOCKS partials of channel c, in a fixed order.
__global__ void __launch_bounds__(1024) k_vi_reduce(const double *__restrict__ part, double *__restrict__ sums) {
    const int c = blockIdx.x;
    const double t = wave_sum_d(part[(size_t)c * VI_BLOCKS + threadIdx.x]);
    __shared__ double s[16];
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0.0;
        for (int k = 0; k < 16; ++k) x += s[k];
        sums[c] = x;
    }
}
static_assert(VI_BLOCKS == 1024, "k_vi_reduce takes one partial per thread");

// g_next = g + tau (W (f - u)) on the mask, 0 elsewhere. DIRECT: the mean of
// f - u over the clipped 3x3 window; otherwise the cell sum in acc, which is
// cleared for the next pass.
template <bool DIRECT>
__global__ void k_vi_update(int W, int H, int C, double tau, const uint8_t *__restrict__ mask,
                            const float *__restrict__ f, const double *__restrict__ u, long long *__restrict__ acc,
                            const double *__restrict__ g, double *__restrict__ g_next) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = W * H;
    if (i >= N) return;
    if (!mask[i]) {
        for (int c = 0; c < C; ++c) g_next[(size_t)c * N + i] = 0.0;
        return;
    }
    const int x = i % W, y = i / W;
    for (int c = 0; c < C; ++c) {
        const size_t o = (size_t)c * N;
        double a;
        if (DIRECT) {
            double sum = 0.0;
            int cnt = 0;
            for (int yy = max(y - 1, 0); yy <= min(y + 1, H - 1); ++yy)
                for (int xx = max(x - 1, 0); xx <= min(x + 1, W - 1); ++xx) {
                    const size_t j = o + (size_t)yy * W + xx;
                    sum += (double)f[j] - u[j];
                    ++cnt;
                }
            a = sum / cnt;
        } else {
            a = (double)acc[o + i] * FIX_INV;
            acc[o + i] = 0;
        }
        g_next[o + i] = g[o + i] + tau * a;
    }
}

struct VinitWs {
    Hierarchy h;
    double *g_alt, *u_a, *u_b, *w, *part, *sums;
    int *labels, *scratch, *flag;
    long long *acc;
};

bool plan_vinit(VinitWs &v, Arena &a, int W, int H, int C, int overlap, const uint8_t *mask, int small_from) {
    if (!plan_hierarchy(v.h, a, W, H, C, overlap, mask, small_from)) return false;
    const size_t N = (size_t)W * H;
    v.g_alt = (double *)a.take(N * C * sizeof(double));
    v.u_a = (double *)a.take(N * C * sizeof(double));
    v.u_b = (double *)a.take(N * C * sizeof(double));
    v.w = (double *)a.take(N * sizeof(double));
    v.acc = (long long *)a.take(N * C * sizeof(long long));
    v.labels = (int *)a.take(N * sizeof(int));
    v.scratch = (int *)a.take(voronoi_scratch_ints(W, H) * sizeof(int));
    v.part = (double *)a.take((size_t)C * VI_BLOCKS * sizeof(double));
    v.sums = (double *)a.take(4 * sizeof(double));
    v.flag = (int *)a.take(sizeof(long long));   // cleared as one 64-bit word
    return a.base == nullptr || a.used <= a.size;
}

size_t vinit_ws_bytes(int W, int H, int C) {
    VinitWs v;
    Arena a{nullptr, 0, 0};
    plan_vinit(v, a, W, H, C, 4, nullptr, -1);
    return a.used + 256;
}

#define V_TRY(expr)                                                                                  \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) {                                                                      \
            set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__);   \
            return HDI_ERR_HIP;                                                                      \
        }                                                                                            \
    } while (0)

struct Vinit {
    VinitWs &v;
    int W, H, C, N;
    const uint8_t *mask;
    const float *f;
    int weighting;
    hipStream_t s;

    // MSE of u (and, for Voronoi weights, the cell sums of W (f - u) into acc)
    int32_t scan(const double *u, double &mse) {
        const bool vor = weighting != HDI_VINIT_DIRECT;
        hipLaunchKernelGGL(k_vi_fill_ll, dim3(1), dim3(64), 0, s, 1L, (long long *)v.flag);
        if (C == 3) {
            if (vor)
                hipLaunchKernelGGL((k_vi_scan<3, true>), dim3(VI_BLOCKS), dim3(VI_THREADS), 0, s, N, f, u, v.labels,
                                   v.w, v.acc, v.part, v.flag);
            else
                hipLaunchKernelGGL((k_vi_scan<3, false>), dim3(VI_BLOCKS), dim3(VI_THREADS), 0, s, N, f, u, v.labels,
                                   v.w, v.acc, v.part, v.flag);
        } else {
            if (vor)
                hipLaunchKernelGGL((k_vi_scan<1, true>), dim3(VI_BLOCKS), dim3(VI_THREADS), 0, s, N, f, u, v.labels,
                                   v.w, v.acc, v.part, v.flag);
            else
                hipLaunchKernelGGL((k_vi_scan<1, false>), dim3(VI_BLOCKS), dim3(VI_THREADS), 0, s, N, f, u, v.labels,
                                   v.w, v.acc, v.part, v.flag);
        }
        hipLaunchKernelGGL(k_vi_reduce, dim3(C), dim3(1024), 0, s, v.part, v.sums);
        V_TRY(hipGetLastError());
        double sums[3];
        int flag = 0;
        V_TRY(hipMemcpyAsync(sums, v.sums, sizeof(double) * C, hipMemcpyDeviceToHost, s));
        V_TRY(read_to_host(&flag, v.flag, sizeof(int), s));
        if (flag) {
            set_error("|f - B g| reached 2^30 or is not finite: the Richardson steps diverge (step size too large)");
            return HDI_ERR_ARG;
        }
        double t = 0.0;
        for (int c = 0; c < C; ++c) t += sums[c];
        mse = t / ((double)C * N);
        return HDI_OK;
    }
};

}  // namespace
}  // namespace hdi

using namespace hdi;

extern "C" {

size_t hdi_vinit_workspace_bytes(hdi_image img) {
    if (img.width < 1 || img.height < 1 || (img.channels != 1 && img.channels != 3)) return 0;
    return vinit_ws_bytes(img.width, img.height, img.channels);
}

int32_t voronoi_init(hdi_image img, const uint8_t *mask, const float *f, double *g, double *u, void *ws,
                     size_t ws_bytes, const hdi_vinit_params *params, hdi_vinit_report *report, void *stream) {
    if (!check_image(img)) return HDI_ERR_ARG;
    if (!mask || !f || !g) {
        set_error("mask, f and g must be non-null device pointers");
        return HDI_ERR_ARG;
    }
    const int weighting = params ? params->weighting : HDI_VINIT_VORONOI_LOG;
    const int max_iters = (params && params->max_iters > 0) ? params->max_iters : 20;
    const double tau = (params && params->tau != 0.0) ? params->tau : 1.0;
    const int flags = params ? params->flags : 0;
    if (weighting < HDI_VINIT_DIRECT || weighting > HDI_VINIT_VORONOI_LOG || max_iters > 1000 ||
        !(tau > 0.0 && tau < 1e6) || (flags & ~(HDI_VINIT_FROM_F | HDI_VINIT_NO_STOP))) {
        set_error("Voronoi-initialisation parameter out of range (weighting 0..2, max_iters <= 1000, tau > 0, "
                  "flags HDI_VINIT_FROM_F | HDI_VINIT_NO_STOP)");
        return HDI_ERR_ARG;
    }
    SolveCfg cfg;
    int overlap;
    int32_t st = fill_cfg(params ? &params->solve : nullptr, cfg, overlap);
    if (st) return st;
    const int W = img.width, H = img.height, C = img.channels, N = W * H;
    const size_t need = vinit_ws_bytes(W, H, C);
    if (!ws || ws_bytes < need) {
        set_error("workspace of %zu bytes given, %zu needed", ws ? ws_bytes : (size_t)0, need);
        return HDI_ERR_WORKSPACE;
    }
    hipStream_t s = (hipStream_t)stream;
    CallTimer tm;
    V_TRY(tm.start(s));
    Arena a{(char *)ws, ws_bytes, 0};
    VinitWs v;
    plan_vinit(v, a, W, H, C, overlap, mask, cfg.small_from);
    st = prepare_mask(v.h, s);
    if (st) return st;
    cfg.known = v.h.known[0];
    Vinit X{v, W, H, C, N, mask, f, weighting, s};

    hipLaunchKernelGGL(k_vi_start, gd(N), dim3(256), 0, s, N, C, mask, f, (flags & HDI_VINIT_FROM_F) != 0, g);
    const long nacc = (long)N * C;
    hipLaunchKernelGGL(k_vi_fill_ll, gd(nacc), dim3(256), 0, s, nacc, v.acc);
    if (weighting != HDI_VINIT_DIRECT) {
        launch_voronoi_labels(W, H, mask, v.scratch, v.labels, s);
        hipLaunchKernelGGL(k_vi_weights, gd(N), dim3(256), 0, s, W, H, weighting == HDI_VINIT_VORONOI_LOG, v.labels,
                           v.w, v.acc);
        hipLaunchKernelGGL(k_vi_normalise, gd(N), dim3(256), 0, s, N, v.labels, v.acc, v.w);
        hipLaunchKernelGGL(k_vi_fill_ll, gd(N), dim3(256), 0, s, (long)N, v.acc);
    }
    V_TRY(hipGetLastError());

    double *gc = g, *gn = v.g_alt, *uc = v.u_a, *un = v.u_b;
    const size_t bytes = sizeof(double) * C * N;
    int solves = 0, steps = 0, best = 0;
    double trace[HDI_VINIT_TRACE] = {};
    double mse_prev = 0.0, mse = 0.0;
    st = solve_system<double>(v.h, W, H, C, mask, gc, nullptr, uc, false, cfg, nullptr, s, nullptr, &uc);
    ++solves;
    if (st == HDI_OK) st = X.scan(uc, mse);
    if (st == HDI_OK) {
        trace[0] = mse;
        for (int k = 1; k <= max_iters; ++k) {
            if (weighting == HDI_VINIT_DIRECT)
                hipLaunchKernelGGL(k_vi_update<true>, gd(N), dim3(256), 0, s, W, H, C, tau, mask, f, uc, v.acc, gc,
                                   gn);
            else
                hipLaunchKernelGGL(k_vi_update<false>, gd(N), dim3(256), 0, s, W, H, C, tau, mask, f, uc, v.acc, gc,
                                   gn);
            V_TRY(hipMemcpyAsync(un, uc, bytes, hipMemcpyDeviceToDevice, s));   // warm start
            st = solve_system<double>(v.h, W, H, C, mask, gn, nullptr, un, true, cfg, nullptr, s, nullptr, &un);
            ++solves;
            if (st == HDI_OK) {
                mse_prev = mse;
                st = X.scan(un, mse);
            }
            if (st != HDI_OK) break;
            steps = k;
            if (k < HDI_VINIT_TRACE) trace[k] = mse;
            if (!(flags & HDI_VINIT_NO_STOP) && mse > mse_prev) break;
            std::swap(gc, gn);
            std::swap(uc, un);
            best = k;
        }
    }
    if (st == HDI_OK) {
        if (gc != g) V_TRY(hipMemcpyAsync(g, gc, bytes, hipMemcpyDeviceToDevice, s));
        if (u) V_TRY(hipMemcpyAsync(u, uc, bytes, hipMemcpyDeviceToDevice, s));
    }
    V_TRY(hipGetLastError());
    float ms = 0.f;
    V_TRY(tm.stop(s, &ms));
    if (report) {
        report->steps = steps;
        report->best = best;
        report->solves = solves;
        for (int k = 0; k < HDI_VINIT_TRACE; ++k) report->mse[k] = k <= steps ? trace[k] : 0.0;
        report->ms = ms;
    }
    return st;
}

}  // extern "C"
