// Spatial optimisation: image-adaptive initial mask and the densification loop.
//
// Sec. 4.2 draws the initial mask by random dithering of the Laplacian
// magnitude: one biased coin flip per pixel, with a probability proportional to
// the magnitude. Alg. 1 then grows the mask over n steps, each one an
// inpainting, an error map and one densification step (Sec. 4.1).
//
// Readings that make the mask reproducible bit for bit: the magnitude is
// sum_c |Delta f_c| in FP64, added in a fixed order (up, down, left, right,
// minus four times the centre; channels in order), which is also exact for
// image data (five FP32 values whose exponents span fewer than 29 binades);
// the probabilities are
// alpha * l with alpha = n0 / (S 2^-16), S = sum_p round(l_p 2^16) summed as
// 64-bit integers (exact, so independent of the order); pixel p joins iff
// r_p < alpha * l_p for the caller's uniforms r. A constant image (S = 0) uses
// the uniform probability n0 / N.
#include <algorithm>
#include <cmath>
#include <vector>

#include "hdi_internal.h"

namespace hdi {

bool check_image(const hdi_image &img);

#define S_TRY(expr)                                                                                  \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) {                                                                      \
            set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__);   \
            return HDI_ERR_HIP;                                                                      \
        }                                                                                            \
    } while (0)

constexpr int LAP_SHIFT = 16;

// l_p = sum_c |f_up + f_down + f_left + f_right - 4 f| with a neighbour outside
// the image replaced by the pixel itself; adds round(l 2^16) per workgroup to
// the 64-bit total.
__global__ void __launch_bounds__(256)
k_lapmag(int W, int H, int C, const float *__restrict__ f, double *__restrict__ lap,
         unsigned long long *__restrict__ total) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long q = 0;
    if (i < W * H) {
        const int x = i % W, y = i / W;
        const int xl = x > 0 ? i - 1 : i, xr = x < W - 1 ? i + 1 : i;
        const int yu = y > 0 ? i - W : i, yd = y < H - 1 ? i + W : i;
        double acc = 0.0;
        for (int c = 0; c < C; ++c) {
            const float *fc = f + (size_t)c * W * H;
            // fixed order; exact for image data
            const double s = (double)fc[yu] + (double)fc[yd] + (double)fc[xl] + (double)fc[xr] - 4.0 * (double)fc[i];
            acc += fabs(s);
        }
        lap[i] = acc;
        q = (unsigned long long)rint(ldexp(acc, LAP_SHIFT));
    }
    // integer sums are exact in any order
    __shared__ unsigned long long s_q[4];
    for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off);
    if ((threadIdx.x & 63) == 0) s_q[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(total, s_q[0] + s_q[1] + s_q[2] + s_q[3]);
}

__global__ void __launch_bounds__(256)
k_coins(int N, const double *__restrict__ lap, const double *__restrict__ rnd, double alpha, double uniform_p,
        uint8_t *__restrict__ mask, unsigned long long *__restrict__ count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int hit = 0;
    if (i < N) {
        const double p = alpha > 0.0 ? alpha * lap[i] : uniform_p;
        hit = rnd[i] < p;
        mask[i] = (uint8_t)hit;
    }
    unsigned long long b = __ballot(hit);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(count, (unsigned long long)__popcll(b));
}

__global__ void k_zero_u64(int n, unsigned long long *p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// the initial mask of the loop; `lap` N doubles, `sums` two 64-bit counters
static int32_t init_mask(int W, int H, int C, const float *f, const double *rnd, long long n0, uint8_t *mask,
                         double *lap, unsigned long long *sums, long long *count, hipStream_t s) {
    const int N = W * H;
    const dim3 g((N + 255) / 256), b(256);
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, 2, sums);
    hipLaunchKernelGGL(k_lapmag, g, b, 0, s, W, H, C, f, lap, sums);
    unsigned long long S = 0;
    S_TRY(read_to_host(&S, sums, sizeof S, s));
    const double alpha = S > 0 ? (double)n0 / ((double)S * std::ldexp(1.0, -LAP_SHIFT)) : 0.0;
    const double uniform_p = (double)n0 / N;
    hipLaunchKernelGGL(k_coins, g, b, 0, s, N, lap, rnd, alpha, uniform_p, mask, sums + 1);
    unsigned long long cnt = 0;
    S_TRY(read_to_host(&cnt, sums + 1, sizeof cnt, s));
    *count = (long long)cnt;
    return HDI_OK;
}

// Cumulative mask sizes after each step: the added counts grow by the factor t
// and reach n_target after n steps (t = 1: equal steps, rounded half to even).
static std::vector<long long> schedule(long long n0, long long n_target, int n, double t) {
    std::vector<long long> out;
    const double delta = (double)(n_target - n0);
    if (t == 1.0) {
        for (int k = 1; k <= n; ++k) out.push_back(n0 + (long long)std::nearbyint(delta * k / n));
    } else {
        double tk = 1.0;
        const double tn = std::pow(t, n);
        for (int k = 1; k <= n; ++k) {
            tk *= t;
            out.push_back(n0 + (long long)std::floor(delta * (tk - 1.0) / (tn - 1.0) + 0.5));
        }
    }
    return out;
}

struct SpatialWs {
    void *inp, *dens;
    size_t inp_bytes, dens_bytes;
    float *err;
    double *u_alt, *u_own, *lap;
    int32_t *added;
    unsigned long long *sums;
};

static bool plan_spatial(SpatialWs &w, Arena &a, const hdi_image &img, bool own_u) {
    const size_t N = (size_t)img.width * img.height, C = img.channels;
    w.inp_bytes = hdi_inpaint_workspace_bytes(img);
    w.dens_bytes = hdi_densify_workspace_bytes(img.width, img.height);
    w.inp = a.take(w.inp_bytes);
    w.dens = a.take(w.dens_bytes);
    w.err = (float *)a.take(N * 4);
    w.u_alt = (double *)a.take(N * C * 8);
    w.u_own = own_u ? (double *)a.take(N * C * 8) : nullptr;
    w.lap = (double *)a.take(N * 8);
    w.added = (int32_t *)a.take(N * 4);
    w.sums = (unsigned long long *)a.take(16);
    return a.base == nullptr || a.used <= a.size;
}

}  // namespace hdi

using namespace hdi;

extern "C" {

size_t hdi_initial_mask_workspace_bytes(hdi_image img) {
    if (img.width < 1 || img.height < 1 || (img.channels != 1 && img.channels != 3)) return 0;
    return (size_t)img.width * img.height * 8 + 512;
}

int32_t hdi_initial_mask(hdi_image img, const float *f, const double *rand, int64_t n0, uint8_t *mask,
                         int64_t *count, void *ws, size_t ws_bytes, void *stream) {
    if (!check_image(img)) return HDI_ERR_ARG;
    if (!f || !rand || !mask || !count || n0 < 0) {
        set_error("f, rand, mask and count must be non-null and n0 >= 0");
        return HDI_ERR_ARG;
    }
    const size_t need = hdi_initial_mask_workspace_bytes(img);
    if (!ws || ws_bytes < need) {
        set_error("workspace of %zu bytes given, %zu needed", ws ? ws_bytes : (size_t)0, need);
        return HDI_ERR_WORKSPACE;
    }
    Arena a{(char *)ws, ws_bytes, 0};
    double *lap = (double *)a.take((size_t)img.width * img.height * 8);
    unsigned long long *sums = (unsigned long long *)a.take(16);
    long long c = 0;
    const int32_t st = init_mask(img.width, img.height, img.channels, f, rand, n0, mask, lap, sums, &c,
                                 (hipStream_t)stream);
    *count = c;
    return st;
}

size_t hdi_spatial_workspace_bytes(hdi_image img) {
    if (img.width < 1 || img.height < 1 || (img.channels != 1 && img.channels != 3)) return 0;
    SpatialWs w;
    Arena a{nullptr, 0, 0};
    plan_spatial(w, a, img, true);
    return a.used + 256;
}

int32_t spatial_optimize(hdi_image img, const float *f, const double *rand, const hdi_spatial_params *params,
                         uint8_t *mask, double *u, void *ws, size_t ws_bytes, hdi_spatial_report *report,
                         hdi_step_hook hook, void *hook_user, void *stream) {
    if (!check_image(img)) return HDI_ERR_ARG;
    if (!f || !rand || !mask || !params) {
        set_error("f, rand, mask and params must be non-null");
        return HDI_ERR_ARG;
    }
    const hdi_spatial_params &P = *params;
    const long long N = (long long)img.width * img.height;
    if (!(P.density > 0.0 && P.density <= 1.0) || P.n_steps < 1 || P.n_steps > 10000 || !(P.t > 0.0) ||
        ((P.partition & ~HDI_PART_JFA) != HDI_PART_DELAUNAY && (P.partition & ~HDI_PART_JFA) != HDI_PART_VORONOI)) {
        set_error("spatial parameters out of range (0 < density <= 1, 1 <= n_steps <= 10000, t > 0, partition)");
        return HDI_ERR_ARG;
    }
    const long long n_target = (long long)std::floor(P.density * (double)N);
    const long long n0 = P.n0 > 0 ? P.n0 : (long long)std::nearbyint((double)n_target / (P.n_steps + 1));
    if (n0 > n_target) {
        set_error("initial size %lld above the target %lld", n0, n_target);
        return HDI_ERR_ARG;
    }
    SpatialWs w;
    {
        Arena a{nullptr, 0, 0};
        plan_spatial(w, a, img, u == nullptr);
        if (!ws || ws_bytes < a.used + 256) {
            set_error("workspace of %zu bytes given, %zu needed", ws ? ws_bytes : (size_t)0, a.used + 256);
            return HDI_ERR_WORKSPACE;
        }
    }
    Arena a{(char *)ws, ws_bytes, 0};
    plan_spatial(w, a, img, u == nullptr);
    hipStream_t s = (hipStream_t)stream;
    CallTimer tm;
    S_TRY(tm.start(s));

    long long count = 0;
    int32_t st = init_mask(img.width, img.height, img.channels, f, rand, n0, mask, w.lap, w.sums, &count, s);
    if (st) return st;
    if (count == 0) {
        set_error("the initial mask came out empty (n0 = %lld)", n0);
        return HDI_ERR_EMPTY_MASK;
    }
    const long long c0 = count;
    const std::vector<long long> targets = schedule(c0, n_target, P.n_steps, P.t);
    double *cur = u ? u : w.u_own, *prev = w.u_alt;
    hdi_solve_report sr{};
    int rounds = 0;
    st = inpaint_solve(img, mask, f, cur, nullptr, w.inp, w.inp_bytes, &P.solve, &sr, stream);
    rounds += sr.outer_iters;
    if (st) return st;
    const size_t Nz = (size_t)N;
    std::vector<uint8_t> h_mask;
    std::vector<float> h_err;
    std::vector<int32_t> h_added;
    int jfa_k0 = 0;   // jump-flooding start of the next step (0: the default)
    for (int k = 0; k < P.n_steps; ++k) {
        st = hdi_error_map(img, cur, f, w.err, stream);
        if (st) return st;
        const long long want = std::max(targets[k] - count, 0LL);
        if (hook) {
            // host copies of what the step sees, for the caller's inspection
            h_mask.resize(Nz);
            h_err.resize(Nz);
            S_TRY(read_to_host(h_mask.data(), mask, Nz, s));
            S_TRY(read_to_host(h_err.data(), w.err, Nz * 4, s));
        }
        int64_t n_added = 0;
        uint64_t max_d2 = 0;
        st = densify_step_ex(img.width, img.height, mask, w.err, want, P.partition, jfa_k0, w.added, &n_added,
                             (P.partition & HDI_PART_JFA) ? &max_d2 : nullptr, w.dens, w.dens_bytes, s);
        if (st) return st;
        if (P.partition & HDI_PART_JFA) {
            // the mask only grows, so this step's largest distance bounds the next
            jfa_k0 = 1;
            while ((uint64_t)jfa_k0 * jfa_k0 < max_d2) jfa_k0 *= 2;
        }
        count += n_added;
        if (hook) {
            h_added.resize(std::max<int64_t>(n_added, 1));
            if (n_added)
                S_TRY(hipMemcpy(h_added.data(), w.added, sizeof(int32_t) * n_added, hipMemcpyDeviceToHost));
            hook(k, h_mask.data(), h_err.data(), h_added.data(), n_added, hook_user);
        }
        std::swap(cur, prev);
        st = inpaint_solve(img, mask, f, cur, prev, w.inp, w.inp_bytes, &P.solve, &sr, stream);
        rounds += sr.outer_iters;
        if (st) return st;
    }
    if (u && cur != u) S_TRY(hipMemcpyAsync(u, cur, sizeof(double) * Nz * img.channels, hipMemcpyDeviceToDevice, s));
    float ms = 0.f;
    S_TRY(tm.stop(s, &ms));
    if (report) {
        report->initial_count = c0;
        report->final_count = count;
        report->solve_rounds = rounds;
        for (int c = 0; c < 3; ++c) report->rel_residual[c] = sr.rel_residual[c];
        report->ms = ms;
    }
    return HDI_OK;
}

}  // extern "C"
