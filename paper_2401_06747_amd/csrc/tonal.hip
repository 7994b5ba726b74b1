// Host driver of tonal optimisation (paper Sec. 5) and its C-ABI entry point.
//
// Solves the normal equations B^T B g = B^T f on the mask pixels
// (eq. tonal-normal-equations) matrix-free: every product with B is one
// inpainting solve and every product with B^T one solve of the symmetrised
// system plus a neighbour gather (Sec. 5.1). Three outer methods:
//   PCG_RAS  flexible conjugate gradients preconditioned by one RAS sweep of
//            local normal-equation solves on overlapping blocks (Sec. 5.2)
//   RAS      the stationary RAS iteration of Alg. 2 with warm-started global
//            inpaintings (Sec. 5.2)
//   CGNR     conjugate gradients on the normal equations (Sec. 5.1)
// Outer dot products and vectors are FP64; the inner solves are the FP64
// refinement around FP32 multigrid of inpaint.hip, with tolerances relaxed as
// the outer residual falls, and the final normal residual is recomputed with
// tight solves before convergence is reported.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "hdi_internal.h"

namespace hdi {

// tonal_kernels.hip
void launch_compact(int N, const uint8_t *mask, int *chunk_cnt, int *chunk_off, int *total, int *idx, int *pos,
                    hipStream_t s);
void launch_scatter_K(int m, int C, int N, const int *idx, const double *v, double *img, hipStream_t s);
void launch_gather_f(int m, int C, int N, const int *idx, const float *f, double *v, hipStream_t s);
void launch_gather_Bt(int W, int H, int m, int C, const int *idx, const uint8_t *mask, const double *y,
                      const double *yK, const double *w, double *out, hipStream_t s);
void launch_image_residual(int N, int C, const float *f, const double *u, double *rho, double *partials,
                           double *sums, hipStream_t s);
void launch_dots(int m, int C, int np, const double *const *a, const double *const *b, double *partials,
                 double *sums, hipStream_t s);
void launch_axpby(int m, int C, const double *a, const double *b, const double *x, double *y, hipStream_t s);
void launch_ras_local(int W, int H, int C, int m, int block, int overlap, int nc, int ni, const uint8_t *mask,
                      const int *pos, const double *r, double *z, unsigned int *steps, hipStream_t s);
void launch_sum_steps(int n, const unsigned int *steps, unsigned long long *totals, hipStream_t s);
bool check_image(const hdi_image &img);
int32_t fill_cfg(const hdi_solve_params *p, SolveCfg &cfg, int &overlap);

#define T_TRY(expr)                                                                                  \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) {                                                                      \
            set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__);   \
            return HDI_ERR_HIP;                                                                      \
        }                                                                                            \
    } while (0)
#define T_ST(expr)                        \
    do {                                  \
        int32_t s_ = (expr);              \
        if (s_ != HDI_OK) return s_;      \
    } while (0)

struct TonalWs {
    Hierarchy h;
    int *pos, *idx, *chunk_cnt, *chunk_off, *total;
    double *gK, *rK, *zK, *pK, *qK, *qprev, *bK;   // compact [C][m] (allocated for m = N)
    double *img_d, *uB, *wA, *rho;                 // full images C x N
    double *ug, *wr;                               // B g and L_UU^{-1} rho_U (running estimates)
    double *partials, *sums;                      // reductions
    unsigned int *ras_steps;                      // per-wave step counts of a RAS sweep (statistics)
    unsigned long long *ras_totals;
};

static bool plan_tonal(TonalWs &t, Arena &a, int W, int H, int C, int overlap, const uint8_t *mask,
                       int small_from = -1) {
    if (!plan_hierarchy(t.h, a, W, H, C, overlap, mask, small_from)) return false;
    const size_t N = (size_t)W * H;
    const int nch = (int)((N + 1023) / 1024);
    t.pos = (int *)a.take(N * sizeof(int));
    t.idx = (int *)a.take(N * sizeof(int));
    t.chunk_cnt = (int *)a.take(nch * sizeof(int));
    t.chunk_off = (int *)a.take(nch * sizeof(int));
    t.total = (int *)a.take(sizeof(int));
    double **vecs[] = {&t.gK, &t.rK, &t.zK, &t.pK, &t.qK, &t.qprev, &t.bK};
    for (double **v : vecs) *v = (double *)a.take(N * C * sizeof(double));
    double **imgs[] = {&t.img_d, &t.uB, &t.wA, &t.rho, &t.ug, &t.wr};
    for (double **v : imgs) *v = (double *)a.take(N * C * sizeof(double));
    t.partials = (double *)a.take(12 * 512 * sizeof(double));
    t.sums = (double *)a.take(16 * sizeof(double));
    // sized for the narrowest block stride (overlap 16)
    const size_t nwaves = (size_t)make_blocks(W, 16).count * make_blocks(H, 16).count * C;
    t.ras_steps = (unsigned int *)a.take(nwaves * sizeof(unsigned int));
    t.ras_totals = (unsigned long long *)a.take(2 * sizeof(unsigned long long));
    return a.base == nullptr || a.used <= a.size;
}

size_t tonal_ws_bytes(int W, int H, int C) {
    TonalWs t;
    Arena a{nullptr, 0, 0};
    plan_tonal(t, a, W, H, C, 6, nullptr);
    return a.used + 256;
}

struct TonalCtx {
    TonalWs &t;
    int W, H, C, N, m;
    const uint8_t *mask;
    const float *f;
    SolveCfg inner;
    hipStream_t s;
    Prof *prof;
    SolveHook *hook;   // runs the inner solves when set
    int overlap;       // block overlap of the inner solves' hierarchy
    int solves = 0, vcycles = 0;

    // One inner solve on this thread, or through the hook. x: a workspace
    // buffer, which on this thread may trade places with the hierarchy's
    // second iterate buffer instead of receiving a copy.
    int32_t inner_solve(const double *data, const double *src, double *&x, bool warm, const SolveCfg &c,
                        hdi_solve_report &rep) {
        if (hook) return hook->solve(t.h, overlap, W, H, C, mask, data, src, x, warm, c, &rep, s);
        // the inner solves' own device times are not reported, so the host
        // goes on queueing as soon as the last convergence test is read
        SolveCfg cu = c;
        cu.untimed = true;
        return solve_system<double>(t.h, W, H, C, mask, data, src, x, warm, cu, &rep, s, prof, &x);
    }

    // u = B x for x given on K (compact); cold start with FMG unless warm.
    int32_t apply_B(const double *xK, double *&u, bool warm, double tol) {
        launch_scatter_K(m, C, N, t.idx, xK, t.img_d, s);
        SolveCfg c = inner;
        c.rel_tol = tol;
        hdi_solve_report rep;
        int32_t st = inner_solve(t.img_d, nullptr, u, warm, c, rep);
        if (st) set_error("inner B solve (tol %.1e, warm %d): %s", tol, (int)warm, hdi_last_error());
        ++solves;
        vcycles += (c.flags & HDI_FLAG_CG) ? rep.outer_iters : rep.vcycles;
        return st;
    }
    // out = B^T y for an image y (whose K part is read from y, or from yK if
    // y is null): w solves L_UU w = y_U (source problem, zero data), in the
    // buffer w (warm-started from its contents when warm).
    int32_t apply_Bt(const double *y, const double *yK, const double *ysrc, double *out, bool warm, double tol,
                     double *&w) {
        SolveCfg c = inner;
        c.rel_tol = tol;
        hdi_solve_report rep;
        int32_t st = inner_solve(nullptr, ysrc, w, warm, c, rep);
        if (st) set_error("inner B^T solve (tol %.1e, warm %d): %s", tol, (int)warm, hdi_last_error());
        ++solves;
        vcycles += (c.flags & HDI_FLAG_CG) ? rep.outer_iters : rep.vcycles;
        launch_gather_Bt(W, H, m, C, t.idx, mask, y, yK, w, out, s);
        return st;
    }
    // rho = f - u, returns sum of squares per channel
    int32_t image_residual(double *ss, const double *u) {
        launch_image_residual(N, C, f, u, t.rho, t.partials, t.sums, s);
        T_TRY(read_to_host(ss, t.sums, sizeof(double) * C, s));
        return HDI_OK;
    }
    int32_t dots(int np, const double *const *a, const double *const *b, double out[4][3]) {
        launch_dots(m, C, np, a, b, t.partials, t.sums, s);
        double tmp[12];
        T_TRY(read_to_host(tmp, t.sums, sizeof(double) * 3 * np, s));
        for (int q = 0; q < np; ++q)
            for (int c = 0; c < 3; ++c) out[q][c] = c < C ? tmp[q * 3 + c] : 0.0;
        return HDI_OK;
    }
    int32_t norms(const double *v, double *out) {
        const double *a[1] = {v};
        double d[4][3];
        T_ST(dots(1, a, a, d));
        for (int c = 0; c < C; ++c) out[c] = std::sqrt(d[0][c]);
        return HDI_OK;
    }
    // r = B^T (f - B g) into rK; B g goes to ug and L_UU^{-1} rho_U to wr,
    // whose contents are the starting guesses when warm. Returns the
    // per-channel squared error sum.
    int32_t normal_residual(bool warm, double tol, double *sse) {
        T_ST(apply_B(t.gK, t.ug, warm, tol));
        T_ST(image_residual(sse, t.ug));
        return apply_Bt(t.rho, nullptr, t.rho, t.rK, warm, tol, t.wr);
    }
};

__global__ void k_image_from_K(int N, int C, int m, const int *__restrict__ pos, const double *__restrict__ vK,
                               double *__restrict__ img) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int j = pos[i];
    for (int c = 0; c < C; ++c) img[(size_t)c * N + i] = j >= 0 ? vK[(size_t)c * m + j] : 0.0;
}

__global__ void k_gather_d(int m, int C, int N, const int *__restrict__ idx, const double *__restrict__ img,
                           double *__restrict__ v) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    for (int c = 0; c < C; ++c) v[(size_t)c * m + j] = img[(size_t)c * N + idx[j]];
}

// Loosest tolerance of an inner solve inside a Krylov product. Late outer
// iterations reach it: from 1e-3 to 3e-2, a loose product takes one V-cycle
// fewer (4K RGB, 3% mask: 47 -> 43 V-cycles per call at the same 6 outer
// iterations; the final residual is certified with tight solves either way).
constexpr double KRYLOV_TOL_CAP = 3e-2;

static int32_t run_tonal(TonalCtx &X, const TonalCfg &tc, double *g_out, double *u_out, hdi_tonal_report *rep) {
    TonalWs &t = X.t;
    const int C = X.C, m = X.m;
    hipStream_t s = X.s;
    const double tight = std::min(1e-9, 1e-3 * tc.rel_tol);

    // ||B^T f|| (the scale of the relative normal residual)
    double bnorm[3], sse[3], r0[3], rel[3] = {0, 0, 0};
    // (it only sets the scale of the stopping test, so a loose solve suffices)
    launch_image_residual(X.N, C, X.f, nullptr, t.rho, t.partials, t.sums, s);   // rho = f
    T_ST(X.apply_Bt(t.rho, nullptr, t.rho, t.bK, false, 1e-4, t.wA));
    T_ST(X.norms(t.bK, bnorm));

    // initial residual r = B^T (f - B g); errors here are corrected by the
    // final true-residual check (solving it tighter than rel_tol bought no
    // iterations in measurements)
    T_ST(X.normal_residual(false, std::max(tight, tc.rel_tol), sse));
    double mse0 = 0.0;
    for (int c = 0; c < C; ++c) mse0 += sse[c];
    mse0 /= (double)C * X.N;
    T_ST(X.norms(t.rK, r0));
    double rnorm[3];
    for (int c = 0; c < C; ++c) {
        rnorm[c] = r0[c];
        rel[c] = bnorm[c] > 0 ? r0[c] / bnorm[c] : r0[c];
    }
    auto worst = [&]() {
        double w = 0;
        for (int c = 0; c < C; ++c) w = std::max(w, rel[c]);
        return w;
    };

    int it = 0, restarts = 0, fallbacks = 0, tightenings = 0;
    // inexact-Krylov factor of the inner tolerances; tightened when the outer
    // residual stalls (the products' errors then limit what the recurrence
    // can reach, which happens for sparse masks, where A^{-1} is large).
    // Krylov products are relaxed as 1e-1 * rel_tol / ||r||_rel (against 3e-2,
    // fewer V-cycles at the same outer iteration counts on most masks; on a
    // sparse 1% mask one more outer iteration), at most KRYLOV_TOL_CAP;
    // the stationary RAS residual evaluation keeps 1e-3.
    double fac = tc.mode == HDI_TONAL_RAS ? 1e-3 : 1e-1, best = 1e300;
    int stall = 0;
    // stationary RAS step length: halved whenever the residual grows (with
    // 32x32 blocks on sparse masks the undamped iteration can diverge)
    double omega = 1.0, prev_worst = worst(), best_ever = worst();
    bool done = worst() <= tc.rel_tol;
    int32_t status = HDI_OK;
    double pq_prev[3] = {1, 1, 1};
    bool first = true;
    double mse_prev = mse0;
    bool mse_stop = false;
    while (!done) {
        if (it >= tc.max_outer) {
            status = HDI_ERR_NO_CONVERGENCE;
            set_error("tonal: relative normal residual %.3e above %.3e after %d iterations", worst(), tc.rel_tol, it);
            break;
        }
        double rmin = 1e300;
        for (int c = 0; c < C; ++c) rmin = std::min(rmin, rel[c] > 0 ? rel[c] : 1e300);
        // Krylov modes: a product with a search direction may be relaxed as the
        // outer residual falls (inexact Krylov). The stationary RAS iteration
        // instead evaluates the residual itself, which must stay accurate
        // relative to its own size, so its warm-started solves tighten with it.
        const double tol_in =
            tc.mode == HDI_TONAL_RAS
                ? std::min(1e-4, std::max(tight, fac * rmin))
                : std::min(KRYLOV_TOL_CAP, std::max(tight, fac * tc.rel_tol / std::max(rmin, 1e-300)));

        const Blocks1D tbx = make_blocks(X.W, tc.overlap, tc.block), tby = make_blocks(X.H, tc.overlap, tc.block);
        const double block_px = (double)std::min(tc.block, X.W) * std::min(tc.block, X.H);
        const double ras_bytes = (double)X.N * 5.0 + 16.0 * C * m;   // mask + pos, r in, z out
        auto ras_sweep = [&]() -> int32_t {
            if (!X.prof) {
                launch_ras_local(X.W, X.H, C, m, tc.block, tc.overlap, tc.local_outer, tc.local_inner, X.mask, t.pos, t.rK,
                                 t.zK, nullptr, s);
                return HDI_OK;
            }
            // timed: the FLOPs are those of the local steps actually taken (a
            // local CG stops early at its FP32 residual floor): 15 per block
            // pixel and local CG step, 20 per block pixel and local CGNR step
            X.prof->begin(6, ras_bytes, s, 0.0);
            launch_ras_local(X.W, X.H, C, m, tc.block, tc.overlap, tc.local_outer, tc.local_inner, X.mask, t.pos, t.rK,
                             t.zK,
                             t.ras_steps, s);
            X.prof->end(s);
            launch_sum_steps(tbx.count * tby.count * C, t.ras_steps, t.ras_totals, s);
            unsigned long long tot[2] = {0, 0};
            T_TRY(read_to_host(tot, t.ras_totals, sizeof tot, s));
            // LDS bytes, every lane of a TB x TB tile issuing the tile's LDS
            // operations: per pixel and local CG step the direction written to
            // the tile (4) and the halo of the lane's 4x4 read back (4), plus
            // the four wavefront slots read per block sum (1 each, two sums, 64
            // blocks only); per pixel and local CGNR step two such exchanges,
            // t parked and read back (8) and four block sums; once per block
            // the zeroed tile and the first sum. (The slot writes, one lane per
            // wavefront, are left out.)
            const double tpx = (double)tc.block * tc.block, sb = tc.block == 64 ? 1.0 : 0.0;
            const double nblk = (double)tbx.count * tby.count * C;
            const double lds = nblk * ((tc.block + 2.0) * (tc.block + 8.0) * 4.0 + sb * tpx) +
                               tpx * ((8.0 + 2.0 * sb) * (double)tot[0] + (24.0 + 4.0 * sb) * (double)tot[1]);
            X.prof->set_last(block_px * (15.0 * (double)tot[0] + 20.0 * (double)tot[1]), lds);
            return HDI_OK;
        };
        if (tc.mode == HDI_TONAL_RAS) {
            // Alg. 2: local corrections, then the global residual with warm starts
            T_ST(ras_sweep());
            const double one[3] = {1, 1, 1}, om[3] = {omega, omega, omega};
            // with the MSE stop, keep the iterate before the step (uB is free in
            // this mode): a step that raises the MSE is undone
            if (tc.mse_gain > 0.0) T_TRY(hipMemcpyAsync(t.uB, t.gK, sizeof(double) * C * m, hipMemcpyDeviceToDevice, s));
            launch_axpby(m, C, om, one, t.zK, t.gK, s);
            ++it;
            T_ST(X.normal_residual(true, tol_in, sse));
            T_ST(X.norms(t.rK, rnorm));
            for (int c = 0; c < C; ++c) rel[c] = bnorm[c] > 0 ? rnorm[c] / bnorm[c] : rnorm[c];
            if (worst() > prev_worst) omega = std::max(omega * 0.5, 1.0 / 64);
            prev_worst = worst();
            best_ever = std::min(best_ever, worst());
            // (with the MSE stop, a step that raises the MSE ends the run instead)
            if (tc.mse_gain <= 0.0 && (worst() > 10.0 * best_ever || (omega <= 1.0 / 64 && worst() > 1.05 * best_ever))) {
                status = HDI_ERR_NO_CONVERGENCE;
                set_error("tonal: stationary RAS diverges on this mask (relative normal residual %.3e); "
                          "the flexible-CG mode converges", worst());
                break;
            }
        } else {
            // flexible CG (Notay's FCG with one stored direction)
            const double *z = t.rK;
            if (tc.mode == HDI_TONAL_PCG_RAS) {
                T_ST(ras_sweep());
                z = t.zK;
            }
            double beta[3] = {0, 0, 0};
            {
                // one reduction: <z, r> and <z, z> for the descent test, and
                // <z, q_prev> for the FCG coefficient
                const double *a[3] = {z, z, z}, *b[3] = {t.rK, z, t.qprev};
                double d[4][3];
                T_ST(X.dots(first ? 2 : 3, a, b, d));
                bool descent = true;
                for (int c = 0; c < C; ++c)
                    if (rel[c] > 0.5 * tc.rel_tol && !(d[0][c] > 1e-3 * std::sqrt(d[1][c]) * rnorm[c])) descent = false;
                if (!descent) {
                    // the preconditioned direction is (nearly) orthogonal to the
                    // residual: take the plain normal-equation residual this step
                    z = t.rK;
                    ++fallbacks;
                    if (!first) {
                        const double *a1[1] = {z}, *b1[1] = {t.qprev};
                        T_ST(X.dots(1, a1, b1, d));
                        for (int c = 0; c < C; ++c) d[2][c] = d[0][c];
                    }
                }
                if (!first)
                    for (int c = 0; c < C; ++c) beta[c] = d[2][c] / pq_prev[c];
            }
            const double one[3] = {1, 1, 1};
            double nb[3];
            for (int c = 0; c < 3; ++c) nb[c] = -beta[c];
            if (first) {
                const double zero[3] = {0, 0, 0};
                launch_axpby(m, C, one, zero, z, t.pK, s);
            } else {
                launch_axpby(m, C, one, nb, z, t.pK, s);
            }
            // q = B^T B p
            T_ST(X.apply_B(t.pK, t.uB, false, tol_in));
            T_ST(X.apply_Bt(nullptr, t.pK, t.uB, t.qK, false, tol_in, t.wA));
            const double *a2[2] = {t.pK, t.pK}, *b2[2] = {t.rK, t.qK};
            double d[4][3];
            T_ST(X.dots(2, a2, b2, d));
            double alpha[3] = {0, 0, 0}, nalpha[3] = {0, 0, 0};
            for (int c = 0; c < C; ++c) {
                const bool active = rel[c] > 0.5 * tc.rel_tol && d[1][c] > 0;
                alpha[c] = active ? d[0][c] / d[1][c] : 0.0;
                nalpha[c] = -alpha[c];
                pq_prev[c] = d[1][c] > 0 ? d[1][c] : 1.0;
            }
            launch_axpby(m, C, alpha, one, t.pK, t.gK, s);
            launch_axpby(m, C, nalpha, one, t.qK, t.rK, s);
            // running B g and L_UU^{-1} rho_U (linear in g): warm starts for the
            // true-residual solves
            launch_axpby(X.N, C, alpha, one, t.uB, t.ug, s);
            launch_axpby(X.N, C, nalpha, one, t.wA, t.wr, s);
            std::swap(t.qK, t.qprev);
            first = false;
            ++it;
            T_ST(X.norms(t.rK, rnorm));
            for (int c = 0; c < C; ++c) rel[c] = bnorm[c] > 0 ? rnorm[c] / bnorm[c] : rnorm[c];
        }
        if (tc.mse_gain > 0.0) {
            // relative MSE improvement of this iteration (Sec. 5.1): the
            // evaluated error for stationary RAS, the running B g otherwise
            double ss[3] = {0, 0, 0};
            if (tc.mode == HDI_TONAL_RAS)
                for (int c = 0; c < C; ++c) ss[c] = sse[c];
            else
                T_ST(X.image_residual(ss, t.ug));
            double mse_now = 0.0;
            for (int c = 0; c < C; ++c) mse_now += ss[c];
            mse_now /= (double)C * X.N;
            if (mse_prev - mse_now < tc.mse_gain * mse_prev) {
                if (tc.mode == HDI_TONAL_RAS && mse_now > mse_prev)
                    T_TRY(hipMemcpyAsync(t.gK, t.uB, sizeof(double) * C * m, hipMemcpyDeviceToDevice, s));
                mse_stop = true;
                break;
            }
            mse_prev = mse_now;
        }
        if (tc.flags & HDI_TONAL_TRACE)
            fprintf(stderr, "[hdi tonal] it %d mode %d rel %.3e tol_in %.1e solves %d vcycles %d fallbacks %d\n", it,
                    tc.mode, worst(), tol_in, X.solves, X.vcycles, fallbacks);
        if (worst() < 0.95 * best) {
            best = worst();
            stall = 0;
        } else if (tc.mode != HDI_TONAL_RAS && ++stall >= 3 && tightenings < 3 && worst() > tc.rel_tol) {
            // stalled: tighten the inner solves and restart from the true residual
            fac *= 1e-2;
            ++tightenings;
            stall = 0;
            T_ST(X.normal_residual(true, tight, sse));
            T_ST(X.norms(t.rK, rnorm));
            for (int c = 0; c < C; ++c) rel[c] = bnorm[c] > 0 ? rnorm[c] / bnorm[c] : rnorm[c];
            best = worst();
            first = true;
            done = worst() <= tc.rel_tol;
            continue;
        }
        if (worst() <= 0.8 * tc.rel_tol || (tc.mode == HDI_TONAL_RAS && worst() <= tc.rel_tol)) {
            // true normal residual with tight solves, warm-started from the
            // running estimates
            T_ST(X.normal_residual(true, tight, sse));
            T_ST(X.norms(t.rK, rnorm));
            for (int c = 0; c < C; ++c) rel[c] = bnorm[c] > 0 ? rnorm[c] / bnorm[c] : rnorm[c];
            if (worst() <= tc.rel_tol) {
                done = true;
            } else {
                first = true;   // restart the recurrences from the true residual
                if (++restarts > 20) {
                    status = HDI_ERR_NO_CONVERGENCE;
                    set_error("tonal: true residual %.3e stays above %.3e", worst(), tc.rel_tol);
                    break;
                }
            }
        }
    }
    if (status != HDI_OK || it == 0 || mse_stop) {
        // the final state still needs B g and its error for the report
        T_ST(X.normal_residual(it > 0, tight, sse));
        T_ST(X.norms(t.rK, rnorm));
        for (int c = 0; c < C; ++c) rel[c] = bnorm[c] > 0 ? rnorm[c] / bnorm[c] : rnorm[c];
    }
    double mse1 = 0.0;
    for (int c = 0; c < C; ++c) mse1 += sse[c];
    mse1 /= (double)C * X.N;

    hipLaunchKernelGGL(k_image_from_K, dim3((X.N + 255) / 256), dim3(256), 0, s, X.N, C, m, t.pos, t.gK, g_out);
    if (u_out) T_TRY(hipMemcpyAsync(u_out, t.ug, sizeof(double) * C * X.N, hipMemcpyDeviceToDevice, s));
    T_TRY(hipGetLastError());
    T_TRY(wait_for(s));
    if (rep) {
        rep->mse_initial = mse0;
        rep->mse_final = mse1;
        rep->rel_normal_residual = worst();
        rep->outer_iters = it;
        rep->inner_solves = X.solves;
        rep->inner_vcycles = X.vcycles;
    }
    return status;
}

}  // namespace hdi

using namespace hdi;

extern "C" {

size_t hdi_tonal_workspace_bytes(hdi_image img) {
    if (img.width < 1 || img.height < 1 || (img.channels != 1 && img.channels != 3)) return 0;
    return tonal_ws_bytes(img.width, img.height, img.channels);
}

int32_t tonal_optimize(hdi_image img, const uint8_t *mask, const float *f, double *g, double *u, void *ws,
                       size_t ws_bytes, const hdi_tonal_params *params, hdi_tonal_report *report, void *stream) {
    return tonal_optimize_hooked(img, mask, f, g, u, ws, ws_bytes, params, report, stream, nullptr);
}

}  // extern "C"

namespace hdi {

int32_t fill_tonal_cfg(const hdi_tonal_params *params, TonalCfg &tc, SolveCfg &inner, int &ov_inner) {
    tc.rel_tol = (params && params->rel_tol > 0) ? params->rel_tol : 1e-6;
    tc.max_outer = (params && params->max_outer > 0) ? params->max_outer : 500;
    tc.mode = params ? params->mode : HDI_TONAL_PCG_RAS;
    tc.block = (params && params->block > 0) ? params->block : 64;
    tc.overlap = (params && params->overlap > 0) ? params->overlap : (tc.block == 64 ? 16 : 14);
    tc.local_outer = (params && params->local_outer > 0) ? params->local_outer : (tc.block == 64 ? 5 : 3);
    tc.local_inner = (params && params->local_inner > 0) ? params->local_inner : (tc.block == 64 ? 20 : 24);
    tc.flags = params ? params->flags : 0;
    tc.mse_gain = params ? params->mse_gain : 0.0;
    if (tc.mode < 0 || tc.mode > 2 || !(tc.rel_tol < 1.0) || !(tc.mse_gain >= 0.0 && tc.mse_gain < 1.0) ||
        (tc.block != 32 && tc.block != 64) || tc.overlap < 2 || tc.overlap > tc.block / 2 || (tc.overlap & 1) ||
        tc.local_outer > 64 || tc.local_inner > 256) {
        set_error("tonal parameter out of range (mode 0..2, rel_tol < 1, 0 <= mse_gain < 1, block 32 or 64, "
                  "even overlap 2..block/2)");
        return HDI_ERR_ARG;
    }
    return fill_cfg(params ? &params->inner : nullptr, inner, ov_inner);
}

int32_t tonal_optimize_hooked(hdi_image img, const uint8_t *mask, const float *f, double *g, double *u, void *ws,
                              size_t ws_bytes, const hdi_tonal_params *params, hdi_tonal_report *report, void *stream,
                              SolveHook *hook) {
    if (!check_image(img)) return HDI_ERR_ARG;
    if (!mask || !f || !g) {
        set_error("mask, f and g must be non-null device pointers");
        return HDI_ERR_ARG;
    }
    TonalCfg tc;
    SolveCfg inner;
    int ov_inner;
    int32_t st = fill_tonal_cfg(params, tc, inner, ov_inner);
    if (st) return st;
    if (hook && (inner.flags & HDI_FLAG_CG)) {
        set_error("inner solves by the batch engine run the multigrid solver only (HDI_FLAG_CG is for single solves)");
        return HDI_ERR_ARG;
    }
    const size_t need = tonal_ws_bytes(img.width, img.height, img.channels);
    if (!ws || ws_bytes < need) {
        set_error("workspace of %zu bytes given, %zu needed", ws ? ws_bytes : (size_t)0, need);
        return HDI_ERR_WORKSPACE;
    }
    hipStream_t s = (hipStream_t)stream;
    CallTimer tm;
    T_TRY(tm.start(s));
    Arena a{(char *)ws, ws_bytes, 0};
    TonalWs t;
    plan_tonal(t, a, img.width, img.height, img.channels, ov_inner, mask, inner.small_from);
    st = prepare_mask(t.h, s);
    if (st) return st;
    const int N = img.width * img.height, C = img.channels;
    launch_compact(N, mask, t.chunk_cnt, t.chunk_off, t.total, t.idx, t.pos, s);
    int m = 0;
    T_TRY(read_to_host(&m, t.total, sizeof(int), s));
    if (tc.flags & HDI_TONAL_INIT_FROM_F)
        launch_gather_f(m, C, N, t.idx, f, t.gK, s);
    else
        hipLaunchKernelGGL(k_gather_d, dim3((m + 255) / 256), dim3(256), 0, s, m, C, N, t.idx, g, t.gK);
    // the scatter buffer for products with B holds finite values everywhere
    hipLaunchKernelGGL(k_image_from_K, dim3((N + 255) / 256), dim3(256), 0, s, N, C, m, t.pos, t.gK, t.img_d);
    T_TRY(hipGetLastError());
    inner.known = t.h.known[0];
    Prof *prof = prof_for_call();
    TonalCtx X{t, img.width, img.height, C, N, m, mask, f, inner, s, prof, hook, ov_inner};
    st = run_tonal(X, tc, g, u, report);
    if (prof) {
        prof->flush();
        delete prof;
    }
    float ms = 0.f;
    T_TRY(tm.stop(s, &ms));
    if (report) report->ms = ms;
    return st;
}

}  // namespace hdi
