// Host driver of the inpainting solve and the C-ABI entry points.
//
// Solve of eq. (inp-discrete-lsi) (Sec. 2.1): an FP64 iterative refinement
// around an FP32 multigrid V-cycle whose smoother is the restricted additive
// Schwarz step on overlapping 32x32 blocks with local conjugate gradients
// (Sec. 3.1-3.3). Cold starts use the reduced full multigrid of Sec. 3.2:
// solve on the coarsest level (a single block), then prolongate and apply one
// smoothing step per finer level.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <vector>

#include "hdi_internal.h"

namespace hdi {

// ------------------------------------------------------------------ kernel timing

struct KStats { int64_t launches; double ms, bytes, flops, lds; };
static std::mutex g_stats_mu;
static KStats g_stats[HDI_NUM_KERNEL_IDS];
static std::atomic<int> g_stats_on{0};

void Prof::begin(int id, double bytes, hipStream_t s, double flops) {
    pending = false;
    ended = false;
    if (!on || n >= (int)(sizeof recs / sizeof recs[0])) return;
    Rec &r = recs[n];
    r.id = id;
    r.bytes = bytes;
    r.flops = flops;
    r.lds = 0.0;
    if (hipEventCreate(&r.a) != hipSuccess) return;
    if (hipEventCreate(&r.b) != hipSuccess) {
        (void)hipEventDestroy(r.a);
        return;
    }
    (void)hipEventRecord(r.a, s);
    pending = true;
}
void Prof::end(hipStream_t s) {
    if (!pending) return;   // timing off, full, or the events could not be made
    (void)hipEventRecord(recs[n].b, s);
    ++n;
    pending = false;
    ended = true;
}
void Prof::flush() {
    std::lock_guard<std::mutex> lk(g_stats_mu);
    for (int i = 0; i < n; ++i) {
        float ms = 0.f;
        if (recs[i].id >= 0 && hipEventSynchronize(recs[i].b) == hipSuccess &&
            hipEventElapsedTime(&ms, recs[i].a, recs[i].b) == hipSuccess) {
            g_stats[recs[i].id].launches += 1;
            g_stats[recs[i].id].ms += ms;
            g_stats[recs[i].id].bytes += recs[i].bytes;
            g_stats[recs[i].id].flops += recs[i].flops;
            g_stats[recs[i].id].lds += recs[i].lds;
        }
        (void)hipEventDestroy(recs[i].a);
        (void)hipEventDestroy(recs[i].b);
    }
    n = 0;
    ended = false;
}
// pinned staging for read_to_host: one buffer per host thread, kept for the
// life of the process (freeing it at thread exit could run after the HIP
// runtime has shut down)
constexpr size_t STAGING_BYTES = 16384;
static thread_local void *t_staging = nullptr;
static thread_local bool t_staging_failed = false;

hipError_t wait_for(hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        const hipError_t e = hipStreamQuery(s);
        if (e != hipErrorNotReady) return e;
        if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(5)) return hipStreamSynchronize(s);
    }
}

hipError_t wait_for(hipEvent_t ev) {
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        const hipError_t e = hipEventQuery(ev);
        if (e != hipErrorNotReady) return e;
        if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(5)) return hipEventSynchronize(ev);
    }
}

static thread_local int t_no_alloc = 0;
NoAllocScope::NoAllocScope() { ++t_no_alloc; }
NoAllocScope::~NoAllocScope() { --t_no_alloc; }
bool no_alloc_active() { return t_no_alloc > 0; }

static void *staging(size_t bytes) {
    if (bytes > STAGING_BYTES) return nullptr;
    if (!t_staging && !t_staging_failed && !no_alloc_active()) {
        if (hipHostMalloc(&t_staging, STAGING_BYTES, hipHostMallocPortable) != hipSuccess) {
            t_staging = nullptr;
            t_staging_failed = true;
            (void)hipGetLastError();
        }
    }
    return t_staging;
}

hipError_t read_to_host(void *dst, const void *src, size_t bytes, hipStream_t s) {
    if (staging(bytes)) {
        hipError_t e = hipMemcpyAsync(t_staging, src, bytes, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = wait_for(s);
        if (e == hipSuccess) std::memcpy(dst, t_staging, bytes);
        return e;
    }
    const hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s);
    return e == hipSuccess ? wait_for(s) : e;
}

// The event behind the last read_begin of this host thread (made once, kept
// for the life of the process like the staging buffer).
static thread_local hipEvent_t t_read_ev = nullptr;
static thread_local bool t_read_ev_failed = false;

// Queues a copy of `bytes` from device memory into the thread's pinned staging
// buffer and an event behind it. read_end then waits for that event only, so
// work queued on s after read_begin keeps the device busy while the host
// waits. Returns false with nothing queued when the staging buffer or the
// event is unavailable (use read_to_host then); err reports a failed queueing.
static bool read_begin(const void *src, size_t bytes, hipStream_t s, hipError_t &err) {
    err = hipSuccess;
    if (!staging(bytes)) return false;
    if (!t_read_ev && !t_read_ev_failed && !no_alloc_active()) {
        if (hipEventCreateWithFlags(&t_read_ev, hipEventDisableTiming) != hipSuccess) {
            t_read_ev = nullptr;
            t_read_ev_failed = true;
            (void)hipGetLastError();
        }
    }
    if (!t_read_ev) return false;
    err = hipMemcpyAsync(t_staging, src, bytes, hipMemcpyDeviceToHost, s);
    if (err == hipSuccess) err = hipEventRecord(t_read_ev, s);
    return err == hipSuccess;
}

static hipError_t read_end(void *dst, size_t bytes) {
    const hipError_t e = wait_for(t_read_ev);
    if (e == hipSuccess) std::memcpy(dst, t_staging, bytes);
    return e;
}

Prof *prof_for_call() {
    if (!g_stats_on.load() || no_alloc_active()) return nullptr;
    Prof *p = new Prof;
    p->on = true;
    return p;
}

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) {                                                                \
            set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
            return HDI_ERR_HIP;                                                                \
        }                                                                                      \
    } while (0)

bool plan_hierarchy(Hierarchy &h, Arena &a, int W, int H, int C, int overlap, const uint8_t *mask0,
                    int small_from) {
    h.C = C;
    // small buffers first, so that the large ones form one region the CG
    // vectors can alias
    h.counts = (unsigned int *)a.take(MAX_LEVELS * sizeof(unsigned int));
    const dim3 g = residual_grid(W, H);
    h.nblk = (int)(g.x * g.y);
    h.partials = (double *)a.take((size_t)C * h.nblk * 2 * sizeof(double));
    h.norms = (double *)a.take((size_t)C * 2 * sizeof(double));
    h.cg_part = (double *)a.take((size_t)C * CG_BLOCKS * 2 * sizeof(double));
    h.cg_scal = (double *)a.take(64 * sizeof(double));
    const size_t big0 = (a.used + 255) & ~(size_t)255;
    int l = 0;
    int w = W, hh = H;
    for (;;) {
        Level &L = h.lev[l];
        L.W = w;
        L.H = hh;
        if (small_from == 0 && l >= 1) {
            // automatic: switch once a level has too few 32x32 blocks to keep
            // the chip busy (about 4 waves per SIMD), and stay switched
            const long nb = (long)make_blocks(w, overlap).count * make_blocks(hh, overlap).count * C;
            if (nb < 4096) small_from = l;
        }
        const bool small = small_from > 0 && l >= small_from;
        L.tile = small ? TILE_SMALL : TILE;
        // the coarse levels smooth with half the overlap (even, at least 2):
        // their blocks only need to pass the correction on, and the coarse-grid
        // correction below does what more overlap would
        const int ov = l >= 1 ? coarse_overlap(overlap) : overlap;
        L.bx = make_blocks(w, ov, L.tile);
        L.by = make_blocks(hh, ov, L.tile);
        const size_t n = (size_t)w * hh;
        L.mask = l == 0 ? const_cast<uint8_t *>(mask0) : (uint8_t *)a.take(n);
        L.r = (float *)a.take(n * C * sizeof(float));
        L.ea = (float *)a.take(n * C * sizeof(float));
        L.eb = (float *)a.take(n * C * sizeof(float));
        L.aux = l == 0 ? nullptr : (float *)a.take(n * C * sizeof(float));
        ++l;
        if ((w <= TILE && hh <= TILE) || l == MAX_LEVELS) break;
        w = (w + 1) / 2;
        hh = (hh + 1) / 2;
    }
    h.nlev = h.nlev_full = l;
    h.u_alt = (double *)a.take((size_t)W * H * C * sizeof(double));
    // CG vectors over the same region (extended where small images leave it short)
    const size_t vec = ((size_t)W * H * C * sizeof(double) + 255) & ~(size_t)255;
    if (a.used < big0 + 3 * vec) a.take(big0 + 3 * vec - a.used);
    auto at = [&](int k) { return a.base ? (double *)(a.base + big0 + k * vec) : nullptr; };
    h.cg_r = at(0);
    h.cg_p[0] = at(1);
    h.cg_p[1] = at(2);
    return a.base == nullptr || a.used <= a.size;
}

// Algorithmic bytes and FLOPs of a V-cycle from level l down, with the
// per-launch counts of the finest level applied to every level: pre-smoothing
// N(1 + 8C) bytes, residual restriction N(1 + 8C) + Nc(1 + 4C), post-smoothing
// N(1 + 12C) + 4C Nc, the coarsest level's smoothing N(1 + 8C); 15 FLOPs per
// block pixel and local CG step.
static void vcycle_cost(const Hierarchy &h, int l, const SolveCfg &cfg, double &bytes, double &flops) {
    bytes = flops = 0.0;
    const int C = h.C;
    for (int k = l; k < h.nlev; ++k) {
        const Level &L = h.lev[k];
        const double N = (double)L.W * L.H;
        const double blk_px = (double)L.bx.count * L.by.count * std::min(L.tile, L.W) * std::min(L.tile, L.H) * C;
        if (k == h.nlev - 1) {
            bytes += N * (1 + 8.0 * C);
            flops += 15.0 * blk_px * cfg.coarse_iters;
        } else {
            const double Nc = (double)h.lev[k + 1].W * h.lev[k + 1].H;
            bytes += 2.0 * N * (1 + 8.0 * C) + Nc * (1 + 4.0 * C) + N * (1 + 12.0 * C) + 4.0 * C * Nc;
            flops += 2.0 * 15.0 * blk_px * (k == 0 ? cfg.local_iters : cfg.mid_iters);
        }
    }
}

// The pre-smoothing launch of a V-cycle on level l < nlev - 1. guard >= 0 (level
// 0 only): the launch is queued before the host has seen the residual norms
// in h.norms, and its blocks return at once when those norms already meet
// the relative tolerance guard.
static void smooth_pre(Hierarchy &h, int l, const SolveCfg &cfg, hipStream_t s, Prof *prof, double guard = -1.0) {
    Level &L = h.lev[l];
    const int C = h.C;
    const double N = (double)L.W * L.H;
    const double blk_px = (double)L.bx.count * L.by.count * std::min(L.tile, L.W) * std::min(L.tile, L.H) * C;
    const int iters = l == 0 ? cfg.local_iters : cfg.mid_iters;
    if (prof) prof->begin(1, N * (1 + 8.0 * C), s, 15.0 * blk_px * iters);
    // the global-relative local stop on the finest level, against the norms
    // of the residual sweep that precedes the V-cycle
    const double *gnorm = l == 0 ? h.norms : nullptr;
    launch_smooth_pre(L, C, iters, cfg.robin, gnorm, cfg.local_stop, L.ea, s, guard);
    if (prof) prof->end(s);
}

// One V-cycle for A e = r on level l (r in lev[l].r); returns the buffer with e.
// pre_queued: smooth_pre of level l is already on the stream. With `prof`, the
// finest level's launches are timed one by one and the whole coarse recursion
// as one record.
static float *vcycle(Hierarchy &h, int l, const SolveCfg &cfg, hipStream_t s, Prof *prof = nullptr,
                     bool pre_queued = false) {
    Level &L = h.lev[l];
    const int C = h.C;
    if (l == h.nlev - 1) {
        launch_smooth_pre(L, C, cfg.coarse_iters, cfg.robin, nullptr, 0.f, L.ea, s);
        return L.ea;
    }
    Level &Lc = h.lev[l + 1];
    const double N = (double)L.W * L.H, Nc = (double)Lc.W * Lc.H;
    const double blk_px = (double)L.bx.count * L.by.count * std::min(L.tile, L.W) * std::min(L.tile, L.H) * C;
    const int iters = l == 0 ? cfg.local_iters : cfg.mid_iters;
    const double cg_flops = 15.0 * blk_px * iters;
    const double *gnorm = l == 0 ? h.norms : nullptr;
    if (!pre_queued) smooth_pre(h, l, cfg, s, prof);
    if (prof) prof->begin(3, N * (1 + 8.0 * C) + Nc * (1 + 4.0 * C), s);
    launch_restrict_residual(L, Lc, C, L.ea, s);
    if (prof) {
        prof->end(s);
        double cb = 0.0, cf = 0.0;
        vcycle_cost(h, l + 1, cfg, cb, cf);
        prof->begin(5, cb, s, cf);
    }
    const float *ec = vcycle(h, l + 1, cfg, s);
    if (prof) { prof->end(s); prof->begin(2, N * (1 + 12.0 * C) + 4.0 * C * Nc, s, cg_flops); }
    launch_smooth_post(L, Lc, C, iters, cfg.robin, gnorm, cfg.local_stop, L.ea, ec, L.eb, s);
    if (prof) prof->end(s);
    return L.eb;
}

// Reduced full multigrid initial guess (Sec. 3.2, Fig. multigrid_reduced).
template <typename TD>
static void fmg_init(Hierarchy &h, int W, int H, int C, const uint8_t *mask, const TD *data, double *u,
                     const SolveCfg &cfg, hipStream_t s) {
    launch_data_restrict0<TD>(W, H, C, mask, data, h.lev[1], s);
    for (int l = 2; l < h.nlev; ++l) launch_data_restrict(h.lev[l - 1], h.lev[l], C, s);
    Level &Lc = h.lev[h.nlev - 1];
    launch_smooth_fmg(Lc, C, cfg.coarse_iters, cfg.robin, Lc.aux, Lc.ea, s);
    const float *cur = Lc.ea;
    for (int l = h.nlev - 2; l >= 1; --l) {
        Level &L = h.lev[l];
        launch_fmg_prolong(L, h.lev[l + 1], C, cur, L.eb, s);
        launch_smooth_fmg(L, C, cfg.mid_iters, cfg.robin, L.eb, L.ea, s);
        cur = L.ea;
    }
    launch_fmg_prolong0(W, H, C, mask, h.lev[1], cur, u, s);
}

// Plain FP64 conjugate gradients on the unknown pixels (comparator, Sec. 2.1
// and the GPU baseline of Sec. 6.1). The recursive residual is read back every
// CG_CHECK steps; once it meets the tolerance the true residual is recomputed
// and, if that misses it, CG restarts from it. Returns the status; rounds
// counts CG steps.
constexpr int CG_CHECK = 10;

template <typename TD>
static int32_t solve_cg(Hierarchy &h, int W, int H, int C, const uint8_t *mask, const TD *data, const double *src,
                        double *u, const SolveCfg &cfg, double *rel, int &rounds, hipStream_t s, Prof *prof) {
    const double N = (double)W * H, nU = N - (double)cfg.known;
    const int64_t cap = (int64_t)cfg.max_outer * 1000;
    double sc[3 * 8];
    int cur = 0;
    bool from_true = true;   // the residual in cg_r was just recomputed
    if (prof) prof->begin(0, N * (1 + 16.0 * C) + C * (double)cfg.known * sizeof(TD) + (src ? 8.0 * C * nU : 0.0), s);
    launch_cg_start<TD>(W, H, C, mask, u, data, src, h.cg_r, h.cg_part, h.cg_scal, s);
    if (prof) prof->end(s);
    for (;;) {
        HIP_TRY(hipGetLastError());
        HIP_TRY(read_to_host(sc, h.cg_scal, sizeof(double) * 8 * C, s));
        double worst = 0.0;
        bool finite = true;
        for (int c = 0; c < C; ++c) {
            const double rr = sc[8 * c], bb = sc[8 * c + 1];
            finite = finite && std::isfinite(rr) && std::isfinite(bb);
            rel[c] = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
            worst = std::fmax(worst, rel[c]);
        }
        if (!finite) {
            set_error("non-finite residual: the input holds NaN/Inf or the iteration diverged");
            return HDI_ERR_ARG;
        }
        if (worst <= cfg.rel_tol) {
            if (from_true) return HDI_OK;
            launch_cg_start<TD>(W, H, C, mask, u, data, src, h.cg_r, h.cg_part, h.cg_scal, s);
            from_true = true;
            continue;
        }
        if (rounds >= cap) {
            set_error("relative residual %.3e above tolerance %.3e after %d CG steps", worst, cfg.rel_tol, rounds);
            return HDI_ERR_NO_CONVERGENCE;
        }
        // per step and unknown pixel-channel: direction reads r, p and writes p;
        // the update reads p, u, r and writes u, r (8 bytes each), mask twice
        if (prof) prof->begin(4, CG_CHECK * (nU * C * 64.0 + 2.0 * N), s);
        for (int k = 0; k < CG_CHECK && rounds < cap; ++k, ++rounds) {
            launch_cg_iteration(W, H, C, mask, u, h.cg_r, h.cg_p[cur], h.cg_p[cur ^ 1], h.cg_part, h.cg_scal, s);
            cur ^= 1;
        }
        if (prof) prof->end(s);
        from_true = false;
    }
}

template <typename TD>
int32_t solve_system(Hierarchy &h, int W, int H, int C, const uint8_t *mask, const TD *data, const double *src,
                     double *u, bool warm, const SolveCfg &cfg, hdi_solve_report *rep, hipStream_t s, Prof *prof,
                     double **swap) {
    if ((data == nullptr) == (src == nullptr)) {
        set_error("internal: a solve takes either data on the mask or a source off it");
        return HDI_ERR_ARG;
    }
    CallTimer tm;
    if (!cfg.untimed) HIP_TRY(tm.start(s));
    if (cfg.flags & HDI_FLAG_CG) {
        if (h.u_alt_moved) {
            set_error("internal: a CG solve after a multigrid solve handed over its buffer");
            return HDI_ERR_ARG;
        }
        launch_init_u<TD>(W, H, C, mask, data, warm, u, s);
        double rel[3] = {0, 0, 0};
        int steps = 0;
        const int32_t st = solve_cg<TD>(h, W, H, C, mask, data, src, u, cfg, rel, steps, s, prof);
        float ms = 0.f;
        if (!cfg.untimed) HIP_TRY(tm.stop(s, &ms));
        if (prof) prof->flush();
        if (rep) {
            for (int c = 0; c < 3; ++c) rep->rel_residual[c] = c < C ? rel[c] : 0.0;
            rep->outer_iters = steps;
            rep->vcycles = 0;
            rep->ms = ms;
        }
        return st;
    }
    const double N = (double)W * H, nK = (double)cfg.known, nU = N - nK;
    (void)nU;
    if (prof) prof->begin(5, 0.0, s);
    const bool fmg = !warm && !(cfg.flags & HDI_FLAG_NO_FMG) && src == nullptr && h.nlev > 1;
    // A cold source problem starts from u = 0 everywhere: instead of filling u,
    // the first residual pass and the first refinement step take a null
    // iterate (read as zero), and the first step writes the whole iterate.
    bool zero = !warm && src != nullptr;
    if (!zero) launch_init_u<TD>(W, H, C, mask, data, warm || fmg, u, s);
    if (fmg) fmg_init<TD>(h, W, H, C, mask, data, u, cfg, s);
    if (prof) prof->end(s);
    HIP_TRY(hipGetLastError());

    int32_t status = HDI_OK;
    int rounds = 0, vcycles = 0;
    double rel[3] = {0, 0, 0};
    double norms[6];
    // The refinement step u += e is fused into the next residual pass, which
    // reads the iterate with a halo, so the iterate alternates between the
    // caller's u and the workspace copy.
    double *cur = u, *oth = h.u_alt;
    const float *e = nullptr;
    for (;;) {
        // mask, u in, r out; the source off the mask; e in and u out after a
        // V-cycle (the data is not read: u holds it on the mask)
        const double res_bytes = N * (1 + (zero ? 4.0 : 12.0) * C) + (src ? 8.0 * C * nU : 0.0) +
                                 (e ? 12.0 * C * N : 0.0);
        if (prof) prof->begin(0, res_bytes, s);
        launch_residual<TD>(W, H, C, mask, zero ? nullptr : cur, e, e ? oth : nullptr, data, src, h.lev[0].r,
                            h.partials, h.norms, s);
        if (prof) prof->end(s);
        if (e) {
            std::swap(cur, oth);
            zero = false;
        }
        // When a V-cycle may follow, its first launch is queued behind the copy
        // of the norms, guarded on the device by the same test with a margin
        // (so that a guarded exit implies the host's stop below), and the host
        // waits for the copy alone: the device smooths while the host decides.
        bool queued = false;
        if (h.nlev > 1 && rounds < cfg.max_outer) {
            hipError_t err;
            queued = read_begin(h.norms, sizeof(double) * 2 * C, s, err);
            HIP_TRY(err);
            if (queued) {
                smooth_pre(h, 0, cfg, s, prof, cfg.rel_tol * (1.0 - 1e-12));
                HIP_TRY(read_end(norms, sizeof(double) * 2 * C));
            }
        }
        if (!queued) HIP_TRY(read_to_host(norms, h.norms, sizeof(double) * 2 * C, s));
        double worst = 0.0;
        bool finite = true;
        for (int c = 0; c < C; ++c) {
            const double rr = norms[2 * c], bb = norms[2 * c + 1];
            finite = finite && std::isfinite(rr) && std::isfinite(bb);
            rel[c] = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
            worst = std::fmax(worst, rel[c]);
        }
        if (!finite || worst <= cfg.rel_tol) {
            // the queued pre-smoothing returned at once or is left unused
            if (queued && prof) prof->drop_last();
        }
        if (!finite) {
            set_error("non-finite residual: the input holds NaN/Inf or the iteration diverged");
            status = HDI_ERR_ARG;
            break;
        }
        if (worst <= cfg.rel_tol) break;
        if (rounds >= cfg.max_outer) {
            set_error("relative residual %.3e above tolerance %.3e after %d rounds", worst, cfg.rel_tol, rounds);
            status = HDI_ERR_NO_CONVERGENCE;
            break;
        }
        e = vcycle(h, 0, cfg, s, prof, queued);
        ++rounds;
        ++vcycles;
    }
    // stopped before the first refinement step: the zero iterate was never written
    if (zero) launch_init_u<TD>(W, H, C, mask, data, false, u, s);
    if (cur != u) {
        if (swap && *swap == u) {
            *swap = cur;
            h.u_alt = u;
            h.u_alt_moved = true;
        } else {
            HIP_TRY(hipMemcpyAsync(u, cur, sizeof(double) * C * W * H, hipMemcpyDeviceToDevice, s));
        }
    }
    HIP_TRY(hipGetLastError());
    float ms = 0.f;
    if (!cfg.untimed) HIP_TRY(tm.stop(s, &ms));
    if (prof) prof->flush();
    if (rep) {
        for (int c = 0; c < 3; ++c) rep->rel_residual[c] = c < C ? rel[c] : 0.0;
        rep->outer_iters = rounds;
        rep->vcycles = vcycles;
        rep->ms = ms;
    }
    return status;
}

template int32_t solve_system<float>(Hierarchy &, int, int, int, const uint8_t *, const float *, const double *,
                                     double *, bool, const SolveCfg &, hdi_solve_report *, hipStream_t, Prof *,
                                     double **);
template int32_t solve_system<double>(Hierarchy &, int, int, int, const uint8_t *, const double *, const double *,
                                      double *, bool, const SolveCfg &, hdi_solve_report *, hipStream_t, Prof *,
                                      double **);

bool check_image(const hdi_image &img) {
    if (img.width < 1 || img.height < 1 || (img.channels != 1 && img.channels != 3)) {
        set_error("bad image shape %dx%dx%d (need width, height >= 1 and 1 or 3 channels)", img.width, img.height,
                  img.channels);
        return false;
    }
    if ((int64_t)img.width * img.height > (int64_t)1 << 30) {
        set_error("image of %lld pixels exceeds the 2^30 limit", (long long)img.width * img.height);
        return false;
    }
    return true;
}

int32_t fill_cfg(const hdi_solve_params *p, SolveCfg &cfg, int &overlap) {
    cfg.rel_tol = (p && p->rel_tol > 0) ? p->rel_tol : 1e-6;
    cfg.max_outer = (p && p->max_outer > 0) ? p->max_outer : 40;
    cfg.local_iters = (p && p->local_iters > 0) ? p->local_iters : 12;
    cfg.mid_iters = (p && p->mid_iters > 0) ? p->mid_iters : 8;
    cfg.coarse_iters = (p && p->coarse_iters > 0) ? p->coarse_iters : 64;
    cfg.vcycles = 1;
    cfg.flags = p ? p->flags : 0;
    cfg.small_from = p ? p->small_from : 0;
    // Robin weight: 0 selects the default 0.6, a negative value Dirichlet (0)
    cfg.robin = (p && p->robin != 0.f) ? std::max(p->robin, 0.f) : 0.6f;
    cfg.local_stop = p ? p->local_stop : 0.f;
    overlap = (p && p->overlap > 0) ? p->overlap : 6;
    if (cfg.flags & ~(HDI_FLAG_NO_FMG | HDI_FLAG_CG)) {
        set_error("unknown solve flags 0x%x", cfg.flags);
        return HDI_ERR_ARG;
    }
    if (overlap < 2 || overlap > 16 || (overlap & 1)) {
        set_error("overlap %d outside 2..16 or odd", overlap);
        return HDI_ERR_ARG;
    }
    if (!(cfg.rel_tol < 1.0) || cfg.local_iters > 256 || cfg.mid_iters > 256 || cfg.coarse_iters > 4096 ||
        cfg.max_outer > 100000 ||
        cfg.small_from < -1 || cfg.small_from >= MAX_LEVELS || !(cfg.robin >= 0.f && cfg.robin <= 0.9f) ||
        !(cfg.local_stop >= 0.f && cfg.local_stop < 1.f)) {
        set_error("parameter out of range (rel_tol < 1, local_iters and mid_iters <= 256, coarse_iters <= 4096, "
                  "small_from -1..%d, robin 0..0.9, local_stop 0..1)", MAX_LEVELS - 1);
        return HDI_ERR_ARG;
    }
    return HDI_OK;
}

// Coarse masks and per-level known counts for a new mask (one readback). Picks
// the number of levels used: coarsening stops at the first level whose mask is
// at least 99% known (with the "any of four" rule coarse masks fill up fast, and
// a smoothing step with local CG is then an almost exact solve there), and in
// any case at the level that is a single 32x32 block (Sec. 3.3).
int32_t prepare_mask(Hierarchy &h, hipStream_t s) {
    launch_mask_pyramid(h, h.nlev_full, h.counts, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(read_to_host(h.known, h.counts, sizeof(unsigned int) * MAX_LEVELS, s));
    if (h.known[0] == 0) {
        set_error("empty mask: the inpainting matrix is singular");
        return HDI_ERR_EMPTY_MASK;
    }
    h.nlev = h.nlev_full;
    for (int l = 1; l < h.nlev_full; ++l) {
        const double n = (double)h.lev[l].W * h.lev[l].H;
        if (n - (double)h.known[l] <= 0.01 * n) {
            h.nlev = l + 1;
            break;
        }
    }
    return HDI_OK;
}

size_t inpaint_ws_bytes(int W, int H, int C) {
    Hierarchy h;
    Arena a{nullptr, 0, 0};
    plan_hierarchy(h, a, W, H, C, 4, nullptr);
    return a.used + 256;
}

}  // namespace hdi

using namespace hdi;

extern "C" {

size_t hdi_inpaint_workspace_bytes(hdi_image img) {
    if (img.width < 1 || img.height < 1 || (img.channels != 1 && img.channels != 3)) return 0;
    return inpaint_ws_bytes(img.width, img.height, img.channels);
}

int32_t inpaint_solve(hdi_image img, const uint8_t *mask, const float *f, double *u, const double *u0, void *ws,
                      size_t ws_bytes, const hdi_solve_params *params, hdi_solve_report *report, void *stream) {
    if (!check_image(img)) return HDI_ERR_ARG;
    if (!mask || !f || !u) {
        set_error("mask, f and u must be non-null device pointers");
        return HDI_ERR_ARG;
    }
    SolveCfg cfg;
    int overlap;
    int32_t st = fill_cfg(params, cfg, overlap);
    if (st) return st;
    const size_t need = inpaint_ws_bytes(img.width, img.height, img.channels);
    if (!ws || ws_bytes < need) {
        set_error("workspace of %zu bytes given, %zu needed", ws ? ws_bytes : (size_t)0, need);
        return HDI_ERR_WORKSPACE;
    }
    hipStream_t s = (hipStream_t)stream;
    Arena a{(char *)ws, ws_bytes, 0};
    Hierarchy h;
    plan_hierarchy(h, a, img.width, img.height, img.channels, overlap, mask, cfg.small_from);
    st = prepare_mask(h, s);
    if (st) return st;
    const int C = img.channels;
    if (u0 && u0 != u) {
        hipError_t e = hipMemcpyAsync(u, u0, sizeof(double) * C * img.width * img.height, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) {
            set_error("hipMemcpyAsync: %s", hipGetErrorString(e));
            return HDI_ERR_HIP;
        }
    }
    cfg.known = h.known[0];
    Prof *prof = prof_for_call();
    st = solve_system<float>(h, img.width, img.height, C, mask, f, nullptr, u, u0 != nullptr, cfg, report, s, prof);
    delete prof;
    return st;
}

int32_t hdi_autotune(hdi_image img, const uint8_t *mask, const float *f, void *ws, size_t ws_bytes,
                     const hdi_solve_params *candidates, int32_t n_candidates, int32_t reps,
                     int32_t *best_index, float *best_ms, void *stream) {
    if (!check_image(img)) return HDI_ERR_ARG;
    if (!mask || !f || !candidates || n_candidates < 1 || reps < 1 || !best_index || !best_ms) {
        set_error("autotune needs mask, f, at least one candidate, reps >= 1 and result pointers");
        return HDI_ERR_ARG;
    }
    const size_t N = (size_t)img.width * img.height * img.channels;
    const size_t need = inpaint_ws_bytes(img.width, img.height, img.channels) + N * sizeof(double) + 512;
    if (!ws || ws_bytes < need) {
        set_error("workspace of %zu bytes given, %zu needed", ws ? ws_bytes : (size_t)0, need);
        return HDI_ERR_WORKSPACE;
    }
    Arena a{(char *)ws, ws_bytes, 0};
    double *u = (double *)a.take(N * sizeof(double));
    const size_t rest = ws_bytes - a.used - 256;
    void *sub = (char *)ws + ((a.used + 255) & ~(size_t)255);
    *best_index = -1;
    *best_ms = 0.f;
    for (int k = 0; k < n_candidates; ++k) {
        float tmin = 1e30f;
        bool ok = true;
        for (int r = 0; r < reps && ok; ++r) {
            hdi_solve_report rep;
            const int32_t st = inpaint_solve(img, mask, f, u, nullptr, sub, rest, &candidates[k], &rep, stream);
            if (st == HDI_ERR_ARG || st == HDI_ERR_HIP || st == HDI_ERR_WORKSPACE || st == HDI_ERR_EMPTY_MASK)
                return st;
            ok = st == HDI_OK;
            tmin = std::min(tmin, rep.ms);
        }
        if (ok && (*best_index < 0 || tmin < *best_ms)) {
            *best_index = k;
            *best_ms = tmin;
        }
    }
    if (*best_index < 0) {
        set_error("no candidate reached its tolerance");
        return HDI_ERR_NO_CONVERGENCE;
    }
    return HDI_OK;
}

int64_t hdi_block_count(int32_t width, int32_t height, int32_t overlap) {
    if (width < 1 || height < 1 || overlap < 0 || overlap >= TILE) return -1;
    return (int64_t)make_blocks(width, overlap).count * make_blocks(height, overlap).count;
}

void hdi_stats_enable(int32_t on) { g_stats_on.store(on ? 1 : 0); }

void hdi_stats_reset(void) {
    std::lock_guard<std::mutex> lk(g_stats_mu);
    for (auto &k : g_stats) k = KStats{0, 0.0, 0.0, 0.0, 0.0};
}

int32_t hdi_stats_get(int32_t id, int64_t *launches, double *total_ms, double *alg_bytes, double *alg_flops) {
    if (id < 0 || id >= HDI_NUM_KERNEL_IDS) {
        set_error("kernel id %d outside 0..%d", id, HDI_NUM_KERNEL_IDS - 1);
        return HDI_ERR_ARG;
    }
    std::lock_guard<std::mutex> lk(g_stats_mu);
    if (launches) *launches = g_stats[id].launches;
    if (total_ms) *total_ms = g_stats[id].ms;
    if (alg_bytes) *alg_bytes = g_stats[id].bytes;
    if (alg_flops) *alg_flops = g_stats[id].flops;
    return HDI_OK;
}

int32_t hdi_stats_get_lds(int32_t id, double *lds_bytes) {
    if (id < 0 || id >= HDI_NUM_KERNEL_IDS || !lds_bytes) {
        set_error("kernel id %d outside 0..%d, or no output", id, HDI_NUM_KERNEL_IDS - 1);
        return HDI_ERR_ARG;
    }
    std::lock_guard<std::mutex> lk(g_stats_mu);
    *lds_bytes = g_stats[id].lds;
    return HDI_OK;
}

const char *hdi_status_string(int32_t s) {
    switch (s) {
        case HDI_OK: return "ok";
        case HDI_ERR_ARG: return "invalid argument";
        case HDI_ERR_EMPTY_MASK: return "empty mask";
        case HDI_ERR_NO_CONVERGENCE: return "no convergence";
        case HDI_ERR_WORKSPACE: return "workspace too small";
        case HDI_ERR_HIP: return "HIP runtime error";
        case HDI_ERR_BUDGET: return "exceeds memory budget";
        default: return "unknown status";
    }
}

const char *hdi_last_error(void) { return g_err.c_str(); }

}  // extern "C"
