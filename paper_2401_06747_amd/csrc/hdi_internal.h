// Internal declarations shared by the host driver and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <chrono>
#include <string>

#include "../../include/hdi.h"
#include "arena.h"

namespace hdi {

constexpr int TILE = 32;          // Schwarz block edge of the fine levels (Sec. 3.3 uses 32x32)
constexpr int TILE_SMALL = 16;    // block edge of the small-tile smoother
constexpr int MAX_LEVELS = 16;
constexpr int RED_THREADS = 256;  // threads of the reduction kernels

void set_error(const char *fmt, ...);
bool check_image(const hdi_image &img);   // sizes >= 1, 1 or 3 channels, at most 2^30 pixels

// A small device-to-host read that the host waits for (a convergence test, a
// count): staged through a pinned per-thread buffer, so that the copy is
// asynchronous, and waited for by polling the stream for up to 5 ms before a
// blocking wait (a blocking wait adds tens of microseconds of wake-up to each
// test). Larger reads take a plain copy and the same wait. Returns the first
// HIP error.
hipError_t read_to_host(void *dst, const void *src, size_t bytes, hipStream_t s);

// Blocks of the fine-level TILE x TILE smoother along one dimension.
inline Blocks1D make_blocks(int n, int overlap) { return make_blocks(n, overlap, TILE); }

struct Level {
    int W, H;
    int tile;        // block edge of this level's smoother (32 or 16)
    Blocks1D bx, by;
    uint8_t *mask;   // level mask (level 0: the caller's mask)
    float *r;        // right-hand side of the correction equation, C x H x W
    float *ea, *eb;  // correction ping-pong buffers, C x H x W
    float *aux;      // FMG: restricted data on this level, C x H x W
};

// A laid-out multigrid hierarchy for one image shape.
struct Hierarchy {
    int C, nlev;
    Level lev[MAX_LEVELS];
    double *partials;   // [C][nblk][2] block partial sums of the residual kernel
    double *norms;      // [C][2] (||r||^2, ||b||^2)
    double *u_alt;      // C x H x W FP64 second iterate buffer (fused refinement step)
    unsigned int *counts;  // [MAX_LEVELS] known pixels per level
    int nblk;           // blocks of the residual kernel
    int nlev_full;      // levels down to one block
    unsigned int known[MAX_LEVELS];  // host copy of counts
    // plain CG solver (HDI_FLAG_CG): three FP64 C x H x W vectors (residual and
    // two search directions) aliasing the multigrid buffers (a solve uses one
    // method or the other), its block partial sums and scalars
    double *cg_r, *cg_p[2], *cg_part, *cg_scal;
    // set once a solve has handed its u_alt buffer to the caller (the region
    // the CG vectors alias then holds the caller's data)
    bool u_alt_moved = false;
};
constexpr int CG_BLOCKS = 4096;   // workgroups of the CG kernels (grid-stride)

// Lay out the hierarchy in the arena (base == nullptr: size query only).
// overlap: of the finest level's blocks; the coarser levels use half of it
// (even, at least 2). small_from: the first level smoothed with 16x16 blocks;
// 0 picks it from the block counts, -1 keeps 32x32 blocks on every level
bool plan_hierarchy(Hierarchy &h, Arena &a, int W, int H, int C, int overlap, const uint8_t *mask0,
                    int small_from = -1);
inline int coarse_overlap(int overlap) { return overlap / 2 >= 2 ? (overlap / 2) & ~1 : 2; }

struct SolveCfg {
    double rel_tol;
    int max_outer, local_iters, coarse_iters, vcycles, flags;
    int mid_iters;     // local CG steps on the levels between the finest and the coarsest
    float robin;       // Robin weight of the Schwarz smoother (hdi_solve_params::robin)
    float local_stop;  // global-relative local stop (hdi_solve_params::local_stop)
    int small_from;  // hdi_solve_params::small_from (0 automatic, -1 none)
    int64_t known;   // number of known pixels (for the byte accounting)
    bool untimed = false;   // no device time in the report (no wait for the stream at the end)
};

// A call that must not allocate (inpaint_solve_noalloc) holds one of these on
// its thread for its duration. Meanwhile small host reads skip the pinned
// staging buffer (a plain copy into the caller's host memory), call timers use
// the host clock instead of HIP events, and per-kernel statistics are off.
struct NoAllocScope {
    NoAllocScope();
    ~NoAllocScope();
};
bool no_alloc_active();

// Device time of one call: the start and stop events live as long as the
// object, so every return path releases them. Under a NoAllocScope it makes no
// events and measures host time from start() to the end of the stream's work.
// Waits for a stream or an event by polling for up to 5 ms, then blocks (a
// blocking wait wakes the host tens of microseconds after the device is done).
hipError_t wait_for(hipStream_t s);
hipError_t wait_for(hipEvent_t ev);

struct CallTimer {
    hipEvent_t a = nullptr, b = nullptr;
    bool host = false;
    std::chrono::steady_clock::time_point t0;
    hipError_t start(hipStream_t s) {
        if (no_alloc_active()) {
            host = true;
            t0 = std::chrono::steady_clock::now();
            return hipSuccess;
        }
        hipError_t e = hipEventCreate(&a);
        if (e == hipSuccess) e = hipEventCreate(&b);
        if (e == hipSuccess) e = hipEventRecord(a, s);
        return e;
    }
    // records the stop event, waits for it, and stores the elapsed time in *ms
    hipError_t stop(hipStream_t s, float *ms) {
        if (host) {
            const hipError_t e = wait_for(s);
            *ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
            return e;
        }
        hipError_t e = hipEventRecord(b, s);
        if (e == hipSuccess) e = wait_for(b);
        if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
        return e;
    }
    ~CallTimer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Optional per-kernel event timing (hdi_stats_*). One Prof per call; records
// are resolved after the call's final synchronisation.
struct Prof {
    bool on = false;
    struct Rec { int id; double bytes, flops, lds; hipEvent_t a, b; };
    Rec recs[4096];
    int n = 0;
    bool pending = false;   // begin() made the events of recs[n]
    bool ended = false;     // the last begin() was closed by end() as recs[n - 1]
    void begin(int id, double bytes, hipStream_t s, double flops = 0.0);
    void end(hipStream_t s);
    void flush();   // accumulate into the global counters and free the events
    // FLOPs and LDS bytes of the record the last begin()/end() pair made, when
    // they are known only after the launch (nothing if that pair made none)
    void set_last(double flops, double lds) {
        if (on && ended) {
            recs[n - 1].flops = flops;
            recs[n - 1].lds = lds;
        }
    }
    // The record the last begin()/end() pair made is left out of the counters
    // (a launch that turned out to be unneeded); its events are still freed.
    void drop_last() {
        if (on && ended) recs[n - 1].id = -1;
        ended = false;
    }
};
Prof *prof_for_call();   // nullptr when timing is off

// Kernel launchers (solver_kernels.hip).

// u = data (or 0) on known pixels; on unknown pixels 0, or left unchanged
// with keep_unknown (a warm start, or before the FMG prolongation writes them)
template <typename TD>
void launch_init_u(int W, int H, int C, const uint8_t *mask, const TD *data, bool keep_unknown, double *u,
                   hipStream_t s);
dim3 residual_grid(int W, int H);
template <typename TD>
void launch_residual(int W, int H, int C, const uint8_t *mask, const double *u_in, const float *e, double *u_out,
                     const TD *data, const double *src, float *r, double *partials, double *norms, hipStream_t s);
void launch_update(int W, int H, int C, const uint8_t *mask, const float *e, double *u, hipStream_t s);
// Schwarz smoothing steps. robin: weight of the Robin transmission condition
// at inner block boundaries (0: zero Dirichlet values outside the block).
// gnorm, frac: a block's local CG also stops once its squared residual is at
// most frac times the channel's global squared residual gnorm[2 c] (nullptr or
// 0: fixed step count).
// guard >= 0 (finest level): every block returns at once when the residual
// norms in gnorm (rr, bb per channel) already give rr <= guard^2 bb in every
// channel (rr <= guard^2 where bb = 0); the launch can then be queued before
// the host has tested them.
void launch_smooth_pre(const Level &L, int C, int iters, float robin, const double *gnorm, float frac, float *e_out,
                       hipStream_t s, double guard = -1.0);
void launch_smooth_post(const Level &L, const Level &Lc, int C, int iters, float robin, const double *gnorm,
                        float frac, const float *e_in, const float *ec, float *e_out, hipStream_t s);
void launch_restrict_residual(const Level &L, const Level &Lc, int C, const float *e, hipStream_t s);
// FMG helpers
template <typename TD>
void launch_data_restrict0(int W, int H, int C, const uint8_t *mask, const TD *data, const Level &Lc, hipStream_t s);
void launch_data_restrict(const Level &L, const Level &Lc, int C, hipStream_t s);
void launch_fmg_prolong(const Level &L, const Level &Lc, int C, const float *ec, float *out, hipStream_t s);
void launch_fmg_prolong0(int W, int H, int C, const uint8_t *mask, const Level &Lc, const float *ec, double *u, hipStream_t s);
void launch_smooth_fmg(const Level &L, int C, int iters, float robin, const float *e_in, float *e_out,
                       hipStream_t s);

// Build the coarse masks of levels 1..nlev-1 and count known pixels per level
// into counts[0..nlev) (counts must hold MAX_LEVELS entries).
void launch_mask_pyramid(const Hierarchy &h, int nlev, unsigned int *counts, hipStream_t s);

// ------------------------------------------------------------------ batched solves
// Descriptor of one level of one image in a batch (device table [img][MAX_LEVELS]).
struct BLev {
    int W, H, ntx, nty, sx, sy;
    int Wc, Hc;                 // next coarser level (0 x 0 on the last level)
    const uint8_t *mask;
    uint8_t *mask_c;            // next level's mask
    float *r, *ea, *eb, *aux;   // this level's buffers
    float *r_c, *aux_c;         // next level's right-hand side and FMG data
    const float *ec;            // next level's final correction (post-smoothing input)
};
// What a batched solve's right-hand side is: A x = C d + (I - C) s with d the
// FP32 image (inpainting), d an FP64 image (tonal: x = B g), or s an FP64
// source off the mask and d = 0 (tonal: the symmetrised solve of B^T).
enum { EK_DATA_F32 = 0, EK_DATA_F64 = 1, EK_SRC_F64 = 2 };

// Descriptor of one image in a batch.
struct BImg {
    int W, H, C, nlev, local_iters, coarse_iters, gx, nblk;
    int mid_iters;
    float robin, local_stop;
    int kind;                 // EK_*
    int warm;                 // 1: u holds the start on unknown pixels (no FMG)
    const uint8_t *mask;
    const float *f;           // EK_DATA_F32
    const double *data_d;     // EK_DATA_F64
    const double *src;        // EK_SRC_F64
    double *u, *u_alt, *partials, *norms;
    unsigned int *counts;
};
// One launch's work list: nseg segments {img, level, first workgroup, unit}
// (device table, starts ascending from 0) covering n workgroups.
struct BPhase {
    const int4 *seg;
    int nseg, n;
};
void launch_b_count(const BPhase &ph, const BLev *L, const BImg *I, hipStream_t s);
void launch_b_init_u(const BPhase &ph, const BImg *I, hipStream_t s);
void launch_b_residual(const BPhase &ph, int C, const BImg *I, const uint8_t *flags, const BLev *L, hipStream_t s);
void launch_b_reduce(const BPhase &ph, const BImg *I, hipStream_t s);
// mode 0 pre-smoothing (coarsest: uses coarse_iters), 1 post, 2 FMG (coarsest: e_in = aux);
// tile: the block edge of the level in every segment of the launch
void launch_b_schwarz(int mode, bool coarsest, int tile, const BPhase &ph, const BLev *L, const BImg *I,
                      hipStream_t s);
void launch_b_restrict(const BPhase &ph, const BLev *L, const BImg *I, hipStream_t s);
void launch_b_data_restrict(bool from_f, const BPhase &ph, const BLev *L, const BImg *I, hipStream_t s);
void launch_b_fmg_prolong(const BPhase &ph, const BLev *L, const BImg *I, hipStream_t s);
void launch_b_fmg_prolong0(const BPhase &ph, const BLev *L, const BImg *I, hipStream_t s);

// Plain CG (comparator): start computes r = b - A u, r.r and b.b (beta = 0);
// one iteration is direction, alpha, update, beta (scalars stay on the device).
template <typename TD>
void launch_cg_start(int W, int H, int C, const uint8_t *mask, const double *u, const TD *data, const double *src,
                     double *r, double *part, double *scal, hipStream_t s);
void launch_cg_iteration(int W, int H, int C, const uint8_t *mask, double *u, double *r, const double *p_old,
                         double *p_new, double *part, double *scal, hipStream_t s);

// Exact Voronoi labels (nearest mask pixel by squared distance, then index)
// into labels[W*H], using voronoi_scratch_ints(W, H) ints of scratch.
size_t voronoi_scratch_ints(int W, int H);
void launch_voronoi_labels(int W, int H, const uint8_t *mask, int *scratch, int *labels, hipStream_t s);

// densify_step with a jump-flooding start step (0: the default) when the
// partition carries HDI_PART_JFA, and the largest squared pixel-to-label
// distance of the labels it used (host, nullable).
int32_t densify_step_ex(int W, int H, uint8_t *mask, const float *err, long long n_add, int partition, int jfa_k0,
                        int32_t *added, int64_t *n_added, uint64_t *max_d2, void *ws, size_t ws_bytes, hipStream_t s);

// Coarse masks, known counts and the number of levels for a new mask.
int32_t prepare_mask(Hierarchy &h, hipStream_t s);

// An executor of inner solves for tonal optimisation (the server's batch
// engine): A x = C data + (I - C) src on the hierarchy h (planned for `mask`
// with blocks of `overlap`), with exactly one of data and src given, x the
// start on unknown pixels when warm. The solve is ordered after the work
// enqueued on s before the call, later work on s after the solve; x holds the
// solution when later work on s runs. Returns the status (with the message set
// on failure) and fills rep's residuals, rounds and V-cycles.
struct SolveHook {
    virtual ~SolveHook() = default;
    virtual int32_t solve(Hierarchy &h, int overlap, int W, int H, int C, const uint8_t *mask, const double *data,
                          const double *src, double *x, bool warm, const SolveCfg &cfg, hdi_solve_report *rep,
                          hipStream_t s) = 0;
};

// tonal_optimize with its inner solves run by `hook` (nullptr: on the calling
// thread, as tonal_optimize does); the results are the same bit for bit.
int32_t tonal_optimize_hooked(hdi_image img, const uint8_t *mask, const float *f, double *g, double *u, void *ws,
                              size_t ws_bytes, const hdi_tonal_params *params, hdi_tonal_report *report, void *stream,
                              SolveHook *hook);
// Checks tonal parameters and fills the outer configuration and the inner
// solves' configuration (HDI_ERR_ARG on a bad value).
struct TonalCfg {
    double rel_tol;
    int max_outer, mode, overlap, local_outer, local_inner, flags;
    double mse_gain;   // > 0: stop when an iteration improves the MSE by less than this fraction
    int block;         // RAS block edge, 32 or 64
};
int32_t fill_tonal_cfg(const hdi_tonal_params *params, TonalCfg &tc, SolveCfg &inner, int &ov_inner);

// Host driver: solve A x = C data + (I - C) src on the caller's buffers.
// swap: optional address of the caller's pointer to u. When the refinement ends
// in the workspace copy, the two buffers trade places (*swap and h.u_alt are
// exchanged) instead of copying the result back; then no CG solve may follow
// on this hierarchy.
template <typename TD>
int32_t solve_system(Hierarchy &h, int W, int H, int C, const uint8_t *mask, const TD *data,
                     const double *src, double *u, bool warm, const SolveCfg &cfg,
                     hdi_solve_report *rep, hipStream_t s, Prof *prof = nullptr, double **swap = nullptr);

}  // namespace hdi
