/* hdi.h -- C ABI of libhdi: homogeneous diffusion inpainting and its data
 * optimisation on AMD Instinct MI355X (gfx950).
 *
 * The library solves the masked 5-point Laplace system of the paper's
 * Sec. 2.1, eq. (inp-discrete-lsi):
 *
 *     A u = C f,   A = C + (I - C) L,
 *
 * C = diag(c) for a binary mask c, L the negated 5-point Laplacian with
 * reflecting boundary (the 4-neighbour grid-graph Laplacian, unit spacing).
 * On top of that solve it offers tonal optimisation (Sec. 5) and one step of
 * Delaunay densification (Sec. 4.1, Alg. 1).
 *
 * Conventions shared by every entry point
 *   Layout     planar C x H x W, row-major, x fastest: element (c, y, x) is at
 *              index c*H*W + y*W + x. Masks are H x W uint8, nonzero = known.
 *   Memory     every array argument is DEVICE memory owned by the caller
 *              (for example torch tensors). The library never allocates or
 *              frees device memory on these paths: scratch space comes from the
 *              caller's workspace buffer, whose size the *_workspace_bytes query
 *              gives. Report structs and n_added are HOST memory.
 *   Streams    `stream` is a hipStream_t passed as void* (NULL = default stream).
 *              Calls are host-synchronous: they return once outputs and reports
 *              are final.
 *   Errors     arguments are checked before any launch; on failure nothing is
 *              launched, outputs are untouched and hdi_last_error() (per thread)
 *              describes the problem. A HIP failure maps to HDI_ERR_HIP. The
 *              library never aborts or exits.
 *   Threads    calls on distinct workspaces may run concurrently.
 */
#ifndef HDI_H
#define HDI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HDI_OK = 0,
    HDI_ERR_ARG = 1,             /* bad size, pointer, parameter or non-finite input */
    HDI_ERR_EMPTY_MASK = 2,      /* c = 0: A is singular (Sec. 2.1) */
    HDI_ERR_NO_CONVERGENCE = 3,  /* tolerance not met within the iteration cap;
                                    outputs hold the last iterate, the report the
                                    achieved residual */
    HDI_ERR_WORKSPACE = 4,       /* workspace missing or smaller than the query */
    HDI_ERR_HIP = 5,             /* a HIP runtime call failed */
    HDI_ERR_BUDGET = 6           /* a server job can never fit the arena */
} hdi_status;

typedef struct {
    int32_t width, height;   /* >= 1 */
    int32_t channels;        /* 1 or 3: colour channels are independent systems
                                sharing one matrix (Sec. 2.1) */
} hdi_image;

/* Inner solver parameters. A zero field selects the default.
 *   rel_tol      stop when max_c ||C f - A u||_2 / ||C f||_2 <= rel_tol
 *                (FP64 residual; default 1e-6)
 *   max_outer    cap on refinement rounds (default 40)
 *   overlap      overlap of the 32x32 subdomain blocks of the Schwarz smoother
 *                on the finest level (Sec. 3.1, 3.3; default 6 as in Sec. 3.3,
 *                valid 2..16, even); the coarser levels use half of it (even,
 *                at least 2)
 *   local_iters  conjugate-gradient iterations per block and smoothing step
 *                on the finest level (Sec. 3.3; default 12)
 *   coarse_iters CG iterations on the coarsest level, which is a single block
 *                (Sec. 3.3; default 64)
 *   flags        HDI_FLAG_* bits
 *   small_from   first level smoothed with 16x16 blocks:
 *                0 automatic (from level 1, the first level with fewer than
 *                4096 blocks of 32x32 over all channels, where the smoother is
 *                bound by the latency of its steps), -1 none, k >= 1 level k
 *   robin        weight w in (0, 0.9] of the Robin transmission condition on
 *                the inner block boundaries of the smoother (the optimised
 *                Schwarz method of Sec. 3.1): in a block's local operator each
 *                edge to a pixel outside the block adds 1 - w to the pixel's
 *                diagonal, which is du/dn + p u = 0 on the edge's midpoint
 *                with p = 2 (1 - w) / (1 + w); w -> 1 tends to a Neumann
 *                condition. 0 selects the default 0.6; a negative value gives
 *                w = 0, a zero Dirichlet value on the outside pixel (plain
 *                restricted additive Schwarz).
 *   local_stop   fraction in [0, 1) for the finest level's smoothing: a
 *                block's local CG also stops once its squared residual is at
 *                most local_stop times the channel's global squared residual
 *                of the refinement round (Sec. 3.3); 0 (the default) runs
 *                local_iters steps (fewer only at the FP32 rounding floor).
 *                Coarse levels always run their fixed step counts.
 *   mid_iters    conjugate-gradient iterations per block and smoothing step on
 *                the levels between the finest and the coarsest, and in the
 *                full-multigrid start (default 8)
 * Each refinement round applies one V-cycle with one pre- and one
 * post-smoothing step (Sec. 3.3).                                            */
typedef struct {
    double rel_tol;
    int32_t max_outer, overlap, local_iters, coarse_iters, flags, small_from;
    float robin, local_stop;
    int32_t mid_iters;
} hdi_solve_params;

#define HDI_FLAG_NO_FMG 1   /* cold start from u = C f instead of the reduced
                               full-multigrid initialisation (Sec. 3.2) */
#define HDI_FLAG_CG 2       /* comparator: plain FP64 conjugate gradients on the
                               unknown pixels (Sec. 2.1) instead of the multigrid
                               method; the baseline of the paper's tonal
                               experiments nests it in CGNR (Sec. 6.1). The same
                               rel_tol criterion on the true FP64 residual; the cap
                               is 1000 * max_outer CG steps, outer_iters reports
                               CG steps and vcycles 0. Single solves only:
                               hdi_solve_batch and the server reject it. */

typedef struct {
    double rel_residual[3];  /* achieved FP64 relative residual per channel */
    int32_t outer_iters;     /* refinement rounds */
    int32_t vcycles;         /* V-cycles applied in total */
    float ms;                /* device time of the call (HIP events) */
} hdi_solve_report;

/* Bytes of workspace inpaint_solve needs for this image. 0 on bad sizes. */
size_t hdi_inpaint_workspace_bytes(hdi_image img);

/* Homogeneous diffusion inpainting, Sec. 2.1 eq. (inp-discrete-lsi), solved
 * with the multigrid Schwarz method of Sec. 3 in FP32 inside an FP64
 * iterative refinement.
 *   mask  H x W uint8, nonzero = known (device)
 *   f     C x H x W float32 image; only values on the mask are read (device)
 *   u     C x H x W float64 output; u = f exactly on the mask (device)
 *   u0    optional C x H x W float64 warm start (device), NULL for none
 *   ws    workspace of at least hdi_inpaint_workspace_bytes(img) (device)
 *   params, report  host, both nullable
 * Returns HDI_ERR_EMPTY_MASK for an all-zero mask and HDI_ERR_NO_CONVERGENCE
 * when rel_tol is not reached within max_outer rounds. */
int32_t inpaint_solve(hdi_image img, const uint8_t *mask, const float *f, double *u,
                      const double *u0, void *ws, size_t ws_bytes,
                      const hdi_solve_params *params, hdi_solve_report *report, void *stream);

/* ------------------------------------------------------------------ no-allocation solve */

/* Size in MiB of the scratch array behind inpaint_solve_noalloc, per GPU. */
#define HDI_NOALLOC_SCRATCH_MB 64

/* Bytes of that array (HDI_NOALLOC_SCRATCH_MB MiB). */
size_t hdi_noalloc_scratch_bytes(void);

/* inpaint_solve for callers that cannot allocate device memory: code that may
 * not call hipMalloc (tight serving loops, harnesses that forbid allocation).
 * The operation, arguments, results and errors are those of inpaint_solve,
 * but the workspace is an array of HDI_NOALLOC_SCRATCH_MB MiB inside the
 * library; each GPU holds its own copy from the first call on it until the
 * process ends. The call makes no device or pinned-host allocation and creates
 * no HIP events: report->ms is host time from entry until the stream's work is
 * done, and the per-kernel statistics do not see the call.
 *   Limit   an image whose hdi_inpaint_workspace_bytes exceeds the array
 *           (beyond about 1024x768 RGB or 1920x1080 gray) returns
 *           HDI_ERR_WORKSPACE before any launch.
 *   Sharing every call on one GPU uses that GPU's array, which keeps the last
 *           call's contents (a solve writes each scratch byte before reading
 *           it). Overlapping calls would race on it, so the calls of one
 *           process on one GPU are serialised by a lock held for the whole
 *           call. */
int32_t inpaint_solve_noalloc(hdi_image img, const uint8_t *mask, const float *f, double *u, const double *u0,
                              const hdi_solve_params *params, hdi_solve_report *report, void *stream);

/* ------------------------------------------------------------------ tonal */

#define HDI_TONAL_PCG_RAS 0   /* flexible CG, one RAS sweep as preconditioner (default) */
#define HDI_TONAL_RAS 1       /* stationary RAS iteration, Alg. 2 */
#define HDI_TONAL_CGNR 2      /* CG on the normal equations, Sec. 5.1 */
#define HDI_TONAL_INIT_FROM_F 1   /* flags: start from g = f on the mask (g input ignored) */
#define HDI_TONAL_TRACE 2         /* flags: print one line per outer iteration to stderr */

/* Tonal optimisation parameters. A zero field selects the default.
 *   rel_tol      stop when max_c ||B^T(f - B g)||_2 / ||B^T f||_2 <= rel_tol,
 *                recomputed with tight inner solves (default 1e-6)
 *   max_outer    outer iteration cap (default 500)
 *   mode         HDI_TONAL_PCG_RAS / HDI_TONAL_RAS / HDI_TONAL_CGNR
 *   overlap      overlap of the blocks of the RAS sweep, even, 2..block/2
 *                (default 16 for 64x64 blocks, 14 for 32x32; Sec. 5.2 uses 6
 *                with 64x64 blocks: here a wider overlap buys fewer outer
 *                iterations than its sweep costs)
 *   local_outer  CG steps on each block's local normal equations (default 5
 *                for 64x64 blocks, 3 for 32x32)
 *   local_inner  CG steps of each local inpainting inside them (default 20
 *                for 64x64 blocks, 24 for 32x32; far fewer steps truncate the
 *                local echoes, which makes the stationary RAS iteration
 *                overshoot)
 *   flags        HDI_TONAL_INIT_FROM_F
 *   inner        parameters of the global inpainting solves (rel_tol is set
 *                per solve by the outer method)
 *   block        edge of the RAS blocks: 64 (Sec. 5.2's size, four wavefronts
 *                per block, the default) or 32 (one wavefront per block)
 *   mse_gain     > 0: also stop once an outer iteration lowers the MSE by less
 *                than this fraction of its previous value, the criterion the
 *                paper proposes with CGNR (Sec. 5.1) and uses in its
 *                comparisons with 1e-3 (Sec. 6.3). The MSE is the running
 *                estimate ||f - B g||^2 / (C N) of the Krylov modes (the
 *                evaluated one for stationary RAS, which undoes a last step
 *                that raised it); the report holds the final values
 *                recomputed with tight solves. 0: off (default)            */
typedef struct {
    double rel_tol;
    int32_t max_outer, mode, overlap, local_outer, local_inner, flags;
    hdi_solve_params inner;
    double mse_gain;
    int32_t block;
} hdi_tonal_params;

typedef struct {
    double mse_initial;          /* ||f - B g0||^2 / (C N) at the start */
    double mse_final;            /* the same at the returned g */
    double rel_normal_residual;  /* true relative normal residual, max over channels */
    int32_t outer_iters, inner_solves;
    int32_t inner_vcycles;       /* V-cycles of the inner solves (CG steps when
                                    the inner parameters set HDI_FLAG_CG) */
    float ms;
} hdi_tonal_report;

/* Bytes of workspace tonal_optimize needs for this image. 0 on bad sizes. */
size_t hdi_tonal_workspace_bytes(hdi_image img);

/* Tonal optimisation, Sec. 5, eq. (tonal-opt-minimisation): the values g on
 * the mask minimising ||f - B g||_2^2 with B = A^{-1} C, found by solving the
 * normal equations B^T B g = B^T f (eq. tonal-normal-equations) matrix-free.
 *   mask  H x W uint8 (device);  f  C x H x W float32 image (device)
 *   g     C x H x W float64 (device). In: the starting values on the mask
 *         (ignored with HDI_TONAL_INIT_FROM_F). Out: the optimised values on
 *         the mask, 0 elsewhere (Sec. 5).
 *   u     nullable C x H x W float64 output: the reconstruction B g (device)
 *   ws    workspace of at least hdi_tonal_workspace_bytes(img) (device)
 * Returns HDI_ERR_EMPTY_MASK for an all-zero mask and HDI_ERR_NO_CONVERGENCE
 * (with the last iterate in g) when the tolerance is not met. */
int32_t tonal_optimize(hdi_image img, const uint8_t *mask, const float *f, double *g, double *u,
                       void *ws, size_t ws_bytes, const hdi_tonal_params *params,
                       hdi_tonal_report *report, void *stream);

/* ------------------------------------------------------------------ batches */

#define HDI_JOB_INPAINT 0
#define HDI_JOB_TONAL 1

/* One job of a batch, with device pointers as for inpaint_solve and
 * tonal_optimize (mask H x W uint8, f C x H x W float32, out C x H x W
 * float64: u for an inpainting job, g for a tonal job, 0 off the mask).
 *   kind          HDI_JOB_INPAINT or HDI_JOB_TONAL
 *   tonal         tonal jobs: nullable parameters (defaults); the job starts
 *                 from g = f on the mask and its inner parameters must not set
 *                 HDI_FLAG_CG
 *   tonal_report  tonal jobs: nullable host report                          */
typedef struct {
    int32_t kind;
    hdi_image img;
    const uint8_t *mask;
    const float *f;
    double *out;
    const hdi_tonal_params *tonal;
    hdi_tonal_report *tonal_report;
} hdi_job;

/* Bytes of workspace hdi_solve_batch needs for these jobs. 0 on bad input. */
size_t hdi_batch_workspace_bytes(int32_t n, const hdi_job *jobs);

/* n inpainting (eq. inp-discrete-lsi) and tonal optimisation (Sec. 5) jobs of
 * any sizes in shared launches: every phase of an inpainting solve is one
 * kernel launch over the work items (image, level, block) of all solves taking
 * part, and each solve refines until its own tolerance. A tonal job's inner
 * solves (B g and the symmetrised solve behind B^T, Sec. 5.1) are solves of
 * these shared launches too, while its own kernels run on a stream of its own.
 * Every result is bit-for-bit what inpaint_solve or tonal_optimize returns for
 * it with the same parameters, whatever else is in the batch.
 *   params   nullable array of n per-job parameter sets (each image its own;
 *            the inpainting parameters of inpainting jobs)
 *   reports  nullable host array of n reports; for a tonal job outer_iters is
 *            its outer iterations and rel_residual[0] its relative normal
 *            residual (ms: the whole batch)
 * Returns the first failing job's status (HDI_ERR_EMPTY_MASK for a job with
 * an empty mask, which ends at once while the others are solved;
 * HDI_ERR_NO_CONVERGENCE with the last iterates). */
int32_t hdi_solve_batch(int32_t n, const hdi_job *jobs, void *ws, size_t ws_bytes,
                        const hdi_solve_params *params, hdi_solve_report *reports, void *stream);

/* ------------------------------------------------------------------ Voronoi initialisation */

/* Starting values for tonal optimisation, Sec. 5.3: make the inpainting match
 * weighted local averages of f around each mask pixel, C W B g = C W f, by
 * Richardson steps g <- g + tau C W (f - B g) from g = f, stopping once the MSE
 * rises and keeping the best iterate. W averages over (weighting):          */
#define HDI_VINIT_DIRECT 0       /* the 3x3 window around the mask pixel, clipped
                                    to the image (one step at tau = 1 is the
                                    error balancing of Galic et al.) */
#define HDI_VINIT_VORONOI 1      /* the mask pixel's Voronoi cell, equal weights */
#define HDI_VINIT_VORONOI_LOG 2  /* the Voronoi cell, weights 1 / (1 + ln(1 + d))
                                    at distance d from the mask pixel (default) */
#define HDI_VINIT_FROM_F 1       /* flags: start from g = f on the mask */
#define HDI_VINIT_NO_STOP 2      /* flags: take max_iters steps regardless of the MSE */
#define HDI_VINIT_TRACE 64       /* MSE values kept in the report */

/*   weighting  HDI_VINIT_*;  max_iters  Richardson steps at most (default 20,
 *   at most 1000);  tau  step size (default 1; the paper asks for a stable one,
 *   the MSE stop guards the rest);  flags  HDI_VINIT_FROM_F | HDI_VINIT_NO_STOP;
 *   solve  parameters of the inpaintings (zero fields: defaults). */
typedef struct {
    int32_t weighting, max_iters;
    double tau;
    int32_t flags;
    hdi_solve_params solve;
} hdi_vinit_params;

typedef struct {
    int32_t steps;                  /* Richardson steps taken */
    int32_t best;                   /* index of the returned iterate (0: the start) */
    int32_t solves;                 /* inpaintings */
    double mse[HDI_VINIT_TRACE];    /* ||f - B g^k||^2 / (C N) for k = 0..steps (first 64) */
    float ms;                       /* device time of the call */
} hdi_vinit_report;

/* Bytes of workspace voronoi_init needs for this image. 0 on bad sizes. */
size_t hdi_vinit_workspace_bytes(hdi_image img);

/* Voronoi initialisation (Sec. 5.3).
 *   mask  H x W uint8 (device);  f  C x H x W float32 image (device)
 *   g     C x H x W float64 (device). In: the starting values on the mask
 *         (ignored with HDI_VINIT_FROM_F). Out: the best iterate on the mask,
 *         0 elsewhere; pass it to tonal_optimize as its start.
 *   u     nullable C x H x W float64 output: B g of the returned g (device)
 *   ws    workspace of at least hdi_vinit_workspace_bytes(img) (device)
 * Cell averages are sums of round(W_ij (f_j - u_j) 2^32) in 64-bit integers
 * (exact and order independent); a value |f - u| >= 2^30 (a diverging step
 * size) returns HDI_ERR_ARG. Returns HDI_ERR_EMPTY_MASK for an all-zero mask
 * and the inpainting's status if a solve fails. */
int32_t voronoi_init(hdi_image img, const uint8_t *mask, const float *f, double *g, double *u,
                     void *ws, size_t ws_bytes, const hdi_vinit_params *params,
                     hdi_vinit_report *report, void *stream);

/* ------------------------------------------------------------------ serving */

/* A request loop over one device: inpainting and tonal requests of any sizes
 * are submitted as they arrive and run with continuous batching. Inpainting
 * requests join the shared launches of the batch engine between refinement
 * rounds; each keeps its own rounds and tolerance and gives bit for bit what
 * inpaint_solve gives. A tonal request runs on a worker thread with a stream of
 * its own, so its kernels overlap the engine's rounds, and gives bit for bit
 * what tonal_optimize gives. With HDI_SERVER_TONAL_SHARED its inner solves (B g
 * and the symmetrised solve behind B^T, Sec. 5.1) join the engine's shared
 * rounds too, while its gathers, RAS sweeps and vector updates stay on its
 * stream. Every request is admitted when its memory in the caller's arena is
 * free (inpainting requests also need an engine slot), in arrival order per
 * kind, and its state stays in device memory until it ends. */
#define HDI_REQ_INPAINT 0
#define HDI_REQ_TONAL 1
#define HDI_REQ_HOST_IO 1   /* request flags: mask, f and out are pinned host memory
                               (copied in and out on the server's copy stream) */
#define HDI_SERVER_PLAIN 1  /* server flags: one request at a time through
                               inpaint_solve / tonal_optimize (the control) */
#define HDI_SERVER_TONAL_SHARED 2  /* server flags: tonal requests hand their inner
                               solves to the engine's shared rounds instead of
                               running them on their worker's own stream (same
                               results; more sharing, longer tonal latency) */

/* One request. Without HDI_REQ_HOST_IO the pointers are device memory that
 * must stay valid and unchanged until the request is done. Tonal requests
 * start from g = f on the mask; with HDI_SERVER_TONAL_SHARED their inner
 * parameters must not set HDI_FLAG_CG (the engine runs the multigrid solver).
 *   out   u (inpaint, C x H x W float64) or g (tonal, 0 off the mask)      */
typedef struct {
    int32_t kind, flags;
    hdi_image img;
    const uint8_t *mask;
    const float *f;
    double *out;
    hdi_solve_params solve;          /* inpaint parameters, zero fields: defaults */
    const hdi_tonal_params *tonal;   /* nullable: tonal defaults */
} hdi_request;

typedef struct {
    int32_t status, kind;
    int32_t outer_iters;       /* refinement rounds (inpaint) or outer iterations (tonal) */
    int32_t inner_solves;      /* tonal: inpainting solves */
    int32_t max_running;       /* most solves sharing one engine round with it (tonal:
                                  with any of its inner solves; 0 when they ran on
                                  the worker's stream) */
    double rel_residual[3];    /* inpaint: per channel; tonal: [0] relative normal residual */
    double mse_initial, mse_final;
    double t_submit_ms, t_start_ms, t_done_ms;   /* host clock, ms since hdi_server_create */
} hdi_request_report;

typedef struct hdi_server hdi_server;

/* Arena bytes one request takes while it runs. 0 on bad input. */
size_t hdi_request_bytes(const hdi_request *req);

/* Start a server on the current device. The arena (caller-owned device memory,
 * not freed by the server) holds the engine tables and every running request's
 * state; max_slots bounds the solves in one engine round (inpainting
 * requests and tonal inner solves), tonal_workers the tonal requests running
 * at once. Returns NULL on bad arguments or HIP
 * failure (hdi_last_error says which). */
hdi_server *hdi_server_create(void *arena, size_t arena_bytes, int32_t max_slots, int32_t tonal_workers,
                              int32_t flags);
/* Queue a request. HDI_ERR_BUDGET if it can never fit the arena. */
int32_t hdi_server_submit(hdi_server *srv, const hdi_request *req, uint64_t *ticket);
/* done = 1 and the report once the request has ended (its outputs final);
 * a ticket is forgotten after the poll that reports it done. */
int32_t hdi_server_poll(hdi_server *srv, uint64_t ticket, int32_t *done, hdi_request_report *report);
/* Wait until every submitted request has ended. */
int32_t hdi_server_drain(hdi_server *srv);
/* Drain, stop the worker threads and release the server's streams. */
void hdi_server_destroy(hdi_server *srv);


/* ------------------------------------------------------------------ densification */

#define HDI_PART_DELAUNAY 0   /* triangles of mask pixels (Sec. 4.1) */
#define HDI_PART_VORONOI 1    /* Voronoi cells of mask pixels (the ablation of Sec. 6.2) */
#define HDI_PART_JFA 4        /* or'ed in: labels by jump flooding (Sec. 4.2) instead of
                                 the exact nearest mask pixel; passes with steps k0,
                                 k0/2, ..., 1 over the nine pixels p + k (i, j),
                                 i, j in {-1, 0, 1}, best by (squared distance, index),
                                 k0 the largest power of two below max(W, H). Exact
                                 integer arithmetic: reproducible, but a few pixels
                                 can get a farther label than the nearest. */

/* Bytes of workspace hdi_voronoi_labels needs. 0 on bad sizes. */
size_t hdi_labels_workspace_bytes(int32_t width, int32_t height);

/* Voronoi labels of a mask (Sec. 4.2: the diagram behind the Delaunay
 * partition): labels[p] = the linear index of p's nearest mask pixel.
 *   jfa_step  0: exact, ties to the smaller index (the labels densify_step
 *             uses); -1: jump flooding from the default start; k > 0, a power of
 *             two: jump flooding from k (fewer passes when every pixel lies
 *             within about k of a mask pixel)
 *   mask      H x W uint8 (device), at least one pixel set (else HDI_ERR_EMPTY_MASK)
 *   labels    H x W int32 output (device)
 *   max_d2    nullable host output: the largest squared pixel-to-label distance
 *             (over labelled pixels: jump flooding from too small a start can
 *             leave pixels at -1) */
int32_t hdi_voronoi_labels(int32_t width, int32_t height, const uint8_t *mask, int32_t *labels, int32_t jfa_step,
                           uint64_t *max_d2, void *ws, size_t ws_bytes, void *stream);

/* Error map that drives densification (Sec. 4.1: the squared error of the
 * current reconstruction, summed over the colour channels):
 * err_i = fp32(sum_c (u_c,i - f_c,i)^2), accumulated in FP64 in channel order
 * and rounded once to nearest, so equal inputs give equal maps everywhere.
 *   u    C x H x W float64, f C x H x W float32, err H x W float32 (device)
 * Enqueued on `stream`; returns without waiting. */
int32_t hdi_error_map(hdi_image img, const double *u, const float *f, float *err, void *stream);

/* Bytes of workspace densify_step needs for a width x height mask. 0 on bad sizes. */
size_t hdi_densify_workspace_bytes(int32_t width, int32_t height);

/* One step of Delaunay densification, Sec. 4.1 Alg. 1: partition the image by
 * the triangulation of the current mask pixels (built from their Voronoi
 * diagram, Sec. 4.2), sum the error map per cell, and in the cells with the
 * largest sums add the pixel of largest error, at most one per cell.
 * Exact discrete reading (every step integer, so results are reproducible):
 * nearest mask pixel by (squared distance, linear index); a 2x2 pixel quad with
 * three or four distinct labels gives one or two triangles (the sorted index
 * triple is the key; duplicates merged, collinear triples dropped); a pixel
 * belongs to the covering closed triangle of smallest key, else to its Voronoi
 * cell; cells rank by (sum of round(e * 2^20) descending, key ascending); the
 * chosen pixel maximises e, ties to the smaller index.
 *   mask     H x W uint8, in/out (device); at least one pixel set
 *   err      H x W float32 error map (device): 0 <= e <= 2^43 / (W H), so that
 *            the fixed-point cell sums stay exact; anything else (negative,
 *            NaN, Inf, too large) is HDI_ERR_ARG before the mask is touched
 *   n_add    pixels to add (>= 0)
 *   added    nullable int32 output (device), capacity n_add: the added
 *            linear indices in ascending order
 *   n_added  host output: min(n_add, number of cells with a free pixel)     */
int32_t densify_step(int32_t width, int32_t height, uint8_t *mask, const float *err, int64_t n_add,
                     int32_t partition, int32_t *added, int64_t *n_added, void *ws, size_t ws_bytes,
                     void *stream);

/* ------------------------------------------------------------------ spatial optimisation */

/* Initial mask by random dithering of the Laplacian magnitude (Sec. 4.2): one
 * coin flip per pixel with a probability proportional to
 * l = sum_c |Delta f_c| (5-point stencil, reflecting boundary, FP64). Pixel p
 * joins iff rand_p < alpha l_p, alpha = n0 / (S 2^-16) with S the exact 64-bit
 * sum of round(l 2^16), so the expected size is n0 (a constant image uses
 * n0 / N). Deterministic for given uniforms.
 *   f      C x H x W float32 (device); rand H x W float64 uniforms in [0, 1)
 *   mask   H x W uint8 output (device); count: host output, its size
 *   ws     device workspace of hdi_initial_mask_workspace_bytes(img) bytes   */
size_t hdi_initial_mask_workspace_bytes(hdi_image img);
int32_t hdi_initial_mask(hdi_image img, const float *f, const double *rand, int64_t n0, uint8_t *mask,
                         int64_t *count, void *ws, size_t ws_bytes, void *stream);

typedef struct {
    double density;          /* final mask density d: floor(d W H) pixels, 0 < d <= 1 */
    double t;                /* factor of the added counts from step to step (1: equal steps) */
    int64_t n0;              /* expected initial size (0: round(floor(d W H) / (n_steps + 1))) */
    int32_t n_steps;         /* densification steps (Alg. 1; the paper's experiments use 20) */
    int32_t partition;       /* HDI_PART_DELAUNAY or HDI_PART_VORONOI, optionally | HDI_PART_JFA:
                                jump-flooding labels whose start step shrinks with the
                                mask (the smallest power of two at least the previous
                                step's largest pixel-to-label distance) */
    hdi_solve_params solve;  /* parameters of every inpainting solve */
} hdi_spatial_params;

typedef struct {
    int64_t initial_count, final_count;
    int32_t solve_rounds;      /* refinement rounds over all solves */
    double rel_residual[3];    /* of the final solve */
    float ms;                  /* device time of the whole optimisation */
} hdi_spatial_report;

/* Called after each densification step with host copies of the mask before the
 * step, the error map the step used and the added pixels (ascending). */
typedef void (*hdi_step_hook)(int32_t step, const uint8_t *mask_before, const float *err,
                              const int32_t *added, int64_t n_added, void *user);

size_t hdi_spatial_workspace_bytes(hdi_image img);

/* Spatial optimisation (Sec. 4, Alg. 1): the initial mask above, then n steps,
 * each an inpainting (warm-started from the previous one after the first), the
 * error map e = fp32(sum_c (u_c - f_c)^2) and densify_step up to the schedule
 * target (cumulative sizes from the realised initial size to floor(d W H); with
 * t = 1 equal steps rounded half to even, else growing by t), and a final
 * inpainting.
 *   mask   H x W uint8 output (device)
 *   u      nullable C x H x W float64 output: the final reconstruction
 *   hook   nullable step hook (host copies; costs a device-to-host copy per step) */
int32_t spatial_optimize(hdi_image img, const float *f, const double *rand, const hdi_spatial_params *params,
                         uint8_t *mask, double *u, void *ws, size_t ws_bytes, hdi_spatial_report *report,
                         hdi_step_hook hook, void *hook_user, void *stream);

/* Autotuner of the inpainting solver: runs inpaint_solve on this image once
 * per candidate parameter set (reps times each, keeping the fastest device
 * time) and returns the index of the fastest candidate that reached its
 * tolerance. The tunables are the block overlap, the local CG steps per
 * smoothing and the coarsest-level CG steps (Sec. 3.3 tuned these for its GPU;
 * the best values depend on image size and mask density).
 *   ws  device workspace of at least hdi_inpaint_workspace_bytes(img) plus
 *       C*H*W doubles plus 512 bytes (it also holds the trial solutions)     */
int32_t hdi_autotune(hdi_image img, const uint8_t *mask, const float *f, void *ws, size_t ws_bytes,
                     const hdi_solve_params *candidates, int32_t n_candidates, int32_t reps,
                     int32_t *best_index, float *best_ms, void *stream);

/* Number of 32x32 Schwarz blocks with the given overlap on one level of one
 * channel: per dimension ceil((n - 32) / (32 - overlap)) + 1 (1 if n <= 32),
 * the last block shifted to end at the border (Sec. 3.3). Host-only. */
int64_t hdi_block_count(int32_t width, int32_t height, int32_t overlap);

/* Kernel timing (host-only switches; the numbers come from HIP events recorded
 * around each launch on the caller's stream while enabled). Kernel ids:
 *   0 FP64 residual (finest level)     1 Schwarz pre-smoothing (finest level)
 *   2 Schwarz post-smoothing (finest)  3 residual restriction (finest level)
 *   4 FP64 refinement update           5 all coarser levels and the FMG start
 *   6 tonal RAS sweep (local normal equations)
 *   7 tonal vector kernels (gathers, scatters, dot products, updates)
 * For each id the library accumulates the number of launches, their summed
 * device time in ms, the algorithmic bytes those launches must move (every
 * input element read once, every output element written once) and the
 * algorithmic floating-point operations of the block solvers (15 per pixel and
 * local CG step: stencil 5, two dot products 4, three vector updates 6; 20 per
 * pixel and local CGNR step of the tonal sweep). The tonal RAS sweep counts the
 * local steps it actually takes (a local CG stops at its FP32 residual floor);
 * the Schwarz smoother's figure assumes every configured step (an upper bound).
 * Id 5 counts the coarse recursion of each V-cycle by the finest level's
 * per-launch bytes and FLOPs applied level by level; the launches of the FMG
 * start, timed under the same id, carry no byte or FLOP count. */
#define HDI_NUM_KERNEL_IDS 8
void hdi_stats_enable(int32_t on);
void hdi_stats_reset(void);
int32_t hdi_stats_get(int32_t kernel_id, int64_t *launches, double *total_ms, double *alg_bytes,
                      double *alg_flops);

/* LDS bytes of the launches timed under the same switches (kernel id as above;
 * counted for the tonal RAS sweep, 0 for the other ids). Every lane of a
 * TB x TB tile issues the tile's LDS operations, so per tile pixel:
 *   local CG step    8 bytes (the direction written to the tile, the halo of
 *                    the lane's 4x4 pixels read back), plus 1 byte per block
 *                    sum on 64x64 blocks (four wavefront slots read; two sums)
 *   local CGNR step  24 bytes (two such exchanges, t parked in LDS and read
 *                    back), plus 4 bytes of block sums on 64x64 blocks
 *   once per block   the zeroed tile and, on 64x64 blocks, the first sum
 * over the local steps the sweep takes (the slot writes, one lane per
 * wavefront, are left out). ARG for an unknown id or a null output. */
int32_t hdi_stats_get_lds(int32_t kernel_id, double *lds_bytes);

/* Measured LDS bandwidth of the current device: a kernel that only writes and
 * reads float4s through LDS (16 blocks of 256 threads per CU, 128 bytes per
 * lane and iteration) is launched four times on `stream`; *bytes_per_s is the
 * rate of the fastest of the last three. It is the ceiling against which the
 * block solvers' LDS traffic is set.
 *   iters        1..2^20 (4096 take a few milliseconds)
 *   sink         device pointer to one float (caller-owned; never written in
 *                practice, it keeps the compiler from removing the loop)
 * Host-synchronous. ARG for bad arguments, HIP if a launch or event fails. */
int32_t hdi_lds_calibrate(int32_t iters, float *sink, double *bytes_per_s, void *stream);

const char *hdi_status_string(int32_t status);
const char *hdi_last_error(void);   /* thread-local message of the last failure */

#ifdef __cplusplus
}
#endif
#endif /* HDI_H */
