/* The C ABI of libhdi (include/hdi.h) called from C, on its host-only paths:
 * status strings, the block-count rule, workspace and request size queries,
 * and argument errors, which every entry point reports before any HIP call
 * (so this runs without a GPU). Dummy device pointers are never dereferenced.
 * Prints "abi host: ok" and exits 0 when every check holds. */
#include <pthread.h>
#include <stdio.h>
#include <string.h>

#include "../../include/hdi.h"

static int g_fail = 0;
#define CHECK(cond)                                                        \
    do {                                                                   \
        if (!(cond)) {                                                     \
            printf("check failed: %s (line %d): last error '%s'\n", #cond, \
                   __LINE__, hdi_last_error());                            \
            ++g_fail;                                                      \
        }                                                                  \
    } while (0)
/* a call that must fail with `code` and leave a message */
#define FAILS(code, call)                                       \
    do {                                                        \
        int32_t st_ = (call);                                   \
        CHECK(st_ == (code));                                   \
        CHECK(hdi_last_error() && hdi_last_error()[0] != '\0'); \
    } while (0)

static void *const DEV = (void *)256; /* a non-null device address, never touched */

static void strings(void) {
    CHECK(strcmp(hdi_status_string(HDI_OK), "ok") == 0);
    CHECK(strcmp(hdi_status_string(HDI_ERR_EMPTY_MASK), "empty mask") == 0);
    CHECK(strcmp(hdi_status_string(HDI_ERR_WORKSPACE), "workspace too small") == 0);
    CHECK(strcmp(hdi_status_string(HDI_ERR_BUDGET), "exceeds memory budget") == 0);
    CHECK(strcmp(hdi_status_string(77), "unknown status") == 0);
    for (int s = 0; s <= 6; ++s) CHECK(strcmp(hdi_status_string(s), "unknown status") != 0);
}

static void geometry(void) {
    /* Sec. 3.3: 36852 local problems for 32x32 blocks, overlap 6, 4K RGB */
    CHECK(hdi_block_count(3840, 2160, 6) * 3 == 36852);
    CHECK(hdi_block_count(32, 32, 6) == 1);
    CHECK(hdi_block_count(33, 1, 6) == 2);
    CHECK(hdi_block_count(0, 5, 6) == -1);
    CHECK(hdi_block_count(64, 64, 32) == -1);
}

static void sizes(void) {
    const hdi_image bad[] = {{0, 5, 1}, {5, 0, 1}, {5, 5, 2}, {-3, 5, 3}};
    for (int i = 0; i < 4; ++i) {
        CHECK(hdi_inpaint_workspace_bytes(bad[i]) == 0);
        CHECK(hdi_tonal_workspace_bytes(bad[i]) == 0);
        CHECK(hdi_vinit_workspace_bytes(bad[i]) == 0);
        CHECK(hdi_initial_mask_workspace_bytes(bad[i]) == 0);
        CHECK(hdi_spatial_workspace_bytes(bad[i]) == 0);
    }
    CHECK(hdi_densify_workspace_bytes(0, 7) == 0);
    CHECK(hdi_labels_workspace_bytes(7, 0) == 0);
    const hdi_image small = {64, 48, 1}, rgb = {64, 48, 3}, big = {1920, 1080, 3};
    CHECK(hdi_inpaint_workspace_bytes(small) > 0);
    CHECK(hdi_inpaint_workspace_bytes(rgb) > hdi_inpaint_workspace_bytes(small));
    CHECK(hdi_inpaint_workspace_bytes(big) > hdi_inpaint_workspace_bytes(rgb));
    CHECK(hdi_tonal_workspace_bytes(big) > hdi_inpaint_workspace_bytes(big));
    CHECK(hdi_vinit_workspace_bytes(big) > 0 && hdi_spatial_workspace_bytes(big) > 0);
    CHECK(hdi_densify_workspace_bytes(1920, 1080) > hdi_densify_workspace_bytes(64, 48));
    CHECK(hdi_labels_workspace_bytes(1920, 1080) > 0 && hdi_initial_mask_workspace_bytes(big) > 0);
    CHECK(hdi_noalloc_scratch_bytes() == ((size_t)HDI_NOALLOC_SCRATCH_MB << 20));

    hdi_job jobs[2] = {{HDI_JOB_INPAINT, {64, 48, 1}, DEV, DEV, DEV, NULL, NULL},
                       {HDI_JOB_INPAINT, {100, 70, 3}, DEV, DEV, DEV, NULL, NULL}};
    const size_t two = hdi_batch_workspace_bytes(2, jobs);
    CHECK(two >= hdi_inpaint_workspace_bytes(jobs[0].img) + hdi_inpaint_workspace_bytes(jobs[1].img));
    CHECK(hdi_batch_workspace_bytes(1, jobs) < two);
    /* a tonal job runs with its tonal workspace (plus staging-free request state) */
    jobs[1].kind = HDI_JOB_TONAL;
    CHECK(hdi_batch_workspace_bytes(2, jobs) >= hdi_tonal_workspace_bytes(jobs[1].img));
    jobs[1].kind = 5;
    CHECK(hdi_batch_workspace_bytes(2, jobs) == 0);
    jobs[1].kind = HDI_JOB_INPAINT;
    jobs[1].img.channels = 2;
    CHECK(hdi_batch_workspace_bytes(2, jobs) == 0);
    CHECK(hdi_batch_workspace_bytes(0, jobs) == 0);

    hdi_request r;
    memset(&r, 0, sizeof r);
    r.kind = HDI_REQ_INPAINT;
    r.img = rgb;
    const size_t rin = hdi_request_bytes(&r);
    CHECK(rin >= hdi_inpaint_workspace_bytes(rgb));
    r.kind = HDI_REQ_TONAL;
    CHECK(hdi_request_bytes(&r) >= hdi_tonal_workspace_bytes(rgb));
    r.flags = HDI_REQ_HOST_IO; /* plus the staged mask, f and out */
    CHECK(hdi_request_bytes(&r) >= hdi_tonal_workspace_bytes(rgb) + 64 * 48 * (1 + 12 * 3));
    r.kind = 9;
    CHECK(hdi_request_bytes(&r) == 0);
    CHECK(hdi_request_bytes(NULL) == 0);
}

static void argument_errors(void) {
    const hdi_image img = {40, 30, 3};
    hdi_solve_report rep;
    hdi_solve_params sp;
    memset(&sp, 0, sizeof sp);
    FAILS(HDI_ERR_ARG, inpaint_solve((hdi_image){40, 30, 2}, DEV, DEV, DEV, NULL, DEV, 1 << 30, NULL, &rep, NULL));
    FAILS(HDI_ERR_ARG, inpaint_solve(img, NULL, DEV, DEV, NULL, DEV, 1 << 30, NULL, &rep, NULL));
    sp.overlap = 5;
    FAILS(HDI_ERR_ARG, inpaint_solve(img, DEV, DEV, DEV, NULL, DEV, 1 << 30, &sp, &rep, NULL));
    sp.overlap = 0;
    sp.flags = 64;
    FAILS(HDI_ERR_ARG, inpaint_solve(img, DEV, DEV, DEV, NULL, DEV, 1 << 30, &sp, &rep, NULL));
    sp.flags = 0;
    sp.rel_tol = 2.0;
    FAILS(HDI_ERR_ARG, inpaint_solve(img, DEV, DEV, DEV, NULL, DEV, 1 << 30, &sp, &rep, NULL));
    sp.rel_tol = 0.0;
    sp.robin = 0.95f; /* Robin weight above 0.9 */
    FAILS(HDI_ERR_ARG, inpaint_solve(img, DEV, DEV, DEV, NULL, DEV, 1 << 30, &sp, &rep, NULL));
    sp.robin = 0.5f;
    sp.local_stop = 1.0f; /* local stop fraction must be below 1 */
    FAILS(HDI_ERR_ARG, inpaint_solve(img, DEV, DEV, DEV, NULL, DEV, 1 << 30, &sp, &rep, NULL));
    sp.local_stop = -0.5f;
    FAILS(HDI_ERR_ARG, inpaint_solve(img, DEV, DEV, DEV, NULL, DEV, 1 << 30, &sp, &rep, NULL));
    sp.robin = 0.0f;
    sp.local_stop = 0.0f;
    FAILS(HDI_ERR_WORKSPACE, inpaint_solve(img, DEV, DEV, DEV, NULL, DEV, 16, &sp, &rep, NULL));
    FAILS(HDI_ERR_WORKSPACE, inpaint_solve(img, DEV, DEV, DEV, NULL, NULL, 1 << 30, &sp, &rep, NULL));
    FAILS(HDI_ERR_WORKSPACE, inpaint_solve_noalloc((hdi_image){3840, 2160, 3}, DEV, DEV, DEV, NULL, NULL, &rep, NULL));
    FAILS(HDI_ERR_ARG, inpaint_solve_noalloc(img, DEV, NULL, DEV, NULL, NULL, &rep, NULL));

    hdi_tonal_params tp;
    hdi_tonal_report trep;
    memset(&tp, 0, sizeof tp);
    FAILS(HDI_ERR_ARG, tonal_optimize(img, DEV, DEV, NULL, NULL, DEV, 1 << 30, &tp, &trep, NULL));
    tp.mode = 7;
    FAILS(HDI_ERR_ARG, tonal_optimize(img, DEV, DEV, DEV, NULL, DEV, 1 << 30, &tp, &trep, NULL));
    tp.mode = 0;
    tp.mse_gain = 1.5;
    FAILS(HDI_ERR_ARG, tonal_optimize(img, DEV, DEV, DEV, NULL, DEV, 1 << 30, &tp, &trep, NULL));
    tp.mse_gain = 0.0;
    FAILS(HDI_ERR_WORKSPACE, tonal_optimize(img, DEV, DEV, DEV, NULL, DEV, 64, &tp, &trep, NULL));

    hdi_vinit_params vp;
    hdi_vinit_report vrep;
    memset(&vp, 0, sizeof vp);
    vp.weighting = 9;
    FAILS(HDI_ERR_ARG, voronoi_init(img, DEV, DEV, DEV, NULL, DEV, 1 << 30, &vp, &vrep, NULL));
    vp.weighting = 0;
    vp.max_iters = 5000;
    FAILS(HDI_ERR_ARG, voronoi_init(img, DEV, DEV, DEV, NULL, DEV, 1 << 30, &vp, &vrep, NULL));

    int64_t n_added = -1;
    FAILS(HDI_ERR_ARG, densify_step(0, 30, DEV, DEV, 5, HDI_PART_DELAUNAY, NULL, &n_added, DEV, 1 << 30, NULL));
    FAILS(HDI_ERR_ARG, densify_step(40, 30, DEV, DEV, -1, HDI_PART_DELAUNAY, NULL, &n_added, DEV, 1 << 30, NULL));
    FAILS(HDI_ERR_ARG, densify_step(40, 30, DEV, DEV, 5, 3, NULL, &n_added, DEV, 1 << 30, NULL));
    FAILS(HDI_ERR_WORKSPACE, densify_step(40, 30, DEV, DEV, 5, HDI_PART_DELAUNAY, NULL, &n_added, DEV, 8, NULL));
    uint64_t d2 = 0;
    FAILS(HDI_ERR_ARG, hdi_voronoi_labels(40, 30, NULL, DEV, -1, &d2, DEV, 1 << 30, NULL));
    FAILS(HDI_ERR_ARG, hdi_error_map(img, NULL, DEV, DEV, NULL));
    int64_t count = 0;
    FAILS(HDI_ERR_ARG, hdi_initial_mask(img, NULL, DEV, 10, DEV, &count, DEV, 1 << 30, NULL));

    hdi_spatial_params pp;
    hdi_spatial_report prep;
    memset(&pp, 0, sizeof pp);
    pp.density = 0.0;
    pp.n_steps = 4;
    FAILS(HDI_ERR_ARG, spatial_optimize(img, DEV, DEV, &pp, DEV, DEV, DEV, 1 << 30, &prep, NULL, NULL, NULL));

    int32_t best = 0;
    float best_ms = 0.f;
    FAILS(HDI_ERR_ARG, hdi_autotune(img, DEV, DEV, DEV, 1 << 30, &sp, 0, 1, &best, &best_ms, NULL));

    hdi_job job = {HDI_JOB_INPAINT, {40, 30, 3}, DEV, DEV, DEV, NULL, NULL};
    FAILS(HDI_ERR_ARG, hdi_solve_batch(-1, &job, DEV, 1 << 30, NULL, NULL, NULL));
    FAILS(HDI_ERR_WORKSPACE, hdi_solve_batch(1, &job, DEV, 64, NULL, NULL, NULL));
    job.kind = 7;
    FAILS(HDI_ERR_ARG, hdi_solve_batch(1, &job, DEV, 1 << 30, NULL, NULL, NULL));
    job.kind = HDI_JOB_TONAL;
    hdi_tonal_params bad_tp;
    memset(&bad_tp, 0, sizeof bad_tp);
    bad_tp.inner.flags = HDI_FLAG_CG; /* the engine runs the multigrid solver only */
    job.tonal = &bad_tp;
    FAILS(HDI_ERR_ARG, hdi_solve_batch(1, &job, DEV, 1 << 30, NULL, NULL, NULL));
    job.tonal = NULL;
    job.kind = HDI_JOB_INPAINT;
    job.img.channels = 4;
    FAILS(HDI_ERR_ARG, hdi_solve_batch(1, &job, DEV, 1 << 30, NULL, NULL, NULL));

    uint64_t ticket = 0;
    int32_t done = 0;
    hdi_request req;
    memset(&req, 0, sizeof req);
    FAILS(HDI_ERR_ARG, hdi_server_submit(NULL, &req, &ticket));
    FAILS(HDI_ERR_ARG, hdi_server_poll(NULL, 1, &done, NULL));
    FAILS(HDI_ERR_ARG, hdi_server_drain(NULL));
    hdi_server_destroy(NULL);
    CHECK(hdi_server_create(NULL, 0, 4, 1, 0) == NULL);

    int64_t launches = 0;
    double lds = 0.0;
    FAILS(HDI_ERR_ARG, hdi_stats_get(HDI_NUM_KERNEL_IDS, &launches, NULL, NULL, NULL));
    FAILS(HDI_ERR_ARG, hdi_stats_get_lds(-1, &lds));
    hdi_stats_reset();
    CHECK(hdi_stats_get(0, &launches, NULL, NULL, NULL) == HDI_OK && launches == 0);
}

/* the last error is per thread */
static void *other_thread(void *arg) {
    hdi_solve_report rep;
    (void)arg;
    int32_t st = inpaint_solve((hdi_image){40, 30, 2}, DEV, DEV, DEV, NULL, DEV, 0, NULL, &rep, NULL);
    return (void *)(size_t)(st == HDI_ERR_ARG && strstr(hdi_last_error(), "bad image shape") != NULL);
}

static void thread_local_errors(void) {
    hdi_solve_report rep;
    const hdi_image img = {40, 30, 1};
    CHECK(inpaint_solve(img, NULL, DEV, DEV, NULL, DEV, 0, NULL, &rep, NULL) == HDI_ERR_ARG);
    char mine[256];
    snprintf(mine, sizeof mine, "%s", hdi_last_error());
    pthread_t th;
    void *ok = NULL;
    CHECK(pthread_create(&th, NULL, other_thread, NULL) == 0);
    CHECK(pthread_join(th, &ok) == 0);
    CHECK(ok != NULL);
    CHECK(strcmp(mine, hdi_last_error()) == 0);
    CHECK(strstr(mine, "non-null") != NULL);
}

int main(void) {
    strings();
    geometry();
    sizes();
    argument_errors();
    thread_local_errors();
    if (g_fail) {
        printf("abi host: %d checks failed\n", g_fail);
        return 1;
    }
    printf("abi host: ok\n");
    return 0;
}
