// Batched inpainting solves: many images of uneven size per launch.
//
// Every image keeps its own multigrid hierarchy, tolerance and refinement
// rounds; what is shared is the launch. For each phase of the solve (mask
// pyramid, reduced FMG start, FP64 residual, each level of the V-cycle) one
// kernel launch covers the work items (image, level, block) of all images that
// take part, and per-image descriptor tables tell each workgroup which image
// and level it serves. The block functions are the ones the single-image
// kernels use and every reduction keeps its per-image order, so an image's
// result is bit-for-bit the same alone, in any batch, and through
// inpaint_solve with the same parameters.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "hdi_internal.h"

namespace hdi {

bool check_image(const hdi_image &img);
int32_t fill_cfg(const hdi_solve_params *p, SolveCfg &cfg, int &overlap);

#define B_TRY(expr)                                                                                  \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) {                                                                      \
            set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__);   \
            return HDI_ERR_HIP;                                                                      \
        }                                                                                            \
    } while (0)

struct BatchPlan {
    std::vector<Hierarchy> h;
    BLev *d_lev;
    BImg *d_img;
    uint8_t *d_active;
    unsigned int *d_counts;   // [n][MAX_LEVELS]
    double *d_norms;          // [n][6]
    int4 *d_items;
    size_t max_items;
};

static size_t tiles_of(const Level &L) { return (size_t)L.bx.count * L.by.count; }

// Upper bound of the work items one call can create (full hierarchies).
static size_t item_bound(const std::vector<Hierarchy> &hs) {
    size_t n = 0;
    for (const Hierarchy &h : hs) {
        const size_t N = (size_t)h.lev[0].W * h.lev[0].H;
        n += 2 * ((N + 255) / 256) + 1024 * MAX_LEVELS;     // init_u, prolong0, counts
        n += (size_t)h.nblk + h.C;                           // residual, reduce
        for (int l = 0; l < h.nlev_full; ++l) {
            const size_t Nl = (size_t)h.lev[l].W * h.lev[l].H;
            n += 4 * tiles_of(h.lev[l]) * h.C;               // pre, post, coarsest, FMG smoothing
            n += 3 * ((Nl + 255) / 256);                     // restrict, data restrict, FMG prolong
        }
    }
    return n;
}

// overlaps: per-job block overlap (nullptr: the largest valid overlap, whose
// smallest block stride gives the most blocks and so bounds any choice)
static bool plan_batch(BatchPlan &b, Arena &a, int n, const hdi_job *jobs, const int *overlaps) {
    b.h.assign(n, Hierarchy());
    for (int i = 0; i < n; ++i)
        if (!plan_hierarchy(b.h[i], a, jobs[i].img.width, jobs[i].img.height, jobs[i].img.channels,
                            overlaps ? overlaps[i] : 16, jobs[i].mask))
            return false;
    b.d_lev = (BLev *)a.take(sizeof(BLev) * n * MAX_LEVELS);
    b.d_img = (BImg *)a.take(sizeof(BImg) * n);
    b.d_active = (uint8_t *)a.take(n);
    b.d_counts = (unsigned int *)a.take(sizeof(unsigned int) * n * MAX_LEVELS);
    b.d_norms = (double *)a.take(sizeof(double) * n * 6);
    b.max_items = item_bound(b.h);
    b.d_items = (int4 *)a.take(sizeof(int4) * b.max_items);
    return a.base == nullptr || a.used <= a.size;
}

__global__ void kb_zero_counts(int n, unsigned int *c) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = 0u;
}

// A list of work items inside the uploaded item buffer.
struct Span { size_t off = 0; int n = 0; };

struct ItemBuilder {
    std::vector<int4> v;
    Span begin() { Span s; s.off = v.size(); return s; }
    void end(Span &s) { s.n = (int)(v.size() - s.off); }
    void points(int img, int lev, size_t count) {
        for (size_t k = 0; k < (count + 255) / 256; ++k) v.push_back(make_int4(img, lev, (int)k, 0));
    }
    void tiles(int img, int lev, const Level &L, int C) {
        for (int c = 0; c < C; ++c)
            for (int t = 0; t < L.bx.count * L.by.count; ++t) v.push_back(make_int4(img, lev, t, c));
    }
};

static void fill_tables(const BatchPlan &b, int n, const hdi_job *jobs, const std::vector<SolveCfg> &cfg,
                        std::vector<BLev> &lev, std::vector<BImg> &img) {
    lev.assign((size_t)n * MAX_LEVELS, BLev{});
    img.assign(n, BImg{});
    for (int i = 0; i < n; ++i) {
        const Hierarchy &h = b.h[i];
        for (int l = 0; l < h.nlev; ++l) {
            const Level &L = h.lev[l];
            BLev &d = lev[(size_t)i * MAX_LEVELS + l];
            d.W = L.W;
            d.H = L.H;
            d.ntx = L.bx.count;
            d.nty = L.by.count;
            d.sx = L.bx.stride;
            d.sy = L.by.stride;
            d.mask = L.mask;
            d.r = L.r;
            d.ea = L.ea;
            d.eb = L.eb;
            d.aux = L.aux;
            if (l + 1 < h.nlev_full) {
                const Level &Lc = h.lev[l + 1];
                d.Wc = Lc.W;
                d.Hc = Lc.H;
                d.mask_c = Lc.mask;
                d.r_c = Lc.r;
                d.aux_c = Lc.aux;
                // the coarser level's final correction: its smoothing output if it
                // is the coarsest level in use, its post-smoothing output otherwise
                d.ec = (l + 1 == h.nlev - 1) ? Lc.ea : Lc.eb;
            }
        }
        BImg &m = img[i];
        m.W = jobs[i].img.width;
        m.H = jobs[i].img.height;
        m.C = jobs[i].img.channels;
        m.nlev = h.nlev;
        m.local_iters = cfg[i].local_iters;
        m.coarse_iters = cfg[i].coarse_iters;
        const dim3 g = residual_grid(m.W, m.H);
        m.gx = (int)g.x;
        m.nblk = h.nblk;
        m.mask = jobs[i].mask;
        m.f = jobs[i].f;
        m.u = jobs[i].u;
        m.u_alt = h.u_alt;
        m.partials = h.partials;
        m.norms = b.d_norms + (size_t)i * 6;
        m.counts = b.d_counts + (size_t)i * MAX_LEVELS;
    }
}

static int32_t run_batch(BatchPlan &b, int n, const hdi_job *jobs, const std::vector<SolveCfg> &cfg,
                         hdi_solve_report *reports, hipStream_t s) {
    std::vector<BLev> lev;
    std::vector<BImg> img;
    int maxL = 0;
    for (int i = 0; i < n; ++i) maxL = std::max(maxL, b.h[i].nlev_full);
    // 1. mask pyramids and per-level counts, level by level across the batch
    fill_tables(b, n, jobs, cfg, lev, img);
    B_TRY(hipMemcpyAsync(b.d_lev, lev.data(), sizeof(BLev) * lev.size(), hipMemcpyHostToDevice, s));
    B_TRY(hipMemcpyAsync(b.d_img, img.data(), sizeof(BImg) * n, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(kb_zero_counts, dim3((n * MAX_LEVELS + 255) / 256), dim3(256), 0, s, n * MAX_LEVELS,
                       b.d_counts);
    {
        ItemBuilder ib;
        std::vector<Span> per_level(maxL);
        for (int l = 0; l < maxL; ++l) {
            per_level[l] = ib.begin();
            for (int i = 0; i < n; ++i) {
                const Hierarchy &h = b.h[i];
                if (l >= h.nlev_full) continue;
                const long cnt = (long)h.lev[l].W * h.lev[l].H;
                const int nb = (int)std::min<long>((cnt + 255) / 256, 1024);
                for (int k = 0; k < nb; ++k) ib.v.push_back(make_int4(i, l, k, nb));
            }
            ib.end(per_level[l]);
        }
        B_TRY(hipMemcpyAsync(b.d_items, ib.v.data(), sizeof(int4) * ib.v.size(), hipMemcpyHostToDevice, s));
        for (int l = 0; l < maxL; ++l)
            launch_b_count(b.d_items + per_level[l].off, per_level[l].n, b.d_lev, b.d_img, s);
        std::vector<unsigned int> counts((size_t)n * MAX_LEVELS);
        B_TRY(hipMemcpyAsync(counts.data(), b.d_counts, sizeof(unsigned int) * counts.size(),
                             hipMemcpyDeviceToHost, s));
        B_TRY(hipStreamSynchronize(s));
        for (int i = 0; i < n; ++i) {
            Hierarchy &h = b.h[i];
            for (int l = 0; l < MAX_LEVELS; ++l) h.known[l] = counts[(size_t)i * MAX_LEVELS + l];
            if (h.known[0] == 0) {
                set_error("job %d: empty mask (the inpainting matrix is singular)", i);
                return HDI_ERR_EMPTY_MASK;
            }
            // same level rule as the single-image solve
            h.nlev = h.nlev_full;
            for (int l = 1; l < h.nlev_full; ++l) {
                const double N = (double)h.lev[l].W * h.lev[l].H;
                if (N - (double)h.known[l] <= 0.01 * N) {
                    h.nlev = l + 1;
                    break;
                }
            }
        }
    }
    fill_tables(b, n, jobs, cfg, lev, img);
    B_TRY(hipMemcpyAsync(b.d_lev, lev.data(), sizeof(BLev) * lev.size(), hipMemcpyHostToDevice, s));
    B_TRY(hipMemcpyAsync(b.d_img, img.data(), sizeof(BImg) * n, hipMemcpyHostToDevice, s));

    // 2. work lists of every phase
    ItemBuilder ib;
    Span init_u = ib.begin();
    for (int i = 0; i < n; ++i) ib.points(i, 0, (size_t)img[i].W * img[i].H);
    ib.end(init_u);
    std::vector<Span> drestrict(maxL), fmg_coarse(maxL), fmg_prolong(maxL), fmg_smooth(maxL);
    for (int l = 0; l + 1 < maxL; ++l) {   // data restriction l -> l+1
        drestrict[l] = ib.begin();
        for (int i = 0; i < n; ++i)
            if (!(cfg[i].flags & HDI_FLAG_NO_FMG) && l + 1 < b.h[i].nlev)
                ib.points(i, l, (size_t)b.h[i].lev[l + 1].W * b.h[i].lev[l + 1].H);
        ib.end(drestrict[l]);
    }
    for (int l = 1; l < maxL; ++l) {
        fmg_coarse[l] = ib.begin();
        for (int i = 0; i < n; ++i)
            if (!(cfg[i].flags & HDI_FLAG_NO_FMG) && b.h[i].nlev > 1 && l == b.h[i].nlev - 1)
                ib.tiles(i, l, b.h[i].lev[l], img[i].C);
        ib.end(fmg_coarse[l]);
        fmg_prolong[l] = ib.begin();
        for (int i = 0; i < n; ++i)
            if (!(cfg[i].flags & HDI_FLAG_NO_FMG) && l < b.h[i].nlev - 1)
                ib.points(i, l, (size_t)b.h[i].lev[l].W * b.h[i].lev[l].H);
        ib.end(fmg_prolong[l]);
        fmg_smooth[l] = ib.begin();
        for (int i = 0; i < n; ++i)
            if (!(cfg[i].flags & HDI_FLAG_NO_FMG) && l < b.h[i].nlev - 1) ib.tiles(i, l, b.h[i].lev[l], img[i].C);
        ib.end(fmg_smooth[l]);
    }
    Span prolong0 = ib.begin();
    for (int i = 0; i < n; ++i)
        if (!(cfg[i].flags & HDI_FLAG_NO_FMG) && b.h[i].nlev > 1) ib.points(i, 0, (size_t)img[i].W * img[i].H);
    ib.end(prolong0);
    Span resid[2], reduce = ib.begin();
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < img[i].C; ++c) ib.v.push_back(make_int4(i, c, 0, 0));
    ib.end(reduce);
    for (int k = 0; k < 2; ++k) {
        const int C = k == 0 ? 1 : 3;
        resid[k] = ib.begin();
        for (int i = 0; i < n; ++i) {
            if (img[i].C != C) continue;
            const dim3 g = residual_grid(img[i].W, img[i].H);
            for (unsigned by = 0; by < g.y; ++by)
                for (unsigned bx = 0; bx < g.x; ++bx) ib.v.push_back(make_int4(i, (int)bx, (int)by, 0));
        }
        ib.end(resid[k]);
    }
    std::vector<Span> pre(maxL), coarsest(maxL), restr(maxL), post(maxL);
    for (int l = 0; l < maxL; ++l) {
        pre[l] = ib.begin();
        for (int i = 0; i < n; ++i)
            if (l < b.h[i].nlev - 1) ib.tiles(i, l, b.h[i].lev[l], img[i].C);
        ib.end(pre[l]);
        coarsest[l] = ib.begin();
        for (int i = 0; i < n; ++i)
            if (l == b.h[i].nlev - 1) ib.tiles(i, l, b.h[i].lev[l], img[i].C);
        ib.end(coarsest[l]);
        restr[l] = ib.begin();
        for (int i = 0; i < n; ++i)
            if (l < b.h[i].nlev - 1) ib.points(i, l, (size_t)b.h[i].lev[l + 1].W * b.h[i].lev[l + 1].H);
        ib.end(restr[l]);
        post[l] = ib.begin();
        for (int i = 0; i < n; ++i)
            if (l < b.h[i].nlev - 1) ib.tiles(i, l, b.h[i].lev[l], img[i].C);
        ib.end(post[l]);
    }
    if (ib.v.size() > b.max_items) {
        set_error("internal: %zu work items exceed the planned %zu", ib.v.size(), b.max_items);
        return HDI_ERR_WORKSPACE;
    }
    B_TRY(hipMemcpyAsync(b.d_items, ib.v.data(), sizeof(int4) * ib.v.size(), hipMemcpyHostToDevice, s));
    auto at = [&](const Span &sp) { return b.d_items + sp.off; };

    // 3. starting iterate: u = f on the mask, reduced FMG elsewhere (Sec. 3.2)
    std::vector<uint8_t> active(n, 1);
    B_TRY(hipMemcpyAsync(b.d_active, active.data(), n, hipMemcpyHostToDevice, s));
    hipEvent_t e0, e1;
    B_TRY(hipEventCreate(&e0));
    B_TRY(hipEventCreate(&e1));
    B_TRY(hipEventRecord(e0, s));
    launch_b_init_u(at(init_u), init_u.n, b.d_img, b.d_active, s);
    for (int l = 0; l + 1 < maxL; ++l)
        launch_b_data_restrict(l == 0, at(drestrict[l]), drestrict[l].n, b.d_lev, b.d_img, s);
    for (int l = maxL - 1; l >= 1; --l) {
        launch_b_schwarz(2, true, at(fmg_coarse[l]), fmg_coarse[l].n, b.d_lev, b.d_img, nullptr, s);
        launch_b_fmg_prolong(at(fmg_prolong[l]), fmg_prolong[l].n, b.d_lev, b.d_img, s);
        launch_b_schwarz(2, false, at(fmg_smooth[l]), fmg_smooth[l].n, b.d_lev, b.d_img, nullptr, s);
    }
    launch_b_fmg_prolong0(at(prolong0), prolong0.n, b.d_lev, b.d_img, s);
    B_TRY(hipGetLastError());

    // 4. refinement rounds, each image until its own tolerance
    std::vector<int> rounds(n, 0), status(n, HDI_OK), final_parity(n, 0);
    std::vector<double> rel((size_t)n * 3, 0.0), norms((size_t)n * 6);
    int round = 0;
    int nactive = n;
    for (;;) {
        const int parity = (round > 0 && round % 2 == 0) ? 1 : 0;
        for (int k = 0; k < 2; ++k)
            launch_b_residual(at(resid[k]), resid[k].n, k == 0 ? 1 : 3, b.d_img, b.d_active, round > 0, parity,
                              b.d_lev, s);
        launch_b_reduce(at(reduce), reduce.n, b.d_img, b.d_active, s);
        B_TRY(hipMemcpyAsync(norms.data(), b.d_norms, sizeof(double) * norms.size(), hipMemcpyDeviceToHost, s));
        B_TRY(hipStreamSynchronize(s));
        // where this round's iterate lives: u for round 0, else the residual's output
        const int where = round == 0 ? 0 : (parity ? 0 : 1);
        for (int i = 0; i < n; ++i) {
            if (!active[i]) continue;
            final_parity[i] = where;
            double worst = 0.0;
            bool finite = true;
            for (int c = 0; c < img[i].C; ++c) {
                const double rr = norms[(size_t)i * 6 + 2 * c], bb = norms[(size_t)i * 6 + 2 * c + 1];
                finite = finite && std::isfinite(rr) && std::isfinite(bb);
                rel[(size_t)i * 3 + c] = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
                worst = std::fmax(worst, rel[(size_t)i * 3 + c]);
            }
            if (!finite) {
                status[i] = HDI_ERR_ARG;
                active[i] = 0;
            } else if (worst <= cfg[i].rel_tol) {
                active[i] = 0;
            } else if (rounds[i] >= cfg[i].max_outer) {
                status[i] = HDI_ERR_NO_CONVERGENCE;
                active[i] = 0;
            }
        }
        nactive = (int)std::count(active.begin(), active.end(), (uint8_t)1);
        if (nactive == 0) break;
        B_TRY(hipMemcpyAsync(b.d_active, active.data(), n, hipMemcpyHostToDevice, s));
        for (int l = 0; l < maxL; ++l) {
            launch_b_schwarz(0, false, at(pre[l]), pre[l].n, b.d_lev, b.d_img, b.d_active, s);
            launch_b_schwarz(0, true, at(coarsest[l]), coarsest[l].n, b.d_lev, b.d_img, b.d_active, s);
            launch_b_restrict(at(restr[l]), restr[l].n, b.d_lev, b.d_img, b.d_active, s);
        }
        for (int l = maxL - 2; l >= 0; --l)
            launch_b_schwarz(1, false, at(post[l]), post[l].n, b.d_lev, b.d_img, b.d_active, s);
        for (int i = 0; i < n; ++i) rounds[i] += active[i];
        ++round;
    }
    // iterates that ended in the workspace copy go back to the caller's u
    for (int i = 0; i < n; ++i)
        if (final_parity[i] == 1)
            B_TRY(hipMemcpyAsync(jobs[i].u, b.h[i].u_alt, sizeof(double) * img[i].C * img[i].W * img[i].H,
                                 hipMemcpyDeviceToDevice, s));
    B_TRY(hipGetLastError());
    B_TRY(hipEventRecord(e1, s));
    B_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    B_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int32_t worst_status = HDI_OK;
    for (int i = 0; i < n; ++i) {
        if (reports) {
            for (int c = 0; c < 3; ++c) reports[i].rel_residual[c] = c < img[i].C ? rel[(size_t)i * 3 + c] : 0.0;
            reports[i].outer_iters = rounds[i];
            reports[i].vcycles = rounds[i];
            reports[i].ms = ms;
        }
        if (status[i] != HDI_OK && worst_status == HDI_OK) {
            worst_status = status[i];
            set_error("job %d: %s", i, status[i] == HDI_ERR_NO_CONVERGENCE ? "no convergence" : "non-finite residual");
        }
    }
    return worst_status;
}

}  // namespace hdi

using namespace hdi;

extern "C" {

size_t hdi_batch_workspace_bytes(int32_t n, const hdi_job *jobs) {
    if (n < 1 || !jobs) return 0;
    for (int i = 0; i < n; ++i)
        if (jobs[i].img.width < 1 || jobs[i].img.height < 1 || (jobs[i].img.channels != 1 && jobs[i].img.channels != 3))
            return 0;
    BatchPlan b;
    Arena a{nullptr, 0, 0};
    plan_batch(b, a, n, jobs, nullptr);
    return a.used + 256;
}

int32_t hdi_solve_batch(int32_t n, const hdi_job *jobs, void *ws, size_t ws_bytes, const hdi_solve_params *params,
                        hdi_solve_report *reports, void *stream) {
    if (n < 1 || !jobs) {
        set_error("need n >= 1 jobs");
        return HDI_ERR_ARG;
    }
    std::vector<SolveCfg> cfg(n);
    std::vector<int> overlap(n, 4);
    for (int i = 0; i < n; ++i) {
        if (!check_image(jobs[i].img)) return HDI_ERR_ARG;
        if (!jobs[i].mask || !jobs[i].f || !jobs[i].u) {
            set_error("job %d: mask, f and u must be non-null device pointers", i);
            return HDI_ERR_ARG;
        }
        int32_t st = fill_cfg(params ? &params[i] : nullptr, cfg[i], overlap[i]);
        if (st) return st;
    }
    const size_t need = hdi_batch_workspace_bytes(n, jobs);
    if (!ws || ws_bytes < need) {
        set_error("workspace of %zu bytes given, %zu needed", ws ? ws_bytes : (size_t)0, need);
        return HDI_ERR_WORKSPACE;
    }
    Arena a{(char *)ws, ws_bytes, 0};
    BatchPlan b;
    plan_batch(b, a, n, jobs, overlap.data());
    return run_batch(b, n, jobs, cfg, reports, (hipStream_t)stream);
}

}  // extern "C"
