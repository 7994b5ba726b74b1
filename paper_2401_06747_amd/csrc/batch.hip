// Batched inpainting solves: many images of uneven size per launch, joining and
// leaving between refinement rounds.
//
// Every image keeps its own multigrid hierarchy, tolerance and refinement
// rounds; what is shared is the launch. For each phase of the solve (mask
// pyramid, reduced FMG start, FP64 residual, each level of the V-cycle) one
// kernel launch covers the blocks of all images that take part; a small
// segment table per launch tells each workgroup which image and level it
// serves. The block functions are the ones the single-image kernels use and
// every reduction keeps its per-image order, so an image's result is
// bit-for-bit the same alone, in any batch, and through inpaint_solve with the
// same parameters.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "engine.h"

namespace hdi {

#define B_TRY(expr)                                                                                  \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) {                                                                      \
            set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__);   \
            return HDI_ERR_HIP;                                                                      \
        }                                                                                            \
    } while (0)

static constexpr int POINTS = 1 << 30;          // segment unit of point (256-pixel chunk) phases
static constexpr int ADMIT_PHASES = 7 * MAX_LEVELS + 2;   // smoothing phases split by block size
static constexpr int RES_PHASES = 3;
static constexpr int VC_PHASES = 7 * MAX_LEVELS;

__global__ void kb_zero_counts(int n, unsigned int *c) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = 0u;
}

BPhase Engine::SegList::begin(const int4 *dev_base) const { return BPhase{dev_base + v.size(), 0, 0}; }

void Engine::SegList::add(BPhase &ph, int img, int lev, long count, int unit) {
    if (count <= 0) return;
    v.push_back(make_int4(img, lev, ph.n, unit));
    ph.nseg += 1;
    ph.n += (int)count;
}

bool Engine::plan(Arena &a, int max_slots) {
    nslots_ = max_slots;
    d_lev_ = (BLev *)a.take(sizeof(BLev) * max_slots * MAX_LEVELS);
    d_img_ = (BImg *)a.take(sizeof(BImg) * max_slots);
    d_flags_ = (uint8_t *)a.take(max_slots);
    d_counts_ = (unsigned int *)a.take(sizeof(unsigned int) * max_slots * MAX_LEVELS);
    d_norms_ = (double *)a.take(sizeof(double) * max_slots * 6);
    seg_cap_admit_ = (size_t)ADMIT_PHASES * max_slots;
    seg_cap_res_ = (size_t)RES_PHASES * max_slots;
    seg_cap_vc_ = (size_t)VC_PHASES * max_slots;
    d_seg_admit_ = (int4 *)a.take(sizeof(int4) * seg_cap_admit_);
    d_seg_res_ = (int4 *)a.take(sizeof(int4) * seg_cap_res_);
    d_seg_vc_ = (int4 *)a.take(sizeof(int4) * seg_cap_vc_);
    slot_.assign(max_slots, nullptr);
    h_lev_.assign((size_t)max_slots * MAX_LEVELS, BLev{});
    h_img_.assign(max_slots, BImg{});
    h_flags_.assign(max_slots, 0);
    h_counts_.assign((size_t)max_slots * MAX_LEVELS, 0);
    h_norms_.assign((size_t)max_slots * 6, 0.0);
    return a.base == nullptr || a.used <= a.size;
}

std::vector<int> Engine::free_slots() const {
    std::vector<int> out;
    for (int i = 0; i < nslots_; ++i)
        if (!slot_[i]) out.push_back(i);
    return out;
}

void Engine::abort_all(std::vector<EJob *> &ended) {
    for (EJob *&j : slot_)
        if (j) {
            ended.push_back(j);
            j = nullptr;
        }
}

int Engine::running() const {
    int n = 0;
    for (EJob *j : slot_) n += j != nullptr;
    return n;
}

// Host copy of the descriptors of one job's slot.
void Engine::describe(const EJob &j) {
    const Hierarchy &h = j.h;
    const int i = j.slot;
    for (int l = 0; l < MAX_LEVELS; ++l) h_lev_[(size_t)i * MAX_LEVELS + l] = BLev{};
    for (int l = 0; l < h.nlev_full; ++l) {
        const Level &L = h.lev[l];
        BLev &d = h_lev_[(size_t)i * MAX_LEVELS + l];
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
    BImg &m = h_img_[i];
    m = BImg{};
    m.W = j.job.img.width;
    m.H = j.job.img.height;
    m.C = j.job.img.channels;
    m.nlev = h.nlev;
    m.local_iters = j.cfg.local_iters;
    m.mid_iters = j.cfg.mid_iters;
    m.coarse_iters = j.cfg.coarse_iters;
    m.robin = j.cfg.robin;
    m.local_stop = j.cfg.local_stop;
    m.kind = j.kind;
    m.warm = j.warm ? 1 : 0;
    m.data_d = j.data_d;
    m.src = j.src;
    const dim3 g = residual_grid(m.W, m.H);
    m.gx = (int)g.x;
    m.nblk = h.nblk;
    m.mask = j.job.mask;
    m.f = j.job.f;
    m.u = j.job.out;
    m.u_alt = h.u_alt;
    m.partials = h.partials;
    m.norms = d_norms_ + (size_t)i * 6;
    m.counts = d_counts_ + (size_t)i * MAX_LEVELS;
}

// The descriptors of the slots lo..hi in two copies (each small copy from
// host memory costs the host tens of microseconds, so the slots of a whole
// admission go together; slots in between that are running hold the same
// descriptors on both sides).
int32_t Engine::upload_desc(int lo, int hi, hipStream_t s) {
    if (lo > hi) return HDI_OK;
    const size_t n = (size_t)(hi - lo + 1);
    B_TRY(hipMemcpyAsync(d_lev_ + (size_t)lo * MAX_LEVELS, &h_lev_[(size_t)lo * MAX_LEVELS],
                         sizeof(BLev) * MAX_LEVELS * n, hipMemcpyHostToDevice, s));
    B_TRY(hipMemcpyAsync(d_img_ + lo, &h_img_[lo], sizeof(BImg) * n, hipMemcpyHostToDevice, s));
    return HDI_OK;
}

int32_t Engine::admit(const std::vector<EJob *> &news, std::vector<EJob *> &ended, hipStream_t s) {
    if (news.empty()) return HDI_OK;
    int maxL = 0;
    for (EJob *j : news) {
        if (j->slot < 0 || j->slot >= nslots_ || slot_[j->slot]) {
            set_error("internal: bad engine slot %d", j->slot);
            return HDI_ERR_ARG;
        }
        slot_[j->slot] = j;
        j->h.nlev = j->h.nlev_full;
        j->rounds = 0;
        j->status = HDI_OK;
        j->where = 0;
        maxL = std::max(maxL, j->h.nlev_full);
        describe(*j);
    }
    {
        int lo = nslots_, hi = -1;
        for (EJob *j : news) { lo = std::min(lo, j->slot); hi = std::max(hi, j->slot); }
        const int32_t st = upload_desc(lo, hi, s);
        if (st) return st;
    }
    hipLaunchKernelGGL(kb_zero_counts, dim3((nslots_ * MAX_LEVELS + 255) / 256), dim3(256), 0, s,
                       nslots_ * MAX_LEVELS, d_counts_);

    // 1. coarse masks and known counts, level by level
    seg_admit_.v.clear();
    std::vector<BPhase> cnt(maxL);
    for (int l = 0; l < maxL; ++l) {
        cnt[l] = seg_admit_.begin(d_seg_admit_);
        for (EJob *j : news) {
            if (l >= j->h.nlev_full) continue;
            const long N = (long)j->h.lev[l].W * j->h.lev[l].H;
            seg_admit_.add(cnt[l], j->slot, l, std::min<long>((N + 255) / 256, 1024), POINTS);
        }
    }
    B_TRY(hipMemcpyAsync(d_seg_admit_, seg_admit_.v.data(), sizeof(int4) * seg_admit_.v.size(),
                         hipMemcpyHostToDevice, s));
    for (int l = 0; l < maxL; ++l) launch_b_count(cnt[l], d_lev_, d_img_, s);
    B_TRY(hipGetLastError());
    B_TRY(hipMemcpyAsync(h_counts_.data(), d_counts_, sizeof(unsigned int) * h_counts_.size(), hipMemcpyDeviceToHost,
                         s));
    B_TRY(wait_for(s));

    // 2. levels in use: the same rule as the single-image solve
    std::vector<EJob *> go;
    for (EJob *j : news) {
        Hierarchy &h = j->h;
        for (int l = 0; l < MAX_LEVELS; ++l) h.known[l] = h_counts_[(size_t)j->slot * MAX_LEVELS + l];
        if (h.known[0] == 0) {
            j->status = HDI_ERR_EMPTY_MASK;
            slot_[j->slot] = nullptr;
            ended.push_back(j);
            continue;
        }
        h.nlev = h.nlev_full;
        for (int l = 1; l < h.nlev_full; ++l) {
            const double N = (double)h.lev[l].W * h.lev[l].H;
            if (N - (double)h.known[l] <= 0.01 * N) {
                h.nlev = l + 1;
                break;
            }
        }
        describe(*j);
        go.push_back(j);
    }
    if (go.empty()) return HDI_OK;
    {
        int lo = nslots_, hi = -1;
        for (EJob *j : go) { lo = std::min(lo, j->slot); hi = std::max(hi, j->slot); }
        const int32_t st = upload_desc(lo, hi, s);
        if (st) return st;
    }

    // 3. starting iterate: the data on the mask, and elsewhere the reduced FMG
    // (Sec. 3.2) for cold data problems, the caller's start for warm ones, 0
    // otherwise
    seg_admit_.v.clear();
    auto fmg = [](const EJob *j) {
        return !(j->cfg.flags & HDI_FLAG_NO_FMG) && !j->warm && j->kind != EK_SRC_F64;
    };
    auto chunks = [](const Level &L) { return ((long)L.W * L.H + 255) / 256; };
    auto tiles = [](const Level &L) { return (long)L.bx.count * L.by.count; };
    BPhase init_u = seg_admit_.begin(d_seg_admit_);
    for (EJob *j : go) seg_admit_.add(init_u, j->slot, 0, chunks(j->h.lev[0]), POINTS);
    // smoothing phases come in one launch per block size (index 0: 32x32, 1: 16x16)
    auto ti = [](const Level &L) { return L.tile == TILE_SMALL ? 1 : 0; };
    std::vector<BPhase> drestrict(maxL), fmg_prolong(maxL), fmg_coarse(2 * maxL), fmg_smooth(2 * maxL);
    for (int l = 0; l + 1 < maxL; ++l) {   // data restriction l -> l+1
        drestrict[l] = seg_admit_.begin(d_seg_admit_);
        for (EJob *j : go)
            if (fmg(j) && l + 1 < j->h.nlev) seg_admit_.add(drestrict[l], j->slot, l, chunks(j->h.lev[l + 1]), POINTS);
    }
    for (int l = 1; l < maxL; ++l) {
        for (int tv = 0; tv < 2; ++tv) {
            fmg_coarse[2 * l + tv] = seg_admit_.begin(d_seg_admit_);
            for (EJob *j : go)
                if (fmg(j) && j->h.nlev > 1 && l == j->h.nlev - 1 && ti(j->h.lev[l]) == tv)
                    seg_admit_.add(fmg_coarse[2 * l + tv], j->slot, l, tiles(j->h.lev[l]) * j->h.C,
                                   (int)tiles(j->h.lev[l]));
        }
        fmg_prolong[l] = seg_admit_.begin(d_seg_admit_);
        for (EJob *j : go)
            if (fmg(j) && l < j->h.nlev - 1) seg_admit_.add(fmg_prolong[l], j->slot, l, chunks(j->h.lev[l]), POINTS);
        for (int tv = 0; tv < 2; ++tv) {
            fmg_smooth[2 * l + tv] = seg_admit_.begin(d_seg_admit_);
            for (EJob *j : go)
                if (fmg(j) && l < j->h.nlev - 1 && ti(j->h.lev[l]) == tv)
                    seg_admit_.add(fmg_smooth[2 * l + tv], j->slot, l, tiles(j->h.lev[l]) * j->h.C,
                                   (int)tiles(j->h.lev[l]));
        }
    }
    BPhase prolong0 = seg_admit_.begin(d_seg_admit_);
    for (EJob *j : go)
        if (fmg(j) && j->h.nlev > 1) seg_admit_.add(prolong0, j->slot, 0, chunks(j->h.lev[0]), POINTS);
    if (seg_admit_.v.size() > seg_cap_admit_) {
        set_error("internal: %zu segments exceed the planned %zu", seg_admit_.v.size(), seg_cap_admit_);
        return HDI_ERR_WORKSPACE;
    }
    B_TRY(hipMemcpyAsync(d_seg_admit_, seg_admit_.v.data(), sizeof(int4) * seg_admit_.v.size(),
                         hipMemcpyHostToDevice, s));
    launch_b_init_u(init_u, d_img_, s);
    for (int l = 0; l + 1 < maxL; ++l) launch_b_data_restrict(l == 0, drestrict[l], d_lev_, d_img_, s);
    const int tile_of[2] = {TILE, TILE_SMALL};
    for (int l = maxL - 1; l >= 1; --l) {
        for (int tv = 0; tv < 2; ++tv) launch_b_schwarz(2, true, tile_of[tv], fmg_coarse[2 * l + tv], d_lev_, d_img_, s);
        launch_b_fmg_prolong(fmg_prolong[l], d_lev_, d_img_, s);
        for (int tv = 0; tv < 2; ++tv) launch_b_schwarz(2, false, tile_of[tv], fmg_smooth[2 * l + tv], d_lev_, d_img_, s);
    }
    launch_b_fmg_prolong0(prolong0, d_lev_, d_img_, s);
    B_TRY(hipGetLastError());
    return HDI_OK;
}

int32_t Engine::round(std::vector<EJob *> &ended, hipStream_t s) {
    std::vector<EJob *> run;
    for (EJob *j : slot_)
        if (j) run.push_back(j);
    if (run.empty()) return HDI_OK;

    // 1. FP64 residual (and, after a V-cycle, the fused update) of every job
    seg_res_.v.clear();
    BPhase res[2];
    for (int k = 0; k < 2; ++k) {
        const int C = k == 0 ? 1 : 3;
        res[k] = seg_res_.begin(d_seg_res_);
        for (EJob *j : run) {
            if (j->h.C != C) continue;
            const dim3 g = residual_grid(j->job.img.width, j->job.img.height);
            seg_res_.add(res[k], j->slot, 0, (long)g.x * g.y, (int)g.x);
        }
    }
    BPhase red = seg_res_.begin(d_seg_res_);
    for (EJob *j : run) seg_res_.add(red, j->slot, 0, j->h.C, POINTS);
    for (EJob *j : run) {
        const int r = j->rounds;
        h_flags_[j->slot] = (uint8_t)(1 | (r > 0 ? 2 : 0) | ((r > 0 && r % 2 == 0) ? 4 : 0));
    }
    B_TRY(hipMemcpyAsync(d_seg_res_, seg_res_.v.data(), sizeof(int4) * seg_res_.v.size(), hipMemcpyHostToDevice, s));
    B_TRY(hipMemcpyAsync(d_flags_, h_flags_.data(), nslots_, hipMemcpyHostToDevice, s));
    for (int k = 0; k < 2; ++k) launch_b_residual(res[k], k == 0 ? 1 : 3, d_img_, d_flags_, d_lev_, s);
    launch_b_reduce(red, d_img_, s);
    B_TRY(hipGetLastError());
    B_TRY(read_to_host(h_norms_.data(), d_norms_, sizeof(double) * h_norms_.size(), s));

    // 2. per-job decision
    std::vector<EJob *> go;
    for (EJob *j : run) {
        const int r = j->rounds;
        // where the residual's iterate lives: u after round 0 and after even
        // rounds, u_alt after odd ones
        j->where = (r % 2 == 1) ? 1 : 0;
        double worst = 0.0;
        bool finite = true;
        for (int c = 0; c < j->h.C; ++c) {
            const double rr = h_norms_[(size_t)j->slot * 6 + 2 * c], bb = h_norms_[(size_t)j->slot * 6 + 2 * c + 1];
            finite = finite && std::isfinite(rr) && std::isfinite(bb);
            j->rel[c] = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
            worst = std::fmax(worst, j->rel[c]);
        }
        bool stop = true;
        if (!finite)
            j->status = HDI_ERR_ARG;
        else if (worst <= j->cfg.rel_tol)
            j->status = HDI_OK;
        else if (r >= j->cfg.max_outer)
            j->status = HDI_ERR_NO_CONVERGENCE;
        else
            stop = false;
        if (!stop) {
            go.push_back(j);
            continue;
        }
        // iterates that ended in the workspace copy go back to the caller's u
        if (j->where == 1)
            B_TRY(hipMemcpyAsync(j->job.out, j->h.u_alt,
                                 sizeof(double) * j->h.C * j->job.img.width * j->job.img.height,
                                 hipMemcpyDeviceToDevice, s));
        slot_[j->slot] = nullptr;
        ended.push_back(j);
    }
    if (go.empty()) return HDI_OK;

    // 3. one V-cycle for the jobs that go on
    int maxL = 0;
    for (EJob *j : go) maxL = std::max(maxL, j->h.nlev);
    seg_vc_.v.clear();
    // smoothing phases come in one launch per block size (index 0: 32x32, 1: 16x16)
    std::vector<BPhase> pre(2 * maxL), coarsest(2 * maxL), restr(maxL), post(2 * maxL);
    for (int l = 0; l < maxL; ++l) {
        auto tiles = [&](BPhase &ph, bool above_coarsest, int tile) {
            for (EJob *j : go)
                if ((above_coarsest ? l < j->h.nlev - 1 : l == j->h.nlev - 1) && j->h.lev[l].tile == tile) {
                    const Level &L = j->h.lev[l];
                    const long nt = (long)L.bx.count * L.by.count;
                    seg_vc_.add(ph, j->slot, l, nt * j->h.C, (int)nt);
                }
        };
        for (int tv = 0; tv < 2; ++tv) {
            const int tile = tv ? TILE_SMALL : TILE;
            pre[2 * l + tv] = seg_vc_.begin(d_seg_vc_);
            tiles(pre[2 * l + tv], true, tile);
            coarsest[2 * l + tv] = seg_vc_.begin(d_seg_vc_);
            tiles(coarsest[2 * l + tv], false, tile);
            post[2 * l + tv] = seg_vc_.begin(d_seg_vc_);
            tiles(post[2 * l + tv], true, tile);
        }
        restr[l] = seg_vc_.begin(d_seg_vc_);
        for (EJob *j : go)
            if (l < j->h.nlev - 1)
                seg_vc_.add(restr[l], j->slot, l, ((long)j->h.lev[l + 1].W * j->h.lev[l + 1].H + 255) / 256, POINTS);
    }
    B_TRY(hipMemcpyAsync(d_seg_vc_, seg_vc_.v.data(), sizeof(int4) * seg_vc_.v.size(), hipMemcpyHostToDevice, s));
    const int tile_of[2] = {TILE, TILE_SMALL};
    for (int l = 0; l < maxL; ++l) {
        for (int tv = 0; tv < 2; ++tv) {
            launch_b_schwarz(0, false, tile_of[tv], pre[2 * l + tv], d_lev_, d_img_, s);
            launch_b_schwarz(0, true, tile_of[tv], coarsest[2 * l + tv], d_lev_, d_img_, s);
        }
        launch_b_restrict(restr[l], d_lev_, d_img_, s);
    }
    for (int l = maxL - 2; l >= 0; --l)
        for (int tv = 0; tv < 2; ++tv) launch_b_schwarz(1, false, tile_of[tv], post[2 * l + tv], d_lev_, d_img_, s);
    B_TRY(hipGetLastError());
    for (EJob *j : go) j->rounds += 1;
    return HDI_OK;
}

// Workspace layout of hdi_solve_batch: engine tables for n slots, then the
// hierarchies of the jobs in order.
static bool plan_batch(Engine &e, std::vector<EJob> &jobs, Arena &a) {
    if (!e.plan(a, (int)jobs.size())) return false;
    for (EJob &j : jobs)
        if (!plan_hierarchy(j.h, a, j.job.img.width, j.job.img.height, j.job.img.channels, j.overlap, j.job.mask,
                            j.cfg.small_from))
            return false;
    return true;
}

}  // namespace hdi

using namespace hdi;

extern "C" {

size_t hdi_batch_workspace_bytes(int32_t n, const hdi_job *jobs) {
    if (n < 1 || !jobs) return 0;
    std::vector<EJob> ej(n);
    bool tonal = false;
    for (int i = 0; i < n; ++i) {
        if (jobs[i].img.width < 1 || jobs[i].img.height < 1 || (jobs[i].img.channels != 1 && jobs[i].img.channels != 3))
            return 0;
        if (jobs[i].kind != HDI_JOB_INPAINT && jobs[i].kind != HDI_JOB_TONAL) return 0;
        tonal = tonal || jobs[i].kind == HDI_JOB_TONAL;
        ej[i].job = jobs[i];
    }
    if (tonal) return batch_served_bytes(n, jobs);
    Engine e;
    Arena a{nullptr, 0, 0};
    plan_batch(e, ej, a);
    return a.used + 256;
}

int32_t hdi_solve_batch(int32_t n, const hdi_job *jobs, void *ws, size_t ws_bytes, const hdi_solve_params *params,
                        hdi_solve_report *reports, void *stream) {
    if (n < 1 || !jobs) {
        set_error("need n >= 1 jobs");
        return HDI_ERR_ARG;
    }
    std::vector<EJob> ej(n);
    bool tonal = false;
    for (int i = 0; i < n; ++i) {
        if (!check_image(jobs[i].img)) return HDI_ERR_ARG;
        if (jobs[i].kind != HDI_JOB_INPAINT && jobs[i].kind != HDI_JOB_TONAL) {
            set_error("job %d: kind %d is neither HDI_JOB_INPAINT nor HDI_JOB_TONAL", i, jobs[i].kind);
            return HDI_ERR_ARG;
        }
        if (!jobs[i].mask || !jobs[i].f || !jobs[i].out) {
            set_error("job %d: mask, f and out must be non-null device pointers", i);
            return HDI_ERR_ARG;
        }
        int32_t st = fill_cfg(params ? &params[i] : nullptr, ej[i].cfg, ej[i].overlap);
        if (st) return st;
        if (ej[i].cfg.flags & HDI_FLAG_CG) {
            set_error("job %d: batches run the multigrid solver only (HDI_FLAG_CG is for single solves)", i);
            return HDI_ERR_ARG;
        }
        if (jobs[i].kind == HDI_JOB_TONAL) {
            TonalCfg tc;
            SolveCfg inner;
            int ov = 0;
            st = fill_tonal_cfg(jobs[i].tonal, tc, inner, ov);
            if (st) return st;
            if (inner.flags & HDI_FLAG_CG) {
                set_error("job %d: batches run the multigrid solver only (HDI_FLAG_CG is for single solves)", i);
                return HDI_ERR_ARG;
            }
            tonal = true;
        }
        ej[i].job = jobs[i];
        ej[i].slot = i;
    }
    const size_t need = hdi_batch_workspace_bytes(n, jobs);
    if (!ws || ws_bytes < need) {
        set_error("workspace of %zu bytes given, %zu needed", ws ? ws_bytes : (size_t)0, need);
        return HDI_ERR_WORKSPACE;
    }
    hipStream_t s = (hipStream_t)stream;
    if (tonal) return solve_batch_served(n, jobs, ws, ws_bytes, params, reports, s);
    Arena a{(char *)ws, ws_bytes, 0};
    Engine e;
    plan_batch(e, ej, a);
    CallTimer tm;
    B_TRY(tm.start(s));
    std::vector<EJob *> news, ended;
    for (EJob &j : ej) news.push_back(&j);
    int32_t st = e.admit(news, ended, s);
    while (st == HDI_OK && e.running() > 0) st = e.round(ended, s);
    float ms = 0.f;
    B_TRY(tm.stop(s, &ms));
    if (st) return st;
    int32_t worst = HDI_OK;
    for (int i = 0; i < n; ++i) {
        const EJob &j = ej[i];
        if (reports) {
            for (int c = 0; c < 3; ++c) reports[i].rel_residual[c] = c < j.h.C ? j.rel[c] : 0.0;
            reports[i].outer_iters = j.rounds;
            reports[i].vcycles = j.rounds;
            reports[i].ms = ms;
        }
        if (j.status != HDI_OK && worst == HDI_OK) {
            worst = j.status;
            set_error("job %d: %s", i,
                      j.status == HDI_ERR_NO_CONVERGENCE ? "no convergence"
                      : j.status == HDI_ERR_EMPTY_MASK   ? "empty mask (the inpainting matrix is singular)"
                                                          : "non-finite residual");
        }
    }
    return worst;
}

}  // extern "C"
