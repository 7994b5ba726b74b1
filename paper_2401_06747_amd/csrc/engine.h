// Continuous-batching engine of the inpainting solve.
//
// The engine holds up to max_slots images. Images join between refinement
// rounds (admit: mask pyramid, level choice, reduced FMG start) and leave when
// their own tolerance is met (round: one FP64 residual launch and, for the
// images that go on, one V-cycle, each phase one launch over every image). Each
// image keeps its own hierarchy, parameters and round count, so its result is
// bit-for-bit that of the single-image solve, whatever else is in the engine.
#pragma once

#include <vector>

#include "hdi_internal.h"

namespace hdi {

// One image in the engine. The caller owns it and its hierarchy memory.
// job.out receives the solution; kind says whether the right-hand side is the
// FP32 image job.f on the mask, an FP64 image data_d on the mask, or an FP64
// source src off it (EK_*); warm: job.out holds the start on unknown pixels.
struct EJob {
    hdi_job job{};
    int kind = EK_DATA_F32;
    const double *data_d = nullptr, *src = nullptr;
    bool warm = false;
    SolveCfg cfg{};
    int overlap = 4;
    Hierarchy h{};
    int slot = -1;
    int rounds = 0;          // V-cycles done
    int status = HDI_OK;
    int where = 0;           // 1: the last iterate is in h.u_alt
    double rel[3] = {0, 0, 0};
    void *user = nullptr;    // the caller's handle
};

class Engine {
public:
    // Device tables for max_slots images, taken from a (or only counted).
    bool plan(Arena &a, int max_slots);
    int max_slots() const { return nslots_; }
    std::vector<int> free_slots() const;
    int running() const;
    // Start the given jobs (slots assigned by the caller, hierarchies planned).
    // Jobs with an empty mask end at once with HDI_ERR_EMPTY_MASK and are
    // returned in `ended`; the others are running afterwards.
    int32_t admit(const std::vector<EJob *> &news, std::vector<EJob *> &ended, hipStream_t s);
    // One refinement round over every running job. Jobs that met their
    // tolerance, ran out of rounds or went non-finite are returned in `ended`
    // with their final iterate copied to job.out (enqueued on s, not waited for)
    // and their slots freed.
    int32_t round(std::vector<EJob *> &ended, hipStream_t s);
    // After a HIP failure: every running job leaves (returned in `ended`).
    void abort_all(std::vector<EJob *> &ended);

private:
    struct SegList {
        std::vector<int4> v;
        BPhase begin(const int4 *dev_base) const;
        void add(BPhase &ph, int img, int lev, long count, int unit);
    };
    void describe(const EJob &j);
    int32_t upload_desc(int lo, int hi, hipStream_t s);

    int nslots_ = 0;
    BLev *d_lev_ = nullptr;
    BImg *d_img_ = nullptr;
    uint8_t *d_flags_ = nullptr;
    unsigned int *d_counts_ = nullptr;
    double *d_norms_ = nullptr;
    int4 *d_seg_admit_ = nullptr, *d_seg_res_ = nullptr, *d_seg_vc_ = nullptr;
    size_t seg_cap_admit_ = 0, seg_cap_res_ = 0, seg_cap_vc_ = 0;
    std::vector<EJob *> slot_;
    std::vector<BLev> h_lev_;
    std::vector<BImg> h_img_;
    std::vector<uint8_t> h_flags_;
    std::vector<unsigned int> h_counts_;
    std::vector<double> h_norms_;
    SegList seg_admit_, seg_res_, seg_vc_;
};

int32_t fill_cfg(const hdi_solve_params *p, SolveCfg &cfg, int &overlap);

// Batches with tonal jobs run as the requests of a server over the batch
// workspace (server.hip): the workspace they need, and the run (arguments
// already checked; host-synchronous, after the work enqueued on s).
size_t batch_served_bytes(int n, const hdi_job *jobs);
int32_t solve_batch_served(int n, const hdi_job *jobs, void *ws, size_t ws_bytes, const hdi_solve_params *params,
                           hdi_solve_report *reports, hipStream_t s);

}  // namespace hdi
