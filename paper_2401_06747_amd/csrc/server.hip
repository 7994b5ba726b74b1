// Request loop with continuous batching over one device.
//
// Inpainting requests go through the batch engine: an engine thread admits
// waiting work between refinement rounds (as slots and arena memory free up),
// runs one round over everything running, and hands back the solves that met
// their tolerance. Each tonal request's outer iteration (Sec. 5) runs on a
// tonal worker thread and stream. Its inner solves (x = B g and the
// symmetrised solve of B^T) run on that stream too, overlapping the engine's
// rounds on the device, or, with HDI_SERVER_TONAL_SHARED, join the engine's
// shared rounds like inpainting requests do (events order the two streams).
// With HDI_SERVER_PLAIN one worker runs the requests one at a time through
// inpaint_solve and tonal_optimize: the one-request-per-launch control.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "engine.h"

namespace hdi {

struct Ticket {
    uint64_t id = 0;
    hdi_request req{};
    hdi_tonal_params tonal{};
    hdi_request_report rep{};
    hdi_tonal_report tonal_rep{};   // tonal requests: the full report
    std::string message;
    bool done = false;
    char *mem = nullptr;
    size_t bytes = 0;
    // the device buffers the request runs on (the caller's, or staged copies)
    const uint8_t *mask = nullptr;
    const float *f = nullptr;
    double *out = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    EJob ej;
    hipEvent_t ev = nullptr;
};

// An inner solve of a tonal request, waiting for or running in the engine.
// It lives on the tonal worker's stack until the engine thread marks it
// finished; the engine thread does not touch it afterwards.
struct EngineSolve {
    EJob ej;
    hipEvent_t ready = nullptr;   // recorded on the worker's stream: the inputs are written
    hipEvent_t done = nullptr;    // recorded on the compute stream when the solution is in place
    int max_running = 0;          // most solves sharing one round with it
    bool finished = false;
    int32_t status = HDI_OK;      // HDI_ERR_HIP if the engine failed
};

static size_t image_px(const hdi_image &img) { return (size_t)img.width * img.height; }

static size_t io_bytes(const hdi_request &r) {
    if (!(r.flags & HDI_REQ_HOST_IO)) return 0;
    const size_t N = image_px(r.img), C = r.img.channels;
    return up256(N) + up256(4 * C * N) + up256(8 * C * N);
}

static size_t work_bytes(const hdi_request &r) {
    return r.kind == HDI_REQ_TONAL ? hdi_tonal_workspace_bytes(r.img) : hdi_inpaint_workspace_bytes(r.img);
}

}  // namespace hdi

using namespace hdi;

struct hdi_server {
    int device = 0;
    int flags = 0;
    int max_slots = 0;
    Engine eng;
    ArenaAlloc alloc;
    hipStream_t compute = nullptr, copy = nullptr;
    std::vector<hipStream_t> tonal_streams;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Ticket *> q_inp, q_ton, q_all;
    std::deque<EngineSolve *> q_solve;   // inner solves of tonal requests
    std::vector<hipEvent_t> worker_events;   // two per tonal worker
    std::unordered_map<uint64_t, std::unique_ptr<Ticket>> tickets;
    std::vector<std::thread> threads;
    uint64_t next_id = 1;
    int inflight = 0;
    bool stop = false;
    std::chrono::steady_clock::time_point t0;

    double now_ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }

    // Carve the request's buffers from its arena block and stage host inputs
    // (on the copy stream, which `s` then waits for).
    int32_t place(Ticket *t, hipStream_t s) {
        const hdi_request &r = t->req;
        const size_t N = image_px(r.img), C = r.img.channels;
        char *p = t->mem;
        if (r.flags & HDI_REQ_HOST_IO) {
            uint8_t *m = (uint8_t *)p;
            p += up256(N);
            float *f = (float *)p;
            p += up256(4 * C * N);
            t->out = (double *)p;
            p += up256(8 * C * N);
            if (hipMemcpyAsync(m, r.mask, N, hipMemcpyHostToDevice, copy) != hipSuccess ||
                hipMemcpyAsync(f, r.f, 4 * C * N, hipMemcpyHostToDevice, copy) != hipSuccess ||
                hipEventRecord(t->ev, copy) != hipSuccess || hipStreamWaitEvent(s, t->ev, 0) != hipSuccess) {
                set_error("staging the request's inputs failed");
                return HDI_ERR_HIP;
            }
            t->mask = m;
            t->f = f;
        } else {
            t->mask = r.mask;
            t->f = r.f;
            t->out = r.out;
        }
        t->ws = p;
        t->ws_bytes = t->bytes - (size_t)(p - t->mem);
        return HDI_OK;
    }

    // Enqueue the result's way home (host outputs on the copy stream) and the
    // event whose completion ends the request.
    int32_t seal(Ticket *t, hipStream_t s) {
        const hdi_request &r = t->req;
        if (hipEventRecord(t->ev, s) != hipSuccess) return HDI_ERR_HIP;
        if (r.flags & HDI_REQ_HOST_IO) {
            const size_t bytes = 8 * (size_t)r.img.channels * image_px(r.img);
            if (hipStreamWaitEvent(copy, t->ev, 0) != hipSuccess ||
                hipMemcpyAsync(r.out, t->out, bytes, hipMemcpyDeviceToHost, copy) != hipSuccess ||
                hipEventRecord(t->ev, copy) != hipSuccess)
                return HDI_ERR_HIP;
        }
        return HDI_OK;
    }

    // Before a failed request's arena block goes back to the allocator: wait
    // for whatever its stream (and, with host I/O, the copy stream) may still
    // do with that memory, such as a staging copy or a solve's last copy.
    void quiesce(Ticket *t, hipStream_t s) {
        (void)hipStreamSynchronize(s);
        if (t->req.flags & HDI_REQ_HOST_IO) (void)hipStreamSynchronize(copy);
    }

    void finish(Ticket *t, int32_t status, const char *msg) {
        std::lock_guard<std::mutex> lk(mu);
        t->rep.status = status;
        if (status != HDI_OK && msg) t->message = msg;
        t->rep.t_done_ms = now_ms();
        if (t->mem) alloc.release(t->mem, t->bytes);
        t->mem = nullptr;
        t->done = true;
        --inflight;
        cv.notify_all();
    }

    // The tonal workers' inner solves, handed to the engine thread.
    struct Hook : SolveHook {
        hdi_server *srv;
        hipEvent_t ready, done;
        int max_running = 0;
        int32_t solve(Hierarchy &h, int overlap, int W, int H, int C, const uint8_t *mask, const double *data,
                      const double *src, double *x, bool warm, const SolveCfg &cfg, hdi_solve_report *rep,
                      hipStream_t s) override {
            EngineSolve es;
            es.ej.job = hdi_job{HDI_JOB_INPAINT, hdi_image{W, H, C}, mask, nullptr, x, nullptr, nullptr};
            es.ej.kind = data ? EK_DATA_F64 : EK_SRC_F64;
            es.ej.data_d = data;
            es.ej.src = src;
            es.ej.warm = warm;
            es.ej.cfg = cfg;
            es.ej.overlap = overlap;
            es.ej.h = h;
            es.ej.user = &es;
            es.ready = ready;
            es.done = done;
            if (hipEventRecord(ready, s) != hipSuccess) {
                set_error("recording an inner solve's start failed");
                return HDI_ERR_HIP;
            }
            {
                std::unique_lock<std::mutex> lk(srv->mu);
                srv->q_solve.push_back(&es);
                srv->cv.notify_all();
                srv->cv.wait(lk, [&] { return es.finished; });
            }
            max_running = std::max(max_running, es.max_running);
            if (es.status != HDI_OK) {
                set_error("the batch engine failed during an inner solve");
                return es.status;
            }
            if (hipStreamWaitEvent(s, done, 0) != hipSuccess) {
                set_error("waiting for an inner solve failed");
                return HDI_ERR_HIP;
            }
            const EJob &j = es.ej;
            for (int c = 0; c < 3; ++c) rep->rel_residual[c] = c < C ? j.rel[c] : 0.0;
            rep->outer_iters = j.rounds;
            rep->vcycles = j.rounds;
            rep->ms = 0.f;
            if (j.status == HDI_ERR_NO_CONVERGENCE) {
                set_error("relative residual %.3e above tolerance %.3e after %d rounds",
                          std::max(j.rel[0], std::max(j.rel[1], j.rel[2])), cfg.rel_tol, j.rounds);
            } else if (j.status == HDI_ERR_ARG) {
                set_error("non-finite residual: the input holds NaN/Inf or the iteration diverged");
            }
            return j.status;
        }
    };

    void run_tonal(Ticket *t, hipStream_t s, Hook *hook = nullptr) {
        int32_t st = place(t, s);
        hdi_tonal_report tr{};
        if (!st) {
            t->tonal.flags |= HDI_TONAL_INIT_FROM_F;
            st = tonal_optimize_hooked(t->req.img, t->mask, t->f, t->out, nullptr, t->ws, t->ws_bytes, &t->tonal, &tr,
                                       s, hook);
        }
        const std::string msg = st ? hdi_last_error() : "";
        bool sealed = false;
        if (st == HDI_OK || st == HDI_ERR_NO_CONVERGENCE) {
            if (seal(t, s) || hipEventSynchronize(t->ev) != hipSuccess) st = HDI_ERR_HIP;
            else sealed = true;
        }
        if (!sealed) quiesce(t, s);
        t->tonal_rep = tr;
        t->rep.outer_iters = tr.outer_iters;
        t->rep.inner_solves = tr.inner_solves;
        if (hook) {
            t->rep.max_running = hook->max_running;
            hook->max_running = 0;
        }
        t->rep.rel_residual[0] = tr.rel_normal_residual;
        t->rep.mse_initial = tr.mse_initial;
        t->rep.mse_final = tr.mse_final;
        finish(t, st, msg.c_str());
    }

    void run_inpaint_plain(Ticket *t, hipStream_t s) {
        int32_t st = place(t, s);
        hdi_solve_report sr{};
        if (!st) st = inpaint_solve(t->req.img, t->mask, t->f, t->out, nullptr, t->ws, t->ws_bytes, &t->req.solve, &sr, s);
        const std::string msg = st ? hdi_last_error() : "";
        bool sealed = false;
        if (st == HDI_OK || st == HDI_ERR_NO_CONVERGENCE) {
            if (seal(t, s) || hipEventSynchronize(t->ev) != hipSuccess) st = HDI_ERR_HIP;
            else sealed = true;
        }
        if (!sealed) quiesce(t, s);
        t->rep.outer_iters = sr.outer_iters;
        t->rep.max_running = 1;
        for (int c = 0; c < 3; ++c) t->rep.rel_residual[c] = sr.rel_residual[c];
        finish(t, st, msg.c_str());
    }

    // Take the head of q if its memory is free (strict arrival order).
    Ticket *take(std::deque<Ticket *> &q) {
        if (q.empty()) return nullptr;
        Ticket *t = q.front();
        t->mem = alloc.alloc(t->bytes);
        if (!t->mem) return nullptr;
        q.pop_front();
        t->rep.t_start_ms = now_ms();
        return t;
    }

    void plain_loop() {
        (void)hipSetDevice(device);
        for (;;) {
            Ticket *t = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return (t = take(q_all)) != nullptr || (stop && q_all.empty()); });
            }
            if (!t) return;
            if (t->req.kind == HDI_REQ_TONAL)
                run_tonal(t, compute);
            else
                run_inpaint_plain(t, compute);
        }
    }

    void tonal_loop(int w) {
        (void)hipSetDevice(device);
        Hook hook;
        hook.srv = this;
        hook.ready = worker_events[2 * w];
        hook.done = worker_events[2 * w + 1];
        for (;;) {
            Ticket *t = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return (t = take(q_ton)) != nullptr || (stop && q_ton.empty()); });
            }
            if (!t) return;
            run_tonal(t, tonal_streams[w], (flags & HDI_SERVER_TONAL_SHARED) ? &hook : nullptr);
        }
    }

    // End an inner solve (under the lock): its waiting worker may go on.
    void end_solve(EngineSolve *es, int32_t status) {
        std::lock_guard<std::mutex> lk(mu);
        es->status = status;
        es->finished = true;
        cv.notify_all();
    }

    void engine_loop() {
        (void)hipSetDevice(device);
        std::vector<Ticket *> sealed;   // device work enqueued, waiting for its event
        std::vector<EJob *> live;       // jobs in the engine (requests and inner solves)
        for (;;) {
            std::vector<Ticket *> admitted;
            std::vector<EngineSolve *> solves;
            {
                std::unique_lock<std::mutex> lk(mu);
                for (;;) {
                    std::vector<int> slots = eng.free_slots();
                    size_t k = 0;
                    // inner solves first: their requests hold memory already
                    while (k < slots.size() && !q_solve.empty()) {
                        EngineSolve *es = q_solve.front();
                        q_solve.pop_front();
                        es->ej.slot = slots[k++];
                        solves.push_back(es);
                    }
                    while (k < slots.size()) {
                        Ticket *t = take(q_inp);
                        if (!t) break;
                        t->ej.slot = slots[k++];
                        admitted.push_back(t);
                    }
                    if (!admitted.empty() || !solves.empty() || eng.running() > 0 || !sealed.empty()) break;
                    if (stop && q_inp.empty()) return;
                    cv.wait(lk);
                }
            }
            std::vector<EJob *> news, ended;
            for (EngineSolve *es : solves) {
                if (hipStreamWaitEvent(compute, es->ready, 0) != hipSuccess) {
                    end_solve(es, HDI_ERR_HIP);
                    continue;
                }
                news.push_back(&es->ej);
            }
            for (Ticket *t : admitted) {
                int32_t st = place(t, compute);
                if (st) {
                    const std::string msg = hdi_last_error();
                    quiesce(t, compute);
                    finish(t, st, msg.c_str());
                    continue;
                }
                EJob &j = t->ej;
                j.job = hdi_job{HDI_JOB_INPAINT, t->req.img, t->mask, t->f, t->out, nullptr, nullptr};
                j.user = t;
                Arena a{t->ws, t->ws_bytes, 0};
                plan_hierarchy(j.h, a, t->req.img.width, t->req.img.height, t->req.img.channels, j.overlap, t->mask,
                               j.cfg.small_from);
                news.push_back(&j);
            }
            int32_t st = eng.admit(news, ended, compute);
            if (!st) st = eng.round(ended, compute);
            if (st) {
                // a HIP failure leaves the batch undefined: end every running job
                const std::string msg = hdi_last_error();
                eng.abort_all(ended);
                live.clear();
                (void)hipStreamSynchronize(compute);
                for (EJob *j : ended) {
                    if (j->kind != EK_DATA_F32) {
                        end_solve((EngineSolve *)j->user, st);
                        continue;
                    }
                    Ticket *t = (Ticket *)j->user;
                    quiesce(t, compute);
                    finish(t, st, msg.c_str());
                }
                continue;
            }
            // this round ran every live job, the ones that just ended included
            for (EJob *j : news) live.push_back(j);
            const int nround = (int)live.size();
            for (EJob *j : live) {
                if (j->kind == EK_DATA_F32) {
                    Ticket *t = (Ticket *)j->user;
                    t->rep.max_running = std::max(t->rep.max_running, nround);
                } else {
                    EngineSolve *es = (EngineSolve *)j->user;
                    es->max_running = std::max(es->max_running, nround);
                }
            }
            for (EJob *j : ended) live.erase(std::find(live.begin(), live.end(), j));
            for (EJob *j : ended) {
                if (j->kind != EK_DATA_F32) {
                    // an inner solve: its solution (copied back on the compute
                    // stream) is in place once `done` has passed
                    EngineSolve *es = (EngineSolve *)j->user;
                    end_solve(es, hipEventRecord(es->done, compute) == hipSuccess ? HDI_OK : HDI_ERR_HIP);
                    continue;
                }
                Ticket *t = (Ticket *)j->user;
                t->rep.outer_iters = j->rounds;
                for (int c = 0; c < 3; ++c) t->rep.rel_residual[c] = c < j->h.C ? j->rel[c] : 0.0;
                if (j->status == HDI_ERR_EMPTY_MASK) {
                    quiesce(t, compute);
                    finish(t, j->status, "empty mask (the inpainting matrix is singular)");
                    continue;
                }
                if (seal(t, compute)) {
                    quiesce(t, compute);
                    finish(t, HDI_ERR_HIP, "recording the request's completion failed");
                    continue;
                }
                t->rep.status = j->status;
                sealed.push_back(t);
            }
            // requests whose outputs are final end now; with nothing left to
            // run, wait for the oldest instead of spinning
            if (eng.running() == 0 && !sealed.empty()) (void)hipEventSynchronize(sealed.front()->ev);
            for (size_t i = 0; i < sealed.size();) {
                Ticket *t = sealed[i];
                if (hipEventQuery(t->ev) == hipSuccess) {
                    const int32_t s2 = t->rep.status;
                    finish(t, s2, s2 == HDI_ERR_NO_CONVERGENCE ? "no convergence" : s2 ? "non-finite residual" : nullptr);
                    sealed.erase(sealed.begin() + i);
                } else {
                    ++i;
                }
            }
        }
    }
};

extern "C" {

size_t hdi_request_bytes(const hdi_request *r) {
    if (!r || (r->kind != HDI_REQ_INPAINT && r->kind != HDI_REQ_TONAL)) return 0;
    if (r->img.width < 1 || r->img.height < 1 || (r->img.channels != 1 && r->img.channels != 3)) return 0;
    return up256(work_bytes(*r)) + io_bytes(*r);
}

hdi_server *hdi_server_create(void *arena, size_t arena_bytes, int32_t max_slots, int32_t tonal_workers,
                              int32_t flags) {
    if (!arena || max_slots < 1 || max_slots > 4096 || tonal_workers < 0 || tonal_workers > 16) {
        set_error("server needs an arena, 1..4096 slots and 0..16 tonal workers");
        return nullptr;
    }
    std::unique_ptr<hdi_server> srv(new hdi_server);
    srv->flags = flags;
    srv->max_slots = max_slots;
    srv->t0 = std::chrono::steady_clock::now();
    if (hipGetDevice(&srv->device) != hipSuccess) {
        set_error("no current device");
        return nullptr;
    }
    Arena a{(char *)arena, arena_bytes, 0};
    if (!srv->eng.plan(a, max_slots)) {
        set_error("arena of %zu bytes too small for the tables of %d slots", arena_bytes, max_slots);
        return nullptr;
    }
    const size_t used = up256(a.used);
    srv->alloc.init((char *)arena + used, arena_bytes > used ? arena_bytes - used : 0);
    if (hipStreamCreateWithFlags(&srv->compute, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&srv->copy, hipStreamNonBlocking) != hipSuccess) {
        set_error("stream creation failed");
        return nullptr;
    }
    const int nt = (flags & HDI_SERVER_PLAIN) ? 0 : tonal_workers;
    for (int w = 0; w < nt; ++w) {
        hipStream_t s;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            set_error("stream creation failed");
            return nullptr;
        }
        srv->tonal_streams.push_back(s);
        for (int k = 0; k < 2; ++k) {
            hipEvent_t e;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                set_error("event creation failed");
                return nullptr;
            }
            srv->worker_events.push_back(e);
        }
    }
    hdi_server *p = srv.get();
    if (flags & HDI_SERVER_PLAIN) {
        srv->threads.emplace_back([p] { p->plain_loop(); });
    } else {
        srv->threads.emplace_back([p] { p->engine_loop(); });
        for (int w = 0; w < nt; ++w) srv->threads.emplace_back([p, w] { p->tonal_loop(w); });
    }
    return srv.release();
}

int32_t hdi_server_submit(hdi_server *srv, const hdi_request *req, uint64_t *ticket) {
    if (!srv || !req || !ticket) {
        set_error("server, request and ticket must be non-null");
        return HDI_ERR_ARG;
    }
    if (req->kind != HDI_REQ_INPAINT && req->kind != HDI_REQ_TONAL) {
        set_error("request kind %d is neither HDI_REQ_INPAINT nor HDI_REQ_TONAL", req->kind);
        return HDI_ERR_ARG;
    }
    if (!check_image(req->img)) return HDI_ERR_ARG;
    if (!req->mask || !req->f || !req->out) {
        set_error("mask, f and out must be non-null");
        return HDI_ERR_ARG;
    }
    std::unique_ptr<Ticket> t(new Ticket);
    t->req = *req;
    if (req->tonal) t->tonal = *req->tonal;
    t->req.tonal = nullptr;
    int32_t st = fill_cfg(&t->req.solve, t->ej.cfg, t->ej.overlap);
    if (st) return st;
    if (req->kind == HDI_REQ_TONAL) {
        TonalCfg tc;
        SolveCfg inner;
        int ov = 0;
        st = fill_tonal_cfg(req->tonal, tc, inner, ov);
        if (st) return st;
        if ((inner.flags & HDI_FLAG_CG) && (srv->flags & HDI_SERVER_TONAL_SHARED) && !(srv->flags & HDI_SERVER_PLAIN)) {
            set_error("tonal requests' inner solves run in the batch engine, which runs the multigrid solver only "
                      "(HDI_FLAG_CG is for single solves)");
            return HDI_ERR_ARG;
        }
    }
    if (t->ej.cfg.flags & HDI_FLAG_CG) {
        set_error("the server runs the multigrid solver only (HDI_FLAG_CG is for single solves)");
        return HDI_ERR_ARG;
    }
    if (req->kind == HDI_REQ_TONAL && !(srv->flags & HDI_SERVER_PLAIN) && srv->tonal_streams.empty()) {
        set_error("this server has no tonal workers");
        return HDI_ERR_ARG;
    }
    t->bytes = hdi_request_bytes(req);
    if (t->bytes > srv->alloc.capacity()) {
        set_error("request needs %zu arena bytes, the arena has %zu", t->bytes, srv->alloc.capacity());
        return HDI_ERR_BUDGET;
    }
    if (hipEventCreateWithFlags(&t->ev, hipEventDisableTiming) != hipSuccess) {
        set_error("event creation failed");
        return HDI_ERR_HIP;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) {
        (void)hipEventDestroy(t->ev);
        set_error("server is shutting down");
        return HDI_ERR_ARG;
    }
    t->id = srv->next_id++;
    t->rep.kind = req->kind;
    t->rep.t_submit_ms = srv->now_ms();
    Ticket *raw = t.get();
    if (srv->flags & HDI_SERVER_PLAIN)
        srv->q_all.push_back(raw);
    else
        (req->kind == HDI_REQ_TONAL ? srv->q_ton : srv->q_inp).push_back(raw);
    srv->tickets[raw->id] = std::move(t);
    ++srv->inflight;
    *ticket = raw->id;
    srv->cv.notify_all();
    return HDI_OK;
}

int32_t hdi_server_poll(hdi_server *srv, uint64_t ticket, int32_t *done, hdi_request_report *report) {
    if (!srv || !done) {
        set_error("server and done must be non-null");
        return HDI_ERR_ARG;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) {
        set_error("unknown ticket %llu", (unsigned long long)ticket);
        return HDI_ERR_ARG;
    }
    Ticket *t = it->second.get();
    *done = t->done ? 1 : 0;
    if (!t->done) return HDI_OK;
    if (report) *report = t->rep;
    if (t->rep.status != HDI_OK) set_error("request %llu: %s", (unsigned long long)ticket, t->message.c_str());
    (void)hipEventDestroy(t->ev);
    srv->tickets.erase(it);
    return HDI_OK;
}

int32_t hdi_server_drain(hdi_server *srv) {
    if (!srv) {
        set_error("server must be non-null");
        return HDI_ERR_ARG;
    }
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv.wait(lk, [&] { return srv->inflight == 0; });
    return HDI_OK;
}

void hdi_server_destroy(hdi_server *srv) {
    if (!srv) return;
    hdi_server_drain(srv);
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->cv.notify_all();
    }
    for (std::thread &th : srv->threads) th.join();
    for (auto &kv : srv->tickets) (void)hipEventDestroy(kv.second->ev);
    for (hipEvent_t e : srv->worker_events) (void)hipEventDestroy(e);
    for (hipStream_t s : srv->tonal_streams) (void)hipStreamDestroy(s);
    (void)hipStreamDestroy(srv->copy);
    (void)hipStreamDestroy(srv->compute);
    delete srv;
}

}  // extern "C"

namespace hdi {

size_t batch_served_bytes(int n, const hdi_job *jobs) {
    Engine e;
    Arena a{nullptr, 0, 0};
    e.plan(a, n);
    size_t total = up256(a.used);
    for (int i = 0; i < n; ++i) {
        hdi_request r{};
        r.kind = jobs[i].kind == HDI_JOB_TONAL ? HDI_REQ_TONAL : HDI_REQ_INPAINT;
        r.img = jobs[i].img;
        const size_t b = hdi_request_bytes(&r);
        if (!b) return 0;
        total += up256(b);
    }
    return total + 256;
}

int32_t solve_batch_served(int n, const hdi_job *jobs, void *ws, size_t ws_bytes, const hdi_solve_params *params,
                           hdi_solve_report *reports, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    // the jobs' inputs were written on the caller's stream
    if (hipStreamSynchronize(s) != hipSuccess) {
        set_error("synchronising the caller's stream failed");
        return HDI_ERR_HIP;
    }
    int ntonal = 0;
    for (int i = 0; i < n; ++i) ntonal += jobs[i].kind == HDI_JOB_TONAL;
    hdi_server *srv = hdi_server_create(ws, ws_bytes, n, std::min(ntonal, 16), HDI_SERVER_TONAL_SHARED);
    if (!srv) return HDI_ERR_HIP;
    std::vector<uint64_t> tickets(n, 0);
    int32_t st = HDI_OK;
    for (int i = 0; i < n && st == HDI_OK; ++i) {
        hdi_request r{};
        r.kind = jobs[i].kind == HDI_JOB_TONAL ? HDI_REQ_TONAL : HDI_REQ_INPAINT;
        r.img = jobs[i].img;
        r.mask = jobs[i].mask;
        r.f = jobs[i].f;
        r.out = jobs[i].out;
        if (params) r.solve = params[i];
        r.tonal = jobs[i].tonal;
        st = hdi_server_submit(srv, &r, &tickets[i]);
    }
    hdi_server_drain(srv);
    const float ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int32_t worst = st;
    std::string first_msg = st ? hdi_last_error() : "";
    for (int i = 0; i < n; ++i) {
        if (!tickets[i]) continue;
        Ticket *t = nullptr;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            auto it = srv->tickets.find(tickets[i]);
            if (it != srv->tickets.end()) t = it->second.get();
        }
        if (!t) continue;
        if (reports) {
            for (int c = 0; c < 3; ++c) reports[i].rel_residual[c] = t->rep.rel_residual[c];
            reports[i].outer_iters = t->rep.outer_iters;
            reports[i].vcycles = t->req.kind == HDI_REQ_TONAL ? t->tonal_rep.inner_vcycles : t->rep.outer_iters;
            reports[i].ms = ms;
        }
        if (t->req.kind == HDI_REQ_TONAL && jobs[i].tonal_report) {
            *jobs[i].tonal_report = t->tonal_rep;
            jobs[i].tonal_report->ms = ms;
        }
        if (t->rep.status != HDI_OK && worst == HDI_OK) {
            worst = t->rep.status;
            first_msg = "job " + std::to_string(i) + ": " + t->message;
        }
    }
    hdi_server_destroy(srv);
    if (worst != HDI_OK) set_error("%s", first_msg.c_str());
    return worst;
}

}  // namespace hdi
