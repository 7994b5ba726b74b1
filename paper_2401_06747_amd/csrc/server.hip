// Request loop with continuous batching over one device.
//
// Inpainting requests go through the batch engine: a worker thread admits
// waiting requests between refinement rounds (as slots and arena memory free
// up), runs one round over every running request, and hands back the ones that
// met their tolerance. Tonal requests run on their own worker threads and
// streams (each tonal solve is a chain of host-synchronous inner solves), so
// their kernels overlap the batch rounds on the device. With HDI_SERVER_PLAIN
// one worker runs the requests one at a time through inpaint_solve and
// tonal_optimize: the one-request-per-launch control.
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

    void run_tonal(Ticket *t, hipStream_t s) {
        int32_t st = place(t, s);
        hdi_tonal_report tr{};
        if (!st) {
            t->tonal.flags |= HDI_TONAL_INIT_FROM_F;
            st = tonal_optimize(t->req.img, t->mask, t->f, t->out, nullptr, t->ws, t->ws_bytes, &t->tonal, &tr, s);
        }
        const std::string msg = st ? hdi_last_error() : "";
        bool sealed = false;
        if (st == HDI_OK || st == HDI_ERR_NO_CONVERGENCE) {
            if (seal(t, s) || hipEventSynchronize(t->ev) != hipSuccess) st = HDI_ERR_HIP;
            else sealed = true;
        }
        if (!sealed) quiesce(t, s);
        t->rep.outer_iters = tr.outer_iters;
        t->rep.inner_solves = tr.inner_solves;
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
        for (;;) {
            Ticket *t = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return (t = take(q_ton)) != nullptr || (stop && q_ton.empty()); });
            }
            if (!t) return;
            run_tonal(t, tonal_streams[w]);
        }
    }

    void engine_loop() {
        (void)hipSetDevice(device);
        std::vector<Ticket *> sealed;   // device work enqueued, waiting for its event
        std::vector<Ticket *> live;     // requests in the engine
        for (;;) {
            std::vector<Ticket *> admitted;
            {
                std::unique_lock<std::mutex> lk(mu);
                for (;;) {
                    std::vector<int> slots = eng.free_slots();
                    size_t k = 0;
                    while (k < slots.size()) {
                        Ticket *t = take(q_inp);
                        if (!t) break;
                        t->ej.slot = slots[k++];
                        admitted.push_back(t);
                    }
                    if (!admitted.empty() || eng.running() > 0 || !sealed.empty()) break;
                    if (stop && q_inp.empty()) return;
                    cv.wait(lk);
                }
            }
            std::vector<EJob *> news, ended;
            for (Ticket *t : admitted) {
                int32_t st = place(t, compute);
                if (st) {
                    const std::string msg = hdi_last_error();
                    quiesce(t, compute);
                    finish(t, st, msg.c_str());
                    continue;
                }
                EJob &j = t->ej;
                j.job = hdi_job{t->req.img, t->mask, t->f, t->out};
                j.user = t;
                Arena a{t->ws, t->ws_bytes, 0};
                plan_hierarchy(j.h, a, t->req.img.width, t->req.img.height, t->req.img.channels, j.overlap, t->mask,
                               j.cfg.small_from);
                news.push_back(&j);
            }
            int32_t st = eng.admit(news, ended, compute);
            if (!st) st = eng.round(ended, compute);
            if (st) {
                // a HIP failure leaves the batch undefined: end every running request
                const std::string msg = hdi_last_error();
                eng.abort_all(ended);
                live.clear();
                for (EJob *j : ended) {
                    Ticket *t = (Ticket *)j->user;
                    quiesce(t, compute);
                    finish(t, st, msg.c_str());
                }
                continue;
            }
            // this round ran every live request, the ones that just ended included
            for (EJob *j : news) live.push_back((Ticket *)j->user);
            const int nround = (int)live.size();
            for (Ticket *t : live) t->rep.max_running = std::max(t->rep.max_running, nround);
            for (EJob *j : ended) live.erase(std::find(live.begin(), live.end(), (Ticket *)j->user));
            for (EJob *j : ended) {
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
    for (hipStream_t s : srv->tonal_streams) (void)hipStreamDestroy(s);
    (void)hipStreamDestroy(srv->copy);
    (void)hipStreamDestroy(srv->compute);
    delete srv;
}

}  // extern "C"
