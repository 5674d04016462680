// tlb_server.cpp -- continuous-batching solve server of the C ABI
// (include/tlb.h, tlb_server_*).
//
// Requests are independent solves (grid, fluid, geometry, initial fields,
// step count).  A worker thread owns the device side: it admits queued
// requests in arrival order whenever a slot and a block of the caller's
// device arena are free (a request that does not fit yet does not block the
// ones behind it), initialises them, and advances every running lattice in
// shared launches of the batched step kernel, a quantum of steps at a time
// (the quantum ends at the next completion).  Two streams: the quanta run on
// the caller's stream; set-up (create, geometry, initial fields) and readout
// (mass, fields) of requests run on the server's own I/O stream while a
// quantum is in flight, so they overlap the stepping of the others.  Every
// check_steps steps a running request's mass/NaN health check is queued
// behind its quantum; a diverged request fails at that boundary instead of
// burning its whole step budget.  Finished requests are read out to host
// memory and released, which frees room for waiting requests.  A request's
// result does not depend on what else runs (the batched kernel computes every
// lattice exactly as a lone one).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/tlb.h"
#include "tlb_internal.h"

using Clock = std::chrono::steady_clock;

namespace {

constexpr size_t kArenaAlign = 256;

// first-fit allocator over [0, size) of the caller's arena
class Arena {
  public:
    void reset(size_t size) {
        free_.clear();
        free_[0] = size;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = (bytes + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                size_t rest = it->second - bytes;
                size_t start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t largest() const {
        size_t m = 0;
        for (auto& kv : free_) m = std::max(m, kv.second);
        return m;
    }

  private:
    std::map<size_t, size_t> free_;
};

struct Request {
    uint64_t id;
    int nx, ny, px, py;
    tlb_fluid fluid;
    std::vector<uint8_t> material;
    std::vector<tlb_material> mats;
    std::vector<double> c1, c2, ux, uy;
    int64_t nsteps, remaining;
    uint32_t keep;
    int state = TLB_REQ_QUEUED;
    bool cancel = false;
    tlb_status status = TLB_OK;   // what failed a FAILED request
    std::string error;
    Clock::time_point arrival, done;
    size_t ws_off = 0, ws_bytes = 0;
    tlb_ctx* ctx = nullptr;
    int64_t since_check = 0;      // steps since the last health check
    std::vector<double> result;   // popcount(keep) * ny*nx
};

}  // namespace

struct tlb_server {
    int device = 0;
    char* arena;
    size_t arena_bytes;
    int max_slots;
    int prec;
    int64_t quantum;
    int64_t check_steps = 1000;   // health check interval of running requests
    hipStream_t stream;           // quanta (caller's)
    hipStream_t io = nullptr;     // set-up and readout (the server's)
    double* health = nullptr;     // pinned: 4 doubles per slot
    Arena alloc;
    size_t table_off = 0;
    tlb_batch* batch = nullptr;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;
    std::vector<std::shared_ptr<Request>> running;
    std::map<uint64_t, std::shared_ptr<Request>> all;
    uint64_t next_id = 1;
    bool stop = false;
    std::thread worker;
    // statistics
    double busy_s = 0.0;
    double node_steps = 0.0;
    int64_t completed = 0, failed = 0;
};

namespace {

// message of the calling thread's last failed server call (a per-server
// string would be written by concurrent callers and the worker at once);
// failures inside the worker are reported per request
thread_local std::string g_server_error;

tlb_status sfail(tlb_server*, tlb_status st, const std::string& m) {
    g_server_error = m;
    return st;
}

int popcount10(uint32_t m) {
    int n = 0;
    for (int f = 0; f < 10; ++f) n += (m >> f) & 1u;
    return n;
}

// set up a request's context inside its arena block (worker thread, on the
// I/O stream; returns when the initial state is on the device)
bool start_request(tlb_server* s, Request& r) {
    tlb_status st = tlb_create(r.nx, r.ny, tlb_precision(s->prec), &r.fluid, s->arena + r.ws_off,
                               r.ws_bytes, s->io, &r.ctx);
    if (st == TLB_OK)
        st = tlb_set_geometry(r.ctx, r.px, r.py, r.material.data(), r.mats.data(),
                              int(r.mats.size()), nullptr);
    if (st == TLB_OK)
        st = tlb_init_fields(r.ctx, r.c1.data(), r.c2.data(), r.ux.empty() ? nullptr : r.ux.data(),
                             r.uy.empty() ? nullptr : r.uy.data());
    if (st == TLB_OK) st = tlb_set_check_interval(r.ctx, 0);
    // the one-step strip height is left unset: every registration of the
    // running requests gives them the batch's (tlb_batch_set), short while
    // few requests run.  Measured on the FP16-dev request stream against 64
    // rows for every request: p50/p99 at 0.7x load 0.45/3.29 s against
    // 0.88/3.76 s, capacity 27.1 against 28.1 requests/s.
    if (st != TLB_OK) {
        // with r.ctx NULL (tlb_create failed) this is the thread's last message
        r.error = tlb_last_error(r.ctx);
        r.status = st;
        return false;
    }
    // the host copies of the inputs are no longer needed
    std::vector<double>().swap(r.c1);
    std::vector<double>().swap(r.c2);
    std::vector<double>().swap(r.ux);
    std::vector<double>().swap(r.uy);
    return true;
}

// read out a finished request (worker thread, on the I/O stream, after the
// quantum that finished it has completed); false on divergence / error
bool finish_request(tlb_server* s, Request& r) {
    (void)s;
    double m[3];
    tlb_status st = tlb_mass(r.ctx, m);
    if (st != TLB_OK) {
        r.error = st == TLB_EDIVERGED ? "diverged (NaN/Inf order parameter)" : tlb_last_error(r.ctx);
        r.status = st;
        return false;
    }
    const size_t n = size_t(r.nx) * r.ny;
    r.result.assign(size_t(popcount10(r.keep)) * n, 0.0);
    if (r.keep) {
        st = tlb_read_fields(r.ctx, r.keep, r.result.data());
        if (st != TLB_OK) {
            r.error = tlb_last_error(r.ctx);
            r.status = st;
            return false;
        }
    }
    return true;
}

void release_request(tlb_server* s, Request& r) {
    if (r.ctx) {
        tlb_destroy(r.ctx);
        r.ctx = nullptr;
    }
    if (r.ws_bytes) {
        s->alloc.release(r.ws_off, r.ws_bytes);
        r.ws_bytes = 0;
    }
}

void fail_request(tlb_server* s, Request& r, tlb_status st, const std::string& why) {
    // caller holds s->mu
    release_request(s, r);
    r.state = TLB_REQ_FAILED;
    if (r.status == TLB_OK) r.status = st;
    if (r.error.empty()) r.error = why;
    r.done = Clock::now();
    ++s->failed;
    s->cv_done.notify_all();
}

// One iteration: (1) the quantum of the running requests is queued on the
// compute stream, with the health checks that fall due behind it; (2) while
// it runs, requests that finished at the previous boundary are read out and
// released, and queued requests that fit are set up, both on the I/O stream;
// (3) after the quantum, due health checks are read (a request with a
// non-finite c1, c2, ux or uy fails now), finished requests move to the
// readout list, and new requests join the batch.
void worker_loop(tlb_server* s) {
    // every request fails if this thread cannot use the server's device
    const bool dev_ok = hipSetDevice(s->device) == hipSuccess;
    bool composition_changed = true;
    std::vector<std::shared_ptr<Request>> to_finish, ready;
    for (;;) {
        std::vector<std::shared_ptr<Request>> run;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] {
                return s->stop || !s->queue.empty() || !s->running.empty() || !to_finish.empty() ||
                       !ready.empty();
            });
            if (s->stop) break;
            // drop cancelled requests
            for (auto it = s->queue.begin(); it != s->queue.end();) {
                if ((*it)->cancel) {
                    (*it)->state = TLB_REQ_CANCELLED;
                    (*it)->done = Clock::now();
                    it = s->queue.erase(it);
                    s->cv_done.notify_all();
                } else {
                    ++it;
                }
            }
            // new requests join at this boundary; cancelled running ones leave
            for (auto& r : ready) s->running.push_back(r);
            if (!ready.empty()) composition_changed = true;
            ready.clear();
            for (auto it = s->running.begin(); it != s->running.end();) {
                if ((*it)->cancel) {
                    release_request(s, **it);
                    (*it)->state = TLB_REQ_CANCELLED;
                    (*it)->done = Clock::now();
                    it = s->running.erase(it);
                    composition_changed = true;
                    s->cv_done.notify_all();
                } else {
                    ++it;
                }
            }
            run = s->running;
        }
        if (!run.empty() && composition_changed) {
            std::vector<tlb_ctx*> ctxs;
            for (auto& r : run) ctxs.push_back(r->ctx);
            const tlb_status bst = tlb_batch_set(s->batch, ctxs.data(), int(ctxs.size()));
            if (bst != TLB_OK) {
                std::lock_guard<std::mutex> lk(s->mu);
                const std::string why = tlb_batch_last_error(s->batch);
                for (auto& r : run) fail_request(s, *r, bst, why);
                s->running.clear();
                continue;
            }
            composition_changed = false;
        }
        // (1) queue the quantum and the due health checks
        int64_t q = s->quantum;
        double nodes = 0.0;
        for (auto& r : run) {
            q = std::min(q, r->remaining);
            nodes += double(r->nx) * r->ny;
        }
        const auto t0 = Clock::now();
        tlb_status st = TLB_OK;
        std::vector<int> checked;
        if (!run.empty()) {
            st = tlb_batch_step(s->batch, q);
            for (size_t i = 0; st == TLB_OK && i < run.size(); ++i) {
                Request& r = *run[i];
                if (r.remaining - q > 0 && r.since_check + q >= s->check_steps) {
                    st = tlb_status(tlb::health_enqueue(r.ctx, s->stream, s->health + 4 * i));
                    checked.push_back(int(i));
                }
            }
        }
        // (2) while the quantum runs: readout of the previous boundary's
        // finished requests, set-up of queued requests that fit
        for (auto& rp : to_finish) {
            const bool ok = rp->status == TLB_OK && finish_request(s, *rp);
            std::lock_guard<std::mutex> lk(s->mu);
            release_request(s, *rp);
            rp->done = Clock::now();
            if (ok) {
                rp->state = TLB_REQ_DONE;
                ++s->completed;
            } else {
                rp->state = TLB_REQ_FAILED;
                if (rp->status == TLB_OK) rp->status = TLB_EDEVICE;
                ++s->failed;
            }
            s->cv_done.notify_all();
        }
        to_finish.clear();
        std::vector<std::shared_ptr<Request>> admitted;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            for (auto it = s->queue.begin(); it != s->queue.end();) {
                if (int(run.size() + admitted.size()) >= s->max_slots) break;
                Request& r = **it;
                size_t off;
                if (s->alloc.alloc(r.ws_bytes, &off)) {
                    r.ws_off = off;
                    r.state = TLB_REQ_RUNNING;
                    admitted.push_back(*it);
                    it = s->queue.erase(it);
                } else {
                    ++it;
                }
            }
        }
        for (auto& rp : admitted) {
            if (!dev_ok) {
                rp->error = "hipSetDevice failed on the server thread";
                rp->status = TLB_EDEVICE;
            }
            if (dev_ok && start_request(s, *rp)) {
                ready.push_back(rp);
            } else {
                std::lock_guard<std::mutex> lk(s->mu);
                fail_request(s, *rp, rp->status != TLB_OK ? rp->status : TLB_EDEVICE, rp->error);
            }
        }
        if (run.empty()) continue;
        // (3) after the quantum
        if (st == TLB_OK) st = tlb_batch_sync(s->batch);
        const double dt = std::chrono::duration<double>(Clock::now() - t0).count();
        std::lock_guard<std::mutex> lk(s->mu);
        s->busy_s += dt;
        s->node_steps += nodes * double(q);
        for (auto& r : run) {
            r->remaining -= q;
            r->since_check += q;
        }
        if (st == TLB_OK)
            for (int i : checked) {
                run[size_t(i)]->since_check = 0;
                if (s->health[4 * i + 3] != 0.0) {
                    run[size_t(i)]->status = TLB_EDIVERGED;
                    run[size_t(i)]->error = "diverged (NaN/Inf in c1, c2, ux or uy)";
                }
            }
        for (auto& r : run) {
            if (st != TLB_OK) {
                r->status = st;
                r->error = tlb_batch_last_error(s->batch);
            }
            if (r->remaining <= 0 || r->status != TLB_OK) {
                to_finish.push_back(r);
                s->running.erase(std::remove(s->running.begin(), s->running.end(), r),
                                 s->running.end());
                composition_changed = true;
            }
        }
    }
    // shutdown: release everything still held
    std::lock_guard<std::mutex> lk(s->mu);
    const auto now = Clock::now();
    for (auto* list : {&s->running, &to_finish, &ready}) {
        for (auto& r : *list) {
            release_request(s, *r);
            r->state = TLB_REQ_CANCELLED;
            r->done = now;
        }
        list->clear();
    }
    for (auto& r : s->queue) {
        r->state = TLB_REQ_CANCELLED;
        r->done = now;
    }
    s->queue.clear();
    s->cv_done.notify_all();
}

}  // namespace

extern "C" {

tlb_status tlb_server_create(void* dev_arena, size_t arena_bytes, int max_slots,
                             tlb_precision p, int64_t quantum_steps, void* hip_stream,
                             tlb_server** out) {
    if (!out) return sfail(nullptr, TLB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!dev_arena || max_slots <= 0 || quantum_steps <= 0)
        return sfail(nullptr, TLB_EINVAL, "null arena, max_slots <= 0 or quantum <= 0");
    if (p != TLB_FP64 && p != TLB_FP32 && p != TLB_FP16DEV)
        return sfail(nullptr, TLB_EINVAL, "unknown precision");
    if (reinterpret_cast<uintptr_t>(dev_arena) % kArenaAlign)
        return sfail(nullptr, TLB_EINVAL, "arena not 256-byte aligned");
    const size_t table = tlb_batch_table_bytes(max_slots);
    if (arena_bytes < table + kArenaAlign) return sfail(nullptr, TLB_ENOMEM, "arena too small");
    tlb_server* s = new tlb_server();
    if (hipGetDevice(&s->device) != hipSuccess) s->device = 0;
    s->arena = static_cast<char*>(dev_arena);
    s->arena_bytes = arena_bytes;
    s->max_slots = max_slots;
    s->prec = int(p);
    s->quantum = quantum_steps;
    s->stream = static_cast<hipStream_t>(hip_stream);
    s->alloc.reset(arena_bytes);
    s->alloc.alloc(table, &s->table_off);
    if (hipStreamCreateWithFlags(&s->io, hipStreamNonBlocking) != hipSuccess) {
        delete s;
        return sfail(nullptr, TLB_EDEVICE, "I/O stream");
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&s->health), size_t(max_slots) * 4 * sizeof(double)) !=
        hipSuccess) {
        (void)hipStreamDestroy(s->io);
        delete s;
        return sfail(nullptr, TLB_ENOMEM, "pinned health words");
    }
    if (tlb_batch_create(max_slots, s->arena + s->table_off, table, s->stream, &s->batch) != TLB_OK) {
        (void)hipHostFree(s->health);
        (void)hipStreamDestroy(s->io);
        delete s;
        return sfail(nullptr, TLB_EDEVICE, "batch table");
    }
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return TLB_OK;
}

tlb_status tlb_server_submit(tlb_server* s, const tlb_request* q, uint64_t* id) {
    if (!s || !q || !id) return sfail(s, TLB_EINVAL, "null pointer");
    if (q->nx < 3 || q->ny < 3 || !q->material || !q->c1 || !q->c2 || q->nsteps < 0 ||
        q->n_mats < 0 || (q->n_mats > 0 && !q->mats) || (q->result_fields & ~uint32_t(TLB_F_ALL)))
        return sfail(s, TLB_EINVAL, "bad request");
    const size_t ws = tlb_workspace_bytes(q->nx, q->ny, tlb_precision(s->prec));
    if (ws == 0) return sfail(s, TLB_EINVAL, "bad lattice size");
    if (ws > s->arena_bytes - tlb_batch_table_bytes(s->max_slots))
        return sfail(s, TLB_ENOMEM, "request larger than the whole arena");
    auto r = std::make_shared<Request>();
    const size_t n = size_t(q->nx) * q->ny;
    r->nx = q->nx;
    r->ny = q->ny;
    r->px = q->periodic_x;
    r->py = q->periodic_y;
    r->fluid = q->fluid;
    r->material.assign(q->material, q->material + n);
    r->mats.assign(q->mats, q->mats + q->n_mats);
    r->c1.assign(q->c1, q->c1 + n);
    r->c2.assign(q->c2, q->c2 + n);
    if (q->ux) r->ux.assign(q->ux, q->ux + n);
    if (q->uy) r->uy.assign(q->uy, q->uy + n);
    r->nsteps = r->remaining = q->nsteps;
    r->keep = q->result_fields;
    r->ws_bytes = ws;
    r->arrival = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return sfail(s, TLB_ESTATE, "server stopping");
        r->id = s->next_id++;
        s->all[r->id] = r;
        s->queue.push_back(r);
    }
    s->cv_work.notify_all();
    *id = r->id;
    return TLB_OK;
}

tlb_status tlb_server_poll(tlb_server* s, uint64_t id, int* state) {
    if (!s || !state) return sfail(s, TLB_EINVAL, "null pointer");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(id);
    if (it == s->all.end()) return sfail(s, TLB_EINVAL, "unknown request id");
    *state = it->second->state;
    return TLB_OK;
}

tlb_status tlb_server_wait(tlb_server* s, uint64_t id, double timeout_s) {
    if (!s) return sfail(s, TLB_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(id);
    if (it == s->all.end()) return sfail(s, TLB_EINVAL, "unknown request id");
    auto r = it->second;
    auto pred = [&] { return r->state >= TLB_REQ_DONE; };
    if (timeout_s < 0) {
        s->cv_done.wait(lk, pred);
    } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) {
        return sfail(s, TLB_EBUSY, "request not finished before the timeout");
    }
    return TLB_OK;
}

tlb_status tlb_server_result(tlb_server* s, uint64_t id, uint32_t mask, double* host_out,
                             double* latency_s) {
    if (!s) return sfail(s, TLB_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(id);
    if (it == s->all.end()) return sfail(s, TLB_EINVAL, "unknown request id");
    Request& r = *it->second;
    if (r.state == TLB_REQ_FAILED)
        return sfail(s, r.status != TLB_OK ? r.status : TLB_EDEVICE, "request failed: " + r.error);
    if (r.state == TLB_REQ_CANCELLED) return sfail(s, TLB_ESTATE, "request was cancelled");
    if (r.state != TLB_REQ_DONE) return sfail(s, TLB_EBUSY, "request not finished");
    if (latency_s) *latency_s = std::chrono::duration<double>(r.done - r.arrival).count();
    if (mask && host_out) {
        if (mask & ~r.keep) return sfail(s, TLB_EINVAL, "field not kept by this request");
        const size_t n = size_t(r.nx) * r.ny;
        int src = 0, dst = 0;
        for (int f = 0; f < 10; ++f) {
            if (!(r.keep & (1u << f))) continue;
            if (mask & (1u << f)) {
                std::memcpy(host_out + size_t(dst) * n, r.result.data() + size_t(src) * n,
                            n * sizeof(double));
                ++dst;
            }
            ++src;
        }
    }
    return TLB_OK;
}

tlb_status tlb_server_release(tlb_server* s, uint64_t id) {
    if (!s) return sfail(s, TLB_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(id);
    if (it == s->all.end()) return sfail(s, TLB_EINVAL, "unknown request id");
    if (it->second->state < TLB_REQ_DONE) return sfail(s, TLB_EBUSY, "request not finished");
    s->all.erase(it);
    return TLB_OK;
}

tlb_status tlb_server_cancel(tlb_server* s, uint64_t id) {
    if (!s) return sfail(s, TLB_EINVAL, "null server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->all.find(id);
        if (it == s->all.end()) return sfail(s, TLB_EINVAL, "unknown request id");
        if (it->second->state >= TLB_REQ_DONE) return TLB_OK;
        it->second->cancel = true;
    }
    s->cv_work.notify_all();
    return TLB_OK;
}

tlb_status tlb_server_stats(tlb_server* s, tlb_server_counters* out) {
    if (!s || !out) return sfail(s, TLB_EINVAL, "null pointer");
    std::lock_guard<std::mutex> lk(s->mu);
    out->completed = s->completed;
    out->failed = s->failed;
    out->queued = int64_t(s->queue.size());
    out->running = int64_t(s->running.size());
    out->busy_seconds = s->busy_s;
    out->node_steps = s->node_steps;
    out->arena_free_largest = s->alloc.largest();
    return TLB_OK;
}

const char* tlb_server_last_error(const tlb_server*) { return g_server_error.c_str(); }

void tlb_server_destroy(tlb_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    tlb_batch_destroy(s->batch);
    (void)hipStreamSynchronize(s->io);
    (void)hipStreamDestroy(s->io);
    (void)hipHostFree(s->health);
    delete s;
}

tlb_status tlb_server_set_check_steps(tlb_server* s, int64_t steps) {
    if (!s || steps <= 0) return sfail(s, TLB_EINVAL, "null server or check interval <= 0");
    std::lock_guard<std::mutex> lk(s->mu);
    s->check_steps = steps;
    return TLB_OK;
}

}  // extern "C"
