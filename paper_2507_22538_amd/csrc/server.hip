// Serving loop: HBM-budget admission, a pool of worker streams for large
// requests, continuous batching of small ones: they join the running batched
// solve between chunks of rounds and leave it when their own solve ends.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <vector>

#include "../../include/ipi_server.h"
#include "internal.hpp"

namespace ipi {
ipi_mdp_s* create_mdp(int64_t S, int32_t A, int64_t nnz, const int64_t* row_ptr, const int32_t* col,
                      const double* val, const double* g, double gamma, uint32_t flags, hipStream_t st);
void destroy_mdp(ipi_mdp_s* m);
void release_mdp(ipi_mdp_s* m);
void validate_host_arrays(int64_t S, int32_t A, int64_t nnz, const int64_t* rp, const int32_t* col, const double* val,
                          const double* g, double gamma, uint32_t flags, int32_t* kmax);
}  // namespace ipi

using namespace ipi;

namespace {

using Clock = std::chrono::steady_clock;

enum class RState { Queued, Admitted, Done };

struct Request {
    uint64_t ticket = 0;
    int64_t S = 0;
    int32_t A = 0;
    int64_t nnz = 0;
    double gamma = 0;
    uint32_t flags = 0;
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> col;
    std::vector<double> val, g;
    ipi_solve_opts opts{};
    int64_t footprint = 0;
    bool batchable = false;
    RState state = RState::Queued;
    bool cancel = false;
    ipi_status status = IPI_E_PENDING;
    std::string error;  // message of a failed solve
    std::vector<double> V;
    std::vector<int32_t> pi;
    ipi_solve_info info{};
    ipi_latency lat{};
    // device side while admitted
    ipi_mdp_s* mdp = nullptr;
    double* dV = nullptr;
    int32_t* dpi = nullptr;
};

}  // namespace

struct ipi_server_s {
    ipi_server_opts o{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_sched, cv_work, cv_small, cv_done;
    std::deque<Request*> queue;        // submitted, not admitted
    std::deque<Request*> ready;        // admitted, for the single-MDP workers
    std::deque<Request*> small_ready;  // admitted, for the batched solver
    std::map<uint64_t, std::unique_ptr<Request>> all;
    int64_t used = 0;
    int active = 0;
    bool stop = false;
    uint64_t next_ticket = 1;
    Clock::time_point t0;
    std::thread sched, batcher;
    std::vector<std::thread> workers;

    double now_ms() const { return std::chrono::duration<double, std::milli>(Clock::now() - t0).count(); }
};

namespace {

void scheduler_loop(ipi_server_s* s) {
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_sched.wait(lk, [&] { return s->stop || !s->queue.empty(); });
        if (s->stop) {
            // no new admissions after shutdown starts: cancel what is queued
            for (Request* r : s->queue) {
                r->state = RState::Done;
                r->status = IPI_E_CANCELLED;
                r->lat.done_ms = s->now_ms();
            }
            s->queue.clear();
            s->cv_done.notify_all();
            return;
        }
        // admit: the head, then bounded backfill behind it
        bool any = false;
        const size_t look = std::min(s->queue.size(), (size_t)std::max(1, 1 + s->o.backfill));
        for (size_t i = 0; i < look && i < s->queue.size();) {
            Request* r = s->queue[i];
            if (r->cancel) {
                r->state = RState::Done;
                r->status = IPI_E_CANCELLED;
                r->lat.done_ms = s->now_ms();
                s->queue.erase(s->queue.begin() + (long)i);
                s->cv_done.notify_all();
                continue;
            }
            if (s->active < s->o.max_slots && r->footprint <= s->o.hbm_budget_bytes - s->used) {
                s->used += r->footprint;
                s->active += 1;
                r->state = RState::Admitted;
                r->lat.admit_ms = s->now_ms();
                // small requests join the running batched solve at its next
                // chunk boundary; the others take a worker of their own
                if (r->batchable) s->small_ready.push_back(r);
                else s->ready.push_back(r);
                s->queue.erase(s->queue.begin() + (long)i);
                any = true;
                continue;
            }
            ++i;
        }
        if (!any) {
            // wait for memory or a slot to free up (a finished request notifies)
            s->cv_sched.wait(lk);
            continue;
        }
        s->cv_work.notify_all();
        s->cv_small.notify_all();
    }
}

// device side of an admitted request: the MDP (uploaded on stream st) and
// its output buffers
void materialise(Request* r, hipStream_t st) {
    r->mdp = create_mdp(r->S, r->A, r->nnz, r->row_ptr.data(), r->col.data(), r->val.data(), r->g.data(), r->gamma,
                        (r->flags & (IPI_VAL_FP32 | IPI_VAL_FP32_ONLY)) | IPI_NO_VALIDATE, st);
    // resident (create returns after the upload): the host copy is not needed
    std::vector<int64_t>().swap(r->row_ptr);
    std::vector<int32_t>().swap(r->col);
    std::vector<double>().swap(r->val);
    std::vector<double>().swap(r->g);
    std::lock_guard<std::recursive_mutex> lk(device_sync_mutex());
    IPI_HIP(hipMalloc(&r->dV, sizeof(double) * (size_t)r->S));
    IPI_HIP(hipMalloc(&r->dpi, sizeof(int32_t) * (size_t)r->S));
}

// results back to the host; the request's done time is stamped when they
// have arrived (before its device memory is released)
void collect(ipi_server_s* s, Request* r, hipStream_t st) {
    r->V.resize((size_t)r->S);
    r->pi.resize((size_t)r->S);
    IPI_HIP(hipMemcpyAsync(r->V.data(), r->dV, sizeof(double) * (size_t)r->S, hipMemcpyDeviceToHost, st));
    IPI_HIP(hipMemcpyAsync(r->pi.data(), r->dpi, sizeof(int32_t) * (size_t)r->S, hipMemcpyDeviceToHost, st));
    IPI_HIP(hipStreamSynchronize(st));
    r->lat.done_ms = s->now_ms();
}

// releases the request's device memory after waiting for its own stream
// only (no device-wide synchronisation), then its budget and slot
void retire(ipi_server_s* s, Request* r, hipStream_t st) {
    hipStreamSynchronize(st);
    {
        std::lock_guard<std::recursive_mutex> lk(device_sync_mutex());
        hipFree(r->dV);
        hipFree(r->dpi);
        release_mdp(r->mdp);
    }
    r->dV = nullptr;
    r->dpi = nullptr;
    r->mdp = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (r->cancel) r->status = IPI_E_CANCELLED;
        if (r->lat.done_ms == 0.0) r->lat.done_ms = s->now_ms();
        r->state = RState::Done;
        s->used -= r->footprint;
        s->active -= 1;
        // inputs of a request that failed before its upload
        std::vector<int64_t>().swap(r->row_ptr);
        std::vector<int32_t>().swap(r->col);
        std::vector<double>().swap(r->val);
        std::vector<double>().swap(r->g);
    }
    s->cv_done.notify_all();
    s->cv_sched.notify_all();
}

void fail(Request* r, const Error& e) {
    r->status = e.status;
    r->error = e.what();
}

void worker_loop(ipi_server_s* s) {
    hipSetDevice(s->device);
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
    for (;;) {
        Request* r = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stop || !s->ready.empty(); });
            if (s->ready.empty()) {
                if (s->stop) break;
                continue;
            }
            r = s->ready.front();
            s->ready.pop_front();
        }
        r->lat.start_ms = s->now_ms();
        r->lat.batched = 0;
        r->lat.batch_size = 1;
        try {
            materialise(r, st);
            r->status = solve_single(r->mdp, r->opts, r->dV, r->dpi, &r->info, st);
            if (r->status != IPI_OK) r->error = ipi_last_error();
            collect(s, r, st);
        } catch (const Error& e) {
            fail(r, e);
        } catch (...) {
            r->status = IPI_E_DEVICE;
            r->error = "unknown exception";
        }
        retire(s, r, st);
    }
    if (st) hipStreamDestroy(st);
}

// Continuous batching: one thread owns the batched solver.  Between chunks
// of rounds it admits waiting small requests into free slots (they start at
// the next chunk while the others keep running) and hands back each member
// as soon as its own solve has finished.
void batch_loop(ipi_server_s* s) {
    hipSetDevice(s->device);
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
    std::unique_ptr<BatchEngine> eng;
    try {
        eng.reset(new BatchEngine(std::max(1, s->o.max_batch), st));
    } catch (const Error&) {
        eng.reset();
    }
    std::vector<Request*> member((size_t)std::max(1, s->o.max_batch), nullptr);
    for (;;) {
        std::vector<Request*> joining;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            const bool idle = !eng || eng->active() == 0;
            if (idle)
                s->cv_small.wait(lk, [&] { return s->stop || !s->small_ready.empty(); });
            if (s->stop && s->small_ready.empty() && idle) break;
            while (!s->small_ready.empty() && eng && eng->active() + (int)joining.size() < eng->capacity()) {
                joining.push_back(s->small_ready.front());
                s->small_ready.pop_front();
            }
            if (!eng) {  // no engine: every small request fails
                while (!s->small_ready.empty()) {
                    joining.push_back(s->small_ready.front());
                    s->small_ready.pop_front();
                }
            }
        }
        for (Request* r : joining) {
            r->lat.start_ms = s->now_ms();
            r->lat.batched = 1;
            try {
                IPI_REQUIRE(eng != nullptr, IPI_E_DEVICE, "the batched solver could not be set up");
                materialise(r, st);
                const int slot = eng->add(r->mdp, r->opts, r->dV, r->dpi);
                member[(size_t)slot] = r;
                r->lat.batch_size = eng->active();
            } catch (const Error& e) {
                fail(r, e);
                retire(s, r, st);
            }
        }
        if (!eng || eng->active() == 0) continue;
        std::vector<int> fin;
        try {
            fin = eng->step();
        } catch (const Error& e) {
            // a device error ends every member of the batch
            for (size_t i = 0; i < member.size(); ++i) {
                if (!member[i]) continue;
                fail(member[i], e);
                retire(s, member[i], st);
                member[i] = nullptr;
            }
            eng.reset();
            try {
                eng.reset(new BatchEngine(std::max(1, s->o.max_batch), st));
            } catch (const Error&) {
                eng.reset();
            }
            continue;
        }
        for (int slot : fin) {
            Request* r = member[(size_t)slot];
            member[(size_t)slot] = nullptr;
            try {
                eng->take(slot, &r->status, &r->info);
                if (r->status != IPI_OK) r->error = ipi_last_error();
                collect(s, r, st);
            } catch (const Error& e) {
                fail(r, e);
            }
            retire(s, r, st);
        }
        // members cancelled while running leave at the chunk boundary
        for (size_t i = 0; i < member.size(); ++i) {
            Request* r = member[i];
            if (!r) continue;
            bool cancel;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                cancel = r->cancel;
            }
            if (!cancel) continue;
            member[i] = nullptr;
            try {
                eng->drop((int)i);
            } catch (const Error&) {
            }
            r->status = IPI_E_CANCELLED;
            retire(s, r, st);
        }
    }
    eng.reset();
    if (st) hipStreamDestroy(st);
}

bool batch_compatible(const ipi_solve_opts& o, int32_t A) {
    return (o.inner == IPI_INNER_GMRES || o.inner == IPI_INNER_RICHARDSON) && o.pc == IPI_PC_NONE &&
           o.mode == IPI_MINCOST && (o.inner != IPI_INNER_GMRES || o.gmres_restart <= 32) && A <= 1024;
}

}  // namespace

#define IPI_GUARD_BEGIN try {
#define IPI_GUARD_END                              \
    }                                              \
    catch (const ipi::Error& e) {                  \
        set_last_error(e.what());                  \
        return e.status;                           \
    }                                              \
    catch (const std::bad_alloc&) {                \
        set_last_error("host allocation failed");  \
        return IPI_E_OOM;                          \
    }                                              \
    catch (const std::exception& e) {              \
        set_last_error(e.what());                  \
        return IPI_E_DEVICE;                       \
    }

extern "C" {

void ipi_server_opts_default(ipi_server_opts* o) {
    if (!o) return;
    o->hbm_budget_bytes = (int64_t)200 << 30;
    o->max_slots = 16;
    o->n_streams = 4;
    o->small_nnz_threshold = 8 << 20;
    o->max_batch = 32;
    o->backfill = 4;
}

ipi_status ipi_server_create(const ipi_server_opts* opts, ipi_server_t* out) {
    IPI_GUARD_BEGIN
    IPI_REQUIRE(opts && out, IPI_E_INVALID_ARG, "NULL argument");
    IPI_REQUIRE(opts->hbm_budget_bytes > 0 && opts->max_slots >= 1 && opts->n_streams >= 1 && opts->n_streams <= 16 &&
                    opts->max_batch >= 1 && opts->backfill >= 0 && opts->small_nnz_threshold >= 0,
                IPI_E_INVALID_ARG, "bad server options");
    auto* s = new ipi_server_s();
    s->o = *opts;
    hipGetDevice(&s->device);
    s->t0 = Clock::now();
    s->sched = std::thread(scheduler_loop, s);
    s->batcher = std::thread(batch_loop, s);
    for (int i = 0; i < opts->n_streams; ++i) s->workers.emplace_back(worker_loop, s);
    *out = s;
    return IPI_OK;
    IPI_GUARD_END
}

ipi_status ipi_server_submit(ipi_server_t s, int64_t S, int32_t A, int64_t nnz, const int64_t* row_ptr,
                             const int32_t* col, const double* val, const double* g, double gamma, uint32_t flags,
                             const ipi_solve_opts* opts, uint64_t* ticket) {
    IPI_GUARD_BEGIN
    IPI_REQUIRE(s && opts && ticket, IPI_E_INVALID_ARG, "NULL argument");
    IPI_REQUIRE(!(flags & (IPI_DEVICE_PTRS | IPI_BORROW)), IPI_E_INVALID_ARG, "server requests take host arrays");
    IPI_REQUIRE(opts->v0 == nullptr, IPI_E_INVALID_ARG, "server requests start from V_0 = 0");
    int32_t kmax = 0;
    validate_host_arrays(S, A, nnz, row_ptr, col, val, g, gamma, flags, &kmax);
    auto r = std::make_unique<Request>();
    r->S = S;
    r->A = A;
    r->nnz = nnz;
    r->gamma = gamma;
    // fp32_mixed requests keep float32 values only (the FP64 ones are never
    // uploaded; the result states its bound from the rounding of P);
    // fp32_inner requests keep both (the batched solver reads the float copy)
    r->flags = flags;
    if (opts->precision == IPI_FP32_MIXED) r->flags |= IPI_VAL_FP32_ONLY;
    else if (opts->precision == IPI_FP32_INNER) r->flags |= IPI_VAL_FP32;
    r->opts = *opts;
    r->batchable = nnz <= s->o.small_nnz_threshold && batch_compatible(*opts, A);
    ipi_solve_opts fo = *opts;
    if (r->batchable) fo.gmres_restart = 32;
    r->footprint = ipi_footprint_bytes(S, A, nnz, kmax, &fo) + 16 * S;
    if (r->flags & IPI_VAL_FP32_ONLY) r->footprint -= 8 * nnz;  // no FP64 values held
    IPI_REQUIRE(r->footprint <= s->o.hbm_budget_bytes, IPI_E_TOO_LARGE,
                "request footprint exceeds the server's HBM budget");
    r->row_ptr.assign(row_ptr, row_ptr + S * (int64_t)A + 1);
    r->col.assign(col, col + nnz);
    r->val.assign(val, val + nnz);
    r->g.assign(g, g + S * (int64_t)A);
    std::lock_guard<std::mutex> lk(s->mu);
    IPI_REQUIRE(!s->stop, IPI_E_INVALID_ARG, "server is shutting down");
    r->ticket = s->next_ticket++;
    r->lat.arrival_ms = s->now_ms();
    *ticket = r->ticket;
    s->queue.push_back(r.get());
    s->all[r->ticket] = std::move(r);
    s->cv_sched.notify_all();
    return IPI_OK;
    IPI_GUARD_END
}

ipi_status ipi_server_poll(ipi_server_t s, uint64_t ticket, int32_t* done) {
    IPI_GUARD_BEGIN
    IPI_REQUIRE(s && done, IPI_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return IPI_E_NOT_FOUND;
    *done = it->second->state == RState::Done ? 1 : 0;
    return IPI_OK;
    IPI_GUARD_END
}

ipi_status ipi_server_wait(ipi_server_t s, uint64_t ticket, double* V, int32_t* pi, ipi_solve_info* info,
                           ipi_latency* lat) {
    IPI_GUARD_BEGIN
    IPI_REQUIRE(s, IPI_E_INVALID_ARG, "NULL argument");
    std::unique_ptr<Request> r;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->all.find(ticket);
        if (it == s->all.end()) return IPI_E_NOT_FOUND;
        Request* rp = it->second.get();
        s->cv_done.wait(lk, [&] { return rp->state == RState::Done; });
        r = std::move(it->second);
        s->all.erase(it);
    }
    if (V && !r->V.empty()) std::memcpy(V, r->V.data(), sizeof(double) * (size_t)r->S);
    if (pi && !r->pi.empty()) std::memcpy(pi, r->pi.data(), sizeof(int32_t) * (size_t)r->S);
    if (info) *info = r->info;
    if (lat) *lat = r->lat;
    if (r->status != IPI_OK) set_last_error(r->error);
    return r->status;
    IPI_GUARD_END
}

ipi_status ipi_server_cancel(ipi_server_t s, uint64_t ticket) {
    IPI_GUARD_BEGIN
    IPI_REQUIRE(s, IPI_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return IPI_E_NOT_FOUND;
    Request* r = it->second.get();
    r->cancel = true;
    if (r->state == RState::Queued) {
        for (auto q = s->queue.begin(); q != s->queue.end(); ++q)
            if (*q == r) {
                s->queue.erase(q);
                break;
            }
        r->state = RState::Done;
        r->status = IPI_E_CANCELLED;
        r->lat.done_ms = s->now_ms();
        s->cv_done.notify_all();
    }
    return IPI_OK;
    IPI_GUARD_END
}

ipi_status ipi_server_destroy(ipi_server_t s) {
    IPI_GUARD_BEGIN
    if (!s) return IPI_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_sched.notify_all();
    s->cv_work.notify_all();
    s->cv_small.notify_all();
    if (s->sched.joinable()) s->sched.join();
    s->cv_work.notify_all();
    s->cv_small.notify_all();
    for (auto& t : s->workers)
        if (t.joinable()) t.join();
    if (s->batcher.joinable()) s->batcher.join();
    delete s;
    return IPI_OK;
    IPI_GUARD_END
}

}  // extern "C"
