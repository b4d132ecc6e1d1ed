// Request server: continuous admission of BiCGStab-ILU0 solves of mixed
// sizes under a device-memory budget.
//
// Requests are queued in arrival order.  Each of `max_slots` worker threads
// owns a HIP stream and a cached (matrix, preconditioner) handle pair; it
// takes the request at the head of the queue as soon as that request's
// device footprint fits in the budget, so requests that arrive while others
// run are admitted as slots and memory free up, and the work of different
// slots overlaps on the device.  A slot keeps its handles after a request:
// the next request with the same pattern reuses the analysis, schedule,
// buffers and captured graphs and only uploads values, factors and solves.
// When the head of the queue does not fit, idle slots drop their cached
// handles until it does (a request larger than the whole budget is refused
// at submission), so admission cannot deadlock.
//
// Inputs are borrowed: pattern arrays must be host memory; values, b and x
// live where `mem` says, and must stay valid until the request completes.
// Slots launch their kernels directly (no graph capture): a capture on one
// slot's stream would be invalidated by another slot's device-synchronising
// calls (frees, synchronous copies).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/rsolve.h"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

uint64_t pattern_hash(int32_t n, int32_t nnzb, const int32_t *rowptr, const int32_t *colidx) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void *p, size_t bytes) {
        const unsigned char *c = (const unsigned char *)p;
        for (size_t i = 0; i < bytes; ++i) h = (h ^ c[i]) * 1099511628211ull;
    };
    mix(&n, sizeof n);
    mix(&nnzb, sizeof nnzb);
    mix(rowptr, sizeof(int32_t) * ((size_t)n + 1));
    mix(colidx, sizeof(int32_t) * (size_t)nnzb);
    return h;
}

struct Request {
    int64_t id = 0;
    int32_t n = 0, nnzb = 0, mem = RS_MEM_HOST, max_iter = 200;
    const int32_t *rowptr = nullptr, *colidx = nullptr;
    const double *vals = nullptr, *b = nullptr;
    double *x = nullptr;
    double reduction = 1e-2;
    uint64_t hash = 0;
    size_t bytes = 0;
    Clock::time_point t_submit;
    bool done = false;
    int32_t status = RS_OK;
    solve_info info{};
    server_timing timing{};
};

struct Slot {
    int id = 0;
    hipStream_t stream = nullptr;
    bcsr_t A = nullptr;
    ilu0_t M = nullptr;
    uint64_t hash = 0;
    int32_t n = -1, nnzb = -1;
    size_t held = 0;   // bytes of the budget this slot holds (server lock)
    bool tuned = false;
    std::thread th;
    void drop() {      // destroy the cached handles (budget accounting is the caller's)
        ilu0_destroy(M);
        bcsr_destroy(A);
        M = nullptr;
        A = nullptr;
        hash = 0;
        n = nnzb = -1;
        tuned = false;
    }
};

}  // namespace

struct rs_server {
    server_config cfg{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::unordered_map<int64_t, Request *> live;
    std::vector<Slot *> slots;
    size_t reserved = 0, peak = 0;
    int64_t next_id = 1;
    int64_t completed = 0, running = 0;
    bool stopping = false;
};

// Device bytes a request keeps while it is resident: the caller's matrix,
// its reordered copy and factors, the schedule, the Krylov workspace and
// staging, as allocated by bcsr_create / ilu0_analyse / ilu0_factor /
// bicgstab_solve.
static size_t footprint(int32_t n, int32_t nnzb, int32_t precision) {
    const double N = n, Z = nnzb;
    const double vec = 3.0 * N + 1024.0;
    double b = 72 * Z + 4 * (N + Z)                  // caller's matrix
               + 72 * Z                              // reordered copy
               + 72 * Z                              // FP64 factors (L, U, inv(U_ii))
               + 4 * (8 * Z + 14 * N)                // schedule and update lists
               + 8 * (10 * vec + 2 * 3 * N)          // Krylov vectors, sweep intermediate, staging
               + 8 * (2 * N / 21 + 8192)             // reduction partials
               + (1 << 20);                          // small buffers
    if (precision == RS_PREC_FP32_FACTORS) b += 36 * Z;
    return (size_t)b;
}

static bool hard_error(int st) { return st < 0 && st != RS_ZERO_PIVOT && st != RS_NON_FINITE; }

static void slot_main(rs_server *S, Slot *sl) {
    (void)hipSetDevice(S->device);
    for (;;) {
        Request *r = nullptr;
        bool reuse = false;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (;;) {
                if (!S->queue.empty()) {
                    Request *h = S->queue.front();
                    reuse = sl->M && sl->hash == h->hash && sl->n == h->n && sl->nnzb == h->nnzb;
                    const size_t after = reuse ? S->reserved : S->reserved - sl->held + h->bytes;
                    if (after <= S->cfg.hbm_budget_bytes) {
                        S->queue.pop_front();
                        r = h;
                        if (!reuse) sl->held = h->bytes;
                        S->reserved = after;
                        S->peak = std::max(S->peak, S->reserved);
                        ++S->running;
                        break;
                    }
                    if (sl->M) {
                        // the head does not fit: give back this idle slot's handles
                        const size_t freed = sl->held;
                        sl->held = 0;
                        lk.unlock();
                        sl->drop();
                        lk.lock();
                        S->reserved -= freed;
                        S->cv_work.notify_all();
                        continue;
                    }
                } else if (S->stopping) {
                    S->reserved -= sl->held;
                    sl->held = 0;
                    lk.unlock();
                    sl->drop();
                    return;
                }
                S->cv_work.wait(lk);
            }
        }
        const Clock::time_point t0 = Clock::now();
        r->timing.queue_ms = ms_between(r->t_submit, t0);
        r->timing.slot = sl->id;
        int st = RS_OK;
        if (!reuse) {
            sl->drop();
            int32_t bad = -1;
            st = bcsr_create(r->n, r->nnzb, 3, 1, r->rowptr, r->colidx, nullptr, RS_MEM_HOST, sl->stream, &sl->A, &bad);
            if (st == RS_OK) st = ilu0_analyse(sl->A, S->cfg.ordering, &sl->M);
            // other slots allocate, free and copy synchronously at any time,
            // which would invalidate a stream capture: launch directly
            if (st == RS_OK) st = ilu0_set_option(sl->M, RS_OPT_USE_GRAPH, 0);
            if (st == RS_OK) {
                sl->hash = r->hash;
                sl->n = r->n;
                sl->nnzb = r->nnzb;
            }
        }
        const Clock::time_point t1 = Clock::now();
        r->timing.analyse_ms = ms_between(t0, t1);
        if (st == RS_OK) st = bcsr_set_values(sl->A, r->vals, 0, 1, r->mem, sl->stream);
        if (st == RS_OK) {
            int32_t bad = -1;
            st = ilu0_factor(sl->M, sl->A, S->cfg.precision, sl->stream, &bad);
        }
        const Clock::time_point t2 = Clock::now();
        r->timing.factor_ms = ms_between(t1, t2);
        if (st == RS_OK && S->cfg.autotune && !sl->tuned) {
            rs_tune_result tr{};
            st = ilu0_autotune(sl->M, sl->A, r->b, r->mem, r->reduction, 1, sl->stream, &tr);
            sl->tuned = true;
        }
        const Clock::time_point t3 = Clock::now();
        r->timing.tune_ms = ms_between(t2, t3);
        if (st == RS_OK)
            st = bicgstab_solve(sl->M, sl->A, r->b, r->x, r->reduction, r->max_iter, r->mem, sl->stream, &r->info);
        else
            r->info.status = st;
        const Clock::time_point t4 = Clock::now();
        r->timing.solve_ms = ms_between(t3, t4);
        r->timing.total_ms = ms_between(r->t_submit, t4);
        if (hard_error(st)) sl->drop();   // the handles may be unusable
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (hard_error(st)) {
                S->reserved -= sl->held;
                sl->held = 0;
            }
            r->status = st;
            r->done = true;
            --S->running;
            ++S->completed;
        }
        S->cv_done.notify_all();
        S->cv_work.notify_all();
    }
}

extern "C" {

int server_create(const server_config *cfg, server_t *out) {
    if (!cfg || !out || cfg->max_slots < 1 || cfg->max_slots > 64 || cfg->hbm_budget_bytes == 0 ||
        cfg->ordering < 0 || cfg->ordering > 2 || (cfg->precision != RS_PREC_FP64 && cfg->precision != RS_PREC_FP32_FACTORS))
        return RS_INVALID_ARG;
    *out = nullptr;
    rs_server *S = new rs_server();
    S->cfg = *cfg;
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return RS_HIP_ERROR;
    }
    for (int i = 0; i < cfg->max_slots; ++i) {
        Slot *sl = new Slot();
        sl->id = i;
        if (hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) != hipSuccess) {
            delete sl;
            server_destroy(S);
            return RS_HIP_ERROR;
        }
        S->slots.push_back(sl);
    }
    for (Slot *sl : S->slots) sl->th = std::thread(slot_main, S, sl);
    *out = S;
    return RS_OK;
}

int server_request_bytes(int32_t n_brows, int32_t nnzb, int32_t precision, size_t *bytes) {
    if (n_brows < 0 || nnzb < 0 || !bytes) return RS_INVALID_ARG;
    *bytes = footprint(n_brows, nnzb, precision);
    return RS_OK;
}

int server_submit(server_t S, int32_t n_brows, int32_t nnzb, const int32_t *row_ptr, const int32_t *col_idx,
                  const double *vals, const double *b, double *x, double reduction, int32_t max_iter, int32_t mem,
                  int64_t *ticket) {
    if (!S || !ticket || n_brows < 0 || nnzb < 0 || !row_ptr || (nnzb > 0 && !col_idx) || !vals || !b || !x ||
        !(reduction >= 0.0) || max_iter < 0 || (mem != RS_MEM_HOST && mem != RS_MEM_DEVICE))
        return RS_INVALID_ARG;
    Request *r = new Request();
    r->n = n_brows;
    r->nnzb = nnzb;
    r->rowptr = row_ptr;
    r->colidx = col_idx;
    r->vals = vals;
    r->b = b;
    r->x = x;
    r->mem = mem;
    r->reduction = reduction;
    r->max_iter = max_iter;
    r->hash = pattern_hash(n_brows, nnzb, row_ptr, col_idx);
    r->bytes = footprint(n_brows, nnzb, S->cfg.precision);
    if (r->bytes > S->cfg.hbm_budget_bytes) {
        delete r;
        return RS_OUT_OF_MEMORY;
    }
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stopping) {
            delete r;
            return RS_INVALID_ARG;
        }
        r->id = S->next_id++;
        S->live[r->id] = r;
        S->queue.push_back(r);
        *ticket = r->id;
    }
    S->cv_work.notify_all();
    return RS_OK;
}

static int collect(rs_server *S, Request *r, solve_info *info, server_timing *timing) {
    if (info) *info = r->info;
    if (timing) *timing = r->timing;
    const int st = r->status;
    S->live.erase(r->id);
    delete r;
    return st;
}

int server_poll(server_t S, int64_t ticket, solve_info *info, server_timing *timing) {
    if (!S) return RS_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->live.find(ticket);
    if (it == S->live.end()) return RS_INVALID_ARG;
    if (!it->second->done) return RS_PENDING;
    return collect(S, it->second, info, timing);
}

int server_wait(server_t S, int64_t ticket, solve_info *info, server_timing *timing) {
    if (!S) return RS_INVALID_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->live.find(ticket);
    if (it == S->live.end()) return RS_INVALID_ARG;
    Request *r = it->second;
    S->cv_done.wait(lk, [&] { return r->done; });
    return collect(S, r, info, timing);
}

int server_get_stats(server_t S, server_stats *out) {
    if (!S || !out) return RS_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    out->queued = (int64_t)S->queue.size();
    out->running = S->running;
    out->completed = S->completed;
    out->reserved_bytes = S->reserved;
    out->peak_reserved_bytes = S->peak;
    return RS_OK;
}

int server_destroy(server_t S) {
    if (!S) return RS_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
    }
    S->cv_work.notify_all();
    for (Slot *sl : S->slots)
        if (sl->th.joinable()) sl->th.join();
    for (Slot *sl : S->slots) {
        sl->drop();
        if (sl->stream) (void)hipStreamDestroy(sl->stream);
        delete sl;
    }
    for (auto &kv : S->live) delete kv.second;
    delete S;
    return RS_OK;
}

}  // extern "C"
