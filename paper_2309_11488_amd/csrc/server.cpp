// Request server: continuous admission of BiCGStab-ILU0 solves of mixed
// sizes under a device-memory budget.
//
// Patterns are registered once (a reservoir model keeps its sparsity
// pattern across Newton steps); requests name one and bring values, b and x.
// Requests are queued in arrival order.  Each of `max_slots` worker threads
// owns a HIP stream; it takes the request at the head of the queue as soon
// as either an idle resident instance of the request's pattern exists, or a
// new instance fits in the budget.  An instance is a (matrix,
// preconditioner) handle pair with its factors and Krylov workspace; it
// stays resident after its request, so the steady state allocates nothing
// and runs no analysis.  All instances of one pattern share one analysis
// (ilu0_analyse_shared), which is reserved once per pattern.  When the head
// of the queue does not fit, idle instances are freed, least recently used
// first; a pattern whose single instance exceeds the budget is refused at
// registration, so admission cannot deadlock.  The budget is an account of
// the footprints: an evicted instance's memory is released right after the
// admission that evicted it.
//
// Inputs are borrowed: values, b and x live where `mem` says and must stay
// valid until the request completes.  Slots launch their kernels directly
// (no graph capture): a capture on one slot's stream would be invalidated
// by another slot's device-synchronising calls (frees, synchronous copies).
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
#include "analysis.h"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

uint64_t words_hash(const std::vector<int32_t> &a, const std::vector<int32_t> &b) {
    uint64_t h = 1469598103934665603ull;
    for (const auto *v : {&a, &b})
        for (int32_t w : *v) h = (h ^ (uint32_t)w) * 1099511628211ull;
    return h;
}

struct Instance;

struct Pattern {
    int32_t id = 0, n = 0, nnzb = 0;
    std::vector<int32_t> rowptr, colidx;
    uint64_t hash = 0;
    size_t inst_bytes = 0, an_bytes = 0;
    std::vector<Instance *> inst;   // resident instances and those being created
    bool tuned = false;             // a tuner ran or runs; `opts` valid once opts_version > 0
    bool tune_done = false;         // the tuner has ended (requests of the pattern wait for it)
    int opts_version = 0;
    int32_t opts[5] = {};           // spmv variant, sweep variant, sweep tiles, sweep grid, reduce split
};

struct Instance {
    Pattern *pat = nullptr;
    bcsr_t A = nullptr;
    ilu0_t M = nullptr;
    bool ready = false;   // handles created
    bool busy = false;    // a request runs on it, or it is being created
    int pins = 0;         // creators reading its analysis
    uint64_t seq = 0;     // creation order
    int opts_version = 0;
    size_t bytes = 0;
    uint64_t last_use = 0;
};

struct Request {
    int64_t id = 0;
    Pattern *pat = nullptr;
    int32_t mem = RS_MEM_HOST, max_iter = 200;
    const double *vals = nullptr, *b = nullptr;
    double *x = nullptr;
    double reduction = 1e-2;
    Clock::time_point t_submit;
    bool done = false;
    int32_t status = RS_OK;
    solve_info info{};
    server_timing timing{};
};

struct Slot {
    int id = 0;
    hipStream_t stream = nullptr;
    std::thread th;
};

void destroy_instance(Instance *I) {
    ilu0_destroy(I->M);
    bcsr_destroy(I->A);
    delete I;
}

// An instance of P created before `self` is still being created (only the
// earliest creator analyses; later ones wait for it and share).
bool earlier_creating(const Pattern *P, const Instance *self) {
    for (const Instance *J : P->inst)
        if (J->seq < self->seq && !J->ready) return true;
    return false;
}

Instance *ready_instance(const Pattern *P) {
    for (Instance *J : P->inst)
        if (J->ready) return J;
    return nullptr;
}

}  // namespace

struct rs_server {
    server_config cfg{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_ready, cv_tuned;
    std::deque<Request *> queue;
    std::unordered_map<int64_t, Request *> live;
    std::vector<Pattern *> patterns;
    std::vector<Slot *> slots;
    size_t reserved = 0, peak = 0;
    int64_t next_id = 1;
    int64_t completed = 0, running = 0, instances = 0, created = 0, evicted = 0, analyses = 0;
    uint64_t clock = 0;
    bool stopping = false;
};

// Device bytes of one instance while it is resident, as allocated by
// bcsr_create / ilu0_factor / bicgstab_solve: the caller-order matrix, its
// reordered copy and FP64 factors (plus FP32 copies), the Krylov vectors,
// sweep intermediate, staging and reduction partials.
static size_t instance_bytes(int32_t n, int32_t nnzb, int32_t precision) {
    const double N = n, Z = nnzb;
    const double vec = 3.0 * N + 1024.0;
    double b = 72 * Z + 4 * (N + Z)                  // caller's matrix
               + 72 * Z                              // reordered copy
               + 72 * Z                              // FP64 factors (L, U, inv(U_ii))
               + 8 * (10 * vec + 2 * 3 * N)          // Krylov vectors, sweep intermediate, staging
               + 8 * (2 * N / 21 + 8192)             // reduction partials
               + (1 << 20);                          // small buffers
    if (precision == RS_PREC_FP32_FACTORS) b += 36 * Z;
    else b += 8 * 2 * vec;                           // lower parts of the second application (two-level patterns)
    return (size_t)b;
}

// Device bytes of a pattern's shared analysis: permutation, reordered
// pattern, sweep schedules and factor update lists (a bound for 7-point
// patterns with non-neighbour connections).
static size_t analysis_bytes(int32_t n, int32_t nnzb) {
    return (size_t)(4 * (8.0 * nnzb + 14.0 * n)) + (1 << 16);
}

static bool hard_error(int st) { return st < 0 && st != RS_ZERO_PIVOT && st != RS_NON_FINITE; }

// Under the lock: take the head request if it can run now, on an idle
// resident instance of its pattern or on a new one (returned not ready).
// Idle instances freed to make room are appended to `victims`; the caller
// destroys them after unlocking.
static Request *admit(rs_server *S, Instance **out, std::vector<Instance *> &victims) {
    Request *h = S->queue.front();
    Pattern *P = h->pat;
    Instance *idle = nullptr;
    for (Instance *I : P->inst)
        if (I->ready && !I->busy && (!idle || I->last_use > idle->last_use)) idle = I;
    if (idle) {
        idle->busy = true;
        S->queue.pop_front();
        *out = idle;
        return h;
    }
    for (;;) {
        const size_t need = P->inst_bytes + (P->inst.empty() ? P->an_bytes : 0);
        if (S->reserved + need <= S->cfg.hbm_budget_bytes) break;
        // free the least recently used idle instance of any pattern
        Instance *v = nullptr;
        for (Pattern *Q : S->patterns)
            for (Instance *I : Q->inst)
                if (I->ready && !I->busy && I->pins == 0 && (!v || I->last_use < v->last_use)) v = I;
        if (!v) return nullptr;
        Pattern *Q = v->pat;
        Q->inst.erase(std::find(Q->inst.begin(), Q->inst.end(), v));
        S->reserved -= v->bytes + (Q->inst.empty() ? Q->an_bytes : 0);
        --S->instances;
        ++S->evicted;
        victims.push_back(v);
    }
    const size_t need = P->inst_bytes + (P->inst.empty() ? P->an_bytes : 0);
    Instance *I = new Instance();
    I->pat = P;
    I->busy = true;
    I->bytes = P->inst_bytes;
    I->seq = ++S->clock;
    P->inst.push_back(I);
    S->reserved += need;
    S->peak = std::max(S->peak, S->reserved);
    ++S->instances;
    ++S->created;
    S->queue.pop_front();
    *out = I;
    return h;
}

// Create the handles of a new instance: share the analysis of a ready
// instance of the pattern, waiting for one that is being created, else
// analyse.
static int create_instance(rs_server *S, Slot *sl, Instance *I) {
    Pattern *P = I->pat;
    int32_t bad = -1;
    int st = bcsr_create(P->n, P->nnzb, 3, 1, P->rowptr.data(), P->colidx.data(), nullptr, RS_MEM_HOST, sl->stream,
                         &I->A, &bad);
    if (st != RS_OK) return st;
    Instance *like = nullptr;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv_ready.wait(lk, [&] { return ready_instance(P) || !earlier_creating(P, I); });
        like = ready_instance(P);
        if (like) ++like->pins;
    }
    if (like) {
        st = ilu0_analyse_shared(I->A, like->M, &I->M);
    } else {
        st = ilu0_analyse(I->A, S->cfg.ordering, &I->M);
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (like) --like->pins;
        else if (st == RS_OK) ++S->analyses;
    }
    if (st == RS_OK) st = ilu0_set_option(I->M, RS_OPT_USE_GRAPH, 0);
    // the factorisation is only queued: its pivot check reaches the request
    // through the solve's status, and the worker does not wait in between
    if (st == RS_OK) st = ilu0_set_option(I->M, RS_OPT_FACTOR_ASYNC, 1);
    return st;
}

static void apply_opts(Instance *I, const int32_t (&o)[5]) {
    (void)bcsr_set_option(I->A, RS_OPT_SPMV_VARIANT, o[0]);
    (void)ilu0_set_option(I->M, RS_OPT_SPMV_VARIANT, o[0]);
    (void)ilu0_set_option(I->M, RS_OPT_SWEEP_VARIANT, o[1]);
    (void)ilu0_set_option(I->M, RS_OPT_SWEEP_TILES, o[2]);
    (void)ilu0_set_option(I->M, RS_OPT_SWEEP_GRID, o[3]);
    (void)ilu0_set_option(I->M, RS_OPT_REDUCE_SPLIT, o[4]);
}

static void slot_main(rs_server *S, Slot *sl) {
    (void)hipSetDevice(S->device);
    for (;;) {
        Request *r = nullptr;
        Instance *I = nullptr;
        std::vector<Instance *> victims;
        bool stop = false;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (;;) {
                if (!S->queue.empty() && (r = admit(S, &I, victims))) break;
                if (S->queue.empty() && S->stopping) {
                    stop = true;
                    break;
                }
                if (!victims.empty()) break;     // free them, then look again
                S->cv_work.wait(lk);
            }
            if (r) ++S->running;
        }
        for (Instance *v : victims) destroy_instance(v);
        if (stop) return;
        if (!r) continue;
        const Clock::time_point t0 = Clock::now();
        r->timing.queue_ms = ms_between(r->t_submit, t0);
        r->timing.slot = sl->id;
        r->timing.resident = I->ready ? 1 : 0;
        Pattern *P = I->pat;
        int st = RS_OK;
        if (!I->ready) {
            st = create_instance(S, sl, I);
            {
                std::lock_guard<std::mutex> lk(S->mu);
                I->ready = st == RS_OK;
            }
            S->cv_ready.notify_all();
        }
        // with autotune, the first request of a pattern tunes it; the others
        // wait here until the tuner has ended, so every result of the
        // pattern comes from the same launch configuration
        bool tune = false;
        if (st == RS_OK && S->cfg.autotune) {
            std::unique_lock<std::mutex> lk(S->mu);
            if (!P->tuned) {
                P->tuned = true;          // one tuner per pattern
                tune = true;
            } else {
                S->cv_tuned.wait(lk, [&] { return P->tune_done; });
            }
        }
        int32_t opts[5];
        int version = 0;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (P->opts_version > I->opts_version) {
                std::memcpy(opts, P->opts, sizeof opts);
                version = P->opts_version;
            }
        }
        if (st == RS_OK && version) {
            apply_opts(I, opts);
            I->opts_version = version;
        }
        const Clock::time_point t1 = Clock::now();
        r->timing.analyse_ms = ms_between(t0, t1);
        if (st == RS_OK) st = bcsr_set_values(I->A, r->vals, 0, 1, r->mem, sl->stream);
        if (st == RS_OK) {
            int32_t bad = -1;
            st = ilu0_factor(I->M, I->A, S->cfg.precision, sl->stream, &bad);
            // the tuner times solves of this factorisation: it must be sound
            if (st == RS_OK && tune) st = ilu0_factor_status(I->M, &bad);
        }
        const Clock::time_point t2 = Clock::now();
        r->timing.factor_ms = ms_between(t1, t2);
        if (tune) {
            // a factorisation that failed tunes nothing; the waiting requests
            // then keep the default configuration
            rs_tune_result tr{};
            const int ts = st == RS_OK ? ilu0_autotune(I->M, I->A, r->b, r->mem, r->reduction, 1, sl->stream, &tr)
                                       : st;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                if (ts == RS_OK) {
                    P->opts[0] = tr.spmv_variant;
                    P->opts[1] = tr.sweep_variant;
                    P->opts[2] = tr.sweep_tiles;
                    P->opts[3] = tr.sweep_grid;
                    P->opts[4] = tr.reduce_split;
                    I->opts_version = ++P->opts_version;
                }
                P->tune_done = true;
            }
            S->cv_tuned.notify_all();
            if (ts != RS_OK && hard_error(ts)) st = ts;
        }
        const Clock::time_point t3 = Clock::now();
        r->timing.tune_ms = ms_between(t2, t3);
        if (st == RS_OK)
            st = bicgstab_solve(I->M, I->A, r->b, r->x, r->reduction, r->max_iter, r->mem, sl->stream, &r->info);
        else
            r->info.status = st;
        const Clock::time_point t4 = Clock::now();
        r->timing.solve_ms = ms_between(t3, t4);
        r->timing.total_ms = ms_between(r->t_submit, t4);
        Instance *dead = nullptr;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            I->busy = false;
            I->last_use = ++S->clock;
            if ((hard_error(st) || !I->ready) && I->pins == 0) {
                // the handles may be unusable: give the instance back
                P->inst.erase(std::find(P->inst.begin(), P->inst.end(), I));
                S->reserved -= I->bytes + (P->inst.empty() ? P->an_bytes : 0);
                --S->instances;
                dead = I;
            }
            r->status = st;
            r->done = true;
            --S->running;
            ++S->completed;
        }
        if (dead) {
            destroy_instance(dead);
            S->cv_ready.notify_all();
        }
        S->cv_done.notify_all();
        S->cv_work.notify_all();
    }
}

extern "C" {

int server_create(const server_config *cfg, server_t *out) {
    if (!cfg || !out || cfg->max_slots < 1 || cfg->max_slots > 64 || cfg->hbm_budget_bytes == 0 ||
        cfg->ordering < 0 || cfg->ordering > RS_ORDER_RCM_LEVEL_SET || (cfg->precision != RS_PREC_FP64 && cfg->precision != RS_PREC_FP32_FACTORS))
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
    *bytes = instance_bytes(n_brows, nnzb, precision);
    return RS_OK;
}

int server_analysis_bytes(int32_t n_brows, int32_t nnzb, size_t *bytes) {
    if (n_brows < 0 || nnzb < 0 || !bytes) return RS_INVALID_ARG;
    *bytes = analysis_bytes(n_brows, nnzb);
    return RS_OK;
}

int server_add_pattern(server_t S, int32_t n_brows, int32_t nnzb, const int32_t *row_ptr, const int32_t *col_idx,
                       int32_t *pattern, int32_t *bad_row) {
    if (bad_row) *bad_row = -1;
    if (!S || !pattern || n_brows < 0 || nnzb < 0 || !row_ptr || (nnzb > 0 && !col_idx)) return RS_INVALID_ARG;
    Pattern *P = new Pattern();
    P->n = n_brows;
    P->nnzb = nnzb;
    P->rowptr.assign(row_ptr, row_ptr + (size_t)n_brows + 1);
    P->colidx.assign(col_idx, col_idx + nnzb);
    int bad = -1;
    const int st = rs::validate_pattern(n_brows, nnzb, P->rowptr.data(), P->colidx.data(), &bad);
    if (st != RS_OK) {
        if (bad_row) *bad_row = bad;
        delete P;
        return st;
    }
    P->hash = words_hash(P->rowptr, P->colidx);
    P->inst_bytes = instance_bytes(n_brows, nnzb, S->cfg.precision);
    P->an_bytes = analysis_bytes(n_brows, nnzb);
    if (P->inst_bytes + P->an_bytes > S->cfg.hbm_budget_bytes) {
        delete P;
        return RS_OUT_OF_MEMORY;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    for (Pattern *Q : S->patterns)
        if (Q->hash == P->hash && Q->n == P->n && Q->nnzb == P->nnzb && Q->rowptr == P->rowptr &&
            Q->colidx == P->colidx) {
            *pattern = Q->id;
            delete P;
            return RS_OK;
        }
    P->id = (int32_t)S->patterns.size();
    S->patterns.push_back(P);
    *pattern = P->id;
    return RS_OK;
}

int server_submit(server_t S, int32_t pattern, const double *vals, const double *b, double *x, double reduction,
                  int32_t max_iter, int32_t mem, int64_t *ticket) {
    if (!S || !ticket || !vals || !b || !x || !(reduction >= 0.0) || max_iter < 0 ||
        (mem != RS_MEM_HOST && mem != RS_MEM_DEVICE))
        return RS_INVALID_ARG;
    Request *r = new Request();
    r->vals = vals;
    r->b = b;
    r->x = x;
    r->mem = mem;
    r->reduction = reduction;
    r->max_iter = max_iter;
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stopping || pattern < 0 || pattern >= (int32_t)S->patterns.size()) {
            delete r;
            return RS_INVALID_ARG;
        }
        r->pat = S->patterns[pattern];
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
    size_t fr = 0, tot = 0;
    if (hipSetDevice(S->device) != hipSuccess || hipMemGetInfo(&fr, &tot) != hipSuccess) fr = tot = 0;
    out->device_used_bytes = tot - fr;
    out->device_total_bytes = tot;
    std::lock_guard<std::mutex> lk(S->mu);
    out->queued = (int64_t)S->queue.size();
    out->running = S->running;
    out->completed = S->completed;
    out->instances = S->instances;
    out->created = S->created;
    out->evicted = S->evicted;
    out->analyses = S->analyses;
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
    for (Pattern *P : S->patterns) {
        for (Instance *I : P->inst) destroy_instance(I);
        delete P;
    }
    for (Slot *sl : S->slots) {
        if (sl->stream) (void)hipStreamDestroy(sl->stream);
        delete sl;
    }
    for (auto &kv : S->live) delete kv.second;
    delete S;
    return RS_OK;
}

}  // extern "C"
