// Serving loop: continuous batching of packed matrix products, sign/ReLU evaluations and
// low powers on one device.
//
// An issuing thread owns execution.  Submitted requests wait in FIFO order.  Requests with
// the same operation, parameters and level are one type; a type is ready once min_batch of
// its requests wait or its oldest has waited max_wait (the batching window is per type, so
// a mix of many types still forms full cohorts).  Ready requests are admitted in arrival
// order while the device footprint of in-flight requests stays within the budget; admitted
// requests of one type form a cohort that runs in lockstep (group kernels, keys and masks
// read once per cohort).
// Each round advances every active cohort by one phase (Step 1 of a product, then a chunk
// of Step 2-3 rounds, then the final relinearisation/RS; one g_d composition of a sign
// evaluation), so requests that arrive while others are on the device start at the next
// round and their kernels interleave with the running cohorts on the stream.  Rounds are
// pipelined: the issuing thread never synchronises the stream; it records an event after
// each round and, before issuing the next, waits only for the round before it, so the
// device always has the current round queued while the host prepares the next one.  A
// cohort that has issued its last phase records an event; a completion thread waits for
// these events in order and hands the results out, so a request completes when its own
// kernels are done, not at a round boundary.
// Footprints are measured: while a cohort issues a phase, the allocation cache's in-use and
// peak figures give the bytes the cohort holds and its transient peak; the largest
// per-member figure seen for a type is its admission footprint (a first request of a type is
// admitted on a conservative estimate).
// A request's result is the same operation DAG as running it alone: bit-identical.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <tuple>

#include "he_internal.hpp"

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

typedef std::tuple<uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, int> ReqKey;  // op, h, d, k, mode, level

struct Req {
    he_request r;
    ReqKey key;
    const CtData* a = nullptr;
    const CtData* b = nullptr;
    CtPtr keep_a, keep_b;  // the inputs stay alive while the request is in flight
    double t_submit = 0, t_done = 0;
    size_t footprint = 0;
    he_status status = HE_OK;
    CtPtr result;
    bool done = false, taken = false;
};

struct Cohort {
    uint32_t op = 0;
    ReqKey key;
    std::vector<uint64_t> ids;
    MatmulJob mj;
    SignJob sj;
    int64_t held = 0;   // bytes of the allocation cache the cohort holds between phases
    int64_t peak = 0;   // the most it held at any point of a phase
};

// a cohort whose last phase is queued: its results are handed out once its event completes
struct Done {
    std::vector<uint64_t> ids;
    std::vector<CtPtr> res;
    he_status st = HE_OK;
    hipEvent_t ev = nullptr;
};

}  // namespace

struct he_server {
    he_ctx* ctx = nullptr;
    Ctx* c = nullptr;
    uint64_t budget = 0;
    uint32_t max_batch = 32;
    uint32_t min_batch = 1;
    double max_wait_s = 0;
    int k_chunk = 8;
    std::mutex mu;
    std::condition_variable cv;       // submissions, completions, stop
    std::condition_variable done_cv;  // work for the completion thread
    std::deque<uint64_t> pending;
    std::map<uint64_t, Req> reqs;
    std::vector<Cohort> active;
    std::deque<Done> completing;
    std::map<ReqKey, size_t> measured;  // admission footprint per member, per type
    std::vector<hipEvent_t> ev_free;
    uint64_t inflight = 0, next_id = 1;
    uint64_t peak_cohort_bytes = 0;    // the largest measured cohort footprint
    uint64_t peak_in_use = 0;          // the allocation cache's largest in-use figure while serving
    bool stop = false, issuing_done = false;
    std::thread th, done_th;
};

// a conservative first estimate of a request's device footprint (before its type is measured)
static size_t footprint_estimate(const Ctx* c, const he_request& r, int level) {
    const size_t ct = 2 * (size_t)(level + 1) * c->N * 8;
    const int beta = (level + 1 + c->alpha - 1) / c->alpha;
    const size_t lift = (size_t)beta * (level + 1 + c->n_p) * c->N * 8;
    const size_t ext = 2 * (size_t)(level + 1 + c->n_p) * c->N * 8;  // an extended-basis sum
    if (r.op == HE_REQ_MATMUL) {
        const int bg = c->step3_baby((int)r.h);
        const size_t pb = (size_t)std::max(1, c->pair_batch);
        return 2 * ((size_t)(c->bsgs((int)r.h) + (bg < (int)r.h ? bg : 0) + 11 + pb) * ct + 4 * lift +
                    (1 + pb) * ext);
    }
    return 2 * (12 * ct + 2 * lift + 2 * ext);
}

static size_t footprint(he_server* S, const Req& q) {
    auto it = S->measured.find(q.key);
    return it != S->measured.end() ? it->second : footprint_estimate(S->c, q.r, std::get<5>(q.key));
}

// types whose batching window has closed, and the time at which the next one closes
static std::map<ReqKey, bool> ready_types(he_server* S, double now, double* next_close) {
    std::map<ReqKey, std::pair<size_t, double>> by;  // count, oldest submit time
    for (uint64_t id : S->pending) {
        const Req& q = S->reqs[id];
        auto it = by.find(q.key);
        if (it == by.end())
            by[q.key] = {1, q.t_submit};
        else
            ++it->second.first;
    }
    std::map<ReqKey, bool> ready;
    *next_close = 1e300;
    for (auto& kv : by) {
        const bool r = S->stop || kv.second.first >= S->min_batch || now - kv.second.second >= S->max_wait_s;
        ready[kv.first] = r;
        if (!r) *next_close = std::min(*next_close, kv.second.second + S->max_wait_s);
    }
    return ready;
}

static hipEvent_t take_event(he_server* S) {
    if (!S->ev_free.empty()) {
        hipEvent_t e = S->ev_free.back();
        S->ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// admission of ready requests in arrival order while the footprint fits; the others keep
// their place in the queue (called with S->mu held)
static void admit(he_server* S, const std::map<ReqKey, bool>& ready) {
    std::map<ReqKey, size_t> slot;
    std::vector<Cohort> fresh;
    std::deque<uint64_t> keep;
    bool full = false;
    while (!S->pending.empty()) {
        const uint64_t id = S->pending.front();
        S->pending.pop_front();
        Req& q = S->reqs[id];
        auto rt = ready.find(q.key);
        if (full || rt == ready.end() || !rt->second) {
            keep.push_back(id);
            continue;
        }
        q.footprint = footprint(S, q);
        if (S->budget && S->inflight + q.footprint > S->budget && S->inflight > 0) {
            full = true;  // head of line: nothing behind it overtakes it
            keep.push_back(id);
            continue;
        }
        S->inflight += q.footprint;
        const int lvl = std::get<5>(q.key);
        auto it = slot.find(q.key);
        if (it == slot.end() || fresh[it->second].ids.size() >= S->max_batch) {
            Cohort co;
            co.op = q.r.op;
            co.key = q.key;
            if (q.r.op == HE_REQ_MATMUL) {
                co.mj.h = (int)q.r.h;
                co.mj.lvl = lvl;
            } else {
                co.sj.d = (int)q.r.d;
                co.sj.k = (int)q.r.k;
                co.sj.mode = q.r.op == HE_REQ_POWER ? 3 : (int)q.r.mode;
                co.sj.lvl = lvl;
            }
            fresh.push_back(co);
            slot[q.key] = fresh.size() - 1;
            it = slot.find(q.key);
        }
        Cohort& co = fresh[it->second];
        co.ids.push_back(id);
        if (q.r.op == HE_REQ_MATMUL) {
            co.mj.A.push_back(q.a);
            co.mj.B.push_back(q.b);
        } else {
            co.sj.X.push_back(q.a);
        }
    }
    S->pending.swap(keep);
    for (auto& co : fresh) S->active.push_back(std::move(co));
}

static void serve_loop(he_server* S) {
    hipEvent_t prev_round = nullptr;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (;;) {
                if (S->stop && S->pending.empty() && S->active.empty()) {
                    S->issuing_done = true;
                    S->done_cv.notify_all();
                    lk.unlock();
                    if (prev_round) {
                        (void)hipEventSynchronize(prev_round);
                        (void)hipEventDestroy(prev_round);
                    }
                    return;
                }
                double next_close = 1e300;
                const double now = now_s();
                if (!S->pending.empty()) admit(S, ready_types(S, now, &next_close));
                if (!S->active.empty()) break;
                // nothing to issue: wait for a submission, a completion (budget freed), a
                // closing window or stop
                if (next_close < 1e299)
                    S->cv.wait_for(lk, std::chrono::duration<double>(std::max(0.0, next_close - now)));
                else
                    S->cv.wait(lk);
            }
        }
        // one round: every active cohort advances one phase; a cohort whose last phase is now
        // queued records its completion event right behind its own kernels
        std::vector<std::pair<size_t, he_status>> finished;
        std::vector<hipEvent_t> evs(S->active.size(), nullptr);
        {
            std::lock_guard<std::recursive_mutex> lk(S->c->api_mu);
            for (size_t i = 0; i < S->active.size(); ++i) {
                Cohort& co = S->active[i];
                const size_t in0 = S->c->pool.restart_peak();
                bool done = false;
                he_status st = HE_OK;
                try {
                    // Step-2/3 rounds per phase: large products advance in larger chunks, so that
                    // their number of phases (and rounds) stays near that of the smaller ones
                    const int chunk = std::max(S->k_chunk, co.mj.h / 4);
                    done = co.op == HE_REQ_MATMUL ? S->c->matmul_step(co.mj, chunk) : S->c->sign_step(co.sj);
                } catch (const HeError& e) {
                    st = e.s;
                } catch (const LaunchError&) {
                    st = HE_EDEVICE;
                } catch (...) {
                    st = HE_EDEVICE;
                }
                const auto use = S->c->pool.usage();
                S->peak_in_use = std::max<uint64_t>(S->peak_in_use, use.second);
                co.peak = std::max(co.peak, co.held + (int64_t)use.second - (int64_t)in0);
                co.held += (int64_t)use.first - (int64_t)in0;
                if (done && st == HE_OK) {
                    {
                        std::lock_guard<std::mutex> lk2(S->mu);
                        evs[i] = take_event(S);
                    }
                    if (!evs[i] || hipEventRecord(evs[i], S->c->stream) != hipSuccess) {
                        (void)hipGetLastError();
                        st = HE_EDEVICE;
                    }
                }
                if (st != HE_OK || done) finished.push_back({i, st});
            }
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            std::vector<bool> drop(S->active.size(), false);
            for (auto& f : finished) {
                Cohort& co = S->active[f.first];
                drop[f.first] = true;
                Done d;
                d.ids = co.ids;
                d.st = f.second;
                d.ev = evs[f.first];
                if (f.second == HE_OK) {
                    d.res = co.op == HE_REQ_MATMUL ? co.mj.result : co.sj.result;
                    // the type's footprint per member, as measured
                    const size_t per = (size_t)std::max<int64_t>(co.peak, 0) / std::max<size_t>(1, co.ids.size());
                    size_t& m = S->measured[co.key];
                    m = std::max(m, per);
                    S->peak_cohort_bytes = std::max<uint64_t>(S->peak_cohort_bytes, (uint64_t)std::max<int64_t>(co.peak, 0));
                }
                S->completing.push_back(std::move(d));
            }
            std::vector<Cohort> keep;
            for (size_t i = 0; i < S->active.size(); ++i)
                if (!drop[i]) keep.push_back(std::move(S->active[i]));
            S->active.swap(keep);
        }
        S->done_cv.notify_all();
        // pipelining: the round just issued stays queued while the host prepares the next;
        // the host waits only for the round before it
        hipEvent_t r = nullptr;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            r = take_event(S);
        }
        if (r && hipEventRecord(r, S->c->stream) != hipSuccess) {
            (void)hipGetLastError();
            r = nullptr;
        }
        if (prev_round) {
            (void)hipEventSynchronize(prev_round);
            std::lock_guard<std::mutex> lk(S->mu);
            S->ev_free.push_back(prev_round);
        }
        prev_round = r;
    }
}

// completion thread: waits for the finished cohorts' events in order and hands out results
static void done_loop(he_server* S) {
    for (;;) {
        Done d;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->done_cv.wait(lk, [&] { return !S->completing.empty() || S->issuing_done; });
            if (S->completing.empty()) return;  // issuing has ended and everything is handed out
            d = std::move(S->completing.front());
            S->completing.pop_front();
        }
        if (d.ev && hipEventSynchronize(d.ev) != hipSuccess) {
            (void)hipGetLastError();
            d.st = HE_EDEVICE;
        }
        const double t = now_s();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (d.ev) S->ev_free.push_back(d.ev);
            for (size_t m = 0; m < d.ids.size(); ++m) {
                Req& q = S->reqs[d.ids[m]];
                q.status = d.st;
                if (d.st == HE_OK && m < d.res.size()) q.result = d.res[m];
                q.done = true;
                q.t_done = t;
                q.keep_a.reset();
                q.keep_b.reset();
                S->inflight -= q.footprint;
            }
        }
        S->cv.notify_all();
    }
}

extern "C" {

he_status he_serve_start(he_ctx* ctx, const he_serve_config* cfg, he_server** out) {
    if (!ctx || !out) return HE_EINVAL;
    auto* S = new he_server();
    S->ctx = ctx;
    S->c = ctx->c.get();
    if (cfg) {
        S->budget = cfg->mem_budget_bytes;
        if (cfg->max_batch) S->max_batch = cfg->max_batch;
        if (cfg->min_batch) S->min_batch = std::min(cfg->min_batch, S->max_batch);
        S->max_wait_s = cfg->max_wait_us * 1e-6;
    }
    S->th = std::thread(serve_loop, S);
    S->done_th = std::thread(done_loop, S);
    *out = S;
    return HE_OK;
}

he_status he_serve_submit(he_server* S, const he_request* req, uint64_t* ticket) {
    if (!S || !req || !ticket || !req->a) return HE_EINVAL;
    if (req->op == HE_REQ_MATMUL && !req->b) return HE_EINVAL;
    if (req->op > HE_REQ_POWER) return HE_EINVAL;
    if (req->a->ctx != S->c || (req->b && req->b->ctx != S->c)) return HE_EMISMATCH;
    Req q;
    q.r = *req;
    q.a = req->a->c.get();
    q.b = req->b ? req->b->c.get() : nullptr;
    q.keep_a = req->a->c;
    if (req->b) q.keep_b = req->b->c;
    // validate what the device would reject, before queueing
    if (q.r.op == HE_REQ_MATMUL) {
        const int h = (int)q.r.h;
        if (h < 1 || (h & (h - 1)) || (int64_t)h * h > S->c->N / 2) return HE_ESHAPE;
        if (std::min(q.a->level, q.b->level) < 3) return HE_ELEVEL;
        if (q.a->deg != 1 || q.b->deg != 1) return HE_EMISMATCH;
        int lg = 0;
        while ((1 << lg) < h) ++lg;
        if (!(S->c->prepared_mask.load() & (1u << lg))) {  // first request of this h: make keys and masks
            std::lock_guard<std::recursive_mutex> lk(S->c->api_mu);
            try {
                S->c->prepare_h(h);
            } catch (const HeError& e) {
                return e.s;
            }
        }
    } else if (q.r.op == HE_REQ_SIGN) {
        if (q.r.d < 1 || q.r.d > 7 || q.r.mode > 1) return HE_EINVAL;
        if (q.a->deg != 1) return HE_EMISMATCH;
        int nb = 0;
        while ((1u << nb) <= q.r.d) ++nb;
        if (q.a->level < (int)(q.r.k * (nb + 1) + q.r.mode)) return HE_ELEVEL;
    } else {  // x^2 (depth 1) or x^3 (depth 2)
        if (q.r.k < 2 || q.r.k > 3) return HE_EINVAL;
        if (q.a->deg != 1) return HE_EMISMATCH;
        if (q.a->level < (int)q.r.k - 1) return HE_ELEVEL;
    }
    const int lvl = q.r.op == HE_REQ_MATMUL ? std::min(q.a->level, q.b->level) : q.a->level;
    const bool sg = q.r.op == HE_REQ_SIGN;
    q.key = std::make_tuple(q.r.op, q.r.op == HE_REQ_MATMUL ? q.r.h : 0u, sg ? q.r.d : 0u,
                            q.r.op != HE_REQ_MATMUL ? q.r.k : 0u, sg ? q.r.mode : 0u, lvl);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        q.footprint = footprint(S, q);
    }
    if (S->budget && q.footprint > S->budget) return HE_ENOMEM;
    q.t_submit = std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) return HE_EINVAL;
        const uint64_t id = S->next_id++;
        S->reqs[id] = std::move(q);
        S->pending.push_back(id);
        *ticket = id;
    }
    S->cv.notify_all();
    return HE_OK;
}

he_status he_serve_poll(he_server* S, uint64_t ticket, int* done, he_ct** result, he_status* req_status,
                        double* latency_s) {
    if (!S || !done) return HE_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end() || it->second.taken) return HE_EINVAL;
    Req& q = it->second;
    *done = q.done ? 1 : 0;
    if (!q.done) return HE_OK;
    if (req_status) *req_status = q.status;
    if (latency_s) *latency_s = q.t_done - q.t_submit;
    if (result) *result = (q.status == HE_OK && q.result) ? wrap(S->c, q.result) : nullptr;
    q.taken = true;
    q.result.reset();
    S->reqs.erase(it);
    return HE_OK;
}

he_status he_serve_stop(he_server* S) {
    if (!S) return HE_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->th.joinable()) S->th.join();
    S->done_cv.notify_all();
    if (S->done_th.joinable()) S->done_th.join();
    {
        std::lock_guard<std::recursive_mutex> lk(S->c->api_mu);
        for (hipEvent_t e : S->ev_free) (void)hipEventDestroy(e);
        delete S;
    }
    return HE_OK;
}

he_status he_serve_stats(he_server* S, uint64_t* inflight_bytes, uint64_t* peak_cohort_bytes, uint64_t* peak_in_use,
                         size_t n_types, uint64_t* type_bytes, size_t* n_measured) {
    if (!S) return HE_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (inflight_bytes) *inflight_bytes = S->inflight;
    if (peak_cohort_bytes) *peak_cohort_bytes = S->peak_cohort_bytes;
    if (peak_in_use) *peak_in_use = S->peak_in_use;
    size_t i = 0;
    for (auto& kv : S->measured) {
        if (type_bytes && i < n_types) type_bytes[i] = kv.second;
        ++i;
    }
    if (n_measured) *n_measured = i;
    return HE_OK;
}

}  // extern "C"
