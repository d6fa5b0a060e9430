// Serving loop: continuous batching of packed matrix products and sign/ReLU
// evaluations on one device.
//
// A host thread owns execution.  Submitted requests wait in FIFO order.  Requests with
// the same operation, parameters and level are one type; a type is ready once min_batch
// of its requests wait or its oldest has waited max_wait (the batching window is per
// type, so a mix of many types still forms full cohorts).  Ready requests are admitted
// in arrival order while the summed device footprint of in-flight requests stays within
// the budget; admitted requests of one type form a cohort that runs in lockstep (group
// kernels, keys and masks read once per cohort).
// Each round advances every active cohort by one phase (Step 1 of a product, then a
// chunk of Step 2-3 rounds, then the final relinearisation/RS; one g_d composition of
// a sign evaluation), so requests that arrive while others are on the device start at
// the next round and their kernels interleave with the running cohorts on the stream.
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
    std::vector<uint64_t> ids;
    MatmulJob mj;
    SignJob sj;
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
    std::condition_variable cv;
    std::deque<uint64_t> pending;
    std::map<uint64_t, Req> reqs;
    std::vector<Cohort> active;
    uint64_t inflight = 0, next_id = 1;
    bool stop = false;
    std::thread th;
};

static size_t footprint(const Ctx* c, const he_request& r, int level) {
    const size_t ct = 2 * (size_t)(level + 1) * c->N * 8;
    const int beta = (level + 1 + c->alpha - 1) / c->alpha;
    const size_t lift = (size_t)beta * (level + 1 + c->n_p) * c->N * 8;
    if (r.op == HE_REQ_MATMUL) {
        // Step-1 baby steps, the Step-3 baby rotations of B0 kept across blocks, temporaries,
        // the Step-2 mask pairs that share one ModDown (their extended-basis sums and results),
        // and the lifts of A0 and B0 beside a rotation-sum term waiting for its partner
        const int bg = c->step3_baby((int)r.h);
        const size_t ext = 2 * (size_t)(level + 1 + c->n_p) * c->N * 8;  // a hoisted rotation sum
        const size_t pb = (size_t)std::max(1, c->pair_batch);
        return (size_t)(c->bsgs((int)r.h) + (bg < (int)r.h ? bg : 0) + 11 + pb) * ct + 4 * lift + (1 + pb) * ext;
    }
    return 12 * ct + 2 * lift;
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

static void serve_loop(he_server* S) {
    for (;;) {
        std::vector<Cohort> fresh;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            std::map<ReqKey, bool> ready;
            bool any = false;
            for (;;) {
                if (S->stop && S->pending.empty() && S->active.empty()) return;
                if (!S->pending.empty()) {
                    double next_close = 0;
                    const double now = now_s();
                    ready = ready_types(S, now, &next_close);
                    any = false;
                    for (auto& kv : ready) any |= kv.second;
                    if (any || !S->active.empty()) break;
                    S->cv.wait_for(lk, std::chrono::duration<double>(std::max(0.0, next_close - now)));
                } else {
                    if (!S->active.empty()) break;
                    S->cv.wait(lk);
                }
            }
            // admission of ready requests in arrival order while the footprint fits; the
            // others keep their place in the queue
            std::map<ReqKey, size_t> slot;
            std::deque<uint64_t> keep;
            bool full = false;
            while (!S->pending.empty()) {
                const uint64_t id = S->pending.front();
                S->pending.pop_front();
                Req& q = S->reqs[id];
                if (full || !ready[q.key]) {
                    keep.push_back(id);
                    continue;
                }
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
                    if (q.r.op == HE_REQ_MATMUL) {
                        co.mj.h = (int)q.r.h;
                        co.mj.lvl = lvl;
                    } else {
                        co.sj.d = (int)q.r.d;
                        co.sj.k = (int)q.r.k;
                        co.sj.mode = (int)q.r.mode;
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
        // one round: every active cohort advances one phase
        std::vector<std::pair<size_t, he_status>> finished;
        {
            std::lock_guard<std::recursive_mutex> lk(S->c->api_mu);
            for (size_t i = 0; i < S->active.size(); ++i) {
                Cohort& co = S->active[i];
                try {
                    const bool done = co.op == HE_REQ_MATMUL ? S->c->matmul_step(co.mj, S->k_chunk) : S->c->sign_step(co.sj);
                    if (done) finished.push_back({i, HE_OK});
                } catch (const HeError& e) {
                    finished.push_back({i, e.s});
                } catch (const LaunchError&) {
                    finished.push_back({i, HE_EDEVICE});
                } catch (...) {
                    finished.push_back({i, HE_EDEVICE});
                }
            }
            if (hipStreamSynchronize(S->c->stream) != hipSuccess) {
                (void)hipGetLastError();
                for (size_t i = 0; i < S->active.size(); ++i) finished.push_back({i, HE_EDEVICE});
            }
        }
        const double t = now_s();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            std::vector<bool> drop(S->active.size(), false);
            for (auto& f : finished) {
                if (drop[f.first]) continue;
                drop[f.first] = true;
                Cohort& co = S->active[f.first];
                auto& res = co.op == HE_REQ_MATMUL ? co.mj.result : co.sj.result;
                for (size_t m = 0; m < co.ids.size(); ++m) {
                    Req& q = S->reqs[co.ids[m]];
                    q.status = f.second;
                    if (f.second == HE_OK && m < res.size()) q.result = res[m];
                    q.done = true;
                    q.t_done = t;
                    q.keep_a.reset();
                    q.keep_b.reset();
                    S->inflight -= q.footprint;
                }
            }
            std::vector<Cohort> keep;
            for (size_t i = 0; i < S->active.size(); ++i)
                if (!drop[i]) keep.push_back(std::move(S->active[i]));
            S->active.swap(keep);
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
    *out = S;
    return HE_OK;
}

he_status he_serve_submit(he_server* S, const he_request* req, uint64_t* ticket) {
    if (!S || !req || !ticket || !req->a) return HE_EINVAL;
    if (req->op == HE_REQ_MATMUL && !req->b) return HE_EINVAL;
    if (req->op > HE_REQ_SIGN) return HE_EINVAL;
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
    } else {
        if (q.r.d < 1 || q.r.d > 7 || q.r.mode > 1) return HE_EINVAL;
        int nb = 0;
        while ((1u << nb) <= q.r.d) ++nb;
        if (q.a->level < (int)(q.r.k * (nb + 1) + q.r.mode)) return HE_ELEVEL;
    }
    const int lvl = q.r.op == HE_REQ_MATMUL ? std::min(q.a->level, q.b->level) : q.a->level;
    q.footprint = footprint(S->c, q.r, lvl);
    if (S->budget && q.footprint > S->budget) return HE_ENOMEM;
    q.key = std::make_tuple(q.r.op, q.r.op == HE_REQ_MATMUL ? q.r.h : 0u, q.r.op == HE_REQ_SIGN ? q.r.d : 0u,
                            q.r.op == HE_REQ_SIGN ? q.r.k : 0u, q.r.op == HE_REQ_SIGN ? q.r.mode : 0u, lvl);
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
    {
        std::lock_guard<std::recursive_mutex> lk(S->c->api_mu);
        delete S;
    }
    return HE_OK;
}

}  // extern "C"
