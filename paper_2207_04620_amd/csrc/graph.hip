// A batched product captured once into a HIP graph and replayed.
//
// The capture records every launch and device copy of one he_matmul_batch call on the
// context stream.  The graph's kernels keep reading the inputs' buffers and writing the
// outputs' and temporaries' buffers on every replay, so the graph owns all of them: while the
// capture records, the allocation cache hands out and takes back blocks on the graph's own
// account (GraphBlocks), and the graph keeps the inputs and outputs alive until it is
// destroyed.  Nothing in the product's path clears memory with a memset node; the path has no
// host synchronisation, so it records as is.
#include <hip/hip_runtime.h>

#include <vector>

#include "he_internal.hpp"

struct he_graph {
    he_ctx* ctx = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    GraphBlocks blocks;
    std::vector<CtPtr> keep;  // inputs and outputs: their buffers are the graph's operands
    size_t nodes = 0;
};

extern "C" {

he_status he_matmul_batch_capture(he_ctx* ctx, size_t n, const he_ct* const* a, const he_ct* const* b,
                                  const uint32_t* h, he_graph** out_graph, he_ct** out) {
    if (!ctx || !out_graph || !out || n == 0 || !a || !b || !h) return HE_EINVAL;
    for (size_t i = 0; i < n; ++i) {
        if (!a[i] || !b[i]) return HE_EINVAL;
        if (a[i]->ctx != ctx->c.get() || b[i]->ctx != ctx->c.get()) return HE_EMISMATCH;
    }
    Ctx* c = ctx->c.get();
    auto* g = new he_graph();
    g->ctx = ctx;
    std::vector<CtPtr> res;
    const he_status st = run_guarded(ctx, [&]() {
        if (prof_active()) throw HeError(HE_EUNSUPPORTED);  // launch-timing events would be recorded
        std::vector<const CtData*> va(n), vb(n);
        std::vector<MatShape> sh(n);
        for (size_t i = 0; i < n; ++i) {
            va[i] = a[i]->c.get();
            vb[i] = b[i]->c.get();
            sh[i] = MatShape{(int)h[i], (int)h[i], 1};
            g->keep.push_back(a[i]->c);
            g->keep.push_back(b[i]->c);
        }
        // keys and masks first, with their synchronisations, outside the capture
        for (auto& s1 : sh) {
            c->check_shape(s1);
            c->prepare_shape(s1);
        }
        hip_check(hipStreamSynchronize(c->stream), "capture prepare");
        {
            std::lock_guard<std::mutex> lk(c->pool.m);
            c->pool.capture = &g->blocks;
        }
        struct EndCapture {  // the pool leaves capture mode and the stream stops recording
            Ctx* c;
            he_graph* g;
            bool open = true;
            ~EndCapture() {
                std::lock_guard<std::mutex> lk(c->pool.m);
                c->pool.capture = nullptr;
                if (open) {
                    hipGraph_t tmp = nullptr;
                    (void)hipStreamEndCapture(c->stream, &tmp);
                    if (tmp) (void)hipGraphDestroy(tmp);
                    (void)hipGetLastError();
                }
            }
        } end{c, g};
        // the capture records the context stream alone: no side-stream work inside the graph
        struct NoOverlap {
            Ctx* c;
            int saved, saved_groups;
            ~NoOverlap() {
                c->overlap = saved;
                c->concurrent_groups = saved_groups;
            }
        } no_overlap{c, c->overlap, c->concurrent_groups};
        c->overlap = 0;
        c->concurrent_groups = 0;
        hip_check(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed), "begin capture");
        res = c->matmul_batch(va, vb, sh);
        end.open = false;
        hip_check(hipStreamEndCapture(c->stream, &g->graph), "end capture");
        hip_check(hipGraphGetNodes(g->graph, nullptr, &g->nodes), "graph nodes");
        hip_check(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0), "graph instantiate");
        for (auto& r : res) g->keep.push_back(r);
        // the capture only recorded the work: the first replay computes the first results
        hip_check(hipGraphLaunch(g->exec, c->stream), "graph launch");
    });
    if (st != HE_OK) {
        he_graph_destroy(g);
        return st;
    }
    for (size_t i = 0; i < n; ++i) out[i] = wrap(c, res[i]);
    *out_graph = g;
    return HE_OK;
}

he_status he_graph_launch(he_graph* g) {
    if (!g || !g->exec) return HE_EINVAL;
    return run_guarded(g->ctx, [&]() { hip_check(hipGraphLaunch(g->exec, g->ctx->c->stream), "graph launch"); });
}

he_status he_graph_info(const he_graph* g, size_t* nodes, uint64_t* bytes) {
    if (!g) return HE_EINVAL;
    if (nodes) *nodes = g->nodes;
    if (bytes) {
        uint64_t t = 0;
        for (auto& kv : g->blocks.owned) t += kv.second;
        *bytes = t;
    }
    return HE_OK;
}

void he_graph_destroy(he_graph* g) {
    if (!g) return;
    Ctx* c = g->ctx ? g->ctx->c.get() : nullptr;
    if (c) {
        std::lock_guard<std::recursive_mutex> lk(c->api_mu);
        // queued replays finish before the graph's blocks can serve anything else
        (void)hipStreamSynchronize(c->stream);
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        {
            std::lock_guard<std::mutex> lk2(c->pool.m);
            for (auto& kv : g->blocks.free_)
                for (void* p : kv.second) {
                    c->pool.free_[kv.first].push_back(p);
                    c->pool.cached += kv.first;
                }
        }
        g->keep.clear();  // inputs and outputs the caller no longer holds go back to the cache
    }
    delete g;
}

}  // extern "C"
