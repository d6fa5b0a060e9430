// Autotuner of the batched product's scheduling knobs.
//
// Three knobs shape the launches of a lockstep product without changing any result: the number
// of rotation sets that share one key-switch inner-product launch and one ModDown launch
// (pair_batch: Step-2 mask pairs, baby rotations), the cap on members per lockstep group
// (max_group: larger groups read each key and mask once for more members; smaller ones keep
// the working set nearer the device caches), and whether the next Step-2 pair group's inner
// products overlap the current group's ModDown on a second stream (overlap).  The tuner times the batched product of the
// requested shape on the device under each candidate, keeps the fastest, applies it to the
// context and caches it per (ring, chain, shape, batch, device), in the process and optionally
// in a text file.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "he_internal.hpp"

namespace {

std::mutex g_tune_mu;
std::map<std::string, he_tuning> g_tune_cache;

std::string device_name() {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string s = p.gcnArchName;
    for (char& ch : s)
        if (ch == ' ' || ch == ':') ch = '_';
    return s + "_cu" + std::to_string(p.multiProcessorCount);
}

std::string tune_key(const Ctx* c, int h, int level, int batch) {
    std::ostringstream o;
    o << "N" << c->N << "_q" << c->n_q << "_p" << c->n_p << "_a" << c->alpha << "_s" << c->schedule << "_h" << h
      << "_l" << level << "_b" << batch << "_" << device_name();
    return o.str();
}

bool file_lookup(const char* path, const std::string& key, he_tuning* t) {
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream in(line);
        std::string k;
        unsigned pb = 0, mg = 0, ov = 0;
        if ((in >> k >> pb >> mg >> ov) && k == key && pb >= 1 && mg >= 1 && ov <= 1) {
            t->pair_batch = pb;
            t->max_group = mg;
            t->overlap = ov;
            return true;
        }
    }
    return false;
}

}  // namespace

extern "C" {

he_status he_tuning_get(const he_ctx* ctx, he_tuning* out) {
    if (!ctx || !out) return HE_EINVAL;
    out->pair_batch = (uint32_t)ctx->c->pair_batch;
    out->max_group = (uint32_t)ctx->c->max_group;
    out->overlap = (uint32_t)ctx->c->overlap;
    out->concurrent_groups = (uint32_t)ctx->c->concurrent_groups;
    return HE_OK;
}

he_status he_tuning_set(he_ctx* ctx, const he_tuning* t) {
    if (!ctx || !t || t->pair_batch < 1 || t->pair_batch > IP_MAXSET || t->max_group < 1 || t->max_group > 256 ||
        t->overlap > 1 || t->concurrent_groups > 1)
        return HE_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(ctx->c->api_mu);
    ctx->c->pair_batch = (int)t->pair_batch;
    ctx->c->max_group = (int)t->max_group;
    ctx->c->overlap = (int)t->overlap;
    ctx->c->concurrent_groups = (int)t->concurrent_groups;
    return HE_OK;
}

he_status he_autotune(he_ctx* ctx, uint32_t h, uint32_t level, uint32_t batch, const char* cache_path,
                      he_tuning* out, char* report, size_t report_n) {
    if (!ctx || !out || batch < 1 || batch > 256 || h < 1) return HE_EINVAL;
    Ctx* c = ctx->c.get();
    if ((int)level >= c->n_q) return HE_ELEVEL;
    if (level < 3) return HE_ELEVEL;
    const std::string key = tune_key(c, (int)h, (int)level, (int)batch);
    std::string rep = "{\"key\": \"" + key + "\"";
    he_tuning best{};
    best.concurrent_groups = (uint32_t)c->concurrent_groups;  // not a tuned knob
    bool have = false;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            best = it->second;
            have = true;
            rep += ", \"source\": \"process cache\"";
        }
    }
    if (!have && cache_path && *cache_path && file_lookup(cache_path, key, &best)) {
        have = true;
        rep += ", \"source\": \"file cache\"";
    }
    best.concurrent_groups = (uint32_t)c->concurrent_groups;
    he_status st = HE_OK;
    if (!have) {
        st = run_guarded(ctx, [&]() {
            c->check_shape(MatShape{(int)h, (int)h, 1});
            c->prepare_h((int)h);
            // two encryptions of zero shared by every member (the times do not depend on the data)
            std::vector<int64_t> zero(c->N, 0);
            CtPtr a = c->encrypt_coeffs(zero.data(), (int)level, c->scale, 0x7fff0001ull);
            CtPtr b = c->encrypt_coeffs(zero.data(), (int)level, c->scale, 0x7fff0002ull);
            std::vector<const CtData*> va(batch, a.get()), vb(batch, b.get());
            std::vector<MatShape> sh(batch, MatShape{(int)h, (int)h, 1});
            // the context's knobs come back whatever happens to a candidate
            struct Restore {
                Ctx* c;
                int pb, mg, ov;
                ~Restore() {
                    c->pair_batch = pb;
                    c->max_group = mg;
                    c->overlap = ov;
                }
            } restore{c, c->pair_batch, c->max_group, c->overlap};
            hipEvent_t e0, e1;
            hip_check(hipEventCreate(&e0), "tune event");
            hip_check(hipEventCreate(&e1), "tune event");
            double best_ms = 1e300;
            rep += ", \"candidates\": [";
            bool first = true;
            auto time_it = [&]() {
                c->matmul_batch(va, vb, sh);  // warm-up: the cache holds this shape's buffers
                double ms = 1e300;
                for (int rep_i = 0; rep_i < 2; ++rep_i) {
                    hip_check(hipEventRecord(e0, c->stream), "tune record");
                    c->matmul_batch(va, vb, sh);
                    hip_check(hipEventRecord(e1, c->stream), "tune record");
                    hip_check(hipEventSynchronize(e1), "tune sync");
                    float t = 0;
                    hip_check(hipEventElapsedTime(&t, e0, e1), "tune time");
                    ms = std::min(ms, (double)t);
                }
                return ms;
            };
            auto candidate = [&](int pb, int mg, int ov) {
                c->pair_batch = pb;
                c->max_group = mg;
                c->overlap = ov;
                const double ms = time_it();
                char buf[160];
                snprintf(buf, sizeof buf, "%s{\"pair_batch\": %d, \"max_group\": %d, \"overlap\": %d, \"ms\": %.3f}",
                         first ? "" : ", ", pb, mg, ov, ms);
                rep += buf;
                first = false;
                // the fastest wins; a later candidate must be faster by 1 % to displace it
                if (ms < best_ms * 0.99) {
                    best_ms = ms;
                    best.pair_batch = (uint32_t)pb;
                    best.max_group = (uint32_t)mg;
                    best.overlap = (uint32_t)ov;
                }
            };
            // the context's own setting first: another candidate must beat it by 1 % to replace it
            const int pb0 = restore.pb, mg0 = std::min(restore.mg, (int)batch);
            candidate(pb0, mg0, 0);
            const int groups[2] = {(int)batch, (int)batch / 2};
            for (int gi = 0; gi < (batch >= 16 ? 2 : 1); ++gi)
                for (int pb : {1, 2, 4, 8})
                    if (pb != pb0 || groups[gi] != mg0) candidate(pb, groups[gi], 0);
            candidate((int)best.pair_batch, (int)best.max_group, 1);
            rep += "]";
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
        });
        if (st != HE_OK) return st;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = best;
        if (cache_path && *cache_path) {
            std::ofstream f(cache_path, std::ios::app);
            f << key << " " << best.pair_batch << " " << best.max_group << " " << best.overlap << "\n";
        }
        rep += ", \"source\": \"timed\"";
    }
    {
        std::lock_guard<std::recursive_mutex> lk(c->api_mu);
        c->pair_batch = (int)best.pair_batch;
        c->max_group = (int)best.max_group;
        c->overlap = (int)best.overlap;
    }
    char buf[128];
    snprintf(buf, sizeof buf,
             ", \"chosen\": {\"pair_batch\": %u, \"max_group\": %u, \"overlap\": %u, \"concurrent_groups\": %u}}",
             best.pair_batch, best.max_group, best.overlap, best.concurrent_groups);
    rep += buf;
    if (report && report_n) {
        const size_t m = std::min(report_n - 1, rep.size());
        memcpy(report, rep.data(), m);
        report[m] = 0;
    }
    *out = best;
    return HE_OK;
}

}  // extern "C"
