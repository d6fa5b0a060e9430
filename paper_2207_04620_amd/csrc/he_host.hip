// libhe host runtime: context (primes, twiddles, keys, masks), the Fig. 1 operations,
// the packed product HE-MatMult (Alg. 3 + App. B) with hoisted rotations, the
// composite sign approximation (Sec. 4.2) and the C ABI declared in include/he.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/he.h"
#include "he_internal.hpp"

using namespace hm;

// ====================================================================== errors
const char* he_status_string(he_status s) {
    switch (s) {
        case HE_OK: return "ok";
        case HE_EINVAL: return "invalid argument";
        case HE_ENOMEM: return "out of memory";
        case HE_ELEVEL: return "level too low";
        case HE_ESCALE: return "scale out of range";
        case HE_EKEY: return "rotation key missing";
        case HE_ESHAPE: return "bad matrix shape";
        case HE_EMISMATCH: return "mismatched handles";
        case HE_EDEVICE: return "device error";
        default: return "unsupported";
    }
}

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        fprintf(stderr, "libhe: HIP error %s in %s\n", hipGetErrorString(e), what);
        throw HeError(HE_EDEVICE);
    }
}

// ====================================================================== device pool
void* Pool::alloc(size_t bytes) {
    std::lock_guard<std::mutex> lk(m);
    bytes = (bytes + 255) & ~(size_t)255;
    if (capture) {  // a graph reuses its own blocks first; whatever it takes becomes its own
        auto gi = capture->free_.find(bytes);
        if (gi != capture->free_.end() && !gi->second.empty()) {
            void* p = gi->second.back();
            gi->second.pop_back();
            return p;
        }
    }
    void* p0 = alloc_locked(bytes);
    if (capture) capture->owned[p0] = bytes;
    return p0;
}
void* Pool::alloc_locked(size_t bytes) {
    auto it = free_.find(bytes);
    if (it != free_.end() && !it->second.empty()) {
        void* p = it->second.back();
        it->second.pop_back();
        cached -= bytes;
        peak = std::max(peak, held - cached);
        return p;
    }
    void* p = nullptr;
    if (limit && held + bytes > limit) {
        trim_locked();  // cached blocks of other sizes go back to the device first
        if (held + bytes > limit) throw HeError(HE_ENOMEM);
    }
    if (dev_alloc) {
        p = dev_alloc(bytes, user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        trim_locked();
        if (sibling) {  // the other cache's free blocks too (hipFree waits for the device)
            std::lock_guard<std::mutex> lk2(sibling->m);
            sibling->trim_locked();
        }
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
        }
    }
    if (!p) throw HeError(HE_ENOMEM);
    held += bytes;
    peak = std::max(peak, held - cached);
    return p;
}
void Pool::release(void* p, size_t bytes) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(m);
    bytes = (bytes + 255) & ~(size_t)255;
    if (capture) {  // released while capturing: the graph's, reused only by that capture
        capture->owned[p] = bytes;
        capture->free_[bytes].push_back(p);
        return;
    }
    free_[bytes].push_back(p);
    cached += bytes;
}
void Pool::trim() {
    std::lock_guard<std::mutex> lk(m);
    trim_locked();
}
void Pool::trim_locked() {
    for (auto& kv : free_)
        for (void* p : kv.second) {
            if (dev_free) dev_free(p, user);
            else (void)hipFree(p);
            held -= kv.first;
            cached -= kv.first;
        }
    free_.clear();
}

DBuf::DBuf(Ctx* c, size_t n_u64) : ctx(c), pool(c->alloc_side ? &c->pool_side : &c->pool), n(n_u64) {
    p = (u64*)pool->alloc(n_u64 * 8);
}
DBuf::~DBuf() {
    if (p) pool->release(p, n * 8);
}
void Pool::absorb(Pool& o) {
    if (&o == this) return;
    std::scoped_lock lk(m, o.m);
    for (auto& kv : o.free_) {
        auto& dst = free_[kv.first];
        for (void* p : kv.second) {
            dst.push_back(p);
            o.held -= kv.first;
            o.cached -= kv.first;
            held += kv.first;
            cached += kv.first;
        }
    }
    o.free_.clear();
}

// ====================================================================== context setup
static void gen_primes(int log_n, const std::vector<uint32_t>& bits, std::vector<uint64_t>& out) {
    const uint64_t m2n = 2ull << log_n;
    for (uint32_t b : bits) {
        if (b < 20 || b > 60) throw HeError(HE_EINVAL);
        const uint64_t top = 1ull << b;
        uint64_t cand = (top - 1) / m2n * m2n + 1;
        for (;; cand -= m2n) {
            if (cand <= (top >> 1)) throw HeError(HE_EINVAL);
            if (std::find(out.begin(), out.end(), cand) != out.end()) continue;
            if (is_prime(cand)) break;
        }
        out.push_back(cand);
    }
}

// smallest primitive 2N-th root of unity modulo q
static uint64_t min_root(uint64_t q, int64_t N) {
    uint64_t g = 0;
    for (uint64_t x = 2;; ++x) {
        const uint64_t r = powmod(x, (q - 1) / (2 * N), q);
        if (powmod(r, N, q) == q - 1) {
            g = r;
            break;
        }
    }
    uint64_t best = g, cur = g;
    const uint64_t g2 = mulmod(g, g, q);
    for (int64_t k = 1; k < N; ++k) {
        cur = mulmod(cur, g2, q);
        best = std::min(best, cur);
    }
    return best;
}

// host buffers handed to upload() may be freed right after it returns
static void upload(Ctx* c, void* dst, const void* src, size_t bytes) {
    hip_check(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream), "upload");
    hip_check(hipStreamSynchronize(c->stream), "upload sync");
}

// CDT thresholds T[k] = floor(2^63 Pr[|e| <= k]) of the rounded Gaussian on [-19, 19],
// rho(x) = exp(-x^2 / (2 sigma^2)), sigma = 3.2, computed in __float128
static void gauss_cdt(uint64_t out[19]) {
    auto exp128 = [](f128 x) {  // exp(x) = (exp(x / 2^10))^(2^10)
        f128 y = x / 1024, t = 1, s = 1;
        for (int k = 1; k < 40; ++k) {
            t *= y / (f128)k;
            s += t;
        }
        for (int k = 0; k < 10; ++k) s *= s;
        return s;
    };
    const f128 sigma = (f128)32 / (f128)10;
    f128 rho[20], tot = 0;
    for (int x = 0; x < 20; ++x) rho[x] = exp128(-(f128)(x * x) / (2 * sigma * sigma));
    tot = rho[0];
    for (int x = 1; x < 20; ++x) tot += 2 * rho[x];
    f128 cum = rho[0];
    const f128 two63 = (f128)(1ull << 62) * 2;
    for (int k = 0; k < 19; ++k) {
        if (k) cum += 2 * rho[k];
        out[k] = (uint64_t)(cum / tot * two63);
    }
}

int Ctx::ext_mod(int level, int i) const { return i <= level ? i : n_q + (i - level - 1); }

void Ctx::build_tables() {
    const int M = n_q + n_p;
    std::vector<ModP> mp(M);
    std::vector<u64> psi(M * (size_t)N), psi_sh(M * (size_t)N), ipsi(M * (size_t)N), ipsi_sh(M * (size_t)N);
    for (int m = 0; m < M; ++m) {
        const u64 q = mods[m];
        const u64 r = min_root(q, N), ri = invmod(r, q);
        roots.push_back(r);
        ModP& e = mp[m];
        e.q = q;
        e.qninv = mont_neg_inv(q);
        const u64 rm = r_mod(q);
        e.r2 = mulmod(rm, rm, q);
        e.bar = ~0ull / q;
        e.ninv = invmod((u64)N % q, q);
        e.ninv_sh = shoup(e.ninv, q);
        e.half = (q - 1) / 2;
        e.pad = 0;
        // psi^(bitrev k)
        std::vector<u64> pw(N), ipw(N);
        u64 a = 1, b = 1;
        for (int64_t k = 0; k < N; ++k) {
            pw[k] = a;
            ipw[k] = b;
            a = mulmod(a, r, q);
            b = mulmod(b, ri, q);
        }
        for (int64_t k = 0; k < N; ++k) {
            const uint32_t br = bitrev((uint32_t)k, log_n);
            const size_t o = (size_t)m * N + k;
            psi[o] = pw[br];
            psi_sh[o] = shoup(pw[br], q);
            ipsi[o] = ipw[br];
            ipsi_sh[o] = shoup(ipw[br], q);
        }
    }
    d_mods = std::make_unique<DBuf>(this, (M * sizeof(ModP) + 7) / 8);
    d_psi = std::make_unique<DBuf>(this, (size_t)M * N);
    d_psi_sh = std::make_unique<DBuf>(this, (size_t)M * N);
    d_ipsi = std::make_unique<DBuf>(this, (size_t)M * N);
    d_ipsi_sh = std::make_unique<DBuf>(this, (size_t)M * N);
    upload(this, d_mods->p, mp.data(), M * sizeof(ModP));
    upload(this, d_psi->p, psi.data(), psi.size() * 8);
    upload(this, d_psi_sh->p, psi_sh.data(), psi.size() * 8);
    upload(this, d_ipsi->p, ipsi.data(), psi.size() * 8);
    upload(this, d_ipsi_sh->p, ipsi_sh.data(), psi.size() * 8);
    T.mods = (const ModP*)d_mods->p;
    T.psi = d_psi->p;
    T.psi_sh = d_psi_sh->p;
    T.ipsi = d_ipsi->p;
    T.ipsi_sh = d_ipsi_sh->p;
    T.log_n = log_n;
    T.n2_log = std::min(log_n, 11);
    T.n1_log = log_n - T.n2_log;
    T.fp64_mods = 0;
    for (int m = 0; m < M; ++m)
        if (fp64_limb(mp[m].q, T.n1_log, 1 << T.n2_log)) T.fp64_mods |= 1ull << m;
    host_mods = mp;

    // ---- row-pass twiddles in consumption order (N >= 2^11): row r of the second pass works
    // on twiddle exponents (N1 + r) 2^st + j; a group J of a round starting at stage s0 uses, for
    // its stages s0 + i (forward) or s0 - i (inverse), the pairs at (N1 + r) 2^st + (J << shift) + b
    T.rtw = T.irtw = nullptr;
    T.rtwd = T.irtwd = T.cold = T.icold = nullptr;
    if (T.n2_log == 11) {
        const int N1 = 1 << T.n1_log;
        std::vector<u64> rtw((size_t)M * N1 * ROW_TW * 2), irtw((size_t)M * N1 * ROW_TW * 2);
        static const int fr[4][2] = {{0, 3}, {3, 3}, {6, 3}, {9, 2}};
        static const int ir[4][2] = {{10, 3}, {7, 3}, {4, 3}, {1, 2}};
        for (int m = 0; m < M; ++m)
            for (int r = 0; r < N1; ++r) {
                const int64_t X = N1 + r;
                const size_t o = ((size_t)m * N1 + r) * ROW_TW * 2;
                size_t pos = 0;
                for (const auto& rd : fr) {
                    const int s0 = rd[0], R = rd[1];
                    for (int J = 0; J < (1 << s0); ++J)
                        for (int i = 0; i < R; ++i)
                            for (int b = 0; b < (1 << i); ++b) {
                                const size_t k = (size_t)m * N + (X << (s0 + i)) + ((int64_t)J << i) + b;
                                rtw[o + 2 * pos] = psi[k];
                                rtw[o + 2 * pos + 1] = psi_sh[k];
                                ++pos;
                            }
                }
                if (pos != ROW_TW) throw HeError(HE_EINVAL);
                pos = 0;
                for (const auto& rd : ir) {
                    const int s0 = rd[0], R = rd[1], G = 1 << R;
                    for (int J = 0; J < ((2048 / G) >> (11 - s0 - 1)); ++J)
                        for (int i = 0; i < R; ++i)
                            for (int b = 0; b < (G >> (i + 1)); ++b) {
                                const size_t k = (size_t)m * N + (X << (s0 - i)) + ((int64_t)J << (R - 1 - i)) + b;
                                irtw[o + 2 * pos] = ipsi[k];
                                irtw[o + 2 * pos + 1] = ipsi_sh[k];
                                ++pos;
                            }
                }
                if (pos != ROW_TW) throw HeError(HE_EINVAL);
            }
        d_rtw = std::make_unique<DBuf>(this, rtw.size());
        d_irtw = std::make_unique<DBuf>(this, irtw.size());
        upload(this, d_rtw->p, rtw.data(), rtw.size() * 8);
        upload(this, d_irtw->p, irtw.data(), irtw.size() * 8);
        T.rtw = d_rtw->p;
        T.irtw = d_irtw->p;
        // FP64 forms for primes below 2^46 (exact as doubles): w and fl(w / q)
        std::vector<double> rtwd(rtw.size(), 0.0), irtwd(irtw.size(), 0.0), cold((size_t)M * N1 * 2, 0.0),
            icold((size_t)M * N1 * 2, 0.0);
        for (int m = 0; m < M; ++m) {
            const u64 q = mods[m];
            if (q >= (1ull << 46)) continue;
            const double qd = (double)q;
            const size_t o = (size_t)m * N1 * ROW_TW * 2;
            for (size_t k = 0; k < (size_t)N1 * ROW_TW; ++k) {
                rtwd[o + 2 * k] = (double)rtw[o + 2 * k];
                rtwd[o + 2 * k + 1] = (double)rtw[o + 2 * k] / qd;
                irtwd[o + 2 * k] = (double)irtw[o + 2 * k];
                irtwd[o + 2 * k + 1] = (double)irtw[o + 2 * k] / qd;
            }
            for (int j = 0; j < N1; ++j) {
                const size_t c = ((size_t)m * N1 + j) * 2;
                cold[c] = (double)psi[(size_t)m * N + j];
                cold[c + 1] = cold[c] / qd;
                icold[c] = (double)ipsi[(size_t)m * N + j];
                icold[c + 1] = icold[c] / qd;
            }
        }
        d_rtwd = std::make_unique<DBuf>(this, rtwd.size());
        d_irtwd = std::make_unique<DBuf>(this, irtwd.size());
        d_cold = std::make_unique<DBuf>(this, cold.size());
        d_icold = std::make_unique<DBuf>(this, icold.size());
        upload(this, d_rtwd->p, rtwd.data(), rtwd.size() * 8);
        upload(this, d_irtwd->p, irtwd.data(), irtwd.size() * 8);
        upload(this, d_cold->p, cold.data(), cold.size() * 8);
        upload(this, d_icold->p, icold.data(), icold.size() * 8);
        T.rtwd = (const double*)d_rtwd->p;
        T.irtwd = (const double*)d_irtwd->p;
        T.cold = (const double*)d_cold->p;
        T.icold = (const double*)d_icold->p;
    }

    // ---- rescale constants: qinv[l][i] = q_l^-1 mod q_i
    std::vector<u64> qi((size_t)n_q * n_q, 0), qis((size_t)n_q * n_q, 0);
    for (int l = 1; l < n_q; ++l)
        for (int i = 0; i < l; ++i) {
            const u64 v = invmod(mods[l] % mods[i], mods[i]);
            qi[(size_t)l * n_q + i] = v;
            qis[(size_t)l * n_q + i] = shoup(v, mods[i]);
        }
    d_rs = std::make_unique<DBuf>(this, 2 * (size_t)n_q * n_q);
    upload(this, d_rs->p, qi.data(), qi.size() * 8);
    upload(this, d_rs->p + qi.size(), qis.data(), qis.size() * 8);

    // ---- ModDown: sources P, targets every Q limb; P^-1 mod q_t
    {
        std::vector<u64> tab((size_t)n_p * n_q * 2), pinv(n_q), pinv_sh(n_q);
        for (int s = 0; s < n_p; ++s) {
            const u64 qs = mods[n_q + s];
            u64 hs = 1;
            for (int r = 0; r < n_p; ++r)
                if (r != s) hs = mulmod(hs, mods[n_q + r] % qs, qs);
            md_hinv.push_back(invmod(hs, qs));
            md_hinv_sh.push_back(shoup(md_hinv.back(), qs));
            for (int t = 0; t < n_q; ++t) {
                const u64 qt = mods[t];
                u64 ht = 1;
                for (int r = 0; r < n_p; ++r)
                    if (r != s) ht = mulmod(ht, mods[n_q + r] % qt, qt);
                tab[((size_t)s * n_q + t) * 2 + 0] = to_mont(ht, qt);
                tab[((size_t)s * n_q + t) * 2 + 1] = to_mont((qt - mulmod(qs % qt, ht, qt)) % qt, qt);
            }
        }
        for (int t = 0; t < n_q; ++t) {
            u64 P = 1;
            for (int k = 0; k < n_p; ++k) P = mulmod(P, mods[n_q + k] % mods[t], mods[t]);
            pmod.push_back(P);
            pinv[t] = invmod(P, mods[t]);
            pinv_sh[t] = shoup(pinv[t], mods[t]);
        }
        d_md_tab = std::make_unique<DBuf>(this, tab.size());
        upload(this, d_md_tab->p, tab.data(), tab.size() * 8);
        d_pinv = std::make_unique<DBuf>(this, 2 * (size_t)n_q);
        upload(this, d_pinv->p, pinv.data(), n_q * 8);
        upload(this, d_pinv->p + n_q, pinv_sh.data(), n_q * 8);
    }

    // ---- ModUp: for each level l and digit j, sources I_j = [j a, min((j+1) a, l+1)),
    // targets all ext limbs (tab rows indexed by ext limb t in [0, l+1+K))
    mu.assign(n_q, {});
    size_t total = 0;
    for (int l = 0; l < n_q; ++l) {
        const int nl = l + 1, ne = nl + n_p, beta = (nl + alpha - 1) / alpha;
        for (int j = 0; j < beta; ++j) {
            ModUpInfo inf;
            inf.lo = j * alpha;
            inf.hi = std::min((j + 1) * alpha, nl);
            inf.off = total;
            total += (size_t)(inf.hi - inf.lo) * ne * 2;
            mu[l].push_back(inf);
        }
    }
    std::vector<u64> tab(total, 0);
    for (int l = 0; l < n_q; ++l) {
        const int nl = l + 1, ne = nl + n_p;
        for (auto& inf : mu[l]) {
            const int ns = inf.hi - inf.lo;
            for (int s = 0; s < ns; ++s) {
                const u64 qs = mods[inf.lo + s];
                u64 hs = 1;
                for (int r = 0; r < ns; ++r)
                    if (r != s) hs = mulmod(hs, mods[inf.lo + r] % qs, qs);
                inf.hinv[s] = invmod(hs, qs);
                inf.hinv_sh[s] = shoup(inf.hinv[s], qs);
                for (int t = 0; t < ne; ++t) {
                    const int tm = ext_mod(l, t);
                    const u64 qt = mods[tm];
                    u64 ht = 1;
                    for (int r = 0; r < ns; ++r)
                        if (r != s) ht = mulmod(ht, mods[inf.lo + r] % qt, qt);
                    tab[inf.off + ((size_t)s * ne + t) * 2 + 0] = to_mont(ht, qt);
                    tab[inf.off + ((size_t)s * ne + t) * 2 + 1] = to_mont((qt - mulmod(qs % qt, ht, qt)) % qt, qt);
                }
            }
        }
    }
    d_mu_tab = std::make_unique<DBuf>(this, std::max<size_t>(total, 1));
    upload(this, d_mu_tab->p, tab.data(), total * 8);

    // ---- output constants of the inverse transforms that feed a fused base conversion:
    // N^-1 (D/q_s)^-1 mod q_s as Shoup pairs, ModUp per (level, limb), ModDown per P prime
    {
        std::vector<u64> mus((size_t)n_q * n_q * 2, 0), mds((size_t)n_p * 2);
        for (int l = 0; l < n_q; ++l)
            for (const auto& inf : mu[l])
                for (int i = inf.lo; i < inf.hi; ++i) {
                    const u64 q = mods[i], f = mulmod(invmod((u64)N % q, q), inf.hinv[i - inf.lo], q);
                    mus[((size_t)l * n_q + i) * 2] = f;
                    mus[((size_t)l * n_q + i) * 2 + 1] = shoup(f, q);
                }
        for (int k = 0; k < n_p; ++k) {
            const u64 q = mods[n_q + k], f = mulmod(invmod((u64)N % q, q), md_hinv[k], q);
            mds[2 * k] = f;
            mds[2 * k + 1] = shoup(f, q);
        }
        d_mu_scale = std::make_unique<DBuf>(this, mus.size());
        upload(this, d_mu_scale->p, mus.data(), mus.size() * 8);
        d_md_scale = std::make_unique<DBuf>(this, mds.size());
        upload(this, d_md_scale->p, mds.data(), mds.size() * 8);
    }
    gauss_cdt(cdt);
}

// ====================================================================== small helpers
void Ctx::ntt(u64* base, int npoly, int64_t pstride_limbs, int nl, bool inverse, int level_for_ext) {
    // job lists are capped; long ones are split
    Jobs J;
    J.base = base;
    J.cstride = 0;
    J.nct = 1;
    J.n = 0;
    for (int p = 0; p < npoly; ++p)
        for (int i = 0; i < nl; ++i) {
            J.off[J.n] = (uint16_t)(p * pstride_limbs + i);
            J.mod[J.n] = (uint8_t)(level_for_ext < 0 ? i : ext_mod(level_for_ext, i));
            if (++J.n == HE_MAXJ) {
                launch_ntt(T, J, inverse, stream);
                J.n = 0;
            }
        }
    if (J.n) launch_ntt(T, J, inverse, stream);
}

static ModMap qmap(const Ctx* c) { return ModMap{1 << 20, c->n_q}; }

// ====================================================================== keys
void Ctx::sample_into(u64* dst, int nl_modidx_count, const int* modidx, int kind, uint32_t purpose, u64 index,
                      const u64* uidx) {
    Jobs J;
    J.base = dst;
    J.cstride = 0;
    J.nct = 1;
    J.n = nl_modidx_count;
    for (int k = 0; k < J.n; ++k) {
        J.off[k] = (uint16_t)k;
        J.mod[k] = (uint8_t)modidx[k];
    }
    SampleArgs A;
    memset(&A, 0, sizeof A);
    A.seed = seed;
    A.purpose = purpose;
    A.index = index;
    A.kind = kind;
    if (uidx)
        for (int k = 0; k < J.n; ++k) A.uidx[k] = uidx[k];
    memcpy(A.cdt, cdt, sizeof cdt);
    launch_sample(T, J, A, stream);
}

void Ctx::keygen_base() {
    const int M = n_q + n_p;
    std::vector<int> all(M);
    for (int m = 0; m < M; ++m) all[m] = m;
    s_eval = std::make_unique<DBuf>(this, (size_t)M * N);
    sample_into(s_eval->p, M, all.data(), 0, P_SK, 0, nullptr);
    ntt(s_eval->p, 1, 0, M, false, -1);
    s2_eval = std::make_unique<DBuf>(this, (size_t)M * N);
    launch_ew(T, ModMap{1 << 20, n_q}, M, 1, s2_eval->p, 0, s_eval->p, 0, s_eval->p, 0, EW_MUL_PLAIN, stream);
    // public key over Q
    pk = std::make_unique<DBuf>(this, 2 * (size_t)n_q * N);
    u64* pk0 = pk->p;
    u64* pk1 = pk->p + (size_t)n_q * N;
    std::vector<u64> uidx(n_q);
    for (int i = 0; i < n_q; ++i) uidx[i] = (u64)i;
    sample_into(pk1, n_q, all.data(), 2, P_PK_A, 0, uidx.data());
    sample_into(pk0, n_q, all.data(), 1, P_PK_E, 0, nullptr);
    ntt(pk->p, 2, n_q, n_q, false, -1);
    // pk0 = e - a s
    DBuf as(this, (size_t)n_q * N);
    launch_ew(T, qmap(this), n_q, 1, as.p, 0, pk1, 0, s_eval->p, 0, EW_MUL_PLAIN, stream);
    launch_ew(T, qmap(this), n_q, 1, pk0, 0, pk0, 0, as.p, 0, EW_SUB, stream);
    launch_to_mont(T, qmap(this), n_q, 2, pk->p, (int64_t)n_q * N, stream);
    keys_bytes += (size_t)(2 * M + 2 * n_q) * N * 8;
}

// switching key from s' (evaluation form over all M primes) to s; layout [beta][2][M][N]
std::unique_ptr<DBuf> Ctx::make_swk(u64 key_id, const u64* sp) {
    const int M = n_q + n_p, beta = (n_q + alpha - 1) / alpha;
    auto key = std::make_unique<DBuf>(this, (size_t)beta * 2 * M * N);
    std::vector<int> all(M);
    for (int m = 0; m < M; ++m) all[m] = m;
    DBuf e(this, (size_t)M * N);
    std::vector<uint8_t> flag(M);
    DBuf d_flag(this, (M + 7) / 8 + 1);
    DBuf d_pm(this, M);
    std::vector<u64> pm(M, 0);
    for (int t = 0; t < n_q; ++t) pm[t] = pmod[t];
    upload(this, d_pm.p, pm.data(), M * 8);
    for (int j = 0; j < beta; ++j) {
        u64* b = key->p + ((size_t)j * 2 + 0) * M * N;
        u64* a = key->p + ((size_t)j * 2 + 1) * M * N;
        std::vector<u64> uidx(M);
        for (int m = 0; m < M; ++m) uidx[m] = (key_id << 16) | ((u64)j << 8) | (u64)m;
        sample_into(a, M, all.data(), 2, P_SWK_A, 0, uidx.data());
        sample_into(e.p, M, all.data(), 1, P_SWK_E, (key_id << 8) | (u64)j, nullptr);
        ntt(a, 1, 0, M, false, -1);
        ntt(e.p, 1, 0, M, false, -1);
        for (int m = 0; m < M; ++m) flag[m] = (m < n_q && m / alpha == j) ? 1 : 0;
        upload(this, d_flag.p, flag.data(), M);
        launch_swk_finish(T, M, b, a, e.p, s_eval->p, sp, d_pm.p, (const uint8_t*)d_flag.p, stream);
        launch_to_mont(T, ModMap{1 << 20, n_q}, M, 2, b, (int64_t)M * N, stream);
        hip_check(hipStreamSynchronize(stream), "swk");  // flag buffer reused
    }
    keys_bytes += (size_t)beta * 2 * M * N * 8;
    return key;
}

const u64* Ctx::relin_key() {
    if (!rlk) rlk = make_swk(0, s2_eval->p);
    return rlk->p;
}

u64 Ctx::galois(int64_t k) const {
    const int64_t half = N / 2;
    const int64_t kk = ((k % half) + half) % half;
    return powmod(5, (u64)kk, 2 * (u64)N);
}

const u64* Ctx::rot_key(u64 g, bool create) {
    auto it = rot_keys.find(g);
    if (it != rot_keys.end()) return it->second->p;
    if (!create) throw HeError(HE_EKEY);
    const int M = n_q + n_p;
    DBuf sp(this, (size_t)M * N);
    launch_automorph(T, M, 1, sp.p, 0, s_eval->p, 0, g, stream);
    auto key = make_swk(g, sp.p);
    const u64* p = key->p;
    rot_keys[g] = std::move(key);
    return p;
}

// ====================================================================== ciphertexts
CtPtr Ctx::new_ct(int level, int deg, double scale) {
    auto c = std::make_shared<CtData>();
    c->level = level;
    c->deg = deg;
    c->scale = scale;
    c->buf = std::make_unique<DBuf>(this, (size_t)(deg + 1) * (level + 1) * N);
    return c;
}

CtPtr Ctx::encrypt_coeffs(const int64_t* m_host, int level, double scale, u64 nonce) {
    if (level < 0 || level >= n_q) throw HeError(HE_ELEVEL);
    const int nl = level + 1;
    std::vector<int> idx(nl);
    for (int i = 0; i < nl; ++i) idx[i] = i;
    DBuf v(this, (size_t)nl * N), x(this, 2 * (size_t)nl * N), dm(this, N);
    sample_into(v.p, nl, idx.data(), 0, P_ENC_V, nonce, nullptr);
    sample_into(x.p, nl, idx.data(), 1, P_ENC_E0, nonce, nullptr);
    sample_into(x.p + (size_t)nl * N, nl, idx.data(), 1, P_ENC_E1, nonce, nullptr);
    upload(this, dm.p, m_host, N * 8);
    launch_add_signed(T, nl, x.p, (const int64_t*)dm.p, stream);
    ntt(v.p, 1, 0, nl, false, -1);
    ntt(x.p, 2, nl, nl, false, -1);
    CtPtr c = new_ct(level, 1, scale);
    u64* c0 = c->buf->p;
    u64* c1 = c0 + (size_t)nl * N;
    launch_enc_combine(T, nl, v.p, pk->p, pk->p + (size_t)n_q * N, x.p, x.p + (size_t)nl * N, c0, c1, stream);
    // the host message buffer may be released by the caller once we return
    hip_check(hipStreamSynchronize(stream), "encrypt");
    return c;
}

void Ctx::decrypt_coeffs(const CtData& c, double* out) {
    const int nl = c.level + 1;
    DBuf m(this, (size_t)nl * N);
    const int64_t ps = (int64_t)nl * N;
    launch_dec_dot(T, nl, c.deg, c.buf->p, ps, s_eval->p, s2_eval->p, m.p, stream);
    ntt(m.p, 1, 0, nl, true, -1);
    std::vector<u64> h((size_t)nl * N);
    hip_check(hipMemcpyAsync(h.data(), m.p, h.size() * 8, hipMemcpyDeviceToHost, stream), "dec copy");
    hip_check(hipStreamSynchronize(stream), "dec sync");
    const u64 q0 = mods[0];
    bool bad = false;
    if (nl == 1) {
        for (int64_t t = 0; t < N; ++t) out[t] = (double)(h[t] > (q0 - 1) / 2 ? (int64_t)h[t] - (int64_t)q0 : (int64_t)h[t]);
        return;
    }
    const u64 q1 = mods[1];
    const u64 q0inv = invmod(q0 % q1, q1);
    const u128h Q2 = (u128h)q0 * q1;
    for (int64_t t = 0; t < N; ++t) {
        const u64 x0 = h[t], x1 = h[N + t];
        const u64 d = (x1 + q1 - x0 % q1) % q1;
        const u64 k = mulmod(d, q0inv, q1);
        const u128h w = (u128h)x0 + (u128h)q0 * k;
        __int128 v = w > Q2 / 2 ? (__int128)w - (__int128)Q2 : (__int128)w;
        for (int i = 2; i < nl && !bad; ++i) {
            const __int128 qi = (__int128)mods[i];
            __int128 r = v % qi;
            if (r < 0) r += qi;
            if ((u64)r != h[(size_t)i * N + t]) bad = true;
        }
        out[t] = (double)v;
    }
    if (bad) throw HeError(HE_ESCALE);
}

CtPtr Ctx::drop(const CtData& a, int level) {
    if (level > a.level || level < 0) throw HeError(HE_ELEVEL);
    CtPtr r = new_ct(level, a.deg, a.scale);
    const int nl = level + 1, nla = a.level + 1;
    for (int p = 0; p <= a.deg; ++p)
        hip_check(hipMemcpyAsync(r->buf->p + (size_t)p * nl * N, a.buf->p + (size_t)p * nla * N, (size_t)nl * N * 8,
                                 hipMemcpyDeviceToDevice, stream),
                  "drop");
    return r;
}

CtPtr Ctx::add_sub(const CtData& a, const CtData& b, bool sub) {
    const int level = std::min(a.level, b.level);
    const int deg = std::max(a.deg, b.deg);
    CtPtr r = new_ct(level, deg, std::max(a.scale, b.scale));
    const int nl = level + 1;
    const int64_t ps = (int64_t)nl * N, pa = (int64_t)(a.level + 1) * N, pb = (int64_t)(b.level + 1) * N;
    const int common = std::min(a.deg, b.deg) + 1;
    launch_ew(T, qmap(this), nl, common, r->buf->p, ps, a.buf->p, pa, b.buf->p, pb, sub ? EW_SUB : EW_ADD, stream);
    for (int p = common; p <= deg; ++p) {
        const CtData& src = a.deg >= p ? a : b;
        const int64_t psrc = (int64_t)(src.level + 1) * N;
        if (a.deg >= p || !sub) {
            hip_check(hipMemcpyAsync(r->buf->p + p * ps, src.buf->p + p * psrc, (size_t)nl * N * 8,
                                     hipMemcpyDeviceToDevice, stream),
                      "add copy");
        } else {  // 0 - b_p
            hip_check(hipMemsetAsync(r->buf->p + p * ps, 0, (size_t)nl * N * 8, stream), "sub zero");
            launch_ew(T, qmap(this), nl, 1, r->buf->p + p * ps, 0, r->buf->p + p * ps, 0, src.buf->p + p * psrc, 0,
                      EW_SUB, stream);
        }
    }
    cnt[C_ADD]++;
    return r;
}

// (a0 b0, a0 b1 + a1 b0, a1 b1) at the lower level (Fig. 1 Mul_ct before relinearisation)
CtPtr Ctx::tensor(const CtData& a, const CtData& b) {
    if (a.deg != 1 || b.deg != 1) throw HeError(HE_EMISMATCH);
    const int level = std::min(a.level, b.level), nl = level + 1;
    CtPtr r = new_ct(level, 2, a.scale * b.scale);
    launch_tensor(T, nl, a.buf->p, (int64_t)(a.level + 1) * N, b.buf->p, (int64_t)(b.level + 1) * N, r->buf->p,
                  (int64_t)nl * N, 0, stream);
    cnt[C_MULCT]++;
    return r;
}

// ---------------------------------------------------------------- key switching
// Digits of d (evaluation form, limbs 0..level) lifted to Q_l and P: [beta][ne][N]
std::unique_ptr<DBuf> Ctx::ks_lift(const u64* d, int level) {
    const int nl = level + 1, ne = nl + n_p;
    const int beta = (int)mu[level].size();
    auto lift = std::make_unique<DBuf>(this, (size_t)beta * ne * N);
    DBuf coef(this, (size_t)nl * N);
    ks_lift_into(d, level, lift->p, coef.p);
    return lift;
}

// the same into caller buffers: lift [beta][ne][N], coef [nl][N] (the digits' coefficient form)
void Ctx::ks_lift_into(const u64* d, int level, u64* lift, u64* coef) {
    const int nl = level + 1, ne = nl + n_p;
    const auto& infos = mu[level];
    const int beta = (int)infos.size();
    {  // the digits' coefficient form: the inverse transform reads d in place, writes coef
        Jobs Ji;
        Ji.base = coef;
        Ji.cstride = 0;
        Ji.src = d;
        Ji.nct = 1;
        Ji.n = nl;
        for (int i = 0; i < nl; ++i) {
            Ji.off[i] = (uint16_t)i;
            Ji.mod[i] = (uint8_t)i;
        }
        launch_ntt(T, Ji, true, stream);
    }
    Jobs J;
    J.base = lift;
    J.cstride = 0;
    J.nct = 1;
    J.n = 0;
    for (int j = 0; j < beta; ++j) {
        const ModUpInfo& inf = infos[j];
        ConvDesc D;
        memset(&D, 0, sizeof D);
        D.nct = 1;
        D.src = coef + (size_t)inf.lo * N;
        D.src_pstride = 0;
        D.dst = lift + (size_t)j * ne * N;
        D.dst_pstride = 0;
        D.tab = d_mu_tab->p + inf.off;
        D.ns = inf.hi - inf.lo;
        D.npoly = 1;
        D.tab_ld = ne;
        int nt = 0;
        for (int t = 0; t < ne; ++t) {
            if (t >= inf.lo && t < inf.hi) continue;
            D.doff[nt] = (uint16_t)t;
            D.dmod[nt] = (uint8_t)ext_mod(level, t);
            D.tcol[nt] = (uint16_t)t;
            ++nt;
            J.off[J.n] = (uint16_t)(j * ne + t);
            J.mod[J.n] = (uint8_t)ext_mod(level, t);
            if (++J.n == HE_MAXJ) {
                throw HeError(HE_EUNSUPPORTED);
            }
        }
        D.nt = nt;
        for (int s = 0; s < D.ns; ++s) {
            D.smod[s] = inf.lo + s;
            D.hinv[s] = inf.hinv[s];
            D.hinv_sh[s] = inf.hinv_sh[s];
        }
        launch_baseconv(T, D, stream);
        // the digit's own limbs are d itself
        hip_check(hipMemcpyAsync(lift + ((size_t)j * ne + inf.lo) * N, d + (size_t)inf.lo * N,
                                 (size_t)(inf.hi - inf.lo) * N * 8, hipMemcpyDeviceToDevice, stream),
                  "lift digit");
    }
    launch_ntt(T, J, false, stream);
}

// (out0, out1) = ModDown(<lift permuted by g, key>) (+ add0, add1); out pointers [nl][N]
void Ctx::ks_apply(const u64* lift, int level, const u64* key, u64 g, const u64* add0, const u64* add1, u64* out0,
                   u64* out1) {
    const int nl = level + 1, ne = nl + n_p;
    DBuf u(this, 2 * (size_t)ne * N);
    DBuf conv(this, 2 * (size_t)nl * N);
    ks_apply_into(lift, level, key, g, add0, add1, out0, out1, u.p, conv.p);
}

// the same with caller buffers: u [2][ne][N] (the inner product over Q_l and P), conv [2][nl][N]
void Ctx::ks_apply_into(const u64* lift, int level, const u64* key, u64 g, const u64* add0, const u64* add1,
                        u64* out0, u64* out1, u64* u, u64* conv) {
    const int nl = level + 1, ne = nl + n_p;
    const int beta = (int)mu[level].size();
    IpDesc D;
    memset(&D, 0, sizeof D);
    D.lift = lift;
    D.u = u;
    D.ne = ne;
    D.beta = beta;
    D.M = n_q + n_p;
    D.nrot = 1;
    D.nset = 1;
    D.s[0].key = key;
    D.s[0].g = g;
    D.nct = 1;
    D.lift_cs = 0;
    D.u_cs = 0;
    for (int t = 0; t < ne; ++t) D.mod[t] = (uint8_t)ext_mod(level, t);
    launch_inner_product(T, D, stream);
    // ModDown
    Jobs J;
    J.base = u;
    J.cstride = 0;
    J.nct = 1;
    J.n = 0;
    for (int p = 0; p < 2; ++p)
        for (int k = 0; k < n_p; ++k) {
            J.off[J.n] = (uint16_t)(p * ne + nl + k);
            J.mod[J.n] = (uint8_t)(n_q + k);
            ++J.n;
        }
    launch_ntt(T, J, true, stream);
    ConvDesc C;
    memset(&C, 0, sizeof C);
    C.nct = 1;
    C.src = u + (size_t)nl * N;
    C.src_pstride = (int64_t)ne * N;
    C.dst = conv;
    C.dst_pstride = (int64_t)nl * N;
    C.tab = d_md_tab->p;
    C.tab_ld = n_q;
    C.ns = n_p;
    C.nt = nl;
    C.npoly = 2;
    for (int s = 0; s < n_p; ++s) {
        C.smod[s] = n_q + s;
        C.hinv[s] = md_hinv[s];
        C.hinv_sh[s] = md_hinv_sh[s];
    }
    for (int t = 0; t < nl; ++t) {
        C.doff[t] = (uint16_t)t;
        C.dmod[t] = (uint8_t)t;
        C.tcol[t] = (uint16_t)t;
    }
    launch_baseconv(T, C, stream);
    ntt(conv, 2, nl, nl, false, -1);
    const u64* pinv = d_pinv->p;
    launch_moddown_combine(T, nl, 1, u, 0, conv, 0, pinv, pinv + n_q, add0, 0, out0, 0, stream);
    launch_moddown_combine(T, nl, 1, u + (size_t)ne * N, 0, conv + (size_t)nl * N, 0, pinv, pinv + n_q, add1, 0,
                           out1, 0, stream);
    cnt[C_KS]++;
}

CtPtr Ctx::relin(const CtData& a) {
    if (a.deg != 2) throw HeError(HE_EMISMATCH);
    const int nl = a.level + 1;
    const int64_t ps = (int64_t)nl * N;
    const u64* key = relin_key();
    auto lift = ks_lift(a.buf->p + 2 * ps, a.level);
    CtPtr r = new_ct(a.level, 1, a.scale);
    ks_apply(lift->p, a.level, key, 1, a.buf->p, a.buf->p + ps, r->buf->p, r->buf->p + ps);
    return r;
}

CtPtr Ctx::rescale(const CtData& a) {
    if (a.level < 1) throw HeError(HE_ELEVEL);
    const int l = a.level, nl = l + 1, np = a.deg + 1;
    const int64_t ps = (int64_t)nl * N;
    DBuf last(this, (size_t)np * N);
    for (int p = 0; p < np; ++p)
        hip_check(hipMemcpyAsync(last.p + (size_t)p * N, a.buf->p + p * ps + (size_t)l * N, N * 8,
                                 hipMemcpyDeviceToDevice, stream),
                  "rs copy");
    {
        Jobs J;
        J.base = last.p;
        J.cstride = 0;
        J.nct = 1;
        J.n = np;
        for (int p = 0; p < np; ++p) {
            J.off[p] = (uint16_t)p;
            J.mod[p] = (uint8_t)l;
        }
        launch_ntt(T, J, true, stream);
    }
    DBuf tmp(this, (size_t)np * l * N);
    launch_rescale_spread(T, l, np, last.p, N, l, tmp.p, (int64_t)l * N, stream);
    ntt(tmp.p, np, l, l, false, -1);
    CtPtr r = new_ct(l - 1, a.deg, a.scale / (double)mods[l]);
    const u64* qi = d_rs->p + (size_t)l * n_q;
    const u64* qis = d_rs->p + (size_t)n_q * n_q + (size_t)l * n_q;
    launch_rescale_combine(T, l, np, a.buf->p, ps, tmp.p, (int64_t)l * N, qi, qis, r->buf->p, (int64_t)l * N, stream);
    cnt[C_RS]++;
    return r;
}

CtPtr Ctx::rotate_from_lift(const CtData& a, const u64* lift, int64_t k) {
    const u64 g = galois(k);
    if (g == 1) return drop(a, a.level);
    const u64* key = rot_key(g, false);
    const int nl = a.level + 1;
    const int64_t ps = (int64_t)nl * N;
    CtPtr r = new_ct(a.level, 1, a.scale);
    launch_automorph(T, nl, 1, r->buf->p, 0, a.buf->p, 0, g, stream);
    ks_apply(lift, a.level, key, g, r->buf->p, nullptr, r->buf->p, r->buf->p + ps);
    cnt[C_ROT]++;
    return r;
}

CtPtr Ctx::rotate(const CtData& a, int64_t k) {
    if (a.deg != 1) throw HeError(HE_EMISMATCH);
    const u64 g = galois(k);
    if (g == 1) return drop(a, a.level);
    rot_key(g, false);
    auto lift = ks_lift(a.buf->p + (size_t)(a.level + 1) * N, a.level);
    return rotate_from_lift(a, lift->p, k);
}

CtPtr Ctx::mul_int(const CtData& a, int64_t k) {
    const int nl = a.level + 1;
    std::vector<u64> c(nl), cs(nl);
    for (int i = 0; i < nl; ++i) {
        const u64 q = mods[i];
        const u64 r = k >= 0 ? (u64)k % q : (q - (u64)(-(k + 1)) % q - 1) % q;
        c[i] = r;
        cs[i] = shoup(r, q);
    }
    DBuf dc(this, 2 * (size_t)nl);
    upload(this, dc.p, c.data(), nl * 8);
    upload(this, dc.p + nl, cs.data(), nl * 8);
    CtPtr r = new_ct(a.level, a.deg, a.scale);
    const int64_t ps = (int64_t)nl * N;
    launch_mul_const(T, qmap(this), nl, a.deg + 1, r->buf->p, ps, a.buf->p, ps, dc.p, dc.p + nl, stream);
    hip_check(hipStreamSynchronize(stream), "mul_int");
    return r;
}

// plaintext (signed integer coefficients) to Montgomery evaluation form over all Q limbs
// a plaintext's residues on every modulus (Q and P, so that it can also multiply a value
// in the extended basis), evaluation form, Montgomery form: [M][N]
std::unique_ptr<DBuf> Ctx::plaintext_mont(const int64_t* coeffs) {
    const int M = n_q + n_p;
    auto pt = std::make_unique<DBuf>(this, (size_t)M * N);
    DBuf dm(this, N);
    upload(this, dm.p, coeffs, N * 8);
    hip_check(hipMemsetAsync(pt->p, 0, (size_t)M * N * 8, stream), "pt zero");
    launch_add_signed(T, M, pt->p, (const int64_t*)dm.p, stream);
    ntt(pt->p, 1, 0, M, false, -1);
    launch_to_mont(T, ModMap{1 << 20, n_q}, M, 1, pt->p, 0, stream);
    hip_check(hipStreamSynchronize(stream), "plaintext");
    return pt;
}

// Alg. 6 aggregation: W - coeff sum_i G_i.  The n gradients are summed in one pass over HBM
// (16 inputs per launch), multiplied by the constant coeff = eta / (B N) encoded at the scale
// q_l of the prime the rescale removes (Mul_pt; the product returns exactly to the gradients'
// scale), rescaled, and subtracted from W dropped to the result's level.
CtPtr Ctx::fl_update(const CtData& w, const std::vector<const CtData*>& grads, double coeff) {
    if (grads.empty()) throw HeError(HE_EINVAL);
    int lvl = grads[0]->level;
    double sc = grads[0]->scale;
    for (auto* g : grads) {
        if (g->deg != 1) throw HeError(HE_EMISMATCH);
        lvl = std::min(lvl, g->level);
        sc = std::max(sc, g->scale);
    }
    if (lvl < 1 || w.deg != 1) throw HeError(lvl < 1 ? HE_ELEVEL : HE_EMISMATCH);
    const int nl = lvl + 1;
    CtPtr sum = new_ct(lvl, 1, sc);
    for (size_t base = 0; base < grads.size(); base += 16) {
        SumDesc D;
        memset(&D, 0, sizeof D);
        D.n = (int)std::min<size_t>(16, grads.size() - base);
        for (int t = 0; t < D.n; ++t) {
            D.in[t] = grads[base + t]->buf->p;
            D.in_ps[t] = (int64_t)(grads[base + t]->level + 1) * N;
        }
        launch_sum_many(T, nl, 2, D, sum->buf->p, (int64_t)nl * N, base > 0, stream);
    }
    cnt[C_ADD] += (int64_t)grads.size() - 1;
    std::vector<int64_t> m(N);
    const double ql = (double)mods[lvl];
    enc.encode(&coeff, 1, ql, m.data());
    auto pt = plaintext_mont(m.data());
    CtPtr t = mask_sum({{sum.get(), pt->p}}, ql);
    CtPtr u = rescale(*t);
    CtPtr wd = drop(w, std::min(u->level, w.level));
    return add_sub(*wd, *u, true);
}

// sum_r in_r * mask_r (Mul_pt terms of one diagonal sum, Alg. 2 / Eq. 1)
CtPtr Ctx::mask_sum(const std::vector<std::pair<const CtData*, const u64*>>& terms, double mask_scale) {
    const CtData& a0 = *terms[0].first;
    const int level = a0.level, nl = level + 1;
    CtPtr r = new_ct(level, 1, a0.scale * mask_scale);
    for (size_t base = 0; base < terms.size(); base += 16) {
        MacDesc D;
        memset(&D, 0, sizeof D);
        D.nct = 1;
        D.nterm = (int)std::min<size_t>(16, terms.size() - base);
        for (int t = 0; t < D.nterm; ++t) {
            const CtData* c = terms[base + t].first;
            if (c->level != level || c->deg != 1) throw HeError(HE_EMISMATCH);
            D.in[t] = c->buf->p;
            D.in_ps[t] = (int64_t)nl * N;
            D.mask[t] = terms[base + t].second;
        }
        launch_mask_mac(T, nl, 2, D, r->buf->p, (int64_t)nl * N, base > 0, stream);
    }
    cnt[C_MULPT] += (int64_t)terms.size();
    cnt[C_ADD] += (int64_t)terms.size() - 1;
    return r;
}

// ====================================================================== masks (Sec. 3.5-3.6, App. B)
static void mask_slots(int kind, int h, int k, std::vector<double>& out) {
    const int n = h * h;
    out.assign(n, 0.0);
    for (int t = 0; t < n; ++t) {
        bool v;
        switch (kind) {
            case 0:  // u^mu_k
                v = k >= 0 ? (t - h * k >= 0 && t - h * k < h - k) : (-k <= t - (h + k) * h && t - (h + k) * h < h);
                break;
            case 1: v = (t % h) == k; break;      // u^zeta_{h k}
            case 2: v = (t % h) < h - k; break;   // v_k (all ones for k = 0)
            case 3: v = (t % h) >= h - k; break;  // v_{k-h}
            default:  // App. C: diagonal (h-1) k of the transpose map (output h i + j reads h j + i)
                v = (t % h) - (t / h) == k;
                break;
        }
        out[t] = v ? 1.0 : 0.0;
    }
}

const u64* Ctx::mask(int kind, int h, int k, int64_t rot, int beta) {
    const MaskKey key{kind, h, beta, k, rot};
    auto it = masks.find(key);
    if (it != masks.end()) return it->second->p;
    prepare_masks({key});
    return masks.at(key)->p;
}

void Ctx::prepare_masks(const std::vector<MaskKey>& keys) {
    std::vector<MaskKey> todo;
    for (auto& k : keys)
        if (!masks.count(k) && std::find(todo.begin(), todo.end(), k) == todo.end()) todo.push_back(k);
    if (todo.empty()) return;
    std::vector<std::vector<int64_t>> coeffs(todo.size(), std::vector<int64_t>(N));
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (unsigned w = 0; w < nth; ++w)
        th.emplace_back([&, w]() {
            std::vector<double> u, ur;
            for (size_t i = w; i < todo.size(); i += nth) {
                const MaskKey& m = todo[i];
                mask_slots(m.kind, m.h, m.k, u);
                const int n = m.h * m.h;
                // R(u, rot), each entry repeated beta times (packing iota_beta: entry t of every
                // matrix sits at slots beta t .. beta t + beta - 1)
                ur.resize((size_t)n * m.beta);
                for (int t = 0; t < n; ++t)
                    for (int e = 0; e < m.beta; ++e)
                        ur[(size_t)m.beta * t + e] = u[(size_t)((((t + m.rot) % n) + n) % n)];
                enc.encode(ur.data(), (int64_t)n * m.beta, scale, coeffs[i].data());
            }
        });
    for (auto& t : th) t.join();
    for (size_t i = 0; i < todo.size(); ++i) {
        masks[todo[i]] = plaintext_mont(coeffs[i].data());
        keys_bytes += (size_t)(n_q + n_p) * N * 8;
    }
}

static int ilog2i(int h) {
    int l = 0;
    while ((1 << l) < h) ++l;
    return l;
}
static int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
int Ctx::bsgs(int h) const { return 1 << ((ilog2i(h) + 1) / 2); }
// baby steps bg of the Step-3 split k = bg i + j (2^ceil((log2 h + 1) / 2), at most h); one
// block of h terms without the flag
int Ctx::step3_baby(int h) const {
    if (!(schedule & HE_SCHED_STEP3_BSGS)) return h;
    return std::min(h, 1 << ((ilog2i(h) + 2) / 2));
}

// masks of HE-LinTrans with BSGS over diagonals [dlo, dhi] at unit u: R(mask_d, -u b floor(d/b))
static void lintrans_masks(std::vector<MaskKey>& out, int kind, int h, int beta, int64_t unit, int dlo, int dhi,
                           int b) {
    for (int d = dlo; d <= dhi; ++d) out.push_back({kind, h, beta, d, -unit * b * floordiv(d, b)});
}
// rotation amounts of the same: baby steps u j, giant steps u b i (i != 0)
static void lintrans_rotations(std::vector<int64_t>& r, int b, int64_t unit, int dlo, int dhi) {
    for (int j = 1; j < b; ++j) r.push_back(unit * j);
    for (int i = floordiv(dlo, b); i <= floordiv(dhi, b); ++i)
        if (i) r.push_back(unit * b * i);
}

void Ctx::check_shape(const MatShape& s) const {
    const auto pow2 = [](int x) { return x >= 1 && !(x & (x - 1)); };
    if (!pow2(s.h) || !pow2(s.t) || s.t > s.h || !pow2(s.beta) || (int64_t)s.beta * s.h * s.h > N / 2)
        throw HeError(HE_ESHAPE);
}

std::vector<MaskKey> Ctx::matmul_masks(const MatShape& s) const {
    std::vector<MaskKey> out;
    const int h = s.h, b = bsgs(h), bg = step3_baby(s.t);
    lintrans_masks(out, 0, h, s.beta, 1, 1 - h, h - 1, b);
    lintrans_masks(out, 1, h, s.beta, h, 0, h - 1, b);
    out.push_back({2, h, s.beta, 0, 0});
    for (int k = 1; k < s.t; ++k) {
        const int64_t shift = (int64_t)h * bg * (k / bg);
        out.push_back({2, h, s.beta, k, -shift});
        out.push_back({3, h, s.beta, k, -shift});
    }
    return out;
}

// amounts before the packing factor; every amount is multiplied by beta
std::vector<int64_t> Ctx::matmul_rotations(const MatShape& s) const {
    const int h = s.h, t = s.t, b = bsgs(h), bg = step3_baby(t);
    std::vector<int64_t> r;
    lintrans_rotations(r, b, 1, 1 - h, h - 1);
    lintrans_rotations(r, b, h, 0, h - 1);
    for (int k = 1; k < t; ++k) {
        const int64_t shift = (int64_t)h * bg * (k / bg);
        r.push_back(k - shift);
        r.push_back(k - h - shift);
    }
    for (int j = 1; j < bg; ++j) r.push_back((int64_t)h * j);
    for (int i = 1; i * bg < t; ++i) r.push_back((int64_t)h * bg * i);
    for (int sh = 0; (t << sh) < h; ++sh) r.push_back(((int64_t)t * h) << sh);
    for (auto& v : r) v *= s.beta;
    return r;
}

std::vector<MaskKey> Ctx::transpose_masks(int h, int beta) const {
    std::vector<MaskKey> out;
    lintrans_masks(out, 4, h, beta, h - 1, 1 - h, h - 1, bsgs(h));
    return out;
}

std::vector<int64_t> Ctx::transpose_rotations(int h, int beta) const {
    std::vector<int64_t> r;
    lintrans_rotations(r, bsgs(h), h - 1, 1 - h, h - 1);
    for (auto& v : r) v *= beta;
    return r;
}

void Ctx::prepare_shape(const MatShape& s) {
    check_shape(s);
    if (prepared.count(s)) return;
    for (int64_t k : matmul_rotations(s)) rot_key(galois(k), true);
    prepare_masks(matmul_masks(s));
    hip_check(hipStreamSynchronize(stream), "prepare_shape");
    prepared.insert(s);
    if (s.t == s.h && s.beta == 1) {
        int lg = 0;
        while ((1 << lg) < s.h) ++lg;
        prepared_mask.fetch_or(1u << lg);
    }
}

void Ctx::prepare_transpose(int h, int beta) {
    check_shape(MatShape{h, h, beta});
    if (prepared_tr.count({h, beta})) return;
    for (int64_t k : transpose_rotations(h, beta)) rot_key(galois(k), true);
    prepare_masks(transpose_masks(h, beta));
    hip_check(hipStreamSynchronize(stream), "prepare_transpose");
    prepared_tr.insert({h, beta});
}

// ====================================================================== C ABI


template <class F>
static he_status guard(F&& f);
template <class F>
static he_status guardc(he_ctx* ctx, F&& f) {
    std::lock_guard<std::recursive_mutex> lk(ctx->c->api_mu);
    return guard(std::forward<F>(f));
}
template <class F>
static he_status guard(F&& f) {
    try {
        f();
        return HE_OK;
    } catch (const HeError& e) {
        return e.s;
    } catch (const LaunchError&) {
        return HE_EDEVICE;
    } catch (const std::bad_alloc&) {
        return HE_ENOMEM;
    } catch (...) {
        return HE_EDEVICE;
    }
}

he_ct* wrap(Ctx* c, CtPtr p) { return new he_ct{c, std::move(p)}; }

extern "C" {

// iota_beta (App. E): entry e of matrix m at position beta e + m
he_status he_pack_beta(size_t beta, size_t n, const double* const* mats, double* out) {
    if (!mats || !out || beta == 0 || n == 0) return HE_EINVAL;
    for (size_t m = 0; m < beta; ++m)
        if (!mats[m]) return HE_EINVAL;
    for (size_t e = 0; e < n; ++e)
        for (size_t m = 0; m < beta; ++m) out[beta * e + m] = mats[m][e];
    return HE_OK;
}

// ====================================================================== allocation-free rotation
// Scratch of he_rotate_noalloc: file-scope device memory, one copy on every device the library
// runs on, held until the process ends.  Host code never passes the array's name to a kernel or
// a copy (on the host it only names the symbol); it uses the device address taken once per
// device by hipGetSymbolAddress with that device current.
#define HE_SCRATCH_BYTES (64ull << 20)
#define HE_MAX_DEVICES 64
static __device__ __align__(256) u64 scratch[HE_SCRATCH_BYTES / 8];
static std::mutex g_scratch_mu;
static u64* g_scratch_dev[HE_MAX_DEVICES];

// the current device's scratch address (taken on the first call for that device)
static u64* scratch_of_current_device(int* dev_out) {
    int dev = 0;
    hip_check(hipGetDevice(&dev), "scratch device");
    if (dev < 0 || dev >= HE_MAX_DEVICES) throw HeError(HE_EUNSUPPORTED);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch address");
        g_scratch_dev[dev] = (u64*)p;
    }
    *dev_out = dev;
    return g_scratch_dev[dev];
}

he_status he_ctx_create(const he_params* prm, const he_device* dev, he_ctx** out) {
    if (!prm || !out || !prm->q_bits || (prm->n_p && !prm->p_bits)) return HE_EINVAL;
    return guard([&]() {
        if (prm->log_n < 8 || prm->log_n > 17 || prm->n_q < 1 || prm->n_p < 1 || prm->alpha < 1 ||
            prm->n_q + prm->n_p > HE_MAXT || prm->alpha > HE_MAXSRC || prm->n_p > HE_MAXSRC ||
            (prm->n_q + prm->alpha - 1) / prm->alpha > HE_MAXSRC || (prm->schedule & ~HE_SCHED_ALL))
            throw HeError(HE_EINVAL);
        auto c = std::make_unique<Ctx>();
        c->scratch = scratch_of_current_device(&c->device);
        c->log_n = (int)prm->log_n;
        c->N = (int64_t)1 << prm->log_n;
        c->n_q = (int)prm->n_q;
        c->n_p = (int)prm->n_p;
        c->alpha = (int)prm->alpha;
        c->scale = std::pow(2.0, prm->log_scale);
        c->seed = prm->seed;
        c->schedule = prm->schedule;
        if (dev) {
            c->pool.dev_alloc = c->pool_side.dev_alloc = dev->alloc;
            c->pool.dev_free = c->pool_side.dev_free = dev->free;
            c->pool.user = c->pool_side.user = dev->user;
        }
        if (dev && dev->stream) {
            c->stream = (hipStream_t)dev->stream;
        } else {
            hip_check(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking), "stream");
            c->own_stream = true;
        }
        c->pool.sibling = &c->pool_side;
        c->pool_side.sibling = &c->pool;

        std::vector<uint32_t> qb(prm->q_bits, prm->q_bits + prm->n_q), pb(prm->p_bits, prm->p_bits + prm->n_p);
        gen_primes(c->log_n, qb, c->mods);
        gen_primes(c->log_n, pb, c->mods);
        // the REDC accumulations need (terms) * q < 2^64
        for (u64 q : c->mods)
            if (q >= (1ull << 60) + 1) throw HeError(HE_EINVAL);
        c->enc.init(c->log_n);
        c->build_tables();
        c->keygen_base();
        c->relin_key();
        for (uint32_t i = 0; i < prm->n_h; ++i) c->prepare_h((int)prm->h_list[i]);
        hip_check(hipStreamSynchronize(c->stream), "create");
        *out = new he_ctx{std::move(c)};
    });
}

void he_ctx_destroy(he_ctx* ctx) {
    if (!ctx) return;
    try {
        (void)hipStreamSynchronize(ctx->c->stream);
        if (ctx->c->side) (void)hipStreamSynchronize(ctx->c->side);
        ctx->c->release_all();
        if (ctx->c->own_stream) (void)hipStreamDestroy(ctx->c->stream);
    } catch (...) {
    }
    delete ctx;
}

he_status he_ctx_moduli(const he_ctx* ctx, uint64_t* out, size_t n) {
    if (!ctx || !out || n < ctx->c->mods.size()) return HE_EINVAL;
    std::copy(ctx->c->mods.begin(), ctx->c->mods.end(), out);
    return HE_OK;
}

he_status he_sync(he_ctx* ctx) {
    if (!ctx) return HE_EINVAL;
    return guardc(ctx, [&]() { hip_check(hipStreamSynchronize(ctx->c->stream), "sync"); });
}

he_status he_counters(const he_ctx* ctx, int64_t out[6], int reset) {
    if (!ctx || !out) return HE_EINVAL;
    for (int i = 0; i < 6; ++i) out[i] = ctx->c->cnt[i];
    if (reset)
        for (int i = 0; i < 6; ++i) const_cast<Ctx*>(ctx->c.get())->cnt[i] = 0;
    return HE_OK;
}

he_status he_memory(const he_ctx* ctx, uint64_t* keys_bytes, uint64_t* pool_bytes) {
    if (!ctx) return HE_EINVAL;
    if (keys_bytes) *keys_bytes = ctx->c->keys_bytes;
    if (pool_bytes) *pool_bytes = ctx->c->pool.held;
    return HE_OK;
}

he_status he_pool_limit(he_ctx* ctx, uint64_t bytes) {
    if (!ctx) return HE_EINVAL;
    return guardc(ctx, [&]() {
        // cached blocks above the new cap go back to the device once queued work is done
        hip_check(hipStreamSynchronize(ctx->c->stream), "pool limit");
        Pool& P = ctx->c->pool;
        std::lock_guard<std::mutex> lk(P.m);
        P.limit = bytes;
        if (bytes && P.held > bytes) P.trim_locked();
    });
}
he_status he_pool_stats(he_ctx* ctx, uint64_t* in_use, uint64_t* peak, int reset) {
    if (!ctx) return HE_EINVAL;
    Pool& P = ctx->c->pool;
    std::lock_guard<std::mutex> lk(P.m);
    if (in_use) *in_use = P.held - P.cached;
    if (peak) *peak = P.peak;
    if (reset) P.peak = P.held - P.cached;
    return HE_OK;
}

he_status he_encode(he_ctx* ctx, const double* vals, size_t n_vals, double scale, int64_t* out) {
    if (!ctx || !vals || !out || n_vals == 0 || (size_t)(ctx->c->N / 2) % n_vals) return HE_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(ctx->c->api_mu);
    ctx->c->enc.encode(vals, (int64_t)n_vals, scale, out);
    return HE_OK;
}

he_status he_encrypt(he_ctx* ctx, const double* vals, size_t n_vals, uint32_t level, uint64_t nonce, he_ct** out) {
    if (!ctx || !vals || !out || n_vals == 0 || (size_t)(ctx->c->N / 2) % n_vals) return HE_EINVAL;
    return guardc(ctx, [&]() {
        Ctx* c = ctx->c.get();
        std::vector<int64_t> m(c->N);
        c->enc.encode(vals, (int64_t)n_vals, c->scale, m.data());
        *out = wrap(c, c->encrypt_coeffs(m.data(), (int)level, c->scale, nonce));
    });
}

he_status he_encrypt_coeffs(he_ctx* ctx, const int64_t* coeffs, uint32_t level, double scale, uint64_t nonce,
                            he_ct** out) {
    if (!ctx || !coeffs || !out) return HE_EINVAL;
    return guardc(ctx, [&]() { *out = wrap(ctx->c.get(), ctx->c->encrypt_coeffs(coeffs, (int)level, scale, nonce)); });
}

he_status he_decrypt_coeffs(he_ctx* ctx, const he_ct* ct, double* out, size_t n) {
    if (!ctx || !ct || !out || n < (size_t)ctx->c->N) return HE_EINVAL;
    if (ct->ctx != ctx->c.get()) return HE_EMISMATCH;
    return guardc(ctx, [&]() { ctx->c->decrypt_coeffs(*ct->c, out); });
}

he_status he_decrypt(he_ctx* ctx, const he_ct* ct, double* out, size_t n_out) {
    if (!ctx || !ct || !out) return HE_EINVAL;
    if (ct->ctx != ctx->c.get()) return HE_EMISMATCH;
    return guardc(ctx, [&]() {
        std::vector<double> co(ctx->c->N);
        ctx->c->decrypt_coeffs(*ct->c, co.data());
        ctx->c->enc.decode(co.data(), ct->c->scale, out, (int64_t)n_out);
    });
}

void he_ct_free(he_ct* ct) {
    if (!ct) return;
    std::lock_guard<std::recursive_mutex> lk(ct->ctx->api_mu);
    delete ct;
}

he_status he_ct_info(const he_ct* ct, uint32_t* level, uint32_t* degree, double* scale) {
    if (!ct) return HE_EINVAL;
    if (level) *level = (uint32_t)ct->c->level;
    if (degree) *degree = (uint32_t)ct->c->deg;
    if (scale) *scale = ct->c->scale;
    return HE_OK;
}

he_status he_ct_export(he_ctx* ctx, const he_ct* ct, uint64_t* buf, size_t n) {
    if (!ctx || !ct || !buf) return HE_EINVAL;
    if (ct->ctx != ctx->c.get()) return HE_EMISMATCH;
    Ctx* c = ctx->c.get();
    const CtData& d = *ct->c;
    const size_t tot = (size_t)(d.deg + 1) * (d.level + 1) * c->N;
    if (n < tot) return HE_EINVAL;
    return guardc(ctx, [&]() {
        DBuf tmp(c, tot);
        hip_check(hipMemcpyAsync(tmp.p, d.buf->p, tot * 8, hipMemcpyDeviceToDevice, c->stream), "export");
        c->ntt(tmp.p, d.deg + 1, d.level + 1, d.level + 1, true, -1);
        hip_check(hipMemcpyAsync(buf, tmp.p, tot * 8, hipMemcpyDeviceToHost, c->stream), "export d2h");
        hip_check(hipStreamSynchronize(c->stream), "export sync");
    });
}

he_status he_ct_import(he_ctx* ctx, const uint64_t* buf, size_t n, uint32_t level, uint32_t degree, double scale,
                       he_ct** out) {
    if (!ctx || !buf || !out || degree < 1 || degree > 2) return HE_EINVAL;
    Ctx* c = ctx->c.get();
    if ((int)level >= c->n_q) return HE_ELEVEL;
    const size_t tot = (size_t)(degree + 1) * (level + 1) * c->N;
    if (n < tot) return HE_EINVAL;
    // every residue of limb i must lie in [0, q_i): the transform takes canonical words (its
    // FP64 butterflies convert a word exactly only below 2^52), so a corrupt or foreign
    // checkpoint is refused here instead of becoming a silently wrong ciphertext
    for (size_t p = 0; p <= degree; ++p)
        for (size_t i = 0; i <= level; ++i) {
            const uint64_t q = c->mods[i];
            const uint64_t* w = buf + (p * (level + 1) + i) * c->N;
            for (int64_t t = 0; t < c->N; ++t)
                if (w[t] >= q) return HE_EINVAL;
        }
    return guardc(ctx, [&]() {
        CtPtr r = c->new_ct((int)level, (int)degree, scale);
        upload(c, r->buf->p, buf, tot * 8);
        c->ntt(r->buf->p, degree + 1, level + 1, level + 1, false, -1);
        hip_check(hipStreamSynchronize(c->stream), "import");
        *out = wrap(c, r);
    });
}

#define CHECK2(a, b)                                                  \
    if (!ctx || !(a) || !(b) || !out) return HE_EINVAL;               \
    if ((a)->ctx != ctx->c.get() || (b)->ctx != ctx->c.get()) return HE_EMISMATCH;
#define CHECK1(a)                               \
    if (!ctx || !(a) || !out) return HE_EINVAL; \
    if ((a)->ctx != ctx->c.get()) return HE_EMISMATCH;

he_status he_add(he_ctx* ctx, const he_ct* a, const he_ct* b, he_ct** out) {
    CHECK2(a, b);
    return guardc(ctx, [&]() { *out = wrap(ctx->c.get(), ctx->c->add_sub(*a->c, *b->c, false)); });
}
he_status he_sub(he_ctx* ctx, const he_ct* a, const he_ct* b, he_ct** out) {
    CHECK2(a, b);
    return guardc(ctx, [&]() { *out = wrap(ctx->c.get(), ctx->c->add_sub(*a->c, *b->c, true)); });
}
he_status he_drop(he_ctx* ctx, const he_ct* a, uint32_t level, he_ct** out) {
    CHECK1(a);
    return guardc(ctx, [&]() { *out = wrap(ctx->c.get(), ctx->c->drop(*a->c, (int)level)); });
}
he_status he_mul_plain(he_ctx* ctx, const he_ct* a, const int64_t* coeffs, double pt_scale, he_ct** out) {
    CHECK1(a);
    if (!coeffs) return HE_EINVAL;
    return guardc(ctx, [&]() {
        Ctx* c = ctx->c.get();
        auto pt = c->plaintext_mont(coeffs);
        if (a->c->deg != 1) throw HeError(HE_EMISMATCH);
        CtPtr r = c->mask_sum({{a->c.get(), pt->p}}, pt_scale);
        hip_check(hipStreamSynchronize(c->stream), "mul_plain");
        *out = wrap(c, r);
    });
}
he_status he_mul_int(he_ctx* ctx, const he_ct* a, int64_t k, he_ct** out) {
    CHECK1(a);
    return guardc(ctx, [&]() { *out = wrap(ctx->c.get(), ctx->c->mul_int(*a->c, k)); });
}
he_status he_tensor(he_ctx* ctx, const he_ct* a, const he_ct* b, he_ct** out) {
    CHECK2(a, b);
    return guardc(ctx, [&]() { *out = wrap(ctx->c.get(), ctx->c->tensor(*a->c, *b->c)); });
}
he_status he_relin(he_ctx* ctx, const he_ct* a, he_ct** out) {
    CHECK1(a);
    return guardc(ctx, [&]() { *out = wrap(ctx->c.get(), ctx->c->relin(*a->c)); });
}
he_status he_mul(he_ctx* ctx, const he_ct* a, const he_ct* b, he_ct** out) {
    CHECK2(a, b);
    return guardc(ctx, [&]() { *out = wrap(ctx->c.get(), ctx->c->relin(*ctx->c->tensor(*a->c, *b->c))); });
}
he_status he_rescale(he_ctx* ctx, const he_ct* a, he_ct** out) {
    CHECK1(a);
    return guardc(ctx, [&]() { *out = wrap(ctx->c.get(), ctx->c->rescale(*a->c)); });
}
he_status he_rotate(he_ctx* ctx, const he_ct* a, int64_t k, he_ct** out) {
    CHECK1(a);
    return guardc(ctx, [&]() { *out = wrap(ctx->c.get(), ctx->c->rotate(*a->c, k)); });
}

// Rot(a, k) with every temporary in the static scratch: the digit lift [beta][ne][N], the
// inner product over Q_l and P [2][ne][N], and one region shared by the digits' coefficient
// form (used while lifting) and the converted P part (used by ModDown afterwards) [2][nl][N].
// Every scratch word a call reads was written earlier in that call, so nothing is cleared.
he_status he_rotate_noalloc(he_ctx* ctx, const uint64_t* in, uint32_t level, int64_t k, uint64_t* out) {
    if (!ctx || !in || !out) return HE_EINVAL;
    Ctx* c = ctx->c.get();
    if ((int)level >= c->n_q) return HE_ELEVEL;
    const int nl = (int)level + 1, ne = nl + c->n_p;
    const int64_t N = c->N;
    const size_t ct_words = 2 * (size_t)nl * N;
    if (in < out + ct_words && out < in + ct_words) return HE_EINVAL;  // in and out overlap
    const int beta = (int)c->mu[level].size();
    const size_t lift_w = (size_t)beta * ne * N, u_w = 2 * (size_t)ne * N, tmp_w = 2 * (size_t)nl * N;
    if ((lift_w + u_w + tmp_w) * 8 > HE_SCRATCH_BYTES) {
        fprintf(stderr, "libhe: he_rotate_noalloc needs %zu scratch bytes at level %u, more than the %llu it has\n",
                (lift_w + u_w + tmp_w) * 8, level, HE_SCRATCH_BYTES);
        return HE_ENOMEM;
    }
    return guardc(ctx, [&]() {
        int dev = 0;
        hip_check(hipGetDevice(&dev), "device");
        if (dev != c->device) throw HeError(HE_EMISMATCH);  // the scratch address is per device
        const u64 g = c->galois(k);
        if (g == 1) {
            hip_check(hipMemcpyAsync(out, in, ct_words * 8, hipMemcpyDeviceToDevice, c->stream), "rotate copy");
            return;
        }
        const u64* key = c->rot_key(g, false);
        u64 *lift = c->scratch, *u = lift + lift_w, *tmp = u + u_w;
        c->ks_lift_into(in + (size_t)nl * N, (int)level, lift, tmp);
        launch_automorph(c->T, nl, 1, out, 0, in, 0, g, c->stream);
        c->ks_apply_into(lift, (int)level, key, g, out, nullptr, out, out + (size_t)nl * N, u, tmp);
        c->cnt[C_ROT]++;
    });
}
he_status he_gen_rotation_key(he_ctx* ctx, int64_t k) {
    if (!ctx) return HE_EINVAL;
    return guardc(ctx, [&]() {
        ctx->c->rot_key(ctx->c->galois(k), true);
        hip_check(hipStreamSynchronize(ctx->c->stream), "genkey");
    });
}
he_status he_matmul(he_ctx* ctx, const he_ct* a, const he_ct* b, uint32_t h, he_ct** out) {
    CHECK2(a, b);
    return guardc(ctx, [&]() { *out = wrap(ctx->c.get(), ctx->c->matmul(*a->c, *b->c, (int)h)); });
}
he_status he_matmul_batch(he_ctx* ctx, size_t n, const he_ct* const* a, const he_ct* const* b, const uint32_t* h,
                          he_ct** out) {
    if (!ctx || (n && (!a || !b || !h || !out))) return HE_EINVAL;
    for (size_t i = 0; i < n; ++i) {
        if (!a[i] || !b[i]) return HE_EINVAL;
        if (a[i]->ctx != ctx->c.get() || b[i]->ctx != ctx->c.get()) return HE_EMISMATCH;
    }
    return guardc(ctx, [&]() {
        std::vector<const CtData*> va(n), vb(n);
        std::vector<int> vh(n);
        for (size_t i = 0; i < n; ++i) {
            va[i] = a[i]->c.get();
            vb[i] = b[i]->c.get();
            vh[i] = (int)h[i];
        }
        std::vector<MatShape> sh(n);
        for (size_t i = 0; i < n; ++i) sh[i] = MatShape{vh[i], vh[i], 1};
        auto res = ctx->c->matmul_batch(va, vb, sh);
        for (size_t i = 0; i < n; ++i) out[i] = wrap(ctx->c.get(), res[i]);
    });
}
he_status he_matmul_ex(he_ctx* ctx, const he_ct* a, const he_ct* b, const he_mat_shape* shape, he_ct** out) {
    return he_matmul_batch_ex(ctx, 1, &a, &b, shape, out);
}
he_status he_matmul_batch_ex(he_ctx* ctx, size_t n, const he_ct* const* a, const he_ct* const* b,
                             const he_mat_shape* shapes, he_ct** out) {
    if (!ctx || (n && (!a || !b || !shapes || !out))) return HE_EINVAL;
    for (size_t i = 0; i < n; ++i) {
        if (!a[i] || !b[i]) return HE_EINVAL;
        if (a[i]->ctx != ctx->c.get() || b[i]->ctx != ctx->c.get()) return HE_EMISMATCH;
    }
    return guardc(ctx, [&]() {
        std::vector<const CtData*> va(n), vb(n);
        std::vector<MatShape> sh(n);
        for (size_t i = 0; i < n; ++i) {
            va[i] = a[i]->c.get();
            vb[i] = b[i]->c.get();
            sh[i] = MatShape{(int)shapes[i].h, (int)shapes[i].t, (int)shapes[i].beta};
        }
        auto res = ctx->c->matmul_batch(va, vb, sh);
        for (size_t i = 0; i < n; ++i) out[i] = wrap(ctx->c.get(), res[i]);
    });
}
he_status he_transpose(he_ctx* ctx, const he_ct* a, uint32_t h, uint32_t beta, he_ct** out) {
    return he_transpose_batch(ctx, 1, &a, h, beta, out);
}
he_status he_transpose_batch(he_ctx* ctx, size_t n, const he_ct* const* a, uint32_t h, uint32_t beta,
                             he_ct** out) {
    if (!ctx || (n && (!a || !out))) return HE_EINVAL;
    for (size_t i = 0; i < n; ++i) {
        if (!a[i]) return HE_EINVAL;
        if (a[i]->ctx != ctx->c.get()) return HE_EMISMATCH;
    }
    return guardc(ctx, [&]() {
        std::vector<const CtData*> va(n);
        for (size_t i = 0; i < n; ++i) va[i] = a[i]->c.get();
        auto res = ctx->c->transpose_batch(va, (int)h, (int)beta);
        for (size_t i = 0; i < n; ++i) out[i] = wrap(ctx->c.get(), res[i]);
    });
}
he_status he_sign_approx(he_ctx* ctx, const he_ct* x, uint32_t d, uint32_t k, uint32_t mode, he_ct** out) {
    CHECK1(x);
    if (mode > 1) return HE_EINVAL;
    return guardc(ctx, [&]() { *out = wrap(ctx->c.get(), ctx->c->sign_group({x->c.get()}, (int)d, (int)k, (int)mode)[0]); });
}
he_status he_sign_approx_batch(he_ctx* ctx, size_t n, const he_ct* const* x, uint32_t d, uint32_t k, uint32_t mode,
                               he_ct** out) {
    if (!ctx || (n && (!x || !out)) || mode > 1) return HE_EINVAL;
    for (size_t i = 0; i < n; ++i) {
        if (!x[i]) return HE_EINVAL;
        if (x[i]->ctx != ctx->c.get()) return HE_EMISMATCH;
    }
    return guardc(ctx, [&]() {
        // lockstep groups of equal level
        std::map<int, std::vector<size_t>> byl;
        for (size_t i = 0; i < n; ++i) byl[x[i]->c->level].push_back(i);
        std::vector<CtPtr> res(n);
        for (auto& kv : byl) {
            for (size_t s = 0; s < kv.second.size(); s += (size_t)ctx->c->max_group) {
                std::vector<const CtData*> v;
                const size_t e = std::min(kv.second.size(), s + (size_t)ctx->c->max_group);
                for (size_t t = s; t < e; ++t) v.push_back(x[kv.second[t]]->c.get());
                auto r = ctx->c->sign_group(v, (int)d, (int)k, (int)mode);
                for (size_t t = s; t < e; ++t) res[kv.second[t]] = r[t - s];
            }
        }
        for (size_t i = 0; i < n; ++i) out[i] = wrap(ctx->c.get(), res[i]);
    });
}
he_status he_appmax(he_ctx* ctx, const he_ct* a, const he_ct* b, uint32_t d, uint32_t k, he_ct** out) {
    return he_appmax_batch(ctx, 1, &a, &b, d, k, out);
}
he_status he_appmax_batch(he_ctx* ctx, size_t n, const he_ct* const* a, const he_ct* const* b, uint32_t d,
                          uint32_t k, he_ct** out) {
    if (!ctx || (n && (!a || !b || !out))) return HE_EINVAL;
    for (size_t i = 0; i < n; ++i) {
        if (!a[i] || !b[i]) return HE_EINVAL;
        if (a[i]->ctx != ctx->c.get() || b[i]->ctx != ctx->c.get()) return HE_EMISMATCH;
    }
    return guardc(ctx, [&]() {
        // lockstep groups of equal operand levels
        std::map<std::pair<int, int>, std::vector<size_t>> byl;
        for (size_t i = 0; i < n; ++i) byl[{a[i]->c->level, b[i]->c->level}].push_back(i);
        std::vector<CtPtr> res(n);
        for (auto& kv : byl) {
            for (size_t s = 0; s < kv.second.size(); s += (size_t)ctx->c->max_group) {
                std::vector<const CtData*> va, vb;
                const size_t e = std::min(kv.second.size(), s + (size_t)ctx->c->max_group);
                for (size_t t = s; t < e; ++t) {
                    va.push_back(a[kv.second[t]]->c.get());
                    vb.push_back(b[kv.second[t]]->c.get());
                }
                auto r = ctx->c->sign_group(va, (int)d, (int)k, 2, vb);
                for (size_t t = s; t < e; ++t) res[kv.second[t]] = r[t - s];
            }
        }
        for (size_t i = 0; i < n; ++i) out[i] = wrap(ctx->c.get(), res[i]);
    });
}
he_status he_maxpool2(he_ctx* ctx, const he_ct* x, uint32_t h, uint32_t d, uint32_t k, he_ct** out) {
    return he_maxpool2_batch(ctx, 1, &x, h, d, k, out);
}
he_status he_maxpool2_batch(he_ctx* ctx, size_t n, const he_ct* const* x, uint32_t h, uint32_t d, uint32_t k,
                            he_ct** out) {
    if (!ctx || (n && (!x || !out))) return HE_EINVAL;
    for (size_t i = 0; i < n; ++i) {
        if (!x[i]) return HE_EINVAL;
        if (x[i]->ctx != ctx->c.get()) return HE_EMISMATCH;
    }
    return guardc(ctx, [&]() {
        std::vector<const CtData*> v(n);
        for (size_t i = 0; i < n; ++i) v[i] = x[i]->c.get();
        auto r = ctx->c->maxpool_batch(v, (int)h, (int)d, (int)k);
        for (size_t i = 0; i < n; ++i) out[i] = wrap(ctx->c.get(), r[i]);
    });
}
he_status he_fl_update(he_ctx* ctx, const he_ct* w, size_t n, const he_ct* const* grads, double coeff, he_ct** out) {
    if (!ctx || !w || !out || n == 0 || !grads) return HE_EINVAL;
    if (w->ctx != ctx->c.get()) return HE_EMISMATCH;
    for (size_t i = 0; i < n; ++i) {
        if (!grads[i]) return HE_EINVAL;
        if (grads[i]->ctx != ctx->c.get()) return HE_EMISMATCH;
    }
    return guardc(ctx, [&]() {
        std::vector<const CtData*> g(n);
        for (size_t i = 0; i < n; ++i) g[i] = grads[i]->c.get();
        *out = wrap(ctx->c.get(), ctx->c->fl_update(*w->c, g, coeff));
    });
}
he_status he_profile_enable(he_ctx* ctx, int on, const char* only) {
    if (!ctx) return HE_EINVAL;
    return prof_enable(on != 0, only) ? HE_OK : HE_EINVAL;
}
he_status he_debug_fail_launch(uint64_t n) {
    launch_inject(n);
    return HE_OK;
}
he_status he_profile_report(he_ctx* ctx, char* buf, size_t n) {
    if (!ctx || !buf || n == 0) return HE_EINVAL;
    return guardc(ctx, [&]() {
        const std::string r = prof_report();
        const size_t m = std::min(n - 1, r.size());
        memcpy(buf, r.data(), m);
        buf[m] = 0;
    });
}
he_status he_ntt(he_ctx* ctx, uint64_t* dev_ptr, uint32_t n_limbs, const uint32_t* mod_idx, int inverse) {
    if (!ctx || !dev_ptr || !mod_idx || n_limbs == 0) return HE_EINVAL;
    Ctx* c = ctx->c.get();
    for (uint32_t i = 0; i < n_limbs; ++i)
        if (mod_idx[i] >= c->mods.size()) return HE_EINVAL;
    return guardc(ctx, [&]() {
        for (uint32_t start = 0; start < n_limbs; start += HE_MAXJ) {
            Jobs J;
            J.base = dev_ptr + (size_t)start * c->N;
            J.cstride = 0;
            J.nct = 1;
            J.n = (int)std::min<uint32_t>(HE_MAXJ, n_limbs - start);
            for (int k = 0; k < J.n; ++k) {
                J.off[k] = (uint16_t)k;
                J.mod[k] = (uint8_t)mod_idx[start + k];
            }
            launch_ntt(c->T, J, inverse != 0, c->stream);
        }
        hip_check(hipGetLastError(), "ntt launch");
    });
}

}  // extern "C"

