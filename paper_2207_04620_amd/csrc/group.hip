// Lockstep execution of HE-MatMult (Alg. 3 + App. B) over a group of ciphertext pairs
// with the same matrix side h and level.  Every operation of the product runs once
// per group: each launch covers all members, and the kernels that read a shared
// operand (a switching key in the key-switch inner product, a diagonal mask in the
// mask multiply-accumulate) load it once and reuse it for every member, so a key
// crosses HBM once per rotation round of the whole group.  The operation DAG is the
// one of the single product, so every member's result is bit-identical to running
// it alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>

#include "he_internal.hpp"

static void copy2d(Ctx* c, u64* dst, int64_t dpitch, const u64* src, int64_t spitch, int64_t width, int64_t height) {
    if (height <= 0 || width <= 0) return;
    hip_check(hipMemcpy2DAsync(dst, (size_t)dpitch * 8, src, (size_t)spitch * 8, (size_t)width * 8, (size_t)height,
                               hipMemcpyDeviceToDevice, c->stream),
              "copy2d");
}

Grp Ctx::g_new(int B, int level, int deg, const std::vector<double>& sc) {
    Grp g;
    g.B = B;
    g.level = level;
    g.deg = deg;
    g.scale = sc;
    g.ps = (int64_t)(level + 1) * N;
    g.cs = (int64_t)(deg + 1) * g.ps;
    g.buf = std::make_shared<DBuf>(this, (size_t)B * g.cs);
    g.p = g.buf->p;
    return g;
}

Grp Ctx::g_gather(const std::vector<const CtData*>& v, int level) {
    std::vector<double> sc;
    for (auto* c : v) {
        if (c->deg != 1 || c->level < level) throw HeError(HE_EMISMATCH);
        sc.push_back(c->scale);
    }
    Grp g = g_new((int)v.size(), level, 1, sc);
    // the members' limb prefixes, up to CP_MAX members per copy launch
    CopyDesc D;
    for (size_t i = 0; i < v.size(); ++i) {
        D.src[D.n] = v[i]->buf->p;
        D.dst[D.n] = g.p + i * g.cs;
        D.width[D.n] = g.ps;
        D.spitch[D.n] = (int64_t)(v[i]->level + 1) * N;
        D.dpitch[D.n] = g.ps;
        D.rows[D.n] = 2;
        if (++D.n == CP_MAX || i + 1 == v.size()) {
            launch_copy(D, stream);
            D.n = 0;
        }
    }
    return g;
}

std::vector<CtPtr> Ctx::g_scatter(const Grp& g) {
    std::vector<CtPtr> out;
    CopyDesc D;
    for (int i = 0; i < g.B; ++i) {
        CtPtr c = new_ct(g.level, g.deg, g.scale[i]);
        D.src[D.n] = g.p + i * g.cs;
        D.dst[D.n] = c->buf->p;
        D.width[D.n] = g.cs;
        D.spitch[D.n] = D.dpitch[D.n] = g.cs;
        D.rows[D.n] = 1;
        if (++D.n == CP_MAX || i + 1 == g.B) {
            launch_copy(D, stream);
            D.n = 0;
        }
        out.push_back(c);
    }
    return out;
}

Grp Ctx::g_drop(const Grp& a, int level) {
    if (level > a.level) throw HeError(HE_ELEVEL);
    Grp g = g_new(a.B, level, a.deg, a.scale);
    copy2d(this, g.p, g.ps, a.p, a.ps, g.ps, (int64_t)a.B * (a.deg + 1));
    return g;
}

void Ctx::g_add_into(Grp& acc, const Grp& t) {
    if (acc.B != t.B || acc.deg != t.deg || acc.level != t.level) throw HeError(HE_EMISMATCH);
    launch_ew(T, ModMap{1 << 20, n_q}, acc.level + 1, acc.deg + 1, acc.p, acc.ps, acc.p, acc.ps, t.p, t.ps, EW_ADD,
              stream, acc.B, acc.cs, acc.cs, t.cs);
    for (int i = 0; i < acc.B; ++i) acc.scale[i] = std::max(acc.scale[i], t.scale[i]);
    cnt[C_ADD] += acc.B;
}

// digits of poly 'poly' of every member, lifted to Q_l and P: [B][beta][ne][N]
std::shared_ptr<DBuf> Ctx::g_lift(const Grp& a, int poly) {
    const int level = a.level, nl = level + 1, ne = nl + n_p, B = a.B;
    const auto& infos = mu[level];
    const int beta = (int)infos.size();
    const int64_t lcs = (int64_t)beta * ne * N;
    auto lift = std::make_shared<DBuf>(this, (size_t)B * lcs);
    DBuf coef(this, (size_t)B * nl * N);
    // with the fused conversion, the inverse transform also applies each digit's (D/q_s)^-1;
    // it reads the polynomial in place and writes its coefficient form to coef
    bool fused = true;
    for (const auto& inf : infos) fused = fused && conv_cols_fits(T, inf.hi - inf.lo);
    {
        Jobs J;
        J.base = coef.p;
        J.cstride = (int64_t)nl * N;
        J.src = a.p + poly * a.ps;
        J.src_cstride = a.cs;
        J.nct = B;
        J.n = nl;
        for (int i = 0; i < nl; ++i) {
            J.off[i] = (uint16_t)i;
            J.mod[i] = (uint8_t)i;
        }
        launch_ntt(T, J, true, stream, fused ? d_mu_scale->p + (size_t)level * n_q * 2 : nullptr, nl);
    }
    Jobs J;
    J.base = lift->p;
    J.cstride = lcs;
    J.nct = B;
    J.n = 0;
    // every digit's conversion in one fused launch (one grid over all targets: the digits' few
    // blocks each would leave the device part idle at their ends)
    const bool merged = fused && beta <= HE_MAXDIG && beta * ne - nl <= HE_MAXT;
    ConvDesc M;
    memset(&M, 0, sizeof M);
    if (merged) {
        M.src = coef.p;
        M.src_cstride = (int64_t)nl * N;
        M.dst = lift->p;
        M.dst_cstride = lcs;
        M.nct = B;
        M.npoly = 1;
        M.tab = d_mu_tab->p;
        M.tab_ld = ne;
        M.prescaled = 1;
        M.ndig = beta;
    }
    for (int j = 0; j < beta; ++j) {
        const ModUpInfo& inf = infos[j];
        if (merged) {
            M.dns[j] = inf.hi - inf.lo;
            M.dsrc[j] = (int64_t)inf.lo * N;
            M.dtab[j] = (int64_t)inf.off;
            M.ns = std::max(M.ns, inf.hi - inf.lo);
            for (int t = 0; t < ne; ++t) {
                if (t >= inf.lo && t < inf.hi) continue;
                M.doff[M.nt] = (uint16_t)(j * ne + t);
                M.dmod[M.nt] = (uint8_t)ext_mod(level, t);
                M.tcol[M.nt] = (uint16_t)t;
                M.tdig[M.nt] = (uint8_t)j;
                ++M.nt;
                if (J.n >= HE_MAXJ) throw HeError(HE_EUNSUPPORTED);
                J.off[J.n] = (uint16_t)(j * ne + t);
                J.mod[J.n] = (uint8_t)ext_mod(level, t);
                ++J.n;
            }
            continue;
        }
        ConvDesc D;
        memset(&D, 0, sizeof D);
        D.src = coef.p + (size_t)inf.lo * N;
        D.src_cstride = (int64_t)nl * N;
        D.dst = lift->p + (size_t)j * ne * N;
        D.dst_cstride = lcs;
        D.nct = B;
        D.npoly = 1;
        D.tab = d_mu_tab->p + inf.off;
        D.tab_ld = ne;
        D.ns = inf.hi - inf.lo;
        int nt = 0;
        for (int t = 0; t < ne; ++t) {
            if (t >= inf.lo && t < inf.hi) continue;
            D.doff[nt] = (uint16_t)t;
            D.dmod[nt] = (uint8_t)ext_mod(level, t);
            D.tcol[nt] = (uint16_t)t;
            ++nt;
            if (J.n >= HE_MAXJ) throw HeError(HE_EUNSUPPORTED);
            J.off[J.n] = (uint16_t)(j * ne + t);
            J.mod[J.n] = (uint8_t)ext_mod(level, t);
            ++J.n;
        }
        D.nt = nt;
        for (int s = 0; s < D.ns; ++s) {
            D.smod[s] = inf.lo + s;
            D.hinv[s] = inf.hinv[s];
            D.hinv_sh[s] = inf.hinv_sh[s];
        }
        D.prescaled = fused ? 1 : 0;
        if (fused) launch_conv_cols(T, D, stream);
        else launch_baseconv(T, D, stream);
    }
    if (merged) launch_conv_cols(T, M, stream);
    launch_ntt(T, J, false, stream, nullptr, 0, !fused);
    // the digits' own limbs stay where they are: the inner product reads them from the
    // polynomial (which outlives the lift wherever a lift is used)
    lift_own[lift->p] = {a.p + poly * a.ps, a.cs};
    return lift;
}

// g^-1 mod 2N (g odd): Newton's iteration x <- x (2 - g x) doubles the correct low bits
static u64 galois_inverse(u64 g, int log_n) {
    u64 x = g;  // g g = 1 mod 8
    for (int it = 0; it < 6; ++it) x *= 2 - g * x;
    return x & ((2ull << log_n) - 1);
}

// Key-switch inner products of several rotation sets of one lift in one launch: set s writes
// <lift o sigma_g, key> (+ P sigma_g(c0) on the Q limbs) of every member into
// u + s B [2][ne][N] (added to what u holds with accumulate); with nrot = 2 a set is the
// masked sum of two rotations (one ModDown then serves both)
void Ctx::g_ks_inner_sets(u64* u, const u64* lift, int B, int level, std::vector<IpSet> sets, int nrot,
                          const u64* c0, int64_t c0_cs, bool accumulate) {
    const int nl = level + 1, ne = nl + n_p;
    const int beta = (int)mu[level].size();
    if (sets.empty() || sets.size() > IP_MAXSET) throw HeError(HE_EUNSUPPORTED);
    IpDesc D;
    memset(&D, 0, sizeof D);
    D.lift = lift;
    D.u = u;
    D.lift_cs = (int64_t)beta * ne * N;
    D.u_cs = 2 * (int64_t)ne * N;
    D.nct = B;
    D.ne = ne;
    D.beta = beta;
    D.M = n_q + n_p;
    for (int t = 0; t < ne; ++t) D.mod[t] = (uint8_t)ext_mod(level, t);
    D.c0 = c0;
    D.c0_cs = c0_cs;
    D.nq = nl;
    for (int t = 0; t < nl; ++t) D.pmont[t] = hm::to_mont(pmod[t], mods[t]);
    // every group lift leaves its digits' own limbs in the lifted polynomial
    auto own_of = [&](const u64* l) {
        auto it = lift_own.find(l);
        if (it == lift_own.end()) throw HeError(HE_EUNSUPPORTED);
        return it->second;
    };
    const auto own = own_of(lift);
    D.own = own.first;
    D.own_cs = own.second;
    for (int j = 0; j < beta; ++j) {
        D.dlo[j] = (uint8_t)mu[level][j].lo;
        D.dhi[j] = (uint8_t)mu[level][j].hi;
    }
    D.nrot = nrot;
    D.nset = (int)sets.size();
    for (size_t j = 0; j < sets.size(); ++j) {
        D.s[j] = sets[j];
        D.s[j].ginv = galois_inverse(sets[j].g, log_n);
        if (sets[j].lift2) {
            const auto o2 = own_of(sets[j].lift2);
            D.s[j].own2 = o2.first;
            D.s[j].own2_cs = o2.second;
        }
    }
    D.accumulate = accumulate ? 1 : 0;
    launch_inner_product(T, D, stream);
    cnt[C_KS] += (int64_t)B * nrot * D.nset;
}

// Key-switch inner product <lift o sigma_g, key> (+ P sigma_g(c0) on the Q limbs) of every
// member into u [B][2][ne][N] (added to what u holds with accumulate); with a second
// (g2, key2) and masks, the masked sum of two rotations of the same lift (one ModDown then
// serves both)
void Ctx::g_ks_inner(u64* u, const u64* lift, int B, int level, const u64* key, u64 g, const u64* c0,
                     int64_t c0_cs, const u64* mask, const u64* key2, u64 g2, const u64* mask2, bool accumulate) {
    IpSet S;
    memset(&S, 0, sizeof S);
    S.key = key;
    S.g = g;
    S.mask = mask;
    S.key2 = key2;
    S.g2 = g2;
    S.mask2 = mask2;
    g_ks_inner_sets(u, lift, B, level, {S}, key2 ? 2 : 1, c0, c0_cs, accumulate);
}

// out = ModDown(u) (+ add gathered by add_g) (. mask) (+ acc), for every member; u as made
// by g_ks_inner.  The combine runs in the epilogue of the forward NTT of the converted
// special-prime part.
void Ctx::g_moddown(u64* u, int B, int level, const u64* add0, const u64* add1, int64_t add_cs, u64* out0,
                    u64* out1, int64_t out_cs, u64 add_g, const u64* mask, const u64* acc0, const u64* acc1,
                    int64_t acc_cs) {
    const int nl = level + 1, ne = nl + n_p;
    const int64_t ucs = 2 * (int64_t)ne * N, ccs = 2 * (int64_t)nl * N;
    // with the fused conversion, the inverse transform also applies (P/p_k)^-1
    const bool fused = conv_cols_fits(T, n_p);
    {
        Jobs J;
        J.base = u;
        J.cstride = ucs;
        J.nct = B;
        J.n = 0;
        for (int p = 0; p < 2; ++p)
            for (int k = 0; k < n_p; ++k) {
                J.off[J.n] = (uint16_t)(p * ne + nl + k);
                J.mod[J.n] = (uint8_t)(n_q + k);
                ++J.n;
            }
        launch_ntt(T, J, true, stream, fused ? d_md_scale->p : nullptr, n_p);
    }
    DBuf conv(this, (size_t)B * ccs);
    ConvDesc C;
    memset(&C, 0, sizeof C);
    C.src = u + (size_t)nl * N;
    C.src_pstride = (int64_t)ne * N;
    C.src_cstride = ucs;
    C.dst = conv.p;
    C.dst_pstride = (int64_t)nl * N;
    C.dst_cstride = ccs;
    C.nct = B;
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
    C.prescaled = fused ? 1 : 0;
    if (fused) launch_conv_cols(T, C, stream);
    else launch_baseconv(T, C, stream);
    Jobs J;
    J.base = conv.p;
    J.cstride = ccs;
    J.nct = B;
    J.n = 2 * nl;
    for (int p = 0; p < 2; ++p)
        for (int t = 0; t < nl; ++t) {
            J.off[p * nl + t] = (uint16_t)(p * nl + t);
            J.mod[p * nl + t] = (uint8_t)t;
        }
    Epi E;
    memset(&E, 0, sizeof E);
    E.on = 1;
    E.nl = nl;
    E.u = u;
    E.u_cs = ucs;
    E.u_ps = (int64_t)ne * N;
    E.add[0] = add0;
    E.add[1] = add1;
    E.add_cs = add_cs;
    E.out[0] = out0;
    E.out[1] = out1;
    E.out_cs = out_cs;
    E.pinv = d_pinv->p;
    E.pinv_sh = d_pinv->p + n_q;
    E.g = add_g;
    E.mask = mask;
    E.acc[0] = acc0;
    E.acc[1] = acc1;
    E.acc_cs = acc_cs;
    launch_ntt_moddown(T, J, E, stream, !fused);
}

// ModDown(<lift o sigma_g, key>) (+ add) into out, for every member
void Ctx::g_ks_apply(const u64* lift, int B, int level, const u64* key, u64 g, const u64* add0, const u64* add1,
                     int64_t add_cs, u64* out0, u64* out1, int64_t out_cs, u64 add_g, const u64* mask,
                     const u64* acc0, const u64* acc1, int64_t acc_cs, const u64* c0, int64_t c0_cs) {
    DBuf u(this, (size_t)B * 2 * (level + 1 + n_p) * N);
    g_ks_inner(u.p, lift, B, level, key, g, c0, c0_cs, nullptr, nullptr, 1, nullptr, false);
    g_moddown(u.p, B, level, add0, add1, add_cs, out0, out1, out_cs, add_g, mask, acc0, acc1, acc_cs);
}

// Several rotation sets of one ciphertext at once: each set's inner product goes into its
// slice of one extended-basis buffer (one launch: the sets' gathers of the shared lift meet
// in L2), and a single ModDown then serves all sets, so its transforms and conversion run as
// one launch over nset x B members; the results are views into one block
Ctx::PendingSets Ctx::g_sets_ip(const Grp& a, const u64* lift, const std::vector<IpSet>& sets, int nrot,
                                double mask_scale) {
    const int P = (int)sets.size(), B = a.B, ne = a.level + 1 + n_p;
    if (a.deg != 1) throw HeError(HE_EMISMATCH);
    PendingSets ps;
    for (int j = 0; j < P; ++j)
        for (double v : a.scale) ps.sc.push_back(v * mask_scale);
    ps.out = g_new(P * B, a.level, 1, ps.sc);
    ps.u = std::make_shared<DBuf>(this, (size_t)P * B * 2 * ne * N);
    ps.P = P;
    ps.B = B;
    ps.level = a.level;
    g_ks_inner_sets(ps.u->p, lift, B, a.level, sets, nrot, a.p, a.cs, false);
    return ps;
}

std::vector<Grp> Ctx::g_sets_finish(PendingSets& ps) {
    const int P = ps.P, B = ps.B;
    Grp& out = ps.out;
    g_moddown(ps.u->p, P * B, ps.level, nullptr, nullptr, 0, out.p, out.p + out.ps, out.cs, 1, nullptr, nullptr,
              nullptr, 0);
    ps.u.reset();
    std::vector<Grp> res(P);
    for (int j = 0; j < P; ++j) {
        res[j] = out;
        res[j].B = B;
        res[j].p = out.p + (size_t)j * B * out.cs;
        res[j].scale.assign(ps.sc.begin() + (size_t)j * B, ps.sc.begin() + (size_t)(j + 1) * B);
    }
    return res;
}

std::vector<Grp> Ctx::g_rotate_sets_hoisted(const Grp& a, const u64* lift, const std::vector<IpSet>& sets,
                                            int nrot, double mask_scale) {
    PendingSets ps = g_sets_ip(a, lift, sets, nrot, mask_scale);
    return g_sets_finish(ps);
}

// Several mask pairs of one ciphertext at once (Step 2 under the hoisted-ModDown schedule):
// mask1 . Rot(a, k1) + mask2 . Rot(a, k2) for every pair, with one shared ModDown; the inner
// products here, the ModDown by g_sets_finish
Ctx::PendingSets Ctx::g_pairs_ip(const Grp& a, const u64* lift, const std::vector<MaskPair>& pr, double mask_scale) {
    const int P = (int)pr.size(), B = a.B;
    std::vector<IpSet> sets(P);
    for (int j = 0; j < P; ++j) {
        const u64 g1 = galois(pr[j].k1), g2 = galois(pr[j].k2);
        if (g1 == 1 || g2 == 1) throw HeError(HE_EUNSUPPORTED);
        memset(&sets[j], 0, sizeof(IpSet));
        sets[j].key = rot_key(g1, false);
        sets[j].g = g1;
        sets[j].mask = pr[j].m1;
        sets[j].key2 = rot_key(g2, false);
        sets[j].g2 = g2;
        sets[j].mask2 = pr[j].m2;
    }
    PendingSets ps = g_sets_ip(a, lift, sets, 2, mask_scale);
    cnt[C_ROT] += 2 * P * B;
    cnt[C_MULPT] += 2 * P * B;
    cnt[C_ADD] += P * B;
    return ps;
}

std::vector<Grp> Ctx::g_rotate_pairs_hoisted(const Grp& a, const u64* lift, const std::vector<MaskPair>& pr,
                                             double mask_scale) {
    PendingSets ps = g_pairs_ip(a, lift, pr, mask_scale);
    return g_sets_finish(ps);
}

// Rot(a, k) for several k of one lift, with one shared ModDown (Step 3's baby rotations
// under the hoisted-ModDown schedule); identical to rotating one at a time
std::vector<Grp> Ctx::g_rotate_many_hoisted(const Grp& a, const u64* lift, const std::vector<int64_t>& ks) {
    const int P = (int)ks.size(), B = a.B;
    std::vector<IpSet> sets(P);
    for (int j = 0; j < P; ++j) {
        const u64 g = galois(ks[j]);
        if (g == 1) throw HeError(HE_EUNSUPPORTED);
        memset(&sets[j], 0, sizeof(IpSet));
        sets[j].key = rot_key(g, false);
        sets[j].g = g;
    }
    auto res = g_rotate_sets_hoisted(a, lift, sets, 1, 1.0);
    cnt[C_ROT] += (int64_t)P * B;
    return res;
}

// Hoisted rotation sums: base + sum_w Rot(a_w, r_w) with one ModDown.  The terms' key-switch
// inner products (with P sigma_g(c0_w)) are accumulated in the extended basis two at a time
// (a term waits for the next one, then both go in one launch and their lifts are freed);
// finish adds a last unpaired term, brings the sum down once and adds the unrotated base in
// the ModDown epilogue.  Exact apart from the one shared ModDown rounding.
void Ctx::g_rotsum_add(RotSum& S, const Grp& a, int64_t r) {
    if (a.deg != 1) throw HeError(HE_EMISMATCH);
    if (!S.u) {
        S.B = a.B;
        S.level = a.level;
        S.n = 0;
        S.filled = false;
        S.scale = a.scale;
        S.u = std::make_shared<DBuf>(this, (size_t)a.B * 2 * (a.level + 1 + n_p) * N);
    }
    if (a.B != S.B || a.level != S.level) throw HeError(HE_EMISMATCH);
    const u64 g = galois(r);
    if (g == 1) throw HeError(HE_EUNSUPPORTED);
    rot_key(g, false);
    auto lift = g_lift(a, 1);
    if (!S.plift) {
        S.plift = lift;
        S.pa = a;
        S.pg = g;
    } else {
        // the waiting term and this one in one launch, each rotation gathering its own lift
        IpSet st;
        memset(&st, 0, sizeof st);
        st.key = rot_key(S.pg, false);
        st.g = S.pg;
        st.key2 = rot_key(g, false);
        st.g2 = g;
        st.lift2 = lift->p;
        st.c0_2 = a.p;
        st.c0_2_cs = a.cs;
        g_ks_inner_sets(S.u->p, S.plift->p, a.B, a.level, {st}, 2, S.pa.p, S.pa.cs, S.filled);
        S.filled = true;
        S.plift.reset();
        S.pa = Grp();
    }
    for (int i = 0; i < a.B; ++i) S.scale[i] = std::max(S.scale[i], a.scale[i]);
    ++S.n;
    cnt[C_ROT] += a.B;
}

Grp Ctx::g_rotsum_finish(RotSum& S, const Grp* base) {
    if (!S.u) throw HeError(HE_EUNSUPPORTED);
    if (base && (base->B != S.B || base->level != S.level || base->deg != 1)) throw HeError(HE_EMISMATCH);
    if (S.plift) {  // a last term without a partner
        g_ks_inner(S.u->p, S.plift->p, S.B, S.level, rot_key(S.pg, false), S.pg, S.pa.p, S.pa.cs, nullptr, nullptr,
                   1, nullptr, S.filled);
        S.filled = true;
        S.plift.reset();
        S.pa = Grp();
    }
    std::vector<double> sc(S.scale);
    if (base)
        for (int i = 0; i < S.B; ++i) sc[i] = std::max(sc[i], base->scale[i]);
    Grp out = g_new(S.B, S.level, 1, sc);
    g_moddown(S.u->p, S.B, S.level, base ? base->p : nullptr, base ? base->p + base->ps : nullptr, base ? base->cs : 0,
              out.p, out.p + out.ps, out.cs, 1, nullptr, nullptr, nullptr, 0);
    cnt[C_ADD] += (int64_t)S.B * (S.n - 1 + (base ? 1 : 0));
    S = RotSum();
    return out;
}

Grp Ctx::g_rotate_from_lift(const Grp& a, const u64* lift, int64_t k) {
    const u64 g = galois(k);
    if (g == 1) return g_drop(a, a.level);
    const u64* key = rot_key(g, false);
    Grp out = g_new(a.B, a.level, 1, a.scale);
    // out0 = ModDown(.) + sigma_g(c0): the automorphism of c0 is a gather in the epilogue
    g_ks_apply(lift, a.B, a.level, key, g, nullptr, nullptr, 0, out.p, out.p + out.ps, out.cs, g, nullptr, nullptr,
               nullptr, 0, a.p, a.cs);
    cnt[C_ROT] += a.B;
    return out;
}

// Rot(a, k) . mask (+ acc): the Mul_pt (and the Add of a diagonal sum) fused into the
// rotation's ModDown epilogue; exact residues, so identical to rotating then masking
Grp Ctx::g_rotate_mask_from_lift(const Grp& a, const u64* lift, int64_t k, const u64* mask, double mask_scale,
                                 const Grp* acc) {
    const u64 g = galois(k);
    if (g == 1) throw HeError(HE_EUNSUPPORTED);
    const u64* key = rot_key(g, false);
    std::vector<double> sc(a.scale);
    for (auto& v : sc) v *= mask_scale;
    Grp out = g_new(a.B, a.level, 1, sc);
    g_ks_apply(lift, a.B, a.level, key, g, nullptr, nullptr, 0, out.p, out.p + out.ps, out.cs, g, mask,
               acc ? acc->p : nullptr, acc ? acc->p + acc->ps : nullptr, acc ? acc->cs : 0, a.p, a.cs);
    cnt[C_ROT] += a.B;
    cnt[C_MULPT] += a.B;
    if (acc) {
        cnt[C_ADD] += a.B;
        for (int i = 0; i < a.B; ++i) out.scale[i] = std::max(out.scale[i], acc->scale[i]);
    }
    return out;
}

Grp Ctx::g_rotate(const Grp& a, int64_t k) {
    if (galois(k) == 1) return g_drop(a, a.level);
    rot_key(galois(k), false);
    auto lift = g_lift(a, 1);
    return g_rotate_from_lift(a, lift->p, k);
}

Grp Ctx::g_mask_sum(const std::vector<std::pair<const Grp*, const u64*>>& terms, double mask_scale) {
    const Grp& a0 = *terms[0].first;
    std::vector<double> sc(a0.scale);
    for (auto& s : sc) s *= mask_scale;
    Grp out = g_new(a0.B, a0.level, 1, sc);
    for (size_t base = 0; base < terms.size(); base += 16) {
        MacDesc D;
        memset(&D, 0, sizeof D);
        D.nct = a0.B;
        D.nterm = (int)std::min<size_t>(16, terms.size() - base);
        for (int t = 0; t < D.nterm; ++t) {
            const Grp* g = terms[base + t].first;
            if (g->level != a0.level || g->deg != 1 || g->B != a0.B) throw HeError(HE_EMISMATCH);
            D.in[t] = g->p;
            D.in_ps[t] = g->ps;
            D.in_cs[t] = g->cs;
            D.mask[t] = terms[base + t].second;
        }
        launch_mask_mac(T, a0.level + 1, 2, D, out.p, out.ps, base > 0, stream, out.cs);
    }
    cnt[C_MULPT] += (int64_t)terms.size() * a0.B;
    cnt[C_ADD] += ((int64_t)terms.size() - 1) * a0.B;
    return out;
}

Grp Ctx::g_rescale(const Grp& a) {
    if (a.level < 1) throw HeError(HE_ELEVEL);
    const int l = a.level, np = a.deg + 1, B = a.B;
    DBuf last(this, (size_t)B * np * N);
    copy2d(this, last.p, N, a.p + (size_t)l * N, a.ps, N, (int64_t)B * np);
    {
        Jobs J;
        J.base = last.p;
        J.cstride = N;
        J.nct = B * np;
        J.n = 1;
        J.off[0] = 0;
        J.mod[0] = (uint8_t)l;
        launch_ntt(T, J, true, stream);
    }
    DBuf tmp(this, (size_t)B * np * l * N);
    launch_rescale_spread(T, l, B * np, last.p, N, l, tmp.p, (int64_t)l * N, stream);
    {
        Jobs J;
        J.base = tmp.p;
        J.cstride = (int64_t)l * N;
        J.nct = B * np;
        J.n = l;
        for (int i = 0; i < l; ++i) {
            J.off[i] = (uint16_t)i;
            J.mod[i] = (uint8_t)i;
        }
        launch_ntt(T, J, false, stream);
    }
    std::vector<double> sc(a.scale);
    for (auto& s : sc) s /= (double)mods[l];
    Grp out = g_new(B, l - 1, a.deg, sc);
    const u64* qi = d_rs->p + (size_t)l * n_q;
    const u64* qis = d_rs->p + (size_t)n_q * n_q + (size_t)l * n_q;
    launch_rescale_combine(T, l, np, a.p, a.ps, tmp.p, (int64_t)l * N, qi, qis, out.p, out.ps, stream, B, a.cs,
                           (int64_t)np * l * N, out.cs);
    cnt[C_RS] += B;
    return out;
}

Grp Ctx::g_tensor(const Grp& a, const Grp& b) {
    if (a.deg != 1 || b.deg != 1 || a.B != b.B || a.level != b.level) throw HeError(HE_EMISMATCH);
    std::vector<double> sc(a.B);
    for (int i = 0; i < a.B; ++i) sc[i] = a.scale[i] * b.scale[i];
    Grp out = g_new(a.B, a.level, 2, sc);
    launch_tensor(T, a.level + 1, a.p, a.ps, b.p, b.ps, out.p, out.ps, 0, stream, a.B, a.cs, b.cs, out.cs);
    cnt[C_MULCT] += a.B;
    return out;
}

void Ctx::g_tensor_acc(Grp& acc, const Grp& a, const Grp& b) {
    if (a.deg != 1 || b.deg != 1 || acc.deg != 2 || a.level != acc.level || b.level != acc.level)
        throw HeError(HE_EMISMATCH);
    launch_tensor(T, a.level + 1, a.p, a.ps, b.p, b.ps, acc.p, acc.ps, 1, stream, a.B, a.cs, b.cs, acc.cs);
    cnt[C_MULCT] += a.B;
    cnt[C_ADD] += a.B;
}

// J.S (+)= sum over the pending pairs of A (x) B in one pass (relin-once schedules)
void Ctx::g_tensor_sum(MatmulJob& J) {
    if (J.pendA.empty()) return;
    const Grp& a0 = J.pendA[0];
    if (!J.haveS) {
        std::vector<double> sc(a0.B);
        for (int i = 0; i < a0.B; ++i) sc[i] = a0.scale[i] * J.pendB[0].scale[i];
        J.S = g_new(a0.B, a0.level, 2, sc);
    }
    TensorSumDesc D;
    memset(&D, 0, sizeof D);
    D.n = (int)J.pendA.size();
    D.nct = a0.B;
    D.acc = J.haveS ? 1 : 0;
    D.d = J.S.p;
    D.d_ps = J.S.ps;
    D.d_cs = J.S.cs;
    for (int j = 0; j < D.n; ++j) {
        const Grp &a = J.pendA[j], &b = J.pendB[j];
        if (a.deg != 1 || b.deg != 1 || a.level != J.S.level || b.level != J.S.level || a.B != a0.B)
            throw HeError(HE_EMISMATCH);
        D.a[j] = a.p;
        D.a_ps[j] = a.ps;
        D.a_cs[j] = a.cs;
        D.b[j] = b.p;
        D.b_ps[j] = b.ps;
        D.b_cs[j] = b.cs;
        // Add of Fig. 1: scale max (all terms of a block share one scale)
        for (int i = 0; i < a0.B; ++i) J.S.scale[i] = std::max(J.S.scale[i], a.scale[i] * b.scale[i]);
    }
    launch_tensor_sum(T, J.S.level + 1, D, stream);
    cnt[C_MULCT] += (int64_t)D.n * a0.B;
    cnt[C_ADD] += (int64_t)(D.n - 1 + D.acc) * a0.B;
    J.haveS = true;
    J.pendA.clear();
    J.pendB.clear();
}

Grp Ctx::g_relin(const Grp& a) {
    if (a.deg != 2) throw HeError(HE_EMISMATCH);
    const u64* key = relin_key();
    auto lift = g_lift(a, 2);
    Grp out = g_new(a.B, a.level, 1, a.scale);
    g_ks_apply(lift->p, a.B, a.level, key, 1, a.p, a.p + a.ps, a.cs, out.p, out.p + out.ps, out.cs, 1, nullptr,
               nullptr, nullptr, 0, nullptr, 0);
    return out;
}

// ------------------------------------------------------------------ the product
static int floordiv_g(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Phase 0: Step 1-1 and Step 1-2 and the lifts of A0, B0.  Phases 1..: k_chunk rounds
// of Steps 2-3 each.  Last phase: relinearisation (relin-once schedule) and the final
// RS.  The phases follow the order of the unphased evaluation exactly.
// HE-LinTrans (Alg. 2) with the baby-step/giant-step split (App. B) for every member: the sum
// over diagonals d in [dlo, dhi] of mask_d . R(a, unit d), as
//   sum_i Rot( sum_j R(mask_{b i + j}, -unit b i) . Rot(a, unit j), unit b i ),
// under the packing iota_beta (amounts times beta); baby rotations share one lift, giant
// steps share one ModDown under the hoisting flag.  No rescale.
Grp Ctx::g_lintrans(const Grp& a, int kind, int h, int beta, int64_t unit, int dlo, int dhi) {
    const int b = bsgs(h);
    const double ms = scale;
    const bool hoist = (schedule & HE_SCHED_HOIST_MODDOWN) != 0;
    std::vector<Grp> baby(b);
    baby[0] = a;
    if (b > 1) {
        auto lift = g_lift(a, 1);
        if (hoist) {
            // up to pair_batch babies per launch, with one shared ModDown
            // (a rotation that is the identity on the slots is the ciphertext itself)
            std::vector<int> js;
            for (int j = 1; j < b; ++j) {
                if (galois((int64_t)beta * unit * j) == 1) baby[j] = g_drop(a, a.level);
                else js.push_back(j);
            }
            const size_t pb = (size_t)std::max(1, pair_batch);
            for (size_t j0 = 0; j0 < js.size(); j0 += pb) {
                std::vector<int64_t> ks;
                for (size_t j = j0; j < std::min(js.size(), j0 + pb); ++j) ks.push_back((int64_t)beta * unit * js[j]);
                auto r = g_rotate_many_hoisted(a, lift->p, ks);
                for (size_t j = 0; j < r.size(); ++j) baby[js[j0 + j]] = r[j];
            }
        } else {
            for (int j = 1; j < b; ++j) baby[j] = g_rotate_from_lift(a, lift->p, (int64_t)beta * unit * j);
        }
    }
    RotSum gsum;
    Grp acc;
    bool have = false;
    // the giant-step inner sums sum_j R(mask_{b i + j}, -unit b i) . baby_j, computed a few
    // giant steps per launch (the babies are read once per launch), each chunk consumed
    // before the next is made
    const int glo = floordiv_g(dlo, b), ghi = floordiv_g(dhi, b);
    const int per = b > 8 ? 2 : MM_OUT;
    for (int i0 = glo; i0 <= ghi; i0 += per) {
        MultiMacDesc D;
        memset(&D, 0, sizeof D);
        D.nin = b;
        D.nct = a.B;
        for (int j = 0; j < b; ++j) {
            D.in[j] = baby[j].p;
            D.in_ps[j] = baby[j].ps;
            D.in_cs[j] = baby[j].cs;
        }
        std::vector<std::pair<int, Grp>> inners;
        for (int i = i0; i <= std::min(ghi, i0 + per - 1); ++i) {
            int nterm = 0;
            const u64* mk[16] = {nullptr};
            for (int j = 0; j < b; ++j) {
                const int d = b * i + j;
                if (d < dlo || d > dhi) continue;
                mk[j] = mask(kind, h, d, -unit * b * i, beta);
                ++nterm;
            }
            if (!nterm) continue;
            std::vector<double> sc(a.scale);
            for (auto& v : sc) v *= ms;
            Grp g = g_new(a.B, a.level, 1, sc);
            D.out_ps = g.ps;
            D.out_cs = g.cs;
            for (int j = 0; j < b; ++j) D.mask[D.nout][j] = mk[j];
            D.out[D.nout++] = g.p;
            inners.push_back({i, g});
            cnt[C_MULPT] += (int64_t)nterm * a.B;
            cnt[C_ADD] += (int64_t)(nterm - 1) * a.B;
        }
        if (D.nout) launch_mask_mac_multi(T, a.level + 1, 2, D, stream);
        for (auto& ig : inners) {
            const int i = ig.first;
            Grp inner = ig.second;
            const int64_t r = (int64_t)beta * unit * b * i;
            if (i && hoist) {
                g_rotsum_add(gsum, inner, r);
                continue;
            }
            if (i) inner = g_rotate(inner, r);
            if (!have) {
                acc = inner;
                have = true;
            } else {
                g_add_into(acc, inner);
            }
        }
    }
    if (gsum.u) acc = g_rotsum_finish(gsum, have ? &acc : nullptr);
    return acc;
}

// Phase 0: Step 1-1 and Step 1-2 and the lifts of A0, B0.  Phases 1..: k_chunk rounds
// of Steps 2-3 each (t rounds in all; t < h for HE-RMatMult).  Last phase: the final RS
// (twice under late rescaling) and, for t < h, the fold of the h/t row blocks (Alg. 6).
// The phases follow the order of the unphased evaluation exactly.
bool Ctx::matmul_step(MatmulJob& J, int k_chunk) {
    const int h = J.h, t = J.t ? J.t : J.h, beta = J.beta;
    const double ms = scale;
    const bool hoist = (schedule & HE_SCHED_HOIST_MODDOWN) != 0;
    if (J.phase == 0) {
        Grp a = g_gather(J.A, J.lvl), bb = g_gather(J.B, J.lvl);
        // Step 1-1: A0 = U^mu A (diagonals k in (-h, h) at unit 1), then RS
        J.A0 = g_rescale(g_lintrans(a, 0, h, beta, 1, 1 - h, h - 1));
        // Step 1-2: B0 = U^zeta B (diagonals h k, k in [0, h)), then RS
        J.B0 = g_rescale(g_lintrans(bb, 1, h, beta, h, 0, h - 1));
        // brought to the Step-3 level before its rotations (with late rescaling Step 3
        // multiplies at this level)
        if (!(schedule & HE_SCHED_RESCALE_LATE)) J.B0 = g_drop(J.B0, J.B0.level - 1);
        J.liftA = g_lift(J.A0, 1);
        J.liftB = g_lift(J.B0, 1);
        J.k = 0;
        J.phase = 1;
        return false;
    }
    if (J.phase == 1) {
        // Steps 2 and 3 in blocks k = bg i + j (one block of h without the Step-3 split):
        //   A^(k) shifted by s = h bg i: R(v_k, -s) . Rot(A0, k - s) + R(v_{k-h}, -s) . Rot(A0, k - h - s)
        //   (RS unless late), times Rot(B0, h j), summed over j; the block sum is relinearised
        //   (relin-once) and rotated by s
        const int bg = step3_baby(t);
        const bool keep_baby = bg < t;
        if (keep_baby && J.babyB.empty()) J.babyB.resize(bg);
        const int kend = std::min(t, J.k + std::max(1, k_chunk));
        // hoisted schedule: the mask pairs of up to pair_batch consecutive k share one ModDown;
        // with overlap, the next group's inner products run on the side stream during this
        // group's ModDown (within this chunk of rounds only)
        std::vector<Grp> pairs, babies;
        int pairs_k0 = 0, babies_j0 = 0;
        auto pair_group = [&](int k0) {
            std::vector<MaskPair> pr;
            for (int kk = k0; kk < std::min(kend, k0 + std::max(1, pair_batch)); ++kk) {
                const int64_t sh = (int64_t)h * bg * (kk / bg);
                pr.push_back({beta * (kk - sh), mask(2, h, kk, -sh, beta), beta * (kk - h - sh),
                              mask(3, h, kk, -sh, beta)});
            }
            return pr;
        };
        PendingSets next;
        int next_k0 = -1;
        struct SideJoin {  // side-stream work still queued (an error path) ends before its buffers go
            Ctx* c;
            const int* pending;
            ~SideJoin() {
                if (*pending >= 0) (void)hipStreamSynchronize(c->side);
            }
        } side_join{this, &next_k0};
        for (int k = J.k; k < kend; ++k) {
            const int i = k / bg, j = k % bg;
            const int64_t shift = (int64_t)h * bg * i;
            Grp Ak;
            if (k == 0) {
                Ak = g_mask_sum({{&J.A0, mask(2, h, 0, 0, beta)}}, ms);
            } else if (hoist) {
                if (pairs.empty() || k - pairs_k0 >= (int)pairs.size()) {
                    PendingSets cur;
                    if (next_k0 == k) {  // issued on the side stream: join it
                        hip_check(hipStreamWaitEvent(stream, ev_join, 0), "join side stream");
                        cur = std::move(next);
                        next = PendingSets();
                        next_k0 = -1;
                    } else {
                        cur = g_pairs_ip(J.A0, J.liftA->p, pair_group(k), ms);
                    }
                    const int k1 = k + cur.P;
                    if (overlap && k1 < kend && ensure_side() && stream != side) {
                        std::vector<MaskPair> pr = pair_group(k1);  // masks on the context stream
                        hip_check(hipEventRecord(ev_fork, stream), "fork side stream");
                        hip_check(hipStreamWaitEvent(side, ev_fork, 0), "fork side stream");
                        hipStream_t main_stream = stream;
                        stream = side;
                        try {
                            next = g_pairs_ip(J.A0, J.liftA->p, pr, ms);
                            next_k0 = k1;
                            hip_check(hipEventRecord(ev_join, side), "side stream done");
                        } catch (...) {
                            stream = main_stream;
                            throw;
                        }
                        stream = main_stream;
                    }
                    pairs = g_sets_finish(cur);
                    pairs_k0 = k;
                }
                Ak = pairs[k - pairs_k0];
            } else {
                // masks applied in the ModDown epilogues
                Grp t1 = g_rotate_mask_from_lift(J.A0, J.liftA->p, beta * (k - shift), mask(2, h, k, -shift, beta), ms,
                                                 nullptr);
                Ak = g_rotate_mask_from_lift(J.A0, J.liftA->p, beta * (k - h - shift), mask(3, h, k, -shift, beta), ms,
                                             &t1);
            }
            if (!(schedule & HE_SCHED_RESCALE_LATE)) Ak = g_rescale(Ak);
            Grp Bj;
            if (j == 0) {
                Bj = J.B0;
            } else if (i > 0) {
                Bj = J.babyB[j];
            } else if (hoist) {
                // baby rotations of B0, up to pair_batch at a time with one shared ModDown
                // (kept for the later blocks, or until used within this chunk)
                if (keep_baby ? !J.babyB[j].p : (babies.empty() || j - babies_j0 >= (int)babies.size())) {
                    const int jend = std::min(keep_baby ? bg : kend, j + std::max(1, pair_batch));
                    std::vector<int64_t> ks;
                    for (int jj = j; jj < jend; ++jj) ks.push_back((int64_t)beta * h * jj);
                    babies = g_rotate_many_hoisted(J.B0, J.liftB->p, ks);
                    babies_j0 = j;
                    if (keep_baby)
                        for (int jj = j; jj < jend; ++jj) J.babyB[jj] = babies[jj - j];
                }
                Bj = keep_baby ? J.babyB[j] : babies[j - babies_j0];
            } else {
                Bj = g_rotate_from_lift(J.B0, J.liftB->p, (int64_t)beta * h * j);
                if (keep_baby) J.babyB[j] = Bj;
            }
            if (!(schedule & HE_SCHED_RELIN_ONCE)) {
                Grp prod = g_relin(g_tensor(Ak, Bj));
                if (!J.haveS) {
                    J.S = prod;
                    J.haveS = true;
                } else {
                    g_add_into(J.S, prod);
                }
            } else {
                // products of a block are summed in one pass (at most 16 pairs per pass)
                J.pendA.push_back(Ak);
                J.pendB.push_back(Bj);
                if (J.pendA.size() == 16) g_tensor_sum(J);
            }
            if (j == bg - 1 || k == t - 1) {
                g_tensor_sum(J);
                Grp blk = J.S;
                J.S = Grp();
                J.haveS = false;
                if (schedule & HE_SCHED_RELIN_ONCE) blk = g_relin(blk);
                if (i > 0 && hoist) {
                    g_rotsum_add(J.giant, blk, beta * shift);
                    continue;
                }
                if (i > 0) blk = g_rotate(blk, beta * shift);
                if (!J.have) {
                    J.acc = blk;
                    J.have = true;
                } else {
                    g_add_into(J.acc, blk);
                }
            }
        }
        J.k = kend;
        if (J.k == t) {
            J.liftA.reset();
            J.liftB.reset();
            J.A0 = Grp();
            J.B0 = Grp();
            J.babyB.clear();
            J.phase = 2;
        }
        return false;
    }
    if (J.giant.u) J.acc = g_rotsum_finish(J.giant, J.have ? &J.acc : nullptr);
    J.acc = g_rescale(J.acc);
    if (schedule & HE_SCHED_RESCALE_LATE) J.acc = g_rescale(J.acc);
    // Alg. 6's last loop: fold the h/t row blocks of t rows (after the rescales: fewer limbs)
    for (int sh = 0; (t << sh) < h; ++sh) {
        Grp r = g_rotate(J.acc, ((int64_t)beta * t * h) << sh);
        g_add_into(J.acc, r);
    }
    if (!J.keep_acc) {
        J.result = g_scatter(J.acc);
        J.acc = Grp();
    }
    J.phase = 3;
    return true;
}

std::vector<CtPtr> Ctx::matmul_group(const std::vector<const CtData*>& A, const std::vector<const CtData*>& Bv,
                                     const MatShape& sh, int lvl) {
    MatmulJob J;
    J.A = A;
    J.B = Bv;
    J.h = sh.h;
    J.t = sh.t;
    J.beta = sh.beta;
    J.lvl = lvl;
    while (!matmul_step(J, sh.h)) {
    }
    return J.result;
}

// ------------------------------------------------------------------ sign (Sec. 4.2), lockstep
// numerators of the m^(2i+1) coefficients of g_d over 2^(2d-1)
static std::vector<int64_t> gd_numerators(int d) {
    auto binom = [](int n, int r) {
        int64_t v = 1;
        for (int i = 1; i <= r; ++i) v = v * (n - r + i) / i;
        return v;
    };
    std::vector<int64_t> num(d + 1, 0);
    for (int j = 0; j <= d; ++j)  // 4^-j C(2j, j) m (1 - m^2)^j, scaled by 4^d
        for (int i = 0; i <= j; ++i) {
            const int64_t t = binom(2 * j, j) * binom(j, i) * ((int64_t)1 << (2 * (d - j)));
            num[i] += (i & 1) ? -t : t;
        }
    for (auto& v : num) v /= 2;
    return num;
}

// the integer constant of x_c = RS(x K) for the coefficient num / 2^e:
// K = round(num / 2^e * q_l * ratio), half away from zero, ratio = (scale x_c must carry) /
// (scale of x); double arithmetic in this exact order
static int64_t scaled_const(int64_t num, int e, u64 ql, double ratio) {
    return std::llround((double)num / (double)((int64_t)1 << e) * (double)ql * ratio);
}

// every member times its own integer constant k[m] (members with equal constants share a
// launch)
Grp Ctx::g_mul_int(const Grp& a, const std::vector<int64_t>& k) {
    const int nl = a.level + 1;
    Grp r = g_new(a.B, a.level, a.deg, a.scale);
    std::vector<u64> c(2 * nl);
    for (int m0 = 0; m0 < a.B;) {
        int m1 = m0 + 1;
        while (m1 < a.B && k[m1] == k[m0]) ++m1;
        for (int i = 0; i < nl; ++i) {
            const u64 q = mods[i];
            const u64 v = k[m0] >= 0 ? (u64)k[m0] % q : (q - (u64)(-(k[m0] + 1)) % q - 1) % q;
            c[i] = v;
            c[nl + i] = hm::shoup(v, q);
        }
        DBuf dc(this, 2 * (size_t)nl);
        hip_check(hipMemcpyAsync(dc.p, c.data(), c.size() * 8, hipMemcpyHostToDevice, stream), "mul_int consts");
        hip_check(hipStreamSynchronize(stream), "mul_int consts");
        // members m0..m1-1 are (m1 - m0) * (deg+1) polynomials with a uniform poly stride
        launch_mul_const(T, ModMap{1 << 20, n_q}, nl, (m1 - m0) * (a.deg + 1), r.p + (size_t)m0 * r.cs, r.ps,
                         a.p + (size_t)m0 * a.cs, a.ps, dc.p, dc.p + nl, stream);
        m0 = m1;
    }
    return r;
}

Grp Ctx::g_mul_rs(const Grp& x, const Grp& y) {
    const int l = std::min(x.level, y.level);
    Grp a = x.level == l ? x : g_drop(x, l);
    Grp b = y.level == l ? y : g_drop(y, l);
    return g_rescale(g_relin(g_tensor(a, b)));
}

// g_d(x) = sum_i c_{2i+1} x^(2i+1): x_c = RS(x * round(c q_l)) lands at the scale of x;
// x^(2i) comes from the powers x^2, x^4, ... multiplied in along the set bits of i.
Grp Ctx::g_eval_gd(const Grp& x, int d, const std::vector<double>& target) {
    const auto num = gd_numerators(d);
    const int e = 2 * d - 1;
    int nb = 0;
    while ((1 << nb) <= d) ++nb;
    std::vector<Grp> pw(nb);
    for (int b = 0; b < nb; ++b) pw[b] = b ? g_mul_rs(pw[b - 1], pw[b - 1]) : g_mul_rs(x, x);
    const u64 ql = mods[x.level];
    Grp y;
    bool have = false;
    for (int i = 0; i <= d; ++i) {
        // scale matching: x_c carries the scale 'need' that the products with the powers
        // and their rescales bring back exactly to the scale of x, so every term of the sum
        // lands on one scale; need / scale(x) is folded into the integer constant
        std::vector<double> need(x.B);
        std::vector<int64_t> K(x.B);
        for (int m = 0; m < x.B; ++m) {
            double nd = target[m];
            int lv = x.level - 1;
            for (int b = 0; b < nb; ++b)
                if ((i >> b) & 1) {
                    const int l = std::min(lv, pw[b].level);
                    nd = nd * (double)mods[l] / pw[b].scale[m];
                    lv = l - 1;
                }
            need[m] = nd;
            K[m] = scaled_const(num[i], e, ql, nd / x.scale[m]);
        }
        Grp term = g_rescale(g_mul_int(x, K));
        term.scale = need;  // value c_i x carried at scale need
        for (int b = 0; b < nb; ++b)
            if ((i >> b) & 1) term = g_mul_rs(term, pw[b]);
        if (!have) {
            y = term;
            have = true;
        } else {
            // Add: level min, scale max (Fig. 1)
            const int l = std::min(y.level, term.level);
            if (y.level != l) y = g_drop(y, l);
            if (term.level != l) term = g_drop(term, l);
            g_add_into(y, term);
        }
    }
    return y;
}

Grp Ctx::g_ew(const Grp& a, const Grp& b, int op) {
    if (a.B != b.B || a.level != b.level || a.deg != b.deg) throw HeError(HE_EMISMATCH);
    std::vector<double> sc(a.B);
    for (int i = 0; i < a.B; ++i) sc[i] = std::max(a.scale[i], b.scale[i]);  // Fig. 1 Add/Sub
    Grp out = g_new(a.B, a.level, a.deg, sc);
    launch_ew(T, ModMap{1 << 20, n_q}, a.level + 1, a.deg + 1, out.p, out.ps, a.p, a.ps, b.p, b.ps, op, stream, a.B,
              out.cs, a.cs, b.cs);
    cnt[C_ADD] += a.B;
    return out;
}

bool Ctx::sign_step(SignJob& J) {
    if (J.it == 0 && !J.started) {
        if (J.mode == 2) {  // AppMax: m = a - b, s = a + b
            Grp a = J.pre ? J.ga : g_gather(J.X, J.lvl), b = J.pre ? J.gb : g_gather(J.Y, J.lvl);
            J.x = g_ew(a, b, EW_SUB);
            J.s = g_ew(a, b, EW_ADD);
            J.ga = Grp();
            J.gb = Grp();
        } else {
            J.x = J.pre ? J.ga : g_gather(J.X, J.lvl);
        }
        J.cur = J.x;
        J.started = true;
    }
    if (J.mode == 3) {  // x^2 or x . x^2
        J.cur = g_mul_rs(J.x, J.x);
        if (J.k == 3) J.cur = g_mul_rs(J.x, J.cur);
        J.result = g_scatter(J.cur);
        J.x = Grp();
        J.cur = Grp();
        return true;
    }
    if (J.it < J.k) {
        // each composition returns its input's scale; for ReLU / AppMax the last one lands on
        // the prime q_l that the product x g rescales by, so x g comes out exactly at the
        // scale of x and the final sum adds equal scales
        std::vector<double> target(J.cur.scale);
        if (J.mode && J.it == J.k - 1) {
            int nb = 0;
            while ((1 << nb) <= J.d) ++nb;
            for (auto& t : target) t = (double)mods[J.cur.level - (nb + 1)];
        }
        J.cur = g_eval_gd(J.cur, J.d, target);
        ++J.it;
        if (J.it < J.k || J.mode) return false;
    }
    if (J.mode) {  // ReLU: (x + x g) / 2; AppMax: ((a + b) + m g) / 2; the halving kept in the scale
        Grp r = g_mul_rs(J.x, J.cur);
        Grp xd = g_drop(J.mode == 2 ? J.s : J.x, r.level);
        g_add_into(r, xd);
        for (auto& sc : r.scale) sc *= 2.0;
        J.cur = r;
    }
    if (J.keep)
        J.out = J.cur;
    else
        J.result = g_scatter(J.cur);
    J.x = Grp();
    J.s = Grp();
    J.cur = Grp();
    return true;
}

// Alg. 5 on groups (used by max pooling)
Grp Ctx::g_appmax(const Grp& a, const Grp& b, int d, int k) {
    SignJob J;
    J.pre = J.keep = true;
    J.ga = a;
    J.gb = b;
    J.d = d;
    J.k = k;
    J.mode = 2;
    J.lvl = a.level;
    while (!sign_step(J)) {
    }
    return J.out;
}

// 2 x 2 max pooling of packed h x h matrices: AppMax over horizontal neighbours (rotation by
// 1), then over vertical neighbours (rotation by h), for every member (grouped by level)
std::vector<CtPtr> Ctx::maxpool_batch(const std::vector<const CtData*>& X, int h, int d, int k) {
    if (h < 2 || (h & (h - 1)) || (int64_t)h * h > N / 2) throw HeError(HE_ESHAPE);
    if (d < 1 || d > 7 || k < 1) throw HeError(HE_EINVAL);
    int nb = 0;
    while ((1 << nb) <= d) ++nb;
    rot_key(galois(1), true);
    rot_key(galois(h), true);
    std::map<int, std::vector<size_t>> groups;
    for (size_t i = 0; i < X.size(); ++i) {
        if (X[i]->deg != 1) throw HeError(HE_EMISMATCH);
        if (X[i]->level < 2 * (k * (nb + 1) + 1)) throw HeError(HE_ELEVEL);
        groups[X[i]->level].push_back(i);
    }
    std::vector<CtPtr> out(X.size());
    const size_t cap = (size_t)std::max(1, max_group);
    for (auto& kv : groups) {
        const auto& idx = kv.second;
        for (size_t s0 = 0; s0 < idx.size(); s0 += cap) {
            std::vector<const CtData*> v;
            for (size_t t = s0; t < std::min(idx.size(), s0 + cap); ++t) v.push_back(X[idx[t]]);
            Grp x = g_gather(v, kv.first);
            Grp m1 = g_appmax(x, g_rotate(x, 1), d, k);
            Grp m2 = g_appmax(m1, g_rotate(m1, h), d, k);
            auto r = g_scatter(m2);
            for (size_t t = 0; t < r.size(); ++t) out[idx[s0 + t]] = r[t];
        }
    }
    return out;
}

std::vector<CtPtr> Ctx::sign_group(const std::vector<const CtData*>& X, int d, int k, int mode,
                                   const std::vector<const CtData*>& Y) {
    if (d < 1 || d > 7 || k < 0 || mode > 2 || (mode == 2 && (k < 1 || Y.size() != X.size())))
        throw HeError(HE_EINVAL);
    int nb = 0;
    while ((1 << nb) <= d) ++nb;
    int lvl = 1 << 30;
    for (auto* x : X) {
        if (x->deg != 1) throw HeError(HE_EMISMATCH);
        lvl = std::min(lvl, x->level);
    }
    for (auto* y : Y) {
        if (y->deg != 1) throw HeError(HE_EMISMATCH);
        lvl = std::min(lvl, y->level);
    }
    if (lvl < k * (nb + 1) + (mode ? 1 : 0)) throw HeError(HE_ELEVEL);
    SignJob J;
    J.X = X;
    J.Y = Y;
    J.lvl = lvl;
    J.d = d;
    J.k = k;
    J.mode = mode;
    while (!sign_step(J)) {
    }
    return J.result;
}

CtPtr Ctx::matmul(const CtData& A, const CtData& B, int h) {
    return matmul_batch({&A}, {&B}, {MatShape{h, h, 1}})[0];
}

// Members are grouped by (shape, level); each group runs in lockstep.  Group size is
// capped so the working set (about 12 ciphertext-sized blocks per member plus two
// lifted-digit blocks) stays well inside HBM.
std::vector<CtPtr> Ctx::matmul_batch(const std::vector<const CtData*>& A, const std::vector<const CtData*>& B,
                                     const std::vector<MatShape>& shapes) {
    const size_t n = A.size();
    std::vector<CtPtr> out(n);
    std::map<std::pair<MatShape, int>, std::vector<size_t>> groups;
    for (size_t i = 0; i < n; ++i) {
        check_shape(shapes[i]);
        if (A[i]->deg != 1 || B[i]->deg != 1) throw HeError(HE_EMISMATCH);
        const int lvl = std::min(A[i]->level, B[i]->level);
        if (lvl < 3) throw HeError(HE_ELEVEL);
        groups[{shapes[i], lvl}].push_back(i);
    }
    for (auto& kv : groups) prepare_shape(kv.first.first);
    const size_t cap = (size_t)std::max(1, max_group);
    struct Chunk {
        MatShape sh;
        int lvl;
        std::vector<size_t> idx;
    };
    std::vector<Chunk> chunks;
    for (auto& kv : groups) {
        const auto& idx = kv.second;
        for (size_t s = 0; s < idx.size(); s += cap)
            chunks.push_back({kv.first.first, kv.first.second,
                              std::vector<size_t>(idx.begin() + s, idx.begin() + std::min(idx.size(), s + cap))});
    }
    auto run = [&](const Chunk& ch, bool keep_acc, Grp* acc) {
        MatmulJob J;
        for (size_t i : ch.idx) {
            J.A.push_back(A[i]);
            J.B.push_back(B[i]);
        }
        J.h = ch.sh.h;
        J.t = ch.sh.t;
        J.beta = ch.sh.beta;
        J.lvl = ch.lvl;
        J.keep_acc = keep_acc;
        while (!matmul_step(J, ch.sh.h)) {
        }
        if (keep_acc) *acc = J.acc;
        else
            for (size_t t = 0; t < J.result.size(); ++t) out[ch.idx[t]] = J.result[t];
    };
    if (groups.size() < 2 || !concurrent_groups || !ensure_side()) {
        for (auto& ch : chunks) run(ch, false, nullptr);
        return out;
    }
    // The (shape, level) groups of a mixed batch share out the two streams so that the smaller
    // launches of different groups fill the device together.  The side stream starts after the work issued
    // so far, takes its buffers from its own allocation cache, and leaves each group's result
    // in that group's accumulator; after the join the context stream copies the results out
    // (into buffers of the main cache) and the side cache's free blocks return to the main one.
    struct Absorb {
        Ctx* c;
        ~Absorb() { c->pool.absorb(c->pool_side); }
    } absorb{this};
    std::vector<Grp> side_acc(chunks.size());
    struct SideGuard {  // error path: side work ends before its buffers go back
        Ctx* c;
        bool pending = false;
        ~SideGuard() {
            c->alloc_side = false;
            if (pending) (void)hipStreamSynchronize(c->side);
        }
    } guard{this};
    hip_check(hipEventRecord(ev_fork, stream), "fork side stream");
    hip_check(hipStreamWaitEvent(side, ev_fork, 0), "fork side stream");
    guard.pending = true;
    const hipStream_t main_stream = stream;
    // (shape, level) groups, largest first, each onto the less loaded stream; the chunks of one
    // group stay on one stream (one group's working set in flight at a time)
    auto work = [&](const Chunk& ch) {
        return (double)ch.idx.size() * ch.sh.t * ch.sh.h * (ch.lvl + 1 + n_p);
    };
    std::map<std::pair<MatShape, int>, double> gwork;
    for (auto& ch : chunks) gwork[{ch.sh, ch.lvl}] += work(ch);
    std::vector<std::pair<double, std::pair<MatShape, int>>> gorder;
    for (auto& kv : gwork) gorder.push_back({kv.second, kv.first});
    std::stable_sort(gorder.begin(), gorder.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    std::map<std::pair<MatShape, int>, int> gstream;
    double load[2] = {0, 0};
    for (auto& g : gorder) {
        const int sidx = load[1] < load[0] ? 1 : 0;  // the less loaded stream
        load[sidx] += g.first;
        gstream[g.second] = sidx;
    }
    std::vector<size_t> order(chunks.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
        return gwork[{chunks[x].sh, chunks[x].lvl}] > gwork[{chunks[y].sh, chunks[y].lvl}];
    });
    for (size_t i : order) {
        const int sidx = gstream[{chunks[i].sh, chunks[i].lvl}];
        if (sidx == 0) {
            run(chunks[i], false, nullptr);
            continue;
        }
        stream = side;
        alloc_side = true;
        try {
            run(chunks[i], true, &side_acc[i]);
        } catch (...) {
            stream = main_stream;
            alloc_side = false;
            throw;
        }
        stream = main_stream;
        alloc_side = false;
    }
    hip_check(hipEventRecord(ev_join, side), "join side stream");
    hip_check(hipStreamWaitEvent(stream, ev_join, 0), "join side stream");
    guard.pending = false;
    for (size_t i = 0; i < chunks.size(); ++i) {
        if (!side_acc[i].p) continue;
        auto r = g_scatter(side_acc[i]);
        for (size_t t = 0; t < r.size(); ++t) out[chunks[i].idx[t]] = r[t];
        side_acc[i] = Grp();
    }
    return out;
}

// App. C for every member (grouped by level): the transpose of each packed h x h matrix,
// one linear transform with BSGS, then RS
std::vector<CtPtr> Ctx::transpose_batch(const std::vector<const CtData*>& X, int h, int beta) {
    prepare_transpose(h, beta);
    std::map<int, std::vector<size_t>> groups;
    for (size_t i = 0; i < X.size(); ++i) {
        if (X[i]->deg != 1) throw HeError(HE_EMISMATCH);
        if (X[i]->level < 1) throw HeError(HE_ELEVEL);
        groups[X[i]->level].push_back(i);
    }
    std::vector<CtPtr> out(X.size());
    const size_t cap = (size_t)std::max(1, max_group);
    for (auto& kv : groups) {
        const auto& idx = kv.second;
        for (size_t s = 0; s < idx.size(); s += cap) {
            std::vector<const CtData*> v;
            for (size_t t = s; t < std::min(idx.size(), s + cap); ++t) v.push_back(X[idx[t]]);
            auto r = g_scatter(g_rescale(g_lintrans(g_gather(v, kv.first), 4, h, beta, h - 1, 1 - h, h - 1)));
            for (size_t t = 0; t < r.size(); ++t) out[idx[s + t]] = r[t];
        }
    }
    return out;
}
