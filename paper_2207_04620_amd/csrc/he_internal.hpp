// Internal types of the libhe runtime.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <mutex>
#include <set>
#include <tuple>
#include <memory>
#include <unordered_map>
#include <vector>

#include "../../include/he.h"
#include "host_math.hpp"
#include "kernels.hpp"

struct HeError {
    he_status s;
    explicit HeError(he_status v) : s(v) {}
};
void hip_check(hipError_t e, const char* what);

// ChaCha20 stream purposes
enum { P_SK = 1, P_PK_A = 2, P_PK_E = 3, P_SWK_A = 4, P_SWK_E = 5, P_ENC_V = 6, P_ENC_E0 = 7, P_ENC_E1 = 8 };
// op counters
enum { C_ROT = 0, C_KS = 1, C_MULPT = 2, C_MULCT = 3, C_ADD = 4, C_RS = 5 };

// Size-bucketed cache over hipMalloc; all work is ordered on one stream, so a block
// released here may be handed out again at once.  Thread-safe (the serving thread and
// the caller release buffers concurrently).
// Blocks of a captured HIP graph: every block handed out or released while a stream capture
// records into the graph belongs to it (the graph's kernels and copies keep reading and writing
// those addresses on every replay), and its blocks are reused only within that capture.
struct GraphBlocks {
    std::unordered_map<void*, size_t> owned;
    std::unordered_map<size_t, std::vector<void*>> free_;
};

struct Pool {
    std::mutex m;
    std::unordered_map<size_t, std::vector<void*>> free_;
    GraphBlocks* capture = nullptr;  // set while a graph is being captured
    size_t held = 0, cached = 0;  // device bytes held (in use + cached), of them cached
    size_t limit = 0;             // cap on held bytes (0: none); beyond it alloc is HE_ENOMEM
    size_t peak = 0;              // largest in-use byte count (held - cached) since the last reset
    Pool* sibling = nullptr;  // the context's other cache: its free blocks go back too when memory runs out
    void* (*dev_alloc)(size_t, void*) = nullptr;
    void (*dev_free)(void*, void*) = nullptr;
    void* user = nullptr;
    void* alloc(size_t bytes);
    void* alloc_locked(size_t bytes);
    void release(void* p, size_t bytes);
    void trim();
    void trim_locked();
    // take over o's cached (free) blocks; only when none of o's work can still be pending
    void absorb(Pool& o);
    // bytes in use now; restart the peak figure from it
    size_t restart_peak() {
        std::lock_guard<std::mutex> lk(m);
        peak = held - cached;
        return peak;
    }
    // (bytes in use now, peak since the last restart)
    std::pair<size_t, size_t> usage() {
        std::lock_guard<std::mutex> lk(m);
        return {held - cached, peak};
    }
};

struct Ctx;
struct DBuf {
    Ctx* ctx;
    Pool* pool;  // the allocation cache it came from and goes back to
    u64* p = nullptr;
    size_t n;
    DBuf(Ctx* c, size_t n_u64);
    ~DBuf();
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
};

struct CtData {
    int level = 0, deg = 1;
    double scale = 1.0;
    std::unique_ptr<DBuf> buf;  // u64[deg+1][level+1][N], evaluation form
};
typedef std::shared_ptr<CtData> CtPtr;

// B ciphertexts of one level and degree in one block [B][deg+1][level+1][N]
struct Grp {
    int B = 0, level = 0, deg = 1;
    std::vector<double> scale;
    std::shared_ptr<DBuf> buf;
    u64* p = nullptr;
    int64_t ps = 0, cs = 0;  // poly and ciphertext strides (elements)
};

// a sum of rotations of different ciphertexts being accumulated in the extended basis
// before its single ModDown (key-switch inner products + P sigma_g(c0) per term)
struct RotSum {
    std::shared_ptr<DBuf> u;
    int B = 0, level = -1, n = 0;
    bool filled = false;  // u holds at least one term
    std::vector<double> scale;
    // a term waiting for a partner: two terms share one inner-product launch, so u is read
    // and rewritten once per pair (its lift, its ciphertext for c0, its Galois element)
    std::shared_ptr<DBuf> plift;
    Grp pa;
    u64 pg = 0;
};

// resumable state of one lockstep product group
struct MatmulJob {
    std::vector<const CtData*> A, B;
    int h = 0, t = 0, beta = 1, lvl = 0, phase = 0, k = 0;  // t: Step-2/3 rounds (h, or t < h)
    Grp A0, B0, acc, S;   // S: the current Step-3 block sum
    bool have = false, haveS = false;
    std::vector<Grp> babyB;  // Rot(B0, h j), j < bg, kept across blocks (Step-3 split)
    RotSum giant;            // Step-3 giant-step rotations sharing one ModDown (ModDown hoisting)
    std::vector<Grp> pendA, pendB;  // Step-3 pairs awaiting one block tensor-sum (relin-once)
    std::shared_ptr<DBuf> liftA, liftB;
    std::vector<CtPtr> result;
    bool keep_acc = false;  // leave the result as the group acc (the caller scatters it)
};
// resumable state of one lockstep sign/ReLU group
// mode 0: g_d^(k)(x); mode 1: ReLU (x + x g) / 2; mode 2: AppMax(a, b) (Alg. 5) with
// a = X, b = Y: ((a + b) + m g_d^(k)(m)) / 2, m = a - b; mode 3: the power x^k (k = 2: one
// Mul_ct and RS, depth 1; k = 3: x . x^2, depth 2), the served requests of depth 1 and 2
struct SignJob {
    std::vector<const CtData*> X, Y;
    int lvl = 0, d = 3, k = 1, mode = 0, it = 0;
    bool started = false;
    bool pre = false, keep = false;  // inputs given as groups (ga, gb); result kept as a group
    Grp ga, gb, out;
    Grp x, s, cur;
    std::vector<CtPtr> result;
};

struct ModUpInfo {
    int lo = 0, hi = 0;
    size_t off = 0;  // into the ModUp table
    u64 hinv[HE_MAXSRC] = {0}, hinv_sh[HE_MAXSRC] = {0};
};

// a diagonal mask: kind (Alg. 3 / App. C diagonal family), side h, packing beta (App. E),
// diagonal index k, pre-rotation rot (positions of the h^2 vector)
struct MaskKey {
    int kind, h, beta, k;
    int64_t rot;
    bool operator<(const MaskKey& o) const {
        return std::tie(kind, h, beta, k, rot) < std::tie(o.kind, o.h, o.beta, o.k, o.rot);
    }
    bool operator==(const MaskKey& o) const {
        return kind == o.kind && h == o.h && beta == o.beta && k == o.k && rot == o.rot;
    }
};

// shape of a packed product: h x h (t = h, Alg. 3) or t x h by h x h (t < h, HE-RMatMult,
// App. D), beta matrix pairs per ciphertext pair (iota_beta, App. E)
struct MatShape {
    int h = 0, t = 0, beta = 1;
    bool operator<(const MatShape& o) const { return std::tie(h, t, beta) < std::tie(o.h, o.t, o.beta); }
};

// one Step-2 term: v1 . Rot(a, k1) + v2 . Rot(a, k2)
struct MaskPair {
    int64_t k1;
    const u64* m1;
    int64_t k2;
    const u64* m2;
};

struct Ctx {
    int log_n = 0;
    int64_t N = 0;
    int n_q = 0, n_p = 0, alpha = 1;
    double scale = 1.0;
    u64 seed = 0;
    uint32_t schedule = 0;
    int device = 0;            // the HIP device current at creation
    u64* scratch = nullptr;    // that device's copy of the allocation-free entry point's scratch
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // second stream of the context: the next Step-2 pair group's key-switch inner products
    // run there while the current group's ModDown runs on the context stream (fork and join by
    // the two events; every buffer it touches is allocated after the fork and released only
    // after the join, so the allocation cache stays ordered by the context stream)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // the side stream (default priority) and its events, made on first use: a context that
    // never overlaps work holds no second stream (hardware queues are few per process)
    bool ensure_side() {
        if (side) return true;
        hipStream_t s2 = nullptr;
        hipEvent_t e1 = nullptr, e2 = nullptr;
        if (hipStreamCreateWithFlags(&s2, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&e1, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&e2, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            if (s2) (void)hipStreamDestroy(s2);
            if (e1) (void)hipEventDestroy(e1);
            if (e2) (void)hipEventDestroy(e2);
            return false;  // the work then runs on the context stream alone
        }
        side = s2;
        ev_fork = e1;
        ev_join = e2;
        return true;
    }
    ~Ctx() {
        if (side) (void)hipStreamSynchronize(side);
        if (side) (void)hipStreamDestroy(side);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
    }
    Pool pool;
    // the side stream's own allocation cache: lockstep groups issued on the side stream take
    // their buffers from it (alloc_side set), so a block never passes between the streams while
    // either may still use it; its free blocks return to the main cache after the streams join
    Pool pool_side;
    bool alloc_side = false;
    hm::Encoder enc;
    std::vector<u64> mods, roots, pmod;
    std::vector<ModP> host_mods;
    DevTables T{};
    u64 cdt[19];
    // device tables
    std::unique_ptr<DBuf> d_mods, d_psi, d_psi_sh, d_ipsi, d_ipsi_sh, d_rtw, d_irtw, d_rtwd, d_irtwd, d_cold, d_icold, d_rs, d_md_tab,
        d_pinv, d_mu_tab, d_mu_scale, d_md_scale;
    std::vector<u64> md_hinv, md_hinv_sh;
    std::vector<std::vector<ModUpInfo>> mu;  // [level][digit]
    // keys
    std::unique_ptr<DBuf> s_eval, s2_eval, pk, rlk;
    std::map<u64, std::unique_ptr<DBuf>> rot_keys;
    std::map<MaskKey, std::unique_ptr<DBuf>> masks;
    size_t keys_bytes = 0;
    std::set<MatShape> prepared;                // shapes whose rotation keys and masks exist
    std::set<std::pair<int, int>> prepared_tr;  // (h, beta) of transposes
    std::atomic<uint32_t> prepared_mask{0};  // bit log2(h) set once keys and masks for h exist
    int64_t cnt[6] = {0, 0, 0, 0, 0, 0};

    int ext_mod(int level, int i) const;
    void build_tables();
    void ntt(u64* base, int npoly, int64_t pstride_limbs, int nl, bool inverse, int level_for_ext);
    void sample_into(u64* dst, int count, const int* modidx, int kind, uint32_t purpose, u64 index, const u64* uidx);
    void keygen_base();
    std::unique_ptr<DBuf> make_swk(u64 key_id, const u64* sp);
    const u64* relin_key();
    u64 galois(int64_t k) const;
    const u64* rot_key(u64 g, bool create);

    CtPtr new_ct(int level, int deg, double scale);
    CtPtr encrypt_coeffs(const int64_t* m, int level, double scale, u64 nonce);
    void decrypt_coeffs(const CtData& c, double* out);
    CtPtr drop(const CtData& a, int level);
    CtPtr add_sub(const CtData& a, const CtData& b, bool sub);
    CtPtr tensor(const CtData& a, const CtData& b);
    std::unique_ptr<DBuf> ks_lift(const u64* d, int level);
    void ks_lift_into(const u64* d, int level, u64* lift, u64* coef);
    void ks_apply_into(const u64* lift, int level, const u64* key, u64 g, const u64* add0, const u64* add1,
                       u64* out0, u64* out1, u64* u, u64* conv);
    void ks_apply(const u64* lift, int level, const u64* key, u64 g, const u64* add0, const u64* add1, u64* out0,
                  u64* out1);
    CtPtr relin(const CtData& a);
    CtPtr rescale(const CtData& a);
    CtPtr rotate_from_lift(const CtData& a, const u64* lift, int64_t k);
    CtPtr rotate(const CtData& a, int64_t k);
    CtPtr mul_int(const CtData& a, int64_t k);
    std::unique_ptr<DBuf> plaintext_mont(const int64_t* coeffs);
    CtPtr mask_sum(const std::vector<std::pair<const CtData*, const u64*>>& terms, double mask_scale);

    const u64* mask(int kind, int h, int k, int64_t rot, int beta = 1);
    void prepare_masks(const std::vector<MaskKey>& keys);
    int bsgs(int h) const;
    int step3_baby(int h) const;
    std::vector<MaskKey> matmul_masks(const MatShape& s) const;
    std::vector<int64_t> matmul_rotations(const MatShape& s) const;
    std::vector<MaskKey> transpose_masks(int h, int beta) const;
    std::vector<int64_t> transpose_rotations(int h, int beta) const;
    void check_shape(const MatShape& s) const;
    void prepare_shape(const MatShape& s);
    void prepare_h(int h) { prepare_shape(MatShape{h, h, 1}); }
    void prepare_transpose(int h, int beta);
    CtPtr matmul(const CtData& A, const CtData& B, int h);
    std::vector<CtPtr> matmul_batch(const std::vector<const CtData*>& A, const std::vector<const CtData*>& B,
                                    const std::vector<MatShape>& shapes);
    std::vector<CtPtr> transpose_batch(const std::vector<const CtData*>& X, int h, int beta);
    int max_group = 32;
    int pair_batch = 4;  // Step-2 mask pairs per shared ModDown launch
    int overlap = 0;     // Step-2 pair groups pipelined over the two streams (measured slower: off)
    int concurrent_groups = 1;  // lockstep groups of a mixed batch spread over the two streams
    // a group lift holds only the converted limbs of each digit; its own limbs are read from the
    // lifted polynomial: lift buffer -> (that polynomial of member 0, member stride)
    std::unordered_map<const u64*, std::pair<const u64*, int64_t>> lift_own;

    // lockstep group operations (group.hip)
    Grp g_new(int B, int level, int deg, const std::vector<double>& sc);
    Grp g_gather(const std::vector<const CtData*>& v, int level);
    std::vector<CtPtr> g_scatter(const Grp& g);
    Grp g_drop(const Grp& a, int level);
    void g_add_into(Grp& acc, const Grp& t);
    std::shared_ptr<DBuf> g_lift(const Grp& a, int poly);
    void g_ks_inner(u64* u, const u64* lift, int B, int level, const u64* key, u64 g, const u64* c0, int64_t c0_cs,
                    const u64* mask, const u64* key2, u64 g2, const u64* mask2, bool accumulate);
    void g_ks_inner_sets(u64* u, const u64* lift, int B, int level, std::vector<IpSet> sets, int nrot,
                         const u64* c0, int64_t c0_cs, bool accumulate);
    void g_rotsum_add(RotSum& S, const Grp& a, int64_t r);
    Grp g_rotsum_finish(RotSum& S, const Grp* base);
    void g_moddown(u64* u, int B, int level, const u64* add0, const u64* add1, int64_t add_cs, u64* out0,
                   u64* out1, int64_t out_cs, u64 add_g, const u64* mask, const u64* acc0, const u64* acc1,
                   int64_t acc_cs);
    std::vector<Grp> g_rotate_sets_hoisted(const Grp& a, const u64* lift, const std::vector<IpSet>& sets, int nrot,
                                           double mask_scale);
    // the two halves of g_rotate_sets_hoisted: the inner products of every set (on the stream
    // current in the context), then the shared ModDown
    struct PendingSets {
        Grp out;
        std::shared_ptr<DBuf> u;
        std::vector<double> sc;
        int P = 0, B = 0, level = 0;
    };
    PendingSets g_sets_ip(const Grp& a, const u64* lift, const std::vector<IpSet>& sets, int nrot, double mask_scale);
    std::vector<Grp> g_sets_finish(PendingSets& ps);
    PendingSets g_pairs_ip(const Grp& a, const u64* lift, const std::vector<MaskPair>& pr, double mask_scale);
    std::vector<Grp> g_rotate_many_hoisted(const Grp& a, const u64* lift, const std::vector<int64_t>& ks);
    std::vector<Grp> g_rotate_pairs_hoisted(const Grp& a, const u64* lift, const std::vector<MaskPair>& pr,
                                            double mask_scale);
    void g_ks_apply(const u64* lift, int B, int level, const u64* key, u64 g, const u64* add0, const u64* add1,
                    int64_t add_cs, u64* out0, u64* out1, int64_t out_cs, u64 add_g, const u64* mask,
                    const u64* acc0, const u64* acc1, int64_t acc_cs, const u64* c0, int64_t c0_cs);
    Grp g_rotate_mask_from_lift(const Grp& a, const u64* lift, int64_t k, const u64* mask, double mask_scale,
                                const Grp* acc);
    Grp g_rotate_from_lift(const Grp& a, const u64* lift, int64_t k);
    Grp g_rotate(const Grp& a, int64_t k);
    Grp g_mask_sum(const std::vector<std::pair<const Grp*, const u64*>>& terms, double mask_scale);
    Grp g_rescale(const Grp& a);
    Grp g_tensor(const Grp& a, const Grp& b);
    void g_tensor_acc(Grp& acc, const Grp& a, const Grp& b);
    void g_tensor_sum(MatmulJob& J);
    Grp g_relin(const Grp& a);
    Grp g_lintrans(const Grp& a, int kind, int h, int beta, int64_t unit, int dlo, int dhi);
    std::vector<CtPtr> matmul_group(const std::vector<const CtData*>& A, const std::vector<const CtData*>& B,
                                    const MatShape& s, int lvl);
    bool matmul_step(MatmulJob& J, int k_chunk);
    Grp g_mul_int(const Grp& a, const std::vector<int64_t>& k);
    Grp g_mul_rs(const Grp& x, const Grp& y);
    Grp g_eval_gd(const Grp& x, int d, const std::vector<double>& target);
    bool sign_step(SignJob& J);
    std::vector<CtPtr> sign_group(const std::vector<const CtData*>& X, int d, int k, int mode,
                                  const std::vector<const CtData*>& Y = {});
    Grp g_ew(const Grp& a, const Grp& b, int op);
    Grp g_appmax(const Grp& a, const Grp& b, int d, int k);
    std::vector<CtPtr> maxpool_batch(const std::vector<const CtData*>& X, int h, int d, int k);
    CtPtr fl_update(const CtData& w, const std::vector<const CtData*>& grads, double coeff);

    std::recursive_mutex api_mu;  // every C-ABI call on the context (and the serving thread) holds it

    void release_all() {
        masks.clear();
        rot_keys.clear();
        rlk.reset();
        pk.reset();
        s2_eval.reset();
        s_eval.reset();
        d_mods.reset(); d_psi.reset(); d_psi_sh.reset(); d_ipsi.reset(); d_ipsi_sh.reset();
        d_rtw.reset(); d_irtw.reset(); d_rtwd.reset(); d_irtwd.reset(); d_cold.reset(); d_icold.reset();
        d_mu_scale.reset(); d_md_scale.reset();
        d_rs.reset(); d_md_tab.reset(); d_pinv.reset(); d_mu_tab.reset();
        pool.trim();
        pool_side.trim();
    }
};

// C-ABI handles
struct he_ct {
    Ctx* ctx;
    CtPtr c;
};
struct he_ctx {
    std::unique_ptr<Ctx> c;
};
he_ct* wrap(Ctx* c, CtPtr p);

// runs f under the context's API lock, turning exceptions into status codes
template <class F>
inline he_status run_guarded(he_ctx* ctx, F&& f) {
    std::lock_guard<std::recursive_mutex> lk(ctx->c->api_mu);
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
