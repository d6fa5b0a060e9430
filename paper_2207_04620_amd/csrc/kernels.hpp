// Kernel descriptors and launchers shared by the host runtime (he_host.hip)
// and the kernels (kernels.hip).
//
// Memory layout: a ciphertext of degree d at level l is one compact device block
// u64[d+1][l+1][N]; every limb is in the evaluation (NTT, bit-reversed) domain.
// An "extended" polynomial over Q_l and P has l+1+K limbs: Q limbs 0..l (prime
// index = limb index) followed by the K special primes (prime index n_q + k).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "modarith.hpp"

#define HE_MAXJ 192   // limbs in one job list
#define HE_MAXSRC 8   // source limbs of one base conversion (digit width / K)
#define HE_MAXT 64    // target limbs of one base conversion / ext limbs
#define HE_MAXDIG 8   // digits of one merged ModUp conversion (fused conversion only)

// A list of limbs: limb k of copy c lives at base + c * cstride + off[k] * N and is
// reduced modulo the prime with index mod[k].
struct Jobs {
    u64* base;
    int64_t cstride;
    int n;
    int nct;
    uint16_t off[HE_MAXJ];
    uint8_t mod[HE_MAXJ];
    // inverse transforms only: the first pass reads limb k of copy c from
    // src + c * src_cstride + off[k] * N instead of from base (the transform out of place)
    const u64* src = nullptr;
    int64_t src_cstride = 0;
};

// Several 2-D device copies in one launch: region r moves rows[r] rows of width[r] words
// (even) from src[r] (row pitch spitch[r]) to dst[r] (pitch dpitch[r]); every address and
// pitch is a multiple of two words (16-byte accesses)
#define CP_MAX 40
struct CopyDesc {
    int n = 0;
    const u64* src[CP_MAX];
    u64* dst[CP_MAX];
    int64_t width[CP_MAX], spitch[CP_MAX], dpitch[CP_MAX];
    int rows[CP_MAX];
    int64_t start[CP_MAX + 1];  // word pairs before region r
};

// limb i of an (extended) polynomial -> prime index
struct ModMap {
    int nq_l;  // limbs below this are Q limbs with prime index i
    int n_q;   // limbs at or above nq_l map to n_q + (i - nq_l)
    __device__ __forceinline__ int operator()(int i) const { return i < nq_l ? i : n_q + (i - nq_l); }
};

// Device-resident tables of one context.
#define ROW_TW 2047  // twiddle pairs per row of the 2048-point row pass

struct DevTables {
    const ModP* mods;    // [M]
    const u64* psi;      // [M][N]  psi^(bitrev k)
    const u64* psi_sh;   // [M][N]
    const u64* ipsi;     // [M][N]  psi^-(bitrev k)
    const u64* ipsi_sh;  // [M][N]
    // row-pass twiddle pairs (w, w') for N >= 2^11, [M][N1][ROW_TW][2], each row's in the order
    // its rounds consume them (forward: rtw, inverse: irtw)
    const u64* rtw;
    const u64* irtw;
    // the same twiddles as doubles (w, fl(w / q)) for the FP64 butterflies of primes below
    // 2^46 (zero for the others): row tables as above, column tables [M][N1]
    const double* rtwd;
    const double* irtwd;
    const double* cold;
    const double* icold;
    int log_n;
    int n1_log;  // column-pass stages
    int n2_log;  // row-pass stages
    u64 fp64_mods;  // bit m set: limbs of prime m run the FP64 butterflies (host-side count)
};

// The transforms of a limb use FP64 butterflies when its prime is below 2^46, the row pass
// holds 2048 elements and the column pass has at most five stages; both passes of a limb
// decide by this one rule.
#define FP64_QMAX (1ull << 46)
__host__ __device__ inline bool fp64_limb(u64 q, int L1, int N2) { return q < FP64_QMAX && N2 == 2048 && L1 <= 5; }

// Centered fast base conversion from ns source limbs to nt target limbs, for npoly
// polynomials.  Source limb s of poly p at src + p * src_pstride + s * N (coefficient
// form, prime smod[s]); target t of poly p at dst + p * dst_pstride + doff[t] * N.
// tab[(s * tab_ld + tcol[t]) * 2 + 0] = (D/q_s mod q_t) R mod q_t,
// tab[(s * tab_ld + tcol[t]) * 2 + 1] = (-q_s (D/q_s) mod q_t) R mod q_t.
struct ConvDesc {
    const u64* src;
    int64_t src_pstride;
    u64* dst;
    int64_t dst_pstride;
    int64_t src_cstride = 0, dst_cstride = 0;  // ciphertext strides
    int nct = 1;
    int prescaled = 0;  // sources multiplied by (D/q_s)^-1 and centred by the inverse NTT (conv_cols)
    const u64* tab;
    int tab_ld;  // table row length: entry (s, col) at tab[(s * tab_ld + col) * 2]
    int ns, nt, npoly;
    int smod[HE_MAXSRC];
    u64 hinv[HE_MAXSRC], hinv_sh[HE_MAXSRC];
    uint16_t doff[HE_MAXT];
    uint16_t tcol[HE_MAXT];  // table column of target t
    uint8_t dmod[HE_MAXT];
    // The digits of one ModUp in one fused launch (ndig > 0): target t belongs to digit tdig[t],
    // whose ns_d = dns[d] sources start dsrc[d] words after src and whose table starts dtab[d]
    // words after tab; ns is the largest ns_d.  ndig = 0: one digit, no offsets.
    int ndig;
    int dns[HE_MAXDIG];
    int64_t dsrc[HE_MAXDIG];
    int64_t dtab[HE_MAXDIG];
    uint8_t tdig[HE_MAXT];
};

struct SampleArgs {
    u64 seed;
    uint32_t purpose;
    u64 index;
    int kind;          // 0 ternary, 1 Gaussian, 2 uniform mod the limb's prime
    u64 uidx[HE_MAXJ]; // uniform: stream index of limb k
    u64 cdt[19];
};

// Key switch inner product: for ext limb t (prime mod[t]) and coefficient i,
//  u0[t][i] = sum_j lift[j][t][perm_g(i)] kb[j][mod[t]][i], u1 likewise with ka.
// One rotation set of a key-switch inner product: a rotation (g, key), or with nrot = 2 the
// masked sum mask . IP(g, key) + mask2 . IP(g2, key2) of two rotations of the same lift (one
// ModDown then serves both).  ginv = g^-1 mod 2N numbers the set's blocks by lift region.
struct IpSet {
    const u64* key;    // [beta_top][2][M][N] Montgomery form
    const u64* key2;
    const u64* mask;   // [M][N] Montgomery form, row = modulus index; null = no mask
    const u64* mask2;
    u64 g, g2, ginv;   // Galois elements (1 = identity)
    // optional: the second rotation is of another ciphertext (a term of a rotation sum): its
    // lift and c0 (same level and strides as the descriptor's lift, c0 stride c0_2_cs)
    const u64* lift2;
    const u64* c0_2;
    int64_t c0_2_cs;
    const u64* own2;  // where lift2's own digit limbs are read (see IpDesc::own)
    int64_t own2_cs;
};
#define IP_MAXSET 16

struct IpDesc {
    const u64* lift;  // [nct][beta][ne][N] (ciphertext stride lift_cs)
    u64* u;           // [nset][nct][2][ne][N] (ciphertext stride u_cs)
    int64_t lift_cs, u_cs;
    int nct;
    int ne, beta, M;
    uint8_t mod[HE_MAXT];
    // optional: u0[t] += P * c0[t][perm_g(i)] on the Q limbs t < nq (c0 of the rotated
    // ciphertext; ModDown then yields (u0 - conv) P^-1 + sigma_g(c0) exactly)
    const u64* c0;
    int64_t c0_cs;
    int nq;
    u64 pmont[HE_MAXT];  // (P mod q_t) R mod q_t
    // optional: each digit's own limbs [dlo[j], dhi[j]) are not in the lift but read from the
    // lifted polynomial itself (evaluation form): limb t of member c at own + c * own_cs + t N
    const u64* own;
    int64_t own_cs;
    uint8_t dlo[HE_MAXSRC], dhi[HE_MAXSRC];
    int nrot;            // rotations per set (1 or 2)
    int nset;            // sets of the same lift in this launch (at most IP_MAXSET)
    IpSet s[IP_MAXSET];
    int accumulate;    // u += the result (a sum of rotations of different ciphertexts)
};

// n-ary sum of ciphertext polynomials (up to 16 inputs per launch), each input with its own
// poly stride (inputs above the output level contribute their limb prefix)
struct SumDesc {
    const u64* in[16];
    int64_t in_ps[16];
    int n;
};
void launch_sum_many(const DevTables& T, int nl, int npoly, const SumDesc& D, u64* out, int64_t out_ps,
                     int accumulate, hipStream_t st);

// several diagonal sums over the same inputs (the giant steps of one BSGS linear transform):
// out[g] = sum_j mask[g][j] . in[j]; a null mask is an absent term
#define MM_OUT 4
struct MultiMacDesc {
    const u64* in[16];
    int64_t in_ps[16], in_cs[16];
    const u64* mask[MM_OUT][16];  // Montgomery form, rows = limbs
    u64* out[MM_OUT];
    int64_t out_ps, out_cs;
    int nin, nout, nct;
};
void launch_mask_mac_multi(const DevTables& T, int nl, int npoly, const MultiMacDesc& D, hipStream_t st);

// sum_j A_j (x) B_j of up to 16 pairs of degree-1 groups into a degree-2 group (+= with acc)
struct TensorSumDesc {
    const u64* a[16];
    const u64* b[16];
    int64_t a_ps[16], a_cs[16], b_ps[16], b_cs[16];
    u64* d;
    int64_t d_ps, d_cs;
    int n, nct, acc;
};
void launch_tensor_sum(const DevTables& T, int nl, const TensorSumDesc& D, hipStream_t st);

struct MacDesc {
    const u64* in[16];
    const u64* mask[16];
    int64_t in_ps[16];
    int64_t in_cs[16];
    int nterm;
    int nct;
};

enum EwOp { EW_ADD = 0, EW_SUB = 1, EW_MUL_MONT = 2, EW_MUL_PLAIN = 3 };

// ModDown epilogue fused into a forward NTT over the converted P-part: for job k of
// ciphertext c (limb t = k % nl of poly p = k / nl) the transformed value v is not
// stored; instead out_p[c][t][i] = (u[c][p][t][i] - v) * P^-1 + add_p[c][t][perm_g(i)]
// (add_p may be null; g = 1 is the identity gather).
struct Epi {
    int on;
    int nl;
    const u64* u;
    int64_t u_cs, u_ps;
    const u64* add[2];
    u64* out[2];
    int64_t add_cs, out_cs;
    const u64* pinv;
    const u64* pinv_sh;
    u64 g;
    // optional Mul_pt fused into the epilogue: out = w * mask (Montgomery form, rows = limbs)
    // (+ acc_p[c][t][i] when acc_p is set): one term of a diagonal sum (Eq. 1)
    const u64* mask;
    const u64* acc[2];
    int64_t acc_cs;
};

// ------------------------------------------------------------------ launch timing
enum ProfKind {
    PK_NTT_FWD_COLS = 0, PK_NTT_FWD_ROWS, PK_NTT_INV_ROWS, PK_NTT_INV_COLS, PK_BASECONV, PK_INNER, PK_MODDOWN,
    PK_RS_SPREAD, PK_RS_COMBINE, PK_TENSOR, PK_MASKMAC, PK_AUTOMORPH, PK_EW, PK_CONV_COLS, PK_COPY, PK_COUNT
};
#include <string>
// Launch discipline: every kernel launch goes through HE_LAUNCH.  launch_gate() clears the
// thread's last HIP error and, while a host-side failure injection is armed
// (launch_inject), fails the launch before anything is queued, so tests of the error paths
// never run a faulty kernel.  launch_check() reads the launch status at once, so a launch
// that fails is reported by the call that issued it, not at a later synchronisation.  Both
// throw LaunchError, which every C-ABI entry point returns as HE_EDEVICE.
struct LaunchError {
    hipError_t e;
    const char* what;
};
void launch_gate(const char* what);
void launch_check(const char* what);
// fail the n-th launch from now on in this process (n >= 1); n = 0 disarms
void launch_inject(uint64_t n);
#define HE_LAUNCH(kernel, ...)                     \
    do {                                           \
        launch_gate(#kernel);                      \
        hipLaunchKernelGGL(kernel, __VA_ARGS__);   \
        launch_check(#kernel);                     \
    } while (0)

// only: null for every kernel kind, else one kind's name; false for an unknown name
bool prof_enable(bool on, const char* only);
bool prof_active();
std::string prof_report();  // JSON: per kernel kind {launches, ms, bytes}; clears the records

// ------------------------------------------------------------------ launchers
// inverse: the last pass multiplies limb job k by scale[k mod scale_n] (a (c, c') Shoup pair)
// instead of N^-1 when scale is set, and stores centred two's-complement words; forward: cols = false skips the column pass (done by
// launch_conv_cols)
void launch_ntt(const DevTables& T, const Jobs& J, bool inverse, hipStream_t st, const u64* scale = nullptr,
                int scale_n = 0, bool cols = true);
void launch_ntt_moddown(const DevTables& T, const Jobs& J, const Epi& E, hipStream_t st, bool cols = true);
void launch_baseconv(const DevTables& T, const ConvDesc& D, hipStream_t st);
// base conversion of prescaled sources fused with the forward column pass of every target
// (N > 2^11); the row pass is then run with launch_ntt(..., cols = false)
bool conv_cols_fits(const DevTables& T, int ns);
void launch_conv_cols(const DevTables& T, const ConvDesc& D, hipStream_t st);
void launch_sample(const DevTables& T, const Jobs& J, const SampleArgs& A, hipStream_t st);
// the regions of D (start[] is filled here)
void launch_copy(CopyDesc& D, hipStream_t st);
// out[p][i] = a[p][i] (op) b[p][i] over nl limbs (prime map mm) and npoly polys;
// b_ps = 0 broadcasts one b polynomial to every poly
void launch_ew(const DevTables& T, ModMap mm, int nl, int npoly, u64* out, int64_t out_ps, const u64* a,
               int64_t a_ps, const u64* b, int64_t b_ps, int op, hipStream_t st, int nct = 1, int64_t out_cs = 0,
               int64_t a_cs = 0, int64_t b_cs = 0);
// out[p][i] = a[p][i] * c_i (Shoup constants in device arrays c, c_sh indexed by limb)
void launch_mul_const(const DevTables& T, ModMap mm, int nl, int npoly, u64* out, int64_t out_ps, const u64* a,
                      int64_t a_ps, const u64* c, const u64* c_sh, hipStream_t st);
// evaluation-domain automorphism: out[p][i][j] = in[p][i][perm_g(j)]
void launch_automorph(const DevTables& T, int nl, int npoly, u64* out, int64_t out_ps, const u64* in,
                      int64_t in_ps, u64 g, hipStream_t st, int nct = 1, int64_t out_cs = 0, int64_t in_cs = 0);
void launch_to_mont(const DevTables& T, ModMap mm, int nl, int npoly, u64* x, int64_t ps, hipStream_t st);
// b = e - a s (+ pmod_i s' on flagged limbs), all limbs of the full chain [M][N]
void launch_swk_finish(const DevTables& T, int M, u64* b, const u64* a, const u64* e, const u64* s,
                       const u64* sp, const u64* pmod, const uint8_t* in_digit, hipStream_t st);
void launch_inner_product(const DevTables& T, const IpDesc& D, hipStream_t st);
// out[p][t] = (u[p][t] - conv[p][t]) * Pinv_t (+ add[p][t])
void launch_moddown_combine(const DevTables& T, int nl, int npoly, const u64* u, int64_t u_ps, const u64* conv,
                            int64_t conv_ps, const u64* pinv, const u64* pinv_sh, const u64* add, int64_t add_ps,
                            u64* out, int64_t out_ps, hipStream_t st, int nct = 1, int64_t u_cs = 0,
                            int64_t conv_cs = 0, int64_t add_cs = 0, int64_t out_cs = 0);
// tmp[p][i] = centered(last[p]) mod q_i (coefficient form)
void launch_rescale_spread(const DevTables& T, int nl_out, int npoly, const u64* last, int64_t last_ps,
                           int last_mod, u64* tmp, int64_t tmp_ps, hipStream_t st);
// out[p][i] = (c[p][i] - tmp[p][i]) * qinv_i
void launch_rescale_combine(const DevTables& T, int nl_out, int npoly, const u64* c, int64_t c_ps, const u64* tmp,
                            int64_t tmp_ps, const u64* qinv, const u64* qinv_sh, u64* out, int64_t out_ps,
                            hipStream_t st, int nct = 1, int64_t c_cs = 0, int64_t tmp_cs = 0, int64_t out_cs = 0);
// d0 (+)= a0 b0, d1 (+)= a0 b1 + a1 b0, d2 (+)= a1 b1
void launch_tensor(const DevTables& T, int nl, const u64* a, int64_t a_ps, const u64* b, int64_t b_ps, u64* d,
                   int64_t d_ps, int acc, hipStream_t st, int nct = 1, int64_t a_cs = 0, int64_t b_cs = 0,
                   int64_t d_cs = 0);
// out[p][i] (+)= sum_r in_r[p][i] mask_r[i]  (masks in Montgomery form, compact [nl_top][N])
void launch_mask_mac(const DevTables& T, int nl, int npoly, const MacDesc& D, u64* out, int64_t out_ps, int acc,
                     hipStream_t st, int64_t out_cs = 0);
// m = c0 + c1 s (+ c2 s^2); s, s2 plain evaluation form [M][N]
void launch_dec_dot(const DevTables& T, int nl, int deg, const u64* c, int64_t c_ps, const u64* s, const u64* s2,
                    u64* m, hipStream_t st);
// c0 = v pk0 + x0, c1 = v pk1 + x1 (pk in Montgomery form)
void launch_enc_combine(const DevTables& T, int nl, const u64* v, const u64* pk0, const u64* pk1, const u64* x0,
                        const u64* x1, u64* c0, u64* c1, hipStream_t st);
// x[i][j] += m[j] mod q_i (signed 64-bit message)
void launch_add_signed(const DevTables& T, int nl, u64* x, const int64_t* m, hipStream_t st);
