/*
 * ckks_oracle.h -- CPU oracle for the Hercules packed ciphertext matrix product.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously-correct scalar
 * implementation of single-key RNS-CKKS (the operations of the paper's Fig. 1
 * that run without other parties), the diagonal linear transform (Eq. 1,
 * Alg. 2), the packed matrix product HE-MatMult (Alg. 3 with the baby-step /
 * giant-step split of App. B) and the composite sign approximation g_d^(k)
 * (Sec. 4.2, Alg. 5).  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code with the GPU library.
 *
 * Conventions (readings where the paper is silent):
 *  - ring Z_Q[X]/(X^N+1), Q = q_0 ... q_L, special modulus P = p_0 ... p_{K-1};
 *  - primes: for each requested bit size, in list order (Q list, then P list),
 *    the largest unused prime p < 2^bits with p = 1 mod 2N;
 *  - slot j of a plaintext is its evaluation at zeta^(5^j), zeta = exp(i pi/N);
 *  - Rot(c,k) is the LEFT rotation R(m,k)[t] = m[t+k] (Sec. 3.2 definition);
 *  - hybrid key switching with digits of alpha Q-limbs, centered fast base
 *    conversion for ModUp and ModDown;
 *  - randomness: ChaCha20 (RFC 8439) keyed by the 64-bit seed, nonce =
 *    (purpose, index), counter = block number.
 * Ciphertexts are kept in the coefficient domain.
 */
#ifndef CKKS_ORACLE_H
#define CKKS_ORACLE_H
#include <stdint.h>

typedef struct orc_ctx orc_ctx;
typedef struct orc_ct orc_ct;

orc_ctx *orc_create(int log_n, int n_q, const int *q_bits, int n_p, const int *p_bits,
                    int alpha, double log_scale, uint64_t seed, int n_threads);
void orc_destroy(orc_ctx *c);
int orc_n_moduli(const orc_ctx *c);
void orc_moduli(const orc_ctx *c, uint64_t *out);      /* Q primes then P primes */
uint64_t orc_psi(const orc_ctx *c, int mod_idx);      /* chosen primitive 2N-th root */

/* ---- primitives exposed for pins ---- */
uint64_t orc_mulmod(uint64_t a, uint64_t b, uint64_t q);
int orc_is_prime(uint64_t n);
void orc_chacha20_block(const uint32_t key[8], uint32_t counter, const uint32_t nonce[3],
                        uint32_t out[16]);
uint64_t orc_word(uint64_t seed, uint32_t purpose, uint64_t index, uint64_t w);
void orc_gauss_table(uint64_t out[19]);
void orc_sample_ternary(uint64_t seed, uint32_t purpose, uint64_t index, int64_t n, int64_t *out);
void orc_sample_gauss(uint64_t seed, uint32_t purpose, uint64_t index, int64_t n, int64_t *out);
void orc_sample_uniform(uint64_t seed, uint32_t purpose, uint64_t index, uint64_t q, int64_t n,
                        uint64_t *out);
/* negacyclic product of a,b mod moduli[mod_idx] via the oracle's NTT */
void orc_poly_mul(const orc_ctx *c, int mod_idx, const uint64_t *a, const uint64_t *b,
                  uint64_t *out);
/* a(psi^(2*bitrev(j)+1)) for j in [0,N): the evaluation order a GPU NTT produces */
void orc_eval_bitrev(const orc_ctx *c, int mod_idx, const uint64_t *a, uint64_t *out);
/* centered fast base conversion of x (given mod src moduli) into dst modulus */
void orc_base_conv(const orc_ctx *c, int n_src, const int *src_idx, int dst_idx,
                   const uint64_t *x /* [n_src][N] */, uint64_t *out /* [N] */);

/* ---- encoding (Fig. 1 Ecd / Dcd) ---- */
/* encode n_slots (<= N/2) real values, replicated to fill N/2 slots; returns the
 * minimal distance of any scaled coefficient to a rounding tie (0.5) */
double orc_encode(const orc_ctx *c, const double *vals, int64_t n_vals, double scale,
                  int64_t *out_coeffs);
void orc_decode(const orc_ctx *c, const double *coeffs, double scale, double *out_re /* N/2 */);

/* ---- ciphertexts ---- */
orc_ct *orc_encrypt_coeffs(orc_ctx *c, const int64_t *m, int level, double scale, uint64_t nonce);
orc_ct *orc_encrypt(orc_ctx *c, const double *vals, int64_t n_vals, int level, uint64_t nonce);
int orc_decrypt_coeffs(orc_ctx *c, const orc_ct *ct, double *out /* N, unscaled centered */);
int orc_decrypt(orc_ctx *c, const orc_ct *ct, double *out_slots /* N/2 real parts */);
void orc_ct_free(orc_ct *ct);
int orc_ct_level(const orc_ct *ct);
double orc_ct_scale(const orc_ct *ct);
int orc_ct_degree(const orc_ct *ct);
/* coefficient-domain residues [deg+1][level+1][N] */
void orc_ct_export(const orc_ct *ct, uint64_t *out);
orc_ct *orc_ct_import(orc_ctx *c, const uint64_t *in, int level, double scale);

/* ---- operations of Fig. 1 ---- */
orc_ct *orc_add(orc_ctx *c, const orc_ct *a, const orc_ct *b);
orc_ct *orc_sub(orc_ctx *c, const orc_ct *a, const orc_ct *b);
orc_ct *orc_drop(orc_ctx *c, const orc_ct *a, int level);
orc_ct *orc_mul_plain(orc_ctx *c, const orc_ct *a, const int64_t *pt, double pt_scale);
orc_ct *orc_mul_int(orc_ctx *c, const orc_ct *a, int64_t k);
orc_ct *orc_tensor(orc_ctx *c, const orc_ct *a, const orc_ct *b);     /* degree 2 */
orc_ct *orc_relin(orc_ctx *c, const orc_ct *a);
orc_ct *orc_mul(orc_ctx *c, const orc_ct *a, const orc_ct *b);        /* tensor + relin */
orc_ct *orc_rescale(orc_ctx *c, const orc_ct *a);
orc_ct *orc_rotate(orc_ctx *c, const orc_ct *a, int64_t k);
/* hoisted rotations of one ciphertext (Halevi-Shoup); must equal orc_rotate bit for bit */
void orc_rotate_hoisted(orc_ctx *c, const orc_ct *a, int n, const int64_t *ks, orc_ct **out);

/* ---- the packed matrix product (Alg. 3 + App. B) ---- */
/* schedule flags of the product (each combination is its own bit-exact reference):
 * RELIN_ONCE: relinearise the accumulated Step-3 sum once instead of every product;
 * HOIST_MODDOWN: sums of rotations share one ModDown, the terms being formed in the
 *   extended basis: Step 2's v_k . Rot(A0, k) + v_(k-h) . Rot(A0, k-h), and the giant-step
 *   sums of Steps 1-1 and 1-2 (and of Step 3 under STEP3_BSGS);
 * RESCALE_LATE: A^(k) is not rescaled; Step 3 multiplies one level higher and the sum is
 *   rescaled twice (same depth);
 * STEP3_BSGS: the Step-3 sum is split into baby and giant steps (k = bg i + j), so that B0
 *   is rotated bg - 1 times and each of the h / bg block sums once, instead of h - 1 rotations
 *   of B0; the A-side rotations absorb the giant-step shift. */
#define ORC_RELIN_EACH 0
#define ORC_RELIN_ONCE 1
#define ORC_HOIST_MODDOWN 2
#define ORC_RESCALE_LATE 4
#define ORC_STEP3_BSGS 8
orc_ct *orc_matmul(orc_ctx *c, const orc_ct *a, const orc_ct *b, int h, int relin_mode);
/* the product for a shape: t = h is Alg. 3; t < h (t | h) is HE-RMatMult (Alg. 6, App. D) with
 * a holding h/t vertical copies of a t x h matrix, the result holding h/t copies of the t x h
 * product; beta > 1 multiplies beta pairs of matrices packed by iota_beta (App. E:
 * matrix m, entry (i, j) at slot beta (h i + j) + m).  h, t, beta powers of two,
 * beta h^2 <= N/2. */
orc_ct *orc_matmul_ex(orc_ctx *c, const orc_ct *a, const orc_ct *b, int h, int t, int beta, int mode);
/* App. C: the transpose of every packed h x h matrix (diagonals (h-1) k, BSGS); depth 1;
 * the ModDown-hoisting flag of 'mode' applies to its giant steps */
orc_ct *orc_transpose(orc_ctx *c, const orc_ct *a, int h, int beta, int mode);
/* slot-domain 0/1 vectors of length h*h for the diagonals used by Alg. 3:
 * kind 0: u^mu_k (k in (-h,h)), 1: u^zeta_{h k} (k in [0,h)), 2: v_k (k in [0,h)), 3: v_{k-h},
 * 4: t_{(h-1)k}, the transpose diagonals of App. C (k in (-h,h)) */
void orc_mask_slots(int kind, int h, int k, double *out);
/* rotation amounts (mod N/2, normalised into [0,N/2)) the product needs for h under the
 * given schedule flags */
int orc_matmul_rotations(const orc_ctx *c, int h, int mode, int64_t *out, int cap);
int orc_matmul_rotations_ex(const orc_ctx *c, int h, int t, int beta, int mode, int64_t *out, int cap);
int orc_transpose_rotations(const orc_ctx *c, int h, int beta, int64_t *out, int cap);
/* 0 rotations, 1 key switches, 2 mul_pt, 3 mul_ct, 4 add, 5 rescale */
void orc_counters(const orc_ctx *c, int64_t out[6]);
void orc_reset_counters(orc_ctx *c);

/* ---- composite sign approximation (Sec. 4.2) ---- */
orc_ct *orc_sign(orc_ctx *c, const orc_ct *x, int d, int k, int relu);
/* numerators n_0 .. n_d of g_d's coefficients of x, x^3, ..., x^(2d+1), each over 2^(2d-1) */
void orc_gd_numerators(int d, int64_t *num);
/* Alg. 5: max(a, b) ~ (a + b)/2 + (a - b)/2 . g_d^(k)(a - b) */
orc_ct *orc_appmax(orc_ctx *c, const orc_ct *a, const orc_ct *b, int d, int k);
/* 2 x 2 max pooling of a packed h x h matrix by two AppMax levels (rotations 1 and h) */
orc_ct *orc_maxpool2(orc_ctx *c, const orc_ct *x, int h, int d, int k);
/* Alg. 6 aggregation: W - coeff . sum_i G_i (coeff = eta / (B N)) */
orc_ct *orc_fl_update(orc_ctx *c, const orc_ct *w, orc_ct *const *g, int n, double coeff);

#endif
