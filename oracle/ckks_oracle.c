/*
 * ckks_oracle.c -- CPU oracle for the Hercules packed ciphertext matrix product.
 *
 * TEST INFRASTRUCTURE ONLY (see ckks_oracle.h).  Plain scalar C: every modular
 * product is an unsigned __int128 product reduced with '%', polynomial products
 * go through a textbook twisted cyclic NTT, encoding runs in __float128.  The GPU
 * library never includes, links or calls this file.
 *
 * Paper passages followed (arXiv 2207.04620):
 *  - Sec. 2.2 and Fig. 1: the MCKKS operations Ecd, Dcd, Enc, Add, Sub, Mul_pt,
 *    Mul_ct, Rot, RS (single-key versions; the D* operations need other parties);
 *  - Sec. 3.2, Eq. 1 and Alg. 2: diagonal linear transforms, R(m,k) = left shift;
 *  - Sec. 3.3-3.6, Eqs. 2-16, Alg. 3: the packed product HE-MatMult;
 *  - App. B: baby-step/giant-step form of Steps 1-1 and 1-2;
 *  - Sec. 4.2: g_d(m) = sum_i 4^-i C(2i,i) m (1-m^2)^i and its k-fold composition;
 *    Alg. 5 / Sec. 4.4 for ReLU(x) = (x + x g_d^(k)(x)) / 2.
 * The RNS-CKKS internals (hybrid key switching, centered fast base conversion,
 * rescale by the last prime) are not described by the paper; they follow the
 * standard published constructions (Cheon-Han-Kim-Kim-Song 2018 RNS-CKKS,
 * Han-Ki 2020 hybrid key switching) under the conventions stated in ckks_oracle.h.
 */
#include "ckks_oracle.h"

#include <math.h>
#include <omp.h>
#include <quadmath.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;
typedef unsigned __int128 u128;
typedef __int128 i128;

#define MAXMOD 48

/* ------------------------------------------------------------------ */
/* integer helpers                                                     */
/* ------------------------------------------------------------------ */
static inline u64 mulmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }
static inline u64 addmod(u64 a, u64 b, u64 q) { u64 s = a + b; return s >= q ? s - q : s; }
static inline u64 submod(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + q - b; }
static u64 powmod(u64 a, u64 e, u64 q) {
    u64 r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = mulmod(r, a, q);
        a = mulmod(a, a, q);
        e >>= 1;
    }
    return r;
}
static u64 invmod(u64 a, u64 q) { return powmod(a, q - 2, q); } /* q prime */
/* signed integer -> residue */
static inline u64 smod(i128 v, u64 q) {
    i128 r = v % (i128)q;
    if (r < 0) r += q;
    return (u64)r;
}
/* centered representative of x in [0,q), q odd: (-(q-1)/2 .. (q-1)/2] */
static inline int64_t center(u64 x, u64 q) { return x > (q - 1) / 2 ? (int64_t)x - (int64_t)q : (int64_t)x; }

uint64_t orc_mulmod(uint64_t a, uint64_t b, uint64_t q) { return mulmod(a, b, q); }

/* deterministic Miller-Rabin for 64-bit integers */
int orc_is_prime(uint64_t n) {
    static const u64 bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++) {
        if (n == bases[i]) return 1;
        if (n % bases[i] == 0) return 0;
    }
    u64 d = n - 1;
    int r = 0;
    while (!(d & 1)) { d >>= 1; r++; }
    for (int i = 0; i < 12; i++) {
        u64 x = powmod(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int comp = 1;
        for (int j = 1; j < r; j++) {
            x = mulmod(x, x, n);
            if (x == n - 1) { comp = 0; break; }
        }
        if (comp) return 0;
    }
    return 1;
}

static int bitrev(int x, int bits) {
    int r = 0;
    for (int i = 0; i < bits; i++) r |= ((x >> i) & 1) << (bits - 1 - i);
    return r;
}

/* ------------------------------------------------------------------ */
/* ChaCha20 (RFC 8439 section 2.3)                                     */
/* ------------------------------------------------------------------ */
static inline uint32_t rotl32(uint32_t v, int c) { return (v << c) | (v >> (32 - c)); }
#define QR(a, b, c, d)                                   \
    do {                                                 \
        a += b; d ^= a; d = rotl32(d, 16);               \
        c += d; b ^= c; b = rotl32(b, 12);               \
        a += b; d ^= a; d = rotl32(d, 8);                \
        c += d; b ^= c; b = rotl32(b, 7);                \
    } while (0)

void orc_chacha20_block(const uint32_t key[8], uint32_t counter, const uint32_t nonce[3],
                        uint32_t out[16]) {
    uint32_t st[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u,
                       key[0], key[1], key[2], key[3], key[4], key[5], key[6], key[7],
                       counter, nonce[0], nonce[1], nonce[2]};
    uint32_t x[16];
    memcpy(x, st, sizeof x);
    for (int i = 0; i < 10; i++) {
        QR(x[0], x[4], x[8], x[12]);
        QR(x[1], x[5], x[9], x[13]);
        QR(x[2], x[6], x[10], x[14]);
        QR(x[3], x[7], x[11], x[15]);
        QR(x[0], x[5], x[10], x[15]);
        QR(x[1], x[6], x[11], x[12]);
        QR(x[2], x[7], x[8], x[13]);
        QR(x[3], x[4], x[9], x[14]);
    }
    for (int i = 0; i < 16; i++) out[i] = x[i] + st[i];
}

/* 64-bit word w of the stream (seed, purpose, index): block w/8, words 2(w%8), 2(w%8)+1 */
uint64_t orc_word(uint64_t seed, uint32_t purpose, uint64_t index, uint64_t w) {
    uint32_t key[8] = {(uint32_t)seed, (uint32_t)(seed >> 32), 0, 0, 0, 0, 0, 0};
    uint32_t nonce[3] = {purpose, (uint32_t)index, (uint32_t)(index >> 32)};
    uint32_t out[16];
    orc_chacha20_block(key, (uint32_t)(w / 8), nonce, out);
    int k = (int)(w % 8);
    return (u64)out[2 * k] | ((u64)out[2 * k + 1] << 32);
}

/* bulk stream: words [0, n) */
static void stream_words(u64 seed, uint32_t purpose, u64 index, int64_t n, u64 *out) {
    uint32_t key[8] = {(uint32_t)seed, (uint32_t)(seed >> 32), 0, 0, 0, 0, 0, 0};
    uint32_t nonce[3] = {purpose, (uint32_t)index, (uint32_t)(index >> 32)};
    for (int64_t b = 0; b * 8 < n; b++) {
        uint32_t o[16];
        orc_chacha20_block(key, (uint32_t)b, nonce, o);
        for (int k = 0; k < 8 && b * 8 + k < n; k++) out[b * 8 + k] = (u64)o[2 * k] | ((u64)o[2 * k + 1] << 32);
    }
}

/* Discrete Gaussian on [-19,19], rho(x) = exp(-x^2 / (2 sigma^2)), sigma = 3.2.
 * T[k] = floor(2^63 * Pr[|e| <= k]) for k in [0,19). */
void orc_gauss_table(uint64_t out[19]) {
    const __float128 sigma = 3.2Q;
    __float128 rho[20], tot = 0;
    for (int x = 0; x <= 19; x++) rho[x] = expq(-(__float128)(x * x) / (2 * sigma * sigma));
    tot = rho[0];
    for (int x = 1; x <= 19; x++) tot += 2 * rho[x];
    __float128 cum = rho[0];
    for (int k = 0; k < 19; k++) {
        if (k > 0) cum += 2 * rho[k];
        out[k] = (u64)floorq(cum / tot * 9223372036854775808.0Q);
    }
}

void orc_sample_ternary(uint64_t seed, uint32_t purpose, uint64_t index, int64_t n, int64_t *out) {
    u64 *w = malloc(sizeof(u64) * n);
    stream_words(seed, purpose, index, n, w);
    for (int64_t t = 0; t < n; t++) out[t] = (int64_t)(w[t] % 3) - 1;
    free(w);
}

void orc_sample_gauss(uint64_t seed, uint32_t purpose, uint64_t index, int64_t n, int64_t *out) {
    u64 T[19];
    orc_gauss_table(T);
    u64 *w = malloc(sizeof(u64) * n);
    stream_words(seed, purpose, index, n, w);
    for (int64_t t = 0; t < n; t++) {
        u64 u = w[t] >> 1;
        int mag = 0;
        for (int k = 0; k < 19; k++) mag += (u >= T[k]);
        out[t] = (w[t] & 1) ? -mag : mag;
    }
    free(w);
}

void orc_sample_uniform(uint64_t seed, uint32_t purpose, uint64_t index, uint64_t q, int64_t n,
                        uint64_t *out) {
    u64 *w = malloc(sizeof(u64) * 2 * n);
    stream_words(seed, purpose, index, 2 * n, w);
    for (int64_t t = 0; t < n; t++) out[t] = (u64)((((u128)w[2 * t + 1]) << 64 | w[2 * t]) % q);
    free(w);
}

/* stream purposes */
enum { P_SK = 1, P_PK_A = 2, P_PK_E = 3, P_SWK_A = 4, P_SWK_E = 5, P_ENC_V = 6, P_ENC_E0 = 7, P_ENC_E1 = 8 };

/* ------------------------------------------------------------------ */
/* context                                                             */
/* ------------------------------------------------------------------ */
typedef struct {
    u64 key_id;
    u64 *b, *a; /* evaluation form, [beta][n_q + n_p][N] */
} swk_t;

struct orc_ctx {
    int log_n;
    int64_t n;
    int n_q, n_p, alpha, beta;
    double scale;
    u64 seed;
    int threads;
    u64 mod[MAXMOD];
    u64 psi[MAXMOD];
    u64 *psi_pow[MAXMOD], *psi_ipow[MAXMOD], *w_pow[MAXMOD], *w_ipow[MAXMOD];
    u64 n_inv[MAXMOD];
    int64_t *s;
    u64 *s_eval;  /* [n_q+n_p][N] */
    u64 *pk0, *pk1; /* evaluation form [n_q][N] */
    swk_t *keys;
    int n_keys, cap_keys;
    int64_t cnt[6];
    /* mask cache */
    struct mask_ent { int kind, h, beta, k; int64_t rot; int64_t *coef; } *masks;
    int n_masks, cap_masks;
};

struct orc_ct {
    int level, deg;
    double scale;
    int64_t n;
    u64 *c[3]; /* coefficient form, [level+1][N] each */
};

enum { C_ROT = 0, C_KS, C_MULPT, C_MULCT, C_ADD, C_RS };

static void ntt_fwd(const orc_ctx *c, int mi, u64 *a);
static void ntt_inv(const orc_ctx *c, int mi, u64 *a);

static void setup_ntt(orc_ctx *c, int mi) {
    int64_t N = c->n;
    u64 q = c->mod[mi];
    /* a primitive 2N-th root: x^((q-1)/2N) for the first x whose N-th power of it is -1 */
    u64 root = 0;
    for (u64 x = 2;; x++) {
        u64 r = powmod(x, (q - 1) / (2 * N), q);
        if (powmod(r, N, q) == q - 1) { root = r; break; }
    }
    /* smallest primitive 2N-th root = min over odd powers */
    u64 best = root, r2 = mulmod(root, root, q), cur = root;
    for (int64_t k = 1; k < N; k++) {
        cur = mulmod(cur, r2, q);
        if (cur < best) best = cur;
    }
    c->psi[mi] = best;
    u64 psi = best, psii = invmod(best, q), w = mulmod(psi, psi, q), wi = mulmod(psii, psii, q);
    c->psi_pow[mi] = malloc(sizeof(u64) * N);
    c->psi_ipow[mi] = malloc(sizeof(u64) * N);
    c->w_pow[mi] = malloc(sizeof(u64) * N);
    c->w_ipow[mi] = malloc(sizeof(u64) * N);
    u64 a = 1, b = 1, e = 1, f = 1;
    for (int64_t j = 0; j < N; j++) {
        c->psi_pow[mi][j] = a; c->psi_ipow[mi][j] = b; c->w_pow[mi][j] = e; c->w_ipow[mi][j] = f;
        a = mulmod(a, psi, q); b = mulmod(b, psii, q); e = mulmod(e, w, q); f = mulmod(f, wi, q);
    }
    c->n_inv[mi] = invmod((u64)N % q, q);
}

static void gen_primes(orc_ctx *c, int n, const int *bits, int off) {
    u64 m2n = 2 * (u64)c->n;
    for (int i = 0; i < n; i++) {
        u64 cand = ((((u64)1) << bits[i]) - 1) / m2n * m2n + 1; /* largest = 1 mod 2N below 2^bits */
        for (;; cand -= m2n) {
            if (cand >= (((u64)1) << bits[i])) continue;
            int used = 0;
            for (int j = 0; j < off + i; j++) used |= (c->mod[j] == cand);
            if (!used && orc_is_prime(cand)) break;
        }
        c->mod[off + i] = cand;
    }
}

orc_ctx *orc_create(int log_n, int n_q, const int *q_bits, int n_p, const int *p_bits, int alpha,
                    double log_scale, uint64_t seed, int n_threads) {
    if (n_q + n_p > MAXMOD || alpha < 1) return NULL;
    orc_ctx *c = calloc(1, sizeof(orc_ctx));
    c->log_n = log_n;
    c->n = (int64_t)1 << log_n;
    c->n_q = n_q; c->n_p = n_p; c->alpha = alpha;
    c->beta = (n_q + alpha - 1) / alpha;
    c->scale = ldexp(1.0, 0) * pow(2.0, log_scale);
    c->seed = seed;
    c->threads = n_threads > 0 ? n_threads : omp_get_max_threads();
    gen_primes(c, n_q, q_bits, 0);
    gen_primes(c, n_p, p_bits, n_q);
    int M = n_q + n_p;
#pragma omp parallel for num_threads(c->threads)
    for (int i = 0; i < M; i++) setup_ntt(c, i);
    int64_t N = c->n;
    /* secret key: uniform ternary (Fig. 1 SecKeyGen, single party) */
    c->s = malloc(sizeof(int64_t) * N);
    orc_sample_ternary(seed, P_SK, 0, N, c->s);
    c->s_eval = malloc(sizeof(u64) * M * N);
#pragma omp parallel for num_threads(c->threads)
    for (int i = 0; i < M; i++) {
        u64 *x = c->s_eval + (int64_t)i * N;
        for (int64_t t = 0; t < N; t++) x[t] = smod(c->s[t], c->mod[i]);
        ntt_fwd(c, i, x);
    }
    /* public key pk = (-a s + e, a) over Q (Fig. 1 DKeyGen, single party) */
    c->pk0 = malloc(sizeof(u64) * n_q * N);
    c->pk1 = malloc(sizeof(u64) * n_q * N);
    int64_t *e = malloc(sizeof(int64_t) * N);
    orc_sample_gauss(seed, P_PK_E, 0, N, e);
#pragma omp parallel for num_threads(c->threads)
    for (int i = 0; i < n_q; i++) {
        u64 q = c->mod[i];
        u64 *a = c->pk1 + (int64_t)i * N, *b = c->pk0 + (int64_t)i * N;
        orc_sample_uniform(seed, P_PK_A, (u64)i, q, N, a);
        ntt_fwd(c, i, a);
        for (int64_t t = 0; t < N; t++) b[t] = smod(e[t], q);
        ntt_fwd(c, i, b);
        const u64 *se = c->s_eval + (int64_t)i * N;
        for (int64_t t = 0; t < N; t++) b[t] = submod(b[t], mulmod(a[t], se[t], q), q);
    }
    free(e);
    return c;
}

void orc_destroy(orc_ctx *c) {
    if (!c) return;
    for (int i = 0; i < c->n_q + c->n_p; i++) {
        free(c->psi_pow[i]); free(c->psi_ipow[i]); free(c->w_pow[i]); free(c->w_ipow[i]);
    }
    free(c->s); free(c->s_eval); free(c->pk0); free(c->pk1);
    for (int i = 0; i < c->n_keys; i++) { free(c->keys[i].a); free(c->keys[i].b); }
    free(c->keys);
    for (int i = 0; i < c->n_masks; i++) free(c->masks[i].coef);
    free(c->masks);
    free(c);
}

int orc_n_moduli(const orc_ctx *c) { return c->n_q + c->n_p; }
void orc_moduli(const orc_ctx *c, uint64_t *out) { memcpy(out, c->mod, sizeof(u64) * (c->n_q + c->n_p)); }
uint64_t orc_psi(const orc_ctx *c, int mi) { return c->psi[mi]; }
void orc_counters(const orc_ctx *c, int64_t out[6]) { memcpy(out, c->cnt, sizeof c->cnt); }
void orc_reset_counters(orc_ctx *c) { memset(c->cnt, 0, sizeof c->cnt); }

/* ------------------------------------------------------------------ */
/* NTT: negacyclic transform = psi-twist + cyclic DFT with omega = psi^2 */
/* ------------------------------------------------------------------ */
static void cyclic_dft(const orc_ctx *c, u64 *a, const u64 *wp, u64 q) {
    int64_t N = c->n;
    int L = c->log_n;
    for (int64_t i = 0; i < N; i++) {
        int64_t j = bitrev((int)i, L);
        if (j > i) { u64 t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    for (int64_t len = 2; len <= N; len <<= 1) {
        int64_t half = len / 2, step = N / len;
        for (int64_t i = 0; i < N; i += len)
            for (int64_t j = 0; j < half; j++) {
                u64 u = a[i + j], v = mulmod(a[i + j + half], wp[j * step], q);
                a[i + j] = addmod(u, v, q);
                a[i + j + half] = submod(u, v, q);
            }
    }
}

/* out[k] = a(psi^(2k+1)), natural order */
static void ntt_fwd(const orc_ctx *c, int mi, u64 *a) {
    u64 q = c->mod[mi];
    for (int64_t j = 0; j < c->n; j++) a[j] = mulmod(a[j], c->psi_pow[mi][j], q);
    cyclic_dft(c, a, c->w_pow[mi], q);
}

static void ntt_inv(const orc_ctx *c, int mi, u64 *a) {
    u64 q = c->mod[mi];
    cyclic_dft(c, a, c->w_ipow[mi], q);
    for (int64_t j = 0; j < c->n; j++) a[j] = mulmod(mulmod(a[j], c->n_inv[mi], q), c->psi_ipow[mi][j], q);
}

void orc_poly_mul(const orc_ctx *c, int mi, const uint64_t *a, const uint64_t *b, uint64_t *out) {
    int64_t N = c->n;
    u64 q = c->mod[mi];
    u64 *x = malloc(sizeof(u64) * N), *y = malloc(sizeof(u64) * N);
    memcpy(x, a, sizeof(u64) * N);
    memcpy(y, b, sizeof(u64) * N);
    ntt_fwd(c, mi, x);
    ntt_fwd(c, mi, y);
    for (int64_t t = 0; t < N; t++) x[t] = mulmod(x[t], y[t], q);
    ntt_inv(c, mi, x);
    memcpy(out, x, sizeof(u64) * N);
    free(x); free(y);
}

void orc_eval_bitrev(const orc_ctx *c, int mi, const uint64_t *a, uint64_t *out) {
    int64_t N = c->n;
    u64 *x = malloc(sizeof(u64) * N);
    memcpy(x, a, sizeof(u64) * N);
    ntt_fwd(c, mi, x);
    for (int64_t j = 0; j < N; j++) out[j] = x[bitrev((int)j, c->log_n)];
    free(x);
}

/* ------------------------------------------------------------------ */
/* centered fast base conversion                                        */
/* ------------------------------------------------------------------ */
/* x_s given modulo mod[src[s]] (s < n_src); returns sum_s y_s * (D/q_s) mod mod[dst]
 * with y_s = centered([x_s * (D/q_s)^-1]_{q_s}) and D = prod q_s. */
static void base_conv(const orc_ctx *c, int n_src, const int *src, const u64 *const *x, int dst, u64 *out) {
    int64_t N = c->n;
    u64 t = c->mod[dst];
    u64 hat_inv[MAXMOD], hat_t[MAXMOD];
    for (int s = 0; s < n_src; s++) {
        u64 qs = c->mod[src[s]], hs = 1 % qs, ht = 1 % t;
        for (int r = 0; r < n_src; r++)
            if (r != s) { hs = mulmod(hs, c->mod[src[r]] % qs, qs); ht = mulmod(ht, c->mod[src[r]] % t, t); }
        hat_inv[s] = invmod(hs, qs);
        hat_t[s] = ht;
    }
    for (int64_t i = 0; i < N; i++) {
        i128 acc = 0;
        for (int s = 0; s < n_src; s++) {
            u64 qs = c->mod[src[s]];
            int64_t y = center(mulmod(x[s][i], hat_inv[s], qs), qs);
            acc += (i128)y * (i128)hat_t[s];
        }
        out[i] = smod(acc, t);
    }
}

void orc_base_conv(const orc_ctx *c, int n_src, const int *src_idx, int dst_idx, const uint64_t *x,
                   uint64_t *out) {
    const u64 *ptr[MAXMOD];
    for (int s = 0; s < n_src; s++) ptr[s] = x + (int64_t)s * c->n;
    base_conv(c, n_src, src_idx, ptr, dst_idx, out);
}

/* ------------------------------------------------------------------ */
/* switching keys                                                      */
/* ------------------------------------------------------------------ */
/* key switching key from s' (given per modulus in evaluation form, [n_q+n_p][N]) to s.
 * digit j: b = -a s + e + [P]_{q_i} s' on the Q limbs of digit j, -a s + e elsewhere. */
static swk_t *get_key(orc_ctx *c, u64 key_id) {
    for (int i = 0; i < c->n_keys; i++)
        if (c->keys[i].key_id == key_id) return &c->keys[i];
    int64_t N = c->n;
    int M = c->n_q + c->n_p;
    /* s' in evaluation form: s^2 for key_id 0, sigma_g(s) for a Galois element g */
    u64 *sp = malloc(sizeof(u64) * M * N);
    if (key_id == 0) {
        for (int i = 0; i < M; i++)
            for (int64_t t = 0; t < N; t++)
                sp[(int64_t)i * N + t] = mulmod(c->s_eval[(int64_t)i * N + t], c->s_eval[(int64_t)i * N + t], c->mod[i]);
    } else {
        int64_t *gs = malloc(sizeof(int64_t) * N);
        for (int64_t i = 0; i < N; i++) {
            u64 e = ((u64)i * key_id) % (2 * (u64)N);
            if (e < (u64)N) gs[e] = c->s[i]; else gs[e - N] = -c->s[i];
        }
#pragma omp parallel for num_threads(c->threads)
        for (int i = 0; i < M; i++) {
            u64 *x = sp + (int64_t)i * N;
            for (int64_t t = 0; t < N; t++) x[t] = smod(gs[t], c->mod[i]);
            ntt_fwd(c, i, x);
        }
        free(gs);
    }
    u64 Pmod[MAXMOD];
    for (int i = 0; i < c->n_q; i++) {
        u64 p = 1;
        for (int k = 0; k < c->n_p; k++) p = mulmod(p, c->mod[c->n_q + k] % c->mod[i], c->mod[i]);
        Pmod[i] = p;
    }
    swk_t k;
    k.key_id = key_id;
    k.a = malloc(sizeof(u64) * c->beta * M * N);
    k.b = malloc(sizeof(u64) * c->beta * M * N);
    for (int j = 0; j < c->beta; j++) {
        int64_t *e = malloc(sizeof(int64_t) * N);
        orc_sample_gauss(c->seed, P_SWK_E, (key_id << 8) | (u64)j, N, e);
#pragma omp parallel for num_threads(c->threads)
        for (int i = 0; i < M; i++) {
            u64 q = c->mod[i];
            u64 *a = k.a + ((int64_t)j * M + i) * N, *b = k.b + ((int64_t)j * M + i) * N;
            orc_sample_uniform(c->seed, P_SWK_A, (key_id << 16) | ((u64)j << 8) | (u64)i, q, N, a);
            ntt_fwd(c, i, a);
            for (int64_t t = 0; t < N; t++) b[t] = smod(e[t], q);
            ntt_fwd(c, i, b);
            const u64 *se = c->s_eval + (int64_t)i * N;
            int in_digit = (i < c->n_q) && (i / c->alpha == j);
            for (int64_t t = 0; t < N; t++) {
                u64 v = submod(b[t], mulmod(a[t], se[t], q), q);
                if (in_digit) v = addmod(v, mulmod(Pmod[i], sp[(int64_t)i * N + t], q), q);
                b[t] = v;
            }
        }
        free(e);
    }
    free(sp);
    if (c->n_keys == c->cap_keys) {
        c->cap_keys = c->cap_keys ? 2 * c->cap_keys : 16;
        c->keys = realloc(c->keys, sizeof(swk_t) * c->cap_keys);
    }
    c->keys[c->n_keys] = k;
    return &c->keys[c->n_keys++];
}

/* ------------------------------------------------------------------ */
/* ciphertext helpers                                                  */
/* ------------------------------------------------------------------ */
static orc_ct *ct_new(const orc_ctx *c, int level, int deg, double scale) {
    orc_ct *r = calloc(1, sizeof(orc_ct));
    r->level = level; r->deg = deg; r->scale = scale; r->n = c->n;
    for (int p = 0; p <= deg; p++) r->c[p] = calloc((size_t)(level + 1) * c->n, sizeof(u64));
    return r;
}
void orc_ct_free(orc_ct *ct) {
    if (!ct) return;
    for (int p = 0; p < 3; p++) free(ct->c[p]);
    free(ct);
}
int orc_ct_level(const orc_ct *ct) { return ct->level; }
double orc_ct_scale(const orc_ct *ct) { return ct->scale; }
int orc_ct_degree(const orc_ct *ct) { return ct->deg; }
static inline u64 *limb(const orc_ct *ct, int p, int i) { return ct->c[p] + (int64_t)i * ct->n; }

void orc_ct_export(const orc_ct *ct, uint64_t *out) {
    size_t sz = (size_t)(ct->level + 1) * ct->n;
    for (int p = 0; p <= ct->deg; p++) memcpy(out + p * sz, ct->c[p], sz * sizeof(u64));
}
orc_ct *orc_ct_import(orc_ctx *c, const uint64_t *in, int level, double scale) {
    orc_ct *r = ct_new(c, level, 1, scale);
    size_t sz = (size_t)(level + 1) * c->n;
    for (int p = 0; p < 2; p++) memcpy(r->c[p], in + p * sz, sz * sizeof(u64));
    return r;
}

orc_ct *orc_drop(orc_ctx *c, const orc_ct *a, int level) {
    if (level > a->level) return NULL;
    orc_ct *r = ct_new(c, level, a->deg, a->scale);
    for (int p = 0; p <= a->deg; p++) memcpy(r->c[p], a->c[p], sizeof(u64) * (level + 1) * c->n);
    return r;
}
static orc_ct *ct_copy(orc_ctx *c, const orc_ct *a) { return orc_drop(c, a, a->level); }

/* ------------------------------------------------------------------ */
/* encoding (Fig. 1 Ecd/Dcd), in __float128                             */
/* ------------------------------------------------------------------ */
/* in-place complex DFT of size N: X_k = sum_j x_j exp(sign * 2 pi i j k / N) */
static void qfft(int log_n, __float128 *re, __float128 *im, int sign) {
    int64_t N = (int64_t)1 << log_n;
    for (int64_t i = 0; i < N; i++) {
        int64_t j = bitrev((int)i, log_n);
        if (j > i) {
            __float128 t = re[i]; re[i] = re[j]; re[j] = t;
            t = im[i]; im[i] = im[j]; im[j] = t;
        }
    }
    __float128 *cr = malloc(sizeof(__float128) * N / 2), *ci = malloc(sizeof(__float128) * N / 2);
    for (int64_t k = 0; k < N / 2; k++) {
        __float128 ang = 2 * M_PIq * (__float128)k / (__float128)N;
        cr[k] = cosq(ang);
        ci[k] = sign * sinq(ang);
    }
    for (int64_t len = 2; len <= N; len <<= 1) {
        int64_t half = len / 2, step = N / len;
        for (int64_t i = 0; i < N; i += len)
            for (int64_t j = 0; j < half; j++) {
                __float128 wr = cr[j * step], wi = ci[j * step];
                __float128 xr = re[i + j + half], xi = im[i + j + half];
                __float128 vr = xr * wr - xi * wi, vi = xr * wi + xi * wr;
                re[i + j + half] = re[i + j] - vr; im[i + j + half] = im[i + j] - vi;
                re[i + j] += vr; im[i + j] += vi;
            }
    }
    free(cr); free(ci);
}

/* coefficient i of the real polynomial m with m(zeta^(5^j)) = z_j (z real here):
 * m_i = (1/N) sum over odd r of w_r zeta^(-r i), with w_{5^j} = z_j = w_{-5^j}. */
double orc_encode(const orc_ctx *c, const double *vals, int64_t n_vals, double scale, int64_t *out) {
    int64_t N = c->n, slots = N / 2;
    __float128 *re = calloc(N, sizeof(__float128)), *im = calloc(N, sizeof(__float128));
    u64 r = 1;
    for (int64_t j = 0; j < slots; j++) {
        double z = vals[j % n_vals];
        re[(r - 1) / 2] = z;
        re[(2 * N - r - 1) / 2] = z;
        r = (r * 5) % (2 * (u64)N);
    }
    qfft(c->log_n, re, im, -1);
    double min_tie = 1.0;
    for (int64_t i = 0; i < N; i++) {
        __float128 ang = -M_PIq * (__float128)i / (__float128)N; /* zeta^-i */
        __float128 v = (re[i] * cosq(ang) - im[i] * sinq(ang)) / (__float128)N * (__float128)scale;
        __float128 fl = floorq(v);
        double d = fabs((double)(v - fl) - 0.5);
        if (d < min_tie) min_tie = d;
        out[i] = (int64_t)roundq(v);
    }
    free(re); free(im);
    return min_tie;
}

void orc_decode(const orc_ctx *c, const double *coeffs, double scale, double *out_re) {
    int64_t N = c->n, slots = N / 2;
    __float128 *re = calloc(N, sizeof(__float128)), *im = calloc(N, sizeof(__float128));
    for (int64_t i = 0; i < N; i++) {
        __float128 ang = M_PIq * (__float128)i / (__float128)N; /* m_i zeta^i */
        re[i] = (__float128)coeffs[i] * cosq(ang);
        im[i] = (__float128)coeffs[i] * sinq(ang);
    }
    qfft(c->log_n, re, im, +1);
    u64 r = 1;
    for (int64_t j = 0; j < slots; j++) {
        out_re[j] = (double)(re[(r - 1) / 2] / (__float128)scale);
        r = (r * 5) % (2 * (u64)N);
    }
    free(re); free(im);
}

/* ------------------------------------------------------------------ */
/* encryption / decryption (Fig. 1 Enc, single-key Dec)                 */
/* ------------------------------------------------------------------ */
orc_ct *orc_encrypt_coeffs(orc_ctx *c, const int64_t *m, int level, double scale, uint64_t nonce) {
    if (level < 0 || level >= c->n_q) return NULL;
    int64_t N = c->n;
    int64_t *v = malloc(sizeof(int64_t) * N), *e0 = malloc(sizeof(int64_t) * N), *e1 = malloc(sizeof(int64_t) * N);
    orc_sample_ternary(c->seed, P_ENC_V, nonce, N, v);
    orc_sample_gauss(c->seed, P_ENC_E0, nonce, N, e0);
    orc_sample_gauss(c->seed, P_ENC_E1, nonce, N, e1);
    orc_ct *r = ct_new(c, level, 1, scale);
#pragma omp parallel for num_threads(c->threads)
    for (int i = 0; i <= level; i++) {
        u64 q = c->mod[i];
        u64 *x = malloc(sizeof(u64) * N);
        for (int64_t t = 0; t < N; t++) x[t] = smod(v[t], q);
        ntt_fwd(c, i, x);
        u64 *c0 = limb(r, 0, i), *c1 = limb(r, 1, i);
        for (int64_t t = 0; t < N; t++) {
            c0[t] = mulmod(x[t], c->pk0[(int64_t)i * N + t], q);
            c1[t] = mulmod(x[t], c->pk1[(int64_t)i * N + t], q);
        }
        ntt_inv(c, i, c0);
        ntt_inv(c, i, c1);
        for (int64_t t = 0; t < N; t++) {
            c0[t] = addmod(c0[t], smod((i128)m[t] + e0[t], q), q);
            c1[t] = addmod(c1[t], smod(e1[t], q), q);
        }
        free(x);
    }
    free(v); free(e0); free(e1);
    return r;
}

orc_ct *orc_encrypt(orc_ctx *c, const double *vals, int64_t n_vals, int level, uint64_t nonce) {
    int64_t *m = malloc(sizeof(int64_t) * c->n);
    orc_encode(c, vals, n_vals, c->scale, m);
    orc_ct *r = orc_encrypt_coeffs(c, m, level, c->scale, nonce);
    free(m);
    return r;
}

/* centered value of c0 + c1 s (+ c2 s^2) from the first two limbs (Garner); every
 * further limb must agree, else the plaintext exceeded q0 q1 / 2 and -1 is returned */
int orc_decrypt_coeffs(orc_ctx *c, const orc_ct *ct, double *out) {
    int64_t N = c->n;
    int nl = ct->level + 1;
    u64 *m = malloc(sizeof(u64) * nl * N);
#pragma omp parallel for num_threads(c->threads)
    for (int i = 0; i < nl; i++) {
        u64 q = c->mod[i];
        u64 *x = m + (int64_t)i * N, *y = malloc(sizeof(u64) * N), *s = malloc(sizeof(u64) * N);
        for (int64_t t = 0; t < N; t++) s[t] = smod(c->s[t], q);
        memcpy(x, limb(ct, 0, i), sizeof(u64) * N);
        orc_poly_mul(c, i, limb(ct, 1, i), s, y);
        for (int64_t t = 0; t < N; t++) x[t] = addmod(x[t], y[t], q);
        if (ct->deg == 2) {
            u64 *s2 = malloc(sizeof(u64) * N);
            orc_poly_mul(c, i, s, s, s2);
            orc_poly_mul(c, i, limb(ct, 2, i), s2, y);
            for (int64_t t = 0; t < N; t++) x[t] = addmod(x[t], y[t], q);
            free(s2);
        }
        free(y); free(s);
    }
    int bad = 0;
    u64 q0 = c->mod[0], q1 = nl > 1 ? c->mod[1] : 0;
    u64 q0inv = nl > 1 ? invmod(q0 % q1, q1) : 0;
    for (int64_t t = 0; t < N; t++) {
        i128 v;
        if (nl == 1) {
            v = center(m[t], q0);
        } else {
            u64 x0 = m[t], x1 = m[N + t];
            u64 k = mulmod(submod(x1, x0 % q1, q1), q0inv, q1);
            u128 w = (u128)x0 + (u128)q0 * k;
            u128 Q2 = (u128)q0 * q1;
            v = w > Q2 / 2 ? (i128)w - (i128)Q2 : (i128)w;
            for (int i = 2; i < nl; i++)
                if (smod(v, c->mod[i]) != m[(int64_t)i * N + t]) bad = 1;
        }
        out[t] = (double)v;
    }
    free(m);
    return bad ? -1 : 0;
}

int orc_decrypt(orc_ctx *c, const orc_ct *ct, double *out_slots) {
    double *co = malloc(sizeof(double) * c->n);
    int rc = orc_decrypt_coeffs(c, ct, co);
    orc_decode(c, co, ct->scale, out_slots);
    free(co);
    return rc;
}

/* ------------------------------------------------------------------ */
/* homomorphic operations                                              */
/* ------------------------------------------------------------------ */
static orc_ct *add_sub(orc_ctx *c, const orc_ct *a, const orc_ct *b, int sub) {
    int level = a->level < b->level ? a->level : b->level;
    int deg = a->deg > b->deg ? a->deg : b->deg;
    orc_ct *r = ct_new(c, level, deg, a->scale > b->scale ? a->scale : b->scale);
    for (int p = 0; p <= deg; p++)
        for (int i = 0; i <= level; i++) {
            u64 q = c->mod[i], *o = limb(r, p, i);
            const u64 *x = p <= a->deg ? limb(a, p, i) : NULL, *y = p <= b->deg ? limb(b, p, i) : NULL;
            for (int64_t t = 0; t < c->n; t++) {
                u64 u = x ? x[t] : 0, v = y ? y[t] : 0;
                o[t] = sub ? submod(u, v, q) : addmod(u, v, q);
            }
        }
    c->cnt[C_ADD]++;
    return r;
}
orc_ct *orc_add(orc_ctx *c, const orc_ct *a, const orc_ct *b) { return add_sub(c, a, b, 0); }
orc_ct *orc_sub(orc_ctx *c, const orc_ct *a, const orc_ct *b) { return add_sub(c, a, b, 1); }

orc_ct *orc_mul_plain(orc_ctx *c, const orc_ct *a, const int64_t *pt, double pt_scale) {
    orc_ct *r = ct_new(c, a->level, a->deg, a->scale * pt_scale);
    int64_t N = c->n;
#pragma omp parallel for num_threads(c->threads)
    for (int i = 0; i <= a->level; i++) {
        u64 q = c->mod[i];
        u64 *m = malloc(sizeof(u64) * N);
        for (int64_t t = 0; t < N; t++) m[t] = smod(pt[t], q);
        for (int p = 0; p <= a->deg; p++) orc_poly_mul(c, i, limb(a, p, i), m, limb(r, p, i));
        free(m);
    }
    c->cnt[C_MULPT]++;
    return r;
}

orc_ct *orc_mul_int(orc_ctx *c, const orc_ct *a, int64_t k) {
    orc_ct *r = ct_new(c, a->level, a->deg, a->scale);
    for (int p = 0; p <= a->deg; p++)
        for (int i = 0; i <= a->level; i++) {
            u64 q = c->mod[i], kk = smod(k, q);
            const u64 *x = limb(a, p, i);
            u64 *o = limb(r, p, i);
            for (int64_t t = 0; t < c->n; t++) o[t] = mulmod(x[t], kk, q);
        }
    return r;
}

/* (a0 b0, a0 b1 + a1 b0, a1 b1) at the lower level; scale multiplies (Fig. 1 Mul_ct) */
orc_ct *orc_tensor(orc_ctx *c, const orc_ct *a, const orc_ct *b) {
    if (a->deg != 1 || b->deg != 1) return NULL;
    int level = a->level < b->level ? a->level : b->level;
    orc_ct *r = ct_new(c, level, 2, a->scale * b->scale);
    int64_t N = c->n;
#pragma omp parallel for num_threads(c->threads)
    for (int i = 0; i <= level; i++) {
        u64 q = c->mod[i];
        u64 *t1 = malloc(sizeof(u64) * N), *t2 = malloc(sizeof(u64) * N);
        orc_poly_mul(c, i, limb(a, 0, i), limb(b, 0, i), limb(r, 0, i));
        orc_poly_mul(c, i, limb(a, 0, i), limb(b, 1, i), t1);
        orc_poly_mul(c, i, limb(a, 1, i), limb(b, 0, i), t2);
        for (int64_t t = 0; t < N; t++) limb(r, 1, i)[t] = addmod(t1[t], t2[t], q);
        orc_poly_mul(c, i, limb(a, 1, i), limb(b, 1, i), limb(r, 2, i));
        free(t1); free(t2);
    }
    c->cnt[C_MULCT]++;
    return r;
}

/* digit j of d (coefficient form, limbs 0..level) lifted to modulus index t */
static void modup_digit(const orc_ctx *c, int level, u64 *const *d, int j, int t, u64 *out) {
    int lo = j * c->alpha, hi = lo + c->alpha;
    if (hi > level + 1) hi = level + 1;
    if (t >= lo && t < hi) { memcpy(out, d[t], sizeof(u64) * c->n); return; }
    int src[MAXMOD];
    const u64 *x[MAXMOD];
    for (int s = lo; s < hi; s++) { src[s - lo] = s; x[s - lo] = d[s]; }
    base_conv(c, hi - lo, src, x, t, out);
}

/* inner product of lifted digits with the key, then ModDown; d in coefficient form.
 * 'lift' (optional) holds precomputed lifted digits [beta][level+1+K][N] in coefficient form. */
/* inner product of the lifted digits with the key over Q_l and P: u0, u1 in coefficient
 * form, [level+1+K][N] (Q limbs 0..level, then the K special primes) */
static void ks_inner(orc_ctx *c, int level, u64 *const *d, const u64 *lift, const swk_t *k, u64 *u0, u64 *u1) {
    int64_t N = c->n;
    int nl = level + 1, K = c->n_p, M = c->n_q + c->n_p;
    int beta = (nl + c->alpha - 1) / c->alpha;
    int ext[MAXMOD];
    for (int i = 0; i < nl; i++) ext[i] = i;
    for (int i = 0; i < K; i++) ext[nl + i] = c->n_q + i;
#pragma omp parallel for num_threads(c->threads)
    for (int ti = 0; ti < nl + K; ti++) {
        int t = ext[ti];
        u64 q = c->mod[t];
        u64 *x = malloc(sizeof(u64) * N);
        u64 *a0 = u0 + (int64_t)ti * N, *a1 = u1 + (int64_t)ti * N;
        memset(a0, 0, sizeof(u64) * N);
        memset(a1, 0, sizeof(u64) * N);
        for (int j = 0; j < beta; j++) {
            if (lift) memcpy(x, lift + ((int64_t)j * (nl + K) + ti) * N, sizeof(u64) * N);
            else modup_digit(c, level, d, j, t, x);
            ntt_fwd(c, t, x);
            const u64 *kb = k->b + ((int64_t)j * M + t) * N, *ka = k->a + ((int64_t)j * M + t) * N;
            for (int64_t s = 0; s < N; s++) {
                a0[s] = addmod(a0[s], mulmod(x[s], kb[s], q), q);
                a1[s] = addmod(a1[s], mulmod(x[s], ka[s], q), q);
            }
        }
        ntt_inv(c, t, a0);
        ntt_inv(c, t, a1);
        free(x);
    }
    c->cnt[C_KS]++;
}

/* ModDown of one polynomial over Q_l and P: out_i = (u_i - conv_P(u)_i) * P^-1 mod q_i */
static void ks_moddown(orc_ctx *c, int level, const u64 *u, u64 *out) {
    int64_t N = c->n;
    int nl = level + 1, K = c->n_p;
    int psrc[MAXMOD];
    for (int i = 0; i < K; i++) psrc[i] = c->n_q + i;
    const u64 *px[MAXMOD];
    for (int i = 0; i < K; i++) px[i] = u + (int64_t)(nl + i) * N;
#pragma omp parallel for num_threads(c->threads)
    for (int i = 0; i < nl; i++) {
        u64 q = c->mod[i], P = 1;
        for (int kk = 0; kk < K; kk++) P = mulmod(P, c->mod[c->n_q + kk] % q, q);
        u64 pinv = invmod(P, q);
        u64 *cv = malloc(sizeof(u64) * N);
        base_conv(c, K, psrc, px, i, cv);
        for (int64_t s = 0; s < N; s++) out[(int64_t)i * N + s] = mulmod(submod(u[(int64_t)i * N + s], cv[s], q), pinv, q);
        free(cv);
    }
}

/* inner product of the lifted digits with the key, then ModDown; d in coefficient form.
 * 'lift' (optional) holds precomputed lifted digits [beta][level+1+K][N] in coefficient form. */
static void keyswitch_core(orc_ctx *c, int level, u64 *const *d, const u64 *lift, const swk_t *k,
                           u64 *out0, u64 *out1) {
    int64_t N = c->n;
    int nl = level + 1, K = c->n_p;
    u64 *u0 = malloc(sizeof(u64) * (nl + K) * N), *u1 = malloc(sizeof(u64) * (nl + K) * N);
    ks_inner(c, level, d, lift, k, u0, u1);
    ks_moddown(c, level, u0, out0);
    ks_moddown(c, level, u1, out1);
    free(u0); free(u1);
}

orc_ct *orc_relin(orc_ctx *c, const orc_ct *a) {
    if (a->deg != 2) return ct_copy(c, a);
    const swk_t *k = get_key(c, 0);
    int64_t N = c->n;
    int nl = a->level + 1;
    u64 *d[MAXMOD];
    for (int i = 0; i < nl; i++) d[i] = limb(a, 2, i);
    u64 *o0 = malloc(sizeof(u64) * nl * N), *o1 = malloc(sizeof(u64) * nl * N);
    keyswitch_core(c, a->level, d, NULL, k, o0, o1);
    orc_ct *r = ct_new(c, a->level, 1, a->scale);
    for (int i = 0; i < nl; i++) {
        u64 q = c->mod[i];
        for (int64_t t = 0; t < N; t++) {
            limb(r, 0, i)[t] = addmod(limb(a, 0, i)[t], o0[(int64_t)i * N + t], q);
            limb(r, 1, i)[t] = addmod(limb(a, 1, i)[t], o1[(int64_t)i * N + t], q);
        }
    }
    free(o0); free(o1);
    return r;
}

orc_ct *orc_mul(orc_ctx *c, const orc_ct *a, const orc_ct *b) {
    orc_ct *t = orc_tensor(c, a, b);
    if (!t) return NULL;
    orc_ct *r = orc_relin(c, t);
    orc_ct_free(t);
    return r;
}

/* Fig. 1 RS: divide by the last prime q_l with centered rounding; level - 1 */
orc_ct *orc_rescale(orc_ctx *c, const orc_ct *a) {
    if (a->level < 1) return NULL;
    int l = a->level;
    u64 ql = c->mod[l];
    orc_ct *r = ct_new(c, l - 1, a->deg, a->scale / (double)ql);
    for (int p = 0; p <= a->deg; p++) {
        const u64 *last = limb(a, p, l);
#pragma omp parallel for num_threads(c->threads)
        for (int i = 0; i < l; i++) {
            u64 q = c->mod[i], inv = invmod(ql % q, q);
            const u64 *x = limb(a, p, i);
            u64 *o = limb(r, p, i);
            for (int64_t t = 0; t < c->n; t++) o[t] = mulmod(submod(x[t], smod(center(last[t], ql), q), q), inv, q);
        }
    }
    c->cnt[C_RS]++;
    return r;
}

static u64 galois_elt(const orc_ctx *c, int64_t k) {
    int64_t half = c->n / 2;
    int64_t kk = ((k % half) + half) % half;
    return powmod(5, (u64)kk, 2 * (u64)c->n);
}

/* sigma_g: X^i -> X^(i g) in Z_q[X]/(X^N+1) */
static void automorph(const orc_ctx *c, const u64 *in, u64 *out, u64 g, u64 q) {
    int64_t N = c->n;
    for (int64_t i = 0; i < N; i++) {
        u64 e = ((u64)i * g) % (2 * (u64)N);
        if (e < (u64)N) out[e] = in[i]; else out[e - N] = in[i] ? q - in[i] : 0;
    }
}

/* Fig. 1 Rot, left rotation R(m,k) (Sec. 3.2): sigma_g with g = 5^k, key switch back to s */
orc_ct *orc_rotate(orc_ctx *c, const orc_ct *a, int64_t k) {
    if (a->deg != 1) return NULL;
    u64 g = galois_elt(c, k);
    if (g == 1) return ct_copy(c, a);
    const swk_t *key = get_key(c, g);
    int64_t N = c->n;
    int nl = a->level + 1;
    orc_ct *r = ct_new(c, a->level, 1, a->scale);
    u64 *p1 = malloc(sizeof(u64) * nl * N);
    u64 *d[MAXMOD];
    for (int i = 0; i < nl; i++) {
        automorph(c, limb(a, 0, i), limb(r, 0, i), g, c->mod[i]);
        automorph(c, limb(a, 1, i), p1 + (int64_t)i * N, g, c->mod[i]);
        d[i] = p1 + (int64_t)i * N;
    }
    u64 *o0 = malloc(sizeof(u64) * nl * N);
    keyswitch_core(c, a->level, d, NULL, key, o0, limb(r, 1, 0));
    for (int i = 0; i < nl; i++) {
        u64 q = c->mod[i];
        for (int64_t t = 0; t < N; t++) limb(r, 0, i)[t] = addmod(limb(r, 0, i)[t], o0[(int64_t)i * N + t], q);
    }
    free(o0); free(p1);
    c->cnt[C_ROT]++;
    return r;
}

/* Hoisted form: lift the digits of c1 once, then permute the lifted digits.  Exact
 * because the centered lift of -x is minus the lift of x (odd moduli). */
void orc_rotate_hoisted(orc_ctx *c, const orc_ct *a, int n, const int64_t *ks, orc_ct **out) {
    int64_t N = c->n;
    int nl = a->level + 1, K = c->n_p, ne = nl + K;
    int beta = (nl + c->alpha - 1) / c->alpha;
    int ext[MAXMOD];
    for (int i = 0; i < nl; i++) ext[i] = i;
    for (int i = 0; i < K; i++) ext[nl + i] = c->n_q + i;
    u64 *d[MAXMOD];
    for (int i = 0; i < nl; i++) d[i] = limb(a, 1, i);
    u64 *lift = malloc(sizeof(u64) * beta * ne * N);
    for (int j = 0; j < beta; j++)
#pragma omp parallel for num_threads(c->threads)
        for (int ti = 0; ti < ne; ti++) modup_digit(c, a->level, d, j, ext[ti], lift + ((int64_t)j * ne + ti) * N);
    u64 *perm = malloc(sizeof(u64) * beta * ne * N);
    for (int r = 0; r < n; r++) {
        u64 g = galois_elt(c, ks[r]);
        if (g == 1) { out[r] = ct_copy(c, a); continue; }
        const swk_t *key = get_key(c, g);
        for (int j = 0; j < beta; j++)
            for (int ti = 0; ti < ne; ti++)
                automorph(c, lift + ((int64_t)j * ne + ti) * N, perm + ((int64_t)j * ne + ti) * N, g, c->mod[ext[ti]]);
        orc_ct *o = ct_new(c, a->level, 1, a->scale);
        u64 *o0 = malloc(sizeof(u64) * nl * N);
        keyswitch_core(c, a->level, NULL, perm, key, o0, limb(o, 1, 0));
        for (int i = 0; i < nl; i++) {
            u64 q = c->mod[i];
            automorph(c, limb(a, 0, i), limb(o, 0, i), g, q);
            for (int64_t t = 0; t < N; t++) limb(o, 0, i)[t] = addmod(limb(o, 0, i)[t], o0[(int64_t)i * N + t], q);
        }
        free(o0);
        c->cnt[C_ROT]++;
        out[r] = o;
    }
    free(lift); free(perm);
}

/* ------------------------------------------------------------------ */
/* Alg. 3 HE-MatMult with the App. B baby-step/giant-step split          */
/* ------------------------------------------------------------------ */
/* diagonal vectors of Sec. 3.5 / 3.6 (Fig. 2 gives them for h = 3) */
void orc_mask_slots(int kind, int h, int k, double *out) {
    int n = h * h;
    for (int t = 0; t < n; t++) {
        int v = 0;
        if (kind == 0) {        /* u^mu_k, k in (-h, h) */
            if (k >= 0) v = (t - h * k >= 0) && (t - h * k < h - k);
            else v = (-k <= t - (h + k) * h) && (t - (h + k) * h < h);
        } else if (kind == 1) { /* u^zeta_{h k}: t = k + h i */
            v = (t % h) == k;
        } else if (kind == 2) { /* v_k: 0 <= [t]_h < h - k  (k = 0 gives all ones) */
            v = (t % h) < h - k;
        } else if (kind == 3) { /* v_{k-h}: h - k <= [t]_h < h */
            v = (t % h) >= h - k;
        } else {                /* kind 4, App. C: diagonal (h-1) k of U^T, k in (-h, h).  Output
                                 * t = h i + j reads a[h j + i] = a[t + (h-1)(j - i)], so the
                                 * diagonal (h-1) k is 1 exactly where j - i = k */
            v = (t % h) - (t / h) == k;
        }
        out[t] = v;
    }
}
/* the encoded mask R(u, rot) of kind/h/k (rot in positions of the h^2 vector), expanded for
 * the packing iota_beta (App. E): entry t of the matrix vector fills slots beta t .. beta t +
 * beta - 1, so a rotation by beta r of the packed vector is a rotation by r of every matrix */
static const int64_t *get_mask_b(orc_ctx *c, int kind, int h, int beta, int k, int64_t rot) {
    for (int i = 0; i < c->n_masks; i++) {
        struct mask_ent *m = &c->masks[i];
        if (m->kind == kind && m->h == h && m->beta == beta && m->k == k && m->rot == rot) return m->coef;
    }
    int n = h * h;
    double *u = malloc(sizeof(double) * n), *ur = malloc(sizeof(double) * (size_t)n * beta);
    orc_mask_slots(kind, h, k, u);
    for (int t = 0; t < n; t++)
        for (int e = 0; e < beta; e++) ur[(int64_t)beta * t + e] = u[(((t + rot) % n) + n) % n]; /* R(u, rot)[t] = u[t + rot] */
    int64_t *coef = malloc(sizeof(int64_t) * c->n);
    orc_encode(c, ur, (int64_t)n * beta, c->scale, coef);
    free(u); free(ur);
    if (c->n_masks == c->cap_masks) {
        c->cap_masks = c->cap_masks ? 2 * c->cap_masks : 64;
        c->masks = realloc(c->masks, sizeof(struct mask_ent) * c->cap_masks);
    }
    struct mask_ent e = {kind, h, beta, k, rot, coef};
    c->masks[c->n_masks++] = e;
    return coef;
}
static const int64_t *get_mask(orc_ctx *c, int kind, int h, int k, int64_t rot) {
    return get_mask_b(c, kind, h, 1, k, rot);
}

static int ilog2(int h) { int l = 0; while ((1 << l) < h) l++; return l; }
static int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
static orc_ct *acc_add(orc_ctx *c, orc_ct *acc, orc_ct *t) {
    if (!acc) return t;
    orc_ct *r = orc_add(c, acc, t);
    orc_ct_free(acc); orc_ct_free(t);
    return r;
}

/* baby-step count of the Step-3 split k = bg i + j over t rounds (t = h for a square
 * product): bg = 2^ceil((log2 t + 1) / 2), at most t; without the Step-3 flag the sum is one
 * block of t terms */
static int step3_baby(int t, int mode) {
    if (!(mode & ORC_STEP3_BSGS)) return t;
    int bg = 1 << ((ilog2(t) + 2) / 2);
    return bg < t ? bg : t;
}

/* rotation amounts of HE-LinTrans with BSGS (App. B) over diagonals d in [dlo, dhi] at
 * rotation unit u: baby steps u j (0 < j < b), giant steps u b i (i != 0) */
static int lintrans_rotations(int b, int64_t unit, int dlo, int dhi, int64_t *out) {
    int m = 0;
    for (int j = 1; j < b; j++) out[m++] = unit * j;
    for (int i = floordiv(dlo, b); i <= floordiv(dhi, b); i++)
        if (i) out[m++] = unit * b * i;
    return m;
}

/* normalise amounts (times beta) into [0, N/2), drop 0 and duplicates */
static int normalise_rotations(const orc_ctx *c, const int64_t *tmp, int m, int beta, int64_t *out, int cap) {
    int64_t half = c->n / 2;
    int n = 0;
    for (int i = 0; i < m; i++) {
        int64_t v = (((tmp[i] * beta) % half) + half) % half;
        int dup = 0;
        for (int j = 0; j < n && j < cap; j++) dup |= out[j] == v;
        if (!dup && v != 0) { if (n < cap) out[n] = v; n++; }
    }
    return n;
}

int orc_matmul_rotations_ex(const orc_ctx *c, int h, int t, int beta, int mode, int64_t *out, int cap) {
    int b = 1 << ((ilog2(h) + 1) / 2), bg = step3_baby(t, mode);
    int64_t tmp[8192];
    int m = 0;
    m += lintrans_rotations(b, 1, 1 - h, h - 1, tmp + m);
    m += lintrans_rotations(b, h, 0, h - 1, tmp + m);
    for (int k = 1; k < t; k++) {
        int64_t shift = (int64_t)h * bg * (k / bg);
        tmp[m++] = k - shift;
        tmp[m++] = k - h - shift;
    }
    for (int j = 1; j < bg; j++) tmp[m++] = (int64_t)h * j;
    for (int i = 1; i * bg < t; i++) tmp[m++] = (int64_t)h * bg * i;
    for (int s = 0; (t << s) < h; s++) tmp[m++] = ((int64_t)t * h) << s;
    return normalise_rotations(c, tmp, m, beta, out, cap);
}

int orc_matmul_rotations(const orc_ctx *c, int h, int mode, int64_t *out, int cap) {
    return orc_matmul_rotations_ex(c, h, h, 1, mode, out, cap);
}

int orc_transpose_rotations(const orc_ctx *c, int h, int beta, int64_t *out, int cap) {
    int64_t tmp[1024];
    int m = lintrans_rotations(1 << ((ilog2(h) + 1) / 2), h - 1, 1 - h, h - 1, tmp);
    return normalise_rotations(c, tmp, m, beta, out, cap);
}

/* sum_w v_w . Rot(a_w, r_w) (v_w = 1 when masks is NULL or masks[w] is NULL) with one
 * ModDown: each rotation's key-switch inner product, plus P * sigma_g(c0) on the Q limbs, is
 * multiplied by its mask in the extended basis Q_l u P; the terms are added there and the
 * sum is brought down once.  ModDown(X + P c) = ModDown(X) + c exactly, so each term
 * contributes Rot(a_w, r_w) up to the one shared rounding. */
static orc_ct *rot_sum_hoisted(orc_ctx *c, int n, orc_ct *const *a, const int64_t *r, const int64_t *const *masks,
                               double ms) {
    int64_t N = c->n;
    int level = a[0]->level, nl = level + 1, K = c->n_p, ne = nl + K;
    int ext[MAXMOD];
    for (int i = 0; i < nl; i++) ext[i] = i;
    for (int i = 0; i < K; i++) ext[nl + i] = c->n_q + i;
    u64 *X0 = calloc((size_t)ne * N, sizeof(u64)), *X1 = calloc((size_t)ne * N, sizeof(u64));
    u64 *u0 = malloc(sizeof(u64) * ne * N), *u1 = malloc(sizeof(u64) * ne * N);
    u64 *p1 = malloc(sizeof(u64) * nl * N), *c0r = malloc(sizeof(u64) * nl * N);
    double scale = 0;
    for (int w = 0; w < n; w++) {
        const int64_t *mask = masks ? masks[w] : NULL;
        u64 g = galois_elt(c, r[w]);
        const swk_t *key = get_key(c, g);
        u64 *d[MAXMOD];
        for (int i = 0; i < nl; i++) {
            automorph(c, limb(a[w], 1, i), p1 + (int64_t)i * N, g, c->mod[i]);
            automorph(c, limb(a[w], 0, i), c0r + (int64_t)i * N, g, c->mod[i]);
            d[i] = p1 + (int64_t)i * N;
        }
        ks_inner(c, level, d, NULL, key, u0, u1);
#pragma omp parallel for num_threads(c->threads)
        for (int ti = 0; ti < ne; ti++) {
            int t = ext[ti];
            u64 q = c->mod[t];
            u64 *x0 = u0 + (int64_t)ti * N, *x1 = u1 + (int64_t)ti * N;
            if (ti < nl) {  /* + P sigma_g(c0) on the Q limbs (P = 0 mod the special primes) */
                u64 P = 1;
                for (int kk = 0; kk < K; kk++) P = mulmod(P, c->mod[c->n_q + kk] % q, q);
                for (int64_t s2 = 0; s2 < N; s2++) x0[s2] = addmod(x0[s2], mulmod(P, c0r[(int64_t)ti * N + s2], q), q);
            }
            if (mask) {
                u64 *m = malloc(sizeof(u64) * N), *tmp = malloc(sizeof(u64) * N);
                for (int64_t s2 = 0; s2 < N; s2++) m[s2] = smod(mask[s2], q);
                orc_poly_mul(c, t, x0, m, tmp);
                memcpy(x0, tmp, sizeof(u64) * N);
                orc_poly_mul(c, t, x1, m, tmp);
                memcpy(x1, tmp, sizeof(u64) * N);
                free(m); free(tmp);
            }
            for (int64_t s2 = 0; s2 < N; s2++) {
                X0[(int64_t)ti * N + s2] = addmod(X0[(int64_t)ti * N + s2], x0[s2], q);
                X1[(int64_t)ti * N + s2] = addmod(X1[(int64_t)ti * N + s2], x1[s2], q);
            }
        }
        c->cnt[C_ROT]++;
        if (mask) c->cnt[C_MULPT]++;
        double sc = a[w]->scale * (mask ? ms : 1.0);
        if (sc > scale) scale = sc;
    }
    orc_ct *out = ct_new(c, level, 1, scale);
    ks_moddown(c, level, X0, out->c[0]);
    ks_moddown(c, level, X1, out->c[1]);
    c->cnt[C_ADD] += n - 1;
    free(X0); free(X1); free(u0); free(u1); free(p1); free(c0r);
    return out;
}

/* HE-LinTrans (Alg. 2) with the baby-step/giant-step split (App. B): the sum over the
 * diagonals d in [dlo, dhi] of mask_d . R(a, unit d), evaluated as
 *   sum_i Rot( sum_j R(mask_{b i + j}, -unit b i) . Rot(a, unit j), unit b i ),
 * masks of 'kind' for side h under the packing iota_beta (every amount times beta); the giant
 * steps share one ModDown under the hoisting flag.  No rescale. */
static orc_ct *lintrans(orc_ctx *c, const orc_ct *a, int kind, int h, int beta, int64_t unit, int dlo, int dhi,
                        int b, int hoist) {
    const double ms = c->scale;
    orc_ct **baby = calloc(b, sizeof(orc_ct *));
    baby[0] = ct_copy(c, a);
    for (int j = 1; j < b; j++) baby[j] = orc_rotate(c, a, (int64_t)beta * unit * j);
    int ngmax = floordiv(dhi, b) - floordiv(dlo, b) + 1, ng = 0;
    orc_ct **gi = calloc(ngmax, sizeof(orc_ct *));
    int64_t *gr = calloc(ngmax, sizeof(int64_t));
    orc_ct *acc = NULL;
    for (int i = floordiv(dlo, b); i <= floordiv(dhi, b); i++) {
        orc_ct *inner = NULL;
        for (int j = 0; j < b; j++) {
            int d = b * i + j;
            if (d < dlo || d > dhi) continue;
            inner = acc_add(c, inner, orc_mul_plain(c, baby[j], get_mask_b(c, kind, h, beta, d, -unit * b * i), ms));
        }
        if (!inner) continue;
        const int64_t r = (int64_t)beta * unit * b * i;
        if (i && hoist) { gi[ng] = inner; gr[ng++] = r; continue; }
        if (i) { orc_ct *t = orc_rotate(c, inner, r); orc_ct_free(inner); inner = t; }
        acc = acc_add(c, acc, inner);
    }
    if (ng) {
        acc = acc_add(c, acc, rot_sum_hoisted(c, ng, gi, gr, NULL, ms));
        while (ng) orc_ct_free(gi[--ng]);
    }
    for (int j = 0; j < b; j++) orc_ct_free(baby[j]);
    free(baby); free(gi); free(gr);
    return acc;
}

static int valid_shape(const orc_ctx *c, int h, int t, int beta) {
    if (h < 1 || (h & (h - 1)) || t < 1 || (t & (t - 1)) || t > h || beta < 1 || (beta & (beta - 1))) return 0;
    return (int64_t)beta * h * h <= c->n / 2;
}

/* HE-MatMult (Alg. 3, t = h) and HE-RMatMult (Alg. 6, App. D: A~ holds h/t vertical copies
 * of a t x h matrix A; Steps 2-3 run t rounds, then the row blocks are folded by rotations
 * t h 2^s so every block holds A B), for beta products packed by iota_beta (App. E). */
orc_ct *orc_matmul_ex(orc_ctx *c, const orc_ct *A, const orc_ct *B, int h, int t, int beta, int mode) {
    if (!valid_shape(c, h, t, beta)) return NULL;
    int lvl = A->level < B->level ? A->level : B->level;
    if (lvl < 3) return NULL;
    orc_ct *a = orc_drop(c, A, lvl), *bb = orc_drop(c, B, lvl);
    const int b = 1 << ((ilog2(h) + 1) / 2);
    const double ms = c->scale;
    const int once = mode & ORC_RELIN_ONCE, hoist = mode & ORC_HOIST_MODDOWN, late = mode & ORC_RESCALE_LATE;

    /* Step 1-1: A0 = U^mu A, diagonals k in (-h, h) at unit 1, then RS */
    orc_ct *A0 = lintrans(c, a, 0, h, beta, 1, 1 - h, h - 1, b, hoist);
    { orc_ct *x = orc_rescale(c, A0); orc_ct_free(A0); A0 = x; }
    /* Step 1-2: B0 = U^zeta B, diagonals h k, k in [0, h), then RS */
    orc_ct *B0 = lintrans(c, bb, 1, h, beta, h, 0, h - 1, b, hoist);
    { orc_ct *x = orc_rescale(c, B0); orc_ct_free(B0); B0 = x; }
    /* B0 is brought to the Step-3 level before its rotations (the late-rescale schedule
     * multiplies one level higher and keeps it) */
    if (!late) { orc_ct *x = orc_drop(c, B0, B0->level - 1); orc_ct_free(B0); B0 = x; }

    /* Steps 2 and 3 over k in [0, t).  The Step-3 sum is taken in blocks k = bg i + j:
     *   sum_i Rot( sum_j Rot(A^(k), -h bg i) . Rot(B0, h j), h bg i ),
     * where Rot(A^(k), -s) = R(v_k, -s) . Rot(A0, k - s) + R(v_(k-h), -s) . Rot(A0, k - h - s).
     * Without the Step-3 flag there is one block (bg = t) and no giant-step rotation, which
     * is Alg. 3's (Alg. 6's) Step 3 as printed.  Rotation amounts are times beta. */
    const int bg = step3_baby(t, mode);
    orc_ct **bj = calloc(bg, sizeof(orc_ct *));
    bj[0] = ct_copy(c, B0);
    for (int j = 1; j < bg; j++) bj[j] = orc_rotate(c, B0, (int64_t)beta * h * j);
    orc_ct **gi = calloc(t / bg + 1, sizeof(orc_ct *));
    int64_t *gr = calloc(t / bg + 1, sizeof(int64_t));
    int ng = 0;
    orc_ct *acc = NULL;
    for (int i = 0; i * bg < t; i++) {
        const int64_t shift = (int64_t)h * bg * i;
        orc_ct *S = NULL;
        for (int j = 0; j < bg; j++) {
            const int k = bg * i + j;
            orc_ct *Ak;
            if (k == 0) {
                Ak = orc_mul_plain(c, A0, get_mask_b(c, 2, h, beta, 0, 0), ms);
            } else if (hoist) {
                const int64_t rr[2] = {beta * (k - shift), beta * (k - h - shift)};
                const int64_t *mm[2] = {get_mask_b(c, 2, h, beta, k, -shift), get_mask_b(c, 3, h, beta, k, -shift)};
                orc_ct *const aa[2] = {A0, A0};
                Ak = rot_sum_hoisted(c, 2, aa, rr, mm, ms);
            } else {
                orc_ct *r1 = orc_rotate(c, A0, beta * (k - shift)), *r2 = orc_rotate(c, A0, beta * (k - h - shift));
                orc_ct *t1 = orc_mul_plain(c, r1, get_mask_b(c, 2, h, beta, k, -shift), ms);
                orc_ct *t2 = orc_mul_plain(c, r2, get_mask_b(c, 3, h, beta, k, -shift), ms);
                Ak = orc_add(c, t1, t2);
                orc_ct_free(r1); orc_ct_free(r2); orc_ct_free(t1); orc_ct_free(t2);
            }
            if (!late) { orc_ct *x = orc_rescale(c, Ak); orc_ct_free(Ak); Ak = x; }
            orc_ct *prod = orc_tensor(c, Ak, bj[j]);
            if (!once) { orc_ct *x = orc_relin(c, prod); orc_ct_free(prod); prod = x; }
            S = acc_add(c, S, prod);
            orc_ct_free(Ak);
        }
        if (once) { orc_ct *x = orc_relin(c, S); orc_ct_free(S); S = x; }
        if (i && hoist) { gi[ng] = S; gr[ng++] = beta * shift; continue; }
        if (i) { orc_ct *x = orc_rotate(c, S, beta * shift); orc_ct_free(S); S = x; }
        acc = acc_add(c, acc, S);
    }
    if (ng) {
        acc = acc_add(c, acc, rot_sum_hoisted(c, ng, gi, gr, NULL, 1.0));
        while (ng) orc_ct_free(gi[--ng]);
    }
    free(gi); free(gr);
    for (int j = 0; j < bg; j++) orc_ct_free(bj[j]);
    free(bj);
    orc_ct *res = orc_rescale(c, acc);
    if (late) { orc_ct *x = orc_rescale(c, res); orc_ct_free(res); res = x; }
    /* Alg. 6's last loop: fold the h/t row blocks of t rows (after the rescales, on fewer limbs) */
    for (int s2 = 0; (t << s2) < h; s2++) {
        orc_ct *r = orc_rotate(c, res, (int64_t)beta * t * h << s2);
        orc_ct *x = orc_add(c, res, r);
        orc_ct_free(r); orc_ct_free(res);
        res = x;
    }
    orc_ct_free(acc); orc_ct_free(A0); orc_ct_free(B0); orc_ct_free(a); orc_ct_free(bb);
    return res;
}

orc_ct *orc_matmul(orc_ctx *c, const orc_ct *A, const orc_ct *B, int h, int mode) {
    return orc_matmul_ex(c, A, B, h, h, 1, mode);
}

/* App. C: A^T = sum_{-h<k<h} t_{(h-1)k} . R(a, (h-1) k), with BSGS (App. B), then RS */
orc_ct *orc_transpose(orc_ctx *c, const orc_ct *A, int h, int beta, int mode) {
    if (!valid_shape(c, h, h, beta) || A->level < 1) return NULL;
    orc_ct *r = lintrans(c, A, 4, h, beta, h - 1, 1 - h, h - 1, 1 << ((ilog2(h) + 1) / 2), mode & ORC_HOIST_MODDOWN);
    orc_ct *x = orc_rescale(c, r);
    orc_ct_free(r);
    return x;
}

/* ------------------------------------------------------------------ */
/* Sec. 4.2: g_d(m) = sum_{i=0..d} 4^-i C(2i,i) m (1-m^2)^i, k compositions   */
/* ------------------------------------------------------------------ */
/* numerators n_i of the m^(2i+1) coefficients over 2^(2d-1) (Sec. 4.2: n / 2^(2d-1)) */
static void gd_numerators(int d, int64_t *num) {
    /* coefficient of m^(2i+1) = sum_{j>=i} 4^-j C(2j,j) C(j,i) (-1)^i ; scale by 4^d */
    for (int i = 0; i <= d; i++) num[i] = 0;
    int64_t C[24][24] = {{0}};
    for (int n = 0; n < 24; n++) { C[n][0] = 1; for (int r = 1; r <= n; r++) C[n][r] = C[n - 1][r - 1] + (r <= n - 1 ? C[n - 1][r] : 0); }
    for (int j = 0; j <= d; j++)
        for (int i = 0; i <= j; i++) {
            int64_t t = C[2 * j][j] * C[j][i] * ((int64_t)1 << (2 * (d - j)));
            num[i] += (i & 1) ? -t : t;
        }
    /* now coefficients are num[i] / 4^d; reduce to denominator 2^(2d-1) (exact: all even) */
    for (int i = 0; i <= d; i++) num[i] /= 2;
}

void orc_gd_numerators(int d, int64_t *num) {
    if (d >= 1 && d <= 7) gd_numerators(d, num);
}

/* the integer constant of x_c = RS(x * K) for the coefficient num / 2^e:
 * K = round(num / 2^e * q_l * ratio), half away from zero, where ratio = (scale x_c must
 * carry) / (scale of x); computed in double in this exact order */
static int64_t scaled_const(int64_t num, int e, u64 ql, double ratio) {
    return llround((double)num / (double)((int64_t)1 << e) * (double)ql * ratio);
}

static orc_ct *mul_rs(orc_ctx *c, const orc_ct *x, const orc_ct *y) {
    int l = x->level < y->level ? x->level : y->level;
    orc_ct *a = orc_drop(c, x, l), *b = orc_drop(c, y, l);
    orc_ct *p = orc_mul(c, a, b);
    orc_ct *r = orc_rescale(c, p);
    orc_ct_free(a); orc_ct_free(b); orc_ct_free(p);
    return r;
}

/* g_d(x) with every term landing on the scale 'target' */
static orc_ct *eval_gd(orc_ctx *c, const orc_ct *x, int d, double target) {
    int64_t num[16];
    gd_numerators(d, num);
    int e = 2 * d - 1;
    orc_ct *pw[8] = {0}; /* pw[b] = x^(2^(b+1)) */
    int nb = 0;
    while ((1 << nb) <= d) nb++;
    for (int b = 0; b < nb; b++) pw[b] = mul_rs(c, b ? pw[b - 1] : x, b ? pw[b - 1] : x);
    orc_ct *y = NULL;
    u64 ql = c->mod[x->level];
    for (int i = 0; i <= d; i++) {
        /* scale matching: the finished term c_i x^(2i+1) must land exactly on the scale of
         * x, so x_c has to carry the scale 'need' that the products with the powers and
         * their rescales then bring back to it; the ratio need / scale(x) is folded into
         * the integer constant.  All terms of the sum then share one scale. */
        double need = target;
        int lv = x->level - 1;
        for (int b = 0; b < nb; b++)
            if ((i >> b) & 1) {
                int l = lv < pw[b]->level ? lv : pw[b]->level;
                need = need * (double)c->mod[l] / pw[b]->scale;
                lv = l - 1;
            }
        orc_ct *t = orc_mul_int(c, x, scaled_const(num[i], e, ql, need / x->scale));
        orc_ct *term = orc_rescale(c, t);
        term->scale = need; /* value c_i x carried at scale need (K q_l^-1 rides with it) */
        orc_ct_free(t);
        for (int b = 0; b < nb; b++)
            if ((i >> b) & 1) { orc_ct *u = mul_rs(c, term, pw[b]); orc_ct_free(term); term = u; }
        y = acc_add(c, y, term);
    }
    for (int b = 0; b < nb; b++) orc_ct_free(pw[b]);
    return y;
}

orc_ct *orc_sign(orc_ctx *c, const orc_ct *x, int d, int k, int relu) {
    if (d < 1 || d > 7 || k < 0) return NULL;
    int nb = 0;
    while ((1 << nb) <= d) nb++;
    if (x->level < k * (nb + 1) + (relu ? 1 : 0)) return NULL;
    orc_ct *cur = ct_copy(c, x);
    for (int it = 0; it < k; it++) {
        /* each composition returns its input's scale; for ReLU the last one lands on the
         * prime q_l that the product x g rescales by, so that x g comes out exactly at the
         * scale of x and the sum x + x g adds equal scales */
        double target = cur->scale;
        if (relu && it == k - 1) target = (double)c->mod[cur->level - (nb + 1)];
        orc_ct *t = eval_gd(c, cur, d, target);
        orc_ct_free(cur);
        cur = t;
    }
    if (!relu) return cur;
    orc_ct *r = mul_rs(c, x, cur);
    orc_ct *xd = orc_drop(c, x, r->level);
    orc_ct *y = orc_add(c, r, xd);
    y->scale *= 2.0; /* (x + x g) / 2 */
    orc_ct_free(cur); orc_ct_free(r); orc_ct_free(xd);
    return y;
}

/* Alg. 5: AppMax(a, b) = (a + b) / 2 + (a - b) / 2 . g_d^(k)(a - b), evaluated as
 * ((a + b) + m g_d^(k)(m)) with m = a - b and the halving kept in the scale; the last
 * composition lands on the prime the product m g rescales by, so both terms of the sum share
 * one scale (as for ReLU, the case b = 0) */
orc_ct *orc_appmax(orc_ctx *c, const orc_ct *a, const orc_ct *b, int d, int k) {
    if (d < 1 || d > 7 || k < 1) return NULL;
    int nb = 0;
    while ((1 << nb) <= d) nb++;
    int lvl = a->level < b->level ? a->level : b->level;
    if (lvl < k * (nb + 1) + 1) return NULL;
    orc_ct *m = orc_sub(c, a, b), *s = orc_add(c, a, b);
    orc_ct *cur = ct_copy(c, m);
    for (int it = 0; it < k; it++) {
        double target = cur->scale;
        if (it == k - 1) target = (double)c->mod[cur->level - (nb + 1)];
        orc_ct *t = eval_gd(c, cur, d, target);
        orc_ct_free(cur);
        cur = t;
    }
    orc_ct *r = mul_rs(c, m, cur);
    orc_ct *sd = orc_drop(c, s, r->level);
    orc_ct *y = orc_add(c, r, sd);
    y->scale *= 2.0;
    orc_ct_free(m); orc_ct_free(s); orc_ct_free(cur); orc_ct_free(r); orc_ct_free(sd);
    return y;
}

/* 2 x 2 max pooling of a row-major h x h matrix: AppMax over horizontal neighbours
 * (rotation by 1), then over vertical neighbours (rotation by h); entry (i, j) holds the
 * maximum of the window with top-left corner (i, j) (cyclically at the last row/column) */
orc_ct *orc_maxpool2(orc_ctx *c, const orc_ct *x, int h, int d, int k) {
    orc_ct *r1 = orc_rotate(c, x, 1);
    orc_ct *m1 = orc_appmax(c, x, r1, d, k);
    orc_ct_free(r1);
    if (!m1) return NULL;
    orc_ct *r2 = orc_rotate(c, m1, h);
    orc_ct *m2 = orc_appmax(c, m1, r2, d, k);
    orc_ct_free(r2); orc_ct_free(m1);
    return m2;
}

/* Alg. 6, aggregation: W - (eta / (B N)) sum_i G_i; the constant is a plaintext encoded at
 * the scale q_l of the prime the rescale removes (one Mul_pt and one rescale), so the product
 * returns exactly to the gradients' scale; W is dropped to the result's level */
orc_ct *orc_fl_update(orc_ctx *c, const orc_ct *w, orc_ct *const *g, int n, double coeff) {
    if (n < 1) return NULL;
    orc_ct *sum = ct_copy(c, g[0]);
    for (int i = 1; i < n; i++) sum = acc_add(c, sum, ct_copy(c, g[i]));
    if (sum->level < 1) { orc_ct_free(sum); return NULL; }
    int64_t *pt = malloc(sizeof(int64_t) * c->n);
    const double ql = (double)c->mod[sum->level];
    orc_encode(c, &coeff, 1, ql, pt);
    orc_ct *t = orc_mul_plain(c, sum, pt, ql);
    orc_ct *u = orc_rescale(c, t);
    orc_ct *wd = orc_drop(c, w, u->level < w->level ? u->level : w->level);
    orc_ct *r = orc_sub(c, wd, u);
    free(pt); orc_ct_free(sum); orc_ct_free(t); orc_ct_free(u); orc_ct_free(wd);
    return r;
}
