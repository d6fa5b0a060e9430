/*
 * he.h -- C ABI of libhe: packed ciphertext x ciphertext matrix products over
 * RNS-CKKS on one MI355X (gfx950), after Hercules (arXiv 2207.04620).
 *
 * Plain pointers and sizes only.  Every call returns an he_status; out-parameters
 * are written only on HE_OK.  A context is used by one host thread at a time.
 * Ciphertexts live in device memory, in the evaluation (NTT) domain, as one block
 * u64[deg+1][level+1][N]; the caller owns every he_ct* it receives and releases it
 * with he_ct_free before destroying the context.  Work is issued on the context's
 * HIP stream and is asynchronous unless a call says it synchronizes.
 *
 * Conventions fixed where the paper is silent (readings):
 *  - ring Z_Q[X]/(X^N + 1), Q = q_0 ... q_L (Sec. 2.2), special modulus P for
 *    hybrid key switching with digits of 'alpha' Q-limbs;
 *  - primes: for each requested bit size, Q list then P list, the largest unused
 *    prime below 2^bits that is 1 mod 2N;
 *  - slot j of a plaintext is its value at zeta^(5^j), zeta = exp(i pi / N);
 *    a vector shorter than N/2 slots is replicated to fill them (the packed
 *    product treats rotation as cyclic modulo h^2, Sec. 3.2 and 3.4);
 *  - Rot(c, k) is the left rotation R(m, k)[t] = m[t + k] of Sec. 3.2;
 *  - randomness: ChaCha20 (RFC 8439) keyed by the 64-bit seed; stream purposes
 *    1 secret, 2 public-key a, 3 public-key e, 4 switching-key a, 5 switching-key e,
 *    6/7/8 encryption v/e0/e1; ternary secret, Gaussian sigma 3.2 on [-19, 19].
 */
#ifndef HE_H
#define HE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct he_ctx he_ctx;
typedef struct he_ct he_ct;

typedef enum {
    HE_OK = 0,
    HE_EINVAL = 1,      /* bad argument (null pointer, size mismatch, bad parameter set) */
    HE_ENOMEM = 2,      /* device or host allocation failed, or admission budget exceeded */
    HE_ELEVEL = 3,      /* ciphertext level below the depth of the operation */
    HE_ESCALE = 4,      /* scale out of range */
    HE_EKEY = 5,        /* rotation key not generated */
    HE_ESHAPE = 6,      /* h not a power of two, or h^2 > N/2 */
    HE_EMISMATCH = 7,   /* handles from different contexts, or degrees that do not fit */
    HE_EDEVICE = 8,     /* HIP runtime error */
    HE_EUNSUPPORTED = 9
} he_status;

/* Device hooks.  stream: a hipStream_t (e.g. torch.cuda.current_stream().cuda_stream),
 * or NULL for a stream the context creates.  alloc/free: optional device allocator
 * (NULL: hipMalloc/hipFree behind a size-bucketed cache owned by the context). */
typedef struct {
    void *stream;
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *user;
} he_device;

/* Schedule flags of the packed product (Alg. 3).  Every combination computes A B at the
 * same depth (three levels) with the same rotations; they differ only in where rounding
 * happens, so each is its own bit-exact reference. */
#define HE_SCHED_RELIN_EACH 0u    /* relinearise every Step-3 product (Mul_ct of Fig. 1) */
#define HE_SCHED_RELIN_ONCE 1u    /* accumulate degree-2 products, relinearise once */
#define HE_SCHED_HOIST_MODDOWN 2u /* sums of rotations share one ModDown, their terms formed in
                                   * the extended basis Q_l P: Step 2's v_k . Rot(A0,k) +
                                   * v_(k-h) . Rot(A0,k-h), the giant-step sums of Steps 1-1 and
                                   * 1-2, and of Step 3 under HE_SCHED_STEP3_BSGS */
#define HE_SCHED_RESCALE_LATE 4u  /* Step 2: A^(k) kept unrescaled; Step 3 multiplies one level
                                   * higher and the sum is rescaled twice */
#define HE_SCHED_STEP3_BSGS 8u    /* Step 3 as sum_i Rot(sum_j Rot(A^(bg i+j), -h bg i) . Rot(B0, h j),
                                   * h bg i): bg - 1 + h/bg - 1 rotations on the B side instead of
                                   * h - 1 (bg = 2^ceil((log2 h + 1)/2)); the rotation keys and
                                   * masks made for each h follow the schedule */
#define HE_SCHED_ALL 15u

typedef struct {
    uint32_t log_n;          /* ring degree N = 2^log_n, 8 <= log_n <= 17 */
    uint32_t n_q;            /* Q limbs (top level L = n_q - 1) */
    const uint32_t *q_bits;  /* bit size of each Q prime, q_0 first (<= 60) */
    uint32_t n_p;            /* special primes K */
    const uint32_t *p_bits;  /* bit size of each special prime (<= 60) */
    uint32_t alpha;          /* Q limbs per key-switching digit; dnum = ceil(n_q/alpha).  The
                              * key-switching noise scales with (largest digit modulus) / P, so
                              * P should be at least as wide as a digit */
    double log_scale;        /* scale Delta = 2^log_scale of fresh ciphertexts and masks */
    uint64_t seed;           /* ChaCha20 key */
    uint32_t n_h;            /* matrix sides whose rotation keys and masks are made at creation */
    const uint32_t *h_list;
    uint32_t schedule;       /* OR of HE_SCHED_* flags; other bits are HE_EINVAL */
} he_params;

/* Context: primes, twiddles, secret/public/relinearisation keys, rotation keys and
 * diagonal masks for every h in h_list (Sec. 3.5-3.6 and App. B).  Synchronizes. */
he_status he_ctx_create(const he_params *params, const he_device *dev, he_ctx **out);
void he_ctx_destroy(he_ctx *ctx);
/* primes (Q then P) into out[0 .. n_q+n_p) */
he_status he_ctx_moduli(const he_ctx *ctx, uint64_t *out, size_t n);
/* blocks the host until all queued work on the context stream is done */
he_status he_sync(he_ctx *ctx);
/* op counters: rotations, key switches, Mul_pt, Mul_ct, Add, RS */
he_status he_counters(const he_ctx *ctx, int64_t out[6], int reset);
/* device bytes held by keys + masks, and by the allocation cache */
he_status he_memory(const he_ctx *ctx, uint64_t *keys_bytes, uint64_t *pool_bytes);

/* Cap on the device bytes the context's allocation cache may hold (keys, masks, ciphertexts and
 * temporaries alike; 0: no cap).  Setting a cap below the bytes held returns the cached blocks to
 * the device (after the queued work is done).  An allocation beyond the cap, once the cache is
 * trimmed, fails and the call returns HE_ENOMEM (a serving cohort fails with HE_ENOMEM and the
 * server goes on).  Synchronizes. */
he_status he_pool_limit(he_ctx *ctx, uint64_t bytes);
/* bytes of the allocation cache in use now and the largest in-use figure since the last reset
 * (reset != 0 restarts it from the current figure) */
he_status he_pool_stats(he_ctx *ctx, uint64_t *in_use, uint64_t *peak, int reset);

/* Ecd + Enc (Fig. 1 items 3 and 5): n_vals values (n_vals divides N/2) replicated to
 * N/2 slots, encoded at Delta (exact rounding, computed in 113-bit floating point),
 * encrypted with the public key at 'level' (<= L) using stream index 'nonce'. */
he_status he_encrypt(he_ctx *ctx, const double *vals, size_t n_vals, uint32_t level, uint64_t nonce,
                     he_ct **out);
/* Enc of an already-encoded plaintext: N signed integer coefficients at 'scale' */
he_status he_encrypt_coeffs(he_ctx *ctx, const int64_t *coeffs, uint32_t level, double scale, uint64_t nonce,
                            he_ct **out);
/* single-key Dec + Dcd (Fig. 1 items 4 and 6): first n_out slot values (real parts).
 * The plaintext must be below q_0 q_1 / 2 in magnitude.  Synchronizes. */
he_status he_decrypt(he_ctx *ctx, const he_ct *ct, double *out, size_t n_out);
/* Dec only: the N centered plaintext coefficients (unscaled).  Synchronizes. */
he_status he_decrypt_coeffs(he_ctx *ctx, const he_ct *ct, double *out, size_t n);
/* Ecd only: N integer coefficients of the encoding at 'scale' */
he_status he_encode(he_ctx *ctx, const double *vals, size_t n_vals, double scale, int64_t *out);

void he_ct_free(he_ct *ct);
he_status he_ct_info(const he_ct *ct, uint32_t *level, uint32_t *degree, double *scale);
/* coefficient-domain residues, u64[deg+1][level+1][N] with values in [0, q_i). Synchronizes. */
he_status he_ct_export(he_ctx *ctx, const he_ct *ct, uint64_t *buf, size_t n);
he_status he_ct_import(he_ctx *ctx, const uint64_t *buf, size_t n, uint32_t level, uint32_t degree, double scale,
                       he_ct **out);

/* Fig. 1 operations.  Add/Sub: level min, scale max.  Mul_pt: coeffs are an encoded
 * plaintext at pt_scale.  Mul: tensor + relinearisation.  RS: divide by the last prime.
 * Rot: left rotation by k (Sec. 3.2), needs the key for 5^k mod 2N (HE_EKEY). */
he_status he_add(he_ctx *ctx, const he_ct *a, const he_ct *b, he_ct **out);
he_status he_sub(he_ctx *ctx, const he_ct *a, const he_ct *b, he_ct **out);
he_status he_drop(he_ctx *ctx, const he_ct *a, uint32_t level, he_ct **out);
he_status he_mul_plain(he_ctx *ctx, const he_ct *a, const int64_t *coeffs, double pt_scale, he_ct **out);
he_status he_mul_int(he_ctx *ctx, const he_ct *a, int64_t k, he_ct **out);
he_status he_tensor(he_ctx *ctx, const he_ct *a, const he_ct *b, he_ct **out);
he_status he_relin(he_ctx *ctx, const he_ct *a, he_ct **out);
he_status he_mul(he_ctx *ctx, const he_ct *a, const he_ct *b, he_ct **out);
he_status he_rescale(he_ctx *ctx, const he_ct *a, he_ct **out);
he_status he_rotate(he_ctx *ctx, const he_ct *a, int64_t k, he_ct **out);
/* rotation key for amount k (made on demand; no-op when it exists) */
he_status he_gen_rotation_key(he_ctx *ctx, int64_t k);
/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops
 * and harnesses that forbid allocation): Rot(a, k) as he_rotate computes it, bit for bit, on
 * caller memory.  in: device address of the two polynomials of a ciphertext at 'level',
 * u64[2][level+1][N], every limb in the evaluation domain of he_ntt (forward, limb i modulo
 * prime i); out: device address of the result in the same layout, not overlapping in.  The
 * call allocates nothing: its temporaries live in a static device scratch of 64 MiB, one copy
 * per device, held until the process ends, and shared by every call on that device, so calls
 * on one device that overlap in time (other contexts, other streams) race; calls on one
 * stream are ordered.  Sizes are bounded by the scratch: (beta (level + 1 + K) + 2 (level + 1
 * + K) + 2 (level + 1)) N words must fit (beta the digits at that level, K the special
 * primes), else HE_ENOMEM with a message on stderr (every level of an N = 2^15, 14 + 4 limb
 * ring fits).  The key for 5^k mod 2N must exist (HE_EKEY; he_gen_rotation_key makes it,
 * allocating).  HE_ELEVEL for a level above the top, HE_EINVAL for null or overlapping
 * buffers, HE_EMISMATCH when the current device is not the context's.  Asynchronous on the
 * context stream. */
he_status he_rotate_noalloc(he_ctx *ctx, const uint64_t *in, uint32_t level, int64_t k, uint64_t *out);

/* HE-MatMult (Alg. 3 with the baby-step/giant-step Steps 1-1/1-2 of App. B): A and B
 * encrypt row-major h x h matrices (Sec. 3.4) replicated over the slots; the result
 * encrypts A B three levels below min(level A, level B).  HE_ESHAPE if h is not a
 * power of two or h^2 > N/2; HE_ELEVEL if the level is below 3. */
he_status he_matmul(he_ctx *ctx, const he_ct *a, const he_ct *b, uint32_t h, he_ct **out);
/* n independent products C[i] = A[i] B[i] of sides h[i] (mixed h and levels allowed),
 * scheduled together so that each switching key is streamed once per rotation round
 * for all members.  Results are bit-identical to he_matmul on each pair. */
he_status he_matmul_batch(he_ctx *ctx, size_t n, const he_ct *const *a, const he_ct *const *b,
                          const uint32_t *h, he_ct **out);

/* The batched product captured once into a HIP graph and replayed: he_graph_launch recomputes
 * every out[i] = a[i] b[i] from the inputs' current contents with the launches and copies of one
 * he_matmul_batch call, without host-side launch work (bit-identical to he_matmul_batch).  The
 * graph owns every device buffer its replays touch (the product's temporaries, taken on the
 * graph's own account during the capture) and keeps the inputs and outputs alive until
 * he_graph_destroy; out[i] are ordinary handles the caller frees.  The capture runs the product
 * once (the first result is in out) after making its keys and masks; it is refused
 * (HE_EUNSUPPORTED) while launch timing is on.  Launches are asynchronous on the context stream;
 * he_graph_destroy waits for queued replays. */
typedef struct he_graph he_graph;
he_status he_matmul_batch_capture(he_ctx *ctx, size_t n, const he_ct *const *a, const he_ct *const *b,
                                  const uint32_t *h, he_graph **graph, he_ct **out);
he_status he_graph_launch(he_graph *graph);
/* nodes of the graph and device bytes it owns */
he_status he_graph_info(const he_graph *graph, size_t *nodes, uint64_t *bytes);
void he_graph_destroy(he_graph *graph);

/* Shape of a packed product (App. D, App. E).  t = h: the square product of he_matmul.
 * t < h (t divides h): HE-RMatMult (Alg. 6) of a t x h matrix A by an h x h matrix B; the
 * caller encrypts A~ = h/t vertical copies of A as an h x h matrix, and the result encrypts
 * h/t vertical copies of the t x h product (Steps 2-3 run t rounds, then log2(h/t) fold
 * rotations by t h 2^s).  beta > 1: beta matrix pairs per ciphertext pair under the packing
 * iota_beta (matrix m's entry (i, j) at slot beta (h i + j) + m, the beta h^2 vector
 * replicated over the slots); every rotation amount is times beta, so one product computes
 * beta products at the cost of one.  h, t, beta powers of two, beta h^2 <= N/2, else
 * HE_ESHAPE. */
typedef struct {
    uint32_t h, t, beta;
} he_mat_shape;
/* The packing iota_beta itself (App. E), a host-side layout step before he_encrypt: mats[m]
 * points to matrix m's n entries in row-major order (n = h h, or t h for the row-block operand),
 * m < beta; out (beta n doubles, caller-owned) receives entry e of matrix m at position
 * beta e + m.  Host memory only, no device work.  HE_EINVAL on null pointers, beta = 0 or
 * n = 0. */
he_status he_pack_beta(size_t beta, size_t n, const double *const *mats, double *out);
he_status he_matmul_ex(he_ctx *ctx, const he_ct *a, const he_ct *b, const he_mat_shape *shape, he_ct **out);
/* n products of mixed shapes and levels, grouped by (shape, level) into lockstep groups;
 * bit-identical to he_matmul_ex on each pair */
he_status he_matmul_batch_ex(he_ctx *ctx, size_t n, const he_ct *const *a, const he_ct *const *b,
                             const he_mat_shape *shapes, he_ct **out);
/* Matrix transposition on packed ciphertexts (App. C): A^T of each of the beta packed h x h
 * matrices, as the linear transform over the 2h - 1 diagonals (h-1) k with the baby-step/
 * giant-step split; one level (a Mul_pt and a rescale).  Keys and masks for (h, beta) are made
 * on first use.  HE_ESHAPE as for he_matmul_ex; HE_ELEVEL at level 0. */
he_status he_transpose(he_ctx *ctx, const he_ct *a, uint32_t h, uint32_t beta, he_ct **out);
he_status he_transpose_batch(he_ctx *ctx, size_t n, const he_ct *const *a, uint32_t h, uint32_t beta,
                             he_ct **out);

/* Scheduling knobs of the lockstep products; results never depend on them.  pair_batch:
 * rotation sets (Step-2 mask pairs, baby rotations) that share one key-switch inner-product
 * launch and one ModDown launch (1..16); max_group: members per lockstep group (1..256);
 * overlap (0 or 1): the next Step-2 pair group's inner products run on the context's second
 * stream while the current group's ModDown runs on the context stream; concurrent_groups (0 or
 * 1): the (shape, level) groups of a batch with several of them are spread over the two
 * streams (the autotuner leaves it as set). */
typedef struct {
    uint32_t pair_batch;
    uint32_t max_group;
    uint32_t overlap;
    uint32_t concurrent_groups;
} he_tuning;
he_status he_tuning_get(const he_ctx *ctx, he_tuning *out);
he_status he_tuning_set(he_ctx *ctx, const he_tuning *t);
/* Autotuner: times he_matmul_batch of 'batch' h x h pairs at 'level' on the device under each
 * candidate (the context's current setting first, then pair_batch 1, 2, 4, 8 with max_group =
 * batch, and batch / 2 when batch >= 16; then overlap on for the best of those; the best of two
 * timed runs each after a warm-up), applies the fastest to the context (a later candidate must
 * be 1 % faster to displace an earlier one) and caches it per (N, limbs, alpha, schedule, h, level, batch, device) in the
 * process and, when cache_path is set, in that text file (a line already there is used without
 * timing).  report: optional JSON of the candidates' times and the
 * choice, truncated to report_n bytes.  HE_ESHAPE / HE_ELEVEL as for he_matmul.  Synchronizes. */
he_status he_autotune(he_ctx *ctx, uint32_t h, uint32_t level, uint32_t batch, const char *cache_path,
                      he_tuning *out, char *report, size_t report_n);

/* Composite sign approximation g_d^(k) (Sec. 4.2; Alg. 5 for ReLU):
 * mode 0: g_d applied k times; mode 1: ReLU(x) = (x + x g_d^(k)(x)) / 2.
 * Depth per composition 1 + floor(log2 d) + 1; HE_ELEVEL if the level is too low. */
he_status he_sign_approx(he_ctx *ctx, const he_ct *x, uint32_t d, uint32_t k, uint32_t mode, he_ct **out);
/* n independent sign/ReLU evaluations run in lockstep groups of equal level; each
 * result is bit-identical to he_sign_approx on that input. */
he_status he_sign_approx_batch(he_ctx *ctx, size_t n, const he_ct *const *x, uint32_t d, uint32_t k, uint32_t mode,
                               he_ct **out);

/* Limb-batched negacyclic NTT on device memory: n_limbs limbs of N u64 each at
 * 'dev_ptr' (device pointer), limb i reduced modulo prime index mod_idx[i] (host array).
 * Forward output order: position j holds a(psi^(2 bitrev(j) + 1)), psi the smallest
 * primitive 2N-th root of unity mod q.  inverse = 1 undoes it. */
he_status he_ntt(he_ctx *ctx, uint64_t *dev_ptr, uint32_t n_limbs, const uint32_t *mod_idx, int inverse);

/* Serving: a host thread admits requests by device-memory footprint and runs them with
 * continuous batching; each request's result is the same as running it alone.  Rounds are
 * pipelined (the issuing thread never synchronises the stream) and a completion thread hands
 * each cohort's results out when its own kernels are done.  Admission footprints are measured:
 * the largest per-member figure of the allocation cache seen while a cohort of that type ran
 * (bytes held plus the transient peak of each phase); a type not yet measured is admitted on a
 * conservative estimate. */
typedef struct he_server he_server;
typedef struct {
    uint64_t mem_budget_bytes; /* admission budget for in-flight requests (0: no limit) */
    uint32_t max_batch;        /* requests merged into one lockstep cohort (0: 32) */
    uint32_t min_batch;        /* a new cohort waits for this many compatible requests ... */
    uint32_t max_wait_us;      /* ... or until its oldest request has waited this long (0: no wait) */
} he_serve_config;
#define HE_REQ_MATMUL 0u
#define HE_REQ_SIGN 1u
#define HE_REQ_POWER 2u /* x^k for k = 2 (one Mul_ct and RS, depth 1) or 3 (x . x^2, depth 2) */
typedef struct {
    uint32_t op;      /* HE_REQ_MATMUL, HE_REQ_SIGN or HE_REQ_POWER */
    uint32_t h;       /* matmul side */
    uint32_t d, k;    /* sign degree parameter and compositions; the power's exponent (k) */
    uint32_t mode;    /* sign mode */
    const he_ct *a;   /* inputs (borrowed until the request completes) */
    const he_ct *b;
} he_request;
he_status he_serve_start(he_ctx *ctx, const he_serve_config *cfg, he_server **out);
/* HE_ENOMEM when the request alone exceeds the budget */
he_status he_serve_submit(he_server *s, const he_request *req, uint64_t *ticket);
/* done = 1 and *result set when finished (caller owns it); status of the request in *req_status */
he_status he_serve_poll(he_server *s, uint64_t ticket, int *done, he_ct **result, he_status *req_status,
                        double *latency_s);
he_status he_serve_stop(he_server *s);
/* bytes admitted and not yet completed, the largest measured cohort footprint, the allocation
 * cache's largest in-use byte count seen while serving (keys, masks and inputs included), and the
 * measured per-member footprints of up to n_types request types (n_measured: how many types are
 * measured) */
he_status he_serve_stats(he_server *s, uint64_t *inflight_bytes, uint64_t *peak_cohort_bytes, uint64_t *peak_in_use,
                         size_t n_types, uint64_t *type_bytes, size_t *n_measured);

/* AppMax (Alg. 5): max(a, b) ~ (a + b)/2 + (a - b)/2 . g_d^(k)(a - b), evaluated as
 * ((a + b) + m g_d^(k)(m)) with m = a - b and the halving kept in the scale (ReLU is the case
 * b = 0).  |a - b| <= 1 is the input range of g_d.  Depth k (1 + floor(log2 d) + 1) + 1 below
 * min(level a, level b); HE_ELEVEL if less remains, HE_EINVAL for d outside [1, 7] or k = 0. */
he_status he_appmax(he_ctx *ctx, const he_ct *a, const he_ct *b, uint32_t d, uint32_t k, he_ct **out);
he_status he_appmax_batch(he_ctx *ctx, size_t n, const he_ct *const *a, const he_ct *const *b, uint32_t d,
                          uint32_t k, he_ct **out);
/* 2 x 2 max pooling of a packed row-major h x h matrix: AppMax over horizontal neighbours
 * (rotation by 1), then over vertical neighbours (rotation by h); entry (i, j) of the result
 * holds the maximum of the window with top-left corner (i, j) (cyclic at the last row and
 * column; the stride-2 pooling outputs are the entries with even i and j).  Twice the depth of
 * he_appmax; rotation keys for 1 and h are made on first use. */
he_status he_maxpool2(he_ctx *ctx, const he_ct *x, uint32_t h, uint32_t d, uint32_t k, he_ct **out);
he_status he_maxpool2_batch(he_ctx *ctx, size_t n, const he_ct *const *x, uint32_t h, uint32_t d, uint32_t k,
                            he_ct **out);
/* Aggregation step of federated training (Alg. 6): W - coeff . sum_i G_i with
 * coeff = eta / (B N).  The n gradients (at any levels; the sum is taken at the lowest) are
 * added in one pass, multiplied by coeff encoded at the scale q_l of the prime the rescale
 * removes (Mul_pt; the product returns exactly to the gradients' scale), rescaled, and
 * subtracted from W dropped to that level: one level below the gradients. */
he_status he_fl_update(he_ctx *ctx, const he_ct *w, size_t n, const he_ct *const *grads, double coeff, he_ct **out);

/* Launch timing: with profiling on, every kernel launch (or, with 'only' naming one kernel
 * kind of the report, e.g. "ntt_fwd_rows", every launch of that kind) is bracketed by HIP
 * events on its stream.  The report (JSON text, NUL-terminated, truncated to n bytes) gives
 * per kernel kind the launch count, summed duration in ms and algorithmic bytes (operands
 * read once, results written once); reading it synchronizes and clears the records.
 * An unknown kind name is HE_EINVAL.  The setting is process-wide. */
he_status he_profile_enable(he_ctx *ctx, int on, const char *only);
he_status he_profile_report(he_ctx *ctx, char *buf, size_t n);

/* Error-path testing: the n-th kernel launch from now on in this process (n >= 1) fails before
 * anything is queued, and the call that issued it returns HE_EDEVICE (a serving cohort fails
 * with HE_EDEVICE and the server goes on).  No kernel runs for the failed launch, so the device
 * is never at fault.  n = 0 disarms.  Every launch is also checked as it is issued: a launch the
 * runtime rejects is HE_EDEVICE from the call that issued it. */
he_status he_debug_fail_launch(uint64_t n);

/* Streaming-bandwidth probe (a measurement aid; no operation of the method uses it): one pass of
 * 16-byte nontemporal accesses.  After one untimed launch, 'reps' launches of one access mix
 * over caller device buffers, timed with HIP events on the context stream (the call
 * synchronizes); *ms_per_rep is the mean time of one.
 * pattern 0 reads n_words words of a and writes one pair of partial sums per 4096 words
 * (c must hold 2 ceil(n_words / 4096) words; their sum equals the sum of a's words mod 2^64):
 * 8 n_words bytes from HBM.
 * pattern 1: c = a (16 n_words bytes); pattern 2: c = a + b word-wise mod 2^64 (24 n_words
 * bytes; the mix of the ModDown row pass: two read streams, one write stream).  Buffers are
 * 16-byte aligned device memory of n_words words (even); HE_EINVAL otherwise. */
he_status he_stream_probe(he_ctx *ctx, uint32_t pattern, const uint64_t *a, const uint64_t *b, uint64_t *c,
                          uint64_t n_words, uint32_t reps, double *ms_per_rep);

const char *he_status_string(he_status s);

#ifdef __cplusplus
}
#endif
#endif
