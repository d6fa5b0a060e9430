// HIP kernels for gfx950: limb-batched negacyclic NTT staged in LDS, centered fast
// base conversion, key-switch inner product with fused automorphism, rescale,
// tensor product, mask multiply-accumulate and the ChaCha20 samplers.
//
// The ring is Z_q[X]/(X^N+1) (Sec. 2.2 of the paper); the transforms and the
// RNS-CKKS internals are not described by the paper and follow the published
// constructions named at each kernel.
#include "kernels.hpp"
#include <atomic>
#include <cstring>
#include <stdexcept>
#include <type_traits>

#include <cstdio>
#include <string>
#include <vector>

#define TPB 256
#define NTT_E 2048  // elements held in LDS by one NTT block (16 KiB)

static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
static bool misaligned16(const void* p) { return ((uintptr_t)p & 15) != 0; }

// ------------------------------------------------------------------ launch timing
// Optional HIP-event timing of every launch (he_profile_enable): a pair of events on
// the launch stream brackets each kernel; durations are read back on report.  The
// byte count attached to a launch is its algorithmic traffic: each operand read once
// and each result written once (tables of constants excluded).
static const char* const kProfNames[PK_COUNT] = {
    "ntt_fwd_cols", "ntt_fwd_rows", "ntt_inv_rows", "ntt_inv_cols", "baseconv", "inner_product",
    "moddown_combine", "rescale_spread", "rescale_combine", "tensor", "mask_mac", "automorph", "elementwise",
    "conv_ntt_cols", "copy"};
struct ProfRec {
    int kind;
    hipEvent_t a, b;
    double bytes, ops, fp_ops;
};
static bool g_prof_on = false;
static int g_prof_only = -1;  // -1: every kind, else the one kind that is timed
static std::vector<ProfRec> g_prof;
static std::vector<hipEvent_t> g_ev_free;

static hipEvent_t ev_get() {
    if (!g_ev_free.empty()) {
        hipEvent_t e = g_ev_free.back();
        g_ev_free.pop_back();
        return e;
    }
    hipEvent_t e;
    (void)hipEventCreate(&e);
    return e;
}

struct ProfScope {
    int kind;
    double bytes, ops, fp_ops;
    hipStream_t st;
    hipEvent_t a = nullptr;
    // ops: butterflies of the launch, fp_ops of them FP64
    ProfScope(int k, double b, hipStream_t s, double o = 0, double fo = 0)
        : kind(k), bytes(b), ops(o), fp_ops(fo), st(s) {
        if (g_prof_on && (g_prof_only < 0 || g_prof_only == k)) {
            a = ev_get();
            (void)hipEventRecord(a, st);
        }
    }
    ~ProfScope() {
        if (g_prof_on && a) {
            hipEvent_t b = ev_get();
            (void)hipEventRecord(b, st);
            g_prof.push_back({kind, a, b, bytes, ops, fp_ops});
        }
    }
};

// ------------------------------------------------------------------ launch checks
static std::atomic<uint64_t> g_inject{0};  // launches until the injected failure (0: none)

void launch_inject(uint64_t n) { g_inject.store(n); }

void launch_gate(const char* what) {
    (void)hipGetLastError();  // the launch's own status is read right after it
    uint64_t n = g_inject.load();
    while (n) {
        if (g_inject.compare_exchange_weak(n, n - 1)) {
            if (n == 1) throw LaunchError{hipErrorLaunchFailure, what};
            break;
        }
    }
}

void launch_check(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        fprintf(stderr, "libhe: launch of %s failed: %s\n", what, hipGetErrorString(e));
        throw LaunchError{e, what};
    }
}

bool prof_active() { return g_prof_on; }

bool prof_enable(bool on, const char* only) {
    int k = -1;
    if (only) {
        for (int i = 0; i < PK_COUNT; ++i)
            if (!strcmp(only, kProfNames[i])) k = i;
        if (k < 0) return false;
    }
    g_prof_on = on;
    g_prof_only = k;
    return true;
}

std::string prof_report() {
    double ms[PK_COUNT] = {0}, by[PK_COUNT] = {0}, op[PK_COUNT] = {0}, fo[PK_COUNT] = {0};
    long cnt[PK_COUNT] = {0};
    for (auto& r : g_prof) {
        (void)hipEventSynchronize(r.b);
        float t = 0;
        (void)hipEventElapsedTime(&t, r.a, r.b);
        ms[r.kind] += t;
        by[r.kind] += r.bytes;
        op[r.kind] += r.ops;
        fo[r.kind] += r.fp_ops;
        cnt[r.kind]++;
        g_ev_free.push_back(r.a);
        g_ev_free.push_back(r.b);
    }
    g_prof.clear();
    std::string out = "{";
    for (int k = 0; k < PK_COUNT; ++k) {
        char buf[256];
        snprintf(buf, sizeof buf,
                 "%s\"%s\": {\"launches\": %ld, \"ms\": %.6f, \"bytes\": %.0f, \"ops\": %.0f, \"fp_ops\": %.0f}",
                 k ? ", " : "", kProfNames[k], cnt[k], ms[k], by[k], op[k], fo[k]);
        out += buf;
    }
    return out + "}";
}

// ------------------------------------------------------------------ NTT
// Forward transform: Cooley-Tukey with the psi twist merged into the twiddles
// (Longa-Naehrig 2016), bit-reversed output: stage s (m = 2^s butterfly groups),
// group i uses psi^(bitrev(m+i)).  N = N1 * N2: the first log N1 stages pair elements
// a multiple of N2 apart (column pass), the last log N2 stages stay inside contiguous
// rows of N2 elements (row pass).  A block holds NTT_E = 2048 elements: one row, or
// NTT_E/N1 columns.  Each thread keeps 8 elements in registers and runs up to three
// stages on them (a radix-8 round) between LDS exchanges; butterflies use Harvey's
// lazy reduction (values in [0, 4q) forward, [0, 2q) inverse; q < 2^61).
//
// Element (transform u, position j) of a block lives at LDS address j * T + u where
// T is the number of transforms in the block (1 for rows, NTT_E / N1 for columns);
// the twiddle index of stage s at position j is (X << s) + (j >> (L - s)) with X = 1
// for the column pass and X = N1 + row for the row pass.

__device__ __forceinline__ u64 red4(u64 x, u64 q2) { return x >= q2 ? x - q2 : x; }

// LDS address of element a: the row pass inserts one pad word every 32 words, which
// spreads the strided accesses of its later rounds over the banks (16-way -> 4-way
// conflicts at distance 4, 8-way -> 2-way at distance 1); the column pass needs none.
template <bool PAD>
__device__ __forceinline__ int lds_at(int a) {
    return PAD ? a + (a >> 5) : a;
}
#define NTT_LDS (NTT_E + NTT_E / 32)

// two consecutive residues per lane: 16-byte global loads and stores (the limb buffers and
// their strides are multiples of 2 elements and 16-byte aligned; the launchers check)
typedef u64 u64x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ u64x2 ld2(const u64* p) { return *reinterpret_cast<const u64x2*>(p); }
__device__ __forceinline__ void st2(u64* p, u64x2 v) { *reinterpret_cast<u64x2*>(p) = v; }
// Operands a launch reads exactly once and nothing reads soon after (switching-key words, the
// tensor factors, the Step-1 diagonal-sum inputs and masks) are loaded nontemporally, so they do
// not displace lines that later launches of the step reuse from the caches; measured per kernel:
// tensor sums 8 %, mask sums 7 %, inner product 2 % faster.  Loads of operands that a later
// launch reads again (a transform's limbs, lifts, the row pass's u words) stay ordinary: made
// nontemporal they slowed the launches after them by as much as they gained.
__device__ __forceinline__ u64 ldnt(const u64* p) { return __builtin_nontemporal_load(p); }

// stages s0 .. s0+R-1 of a length-2^L forward transform; each thread owns 8/2^R groups of
// 2^R elements.  Within a group, stage s0+r has 2^r distinct twiddles (one per block of
// 2*half consecutive elements), loaded once each.
template <int R, bool PAD>
__device__ __forceinline__ void fwd_round(u64* s, int L, int s0, int logT, u64 X, const u64* __restrict__ W,
                                          const u64* __restrict__ Ws, u64 q) {
    constexpr int G = 1 << R, NG = 8 / G;
    const int ld = L - s0 - R, d = 1 << ld, T = 1 << logT;
    const u64 q2 = 2 * q;
#pragma unroll
    for (int gg = 0; gg < NG; ++gg) {
        const int g = gg * TPB + threadIdx.x;
        const int u = g & (T - 1), gi = g >> logT;
        const int base = ((gi >> ld) << (ld + R)) + (gi & (d - 1));
        u64 x[G];
#pragma unroll
        for (int k = 0; k < G; ++k) x[k] = s[lds_at<PAD>(((base + k * d) << logT) + u)];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int st = s0 + r;
            const int half = G >> (r + 1);
#pragma unroll
            for (int b = 0; b < (1 << r); ++b) {
                const int idx = (int)(X << st) + ((base + b * 2 * half * d) >> (L - st));
                const u64 w = W[idx], ws = Ws[idx];
#pragma unroll
                for (int k = b * 2 * half; k < b * 2 * half + half; ++k) {
                    const u64 U = red4(x[k], q2);
                    const u64 V = mul_shoup_lazy(x[k + half], w, ws, q);
                    x[k] = U + V;
                    x[k + half] = U - V + q2;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < G; ++k) s[lds_at<PAD>(((base + k * d) << logT) + u)] = x[k];
    }
}

// stages s0 .. s0-R+1 (descending) of a length-2^L inverse transform
template <int R, bool PAD>
__device__ __forceinline__ void inv_round(u64* s, int L, int s0, int logT, u64 X, const u64* __restrict__ W,
                                          const u64* __restrict__ Ws, u64 q) {
    constexpr int G = 1 << R, NG = 8 / G;
    // the round covers stages s0-R+1 .. s0; its smallest distance belongs to stage s0
    const int ld = L - s0 - 1, d = 1 << ld, T = 1 << logT;
    const u64 q2 = 2 * q;
#pragma unroll
    for (int gg = 0; gg < NG; ++gg) {
        const int g = gg * TPB + threadIdx.x;
        const int u = g & (T - 1), gi = g >> logT;
        const int base = ((gi >> ld) << (ld + R)) + (gi & (d - 1));
        u64 x[G];
#pragma unroll
        for (int k = 0; k < G; ++k) x[k] = s[lds_at<PAD>(((base + k * d) << logT) + u)];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int st = s0 - r, half = 1 << r;
#pragma unroll
            for (int b = 0; b < (G >> (r + 1)); ++b) {
                const int idx = (int)(X << st) + ((base + b * 2 * half * d) >> (L - st));
                const u64 w = W[idx], ws = Ws[idx];
#pragma unroll
                for (int k = b * 2 * half; k < b * 2 * half + half; ++k) {
                    const u64 U = x[k], V = x[k + half];
                    x[k] = red4(U + V, q2);
                    x[k + half] = mul_shoup_lazy(U - V + q2, w, ws, q);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < G; ++k) s[lds_at<PAD>(((base + k * d) << logT) + u)] = x[k];
    }
}

template <bool PAD>
__device__ __forceinline__ void fwd_all(u64* s, int L, int logT, u64 X, const u64* W, const u64* Ws, u64 q) {
    int st = 0;
    while (L - st >= 3) {
        fwd_round<3, PAD>(s, L, st, logT, X, W, Ws, q);
        __syncthreads();
        st += 3;
    }
    if (L - st == 2) {
        fwd_round<2, PAD>(s, L, st, logT, X, W, Ws, q);
        __syncthreads();
    } else if (L - st == 1) {
        fwd_round<1, PAD>(s, L, st, logT, X, W, Ws, q);
        __syncthreads();
    }
}

template <bool PAD>
__device__ __forceinline__ void inv_all(u64* s, int L, int logT, u64 X, const u64* W, const u64* Ws, u64 q) {
    int st = L - 1;  // highest stage first
    while (st + 1 >= 3) {
        inv_round<3, PAD>(s, L, st, logT, X, W, Ws, q);
        __syncthreads();
        st -= 3;
    }
    if (st + 1 == 2) {
        inv_round<2, PAD>(s, L, st, logT, X, W, Ws, q);
        __syncthreads();
    } else if (st + 1 == 1) {
        inv_round<1, PAD>(s, L, st, logT, X, W, Ws, q);
        __syncthreads();
    }
}

// ---- row pass of a 2048-point block (N2 = 2^11), round structure fixed at compile time:
// forward stages 0-2, 3-5, 6-8, 9-10; inverse 10-8, 7-5, 4-2, 1-0.  A group of 2^R elements
// base + k d (base = (J << (ld + R)) + (g mod d)) sits at padded offsets base' + k d + (k d >> 5)
// from its padded base, so its LDS accesses are one address plus constants; its 2^R - 1
// twiddle pairs (w, w') are contiguous in a per-row table built on the host in the order the
// round consumes them (ROW_TW pairs per row, round after round, group J after group J).
// butterflies of one forward group of 2^R elements in registers, twiddle pairs at t
template <int R>
__device__ __forceinline__ void fwd_group(u64 (&x)[1 << R], const u64* __restrict__ t, u64 q) {
    constexpr int G = 1 << R;
    const u64 q2 = 2 * q;
    u64x2 w[G - 1];
#pragma unroll
    for (int i = 0; i < G - 1; ++i) w[i] = ld2(t + 2 * i);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int half = G >> (r + 1);
#pragma unroll
        for (int b = 0; b < (1 << r); ++b) {
            const u64x2 wb = w[(1 << r) - 1 + b];
#pragma unroll
            for (int k = b * 2 * half; k < b * 2 * half + half; ++k) {
                const u64 U = red4(x[k], q2);
                const u64 V = mul_shoup_lazy(x[k + half], wb.x, wb.y, q);
                x[k] = U + V;
                x[k + half] = U - V + q2;
            }
        }
    }
}

template <int R>
__device__ __forceinline__ void inv_group(u64 (&x)[1 << R], const u64* __restrict__ t, u64 q) {
    constexpr int G = 1 << R;
    const u64 q2 = 2 * q;
    u64x2 w[G - 1];
#pragma unroll
    for (int i = 0; i < G - 1; ++i) w[i] = ld2(t + 2 * i);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int half = 1 << r;
#pragma unroll
        for (int b = 0; b < (G >> (r + 1)); ++b) {
            const u64x2 wb = w[G - (G >> r) + b];
#pragma unroll
            for (int k = b * 2 * half; k < b * 2 * half + half; ++k) {
                const u64 U = x[k], V = x[k + half];
                x[k] = red4(U + V, q2);
                x[k + half] = mul_shoup_lazy(U - V + q2, wb.x, wb.y, q);
            }
        }
    }
}

template <int R, int S0>
__device__ __forceinline__ void fwd_row_round(u64* s, const u64* __restrict__ tw, int off, u64 q) {
    constexpr int G = 1 << R, NG = 8 / G, LD = 11 - S0 - R, D = 1 << LD;
#pragma unroll
    for (int gg = 0; gg < NG; ++gg) {
        const int g = gg * TPB + threadIdx.x;
        const int J = g >> LD;
        const int base = (J << (LD + R)) + (g & (D - 1));
        u64* sb = s + base + (base >> 5);
        u64 x[G];
#pragma unroll
        for (int k = 0; k < G; ++k) x[k] = sb[k * D + ((k * D) >> 5)];
        fwd_group<R>(x, tw + 2 * (off + J * (G - 1)), q);
#pragma unroll
        for (int k = 0; k < G; ++k) sb[k * D + ((k * D) >> 5)] = x[k];
    }
}

template <int R, int S0>
__device__ __forceinline__ void inv_row_round(u64* s, const u64* __restrict__ tw, int off, u64 q) {
    constexpr int G = 1 << R, NG = 8 / G, LD = 11 - S0 - 1, D = 1 << LD;
#pragma unroll
    for (int gg = 0; gg < NG; ++gg) {
        const int g = gg * TPB + threadIdx.x;
        const int J = g >> LD;
        const int base = (J << (LD + R)) + (g & (D - 1));
        u64* sb = s + base + (base >> 5);
        u64 x[G];
#pragma unroll
        for (int k = 0; k < G; ++k) x[k] = sb[k * D + ((k * D) >> 5)];
        inv_group<R>(x, tw + 2 * (off + J * (G - 1)), q);
#pragma unroll
        for (int k = 0; k < G; ++k) sb[k * D + ((k * D) >> 5)] = x[k];
    }
}

// The first and last rounds of a row pass run on registers: the first round's group of a
// lane is the lane's own slice of the row (forward: elements tid + 256 k; inverse: the eight
// contiguous elements 8 tid + k), loaded by the caller straight from global memory, and the
// last round's groups (forward: elements 4 g + k; inverse: g + 512 k, for g = tid and
// 256 + tid) go back to the caller, which stores them with its epilogue.  Two LDS round
// trips and two barriers fewer than staging the whole row through LDS.
// after_first() runs once the first round's results are in LDS: the lane's registers of the
// first round are free there, so the caller can start its epilogue loads early
template <class F>
__device__ __forceinline__ void fwd_rows_2048(u64* s, const u64* tw, u64 q, u64 (&x)[8], u64 (&y)[8],
                                              F&& after_first) {
    const int tid = threadIdx.x;
    fwd_group<3>(x, tw, q);
    u64* sb = s + tid + (tid >> 5);
#pragma unroll
    for (int k = 0; k < 8; ++k) sb[264 * k] = x[k];
    after_first();
    __syncthreads();
    fwd_row_round<3, 3>(s, tw, 7, q);
    __syncthreads();
    fwd_row_round<3, 6>(s, tw, 63, q);
    __syncthreads();
#pragma unroll
    for (int gg = 0; gg < 2; ++gg) {
        const int g = gg * TPB + tid;
        const u64* sg = s + 4 * g + (g >> 3);
        u64 z[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) z[k] = sg[k];
        fwd_group<2>(z, tw + 2 * (511 + 3 * g), q);
#pragma unroll
        for (int k = 0; k < 4; ++k) y[4 * gg + k] = z[k];
    }
}

__device__ __forceinline__ void inv_rows_2048(u64* s, const u64* tw, u64 q, u64 (&x)[8], u64 (&y)[8]) {
    const int tid = threadIdx.x;
    inv_group<3>(x, tw + 2 * 7 * tid, q);
    u64* sb = s + 8 * tid + (tid >> 2);
#pragma unroll
    for (int k = 0; k < 8; ++k) sb[k] = x[k];
    __syncthreads();
    inv_row_round<3, 7>(s, tw, 1792, q);
    __syncthreads();
    inv_row_round<3, 4>(s, tw, 2016, q);
    __syncthreads();
#pragma unroll
    for (int gg = 0; gg < 2; ++gg) {
        const int g = gg * TPB + tid;
        const u64* sg = s + g + (g >> 5);
        u64 z[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) z[k] = sg[528 * k];
        inv_group<2>(z, tw + 2 * 2044, q);
#pragma unroll
        for (int k = 0; k < 4; ++k) y[4 * gg + k] = z[k];
    }
}

// ---- column pass with L1 <= 5 stages (N <= 2^16): the 2^(11 - L1) >= 64 columns of a
// block make the group index g >> (11 - L1) the same for the 64 lanes of a wave, so each
// twiddle is one scalar load shared by the wave.
template <int R, int S0, int L1>
__device__ __forceinline__ void fwd_col_round(u64* s, const u64* __restrict__ W, const u64* __restrict__ Ws,
                                              u64 q) {
    constexpr int G = 1 << R, NG = 8 / G, LD = L1 - S0 - R, D = 1 << LD, LOGT = 11 - L1, TC = 1 << LOGT;
    const u64 q2 = 2 * q;
#pragma unroll
    for (int gg = 0; gg < NG; ++gg) {
        const int g = gg * TPB + threadIdx.x;
        const int u = g & (TC - 1);
        const int gi = __builtin_amdgcn_readfirstlane(g >> LOGT);
        const int J = gi >> LD;
        const int base = (J << (LD + R)) + (gi & (D - 1));
        u64 x[G];
#pragma unroll
        for (int k = 0; k < G; ++k) x[k] = s[((base + k * D) << LOGT) + u];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int half = G >> (r + 1);
#pragma unroll
            for (int b = 0; b < (1 << r); ++b) {
                const int idx = (1 << (S0 + r)) + (J << r) + b;
                const u64 w = W[idx], ws = Ws[idx];
#pragma unroll
                for (int k = b * 2 * half; k < b * 2 * half + half; ++k) {
                    const u64 U = red4(x[k], q2);
                    const u64 V = mul_shoup_lazy(x[k + half], w, ws, q);
                    x[k] = U + V;
                    x[k + half] = U - V + q2;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < G; ++k) s[((base + k * D) << LOGT) + u] = x[k];
    }
}

template <int R, int S0, int L1>
__device__ __forceinline__ void inv_col_round(u64* s, const u64* __restrict__ W, const u64* __restrict__ Ws,
                                              u64 q) {
    constexpr int G = 1 << R, NG = 8 / G, LD = L1 - S0 - 1, D = 1 << LD, LOGT = 11 - L1, TC = 1 << LOGT;
    const u64 q2 = 2 * q;
#pragma unroll
    for (int gg = 0; gg < NG; ++gg) {
        const int g = gg * TPB + threadIdx.x;
        const int u = g & (TC - 1);
        const int gi = __builtin_amdgcn_readfirstlane(g >> LOGT);
        const int J = gi >> LD;
        const int base = (J << (LD + R)) + (gi & (D - 1));
        u64 x[G];
#pragma unroll
        for (int k = 0; k < G; ++k) x[k] = s[((base + k * D) << LOGT) + u];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int half = 1 << r;
#pragma unroll
            for (int b = 0; b < (G >> (r + 1)); ++b) {
                const int idx = (1 << (S0 - r)) + (J << (R - 1 - r)) + b;
                const u64 w = W[idx], ws = Ws[idx];
#pragma unroll
                for (int k = b * 2 * half; k < b * 2 * half + half; ++k) {
                    const u64 U = x[k], V = x[k + half];
                    x[k] = red4(U + V, q2);
                    x[k + half] = mul_shoup_lazy(U - V + q2, w, ws, q);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < G; ++k) s[((base + k * D) << LOGT) + u] = x[k];
    }
}

template <int L1, int S0>
__device__ __forceinline__ void fwd_cols_from(u64* s, const u64* W, const u64* Ws, u64 q) {
    if constexpr (S0 < L1) {
        constexpr int R = L1 - S0 >= 3 ? 3 : L1 - S0;
        fwd_col_round<R, S0, L1>(s, W, Ws, q);
        __syncthreads();
        fwd_cols_from<L1, S0 + R>(s, W, Ws, q);
    }
}

template <int L1, int ST>
__device__ __forceinline__ void inv_cols_from(u64* s, const u64* W, const u64* Ws, u64 q) {
    if constexpr (ST >= 0) {
        constexpr int R = ST + 1 >= 3 ? 3 : ST + 1;
        inv_col_round<R, ST, L1>(s, W, Ws, q);
        __syncthreads();
        inv_cols_from<L1, ST - R>(s, W, Ws, q);
    }
}

// column stages of a block: compile-time rounds for L1 <= 5, the generic rounds beyond
__device__ __forceinline__ void fwd_cols_any(u64* s, int L1, const u64* W, const u64* Ws, u64 q) {
    switch (L1) {
        case 1: fwd_cols_from<1, 0>(s, W, Ws, q); break;
        case 2: fwd_cols_from<2, 0>(s, W, Ws, q); break;
        case 3: fwd_cols_from<3, 0>(s, W, Ws, q); break;
        case 4: fwd_cols_from<4, 0>(s, W, Ws, q); break;
        case 5: fwd_cols_from<5, 0>(s, W, Ws, q); break;
        default: fwd_all<false>(s, L1, 11 - L1, 1, W, Ws, q); break;
    }
}

__device__ __forceinline__ void inv_cols_any(u64* s, int L1, const u64* W, const u64* Ws, u64 q) {
    switch (L1) {
        case 1: inv_cols_from<1, 0>(s, W, Ws, q); break;
        case 2: inv_cols_from<2, 1>(s, W, Ws, q); break;
        case 3: inv_cols_from<3, 2>(s, W, Ws, q); break;
        case 4: inv_cols_from<4, 3>(s, W, Ws, q); break;
        case 5: inv_cols_from<5, 4>(s, W, Ws, q); break;
        default: inv_all<false>(s, L1, 11 - L1, 1, W, Ws, q); break;
    }
}

// ---- FP64 butterflies for primes below 2^46.  A residue is held as an integer-valued double
// (balanced: any sign, |x| a small multiple of q).  x w mod q: the product is split exactly as
// hi + lo (hi = fl(x w), lo = fma(x, w, -hi)), c = rint(x fl(w / q)) is within one of the
// rounded quotient, and fma(-c, q, hi) + lo = x w - c q exactly; for |x| < 32 q and q < 2^46 the
// result lies in (-q, q).  Forward (Cooley-Tukey) passes add at most q per stage, so 15 stages
// from |x| < 4q need no reduction; inverse (Gentleman-Sande) rounds reduce their inputs to
// |x| <= q/2 + 1 first (x - rint(x / q) q).  One FP64 butterfly is 8 instructions (v_mul_f64,
// v_fma_f64, v_rndne_f64, v_add_f64), against 27 for the 64-bit integer Shoup butterfly.
// Between the two passes of a transform the limb holds the raw double words; the transform's
// output is canonical.  Both passes of a limb decide by the same rule (fp64_limb).
typedef double f64x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ f64x2 ld2d(const double* p) { return *reinterpret_cast<const f64x2*>(p); }
static_assert(NTT_E == 2048, "the FP64 rule assumes 2048-element rows");
// exact for x < 2^52
__device__ __forceinline__ double u2d(u64 x) {
    return __longlong_as_double((long long)(x | 0x4330000000000000ull)) - 4503599627370496.0;
}
__device__ __forceinline__ double bits_d(u64 x) { return __longlong_as_double((long long)x); }
__device__ __forceinline__ u64 d_bits(double x) { return (u64)__double_as_longlong(x); }
__device__ __forceinline__ double red_d(double x, double q, double qinv) {
#pragma clang fp contract(off)
    return __fma_rn(-rint(x * qinv), q, x);
}
// any integer-valued |x| < 2^50 -> its residue in [0, q) as a word
__device__ __forceinline__ u64 canon_d(double x, double q, double qinv) {
#pragma clang fp contract(off)
    double r = red_d(x, q, qinv);
    r = r < 0.0 ? r + q : r;
    return (u64)__double_as_longlong(r + 4503599627370496.0) & 0xFFFFFFFFFFFFFull;
}
__device__ __forceinline__ double mulmod_d(double a, double w, double wq, double q) {
#pragma clang fp contract(off)
    const double hi = a * w;
    const double lo = __fma_rn(a, w, -hi);
    const double c = rint(a * wq);
    return __fma_rn(-c, q, hi) + lo;
}

template <int R>
__device__ __forceinline__ void fwd_group_d(double (&x)[1 << R], const double* __restrict__ t, double q) {
#pragma clang fp contract(off)
    constexpr int G = 1 << R;
    f64x2 w[G - 1];
#pragma unroll
    for (int i = 0; i < G - 1; ++i) w[i] = ld2d(t + 2 * i);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int half = G >> (r + 1);
#pragma unroll
        for (int b = 0; b < (1 << r); ++b) {
            const f64x2 wb = w[(1 << r) - 1 + b];
#pragma unroll
            for (int k = b * 2 * half; k < b * 2 * half + half; ++k) {
                const double V = mulmod_d(x[k + half], wb.x, wb.y, q);
                const double U = x[k];
                x[k] = U + V;
                x[k + half] = U - V;
            }
        }
    }
}

// the inverse group reduces its inputs first (|x| <= q/2 + 1)
template <int R>
__device__ __forceinline__ void inv_group_d(double (&x)[1 << R], const double* __restrict__ t, double q,
                                            double qinv) {
#pragma clang fp contract(off)
    constexpr int G = 1 << R;
#pragma unroll
    for (int k = 0; k < G; ++k) x[k] = red_d(x[k], q, qinv);
    f64x2 w[G - 1];
#pragma unroll
    for (int i = 0; i < G - 1; ++i) w[i] = ld2d(t + 2 * i);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int half = 1 << r;
#pragma unroll
        for (int b = 0; b < (G >> (r + 1)); ++b) {
            const f64x2 wb = w[G - (G >> r) + b];
#pragma unroll
            for (int k = b * 2 * half; k < b * 2 * half + half; ++k) {
                const double U = x[k], V = x[k + half];
                x[k] = U + V;
                x[k + half] = mulmod_d(U - V, wb.x, wb.y, q);
            }
        }
    }
}

template <int R, int S0>
__device__ __forceinline__ void fwd_row_round_d(double* s, const double* __restrict__ tw, int off, double q) {
    constexpr int G = 1 << R, NG = 8 / G, LD = 11 - S0 - R, D = 1 << LD;
#pragma unroll
    for (int gg = 0; gg < NG; ++gg) {
        const int g = gg * TPB + threadIdx.x;
        const int J = g >> LD;
        const int base = (J << (LD + R)) + (g & (D - 1));
        double* sb = s + base + (base >> 5);
        double x[G];
#pragma unroll
        for (int k = 0; k < G; ++k) x[k] = sb[k * D + ((k * D) >> 5)];
        fwd_group_d<R>(x, tw + 2 * (off + J * (G - 1)), q);
#pragma unroll
        for (int k = 0; k < G; ++k) sb[k * D + ((k * D) >> 5)] = x[k];
    }
}

template <int R, int S0>
__device__ __forceinline__ void inv_row_round_d(double* s, const double* __restrict__ tw, int off, double q,
                                                double qinv) {
    constexpr int G = 1 << R, NG = 8 / G, LD = 11 - S0 - 1, D = 1 << LD;
#pragma unroll
    for (int gg = 0; gg < NG; ++gg) {
        const int g = gg * TPB + threadIdx.x;
        const int J = g >> LD;
        const int base = (J << (LD + R)) + (g & (D - 1));
        double* sb = s + base + (base >> 5);
        double x[G];
#pragma unroll
        for (int k = 0; k < G; ++k) x[k] = sb[k * D + ((k * D) >> 5)];
        inv_group_d<R>(x, tw + 2 * (off + J * (G - 1)), q, qinv);
#pragma unroll
        for (int k = 0; k < G; ++k) sb[k * D + ((k * D) >> 5)] = x[k];
    }
}

// register-first and register-last row passes, as the integer ones above
template <class F>
__device__ __forceinline__ void fwd_rows_2048_d(double* s, const double* tw, double q, double (&x)[8],
                                                double (&y)[8], F&& after_first) {
    const int tid = threadIdx.x;
    fwd_group_d<3>(x, tw, q);
    double* sb = s + tid + (tid >> 5);
#pragma unroll
    for (int k = 0; k < 8; ++k) sb[264 * k] = x[k];
    after_first();
    __syncthreads();
    fwd_row_round_d<3, 3>(s, tw, 7, q);
    __syncthreads();
    fwd_row_round_d<3, 6>(s, tw, 63, q);
    __syncthreads();
#pragma unroll
    for (int gg = 0; gg < 2; ++gg) {
        const int g = gg * TPB + tid;
        const double* sg = s + 4 * g + (g >> 3);
        double z[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) z[k] = sg[k];
        fwd_group_d<2>(z, tw + 2 * (511 + 3 * g), q);
#pragma unroll
        for (int k = 0; k < 4; ++k) y[4 * gg + k] = z[k];
    }
}

__device__ __forceinline__ void inv_rows_2048_d(double* s, const double* tw, double q, double qinv,
                                                double (&x)[8], double (&y)[8]) {
    const int tid = threadIdx.x;
    inv_group_d<3>(x, tw + 2 * 7 * tid, q, qinv);
    double* sb = s + 8 * tid + (tid >> 2);
#pragma unroll
    for (int k = 0; k < 8; ++k) sb[k] = x[k];
    __syncthreads();
    inv_row_round_d<3, 7>(s, tw, 1792, q, qinv);
    __syncthreads();
    inv_row_round_d<3, 4>(s, tw, 2016, q, qinv);
    __syncthreads();
#pragma unroll
    for (int gg = 0; gg < 2; ++gg) {
        const int g = gg * TPB + tid;
        const double* sg = s + g + (g >> 5);
        double z[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) z[k] = sg[528 * k];
        inv_group_d<2>(z, tw + 2 * 2044, q, qinv);
#pragma unroll
        for (int k = 0; k < 4; ++k) y[4 * gg + k] = z[k];
    }
}

// column rounds (L1 <= 5): wave-uniform twiddles (w, fl(w / q)) from the [M][N1] column table
template <int R, int S0, int L1>
__device__ __forceinline__ void fwd_col_round_d(double* s, const double* __restrict__ W, double q) {
#pragma clang fp contract(off)
    constexpr int G = 1 << R, NG = 8 / G, LD = L1 - S0 - R, D = 1 << LD, LOGT = 11 - L1, TC = 1 << LOGT;
#pragma unroll
    for (int gg = 0; gg < NG; ++gg) {
        const int g = gg * TPB + threadIdx.x;
        const int u = g & (TC - 1);
        const int gi = __builtin_amdgcn_readfirstlane(g >> LOGT);
        const int J = gi >> LD;
        const int base = (J << (LD + R)) + (gi & (D - 1));
        double x[G];
#pragma unroll
        for (int k = 0; k < G; ++k) x[k] = s[((base + k * D) << LOGT) + u];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int half = G >> (r + 1);
#pragma unroll
            for (int b = 0; b < (1 << r); ++b) {
                const int idx = (1 << (S0 + r)) + (J << r) + b;
                const double w = W[2 * idx], wq = W[2 * idx + 1];
#pragma unroll
                for (int k = b * 2 * half; k < b * 2 * half + half; ++k) {
                    const double V = mulmod_d(x[k + half], w, wq, q);
                    const double U = x[k];
                    x[k] = U + V;
                    x[k + half] = U - V;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < G; ++k) s[((base + k * D) << LOGT) + u] = x[k];
    }
}

template <int R, int S0, int L1>
__device__ __forceinline__ void inv_col_round_d(double* s, const double* __restrict__ W, double q, double qinv) {
#pragma clang fp contract(off)
    constexpr int G = 1 << R, NG = 8 / G, LD = L1 - S0 - 1, D = 1 << LD, LOGT = 11 - L1, TC = 1 << LOGT;
#pragma unroll
    for (int gg = 0; gg < NG; ++gg) {
        const int g = gg * TPB + threadIdx.x;
        const int u = g & (TC - 1);
        const int gi = __builtin_amdgcn_readfirstlane(g >> LOGT);
        const int J = gi >> LD;
        const int base = (J << (LD + R)) + (gi & (D - 1));
        double x[G];
#pragma unroll
        for (int k = 0; k < G; ++k) x[k] = red_d(s[((base + k * D) << LOGT) + u], q, qinv);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int half = 1 << r;
#pragma unroll
            for (int b = 0; b < (G >> (r + 1)); ++b) {
                const int idx = (1 << (S0 - r)) + (J << (R - 1 - r)) + b;
                const double w = W[2 * idx], wq = W[2 * idx + 1];
#pragma unroll
                for (int k = b * 2 * half; k < b * 2 * half + half; ++k) {
                    const double U = x[k], V = x[k + half];
                    x[k] = U + V;
                    x[k + half] = mulmod_d(U - V, w, wq, q);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < G; ++k) s[((base + k * D) << LOGT) + u] = x[k];
    }
}

template <int L1, int S0>
__device__ __forceinline__ void fwd_cols_from_d(double* s, const double* W, double q) {
    if constexpr (S0 < L1) {
        constexpr int R = L1 - S0 >= 3 ? 3 : L1 - S0;
        fwd_col_round_d<R, S0, L1>(s, W, q);
        __syncthreads();
        fwd_cols_from_d<L1, S0 + R>(s, W, q);
    }
}

template <int L1, int ST>
__device__ __forceinline__ void inv_cols_from_d(double* s, const double* W, double q, double qinv) {
    if constexpr (ST >= 0) {
        constexpr int R = ST + 1 >= 3 ? 3 : ST + 1;
        inv_col_round_d<R, ST, L1>(s, W, q, qinv);
        __syncthreads();
        inv_cols_from_d<L1, ST - R>(s, W, q, qinv);
    }
}

// L1 in 1..5 (fp64_limb holds)
__device__ __forceinline__ void fwd_cols_any_d(double* s, int L1, const double* W, double q) {
    switch (L1) {
        case 1: fwd_cols_from_d<1, 0>(s, W, q); break;
        case 2: fwd_cols_from_d<2, 0>(s, W, q); break;
        case 3: fwd_cols_from_d<3, 0>(s, W, q); break;
        case 4: fwd_cols_from_d<4, 0>(s, W, q); break;
        default: fwd_cols_from_d<5, 0>(s, W, q); break;
    }
}

__device__ __forceinline__ void inv_cols_any_d(double* s, int L1, const double* W, double q, double qinv) {
    switch (L1) {
        case 1: inv_cols_from_d<1, 0>(s, W, q, qinv); break;
        case 2: inv_cols_from_d<2, 1>(s, W, q, qinv); break;
        case 3: inv_cols_from_d<3, 2>(s, W, q, qinv); break;
        case 4: inv_cols_from_d<4, 3>(s, W, q, qinv); break;
        default: inv_cols_from_d<5, 4>(s, W, q, qinv); break;
    }
}

__global__ __launch_bounds__(TPB) void k_ntt_fwd_cols(DevTables T, Jobs J) {
    __shared__ u64 s[NTT_E];
    const int N = 1 << T.log_n, L1 = T.n1_log, N2 = N >> L1;
    const int logC = 11 - L1, C = 1 << logC;
    const int job = blockIdx.y, c = job / J.n, k = job % J.n;
    u64* a = J.base + c * J.cstride + (int64_t)J.off[k] * N;
    const int mi = J.mod[k];
    const u64 q = T.mods[mi].q;
    const u64* W = T.psi + (int64_t)mi * N;
    const u64* Ws = T.psi_sh + (int64_t)mi * N;
    const int c0 = blockIdx.x * C;
    if (fp64_limb(q, L1, N2)) {
        double* sd = reinterpret_cast<double*>(s);
        for (int e = 2 * threadIdx.x; e < NTT_E; e += 2 * TPB) {
            const u64x2 v = ld2(a + (int64_t)(e >> logC) * N2 + c0 + (e & (C - 1)));
            sd[e] = u2d(v.x);
            sd[e + 1] = u2d(v.y);
        }
        __syncthreads();
        fwd_cols_any_d(sd, L1, T.cold + (int64_t)mi * (2 << L1), (double)q);
        // raw double words for the FP64 row pass of this limb
        for (int e = 2 * threadIdx.x; e < NTT_E; e += 2 * TPB)
            st2(a + (int64_t)(e >> logC) * N2 + c0 + (e & (C - 1)), u64x2{d_bits(sd[e]), d_bits(sd[e + 1])});
        return;
    }
    for (int e = 2 * threadIdx.x; e < NTT_E; e += 2 * TPB) {
        const u64x2 v = ld2(a + (int64_t)(e >> logC) * N2 + c0 + (e & (C - 1)));
        s[e] = v.x;
        s[e + 1] = v.y;
    }
    __syncthreads();
    fwd_cols_any(s, L1, W, Ws, q);
    // output stays lazy in [0, 4q) for the row pass
    for (int e = 2 * threadIdx.x; e < NTT_E; e += 2 * TPB)
        st2(a + (int64_t)(e >> logC) * N2 + c0 + (e & (C - 1)), u64x2{s[e], s[e + 1]});
}

__device__ __forceinline__ int perm_g(int j, u64 g, int log_n);

// EPI: the ModDown epilogue (E.on) is compiled in; without it the plain transform keeps its
// smaller register footprint
template <bool EPI>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(6))) void k_ntt_fwd_rows(DevTables T, Jobs J, Epi E) {
    __shared__ u64 s[NTT_LDS];
    const int N = 1 << T.log_n, L1 = T.n1_log, L2 = T.n2_log, N1 = 1 << L1, N2 = 1 << L2;
    // jobs in reverse order: the column pass before it wrote the last jobs last, so their limbs
    // are the likeliest to still be in the memory-side cache
    const int job = (int)gridDim.y - 1 - (int)blockIdx.y, c = job / J.n, k = job % J.n;
    const int r = blockIdx.x, tid = threadIdx.x;
    u64* a = J.base + c * J.cstride + (int64_t)J.off[k] * N + (int64_t)r * N2;
    const int mi = J.mod[k];
    const u64 q = T.mods[mi].q, q2 = 2 * q;
    const bool fp = fp64_limb(q, L1, N2), full = N2 == NTT_E;
    // 2048-element rows: the last round's elements 4 g + k (g = tid, 256 + tid) as words,
    // canonical (FP64 path) or lazy in [0, 4q) (integer path)
    u64 y[8];
    // the ModDown epilogue's u words of those elements, loaded while the middle rounds run
    u64x2 uu[4];
    const u64* u = nullptr;
    if constexpr (EPI) {
        const int p = J.off[k] / E.nl, t = J.off[k] % E.nl;
        u = E.u + c * E.u_cs + p * E.u_ps + (int64_t)t * N;
    }
    auto prefetch_u = [&]() {
        if constexpr (EPI) {
#pragma unroll
            for (int i = 0; i < 4; ++i) uu[i] = ld2(u + r * N2 + 4 * ((i >> 1) * TPB + tid) + 2 * (i & 1));
        }
    };
    if (fp) {
        const double qd = (double)q, qinv = 1.0 / qd;
        double x[8], yd[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {  // the column pass left raw doubles (N1 > 1), else canonical words
            const u64 v = a[tid + TPB * i];
            x[i] = L1 ? bits_d(v) : u2d(v);
        }
        fwd_rows_2048_d(reinterpret_cast<double*>(s), T.rtwd + ((int64_t)mi * N1 + r) * (2 * ROW_TW), qd, x, yd,
                        prefetch_u);
#pragma unroll
        for (int i = 0; i < 8; ++i) y[i] = canon_d(yd[i], qd, qinv);
    } else if (full) {
        u64 x[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = a[tid + TPB * i];
        fwd_rows_2048(s, T.rtw + ((int64_t)mi * N1 + r) * (2 * ROW_TW), q, x, y, prefetch_u);
    } else {  // small rings (N < 2048): the row through LDS, plain radix-2 stages
        const u64* W = T.psi + (int64_t)mi * N;
        const u64* Ws = T.psi_sh + (int64_t)mi * N;
        for (int e = 2 * tid; e < N2; e += 2 * TPB) {
            const u64x2 v = ld2(a + e);
            s[lds_at<true>(e)] = v.x;
            s[lds_at<true>(e + 1)] = v.y;
        }
        __syncthreads();
        for (int st = 0; st < L2; st++) {
            const int lt = L2 - st - 1, t = 1 << lt;
            for (int b = tid; b < N2 / 2; b += TPB) {
                const int i = b >> lt, j = b & (t - 1);
                const int j1 = (i << (lt + 1)) + j;
                const int idx = (1 << st) * (N1 + r) + i;
                const u64 U = red4(s[lds_at<true>(j1)], q2);
                const u64 V = mul_shoup_lazy(s[lds_at<true>(j1 + t)], W[idx], Ws[idx], q);
                s[lds_at<true>(j1)] = U + V;
                s[lds_at<true>(j1 + t)] = U - V + q2;
            }
            __syncthreads();
        }
    }
    // emit(i, e, v0, v1): elements e, e + 1 of the row (words below 4q) to their destination;
    // i is the pair's slot in uu (2048-element rows), or -1
    auto for_pairs = [&](auto&& emit) {
        if (fp || full) {
#pragma unroll
            for (int i = 0; i < 4; ++i) emit(i, 4 * ((i >> 1) * TPB + tid) + 2 * (i & 1), y[2 * i], y[2 * i + 1]);
        } else {
            for (int e = 2 * tid; e < N2; e += 2 * TPB) emit(-1, e, s[lds_at<true>(e)], s[lds_at<true>(e + 1)]);
        }
    };
    if constexpr (!EPI) {
        for_pairs([&](int, int e, u64 v0, u64 v1) {
            if (!fp) {
                v0 = red4(v0, q2);
                v1 = red4(v1, q2);
                v0 = v0 >= q ? v0 - q : v0;
                v1 = v1 >= q ? v1 - q : v1;
            }
            st2(a + e, u64x2{v0, v1});
        });
        return;
    }
    const int p = J.off[k] / E.nl, t = J.off[k] % E.nl;
    const u64* add = E.add[p] ? E.add[p] + c * E.add_cs + (int64_t)t * N : nullptr;
    u64* out = E.out[p] + c * E.out_cs + (int64_t)t * N;
    const u64 pi = E.pinv[t], pis = E.pinv_sh[t];
    const u64* mask = E.mask ? E.mask + (int64_t)t * N : nullptr;
    const u64* acc = E.acc[p] ? E.acc[p] + c * E.acc_cs + (int64_t)t * N : nullptr;
    const u64 qninv = T.mods[mi].qninv;
    for_pairs([&](int slot, int e, u64 v0, u64 v1) {
        const int i = r * N2 + e;
        const u64x2 uw = slot >= 0 ? uu[slot] : ld2(u + i);
        // v is below 4q and u < q, so u + 4q - v lies in (0, 5q); the Shoup product
        // reduces any 64-bit operand to [0, q)
        u64 w[2] = {mul_shoup(uw.x + 2 * q2 - v0, pi, pis, q), mul_shoup(uw.y + 2 * q2 - v1, pi, pis, q)};
        if (add) {
            if (E.g == 1) {
                const u64x2 ad = ld2(add + i);
                w[0] = add_mod(w[0], ad.x, q);
                w[1] = add_mod(w[1], ad.y, q);
            } else {
                w[0] = add_mod(w[0], add[perm_g(i, E.g, T.log_n)], q);
                w[1] = add_mod(w[1], add[perm_g(i + 1, E.g, T.log_n)], q);
            }
        }
        if (mask) {
            const u64x2 m = ld2(mask + i);
            w[0] = mul_mont(w[0], m.x, q, qninv);
            w[1] = mul_mont(w[1], m.y, q, qninv);
        }
        if (acc) {
            const u64x2 ac = ld2(acc + i);
            w[0] = add_mod(w[0], ac.x, q);
            w[1] = add_mod(w[1], ac.y, q);
        }
        st2(out + i, u64x2{w[0], w[1]});
    });
}

// Inverse transform: Gentleman-Sande, bit-reversed input, natural output, then N^-1.
// The last pass of the inverse transform multiplies by N^-1, or, with 'scale' set, by the
// per-job constant scale[k mod scale_n] (pairs (c, c')): N^-1 times the (D/q_s)^-1 of a base
// conversion that follows, and then stores the centred representative (y - q when y > (q-1)/2,
// as a two's-complement word), so the conversion reads its prepared inputs directly.
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(8))) void k_ntt_inv_rows(DevTables T, Jobs J, const u64* scale, int scale_n) {
    __shared__ u64 s[NTT_LDS];
    const int N = 1 << T.log_n, L1 = T.n1_log, L2 = T.n2_log, N1 = 1 << L1, N2 = 1 << L2;
    const int job = blockIdx.y, c = job / J.n, k = job % J.n;
    const int r = blockIdx.x, tid = threadIdx.x;
    u64* a = J.base + c * J.cstride + (int64_t)J.off[k] * N + (int64_t)r * N2;
    // out of place: the row comes from the source, the result goes to base
    const u64* src = J.src ? J.src + c * J.src_cstride + (int64_t)J.off[k] * N + (int64_t)r * N2 : a;
    const int mi = J.mod[k];
    const ModP mp_ = T.mods[mi];
    const u64 q = mp_.q, q2 = 2 * q;
    // 2048-element rows: every lane loads its eight elements 8 tid + k before the first
    // barrier and stores g + 512 k (g = tid, 256 + tid) after the last, so in place is safe
    if (fp64_limb(q, L1, N2)) {
        const double qd = (double)q, qinv = 1.0 / qd;
        double x[8], y[8];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const u64x2 v = ld2(src + 8 * tid + 2 * i);
            x[2 * i] = u2d(v.x);
            x[2 * i + 1] = u2d(v.y);
        }
        inv_rows_2048_d(reinterpret_cast<double*>(s), T.irtwd + ((int64_t)mi * N1 + r) * (2 * ROW_TW), qd, qinv, x,
                        y);
        if (L1 == 0) {
            const u64 f = scale ? scale[2 * (k % scale_n)] : mp_.ninv;
            const double fd = (double)f, fq = fd / qd;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                u64 w = canon_d(mulmod_d(y[i], fd, fq, qd), qd, qinv);
                if (scale) w = w > mp_.half ? w - q : w;
                a[(i >> 2) * TPB + tid + 512 * (i & 3)] = w;
            }
        } else {  // raw double words for the FP64 column pass of this limb
#pragma unroll
            for (int i = 0; i < 8; ++i) a[(i >> 2) * TPB + tid + 512 * (i & 3)] = d_bits(y[i]);
        }
        return;
    }
    if (N2 == NTT_E) {
        u64 x[8], y[8];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const u64x2 v = ld2(src + 8 * tid + 2 * i);
            x[2 * i] = v.x;
            x[2 * i + 1] = v.y;
        }
        inv_rows_2048(s, T.irtw + ((int64_t)mi * N1 + r) * (2 * ROW_TW), q, x, y);
        if (L1 == 0) {
            const u64 f = scale ? scale[2 * (k % scale_n)] : mp_.ninv;
            const u64 fs = scale ? scale[2 * (k % scale_n) + 1] : mp_.ninv_sh;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                u64 w = mul_shoup(y[i], f, fs, q);
                if (scale) w = w > mp_.half ? w - q : w;
                a[(i >> 2) * TPB + tid + 512 * (i & 3)] = w;
            }
        } else {  // lazy in [0, 2q)
#pragma unroll
            for (int i = 0; i < 8; ++i) a[(i >> 2) * TPB + tid + 512 * (i & 3)] = y[i];
        }
        return;
    }
    // small rings (N < 2048): the row through LDS, plain radix-2 stages, then N^-1
    const u64* W = T.ipsi + (int64_t)mi * N;
    const u64* Ws = T.ipsi_sh + (int64_t)mi * N;
    for (int e = 2 * tid; e < N2; e += 2 * TPB) {
        const u64x2 v = ld2(src + e);
        s[lds_at<true>(e)] = v.x;
        s[lds_at<true>(e + 1)] = v.y;
    }
    __syncthreads();
    for (int st = L2 - 1; st >= 0; st--) {
        const int lt = L2 - st - 1, t = 1 << lt;
        for (int b = tid; b < N2 / 2; b += TPB) {
            const int i = b >> lt, j = b & (t - 1);
            const int j1 = (i << (lt + 1)) + j;
            const int idx = (1 << st) * (N1 + r) + i;
            const u64 U = s[lds_at<true>(j1)], V = s[lds_at<true>(j1 + t)];
            s[lds_at<true>(j1)] = red4(U + V, q2);
            s[lds_at<true>(j1 + t)] = mul_shoup_lazy(U - V + q2, W[idx], Ws[idx], q);
        }
        __syncthreads();
    }
    // N < 2048 means one row (L1 = 0)
    const u64 f = scale ? scale[2 * (k % scale_n)] : mp_.ninv, fs = scale ? scale[2 * (k % scale_n) + 1] : mp_.ninv_sh;
    for (int e = 2 * tid; e < N2; e += 2 * TPB) {
        u64 y0 = mul_shoup(s[lds_at<true>(e)], f, fs, q), y1 = mul_shoup(s[lds_at<true>(e + 1)], f, fs, q);
        if (scale) {
            y0 = y0 > mp_.half ? y0 - q : y0;
            y1 = y1 > mp_.half ? y1 - q : y1;
        }
        st2(a + e, u64x2{y0, y1});
    }
}

__global__ __launch_bounds__(TPB) void k_ntt_inv_cols(DevTables T, Jobs J, const u64* scale, int scale_n) {
    __shared__ u64 s[NTT_E];
    const int N = 1 << T.log_n, L1 = T.n1_log, N2 = N >> L1;
    const int logC = 11 - L1, C = 1 << logC;
    const int job = blockIdx.y, c = job / J.n, k = job % J.n;
    u64* a = J.base + c * J.cstride + (int64_t)J.off[k] * N;
    const int mi = J.mod[k];
    const ModP mp_ = T.mods[mi];
    const u64 q = mp_.q;
    const u64* W = T.ipsi + (int64_t)mi * N;
    const u64* Ws = T.ipsi_sh + (int64_t)mi * N;
    const int c0 = blockIdx.x * C;
    if (fp64_limb(q, L1, N2)) {
        const double qd = (double)q, qinv = 1.0 / qd;
        double* sd = reinterpret_cast<double*>(s);
        for (int e = 2 * threadIdx.x; e < NTT_E; e += 2 * TPB) {  // raw doubles of the row pass
            const u64x2 v = ld2(a + (int64_t)(e >> logC) * N2 + c0 + (e & (C - 1)));
            sd[e] = bits_d(v.x);
            sd[e + 1] = bits_d(v.y);
        }
        __syncthreads();
        inv_cols_any_d(sd, L1, T.icold + (int64_t)mi * (2 << L1), qd, qinv);
        const u64 f = scale ? scale[2 * (k % scale_n)] : mp_.ninv;
        const double fd = (double)f, fq = fd / qd;
        for (int e = 2 * threadIdx.x; e < NTT_E; e += 2 * TPB) {
            u64 y[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                y[h] = canon_d(mulmod_d(sd[e + h], fd, fq, qd), qd, qinv);
                if (scale) y[h] = y[h] > mp_.half ? y[h] - q : y[h];
            }
            st2(a + (int64_t)(e >> logC) * N2 + c0 + (e & (C - 1)), u64x2{y[0], y[1]});
        }
        return;
    }
    for (int e = 2 * threadIdx.x; e < NTT_E; e += 2 * TPB) {
        const u64x2 v = ld2(a + (int64_t)(e >> logC) * N2 + c0 + (e & (C - 1)));
        s[e] = v.x;
        s[e + 1] = v.y;
    }
    __syncthreads();
    inv_cols_any(s, L1, W, Ws, q);
    const u64 f = scale ? scale[2 * (k % scale_n)] : mp_.ninv, fs = scale ? scale[2 * (k % scale_n) + 1] : mp_.ninv_sh;
    for (int e = 2 * threadIdx.x; e < NTT_E; e += 2 * TPB) {
        u64 y0 = mul_shoup(s[e], f, fs, q), y1 = mul_shoup(s[e + 1], f, fs, q);
        if (scale) {
            y0 = y0 > mp_.half ? y0 - q : y0;
            y1 = y1 > mp_.half ? y1 - q : y1;
        }
        st2(a + (int64_t)(e >> logC) * N2 + c0 + (e & (C - 1)), u64x2{y0, y1});
    }
}

// ---- base conversion fused with the column pass of the forward transform.  A block converts
// one column block (N1 rows x 2^(11 - L1) columns, 2048 slots) of one target limb from the
// ns source limbs, which the inverse transform has already multiplied by their (D/q_s)^-1 and
// centred (signed words), so out_t = sum_s y_s (D/q_s) mod q_t needs no correction term; the
// sum stays lazy in [0, 3q), which the forward butterflies accept, and the column stages run on
// it; the row pass follows as usual.  Workgroups are handed to
// the 8 XCDs round-robin, so the blocks of all targets of one source block are numbered to
// run back to back on one XCD, where the source words stay in that XCD's L2.
// MD: the digits of one ModUp in one launch (targets carry their digit; a block reads its own
// digit's sources); without it the single-digit form keeps its loads free of the digit logic
template <int NS, bool MD>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(8))) void k_conv_cols(DevTables T, ConvDesc D) {
    __shared__ u64 s[NTT_E];
    const int N = 1 << T.log_n, L1 = T.n1_log, N2 = N >> L1;
    const int logC = 11 - L1, C = 1 << logC;
    const int tiles = N / NTT_E, npairs = tiles * D.npoly * D.nct;
    const int lb = blockIdx.x;
    int pair, t;
    if ((npairs & 7) == 0) {
        const int j = lb >> 3;
        pair = ((j / D.nt) << 3) + (lb & 7);
        t = j % D.nt;
    } else {
        pair = lb / D.nt;
        t = lb % D.nt;
    }
    const int x = pair % tiles, pc = pair / tiles, p = pc % D.npoly, c = pc / D.npoly;
    const int mi = D.dmod[t];
    const ModP m = T.mods[mi];
    const bool fp = fp64_limb(m.q, L1, N2);
    double* sd = reinterpret_cast<double*>(s);
    constexpr bool BAL = NS > 5;  // the balanced split keeps six to eight products in int64
    // a digit with fewer sources than NS: its missing terms get a zero constant and re-read its
    // last source, so every lane runs the same loads and the sum is unchanged
    const int dg = MD ? D.tdig[t] : 0;
    const int ns = MD ? D.dns[dg] : NS;
    const u64* tab = MD ? D.tab + D.dtab[dg] : D.tab;
    Split30 tw[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i)
        tw[i] = i < ns ? split30(tab[((int64_t)i * D.tab_ld + D.tcol[t]) * 2]) : Split30{0, 0};
    const u64* src = D.src + (MD ? D.dsrc[dg] : 0) + c * D.src_cstride + p * D.src_pstride;
    const int col0 = x * C;
    for (int e = 2 * threadIdx.x; e < NTT_E; e += 2 * TPB) {
        const int64_t slot = (int64_t)(e >> logC) * N2 + col0 + (e & (C - 1));
        AccS a0 = {0, 0, 0}, a1 = {0, 0, 0};
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            const u64x2 y = ld2(src + (int64_t)(i < ns ? i : ns - 1) * N + slot);
            int32_t lo, hi;
            split30s<BAL>((int64_t)y.x, lo, hi);
            macs(a0, lo, hi, tw[i]);
            split30s<BAL>((int64_t)y.y, lo, hi);
            macs(a1, lo, hi, tw[i]);
        }
        const u64 r0 = redcs_lazy(a0, m.q, m.qninv), r1 = redcs_lazy(a1, m.q, m.qninv);
        if (fp) {
            sd[e] = u2d(r0);
            sd[e + 1] = u2d(r1);
        } else {
            s[e] = r0;
            s[e + 1] = r1;
        }
    }
    __syncthreads();
    u64* a = D.dst + c * D.dst_cstride + p * D.dst_pstride + (int64_t)D.doff[t] * N;
    if (fp) {  // raw double words for the FP64 row pass of this limb
        fwd_cols_any_d(sd, L1, T.cold + (int64_t)mi * (2 << L1), (double)m.q);
        for (int e = 2 * threadIdx.x; e < NTT_E; e += 2 * TPB)
            st2(a + (int64_t)(e >> logC) * N2 + col0 + (e & (C - 1)), u64x2{d_bits(sd[e]), d_bits(sd[e + 1])});
        return;
    }
    fwd_cols_any(s, L1, T.psi + (int64_t)mi * N, T.psi_sh + (int64_t)mi * N, m.q);
    for (int e = 2 * threadIdx.x; e < NTT_E; e += 2 * TPB)
        st2(a + (int64_t)(e >> logC) * N2 + col0 + (e & (C - 1)), u64x2{s[e], s[e + 1]});
}


// the NTT kernels move two residues per lane with 16-byte accesses
static void check_ntt_alignment(const Jobs& J, const Epi* E) {
    bool bad = misaligned16(J.base) || (J.cstride & 1);
    if (E && E->on) {
        bad = bad || misaligned16(E->u) || ((E->u_cs | E->u_ps | E->add_cs | E->out_cs | E->acc_cs) & 1) ||
              misaligned16(E->mask);
        for (int p = 0; p < 2; ++p) bad = bad || misaligned16(E->add[p]) || misaligned16(E->out[p]) ||
                                          misaligned16(E->acc[p]);
    }
    if (bad) throw std::runtime_error("NTT operand not 16-byte aligned");
}

// limbs of a job list that run FP64 butterflies (for the profile's operation counts)
static double fp64_limbs(const DevTables& T, const Jobs& J) {
    int n = 0;
    for (int k = 0; k < J.n; ++k) n += (int)((T.fp64_mods >> J.mod[k]) & 1);
    return (double)n * J.nct;
}

void launch_ntt_moddown(const DevTables& T, const Jobs& J, const Epi& E, hipStream_t st, bool cols) {
    if (J.n == 0 || J.nct == 0) return;
    check_ntt_alignment(J, &E);
    const int N = 1 << T.log_n, N1 = 1 << T.n1_log;
    dim3 grid_rows(N1, J.n * J.nct), grid_cols(N / NTT_E, J.n * J.nct);
    const double limbs = (double)J.n * J.nct, fl = fp64_limbs(T, J);
    if (T.n1_log > 0 && cols) {
        ProfScope p(PK_NTT_FWD_COLS, 16.0 * limbs * N, st, limbs * (N / 2) * T.n1_log, fl * (N / 2) * T.n1_log);
        HE_LAUNCH(k_ntt_fwd_cols, grid_cols, dim3(TPB), 0, st, T, J);
    }
    // reads the converted limb and u, writes the output; plus the optional add and
    // accumulator operands (per ciphertext) and the mask (shared by the group)
    const double per_ct = (E.add[0] ? 1 : 0) + (E.add[1] ? 1 : 0) + (E.acc[0] ? 1 : 0) + (E.acc[1] ? 1 : 0);
    const double rows_bytes = 8.0 * N * (3 * limbs + per_ct * E.nl * J.nct + (E.mask ? E.nl : 0));
    ProfScope p(PK_NTT_FWD_ROWS, rows_bytes, st, limbs * (N / 2) * T.n2_log, fl * (N / 2) * T.n2_log);
    if (!E.on) throw std::runtime_error("ModDown row pass without its epilogue");
    HE_LAUNCH(k_ntt_fwd_rows<true>, grid_rows, dim3(TPB), 0, st, T, J, E);
}

void launch_ntt(const DevTables& T, const Jobs& J, bool inverse, hipStream_t st, const u64* scale, int scale_n,
                bool cols) {
    if (J.n == 0 || J.nct == 0) return;
    if (scale && (!inverse || scale_n < 1)) throw std::runtime_error("NTT output scale: inverse transforms only");
    if (J.src && (!inverse || misaligned16(J.src) || (J.src_cstride & 1)))
        throw std::runtime_error("NTT source: inverse transforms with aligned sources only");
    check_ntt_alignment(J, nullptr);
    Epi E;
    E.on = 0;
    const int N = 1 << T.log_n, N1 = 1 << T.n1_log;
    dim3 grid_rows(N1, J.n * J.nct), grid_cols(N / NTT_E, J.n * J.nct);
    const double limbs = (double)J.n * J.nct;
    const double bytes = 16.0 * limbs * N, b1 = limbs * (N / 2) * T.n1_log, b2 = limbs * (N / 2) * T.n2_log;
    const double fl = fp64_limbs(T, J), f1 = fl * (N / 2) * T.n1_log, f2 = fl * (N / 2) * T.n2_log;
    if (!inverse) {
        if (T.n1_log > 0 && cols) {
            ProfScope p(PK_NTT_FWD_COLS, bytes, st, b1, f1);
            HE_LAUNCH(k_ntt_fwd_cols, grid_cols, dim3(TPB), 0, st, T, J);
        }
        ProfScope p(PK_NTT_FWD_ROWS, bytes, st, b2, f2);
        HE_LAUNCH(k_ntt_fwd_rows<false>, grid_rows, dim3(TPB), 0, st, T, J, E);
    } else {
        {
            ProfScope p(PK_NTT_INV_ROWS, bytes, st, b2, f2);
            HE_LAUNCH(k_ntt_inv_rows, grid_rows, dim3(TPB), 0, st, T, J, scale, scale_n);
        }
        if (T.n1_log > 0) {
            ProfScope p(PK_NTT_INV_COLS, bytes, st, b1, f1);
            HE_LAUNCH(k_ntt_inv_cols, grid_cols, dim3(TPB), 0, st, T, J, scale, scale_n);
        }
    }
}

// ------------------------------------------------------------------ batched copies
// grid (x, row, region): each block row copies a slice of one row of one region
__global__ __launch_bounds__(TPB) void k_copy(CopyDesc D) {
    const int r = blockIdx.z, row = blockIdx.y;
    if (row >= D.rows[r]) return;
    const u64* src = D.src[r] + row * D.spitch[r];
    u64* dst = D.dst[r] + row * D.dpitch[r];
    const int64_t w = D.width[r];
    for (int64_t c = 2 * ((int64_t)blockIdx.x * TPB + threadIdx.x); c < w; c += 2 * (int64_t)gridDim.x * TPB)
        st2(dst + c, ld2(src + c));
}

void launch_copy(CopyDesc& D, hipStream_t st) {
    if (D.n <= 0) return;
    if (D.n > CP_MAX) throw std::runtime_error("copy: too many regions");
    D.start[0] = 0;
    double bytes = 0;
    int64_t wmax = 0;
    int rmax = 0;
    for (int r = 0; r < D.n; ++r) {
        if ((D.width[r] & 1) || (D.spitch[r] & 1) || (D.dpitch[r] & 1) || misaligned16(D.src[r]) ||
            misaligned16(D.dst[r]) || D.rows[r] < 0 || D.width[r] < 0 || D.rows[r] > 65535)
            throw std::runtime_error("copy: region not 16-byte aligned");
        D.start[r + 1] = D.start[r] + (D.width[r] >> 1) * D.rows[r];
        bytes += 16.0 * D.width[r] * D.rows[r];
        wmax = std::max(wmax, D.width[r]);
        rmax = std::max(rmax, D.rows[r]);
    }
    if (D.start[D.n] == 0) return;
    // about 4 word pairs per thread along a row
    const int64_t bx = std::max<int64_t>(1, std::min<int64_t>(ceil_div(wmax / 2, 4 * TPB), 1024));
    ProfScope p(PK_COPY, bytes, st);
    HE_LAUNCH(k_copy, dim3((unsigned)bx, (unsigned)rmax, (unsigned)D.n), dim3(TPB), 0, st, D);
}

// ------------------------------------------------------------------ base conversion
// Centered fast base conversion (Bajard et al. 2016 / Halevi-Polyakov-Shoup 2019 in
// its centered form): y_s = centered([x_s (D/q_s)^-1]_{q_s}),
// out_t = sum_s y_s (D/q_s) mod q_t, accumulated in 128 bits and reduced once (REDC).
#define BC_TG 32  // targets per block of the base conversion
template <int NS>
__global__ __launch_bounds__(TPB) void k_baseconv(DevTables T, ConvDesc D) {
    // the block's slice of the constant table (NS sources x up to BC_TG targets) goes to LDS
    // once; the sources are read and prepared once for all the targets of the slice.  Each
    // thread converts two adjacent slots (16-byte loads and stores, two independent sums).
    __shared__ u64 tab[NS * BC_TG * 2];
    __shared__ ModP tm[BC_TG];
    const int N = 1 << T.log_n;
    const int i = 2 * (blockIdx.x * TPB + threadIdx.x);
    const int p = blockIdx.z % D.npoly, c = blockIdx.z / D.npoly;
    const int t0 = blockIdx.y * BC_TG, nt = min(D.nt - t0, BC_TG);
    for (int e = threadIdx.x; e < NS * nt * 2; e += TPB) {
        const int sI = e / (nt * 2), rem = e % (nt * 2), tt = rem >> 1, w = rem & 1;
        const u64 v = D.tab[((int64_t)sI * D.tab_ld + D.tcol[t0 + tt]) * 2 + w];
        if (w == 0) {  // the multiplier, split at bit 30 (hi word: bits 30.., lo word: bits 0..29)
            const Split30 sp = split30(v);
            tab[(sI * BC_TG + tt) * 2] = ((u64)sp.hi << 32) | sp.lo;
        } else {
            tab[(sI * BC_TG + tt) * 2 + 1] = v;
        }
    }
    if (threadIdx.x < nt) tm[threadIdx.x] = T.mods[D.dmod[t0 + threadIdx.x]];
    __syncthreads();
    if (i >= N) return;
    Split30 y[NS][2];
    u64 negm[NS][2];
    const u64* src = D.src + c * D.src_cstride + p * D.src_pstride;
#pragma unroll
    for (int s = 0; s < NS; s++) {
        const ModP m = T.mods[D.smod[s]];
        const u64x2 x = ld2(src + (int64_t)s * N + i);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const u64 v = mul_shoup(x[h], D.hinv[s], D.hinv_sh[s], m.q);
            y[s][h] = split30(v);
            negm[s][h] = v > m.half ? ~0ull : 0ull;
        }
    }
    u64* dst = D.dst + c * D.dst_cstride + p * D.dst_pstride;
    for (int tt = 0; tt < nt; tt++) {
        const ModP m = tm[tt];
        // NS <= 8 terms y_s t_s plus the centering corrections: column sums stay below 2^64
        Acc3 acc0 = {0, 0, 0}, acc1 = {0, 0, 0};
#pragma unroll
        for (int s = 0; s < NS; s++) {
            const u64 tw = tab[(s * BC_TG + tt) * 2], tc = tab[(s * BC_TG + tt) * 2 + 1];
            const Split30 ts = {(u32)tw, (u32)(tw >> 32)};
            mac3(acc0, y[s][0], ts);
            mac3(acc1, y[s][1], ts);
            acc0.c0 += tc & negm[s][0];
            acc1.c0 += tc & negm[s][1];
        }
        st2(dst + (int64_t)D.doff[t0 + tt] * N + i, u64x2{redc3(acc0, m.q, m.qninv), redc3(acc1, m.q, m.qninv)});
    }
}

void launch_baseconv(const DevTables& T, const ConvDesc& D, hipStream_t st) {
    ProfScope prof_(PK_BASECONV, (double)(D.ns + D.nt) * D.npoly * D.nct * 8.0 * (1 << T.log_n), st);
    const int N = 1 << T.log_n;
    if (D.prescaled) throw std::runtime_error("base conversion: prescaled sources are read by conv_cols only");
    if (misaligned16(D.src) || misaligned16(D.dst) || ((D.src_pstride | D.dst_pstride | D.src_cstride |
                                                         D.dst_cstride) & 1))
        throw std::runtime_error("base conversion operand not 16-byte aligned");
    dim3 grid(ceil_div(N, 2 * TPB), ceil_div(D.nt, BC_TG), D.npoly * D.nct);
    switch (D.ns) {
        case 1: HE_LAUNCH(k_baseconv<1>, grid, dim3(TPB), 0, st, T, D); break;
        case 2: HE_LAUNCH(k_baseconv<2>, grid, dim3(TPB), 0, st, T, D); break;
        case 3: HE_LAUNCH(k_baseconv<3>, grid, dim3(TPB), 0, st, T, D); break;
        case 4: HE_LAUNCH(k_baseconv<4>, grid, dim3(TPB), 0, st, T, D); break;
        case 5: HE_LAUNCH(k_baseconv<5>, grid, dim3(TPB), 0, st, T, D); break;
        case 6: HE_LAUNCH(k_baseconv<6>, grid, dim3(TPB), 0, st, T, D); break;
        case 7: HE_LAUNCH(k_baseconv<7>, grid, dim3(TPB), 0, st, T, D); break;
        default: HE_LAUNCH(k_baseconv<8>, grid, dim3(TPB), 0, st, T, D); break;
    }
}

template <bool MD>
static void launch_conv_cols_ns(int ns, dim3 grid, hipStream_t st, const DevTables& T, const ConvDesc& D) {
    switch (ns) {
        case 1: HE_LAUNCH((k_conv_cols<1, MD>), grid, dim3(TPB), 0, st, T, D); break;
        case 2: HE_LAUNCH((k_conv_cols<2, MD>), grid, dim3(TPB), 0, st, T, D); break;
        case 3: HE_LAUNCH((k_conv_cols<3, MD>), grid, dim3(TPB), 0, st, T, D); break;
        case 4: HE_LAUNCH((k_conv_cols<4, MD>), grid, dim3(TPB), 0, st, T, D); break;
        case 5: HE_LAUNCH((k_conv_cols<5, MD>), grid, dim3(TPB), 0, st, T, D); break;
        case 6: HE_LAUNCH((k_conv_cols<6, MD>), grid, dim3(TPB), 0, st, T, D); break;
        case 7: HE_LAUNCH((k_conv_cols<7, MD>), grid, dim3(TPB), 0, st, T, D); break;
        default: HE_LAUNCH((k_conv_cols<8, MD>), grid, dim3(TPB), 0, st, T, D); break;
    }
}

bool conv_cols_fits(const DevTables& T, int ns) { return T.n1_log >= 1 && ns >= 1 && ns <= HE_MAXSRC; }

void launch_conv_cols(const DevTables& T, const ConvDesc& D, hipStream_t st) {
    if (!conv_cols_fits(T, D.ns) || !D.prescaled || D.nt < 1 || D.nt > HE_MAXT || D.ndig < 0 ||
        D.ndig > HE_MAXDIG)
        throw std::runtime_error("conv_cols: unsupported shape");
    bool odd = (D.src_pstride | D.dst_pstride | D.src_cstride | D.dst_cstride) & 1;
    double src_limbs = D.ns;  // source limbs read per (poly, ciphertext)
    if (D.ndig) {
        src_limbs = 0;
        for (int d = 0; d < D.ndig; ++d) {
            if (D.dns[d] < 1 || D.dns[d] > D.ns) throw std::runtime_error("conv_cols: unsupported shape");
            odd = odd || (D.dsrc[d] & 1);
            src_limbs += D.dns[d];
        }
        for (int t = 0; t < D.nt; ++t)
            if (D.tdig[t] >= D.ndig) throw std::runtime_error("conv_cols: unsupported shape");
    }
    if (misaligned16(D.src) || misaligned16(D.dst) || odd)
        throw std::runtime_error("conv_cols operand not 16-byte aligned");
    const int N = 1 << T.log_n;
    const double units = (double)D.nt * D.npoly * D.nct;
    double fpu = 0;
    for (int t = 0; t < D.nt; ++t) fpu += (double)((T.fp64_mods >> D.dmod[t]) & 1) * D.npoly * D.nct;
    ProfScope prof_(PK_CONV_COLS, (src_limbs * D.npoly * D.nct + units) * 8.0 * N, st,
                    units * (N / 2) * T.n1_log, fpu * (N / 2) * T.n1_log);
    dim3 grid((N / NTT_E) * D.npoly * D.nct * D.nt);
    if (D.ndig)
        launch_conv_cols_ns<true>(D.ns, grid, st, T, D);
    else
        launch_conv_cols_ns<false>(D.ns, grid, st, T, D);
}

// ------------------------------------------------------------------ ChaCha20 samplers
__device__ __forceinline__ u32 rotl(u32 v, int c) { return (v << c) | (v >> (32 - c)); }
#define CQR(a, b, c, d)                    \
    a += b; d ^= a; d = rotl(d, 16);       \
    c += d; b ^= c; b = rotl(b, 12);       \
    a += b; d ^= a; d = rotl(d, 8);        \
    c += d; b ^= c; b = rotl(b, 7);

// RFC 8439 section 2.3 block function; key = seed (little-endian) zero-extended,
// nonce = (purpose, index lo, index hi).
__device__ void chacha_block(u64 seed, u32 purpose, u64 index, u32 counter, u32 out[16]) {
    const u32 st[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u, (u32)seed, (u32)(seed >> 32), 0, 0,
                        0, 0, 0, 0, counter, purpose, (u32)index, (u32)(index >> 32)};
    u32 x[16];
#pragma unroll
    for (int i = 0; i < 16; i++) x[i] = st[i];
#pragma unroll
    for (int r = 0; r < 10; r++) {
        CQR(x[0], x[4], x[8], x[12]);
        CQR(x[1], x[5], x[9], x[13]);
        CQR(x[2], x[6], x[10], x[14]);
        CQR(x[3], x[7], x[11], x[15]);
        CQR(x[0], x[5], x[10], x[15]);
        CQR(x[1], x[6], x[11], x[12]);
        CQR(x[2], x[7], x[8], x[13]);
        CQR(x[3], x[4], x[9], x[14]);
    }
#pragma unroll
    for (int i = 0; i < 16; i++) out[i] = x[i] + st[i];
}

__device__ __forceinline__ u64 signed_to_res(int64_t v, u64 q) { return v >= 0 ? (u64)v : q - (u64)(-v); }

// ternary / Gaussian: one 64-bit word per coefficient, word w = block w/8, words 2(w%8)+{0,1}
__global__ __launch_bounds__(TPB) void k_sample_small(DevTables T, Jobs J, SampleArgs A) {
    const int N = 1 << T.log_n;
    const int blk = blockIdx.x * TPB + threadIdx.x;
    if (blk * 8 >= N) return;
    u32 o[16];
    chacha_block(A.seed, A.purpose, A.index, (u32)blk, o);
    for (int w = 0; w < 8; w++) {
        const u64 word = (u64)o[2 * w] | ((u64)o[2 * w + 1] << 32);
        int64_t v;
        if (A.kind == 0) {
            v = (int64_t)(word % 3) - 1;
        } else {
            const u64 u = word >> 1;
            int mag = 0;
            for (int k = 0; k < 19; k++) mag += (u >= A.cdt[k]) ? 1 : 0;
            v = (word & 1) ? -mag : mag;
        }
        const int x = blk * 8 + w;
        for (int k = 0; k < J.n; k++) {
            const u64 q = T.mods[J.mod[k]].q;
            J.base[(int64_t)J.off[k] * N + x] = signed_to_res(v, q);
        }
    }
}

// uniform mod q: two words per coefficient, value = (w[2x+1] 2^64 + w[2x]) mod q
__global__ __launch_bounds__(TPB) void k_sample_uniform(DevTables T, Jobs J, SampleArgs A) {
    const int N = 1 << T.log_n;
    const int blk = blockIdx.x * TPB + threadIdx.x;
    const int k = blockIdx.y;
    if (blk * 4 >= N) return;
    u32 o[16];
    chacha_block(A.seed, A.purpose, A.uidx[k], (u32)blk, o);
    const ModP m = T.mods[J.mod[k]];
    for (int w = 0; w < 4; w++) {
        const u64 lo = (u64)o[4 * w] | ((u64)o[4 * w + 1] << 32);
        const u64 hi = (u64)o[4 * w + 2] | ((u64)o[4 * w + 3] << 32);
        // (hi 2^64 + lo) mod q = REDC(hi' 2^64 + lo) * R mod q with hi' = hi mod q
        const u64 t = redc(lo, reduce64(hi, m), m.q, m.qninv);
        J.base[(int64_t)J.off[k] * N + blk * 4 + w] = redc(t * m.r2, __umul64hi(t, m.r2), m.q, m.qninv);
    }
}

void launch_sample(const DevTables& T, const Jobs& J, const SampleArgs& A, hipStream_t st) {
    ProfScope prof_(PK_EW, 1.0 * J.n * 8.0 * (1 << T.log_n), st);
    const int N = 1 << T.log_n;
    if (A.kind == 2) {
        dim3 grid(ceil_div(N / 4, TPB), J.n);
        HE_LAUNCH(k_sample_uniform, grid, dim3(TPB), 0, st, T, J, A);
    } else {
        dim3 grid(ceil_div(N / 8, TPB));
        HE_LAUNCH(k_sample_small, grid, dim3(TPB), 0, st, T, J, A);
    }
}

// ------------------------------------------------------------------ element-wise
__global__ __launch_bounds__(TPB) void k_ew(DevTables T, ModMap mm, int npoly, u64* out, int64_t out_ps,
                                            const u64* a, int64_t a_ps, const u64* b, int64_t b_ps, int op,
                                            int64_t out_cs, int64_t a_cs, int64_t b_cs) {
    const int N = 1 << T.log_n;
    const int i = blockIdx.x * TPB + threadIdx.x;
    const int l = blockIdx.y, p = blockIdx.z % npoly, c = blockIdx.z / npoly;
    const ModP m = T.mods[mm(l)];
    const int64_t o = (int64_t)l * N + i;
    out += c * out_cs;
    a += c * a_cs;
    b += c * b_cs;
    const u64 x = a[p * a_ps + o], y = b[p * b_ps + o];
    u64 r;
    switch (op) {
        case EW_ADD: r = add_mod(x, y, m.q); break;
        case EW_SUB: r = sub_mod(x, y, m.q); break;
        case EW_MUL_MONT: r = mul_mont(x, y, m.q, m.qninv); break;
        default: r = mul_plain(x, y, m); break;
    }
    out[p * out_ps + o] = r;
}

void launch_ew(const DevTables& T, ModMap mm, int nl, int npoly, u64* out, int64_t out_ps, const u64* a,
               int64_t a_ps, const u64* b, int64_t b_ps, int op, hipStream_t st, int nct, int64_t out_cs,
               int64_t a_cs, int64_t b_cs) {
    ProfScope prof_(PK_EW, 3.0 * nl * npoly * nct * 8.0 * (1 << T.log_n), st);
    const int N = 1 << T.log_n;
    dim3 grid(ceil_div(N, TPB), nl, npoly * nct);
    HE_LAUNCH(k_ew, grid, dim3(TPB), 0, st, T, mm, npoly, out, out_ps, a, a_ps, b, b_ps, op, out_cs, a_cs,
                       b_cs);
}

__global__ __launch_bounds__(TPB) void k_mul_const(DevTables T, ModMap mm, u64* out, int64_t out_ps,
                                                   const u64* a, int64_t a_ps, const u64* c, const u64* c_sh) {
    const int N = 1 << T.log_n;
    const int i = blockIdx.x * TPB + threadIdx.x;
    const int l = blockIdx.y, p = blockIdx.z;
    const u64 q = T.mods[mm(l)].q;
    const int64_t o = (int64_t)l * N + i;
    out[p * out_ps + o] = mul_shoup(a[p * a_ps + o], c[l], c_sh[l], q);
}

void launch_mul_const(const DevTables& T, ModMap mm, int nl, int npoly, u64* out, int64_t out_ps, const u64* a,
                      int64_t a_ps, const u64* c, const u64* c_sh, hipStream_t st) {
    ProfScope prof_(PK_EW, 2.0 * nl * npoly * 8.0 * (1 << T.log_n), st);
    const int N = 1 << T.log_n;
    dim3 grid(ceil_div(N, TPB), nl, npoly);
    HE_LAUNCH(k_mul_const, grid, dim3(TPB), 0, st, T, mm, out, out_ps, a, a_ps, c, c_sh);
}

// position j of the bit-reversed evaluation layout holds a(psi^(2 brev(j) + 1)); sigma_g
// evaluates there as a(psi^(g (2 brev(j) + 1)))
__device__ __forceinline__ int perm_g(int j, u64 g, int log_n) {
    const u32 two_n_mask = (2u << log_n) - 1;
    const u32 e = 2 * brev_bits((u32)j, log_n) + 1;
    const u32 e2 = (u32)(((u64)e * g) & two_n_mask);
    return (int)brev_bits((e2 - 1) >> 1, log_n);
}

__global__ __launch_bounds__(TPB) void k_automorph(DevTables T, int npoly, u64* out, int64_t out_ps, const u64* in,
                                                   int64_t in_ps, u64 g, int64_t out_cs, int64_t in_cs) {
    const int N = 1 << T.log_n;
    const int i = blockIdx.x * TPB + threadIdx.x;
    const int l = blockIdx.y, p = blockIdx.z % npoly, c = blockIdx.z / npoly;
    out[c * out_cs + p * out_ps + (int64_t)l * N + i] = in[c * in_cs + p * in_ps + (int64_t)l * N + perm_g(i, g, T.log_n)];
}

void launch_automorph(const DevTables& T, int nl, int npoly, u64* out, int64_t out_ps, const u64* in,
                      int64_t in_ps, u64 g, hipStream_t st, int nct, int64_t out_cs, int64_t in_cs) {
    ProfScope prof_(PK_AUTOMORPH, 2.0 * nl * npoly * nct * 8.0 * (1 << T.log_n), st);
    const int N = 1 << T.log_n;
    dim3 grid(ceil_div(N, TPB), nl, npoly * nct);
    HE_LAUNCH(k_automorph, grid, dim3(TPB), 0, st, T, npoly, out, out_ps, in, in_ps, g, out_cs, in_cs);
}

__global__ __launch_bounds__(TPB) void k_to_mont(DevTables T, ModMap mm, u64* x, int64_t ps) {
    const int N = 1 << T.log_n;
    const int i = blockIdx.x * TPB + threadIdx.x;
    const int l = blockIdx.y, p = blockIdx.z;
    const ModP m = T.mods[mm(l)];
    u64* v = x + p * ps + (int64_t)l * N + i;
    *v = to_mont(*v, m);
}

void launch_to_mont(const DevTables& T, ModMap mm, int nl, int npoly, u64* x, int64_t ps, hipStream_t st) {
    ProfScope prof_(PK_EW, 2.0 * nl * npoly * 8.0 * (1 << T.log_n), st);
    const int N = 1 << T.log_n;
    dim3 grid(ceil_div(N, TPB), nl, npoly);
    HE_LAUNCH(k_to_mont, grid, dim3(TPB), 0, st, T, mm, x, ps);
}

__global__ __launch_bounds__(TPB) void k_swk_finish(DevTables T, u64* b, const u64* a, const u64* e,
                                                    const u64* s, const u64* sp, const u64* pmod,
                                                    const uint8_t* in_digit) {
    const int N = 1 << T.log_n;
    const int i = blockIdx.x * TPB + threadIdx.x;
    const int l = blockIdx.y;
    const ModP m = T.mods[l];
    const int64_t o = (int64_t)l * N + i;
    u64 v = sub_mod(e[o], mul_plain(a[o], s[o], m), m.q);
    if (in_digit[l]) v = add_mod(v, mul_plain(pmod[l], sp[o], m), m.q);
    b[o] = v;
}

void launch_swk_finish(const DevTables& T, int M, u64* b, const u64* a, const u64* e, const u64* s, const u64* sp,
                       const u64* pmod, const uint8_t* in_digit, hipStream_t st) {
    ProfScope prof_(PK_EW, 6.0 * M * 8.0 * (1 << T.log_n), st);
    const int N = 1 << T.log_n;
    dim3 grid(ceil_div(N, TPB), M);
    HE_LAUNCH(k_swk_finish, grid, dim3(TPB), 0, st, T, b, a, e, s, sp, pmod, in_digit);
}

// ------------------------------------------------------------------ key switching
// Hybrid key switching (Han-Ki 2020): inner product of the lifted digits with the
// switching key over Q_l and P.  The automorphism of a rotation is fused as a
// gather: the digits of sigma_g(c1) are the permuted digits of c1 (hoisting).
// The key values of one (limb, coefficient) are loaded once and reused for every
// ciphertext of the group: a switching key crosses HBM once per launch.
// one rotation's key-switch inner product of one member, reduced: sum_j x_j key_j (+ P
// sigma_g(c0) on the Q limbs), optionally times a Montgomery-form mask; x are the member's
// lift words at the automorphism source position
// up to seven digits (plus the c0 term) use the carry-free column sums with the key words
// split at bit 30; eight digits use 128-bit accumulation
template <int NB>
using IpKey = typename std::conditional<(NB <= 7), Split30, u64>::type;
template <int NB>
__device__ __forceinline__ IpKey<NB> ip_key(u64 v) {
    if constexpr (NB <= 7) return split30(v);
    else return v;
}

// The inner products of all NR rotations of one member for one slot: sum_r sum_j x_rj k_rj
// (+ z_r pm_r on the Q limbs), the masks already folded into the key words and the c0
// constant (mask . sum_j x_j k_j = sum_j x_j (k_j . mask) mod q).  Up to eight products share
// one set of column sums and one REDC; otherwise each rotation is reduced on its own.
template <int NB, int NR>
__device__ __forceinline__ void ip_reduce(const u64 (&x)[NR][NB], const u64 (&z)[NR], const IpKey<NB> (&kb)[NR][NB],
                                          const IpKey<NB> (&ka)[NR][NB], const IpKey<NB> (&pm)[NR], bool with_c0,
                                          const ModP& m, u64& v0, u64& v1) {
    if constexpr (NB <= 7 && NR * (NB + 1) <= 8) {
        Acc3 a0 = {0, 0, 0}, a1 = {0, 0, 0};
#pragma unroll
        for (int r = 0; r < NR; r++) {
#pragma unroll
            for (int j = 0; j < NB; j++) {
                const Split30 xs = split30(x[r][j]);
                mac3(a0, xs, kb[r][j]);
                mac3(a1, xs, ka[r][j]);
            }
            if (with_c0) mac3(a0, split30(z[r]), pm[r]);
        }
        v0 = redc3(a0, m.q, m.qninv);
        v1 = redc3(a1, m.q, m.qninv);
    } else if constexpr (NB <= 7) {
        v0 = v1 = 0;
#pragma unroll
        for (int r = 0; r < NR; r++) {
            Acc3 a0 = {0, 0, 0}, a1 = {0, 0, 0};
#pragma unroll
            for (int j = 0; j < NB; j++) {
                const Split30 xs = split30(x[r][j]);
                mac3(a0, xs, kb[r][j]);
                mac3(a1, xs, ka[r][j]);
            }
            if (with_c0) mac3(a0, split30(z[r]), pm[r]);
            v0 = add_mod(v0, redc3(a0, m.q, m.qninv), m.q);
            v1 = add_mod(v1, redc3(a1, m.q, m.qninv), m.q);
        }
    } else {
        v0 = v1 = 0;
#pragma unroll
        for (int r = 0; r < NR; r++) {
            Acc128 a0 = {0, 0}, a1 = {0, 0};
#pragma unroll
            for (int j = 0; j < NB; j++) {
                mac128(a0, x[r][j], kb[r][j]);
                mac128(a1, x[r][j], ka[r][j]);
            }
            if (with_c0) mac128(a0, z[r], pm[r]);
            v0 = add_mod(v0, redc(a0.lo, a0.hi, m.q, m.qninv), m.q);
            v1 = add_mod(v1, redc(a1.lo, a1.hi, m.q, m.qninv), m.q);
        }
    }
}

// Grid (nset N / TPB, ne): one thread per (set, slot, extended limb) for every member, so
// each key word (and mask word) is read once per group.  The digit count NB is a template
// parameter so that the key words stay in registers; the member loop is software-
// pipelined (the next member's lift and c0 words are loaded before the current member's
// arithmetic) to keep more loads in flight.  sigma_g maps each aligned block of TPB slots
// onto one aligned block of TPB source slots (the top bits of perm_g(i) depend only on the
// top bits of i), so with several sets the blocks are numbered by the lift block they
// gather: the sets' blocks of one source block get consecutive numbers on one XCD
// (workgroups are dealt to the 8 XCDs round-robin), run together there, and read the
// lift and c0 words of each member through that XCD's L2 once for all sets.
template <int NB, int NR>
__global__ __launch_bounds__(TPB) void k_inner_product(DevTables T, IpDesc D) {
    const int N = 1 << T.log_n, nb = N / TPB;
    int xb = blockIdx.x, sj = 0;
    if (D.nset > 1) {
        int R;
        if ((nb & 7) == 0) {
            const int hi = xb >> 3;
            sj = hi % D.nset;
            R = (hi / D.nset) * 8 + (xb & 7);
        } else {
            sj = xb / nb;
            R = xb % nb;
        }
        // the output block whose first rotation gathers from source block R
        xb = perm_g(R * TPB, D.s[sj].ginv, T.log_n) / TPB;
    }
    const IpSet& S = D.s[sj];
    const int i = xb * TPB + threadIdx.x;
    const int t = blockIdx.y;
    const int mi = D.mod[t];
    const ModP m = T.mods[mi];
    // key words (and P . c0's constant) with the rotation's mask folded in, Montgomery form
    const bool with_c0 = D.c0 && t < D.nq;
    const u64 pmont = with_c0 ? D.pmont[t] : 0;
    IpKey<NB> kb[NR][NB], ka[NR][NB], pm[NR];
    int src[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const u64 g = r ? S.g2 : S.g;
        const u64* key = r ? S.key2 : S.key;
        const u64* mask = r ? S.mask2 : S.mask;
        src[r] = g == 1 ? i : perm_g(i, g, T.log_n);
        const u64 mk = mask ? mask[(int64_t)mi * N + i] : 0;
#pragma unroll
        for (int j = 0; j < NB; j++) {
            u64 b = ldnt(key + (((int64_t)j * 2 + 0) * D.M + mi) * N + i);
            u64 a = ldnt(key + (((int64_t)j * 2 + 1) * D.M + mi) * N + i);
            if (mask) {
                b = mul_mont(b, mk, m.q, m.qninv);
                a = mul_mont(a, mk, m.q, m.qninv);
            }
            kb[r][j] = ip_key<NB>(b);
            ka[r][j] = ip_key<NB>(a);
        }
        pm[r] = ip_key<NB>(mask ? mul_mont(pmont, mk, m.q, m.qninv) : pmont);
    }
    // the second rotation may read another ciphertext's lift and c0 (a rotation-sum term); the
    // digit whose own limbs include t (none for the special primes) is read from the lifted
    // polynomial itself.  Every operand word of member c sits at a block-uniform base plus c
    // times a uniform stride plus the lane's gather offset, so the member loop only advances
    // uniform pointers and loads with one 32-bit lane offset per rotation.
    int jo = -1;
#pragma unroll
    for (int j = 0; j < NB; j++)
        if (t >= D.dlo[j] && t < D.dhi[j]) jo = j;
    const u64* xp[NR][NB];
    int64_t xcs[NR][NB];
    const u64* zb[NR];
    int64_t zcs[NR];
    uint32_t so[NR];  // byte offset of the lane's source slot
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const bool other = r && S.lift2;
        const u64* lift = (other ? S.lift2 : D.lift) + (int64_t)t * N;
        const u64* own = other ? S.own2 : D.own;
        const int64_t owncs = other ? S.own2_cs : D.own_cs;
#pragma unroll
        for (int j = 0; j < NB; j++) {
            const bool from_own = own && j == jo;
            xp[r][j] = from_own ? own + (int64_t)t * N : lift + (int64_t)j * D.ne * N;
            xcs[r][j] = from_own ? owncs : D.lift_cs;
        }
        zb[r] = with_c0 ? (other ? S.c0_2 : D.c0) + (int64_t)t * N : nullptr;
        zcs[r] = other ? S.c0_2_cs : D.c0_cs;
        so[r] = (uint32_t)src[r] * 8u;
    }
    auto at = [](const u64* base, uint32_t off) { return *reinterpret_cast<const u64*>(reinterpret_cast<const char*>(base) + off); };
    auto load = [&](u64(&xo)[NR][NB], u64(&zo)[NR]) {
#pragma unroll
        for (int r = 0; r < NR; r++) {
#pragma unroll
            for (int j = 0; j < NB; j++) xo[r][j] = at(xp[r][j], so[r]);
            zo[r] = with_c0 ? at(zb[r], so[r]) : 0;
        }
    };
    auto advance = [&]() {
#pragma unroll
        for (int r = 0; r < NR; r++) {
#pragma unroll
            for (int j = 0; j < NB; j++) xp[r][j] += xcs[r][j];
            if (with_c0) zb[r] += zcs[r];
        }
    };
    u64* u0 = D.u + (int64_t)sj * D.nct * D.u_cs + (int64_t)t * N;
    u64* u1 = u0 + (int64_t)D.ne * N;
    const uint32_t io = (uint32_t)i * 8u;
    auto finish = [&](const u64(&xv)[NR][NB], const u64(&zv)[NR]) {
        u64 v0, v1;
        ip_reduce<NB, NR>(xv, zv, kb, ka, pm, with_c0, m, v0, v1);
        u64* p0 = reinterpret_cast<u64*>(reinterpret_cast<char*>(u0) + io);
        u64* p1 = reinterpret_cast<u64*>(reinterpret_cast<char*>(u1) + io);
        if (D.accumulate) {
            v0 = add_mod(v0, *p0, m.q);
            v1 = add_mod(v1, *p1, m.q);
        }
        *p0 = v0;
        *p1 = v1;
        u0 += D.u_cs;
        u1 += D.u_cs;
    };
    // software pipeline over the members, three register sets in turn: the lift and c0 words
    // of the next two members are in flight during the current member's arithmetic (one
    // member's arithmetic is shorter than a load's latency under full bandwidth)
    u64 x0[NR][NB], z0[NR], x1[NR][NB], z1[NR], x2[NR][NB], z2[NR];
    load(x0, z0);
    advance();
    if (D.nct > 1) {
        load(x1, z1);
        advance();
    }
    for (int c = 0; c < D.nct; c += 3) {
        if (c + 2 < D.nct) {
            load(x2, z2);
            advance();
        }
        finish(x0, z0);
        if (c + 1 >= D.nct) break;
        if (c + 3 < D.nct) {
            load(x0, z0);
            advance();
        }
        finish(x1, z1);
        if (c + 2 >= D.nct) break;
        if (c + 4 < D.nct) {
            load(x1, z1);
            advance();
        }
        finish(x2, z2);
    }
}

template <int NB>
static void launch_ip_nb(const DevTables& T, const IpDesc& D, dim3 grid, hipStream_t st) {
    if (D.nrot == 2)
        HE_LAUNCH((k_inner_product<NB, 2>), grid, dim3(TPB), 0, st, T, D);
    else
        HE_LAUNCH((k_inner_product<NB, 1>), grid, dim3(TPB), 0, st, T, D);
}

void launch_inner_product(const DevTables& T, const IpDesc& D, hipStream_t st) {
    const int nr = D.nrot == 2 ? 2 : 1, ns = D.nset;
    const int N = 1 << T.log_n;
    if (ns < 1 || ns > IP_MAXSET) throw std::runtime_error("inner product: set count out of range");
    if (N < TPB) throw std::runtime_error("inner product: ring smaller than a block");
    // keys (and masks) once per group; per member the lift digits and c0 once (the rotations
    // of a pair and the sets of a launch gather the same lift) and u per set
    double masks = 0, lifts = 1;
    for (int j = 0; j < ns; ++j) {
        masks += (D.s[j].mask ? 1.0 : 0.0) + (nr == 2 && D.s[j].mask2 ? 1.0 : 0.0);
        if (nr == 2 && D.s[j].lift2) lifts += 1;  // another ciphertext's lift and c0
    }
    const double words = (double)D.ne * (ns * nr * 2.0 * D.beta + masks +
                                         D.nct * (lifts * D.beta + ns * (D.accumulate ? 4.0 : 2.0))) +
                         (D.c0 ? lifts * D.nq * D.nct : 0.0);
    for (int j = 0; j < ns; ++j) {
        if (D.s[j].lift2 && (nr != 2 || (D.c0 != nullptr) != (D.s[j].c0_2 != nullptr)))
            throw std::runtime_error("inner product: second lift without a second rotation or c0");
        if (D.s[j].lift2 && (D.own != nullptr) != (D.s[j].own2 != nullptr))
            throw std::runtime_error("inner product: lifts with and without their own limbs in one launch");
    }
    ProfScope prof_(PK_INNER, words * 8.0 * N, st);
    dim3 grid((N / TPB) * ns, D.ne);
    switch (D.beta) {
        case 1: launch_ip_nb<1>(T, D, grid, st); break;
        case 2: launch_ip_nb<2>(T, D, grid, st); break;
        case 3: launch_ip_nb<3>(T, D, grid, st); break;
        case 4: launch_ip_nb<4>(T, D, grid, st); break;
        case 5: launch_ip_nb<5>(T, D, grid, st); break;
        case 6: launch_ip_nb<6>(T, D, grid, st); break;
        case 7: launch_ip_nb<7>(T, D, grid, st); break;
        case 8: launch_ip_nb<8>(T, D, grid, st); break;
        default: abort();
    }
}

__global__ __launch_bounds__(TPB) void k_moddown_combine(DevTables T, int npoly, const u64* u, int64_t u_ps,
                                                         const u64* conv, int64_t conv_ps, const u64* pinv,
                                                         const u64* pinv_sh, const u64* add, int64_t add_ps,
                                                         u64* out, int64_t out_ps, int64_t u_cs, int64_t conv_cs,
                                                         int64_t add_cs, int64_t out_cs) {
    const int N = 1 << T.log_n;
    const int i = blockIdx.x * TPB + threadIdx.x;
    const int l = blockIdx.y, p = blockIdx.z % npoly, c = blockIdx.z / npoly;
    u += c * u_cs;
    conv += c * conv_cs;
    if (add) add += c * add_cs;
    out += c * out_cs;
    const u64 q = T.mods[l].q;
    const int64_t o = (int64_t)l * N + i;
    u64 v = mul_shoup(sub_mod(u[p * u_ps + o], conv[p * conv_ps + o], q), pinv[l], pinv_sh[l], q);
    if (add) v = add_mod(v, add[p * add_ps + o], q);
    out[p * out_ps + o] = v;
}

void launch_moddown_combine(const DevTables& T, int nl, int npoly, const u64* u, int64_t u_ps, const u64* conv,
                            int64_t conv_ps, const u64* pinv, const u64* pinv_sh, const u64* add, int64_t add_ps,
                            u64* out, int64_t out_ps, hipStream_t st, int nct, int64_t u_cs, int64_t conv_cs,
                            int64_t add_cs, int64_t out_cs) {
    ProfScope prof_(PK_MODDOWN, (add ? 4.0 : 3.0) * nl * npoly * nct * 8.0 * (1 << T.log_n), st);
    const int N = 1 << T.log_n;
    dim3 grid(ceil_div(N, TPB), nl, npoly * nct);
    HE_LAUNCH(k_moddown_combine, grid, dim3(TPB), 0, st, T, npoly, u, u_ps, conv, conv_ps, pinv, pinv_sh,
                       add, add_ps, out, out_ps, u_cs, conv_cs, add_cs, out_cs);
}

// ------------------------------------------------------------------ n-ary sum
__global__ __launch_bounds__(TPB) void k_sum_many(DevTables T, SumDesc D, u64* out, int64_t out_ps, int accumulate) {
    const int N = 1 << T.log_n;
    const int i = blockIdx.x * TPB + threadIdx.x;
    const int l = blockIdx.y, p = blockIdx.z;
    const u64 q = T.mods[l].q;
    const int64_t o = (int64_t)l * N + i;
    u64 v = accumulate ? out[p * out_ps + o] : 0;
    for (int t = 0; t < D.n; t++) v = add_mod(v, D.in[t][p * D.in_ps[t] + o], q);
    out[p * out_ps + o] = v;
}

void launch_sum_many(const DevTables& T, int nl, int npoly, const SumDesc& D, u64* out, int64_t out_ps,
                     int accumulate, hipStream_t st) {
    ProfScope prof_(PK_EW, (D.n + 1.0 + accumulate) * nl * npoly * 8.0 * (1 << T.log_n), st);
    const int N = 1 << T.log_n;
    dim3 grid(ceil_div(N, TPB), nl, npoly);
    HE_LAUNCH(k_sum_many, grid, dim3(TPB), 0, st, T, D, out, out_ps, accumulate);
}

// ------------------------------------------------------------------ rescale
__global__ __launch_bounds__(TPB) void k_rescale_spread(DevTables T, const u64* last, int64_t last_ps, int last_mod,
                                                        u64* tmp, int64_t tmp_ps) {
    const int N = 1 << T.log_n;
    const int i = blockIdx.x * TPB + threadIdx.x;
    const int l = blockIdx.y, p = blockIdx.z;  // p runs over (ciphertext, poly) pairs
    const ModP ml = T.mods[last_mod], m = T.mods[l];
    const u64 r = last[p * last_ps + i];
    u64 v = reduce64(r, m);
    if (r > ml.half) v = sub_mod(v, reduce64(ml.q, m), m.q);
    tmp[p * tmp_ps + (int64_t)l * N + i] = v;
}

void launch_rescale_spread(const DevTables& T, int nl_out, int npoly, const u64* last, int64_t last_ps,
                           int last_mod, u64* tmp, int64_t tmp_ps, hipStream_t st) {
    ProfScope prof_(PK_RS_SPREAD, (1.0 + nl_out) * npoly * 8.0 * (1 << T.log_n), st);
    const int N = 1 << T.log_n;
    dim3 grid(ceil_div(N, TPB), nl_out, npoly);
    HE_LAUNCH(k_rescale_spread, grid, dim3(TPB), 0, st, T, last, last_ps, last_mod, tmp, tmp_ps);
}

__global__ __launch_bounds__(TPB) void k_rescale_combine(DevTables T, int npoly, const u64* c, int64_t c_ps,
                                                         const u64* tmp, int64_t tmp_ps, const u64* qinv,
                                                         const u64* qinv_sh, u64* out, int64_t out_ps, int64_t c_cs,
                                                         int64_t tmp_cs, int64_t out_cs) {
    const int N = 1 << T.log_n;
    const int i = blockIdx.x * TPB + threadIdx.x;
    const int l = blockIdx.y, p = blockIdx.z % npoly, ct = blockIdx.z / npoly;
    const u64 q = T.mods[l].q;
    const int64_t o = (int64_t)l * N + i;
    out[ct * out_cs + p * out_ps + o] =
        mul_shoup(sub_mod(c[ct * c_cs + p * c_ps + o], tmp[ct * tmp_cs + p * tmp_ps + o], q), qinv[l], qinv_sh[l], q);
}

void launch_rescale_combine(const DevTables& T, int nl_out, int npoly, const u64* c, int64_t c_ps, const u64* tmp,
                            int64_t tmp_ps, const u64* qinv, const u64* qinv_sh, u64* out, int64_t out_ps,
                            hipStream_t st, int nct, int64_t c_cs, int64_t tmp_cs, int64_t out_cs) {
    ProfScope prof_(PK_RS_COMBINE, 3.0 * nl_out * npoly * nct * 8.0 * (1 << T.log_n), st);
    const int N = 1 << T.log_n;
    dim3 grid(ceil_div(N, TPB), nl_out, npoly * nct);
    HE_LAUNCH(k_rescale_combine, grid, dim3(TPB), 0, st, T, npoly, c, c_ps, tmp, tmp_ps, qinv, qinv_sh, out,
                       out_ps, c_cs, tmp_cs, out_cs);
}

// ------------------------------------------------------------------ products
__global__ __launch_bounds__(TPB) void k_tensor(DevTables T, const u64* a, int64_t a_ps, const u64* b,
                                                int64_t b_ps, u64* d, int64_t d_ps, int acc, int64_t a_cs,
                                                int64_t b_cs, int64_t d_cs) {
    const int N = 1 << T.log_n;
    const int i = blockIdx.x * TPB + threadIdx.x;
    const int l = blockIdx.y, c = blockIdx.z;
    a += c * a_cs;
    b += c * b_cs;
    d += c * d_cs;
    const ModP m = T.mods[l];
    const int64_t o = (int64_t)l * N + i;
    const u64 a0 = a[o], a1 = a[a_ps + o];
    const u64 b0 = to_mont(b[o], m), b1 = to_mont(b[b_ps + o], m);
    const u64 d0 = mul_mont(a0, b0, m.q, m.qninv);
    Acc128 t = {0, 0};
    mac128(t, a0, b1);
    mac128(t, a1, b0);
    const u64 d1 = redc(t.lo, t.hi, m.q, m.qninv);
    const u64 d2 = mul_mont(a1, b1, m.q, m.qninv);
    if (acc) {
        d[o] = add_mod(d[o], d0, m.q);
        d[d_ps + o] = add_mod(d[d_ps + o], d1, m.q);
        d[2 * d_ps + o] = add_mod(d[2 * d_ps + o], d2, m.q);
    } else {
        d[o] = d0;
        d[d_ps + o] = d1;
        d[2 * d_ps + o] = d2;
    }
}

void launch_tensor(const DevTables& T, int nl, const u64* a, int64_t a_ps, const u64* b, int64_t b_ps, u64* d,
                   int64_t d_ps, int acc, hipStream_t st, int nct, int64_t a_cs, int64_t b_cs, int64_t d_cs) {
    ProfScope prof_(PK_TENSOR, (acc ? 10.0 : 7.0) * nl * nct * 8.0 * (1 << T.log_n), st);
    const int N = 1 << T.log_n;
    dim3 grid(ceil_div(N, TPB), nl, nct);
    HE_LAUNCH(k_tensor, grid, dim3(TPB), 0, st, T, a, a_ps, b, b_ps, d, d_ps, acc, a_cs, b_cs, d_cs);
}

// Step-3 block: d = sum_j a_j (x) b_j (d0 = sum a0 b0, d1 = sum a0 b1 + a1 b0, d2 = sum a1 b1),
// one pass over the inputs and one write of d.  Plain products are accumulated in 128 bits
// (n q^2 < q 2^64 for n <= 16, q < 2^60; d1 keeps its two halves apart) and reduced once per
// output: REDC gives the sum times R^-1, a Montgomery product with R^2 removes it.
__global__ __launch_bounds__(TPB) void k_tensor_sum(DevTables T, TensorSumDesc D) {
    const int N = 1 << T.log_n;
    const int i = blockIdx.x * TPB + threadIdx.x;
    const int l = blockIdx.y, c = blockIdx.z;
    const ModP m = T.mods[l];
    const int64_t o = (int64_t)l * N + i;
    Acc128 s0 = {0, 0}, s1a = {0, 0}, s1b = {0, 0}, s2 = {0, 0};
    for (int j = 0; j < D.n; j++) {
        const u64* a = D.a[j] + c * D.a_cs[j];
        const u64* b = D.b[j] + c * D.b_cs[j];
        const u64 a0 = ldnt(a + o), a1 = ldnt(a + D.a_ps[j] + o), b0 = ldnt(b + o), b1 = ldnt(b + D.b_ps[j] + o);
        mac128(s0, a0, b0);
        mac128(s1a, a0, b1);
        mac128(s1b, a1, b0);
        mac128(s2, a1, b1);
    }
    const u64 t0 = redc(s0.lo, s0.hi, m.q, m.qninv);
    const u64 t1 = add_mod(redc(s1a.lo, s1a.hi, m.q, m.qninv), redc(s1b.lo, s1b.hi, m.q, m.qninv), m.q);
    const u64 t2 = redc(s2.lo, s2.hi, m.q, m.qninv);
    u64 v0 = mul_mont(t0, m.r2, m.q, m.qninv), v1 = mul_mont(t1, m.r2, m.q, m.qninv),
        v2 = mul_mont(t2, m.r2, m.q, m.qninv);
    u64* d = D.d + c * D.d_cs;
    if (D.acc) {
        v0 = add_mod(v0, d[o], m.q);
        v1 = add_mod(v1, d[D.d_ps + o], m.q);
        v2 = add_mod(v2, d[2 * D.d_ps + o], m.q);
    }
    d[o] = v0;
    d[D.d_ps + o] = v1;
    d[2 * D.d_ps + o] = v2;
}

void launch_tensor_sum(const DevTables& T, int nl, const TensorSumDesc& D, hipStream_t st) {
    ProfScope prof_(PK_TENSOR, (4.0 * D.n + 3.0 * (1 + D.acc)) * nl * D.nct * 8.0 * (1 << T.log_n), st);
    const int N = 1 << T.log_n;
    dim3 grid(ceil_div(N, TPB), nl, D.nct);
    HE_LAUNCH(k_tensor_sum, grid, dim3(TPB), 0, st, T, D);
}

// sum of up to 16 (ciphertext limb x mask) products, one REDC per output
// masks are shared by every ciphertext of the group: loaded once, reused per member
__global__ __launch_bounds__(TPB) void k_mask_mac(DevTables T, MacDesc D, u64* out, int64_t out_ps, int acc,
                                                  int64_t out_cs) {
    const int N = 1 << T.log_n;
    const int i = blockIdx.x * TPB + threadIdx.x;
    const int l = blockIdx.y, p = blockIdx.z;
    const ModP m = T.mods[l];
    const int64_t o = (int64_t)l * N + i;
    u64 mk[16];
    for (int r = 0; r < D.nterm; r++) mk[r] = D.mask[r][o];
    for (int c = 0; c < D.nct; c++) {
        Acc128 s = {0, 0};
        for (int r = 0; r < D.nterm; r++) mac128(s, D.in[r][c * D.in_cs[r] + p * D.in_ps[r] + o], mk[r]);
        // nterm * q^2 < q 2^64 for nterm <= 16 and q < 2^60
        u64 v = redc(s.lo, s.hi, m.q, m.qninv);
        u64* dst = out + c * out_cs + p * out_ps + o;
        if (acc) v = add_mod(v, *dst, m.q);
        *dst = v;
    }
}

void launch_mask_mac(const DevTables& T, int nl, int npoly, const MacDesc& D, u64* out, int64_t out_ps, int acc,
                     hipStream_t st, int64_t out_cs) {
    ProfScope prof_(PK_MASKMAC, (D.nterm + D.nct * npoly * (D.nterm + 1.0 + acc)) * nl * 8.0 * (1 << T.log_n), st);
    const int N = 1 << T.log_n;
    dim3 grid(ceil_div(N, TPB), nl, npoly);
    HE_LAUNCH(k_mask_mac, grid, dim3(TPB), 0, st, T, D, out, out_ps, acc, out_cs);
}

// Up to MM_OUT diagonal sums of one BSGS linear transform at once: each thread keeps the masks
// of every output in registers and reads each input word once per member, so the baby-step
// rotations cross HBM once per MM_OUT giant steps instead of once per giant step.
template <int NI>
__global__ __launch_bounds__(TPB) void k_mask_mac_multi(DevTables T, MultiMacDesc D) {
    constexpr int G = NI > 8 ? 2 : MM_OUT;
    const int N = 1 << T.log_n;
    const int i = blockIdx.x * TPB + threadIdx.x;
    const int l = blockIdx.y, p = blockIdx.z;
    const ModP m = T.mods[l];
    const int64_t o = (int64_t)l * N + i;
    // up to eight terms: carry-free column sums (the inputs split once for all outputs);
    // sixteen: 128-bit accumulation.  NI q^2 < q 2^64 for NI <= 16 and q < 2^60.
    constexpr bool COLS = NI <= 8;
    using MK = typename std::conditional<COLS, Split30, u64>::type;
    MK mk[G][NI];
#pragma unroll
    for (int g = 0; g < G; g++)
#pragma unroll
        for (int j = 0; j < NI; j++) {
            const u64 v = (g < D.nout && D.mask[g][j]) ? ldnt(D.mask[g][j] + o) : 0;
            if constexpr (COLS) mk[g][j] = split30(v);
            else mk[g][j] = v;
        }
    for (int c = 0; c < D.nct; c++) {
        u64 x[NI];
#pragma unroll
        for (int j = 0; j < NI; j++) x[j] = ldnt(D.in[j] + (c * D.in_cs[j] + p * D.in_ps[j] + o));
        if constexpr (COLS) {
            Split30 xs[NI];
#pragma unroll
            for (int j = 0; j < NI; j++) xs[j] = split30(x[j]);
#pragma unroll
            for (int g = 0; g < G; g++) {
                if (g >= D.nout) break;
                Acc3 s = {0, 0, 0};
#pragma unroll
                for (int j = 0; j < NI; j++) mac3(s, xs[j], mk[g][j]);
                D.out[g][c * D.out_cs + p * D.out_ps + o] = redc3(s, m.q, m.qninv);
            }
        } else {
#pragma unroll
            for (int g = 0; g < G; g++) {
                if (g >= D.nout) break;
                Acc128 s = {0, 0};
#pragma unroll
                for (int j = 0; j < NI; j++) mac128(s, x[j], mk[g][j]);
                D.out[g][c * D.out_cs + p * D.out_ps + o] = redc(s.lo, s.hi, m.q, m.qninv);
            }
        }
    }
}

void launch_mask_mac_multi(const DevTables& T, int nl, int npoly, const MultiMacDesc& D, hipStream_t st) {
    int terms = 0;
    for (int g = 0; g < D.nout; g++)
        for (int j = 0; j < D.nin; j++) terms += D.mask[g][j] != nullptr;
    ProfScope prof_(PK_MASKMAC, (terms + D.nct * npoly * ((double)D.nin + D.nout)) * nl * 8.0 * (1 << T.log_n), st);
    const int N = 1 << T.log_n;
    dim3 grid(ceil_div(N, TPB), nl, npoly);
    switch (D.nin) {
        case 1: HE_LAUNCH(k_mask_mac_multi<1>, grid, dim3(TPB), 0, st, T, D); break;
        case 2: HE_LAUNCH(k_mask_mac_multi<2>, grid, dim3(TPB), 0, st, T, D); break;
        case 4: HE_LAUNCH(k_mask_mac_multi<4>, grid, dim3(TPB), 0, st, T, D); break;
        case 8: HE_LAUNCH(k_mask_mac_multi<8>, grid, dim3(TPB), 0, st, T, D); break;
        default: HE_LAUNCH(k_mask_mac_multi<16>, grid, dim3(TPB), 0, st, T, D); break;
    }
}

// ------------------------------------------------------------------ encrypt / decrypt
__global__ __launch_bounds__(TPB) void k_dec_dot(DevTables T, int deg, const u64* c, int64_t c_ps, const u64* s,
                                                 const u64* s2, u64* mo) {
    const int N = 1 << T.log_n;
    const int i = blockIdx.x * TPB + threadIdx.x;
    const int l = blockIdx.y;
    const ModP m = T.mods[l];
    const int64_t o = (int64_t)l * N + i;
    u64 v = add_mod(c[o], mul_plain(c[c_ps + o], s[o], m), m.q);
    if (deg == 2) v = add_mod(v, mul_plain(c[2 * c_ps + o], s2[o], m), m.q);
    mo[o] = v;
}

void launch_dec_dot(const DevTables& T, int nl, int deg, const u64* c, int64_t c_ps, const u64* s, const u64* s2,
                    u64* m, hipStream_t st) {
    ProfScope prof_(PK_EW, (2.0 + 2.0 * deg) * nl * 8.0 * (1 << T.log_n), st);
    const int N = 1 << T.log_n;
    dim3 grid(ceil_div(N, TPB), nl);
    HE_LAUNCH(k_dec_dot, grid, dim3(TPB), 0, st, T, deg, c, c_ps, s, s2, m);
}

__global__ __launch_bounds__(TPB) void k_enc_combine(DevTables T, const u64* v, const u64* pk0, const u64* pk1,
                                                     const u64* x0, const u64* x1, u64* c0, u64* c1) {
    const int N = 1 << T.log_n;
    const int i = blockIdx.x * TPB + threadIdx.x;
    const int l = blockIdx.y;
    const ModP m = T.mods[l];
    const int64_t o = (int64_t)l * N + i;
    c0[o] = add_mod(mul_mont(v[o], pk0[o], m.q, m.qninv), x0[o], m.q);
    c1[o] = add_mod(mul_mont(v[o], pk1[o], m.q, m.qninv), x1[o], m.q);
}

void launch_enc_combine(const DevTables& T, int nl, const u64* v, const u64* pk0, const u64* pk1, const u64* x0,
                        const u64* x1, u64* c0, u64* c1, hipStream_t st) {
    ProfScope prof_(PK_EW, 7.0 * nl * 8.0 * (1 << T.log_n), st);
    const int N = 1 << T.log_n;
    dim3 grid(ceil_div(N, TPB), nl);
    HE_LAUNCH(k_enc_combine, grid, dim3(TPB), 0, st, T, v, pk0, pk1, x0, x1, c0, c1);
}

__global__ __launch_bounds__(TPB) void k_add_signed(DevTables T, u64* x, const int64_t* msg) {
    const int N = 1 << T.log_n;
    const int i = blockIdx.x * TPB + threadIdx.x;
    const int l = blockIdx.y;
    const ModP m = T.mods[l];
    const int64_t v = msg[i];
    const u64 r = v >= 0 ? reduce64((u64)v, m) : neg_mod(reduce64((u64)(-v), m), m.q);
    x[(int64_t)l * N + i] = add_mod(x[(int64_t)l * N + i], r, m.q);
}

void launch_add_signed(const DevTables& T, int nl, u64* x, const int64_t* m, hipStream_t st) {
    ProfScope prof_(PK_EW, 3.0 * nl * 8.0 * (1 << T.log_n), st);
    const int N = 1 << T.log_n;
    dim3 grid(ceil_div(N, TPB), nl);
    HE_LAUNCH(k_add_signed, grid, dim3(TPB), 0, st, T, x, m);
}
