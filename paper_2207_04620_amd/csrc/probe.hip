// Streaming-bandwidth probe: what a plain streaming kernel moves through HBM per second, for
// the three access mixes the method's kernels have — read only, one read stream and one write
// stream (a copy), two read streams and one write stream (the ModDown row pass reads the
// converted limb and u and writes the result).  It is a measurement aid: the method never calls
// it.  The kernels sit here, apart from the method's kernels, so that changing one never
// touches the other.
#include <hip/hip_runtime.h>

#include <stdexcept>

#include "he_internal.hpp"
#include "kernels.hpp"

namespace {

typedef uint64_t w64;
typedef w64 w64x2 __attribute__((ext_vector_type(2)));

constexpr int PTPB = 256;  // threads per block
constexpr int RPU = 8;     // the read mix: 16-byte loads per lane (one pass, 2048 pairs per block)

// Accesses bypass the caches' normal retention (nontemporal): each word is touched once, and
// these were the fastest forms of each mix measured on the device (one pass, 16-byte accesses;
// one pair per lane for the copy and the two-read mix, eight for the read mix).

// pattern 0: a block sums its 2048 pairs (two lanes of 64-bit sums, mod 2^64) and writes one
// pair to c[block]
__global__ __launch_bounds__(PTPB) void k_stream_read(const w64x2* __restrict__ a, w64x2* __restrict__ c,
                                                      int64_t n2) {
    __shared__ w64x2 red[PTPB];
    const int64_t base = (int64_t)blockIdx.x * (PTPB * RPU) + threadIdx.x;
    w64x2 s = {0, 0};
#pragma unroll
    for (int k = 0; k < RPU; ++k) {
        const int64_t i = base + (int64_t)k * PTPB;
        if (i < n2) s += __builtin_nontemporal_load(a + i);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = PTPB / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) c[blockIdx.x] = red[0];
}

// patterns 1 and 2: one pair per lane, c = a or c = a + b (mod 2^64 per word)
template <bool ADD>
__global__ __launch_bounds__(PTPB) void k_stream_map(const w64x2* __restrict__ a, const w64x2* __restrict__ b,
                                                     w64x2* __restrict__ c, int64_t n2) {
    const int64_t i = (int64_t)blockIdx.x * PTPB + threadIdx.x;
    if (i < n2) {
        w64x2 v = __builtin_nontemporal_load(a + i);
        if constexpr (ADD) v += __builtin_nontemporal_load(b + i);
        __builtin_nontemporal_store(v, c + i);
    }
}

void launch_stream(uint32_t pattern, const w64x2* a, const w64x2* b, w64x2* c, int64_t n2, hipStream_t st) {
    if (pattern == 0) {
        const int64_t blocks = (n2 + PTPB * RPU - 1) / (PTPB * RPU);
        HE_LAUNCH(k_stream_read, dim3((unsigned)blocks), dim3(PTPB), 0, st, a, c, n2);
    } else {
        const int64_t blocks = (n2 + PTPB - 1) / PTPB;
        if (pattern == 1)
            HE_LAUNCH(k_stream_map<false>, dim3((unsigned)blocks), dim3(PTPB), 0, st, a, b, c, n2);
        else
            HE_LAUNCH(k_stream_map<true>, dim3((unsigned)blocks), dim3(PTPB), 0, st, a, b, c, n2);
    }
}

bool misaligned(const void* p) { return ((uintptr_t)p & 15) != 0; }

}  // namespace

extern "C" {

he_status he_stream_probe(he_ctx* ctx, uint32_t pattern, const uint64_t* a, const uint64_t* b, uint64_t* c,
                          uint64_t n_words, uint32_t reps, double* ms_per_rep) {
    if (!ctx || !a || !c || !ms_per_rep || pattern > 2 || reps == 0 || n_words == 0 || (n_words & 1)) return HE_EINVAL;
    if (pattern == 2 && !b) return HE_EINVAL;
    if (misaligned(a) || misaligned(c) || (b && misaligned(b))) return HE_EINVAL;
    // one grid dimension of blocks for the one-pass mixes
    if (n_words / 2 > (uint64_t)0x7fffffff * PTPB) return HE_EINVAL;
    const int64_t n2 = (int64_t)(n_words / 2);
    return run_guarded(ctx, [&]() {
        hipStream_t st = ctx->c->stream;
        const w64x2* pa = reinterpret_cast<const w64x2*>(a);
        const w64x2* pb = reinterpret_cast<const w64x2*>(b);
        w64x2* pc = reinterpret_cast<w64x2*>(c);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        hip_check(hipEventCreate(&e0), "probe event");
        try {
            hip_check(hipEventCreate(&e1), "probe event");
            launch_stream(pattern, pa, pb, pc, n2, st);  // untimed first pass
            hip_check(hipEventRecord(e0, st), "probe event");
            for (uint32_t r = 0; r < reps; ++r) launch_stream(pattern, pa, pb, pc, n2, st);
            hip_check(hipEventRecord(e1, st), "probe event");
            hip_check(hipEventSynchronize(e1), "probe sync");
            float ms = 0.f;
            hip_check(hipEventElapsedTime(&ms, e0, e1), "probe timing");
            *ms_per_rep = (double)ms / reps;
        } catch (...) {
            (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            throw;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    });
}

}  // extern "C"
