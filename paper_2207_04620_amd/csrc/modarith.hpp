// Device modular arithmetic over word-size primes q < 2^61 (gfx950, 64-wide waves).
//
// Two reductions are used, both exact:
//  - Shoup/Harvey products a*w mod q with a precomputed companion
//    w' = floor(w 2^64 / q) for fixed operands (twiddles, per-limb constants);
//  - Montgomery REDC with R = 2^64 for products with keys and masks stored as
//    x R mod q, and for 128-bit multiply-accumulate chains (sum < q 2^64).
// gfx950 has no 64-bit multiplier: the compiler lowers the 64x64 products to
// v_mad_u64_u32 / v_mul_hi_u32 chains.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef uint64_t u64;
typedef uint32_t u32;

struct ModP {
    u64 q;      // the prime
    u64 qninv;  // -q^-1 mod 2^64
    u64 r2;     // 2^128 mod q  (to enter Montgomery form)
    u64 bar;    // floor((2^64 - 1) / q)
    u64 ninv;   // N^-1 mod q
    u64 ninv_sh;
    u64 half;   // (q - 1) / 2
    u64 pad;
};

__device__ __forceinline__ u64 add_mod(u64 a, u64 b, u64 q) {
    u64 s = a + b;
    return s >= q ? s - q : s;
}
__device__ __forceinline__ u64 sub_mod(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + q - b; }
__device__ __forceinline__ u64 neg_mod(u64 a, u64 q) { return a ? q - a : 0; }

// a * w mod q, w < q, w_sh = floor(w 2^64 / q); any a < 2^64
__device__ __forceinline__ u64 mul_shoup(u64 a, u64 w, u64 w_sh, u64 q) {
    u64 qh = __umul64hi(a, w_sh);
    u64 r = a * w - qh * q;
    return r >= q ? r - q : r;
}
// lazy form: result in [0, 2q)
__device__ __forceinline__ u64 mul_shoup_lazy(u64 a, u64 w, u64 w_sh, u64 q) {
    u64 qh = __umul64hi(a, w_sh);
    return a * w - qh * q;
}

// (hi 2^64 + lo) R^-1 mod q for hi 2^64 + lo < q 2^64
__device__ __forceinline__ u64 redc(u64 lo, u64 hi, u64 q, u64 qninv) {
    u64 m = lo * qninv;
    u64 mh = __umul64hi(m, q);
    u64 r = hi + mh + (lo != 0 ? 1 : 0);
    return r >= q ? r - q : r;
}
// a * (b R) R^-1 = a b mod q
__device__ __forceinline__ u64 mul_mont(u64 a, u64 bR, u64 q, u64 qninv) {
    return redc(a * bR, __umul64hi(a, bR), q, qninv);
}
// a b mod q for two plain residues: a b R^-1, then times R^2 R^-1
__device__ __forceinline__ u64 mul_plain(u64 a, u64 b, const ModP& m) {
    u64 t = redc(a * b, __umul64hi(a, b), m.q, m.qninv);
    return redc(t * m.r2, __umul64hi(t, m.r2), m.q, m.qninv);
}
// to Montgomery form
__device__ __forceinline__ u64 to_mont(u64 a, const ModP& m) { return redc(a * m.r2, __umul64hi(a, m.r2), m.q, m.qninv); }

struct Acc128 {
    u64 lo, hi;
};
// full 64x64 -> 128 product from four 32x32 -> 64 partial products (v_mad_u64_u32),
// the carries folded into the multiply-adds
__device__ __forceinline__ void mul_wide(u64 a, u64 b, u64& lo, u64& hi) {
    const u32 a0 = (u32)a, a1 = (u32)(a >> 32), b0 = (u32)b, b1 = (u32)(b >> 32);
    const u64 p00 = (u64)a0 * b0;
    const u64 t = (u64)a0 * b1 + (p00 >> 32);          // < 2^64
    const u64 u = (u64)a1 * b0 + (u32)t;               // < 2^64
    lo = (u << 32) | (u32)p00;
    hi = (u64)a1 * b1 + (t >> 32) + (u >> 32);
}
__device__ __forceinline__ void mac128(Acc128& acc, u64 a, u64 b) {
    u64 lo, hi;
    mul_wide(a, b, lo, hi);
    acc.lo += lo;
    acc.hi += hi + (acc.lo < lo ? 1 : 0);
}
__device__ __forceinline__ void add128(Acc128& acc, u64 a) {
    acc.lo += a;
    acc.hi += (acc.lo < a ? 1 : 0);
}

// Sums of up to eight products of residues below 2^60 with no carry handling: each operand
// is split at bit 30 (x = x.hi 2^30 + x.lo), and the four 30 x 30-bit partial products go
// into three 64-bit column sums, value = c0 + c1 2^30 + c2 2^60.  A product adds < 2^60 to
// c0 and c2 and < 2^61 to c1, so eight of them (plus one residue per product added to c0)
// stay below 2^64.  Each partial product is one v_mad_u64_u32.
struct Split30 {
    u32 lo, hi;
};
struct Acc3 {
    u64 c0, c1, c2;
};
__device__ __forceinline__ Split30 split30(u64 v) { return {(u32)v & 0x3fffffffu, (u32)(v >> 30)}; }
__device__ __forceinline__ void mac3(Acc3& a, Split30 x, Split30 y) {
    a.c0 += (u64)x.lo * y.lo;
    a.c1 += (u64)x.lo * y.hi;
    a.c1 += (u64)x.hi * y.lo;
    a.c2 += (u64)x.hi * y.hi;
}
// the 128-bit value of the column sums, without carry detection: with t = c1 + (c0 >> 30) and
// t2 = c2 + (t >> 30) the value is (c0 mod 2^30) + (t mod 2^30) 2^30 + t2 2^60, whose part
// below t2's top bits, (t2 mod 16) 2^60 + ..., is below 2^64; so hi = t2 >> 4 and lo is the
// value mod 2^64.  Bounds: c0, c2 < 2^63 and c1 < 2^64 - 2^35 (eight products), so t and t2
// do not wrap.
__device__ __forceinline__ void acc3_wide(const Acc3& a, u64& lo, u64& hi) {
    const u64 t = a.c1 + (a.c0 >> 30);
    const u64 t2 = a.c2 + (t >> 30);
    hi = t2 >> 4;
    lo = a.c0 + (a.c1 << 30) + (a.c2 << 60);
}
__device__ __forceinline__ u64 redc3(const Acc3& a, u64 q, u64 qninv) {
    u64 lo, hi;
    acc3_wide(a, lo, hi);
    return redc(lo, hi, q, qninv);
}

// Signed form for centred inputs |y| < 2^59 (y = y_c, the centred representative of a residue
// of a prime below 2^60): y = hi 2^30 + lo, the four partial products with the (unsigned) 30-bit
// halves of t are signed v_mad_i64_i32 into three int64 column sums.  With lo in [0, 2^30) a
// product adds |.| < 1.5 2^60 to c1, so up to five products fit; the balanced split
// (lo in [-2^29, 2^29)) keeps every term below 2^60 in magnitude, for up to eight.
struct AccS {
    int64_t c0, c1, c2;
};
template <bool BAL>
__device__ __forceinline__ void split30s(int64_t y, int32_t& lo, int32_t& hi) {
    if constexpr (BAL) {
        const int64_t z = y + (1ll << 29);
        hi = (int32_t)(z >> 30);
        lo = (int32_t)(z & 0x3fffffff) - (1 << 29);
    } else {
        hi = (int32_t)(y >> 30);
        lo = (int32_t)(y & 0x3fffffff);
    }
}
__device__ __forceinline__ void macs(AccS& a, int32_t lo, int32_t hi, Split30 t) {
    a.c0 += (int64_t)lo * (int64_t)(int32_t)t.lo;
    a.c1 += (int64_t)lo * (int64_t)(int32_t)t.hi;
    a.c1 += (int64_t)hi * (int64_t)(int32_t)t.lo;
    a.c2 += (int64_t)hi * (int64_t)(int32_t)t.hi;
}
// V R^-1 mod q for the signed V = c0 + c1 2^30 + c2 2^60 with |V| < q 2^64, lazy in [0, 3q):
// REDC of V + q 2^64, which lies in (0, 2q 2^64).  floor(V / 2^64) is t2 >> 4 (arithmetic
// shifts, as in acc3_wide; |c1| < 7.5 2^60 keeps t in range), the low word V mod 2^64.
__device__ __forceinline__ u64 redcs_lazy(const AccS& a, u64 q, u64 qninv) {
    const int64_t t = a.c1 + (a.c0 >> 30);
    const int64_t t2 = a.c2 + (t >> 30);
    const u64 lo = (u64)a.c0 + ((u64)a.c1 << 30) + ((u64)a.c2 << 60);
    const u64 hi = (u64)(t2 >> 4) + q;
    const u64 m = lo * qninv;
    return hi + __umul64hi(m, q) + (lo != 0 ? 1 : 0);
}

// x mod q for any 64-bit x
__device__ __forceinline__ u64 reduce64(u64 x, const ModP& m) {
    u64 qh = __umul64hi(x, m.bar);
    u64 r = x - qh * m.q;
    return r >= m.q ? r - m.q : r;
}

__device__ __forceinline__ u32 brev_bits(u32 x, int bits) { return __builtin_bitreverse32(x) >> (32 - bits); }
