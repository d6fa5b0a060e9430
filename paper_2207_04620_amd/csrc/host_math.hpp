// Host-side number theory and the canonical-embedding encoder of libhe.
//
// Primes, roots of unity and Montgomery/Shoup constants are exact integer
// computations.  Ecd (Fig. 1 item 3) is computed in __float128 so that the rounded
// coefficients are the exact rounding of Delta * sigma^-1(z): the 113-bit result is
// ~2^-50 from the true value at N = 2^16, far inside the distance to a rounding tie.
#pragma once
#include <stdint.h>

#include <complex>
#include <vector>

typedef unsigned __int128 u128h;
typedef __float128 f128;

namespace hm {

inline uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128h)a * b % q); }
inline uint64_t powmod(uint64_t a, uint64_t e, uint64_t q) {
    uint64_t r = 1 % q;
    a %= q;
    for (; e; e >>= 1) {
        if (e & 1) r = mulmod(r, a, q);
        a = mulmod(a, a, q);
    }
    return r;
}
inline uint64_t invmod(uint64_t a, uint64_t q) { return powmod(a, q - 2, q); }

// Miller-Rabin with the first twelve prime bases: deterministic below 3.3e24
inline bool is_prime(uint64_t n) {
    const uint64_t B[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return false;
    for (uint64_t b : B) {
        if (n % b == 0) return n == b;
    }
    uint64_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) {
        d >>= 1;
        ++s;
    }
    for (uint64_t b : B) {
        uint64_t x = powmod(b, d, n);
        if (x == 1 || x == n - 1) continue;
        bool witness = true;
        for (int r = 1; r < s && witness; ++r) {
            x = mulmod(x, x, n);
            if (x == n - 1) witness = false;
        }
        if (witness) return false;
    }
    return true;
}

inline uint64_t shoup(uint64_t w, uint64_t q) { return (uint64_t)(((u128h)w << 64) / q); }
// -q^-1 mod 2^64 by Newton iteration (q odd)
inline uint64_t mont_neg_inv(uint64_t q) {
    uint64_t x = q;  // q * q = 1 mod 8
    for (int i = 0; i < 6; ++i) x *= 2 - q * x;
    return (uint64_t)0 - x;
}
inline uint64_t r_mod(uint64_t q) { return (uint64_t)(((u128h)1 << 64) % q); }
inline uint64_t to_mont(uint64_t a, uint64_t q) { return (uint64_t)(((u128h)a << 64) % q); }

inline uint32_t bitrev(uint32_t x, int bits) {
    uint32_t r = 0;
    for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
    return r;
}

// ------------------------------------------------------------------ 113-bit trigonometry
inline f128 pi128() {
    // pi = 16 atan(1/5) - 4 atan(1/239) (Machin)
    auto atan_inv = [](int x) {
        f128 t = (f128)1 / (f128)x, x2 = t * t, s = 0;
        for (int k = 0; k < 80; ++k) {
            f128 term = t / (f128)(2 * k + 1);
            s += (k & 1) ? -term : term;
            t *= x2;
        }
        return s;
    };
    return 16 * atan_inv(5) - 4 * atan_inv(239);
}

// cos, sin of x in [0, pi/4] by Taylor series
inline void sincos_small(f128 x, f128& c, f128& s) {
    f128 x2 = x * x, tc = 1, ts = x, sc = 1, ss = x;
    for (int k = 1; k < 40; ++k) {
        tc *= -x2 / (f128)((2 * k - 1) * (2 * k));
        ts *= -x2 / (f128)((2 * k) * (2 * k + 1));
        sc += tc;
        ss += ts;
    }
    c = sc;
    s = ss;
}

// (cos, sin)(2 pi k / K) for K divisible by 8, reduced exactly by quadrant and co-function
inline void cis(int64_t k, int64_t K, const f128& pi, f128& c, f128& s) {
    k %= K;
    if (k < 0) k += K;
    const int64_t K4 = K / 4;
    const int64_t qd = k / K4, rem = k % K4;
    f128 cc, ss;
    if (2 * rem <= K4) {
        sincos_small(2 * pi * (f128)rem / (f128)K, cc, ss);
    } else {
        f128 a, b;
        sincos_small(2 * pi * (f128)(K4 - rem) / (f128)K, a, b);
        cc = b;
        ss = a;
    }
    switch (qd) {
        case 0: c = cc; s = ss; break;
        case 1: c = -ss; s = cc; break;
        case 2: c = -cc; s = -ss; break;
        default: c = ss; s = -cc; break;
    }
}

// ------------------------------------------------------------------ encoder
struct Encoder {
    int log_n = 0;
    int64_t n = 0;
    std::vector<f128> wr, wi;    // exp(-2 pi i k / N), k < N/2
    std::vector<f128> zr, zi;    // zeta^-i = exp(-pi i i / N), i < N
    std::vector<int64_t> slot_pos;   // position of w_{5^j} in the length-N array
    std::vector<int64_t> slot_neg;   // position of w_{-5^j}
    std::vector<std::complex<double>> dw, dz;  // double tables for decoding

    void init(int lg) {
        log_n = lg;
        n = (int64_t)1 << lg;
        const f128 pi = pi128();
        wr.resize(n / 2); wi.resize(n / 2);
        for (int64_t k = 0; k < n / 2; ++k) {
            f128 c, s;
            cis(-k, n, pi, c, s);
            wr[k] = c; wi[k] = s;
        }
        zr.resize(n); zi.resize(n);
        for (int64_t i = 0; i < n; ++i) {
            f128 c, s;
            cis(-i, 2 * n, pi, c, s);
            zr[i] = c; zi[i] = s;
        }
        slot_pos.resize(n / 2); slot_neg.resize(n / 2);
        uint64_t r = 1, two_n = 2 * (uint64_t)n;
        for (int64_t j = 0; j < n / 2; ++j) {
            slot_pos[j] = (int64_t)((r - 1) / 2);
            slot_neg[j] = (int64_t)((two_n - r - 1) / 2);
            r = r * 5 % two_n;
        }
        dw.resize(n / 2); dz.resize(n);
        for (int64_t k = 0; k < n / 2; ++k) dw[k] = std::complex<double>((double)wr[k], -(double)wi[k]);
        for (int64_t i = 0; i < n; ++i) dz[i] = std::complex<double>((double)zr[i], -(double)zi[i]);
    }

    // Gentleman-Sande DIF transform X_k = sum_j x_j exp(-2 pi i j k / N): natural in,
    // bit-reversed out
    void dif(std::vector<f128>& re, std::vector<f128>& im) const {
        for (int64_t half = n / 2, stride = 1; half >= 1; half >>= 1, stride <<= 1) {
            for (int64_t b = 0; b < n; b += 2 * half) {
                for (int64_t j = 0; j < half; ++j) {
                    const int64_t p = b + j, q = p + half;
                    const f128 ur = re[p] - re[q], ui = im[p] - im[q];
                    re[p] += re[q];
                    im[p] += im[q];
                    const f128 c = wr[j * stride], s = wi[j * stride];
                    re[q] = ur * c - ui * s;
                    im[q] = ur * s + ui * c;
                }
            }
        }
    }

    // m_i = round(scale * (1/N) Re(zeta^-i sum_u W_u omega^-(u i))), W at odd exponents
    // 2u+1 = +-5^j holds z_j (real slots).  Returns min distance to a rounding tie.
    double encode(const double* vals, int64_t n_vals, double scale, int64_t* out) const {
        std::vector<f128> re(n, 0), im(n, 0);
        for (int64_t j = 0; j < n / 2; ++j) {
            const f128 z = (f128)vals[j % n_vals];
            re[slot_pos[j]] = z;
            re[slot_neg[j]] = z;
        }
        // sum_u W_u omega^(-u i) is a forward DFT in the sign convention of dif()
        dif(re, im);
        double tie = 1.0;
        const f128 sc = (f128)scale / (f128)n;
        for (int64_t i = 0; i < n; ++i) {
            const int64_t u = bitrev((uint32_t)i, log_n);  // X_i sits at bitrev(i)
            const f128 v = (re[u] * zr[i] - im[u] * zi[i]) * sc;
            const f128 a = v < 0 ? -v : v;
            const int64_t fl = (int64_t)a;
            const double d = (double)(a - (f128)fl) - 0.5;
            const double dd = d < 0 ? -d : d;
            if (dd < tie) tie = dd;
            const int64_t r = (int64_t)(a + (f128)0.5);
            out[i] = v < 0 ? -r : r;
        }
        return tie;
    }

    // z_j = sum_i m_i zeta^(i 5^j) / scale, in double precision
    void decode(const double* coeffs, double scale, double* out_re, int64_t n_out) const {
        std::vector<std::complex<double>> x(n);
        for (int64_t i = 0; i < n; ++i) x[i] = coeffs[i] * dz[i];
        // DIF with exp(+2 pi i j k / N)
        for (int64_t half = n / 2, stride = 1; half >= 1; half >>= 1, stride <<= 1)
            for (int64_t b = 0; b < n; b += 2 * half)
                for (int64_t j = 0; j < half; ++j) {
                    const int64_t p = b + j, q = p + half;
                    const std::complex<double> u = x[p] - x[q];
                    x[p] += x[q];
                    x[q] = u * dw[j * stride];
                }
        for (int64_t j = 0; j < n_out && j < n / 2; ++j)
            out_re[j] = x[bitrev((uint32_t)slot_pos[j], log_n)].real() / scale;
    }
};

}  // namespace hm
