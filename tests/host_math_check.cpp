// Host-only driver of the library's host number theory and encoder (csrc/host_math.hpp),
// built by tests/test_sanitizers.py with g++ and AddressSanitizer / UndefinedBehaviorSanitizer.
//
//   host_math_check primes <log_n> <bits...>    the largest primes p < 2^bits, p = 1 mod 2N
//   host_math_check encode <log_n> <log_scale>  values on stdin (one per line) -> Ecd
//                                                coefficients, then the decoded slots
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../paper_2207_04620_amd/csrc/host_math.hpp"

static int primes(int log_n, int argc, char** argv) {
    const uint64_t m2n = 2ull << log_n;
    std::vector<uint64_t> got;
    for (int a = 0; a < argc; ++a) {
        const int b = atoi(argv[a]);
        uint64_t cand = ((1ull << b) - 1) / m2n * m2n + 1;
        for (;; cand -= m2n) {
            bool dup = false;
            for (uint64_t g : got) dup |= g == cand;
            if (!dup && hm::is_prime(cand)) break;
        }
        got.push_back(cand);
        // Montgomery and Shoup constants of the prime, checked against their definitions
        const uint64_t ninv = hm::mont_neg_inv(cand);
        if ((uint64_t)(cand * ninv) != ~0ull) return 2;  // q * (-q^-1) = -1 mod 2^64
        const uint64_t w = cand / 3, ws = hm::shoup(w, cand);
        const unsigned __int128 lhs = (unsigned __int128)ws * cand, rhs = (unsigned __int128)w << 64;
        if (lhs > rhs || rhs - lhs >= cand) return 3;  // ws = floor(w 2^64 / q)
        printf("%llu\n", (unsigned long long)cand);
    }
    return 0;
}

static int encode(int log_n, double log_scale) {
    std::vector<double> vals;
    double v;
    while (scanf("%lf", &v) == 1) vals.push_back(v);
    hm::Encoder E;
    E.init(log_n);
    const int64_t n = (int64_t)1 << log_n;
    if (vals.empty() || (n / 2) % (int64_t)vals.size()) return 4;
    std::vector<int64_t> m(n);
    const double scale = ldexp(1.0, (int)log_scale);
    const double tie = E.encode(vals.data(), (int64_t)vals.size(), scale, m.data());
    printf("%.17g\n", tie);
    for (int64_t i = 0; i < n; ++i) printf("%lld\n", (long long)m[i]);
    std::vector<double> c(m.begin(), m.end()), out(n / 2);
    E.decode(c.data(), scale, out.data(), n / 2);
    for (int64_t j = 0; j < n / 2; ++j) printf("%.17g\n", out[j]);
    return 0;
}

int main(int argc, char** argv) {
    if (argc >= 4 && !strcmp(argv[1], "primes")) return primes(atoi(argv[2]), argc - 3, argv + 3);
    if (argc == 4 && !strcmp(argv[1], "encode")) return encode(atoi(argv[2]), atof(argv[3]));
    fprintf(stderr, "usage: host_math_check primes <log_n> <bits...> | encode <log_n> <log_scale>\n");
    return 1;
}
