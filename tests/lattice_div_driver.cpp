// Checks the lattice-index division used by the integration kernels: for
// every divisor d in [1, 70000] and a set of large ones, and indices n < 2^31
// (edges around multiples of d, the largest index, pseudo-random ones),
// (n * m) >> s with the divisors set_lattice_divisors computes equals n / d.
// Prints the number of checks and exits 0 when all agree.
#include "tsdf_internal.hpp"

#include <cstdio>

static unsigned long long state = 0x9E3779B97F4A7C15ull;
static uint32_t next_index()
{
    state = state * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)(state >> 33);   // 31 bits
}

static bool check(uint32_t d, uint32_t n, uint32_t m, int s)
{
    const uint32_t q = (uint32_t)(((unsigned long long)n * (unsigned long long)m) >> s);
    if (q != n / d) {
        std::fprintf(stderr, "d=%u n=%u: got %u, expected %u (m=%u s=%d)\n", d, n, q, n / d, m, s);
        return false;
    }
    return true;
}

int main()
{
    const uint32_t n_max = 0x7FFFFFFFu;   // indices are below 2^31
    long long checks = 0;
    int bad = 0;
    auto test = [&](uint32_t d) {
        tsdf::Lattice l{};
        l.lat_dim[0] = (int)d;
        l.lat_dim[1] = 1;
        tsdf::set_lattice_divisors(l);
        const uint32_t m = l.div_m[0];
        const int s = l.div_s[0];
        const uint32_t fixed[] = {0u, 1u, d - 1u, d, d + 1u, n_max, n_max - 1u, n_max - d, n_max / d * d,
                                  n_max / d * d - 1u};
        for (uint32_t n : fixed)
            if (n <= n_max) {
                bad += !check(d, n, m, s);
                ++checks;
            }
        for (uint32_t k = 1; k < 40; ++k) {
            const unsigned long long base = (unsigned long long)(next_index() / d) * d;
            for (int off = -1; off <= 1; ++off) {
                const long long n = (long long)base + off;
                if (n >= 0 && n <= (long long)n_max) {
                    bad += !check(d, (uint32_t)n, m, s);
                    ++checks;
                }
            }
            bad += !check(d, next_index(), m, s);
            ++checks;
        }
    };
    for (uint32_t d = 1; d <= 70000u; ++d)
        test(d);
    const uint32_t large[] = {1u << 16, (1u << 16) + 1u, 1u << 20, (1u << 24) + 1u, 1u << 30, (1u << 30) + 7u,
                              n_max - 1u, n_max};
    for (uint32_t d : large)
        test(d);
    std::printf("%lld checks, %d wrong\n", checks, bad);
    return bad == 0 ? 0 : 1;
}
