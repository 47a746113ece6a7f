// Host check (built by tests/test_host_checks_cpu.py): division through one
// multiply equals integer division, and the decodes that use it give the
// points of the plain decodes, for every box shape up to a size and every t.
#include "kernels.h"
#include <cstdio>
#include <random>
using namespace ibmg;

int main()
{
    long long checks = 0, bad = 0;
    // every divisor up to 5000 against every t up to 20000, then random
    // divisors and dividends across the whole range
    for (int d = 1; d <= 5000; ++d) {
        const Div v = make_div(d);
        for (int t = 0; t < 20000; ++t, ++checks)
            if (div_by(v, t) != t / d) ++bad;
        for (int t : {0x7fffffff, 0x7ffffffe, 0x40000000, 0x3fffffff})
            if (div_by(v, t) != t / d) ++bad;
    }
    std::mt19937_64 rng(7);
    for (int it = 0; it < 2000000; ++it, ++checks) {
        const int d = 1 + (int)(rng() % 0x7fffffff);
        const int t = (int)(rng() % 0x80000000ull);
        if (div_by(make_div(d), t) != t / d) ++bad;
    }
    // the decodes over whole boxes
    for (int e0 = 1; e0 <= 40; ++e0)
        for (int e1 = 1; e1 <= 12; ++e1)
            for (int e2 = 1; e2 <= 6; ++e2) {
                const Box b{{e0 % 3 - 1, e1 % 2, 1 - e2 % 2}, {e0, e1, e2}};
                const BoxDiv bd = box_div(b);
                const int n = e0 * e1 * e2;
                for (int t = 0; t < n + 70; ++t) {
                    int i0, j0, k0, i1, j1, k1;
                    const bool a = box_pos(b, t, i0, j0, k0), c = box_pos(b, bd, t, i1, j1, k1);
                    ++checks;
                    if (a != c || (a && (i0 != i1 || j0 != j1 || k0 != k1))) ++bad;
                    for (int colour = 0; colour < 2; ++colour) {
                        const bool p = box_colour_pos(b, colour, t, i0, j0, k0);
                        const bool q = box_colour_pos(b, bd, colour, t, i1, j1, k1);
                        ++checks;
                        if (p != q || (p && (i0 != i1 || j0 != j1 || k0 != k1))) ++bad;
                    }
                }
            }
    printf("%lld checks, %lld mismatches\n", checks, bad);
    return bad != 0;
}
