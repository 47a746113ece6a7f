// Host check (built by tests/test_host_checks_cpu.py): the compact ghost-image
// writer stores exactly what the general one does, for every lattice,
// role, boundary kind and position on lattices of one to five points a side.
#include "common.h"
#include <cstdio>
#include <vector>
using namespace ibmg;

static Grid mk(int D, int n0, int n1, int n2, int b0, int b1, int b2)
{
    Grid g{};
    g.D = D; g.n[0] = n0; g.n[1] = n1; g.n[2] = D == 3 ? n2 : 1;
    g.bc[0] = b0; g.bc[1] = b1; g.bc[2] = b2;
    g.NX = n0 + 3; g.NY = n1 + 3; g.NXY = (long long)g.NX * g.NY;
    g.nel = g.NXY * (D == 3 ? n2 + 3 : 1);
    g.h = 1.0;
    return g;
}

int main()
{
    long long checks = 0, bad = 0;
    const int sizes[] = {1, 2, 3, 4, 5};
    for (int D = 2; D <= 3; ++D)
        for (int n0 : sizes) for (int n1 : sizes) for (int n2 : sizes)
            for (int b0 = 0; b0 < 3; ++b0) for (int b1 = 0; b1 < 3; ++b1) for (int b2 = 0; b2 < 3; ++b2) {
                if (D == 2 && (n2 != 1 || b2 != 0)) continue;
                const Grid g = mk(D, n0, n1, n2, b0, b1, b2);
                for (int role : {ROLE_P, ROLE_V, ROLE_C})
                    for (int vmask = 0; vmask < (1 << D); ++vmask)
                        for (int k = (D == 3 ? -1 : 0); k <= (D == 3 ? n2 + 1 : 0); ++k)
                            for (int j = -1; j <= n1 + 1; ++j)
                                for (int i = -1; i <= n0 + 1; ++i) {
                                    std::vector<double> a(g.nel, 0.0), b(g.nel, 0.0);
                                    write_images(g, vmask, role, a.data(), i, j, k, 1.5);
                                    const int q[3] = {i, j, k};
                                    AxisImages im[3];
                                    for (int d = 0; d < 3; ++d)
                                        im[d] = d < g.D ? images_of(g, d, (vmask >> d) & 1, role, q[d]) : AxisImages{{0, 0}, {0, 0}};
                                    if (im[0].s[0] | im[0].s[1] | im[1].s[0] | im[1].s[1] | im[2].s[0] | im[2].s[1])
                                        write_images_any(g, im, b.data(), i, j, k, 1.5);
                                    ++checks;
                                    if (a != b) {
                                        if (bad < 5) printf("mismatch D%d n %d %d %d bc %d %d %d role %d vmask %d at %d %d %d\n", D, n0, n1, n2, b0, b1, b2, role, vmask, i, j, k);
                                        ++bad;
                                    }
                                }
            }
    printf("%lld positions checked, %lld mismatches\n", checks, bad);
    return bad != 0;
}
