// Sanitizer driver of the library's host-side code: built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitizers.py
// together with csrc/quadrature.cpp (collocation rules, gPC basis) and
// csrc/hostcheck.hip compiled as plain C++ (the kernels' link rules, flags,
// solid-link masks, the in-place slot maps and their adjoint, evaluated on
// the host).  Fails on any memory or undefined-behaviour error, or a check
// that does not hold.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "quadrature.h"

extern "C" {
void lbmhc_rules(int nx, int ny, int nz, const int *face, const uint8_t *solid, int *rules);
int lbmhc_check(int nx, int ny, int nz, const int *face, const uint8_t *solid, int block, int64_t *stats);
void lbmhc_flags(int nx, int ny, int nz, const int *face, const uint8_t *solid, uint8_t *fl);
int64_t lbmhc_check_adjoint_inplace(int nx, int ny, int nz, const int *face, const uint8_t *solid,
                                    const double *lam_in);
int lbmhc_check_relative(int nx, int ny, int nz, const int *face, const uint8_t *solid);
}

using namespace lbmsc;

static int bad = 0;

static void expect(bool ok, const char *what)
{
    if (!ok) {
        std::fprintf(stderr, "FAIL: %s\n", what);
        bad = 1;
    }
}

static double sum(const std::vector<double> &v)
{
    double s = 0.0;
    for (double x : v) s += x;
    return s;
}

static void geometry(int nx, int ny, int nz, const int face[6], const std::vector<uint8_t> &solid)
{
    const int64_t n = (int64_t)nx * ny * nz;
    std::vector<int> rules(19 * n);
    lbmhc_rules(nx, ny, nz, face, solid.data(), rules.data());
    std::vector<uint8_t> fl(n);
    lbmhc_flags(nx, ny, nz, face, solid.data(), fl.data());
    for (int block : {64, 128, 256}) {
        int64_t stats[7];
        expect(lbmhc_check(nx, ny, nz, face, solid.data(), block, stats) == 0, "odd-step slot checks");
    }
    expect(lbmhc_check_relative(nx, ny, nz, face, solid.data()) == 0, "wavefront rule forms");
    std::vector<double> lam(19 * n);
    for (int64_t i = 0; i < 19 * n; ++i) lam[i] = 1e-3 * (double)((i * 7919) % 101) - 0.05;
    expect(lbmhc_check_adjoint_inplace(nx, ny, nz, face, solid.data(), lam.data()) == 0, "in-place adjoint map");
}

int main()
{
    // collocation rules
    for (int n = 1; n <= 24; ++n) {
        std::vector<double> x, w;
        expect(gauss_legendre(n, x, w) && std::fabs(sum(w) - 1.0) < 1e-13, "Gauss-Legendre");
        expect(gauss_hermite(n, x, w) && std::fabs(sum(w) - 1.0) < 1e-12, "Gauss-Hermite");
    }
    for (int m : {1, 3, 5, 9, 17}) {
        std::vector<double> x, w;
        expect(clenshaw_curtis(m, x, w) && std::fabs(sum(w) - 1.0) < 1e-13, "Clenshaw-Curtis");
    }
    for (int dim = 1; dim <= 3; ++dim)
        for (int level = 0; level <= 3; ++level) {
            std::vector<double> x, w;
            expect(smolyak_cc(level, dim, x, w) && std::fabs(sum(w) - 1.0) < 1e-12, "Smolyak");
        }
    {
        std::vector<double> x, w, phi;
        expect(tensor_gauss_hermite(11, 2, x, w) && w.size() == 121, "tensor Gauss-Hermite");
        std::vector<int> alpha;
        gpc_multi_indices(2, 5, alpha);
        expect(alpha.size() == 42, "gPC multi-indices");
        gpc_basis(x.data(), 121, 2, alpha, phi);
        expect(phi.size() == 121 * 21, "gPC basis");
    }
    // link rules on boxes with every face kind, buildings and a cylinder mantle
    const int nx = 16, ny = 8, nz = 8;
    std::vector<uint8_t> box((size_t)nx * ny * nz, 0);
    for (int z = 0; z < 4; ++z)
        for (int y = 2; y < 5; ++y)
            for (int x = 4; x < 7; ++x) box[((size_t)z * ny + y) * nx + x] = 1;
    for (int z = 0; z < 6; ++z) box[((size_t)z * ny + 6) * nx + 10] = 1;
    const int urban[6] = {1, 2, 4, 4, 0, 3};
    const int closed[6] = {0, 0, 0, 0, 0, 0};
    const int walls_y[6] = {1, 2, 0, 0, 0, 3};
    geometry(nx, ny, nz, urban, box);
    geometry(nx, ny, nz, closed, box);
    geometry(nx, ny, nz, walls_y, box);
    std::vector<uint8_t> none((size_t)nx * ny * nz, 0);
    const int per[6] = {4, 4, 4, 4, 4, 4};
    geometry(nx, ny, nz, per, none);
    const int cn = 16, ch = 6;
    std::vector<uint8_t> cyl((size_t)cn * cn * ch, 0);
    for (int z = 0; z < ch; ++z)
        for (int y = 0; y < cn; ++y)
            for (int x = 0; x < cn; ++x) {
                const double dx = x + 0.5 - cn / 2.0, dy = y + 0.5 - cn / 2.0;
                if (dx * dx + dy * dy > 36.0) cyl[((size_t)z * cn + y) * cn + x] = 2;
            }
    cyl[((size_t)0 * cn + 8) * cn + 8] = 1;
    const int cfaces[6] = {0, 0, 0, 0, 0, 3};
    geometry(cn, cn, ch, cfaces, cyl);
    if (bad) std::fprintf(stderr, "host sanitizer driver: FAILED\n");
    else std::printf("host sanitizer driver: ok\n");
    return bad;
}
