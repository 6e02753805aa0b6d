/* Sanitizer driver of the FP64 oracle: built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_sanitizers.py, it runs every
 * exported oracle routine on small cases that reach every boundary rule
 * (inlet, outlet, free-slip sky, ground, buildings, periodic faces, the
 * cylinder mantle), every collision model and every inflow kind, and fails
 * on any memory or undefined-behaviour error, or a non-finite result. */
#include "../../oracle/lbm_oracle.c"

#include <stdio.h>

static int bad = 0;

static void check_finite(const double *v, long n, const char *what)
{
    for (long i = 0; i < n; ++i)
        if (!isfinite(v[i])) {
            fprintf(stderr, "non-finite %s at %ld\n", what, i);
            bad = 1;
            return;
        }
}

static void run_case(int nx, int ny, int nz, const int face[6], const unsigned char *solid, int model, int inflow,
                     const double *series, int series_len)
{
    orc_case k;
    memset(&k, 0, sizeof k);
    k.nx = nx; k.ny = ny; k.nz = nz;
    for (int i = 0; i < 6; ++i) k.face[i] = face[i];
    k.solid = solid;
    k.model = model;
    k.tau0 = 0.56;
    k.cs = model ? 0.15 : 0.0;
    k.inflow = inflow;
    k.theta[0] = inflow == IN_SERIES ? 1.05 : (inflow == IN_LOGLAW ? 0.004 : 0.03);
    k.theta[1] = 0.1;
    k.theta[2] = inflow == IN_UNIFORM ? 0.0 : 0.5;
    k.ramp = 4;
    k.series = series;
    k.series_len = series_len;
    k.hour_steps = 3;
    k.blend_steps = 2;
    k.ref_height = nz;
    if (orc_check_case(&k) != 0) {
        fprintf(stderr, "case rejected (model %d inflow %d)\n", model, inflow);
        bad = 1;
        return;
    }
    long n = (long)nx * ny * nz;
    double *f = malloc(sizeof(double) * NQ * n), *g = malloc(sizeof(double) * NQ * n);
    double *lam = malloc(sizeof(double) * NQ * n), *lam2 = malloc(sizeof(double) * NQ * n);
    double *rho = malloc(sizeof(double) * n), *u = malloc(sizeof(double) * 3 * n);
    int *rules = malloc(sizeof(int) * NQ * n);
    orc_init(&k, f);
    for (long s = 0; s < 12; ++s) {
        orc_step(&k, s, f, g);
        double *t = f; f = g; g = t;
    }
    check_finite(f, NQ * n, "populations");
    orc_macros(&k, f, rho, u);
    check_finite(u, 3 * n, "velocity");
    orc_link_rules(&k, rules);
    for (long i = 0; i < NQ * n; ++i) lam[i] = 1e-3 * (double)((i * 7919) % 101) - 0.05;
    double grad[3] = {0.0, 0.0, 0.0};
    for (long s = 11; s >= 0; --s) {
        orc_adjoint_step(&k, s, f, lam, lam2, grad);
        double *t = lam; lam = lam2; lam2 = t;
    }
    check_finite(lam, NQ * n, "adjoint");
    check_finite(grad, 3, "gradient");
    double fc[NQ], fs[NQ], J[NQ * NQ], uin[3];
    for (int i = 0; i < NQ; ++i) fc[i] = f[(long)i * n];
    orc_collide_cell(&k, fc, fs);
    orc_collision_jacobian(&k, fc, J);
    check_finite(J, NQ * NQ, "jacobian");
    for (int z = 0; z < nz; ++z) orc_inflow_velocity(&k, z, 7, uin);
    free(f); free(g); free(lam); free(lam2); free(rho); free(u); free(rules);
}

int main(void)
{
    int c[NQ * 3], opp[NQ];
    double w[NQ], feq[NQ], P[16 * NQ], N[16], uu[3] = {0.02, -0.01, 0.005};
    orc_lattice(c, w, opp);
    orc_equilibrium(1.01, uu, feq);
    orc_equilibrium3(1.01, uu, feq);
    orc_rr3_basis(P, N);
    check_finite(feq, NQ, "equilibrium");
    if (!isfinite(orc_tau_eff(0.51, 0.1, 1.0, 0.01))) bad = 1;
    (void)orc_set_threads(0);

    /* urban box: inlet, outlet, periodic y, ground, free-slip sky, two buildings */
    const int nx = 12, ny = 6, nz = 7;
    unsigned char box[12 * 6 * 7];
    memset(box, 0, sizeof box);
    for (int z = 0; z < 3; ++z)
        for (int y = 1; y < 3; ++y)
            for (int x = 3; x < 5; ++x) box[(z * ny + y) * nx + x] = S_BUILDING;
    for (int z = 0; z < 5; ++z) box[(z * ny + 4) * nx + 7] = S_BUILDING;
    const int urban[6] = {F_INLET, F_OUTLET, F_PERIODIC, F_PERIODIC, F_WALL, F_FREESLIP};
    const double series[6] = {0.02, 0.0, 0.025, 0.3, 0.018, -2.9};
    for (int m = 0; m < 3; ++m) {
        run_case(nx, ny, nz, urban, box, m, IN_UNIFORM, NULL, 0);
        run_case(nx, ny, nz, urban, box, m, IN_LOGLAW, NULL, 0);
        run_case(nx, ny, nz, urban, box, m, IN_SERIES, series, 3);
    }
    /* closed box with walls everywhere, and a fully periodic box */
    const int walls[6] = {F_WALL, F_WALL, F_WALL, F_WALL, F_WALL, F_WALL};
    const int per[6] = {F_PERIODIC, F_PERIODIC, F_PERIODIC, F_PERIODIC, F_PERIODIC, F_PERIODIC};
    run_case(nx, ny, nz, walls, box, 1, IN_UNIFORM, NULL, 0);
    unsigned char none[12 * 6 * 7];
    memset(none, 0, sizeof none);
    run_case(nx, ny, nz, per, none, 2, IN_UNIFORM, NULL, 0);
    /* cylinder: mantle cells outside a disk, free-slip sky, ground */
    const int cn = 14, ch = 5;
    unsigned char cyl[14 * 14 * 5];
    for (int z = 0; z < ch; ++z)
        for (int y = 0; y < cn; ++y)
            for (int x = 0; x < cn; ++x) {
                double dx = x + 0.5 - cn / 2.0, dy = y + 0.5 - cn / 2.0;
                cyl[(z * cn + y) * cn + x] = (dx * dx + dy * dy > 25.0) ? S_MANTLE : S_FLUID;
            }
    cyl[(0 * cn + 7) * cn + 7] = S_BUILDING;
    const int cfaces[6] = {F_WALL, F_WALL, F_WALL, F_WALL, F_WALL, F_FREESLIP};
    for (int m = 0; m < 3; ++m) run_case(cn, cn, ch, cfaces, cyl, m, IN_SERIES, series, 3);
    if (bad) fprintf(stderr, "oracle sanitizer driver: FAILED\n");
    else printf("oracle sanitizer driver: ok\n");
    return bad;
}
