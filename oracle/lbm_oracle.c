/*
 * lbm_oracle.c -- plain, slow FP64 reference of the SC-LBM hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or table with the
 * GPU library.
 *
 * What it computes (arXiv 2508.18202, Sec. 2.2 "Deterministic lattice
 * Boltzmann method"):
 *   - D3Q19 velocity set (Fig. 1), c_s^2 = 1/3;
 *   - the lattice Boltzmann update of Eq. (deterministicLBE) with the
 *     non-equilibrium part left unprojected (BGK), second-order equilibrium
 *     (the truncation of the Hermite equilibrium of Sec. 2.2 at n = 2);
 *   - effective relaxation time of Eq. (tauEff) with the Smagorinsky-Lilly
 *     eddy viscosity of Eq. (turbVisc), |S| evaluated from the local
 *     non-equilibrium stress;
 *   - the regularised collision of Eq. (deterministicLBE) as printed: the
 *     equilibrium expanded to third order and f^(1) = f - f^eq replaced by
 *     its expansion to third order with the Hermite coefficients of
 *     Eq. (hermiteCoeff), in the Hermite polynomials that are orthogonal on
 *     D3Q19 (model M_RR3, with the Smagorinsky tau_eff);
 *   - bounce-back walls/ground, a local velocity (moving-wall bounce-back)
 *     inflow, a zero-gradient outflow and a free-slip sky (Sec. 2.2 boundary
 *     list), plus periodic faces;
 *   - the cylindrical domain of Secs. 2.2 and 3: cells of the solid mask
 *     coded 2 are the exterior of the cylinder, and every link crossing into
 *     them carries the local velocity condition of the wind (the mantle);
 *   - the discrete adjoint of one step (not in the paper; used for the
 *     inflow-parameter gradients).
 *
 * Storage: full populations f_i (not shifted), layout [q][z][y][x], x fastest.
 * Every step is a two-lattice pull: f_out(x, i) = rule(x, i) applied to the
 * post-collision populations of f_in.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NQ 19

enum { F_WALL = 0, F_INLET = 1, F_OUTLET = 2, F_FREESLIP = 3, F_PERIODIC = 4 };
enum { M_BGK = 0, M_SMAG = 1, M_RR3 = 2 };
enum { IN_UNIFORM = 0, IN_LOGLAW = 1, IN_SERIES = 2 };

typedef struct {
    int nx, ny, nz;
    int face[6];                 /* -x, +x, -y, +y, -z, +z */
    const unsigned char *solid;  /* nx*ny*nz, 1 = solid */
    int model;
    double tau0, cs;
    int inflow;
    double theta[3];             /* uniform: (U, phi, -); log-law: (u*, phi, z0) */
    int ramp;                    /* inflow ramp length in steps (0 = none) */
    double force[3];             /* uniform body force (Guo); zero in the workloads */
    /* measured-series inflow (IN_SERIES): hourly reference speed and direction
     * (rad) as series[2 h], series[2 h + 1], h < series_len; theta = (zeta1
     * speed multiplier, zeta2 direction offset in rad, z0) */
    const double *series;
    int series_len, hour_steps, blend_steps;
    double ref_height;           /* H of the normalised log profile (cells) */
} orc_case;

/* D3Q19 velocities in the canonical order: rest, 6 faces (+x,-x,+y,-y,+z,-z),
 * then the 12 edges (+x+y, -x-y, +x-y, -x+y, +x+z, -x-z, +x-z, -x+z,
 * +y+z, -y-z, +y-z, -y+z).  Fig. 1 shows the set; the order is ours. */
static const int C[NQ][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
};

/* Weight from the energy shell |c|^2 = 0, 1, 2 (Fig. 1 caption). */
static double weight(int i)
{
    int c2 = C[i][0] * C[i][0] + C[i][1] * C[i][1] + C[i][2] * C[i][2];
    return c2 == 0 ? 1.0 / 3.0 : (c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

/* Index of the velocity (a, b, c), found by search. */
static int find_vel(int a, int b, int c)
{
    for (int j = 0; j < NQ; ++j)
        if (C[j][0] == a && C[j][1] == b && C[j][2] == c) return j;
    return -1;
}

static int opposite(int i) { return find_vel(-C[i][0], -C[i][1], -C[i][2]); }
static int zflip(int i) { return find_vel(C[i][0], C[i][1], -C[i][2]); }

static long cell_index(const orc_case *k, int x, int y, int z)
{
    return ((long)z * k->ny + y) * k->nx + x;
}

static long ncells(const orc_case *k) { return (long)k->nx * k->ny * k->nz; }

static int wrap(int v, int n) { return ((v % n) + n) % n; }

void orc_lattice(int *c_out, double *w_out, int *opp_out)
{
    for (int i = 0; i < NQ; ++i) {
        for (int a = 0; a < 3; ++a) c_out[3 * i + a] = C[i][a];
        w_out[i] = weight(i);
        opp_out[i] = opposite(i);
    }
}

/* Second-order equilibrium, f_i^eq = w_i rho (1 + c.u/cs2 + (c.u)^2/(2 cs4) - u.u/(2 cs2)). */
void orc_equilibrium(double rho, const double *u, double *feq)
{
    const double cs2 = 1.0 / 3.0;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < NQ; ++i) {
        double cu = C[i][0] * u[0] + C[i][1] * u[1] + C[i][2] * u[2];
        feq[i] = weight(i) * rho *
                 (1.0 + cu / cs2 + cu * cu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
    }
}

/* rho = sum f, rho u = sum c f (+ F/2 with a body force, Guo et al. 2002). */
static void moments(const orc_case *k, const double *f, double *rho, double *u)
{
    double r = 0.0, m[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < NQ; ++i) {
        r += f[i];
        for (int a = 0; a < 3; ++a) m[a] += C[i][a] * f[i];
    }
    *rho = r;
    for (int a = 0; a < 3; ++a) u[a] = (m[a] + 0.5 * k->force[a]) / r;
}

/* Smagorinsky effective relaxation time.  With nu_t = (Cs dx)^2 |S|,
 * |S| = sqrt(2 S:S) and S = -Pi_neq / (2 rho cs2 tau_eff) (dt = dx = 1),
 * Eq. (tauEff) becomes tau^2 - tau0 tau - 9 Cs^2 Q / (sqrt(2) rho) = 0 with
 * Q = sqrt(Pi_neq : Pi_neq); the positive root is returned. */
double orc_tau_eff(double tau0, double cs, double rho, double q)
{
    return 0.5 * (tau0 + sqrt(tau0 * tau0 + 18.0 * sqrt(2.0) * cs * cs * q / rho));
}

/* Q = sqrt(Pi:Pi) of the non-equilibrium second moment. */
static double neq_norm(const double *f, const double *feq, double pi[3][3])
{
    double s = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double p = 0.0;
            for (int i = 0; i < NQ; ++i) p += C[i][a] * C[i][b] * (f[i] - feq[i]);
            pi[a][b] = p;
            s += p * p;
        }
    return sqrt(s);
}

/* ---- Regularised third-order collision (Sec. 2.2, Eq. (deterministicLBE),
 * Eq. (hermiteCoeff)).
 *
 * Basis: the Hermite polynomials in c_i up to third order that are mutually
 * orthogonal on D3Q19 under sum_i w_i P(c_i) Q(c_i):
 *   order 0: 1;  order 1: c_a;  order 2: H_aa = c_a^2 - cs2, H_ab = c_a c_b;
 *   order 3: H_xxy +- H_yzz, H_xzz +- H_xyy, H_yyz +- H_xxz, with
 *   H_aab = c_b (c_a^2 - cs2).  (H_aaa and H_xyz vanish on D3Q19, and the six
 *   mixed third-order polynomials are orthogonal only in these sums and
 *   differences.)
 * Each basis polynomial P_k is paired with the Maxwellian's Hermite
 * coefficient in the same combination, per unit density: A_k(u) = 1, u_a,
 * u_a u_b, u_x^2 u_y +- u_y u_z^2, ...  With the norms
 * N_k = sum_i w_i P_k(c_i)^2 of the velocity set:
 *   f_eq_i   = w_i rho sum_k P_k(c_i) A_k(u) / N_k            (orders 0..3)
 *   a1_k     = sum_i P_k(c_i) (f_i - f_eq_i)                    (orders 2, 3)
 *   f1_reg_i = w_i sum_k P_k(c_i) a1_k / N_k                   (orders 2, 3)
 *   f*_i     = f_eq_i + (1 - 1/tau_eff) f1_reg_i. */
#define NB 16
static int basis_order(int k) { return k == 0 ? 0 : (k < 4 ? 1 : (k < 10 ? 2 : 3)); }

static double basis_poly(int k, const double *c)
{
    const double s = 1.0 / 3.0;
    const double x = c[0], y = c[1], z = c[2];
    const double hxxy = y * (x * x - s), hyzz = y * (z * z - s);
    const double hxzz = x * (z * z - s), hxyy = x * (y * y - s);
    const double hyyz = z * (y * y - s), hxxz = z * (x * x - s);
    switch (k) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * x - s;
    case 5: return y * y - s;
    case 6: return z * z - s;
    case 7: return x * y;
    case 8: return x * z;
    case 9: return y * z;
    case 10: return hxxy + hyzz;
    case 11: return hxxy - hyzz;
    case 12: return hxzz + hxyy;
    case 13: return hxzz - hxyy;
    case 14: return hyyz + hxxz;
    default: return hyyz - hxxz;
    }
}

/* Maxwellian Hermite coefficient of P_k per unit density: the same
 * combination of the monomials u_a u_b (u_c). */
static double basis_coef(int k, const double *u)
{
    const double x = u[0], y = u[1], z = u[2];
    switch (k) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * x;
    case 5: return y * y;
    case 6: return z * z;
    case 7: return x * y;
    case 8: return x * z;
    case 9: return y * z;
    case 10: return x * x * y + y * z * z;
    case 11: return x * x * y - y * z * z;
    case 12: return x * z * z + x * y * y;
    case 13: return x * z * z - x * y * y;
    case 14: return y * y * z + x * x * z;
    default: return y * y * z - x * x * z;
    }
}

/* g[a] = d A_k(u) / d u_a of the coefficient above. */
static void basis_coef_grad(int k, const double *u, double g[3])
{
    const double x = u[0], y = u[1], z = u[2];
    g[0] = g[1] = g[2] = 0.0;
    switch (k) {
    case 0: break;
    case 1: g[0] = 1.0; break;
    case 2: g[1] = 1.0; break;
    case 3: g[2] = 1.0; break;
    case 4: g[0] = 2.0 * x; break;
    case 5: g[1] = 2.0 * y; break;
    case 6: g[2] = 2.0 * z; break;
    case 7: g[0] = y; g[1] = x; break;
    case 8: g[0] = z; g[2] = x; break;
    case 9: g[1] = z; g[2] = y; break;
    case 10: g[0] = 2.0 * x * y; g[1] = x * x + z * z; g[2] = 2.0 * y * z; break;
    case 11: g[0] = 2.0 * x * y; g[1] = x * x - z * z; g[2] = -2.0 * y * z; break;
    case 12: g[0] = z * z + y * y; g[1] = 2.0 * x * y; g[2] = 2.0 * x * z; break;
    case 13: g[0] = z * z - y * y; g[1] = -2.0 * x * y; g[2] = 2.0 * x * z; break;
    case 14: g[0] = 2.0 * x * z; g[1] = 2.0 * y * z; g[2] = y * y + x * x; break;
    default: g[0] = -2.0 * x * z; g[1] = 2.0 * y * z; g[2] = y * y - x * x; break;
    }
}

/* P[k][i] = P_k(c_i) and N[k] = sum_i w_i P_k(c_i)^2. */
void orc_rr3_basis(double *P, double *N)
{
    for (int k = 0; k < NB; ++k) {
        N[k] = 0.0;
        for (int i = 0; i < NQ; ++i) {
            double c[3] = {C[i][0], C[i][1], C[i][2]};
            P[k * NQ + i] = basis_poly(k, c);
            N[k] += weight(i) * P[k * NQ + i] * P[k * NQ + i];
        }
    }
}

/* Third-order equilibrium in the D3Q19-orthogonal Hermite basis. */
void orc_equilibrium3(double rho, const double *u, double *feq)
{
    double P[NB * NQ], N[NB];
    orc_rr3_basis(P, N);
    for (int i = 0; i < NQ; ++i) {
        double s = 0.0;
        for (int k = 0; k < NB; ++k) s += P[k * NQ + i] * basis_coef(k, u) / N[k];
        feq[i] = weight(i) * rho * s;
    }
}

static void collide_rr3(const orc_case *k, const double *f, double *fstar)
{
    double rho, u[3], feq[NQ], f1[NQ], pi[3][3], P[NB * NQ], N[NB];
    moments(k, f, &rho, u);
    orc_equilibrium3(rho, u, feq);
    for (int i = 0; i < NQ; ++i) f1[i] = f[i] - feq[i];
    const double tau = orc_tau_eff(k->tau0, k->cs, rho, neq_norm(f, feq, pi));
    orc_rr3_basis(P, N);
    double a1[NB];
    for (int b = 0; b < NB; ++b) {
        a1[b] = 0.0;
        if (basis_order(b) < 2) continue;
        for (int i = 0; i < NQ; ++i) a1[b] += P[b * NQ + i] * f1[i];
    }
    for (int i = 0; i < NQ; ++i) {
        double r = 0.0;
        for (int b = 0; b < NB; ++b)
            if (basis_order(b) >= 2) r += P[b * NQ + i] * a1[b] / N[b];
        fstar[i] = feq[i] + (1.0 - 1.0 / tau) * weight(i) * r;
    }
}

/* Local collision of one fluid cell: f* = f - (1/tau_eff)(f - f_eq) [+ Guo force term];
 * the regularised model goes through collide_rr3. */
void orc_collide_cell(const orc_case *k, const double *f, double *fstar)
{
    double rho, u[3], feq[NQ], pi[3][3];
    if (k->model == M_RR3) {
        collide_rr3(k, f, fstar);
        return;
    }
    moments(k, f, &rho, u);
    orc_equilibrium(rho, u, feq);
    double tau = k->tau0;
    if (k->model == M_SMAG) tau = orc_tau_eff(k->tau0, k->cs, rho, neq_norm(f, feq, pi));
    double om = 1.0 / tau;
    for (int i = 0; i < NQ; ++i) {
        double fi = 0.0;
        if (k->force[0] != 0.0 || k->force[1] != 0.0 || k->force[2] != 0.0) {
            double cu = C[i][0] * u[0] + C[i][1] * u[1] + C[i][2] * u[2];
            for (int a = 0; a < 3; ++a)
                fi += (3.0 * (C[i][a] - u[a]) + 9.0 * cu * C[i][a]) * k->force[a];
            fi *= (1.0 - 0.5 * om) * weight(i);
        }
        fstar[i] = f[i] - om * (f[i] - feq[i]) + fi;
    }
}

/* Inflow ramp r(n) = (1 - cos(pi n / T_r)) / 2 for n < T_r, else 1. */
static double ramp_factor(const orc_case *k, long n)
{
    if (k->ramp <= 0 || n >= k->ramp) return 1.0;
    return 0.5 * (1.0 - cos(M_PI * (double)n / (double)k->ramp));
}

/* Reference speed and direction of the measured series at step n (Sec. 3):
 * hour h starts at step ramp + h * hour_steps; during its first blend_steps
 * steps the values move from those of hour h-1 to those of hour h with the
 * weight (1 - cos(pi t / blend_steps)) / 2, the direction along the shorter
 * arc; afterwards they are held.  Before and during the ramp the values of
 * hour 0 apply; past the last hour its values are held. */
static void series_at(const orc_case *k, long n, double *U, double *D)
{
    long t = n - k->ramp;
    if (t < 0) t = 0;
    long h = t / k->hour_steps, tp = t - h * k->hour_steps;
    if (h >= k->series_len) {
        h = k->series_len - 1;
        tp = k->hour_steps;
    }
    *U = k->series[2 * h];
    *D = k->series[2 * h + 1];
    if (h > 0 && tp < k->blend_steps) {
        double s = 0.5 * (1.0 - cos(M_PI * (double)tp / (double)k->blend_steps));
        double U0 = k->series[2 * h - 2], D0 = k->series[2 * h - 1];
        double dD = remainder(*D - D0, 2.0 * M_PI);   /* shorter arc, in [-pi, pi] */
        *U = U0 + s * (*U - U0);
        *D = D0 + s * dD;
    }
}

/* Inflow velocity u_in(z, n) (ramp included) and its derivatives w.r.t.
 * theta at height index z (cell centre z + 1/2 above the half-way ground).
 *   uniform: U = theta0, direction phi = theta1;
 *   log-law: U(z) = (u_star / 0.41) ln((z + 1/2) / z0), theta = (u_star, phi, z0);
 *   series:  U(z) = zeta1 U_H(n) ln((h + z0) / z0) / ln((H + z0) / z0), h = z + 1/2,
 *            direction Theta(n) + zeta2 (Sec. 3 perturbation of the measured
 *            series and normalised log profile), theta = (zeta1, zeta2, z0).
 * Velocity U (cos phi, sin phi, 0); dudth[3][3]: d u_a / d theta_k. */
static void inflow_at(const orc_case *k, int z, long n, double u[3], double dudth[3][3])
{
    double phi = k->theta[1];
    double U, dU[3] = {0.0, 0.0, 0.0};
    if (k->inflow == IN_UNIFORM) {
        U = k->theta[0];
        dU[0] = 1.0;
    } else if (k->inflow == IN_LOGLAW) {
        double us = k->theta[0], z0 = k->theta[2], h = z + 0.5;
        U = us / 0.41 * log(h / z0);
        dU[0] = log(h / z0) / 0.41;
        dU[2] = -us / (0.41 * z0);
    } else {
        double UH, Th;
        series_at(k, n, &UH, &Th);
        double z1 = k->theta[0], z0 = k->theta[2], h = z + 0.5, H = k->ref_height;
        double A = log((h + z0) / z0), B = log((H + z0) / z0);
        double dA = 1.0 / (h + z0) - 1.0 / z0, dB = 1.0 / (H + z0) - 1.0 / z0;
        U = z1 * UH * A / B;
        dU[0] = UH * A / B;
        dU[2] = z1 * UH * (dA * B - A * dB) / (B * B);
        phi = Th + k->theta[1];
    }
    double r = ramp_factor(k, n);
    double dir[3] = {cos(phi), sin(phi), 0.0};
    double ddir[3] = {-sin(phi), cos(phi), 0.0};
    for (int a = 0; a < 3; ++a) {
        u[a] = r * U * dir[a];
        for (int t = 0; t < 3; ++t) dudth[a][t] = r * dU[t] * dir[a];
        dudth[a][1] = r * U * ddir[a];
    }
}

void orc_inflow_velocity(const orc_case *k, int z, long n, double *u)
{
    double d[3][3];
    inflow_at(k, z, n, u, d);
}

enum { R_STREAM = 0, R_BOUNCE = 1, R_INLET = 2, R_FREESLIP = 3, R_OUTLET = 4, R_REST = 5, R_MANTLE = 6 };

/* Cell kinds of the solid mask: fluid, building (no-slip bounce-back) and
 * mantle (the exterior of a cylindrical domain, whose surface carries the
 * local velocity condition of the wind). */
enum { S_FLUID = 0, S_BUILDING = 1, S_MANTLE = 2 };

/* Pull rule of destination link (x, i): returns the rule kind and writes the
 * source cell and the post-collision population index that f_out(x, i) is
 * taken from.  Rules, first match wins, with s = x - c_i (periodic axes
 * wrapped):
 *   R1 s is a building cell, or s leaves the box through a WALL face:
 *      bounce-back, source (x, opp(i));
 *   R6 s is a mantle cell: the velocity condition of the mantle, the
 *      moving-wall bounce-back of R2 with the wind u_in(z, n) of the cell's
 *      height;
 *   R2 s.x < 0 through the INLET face: moving-wall bounce-back, source
 *      (x, opp(i)) plus 6 w_i rho_w c_i.u_in with rho_w = 1;
 *   R3 s.z >= nz through the FREESLIP sky: specular reflection, source
 *      m = (x - c_ix, y - c_iy, nz-1) with c_z flipped, a source at x = nx
 *      clamped to nx-1; when m is a mantle cell the reflected path crosses the
 *      mantle and R6 applies instead;
 *   R4 s.x >= nx through the OUTLET face: zero gradient, source (nx-1, s.y, s.z),
 *      same population;
 *   R5 otherwise plain streaming from (s, i).
 */
static int pull_rule(const orc_case *k, int x, int y, int z, int i,
                     int *sx_o, int *sy_o, int *sz_o, int *pop_o)
{
    if (i == 0) { *sx_o = x; *sy_o = y; *sz_o = z; *pop_o = 0; return R_REST; }
    int sx = x - C[i][0], sy = y - C[i][1], sz = z - C[i][2];
    if (k->face[0] == F_PERIODIC) sx = wrap(sx, k->nx);
    if (k->face[2] == F_PERIODIC) sy = wrap(sy, k->ny);
    if (k->face[4] == F_PERIODIC) sz = wrap(sz, k->nz);
    int inside = sx >= 0 && sx < k->nx && sy >= 0 && sy < k->ny && sz >= 0 && sz < k->nz;
    int wall_exit = (sx < 0 && k->face[0] == F_WALL) || (sx >= k->nx && k->face[1] == F_WALL) ||
                    (sy < 0 && k->face[2] == F_WALL) || (sy >= k->ny && k->face[3] == F_WALL) ||
                    (sz < 0 && k->face[4] == F_WALL) || (sz >= k->nz && k->face[5] == F_WALL);
    int kind = inside ? k->solid[cell_index(k, sx, sy, sz)] : S_FLUID;
    if (kind == S_BUILDING || wall_exit) {
        *sx_o = x; *sy_o = y; *sz_o = z; *pop_o = opposite(i);
        return R_BOUNCE;
    }
    if (kind == S_MANTLE) {
        *sx_o = x; *sy_o = y; *sz_o = z; *pop_o = opposite(i);
        return R_MANTLE;
    }
    if (sx < 0 && k->face[0] == F_INLET) {
        *sx_o = x; *sy_o = y; *sz_o = z; *pop_o = opposite(i);
        return R_INLET;
    }
    if (sz >= k->nz && k->face[5] == F_FREESLIP) {
        int px = sx;  /* x - c_ix, already wrapped when x is periodic */
        if (px >= k->nx && k->face[1] == F_OUTLET) px = k->nx - 1;
        if (k->solid[cell_index(k, px, sy, k->nz - 1)] == S_MANTLE) {
            *sx_o = x; *sy_o = y; *sz_o = z; *pop_o = opposite(i);
            return R_MANTLE;
        }
        *sx_o = px; *sy_o = sy; *sz_o = k->nz - 1; *pop_o = zflip(i);
        return R_FREESLIP;
    }
    if (sx >= k->nx && k->face[1] == F_OUTLET) {
        *sx_o = k->nx - 1; *sy_o = sy; *sz_o = sz; *pop_o = i;
        return R_OUTLET;
    }
    *sx_o = sx; *sy_o = sy; *sz_o = sz; *pop_o = i;
    return R_STREAM;
}

/* Validity of a case: face combinations and the cells the rules read. */
int orc_check_case(const orc_case *k)
{
    if (k->nx < 1 || k->ny < 1 || k->nz < 1) return 1;
    int ok0 = k->face[0] == F_WALL || k->face[0] == F_INLET || k->face[0] == F_PERIODIC;
    int ok1 = k->face[1] == F_WALL || k->face[1] == F_OUTLET || k->face[1] == F_PERIODIC;
    int ok5 = k->face[5] == F_WALL || k->face[5] == F_FREESLIP || k->face[5] == F_PERIODIC;
    int oky = (k->face[2] == F_WALL || k->face[2] == F_PERIODIC) &&
              (k->face[3] == F_WALL || k->face[3] == F_PERIODIC);
    int ok4 = k->face[4] == F_WALL || k->face[4] == F_PERIODIC;
    if (!(ok0 && ok1 && ok5 && oky && ok4)) return 2;
    for (int a = 0; a < 3; ++a)
        if ((k->face[2 * a] == F_PERIODIC) != (k->face[2 * a + 1] == F_PERIODIC)) return 3;
    if (k->tau0 <= 0.5) return 4;
    if (k->inflow == IN_SERIES &&
        (!k->series || k->series_len < 1 || k->hour_steps < 1 || k->blend_steps < 0 ||
         k->blend_steps > k->hour_steps || !(k->ref_height > 0.0) || !(k->theta[2] > 0.0)))
        return 7;
    /* the free-slip and outflow rules read top-layer / last-column cells; a
     * mantle column may reach the sky (R3 turns into R6 there) */
    for (int z = 0; z < k->nz; ++z)
        for (int y = 0; y < k->ny; ++y)
            for (int x = 0; x < k->nx; ++x) {
                int kind = k->solid[cell_index(k, x, y, z)];
                if (kind > S_MANTLE) return 9;
                if (kind == S_FLUID) {
                    /* one fluid cell borders buildings or the mantle, not both */
                    int seen = 0;
                    for (int i = 1; i < NQ; ++i) {
                        int sx = x - C[i][0], sy = y - C[i][1], sz = z - C[i][2];
                        if (k->face[0] == F_PERIODIC) sx = wrap(sx, k->nx);
                        if (k->face[2] == F_PERIODIC) sy = wrap(sy, k->ny);
                        if (k->face[4] == F_PERIODIC) sz = wrap(sz, k->nz);
                        if (sx < 0 || sx >= k->nx || sy < 0 || sy >= k->ny || sz < 0 || sz >= k->nz) continue;
                        seen |= 1 << k->solid[cell_index(k, sx, sy, sz)];
                    }
                    if ((seen & (1 << S_BUILDING)) && (seen & (1 << S_MANTLE))) return 8;
                    continue;
                }
                if (k->face[5] == F_FREESLIP && z == k->nz - 1 && kind == S_BUILDING) return 5;
                if (k->face[1] == F_OUTLET && x == k->nx - 1) return 6;
            }
    return 0;
}

void orc_init(const orc_case *k, double *f)
{
    long n = ncells(k);
    for (int i = 0; i < NQ; ++i)
        for (long c = 0; c < n; ++c) f[i * n + c] = weight(i);
}

/* rho, u (layout [3][cells]) of every cell; solid cells report rho = 1, u = 0. */
void orc_macros(const orc_case *k, const double *f, double *rho, double *u)
{
    long n = ncells(k);
    for (long c = 0; c < n; ++c) {
        if (k->solid[c]) {
            rho[c] = 1.0; u[c] = u[n + c] = u[2 * n + c] = 0.0;
            continue;
        }
        double fl[NQ], r, v[3];
        for (int i = 0; i < NQ; ++i) fl[i] = f[i * n + c];
        moments(k, fl, &r, v);
        rho[c] = r;
        for (int a = 0; a < 3; ++a) u[a * n + c] = v[a];
    }
}

/* One time step n -> n+1 (two lattices): collide every fluid cell, then pull. */
void orc_step(const orc_case *k, long step, const double *fin, double *fout)
{
    long n = ncells(k);
    double *fs = (double *)malloc(sizeof(double) * NQ * n);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c) {
        double fl[NQ], fsl[NQ];
        if (k->solid[c]) {
            for (int i = 0; i < NQ; ++i) fs[i * n + c] = weight(i);
            continue;
        }
        for (int i = 0; i < NQ; ++i) fl[i] = fin[i * n + c];
        orc_collide_cell(k, fl, fsl);
        for (int i = 0; i < NQ; ++i) fs[i * n + c] = fsl[i];
    }
#pragma omp parallel for schedule(static)
    for (int z = 0; z < k->nz; ++z)
        for (int y = 0; y < k->ny; ++y)
            for (int x = 0; x < k->nx; ++x) {
                long c = cell_index(k, x, y, z);
                if (k->solid[c]) {
                    for (int i = 0; i < NQ; ++i) fout[i * n + c] = weight(i);
                    continue;
                }
                for (int i = 0; i < NQ; ++i) {
                    int sx, sy, sz, p;
                    int rule = pull_rule(k, x, y, z, i, &sx, &sy, &sz, &p);
                    double v = fs[p * n + cell_index(k, sx, sy, sz)];
                    if (rule == R_INLET || rule == R_MANTLE) {
                        double uin[3], d[3][3];
                        inflow_at(k, z, step, uin, d);
                        double cu = C[i][0] * uin[0] + C[i][1] * uin[1] + C[i][2] * uin[2];
                        v += 6.0 * weight(i) * 1.0 * cu;
                    }
                    fout[i * n + c] = v;
                }
            }
    free(fs);
}

/* Rule of every link, for tests: rules[i*ncells + c] (-1 for solid cells). */
void orc_link_rules(const orc_case *k, int *rules)
{
    long n = ncells(k);
    for (int z = 0; z < k->nz; ++z)
        for (int y = 0; y < k->ny; ++y)
            for (int x = 0; x < k->nx; ++x) {
                long c = cell_index(k, x, y, z);
                for (int i = 0; i < NQ; ++i) {
                    int sx, sy, sz, p;
                    rules[i * n + c] = k->solid[c] ? -1 : pull_rule(k, x, y, z, i, &sx, &sy, &sz, &p);
                }
            }
}

/* Jacobian J[i][k] = d fstar_i / d f_k of the local collision (no body force),
 * by the chain rule through rho, u, f_eq and (Smagorinsky) tau_eff.  For the
 * regularised model, f* = f_eq3 + (1 - om) R (f - f_eq3) with the linear
 * projector R_ij = w_i sum_{order 2, 3} P_b(c_i) P_b(c_j) / N_b, so
 * J = A + (1 - om) R (I - A) - (R (f - f_eq3)) d om / d f with A = d f_eq3 / d f. */
static void collision_jacobian(const orc_case *k, const double *f, double J[NQ][NQ])
{
    double rho, u[3], feq[NQ], pi[3][3];
    const int rr3 = k->model == M_RR3;
    moments(k, f, &rho, u);
    if (rr3) orc_equilibrium3(rho, u, feq);
    else orc_equilibrium(rho, u, feq);
    const double cs2 = 1.0 / 3.0;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];

    /* d rho / d f_k = 1 ; d u_a / d f_k = (c_ka - u_a) / rho */
    double du[3][NQ];
    for (int kk = 0; kk < NQ; ++kk)
        for (int a = 0; a < 3; ++a) du[a][kk] = (C[kk][a] - u[a]) / rho;

    /* d feq_i / d f_k */
    double dfeq[NQ][NQ];
    double P[NB * NQ], N[NB];
    orc_rr3_basis(P, N);
    for (int i = 0; i < NQ; ++i) {
        double drho, dua[3];
        if (rr3) {
            /* f_eq3_i = w_i rho sum_b P_b(c_i) A_b(u) / N_b */
            drho = feq[i] / rho;
            dua[0] = dua[1] = dua[2] = 0.0;
            for (int b = 0; b < NB; ++b) {
                double g[3];
                basis_coef_grad(b, u, g);
                for (int a = 0; a < 3; ++a) dua[a] += weight(i) * rho * P[b * NQ + i] * g[a] / N[b];
            }
        } else {
            double cu = C[i][0] * u[0] + C[i][1] * u[1] + C[i][2] * u[2];
            drho = weight(i) * (1.0 + cu / cs2 + cu * cu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
            for (int a = 0; a < 3; ++a)
                dua[a] = weight(i) * rho * (C[i][a] / cs2 + cu * C[i][a] / (cs2 * cs2) - u[a] / cs2);
        }
        for (int kk = 0; kk < NQ; ++kk)
            dfeq[i][kk] = drho + dua[0] * du[0][kk] + dua[1] * du[1][kk] + dua[2] * du[2][kk];
    }

    double tau = k->tau0;
    double dom[NQ];
    for (int kk = 0; kk < NQ; ++kk) dom[kk] = 0.0;
    if (k->model == M_SMAG || rr3) {
        double q = neq_norm(f, feq, pi);
        tau = orc_tau_eff(k->tau0, k->cs, rho, q);
        double K = 18.0 * sqrt(2.0) * k->cs * k->cs;
        double root = sqrt(k->tau0 * k->tau0 + K * q / rho);
        double dtau_dq = 0.25 * K / (rho * root);
        double dtau_drho = -0.25 * K * q / (rho * rho * root);
        for (int kk = 0; kk < NQ; ++kk) {
            double dq = 0.0;
            if (q > 0.0) {
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        double dpi = C[kk][a] * C[kk][b];
                        for (int i = 0; i < NQ; ++i) dpi -= C[i][a] * C[i][b] * dfeq[i][kk];
                        dq += pi[a][b] * dpi;
                    }
                dq /= q;
            }
            double dtau = dtau_dq * dq + dtau_drho * 1.0;
            dom[kk] = -dtau / (tau * tau);
        }
    }
    double om = 1.0 / tau;
    if (!rr3) {
        for (int i = 0; i < NQ; ++i)
            for (int kk = 0; kk < NQ; ++kk)
                J[i][kk] = (i == kk ? 1.0 - om : 0.0) + om * dfeq[i][kk] - (f[i] - feq[i]) * dom[kk];
        return;
    }
    double R[NQ][NQ], Rf1[NQ], IA[NQ][NQ];
    for (int i = 0; i < NQ; ++i)
        for (int j = 0; j < NQ; ++j) {
            double r = 0.0;
            for (int b = 0; b < NB; ++b)
                if (basis_order(b) >= 2) r += P[b * NQ + i] * P[b * NQ + j] / N[b];
            R[i][j] = weight(i) * r;
            IA[i][j] = (i == j ? 1.0 : 0.0) - dfeq[i][j];
        }
    for (int i = 0; i < NQ; ++i) {
        Rf1[i] = 0.0;
        for (int j = 0; j < NQ; ++j) Rf1[i] += R[i][j] * (f[j] - feq[j]);
    }
    for (int i = 0; i < NQ; ++i)
        for (int kk = 0; kk < NQ; ++kk) {
            double rj = 0.0;
            for (int j = 0; j < NQ; ++j) rj += R[i][j] * IA[j][kk];
            J[i][kk] = dfeq[i][kk] + (1.0 - om) * rj - Rf1[i] * dom[kk];
        }
}

void orc_collision_jacobian(const orc_case *k, const double *f, double *J)
{
    double Jl[NQ][NQ];
    collision_jacobian(k, f, Jl);
    for (int i = 0; i < NQ; ++i)
        for (int kk = 0; kk < NQ; ++kk) J[i * NQ + kk] = Jl[i][kk];
}

/* Discrete adjoint of step n -> n+1.
 *   mu      = P^T lam_next           (scatter-add of every pull link to its source)
 *   lam_n   = J(f_n)^T mu            (fluid cells; zero on solid cells)
 *   grad_k += sum over inlet and mantle links (x,i) of lam_next(x,i) * d b_i / d theta_k,
 * with b_i = 6 w_i rho_w c_i.u_in(z; theta) r(n).  lam_n receives no
 * objective source here; callers add dj_n/df_n. */
void orc_adjoint_step(const orc_case *k, long step, const double *f_n,
                      const double *lam_next, double *lam_n, double *grad)
{
    long n = ncells(k);
    double *mu = (double *)calloc((size_t)NQ * n, sizeof(double));
    double g[3] = {0.0, 0.0, 0.0};
    for (int z = 0; z < k->nz; ++z)
        for (int y = 0; y < k->ny; ++y)
            for (int x = 0; x < k->nx; ++x) {
                long c = cell_index(k, x, y, z);
                if (k->solid[c]) continue;
                for (int i = 0; i < NQ; ++i) {
                    int sx, sy, sz, p;
                    int rule = pull_rule(k, x, y, z, i, &sx, &sy, &sz, &p);
                    double lam = lam_next[i * n + c];
                    mu[p * n + cell_index(k, sx, sy, sz)] += lam;
                    if (rule == R_INLET || rule == R_MANTLE) {
                        double uin[3], d[3][3];
                        inflow_at(k, z, step, uin, d);
                        for (int t = 0; t < 3; ++t) {
                            double cd = C[i][0] * d[0][t] + C[i][1] * d[1][t] + C[i][2] * d[2][t];
                            g[t] += lam * 6.0 * weight(i) * cd;
                        }
                    }
                }
            }
    for (int t = 0; t < 3; ++t) grad[t] += g[t];
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c) {
        if (k->solid[c]) {
            for (int i = 0; i < NQ; ++i) lam_n[i * n + c] = 0.0;
            continue;
        }
        double fl[NQ], J[NQ][NQ];
        for (int i = 0; i < NQ; ++i) fl[i] = f_n[i * n + c];
        collision_jacobian(k, fl, J);
        for (int kk = 0; kk < NQ; ++kk) {
            double s = 0.0;
            for (int i = 0; i < NQ; ++i) s += J[i][kk] * mu[i * n + c];
            lam_n[kk * n + c] = s;
        }
    }
    free(mu);
}

/* Thread count of the OpenMP loops over cells (timing of the CPU baseline on
 * one core and on all cores); returns the count now in effect. */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
