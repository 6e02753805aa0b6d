// device.h -- device code shared by the translation units of the gfx950
// library: memory helpers, boundary rules in their wavefront form, the
// collisions, the step kernel and the adjoint kernel templates.
//
// In-place AA streaming on one FP32 population array per instance (values
// f_i - w_i):
//   even step n (state stored naturally: slot i of cell x holds f_i^n(x))
//     each cell reads its own 19 slots, collides, and writes f*_i into its own
//     slot opp(i);
//   odd step n (slots hold the swapped post-collision values of step n-1)
//     each cell gathers f_i^n(x) through the link rules of rules.h, collides,
//     and scatters f*_i(x) to every destination link of the next state, which
//     is then stored naturally again.
// Both steps move 19 floats in and 19 floats out per fluid cell.  In the odd
// step the outflow column reads values that its upstream neighbour in the
// same x-row overwrites, so each workgroup finishes all gathers before any
// scatter (one barrier); a workgroup is a run of consecutive cells of one
// instance, which never separates cells nx-2 and nx-1 of a row when nx is even.
//
// Collisions (Sec. 2.2): model 0, Eq. (deterministicLBE) with an unprojected
// non-equilibrium part, f* = f - omega (f - f_eq), second-order equilibrium;
// model 1, the same with the Smagorinsky omega = 1 / tau_eff,
// tau_eff = (tau0 + sqrt(tau0^2 + 18 sqrt(2) Cs^2 Q / rho)) / 2,
// Q = |Pi_neq| (Eqs. tauEff, turbVisc with |S| from the local
// non-equilibrium stress); model 2, Eq. (deterministicLBE) as printed, the
// regularised collision with equilibrium and non-equilibrium part expanded to
// third order in the Hermite polynomials orthogonal on D3Q19, with the
// Smagorinsky tau_eff.
//
// The step kernels of the three collision models are instantiated in
// separate translation units (steps.hip, built once per model), the adjoint
// kernels in adjoint.hip, everything else in kernels.hip.
#pragma once

#include <utility>

#include "kernels.h"

namespace lbmsc {

namespace {

constexpr float KAPPA_INV = 1.0f / 0.41f;

// Pointers taken from the instance table are generic; casting them to the
// global address space lets the compiler emit global (not flat) memory
// instructions with a scalar base and 32-bit lane offsets.
#define GLOBAL_AS __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ GLOBAL_AS T *gp(T *p)
{
    return (GLOBAL_AS T *)p;
}
template <class T>
__device__ __forceinline__ const GLOBAL_AS T *gp(const T *p)
{
    return (const GLOBAL_AS T *)p;
}

// Element idx of a uniform base through a 32-bit byte offset, so that the
// access uses a scalar base address plus one 32-bit lane offset.  NT marks
// streaming (non-temporal) accesses.
template <bool NT = false, class T>
__device__ __forceinline__ T ldg(const GLOBAL_AS T *base, uint32_t idx)
{
    const GLOBAL_AS T *p = (const GLOBAL_AS T *)((const GLOBAL_AS char *)base + idx * (uint32_t)sizeof(T));
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT = false, class T>
__device__ __forceinline__ void stg(GLOBAL_AS T *base, uint32_t idx, T v)
{
    GLOBAL_AS T *p = (GLOBAL_AS T *)((GLOBAL_AS char *)base + idx * (uint32_t)sizeof(T));
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

__device__ __forceinline__ uint32_t umin_u32(uint32_t a, uint32_t b) { return a < b ? a : b; }

// Workgroups are dispatched round-robin over the 8 XCDs; tile_order() (see
// rules.h) chooses which tile each block index takes.
__device__ __forceinline__ int xcd_tile() { return tile_order((int)blockIdx.x, (int)gridDim.x, 1); }
__device__ __forceinline__ int tile_of(int mode) { return tile_order((int)blockIdx.x, (int)gridDim.x, mode); }

__device__ __forceinline__ float ramp_factor(const Geo &G, int64_t n)
{
    if (G.ramp <= 0 || n >= G.ramp) return 1.0f;
    return 0.5f * (1.0f - cosf(3.14159265358979323846f * (float)n / (float)G.ramp));
}

// Height profile of the inflow speed at cell z (h = z + 1/2 above the
// half-way ground): uniform U; log-law (u* / 0.41) ln(h / z0); measured series
// ln((h + z0) / z0), its normalisation and speed being in InflowT.
__device__ __forceinline__ float inflow_speed(const Geo &G, int z)
{
    if (G.inflow == 0) return G.speed;
    if (G.inflow == 1) return G.speed * KAPPA_INV * logf(((float)z + 0.5f) / G.z0);
    return logf(((float)z + 0.5f + G.z0) / G.z0);
}

// The time-dependent part of u_in at step n: u_in(z, n) = scale * profile(z) *
// (cphi, sphi, 0).  base is scale without the speed parameter (ramp only for
// the uniform and log-law kinds; ramp * U_H(n) / ln((H + z0)/z0) for the series).
struct InflowT {
    float scale, base, cphi, sphi;
};

// Reference speed and direction of the hourly series at step n: hour h starts
// at step ramp + h * hour_steps and moves from hour h-1's values over its first
// blend_steps steps with weight (1 - cos(pi t / blend_steps)) / 2, the
// direction along the shorter arc; hour 0 before and during the ramp, the
// last hour held after the series.
__device__ __forceinline__ void series_at(const Geo &G, int64_t n, float &U, float &D)
{
    int32_t t = (int32_t)(n > (int64_t)G.ramp ? n - G.ramp : 0);
    int32_t h = t / G.hour_steps;
    int32_t tp = t - h * G.hour_steps;
    if (h >= G.series_len) {
        h = G.series_len - 1;
        tp = G.hour_steps;
    }
    U = G.series[2 * h];
    D = G.series[2 * h + 1];
    if (h > 0 && tp < G.blend_steps) {
        const float s = 0.5f * (1.0f - cosf(3.14159265358979323846f * (float)tp / (float)G.blend_steps));
        const float U0 = G.series[2 * h - 2], D0 = G.series[2 * h - 1];
        const float dD = remainderf(D - D0, 6.28318530717958647692f);
        U = U0 + s * (U - U0);
        D = D0 + s * dD;
    }
}

__device__ __forceinline__ InflowT inflow_at(const Geo &G, int64_t n)
{
    const float r = ramp_factor(G, n);
    if (G.inflow != 2) return InflowT{r, r, G.cphi, G.sphi};
    float U, D;
    series_at(G, n, U, D);
    const float base = r * U * G.inv_log_h;
    const float phi = D + G.phi;
    return InflowT{base * G.speed, base, cosf(phi), sinf(phi)};
}

// 6 w_i c_i . u_in, the moving-wall momentum of link i.
__device__ __forceinline__ float inlet_term(int i, float U, const InflowT &T)
{
    return 6.0f * wgt(i) * U * T.scale * ((float)cx(i) * T.cphi + (float)cy(i) * T.sphi);
}

// The cell has links with the moving-wall momentum: on the inflow face, or
// next to the mantle region.
__device__ __forceinline__ bool inflow_lane(const Geo &G, uint8_t fl)
{
    return (fl & FL_MANTLE) || ((fl & FL_XLO) && G.box.face[0] == FACE_INLET);
}

__device__ __forceinline__ int probe_index(const Geo &G, int32_t c)
{
    int lo = 0, hi = G.n_probes - 1;
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        int v = gp(G.probes)[mid];
        if (v == c) return mid;
        if (v < c) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

__device__ __forceinline__ void coords(const Geo &G, uint32_t c, int &x, int &y, int &z)
{
    const uint32_t zz = fdiv(c, G.dxy);
    const uint32_t rem = c - zz * (uint32_t)(G.box.nx * G.box.ny);
    const uint32_t yy = fdiv(rem, G.dx);
    x = (int)(rem - yy * (uint32_t)G.box.nx);
    y = (int)yy;
    z = (int)zz;
}

__device__ __forceinline__ uint32_t cell_of(const Geo &G, const Link &l)
{
    return ((uint32_t)l.z * (uint32_t)G.box.ny + (uint32_t)l.y) * (uint32_t)G.box.nx + (uint32_t)l.x;
}

__device__ __forceinline__ int32_t off_of(const Geo &G, int i)
{
    return cx(i) + cy(i) * G.offy + cz(i) * G.offz;
}

__device__ __forceinline__ Shape shape_of(const Geo &G)
{
    Shape S;
    S.nx = G.box.nx;
    S.ny = G.box.ny;
    S.nz = G.box.nz;
    S.offy = G.offy;
    S.offz = G.offz;
#pragma unroll
    for (int k = 0; k < 6; ++k) S.face[k] = G.box.face[k];
    return S;
}

// Boundary-aware gather of all 19 populations f^n(x) from the swapped
// post-collision values of step n-1, one compile-time direction at a time.
// CLAMP: the neighbour index is clamped into the instance (speculative
// gathers of lanes whose cell kind is not known yet).
template <bool NT = false, bool CLAMP = false, int... Is>
__device__ __forceinline__ void gather_all(const Geo &G, const Shape &S, const Preds &p, uint32_t sm, uint32_t c,
                                           float U, const InflowT &T, float g[Q], std::integer_sequence<int, Is...>)
{
    const GLOBAL_AS float *__restrict__ f = gp(G.f);
    const uint32_t qs = (uint32_t)G.qs;
    const uint32_t last = (uint32_t)G.ncells - 1u;
    (
        [&] {
            const RelLink l = gather_rel<Is>(S, p, sm);
            uint32_t n = (uint32_t)((int32_t)c + l.delta);
            if (CLAMP) n = umin_u32(n, last);
            const float v = ldg<NT>(f, (uint32_t)l.slot * qs + n);
            g[Is] = l.inlet ? v + inlet_term(Is, U, T) : v;
        }(),
        ...);
}

// Boundary-aware scatter of the post-collision values to every destination
// link of the next (naturally stored) state.
template <bool NT = false, int... Ks>
__device__ __forceinline__ void scatter_all(const Geo &G, const Shape &S, const Preds &p, uint32_t sm, uint32_t c,
                                            float U, const InflowT &T, const float g[Q], std::integer_sequence<int, Ks...>)
{
    GLOBAL_AS float *__restrict__ f = gp(G.f);
    const uint32_t qs = (uint32_t)G.qs;
    (
        [&] {
            RelLink a, e;
            scatter_rel<Ks>(S, p, sm, a, e);
            if (a.valid) {
                const float v = a.inlet ? g[Ks] + inlet_term(opp(Ks), U, T) : g[Ks];
                stg<NT>(f, (uint32_t)a.slot * qs + (uint32_t)((int32_t)c + a.delta), v);
            }
            if (e.valid) stg<NT>(f, (uint32_t)e.slot * qs + (uint32_t)((int32_t)c + e.delta), g[Ks]);
        }(),
        ...);
}

// Wavefronts of rule class 1 hold boundary lanes only in the first and last
// x column, with the -x face an inlet or a wall and the +x face an outlet or
// a wall (periodic x faces, y/z faces and solid neighbours are classes 2 and
// 3).  Their links are the plain stencil except for the five directions that
// cross an x face, which these forms patch per lane:
//   gather, c_x = +1 at x = 0:      own slot I (bounce-back), plus the
//                                   moving-wall momentum at an inlet;
//   gather, c_x = -1 at x = nx-1:   outlet: slot opp(I) of (nx-1, y - c_y,
//                                   z - c_z); wall: own slot I;
//   scatter, c_x = -1 at x = 0:     own slot opp(K) (plus the moving-wall
//                                   momentum at an inlet);
//   scatter, c_x = +1 at x = nx-1:  outlet: no destination; wall: own slot
//                                   opp(K);
//   scatter, c_x = -1 at x = nx-1:  outlet: also slot K of (nx-1, y + c_y,
//                                   z + c_z), the zero-gradient link of that
//                                   cell.
// Indices are clamped into the instance (lanes of solid cells gather before
// their kind is known; their values are dropped).
template <bool NT = false, int... Is>
__device__ __forceinline__ void gather_x(const Geo &G, const Shape &S, bool xlo, bool xhi, uint32_t c, float U,
                                         const InflowT &T, float g[Q], std::integer_sequence<int, Is...>)
{
    const GLOBAL_AS float *__restrict__ f = gp(G.f);
    const uint32_t qs = (uint32_t)G.qs;
    const uint32_t last = (uint32_t)G.ncells - 1u;
    const bool inl = S.face[0] == FACE_INLET, out = S.face[1] == FACE_OUTLET;
    (
        [&] {
            constexpr int I = Is;
            const uint32_t pn = umin_u32((uint32_t)((int32_t)c - off_of(G, I)), last);
            if constexpr (cx(I) == 1) {
                const float v = ldg<NT>(f, xlo ? (uint32_t)I * qs + c : (uint32_t)opp(I) * qs + pn);
                g[I] = (xlo && inl) ? v + inlet_term(I, U, T) : v;
            } else if constexpr (cx(I) == -1) {
                const uint32_t po = umin_u32(pn - 1u, last);
                g[I] = ldg<NT>(f, !xhi ? (uint32_t)opp(I) * qs + pn
                                       : (out ? (uint32_t)opp(I) * qs + po : (uint32_t)I * qs + c));
            } else {
                g[I] = ldg<NT>(f, (uint32_t)opp(I) * qs + pn);
            }
        }(),
        ...);
}

template <bool NT = false, int... Ks>
__device__ __forceinline__ void scatter_x(const Geo &G, const Shape &S, bool xlo, bool xhi, uint32_t c, float U,
                                          const InflowT &T, const float g[Q], std::integer_sequence<int, Ks...>)
{
    GLOBAL_AS float *__restrict__ f = gp(G.f);
    const uint32_t qs = (uint32_t)G.qs;
    const bool inl = S.face[0] == FACE_INLET, out = S.face[1] == FACE_OUTLET;
    (
        [&] {
            constexpr int K = Ks;
            const uint32_t pn = (uint32_t)((int32_t)c + off_of(G, K));
            if constexpr (cx(K) == -1) {
                const float v = (xlo && inl) ? g[K] + inlet_term(opp(K), U, T) : g[K];
                stg<NT>(f, xlo ? (uint32_t)opp(K) * qs + c : (uint32_t)K * qs + pn, v);
                if (xhi && out)
                    stg<NT>(f, (uint32_t)K * qs + (uint32_t)((int32_t)c + cy(K) * G.offy + cz(K) * G.offz), g[K]);
            } else if constexpr (cx(K) == 1) {
                if (!(xhi && out)) stg<NT>(f, xhi ? (uint32_t)opp(K) * qs + c : (uint32_t)K * qs + pn, g[K]);
            } else {
                stg<NT>(f, (uint32_t)K * qs + pn, g[K]);
            }
        }(),
        ...);
}

using Dirs = std::make_integer_sequence<int, Q>;

// Populations f^n(x) of a fluid cell in the current storage state.
// parity 0: natural slots; parity 1: gathered from the swapped
// post-collision values of step n-1 (inlet momentum uses r(n-1)).
template <int PARITY>
__device__ __forceinline__ void load_state(const Geo &G, uint32_t c, uint8_t fl, int x, int y, int z,
                                           int64_t n, float g[Q])
{
    const GLOBAL_AS float *__restrict__ f = gp(G.f);
    const uint32_t qs = (uint32_t)G.qs;
    if (PARITY == 0) {
#pragma unroll
        for (int i = 0; i < Q; ++i) g[i] = ldg(f + (size_t)i * qs, c);
    } else if (!(fl & FL_NEAR)) {
#pragma unroll
        for (int i = 0; i < Q; ++i) g[i] = ldg(f + (size_t)opp(i) * qs - off_of(G, i), c);
    } else {
        const Shape S = shape_of(G);
        const Preds p = preds_of(S, x, y, z, fl);
        const uint32_t sm = gp(G.smask)[c];
        const float U = inflow_lane(G, fl) ? inflow_speed(G, z) : 0.0f;
        gather_all(G, S, p, sm, c, U, inflow_at(G, n - 1), g, Dirs{});
    }
}

struct Macro {
    float drho, rho, ux, uy, uz;
};

// Opposite directions come in pairs (2k+1, 2k+2), k = 0..8: their sums carry
// the even moments (density, stress), their differences the odd ones
// (momentum), which halves the additions of the moment sums.
struct PairSums {
    float s[9], d[9];
};

__device__ __forceinline__ PairSums pair_sums(const float g[Q])
{
    PairSums p;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        p.s[k] = g[2 * k + 1] + g[2 * k + 2];
        p.d[k] = g[2 * k + 1] - g[2 * k + 2];
    }
    return p;
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

__device__ __forceinline__ Macro macro_of(const float g[Q], const PairSums &p)
{
    Macro m;
    float d = g[0], jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int i = 2 * k + 1;
        d += p.s[k];
        if (cx(i)) jx += cx(i) * p.d[k];
        if (cy(i)) jy += cy(i) * p.d[k];
        if (cz(i)) jz += cz(i) * p.d[k];
    }
    m.drho = d;
    m.rho = 1.0f + d;
    const float inv = fast_rcp(m.rho);
    m.ux = jx * inv;
    m.uy = jy * inv;
    m.uz = jz * inv;
    return m;
}

__device__ __forceinline__ Macro macro_of(const float g[Q]) { return macro_of(g, pair_sums(g)); }

// Non-equilibrium stress Pi = sum c c (f - f_eq) from the shifted populations:
// sum c c g - (drho/3) I - rho u u.  Order: xx, yy, zz, xy, xz, yz.
__device__ __forceinline__ void neq_stress(const PairSums &p, const Macro &m, float P[6])
{
    float xx = 0.f, yy = 0.f, zz = 0.f, xy = 0.f, xz = 0.f, yz = 0.f;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int i = 2 * k + 1;
        if (cx(i)) xx += p.s[k];
        if (cy(i)) yy += p.s[k];
        if (cz(i)) zz += p.s[k];
        if (cx(i) && cy(i)) xy += cx(i) * cy(i) * p.s[k];
        if (cx(i) && cz(i)) xz += cx(i) * cz(i) * p.s[k];
        if (cy(i) && cz(i)) yz += cy(i) * cz(i) * p.s[k];
    }
    const float d3 = m.drho * (1.0f / 3.0f);
    P[0] = xx - d3 - m.rho * m.ux * m.ux;
    P[1] = yy - d3 - m.rho * m.uy * m.uy;
    P[2] = zz - d3 - m.rho * m.uz * m.uz;
    P[3] = xy - m.rho * m.ux * m.uy;
    P[4] = xz - m.rho * m.ux * m.uz;
    P[5] = yz - m.rho * m.uy * m.uz;
}

__device__ __forceinline__ void neq_stress(const float g[Q], const Macro &m, float P[6])
{
    neq_stress(pair_sums(g), m, P);
}

__device__ __forceinline__ float stress_norm(const float P[6])
{
    return fast_sqrt(P[0] * P[0] + P[1] * P[1] + P[2] * P[2] +
                     2.0f * (P[3] * P[3] + P[4] * P[4] + P[5] * P[5]));
}

template <int MODEL>
__device__ __forceinline__ float tau_of(const Geo &G, const PairSums &p, const Macro &m)
{
    if (MODEL == 0) return G.tau0;
    float P[6];
    neq_stress(p, m, P);
    const float q = stress_norm(P);
    return 0.5f * (G.tau0 + fast_sqrt(G.tau0 * G.tau0 + G.kcs * q * fast_rcp(m.rho)));
}

// shifted equilibrium f_eq - w
__device__ __forceinline__ float geq(int i, const Macro &m, float usq15)
{
    const float cu = cx(i) * m.ux + cy(i) * m.uy + cz(i) * m.uz;
    return wgt(i) * (m.drho + m.rho * (3.0f * cu + 4.5f * cu * cu - usq15));
}

// Third-order Hermite polynomials orthogonal on D3Q19 at velocity i, in the
// order H_xxy + H_yzz, H_xxy - H_yzz, H_xzz + H_xyy, H_xzz - H_xyy,
// H_yyz + H_xxz, H_yyz - H_xxz (H_aab = c_b (c_a^2 - 1/3)), and their inverse
// norms on the velocity set: 1 / (2 cs^6) = 13.5 for the sums,
// 1 / (6 cs^6) = 4.5 for the differences.  All fold to constants per
// direction.
__host__ __device__ constexpr float herm3(int k, int i)
{
    const float x = (float)cx(i), y = (float)cy(i), z = (float)cz(i), s = 1.0f / 3.0f;
    const float hxxy = y * (x * x - s), hyzz = y * (z * z - s);
    const float hxzz = x * (z * z - s), hxyy = x * (y * y - s);
    const float hyyz = z * (y * y - s), hxxz = z * (x * x - s);
    return k == 0 ? hxxy + hyzz : k == 1 ? hxxy - hyzz : k == 2 ? hxzz + hxyy
         : k == 3 ? hxzz - hxyy : k == 4 ? hyyz + hxxz : hyyz - hxxz;
}
__host__ __device__ constexpr float herm3_inv_norm(int k) { return (k & 1) ? 4.5f : 13.5f; }

// What the regularised adjoint needs of the pre-collision state: rho, u,
// the non-equilibrium stress P and the third-order Hermite moments
// t3_j = sum_i P_j(c_i) (f_i - w_i) (16 values: record kind 3 stores them).
struct Rr3State {
    float rho, ux, uy, uz, P[6], t3[6];
};

__device__ __forceinline__ Rr3State rr3_state(const float g[Q])
{
    Rr3State r;
    const PairSums ps = pair_sums(g);
    const Macro m = macro_of(g, ps);
    r.rho = m.rho;
    r.ux = m.ux;
    r.uy = m.uy;
    r.uz = m.uz;
    neq_stress(ps, m, r.P);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        float t = 0.0f;
#pragma unroll
        for (int k = 0; k < 9; ++k)
            if (herm3(j, 2 * k + 1) != 0.0f) t += herm3(j, 2 * k + 1) * ps.d[k];
        r.t3[j] = t;
    }
    return r;
}


// Regularised collision (Eq. deterministicLBE as printed), with the
// Smagorinsky tau_eff:
//   f* = f_eq3 + (1 - 1/tau) [w (H2 : Pi / (2 cs^4) + sum_k P_k a1_k / N_k)],
// f_eq3 the equilibrium to third order and a1_k = sum_i P_k(c_i)(f_i - f_eq3_i)
// for the six third-order polynomials P_k above.  The third-order terms are
// odd in c, so per opposite pair they enter with opposite signs and only the
// pair's antisymmetric part of f - f_eq3 projects onto them; they have no
// second moment, so Pi and tau_eff are those of the second-order equilibrium.
__device__ __forceinline__ void collide_rr3(const Geo &G, float g[Q], const Macro &m, const PairSums &p)
{
    float P[6];
    neq_stress(p, m, P);
    const float q = stress_norm(P);
    const float tau = 0.5f * (G.tau0 + fast_sqrt(G.tau0 * G.tau0 + G.kcs * q * fast_rcp(m.rho)));
    const float keep = 1.0f - fast_rcp(tau);
    const float ux = m.ux, uy = m.uy, uz = m.uz;
    const float usq15 = 1.5f * (ux * ux + uy * uy + uz * uz);
    // Maxwellian coefficients of the six third-order polynomials (per unit density)
    const float A[6] = {ux * ux * uy + uy * uz * uz, ux * ux * uy - uy * uz * uz,
                        ux * uz * uz + ux * uy * uy, ux * uz * uz - ux * uy * uy,
                        uy * uy * uz + ux * ux * uz, uy * uy * uz - ux * ux * uz};
    const float trP = P[0] + P[1] + P[2];
    float sym[9], asym[9], t3[9], a1[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int i = 2 * k + 1;
        const float cu = cx(i) * ux + cy(i) * uy + cz(i) * uz;
        sym[k] = wgt(i) * (m.drho + m.rho * (4.5f * cu * cu - usq15));
        asym[k] = 3.0f * wgt(i) * m.rho * cu;
        float t = 0.0f;
#pragma unroll
        for (int j = 0; j < 6; ++j)
            if (herm3(j, i) != 0.0f) t += herm3(j, i) * herm3_inv_norm(j) * A[j];
        t3[k] = wgt(i) * m.rho * t;
        // (f - f_eq3)_i - (f - f_eq3)_opp(i)
        const float D = p.d[k] - 2.0f * (asym[k] + t3[k]);
#pragma unroll
        for (int j = 0; j < 6; ++j)
            if (herm3(j, i) != 0.0f) a1[j] += herm3(j, i) * D;
    }
    g[0] = wgt(0) * (m.drho - m.rho * usq15) + keep * wgt(0) * (-1.5f * trP);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int i = 2 * k + 1;
        const float X = (float)cx(i), Y = (float)cy(i), Z = (float)cz(i);
        const float cpc = X * X * P[0] + Y * Y * P[1] + Z * Z * P[2] +
                          2.0f * (X * Y * P[3] + X * Z * P[4] + Y * Z * P[5]);
        const float r2 = wgt(i) * (4.5f * cpc - 1.5f * trP);
        float r3 = 0.0f;
#pragma unroll
        for (int j = 0; j < 6; ++j)
            if (herm3(j, i) != 0.0f) r3 += herm3(j, i) * herm3_inv_norm(j) * a1[j];
        r3 *= wgt(i);
        g[i] = sym[k] + asym[k] + t3[k] + keep * (r2 + r3);
        g[i + 1] = sym[k] - asym[k] - t3[k] + keep * (r2 - r3);
    }
}

// f* = f - omega (f - f_eq), the equilibrium of each opposite pair split into
// its symmetric part w (drho + rho (4.5 (c.u)^2 - 1.5 u.u)) and its
// antisymmetric part 3 w rho c.u.
template <int MODEL>
__device__ __forceinline__ void collide(const Geo &G, float g[Q], const Macro &m, const PairSums &p)
{
    if constexpr (MODEL == 2) {
        collide_rr3(G, g, m, p);
        return;
    }
    const float om = fast_rcp(tau_of<MODEL>(G, p, m));
    const float usq15 = 1.5f * (m.ux * m.ux + m.uy * m.uy + m.uz * m.uz);
    g[0] = g[0] - om * (g[0] - wgt(0) * (m.drho - m.rho * usq15));
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int i = 2 * k + 1;
        const float cu = cx(i) * m.ux + cy(i) * m.uy + cz(i) * m.uz;
        const float sym = wgt(i) * (m.drho + m.rho * (4.5f * cu * cu - usq15));
        const float asym = 3.0f * wgt(i) * m.rho * cu;
        g[i] = g[i] - om * (g[i] - (sym + asym));
        g[i + 1] = g[i + 1] - om * (g[i + 1] - (sym - asym));
    }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 partial sums (ux, uy, uz, |u|) of one cell: one 16-byte load and store
__device__ __forceinline__ void accumulate_qoi(const Geo &G, uint32_t c, uint8_t fl, const Macro &m)
{
    if (G.qpart) {
        GLOBAL_AS f32x4 *p = (GLOBAL_AS f32x4 *)gp(G.qpart) + c;
        f32x4 v = *p;
        v.x += m.ux;
        v.y += m.uy;
        v.z += m.uz;
        v.w += sqrtf(m.ux * m.ux + m.uy * m.uy + m.uz * m.uz);
        *p = v;
    }
    if ((fl & FL_PROBE) && G.psum) {
        const int p = probe_index(G, (int32_t)c);
        if (p >= 0) gp(G.psum)[p] += (double)m.ux;
    }
}

// One time step of every instance.  A workgroup of BS threads owns a tile of
// BS * CPT consecutive cells of one instance; thread t handles cells
// t, t + BS, ... so every load and store instruction stays coalesced.
template <int BS, int CPT, bool NT, int MODEL, int PARITY>
__global__ __launch_bounds__(BS) void k_step(const Geo *__restrict__ geo, const int32_t *__restrict__ tile_inst,
                                             int32_t n_tiles, StepArgs a, int32_t *__restrict__ health)
{
    const int tile = a.tile_base + tile_of(a.xcd_remap);
    if (tile >= n_tiles) return;
    const int ii = __builtin_amdgcn_readfirstlane(tile_inst[tile]);
    const Geo &G = geo[ii];
    GLOBAL_AS float *__restrict__ f = gp(G.f);
    const uint32_t qs = (uint32_t)G.qs;
    const int32_t base = (tile - G.tile0) * (BS * CPT) + (int32_t)threadIdx.x;
    // per-tile words: all-solid lines (skipped like cells past the end: they
    // carry no state and no neighbour's rule touches them) and the rule class
    // of each wavefront (launch_tile_info)
    const uint64_t dead = a.tinfo ? a.tinfo[2 * (size_t)tile] : 0ull;
    const uint64_t wcls = a.tinfo ? a.tinfo[2 * (size_t)tile + 1] : ~0ull;

    uint32_t c[CPT];
    uint8_t fl[CPT];
    int cls[CPT];
    bool act[CPT], fluid[CPT], flow_wave[CPT];
    Preds pr[CPT];
    uint32_t sm[CPT];
    float U[CPT];
    float g[CPT][Q];
    Shape S;
    if (PARITY == 1) S = shape_of(G);
    const uint32_t last = (uint32_t)G.ncells - 1u;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int32_t lc = base + j * BS;
        const bool active = lc < G.ncells && !((dead >> ((j * BS + (int)threadIdx.x) >> 5)) & 1ull);
        act[j] = active;
        c[j] = active ? (uint32_t)lc : 0u;
        // Even steps touch only the cell's own 19 slots.  The slots of a solid
        // cell are never read or written by any other cell (every link into a
        // solid cell resolves to a rule on the fluid side's own slots), so the
        // even step swaps them like a fluid cell's, without collision: the
        // loads do not wait for the flag byte and every wavefront writes whole
        // cache lines instead of lines with holes at solid cells.
        if (PARITY == 0 && active) {
#pragma unroll
            for (int i = 0; i < Q; ++i) g[j][i] = ldg<NT>(f + (size_t)i * qs, c[j]);
        }
        // Odd steps, per wavefront (class from the tile words): 0 the plain
        // stencil; 1 the x rules (boundary cells only in the x = 0 / nx-1
        // columns); 2 the x and solid-link rules (solid neighbours but no y/z
        // face, wrap or sky link; y/z terms dropped at compile time); 3 the
        // full rules.  Classes 0 and 1 take their addresses from the cell
        // index alone, so their gathers are issued before the flag byte
        // arrives, with the neighbour index clamped into the instance: lanes
        // of solid cells stay in bounds and their values are dropped.  The
        // inflow is evaluated only in wavefronts with a moving-wall lane.
        cls[j] = PARITY == 1 ? (int)((wcls >> (2 * ((j * BS + (int)threadIdx.x) >> 6))) & 3ull) : 0;
        pr[j] = Preds{false, false, false, false, false, false, false};
        sm[j] = 0;
        U[j] = 0.0f;
        flow_wave[j] = false;
        if (PARITY == 1 && cls[j] == 0) {
            if (active) {
#pragma unroll
                for (int i = 0; i < Q; ++i)
                    g[j][i] = ldg<NT>(f + (size_t)opp(i) * qs, umin_u32((uint32_t)((int32_t)c[j] - off_of(G, i)), last));
            }
        } else if (PARITY == 1 && cls[j] == 1) {
            int x, y, z;
            coords(G, c[j], x, y, z);
            pr[j].xlo = x == 0;
            pr[j].xhi = x == S.nx - 1;
            const bool inl = active && pr[j].xlo && S.face[0] == FACE_INLET;
            flow_wave[j] = __any(inl);
            if (inl) U[j] = inflow_speed(G, z);
            if (active) {
                const InflowT T = flow_wave[j] ? inflow_at(G, a.step - 1) : InflowT{0.f, 0.f, 0.f, 0.f};
                gather_x<NT>(G, S, pr[j].xlo, pr[j].xhi, c[j], U[j], T, g[j], Dirs{});
            }
        }
        fl[j] = active ? gp(G.flags)[c[j]] : (uint8_t)FL_SOLID;
        // classes 2 and 3 need the solid-link mask as well: issued with the
        // flag byte (the mask of a solid cell is zero)
        const uint32_t smv = (PARITY == 1 && cls[j] >= 2 && active) ? gp(G.smask)[c[j]] : 0u;
        fluid[j] = !(fl[j] & FL_SOLID);
        if (PARITY == 1 && cls[j] >= 2) {
            const bool flow = fluid[j] && inflow_lane(G, fl[j]);
            flow_wave[j] = __any(flow);
            if (fluid[j]) {
                sm[j] = smv;
                if (cls[j] == 3) {
                    int x, y, z;
                    coords(G, c[j], x, y, z);
                    pr[j] = preds_of(S, x, y, z, fl[j]);
                    if (flow) U[j] = inflow_speed(G, z);
                } else {
                    pr[j] = preds_xs(fl[j]);
                    if (flow) U[j] = inflow_speed(G, (int)fdiv(c[j], G.dxy));
                }
            }
        }
    }
    // classes 2 and 3: gathers after the flag byte and solid-link mask
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        if (PARITY == 0 || cls[j] < 2 || !fluid[j]) continue;
        const InflowT T = flow_wave[j] ? inflow_at(G, a.step - 1) : InflowT{0.f, 0.f, 0.f, 0.f};
        if (cls[j] == 3) {
            gather_all<NT>(G, S, pr[j], sm[j], c[j], U[j], T, g[j], Dirs{});
        } else {
            const Preds ps{pr[j].xlo, pr[j].xhi, false, false, false, false, pr[j].mantle};
            gather_all<NT>(G, S, ps, sm[j], c[j], U[j], T, g[j], Dirs{});
        }
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        if (!fluid[j]) {
            // the partial sums of solid cells stay zero; writing them keeps
            // the wavefront's partial-sum stores on whole lines
            if (a.accumulate && act[j] && G.qpart) ((GLOBAL_AS f32x4 *)gp(G.qpart))[c[j]] = f32x4{0.f, 0.f, 0.f, 0.f};
            continue;
        }
        const PairSums ps = pair_sums(g[j]);
        const Macro m = macro_of(g[j], ps);
        if (!(m.rho > 0.0f) || !isfinite(m.rho)) atomicOr(health + ii, 1);
        if (a.accumulate) accumulate_qoi(G, c[j], fl[j], m);
        // records are read once, in reverse order, a whole segment later:
        // streaming stores keep them from displacing the populations in the
        // caches (the adjoint reads them with streaming loads)
        if (a.record == 1) {
            GLOBAL_AS f32x4 *r = (GLOBAL_AS f32x4 *)gp(a.rec[ii]) + ((size_t)a.rec_slot * (size_t)G.ncells + c[j]);
            __builtin_nontemporal_store(f32x4{m.rho, m.ux, m.uy, m.uz}, r);
        } else if (a.record == 2) {
            GLOBAL_AS float *r = gp(a.rec[ii]) + (size_t)a.rec_slot * (size_t)Q * G.qs;
#pragma unroll
            for (int i = 0; i < Q; ++i) stg<true>(r + (size_t)i * qs, c[j], g[j][i]);
        } else if (MODEL == 2 && a.record == 3) {
            // record kind 3: the regularised adjoint's 16 state values
            const Rr3State st = rr3_state(g[j]);
            const float v[RR3_REC] = {st.rho,   st.ux,   st.uy,   st.uz,   st.P[0],  st.P[1],
                                      st.P[2],  st.P[3], st.P[4], st.P[5], st.t3[0], st.t3[1],
                                      st.t3[2], st.t3[3], st.t3[4], st.t3[5]};
            GLOBAL_AS float *r = gp(a.rec[ii]) + (size_t)a.rec_slot * (size_t)RR3_REC * G.qs;
#pragma unroll
            for (int i = 0; i < RR3_REC; ++i) stg<true>(r + (size_t)i * qs, c[j], v[i]);
        }
        collide<MODEL>(G, g[j], m, ps);
    }
    if (PARITY == 1) __syncthreads();
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        if (PARITY == 0) {
            if (!act[j]) continue;
#pragma unroll
            for (int i = 0; i < Q; ++i) stg<NT>(f + (size_t)opp(i) * qs, c[j], g[j][i]);
            continue;
        }
        if (!fluid[j]) {
            // no fluid cell reads or writes a slot of a solid cell (links into
            // solids resolve to the fluid side's own slots), so each solid cell
            // of a live line writes zero into its own 19 slots: with the fluid
            // cells' scatter, every line of every plane is written whole
            if (act[j]) {
#pragma unroll
                for (int k = 0; k < Q; ++k) stg<NT>(f + (size_t)k * qs, c[j], 0.0f);
            }
            continue;
        }
        if (cls[j] == 0) {
#pragma unroll
            for (int i = 0; i < Q; ++i) stg<NT>(f + (size_t)i * qs + off_of(G, i), c[j], g[j][i]);
            continue;
        }
        const InflowT T = flow_wave[j] ? inflow_at(G, a.step) : InflowT{0.f, 0.f, 0.f, 0.f};
        if (cls[j] == 3) {
            scatter_all<NT>(G, S, pr[j], sm[j], c[j], U[j], T, g[j], Dirs{});
        } else if (cls[j] == 2) {
            const Preds ps{pr[j].xlo, pr[j].xhi, false, false, false, false, pr[j].mantle};
            scatter_all<NT>(G, S, ps, sm[j], c[j], U[j], T, g[j], Dirs{});
        } else {
            scatter_x<NT>(G, S, pr[j].xlo, pr[j].xhi, c[j], U[j], T, g[j], Dirs{});
        }
    }
}

// ------------------------------------------------------------------ adjoint

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Gradient of the moving-wall momentum of a cell's inlet links: with link
// weights s_q (the adjoint value of each link times 6 w_q), the sum over the
// links of s_q c_q . d u_in / d theta_t at height z and step n (T =
// inflow_at(n), ramp included).  The derivative is linear in (c_qx, c_qy),
// so only Sx = sum s_q c_qx and Sy = sum s_q c_qy enter: the speed parameter
// and z0 through c . dir, the direction through U c . d dir / d phi.
__device__ __forceinline__ void inflow_grad(const Geo &G, int z, const InflowT &T, double sx, double sy, double &g0,
                                            double &g1, double &g2)
{
    const double cd = sx * (double)T.cphi + sy * (double)T.sphi;
    const double cdd = -sx * (double)T.sphi + sy * (double)T.cphi;
    float a0, b1, a2;
    if (G.inflow == 0) {
        a0 = T.base;
        b1 = T.base * G.speed;
        a2 = 0.0f;
    } else if (G.inflow == 1) {
        const float L = logf(((float)z + 0.5f) / G.z0);
        a0 = T.base * KAPPA_INV * L;
        b1 = T.base * G.speed * KAPPA_INV * L;
        a2 = -T.base * G.speed * KAPPA_INV / G.z0;
    } else {
        // u = base zeta1 A / B-normalised: A = ln((h + z0)/z0), 1/B in base
        const float h = (float)z + 0.5f;
        const float A = logf((h + G.z0) / G.z0);
        const float dA = 1.0f / (h + G.z0) - 1.0f / G.z0;
        a0 = T.base * A;
        b1 = T.scale * A;
        a2 = T.scale * (dA - A * G.dlog_h * G.inv_log_h);
    }
    g0 += (double)a0 * cd;
    g1 += (double)b1 * cdd;
    g2 += (double)a2 * cd;
}

// Weighted moments of a field v over the velocity set, from the sums and
// differences of opposite pairs: m0 = sum w v, m1_a = sum w c_a v, the
// second-order tensor m2 = sum w c c v (xx, yy, zz, xy, xz, yz) and h3_j =
// sum w P_j(c) v for the six third-order polynomials P_j above.
struct WMoments {
    float m0, m1[3], m2[6], h3[6];
};

__device__ __forceinline__ WMoments weighted_moments(const float v[Q])
{
    WMoments M;
    M.m0 = wgt(0) * v[0];
#pragma unroll
    for (int a = 0; a < 3; ++a) M.m1[a] = 0.0f;
#pragma unroll
    for (int a = 0; a < 6; ++a) M.m2[a] = M.h3[a] = 0.0f;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int i = 2 * k + 1;
        const float ws = wgt(i) * (v[i] + v[i + 1]);
        const float wd = wgt(i) * (v[i] - v[i + 1]);
        M.m0 += ws;
        if (cx(i)) { M.m1[0] += cx(i) * wd; M.m2[0] += ws; }
        if (cy(i)) { M.m1[1] += cy(i) * wd; M.m2[1] += ws; }
        if (cz(i)) { M.m1[2] += cz(i) * wd; M.m2[2] += ws; }
        if (cx(i) && cy(i)) M.m2[3] += cx(i) * cy(i) * ws;
        if (cx(i) && cz(i)) M.m2[4] += cx(i) * cz(i) * ws;
        if (cy(i) && cz(i)) M.m2[5] += cy(i) * cz(i) * ws;
#pragma unroll
        for (int j = 0; j < 6; ++j)
            if (herm3(j, i) != 0.0f) M.h3[j] += herm3(j, i) * wd;
    }
    return M;
}

// out_k = scale base_k + alpha + beta . c_k + c_k^T Gam c_k + sum_j gam_j P_j(c_k)
// for every direction k (Gam symmetric: xx, yy, zz, xy, xz, yz), evaluated
// per opposite pair as its even part plus or minus its odd part.
template <bool THIRD, bool BASE>
__device__ __forceinline__ void eval_poly(float out[Q], const float base[Q], float scale, float alpha,
                                          const float beta[3], const float Gam[6], const float gam[6])
{
    out[0] = BASE ? scale * base[0] + alpha : alpha;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int i = 2 * k + 1;
        float E = alpha, O = 0.0f;
        if (cx(i)) { E += Gam[0]; O += cx(i) * beta[0]; }
        if (cy(i)) { E += Gam[1]; O += cy(i) * beta[1]; }
        if (cz(i)) { E += Gam[2]; O += cz(i) * beta[2]; }
        if (cx(i) && cy(i)) E += (float)(2 * cx(i) * cy(i)) * Gam[3];
        if (cx(i) && cz(i)) E += (float)(2 * cx(i) * cz(i)) * Gam[4];
        if (cy(i) && cz(i)) E += (float)(2 * cy(i) * cz(i)) * Gam[5];
        if constexpr (THIRD) {
#pragma unroll
            for (int j = 0; j < 6; ++j)
                if (herm3(j, i) != 0.0f) O += herm3(j, i) * gam[j];
        }
        out[i] = BASE ? scale * base[i] + (E + O) : E + O;
        out[i + 1] = BASE ? scale * base[i + 1] + (E - O) : E - O;
    }
}

// lambda = J^T mu of the regularised collision f* = f_eq3 + (1 - om) R f1,
// f1 = f - f_eq3, with R the regularisation (the second-order stress and
// third-order Hermite projections), written in moments.  With nu = R^T mu and
// x = mu - (1 - om) nu,
//   lambda_k = s_rho(x) + (c_k - u).t(x) + (1 - om) nu_k + (mu.R f1 / tau^2) dtau/df_k,
// s_rho + (c - u).t being the transposed derivative of f_eq3 (orders 0..3),
// which needs only the weighted moments of x.  nu_k = 4.5 c_k^T M' c_k +
// sum_j b_j P_j(c_k) / N_j with M = sum w mu c c, M' = M - (sum w mu) I / 3 and
// b_j = sum w mu P_j(c); the D3Q19 lattice moments (sum w = 1,
// sum w c_a c_b = delta / 3, sum w c_a c_b c_c c_d = (three deltas) / 9, odd
// moments zero, sum w P_j P_j' = N_j delta_jj') give the moments of w nu in
// closed form: order 0 1.5 tr M', order 1 zero, order 2
// (tr M' I + 2 M') / 2, third order b_j.  lambda_k is then a cubic
// polynomial in c_k with sixteen coefficients.  srcw: objective weight of
// u_x (adds srcw (c_kx - u_x) / rho).
__device__ __forceinline__ void adjoint_rr3_moments(const Geo &G, const Rr3State &st, const float mu[Q], float srcw,
                                                    float lam[Q])
{
    const float *P = st.P;
    const float qn = stress_norm(P);
    const float R = sqrtf(G.tau0 * G.tau0 + G.kcs * qn / st.rho);
    const float tau = 0.5f * (G.tau0 + R);
    const float om = 1.0f / tau;
    const float keep = 1.0f - om;
    const float ux = st.ux, uy = st.uy, uz = st.uz, rho = st.rho;
    const float A3[6] = {ux * ux * uy + uy * uz * uz, ux * ux * uy - uy * uz * uz,
                         ux * uz * uz + ux * uy * uy, ux * uz * uz - ux * uy * uy,
                         uy * uy * uz + ux * ux * uz, uy * uy * uz - ux * ux * uz};
    const float dA3[6][3] = {{2.f * ux * uy, ux * ux + uz * uz, 2.f * uy * uz},
                             {2.f * ux * uy, ux * ux - uz * uz, -2.f * uy * uz},
                             {uz * uz + uy * uy, 2.f * ux * uy, 2.f * ux * uz},
                             {uz * uz - uy * uy, -2.f * ux * uy, 2.f * ux * uz},
                             {2.f * ux * uz, 2.f * uy * uz, uy * uy + ux * ux},
                             {-2.f * ux * uz, 2.f * uy * uz, uy * uy - ux * ux}};
    // third-order projections of f1: sum_i P_j(c_i) f_eq3_i = rho A3_j (the
    // lower orders are orthogonal to P_j), and sum_i P_j(c_i) w_i = 0
    float a1[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) a1[j] = st.t3[j] - rho * A3[j];
    const WMoments W = weighted_moments(mu);
    const float M0 = W.m0;
    const float trp = W.m2[0] + W.m2[1] + W.m2[2] - M0;     // tr M'
    const float Mp[6] = {W.m2[0] - M0 * (1.0f / 3.0f), W.m2[1] - M0 * (1.0f / 3.0f), W.m2[2] - M0 * (1.0f / 3.0f),
                         W.m2[3], W.m2[4], W.m2[5]};
    // mu . R f1
    float sR = 4.5f * (Mp[0] * P[0] + Mp[1] * P[1] + Mp[2] * P[2] + 2.0f * (Mp[3] * P[3] + Mp[4] * P[4] + Mp[5] * P[5]));
#pragma unroll
    for (int j = 0; j < 6; ++j) sR += herm3_inv_norm(j) * a1[j] * W.h3[j];
    // weighted moments of x = mu - keep nu
    const float m0 = M0 - keep * 1.5f * trp;
    const float m1x = W.m1[0], m1y = W.m1[1], m1z = W.m1[2];
    const float mxx = W.m2[0] - keep * (0.5f * trp + Mp[0]);
    const float myy = W.m2[1] - keep * (0.5f * trp + Mp[1]);
    const float mzz = W.m2[2] - keep * (0.5f * trp + Mp[2]);
    const float mxy = W.m2[3] - keep * Mp[3];
    const float mxz = W.m2[4] - keep * Mp[4];
    const float myz = W.m2[5] - keep * Mp[5];
    const float usq = ux * ux + uy * uy + uz * uz;
    const float m2ux = mxx * ux + mxy * uy + mxz * uz;
    const float m2uy = mxy * ux + myy * uy + myz * uz;
    const float m2uz = mxz * ux + myz * uy + mzz * uz;
    float srho = m0 * (1.0f - 1.5f * usq) + 3.0f * (m1x * ux + m1y * uy + m1z * uz) +
                 4.5f * (ux * m2ux + uy * m2uy + uz * m2uz);
    float t[3] = {3.0f * m1x + 9.0f * m2ux - 3.0f * ux * m0, 3.0f * m1y + 9.0f * m2uy - 3.0f * uy * m0,
                  3.0f * m1z + 9.0f * m2uz - 3.0f * uz * m0};
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        // third-order moments of w x: (1 - keep) b_j
        const float h = herm3_inv_norm(j) * om * W.h3[j];
        srho += h * A3[j];
        t[0] += h * dA3[j][0];
        t[1] += h * dA3[j][1];
        t[2] += h * dA3[j][2];
    }
    // Smagorinsky tau_eff: + (mu.R f1 / tau^2) dtau/df_k = sa (c_k - u)^T P (c_k - u) + sb
    float sa = 0.0f, sb = 0.0f;
    if (qn > 0.0f) {
        const float pre = sR / (tau * tau) * G.kcs / (4.0f * R);
        sa = pre / (rho * qn);
        sb = -pre * qn / (rho * rho) - sa * (P[0] + P[1] + P[2]) * (1.0f / 3.0f);
    }
    const float src = srcw / rho;
    const float Pu[3] = {P[0] * ux + P[3] * uy + P[4] * uz, P[3] * ux + P[1] * uy + P[5] * uz,
                         P[4] * ux + P[5] * uy + P[2] * uz};
    const float alpha = srho - (ux * t[0] + uy * t[1] + uz * t[2]) + sb - src * ux +
                        sa * (ux * Pu[0] + uy * Pu[1] + uz * Pu[2]);
    const float beta[3] = {t[0] - 2.0f * sa * Pu[0] + src, t[1] - 2.0f * sa * Pu[1], t[2] - 2.0f * sa * Pu[2]};
    const float k45 = 4.5f * keep;
    const float Gam[6] = {k45 * Mp[0] + sa * P[0], k45 * Mp[1] + sa * P[1], k45 * Mp[2] + sa * P[2],
                          k45 * Mp[3] + sa * P[3], k45 * Mp[4] + sa * P[4], k45 * Mp[5] + sa * P[5]};
    float gam[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) gam[j] = keep * herm3_inv_norm(j) * W.h3[j];
    eval_poly<true, false>(lam, nullptr, 0.0f, alpha, beta, Gam, gam);
}

// mu_k = sum of lam^{n+1} over the destination links of direction k, and the
// inflow-parameter gradient of the moving-wall links among them.
// CLAMP: neighbour indices clamped into the instance (speculative gathers).
template <bool CLAMP = false, int... Ks>
__device__ __forceinline__ void adjoint_gather(const Geo &G, const Shape &S, const Preds &p, uint32_t sm, uint32_t c,
                                               int z, const InflowT &T, const GLOBAL_AS float *__restrict__ lin,
                                               float mu[Q],
                                               double &gr0,
                                               double &gr1, double &gr2, std::integer_sequence<int, Ks...>)
{
    const uint32_t qs = (uint32_t)G.qs;
    const uint32_t last = (uint32_t)G.ncells - 1u;
    auto cell = [&](int32_t delta) {
        const uint32_t n = (uint32_t)((int32_t)c + delta);
        return CLAMP ? umin_u32(n, last) : n;
    };
    double sx = 0.0, sy = 0.0;
    bool inl = false;
    // Every lane loads its links (a missing one reads the cell's own slot and
    // is dropped) and the moving-wall terms are selected, not branched on: a
    // load under a lane condition is waited for inside its branch, one
    // direction after the other, which took a third of the adjoint step.
    (
        [&] {
            RelLink a, e;
            scatter_rel<Ks>(S, p, sm, a, e);
            const uint32_t own = (uint32_t)Ks * qs + c;
            float s = 0.0f;
            if constexpr (cx(Ks) == -1) {
                const float v = ldg(lin, e.valid ? (uint32_t)e.slot * qs + cell(e.delta) : own);
                s = e.valid ? v : 0.0f;
            }
            const float l = ldg(lin, a.valid ? (uint32_t)a.slot * qs + cell(a.delta) : own);
            mu[Ks] = a.valid ? s + l : s;
            constexpr int q = opp(Ks);
            const double f6 = a.inlet ? 6.0 * (double)wgt(q) * (double)l : 0.0;
            sx += (double)cx(q) * f6;
            sy += (double)cy(q) * f6;
            inl = inl || a.inlet;
        }(),
        ...);
    if (inl) inflow_grad(G, z, T, sx, sy, gr0, gr1, gr2);
}

// In-place adjoint of the odd step, one direction at a time: the lambda
// of the cell's gathered (pre-collision) population I goes into the slot
// the forward step gathered it from, with the moving-wall gradient of a
// gathered inlet link (inflow of step n-1).  On the outflow column, the
// links with c_x = -1 that do not bounce back (the zero-gradient outlet, and
// the free-slip sky whose source is clamped to the column) gather from a
// slot that the upstream neighbour gathers from too: their lambda goes one
// lane down (rows start at even cells, so the pair shares a wavefront) and
// the neighbour adds it before it stores.  The extra destinations of the
// outflow column, which the forward step writes and none of its gathers
// reads, are zeroed.  Every slot is thus read (as a scatter destination) and
// written by one lane.  plain: a wavefront without boundary rules (class 0),
// whose gathered slots are the plain shifted ones.
template <class F, int... Is>
__device__ __forceinline__ void adjoint_emit(const Geo &G, const Shape &S, const Preds &p, uint32_t sm, uint32_t c,
                                             int z, const InflowT &T, GLOBAL_AS float *lam, bool plain,
                                             bool wave_out, bool outflow, bool owner, F lk_of, double &gr0,
                                             double &gr1, double &gr2, std::integer_sequence<int, Is...>)
{
    const uint32_t qs = (uint32_t)G.qs;
    double sx = 0.0, sy = 0.0;
    bool inl = false;
    (
        [&] {
            float v = lk_of(Is);
            if (plain) {
                stg(lam + (size_t)opp(Is) * qs, (uint32_t)((int32_t)c - off_of(G, Is)), v);
                return;
            }
            const RelLink l = gather_rel<Is>(S, p, sm);
            bool shared = false;
            if constexpr (cx(Is) == -1) {
                if (wave_out) {
                    shared = outflow && l.slot != Is;
                    const float recv = __shfl_down(shared ? v : 0.0f, 1, 64);
                    if (owner) v += recv;
                }
            }
            if (!shared) stg(lam, (uint32_t)l.slot * qs + (uint32_t)((int32_t)c + l.delta), v);
            if (l.inlet) {
                const double f6 = 6.0 * (double)wgt(Is) * (double)v;
                sx += (double)cx(Is) * f6;
                sy += (double)cy(Is) * f6;
                inl = true;
            }
            if constexpr (cx(Is) == -1) {
                if (wave_out && outflow) {
                    RelLink pr, ex;
                    scatter_rel<Is>(S, p, sm, pr, ex);
                    if (ex.valid) stg(lam, (uint32_t)ex.slot * qs + (uint32_t)((int32_t)c + ex.delta), 0.0f);
                }
            }
        }(),
        ...);
    if (inl) inflow_grad(G, z, T, sx, sy, gr0, gr1, gr2);
}

// The transposed links of a class-1 wavefront (see gather_x / scatter_x):
// mu_K sums lam^{n+1} over the destinations of the post-collision value K,
// the plain one except at the x faces (x = 0, c_x = -1: own slot opp(K),
// with the moving-wall gradient at an inlet; x = nx-1, c_x = +1: none at an
// outlet, own slot opp(K) at a wall; x = nx-1, c_x = -1 at an outlet: plus
// slot K of (nx-1, y + c_y, z + c_z)).
template <int... Ks>
__device__ __forceinline__ void adjoint_gather_x(const Geo &G, const Shape &S, bool xlo, bool xhi, uint32_t c, int z,
                                                 const InflowT &T, const GLOBAL_AS float *__restrict__ lin,
                                                 float mu[Q], double &gr0, double &gr1, double &gr2,
                                                 std::integer_sequence<int, Ks...>)
{
    const uint32_t qs = (uint32_t)G.qs;
    const uint32_t last = (uint32_t)G.ncells - 1u;
    const bool inl = S.face[0] == FACE_INLET, out = S.face[1] == FACE_OUTLET;
    double sx = 0.0, sy = 0.0;
    (
        [&] {
            constexpr int K = Ks;
            const uint32_t pn = umin_u32((uint32_t)((int32_t)c + off_of(G, K)), last);
            if constexpr (cx(K) == -1) {
                float v = ldg(lin, xlo ? (uint32_t)opp(K) * qs + c : (uint32_t)K * qs + pn);
                // the outlet's second link, loaded by every lane (see adjoint_gather)
                const float w = ldg(lin, (uint32_t)K * qs +
                                             umin_u32((uint32_t)((int32_t)c + cy(K) * G.offy + cz(K) * G.offz), last));
                if (xlo && inl) {
                    constexpr int q = opp(K);
                    const double f6 = 6.0 * (double)wgt(q) * (double)v;
                    sx += (double)cx(q) * f6;
                    sy += (double)cy(q) * f6;
                }
                if (xhi && out) v += w;
                mu[K] = v;
            } else if constexpr (cx(K) == 1) {
                const float v = ldg(lin, xhi ? (uint32_t)opp(K) * qs + c : (uint32_t)K * qs + pn);
                mu[K] = (xhi && out) ? 0.0f : v;
            } else {
                mu[K] = ldg(lin, (uint32_t)K * qs + pn);
            }
        }(),
        ...);
    if (xlo && inl) inflow_grad(G, z, T, sx, sy, gr0, gr1, gr2);
}

// In-place adjoint of the odd step in a class-1 wavefront (see
// adjoint_emit): lam of the gathered population I goes to the slot the
// forward step gathered it from, the plain one except at the x faces
// (x = 0, c_x = +1: own slot I, with the moving-wall gradient at an inlet;
// x = nx-1, c_x = -1: own slot I at a wall; at an outlet the slot is the one
// the upstream neighbour, one lane down, gathers from too: the value goes to
// that lane, which adds it before it stores, and the outflow column's extra
// destination, slot I of (nx-1, y + c_y, z + c_z), is zeroed).
template <class F, int... Is>
__device__ __forceinline__ void adjoint_emit_x(const Geo &G, const Shape &S, bool xlo, bool xhi, bool owner,
                                               bool wave_out, uint32_t c, int z, const InflowT &T,
                                               GLOBAL_AS float *lam, F lk_of, double &gr0, double &gr1, double &gr2,
                                               std::integer_sequence<int, Is...>)
{
    const uint32_t qs = (uint32_t)G.qs;
    const bool inl = S.face[0] == FACE_INLET, out = S.face[1] == FACE_OUTLET;
    double sx = 0.0, sy = 0.0;
    (
        [&] {
            constexpr int I = Is;
            float v = lk_of(I);
            const uint32_t pn = (uint32_t)opp(I) * qs + (uint32_t)((int32_t)c - off_of(G, I));
            if constexpr (cx(I) == 1) {
                stg(lam, xlo ? (uint32_t)I * qs + c : pn, v);
                if (xlo && inl) {
                    const double f6 = 6.0 * (double)wgt(I) * (double)v;
                    sx += (double)cx(I) * f6;
                    sy += (double)cy(I) * f6;
                }
            } else if constexpr (cx(I) == -1) {
                const bool shared = xhi && out;
                if (wave_out) {
                    const float recv = __shfl_down(shared ? v : 0.0f, 1, 64);
                    if (owner) v += recv;
                }
                if (!shared)
                    stg(lam, xhi ? (uint32_t)I * qs + c : pn, v);
                else
                    stg(lam, (uint32_t)I * qs + (uint32_t)((int32_t)c + cy(I) * G.offy + cz(I) * G.offz), 0.0f);
            } else {
                stg(lam, pn, v);
            }
        }(),
        ...);
    if (xlo && inl) inflow_grad(G, z, T, sx, sy, gr0, gr1, gr2);
}

// One adjoint step of every instance, with the tiling of the step kernels:
// a workgroup of BS threads owns BS * CPT consecutive cells of one instance.
// Gather: per wavefront class the plain shifted pattern, the transposed x
// rules, the transposed x and solid-link rules or the full transposed rules.
// Then per cell the transposed collision and the probe source; solid cells
// write zero (their lambda is never read) so the stores cover whole lines.
// MODE 0: lambda^{n+1} and lambda^n in two buffers, both in the natural
// layout.  MODE 1 and 2: one buffer updated in place, in the storage layout
// of the populations (the transposed in-place streaming): MODE 1 is the
// adjoint of an odd step (lambda read at the slots the step scattered to,
// written to the slots it gathered from), MODE 2 of an even step (own
// slots, swapped back).  REC: the record kind the sweep recorded (1 (rho, u),
// 2 populations, 3 the regularised state), a template parameter so that each
// instantiation carries one record path.
template <int BS, int CPT, int MODEL, int MODE, int REC>
__global__ __launch_bounds__(BS) void k_adjoint(const Geo *__restrict__ geo, const int32_t *__restrict__ tile_inst,
                                                int32_t n_tiles, int32_t xcd_remap, AdjArgs a)
{
    const int tile = tile_of(xcd_remap);
    if (tile >= n_tiles) return;
    const int ii = __builtin_amdgcn_readfirstlane(tile_inst[tile]);
    const Geo &G = geo[ii];
    const uint32_t qs = (uint32_t)G.qs;
    const GLOBAL_AS float *__restrict__ lin = gp(a.lam_in[ii]);
    GLOBAL_AS float *__restrict__ lout = gp(a.lam_out[ii]);
    GLOBAL_AS float *lbuf = gp(a.lam_out[ii]);   // MODE 1, 2: read and written in place (no restrict)
    const int32_t base = (tile - G.tile0) * (BS * CPT) + (int32_t)threadIdx.x;
    const uint64_t wcls = a.tinfo ? a.tinfo[2 * (size_t)tile + 1] : ~0ull;
    const uint32_t last = (uint32_t)G.ncells - 1u;
    double gr0 = 0.0, gr1 = 0.0, gr2 = 0.0;
    bool inlet_lane = false;

    uint32_t c[CPT];
    uint8_t fl[CPT];
    int cls[CPT];
    bool act[CPT], fluid[CPT];
    float mu[CPT][Q];
    double sg[CPT][3];             // gradient of a speculative x-rule gather
    uint32_t smv[CPT];             // solid-link mask (classes 2 and 3)
    f32x4 st[CPT];                 // (rho, ux, uy, uz) of a kind-1 record
    float gs[CPT][Q];              // populations of a kind-2 record
    const Shape S = shape_of(G);
    // mu = P^T lam^{n+1}: the sum over the destination links of each
    // post-collision value.  Wavefronts of class 0 (plain) and 1 (x rules
    // only, see launch_tile_info) take their addresses from the cell index
    // alone and issue their gathers at once, with the neighbour index
    // clamped into the instance (values and gradients of solid lanes are
    // dropped); flags and records of all of the thread's cells follow, and
    // classes 2 and 3 gather after them.
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int32_t lc = base + j * BS;
        act[j] = lc < G.ncells;
        c[j] = act[j] ? (uint32_t)lc : 0u;
        cls[j] = (int)((wcls >> (2 * ((j * BS + (int)threadIdx.x) >> 6))) & 3ull);
        sg[j][0] = sg[j][1] = sg[j][2] = 0.0;
        if (MODE == 2) {
            // adjoint of an even step: the cell's own slots, swapped
            cls[j] = 0;
            if (act[j]) {
#pragma unroll
                for (int k = 0; k < Q; ++k) mu[j][k] = ldg(lbuf + (size_t)opp(k) * qs, c[j]);
            }
        } else if (cls[j] == 0) {
            if (act[j]) {
#pragma unroll
                for (int k = 0; k < Q; ++k)
                    mu[j][k] = ldg((MODE == 0 ? lin : lbuf) + (size_t)k * qs,
                                   umin_u32((uint32_t)((int32_t)c[j] + off_of(G, k)), last));
            }
        } else if (cls[j] == 1) {
            int x, y, z;
            coords(G, c[j], x, y, z);
            const bool inl = act[j] && x == 0 && S.face[0] == FACE_INLET;
            const InflowT Tx = __any(inl) ? inflow_at(G, a.step) : InflowT{0.f, 0.f, 0.f, 0.f};
            if (act[j])
                adjoint_gather_x(G, S, x == 0, x == S.nx - 1, c[j], z, Tx, MODE == 0 ? lin : lbuf, mu[j], sg[j][0],
                                 sg[j][1], sg[j][2], Dirs{});
        }
        fl[j] = act[j] ? gp(G.flags)[c[j]] : (uint8_t)FL_SOLID;
        smv[j] = (cls[j] >= 2 && act[j]) ? gp(G.smask)[c[j]] : 0u;
        if (REC == 1 && act[j])
            st[j] = __builtin_nontemporal_load((const GLOBAL_AS f32x4 *)gp(a.rec[ii]) + ((size_t)a.rec_slot * (size_t)G.ncells + c[j]));
    }
    bool flow2 = false;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        fluid[j] = !(fl[j] & FL_SOLID);
        const bool flow = fluid[j] && inflow_lane(G, fl[j]);
        if (flow) inlet_lane = true;
        if (cls[j] >= 2 && flow) flow2 = true;
        if (cls[j] == 1 && fluid[j]) {
            gr0 += sg[j][0];
            gr1 += sg[j][1];
            gr2 += sg[j][2];
        }
    }
    // the inflow only where a lane of the wavefront has moving-wall links
    const InflowT T = __any(flow2) ? inflow_at(G, a.step) : InflowT{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        if (!fluid[j]) continue;
        if (cls[j] == 3) {
            int x, y, z;
            coords(G, c[j], x, y, z);
            const Preds pr = preds_of(S, x, y, z, fl[j]);
            adjoint_gather(G, S, pr, smv[j], c[j], z, T, MODE == 0 ? lin : lbuf, mu[j], gr0, gr1, gr2, Dirs{});
        } else if (cls[j] == 2) {
            const Preds ps = preds_xs(fl[j]);
            const int z = inflow_lane(G, fl[j]) ? (int)fdiv(c[j], G.dxy) : 0;
            adjoint_gather(G, S, ps, smv[j], c[j], z, T, MODE == 0 ? lin : lbuf, mu[j], gr0, gr1, gr2, Dirs{});
        }
        if (REC == 2) {
            const GLOBAL_AS float *rp = gp(a.rec[ii]) + (size_t)a.rec_slot * (size_t)Q * G.qs;
#pragma unroll
            for (int i = 0; i < Q; ++i) gs[j][i] = ldg<true>(rp, (uint32_t)i * qs + c[j]);
        } else if (MODEL == 2 && REC == 3) {
            const GLOBAL_AS float *rp = gp(a.rec[ii]) + (size_t)a.rec_slot * (size_t)RR3_REC * G.qs;
#pragma unroll
            for (int i = 0; i < RR3_REC; ++i) gs[j][i] = ldg<true>(rp, (uint32_t)i * qs + c[j]);
        }
    }
    // MODE 1: the rules of each cell's stores (see adjoint_emit)
    Preds pg[MODE == 1 ? CPT : 1];
    int zg[MODE == 1 ? CPT : 1];
    bool wout[MODE == 1 ? CPT : 1], outflow[MODE == 1 ? CPT : 1], owner[MODE == 1 ? CPT : 1];
    InflowT Tg{0.f, 0.f, 0.f, 0.f};
    if constexpr (MODE == 1) {
        const bool out_face = S.face[1] == FACE_OUTLET;
        bool flowg = false;
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            pg[j] = Preds{false, false, false, false, false, false, false};
            zg[j] = 0;
            owner[j] = false;
            if (act[j] && fluid[j] && cls[j] >= 1) {
                int x, y, z;
                coords(G, c[j], x, y, z);
                zg[j] = z;
                pg[j] = cls[j] == 3 ? preds_of(S, x, y, z, fl[j])
                                    : (cls[j] == 2 ? preds_xs(fl[j])
                                                   : Preds{x == 0, x == S.nx - 1, false, false, false, false, false});
                owner[j] = out_face && x == S.nx - 2;
                if (inflow_lane(G, fl[j])) flowg = true;
            }
            outflow[j] = act[j] && fluid[j] && out_face && pg[j].xhi;
            wout[j] = __any(outflow[j]);
        }
        if (__any(flowg)) Tg = inflow_at(G, a.step - 1);
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        if (!act[j]) continue;
        if (!fluid[j]) {
#pragma unroll
            for (int k = 0; k < Q; ++k) stg((MODE == 0 ? lout : lbuf) + (size_t)k * qs, c[j], 0.0f);
            continue;
        }
        if constexpr (MODEL == 2) {
            float srcw = 0.0f, lam[Q];
            if (a.in_window && (fl[j] & FL_PROBE) && a.pw[ii]) {
                const int p = probe_index(G, (int32_t)c[j]);
                if (p >= 0) srcw = (float)(a.pw[ii][p] * a.inv_count);
            }
            Rr3State st;
            if (REC == 3) {
                st.rho = gs[j][0];
                st.ux = gs[j][1];
                st.uy = gs[j][2];
                st.uz = gs[j][3];
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    st.P[k] = gs[j][4 + k];
                    st.t3[k] = gs[j][10 + k];
                }
            } else {
                st = rr3_state(gs[j]);
            }
            adjoint_rr3_moments(G, st, mu[j], srcw, lam);
            if constexpr (MODE == 1) {
                if (cls[j] == 1)
                    adjoint_emit_x(G, S, pg[j].xlo, pg[j].xhi, owner[j], wout[j], c[j], zg[j], Tg, lbuf,
                                   [&](int k) { return lam[k]; }, gr0, gr1, gr2, Dirs{});
                else
                    adjoint_emit(G, S, pg[j], smv[j], c[j], zg[j], Tg, lbuf, cls[j] == 0, wout[j], outflow[j],
                                 owner[j], [&](int k) { return lam[k]; }, gr0, gr1, gr2, Dirs{});
            } else {
#pragma unroll
                for (int k = 0; k < Q; ++k) stg((MODE == 0 ? lout : lbuf) + (size_t)k * qs, c[j], lam[k]);
            }
            continue;
        }
        // state of step n (the relaxation rate as the forward step forms it)
        float rho, ux, uy, uz;
        float muf = 0.0f, P[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, qn = 0.0f, tau = G.tau0;
        if (REC == 1) {
            rho = st[j].x;
            ux = st[j].y;
            uy = st[j].z;
            uz = st[j].w;
        } else {
            const float *g = gs[j];
            const PairSums ps = pair_sums(g);
            const Macro m = macro_of(g, ps);
            rho = m.rho;
            ux = m.ux;
            uy = m.uy;
            uz = m.uz;
            if (MODEL == 1) {
                neq_stress(ps, m, P);
                qn = stress_norm(P);
                tau = tau_of<1>(G, ps, m);
#pragma unroll
                for (int i = 0; i < Q; ++i) muf += mu[j][i] * g[i];
            }
        }
        const float om = fast_rcp(tau);
        // BGK part: (1 - om) mu_k + om [s_rho + (c_k - u) . t], from the
        // weighted moments of mu
        const WMoments W = weighted_moments(mu[j]);
        const float m0 = W.m0, m1x = W.m1[0], m1y = W.m1[1], m1z = W.m1[2];
        const float mxx = W.m2[0], myy = W.m2[1], mzz = W.m2[2], mxy = W.m2[3], mxz = W.m2[4], myz = W.m2[5];
        const float usq = ux * ux + uy * uy + uz * uz;
        const float m2ux = mxx * ux + mxy * uy + mxz * uz;
        const float m2uy = mxy * ux + myy * uy + myz * uz;
        const float m2uz = mxz * ux + myz * uy + mzz * uz;
        const float srho = m0 * (1.0f - 1.5f * usq) + 3.0f * (m1x * ux + m1y * uy + m1z * uz) +
                           4.5f * (ux * m2ux + uy * m2uy + uz * m2uz);
        const float tx = 3.0f * m1x + 9.0f * m2ux - 3.0f * ux * m0;
        const float ty = 3.0f * m1y + 9.0f * m2uy - 3.0f * uy * m0;
        const float tz = 3.0f * m1z + 9.0f * m2uz - 3.0f * uz * m0;
        // Smagorinsky: + (A / tau^2) dtau/df_k = sa (c_k - u)^T P (c_k - u) + sb
        // with A = mu . (f - f_eq) = mu . f - mu . f_eq, where (f - w and f_eq
        // - w stored) mu . f_eq = rho s_rho - m0 comes from the same weighted
        // moments, and R = 2 tau - tau0 the root of tau_eff
        float sa = 0.0f, sb = 0.0f;
        if (MODEL == 1 && qn > 0.0f) {
            const float A = muf - (rho * srho - m0);
            const float R = 2.0f * tau - G.tau0;
            const float pre = A * G.kcs * fast_rcp(4.0f * tau * tau * R);
            const float irho = fast_rcp(rho);
            sa = pre * irho * fast_rcp(qn);
            sb = -pre * qn * irho * irho - sa * (P[0] + P[1] + P[2]) * (1.0f / 3.0f);
        }
        // objective source at the probes: pw_p / count * (c_kx - u_x) / rho
        float src = 0.0f;
        if (a.in_window && (fl[j] & FL_PROBE) && a.pw[ii]) {
            const int p = probe_index(G, (int32_t)c[j]);
            if (p >= 0) src = (float)(a.pw[ii][p] * a.inv_count) / rho;
        }
        // lambda_k = (1 - om) mu_k + alpha + beta . c_k + c_k^T (sa P) c_k
        const float Pu[3] = {P[0] * ux + P[3] * uy + P[4] * uz, P[3] * ux + P[1] * uy + P[5] * uz,
                             P[4] * ux + P[5] * uy + P[2] * uz};
        const float alpha = om * (srho - (ux * tx + uy * ty + uz * tz)) + sb - src * ux +
                            sa * (ux * Pu[0] + uy * Pu[1] + uz * Pu[2]);
        const float beta[3] = {om * tx - 2.0f * sa * Pu[0] + src, om * ty - 2.0f * sa * Pu[1],
                               om * tz - 2.0f * sa * Pu[2]};
        const float Gam[6] = {sa * P[0], sa * P[1], sa * P[2], sa * P[3], sa * P[4], sa * P[5]};
        eval_poly<false, true>(mu[j], mu[j], 1.0f - om, alpha, beta, Gam, nullptr);
        auto lk_of = [&](int k) { return mu[j][k]; };
        if constexpr (MODE == 1) {
            if (cls[j] == 1)
                adjoint_emit_x(G, S, pg[j].xlo, pg[j].xhi, owner[j], wout[j], c[j], zg[j], Tg, lbuf, lk_of, gr0, gr1,
                               gr2, Dirs{});
            else
                adjoint_emit(G, S, pg[j], smv[j], c[j], zg[j], Tg, lbuf, cls[j] == 0, wout[j], outflow[j], owner[j],
                             lk_of, gr0, gr1, gr2, Dirs{});
        } else {
#pragma unroll
            for (int k = 0; k < Q; ++k) stg((MODE == 0 ? lout : lbuf) + (size_t)k * qs, c[j], lk_of(k));
        }
    }
    // gradient: wavefront sums, then one partial per tile (the per-instance
    // sums are formed afterwards in a fixed order, without atomics)
    __shared__ double red[BS / 64][3];
    const int wv = threadIdx.x >> 6;
    if (__any(inlet_lane)) {
        gr0 = wave_sum(gr0);
        gr1 = wave_sum(gr1);
        gr2 = wave_sum(gr2);
    }
    if ((threadIdx.x & 63) == 0) {
        red[wv][0] = gr0;
        red[wv][1] = gr1;
        red[wv][2] = gr2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < BS / 64; ++w) t += red[w][threadIdx.x];
        a.part[3 * (size_t)tile + threadIdx.x] = t;
    }
}

inline int grid_of(int32_t n_tiles) { return ((n_tiles + 7) / 8) * 8; }

}  // namespace

}  // namespace lbmsc
