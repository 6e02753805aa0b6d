// hostcheck.hip -- host-only checks of the link rules used by the kernels.
//
// Built into a separate host library so that CPU tests can verify, without a
// GPU, that the in-place update is well defined for a geometry and a
// workgroup size:
//   * push_dsts() is the exact inverse of pull_src(): every fluid destination
//     link has exactly one source, and that source lists it;
//   * in the odd (gather-then-scatter) step, every memory slot is written at
//     most once, and every slot touched by more than one cell is touched only
//     by cells of one workgroup, where a barrier orders the reads before the
//     writes.
// It also exposes the per-link rule kinds so they can be compared with an
// independent implementation.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <unordered_map>
#include <utility>
#include <vector>

#include "rules.h"

using namespace lbmsc;

namespace {

struct Geo3 {
    Box b;
    const uint8_t *solid;
    std::vector<uint8_t> fl;
    std::vector<uint32_t> m;
    int64_t n;
    int64_t cell(int x, int y, int z) const { return ((int64_t)z * b.ny + y) * b.nx + x; }
};

bool mantle_of(const Geo3 &g, int64_t c) { return (g.fl[c] & FL_MANTLE) != 0; }

void build(Geo3 &g, int nx, int ny, int nz, const int *face, const uint8_t *solid)
{
    g.b.nx = nx;
    g.b.ny = ny;
    g.b.nz = nz;
    for (int k = 0; k < 6; ++k) g.b.face[k] = face[k];
    g.solid = solid;
    g.n = (int64_t)nx * ny * nz;
    g.fl.assign(g.n, 0);
    g.m.assign(g.n, 0);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int64_t c = g.cell(x, y, z);
                cell_flags(g.b, solid, x, y, z, g.fl[c], g.m[c]);
            }
}

}  // namespace

extern "C" {

// Rule kind of every link ([19][ncells], -1 for solid cells).
void lbmhc_rules(int nx, int ny, int nz, const int *face, const uint8_t *solid, int *rules)
{
    Geo3 g;
    build(g, nx, ny, nz, face, solid);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int64_t c = g.cell(x, y, z);
                for (int i = 0; i < Q; ++i)
                    rules[i * g.n + c] = (g.fl[c] & FL_SOLID) ? -1 : pull_src(g.b, x, y, z, i, g.m[c], mantle_of(g, c)).kind;
            }
}

// Returns 0 when all properties hold, otherwise a code; stats[0..6] =
// fluid links, links through a non-plain rule, values with two destinations,
// shared slots, shared slots spanning two workgroups, slots written twice,
// zero writes of solid cells into their own slots.
int lbmhc_check(int nx, int ny, int nz, const int *face, const uint8_t *solid, int block, int64_t *stats)
{
    Geo3 g;
    build(g, nx, ny, nz, face, solid);
    for (int k = 0; k < 7; ++k) stats[k] = 0;
    // 1. inverse property
    std::vector<int8_t> hit((size_t)Q * g.n, 0);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int64_t c = g.cell(x, y, z);
                if (g.fl[c] & FL_SOLID) continue;
                for (int k = 1; k < Q; ++k) {
                    Link d[2];
                    const int nd = push_dsts(g.b, x, y, z, k, g.m[c], mantle_of(g, c), d[0], d[1]);
                    if (nd == 2) ++stats[2];
                    for (int j = 0; j < nd; ++j) {
                        if (d[j].x < 0 || d[j].x >= nx || d[j].y < 0 || d[j].y >= ny || d[j].z < 0 || d[j].z >= nz)
                            return 1;
                        const int64_t dc = g.cell(d[j].x, d[j].y, d[j].z);
                        if (g.fl[dc] & FL_SOLID) return 2;
                        const Link s = pull_src(g.b, d[j].x, d[j].y, d[j].z, d[j].pop, g.m[dc], mantle_of(g, dc));
                        if (s.x != x || s.y != y || s.z != z || s.pop != k || s.kind != d[j].kind) return 3;
                        if (hit[(size_t)d[j].pop * g.n + dc]++) return 4;
                    }
                }
            }
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int64_t c = g.cell(x, y, z);
                if (g.fl[c] & FL_SOLID) continue;
                for (int i = 1; i < Q; ++i) {
                    ++stats[0];
                    const Link s = pull_src(g.b, x, y, z, i, g.m[c], mantle_of(g, c));
                    if (s.kind != R_STREAM) ++stats[1];
                    if (!hit[(size_t)i * g.n + c]) return 5;  // a link without a source
                    const int64_t sc = g.cell(s.x, s.y, s.z);
                    if (g.fl[sc] & FL_SOLID) return 6;
                    // fast paths: a cell without FL_NEAR must stream plainly both ways
                    if (!(g.fl[c] & FL_NEAR)) {
                        if (s.kind != R_STREAM || s.x != x - cx(i) || s.y != y - cy(i) || s.z != z - cz(i)) return 7;
                        Link d[2];
                        if (push_dsts(g.b, x, y, z, i, g.m[c], mantle_of(g, c), d[0], d[1]) != 1 || d[0].kind != R_STREAM) return 8;
                    }
                }
            }
    // 2. odd-step slot ownership: cells touching each slot (read of swapped
    // value or write of the next natural value)
    std::unordered_map<int64_t, std::vector<int64_t>> touch;
    std::unordered_map<int64_t, int> writes;
    auto slot = [&](int pop, int64_t cell) { return (int64_t)pop * g.n + cell; };
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int64_t c = g.cell(x, y, z);
                if (g.fl[c] & FL_SOLID) continue;
                for (int i = 0; i < Q; ++i) {
                    const Link s = pull_src(g.b, x, y, z, i, g.m[c], mantle_of(g, c));
                    touch[slot(opp(s.pop), g.cell(s.x, s.y, s.z))].push_back(c);
                }
                touch[slot(0, c)].push_back(c);
                ++writes[slot(0, c)];
                for (int k = 1; k < Q; ++k) {
                    Link d[2];
                    const int nd = push_dsts(g.b, x, y, z, k, g.m[c], mantle_of(g, c), d[0], d[1]);
                    for (int j = 0; j < nd; ++j) {
                        const int64_t s = slot(d[j].pop, g.cell(d[j].x, d[j].y, d[j].z));
                        touch[s].push_back(c);
                        if (++writes[s] > 1) ++stats[5];
                    }
                }
            }
    if (stats[5]) return 9;
    // the odd step writes zero into every slot of every solid cell: no fluid
    // cell may read or write any of them
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int64_t c = g.cell(x, y, z);
                if (!(g.fl[c] & FL_SOLID)) continue;
                for (int k = 0; k < Q; ++k) {
                    if (touch.count(slot(k, c))) return 12;
                    ++stats[6];
                }
            }
    for (auto &kv : touch) {
        const std::vector<int64_t> &v = kv.second;
        bool shared = false, cross = false;
        for (int64_t c : v) {
            if (c != v[0]) shared = true;
            if (c / block != v[0] / block) cross = true;
        }
        if (shared) ++stats[3];
        if (cross) ++stats[4];
    }
    if (stats[4]) return 10;
    return 0;
}

// Per-cell flag bytes as the kernels see them.
void lbmhc_flags(int nx, int ny, int nz, const int *face, const uint8_t *solid, uint8_t *fl)
{
    Geo3 g;
    build(g, nx, ny, nz, face, solid);
    for (int64_t c = 0; c < g.n; ++c) fl[c] = g.fl[c];
}

// Tile order of a launch: out[p] = tile_order(p, grid, mode) for p < grid.
void lbmhc_tile_order(int grid, int mode, int32_t *out)
{
    for (int p = 0; p < grid; ++p) out[p] = tile_order(p, grid, mode);
}

// Fast division: checks v / d against fdiv for the given values.
int lbmhc_fastdiv(uint32_t d, const uint32_t *v, int64_t n)
{
    const FastDiv f = make_fastdiv(d);
    for (int64_t k = 0; k < n; ++k)
        if (fdiv(v[k], f) != v[k] / d) return 1;
    return 0;
}

// Velocity set as the kernels see it: c [19][3], w [19], opp [19], zflip [19].
void lbmhc_lattice(int *c, float *w, int *o, int *zf)
{
    for (int i = 0; i < Q; ++i) {
        c[3 * i] = cx(i);
        c[3 * i + 1] = cy(i);
        c[3 * i + 2] = cz(i);
        w[i] = wgt(i);
        o[i] = opp(i);
        zf[i] = zflip(i);
    }
}

}  // extern "C"

namespace {

// One direction K of the in-place adjoint of the odd step, as the kernel
// evaluates it (relative rules): phase 0 the reads at the scatter
// destinations, 1 the hand-over of the outflow column's shared links to the
// upstream cell, 2 the stores at the gathered slots and the zeroed extras.
template <int K>
void adj_dir(int phase, const Geo3 &g, const Shape &S, int64_t c, int x, int y, int z, const std::vector<double> &in,
             std::vector<double> &out, std::vector<std::vector<double>> &nu)
{
    const int64_t n = g.n;
    const Preds p = preds_of(S, x, y, z, g.fl[c]);
    const uint32_t sm = g.m[c];
    if (phase == 0) {
        RelLink a, e;
        scatter_rel<K>(S, p, sm, a, e);
        double v = 0.0;
        if (a.valid) v += in[(int64_t)a.slot * n + c + a.delta];
        if (e.valid) v += in[(int64_t)e.slot * n + c + e.delta];
        nu[c][K] = v;
        return;
    }
    const RelLink l = gather_rel<K>(S, p, sm);
    const bool shared = cx(K) == -1 && p.xhi && S.face[1] == FACE_OUTLET && l.slot != K;
    if (phase == 1) {
        if (shared) nu[c - 1][K] += nu[c][K];
        return;
    }
    if (!shared) out[(int64_t)l.slot * n + c + l.delta] = nu[c][K];
    RelLink a, e;
    scatter_rel<K>(S, p, sm, a, e);
    if (e.valid) out[(int64_t)e.slot * n + c + e.delta] = 0.0;
}

template <int... Ks>
void adj_all(int phase, const Geo3 &g, const Shape &S, int64_t c, int x, int y, int z, const std::vector<double> &in,
             std::vector<double> &out, std::vector<std::vector<double>> &nu, std::integer_sequence<int, Ks...>)
{
    (adj_dir<Ks>(phase, g, S, c, x, y, z, in, out, nu), ...);
}

}  // namespace

extern "C" {

// The in-place adjoint of the odd step (identity collision, so that only the
// storage map is tested) against the exact transpose of that step's slot map
// built from pull_src / push_dsts: lam_in [19][n] is the adjoint after the
// step, both results are the adjoint before it.  Returns the number of slots
// where the kernel's rules (read at the scatter destinations, hand the
// outflow column's shared links to the upstream cell, store at the gathered
// slots, zero the extra destinations, solid cells zero) differ from the
// transpose by more than 1e-12.
int64_t lbmhc_check_adjoint_inplace(int nx, int ny, int nz, const int *face, const uint8_t *solid,
                                    const double *lam_in)
{
    Geo3 g;
    build(g, nx, ny, nz, face, solid);
    const int64_t n = g.n;
    Shape S;
    S.nx = nx;
    S.ny = ny;
    S.nz = nz;
    S.offy = nx;
    S.offz = nx * ny;
    for (int k = 0; k < 6; ++k) S.face[k] = face[k];
    std::vector<double> in(lam_in, lam_in + (size_t)Q * n), ref((size_t)Q * n, 0.0), out(in);
    // exact transpose: the forward step sets next[W(x,k)] = cur[R(x,k)]
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int64_t c = g.cell(x, y, z);
                if (g.fl[c] & FL_SOLID) continue;
                for (int k = 0; k < Q; ++k) {
                    const Link s = pull_src(g.b, x, y, z, k, g.m[c], mantle_of(g, c));
                    double mu = 0.0;
                    if (k == 0) {
                        mu = in[c];
                    } else {
                        Link d[2];
                        const int nd = push_dsts(g.b, x, y, z, k, g.m[c], mantle_of(g, c), d[0], d[1]);
                        for (int j = 0; j < nd; ++j) mu += in[(int64_t)d[j].pop * n + g.cell(d[j].x, d[j].y, d[j].z)];
                    }
                    ref[(int64_t)opp(s.pop) * n + g.cell(s.x, s.y, s.z)] += mu;
                }
            }
    std::vector<std::vector<double>> nu((size_t)n, std::vector<double>(Q, 0.0));
    for (int phase = 0; phase < 3; ++phase)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const int64_t c = g.cell(x, y, z);
                    if (g.fl[c] & FL_SOLID) {
                        if (phase == 2)
                            for (int k = 0; k < Q; ++k) out[(int64_t)k * n + c] = 0.0;
                        continue;
                    }
                    adj_all(phase, g, S, c, x, y, z, in, out, nu, std::make_integer_sequence<int, Q>{});
                }
    int64_t bad = 0;
    for (int64_t sl = 0; sl < (int64_t)Q * n; ++sl)
        if (std::fabs(out[sl] - ref[sl]) > 1e-12) ++bad;
    return bad;
}

}  // extern "C"

namespace {

Shape shape_of(const Geo3 &g)
{
    Shape s;
    s.nx = g.b.nx;
    s.ny = g.b.ny;
    s.nz = g.b.nz;
    s.offy = g.b.nx;
    s.offz = g.b.nx * g.b.ny;
    for (int k = 0; k < 6; ++k) s.face[k] = g.b.face[k];
    return s;
}

// 0 when gather_rel<I> and scatter_rel<I> agree with pull_src / push_dsts at cell (x,y,z)
template <int I>
int check_rel_one(const Geo3 &g, const Shape &s, int x, int y, int z)
{
    const int64_t c = g.cell(x, y, z);
    const Preds p = preds_of(s, x, y, z, g.fl[c]);
    const uint32_t m = g.m[c];
    const RelLink r = gather_rel<I>(s, p, m);
    const Link src = pull_src(g.b, x, y, z, I, m, p.mantle);
    if (I == 0) {
        if (r.slot != 0 || r.delta != 0 || r.inlet) return 20;
    } else {
        const int64_t want = g.cell(src.x, src.y, src.z);
        if (c + r.delta != want || r.slot != opp(src.pop)) return 21;
        if (r.inlet != (src.kind == R_INLET || src.kind == R_MANTLE)) return 22;
        Link d[2];
        const int nd = push_dsts(g.b, x, y, z, I, m, p.mantle, d[0], d[1]);
        RelLink a, e;
        scatter_rel<I>(s, p, m, a, e);
        const int nr = (int)a.valid + (int)e.valid;
        if (nr != nd) return 23;
        RelLink got[2];
        int k = 0;
        if (a.valid) got[k++] = a;
        if (e.valid) got[k++] = e;
        for (int j = 0; j < nd; ++j) {
            const int64_t dc = g.cell(d[j].x, d[j].y, d[j].z);
            if (c + got[j].delta != dc || got[j].slot != d[j].pop) return 24;
            if (got[j].inlet != (d[j].kind == R_INLET || d[j].kind == R_MANTLE)) return 25;
        }
    }
    return 0;
}

// cells flagged NEAR but not GENERAL: the x-column form (y/z predicates and
// the solid mask dropped) must give the full form's links
template <int I>
int check_xpath_one(const Geo3 &g, const Shape &s, int x, int y, int z)
{
    const int64_t c = g.cell(x, y, z);
    const uint8_t fl = g.fl[c];
    if (!(fl & FL_NEAR) || (fl & FL_GENERAL)) return 0;
    const Preds p = preds_of(s, x, y, z, fl);
    const Preds px{(fl & FL_XLO) != 0, (fl & FL_XHI) != 0, false, false, false, false, false};
    if (p.ylo || p.yhi || p.zlo || p.zhi || p.mantle || g.m[c]) return 30;
    const RelLink a = gather_rel<I>(s, p, g.m[c]), b = gather_rel<I>(s, px, 0u);
    if (a.slot != b.slot || a.delta != b.delta || a.inlet != b.inlet) return 31;
    RelLink pa, pe, qa, qe;
    scatter_rel<I>(s, p, g.m[c], pa, pe);
    scatter_rel<I>(s, px, 0u, qa, qe);
    if (pa.valid != qa.valid || pe.valid != qe.valid) return 32;
    if (pa.valid && (pa.slot != qa.slot || pa.delta != qa.delta || pa.inlet != qa.inlet)) return 33;
    if (pe.valid && (pe.slot != qe.slot || pe.delta != qe.delta)) return 34;
    return 0;
}

// cells flagged GENERAL but not FACE: the x and solid-link form (y/z
// predicates dropped, solid mask and mantle bit kept) must give the full
// form's links
template <int I>
int check_xs_one(const Geo3 &g, const Shape &s, int x, int y, int z)
{
    const int64_t c = g.cell(x, y, z);
    const uint8_t fl = g.fl[c];
    if (!(fl & FL_GENERAL) || (fl & FL_FACE)) return 0;
    const Preds p = preds_of(s, x, y, z, fl);
    const Preds q = preds_xs(fl);
    if (p.ylo || p.yhi || p.zlo || p.zhi) return 40;
    const RelLink a = gather_rel<I>(s, p, g.m[c]), b = gather_rel<I>(s, q, g.m[c]);
    if (a.slot != b.slot || a.delta != b.delta || a.inlet != b.inlet) return 41;
    RelLink pa, pe, qa, qe;
    scatter_rel<I>(s, p, g.m[c], pa, pe);
    scatter_rel<I>(s, q, g.m[c], qa, qe);
    if (pa.valid != qa.valid || pe.valid != qe.valid) return 42;
    if (pa.valid && (pa.slot != qa.slot || pa.delta != qa.delta || pa.inlet != qa.inlet)) return 43;
    if (pe.valid && (pe.slot != qe.slot || pe.delta != qe.delta)) return 44;
    return 0;
}

template <int... Is>
int check_xs_all(const Geo3 &g, const Shape &s, int x, int y, int z, std::integer_sequence<int, Is...>)
{
    int r = 0;
    ((r = r ? r : check_xs_one<Is>(g, s, x, y, z)), ...);
    return r;
}

template <int... Is>
int check_xpath_all(const Geo3 &g, const Shape &s, int x, int y, int z, std::integer_sequence<int, Is...>)
{
    int r = 0;
    ((r = r ? r : check_xpath_one<Is>(g, s, x, y, z)), ...);
    return r;
}

template <int... Is>
int check_rel_all(const Geo3 &g, const Shape &s, int x, int y, int z, std::integer_sequence<int, Is...>)
{
    int r = 0;
    ((r = r ? r : check_rel_one<Is>(g, s, x, y, z)), ...);
    return r;
}

}  // namespace

extern "C" int lbmhc_check_relative(int nx, int ny, int nz, const int *face, const uint8_t *solid)
{
    Geo3 g;
    build(g, nx, ny, nz, face, solid);
    const Shape s = shape_of(g);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                if (g.fl[g.cell(x, y, z)] & FL_SOLID) continue;
                int r = check_rel_all(g, s, x, y, z, std::make_integer_sequence<int, Q>{});
                if (!r) r = check_xpath_all(g, s, x, y, z, std::make_integer_sequence<int, Q>{});
                if (!r) r = check_xs_all(g, s, x, y, z, std::make_integer_sequence<int, Q>{});
                if (r) return r;
            }
    return 0;
}
