// rules.h -- per-link streaming/boundary rules of the in-place update.
//
// The boundary kinds are those of the Sec. 2.2 list of arXiv 2508.18202
// (bounce-back walls and ground, a local velocity condition on the inflow
// side, a free-slip sky) on a box, plus a zero-gradient outflow and periodic
// faces.  For a destination link (x, i) the population after streaming is
// taken from a post-collision value (cell, pop), first matching rule wins,
// with s = x - c_i (periodic axes wrapped):
//   BOUNCE   s a building cell, or s outside through a WALL face -> (x, opp(i))
//   MANTLE   s in the mantle region of a cylindrical domain      -> (x, opp(i)) + 6 w_i c_i.u_in
//   INLET    s.x < 0 through the INLET face                      -> (x, opp(i)) + 6 w_i c_i.u_in
//   FREESLIP s.z >= nz through the FREESLIP sky                  -> (x - c_ix [x = nx clamped to
//                                                                   nx-1], y - c_iy, nz-1), zflip(i);
//            MANTLE instead when that reflected source is a mantle cell
//   OUTLET   s.x >= nx through the OUTLET face                   -> (nx-1, s.y, s.z), i
//   STREAM   otherwise                                           -> (s, i)
// The mantle carries the wind by the local velocity condition on the whole
// surface of the cylinder (Sec. 2.2), in the moving-wall form of the inlet.
// pull_src() evaluates this map; push_dsts() is its exact inverse (every
// destination link whose source is a given post-collision value).  Both are
// compiled for the device (kernels) and the host (exhaustive checks).
#pragma once

#include "d3q19.h"

namespace lbmsc {

enum : int { R_STREAM = 0, R_BOUNCE = 1, R_INLET = 2, R_FREESLIP = 3, R_OUTLET = 4, R_REST = 5, R_MANTLE = 6 };

struct Box {
    int nx, ny, nz;
    int face[6];
};

struct Link {
    int x, y, z;   // cell
    int pop;       // population index
    int kind;      // R_*
};

LBM_HD int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Source of destination link (x, i).  smask bit i: the (wrapped) neighbour
// x - c_i lies in the box and is solid; mantle: those neighbours are mantle
// cells (FL_MANTLE).
LBM_HD Link pull_src(const Box &b, int x, int y, int z, int i, uint32_t smask, bool mantle)
{
    if (i == 0) return Link{x, y, z, 0, R_REST};
    int sx = x - cx(i), sy = y - cy(i), sz = z - cz(i);
    if (b.face[0] == FACE_PERIODIC) sx = wrap1(sx, b.nx);
    if (b.face[2] == FACE_PERIODIC) sy = wrap1(sy, b.ny);
    if (b.face[4] == FACE_PERIODIC) sz = wrap1(sz, b.nz);
    const bool inside = sx >= 0 && sx < b.nx && sy >= 0 && sy < b.ny && sz >= 0 && sz < b.nz;
    const bool wall = (sx < 0 && b.face[0] == FACE_WALL) || (sx >= b.nx && b.face[1] == FACE_WALL) ||
                      (sy < 0 && b.face[2] == FACE_WALL) || (sy >= b.ny && b.face[3] == FACE_WALL) ||
                      (sz < 0 && b.face[4] == FACE_WALL) || (sz >= b.nz && b.face[5] == FACE_WALL);
    if (inside && ((smask >> i) & 1u)) return Link{x, y, z, opp(i), mantle ? R_MANTLE : R_BOUNCE};
    if (wall) return Link{x, y, z, opp(i), R_BOUNCE};
    if (sx < 0 && b.face[0] == FACE_INLET) return Link{x, y, z, opp(i), R_INLET};
    if (sz >= b.nz && b.face[5] == FACE_FREESLIP) {
        // the reflected source is the in-plane neighbour x - (c_x, c_y, 0)
        if (mantle && ((smask >> dir_xy(cx(i), cy(i))) & 1u)) return Link{x, y, z, opp(i), R_MANTLE};
        int px = (sx >= b.nx) ? b.nx - 1 : sx;
        return Link{px, sy, b.nz - 1, zflip(i), R_FREESLIP};
    }
    if (sx >= b.nx && b.face[1] == FACE_OUTLET) return Link{b.nx - 1, sy, sz, i, R_OUTLET};
    return Link{sx, sy, sz, i, R_STREAM};
}

// All destination links (cell, slot = population after streaming) whose
// source is the post-collision value (x, k), k != 0, of a fluid cell x.
// Returns how many (0, 1 or 2), in d0 and d1.  smask is x's own solid-link
// mask: the neighbour x + c_k is x - c_opp(k), i.e. bit opp(k).
LBM_HD int push_dsts(const Box &b, int x, int y, int z, int k, uint32_t smask, bool mantle, Link &d0, Link &d1)
{
    int dx = x + cx(k), dy = y + cy(k), dz = z + cz(k);
    if (b.face[0] == FACE_PERIODIC) dx = wrap1(dx, b.nx);
    if (b.face[2] == FACE_PERIODIC) dy = wrap1(dy, b.ny);
    if (b.face[4] == FACE_PERIODIC) dz = wrap1(dz, b.nz);
    const bool inside = dx >= 0 && dx < b.nx && dy >= 0 && dy < b.ny && dz >= 0 && dz < b.nz;
    const bool solid = inside && ((smask >> opp(k)) & 1u);
    const bool wall = (dx < 0 && b.face[0] == FACE_WALL) || (dx >= b.nx && b.face[1] == FACE_WALL) ||
                      (dy < 0 && b.face[2] == FACE_WALL) || (dy >= b.ny && b.face[3] == FACE_WALL) ||
                      (dz < 0 && b.face[4] == FACE_WALL) || (dz >= b.nz && b.face[5] == FACE_WALL);
    Link prim{0, 0, 0, 0, R_STREAM};
    bool has_prim = true;
    if (inside && !solid) {
        prim = Link{dx, dy, dz, k, R_STREAM};
    } else if (solid || wall) {
        prim = Link{x, y, z, opp(k), (solid && mantle) ? R_MANTLE : R_BOUNCE};
    } else if (dx < 0 && b.face[0] == FACE_INLET) {
        prim = Link{x, y, z, opp(k), R_INLET};
    } else if (dz >= b.nz && b.face[5] == FACE_FREESLIP && dx >= 0 && dx < b.nx) {
        // x is in the top layer and c_kz = +1: reflected into (x + c_kx, y + c_ky, nz-1),
        // unless that cell, x - (-c_kx, -c_ky, 0), is a mantle cell
        if (mantle && ((smask >> dir_xy(-cx(k), -cy(k))) & 1u))
            prim = Link{x, y, z, opp(k), R_MANTLE};
        else
            prim = Link{dx, dy, b.nz - 1, zflip(k), R_FREESLIP};
    } else {
        has_prim = false;  // leaves through the outflow or past the sky corner
    }
    // the outflow column also feeds the zero-gradient links of its neighbours
    Link ext{0, 0, 0, 0, R_OUTLET};
    bool has_ext = false;
    if (x == b.nx - 1 && cx(k) == -1 && b.face[1] == FACE_OUTLET) {
        int ty = y + cy(k), tz = z + cz(k);
        if (b.face[2] == FACE_PERIODIC) ty = wrap1(ty, b.ny);
        if (b.face[4] == FACE_PERIODIC) tz = wrap1(tz, b.nz);
        const bool yin = ty >= 0 && ty < b.ny;
        if (yin && tz >= 0 && tz < b.nz) {
            ext = Link{b.nx - 1, ty, tz, k, R_OUTLET};
            has_ext = true;
        } else if (yin && tz >= b.nz && b.face[5] == FACE_FREESLIP) {
            // sky corner: the clamped free-slip source of (nx-1, ty, nz-1)
            ext = Link{b.nx - 1, ty, b.nz - 1, zflip(k), R_FREESLIP};
            has_ext = true;
        }
    }
    if (has_prim) {
        d0 = prim;
        d1 = ext;
    } else {
        d0 = ext;
    }
    return (int)has_prim + (int)has_ext;
}

// FL_NEAR marks cells whose links are not all plain in-box streaming from
// fluid cells (solid or wrapped neighbours, box faces, the outflow column and
// the sky layer, which also write extra links); the kernels take the general
// rule path only for those.  FL_MANTLE marks fluid cells next to the mantle
// region (mask code 2).
// Per-cell flags and mask.  Fluid cell: bit i of m = the (wrapped) neighbour
// x - c_i lies in the box and is solid.  Solid cell: FL_SOLID, no mask.
LBM_HD void cell_flags(const Box &b, const uint8_t *solid, int x, int y, int z, uint8_t &fl, uint32_t &m)
{
    fl = 0;
    m = 0;
    if (solid[((int64_t)z * b.ny + y) * b.nx + x]) {
        fl = FL_SOLID;
        return;
    }
    bool near = (x == b.nx - 1) || (z == b.nz - 1);
    bool general = z == b.nz - 1;
    bool face = z == b.nz - 1;
    for (int i = 1; i < Q; ++i) {
        int sx = x - cx(i), sy = y - cy(i), sz = z - cz(i);
        bool xw = false, yzw = false;
        if (b.face[0] == FACE_PERIODIC && (sx < 0 || sx >= b.nx)) { sx = wrap1(sx, b.nx); xw = true; }
        if (b.face[2] == FACE_PERIODIC && (sy < 0 || sy >= b.ny)) { sy = wrap1(sy, b.ny); yzw = true; }
        if (b.face[4] == FACE_PERIODIC && (sz < 0 || sz >= b.nz)) { sz = wrap1(sz, b.nz); yzw = true; }
        const bool yz_out = sy < 0 || sy >= b.ny || sz < 0 || sz >= b.nz;
        const bool inside = sx >= 0 && sx < b.nx && !yz_out;
        if (!inside || xw || yzw) near = true;
        if (xw || yzw || yz_out) general = true;
        if (yzw || yz_out) face = true;
        const uint8_t kind = inside ? solid[((int64_t)sz * b.ny + sy) * b.nx + sx] : CELL_FLUID;
        if (kind != CELL_FLUID) {
            m |= 1u << i;
            near = true;
            general = true;
            if (kind == CELL_MANTLE) fl |= FL_MANTLE;
        }
    }
    if (near) fl |= FL_NEAR;
    if (near && general) fl |= FL_GENERAL;
    if (face) fl |= FL_FACE;
    if (x == 0) fl |= FL_XLO;
    if (x == b.nx - 1) fl |= FL_XHI;
}


// ---------------------------------------------------------------------------
// The same rules in relative form, for one compile-time direction: the source
// (gather) or destinations (scatter) as a population slot and a cell offset
// from the current cell, chosen by selects on per-cell predicates instead of
// branches.  Equal to pull_src / push_dsts for every link (checked on the
// host), so a wavefront can evaluate them for all of its lanes at once.

struct Preds {
    bool xlo, xhi, ylo, yhi, zlo, zhi;   // cell on the -x, +x, ... face of the box
    bool mantle;                         // solid neighbours are mantle cells (FL_MANTLE)
};

struct Shape {
    int nx, ny, nz;
    int offy, offz;                      // linear offsets of +y and +z neighbours
    int face[6];
};

struct RelLink {
    int slot;      // population slot read or written
    int delta;     // cell offset from the current cell
    bool inlet;    // add the moving-wall momentum of the link
    bool valid;    // the link exists (scatter: a destination)
};

LBM_HD Preds preds_of(const Shape &s, int x, int y, int z, uint8_t fl)
{
    return Preds{x == 0, x == s.nx - 1, y == 0, y == s.ny - 1, z == 0, z == s.nz - 1, (fl & FL_MANTLE) != 0};
}

// A cell without FL_FACE lies strictly inside the box in y and z, so the
// y/z predicates of preds_of() are false for it; this form of the
// predicates lets the compiler drop every y/z face term.
LBM_HD Preds preds_xs(uint8_t fl)
{
    return Preds{(fl & FL_XLO) != 0, (fl & FL_XHI) != 0, false, false, false, false, (fl & FL_MANTLE) != 0};
}

// wrap correction of a periodic axis: moving by -1 from 0, or +1 from n-1
LBM_HD int wrap_corr(bool periodic, bool below, bool above, int span)
{
    return periodic ? (below ? span : (above ? -span : 0)) : 0;
}

template <int I>
LBM_HD RelLink gather_rel(const Shape &s, const Preds &p, uint32_t smask)
{
    constexpr int CX = cx(I), CY = cy(I), CZ = cz(I);
    // source s = x - c leaves the box below/above along each axis
    const bool xb = CX == 1 && p.xlo, xa = CX == -1 && p.xhi;
    const bool yb = CY == 1 && p.ylo, ya = CY == -1 && p.yhi;
    const bool zb = CZ == 1 && p.zlo, za = CZ == -1 && p.zhi;
    const bool px = s.face[0] == FACE_PERIODIC, py = s.face[2] == FACE_PERIODIC, pz = s.face[4] == FACE_PERIODIC;
    const bool outside = (!px && (xb || xa)) || (!py && (yb || ya)) || (!pz && (zb || za));
    const bool wall = (xb && s.face[0] == FACE_WALL) || (xa && s.face[1] == FACE_WALL) ||
                      (yb && s.face[2] == FACE_WALL) || (ya && s.face[3] == FACE_WALL) ||
                      (zb && s.face[4] == FACE_WALL) || (za && s.face[5] == FACE_WALL);
    const bool solid = !outside && ((smask >> I) & 1u);
    const bool bounce = (solid && !p.mantle) || wall;
    const bool mwall = solid && p.mantle;
    const bool face_in = !bounce && !mwall && xb && s.face[0] == FACE_INLET;
    const bool sky = !bounce && !mwall && !face_in && za && s.face[5] == FACE_FREESLIP;
    // the sky's reflected source x - (c_x, c_y, 0) may lie in the mantle
    constexpr int J = CZ == 0 ? 0 : dir_xy(CX, CY);
    const bool sky_mantle = sky && p.mantle && ((smask >> J) & 1u);
    const bool fslip = sky && !sky_mantle;
    const bool inlet = face_in || mwall || sky_mantle;
    const bool outlet = !bounce && !inlet && !fslip && xa && s.face[1] == FACE_OUTLET;
    const int wx = wrap_corr(px, xb, xa, s.nx);
    const int wy = wrap_corr(py, yb, ya, s.ny) * s.offy;
    const int wz = wrap_corr(pz, zb, za, s.nz) * s.offz;
    const int stream_delta = -(CX + CY * s.offy + CZ * s.offz) + wx + wy + wz;
    RelLink r;
    r.valid = true;
    r.inlet = inlet;
    if (bounce || inlet) {
        r.slot = I;
        r.delta = 0;
    } else if (fslip) {
        // (x - c_x [nx clamped to nx-1], y - c_y, nz-1) with c_z mirrored
        const bool clamp = xa && s.face[1] == FACE_OUTLET;
        r.slot = opp(zflip(I));
        r.delta = (clamp ? 0 : -CX + wx) - CY * s.offy + wy;
    } else if (outlet) {
        r.slot = opp(I);
        r.delta = stream_delta - 1;
    } else {
        r.slot = opp(I);
        r.delta = stream_delta;
    }
    return r;
}

// Destinations of the post-collision value of direction K: primary and extra.
template <int K>
LBM_HD void scatter_rel(const Shape &s, const Preds &p, uint32_t smask, RelLink &prim, RelLink &extra)
{
    constexpr int CX = cx(K), CY = cy(K), CZ = cz(K);
    // destination d = x + c leaves the box below/above along each axis
    const bool xb = CX == -1 && p.xlo, xa = CX == 1 && p.xhi;
    const bool yb = CY == -1 && p.ylo, ya = CY == 1 && p.yhi;
    const bool zb = CZ == -1 && p.zlo, za = CZ == 1 && p.zhi;
    const bool px = s.face[0] == FACE_PERIODIC, py = s.face[2] == FACE_PERIODIC, pz = s.face[4] == FACE_PERIODIC;
    const bool outside = (!px && (xb || xa)) || (!py && (yb || ya)) || (!pz && (zb || za));
    const bool wall = (xb && s.face[0] == FACE_WALL) || (xa && s.face[1] == FACE_WALL) ||
                      (yb && s.face[2] == FACE_WALL) || (ya && s.face[3] == FACE_WALL) ||
                      (zb && s.face[4] == FACE_WALL) || (za && s.face[5] == FACE_WALL);
    const bool solid = !outside && ((smask >> opp(K)) & 1u);
    const int wx = wrap_corr(px, xa, xb, s.nx) * -1;
    const int wy = wrap_corr(py, ya, yb, s.ny) * -s.offy;
    const int wz = wrap_corr(pz, za, zb, s.nz) * -s.offz;
    prim.inlet = false;
    prim.valid = true;
    extra.inlet = false;
    extra.valid = false;
    extra.slot = K;
    extra.delta = 0;
    if (!outside && !solid) {
        prim.slot = K;
        prim.delta = CX + CY * s.offy + CZ * s.offz + wx + wy + wz;
    } else if (solid || wall) {
        prim.slot = opp(K);
        prim.delta = 0;
        prim.inlet = solid && p.mantle;
    } else if (xb && s.face[0] == FACE_INLET) {
        prim.slot = opp(K);
        prim.delta = 0;
        prim.inlet = true;
    } else if (za && s.face[5] == FACE_FREESLIP && (px || !(xb || xa))) {
        // reflected into x + (c_x, c_y, 0) = x - c_J, or the mantle there
        constexpr int J = CZ == 0 ? 0 : dir_xy(-CX, -CY);
        if (p.mantle && ((smask >> J) & 1u)) {
            prim.slot = opp(K);
            prim.delta = 0;
            prim.inlet = true;
        } else {
            prim.slot = zflip(K);
            prim.delta = CX + wx + CY * s.offy + wy;
        }
    } else {
        prim.valid = false;
        prim.slot = K;
        prim.delta = 0;
    }
    // the outflow column also feeds the zero-gradient links of its neighbours
    if (CX == -1 && p.xhi && s.face[1] == FACE_OUTLET) {
        const bool tyo = !py && ((CY == -1 && p.ylo) || (CY == 1 && p.yhi));
        const bool tzb = CZ == -1 && p.zlo, tza = CZ == 1 && p.zhi;
        const bool tzo = !pz && (tzb || tza);
        const int ey = wrap_corr(py, CY == 1 && p.yhi, CY == -1 && p.ylo, s.ny) * -s.offy;
        const int ez = wrap_corr(pz, tza, tzb, s.nz) * -s.offz;
        if (!tyo && !tzo) {
            extra.valid = true;
            extra.slot = K;
            extra.delta = CY * s.offy + ey + CZ * s.offz + ez;
        } else if (!tyo && tza && s.face[5] == FACE_FREESLIP) {
            extra.valid = true;
            extra.slot = zflip(K);
            extra.delta = CY * s.offy + ey;
        }
    }
}

// Tile taken by block p of a grid of `grid` blocks (a multiple of 8), with
// blocks dispatched round-robin over 8 XCDs.  mode 0: hardware order (all
// XCDs on one compact front); mode 1: a contiguous range of tiles per XCD
// (neighbouring tiles share an L2).  Both are permutations of 0 .. grid-1.
// (Chunks of 2..16 consecutive tiles per XCD measured 4-8 % slower than
// either on the step kernels; 32 tied the hardware order.)
LBM_HD int tile_order(int p, int grid, int mode)
{
    return mode == 0 ? p : (p & 7) * (grid >> 3) + (p >> 3);
}

// Granlund-Montgomery division by a constant d >= 1 for 0 <= v < 2^31.
struct FastDiv {
    uint32_t m;
    uint32_t s;
};

inline FastDiv make_fastdiv(uint32_t d)
{
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    uint64_t m = ((1ull << (31 + l)) / d) + 1;
    return FastDiv{(uint32_t)m, 31 + l};
}

LBM_HD uint32_t fdiv(uint32_t v, FastDiv f) { return (uint32_t)(((uint64_t)v * f.m) >> f.s); }

}  // namespace lbmsc
