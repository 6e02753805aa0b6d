// rules.h -- per-link streaming/boundary rules of the in-place update.
//
// The boundary kinds are those of the Sec. 2.2 list of arXiv 2508.18202
// (bounce-back walls and ground, a local velocity condition on the inflow
// side, a free-slip sky) on a box, plus a zero-gradient outflow and periodic
// faces.  For a destination link (x, i) the population after streaming is
// taken from a post-collision value (cell, pop), first matching rule wins,
// with s = x - c_i (periodic axes wrapped):
//   BOUNCE   s solid, or s outside through a WALL face      -> (x, opp(i))
//   INLET    s.x < 0 through the INLET face                  -> (x, opp(i)) + 6 w_i c_i.u_in
//   FREESLIP s.z >= nz through the FREESLIP sky              -> (x - c_ix [x = nx clamped to
//                                                               nx-1], y - c_iy, nz-1), zflip(i)
//   OUTLET   s.x >= nx through the OUTLET face               -> (nx-1, s.y, s.z), i
//   STREAM   otherwise                                       -> (s, i)
// pull_src() evaluates this map; push_dsts() is its exact inverse (every
// destination link whose source is a given post-collision value).  Both are
// compiled for the device (kernels) and the host (exhaustive checks).
#pragma once

#include "d3q19.h"

namespace lbmsc {

enum : int { R_STREAM = 0, R_BOUNCE = 1, R_INLET = 2, R_FREESLIP = 3, R_OUTLET = 4, R_REST = 5 };

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
// x - c_i lies in the box and is solid.
LBM_HD Link pull_src(const Box &b, int x, int y, int z, int i, uint32_t smask)
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
    if ((inside && ((smask >> i) & 1u)) || wall) return Link{x, y, z, opp(i), R_BOUNCE};
    if (sx < 0 && b.face[0] == FACE_INLET) return Link{x, y, z, opp(i), R_INLET};
    if (sz >= b.nz && b.face[5] == FACE_FREESLIP) {
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
LBM_HD int push_dsts(const Box &b, int x, int y, int z, int k, uint32_t smask, Link &d0, Link &d1)
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
        prim = Link{x, y, z, opp(k), R_BOUNCE};
    } else if (dx < 0 && b.face[0] == FACE_INLET) {
        prim = Link{x, y, z, opp(k), R_INLET};
    } else if (dz >= b.nz && b.face[5] == FACE_FREESLIP && dx >= 0 && dx < b.nx) {
        // x is in the top layer and c_kz = +1: reflected into (x + c_kx, y + c_ky, nz-1)
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

// Per-cell flags and solid-link mask.  Bit i of the mask: the neighbour
// x - c_i (periodic axes wrapped) is in the box and solid.  FL_NEAR marks
// cells whose links are not all plain in-box streaming from fluid cells
// (solid or wrapped neighbours, box faces, the outflow column and the sky
// layer, which also write extra links); the kernels take the general rule
// path only for those.
LBM_HD void cell_flags(const Box &b, const uint8_t *solid, int x, int y, int z, uint8_t &fl, uint32_t &m)
{
    fl = 0;
    m = 0;
    if (solid[((int64_t)z * b.ny + y) * b.nx + x]) {
        fl = FL_SOLID;
        return;
    }
    bool near = (x == b.nx - 1) || (z == b.nz - 1);
    for (int i = 1; i < Q; ++i) {
        int sx = x - cx(i), sy = y - cy(i), sz = z - cz(i);
        bool wrapped = false;
        if (b.face[0] == FACE_PERIODIC && (sx < 0 || sx >= b.nx)) { sx = wrap1(sx, b.nx); wrapped = true; }
        if (b.face[2] == FACE_PERIODIC && (sy < 0 || sy >= b.ny)) { sy = wrap1(sy, b.ny); wrapped = true; }
        if (b.face[4] == FACE_PERIODIC && (sz < 0 || sz >= b.nz)) { sz = wrap1(sz, b.nz); wrapped = true; }
        const bool inside = sx >= 0 && sx < b.nx && sy >= 0 && sy < b.ny && sz >= 0 && sz < b.nz;
        if (!inside || wrapped) near = true;
        if (inside && solid[((int64_t)sz * b.ny + sy) * b.nx + sx]) {
            m |= 1u << i;
            near = true;
        }
    }
    if (near) fl |= FL_NEAR;
    if (x == 0 && b.face[0] == FACE_INLET) fl |= FL_INLET;
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
