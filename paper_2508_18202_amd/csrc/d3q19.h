// d3q19.h -- D3Q19 velocity set for the gfx950 kernels and the host checker.
//
// The velocity set of Fig. 1 (arXiv 2508.18202): one rest velocity, six face
// neighbours, twelve edge neighbours; weights 1/3, 1/18, 1/36; c_s^2 = 1/3.
// Canonical order: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 = edge pairs,
// each odd index followed by its opposite.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define LBM_HD __host__ __device__ __forceinline__

namespace lbmsc {

constexpr int Q = 19;

LBM_HD constexpr int cx(int i)
{
    constexpr int v[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return v[i];
}
LBM_HD constexpr int cy(int i)
{
    constexpr int v[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return v[i];
}
LBM_HD constexpr int cz(int i)
{
    constexpr int v[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return v[i];
}
// opposite direction: pairs (1,2), (3,4), ..., (17,18)
LBM_HD constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
// same velocity with c_z mirrored (specular reflection at a z = const plane)
LBM_HD constexpr int zflip(int i)
{
    constexpr int v[Q] = {0, 1, 2, 3, 4, 6, 5, 7, 8, 9, 10, 13, 14, 11, 12, 17, 18, 15, 16};
    return v[i];
}
// index of the axis direction (x, y, 0) for at most one non-zero component
// (0 for (0, 0, 0)): the in-plane part of a link with c_z != 0
LBM_HD constexpr int dir_xy(int x, int y) { return x == 1 ? 1 : (x == -1 ? 2 : (y == 1 ? 3 : (y == -1 ? 4 : 0))); }
LBM_HD constexpr float wgt(int i) { return i == 0 ? 1.0f / 3.0f : (i <= 6 ? 1.0f / 18.0f : 1.0f / 36.0f); }
LBM_HD constexpr double wgt_d(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

// face kinds (ABI values)
enum : int { FACE_WALL = 0, FACE_INLET = 1, FACE_OUTLET = 2, FACE_FREESLIP = 3, FACE_PERIODIC = 4 };

// per-cell flag bits
//   SOLID    solid cell
//   NEAR     some link of the cell is not plain in-box streaming
//   PROBE    probe cell
//   FACE     some link of the cell crosses a y or z face of the box (wrapped
//            or not) or the sky
//   GENERAL  NEAR for a reason other than being in the x = 0 or x = nx-1
//            column of non-periodic x faces (solid neighbour, FACE, x wrap)
//   XLO/XHI  x = 0 / x = nx-1
//   MANTLE   fluid cell whose solid neighbours belong to the mantle region
//            of a cylindrical domain (all of them: a cell may not border a
//            building and the mantle at once)
enum : uint8_t {
    FL_SOLID = 1, FL_NEAR = 2, FL_PROBE = 4, FL_FACE = 8, FL_GENERAL = 16, FL_XLO = 32, FL_XHI = 64,
    FL_MANTLE = 128
};

// solid-mask codes (ABI values): fluid, building, mantle region
enum : uint8_t { CELL_FLUID = 0, CELL_BUILDING = 1, CELL_MANTLE = 2 };

}  // namespace lbmsc
