// adjoint.hip -- launches of the adjoint step kernels (BGK, Smagorinsky and
// the regularised collision, every launch shape); the kernels are in device.h.
#include "device.h"

namespace lbmsc {

namespace {

// record kinds per model: BGK 1 or 2, Smagorinsky 2, regularised 2 or 3
template <int BS, int CPT, int M, int MODE>
void adjoint_r(const dim3 &grid, const dim3 &block, const Geo *geo, const int32_t *ti, int32_t nt, int32_t xr,
               const AdjArgs &a, hipStream_t s)
{
    if constexpr (M == 0) {
        if (a.record == 1) hipLaunchKernelGGL((k_adjoint<BS, CPT, M, MODE, 1>), grid, block, 0, s, geo, ti, nt, xr, a);
        else hipLaunchKernelGGL((k_adjoint<BS, CPT, M, MODE, 2>), grid, block, 0, s, geo, ti, nt, xr, a);
    } else if constexpr (M == 2) {
        if (a.record == 3) hipLaunchKernelGGL((k_adjoint<BS, CPT, M, MODE, 3>), grid, block, 0, s, geo, ti, nt, xr, a);
        else hipLaunchKernelGGL((k_adjoint<BS, CPT, M, MODE, 2>), grid, block, 0, s, geo, ti, nt, xr, a);
    } else {
        hipLaunchKernelGGL((k_adjoint<BS, CPT, M, MODE, 2>), grid, block, 0, s, geo, ti, nt, xr, a);
    }
}

template <int BS, int MODE>
void adjoint_m(const Variant &v, const Geo *geo, const int32_t *ti, int32_t nt, const AdjArgs &a, hipStream_t s)
{
    const dim3 grid(grid_of(nt)), block(BS);
    const int32_t xr = v.xcd;
#define LBM_ADJ(C, M) adjoint_r<BS, C, M, MODE>(grid, block, geo, ti, nt, xr, a, s)
    // the adjoint runs a whole tile per workgroup: one cell per thread up
    // to 512 threads, then 2 or 4 cells per thread
    if constexpr (BS < 512) {
        if (a.model == 0) LBM_ADJ(1, 0);
        else if (a.model == 1) LBM_ADJ(1, 1);
        else LBM_ADJ(1, 2);
    } else {
        if (a.model == 0) {
            if (v.cpt == 1) LBM_ADJ(1, 0);
            else if (v.cpt == 2) LBM_ADJ(2, 0);
            else LBM_ADJ(4, 0);
        } else if (a.model == 1) {
            if (v.cpt == 1) LBM_ADJ(1, 1);
            else if (v.cpt == 2) LBM_ADJ(2, 1);
            else LBM_ADJ(4, 1);
        } else {
            if (v.cpt == 1) LBM_ADJ(1, 2);
            else if (v.cpt == 2) LBM_ADJ(2, 2);
            else LBM_ADJ(4, 2);
        }
    }
#undef LBM_ADJ
}

template <int BS>
void adjoint_c(const Variant &v, const Geo *geo, const int32_t *ti, int32_t nt, const AdjArgs &a, int mode,
               hipStream_t s)
{
    if (mode == 0) adjoint_m<BS, 0>(v, geo, ti, nt, a, s);
    else if (mode == 1) adjoint_m<BS, 1>(v, geo, ti, nt, a, s);
    else adjoint_m<BS, 2>(v, geo, ti, nt, a, s);
}

}  // namespace

int launch_adjoint(const Variant &v, const Geo *geo, const int32_t *tile_inst, int32_t n_tiles, const AdjArgs &a,
                   int mode, hipStream_t s)
{
    if (n_tiles <= 0) return 0;
    if (!variant_ok(v) || mode < 0 || mode > 2 || (v.bs < 512 && v.cpt != 1)) return -1;
    if (v.bs == 64) adjoint_c<64>(v, geo, tile_inst, n_tiles, a, mode, s);
    else if (v.bs == 128) adjoint_c<128>(v, geo, tile_inst, n_tiles, a, mode, s);
    else if (v.bs == 256) adjoint_c<256>(v, geo, tile_inst, n_tiles, a, mode, s);
    else adjoint_c<512>(v, geo, tile_inst, n_tiles, a, mode, s);
    return (int)hipGetLastError();
}

}  // namespace lbmsc
