// steps.hip -- launches of the step kernels of one collision model.  The
// build compiles this file once per model (LBM_STEP_MODEL = 0 BGK,
// 1 Smagorinsky, 2 regularised), so the 48 kernel instantiations of each
// model compile in parallel.
#include "device.h"

#ifndef LBM_STEP_MODEL
#error "compile with -DLBM_STEP_MODEL=<0|1|2>"
#endif

namespace lbmsc {

namespace {

constexpr int M = LBM_STEP_MODEL;

template <int BS, int CPT, bool NT>
void step_v(int parity, const Geo *geo, const int32_t *ti, int32_t nt, const StepArgs &a, int32_t *h,
            hipStream_t s)
{
    const dim3 grid(grid_of(nt - a.tile_base)), block(BS);
    if (parity == 0) hipLaunchKernelGGL((k_step<BS, CPT, NT, M, 0>), grid, block, 0, s, geo, ti, nt, a, h);
    else hipLaunchKernelGGL((k_step<BS, CPT, NT, M, 1>), grid, block, 0, s, geo, ti, nt, a, h);
}

// v.nt is a mask: bit 0 non-temporal accesses in even steps, bit 1 in odd steps
template <int BS, int CPT>
void step_n(const Variant &v, int parity, const Geo *geo, const int32_t *ti, int32_t nt, const StepArgs &a,
            int32_t *h, hipStream_t s)
{
    if ((v.nt >> parity) & 1) step_v<BS, CPT, true>(parity, geo, ti, nt, a, h, s);
    else step_v<BS, CPT, false>(parity, geo, ti, nt, a, h, s);
}

template <int BS>
void step_c(const Variant &v, int parity, const Geo *geo, const int32_t *ti, int32_t nt, const StepArgs &a,
            int32_t *h, hipStream_t s)
{
    if (v.cpt == 1) step_n<BS, 1>(v, parity, geo, ti, nt, a, h, s);
    else if (v.cpt == 2) step_n<BS, 2>(v, parity, geo, ti, nt, a, h, s);
    else step_n<BS, 4>(v, parity, geo, ti, nt, a, h, s);
}

}  // namespace

template <>
int launch_step_model<LBM_STEP_MODEL>(const Variant &v, int parity, const Geo *geo, const int32_t *tile_inst,
                                      int32_t n_tiles, const StepArgs &a, int32_t *health, hipStream_t s)
{
    if (v.bs == 64) step_c<64>(v, parity, geo, tile_inst, n_tiles, a, health, s);
    else if (v.bs == 128) step_c<128>(v, parity, geo, tile_inst, n_tiles, a, health, s);
    else if (v.bs == 256) step_c<256>(v, parity, geo, tile_inst, n_tiles, a, health, s);
    else step_c<512>(v, parity, geo, tile_inst, n_tiles, a, health, s);
    return (int)hipGetLastError();
}

}  // namespace lbmsc
