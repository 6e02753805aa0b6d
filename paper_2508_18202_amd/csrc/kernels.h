// kernels.h -- device-side instance table and kernel launch entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rules.h"

namespace lbmsc {

// One instance (one collocation node of one case) as the kernels see it.
struct Geo {
    float *f;                  // populations f - w, [19][qs]
    const uint8_t *flags;      // [ncells] FL_* bits
    const uint32_t *smask;     // [ncells] bit i: neighbour x - c_i is solid
    const int32_t *probes;     // [n_probes] sorted cell indices
    float *qpart;              // [ncells][4] FP32 window partial sums or null
    double *qsum;              // [ncells][4] FP64 window sums or null
    double *psum;              // [n_probes] FP64 probe sums or null
    int64_t qs;                // population plane stride in floats
    int32_t ncells;
    int32_t n_probes;
    Box box;
    int32_t offy, offz;        // linear offsets of +y and +z neighbours
    FastDiv dx, dxy;           // division by nx and nx*ny
    int32_t tile0;             // first tile of this instance in the flattened list
    int32_t inflow;            // 0 uniform, 1 log-law, 2 measured series
    float tau0;
    float kcs;                 // 18 sqrt(2) Cs^2
    float speed, cphi, sphi, phi, z0;
    int32_t ramp;
    int32_t pad_;
    // measured series: [series_len][2] (U_H, Theta), hour length, blend length,
    // 1 / ln((H + z0) / z0) of the normalised log profile
    const float *series;
    int32_t series_len, hour_steps, blend_steps;
    float inv_log_h;
    float dlog_h;              // d ln((H + z0) / z0) / d z0 = 1 / (H + z0) - 1 / z0
};

// Launch arguments that change from step to step.
// values per cell of a record of kind 3 (the regularised adjoint's state:
// rho, u, the non-equilibrium stress, the six third-order Hermite moments)
constexpr int RR3_REC = 16;

struct StepArgs {
    int64_t step;              // time index n of the state being collided
    int32_t accumulate;        // add this state's QoIs to the window sums
    int32_t record;            // 0 none, 1 (rho,u), 2 populations, 3 regularised state
    int32_t xcd_remap;         // tile order over the XCDs (set from the variant, see tile_of)
    int32_t tile_base;         // first tile of this launch (the launch covers tile_base .. n_tiles - 1)
    float *const *rec;         // device array [n_inst] of record buffer bases
    int64_t rec_slot;          // slot index n % n_slots
    const uint64_t *tinfo;     // per tile, two words (see launch_tile_info)
};

// Launch shape of the step kernels: threads per workgroup, cells per
// thread (a tile holds bs * cpt consecutive cells) and non-temporal
// population loads/stores (mask: bit 0 even steps, bit 1 odd steps).
struct Variant {
    int bs;
    int cpt;
    int nt;
    int xcd;                   // tile order: 0 hardware round robin, 1 contiguous per XCD
    int tile() const { return bs * cpt; }
};

bool variant_ok(const Variant &v);
// step-kernel launches of one collision model (0 BGK, 1 Smagorinsky,
// 2 regularised), each compiled in its own translation unit
template <int MODEL>
int launch_step_model(const Variant &v, int parity, const Geo *geo, const int32_t *tile_inst, int32_t n_tiles,
                      const StepArgs &a, int32_t *health, hipStream_t s);
template <>
int launch_step_model<0>(const Variant &, int, const Geo *, const int32_t *, int32_t, const StepArgs &, int32_t *,
                         hipStream_t);
template <>
int launch_step_model<1>(const Variant &, int, const Geo *, const int32_t *, int32_t, const StepArgs &, int32_t *,
                         hipStream_t);
template <>
int launch_step_model<2>(const Variant &, int, const Geo *, const int32_t *, int32_t, const StepArgs &, int32_t *,
                         hipStream_t);
int launch_step(const Variant &v, int model, int parity, const Geo *geo, const int32_t *tile_inst,
                int32_t n_tiles, const StepArgs &a, int32_t *health, hipStream_t s);
int launch_init_geometry(const Box &b, const uint8_t *solid, uint8_t *flags, uint32_t *smask,
                         const int32_t *probes, int32_t n_probes, hipStream_t s);
int launch_capture(int tcells, int parity, const Geo *geo, const int32_t *tile_inst, int32_t n_tiles,
                   int64_t step, int32_t *health, hipStream_t s);
int launch_flush(int tcells, const Geo *geo, const int32_t *tile_inst, int32_t n_tiles, hipStream_t s);
// Per-tile words for tiles of tcells <= 2048 cells, out[2 t] and out[2 t + 1]:
//   dead  bit l set = cells [32 l, 32 l + 32) of the tile are all solid or past
//         the end (one 128-byte line of every plane); the step kernels skip them;
//   class bits 2w, 2w+1 = rule class of the wavefront of cells [64 w, 64 w + 64):
//         0 no fluid cell with FL_NEAR, 1 some FL_NEAR but no FL_GENERAL, 2 some
//         FL_GENERAL but no FL_FACE, 3 some FL_FACE (fluid cells only).
int launch_tile_info(int tcells, const Geo *geo, const int32_t *tile_inst, int32_t n_tiles, uint64_t *out,
                     hipStream_t s);
int launch_fields(int parity, const Geo *geo, int32_t inst, const Geo &g, int64_t step,
                  float *out, int32_t mode, hipStream_t s);
int launch_average(const Geo &g, double inv_count, float *out, float *pout, hipStream_t s);
int launch_zero_qoi(const Geo &g, hipStream_t s);
// coef[p][e] = sum_j wphi[j][p] q[j][e] (FP64), n_basis <= 64; optional
// var = sum_{p >= 1} coef^2 and band = coef[0] -+ 1.96 sqrt(var)
int launch_gpc(const float *q, const double *wphi, int32_t nq, int32_t nb, int64_t n, double *coef, double *var,
               double *band, hipStream_t s);
int launch_moments(const float *q, const double *w, int32_t nq, int64_t n, double *mean,
                   double *var, unsigned long long *nneg, hipStream_t s);

struct AdjArgs {
    int64_t step;
    int32_t model;
    int32_t record;            // 1 (rho,u), 2 populations or 3 regularised state
    int32_t in_window;         // the objective has a term at this step
    double inv_count;          // 1 / (avg_end - avg_begin)
    float *const *lam_in;      // device arrays [n_inst]
    float *const *lam_out;
    float *const *rec;         // device array [n_inst] of record buffer bases
    int64_t rec_slot;          // slot index n % n_slots
    const double *const *pw;   // [n_inst] probe weights (entries may be null)
    double *grad;              // [n_inst][3]
    double *part;              // [n_tiles][3] per-tile gradient partials of this step
    const uint64_t *tinfo;     // per tile, two words (see launch_tile_info)
};

// mode 0: lam_in -> lam_out, both in the natural layout; mode 1 / 2: one
// buffer (lam_in == lam_out) updated in place, adjoint of an odd / even step
int launch_adjoint(const Variant &v, const Geo *geo, const int32_t *tile_inst, int32_t n_tiles,
                   const AdjArgs &a, int mode, hipStream_t s);
// grad[i][k] += sum over instance i's tiles of part[tile][k], in a fixed order
int launch_grad_reduce(int tile_cells, const Geo *geo_h, int32_t n_inst, const Geo *geo, const double *part,
                       double *grad, hipStream_t s);
int launch_adjoint_init(int tcells, const Geo *geo, const int32_t *tile_inst, int32_t n_tiles,
                        const AdjArgs &a, hipStream_t s);

}  // namespace lbmsc
