/*
 * lbm_sc.h -- C ABI of the MI355X (gfx950) stochastic-collocation lattice
 * Boltzmann hot path.
 *
 * The method (arXiv 2508.18202):
 *   Sec. 2.3 / 2.4 steps 2-3  collocation nodes Z^(j) and weights a_j
 *                             (lbm_quadrature, lbm_node_params);
 *   Sec. 2.2                  deterministic D3Q19 LBM per node: the update of
 *                             Eq. (deterministicLBE) with the effective
 *                             relaxation time of Eqs. (tauEff, turbVisc), the
 *                             boundary kinds of the Sec. 2.2 list
 *                             (lbm_init_geometry, lbm_collide_stream);
 *   Sec. 2.4 step 6           QoI capture (time-averaged fields, probes);
 *   Eq. (quad_moments)        mean and variance over the nodes (lbm_sc_moments);
 *   (not in the paper)        discrete adjoint of the update for gradients of
 *                             probe QoIs w.r.t. the inflow parameters
 *                             (lbm_adjoint_step).
 *
 * Conventions shared by every call:
 *   - Return value: LBM_OK (0) or a negative LBM_E_* code; lbm_last_error()
 *     returns a thread-local message describing the last failure.
 *   - Every pointer whose name ends in _dev is device memory of the current
 *     HIP device; _host pointers are host memory.  The caller allocates and
 *     frees all device buffers.  The library allocates device memory only
 *     inside an lbm_plan (instance and tile tables, health words, captured
 *     graphs) and frees it in lbm_plan_destroy; besides, it holds one static
 *     8 MiB scratch array per device for lbm_adjoint_step_inplace_noalloc.
 *   - Calls taking a hipStream_t only enqueue work on that stream (they may
 *     copy small host tables synchronously first); device faults surface on a
 *     later call or on lbm_sync / lbm_check_health.
 *   - Lattice: D3Q19 in the canonical order
 *       0 (0,0,0); 1 (+x); 2 (-x); 3 (+y); 4 (-y); 5 (+z); 6 (-z);
 *       7 (+x+y); 8 (-x-y); 9 (+x-y); 10 (-x+y); 11 (+x+z); 12 (-x-z);
 *       13 (+x-z); 14 (-x+z); 15 (+y+z); 16 (-y-z); 17 (+y-z); 18 (-y+z),
 *     lattice units (dx = dt = 1, c_s^2 = 1/3, rho_0 = 1).
 *   - Cells are numbered x fastest: c = (z*ny + y)*nx + x.
 *   - Populations are FP32 holding f_i - w_i, structure of arrays with a
 *     padded plane stride (lbm_population_stride), streamed in place.
 */
#ifndef LBM_SC_H
#define LBM_SC_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LBM_OK = 0,
    LBM_E_INVALID = -1,      /* bad argument, shape, face combination or geometry */
    LBM_E_HIP = -2,          /* a HIP runtime call failed (message has its string) */
    LBM_E_UNSTABLE = -3,     /* an instance produced a non-finite or non-positive density */
    LBM_E_UNSUPPORTED = -4   /* device is not gfx950, or a feature combination is not built */
};

/* Boundary kind of each box face, order -x, +x, -y, +y, -z, +z (Sec. 2.2
 * boundary list on a box: inflow through the -x face, outflow through +x;
 * the paper's cylindrical domain is a box of WALL side faces whose exterior
 * cells carry the mask code of the mantle, see lbm_init_geometry).
 *   WALL      half-way bounce-back (no-slip building walls and ground);
 *   INLET     local velocity condition as moving-wall bounce-back with
 *             rho_w = 1: f_i = f*_opp(i) + 6 w_i c_i.u_in (only on -x);
 *   OUTLET    zero gradient of the post-collision populations (only on +x);
 *   FREESLIP  specular reflection: zero normal velocity, zero normal gradient
 *             of the tangential velocity (only on +z);
 *   PERIODIC  wrap-around (both faces of an axis). */
enum { LBM_WALL = 0, LBM_INLET = 1, LBM_OUTLET = 2, LBM_FREESLIP = 3, LBM_PERIODIC = 4 };

/* Collision models: BGK (Eq. deterministicLBE with an unprojected
 * non-equilibrium part); BGK with the Smagorinsky-Lilly effective relaxation
 * time (Eqs. tauEff, turbVisc; |S| from the local non-equilibrium stress);
 * and the regularised collision of Eq. (deterministicLBE) as printed, with
 * the Smagorinsky tau_eff (cs = 0 gives tau0): equilibrium and
 * non-equilibrium part expanded to third order (coefficients of
 * Eq. hermiteCoeff) in the Hermite polynomials orthogonal on D3Q19, i.e. up
 * to second order plus H_xxy +- H_yzz, H_xzz +- H_xyy, H_yyz +- H_xxz, each
 * term divided by its norm on the velocity set.  The adjoint covers all
 * three models. */
enum { LBM_BGK = 0, LBM_SMAGORINSKY = 1, LBM_RR3 = 2 };

/* Inflow profiles (Sec. 3, log-law wind profile): theta = (speed, phi, z0).
 *   UNIFORM  u_in = speed (cos phi, sin phi, 0);
 *   LOGLAW   u_in(z) = (speed / 0.41) ln((z + 1/2) / z0) (cos phi, sin phi, 0),
 *            speed = friction velocity u*, z0 = roughness length in cells,
 *            z the cell index above the half-way ground;
 *   SERIES   the measured-series inflow of Sec. 3: theta = (zeta1, zeta2, z0),
 *            u_in(z, n) = zeta1 U_H(n) ln((h + z0)/z0) / ln((H + z0)/z0)
 *                         (cos(Theta(n) + zeta2), sin(Theta(n) + zeta2), 0),
 *            h = z + 1/2, H = ref_height; U_H(n), Theta(n) from the hourly
 *            series (see lbm_instance): hour k starts at step ramp + k hour_steps,
 *            the values move from hour k-1's to hour k's over its first
 *            blend_steps steps with weight (1 - cos(pi t / blend_steps)) / 2,
 *            the direction along the shorter arc, and are then held (hour 0
 *            before and during the ramp, the last hour after the series).
 * Every kind is scaled by the ramp factor below. */
enum { LBM_INFLOW_UNIFORM = 0, LBM_INFLOW_LOGLAW = 1, LBM_INFLOW_SERIES = 2 };

/* Collocation rules (Sec. 2.3, Eq. coef_discrete / quad_moments). */
enum { LBM_QUAD_GAUSS_LEGENDRE = 0, LBM_QUAD_SMOLYAK_CC = 1, LBM_QUAD_GAUSS_HERMITE = 2 };

typedef struct lbm_domain {
    int32_t nx, ny, nz;
    int32_t face[6];
} lbm_domain;

/* One deterministic run (one collocation node of one case). */
typedef struct lbm_instance {
    lbm_domain dom;
    const void *geom_dev;    /* geometry buffer filled by lbm_init_geometry */
    int32_t n_probes;        /* probe count given to lbm_init_geometry */
    float *f_dev;            /* 19 * lbm_population_stride(dom) floats */
    int32_t model;           /* LBM_BGK / LBM_SMAGORINSKY / LBM_RR3 (uniform over a plan) */
    float tau0;              /* molecular relaxation time, > 1/2 */
    float cs;                /* Smagorinsky constant C_S */
    int32_t inflow;          /* LBM_INFLOW_* */
    float theta[3];          /* inflow parameters (speed, phi [rad], z0) */
    int32_t ramp;            /* inflow ramp length T_r in steps: u_in is scaled by
                                (1 - cos(pi n / T_r)) / 2 for n < T_r */
    float *qoi_part_dev;     /* [ncells][4] FP32 partial sums of (ux, uy, uz, |u|) or NULL */
    double *qoi_sum_dev;     /* [ncells][4] FP64 window sums, or NULL (both or neither) */
    double *probe_sum_dev;   /* [n_probes] FP64 window sums of u_x at the probes, or NULL */
    /* LBM_INFLOW_SERIES only (ignored otherwise): */
    const float *series_dev; /* [series_len][2] (U_H, Theta [rad]) per hour, device memory
                                owned by the caller, outliving the plan */
    int32_t series_len;      /* >= 1 hours */
    int32_t hour_steps;      /* >= 1 steps per hour */
    int32_t blend_steps;     /* 0 .. hour_steps */
    float ref_height;        /* H > 0 in cells */
} lbm_instance;

typedef struct lbm_plan_opts {
    int64_t avg_begin;         /* QoI window: states f^n with avg_begin < n <= avg_end */
    int64_t avg_end;           /* avg_end <= avg_begin disables accumulation */
    int32_t use_graph;         /* replay step pairs from captured HIP graphs where possible:
                                  outside the QoI window and once every instance's inflow is
                                  constant in time (after the ramp and, for a series, after
                                  the blend into its last hour) */
    int32_t block;             /* threads per workgroup: 64, 128, 256 or 512; 0 = default (256) */
    int32_t cells_per_thread;  /* 1, 2 or 4; 0 = default (1).  A workgroup owns block *
                                  cells_per_thread consecutive cells of one instance */
    int32_t nontemporal;       /* streaming (non-temporal) population loads and stores:
                                  bit 0 in even steps, bit 1 in odd steps */
    int32_t xcd_order;         /* order of the tiles over the 8 XCDs: 0 hardware round
                                  robin, 1 a contiguous range per XCD.  The last three
                                  fields apply only when block != 0; otherwise the
                                  default shape (256, 1, even steps non-temporal, 0) */
} lbm_plan_opts;

typedef struct lbm_plan lbm_plan;

/* ------------------------------------------------------------------ errors */
const char *lbm_last_error(void);
const char *lbm_version(void);

/* ------------------------------------------------------------ collocation
 * lbm_quadrature: nodes [n][dim] (row-major) and probability weights [n] of
 *   LBM_QUAD_GAUSS_LEGENDRE (level = number of points, dim must be 1; xi ~ U(-1,1)),
 *   LBM_QUAD_SMOLYAK_CC (level L >= 0, dim >= 1; nested Clenshaw-Curtis
 *   rules with 1, 3, 5, 9, ... points, combination technique) or
 *   LBM_QUAD_GAUSS_HERMITE (level = points per dimension, dim >= 1; the dense
 *   tensor-product rule for z ~ N(0, 1)^d of Sec. 3, node j = (i_1 .. i_d)
 *   with the last coordinate fastest; at most 65536 nodes).
 *   Returns the node count through *n_out.  With nodes_host == NULL only the
 *   count is returned.  cap = capacity of the output arrays in nodes.
 * lbm_node_params: theta = (base*(1 + rel*xi_1), radians(angle_deg*xi_2), z0)
 *   -- the multiplicative speed perturbation and additive direction
 *   perturbation of Sec. 3 (dim 1: no direction term); with Gaussian nodes,
 *   base 1, rel sigma_1 and angle_deg sigma_2 give zeta_1 ~ N(1, sigma_1^2)
 *   and zeta_2 ~ N(0, sigma_2^2). */
int lbm_quadrature(int32_t kind, int32_t level, int32_t dim, double *nodes_host,
                   double *weights_host, int32_t cap, int32_t *n_out);
int lbm_node_params(const double *xi_host, int32_t dim, double base, double rel,
                    double angle_deg, double z0, float theta_out[3]);

/* --------------------------------------------------------------- geometry
 * Sizes the caller must allocate: the geometry buffer in bytes and the
 * population plane stride in floats (f_dev holds 19 planes).
 * lbm_init_geometry validates the case, builds per-cell flags and solid-link
 * masks on the device from solid_host ([nz][ny][nx] bytes: 0 fluid,
 * 1 building, 2 mantle region) and the sorted probe list (probe_host,
 * n_probes distinct fluid cell indices, may be NULL when n_probes == 0), and
 * sets f_dev to the rest equilibrium (f_i - w_i = 0).
 * Building cells are no-slip bounce-back walls.  Mantle cells are the
 * exterior of a cylindrical domain (Secs. 2.2 and 3): every link that
 * crosses into them takes the local velocity condition of the wind, the
 * moving-wall bounce-back with the instance's inflow u_in(z, n), also where
 * the free-slip reflection of a top-layer link would come from a mantle cell.
 * A cylinder of radius R about the box centre is the mantle code on every
 * column whose centre lies farther than R from the axis, with WALL side
 * faces (never reached) and typically a free-slip sky.
 * Rejected (LBM_E_INVALID): face kinds outside the list above, unpaired
 * periodic faces, mask codes above 2, building cells in the top layer under a
 * free-slip sky, solid cells in the last two x columns or an odd nx with an
 * outlet, a fluid cell bordering a building and a mantle cell at once, a box
 * whose 19 population planes exceed 4 GiB (the kernels use 32-bit byte
 * offsets within an instance: at most about 56.5 M cells per instance; a
 * batch holds any number of instances). */
int64_t lbm_geometry_bytes(const lbm_domain *dom, int32_t n_probes);
int64_t lbm_population_stride(const lbm_domain *dom);
int lbm_init_geometry(const lbm_domain *dom, const uint8_t *solid_host,
                      const int32_t *probe_host, int32_t n_probes, void *geom_dev,
                      float *f_dev, hipStream_t stream);

/* ----------------------------------------------------------- batched plan
 * A plan binds a batch of instances (any sizes, one collision model) that
 * advance together, one launch per time step over a flattened tile list.
 * lbm_plan_create copies the instance table; device buffers stay owned by
 * the caller and must outlive the plan.  The step counter starts at 0. */
int lbm_plan_create(const lbm_instance *inst, int32_t n_inst, const lbm_plan_opts *opts,
                    lbm_plan **plan_out);
void lbm_plan_destroy(lbm_plan *plan);
int64_t lbm_plan_step(const lbm_plan *plan);
int lbm_plan_set_step(lbm_plan *plan, int64_t step);   /* even steps only (natural layout) */
/* Instance blocks for the device's memory-side cache (not in the paper; a
 * schedule of Sec. 2.4's independent runs): consecutive instances are
 * grouped while their state (populations, per-cell flags and solid-link
 * masks) fits `bytes`, and lbm_collide_stream advances stretches of plain
 * steps (captured graphs) one block at a time through the whole stretch,
 * and ramp, blend and QoI-window steps one block at a time in chunks (ending
 * where the accumulation starts or stops, at the window's last state and
 * every 64 accumulated states, where the batch-wide flush falls), so that a
 * block's state stays in the cache from step to step.  The results are
 * bit-identical to the batched order: the instances are independent and
 * each cell's sums keep their order.  Recording runs
 * (lbm_collide_stream_record, lbm_collide_stream_record_qoi) go one block at
 * a time in chunks as well; records are per instance, so each instance
 * writes the same records in the same order.  Used when there are at least
 * two blocks and every instance fits; default 224 MiB; 0 turns it off.
 * Synchronises the device.  LBM_E_INVALID for a negative size. */
int lbm_plan_set_cache_block(lbm_plan *plan, int64_t bytes);
/* Number of instance blocks in use (0: plain stretches advance the whole
 * batch per step); -1 for a NULL plan. */
int32_t lbm_plan_cache_blocks(const lbm_plan *plan);
int lbm_plan_set_theta(lbm_plan *plan, int32_t inst, const float theta[3]);
int lbm_plan_reset_qoi(lbm_plan *plan, hipStream_t stream);     /* zero QoI sums and health */
int lbm_sync(lbm_plan *plan, hipStream_t stream);
/* Synchronises stream; returns LBM_E_UNSTABLE and the first bad instance
 * index through *bad_inst if any instance saw rho <= 0 or a non-finite rho. */
int lbm_check_health(lbm_plan *plan, hipStream_t stream, int32_t *bad_inst);
/* Launch shape of the step kernels: variant_out = {block, cells_per_thread,
 * nontemporal, xcd_order}.  lbm_plan_autotune times step pairs of every shape on the
 * batch in the order plain stretches run (with instance blocks, each block
 * through its own pairs in turn; populations, step counter and QoI sums are
 * restored afterwards), keeps the fastest and caches it in the JSON file named
 * by LBMSC_TUNE_CACHE (default ~/.cache/lbmsc_tune.json), keyed by
 * architecture, model, instance count, instance-block count and box sizes.
 * Call it after lbm_plan_set_cache_block when both are used. */
int lbm_plan_variant(const lbm_plan *plan, int32_t variant_out[4]);
int lbm_plan_autotune(lbm_plan *plan, hipStream_t stream, int32_t variant_out[4]);

/* ----------------------------------------------------- collide and stream
 * Advance every instance of the plan by n_steps time steps of Eq.
 * (deterministicLBE): per cell read 19 populations, form rho, u
 * (+ Smagorinsky tau_eff), relax, and write the 19 populations to their
 * streamed slots, boundary rules resolved per link.  The in-place AA pattern
 * alternates an even step (own cell, swapped slots) and an odd step
 * (gather from neighbours, scatter to neighbours).  QoIs of every state f^n
 * in the plan's window are accumulated: qoi sums of (ux, uy, uz, |u|) and
 * probe sums of u_x (solid cells contribute nothing).  The 19 slots of a
 * solid cell carry no state: no rule reads them, the even step swaps them
 * pairwise without collision and the odd step writes zero into them (zero
 * stays zero after lbm_init_geometry); runs of 32 consecutive solid cells
 * are not touched at all. */
int lbm_collide_stream(lbm_plan *plan, int32_t n_steps, hipStream_t stream);

/* Same, and also record the state of every step n for the adjoint sweep
 * (recording runs do not add to the QoI sums):
 * record_kind 1 saves (rho, u) as [slot][ncells][4] floats (BGK adjoint),
 * record_kind 2 saves f - w as [slot][19][stride] floats (any model),
 * record_kind 3 saves what the regularised adjoint needs, (rho, u_x, u_y,
 * u_z, the non-equilibrium stress xx, yy, zz, xy, xz, yz, and the six
 * third-order Hermite moments of f - w in the order of the regularised
 * collision's basis), as [slot][16][stride] floats (regularised model only;
 * LBM_E_INVALID otherwise); slot = n % n_slots; rec_dev[i] is instance i's
 * buffer.  Records are written with non-temporal stores. */
int lbm_collide_stream_record(lbm_plan *plan, int32_t n_steps, int32_t record_kind,
                              float *const *rec_dev_host, int32_t n_slots, hipStream_t stream);
/* The same recording run that also adds to the QoI sums like
 * lbm_collide_stream (not in the paper): the forward run of an adjoint sweep
 * records its last steps itself (slot n % n_slots, as above), so that the
 * sweep re-runs none of the segments those records cover; with n_slots at
 * least the run length it keeps every step.  Memory: n_slots records per
 * instance (16, 76 or 64 B per cell and step for kinds 1, 2, 3).  Same
 * arguments and errors as lbm_collide_stream_record. */
int lbm_collide_stream_record_qoi(lbm_plan *plan, int32_t n_steps, int32_t record_kind,
                                  float *const *rec_dev_host, int32_t n_slots, hipStream_t stream);

/* u_x, u_y, u_z, |u| of the current state of instance i ([ncells][4] floats;
 * solid cells 0), and the natural-layout populations f - w ([19][stride]). */
int lbm_read_fields(lbm_plan *plan, int32_t inst, float *out_dev, hipStream_t stream);
int lbm_read_populations(lbm_plan *plan, int32_t inst, float *out_dev, hipStream_t stream);
/* Window averages: out[c][k] = qoi_sum[c][k] / count and probe_sum / count
 * as floats (probe_out may be NULL). */
int lbm_qoi_average(lbm_plan *plan, int32_t inst, float *out_dev, float *probe_out_dev,
                    hipStream_t stream);

/* ---------------------------------------------------------------- moments
 * Eq. (quad_moments) per element e < n_elems of the node-major input
 * q_dev[n_nodes][n_elems] (FP32):
 *   mean[e] = sum_j w_j q[j][e],  var[e] = sum_j w_j (q[j][e] - mean[e])^2,
 * both accumulated in FP64 (two passes over the nodes held in registers for
 * n_nodes <= 32, a shifted single pass otherwise).  Weights may be negative
 * (Smolyak), so var may come out negative; the count of negative variances
 * is added atomically to *n_negative_dev (device, caller-zeroed; may be NULL).
 * Rejected: n_nodes < 1 or > 256, |sum w - 1| > 1e-12. */
int lbm_sc_moments(const float *q_dev, const double *w_host, int32_t n_nodes, int64_t n_elems,
                   double *mean_dev, double *var_dev, unsigned long long *n_negative_dev,
                   hipStream_t stream);

/* ------------------------------------------------------- gPC coefficients
 * Sec. 2.3: the expansion of a QoI in polynomials orthonormal under the
 * input distribution, coefficients by projection with the collocation rule,
 * c_alpha = sum_j a_j Q_j Phi_alpha(Z^(j)); for Gaussian inputs the
 * probabilists' Hermite polynomials, Phi_alpha(z) = prod_k He_{alpha_k}(z_k)
 * / sqrt(alpha_k!).  Mean c_0, variance sum_{alpha != 0} c_alpha^2.
 * lbm_gpc_basis (host): the P multi-indices of total degree <= order in dim
 *   variables (graded: degree 0, 1, ...; within a degree the first
 *   variable's power descending) into alpha_out[P][dim], and
 *   phi_out[j][p] = Phi_alpha_p(nodes[j]) for the n_nodes nodes [n][dim],
 *   or, with the collocation weights given (weights_host[n], may be NULL),
 *   the weighted basis a_j Phi_alpha_p(nodes[j]) that lbm_gpc_coefficients
 *   takes.  P is returned through *n_basis; with phi_out == NULL only the
 *   count.  cap = capacity of phi_out in rows of P values.
 * lbm_gpc_coefficients (device, FP64): coef[p][e] = sum_j wphi[j][p] q[j][e]
 *   for the node-major FP32 input q_dev[n_nodes][n_elems] and the weighted
 *   basis wphi_dev[n_nodes][n_basis] = a_j Phi_p(Z^(j)) (device, caller
 *   owned); coef_dev [n_basis][n_elems].  Optional (may be NULL), with basis
 *   row 0 the constant polynomial as lbm_gpc_basis orders it:
 *   var_dev[e] = sum_{p >= 1} coef[p][e]^2 and the 95 % band
 *   band_dev[0][e] = coef[0][e] - 1.96 sqrt(var), band_dev[1][e] = coef[0][e] + 1.96 sqrt(var).
 *   Rejected: n_nodes < 1, n_basis < 1 or > 64, n_elems < 0. */
int lbm_gpc_basis(const double *nodes_host, const double *weights_host, int32_t n_nodes, int32_t dim,
                  int32_t order, double *phi_out, int32_t *alpha_out, int32_t cap, int32_t *n_basis);
int lbm_gpc_coefficients(const float *q_dev, const double *wphi_dev, int32_t n_nodes, int32_t n_basis,
                         int64_t n_elems, double *coef_dev, double *var_dev, double *band_dev,
                         hipStream_t stream);

/* ---------------------------------------------------------------- adjoint
 * Discrete adjoint of one step n -> n+1 for every instance of the plan
 * (not in the paper):
 *   lam^n = (dC/df |f^n)^T P^T lam^{n+1} + dj_n/df^n,
 *   dJdtheta[i][k] += sum over inlet and mantle links (x,q) of
 *                     lam^{n+1}_q(x) * 6 w_q c_q . d u_in / d theta_k * r(n)   (FP64),
 * with P the streaming/boundary map, C the local collision, and
 * j_n = sum_p pw[p] * u_x(f^n, p) / count for n inside the QoI window
 * (count = avg_end - avg_begin).  Buffers per instance (device pointers in
 * host arrays of length n_inst): lam_in (lam^{n+1}) and lam_out (lam^n),
 * [19][stride] floats; rec, the state recorded by
 * lbm_collide_stream_record for step n (kind 1 or 2 for BGK, 2 for the
 * Smagorinsky model, 2 or 3 for the regularised model; slot n % n_slots);
 * pw, [n_probes] FP64 probe weights or NULL;
 * dJdtheta_dev, [n_inst][3] FP64 accumulated in place, in a fixed summation
 * order (per-tile partials in a plan-owned buffer, then one sum per
 * instance), so repeated sweeps give identical gradients.  lam^n of solid
 * cells is written as zero.  The regularised model's transposed collision
 * is the chain rule through f_eq3, the regularisation projector and the
 * Smagorinsky tau_eff, in Hermite moments.  Rejected (LBM_E_INVALID): a
 * missing buffer, lam_in and lam_out the same buffer (the step reads
 * neighbours' lam^{n+1} while writing lam^n), a record kind the plan's
 * model does not take, n_slots < 1 or a negative step. */
int lbm_adjoint_step(lbm_plan *plan, int64_t step, float *const *lam_in_host,
                     float *const *lam_out_host, float *const *rec_host, int32_t record_kind,
                     int32_t n_slots, const double *const *pw_host, double *dJdtheta_dev,
                     hipStream_t stream);
/* The same adjoint step on one lambda buffer per instance, updated in place
 * ([19][stride] floats, device; lam_host a host array of n_inst pointers):
 * the transpose of the in-place streaming of the populations.  lam^{n+1}
 * is read in the storage layout the populations have after step n (natural
 * for even n + 1, as written by lbm_adjoint_init), and lam^n is left in the
 * layout they have after step n - 1: the adjoint of an odd step reads each
 * cell's lambda at the slots that step scattered to and writes it to the
 * slots it gathered from (the outflow column's zero-gradient links handed
 * to the upstream neighbour within the wavefront, the column's extra
 * destinations zeroed); the adjoint of an even step swaps each cell's own
 * slots back.  Every slot is read and written by one thread, so no other
 * buffer is needed.  The gradient and everything else as lbm_adjoint_step;
 * calls must run n = N-1, N-2, ..., in order, on one buffer. */
int lbm_adjoint_step_inplace(lbm_plan *plan, int64_t step, float *const *lam_host, float *const *rec_host,
                             int32_t record_kind, int32_t n_slots, const double *const *pw_host,
                             double *dJdtheta_dev, hipStream_t stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * step as lbm_adjoint_step_inplace, same arguments and results, but it calls
 * no hipMalloc, hipFree or other allocating routine.  Its scratch (the three
 * tables of buffer pointers, copied from the host arrays with stream-ordered
 * copies, and one FP64 gradient partial triple per tile) lives in a
 * library-owned device array of 8 MiB per device, held until the process
 * ends: 3 * align256(8 n_inst) + 24 n_tiles bytes must fit (about 340 000
 * tiles, e.g. 44 M cells at 128 cells per tile), otherwise LBM_E_INVALID.
 * Every call on one device shares that array and leaves its contents there;
 * every partial is rewritten by each call, so nothing needs clearing.  Calls
 * that may overlap on one device (several streams, several host threads, or
 * several plans without ordering between them) race on the array: the
 * caller orders them, e.g. on one stream. */
int lbm_adjoint_step_inplace_noalloc(lbm_plan *plan, int64_t step, float *const *lam_host,
                                     float *const *rec_host, int32_t record_kind, int32_t n_slots,
                                     const double *const *pw_host, double *dJdtheta_dev,
                                     hipStream_t stream);
/* lam^N = dj_N/df^N from the plan's current (even) state N; lam_out as above. */
int lbm_adjoint_init(lbm_plan *plan, float *const *lam_out_host, const double *const *pw_host,
                     hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* LBM_SC_H */
