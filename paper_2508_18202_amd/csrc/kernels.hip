// kernels.hip -- gfx950 kernels other than the step and adjoint kernels
// (captures, QoI flushes and averages, field read-out, geometry, moments,
// adjoint initialisation and gradient reduction) and the launch dispatch.
#include "device.h"

namespace lbmsc {

namespace {

// QoIs of the current state f^n without advancing it.
template <int PARITY>
__global__ __launch_bounds__(1024) void k_capture(const Geo *__restrict__ geo, const int32_t *__restrict__ tile_inst,
                                                 int32_t n_tiles, int64_t step, int32_t *__restrict__ health)
{
    const int tile = xcd_tile();
    if (tile >= n_tiles) return;
    const int ii = __builtin_amdgcn_readfirstlane(tile_inst[tile]);
    const Geo &G = geo[ii];
    const int32_t lc = (tile - G.tile0) * (int32_t)blockDim.x + (int32_t)threadIdx.x;
    if (lc >= G.ncells) return;
    const uint32_t c = (uint32_t)lc;
    const uint8_t fl = gp(G.flags)[c];
    if (fl & FL_SOLID) return;
    int x = 0, y = 0, z = 0;
    coords(G, c, x, y, z);
    float g[Q];
    load_state<PARITY>(G, c, fl, x, y, z, step, g);
    const Macro m = macro_of(g);
    if (!(m.rho > 0.0f) || !isfinite(m.rho)) atomicOr(health + ii, 1);
    accumulate_qoi(G, c, fl, m);
}

__global__ __launch_bounds__(1024) void k_flush(const Geo *__restrict__ geo, const int32_t *__restrict__ tile_inst,
                                               int32_t n_tiles)
{
    const int tile = xcd_tile();
    if (tile >= n_tiles) return;
    const int ii = __builtin_amdgcn_readfirstlane(tile_inst[tile]);
    const Geo &G = geo[ii];
    if (!G.qpart) return;
    const int32_t lc = (tile - G.tile0) * (int32_t)blockDim.x + (int32_t)threadIdx.x;
    if (lc >= G.ncells) return;
    float4 *p = reinterpret_cast<float4 *>(G.qpart) + lc;
    const float4 v = *p;
    double *s = G.qsum + 4 * (size_t)lc;
    s[0] += v.x;
    s[1] += v.y;
    s[2] += v.z;
    s[3] += v.w;
    *p = make_float4(0.f, 0.f, 0.f, 0.f);
}

// Per-tile words (launch_tile_info): all-solid 32-cell lines and the rule
// class of each 64-cell wavefront.  One wavefront per tile, one lane per line;
// lines and wavefronts of a plane start at multiples of 32 / 64 cells because
// tiles and plane strides are multiples of 64 cells.
__global__ __launch_bounds__(64) void k_tile_info(const Geo *__restrict__ geo, const int32_t *__restrict__ tile_inst,
                                                 int32_t n_tiles, int32_t tcells, uint64_t *__restrict__ out)
{
    const int tile = blockIdx.x;
    if (tile >= n_tiles) return;
    const int ii = __builtin_amdgcn_readfirstlane(tile_inst[tile]);
    const Geo &G = geo[ii];
    const int lines = tcells >> 5;
    const int l = threadIdx.x;
    bool dead = true;
    int cls = 0;
    if (l < lines) {
        const int32_t c0 = (tile - G.tile0) * tcells + 32 * l;
        for (int k = 0; k < 32; ++k) {
            const int32_t c = c0 + k;
            if (c >= G.ncells) break;
            const uint8_t fl = gp(G.flags)[c];
            if (fl & FL_SOLID) continue;
            dead = false;
            const int k_cls = (fl & FL_FACE) ? 3 : ((fl & FL_GENERAL) ? 2 : ((fl & FL_NEAR) ? 1 : 0));
            cls = k_cls > cls ? k_cls : cls;
        }
    }
    const uint64_t d = __ballot(l < lines && dead);
    const uint64_t m1 = __ballot(cls >= 1), m2 = __ballot(cls >= 2), m3 = __ballot(cls >= 3);
    if (l == 0) {
        uint64_t w = 0;
        for (int v = 0; v < (lines >> 1); ++v) {
            const uint64_t pair = 3ull << (2 * v);
            const uint64_t code = (m3 & pair) ? 3 : ((m2 & pair) ? 2 : ((m1 & pair) ? 1 : 0));
            w |= code << (2 * v);
        }
        out[2 * (size_t)tile] = d;
        out[2 * (size_t)tile + 1] = w;
    }
}

// mode 0: fields (ux, uy, uz, |u|) [ncells][4]; mode 1: populations [19][qs]
template <int PARITY>
__global__ __launch_bounds__(256) void k_fields(const Geo *__restrict__ geo, int32_t ii, int64_t step, float *out,
                                                int32_t mode)
{
    const Geo &G = geo[ii];
    const int32_t lc = blockIdx.x * 256 + (int32_t)threadIdx.x;
    if (lc >= G.ncells) return;
    const uint32_t c = (uint32_t)lc;
    const uint8_t fl = gp(G.flags)[c];
    const uint32_t qs = (uint32_t)G.qs;
    if (fl & FL_SOLID) {
        if (mode == 0) reinterpret_cast<float4 *>(out)[c] = make_float4(0.f, 0.f, 0.f, 0.f);
        else
            for (int i = 0; i < Q; ++i) out[i * qs + c] = 0.0f;
        return;
    }
    int x = 0, y = 0, z = 0;
    coords(G, c, x, y, z);
    float g[Q];
    load_state<PARITY>(G, c, fl, x, y, z, step, g);
    if (mode == 0) {
        const Macro m = macro_of(g);
        reinterpret_cast<float4 *>(out)[c] =
            make_float4(m.ux, m.uy, m.uz, sqrtf(m.ux * m.ux + m.uy * m.uy + m.uz * m.uz));
    } else {
        for (int i = 0; i < Q; ++i) out[i * qs + c] = g[i];
    }
}

__global__ __launch_bounds__(256) void k_average(const double *__restrict__ qsum, const double *__restrict__ psum,
                                                 int32_t n4, int32_t np, double inv, float *out, float *pout)
{
    const int32_t e = blockIdx.x * 256 + (int32_t)threadIdx.x;
    if (e < n4) out[e] = (float)(qsum[e] * inv);
    if (pout && e < np) pout[e] = (float)(psum[e] * inv);
}

__global__ __launch_bounds__(256) void k_zero(float *qpart, double *qsum, double *psum, int32_t n4, int32_t np)
{
    const int32_t e = blockIdx.x * 256 + (int32_t)threadIdx.x;
    if (e < n4) {
        if (qpart) qpart[e] = 0.0f;
        if (qsum) qsum[e] = 0.0;
    }
    if (psum && e < np) psum[e] = 0.0;
}

// Geometry: per-cell flags and solid-link masks from the solid mask.
__global__ __launch_bounds__(256) void k_init_geometry(Box b, const uint8_t *__restrict__ solid,
                                                       uint8_t *__restrict__ flags, uint32_t *__restrict__ smask,
                                                       const int32_t *__restrict__ probes, int32_t n_probes,
                                                       int32_t ncells)
{
    const int32_t c = blockIdx.x * 256 + (int32_t)threadIdx.x;
    if (c >= ncells) return;
    const int x = c % b.nx, y = (c / b.nx) % b.ny, z = c / (b.nx * b.ny);
    uint8_t fl;
    uint32_t m;
    cell_flags(b, solid, x, y, z, fl, m);
    if (!(fl & FL_SOLID)) {
        int lo = 0, hi = n_probes - 1;
        while (lo <= hi) {
            int mid = (lo + hi) >> 1;
            if (probes[mid] == c) { fl |= FL_PROBE; break; }
            if (probes[mid] < c) lo = mid + 1; else hi = mid - 1;
        }
    }
    flags[c] = fl;
    smask[c] = m;
}

// ------------------------------------------------------------------ moments

struct Weights {
    double w[256];
};

// Count of negative variances, one atomic per workgroup: per-element atomics
// on the one counter serialise in L2 (1.6 % of the headline batch's 8.4 M
// values are negative).
__device__ __forceinline__ void add_block_count(unsigned int cnt, unsigned long long *nneg)
{
    __shared__ unsigned int sh[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int t = sh[0] + sh[1] + sh[2] + sh[3];
        if (t) atomicAdd(nneg, (unsigned long long)t);
    }
}

// Eq. (quad_moments) per element, grid-stride over groups of four
// consecutive elements (n4 groups: n / 4 when n is a multiple of 4 and q,
// mean and var are 16-byte aligned, else 0): per node one 16-byte load of the
// four values, per element the same FP64 sums in node order as one element
// at a time; the elements past the groups one per thread.
template <int NQMAX>
__device__ __forceinline__ void moments_one(const float v32[NQMAX], int32_t nq, const Weights &W, double &m,
                                            double &s)
{
    double v[NQMAX];
    m = 0.0;
#pragma unroll
    for (int j = 0; j < NQMAX; ++j) {
        if (j < nq) {
            v[j] = (double)v32[j];
            m += W.w[j] * v[j];
        }
    }
    s = 0.0;
#pragma unroll
    for (int j = 0; j < NQMAX; ++j) {
        if (j < nq) {
            const double d = v[j] - m;
            s += W.w[j] * d * d;
        }
    }
}

template <int NQMAX>
__global__ __launch_bounds__(256) void k_moments_arg(const float *__restrict__ q, int32_t nq, int64_t n,
                                                     int64_t n4, Weights W, double *__restrict__ mean,
                                                     double *__restrict__ var, unsigned long long *nneg)
{
    unsigned int cnt = 0;
    const int64_t stride = (int64_t)gridDim.x * 256;
    if constexpr (NQMAX > 16) n4 = 0;                   // 4 x 32 values would not fit in registers
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < n4; g += stride) {
        float4 r[NQMAX];
#pragma unroll
        for (int j = 0; j < NQMAX; ++j)
            if (j < nq) r[j] = reinterpret_cast<const float4 *>(q + (int64_t)j * n)[g];
        double m4[4], s4[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float v32[NQMAX];
#pragma unroll
            for (int j = 0; j < NQMAX; ++j) v32[j] = k == 0 ? r[j].x : k == 1 ? r[j].y : k == 2 ? r[j].z : r[j].w;
            moments_one<NQMAX>(v32, nq, W, m4[k], s4[k]);
            cnt += s4[k] < 0.0 ? 1u : 0u;
        }
        reinterpret_cast<double2 *>(mean)[2 * g] = make_double2(m4[0], m4[1]);
        reinterpret_cast<double2 *>(mean)[2 * g + 1] = make_double2(m4[2], m4[3]);
        reinterpret_cast<double2 *>(var)[2 * g] = make_double2(s4[0], s4[1]);
        reinterpret_cast<double2 *>(var)[2 * g + 1] = make_double2(s4[2], s4[3]);
    }
    for (int64_t e = 4 * n4 + (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += stride) {
        float v32[NQMAX];
#pragma unroll
        for (int j = 0; j < NQMAX; ++j)
            if (j < nq) v32[j] = q[(int64_t)j * n + e];
        double m, s;
        moments_one<NQMAX>(v32, nq, W, m, s);
        mean[e] = m;
        var[e] = s;
        cnt += s < 0.0 ? 1u : 0u;
    }
    if (nneg) add_block_count(cnt, nneg);
}

__global__ __launch_bounds__(256) void k_moments_arg_shift(const float *__restrict__ q, int32_t nq, int64_t n,
                                                           Weights W, double *__restrict__ mean,
                                                           double *__restrict__ var, unsigned long long *nneg)
{
    unsigned int cnt = 0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const double K = (double)q[e];
        double s1 = 0.0, s2 = 0.0;
        for (int j = 0; j < nq; ++j) {
            const double d = (double)q[(int64_t)j * n + e] - K;
            s1 += W.w[j] * d;
            s2 += W.w[j] * d * d;
        }
        mean[e] = K + s1;
        const double s = s2 - s1 * s1;
        var[e] = s;
        cnt += s < 0.0 ? 1u : 0u;
    }
    if (nneg) add_block_count(cnt, nneg);
}


// grad[i][k] += sum of part[tile][k] over instance i's tiles: one workgroup
// per instance; each thread sums tiles t, t + 256, ... in increasing order,
// then a fixed butterfly per wavefront and the four wavefront sums in order
// (deterministic).  The partials were written by every XCD, so each load
// misses this XCD's L2: all of a thread's loads are issued together.
__global__ __launch_bounds__(256) void k_grad_reduce(const Geo *__restrict__ geo, int32_t tile_cells,
                                                     const double *__restrict__ part, double *__restrict__ grad)
{
    const int ii = blockIdx.x;
    const Geo &G = geo[ii];
    const int32_t nt = (G.ncells + tile_cells - 1) / tile_cells;
    __shared__ double sh[3][4];
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    constexpr int U = 16;
    for (int32_t tb = threadIdx.x; tb < nt; tb += 256 * U) {
        double v[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t t = tb + 256 * u;
            if (t < nt) {
                const double *q = part + 3 * (size_t)(G.tile0 + t);
                v[u][0] = q[0];
                v[u][1] = q[1];
                v[u][2] = q[2];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (tb + 256 * u < nt) {
                t0 += v[u][0];
                t1 += v[u][1];
                t2 += v[u][2];
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        t0 += __shfl_xor(t0, o, 64);
        t1 += __shfl_xor(t1, o, 64);
        t2 += __shfl_xor(t2, o, 64);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[0][wv] = t0;
        sh[1][wv] = t1;
        sh[2][wv] = t2;
    }
    __syncthreads();
    if (threadIdx.x < 3) grad[3 * ii + threadIdx.x] += ((sh[threadIdx.x][0] + sh[threadIdx.x][1]) + sh[threadIdx.x][2]) + sh[threadIdx.x][3];
}

// lam^N = dj_N / df^N from the (even, naturally stored) current state.
__global__ __launch_bounds__(1024) void k_adjoint_init(const Geo *__restrict__ geo, const int32_t *__restrict__ tile_inst,
                                                      int32_t n_tiles, AdjArgs a)
{
    const int tile = xcd_tile();
    if (tile >= n_tiles) return;
    const int ii = __builtin_amdgcn_readfirstlane(tile_inst[tile]);
    const Geo &G = geo[ii];
    const int32_t lc = (tile - G.tile0) * (int32_t)blockDim.x + (int32_t)threadIdx.x;
    if (lc >= G.ncells) return;
    const uint32_t c = (uint32_t)lc;
    const uint32_t qs = (uint32_t)G.qs;
    const uint8_t fl = gp(G.flags)[c];
    float *lout = a.lam_out[ii];
    float src = 0.0f, ux = 0.0f;
    if (!(fl & FL_SOLID) && a.in_window && (fl & FL_PROBE) && a.pw[ii]) {
        const int p = probe_index(G, (int32_t)c);
        if (p >= 0) {
            float g[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) g[i] = gp(G.f)[i * qs + c];
            const Macro m = macro_of(g);
            src = (float)(a.pw[ii][p] * a.inv_count) / m.rho;
            ux = m.ux;
        }
    }
    for (int k = 0; k < Q; ++k) lout[k * qs + c] = src * (cx(k) - ux);
}

}  // namespace

// ------------------------------------------------------------------ launches

bool variant_ok(const Variant &v)
{
    return (v.bs == 64 || v.bs == 128 || v.bs == 256 || v.bs == 512) && (v.cpt == 1 || v.cpt == 2 || v.cpt == 4) &&
           v.nt >= 0 && v.nt <= 3 && (v.xcd == 0 || v.xcd == 1);
}

int launch_step(const Variant &v, int model, int parity, const Geo *geo, const int32_t *tile_inst, int32_t n_tiles,
                const StepArgs &a0, int32_t *health, hipStream_t s)
{
    if (n_tiles <= 0) return 0;
    if (!variant_ok(v)) return -1;
    StepArgs a = a0;
    a.xcd_remap = v.xcd;
    if (model == 0) return launch_step_model<0>(v, parity, geo, tile_inst, n_tiles, a, health, s);
    if (model == 1) return launch_step_model<1>(v, parity, geo, tile_inst, n_tiles, a, health, s);
    return launch_step_model<2>(v, parity, geo, tile_inst, n_tiles, a, health, s);
}

int launch_init_geometry(const Box &b, const uint8_t *solid, uint8_t *flags, uint32_t *smask, const int32_t *probes,
                         int32_t n_probes, hipStream_t s)
{
    const int32_t n = b.nx * b.ny * b.nz;
    hipLaunchKernelGGL(k_init_geometry, dim3((n + 255) / 256), dim3(256), 0, s, b, solid, flags, smask, probes,
                       n_probes, n);
    return (int)hipGetLastError();
}

int launch_capture(int tcells, int parity, const Geo *geo, const int32_t *tile_inst, int32_t n_tiles, int64_t step,
                   int32_t *health, hipStream_t s)
{
    const dim3 grid(grid_of(n_tiles)), block(tcells);
    if (parity == 0) hipLaunchKernelGGL(k_capture<0>, grid, block, 0, s, geo, tile_inst, n_tiles, step, health);
    else hipLaunchKernelGGL(k_capture<1>, grid, block, 0, s, geo, tile_inst, n_tiles, step, health);
    return (int)hipGetLastError();
}

int launch_flush(int tcells, const Geo *geo, const int32_t *tile_inst, int32_t n_tiles, hipStream_t s)
{
    hipLaunchKernelGGL(k_flush, dim3(grid_of(n_tiles)), dim3(tcells), 0, s, geo, tile_inst, n_tiles);
    return (int)hipGetLastError();
}

int launch_tile_info(int tcells, const Geo *geo, const int32_t *tile_inst, int32_t n_tiles, uint64_t *out,
                     hipStream_t s)
{
    if (tcells < 64 || tcells > 2048 || (tcells & 63)) return (int)hipErrorInvalidValue;
    if (n_tiles <= 0) return 0;
    hipLaunchKernelGGL(k_tile_info, dim3(n_tiles), dim3(64), 0, s, geo, tile_inst, n_tiles, tcells, out);
    return (int)hipGetLastError();
}

int launch_fields(int parity, const Geo *geo, int32_t inst, const Geo &g, int64_t step, float *out, int32_t mode,
                  hipStream_t s)
{
    const dim3 grid((g.ncells + 255) / 256), block(256);
    if (parity == 0) hipLaunchKernelGGL(k_fields<0>, grid, block, 0, s, geo, inst, step, out, mode);
    else hipLaunchKernelGGL(k_fields<1>, grid, block, 0, s, geo, inst, step, out, mode);
    return (int)hipGetLastError();
}

int launch_average(const Geo &g, double inv_count, float *out, float *pout, hipStream_t s)
{
    const int32_t n4 = 4 * g.ncells;
    const int32_t n = n4 > g.n_probes ? n4 : g.n_probes;
    hipLaunchKernelGGL(k_average, dim3((n + 255) / 256), dim3(256), 0, s, g.qsum, g.psum, g.qsum ? n4 : 0,
                       g.n_probes, inv_count, out, pout);
    return (int)hipGetLastError();
}

int launch_zero_qoi(const Geo &g, hipStream_t s)
{
    const int32_t n4 = 4 * g.ncells;
    const int32_t n = n4 > g.n_probes ? n4 : g.n_probes;
    hipLaunchKernelGGL(k_zero, dim3((n + 255) / 256), dim3(256), 0, s, g.qpart, g.qsum, g.psum, n4, g.n_probes);
    return (int)hipGetLastError();
}

int launch_moments(const float *q, const double *w, int32_t nq, int64_t n, double *mean, double *var,
                   unsigned long long *nneg, hipStream_t s)
{
    Weights W;
    for (int j = 0; j < 256; ++j) W.w[j] = j < nq ? w[j] : 0.0;
    // at most 16 workgroups per compute unit, each striding over the rest
    const int64_t blocks = (n + 255) / 256;
    const dim3 grid((unsigned)(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096)), block(256);
    const bool vec = n % 4 == 0 && ((uintptr_t)q & 15) == 0 && ((uintptr_t)mean & 15) == 0 && ((uintptr_t)var & 15) == 0;
    const int64_t n4 = vec ? n / 4 : 0;
    if (nq <= 8) hipLaunchKernelGGL(k_moments_arg<8>, grid, block, 0, s, q, nq, n, n4, W, mean, var, nneg);
    else if (nq <= 16) hipLaunchKernelGGL(k_moments_arg<16>, grid, block, 0, s, q, nq, n, n4, W, mean, var, nneg);
    else if (nq <= 32) hipLaunchKernelGGL(k_moments_arg<32>, grid, block, 0, s, q, nq, n, n4, W, mean, var, nneg);
    else hipLaunchKernelGGL(k_moments_arg_shift, grid, block, 0, s, q, nq, n, W, mean, var, nneg);
    return (int)hipGetLastError();
}

int launch_grad_reduce(int tile_cells, const Geo *, int32_t n_inst, const Geo *geo, const double *part,
                       double *grad, hipStream_t s)
{
    if (n_inst <= 0) return 0;
    hipLaunchKernelGGL(k_grad_reduce, dim3(n_inst), dim3(256), 0, s, geo, tile_cells, part, grad);
    return (int)hipGetLastError();
}

int launch_adjoint_init(int tcells, const Geo *geo, const int32_t *tile_inst, int32_t n_tiles, const AdjArgs &a,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_adjoint_init, dim3(grid_of(n_tiles)), dim3(tcells), 0, s, geo, tile_inst, n_tiles, a);
    return (int)hipGetLastError();
}

}  // namespace lbmsc
