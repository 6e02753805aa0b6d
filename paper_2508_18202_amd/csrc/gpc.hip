// gpc.hip -- projection of node-major collocation outputs onto the
// orthonormal Hermite chaos (Sec. 2.3 gPC coefficients), one instantiation
// per term count so the coefficient loop carries no guards.
#include "kernels.h"

namespace lbmsc {

namespace {

// gPC coefficients of one element per thread: coef[p][e] = sum_j wphi[j][p] q[j][e]
// in FP64, for exactly NB terms (no per-term guards).  The weighted basis
// index does not depend on the lane, so its values come through the scalar
// cache; q is read node-major (coalesced), eight nodes in flight at a time.
template <int NB>
__global__ __launch_bounds__(256) void k_gpc(const float *__restrict__ q, const double *__restrict__ wphi,
                                             int32_t nq, int64_t n, double *__restrict__ coef,
                                             double *__restrict__ var, double *__restrict__ band)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    double acc[NB];
#pragma unroll
    for (int p = 0; p < NB; ++p) acc[p] = 0.0;
    int32_t j = 0;
    for (; j + 8 <= nq; j += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = (double)q[(int64_t)(j + u) * n + e];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double *b = wphi + (int64_t)(j + u) * NB;
#pragma unroll
            for (int p = 0; p < NB; ++p) acc[p] += b[p] * v[u];
        }
    }
    for (; j < nq; ++j) {
        const double v = (double)q[(int64_t)j * n + e];
        const double *b = wphi + (int64_t)j * NB;
#pragma unroll
        for (int p = 0; p < NB; ++p) acc[p] += b[p] * v;
    }
#pragma unroll
    for (int p = 0; p < NB; ++p) coef[(int64_t)p * n + e] = acc[p];
    if (var || band) {
        double v = 0.0;
#pragma unroll
        for (int p = 1; p < NB; ++p) v += acc[p] * acc[p];
        if (var) var[e] = v;
        if (band) {
            const double h = 1.96 * sqrt(v);
            band[e] = acc[0] - h;
            band[n + e] = acc[0] + h;
        }
    }
}

}  // namespace

// launch k_gpc<NB> for the runtime term count nb (1 .. 64)
template <int NB>
static void gpc_dispatch(int32_t nb, const dim3 &grid, const float *q, const double *wphi, int32_t nq, int64_t n,
                         double *coef, double *var, double *band, hipStream_t s)
{
    if constexpr (NB > 64) {
        return;
    } else {
        if (nb == NB) hipLaunchKernelGGL(k_gpc<NB>, grid, dim3(256), 0, s, q, wphi, nq, n, coef, var, band);
        else gpc_dispatch<NB + 1>(nb, grid, q, wphi, nq, n, coef, var, band, s);
    }
}

int launch_gpc(const float *q, const double *wphi, int32_t nq, int32_t nb, int64_t n, double *coef, double *var,
               double *band, hipStream_t s)
{
    if (nb < 1 || nb > 64) return -1;
    const dim3 grid((unsigned)((n + 255) / 256));
    gpc_dispatch<1>(nb, grid, q, wphi, nq, n, coef, var, band, s);
    return (int)hipGetLastError();
}

}  // namespace lbmsc
