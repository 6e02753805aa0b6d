// quadrature.h -- host-side collocation rules (probability weights on U(-1,1)^d
// and on the standard normal) and the Hermite chaos basis.
#pragma once
#include <vector>

namespace lbmsc {
bool gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);
bool clenshaw_curtis(int m, std::vector<double> &x, std::vector<double> &w);
bool smolyak_cc(int level, int dim, std::vector<double> &nodes, std::vector<double> &weights);
// Gauss-Hermite rule of n points for the standard normal (probabilists'
// polynomials), and its d-fold tensor product (node j = (i_1 ... i_d), the
// last coordinate fastest).
bool gauss_hermite(int n, std::vector<double> &x, std::vector<double> &w);
bool tensor_gauss_hermite(int n, int dim, std::vector<double> &nodes, std::vector<double> &weights);
// Orthonormal Hermite chaos basis of total degree <= order in dim Gaussian
// variables: alpha[p*dim + k] the multi-indices (graded: degree 0, 1, ...;
// within a degree the first variable's power descending), phi[j*P + p] =
// prod_k He_{alpha_pk}(z_jk) / sqrt(alpha_pk!).
void gpc_multi_indices(int dim, int order, std::vector<int> &alpha);
void gpc_basis(const double *nodes, int n_nodes, int dim, const std::vector<int> &alpha, std::vector<double> &phi);
}  // namespace lbmsc
