// quadrature.h -- host-side collocation rules (probability weights on U(-1,1)^d).
#pragma once
#include <vector>

namespace lbmsc {
bool gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);
bool clenshaw_curtis(int m, std::vector<double> &x, std::vector<double> &w);
bool smolyak_cc(int level, int dim, std::vector<double> &nodes, std::vector<double> &weights);
}  // namespace lbmsc
