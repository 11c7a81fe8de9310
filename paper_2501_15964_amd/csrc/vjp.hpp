// Vector-Jacobian product of the clustering solution map (q = 2).
#pragma once
#include <string>

#include "graph.hpp"

namespace ccm {

// See ccm_path_vjp in include/ccm.h.  Edges must be canonical.
ccm_status path_vjp(const double* A, int64_t n, int d, const int* src, const int* dst,
                    const double* w, int64_t m, double gamma, const double* X, const int* labels,
                    const double* dLdX, double* dLdA, double* dLdlogw, double* dLdgamma,
                    double tol, int maxit, int* iters_out, hipStream_t s, std::string& err);

}  // namespace ccm
