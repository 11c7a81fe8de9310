// Path solvers (SSNAL, ADMM, fast AMA) over a device graph.
#pragma once
#include <string>

#include "graph.hpp"

namespace ccm {

class Solver {
   public:
    Solver(const DevGraph& g, int d, int qk, const double* A, hipStream_t s,
           const ccm_options& o, double tol, std::string& err);
    ~Solver();
    Solver(const Solver&) = delete;
    Solver& operator=(const Solver&) = delete;
    // Solves the gammas in order, warm-starting each from the previous one.
    ccm_status run_path(const double* gammas, int T, const double* X_warm, const double* U_warm,
                        double* X_out, double* U_out, int* labels_out, int* n_clusters,
                        double* kkt, int* status, ccm_stats* stats);

   private:
    struct Impl;
    Impl* impl_;
};

}  // namespace ccm
