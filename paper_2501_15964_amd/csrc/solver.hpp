// Path solvers (SSNAL, ADMM, fast AMA) over a device graph.
#pragma once
#include <string>
#include <vector>

#include "graph.hpp"

namespace ccm {

// Instances solved together as one block-diagonal problem (see
// ccm_solve_path_batched): segment s owns union vertices [vseg[s], vseg[s+1])
// and union edges [eseg[s], eseg[s+1]).  Outputs go to the caller's
// per-instance blocks; host arrays are indexed [inst[s] * T + t].
struct BatchSpec {
    int S = 0;
    std::vector<int64_t> vseg, eseg;             // host copies, S + 1 entries
    const int64_t* vseg_dev = nullptr;
    const int64_t* eseg_dev = nullptr;
    const int64_t* xoff_dev = nullptr;           // per segment: first element in X_out_all
    const int64_t* loff_dev = nullptr;           // per segment: first element in labels_all
    std::vector<int> inst;                       // global instance index per segment
    double* X_out_all = nullptr;
    int* labels_all = nullptr;
    int* n_clusters_host = nullptr;
    double* kkt_host = nullptr;
    int* status_host = nullptr;
};

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

    // Batched path: every gamma is solved for all segments at once and each
    // segment's relative KKT residual (its own norms) must reach tol.
    ccm_status run_batched(const double* gammas, int T, const BatchSpec& b);

   private:
    struct Impl;
    Impl* impl_;
};

}  // namespace ccm
