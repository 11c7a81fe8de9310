// k-nearest-neighbour Gaussian weight graph on the device.
#pragma once
#include <string>

#include "graph.hpp"

namespace ccm {

// See ccm_build_knn_graph in include/ccm.h for the definition.
ccm_status knn_graph(const double* A, int64_t n, int d, int k, double phi, int* src, int* dst,
                     double* w, int64_t m_cap, int64_t& m_out, double& phi_out, hipStream_t s,
                     std::string& err);

// See ccm_build_knn_graph_u8 in include/ccm.h.
ccm_status knn_graph_u8(const unsigned char* K, int64_t n, int d, double scale, int k, double phi,
                        int* src, int* dst, double* w, int64_t m_cap, int64_t& m_out,
                        double& phi_out, hipStream_t s, std::string& err);

}  // namespace ccm
