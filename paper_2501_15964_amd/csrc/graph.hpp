// Device graph construction: validation, canonical edge list and the
// vertex-major incidence lists (CSR by vertex).
#pragma once
#include <string>

#include "ccm.h"
#include "launch.hpp"

namespace ccm {

// Device work space of the library: blocks are cached per device after use
// and handed out again (same stream: at once; another stream: after an
// event wait), so repeated calls neither map nor unmap memory.  Sizes are
// rounded up to size classes.  The cache keeps at most half of the device's
// memory; release_workspace() frees every cached block.
hipError_t workspace_alloc(void** p, size_t bytes, hipStream_t s, int& dev);
void workspace_free(void* p, hipStream_t s, int dev);
hipError_t release_workspace();

// Stream-ordered device allocation that is released when the object dies.
struct DevMem {
    void* p = nullptr;
    hipStream_t s = nullptr;
    int dev = 0;  // device of the block
    DevMem() = default;
    DevMem(const DevMem&) = delete;
    DevMem& operator=(const DevMem&) = delete;
    ~DevMem() { release(); }
    void release() {
        if (p) workspace_free(p, s, dev);
        p = nullptr;
    }
    hipError_t alloc(size_t bytes, hipStream_t st) {
        release();
        s = st;
        if (bytes == 0) bytes = 8;
        return workspace_alloc(&p, bytes, st, dev);
    }
    template <class T>
    T* as() const { return static_cast<T*>(p); }
};

struct OwnedGraph {
    DevGraph g;
    DevMem src, dst, w, inc_ptr, inc, irow, epos, win, iso, vord, vrank;
};

// Builds `out` from caller edges for rows of d values.  With
// require_canonical the edges must already be canonical (src < dst, strictly
// increasing (src, dst), w > 0) and are referenced in place; otherwise they
// are canonicalised into owned arrays.  `locality` selects the processing
// order of the vertices in the incidence lists: 0 the input order, 1 a
// locality order (connected components one after another, each in
// breadth-first levels from its smallest vertex, ties by vertex index), -1
// the locality order when n d >= kLocalityMin.  The order changes which
// vertices the vertex kernels work on at the same time (and so what the
// caches hold), never the data layout.  Returns CCM_OK or an error with text
// in `err`.  Synchronises s.
// The windows hold window_for(d, qk, chunk) incidences (chunk <= 0: the
// tuned chunk of d's row layout and q).
constexpr int64_t kLocalityMin = int64_t(1) << 22;
ccm_status graph_build(const int* src, const int* dst, const double* w, int64_t m, int64_t n,
                       int d, bool require_canonical, hipStream_t s, OwnedGraph& out,
                       std::string& err, int locality = -1, int qk = kQ2, int chunk = 0);

// Window split (win, iso) of out.g's incidence lists for rows of d values;
// needs out.g.n, nent, inc_ptr, inc, irow.  Synchronises s.
ccm_status build_windows(int d, hipStream_t s, OwnedGraph& out, std::string& err,
                         int qk = kQ2, int chunk = 0);

// Cluster membership lists as a graph for the vertex kernels: row c lists
// the vertices with labels == c (labels in [0, K)), entries {vertex, 0}.
// With it, launch_scatter(cx = 0, cz = 1, Z = vertex rows) sums vertex rows
// per cluster in vertex order.  Synchronises s.
ccm_status membership_build(const int* labels, int64_t n, int64_t K, int d, hipStream_t s,
                            OwnedGraph& out, std::string& err);

// Number of canonical edges for the given input (synchronises s).
ccm_status graph_canonical_count(const int* src, const int* dst, const double* w, int64_t m,
                                 int64_t n, hipStream_t s, int64_t& m_canon, std::string& err);

}  // namespace ccm
