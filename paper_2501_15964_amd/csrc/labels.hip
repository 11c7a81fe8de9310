// Cluster labels: connected components of the fused edges.
//
// Concurrent union-find with the rule "hook the larger root under the smaller
// one".  When the vertex-major incidence lists are at hand it starts from a
// forest built without retries: every vertex points at its smallest fused
// neighbour, then twice every root at the smallest root across its fused
// edges, each step followed by full path compression.  A
// parent index is never larger than its child's, so every find walks a
// strictly decreasing chain (at most n steps) and each component's final
// root is its smallest vertex.  Labels are then the ranks of the roots in
// vertex order (an exclusive scan of root flags), i.e. clusters are numbered
// by their smallest point index.  Only integer atomics on vertex memory are
// used; the result does not depend on the order in which edges are merged.
#include <hipcub/hipcub.hpp>

#include <algorithm>

#include "launch.hpp"

namespace ccm {
namespace {

__device__ __forceinline__ int ld_parent(const int* parent, int x) {
    return __hip_atomic_load(parent + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int uf_find(int* parent, int x, int64_t n) {
    for (int64_t step = 0; step <= n; ++step) {
        const int p = ld_parent(parent, x);
        if (p == x) return x;
        const int gp = ld_parent(parent, p);
        if (gp != p)  // path halving: moving a pointer to an ancestor is always safe
            __hip_atomic_store(parent + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = gp;
    }
    return x;
}

// root without path halving (read-only walk)
__device__ __forceinline__ int uf_root(const int* parent, int x, int64_t n) {
    for (int64_t step = 0; step <= n; ++step) {
        const int p = ld_parent(parent, x);
        if (p == x) return x;
        x = p;
    }
    return x;
}

__global__ __launch_bounds__(kBlock) void k_uf_init(int64_t n, int* parent) {
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * kBlock)
        parent[i] = int(i);
}

// First hooking, without atomics: every vertex points at its smallest fused
// neighbour (or at itself); 16 lanes share a vertex's incidence list (the
// lists are indexed by rank r, of vertex vord[r], or by vertex if vord is
// null).  Pointers decrease, so this is a forest inside the components, and
// most fused edges then join vertices of one tree.
constexpr int kHookLanes = 16;
__global__ __launch_bounds__(kBlock) void k_uf_hook_min(int64_t n, const int* __restrict__ inc_ptr,
                                                        const Inc* __restrict__ inc,
                                                        const int* __restrict__ vord,
                                                        const int* __restrict__ fused,
                                                        int* __restrict__ parent) {
    const int gl = threadIdx.x % kHookLanes;
    constexpr int GPB = kBlock / kHookLanes;
    for (int64_t r = int64_t(blockIdx.x) * GPB + threadIdx.x / kHookLanes; r < n;
         r += int64_t(gridDim.x) * GPB) {
        const int64_t v = vord ? vord[r] : r;
        int mn = int(v);
        const int e1 = inc_ptr[r + 1];
        for (int p = inc_ptr[r] + gl; p < e1; p += kHookLanes) {
            const Inc e = inc[p];
            const int l = e.e >= 0 ? e.e : ~e.e;
            if (fused[l] && e.o < mn) mn = e.o;
        }
#pragma unroll
        for (int off = kHookLanes / 2; off > 0; off >>= 1) {
            const int o = __shfl_xor(mn, off, 64);
            mn = o < mn ? o : mn;
        }
        if (gl == 0) parent[v] = mn;
    }
}

// Every vertex points at the root of its tree (the forest is read-only here
// except for these pointer moves to ancestors, which readers may or may not
// see: any ancestor is a valid parent).
__global__ __launch_bounds__(kBlock) void k_uf_jump(int64_t n, int* parent) {
    for (int64_t v = int64_t(blockIdx.x) * kBlock + threadIdx.x; v < n;
         v += int64_t(gridDim.x) * kBlock) {
        const int r = uf_root(parent, int(v), n);
        __hip_atomic_store(parent + v, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// One hooking round over the fused edges of a depth-one forest: the larger
// of an edge's two roots is pointed at the smaller (atomicMin keeps the
// smallest of several offers, so no retries).  Pointers still decrease and
// stay inside the component.
__global__ __launch_bounds__(kBlock) void k_uf_hook_edges(int64_t m, const int* __restrict__ src,
                                                          const int* __restrict__ dst,
                                                          const int* __restrict__ fused,
                                                          int* parent) {
    for (int64_t l = int64_t(blockIdx.x) * kBlock + threadIdx.x; l < m;
         l += int64_t(gridDim.x) * kBlock) {
        if (!fused[l]) continue;
        const int ra = ld_parent(parent, src[l]);
        const int rb = ld_parent(parent, dst[l]);
        if (ra != rb) atomicMin(parent + (ra > rb ? ra : rb), ra > rb ? rb : ra);
    }
}

__global__ __launch_bounds__(kBlock) void k_uf_union(int64_t m, const int* __restrict__ src,
                                                     const int* __restrict__ dst,
                                                     const int* __restrict__ fused, int* parent,
                                                     int64_t n) {
    for (int64_t l = int64_t(blockIdx.x) * kBlock + threadIdx.x; l < m;
         l += int64_t(gridDim.x) * kBlock) {
        if (!fused[l]) continue;
        int a = src[l], b = dst[l];
        for (int64_t tries = 0; tries <= n; ++tries) {
            int ra = uf_find(parent, a, n);
            int rb = uf_find(parent, b, n);
            if (ra == rb) break;
            if (ra > rb) {
                const int t = ra;
                ra = rb;
                rb = t;
            }
            // rb is the larger root: hook it under ra if it is still a root
            if (atomicCAS(parent + rb, rb, ra) == rb) break;
            a = ra;
            b = rb;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_uf_flatten(int64_t n, int* parent, int* flag) {
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * kBlock) {
        const int r = uf_find(parent, int(i), n);
        flag[i] = (r == int(i)) ? 1 : 0;
    }
}

__global__ __launch_bounds__(kBlock) void k_uf_store(int64_t n, int* parent, const int* rank,
                                                     const int* last_flag, int* labels,
                                                     int* n_clusters) {
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * kBlock) {
        const int r = uf_find(parent, int(i), n);
        labels[i] = rank[r];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) n_clusters[0] = rank[n - 1] + last_flag[0];
}

}  // namespace

size_t labels_temp_bytes(int64_t n) {
    size_t bytes = 0;
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, (const int*)nullptr, (int*)nullptr,
                                           int(n));
    return bytes + 256;
}

void launch_labels(int64_t n, int64_t m, const int* src, const int* dst, const int* fused,
                   int* parent, int* rank, void* temp, size_t temp_bytes, int* labels,
                   int* n_clusters, hipStream_t s, const int* inc_ptr, const Inc* inc,
                   const int* vord) {
    // rank holds n + 1 ints: [0, n) the scan output, [n] the last root flag.
    // The root flags themselves live in `labels` until the final pass
    // overwrites them with the labels.
    const int g = flat_grid(n);
    int* flag = labels;
    if (inc_ptr && inc && m > 0) {
        const int64_t gpb = kBlock / kHookLanes;
        const int gh = int(std::min<int64_t>((n + gpb - 1) / gpb, kMaxGrid));
        hipLaunchKernelGGL(k_uf_hook_min, dim3(gh), dim3(kBlock), 0, s, n, inc_ptr, inc, vord,
                           fused, parent);
        hipLaunchKernelGGL(k_uf_jump, dim3(g), dim3(kBlock), 0, s, n, parent);
        for (int round = 0; round < 2; ++round) {
            hipLaunchKernelGGL(k_uf_hook_edges, dim3(flat_grid(m)), dim3(kBlock), 0, s, m, src,
                               dst, fused, parent);
            hipLaunchKernelGGL(k_uf_jump, dim3(g), dim3(kBlock), 0, s, n, parent);
        }
    } else
        hipLaunchKernelGGL(k_uf_init, dim3(g), dim3(kBlock), 0, s, n, parent);
    if (m > 0)
        hipLaunchKernelGGL(k_uf_union, dim3(flat_grid(m)), dim3(kBlock), 0, s, m, src, dst, fused,
                           parent, n);
    hipLaunchKernelGGL(k_uf_flatten, dim3(g), dim3(kBlock), 0, s, n, parent, flag);
    size_t tb = temp_bytes;
    (void)hipcub::DeviceScan::ExclusiveSum(temp, tb, flag, rank, int(n), s);
    // n_clusters needs flag[n-1] before labels overwrite it: save it in rank[n]
    (void)hipMemcpyAsync(rank + n, flag + n - 1, sizeof(int), hipMemcpyDeviceToDevice, s);
    hipLaunchKernelGGL(k_uf_store, dim3(g), dim3(kBlock), 0, s, n, parent, rank, rank + n, labels,
                       n_clusters);
}

}  // namespace ccm
