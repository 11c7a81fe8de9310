// Device graph construction (see graph.hpp).
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <utility>
#include <unordered_map>
#include <map>
#include <vector>

#include "graph.hpp"

namespace ccm {
namespace {

__global__ __launch_bounds__(kBlock) void k_validate(int64_t m, int64_t n, const int* __restrict__ src,
                                                     const int* __restrict__ dst,
                                                     const double* __restrict__ w, int* flags) {
    int bad_idx = 0, bad_w = 0, noncanon = 0;
    for (int64_t l = int64_t(blockIdx.x) * kBlock + threadIdx.x; l < m;
         l += int64_t(gridDim.x) * kBlock) {
        const int a = src[l], b = dst[l];
        const double wl = w[l];
        if (a < 0 || a >= n || b < 0 || b >= n) bad_idx = 1;
        if (!(wl >= 0.0) || isinf(wl)) bad_w = 1;
        bool ok = a < b && wl > 0.0;
        if (ok && l > 0) {
            const int pa = src[l - 1], pb = dst[l - 1];
            ok = (pa < a) || (pa == a && pb < b);
        }
        if (!ok) noncanon = 1;
    }
    if (bad_idx) atomicOr(flags + 0, 1);
    if (bad_w) atomicOr(flags + 1, 1);
    if (noncanon) atomicOr(flags + 2, 1);
}

__global__ __launch_bounds__(kBlock) void k_make_keys(int64_t m, const int* __restrict__ src,
                                                      const int* __restrict__ dst,
                                                      const double* __restrict__ w,
                                                      unsigned long long* __restrict__ key) {
    for (int64_t l = int64_t(blockIdx.x) * kBlock + threadIdx.x; l < m;
         l += int64_t(gridDim.x) * kBlock) {
        const unsigned a = unsigned(src[l]), b = unsigned(dst[l]);
        if (a == b || !(w[l] > 0.0)) {
            key[l] = ~0ull;
        } else {
            const unsigned lo = a < b ? a : b, hi = a < b ? b : a;
            key[l] = (static_cast<unsigned long long>(lo) << 32) | hi;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_unpack(int64_t m, const unsigned long long* __restrict__ key,
                                                   int* __restrict__ src, int* __restrict__ dst) {
    for (int64_t l = int64_t(blockIdx.x) * kBlock + threadIdx.x; l < m;
         l += int64_t(gridDim.x) * kBlock) {
        src[l] = int(key[l] >> 32);
        dst[l] = int(key[l] & 0xffffffffull);
    }
}

__global__ __launch_bounds__(kBlock) void k_inc_entries(int64_t m, const int* __restrict__ src,
                                                        const int* __restrict__ dst,
                                                        int* __restrict__ vk,
                                                        Inc* __restrict__ vv) {
    for (int64_t l = int64_t(blockIdx.x) * kBlock + threadIdx.x; l < m;
         l += int64_t(gridDim.x) * kBlock) {
        const int a = src[l], b = dst[l];
        vk[2 * l] = a;
        vv[2 * l] = Inc{int(l), b};
        vk[2 * l + 1] = b;
        vv[2 * l + 1] = Inc{~int(l), a};
    }
}

__global__ __launch_bounds__(kBlock) void k_inc_ptr(int64_t n, int64_t cnt,
                                                    const int* __restrict__ vk_sorted,
                                                    int* __restrict__ ptr, int* max_deg) {
    int best = 0;
    for (int64_t v = int64_t(blockIdx.x) * kBlock + threadIdx.x; v <= n;
         v += int64_t(gridDim.x) * kBlock) {
        // first position with key >= v
        int64_t lo = 0, hi = cnt;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (vk_sorted[mid] < v) lo = mid + 1;
            else hi = mid;
        }
        ptr[v] = int(lo);
        if (v < n) {
            int64_t lo2 = lo, hi2 = cnt;
            while (lo2 < hi2) {
                const int64_t mid = (lo2 + hi2) >> 1;
                if (vk_sorted[mid] < v + 1) lo2 = mid + 1;
                else hi2 = mid;
            }
            const int deg = int(lo2 - lo);
            best = deg > best ? deg : best;
        }
    }
    atomicMax(max_deg, best);
}

// incidence positions of each edge: epos[2 l] (src side), epos[2 l + 1] (dst side)
__global__ __launch_bounds__(kBlock) void k_epos(int64_t cnt, const Inc* __restrict__ inc,
                                                 int* __restrict__ epos) {
    for (int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x; p < cnt;
         p += int64_t(gridDim.x) * kBlock) {
        const int e = inc[p].e;
        if (e >= 0) epos[2 * int64_t(e)] = int(p);
        else epos[2 * int64_t(~e) + 1] = int(p);
    }
}

// ---- locality order ---------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_fill_i32(int64_t n, int v, int* __restrict__ x) {
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * kBlock)
        x[i] = v;
}

// first[c] = smallest vertex of component c (first preset to INT_MAX)
__global__ __launch_bounds__(kBlock) void k_comp_first(int64_t n, const int* __restrict__ comp,
                                                       int* first) {
    for (int64_t v = int64_t(blockIdx.x) * kBlock + threadIdx.x; v < n;
         v += int64_t(gridDim.x) * kBlock)
        atomicMin(first + comp[v], int(v));
}

constexpr int kUnreached = 0x7fffffff;

__global__ __launch_bounds__(kBlock) void k_bfs_init(int64_t n, const int* __restrict__ comp,
                                                     const int* __restrict__ first,
                                                     int* __restrict__ lev) {
    for (int64_t v = int64_t(blockIdx.x) * kBlock + threadIdx.x; v < n;
         v += int64_t(gridDim.x) * kBlock)
        lev[v] = first[comp[v]] == int(v) ? 0 : kUnreached;
}

// One breadth-first level: every vertex at level L gives its unreached
// neighbours level L + 1 (concurrent writers store the same value).  16
// lanes share a vertex's incidence list; inc_ptr is indexed by vertex here.
constexpr int kBfsLanes = 16;
__global__ __launch_bounds__(kBlock) void k_bfs_step(int64_t n, const int* __restrict__ inc_ptr,
                                                     const Inc* __restrict__ inc, int L, int* lev,
                                                     int* changed) {
    constexpr int GPB = kBlock / kBfsLanes;
    const int gl = threadIdx.x % kBfsLanes;
    int ch = 0;
    for (int64_t v = int64_t(blockIdx.x) * GPB + threadIdx.x / kBfsLanes; v < n;
         v += int64_t(gridDim.x) * GPB) {
        if (__hip_atomic_load(lev + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != L) continue;
        const int e1 = inc_ptr[v + 1];
        for (int p = inc_ptr[v] + gl; p < e1; p += kBfsLanes) {
            const int o = inc[p].o;
            if (__hip_atomic_load(lev + o, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                kUnreached) {
                __hip_atomic_store(lev + o, L + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ch = 1;
            }
        }
    }
    if (ch) atomicOr(changed, 1);
}

// sort key (component, level) of every vertex; levels past `cap` share cap
__global__ __launch_bounds__(kBlock) void k_order_keys(int64_t n, const int* __restrict__ comp,
                                                       const int* __restrict__ lev, int cap,
                                                       unsigned long long* __restrict__ key,
                                                       int* __restrict__ val) {
    for (int64_t v = int64_t(blockIdx.x) * kBlock + threadIdx.x; v < n;
         v += int64_t(gridDim.x) * kBlock) {
        const int l = lev[v] < cap ? lev[v] : cap;
        key[v] = static_cast<unsigned long long>(comp[v]) * (unsigned long long)(cap + 1) +
                 static_cast<unsigned long long>(l);
        val[v] = int(v);
    }
}

__global__ __launch_bounds__(kBlock) void k_rank_of(int64_t n, const int* __restrict__ vord,
                                                    int* __restrict__ vrank) {
    for (int64_t r = int64_t(blockIdx.x) * kBlock + threadIdx.x; r < n;
         r += int64_t(gridDim.x) * kBlock)
        vrank[vord[r]] = int(r);
}

__global__ __launch_bounds__(kBlock) void k_entry_rank(int64_t cnt, const int* __restrict__ irow,
                                                       const int* __restrict__ vrank,
                                                       int* __restrict__ rk) {
    for (int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x; p < cnt;
         p += int64_t(gridDim.x) * kBlock)
        rk[p] = vrank[irow[p]];
}

__global__ __launch_bounds__(kBlock) void k_entry_vertex(int64_t cnt, const int* __restrict__ rk,
                                                         const int* __restrict__ vord,
                                                         int* __restrict__ irow) {
    for (int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x; p < cnt;
         p += int64_t(gridDim.x) * kBlock)
        irow[p] = vord[rk[p]];
}

}  // namespace

namespace {
constexpr int kMaxDev = 64;

struct CachedBlock {
    void* p;
    hipStream_t s;   // stream of the last use
    hipEvent_t ev;   // recorded on s when the block was freed
};

struct DevCache {
    std::mutex mu;
    std::multimap<size_t, CachedBlock> free_blocks;            // by size class
    std::unordered_map<void*, std::pair<size_t, hipEvent_t>> live;
    size_t cached = 0;  // bytes in free_blocks
    size_t cap = 0;     // limit on `cached` (0: not yet known)
};

DevCache& dev_cache(int dev) {
    static DevCache caches[kMaxDev];
    return caches[dev];
}

size_t size_class(size_t b) {
    if (b <= 256) return 256;
    if (b < (size_t(1) << 20)) {
        size_t c = 512;
        while (c < b) c <<= 1;
        return c;
    }
    const size_t mb = size_t(1) << 20;
    return (b + mb - 1) / mb * mb;
}

// frees every cached block of c (caller holds c.mu)
hipError_t drop_cached(DevCache& c) {
    hipError_t r = hipSuccess;
    for (auto& kv : c.free_blocks) {
        CachedBlock& b = kv.second;
        if (b.ev) {
            const hipError_t e = hipEventSynchronize(b.ev);
            if (e != hipSuccess) r = e;
            (void)hipEventDestroy(b.ev);
        }
        const hipError_t f = hipFree(b.p);
        if (f != hipSuccess) r = f;
    }
    c.free_blocks.clear();
    c.cached = 0;
    return r;
}
}  // namespace

hipError_t workspace_alloc(void** p, size_t bytes, hipStream_t s, int& dev) {
    *p = nullptr;
    dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
    DevCache& c = dev_cache(dev);
    const size_t cls = size_class(bytes);
    std::lock_guard<std::mutex> lk(c.mu);
    auto range = c.free_blocks.equal_range(cls);
    if (range.first != range.second) {
        auto it = range.first;
        for (auto j = range.first; j != range.second; ++j)
            if (j->second.s == s) {
                it = j;
                break;
            }
        CachedBlock b = it->second;
        // another stream's last use must finish before this stream's work
        if (b.s != s && b.ev) {
            e = hipStreamWaitEvent(s, b.ev, 0);
            if (e != hipSuccess) return e;
        }
        c.free_blocks.erase(it);
        c.cached -= cls;
        c.live[b.p] = {cls, b.ev};
        *p = b.p;
        return hipSuccess;
    }
    e = hipMalloc(p, cls);
    if (e == hipErrorOutOfMemory && !c.free_blocks.empty()) {
        (void)hipGetLastError();
        (void)drop_cached(c);
        e = hipMalloc(p, cls);
    }
    if (e != hipSuccess) return e;
    c.live[*p] = {cls, nullptr};
    return hipSuccess;
}

void workspace_free(void* p, hipStream_t s, int dev) {
    if (!p || dev < 0 || dev >= kMaxDev) return;
    DevCache& c = dev_cache(dev);
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.live.find(p);
    if (it == c.live.end()) return;  // not a block of this device's cache
    const size_t cls = it->second.first;
    hipEvent_t ev = it->second.second;
    c.live.erase(it);
    if (c.cap == 0) {
        size_t fr = 0, tot = 0;
        c.cap = hipMemGetInfo(&fr, &tot) == hipSuccess ? tot / 2 : (size_t(8) << 30);
    }
    bool keep = c.cached + cls <= c.cap;
    if (keep && !ev) keep = hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
    if (keep) keep = hipEventRecord(ev, s) == hipSuccess;
    if (!keep) {
        // over the cap (or no event): hipFree waits for the device
        if (ev) (void)hipEventDestroy(ev);
        int cur = 0;
        (void)hipGetDevice(&cur);
        if (cur != dev) (void)hipSetDevice(dev);
        (void)hipFree(p);
        if (cur != dev) (void)hipSetDevice(cur);
        return;
    }
    c.free_blocks.insert({cls, CachedBlock{p, s, ev}});
    c.cached += cls;
}

hipError_t release_workspace() {
    int cur = 0;
    (void)hipGetDevice(&cur);
    hipError_t r = hipSuccess;
    for (int dv = 0; dv < kMaxDev; ++dv) {
        DevCache& c = dev_cache(dv);
        std::lock_guard<std::mutex> lk(c.mu);
        if (c.free_blocks.empty()) continue;
        if (hipSetDevice(dv) != hipSuccess) continue;
        const hipError_t e = drop_cached(c);
        if (e != hipSuccess) r = e;
    }
    (void)hipSetDevice(cur);
    return r;
}

namespace {

int bits_for(int64_t n) {
    int b = 1;
    while ((int64_t(1) << b) <= n) ++b;
    return b;
}

#define HIPCHK(expr)                                                      \
    do {                                                                  \
        hipError_t e_ = (expr);                                           \
        if (e_ != hipSuccess) {                                           \
            err = std::string(#expr) + ": " + hipGetErrorString(e_);      \
            return e_ == hipErrorOutOfMemory ? CCM_E_NOMEM : CCM_E_HIP;   \
        }                                                                 \
    } while (0)

ccm_status canonicalize(const int* src, const int* dst, const double* w, int64_t m, hipStream_t s,
                        OwnedGraph& out, int64_t& m_c, std::string& err) {
    DevMem key, key_s, val_s, uniq, agg, nruns, temp;
    HIPCHK(key.alloc(m * 8, s));
    HIPCHK(key_s.alloc(m * 8, s));
    HIPCHK(val_s.alloc(m * 8, s));
    HIPCHK(uniq.alloc(m * 8, s));
    HIPCHK(agg.alloc(m * 8, s));
    HIPCHK(nruns.alloc(8, s));
    hipLaunchKernelGGL(k_make_keys, dim3(flat_grid(m)), dim3(kBlock), 0, s, m, src, dst, w,
                       key.as<unsigned long long>());
    size_t b1 = 0, b2 = 0;
    HIPCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, b1, key.as<unsigned long long>(),
                                              key_s.as<unsigned long long>(), w,
                                              val_s.as<double>(), int(m), 0, 64, s));
    HIPCHK(hipcub::DeviceReduce::ReduceByKey(nullptr, b2, key_s.as<unsigned long long>(),
                                             uniq.as<unsigned long long>(), val_s.as<double>(),
                                             agg.as<double>(), nruns.as<int>(), hipcub::Sum(),
                                             int(m), s));
    HIPCHK(temp.alloc(b1 > b2 ? b1 : b2, s));
    HIPCHK(hipcub::DeviceRadixSort::SortPairs(temp.p, b1, key.as<unsigned long long>(),
                                              key_s.as<unsigned long long>(), w,
                                              val_s.as<double>(), int(m), 0, 64, s));
    HIPCHK(hipcub::DeviceReduce::ReduceByKey(temp.p, b2, key_s.as<unsigned long long>(),
                                             uniq.as<unsigned long long>(), val_s.as<double>(),
                                             agg.as<double>(), nruns.as<int>(), hipcub::Sum(),
                                             int(m), s));
    int runs = 0;
    HIPCHK(hipMemcpyAsync(&runs, nruns.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    unsigned long long last = 0;
    if (runs > 0) {
        HIPCHK(hipMemcpyAsync(&last, uniq.as<unsigned long long>() + runs - 1, 8,
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    m_c = runs - ((runs > 0 && last == ~0ull) ? 1 : 0);
    HIPCHK(out.src.alloc(m_c * 4, s));
    HIPCHK(out.dst.alloc(m_c * 4, s));
    HIPCHK(out.w.alloc(m_c * 8, s));
    if (m_c > 0) {
        hipLaunchKernelGGL(k_unpack, dim3(flat_grid(m_c)), dim3(kBlock), 0, s, m_c,
                           uniq.as<unsigned long long>(), out.src.as<int>(), out.dst.as<int>());
        HIPCHK(hipMemcpyAsync(out.w.p, agg.p, m_c * 8, hipMemcpyDeviceToDevice, s));
    }
    return CCM_OK;
}

ccm_status validate(const int* src, const int* dst, const double* w, int64_t m, int64_t n,
                    hipStream_t s, bool& canonical, std::string& err) {
    canonical = true;
    if (m == 0) return CCM_OK;
    DevMem flags;
    HIPCHK(flags.alloc(3 * sizeof(int), s));
    HIPCHK(hipMemsetAsync(flags.p, 0, 3 * sizeof(int), s));
    hipLaunchKernelGGL(k_validate, dim3(flat_grid(m)), dim3(kBlock), 0, s, m, n, src, dst, w,
                       flags.as<int>());
    int h[3] = {0, 0, 0};
    HIPCHK(hipMemcpyAsync(h, flags.p, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h[0]) {
        err = "edge endpoint outside [0, n)";
        return CCM_E_INVALID;
    }
    if (h[1]) {
        err = "edge weight negative or not finite";
        return CCM_E_INVALID;
    }
    canonical = h[2] == 0;
    return CCM_OK;
}

}  // namespace

__global__ __launch_bounds__(kBlock) void k_member_entries(int64_t n, const int* __restrict__ labels,
                                                           int* __restrict__ key,
                                                           Inc* __restrict__ val) {
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * kBlock) {
        key[i] = labels[i];
        val[i] = Inc{int(i), 0};
    }
}

ccm_status membership_build(const int* labels, int64_t n, int64_t K, int d, hipStream_t s,
                            OwnedGraph& out, std::string& err) {
    // rows: clusters; entries: member vertices in ascending order (a stable
    // sort by label keeps vertex order inside each cluster)
    DevMem key, val, temp, maxdeg;
    HIPCHK(key.alloc(size_t(n) * 4, s));
    HIPCHK(out.irow.alloc(size_t(n) * 4, s));
    HIPCHK(val.alloc(size_t(n) * 8, s));
    HIPCHK(out.inc.alloc(size_t(n) * 8, s));
    HIPCHK(out.inc_ptr.alloc(size_t(K + 1) * 4, s));
    HIPCHK(maxdeg.alloc(4, s));
    HIPCHK(hipMemsetAsync(maxdeg.p, 0, 4, s));
    hipLaunchKernelGGL(k_member_entries, dim3(flat_grid(n)), dim3(kBlock), 0, s, n, labels,
                       key.as<int>(), val.as<Inc>());
    size_t b = 0;
    const int nb = bits_for(K);
    HIPCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, b, key.as<int>(), out.irow.as<int>(),
                                              val.as<unsigned long long>(),
                                              out.inc.as<unsigned long long>(), int(n), 0, nb, s));
    HIPCHK(temp.alloc(b, s));
    HIPCHK(hipcub::DeviceRadixSort::SortPairs(temp.p, b, key.as<int>(), out.irow.as<int>(),
                                              val.as<unsigned long long>(),
                                              out.inc.as<unsigned long long>(), int(n), 0, nb, s));
    hipLaunchKernelGGL(k_inc_ptr, dim3(flat_grid(K + 1)), dim3(kBlock), 0, s, K, n,
                       out.irow.as<int>(), out.inc_ptr.as<int>(), maxdeg.as<int>());
    out.g.n = K;
    out.g.m = 0;
    out.g.nent = n;
    out.g.inc_ptr = out.inc_ptr.as<int>();
    out.g.inc = out.inc.as<Inc>();
    out.g.irow = out.irow.as<int>();
    return build_windows(d, s, out, err);
}

ccm_status graph_canonical_count(const int* src, const int* dst, const double* w, int64_t m,
                                 int64_t n, hipStream_t s, int64_t& m_canon, std::string& err) {
    bool canonical = true;
    ccm_status st = validate(src, dst, w, m, n, s, canonical, err);
    if (st != CCM_OK) return st;
    if (canonical) {
        m_canon = m;
        return CCM_OK;
    }
    OwnedGraph tmp;
    return canonicalize(src, dst, w, m, s, tmp, m_canon, err);
}

namespace {

// Re-sorts the vertex-ordered incidence lists of `out` (inc_ptr by vertex)
// into the locality order: connected components by their smallest vertex,
// inside a component by breadth-first level from that vertex, ties by
// vertex index.  Neighbours then sit near each other in the order, so the
// vertex kernels, which run windows of the order roughly in sequence, keep
// the rows they gather in the caches.  Sets vord, vrank, inc_ptr (by rank),
// inc, irow and epos.
ccm_status locality_order(OwnedGraph& out, hipStream_t s, std::string& err) {
    const int64_t n = out.g.n, m = out.g.m, cnt = out.g.nent;
    // components of the whole graph (every edge taken as fused)
    DevMem ones, comp, parent, scan, temp, ncl, first, lev, flag;
    HIPCHK(ones.alloc(std::max<int64_t>(m, 1) * 4, s));
    HIPCHK(comp.alloc(n * 4, s));
    HIPCHK(parent.alloc(n * 4, s));
    HIPCHK(scan.alloc((n + 1) * 4, s));
    const size_t tb = labels_temp_bytes(n);
    HIPCHK(temp.alloc(tb, s));
    HIPCHK(ncl.alloc(4, s));
    hipLaunchKernelGGL(k_fill_i32, dim3(flat_grid(m)), dim3(kBlock), 0, s, m, 1, ones.as<int>());
    launch_labels(n, m, out.g.src, out.g.dst, ones.as<int>(), parent.as<int>(), scan.as<int>(),
                  temp.p, tb, comp.as<int>(), ncl.as<int>(), s, out.g.inc_ptr, out.g.inc);
    HIPCHK(hipGetLastError());
    int K = 0;
    HIPCHK(hipMemcpyAsync(&K, ncl.p, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (K < 1 || K > n) {
        err = "internal: component count out of range in the locality order";
        return CCM_E_HIP;
    }
    // breadth-first levels from each component's smallest vertex
    HIPCHK(first.alloc(size_t(K) * 4, s));
    HIPCHK(lev.alloc(n * 4, s));
    HIPCHK(flag.alloc(4, s));
    hipLaunchKernelGGL(k_fill_i32, dim3(flat_grid(K)), dim3(kBlock), 0, s, int64_t(K), kUnreached,
                       first.as<int>());
    hipLaunchKernelGGL(k_comp_first, dim3(flat_grid(n)), dim3(kBlock), 0, s, n, comp.as<int>(),
                       first.as<int>());
    hipLaunchKernelGGL(k_bfs_init, dim3(flat_grid(n)), dim3(kBlock), 0, s, n, comp.as<int>(),
                       first.as<int>(), lev.as<int>());
    constexpr int kMaxLevels = 4096;  // deeper levels share one key (order only)
    const int64_t gpb = kBlock / kBfsLanes;
    const int gb = int(std::min<int64_t>((n + gpb - 1) / gpb, kMaxGrid));
    int depth = 0;
    for (int L = 0; L < kMaxLevels; ++L) {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, s, int64_t(1), 0, flag.as<int>());
        hipLaunchKernelGGL(k_bfs_step, dim3(gb), dim3(kBlock), 0, s, n, out.g.inc_ptr, out.g.inc,
                           L, lev.as<int>(), flag.as<int>());
        int h = 0;
        HIPCHK(hipMemcpyAsync(&h, flag.p, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        depth = L + 1;
        if (!h) break;
    }
    // vertices by (component, level), stable in vertex index
    DevMem key, key_s, val, tmp2;
    HIPCHK(key.alloc(n * 8, s));
    HIPCHK(key_s.alloc(n * 8, s));
    HIPCHK(val.alloc(n * 4, s));
    HIPCHK(out.vord.alloc(n * 4, s));
    HIPCHK(out.vrank.alloc(n * 4, s));
    hipLaunchKernelGGL(k_order_keys, dim3(flat_grid(n)), dim3(kBlock), 0, s, n, comp.as<int>(),
                       lev.as<int>(), depth, key.as<unsigned long long>(), val.as<int>());
    const int kb = bits_for(int64_t(K) * (depth + 1));
    size_t b = 0;
    HIPCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, b, key.as<unsigned long long>(),
                                              key_s.as<unsigned long long>(), val.as<int>(),
                                              out.vord.as<int>(), int(n), 0, kb, s));
    HIPCHK(tmp2.alloc(b, s));
    HIPCHK(hipcub::DeviceRadixSort::SortPairs(tmp2.p, b, key.as<unsigned long long>(),
                                              key_s.as<unsigned long long>(), val.as<int>(),
                                              out.vord.as<int>(), int(n), 0, kb, s));
    hipLaunchKernelGGL(k_rank_of, dim3(flat_grid(n)), dim3(kBlock), 0, s, n, out.vord.as<int>(),
                       out.vrank.as<int>());
    if (cnt > 0) {
        // entries by the rank of their vertex, stable (each list keeps its
        // ascending edge order)
        DevMem rk, rk_s, inc_s, tmp3, maxdeg;
        HIPCHK(rk.alloc(cnt * 4, s));
        HIPCHK(rk_s.alloc(cnt * 4, s));
        HIPCHK(inc_s.alloc(cnt * 8, s));
        HIPCHK(maxdeg.alloc(4, s));
        hipLaunchKernelGGL(k_entry_rank, dim3(flat_grid(cnt)), dim3(kBlock), 0, s, cnt,
                           out.g.irow, out.vrank.as<int>(), rk.as<int>());
        const int nb = bits_for(n);
        size_t b3 = 0;
        HIPCHK(hipcub::DeviceRadixSort::SortPairs(
            nullptr, b3, rk.as<int>(), rk_s.as<int>(), out.inc.as<unsigned long long>(),
            inc_s.as<unsigned long long>(), int(cnt), 0, nb, s));
        HIPCHK(tmp3.alloc(b3, s));
        HIPCHK(hipcub::DeviceRadixSort::SortPairs(
            tmp3.p, b3, rk.as<int>(), rk_s.as<int>(), out.inc.as<unsigned long long>(),
            inc_s.as<unsigned long long>(), int(cnt), 0, nb, s));
        HIPCHK(hipMemcpyAsync(out.inc.p, inc_s.p, cnt * 8, hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_entry_vertex, dim3(flat_grid(cnt)), dim3(kBlock), 0, s, cnt,
                           rk_s.as<int>(), out.vord.as<int>(), out.irow.as<int>());
        hipLaunchKernelGGL(k_epos, dim3(flat_grid(cnt)), dim3(kBlock), 0, s, cnt,
                           out.inc.as<Inc>(), out.epos.as<int>());
        HIPCHK(hipMemsetAsync(maxdeg.p, 0, 4, s));
        hipLaunchKernelGGL(k_inc_ptr, dim3(flat_grid(n + 1)), dim3(kBlock), 0, s, n, cnt,
                           rk_s.as<int>(), out.inc_ptr.as<int>(), maxdeg.as<int>());
        HIPCHK(hipStreamSynchronize(s));
    }
    out.g.vord = out.vord.as<int>();
    out.g.vrank = out.vrank.as<int>();
    return CCM_OK;
}

}  // namespace

ccm_status graph_build(const int* src, const int* dst, const double* w, int64_t m, int64_t n,
                       int d, bool require_canonical, hipStream_t s, OwnedGraph& out,
                       std::string& err, int locality, int qk, int chunk) {
    if (n < 1 || n > (int64_t(1) << 30) || m < 0 || m > (int64_t(1) << 30)) {
        err = "graph size out of range";
        return CCM_E_INVALID;
    }
    bool canonical = true;
    ccm_status st = validate(src, dst, w, m, n, s, canonical, err);
    if (st != CCM_OK) return st;
    int64_t mc = m;
    if (!canonical) {
        if (require_canonical) {
            err = "edges must be canonical (src < dst, sorted by (src, dst), w > 0)";
            return CCM_E_INVALID;
        }
        st = canonicalize(src, dst, w, m, s, out, mc, err);
        if (st != CCM_OK) return st;
        out.g.src = out.src.as<int>();
        out.g.dst = out.dst.as<int>();
        out.g.w = out.w.as<double>();
    } else {
        out.g.src = src;
        out.g.dst = dst;
        out.g.w = w;
    }
    out.g.n = n;
    out.g.m = mc;
    // vertex-major incidence lists: entries (vertex, edge) sorted stably by
    // vertex keep each list in ascending edge order
    const int64_t cnt = 2 * mc;
    DevMem vk, vv, temp, maxdeg;
    HIPCHK(vk.alloc(cnt * 4, s));
    HIPCHK(vv.alloc(cnt * 8, s));
    HIPCHK(out.irow.alloc(std::max<int64_t>(cnt, 1) * 4, s));
    HIPCHK(out.epos.alloc(std::max<int64_t>(cnt, 1) * 4, s));
    HIPCHK(out.inc.alloc(cnt * 8, s));
    HIPCHK(out.inc_ptr.alloc((n + 1) * 4, s));
    HIPCHK(maxdeg.alloc(4, s));
    HIPCHK(hipMemsetAsync(maxdeg.p, 0, 4, s));
    if (mc > 0) {
        hipLaunchKernelGGL(k_inc_entries, dim3(flat_grid(mc)), dim3(kBlock), 0, s, mc, out.g.src,
                           out.g.dst, vk.as<int>(), vv.as<Inc>());
        size_t b = 0;
        const int nb = bits_for(n);
        HIPCHK(hipcub::DeviceRadixSort::SortPairs(
            nullptr, b, vk.as<int>(), out.irow.as<int>(), vv.as<unsigned long long>(),
            out.inc.as<unsigned long long>(), int(cnt), 0, nb, s));
        HIPCHK(temp.alloc(b, s));
        HIPCHK(hipcub::DeviceRadixSort::SortPairs(
            temp.p, b, vk.as<int>(), out.irow.as<int>(), vv.as<unsigned long long>(),
            out.inc.as<unsigned long long>(), int(cnt), 0, nb, s));
        hipLaunchKernelGGL(k_epos, dim3(flat_grid(cnt)), dim3(kBlock), 0, s, cnt,
                           out.inc.as<Inc>(), out.epos.as<int>());
    }
    hipLaunchKernelGGL(k_inc_ptr, dim3(flat_grid(n + 1)), dim3(kBlock), 0, s, n, cnt,
                       out.irow.as<int>(), out.inc_ptr.as<int>(), maxdeg.as<int>());
    int md = 0;
    HIPCHK(hipMemcpyAsync(&md, maxdeg.p, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    out.g.inc_ptr = out.inc_ptr.as<int>();
    out.g.inc = out.inc.as<Inc>();
    out.g.irow = out.irow.as<int>();
    out.g.epos = out.epos.as<int>();
    out.g.max_deg = md;
    out.g.nent = cnt;
    if (locality > 0 || (locality < 0 && n * int64_t(d) >= kLocalityMin)) {
        st = locality_order(out, s, err);
        if (st != CCM_OK) return st;
    }
    return build_windows(d, s, out, err, qk, chunk);
}

ccm_status build_windows(int d, hipStream_t s, OwnedGraph& out, std::string& err, int qk,
                         int chunk) {
    // Vertex-aligned windows of the incidence array, packed greedily on the
    // host: consecutive whole vertices while the window holds at most S
    // entries; a vertex with more than S entries (a hub) forms a window of
    // its own.  Then the isolated vertices.
    const int64_t n = out.g.n;
    const int64_t cnt = out.g.nent;
    if (cnt > 0 && (!out.g.inc || !out.g.irow || !out.g.inc_ptr)) {
        err = "internal: incidence lists incomplete (entries, vertex ids or offsets missing)";
        return CCM_E_HIP;
    }
    const int64_t S = window_for(d, qk, chunk);
    std::vector<int> ptr(size_t(n) + 1), vord;
    HIPCHK(hipMemcpyAsync(ptr.data(), out.g.inc_ptr, ptr.size() * 4, hipMemcpyDeviceToHost, s));
    if (out.g.vord) {
        vord.resize(size_t(n));
        HIPCHK(hipMemcpyAsync(vord.data(), out.g.vord, size_t(n) * 4, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    std::vector<int2> win;
    std::vector<int> iso;
    win.reserve(size_t(cnt / S + 2));
    int64_t ws = 0;
    for (int64_t r = 0; r < n; ++r) {
        const int64_t b = ptr[r], e = ptr[r + 1];
        if (e == b) {
            iso.push_back(vord.empty() ? int(r) : vord[size_t(r)]);
            continue;
        }
        if (e - ws > S && b > ws) {
            win.push_back(int2{int(ws), int(b)});
            ws = b;
        }
    }
    if (cnt > ws) win.push_back(int2{int(ws), int(cnt)});
    if (out.g.vord) {
        // hub windows first (their long serial work starts early), then the
        // locality order: workgroups are dispatched in window order, so the
        // windows in flight at any time are neighbours in that order
        std::stable_partition(win.begin(), win.end(),
                              [S](const int2& a) { return int64_t(a.y) - a.x > S; });
    } else {
        // input order: longest first (short windows fill the tail), ties in
        // entry order
        std::stable_sort(win.begin(), win.end(),
                         [](const int2& a, const int2& b) { return a.y - a.x > b.y - b.x; });
    }
    HIPCHK(out.win.alloc(std::max<size_t>(win.size(), 1) * 8, s));
    HIPCHK(out.iso.alloc(std::max<size_t>(iso.size(), 1) * 4, s));
    if (!win.empty())
        HIPCHK(hipMemcpyAsync(out.win.p, win.data(), win.size() * 8, hipMemcpyHostToDevice, s));
    if (!iso.empty())
        HIPCHK(hipMemcpyAsync(out.iso.p, iso.data(), iso.size() * 4, hipMemcpyHostToDevice, s));
    // the host vectors die on return: wait for the copies
    HIPCHK(hipStreamSynchronize(s));
    out.g.nwin = int64_t(win.size());
    out.g.niso = int64_t(iso.size());
    out.g.win = out.win.as<int2>();
    out.g.iso = out.iso.as<int>();
    return CCM_OK;
}

}  // namespace ccm
