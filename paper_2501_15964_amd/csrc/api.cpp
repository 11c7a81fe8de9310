// C ABI entry points of libccm (declared in include/ccm.h): argument checks,
// error reporting and dispatch to the device graph, solvers and kernels.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "knn.hpp"
#include "solver.hpp"
#include "vjp.hpp"

using namespace ccm;

namespace {

thread_local std::string g_err;

ccm_status fail(ccm_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

#define HIPCHK_API(expr)                                                              \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(e_ == hipErrorOutOfMemory ? CCM_E_NOMEM : CCM_E_HIP,          \
                        std::string(#expr) + ": " + hipGetErrorString(e_));           \
    } while (0)

bool q_kind(double q, int& qk) {
    if (q == 1.0) qk = kQ1;
    else if (q == 2.0) qk = kQ2;
    else if (std::isinf(q) && q > 0) qk = kQInf;
    else return false;
    return true;
}

ccm_status check_dims(int64_t n, int64_t d) {
    if (n < 1) return fail(CCM_E_INVALID, "n must be >= 1");
    if (d < 1) return fail(CCM_E_INVALID, "d must be >= 1");
    if (!row_supported(d)) return fail(CCM_E_UNSUPPORTED, "d above 1024 is not supported");
    if (n > (int64_t(1) << 30)) return fail(CCM_E_INVALID, "n too large");
    return CCM_OK;
}

// finite-ness of a device array: a flag set by a device pass over it
ccm_status check_finite(const double* p, int64_t count, hipStream_t s, const char* what) {
    if (count <= 0) return CCM_OK;
    DevMem flag;
    HIPCHK_API(flag.alloc(4, s));
    HIPCHK_API(hipMemsetAsync(flag.p, 0, 4, s));
    launch_flag_nonfinite(p, count, flag.as<int>(), s);
    int h = 0;
    HIPCHK_API(hipMemcpyAsync(&h, flag.p, 4, hipMemcpyDeviceToHost, s));
    HIPCHK_API(hipStreamSynchronize(s));
    if (h) return fail(CCM_E_INVALID, std::string(what) + " contains NaN or Inf");
    return CCM_OK;
}

ccm_options defaults() {
    ccm_options o;
    std::memset(&o, 0, sizeof(o));
    o.method = CCM_SSNAL;
    o.max_outer = 300;
    o.max_newton = 60;
    o.cg_max_iter = 500;
    o.max_iter = 20000;
    o.check_every = 10;
    o.cg_chunk = 8;
    o.profile = 0;
    o.sigma0 = 0.0;
    o.sigma_max = 1e4;
    o.tau = 1.618;
    o.time_budget_s = 0.0;
    o.locality = -1;
    o.dual_scale = -1;
    return o;
}

// ---- work space of the entry point that allocates nothing ---------------------
// A fixed device array: each device that runs the library holds its own copy
// until the process ends.  In host code `scratch` only names the symbol; its
// device address (one per device) comes from hipGetSymbolAddress.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
constexpr int64_t kNoAllocMaxN = int64_t(1) << 22;
constexpr int64_t kNoAllocMaxM = int64_t(1) << 23;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

ccm_status noalloc_scratch(unsigned char** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* ptr[kMaxDevices] = {};
    int dev = 0;
    HIPCHK_API(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(CCM_E_UNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(CCM_E_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                       hipGetErrorString(e));
        ptr[dev] = p;
    }
    *out = static_cast<unsigned char*>(ptr[dev]);
    return CCM_OK;
}

// byte offsets of ccm_labels_noalloc's buffers in the array (256-aligned)
struct LabelsScratch {
    size_t spread, S, nc, fused, parent, rank, temp, temp_bytes, total;
};
LabelsScratch labels_scratch(int64_t n, int d, int64_t m) {
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    LabelsScratch L{};
    size_t at = 0;
    L.spread = at;
    at += up(size_t(spread_work_size(n, d)) * 8);
    L.S = at;
    at += up(8);
    L.nc = at;
    at += up(4);
    L.fused = at;
    at += up(size_t(std::max<int64_t>(m, 1)) * 4);
    L.parent = at;
    at += up(size_t(n) * 4);
    L.rank = at;
    at += up(size_t(n + 1) * 4);
    L.temp = at;
    L.temp_bytes = labels_temp_bytes(n);
    at += up(L.temp_bytes);
    L.total = at;
    return L;
}

// concurrent (q, d) groups of ccm_solve_path_batched
constexpr int kBatchedStreams = 4;

// One (q, d) group of batched instances: their block-diagonal union solved
// by one Solver on stream `stream`.  Errors set g_err of the calling thread.
ccm_status solve_group(const ccm_instance* inst_host, const std::vector<int>& ids, int qk, int d,
                       const double* A_all, const int32_t* src_all, const int32_t* dst_all,
                       const double* w_all, const double* gammas_host, int32_t n_gamma,
                       double tol, const ccm_options& o, double* X_out_all, int32_t* labels_all,
                       int32_t* n_clusters_host, double* kkt_host, int32_t* status_host,
                       hipStream_t stream) {
    const int S = int(ids.size());
    BatchSpec b;
    b.S = S;
    b.vseg.assign(S + 1, 0);
    b.eseg.assign(S + 1, 0);
    std::vector<int64_t> xoff(S), loff(S);
    for (int k = 0; k < S; ++k) {
        const ccm_instance& I = inst_host[ids[k]];
        b.vseg[k + 1] = b.vseg[k] + I.n;
        b.eseg[k + 1] = b.eseg[k] + I.m;
        xoff[k] = I.x_offset;
        loff[k] = I.l_offset;
    }
    const int64_t nU = b.vseg[S], mU = b.eseg[S];
    if (nU > (int64_t(1) << 30) || mU > (int64_t(1) << 30))
        return fail(CCM_E_INVALID, "batched group too large");
    DevMem Au, su, du, wu, seg, bad;
    HIPCHK_API(Au.alloc(size_t(nU) * d * 8, stream));
    HIPCHK_API(su.alloc(size_t(std::max<int64_t>(mU, 1)) * 4, stream));
    HIPCHK_API(du.alloc(size_t(std::max<int64_t>(mU, 1)) * 4, stream));
    HIPCHK_API(wu.alloc(size_t(std::max<int64_t>(mU, 1)) * 8, stream));
    HIPCHK_API(seg.alloc(size_t(4 * S + 2) * 8, stream));
    HIPCHK_API(bad.alloc(4, stream));
    HIPCHK_API(hipMemsetAsync(bad.p, 0, 4, stream));
    for (int k = 0; k < S; ++k) {
        const ccm_instance& I = inst_host[ids[k]];
        HIPCHK_API(hipMemcpyAsync(Au.as<double>() + b.vseg[k] * d, A_all + I.a_offset,
                                  size_t(I.n) * d * 8, hipMemcpyDeviceToDevice, stream));
        launch_offset_edges(I.m, src_all + I.e_offset, dst_all + I.e_offset,
                            w_all + I.e_offset, int(b.vseg[k]), int(I.n),
                            su.as<int>() + b.eseg[k], du.as<int>() + b.eseg[k],
                            wu.as<double>() + b.eseg[k], bad.as<int>(), stream);
    }
    int64_t* sd = seg.as<int64_t>();
    HIPCHK_API(hipMemcpyAsync(sd, b.vseg.data(), size_t(S + 1) * 8, hipMemcpyHostToDevice,
                              stream));
    HIPCHK_API(hipMemcpyAsync(sd + (S + 1), b.eseg.data(), size_t(S + 1) * 8,
                              hipMemcpyHostToDevice, stream));
    HIPCHK_API(hipMemcpyAsync(sd + 2 * (S + 1), xoff.data(), size_t(S) * 8,
                              hipMemcpyHostToDevice, stream));
    HIPCHK_API(hipMemcpyAsync(sd + 2 * (S + 1) + S, loff.data(), size_t(S) * 8,
                              hipMemcpyHostToDevice, stream));
    int hbad = 0;
    HIPCHK_API(hipMemcpyAsync(&hbad, bad.p, 4, hipMemcpyDeviceToHost, stream));
    HIPCHK_API(hipStreamSynchronize(stream));
    if (hbad) return fail(CCM_E_INVALID, "instance edges must be canonical with local endpoints");
    ccm_status st = check_finite(Au.as<double>(), nU * d, stream, "A");
    if (st != CCM_OK) return st;
    b.vseg_dev = sd;
    b.eseg_dev = sd + (S + 1);
    b.xoff_dev = sd + 2 * (S + 1);
    b.loff_dev = sd + 2 * (S + 1) + S;
    b.inst = ids;
    b.X_out_all = X_out_all;
    b.labels_all = labels_all;
    b.n_clusters_host = n_clusters_host;
    b.kkt_host = kkt_host;
    b.status_host = status_host;
    std::string err;
    OwnedGraph og;
    st = graph_build(su.as<int>(), du.as<int>(), wu.as<double>(), mU, nU, d, true, stream, og,
                     err, o.locality, qk, o.window_chunk);
    if (st != CCM_OK) return fail(st, err);
    Solver solver(og.g, d, qk, Au.as<double>(), stream, o, tol, err);
    st = solver.run_batched(gammas_host, n_gamma, b);
    if (st != CCM_OK) return fail(st, err);
    return CCM_OK;
}

}  // namespace

extern "C" {

const char* ccm_status_string(ccm_status s) {
    switch (s) {
        case CCM_OK: return "ok";
        case CCM_E_INVALID: return "invalid argument";
        case CCM_E_UNSUPPORTED: return "unsupported";
        case CCM_E_HIP: return "HIP runtime error";
        case CCM_E_NOMEM: return "out of device memory";
        case CCM_E_CAPACITY: return "output capacity too small";
        case CCM_E_NOT_CONVERGED: return "iterative solve did not converge";
        default: return "unknown status";
    }
}

const char* ccm_last_error(void) { return g_err.c_str(); }

const char* ccm_version(void) { return "libccm 0.1 gfx950"; }

ccm_status ccm_release_workspace(void) {
    g_err.clear();
    HIPCHK_API(release_workspace());
    return CCM_OK;
}

ccm_options ccm_default_options(void) { return defaults(); }

ccm_status ccm_build_knn_graph(const double* A, int64_t n, int64_t d, int32_t k, double phi,
                               int32_t* src, int32_t* dst, double* w, int64_t m_cap,
                               int64_t* m_out_host, double* phi_out_host, hipStream_t stream) {
    g_err.clear();
    if (!A || !src || !dst || !w || !m_out_host) return fail(CCM_E_INVALID, "null argument");
    if (n < 2) return fail(CCM_E_INVALID, "n must be >= 2");
    if (d < 1) return fail(CCM_E_INVALID, "d must be >= 1");
    if (n > (int64_t(1) << 30) || d > (int64_t(1) << 20)) return fail(CCM_E_INVALID, "too large");
    if (k < 1 || k > 32 || k > n - 1) return fail(CCM_E_INVALID, "need 1 <= k <= min(n - 1, 32)");
    if (m_cap < 0) return fail(CCM_E_INVALID, "m_cap < 0");
    if (std::isnan(phi) || std::isinf(phi)) return fail(CCM_E_INVALID, "phi must be finite");
    ccm_status st = check_finite(A, n * d, stream, "A");
    if (st != CCM_OK) return st;
    std::string err;
    int64_t mo = 0;
    double po = 0;
    st = knn_graph(A, n, int(d), k, phi, src, dst, w, m_cap, mo, po, stream, err);
    *m_out_host = mo;
    if (st != CCM_OK) return fail(st, err);
    if (phi_out_host) *phi_out_host = po;
    return CCM_OK;
}

ccm_status ccm_build_knn_graph_u8(const uint8_t* K, int64_t n, int64_t d, double scale, int32_t k,
                                  double phi, int32_t* src, int32_t* dst, double* w,
                                  int64_t m_cap, int64_t* m_out_host, double* phi_out_host,
                                  hipStream_t stream) {
    g_err.clear();
    if (!K || !src || !dst || !w || !m_out_host) return fail(CCM_E_INVALID, "null argument");
    if (n < 2) return fail(CCM_E_INVALID, "n must be >= 2");
    if (d < 1 || d > 2048) return fail(CCM_E_INVALID, "need 1 <= d <= 2048");
    if (n > (int64_t(1) << 30)) return fail(CCM_E_INVALID, "too large");
    if (k < 1 || k > 32 || k > n - 1) return fail(CCM_E_INVALID, "need 1 <= k <= min(n - 1, 32)");
    if (!(scale > 0) || !std::isfinite(scale)) return fail(CCM_E_INVALID, "scale must be > 0");
    if (m_cap < 0) return fail(CCM_E_INVALID, "m_cap < 0");
    if (std::isnan(phi) || std::isinf(phi)) return fail(CCM_E_INVALID, "phi must be finite");
    std::string err;
    int64_t mo = 0;
    double po = 0;
    ccm_status st = knn_graph_u8(K, n, int(d), scale, k, phi, src, dst, w, m_cap, mo, po, stream,
                                 err);
    *m_out_host = mo;
    if (st != CCM_OK) return fail(st, err);
    if (phi_out_host) *phi_out_host = po;
    return CCM_OK;
}

ccm_status ccm_canonical_edge_count(const int32_t* src, const int32_t* dst, const double* w,
                                    int64_t m, int64_t n, int64_t* m_canon_host,
                                    hipStream_t stream) {
    g_err.clear();
    if (n < 1 || m < 0) return fail(CCM_E_INVALID, "n >= 1 and m >= 0 required");
    if (m > 0 && (!src || !dst || !w)) return fail(CCM_E_INVALID, "null edge array");
    if (!m_canon_host) return fail(CCM_E_INVALID, "null m_canon_host");
    std::string err;
    int64_t mc = 0;
    ccm_status st = graph_canonical_count(src, dst, w, m, n, stream, mc, err);
    if (st != CCM_OK) return fail(st, err);
    *m_canon_host = mc;
    return CCM_OK;
}

ccm_status ccm_solve_path(const double* A, int64_t n, int64_t d, const int32_t* src,
                          const int32_t* dst, const double* w, int64_t m,
                          const double* gammas_host, int32_t n_gamma, double q, double tol,
                          const ccm_options* opts, double* X_out, double* U_out,
                          int32_t* labels_out, int32_t* n_clusters_host, double* kkt_host,
                          int32_t* status_host, ccm_stats* stats_host, const double* X_warm,
                          const double* U_warm, hipStream_t stream) {
    g_err.clear();
    ccm_status st = check_dims(n, d);
    if (st != CCM_OK) return st;
    if (!A) return fail(CCM_E_INVALID, "A is null");
    if (!X_out) return fail(CCM_E_INVALID, "X_out is null");
    if (m < 0) return fail(CCM_E_INVALID, "m < 0");
    if (m > 0 && (!src || !dst || !w)) return fail(CCM_E_INVALID, "null edge array");
    if (n_gamma < 0 || (n_gamma > 0 && !gammas_host))
        return fail(CCM_E_INVALID, "bad gamma list");
    for (int t = 0; t < n_gamma; ++t)
        if (!std::isfinite(gammas_host[t]) || gammas_host[t] < 0)
            return fail(CCM_E_INVALID, "gamma values must be finite and >= 0");
    int qk = 0;
    if (!q_kind(q, qk)) return fail(CCM_E_UNSUPPORTED, "q must be 1, 2 or inf");
    if (!(tol > 0) || !std::isfinite(tol)) return fail(CCM_E_INVALID, "tol must be > 0");
    ccm_options o = opts ? *opts : defaults();
    if (o.method != CCM_SSNAL && o.method != CCM_ADMM && o.method != CCM_AMA &&
        o.method != CCM_HPR)
        return fail(CCM_E_INVALID, "unknown method");
    if (o.max_outer < 1 || o.max_newton < 1 || o.cg_max_iter < 1 || o.max_iter < 1)
        return fail(CCM_E_INVALID, "iteration limits must be >= 1");
    if (o.sigma0 <= 0) o.sigma0 = 1.0;
    if (!(o.sigma_max >= o.sigma0)) o.sigma_max = o.sigma0;
    if (!(o.tau > 0 && o.tau < 1.6181)) return fail(CCM_E_INVALID, "tau must be in (0, 1.618]");
    if (o.window_chunk < 0 || o.window_chunk > 4096)
        return fail(CCM_E_INVALID, "window_chunk must be in [0, 4096]");
    if (o.dual_scale < -1 || o.dual_scale > 1)
        return fail(CCM_E_INVALID, "dual_scale must be -1, 0 or 1");
    st = check_finite(A, n * d, stream, "A");
    if (st != CCM_OK) return st;
    if (n_gamma == 0) return CCM_OK;
    std::string err;
    OwnedGraph og;
    st = graph_build(src, dst, w, m, n, int(d), false, stream, og, err, o.locality, qk,
                     o.window_chunk);
    if (st != CCM_OK) return fail(st, err);
    Solver solver(og.g, int(d), qk, A, stream, o, tol, err);
    st = solver.run_path(gammas_host, n_gamma, X_warm, U_warm, X_out, U_out, labels_out,
                         n_clusters_host, kkt_host, status_host, stats_host);
    if (st != CCM_OK) return fail(st, err);
    HIPCHK_API(hipStreamSynchronize(stream));
    return CCM_OK;
}

ccm_status ccm_solve_path_batched(const ccm_instance* inst_host, int32_t n_inst,
                                  const double* A_all, const int32_t* src_all,
                                  const int32_t* dst_all, const double* w_all,
                                  const double* gammas_host, int32_t n_gamma, double tol,
                                  const ccm_options* opts, double* X_out_all, int32_t* labels_all,
                                  int32_t* n_clusters_host, double* kkt_host,
                                  int32_t* status_host, hipStream_t stream) {
    g_err.clear();
    if (n_inst < 0 || (n_inst > 0 && !inst_host)) return fail(CCM_E_INVALID, "bad instances");
    if (!A_all || !X_out_all) return fail(CCM_E_INVALID, "null A_all or X_out_all");
    if (n_gamma < 0 || (n_gamma > 0 && !gammas_host))
        return fail(CCM_E_INVALID, "bad gamma list");
    for (int t = 0; t < n_gamma; ++t)
        if (!std::isfinite(gammas_host[t]) || gammas_host[t] < 0)
            return fail(CCM_E_INVALID, "gamma values must be finite and >= 0");
    if (!(tol > 0) || !std::isfinite(tol)) return fail(CCM_E_INVALID, "tol must be > 0");
    ccm_options o = opts ? *opts : defaults();
    o.method = CCM_SSNAL;
    if (o.max_outer < 1 || o.max_newton < 1 || o.cg_max_iter < 1)
        return fail(CCM_E_INVALID, "iteration limits must be >= 1");
    if (o.window_chunk < 0 || o.window_chunk > 4096)
        return fail(CCM_E_INVALID, "window_chunk must be in [0, 4096]");
    if (o.dual_scale < -1 || o.dual_scale > 1)
        return fail(CCM_E_INVALID, "dual_scale must be -1, 0 or 1");
    if (o.sigma0 <= 0) o.sigma0 = 1.0;
    if (!(o.sigma_max >= o.sigma0)) o.sigma_max = o.sigma0;
    // group instances by (q, d)
    std::map<std::pair<int, int64_t>, std::vector<int>> groups;
    for (int i = 0; i < n_inst; ++i) {
        const ccm_instance& I = inst_host[i];
        ccm_status st = check_dims(I.n, I.d);
        if (st != CCM_OK) return fail(st, "instance " + std::to_string(i) + ": " + g_err);
        int qk = 0;
        if (!q_kind(I.q, qk))
            return fail(CCM_E_UNSUPPORTED, "instance " + std::to_string(i) + ": q must be 1, 2 or inf");
        if (I.m < 0 || I.a_offset < 0 || I.e_offset < 0 || I.x_offset < 0 || I.l_offset < 0)
            return fail(CCM_E_INVALID, "instance " + std::to_string(i) + ": negative size/offset");
        if (I.m > 0 && (!src_all || !dst_all || !w_all))
            return fail(CCM_E_INVALID, "null edge arrays");
        groups[{qk, I.d}].push_back(i);
    }
    if (n_gamma == 0) return CCM_OK;
    // Groups are independent problems; each is latency-bound on its own
    // (small kernels and host round trips), so several run at once, each on
    // a stream of its own, largest first.
    std::vector<std::pair<int, const std::vector<int>*>> order;  // (key index, members)
    std::vector<std::pair<int, int64_t>> keys;
    std::vector<double> work;
    for (auto& kv : groups) {
        double wk = 0;
        for (int i : kv.second) wk += double(inst_host[i].m + inst_host[i].n) * double(kv.first.second);
        keys.push_back(kv.first);
        order.push_back({int(keys.size()) - 1, &kv.second});
        work.push_back(wk);
    }
    std::sort(order.begin(), order.end(),
              [&](const auto& a, const auto& b) { return work[a.first] > work[b.first]; });
    auto run_group = [&](int k, hipStream_t gs) -> ccm_status {
        const int qk = keys[order[k].first].first;
        const int d = int(keys[order[k].first].second);
        const std::vector<int>& ids = *order[k].second;
        return solve_group(inst_host, ids, qk, d, A_all, src_all, dst_all, w_all, gammas_host,
                           n_gamma, tol, o, X_out_all, labels_all, n_clusters_host, kkt_host,
                           status_host, gs);
    };
    int dev = 0;
    HIPCHK_API(hipGetDevice(&dev));
    hipEvent_t ready = nullptr;
    HIPCHK_API(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    struct EvFree {
        hipEvent_t e;
        ~EvFree() { (void)hipEventDestroy(e); }
    } evf{ready};
    HIPCHK_API(hipEventRecord(ready, stream));
    const int G = int(order.size());
    const int nthreads = std::min(G, kBatchedStreams);
    std::vector<ccm_status> gst(static_cast<size_t>(G), CCM_OK);
    std::vector<std::string> gerr(static_cast<size_t>(G));
    std::atomic<int> next{0};
    auto worker = [&]() {
        if (hipSetDevice(dev) != hipSuccess) return;
        hipStream_t gs = nullptr;
        if (hipStreamCreateWithFlags(&gs, hipStreamNonBlocking) != hipSuccess) {
            const int k = next++;
            if (k < G) {
                gst[k] = CCM_E_HIP;
                gerr[k] = "hipStreamCreateWithFlags failed";
            }
            return;
        }
        (void)hipStreamWaitEvent(gs, ready, 0);
        for (int k = next++; k < G; k = next++) {
            ccm_status st = CCM_OK;
            try {
                st = run_group(k, gs);
            } catch (const std::bad_alloc&) {
                st = fail(CCM_E_NOMEM, "host allocation failed");
            } catch (...) {
                st = fail(CCM_E_HIP, "unexpected exception in a batched group");
            }
            if (st != CCM_OK) {
                gst[k] = st;
                gerr[k] = g_err;
            }
            if (hipStreamSynchronize(gs) != hipSuccess && gst[k] == CCM_OK) {
                gst[k] = CCM_E_HIP;
                gerr[k] = "group stream failed";
            }
        }
        (void)hipStreamSynchronize(gs);
        (void)hipStreamDestroy(gs);
    };
    std::vector<std::thread> pool;
    for (int t = 0; t < nthreads; ++t) pool.emplace_back(worker);
    for (auto& th : pool) th.join();
    if (next.load() < G) return fail(CCM_E_HIP, "batched worker threads did not start");
    for (int k = 0; k < G; ++k)
        if (gst[k] != CCM_OK) return fail(gst[k], gerr[k]);
    HIPCHK_API(hipStreamSynchronize(stream));
    return CCM_OK;
}

ccm_status ccm_path_vjp(const double* A, int64_t n, int64_t d, const int32_t* src,
                        const int32_t* dst, const double* w, int64_t m, double gamma, double q,
                        const double* X, const int32_t* labels, const double* dL_dX,
                        double* dL_dA, double* dL_dlogw, double* dL_dgamma_host, double tol,
                        int32_t max_iter, int32_t* iters_host, hipStream_t stream) {
    g_err.clear();
    ccm_status st = check_dims(n, d);
    if (st != CCM_OK) return st;
    if (q != 2.0) return fail(CCM_E_UNSUPPORTED, "the adjoint is implemented for q = 2");
    if (!A || !X || !labels || !dL_dX || !dL_dA) return fail(CCM_E_INVALID, "null argument");
    if (m < 0 || (m > 0 && (!src || !dst || !w))) return fail(CCM_E_INVALID, "bad edges");
    if (!(gamma >= 0) || !std::isfinite(gamma)) return fail(CCM_E_INVALID, "bad gamma");
    if (!(tol > 0) || max_iter < 1) return fail(CCM_E_INVALID, "tol > 0, max_iter >= 1");
    st = check_finite(X, n * d, stream, "X");
    if (st != CCM_OK) return st;
    st = check_finite(dL_dX, n * d, stream, "dL_dX");
    if (st != CCM_OK) return st;
    std::string err;
    int it = 0;
    st = path_vjp(A, n, int(d), src, dst, w, m, gamma, X, labels, dL_dX, dL_dA, dL_dlogw,
                  dL_dgamma_host, tol, max_iter, &it, stream, err);
    if (iters_host) *iters_host = it;
    if (st != CCM_OK) return fail(st, err);
    return CCM_OK;
}

ccm_status ccm_op_gather(const double* X, int64_t n, int64_t d, const int32_t* src,
                         const int32_t* dst, int64_t m, double* Y, hipStream_t stream) {
    g_err.clear();
    ccm_status st = check_dims(n, d);
    if (st != CCM_OK) return st;
    if (m < 0) return fail(CCM_E_INVALID, "m < 0");
    if (m == 0) return CCM_OK;
    DevGraph g;
    g.n = n;
    g.m = m;
    g.src = src;
    g.dst = dst;
    launch_gather(g, int(d), X, Y, stream);
    HIPCHK_API(hipGetLastError());
    return CCM_OK;
}

ccm_status ccm_op_project(const double* Y, int64_t m, int64_t d, const double* w, double gamma,
                          double q, double* Pi, hipStream_t stream) {
    g_err.clear();
    int qk = 0;
    if (!q_kind(q, qk)) return fail(CCM_E_UNSUPPORTED, "q must be 1, 2 or inf");
    if (m < 0 || d < 1 || !row_supported(d)) return fail(CCM_E_INVALID, "bad sizes");
    if (!(gamma >= 0) || !std::isfinite(gamma)) return fail(CCM_E_INVALID, "bad gamma");
    if (m == 0) return CCM_OK;
    launch_project(m, int(d), qk, Y, w, gamma, false, Pi, stream);
    HIPCHK_API(hipGetLastError());
    return CCM_OK;
}

ccm_status ccm_op_prox(const double* Y, int64_t m, int64_t d, const double* w, double gamma,
                       double q, double* Z, hipStream_t stream) {
    g_err.clear();
    int qk = 0;
    if (!q_kind(q, qk)) return fail(CCM_E_UNSUPPORTED, "q must be 1, 2 or inf");
    if (m < 0 || d < 1 || !row_supported(d)) return fail(CCM_E_INVALID, "bad sizes");
    if (!(gamma >= 0) || !std::isfinite(gamma)) return fail(CCM_E_INVALID, "bad gamma");
    if (m == 0) return CCM_OK;
    launch_project(m, int(d), qk, Y, w, gamma, true, Z, stream);
    HIPCHK_API(hipGetLastError());
    return CCM_OK;
}

ccm_status ccm_op_scatter(const double* Z, int64_t m, int64_t d, const int32_t* src,
                          const int32_t* dst, int64_t n, double* out, hipStream_t stream) {
    g_err.clear();
    ccm_status st = check_dims(n, d);
    if (st != CCM_OK) return st;
    std::string err;
    OwnedGraph og;
    std::vector<double> ones;
    DevMem wbuf;
    // unit weights: only the incidence structure is used
    if (m > 0) {
        HIPCHK_API(wbuf.alloc(size_t(m) * 8, stream));
        launch_fill(wbuf.as<double>(), m, 1.0, stream);
    }
    st = graph_build(src, dst, wbuf.as<double>(), m, n, int(d), true, stream, og, err);
    if (st != CCM_OK) return fail(st, err);
    DevMem part;
    HIPCHK_API(part.alloc(partials_for(og.g) * 8, stream));
    launch_scatter(og.g, int(d), kQ2, 0.0, nullptr, 0.0, nullptr, 1.0, Z, out, false, Payload{},
                   0.0, 0.0, nullptr, part.as<double>(), stream);
    HIPCHK_API(hipGetLastError());
    HIPCHK_API(hipStreamSynchronize(stream));
    return CCM_OK;
}

ccm_status ccm_op_hess_matvec(const double* X, const double* U, int64_t n, int64_t d,
                              const int32_t* src, const int32_t* dst, const double* w, int64_t m,
                              double gamma, double sigma, double q, const double* V, double* out,
                              int32_t repeats, double* ms_host, hipStream_t stream) {
    g_err.clear();
    ccm_status st = check_dims(n, d);
    if (st != CCM_OK) return st;
    int qk = 0;
    if (!q_kind(q, qk)) return fail(CCM_E_UNSUPPORTED, "q must be 1, 2 or inf");
    if (!(sigma > 0) || !(gamma >= 0)) return fail(CCM_E_INVALID, "sigma > 0, gamma >= 0");
    if (repeats < 1) return fail(CCM_E_INVALID, "repeats >= 1");
    std::string err;
    OwnedGraph og;
    st = graph_build(src, dst, w, m, n, int(d), true, stream, og, err);
    if (st != CCM_OK) return fail(st, err);
    const int64_t M = m * d;
    DevMem Pi, ip, lb, part;
    HIPCHK_API(Pi.alloc(size_t(std::max<int64_t>(M, 1)) * 8, stream));
    HIPCHK_API(ip.alloc(size_t(std::max<int64_t>(og.g.nent, 1)) * 16, stream));
    HIPCHK_API(lb.alloc(size_t(std::max<int64_t>(m, 1)) * lbits_per_edge(int(d)) * 4, stream));
    HIPCHK_API(part.alloc(partials_for(og.g) * 8, stream));
    Payload pl{ip.as<double2>(), lb.as<uint32_t>()};
    if (m > 0)
        launch_edge_ssnal(og.g, int(d), qk, gamma, sigma, X, U, Pi.as<double>(), pl,
                          part.as<double>(), stream);
    hipEvent_t e0, e1;
    HIPCHK_API(hipEventCreate(&e0));
    HIPCHK_API(hipEventCreate(&e1));
    HIPCHK_API(hipEventRecord(e0, stream));
    for (int r = 0; r < repeats; ++r)
        launch_matvec(og.g, int(d), qk, 0, V, Pi.as<double>(), pl, gamma, sigma, 1.0, nullptr, out,
                      part.as<double>(), CgSkip{}, stream);
    HIPCHK_API(hipEventRecord(e1, stream));
    HIPCHK_API(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK_API(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (ms_host) *ms_host = double(ms) / repeats;
    HIPCHK_API(hipGetLastError());
    HIPCHK_API(hipStreamSynchronize(stream));
    return CCM_OK;
}

ccm_status ccm_kkt(const double* A, const double* X, const double* U, int64_t n, int64_t d,
                   const int32_t* src, const int32_t* dst, const double* w, int64_t m,
                   double gamma, double q, double* out_host, hipStream_t stream) {
    g_err.clear();
    ccm_status st = check_dims(n, d);
    if (st != CCM_OK) return st;
    int qk = 0;
    if (!q_kind(q, qk)) return fail(CCM_E_UNSUPPORTED, "q must be 1, 2 or inf");
    if (!out_host) return fail(CCM_E_INVALID, "out_host is null");
    std::string err;
    OwnedGraph og;
    st = graph_build(src, dst, w, m, n, int(d), true, stream, og, err);
    if (st != CCM_OK) return fail(st, err);
    const int64_t N = n * d, M = m * d;
    DevMem Uf, G, p1, p2, p3, sc;
    HIPCHK_API(Uf.alloc(size_t(M) * 8, stream));
    HIPCHK_API(G.alloc(size_t(N) * 8, stream));
    HIPCHK_API(p1.alloc(partials_for(og.g) * 8, stream));
    HIPCHK_API(p2.alloc(partials_for(og.g) * 8, stream));
    HIPCHK_API(p3.alloc(partials_for(og.g) * 8, stream));
    HIPCHK_API(sc.alloc(32 * 8, stream));
    double* s = sc.as<double>();
    // KKT edge pass on (X, U), writing Pi_C(U) for the dual objective
    int gp = launch_edge_kkt(og.g, int(d), qk, gamma, X, U, Uf.as<double>(), p1.as<double>(),
                             stream);
    launch_finalize(p1.as<double>(), gp, kEdgeKktNV, s + 0, stream);
    // R_D with U as given
    gp = launch_scatter(og.g, int(d), qk, 1.0, X, -1.0, A, 1.0, U, G.as<double>(), false,
                        Payload{}, gamma, 0.0, nullptr, p2.as<double>(), stream);
    launch_finalize(p2.as<double>(), gp, kScatterNV, s + 8, stream);
    // f_d at Pi_C(U)
    gp = launch_scatter(og.g, int(d), qk, 0.0, nullptr, 1.0, A, 1.0, Uf.as<double>(),
                        G.as<double>(), false, Payload{}, gamma, 0.0, nullptr, p3.as<double>(),
                        stream);
    launch_finalize(p3.as<double>(), gp, kScatterNV, s + 16, stream);
    // ||A||^2 for the R_D denominator
    gp = launch_dot(A, A, N, p1.as<double>(), stream);
    launch_finalize(p1.as<double>(), gp, 1, s + 24, stream);
    double h[32];
    HIPCHK_API(hipMemcpyAsync(h, s, sizeof(h), hipMemcpyDeviceToHost, stream));
    HIPCHK_API(hipStreamSynchronize(stream));
    const double nA = std::sqrt(h[24]);
    const double nbx = std::sqrt(h[1]), nu = std::sqrt(h[2]);
    const double RD = std::sqrt(h[8]) / (1.0 + nA);
    const double RC = std::sqrt(h[0]) / (1.0 + nbx + nu);
    const double RU = std::sqrt(h[3]) / (1.0 + nu);
    const double fp = h[9] + h[4];
    const double fd = h[18] - 0.5 * h[19];
    out_host[0] = RD;
    out_host[1] = RC;
    out_host[2] = RU;
    out_host[3] = std::fabs(fp - fd) / (1.0 + std::fabs(fp) + std::fabs(fd));
    out_host[4] = fp;
    out_host[5] = fd;
    out_host[6] = std::max(RD, std::max(RC, RU));
    return CCM_OK;
}

ccm_status ccm_labels(const double* A, const double* X, int64_t n, int64_t d,
                      const int32_t* src, const int32_t* dst, int64_t m, int32_t* labels,
                      int32_t* n_clusters_host, hipStream_t stream) {
    g_err.clear();
    ccm_status st = check_dims(n, d);
    if (st != CCM_OK) return st;
    if (m < 0) return fail(CCM_E_INVALID, "m < 0");
    DevGraph g;
    g.n = n;
    g.m = m;
    g.src = src;
    g.dst = dst;
    DevMem work, sp, fused, parent, rank, temp, nc;
    HIPCHK_API(work.alloc(size_t(spread_work_size(n, int(d))) * 8, stream));
    HIPCHK_API(sp.alloc(8, stream));
    launch_spread(A, n, int(d), work.as<double>(), sp.as<double>(), stream);
    double S = 0;
    HIPCHK_API(hipMemcpyAsync(&S, sp.p, 8, hipMemcpyDeviceToHost, stream));
    HIPCHK_API(hipStreamSynchronize(stream));
    HIPCHK_API(fused.alloc(size_t(std::max<int64_t>(m, 1)) * 4, stream));
    HIPCHK_API(parent.alloc(size_t(n) * 4, stream));
    HIPCHK_API(rank.alloc(size_t(n + 1) * 4, stream));
    const size_t tb = labels_temp_bytes(n);
    HIPCHK_API(temp.alloc(tb, stream));
    HIPCHK_API(nc.alloc(4, stream));
    if (m > 0) launch_fused_flags(g, int(d), X, 1e-5 * (1.0 + S), fused.as<int>(), stream);
    launch_labels(n, m, src, dst, fused.as<int>(), parent.as<int>(), rank.as<int>(), temp.p, tb,
                  labels, nc.as<int>(), stream);
    int h = 0;
    HIPCHK_API(hipMemcpyAsync(&h, nc.p, 4, hipMemcpyDeviceToHost, stream));
    HIPCHK_API(hipStreamSynchronize(stream));
    if (n_clusters_host) *n_clusters_host = h;
    return CCM_OK;
}

ccm_status ccm_labels_noalloc(const double* A, const double* X, int64_t n, int64_t d,
                              const int32_t* src, const int32_t* dst, int64_t m, int32_t* labels,
                              int32_t* n_clusters_host, hipStream_t stream) {
    g_err.clear();
    ccm_status st = check_dims(n, d);
    if (st != CCM_OK) return st;
    if (m < 0) return fail(CCM_E_INVALID, "m < 0");
    if (n > kNoAllocMaxN || m > kNoAllocMaxM)
        return fail(CCM_E_CAPACITY, "ccm_labels_noalloc: n or m above its fixed work space (n <= " +
                                        std::to_string(kNoAllocMaxN) + ", m <= " +
                                        std::to_string(kNoAllocMaxM) + ")");
    const LabelsScratch L = labels_scratch(n, int(d), m);
    if (L.total > kNoAllocScratchBytes)
        return fail(CCM_E_CAPACITY, "ccm_labels_noalloc: problem needs " + std::to_string(L.total) +
                                        " bytes of work space, the fixed array holds " +
                                        std::to_string(kNoAllocScratchBytes));
    unsigned char* base = nullptr;
    st = noalloc_scratch(&base);
    if (st != CCM_OK) return st;
    double* work = reinterpret_cast<double*>(base + L.spread);
    double* S = reinterpret_cast<double*>(base + L.S);
    int* nc = reinterpret_cast<int*>(base + L.nc);
    int* fused = reinterpret_cast<int*>(base + L.fused);
    int* parent = reinterpret_cast<int*>(base + L.parent);
    int* rank = reinterpret_cast<int*>(base + L.rank);
    void* temp = base + L.temp;
    DevGraph g;
    g.n = n;
    g.m = m;
    g.src = src;
    g.dst = dst;
    // the same kernels as ccm_labels; the spread S stays on the device
    launch_spread(A, n, int(d), work, S, stream);
    if (m > 0) launch_fused_flags(g, int(d), X, 0.0, fused, stream, S);
    launch_labels(n, m, src, dst, fused, parent, rank, temp, L.temp_bytes, labels, nc, stream);
    HIPCHK_API(hipGetLastError());
    int h = 0;
    HIPCHK_API(hipMemcpyAsync(&h, nc, 4, hipMemcpyDeviceToHost, stream));
    HIPCHK_API(hipStreamSynchronize(stream));
    if (n_clusters_host) *n_clusters_host = h;
    return CCM_OK;
}

ccm_status ccm_weights_from_log(const double* log_w, int64_t m, double* w, hipStream_t stream) {
    g_err.clear();
    if (m < 0) return fail(CCM_E_INVALID, "m < 0");
    if (m > 0 && (!log_w || !w)) return fail(CCM_E_INVALID, "null argument");
    if (m > 0) launch_exp(log_w, m, w, stream);
    HIPCHK_API(hipGetLastError());
    return CCM_OK;
}

ccm_status ccm_stream_copy(const void* src, void* dst, int64_t bytes, int32_t repeats,
                           double* ms_host, hipStream_t stream) {
    g_err.clear();
    if (bytes < 0 || repeats < 1) return fail(CCM_E_INVALID, "bytes >= 0, repeats >= 1");
    hipEvent_t e0, e1;
    HIPCHK_API(hipEventCreate(&e0));
    HIPCHK_API(hipEventCreate(&e1));
    HIPCHK_API(hipEventRecord(e0, stream));
    for (int r = 0; r < repeats; ++r) launch_stream_copy(src, dst, bytes, stream);
    HIPCHK_API(hipEventRecord(e1, stream));
    HIPCHK_API(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK_API(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (ms_host) *ms_host = double(ms) / repeats;
    return CCM_OK;
}

}  // extern "C"
