// Kernels of the solution-map adjoint (q = 2).
//
// At a solution whose clusters are locally constant, the model reduces to a
// smooth problem in the cluster values v_c with curvature
//   diag(|c|) (x) I + B_c^T H B_c,  H_l = gamma w_l (I - ghat ghat^T) / ||delta_l||
// on the edges joining two clusters (delta_l = x_i - x_j, ghat = delta/||delta||).
// The curvature of edge l is stored in the q = 2 payload layout of the
// Newton matvec: per incidence {alpha_l, 1 / r_l} with
// alpha_l = gamma w_l / ||delta_l|| and r_l = gamma w_l, and the row
// gamma w_l ghat_l, so that the matvec's a (dl - <Pi, dl> Pi / r^2) is H_l dl.
#include "launch.hpp"

namespace ccm {
namespace {

template <int LPR, int NPER>
__global__ __launch_bounds__(kBlock) void k_adj_payload(int64_t m, int d, const int* __restrict__ src,
                                                        const int* __restrict__ dst,
                                                        const double* __restrict__ w,
                                                        const double* __restrict__ X,
                                                        const int* __restrict__ labels,
                                                        double gamma,
                                                        const int* __restrict__ epos,
                                                        double2* __restrict__ ipay,
                                                        double* __restrict__ Pi) {
    const int gl = (threadIdx.x & 63) % LPR;
    constexpr int GPB = kBlock / LPR;
    for (int64_t l = int64_t(blockIdx.x) * GPB + threadIdx.x / LPR; l < m;
         l += int64_t(gridDim.x) * GPB) {
        const int64_t i = src[l], j = dst[l];
        double dl[NPER];
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            dl[t] = (k < d) ? X[i * d + k] - X[j * d + k] : 0.0;
            s += dl[t] * dl[t];
        }
        s = group_sum<LPR>(s);
        const double nd = sqrt(s);
        const double r = gamma * w[l];
        const bool inter = labels[i] != labels[j] && nd > 0.0 && r >= kTinyRadius;
        if (gl == 0) {
            const double2 v{inter ? r / nd : 0.0, inter ? 1.0 / r : 0.0};
            ipay[epos[2 * l]] = v;
            ipay[epos[2 * l + 1]] = v;
        }
        const double sc = inter ? r / nd : 0.0;
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            if (k < d) Pi[l * d + k] = dl[t] * sc;
        }
    }
}

template <int LPR, int NPER>
__global__ __launch_bounds__(kBlock) void k_expand(int64_t n, int d, const int* __restrict__ labels,
                                                   const double* __restrict__ lam,
                                                   double* __restrict__ v) {
    const int gl = (threadIdx.x & 63) % LPR;
    constexpr int GPB = kBlock / LPR;
    for (int64_t i = int64_t(blockIdx.x) * GPB + threadIdx.x / LPR; i < n;
         i += int64_t(gridDim.x) * GPB) {
        const int64_t c = labels[i];
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            if (k < d) v[i * d + k] = lam[c * d + k];
        }
    }
}

template <int LPR, int NPER>
__global__ __launch_bounds__(kBlock) void k_adj_edge(int64_t m, int d, const int* __restrict__ src,
                                                     const int* __restrict__ dst,
                                                     const double* __restrict__ w,
                                                     const double* __restrict__ X,
                                                     const int* __restrict__ labels,
                                                     const double* __restrict__ lam, double gamma,
                                                     double* __restrict__ dlogw,
                                                     double* __restrict__ partials) {
    const int gl = (threadIdx.x & 63) % LPR;
    constexpr int GPB = kBlock / LPR;
    double acc[1] = {0.0};
    for (int64_t l = int64_t(blockIdx.x) * GPB + threadIdx.x / LPR; l < m;
         l += int64_t(gridDim.x) * GPB) {
        const int64_t i = src[l], j = dst[l];
        const int64_t ci = labels[i], cj = labels[j];
        double s = 0.0, pr = 0.0;
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            if (k < d) {
                const double dl = X[i * d + k] - X[j * d + k];
                const double bl = lam[ci * d + k] - lam[cj * d + k];
                s += dl * dl;
                pr += bl * dl;
            }
        }
        s = group_sum<LPR>(s);
        pr = group_sum<LPR>(pr);
        const double nd = sqrt(s);
        const bool inter = ci != cj && nd > 0.0;
        const double tl = inter ? pr / nd : 0.0;  // <(B_c lam)_l, ghat_l>
        if (gl == 0) {
            dlogw[l] = -gamma * w[l] * tl;
            acc[0] += w[l] * tl;
        }
    }
    block_reduce_store<1>(acc, partials + blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_rowscale(const double* __restrict__ x,
                                                     const double* __restrict__ rs,
                                                     double* __restrict__ o, int64_t rows, int d) {
    const int64_t N = rows * d;
    for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < N;
         k += int64_t(gridDim.x) * kBlock)
        o[k] = x[k] * rs[k / d];
}

__global__ __launch_bounds__(kBlock) void k_inv_sizes(int64_t K, const int* __restrict__ ptr,
                                                      double* __restrict__ out) {
    for (int64_t c = int64_t(blockIdx.x) * kBlock + threadIdx.x; c < K;
         c += int64_t(gridDim.x) * kBlock) {
        const int sz = ptr[c + 1] - ptr[c];
        out[c] = sz > 0 ? 1.0 / double(sz) : 0.0;
    }
}

__global__ __launch_bounds__(kBlock) void k_label_range(int64_t n, const int* __restrict__ labels,
                                                        int* range) {
    int lo = 0x7fffffff, hi = -1;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * kBlock) {
        const int v = labels[i];
        lo = v < lo ? v : lo;
        hi = v > hi ? v : hi;
    }
    atomicMin(range + 0, lo);
    atomicMax(range + 1, hi);
}

}  // namespace

void launch_inv_sizes(int64_t K, const int* ptr, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_inv_sizes, dim3(flat_grid(K)), dim3(kBlock), 0, s, K, ptr, out);
}

void launch_label_range(int64_t n, const int* labels, int* range, hipStream_t s) {
    hipLaunchKernelGGL(k_label_range, dim3(flat_grid(n)), dim3(kBlock), 0, s, n, labels, range);
}

void launch_adj_payload(const DevGraph& g, int d, const double* X, const int* labels,
                        double gamma, double2* ipay, double* Pi, hipStream_t s) {
    if (g.m == 0) return;
    dispatch_row(d, [&](auto L, auto N) {
        constexpr int lpr = decltype(L)::value, nper = decltype(N)::value;
        hipLaunchKernelGGL((k_adj_payload<lpr, nper>), dim3(row_grid(g.m, lpr)), dim3(kBlock), 0, s,
                           g.m, d, g.src, g.dst, g.w, X, labels, gamma, g.epos, ipay, Pi);
    });
}

void launch_expand(int64_t n, int d, const int* labels, const double* lam, double* v,
                   hipStream_t s) {
    dispatch_row(d, [&](auto L, auto N) {
        constexpr int lpr = decltype(L)::value, nper = decltype(N)::value;
        hipLaunchKernelGGL((k_expand<lpr, nper>), dim3(row_grid(n, lpr)), dim3(kBlock), 0, s, n, d,
                           labels, lam, v);
    });
}

int launch_adj_edge(const DevGraph& g, int d, const double* X, const int* labels,
                    const double* lam, double gamma, double* dlogw, double* partials,
                    hipStream_t s) {
    int grid = 1;
    dispatch_row(d, [&](auto L, auto N) {
        constexpr int lpr = decltype(L)::value, nper = decltype(N)::value;
        grid = row_grid(g.m, lpr);
        hipLaunchKernelGGL((k_adj_edge<lpr, nper>), dim3(grid), dim3(kBlock), 0, s, g.m, d, g.src,
                           g.dst, g.w, X, labels, lam, gamma, dlogw, partials);
    });
    return grid;
}

void launch_rowscale(const double* x, const double* rs, double* out, int64_t rows, int d,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_rowscale, dim3(flat_grid(rows * d)), dim3(kBlock), 0, s, x, rs, out, rows,
                       d);
}

}  // namespace ccm
