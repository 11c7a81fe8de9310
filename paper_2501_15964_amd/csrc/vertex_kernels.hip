// Vertex-centric kernels: the transposed operator B^T (a signed sum of edge
// rows into vertex rows) and the SSNAL Newton matvec V + sigma B^T P B V.
//
// Both run over the vertex-major incidence lists (CSR by vertex, entries in
// ascending edge order).  Each vertex row is owned by one row group that
// accumulates its incident edge rows in registers and writes its output row
// once: no atomics, a fixed summation order, bit-reproducible results.  The
// cost is that an edge row is read by both of its endpoints.
#include "launch.hpp"

namespace ccm {
namespace {

template <int LPR>
__device__ __forceinline__ bool mask_bit(const uint64_t* bits, int64_t l, int W, int NB, int t,
                                         int b, int gl) {
    return (bits[(l * W + t) * NB + b] >> gl) & 1u;
}

template <int LPR, int NPER, int Q, bool DIAG>
__global__ __launch_bounds__(kBlock) void k_scatter(int64_t n, int d, const int* __restrict__ inc_ptr,
                                                    const Inc* __restrict__ inc, double cx,
                                                    const double* __restrict__ X, double ca,
                                                    const double* __restrict__ A, double cz,
                                                    const double* __restrict__ Z,
                                                    double* __restrict__ out, Payload pl,
                                                    const double* __restrict__ w, double gamma,
                                                    double sigma, double* __restrict__ Dinv,
                                                    double* __restrict__ partials) {
    const int gl = (threadIdx.x & 63) % LPR;
    constexpr int GPB = kBlock / LPR;
    const int W = (d + LPR - 1) / LPR;
    double acc4[kScatterNV] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = int64_t(blockIdx.x) * GPB + threadIdx.x / LPR; i < n;
         i += int64_t(gridDim.x) * GPB) {
        double acc[NPER], dg[NPER];
#pragma unroll
        for (int t = 0; t < NPER; ++t) acc[t] = dg[t] = 0.0;
        const int p0 = inc_ptr[i], p1 = inc_ptr[i + 1];
        for (int p = p0; p < p1; ++p) {
            const Inc e = inc[p];
            const bool pos = e.e >= 0;
            const int64_t l = pos ? e.e : ~e.e;
            double zr[NPER];
#pragma unroll
            for (int t = 0; t < NPER; ++t) {
                const int k = gl + LPR * t;
                zr[t] = (k < d) ? Z[l * d + k] : 0.0;
                acc[t] += pos ? zr[t] : -zr[t];
            }
            if constexpr (DIAG) {
                if constexpr (Q == kQ2) {
                    const double a = pl.alpha[l];
                    if (a >= 1.0) {
#pragma unroll
                        for (int t = 0; t < NPER; ++t) dg[t] += 1.0;
                    } else if (a > 0.0) {
                        const double r = gamma * w[l];
                        const double ir = 1.0 / r;
#pragma unroll
                        for (int t = 0; t < NPER; ++t) {
                            const double yh = zr[t] * ir;
                            dg[t] += a * (1.0 - yh * yh);
                        }
                    }
                } else if constexpr (Q == kQ1) {
#pragma unroll
                    for (int t = 0; t < NPER; ++t)
                        if (t < W && mask_bit<LPR>(pl.bits, l, W, 1, t, 0, gl)) dg[t] += 1.0;
                } else {
                    const int c = pl.cnt[l];
                    if (c < 0) {
#pragma unroll
                        for (int t = 0; t < NPER; ++t) dg[t] += 1.0;
                    } else if (c > 0) {
                        const double f = 1.0 - 1.0 / double(c);
#pragma unroll
                        for (int t = 0; t < NPER; ++t)
                            if (t < W && mask_bit<LPR>(pl.bits, l, W, 2, t, 0, gl)) dg[t] += f;
                    }
                }
            }
        }
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            if (k < d) {
                const double xv = X ? X[i * d + k] : 0.0;
                const double av = A ? A[i * d + k] : 0.0;
                const double o = cx * xv + ca * av + cz * acc[t];
                out[i * d + k] = o;
                const double dx = xv - av;
                acc4[0] += o * o;
                acc4[1] += 0.5 * dx * dx;
                acc4[2] += av * acc[t];
                acc4[3] += acc[t] * acc[t];
                if constexpr (DIAG) Dinv[i * d + k] = 1.0 / (1.0 + sigma * dg[t]);
            }
        }
    }
    block_reduce_store<kScatterNV>(acc4, partials + blockIdx.x * kScatterNV);
}

template <int LPR, int NPER, int Q, int MODE>
__global__ __launch_bounds__(kBlock) void k_matvec(int64_t n, int d, const int* __restrict__ inc_ptr,
                                                   const Inc* __restrict__ inc,
                                                   const double* __restrict__ V,
                                                   const double* __restrict__ Pi, Payload pl,
                                                   const double* __restrict__ w, double gamma,
                                                   double sigma, double c0,
                                                   const double* __restrict__ dscale,
                                                   double* __restrict__ out,
                                                   double* __restrict__ partials, CgSkip skip) {
    if (skip.done && *skip.done) return;
    if (skip.rr_partials) {
        const double rr = block_sum_partials(skip.rr_partials, skip.nparts, 2, 1);
        if (rr <= skip.thr) return;
    }
    const int gl = (threadIdx.x & 63) % LPR;
    constexpr int GPB = kBlock / LPR;
    const int W = (d + LPR - 1) / LPR;
    double dot[1] = {0.0};
    for (int64_t i = int64_t(blockIdx.x) * GPB + threadIdx.x / LPR; i < n;
         i += int64_t(gridDim.x) * GPB) {
        double vi[NPER], acc[NPER];
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            vi[t] = (k < d) ? V[i * d + k] : 0.0;
            acc[t] = 0.0;
        }
        const int p0 = inc_ptr[i], p1 = inc_ptr[i + 1];
        for (int p = p0; p < p1; ++p) {
            const Inc e = inc[p];
            const int64_t l = e.e >= 0 ? e.e : ~e.e;
            const int64_t o = e.o;
            double dl[NPER];
#pragma unroll
            for (int t = 0; t < NPER; ++t) {
                const int k = gl + LPR * t;
                dl[t] = (k < d) ? vi[t] - V[o * d + k] : 0.0;
            }
            if constexpr (MODE == 1) {
#pragma unroll
                for (int t = 0; t < NPER; ++t) acc[t] += dl[t];
            } else if constexpr (Q == kQ2) {
                // P = I inside the ball; a (I - yhat yhat^T) outside, with
                // yhat = Pi_l / r_l, applied as a dl - (a / r^2) <Pi_l, dl> Pi_l
                const double a = pl.alpha[l];
                if (a >= 1.0) {
#pragma unroll
                    for (int t = 0; t < NPER; ++t) acc[t] += dl[t];
                } else if (a > 0.0) {
                    const double r = gamma * w[l];
                    double pv[NPER];
                    double c = 0.0;
#pragma unroll
                    for (int t = 0; t < NPER; ++t) {
                        const int k = gl + LPR * t;
                        pv[t] = (k < d) ? Pi[l * d + k] : 0.0;
                        c += pv[t] * dl[t];
                    }
                    c = group_sum<LPR>(c);
                    const double f = a * c / (r * r);
#pragma unroll
                    for (int t = 0; t < NPER; ++t) acc[t] += a * dl[t] - f * pv[t];
                }
            } else if constexpr (Q == kQ1) {
                // P = diag(1[|y_k| <= r])
#pragma unroll
                for (int t = 0; t < NPER; ++t)
                    if (t < W && mask_bit<LPR>(pl.bits, l, W, 1, t, 0, gl)) acc[t] += dl[t];
            } else {
                // P = I inside; diag(1_S) - s_S s_S^T / |S| outside
                const int c = pl.cnt[l];
                if (c < 0) {
#pragma unroll
                    for (int t = 0; t < NPER; ++t) acc[t] += dl[t];
                } else if (c > 0) {
                    bool inS[NPER], neg[NPER];
                    double sd = 0.0;
#pragma unroll
                    for (int t = 0; t < NPER; ++t) {
                        inS[t] = (t < W) && mask_bit<LPR>(pl.bits, l, W, 2, t, 0, gl);
                        neg[t] = (t < W) && mask_bit<LPR>(pl.bits, l, W, 2, t, 1, gl);
                        if (inS[t]) sd += neg[t] ? -dl[t] : dl[t];
                    }
                    sd = group_sum<LPR>(sd) / double(c);
#pragma unroll
                    for (int t = 0; t < NPER; ++t)
                        if (inS[t]) acc[t] += dl[t] - (neg[t] ? -sd : sd);
                }
            }
        }
        const double sc = dscale ? dscale[i] : c0;
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            if (k < d) {
                const double o = sc * vi[t] + sigma * acc[t];
                out[i * d + k] = o;
                dot[0] += vi[t] * o;
            }
        }
    }
    block_reduce_store<kMatvecNV>(dot, partials + blockIdx.x * kMatvecNV);
}

}  // namespace

int launch_scatter(const DevGraph& g, int d, int qk, double cx, const double* X, double ca,
                   const double* A, double cz, const double* Z, double* out, bool diag, Payload pl,
                   double gamma, double sigma, double* Dinv, double* partials, hipStream_t s) {
    int grid = 1;
    dispatch_row(d, [&](auto L, auto N) {
        constexpr int lpr = decltype(L)::value, nper = decltype(N)::value;
        grid = row_grid(g.n, lpr);
        if (!diag) {
            hipLaunchKernelGGL((k_scatter<lpr, nper, kQ2, false>), dim3(grid), dim3(kBlock), 0, s,
                               g.n, d, g.inc_ptr, g.inc, cx, X, ca, A, cz, Z, out, pl, g.w, gamma,
                               sigma, Dinv, partials);
            return;
        }
        dispatch_q(qk, [&](auto Qc) {
            constexpr int q = decltype(Qc)::value;
            hipLaunchKernelGGL((k_scatter<lpr, nper, q, true>), dim3(grid), dim3(kBlock), 0, s,
                               g.n, d, g.inc_ptr, g.inc, cx, X, ca, A, cz, Z, out, pl, g.w, gamma,
                               sigma, Dinv, partials);
        });
    });
    return grid;
}

int launch_matvec(const DevGraph& g, int d, int qk, int mode, const double* V, const double* Pi,
                  Payload pl, double gamma, double sigma, double c0, const double* dscale,
                  double* out, double* partials, CgSkip skip, hipStream_t s) {
    int grid = 1;
    dispatch_row(d, [&](auto L, auto N) {
        constexpr int lpr = decltype(L)::value, nper = decltype(N)::value;
        grid = row_grid(g.n, lpr);
        if (mode == 1) {
            hipLaunchKernelGGL((k_matvec<lpr, nper, kQ2, 1>), dim3(grid), dim3(kBlock), 0, s, g.n,
                               d, g.inc_ptr, g.inc, V, Pi, pl, g.w, gamma, sigma, c0, dscale, out,
                               partials, skip);
            return;
        }
        dispatch_q(qk, [&](auto Qc) {
            constexpr int q = decltype(Qc)::value;
            hipLaunchKernelGGL((k_matvec<lpr, nper, q, 0>), dim3(grid), dim3(kBlock), 0, s, g.n, d,
                               g.inc_ptr, g.inc, V, Pi, pl, g.w, gamma, sigma, c0, dscale, out,
                               partials, skip);
        });
    });
    return grid;
}

}  // namespace ccm
