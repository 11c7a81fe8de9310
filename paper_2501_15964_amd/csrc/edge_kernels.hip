// Edge-parallel kernels: the gather B X, the per-edge projection onto the dual
// ball C_l = {||u||_{q*} <= r_l} (r_l = gamma w_l), the prox of
// r_l ||.||_q by the Moreau identity prox = id - Pi, and the generalized
// Jacobian payload of Pi_C used by the SSNAL Newton matvec.
//
// Layout: edges are rows of an m x d FP64 array in canonical order
// (src < dst, sorted), so edge l's row sits next to edge l+1's and a row
// group of LPR lanes streams it with unit-stride 8-byte loads; the endpoint
// rows x_src, x_dst are gathered from the n x d vertex array.
#include "launch.hpp"
#include "proj.hpp"

namespace ccm {
namespace {

template <int LPR, int NPER, int Q>
__device__ __forceinline__ void store_payload(const RowProj<LPR, NPER, Q>& o, int64_t l, int gl,
                                              const int* __restrict__ epos, Payload pl,
                                              double r) {
    if constexpr (Q == kQ1 || Q == kQInf) pl.lbits[l * LPR + gl] = o.lm;
    if (gl != 0) return;
    double2 v;
    if constexpr (Q == kQ2) v = double2{o.alpha, o.alpha > 0.0 ? 1.0 / r : 0.0};
    else v = double2{double(o.cnt), 0.0};
    if constexpr (Q == kQ2 || Q == kQInf) {
        pl.ipay[epos[2 * l]] = v;
        pl.ipay[epos[2 * l + 1]] = v;
    }
}

template <int LPR, int NPER, int Q>
__global__ __launch_bounds__(kBlock) void k_edge_ssnal(int64_t m, int d, const int* __restrict__ src,
                                                       const int* __restrict__ dst,
                                                       const double* __restrict__ w, double gamma,
                                                       double sigma, const double* __restrict__ X,
                                                       const double* __restrict__ U,
                                                       double* __restrict__ Pi, Payload pl,
                                                       const int* __restrict__ epos,
                                                       double* __restrict__ partials) {
    const int lane = threadIdx.x & 63;
    const int gl = lane % LPR;
    constexpr int GPB = kBlock / LPR;
    double acc[kEdgeSsnalNV] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t l = int64_t(blockIdx.x) * GPB + threadIdx.x / LPR; l < m;
         l += int64_t(gridDim.x) * GPB) {
        const int64_t i = src[l], j = dst[l];
        const double r = gamma * w[l];
        double y[NPER], bx[NPER], u[NPER];
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            if (k < d) {
                bx[t] = X[i * d + k] - X[j * d + k];
                u[t] = U[l * d + k];
            } else {
                bx[t] = 0.0;
                u[t] = 0.0;
            }
            y[t] = u[t] + sigma * bx[t];
        }
        RowProj<LPR, NPER, Q> o;
        project_row<LPR, NPER, Q, true>(y, gl, lane, d, r, o);
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            if (k < d) {
                Pi[l * d + k] = o.pi[t];
                const double e = o.pi[t] - u[t];
                acc[0] += bx[t] * o.pi[t];
                acc[1] += e * e;
                acc[2] += bx[t] * bx[t];
                acc[3] += o.pi[t] * o.pi[t];
            }
        }
        store_payload<LPR, NPER, Q>(o, l, gl, epos, pl, r);
        if (gl == 0) {
            if constexpr (Q == kQ2) acc[4] += (o.alpha < 1.0) ? 1.0 : 0.0;
            else if constexpr (Q == kQInf) acc[4] += (o.cnt >= 0) ? 1.0 : 0.0;
            else acc[4] += 1.0;
        }
    }
    block_reduce_store<kEdgeSsnalNV>(acc, partials + blockIdx.x * kEdgeSsnalNV);
}

template <int LPR, int NPER, int Q>
__global__ __launch_bounds__(kBlock) void k_edge_kkt(int64_t m, int d, const int* __restrict__ src,
                                                     const int* __restrict__ dst,
                                                     const double* __restrict__ w, double gamma,
                                                     const double* __restrict__ X,
                                                     const double* __restrict__ U,
                                                     double* __restrict__ Ufeas,
                                                     double* __restrict__ partials,
                                                     double* __restrict__ rowstats) {
    const int lane = threadIdx.x & 63;
    const int gl = lane % LPR;
    constexpr int GPB = kBlock / LPR;
    double acc[kEdgeKktNV] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t l = int64_t(blockIdx.x) * GPB + threadIdx.x / LPR; l < m;
         l += int64_t(gridDim.x) * GPB) {
        const int64_t i = src[l], j = dst[l];
        const double r = gamma * w[l];
        double bx[NPER], u[NPER], v[NPER];
        double nq = 0.0;
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            if (k < d) {
                bx[t] = X[i * d + k] - X[j * d + k];
                u[t] = U[l * d + k];
            } else {
                bx[t] = 0.0;
                u[t] = 0.0;
            }
            v[t] = bx[t] + u[t];
            if constexpr (Q == kQ1) nq += fabs(bx[t]);
            else if constexpr (Q == kQ2) nq += bx[t] * bx[t];
            else nq = fmax(nq, fabs(bx[t]));
        }
        double pen = 0.0;  // r ||(BX)_l||_q, counted once per edge
        if constexpr (Q == kQ2) {
            nq = group_sum<LPR>(nq);
            pen = r * sqrt(nq);
        } else if constexpr (Q == kQInf) {
            nq = group_max<LPR>(nq);
            pen = r * nq;
        } else {
            pen = group_sum<LPR>(r * nq);
        }
        if (gl == 0) acc[4] += pen;
        RowProj<LPR, NPER, Q> pv, pu;
        project_row<LPR, NPER, Q, false>(v, gl, lane, d, r, pv);
        project_row<LPR, NPER, Q, false>(u, gl, lane, d, r, pu);
        double r4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            if (k < d) {
                const double e = pv.pi[t] - u[t];
                const double f = u[t] - pu.pi[t];
                r4[0] += e * e;
                r4[1] += bx[t] * bx[t];
                r4[2] += u[t] * u[t];
                r4[3] += f * f;
                if (Ufeas) Ufeas[l * d + k] = pu.pi[t];
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] += r4[c];
        if (rowstats) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double tot = group_sum<LPR>(r4[c]);
                if (gl == 0) rowstats[l * 5 + c] = tot;
            }
            if (gl == 0) rowstats[l * 5 + 4] = pen;
        }
    }
    block_reduce_store<kEdgeKktNV>(acc, partials + blockIdx.x * kEdgeKktNV);
}

template <int LPR, int NPER, int Q>
__global__ __launch_bounds__(kBlock) void k_edge_admm(int64_t m, int d, const int* __restrict__ src,
                                                      const int* __restrict__ dst,
                                                      const double* __restrict__ w, double gamma,
                                                      double sigma, double tau,
                                                      const double* __restrict__ X,
                                                      double* __restrict__ Z,
                                                      double* __restrict__ L,
                                                      double* __restrict__ Qo,
                                                      double* __restrict__ Uf,
                                                      double* __restrict__ partials) {
    const int lane = threadIdx.x & 63;
    const int gl = lane % LPR;
    constexpr int GPB = kBlock / LPR;
    double acc[kEdgeAdmmNV] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t l = int64_t(blockIdx.x) * GPB + threadIdx.x / LPR; l < m;
         l += int64_t(gridDim.x) * GPB) {
        const int64_t i = src[l], j = dst[l];
        const double r = gamma * w[l];
        double bx[NPER], lam[NPER], zo[NPER], y[NPER];
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            if (k < d) {
                bx[t] = X[i * d + k] - X[j * d + k];
                lam[t] = L[l * d + k];
                zo[t] = Z[l * d + k];
            } else {
                bx[t] = lam[t] = zo[t] = 0.0;
            }
            y[t] = sigma * bx[t] + lam[t];
        }
        RowProj<LPR, NPER, Q> o;
        project_row<LPR, NPER, Q, false>(y, gl, lane, d, r, o);
        double ln[NPER];
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            const double zn = bx[t] + (lam[t] - o.pi[t]) / sigma;
            ln[t] = lam[t] + tau * sigma * (bx[t] - zn);
            if (k < d) {
                Z[l * d + k] = zn;
                L[l * d + k] = ln[t];
                Qo[l * d + k] = sigma * zn - ln[t];
                const double rp = bx[t] - zn, dz = zn - zo[t];
                acc[0] += rp * rp;
                acc[1] += dz * dz;
                acc[2] += bx[t] * bx[t];
                acc[3] += zn * zn;
            }
        }
        if (Uf) {
            RowProj<LPR, NPER, Q> pu;
            project_row<LPR, NPER, Q, false>(ln, gl, lane, d, r, pu);
#pragma unroll
            for (int t = 0; t < NPER; ++t) {
                const int k = gl + LPR * t;
                if (k < d) Uf[l * d + k] = pu.pi[t];
            }
        }
    }
    block_reduce_store<kEdgeAdmmNV>(acc, partials + blockIdx.x * kEdgeAdmmNV);
}

// One Halpern-Peaceman-Rachford edge step (see launch_edge_hpr).
template <int LPR, int NPER, int Q>
__global__ __launch_bounds__(kBlock) void k_edge_hpr(int64_t m, int d, const int* __restrict__ src,
                                                     const int* __restrict__ dst,
                                                     const double* __restrict__ w, double gamma,
                                                     double sigma, double a,
                                                     const double* __restrict__ X,
                                                     double* __restrict__ Z,
                                                     double* __restrict__ L,
                                                     const double* __restrict__ Za,
                                                     const double* __restrict__ La,
                                                     double* __restrict__ Qo,
                                                     double* __restrict__ Uh,
                                                     double* __restrict__ partials) {
    const int lane = threadIdx.x & 63;
    const int gl = lane % LPR;
    constexpr int GPB = kBlock / LPR;
    double acc[kEdgeHprNV] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t l = int64_t(blockIdx.x) * GPB + threadIdx.x / LPR; l < m;
         l += int64_t(gridDim.x) * GPB) {
        const int64_t i = src[l], j = dst[l];
        const double r = gamma * w[l];
        double bx[NPER], lam[NPER], zo[NPER], y[NPER];
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            if (k < d) {
                bx[t] = X[i * d + k] - X[j * d + k];
                lam[t] = L[l * d + k];
                zo[t] = Z[l * d + k];
            } else {
                bx[t] = lam[t] = zo[t] = 0.0;
            }
            // reflection H = 2 BX - Z, then the point sigma H + L to project
            y[t] = sigma * (2.0 * bx[t] - zo[t]) + lam[t];
        }
        RowProj<LPR, NPER, Q> o;
        project_row<LPR, NPER, Q, false>(y, gl, lane, d, r, o);
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            if (k < d) {
                const double h = 2.0 * bx[t] - zo[t];
                const double lh = o.pi[t];
                const double zh = h + (lam[t] - lh) / sigma;
                const double zn = a * Za[l * d + k] + (1.0 - a) * zh;
                const double ln = a * La[l * d + k] + (1.0 - a) * lh;
                Z[l * d + k] = zn;
                L[l * d + k] = ln;
                Qo[l * d + k] = sigma * zn - ln;
                if (Uh) Uh[l * d + k] = lh;
                const double dz = zo[t] - zh, dl = lam[t] - lh;
                const double mz = zn - Za[l * d + k], ml = ln - La[l * d + k];
                acc[0] += dz * dz;
                acc[1] += dl * dl;
                acc[2] += mz * mz;
                acc[3] += ml * ml;
            }
        }
    }
    block_reduce_store<kEdgeHprNV>(acc, partials + blockIdx.x * kEdgeHprNV);
}

template <int LPR, int NPER, int Q>
__global__ __launch_bounds__(kBlock) void k_edge_ama(int64_t m, int d, const int* __restrict__ src,
                                                     const int* __restrict__ dst,
                                                     const double* __restrict__ w, double gamma,
                                                     double nu, double beta,
                                                     const double* __restrict__ X,
                                                     double* __restrict__ U,
                                                     double* __restrict__ V,
                                                     double* __restrict__ partials) {
    const int lane = threadIdx.x & 63;
    const int gl = lane % LPR;
    constexpr int GPB = kBlock / LPR;
    double acc[kEdgeAmaNV] = {0.0, 0.0};
    for (int64_t l = int64_t(blockIdx.x) * GPB + threadIdx.x / LPR; l < m;
         l += int64_t(gridDim.x) * GPB) {
        const int64_t i = src[l], j = dst[l];
        const double r = gamma * w[l];
        double y[NPER], vo[NPER], uo[NPER];
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            if (k < d) {
                vo[t] = V[l * d + k];
                uo[t] = U[l * d + k];
                y[t] = vo[t] + nu * (X[i * d + k] - X[j * d + k]);
            } else {
                vo[t] = uo[t] = y[t] = 0.0;
            }
        }
        RowProj<LPR, NPER, Q> o;
        project_row<LPR, NPER, Q, false>(y, gl, lane, d, r, o);
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            if (k < d) {
                const double un = o.pi[t];
                const double du = un - uo[t];
                acc[0] += (vo[t] - un) * du;
                acc[1] += du * du;
                U[l * d + k] = un;
                V[l * d + k] = un + beta * du;
            }
        }
    }
    block_reduce_store<kEdgeAmaNV>(acc, partials + blockIdx.x * kEdgeAmaNV);
}

template <int LPR, int NPER>
__global__ __launch_bounds__(kBlock) void k_gather(int64_t m, int d, const int* __restrict__ src,
                                                   const int* __restrict__ dst,
                                                   const double* __restrict__ X,
                                                   double* __restrict__ Y) {
    const int gl = (threadIdx.x & 63) % LPR;
    constexpr int GPB = kBlock / LPR;
    for (int64_t l = int64_t(blockIdx.x) * GPB + threadIdx.x / LPR; l < m;
         l += int64_t(gridDim.x) * GPB) {
        const int64_t i = src[l], j = dst[l];
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            if (k < d) Y[l * d + k] = X[i * d + k] - X[j * d + k];
        }
    }
}

template <int LPR, int NPER, int Q>
__global__ __launch_bounds__(kBlock) void k_project(int64_t m, int d, const double* __restrict__ Y,
                                                    const double* __restrict__ w, double gamma,
                                                    int prox, double* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int gl = lane % LPR;
    constexpr int GPB = kBlock / LPR;
    for (int64_t l = int64_t(blockIdx.x) * GPB + threadIdx.x / LPR; l < m;
         l += int64_t(gridDim.x) * GPB) {
        const double r = gamma * w[l];
        double y[NPER];
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            y[t] = (k < d) ? Y[l * d + k] : 0.0;
        }
        RowProj<LPR, NPER, Q> o;
        project_row<LPR, NPER, Q, false>(y, gl, lane, d, r, o);
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            if (k < d) out[l * d + k] = prox ? (y[t] - o.pi[t]) : o.pi[t];
        }
    }
}

// Path continuation of the dual: the rows of U that lie on the boundary of
// their ball of radius g0 w_l are scaled by rho (q = 1: the coordinates at
// +-g0 w_l, the box being a product of intervals).  A row on the boundary
// belongs to an edge whose endpoints are apart, and there u_l is g0 w_l times
// a unit direction that moves slowly with gamma.
template <int LPR, int NPER, int Q>
__global__ __launch_bounds__(kBlock) void k_scale_boundary(int64_t m, int d,
                                                           const double* __restrict__ w,
                                                           double g0, double rho,
                                                           double* __restrict__ U) {
    constexpr int GPB = kBlock / LPR;
    const int gl = (threadIdx.x & 63) % LPR;
    for (int64_t l = int64_t(blockIdx.x) * GPB + threadIdx.x / LPR; l < m;
         l += int64_t(gridDim.x) * GPB) {
        const double edge = (1.0 - 1e-9) * g0 * w[l];
        double u[NPER];
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            u[t] = (k < d) ? U[l * d + k] : 0.0;
            if constexpr (Q == kQ2) s += u[t] * u[t];
            else if constexpr (Q == kQInf) s += fabs(u[t]);
        }
        bool row = false;
        if constexpr (Q == kQ2) row = sqrt(group_sum<LPR>(s)) >= edge;
        else if constexpr (Q == kQInf) row = group_sum<LPR>(s) >= edge;
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            const bool on = Q == kQ1 ? fabs(u[t]) >= edge : row;
            if (k < d && on) U[l * d + k] = u[t] * rho;
        }
    }
}

template <int LPR, int NPER>
__global__ __launch_bounds__(kBlock) void k_fused_flags(int64_t m, int d,
                                                        const int* __restrict__ src,
                                                        const int* __restrict__ dst,
                                                        const double* __restrict__ X, double thr,
                                                        const double* __restrict__ spread,
                                                        const double* __restrict__ vthr,
                                                        int* __restrict__ fused) {
    if (spread) thr = 1e-5 * (1.0 + spread[0]);
    const int gl = (threadIdx.x & 63) % LPR;
    constexpr int GPB = kBlock / LPR;
    for (int64_t l = int64_t(blockIdx.x) * GPB + threadIdx.x / LPR; l < m;
         l += int64_t(gridDim.x) * GPB) {
        const int64_t i = src[l], j = dst[l];
        const double th = vthr ? vthr[i] : thr;
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            const int k = gl + LPR * t;
            if (k < d) {
                const double e = X[i * d + k] - X[j * d + k];
                s += e * e;
            }
        }
        s = group_sum<LPR>(s);
        if (gl == 0) fused[l] = sqrt(s) <= th ? 1 : 0;
    }
}

}  // namespace

int launch_edge_ssnal(const DevGraph& g, int d, int qk, double gamma, double sigma,
                      const double* X, const double* U, double* Pi, Payload pl,
                      double* partials, hipStream_t s) {
    int grid = 1;
    dispatch_row(d, [&](auto L, auto N) {
        constexpr int lpr = decltype(L)::value, nper = decltype(N)::value;
        grid = row_grid(g.m, lpr);
        dispatch_q(qk, [&](auto Qc) {
            constexpr int q = decltype(Qc)::value;
            hipLaunchKernelGGL((k_edge_ssnal<lpr, nper, q>), dim3(grid), dim3(kBlock), 0, s, g.m,
                               d, g.src, g.dst, g.w, gamma, sigma, X, U, Pi, pl, g.epos,
                               partials);
        });
    });
    return grid;
}

int launch_edge_kkt(const DevGraph& g, int d, int qk, double gamma, const double* X,
                    const double* U, double* Ufeas, double* partials, hipStream_t s,
                    double* rowstats) {
    int grid = 1;
    dispatch_row(d, [&](auto L, auto N) {
        constexpr int lpr = decltype(L)::value, nper = decltype(N)::value;
        grid = row_grid(g.m, lpr);
        dispatch_q(qk, [&](auto Qc) {
            constexpr int q = decltype(Qc)::value;
            hipLaunchKernelGGL((k_edge_kkt<lpr, nper, q>), dim3(grid), dim3(kBlock), 0, s, g.m, d,
                               g.src, g.dst, g.w, gamma, X, U, Ufeas, partials, rowstats);
        });
    });
    return grid;
}

int launch_edge_admm(const DevGraph& g, int d, int qk, double gamma, double sigma, double tau,
                     const double* X, double* Z, double* L_, double* Q, double* Uf,
                     double* partials, hipStream_t s) {
    int grid = 1;
    dispatch_row(d, [&](auto L, auto N) {
        constexpr int lpr = decltype(L)::value, nper = decltype(N)::value;
        grid = row_grid(g.m, lpr);
        dispatch_q(qk, [&](auto Qc) {
            constexpr int q = decltype(Qc)::value;
            hipLaunchKernelGGL((k_edge_admm<lpr, nper, q>), dim3(grid), dim3(kBlock), 0, s, g.m,
                               d, g.src, g.dst, g.w, gamma, sigma, tau, X, Z, L_, Q, Uf, partials);
        });
    });
    return grid;
}

int launch_edge_hpr(const DevGraph& g, int d, int qk, double gamma, double sigma, double a,
                    const double* X, double* Z, double* L_, const double* Za, const double* La,
                    double* Q, double* Uh, double* partials, hipStream_t s) {
    int grid = 1;
    dispatch_row(d, [&](auto L, auto N) {
        constexpr int lpr = decltype(L)::value, nper = decltype(N)::value;
        grid = row_grid(g.m, lpr);
        dispatch_q(qk, [&](auto Qc) {
            constexpr int q = decltype(Qc)::value;
            hipLaunchKernelGGL((k_edge_hpr<lpr, nper, q>), dim3(grid), dim3(kBlock), 0, s, g.m,
                               d, g.src, g.dst, g.w, gamma, sigma, a, X, Z, L_, Za, La, Q, Uh,
                               partials);
        });
    });
    return grid;
}

int launch_edge_ama(const DevGraph& g, int d, int qk, double gamma, double nu, double beta,
                    const double* X, double* U, double* V, double* partials, hipStream_t s) {
    int grid = 1;
    dispatch_row(d, [&](auto L, auto N) {
        constexpr int lpr = decltype(L)::value, nper = decltype(N)::value;
        grid = row_grid(g.m, lpr);
        dispatch_q(qk, [&](auto Qc) {
            constexpr int q = decltype(Qc)::value;
            hipLaunchKernelGGL((k_edge_ama<lpr, nper, q>), dim3(grid), dim3(kBlock), 0, s, g.m, d,
                               g.src, g.dst, g.w, gamma, nu, beta, X, U, V, partials);
        });
    });
    return grid;
}

void launch_gather(const DevGraph& g, int d, const double* X, double* Y, hipStream_t s) {
    dispatch_row(d, [&](auto L, auto N) {
        constexpr int lpr = decltype(L)::value, nper = decltype(N)::value;
        hipLaunchKernelGGL((k_gather<lpr, nper>), dim3(row_grid(g.m, lpr)), dim3(kBlock), 0, s,
                           g.m, d, g.src, g.dst, X, Y);
    });
}

void launch_project(int64_t m, int d, int qk, const double* Y, const double* w, double gamma,
                    bool prox, double* out, hipStream_t s) {
    dispatch_row(d, [&](auto L, auto N) {
        constexpr int lpr = decltype(L)::value, nper = decltype(N)::value;
        dispatch_q(qk, [&](auto Qc) {
            constexpr int q = decltype(Qc)::value;
            hipLaunchKernelGGL((k_project<lpr, nper, q>), dim3(row_grid(m, lpr)), dim3(kBlock), 0,
                               s, m, d, Y, w, gamma, prox ? 1 : 0, out);
        });
    });
}

void launch_scale_boundary(int64_t m, int d, int qk, const double* w, double g0, double rho,
                           double* U, hipStream_t s) {
    if (m <= 0) return;
    dispatch_row(d, [&](auto L, auto N) {
        constexpr int lpr = decltype(L)::value, nper = decltype(N)::value;
        dispatch_q(qk, [&](auto Qc) {
            constexpr int q = decltype(Qc)::value;
            hipLaunchKernelGGL((k_scale_boundary<lpr, nper, q>), dim3(row_grid(m, lpr)),
                               dim3(kBlock), 0, s, m, d, w, g0, rho, U);
        });
    });
}

void launch_fused_flags(const DevGraph& g, int d, const double* X, double thr, int* fused,
                        hipStream_t s, const double* spread, const double* vthr) {
    dispatch_row(d, [&](auto L, auto N) {
        constexpr int lpr = decltype(L)::value, nper = decltype(N)::value;
        hipLaunchKernelGGL((k_fused_flags<lpr, nper>), dim3(row_grid(g.m, lpr)), dim3(kBlock), 0,
                           s, g.m, d, g.src, g.dst, X, thr, spread, vthr, fused);
    });
}

}  // namespace ccm
