// Vertex-centric kernels: the transposed operator B^T (a signed sum of edge
// rows into vertex rows) and the SSNAL Newton matvec V + sigma B^T P B V.
//
// Both read the vertex-major incidence lists (CSR by vertex, entries in
// ascending edge order).  k-NN graphs are skewed (a few hub vertices have
// tens of times the mean degree), so work is not split by vertex but by
// equal chunks of C incidences: a row group takes one chunk, finishes every
// vertex whose incidences all lie inside it, and leaves a partial row for a
// vertex cut by a chunk boundary.  A fix-up pass sums those partials in
// chunk order and finishes isolated vertices.  There are no atomics and the
// summation order is fixed, so results are bit-reproducible.  An edge row is
// read by both of its endpoints.
#include "launch.hpp"

namespace ccm {
namespace {

template <int LPR>
__device__ __forceinline__ bool mask_bit(const uint64_t* bits, int64_t l, int W, int NB, int t,
                                         int b, int gl) {
    return (bits[(l * W + t) * NB + b] >> gl) & 1u;
}

// Incidences are processed U at a time: the U incidence entries are loaded
// together, then every row they point at.
template <int NPER>
struct Unroll {
    static constexpr int U = NPER <= 2 ? 8 : NPER == 4 ? 4 : 2;
};

// Per-incidence data of the generalized Jacobian (q = 2: a = r/||y|| outside
// the ball or 1 inside; outside, f = a / r^2 and ir = 1 / r; q = inf: support
// size, -1 inside).
struct Meta {
    int64_t l;
    int64_t o;
    bool pos;
    double a, f, ir;
    int cnt;
};

template <int Q, bool PAY, bool ADJ = false>
__device__ __forceinline__ Meta load_meta(const Inc* __restrict__ inc, int64_t p,
                                          const Payload& pl, const double* __restrict__ w,
                                          double gamma) {
    const Inc e = inc[p];
    Meta m;
    m.pos = e.e >= 0;
    m.l = m.pos ? e.e : ~e.e;
    m.o = e.o;
    m.a = 1.0;
    m.f = 0.0;
    m.ir = 0.0;
    m.cnt = -1;
    if constexpr (PAY && Q == kQ2) {
        m.a = pl.alpha[m.l];
        if ((ADJ || m.a < 1.0) && m.a > 0.0) {
            const double r = gamma * w[m.l];
            m.ir = 1.0 / r;
            m.f = m.a * m.ir * m.ir;
        }
    } else if constexpr (PAY && Q == kQInf) {
        m.cnt = pl.cnt[m.l];
    }
    return m;
}

// ---- B^T Z (and the Jacobi diagonal of I + sigma B^T P B) -------------------

template <int LPR, int NPER, int Q, bool DIAG>
__device__ __forceinline__ void scatter_range(int64_t pa, int64_t pb, int d, int gl, int W,
                                              const Inc* __restrict__ inc,
                                              const double* __restrict__ Z, const Payload& pl,
                                              const double* __restrict__ w, double gamma,
                                              double (&acc)[NPER], double (&dg)[NPER]) {
    constexpr int U = Unroll<NPER>::U;
    for (int64_t p0 = pa; p0 < pb; p0 += U) {
        Meta mt[U];
        double zr[U][NPER];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (p0 + u < pb) mt[u] = load_meta<Q, DIAG>(inc, p0 + u, pl, w, gamma);
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int t = 0; t < NPER; ++t) {
                const int k = gl + LPR * t;
                zr[u][t] = (p0 + u < pb && k < d) ? Z[mt[u].l * d + k] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (p0 + u >= pb) break;
            const Meta& m = mt[u];
#pragma unroll
            for (int t = 0; t < NPER; ++t) acc[t] += m.pos ? zr[u][t] : -zr[u][t];
            if constexpr (DIAG) {
                if constexpr (Q == kQ2) {
                    if (m.a >= 1.0) {
#pragma unroll
                        for (int t = 0; t < NPER; ++t) dg[t] += 1.0;
                    } else if (m.a > 0.0) {
#pragma unroll
                        for (int t = 0; t < NPER; ++t) {
                            const double yh = zr[u][t] * m.ir;
                            dg[t] += m.a * (1.0 - yh * yh);
                        }
                    }
                } else if constexpr (Q == kQ1) {
#pragma unroll
                    for (int t = 0; t < NPER; ++t)
                        if (t < W && mask_bit<LPR>(pl.bits, m.l, W, 1, t, 0, gl)) dg[t] += 1.0;
                } else {
                    if (m.cnt < 0) {
#pragma unroll
                        for (int t = 0; t < NPER; ++t) dg[t] += 1.0;
                    } else if (m.cnt > 0) {
                        const double f = 1.0 - 1.0 / double(m.cnt);
#pragma unroll
                        for (int t = 0; t < NPER; ++t)
                            if (t < W && mask_bit<LPR>(pl.bits, m.l, W, 2, t, 0, gl)) dg[t] += f;
                    }
                }
            }
        }
    }
}

struct ScatterOut {
    double cx, ca, cz, sigma;
    const double* X;
    const double* A;
    double* out;
    double* Dinv;
    double* rowstats;  // optional n x 4: the four partial-sum terms of each vertex row
};

template <int LPR, int NPER, bool DIAG>
__device__ __forceinline__ void scatter_finish(int64_t v, int d, int gl, const ScatterOut& so,
                                               const double (&acc)[NPER], const double (&dg)[NPER],
                                               double (&acc4)[kScatterNV]) {
    double r4[kScatterNV] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < NPER; ++t) {
        const int k = gl + LPR * t;
        if (k < d) {
            const double xv = so.X ? so.X[v * d + k] : 0.0;
            const double av = so.A ? so.A[v * d + k] : 0.0;
            const double o = so.cx * xv + so.ca * av + so.cz * acc[t];
            so.out[v * d + k] = o;
            const double dx = xv - av;
            r4[0] += o * o;
            r4[1] += 0.5 * dx * dx;
            r4[2] += av * acc[t];
            r4[3] += acc[t] * acc[t];
            if constexpr (DIAG) so.Dinv[v * d + k] = 1.0 / (1.0 + so.sigma * dg[t]);
        }
    }
#pragma unroll
    for (int c = 0; c < kScatterNV; ++c) acc4[c] += r4[c];
    if (so.rowstats) {
#pragma unroll
        for (int c = 0; c < kScatterNV; ++c) {
            const double tot = group_sum<LPR>(r4[c]);
            if (gl == 0) so.rowstats[v * kScatterNV + c] = tot;
        }
    }
}

template <int LPR, int NPER, int Q, bool DIAG>
__global__ __launch_bounds__(kBlock) void k_scatter_chunk(DevGraph g, int d, ScatterOut so,
                                                          const double* __restrict__ Z, Payload pl,
                                                          double gamma,
                                                          double* __restrict__ partials) {
    const int gl = (threadIdx.x & 63) % LPR;
    constexpr int GPB = kBlock / LPR;
    const int W = (d + LPR - 1) / LPR;
    const int64_t T = g.nent;
    const int C = g.chunk;
    const int CW = 2 * d;
    double acc4[kScatterNV] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t c = int64_t(blockIdx.x) * GPB + threadIdx.x / LPR; c < g.nchunks;
         c += int64_t(gridDim.x) * GPB) {
        const int64_t cs = c * C;
        const int64_t ce = cs + C < T ? cs + C : T;
        int64_t v = g.chunk_v[c];
        int64_t p = cs;
        bool first = true;
        while (p < ce) {
            const int64_t vb = g.inc_ptr[v], ve = g.inc_ptr[v + 1];
            const int64_t se = ve < ce ? ve : ce;
            double acc[NPER], dg[NPER];
#pragma unroll
            for (int t = 0; t < NPER; ++t) acc[t] = dg[t] = 0.0;
            scatter_range<LPR, NPER, Q, DIAG>(p, se, d, gl, W, g.inc, Z, pl, g.w, gamma, acc, dg);
            if (vb >= cs && ve <= ce) {
                scatter_finish<LPR, NPER, DIAG>(v, d, gl, so, acc, dg, acc4);
            } else {
                double* cr = g.carry + (c * 2 + (first ? 0 : 1)) * CW;
#pragma unroll
                for (int t = 0; t < NPER; ++t) {
                    const int k = gl + LPR * t;
                    if (k < d) {
                        cr[k] = acc[t];
                        if constexpr (DIAG) cr[d + k] = dg[t];
                    }
                }
            }
            p = se;
            first = false;
            if (p < ce) {
                ++v;
                while (g.inc_ptr[v + 1] <= p) ++v;  // skip isolated vertices
            }
        }
    }
    block_reduce_store<kScatterNV>(acc4, partials + blockIdx.x * kScatterNV);
}

template <int LPR, int NPER, bool DIAG>
__global__ __launch_bounds__(kBlock) void k_scatter_fix(DevGraph g, int d, ScatterOut so,
                                                        double* __restrict__ partials) {
    const int gl = (threadIdx.x & 63) % LPR;
    constexpr int GPB = kBlock / LPR;
    const int C = g.chunk;
    const int CW = 2 * d;
    double acc4[kScatterNV] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t s = int64_t(blockIdx.x) * GPB + threadIdx.x / LPR; s < g.nspecial;
         s += int64_t(gridDim.x) * GPB) {
        const int64_t v = g.special[s];
        const int64_t vb = g.inc_ptr[v], ve = g.inc_ptr[v + 1];
        double acc[NPER], dg[NPER];
#pragma unroll
        for (int t = 0; t < NPER; ++t) acc[t] = dg[t] = 0.0;
        if (ve > vb) {
            for (int64_t c = vb / C; c <= (ve - 1) / C; ++c) {
                const double* cr = g.carry + (c * 2 + (g.chunk_v[c] == v ? 0 : 1)) * CW;
#pragma unroll
                for (int t = 0; t < NPER; ++t) {
                    const int k = gl + LPR * t;
                    if (k < d) {
                        acc[t] += cr[k];
                        if constexpr (DIAG) dg[t] += cr[d + k];
                    }
                }
            }
        }
        scatter_finish<LPR, NPER, DIAG>(v, d, gl, so, acc, dg, acc4);
    }
    block_reduce_store<kScatterNV>(acc4, partials + blockIdx.x * kScatterNV);
}

// ---- Newton matvec ------------------------------------------------------------

template <int LPR, int NPER, int Q, int MODE>
__device__ __forceinline__ void matvec_range(int64_t pa, int64_t pb, int d, int gl, int W,
                                             const Inc* __restrict__ inc,
                                             const double* __restrict__ V,
                                             const double* __restrict__ Pi, const Payload& pl,
                                             const double* __restrict__ w, double gamma,
                                             const double (&vi)[NPER], double (&acc)[NPER]) {
    constexpr int U = Unroll<NPER>::U;
    constexpr bool PAY = MODE == 0 || MODE == 2;
    constexpr int QP = MODE == 2 ? kQ2 : Q;
    for (int64_t p0 = pa; p0 < pb; p0 += U) {
        Meta mt[U];
        double vo[U][NPER];
        double pv[U][NPER];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (p0 + u < pb) mt[u] = load_meta<QP, PAY, MODE == 2>(inc, p0 + u, pl, w, gamma);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = p0 + u < pb;
            const bool rows = ok && PAY && QP == kQ2 && mt[u].f != 0.0;
#pragma unroll
            for (int t = 0; t < NPER; ++t) {
                const int k = gl + LPR * t;
                vo[u][t] = (ok && k < d) ? V[mt[u].o * d + k] : 0.0;
                pv[u][t] = (rows && k < d) ? Pi[mt[u].l * d + k] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (p0 + u >= pb) break;
            const Meta& m = mt[u];
            double dl[NPER];
#pragma unroll
            for (int t = 0; t < NPER; ++t) dl[t] = vi[t] - vo[u][t];
            if constexpr (MODE == 1) {
#pragma unroll
                for (int t = 0; t < NPER; ++t) acc[t] += dl[t];
            } else if constexpr (MODE == 2) {
                // adjoint curvature a (I - yhat yhat^T) on every edge with a > 0
                if (m.a > 0.0) {
                    double c = 0.0;
#pragma unroll
                    for (int t = 0; t < NPER; ++t) c += pv[u][t] * dl[t];
                    c = group_sum<LPR>(c) * m.f;
#pragma unroll
                    for (int t = 0; t < NPER; ++t) acc[t] += m.a * dl[t] - c * pv[u][t];
                }
            } else if constexpr (Q == kQ2) {
                // P = I inside the ball; a (I - yhat yhat^T) outside with
                // yhat = Pi_l / r, applied as a dl - (a / r^2) <Pi_l, dl> Pi_l
                if (m.a >= 1.0) {
#pragma unroll
                    for (int t = 0; t < NPER; ++t) acc[t] += dl[t];
                } else if (m.a > 0.0) {
                    double c = 0.0;
#pragma unroll
                    for (int t = 0; t < NPER; ++t) c += pv[u][t] * dl[t];
                    c = group_sum<LPR>(c) * m.f;
#pragma unroll
                    for (int t = 0; t < NPER; ++t) acc[t] += m.a * dl[t] - c * pv[u][t];
                }
            } else if constexpr (Q == kQ1) {
                // P = diag(1[|y_k| <= r])
#pragma unroll
                for (int t = 0; t < NPER; ++t)
                    if (t < W && mask_bit<LPR>(pl.bits, m.l, W, 1, t, 0, gl)) acc[t] += dl[t];
            } else {
                // P = I inside; diag(1_S) - s_S s_S^T / |S| outside
                if (m.cnt < 0) {
#pragma unroll
                    for (int t = 0; t < NPER; ++t) acc[t] += dl[t];
                } else if (m.cnt > 0) {
                    bool inS[NPER], neg[NPER];
                    double sd = 0.0;
#pragma unroll
                    for (int t = 0; t < NPER; ++t) {
                        inS[t] = (t < W) && mask_bit<LPR>(pl.bits, m.l, W, 2, t, 0, gl);
                        neg[t] = (t < W) && mask_bit<LPR>(pl.bits, m.l, W, 2, t, 1, gl);
                        if (inS[t]) sd += neg[t] ? -dl[t] : dl[t];
                    }
                    sd = group_sum<LPR>(sd) / double(m.cnt);
#pragma unroll
                    for (int t = 0; t < NPER; ++t)
                        if (inS[t]) acc[t] += dl[t] - (neg[t] ? -sd : sd);
                }
            }
        }
    }
}

struct MatvecOut {
    double sigma, c0;
    const double* dscale;
    double* out;
};

template <int LPR, int NPER>
__device__ __forceinline__ void load_row(const double* __restrict__ V, int64_t v, int d, int gl,
                                         double (&r)[NPER]) {
#pragma unroll
    for (int t = 0; t < NPER; ++t) {
        const int k = gl + LPR * t;
        r[t] = (k < d) ? V[v * d + k] : 0.0;
    }
}

template <int LPR, int NPER>
__device__ __forceinline__ void matvec_finish(int64_t v, int d, int gl, const MatvecOut& mo,
                                              const double (&vi)[NPER], const double (&acc)[NPER],
                                              double& dot) {
    const double sc = mo.dscale ? mo.dscale[v] : mo.c0;
#pragma unroll
    for (int t = 0; t < NPER; ++t) {
        const int k = gl + LPR * t;
        if (k < d) {
            const double o = sc * vi[t] + mo.sigma * acc[t];
            mo.out[v * d + k] = o;
            dot += vi[t] * o;
        }
    }
}

__device__ __forceinline__ bool cg_skip(const CgSkip& skip) {
    if (skip.done && *skip.done) return true;
    if (skip.rr_partials) {
        const double rr = block_sum_partials(skip.rr_partials, skip.nparts, 2, 1);
        if (rr <= skip.thr) return true;
    }
    return false;
}

template <int LPR, int NPER, int Q, int MODE>
__global__ __launch_bounds__(kBlock) void k_matvec_chunk(DevGraph g, int d,
                                                         const double* __restrict__ V,
                                                         const double* __restrict__ Pi,
                                                         Payload pl, double gamma, MatvecOut mo,
                                                         double* __restrict__ partials,
                                                         CgSkip skip) {
    if (cg_skip(skip)) return;
    const int gl = (threadIdx.x & 63) % LPR;
    constexpr int GPB = kBlock / LPR;
    const int W = (d + LPR - 1) / LPR;
    const int64_t T = g.nent;
    const int C = g.chunk;
    const int CW = 2 * d;
    double dot[1] = {0.0};
    for (int64_t c = int64_t(blockIdx.x) * GPB + threadIdx.x / LPR; c < g.nchunks;
         c += int64_t(gridDim.x) * GPB) {
        const int64_t cs = c * C;
        const int64_t ce = cs + C < T ? cs + C : T;
        int64_t v = g.chunk_v[c];
        int64_t p = cs;
        bool first = true;
        while (p < ce) {
            const int64_t vb = g.inc_ptr[v], ve = g.inc_ptr[v + 1];
            const int64_t se = ve < ce ? ve : ce;
            double vi[NPER], acc[NPER];
            load_row<LPR, NPER>(V, v, d, gl, vi);
#pragma unroll
            for (int t = 0; t < NPER; ++t) acc[t] = 0.0;
            matvec_range<LPR, NPER, Q, MODE>(p, se, d, gl, W, g.inc, V, Pi, pl, g.w, gamma, vi,
                                             acc);
            if (vb >= cs && ve <= ce) {
                matvec_finish<LPR, NPER>(v, d, gl, mo, vi, acc, dot[0]);
            } else {
                double* cr = g.carry + (c * 2 + (first ? 0 : 1)) * CW;
#pragma unroll
                for (int t = 0; t < NPER; ++t) {
                    const int k = gl + LPR * t;
                    if (k < d) cr[k] = acc[t];
                }
            }
            p = se;
            first = false;
            if (p < ce) {
                ++v;
                while (g.inc_ptr[v + 1] <= p) ++v;  // skip isolated vertices
            }
        }
    }
    block_reduce_store<kMatvecNV>(dot, partials + blockIdx.x * kMatvecNV);
}

template <int LPR, int NPER>
__global__ __launch_bounds__(kBlock) void k_matvec_fix(DevGraph g, int d,
                                                       const double* __restrict__ V, MatvecOut mo,
                                                       double* __restrict__ partials,
                                                       CgSkip skip) {
    if (cg_skip(skip)) return;
    const int gl = (threadIdx.x & 63) % LPR;
    constexpr int GPB = kBlock / LPR;
    const int C = g.chunk;
    const int CW = 2 * d;
    double dot[1] = {0.0};
    for (int64_t s = int64_t(blockIdx.x) * GPB + threadIdx.x / LPR; s < g.nspecial;
         s += int64_t(gridDim.x) * GPB) {
        const int64_t v = g.special[s];
        const int64_t vb = g.inc_ptr[v], ve = g.inc_ptr[v + 1];
        double vi[NPER], acc[NPER];
        load_row<LPR, NPER>(V, v, d, gl, vi);
#pragma unroll
        for (int t = 0; t < NPER; ++t) acc[t] = 0.0;
        if (ve > vb) {
            for (int64_t c = vb / C; c <= (ve - 1) / C; ++c) {
                const double* cr = g.carry + (c * 2 + (g.chunk_v[c] == v ? 0 : 1)) * CW;
#pragma unroll
                for (int t = 0; t < NPER; ++t) {
                    const int k = gl + LPR * t;
                    if (k < d) acc[t] += cr[k];
                }
            }
        }
        matvec_finish<LPR, NPER>(v, d, gl, mo, vi, acc, dot[0]);
    }
    block_reduce_store<kMatvecNV>(dot, partials + blockIdx.x * kMatvecNV);
}

}  // namespace

int launch_scatter(const DevGraph& g, int d, int qk, double cx, const double* X, double ca,
                   const double* A, double cz, const double* Z, double* out, bool diag, Payload pl,
                   double gamma, double sigma, double* Dinv, double* partials, hipStream_t s,
                   double* rowstats) {
    int total = 0;
    ScatterOut so{cx, ca, cz, sigma, X, A, out, Dinv, rowstats};
    dispatch_row(d, [&](auto L, auto N) {
        constexpr int lpr = decltype(L)::value, nper = decltype(N)::value;
        const int g1 = g.nchunks > 0 ? row_grid(g.nchunks, lpr) : 0;
        const int g2 = row_grid(g.nspecial, lpr);
        if (!diag) {
            if (g1 > 0)
                hipLaunchKernelGGL((k_scatter_chunk<lpr, nper, kQ2, false>), dim3(g1), dim3(kBlock),
                                   0, s, g, d, so, Z, pl, gamma, partials);
            hipLaunchKernelGGL((k_scatter_fix<lpr, nper, false>), dim3(g2), dim3(kBlock), 0, s, g,
                               d, so, partials + g1 * kScatterNV);
        } else {
            if (g1 > 0) {
                dispatch_q(qk, [&](auto Qc) {
                    constexpr int q = decltype(Qc)::value;
                    hipLaunchKernelGGL((k_scatter_chunk<lpr, nper, q, true>), dim3(g1),
                                       dim3(kBlock), 0, s, g, d, so, Z, pl, gamma, partials);
                });
            }
            hipLaunchKernelGGL((k_scatter_fix<lpr, nper, true>), dim3(g2), dim3(kBlock), 0, s, g,
                               d, so, partials + g1 * kScatterNV);
        }
        total = g1 + g2;
    });
    return total;
}

int launch_matvec(const DevGraph& g, int d, int qk, int mode, const double* V, const double* Pi,
                  Payload pl, double gamma, double sigma, double c0, const double* dscale,
                  double* out, double* partials, CgSkip skip, hipStream_t s) {
    int total = 0;
    MatvecOut mo{sigma, c0, dscale, out};
    dispatch_row(d, [&](auto L, auto N) {
        constexpr int lpr = decltype(L)::value, nper = decltype(N)::value;
        const int g1 = g.nchunks > 0 ? row_grid(g.nchunks, lpr) : 0;
        const int g2 = row_grid(g.nspecial, lpr);
        if (g1 > 0) {
            if (mode == 1) {
                hipLaunchKernelGGL((k_matvec_chunk<lpr, nper, kQ2, 1>), dim3(g1), dim3(kBlock), 0,
                                   s, g, d, V, Pi, pl, gamma, mo, partials, skip);
            } else if (mode == 2) {
                hipLaunchKernelGGL((k_matvec_chunk<lpr, nper, kQ2, 2>), dim3(g1), dim3(kBlock), 0,
                                   s, g, d, V, Pi, pl, gamma, mo, partials, skip);
            } else {
                dispatch_q(qk, [&](auto Qc) {
                    constexpr int q = decltype(Qc)::value;
                    hipLaunchKernelGGL((k_matvec_chunk<lpr, nper, q, 0>), dim3(g1), dim3(kBlock),
                                       0, s, g, d, V, Pi, pl, gamma, mo, partials, skip);
                });
            }
        }
        hipLaunchKernelGGL((k_matvec_fix<lpr, nper>), dim3(g2), dim3(kBlock), 0, s, g, d, V, mo,
                           partials + g1 * kMatvecNV, skip);
        total = g1 + g2;
    });
    return total;
}

}  // namespace ccm
