// Vertex-centric kernels: the transposed operator B^T (a signed sum of edge
// rows into vertex rows) and the SSNAL Newton matvec V + sigma B^T P B V.
//
// Both walk the vertex-major incidence array (entries sorted by vertex, each
// vertex's entries in ascending edge order).  k-NN graphs are skewed (a few
// hub vertices have tens of times the mean degree), so work is split by
// entries, not by vertices: a workgroup takes a window of whole vertices and
// its row groups split the window's entries evenly.  A row group finishes
// every vertex whose entries lie inside its share; a vertex cut between row
// groups leaves its later pieces in LDS, and the row group where it starts
// adds them in row-group order after a barrier.  There are no atomics and
// the summation order is fixed, so results are bit-reproducible.  An edge row
// is read by both of its endpoints.
//
// Everything needed to issue an entry's row gathers (edge, other endpoint,
// the entry's own vertex, the Jacobian scalars) is stored at the entry's
// position, so a batch of U entries costs one round of independent index
// loads and then one round of row loads; vertex boundaries are read off the
// per-entry vertex ids, and the neighbours irow[p0 - 1], irow[p1] of a row
// group's share [p0, p1) tell whether its first and last vertices are cut.
#include <algorithm>

#include "launch.hpp"
#include "proj.hpp"

namespace ccm {
namespace {

// entries per batch: the batch's rows are gathered together.  Short rows
// are latency-bound, so their kernels also gather the next vertex's own rows
// with the batch; long rows are bandwidth-bound and keep registers for
// occupancy instead.
template <int NPER>
struct Unroll {
    static constexpr int U = NPER <= 2 ? 8 : NPER == 4 ? 4 : NPER == 8 ? 2 : 1;   // matvec
    static constexpr int US = NPER <= 2 ? 8 : NPER == 4 ? 4 : NPER == 8 ? 2 : 1;  // scatter
    static constexpr bool PREFETCH = NPER <= 4;
};

// Per-incidence data.  q = 2: a = r/||y|| outside the ball, 1 inside; ir = 1/r
// and f = a / r^2 where the Jacobian is a (I - yhat yhat^T); q = inf: support
// size, -1 inside.
struct Meta {
    int l, o, v;
    bool pos;
    double a, ir, f;
    int cnt;
};

template <int Q, bool PAY, bool ADJ = false>
__device__ __forceinline__ Meta load_meta(const DevGraph& g, int64_t p, const Payload& pl) {
    const Inc e = g.inc[p];
    Meta m;
    m.pos = e.e >= 0;
    m.l = m.pos ? e.e : ~e.e;
    m.o = e.o;
    m.v = g.irow[p];
    m.a = 1.0;
    m.ir = 0.0;
    m.f = 0.0;
    m.cnt = -1;
    if constexpr (PAY && Q == kQ2) {
        const double2 q = pl.ipay[p];
        m.a = q.x;
        m.ir = q.y;
        if ((ADJ || m.a < 1.0) && m.a > 0.0) m.f = m.a * m.ir * m.ir;
    } else if constexpr (PAY && Q == kQInf) {
        m.cnt = int(pl.ipay[p].x);
    }
    return m;
}

// Row-group share that a layout's incidence prefetch is sized for (the
// window chunk before the window table was tuned); a row group with a longer
// share loads its incidence data in several rounds, one with a shorter share
// leaves slots empty.
template <int LPR, int NPER>
constexpr int chunk_of() {
    return LPR * NPER <= 64 ? 16 : LPR * NPER <= 256 ? 32 : 64;
}

// Slots of LPR entries whose incidence data a row group loads in one round:
// its whole share unless the window is a hub's.
template <int LPR, int NPER>
constexpr int meta_slots() {
    constexpr int c = chunk_of<LPR, NPER>() / LPR;
    return c >= 1 ? c : 1;
}

// Incidence data of up to NM LPR entries, loaded in one round and spread over
// the lanes of the row group (entry j LPR + lane in slot j); an entry's data
// is then fetched with lane shuffles instead of another round of loads.
template <int LPR, int NM>
struct ChunkMeta {
    int e[NM], o[NM], v[NM];
    double a[NM], ir[NM];
};

template <int LPR, int NM, int Q, bool PAY>
__device__ __forceinline__ void chunk_meta_load(const DevGraph& g, int64_t cs, int64_t ce, int gl,
                                                const Payload& pl, ChunkMeta<LPR, NM>& cm) {
#pragma unroll
    for (int j = 0; j < NM; ++j) {
        const int64_t p = cs + j * LPR + gl;
        cm.e[j] = 0;
        cm.o[j] = 0;
        cm.v[j] = -1;
        cm.a[j] = 1.0;
        cm.ir[j] = 0.0;
        if (p < ce) {
            const Inc in = g.inc[p];
            cm.e[j] = in.e;
            cm.o[j] = in.o;
            cm.v[j] = g.irow[p];
            if constexpr (PAY && Q == kQ2) {
                const double2 q = pl.ipay[p];
                cm.a[j] = q.x;
                cm.ir[j] = q.y;
            } else if constexpr (PAY && Q == kQInf) {
                cm.a[j] = pl.ipay[p].x;
            }
        }
    }
}

template <int LPR, int NM, int Q, bool PAY, bool ADJ>
__device__ __forceinline__ Meta chunk_meta_get(const ChunkMeta<LPR, NM>& cm, int q) {
    const int j = q / LPR, src = q % LPR;
    int e = cm.e[0], o = cm.o[0], v = cm.v[0];
    double a = cm.a[0], ir = cm.ir[0];
#pragma unroll
    for (int jj = 1; jj < NM; ++jj) {
        if (j == jj) {
            e = cm.e[jj];
            o = cm.o[jj];
            v = cm.v[jj];
            a = cm.a[jj];
            ir = cm.ir[jj];
        }
    }
    Meta m;
    e = __shfl(e, src, LPR);
    m.o = __shfl(o, src, LPR);
    m.v = __shfl(v, src, LPR);
    if constexpr (LPR == 64) {
        // a whole wave shares the entry: keep its indices in scalar registers,
        // so row addresses are a scalar base plus the lane's offset
        e = __builtin_amdgcn_readfirstlane(e);
        m.o = __builtin_amdgcn_readfirstlane(m.o);
        m.v = __builtin_amdgcn_readfirstlane(m.v);
    }
    m.pos = e >= 0;
    m.l = m.pos ? e : ~e;
    m.a = 1.0;
    m.ir = 0.0;
    m.f = 0.0;
    m.cnt = -1;
    if constexpr (PAY && Q == kQ2) {
        m.a = __shfl(a, src, LPR);
        m.ir = __shfl(ir, src, LPR);
        if ((ADJ || m.a < 1.0) && m.a > 0.0) m.f = m.a * m.ir * m.ir;
    } else if constexpr (PAY && Q == kQInf) {
        m.cnt = int(__shfl(a, src, LPR));
    }
    return m;
}

// Share [p0, p1) of row group rg (of GPB) in window w, and the vertices of the
// entries just before and after it inside the window (-1 if none).
// (Entry positions fit 32 bits: the incidence offsets are 32-bit.)
struct GroupRange {
    int p0, p1;
    int vprev, vnext;
};

__device__ __forceinline__ GroupRange group_range(const DevGraph& g, int w, int rg, int gpb) {
    const int2 wn = g.win[w];
    const int ws = wn.x, we = wn.y;
    const int sc = (we - ws + gpb - 1) / gpb;
    GroupRange r;
    r.p0 = ws + rg * sc < we ? ws + rg * sc : we;
    r.p1 = r.p0 + sc < we ? r.p0 + sc : we;
    const bool any = r.p0 < r.p1;
    r.vprev = (any && r.p0 > ws) ? g.irow[r.p0 - 1] : -1;
    r.vnext = (any && r.p1 < we) ? g.irow[r.p1] : -1;
    return r;
}

template <int LPR, int NPER>
__device__ __forceinline__ void load_row(const double* __restrict__ V, int64_t v, int d, int gl,
                                         double (&r)[NPER]) {
#pragma unroll
    for (int t = 0; t < NPER; ++t) {
        const int k = gl + LPR * t;
        r[t] = (V && k < d) ? V[v * d + k] : 0.0;
    }
}

// ---- B^T Z (and the Jacobi diagonal of I + sigma B^T P B) -------------------

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
                                               const double (&xr)[NPER], const double (&ar)[NPER],
                                               const double (&acc)[NPER], const double (&dg)[NPER],
                                               double (&acc4)[kScatterNV]) {
    double r4[kScatterNV] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < NPER; ++t) {
        const int k = gl + LPR * t;
        if (k < d) {
            const double o = so.cx * xr[t] + so.ca * ar[t] + so.cz * acc[t];
            so.out[v * d + k] = o;
            const double dx = xr[t] - ar[t];
            r4[0] += o * o;
            r4[1] += 0.5 * dx * dx;
            r4[2] += ar[t] * acc[t];
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
__global__ __launch_bounds__(kBlock) void k_scatter_win(DevGraph g, int d, ScatterOut so,
                                                        const double* __restrict__ Z, Payload pl,
                                                        double* __restrict__ partials) {
    constexpr int U = Unroll<NPER>::US;
    constexpr int NM = meta_slots<LPR, NPER>();
    constexpr bool PF = NM <= 4;  // share data fits a few registers per lane
    constexpr int GPB = kBlock / LPR;
    constexpr int NS = DIAG ? 2 : 1;
    // later pieces of cut vertices: [row group][sum][value][lane]
    __shared__ double piece[GPB][NS][NPER][LPR];
    __shared__ int head_v[GPB];  // vertex of the row group's first piece if cut, else -1
    const int gl = (threadIdx.x & 63) % LPR;
    const int rg = threadIdx.x / LPR;
    double acc4[kScatterNV] = {0.0, 0.0, 0.0, 0.0};
    for (int w = blockIdx.x; w < int(g.nwin); w += gridDim.x) {
        const GroupRange gr = group_range(g, w, rg, GPB);
        int vcur = -1;
        bool first = true;
        int head = -1;
        double acc[NPER], dg[NPER], xr[NPER], ar[NPER];
#pragma unroll
        for (int t = 0; t < NPER; ++t) acc[t] = dg[t] = xr[t] = ar[t] = 0.0;
        auto finish = [&]() {
            if constexpr (!Unroll<NPER>::PREFETCH) {
                double x2[NPER], a2[NPER];
                load_row<LPR, NPER>(so.X, vcur, d, gl, x2);
                load_row<LPR, NPER>(so.A, vcur, d, gl, a2);
                scatter_finish<LPR, NPER, DIAG>(vcur, d, gl, so, x2, a2, acc, dg, acc4);
            } else {
                scatter_finish<LPR, NPER, DIAG>(vcur, d, gl, so, xr, ar, acc, dg, acc4);
            }
        };
        // vertex vcur has no more entries in this share
        auto done = [&](bool cut_start) {
            if (!cut_start) {
                finish();
            } else {
#pragma unroll
                for (int t = 0; t < NPER; ++t) {
                    piece[rg][0][t][gl] = acc[t];
                    if constexpr (DIAG) piece[rg][NS - 1][t][gl] = dg[t];
                }
                head = vcur;
            }
        };
        constexpr int CP = NM * LPR;  // entries per round of incidence loads
        for (int pc = gr.p0, pe = 0; pc < gr.p1; pc = pe) {
            pe = (PF && gr.p1 - pc > CP) ? pc + CP : gr.p1;
            ChunkMeta<LPR, PF ? NM : 1> cm;
            if constexpr (PF) chunk_meta_load<LPR, NM, Q, DIAG>(g, pc, pe, gl, pl, cm);
            for (int p0 = pc; p0 < pe; p0 += U) {
                Meta mt[U];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (p0 + u < pe) {
                        if constexpr (PF)
                            mt[u] = chunk_meta_get<LPR, NM, Q, DIAG, false>(cm, p0 + u - pc);
                        else
                            mt[u] = load_meta<Q, DIAG>(g, p0 + u, pl);
                    }
                double zr[U][NPER];
                uint32_t lb[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const bool ok = p0 + u < pe;
#pragma unroll
                    for (int t = 0; t < NPER; ++t) {
                        const int k = gl + LPR * t;
                        zr[u][t] = (ok && k < d) ? Z[int64_t(mt[u].l) * d + k] : 0.0;
                    }
                    lb[u] = 0u;
                    if constexpr (DIAG && Q != kQ2)
                        if (ok) lb[u] = pl.lbits[int64_t(mt[u].l) * LPR + gl];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (p0 + u >= pe) break;
                    const Meta& m = mt[u];
                    if (m.v != vcur) {
                        if (vcur >= 0) {
                            done(first && vcur == gr.vprev);
                            first = false;
                        }
                        vcur = m.v;
                        if constexpr (Unroll<NPER>::PREFETCH) {
                            load_row<LPR, NPER>(so.X, vcur, d, gl, xr);
                            load_row<LPR, NPER>(so.A, vcur, d, gl, ar);
                        }
#pragma unroll
                        for (int t = 0; t < NPER; ++t) acc[t] = dg[t] = 0.0;
                    }
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
                                if ((lb[u] >> t) & 1u) dg[t] += 1.0;
                        } else {
                            if (m.cnt < 0) {
#pragma unroll
                                for (int t = 0; t < NPER; ++t) dg[t] += 1.0;
                            } else if (m.cnt > 0) {
                                const double f = 1.0 - 1.0 / double(m.cnt);
#pragma unroll
                                for (int t = 0; t < NPER; ++t)
                                    if ((lb[u] >> t) & 1u) dg[t] += f;
                            }
                        }
                    }
                }
            }
        }
        // the last vertex: finished here, or (continuing past the share)
        // after the barrier with the later row groups' pieces
        bool pend = false;
        if (vcur >= 0) {
            const bool cs = first && vcur == gr.vprev;
            if (!cs && vcur == gr.vnext) pend = true;
            else done(cs);
        }
        if (gl == 0) head_v[rg] = head;
        __syncthreads();
        if (pend) {
            for (int j = rg + 1; j < GPB && head_v[j] == vcur; ++j) {
#pragma unroll
                for (int t = 0; t < NPER; ++t) {
                    acc[t] += piece[j][0][t][gl];
                    if constexpr (DIAG) dg[t] += piece[j][NS - 1][t][gl];
                }
            }
            finish();
        }
        __syncthreads();
    }
    // isolated vertices
    for (int64_t i = int64_t(blockIdx.x) * GPB + rg; i < g.niso; i += int64_t(gridDim.x) * GPB) {
        const int64_t v = g.iso[i];
        double acc[NPER], dg[NPER], xr[NPER], ar[NPER];
#pragma unroll
        for (int t = 0; t < NPER; ++t) acc[t] = dg[t] = 0.0;
        load_row<LPR, NPER>(so.X, v, d, gl, xr);
        load_row<LPR, NPER>(so.A, v, d, gl, ar);
        scatter_finish<LPR, NPER, DIAG>(v, d, gl, so, xr, ar, acc, dg, acc4);
    }
    block_reduce_store<kScatterNV>(acc4, partials + blockIdx.x * kScatterNV);
}

// ---- SSNAL edge pass fused with the gradient -----------------------------------
// For every incidence of vertex v on edge l = (i, j): y_l = u_l + sigma (x_i -
// x_j) and its projection Pi_l, recomputed by both endpoints from the same
// operands in the same order (so bit-identical); the signed Pi_l enters
// G_v = x_v - a_v + (B^T Pi)_v and the Jacobi diagonal of I + sigma B^T P B.
// The first endpoint alone stores Pi_l, the lane masks and the edge's terms
// of the merit function; each endpoint stores the Jacobian scalars at its own
// incidence position.

template <int NPER>
struct EdgeGradUnroll {
    static constexpr int U = NPER <= 2 ? 4 : NPER == 4 ? 2 : 1;
};

// With KKT, the first endpoint also adds the edge's terms of the KKT
// residuals at (X, U) (as k_edge_kkt: ||Pi_C(BX + U) - U||^2, ||BX||^2,
// ||U||^2, ||U - Pi_C(U)||^2, r ||(BX)_l||_q) into kpart.
// (rows of up to 13 values per lane are held to two waves per SIMD)
template <int NPER>
constexpr int edge_grad_min_waves() { return NPER <= 13 ? 2 : 1; }

template <int LPR, int NPER, int Q, bool KKT>
__global__ __launch_bounds__(kBlock, edge_grad_min_waves<NPER>()) void k_edge_grad_win(
                                                          DevGraph g, int d, ScatterOut so,
                                                          double gamma,
                                                          const double* __restrict__ U,
                                                          double* __restrict__ Pi, Payload pl,
                                                          double* __restrict__ epart,
                                                          double* __restrict__ spart,
                                                          double* __restrict__ kpart) {
    static_assert(!KKT || Q == kQ1 || Q == kQ2, "the fused KKT terms serve q = 1 and q = 2");
    constexpr int UB = EdgeGradUnroll<NPER>::U;
    constexpr int NM = meta_slots<LPR, NPER>();
    constexpr bool PF = NM <= 4;
    constexpr int GPB = kBlock / LPR;
    __shared__ double piece[GPB][2][NPER][LPR];
    __shared__ int head_v[GPB];
    const int lane = threadIdx.x & 63;
    const int gl = lane % LPR;
    const int rg = threadIdx.x / LPR;
    const double sigma = so.sigma;
    double acc4[kScatterNV] = {0.0, 0.0, 0.0, 0.0};
    double eacc[kEdgeSsnalNV] = {0.0, 0.0, 0.0, 0.0, 0.0};
    // the KKT sums of each lane live in LDS (one slot per lane and term,
    // touched only by its lane, in program order), not in registers
    __shared__ double kl[KKT ? 4 : 1][kBlock];
    if constexpr (KKT) {
#pragma unroll
        for (int c = 0; c < 4; ++c) kl[c][threadIdx.x] = 0.0;
    }
    auto kadd = [&](int c, double v) {
        __hip_atomic_fetch_add(&kl[c][threadIdx.x], v, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    for (int w = blockIdx.x; w < int(g.nwin); w += gridDim.x) {
        const GroupRange gr = group_range(g, w, rg, GPB);
        int vcur = -1;
        bool first = true;
        int head = -1;
        double acc[NPER], dg[NPER], xr[NPER], ar[NPER];
#pragma unroll
        for (int t = 0; t < NPER; ++t) acc[t] = dg[t] = xr[t] = ar[t] = 0.0;
        // long rows read A only when the vertex is finished (registers)
        auto finish = [&]() {
            if constexpr (Unroll<NPER>::PREFETCH) {
                scatter_finish<LPR, NPER, true>(vcur, d, gl, so, xr, ar, acc, dg, acc4);
            } else {
                double a2[NPER];
                load_row<LPR, NPER>(so.A, vcur, d, gl, a2);
                scatter_finish<LPR, NPER, true>(vcur, d, gl, so, xr, a2, acc, dg, acc4);
            }
        };
        auto done = [&](bool cut_start) {
            if (!cut_start) {
                finish();
            } else {
#pragma unroll
                for (int t = 0; t < NPER; ++t) {
                    piece[rg][0][t][gl] = acc[t];
                    piece[rg][1][t][gl] = dg[t];
                }
                head = vcur;
            }
        };
        constexpr int CP = NM * LPR;
        for (int pc = gr.p0, pe = 0; pc < gr.p1; pc = pe) {
            pe = (PF && gr.p1 - pc > CP) ? pc + CP : gr.p1;
            ChunkMeta<LPR, PF ? NM : 1> cm;
            if constexpr (PF) chunk_meta_load<LPR, NM, Q, false>(g, pc, pe, gl, pl, cm);
            for (int p0 = pc; p0 < pe; p0 += UB) {
                Meta mt[UB];
#pragma unroll
                for (int u = 0; u < UB; ++u)
                    if (p0 + u < pe) {
                        if constexpr (PF)
                            mt[u] = chunk_meta_get<LPR, NM, Q, false, false>(cm, p0 + u - pc);
                        else
                            mt[u] = load_meta<Q, false>(g, p0 + u, pl);
                    }
                double xo[UB][NPER], ur[UB][NPER], wl[UB];
#pragma unroll
                for (int u = 0; u < UB; ++u) {
                    const bool ok = p0 + u < pe;
                    wl[u] = ok ? g.w[mt[u].l] : 0.0;
#pragma unroll
                    for (int t = 0; t < NPER; ++t) {
                        const int k = gl + LPR * t;
                        xo[u][t] = (ok && k < d) ? so.X[int64_t(mt[u].o) * d + k] : 0.0;
                        ur[u][t] = (ok && k < d) ? U[int64_t(mt[u].l) * d + k] : 0.0;
                    }
                }
#pragma unroll
                for (int u = 0; u < UB; ++u) {
                    if (p0 + u >= pe) break;
                    const Meta& m = mt[u];
                    if (m.v != vcur) {
                        if (vcur >= 0) {
                            done(first && vcur == gr.vprev);
                            first = false;
                        }
                        vcur = m.v;
                        load_row<LPR, NPER>(so.X, vcur, d, gl, xr);
                        if constexpr (Unroll<NPER>::PREFETCH)
                            load_row<LPR, NPER>(so.A, vcur, d, gl, ar);
#pragma unroll
                        for (int t = 0; t < NPER; ++t) acc[t] = dg[t] = 0.0;
                    }
                    // the edge's row, oriented first endpoint minus second
                    const double r = gamma * wl[u];
                    double bx[NPER], pi[NPER];
#pragma unroll
                    for (int t = 0; t < NPER; ++t) {
                        bx[t] = m.pos ? xr[t] - xo[u][t] : xo[u][t] - xr[t];
                        pi[t] = ur[u][t] + sigma * bx[t];
                    }
                    // projection onto the dual ball in place (the same
                    // arithmetic as project_row): q = 2 scales by
                    // min(1, r / ||y||), q = 1 clamps to [-r, r], q = inf
                    // projects onto the l1 ball (project_row itself)
                    double alpha = 1.0;
                    uint32_t lm = 0u;
                    int cnt = -1;
                    if constexpr (Q == kQInf) {
                        RowProj<LPR, NPER, kQInf> o;
                        project_row<LPR, NPER, kQInf, true>(pi, gl, lane, d, r, o);
#pragma unroll
                        for (int t = 0; t < NPER; ++t) pi[t] = o.pi[t];
                        cnt = o.cnt;
                        lm = o.lm;
                    } else if constexpr (Q == kQ2) {
                        double s2 = 0.0;
#pragma unroll
                        for (int t = 0; t < NPER; ++t) s2 += pi[t] * pi[t];
                        const double nrm = sqrt(group_sum<LPR>(s2));
                        if (!(r >= kTinyRadius)) {
                            // a ball too small for 1/r: taken as {0}
                            alpha = 0.0;
#pragma unroll
                            for (int t = 0; t < NPER; ++t) pi[t] = 0.0;
                        } else if (nrm > r) {
                            alpha = r / nrm;
#pragma unroll
                            for (int t = 0; t < NPER; ++t) pi[t] *= alpha;
                        }
                    } else {
#pragma unroll
                        for (int t = 0; t < NPER; ++t) {
                            if (gl + LPR * t < d && fabs(pi[t]) <= r) lm |= 1u << t;
                            pi[t] = fmin(fmax(pi[t], -r), r);
                        }
                    }
#pragma unroll
                    for (int t = 0; t < NPER; ++t) acc[t] += m.pos ? pi[t] : -pi[t];
                    if constexpr (Q == kQ2) {
                        const double ir = alpha > 0.0 ? 1.0 / r : 0.0;
                        if (alpha >= 1.0) {
#pragma unroll
                            for (int t = 0; t < NPER; ++t) dg[t] += 1.0;
                        } else if (alpha > 0.0) {
#pragma unroll
                            for (int t = 0; t < NPER; ++t) {
                                const double yh = pi[t] * ir;
                                dg[t] += alpha * (1.0 - yh * yh);
                            }
                        }
                        if (gl == 0) pl.ipay[p0 + u] = double2{alpha, ir};
                    } else if constexpr (Q == kQInf) {
                        // P = I inside; diag(1_S) - s_S s_S^T / |S| outside
                        if (cnt < 0) {
#pragma unroll
                            for (int t = 0; t < NPER; ++t) dg[t] += 1.0;
                        } else if (cnt > 0) {
                            const double f = 1.0 - 1.0 / double(cnt);
#pragma unroll
                            for (int t = 0; t < NPER; ++t)
                                if ((lm >> t) & 1u) dg[t] += f;
                        }
                        if (gl == 0) pl.ipay[p0 + u] = double2{double(cnt), 0.0};
                    } else {
#pragma unroll
                        for (int t = 0; t < NPER; ++t)
                            if ((lm >> t) & 1u) dg[t] += 1.0;
                    }
                    if (m.pos) {
                        const int64_t l = m.l;
#pragma unroll
                        for (int t = 0; t < NPER; ++t) {
                            const int k = gl + LPR * t;
                            if (k < d) {
                                Pi[l * d + k] = pi[t];
                                const double e = pi[t] - ur[u][t];
                                eacc[0] += bx[t] * pi[t];
                                eacc[1] += e * e;
                                eacc[2] += bx[t] * bx[t];
                                eacc[3] += pi[t] * pi[t];
                            }
                        }
                        if constexpr (Q != kQ2) pl.lbits[l * LPR + gl] = lm;
                        if (gl == 0) {
                            if constexpr (Q == kQ2) eacc[4] += (alpha < 1.0) ? 1.0 : 0.0;
                            else if constexpr (Q == kQInf) eacc[4] += (cnt >= 0) ? 1.0 : 0.0;
                            else eacc[4] += 1.0;
                        }
                        if constexpr (KKT) {
                            // the edge's KKT terms at (X, U): v = (BX)_l + u_l and
                            // the projections of v and u_l, coordinate by
                            // coordinate (q = 2 scales by the row norms, q = 1
                            // clamps), so no projected row is held in registers
                            double nq = 0.0, sv = 0.0, su = 0.0;
#pragma unroll
                            for (int t = 0; t < NPER; ++t) {
                                const double vt = bx[t] + ur[u][t];
                                if constexpr (Q == kQ1) {
                                    nq += fabs(bx[t]);
                                } else {
                                    nq += bx[t] * bx[t];
                                    sv += vt * vt;
                                    su += ur[u][t] * ur[u][t];
                                }
                            }
                            double pen, av = 1.0, au = 1.0;
                            if constexpr (Q == kQ2) {
                                pen = r * sqrt(group_sum<LPR>(nq));
                                const double nv = sqrt(group_sum<LPR>(sv));
                                const double nu = sqrt(group_sum<LPR>(su));
                                if (nv > r) av = r / nv;
                                if (nu > r) au = r / nu;
                            } else {
                                pen = group_sum<LPR>(r * nq);
                            }
                            if (gl == 0) kadd(3, pen);
#pragma unroll
                            for (int t = 0; t < NPER; ++t) {
                                const int k = gl + LPR * t;
                                if (k < d) {
                                    const double vt = bx[t] + ur[u][t];
                                    double pvt, put;
                                    if constexpr (Q == kQ2) {
                                        pvt = av < 1.0 ? vt * av : vt;
                                        put = au < 1.0 ? ur[u][t] * au : ur[u][t];
                                    } else {
                                        pvt = fmin(fmax(vt, -r), r);
                                        put = fmin(fmax(ur[u][t], -r), r);
                                    }
                                    const double e = pvt - ur[u][t];
                                    const double f = ur[u][t] - put;
                                    kadd(0, e * e);
                                    kadd(1, ur[u][t] * ur[u][t]);
                                    kadd(2, f * f);
                                }
                            }
                        }
                    }
                }
            }
        }
        bool pend = false;
        if (vcur >= 0) {
            const bool cs = first && vcur == gr.vprev;
            if (!cs && vcur == gr.vnext) pend = true;
            else done(cs);
        }
        if (gl == 0) head_v[rg] = head;
        __syncthreads();
        if (pend) {
            for (int j = rg + 1; j < GPB && head_v[j] == vcur; ++j) {
#pragma unroll
                for (int t = 0; t < NPER; ++t) {
                    acc[t] += piece[j][0][t][gl];
                    dg[t] += piece[j][1][t][gl];
                }
            }
            finish();
        }
        __syncthreads();
    }
    // isolated vertices
    for (int64_t i = int64_t(blockIdx.x) * GPB + rg; i < g.niso; i += int64_t(gridDim.x) * GPB) {
        const int64_t v = g.iso[i];
        double acc[NPER], dg[NPER], xr[NPER], ar[NPER];
#pragma unroll
        for (int t = 0; t < NPER; ++t) acc[t] = dg[t] = 0.0;
        load_row<LPR, NPER>(so.X, v, d, gl, xr);
        load_row<LPR, NPER>(so.A, v, d, gl, ar);
        scatter_finish<LPR, NPER, true>(v, d, gl, so, xr, ar, acc, dg, acc4);
    }
    block_reduce_store<kScatterNV>(acc4, spart + blockIdx.x * kScatterNV);
    block_reduce_store<kEdgeSsnalNV>(eacc, epart + blockIdx.x * kEdgeSsnalNV);
    if constexpr (KKT) {
        // ||BX||^2 over the first endpoints' rows is the edge pass's own sum
        double kacc[kEdgeKktNV] = {kl[0][threadIdx.x], eacc[2], kl[1][threadIdx.x],
                                   kl[2][threadIdx.x], kl[3][threadIdx.x], 0.0};
        block_reduce_store<kEdgeKktNV>(kacc, kpart + blockIdx.x * kEdgeKktNV);
    }
}

// ---- Newton matvec ------------------------------------------------------------

struct MatvecOut {
    double sigma, c0;
    const double* dscale;
    double* out;
};

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

// the flag and the residual partials are read in the same round of loads
__device__ __forceinline__ bool cg_skip(const CgSkip& skip) {
    const int dn = skip.done ? *skip.done : 0;
    if (skip.rr_partials) {
        const double rr = block_sum_partials(skip.rr_partials, skip.nparts, 2, 1);
        if (rr <= skip.thr) return true;
    }
    return dn != 0;
}

// acc += P_l dl for one incidence (dl = v_i - v_other)
template <int LPR, int NPER, int Q, int MODE>
__device__ __forceinline__ void matvec_term(const Meta& m, const double (&dl)[NPER],
                                            const double (&pv)[NPER], uint32_t lb,
                                            double (&acc)[NPER]) {
    if constexpr (MODE == 1) {
#pragma unroll
        for (int t = 0; t < NPER; ++t) acc[t] += dl[t];
    } else if constexpr (MODE == 2) {
        // adjoint curvature a (I - yhat yhat^T) on every edge with a > 0
        if (m.a > 0.0) {
            double c = 0.0;
#pragma unroll
            for (int t = 0; t < NPER; ++t) c += pv[t] * dl[t];
            c = group_sum<LPR>(c) * m.f;
#pragma unroll
            for (int t = 0; t < NPER; ++t) acc[t] += m.a * dl[t] - c * pv[t];
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
            for (int t = 0; t < NPER; ++t) c += pv[t] * dl[t];
            c = group_sum<LPR>(c) * m.f;
#pragma unroll
            for (int t = 0; t < NPER; ++t) acc[t] += m.a * dl[t] - c * pv[t];
        }
    } else if constexpr (Q == kQ1) {
        // P = diag(1[|y_k| <= r])
#pragma unroll
        for (int t = 0; t < NPER; ++t)
            if ((lb >> t) & 1u) acc[t] += dl[t];
    } else {
        // P = I inside; diag(1_S) - s_S s_S^T / |S| outside
        if (m.cnt < 0) {
#pragma unroll
            for (int t = 0; t < NPER; ++t) acc[t] += dl[t];
        } else if (m.cnt > 0) {
            double sd = 0.0;
#pragma unroll
            for (int t = 0; t < NPER; ++t)
                if ((lb >> t) & 1u) sd += ((lb >> (16 + t)) & 1u) ? -dl[t] : dl[t];
            sd = group_sum<LPR>(sd) / double(m.cnt);
#pragma unroll
            for (int t = 0; t < NPER; ++t)
                if ((lb >> t) & 1u) acc[t] += dl[t] - (((lb >> (16 + t)) & 1u) ? -sd : sd);
        }
    }
}

// rows of 9 to 13 values per lane: held to three waves per SIMD
template <int NPER>
constexpr int matvec_min_waves() { return NPER > 8 && NPER <= 13 ? 3 : 1; }

template <int LPR, int NPER, int Q, int MODE>
__global__ __launch_bounds__(kBlock, matvec_min_waves<NPER>()) void k_matvec_win(DevGraph g, int d,
                                                       const double* __restrict__ V,
                                                       const double* __restrict__ Pi,
                                                       Payload pl, MatvecOut mo,
                                                       double* __restrict__ partials,
                                                       CgSkip skip) {
    if (cg_skip(skip)) return;
    constexpr int U = Unroll<NPER>::U;
    constexpr bool PAY = MODE != 1;
    constexpr int QP = MODE == 2 ? kQ2 : Q;
    constexpr int NM = meta_slots<LPR, NPER>();
    constexpr bool PF = NM <= 4;  // share data fits a few registers per lane
    constexpr int GPB = kBlock / LPR;
    // later pieces of cut vertices: [row group][value][lane]
    __shared__ double piece[GPB][NPER][LPR];
    __shared__ int head_v[GPB];  // vertex of the row group's first piece if cut, else -1
    const int gl = (threadIdx.x & 63) % LPR;
    const int rg = threadIdx.x / LPR;
    double dot = 0.0;
    for (int w = blockIdx.x; w < int(g.nwin); w += gridDim.x) {
        const GroupRange gr = group_range(g, w, rg, GPB);
        int vcur = -1;
        bool first = true;
        int head = -1;
        double vi[NPER], acc[NPER];
#pragma unroll
        for (int t = 0; t < NPER; ++t) vi[t] = acc[t] = 0.0;
        // vertex vcur has no more entries in this share
        auto done = [&](bool cut_start) {
            if (!cut_start) {
                matvec_finish<LPR, NPER>(vcur, d, gl, mo, vi, acc, dot);
            } else {
#pragma unroll
                for (int t = 0; t < NPER; ++t) piece[rg][t][gl] = acc[t];
                head = vcur;
            }
        };
        constexpr int CP = NM * LPR;  // entries per round of incidence loads
        for (int pc = gr.p0, pe = 0; pc < gr.p1; pc = pe) {
            pe = (PF && gr.p1 - pc > CP) ? pc + CP : gr.p1;
            ChunkMeta<LPR, PF ? NM : 1> cm;
            if constexpr (PF) chunk_meta_load<LPR, NM, QP, PAY>(g, pc, pe, gl, pl, cm);
            for (int p0 = pc; p0 < pe; p0 += U) {
                Meta mt[U];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (p0 + u < pe) {
                        if constexpr (PF)
                            mt[u] = chunk_meta_get<LPR, NM, QP, PAY, MODE == 2>(cm, p0 + u - pc);
                        else
                            mt[u] = load_meta<QP, PAY, MODE == 2>(g, p0 + u, pl);
                    }
                // the first vertex starting in this batch has its row gathered
                // with the batch; any further one is loaded when reached
                int un = -1;
                int64_t vnew = -1;
                double vn[NPER];
                if constexpr (Unroll<NPER>::PREFETCH) {
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if (un < 0 && p0 + u < pe &&
                            mt[u].v != (u == 0 ? vcur : int64_t(mt[u > 0 ? u - 1 : 0].v))) {
                            un = u;
                            vnew = mt[u].v;
                        }
                    }
#pragma unroll
                    for (int t = 0; t < NPER; ++t) {
                        const int k = gl + LPR * t;
                        vn[t] = (vnew >= 0 && k < d) ? V[vnew * d + k] : 0.0;
                    }
                }
                double vo[U][NPER], pv[U][NPER];
                uint32_t lb[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const bool ok = p0 + u < pe;
                    const bool rows = ok && PAY && QP == kQ2 && mt[u].f != 0.0;
#pragma unroll
                    for (int t = 0; t < NPER; ++t) {
                        const int k = gl + LPR * t;
                        vo[u][t] = (ok && k < d) ? V[int64_t(mt[u].o) * d + k] : 0.0;
                        pv[u][t] = (rows && k < d) ? Pi[int64_t(mt[u].l) * d + k] : 0.0;
                    }
                    lb[u] = 0u;
                    if constexpr (PAY && QP != kQ2)
                        if (ok) lb[u] = pl.lbits[int64_t(mt[u].l) * LPR + gl];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (p0 + u >= pe) break;
                    const Meta& m = mt[u];
                    if (m.v != vcur) {
                        if (vcur >= 0) {
                            done(first && vcur == gr.vprev);
                            first = false;
                        }
                        vcur = m.v;
                        if (u == un) {
#pragma unroll
                            for (int t = 0; t < NPER; ++t) vi[t] = vn[t];
                        } else {
                            load_row<LPR, NPER>(V, vcur, d, gl, vi);
                        }
#pragma unroll
                        for (int t = 0; t < NPER; ++t) acc[t] = 0.0;
                    }
                    double dl[NPER];
#pragma unroll
                    for (int t = 0; t < NPER; ++t) dl[t] = vi[t] - vo[u][t];
                    matvec_term<LPR, NPER, Q, MODE>(m, dl, pv[u], lb[u], acc);
                }
            }
        }
        // the last vertex: finished here, or (continuing past the share)
        // after the barrier with the later row groups' pieces
        bool pend = false;
        if (vcur >= 0) {
            const bool cs = first && vcur == gr.vprev;
            if (!cs && vcur == gr.vnext) pend = true;
            else done(cs);
        }
        if (gl == 0) head_v[rg] = head;
        __syncthreads();
        if (pend) {
            for (int j = rg + 1; j < GPB && head_v[j] == vcur; ++j) {
#pragma unroll
                for (int t = 0; t < NPER; ++t) acc[t] += piece[j][t][gl];
            }
            matvec_finish<LPR, NPER>(vcur, d, gl, mo, vi, acc, dot);
        }
        __syncthreads();
    }
    // isolated vertices
    for (int64_t i = int64_t(blockIdx.x) * GPB + rg; i < g.niso; i += int64_t(gridDim.x) * GPB) {
        const int64_t v = g.iso[i];
        double vi[NPER], acc[NPER];
#pragma unroll
        for (int t = 0; t < NPER; ++t) acc[t] = 0.0;
        load_row<LPR, NPER>(V, v, d, gl, vi);
        matvec_finish<LPR, NPER>(v, d, gl, mo, vi, acc, dot);
    }
    double dt[1] = {dot};
    block_reduce_store<kMatvecNV>(dt, partials + blockIdx.x * kMatvecNV);
}

}  // namespace

// one workgroup per window, enough to give every isolated vertex a row
// group.  Workgroups are dispatched in window order, so the windows in flight
// at any time are neighbours in the graph's processing order.
template <int LPR>
static int window_grid(const DevGraph& g) {
    const int64_t gpb = kBlock / LPR;
    const int64_t b = std::max<int64_t>(g.nwin, (g.niso + gpb - 1) / gpb);
    return int(std::max<int64_t>(b, 1));
}

int launch_scatter(const DevGraph& g, int d, int qk, double cx, const double* X, double ca,
                   const double* A, double cz, const double* Z, double* out, bool diag, Payload pl,
                   double gamma, double sigma, double* Dinv, double* partials, hipStream_t s,
                   double* rowstats) {
    (void)gamma;  // the Jacobian payload already holds 1 / (gamma w)
    int total = 0;
    ScatterOut so{cx, ca, cz, sigma, X, A, out, Dinv, rowstats};
    dispatch_row(d, [&](auto L, auto N) {
        constexpr int lpr = decltype(L)::value, nper = decltype(N)::value;
        const int g1 = window_grid<lpr>(g);
        if (!diag) {
            hipLaunchKernelGGL((k_scatter_win<lpr, nper, kQ2, false>), dim3(g1), dim3(kBlock), 0,
                               s, g, d, so, Z, pl, partials);
        } else {
            dispatch_q(qk, [&](auto Qc) {
                constexpr int q = decltype(Qc)::value;
                hipLaunchKernelGGL((k_scatter_win<lpr, nper, q, true>), dim3(g1), dim3(kBlock), 0,
                                   s, g, d, so, Z, pl, partials);
            });
        }
        total = g1;
    });
    return total;
}

int launch_edge_grad(const DevGraph& g, int d, int qk, double gamma, double sigma,
                     const double* X, const double* U, const double* A, double* Pi, Payload pl,
                     double* G, double* Dinv, double* epart, double* spart, hipStream_t s,
                     double* kpart) {
    int total = 0;
    ScatterOut so{1.0, -1.0, 1.0, sigma, X, A, G, Dinv, nullptr};
    dispatch_row(d, [&](auto L, auto N) {
        constexpr int lpr = decltype(L)::value, nper = decltype(N)::value;
        const int g1 = window_grid<lpr>(g);
        auto go = [&](auto Qc, auto Kc) {
            constexpr int q = decltype(Qc)::value;
            constexpr bool kkt = decltype(Kc)::value != 0;
            hipLaunchKernelGGL((k_edge_grad_win<lpr, nper, q, kkt>), dim3(g1), dim3(kBlock), 0, s,
                               g, d, so, gamma, U, Pi, pl, epart, spart, kpart);
        };
        if (qk == kQ1) {
            if (kpart) go(IC<kQ1>{}, IC<1>{});
            else go(IC<kQ1>{}, IC<0>{});
        } else if (qk == kQ2) {
            if (kpart) go(IC<kQ2>{}, IC<1>{});
            else go(IC<kQ2>{}, IC<0>{});
        } else {
            // q = inf: whole-wave rows only (at shorter rows the two
            // edge-parallel kernels were faster than projecting at both
            // endpoints), and without the KKT terms
            if constexpr (lpr == 64) {
                if (!kpart) {
                    go(IC<kQInf>{}, IC<0>{});
                    total = g1;
                    return;
                }
            }
            total = -1;
            return;
        }
        total = g1;
    });
    return total;
}

int launch_matvec(const DevGraph& g, int d, int qk, int mode, const double* V, const double* Pi,
                  Payload pl, double gamma, double sigma, double c0, const double* dscale,
                  double* out, double* partials, CgSkip skip, hipStream_t s) {
    (void)gamma;  // the Jacobian payload already holds 1 / (gamma w)
    int total = 0;
    MatvecOut mo{sigma, c0, dscale, out};
    dispatch_row(d, [&](auto L, auto N) {
        constexpr int lpr = decltype(L)::value, nper = decltype(N)::value;
        const int g1 = window_grid<lpr>(g);
        if (mode == 1) {
            hipLaunchKernelGGL((k_matvec_win<lpr, nper, kQ2, 1>), dim3(g1), dim3(kBlock), 0, s, g,
                               d, V, Pi, pl, mo, partials, skip);
        } else if (mode == 2) {
            hipLaunchKernelGGL((k_matvec_win<lpr, nper, kQ2, 2>), dim3(g1), dim3(kBlock), 0, s, g,
                               d, V, Pi, pl, mo, partials, skip);
        } else {
            dispatch_q(qk, [&](auto Qc) {
                constexpr int q = decltype(Qc)::value;
                hipLaunchKernelGGL((k_matvec_win<lpr, nper, q, 0>), dim3(g1), dim3(kBlock), 0, s,
                                   g, d, V, Pi, pl, mo, partials, skip);
            });
        }
        total = g1;
    });
    return total;
}

}  // namespace ccm
