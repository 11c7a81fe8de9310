// Host-side launch interface between the solver drivers and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "common.hpp"
#include "tuned_windows.hpp"

namespace ccm {

template <int V>
using IC = std::integral_constant<int, V>;

// Row layout: LPR lanes of a wave handle one row of d values, NPER values
// per lane (coordinate k = lane_in_group + LPR * t).  Up to 256 values a lane
// holds at most 4, so a wave works on several rows at once and the per-row
// reductions stay short; longer rows use the whole wave, with no more values
// per lane than the row needs in steps that keep registers (and so waves in
// flight) for the common widths.
inline bool row_supported(int64_t d) { return d >= 1 && d <= 1024; }

template <class F>
inline void dispatch_row(int d, F&& f) {
    if (d <= 2) f(IC<1>{}, IC<2>{});
    else if (d <= 4) f(IC<1>{}, IC<4>{});
    else if (d <= 8) f(IC<2>{}, IC<4>{});
    else if (d <= 16) f(IC<4>{}, IC<4>{});
    else if (d <= 32) f(IC<8>{}, IC<4>{});
    else if (d <= 64) f(IC<16>{}, IC<4>{});
    else if (d <= 128) f(IC<32>{}, IC<4>{});
    else if (d <= 256) f(IC<64>{}, IC<4>{});
    else if (d <= 512) f(IC<64>{}, IC<8>{});
    else if (d <= 768) f(IC<64>{}, IC<12>{});
    else if (d <= 832) f(IC<64>{}, IC<13>{});
    else f(IC<64>{}, IC<16>{});
}

template <class F>
inline void dispatch_q(int qk, F&& f) {
    if (qk == kQ1) f(IC<kQ1>{});
    else if (qk == kQ2) f(IC<kQ2>{});
    else f(IC<kQInf>{});
}

inline int lanes_per_row(int d) {
    int l = 1;
    dispatch_row(d, [&](auto L, auto) { l = decltype(L)::value; });
    return l;
}

// grid for a grid-stride loop over `rows` rows of LPR lanes
inline int row_grid(int64_t rows, int lpr) {
    const int64_t gpb = kBlock / lpr;
    int64_t g = (rows + gpb - 1) / gpb;
    if (g < 1) g = 1;
    if (g > kMaxGrid) g = kMaxGrid;
    return int(g);
}

// grid of the element-wise kernels; kept small because the CG update
// re-reduces the partial sums of the previous kernels in every block
inline int flat_grid(int64_t count) {
    int64_t g = (count + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > 1024) g = 1024;
    return int(g);
}

// 32-bit mask words per edge of the q = 1 / q = inf Jacobian payload: one per
// lane of a row group.
inline int lbits_per_edge(int d) { return lanes_per_row(d); }

// Per-edge generalized-Jacobian payload written by the SSNAL edge pass.  The
// scalar part is stored once per incidence entry (both incidences of an edge
// hold the same value), so a vertex kernel reads it at the entry's position
// together with the entry itself instead of through the edge index.
struct Payload {
    double2* ipay = nullptr;   // per incidence: q = 2 {a, 1/r} with a = r/||y||
                               // outside the ball, 1 inside; q = inf {cnt, 0},
                               // cnt = -1 inside the ball, else support size
    uint32_t* lbits = nullptr; // per edge and lane (m x LPR): bit t = mask of
                               // coordinate gl + LPR t (q = 1: |y_k| <= r;
                               // q = inf: k in support), bit 16 + t: y_k < 0
};

struct DevGraph {
    int64_t n = 0, m = 0;
    const int* src = nullptr;
    const int* dst = nullptr;
    const double* w = nullptr;
    // The incidence lists are stored in a processing order of the vertices:
    // vertex vord[r] has rank r and its entries are inc[inc_ptr[r] ..
    // inc_ptr[r + 1]); vrank is the inverse map.  Null vord / vrank mean the
    // identity order (rank = vertex).
    const int* inc_ptr = nullptr;  // n + 1, by rank
    const Inc* inc = nullptr;      // 2 m
    const int* irow = nullptr;     // vertex of each incidence entry (2 m)
    const int* vord = nullptr;     // n: vertex of each rank (null: identity)
    const int* vrank = nullptr;    // n: rank of each vertex (null: identity)
    const int* epos = nullptr;     // incidence positions of edge l: [2 l] at src, [2 l + 1] at dst
    int max_deg = 0;
    // Work split of the incidence array for the vertex kernels: window w holds
    // the entries win[w] = {begin, end} of consecutive whole vertices, at most
    // window_for(d) of them unless the window is a single hub vertex.  One
    // workgroup takes a window; its row groups split the window's entries
    // evenly, and a vertex cut between row groups is summed through LDS, in
    // row-group order, by the group where it starts.  With a locality order
    // (vord set) windows follow it, except that hub windows (longer than
    // window_for(d)) come first; in the input order they are stored longest
    // first.  Isolated vertices have no entries and are listed in `iso`.
    int64_t nent = 0;            // incidence entries (2 m for an edge graph)
    const int2* win = nullptr;   // nwin non-empty windows
    int64_t nwin = 0;
    const int* iso = nullptr;    // vertices without incidences
    int64_t niso = 0;
};

// Doubles of a partials buffer that a kernel over graph g may fill: the
// vertex kernels run one workgroup per window (or per row group of isolated
// vertices), up to 8 values each; the other kernels stay within kPartialsCap.
inline size_t partials_for(const DevGraph& g) {
    const int64_t b = (g.nwin > g.niso ? g.nwin : g.niso) + 1;
    const size_t need = size_t(b) * 8 * 2;
    return need > size_t(kPartialsCap) ? need : size_t(kPartialsCap);
}

// index of d's row layout in dispatch_row's order
inline int layout_index(int d) {
    static constexpr int kMaxD[] = {2, 4, 8, 16, 32, 64, 128, 256, 512, 768, 832, 1024};
    int i = 0;
    while (i + 1 < kTunedLayouts && d > kMaxD[i]) ++i;
    return i;
}

// incidences per row group of a window (about one typical vertex for long
// rows, several short vertices for short rows): `chunk` if positive, else the
// tuned value for d's row layout and q (qk = kQ1, kQ2 or kQInf)
inline int chunk_for(int d, int qk = kQ2, int chunk = 0) {
    if (chunk > 0) return chunk;
    const int qi = qk == kQ1 ? 0 : qk == kQInf ? 2 : 1;
    return kTunedChunk[layout_index(d)][qi];
}

// target entries per window: one chunk for each row group of a workgroup
inline int64_t window_for(int d, int qk = kQ2, int chunk = 0) {
    return int64_t(kBlock / lanes_per_row(d)) * chunk_for(d, qk, chunk);
}

// ---- edge kernels (edge_kernels.hip) --------------------------------------
// SSNAL edge pass: Y = U + sigma B X, Pi = Pi_C(Y), payload; partials per
// block (5): <BX, Pi>, ||Pi - U||^2, ||BX||^2, ||Pi||^2, and the number of
// edges whose Jacobian is not the identity (outside the ball).
constexpr int kEdgeSsnalNV = 5;
int launch_edge_ssnal(const DevGraph& g, int d, int qk, double gamma, double sigma,
                      const double* X, const double* U, double* Pi, Payload pl,
                      double* partials, hipStream_t s);

// KKT edge pass for (X, U): partials (6): ||Pi_C(BX+U) - U||^2, ||BX||^2,
// ||U||^2, ||U - Pi_C(U)||^2, sum_l r_l ||(BX)_l||_q, 0.  Optionally writes
// Pi_C(U) to Ufeas, and the first five terms per edge to rowstats (m x 5).
constexpr int kEdgeKktNV = 6;
int launch_edge_kkt(const DevGraph& g, int d, int qk, double gamma, const double* X,
                    const double* U, double* Ufeas, double* partials, hipStream_t s,
                    double* rowstats = nullptr);

// ADMM edge step: Pi = Pi_C(sigma BX + L), Z <- BX + (L - Pi)/sigma,
// L <- L + tau sigma (BX - Z), Q <- sigma Z - L, optional Uf <- Pi_C(L).
// partials (4): ||BX - Z||^2, ||Z - Zold||^2, ||BX||^2, ||Z||^2.
constexpr int kEdgeAdmmNV = 4;
int launch_edge_admm(const DevGraph& g, int d, int qk, double gamma, double sigma, double tau,
                     const double* X, double* Z, double* L, double* Q, double* Uf,
                     double* partials, hipStream_t s);

// Halpern-Peaceman-Rachford edge step on the state (Z, L) with anchor
// (Za, La) and Halpern weight a: H = 2 BX - Z, Lh = Pi_C(sigma H + L),
// Zh = H + (L - Lh) / sigma; Z <- a Za + (1 - a) Zh, L <- a La + (1 - a) Lh,
// Q <- sigma Z - L, optional Uh <- Lh.  partials (4): ||Z - Zh||^2,
// ||L - Lh||^2 (Z, L before the step), ||Z - Za||^2, ||L - La||^2 (after).
constexpr int kEdgeHprNV = 4;
int launch_edge_hpr(const DevGraph& g, int d, int qk, double gamma, double sigma, double a,
                    const double* X, double* Z, double* L, const double* Za, const double* La,
                    double* Q, double* Uh, double* partials, hipStream_t s);

// Fast AMA edge step on the dual: Unew = Pi_C(V + nu B X); then with momentum
// coefficient beta: Vnew = Unew + beta (Unew - U); U <- Unew.  partials (2):
// <V - Unew, Unew - U> (restart test), ||Unew - U||^2.
constexpr int kEdgeAmaNV = 2;
int launch_edge_ama(const DevGraph& g, int d, int qk, double gamma, double nu, double beta,
                    const double* X, double* U, double* V, double* partials, hipStream_t s);

void launch_gather(const DevGraph& g, int d, const double* X, double* Y, hipStream_t s);
void launch_project(int64_t m, int d, int qk, const double* Y, const double* w, double gamma,
                    bool prox, double* out, hipStream_t s);
// U rows (q = 1: coordinates) on the boundary of their ball of radius g0 w_l
// are multiplied by rho
void launch_scale_boundary(int64_t m, int d, int qk, const double* w, double g0, double rho,
                           double* U, hipStream_t s);
// fused[l] = ||x_src - x_dst||_2 <= thr; with `spread` (a device scalar S)
// the threshold is 1e-5 (1 + S) instead of thr; with `vthr` (per vertex) it is
// vthr[src_l]
void launch_fused_flags(const DevGraph& g, int d, const double* X, double thr, int* fused,
                        hipStream_t s, const double* spread = nullptr,
                        const double* vthr = nullptr);

// ---- vertex kernels (vertex_kernels.hip) ----------------------------------
// out = cx X + ca A + cz B^T Z (X or A may be null).  With `diag` (SSNAL),
// also Dinv = 1 / (1 + sigma diag(B^T P B)) from the payload.  partials (4):
// ||out||^2, 1/2 ||X - A||^2, <A, B^T Z>, ||B^T Z||^2.
constexpr int kScatterNV = 4;
// With rowstats (n x 4) the same four terms are also stored per vertex row.
int launch_scatter(const DevGraph& g, int d, int qk, double cx, const double* X, double ca,
                   const double* A, double cz, const double* Z, double* out, bool diag,
                   Payload pl, double gamma, double sigma, double* Dinv, double* partials,
                   hipStream_t s, double* rowstats = nullptr);

// Newton matvec: out = c0 V + sigma sum_{l ~ i} P_l (v_i - v_other) with the
// SSNAL payload (mode 0), P_l = I (mode 1, the ADMM matrix I + sigma B^T B),
// or P_l = a_l (I - yhat yhat^T) on every edge with a_l > 0 and 0 elsewhere
// (mode 2, the adjoint curvature; q = 2 payload layout, no identity branch).
// Optional per-vertex diagonal scale `dscale` (n values) replaces c0.
// partials (1): <V, out>.  If rr_partials is non-null the kernel returns at
// once when the CG residual recorded there is below thr or *done is set.
struct CgSkip {
    const double* rr_partials = nullptr;
    int nparts = 0;
    double thr = 0.0;
    const int* done = nullptr;
};
constexpr int kMatvecNV = 1;
// SSNAL edge pass fused with the gradient (one launch, vertex-centric; q = 1
// and 2, and q = inf without kpart on rows of 64 lanes; otherwise nothing is
// launched and -1 is returned): Pi =
// Pi_C(U + sigma B X) and its Jacobian payload as launch_edge_ssnal, G = X -
// A + B^T Pi and Dinv as launch_scatter(diag); edge partials (kEdgeSsnalNV)
// to epart and vertex partials (kScatterNV) to spart, one row per block;
// with kpart, also the KKT edge terms at (X, U) as launch_edge_kkt (kEdgeKktNV
// per block).  Returns the number of blocks.
int launch_edge_grad(const DevGraph& g, int d, int qk, double gamma, double sigma,
                     const double* X, const double* U, const double* A, double* Pi, Payload pl,
                     double* G, double* Dinv, double* epart, double* spart, hipStream_t s,
                     double* kpart = nullptr);
int launch_matvec(const DevGraph& g, int d, int qk, int mode, const double* V, const double* Pi,
                  Payload pl, double gamma, double sigma, double c0, const double* dscale,
                  double* out, double* partials, CgSkip skip, hipStream_t s);

// ---- vector kernels (vector_kernels.hip) ----------------------------------
struct CgBufs {
    double *x, *r, *u, *w, *p, *s;  // n*d each
    double* upd[2];                 // update partials (r.u, r.r) per block, parity buffered
    double* wu[2];                  // matvec partials (w.u) per block, parity buffered
    double* state;                  // [2][2]: gamma_j, alpha_j per parity
    int* flag;                      // [0] done (1) / breakdown (2), [1] iterations
    int nparts;                     // partial count of the update kernel
    int nparts_mv;                  // partial count of the matvec kernel
};
// r = b (or -b when neg), u = Dinv r, x = 0 (iteration 0 writes p and s without reading
// them); partials ru[0], rr[0].
void launch_cg_init(int64_t N, const double* b, bool neg, const double* Dinv, CgBufs& cg,
                    hipStream_t s);
// iteration j of the Chronopoulos-Gear PCG update (see vector_kernels.hip).
void launch_cg_update(int64_t N, int j, const double* Dinv, CgBufs& cg, double thr, hipStream_t s);
int cg_update_grid(int64_t N);

// Xt = X + alpha D; partials (2): 1/2 ||Xt - A||^2, <G, D>.
constexpr int kAxpyNV = 2;
int launch_trial(int64_t N, const double* X, const double* D, double alpha, const double* A,
                 const double* G, double* Xt, double* partials, hipStream_t s);
// sum partials[p * nv + c] over p for every c < nv (1 <= nv <= 7); out[c] = total.
void launch_finalize(const double* partials, int nparts, int nv, double* out, hipStream_t s);
// several such sums in one launch (one workgroup each, same arithmetic)
struct FinalizeJob {
    const double* partials;
    int nparts, nv;
    double* out;
};
constexpr int kMaxFinalizeJobs = 8;
struct FinalizeJobs {
    FinalizeJob j[kMaxFinalizeJobs];
};
void launch_finalize_multi(const FinalizeJobs& jobs, int njobs, hipStream_t s);
void launch_fill(double* x, int64_t N, double v, hipStream_t s);
// y = exp(x), elementwise
void launch_exp(const double* x, int64_t n, double* y, hipStream_t s);
// flag[0] = 1 if some x[k] (k < count) is NaN or infinite; flag[0] is not cleared
void launch_flag_nonfinite(const double* x, int64_t count, int* flag, hipStream_t s);
// x += alpha y
void launch_axpy(double* x, double alpha, const double* y, int64_t N, hipStream_t s);
// out = a x + b y
void launch_axpby(double a, const double* x, double b, const double* y, double* out, int64_t N,
                  hipStream_t s);
// partials (1): <x, y>
int launch_dot(const double* x, const double* y, int64_t N, double* partials, hipStream_t s);
void launch_copy(const double* a, double* b, int64_t N, hipStream_t s);
// out = a - b (elementwise)
void launch_sub(const double* a, const double* b, double* out, int64_t N, hipStream_t s);
// Dinv[i, :] = 1 / (c0 + sigma deg_i)
void launch_lap_dinv(const DevGraph& g, int d, double c0, double sigma, double* Dinv,
                     hipStream_t s);
// column sums partials of A (n x d): partials[p * d + k]; then spread
// S = max_i ||a_i - mean||; result written to out[0].
void launch_spread(const double* A, int64_t n, int d, double* work, double* out, hipStream_t s);
int spread_work_size(int64_t n, int d);
// per vertex: the fusion threshold 1e-5 (1 + S_s) of its segment s, with
// S_s the spread of the segment's rows of A computed exactly as
// launch_spread computes it for those rows alone.  work: doubles of
// seg_threshold_work_size(nseg, d).
void launch_seg_thresholds(const double* A, const int64_t* seg, int nseg, int d, double* work,
                           double* vthr, hipStream_t s);
int seg_threshold_work_size(int nseg, int d);
void launch_stream_copy(const void* src, void* dst, int64_t bytes, hipStream_t s);
// batched solves: copy union rows (and labels, offset to start at 0 per
// instance) into per-instance output blocks: instance s owns rows
// [vseg[s], vseg[s+1]); its gamma-t block starts at xoff[s] + t n_s d
// (labels: loff[s] + t n_s)
void launch_split(int64_t nU, int d, const double* X, const int* lab, const int64_t* vseg, int S,
                  const int64_t* xoff, const int64_t* loff, int t, double* Xout, int* Lout,
                  hipStream_t s);
// out[i] = ||x_i||^2 for the n rows of X
void launch_row_sqnorm(const double* X, int64_t n, int d, double* out, hipStream_t s);
void launch_first_labels(const int* lab, const int64_t* vseg, int S, int* out, hipStream_t s);
// so = src + voff, dso = dst + voff, wo = w; *bad |= 1 unless 0 <= src < dst < nloc
void launch_offset_edges(int64_t m, const int* src, const int* dst, const double* w, int voff,
                         int nloc, int* so, int* dso, double* wo, int* bad, hipStream_t s);
// out[s * nv + c] = sum over rows r in [seg[s], seg[s + 1]) of rows[r * nv + c],
// in row order (one block per segment)
void launch_segsum(const double* rows, int nv, const int64_t* seg, int nseg, double* out,
                   hipStream_t s);

// ---- adjoint (adjoint.hip) ----------------------------------------------------
// Per edge: delta = x_i - x_j; for an edge joining two clusters
// alpha = gamma w / ||delta|| and Pi = gamma w delta / ||delta||, else alpha = 0;
// ipay (per incidence, q = 2 payload layout) = {alpha, 1 / (gamma w)}.
void launch_adj_payload(const DevGraph& g, int d, const double* X, const int* labels,
                        double gamma, double2* ipay, double* Pi, hipStream_t s);
// v[i, :] = lam[labels[i], :]
void launch_expand(int64_t n, int d, const int* labels, const double* lam, double* v,
                   hipStream_t s);
// dlogw_l = -gamma w_l <lam_ci - lam_cj, ghat_l> on inter-cluster edges (0
// inside a cluster); partials (1): sum_l w_l <lam_ci - lam_cj, ghat_l>.
int launch_adj_edge(const DevGraph& g, int d, const double* X, const int* labels,
                    const double* lam, double gamma, double* dlogw, double* partials,
                    hipStream_t s);
// out[c] = 1 / (ptr[c + 1] - ptr[c])
void launch_inv_sizes(int64_t K, const int* ptr, double* out, hipStream_t s);
// range[0] = min label, range[1] = max label (range preset to INT_MAX, -1)
void launch_label_range(int64_t n, const int* labels, int* range, hipStream_t s);
// per-row scale: out[i, :] = x[i, :] * rs[i]
void launch_rowscale(const double* x, const double* rs, double* out, int64_t rows, int d,
                     hipStream_t s);

// ---- labels (labels.hip) --------------------------------------------------
// labels from fused flags: connected components, numbered by smallest vertex.
// work: int[n] parent + int[n + 1] scan + hipcub temp.  n_clusters (device int).
size_t labels_temp_bytes(int64_t n);
void launch_labels(int64_t n, int64_t m, const int* src, const int* dst, const int* fused,
                   int* parent, int* rank, void* temp, size_t temp_bytes, int* labels,
                   int* n_clusters, hipStream_t s,
                   const int* inc_ptr = nullptr, const Inc* inc = nullptr,
                   const int* vord = nullptr);

}  // namespace ccm
