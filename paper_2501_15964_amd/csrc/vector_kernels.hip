// Element-wise and reduction kernels on n x d vertex arrays: the conjugate
// gradient vector updates, line-search trial points, partial-sum
// finalisation and small utilities.
#include "launch.hpp"

namespace ccm {
namespace {

__global__ __launch_bounds__(kBlock) void k_cg_init(int64_t N, const double* __restrict__ b,
                                                    double sgn, const double* __restrict__ Dinv,
                                                    double* __restrict__ x, double* __restrict__ r,
                                                    double* __restrict__ u, double* __restrict__ p,
                                                    double* __restrict__ s,
                                                    double* __restrict__ upd0, int* flag) {
    double acc[2] = {0.0, 0.0};
    for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < N;
         k += int64_t(gridDim.x) * kBlock) {
        const double rv = sgn * b[k];
        const double uv = Dinv[k] * rv;
        r[k] = rv;
        u[k] = uv;
        x[k] = 0.0;  // p and s are first written by iteration 0, which reads neither
        acc[0] += rv * uv;
        acc[1] += rv * rv;
    }
    block_reduce_store<2>(acc, upd0 + blockIdx.x * 2);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        flag[0] = 0;
        flag[1] = 0;
    }
}

// Iteration j of preconditioned CG in the Chronopoulos-Gear arrangement, which
// needs one global reduction point per iteration: the dot products r.u (from
// this kernel) and w.u (from the matvec w = A u that follows it) are both
// consumed by the next update.  With gamma_j = r_j.u_j, delta_j = w_j.u_j:
//   beta_j  = gamma_j / gamma_{j-1},  alpha_j = gamma_j / (delta_j - beta_j gamma_j / alpha_{j-1})
//   p = u + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s,  u = M^{-1} r
// (j = 0: beta = 0, alpha = gamma_0 / delta_0).  Every block re-reduces the
// partials in the same order, so all blocks agree bit for bit on alpha and
// beta; scalars and partials alternate between two slots by parity of j.
__global__ __launch_bounds__(kBlock) void k_cg_update(
    int64_t N, int j, const double* __restrict__ Dinv, double* __restrict__ x,
    double* __restrict__ r, double* __restrict__ u, const double* __restrict__ w,
    double* __restrict__ p, double* __restrict__ s, const double* __restrict__ upd_prev,
    double* __restrict__ upd_next, const double* __restrict__ wu, int nparts_upd, int nparts_mv,
    double* __restrict__ state, int* flag, double thr) {
    if (flag[0]) return;
    const int par = j & 1;
    // r.r (stop test), gamma = r.u, delta = w.u in one pass
    const double* ptr[3] = {upd_prev + 1, upd_prev, wu};
    const int cnt[3] = {nparts_upd, nparts_upd, nparts_mv};
    const int st[3] = {2, 2, 1};
    double sums[3];
    block_sums<3>(ptr, cnt, st, sums);
    const double rr = sums[0], gam = sums[1], del = sums[2];
    if (rr <= thr) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            flag[0] = 1;
            flag[1] = j;
        }
        return;
    }
    double alpha, beta;
    if (j == 0) {
        beta = 0.0;
        alpha = gam / del;
    } else {
        const double gp = state[par * 2 + 0];
        const double ap = state[par * 2 + 1];
        beta = gam / gp;
        alpha = gam / (del - beta * gam / ap);
    }
    if (!(alpha > 0.0) || !isfinite(alpha) || !isfinite(beta)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            flag[0] = 2;
            flag[1] = j;
        }
        return;
    }
    double acc[2] = {0.0, 0.0};
    if (j == 0) {
        // p = u, s = w, x = alpha p (x, p, s are zero before iteration 0,
        // so this is the general update with the zero terms left out)
        for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < N;
             k += int64_t(gridDim.x) * kBlock) {
            const double pk = u[k];
            const double sk = w[k];
            x[k] = alpha * pk;
            const double rk = r[k] - alpha * sk;
            const double uk = Dinv[k] * rk;
            p[k] = pk;
            s[k] = sk;
            r[k] = rk;
            u[k] = uk;
            acc[0] += rk * uk;
            acc[1] += rk * rk;
        }
    } else {
        for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < N;
             k += int64_t(gridDim.x) * kBlock) {
            const double pk = u[k] + beta * p[k];
            const double sk = w[k] + beta * s[k];
            x[k] += alpha * pk;
            const double rk = r[k] - alpha * sk;
            const double uk = Dinv[k] * rk;
            p[k] = pk;
            s[k] = sk;
            r[k] = rk;
            u[k] = uk;
            acc[0] += rk * uk;
            acc[1] += rk * rk;
        }
    }
    block_reduce_store<2>(acc, upd_next + blockIdx.x * 2);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        state[(par ^ 1) * 2 + 0] = gam;
        state[(par ^ 1) * 2 + 1] = alpha;
        flag[1] = j + 1;
    }
}

__global__ __launch_bounds__(kBlock) void k_trial(int64_t N, const double* __restrict__ X,
                                                  const double* __restrict__ D, double alpha,
                                                  const double* __restrict__ A,
                                                  const double* __restrict__ G,
                                                  double* __restrict__ Xt,
                                                  double* __restrict__ partials) {
    double acc[kAxpyNV] = {0.0, 0.0};
    for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < N;
         k += int64_t(gridDim.x) * kBlock) {
        const double dk = D[k];
        const double xt = X[k] + alpha * dk;
        Xt[k] = xt;
        const double e = xt - A[k];
        acc[0] += 0.5 * e * e;
        acc[1] += G[k] * dk;
    }
    block_reduce_store<kAxpyNV>(acc, partials + blockIdx.x * kAxpyNV);
}

// one wide block: the partials of up to a few thousand blocks are read in
// four loads per thread
constexpr int kFinalizeWaves = 16;

template <int NV>
__device__ __forceinline__ void finalize_one(const double* __restrict__ partials, int nparts,
                                             double* __restrict__ out) {
    const double* ptr[NV];
    int cnt[NV], st[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        ptr[c] = partials + c;
        cnt[c] = nparts;
        st[c] = NV;
    }
    double t[NV];
    block_sums<NV, kFinalizeWaves>(ptr, cnt, st, t);
    if (threadIdx.x < NV) {
#pragma unroll
        for (int c = 0; c < NV; ++c)
            if (threadIdx.x == c) out[c] = t[c];
    }
}

template <int NV>
__global__ __launch_bounds__(kFinalizeWaves * 64) void k_finalize(const double* __restrict__ partials,
                                                                  int nparts, double* __restrict__ out) {
    finalize_one<NV>(partials, nparts, out);
}

// one block per job, each reduced exactly as k_finalize reduces it
__global__ __launch_bounds__(kFinalizeWaves * 64) void k_finalize_multi(FinalizeJobs jobs) {
    const FinalizeJob jb = jobs.j[blockIdx.x];
    switch (jb.nv) {
        case 1: finalize_one<1>(jb.partials, jb.nparts, jb.out); break;
        case 2: finalize_one<2>(jb.partials, jb.nparts, jb.out); break;
        case 3: finalize_one<3>(jb.partials, jb.nparts, jb.out); break;
        case 4: finalize_one<4>(jb.partials, jb.nparts, jb.out); break;
        case 5: finalize_one<5>(jb.partials, jb.nparts, jb.out); break;
        case 6: finalize_one<6>(jb.partials, jb.nparts, jb.out); break;
        default: finalize_one<7>(jb.partials, jb.nparts, jb.out); break;
    }
}

// flag[0] = 1 if any of the count values is NaN or infinite (every writer
// stores the same value)
__global__ __launch_bounds__(kBlock) void k_flag_nonfinite(const double* __restrict__ x,
                                                           int64_t count, int* __restrict__ flag) {
    bool bad = false;
    for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < count;
         k += int64_t(gridDim.x) * kBlock)
        bad |= !isfinite(x[k]);
    if (bad) flag[0] = 1;
}

__global__ __launch_bounds__(kBlock) void k_fill(double* __restrict__ x, int64_t N, double v) {
    for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < N;
         k += int64_t(gridDim.x) * kBlock)
        x[k] = v;
}

__global__ __launch_bounds__(kBlock) void k_axpy(double* __restrict__ x, double alpha,
                                                 const double* __restrict__ y, int64_t N) {
    for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < N;
         k += int64_t(gridDim.x) * kBlock)
        x[k] += alpha * y[k];
}

__global__ __launch_bounds__(kBlock) void k_axpby(double a, const double* __restrict__ x, double b,
                                                  const double* __restrict__ y,
                                                  double* __restrict__ o, int64_t N) {
    for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < N;
         k += int64_t(gridDim.x) * kBlock)
        o[k] = a * x[k] + b * y[k];
}

__global__ __launch_bounds__(kBlock) void k_dot(const double* __restrict__ x,
                                                const double* __restrict__ y, int64_t N,
                                                double* __restrict__ partials) {
    double acc[1] = {0.0};
    for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < N;
         k += int64_t(gridDim.x) * kBlock)
        acc[0] += x[k] * y[k];
    block_reduce_store<1>(acc, partials + blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_copy(const double* __restrict__ a,
                                                 double* __restrict__ b, int64_t N) {
    for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < N;
         k += int64_t(gridDim.x) * kBlock)
        b[k] = a[k];
}

__global__ __launch_bounds__(kBlock) void k_sub(const double* __restrict__ a,
                                                const double* __restrict__ b,
                                                double* __restrict__ o, int64_t N) {
    for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < N;
         k += int64_t(gridDim.x) * kBlock)
        o[k] = a[k] - b[k];
}

__global__ __launch_bounds__(kBlock) void k_lap_dinv(int64_t n, int d,
                                                     const int* __restrict__ inc_ptr,
                                                     const int* __restrict__ vrank, double c0,
                                                     double sigma, double* __restrict__ Dinv) {
    const int64_t N = n * d;
    for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < N;
         k += int64_t(gridDim.x) * kBlock) {
        const int64_t i = k / d;
        const int64_t r = vrank ? vrank[i] : i;
        Dinv[k] = 1.0 / (c0 + sigma * double(inc_ptr[r + 1] - inc_ptr[r]));
    }
}

// column sums of A over a contiguous range of rows per block
__global__ __launch_bounds__(kBlock) void k_colsum(const double* __restrict__ A, int64_t n, int d,
                                                   double* __restrict__ part) {
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = int64_t(blockIdx.x) * per;
    const int64_t r1 = r0 + per < n ? r0 + per : n;
    for (int k = threadIdx.x; k < d; k += blockDim.x) {
        double t = 0.0;
        for (int64_t i = r0; i < r1; ++i) t += A[i * d + k];
        part[int64_t(blockIdx.x) * d + k] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_colmean(const double* __restrict__ part, int nparts,
                                                    int64_t n, int d, double* __restrict__ mean) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < d; k += gridDim.x * blockDim.x) {
        double t = 0.0;
        for (int p = 0; p < nparts; ++p) t += part[int64_t(p) * d + k];
        mean[k] = t / double(n);
    }
}

// per-block max over rows of ||a_i - mean||^2 (max is order independent)
__global__ __launch_bounds__(kBlock) void k_rowdev_max(const double* __restrict__ A, int64_t n,
                                                       int d, const double* __restrict__ mean,
                                                       double* __restrict__ bmax) {
    double best = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * kBlock) {
        double t = 0.0;
        for (int k = 0; k < d; ++k) {
            const double e = A[i * d + k] - mean[k];
            t += e * e;
        }
        best = fmax(best, t);
    }
    __shared__ double red[kBlock];
    red[threadIdx.x] = best;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) bmax[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kBlock) void k_max_sqrt(const double* __restrict__ bmax, int nb,
                                                     double* __restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double t = 0.0;
        for (int b = 0; b < nb; ++b) t = fmax(t, bmax[b]);
        out[0] = sqrt(t);
    }
}

// The same three steps per segment of rows [seg[s], seg[s + 1]) (blockIdx.y
// = s), with the same row chunks and summation order as for a matrix of the
// segment's rows alone, so each segment's S is bit-identical to its own.
__global__ __launch_bounds__(kBlock) void k_colsum_seg(const double* __restrict__ A,
                                                       const int64_t* __restrict__ seg, int d,
                                                       double* __restrict__ part) {
    const int64_t a = seg[blockIdx.y], n = seg[blockIdx.y + 1] - a;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = int64_t(blockIdx.x) * per;
    const int64_t r1 = r0 + per < n ? r0 + per : n;
    double* out = part + (int64_t(blockIdx.y) * gridDim.x + blockIdx.x) * d;
    for (int k = threadIdx.x; k < d; k += blockDim.x) {
        double t = 0.0;
        for (int64_t i = r0; i < r1; ++i) t += A[(a + i) * d + k];
        out[k] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_colmean_seg(const double* __restrict__ part,
                                                        int nparts,
                                                        const int64_t* __restrict__ seg, int d,
                                                        double* __restrict__ mean) {
    const int64_t n = seg[blockIdx.y + 1] - seg[blockIdx.y];
    const double* p0 = part + int64_t(blockIdx.y) * nparts * d;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < d; k += gridDim.x * blockDim.x) {
        double t = 0.0;
        for (int p = 0; p < nparts; ++p) t += p0[int64_t(p) * d + k];
        mean[int64_t(blockIdx.y) * d + k] = t / double(n);
    }
}

__global__ __launch_bounds__(kBlock) void k_rowdev_max_seg(const double* __restrict__ A,
                                                           const int64_t* __restrict__ seg, int d,
                                                           const double* __restrict__ mean,
                                                           double* __restrict__ bmax) {
    const int64_t a = seg[blockIdx.y], n = seg[blockIdx.y + 1] - a;
    const double* mu = mean + int64_t(blockIdx.y) * d;
    double best = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * kBlock) {
        double t = 0.0;
        for (int k = 0; k < d; ++k) {
            const double e = A[(a + i) * d + k] - mu[k];
            t += e * e;
        }
        best = fmax(best, t);
    }
    __shared__ double red[kBlock];
    red[threadIdx.x] = best;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) bmax[int64_t(blockIdx.y) * gridDim.x + blockIdx.x] = red[0];
}

// per vertex of segment s: thr = 1e-5 (1 + S_s), S_s = sqrt(max of the
// segment's nb block maxima)
__global__ __launch_bounds__(kBlock) void k_seg_thresholds(const double* __restrict__ bmax, int nb,
                                                           const int64_t* __restrict__ seg,
                                                           double* __restrict__ vthr) {
    __shared__ double S;
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int b = 0; b < nb; ++b) t = fmax(t, bmax[int64_t(blockIdx.x) * nb + b]);
        S = sqrt(t);
    }
    __syncthreads();
    const double thr = 1e-5 * (1.0 + S);
    for (int64_t i = seg[blockIdx.x] + threadIdx.x; i < seg[blockIdx.x + 1]; i += kBlock)
        vthr[i] = thr;
}

// Streaming copy: each workgroup copies one contiguous chunk, 16-byte
// elements, four loads in flight per thread, non-temporal loads and stores
// (the data is touched once, so it should not displace cached lines).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kCopyGrid = 16384;
__global__ __launch_bounds__(kBlock) void k_stream_copy(const u32x4* __restrict__ a,
                                                        u32x4* __restrict__ b, int64_t N,
                                                        int64_t per) {
    const int64_t s0 = int64_t(blockIdx.x) * per;
    const int64_t e0 = s0 + per < N ? s0 + per : N;
    for (int64_t k = s0 + threadIdx.x; k < e0; k += 4 * kBlock) {
        u32x4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (k + u * kBlock < e0) v[u] = __builtin_nontemporal_load(a + k + u * kBlock);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (k + u * kBlock < e0) __builtin_nontemporal_store(v[u], b + k + u * kBlock);
    }
}

__global__ void k_copy_bytes(const unsigned char* __restrict__ a, unsigned char* __restrict__ b,
                             int64_t N) {
    for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N;
         k += int64_t(gridDim.x) * blockDim.x)
        b[k] = a[k];
}

__global__ __launch_bounds__(kBlock) void k_segsum(const double* __restrict__ rows, int nv,
                                                   const int64_t* __restrict__ seg,
                                                   double* __restrict__ out) {
    const int64_t a = seg[blockIdx.x], b = seg[blockIdx.x + 1];
    for (int c = 0; c < nv; ++c) {
        __shared__ double red[kBlock];
        double t = 0.0;
        for (int64_t r = a + threadIdx.x; r < b; r += kBlock) t += rows[r * nv + c];
        red[threadIdx.x] = t;
        __syncthreads();
        for (int off = kBlock / 2; off > 0; off >>= 1) {
            if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[int64_t(blockIdx.x) * nv + c] = red[0];
        __syncthreads();
    }
}

// scatter union rows back to per-instance output blocks (batched solves)
__global__ __launch_bounds__(kBlock) void k_split(int64_t nU, int d, const double* __restrict__ X,
                                                  const int* __restrict__ lab,
                                                  const int64_t* __restrict__ vseg, int S,
                                                  const int64_t* __restrict__ xoff,
                                                  const int64_t* __restrict__ loff, int t,
                                                  double* __restrict__ Xout,
                                                  int* __restrict__ Lout) {
    const int64_t N = nU * d;
    for (int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x; e < N;
         e += int64_t(gridDim.x) * kBlock) {
        const int64_t i = e / d, k = e % d;
        int lo = 0, hi = S;  // last segment with vseg[s] <= i
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (vseg[mid] <= i) lo = mid;
            else hi = mid;
        }
        const int64_t v0 = vseg[lo], ns = vseg[lo + 1] - v0, li = i - v0;
        Xout[xoff[lo] + int64_t(t) * ns * d + li * d + k] = X[e];
        if (Lout && k == 0) Lout[loff[lo] + int64_t(t) * ns + li] = lab[i] - lab[v0];
    }
}

__global__ __launch_bounds__(kBlock) void k_row_sqnorm(const double* __restrict__ X, int64_t n,
                                                       int d, double* __restrict__ out) {
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * kBlock) {
        double t = 0.0;
        for (int k = 0; k < d; ++k) t += X[i * d + k] * X[i * d + k];
        out[i] = t;
    }
}

__global__ void k_first_labels(const int* __restrict__ lab, const int64_t* __restrict__ vseg,
                               int S, int* __restrict__ out) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < S; s += gridDim.x * blockDim.x)
        out[s] = lab[vseg[s]];
}

__global__ __launch_bounds__(kBlock) void k_offset_edges(int64_t m, const int* __restrict__ src,
                                                         const int* __restrict__ dst,
                                                         const double* __restrict__ w,
                                                         int voff, int nloc,
                                                         int* __restrict__ so,
                                                         int* __restrict__ dso,
                                                         double* __restrict__ wo, int* bad) {
    int b = 0;
    for (int64_t l = int64_t(blockIdx.x) * kBlock + threadIdx.x; l < m;
         l += int64_t(gridDim.x) * kBlock) {
        const int a = src[l], c = dst[l];
        if (a < 0 || c >= nloc || a >= c) b = 1;
        so[l] = a + voff;
        dso[l] = c + voff;
        wo[l] = w[l];
    }
    if (b) atomicOr(bad, 1);
}

constexpr int kSpreadBlocks = 128;

}  // namespace

// CG vector kernels: every block of the update (and the skip test of every
// matvec block) re-reduces the previous kernels' partials, so for vectors of
// up to 4M values the grid is kept to 256 blocks (a grid-stride loop covers
// the rest: at n = 1e4, d = 64 the step is 2.5 % shorter than with 1024);
// longer vectors keep the full grid for bandwidth.
int cg_update_grid(int64_t N) {
    const int cap = N < (int64_t(1) << 22) ? 256 : 1024;
    return flat_grid(N) < cap ? flat_grid(N) : cap;
}

void launch_cg_init(int64_t N, const double* b, bool neg, const double* Dinv, CgBufs& cg,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_cg_init, dim3(cg_update_grid(N)), dim3(kBlock), 0, s, N, b, neg ? -1.0 : 1.0,
                       Dinv, cg.x, cg.r, cg.u, cg.p, cg.s, cg.upd[0], cg.flag);
}

void launch_cg_update(int64_t N, int j, const double* Dinv, CgBufs& cg, double thr,
                      hipStream_t s) {
    const int par = j & 1;
    hipLaunchKernelGGL(k_cg_update, dim3(cg_update_grid(N)), dim3(kBlock), 0, s, N, j, Dinv,
                       cg.x, cg.r, cg.u, cg.w, cg.p, cg.s, cg.upd[par], cg.upd[par ^ 1],
                       cg.wu[par], cg.nparts, cg.nparts_mv, cg.state, cg.flag, thr);
}

int launch_trial(int64_t N, const double* X, const double* D, double alpha, const double* A,
                 const double* G, double* Xt, double* partials, hipStream_t s) {
    const int grid = flat_grid(N);
    hipLaunchKernelGGL(k_trial, dim3(grid), dim3(kBlock), 0, s, N, X, D, alpha, A, G, Xt,
                       partials);
    return grid;
}

void launch_flag_nonfinite(const double* x, int64_t count, int* flag, hipStream_t s) {
    int64_t g = (count + kBlock - 1) / kBlock;
    g = g < 1 ? 1 : g > kMaxGrid ? kMaxGrid : g;
    hipLaunchKernelGGL(k_flag_nonfinite, dim3(unsigned(g)), dim3(kBlock), 0, s, x, count, flag);
}

void launch_finalize_multi(const FinalizeJobs& jobs, int njobs, hipStream_t s) {
    if (njobs > 0)
        hipLaunchKernelGGL(k_finalize_multi, dim3(njobs), dim3(kFinalizeWaves * 64), 0, s, jobs);
}

void launch_finalize(const double* partials, int nparts, int nv, double* out, hipStream_t s) {
    switch (nv) {
        case 1: hipLaunchKernelGGL(k_finalize<1>, dim3(1), dim3(kFinalizeWaves * 64), 0, s, partials, nparts, out); break;
        case 2: hipLaunchKernelGGL(k_finalize<2>, dim3(1), dim3(kFinalizeWaves * 64), 0, s, partials, nparts, out); break;
        case 3: hipLaunchKernelGGL(k_finalize<3>, dim3(1), dim3(kFinalizeWaves * 64), 0, s, partials, nparts, out); break;
        case 4: hipLaunchKernelGGL(k_finalize<4>, dim3(1), dim3(kFinalizeWaves * 64), 0, s, partials, nparts, out); break;
        case 5: hipLaunchKernelGGL(k_finalize<5>, dim3(1), dim3(kFinalizeWaves * 64), 0, s, partials, nparts, out); break;
        case 6: hipLaunchKernelGGL(k_finalize<6>, dim3(1), dim3(kFinalizeWaves * 64), 0, s, partials, nparts, out); break;
        default: hipLaunchKernelGGL(k_finalize<7>, dim3(1), dim3(kFinalizeWaves * 64), 0, s, partials, nparts, out); break;
    }
}

void launch_fill(double* x, int64_t N, double v, hipStream_t s) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3(flat_grid(N)), dim3(kBlock), 0, s, x, N, v);
}

void launch_axpy(double* x, double alpha, const double* y, int64_t N, hipStream_t s) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_axpy, dim3(flat_grid(N)), dim3(kBlock), 0, s, x, alpha, y, N);
}

void launch_axpby(double a, const double* x, double b, const double* y, double* out, int64_t N,
                  hipStream_t s) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_axpby, dim3(flat_grid(N)), dim3(kBlock), 0, s, a, x, b, y, out, N);
}

int launch_dot(const double* x, const double* y, int64_t N, double* partials, hipStream_t s) {
    const int g = flat_grid(N);
    hipLaunchKernelGGL(k_dot, dim3(g), dim3(kBlock), 0, s, x, y, N, partials);
    return g;
}

void launch_copy(const double* a, double* b, int64_t N, hipStream_t s) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_copy, dim3(flat_grid(N)), dim3(kBlock), 0, s, a, b, N);
}

void launch_sub(const double* a, const double* b, double* out, int64_t N, hipStream_t s) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_sub, dim3(flat_grid(N)), dim3(kBlock), 0, s, a, b, out, N);
}

void launch_lap_dinv(const DevGraph& g, int d, double c0, double sigma, double* Dinv,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_lap_dinv, dim3(flat_grid(g.n * d)), dim3(kBlock), 0, s, g.n, d,
                       g.inc_ptr, g.vrank, c0, sigma, Dinv);
}

int spread_work_size(int64_t n, int d) { return kSpreadBlocks * d + d + kSpreadBlocks; }

void launch_spread(const double* A, int64_t n, int d, double* work, double* out, hipStream_t s) {
    double* part = work;
    double* mean = work + int64_t(kSpreadBlocks) * d;
    double* bmax = mean + d;
    hipLaunchKernelGGL(k_colsum, dim3(kSpreadBlocks), dim3(kBlock), 0, s, A, n, d, part);
    hipLaunchKernelGGL(k_colmean, dim3((d + kBlock - 1) / kBlock), dim3(kBlock), 0, s, part,
                       kSpreadBlocks, n, d, mean);
    hipLaunchKernelGGL(k_rowdev_max, dim3(kSpreadBlocks), dim3(kBlock), 0, s, A, n, d, mean, bmax);
    hipLaunchKernelGGL(k_max_sqrt, dim3(1), dim3(kBlock), 0, s, bmax, kSpreadBlocks, out);
}

__global__ __launch_bounds__(kBlock) void k_exp(const double* __restrict__ x, int64_t n,
                                                double* __restrict__ y) {
    for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < n;
         k += int64_t(gridDim.x) * kBlock)
        y[k] = exp(x[k]);
}

void launch_exp(const double* x, int64_t n, double* y, hipStream_t s) {
    hipLaunchKernelGGL(k_exp, dim3(flat_grid(n)), dim3(kBlock), 0, s, x, n, y);
}

int seg_threshold_work_size(int nseg, int d) {
    return nseg * (kSpreadBlocks * d + d + kSpreadBlocks);
}

void launch_seg_thresholds(const double* A, const int64_t* seg, int nseg, int d, double* work,
                           double* vthr, hipStream_t s) {
    if (nseg < 1) return;
    double* part = work;
    double* mean = part + int64_t(nseg) * kSpreadBlocks * d;
    double* bmax = mean + int64_t(nseg) * d;
    hipLaunchKernelGGL(k_colsum_seg, dim3(kSpreadBlocks, nseg), dim3(kBlock), 0, s, A, seg, d,
                       part);
    hipLaunchKernelGGL(k_colmean_seg, dim3((d + kBlock - 1) / kBlock, nseg), dim3(kBlock), 0, s,
                       part, kSpreadBlocks, seg, d, mean);
    hipLaunchKernelGGL(k_rowdev_max_seg, dim3(kSpreadBlocks, nseg), dim3(kBlock), 0, s, A, seg, d,
                       mean, bmax);
    hipLaunchKernelGGL(k_seg_thresholds, dim3(nseg), dim3(kBlock), 0, s, bmax, kSpreadBlocks, seg,
                       vthr);
}

void launch_segsum(const double* rows, int nv, const int64_t* seg, int nseg, double* out,
                   hipStream_t s) {
    if (nseg <= 0) return;
    hipLaunchKernelGGL(k_segsum, dim3(nseg), dim3(kBlock), 0, s, rows, nv, seg, out);
}

void launch_split(int64_t nU, int d, const double* X, const int* lab, const int64_t* vseg, int S,
                  const int64_t* xoff, const int64_t* loff, int t, double* Xout, int* Lout,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_split, dim3(flat_grid(nU * d)), dim3(kBlock), 0, s, nU, d, X, lab, vseg,
                       S, xoff, loff, t, Xout, Lout);
}

void launch_row_sqnorm(const double* X, int64_t n, int d, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_row_sqnorm, dim3(flat_grid(n)), dim3(kBlock), 0, s, X, n, d, out);
}

void launch_first_labels(const int* lab, const int64_t* vseg, int S, int* out, hipStream_t s) {
    hipLaunchKernelGGL(k_first_labels, dim3((S + 255) / 256), dim3(256), 0, s, lab, vseg, S, out);
}

void launch_offset_edges(int64_t m, const int* src, const int* dst, const double* w, int voff,
                         int nloc, int* so, int* dso, double* wo, int* bad, hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_offset_edges, dim3(flat_grid(m)), dim3(kBlock), 0, s, m, src, dst, w, voff,
                       nloc, so, dso, wo, bad);
}

void launch_stream_copy(const void* src, void* dst, int64_t bytes, hipStream_t s) {
    const int64_t n16 = bytes / 16;
    if (n16 > 0 && (reinterpret_cast<uintptr_t>(src) % 16 == 0) &&
        (reinterpret_cast<uintptr_t>(dst) % 16 == 0)) {
        int64_t g = (n16 + kBlock - 1) / kBlock;
        if (g > kCopyGrid) g = kCopyGrid;
        const int64_t per = (n16 + g - 1) / g;
        hipLaunchKernelGGL(k_stream_copy, dim3(g), dim3(kBlock), 0, s,
                           reinterpret_cast<const u32x4*>(src), reinterpret_cast<u32x4*>(dst), n16,
                           per);
        const int64_t rest = bytes - n16 * 16;
        if (rest > 0)
            hipLaunchKernelGGL(k_copy_bytes, dim3(1), dim3(64), 0, s,
                               reinterpret_cast<const unsigned char*>(src) + n16 * 16,
                               reinterpret_cast<unsigned char*>(dst) + n16 * 16, rest);
    } else if (bytes > 0) {
        hipLaunchKernelGGL(k_copy_bytes, dim3(1024), dim3(kBlock), 0, s,
                           reinterpret_cast<const unsigned char*>(src),
                           reinterpret_cast<unsigned char*>(dst), bytes);
    }
}

}  // namespace ccm
