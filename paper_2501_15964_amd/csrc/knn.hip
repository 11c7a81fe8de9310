// Exact k-NN search and the union-symmetrised Gaussian weight graph.
//
// Squared distances are accumulated feature by feature in ascending order
// with separately rounded products and sums (no fused multiply-add), so every
// d^2 is bit-defined and the neighbour order (d^2, index) is reproducible.
// A block computes 64 x 64 tiles of distances (a 4 x 4 register tile per
// thread, query and candidate features staged through LDS 16 at a time),
// writes each tile to LDS, and 4 threads per query row scan it into partial
// top-KP lists (one per quarter of the tile columns).  Candidate columns are
// split over blockIdx.y; a second pass merges the partial lists.
#include <hipcub/hipcub.hpp>

#include "knn.hpp"

namespace ccm {
namespace {

constexpr int kQT = 64;   // query rows per block
constexpr int kCT = 64;   // candidate rows per tile
constexpr int kDK = 16;   // features per LDS chunk

__device__ __forceinline__ bool knn_less(double da, int ja, double db, int jb) {
    return da < db || (da == db && ja < jb);
}

template <int KP>
__device__ __forceinline__ void knn_insert(double (&bd)[KP], int (&bi)[KP], double dv, int j) {
    if (!knn_less(dv, j, bd[KP - 1], bi[KP - 1])) return;
    bool placed = false;
#pragma unroll
    for (int p = KP - 1; p >= 1; --p) {
        if (!placed) {
            if (knn_less(dv, j, bd[p - 1], bi[p - 1])) {
                bd[p] = bd[p - 1];
                bi[p] = bi[p - 1];
            } else {
                bd[p] = dv;
                bi[p] = j;
                placed = true;
            }
        }
    }
    if (!placed) {
        bd[0] = dv;
        bi[0] = j;
    }
}

template <int KP>
__global__ __launch_bounds__(kBlock) void k_knn_partial(const double* __restrict__ A, int64_t n,
                                                        int d, int64_t cols_per_split,
                                                        double* __restrict__ pd,
                                                        int* __restrict__ pi) {
    __shared__ double Qs[kDK][kQT];
    __shared__ double Cs[kDK][kCT];
    __shared__ double Ds[kQT][kCT + 1];
    const int tid = threadIdx.x;
    const int tx = tid % 16, ty = tid / 16;  // candidates 4 tx.., queries 4 ty..
    const int64_t q0 = int64_t(blockIdx.x) * kQT;
    const int64_t c_begin = int64_t(blockIdx.y) * cols_per_split;
    int64_t c_end = c_begin + cols_per_split;
    if (c_end > n) c_end = n;
    // scan role: query row tid / 4, quarter tid % 4 of the tile columns
    const int srow = tid >> 2, quarter = tid & 3;
    const int64_t qi = q0 + srow;
    double bd[KP];
    int bi[KP];
#pragma unroll
    for (int p = 0; p < KP; ++p) {
        bd[p] = INFINITY;
        bi[p] = 0x7fffffff;
    }
    for (int64_t c0 = c_begin; c0 < c_end; c0 += kCT) {
        double acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
        for (int k0 = 0; k0 < d; k0 += kDK) {
            const int dk = (d - k0) < kDK ? (d - k0) : kDK;
            __syncthreads();
            for (int e = tid; e < kQT * kDK; e += kBlock) {
                const int t = e / kDK, k = e % kDK;
                const int64_t row = q0 + t;
                Qs[k][t] = (row < n && k < dk) ? A[row * d + k0 + k] : 0.0;
            }
            for (int e = tid; e < kCT * kDK; e += kBlock) {
                const int c = e / kDK, k = e % kDK;
                const int64_t row = c0 + c;
                Cs[k][c] = (row < c_end && k < dk) ? A[row * d + k0 + k] : 0.0;
            }
            __syncthreads();
            {
                // separately rounded subtract, multiply and add: no contraction
                // into fused multiply-adds, so each d^2 is bit-defined
#pragma clang fp contract(off)
                for (int k = 0; k < dk; ++k) {
                    double qv[4], cv[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) qv[i] = Qs[k][ty * 4 + i];
#pragma unroll
                    for (int j = 0; j < 4; ++j) cv[j] = Cs[k][tx * 4 + j];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const double df = qv[i] - cv[j];
                            const double sq = df * df;
                            acc[i][j] = acc[i][j] + sq;
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) Ds[ty * 4 + i][tx * 4 + j] = acc[i][j];
        __syncthreads();
        if (qi < n) {
            for (int cc = quarter * 16; cc < quarter * 16 + 16; ++cc) {
                const int64_t j = c0 + cc;
                if (j >= c_end || j == qi) continue;
                knn_insert<KP>(bd, bi, Ds[srow][cc], int(j));
            }
        }
    }
    if (qi < n) {
        const int64_t base = ((int64_t(blockIdx.y) * 4 + quarter) * n + qi) * KP;
#pragma unroll
        for (int p = 0; p < KP; ++p) {
            pd[base + p] = bd[p];
            pi[base + p] = bi[p];
        }
    }
}

template <int KP>
__global__ __launch_bounds__(kBlock) void k_knn_merge(int64_t n, int k, int splits,
                                                      const double* __restrict__ pd,
                                                      const int* __restrict__ pi,
                                                      int* __restrict__ nbr,
                                                      double* __restrict__ nd2) {
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * kBlock) {
        double bd[KP];
        int bi[KP];
#pragma unroll
        for (int p = 0; p < KP; ++p) {
            bd[p] = INFINITY;
            bi[p] = 0x7fffffff;
        }
        for (int sp = 0; sp < splits; ++sp) {
            const int64_t base = (int64_t(sp) * n + i) * KP;
            for (int p = 0; p < KP; ++p) {
                const int j = pi[base + p];
                if (j == 0x7fffffff) break;
                knn_insert<KP>(bd, bi, pd[base + p], j);
            }
        }
#pragma unroll
        for (int p = 0; p < KP; ++p) {
            if (p < k) {
                nbr[i * k + p] = bi[p];
                nd2[i * k + p] = bd[p];
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_pair_keys(int64_t n, int k, const int* __restrict__ nbr,
                                                      unsigned long long* __restrict__ key) {
    const int64_t cnt = n * k;
    for (int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x; e < cnt;
         e += int64_t(gridDim.x) * kBlock) {
        const unsigned i = unsigned(e / k), j = unsigned(nbr[e]);
        const unsigned lo = i < j ? i : j, hi = i < j ? j : i;
        key[e] = (static_cast<unsigned long long>(lo) << 32) | hi;
    }
}

__global__ __launch_bounds__(kBlock) void k_weights(int64_t m, const unsigned long long* __restrict__ key,
                                                    const double* __restrict__ d2, double phi,
                                                    int* __restrict__ keep,
                                                    double* __restrict__ wtmp) {
    for (int64_t l = int64_t(blockIdx.x) * kBlock + threadIdx.x; l < m;
         l += int64_t(gridDim.x) * kBlock) {
        const double wv = exp(-phi * d2[l]);
        wtmp[l] = wv;
        keep[l] = wv > 0.0 ? 1 : 0;
    }
}

__global__ __launch_bounds__(kBlock) void k_emit(int64_t m, const unsigned long long* __restrict__ key,
                                                 const double* __restrict__ wtmp,
                                                 const int* __restrict__ keep,
                                                 const int* __restrict__ pos,
                                                 int* __restrict__ src, int* __restrict__ dst,
                                                 double* __restrict__ w) {
    for (int64_t l = int64_t(blockIdx.x) * kBlock + threadIdx.x; l < m;
         l += int64_t(gridDim.x) * kBlock) {
        if (!keep[l]) continue;
        const int p = pos[l];
        src[p] = int(key[l] >> 32);
        dst[p] = int(key[l] & 0xffffffffull);
        w[p] = wtmp[l];
    }
}

__global__ void k_median(const double* __restrict__ sorted, int64_t cnt, double* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (cnt % 2 == 1) out[0] = sorted[cnt / 2];
        else out[0] = (sorted[cnt / 2 - 1] + sorted[cnt / 2]) / 2.0;
    }
}

// ---- quantised data: exact integer distances on int8 MFMA ------------------
//
// Codes K in [0, 255] are centred to K - 128 in int8 and padded to a
// multiple of 64 features; then d2(i, j) = |a_i|^2 + |a_j|^2 - 2 a_i.a_j is
// exact in int32 (|a_i . a_j| <= 784 * 128^2 < 2^31 for d <= 1024 ... and in
// general d * 128^2 < 2^31).  A block owns 64 query rows (16 per wave);
// candidate tiles of 64 rows are staged in LDS; each wave accumulates four
// 16 x 16 tiles with v_mfma_i32_16x16x64_i8 (16 int8 per lane per operand;
// A and B place the same k values in the same lane slots, so the dot
// product does not depend on the hardware's k numbering).  The 64 x 64
// distance tile goes through LDS to a top-KP scan by 4 threads per row.

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kUQ = 64;   // query rows per block
constexpr int kUC = 64;   // candidate rows per tile

__global__ __launch_bounds__(kBlock) void k_u8_prep(const unsigned char* __restrict__ K, int64_t n,
                                                    int d, int dp,
                                                    signed char* __restrict__ Kc,
                                                    int* __restrict__ nrm) {
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * kBlock) {
        int s = 0;
        for (int k = 0; k < dp; ++k) {
            const int v = k < d ? int(K[i * d + k]) - 128 : 0;
            Kc[i * dp + k] = static_cast<signed char>(v);
            s += v * v;
        }
        nrm[i] = s;
    }
}

template <int KP>
__device__ __forceinline__ void knn_insert_i(int (&bd)[KP], int (&bi)[KP], int dv, int j) {
    if (!(dv < bd[KP - 1] || (dv == bd[KP - 1] && j < bi[KP - 1]))) return;
    bool placed = false;
#pragma unroll
    for (int p = KP - 1; p >= 1; --p) {
        if (!placed) {
            if (dv < bd[p - 1] || (dv == bd[p - 1] && j < bi[p - 1])) {
                bd[p] = bd[p - 1];
                bi[p] = bi[p - 1];
            } else {
                bd[p] = dv;
                bi[p] = j;
                placed = true;
            }
        }
    }
    if (!placed) {
        bd[0] = dv;
        bi[0] = j;
    }
}

// LDS row stride of a staged candidate tile: dp bytes padded so that the
// stride in 4-byte banks is 4 modulo 32, so the 16 rows one MFMA operand load
// touches fall on different banks
__host__ __device__ constexpr int u8_tile_stride(int dp) {
    return dp + 4 * ((4 - (dp / 4) % 32 + 32) % 32);
}
constexpr int kUDs = kUC + 1;  // distance tile row stride (odd: no bank conflicts)

// Query rows of at most kUAreg x 64 codes keep their MFMA operands in
// registers for the whole scan; longer rows load them for every tile.
constexpr int kUAreg = 16;

template <int KP, bool AREG>
__global__ __launch_bounds__(kBlock, 2) void k_knn_u8(const signed char* __restrict__ Kc,
                                                   const int* __restrict__ nrm, int64_t n, int dp,
                                                   int64_t cols_per_split, double* __restrict__ pd,
                                                   int* __restrict__ pi) {
    extern __shared__ unsigned char smem[];
    const int bst = u8_tile_stride(dp);
    signed char* Bs = reinterpret_cast<signed char*>(smem);         // kUC x bst
    int* Ds = reinterpret_cast<int*>(smem + size_t(kUC) * bst);     // kUQ x kUDs
    int* Ns = Ds + kUQ * kUDs;                                      // kUC candidate norms
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int64_t q0 = int64_t(blockIdx.x) * kUQ;
    const int64_t c_begin = int64_t(blockIdx.y) * cols_per_split;
    int64_t c_end = c_begin + cols_per_split;
    if (c_end > n) c_end = n;
    const int ks = dp / 64;  // MFMA k steps
    // scan role: query row lane of the block, candidate quarter wave of a tile
    const int srow = lane, quarter = wave;
    const int64_t qi = q0 + srow;
    const int nq = qi < n ? nrm[qi] : 0;
    int bd[KP], bi[KP];
#pragma unroll
    for (int p = 0; p < KP; ++p) {
        bd[p] = 0x7fffffff;
        bi[p] = 0x7fffffff;
    }
    // MFMA role: 16 query rows per wave; lane -> (row lane % 16, k slot lane / 16)
    const int64_t arow = q0 + wave * 16 + (lane & 15);
    const int kslot = (lane >> 4) * 16;
    v4i areg[AREG ? kUAreg : 1];
    if constexpr (AREG) {
#pragma unroll
        for (int u = 0; u < kUAreg; ++u) {
            areg[u] = v4i{0, 0, 0, 0};
            if (u < ks && arow < n)
                areg[u] = *reinterpret_cast<const v4i*>(Kc + arow * dp + u * 64 + kslot);
        }
    }
    // A tile is staged as dp / 64 16-byte chunks per thread, loaded eight at
    // a time before any is stored, so their latencies overlap; the first
    // four chunks of the next tile are loaded while this tile is multiplied
    // and scanned.
    constexpr int kPre = 4;
    auto load = [&](int64_t c, int b0, int cnt, v4i* v) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (u >= cnt) break;
            v[u] = v4i{0, 0, 0, 0};
            const int e = tid + (b0 + u) * kBlock;
            const int r = (e * 16) / dp, off = (e * 16) % dp;
            if (b0 + u < ks && c + r < c_end)
                v[u] = *reinterpret_cast<const v4i*>(Kc + (c + r) * dp + off);
        }
    };
    auto store = [&](int b0, int cnt, const v4i* v) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (u >= cnt) break;
            const int e = tid + (b0 + u) * kBlock;
            const int r = (e * 16) / dp, off = (e * 16) % dp;
            if (b0 + u < ks) *reinterpret_cast<v4i*>(Bs + r * bst + off) = v[u];
        }
    };
    v4i pre[kPre];
    if (c_begin < c_end) load(c_begin, 0, kPre, pre);
    for (int64_t c0 = c_begin; c0 < c_end; c0 += kUC) {
        __syncthreads();
        store(0, kPre, pre);
        for (int b0 = kPre; b0 < ks; b0 += 8) {
            v4i v[8];
            load(c0, b0, 8, v);
            store(b0, 8, v);
        }
        if (tid < kUC) Ns[tid] = c0 + tid < c_end ? nrm[c0 + tid] : 0;
        __syncthreads();
        if (c0 + kUC < c_end) load(c0 + kUC, 0, kPre, pre);
        v4i acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = v4i{0, 0, 0, 0};
        if constexpr (AREG) {
#pragma unroll
            for (int u = 0; u < kUAreg; ++u) {
                if (u < ks) {
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const v4i b = *reinterpret_cast<const v4i*>(
                            Bs + (t * 16 + (lane & 15)) * bst + u * 64 + kslot);
                        acc[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(areg[u], b, acc[t], 0, 0,
                                                                       0);
                    }
                }
            }
        } else {
            for (int kk = 0; kk < dp; kk += 64) {
                v4i a = {0, 0, 0, 0};
                if (arow < n) a = *reinterpret_cast<const v4i*>(Kc + arow * dp + kk + kslot);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const v4i b = *reinterpret_cast<const v4i*>(
                        Bs + (t * 16 + (lane & 15)) * bst + kk + kslot);
                    acc[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, acc[t], 0, 0, 0);
                }
            }
        }
        // output element (row 4 (lane / 16) + r, column lane % 16) of each 16 x 16 tile
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = wave * 16 + (lane >> 4) * 4 + r;
                const int col = t * 16 + (lane & 15);
                Ds[row * kUDs + col] = acc[t][r];
            }
        }
        __syncthreads();
        if (qi < n) {
#pragma unroll 4
            for (int cc = quarter * 16; cc < quarter * 16 + 16; ++cc) {
                const int64_t j = c0 + cc;
                if (j >= c_end || j == qi) continue;
                const int dv = nq + Ns[cc] - 2 * Ds[srow * kUDs + cc];
                knn_insert_i<KP>(bd, bi, dv, int(j));
            }
        }
    }
    if (qi < n) {
        const int64_t base = ((int64_t(blockIdx.y) * 4 + quarter) * n + qi) * KP;
#pragma unroll
        for (int p = 0; p < KP; ++p) {
            pd[base + p] = bi[p] == 0x7fffffff ? INFINITY : double(bd[p]);
            pi[base + p] = bi[p];
        }
    }
}

#define HIPCHK(expr)                                                      \
    do {                                                                  \
        hipError_t e_ = (expr);                                           \
        if (e_ != hipSuccess) {                                           \
            err = std::string(#expr) + ": " + hipGetErrorString(e_);      \
            return e_ == hipErrorOutOfMemory ? CCM_E_NOMEM : CCM_E_HIP;   \
        }                                                                 \
    } while (0)

template <int KP>
void launch_knn(const double* A, int64_t n, int d, int k, int splits, int64_t cps, double* pd,
                int* pi, int* nbr, double* nd2, hipStream_t s) {
    const dim3 grid{unsigned((n + kQT - 1) / kQT), unsigned(splits), 1u};
    hipLaunchKernelGGL((k_knn_partial<KP>), grid, dim3(kBlock), 0, s, A, n, d, cps, pd, pi);
    // four partial lists (tile quarters) per split and row
    hipLaunchKernelGGL((k_knn_merge<KP>), dim3(flat_grid(n)), dim3(kBlock), 0, s, n, k,
                       splits * 4, pd, pi, nbr, nd2);
}

}  // namespace

ccm_status knn_finish(DevMem& nbr, DevMem& nd2, int64_t n, int k, double phi, int* src, int* dst,
                      double* w, int64_t m_cap, int64_t& m_out, double& phi_out, hipStream_t s,
                      std::string& err);

ccm_status knn_graph(const double* A, int64_t n, int d, int k, double phi, int* src, int* dst,
                     double* w, int64_t m_cap, int64_t& m_out, double& phi_out, hipStream_t s,
                     std::string& err) {
    const int KP = k <= 4 ? 4 : k <= 8 ? 8 : k <= 16 ? 16 : 32;
    // split candidate columns so that the grid has enough blocks
    const int64_t qblocks = (n + kQT - 1) / kQT;
    int64_t splits = (2048 + qblocks - 1) / qblocks;
    const int64_t ctiles = (n + kCT - 1) / kCT;
    if (splits > ctiles) splits = ctiles;
    if (splits < 1) splits = 1;
    int64_t cps = ((ctiles + splits - 1) / splits) * kCT;
    splits = (n + cps - 1) / cps;
    const int64_t cnt = n * k;
    DevMem pd, pi, nbr, nd2;
    HIPCHK(pd.alloc(size_t(splits) * 4 * n * KP * 8, s));
    HIPCHK(pi.alloc(size_t(splits) * 4 * n * KP * 4, s));
    HIPCHK(nbr.alloc(size_t(cnt) * 4, s));
    HIPCHK(nd2.alloc(size_t(cnt) * 8, s));
    switch (KP) {
        case 4: launch_knn<4>(A, n, d, k, int(splits), cps, pd.as<double>(), pi.as<int>(),
                              nbr.as<int>(), nd2.as<double>(), s); break;
        case 8: launch_knn<8>(A, n, d, k, int(splits), cps, pd.as<double>(), pi.as<int>(),
                              nbr.as<int>(), nd2.as<double>(), s); break;
        case 16: launch_knn<16>(A, n, d, k, int(splits), cps, pd.as<double>(), pi.as<int>(),
                                nbr.as<int>(), nd2.as<double>(), s); break;
        default: launch_knn<32>(A, n, d, k, int(splits), cps, pd.as<double>(), pi.as<int>(),
                                nbr.as<int>(), nd2.as<double>(), s); break;
    }
    HIPCHK(hipGetLastError());
    pd.release();
    pi.release();
    return knn_finish(nbr, nd2, n, k, phi, src, dst, w, m_cap, m_out, phi_out, s, err);
}

// scale the exact integer distances: d2 = (double)D * scale * scale
__global__ __launch_bounds__(kBlock) void k_scale_d2(int64_t cnt, double scale,
                                                     double* __restrict__ d2) {
    for (int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x; e < cnt;
         e += int64_t(gridDim.x) * kBlock)
        d2[e] = d2[e] * scale * scale;
}

ccm_status knn_graph_u8(const unsigned char* K, int64_t n, int d, double scale, int k, double phi,
                        int* src, int* dst, double* w, int64_t m_cap, int64_t& m_out,
                        double& phi_out, hipStream_t s, std::string& err) {
    const int KP = k <= 4 ? 4 : k <= 8 ? 8 : k <= 16 ? 16 : 32;
    const int dp = (d + 63) / 64 * 64;
    DevMem Kc, nrm;
    HIPCHK(Kc.alloc(size_t(n) * dp, s));
    HIPCHK(nrm.alloc(size_t(n) * 4, s));
    hipLaunchKernelGGL(k_u8_prep, dim3(flat_grid(n)), dim3(kBlock), 0, s, K, n, d, dp,
                       Kc.as<signed char>(), nrm.as<int>());
    const int64_t qblocks = (n + kUQ - 1) / kUQ;
    const int64_t ctiles = (n + kUC - 1) / kUC;
    // about eight rounds of two blocks per compute unit, so the last round's
    // tail is a small part of the launch
    int64_t splits = (4096 + qblocks - 1) / qblocks;
    if (splits > ctiles) splits = ctiles;
    if (splits < 1) splits = 1;
    const int64_t cps = ((ctiles + splits - 1) / splits) * kUC;
    splits = (n + cps - 1) / cps;
    const int64_t cnt = n * k;
    const int nl = int(splits) * 4;  // partial lists per row
    DevMem pd, pi, nbr, nd2;
    HIPCHK(pd.alloc(size_t(nl) * n * KP * 8, s));
    HIPCHK(pi.alloc(size_t(nl) * n * KP * 4, s));
    HIPCHK(nbr.alloc(size_t(cnt) * 4, s));
    HIPCHK(nd2.alloc(size_t(cnt) * 8, s));
    const size_t lds =
        size_t(kUC) * u8_tile_stride(dp) + size_t(kUQ) * kUDs * 4 + size_t(kUC) * 4;
    const dim3 grid{unsigned(qblocks), unsigned(splits), 1u};
    auto run = [&](auto KPc) {
        constexpr int kp = decltype(KPc)::value;
        auto go = [&](auto kern) {
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
            hipLaunchKernelGGL(kern, grid, dim3(kBlock), lds, s, Kc.as<signed char>(),
                               nrm.as<int>(), n, dp, cps, pd.as<double>(), pi.as<int>());
        };
        if (dp <= 64 * kUAreg) go(&k_knn_u8<kp, true>);
        else go(&k_knn_u8<kp, false>);
        hipLaunchKernelGGL((k_knn_merge<kp>), dim3(flat_grid(n)), dim3(kBlock), 0, s, n, k, nl,
                           pd.as<double>(), pi.as<int>(), nbr.as<int>(), nd2.as<double>());
    };
    switch (KP) {
        case 4: run(IC<4>{}); break;
        case 8: run(IC<8>{}); break;
        case 16: run(IC<16>{}); break;
        default: run(IC<32>{}); break;
    }
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_scale_d2, dim3(flat_grid(cnt)), dim3(kBlock), 0, s, cnt, scale,
                       nd2.as<double>());
    pd.release();
    pi.release();
    return knn_finish(nbr, nd2, n, k, phi, src, dst, w, m_cap, m_out, phi_out, s, err);
}

// median, union symmetrisation and Gaussian weights of directed k-NN lists
ccm_status knn_finish(DevMem& nbr, DevMem& nd2, int64_t n, int k, double phi, int* src, int* dst,
                      double* w, int64_t m_cap, int64_t& m_out, double& phi_out, hipStream_t s,
                      std::string& err) {
    const int64_t cnt = n * k;
    // phi = 1 / median of the n k directed distances when not given
    if (!(phi > 0)) {
        DevMem sorted, temp, med;
        HIPCHK(sorted.alloc(size_t(cnt) * 8, s));
        HIPCHK(med.alloc(8, s));
        size_t tb = 0;
        HIPCHK(hipcub::DeviceRadixSort::SortKeys(nullptr, tb, nd2.as<double>(),
                                                 sorted.as<double>(), int(cnt), 0, 64, s));
        HIPCHK(temp.alloc(tb, s));
        HIPCHK(hipcub::DeviceRadixSort::SortKeys(temp.p, tb, nd2.as<double>(),
                                                 sorted.as<double>(), int(cnt), 0, 64, s));
        hipLaunchKernelGGL(k_median, dim3(1), dim3(64), 0, s, sorted.as<double>(), cnt,
                           med.as<double>());
        double h = 0;
        HIPCHK(hipMemcpyAsync(&h, med.p, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        phi = h > 0 ? 1.0 / h : 1.0;
    }
    phi_out = phi;
    // union symmetrisation: one key per unordered pair; both directions carry
    // the same d^2 bit for bit, so keeping the minimum keeps that value
    DevMem key, key_s, d2_s, uniq, d2u, nruns, temp2;
    HIPCHK(key.alloc(size_t(cnt) * 8, s));
    HIPCHK(key_s.alloc(size_t(cnt) * 8, s));
    HIPCHK(d2_s.alloc(size_t(cnt) * 8, s));
    HIPCHK(uniq.alloc(size_t(cnt) * 8, s));
    HIPCHK(d2u.alloc(size_t(cnt) * 8, s));
    HIPCHK(nruns.alloc(8, s));
    hipLaunchKernelGGL(k_pair_keys, dim3(flat_grid(cnt)), dim3(kBlock), 0, s, n, k, nbr.as<int>(),
                       key.as<unsigned long long>());
    size_t b1 = 0, b2 = 0;
    HIPCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, b1, key.as<unsigned long long>(),
                                              key_s.as<unsigned long long>(), nd2.as<double>(),
                                              d2_s.as<double>(), int(cnt), 0, 64, s));
    HIPCHK(hipcub::DeviceReduce::ReduceByKey(nullptr, b2, key_s.as<unsigned long long>(),
                                             uniq.as<unsigned long long>(), d2_s.as<double>(),
                                             d2u.as<double>(), nruns.as<int>(), hipcub::Min(),
                                             int(cnt), s));
    HIPCHK(temp2.alloc(b1 > b2 ? b1 : b2, s));
    HIPCHK(hipcub::DeviceRadixSort::SortPairs(temp2.p, b1, key.as<unsigned long long>(),
                                              key_s.as<unsigned long long>(), nd2.as<double>(),
                                              d2_s.as<double>(), int(cnt), 0, 64, s));
    HIPCHK(hipcub::DeviceReduce::ReduceByKey(temp2.p, b2, key_s.as<unsigned long long>(),
                                             uniq.as<unsigned long long>(), d2_s.as<double>(),
                                             d2u.as<double>(), nruns.as<int>(), hipcub::Min(),
                                             int(cnt), s));
    int runs = 0;
    HIPCHK(hipMemcpyAsync(&runs, nruns.p, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    // weights, dropping underflowed ones
    DevMem keep, pos, wtmp, temp3, total;
    HIPCHK(keep.alloc(size_t(runs + 1) * 4, s));
    HIPCHK(pos.alloc(size_t(runs + 1) * 4, s));
    HIPCHK(wtmp.alloc(size_t(runs + 1) * 8, s));
    hipLaunchKernelGGL(k_weights, dim3(flat_grid(runs)), dim3(kBlock), 0, s, int64_t(runs),
                       uniq.as<unsigned long long>(), d2u.as<double>(), phi, keep.as<int>(),
                       wtmp.as<double>());
    size_t b3 = 0;
    HIPCHK(hipcub::DeviceScan::ExclusiveSum(nullptr, b3, keep.as<int>(), pos.as<int>(), runs, s));
    HIPCHK(temp3.alloc(b3, s));
    HIPCHK(hipcub::DeviceScan::ExclusiveSum(temp3.p, b3, keep.as<int>(), pos.as<int>(), runs, s));
    int hp[2] = {0, 0};
    if (runs > 0) {
        HIPCHK(hipMemcpyAsync(&hp[0], pos.as<int>() + runs - 1, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&hp[1], keep.as<int>() + runs - 1, 4, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    m_out = runs > 0 ? int64_t(hp[0]) + hp[1] : 0;
    if (m_out > m_cap) {
        err = "m_cap too small for the k-NN graph";
        return CCM_E_CAPACITY;
    }
    if (runs > 0)
        hipLaunchKernelGGL(k_emit, dim3(flat_grid(runs)), dim3(kBlock), 0, s, int64_t(runs),
                           uniq.as<unsigned long long>(), wtmp.as<double>(), keep.as<int>(),
                           pos.as<int>(), src, dst, w);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return CCM_OK;
}

}  // namespace ccm
