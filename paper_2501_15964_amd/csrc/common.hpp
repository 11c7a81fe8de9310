// Shared device helpers for the CCM kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ccm {

constexpr int kBlock = 256;          // threads per workgroup for all row kernels
constexpr int kWaves = kBlock / 64;  // waves per workgroup
constexpr int kMaxGrid = 2048;       // cap on grid-stride grids (partials per kernel)
// doubles in a partials buffer: two kernels of kMaxGrid blocks, up to 8 values each
constexpr int kPartialsCap = 2 * kMaxGrid * 8;

// Radius below which an l2 dual ball (q = 2) is taken as {0}: the projection
// is 0 and its Jacobian 0.  The Newton payload carries 1/r and the matvec
// a/r^2 (a <= 1), both finite for r >= 2^-500; r = gamma w falls below it when
// a Gaussian weight of a far neighbour underflows, and the exact projection
// differs from 0 by less than r there.
constexpr double kTinyRadius = 0x1p-500;

// q selector for the per-edge norm ||.||_q; the dual ball is in the q* norm.
enum QKind : int { kQ1 = 1, kQ2 = 2, kQInf = 3 };

// Sum over the LPR consecutive lanes of a row group with an xor butterfly.
// Every lane of the group ends with the bit-identical total (IEEE addition
// is commutative, and each butterfly stage adds the same pair of values).
template <int LPR>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int LPR>
__device__ __forceinline__ double group_max(double v) {
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

template <int LPR>
__device__ __forceinline__ int group_sum_i(int v) {
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic block reduction of NV per-thread values; thread v < NV of
// the block writes the block total of value v to out[v].
template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&v)[NV], double* out) {
    __shared__ double red[kWaves][NV > 0 ? NV : 1];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int s = 0; s < NV; ++s) {
        double x = v[s];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) red[wave][s] = x;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) t += red[w][threadIdx.x];
        out[threadIdx.x] = t;
    }
}

// Deterministic sums of K partials arrays (array i: count[i] entries with
// stride nv[i], starting at ptr[i]), computed identically by every block
// that calls it: thread t adds entries t, t + 64 WAVES, ... in order, then a
// fixed xor butterfly inside the wave and the waves in order.  All K sums
// share one pass of loads and one pair of barriers.  The block must have
// exactly WAVES waves; the results are returned to every thread.
template <int K, int WAVES = kWaves>
__device__ __forceinline__ void block_sums(const double* const (&ptr)[K], const int (&count)[K],
                                           const int (&nv)[K], double (&out)[K]) {
    __shared__ double red[WAVES][K];
    double x[K];
    int maxc = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        x[i] = 0.0;
        maxc = count[i] > maxc ? count[i] : maxc;
    }
    // the K arrays are read in the same loop so their loads overlap
    for (int p = threadIdx.x; p < maxc; p += WAVES * 64) {
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (p < count[i]) x[i] += ptr[i][p * nv[i]];
    }
#pragma unroll
    for (int i = 0; i < K; ++i) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x[i] += __shfl_xor(x[i], off, 64);
    }
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < K; ++i) red[wave][i] = x[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < K; ++i) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) t += red[w][i];
        out[i] = t;
    }
}

// Sum of one partials array (count entries with stride nv, component c).
__device__ __forceinline__ double block_sum_partials(const double* partials, int count, int nv,
                                                     int c) {
    const double* ptr[1] = {partials + c};
    const int cnt[1] = {count};
    const int st[1] = {nv};
    double out[1];
    block_sums<1>(ptr, cnt, st, out);
    return out[0];
}

// Incidence entry of the vertex-major (CSR) layout: e >= 0 means the vertex is
// the first endpoint of edge e (sign +1), e < 0 means it is the second
// endpoint of edge ~e (sign -1); o is the other endpoint.
struct Inc {
    int e;
    int o;
};

}  // namespace ccm
