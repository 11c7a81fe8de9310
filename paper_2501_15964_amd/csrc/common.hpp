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

// Bits of this lane's row group inside a wave-wide ballot, in lane order.
template <int LPR>
__device__ __forceinline__ uint64_t group_bits(uint64_t ballot, int lane) {
    if constexpr (LPR == 64) {
        return ballot;
    } else {
        const int base = (lane / LPR) * LPR;
        return (ballot >> base) & ((uint64_t(1) << LPR) - 1);
    }
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

// Deterministic sum of a partials array (count entries with stride nv,
// component c), computed identically by every block that calls it.  Uses
// the whole block; the result is returned to every thread.
__device__ __forceinline__ double block_sum_partials(const double* partials, int count, int nv,
                                                     int c) {
    __shared__ double red[kWaves];
    double x = 0.0;
    for (int p = threadIdx.x; p < count; p += blockDim.x) x += partials[p * nv + c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = x;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) t += red[w];
    return t;
}

// Incidence entry of the vertex-major (CSR) layout: e >= 0 means the vertex is
// the first endpoint of edge e (sign +1), e < 0 means it is the second
// endpoint of edge ~e (sign -1); o is the other endpoint.
struct Inc {
    int e;
    int o;
};

}  // namespace ccm
