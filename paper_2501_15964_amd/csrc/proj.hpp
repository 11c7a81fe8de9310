// Projection of one edge row onto its dual ball, shared by the edge-parallel
// kernels and the fused vertex kernel.  The ball of edge l is
// {||u||_{q*} <= r} with r = gamma w_l (q* the dual exponent of q).
#pragma once
#include "common.hpp"

namespace ccm {

// Per-edge projection of y (held in registers, NPER values per lane) onto
// the dual ball of radius r, with the Jacobian payload.
template <int LPR, int NPER, int Q>
struct RowProj {
    double pi[NPER];
    double alpha = 1.0;    // q = 2
    int cnt = -1;          // q = inf
    uint32_t lm = 0;       // this lane's masks: bit t for coordinate gl + LPR t
                           // (q = 1: |y_k| <= r; q = inf: k in support),
                           // bit 16 + t: y_k < 0 (q = inf)
};

template <int LPR, int NPER, int Q, bool BITS>
__device__ __forceinline__ void project_row(const double (&y)[NPER], int gl, int lane, int d,
                                            double r, RowProj<LPR, NPER, Q>& o) {
    if constexpr (Q == kQ2) {
        // l2 ball: scale y by min(1, r / ||y||); the boundary counts as inside
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < NPER; ++t) s += y[t] * y[t];
        s = group_sum<LPR>(s);
        const double nrm = sqrt(s);
        if (!(r >= kTinyRadius)) {
            o.alpha = 0.0;
#pragma unroll
            for (int t = 0; t < NPER; ++t) o.pi[t] = 0.0;
        } else if (nrm > r) {
            const double a = r / nrm;
            o.alpha = a;
#pragma unroll
            for (int t = 0; t < NPER; ++t) o.pi[t] = y[t] * a;
        } else {
            o.alpha = 1.0;
#pragma unroll
            for (int t = 0; t < NPER; ++t) o.pi[t] = y[t];
        }
    } else if constexpr (Q == kQ1) {
        // l_inf ball (box): clamp each coordinate to [-r, r]
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            o.pi[t] = fmin(fmax(y[t], -r), r);
            if constexpr (BITS) {
                const bool valid = gl + LPR * t < d;
                if (valid && fabs(y[t]) <= r) o.lm |= 1u << t;
            }
        }
    } else {
        // l1 ball by support pruning (Michelot 1986): theta from the current
        // support, drop coordinates with |y_k| <= theta, repeat until the
        // support is stable; then Pi_k = sign(y_k) (|y_k| - theta)_+.
        double v[NPER];
        double s = 0.0;
        int c = 0;
#pragma unroll
        for (int t = 0; t < NPER; ++t) {
            v[t] = fabs(y[t]);
            s += v[t];
            c += (gl + LPR * t < d) ? 1 : 0;
        }
        s = group_sum<LPR>(s);
        if (s <= r) {
            o.cnt = -1;
#pragma unroll
            for (int t = 0; t < NPER; ++t) {
                o.pi[t] = y[t];
            }
        } else if (!(r > 0.0)) {
            o.cnt = 0;
#pragma unroll
            for (int t = 0; t < NPER; ++t) {
                o.pi[t] = 0.0;
            }
        } else {
            int cc = group_sum_i<LPR>(c);
            double theta = (s - r) / double(cc);
            for (int it = 0; it <= d; ++it) {
                double s2 = 0.0;
                int c2 = 0;
#pragma unroll
                for (int t = 0; t < NPER; ++t) {
                    if (v[t] > theta) { s2 += v[t]; ++c2; }
                }
                s2 = group_sum<LPR>(s2);
                c2 = group_sum_i<LPR>(c2);
                if (c2 == cc) break;
                if (c2 == 0) {
                    // r is below the rounding resolution of max |y_k|: the
                    // projection rounds to 0 (theta = max |y_k|, P = 0)
                    double vm = 0.0;
#pragma unroll
                    for (int t = 0; t < NPER; ++t) vm = fmax(vm, v[t]);
                    theta = group_max<LPR>(vm);
                    cc = 0;
                    break;
                }
                cc = c2;
                theta = (s2 - r) / double(c2);
            }
            o.cnt = cc;
#pragma unroll
            for (int t = 0; t < NPER; ++t) {
                const double mag = fmax(v[t] - theta, 0.0);
                o.pi[t] = copysign(mag, y[t]);
                if constexpr (BITS) {
                    const bool valid = gl + LPR * t < d;
                    if (valid && v[t] > theta) o.lm |= 1u << t;
                    if (valid && y[t] < 0.0) o.lm |= 1u << (16 + t);
                }
            }
        }
    }
}

}  // namespace ccm
