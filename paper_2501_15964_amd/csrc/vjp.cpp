// Vector-Jacobian product of the solution map X*(A, w, gamma) for q = 2.
//
// With clusters c fixed (labels from a tight forward solve) the adjoint
// system in cluster space is
//   (diag(|c|) (x) I + B_c^T H B_c) lambda = g,   g_c = sum_{i in c} dL/dx_i,
// solved by Jacobi-preconditioned CG (preconditioner 1 / |c|).  The operator
// is applied without forming B_c: expand lambda to the vertices, apply the
// vertex Newton matvec with the curvature H_l of every inter-cluster edge
// (intra-cluster differences vanish), and sum the result over each cluster
// with the membership lists.  Then dL/da_i = lambda_{c(i)},
// dL/dlog w_l = -gamma w_l <lambda_ci - lambda_cj, ghat_l>, and
// dL/dgamma = -sum_l w_l <lambda_ci - lambda_cj, ghat_l>.
#include <algorithm>
#include <cmath>
#include <string>
#include "vjp.hpp"

#include <cmath>

namespace ccm {

#define HIPCHK(expr)                                                      \
    do {                                                                  \
        hipError_t e_ = (expr);                                           \
        if (e_ != hipSuccess) {                                           \
            err = std::string(#expr) + ": " + hipGetErrorString(e_);      \
            return e_ == hipErrorOutOfMemory ? CCM_E_NOMEM : CCM_E_HIP;   \
        }                                                                 \
    } while (0)

namespace {

struct Dot {
    DevMem part, res;
    double* h = nullptr;
    ~Dot() {
        if (h) (void)hipHostFree(h);
    }
};

}  // namespace

ccm_status path_vjp(const double* A, int64_t n, int d, const int* src, const int* dst,
                    const double* w, int64_t m, double gamma, const double* X, const int* labels,
                    const double* dLdX, double* dLdA, double* dLdlogw, double* dLdgamma,
                    double tol, int maxit, int* iters_out, hipStream_t s, std::string& err) {
    (void)A;
    OwnedGraph og;
    ccm_status st = graph_build(src, dst, w, m, n, d, true, s, og, err);
    if (st != CCM_OK) return st;
    // cluster count from the labels (must be 0 .. K-1)
    DevMem range;
    HIPCHK(range.alloc(8, s));
    {
        int init[2] = {0x7fffffff, -1};
        HIPCHK(hipMemcpyAsync(range.p, init, 8, hipMemcpyHostToDevice, s));
        launch_label_range(n, labels, range.as<int>(), s);
        int h[2];
        HIPCHK(hipMemcpyAsync(h, range.p, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (h[0] < 0 || h[1] >= n) {
            err = "labels must lie in [0, n)";
            return CCM_E_INVALID;
        }
        const int64_t K = int64_t(h[1]) + 1;
        OwnedGraph cg;
        st = membership_build(labels, n, K, d, s, cg, err);
        if (st != CCM_OK) return st;
        const int64_t NK = K * d, NV = n * d;
        DevMem ipay, Pi, rhs, x, r, z, p, q, pv, ov, minv, part, sc;
        HIPCHK(ipay.alloc(size_t(std::max<int64_t>(og.g.nent, 1)) * 16, s));
        HIPCHK(Pi.alloc(size_t(std::max<int64_t>(m, 1)) * d * 8, s));
        for (DevMem* b : {&rhs, &x, &r, &z, &p, &q}) HIPCHK(b->alloc(size_t(NK) * 8, s));
        HIPCHK(pv.alloc(size_t(NV) * 8, s));
        HIPCHK(ov.alloc(size_t(NV) * 8, s));
        HIPCHK(minv.alloc(size_t(K) * 8, s));
        HIPCHK(part.alloc(std::max(partials_for(og.g), partials_for(cg.g)) * 8, s));
        HIPCHK(sc.alloc(8 * 8, s));
        double* hs = nullptr;
        HIPCHK(hipHostMalloc((void**)&hs, 8 * 8, hipHostMallocDefault));
        struct HostFree {
            double* p;
            ~HostFree() { (void)hipHostFree(p); }
        } hf{hs};
        auto dot = [&](const double* a, const double* b, int64_t N, double& out) -> ccm_status {
            const int gp = launch_dot(a, b, N, part.as<double>(), s);
            launch_finalize(part.as<double>(), gp, 1, sc.as<double>(), s);
            HIPCHK(hipMemcpyAsync(hs, sc.p, 8, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            out = hs[0];
            return CCM_OK;
        };
        Payload pl{ipay.as<double2>(), nullptr};
        launch_adj_payload(og.g, d, X, labels, gamma, ipay.as<double2>(), Pi.as<double>(), s);
        launch_inv_sizes(K, cg.g.inc_ptr, minv.as<double>(), s);
        // g_c = sum over members of dL/dx
        launch_scatter(cg.g, d, kQ2, 0.0, nullptr, 0.0, nullptr, 1.0, dLdX, rhs.as<double>(),
                       false, Payload{}, 0.0, 0.0, nullptr, part.as<double>(), s);
        auto apply = [&](const double* in, double* out) {
            launch_expand(n, d, labels, in, pv.as<double>(), s);
            launch_matvec(og.g, d, kQ2, 2, pv.as<double>(), Pi.as<double>(), pl, gamma, 1.0, 1.0,
                          nullptr, ov.as<double>(), part.as<double>(), CgSkip{}, s);
            launch_scatter(cg.g, d, kQ2, 0.0, nullptr, 0.0, nullptr, 1.0, ov.as<double>(), out,
                           false, Payload{}, 0.0, 0.0, nullptr, part.as<double>(), s);
        };
        // PCG from lambda = 0
        double bb = 0;
        if ((st = dot(rhs.as<double>(), rhs.as<double>(), NK, bb)) != CCM_OK) return st;
        launch_fill(x.as<double>(), NK, 0.0, s);
        launch_copy(rhs.as<double>(), r.as<double>(), NK, s);
        launch_rowscale(r.as<double>(), minv.as<double>(), z.as<double>(), K, d, s);
        launch_copy(z.as<double>(), p.as<double>(), NK, s);
        double rz = 0;
        if ((st = dot(r.as<double>(), z.as<double>(), NK, rz)) != CCM_OK) return st;
        int it = 0;
        const double thr = tol * tol * bb;
        double rr = bb;
        while (it < maxit && rr > thr && bb > 0) {
            apply(p.as<double>(), q.as<double>());
            double pq = 0;
            if ((st = dot(p.as<double>(), q.as<double>(), NK, pq)) != CCM_OK) return st;
            if (!(pq > 0)) break;
            const double a = rz / pq;
            launch_axpy(x.as<double>(), a, p.as<double>(), NK, s);
            launch_axpy(r.as<double>(), -a, q.as<double>(), NK, s);
            ++it;
            if ((st = dot(r.as<double>(), r.as<double>(), NK, rr)) != CCM_OK) return st;
            if (rr <= thr) break;
            launch_rowscale(r.as<double>(), minv.as<double>(), z.as<double>(), K, d, s);
            double rz2 = 0;
            if ((st = dot(r.as<double>(), z.as<double>(), NK, rz2)) != CCM_OK) return st;
            launch_axpby(1.0, z.as<double>(), rz2 / rz, p.as<double>(), p.as<double>(), NK, s);
            rz = rz2;
        }
        if (iters_out) *iters_out = it;
        // a CG that stopped short of the tolerance (iteration cap or a
        // breakdown) still writes the gradients of its last iterate, but the
        // call reports it
        const bool short_stop = bb > 0 && !(rr <= thr);
        // gradients
        launch_expand(n, d, labels, x.as<double>(), dLdA, s);
        DevMem dlw;
        double* dlogw = dLdlogw;
        if (!dlogw) {
            HIPCHK(dlw.alloc(size_t(std::max<int64_t>(m, 1)) * 8, s));
            dlogw = dlw.as<double>();
        }
        double dg = 0.0;
        if (m > 0) {
            const int gp = launch_adj_edge(og.g, d, X, labels, x.as<double>(), gamma, dlogw,
                                           part.as<double>(), s);
            launch_finalize(part.as<double>(), gp, 1, sc.as<double>(), s);
            HIPCHK(hipMemcpyAsync(hs, sc.p, 8, hipMemcpyDeviceToHost, s));
        }
        HIPCHK(hipStreamSynchronize(s));
        if (m > 0) dg = -hs[0];
        if (dLdgamma) *dLdgamma = dg;
        HIPCHK(hipGetLastError());
        if (short_stop) {
            err = "adjoint CG stopped after " + std::to_string(it) +
                  " iterations above its tolerance (relative residual " +
                  std::to_string(std::sqrt(rr / bb)) + ")";
            return CCM_E_NOT_CONVERGED;
        }
    }
    return CCM_OK;
}

}  // namespace ccm
