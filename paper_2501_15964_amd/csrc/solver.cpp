// Host drivers of the path solvers: SSNAL (semismooth Newton augmented
// Lagrangian), ADMM and fast AMA for the convex clustering model, warm-started
// along a gamma sequence.  Every arithmetic step runs in the HIP kernels; the
// host only sequences launches and reads back a handful of FP64 scalars
// (objective pieces, residual norms, CG status) to take control decisions.
#include "solver.hpp"

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

namespace ccm {

namespace {

#define HIPCHK(expr)                                                      \
    do {                                                                  \
        hipError_t e_ = (expr);                                           \
        if (e_ != hipSuccess) {                                           \
            err = std::string(#expr) + ": " + hipGetErrorString(e_);      \
            return e_ == hipErrorOutOfMemory ? CCM_E_NOMEM : CCM_E_HIP;   \
        }                                                                 \
    } while (0)

#define CHK(expr)                              \
    do {                                       \
        ccm_status st_ = (expr);               \
        if (st_ != CCM_OK) return st_;         \
    } while (0)

using Clock = std::chrono::steady_clock;

// scalar slots in the device/host scalar block
enum Slot {
    kE = 0,    // edge pass at the current point (5)
    kS = 5,    // scatter at the current point (4)
    kT = 9,    // trial axpy (2)
    kET = 11,  // edge pass at the trial point (5)
    kST = 16,  // scatter at the trial point (4)
    kK = 20,   // KKT edge pass (6)
    kM = 26,   // misc (ADMM residuals, dots) (8)
    kNA = 34,  // ||A||^2
    kSP = 35,  // data spread S
    kNS = 40
};

// HIP-event timing of kernel classes (ccm_options.profile)
struct Prof {
    bool on = false;
    bool matvec_only = false;   // time only the Newton/CG matvec class,
    int sample = 1;             // every sample-th launch of it
    int64_t seen = 0;
    bool last_recorded = false;
    hipStream_t s = nullptr;
    std::vector<hipEvent_t> ev;
    std::vector<int> cls;
    std::vector<double> pbytes;  // algorithmic bytes of each timed launch
    size_t used = 0;
    double ms[CCM_NK] = {0};
    int64_t calls[CCM_NK] = {0};
    double bytes[CCM_NK] = {0};
    int open_cls = -1;
    double open_bytes = 0;
    ~Prof() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
    void begin(int c, double b) {
        last_recorded = false;
        if (!on || (matvec_only && c != CCM_K_MATVEC)) return;
        if (matvec_only && (seen++ % sample) != 0) return;
        if (used + 2 > ev.size()) {
            for (int k = 0; k < 64; ++k) {
                hipEvent_t e;
                if (hipEventCreate(&e) == hipSuccess) ev.push_back(e);
            }
            cls.resize(ev.size() / 2 + 1);
            pbytes.resize(ev.size() / 2 + 1);
        }
        if (used + 2 > ev.size()) return;
        (void)hipEventRecord(ev[used], s);
        open_cls = c;
        open_bytes = b;
    }
    void end() {
        if (!on || open_cls < 0) return;
        (void)hipEventRecord(ev[used + 1], s);
        cls[used / 2] = open_cls;
        pbytes[used / 2] = open_bytes;
        used += 2;
        open_cls = -1;
        last_recorded = true;
    }
    // Pairs carry ids base + local index, so they can be reclassified or
    // harvested while later pairs are still in flight.
    size_t base = 0;
    int64_t last_pair() const {
        return on && last_recorded && used >= 2 ? int64_t(base + used / 2) - 1 : -1;
    }
    int64_t next_pair() const { return int64_t(base + used / 2); }
    void reclass(int64_t id, int c) {
        if (!on || id < int64_t(base)) return;
        const size_t loc = size_t(id) - base;
        if (loc < used / 2) cls[loc] = c;
    }
    // algorithmic bytes of a recorded launch, known only after it was issued
    void set_bytes(int64_t id, double b) {
        if (!on || id < int64_t(base)) return;
        const size_t loc = size_t(id) - base;
        if (loc < used / 2) pbytes[loc] = b;
    }
    // accumulate the pairs with id < id_end (their events have completed)
    void harvest_until(int64_t id_end) {
        if (!on) return;
        const size_t have = used / 2;
        const size_t np =
            std::min(have, size_t(std::max<int64_t>(0, id_end - int64_t(base))));
        for (size_t k = 0; k < np; ++k) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, ev[2 * k], ev[2 * k + 1]) == hipSuccess) {
                ms[cls[k]] += t;
                calls[cls[k]] += 1;
                bytes[cls[k]] += pbytes[k];
            }
        }
        const size_t rem = have - np;
        for (size_t r = 0; r < rem; ++r) {
            std::swap(ev[2 * r], ev[2 * (np + r)]);
            std::swap(ev[2 * r + 1], ev[2 * (np + r) + 1]);
            cls[r] = cls[np + r];
            pbytes[r] = pbytes[np + r];
        }
        used = rem * 2;
        base += np;
    }
    // after a stream synchronisation: accumulate every recorded pair
    void harvest() { harvest_until(next_pair()); }
    void take(ccm_stats& st) {
        for (int c = 0; c < CCM_NK; ++c) {
            st.kern_ms[c] = ms[c];
            st.kern_calls[c] = calls[c];
            ms[c] = 0;
            calls[c] = 0;
        }
        // algorithmic bytes of exactly the matvec launches that were timed
        st.matvec_bytes = bytes[CCM_K_MATVEC];
        st.matvec_launches = st.kern_calls[CCM_K_MATVEC];
        for (double& b : bytes) b = 0;
    }
};

struct Timed {
    Prof& p;
    Timed(Prof& pr, int c, double bytes = 0.0) : p(pr) { p.begin(c, bytes); }
    ~Timed() { p.end(); }
};

struct Ev {
    double phi = 0, gn = 0, rp = 0;
    double G2 = 0, hx = 0, aBtPi = 0, BtPi2 = 0;
    double bxpi = 0, pu2 = 0, bx2 = 0, pi2 = 0, nout = 0;
};

}  // namespace

struct Solver::Impl {
    // problem
    const DevGraph& g;
    int d;
    int64_t n, m, N, M;
    int qk;
    const double* A;
    hipStream_t s;
    ccm_options o;
    double tol;
    std::string& err;
    Prof prof;
    Clock::time_point t_start;

    // vertex buffers
    DevMem bX, bXt, bG, bGt, bDinv, bDinvt, bTmp, bTmp2;
    DevMem cgx, cgr, cgu, cgw, cgp, cgs;
    // edge buffers
    DevMem bU, bPi, bPit, bZ, bL, bQ, bZold, bLa;
    DevMem ip0, ip1, lb0, lb1;  // Jacobian payload (current, trial)
    int cg_pred[2] = {8, 8};    // predicted CG iterations (Newton, Laplacian systems)
    DevMem fused, parent, rank, ltemp;
    size_t ltemp_bytes = 0;
    // reductions
    DevMem pe, pet, ps, pst, pt, pk, pm, pm2, pupd0, pupd1, pwu0, pwu1, cgstate, cgflag,
        spread_work;
    double* hs = nullptr;          // scalar slots (host view)
    double* dslot = nullptr;       // the same slots as the kernels address them
    hipEvent_t sync_ev = nullptr;  // progress marker of the solver's stream
    int* hflag = nullptr;          // [0..1] status, [4..5] second pending chunk
    hipEvent_t cg_ev[2] = {nullptr, nullptr};
    CgBufs cg{};

    double *X = nullptr, *Xt = nullptr, *G = nullptr, *Gt = nullptr, *Dinv = nullptr,
           *Dinvt = nullptr, *U = nullptr, *Pi = nullptr, *Pit = nullptr;
    Payload pl{}, plt{};
    double nA = 0, spread = 0;
    bool have_U = false;  // U holds a multiplier (else zero)
    double sigma = 0;
    // ADMM state validity
    bool admm_state = false;
    double last_bytes = 0;      // algorithmic bytes of one Newton matvec at the current state
    // batched mode
    const BatchSpec* batch = nullptr;
    double floor_scale = 1.0;               // inner gradient floor relative to tol
    std::vector<double> nA_inst;            // ||A|| per segment
    std::vector<std::array<double, 7>> inst_res;
    DevMem vrows, erows, vsum, esum, vthr;

    Impl(const DevGraph& graph, int d_, int qk_, const double* A_, hipStream_t s_,
         const ccm_options& opt, double tol_, std::string& e)
        : g(graph), d(d_), n(graph.n), m(graph.m), N(graph.n * d_), M(graph.m * d_), qk(qk_),
          A(A_), s(s_), o(opt), tol(tol_), err(e) {
        prof.on = o.profile != 0;
        prof.matvec_only = o.profile == 2;
        prof.sample = o.profile == 2 ? 4 : 1;
        prof.s = s;
    }
    ~Impl() {
        if (hs) (void)hipHostFree(hs);
        if (hflag) (void)hipHostFree(hflag);
        for (auto e : cg_ev)
            if (e) (void)hipEventDestroy(e);
        if (sync_ev) (void)hipEventDestroy(sync_ev);
    }

    ccm_status alloc() {
        const size_t vb = size_t(N) * 8, eb = size_t(M) * 8;
        for (DevMem* b : {&bX, &bXt, &bG, &bGt, &bDinv, &bDinvt, &bTmp, &bTmp2, &cgx, &cgr, &cgu,
                          &cgw, &cgp, &cgs})
            HIPCHK(b->alloc(vb, s));
        HIPCHK(bU.alloc(eb, s));
        if (o.method == CCM_SSNAL) {
            HIPCHK(bPi.alloc(eb, s));
            HIPCHK(bPit.alloc(eb, s));
            const size_t ne = size_t(std::max<int64_t>(g.nent, 1));
            if (qk != kQ1) {
                HIPCHK(ip0.alloc(ne * 16, s));
                HIPCHK(ip1.alloc(ne * 16, s));
            }
            if (qk != kQ2) {
                const size_t lw = size_t(std::max<int64_t>(m, 1)) * lbits_per_edge(d);
                HIPCHK(lb0.alloc(lw * 4, s));
                HIPCHK(lb1.alloc(lw * 4, s));
            }
        } else if (o.method == CCM_ADMM || o.method == CCM_HPR) {
            HIPCHK(bZ.alloc(eb, s));
            HIPCHK(bL.alloc(eb, s));
            HIPCHK(bQ.alloc(eb, s));
            HIPCHK(bZold.alloc(eb, s));  // HPR: the anchor's Z
            if (o.method == CCM_HPR) HIPCHK(bLa.alloc(eb, s));
        } else {
            HIPCHK(bZ.alloc(eb, s));  // momentum point V
        }
        HIPCHK(fused.alloc(std::max<int64_t>(m, 1) * 4, s));
        HIPCHK(parent.alloc(n * 4, s));
        HIPCHK(rank.alloc((n + 1) * 4, s));
        ltemp_bytes = labels_temp_bytes(n);
        HIPCHK(ltemp.alloc(ltemp_bytes, s));
        const size_t pb = partials_for(g) * 8;
        for (DevMem* b : {&pe, &pet, &ps, &pst, &pt, &pk, &pm, &pm2, &pupd0, &pupd1, &pwu0, &pwu1})
            HIPCHK(b->alloc(pb, s));
        HIPCHK(cgstate.alloc(8 * 8, s));
        HIPCHK(cgflag.alloc(8 * 4, s));
        HIPCHK(spread_work.alloc(size_t(spread_work_size(n, d)) * 8, s));
        // scalar slots: coherent pinned host memory that the reduction kernels
        // write directly, so a read needs no copy, only the stream's progress
        HIPCHK(hipHostMalloc((void**)&hs, kNS * 8, hipHostMallocCoherent | hipHostMallocMapped));
        std::memset(hs, 0, kNS * 8);
        HIPCHK(hipHostGetDevicePointer((void**)&dslot, hs, 0));
        HIPCHK(hipHostMalloc((void**)&hflag, 8 * 4, hipHostMallocDefault));
        for (auto& e : cg_ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&sync_ev, hipEventDisableTiming));
        X = bX.as<double>();
        Xt = bXt.as<double>();
        G = bG.as<double>();
        Gt = bGt.as<double>();
        Dinv = bDinv.as<double>();
        Dinvt = bDinvt.as<double>();
        U = bU.as<double>();
        Pi = bPi.as<double>();
        Pit = bPit.as<double>();
        pl = Payload{ip0.as<double2>(), lb0.as<uint32_t>()};
        plt = Payload{ip1.as<double2>(), lb1.as<uint32_t>()};
        cg.x = cgx.as<double>();
        cg.r = cgr.as<double>();
        cg.u = cgu.as<double>();
        cg.w = cgw.as<double>();
        cg.p = cgp.as<double>();
        cg.s = cgs.as<double>();
        cg.upd[0] = pupd0.as<double>();
        cg.upd[1] = pupd1.as<double>();
        cg.wu[0] = pwu0.as<double>();
        cg.wu[1] = pwu1.as<double>();
        cg.state = cgstate.as<double>();
        cg.flag = cgflag.as<int>();
        cg.nparts = cg_update_grid(N);
        return CCM_OK;
    }

    // Wait until event e has passed by polling it: a blocking wait sleeps and
    // wakes up tens of microseconds after the device is done.
    ccm_status spin(hipEvent_t e) {
        hipError_t r;
        while ((r = hipEventQuery(e)) == hipErrorNotReady) {
        }
        HIPCHK(r);
        return CCM_OK;
    }
    // wait for the scalar slots written so far (the range [a, b) documents
    // what the caller reads) and accumulate the profiling events recorded so
    // far, unless harvest is false
    ccm_status read(int a, int b, bool harvest = true) {
        (void)a;
        (void)b;
        CHK(read_begin());
        return read_wait(harvest);
    }
    // The same in two halves: work enqueued between them runs on the device
    // while the host waits for, and then acts on, the values.
    int64_t read_pid = 0;
    ccm_status read_begin() {
        flush_finalize();
        HIPCHK(hipEventRecord(sync_ev, s));
        read_pid = prof.next_pair();
        return CCM_OK;
    }
    ccm_status read_wait(bool harvest = true) {
        CHK(spin(sync_ev));
        if (harvest) prof.harvest_until(read_pid);
        return CCM_OK;
    }
    // The next Newton step's CG start (x = 0, r = -G, the first matvec) needs
    // nothing the host decides, so it is enqueued right after a read that
    // opens an outer iteration; the host fills in the CG threshold before the
    // first update.  Unused if the iteration takes no Newton step.
    bool cg_pre = false;
    int64_t cg_pre_pair = -1;
    void cg_prestart(double gamma) {
        cg_begin(0, G, true, Dinv, 0.0, gamma, Pi, pl);
        cg_pre_pair = prof.last_pair();
        cg_pre = true;
    }
    double* slot(int k) { return dslot + k; }

    // Reductions of per-block partials into scalar slots are deferred to the
    // next read, which runs all of them in one launch.  A partials buffer with
    // a pending reduction is not rewritten before that read except by another
    // producer for the same slots (whose reduction then replaces it).
    FinalizeJobs fin{};
    int nfin = 0;
    void defer_finalize(const double* part, int count, int nv, double* out, hipStream_t) {
        for (int i = 0; i < nfin; ++i) {
            if (fin.j[i].out == out) {
                fin.j[i] = FinalizeJob{part, count, nv, out};
                return;
            }
        }
        if (nfin == kMaxFinalizeJobs) flush_finalize();
        fin.j[nfin++] = FinalizeJob{part, count, nv, out};
    }
    void flush_finalize() {
        launch_finalize_multi(fin, nfin, s);
        nfin = 0;
    }

    // SSNAL path continuation (ccm_options.dual_scale): before a new gamma,
    // the multiplier rows on the boundary of the previous gamma's balls are
    // moved to the new radii
    void continue_dual(double g_prev, double g_new) {
        const bool on = o.dual_scale > 0 || (o.dual_scale < 0 && qk == kQ2);
        if (!on || !have_U || M == 0 || !(g_prev > 0.0) || !(g_new > 0.0) || g_new == g_prev)
            return;
        launch_scale_boundary(m, d, qk, g.w, g_prev, g_new / g_prev, U, s);
    }

    bool out_of_time() const {
        if (!(o.time_budget_s > 0)) return false;
        const double el = std::chrono::duration<double>(Clock::now() - t_start).count();
        return el > o.time_budget_s;
    }

    // ---- set-up --------------------------------------------------------------
    ccm_status setup(const double* Xw, const double* Uw) {
        CHK(alloc());
        // ||A||^2 and the data spread S (label threshold)
        {
            const int gp = launch_dot(A, A, N, pm.as<double>(), s);
            defer_finalize(pm.as<double>(), gp, 1, slot(kNA), s);
            launch_spread(A, n, d, spread_work.as<double>(), slot(kSP), s);
            CHK(read(kNA, kSP + 1));
            nA = std::sqrt(hs[kNA]);
            spread = hs[kSP];
        }
        if (Xw) HIPCHK(hipMemcpyAsync(X, Xw, size_t(N) * 8, hipMemcpyDeviceToDevice, s));
        else HIPCHK(hipMemcpyAsync(X, A, size_t(N) * 8, hipMemcpyDeviceToDevice, s));
        if (Uw) {
            HIPCHK(hipMemcpyAsync(U, Uw, size_t(M) * 8, hipMemcpyDeviceToDevice, s));
            have_U = true;
        } else {
            launch_fill(U, M, 0.0, s);
            have_U = false;
        }
        return CCM_OK;
    }

    // ---- shared pieces -------------------------------------------------------
    // The SSNAL edge pass (Pi, payload, merit terms) and the gradient G with
    // the Jacobi diagonal.  q = 1, 2, and q = inf on rows of more than 256
    // values: one vertex-centric launch in which both endpoints of an edge
    // project its row.  q = inf on shorter rows: the edge-parallel pass then
    // the vertex scatter, since there its l1-ball projection (an iteration)
    // costs more twice than Pi's extra read.
    void edge_grad(const double* Xc, double* Pic, Payload p, double gamma, double* Gc, double* Dc,
                   double* epart, double* spart, int eslot, int sslot) {
        Timed t(prof, CCM_K_EDGE);
        if (qk != kQInf || d > 256) {
            const int gp = launch_edge_grad(g, d, qk, gamma, sigma, Xc, U, A, Pic, p, Gc, Dc,
                                            epart, spart, s);
            defer_finalize(epart, gp, kEdgeSsnalNV, slot(eslot), s);
            defer_finalize(spart, gp, kScatterNV, slot(sslot), s);
            return;
        }
        const int ge = launch_edge_ssnal(g, d, qk, gamma, sigma, Xc, U, Pic, p, epart, s);
        defer_finalize(epart, ge, kEdgeSsnalNV, slot(eslot), s);
        const int gs = launch_scatter(g, d, qk, 1.0, Xc, -1.0, A, 1.0, Pic, Gc, true, p, gamma,
                                      sigma, Dc, spart, s);
        defer_finalize(spart, gs, kScatterNV, slot(sslot), s);
    }
    Ev make_ev(int e, int sc) const {
        Ev v;
        v.bxpi = hs[e + 0];
        v.pu2 = hs[e + 1];
        v.bx2 = hs[e + 2];
        v.pi2 = hs[e + 3];
        v.nout = hs[e + 4];
        v.G2 = hs[sc + 0];
        v.hx = hs[sc + 1];
        v.aBtPi = hs[sc + 2];
        v.BtPi2 = hs[sc + 3];
        // phi = 1/2||X-A||^2 + <BX, Pi> - ||Pi - U||^2 / (2 sigma)
        v.phi = v.hx + v.bxpi - v.pu2 / (2.0 * sigma);
        v.gn = std::sqrt(v.G2) / (1.0 + nA);
        v.rp = std::sqrt(v.pu2) / (sigma * (1.0 + std::sqrt(v.bx2) + std::sqrt(v.pi2)));
        return v;
    }

    double lap_bytes() const {
        // ADMM matrix I + sigma B^T B: read V, write out, incidence entries
        // and their vertex ids
        return 16.0 * double(N) + 12.0 * double(g.nent);
    }
    double matvec_bytes(double nout) const {
        // one-pass minimum traffic of a Newton matvec launch: read V, write
        // out, the incidence entries with their vertex ids, and the Jacobian
        // payload: per-incidence scalars, lane masks, and the rows of Pi of
        // the edges whose Jacobian is not the identity (q = 2)
        double b = 16.0 * double(N) + 12.0 * double(g.nent);
        if (qk == kQ2) b += 16.0 * double(g.nent) + nout * 8.0 * d;
        else if (qk == kQ1) b += double(m) * lbits_per_edge(d) * 4.0;
        else b += 16.0 * double(g.nent) + nout * lbits_per_edge(d) * 4.0;
        return b;
    }

    // ---- Jacobi-preconditioned CG ------------------------------------------------
    // Solve M x = b (M = I + sigma B^T P B for mode 0, I + sigma B^T B for
    // mode 1) from x = 0; result in cg.x.  Iterations are enqueued in chunks;
    // each launch issued after convergence returns at once (device-side flag)
    // and is timed as "other".  The host waits for chunk k's status only after
    // chunk k + 1 is enqueued, so its decision overlaps device work.  The first
    // chunk is sized from the previous solve's iteration count (consecutive
    // Newton systems need similar counts), later ones are half a chunk.
    struct CgPending {
        int j0 = 0, j1 = 0;
        int64_t pid_end = 0;
        std::vector<int64_t> upd, mv;
        int* hf = nullptr;
        hipEvent_t e = nullptr;
    };
    struct CgRun {
        int mode = 0;
        const double* Dv = nullptr;
        double thr = 0, gamma = 0;
        const double* Pic = nullptr;
        Payload p{};
        double mv_bytes = 0;
        int j = 0;  // iterations enqueued
        CgPending P[2];
    } cr;

    int cg_first(int mode) const {
        const int chunk = std::max(1, o.cg_chunk);
        return std::max(2, std::min(2 * chunk, cg_pred[mode & 1]));
    }
    int cg_later() const { return std::max(2, std::max(1, o.cg_chunk) / 2); }

    // x = 0, r = b (negated if neg), the preconditioned residual and its matvec
    void cg_begin(int mode, const double* b, bool neg, const double* Dv, double thr,
                  double gamma, const double* Pic, Payload p) {
        cr.mode = mode;
        cr.Dv = Dv;
        cr.thr = thr;
        cr.gamma = gamma;
        cr.Pic = Pic;
        cr.p = p;
        cr.mv_bytes = mode == 0 ? last_bytes : lap_bytes();
        cr.j = 0;
        cr.P[0].hf = hflag;
        cr.P[1].hf = hflag + 4;
        cr.P[0].e = cg_ev[0];
        cr.P[1].e = cg_ev[1];
        {
            Timed t(prof, CCM_K_CGUPDATE);
            launch_cg_init(N, b, neg, Dv, cg, s);
        }
        {
            Timed t(prof, CCM_K_MATVEC, cr.mv_bytes);
            cg.nparts_mv = launch_matvec(g, d, qk, mode, cg.u, Pic, p, gamma, sigma, 1.0, nullptr,
                                         cg.w, cg.wu[0], CgSkip{}, s);
        }
    }

    // enqueue `count` iterations, then a copy of the status flag to q.hf
    ccm_status cg_issue(CgPending& q, int count) {
        q.j0 = cr.j;
        q.upd.clear();
        q.mv.clear();
        for (int c = 0; c < count && cr.j < o.cg_max_iter; ++c, ++cr.j) {
            const int j = cr.j;
            {
                Timed t(prof, CCM_K_CGUPDATE);
                launch_cg_update(N, j, cr.Dv, cg, cr.thr, s);
            }
            q.upd.push_back(prof.last_pair());
            {
                Timed t(prof, CCM_K_MATVEC, cr.mv_bytes);
                CgSkip sk;
                sk.rr_partials = cg.upd[(j + 1) & 1];
                sk.nparts = cg.nparts;
                sk.thr = cr.thr;
                sk.done = cg.flag;
                launch_matvec(g, d, qk, cr.mode, cg.u, cr.Pic, cr.p, cr.gamma, sigma, 1.0, nullptr,
                              cg.w, cg.wu[(j + 1) & 1], sk, s);
            }
            q.mv.push_back(prof.last_pair());
        }
        q.j1 = cr.j;
        HIPCHK(hipMemcpyAsync(q.hf, cg.flag, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(q.e, s));
        q.pid_end = prof.next_pair();
        return CCM_OK;
    }

    // launches of q issued at or after convergence (iteration done_at)
    void cg_reclass(const CgPending& q, int done_at) {
        for (size_t c = 0; c < q.upd.size(); ++c) {
            const int jj = q.j0 + int(c);
            if (jj >= done_at) prof.reclass(q.upd[c], CCM_K_OTHER);
            if (jj + 1 >= done_at) prof.reclass(q.mv[c], CCM_K_OTHER);
        }
    }

    // P[cur] is enqueued with its status not yet seen: wait for convergence or
    // the iteration cap; iters = iterations taken
    ccm_status cg_wait(int cur, int& iters) {
        bool done = false;
        int done_at = 0;
        while (true) {
            const bool more = cr.j < o.cg_max_iter;
            if (more) CHK(cg_issue(cr.P[cur ^ 1], cg_later()));
            CHK(spin(cr.P[cur].e));
            const CgPending& q = cr.P[cur];
            if (q.hf[0]) {
                done = true;
                done_at = q.hf[1];
                cg_reclass(q, done_at);
                if (more) cg_reclass(cr.P[cur ^ 1], 0);
            }
            prof.harvest_until(q.pid_end);
            if (done || !more) break;
            cur ^= 1;
        }
        iters = done ? done_at : cr.j;
        cg_pred[cr.mode & 1] = iters + 1;
        return CCM_OK;
    }

    ccm_status cg_solve(int mode, const double* b, bool neg, const double* Dv, double thr,
                        double gamma, const double* Pic, Payload p, int& iters) {
        cg_begin(mode, b, neg, Dv, thr, gamma, Pic, p);
        CHK(cg_issue(cr.P[0], cg_first(mode)));
        return cg_wait(0, iters);
    }

    // ---- KKT of (X, Uc) with Uc feasible up to rounding -------------------------
    // scalars: scatter at (X, Uc) in kS.., KKT edge pass in kK..
    ccm_status kkt_of(const double* Uc, double gamma, double* Gout, double (&res)[7]) {
        {
            Timed t(prof, CCM_K_SCATTER);
            const int gp = launch_scatter(g, d, qk, 1.0, X, -1.0, A, 1.0, Uc, Gout, false, Payload{},
                                          gamma, sigma, nullptr, ps.as<double>(), s);
            defer_finalize(ps.as<double>(), gp, kScatterNV, slot(kS), s);
        }
        {
            Timed t(prof, CCM_K_EDGE);
            const int gp = launch_edge_kkt(g, d, qk, gamma, X, Uc, nullptr, pk.as<double>(), s);
            defer_finalize(pk.as<double>(), gp, kEdgeKktNV, slot(kK), s);
        }
        CHK(read(kS, kK + kEdgeKktNV));
        kkt_from_slots(res);
        return CCM_OK;
    }
    // residuals with the scatter values of `ev` (taken at (X, U)) and the KKT
    // edge pass in the kK slots
    void kkt_from(const Ev& ev, double (&res)[7]) {
        const double nbx = std::sqrt(hs[kK + 1]), nu = std::sqrt(hs[kK + 2]);
        const double RD = ev.gn;
        const double RC = std::sqrt(hs[kK + 0]) / (1.0 + nbx + nu);
        const double RU = std::sqrt(hs[kK + 3]) / (1.0 + nu);
        const double fp = ev.hx + hs[kK + 4];
        const double fd = ev.aBtPi - 0.5 * ev.BtPi2;
        const double eta = std::fabs(fp - fd) / (1.0 + std::fabs(fp) + std::fabs(fd));
        res[0] = RD;
        res[1] = RC;
        res[2] = RU;
        res[3] = eta;
        res[4] = fp;
        res[5] = fd;
        res[6] = std::max(RD, std::max(RC, RU));
    }
    void kkt_from_slots(double (&res)[7]) {
        const double RD = std::sqrt(hs[kS]) / (1.0 + nA);
        const double nbx = std::sqrt(hs[kK + 1]), nu = std::sqrt(hs[kK + 2]);
        const double RC = std::sqrt(hs[kK + 0]) / (1.0 + nbx + nu);
        const double RU = std::sqrt(hs[kK + 3]) / (1.0 + nu);
        const double fp = hs[kS + 1] + hs[kK + 4];
        const double fd = hs[kS + 2] - 0.5 * hs[kS + 3];
        const double eta = std::fabs(fp - fd) / (1.0 + std::fabs(fp) + std::fabs(fd));
        res[0] = RD;
        res[1] = RC;
        res[2] = RU;
        res[3] = eta;
        res[4] = fp;
        res[5] = fd;
        res[6] = std::max(RD, std::max(RC, RU));
    }

    // ---- SSNAL at one gamma ------------------------------------------------------
    // trial point Xt = X + alpha D with its edge pass and gradient (no wait)
    void trial_eval(double alpha, double gamma) {
        {
            Timed tt(prof, CCM_K_OTHER);
            const int gp = launch_trial(N, X, cg.x, alpha, A, G, Xt, pt.as<double>(), s);
            defer_finalize(pt.as<double>(), gp, kAxpyNV, slot(kT), s);
        }
        // with the gradient at the trial point (used if accepted)
        edge_grad(Xt, Pit, plt, gamma, Gt, Dinvt, pet.as<double>(), pst.as<double>(), kET, kST);
    }

    ccm_status ssnal(double gamma, int& status, ccm_stats& st, double (&res)[7]) {
        const double mu = 1e-4, ls_slack = 1e-14;
        // first trial step of a line search: for q = 1 and inf twice the last
        // accepted step, at most 1 (their semismooth steps are often halved
        // several times in a row); for q = 2 always the full step
        double a0 = 1.0;
        // inner Newton stop: gradient norm below this fraction of R_P (q = inf
        // takes a looser inner solve and a slower penalty growth, below)
        const double inner = qk == kQInf ? 0.5 : 0.2;
        double rp_prev = INFINITY;
        status = CCM_MAX_ITER;
        bool numerical = false;
        // values of the first outer iteration's merit function; later ones are
        // enqueued with the KKT pass of the iteration before
        edge_grad(X, Pi, pl, gamma, G, Dinv, pe.as<double>(), ps.as<double>(), kE, kS);
        CHK(read_begin());
        cg_prestart(gamma);
        CHK(read_wait());
        Ev ev = make_ev(kE, kS);
        for (int k = 0; k < o.max_outer; ++k) {
            st.outer++;
            last_bytes = matvec_bytes(ev.nout);
            for (int it = 0; it < o.max_newton; ++it) {
                if (!std::isfinite(ev.phi) || !std::isfinite(ev.gn)) {
                    numerical = true;
                    break;
                }
                if (ev.gn <= std::max(0.5 * tol * floor_scale, inner * ev.rp)) break;
                if (out_of_time()) {
                    status = CCM_TIMEOUT;
                    return CCM_OK;
                }
                // Newton direction: (I + sigma B^T P B) D = -G.  The first
                // chunk of CG iterations (three more than the last solve took:
                // a launch returning at once costs far less than a miss)
                // and the full-step trial are enqueued together; the trial's
                // read also brings the CG status, and only if the CG needs more
                // iterations is it continued and the trial redone.
                const double rtol = std::min(0.1, std::pow(ev.gn, 0.2));
                const double thr = rtol * rtol * ev.G2;
                int iters = 0;
                if (cg_pre) {
                    cr.thr = thr;
                    cr.mv_bytes = last_bytes;
                    prof.set_bytes(cg_pre_pair, last_bytes);
                    cg_pre = false;
                } else {
                    cg_begin(0, G, true, Dinv, thr, gamma, Pi, pl);
                }
                CHK(cg_issue(cr.P[0], cg_first(0) + 2));
                trial_eval(a0, gamma);
                CHK(read(kT, kST + kScatterNV, false));
                if (cr.P[0].hf[0]) {
                    iters = cr.P[0].hf[1];
                    cg_reclass(cr.P[0], iters);
                    cg_pred[0] = iters + 1;
                    prof.harvest();
                } else if (cr.j >= o.cg_max_iter) {
                    iters = cr.j;
                    cg_pred[0] = iters + 1;
                    prof.harvest();
                } else {
                    prof.harvest();
                    CHK(cg_issue(cr.P[1], cg_later()));
                    CHK(cg_wait(1, iters));
                    trial_eval(a0, gamma);
                    CHK(read(kT, kST + kScatterNV));
                }
                st.cg += iters;
                st.newton++;
                // Armijo backtracking on phi
                double alpha = a0;
                bool accepted = false;
                Ev evt;
                for (int t = 0; t < 40; ++t) {
                    st.linesearch++;
                    if (t > 0) {
                        trial_eval(alpha, gamma);
                        CHK(read(kT, kST + kScatterNV));
                    }
                    double slope = hs[kT + 1];
                    if (t == 0 && !(slope < 0.0)) {
                        // not a descent direction: fall back to steepest descent
                        launch_axpby(-1.0, G, 0.0, G, cg.x, N, s);
                        alpha = 1.0;
                        trial_eval(alpha, gamma);
                        CHK(read(kT, kST + kScatterNV));
                        slope = hs[kT + 1];
                    }
                    evt = make_ev(kET, kST);
                    const double slack = ls_slack * (1.0 + std::fabs(ev.phi));
                    if (evt.phi <= ev.phi + mu * alpha * slope + slack) {
                        accepted = true;
                        break;
                    }
                    alpha *= 0.5;
                }
                (void)accepted;  // after 40 halvings the last (tiny) step is taken
                if (qk != kQ2) a0 = std::min(1.0, 2.0 * alpha);
                std::swap(X, Xt);
                std::swap(Pi, Pit);
                std::swap(pl, plt);
                std::swap(G, Gt);
                std::swap(Dinv, Dinvt);
                ev = evt;
                last_bytes = matvec_bytes(ev.nout);
                cg_pre = false;
            }
            if (numerical) break;
            // multiplier update U <- Pi_C(U + sigma B X), already in Pi
            std::swap(U, Pi);
            have_U = true;
            // penalty of the next outer iteration: doubled when the primal
            // residual fell by less than a factor (2 for q = 2, whose Newton
            // systems stay well conditioned as sigma grows; 1/0.9 for q = 1
            // and 1/0.95 for q = inf, where a faster growth multiplies the CG
            // iterations)
            const double sigma_cur = sigma;
            const double stall = qk == kQ2 ? 0.5 : qk == kQ1 ? 0.9 : 0.95;
            if (k >= 1 && ev.rp > stall * rp_prev) sigma = std::min(o.sigma_max, 2.0 * sigma);
            rp_prev = ev.rp;
            // KKT at (X, U): R_D from the last gradient, the rest from one pass;
            // the next outer iteration's edge pass and gradient are enqueued
            // with it (discarded if this one converges)
            const bool next = k + 1 < o.max_outer;
            // Rows of more than 256 values: one launch, the KKT terms from the
            // next pass's edge rows (saves reading X and U again; at these
            // widths the kernel runs at its lowest occupancy either way, while
            // for shorter rows the extra terms cost occupancy and time)
            if (next && qk != kQInf && d > 256) {
                Timed t(prof, CCM_K_EDGE);
                const int gp = launch_edge_grad(g, d, qk, gamma, sigma, X, U, A, Pi, pl, G, Dinv,
                                                pe.as<double>(), ps.as<double>(), s,
                                                pk.as<double>());
                defer_finalize(pe.as<double>(), gp, kEdgeSsnalNV, slot(kE), s);
                defer_finalize(ps.as<double>(), gp, kScatterNV, slot(kS), s);
                defer_finalize(pk.as<double>(), gp, kEdgeKktNV, slot(kK), s);
            } else {
                {
                    Timed t(prof, CCM_K_EDGE);
                    const int gp =
                        launch_edge_kkt(g, d, qk, gamma, X, U, nullptr, pk.as<double>(), s);
                    defer_finalize(pk.as<double>(), gp, kEdgeKktNV, slot(kK), s);
                }
                if (next)
                    edge_grad(X, Pi, pl, gamma, G, Dinv, pe.as<double>(), ps.as<double>(), kE, kS);
            }
            CHK(read_begin());
            if (next) cg_prestart(gamma);
            CHK(read_wait());
            kkt_from(ev, res);
            if (!std::isfinite(res[6])) {
                numerical = true;
                break;
            }
            double crit = res[6];
            if (batch) {
                CHK(batch_kkt(gamma));
                crit = 0.0;
                for (const auto& r : inst_res) crit = std::max(crit, r[6]);
                if (!std::isfinite(crit)) {
                    numerical = true;
                    break;
                }
            }
            if (crit <= tol) {
                sigma = sigma_cur;
                status = CCM_CONVERGED;
                break;
            }
            if (out_of_time()) {
                sigma = sigma_cur;
                status = CCM_TIMEOUT;
                break;
            }
            if (next) ev = make_ev(kE, kS);
        }
        if (numerical) status = CCM_NUMERICAL;
        return CCM_OK;
    }

    // ---- ADMM at one gamma -------------------------------------------------------
    ccm_status admm(double gamma, int& status, ccm_stats& st, double (&res)[7]) {
        const int ce = std::max(1, o.check_every);
        const int balance = 50;
        double* Z = bZ.as<double>();
        double* L = bL.as<double>();
        double* Q = bQ.as<double>();
        double* R = bTmp.as<double>();
        double* T = bTmp2.as<double>();
        status = CCM_MAX_ITER;
        if (!admm_state) {
            // cold start: Z = B X, L = 0
            launch_gather(g, d, X, Z, s);
            launch_fill(L, M, 0.0, s);
            admm_state = true;
        }
        launch_axpby(sigma, Z, -1.0, L, Q, M, s);
        launch_lap_dinv(g, d, 1.0, sigma, Dinv, s);
        const double thr_abs = 0.01 * tol * (1.0 + nA);
        for (int it = 1; it <= o.max_iter; ++it) {
            st.outer++;
            {
                Timed t(prof, CCM_K_SCATTER);
                launch_scatter(g, d, qk, 0.0, nullptr, 1.0, A, 1.0, Q, R, false, Payload{}, gamma,
                               sigma, nullptr, ps.as<double>(), s);
            }
            {
                Timed t(prof, CCM_K_MATVEC, lap_bytes());
                launch_matvec(g, d, qk, 1, X, nullptr, Payload{}, gamma, sigma, 1.0, nullptr, T,
                              pm2.as<double>(), CgSkip{}, s);
            }
            launch_sub(R, T, R, N, s);  // residual of the warm start
            int iters = 0;
            CHK(cg_solve(1, R, false, Dinv, thr_abs * thr_abs, gamma, nullptr, Payload{}, iters));
            st.cg += iters;
            launch_axpy(X, 1.0, cg.x, N, s);
            const bool check = (it % ce) == 0;
            const bool bal = (it % balance) == 0;
            if (bal) launch_copy(Z, bZold.as<double>(), M, s);
            {
                Timed t(prof, CCM_K_EDGE);
                const int gp = launch_edge_admm(g, d, qk, gamma, sigma, o.tau, X, Z, L, Q,
                                                check ? U : nullptr, pe.as<double>(), s);
                defer_finalize(pe.as<double>(), gp, kEdgeAdmmNV, slot(kM), s);
            }
            if (check) {
                CHK(kkt_of(U, gamma, G, res));
                if (!std::isfinite(res[6])) {
                    status = CCM_NUMERICAL;
                    break;
                }
                if (res[6] <= tol) {
                    status = CCM_CONVERGED;
                    break;
                }
                if (out_of_time()) {
                    status = CCM_TIMEOUT;
                    break;
                }
            }
            if (bal) {
                launch_sub(Z, bZold.as<double>(), bZold.as<double>(), M, s);
                const int gp = launch_scatter(g, d, qk, 0.0, nullptr, 0.0, nullptr, 1.0,
                                              bZold.as<double>(), T, false, Payload{}, gamma,
                                              sigma, nullptr, pm2.as<double>(), s);
                defer_finalize(pm2.as<double>(), gp, kScatterNV, slot(kM + 4), s);
                CHK(read(kM, kM + 8));
                const double rp = std::sqrt(hs[kM + 0]);
                const double rd = sigma * std::sqrt(hs[kM + 4]);
                double ns = sigma;
                if (rp > 10.0 * rd) ns = 2.0 * sigma;
                else if (rd > 10.0 * rp) ns = 0.5 * sigma;
                if (ns != sigma) {
                    sigma = ns;
                    launch_axpby(sigma, Z, -1.0, L, Q, M, s);
                    launch_lap_dinv(g, d, 1.0, sigma, Dinv, s);
                }
            }
        }
        if (status != CCM_CONVERGED) CHK(kkt_last_admm(gamma, res));
        return CCM_OK;
    }
    // ---- Halpern-Peaceman-Rachford at one gamma --------------------------------
    // The Peaceman-Rachford step of ADMM's splitting (exact X solve by CG as
    // in ADMM, reflection H = 2 BX - Z, multiplier Pi_C(sigma H + L)) inside
    // Halpern's iteration anchored at (Za, La); every check_every iterations
    // the KKT test at (X, Lh) and the anchor restart test on the fixed-point
    // residual R = (sigma ||Z - Zh||^2 + ||L - Lh||^2 / sigma)^(1/2):
    // restart when R fell below 0.2 of its anchor value, below 0.8 of it
    // while rising, or when the anchor is older than 0.2 of the iterations;
    // at a restart sigma becomes ||L - La|| / ||Z - Za|| within a factor 10
    // of the old value.  The state (Z, L, sigma) is carried to the next gamma.
    ccm_status hpr(double gamma, int& status, ccm_stats& st, double (&res)[7]) {
        const int ce = std::max(1, o.check_every);
        double* Z = bZ.as<double>();
        double* L = bL.as<double>();
        double* Q = bQ.as<double>();
        double* Za = bZold.as<double>();
        double* La = bLa.as<double>();
        double* R = bTmp.as<double>();
        double* T = bTmp2.as<double>();
        status = CCM_MAX_ITER;
        if (!admm_state) {
            launch_gather(g, d, X, Z, s);
            launch_fill(L, M, 0.0, s);
            admm_state = true;
        }
        launch_axpby(sigma, Z, -1.0, L, Q, M, s);
        launch_lap_dinv(g, d, 1.0, sigma, Dinv, s);
        launch_copy(Z, Za, M, s);
        launch_copy(L, La, M, s);
        const double thr_abs = 0.01 * tol * (1.0 + nA);
        int k = 0;
        double R_anchor = -1.0, R_prev = -1.0;
        for (int it = 1; it <= o.max_iter; ++it) {
            st.outer++;
            {
                Timed t(prof, CCM_K_SCATTER);
                launch_scatter(g, d, qk, 0.0, nullptr, 1.0, A, 1.0, Q, R, false, Payload{}, gamma,
                               sigma, nullptr, ps.as<double>(), s);
            }
            {
                Timed t(prof, CCM_K_MATVEC, lap_bytes());
                launch_matvec(g, d, qk, 1, X, nullptr, Payload{}, gamma, sigma, 1.0, nullptr, T,
                              pm2.as<double>(), CgSkip{}, s);
            }
            launch_sub(R, T, R, N, s);
            int iters = 0;
            CHK(cg_solve(1, R, false, Dinv, thr_abs * thr_abs, gamma, nullptr, Payload{}, iters));
            st.cg += iters;
            launch_axpy(X, 1.0, cg.x, N, s);
            const bool check = (it % ce) == 0;
            {
                Timed t(prof, CCM_K_EDGE);
                const double a = 1.0 / (double(k) + 2.0);
                const int gp = launch_edge_hpr(g, d, qk, gamma, sigma, a, X, Z, L, Za, La, Q,
                                               check ? U : nullptr, pe.as<double>(), s);
                defer_finalize(pe.as<double>(), gp, kEdgeHprNV, slot(kM), s);
            }
            ++k;
            if (!check) continue;
            CHK(kkt_of(U, gamma, G, res));
            if (!std::isfinite(res[6])) {
                status = CCM_NUMERICAL;
                break;
            }
            if (res[6] <= tol) {
                status = CCM_CONVERGED;
                break;
            }
            if (out_of_time()) {
                status = CCM_TIMEOUT;
                break;
            }
            const double dz2 = hs[kM + 0], dl2 = hs[kM + 1];
            const double mz = std::sqrt(hs[kM + 2]), ml = std::sqrt(hs[kM + 3]);
            const double Rk = std::sqrt(sigma * dz2 + dl2 / sigma);
            if (R_anchor < 0.0) {
                R_anchor = Rk;
            } else if (Rk <= 0.2 * R_anchor || (Rk <= 0.8 * R_anchor && R_prev >= 0.0 &&
                                                Rk > R_prev) ||
                       double(k) >= 0.2 * double(it)) {
                launch_copy(Z, Za, M, s);
                launch_copy(L, La, M, s);
                k = 0;
                double ns = sigma;
                if (mz > 0.0 && ml > 0.0) ns = std::min(std::max(ml / mz, 0.1 * sigma), 10.0 * sigma);
                if (ns != sigma) {
                    sigma = ns;
                    launch_axpby(sigma, Z, -1.0, L, Q, M, s);
                    launch_lap_dinv(g, d, 1.0, sigma, Dinv, s);
                }
                R_anchor = std::sqrt(sigma * dz2 + dl2 / sigma);
                R_prev = -1.0;
                continue;
            }
            R_prev = Rk;
        }
        if (status != CCM_CONVERGED) CHK(kkt_last_admm(gamma, res));
        return CCM_OK;
    }

    ccm_status kkt_last_admm(double gamma, double (&res)[7]) {
        // U <- Pi_C(L) through the KKT edge pass with U = L (writes Pi_C(L))
        {
            Timed t(prof, CCM_K_EDGE);
            const int gp = launch_edge_kkt(g, d, qk, gamma, X, bL.as<double>(), U,
                                           pk.as<double>(), s);
            defer_finalize(pk.as<double>(), gp, kEdgeKktNV, slot(kK), s);
        }
        return kkt_of(U, gamma, G, res);
    }

    // ---- fast AMA at one gamma ----------------------------------------------------
    ccm_status ama(double gamma, int& status, ccm_stats& st, double (&res)[7]) {
        const int ce = std::max(1, o.check_every);
        double* V = bZ.as<double>();
        status = CCM_MAX_ITER;
        // U is projected onto the new (larger) balls first, V = U
        launch_edge_kkt(g, d, qk, gamma, X, U, V, pk.as<double>(), s);
        launch_copy(V, U, M, s);
        const double nu = 1.0 / (2.0 * double(std::max(1, g.max_deg)));
        double t = 1.0;
        bool restart_next = true;
        for (int it = 1; it <= o.max_iter; ++it) {
            st.outer++;
            // X = A - B^T V
            {
                Timed tt(prof, CCM_K_SCATTER);
                launch_scatter(g, d, qk, 0.0, nullptr, 1.0, A, -1.0, V, X, false, Payload{},
                               gamma, sigma, nullptr, ps.as<double>(), s);
            }
            double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
            double beta = restart_next ? 0.0 : (t - 1.0) / tn;
            {
                Timed tt(prof, CCM_K_EDGE);
                const int gp = launch_edge_ama(g, d, qk, gamma, nu, beta, X, U, V, pe.as<double>(),
                                               s);
                defer_finalize(pe.as<double>(), gp, kEdgeAmaNV, slot(kM), s);
            }
            CHK(read(kM, kM + 2));
            if (hs[kM + 0] > 0.0) {
                // momentum points uphill: restart from the new point
                launch_copy(U, V, M, s);
                t = 1.0;
                restart_next = false;
            } else {
                t = restart_next ? 1.0 : tn;
                restart_next = false;
            }
            if ((it % ce) == 0) {
                // X = A - B^T U for the test
                launch_scatter(g, d, qk, 0.0, nullptr, 1.0, A, -1.0, U, X, false, Payload{},
                               gamma, sigma, nullptr, ps.as<double>(), s);
                CHK(kkt_of(U, gamma, G, res));
                if (!std::isfinite(res[6])) {
                    status = CCM_NUMERICAL;
                    break;
                }
                if (res[6] <= tol) {
                    status = CCM_CONVERGED;
                    break;
                }
                if (out_of_time()) {
                    status = CCM_TIMEOUT;
                    break;
                }
            }
        }
        if (status != CCM_CONVERGED) {
            launch_scatter(g, d, qk, 0.0, nullptr, 1.0, A, -1.0, U, X, false, Payload{}, gamma,
                           sigma, nullptr, ps.as<double>(), s);
            CHK(kkt_of(U, gamma, G, res));
        }
        return CCM_OK;
    }

    // per-segment KKT residuals of (X, U), each with the segment's own norms
    ccm_status batch_kkt(double gamma) {
        const BatchSpec& b = *batch;
        const int S = b.S;
        if (!vrows.p) {
            HIPCHK(vrows.alloc(size_t(n) * kScatterNV * 8, s));
            HIPCHK(erows.alloc(size_t(std::max<int64_t>(m, 1)) * 5 * 8, s));
            HIPCHK(vsum.alloc(size_t(S) * kScatterNV * 8, s));
            HIPCHK(esum.alloc(size_t(S) * 5 * 8, s));
        }
        {
            Timed t(prof, CCM_K_SCATTER);
            launch_scatter(g, d, qk, 1.0, X, -1.0, A, 1.0, U, bTmp.as<double>(), false, Payload{},
                           gamma, sigma, nullptr, ps.as<double>(), s, vrows.as<double>());
        }
        {
            Timed t(prof, CCM_K_EDGE);
            if (m > 0)
                launch_edge_kkt(g, d, qk, gamma, X, U, nullptr, pk.as<double>(), s,
                                erows.as<double>());
        }
        launch_segsum(vrows.as<double>(), kScatterNV, b.vseg_dev, S, vsum.as<double>(), s);
        std::vector<double> hv(size_t(S) * kScatterNV), he(size_t(S) * 5, 0.0);
        if (m > 0) {
            launch_segsum(erows.as<double>(), 5, b.eseg_dev, S, esum.as<double>(), s);
            HIPCHK(hipMemcpyAsync(he.data(), esum.p, he.size() * 8, hipMemcpyDeviceToHost, s));
        }
        HIPCHK(hipMemcpyAsync(hv.data(), vsum.p, hv.size() * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        prof.harvest();
        inst_res.assign(S, {0, 0, 0, 0, 0, 0, 0});
        for (int i = 0; i < S; ++i) {
            const double* v = &hv[size_t(i) * kScatterNV];
            const double* e = &he[size_t(i) * 5];
            const double RD = std::sqrt(v[0]) / (1.0 + nA_inst[i]);
            const double nbx = std::sqrt(e[1]), nu = std::sqrt(e[2]);
            const double RC = std::sqrt(e[0]) / (1.0 + nbx + nu);
            const double RU = std::sqrt(e[3]) / (1.0 + nu);
            const double fp = v[1] + e[4];
            const double fd = v[2] - 0.5 * v[3];
            const double eta = std::fabs(fp - fd) / (1.0 + std::fabs(fp) + std::fabs(fd));
            inst_res[i] = {RD, RC, RU, eta, fp, fd, std::max(RD, std::max(RC, RU))};
        }
        return CCM_OK;
    }

    ccm_status labels(int* lab_out, int* nclus_host) {
        Timed t(prof, CCM_K_OTHER);
        const double thr = 1e-5 * (1.0 + spread);
        // batched: each instance's own threshold (from its own spread)
        if (m > 0)
            launch_fused_flags(g, d, X, thr, fused.as<int>(), s, nullptr,
                               batch ? vthr.as<double>() : nullptr);
        int* lab = lab_out;
        DevMem scratch;
        if (!lab) {
            HIPCHK(scratch.alloc(n * 4, s));
            lab = scratch.as<int>();
        }
        launch_labels(n, m, g.src, g.dst, fused.as<int>(), parent.as<int>(), rank.as<int>(),
                      ltemp.p, ltemp_bytes, lab, cgflag.as<int>() + 2, s, g.inc_ptr, g.inc, g.vord);
        HIPCHK(hipMemcpyAsync(hflag + 2, cgflag.as<int>() + 2, sizeof(int), hipMemcpyDeviceToHost,
                              s));
        HIPCHK(hipStreamSynchronize(s));
        prof.harvest();
        if (nclus_host) *nclus_host = hflag[2];
        return CCM_OK;
    }
};

Solver::Solver(const DevGraph& g, int d, int qk, const double* A, hipStream_t s,
               const ccm_options& o, double tol, std::string& err)
    : impl_(new Impl(g, d, qk, A, s, o, tol, err)) {}
Solver::~Solver() { delete impl_; }

ccm_status Solver::run_path(const double* gammas, int T, const double* Xw, const double* Uw,
                            double* X_out, double* U_out, int* labels_out, int* n_clusters,
                            double* kkt, int* status, ccm_stats* stats) {
    Impl& I = *impl_;
    std::string& err = I.err;
    I.t_start = Clock::now();
    CHK(I.setup(Xw, Uw));
    I.sigma = I.o.sigma0;
    for (int t = 0; t < T; ++t) {
        const double gamma = gammas[t];
        const auto t0 = Clock::now();
        ccm_stats st;
        std::memset(&st, 0, sizeof(st));
        int stat = CCM_CONVERGED;
        double res[7] = {0, 0, 0, 0, 0, 0, 0};
        if (gamma == 0.0 || I.m == 0) {
            // the model reduces to X = A (and U = 0 is a dual solution)
            HIPCHK(hipMemcpyAsync(I.X, I.A, size_t(I.N) * 8, hipMemcpyDeviceToDevice, I.s));
            launch_fill(I.U, I.M, 0.0, I.s);
            I.admm_state = false;
            // f_p = f_d = 0 and every residual is 0
        } else if (I.o.method == CCM_SSNAL) {
            // the penalty restarts at sigma0 for every gamma: a penalty grown
            // on one problem makes the next, more fused one ill-conditioned
            I.sigma = I.o.sigma0;
            if (t > 0) I.continue_dual(gammas[t - 1], gamma);
            CHK(I.ssnal(gamma, stat, st, res));
        } else if (I.o.method == CCM_ADMM) {
            CHK(I.admm(gamma, stat, st, res));
        } else if (I.o.method == CCM_HPR) {
            CHK(I.hpr(gamma, stat, st, res));
        } else {
            CHK(I.ama(gamma, stat, st, res));
        }
        if (X_out)
            HIPCHK(hipMemcpyAsync(X_out + size_t(t) * I.N, I.X, size_t(I.N) * 8,
                                  hipMemcpyDeviceToDevice, I.s));
        if (U_out && I.M > 0)
            HIPCHK(hipMemcpyAsync(U_out + size_t(t) * I.M, I.U, size_t(I.M) * 8,
                                  hipMemcpyDeviceToDevice, I.s));
        int nc = 0;
        CHK(I.labels(labels_out ? labels_out + size_t(t) * I.n : nullptr, &nc));
        if (n_clusters) n_clusters[t] = nc;
        if (kkt) {
            kkt[4 * t + 0] = res[0];
            kkt[4 * t + 1] = res[1];
            kkt[4 * t + 2] = res[2];
            kkt[4 * t + 3] = res[3];
        }
        if (status) status[t] = stat;
        st.seconds = std::chrono::duration<double>(Clock::now() - t0).count();
        st.f_p = res[4];
        st.f_d = res[5];
        st.sigma = I.sigma;
        I.prof.take(st);
        if (stats) stats[t] = st;
    }
    HIPCHK(hipStreamSynchronize(I.s));
    return CCM_OK;
}

ccm_status Solver::run_batched(const double* gammas, int T, const BatchSpec& b) {
    Impl& I = *impl_;
    std::string& err = I.err;
    I.t_start = Clock::now();
    I.batch = &b;
    CHK(I.setup(nullptr, nullptr));
    I.sigma = I.o.sigma0;
    const int S = b.S;
    // per-segment ||A||, and the inner gradient floor that makes the global
    // test imply every segment's R_D test
    {
        DevMem rn, sums;
        HIPCHK(rn.alloc(size_t(I.n) * 8, I.s));
        HIPCHK(sums.alloc(size_t(S) * 8, I.s));
        launch_row_sqnorm(I.A, I.n, I.d, rn.as<double>(), I.s);
        launch_segsum(rn.as<double>(), 1, b.vseg_dev, S, sums.as<double>(), I.s);
        std::vector<double> h(S);
        HIPCHK(hipMemcpyAsync(h.data(), sums.p, size_t(S) * 8, hipMemcpyDeviceToHost, I.s));
        HIPCHK(hipStreamSynchronize(I.s));
        I.nA_inst.resize(S);
        double mn = INFINITY;
        for (int i = 0; i < S; ++i) {
            I.nA_inst[i] = std::sqrt(h[i]);
            mn = std::min(mn, I.nA_inst[i]);
        }
        I.floor_scale = (1.0 + mn) / (1.0 + I.nA);
    }
    // per-vertex fusion thresholds from each instance's own spread
    {
        DevMem work;
        HIPCHK(work.alloc(size_t(seg_threshold_work_size(S, I.d)) * 8, I.s));
        HIPCHK(I.vthr.alloc(size_t(I.n) * 8, I.s));
        launch_seg_thresholds(I.A, b.vseg_dev, S, I.d, work.as<double>(), I.vthr.as<double>(),
                              I.s);
        HIPCHK(hipStreamSynchronize(I.s));
    }
    DevMem lab, firsts;
    HIPCHK(lab.alloc(size_t(I.n) * 4, I.s));
    HIPCHK(firsts.alloc(size_t(S) * 4, I.s));
    std::vector<int> hf(S);
    for (int t = 0; t < T; ++t) {
        const double gamma = gammas[t];
        ccm_stats st;
        std::memset(&st, 0, sizeof(st));
        int stat = CCM_CONVERGED;
        double res[7] = {0, 0, 0, 0, 0, 0, 0};
        if (gamma == 0.0 || I.m == 0) {
            HIPCHK(hipMemcpyAsync(I.X, I.A, size_t(I.N) * 8, hipMemcpyDeviceToDevice, I.s));
            launch_fill(I.U, I.M, 0.0, I.s);
            I.inst_res.assign(S, {0, 0, 0, 0, 0, 0, 0});
        } else {
            I.sigma = I.o.sigma0;
            if (t > 0) I.continue_dual(gammas[t - 1], gamma);
            CHK(I.ssnal(gamma, stat, st, res));
        }
        int ncl = 0;
        CHK(I.labels(lab.as<int>(), &ncl));
        launch_split(I.n, I.d, I.X, lab.as<int>(), b.vseg_dev, S, b.xoff_dev, b.loff_dev, t,
                     b.X_out_all, b.labels_all, I.s);
        launch_first_labels(lab.as<int>(), b.vseg_dev, S, firsts.as<int>(), I.s);
        HIPCHK(hipMemcpyAsync(hf.data(), firsts.p, size_t(S) * 4, hipMemcpyDeviceToHost, I.s));
        HIPCHK(hipStreamSynchronize(I.s));
        for (int i = 0; i < S; ++i) {
            const int gi = b.inst[i];
            const int next = (i + 1 < S) ? hf[i + 1] : ncl;
            if (b.n_clusters_host) b.n_clusters_host[size_t(gi) * T + t] = next - hf[i];
            const auto& r = I.inst_res[i];
            if (b.kkt_host)
                for (int c = 0; c < 4; ++c) b.kkt_host[(size_t(gi) * T + t) * 4 + c] = r[c];
            if (b.status_host) {
                int si = stat;
                if (r[6] <= I.tol && stat != CCM_NUMERICAL) si = CCM_CONVERGED;
                else if (stat == CCM_CONVERGED) si = CCM_MAX_ITER;
                b.status_host[size_t(gi) * T + t] = si;
            }
        }
        I.prof.take(st);
    }
    HIPCHK(hipStreamSynchronize(I.s));
    return CCM_OK;
}

}  // namespace ccm
