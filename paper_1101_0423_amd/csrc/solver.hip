// solver.hip -- the solve of D x = b through the even-odd factorisation of
// Eq. (10):
//   b' = S1 b,  b'' = b'_o - M5 D^OE b'_e,  C y = b'',  y_e = b'_e - M5 D^EO y_o,
//   x = S2 y,
// with the Schur system solved by CG (Algorithm 1) on C C^dag in the form
// that tracks y = C^dag w (so that r stays the residual of C y = b''), in a
// low precision (FP32, or FP16 storage with FP32 arithmetic), driven by the
// FP64 defect correction of Algorithm 2 and reliable updates (the search
// direction p is kept across restarts), with the automatic switch to defect
// correction when reliable updates stall (Sec. 2.3).
//
// One inner CG iteration is five fused stencil kernels plus two one-block
// reduction finishers (Secs. 3.2-3.5):
//   E: p = r + beta p;          t1 = M5^T g5 p            (odd)
//   A: t2 = M5^T D^EO t1                                    (even)
//   B: u  = p - g5 D^OE t2,     |u|^2 = (p, C C^dag p)     (odd)   -> alpha
//   C: t3 = M5 D^EO u                                       (even)
//   D: q  = u - M5 D^OE t3;  y += alpha u;  r -= alpha q;  |r|^2 (odd) -> beta
// alpha, beta and the convergence flags never leave the device; the host
// replays a captured hipGraph of several iterations and reads the state back
// between replays.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "dwf_ctx.h"

namespace dwf {

template <class F>
F fld(const HalfField& h);
template <class Real>
const Real* tab(const TableSet* ts, int t, int Ns);
template <class Real>
const Real* stab(const TableSet* ts, int t, int Ns);

double flops_per_iter(const dwf_ctx* c) {
    return (double)c->V5h * (5280.0 + 192.0 * c->Ns + 288.0);
}

static double spinor_bytes(int prec) { return prec == DWF_PREC_FP64 ? 192.0 : prec == DWF_PREC_FP32 ? 96.0 : 52.0; }
static double link_bytes(int fmt) { return fmt == LINK_D18 ? 144.0 : fmt == LINK_S18 ? 72.0 : fmt == LINK_S12 ? 48.0 : 24.0; }

double bytes_per_iter(const dwf_ctx* c, int inner_prec, int link_fmt) {
    const double sb = spinor_bytes(inner_prec);
    const double yb = inner_prec == DWF_PREC_FP64 ? 192.0 : 96.0;
    return (double)c->V5h * (15.0 * sb + 2.0 * yb) + 4.0 * (double)c->V4h * 8.0 * link_bytes(link_fmt);
}

namespace {

enum { B_E = 0, B_O, BP_E, BP_O, BPP, YH_E, YH_O, T64_E, NF64 };
enum { L_R = NF64, L_P, L_U, L_T1, L_T23, L_Y, NFALL };

struct HostState {
    std::vector<double> rr, aux;
    std::vector<int> live, iters, status;
};

template <class Real, class F, class FY, class LF>
struct Solver {
    dwf_ctx* c;
    const TableSet* ts;
    Workspace* w;
    LF lk[2];
    LinkD18 lk64[2];
    int nrhs;
    hipStream_t s;
    DevBuf* partials;
    int* mask_a;  // device int[nrhs]
    int* mask_b;
    const dwf_solve_params& p;

    Geom g64(int par) const { return c->geom(par, true); }
    Geom glo(int par) const { return c->geom(par, sizeof(Real) == 8); }
    FD d(int i) const { return w->f(i).fd(); }
    F lo(int i) const { return fld<F>(w->f(i)); }
    FY ylo() const { return fld<FY>(w->f(L_Y)); }
    const double* t64(int t) const { return tab<double>(ts, t, c->Ns); }
    const Real* tlo(int t) const { return tab<Real>(ts, t, c->Ns); }
    const double* s64(int t) const { return stab<double>(ts, t, c->Ns); }
    const Real* slo(int t) const { return stab<Real>(ts, t, c->Ns); }
    double* part() const { return partials->as<double>(); }
    KOpt kopt(const int* live, bool red) const { return KOpt{live, red ? part() : nullptr, nrhs, 0}; }

    // ---------------- FP64 pieces ----------------
    hipError_t local64(int par, int in, int table, int out) {
        return launch_dwf<double, FD, LinkD18, false, MIX_DENSE, ProLoad<FD>, EpiStore<FD>>(
            g64(par), d(in), lk64[par], t64(table), ProLoad<FD>{d(in)}, EpiStore<FD>{d(out)}, kopt(nullptr, false), s);
    }
    hipError_t norm64(int par, int in) {
        return launch_dwf<double, FD, LinkD18, false, MIX_NONE, ProLoad<FD>, EpiNorm>(
            g64(par), d(in), lk64[par], nullptr, ProLoad<FD>{d(in)}, EpiNorm{}, kopt(nullptr, true), s);
    }
    // out = a - M5 D^{par,1-par} in
    hipError_t xmy_m5hop64(int par, int in, int a, int out, bool red) {
        if (red)
            return launch_dwf<double, FD, LinkD18, true, MIX_SA, ProLoad<FD>, EpiLin<FD, FD, true, false>>(
                g64(par), d(in), lk64[par], s64(ST_M5), ProLoad<FD>{d(in)},
                EpiLin<FD, FD, true, false>{d(a), d(out), 1.0, -1.0}, kopt(nullptr, true), s);
        return launch_dwf<double, FD, LinkD18, true, MIX_SA, ProLoad<FD>, EpiLin<FD, FD, false, false>>(
            g64(par), d(in), lk64[par], s64(ST_M5), ProLoad<FD>{d(in)},
            EpiLin<FD, FD, false, false>{d(a), d(out), 1.0, -1.0}, kopt(nullptr, false), s);
    }
    hipError_t fin(int nblocks, int mode) { return launch_finish(part(), nblocks, nrhs, w->st, mode, s); }

    // rhat = b'' - C yhat_o  (FP64), r_lo = rhat, y_lo = 0, rr = aux = |rhat|^2
    hipError_t outer_residual() {
        hipError_t e = launch_dwf<double, FD, LinkD18, true, MIX_SA, ProLoad<FD>, EpiStore<FD>>(
            g64(0), d(YH_O), lk64[0], s64(ST_M5), ProLoad<FD>{d(YH_O)}, EpiStore<FD>{d(T64_E)}, kopt(nullptr, false), s);
        if (e != hipSuccess) return e;
        e = launch_dwf<double, FD, LinkD18, true, MIX_SA, ProLoad<FD>, EpiOuter<FD, FD, F, FY>>(
            g64(1), d(T64_E), lk64[1], s64(ST_M5), ProLoad<FD>{d(T64_E)},
            EpiOuter<FD, FD, F, FY>{d(BPP), d(YH_O), lo(L_R), ylo()}, kopt(nullptr, true), s);
        if (e != hipSuccess) return e;
        return fin(g64(1).nblocks, FIN_OUTER);
    }

    // ---------------- inner CG kernels ----------------
    hipError_t kE(const int* live, const int* reset) {
        return launch_dwf<Real, F, LF, false, MIX_AS, ProCgE<F, F>, EpiStore<F>>(
            glo(1), lo(L_R), lk[1], slo(ST_M5TG5), ProCgE<F, F>{lo(L_R), lo(L_P), w->st.beta, reset},
            EpiStore<F>{lo(L_T1)}, kopt(live, false), s);
    }
    hipError_t kA() {
        return launch_dwf<Real, F, LF, true, MIX_AS, ProLoad<F>, EpiStore<F>>(
            glo(0), lo(L_T1), lk[0], slo(ST_M5T), ProLoad<F>{lo(L_T1)}, EpiStore<F>{lo(L_T23)}, kopt(w->st.live, false),
            s);
    }
    hipError_t kB() {
        return launch_dwf<Real, F, LF, true, MIX_NONE, ProLoad<F>, EpiCgB<F, F>>(
            glo(1), lo(L_T23), lk[1], nullptr, ProLoad<F>{lo(L_T23)}, EpiCgB<F, F>{lo(L_P), lo(L_U)},
            kopt(w->st.live, true), s);
    }
    hipError_t kC() {
        return launch_dwf<Real, F, LF, true, MIX_SA, ProLoad<F>, EpiStore<F>>(
            glo(0), lo(L_U), lk[0], slo(ST_M5), ProLoad<F>{lo(L_U)}, EpiStore<F>{lo(L_T23)}, kopt(w->st.live, false), s);
    }
    hipError_t kD() {
        return launch_dwf<Real, F, LF, true, MIX_SA, ProLoad<F>, EpiCgD<F, F, FY>>(
            glo(1), lo(L_T23), lk[1], slo(ST_M5), ProLoad<F>{lo(L_T23)},
            EpiCgD<F, F, FY>{lo(L_U), lo(L_R), ylo(), w->st.alpha}, kopt(w->st.live, true), s);
    }
    hipError_t iteration(bool with_e) {
        hipError_t e;
        if (with_e && (e = kE(w->st.live, nullptr)) != hipSuccess) return e;
        if ((e = kA()) != hipSuccess) return e;
        if ((e = kB()) != hipSuccess) return e;
        if ((e = fin(glo(1).nblocks, FIN_ALPHA)) != hipSuccess) return e;
        if ((e = kC()) != hipSuccess) return e;
        if ((e = kD()) != hipSuccess) return e;
        return fin(glo(1).nblocks, FIN_BETA);
    }

    int ensure_graph(int iters_per_graph) {
        if (w->gexec && w->graph_iters == iters_per_graph) return DWF_OK;
        if (w->gexec) (void)hipGraphExecDestroy(w->gexec);
        if (w->graph) (void)hipGraphDestroy(w->graph);
        w->gexec = nullptr;
        w->graph = nullptr;
        DWF_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int i = 0; i < iters_per_graph && e == hipSuccess; ++i) e = iteration(true);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(s, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(DWF_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
        }
        w->graph = g;
        DWF_HIP(hipGraphInstantiate(&w->gexec, g, nullptr, nullptr, 0));
        w->graph_iters = iters_per_graph;
        return DWF_OK;
    }
};

template <class Real, class F, class FY, class LF>
int run_solve(dwf_ctx* c, const double* b_dev, double* x_dev, int nrhs, const dwf_solve_params& p,
              dwf_solve_stats* stats, hipStream_t s, int link_fmt, LF lke, LF lko) {
    int rc;
    const TableSet* ts = c->table_set(c->mq, &rc);
    if (!ts) return rc;
    const int prec = p.inner_prec;
    std::string key = "solve:" + std::to_string(prec) + ":" + std::to_string(link_fmt) + ":" + std::to_string(nrhs);
    auto& slot = c->ws[key];
    if (!slot) {
        slot.reset(new Workspace);
        std::vector<int> precs(NF64, DWF_PREC_FP64);
        for (int i = 0; i < 5; ++i) precs.push_back(prec);
        precs.push_back(prec == DWF_PREC_FP64 ? DWF_PREC_FP64 : DWF_PREC_FP32);  // y
        if ((rc = slot->alloc(precs, c->V5h, c->Ns, nrhs)) || (rc = slot->alloc_state(nrhs))) {
            slot.reset();
            return rc;
        }
    }
    Workspace* w = slot.get();
    // per-workspace block sums and masks (fixed addresses: the graph keeps them)
    auto& pslot = c->ws[key + ":aux"];
    if (!pslot) {
        pslot.reset(new Workspace);
        long nb = std::max(c->geom(0, true).nblocks, c->geom(0, false).nblocks);
        if ((rc = pslot->state.alloc((size_t)nb * nrhs * sizeof(double) + 2 * (size_t)nrhs * sizeof(int)))) {
            pslot.reset();
            return rc;
        }
    }
    DevBuf* partials_buf = &pslot->state;
    long nbmax = std::max(c->geom(0, true).nblocks, c->geom(0, false).nblocks);
    int* mask_a = (int*)(partials_buf->as<double>() + nbmax * nrhs);
    int* mask_b = mask_a + nrhs;

    Solver<Real, F, FY, LF> S{c, ts, w, {lke, lko},
                              {LinkD18{c->links[0][LINK_D18].as<double>()}, LinkD18{c->links[1][LINK_D18].as<double>()}},
                              nrhs, s, partials_buf, mask_a, mask_b, p};

    // pinned host mirrors of the device state
    struct Pinned {
        void* p = nullptr;
        ~Pinned() { if (p) (void)hipHostFree(p); }
    } pin;
    const size_t nd = 6 * (size_t)nrhs, ni = 4 * (size_t)nrhs;
    DWF_HIP(hipHostMalloc(&pin.p, nd * sizeof(double) + ni * sizeof(int) + 2 * nrhs * sizeof(int), hipHostMallocDefault));
    double* hd = (double*)pin.p;
    int* hi = (int*)(hd + nd);
    double* h_rr = hd;
    double* h_target = hd + 4 * nrhs;
    double* h_aux = hd + 5 * nrhs;
    int* h_live = hi;
    int* h_iters = hi + nrhs;
    int* h_status = hi + 2 * nrhs;
    int* h_maxiter = hi + 3 * nrhs;
    int* h_mask = hi + 4 * nrhs;  // 2 * nrhs
    const CgState& st = w->st;

    auto pull = [&]() -> int {
        DWF_HIP(hipMemcpyAsync(hd, st.rr, nd * sizeof(double), hipMemcpyDeviceToHost, s));
        DWF_HIP(hipMemcpyAsync(hi, st.live, ni * sizeof(int), hipMemcpyDeviceToHost, s));
        DWF_HIP(hipStreamSynchronize(s));
        return DWF_OK;
    };
    auto push_ctl = [&]() -> int {
        DWF_HIP(hipMemcpyAsync(st.rr_target, h_target, nrhs * sizeof(double), hipMemcpyHostToDevice, s));
        DWF_HIP(hipMemcpyAsync(st.live, h_live, nrhs * sizeof(int), hipMemcpyHostToDevice, s));
        DWF_HIP(hipMemcpyAsync(st.maxiter, h_maxiter, nrhs * sizeof(int), hipMemcpyHostToDevice, s));
        DWF_HIP(hipMemcpyAsync(st.status, h_status, nrhs * sizeof(int), hipMemcpyHostToDevice, s));
        DWF_HIP(hipMemcpyAsync(mask_a, h_mask, 2 * nrhs * sizeof(int), hipMemcpyHostToDevice, s));
        return DWF_OK;
    };
#define CKE(x)                                                                                  \
    do {                                                                                        \
        hipError_t e_ = (x);                                                                    \
        if (e_ != hipSuccess) return fail(DWF_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)
#define CKR(x)          \
    do {                \
        int r_ = (x);   \
        if (r_) return r_; \
    } while (0)

    hipEvent_t ev0, ev1;
    DWF_HIP(hipEventCreate(&ev0));
    DWF_HIP(hipEventCreate(&ev1));
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
    } evg{ev0, ev1};
    DWF_HIP(hipEventRecord(ev0, s));

    // reset per-solve state
    for (int r = 0; r < nrhs; ++r) {
        h_live[r] = 0;
        h_status[r] = 0;
        h_maxiter[r] = p.maxiter;
        h_target[r] = 0;
        h_mask[r] = 0;
        h_mask[nrhs + r] = 0;
    }
    DWF_HIP(hipMemsetAsync(st.iters, 0, nrhs * sizeof(int), s));
    CKR(push_ctl());

    const int nb64o = S.g64(1).nblocks, nb64e = S.g64(0).nblocks;

    // ---- setup: b -> SoA, |b|^2, b' = S1 b, b'' = b'_o - M5 D^OE b'_e, |b''|^2
    CKE(host_to_half(c, b_dev, nrhs, w->f(B_E), w->f(B_O), s));
    std::vector<double> bnorm2(nrhs, 0.0), bpp2(nrhs, 0.0);
    CKE(S.norm64(0, B_E));
    CKE(S.fin(nb64e, FIN_AUX));
    CKR(pull());
    for (int r = 0; r < nrhs; ++r) bnorm2[r] = h_aux[r];
    CKE(S.norm64(1, B_O));
    CKE(S.fin(nb64o, FIN_AUX));
    CKR(pull());
    for (int r = 0; r < nrhs; ++r) bnorm2[r] += h_aux[r];

    if (p.use_guess) {
        CKE(host_to_half(c, x_dev, nrhs, w->f(BP_E), w->f(BP_O), s));
        CKE(S.local64(1, BP_O, TB_S2INV, YH_O));
    } else {
        CKE(half_zero(c, w->f(YH_O), nrhs, s));
    }
    CKE(S.local64(0, B_E, TB_S1, BP_E));
    CKE(S.local64(1, B_O, TB_S1, BP_O));
    CKE(S.xmy_m5hop64(1, BP_E, BP_O, BPP, true));
    CKE(S.fin(nb64o, FIN_AUX));
    CKR(pull());
    for (int r = 0; r < nrhs; ++r) bpp2[r] = h_aux[r];

    // ---- per-rhs control state
    // Inner relative tolerance per restart.  Defect correction rebuilds the
    // Krylov space at every restart and can run far (eps_dc).  Reliable updates
    // keep p, so they restart each time the iterated residual has dropped by
    // eps_ru, before the low-precision drift between the iterated and the true
    // residual grows comparable to the residual itself.
    const double eps_dc = p.eps_inner > 0 ? p.eps_inner
                                          : (prec == DWF_PREC_FP32 ? 1e-5 : prec == DWF_PREC_FP16 ? 2e-3 : 0.0);
    const double eps_ru = p.eps_inner > 0 ? p.eps_inner : (prec == DWF_PREC_FP64 ? 0.0 : 0.1);
    std::vector<int> mode_ru(nrhs, p.reliable ? 1 : 0), cycles(nrhs, 0), fellback(nrhs, 0), done(nrhs, 0),
        noprog(nrhs, 0), ru_restarts(nrhs, 0), have_backup(nrhs, 0), reverted(nrhs, 0);
    std::vector<double> rhat_prev(nrhs, 0.0), tol_schur(nrhs, p.tol), true_res(nrhs, 0.0), schur_res(nrhs, 0.0);
    int restarts = 0;
    const int iters_per_graph = 4;
    const bool verbose = getenv("DWF_VERBOSE") != nullptr;
    if (p.use_graph) CKR(S.ensure_graph(iters_per_graph));
    bool failed_any = false;

    for (int round = 0; round < 6; ++round) {
        // ================= outer loop (Algorithm 2 with reliable updates) =================
        for (int cyc = 0; cyc < 400; ++cyc) {
            CKE(S.outer_residual());
            ++restarts;
            CKR(pull());
            // A cycle that did not lower the true residual is rejected: the
            // previous iterate (kept in YH_E) is restored, and reliable updates
            // give way to defect correction (Sec. 2.3's automatic switch).
            bool revert = false;
            for (int r = 0; r < nrhs; ++r) {
                reverted[r] = 0;
                h_mask[r] = (!done[r] && have_backup[r] && !(sqrt(h_aux[r]) < rhat_prev[r])) ? 1 : 0;
                revert |= h_mask[r] != 0;
            }
            if (revert) {
                DWF_HIP(hipMemcpyAsync(mask_a, h_mask, nrhs * sizeof(int), hipMemcpyHostToDevice, s));
                CKE(half_copy(c, w->f(YH_O), w->f(YH_E), nrhs, mask_a, s));
                CKE(S.outer_residual());
                ++restarts;
                CKR(pull());
                for (int r = 0; r < nrhs; ++r)
                    if (h_mask[r]) {
                        reverted[r] = 1;
                        if (mode_ru[r]) {
                            mode_ru[r] = 0;
                            fellback[r] = 1;
                        } else if (++noprog[r] >= 4) {  // defect correction no longer converges
                            done[r] = 1;
                            failed_any = true;
                        }
                    }
            }
            bool any = false;
            for (int r = 0; r < nrhs; ++r) {
                double rh2 = h_aux[r];
                double rel = bpp2[r] > 0 ? sqrt(rh2 / bpp2[r]) : 0.0;
                schur_res[r] = rel;
                h_mask[r] = 0;           // mask_a: reset p := r (defect correction / first cycle)
                h_mask[nrhs + r] = 0;    // mask_b: continuing with p kept
                if (done[r] || !(rel > tol_schur[r]) || !std::isfinite(rh2)) {
                    if (!std::isfinite(rh2)) failed_any = true;
                    done[r] = 1;
                    h_live[r] = 0;
                    continue;
                }
                if (cycles[r] > 0 && !reverted[r]) {
                    if (mode_ru[r]) {
                        // reliable-update stall test
                        bool stalled = sqrt(rh2) > 0.5 * rhat_prev[r] || h_status[r] == 2 || h_status[r] == 4 ||
                                       (p.debug_stall_after > 0 && ru_restarts[r] >= p.debug_stall_after);
                        if (stalled) {
                            mode_ru[r] = 0;
                            fellback[r] = 1;
                        } else {
                            ++ru_restarts[r];
                        }
                    } else if (sqrt(rh2) > 0.9 * rhat_prev[r]) {
                        if (++noprog[r] >= 4) {
                            done[r] = 1;
                            failed_any = true;
                            h_live[r] = 0;
                            continue;
                        }
                    } else {
                        noprog[r] = 0;
                    }
                }
                rhat_prev[r] = sqrt(rh2);
                const double eps = mode_ru[r] ? eps_ru : eps_dc;
                double stop = 0.5 * tol_schur[r] * sqrt(bpp2[r]);
                double tgt = std::max(eps * sqrt(rh2), stop);
                h_target[r] = tgt * tgt;
                h_live[r] = 1;
                h_status[r] = 0;
                if (cycles[r] == 0 || !mode_ru[r] || reverted[r])
                    h_mask[r] = 1;
                else
                    h_mask[nrhs + r] = 1;
                ++cycles[r];
                any = true;
            }
            for (int r = 0; r < nrhs; ++r) h_maxiter[r] = p.maxiter;
            if (verbose)
                for (int r = 0; r < nrhs; ++r)
                    fprintf(stderr, "[dwf] round %d cycle %d rhs %d: |rhat|/|b''| = %.3e  mode=%s iters=%d live=%d%s\n",
                            round, cyc, r, schur_res[r], mode_ru[r] ? "RU" : "DC", h_iters[r], h_live[r],
                            reverted[r] ? " (reverted)" : "");
            if (!any) break;
            // iteration cap over all cycles
            for (int r = 0; r < nrhs; ++r)
                if (h_live[r] && h_iters[r] >= p.maxiter) {
                    h_live[r] = 0;
                    done[r] = 1;
                    failed_any = true;
                }
            CKR(push_ctl());
            // p := r for the rhs that restart from scratch
            CKE(S.kE(mask_a, mask_a));
            // first iteration without the direction update, then graph replays
            CKE(S.iteration(false));
            int replays = 1;
            double rr_last = -1;
            int it_last = 0;
            long launched = 1;
            for (;;) {
                // host-side bound: the device stops every rhs at maxiter, so this
                // only trips if the device state stops advancing
                if (launched > (long)p.maxiter + 8L * iters_per_graph) {
                    failed_any = true;
                    for (int r = 0; r < nrhs; ++r) done[r] = 1;
                    break;
                }
                launched += (long)replays * iters_per_graph;
                if (p.use_graph) {
                    for (int k = 0; k < replays; ++k) CKE(hipGraphLaunch(w->gexec, s));
                } else {
                    for (int k = 0; k < replays * iters_per_graph; ++k) CKE(S.iteration(true));
                }
                CKR(pull());
                bool alive = false;
                double worst = 0;
                int itmin = 1 << 30;
                for (int r = 0; r < nrhs; ++r)
                    if (h_live[r]) {
                        alive = true;
                        worst = std::max(worst, h_rr[r] / std::max(h_target[r], 1e-300));
                        itmin = std::min(itmin, h_iters[r]);
                    }
                if (!alive) break;
                // adapt the number of replays between checks to the convergence rate
                if (rr_last > 0 && itmin > it_last && worst < rr_last) {
                    double per_it = log(worst / rr_last) / (double)(itmin - it_last);
                    double need = per_it < 0 ? log(worst) / -per_it : 1e9;
                    replays = (int)std::min(64.0, std::max(1.0, 0.8 * need / iters_per_graph));
                } else {
                    replays = std::min(64, replays * 2);
                }
                rr_last = worst;
                it_last = itmin;
            }
            // reliable updates: finish the last direction update p = r + beta p
            // (Algorithm 1 computes p_{k+1} before testing convergence)
            for (int r = 0; r < nrhs; ++r) h_mask[nrhs + r] = (mode_ru[r] && h_status[r] == 1 && !done[r]) ? 1 : 0;
            DWF_HIP(hipMemcpyAsync(mask_b, h_mask + nrhs, nrhs * sizeof(int), hipMemcpyHostToDevice, s));
            CKE(S.kE(mask_b, nullptr));
            // keep the current iterate, then yhat += y
            CKE(half_copy(c, w->f(YH_E), w->f(YH_O), nrhs, nullptr, s));
            for (int r = 0; r < nrhs; ++r) have_backup[r] = 1;
            CKE(half_acc(c, w->f(YH_O), w->f(L_Y), nrhs, nullptr, s));
            for (int r = 0; r < nrhs; ++r)
                if (h_status[r] == 2 && !mode_ru[r]) {  // breakdown in defect correction: give up
                    done[r] = 1;
                    failed_any = true;
                }
        }
        // ================= reconstruction and the true residual =================
        // y_e = b'_e - M5 D^EO y_o ; x = S2 y  (into BP_E/BP_O)
        CKE(S.xmy_m5hop64(0, YH_O, BP_E, YH_E, false));
        CKE(S.local64(0, YH_E, TB_S2, BP_E));
        CKE(S.local64(1, YH_O, TB_S2, BP_O));
        // D x = X x + D_w (Y x) per parity; Y x -> YH_*, X x -> T64_E (even), BPP (odd)
        // (BPP is rebuilt below if another round is needed)
        CKE(S.local64(0, BP_E, TB_Y, YH_E));
        CKE(S.local64(1, BP_O, TB_Y, T64_E));  // temporarily Yx_o in T64_E
        std::vector<double> tr(nrhs, 0.0);
        {
            // even rows: b_e - X x_e - D^EO (Y x)_o ; X x_e -> YH_O is free? no: keep yhat_o.
            // use BPP for X x_e, then odd rows with X x_o in BPP again.
            CKE(S.local64(0, BP_E, TB_X, BPP));
            CKE((launch_dwf<double, FD, LinkD18, true, MIX_NONE, ProLoad<FD>, EpiTrueRes<FD, FD>>(
                S.g64(0), S.d(T64_E), S.lk64[0], nullptr, ProLoad<FD>{S.d(T64_E)},
                EpiTrueRes<FD, FD>{S.d(B_E), S.d(BPP)}, S.kopt(nullptr, true), s)));
            CKE(S.fin(nb64e, FIN_AUX));
            CKR(pull());
            for (int r = 0; r < nrhs; ++r) tr[r] = h_aux[r];
            CKE(S.local64(1, BP_O, TB_X, BPP));
            CKE((launch_dwf<double, FD, LinkD18, true, MIX_NONE, ProLoad<FD>, EpiTrueRes<FD, FD>>(
                S.g64(1), S.d(YH_E), S.lk64[1], nullptr, ProLoad<FD>{S.d(YH_E)},
                EpiTrueRes<FD, FD>{S.d(B_O), S.d(BPP)}, S.kopt(nullptr, true), s)));
            CKE(S.fin(nb64o, FIN_AUX));
            CKR(pull());
            for (int r = 0; r < nrhs; ++r) tr[r] += h_aux[r];
        }
        bool again = false;
        for (int r = 0; r < nrhs; ++r) {
            true_res[r] = bnorm2[r] > 0 ? sqrt(tr[r] / bnorm2[r]) : sqrt(tr[r]);
            if (true_res[r] > p.tol && done[r] && schur_res[r] <= tol_schur[r] && std::isfinite(true_res[r])) {
                // tighten the Schur target and continue from the current iterate
                tol_schur[r] *= std::max(0.01, 0.5 * p.tol / true_res[r]);
                done[r] = 0;
                again = true;
            }
        }
        if (!again || round == 5) break;
        // restore the pieces the reconstruction overwrote: b' and b''
        CKE(S.local64(0, B_E, TB_S1, BP_E));
        CKE(S.local64(1, B_O, TB_S1, BP_O));
        CKE(S.xmy_m5hop64(1, BP_E, BP_O, BPP, false));
    }
    // the last reconstruction left x in BP_E/BP_O
    CKE(half_to_host(c, w->f(BP_E), w->f(BP_O), nrhs, x_dev, s));
    DWF_HIP(hipEventRecord(ev1, s));
    CKR(pull());
    DWF_HIP(hipEventSynchronize(ev1));
    float ms = 0;
    DWF_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    int status = DWF_OK;
    for (int r = 0; r < nrhs; ++r)
        if (!(true_res[r] <= p.tol)) status = DWF_ENOCONV;
    if (failed_any) status = DWF_ENOCONV;
    if (stats) {
        const double fi = flops_per_iter(c);
        const double bi = bytes_per_iter(c, prec, link_fmt);
        const double V = (double)c->V5h;
        const double fo = V * (2640.0 + 96.0 * c->Ns + 72.0);
        const double fsetup = V * (144.0 * c->Ns + 1392.0);
        const double ffinal = V * (336.0 * c->Ns + 4080.0);
        long tot_it = 0;
        for (int r = 0; r < nrhs; ++r) tot_it += h_iters[r];
        for (int r = 0; r < nrhs; ++r) {
            dwf_solve_stats& o = stats[r];
            memset(&o, 0, sizeof(o));
            o.status = (true_res[r] <= p.tol) ? DWF_OK : DWF_ENOCONV;
            o.iters = h_iters[r];
            o.restarts = restarts;
            o.reliable_updates = ru_restarts[r];
            o.fallback = fellback[r];
            o.true_residual = true_res[r];
            o.schur_residual = schur_res[r];
            o.seconds = ms * 1e-3;
            const double flops = fi * tot_it + (fo * restarts + fsetup + ffinal) * nrhs;
            o.gflops = o.seconds > 0 ? flops / o.seconds * 1e-9 : 0;
            o.hbm_gbytes = (bi * tot_it + 12.0 * V * 192.0 * (restarts + 4) * nrhs) * 1e-9;
        }
    }
    if (status != DWF_OK) fail(DWF_ENOCONV, "solve did not reach the requested tolerance");
    return status;
#undef CKE
#undef CKR
}

template <class Real, class F, class FY, class LF>
int time_kernels(dwf_ctx* c, const dwf_solve_params& p, int nrhs, int launches, double* ms, double* bytes,
                 int link_fmt, LF lke, LF lko) {
    int rc;
    const TableSet* ts = c->table_set(c->mq, &rc);
    if (!ts) return rc;
    std::string key = "solve:" + std::to_string(p.inner_prec) + ":" + std::to_string(link_fmt) + ":" +
                      std::to_string(nrhs);
    auto it = c->ws.find(key);
    auto ip = c->ws.find(key + ":aux");
    if (it == c->ws.end() || !it->second || ip == c->ws.end() || !ip->second)
        return fail(DWF_EINVAL, "no solve workspace for these parameters; run a solve first");
    Workspace* w = it->second.get();
    DevBuf* partials_buf = &ip->second->state;
    hipStream_t s = c->stream;
    Solver<Real, F, FY, LF> S{c, ts, w, {lke, lko},
                              {LinkD18{c->links[0][LINK_D18].as<double>()}, LinkD18{c->links[1][LINK_D18].as<double>()}},
                              nrhs, s, partials_buf, nullptr, nullptr, p};
    // all kernels forced on (live = NULL); A, C are idempotent, B/D/E update
    // their outputs from finite inputs
    auto runk = [&](int k) -> hipError_t {
        const int* nolive = nullptr;
        switch (k) {
            case 0: return S.kE(nolive, nullptr);
            case 1:
                return launch_dwf<Real, F, LF, true, MIX_AS, ProLoad<F>, EpiStore<F>>(
                    S.glo(0), S.lo(L_T1), S.lk[0], S.slo(ST_M5T), ProLoad<F>{S.lo(L_T1)}, EpiStore<F>{S.lo(L_T23)},
                    S.kopt(nolive, false), s);
            case 2:
                return launch_dwf<Real, F, LF, true, MIX_NONE, ProLoad<F>, EpiCgB<F, F>>(
                    S.glo(1), S.lo(L_T23), S.lk[1], nullptr, ProLoad<F>{S.lo(L_T23)}, EpiCgB<F, F>{S.lo(L_P), S.lo(L_U)},
                    S.kopt(nolive, true), s);
            case 3:
                return launch_dwf<Real, F, LF, true, MIX_SA, ProLoad<F>, EpiStore<F>>(
                    S.glo(0), S.lo(L_U), S.lk[0], S.slo(ST_M5), ProLoad<F>{S.lo(L_U)}, EpiStore<F>{S.lo(L_T23)},
                    S.kopt(nolive, false), s);
            default:
                return launch_dwf<Real, F, LF, true, MIX_SA, ProLoad<F>, EpiCgD<F, F, FY>>(
                    S.glo(1), S.lo(L_T23), S.lk[1], S.slo(ST_M5), ProLoad<F>{S.lo(L_T23)},
                    EpiCgD<F, F, FY>{S.lo(L_U), S.lo(L_R), S.ylo(), w->st.alpha}, S.kopt(nolive, true), s);
        }
    };
    // one event pair around every launch: the average is the kernels' own
    // device time, without the dispatch gap between back-to-back launches
    std::vector<hipEvent_t> ev(2 * (size_t)launches, nullptr);
    for (auto& e : ev) DWF_HIP(hipEventCreate(&e));
    const double sb = spinor_bytes(p.inner_prec) * (double)c->V5h * nrhs;
    const double yb = (p.inner_prec == DWF_PREC_FP64 ? 192.0 : 96.0) * (double)c->V5h * nrhs;
    const double lb = (double)c->V4h * 8.0 * link_bytes(link_fmt);
    const double model[5] = {4 * sb, 2 * sb + lb, 3 * sb + lb, 2 * sb + lb, 4 * sb + 2 * yb + lb};
    int result = DWF_OK;
    for (int k = 0; k < 5 && result == DWF_OK; ++k) {
        hipError_t e = runk(k);  // warm-up launch
        for (int i = 0; i < launches && e == hipSuccess; ++i) {
            e = hipEventRecord(ev[2 * i], s);
            if (e == hipSuccess) e = runk(k);
            if (e == hipSuccess) e = hipEventRecord(ev[2 * i + 1], s);
        }
        if (e == hipSuccess) e = hipEventSynchronize(ev[2 * launches - 1]);
        double tot = 0;
        for (int i = 0; i < launches && e == hipSuccess; ++i) {
            float t = 0;
            e = hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]);
            tot += t;
        }
        if (e != hipSuccess) {
            result = fail(DWF_EDEVICE, std::string("kernel timing: ") + hipGetErrorString(e));
            break;
        }
        ms[k] = tot / launches;
        bytes[k] = model[k];
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    return result;
}

}  // namespace

int time_inner_kernels(dwf_ctx* c, const dwf_solve_params& p, int nrhs, int launches, double* ms, double* bytes) {
    const LinkD18 d0{c->links[0][LINK_D18].as<double>()}, d1{c->links[1][LINK_D18].as<double>()};
    switch (p.inner_prec) {
        case DWF_PREC_FP64:
            return time_kernels<double, FD, FD, LinkD18>(c, p, nrhs, launches, ms, bytes, LINK_D18, d0, d1);
        case DWF_PREC_FP32:
            if (p.link_compress == 1)
                return time_kernels<float, FS, FS, LinkS12>(c, p, nrhs, launches, ms, bytes, LINK_S12,
                                                            LinkS12{c->links[0][LINK_S12].as<float>()},
                                                            LinkS12{c->links[1][LINK_S12].as<float>()});
            return time_kernels<float, FS, FS, LinkS18>(c, p, nrhs, launches, ms, bytes, LINK_S18,
                                                        LinkS18{c->links[0][LINK_S18].as<float>()},
                                                        LinkS18{c->links[1][LINK_S18].as<float>()});
        default:
            return time_kernels<float, FH, FS, LinkH12>(c, p, nrhs, launches, ms, bytes, LINK_H12,
                                                        LinkH12{c->links[0][LINK_H12].as<_Float16>()},
                                                        LinkH12{c->links[1][LINK_H12].as<_Float16>()});
    }
}

int solve(dwf_ctx* c, const double* b_dev, double* x_dev, int nrhs, const dwf_solve_params& p,
          dwf_solve_stats* stats, hipStream_t s, const double* mq_per_rhs) {
    (void)mq_per_rhs;
    const LinkD18 d0{c->links[0][LINK_D18].as<double>()}, d1{c->links[1][LINK_D18].as<double>()};
    switch (p.inner_prec) {
        case DWF_PREC_FP64:
            return run_solve<double, FD, FD, LinkD18>(c, b_dev, x_dev, nrhs, p, stats, s, LINK_D18, d0, d1);
        case DWF_PREC_FP32:
            if (p.link_compress == 1)
                return run_solve<float, FS, FS, LinkS12>(c, b_dev, x_dev, nrhs, p, stats, s, LINK_S12,
                                                         LinkS12{c->links[0][LINK_S12].as<float>()},
                                                         LinkS12{c->links[1][LINK_S12].as<float>()});
            return run_solve<float, FS, FS, LinkS18>(c, b_dev, x_dev, nrhs, p, stats, s, LINK_S18,
                                                     LinkS18{c->links[0][LINK_S18].as<float>()},
                                                     LinkS18{c->links[1][LINK_S18].as<float>()});
        default:
            return run_solve<float, FH, FS, LinkH12>(c, b_dev, x_dev, nrhs, p, stats, s, LINK_H12,
                                                     LinkH12{c->links[0][LINK_H12].as<_Float16>()},
                                                     LinkH12{c->links[1][LINK_H12].as<_Float16>()});
    }
}

}  // namespace dwf
