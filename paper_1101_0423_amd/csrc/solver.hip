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
// One inner CG iteration is four fused stencil kernels plus one one-block
// reduction finisher (Secs. 3.2-3.5).  The search direction is carried as
// u = C^dag p: C^dag is linear, so u follows p's recurrence p = r + beta p as
// u = C^dag r + beta u, and p itself is never formed (it is only for the
// solution update, which takes y += alpha u):
//   A: t2 = M5^T D^EO t1                                            (even)
//   B: u  = r - g5 D^OE t2 + beta u,  |u|^2 = (p, C C^dag p)        (odd)
//   C: t3 = M5 D^EO u; its first workgroups finish B's |u|^2 -> alpha (even)
//   D: q  = u - M5 D^OE t3;  y += alpha u;  r -= alpha q;  |r|^2;
//      t1 = M5^T g5 r for the next iteration                       (odd) -> beta
// (C^dag r = r - g5 D^OE M5^T D^EO M5^T g5 r.)
// alpha, beta and the convergence flags never leave the device; the host
// replays a hipGraph of four iterations and watches the live flags that the
// finisher mirrors into mapped host memory, so that a round of replays ends
// when a right-hand side ends its cycle.
//
// The engine runs K right-hand sides ("slots") through these kernels at once:
// every kernel reads each gauge link once for all live slots.  Each slot has
// its own phase (setup, outer step, inner iterations, reconstruction, done),
// its own quark mass (its row of the fifth-dimension tables) and its own
// tolerances, so one slot can restart, finish or be replaced while the others
// keep iterating.  dwf_solve fills all slots at once; the request server
// admits and retires slots as requests come and go.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <vector>

#include "dwf_ctx.h"

namespace dwf {

template <class F>
F fld(const HalfField& h);

double flops_per_iter(const dwf_ctx* c) {
    return (double)c->V5h * (5280.0 + 192.0 * c->Ns + 288.0);
}

static double spinor_bytes(int prec) { return prec == DWF_PREC_FP64 ? 192.0 : prec == DWF_PREC_FP32 ? 96.0 : 52.0; }
static double link_bytes(int fmt) { return fmt == LINK_D18 ? 144.0 : fmt == LINK_S18 ? 72.0 : fmt == LINK_S12 ? 48.0 : 24.0; }

double bytes_per_iter(const dwf_ctx* c, int inner_prec, int link_fmt) {
    const double sb = spinor_bytes(inner_prec);
    const double yb = inner_prec == DWF_PREC_FP64 ? 192.0 : 96.0;
    return (double)c->V5h * (13.0 * sb + 2.0 * yb) + 4.0 * (double)c->V4h * 8.0 * link_bytes(link_fmt);
}

// ---------------------------------------------------------------------------
// Tile candidates of the inner kernels and the tuning cache
// ---------------------------------------------------------------------------

// The inner kernels' tiles the autotuner tries: the default sites per
// workgroup and half of it (while a workgroup keeps at least one wave), each
// in the automatic block order, then plain, t-fastest and tiled orders
// (geometries equal to an earlier candidate are left out).  A fixed
// dwf_opts.sites_per_block keeps its G.  Candidate 0 is the automatic order
// at the default G.
std::vector<TileCand> tile_candidates(const dwf_ctx* c, bool fp64) {
    const int G0 = fp64 ? c->G64 : c->G32;
    std::vector<int> Gs{G0};
    if (c->opts.sites_per_block <= 0 && G0 % 2 == 0 && (G0 / 2) * c->Ns >= 64) Gs.push_back(G0 / 2);
    std::vector<TileCand> out;
    std::vector<Geom> seen;
    auto same = [](const Geom& a, const Geom& b) {
        return a.G == b.G && a.nsb == b.nsb && a.tchunk == b.tchunk && a.nsb0 == b.nsb0 && a.tilew == b.tilew;
    };
    for (int G : Gs)
        for (int order : {(int)ORDER_AUTO, (int)ORDER_TFAST, (int)ORDER_PLAIN, 2, 3, 4, 6}) {
            const Geom g = c->geom_tile(0, G, order);
            if (order >= 2 && g.tilew != order) continue;  // not a whole number of tiles per plane
            bool dup = false;
            for (auto& h : seen) dup |= same(g, h);
            if (dup) continue;
            seen.push_back(g);
            // report the order the geometry actually walks
            const int eff = g.nsb == 0 ? ORDER_PLAIN : g.tilew >= 2 ? g.tilew : ORDER_TFAST;
            out.push_back(TileCand{G, order, eff});
        }
    return out;
}

namespace {

struct TuneVal {
    int tile, kgroup;
};

std::mutex g_tune_mu;
std::map<std::string, TuneVal> g_tune;
bool g_tune_loaded = false;

// The tuning cache: in the process, and in the file named by DWF_TUNE_CACHE
// (lines "key tile kgroup"), read once and appended to, when it is set.
void tune_load() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = getenv("DWF_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char key[512];
    int t, k;
    while (fscanf(f, "%511s %d %d", key, &t, &k) == 3) g_tune[key] = TuneVal{t, k};
    fclose(f);
}

bool tune_get(const std::string& key, TuneVal* v) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load();
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    *v = it->second;
    return true;
}

void tune_put(const std::string& key, TuneVal v) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load();
    g_tune[key] = v;
    if (const char* path = getenv("DWF_TUNE_CACHE")) {
        if (FILE* f = fopen(path, "a")) {
            fprintf(f, "%s %d %d\n", key.c_str(), v.tile, v.kgroup);
            fclose(f);
        }
    }
}

std::string arch_name(int device) {
    static std::mutex mu;
    static std::map<int, std::string> names;
    std::lock_guard<std::mutex> lk(mu);
    auto it = names.find(device);
    if (it != names.end()) return it->second;
    hipDeviceProp_t prop;
    std::string n = "unknown";
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        n = prop.gcnArchName;
        for (auto& ch : n)
            if (ch == ' ' || ch == ':') ch = '_';
    }
    names[device] = n;
    return n;
}

}  // namespace

namespace {

// half fields of an engine
enum { B_E = 0, B_O, BP_E, BP_O, BPP, YH_E, YH_O, T64_E, NF64 };
enum { L_R = NF64, L_P, L_U, L_T1, L_T23, L_Y, NFALL };
// per-slot masks on the device (each has its own pinned staging row)
enum { M_SETUP = 0, M_GUESS, M_NOGUESS, M_OUTER, M_REVERT, M_RESET, M_RUFIN, M_POST, M_FINAL, M_AGAIN,
       M_SETUP0, M_SETUP1, M_GUESS1, M_F0, M_F1, M_FIN0, M_FORM, M_START, NMASK };
enum { LIST_INNER = 0, LIST_RUFIN, LIST_F1, LIST_RUF1, NLIST };

constexpr int kItersPerGraph = 4;

long field_elems(long V5h, int prec) {
    const int nblk = prec == DWF_PREC_FP64 ? 12 : prec == DWF_PREC_FP32 ? 6 : 3;
    return ((V5h * nblk + 255) / 256) * 256;
}

// host control state of one slot
struct SlotCtl {
    int phase = PH_FREE;
    dwf_solve_params p{};
    double mq = 0;
    int use_guess = 0;
    int form = DWF_SYSTEM_D;  // D x = b, or C C^dag w = b on the odd sites
    int mode_ru = 1, cycles = 0, fellback = 0, noprog = 0, ru_restarts = 0, have_backup = 0, reverted = 0;
    int failed = 0, round = 0, restarts = 0, stuck = 0;
    double rhat_prev = 0, tol_schur = 0, true_res = 0, schur_res = 0, bnorm2 = 0, bpp2 = 0;
    double eps_dc = 0, eps_ru = 0;
    std::chrono::steady_clock::time_point t0;
    double seconds = 0;
};

template <class Real, class F, class FY, class LF>
class Engine : public EngineBase {
  public:
    Engine(dwf_ctx* c_, int prec_, int fmt_, int K_, hipStream_t s_, LF e, LF o, int forced_tile_)
        : c(c_), prec(prec_), link_fmt(fmt_), K(K_), s(s_), lk{e, o}, forced_tile(forced_tile_),
          lk64{LinkD18{c_->links[0][LINK_D18].as<double>()}, LinkD18{c_->links[1][LINK_D18].as<double>()}},
          sl((size_t)K_) {}
    ~Engine() override {
        if (ev[0]) (void)hipEventDestroy(ev[0]);
        if (ev[1]) (void)hipEventDestroy(ev[1]);
        if (live_pin) (void)hipHostFree(live_pin);
        for (auto& kv : graphs) {
            (void)hipGraphExecDestroy(kv.second.second);
            (void)hipGraphDestroy(kv.second.first);
        }
        if (pin) (void)hipHostFree(pin);
    }

    int init() {
        int rc;
        std::vector<int> precs(NF64, DWF_PREC_FP64);
        for (int i = 0; i < 5; ++i) precs.push_back(prec);
        precs.push_back(prec == DWF_PREC_FP64 ? DWF_PREC_FP64 : DWF_PREC_FP32);  // y
        if ((rc = w.alloc(precs, c->V5h, c->Ns, K)) || (rc = w.alloc_state(K, s))) return rc;
        // live flags mirrored by the finisher into mapped host memory
        DWF_HIP(hipHostMalloc(&live_pin, (size_t)K * sizeof(int), hipHostMallocMapped));
        memset(live_pin, 0, (size_t)K * sizeof(int));
        DWF_HIP(hipHostGetDevicePointer((void**)&w.st.live_host, live_pin, 0));
        // a copy of the state's pointers in device memory, for kernel C's alpha
        if ((rc = st_dev.alloc(sizeof(CgState)))) return rc;
        DWF_HIP(hipMemcpyAsync(st_dev.p, &w.st, sizeof(CgState), hipMemcpyHostToDevice, s));
        DWF_HIP(hipStreamSynchronize(s));
        DWF_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
        DWF_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
        TS = (long)tables_size(c->Ns);
        if ((rc = tabs64.alloc((size_t)TS * K * sizeof(double))) || (rc = tabs32.alloc((size_t)TS * K * sizeof(float))))
            return rc;
        cands = tile_candidates(c, sizeof(Real) == 8);
        if (forced_tile >= (int)cands.size())
            return fail(DWF_EINVAL, "params.tile: there are " + std::to_string(cands.size()) + " tile candidates");
        nbmax = c->geom(0, true).nblocks;
        for (auto& t : cands) nbmax = std::max(nbmax, c->geom_tile(0, t.G, t.order).nblocks);
        set_tile(forced_tile >= 0 ? forced_tile : 0);
        if ((rc = aux.alloc((size_t)nbmax * K * sizeof(double) + ((size_t)NMASK * K + NLIST * (K + 1)) * sizeof(int))))
            return rc;
        for (int m = 0; m < NMASK; ++m) dmask[m] = (int*)(aux.as<double>() + (size_t)nbmax * K) + (size_t)m * K;
        for (int l = 0; l < NLIST; ++l) dlist[l] = dmask[0] + (size_t)NMASK * K + (size_t)l * (K + 1);
        DWF_HIP(hipMemsetAsync(aux.p, 0, aux.bytes, s));
        DWF_HIP(hipStreamSynchronize(s));
        const size_t bytes = 7 * (size_t)K * sizeof(double) + ((4 + NMASK) * (size_t)K + NLIST * (K + 1)) * sizeof(int);
        DWF_HIP(hipHostMalloc(&pin, bytes, hipHostMallocDefault));
        memset(pin, 0, bytes);
        hd = (double*)pin;
        hi = (int*)(hd + 7 * (size_t)K);
        for (int m = 0; m < NMASK; ++m) hmask[m] = hi + 4 * (size_t)K + (size_t)m * K;
        for (int l = 0; l < NLIST; ++l) hlist[l] = hmask[0] + (size_t)NMASK * K + (size_t)l * (K + 1);
        return autotune();
    }

    int capacity() const override { return K; }
    int rhs_per_block() const override { return kgroup; }
    void tile(int* index, int* sites, int* order) const override {
        *index = tidx;
        *sites = cands[tidx].G;
        *order = cands[tidx].eff;
    }
    int phase(int r) const override { return sl[r].phase; }
    int busy() const override {
        int n = 0;
        for (auto& x : sl) n += x.phase != PH_FREE;
        return n;
    }
    int pending() const override {
        int n = 0;
        for (auto& x : sl) n += x.phase != PH_FREE && x.phase != PH_DONE;
        return n;
    }
    void set_stream(hipStream_t st) override { s = st; }
    void set_use_graph(bool on) override { use_graph = on; }
    void set_replay_cap(int n) override { replay_cap = std::max(1, n); }
    size_t device_bytes() const override {
        size_t b = w.state.bytes + tabs64.bytes + tabs32.bytes + aux.bytes;
        for (auto& f : w.fields) b += f->data.bytes + f->nrm.bytes;
        return b;
    }

    int admit(int r, const double* b_dev, const double* x0_dev, double mq, const dwf_solve_params& p) override {
        if (r < 0 || r >= K || sl[r].phase != PH_FREE) return fail(DWF_EINVAL, "slot not free");
        int rc;
        const TableSet* ts = c->table_set(mq, &rc);
        if (!ts) return rc;
        DWF_HIP(hipMemcpyAsync(tabs64.as<double>() + (size_t)r * TS, ts->d64.p, TS * sizeof(double),
                               hipMemcpyDeviceToDevice, s));
        DWF_HIP(hipMemcpyAsync(tabs32.as<float>() + (size_t)r * TS, ts->d32.p, TS * sizeof(float),
                               hipMemcpyDeviceToDevice, s));
        DWF_HIP(host_to_half(c, b_dev, 1, w.f(B_E), w.f(B_O), s, r));
        if (x0_dev) DWF_HIP(host_to_half(c, x0_dev, 1, w.f(BP_E), w.f(BP_O), s, r));
        SlotCtl& q = sl[r];
        q = SlotCtl{};
        q.phase = PH_SETUP;
        q.p = p;
        q.mq = mq;
        q.use_guess = x0_dev != nullptr;
        q.form = p.system == DWF_SYSTEM_CCDAG ? DWF_SYSTEM_CCDAG : DWF_SYSTEM_D;
        q.mode_ru = p.reliable ? 1 : 0;
        q.tol_schur = p.tol;
        q.eps_dc = p.eps_inner > 0 ? p.eps_inner
                                   : (prec == DWF_PREC_FP32 ? 1e-5 : prec == DWF_PREC_FP16 ? 2e-3 : 0.0);
        // reliable updates: replace the iterated residual by the true one each
        // time it has fallen to eps_ru of its value at the last restart;
        // binary16 storage drifts faster, and
        // restarting at 0.3 rather than 0.1 saves 14% of its iterations
        // (16^3x32: 2289 -> 1972), while FP32 is best at 0.1 (1662 vs 1686)
        q.eps_ru = p.eps_inner > 0 ? p.eps_inner
                                   : (prec == DWF_PREC_FP64 ? 0.0 : prec == DWF_PREC_FP16 ? 0.3 : 0.1);
        q.t0 = std::chrono::steady_clock::now();
        return DWF_OK;
    }

    int tick() override {
        int rc;
        using clk = std::chrono::steady_clock;
        const auto t0 = clk::now();
        if (any(PH_SETUP) && (rc = setup())) return rc;
        for (int guard = 0; any(PH_OUTER) || any(PH_FINAL); ++guard) {
            if (guard > 64) return fail(DWF_EDEVICE, "solve engine: outer loop does not settle");
            if (any(PH_OUTER) && (rc = outer())) return rc;
            if (any(PH_FINAL) && (rc = final_check())) return rc;
        }
        const auto t1 = clk::now();
        if (any(PH_INNER) && (rc = inner())) return rc;
        const auto t2 = clk::now();
        prof.ticks++;
        prof.outer_s += std::chrono::duration<double>(t1 - t0).count();
        prof.inner_s += std::chrono::duration<double>(t2 - t1).count();
        return DWF_OK;
    }

    int retire(int r, double* x_dev, SlotResult* res) override {
        if (r < 0 || r >= K || sl[r].phase != PH_DONE) return fail(DWF_EINVAL, "slot not done");
        SlotCtl& q = sl[r];
        if (x_dev) {
            if (q.form == DWF_SYSTEM_CCDAG)  // w on the odd sites, zero even half (B_E)
                DWF_HIP(half_to_host(c, w.f(B_E), w.f(YH_O), 1, x_dev, s, r));
            else
                DWF_HIP(half_to_host(c, w.f(BP_E), w.f(BP_O), 1, x_dev, s, r));
        }
        if (res) {
            const double V = (double)c->V5h;
            const double fo = V * (2640.0 + 96.0 * c->Ns + 72.0);
            const double fsetup = V * (144.0 * c->Ns + 1392.0);
            const double ffinal = V * (336.0 * c->Ns + 4080.0);
            res->status = (!q.failed && q.true_res <= q.p.tol) ? DWF_OK : DWF_ENOCONV;
            res->iters = hi[K + r];
            res->restarts = q.restarts;
            res->reliable_updates = q.ru_restarts;
            res->fallback = q.fellback;
            res->true_residual = q.true_res;
            res->schur_residual = q.schur_res;
            res->seconds = q.seconds;
            res->flops = flops_per_iter(c) * res->iters +
                         (q.form == DWF_SYSTEM_CCDAG ? 2.0 * fo * q.restarts
                                                     : fo * q.restarts + fsetup + ffinal * (q.round + 1));
            res->bytes = bytes_per_iter(c, prec, link_fmt) * res->iters + 12.0 * V * 192.0 * (q.restarts + 4);
        }
        q.phase = PH_FREE;
        return DWF_OK;
    }

    int time_kernels(int launches, double* ms, double* bytes) override;

    // The tile of the inner kernels (sites per workgroup and block order) and
    // the right-hand sides per workgroup: each candidate is timed over one
    // inner iteration (every slot forced on; the fields may hold anything,
    // which the solve overwrites before use), tiles first with one right-hand
    // side per workgroup, then the group size with the chosen tile.  Reading
    // each link once for more right-hand sides saves link bytes, while fewer
    // keep the neighbour re-reads of adjacent workgroups in L2.  Results are
    // cached per (arch, lattice, Ns, precision, links, K, fixed G).  Runs
    // before any graph is built.
    int autotune() {
        const std::string key = arch_name(c->device) + ":" + std::to_string(c->dims[0]) + "x" +
                                std::to_string(c->dims[1]) + "x" + std::to_string(c->dims[2]) + "x" +
                                std::to_string(c->dims[3]) + ":ns" + std::to_string(c->Ns) + ":p" +
                                std::to_string(prec) + ":l" + std::to_string(link_fmt) + ":k" + std::to_string(K) +
                                ":g" + std::to_string(c->opts.sites_per_block) + ":x" +
                                std::to_string(c->opts.xcd_remap < 0 ? 0 : 1);
        TuneVal v;
        if (forced_tile < 0 && tune_get(key, &v) && v.tile >= 0 && v.tile < (int)cands.size() && v.kgroup >= 1 &&
            v.kgroup <= K) {
            set_tile(v.tile);
            kgroup = v.kgroup;
            return DWF_OK;
        }
        hipEvent_t e0, e1;
        DWF_HIP(hipEventCreate(&e0));
        DWF_HIP(hipEventCreate(&e1));
        hipError_t e = hipSuccess;
        auto pass = [&]() {
            hipError_t r = kA(nullptr);
            if (r == hipSuccess) r = kB(nullptr);
            if (r == hipSuccess) r = kC(nullptr);
            if (r == hipSuccess) r = kD(nullptr);
            return r;
        };
        auto timed = [&](float* ms) {
            e = pass();
            if (e == hipSuccess) e = hipEventRecord(e0, s);
            for (int i = 0; i < 2 && e == hipSuccess; ++i) e = pass();
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
            return e == hipSuccess;
        };
        if (forced_tile < 0 && cands.size() > 1) {
            kgroup = 1;
            float best = 1e30f;
            int besti = 0;
            for (int i = 0; i < (int)cands.size(); ++i) {
                set_tile(i);
                float ms = 0;
                if (!timed(&ms)) break;
                if (verbose)
                    fprintf(stderr, "[dwf] autotune K=%d: tile %d (G=%d order=%d) %.3f ms\n", K, i, cands[i].G,
                            cands[i].eff, ms / 2);
                if (ms < best) {
                    best = ms;
                    besti = i;
                }
            }
            set_tile(besti);
        }
        kgroup = K;
        if (K > 1 && e == hipSuccess) {
            std::vector<int> cand;
            for (int k : {1, 2, 3, 4, 6, 8, 12, 16, 24, 32})
                if (k < K) cand.push_back(k);
            cand.push_back(K);
            float best = 1e30f;
            int bestk = K;
            for (int k : cand) {
                kgroup = k;
                float ms = 0;
                if (!timed(&ms)) break;
                if (verbose) fprintf(stderr, "[dwf] autotune K=%d: %d per workgroup %.3f ms\n", K, k, ms / 2);
                if (ms < best) {
                    best = ms;
                    bestk = k;
                }
            }
            kgroup = bestk;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (e != hipSuccess) return fail(DWF_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
        if (forced_tile < 0) tune_put(key, TuneVal{tidx, kgroup});
        return DWF_OK;
    }

  private:
    dwf_ctx* c;
    int prec, link_fmt, K;
    hipStream_t s;
    LF lk[2];
    int forced_tile;               // >= 0: params.tile - 1 (no tuning of the tile)
    std::vector<TileCand> cands;   // tiles of the inner kernels
    int tidx = 0;                  // the tile in use
    Geom gt[2];                    // its geometry per output parity
    void set_tile(int i) {
        tidx = i;
        for (int par = 0; par < 2; ++par) gt[par] = c->geom_tile(par, cands[i].G, cands[i].order);
    }
    LinkD18 lk64[2];
    std::vector<SlotCtl> sl;
    Workspace w;
    DevBuf tabs64, tabs32, aux, st_dev;
    long TS = 0;
    int nbmax = 0;
    int* dmask[NMASK] = {};
    int* dlist[NLIST] = {};  // compacted slot lists for the inner kernels' grids
    int* hlist[NLIST] = {};
    const int* cur_list = nullptr;  // list and group count the inner kernels launch over
    int cur_ng = 0;
    int cur_ng1 = 0;  // groups of the C C^dag w = b slots of the list (kernel E)
    // by group counts of the slot list and of its C C^dag w = b slots
    std::map<long, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
    void* pin = nullptr;
    double* hd = nullptr;  // rr, uu, alpha, beta, rr_target, aux, ecr  (K each)
    int* hi = nullptr;     // live, iters, status, maxiter  (K each), then the masks
    int* hmask[NMASK] = {};
    bool use_graph = true;
    int replay_cap = 64;
    void* live_pin = nullptr;  // host side of st.live_host
    hipEvent_t ev[2] = {nullptr, nullptr};
    const int verbose = getenv("DWF_VERBOSE") ? atoi(getenv("DWF_VERBOSE")) : 0;
    int kgroup = 1;  // right-hand sides per workgroup in the inner kernels
    // host-side accounting of where a solve's time goes (DWF_VERBOSE)
    struct {
        long ticks = 0, replays = 0, slot_iters_launched = 0, slot_iters_done = 0;
        double outer_s = 0, inner_s = 0;
    } prof;

  public:
    void report() override {
        if (!getenv("DWF_VERBOSE")) return;
        fprintf(stderr,
                "[dwf] engine K=%d: %ld rounds, %ld graph replays, outer+setup+final %.3f s, inner %.3f s, "
                "slot iterations done %ld of %ld launched\n",
                K, prof.ticks, prof.replays, prof.outer_s, prof.inner_s, prof.slot_iters_done,
                prof.slot_iters_launched);
        prof = {};
    }

  private:

    // host mirrors
    double& h_rr(int r) { return hd[r]; }
    double& h_beta(int r) { return hd[3 * K + r]; }
    double& h_target(int r) { return hd[4 * K + r]; }
    double& h_aux(int r) { return hd[5 * K + r]; }
    double& h_ecr(int r) { return hd[6 * K + r]; }
    int& h_live(int r) { return hi[r]; }
    int& h_iters(int r) { return hi[K + r]; }
    int& h_status(int r) { return hi[2 * K + r]; }
    int& h_maxiter(int r) { return hi[3 * K + r]; }

    bool any(int ph) const {
        for (auto& x : sl)
            if (x.phase == ph) return true;
        return false;
    }

    // ---------------- device state transfers ----------------
    // The host writes a mirror only after a pull (the stream is idle then) and
    // pushes it before the next pull, so the mirrors never race an async copy.
    int pull() {
        DWF_HIP(hipMemcpyAsync(hd, w.st.rr, 7 * (size_t)K * sizeof(double), hipMemcpyDeviceToHost, s));
        DWF_HIP(hipMemcpyAsync(hi, w.st.live, 4 * (size_t)K * sizeof(int), hipMemcpyDeviceToHost, s));
        DWF_HIP(hipStreamSynchronize(s));
        return DWF_OK;
    }
    // beta, rr_target, aux, ecr and the int state
    int push_ctl() {
        DWF_HIP(hipMemcpyAsync(w.st.beta, &h_beta(0), 4 * (size_t)K * sizeof(double), hipMemcpyHostToDevice, s));
        DWF_HIP(hipMemcpyAsync(w.st.live, hi, 4 * (size_t)K * sizeof(int), hipMemcpyHostToDevice, s));
        return DWF_OK;
    }
    // Uploads return the number of slots selected; a failed copy is kept in
    // upload_err and turned into the phase's return code (CKU).
    template <class Pred>
    int upload_mask(int m, Pred pred) {
        int n = 0;
        for (int r = 0; r < K; ++r) n += (hmask[m][r] = pred(r) ? 1 : 0);
        hipError_t e = hipMemcpyAsync(dmask[m], hmask[m], (size_t)K * sizeof(int), hipMemcpyHostToDevice, s);
        if (e != hipSuccess && upload_err == hipSuccess) upload_err = e;
        return n;
    }
    hipError_t upload_err = hipSuccess;

    // ---------------- kernels ----------------
    Geom g64(int par) const { return c->geom(par, true); }
    Geom glo(int par) const { return gt[par]; }
    FD d(int i) { return w.f(i).fd(); }
    F lo(int i) { return fld<F>(w.f(i)); }
    FY ylo() { return fld<FY>(w.f(L_Y)); }
    const double* t64(int t) const { return tabs64.as<double>() + dense_table_offset(c->Ns, t); }
    const double* s64(int t) const { return tabs64.as<double>() + struct_table_offset(c->Ns, t); }
    const Real* slo(int t) const {
        if constexpr (sizeof(Real) == 8)
            return tabs64.as<double>() + struct_table_offset(c->Ns, t);
        else
            return tabs32.as<float>() + struct_table_offset(c->Ns, t);
    }
    double* part() const { return aux.as<double>(); }
    // low-precision inner kernels take the tuned group of right-hand sides per
    // workgroup; the FP64 kernels (outer steps, once per cycle) take them all
    KOpt kopt(const int* live, bool red) const { return KOpt{live, red ? part() : nullptr, K, TS, 0}; }
    // Inner kernels launch over a compacted list of slots (cur_list) when one is
    // set, so that free, finished or waiting slots cost no workgroups.
    KOpt kopt_in(const int* live, bool red) const {
        return KOpt{live, red ? part() : nullptr, K, TS, kgroup, cur_list, cur_list ? cur_ng : 0};
    }
    // upload the slots that satisfy pred as list l; returns their number
    template <class Pred>
    int upload_list(int l, Pred pred) {
        int n = 0;
        for (int r = 0; r < K; ++r)
            if (pred(r)) hlist[l][1 + n++] = r;
        hlist[l][0] = n;
        hipError_t e = hipMemcpyAsync(dlist[l], hlist[l], (size_t)(K + 1) * sizeof(int), hipMemcpyHostToDevice, s);
        if (e != hipSuccess && upload_err == hipSuccess) upload_err = e;
        return n;
    }
    void use_list(int l, int n) {
        cur_list = dlist[l];
        cur_ng = (n + kgroup - 1) / kgroup;
    }
    hipError_t fin(int nblocks, int mode, const int* mask = nullptr) {
        return launch_finish(part(), nblocks, K, w.st, mode, s, mask);
    }

    hipError_t local64(int par, int in, int table, int out, const int* m) {
        return launch_dwf<double, FD, LinkD18, false, MIX_DENSE, ProLoad<FD>, EpiStore<FD>>(
            g64(par), d(in), lk64[par], t64(table), ProLoad<FD>{d(in)}, EpiStore<FD>{d(out)}, kopt(m, false), s);
    }
    hipError_t norm64(int par, int in, const int* m) {
        return launch_dwf<double, FD, LinkD18, false, MIX_NONE, ProLoad<FD>, EpiNorm>(
            g64(par), d(in), lk64[par], nullptr, ProLoad<FD>{d(in)}, EpiNorm{}, kopt(m, true), s);
    }
    // out = a - M5 D^{par,1-par} in
    hipError_t xmy_m5hop64(int par, int in, int a, int out, bool red, const int* m) {
        if (red)
            return launch_dwf<double, FD, LinkD18, true, MIX_SA, ProLoad<FD>, EpiLin<FD, FD, true, false>>(
                g64(par), d(in), lk64[par], s64(ST_M5), ProLoad<FD>{d(in)},
                EpiLin<FD, FD, true, false>{d(a), d(out), 1.0, -1.0}, kopt(m, true), s);
        return launch_dwf<double, FD, LinkD18, true, MIX_SA, ProLoad<FD>, EpiLin<FD, FD, false, false>>(
            g64(par), d(in), lk64[par], s64(ST_M5), ProLoad<FD>{d(in)},
            EpiLin<FD, FD, false, false>{d(a), d(out), 1.0, -1.0}, kopt(m, false), s);
    }
    // rhat = b'' - C yhat_o (FP64), r_lo = rhat, y_lo = 0, rr = aux = |rhat|^2.
    // For C C^dag w = b (form 1) yhat_o is w and C^dag w is formed first (in
    // BP_O, with T64_E as the even temporary), so that rhat = b - C C^dag w.
    hipError_t outer_residual(const int* m, int form) {
        hipError_t e = hipSuccess;
        int yh = YH_O;
        if (form == DWF_SYSTEM_CCDAG) {
            e = launch_dwf<double, FD, LinkD18, false, MIX_AS, ProLoad<FD>, EpiStore<FD>>(
                g64(1), d(YH_O), lk64[1], s64(ST_M5TG5), ProLoad<FD>{d(YH_O)}, EpiStore<FD>{d(BP_O)}, kopt(m, false),
                s);  // M5^T g5 w
            if (e == hipSuccess)
                e = launch_dwf<double, FD, LinkD18, true, MIX_AS, ProLoad<FD>, EpiStore<FD>>(
                    g64(0), d(BP_O), lk64[0], s64(ST_M5T), ProLoad<FD>{d(BP_O)}, EpiStore<FD>{d(T64_E)},
                    kopt(m, false), s);  // M5^T D^EO (...)
            if (e == hipSuccess)
                e = launch_dwf<double, FD, LinkD18, true, MIX_NONE, ProLoad<FD>, EpiLin<FD, FD, false, true>>(
                    g64(1), d(T64_E), lk64[1], nullptr, ProLoad<FD>{d(T64_E)},
                    EpiLin<FD, FD, false, true>{d(YH_O), d(BP_O), 1.0, -1.0}, kopt(m, false), s);  // C^dag w
            if (e != hipSuccess) return e;
            yh = BP_O;
        }
        e = launch_dwf<double, FD, LinkD18, true, MIX_SA, ProLoad<FD>, EpiStore<FD>>(
            g64(0), d(yh), lk64[0], s64(ST_M5), ProLoad<FD>{d(yh)}, EpiStore<FD>{d(T64_E)}, kopt(m, false), s);
        if (e != hipSuccess) return e;
        e = launch_dwf<double, FD, LinkD18, true, MIX_SA, ProLoad<FD>, EpiOuter<FD, FD, F, FY>>(
            g64(1), d(T64_E), lk64[1], s64(ST_M5), ProLoad<FD>{d(T64_E)},
            EpiOuter<FD, FD, F, FY>{d(BPP), d(yh), lo(L_R), ylo()}, kopt(m, true), s);
        if (e != hipSuccess) return e;
        return fin(g64(1).nblocks, FIN_OUTER, m);
    }
    // the outer residual of the slots in host mask mk, each with its form
    int outer_residual_masked(int mk) {
        const int n0 = upload_mask(M_F0, [&](int r) { return hmask[mk][r] && sl[r].form == DWF_SYSTEM_D; });
        const int n1 = upload_mask(M_F1, [&](int r) { return hmask[mk][r] && sl[r].form == DWF_SYSTEM_CCDAG; });
        if (upload_err != hipSuccess) {
            hipError_t e = upload_err;
            upload_err = hipSuccess;
            return fail(DWF_EDEVICE, std::string("slot mask upload: ") + hipGetErrorString(e));
        }
        hipError_t e = hipSuccess;
        if (n0) e = outer_residual(dmask[M_F0], DWF_SYSTEM_D);
        if (n1 && e == hipSuccess) e = outer_residual(dmask[M_F1], DWF_SYSTEM_CCDAG);
        if (e != hipSuccess) return fail(DWF_EDEVICE, std::string("outer residual: ") + hipGetErrorString(e));
        return DWF_OK;
    }
    // res = b - D x on one parity, |res|^2 into the block sums; yx = (Y x) of
    // the other parity, xx = X x of this one
    hipError_t true_res(int par, int yx, int b, int xx, const int* m) {
        return launch_dwf<double, FD, LinkD18, true, MIX_NONE, ProLoad<FD>, EpiTrueRes<FD, FD>>(
            g64(par), d(yx), lk64[par], nullptr, ProLoad<FD>{d(yx)}, EpiTrueRes<FD, FD>{d(b), d(xx)}, kopt(m, true), s);
    }

    // inner CG kernels
    // T: t1 = M5^T g5 r, once at the start of an inner cycle (afterwards
    // kernel D forms it for the next iteration)
    hipError_t kT(const int* live) {
        return launch_dwf<Real, F, LF, false, MIX_AS, ProLoad<F>, EpiStore<F>>(
            glo(1), lo(L_R), lk[1], slo(ST_M5TG5), ProLoad<F>{lo(L_R)}, EpiStore<F>{lo(L_T1)}, kopt_in(live, false), s);
    }
    // E: p = c_r r + beta p, t1 = M5^T g5 p for the slots of list l (those
    // that solve C C^dag w = b), in ng groups
    hipError_t kE(const int* live, int l, int ng) {
        return launch_dwf<Real, F, LF, false, MIX_AS, ProCgE<F, F>, EpiStore<F>>(
            glo(1), lo(L_R), lk[1], slo(ST_M5TG5), ProCgE<F, F>{lo(L_R), lo(L_P), w.st.beta, w.st.ecr},
            EpiStore<F>{lo(L_T1)}, KOpt{live, nullptr, K, TS, kgroup, dlist[l], ng}, s);
    }
    hipError_t kA(const int* live) {
        return launch_dwf<Real, F, LF, true, MIX_AS, ProLoad<F>, EpiStore<F>>(
            glo(0), lo(L_T1), lk[0], slo(ST_M5T), ProLoad<F>{lo(L_T1)}, EpiStore<F>{lo(L_T23)}, kopt_in(live, false), s);
    }
    hipError_t kB(const int* live) {
        return launch_dwf<Real, F, LF, true, MIX_NONE, ProLoad<F>, EpiCgB<F, F>>(
            glo(1), lo(L_T23), lk[1], nullptr, ProLoad<F>{lo(L_T23)},
            EpiCgB<F, F>{lo(L_R), lo(L_U), lo(L_P).ptrs(), w.st.beta, w.st.ecr, dmask[M_FORM]}, kopt_in(live, true), s);
    }
    // C also finishes kernel B's reduction (alpha) in its first workgroups
    hipError_t kC(const int* live) {
        return launch_dwf<Real, F, LF, true, MIX_SA, ProLoad<F>, EpiStoreAlpha<F>>(
            glo(0), lo(L_U), lk[0], slo(ST_M5), ProLoad<F>{lo(L_U)},
            EpiStoreAlpha<F>{lo(L_T23), part(), glo(1).nblocks, st_dev.as<CgState>()}, kopt_in(live, false), s);
    }
    hipError_t kD(const int* live) {
        return launch_dwf<Real, F, LF, true, MIX_SA, ProLoad<F>, EpiCgD<F, F, FY>>(
            glo(1), lo(L_T23), lk[1], slo(ST_M5), ProLoad<F>{lo(L_T23)},
            EpiCgD<F, F, FY>{lo(L_U), lo(L_R), ylo(), w.st.alpha, lo(L_P).ptrs(), dmask[M_FORM], lo(L_T1).ptrs(),
                             (int)(slo(ST_M5TG5) - slo(ST_M5))},
            kopt_in(live, true), s);
    }
    hipError_t iteration() {
        hipError_t e;
        const int* live = w.st.live;
        if (cur_ng1 && (e = kE(live, LIST_F1, cur_ng1)) != hipSuccess) return e;
        if ((e = kA(live)) != hipSuccess) return e;
        if ((e = kB(live)) != hipSuccess) return e;
        if ((e = kC(live)) != hipSuccess) return e;
        if ((e = kD(live)) != hipSuccess) return e;
        return fin(glo(1).nblocks, FIN_BETA);
    }
    // one graph of kItersPerGraph iterations over cur_list / cur_ng, built
    // node by node (no stream capture); cached per group count.  The nodes read
    // the slot list and the CG state on the device, so replays need no update.
    int graph_for(hipGraphExec_t* out) {
        const long key = (long)cur_ng * (K + 1) + cur_ng1;
        auto it = graphs.find(key);
        if (it != graphs.end()) {
            *out = it->second.second;
            return DWF_OK;
        }
        GraphBuilder b;
        DWF_HIP(hipGraphCreate(&b.graph, 0));
        tl_builder = &b;
        hipError_t e = hipSuccess;
        for (int i = 0; i < kItersPerGraph && e == hipSuccess; ++i) e = iteration();
        tl_builder = nullptr;
        if (e != hipSuccess) {
            (void)hipGraphDestroy(b.graph);
            return fail(DWF_EDEVICE, std::string("graph build: ") + hipGetErrorString(e));
        }
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, b.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(b.graph);
            return fail(DWF_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
        graphs[key] = {b.graph, ex};
        *out = ex;
        return DWF_OK;
    }

#define CKE(x)                                                                                          \
    do {                                                                                                \
        hipError_t e_ = (x);                                                                            \
        if (e_ != hipSuccess) return fail(DWF_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)
#define CKR(x)             \
    do {                   \
        int r_ = (x);      \
        if (r_) return r_; \
    } while (0)
#define CKU()                                                                                                  \
    do {                                                                                                       \
        if (upload_err != hipSuccess) {                                                                        \
            hipError_t e_ = upload_err;                                                                        \
            upload_err = hipSuccess;                                                                           \
            return fail(DWF_EDEVICE, std::string("slot mask upload: ") + hipGetErrorString(e_));              \
        }                                                                                                      \
    } while (0)

    // ---- b -> |b|^2, b' = S1 b, b'' = b'_o - M5 D^OE b'_e, |b''|^2, initial yhat_o
    int setup() {
        int* m = dmask[M_SETUP];
        upload_mask(M_SETUP, [&](int r) { return sl[r].phase == PH_SETUP; });
        const int n0 = upload_mask(M_SETUP0, [&](int r) { return hmask[M_SETUP][r] && sl[r].form == DWF_SYSTEM_D; });
        const int n1 =
            upload_mask(M_SETUP1, [&](int r) { return hmask[M_SETUP][r] && sl[r].form == DWF_SYSTEM_CCDAG; });
        // the per-slot form flag that kernel D reads
        upload_mask(M_FORM, [&](int r) {
            return (hmask[M_SETUP][r] ? sl[r].form : (sl[r].phase == PH_FREE ? 0 : sl[r].form)) == DWF_SYSTEM_CCDAG;
        });
        CKU();
        CKE(norm64(0, B_E, m));
        CKE(fin(g64(0).nblocks, FIN_AUX, m));
        CKR(pull());
        for (int r = 0; r < K; ++r)
            if (hmask[M_SETUP][r]) sl[r].bnorm2 = sl[r].form == DWF_SYSTEM_D ? h_aux(r) : 0.0;  // even part of b
        CKE(norm64(1, B_O, m));
        CKE(fin(g64(1).nblocks, FIN_AUX, m));
        CKR(pull());
        for (int r = 0; r < K; ++r)
            if (hmask[M_SETUP][r]) sl[r].bnorm2 += h_aux(r);
        // initial yhat_o: (S2^-1 x0)_o for D x = b, the odd part of w0 for C C^dag w = b, else 0
        const int ng = upload_mask(M_GUESS, [&](int r) { return hmask[M_SETUP0][r] && sl[r].use_guess; });
        const int ng1 = upload_mask(M_GUESS1, [&](int r) { return hmask[M_SETUP1][r] && sl[r].use_guess; });
        const int nz = upload_mask(M_NOGUESS, [&](int r) { return hmask[M_SETUP][r] && !sl[r].use_guess; });
        CKU();
        if (ng) CKE(local64(1, BP_O, TB_S2INV, YH_O, dmask[M_GUESS]));
        if (ng1) CKE(half_copy(c, w.f(YH_O), w.f(BP_O), K, dmask[M_GUESS1], s));
        if (nz) CKE(half_zero(c, w.f(YH_O), K, s, dmask[M_NOGUESS]));
        if (n1) {
            // C C^dag w = b: b'' is the odd part of b; B_E becomes the zero even half of w
            CKE(half_copy(c, w.f(BPP), w.f(B_O), K, dmask[M_SETUP1], s));
            CKE(half_zero(c, w.f(B_E), K, s, dmask[M_SETUP1]));
        }
        if (n0) {
            CKE(local64(0, B_E, TB_S1, BP_E, dmask[M_SETUP0]));
            CKE(local64(1, B_O, TB_S1, BP_O, dmask[M_SETUP0]));
            CKE(xmy_m5hop64(1, BP_E, BP_O, BPP, true, dmask[M_SETUP0]));
            CKE(fin(g64(1).nblocks, FIN_AUX, dmask[M_SETUP0]));
        }
        CKR(pull());
        for (int r = 0; r < K; ++r)
            if (hmask[M_SETUP][r]) {
                sl[r].bpp2 = sl[r].form == DWF_SYSTEM_D ? h_aux(r) : sl[r].bnorm2;
                sl[r].phase = PH_OUTER;
                h_live(r) = 0;
                h_iters(r) = 0;
                h_status(r) = 0;
                h_maxiter(r) = sl[r].p.maxiter;
                h_target(r) = 0;
            }
        return push_ctl();
    }

    // ---- outer step (Algorithm 2 with reliable updates) for the slots in PH_OUTER
    int outer() {
        int* m = dmask[M_OUTER];
        upload_mask(M_OUTER, [&](int r) { return sl[r].phase == PH_OUTER; });
        CKU();
        CKR(outer_residual_masked(M_OUTER));
        for (int r = 0; r < K; ++r)
            if (hmask[M_OUTER][r]) {
                sl[r].restarts++;
                sl[r].reverted = 0;
            }
        CKR(pull());
        // A cycle that did not lower the true residual is rejected: the
        // previous iterate (kept in YH_E) is restored, and reliable updates
        // give way to defect correction (Sec. 2.3's automatic switch).
        int nrev = upload_mask(M_REVERT, [&](int r) {
            return hmask[M_OUTER][r] && sl[r].have_backup && !(sqrt(h_aux(r)) < sl[r].rhat_prev);
        });
        CKU();
        if (nrev) {
            CKE(half_copy(c, w.f(YH_O), w.f(YH_E), K, dmask[M_REVERT], s));
            CKR(outer_residual_masked(M_REVERT));
            CKR(pull());
            for (int r = 0; r < K; ++r)
                if (hmask[M_REVERT][r]) {
                    SlotCtl& q = sl[r];
                    q.restarts++;
                    q.reverted = 1;
                    if (q.mode_ru) {
                        q.mode_ru = 0;
                        q.fellback = 1;
                    } else if (++q.noprog >= 4) {  // defect correction no longer converges
                        q.failed = 1;
                    }
                }
        }
        for (int r = 0; r < K; ++r) {
            if (!hmask[M_OUTER][r]) continue;
            SlotCtl& q = sl[r];
            const double rh2 = h_aux(r);
            const double rel = q.bpp2 > 0 ? sqrt(rh2 / q.bpp2) : 0.0;
            q.schur_res = rel;
            h_live(r) = 0;
            if (q.failed || !(rel > q.tol_schur) || !std::isfinite(rh2)) {
                if (!std::isfinite(rh2)) q.failed = 1;
                q.phase = PH_FINAL;
                continue;
            }
            if (q.cycles > 0 && !q.reverted) {
                if (q.mode_ru) {
                    // reliable-update stall test
                    const int st = h_status(r);
                    bool stalled = sqrt(rh2) > 0.5 * q.rhat_prev || st == 2 || st == 4 ||
                                   (q.p.debug_stall_after > 0 && q.ru_restarts >= q.p.debug_stall_after);
                    if (stalled) {
                        q.mode_ru = 0;
                        q.fellback = 1;
                    } else {
                        ++q.ru_restarts;
                    }
                } else if (sqrt(rh2) > 0.9 * q.rhat_prev) {
                    if (++q.noprog >= 4) {
                        q.failed = 1;
                        q.phase = PH_FINAL;
                        continue;
                    }
                } else {
                    q.noprog = 0;
                }
            }
            if (h_iters(r) >= q.p.maxiter) {  // iteration cap over all cycles
                q.failed = 1;
                q.phase = PH_FINAL;
                continue;
            }
            q.rhat_prev = sqrt(rh2);
            const double eps = q.mode_ru ? q.eps_ru : q.eps_dc;
            const double stop = 0.5 * q.tol_schur * sqrt(q.bpp2);
            const double tgt = std::max(eps * sqrt(rh2), stop);
            h_target(r) = tgt * tgt;
            h_live(r) = 1;
            h_status(r) = 0;
            h_maxiter(r) = q.p.maxiter;
            // p := r on the first cycle, in defect correction and after a
            // rejected cycle (u = C^dag p and p zeroed below, c_r = 1,
            // beta = 0); reliable updates keep p (c_r = 0, beta = 1)
            const bool reset = q.cycles == 0 || !q.mode_ru || q.reverted;
            h_ecr(r) = reset ? 1.0 : 0.0;
            h_beta(r) = reset ? 0.0 : 1.0;
            hmask[M_RESET][r] = reset ? 1 : 0;
            ++q.cycles;
            q.phase = PH_INNER;
            q.stuck = 0;
            if (getenv("DWF_VERBOSE"))
                fprintf(stderr, "[dwf] slot %d cycle %d: |rhat|/|b''| = %.3e mode=%s iters=%d%s\n", r, q.cycles,
                        rel, q.mode_ru ? "RU" : "DC", h_iters(r), q.reverted ? " (reverted)" : "");
        }
        CKR(push_ctl());
        int nres = 0;
        for (int r = 0; r < K; ++r) {
            if (!(hmask[M_OUTER][r] && sl[r].phase == PH_INNER)) hmask[M_RESET][r] = 0;
            nres += hmask[M_RESET][r];
        }
        if (nres) {
            DWF_HIP(hipMemcpyAsync(dmask[M_RESET], hmask[M_RESET], (size_t)K * sizeof(int), hipMemcpyHostToDevice, s));
            CKE(half_zero(c, w.f(L_U), K, s, dmask[M_RESET]));
            CKE(half_zero(c, w.f(L_P), K, s, dmask[M_RESET]));
        }
        // t1 = M5^T g5 r of the new residual, for every slot that starts a cycle
        // (a kept direction multiplies it by c_r = 0: it must be finite)
        if (upload_mask(M_START, [&](int r) { return hmask[M_OUTER][r] && sl[r].phase == PH_INNER; })) {
            CKU();
            CKE(kT(dmask[M_START]));
        }
        CKU();
        return DWF_OK;
    }

    // ---- reconstruction y_e = b'_e - M5 D^EO y_o, x = S2 y, and |b - D x| / |b|
    int final_check() {
        upload_mask(M_FINAL, [&](int r) { return sl[r].phase == PH_FINAL; });
        const int n0 = upload_mask(M_FIN0, [&](int r) { return hmask[M_FINAL][r] && sl[r].form == DWF_SYSTEM_D; });
        CKU();
        const auto now = std::chrono::steady_clock::now();
        // C C^dag w = b: the last outer residual was b - C C^dag w in FP64
        for (int r = 0; r < K; ++r)
            if (hmask[M_FINAL][r] && sl[r].form == DWF_SYSTEM_CCDAG) {
                SlotCtl& q = sl[r];
                q.true_res = q.schur_res;
                q.phase = PH_DONE;
                q.seconds = std::chrono::duration<double>(now - q.t0).count();
            }
        if (!n0) return DWF_OK;
        int* m = dmask[M_FIN0];
        CKE(xmy_m5hop64(0, YH_O, BP_E, YH_E, false, m));
        CKE(local64(0, YH_E, TB_S2, BP_E, m));
        CKE(local64(1, YH_O, TB_S2, BP_O, m));
        // D x = X x + D_w (Y x) per parity: Y x -> YH_E (even), T64_E (odd);
        // X x -> BPP one parity at a time
        CKE(local64(0, BP_E, TB_Y, YH_E, m));
        CKE(local64(1, BP_O, TB_Y, T64_E, m));
        CKE(local64(0, BP_E, TB_X, BPP, m));
        CKE(true_res(0, T64_E, B_E, BPP, m));
        CKE(fin(g64(0).nblocks, FIN_AUX, m));
        CKR(pull());
        std::vector<double> tr(K, 0.0);
        for (int r = 0; r < K; ++r) tr[r] = h_aux(r);
        CKE(local64(1, BP_O, TB_X, BPP, m));
        CKE(true_res(1, YH_E, B_O, BPP, m));
        CKE(fin(g64(1).nblocks, FIN_AUX, m));
        CKR(pull());
        for (int r = 0; r < K; ++r) {
            if (!hmask[M_FIN0][r]) continue;
            SlotCtl& q = sl[r];
            tr[r] += h_aux(r);
            q.true_res = q.bnorm2 > 0 ? sqrt(tr[r] / q.bnorm2) : sqrt(tr[r]);
            if (q.true_res > q.p.tol && !q.failed && q.schur_res <= q.tol_schur && std::isfinite(q.true_res) &&
                q.round < 5) {
                // tighten the Schur target and continue from the current iterate
                q.tol_schur *= std::max(0.01, 0.5 * q.p.tol / q.true_res);
                q.round++;
                q.have_backup = 0;  // YH_E was overwritten
                q.phase = PH_OUTER;
            } else {
                q.phase = PH_DONE;
                q.seconds = std::chrono::duration<double>(now - q.t0).count();
            }
        }
        // restore the pieces the reconstruction overwrote: b' and b''
        int na = upload_mask(M_AGAIN, [&](int r) { return hmask[M_FIN0][r] && sl[r].phase == PH_OUTER; });
        CKU();
        if (na) {
            CKE(local64(0, B_E, TB_S1, BP_E, dmask[M_AGAIN]));
            CKE(local64(1, B_O, TB_S1, BP_O, dmask[M_AGAIN]));
            CKE(xmy_m5hop64(1, BP_E, BP_O, BPP, false, dmask[M_AGAIN]));
        }
        return DWF_OK;
    }

    // ---- a run of inner iterations for every live slot, then the slots whose
    // inner cycle ended go on to the outer step
    int inner() {
        int check = 0;
        for (int r = 0; r < K; ++r)
            if (sl[r].phase == PH_INNER && sl[r].p.check_every > 0)
                check = check ? std::min(check, sl[r].p.check_every) : sl[r].p.check_every;
        const int cap = check ? std::max(1, (check + kItersPerGraph - 1) / kItersPerGraph) : replay_cap;
        const int nl = upload_list(LIST_INNER, [&](int r) { return sl[r].phase == PH_INNER; });
        const int n1 =
            upload_list(LIST_F1, [&](int r) { return sl[r].phase == PH_INNER && sl[r].form == DWF_SYSTEM_CCDAG; });
        CKU();
        use_list(LIST_INNER, nl);
        cur_ng1 = (n1 + kgroup - 1) / kgroup;
        volatile int* lh = (volatile int*)live_pin;
        for (int r = 0; r < K; ++r) lh[r] = sl[r].phase == PH_INNER ? 1 : 0;
        hipGraphExec_t ex = nullptr;
        int rc = use_graph ? graph_for(&ex) : DWF_OK;
        auto launch_one = [&]() -> int {
            if (use_graph)
                return hipGraphLaunch(ex, s) == hipSuccess ? DWF_OK : fail(DWF_EDEVICE, "hipGraphLaunch failed");
            for (int k = 0; k < kItersPerGraph; ++k)
                if (iteration() != hipSuccess) return fail(DWF_EDEVICE, "inner iteration launch failed");
            return DWF_OK;
        };
        // Replays until a slot of this round ends its cycle (or the cap): one
        // replay stays queued while the host checks the mirrored live flags
        // after the one before it, so a round overruns a slot's end by at
        // most one replay and the device never waits for the host.
        int n = 0;
        while (!rc && n < cap) {
            if ((rc = launch_one())) break;
            if (hipEventRecord(ev[n & 1], s) != hipSuccess) rc = fail(DWF_EDEVICE, "hipEventRecord failed");
            ++n;
            if (rc || n < 2) continue;
            if (hipEventSynchronize(ev[n & 1]) != hipSuccess) {  // replay n - 2 is done
                rc = fail(DWF_EDEVICE, "hipEventSynchronize failed");
                break;
            }
            bool ended = false;
            for (int r = 0; r < K; ++r) ended |= sl[r].phase == PH_INNER && lh[r] == 0;
            if (ended) break;
        }
        cur_list = nullptr;
        cur_ng1 = 0;
        if (rc) return rc;
        int nlive = 0;
        for (int r = 0; r < K; ++r) nlive += sl[r].phase == PH_INNER;
        prof.replays += n;
        prof.slot_iters_launched += (long)n * kItersPerGraph * nlive;
        std::vector<int> before(K);
        for (int r = 0; r < K; ++r) before[r] = h_iters(r);
        CKR(pull());
        for (int r = 0; r < K; ++r)
            if (sl[r].phase == PH_INNER) prof.slot_iters_done += h_iters(r) - before[r];
        if (verbose >= 2)
            for (int r = 0; r < K; ++r)
                if (sl[r].phase == PH_INNER)
                    fprintf(stderr, "[dwf]   round: %d replays; slot %d iters %d -> %d live=%d rr=%.3e target=%.3e\n",
                            n, r, before[r], h_iters(r), h_live(r), h_rr(r), h_target(r));
        bool ended = false;
        for (int r = 0; r < K; ++r) {
            if (sl[r].phase != PH_INNER) continue;
            SlotCtl& q = sl[r];
            if (!h_live(r)) {
                ended = true;
                continue;
            }
            // the device stops every slot at maxiter; this only trips if the
            // device state stops advancing
            if (h_iters(r) == before[r] && ++q.stuck >= 3) return fail(DWF_EDEVICE, "inner solve does not advance");
        }
        if (ended) CKR(post_cycle());
        return DWF_OK;
    }

    // the slots whose inner cycle ended: finish the direction for reliable
    // updates, keep yhat (backup), yhat += y
    int post_cycle() {
        int nfin = upload_mask(M_RUFIN, [&](int r) {
            return sl[r].phase == PH_INNER && !h_live(r) && sl[r].mode_ru && h_status(r) == 1;
        });
        CKU();
        // reliable updates: the last direction update p = r + beta p
        // (Algorithm 1 computes p_{k+1} before testing convergence), as
        // u = C^dag r + beta u from the t1 = M5^T g5 r that kernel D left, or
        // (C C^dag w = b) p itself by kernel E, whose next cycle forms u
        if (nfin) {
            use_list(LIST_RUFIN, upload_list(LIST_RUFIN, [&](int r) { return hmask[M_RUFIN][r] != 0; }));
            const int n1 = upload_list(
                LIST_RUF1, [&](int r) { return hmask[M_RUFIN][r] != 0 && sl[r].form == DWF_SYSTEM_CCDAG; });
            CKU();
            hipError_t e = hipSuccess;
            if (n1) e = kE(dmask[M_RUFIN], LIST_RUF1, (n1 + kgroup - 1) / kgroup);
            if (n1 < nfin) {
                if (e == hipSuccess) e = kA(dmask[M_RUFIN]);
                if (e == hipSuccess) e = kB(dmask[M_RUFIN]);
            }
            cur_list = nullptr;
            CKE(e);
        }
        upload_mask(M_POST, [&](int r) { return sl[r].phase == PH_INNER && !h_live(r); });
        CKU();
        CKE(half_copy(c, w.f(YH_E), w.f(YH_O), K, dmask[M_POST], s));
        CKE(half_acc(c, w.f(YH_O), w.f(L_Y), K, dmask[M_POST], s));
        for (int r = 0; r < K; ++r) {
            if (!hmask[M_POST][r]) continue;
            SlotCtl& q = sl[r];
            q.have_backup = 1;
            if (h_status(r) == 2 && !q.mode_ru) {  // breakdown in defect correction: give up
                q.failed = 1;
                q.phase = PH_FINAL;
            } else {
                q.phase = PH_OUTER;
            }
        }
        return DWF_OK;
    }
#undef CKE
#undef CKR
#undef CKU
};

template <class Real, class F, class FY, class LF>
int Engine<Real, F, FY, LF>::time_kernels(int launches, double* ms, double* bytes) {
    // all kernels forced on (live = NULL); T, A and C are idempotent, B and D
    // update their outputs from finite inputs
    auto runk = [&](int k) -> hipError_t {
        switch (k) {
            case 0: return kT(nullptr);
            case 1: return kA(nullptr);
            case 2: return kB(nullptr);
            case 3: return kC(nullptr);
            default: return kD(nullptr);
        }
    };
    // One iteration's kernels (A B C D) run back to back `launches` times, so
    // that each finds the caches as the iteration before leaves them, then T
    // (once per cycle in a solve) `launches` times; one event pair around
    // every launch, so the averages are the kernels' own device time.
    const int nk = 5;
    std::vector<hipEvent_t> ev(2 * (size_t)launches * nk, nullptr);
    for (auto& e : ev) DWF_HIP(hipEventCreate(&e));
    const double sb = spinor_bytes(prec) * (double)c->V5h * K;
    const double yb = (prec == DWF_PREC_FP64 ? 192.0 : 96.0) * (double)c->V5h * K;
    const double lb = (double)c->V4h * 8.0 * link_bytes(link_fmt);
    const double model[5] = {2 * sb, 2 * sb + lb, 4 * sb + lb, 2 * sb + lb, 5 * sb + 2 * yb + lb};
    int result = DWF_OK;
    hipError_t e = hipSuccess;
    for (int k = 0; k < nk && e == hipSuccess; ++k) e = runk(k);  // warm-up
    auto timed = [&](int i, int k) {
        const size_t j = 2 * ((size_t)i * nk + k);
        e = hipEventRecord(ev[j], s);
        if (e == hipSuccess) e = runk(k);
        if (e == hipSuccess) e = hipEventRecord(ev[j + 1], s);
    };
    for (int i = 0; i < launches && e == hipSuccess; ++i)
        for (int k = 1; k < nk && e == hipSuccess; ++k) timed(i, k);
    for (int i = 0; i < launches && e == hipSuccess; ++i) timed(i, 0);
    if (e == hipSuccess) e = hipEventSynchronize(ev[2 * ((size_t)(launches - 1) * nk) + 1]);
    for (int k = 0; k < nk && e == hipSuccess; ++k) {
        double tot = 0;
        for (int i = 0; i < launches && e == hipSuccess; ++i) {
            const size_t j = 2 * ((size_t)i * nk + k);
            float t = 0;
            e = hipEventElapsedTime(&t, ev[j], ev[j + 1]);
            tot += t;
        }
        ms[k] = tot / launches;
        bytes[k] = model[k];
    }
    if (e != hipSuccess) result = fail(DWF_EDEVICE, std::string("kernel timing: ") + hipGetErrorString(e));
    for (auto& e : ev) (void)hipEventDestroy(e);
    return result;
}

template <class Real, class F, class FY, class LF>
int build(dwf_ctx* c, int prec, int fmt, int K, hipStream_t s, LF e, LF o, int tile,
          std::unique_ptr<EngineBase>* out) {
    std::unique_ptr<Engine<Real, F, FY, LF>> eng(new Engine<Real, F, FY, LF>(c, prec, fmt, K, s, e, o, tile - 1));
    int rc = eng->init();
    if (rc) return rc;
    *out = std::move(eng);
    return DWF_OK;
}

std::string engine_key(const dwf_ctx* c, const dwf_solve_params& p, int nrhs) {
    return "solve:" + std::to_string(p.inner_prec) + ":" + std::to_string(link_format(c, p)) + ":t" +
           std::to_string(p.tile) + ":" +
           std::to_string(nrhs);
}

}  // namespace

int make_engine(dwf_ctx* c, const dwf_solve_params& p, int K, hipStream_t s, std::unique_ptr<EngineBase>* out) {
    switch (p.inner_prec) {
        case DWF_PREC_FP64:
            return build<double, FD, FD, LinkD18>(c, DWF_PREC_FP64, LINK_D18, K, s,
                                                  LinkD18{c->links[0][LINK_D18].as<double>()},
                                                  LinkD18{c->links[1][LINK_D18].as<double>()}, p.tile, out);
        case DWF_PREC_FP32:
            if (link_format(c, p) == LINK_S12)
                return build<float, FS, FS, LinkS12>(c, DWF_PREC_FP32, LINK_S12, K, s,
                                                     LinkS12{c->links[0][LINK_S12].as<float>()},
                                                     LinkS12{c->links[1][LINK_S12].as<float>()}, p.tile, out);
            return build<float, FS, FS, LinkS18>(c, DWF_PREC_FP32, LINK_S18, K, s,
                                                 LinkS18{c->links[0][LINK_S18].as<float>()},
                                                 LinkS18{c->links[1][LINK_S18].as<float>()}, p.tile, out);
        default:
            return build<float, FH, FS, LinkH12>(c, DWF_PREC_FP16, LINK_H12, K, s,
                                                 LinkH12{c->links[0][LINK_H12].as<_Float16>()},
                                                 LinkH12{c->links[1][LINK_H12].as<_Float16>()}, p.tile, out);
    }
}

size_t engine_bytes(const dwf_ctx* c, int prec, int K) {
    const long lo = field_elems(c->V5h, prec);
    const long y = field_elems(c->V5h, prec == DWF_PREC_FP64 ? DWF_PREC_FP64 : DWF_PREC_FP32);
    const long f64 = field_elems(c->V5h, DWF_PREC_FP64);
    size_t per = ((size_t)NF64 * f64 + 5 * (size_t)lo + (size_t)y) * 16;
    if (prec == DWF_PREC_FP16) per += 5 * (size_t)(((c->V5h + 1023) / 1024) * 1024) * sizeof(float);
    size_t nb = (size_t)c->geom(0, true).nblocks;
    for (auto& t : tile_candidates(c, prec == DWF_PREC_FP64))
        nb = std::max(nb, (size_t)c->geom_tile(0, t.G, t.order).nblocks);
    per += tables_size(c->Ns) * 12 + nb * sizeof(double) + 96;
    return per * (size_t)K;
}

int solve(dwf_ctx* c, const double* b_dev, double* x_dev, int nrhs, const dwf_solve_params& p,
          dwf_solve_stats* stats, hipStream_t s, const HostIO* hio) {
    const std::string key = engine_key(c, p, nrhs);
    auto& slot = c->engines[key];
    if (!slot) {
        int rc = make_engine(c, p, nrhs, s, &slot);
        if (rc) {
            slot.reset();
            return rc;
        }
    }
    EngineBase* eng = slot.get();
    eng->set_stream(s);
    eng->set_use_graph(p.use_graph != 0);
    const long n5 = c->V4 * c->Ns * 24;

    hipEvent_t ev0, ev1;
    DWF_HIP(hipEventCreate(&ev0));
    DWF_HIP(hipEventCreate(&ev1));
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
    } evg{ev0, ev1};
    DWF_HIP(hipEventRecord(ev0, s));

    // after an error the engine's slots are in an unknown state: drop it
    auto abandon = [&](int rc) {
        std::string msg = dwf_last_error();
        (void)hipStreamSynchronize(s);
        c->engines.erase(key);
        return fail(rc, msg);
    };
    int rc;
    for (int r = 0; r < nrhs; ++r) {
        const double* b_r = hio ? hio->stage_in : b_dev + r * n5;
        const double* x0_r = hio ? hio->stage_out : x_dev + r * n5;
        if (hio) {  // one right-hand side (and guess) at a time through the staging spinors
            if (hipMemcpyAsync(hio->stage_in, hio->in + r * n5, n5 * sizeof(double), hipMemcpyHostToDevice, s) !=
                    hipSuccess ||
                (p.use_guess && hipMemcpyAsync(hio->stage_out, hio->out + r * n5, n5 * sizeof(double),
                                               hipMemcpyHostToDevice, s) != hipSuccess))
                return abandon(fail(DWF_EDEVICE, "upload of b or the guess failed"));
        }
        if ((rc = eng->admit(r, b_r, p.use_guess ? x0_r : nullptr, c->mq, p))) return abandon(rc);
        // the staging spinors are reused by the next right-hand side
        if (hio && hipStreamSynchronize(s) != hipSuccess) return abandon(fail(DWF_EDEVICE, "admission failed"));
    }
    // every tick either advances a slot's phase or runs inner iterations,
    // which end at the device-side iteration cap
    while (eng->pending() > 0)
        if ((rc = eng->tick())) return abandon(rc);
    std::vector<SlotResult> res(nrhs);
    for (int r = 0; r < nrhs; ++r) {
        if ((rc = eng->retire(r, hio ? hio->stage_out : x_dev + r * n5, &res[r]))) return abandon(rc);
        if (hio && (hipMemcpyAsync(hio->out + r * n5, hio->stage_out, n5 * sizeof(double), hipMemcpyDeviceToHost,
                                   s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess))
            return abandon(fail(DWF_EDEVICE, "download of x failed"));
    }
    eng->report();
    DWF_HIP(hipEventRecord(ev1, s));
    DWF_HIP(hipEventSynchronize(ev1));
    float ms = 0;
    DWF_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    int status = DWF_OK;
    double flops = 0, bytes = 0;
    for (int r = 0; r < nrhs; ++r) {
        if (res[r].status != DWF_OK) status = DWF_ENOCONV;
        flops += res[r].flops;
        bytes += res[r].bytes;
    }
    if (stats) {
        for (int r = 0; r < nrhs; ++r) {
            dwf_solve_stats& o = stats[r];
            memset(&o, 0, sizeof(o));
            o.status = res[r].status;
            o.iters = res[r].iters;
            o.restarts = res[r].restarts;
            o.reliable_updates = res[r].reliable_updates;
            o.fallback = res[r].fallback;
            o.rhs_per_block = eng->rhs_per_block();
            eng->tile(&o.tile, &o.sites_per_block, &o.block_order);
            o.tile += 1;
            o.true_residual = res[r].true_residual;
            o.schur_residual = res[r].schur_residual;
            // the batch shares the device: time, rate and bytes are the batch's
            o.seconds = ms * 1e-3;
            o.gflops = o.seconds > 0 ? flops / o.seconds * 1e-9 : 0;
            o.hbm_gbytes = bytes * 1e-9;
        }
    }
    if (status != DWF_OK) fail(DWF_ENOCONV, "solve did not reach the requested tolerance");
    return status;
}

int time_inner_kernels(dwf_ctx* c, const dwf_solve_params& p, int nrhs, int launches, double* ms, double* bytes) {
    auto it = c->engines.find(engine_key(c, p, nrhs));
    if (it == c->engines.end() || !it->second)
        return fail(DWF_EINVAL, "no solve workspace for these parameters; run a solve first");
    it->second->set_stream(c->stream);
    return it->second->time_kernels(launches, ms, bytes);
}

}  // namespace dwf
