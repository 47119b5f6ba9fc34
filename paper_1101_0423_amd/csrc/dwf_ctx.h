// dwf_ctx.h -- host-side context of libdwf: resident gauge field in its
// device formats, fifth-dimension tables, workspaces, and the launch helpers
// used by the operator, solver and server code.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <condition_variable>
#include <string>
#include <vector>

#include "../../include/dwf.h"
#include "dwf_device.h"
#include "fifth_dim.h"

namespace dwf {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define DWF_HIP(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return ::dwf::fail(e_ == hipErrorOutOfMemory ? DWF_ENOMEM : DWF_EDEVICE,            \
                               std::string(#call) + ": " + hipGetErrorString(e_));             \
    } while (0)

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    bool own = true;  // false: a view of memory owned elsewhere (never freed here)
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    int alloc(size_t n);
    void view(void* q, size_t n) {
        release();
        p = q;
        bytes = n;
        own = false;
    }
    void release();
    template <class T>
    T* as() const { return (T*)p; }
};

// Block orders of the stencil workgroups (dwf_ctx::geom_tile); w >= 2 means
// t-fastest with z-plane tiles of w blocks.
enum BlockOrder { ORDER_AUTO = -1, ORDER_PLAIN = 0, ORDER_TFAST = 1 };

// Link formats held per parity.
enum LinkFmt { LINK_D18 = 0, LINK_S18 = 1, LINK_S12 = 2, LINK_H12 = 3, LINK_NFMT = 4 };

// The packed gauge links of one field in every format, per output parity.
// Contexts built on the same field (same content, extents and device) share
// one LinkSet: the links do not depend on Ns, the masses or the boundary
// condition in t, which the kernels apply themselves.
struct LinkSet {
    DevBuf buf[2][LINK_NFMT];  // [output parity][format]
};

// Tables of one quark mass (the mass enters through L's corner).
struct TableSet {
    double mq = 0;
    std::vector<double> host;  // tables_size(Ns) reals (fifth_dim.h)
    DevBuf d64, d32;
    const double* t64(int t, int Ns) const { return d64.as<double>() + dense_table_offset(Ns, t); }
    const float* t32(int t, int Ns) const { return d32.as<float>() + dense_table_offset(Ns, t); }
    const double* s64(int st, int Ns) const { return d64.as<double>() + struct_table_offset(Ns, st); }
    const float* s32(int st, int Ns) const { return d32.as<float>() + struct_table_offset(Ns, st); }
};

// A half field (one parity) of nrhs right-hand sides in a given precision,
// site-major: [rhs][h4][component block][Ns] (see the accessors).
struct HalfField {
    int prec = DWF_PREC_FP64;
    long ns = 0;       // Ns
    long rstride = 0;  // elements (16-byte vectors) between right-hand sides
    long nstride = 0;  // FP16 norms between right-hand sides
    int nrhs = 0;
    DevBuf data, nrm;
    int alloc(int prec, long V5h, int Ns, int nrhs);
    // bytes of the data and norm arrays of such a field (each a multiple of 256)
    static void sizes(int prec, long V5h, int nrhs, size_t* data_bytes, size_t* nrm_bytes);
    // the same field laid out in caller-owned device memory (data, then norms)
    void place(int prec, long V5h, int Ns, int nrhs, unsigned char* mem);
    FD fd(int rhs0 = 0) const { return FD{data.as<double2>() + rhs0 * rstride, ns, rstride}; }
    FS fs(int rhs0 = 0) const { return FS{data.as<float4>() + rhs0 * rstride, ns, rstride}; }
    FH fh(int rhs0 = 0) const {
        return FH{data.as<uint4>() + rhs0 * rstride, nrm.as<float>() + rhs0 * nstride, ns, rstride, nstride};
    }
};

// Device workspace of one kind of call (operator application or solve) for
// a given precision and number of right-hand sides; kept by the context.
struct Workspace {
    std::vector<std::unique_ptr<HalfField>> fields;
    DevBuf state;           // CgState arrays
    CgState st{};
    int nrhs = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int graph_iters = 0;
    ~Workspace() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
    }
    HalfField& f(int i) { return *fields[i]; }
    // allocate n fields: precs[i] for field i
    int alloc(const std::vector<int>& precs, long V5h, int Ns, int nrhs_);
    int alloc_state(int nrhs_, hipStream_t s);
};

// Phases of one right-hand side ("slot") of a solve engine.
enum SlotPhase { PH_FREE = 0, PH_SETUP, PH_OUTER, PH_INNER, PH_FINAL, PH_DONE };

// Outcome of one slot, read when it is retired.
struct SlotResult {
    int status = DWF_OK;
    int iters = 0, restarts = 0, reliable_updates = 0, fallback = 0;
    double true_residual = 0, schur_residual = 0;
    double seconds = 0;  // host wall time from admission to the final check
    double flops = 0;    // paper-convention flops of this right-hand side
    double bytes = 0;    // algorithmic HBM bytes of this right-hand side
};

// A solve engine: K slots that share the multi-right-hand-side kernels of one
// operator, inner precision and link format.  Each slot carries its own
// quark mass, tolerances and outer-loop state, and can be admitted or retired
// while the others iterate.  All work goes to one HIP stream.
class EngineBase {
  public:
    virtual ~EngineBase() {}
    virtual int capacity() const = 0;
    virtual int rhs_per_block() const = 0;  // tuned right-hand sides per stencil workgroup
    // the tuned tile of the inner kernels: candidate index (0-based), 4D sites
    // per workgroup, block order (BlockOrder or tile width)
    virtual void tile(int* index, int* sites, int* order) const = 0;
    virtual int phase(int slot) const = 0;
    virtual int busy() const = 0;  // slots not free
    virtual int pending() const = 0;  // slots neither free nor done
    virtual void set_stream(hipStream_t s) = 0;
    virtual void set_use_graph(bool on) = 0;
    virtual void set_replay_cap(int n) = 0;  // graph replays per round (default 64)
    // Convert one right-hand side (device, host layout) into the slot; x0 is
    // an initial guess (device, host layout) or NULL.
    virtual int admit(int slot, const double* b_dev, const double* x0_dev, double mq,
                      const dwf_solve_params& p) = 0;
    // One scheduling round: setup, outer steps, reconstructions, and a run of
    // inner iterations for every live slot.  Ends with the stream idle.
    virtual int tick() = 0;
    // Write the solution of a PH_DONE slot (device, host layout) and free it.
    virtual int retire(int slot, double* x_dev, SlotResult* res) = 0;
    virtual int time_kernels(int launches, double* ms, double* bytes) = 0;
    virtual size_t device_bytes() const = 0;
    virtual void report() = 0;  // time accounting to stderr when DWF_VERBOSE is set
};

int make_engine(dwf_ctx* c, const dwf_solve_params& p, int K, hipStream_t s, std::unique_ptr<EngineBase>* out);
// a tile of the inner kernels: G sites per workgroup, requested block order,
// the order its geometry walks (BlockOrder or tile width)
struct TileCand {
    int G, order, eff;
};
std::vector<TileCand> tile_candidates(const dwf_ctx* c, bool fp64);
// link format of an inner solve: the params' choice, with auto resolved by the
// field's SU(3) check (12-real only for SU(3) fields)
int link_format(const dwf_ctx* c, const dwf_solve_params& p);
// rejects parameters that the field or the library cannot serve (DWF_EINVAL)
int check_params(const dwf_ctx* c, const dwf_solve_params& p);
// max over links of |row 2 - conj(row 0 x row 1)| (+inf for non-finite entries)
double su3_deviation(const double* gauge, long nlinks);
// device bytes of an engine with K slots (fields, tables, state, reductions)
size_t engine_bytes(const dwf_ctx* c, int inner_prec, int K);

}  // namespace dwf

struct dwf_ctx {
    int dims[4];
    int Ns;
    double m0, mq;
    std::vector<double> sigma, omega;
    dwf_opts opts;
    int device;
    hipStream_t stream = nullptr;
    hipStream_t xfer = nullptr;  // table uploads (never a legacy-stream operation: other
                                 // threads may be capturing graphs)
    long V4, V4h, V5h;
    int G64, G32;  // 4D sites per workgroup for FP64 and FP32/FP16 kernels
    std::shared_ptr<dwf::LinkSet> lset;
    dwf::DevBuf (*links)[dwf::LINK_NFMT] = nullptr;  // lset->buf: [output parity][format]
    std::map<double, std::unique_ptr<dwf::TableSet>> tables;
    std::mutex tables_mtx;  // the table map is shared with the server's threads
    std::mutex mtx;  // one call at a time per context
    std::map<std::string, std::unique_ptr<dwf::Workspace>> ws;
    std::map<std::string, std::unique_ptr<dwf::EngineBase>> engines;  // dwf_solve engines by kind
    dwf::DevBuf partials;  // block sums
    size_t partials_bytes = 0;
    std::string gauge_key;
    double su3_dev = 0;    // su3_deviation of the field
    bool su3 = true;       // su3_dev <= DWF_SU3_TOL: 12-real links are exact
    dwf::DevBuf stage;     // host-pointer forms: one spinor in, one out (FP64, host layout)
    dwf::DevBuf prop_ws;   // propagator: wall source, 5D source and 5D solution per source

    dwf::Geom geom(int out_parity, bool fp64) const;
    dwf::Geom geom_tile(int out_parity, int G, int order) const;
    const dwf::TableSet* table_set(double mq_val, int* rc);
    int ensure_partials(size_t nblocks_times_nrhs);
    long spinor_elems() const { return V4 * Ns * 24; }
    // the two staging spinors of the host-pointer forms (allocated once)
    int ensure_stage(double** in, double** out);
};

namespace dwf {

// ---------------------------------------------------------------------------
// kernel launch helper (template; instantiated where used)
// ---------------------------------------------------------------------------

inline int round_up(int a, int b) { return (a + b - 1) / b * b; }

// Explicit graph construction.  While a GraphBuilder is active on a thread,
// the launch helpers append kernel nodes (each depending on the previous one)
// instead of launching.  No stream is captured, so other threads keep full use
// of the device (HIP refuses legacy-stream work while any stream captures).
struct GraphBuilder {
    hipGraph_t graph = nullptr;
    hipGraphNode_t last = nullptr;
    hipError_t err = hipSuccess;
};
inline thread_local GraphBuilder* tl_builder = nullptr;

template <class... Args>
hipError_t launch_kernel(void (*kern)(Args...), dim3 grid, dim3 block, size_t smem, hipStream_t st,
                         Args... args) {
    GraphBuilder* b = tl_builder;
    if (!b) {
        hipLaunchKernelGGL(kern, grid, block, smem, st, args...);
        return hipGetLastError();
    }
    if (b->err != hipSuccess) return b->err;
    void* params[] = {(void*)&args...};  // values are copied into the node
    hipKernelNodeParams kp{};
    kp.func = (void*)kern;
    kp.gridDim = grid;
    kp.blockDim = block;
    kp.sharedMemBytes = (unsigned)smem;
    kp.kernelParams = params;
    kp.extra = nullptr;
    hipGraphNode_t node = nullptr;
    b->err = hipGraphAddKernelNode(&node, b->graph, b->last ? &b->last : nullptr, b->last ? 1 : 0, &kp);
    if (b->err == hipSuccess) b->last = node;
    return b->err;
}

template <class Real, class F, class LF, bool HOP, int MIXM, class Pro, class Epi>
hipError_t launch_dwf(const Geom& g0, const F& in, const LF& links, const Real* table, const Pro& pro,
                      const Epi& epi, KOpt o, hipStream_t st) {
    // The t-fastest block order serves the hop's neighbour re-reads from L2; a
    // kernel without a hop streams its blocks in plain order (each XCD one
    // contiguous range), which measured 7% faster for the streaming kernels.
    Geom g = g0;
    if constexpr (!HOP) g.nsb = 0;
    int T = round_up(g.G * g.Ns, 64);
    // Ns = 8, 16 or 32 with a recurrence-form M5 / M5^T: applied in registers, no LDS buffer
    constexpr bool STRUCT = MIXM == MIX_SA || MIXM == MIX_AS;
    const bool reg = STRUCT && (g.Ns == 8 || g.Ns == 16 || g.Ns == 32);
    size_t sm = kernel_smem<Real>(g.G, g.Ns, HOP, MIXM != MIX_NONE && !reg);
    const int rpb = o.rpb > 0 && o.rpb < o.nrhs ? o.rpb : o.nrhs;
    o.rpb = rpb;
    const unsigned ng = o.ngroups > 0 ? (unsigned)o.ngroups : (unsigned)((o.nrhs + rpb - 1) / rpb);
    const dim3 grid((unsigned)g.nblocks * ng), block(T);
    if (g.Ns <= 8) {
        if constexpr (STRUCT)
            if (reg)
                return launch_kernel(k_dwf<Real, F, LF, 8, HOP, MIXM, true, Pro, Epi>, grid, block, sm, st, g, in,
                                     links, table, pro, epi, o);
        return launch_kernel(k_dwf<Real, F, LF, 8, HOP, MIXM, false, Pro, Epi>, grid, block, sm, st, g, in, links,
                             table, pro, epi, o);
    }
    if (g.Ns <= 16) {
        if constexpr (STRUCT)
            if (reg)
                return launch_kernel(k_dwf<Real, F, LF, 16, HOP, MIXM, true, Pro, Epi>, grid, block, sm, st, g, in,
                                     links, table, pro, epi, o);
        return launch_kernel(k_dwf<Real, F, LF, 16, HOP, MIXM, false, Pro, Epi>, grid, block, sm, st, g, in, links,
                             table, pro, epi, o);
    }
    if constexpr (STRUCT)
        if (reg)
            return launch_kernel(k_dwf<Real, F, LF, 32, HOP, MIXM, true, Pro, Epi>, grid, block, sm, st, g, in,
                                 links, table, pro, epi, o);
    return launch_kernel(k_dwf<Real, F, LF, 32, HOP, MIXM, false, Pro, Epi>, grid, block, sm, st, g, in, links,
                         table, pro, epi, o);
}

// finish kernel modes
// (alpha is finished by kernel C's first workgroups, EpiStoreAlpha)
enum FinMode { FIN_AUX = 0, FIN_BETA = 2, FIN_OUTER = 3 };

// mask (per right-hand side, NULL = all) restricts FIN_AUX and FIN_OUTER
hipError_t launch_finish(const double* partials, int nblocks, int nrhs, CgState st, int mode, hipStream_t s,
                         const int* mask = nullptr);

// elementwise / layout kernels (layout.hip)
// rhs0: first right-hand side of the half fields that the conversion covers
hipError_t host_to_half(const dwf_ctx* c, const double* host, int nrhs, HalfField& even, HalfField& odd,
                        hipStream_t s, int rhs0 = 0);
hipError_t half_to_host(const dwf_ctx* c, const HalfField& even, const HalfField& odd, int nrhs, double* host,
                        hipStream_t s, int rhs0 = 0);
hipError_t half_convert(const dwf_ctx* c, const HalfField& src, HalfField& dst, int nrhs, hipStream_t s);
hipError_t half_zero(const dwf_ctx* c, HalfField& f, int nrhs, hipStream_t s, const int* mask = nullptr);
hipError_t half_copy(const dwf_ctx* c, HalfField& dst, const HalfField& src, int nrhs, const int* mask,
                     hipStream_t s);
hipError_t half_acc(const dwf_ctx* c, HalfField& yhat, const HalfField& y, int nrhs, const int* mask,
                    hipStream_t s);
hipError_t pack_links(const dwf_ctx* c, const double* gauge_dev, hipStream_t s);
// plain copy of bytes (a multiple of 16), cached or non-temporal accesses
hipError_t stream_copy(const void* src, void* dst, size_t bytes, bool nontemporal, hipStream_t s);

// Host-pointer operands of apply_op / solve: the spinors are copied one at a
// time through the context's staging buffers (stage_in, stage_out).
struct HostIO {
    const double* in;   // host, nrhs spinors
    double* out;        // host, nrhs spinors
    double* stage_in;   // device, one spinor
    double* stage_out;  // device, one spinor
};

// operator application on half fields (ops.hip).  prec may carry a DWF_LINKS_*
// storage; in_dev / out_dev are device spinors unless hio is given.
int apply_op(dwf_ctx* c, int op, int prec, const double* in_dev, double* out_dev, int nrhs, hipStream_t s,
             const HostIO* hio = nullptr);
// the same with the workspace in the library's static device scratch array
// (ops.hip): no device allocation; DWF_EINVAL when it does not fit
int apply_op_noalloc(dwf_ctx* c, int op, int prec, const double* in_dev, double* out_dev, int nrhs,
                     hipStream_t s);
// look up the scratch array's address on the current device (once per device)
int scratch_init(int device);

// the solver (solver.hip): nrhs right-hand sides, all with the context's mq;
// b_dev / x_dev are device spinors unless hio is given (hio->in = b, hio->out = x)
int solve(dwf_ctx* c, const double* b_dev, double* x_dev, int nrhs, const dwf_solve_params& p,
          dwf_solve_stats* stats, hipStream_t s, const HostIO* hio = nullptr);

// 4D propagators (prop.hip): out = R D^-1 W eta for nsrc 4D sources, device
// pointers in the host layouts
int propagator(dwf_ctx* c, const double* eta_dev, double* out_dev, int nsrc, const dwf_solve_params& p,
               dwf_solve_stats* stats, hipStream_t s);

// the request server (server.hip): stop and forget the context's engines
void server_detach(dwf_ctx* c);

int time_inner_kernels(dwf_ctx* c, const dwf_solve_params& p, int nrhs, int launches, double* ms, double* bytes);

// paper-convention flops and algorithmic bytes of one inner CG iteration
double flops_per_iter(const dwf_ctx* c);
double bytes_per_iter(const dwf_ctx* c, int inner_prec, int link_fmt);

}  // namespace dwf
