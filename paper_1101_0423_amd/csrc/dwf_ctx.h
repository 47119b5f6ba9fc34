// dwf_ctx.h -- host-side context of libdwf: resident gauge field in its
// device formats, fifth-dimension tables, workspaces, and the launch helpers
// used by the operator, solver and server code.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
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
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    int alloc(size_t n);
    void release();
    template <class T>
    T* as() const { return (T*)p; }
};

// Link formats held per parity.
enum LinkFmt { LINK_D18 = 0, LINK_S18 = 1, LINK_S12 = 2, LINK_H12 = 3, LINK_NFMT = 4 };

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
    int alloc_state(int nrhs_);
};

}  // namespace dwf

struct dwf_ctx {
    int dims[4];
    int Ns;
    double m0, mq;
    std::vector<double> sigma, omega;
    dwf_opts opts;
    int device;
    hipStream_t stream = nullptr;
    long V4, V4h, V5h;
    int G64, G32;  // 4D sites per workgroup for FP64 and FP32/FP16 kernels
    dwf::DevBuf links[2][dwf::LINK_NFMT];  // [output parity][format]
    std::map<double, std::unique_ptr<dwf::TableSet>> tables;
    std::mutex mtx;  // one call at a time per context
    std::map<std::string, std::unique_ptr<dwf::Workspace>> ws;
    dwf::DevBuf partials;  // block sums
    size_t partials_bytes = 0;
    std::string gauge_key;

    dwf::Geom geom(int out_parity, bool fp64) const;
    const dwf::TableSet* table_set(double mq_val, int* rc);
    int ensure_partials(size_t nblocks_times_nrhs);
};

namespace dwf {

// ---------------------------------------------------------------------------
// kernel launch helper (template; instantiated where used)
// ---------------------------------------------------------------------------

inline int round_up(int a, int b) { return (a + b - 1) / b * b; }

template <class Real, class F, class LF, bool HOP, int MIXM, class Pro, class Epi>
hipError_t launch_dwf(const Geom& g, const F& in, const LF& links, const Real* table, const Pro& pro,
                      const Epi& epi, KOpt o, hipStream_t st) {
    int T = round_up(g.G * g.Ns, 64);
    size_t sm = kernel_smem<Real>(g.G, g.Ns, HOP, MIXM != MIX_NONE);
    if (g.Ns <= 8)
        hipLaunchKernelGGL((k_dwf<Real, F, LF, 8, HOP, MIXM, Pro, Epi>), dim3(g.nblocks), dim3(T), sm, st, g, in,
                           links, table, pro, epi, o);
    else if (g.Ns <= 16)
        hipLaunchKernelGGL((k_dwf<Real, F, LF, 16, HOP, MIXM, Pro, Epi>), dim3(g.nblocks), dim3(T), sm, st, g, in,
                           links, table, pro, epi, o);
    else
        hipLaunchKernelGGL((k_dwf<Real, F, LF, 32, HOP, MIXM, Pro, Epi>), dim3(g.nblocks), dim3(T), sm, st, g, in,
                           links, table, pro, epi, o);
    return hipGetLastError();
}

// finish kernel modes
enum FinMode { FIN_AUX = 0, FIN_ALPHA = 1, FIN_BETA = 2, FIN_OUTER = 3 };

hipError_t launch_finish(const double* partials, int nblocks, int nrhs, CgState st, int mode, hipStream_t s);

// elementwise / layout kernels (layout.hip)
hipError_t host_to_half(const dwf_ctx* c, const double* host, int nrhs, HalfField& even, HalfField& odd,
                        hipStream_t s);
hipError_t half_to_host(const dwf_ctx* c, const HalfField& even, const HalfField& odd, int nrhs, double* host,
                        hipStream_t s);
hipError_t half_convert(const dwf_ctx* c, const HalfField& src, HalfField& dst, int nrhs, hipStream_t s);
hipError_t half_zero(const dwf_ctx* c, HalfField& f, int nrhs, hipStream_t s);
hipError_t half_copy(const dwf_ctx* c, HalfField& dst, const HalfField& src, int nrhs, const int* mask,
                     hipStream_t s);
hipError_t half_acc(const dwf_ctx* c, HalfField& yhat, const HalfField& y, int nrhs, const int* mask,
                    hipStream_t s);
hipError_t pack_links(const dwf_ctx* c, const double* gauge_dev, hipStream_t s);

// operator application on half fields (ops.hip)
int apply_op(dwf_ctx* c, int op, int prec, const double* in_dev, double* out_dev, int nrhs, hipStream_t s);

// the solver (solver.hip)
int solve(dwf_ctx* c, const double* b_dev, double* x_dev, int nrhs, const dwf_solve_params& p,
          dwf_solve_stats* stats, hipStream_t s, const double* mq_per_rhs);

int time_inner_kernels(dwf_ctx* c, const dwf_solve_params& p, int nrhs, int launches, double* ms, double* bytes);

// paper-convention flops and algorithmic bytes of one inner CG iteration
double flops_per_iter(const dwf_ctx* c);
double bytes_per_iter(const dwf_ctx* c, int inner_prec, int link_fmt);

}  // namespace dwf
