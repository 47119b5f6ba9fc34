// ops.hip -- the operators of dwf_apply, built from the fused stencil kernel:
// D_w (Eq. (2)), the hopping blocks D_w^EO / D_w^OE (Eq. (14)), M5 and M5^T
// (Eq. (8)), the Schur complement C (Eq. (11)) and C^dag, C C^dag, and the
// 5D operator D (Eq. (5)) and D^dag, each in FP64, FP32 or FP16 storage.
#include <mutex>

#include "dwf_ctx.h"

namespace dwf {

template <class F>
F fld(const HalfField& h);
template <>
FD fld<FD>(const HalfField& h) { return h.fd(); }
template <>
FS fld<FS>(const HalfField& h) { return h.fs(); }
template <>
FH fld<FH>(const HalfField& h) { return h.fh(); }

template <class Real>
const Real* tab(const TableSet* ts, int t, int Ns);
template <>
const double* tab<double>(const TableSet* ts, int t, int Ns) { return ts->t64(t, Ns); }
template <>
const float* tab<float>(const TableSet* ts, int t, int Ns) { return ts->t32(t, Ns); }
template <class Real>
const Real* stab(const TableSet* ts, int t, int Ns);
template <>
const double* stab<double>(const TableSet* ts, int t, int Ns) { return ts->s64(t, Ns); }
template <>
const float* stab<float>(const TableSet* ts, int t, int Ns) { return ts->s32(t, Ns); }

namespace {

enum { IN_E = 0, IN_O, OUT_E, OUT_O, T_E, T_O, T2_E, T2_O, NAPPLY };

template <class Real, class F, class LF>
struct Applier {
    dwf_ctx* c;
    const TableSet* ts;
    Workspace* w;
    LF lk[2];
    KOpt o;
    hipStream_t s;

    Geom geom(int par) const { return c->geom(par, sizeof(Real) == 8); }
    F f(int i) const { return fld<F>(w->f(i)); }
    const Real* t(int which) const { return tab<Real>(ts, which, c->Ns); }
    const Real* ts_(int which) const { return stab<Real>(ts, which, c->Ns); }

    // out(par) = epi( hop(in) )
    template <class Epi>
    hipError_t hop(int par, int in, const Epi& epi) {
        return launch_dwf<Real, F, LF, true, MIX_NONE, ProLoad<F>, Epi>(geom(par), f(in), lk[par], nullptr,
                                                                         ProLoad<F>{f(in)}, epi, o, s);
    }
    // out(par) = epi( M hop(in) ), M = M5 (st = ST_M5) or M5^T (st = ST_M5T) by recurrence
    template <class Epi>
    hipError_t hopmix(int par, int in, int st, const Epi& epi) {
        if (st == ST_M5)
            return launch_dwf<Real, F, LF, true, MIX_SA, ProLoad<F>, Epi>(geom(par), f(in), lk[par], ts_(st),
                                                                          ProLoad<F>{f(in)}, epi, o, s);
        return launch_dwf<Real, F, LF, true, MIX_AS, ProLoad<F>, Epi>(geom(par), f(in), lk[par], ts_(st),
                                                                      ProLoad<F>{f(in)}, epi, o, s);
    }
    // out(par) = epi( T in ) with a dense table
    template <class Epi>
    hipError_t local(int par, int in, int table, const Epi& epi) {
        return launch_dwf<Real, F, LF, false, MIX_DENSE, ProLoad<F>, Epi>(geom(par), f(in), lk[par], t(table),
                                                                          ProLoad<F>{f(in)}, epi, o, s);
    }
    // out(par) = epi( M in ) by recurrence (M5, M5^T or M5^T gamma_5)
    template <class Epi>
    hipError_t local_st(int par, int in, int st, const Epi& epi) {
        if (st == ST_M5)
            return launch_dwf<Real, F, LF, false, MIX_SA, ProLoad<F>, Epi>(geom(par), f(in), lk[par], ts_(st),
                                                                           ProLoad<F>{f(in)}, epi, o, s);
        return launch_dwf<Real, F, LF, false, MIX_AS, ProLoad<F>, Epi>(geom(par), f(in), lk[par], ts_(st),
                                                                       ProLoad<F>{f(in)}, epi, o, s);
    }
    EpiStore<F> store(int i) const { return EpiStore<F>{f(i)}; }
    EpiLin<F, F, false, false> lin(int a, int out, double ca, double cv) const {
        return EpiLin<F, F, false, false>{f(a), f(out), ca, cv};
    }

    hipError_t zero(int i) { return half_zero(c, w->f(i), o.nrhs, s); }

    hipError_t run(int op) {
        hipError_t e = hipSuccess;
#define CK(x)                         \
    do {                              \
        e = (x);                      \
        if (e != hipSuccess) return e; \
    } while (0)
        const double dm = 4.0 - c->m0;
        switch (op) {
            case DWF_OP_HOP_EO:
                CK(hop(0, IN_O, store(OUT_E)));
                CK(zero(OUT_O));
                break;
            case DWF_OP_HOP_OE:
                CK(hop(1, IN_E, store(OUT_O)));
                CK(zero(OUT_E));
                break;
            case DWF_OP_DW:
                CK(hop(0, IN_O, lin(IN_E, OUT_E, dm, 1.0)));
                CK(hop(1, IN_E, lin(IN_O, OUT_O, dm, 1.0)));
                break;
            case DWF_OP_M5:
            case DWF_OP_M5T: {
                int st = op == DWF_OP_M5 ? ST_M5 : ST_M5T;
                CK(local_st(0, IN_E, st, store(OUT_E)));
                CK(local_st(1, IN_O, st, store(OUT_O)));
                break;
            }
            case DWF_OP_C:
                CK(hopmix(0, IN_O, ST_M5, store(T_E)));
                CK(hopmix(1, T_E, ST_M5, lin(IN_O, OUT_O, 1.0, -1.0)));
                CK(zero(OUT_E));
                break;
            case DWF_OP_CDAG:
            case DWF_OP_CCDAG: {
                int dst = op == DWF_OP_CDAG ? OUT_O : T2_O;
                CK(local_st(1, IN_O, ST_M5TG5, store(T_O)));
                CK(hopmix(0, T_O, ST_M5T, store(T_E)));
                CK(hop(1, T_E, EpiLin<F, F, false, true>{f(IN_O), f(dst), 1.0, -1.0}));
                if (op == DWF_OP_CCDAG) {
                    CK(hopmix(0, T2_O, ST_M5, store(T_E)));
                    CK(hopmix(1, T_E, ST_M5, lin(T2_O, OUT_O, 1.0, -1.0)));
                }
                CK(zero(OUT_E));
                break;
            }
            case DWF_OP_D:
                for (int p = 0; p < 2; ++p) {
                    CK(local(p, IN_E + p, TB_Y, store(T_E + p)));
                    CK(local(p, IN_E + p, TB_X, store(T2_E + p)));
                }
                CK(hop(0, T_O, lin(T2_E, OUT_E, 1.0, 1.0)));
                CK(hop(1, T_E, lin(T2_O, OUT_O, 1.0, 1.0)));
                break;
            case DWF_OP_DDAG:
                for (int p = 0; p < 2; ++p) CK(local(p, IN_E + p, TB_G5, store(T_E + p)));   // g = g5 x
                CK(hop(0, T_O, lin(T_E, T2_E, dm, 1.0)));                                   // w = D_w g
                CK(hop(1, T_E, lin(T_O, T2_O, dm, 1.0)));
                for (int p = 0; p < 2; ++p) CK(local(p, IN_E + p, TB_1MLT, store(T_E + p)));  // (1-L)^T x
                for (int p = 0; p < 2; ++p) CK(local(p, T2_E + p, TB_YTG5, lin(T_E + p, OUT_E + p, 1.0, 1.0)));
                break;
            default:
                return hipErrorInvalidValue;
        }
#undef CK
        return e;
    }
};

// The workspace of an application: NAPPLY half fields, kept by the context
// per (precision, nrhs), or laid out in the static scratch array (wsp given).
template <class Real, class F, class LF>
int apply_impl(dwf_ctx* c, int op, int prec, LF e, LF o_, const double* in_dev, double* out_dev, int nrhs,
               hipStream_t s, const HostIO* hio, Workspace* wsp = nullptr) {
    int rc;
    const TableSet* ts = c->table_set(c->mq, &rc);  // built by dwf_create for the context's mass
    if (!ts) return rc;
    Workspace* w = wsp;
    if (!w) {
        std::string key = "apply:" + std::to_string(prec) + ":" + std::to_string(nrhs);
        auto& slot = c->ws[key];
        if (!slot) {
            slot.reset(new Workspace);
            if ((rc = slot->alloc(std::vector<int>(NAPPLY, prec), c->V5h, c->Ns, nrhs))) {
                slot.reset();
                return rc;
            }
        }
        w = slot.get();
    }
    Applier<Real, F, LF> A{c, ts, w, {e, o_}, KOpt{nullptr, nullptr, nrhs, 0}, s};
    const long n5 = c->spinor_elems();
    if (hio) {
        // one right-hand side at a time through the staging spinor; the
        // conversion reading it is done before the next copy overwrites it
        for (int r = 0; r < nrhs; ++r) {
            DWF_HIP(hipMemcpyAsync(hio->stage_in, hio->in + r * n5, n5 * sizeof(double), hipMemcpyHostToDevice, s));
            DWF_HIP(host_to_half(c, hio->stage_in, 1, w->f(IN_E), w->f(IN_O), s, r));
            DWF_HIP(hipStreamSynchronize(s));
        }
    } else {
        DWF_HIP(host_to_half(c, in_dev, nrhs, w->f(IN_E), w->f(IN_O), s));
    }
    hipError_t err = A.run(op);
    if (err != hipSuccess) return fail(DWF_EDEVICE, std::string("operator kernels: ") + hipGetErrorString(err));
    if (hio) {
        for (int r = 0; r < nrhs; ++r) {
            DWF_HIP(half_to_host(c, w->f(OUT_E), w->f(OUT_O), 1, hio->stage_out, s, r));
            DWF_HIP(hipMemcpyAsync(hio->out + r * n5, hio->stage_out, n5 * sizeof(double), hipMemcpyDeviceToHost, s));
            DWF_HIP(hipStreamSynchronize(s));
        }
    } else {
        DWF_HIP(half_to_host(c, w->f(OUT_E), w->f(OUT_O), nrhs, out_dev, s));
    }
    return DWF_OK;
}

int dispatch(dwf_ctx* c, int op, int prec_flags, const double* in_dev, double* out_dev, int nrhs, hipStream_t s,
             const HostIO* hio, Workspace* wsp) {
    const int prec = prec_flags & 0xff, lk = prec_flags & ~0xff;
    switch (prec) {
        case DWF_PREC_FP64:
            return apply_impl<double, FD, LinkD18>(c, op, prec, LinkD18{c->links[0][LINK_D18].as<double>()},
                                                   LinkD18{c->links[1][LINK_D18].as<double>()}, in_dev, out_dev,
                                                   nrhs, s, hio, wsp);
        case DWF_PREC_FP32:
            if (lk == DWF_LINKS_12 || (lk == DWF_LINKS_AUTO && c->su3))
                return apply_impl<float, FS, LinkS12>(c, op, prec, LinkS12{c->links[0][LINK_S12].as<float>()},
                                                      LinkS12{c->links[1][LINK_S12].as<float>()}, in_dev, out_dev,
                                                      nrhs, s, hio, wsp);
            return apply_impl<float, FS, LinkS18>(c, op, prec, LinkS18{c->links[0][LINK_S18].as<float>()},
                                                  LinkS18{c->links[1][LINK_S18].as<float>()}, in_dev, out_dev,
                                                  nrhs, s, hio, wsp);
        default:
            return apply_impl<float, FH, LinkH12>(c, op, prec, LinkH12{c->links[0][LINK_H12].as<_Float16>()},
                                                  LinkH12{c->links[1][LINK_H12].as<_Float16>()}, in_dev, out_dev,
                                                  nrhs, s, hio, wsp);
    }
}

// ---------------------------------------------------------------------------
// The allocation-free form: its workspace is this file-scope device array, of
// which every GPU the library runs on holds one copy for the life of the
// process.  Host code never uses the array's name as an address (that is a
// host-side stand-in); it uses the per-device address that hipGetSymbolAddress
// returns, looked up once per device with that device current.  Calls that
// overlap on one GPU share the array and race.
// ---------------------------------------------------------------------------

constexpr size_t kScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

int scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(DWF_EINVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return DWF_OK;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));  // the current device's copy
    if (e != hipSuccess || !ptr)
        return fail(DWF_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = (unsigned char*)ptr;
    return DWF_OK;
}

// prec: storage precision, or-ed with a DWF_LINKS_* link storage (validated by
// the caller); auto picks what the inner solver uses for this field
int apply_op(dwf_ctx* c, int op, int prec_flags, const double* in_dev, double* out_dev, int nrhs, hipStream_t s,
             const HostIO* hio) {
    return dispatch(c, op, prec_flags, in_dev, out_dev, nrhs, s, hio, nullptr);
}

int apply_op_noalloc(dwf_ctx* c, int op, int prec_flags, const double* in_dev, double* out_dev, int nrhs,
                     hipStream_t s) {
    unsigned char* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (c->device >= 0 && c->device < kMaxDevices) base = g_scratch_ptr[c->device];
    }
    if (!base) return fail(DWF_EDEVICE, "scratch array not set up on this device");
    const int prec = prec_flags & 0xff;
    size_t db, nb;
    HalfField::sizes(prec, c->V5h, nrhs, &db, &nb);
    const size_t need = (size_t)NAPPLY * (db + nb);
    if (need > kScratchBytes)
        return fail(DWF_EINVAL, "the allocation-free operator needs " + std::to_string(need) +
                                    " bytes of workspace (nrhs x V4 x Ns / 2 x 8 half fields); its static scratch "
                                    "array holds " + std::to_string(kScratchBytes));
    // every field of the workspace is written in full before it is read, so
    // nothing in the array has to start at zero
    Workspace w;
    w.nrhs = nrhs;
    for (int i = 0; i < NAPPLY; ++i) {
        w.fields.emplace_back(new HalfField);
        w.fields.back()->place(prec, c->V5h, c->Ns, nrhs, base + (size_t)i * (db + nb));
    }
    return dispatch(c, op, prec_flags, in_dev, out_dev, nrhs, s, nullptr, &w);
}

}  // namespace dwf
