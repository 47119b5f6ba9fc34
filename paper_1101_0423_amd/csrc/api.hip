// api.hip -- the C ABI of libdwf (include/dwf.h): contexts, the resident
// gauge field, the fifth-dimension tables of Eqs. (7)-(9), error reporting,
// and the thin host-pointer wrappers around the device-pointer entry points.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cstdio>

#include "dwf_ctx.h"

namespace dwf {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int DevBuf::alloc(size_t n) {
    release();
    if (n == 0) return DWF_OK;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? DWF_ENOMEM : DWF_EDEVICE,
                    std::string("hipMalloc(") + std::to_string(n) + "): " + hipGetErrorString(e));
    }
    bytes = n;
    return DWF_OK;
}

void DevBuf::release() {
    if (p && own) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    own = true;
}

void HalfField::sizes(int prec, long V5h, int nrhs, size_t* data_bytes, size_t* nrm_bytes) {
    const int nblk = prec == DWF_PREC_FP64 ? 12 : prec == DWF_PREC_FP32 ? 6 : 3;
    *data_bytes = (size_t)(((V5h * nblk + 255) / 256) * 256) * nrhs * 16;
    *nrm_bytes = prec == DWF_PREC_FP16 ? (size_t)(((V5h + 1023) / 1024) * 1024) * nrhs * sizeof(float) : 0;
}

void HalfField::place(int prec_, long V5h, int Ns, int nrhs_, unsigned char* mem) {
    prec = prec_;
    nrhs = nrhs_;
    ns = Ns;
    const int nblk = prec == DWF_PREC_FP64 ? 12 : prec == DWF_PREC_FP32 ? 6 : 3;
    rstride = ((V5h * nblk + 255) / 256) * 256;
    nstride = ((V5h + 1023) / 1024) * 1024;
    size_t db, nb;
    sizes(prec, V5h, nrhs, &db, &nb);
    data.view(mem, db);
    if (nb) nrm.view(mem + db, nb);
}

int HalfField::alloc(int prec_, long V5h, int Ns, int nrhs_) {
    prec = prec_;
    nrhs = nrhs_;
    ns = Ns;
    int nblk = prec == DWF_PREC_FP64 ? 12 : prec == DWF_PREC_FP32 ? 6 : 3;
    // right-hand sides start on 4 KiB boundaries
    rstride = ((V5h * nblk + 255) / 256) * 256;
    int rc = data.alloc((size_t)rstride * nrhs * 16);
    if (rc) return rc;
    if (prec == DWF_PREC_FP16) {
        nstride = ((V5h + 1023) / 1024) * 1024;
        rc = nrm.alloc((size_t)nstride * nrhs * sizeof(float));
        if (rc) return rc;
    }
    return DWF_OK;
}

int Workspace::alloc(const std::vector<int>& precs, long V5h, int Ns, int nrhs_) {
    nrhs = nrhs_;
    fields.clear();
    for (int pr : precs) {
        fields.emplace_back(new HalfField);
        int rc = fields.back()->alloc(pr, V5h, Ns, nrhs_);
        if (rc) return rc;
    }
    return DWF_OK;
}

int Workspace::alloc_state(int n, hipStream_t s) {
    // 7 double arrays + 4 int arrays of length n
    size_t nd = 7 * (size_t)n, ni = 4 * (size_t)n;
    int rc = state.alloc(nd * sizeof(double) + ni * sizeof(int));
    if (rc) return rc;
    double* d = state.as<double>();
    int* i = (int*)(d + nd);
    st.rr = d;
    st.uu = d + n;
    st.alpha = d + 2 * n;
    st.beta = d + 3 * n;
    st.rr_target = d + 4 * n;
    st.aux = d + 5 * n;
    st.ecr = d + 6 * n;
    st.live = i;
    st.iters = i + n;
    st.status = i + 2 * n;
    st.maxiter = i + 3 * n;
    // stream-ordered: a legacy-stream operation would conflict with another
    // thread's graph capture
    hipError_t e = hipMemsetAsync(state.p, 0, state.bytes, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(DWF_EDEVICE, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
    return DWF_OK;
}

}  // namespace dwf

using namespace dwf;

dwf::Geom dwf_ctx::geom(int out_parity, bool fp64) const {
    return geom_tile(out_parity, fp64 ? G64 : G32, dwf::ORDER_AUTO);
}

// Workgroup geometry: G 4D sites per workgroup, walked in block order `order`
// (ORDER_AUTO: t-fastest, with z-plane tiles where a block's +-z neighbour
// would otherwise be read more than 64 workgroups back; ORDER_PLAIN:
// lexicographic blocks; ORDER_TFAST: t-fastest in XCD chunks of t-slices;
// w >= 2: t-fastest with z-plane tiles of w blocks).  Orders that need blocks
// to tile the t-slices or z-planes fall back to the plain order.
dwf::Geom dwf_ctx::geom_tile(int out_parity, int G, int order) const {
    Geom g;
    g.Lx = dims[0];
    g.Ly = dims[1];
    g.Lz = dims[2];
    g.Lt = dims[3];
    g.Lxh = dims[0] / 2;
    g.Ns = Ns;
    g.G = G;
    g.V4h = (int)V4h;
    g.out_parity = out_parity;
    g.antiper = opts.antiperiodic_t ? 1 : 0;
    g.nblocks = (int)((V4h + g.G - 1) / g.G);
    g.xcd = opts.xcd_remap < 0 ? 0 : 1;
    // t-fastest workgroup order when blocks tile the t-slices exactly
    const long V3h = V4h / dims[3];
    g.nsb = 0;
    g.tchunk = 0;
    g.nsb0 = 0;
    g.tilew = 0;
    if (order != dwf::ORDER_PLAIN && g.xcd && V3h % g.G == 0) {
        g.nsb = (int)(V3h / g.G);
        g.tchunk = dims[3] % 8 == 0 ? dims[3] / 8 : dims[3];
        const long plane = (long)g.Lxh * g.Ly;
        if (plane % g.G == 0) {
            g.nsb0 = (int)(plane / g.G);
            if (order == dwf::ORDER_AUTO) {
                // Tile the z-planes when the t-fastest order would put a
                // block's +-z neighbour more than 64 workgroups back (an XCD
                // holds about 128 at once): 24^3 planes (18 blocks, 6 t-slices
                // per chunk) gain 2-8% per hop kernel, 16^3 planes (8 blocks, 4
                // t-slices) lose with tiles.
                if ((long)g.nsb0 * g.tchunk > 64)
                    for (int w = 6; w >= 2; --w)
                        if (g.nsb0 % w == 0) {
                            g.tilew = w;
                            break;
                        }
            } else if (order >= 2 && g.nsb0 % order == 0) {
                g.tilew = order;
            }
        }
    }
    return g;
}

const TableSet* dwf_ctx::table_set(double mq_val, int* rc) {
    std::lock_guard<std::mutex> lk(tables_mtx);
    auto it = tables.find(mq_val);
    if (it != tables.end()) {
        *rc = DWF_OK;
        return it->second.get();
    }
    std::unique_ptr<TableSet> ts(new TableSet);
    ts->mq = mq_val;
    std::string why;
    if (!build_tables(Ns, m0, mq_val, sigma.data(), omega.data(), ts->host, why)) {
        *rc = fail(DWF_EINVAL, why);
        return nullptr;
    }
    size_t n = ts->host.size();
    std::vector<float> h32(n);
    for (size_t i = 0; i < n; ++i) h32[i] = (float)ts->host[i];
    if ((*rc = ts->d64.alloc(n * sizeof(double)))) return nullptr;
    if ((*rc = ts->d32.alloc(n * sizeof(float)))) return nullptr;
    hipError_t e = hipMemcpyAsync(ts->d64.p, ts->host.data(), n * sizeof(double), hipMemcpyHostToDevice, xfer);
    if (e == hipSuccess) e = hipMemcpyAsync(ts->d32.p, h32.data(), n * sizeof(float), hipMemcpyHostToDevice, xfer);
    if (e == hipSuccess) e = hipStreamSynchronize(xfer);
    if (e != hipSuccess) {
        *rc = fail(DWF_EDEVICE, std::string("table upload: ") + hipGetErrorString(e));
        return nullptr;
    }
    TableSet* raw = ts.get();
    tables[mq_val] = std::move(ts);
    *rc = DWF_OK;
    return raw;
}

int dwf_ctx::ensure_stage(double** in, double** out) {
    const size_t n = (size_t)spinor_elems() * sizeof(double);
    if (stage.bytes < 2 * n) {
        int rc = stage.alloc(2 * n);
        if (rc) return rc;
    }
    *in = stage.as<double>();
    *out = stage.as<double>() + spinor_elems();
    return DWF_OK;
}

int dwf_ctx::ensure_partials(size_t n) {
    size_t need = n * sizeof(double);
    if (partials_bytes >= need) return DWF_OK;
    int rc = partials.alloc(need);
    if (rc) return rc;
    partials_bytes = need;
    return DWF_OK;
}

namespace dwf {

double su3_deviation(const double* g, long nlinks) {
    double dev = 0;
    for (long l = 0; l < nlinks; ++l) {
        const double* u = g + 18 * l;
        // entry (a, b) = u[2 (3 a + b)] + i u[2 (3 a + b) + 1]
        for (int b = 0; b < 3; ++b) {
            const int b1 = (b + 1) % 3, b2 = (b + 2) % 3;
            const double ar = u[2 * b1], ai = u[2 * b1 + 1], br = u[2 * (3 + b2)], bi = u[2 * (3 + b2) + 1];
            const double cr = u[2 * b2], ci = u[2 * b2 + 1], dr = u[2 * (3 + b1)], di = u[2 * (3 + b1) + 1];
            // (row0 x row1)_b = row0_{b1} row1_{b2} - row0_{b2} row1_{b1}; row 2 should be its conjugate
            const double xr = (ar * br - ai * bi) - (cr * dr - ci * di);
            const double xi = (ar * bi + ai * br) - (cr * di + ci * dr);
            const double er = u[2 * (6 + b)] - xr, ei = u[2 * (6 + b) + 1] + xi;
            const double d = sqrt(er * er + ei * ei);
            if (!(d <= dev)) dev = std::isfinite(d) ? d : INFINITY;
        }
    }
    return dev;
}

int link_format(const dwf_ctx* c, const dwf_solve_params& p) {
    switch (p.inner_prec) {
        case DWF_PREC_FP64: return LINK_D18;
        case DWF_PREC_FP32:
            if (p.link_compress == 1 || (p.link_compress == -1 && c->su3)) return LINK_S12;
            return LINK_S18;
        default: return LINK_H12;
    }
}

int check_params(const dwf_ctx* c, const dwf_solve_params& p) {
    if (!(p.tol > 0)) return fail(DWF_EINVAL, "tol must be > 0");
    if (p.inner_prec < DWF_PREC_FP64 || p.inner_prec > DWF_PREC_FP16) return fail(DWF_EINVAL, "bad inner_prec");
    if (p.maxiter < 1) return fail(DWF_EINVAL, "maxiter must be >= 1");
    if (p.link_compress < -1 || p.link_compress > 1) return fail(DWF_EINVAL, "link_compress must be -1, 0 or 1");
    if (p.system != DWF_SYSTEM_D && p.system != DWF_SYSTEM_CCDAG) return fail(DWF_EINVAL, "unknown system");
    if (p.tile < 0) return fail(DWF_EINVAL, "tile must be >= 0");
    if (!c->su3 && p.inner_prec == DWF_PREC_FP32 && p.link_compress == 1)
        return fail(DWF_EINVAL, "12-real links need an SU(3) field (row 2 = conj(row 0 x row 1)); this field "
                                "deviates by " + std::to_string(c->su3_dev));
    if (!c->su3 && p.inner_prec == DWF_PREC_FP16)
        return fail(DWF_EINVAL, "FP16 storage uses 12-real links, which need an SU(3) field; this field deviates by " +
                                    std::to_string(c->su3_dev));
    return DWF_OK;
}

}  // namespace dwf

namespace {

std::mutex g_links_mu;
std::map<std::string, std::weak_ptr<LinkSet>> g_links;  // resident fields by content

// Two independent 64-bit hashes of the field's words, with its extents and
// device: contexts on the same field find each other's links.
std::string gauge_key(const double* gauge, const int dims[4], int device) {
    const size_t n = (size_t)dims[0] * dims[1] * dims[2] * dims[3] * 4 * 18;
    uint64_t h1 = 0xcbf29ce484222325ull, h2 = 0x9e3779b97f4a7c15ull;
    for (size_t i = 0; i < n; ++i) {
        uint64_t w;
        memcpy(&w, gauge + i, sizeof(w));
        h1 = (h1 ^ w) * 0x100000001b3ull;
        h2 = (h2 + w) * 0xff51afd7ed558ccdull;
        h2 ^= h2 >> 33;
    }
    char buf[128];
    snprintf(buf, sizeof(buf), "%d:%dx%dx%dx%d:%016llx%016llx", device, dims[0], dims[1], dims[2], dims[3],
             (unsigned long long)h1, (unsigned long long)h2);
    return buf;
}

}  // namespace

extern "C" {

void dwf_default_opts(dwf_opts* o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
}

void dwf_default_params(dwf_solve_params* p) {
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->tol = 1e-10;
    p->inner_prec = DWF_PREC_FP32;
    p->reliable = 1;
    p->eps_inner = 0;
    p->maxiter = 50000;
    p->check_every = 0;
    p->use_graph = 1;
    p->link_compress = -1;
    p->use_guess = 0;
    p->debug_stall_after = 0;
}

const char* dwf_last_error(void) { return g_err.c_str(); }

int dwf_gauge_su3_deviation(const double* gauge, const int dims[4], double* dev) {
    g_err.clear();
    if (!gauge || !dims || !dev) return fail(DWF_EINVAL, "NULL gauge, dims or dev");
    for (int i = 0; i < 4; ++i)
        if (dims[i] < 2 || dims[i] % 2) return fail(DWF_EINVAL, "every lattice extent must be even and >= 2");
    const long V4 = (long)dims[0] * dims[1] * dims[2] * dims[3];
    *dev = su3_deviation(gauge, V4 * 4);
    return DWF_OK;
}

const char* dwf_version(void) { return "libdwf 0.1 (gfx950)"; }

int dwf_create(dwf_ctx** out, const double* gauge, const int dims[4], int Ns, double m0, double mq,
               const double* sigma, const double* omega, const dwf_opts* opts) {
    g_err.clear();
    if (!out) return fail(DWF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!gauge || !dims || !sigma || !omega) return fail(DWF_EINVAL, "NULL gauge, dims, sigma or omega");
    for (int i = 0; i < 4; ++i)
        if (dims[i] < 2 || dims[i] % 2) return fail(DWF_EINVAL, "every lattice extent must be even and >= 2");
    if (Ns < 1 || Ns > 32) return fail(DWF_EINVAL, "Ns must be in [1, 32]");
    if (!(m0 > 0 && m0 < 2)) return fail(DWF_EINVAL, "m0 must be in (0, 2)");
    if (!std::isfinite(mq)) return fail(DWF_EINVAL, "mq must be finite");
    for (int s = 0; s < Ns; ++s) {
        if (!(omega[s] > 0) || !std::isfinite(omega[s])) return fail(DWF_EINVAL, "omega_s must be > 0");
        if (!std::isfinite(sigma[s])) return fail(DWF_EINVAL, "sigma_s must be finite");
    }
    long V4 = (long)dims[0] * dims[1] * dims[2] * dims[3];
    if (V4 / 2 * Ns > (1L << 30)) return fail(DWF_EINVAL, "lattice too large");
    {
        std::vector<double> tmp;
        std::string why;
        if (!build_tables(Ns, m0, mq, sigma, omega, tmp, why)) return fail(DWF_EINVAL, why);
    }
    std::unique_ptr<dwf_ctx> c(new dwf_ctx);
    for (int i = 0; i < 4; ++i) c->dims[i] = dims[i];
    c->Ns = Ns;
    c->m0 = m0;
    c->mq = mq;
    c->sigma.assign(sigma, sigma + Ns);
    c->omega.assign(omega, omega + Ns);
    if (opts)
        c->opts = *opts;
    else
        dwf_default_opts(&c->opts);
    c->device = c->opts.device;
    c->V4 = V4;
    c->V4h = V4 / 2;
    c->V5h = c->V4h * Ns;
    // 12-real links rebuild row 2 from rows 0 and 1: exact only for SU(3)
    // fields (a U(3) field, or one with phases folded into its links, is
    // solved with 18-real links)
    c->su3_dev = su3_deviation(gauge, V4 * 4);
    c->su3 = c->su3_dev <= DWF_SU3_TOL;
    // workgroups of G 4D sites x Ns slices, at most 256 lanes
    int G = c->opts.sites_per_block;
    if (G < 0 || G * Ns > 256) return fail(DWF_EINVAL, "sites_per_block * Ns must be <= 256");
    c->G32 = G > 0 ? G : std::min(64, std::max(1, 256 / Ns));
    c->G64 = G > 0 ? std::max(1, G / 2) : std::min(32, std::max(1, 128 / Ns));

    DWF_HIP(hipSetDevice(c->device));
    int rc = scratch_init(c->device);  // the allocation-free operator's workspace on this device
    if (rc) return rc;
    DWF_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    DWF_HIP(hipStreamCreateWithFlags(&c->xfer, hipStreamNonBlocking));
    {
        // share the resident links of an identical field
        const std::string key = gauge_key(gauge, dims, c->device);
        std::lock_guard<std::mutex> lk(g_links_mu);
        auto it = g_links.find(key);
        if (it != g_links.end()) c->lset = it->second.lock();
        if (!c->lset) {
            std::shared_ptr<LinkSet> ls(new LinkSet);
            c->lset = ls;
            c->links = ls->buf;
            const size_t nl = (size_t)c->V4h * 8;
            for (int par = 0; par < 2; ++par) {
                if ((rc = ls->buf[par][LINK_D18].alloc(nl * 18 * sizeof(double)))) return rc;
                if ((rc = ls->buf[par][LINK_S18].alloc(nl * 18 * sizeof(float)))) return rc;
                if ((rc = ls->buf[par][LINK_S12].alloc(nl * 12 * sizeof(float)))) return rc;
                if ((rc = ls->buf[par][LINK_H12].alloc(nl * 12 * sizeof(_Float16)))) return rc;
            }
            DevBuf g;
            if ((rc = g.alloc((size_t)V4 * 4 * 18 * sizeof(double)))) return rc;
            DWF_HIP(hipMemcpyAsync(g.p, gauge, (size_t)V4 * 4 * 18 * sizeof(double), hipMemcpyHostToDevice,
                                   c->stream));
            DWF_HIP(pack_links(c.get(), g.as<double>(), c->stream));
            DWF_HIP(hipStreamSynchronize(c->stream));
            for (auto i = g_links.begin(); i != g_links.end();) i = i->second.expired() ? g_links.erase(i) : ++i;
            g_links[key] = ls;
        }
        c->links = c->lset->buf;
        c->gauge_key = key;
    }
    c->table_set(mq, &rc);
    if (rc) return rc;
    *out = c.release();
    return DWF_OK;
}

void dwf_destroy(dwf_ctx* c) {
    if (!c) return;
    server_detach(c);
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    hipStream_t s = c->stream, x = c->xfer;
    delete c;
    if (s) (void)hipStreamDestroy(s);
    if (x) (void)hipStreamDestroy(x);
}

}  // extern "C"

namespace {

int check_apply(dwf_ctx* c, int op, int prec, const void* in, const void* out, int nrhs) {
    if (!c || !in || !out) return fail(DWF_EINVAL, "NULL context or buffer");
    if (op < DWF_OP_DW || op > DWF_OP_DDAG) return fail(DWF_EINVAL, "unknown operator");
    const int pr = prec & 0xff, lk = prec & ~0xff;
    if (pr < DWF_PREC_FP64 || pr > DWF_PREC_FP16) return fail(DWF_EINVAL, "unknown precision");
    if (lk != DWF_LINKS_AUTO && lk != DWF_LINKS_18 && lk != DWF_LINKS_12)
        return fail(DWF_EINVAL, "unknown link storage");
    if (pr == DWF_PREC_FP64 && lk == DWF_LINKS_12) return fail(DWF_EINVAL, "FP64 uses 18-real links");
    if (pr == DWF_PREC_FP16 && lk == DWF_LINKS_18) return fail(DWF_EINVAL, "FP16 storage uses 12-real links");
    if (!c->su3 && (lk == DWF_LINKS_12 || pr == DWF_PREC_FP16))
        return fail(DWF_EINVAL, "12-real links need an SU(3) field; this field deviates by " +
                                    std::to_string(c->su3_dev));
    if (nrhs < 1) return fail(DWF_EINVAL, "nrhs must be >= 1");
    return DWF_OK;
}

int check_solve(dwf_ctx* c, const void* b, const void* x, int nrhs, const dwf_solve_params* params,
                dwf_solve_params* p) {
    if (!c || !b || !x) return fail(DWF_EINVAL, "NULL context or buffer");
    if (nrhs < 1) return fail(DWF_EINVAL, "nrhs must be >= 1");
    if (params)
        *p = *params;
    else
        dwf_default_params(p);
    return check_params(c, *p);
}

}  // namespace

extern "C" {

int dwf_apply_dev(dwf_ctx* c, int op, int prec, const double* in_dev, double* out_dev, int nrhs, void* stream) {
    g_err.clear();
    int rc = check_apply(c, op, prec, in_dev, out_dev, nrhs);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(c->mtx);
    DWF_HIP(hipSetDevice(c->device));
    hipStream_t s = stream ? (hipStream_t)stream : c->stream;
    if ((rc = apply_op(c, op, prec, in_dev, out_dev, nrhs, s))) return rc;
    DWF_HIP(hipStreamSynchronize(s));
    return DWF_OK;
}

// The host-pointer forms stage one spinor at a time through the context's
// two-spinor device buffer, on the context's stream (never the legacy stream,
// which would conflict with the request server's graph captures).
int dwf_apply(dwf_ctx* c, int op, int prec, const double* in, double* out, int nrhs) {
    g_err.clear();
    int rc = check_apply(c, op, prec, in, out, nrhs);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(c->mtx);
    DWF_HIP(hipSetDevice(c->device));
    HostIO io{in, out, nullptr, nullptr};
    if ((rc = c->ensure_stage(&io.stage_in, &io.stage_out))) return rc;
    return apply_op(c, op, prec, nullptr, nullptr, nrhs, c->stream, &io);
}

int dwf_apply_dev_noalloc(dwf_ctx* c, int op, int prec, const double* in_dev, double* out_dev, int nrhs,
                          void* stream) {
    g_err.clear();
    int rc = check_apply(c, op, prec, in_dev, out_dev, nrhs);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(c->mtx);
    DWF_HIP(hipSetDevice(c->device));
    hipStream_t s = stream ? (hipStream_t)stream : c->stream;
    if ((rc = apply_op_noalloc(c, op, prec, in_dev, out_dev, nrhs, s))) return rc;
    DWF_HIP(hipStreamSynchronize(s));
    return DWF_OK;
}

int dwf_solve_dev(dwf_ctx* c, const double* b_dev, double* x_dev, int nrhs, const dwf_solve_params* params,
                  dwf_solve_stats* stats, void* stream) {
    g_err.clear();
    dwf_solve_params p;
    int rc = check_solve(c, b_dev, x_dev, nrhs, params, &p);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(c->mtx);
    DWF_HIP(hipSetDevice(c->device));
    hipStream_t s = stream ? (hipStream_t)stream : c->stream;
    return solve(c, b_dev, x_dev, nrhs, p, stats, s);
}

int dwf_time_kernels(dwf_ctx* c, const dwf_solve_params* params, int nrhs, int launches, double ms[5],
                     double bytes[5]) {
    g_err.clear();
    if (!c || !ms || !bytes) return fail(DWF_EINVAL, "NULL argument");
    if (nrhs < 1 || launches < 1) return fail(DWF_EINVAL, "nrhs and launches must be >= 1");
    dwf_solve_params p;
    if (params)
        p = *params;
    else
        dwf_default_params(&p);
    std::lock_guard<std::mutex> lk(c->mtx);
    DWF_HIP(hipSetDevice(c->device));
    return time_inner_kernels(c, p, nrhs, launches, ms, bytes);
}

int dwf_propagator_dev(dwf_ctx* c, const double* eta_dev, double* out_dev, int nsrc,
                       const dwf_solve_params* params, dwf_solve_stats* stats, void* stream) {
    g_err.clear();
    dwf_solve_params p;
    int rc = check_solve(c, eta_dev, out_dev, nsrc, params, &p);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(c->mtx);
    DWF_HIP(hipSetDevice(c->device));
    hipStream_t s = stream ? (hipStream_t)stream : c->stream;
    return propagator(c, eta_dev, out_dev, nsrc, p, stats, s);
}

int dwf_propagator(dwf_ctx* c, const double* eta, double* out, int nsrc, const dwf_solve_params* params,
                   dwf_solve_stats* stats) {
    g_err.clear();
    dwf_solve_params p;
    int rc = check_solve(c, eta, out, nsrc, params, &p);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(c->mtx);
    DWF_HIP(hipSetDevice(c->device));
    // A 4D spinor is Ns times smaller than a 5D one: each half of the
    // context's two-spinor staging buffer holds Ns sources, so the sources go
    // through in groups of up to Ns (each group one batched solve; a source's
    // result does not depend on the others in its group)
    const size_t n4 = (size_t)c->V4 * 24;
    double *si, *so;
    if ((rc = c->ensure_stage(&si, &so))) return rc;
    hipStream_t s = c->stream;
    int status = DWF_OK;
    std::string msg;
    for (int k0 = 0; k0 < nsrc; k0 += c->Ns) {
        const int n = std::min(c->Ns, nsrc - k0);
        DWF_HIP(hipMemcpyAsync(si, eta + k0 * n4, n * n4 * sizeof(double), hipMemcpyHostToDevice, s));
        rc = propagator(c, si, so, n, p, stats ? stats + k0 : nullptr, s);
        if (rc != DWF_OK && rc != DWF_ENOCONV) return rc;
        if (rc) {
            status = rc;
            msg = dwf_last_error();
        }
        DWF_HIP(hipMemcpyAsync(out + k0 * n4, so, n * n4 * sizeof(double), hipMemcpyDeviceToHost, s));
        DWF_HIP(hipStreamSynchronize(s));
    }
    if (status) fail(status, msg);
    return status;
}

int dwf_stream_copy(const void* src_dev, void* dst_dev, size_t bytes, int nontemporal, int device,
                    void* stream) {
    g_err.clear();
    if (!src_dev || !dst_dev) return fail(DWF_EINVAL, "NULL buffer");
    if (bytes % 16) return fail(DWF_EINVAL, "bytes must be a multiple of 16");
    if (nontemporal != 0 && nontemporal != 1) return fail(DWF_EINVAL, "nontemporal must be 0 or 1");
    hipStream_t s = (hipStream_t)stream;
    if (!s) return fail(DWF_EINVAL, "a stream is required");
    DWF_HIP(hipSetDevice(device));
    DWF_HIP(stream_copy(src_dev, dst_dev, bytes, nontemporal != 0, s));
    DWF_HIP(hipStreamSynchronize(s));
    return DWF_OK;
}

int dwf_solve(dwf_ctx* c, const double* b, double* x, int nrhs, const dwf_solve_params* params,
              dwf_solve_stats* stats) {
    g_err.clear();
    dwf_solve_params p;
    int rc = check_solve(c, b, x, nrhs, params, &p);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(c->mtx);
    DWF_HIP(hipSetDevice(c->device));
    HostIO io{b, x, nullptr, nullptr};
    if ((rc = c->ensure_stage(&io.stage_in, &io.stage_out))) return rc;
    return solve(c, nullptr, nullptr, nrhs, p, stats, c->stream, &io);
}

}  // extern "C"
