// prop.hip -- 4D valence-quark propagators from the 5D solve (Sec. 2.2: the
// CG on the 5D system also yields the valence quark propagators; Sec. 5).
//
// The quark mass enters D only through the corner of L (Eq. (4)), which
// couples the + chirality at s = Ns to s = 1 and the - chirality at s = 1 to
// s = Ns: D(mq) = D(0) + kappa W R with kappa = mq / (2 m0),
//     R psi      = P_+ psi_Ns + P_- psi_1                  (5D -> 4D)
//     (W eta)_1  = (1 - sigma_1 D_w) P_+ eta,
//     (W eta)_Ns = (1 - sigma_Ns D_w) P_- eta,  0 on the other slices.
// The 4D quark field is q = R psi (the walls) and the 5D source of a 4D
// spinor eta is W eta, so the propagator is S eta = R D^-1 W eta, for which
// S(mq)^-1 = S(0)^-1 + kappa.  In the chiral basis P_+ keeps spins 0, 1 (the
// first 12 reals of a site) and P_- spins 2, 3.
#include "dwf_ctx.h"

namespace dwf {
namespace {

constexpr int TPB = 256;

struct WallGeom {
    long V4;   // 4D sites
    int Ns;
    int nsrc;
    double sigma[32];  // sigma_s
};

// c = P_+ eta on slice 0, P_- eta on slice Ns - 1, zero elsewhere (host
// layouts: 5D [src][n4][s][24], 4D [src][n4][24]); one thread per 5D site
__global__ void k_wall_inject(const double* __restrict__ eta, double* __restrict__ c, WallGeom g) {
    const long id = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const long n5 = g.V4 * g.Ns;
    if (id >= n5 * g.nsrc) return;
    const long src = id / n5, r = id - src * n5;
    const long n4 = r / g.Ns;
    const int s = (int)(r - n4 * g.Ns);
    const double* e = eta + (src * g.V4 + n4) * 24;
    double* o = c + id * 24;
    const bool up = s == 0, lo = s == g.Ns - 1;  // both when Ns = 1
#pragma unroll
    for (int k = 0; k < 24; ++k) o[k] = ((k < 12 && up) || (k >= 12 && lo)) ? e[k] : 0.0;
}

// b = c - sigma_s (D_w c)_s, in place in dc
__global__ void k_wall_combine(const double* __restrict__ c, double* __restrict__ dc, WallGeom g) {
    const long id = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const long n5 = g.V4 * g.Ns;
    if (id >= n5 * g.nsrc) return;
    const int s = (int)((id % n5) % g.Ns);
    const double sg = g.sigma[s];
#pragma unroll
    for (int k = 0; k < 24; ++k) dc[id * 24 + k] = c[id * 24 + k] - sg * dc[id * 24 + k];
}

// out = P_+ x_{Ns-1} + P_- x_0; one thread per 4D site
__global__ void k_wall_project(const double* __restrict__ x, double* __restrict__ out, WallGeom g) {
    const long id = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (id >= g.V4 * g.nsrc) return;
    const double* up = x + (id * g.Ns + g.Ns - 1) * 24;
    const double* lo = x + (id * g.Ns) * 24;
#pragma unroll
    for (int k = 0; k < 24; ++k) out[id * 24 + k] = k < 12 ? up[k] : lo[k];
}

unsigned nblk(long n) { return (unsigned)((n + TPB - 1) / TPB); }

}  // namespace

int propagator(dwf_ctx* c, const double* eta_dev, double* out_dev, int nsrc, const dwf_solve_params& p,
               dwf_solve_stats* stats, hipStream_t s) {
    if (p.system != DWF_SYSTEM_D) return fail(DWF_EINVAL, "the propagator solves D x = b (params->system)");
    if (c->Ns > 32) return fail(DWF_EINVAL, "Ns must be <= 32");
    const long n5 = c->spinor_elems();  // doubles per 5D spinor
    const size_t need = 3 * (size_t)nsrc * n5 * sizeof(double);
    if (c->prop_ws.bytes < need) {
        int rc = c->prop_ws.alloc(need);
        if (rc) return rc;
    }
    double* cw = c->prop_ws.as<double>();
    double* b = cw + (size_t)nsrc * n5;
    double* x = b + (size_t)nsrc * n5;
    WallGeom g{};
    g.V4 = c->V4;
    g.Ns = c->Ns;
    g.nsrc = nsrc;
    for (int k = 0; k < c->Ns; ++k) g.sigma[k] = c->sigma[k];
    hipLaunchKernelGGL(k_wall_inject, dim3(nblk(c->V4 * c->Ns * nsrc)), dim3(TPB), 0, s, eta_dev, cw, g);
    DWF_HIP(hipGetLastError());
    int rc = apply_op(c, DWF_OP_DW, DWF_PREC_FP64, cw, b, nsrc, s);  // D_w c (FP64)
    if (rc) return rc;
    hipLaunchKernelGGL(k_wall_combine, dim3(nblk(c->V4 * c->Ns * nsrc)), dim3(TPB), 0, s, cw, b, g);
    DWF_HIP(hipGetLastError());
    dwf_solve_params q = p;
    q.use_guess = 0;
    rc = solve(c, b, x, nsrc, q, stats, s);
    if (rc != DWF_OK && rc != DWF_ENOCONV) return rc;
    const std::string msg = dwf_last_error();
    hipLaunchKernelGGL(k_wall_project, dim3(nblk(c->V4 * nsrc)), dim3(TPB), 0, s, x, out_dev, g);
    DWF_HIP(hipGetLastError());
    DWF_HIP(hipStreamSynchronize(s));
    if (rc) fail(rc, msg);
    return rc;
}

}  // namespace dwf
