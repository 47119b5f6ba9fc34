/*
 * dwf.h -- C ABI of libdwf: conjugate gradient on the 4D even-odd
 * preconditioned 5D domain-wall fermion operator on one MI355X (gfx950).
 *
 * The operator is the general domain-wall operator of Eq. (1)/(5) of Chiu,
 * Hsieh, Mao, Ogawa, "GPU-Based Conjugate Gradient Solver for Lattice QCD
 * with Domain-Wall Fermions" (Lattice 2010):
 *
 *     D(mq) = D_w (omega + sigma L) + (1 - L),
 *
 * with the Wilson operator D_w of Eq. (2) (d = 4, 0 < m0 < 2), the chiral
 * fifth-dimension hopping L = P_+ L_+ + P_- L_- of Eqs. (3)-(4) and arbitrary
 * per-slice weights sigma_s, omega_s (Shamir: sigma = 0, omega = 1; Borici:
 * sigma = omega = 1; optimal DWF: sigma = omega).  Solves go through the
 * even-odd factorisation of Eq. (10) and the Schur complement
 * C = 1 - M5 D_w^OE M5 D_w^EO of Eq. (11), with CG (Algorithm 1) on C C^dag,
 * mixed-precision defect correction (Algorithm 2) and reliable updates with
 * automatic fallback to defect correction (Sec. 2.3).
 *
 * Conventions fixed by this library where the paper is silent:
 *   - chiral gamma basis: gamma_k = [[0, -i sigma_k], [i sigma_k, 0]],
 *     gamma_4 = [[0, 1], [1, 0]], gamma_5 = diag(1, 1, -1, -1);
 *     mu = 0, 1, 2, 3 is x, y, z, t;
 *   - periodic boundaries (optionally antiperiodic in t, dwf_opts);
 *   - D_w^EO maps odd 4D sites to even ones; C acts on odd sites;
 *     parity of (x, y, z, t) is (x + y + z + t) mod 2, even = 0.
 *
 * Host layouts (canonical, Sec. 3.1 Eq. (12)):
 *   gauge  : double [Lt][Lz][Ly][Lx][mu][a][b][re, im]; U_mu(x) is the
 *            SU(3) link from x to x + mu^.
 *   spinor : double [Lt][Lz][Ly][Lx][s][24]; the 24 reals of a site are
 *            c = 2 * (3 * spin + colour) + reim.  With nrhs > 1 the
 *            right-hand sides follow each other (stride = one spinor).
 *
 * Errors: every function returns DWF_OK (0) or a negative DWF_E* code and
 * never throws; dwf_last_error() gives a message for the calling thread.
 * Ownership: the caller owns all buffers it passes; the library reads or
 * writes them only during the call (dwf_submit copies b before returning,
 * dwf_poll writes x only when it returns a final status).  A context owns
 * all device memory it allocates; dwf_destroy frees it.
 */
#ifndef DWF_H
#define DWF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define DWF_OK 0
#define DWF_PENDING 1        /* dwf_poll: the request is not finished */
#define DWF_EINVAL (-1)      /* bad argument, size or parameter */
#define DWF_ENOMEM (-2)      /* device or host allocation failed */
#define DWF_EDEVICE (-3)     /* a HIP call failed */
#define DWF_ENOCONV (-4)     /* a solve stopped before its tolerance (x holds the best iterate) */
#define DWF_EBUSY (-5)       /* reserved: no call returns it (calls on one context serialise) */
#define DWF_ENOTFOUND (-6)   /* dwf_poll: unknown or already collected ticket */

/* operators for dwf_apply (all in the host spinor layout, full 5D lattice) */
#define DWF_OP_DW 0      /* D_w on every slice, Eq. (2)                                */
#define DWF_OP_HOP_EO 1  /* D_w^EO: hopping term, odd -> even (Eq. (14)); odd out = 0 */
#define DWF_OP_HOP_OE 2  /* D_w^OE: even -> odd; even out = 0                          */
#define DWF_OP_M5 3      /* M5 of Eq. (8), per 4D site                                 */
#define DWF_OP_M5T 4     /* M5^T                                                       */
#define DWF_OP_C 5       /* C = 1 - M5 D^OE M5 D^EO on odd sites (Eq. (11)); even out = 0 */
#define DWF_OP_CDAG 6    /* C^dag = g5 (1 - D^OE M5^T D^EO M5^T) g5                   */
#define DWF_OP_CCDAG 7   /* C C^dag                                                    */
#define DWF_OP_D 8       /* the 5D operator D of Eq. (5)                               */
#define DWF_OP_DDAG 9    /* D^dag                                                      */

/* arithmetic / storage precision */
#define DWF_PREC_FP64 0
#define DWF_PREC_FP32 1
#define DWF_PREC_FP16 2  /* binary16 storage with one FP32 scale per 5D site, FP32 arithmetic */

/* Gauge-link storage of a dwf_apply, or-ed into its prec argument (Sec. 3.2
 * stages the links of a site once for all Ns slices; the paper gives no
 * storage format):
 *   DWF_LINKS_AUTO : the inner solver's choice -- FP64 18 reals; FP32 and
 *                    FP16 storage 12 reals (rows 0 and 1, row 2 rebuilt as
 *                    conj(row0 x row1)) when the field passes the SU(3) check
 *                    of dwf_create, else 18 reals (FP32)
 *   DWF_LINKS_18   : all 18 reals (FP64, FP32)
 *   DWF_LINKS_12   : 12 reals (FP32, FP16); DWF_EINVAL unless the field is SU(3)
 * Other combinations give DWF_EINVAL. */
#define DWF_LINKS_AUTO 0x000
#define DWF_LINKS_18 0x100
#define DWF_LINKS_12 0x200

/* A field is SU(3) for the 12-real links when every link satisfies
 * max_b |U_2b - conj(U_0 x U_1)_b| <= DWF_SU3_TOL (the FP32 rounding scale):
 * then the third row rebuilt from the first two is the stored one. */
#define DWF_SU3_TOL 1e-6

typedef struct dwf_ctx dwf_ctx;

typedef struct dwf_opts {
    int antiperiodic_t;      /* 0: periodic in t (default); 1: antiperiodic               */
    int device;              /* HIP device ordinal (default 0)                            */
    int sites_per_block;     /* 4D sites per workgroup in the stencil; 0 = automatic      */
    int xcd_remap;           /* 0 (default) or 1: consecutive lattice blocks on one XCD;
                                -1: hardware dispatch order                               */
    size_t hbm_budget_bytes; /* serving admission budget; 0 = 80% of free device memory   */
} dwf_opts;

typedef struct dwf_solve_params {
    double tol;              /* target ||b - D x|| / ||b|| (default 1e-10)               */
    int inner_prec;          /* DWF_PREC_FP32 (default), DWF_PREC_FP16 or DWF_PREC_FP64   */
    int reliable;            /* 1: reliable updates, falling back to defect correction
                                when they stall (default); 0: defect correction only     */
    double eps_inner;        /* inner relative tolerance of a cycle; 0 = per-precision
                                default: reliable updates restart when the iterated residual
                                has fallen to 0.1 (FP32) / 0.3 (FP16 storage) of its value
                                at the last restart; defect correction cycles run to 1e-5
                                (FP32) / 2e-3 (FP16); FP64 inner solves run to tol        */
    int maxiter;             /* cap on inner iterations per right-hand side (default 50000) */
    int check_every;         /* inner iterations between host checks; 0 = adaptive        */
    int use_graph;           /* 1: capture inner iterations in a hipGraph (default)       */
    int link_compress;       /* links in the inner solve: -1 auto (default: 12-real rows 0-1,
                                row 2 = conj(row0 x row1), for FP32 and FP16 storage when
                                the field passes the SU(3) check of dwf_create, else 18-real);
                                0: 18-real (FP32); 1: 12-real (DWF_EINVAL for a field that
                                is not SU(3)).  FP64 always uses 18-real; FP16 storage needs
                                an SU(3) field (DWF_EINVAL otherwise)                      */
    int use_guess;           /* 1: x holds an initial guess on entry; 0: start from zero  */
    int debug_stall_after;   /* test hook: >0 declares reliable updates stalled after this
                                many restarts, forcing the defect-correction fallback     */
    int system;              /* DWF_SYSTEM_D (default): D x = b of Eq. (5), full 5D lattice;
                                DWF_SYSTEM_CCDAG: C C^dag w = b on the odd sites (the solve
                                of the HMC force, Sec. 2.1): the even sites of b are
                                ignored and those of w are zero; true_residual is then
                                ||b_o - C C^dag w|| / ||b_o||                               */
    int tile;                /* 0 (default): tile of the inner kernels chosen by the autotuner
                                (timed at engine creation and cached per arch, lattice, Ns,
                                precision, links and nrhs; DWF_TUNE_CACHE names a file that
                                keeps the cache across processes); k >= 1: candidate k
                                (testing and reproducibility; DWF_EINVAL past the last)   */
} dwf_solve_params;

#define DWF_SYSTEM_D 0
#define DWF_SYSTEM_CCDAG 1

typedef struct dwf_solve_stats {
    int status;              /* DWF_OK or DWF_ENOCONV                                     */
    int iters;               /* inner CG iterations                                       */
    int restarts;            /* outer high-precision residual recomputations              */
    int reliable_updates;    /* restarts taken in reliable-update mode (p kept)           */
    int fallback;            /* 1 if the solve switched to defect correction              */
    int rhs_per_block;       /* right-hand sides per stencil workgroup, tuned per batch   */
    int tile;                /* tile candidate of the inner kernels (1-based, as params.tile) */
    int sites_per_block;     /* its 4D sites per workgroup                                */
    int block_order;         /* its workgroup order: 0 lexicographic blocks, 1 t-fastest in
                                XCD chunks of t-slices, w >= 2 the same with z-plane tiles
                                of w blocks                                               */
    double true_residual;    /* ||b - D x|| / ||b||, FP64 full operator on the GPU        */
    double schur_residual;   /* ||b'' - C y|| / ||b''|| of the final iterate              */
    double seconds;          /* wall time of the solve on the device stream               */
    double gflops;           /* flops of the method / seconds: per inner iteration and odd
                                5D site 5280 + 192 Ns + 288 (four hops, four fifth-
                                dimension matrices, the CG vector algebra)              */
    double hbm_gbytes;       /* algorithmic HBM bytes moved / 1e9                         */
} dwf_solve_stats;

/*
 * dwf_odwf_weights -- the weights omega_s of optimal domain-wall fermions (Sec.
 * 2.1: sigma = omega, with omega_s fixed for optimal chiral symmetry; the
 * paper cites the formula without giving it, so it is derived here).  With
 * sigma = omega the 4D operator on the walls depends on the weights only
 * through the transfer product
 *     Pi(lam) = prod_s (1 - omega_s lam) / (1 + omega_s lam)
 * over the spectrum of H = gamma_5 D_w, and is chirally exact where Pi = 0.
 * The weights returned minimise max |Pi| for lam in [lambda_min, lambda_max]
 * (Zolotarev's third problem):
 *     omega_s = dn((2s - 1) K / (2 Ns), k) / lambda_min,   s = 1 .. Ns,
 *     k = sqrt(1 - (lambda_min / lambda_max)^2),  K = K(k),
 * with the error equioscillating at Ns + 1 points of the interval.  omega_1
 * ~ 1 / lambda_min falls to omega_Ns ~ 1 / lambda_max (the 4D operator does
 * not depend on their order along s).  The caller supplies bounds of |H|'s
 * spectrum; pass omega as both sigma and omega to dwf_create.  Host only.
 *   omega : Ns doubles, written.
 * Errors: DWF_EINVAL unless Ns >= 1 and 0 < lambda_min <= lambda_max < inf.
 */
int dwf_odwf_weights(int Ns, double lambda_min, double lambda_max, double *omega);

/* Fill defaults. */
void dwf_default_opts(dwf_opts *opts);
void dwf_default_params(dwf_solve_params *params);

/*
 * dwf_create -- build one operator: resident gauge field and fifth-dimension
 * tables (Eqs. (1)-(9)).
 *   gauge  : host pointer, FP64, layout above (copied to the device).
 *   dims   : Lx, Ly, Lz, Lt, each even and >= 2.
 *   Ns     : 1 <= Ns <= 32.   m0 in (0, 2).   mq: quark mass (kappa = mq / (2 m0)).
 *            At most 2^30 5D half-lattice sites: Lx Ly Lz Lt / 2 * Ns <= 2^30.
 *   sigma, omega : host arrays of Ns doubles, omega_s > 0.
 *   opts   : NULL for defaults.
 * Errors: DWF_EINVAL for bad sizes or parameters (checked before the gauge
 * field is read), or when (1 + cL) or X of Eq. (7) is singular; DWF_ENOMEM;
 * DWF_EDEVICE.
 */
int dwf_create(dwf_ctx **out, const double *gauge, const int dims[4], int Ns,
               double m0, double mq, const double *sigma, const double *omega,
               const dwf_opts *opts);

/* Release a context and all its device memory (NULL is ignored). */
void dwf_destroy(dwf_ctx *ctx);

/*
 * dwf_gauge_su3_deviation -- host-only check behind the 12-real link storage:
 * *dev = max over links and columns b of |U_2b - conj(U_0 x U_1)_b| (the
 * difference between the third row and the one the 12-real storage rebuilds
 * from the first two; +inf if any entry is not finite).  gauge and dims as in
 * dwf_create.  dwf_create runs the same check; a field above DWF_SU3_TOL is
 * solved with 18-real links in FP32, and 12-real links or FP16 storage are
 * refused for it (DWF_EINVAL).  Touches no device.
 */
int dwf_gauge_su3_deviation(const double *gauge, const int dims[4], double *dev);

/*
 * dwf_apply -- out = op(in) for nrhs spinors in the host layout, in
 * precision prec (inputs are rounded to prec, outputs returned in FP64),
 * optionally or-ed with a DWF_LINKS_* link storage.
 * in, out: host pointers of nrhs * V4 * Ns * 24 doubles.  The host forms
 * stage one spinor at a time through a device buffer that the context keeps
 * (allocated at the first host-pointer call, two spinors), so they allocate
 * no device memory per call.
 */
int dwf_apply(dwf_ctx *ctx, int op, int prec, const double *in, double *out, int nrhs);

/* Same, with device pointers (host layout, FP64) on a HIP stream (NULL =
 * the context's stream); returns after the work is enqueued and finished. */
int dwf_apply_dev(dwf_ctx *ctx, int op, int prec, const double *in_dev, double *out_dev,
                  int nrhs, void *hip_stream);

/*
 * dwf_apply_dev_noalloc -- dwf_apply_dev for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same operators, kernels and results, with the
 * eight half-field workspace taken from a static device array of the library
 * (64 MiB, held by every GPU the library runs on until the process ends)
 * instead of a per-context allocation.  Makes no hipMalloc / hipFree or other
 * allocating call.  Arguments as dwf_apply_dev.  DWF_EINVAL when the
 * workspace, nrhs x (V4 Ns / 2) x 8 half fields of the storage precision
 * (FP64 1536, FP32 768, FP16 416 bytes per 5D half site and right-hand side,
 * rounded up), exceeds the array.  All calls on one GPU share the array:
 * calls that overlap in time on one GPU race (serialize them).
 */
int dwf_apply_dev_noalloc(dwf_ctx *ctx, int op, int prec, const double *in_dev, double *out_dev,
                          int nrhs, void *hip_stream);

/*
 * dwf_solve -- solve D x = b (Eq. (5)) for nrhs right-hand sides.
 *   b, x  : host pointers, nrhs spinors in the host layout.  x is read as
 *           the initial guess when params->use_guess, and holds the
 *           solution on return (the best iterate on DWF_ENOCONV).
 *   params: NULL for defaults.   stats: NULL or nrhs entries.
 * With nrhs > 1 the right-hand sides are solved together through the
 * multi-RHS stencil (each gauge link is read once for all of them).
 * Returns DWF_OK when every right-hand side reached params->tol, else
 * DWF_ENOCONV.  Like dwf_apply, the host form stages one spinor at a time
 * through the context's device buffer (no device allocation per call; the
 * solve engine itself is allocated once per (params, nrhs) and kept).
 */
int dwf_solve(dwf_ctx *ctx, const double *b, double *x, int nrhs,
              const dwf_solve_params *params, dwf_solve_stats *stats);

/* Same, with device pointers (FP64, host layout) on a HIP stream. */
int dwf_solve_dev(dwf_ctx *ctx, const double *b_dev, double *x_dev, int nrhs,
                  const dwf_solve_params *params, dwf_solve_stats *stats, void *hip_stream);

/*
 * dwf_propagator -- 4D valence-quark propagators from the 5D solve (the use of
 * the CG for valence quark propagators, Secs. 2.2 and 5).  The quark mass
 * enters D only through the corner of L (Eq. (4)), which couples the +
 * chirality at s = Ns to s = 1 and the - chirality at s = 1 to s = Ns:
 * D(mq) = D(0) + kappa W R, kappa = mq / (2 m0), with
 *     R psi      = P_+ psi_Ns + P_- psi_1          (the 4D quark field, 5D -> 4D)
 *     (W eta)_1  = (1 - sigma_1 D_w) P_+ eta,
 *     (W eta)_Ns = (1 - sigma_Ns D_w) P_- eta      (the 5D source of a 4D spinor).
 * For each of nsrc 4D sources eta_k it solves D x = W eta_k (as dwf_solve,
 * all sources in one batch, FP64 true residual of the 5D system <= tol) and
 * returns out_k = R x.  With this choice the mass is additive:
 * S(mq)^-1 = S(0)^-1 + kappa (S eta = R D^-1 W eta).  No contact term is
 * subtracted (the paper defines none).
 *   eta, out : host pointers, nsrc 4D spinors [Lt][Lz][Ly][Lx][24] each (the
 *              spinor layout of this header without the s index).
 *   params   : as dwf_solve (system must be DWF_SYSTEM_D; use_guess ignored).
 *   stats    : NULL or nsrc entries, those of the 5D solves.
 * The host form goes through the context's staging buffer in groups of up to
 * Ns sources; the 5D work buffers (three 5D spinors per source) are kept by
 * the context.  Returns DWF_OK, DWF_ENOCONV (out holds the best iterate's
 * projection) or an error.
 */
int dwf_propagator(dwf_ctx *ctx, const double *eta, double *out, int nsrc,
                   const dwf_solve_params *params, dwf_solve_stats *stats);

/* Same, with device pointers (FP64, the 4D layout above) on a HIP stream. */
int dwf_propagator_dev(dwf_ctx *ctx, const double *eta_dev, double *out_dev, int nsrc,
                       const dwf_solve_params *params, dwf_solve_stats *stats, void *hip_stream);

/*
 * dwf_submit -- enqueue one solve request on the context's device server
 * (continuous batching: requests on the same gauge field and fifth-dimension
 * weights are solved together in the multi-RHS kernels, with their own mq;
 * admission is limited by the HBM budget of dwf_opts).  Requests on lattices
 * of at least 2^19 half 5D sites, where one solve nearly fills the GPU, enter
 * service in arrival order, two at a time (environment variable
 * DWF_SERVE_LARGE_LANES), beside the smaller ones.  b (host, one spinor) is
 * copied before the call returns.  *ticket identifies the request.
 */
int dwf_submit(dwf_ctx *ctx, const double *b, const dwf_solve_params *params, uint64_t *ticket);

/* Same, with the quark mass of this request (the context's mq otherwise). */
int dwf_submit_mass(dwf_ctx *ctx, const double *b, double mq, const dwf_solve_params *params,
                    uint64_t *ticket);

/*
 * dwf_poll -- wait up to timeout_us (0: do not wait, <0: forever) for a
 * request.  Returns DWF_PENDING while it runs; otherwise its final status
 * (DWF_OK / DWF_ENOCONV / error), writes x (host, one spinor) and *stats
 * (may be NULL) and forgets the ticket.  DWF_ENOTFOUND for unknown tickets.
 */
int dwf_poll(uint64_t ticket, double *x, dwf_solve_stats *stats, int timeout_us);

/* Server statistics since the last reset: latencies in seconds. */
typedef struct dwf_server_stats {
    int64_t completed;
    int64_t admitted;
    int64_t peak_batch;
    int64_t waits_for_memory;
    double p50_latency;
    double p99_latency;
    double busy_seconds;
} dwf_server_stats;
int dwf_server_stats_get(dwf_server_stats *out, int reset);

/*
 * dwf_time_kernels -- profiling aid: average device time (milliseconds) of
 * the inner CG kernels over `launches` back-to-back launches on the context's
 * stream bracketed by HIP events, and the algorithmic HBM bytes one launch
 * must move (every operand read or written once).  Entries, in launch order:
 *   0  T: t1 = M5^T gamma_5 r, once at the start of an inner cycle;
 *   1  A: t2 = M5^T D^EO t1;
 *   2  B: u = r - gamma_5 D^OE t2 + beta u (the direction as C^dag p), |u|^2;
 *   3  C: t3 = M5 D^EO u;
 *   4  D: r -= alpha (u - M5 D^OE t3), y += alpha u, |r|^2, t1 = M5^T gamma_5 r.
 * One inner iteration is A, B, C, D (Algorithm 1, Secs. 3.2-3.5).  Uses the workspace left by the last
 * dwf_solve/dwf_solve_dev with the same params and nrhs (DWF_EINVAL if there
 * is none); it overwrites that workspace's low-precision vectors.
 */
int dwf_time_kernels(dwf_ctx *ctx, const dwf_solve_params *params, int nrhs, int launches,
                     double ms[5], double bytes[5]);

/*
 * dwf_stream_copy -- profiling aid: a plain copy of bytes (a multiple of 16)
 * from src_dev to dst_dev on device `device` and the given HIP stream (not
 * NULL), with ordinary cached loads and stores (nontemporal = 0, as the hop
 * kernels gather their inputs) or non-temporal ones (1, as the CG kernels
 * stream vectors they touch once).  Its known byte count calibrates the
 * memory counters that measure the other kernels' traffic.  Returns after
 * the copy has finished.
 */
int dwf_stream_copy(const void *src_dev, void *dst_dev, size_t bytes, int nontemporal, int device,
                    void *hip_stream);

/* Message of the last failing call on this thread ("" if none). */
const char *dwf_last_error(void);

/* Library version string. */
const char *dwf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DWF_H */
