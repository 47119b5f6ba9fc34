/*
 * Plain FP64 CPU oracle for the even-odd preconditioned 5D domain-wall
 * fermion solver (Chiu, Hsieh, Mao, Ogawa: "GPU-Based Conjugate Gradient
 * Solver for Lattice QCD with Domain-Wall Fermions", Lattice 2010).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this file's library.  It shares
 * no code, header, table or helper with the HIP library: every operator is
 * written out here from its definition in the paper, with plain loops over
 * full-lattice vectors in the canonical host layout, so that it can be read
 * against the paper by eye.
 *
 * Layouts (host, canonical; Sec. 3.1, Eq. (12)):
 *   4D site   n4 = x + Lx (y + Ly (z + Lz t))
 *   spinor    complex psi[(n4 * Ns + s) * 12 + 3 * spin + colour]
 *             (= reals c + 24 s + 24 Ns n4, c = 2 (3 spin + colour) + reim)
 *   gauge     complex U[(n4 * 4 + mu) * 9 + 3 a + b], U_mu(x) links x -> x+mu
 *   s-space matrices (Ns x Ns, real) are row-major.
 * Parity of a 4D site: (x + y + z + t) mod 2, even = 0.
 *
 * Readings where the paper is silent (stated once here, used throughout):
 *   - gamma matrices in the chiral basis, gamma_k = [[0, -i sigma_k],
 *     [i sigma_k, 0]] (k = 1,2,3), gamma_4 = [[0, 1], [1, 0]]; mu = 0..3 is
 *     x, y, z, t <-> gamma_1..gamma_4, gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4;
 *   - periodic boundaries, with an optional sign bct on links that cross the
 *     t boundary (bct = -1 gives antiperiodic time);
 *   - D^EO maps odd sites to even sites (rows even), the Schur complement C
 *     lives on odd sites;
 *   - the Schur system C y = b'' is solved by CG on C C^dag (Sec. 2.2) in the
 *     form that tracks y = C^dag w directly (Craig's method), so that the CG
 *     residual is the residual of C y = b'' itself.
 *
 * Parity of every function is pinned by the tests in tests/test_oracle_*.py
 * (closed forms, identities, special cases and a dense brute-force solve).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* Gamma matrices (chiral basis).                                            */
/* ------------------------------------------------------------------------ */

/* Loops over fewer 5D sites than this run on one thread: on small lattices the
 * cost of waking a thread team exceeds the work (the arithmetic is the same). */
#define OMP_MIN_WORK 16384

static cplx G[5][4][4];
static int g_ready = 0;

static void gamma_init(void)
{
    if (g_ready) return;
    memset(G, 0, sizeof G);
    const cplx Ii = _Complex_I;
    /* gamma_1 */
    G[0][0][3] = -Ii; G[0][1][2] = -Ii; G[0][2][1] = Ii;  G[0][3][0] = Ii;
    /* gamma_2 */
    G[1][0][3] = -1; G[1][1][2] = 1;  G[1][2][1] = 1;  G[1][3][0] = -1;
    /* gamma_3 */
    G[2][0][2] = -Ii; G[2][1][3] = Ii;  G[2][2][0] = Ii;  G[2][3][1] = -Ii;
    /* gamma_4 */
    G[3][0][2] = 1;  G[3][1][3] = 1;  G[3][2][0] = 1;  G[3][3][1] = 1;
    /* gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4, by matrix product */
    cplx a[4][4], b[4][4];
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            a[i][j] = 0;
            for (int k = 0; k < 4; k++) a[i][j] += G[0][i][k] * G[1][k][j];
        }
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            b[i][j] = 0;
            for (int k = 0; k < 4; k++) b[i][j] += a[i][k] * G[2][k][j];
        }
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            G[4][i][j] = 0;
            for (int k = 0; k < 4; k++) G[4][i][j] += b[i][k] * G[3][k][j];
        }
    g_ready = 1;
}

/* gamma matrix mu (0..3) or gamma_5 (mu = 4), 4x4 complex row-major. */
void orc_gamma(int mu, double *out)
{
    gamma_init();
    cplx *o = (cplx *)out;
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) o[4 * i + j] = G[mu][i][j];
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Lattice helpers.                                                          */
/* ------------------------------------------------------------------------ */

typedef struct { int L[4]; long V; } lat_t;

static lat_t lat_make(const int *dims)
{
    lat_t l;
    for (int i = 0; i < 4; i++) l.L[i] = dims[i];
    l.V = (long)dims[0] * dims[1] * dims[2] * dims[3];
    return l;
}

static void coords(const lat_t *l, long n, int c[4])
{
    for (int i = 0; i < 4; i++) { c[i] = (int)(n % l->L[i]); n /= l->L[i]; }
}

static long index4(const lat_t *l, const int c[4])
{
    return c[0] + (long)l->L[0] * (c[1] + (long)l->L[1] * (c[2] + (long)l->L[2] * c[3]));
}

static int parity(const int c[4]) { return (c[0] + c[1] + c[2] + c[3]) & 1; }

/* ------------------------------------------------------------------------ */
/* Wilson hopping term, Eq. (2) without the mass term (= Eq. (14)).           */
/*   (H psi)(x) = -1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu)            */
/*                            + (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu) ] */
/* Applied on each fifth-dimension slice (U carries no s dependence).         */
/* only_parity: -1 = all output sites, 0/1 = only output sites of that        */
/* parity (others are set to zero); this gives D_w^EO (0) and D_w^OE (1).     */
/* ------------------------------------------------------------------------ */

static void hop_apply(const lat_t *l, int Ns, const cplx *U, double bct,
                      int only_parity, const cplx *in, cplx *out)
{
    gamma_init();
#pragma omp parallel for schedule(static) if (l->V * Ns > OMP_MIN_WORK)
    for (long n = 0; n < l->V; n++) {
        int c[4];
        coords(l, n, c);
        for (int s = 0; s < Ns; s++) {
            cplx *o = out + (n * Ns + s) * 12;
            for (int k = 0; k < 12; k++) o[k] = 0;
        }
        if (only_parity >= 0 && parity(c) != only_parity) continue;
        for (int mu = 0; mu < 4; mu++) {
            int cf[4], cb[4];
            memcpy(cf, c, sizeof cf);
            memcpy(cb, c, sizeof cb);
            cf[mu] = (c[mu] + 1) % l->L[mu];
            cb[mu] = (c[mu] - 1 + l->L[mu]) % l->L[mu];
            double sf = (mu == 3 && c[3] == l->L[3] - 1) ? bct : 1.0;
            double sb = (mu == 3 && c[3] == 0) ? bct : 1.0;
            long nf = index4(l, cf), nb = index4(l, cb);
            const cplx *Uf = U + (n * 4 + mu) * 9;   /* U_mu(x)       */
            const cplx *Ub = U + (nb * 4 + mu) * 9;  /* U_mu(x - mu)  */
            for (int s = 0; s < Ns; s++) {
                const cplx *pf = in + (nf * Ns + s) * 12;
                const cplx *pb = in + (nb * Ns + s) * 12;
                cplx vf[4][3], vb[4][3];
                for (int sp = 0; sp < 4; sp++)
                    for (int a = 0; a < 3; a++) {
                        cplx f = 0, b = 0;
                        for (int bb = 0; bb < 3; bb++) {
                            f += Uf[3 * a + bb] * pf[3 * sp + bb];
                            b += conj(Ub[3 * bb + a]) * pb[3 * sp + bb];
                        }
                        vf[sp][a] = sf * f;
                        vb[sp][a] = sb * b;
                    }
                cplx *o = out + (n * Ns + s) * 12;
                for (int i = 0; i < 4; i++)
                    for (int a = 0; a < 3; a++) {
                        cplx acc = vf[i][a] + vb[i][a];
                        for (int j = 0; j < 4; j++)
                            acc += G[mu][i][j] * (vb[j][a] - vf[j][a]);
                        o[3 * i + a] += -0.5 * acc;
                    }
            }
        }
    }
}

/* D_w psi on every slice, Eq. (2): (d - m0) psi + H psi, d = 4. */
void orc_dw(const double *U, const int *dims, int Ns, double m0, double bct,
            const double *in, double *out)
{
    lat_t l = lat_make(dims);
    hop_apply(&l, Ns, (const cplx *)U, bct, -1, (const cplx *)in, (cplx *)out);
    cplx *o = (cplx *)out;
    const cplx *p = (const cplx *)in;
    long N = l.V * Ns * 12;
    for (long i = 0; i < N; i++) o[i] += (4.0 - m0) * p[i];
}

/* Hopping block: out_parity = 0 gives D_w^EO, 1 gives D_w^OE (Eqs. (6),(14)). */
void orc_hop(const double *U, const int *dims, int Ns, double bct, int out_parity,
             const double *in, double *out)
{
    lat_t l = lat_make(dims);
    hop_apply(&l, Ns, (const cplx *)U, bct, out_parity, (const cplx *)in, (cplx *)out);
}

/* ------------------------------------------------------------------------ */
/* Fifth-dimension operators, Eqs. (3)-(4), (7)-(9).                         */
/* ------------------------------------------------------------------------ */

/* (L_+)_{ss'} (0-based): 1 on s' = s - 1 for s >= 1, -kappa at (0, Ns-1). */
static void lplus(int Ns, double kappa, double *Lp)
{
    memset(Lp, 0, sizeof(double) * Ns * Ns);
    for (int s = 1; s < Ns; s++) Lp[s * Ns + (s - 1)] = 1.0;
    Lp[0 * Ns + (Ns - 1)] += -kappa;
}

static void transpose(int n, const double *A, double *B)
{
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) B[j * n + i] = A[i * n + j];
}

static void matmul(int n, const double *A, const double *B, double *C)
{
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            double acc = 0;
            for (int k = 0; k < n; k++) acc += A[i * n + k] * B[k * n + j];
            C[i * n + j] = acc;
        }
}

/* Gauss-Jordan inverse with partial pivoting; returns -1 if singular. */
static int gj_inverse(int n, const double *A, double *Ainv)
{
    double *a = malloc(sizeof(double) * n * n);
    memcpy(a, A, sizeof(double) * n * n);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) Ainv[i * n + j] = (i == j);
    double scale = 0;
    for (int i = 0; i < n * n; i++) scale = fmax(scale, fabs(A[i]));
    for (int col = 0; col < n; col++) {
        int piv = col;
        for (int r = col + 1; r < n; r++)
            if (fabs(a[r * n + col]) > fabs(a[piv * n + col])) piv = r;
        if (!(fabs(a[piv * n + col]) > 1e-14 * scale)) { free(a); return -1; }
        if (piv != col)
            for (int j = 0; j < n; j++) {
                double t = a[col * n + j]; a[col * n + j] = a[piv * n + j]; a[piv * n + j] = t;
                t = Ainv[col * n + j]; Ainv[col * n + j] = Ainv[piv * n + j]; Ainv[piv * n + j] = t;
            }
        double d = a[col * n + col];
        for (int j = 0; j < n; j++) { a[col * n + j] /= d; Ainv[col * n + j] /= d; }
        for (int r = 0; r < n; r++) {
            if (r == col) continue;
            double f = a[r * n + col];
            if (f == 0) continue;
            for (int j = 0; j < n; j++) {
                a[r * n + j] -= f * a[col * n + j];
                Ainv[r * n + j] -= f * Ainv[col * n + j];
            }
        }
    }
    free(a);
    return 0;
}

int orc_invert(int n, const double *A, double *Ainv) { return gj_inverse(n, A, Ainv); }

/* L_+ and L_- = L_+^T as dense Ns x Ns matrices, Eq. (4), kappa = mq / (2 m0). */
void orc_lmat(int Ns, double m0, double mq, double *Lp, double *Lm)
{
    double kappa = mq / (2.0 * m0);
    lplus(Ns, kappa, Lp);
    transpose(Ns, Lp, Lm);
}

/* X = (d - m0) omega (1 + c L) + (1 - L), Y = omega (1 + c L), c = sigma/omega,
 * for one chirality given its L (Eq. (7)). */
static void xy_one(int Ns, double m0, const double *sigma, const double *omega,
                   const double *Lc, double *X, double *Y)
{
    for (int s = 0; s < Ns; s++)
        for (int t = 0; t < Ns; t++) {
            double id = (s == t);
            double c = sigma[s] / omega[s];
            double onepcl = id + c * Lc[s * Ns + t];
            Y[s * Ns + t] = omega[s] * onepcl;
            X[s * Ns + t] = (4.0 - m0) * omega[s] * onepcl + id - Lc[s * Ns + t];
        }
}

void orc_xy(int Ns, double m0, double mq, const double *sigma, const double *omega,
            double *Xp, double *Xm, double *Yp, double *Ym)
{
    double *Lp = malloc(sizeof(double) * Ns * Ns), *Lm = malloc(sizeof(double) * Ns * Ns);
    orc_lmat(Ns, m0, mq, Lp, Lm);
    xy_one(Ns, m0, sigma, omega, Lp, Xp, Yp);
    xy_one(Ns, m0, sigma, omega, Lm, Xm, Ym);
    free(Lp); free(Lm);
}

/* M5 first form of Eq. (8): sqrt(omega)^-1 Y X^-1 sqrt(omega), per chirality. */
int orc_m5_form1(int Ns, double m0, double mq, const double *sigma, const double *omega,
                 double *M5p, double *M5m)
{
    int n2 = Ns * Ns, rc = 0;
    double *X = malloc(sizeof(double) * n2), *Y = malloc(sizeof(double) * n2);
    double *Xi = malloc(sizeof(double) * n2), *T = malloc(sizeof(double) * n2);
    double *Lp = malloc(sizeof(double) * n2), *Lm = malloc(sizeof(double) * n2);
    orc_lmat(Ns, m0, mq, Lp, Lm);
    for (int ch = 0; ch < 2; ch++) {
        double *M = ch == 0 ? M5p : M5m;
        xy_one(Ns, m0, sigma, omega, ch == 0 ? Lp : Lm, X, Y);
        if (gj_inverse(Ns, X, Xi)) { rc = -1; break; }
        matmul(Ns, Y, Xi, T);
        for (int s = 0; s < Ns; s++)
            for (int t = 0; t < Ns; t++)
                M[s * Ns + t] = T[s * Ns + t] * sqrt(omega[t]) / sqrt(omega[s]);
    }
    free(X); free(Y); free(Xi); free(T); free(Lp); free(Lm);
    return rc;
}

/* M5 second form of Eq. (8):
 * [ (d - m0) + sqrt(omega)^-1 (1 - L) (1 + c L)^-1 sqrt(omega)^-1 ]^-1. */
int orc_m5_form2(int Ns, double m0, double mq, const double *sigma, const double *omega,
                 double *M5p, double *M5m)
{
    int n2 = Ns * Ns, rc = 0;
    double *A = malloc(sizeof(double) * n2), *Ai = malloc(sizeof(double) * n2);
    double *B = malloc(sizeof(double) * n2), *T = malloc(sizeof(double) * n2);
    double *Lp = malloc(sizeof(double) * n2), *Lm = malloc(sizeof(double) * n2);
    orc_lmat(Ns, m0, mq, Lp, Lm);
    for (int ch = 0; ch < 2; ch++) {
        const double *Lc = ch == 0 ? Lp : Lm;
        double *M = ch == 0 ? M5p : M5m;
        for (int s = 0; s < Ns; s++)
            for (int t = 0; t < Ns; t++) {
                double id = (s == t);
                A[s * Ns + t] = id + sigma[s] / omega[s] * Lc[s * Ns + t];  /* 1 + cL */
                B[s * Ns + t] = id - Lc[s * Ns + t];                         /* 1 - L  */
            }
        if (gj_inverse(Ns, A, Ai)) { rc = -1; break; }
        matmul(Ns, B, Ai, T);
        for (int s = 0; s < Ns; s++)
            for (int t = 0; t < Ns; t++)
                A[s * Ns + t] = (s == t) * (4.0 - m0) + T[s * Ns + t] / (sqrt(omega[s]) * sqrt(omega[t]));
        if (gj_inverse(Ns, A, M)) { rc = -1; break; }
    }
    free(A); free(Ai); free(B); free(T); free(Lp); free(Lm);
    return rc;
}

/* Apply s-space matrices per chirality at every 4D site:
 *   out_s = sum_s' [ P_+ Mp_{ss'} + P_- Mm_{ss'} ] in_{s'},  P_pm = (1 pm gamma_5)/2. */
static void apply_s(const lat_t *l, int Ns, const double *Mp, const double *Mm,
                    const cplx *in, cplx *out)
{
    gamma_init();
    cplx Pp[4][4], Pm[4][4];
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            Pp[i][j] = 0.5 * ((i == j) + G[4][i][j]);   /* P_+ = (1 + gamma_5)/2 */
            Pm[i][j] = 0.5 * ((i == j) - G[4][i][j]);   /* P_- = (1 - gamma_5)/2 */
        }
#pragma omp parallel if (l->V * Ns > OMP_MIN_WORK)
    {
        cplx *pp = malloc(sizeof(cplx) * Ns * 12), *pm = malloc(sizeof(cplx) * Ns * 12);
#pragma omp for schedule(static)
        for (long n = 0; n < l->V; n++) {
            /* chiral projections of every slice of this 4D site */
            for (int t = 0; t < Ns; t++) {
                const cplx *p = in + (n * Ns + t) * 12;
                for (int i = 0; i < 4; i++)
                    for (int a = 0; a < 3; a++) {
                        cplx ap = 0, am = 0;
                        for (int j = 0; j < 4; j++) {
                            ap += Pp[i][j] * p[3 * j + a];
                            am += Pm[i][j] * p[3 * j + a];
                        }
                        pp[t * 12 + 3 * i + a] = ap;
                        pm[t * 12 + 3 * i + a] = am;
                    }
            }
            for (int s = 0; s < Ns; s++) {
                cplx *o = out + (n * Ns + s) * 12;
                for (int k = 0; k < 12; k++) {
                    cplx acc = 0;
                    for (int t = 0; t < Ns; t++)
                        acc += Mp[s * Ns + t] * pp[t * 12 + k] + Mm[s * Ns + t] * pm[t * 12 + k];
                    o[k] = acc;
                }
            }
        }
        free(pp);
        free(pm);
    }
}

void orc_apply_s(const int *dims, int Ns, const double *Mp, const double *Mm,
                 const double *in, double *out)
{
    lat_t l = lat_make(dims);
    apply_s(&l, Ns, Mp, Mm, (const cplx *)in, (cplx *)out);
}

/* L psi with L = P_+ L_+ + P_- L_- (Eq. (3)). */
void orc_L(const int *dims, int Ns, double m0, double mq, const double *in, double *out)
{
    double *Lp = malloc(sizeof(double) * Ns * Ns), *Lm = malloc(sizeof(double) * Ns * Ns);
    orc_lmat(Ns, m0, mq, Lp, Lm);
    orc_apply_s(dims, Ns, Lp, Lm, in, out);
    free(Lp); free(Lm);
}

/* gamma_5 on every site. */
static void g5_apply(long nsites5, const cplx *in, cplx *out)
{
    gamma_init();
#pragma omp parallel for schedule(static) if (nsites5 > OMP_MIN_WORK)
    for (long n = 0; n < nsites5; n++) {
        cplx t[12];
        for (int i = 0; i < 4; i++)
            for (int a = 0; a < 3; a++) {
                cplx acc = 0;
                for (int j = 0; j < 4; j++) acc += G[4][i][j] * in[n * 12 + 3 * j + a];
                t[3 * i + a] = acc;
            }
        memcpy(out + n * 12, t, sizeof t);
    }
}

/* ------------------------------------------------------------------------ */
/* The 5D operator, Eq. (5): D = D_w (omega + sigma L) + (1 - L).            */
/* ------------------------------------------------------------------------ */

void orc_d5(const double *U, const int *dims, int Ns, double m0, double mq,
            const double *sigma, const double *omega, double bct,
            const double *in, double *out)
{
    lat_t l = lat_make(dims);
    long N = l.V * Ns * 12;
    cplx *Lpsi = malloc(sizeof(cplx) * N), *t = malloc(sizeof(cplx) * N);
    const cplx *p = (const cplx *)in;
    cplx *o = (cplx *)out;
    orc_L(dims, Ns, m0, mq, in, (double *)Lpsi);
    for (long n = 0; n < l.V; n++)
        for (int s = 0; s < Ns; s++)
            for (int k = 0; k < 12; k++) {
                long i = (n * Ns + s) * 12 + k;
                t[i] = omega[s] * p[i] + sigma[s] * Lpsi[i];
            }
    orc_dw(U, dims, Ns, m0, bct, (const double *)t, out);
    for (long i = 0; i < N; i++) o[i] += p[i] - Lpsi[i];
    free(Lpsi); free(t);
}

/* D^dag = (omega + L^dag sigma) D_w^dag + (1 - L^dag), D_w^dag = g5 D_w g5,
 * L^dag = P_+ L_+^T + P_- L_-^T (real L). */
void orc_d5dag(const double *U, const int *dims, int Ns, double m0, double mq,
               const double *sigma, const double *omega, double bct,
               const double *in, double *out)
{
    lat_t l = lat_make(dims);
    long N = l.V * Ns * 12;
    int n2 = Ns * Ns;
    double *Lp = malloc(sizeof(double) * n2), *Lm = malloc(sizeof(double) * n2);
    double *LpT = malloc(sizeof(double) * n2), *LmT = malloc(sizeof(double) * n2);
    orc_lmat(Ns, m0, mq, Lp, Lm);
    transpose(Ns, Lp, LpT);
    transpose(Ns, Lm, LmT);
    cplx *a = malloc(sizeof(cplx) * N), *b = malloc(sizeof(cplx) * N);
    cplx *c = malloc(sizeof(cplx) * N);
    const cplx *p = (const cplx *)in;
    cplx *o = (cplx *)out;
    g5_apply(l.V * Ns, p, a);
    orc_dw(U, dims, Ns, m0, bct, (const double *)a, (double *)b);
    g5_apply(l.V * Ns, b, b);                 /* b = D_w^dag psi */
    for (long n = 0; n < l.V; n++)
        for (int s = 0; s < Ns; s++)
            for (int k = 0; k < 12; k++) a[(n * Ns + s) * 12 + k] = sigma[s] * b[(n * Ns + s) * 12 + k];
    apply_s(&l, Ns, LpT, LmT, a, c);          /* c = L^dag sigma D_w^dag psi */
    apply_s(&l, Ns, LpT, LmT, p, a);          /* a = L^dag psi */
    for (long n = 0; n < l.V; n++)
        for (int s = 0; s < Ns; s++)
            for (int k = 0; k < 12; k++) {
                long i = (n * Ns + s) * 12 + k;
                o[i] = omega[s] * b[i] + c[i] + p[i] - a[i];
            }
    free(Lp); free(Lm); free(LpT); free(LmT); free(a); free(b); free(c);
}

/* ------------------------------------------------------------------------ */
/* Even-odd Schur complement, Eqs. (10)-(11).                                */
/* ------------------------------------------------------------------------ */

typedef struct {
    lat_t l;
    int Ns;
    const cplx *U;
    double bct;
    double *M5p, *M5m, *M5pT, *M5mT;
    long N;
    cplx *t1, *t2;
} schur_t;

static int schur_init(schur_t *S, const double *U, const int *dims, int Ns, double m0,
                      double mq, const double *sigma, const double *omega, double bct)
{
    S->l = lat_make(dims);
    S->Ns = Ns;
    S->U = (const cplx *)U;
    S->bct = bct;
    int n2 = Ns * Ns;
    S->M5p = malloc(sizeof(double) * n2); S->M5m = malloc(sizeof(double) * n2);
    S->M5pT = malloc(sizeof(double) * n2); S->M5mT = malloc(sizeof(double) * n2);
    int rc = orc_m5_form2(Ns, m0, mq, sigma, omega, S->M5p, S->M5m);
    transpose(Ns, S->M5p, S->M5pT);
    transpose(Ns, S->M5m, S->M5mT);
    S->N = S->l.V * Ns * 12;
    S->t1 = malloc(sizeof(cplx) * S->N);
    S->t2 = malloc(sizeof(cplx) * S->N);
    return rc;
}

static void schur_free(schur_t *S)
{
    free(S->M5p); free(S->M5m); free(S->M5pT); free(S->M5mT); free(S->t1); free(S->t2);
}

/* C psi = psi - M5 D^OE M5 D^EO psi on odd sites (Eq. (11)); even part of out = 0. */
static void schur_c(schur_t *S, const cplx *in, cplx *out)
{
    hop_apply(&S->l, S->Ns, S->U, S->bct, 0, in, S->t1);
    apply_s(&S->l, S->Ns, S->M5p, S->M5m, S->t1, S->t2);
    hop_apply(&S->l, S->Ns, S->U, S->bct, 1, S->t2, S->t1);
    apply_s(&S->l, S->Ns, S->M5p, S->M5m, S->t1, S->t2);
    for (long n = 0; n < S->l.V; n++) {
        int c[4];
        coords(&S->l, n, c);
        int odd = parity(c);
        for (long k = n * S->Ns * 12; k < (n + 1) * S->Ns * 12; k++)
            out[k] = odd ? in[k] - S->t2[k] : 0;
    }
}

/* C^dag psi = g5 (1 - D^OE M5^T D^EO M5^T) g5 psi on odd sites. */
static void schur_cdag(schur_t *S, const cplx *in, cplx *out)
{
    cplx *g = malloc(sizeof(cplx) * S->N);
    g5_apply(S->l.V * S->Ns, in, g);
    apply_s(&S->l, S->Ns, S->M5pT, S->M5mT, g, S->t1);
    hop_apply(&S->l, S->Ns, S->U, S->bct, 0, S->t1, S->t2);
    apply_s(&S->l, S->Ns, S->M5pT, S->M5mT, S->t2, S->t1);
    hop_apply(&S->l, S->Ns, S->U, S->bct, 1, S->t1, S->t2);
    g5_apply(S->l.V * S->Ns, S->t2, S->t2);
    for (long n = 0; n < S->l.V; n++) {
        int c[4];
        coords(&S->l, n, c);
        int odd = parity(c);
        for (long k = n * S->Ns * 12; k < (n + 1) * S->Ns * 12; k++)
            out[k] = odd ? in[k] - S->t2[k] : 0;
    }
    free(g);
}

void orc_schur_c(const double *U, const int *dims, int Ns, double m0, double mq,
                 const double *sigma, const double *omega, double bct,
                 const double *in, double *out)
{
    schur_t S;
    schur_init(&S, U, dims, Ns, m0, mq, sigma, omega, bct);
    schur_c(&S, (const cplx *)in, (cplx *)out);
    schur_free(&S);
}

void orc_schur_cdag(const double *U, const int *dims, int Ns, double m0, double mq,
                    const double *sigma, const double *omega, double bct,
                    const double *in, double *out)
{
    schur_t S;
    schur_init(&S, U, dims, Ns, m0, mq, sigma, omega, bct);
    schur_cdag(&S, (const cplx *)in, (cplx *)out);
    schur_free(&S);
}

static double norm2(long N, const cplx *a)
{
    double s = 0;
#pragma omp parallel for reduction(+ : s) if (N > 4 * OMP_MIN_WORK)
    for (long i = 0; i < N; i++) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return s;
}

/* ------------------------------------------------------------------------ */
/* Conjugate gradient on the normal equations, Algorithm 1.                  */
/* A = K K^dag, solved for w with y = K^dag w tracked directly:               */
/*   u = K^dag p;  alpha = |r|^2 / |u|^2;  y += alpha u;  r -= alpha K u;     */
/*   beta = |r_new|^2 / |r|^2;  p = r + beta p.                               */
/* This is Algorithm 1 with p_k A p_k = |K^dag p_k|^2; r stays the residual  */
/* of K y = b.  Stops when |r| <= tol |b| (2-norm).                           */
/* ------------------------------------------------------------------------ */

typedef void (*op_fn)(void *ctx, const cplx *in, cplx *out);

static int cgne(op_fn K, op_fn Kdag, void *ctx, long N, const cplx *b, cplx *y,
                double tol, int maxiter, int *iters, double *relres)
{
    cplx *r = malloc(sizeof(cplx) * N), *p = malloc(sizeof(cplx) * N);
    cplx *u = malloc(sizeof(cplx) * N), *q = malloc(sizeof(cplx) * N);
    /* r = b - K y for the initial guess y */
    K(ctx, y, q);
    for (long i = 0; i < N; i++) { r[i] = b[i] - q[i]; p[i] = r[i]; }
    double bb = norm2(N, b), rr = norm2(N, r);
    int k = 0;
    while (rr > tol * tol * bb && k < maxiter) {
        Kdag(ctx, p, u);
        double uu = norm2(N, u);
        if (!(uu > 0)) break;
        double alpha = rr / uu;
        K(ctx, u, q);
        for (long i = 0; i < N; i++) { y[i] += alpha * u[i]; r[i] -= alpha * q[i]; }
        double rr_new = norm2(N, r);
        double beta = rr_new / rr;
        for (long i = 0; i < N; i++) p[i] = r[i] + beta * p[i];
        rr = rr_new;
        k++;
    }
    *iters = k;
    *relres = bb > 0 ? sqrt(rr / bb) : 0;
    free(r); free(p); free(u); free(q);
    return (rr <= tol * tol * bb) ? 0 : 1;
}

static void op_c(void *ctx, const cplx *in, cplx *out) { schur_c((schur_t *)ctx, in, out); }
static void op_cdag(void *ctx, const cplx *in, cplx *out) { schur_cdag((schur_t *)ctx, in, out); }

/*
 * Solve D x = b through the factorisation of Eq. (10):
 *   b'  = S1 b = M5 sqrt(omega)^-1 b                      (both parities)
 *   b'' = b'_o - M5 D^OE b'_e                             (odd)
 *   C y_o = b''   by CG on C C^dag                        (odd)
 *   y_e = b'_e - M5 D^EO y_o                              (even)
 *   x   = S2 y = Y^-1 sqrt(omega) y.
 * x is the initial guess on entry only through its odd Schur part
 * y_o = (S2^-1 x)_o; pass zeros for a cold start.
 * Returns 0 if converged, 1 if maxiter was reached, -1 on a singular
 * fifth-dimension matrix.
 */
int orc_solve(const double *U, const int *dims, int Ns, double m0, double mq,
              const double *sigma, const double *omega, double bct,
              const double *b, double *x, double tol, int maxiter,
              int *iters, double *schur_res)
{
    schur_t S;
    if (schur_init(&S, U, dims, Ns, m0, mq, sigma, omega, bct)) { schur_free(&S); return -1; }
    long N = S.N, V = S.l.V;
    int n2 = Ns * Ns;
    const cplx *bb = (const cplx *)b;
    cplx *xx = (cplx *)x;
    cplx *bp = malloc(sizeof(cplx) * N), *bpp = malloc(sizeof(cplx) * N);
    cplx *y = malloc(sizeof(cplx) * N), *w = malloc(sizeof(cplx) * N);
    double *Xp = malloc(sizeof(double) * n2), *Xm = malloc(sizeof(double) * n2);
    double *Yp = malloc(sizeof(double) * n2), *Ym = malloc(sizeof(double) * n2);
    double *Yip = malloc(sizeof(double) * n2), *Yim = malloc(sizeof(double) * n2);
    double *S2p = malloc(sizeof(double) * n2), *S2m = malloc(sizeof(double) * n2);
    double *S2ip = malloc(sizeof(double) * n2), *S2im = malloc(sizeof(double) * n2);
    orc_xy(Ns, m0, mq, sigma, omega, Xp, Xm, Yp, Ym);
    int rc = 0;
    if (gj_inverse(Ns, Yp, Yip) || gj_inverse(Ns, Ym, Yim)) { rc = -1; goto done; }
    for (int s = 0; s < Ns; s++)
        for (int t = 0; t < Ns; t++) {
            S2p[s * Ns + t] = Yip[s * Ns + t] * sqrt(omega[t]);
            S2m[s * Ns + t] = Yim[s * Ns + t] * sqrt(omega[t]);
            /* S2^-1 = sqrt(omega)^-1 Y */
            S2ip[s * Ns + t] = Yp[s * Ns + t] / sqrt(omega[s]);
            S2im[s * Ns + t] = Ym[s * Ns + t] / sqrt(omega[s]);
        }
    /* b' = M5 sqrt(omega)^-1 b */
    for (long n = 0; n < V; n++)
        for (int s = 0; s < Ns; s++)
            for (int k = 0; k < 12; k++) w[(n * Ns + s) * 12 + k] = bb[(n * Ns + s) * 12 + k] / sqrt(omega[s]);
    apply_s(&S.l, Ns, S.M5p, S.M5m, w, bp);
    /* b'' = b'_o - M5 D^OE b'_e  (hop to odd reads only even sites of b') */
    hop_apply(&S.l, Ns, S.U, bct, 1, bp, S.t1);
    apply_s(&S.l, Ns, S.M5p, S.M5m, S.t1, S.t2);
    for (long n = 0; n < V; n++) {
        int c[4];
        coords(&S.l, n, c);
        int odd = parity(c);
        for (long k = n * Ns * 12; k < (n + 1) * Ns * 12; k++) bpp[k] = odd ? bp[k] - S.t2[k] : 0;
    }
    /* initial guess: y_o = (S2^-1 x)_o */
    apply_s(&S.l, Ns, S2ip, S2im, xx, y);
    for (long n = 0; n < V; n++) {
        int c[4];
        coords(&S.l, n, c);
        if (!parity(c))
            for (long k = n * Ns * 12; k < (n + 1) * Ns * 12; k++) y[k] = 0;
    }
    rc = cgne(op_c, op_cdag, &S, N, bpp, y, tol, maxiter, iters, schur_res);
    /* y_e = b'_e - M5 D^EO y_o */
    hop_apply(&S.l, Ns, S.U, bct, 0, y, S.t1);
    apply_s(&S.l, Ns, S.M5p, S.M5m, S.t1, S.t2);
    for (long n = 0; n < V; n++) {
        int c[4];
        coords(&S.l, n, c);
        if (!parity(c))
            for (long k = n * Ns * 12; k < (n + 1) * Ns * 12; k++) y[k] = bp[k] - S.t2[k];
    }
    /* x = S2 y */
    apply_s(&S.l, Ns, S2p, S2m, y, xx);
done:
    free(bp); free(bpp); free(y); free(w); free(Xp); free(Xm); free(Yp); free(Ym);
    free(Yip); free(Yim); free(S2p); free(S2m); free(S2ip); free(S2im);
    schur_free(&S);
    return rc;
}

/*
 * The solve the hybrid Monte Carlo force needs: C C^dag w = b on the odd sites
 * (the paper's use of CG on C C^dag, Sec. 2.1), by Algorithm 1 as printed with
 * A = C C^dag applied as C (C^dag p):
 *   r = b - A w;  p = r;  alpha = |r|^2 / (p, A p);  w += alpha p;
 *   r -= alpha A p;  beta = |r_new|^2 / |r|^2;  p = r + beta p,
 * stopping when |r| <= tol |b|.  The even sites of b are ignored and the even
 * sites of w are zero.  w holds the initial guess on entry.
 * Returns 0 if converged, 1 if maxiter was reached, -1 on a singular
 * fifth-dimension matrix.
 */
int orc_solve_ccdag(const double *U, const int *dims, int Ns, double m0, double mq,
                    const double *sigma, const double *omega, double bct,
                    const double *b, double *w, double tol, int maxiter,
                    int *iters, double *relres)
{
    schur_t S;
    if (schur_init(&S, U, dims, Ns, m0, mq, sigma, omega, bct)) { schur_free(&S); return -1; }
    long N = S.N, V = S.l.V;
    cplx *bo = malloc(sizeof(cplx) * N), *r = malloc(sizeof(cplx) * N), *p = malloc(sizeof(cplx) * N);
    cplx *t = malloc(sizeof(cplx) * N), *ap = malloc(sizeof(cplx) * N);
    cplx *ww = (cplx *)w;
    const cplx *bb = (const cplx *)b;
    for (long n = 0; n < V; n++) {
        int c[4];
        coords(&S.l, n, c);
        int odd = parity(c);
        for (long k = n * Ns * 12; k < (n + 1) * Ns * 12; k++) {
            bo[k] = odd ? bb[k] : 0;
            if (!odd) ww[k] = 0;
        }
    }
    /* r = b - C C^dag w */
    schur_cdag(&S, ww, t);
    schur_c(&S, t, ap);
    for (long i = 0; i < N; i++) { r[i] = bo[i] - ap[i]; p[i] = r[i]; }
    double bn = norm2(N, bo), rr = norm2(N, r);
    int k = 0;
    while (rr > tol * tol * bn && k < maxiter) {
        schur_cdag(&S, p, t);
        schur_c(&S, t, ap);
        double pap = 0;
        for (long i = 0; i < N; i++) pap += creal(conj(p[i]) * ap[i]);
        if (!(pap > 0)) break;
        double alpha = rr / pap;
        for (long i = 0; i < N; i++) { ww[i] += alpha * p[i]; r[i] -= alpha * ap[i]; }
        double rr_new = norm2(N, r);
        double beta = rr_new / rr;
        for (long i = 0; i < N; i++) p[i] = r[i] + beta * p[i];
        rr = rr_new;
        k++;
    }
    *iters = k;
    *relres = bn > 0 ? sqrt(rr / bn) : 0;
    free(bo); free(r); free(p); free(t); free(ap);
    schur_free(&S);
    return (rr <= tol * tol * bn) ? 0 : 1;
}

/* CG on the normal equations of the unpreconditioned 5D operator (no even-odd
 * split), D D^dag w = b, x = D^dag w.  Used to cross-check the Schur route. */
typedef struct {
    const double *U; const int *dims; int Ns; double m0, mq; const double *sigma, *omega; double bct;
} full_t;

static void op_d(void *ctx, const cplx *in, cplx *out)
{
    full_t *f = ctx;
    orc_d5(f->U, f->dims, f->Ns, f->m0, f->mq, f->sigma, f->omega, f->bct, (const double *)in, (double *)out);
}

static void op_ddag(void *ctx, const cplx *in, cplx *out)
{
    full_t *f = ctx;
    orc_d5dag(f->U, f->dims, f->Ns, f->m0, f->mq, f->sigma, f->omega, f->bct, (const double *)in, (double *)out);
}

int orc_cgne_full(const double *U, const int *dims, int Ns, double m0, double mq,
                  const double *sigma, const double *omega, double bct,
                  const double *b, double *x, double tol, int maxiter, int *iters, double *relres)
{
    full_t f = {U, dims, Ns, m0, mq, sigma, omega, bct};
    lat_t l = lat_make(dims);
    return cgne(op_d, op_ddag, &f, l.V * Ns * 12, (const cplx *)b, (cplx *)x, tol, maxiter, iters, relres);
}

/* Relative residual |b - D x| / |b| with the full 5D operator. */
double orc_true_residual(const double *U, const int *dims, int Ns, double m0, double mq,
                         const double *sigma, const double *omega, double bct,
                         const double *b, const double *x)
{
    lat_t l = lat_make(dims);
    long N = l.V * Ns * 12;
    cplx *dx = malloc(sizeof(cplx) * N);
    orc_d5(U, dims, Ns, m0, mq, sigma, omega, bct, x, (double *)dx);
    const cplx *bb = (const cplx *)b;
    for (long i = 0; i < N; i++) dx[i] = bb[i] - dx[i];
    double r = norm2(N, dx), n = norm2(N, bb);
    free(dx);
    return n > 0 ? sqrt(r / n) : sqrt(r);
}

/* ------------------------------------------------------------------------ */
/* 4D valence-quark propagator from the 5D solve (Sec. 2.2: CG on the 5D      */
/* system also gives the valence quark propagators; Sec. 5).  The paper does  */
/* not spell out the 4D fields, so this follows from Eqs. (3)-(5):            */
/*  - the quark mass enters only through the corner of L (Eq. (4)), and that  */
/*    corner couples P_+ psi at s = Ns to s = 1 and P_- psi at s = 1 to        */
/*    s = Ns.  Hence D(mq) = D(0) + kappa W R, kappa = mq / (2 m0), with      */
/*      R psi = P_+ psi_Ns + P_- psi_1                    (5D -> 4D)          */
/*      (W q)_1 = (1 - sigma_1 D_w) P_+ q,                                    */
/*      (W q)_Ns = (1 - sigma_Ns D_w) P_- q, zero on the other slices.        */
/*  - the 4D quark field is q = R psi (the walls, where the chiral modes of    */
/*    the free operator sit for 0 < m0 < 2) and the source of a 4D spinor     */
/*    eta is the 5D vector W eta, so that                                     */
/*      S(mq) eta = R D(mq)^-1 W eta,                                         */
/*    which makes the quark mass additive: S(mq)^-1 = S(0)^-1 + kappa.        */
/* eta, out: 4D spinors [Lt][Lz][Ly][Lx][24].  The 5D solve is orc_solve's    */
/* (Eq. (10) with CG on C C^dag) to tol.  Returns orc_solve's code.           */
/* ------------------------------------------------------------------------ */

int orc_propagator(const double *U, const int *dims, int Ns, double m0, double mq,
                   const double *sigma, const double *omega, double bct,
                   const double *eta, double *out, double tol, int maxiter,
                   int *iters, double *schur_res)
{
    gamma_init();
    lat_t l = lat_make(dims);
    long N = l.V * Ns * 12;
    const cplx *e = (const cplx *)eta;
    cplx *q = (cplx *)out;
    cplx *c = calloc(N, sizeof(cplx)), *dc = malloc(sizeof(cplx) * N);
    cplx *b = malloc(sizeof(cplx) * N), *x = calloc(N, sizeof(cplx));
    cplx Pp[4][4], Pm[4][4];
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            Pp[i][j] = 0.5 * ((i == j) + G[4][i][j]);
            Pm[i][j] = 0.5 * ((i == j) - G[4][i][j]);
        }
    /* c: P_+ eta on slice 1, P_- eta on slice Ns (0-based 0 and Ns - 1) */
    for (long n = 0; n < l.V; n++)
        for (int i = 0; i < 4; i++)
            for (int a = 0; a < 3; a++) {
                cplx ap = 0, am = 0;
                for (int j = 0; j < 4; j++) {
                    ap += Pp[i][j] * e[n * 12 + 3 * j + a];
                    am += Pm[i][j] * e[n * 12 + 3 * j + a];
                }
                c[(n * Ns + 0) * 12 + 3 * i + a] += ap;
                c[(n * Ns + Ns - 1) * 12 + 3 * i + a] += am;
            }
    /* b = W eta = c - sigma_s D_w c (slice by slice) */
    orc_dw(U, dims, Ns, m0, bct, (const double *)c, (double *)dc);
    for (long n = 0; n < l.V; n++)
        for (int s = 0; s < Ns; s++)
            for (int k = 0; k < 12; k++) {
                long i = (n * Ns + s) * 12 + k;
                b[i] = c[i] - sigma[s] * dc[i];
            }
    int rc = orc_solve(U, dims, Ns, m0, mq, sigma, omega, bct, (const double *)b, (double *)x, tol, maxiter,
                       iters, schur_res);
    /* q = R x = P_+ x_Ns + P_- x_1 */
    for (long n = 0; n < l.V; n++)
        for (int i = 0; i < 4; i++)
            for (int a = 0; a < 3; a++) {
                cplx acc = 0;
                for (int j = 0; j < 4; j++)
                    acc += Pp[i][j] * x[(n * Ns + Ns - 1) * 12 + 3 * j + a] + Pm[i][j] * x[(n * Ns + 0) * 12 + 3 * j + a];
                q[n * 12 + 3 * i + a] = acc;
            }
    free(c); free(dc); free(b); free(x);
    return rc;
}
