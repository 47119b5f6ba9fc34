// fifth_dim.h -- host construction of the fifth-dimension operators of
// Eqs. (3)-(4) and (7)-(9): dense per-chirality Ns x Ns tables, and the
// O(Ns) recurrence coefficients with which the stencil kernels apply M5 and
// M5^T without forming them.
//
// Per chirality, L is a cyclic shift with a corner: L_+ w_s = w_{s-1}
// (s >= 1), L_+ w_0 = -kappa w_{Ns-1}, kappa = mq / (2 m0), and L_- = L_+^T is
// the same shift with s reversed.  X = a + b L and Y = omega + sigma L are
// therefore cyclic bidiagonal, with a = (d - m0) omega + 1 and
// b = (d - m0) sigma - 1 (Eq. (7) expanded), and
//     M5   = sqrt(w)^-1 Y X^-1 sqrt(w)          ("solve, then apply")
//     M5^T = sqrt(w)   X^-T Y^T sqrt(w)^-1      ("apply, then solve")
// Written in the order in which the shift is "forward" (s reversed where it is
// not), every solve is one sweep of w_s = alpha_s + beta_s w_0 followed by
// the corner equation for w_0.
#pragma once

#include <cmath>
#include <string>
#include <vector>

namespace dwf {

// Dense tables: [2 chiralities][Ns][Ns] each.
enum Table {
    TB_M5 = 0,    // M5 of Eq. (8)
    TB_M5T,       // M5^T
    TB_M5TG5,     // M5^T gamma_5 (gamma_5 folded into the chirality blocks)
    TB_S1,        // S1 = M5 sqrt(omega)^-1, Eq. (9)
    TB_S2,        // S2 = Y^-1 sqrt(omega), Eq. (9)
    TB_S2INV,     // S2^-1 = sqrt(omega)^-1 Y
    TB_X,         // X of Eq. (7)
    TB_Y,         // Y of Eq. (7)
    TB_YTG5,      // Y^T gamma_5
    TB_1MLT,      // (1 - L)^T
    TB_G5,        // gamma_5
    TB_COUNT
};

// Recurrence forms: [2 chiralities][6 arrays][Ns] each, arrays F, G, B, P, Q, O
// in recurrence order (see the kernel's mix_structured()).
enum StructTable { ST_M5 = 0, ST_M5T, ST_M5TG5, ST_COUNT };
constexpr int ST_ARRAYS = 6;

inline size_t dense_table_size(int N) { return (size_t)TB_COUNT * 2 * N * N; }
inline size_t dense_table_offset(int N, int t) { return (size_t)t * 2 * N * N; }
inline size_t struct_table_offset(int N, int st) {
    return dense_table_size(N) + (size_t)st * 2 * ST_ARRAYS * N;
}
inline size_t tables_size(int N) { return dense_table_size(N) + (size_t)ST_COUNT * 2 * ST_ARRAYS * N; }

// Solve (diag(a) + diag(b) L) w = z with L = L_+ (ch = 0) or L_- (ch = 1).
// Every w_s is affine in w_0; the corner equation fixes w_0.  false if singular.
inline bool cyc_solve(int N, const double* a, const double* b, double kappa, int ch, const double* z, double* w) {
    std::vector<double> A(N), B(N), Z(N), al(N), be(N);
    for (int s = 0; s < N; ++s) {
        int k = ch ? N - 1 - s : s;  // L_- is L_+ with s reversed
        A[s] = a[k];
        B[s] = b[k];
        Z[s] = z[k];
    }
    al[0] = 0;
    be[0] = 1;
    for (int s = 1; s < N; ++s) {
        if (A[s] == 0) return false;
        al[s] = (Z[s] - B[s] * al[s - 1]) / A[s];
        be[s] = -B[s] * be[s - 1] / A[s];
    }
    double den = A[0] - kappa * B[0] * be[N - 1];
    double scale = std::fabs(A[0]) + std::fabs(kappa * B[0] * be[N - 1]);
    if (!(std::fabs(den) > 1e-13 * scale)) return false;
    double w0 = (Z[0] + kappa * B[0] * al[N - 1]) / den;
    for (int s = 0; s < N; ++s) {
        int k = ch ? N - 1 - s : s;
        w[k] = al[s] + be[s] * w0;
    }
    return true;
}

// Recurrence coefficients of one chirality block.
//   solve-then-apply (transposed = false):  out = sqrt(w)^-1 Y X^-1 sqrt(w) x
//   apply-then-solve (transposed = true):   out = sign * sqrt(w) X^-T Y^T sqrt(w)^-1 x
// rev: whether the recurrence runs with s reversed (L_- for the first form,
// L_+^T = L_- for the second).
inline bool struct_coeffs(int N, double kappa, const double* a, const double* b, const double* omega,
                          const double* sigma, bool rev, bool transposed, double sign, double* C) {
    std::vector<double> ar(N), br(N), sw(N), sg(N);
    for (int s = 0; s < N; ++s) {
        int k = rev ? N - 1 - s : s;
        ar[s] = a[k];
        br[s] = b[k];
        sw[s] = std::sqrt(omega[k]);
        sg[s] = sigma[k];
    }
    double *F = C, *G = C + N, *B = C + 2 * N, *P = C + 3 * N, *Q = C + 4 * N, *O = C + 5 * N;
    if (transposed) {
        // in recurrence order L^T diag(v) = diag(v shifted) L
        std::vector<double> bt(N), st(N);
        for (int s = 0; s < N; ++s) {
            bt[s] = br[(s + N - 1) % N];
            st[s] = sg[(s + N - 1) % N];
        }
        for (int s = 0; s < N; ++s) {
            P[s] = sw[s];
            Q[s] = s ? st[s] / sw[s - 1] : -kappa * st[0] / sw[N - 1];
        }
        std::vector<double> beta(N);
        beta[0] = 1;
        for (int s = 1; s < N; ++s) {
            if (ar[s] == 0) return false;
            F[s] = 1.0 / ar[s];
            G[s] = bt[s] / ar[s];
            beta[s] = -G[s] * beta[s - 1];
        }
        double den = ar[0] - kappa * bt[0] * beta[N - 1];
        if (!(std::fabs(den) > 1e-13 * (std::fabs(ar[0]) + std::fabs(kappa * bt[0] * beta[N - 1])))) return false;
        F[0] = 1.0 / den;
        G[0] = kappa * bt[0] / den;
        for (int s = 0; s < N; ++s) {
            O[s] = sign * sw[s];
            B[s] = sign * sw[s] * beta[s];
        }
    } else {
        std::vector<double> beta(N);
        beta[0] = 1;
        for (int s = 1; s < N; ++s) {
            if (ar[s] == 0) return false;
            F[s] = sw[s] / ar[s];
            G[s] = br[s] / ar[s];
            beta[s] = -G[s] * beta[s - 1];
        }
        double den = ar[0] - kappa * br[0] * beta[N - 1];
        if (!(std::fabs(den) > 1e-13 * (std::fabs(ar[0]) + std::fabs(kappa * br[0] * beta[N - 1])))) return false;
        F[0] = sw[0] / den;
        G[0] = kappa * br[0] / den;
        for (int s = 0; s < N; ++s) {
            B[s] = beta[s];
            P[s] = sign * sw[s];
            Q[s] = sign * (s ? sg[s] / sw[s] : -kappa * sg[0] / sw[0]);
            O[s] = 0;
        }
    }
    return true;
}

// All tables of one (Ns, m0, mq, sigma, omega); false (with a reason) if
// (1 + cL), X or Y is singular.
inline bool build_tables(int N, double m0, double mq, const double* sigma, const double* omega,
                         std::vector<double>& out, std::string& why) {
    const double kappa = mq / (2.0 * m0);
    const size_t blk = (size_t)2 * N * N;
    out.assign(tables_size(N), 0.0);
    std::vector<double> a(N), b(N), one(N, 1.0), c(N), col(N), e(N), sw(N);
    for (int s = 0; s < N; ++s) {
        c[s] = sigma[s] / omega[s];
        sw[s] = std::sqrt(omega[s]);
        a[s] = (4.0 - m0) * omega[s] + 1.0;
        b[s] = (4.0 - m0) * sigma[s] - 1.0;
    }
    for (int ch = 0; ch < 2; ++ch) {
        auto T = [&](int t, int s, int u) -> double& { return out[t * blk + (size_t)ch * N * N + (size_t)s * N + u]; };
        std::vector<double> L((size_t)N * N, 0.0);
        for (int s = 1; s < N; ++s) L[(size_t)s * N + s - 1] = 1.0;
        L[N - 1] += -kappa;
        if (ch) {
            std::vector<double> Lt((size_t)N * N);
            for (int s = 0; s < N; ++s)
                for (int u = 0; u < N; ++u) Lt[(size_t)s * N + u] = L[(size_t)u * N + s];
            L.swap(Lt);
        }
        for (int s = 0; s < N; ++s) e[s] = s == 0;
        if (!cyc_solve(N, one.data(), c.data(), kappa, ch, e.data(), col.data())) {
            why = "1 + cL is singular for these weights and mass";
            return false;
        }
        std::vector<double> Xi((size_t)N * N), Yi((size_t)N * N);
        for (int u = 0; u < N; ++u) {
            for (int s = 0; s < N; ++s) e[s] = s == u;
            if (!cyc_solve(N, a.data(), b.data(), kappa, ch, e.data(), col.data())) {
                why = "X of Eq. (7) is singular for these weights and mass";
                return false;
            }
            for (int s = 0; s < N; ++s) Xi[(size_t)s * N + u] = col[s];
            if (!cyc_solve(N, omega, sigma, kappa, ch, e.data(), col.data())) {
                why = "Y of Eq. (7) is singular for these weights and mass";
                return false;
            }
            for (int s = 0; s < N; ++s) Yi[(size_t)s * N + u] = col[s];
        }
        for (int s = 0; s < N; ++s)
            for (int u = 0; u < N; ++u) {
                double id = s == u;
                double Lsu = L[(size_t)s * N + u];
                T(TB_X, s, u) = a[s] * id + b[s] * Lsu;
                T(TB_Y, s, u) = omega[s] * id + sigma[s] * Lsu;
                T(TB_1MLT, u, s) = id - Lsu;
                T(TB_G5, s, u) = ch ? -id : id;
            }
        // M5 = sqrt(w)^-1 Y X^-1 sqrt(w)   (Eq. (8))
        for (int s = 0; s < N; ++s)
            for (int u = 0; u < N; ++u) {
                double acc = 0;
                for (int k = 0; k < N; ++k) acc += T(TB_Y, s, k) * Xi[(size_t)k * N + u];
                T(TB_M5, s, u) = acc * sw[u] / sw[s];
            }
        for (int s = 0; s < N; ++s)
            for (int u = 0; u < N; ++u) {
                const double m = T(TB_M5, s, u);
                T(TB_M5T, u, s) = m;
                T(TB_M5TG5, u, s) = ch ? -m : m;
                T(TB_S1, s, u) = m / sw[u];                      // S1 = M5 sqrt(w)^-1
                T(TB_S2, s, u) = Yi[(size_t)s * N + u] * sw[u];  // S2 = Y^-1 sqrt(w)
                T(TB_S2INV, s, u) = T(TB_Y, s, u) / sw[s];       // S2^-1 = sqrt(w)^-1 Y
                T(TB_YTG5, u, s) = ch ? -T(TB_Y, s, u) : T(TB_Y, s, u);
            }
        // recurrence forms of M5, M5^T and M5^T gamma_5
        const size_t cb = (size_t)ST_ARRAYS * N;
        bool ok = struct_coeffs(N, kappa, a.data(), b.data(), omega, sigma, ch == 1, false, 1.0,
                                &out[struct_table_offset(N, ST_M5) + ch * cb]) &&
                  struct_coeffs(N, kappa, a.data(), b.data(), omega, sigma, ch == 0, true, 1.0,
                                &out[struct_table_offset(N, ST_M5T) + ch * cb]) &&
                  struct_coeffs(N, kappa, a.data(), b.data(), omega, sigma, ch == 0, true, ch ? -1.0 : 1.0,
                                &out[struct_table_offset(N, ST_M5TG5) + ch * cb]);
        if (!ok) {
            why = "X of Eq. (7) is singular for these weights and mass";
            return false;
        }
    }
    for (double v : out)
        if (!std::isfinite(v)) {
            why = "non-finite fifth-dimension table";
            return false;
        }
    return true;
}

}  // namespace dwf
