/*
 * oracle.c -- plain FP64 CPU oracle for feedforward decentralized precoding
 * (K. Li, C. Jeon, J. R. Cavallaro, C. Studer, "Feedforward Architectures for
 * Decentralized Precoding in Massive MU-MIMO Systems", arXiv:1804.10987).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the HIP library.
 *
 * Everything is textbook scalar complex<double> loops in the order the paper
 * states the method; no blocking, no fusion, no BLAS.
 *
 * Convention.  The paper writes the downlink channel of one subcarrier as a
 * U x B matrix (Sec. II-A, downlink model).  This oracle stores its Hermitian
 * transpose H (B x U: antenna rows, user columns), so the paper's cluster
 * column blocks become row blocks H_c (B_c x U), the paper's local Gram
 * H_c H_c^H becomes H_c^H H_c (U x U) and the per-cluster product H_c^H z
 * becomes H_c z.
 *
 * Memory layout (complex values stored as interleaved re,im doubles):
 *   H     [n_sc][B][U]
 *   s     [K][n_sc][U]
 *   x     [K][n_sc][B]
 *   beta  [n_sc]          (PD)
 *   wgt   [n_sc][C]       (FD)
 *   status: 0 = ok, 1 = numerical failure (x, beta / weights set to zero).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

static cplx ld(const double *p) { return p[0] + p[1] * I; }
static void st(double *p, cplx v) { p[0] = creal(v); p[1] = cimag(v); }

/* In-place Cholesky A = L L^H of an n x n Hermitian matrix (row-major,
 * lower triangle used).  The paper inverts the regularized Gram matrix with a
 * batched factorization (Sec. IV-B, PD-WF implementation); A is Hermitian
 * positive definite, so Cholesky is the factorization that applies.
 * Theorem 1 needs A invertible: a pivot that is not above 2^-40 times the
 * original diagonal entry (FP64 roundoff level) marks A numerically singular.
 * Returns 0 on success, 1 on such a pivot or a non-finite value. */
static int cholesky(cplx *A, int n) {
    for (int j = 0; j < n; ++j) {
        const double a0 = creal(A[j * n + j]);
        double d = a0;
        for (int k = 0; k < j; ++k) {
            cplx l = A[j * n + k];
            d -= creal(l * conj(l));
        }
        if (!(d > 0x1p-40 * a0) || !isfinite(d)) return 1;
        d = sqrt(d);
        A[j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            cplx acc = A[i * n + j];
            for (int k = 0; k < j; ++k) acc -= A[i * n + k] * conj(A[j * n + k]);
            A[i * n + j] = acc / d;
        }
        for (int i = 0; i < j; ++i) A[i * n + j] = 0.0;
    }
    return 0;
}

/* Explicit inverse of a Hermitian positive-definite matrix through its
 * Cholesky factor: solve L Y = I by forward substitution, then
 * L^H X = Y by back substitution, one column of the identity at a time. */
static int hpd_inverse(const cplx *A, int n, cplx *Ainv) {
    cplx *L = malloc(sizeof(cplx) * n * n);
    cplx *y = malloc(sizeof(cplx) * n);
    memcpy(L, A, sizeof(cplx) * n * n);
    int bad = cholesky(L, n);
    for (int col = 0; col < n && !bad; ++col) {
        for (int i = 0; i < n; ++i) {
            cplx acc = (i == col) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) acc -= L[i * n + k] * y[k];
            y[i] = acc / L[i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            cplx acc = y[i];
            for (int k = i + 1; k < n; ++k) acc -= conj(L[k * n + i]) * Ainv[k * n + col];
            Ainv[i * n + col] = acc / creal(L[i * n + i]);
        }
    }
    for (int i = 0; i < n * n && !bad; ++i)
        if (!isfinite(creal(Ainv[i])) || !isfinite(cimag(Ainv[i]))) bad = 1;
    free(L);
    free(y);
    return bad;
}

/* ---------------------------------------------------------------------------
 * Partially decentralized WF / ZF precoding (Sec. III-B).
 *
 *   G_c = H_c^H H_c for every cluster           (local Gram, Sec. III-B)
 *   G   = sum_c G_c                             (feedforward adder tree)
 *   A   = G + kappa I_U                         (regularized Gram, App. B)
 *   beta = sqrt(Es/rho^2 (tr A^-1 - kappa ||A^-1||_F^2))    (Lemma 1)
 *   z   = A^-1 s / beta                         (whitening node)
 *   x_c = H_c z                                 (per-cluster precoding)
 *
 * kappa is the WF regularizer U N0 / rho^2 of Theorem 1; ZF is kappa = 0.
 * power = rho^2 (power budget, Sec. II-A), Es = symbol energy.
 * G_out / Ainv_out (optional, [n_sc][U][U] complex) expose intermediates.
 * ------------------------------------------------------------------------- */
int oracle_pd(const double *H, const double *s, int B, int U, int n_sc, int K,
              const int *sizes, int C, double kappa, int zf, double power,
              double Es, int threads, double *x, double *beta, int *status,
              double *G_out, double *Ainv_out) {
    if (zf) kappa = 0.0;
    int bad_args = 0;
    {
        int sum = 0;
        for (int c = 0; c < C; ++c) sum += sizes[c];
        if (sum != B) bad_args = 1;
    }
    if (bad_args) return -1;
#pragma omp parallel for schedule(dynamic) num_threads(threads)
    for (int n = 0; n < n_sc; ++n) {
        const double *Hn = H + (size_t)n * B * U * 2;
        cplx *G = calloc((size_t)U * U, sizeof(cplx));
        cplx *A = malloc(sizeof(cplx) * U * U);
        cplx *Ai = malloc(sizeof(cplx) * U * U);
        cplx *z = malloc(sizeof(cplx) * U);
        /* local Gram matrices, summed cluster by cluster */
        int row0 = 0;
        for (int c = 0; c < C; ++c) {
            for (int u = 0; u < U; ++u)
                for (int v = 0; v < U; ++v) {
                    cplx g = 0.0;
                    for (int b = row0; b < row0 + sizes[c]; ++b)
                        g += conj(ld(Hn + ((size_t)b * U + u) * 2)) * ld(Hn + ((size_t)b * U + v) * 2);
                    G[u * U + v] += g;
                }
            row0 += sizes[c];
        }
        for (int i = 0; i < U * U; ++i) A[i] = G[i];
        for (int u = 0; u < U; ++u) A[u * U + u] += kappa;
        int bad = hpd_inverse(A, U, Ai);
        double t = 0.0;
        if (!bad) {
            double tr = 0.0, fro = 0.0;
            for (int u = 0; u < U; ++u) tr += creal(Ai[u * U + u]);
            for (int i = 0; i < U * U; ++i) fro += creal(Ai[i] * conj(Ai[i]));
            t = tr - kappa * fro;
            if (!(t > 0.0) || !isfinite(t)) bad = 1;
        }
        double b_wf = bad ? 0.0 : sqrt(Es / power * t);
        beta[n] = b_wf;
        if (status) status[n] = bad;
        for (int k = 0; k < K; ++k) {
            const double *sk = s + ((size_t)k * n_sc + n) * U * 2;
            double *xk = x + ((size_t)k * n_sc + n) * B * 2;
            if (bad) {
                memset(xk, 0, sizeof(double) * 2 * B);
                continue;
            }
            for (int u = 0; u < U; ++u) {
                cplx acc = 0.0;
                for (int v = 0; v < U; ++v) acc += Ai[u * U + v] * ld(sk + v * 2);
                z[u] = acc / b_wf;
            }
            for (int b = 0; b < B; ++b) {
                cplx acc = 0.0;
                for (int u = 0; u < U; ++u) acc += ld(Hn + ((size_t)b * U + u) * 2) * z[u];
                st(xk + b * 2, acc);
            }
        }
        if (G_out)
            for (int i = 0; i < U * U; ++i) st(G_out + ((size_t)n * U * U + i) * 2, G[i]);
        if (Ainv_out)
            for (int i = 0; i < U * U; ++i) st(Ainv_out + ((size_t)n * U * U + i) * 2, bad ? 0.0 : Ai[i]);
        free(G);
        free(A);
        free(Ai);
        free(z);
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Fully decentralized WF / ZF precoding (Sec. III-C).
 *
 * Every cluster gets the power rho_c^2 = rho^2 / C and the regularizer
 * kappa_c = tau_c U N0 / rho_c^2 = tau_c C kappa (eq. regularization), and
 * forms its own precoding matrix Q_c (B_c x U in this file's convention):
 *
 *   B_c <  U :  Q_c = (H_c H_c^H + kappa_c I_{B_c})^-1 H_c
 *   B_c >= U :  Q_c = H_c (H_c^H H_c + kappa_c I_U)^-1
 *
 *   x_c = sqrt(rho_c^2 / (tr(Q_c^H Q_c) Es)) Q_c s
 *
 * The weight sqrt(rho_c^2 / (tr(Q_c^H Q_c) Es)) is returned in wgt.
 *
 * Variants of Sec. III-C: tau_c (optional, [C]) gives every cluster its own
 * tau_c of eq. regularization; power_c (optional, [C]) replaces the equal
 * split by per-cluster budgets rho_c^2 with sum_c rho_c^2 = rho^2 (the
 * allocation strategies the power footnote of Sec. III-C mentions); then
 * kappa_c = tau_c U N0 / rho_c^2 = tau_c kappa rho^2 / rho_c^2.
 * ------------------------------------------------------------------------- */
int oracle_fd(const double *H, const double *s, int B, int U, int n_sc, int K,
              const int *sizes, int C, double kappa, int zf, double tau,
              double power, double Es, int threads, double *x, double *wgt,
              int *status, const double *tau_c, const double *power_c) {
    int sum = 0;
    for (int c = 0; c < C; ++c) sum += sizes[c];
    if (sum != B) return -1;
#pragma omp parallel for schedule(dynamic) num_threads(threads)
    for (int n = 0; n < n_sc; ++n) {
        const double *Hn = H + (size_t)n * B * U * 2;
        int row0 = 0;
        for (int c = 0; c < C; ++c) {
            /* rho_c^2 (equal split unless given) and kappa_c = tau_c U N0 /
             * rho_c^2 = tau_c kappa rho^2 / rho_c^2 (eq. regularization) */
            const double rho_c2 = power_c ? power_c[c] : power / C;
            const double kappa_c = zf ? 0.0 : (tau_c ? tau_c[c] : tau) * kappa * power / rho_c2;
            const int Bc = sizes[c];
            const double *Hc = Hn + (size_t)row0 * U * 2;
            const int m = (Bc < U) ? Bc : U; /* order of the local system */
            cplx *A = malloc(sizeof(cplx) * m * m);
            cplx *Ai = malloc(sizeof(cplx) * m * m);
            cplx *Q = calloc((size_t)Bc * U, sizeof(cplx));
            if (Bc >= U) {
                for (int u = 0; u < U; ++u)
                    for (int v = 0; v < U; ++v) {
                        cplx g = 0.0;
                        for (int b = 0; b < Bc; ++b)
                            g += conj(ld(Hc + ((size_t)b * U + u) * 2)) * ld(Hc + ((size_t)b * U + v) * 2);
                        A[u * U + v] = g + ((u == v) ? kappa_c : 0.0);
                    }
            } else {
                for (int a = 0; a < Bc; ++a)
                    for (int b = 0; b < Bc; ++b) {
                        cplx g = 0.0;
                        for (int u = 0; u < U; ++u)
                            g += ld(Hc + ((size_t)a * U + u) * 2) * conj(ld(Hc + ((size_t)b * U + u) * 2));
                        A[a * Bc + b] = g + ((a == b) ? kappa_c : 0.0);
                    }
            }
            int bad = hpd_inverse(A, m, Ai);
            if (!bad) {
                if (Bc >= U) {
                    for (int b = 0; b < Bc; ++b)
                        for (int v = 0; v < U; ++v) {
                            cplx acc = 0.0;
                            for (int u = 0; u < U; ++u) acc += ld(Hc + ((size_t)b * U + u) * 2) * Ai[u * U + v];
                            Q[b * U + v] = acc;
                        }
                } else {
                    for (int a = 0; a < Bc; ++a)
                        for (int v = 0; v < U; ++v) {
                            cplx acc = 0.0;
                            for (int b = 0; b < Bc; ++b) acc += Ai[a * Bc + b] * ld(Hc + ((size_t)b * U + v) * 2);
                            Q[a * U + v] = acc;
                        }
                }
            }
            double t = 0.0;
            for (int i = 0; i < Bc * U && !bad; ++i) t += creal(Q[i] * conj(Q[i]));
            if (!bad && (!(t > 0.0) || !isfinite(t))) bad = 1;
            double w = bad ? 0.0 : sqrt(rho_c2 / (t * Es));
            wgt[(size_t)n * C + c] = w;
            if (status) status[(size_t)n * C + c] = bad;
            for (int k = 0; k < K; ++k) {
                const double *sk = s + ((size_t)k * n_sc + n) * U * 2;
                double *xk = x + (((size_t)k * n_sc + n) * B + row0) * 2;
                for (int b = 0; b < Bc; ++b) {
                    cplx acc = 0.0;
                    if (!bad)
                        for (int u = 0; u < U; ++u) acc += Q[b * U + u] * ld(sk + u * 2);
                    st(xk + b * 2, w * acc);
                }
            }
            free(A);
            free(Ai);
            free(Q);
            row0 += Bc;
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Centralized WF precoding in the B x B form of Theorem 1 (Sec. II-B).
 *
 * In the paper's U x B downlink channel H_dl, Q = (H_dl^H H_dl + kappa I_B)^-1
 * H_dl^H (eq. originalQmatrix); with this file's H = H_dl^H (B x U):
 *
 *   M    = H H^H + kappa I_B                    (B x B, Hermitian PD for kappa > 0)
 *   Q    = M^-1 H                               (B x U; Cholesky of M, one
 *                                                forward and one back substitution
 *                                                per user column)
 *   beta = sqrt(tr(Q^H Q) Es / rho^2)           (eq. precodingfactor)
 *   x    = Q s / beta
 *
 * This is the form Lemma 1 avoids; it serves as the reference the PD
 * architecture must equal.  kappa must be positive (for B > U the matrix
 * H H^H is singular, so ZF has no B x B form).  Returns -2 for kappa <= 0.
 * ------------------------------------------------------------------------- */
int oracle_central(const double *H, const double *s, int B, int U, int n_sc, int K,
                   double kappa, double power, double Es, int threads, double *x,
                   double *beta, int *status) {
    if (!(kappa > 0.0)) return -2;
#pragma omp parallel for schedule(dynamic) num_threads(threads)
    for (int n = 0; n < n_sc; ++n) {
        const double *Hn = H + (size_t)n * B * U * 2;
        cplx *M = malloc(sizeof(cplx) * B * B);
        cplx *Q = malloc(sizeof(cplx) * B * U);
        cplx *y = malloc(sizeof(cplx) * B);
        for (int a = 0; a < B; ++a)
            for (int b = 0; b < B; ++b) {
                cplx g = 0.0;
                for (int u = 0; u < U; ++u)
                    g += ld(Hn + ((size_t)a * U + u) * 2) * conj(ld(Hn + ((size_t)b * U + u) * 2));
                M[a * B + b] = g + ((a == b) ? kappa : 0.0);
            }
        int bad = cholesky(M, B);
        double t = 0.0;
        for (int u = 0; u < U && !bad; ++u) {
            for (int i = 0; i < B; ++i) {
                cplx acc = ld(Hn + ((size_t)i * U + u) * 2);
                for (int k = 0; k < i; ++k) acc -= M[i * B + k] * y[k];
                y[i] = acc / M[i * B + i];
            }
            for (int i = B - 1; i >= 0; --i) {
                cplx acc = y[i];
                for (int k = i + 1; k < B; ++k) acc -= conj(M[k * B + i]) * Q[k * U + u];
                Q[i * U + u] = acc / creal(M[i * B + i]);
            }
            for (int i = 0; i < B; ++i) t += creal(Q[i * U + u] * conj(Q[i * U + u]));
        }
        if (!bad && (!(t > 0.0) || !isfinite(t))) bad = 1;
        const double b_wf = bad ? 0.0 : sqrt(t * Es / power);
        beta[n] = b_wf;
        if (status) status[n] = bad;
        for (int k = 0; k < K; ++k) {
            const double *sk = s + ((size_t)k * n_sc + n) * U * 2;
            double *xk = x + ((size_t)k * n_sc + n) * B * 2;
            for (int b = 0; b < B; ++b) {
                cplx acc = 0.0;
                if (!bad)
                    for (int u = 0; u < U; ++u) acc += Q[b * U + u] * ld(sk + u * 2);
                st(xk + b * 2, bad ? 0.0 : acc / b_wf);
            }
        }
        free(M);
        free(Q);
        free(y);
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Maximum ratio transmission (MRT; named as the fully distributed comparison
 * precoder in Sec. I and Sec. III-D).  The matched filter Q_c = H_c (this
 * file's convention; the paper's H_dl,c^H) with the per-cluster power
 * normalization of Sec. III-C:
 *
 *   x_c = sqrt(rho_c^2 / (||H_c||_F^2 Es)) H_c s,   rho_c^2 = rho^2 / C
 *
 * (power_c, optional [C], gives per-cluster budgets instead).  C = 1 is
 * centralized MRT, whose factor is the beta of eq. precodingfactor with
 * Q = H.  The weight is returned in wgt [n_sc][C]; a cluster with a zero
 * channel has status 1 and weight 0.
 * ------------------------------------------------------------------------- */
int oracle_mrt(const double *H, const double *s, int B, int U, int n_sc, int K,
               const int *sizes, int C, double power, double Es, int threads,
               double *x, double *wgt, int *status, const double *power_c) {
    int sum = 0;
    for (int c = 0; c < C; ++c) sum += sizes[c];
    if (sum != B) return -1;
#pragma omp parallel for schedule(dynamic) num_threads(threads)
    for (int n = 0; n < n_sc; ++n) {
        const double *Hn = H + (size_t)n * B * U * 2;
        int row0 = 0;
        for (int c = 0; c < C; ++c) {
            const int Bc = sizes[c];
            const double rho_c2 = power_c ? power_c[c] : power / C;
            double f = 0.0;
            for (int b = row0; b < row0 + Bc; ++b)
                for (int u = 0; u < U; ++u) {
                    cplx h = ld(Hn + ((size_t)b * U + u) * 2);
                    f += creal(h * conj(h));
                }
            const int bad = !(f > 0.0) || !isfinite(f);
            const double w = bad ? 0.0 : sqrt(rho_c2 / (f * Es));
            wgt[(size_t)n * C + c] = w;
            if (status) status[(size_t)n * C + c] = bad;
            for (int k = 0; k < K; ++k) {
                const double *sk = s + ((size_t)k * n_sc + n) * U * 2;
                double *xk = x + ((size_t)k * n_sc + n) * B * 2;
                for (int b = row0; b < row0 + Bc; ++b) {
                    cplx acc = 0.0;
                    for (int u = 0; u < U; ++u) acc += ld(Hn + ((size_t)b * U + u) * 2) * ld(sk + u * 2);
                    st(xk + b * 2, w * acc);
                }
            }
            row0 += Bc;
        }
    }
    return 0;
}
