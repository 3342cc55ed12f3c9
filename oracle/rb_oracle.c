/*
 * rb_oracle.c -- plain, slow, obviously correct FP64 CPU oracle for the online stage of the
 * velocity-only reduced-basis Navier-Stokes method.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load this library. It shares no code, header or constant with the GPU
 * library; both read the same seeded input arrays and nothing else.
 *
 * What it computes (paper notation, Sections 2.2, 2.4, 3.4, 3.5, 4.1):
 *   For each parameter mu, find the reduced velocity coefficients u in R^N with
 *       F(u) = A(mu) u + C(mu)(u, u) - f(mu) = 0,                   (velocity-only, eqn velonly)
 *   A(mu) = sum_q theta^a_q(mu) A_q,  C(mu)(v,w)_i = sum_q theta^c_q(mu) sum_jk C_q[i,j,k] v_j w_k,
 *   f(mu) = sum_q theta^f_q(mu) f_q                                  (affine forms, eqns split-*)
 *   by Newton's method, the Jacobian assembled from the third-order tensors
 *       J[i,j] = A(mu)[i,j] + sum_q theta^c_q sum_k (C_q[i,j,k] + C_q[i,k,j]) u_k
 *   (the Frechet-derivative formula of Section 3.5, written with row index = test function),
 *   each step solving the dense system J delta = -F(u) by Gaussian elimination with partial
 *   pivoting. Then the pressure is recovered a posteriori (eqns sup-vvar, blocksolve-2):
 *       B(mu) p = f_s(mu) - A_sv(mu) u - C_sv(mu)(u, u).
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - initial iterate u = 0, so the first Newton step is the Stokes solve;
 *   - stop when the update is small relative to the iterate in the H^1 seminorm
 *     (||delta||_H <= tol * ||u||_H, H = the seminorm Gram), the paper's norm (Section 6);
 *   - pivot ties go to the smallest current row index (LAPACK idamax semantics);
 *   - the theta(mu) families below.
 *
 * Status codes per request: 0 converged, 1 iteration limit, 2 zero pivot, 3 non-finite value,
 * 4 basis size out of range.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no FMA contraction, IEEE FP64).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int Nm, Q, Qc, Qf, Npm, Qb;      /* stored sizes: N_max, term counts, Np_max */
    const double *A;                 /* [Q][Nm][Nm]         A[q][i][j]    = a_q(phi_j, phi_i)     */
    const double *C;                 /* [Qc][Nm][Nm][Nm]    C[q][i][j][k] = c_q(phi_j,phi_k,phi_i) */
    const double *F;                 /* [Qf][Nm]                                                   */
    const double *H;                 /* [Nm][Nm] norm Gram, or NULL for the Euclidean norm         */
    const double *Bp;                /* [Qb][Npm][Npm]      Bp[q][i][j]   = b_q(p_j, s_i)          */
    const double *Asv;               /* [Q][Npm][Nm]                                               */
    const double *Csv;               /* [Qc][Npm][Nm][Nm]                                          */
    const double *Fs;                /* [Qf][Npm]                                                  */
} orc_set;

enum { ORC_OK = 0, ORC_MAXIT = 1, ORC_SINGULAR = 2, ORC_NONFINITE = 3, ORC_BADN = 4 };

#define ORC_MAX_Q  64                /* affine terms of a; 4n + 2 = 50 at the paper's n = 12  */
#define ORC_MAX_QC 64                /* affine terms of c                                      */

/* ---------------------------------------------------------------------------------------
 * Parameter functions theta(mu), mu = (alpha [rad], Re). The paper's own coefficients are
 * powers of the rotation angle and the viscosity (Section 5); these families keep that shape:
 * trigonometric and polynomial in alpha, with the viscous term 1/Re.
 * ------------------------------------------------------------------------------------- */
int orc_theta(int Q, int Qc, int Qf, int Qb, double alpha, double Re,
              double *ta, double *tc, double *tf, double *tb)
{
    double a = alpha;
    double ha = sin(0.5 * a);
    double la[12];
    double lc[4];
    int q;
    if (Q < 1 || Q > ORC_MAX_Q || Qc < 1 || Qc > ORC_MAX_QC || Qf < 1 || Qf > 2 || Qb < 1 ||
        Qb > 2)
        return -1;
    la[0] = 1.0 / Re;
    la[1] = cos(a);
    la[2] = sin(a);
    la[3] = a;
    la[4] = a * a;
    la[5] = a * a * a;
    la[6] = cos(2.0 * a);
    la[7] = sin(2.0 * a);
    la[8] = 2.0 * ha * ha;              /* 1 - cos(a), without cancellation */
    la[9] = a * a * a * a;
    la[10] = a * cos(a);
    la[11] = a * sin(a);
    lc[0] = 1.0;
    lc[1] = cos(a);
    lc[2] = sin(a);
    lc[3] = a;
    /* Longer expansions are those of the Piola-mapped forms (Section 5): truncated power
     * series in the angle, every viscous term carrying 1/Re, theta^a_q = a^q / Re and
     * theta^c_q = a^q (q = 0, 1, ...). */
    if (Q <= 12) {
        for (q = 0; q < Q; ++q) ta[q] = la[q];
    } else {
        double pw = 1.0 / Re;
        for (q = 0; q < Q; ++q) { ta[q] = pw; pw *= a; }
    }
    if (Qc <= 4) {
        for (q = 0; q < Qc; ++q) tc[q] = lc[q];
    } else {
        double pw = 1.0;
        for (q = 0; q < Qc; ++q) { tc[q] = pw; pw *= a; }
    }
    if (tf) {
        if (Qf == 1) tf[0] = 1.0;
        else { tf[0] = cos(a); tf[1] = sin(a); }
    }
    if (tb) {
        tb[0] = 1.0;
        if (Qb == 2) tb[1] = a;
    }
    return 0;
}

/* ---------------------------------------------------------------------------------------
 * Dense linear solve by Gaussian elimination with partial pivoting (textbook, row swaps).
 * M is n x n row-major (overwritten by its LU factors), b is overwritten by the solution.
 * piv (optional, length n) receives the pivot row chosen at each step (0-based).
 * ------------------------------------------------------------------------------------- */
int orc_gepp_solve(int n, double *M, double *b, int *piv)
{
    int i, j, k;
    for (i = 0; i < n * n; ++i) if (!isfinite(M[i])) return ORC_NONFINITE;
    for (i = 0; i < n; ++i) if (!isfinite(b[i])) return ORC_NONFINITE;
    for (k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(M[k * n + k]);
        for (i = k + 1; i < n; ++i) {
            double v = fabs(M[i * n + k]);
            if (v > best) { best = v; p = i; }
        }
        if (piv) piv[k] = p;
        if (best == 0.0) return ORC_SINGULAR;
        if (p != k) {
            for (j = 0; j < n; ++j) {
                double t = M[k * n + j]; M[k * n + j] = M[p * n + j]; M[p * n + j] = t;
            }
            { double t = b[k]; b[k] = b[p]; b[p] = t; }
        }
        for (i = k + 1; i < n; ++i) {
            double l = M[i * n + k] / M[k * n + k];
            M[i * n + k] = l;
            for (j = k + 1; j < n; ++j) M[i * n + j] -= l * M[k * n + j];
            b[i] -= l * b[k];
        }
    }
    for (k = n - 1; k >= 0; --k) {
        double s = b[k];
        for (j = k + 1; j < n; ++j) s -= M[k * n + j] * b[j];
        b[k] = s / M[k * n + k];
    }
    for (i = 0; i < n; ++i) if (!isfinite(b[i])) return ORC_NONFINITE;
    return ORC_OK;
}

/* Element accessors into the stored N_max-sized arrays (leading sub-blocks are nested). */
#define AQ(S, q, i, j)     ((S)->A[((size_t)(q) * (S)->Nm + (i)) * (S)->Nm + (j)])
#define CQ(S, q, i, j, k)  ((S)->C[(((size_t)(q) * (S)->Nm + (i)) * (S)->Nm + (j)) * (S)->Nm + (k)])
#define FQ(S, q, i)        ((S)->F[(size_t)(q) * (S)->Nm + (i)])
#define HM(S, i, j)        ((S)->H[(size_t)(i) * (S)->Nm + (j)])

static double seminorm(const orc_set *S, int n, const double *v)
{
    double s = 0.0;
    int i, j;
    if (!S->H) {
        for (i = 0; i < n; ++i) s += v[i] * v[i];
        return sqrt(s);
    }
    for (i = 0; i < n; ++i) {
        double t = 0.0;
        for (j = 0; j < n; ++j) t += HM(S, i, j) * v[j];
        s += v[i] * t;
    }
    return sqrt(s > 0.0 ? s : 0.0);
}

/* A(mu) (n x n, row-major) from the affine terms. */
static void affine_A(const orc_set *S, int n, const double *ta, double *Am)
{
    int q, i, j;
    for (i = 0; i < n; ++i)
        for (j = 0; j < n; ++j) {
            double s = 0.0;
            for (q = 0; q < S->Q; ++q) s += ta[q] * AQ(S, q, i, j);
            Am[i * n + j] = s;
        }
}

/* F(u) = A(mu) u + C(mu)(u,u) - f, straight from the definition. */
static void residual(const orc_set *S, int n, const double *Am, const double *tc,
                     const double *f, const double *u, double *r)
{
    int q, i, j, k;
    for (i = 0; i < n; ++i) {
        double s = 0.0;
        for (j = 0; j < n; ++j) s += Am[i * n + j] * u[j];
        for (q = 0; q < S->Qc; ++q) {
            double c = 0.0;
            for (j = 0; j < n; ++j)
                for (k = 0; k < n; ++k) c += CQ(S, q, i, j, k) * u[j] * u[k];
            s += tc[q] * c;
        }
        r[i] = s - f[i];
    }
}

/* Jacobian J = A(mu) + sum_q theta^c_q sum_k (C_q[i,j,k] + C_q[i,k,j]) u_k. */
static void jacobian(const orc_set *S, int n, const double *Am, const double *tc,
                     const double *u, double *J)
{
    int q, i, j, k;
    for (i = 0; i < n; ++i)
        for (j = 0; j < n; ++j) {
            double s = Am[i * n + j];
            for (q = 0; q < S->Qc; ++q) {
                double c = 0.0;
                for (k = 0; k < n; ++k) c += (CQ(S, q, i, j, k) + CQ(S, q, i, k, j)) * u[k];
                s += tc[q] * c;
            }
            J[i * n + j] = s;
        }
}

/*
 * One reduced Newton solve at basis size n <= Nm.
 * f: the right-hand side f(mu) (length n). u0: initial iterate or NULL (zero).
 * u (out, length n); iters (out): number of Newton updates applied;
 * hist (optional, length maxit): update norms ||delta_t||_H.
 */
int orc_newton(const orc_set *S, int n, const double *ta, const double *tc, const double *f,
               const double *u0, double tol, int maxit, double *u, int *iters, double *hist)
{
    double *Am, *J, *r;
    int t, i, st = ORC_MAXIT;
    if (n < 1 || n > S->Nm) { *iters = 0; return ORC_BADN; }
    Am = (double *)malloc(sizeof(double) * n * n);
    J = (double *)malloc(sizeof(double) * n * n);
    r = (double *)malloc(sizeof(double) * n);
    affine_A(S, n, ta, Am);
    for (i = 0; i < n; ++i) u[i] = u0 ? u0[i] : 0.0;
    *iters = 0;
    for (t = 0; t < maxit; ++t) {
        double nd, nu;
        int s;
        jacobian(S, n, Am, tc, u, J);
        residual(S, n, Am, tc, f, u, r);
        for (i = 0; i < n; ++i) r[i] = -r[i];
        s = orc_gepp_solve(n, J, r, NULL);            /* r <- delta */
        if (s != ORC_OK) { st = s; break; }
        for (i = 0; i < n; ++i) u[i] += r[i];
        *iters = t + 1;
        nd = seminorm(S, n, r);
        nu = seminorm(S, n, u);
        if (hist) hist[t] = nd;
        if (!isfinite(nd) || !isfinite(nu)) { st = ORC_NONFINITE; break; }
        if (nd <= tol * nu) { st = ORC_OK; break; }
    }
    free(Am); free(J); free(r);
    return st;
}

/*
 * Picard (fixed-point) iteration, the alternative nonlinear solver the paper names
 * (Section 3.5): (A(mu) + P(u^m)) u^{m+1} = f with P[i,k] = sum_q theta^c_q sum_j C_q[i,j,k] u^m_j.
 * Used only to cross-check Newton on tiny systems.
 */
int orc_picard(const orc_set *S, int n, const double *ta, const double *tc, const double *f,
               double tol, int maxit, double *u, int *iters)
{
    double *Am, *P, *x;
    int m, i, j, k, q, st = ORC_MAXIT;
    if (n < 1 || n > S->Nm) return ORC_BADN;
    Am = (double *)malloc(sizeof(double) * n * n);
    P = (double *)malloc(sizeof(double) * n * n);
    x = (double *)malloc(sizeof(double) * n);
    affine_A(S, n, ta, Am);
    for (i = 0; i < n; ++i) u[i] = 0.0;
    *iters = 0;
    for (m = 0; m < maxit; ++m) {
        double dn = 0.0, un = 0.0;
        int s;
        for (i = 0; i < n; ++i)
            for (k = 0; k < n; ++k) {
                double v = Am[i * n + k];
                for (q = 0; q < S->Qc; ++q) {
                    double c = 0.0;
                    for (j = 0; j < n; ++j) c += CQ(S, q, i, j, k) * u[j];
                    v += tc[q] * c;
                }
                P[i * n + k] = v;
            }
        for (i = 0; i < n; ++i) x[i] = f[i];
        s = orc_gepp_solve(n, P, x, NULL);
        if (s != ORC_OK) { st = s; break; }
        for (i = 0; i < n; ++i) {
            dn += (x[i] - u[i]) * (x[i] - u[i]);
            un += x[i] * x[i];
            u[i] = x[i];
        }
        *iters = m + 1;
        if (sqrt(dn) <= tol * sqrt(un)) { st = ORC_OK; break; }
    }
    free(Am); free(P); free(x);
    return st;
}

/*
 * A posteriori pressure recovery at velocity size n and pressure size np:
 *   B(mu) p = f_s(mu) - A_sv(mu) u - C_sv(mu)(u, u),  B(mu) = sum_q theta^b_q Bp_q.
 */
int orc_pressure(const orc_set *S, int n, int np, const double *ta, const double *tc,
                 const double *tf, const double *tb, const double *u, double *p)
{
    double *Bm;
    int q, i, j, k, st;
    const int Nm = S->Nm, Npm = S->Npm;
    if (n < 1 || n > Nm || np < 1 || np > Npm) return ORC_BADN;
    Bm = (double *)malloc(sizeof(double) * np * np);
    for (i = 0; i < np; ++i)
        for (j = 0; j < np; ++j) {
            double s = 0.0;
            for (q = 0; q < S->Qb; ++q) s += tb[q] * S->Bp[((size_t)q * Npm + i) * Npm + j];
            Bm[i * np + j] = s;
        }
    for (i = 0; i < np; ++i) {
        double s = 0.0;
        for (q = 0; q < S->Qf; ++q) s += tf[q] * S->Fs[(size_t)q * Npm + i];
        for (q = 0; q < S->Q; ++q) {
            double a = 0.0;
            for (j = 0; j < n; ++j) a += S->Asv[((size_t)q * Npm + i) * Nm + j] * u[j];
            s -= ta[q] * a;
        }
        for (q = 0; q < S->Qc; ++q) {
            double c = 0.0;
            for (j = 0; j < n; ++j)
                for (k = 0; k < n; ++k)
                    c += S->Csv[(((size_t)q * Npm + i) * Nm + j) * Nm + k] * u[j] * u[k];
            s -= tc[q] * c;
        }
        p[i] = s;
    }
    st = orc_gepp_solve(np, Bm, p, NULL);
    free(Bm);
    return st;
}

/*
 * A batch of independent solves (OpenMP over requests). Per request b:
 *   Nreq[b]   basis size (<= Nm), or NULL for Nm;
 *   mu[b]     = (alpha, Re); theta is evaluated here with orc_theta;
 *   fover     (optional) [B][Nm] right-hand sides replacing f(mu) (manufactured solutions);
 *   u0        (optional) [B][Nm] initial iterates;
 *   u, iters, status: outputs ([B][Nm], [B], [B]).
 * With np > 0 and p != NULL the pressure ([B][Npm]) is recovered from the final iterate of
 * every request whose velocity solve ended with status 0 or 1; pstatus[b] gets its status.
 * Returns the number of threads used.
 */
int orc_solve_batch(const orc_set *S, int B, const int *Nreq, const double *mu,
                    const double *fover, const double *u0, double tol, int maxit,
                    double *u, int *iters, int *status, int np, double *p, int *pstatus,
                    int nthreads)
{
    int used = 1;
    int b;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
    {
#pragma omp single
        used = omp_get_num_threads();
    }
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (b = 0; b < B; ++b) {
        const int Nm = S->Nm;
        int n = Nreq ? Nreq[b] : Nm;
        double ta[ORC_MAX_Q], tc[ORC_MAX_QC], tf[2], tb[2];
        double *f = (double *)malloc(sizeof(double) * Nm);
        double *ub = u + (size_t)b * Nm;
        int q, i;
        memset(ub, 0, sizeof(double) * Nm);
        if (n < 1 || n > Nm) { status[b] = ORC_BADN; iters[b] = 0; free(f); continue; }
        orc_theta(S->Q, S->Qc, S->Qf, S->Qb, mu[2 * b], mu[2 * b + 1], ta, tc, tf, tb);
        for (i = 0; i < n; ++i) {
            if (fover) f[i] = fover[(size_t)b * Nm + i];
            else {
                double s = 0.0;
                for (q = 0; q < S->Qf; ++q) s += tf[q] * FQ(S, q, i);
                f[i] = s;
            }
        }
        status[b] = orc_newton(S, n, ta, tc, f, u0 ? u0 + (size_t)b * Nm : NULL, tol, maxit,
                               ub, &iters[b], NULL);
        if (np > 0 && p) {
            double *pb = p + (size_t)b * S->Npm;
            memset(pb, 0, sizeof(double) * S->Npm);
            if (status[b] == ORC_OK || status[b] == ORC_MAXIT)
                pstatus[b] = orc_pressure(S, n, np, ta, tc, tf, tb, ub, pb);
            else
                pstatus[b] = status[b];
        }
        free(f);
    }
    return used;
}
