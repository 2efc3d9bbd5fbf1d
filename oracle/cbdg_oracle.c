/*
 * Plain FP64 CPU oracle for the Chebyshev-BdG hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; it shares no code, header, table or helper with the GPU
 * path.  It is deliberately slow and literal:
 *   - the Nambu BdG Hamiltonian of eq. (hamil2) is built as an explicit sparse
 *     matrix (CSR, complex values) in the interleaved basis r = 2*s + alpha,
 *     alpha = 0 for the electron component (i,e) = c^dag_{i,up}|vac> and
 *     alpha = 1 for the hole component (i,h) = c_{i,down}|vac>;
 *   - the rescaled operator is (H - b)/a (paragraph after eq. (rec));
 *   - each start vector |s,e> is propagated on its own with the three-term
 *     vector recursion of eq. (ref2), and the moments are read off as
 *     <s,e|a_n> and <s,h|a_n> (eqs. (coeff1), (coeff2));
 *   - the adjoint stores every a_n of one start vector (no checkpointing) and
 *     runs the transposed recursion with an explicit transposed product.
 * OpenMP only distributes independent start vectors over threads.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex zdouble;

/* Upper bound on stored entries: per site two on-site entries per row and
 * two entries per neighbour per row, four neighbours, two rows. */
int64_t ora_csr_nnz_bound(int Lx, int Ly)
{
    return (int64_t)Lx * Ly * 2 * (2 + 2 * 4);
}

/* Neighbour j of site (x,y) in direction d (0:+x, 1:-x, 2:+y, 3:-y), or -1
 * when the bond leaves an open lattice.  Also returns the site that owns the
 * bond in the [2][L2] bond arrays and whether the bond is traversed forward. */
static int neighbour(int Lx, int Ly, int bcx, int bcy, int x, int y, int d,
                     int *owner, int *axis, int *forward)
{
    int jx = x, jy = y;
    switch (d) {
    case 0: jx = x + 1; break;
    case 1: jx = x - 1; break;
    case 2: jy = y + 1; break;
    default: jy = y - 1; break;
    }
    if (jx < 0 || jx >= Lx) {
        if (!bcx) return -1;
        jx = (jx + Lx) % Lx;
    }
    if (jy < 0 || jy >= Ly) {
        if (!bcy) return -1;
        jy = (jy + Ly) % Ly;
    }
    int s = x + Lx * y, j = jx + Lx * jy;
    *axis = (d < 2) ? 0 : 1;
    *forward = (d == 0 || d == 2);
    *owner = *forward ? s : j;
    return j;
}

/*
 * Explicit CSR of (H - b)/a, eq. (hamil2).
 *   on-site block   [[eps_i - mu,  Delta_i], [conj(Delta_i), -(eps_i - mu)]]
 *   bond block i!=j [[-t_ij, Delta_ij], [conj(Delta_ij), conj(t_ij)]]
 * with t_ij = t*exp(i theta_ij) for the bond owned by i in the forward
 * direction, t_ji = conj(t_ij), and Delta_ji = Delta_ij (singlet).
 * Complex arrays are interleaved (re, im).  delta_bond and peierls may be NULL.
 * Returns the number of stored entries, or -1 on bad arguments.
 */
int64_t ora_build_csr(int Lx, int Ly, int bcx, int bcy, double t, double mu_c,
                      const double *eps, const double *delta,
                      const double *delta_bond, const double *peierls,
                      double a, double b,
                      int64_t *rowptr, int32_t *col, double *val)
{
    if (Lx < 1 || Ly < 1 || !(a > 0.0)) return -1;
    if ((bcx && Lx < 3) || (bcy && Ly < 3)) return -1;
    const int64_t L2 = (int64_t)Lx * Ly;
    zdouble *v = (zdouble *)val;
    int64_t k = 0;
    for (int y = 0; y < Ly; ++y) {
        for (int x = 0; x < Lx; ++x) {
            int64_t s = x + (int64_t)Lx * y;
            double onsite = eps[s] - mu_c;
            zdouble dl = delta[2 * s] + I * delta[2 * s + 1];
            for (int alpha = 0; alpha < 2; ++alpha) {
                int64_t r = 2 * s + alpha;
                rowptr[r] = k;
                if (alpha == 0) {
                    col[k] = (int32_t)(2 * s);     v[k++] = (onsite - b) / a;
                    col[k] = (int32_t)(2 * s + 1); v[k++] = dl / a;
                } else {
                    col[k] = (int32_t)(2 * s);     v[k++] = conj(dl) / a;
                    col[k] = (int32_t)(2 * s + 1); v[k++] = (-onsite - b) / a;
                }
                for (int d = 0; d < 4; ++d) {
                    int owner, axis, fwd;
                    int j = neighbour(Lx, Ly, bcx, bcy, x, y, d, &owner, &axis, &fwd);
                    if (j < 0) continue;
                    double th = peierls ? peierls[axis * L2 + owner] : 0.0;
                    zdouble t_ij = t * cexp(I * (fwd ? th : -th));
                    zdouble d_ij = 0.0;
                    if (delta_bond) {
                        int64_t q = axis * L2 + owner;
                        d_ij = delta_bond[2 * q] + I * delta_bond[2 * q + 1];
                    }
                    if (alpha == 0) {
                        col[k] = 2 * j;     v[k++] = -t_ij / a;
                        col[k] = 2 * j + 1; v[k++] = d_ij / a;
                    } else {
                        col[k] = 2 * j;     v[k++] = conj(d_ij) / a;
                        col[k] = 2 * j + 1; v[k++] = conj(t_ij) / a;
                    }
                }
            }
        }
    }
    rowptr[2 * L2] = k;
    return k;
}

/* y = A x (complex) */
static void spmv_z(int64_t D, const int64_t *rp, const int32_t *ci,
                   const zdouble *v, const zdouble *x, zdouble *y)
{
    for (int64_t r = 0; r < D; ++r) {
        zdouble acc = 0.0;
        for (int64_t k = rp[r]; k < rp[r + 1]; ++k) acc += v[k] * x[ci[k]];
        y[r] = acc;
    }
}

/* y = A x (real values) */
static void spmv_d(int64_t D, const int64_t *rp, const int32_t *ci,
                   const double *v, const double *x, double *y)
{
    for (int64_t r = 0; r < D; ++r) {
        double acc = 0.0;
        for (int64_t k = rp[r]; k < rp[r + 1]; ++k) acc += v[k] * x[ci[k]];
        y[r] = acc;
    }
}

/* y = A^T x (real values), written as a scatter over the stored entries */
static void spmv_t_d(int64_t D, const int64_t *rp, const int32_t *ci,
                     const double *v, const double *x, double *y)
{
    for (int64_t r = 0; r < D; ++r) y[r] = 0.0;
    for (int64_t r = 0; r < D; ++r)
        for (int64_t k = rp[r]; k < rp[r + 1]; ++k) y[ci[k]] += v[k] * x[r];
}

static void set_threads(int n_threads)
{
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
}

int ora_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Moments of eq. (coeff1)/(coeff2) without the 1/(1+delta_{0n}) factor:
 *   mu_ee[k][n] = <s,e| T_n(Ht) |s,e>,  mu_he[k][n] = <s,h| T_n(Ht) |s,e>
 * for start site s = sites[k], n = 0..N-1, through eq. (ref2):
 *   a_0 = |s,e>, a_1 = Ht a_0, a_n = 2 Ht a_{n-1} - a_{n-2}.
 * is_complex = 0 requires every stored value to be real (checked).
 * mu_he is complex interleaved [n_start][N][2].  Returns 0, or -1 on error.
 */
int ora_moments(int64_t D, const int64_t *rowptr, const int32_t *col,
                const double *val, int is_complex, const int32_t *sites,
                int64_t n_start, int N, double *mu_ee, double *mu_he,
                int n_threads)
{
    if (N < 1 || D < 2) return -1;
    const int64_t nnz = rowptr[D];
    const zdouble *vz = (const zdouble *)val;
    double *vr = NULL;
    if (!is_complex) {
        vr = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
        if (!vr) return -1;
        for (int64_t k = 0; k < nnz; ++k) {
            if (cimag(vz[k]) != 0.0) { free(vr); return -1; }
            vr[k] = creal(vz[k]);
        }
    }
    for (int64_t q = 0; q < n_start; ++q)
        if (sites[q] < 0 || 2 * (int64_t)sites[q] >= D) { free(vr); return -1; }
    set_threads(n_threads);
    int err = 0;
#pragma omp parallel
    {
        void *b0 = calloc((size_t)D, is_complex ? sizeof(zdouble) : sizeof(double));
        void *b1 = calloc((size_t)D, is_complex ? sizeof(zdouble) : sizeof(double));
        void *b2 = calloc((size_t)D, is_complex ? sizeof(zdouble) : sizeof(double));
        if (!b0 || !b1 || !b2) {
#pragma omp atomic write
            err = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < n_start; ++q) {
            if (err) continue;
            const int64_t re = 2 * (int64_t)sites[q], rh = re + 1;
            double *mee = mu_ee + q * N;
            zdouble *mhe = (zdouble *)mu_he + q * N;
            if (is_complex) {
                zdouble *prev = (zdouble *)b0, *cur = (zdouble *)b1, *nxt = (zdouble *)b2;
                memset(prev, 0, sizeof(zdouble) * (size_t)D);
                prev[re] = 1.0;                       /* a_0 = |s,e> */
                mee[0] = creal(prev[re]); mhe[0] = prev[rh];
                if (N > 1) {
                    spmv_z(D, rowptr, col, vz, prev, cur);   /* a_1 = Ht a_0 */
                    mee[1] = creal(cur[re]); mhe[1] = cur[rh];
                }
                for (int n = 2; n < N; ++n) {
                    spmv_z(D, rowptr, col, vz, cur, nxt);
                    for (int64_t r = 0; r < D; ++r) nxt[r] = 2.0 * nxt[r] - prev[r];
                    mee[n] = creal(nxt[re]); mhe[n] = nxt[rh];
                    zdouble *tmp = prev; prev = cur; cur = nxt; nxt = tmp;
                }
            } else {
                double *prev = (double *)b0, *cur = (double *)b1, *nxt = (double *)b2;
                memset(prev, 0, sizeof(double) * (size_t)D);
                prev[re] = 1.0;
                mee[0] = prev[re]; mhe[0] = prev[rh];
                if (N > 1) {
                    spmv_d(D, rowptr, col, vr, prev, cur);
                    mee[1] = cur[re]; mhe[1] = cur[rh];
                }
                for (int n = 2; n < N; ++n) {
                    spmv_d(D, rowptr, col, vr, cur, nxt);
                    for (int64_t r = 0; r < D; ++r) nxt[r] = 2.0 * nxt[r] - prev[r];
                    mee[n] = nxt[re]; mhe[n] = nxt[rh];
                    double *tmp = prev; prev = cur; cur = nxt; nxt = tmp;
                }
            }
        }
        free(b0); free(b1); free(b2);
    }
    free(vr);
    return err ? -1 : 0;
}

/*
 * Reverse-mode derivative of L = sum_k sum_n (dmu_ee[k][n] mu_ee[k][n]
 *                                            + dmu_he[k][n] mu_he[k][n])
 * with respect to the on-site potential eps_j and a real on-site gap Delta_j,
 * for a real operator.  (a, b) are held fixed.
 *
 * With L = sum_n <w_n, a_n>, the adjoint vectors obey the transposed
 * recursion lam_n = w_n + 2 Ht^T lam_{n+1} - lam_{n+2} (lam_N = lam_{N+1} = 0)
 * and dL/dtheta = sum_{n>=1} c_n <lam_n, (dHt/dtheta) a_{n-1}> with c_1 = 1
 * (a_1 = Ht a_0 carries no factor 2) and c_n = 2 otherwise.  Here
 *   dHt/deps_j   = (|j,e><j,e| - |j,h><j,h|) / a
 *   dHt/dDelta_j = (|j,e><j,h| + |j,h><j,e|) / a.
 * Every a_n of a start vector is stored (N*D doubles per thread).
 * grad_eps and grad_delta are overwritten.  Returns 0 or -1.
 */
int ora_moments_backward(int64_t D, const int64_t *rowptr, const int32_t *col,
                         const double *val, const int32_t *sites, int64_t n_start,
                         int N, double a, const double *dmu_ee, const double *dmu_he,
                         double *grad_eps, double *grad_delta, int n_threads)
{
    if (N < 1 || D < 2 || !(a > 0.0)) return -1;
    const int64_t nnz = rowptr[D], L2 = D / 2;
    const zdouble *vz = (const zdouble *)val;
    double *vr = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    if (!vr) return -1;
    for (int64_t k = 0; k < nnz; ++k) {
        if (cimag(vz[k]) != 0.0) { free(vr); return -1; }
        vr[k] = creal(vz[k]);
    }
    for (int64_t q = 0; q < n_start; ++q)
        if (sites[q] < 0 || sites[q] >= L2) { free(vr); return -1; }
    for (int64_t j = 0; j < L2; ++j) { grad_eps[j] = 0.0; grad_delta[j] = 0.0; }
    set_threads(n_threads);
    int nthr = ora_max_threads();
    double *part = (double *)calloc((size_t)nthr * 2 * (size_t)L2, sizeof(double));
    if (!part) { free(vr); return -1; }
    int err = 0;
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *ge = part + (size_t)tid * 2 * L2, *gd = ge + L2;
        double *A = (double *)malloc(sizeof(double) * (size_t)N * (size_t)D);
        double *lam1 = (double *)calloc((size_t)D, sizeof(double));  /* lam_{n+1} */
        double *lam2 = (double *)calloc((size_t)D, sizeof(double));  /* lam_{n+2} */
        double *lam0 = (double *)calloc((size_t)D, sizeof(double));  /* lam_n */
        double *tmp = (double *)calloc((size_t)D, sizeof(double));
        if (!A || !lam1 || !lam2 || !lam0 || !tmp) {
#pragma omp atomic write
            err = 1;
        }
#pragma omp for schedule(static)
        for (int64_t q = 0; q < n_start; ++q) {
            if (err) continue;
            const int64_t re = 2 * (int64_t)sites[q], rh = re + 1;
            /* forward, storing every vector */
            memset(A, 0, sizeof(double) * (size_t)D);
            A[re] = 1.0;
            if (N > 1) spmv_d(D, rowptr, col, vr, A, A + D);
            for (int n = 2; n < N; ++n) {
                double *an = A + (size_t)n * D;
                spmv_d(D, rowptr, col, vr, A + (size_t)(n - 1) * D, an);
                for (int64_t r = 0; r < D; ++r) an[r] = 2.0 * an[r] - A[(size_t)(n - 2) * D + r];
            }
            /* backward */
            memset(lam1, 0, sizeof(double) * (size_t)D);
            memset(lam2, 0, sizeof(double) * (size_t)D);
            for (int n = N - 1; n >= 1; --n) {
                spmv_t_d(D, rowptr, col, vr, lam1, tmp);
                for (int64_t r = 0; r < D; ++r) lam0[r] = 2.0 * tmp[r] - lam2[r];
                lam0[re] += dmu_ee[q * N + n];
                lam0[rh] += dmu_he[q * N + n];
                const double c = (n == 1) ? 1.0 : 2.0;
                const double *ap = A + (size_t)(n - 1) * D;
                for (int64_t j = 0; j < L2; ++j) {
                    const double le = lam0[2 * j], lh = lam0[2 * j + 1];
                    const double xe = ap[2 * j], xh = ap[2 * j + 1];
                    ge[j] += c * (le * xe - lh * xh) / a;
                    gd[j] += c * (le * xh + lh * xe) / a;
                }
                double *t2 = lam2; lam2 = lam1; lam1 = lam0; lam0 = t2;
            }
        }
        free(A); free(lam1); free(lam2); free(lam0); free(tmp);
    }
    for (int th = 0; th < nthr; ++th)
        for (int64_t j = 0; j < L2; ++j) {
            grad_eps[j] += part[(size_t)th * 2 * L2 + j];
            grad_delta[j] += part[(size_t)th * 2 * L2 + L2 + j];
        }
    free(part);
    free(vr);
    return err ? -1 : 0;
}
