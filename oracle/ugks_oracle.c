/*
 * ugks_oracle.c -- plain, slow FP64 CPU oracle of one time step of the
 * memory-saving unified gas-kinetic scheme (UGKS) on unstructured meshes:
 * Y. Zhang, Y. Wei, W. Long, K. Xu, "An efficiency and memory-saving
 * programming paradigm for the unified gas-kinetic scheme", arXiv:2412.06546.
 *
 * TEST INFRASTRUCTURE.  This is the parity reference for the HIP library.
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg load
 * it.  It shares no code, header, table or helper with the HIP path.
 *
 * The step follows Algorithm 1 (Section 3.2) in the paper's order:
 *   1  time step from the CFL condition (once: the velocity grid is fixed)
 *      and the heat flux of every cell;
 *   2  reconstruction of the macroscopic variables;
 *   3  equilibrium state and time coefficients at every interface;
 *   4-8 loop over discrete velocities k: reconstruct f_k (least squares +
 *      Venkatakrishnan limiter), evolve the micro flux (Eqs. microscopicFlux
 *      and fullSolution) and its macro contribution (Eq. macroscopicFlux),
 *      keep f_k and its gradient at wall faces, and overwrite f_k^n with
 *      the stage-1 value (Eq. microS1) in place;
 *   9  wall flux (the wall density needs every k, Eq. maxWalldes);
 *  10  macroscopic update (Eq. macroscopicUpdata);
 *  11  stage-2 update of f (Eq. microS2).
 * Only f (h and b per cell and velocity), the macroscopic fields, per-face
 * data and one velocity's gradient buffer are kept, as in Section 3.2.
 *
 * Readings of points the paper leaves to its references (all stated with
 * the functions that use them):
 *  - R = 1/2, lambda = 1/(2RT) = 1/T; monatomic gas with K = 0, so the
 *    internal velocity xi has M = 3 - D components and the total number of
 *    translational + internal degrees of freedom is N = D + M = 3.
 *  - tau = mu(T)/p with mu = mu_ref T^omega and p = rho R T.
 *  - g0 is the Maxwellian of the moments of the two half-Maxwellians of the
 *    reconstructed macro states (continuous moments, face-normal frame).
 *  - grad g0 uses the average of the two limited cell gradients of W; the
 *    time derivative follows from the compatibility condition.
 *  - interface heat flux = average of the two cells' heat fluxes (Sec. 3.2).
 *  - f(0,t) is integrated over the step: coefficients q1..q5 are the time
 *    integrals of c1..c5 of Eq. fullSolution.
 *  - wall and far-field boundary fluxes are collision-free over the step:
 *    outgoing particles carry f_in - t u.grad f_in, incoming particles the
 *    wall Maxwellian (density from zero mass flux) or the ghost Maxwellian.
 *  - q^{n+1} = q~ / (1 + Pr dt / (2 tau^{n+1})), q~ the heat flux of the
 *    stage-1 distribution about U^{n+1}.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXF 8
#define ORC_MAXD 3
#define ORC_MAXW 5
#define ORC_GH 4 /* Gauss-Hermite nodes per dimension: exact to degree 7 */

typedef struct {
    int dim, n_cells, n_faces, n_vel;
    const double *cell_volume, *cell_centroid;
    const int *face_cells;
    const double *face_normal, *face_area, *face_centroid, *face_shift;
    const int *face_bc, *face_bc_id;
    const double *u, *w;
    double Pr, omega, mu_ref, cfl, dt_override, limiter_k;
    int limiter, n_bc;
    const double *bc_prim;
    const double *prim0;
} orc_input_t;

/* interface data of Algorithm 1's interface-equilibrium step */
typedef struct {
    double p[ORC_MAXW], tau; /* (rho, U, lambda) of g0 */
    double a[ORC_MAXD][ORC_MAXW]; /* spatial slopes of g0 per direction */
    double A[ORC_MAXW];           /* time slope of g0 */
    double q[ORC_MAXD];           /* interface heat flux */
    double c[5];                  /* time integrals of c1..c5 */
} orc_face_eq_t;

typedef struct orc {
    int D, M, N, NC, NW, nc, nf, nv;
    double *vol, *xc, *fn, *fa, *fx, *fs, *u, *w, *bcp;
    int *fcell, *fbc, *fbcid, nbc;
    double Pr, omega, mu_ref, limiter_k;
    int limiter;
    int *ncf, *cf, *cside; /* faces of each cell; side 0 = left, 1 = right */
    double *dcf;           /* [nc][MAXF][D]: cell centroid -> face centroid */
    int *nnb, *nb;         /* least-squares stencil (face neighbours) */
    double *dnb;           /* [nc][MAXF][D]: centroid -> neighbour image */
    double *Ginv;          /* [nc][D][D]; all zero when the stencil is degenerate */
    double *eps2;          /* Venkatakrishnan epsilon^2 per cell */
    int nwall, *wall_face;
    double *wallF; /* [nwall][NW]: macroscopic flux through each wall face in the
                      last step, per unit area and time (Section 2.5) */
    double dt;
    double *f; /* [nv][nc][NC]: velocity-major, as the k loop walks it */
    double *W; /* [nc][NW] conservative */
    double *q; /* [nc][D] heat flux */
    double res[ORC_MAXW];
    long nstep;
} orc_t;

/* ------------------------------------------------------------------------ */
/* Section 2.1: macroscopic variables                                       */
/* ------------------------------------------------------------------------ */
static void prim_of_cons(int D, int N, const double *W, double *p)
{
    double rho = W[0], ke = 0.0;
    p[0] = rho;
    for (int d = 0; d < D; ++d) {
        p[1 + d] = W[1 + d] / rho;
        ke += p[1 + d] * p[1 + d];
    }
    /* rho E = rho/2 (|U|^2 + N/(2 lambda)) */
    p[D + 1] = N * rho / (4.0 * (W[D + 1] - 0.5 * rho * ke));
}

static void cons_of_prim(int D, int N, const double *p, double *W)
{
    double ke = 0.0;
    W[0] = p[0];
    for (int d = 0; d < D; ++d) {
        W[1 + d] = p[0] * p[1 + d];
        ke += p[1 + d] * p[1 + d];
    }
    W[D + 1] = 0.5 * p[0] * (ke + N / (2.0 * p[D + 1]));
}

static double tau_of_prim(const orc_t *o, const double *p)
{
    double lam = p[o->D + 1];
    double T = 1.0 / lam;            /* R = 1/2 */
    double mu = o->mu_ref * pow(T, o->omega);
    double pres = 0.5 * p[0] * T;    /* p = rho R T */
    return mu / pres;
}

/* ------------------------------------------------------------------------ */
/* Section 2.2: reduced Maxwellian H, B and Shakhov parts H+, B+ (K = 0)    */
/* ------------------------------------------------------------------------ */
static void reduced_eq(int D, const double *p, const double *q, double Pr, const double *u,
                       double *H, double *B, double *Hp, double *Bp)
{
    const int K = 0;
    double rho = p[0], lam = p[D + 1], c2 = 0.0, cq = 0.0;
    for (int d = 0; d < D; ++d) {
        double c = u[d] - p[1 + d];
        c2 += c * c;
        cq += c * q[d];
    }
    double h = rho * pow(lam / M_PI, 0.5 * D) * exp(-lam * c2);
    *H = h;
    *B = (3 - D + K) / (2.0 * lam) * h;
    double pre = 4.0 * (1.0 - Pr) * lam * lam / (5.0 * rho) * cq;
    *Hp = pre * (2.0 * lam * c2 - 2.0 - D) * h;
    *Bp = pre * ((2.0 * lam * c2 - D) * (3 - D + K) - 2.0 * K) * h / (2.0 * lam);
}

/* ------------------------------------------------------------------------ */
/* Gaussian moments by product Gauss-Hermite quadrature with weight e^{-x^2} */
/* and 4 nodes per dimension, exact for polynomials of degree 7 (the        */
/* moments used here reach degree 5).  The nodes are the roots of the       */
/* Hermite polynomial H_4(x) = 16x^4 - 48x^2 + 12, i.e. x^2 = (3 -+ sqrt 6)/2, */
/* and the weights are sqrt(pi) 2^{n-1} n! / (n^2 H_{n-1}(x)^2) with n = 4,  */
/* which simplifies to sqrt(pi) / (4 (3 -+ sqrt 6)).  Nodes ascending.       */
/* ------------------------------------------------------------------------ */
static void gauss_hermite4(double *x, double *wt)
{
    const double s6 = sqrt(6.0), sp = sqrt(M_PI);
    const double xin = sqrt((3.0 - s6) / 2.0), xout = sqrt((3.0 + s6) / 2.0);
    const double win = sp / (4.0 * (3.0 - s6)), wout = sp / (4.0 * (3.0 + s6));
    x[0] = -xout; wt[0] = wout;
    x[1] = -xin;  wt[1] = win;
    x[2] = xin;   wt[2] = win;
    x[3] = xout;  wt[3] = wout;
}

/* psi = (1, u, (|u|^2 + |xi|^2)/2) at a point (u, xi) */
static void psi_at(int D, int M, const double *u, const double *xi, double *ps)
{
    double e = 0.0;
    ps[0] = 1.0;
    for (int d = 0; d < D; ++d) {
        ps[1 + d] = u[d];
        e += u[d] * u[d];
    }
    for (int m = 0; m < M; ++m) e += xi[m] * xi[m];
    ps[D + 1] = 0.5 * e;
}

/* Expectation <F> over the normalised Maxwellian with velocity U and lambda,
 * for F built from psi: out[i][j] = <psi_i psi_j> and
 * rhs[i] = -sum_d <psi_i u_d (a^d . psi)> (the compatibility condition). */
static void maxwell_moments(int D, int M, const double *U, double lam, const double (*a)[ORC_MAXW],
                            double *mat, double *rhs)
{
    double gx[ORC_GH], gw[ORC_GH];
    gauss_hermite4(gx, gw);
    int N = D + M, NW = D + 2, tot = 1;
    for (int d = 0; d < N; ++d) tot *= ORC_GH;
    double s = 1.0 / sqrt(lam), norm = pow(M_PI, -0.5 * N);
    if (mat) memset(mat, 0, sizeof(double) * NW * NW);
    if (rhs) memset(rhs, 0, sizeof(double) * NW);
    for (int idx = 0; idx < tot; ++idx) {
        int r = idx;
        double wgt = norm, u[ORC_MAXD], xi[ORC_MAXD], ps[ORC_MAXW];
        for (int d = 0; d < N; ++d) {
            int j = r % ORC_GH;
            r /= ORC_GH;
            wgt *= gw[j];
            if (d < D) u[d] = U[d] + s * gx[j];
            else xi[d - D] = s * gx[j];
        }
        psi_at(D, M, u, xi, ps);
        if (mat)
            for (int i = 0; i < NW; ++i)
                for (int j = 0; j < NW; ++j) mat[i * NW + j] += wgt * ps[i] * ps[j];
        if (rhs) {
            double adv = 0.0;
            for (int d = 0; d < D; ++d) {
                double ap = 0.0;
                for (int j = 0; j < NW; ++j) ap += a[d][j] * ps[j];
                adv += u[d] * ap;
            }
            for (int i = 0; i < NW; ++i) rhs[i] -= wgt * ps[i] * adv;
        }
    }
}

/* Gaussian elimination with partial pivoting, n <= 5 */
static void solve_small(int n, const double *A_in, const double *b_in, double *x)
{
    double A[ORC_MAXW * ORC_MAXW], b[ORC_MAXW];
    memcpy(A, A_in, sizeof(double) * n * n);
    memcpy(b, b_in, sizeof(double) * n);
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[r * n + c]) > fabs(A[piv * n + c])) piv = r;
        if (piv != c) {
            for (int j = 0; j < n; ++j) {
                double t = A[c * n + j];
                A[c * n + j] = A[piv * n + j];
                A[piv * n + j] = t;
            }
            double t = b[c];
            b[c] = b[piv];
            b[piv] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            double m = A[r * n + c] / A[c * n + c];
            for (int j = c; j < n; ++j) A[r * n + j] -= m * A[c * n + j];
            b[r] -= m * b[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int j = r + 1; j < n; ++j) s -= A[r * n + j] * x[j];
        x[r] = s / A[r * n + r];
    }
}

/* Spatial slope of g0: solve <psi (a . psi)> = dW / rho (Section 2.4, g0's
 * expansion r . grad g0). */
static void slope_of_g0(int D, int M, const double *p, const double *dW, double *a)
{
    double mat[ORC_MAXW * ORC_MAXW], rhs[ORC_MAXW];
    maxwell_moments(D, M, p + 1, p[D + 1], NULL, mat, NULL);
    for (int i = 0; i < D + 2; ++i) rhs[i] = dW[i] / p[0];
    solve_small(D + 2, mat, rhs, a);
}

/* Time slope of g0 from the compatibility condition
 * integral psi (u . grad g0 + d g0/dt) = 0. */
static void time_slope_of_g0(int D, int M, const double *p, const double (*a)[ORC_MAXW], double *A)
{
    double mat[ORC_MAXW * ORC_MAXW], rhs[ORC_MAXW];
    maxwell_moments(D, M, p + 1, p[D + 1], a, mat, rhs);
    solve_small(D + 2, mat, rhs, A);
}

/* ------------------------------------------------------------------------ */
/* Half-range moments of a 1D normalised Gaussian N(U, 1/(2 lambda)):       */
/* m[j] = integral over sign*u > 0 of u^j sqrt(lambda/pi) e^{-lambda(u-U)^2}  */
/* ------------------------------------------------------------------------ */
static void half_moments(double U, double lam, int sign, double *m)
{
    double t = sqrt(lam) * U;
    double g = exp(-lam * U * U) / (2.0 * sqrt(M_PI * lam));
    if (sign > 0) {
        m[0] = 0.5 * erfc(-t);
        m[1] = U * m[0] + g;
    } else {
        m[0] = 0.5 * erfc(t);
        m[1] = U * m[0] - g;
    }
    m[2] = U * m[1] + m[0] / (2.0 * lam);
}

/* W0 = integral_{u_n > 0} psi g[left] + integral_{u_n < 0} psi g[right] */
static void half_merge(int D, int N, const double *pl, const double *pr, const double *n, double *W0)
{
    const double *ps[2] = {pl, pr};
    int sg[2] = {+1, -1};
    memset(W0, 0, sizeof(double) * (D + 2));
    for (int s = 0; s < 2; ++s) {
        const double *p = ps[s];
        double rho = p[0], lam = p[D + 1], Un = 0.0;
        for (int d = 0; d < D; ++d) Un += p[1 + d] * n[d];
        double Ut[ORC_MAXD], ut2 = 0.0;
        for (int d = 0; d < D; ++d) {
            Ut[d] = p[1 + d] - Un * n[d];
            ut2 += Ut[d] * Ut[d];
        }
        double m[3];
        half_moments(Un, lam, sg[s], m);
        W0[0] += rho * m[0];
        for (int d = 0; d < D; ++d) W0[1 + d] += rho * (m[1] * n[d] + Ut[d] * m[0]);
        /* energy: u_n^2 from the half range, the other N-1 degrees of freedom
         * (tangential velocity and xi) from the full Gaussian */
        W0[D + 1] += 0.5 * rho * (m[2] + (ut2 + (N - 1) / (2.0 * lam)) * m[0]);
    }
}

/* ------------------------------------------------------------------------ */
/* Time integrals over [0, dt] of c1..c5 of Eq. fullSolution.  Closed forms */
/* lose all precision for small x = dt/tau, so x < 1 uses their Taylor      */
/* series (sum from the smallest term).                                     */
/* ------------------------------------------------------------------------ */
static void time_integrals(double dt, double tau, double *c)
{
    double x = dt / tau;
    if (x < 1.0) {
        const int MT = 30;
        double term[31];
        term[0] = 1.0;
        for (int m = 1; m <= MT; ++m) term[m] = term[m - 1] * x / m; /* x^m/m! */
        double s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0;
        for (int m = MT; m >= 1; --m) {
            double sgn = (m % 2) ? 1.0 : -1.0; /* (-1)^(m+1) */
            s1 += sgn * term[m];
            if (m >= 2) {
                s2 += sgn * (m - 1) * term[m];
                s3 -= sgn * term[m];
            }
            if (m >= 3) {
                s4 -= sgn * (m - 2) * term[m];
                s5 += sgn * term[m];
            }
        }
        c[0] = tau * s1;
        c[1] = tau * tau * s2;
        c[2] = tau * s3;
        c[3] = tau * tau * s4;
        c[4] = tau * tau * s5;
    } else {
        double e = exp(-x), ome = -expm1(-x);
        c[0] = tau * ome;
        c[1] = tau * dt * e - tau * tau * ome;
        c[2] = dt - tau * ome;
        c[3] = 2.0 * tau * tau * ome - tau * dt * (1.0 + e);
        c[4] = 0.5 * dt * dt - tau * dt + tau * tau * ome;
    }
}

/* ------------------------------------------------------------------------ */
/* Reconstruction (Section 3.1 step 2): unweighted least squares about the  */
/* centroid over face neighbours, Venkatakrishnan limiter.                  */
/* ------------------------------------------------------------------------ */
static double venkat(double dm, double dp, double eps2)
{
    if (dm == 0.0) return 1.0;
    return (dp * dp + eps2 + 2.0 * dm * dp) / (dp * dp + 2.0 * dm * dm + dm * dp + eps2);
}

/* limited gradient of a scalar field; val(j) gives the value at cell j */
static void limited_gradient(const orc_t *o, int i, const double *vals, int stride, double *g)
{
    int D = o->D;
    double fi = vals[(size_t)i * stride], rhs[ORC_MAXD] = {0, 0, 0};
    double fmax = fi, fmin = fi;
    for (int j = 0; j < o->nnb[i]; ++j) {
        double fj = vals[(size_t)o->nb[i * ORC_MAXF + j] * stride];
        const double *d = o->dnb + ((size_t)i * ORC_MAXF + j) * D;
        for (int a = 0; a < D; ++a) rhs[a] += d[a] * (fj - fi);
        if (fj > fmax) fmax = fj;
        if (fj < fmin) fmin = fj;
    }
    const double *Gi = o->Ginv + (size_t)i * D * D;
    for (int a = 0; a < D; ++a) {
        g[a] = 0.0;
        for (int b = 0; b < D; ++b) g[a] += Gi[a * D + b] * rhs[b];
    }
    if (!o->limiter) return;
    double phi = 1.0;
    for (int fl = 0; fl < o->ncf[i]; ++fl) {
        const double *r = o->dcf + ((size_t)i * ORC_MAXF + fl) * D;
        double dm = 0.0;
        for (int a = 0; a < D; ++a) dm += g[a] * r[a];
        double dp = dm > 0.0 ? fmax - fi : fmin - fi;
        double ph = venkat(dm, dp, o->eps2[i]);
        if (ph < phi) phi = ph;
    }
    for (int a = 0; a < D; ++a) g[a] *= phi;
}

/* ------------------------------------------------------------------------ */
/* set-up                                                                   */
/* ------------------------------------------------------------------------ */
static double *dup_d(const double *p, size_t n)
{
    double *q = (double *)malloc(sizeof(double) * (n ? n : 1));
    if (p) memcpy(q, p, sizeof(double) * n);
    else memset(q, 0, sizeof(double) * (n ? n : 1));
    return q;
}
static int *dup_i(const int *p, size_t n, int fill)
{
    int *q = (int *)malloc(sizeof(int) * (n ? n : 1));
    if (p) memcpy(q, p, sizeof(int) * n);
    else for (size_t i = 0; i < n; ++i) q[i] = fill;
    return q;
}

static void heat_flux_of(const orc_t *o, int i, const double *U, const double *fsrc, double *qout)
{
    int D = o->D;
    for (int d = 0; d < D; ++d) qout[d] = 0.0;
    for (int k = 0; k < o->nv; ++k) {
        const double *fk = fsrc + ((size_t)k * o->nc + i) * o->NC;
        double c[ORC_MAXD], c2 = 0.0;
        for (int d = 0; d < D; ++d) {
            c[d] = o->u[(size_t)k * D + d] - U[d];
            c2 += c[d] * c[d];
        }
        double b = o->NC > 1 ? fk[1] : 0.0;
        for (int d = 0; d < D; ++d) qout[d] += 0.5 * o->w[k] * c[d] * (c2 * fk[0] + b);
    }
}

/* W and q as direct moments of the stored f */
static void moments_from_f(orc_t *o)
{
    int D = o->D, NW = o->NW;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < o->nc; ++i) {
        double *W = o->W + (size_t)i * NW;
        for (int m = 0; m < NW; ++m) W[m] = 0.0;
        for (int k = 0; k < o->nv; ++k) {
            const double *fk = o->f + ((size_t)k * o->nc + i) * o->NC;
            const double *uk = o->u + (size_t)k * D;
            double u2 = 0.0, b = o->NC > 1 ? fk[1] : 0.0;
            W[0] += o->w[k] * fk[0];
            for (int d = 0; d < D; ++d) {
                W[1 + d] += o->w[k] * uk[d] * fk[0];
                u2 += uk[d] * uk[d];
            }
            W[D + 1] += o->w[k] * 0.5 * (u2 * fk[0] + b);
        }
        double p[ORC_MAXW];
        prim_of_cons(D, o->N, W, p);
        heat_flux_of(o, i, p + 1, o->f, o->q + (size_t)i * D);
    }
}

orc_t *orc_create(const orc_input_t *in)
{
    if (in->dim != 2 && in->dim != 3) return NULL;
    orc_t *o = (orc_t *)calloc(1, sizeof(orc_t));
    int D = o->D = in->dim;
    o->M = 3 - D;
    o->N = D + o->M;
    o->NC = o->M > 0 ? 2 : 1;
    o->NW = D + 2;
    o->nc = in->n_cells;
    o->nf = in->n_faces;
    o->nv = in->n_vel;
    o->vol = dup_d(in->cell_volume, o->nc);
    o->xc = dup_d(in->cell_centroid, (size_t)o->nc * D);
    o->fcell = dup_i(in->face_cells, (size_t)o->nf * 2, 0);
    o->fn = dup_d(in->face_normal, (size_t)o->nf * D);
    o->fa = dup_d(in->face_area, o->nf);
    o->fx = dup_d(in->face_centroid, (size_t)o->nf * D);
    o->fs = dup_d(in->face_shift, (size_t)o->nf * D);
    o->fbc = dup_i(in->face_bc, o->nf, 0);
    o->fbcid = dup_i(in->face_bc_id, o->nf, 0);
    o->u = dup_d(in->u, (size_t)o->nv * D);
    o->w = dup_d(in->w, o->nv);
    o->nbc = in->n_bc;
    o->bcp = dup_d(in->bc_prim, (size_t)(in->n_bc > 0 ? in->n_bc : 1) * (D + 2));
    o->Pr = in->Pr;
    o->omega = in->omega;
    o->mu_ref = in->mu_ref;
    o->limiter = in->limiter;
    o->limiter_k = in->limiter_k;

    /* cell -> faces */
    o->ncf = (int *)calloc(o->nc, sizeof(int));
    o->cf = (int *)calloc((size_t)o->nc * ORC_MAXF, sizeof(int));
    o->cside = (int *)calloc((size_t)o->nc * ORC_MAXF, sizeof(int));
    o->dcf = (double *)calloc((size_t)o->nc * ORC_MAXF * D, sizeof(double));
    o->nnb = (int *)calloc(o->nc, sizeof(int));
    o->nb = (int *)calloc((size_t)o->nc * ORC_MAXF, sizeof(int));
    o->dnb = (double *)calloc((size_t)o->nc * ORC_MAXF * D, sizeof(double));
    o->nwall = 0;
    for (int f = 0; f < o->nf; ++f) {
        if (o->fbc[f] == 3) o->nwall++;
        for (int s = 0; s < 2; ++s) {
            int c = o->fcell[2 * f + s];
            if (c < 0) continue;
            int slot = o->ncf[c]++;
            if (slot >= ORC_MAXF) {
                fprintf(stderr, "oracle: cell %d has more than %d faces\n", c, ORC_MAXF);
                return NULL;
            }
            o->cf[c * ORC_MAXF + slot] = f;
            o->cside[c * ORC_MAXF + slot] = s;
            for (int d = 0; d < D; ++d) {
                /* face centroid in this cell's frame */
                double xf = o->fx[f * D + d] - (s == 1 ? o->fs[f * D + d] : 0.0);
                o->dcf[((size_t)c * ORC_MAXF + slot) * D + d] = xf - o->xc[c * D + d];
            }
            int other = o->fcell[2 * f + 1 - s];
            if (other >= 0) {
                int j = o->nnb[c]++;
                o->nb[c * ORC_MAXF + j] = other;
                for (int d = 0; d < D; ++d) {
                    double xo = o->xc[other * D + d] + (s == 0 ? o->fs[f * D + d] : -o->fs[f * D + d]);
                    o->dnb[((size_t)c * ORC_MAXF + j) * D + d] = xo - o->xc[c * D + d];
                }
            }
        }
    }
    o->wall_face = (int *)malloc(sizeof(int) * (o->nwall ? o->nwall : 1));
    for (int f = 0, n = 0; f < o->nf; ++f)
        if (o->fbc[f] == 3) o->wall_face[n++] = f;
    o->wallF = (double *)calloc((size_t)(o->nwall ? o->nwall : 1) * o->NW, sizeof(double));

    /* least-squares normal matrices, inverted once.  A stencil with no more
     * neighbours than dimensions (a triangle or tetrahedron with a boundary
     * face) has no redundancy: its fit interpolates the neighbours and its
     * extrapolation to the cell's other faces leans downwind, which makes
     * the second-order transport unstable there; such a cell, like one with
     * a degenerate normal matrix, keeps a zero gradient (first order). */
    o->Ginv = (double *)calloc((size_t)o->nc * D * D, sizeof(double));
    o->eps2 = (double *)calloc(o->nc, sizeof(double));
    for (int i = 0; i < o->nc; ++i) {
        double G[9] = {0};
        for (int j = 0; j < o->nnb[i]; ++j) {
            const double *d = o->dnb + ((size_t)i * ORC_MAXF + j) * D;
            for (int a = 0; a < D; ++a)
                for (int b = 0; b < D; ++b) G[a * D + b] += d[a] * d[b];
        }
        double *Gi = o->Ginv + (size_t)i * D * D, tr = 0.0, det;
        for (int a = 0; a < D; ++a) tr += G[a * D + a];
        if (D == 2) {
            det = G[0] * G[3] - G[1] * G[2];
            if (o->nnb[i] > D && det > 1e-10 * pow(tr / D, D)) {
                Gi[0] = G[3] / det; Gi[1] = -G[1] / det;
                Gi[2] = -G[2] / det; Gi[3] = G[0] / det;
            }
        } else {
            double c00 = G[4] * G[8] - G[5] * G[7], c01 = G[5] * G[6] - G[3] * G[8], c02 = G[3] * G[7] - G[4] * G[6];
            det = G[0] * c00 + G[1] * c01 + G[2] * c02;
            if (o->nnb[i] > D && det > 1e-10 * pow(tr / D, D)) {
                Gi[0] = c00 / det;
                Gi[1] = (G[2] * G[7] - G[1] * G[8]) / det;
                Gi[2] = (G[1] * G[5] - G[2] * G[4]) / det;
                Gi[3] = c01 / det;
                Gi[4] = (G[0] * G[8] - G[2] * G[6]) / det;
                Gi[5] = (G[2] * G[3] - G[0] * G[5]) / det;
                Gi[6] = c02 / det;
                Gi[7] = (G[1] * G[6] - G[0] * G[7]) / det;
                Gi[8] = (G[0] * G[4] - G[1] * G[3]) / det;
            }
        }
        double h = pow(o->vol[i], 1.0 / D), kh = o->limiter_k * h;
        o->eps2[i] = kh * kh * kh;
    }

    /* Algorithm 1's first step, time step: the largest dt with every cell's upwind
     * outflow no more than CFL times its volume, over all velocities. */
    if (in->dt_override > 0.0) {
        o->dt = in->dt_override;
    } else {
        double best = INFINITY;
#pragma omp parallel for schedule(static) reduction(min : best)
        for (int i = 0; i < o->nc; ++i)
            for (int k = 0; k < o->nv; ++k) {
                double out = 0.0;
                for (int fl = 0; fl < o->ncf[i]; ++fl) {
                    int f = o->cf[i * ORC_MAXF + fl];
                    double sg = o->cside[i * ORC_MAXF + fl] == 0 ? 1.0 : -1.0, un = 0.0;
                    for (int d = 0; d < D; ++d) un += o->u[(size_t)k * D + d] * o->fn[f * D + d];
                    un *= sg;
                    if (un > 0.0) out += o->fa[f] * un;
                }
                if (out > 0.0 && o->vol[i] / out < best) best = o->vol[i] / out;
            }
        o->dt = in->cfl * best;
    }

    /* initial state: discrete Maxwellian of the given primitive field;
     * W^0 and q^0 are its discrete moments */
    o->f = (double *)malloc(sizeof(double) * (size_t)o->nv * o->nc * o->NC);
    o->W = (double *)calloc((size_t)o->nc * o->NW, sizeof(double));
    o->q = (double *)calloc((size_t)o->nc * D, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int i = 0; i < o->nc; ++i) {
        double p[ORC_MAXW], zq[ORC_MAXD] = {0, 0, 0};
        for (int m = 0; m < D + 1; ++m) p[m] = in->prim0[(size_t)i * (D + 2) + m];
        p[D + 1] = 1.0 / in->prim0[(size_t)i * (D + 2) + D + 1]; /* T -> lambda */
        for (int k = 0; k < o->nv; ++k) {
            double H, B, Hp, Bp;
            reduced_eq(D, p, zq, 1.0, o->u + (size_t)k * D, &H, &B, &Hp, &Bp);
            double *fk = o->f + ((size_t)k * o->nc + i) * o->NC;
            fk[0] = H;
            if (o->NC > 1) fk[1] = B;
        }
    }
    moments_from_f(o);
    return o;
}

void orc_destroy(orc_t *o)
{
    if (!o) return;
    free(o->vol); free(o->xc); free(o->fcell); free(o->fn); free(o->fa); free(o->fx); free(o->fs);
    free(o->fbc); free(o->fbcid); free(o->u); free(o->w); free(o->bcp);
    free(o->ncf); free(o->cf); free(o->cside); free(o->dcf); free(o->nnb); free(o->nb); free(o->dnb);
    free(o->Ginv); free(o->eps2); free(o->wall_face); free(o->wallF); free(o->f); free(o->W); free(o->q);
    free(o);
}

double orc_dt(const orc_t *o) { return o->dt; }

/* threads of the OpenMP loops from now on (timing at one core and at all) */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
long orc_nstep(const orc_t *o) { return o->nstep; }

/* f in [cell][component][velocity] order, then W and q as its moments */
void orc_set_f(orc_t *o, const double *f)
{
    for (int i = 0; i < o->nc; ++i)
        for (int c = 0; c < o->NC; ++c)
            for (int k = 0; k < o->nv; ++k)
                o->f[((size_t)k * o->nc + i) * o->NC + c] = f[((size_t)i * o->NC + c) * o->nv + k];
    moments_from_f(o);
}

void orc_get(const orc_t *o, double *W, double *q, double *f)
{
    if (W) memcpy(W, o->W, sizeof(double) * (size_t)o->nc * o->NW);
    if (q) memcpy(q, o->q, sizeof(double) * (size_t)o->nc * o->D);
    if (f)
        for (int i = 0; i < o->nc; ++i)
            for (int c = 0; c < o->NC; ++c)
                for (int k = 0; k < o->nv; ++k)
                    f[((size_t)i * o->NC + c) * o->nv + k] = o->f[((size_t)k * o->nc + i) * o->NC + c];
}

void orc_residual(const orc_t *o, double *res) { memcpy(res, o->res, sizeof(double) * o->NW); }

/* Section 2.5: the macroscopic flux F_w through every wall face in the last
 * step (wall faces in increasing face index), per unit area and time:
 * mass, momentum [D], energy.  Surface pressure p_w = F_m . n, shear stress
 * |F_m - p_w n| and heat flux F_energy follow from it. */
int orc_n_wall(const orc_t *o) { return o->nwall; }
void orc_wall_flux(const orc_t *o, double *out)
{
    memcpy(out, o->wallF, sizeof(double) * (size_t)o->nwall * o->NW);
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1, macroscopic reconstruction: limited least-squares gradients  */
/* of the conservative                                                      */
/* variables [nc][NW][D].  A cell whose reconstructed state at any of its   */
/* face centroids has rho <= 0 or internal energy <= 0 falls back to first  */
/* order (zero gradient); fell_back[i] (if given) records it.               */
/* ------------------------------------------------------------------------ */
static void macro_gradients(const orc_t *o, double *gW, int *fell_back)
{
    const int D = o->D, NW = o->NW, nc = o->nc;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nc; ++i) {
        for (int m = 0; m < NW; ++m) limited_gradient(o, i, o->W + m, NW, gW + ((size_t)i * NW + m) * D);
        int bad = 0;
        for (int fl = 0; fl < o->ncf[i] && !bad; ++fl) {
            const double *r = o->dcf + ((size_t)i * ORC_MAXF + fl) * D;
            double Wf[ORC_MAXW], ke = 0.0;
            for (int m = 0; m < NW; ++m) {
                Wf[m] = o->W[(size_t)i * NW + m];
                for (int a = 0; a < D; ++a) Wf[m] += gW[((size_t)i * NW + m) * D + a] * r[a];
            }
            for (int d = 0; d < D; ++d) ke += Wf[1 + d] * Wf[1 + d];
            if (!(Wf[0] > 0.0) || !(Wf[D + 1] - 0.5 * ke / Wf[0] > 0.0)) bad = 1;
        }
        if (bad) memset(gW + (size_t)i * NW * D, 0, sizeof(double) * NW * D);
        if (fell_back) fell_back[i] = bad;
    }
}

/* ------------------------------------------------------------------------ */
/* one time step (Algorithm 1)                                              */
/* ------------------------------------------------------------------------ */
static void one_step(orc_t *o)
{
    const int D = o->D, M = o->M, N = o->N, NC = o->NC, NW = o->NW, nc = o->nc, nf = o->nf, nv = o->nv;
    const double dt = o->dt;

    /* time step and heat flux: q^n is the value carried from the previous step
     * (direct moment of f at the start); collision time tau^n */
    double *prim = (double *)malloc(sizeof(double) * nc * NW);
    double *tau = (double *)malloc(sizeof(double) * nc);
    for (int i = 0; i < nc; ++i) {
        prim_of_cons(D, N, o->W + (size_t)i * NW, prim + (size_t)i * NW);
        tau[i] = tau_of_prim(o, prim + (size_t)i * NW);
    }

    /* macroscopic reconstruction: limited gradients of the conservative variables */
    double *gW = (double *)calloc((size_t)nc * NW * D, sizeof(double));
    macro_gradients(o, gW, NULL);

    /* interface equilibrium and time coefficients */
    orc_face_eq_t *fe = (orc_face_eq_t *)calloc(nf, sizeof(orc_face_eq_t));
#pragma omp parallel for schedule(static)
    for (int f = 0; f < nf; ++f) {
        int l = o->fcell[2 * f], r = o->fcell[2 * f + 1];
        if (r < 0) continue;
        const double *n = o->fn + (size_t)f * D;
        double Wl[ORC_MAXW], Wr[ORC_MAXW], pl[ORC_MAXW], pr[ORC_MAXW], W0[ORC_MAXW], p0[ORC_MAXW];
        for (int m = 0; m < NW; ++m) {
            Wl[m] = o->W[(size_t)l * NW + m];
            Wr[m] = o->W[(size_t)r * NW + m];
            for (int a = 0; a < D; ++a) {
                double xf = o->fx[f * D + a];
                Wl[m] += gW[((size_t)l * NW + m) * D + a] * (xf - o->xc[l * D + a]);
                Wr[m] += gW[((size_t)r * NW + m) * D + a] * (xf - o->fs[f * D + a] - o->xc[r * D + a]);
            }
        }
        prim_of_cons(D, N, Wl, pl);
        prim_of_cons(D, N, Wr, pr);
        half_merge(D, N, pl, pr, n, W0);
        prim_of_cons(D, N, W0, p0);
        orc_face_eq_t *e = fe + f;
        for (int m = 0; m < NW; ++m) e->p[m] = p0[m];
        e->tau = tau_of_prim(o, p0);
        for (int d = 0; d < D; ++d) {
            double dW[ORC_MAXW];
            for (int m = 0; m < NW; ++m)
                dW[m] = 0.5 * (gW[((size_t)l * NW + m) * D + d] + gW[((size_t)r * NW + m) * D + d]);
            slope_of_g0(D, M, p0, dW, e->a[d]);
        }
        time_slope_of_g0(D, M, p0, (const double(*)[ORC_MAXW])e->a, e->A);
        for (int d = 0; d < D; ++d) e->q[d] = 0.5 * (o->q[(size_t)l * D + d] + o->q[(size_t)r * D + d]);
        time_integrals(dt, e->tau, e->c);
    }

    /* the velocity loop */
    double *gk = (double *)calloc((size_t)nc * NC * D, sizeof(double)); /* gradient buffer */
    double *Fk = (double *)calloc((size_t)nf * NC, sizeof(double));     /* u_n int f dt */
    double *Fmac = (double *)calloc((size_t)nf * NW, sizeof(double));
    double *wallbuf = (double *)calloc((size_t)(o->nwall ? o->nwall : 1) * nv * NC * (1 + D), sizeof(double));
    const double h0fac = M * (M + 2) / 4.0; /* <|xi|^4> = M(M+2)/(4 lambda^2) */

    for (int k = 0; k < nv; ++k) {
        const double *uk = o->u + (size_t)k * D;
        double *fkk = o->f + (size_t)k * nc * NC;
        double u2 = 0.0;
        for (int d = 0; d < D; ++d) u2 += uk[d] * uk[d];

        /* reconstruct f_k */
#pragma omp parallel for schedule(static)
        for (int i = 0; i < nc; ++i)
            for (int c = 0; c < NC; ++c) limited_gradient(o, i, fkk + c, NC, gk + ((size_t)i * NC + c) * D);

        /* micro flux and its macroscopic contribution */
#pragma omp parallel for schedule(static)
        for (int f = 0; f < nf; ++f) {
            const int bc = o->fbc[f];
            const int l = o->fcell[2 * f], r = o->fcell[2 * f + 1];
            const double *n = o->fn + (size_t)f * D;
            double un = 0.0;
            for (int d = 0; d < D; ++d) un += uk[d] * n[d];
            double I[2] = {0.0, 0.0};
            if (bc == 3) { /* wall: evolved after the loop */
                Fk[(size_t)f * NC] = 0.0;
                if (NC > 1) Fk[(size_t)f * NC + 1] = 0.0;
                continue;
            }
            if (r >= 0) {
                /* upwind side (ties go right) and its reconstruction at the face */
                int s = un > 0.0 ? l : r;
                double dvec[ORC_MAXD];
                for (int d = 0; d < D; ++d)
                    dvec[d] = o->fx[f * D + d] - (s == l ? 0.0 : o->fs[f * D + d]) - o->xc[s * D + d];
                const orc_face_eq_t *e = fe + f;
                double H0, B0, H0p, B0p;
                reduced_eq(D, e->p, e->q, o->Pr, uk, &H0, &B0, &H0p, &B0p);
                /* u . grad g0 and d g0/dt, integrated over xi */
                double Pd = 0.0, Ed = 0.0;
                for (int d = 0; d < D; ++d) {
                    double pa = e->a[d][0] + 0.5 * e->a[d][D + 1] * u2;
                    for (int c = 0; c < D; ++c) pa += e->a[d][1 + c] * uk[c];
                    Pd += uk[d] * pa;
                    Ed += uk[d] * e->a[d][D + 1];
                }
                double PA = e->A[0] + 0.5 * e->A[D + 1] * u2;
                for (int c = 0; c < D; ++c) PA += e->A[1 + c] * uk[c];
                double xi4 = h0fac / (e->p[D + 1] * e->p[D + 1]) * H0; /* integral xi^4 g0 dxi */
                double gH = Pd * H0 + 0.5 * Ed * B0, gB = Pd * B0 + 0.5 * Ed * xi4;
                double tH = PA * H0 + 0.5 * e->A[D + 1] * B0, tB = PA * B0 + 0.5 * e->A[D + 1] * xi4;
                double eqH = H0 + H0p, eqB = B0 + B0p;
                for (int c = 0; c < NC; ++c) {
                    const double *g = gk + ((size_t)s * NC + c) * D;
                    double fs = fkk[(size_t)s * NC + c], ug = 0.0;
                    for (int d = 0; d < D; ++d) {
                        fs += g[d] * dvec[d];
                        ug += uk[d] * g[d];
                    }
                    double eq = c == 0 ? eqH : eqB, gg = c == 0 ? gH : gB, tt = c == 0 ? tH : tB;
                    I[c] = e->c[0] * fs + e->c[1] * ug + e->c[2] * eq + e->c[3] * gg + e->c[4] * tt;
                }
            } else {
                /* far field: outgoing particles transported freely from the
                 * interior reconstruction, incoming ones from the ghost
                 * Maxwellian (free stream, or the interior state on outflow) */
                if (un > 0.0) {
                    for (int c = 0; c < NC; ++c) {
                        const double *g = gk + ((size_t)l * NC + c) * D;
                        double fv = fkk[(size_t)l * NC + c], ug = 0.0;
                        for (int d = 0; d < D; ++d) {
                            fv += g[d] * (o->fx[f * D + d] - o->xc[l * D + d]);
                            ug += uk[d] * g[d];
                        }
                        I[c] = dt * fv - 0.5 * dt * dt * ug;
                    }
                } else {
                    double pg[ORC_MAXW], zq[ORC_MAXD] = {0, 0, 0}, H, B, Hp, Bp;
                    if (bc == 1) {
                        const double *bp = o->bcp + (size_t)o->fbcid[f] * (D + 2);
                        for (int m = 0; m < D + 1; ++m) pg[m] = bp[m];
                        pg[D + 1] = 1.0 / bp[D + 1];
                    } else {
                        for (int m = 0; m < NW; ++m) pg[m] = prim[(size_t)l * NW + m];
                    }
                    reduced_eq(D, pg, zq, 1.0, uk, &H, &B, &Hp, &Bp);
                    I[0] = dt * H;
                    I[1] = dt * B;
                }
            }
            for (int c = 0; c < NC; ++c) Fk[(size_t)f * NC + c] = un * I[c];
            /* Eq. macroscopicFlux */
            double Hf = un * I[0], Bf = NC > 1 ? un * I[1] : 0.0;
            double *F = Fmac + (size_t)f * NW;
            F[0] += o->w[k] * Hf;
            for (int d = 0; d < D; ++d) F[1 + d] += o->w[k] * uk[d] * Hf;
            F[D + 1] += o->w[k] * 0.5 * (u2 * Hf + Bf);
        }

        /* f_k and its gradient at wall faces */
        for (int wi = 0; wi < o->nwall; ++wi) {
            int f = o->wall_face[wi], l = o->fcell[2 * f];
            for (int c = 0; c < NC; ++c) {
                double *slot = wallbuf + (((size_t)wi * nv + k) * NC + c) * (1 + D);
                const double *g = gk + ((size_t)l * NC + c) * D;
                double fv = fkk[(size_t)l * NC + c];
                for (int d = 0; d < D; ++d) {
                    fv += g[d] * (o->fx[f * D + d] - o->xc[l * D + d]);
                    slot[1 + d] = g[d];
                }
                slot[0] = fv;
            }
        }

        /* stage 1 (Eq. microS1), in place */
#pragma omp parallel for schedule(static)
        for (int i = 0; i < nc; ++i) {
            const double *p = prim + (size_t)i * NW;
            double H, B, Hp, Bp;
            reduced_eq(D, p, o->q + (size_t)i * D, o->Pr, uk, &H, &B, &Hp, &Bp);
            double fplus[2] = {H + Hp, B + Bp};
            for (int c = 0; c < NC; ++c) {
                double sum = 0.0;
                for (int fl = 0; fl < o->ncf[i]; ++fl) {
                    int f = o->cf[i * ORC_MAXF + fl];
                    double sg = o->cside[i * ORC_MAXF + fl] == 0 ? 1.0 : -1.0;
                    sum += sg * o->fa[f] * Fk[(size_t)f * NC + c];
                }
                double *fv = fkk + (size_t)i * NC + c;
                *fv = *fv - sum / o->vol[i] + 0.5 * dt * (fplus[c] - *fv) / tau[i];
            }
        }
    }

    /* boundary flux at the wall.  rho_w makes the net mass flux through the wall
     * vanish (Eq. maxWalldes); incident particles carry f_in - t u.grad f_in */
    for (int wi = 0; wi < o->nwall; ++wi) {
        int f = o->wall_face[wi], l = o->fcell[2 * f];
        const double *n = o->fn + (size_t)f * D;
        const double *bp = o->bcp + (size_t)o->fbcid[f] * (D + 2);
        double pw[ORC_MAXW], zq[ORC_MAXD] = {0, 0, 0};
        pw[0] = 1.0;
        for (int d = 0; d < D; ++d) pw[1 + d] = bp[1 + d];
        pw[D + 1] = 1.0 / bp[D + 1];
        double sin_ = 0.0, sout = 0.0;
        for (int k = 0; k < nv; ++k) {
            const double *uk = o->u + (size_t)k * D;
            double un = 0.0;
            for (int d = 0; d < D; ++d) un += uk[d] * n[d];
            if (un > 0.0) {
                const double *slot = wallbuf + (((size_t)wi * nv + k) * NC + 0) * (1 + D);
                double ug = 0.0;
                for (int d = 0; d < D; ++d) ug += uk[d] * slot[1 + d];
                sin_ += o->w[k] * un * (dt * slot[0] - 0.5 * dt * dt * ug);
            } else {
                double H, B, Hp, Bp;
                reduced_eq(D, pw, zq, 1.0, uk, &H, &B, &Hp, &Bp);
                sout += o->w[k] * un * dt * H;
            }
        }
        double rho_w = -sin_ / sout;
        pw[0] = rho_w;
        double *F = Fmac + (size_t)f * NW;
        for (int k = 0; k < nv; ++k) {
            const double *uk = o->u + (size_t)k * D;
            double un = 0.0, u2 = 0.0, I[2] = {0.0, 0.0};
            for (int d = 0; d < D; ++d) {
                un += uk[d] * n[d];
                u2 += uk[d] * uk[d];
            }
            if (un > 0.0) {
                for (int c = 0; c < NC; ++c) {
                    const double *slot = wallbuf + (((size_t)wi * nv + k) * NC + c) * (1 + D);
                    double ug = 0.0;
                    for (int d = 0; d < D; ++d) ug += uk[d] * slot[1 + d];
                    I[c] = dt * slot[0] - 0.5 * dt * dt * ug;
                }
            } else {
                double H, B, Hp, Bp;
                reduced_eq(D, pw, zq, 1.0, uk, &H, &B, &Hp, &Bp);
                I[0] = dt * H;
                I[1] = dt * B;
            }
            double *fv = o->f + ((size_t)k * nc + l) * NC;
            for (int c = 0; c < NC; ++c) fv[c] -= o->fa[f] * un * I[c] / o->vol[l];
            double Hf = un * I[0], Bf = NC > 1 ? un * I[1] : 0.0;
            F[0] += o->w[k] * Hf;
            for (int d = 0; d < D; ++d) F[1 + d] += o->w[k] * uk[d] * Hf;
            F[D + 1] += o->w[k] * 0.5 * (u2 * Hf + Bf);
        }
        /* surface quantities: the wall's macroscopic flux per unit time */
        for (int m = 0; m < NW; ++m) o->wallF[(size_t)wi * NW + m] = F[m] / dt;
    }

    /* macroscopic update, Eq. macroscopicUpdata */
    double resnum[ORC_MAXW] = {0};
    for (int i = 0; i < nc; ++i) {
        double *W = o->W + (size_t)i * NW;
        for (int m = 0; m < NW; ++m) {
            double sum = 0.0;
            for (int fl = 0; fl < o->ncf[i]; ++fl) {
                int f = o->cf[i * ORC_MAXF + fl];
                double sg = o->cside[i * ORC_MAXF + fl] == 0 ? 1.0 : -1.0;
                sum += sg * o->fa[f] * Fmac[(size_t)f * NW + m];
            }
            double dW = -sum / o->vol[i];
            W[m] += dW;
            resnum[m] += dW * dW;
        }
    }
    for (int m = 0; m < NW; ++m) o->res[m] = sqrt(resnum[m]);

    /* micro update: tau^{n+1}, q^{n+1} and stage 2 (Eq. microS2) */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nc; ++i) {
        double p[ORC_MAXW], qt[ORC_MAXD];
        prim_of_cons(D, N, o->W + (size_t)i * NW, p);
        double t1 = tau_of_prim(o, p);
        heat_flux_of(o, i, p + 1, o->f, qt);
        double *qi = o->q + (size_t)i * D;
        for (int d = 0; d < D; ++d) qi[d] = qt[d] / (1.0 + o->Pr * dt / (2.0 * t1));
        for (int k = 0; k < nv; ++k) {
            double H, B, Hp, Bp;
            reduced_eq(D, p, qi, o->Pr, o->u + (size_t)k * D, &H, &B, &Hp, &Bp);
            double fplus[2] = {H + Hp, B + Bp};
            double *fv = o->f + ((size_t)k * nc + i) * NC;
            for (int c = 0; c < NC; ++c) fv[c] = (fv[c] + 0.5 * dt * fplus[c] / t1) / (1.0 + 0.5 * dt / t1);
        }
    }

    free(prim); free(tau); free(gW); free(fe); free(gk); free(Fk); free(Fmac); free(wallbuf);
    o->nstep++;
}

void orc_step(orc_t *o, int nsteps)
{
    for (int s = 0; s < nsteps; ++s) one_step(o);
}

/* ------------------------------------------------------------------------ */
/* pieces exported for the pin tests                                        */
/* ------------------------------------------------------------------------ */
void orc_time_integrals(double dt, double tau, double *c) { time_integrals(dt, tau, c); }
void orc_prim_of_cons(int D, const double *W, double *p) { prim_of_cons(D, 3, W, p); }
void orc_cons_of_prim(int D, const double *p, double *W) { cons_of_prim(D, 3, p, W); }
void orc_reduced_eq(int D, const double *p, const double *q, double Pr, int n, const double *u,
                    double *H, double *B, double *Hp, double *Bp)
{
    for (int k = 0; k < n; ++k) reduced_eq(D, p, q, Pr, u + (size_t)k * D, H + k, B + k, Hp + k, Bp + k);
}
void orc_half_merge(int D, const double *pl, const double *pr, const double *n, double *W0)
{
    half_merge(D, 3, pl, pr, n, W0);
}
void orc_slope_of_g0(int D, const double *p, const double *dW, double *a) { slope_of_g0(D, 3 - D, p, dW, a); }
void orc_time_slope_of_g0(int D, const double *p, const double *a, double *A)
{
    double aa[ORC_MAXD][ORC_MAXW];
    for (int d = 0; d < D; ++d)
        for (int m = 0; m < D + 2; ++m) aa[d][m] = a[d * (D + 2) + m];
    time_slope_of_g0(D, 3 - D, p, (const double(*)[ORC_MAXW])aa, A);
}
double orc_venkat(double dm, double dp, double eps2) { return venkat(dm, dp, eps2); }
/* the macroscopic reconstruction of Algorithm 1 for the current state: gW [nc][D+2][D], and per
 * cell whether it fell back to first order */
void orc_macro_gradients(const orc_t *o, double *gW, int *fell_back) { macro_gradients(o, gW, fell_back); }
/* the 4-point rule (returns the number of nodes written: 4) */
int orc_gauss_hermite(double *x, double *w)
{
    gauss_hermite4(x, w);
    return ORC_GH;
}
