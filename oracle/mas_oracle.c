/*
 * FP64 CPU ORACLE for the implicit viscous solve -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code, header, table or helper with the
 * HIP library; it is a plain, slow, obviously-correct statement of what the
 * GPU path computes, in double precision, without blocking, fusion or
 * reordering beyond what the definitions below state.
 *
 * What is computed (the paper, Section 2: Eq. (1) viscosity term
 * (1/rho) div(nu rho grad v); Section 2.2: the viscous term is advanced
 * implicitly with a PCG solve using the inverse-diagonal (point-Jacobi, "PC1")
 * preconditioner, on a non-uniform logically rectangular spherical grid;
 * Section 4.1: the matrices are symmetric with few off-diagonal entries):
 *
 *   backward-Euler viscous step  (I - dt div(nu grad)) x = rhs
 *   finite-volume form           A x = b,  b = V .* rhs,
 *       (A x)_c = V_c x_c + sum_{faces f of c} c_f (x_c - x_nb(f))
 *       c_f     = dt * nu_f * area_f / dist_f
 *
 * Readings of points the paper leaves open (one scalar field with rho = 1,
 * cell-centred unknowns, homogeneous Dirichlet radial walls imposed at the
 * face, zero-area pole faces, arithmetic-mean face viscosity, midpoint cell
 * centres, metric distances r dtheta and r sin(theta) dphi) are the ones the
 * design document lists; each function below names the reading it uses.
 *
 * Cell index c = (i*nt + j)*np + k, i = r (slowest), j = theta, k = phi
 * (fastest, periodic).  Face arrays:
 *   r faces  : (nr+1)*nt*np, face i sits at r_faces[i]      (i = 0, nr are walls)
 *   th faces : nr*(nt+1)*np, face j sits at t_faces[j]      (j = 0, nt are poles)
 *   ph faces : nr*nt*np,     face k lies between k and k+1 (mod np)
 *
 * Dot products: partial sums per r plane, accumulated serially over planes,
 * so results do not depend on the OpenMP thread count.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_DIRICHLET 0
#define ORA_NEUMANN 1

typedef struct {
    int32_t nr, nt, np;
    const double *r_faces; /* nr+1 */
    const double *t_faces; /* nt+1 */
    int32_t bc_inner, bc_outer;
} ora_grid;

/* Geometry and operator, all owned by the caller (Python allocates). */
typedef struct {
    ora_grid g;
    double dt;
    double *V;      /* N              cell volumes                          */
    double *Ar, *Hr; /* (nr+1)*nt*np  r-face area, centre-to-centre distance */
    double *At, *Ht; /* nr*(nt+1)*np  theta-face area and distance           */
    double *Ap, *Hp; /* N             phi-face area and distance             */
    double *cr;     /* (nr+1)*nt*np   r-face conductance (0 if Neumann wall) */
    double *ct;     /* nr*(nt+1)*np   theta-face conductance (0 at poles)    */
    double *cp;     /* N              phi-face conductance                    */
    double *diag;   /* N              A_cc                                    */
} ora_op;

static inline size_t cidx(const ora_grid *g, int i, int j, int k) {
    return ((size_t)i * g->nt + j) * g->np + k;
}
static inline size_t ridx(const ora_grid *g, int i, int j, int k) { /* i in 0..nr */
    return ((size_t)i * g->nt + j) * g->np + k;
}
static inline size_t tidx(const ora_grid *g, int i, int j, int k) { /* j in 0..nt */
    return ((size_t)i * (g->nt + 1) + j) * g->np + k;
}
static inline size_t ncell(const ora_grid *g) {
    return (size_t)g->nr * g->nt * g->np;
}

/* ------------------------------------------------------------------ geometry
 * Cell volume of the spherical block [r-,r+] x [t-,t+] x [dphi]:
 *     V = (r+^3 - r-^3)/3 * (cos t- - cos t+) * dphi
 * evaluated without cancellation as (r+ - r-)(r+^2 + r+ r- + r-^2)/3 and
 * 2 sin((t+ + t-)/2) sin((t+ - t-)/2).
 * Cell centres are face midpoints.  Face areas are the exact areas of the
 * spherical patches; distances are metric centre-to-centre lengths:
 *     r face at r_f      area r_f^2 (cos t- - cos t+) dphi,  dist r_{i+1}-r_i
 *                        (walls: dist from the wall to the first centre)
 *     theta face at t_f  area sin(t_f) (r+^2 - r-^2)/2 dphi, dist r_i (t_{j+1}-t_j)
 *                        (pole faces t_f = 0, pi: area exactly 0)
 *     phi face           area (r+^2 - r-^2)/2 (t+ - t-),    dist r_i sin(t_j) dphi
 */
static double band(double ta, double tb) { /* cos ta - cos tb, ta < tb */
    return 2.0 * sin(0.5 * (ta + tb)) * sin(0.5 * (tb - ta));
}

int ora_geometry(ora_op *op) {
    const ora_grid *g = &op->g;
    const int nr = g->nr, nt = g->nt, np = g->np;
    const double *rf = g->r_faces, *tf = g->t_faces;
    const double dphi = 2.0 * M_PI / np;
    if (nr < 1 || nt < 1 || np < 1) return -1;

#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; i++) {
        double rm = rf[i], rp = rf[i + 1];
        double rc = 0.5 * (rm + rp);
        for (int j = 0; j < nt; j++) {
            double tm = tf[j], tp = tf[j + 1];
            double tc = 0.5 * (tm + tp);
            for (int k = 0; k < np; k++) {
                size_t c = cidx(g, i, j, k);
                op->V[c] = (rp - rm) * (rp * rp + rp * rm + rm * rm) / 3.0 * band(tm, tp) * dphi;
                op->Ap[c] = 0.5 * (rp * rp - rm * rm) * (tp - tm);
                op->Hp[c] = rc * sin(tc) * dphi;
            }
        }
    }
    /* r faces, including the two walls */
#pragma omp parallel for schedule(static)
    for (int i = 0; i <= nr; i++) {
        double rfa = rf[i];
        double h;
        if (i == 0)
            h = 0.5 * (rf[0] + rf[1]) - rf[0];
        else if (i == nr)
            h = rf[nr] - 0.5 * (rf[nr - 1] + rf[nr]);
        else
            h = 0.5 * (rf[i] + rf[i + 1]) - 0.5 * (rf[i - 1] + rf[i]);
        for (int j = 0; j < nt; j++) {
            double a = rfa * rfa * band(tf[j], tf[j + 1]) * dphi;
            for (int k = 0; k < np; k++) {
                op->Ar[ridx(g, i, j, k)] = a;
                op->Hr[ridx(g, i, j, k)] = h;
            }
        }
    }
    /* theta faces, including the two poles */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; i++) {
        double rm = rf[i], rp = rf[i + 1];
        double rc = 0.5 * (rm + rp);
        for (int j = 0; j <= nt; j++) {
            double a, h;
            if (j == 0 || j == nt) {
                a = 0.0; /* zero-area pole face */
                h = 1.0; /* unused */
            } else {
                a = sin(tf[j]) * 0.5 * (rp * rp - rm * rm) * dphi;
                h = rc * (0.5 * (tf[j] + tf[j + 1]) - 0.5 * (tf[j - 1] + tf[j]));
            }
            for (int k = 0; k < np; k++) {
                op->At[tidx(g, i, j, k)] = a;
                op->Ht[tidx(g, i, j, k)] = h;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ operator
 * Face viscosity: arithmetic mean of the two cells on interior faces; the
 * wall cell's own value on a Dirichlet wall face.  c_f = dt nu_f A_f / H_f.
 * With np == 1 the phi face joins a cell to itself and carries nothing.
 * Neumann walls carry no flux (c = 0).  Pole faces have zero area (c = 0).
 * diag_c = V_c + sum of the six face conductances of c (walls included).
 */
int ora_assemble(ora_op *op, const double *nu) {
    const ora_grid *g = &op->g;
    const int nr = g->nr, nt = g->nt, np = g->np;
    const double dt = op->dt;

#pragma omp parallel for schedule(static)
    for (int i = 0; i <= nr; i++)
        for (int j = 0; j < nt; j++)
            for (int k = 0; k < np; k++) {
                size_t f = ridx(g, i, j, k);
                double nuf;
                if (i == 0)
                    nuf = (g->bc_inner == ORA_DIRICHLET) ? nu[cidx(g, 0, j, k)] : 0.0;
                else if (i == nr)
                    nuf = (g->bc_outer == ORA_DIRICHLET) ? nu[cidx(g, nr - 1, j, k)] : 0.0;
                else
                    nuf = 0.5 * (nu[cidx(g, i - 1, j, k)] + nu[cidx(g, i, j, k)]);
                op->cr[f] = dt * nuf * op->Ar[f] / op->Hr[f];
            }

#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; i++)
        for (int j = 0; j <= nt; j++)
            for (int k = 0; k < np; k++) {
                size_t f = tidx(g, i, j, k);
                if (j == 0 || j == nt) {
                    op->ct[f] = 0.0;
                } else {
                    double nuf = 0.5 * (nu[cidx(g, i, j - 1, k)] + nu[cidx(g, i, j, k)]);
                    op->ct[f] = dt * nuf * op->At[f] / op->Ht[f];
                }
            }

#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; i++)
        for (int j = 0; j < nt; j++)
            for (int k = 0; k < np; k++) {
                size_t f = cidx(g, i, j, k);
                int kp = (k + 1) % np;
                double nuf = 0.5 * (nu[f] + nu[cidx(g, i, j, kp)]);
                /* with a single phi cell the face joins the cell to itself: no flux */
                op->cp[f] = (np == 1) ? 0.0 : dt * nuf * op->Ap[f] / op->Hp[f];
            }

#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; i++)
        for (int j = 0; j < nt; j++)
            for (int k = 0; k < np; k++) {
                size_t c = cidx(g, i, j, k);
                int km = (k + np - 1) % np;
                double s = op->V[c];
                s += op->cr[ridx(g, i, j, k)] + op->cr[ridx(g, i + 1, j, k)];
                s += op->ct[tidx(g, i, j, k)] + op->ct[tidx(g, i, j + 1, k)];
                s += op->cp[c] + op->cp[cidx(g, i, j, km)];
                op->diag[c] = s;
            }
    return 0;
}

/* (A x)_c = V_c x_c + sum_f c_f (x_c - x_nb), x_nb = 0 beyond a wall. */
void ora_apply(const ora_op *op, const double *x, double *y) {
    const ora_grid *g = &op->g;
    const int nr = g->nr, nt = g->nt, np = g->np;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; i++)
        for (int j = 0; j < nt; j++)
            for (int k = 0; k < np; k++) {
                size_t c = cidx(g, i, j, k);
                double xc = x[c];
                double s = op->V[c] * xc;
                /* -r face */
                double xn = (i > 0) ? x[cidx(g, i - 1, j, k)] : 0.0;
                s += op->cr[ridx(g, i, j, k)] * (xc - xn);
                /* +r face */
                xn = (i < nr - 1) ? x[cidx(g, i + 1, j, k)] : 0.0;
                s += op->cr[ridx(g, i + 1, j, k)] * (xc - xn);
                /* -theta face (zero conductance at the pole) */
                xn = (j > 0) ? x[cidx(g, i, j - 1, k)] : 0.0;
                s += op->ct[tidx(g, i, j, k)] * (xc - xn);
                /* +theta face */
                xn = (j < nt - 1) ? x[cidx(g, i, j + 1, k)] : 0.0;
                s += op->ct[tidx(g, i, j + 1, k)] * (xc - xn);
                /* -phi and +phi faces, periodic */
                int km = (k + np - 1) % np, kp = (k + 1) % np;
                s += op->cp[cidx(g, i, j, km)] * (xc - x[cidx(g, i, j, km)]);
                s += op->cp[c] * (xc - x[cidx(g, i, j, kp)]);
                y[c] = s;
            }
}

static double dot(const ora_grid *g, const double *a, const double *b, double *plane) {
    const int nr = g->nr;
    const size_t m = (size_t)g->nt * g->np;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; i++) {
        double s = 0.0;
        for (size_t c = (size_t)i * m; c < (size_t)(i + 1) * m; c++) s += a[c] * b[c];
        plane[i] = s;
    }
    double s = 0.0;
    for (int i = 0; i < nr; i++) s += plane[i];
    return s;
}

double ora_dot(const ora_grid *g, const double *a, const double *b) {
    double *plane = (double *)malloc(sizeof(double) * g->nr);
    double s = dot(g, a, b, plane);
    free(plane);
    return s;
}

/* b = V .* rhs */
void ora_rhs(const ora_op *op, const double *rhs, double *b) {
    size_t n = ncell(&op->g);
#pragma omp parallel for schedule(static)
    for (size_t c = 0; c < n; c++) b[c] = op->V[c] * rhs[c];
}

/* ------------------------------------------------------------------ PCG
 * Preconditioned conjugate gradient with M = diag(A) (point Jacobi, "PC1"),
 * in the order of the classical algorithm (Saad, Iterative Methods for
 * Sparse Linear Systems, preconditioned CG):
 *     r = b - A x;  z = M^-1 r;  p = z
 *     repeat:  q = A p;  alpha = (r,z)/(q,p);  x += alpha p;  r -= alpha q
 *              stop if ||r|| <= tol ||b||
 *              z = M^-1 r;  beta = (r,z)_new/(r,z)_old;  p = z + beta p
 * The stopping test uses the recursively updated residual; the true residual
 * ||b - A x||/||b|| is reported as well.  x holds x0 on entry if use_x0,
 * otherwise it is zeroed.  Returns the number of alpha steps taken, or -1 if
 * (q,p) <= 0 or is not finite.  stats = {rel_res_recursive, rel_res_true}.
 * If hist is non-null, hist[k] = ||r_k||/||b|| for k = 0..iterations.
 */
int ora_pcg(const ora_op *op, const double *b, double *x, double tol, int max_iters,
            int use_x0, double *stats, double *hist) {
    const ora_grid *g = &op->g;
    const size_t n = ncell(g);
    double *r = (double *)malloc(sizeof(double) * n);
    double *z = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    double *q = (double *)malloc(sizeof(double) * n);
    double *plane = (double *)malloc(sizeof(double) * g->nr);
    int it = 0, status = 0;

    if (!use_x0) memset(x, 0, sizeof(double) * n);
    ora_apply(op, x, q);
#pragma omp parallel for schedule(static)
    for (size_t c = 0; c < n; c++) {
        r[c] = b[c] - q[c];
        z[c] = r[c] / op->diag[c];
        p[c] = z[c];
    }
    double bnorm = sqrt(dot(g, b, b, plane));
    if (bnorm == 0.0) bnorm = 1.0;
    double rz = dot(g, r, z, plane);
    double rnorm = sqrt(dot(g, r, r, plane));
    if (hist) hist[0] = rnorm / bnorm;

    while (rnorm > tol * bnorm && it < max_iters) {
        ora_apply(op, p, q);
        double pq = dot(g, p, q, plane);
        if (!(pq > 0.0) || !isfinite(pq)) {
            status = -1;
            break;
        }
        double alpha = rz / pq;
#pragma omp parallel for schedule(static)
        for (size_t c = 0; c < n; c++) {
            x[c] += alpha * p[c];
            r[c] -= alpha * q[c];
        }
        it++;
        rnorm = sqrt(dot(g, r, r, plane));
        if (hist) hist[it] = rnorm / bnorm;
        if (rnorm <= tol * bnorm) break;
#pragma omp parallel for schedule(static)
        for (size_t c = 0; c < n; c++) z[c] = r[c] / op->diag[c];
        double rz_new = dot(g, r, z, plane);
        double beta = rz_new / rz;
        rz = rz_new;
#pragma omp parallel for schedule(static)
        for (size_t c = 0; c < n; c++) p[c] = z[c] + beta * p[c];
    }

    if (stats) {
        stats[0] = rnorm / bnorm;
        ora_apply(op, x, q);
#pragma omp parallel for schedule(static)
        for (size_t c = 0; c < n; c++) r[c] = b[c] - q[c];
        stats[1] = sqrt(dot(g, r, r, plane)) / bnorm;
    }
    free(r), free(z), free(p), free(q), free(plane);
    return status < 0 ? status : it;
}

/* ------------------------------------------------------------------ gradient
 * For L(x) with x = A(nu)^-1 (V .* rhs) and lam = A^-1 dL/dx (A is symmetric):
 *     dL/drhs_c = V_c lam_c
 *     dL/dnu_c  = - sum_f (d c_f / d nu_c) (lam_c - lam_nb)(x_c - x_nb)
 * because dL = -lam^T (dA) x and an interior face adds c_f (e_c - e_nb)(e_c - e_nb)^T
 * to A.  d c_f/d nu_c = dt A_f/(2 H_f) on interior faces, dt A_f/H_f on a
 * Dirichlet wall face (where lam_nb = x_nb = 0), 0 on Neumann walls and poles.
 */
void ora_gradient(const ora_op *op, const double *x, const double *lam, double *g_nu,
                  double *g_rhs) {
    const ora_grid *g = &op->g;
    const int nr = g->nr, nt = g->nt, np = g->np;
    const double dt = op->dt;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; i++)
        for (int j = 0; j < nt; j++)
            for (int k = 0; k < np; k++) {
                size_t c = cidx(g, i, j, k);
                double s = 0.0;
                size_t f;
                /* -r face */
                f = ridx(g, i, j, k);
                if (i > 0) {
                    size_t nb = cidx(g, i - 1, j, k);
                    s += 0.5 * dt * op->Ar[f] / op->Hr[f] * (lam[c] - lam[nb]) * (x[c] - x[nb]);
                } else if (g->bc_inner == ORA_DIRICHLET) {
                    s += dt * op->Ar[f] / op->Hr[f] * lam[c] * x[c];
                }
                /* +r face */
                f = ridx(g, i + 1, j, k);
                if (i < nr - 1) {
                    size_t nb = cidx(g, i + 1, j, k);
                    s += 0.5 * dt * op->Ar[f] / op->Hr[f] * (lam[c] - lam[nb]) * (x[c] - x[nb]);
                } else if (g->bc_outer == ORA_DIRICHLET) {
                    s += dt * op->Ar[f] / op->Hr[f] * lam[c] * x[c];
                }
                /* theta faces (pole faces have zero area) */
                if (j > 0) {
                    f = tidx(g, i, j, k);
                    size_t nb = cidx(g, i, j - 1, k);
                    s += 0.5 * dt * op->At[f] / op->Ht[f] * (lam[c] - lam[nb]) * (x[c] - x[nb]);
                }
                if (j < nt - 1) {
                    f = tidx(g, i, j + 1, k);
                    size_t nb = cidx(g, i, j + 1, k);
                    s += 0.5 * dt * op->At[f] / op->Ht[f] * (lam[c] - lam[nb]) * (x[c] - x[nb]);
                }
                /* phi faces */
                {
                    int km = (k + np - 1) % np, kp = (k + 1) % np;
                    size_t fm = cidx(g, i, j, km), nbm = fm;
                    size_t nbp = cidx(g, i, j, kp);
                    s += 0.5 * dt * op->Ap[fm] / op->Hp[fm] * (lam[c] - lam[nbm]) * (x[c] - x[nbm]);
                    s += 0.5 * dt * op->Ap[c] / op->Hp[c] * (lam[c] - lam[nbp]) * (x[c] - x[nbp]);
                }
                g_nu[c] = -s;
                if (g_rhs) g_rhs[c] = op->V[c] * lam[c];
            }
}

/* ------------------------------------------------------------------ RKL2 super time-stepping
 * The explicit alternative to the implicit solve for the viscous term (the paper, Section 2.2,
 * cites the second-order Runge-Kutta-Legendre scheme RKL2 of Meyer, Balsara and Aslam, 2014;
 * Section 3 reports about 200 such sub-steps per time step; Section 5.2 finds it the faster
 * choice on GPUs).  The stage recursion below is that published method restated, not taken
 * from the paper, which gives no coefficients.
 * It advances du/dt = L u by one step of the operator's dt, where the finite-volume
 * diffusion operator is L u = -(1/V) sum_f (c_f/dt)(u_c - u_nb); with A = V + dt K this is
 *     dt L u = u - (A u)/V.
 * s-stage recursion (w1 = 4/(s^2+s-2); b_0 = b_1 = b_2 = 1/3, b_j = (j^2+j-2)/(2j(j+1));
 * a_j = 1 - b_j; mu_j = (2j-1)/j b_j/b_{j-1}; nu_j = -(j-1)/j b_j/b_{j-2};
 * mt_j = mu_j w1 (mt_1 = b_1 w1); gt_j = -a_{j-1} mt_j):
 *     Y_0 = u,  Y_1 = Y_0 + mt_1 dtL(Y_0),
 *     Y_j = mu_j Y_{j-1} + nu_j Y_{j-2} + (1 - mu_j - nu_j) Y_0 + mt_j dtL(Y_{j-1}) + gt_j dtL(Y_0),
 *     u_new = Y_s.
 * It is stable while dt |lambda| <= (s^2 + s - 2)/2 for every eigenvalue lambda of L.
 */
void ora_rkl2_coefficients(int s, double *mu, double *nu, double *mt, double *gt) {
    double w1 = 4.0 / ((double)s * s + s - 2.0);
    double *b = (double *)malloc(sizeof(double) * (s + 1));
    for (int j = 0; j <= s; j++) b[j] = (j <= 2) ? 1.0 / 3.0 : ((double)j * j + j - 2.0) / (2.0 * j * (j + 1.0));
    for (int j = 0; j <= s; j++) mu[j] = nu[j] = mt[j] = gt[j] = 0.0;
    mt[1] = b[1] * w1;
    for (int j = 2; j <= s; j++) {
        mu[j] = (2.0 * j - 1.0) / j * b[j] / b[j - 1];
        nu[j] = -(j - 1.0) / j * b[j] / b[j - 2];
        mt[j] = mu[j] * w1;
        gt[j] = -(1.0 - b[j - 1]) * mt[j];
    }
    free(b);
}

/* Smallest s >= 2 with (s^2 + s - 2)/2 >= z_max, z_max = max_c 2 (A_cc - V_c)/V_c
 * (a Gershgorin bound of dt |lambda| for V^-1 (A - V)). */
int ora_rkl2_stages(const ora_op *op) {
    size_t n = ncell(&op->g);
    double zmax = 0.0;
    for (size_t c = 0; c < n; c++) {
        double z = 2.0 * (op->diag[c] - op->V[c]) / op->V[c];
        if (z > zmax) zmax = z;
    }
    int s = 2;
    while (((double)s * s + s - 2.0) / 2.0 < zmax) s++;
    return s;
}

static void dtL(const ora_op *op, const double *y, double *ay, double *out) {
    size_t n = ncell(&op->g);
    ora_apply(op, y, ay);
#pragma omp parallel for schedule(static)
    for (size_t c = 0; c < n; c++) out[c] = y[c] - ay[c] / op->V[c];
}

int ora_rkl2_step(const ora_op *op, const double *u0, double *u1, int s) {
    if (s < 2) return -1;
    size_t n = ncell(&op->g);
    double *mu = (double *)malloc(sizeof(double) * (s + 1)), *nu = (double *)malloc(sizeof(double) * (s + 1));
    double *mt = (double *)malloc(sizeof(double) * (s + 1)), *gt = (double *)malloc(sizeof(double) * (s + 1));
    ora_rkl2_coefficients(s, mu, nu, mt, gt);
    double *L0 = (double *)malloc(sizeof(double) * n), *Lj = (double *)malloc(sizeof(double) * n);
    double *ay = (double *)malloc(sizeof(double) * n);
    double *ym2 = (double *)malloc(sizeof(double) * n), *ym1 = (double *)malloc(sizeof(double) * n);
    double *yj = (double *)malloc(sizeof(double) * n);
    dtL(op, u0, ay, L0);
#pragma omp parallel for schedule(static)
    for (size_t c = 0; c < n; c++) {
        ym2[c] = u0[c];
        ym1[c] = u0[c] + mt[1] * L0[c];
    }
    for (int j = 2; j <= s; j++) {
        dtL(op, ym1, ay, Lj);
#pragma omp parallel for schedule(static)
        for (size_t c = 0; c < n; c++)
            yj[c] = mu[j] * ym1[c] + nu[j] * ym2[c] + (1.0 - mu[j] - nu[j]) * u0[c] + mt[j] * Lj[c] + gt[j] * L0[c];
        double *t = ym2;
        ym2 = ym1;
        ym1 = yj;
        yj = t;
    }
    memcpy(u1, ym1, sizeof(double) * n);
    free(mu), free(nu), free(mt), free(gt), free(L0), free(Lj), free(ay), free(ym2), free(ym1), free(yj);
    return 0;
}

/* ------------------------------------------------------------------ PC2: block-Jacobi ILU(0)
 * The paper's second preconditioner (Section 2.2): block-Jacobi whose blocks
 * (one per MPI rank in MAS) are factored by zero-fill incomplete LU (Saad,
 * Iterative Methods, ILU(0)).  Readings: the blocks are boxes of bi x bj x bk
 * cells (r, theta, phi) tiling the grid from index 0 (the last ones ragged);
 * couplings between blocks, and the periodic phi coupling between k = np-1
 * and k = 0, are left out of the factorization; cells are ordered naturally
 * (the cell index order).  A block is then a box with the 7-point graph, and
 * ILU(0) in natural order leaves A's off-diagonal entries as they are and
 * changes only the diagonal:
 *     d_c = A_cc - sum_{lower neighbours nb of c in its block} A_{c,nb}^2 / d_nb,
 * M = (D + L) D^-1 (D + U) with L, U the strict lower / upper parts of the
 * block-diagonal part of A.  Applying M^-1:
 *     forward   y_c = (r_c - sum_{nb < c} A_{c,nb} y_nb) / d_c
 *     backward  z_c = y_c - (sum_{nb > c} A_{c,nb} z_nb) / d_c.
 * A_{c,nb} = -c_f for the face f between c and nb.
 */
typedef struct {
    int bi, bj, bk;
} ora_blocks;

static int same_block(int a, int b, int bs) { return a / bs == b / bs; }

/* couplings to the lower neighbours (i-1, j, k), (i, j-1, k), (i, j, k-1) of
 * cell (i, j, k) inside its block; 0 where the neighbour is outside it */
static void lower_couplings(const ora_op *op, const ora_blocks *B, int i, int j, int k, double *cr_,
                            double *ct_, double *cp_) {
    const ora_grid *g = &op->g;
    *cr_ = (i > 0 && same_block(i - 1, i, B->bi)) ? op->cr[ridx(g, i, j, k)] : 0.0;
    *ct_ = (j > 0 && same_block(j - 1, j, B->bj)) ? op->ct[tidx(g, i, j, k)] : 0.0;
    *cp_ = (k > 0 && same_block(k - 1, k, B->bk)) ? op->cp[cidx(g, i, j, k - 1)] : 0.0;
}

void ora_pc2_factor(const ora_op *op, int bi, int bj, int bk, double *d) {
    const ora_grid *g = &op->g;
    ora_blocks B = {bi, bj, bk};
    /* the natural order visits every lower neighbour before the cell */
    for (int i = 0; i < g->nr; i++)
        for (int j = 0; j < g->nt; j++)
            for (int k = 0; k < g->np; k++) {
                double a, b, c;
                lower_couplings(op, &B, i, j, k, &a, &b, &c);
                const size_t cc = cidx(g, i, j, k);
                double s = op->diag[cc];
                if (a != 0.0) s -= a * a / d[cidx(g, i - 1, j, k)];
                if (b != 0.0) s -= b * b / d[cidx(g, i, j - 1, k)];
                if (c != 0.0) s -= c * c / d[cidx(g, i, j, k - 1)];
                d[cc] = s;
            }
}

void ora_pc2_apply(const ora_op *op, int bi, int bj, int bk, const double *d, const double *r,
                   double *z) {
    const ora_grid *g = &op->g;
    ora_blocks B = {bi, bj, bk};
    const size_t n = ncell(g);
    double *y = (double *)malloc(sizeof(double) * n);
    for (int i = 0; i < g->nr; i++)
        for (int j = 0; j < g->nt; j++)
            for (int k = 0; k < g->np; k++) {
                double a, b, c;
                lower_couplings(op, &B, i, j, k, &a, &b, &c);
                const size_t cc = cidx(g, i, j, k);
                double s = r[cc];
                if (a != 0.0) s += a * y[cidx(g, i - 1, j, k)];
                if (b != 0.0) s += b * y[cidx(g, i, j - 1, k)];
                if (c != 0.0) s += c * y[cidx(g, i, j, k - 1)];
                y[cc] = s / d[cc];
            }
    for (int i = g->nr - 1; i >= 0; i--)
        for (int j = g->nt - 1; j >= 0; j--)
            for (int k = g->np - 1; k >= 0; k--) {
                const size_t cc = cidx(g, i, j, k);
                double s = 0.0, a, b, c;
                /* upper neighbours: the cells whose lower neighbour c is */
                if (i + 1 < g->nr) {
                    lower_couplings(op, &B, i + 1, j, k, &a, &b, &c);
                    if (a != 0.0) s += a * z[cidx(g, i + 1, j, k)];
                }
                if (j + 1 < g->nt) {
                    lower_couplings(op, &B, i, j + 1, k, &a, &b, &c);
                    if (b != 0.0) s += b * z[cidx(g, i, j + 1, k)];
                }
                if (k + 1 < g->np) {
                    lower_couplings(op, &B, i, j, k + 1, &a, &b, &c);
                    if (c != 0.0) s += c * z[cidx(g, i, j, k + 1)];
                }
                z[cc] = y[cc] + s / d[cc];
            }
    free(y);
}

/* Preconditioned CG (the same steps as ora_pcg) with z = M^-1 r by PC2.
 * Returns the iteration count or -1 on breakdown. */
int ora_pcg_pc2(const ora_op *op, int bi, int bj, int bk, const double *b, double *x, double tol,
                int max_iters, int use_x0, double *stats, double *hist) {
    const ora_grid *g = &op->g;
    const size_t n = ncell(g);
    double *r = (double *)malloc(sizeof(double) * n);
    double *z = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    double *q = (double *)malloc(sizeof(double) * n);
    double *d = (double *)malloc(sizeof(double) * n);
    double *plane = (double *)malloc(sizeof(double) * g->nr);
    int it = 0, status = 0;

    ora_pc2_factor(op, bi, bj, bk, d);
    if (!use_x0) memset(x, 0, sizeof(double) * n);
    ora_apply(op, x, q);
    for (size_t c = 0; c < n; c++) r[c] = b[c] - q[c];
    ora_pc2_apply(op, bi, bj, bk, d, r, z);
    for (size_t c = 0; c < n; c++) p[c] = z[c];
    double bnorm = sqrt(dot(g, b, b, plane));
    if (bnorm == 0.0) bnorm = 1.0;
    double rz = dot(g, r, z, plane);
    double rnorm = sqrt(dot(g, r, r, plane));
    if (hist) hist[0] = rnorm / bnorm;

    while (rnorm > tol * bnorm && it < max_iters) {
        ora_apply(op, p, q);
        double pq = dot(g, p, q, plane);
        if (!(pq > 0.0) || !isfinite(pq)) {
            status = -1;
            break;
        }
        double alpha = rz / pq;
        for (size_t c = 0; c < n; c++) {
            x[c] += alpha * p[c];
            r[c] -= alpha * q[c];
        }
        it++;
        rnorm = sqrt(dot(g, r, r, plane));
        if (hist) hist[it] = rnorm / bnorm;
        if (rnorm <= tol * bnorm) break;
        ora_pc2_apply(op, bi, bj, bk, d, r, z);
        double rz_new = dot(g, r, z, plane);
        double beta = rz_new / rz;
        rz = rz_new;
        for (size_t c = 0; c < n; c++) p[c] = z[c] + beta * p[c];
    }
    if (stats) {
        stats[0] = rnorm / bnorm;
        ora_apply(op, x, q);
        for (size_t c = 0; c < n; c++) r[c] = b[c] - q[c];
        stats[1] = sqrt(dot(g, r, r, plane)) / bnorm;
    }
    free(r), free(z), free(p), free(q), free(d), free(plane);
    return status < 0 ? status : it;
}
