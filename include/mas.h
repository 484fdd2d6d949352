/*
 * mas.h -- C ABI of the MI355X (gfx950) implicit viscous-diffusion solver.
 *
 * The library solves the backward-Euler viscous step of a zero-beta MHD code
 * (the paper: Eq. (1), viscosity term div(nu grad v) with rho = 1; Section 2.2:
 * diffusive terms advanced implicitly by a preconditioned conjugate-gradient
 * solve with the inverse-diagonal "PC1" preconditioner; Section 4.1: the
 * matrices are symmetric with few off-diagonal entries)
 *
 *     (I - dt div(nu grad)) x = rhs
 *
 * for one scalar field on a non-uniform logically rectangular spherical-shell
 * grid (r, theta, phi): cells are the blocks between given radial and
 * colatitude faces, phi is uniform and periodic.  The finite-volume system is
 *
 *     A x = b,   b = V .* rhs,
 *     (A x)_c = V_c x_c + sum_{faces f of c} c_f (x_c - x_nb(f)),
 *     c_f = dt nu_f area_f / dist_f,
 *
 * with nu_f the mean of the two cells' nu (the cell's own nu on a Dirichlet
 * wall face), zero flux through the pole faces theta = 0 and pi, and either
 * x = 0 (Dirichlet) or zero flux (Neumann) on the radial walls.
 *
 * Conventions (every entry point):
 *   - Cell arrays are contiguous, length N = nr*nt*np, index
 *     (i*nt + j)*np + k with i = r, j = theta, k = phi (phi fastest).
 *   - "dev" pointers are device memory on the current HIP device; "host"
 *     pointers are host memory.  The library never allocates device memory:
 *     the caller supplies operator storage and solver workspace, sized by the
 *     *_bytes queries, and keeps them alive while they are in use.  The only
 *     host allocation is a small pinned status buffer per calling thread.
 *   - hip_stream is a hipStream_t (NULL = the null stream).  All device work
 *     is ordered on it.  Calls that return a solver result (build, solve,
 *     adjoint) block the calling thread until the result is known; the others
 *     only enqueue work.
 *   - Errors are returned as status codes (never thrown, never abort);
 *     mas_last_error() gives a message for the calling thread.
 */
#ifndef MAS_H
#define MAS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MAS_OK = 0,
    MAS_ENOTCONV = 1,    /* tolerance not reached within the limits; x holds the last iterate */
    MAS_EINVAL = -1,     /* bad argument: null pointer, size < 1, non-monotone faces, dt < 0,
                            nu <= 0 or not finite, precision not available in the operator */
    MAS_EBREAKDOWN = -2, /* (p, A p) <= 0 or not finite inside PCG */
    MAS_EHIP = -3,       /* a HIP runtime call failed */
    MAS_ENOMEM = -4      /* storage or workspace smaller than required */
};

enum { MAS_BC_DIRICHLET0 = 0, MAS_BC_NEUMANN0 = 1 };

/* MAS_FP64: all arithmetic in double precision.
 * MAS_FP32_REFINED: single-precision coefficients, operator apply,
 *   preconditioner and vector updates inside double-precision iterative
 *   refinement; residuals b - A x, the refinement update and every dot
 *   product are accumulated in double precision. */
enum { MAS_FP64 = 0, MAS_FP32_REFINED = 1 };

/* Refinement strategy of MAS_FP32_REFINED.  Both replace the single-precision
 * residual by the double-precision one, r = b - A x, whenever the inner
 * residual has dropped by inner_rtol (or far enough to meet rtol):
 *   MAS_REFINE_RESTART: classical iterative refinement; every inner solve
 *     starts a new conjugate-gradient run from the replaced residual.
 *   MAS_REFINE_RELIABLE: residual replacement; the inner run folds its
 *     pending step into x and continues from its current search direction,
 *     so the Krylov information is not thrown away at each refinement step. */
enum { MAS_REFINE_RESTART = 0, MAS_REFINE_RELIABLE = 1 };

typedef struct {
    int32_t nr, nt, np;       /* cells in r, theta, phi (each >= 1)                   */
    const double *r_faces;    /* host, nr+1, strictly increasing, r_faces[0] > 0       */
    const double *t_faces;    /* host, nt+1, strictly increasing, exactly 0 ... pi     */
    int32_t bc_inner;         /* MAS_BC_DIRICHLET0 | MAS_BC_NEUMANN0 at r_faces[0]      */
    int32_t bc_outer;         /* same at r_faces[nr]                                    */
} mas_grid;

/* Opaque operator: a small host struct pointing into caller storage. */
typedef struct mas_op mas_op;

typedef struct {
    double rtol;          /* stop when ||b - A x||_2 <= rtol ||b||_2               (1e-10) */
    int32_t max_iters;    /* PCG iterations (refined: total inner iterations)     (100000) */
    int32_t precision;    /* MAS_FP64 | MAS_FP32_REFINED                            (FP64) */
    double inner_rtol;    /* refined: drop of the inner (preconditioned) residual
                             between two double-precision residuals            (1e-5) */
    int32_t max_outer;    /* refined: double-precision residual replacements          (20) */
    int32_t check_every;  /* FP64: iterations between residual-norm checks (>= 1)      (8) */
    int32_t use_x0;       /* nonzero: x (or lambda) holds the initial guess            (0) */
    int32_t max_restarts; /* FP64: restarts from the true residual if the recursive
                             residual converged but the true one did not               (3) */
    int32_t sample_timing;/* nonzero: time a sample of PCG iteration kernels with HIP
                             events (reported in mas_pcg_info)                          (0) */
    int32_t refine;       /* refined: MAS_REFINE_RESTART | MAS_REFINE_RELIABLE   (RELIABLE) */
} mas_pcg_opts;

typedef struct {
    int32_t status;              /* the call's return value                                  */
    int32_t iters;               /* PCG iterations (refined: inner iteration kernels run)    */
    int32_t outer_iters;         /* refined: refinement steps taken; FP64: 0                  */
    int32_t restarts;            /* FP64: restarts taken                                      */
    double rel_resid_true;       /* ||b - A x||_2/||b||_2 at exit, double precision           */
    double rel_resid_recursive;  /* last recursively updated residual norm / ||b||            */
    double bnorm;                /* ||b||_2                                                   */
    double seconds;              /* host wall clock of the call                               */
    double iter_kernel_us;       /* mean duration of the sampled PCG iteration kernels (us)   */
    int32_t iter_kernel_samples; /* number of samples behind iter_kernel_us (0: not sampled) */
    int32_t pad_;
} mas_pcg_info;

/* Fill *o with the defaults shown above. */
void mas_pcg_default_opts(mas_pcg_opts *o);

/* Bytes of device storage mas_op_build needs for grid g and precision
 * (MAS_FP32_REFINED also stores single-precision coefficients).  Returns a
 * negative status for an invalid grid. */
int64_t mas_op_storage_bytes(const mas_grid *g, int32_t precision);

/* Assemble the operator A(nu, dt) of the system above into caller storage.
 *   g        host grid (read during the call only)
 *   nu       dev, N viscosity values, each > 0 and finite (read during the call only)
 *   dt       time step >= 0
 *   storage  dev, >= mas_op_storage_bytes(g, precision) bytes, 256-byte aligned;
 *            must outlive *op_out
 *   op_out   receives a new operator handle (free with mas_op_destroy)
 * Blocks until the build has finished (it validates nu on the device).
 * Errors: MAS_EINVAL, MAS_ENOMEM, MAS_EHIP. */
int mas_op_build(const mas_grid *g, const double *nu, double dt, int32_t precision,
                 void *storage, int64_t storage_bytes, void *hip_stream, mas_op **op_out);

/* Free the host handle (not the caller's storage).  NULL is ignored. */
void mas_op_destroy(mas_op *op);

/* y = A x (double precision), x and y dev, N each, distinct.  Enqueues only. */
int mas_op_apply(const mas_op *op, const double *x, double *y, void *hip_stream);

/* Write the operator's entries as the solver stores them (dev, N each; any
 * pointer may be NULL to skip it):
 *   cr[c] = -A(c, c+r)      coupling to the +r neighbour (0 on the last r plane)
 *   ct[c] = -A(c, c+theta)  coupling to the +theta neighbour (0 on the last theta row)
 *   cp[c] = -A(c, c+phi)    coupling to the +phi neighbour (periodic)
 *   diag[c] = A(c, c)
 * Enqueues only. */
int mas_op_export(const mas_op *op, double *cr, double *ct, double *cp, double *diag,
                  void *hip_stream);

/* Bytes of device workspace a solve with options o needs (o may be NULL for
 * the defaults).  The same size serves mas_pcg_solve_adjoint. */
int64_t mas_pcg_workspace_bytes(const mas_op *op, const mas_pcg_opts *o);

/* Solve A x = V .* rhs by point-Jacobi preconditioned CG (paper Section 2.2,
 * PC1), or by the single-precision PCG inside double-precision refinement.
 *   rhs   dev, N
 *   x     dev, N: initial guess on entry if o->use_x0, solution on exit
 *   work  dev, >= mas_pcg_workspace_bytes(op, o), 256-byte aligned
 *   info  host, may be NULL
 * Returns MAS_OK, MAS_ENOTCONV (x holds the last iterate), MAS_EBREAKDOWN,
 * MAS_EINVAL, MAS_ENOMEM or MAS_EHIP.  Blocks until the solve has finished. */
int mas_pcg_solve(const mas_op *op, const double *rhs, double *x, const mas_pcg_opts *o,
                  void *work, int64_t work_bytes, void *hip_stream, mas_pcg_info *info);

/* Reverse-mode derivative of a scalar L(x) through x = A(nu)^-1 (V .* rhs).
 * A is symmetric, so the adjoint is one more solve with the same operator:
 *   lambda = A^-1 gx
 *   g_rhs  = V .* lambda                                       (dL/drhs)
 *   g_nu_c = - sum_{faces f of c} (d c_f/d nu_c)(lambda_c - lambda_nb)(x_c - x_nb)
 *                                                              (dL/dnu)
 * with d c_f/d nu_c = dt area_f/(2 dist_f) on interior faces and
 * dt area_f/dist_f on Dirichlet walls (lambda_nb = x_nb = 0 there).
 *   x       dev, N: the forward solution
 *   gx      dev, N: dL/dx
 *   lambda, g_nu, g_rhs  dev, N outputs (g_rhs may be NULL); lambda is the
 *           initial guess if o->use_x0
 * Same options, workspace, blocking and status codes as mas_pcg_solve; the
 * tolerance applies to ||gx - A lambda|| / ||gx||. */
int mas_pcg_solve_adjoint(const mas_op *op, const double *x, const double *gx, double *lambda,
                          double *g_nu, double *g_rhs, const mas_pcg_opts *o, void *work,
                          int64_t work_bytes, void *hip_stream, mas_pcg_info *info);

/* Bandwidth probe: dst[0:bytes) = src[0:bytes), both dev, 16-byte aligned,
 * bytes a multiple of 16.  A plain streaming copy used to calibrate the HBM
 * byte counters.  Enqueues only. */
int mas_probe_copy(const void *src, void *dst, int64_t bytes, void *hip_stream);

/* Static description of a status code. */
const char *mas_status_string(int status);

/* Message for the last error on the calling thread ("" if none). */
const char *mas_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MAS_H */
