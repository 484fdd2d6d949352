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
 *     (the explicit step included, unless it is asked to time itself) only
 *     enqueue work.
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

/* Preconditioner (the paper, Section 2.2).
 *   MAS_PC1: point Jacobi, the inverse diagonal (the GPU choice in the paper).
 *   MAS_PC2: block Jacobi with a zero-fill incomplete LU (ILU(0)) factor of
 *     each block.  Blocks are boxes of 8 r planes x 8 theta rows x 64 phi
 *     cells tiling the grid from index 0 (the last ones ragged); couplings
 *     between blocks and the periodic phi coupling are left out of the
 *     factors; cells are ordered naturally inside a block, so ILU(0) changes
 *     only the diagonal.  The factor is formed at the start of every solve.
 *     With MAS_FP32_REFINED the factor is the double-precision one rounded
 *     to single precision, the inner PC2-PCG runs in single precision, and
 *     every refinement step restarts it from the replaced residual
 *     (MAS_REFINE_RESTART whatever o->refine says). */
enum { MAS_PC1 = 0, MAS_PC2 = 1 };

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
    int32_t precond;      /* MAS_PC1 | MAS_PC2                                      (PC1) */
    int32_t chunk_planes; /* r planes each block of the PCG iteration kernel marches
                             through; 0: automatic (at least 16 and an eighth of nr,
                             fewer on grids too small to fill the GPU)             (0) */
    int32_t launch;       /* MAS_LAUNCH_AUTO | MAS_LAUNCH_PER_ITERATION |
                             MAS_LAUNCH_PERSISTENT                                  (AUTO) */
} mas_pcg_opts;

/* How a PC1 run (one to four right-hand sides) is launched.
 *   MAS_LAUNCH_PER_ITERATION: an iteration kernel and a one-block finalize per
 *     iteration, the host polling the run flags after each batch.
 *   MAS_LAUNCH_PERSISTENT: the whole run in one cooperative launch whose
 *     blocks are all resident at once, with a grid barrier per iteration and
 *     every block applying the same finalize (the same results bit for bit).
 *     Needs PC1, no sample_timing and a grid whose iteration kernel fits on
 *     the GPU at once (small grids, where launches and latency, not
 *     bandwidth, set the time); MAS_EINVAL otherwise.
 *     With chunk_planes = 0 its r chunks are long enough for about 64
 *     blocks; with the same chunk_planes both modes give the same results
 *     bit for bit (other chunks sum the partial dot products in another
 *     order).  Its blocks wait for each other at every iteration, at most
 *     2 s: if kernels of other streams keep part of its blocks from
 *     starting for longer, the call returns MAS_EHIP instead of hanging.
 *   MAS_LAUNCH_AUTO: persistent where it is possible and the grid has at
 *     most 2^17 cells, per iteration otherwise.
 * PC2 is always launched per iteration. */
enum { MAS_LAUNCH_AUTO = 0, MAS_LAUNCH_PER_ITERATION = 1, MAS_LAUNCH_PERSISTENT = 2 };

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
    int32_t launch;              /* how the last PC1 run was launched: MAS_LAUNCH_PER_ITERATION
                                    or MAS_LAUNCH_PERSISTENT (0: no PC1 run)                  */
    double grad_kernel_us;       /* mas_pcg_solve_adjoint with sample_timing: duration of the
                                    gradient kernel (us), HIP events; otherwise 0             */
} mas_pcg_info;

/* Fill *o with the defaults shown above. */
void mas_pcg_default_opts(mas_pcg_opts *o);

/* Bytes of device storage mas_op_build needs for grid g and precision
 * (MAS_FP32_REFINED also stores single-precision coefficients).  Returns a
 * negative status for an invalid grid. */
int64_t mas_op_storage_bytes(const mas_grid *g, int32_t precision);

/* Assemble the operator A(nu, dt) of the system above into caller storage
 * (with a copy of nu and the bound z_max that the explicit step uses).
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

/* Solve A x = V .* rhs by preconditioned CG (paper Section 2.2: PC1 or PC2),
 * in double precision or by the single-precision PCG inside double-precision
 * refinement.
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

/* ---------------------------------------------------------------- explicit viscous step
 * RKL2 super time-stepping: the explicit alternative to the implicit solve for
 * the viscous term (the paper, Section 2.2, cites the second-order
 * Runge-Kutta-Legendre scheme of Meyer, Balsara and Aslam, 2014; Section 3
 * reports about 200 such sub-steps per time step; Section 5.2 finds it the
 * faster choice on GPUs).  With the operator's nu and dt it advances
 *
 *     du/dt = L u,   dt L u = u - (A u) ./ V = -(1/V) sum_f c_f (u_c - u_nb)
 *
 * over one time step dt by s stages of the Legendre recursion
 *     Y_0 = u0,  Y_1 = Y_0 + mt_1 dtL(Y_0),
 *     Y_j = mu_j Y_{j-1} + nu_j Y_{j-2} + (1 - mu_j - nu_j) Y_0
 *           + mt_j dtL(Y_{j-1}) + gt_j dtL(Y_0),            j = 2..s,
 *     u1 = Y_s,
 * with w1 = 4/(s^2+s-2), b_0 = b_1 = b_2 = 1/3, b_j = (j^2+j-2)/(2j(j+1)),
 * mt_1 = b_1 w1, mu_j = (2j-1)/j b_j/b_{j-1}, nu_j = -(j-1)/j b_j/b_{j-2},
 * mt_j = mu_j w1, gt_j = -(1 - b_{j-1}) mt_j.  The step is second-order
 * accurate and stable while dt |lambda| <= (s^2+s-2)/2 for every eigenvalue
 * lambda of L; the automatic stage count bounds dt |lambda| by the Gershgorin
 * bound z_max = max_c 2 (A_cc - V_c)/V_c taken when the operator was built.
 * The operator may have been built in either precision; the step is always
 * double precision. */
typedef struct {
    int32_t stages;        /* 0: the smallest s >= 2 with (s^2+s-2)/2 >= z_max
                              (mas_sts_stages); else s in [2, 1000000], fewer
                              than the automatic count may be unstable          (0) */
    int32_t sample_timing; /* nonzero: time the step and a sample of its stage
                              kernels with HIP events and wait for completion    (0) */
    int32_t single_stage_kernels; /* nonzero: one stage per kernel.  Zero: for even
                              np, stages 2..s run two per kernel (the second
                              stage formed from the first on each tile plus a
                              two-cell overlap ring), equal bit for bit to one
                              stage per kernel                                   (0) */
    int32_t pad_;
} mas_sts_opts;

typedef struct {
    int32_t status;               /* the call's return value                             */
    int32_t stages;               /* stages run                                          */
    double z_max;                 /* Gershgorin bound of dt * spectral radius of L       */
    double step_us;               /* device time of the whole step (sample_timing only)  */
    double stage_kernel_us;       /* mean device time of the general stage kernels, each
                                     running stages_per_kernel stages (us), from one event
                                     pair around their back-to-back run                  */
    int32_t stage_kernel_samples; /* kernels behind stage_kernel_us (0: not timed)       */
    int32_t stages_per_kernel;    /* 2 when stages ran in pairs, else 1                  */
} mas_sts_info;

/* Fill *o with the defaults shown above. */
void mas_sts_default_opts(mas_sts_opts *o);

/* The automatic stage count for op's dt (>= 2), or a negative status:
 * MAS_EINVAL for a NULL op or a dt needing more than 1000000 stages. */
int32_t mas_sts_stages(const mas_op *op);

/* Bytes of device workspace mas_sts_step needs (five cell arrays). */
int64_t mas_sts_workspace_bytes(const mas_op *op);

/* One RKL2 step of dt: u1 = Y_s from u0 (both dev, N).  u1 may equal u0
 * (in-place step); neither may overlap the workspace.
 *   o     host, may be NULL for the defaults
 *   work  dev, >= mas_sts_workspace_bytes(op) bytes, 256-byte aligned
 *   info  host, may be NULL
 * Enqueues the kernels (dtL(u0), then stages 2..s, one or two per kernel) on
 * hip_stream and returns; with o->sample_timing it also waits for them.
 * Calls sharing one workspace must be ordered on one stream.  Returns MAS_OK,
 * MAS_EINVAL, MAS_ENOMEM or MAS_EHIP. */
int mas_sts_step(const mas_op *op, const double *u0, double *u1, const mas_sts_opts *o,
                 void *work, int64_t work_bytes, void *hip_stream, mas_sts_info *info);

/* ---------------------------------------------------------------- several right-hand sides
 * The paper's viscous operator acts on the three components of v (Eq. (1)),
 * and its semi-implicit solve has the same form (Section 2.2).  With the
 * components treated as scalar fields under one operator (the couplings the
 * vector Laplacian adds on curvilinear grids left out), the component solves
 * share A: one iteration kernel reads the operator's couplings once per cell
 * for all of them.  Each right-hand side keeps its own CG scalars, stopping
 * test and restarts, so the result equals nrhs separate FP64 solves up to
 * rounding (the iterations are the same; the dot products are summed in a
 * different blocking). */

/* Bytes of device workspace mas_pcg_solve_multi needs for nrhs right-hand
 * sides (1 <= nrhs <= 4).  Negative status on error. */
int64_t mas_pcg_multi_workspace_bytes(const mas_op *op, int32_t nrhs);

/* Solve A x_h = V .* rhs_h, h = 0..nrhs-1, by PCG in double precision with
 * o->precond: MAS_PC1 (Jacobi; one iteration kernel for all right-hand sides)
 * or MAS_PC2 (block-Jacobi ILU(0), the factor formed once for all; each PC2
 * iteration runs one direction/SpMV launch and one block-solve launch, each
 * carrying all right-hand sides with the operator read once per cell, and
 * gives each right-hand side the iterates of its single PC2 solve bit for
 * bit).
 *   nrhs  1..4
 *   rhs   dev, nrhs*N, right-hand side h at rhs + h*N
 *   x     dev, nrhs*N, same layout: initial guesses on entry if o->use_x0,
 *         solutions on exit
 *   o     host, may be NULL; o->precision must be MAS_FP64; rtol, max_iters,
 *         check_every, max_restarts, precond and sample_timing apply to
 *         every right-hand side
 *   work  dev, >= mas_pcg_multi_workspace_bytes(op, nrhs), 256-byte aligned
 *   info  host array of nrhs entries, may be NULL; entry h describes
 *         right-hand side h (iter_kernel_us is the shared kernel's time)
 * Returns MAS_OK when every right-hand side converged, else MAS_EBREAKDOWN or
 * MAS_ENOTCONV if any did not (see info[h].status), or MAS_EINVAL, MAS_ENOMEM,
 * MAS_EHIP.  Blocks until the solves have finished. */
int mas_pcg_solve_multi(const mas_op *op, int32_t nrhs, const double *rhs, double *x,
                        const mas_pcg_opts *o, void *work, int64_t work_bytes, void *hip_stream,
                        mas_pcg_info *info);

/* ---------------------------------------------------------------- allocation-free solve
 * For callers that cannot allocate device or pinned memory or create HIP
 * objects during a solve: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  The same solve as mas_pcg_solve (same
 * kernels, options, results and status codes), with its workspace taken from
 * a static device array of MAS_NOALLOC_WORK_BYTES inside the library (one per
 * GPU, held until the process ends) instead of a caller buffer; the host
 * reads the run flags with synchronous copies instead of a pinned buffer and
 * events.  It calls no hipMalloc, hipFree, hipHostMalloc or hipEventCreate.
 *   rhs, x, o, info  as for mas_pcg_solve; o->sample_timing must be 0
 * Returns MAS_ENOMEM when mas_pcg_workspace_bytes(op, o) exceeds
 * MAS_NOALLOC_WORK_BYTES (64 MiB: about 1.1M cells in double precision),
 * MAS_EINVAL for sample_timing; otherwise as mas_pcg_solve.  All calls on
 * one GPU share that GPU's array: calls that overlap in time on one GPU
 * (other host threads, other streams) race and must be serialised by the
 * caller.  Every value the solve reads from the array is written by the same
 * call first.  Blocks until the solve has finished. */
#define MAS_NOALLOC_WORK_BYTES (64LL * 1024 * 1024)
int mas_pcg_solve_noalloc(const mas_op *op, const double *rhs, double *x, const mas_pcg_opts *o,
                          void *hip_stream, mas_pcg_info *info);

/* Bandwidth probe: dst[0:bytes) = src[0:bytes), both dev, 16-byte aligned,
 * bytes a multiple of 16.  A plain streaming copy used to calibrate the HBM
 * byte counters.  Enqueues only. */
int mas_probe_copy(const void *src, void *dst, int64_t bytes, void *hip_stream);

/* Streaming probe with the byte mix of a stencil kernel: nin arrays of n
 * doubles read and nout written, each block walking one contiguous chunk of
 * every array as the marching kernels walk their r chunks, non-temporal
 * accesses, out_t = in_0 + ... + in_{nin-1} + t.  The arrays are laid out
 * in buf (dev, 256-byte aligned, >= mas_probe_stream_bytes(n, nin, nout))
 * with the library's stagger.  Supported mixes: 8/4 and 6/3 (the PCG
 * iteration kernel's launches with and without the x update), 7/4 (an
 * iteration that moves x every time), 6/1 (the FP64 residual), 2/2 (the
 * gradient kernel), 4/1 (an RKL2 stage), 1/1 (a copy); any other mix is
 * MAS_EINVAL.
 * It measures the bandwidth that access pattern reaches, the ceiling the
 * kernels are compared with beside the 8 TB/s peak.  Enqueues only.
 * Returns MAS_OK, MAS_EINVAL, MAS_ENOMEM or MAS_EHIP. */
int64_t mas_probe_stream_bytes(int64_t n, int32_t nin, int32_t nout);
int mas_probe_stream(void *buf, int64_t bytes, int64_t n, int32_t nin, int32_t nout,
                     void *hip_stream);

/* Static description of a status code. */
const char *mas_status_string(int status);

/* Message for the last error on the calling thread ("" if none). */
const char *mas_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MAS_H */
