/* A solve through the C ABI from plain C (C99), with no Python in between:
 * a 16 x 24 x 48 spherical shell, uniform nu, dt = 1, a deterministic
 * right-hand side in [-1, 1).  Builds the operator in caller storage, sizes
 * the workspace, solves to the default tolerance in double precision and in
 * single precision inside double-precision refinement, checks the statuses
 * and reported residuals, and writes its inputs and both solutions to the
 * file named by argv[1] (doubles in host byte order: the nr + 1 radial and
 * nt + 1 polar faces, the N right-hand side values, the two solutions).  The
 * GPU test that runs it solves the same system through the Python binding
 * and against the oracle.  Built as a shared library exporting
 * c_api_solve_run (the test calls it in its own process: no child process
 * on a GPU already in use); with -DC_API_SOLVE_MAIN also as a program.
 * Returns 0 on success. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "mas.h"

enum { NR = 16, NT = 24, NP = 48 };
static const double kPi = 3.14159265358979323846; /* the double nearest pi */

#define HIP_OK(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));     \
            return 1;                                                             \
        }                                                                         \
    } while (0)

int c_api_solve_run(const char *path);

static int solve(const mas_op *op, const double *rhs_d, double *x_d, int precision,
                 double *x_host, int64_t n) {
    mas_pcg_opts o;
    mas_pcg_default_opts(&o);
    o.precision = precision;
    const int64_t wb = mas_pcg_workspace_bytes(op, &o);
    if (wb < 0) {
        fprintf(stderr, "workspace size: %s\n", mas_last_error());
        return 1;
    }
    void *work = NULL;
    HIP_OK(hipMalloc(&work, (size_t)wb));
    mas_pcg_info info;
    const int st = mas_pcg_solve(op, rhs_d, x_d, &o, work, wb, NULL, &info);
    HIP_OK(hipFree(work));
    printf("precision %d: %s, %d iterations (%d outer), relative residual %.3e, launch %d\n",
           precision, mas_status_string(st), info.iters, info.outer_iters, info.rel_resid_true,
           info.launch);
    if (st != MAS_OK || info.status != MAS_OK || !(info.rel_resid_true <= o.rtol)) {
        fprintf(stderr, "solve failed: %s\n", mas_last_error());
        return 1;
    }
    HIP_OK(hipMemcpy(x_host, x_d, (size_t)n * sizeof(double), hipMemcpyDeviceToHost));
    return 0;
}

int c_api_solve_run(const char *path) {
    const int64_t n = (int64_t)NR * NT * NP;
    double rf[NR + 1], tf[NT + 1];
    /* radial faces from 1 to 2.5, cell widths growing by 2% a cell */
    {
        double dr = 1.5 * (1.02 - 1.0) / (pow(1.02, NR) - 1.0), r = 1.0;
        for (int i = 0; i <= NR; ++i) {
            rf[i] = r;
            r += dr;
            dr *= 1.02;
        }
        rf[NR] = 2.5;
    }
    for (int j = 0; j <= NT; ++j) tf[j] = kPi * j / NT;
    tf[0] = 0.0;
    tf[NT] = kPi;
    const mas_grid g = {NR, NT, NP, rf, tf, MAS_BC_DIRICHLET0, MAS_BC_DIRICHLET0};

    double *nu = malloc((size_t)n * sizeof(double)), *rhs = malloc((size_t)n * sizeof(double));
    double *x = malloc((size_t)2 * n * sizeof(double));
    if (!nu || !rhs || !x) return 1;
    uint64_t s = 88172645463325252ull; /* xorshift64 */
    for (int64_t c = 0; c < n; ++c) {
        nu[c] = 1e-3;
        s ^= s << 13;
        s ^= s >> 7;
        s ^= s << 17;
        rhs[c] = (double)(s >> 11) / 9007199254740992.0 * 2.0 - 1.0;
    }

    double *nu_d = NULL, *rhs_d = NULL, *x_d = NULL;
    HIP_OK(hipMalloc((void **)&nu_d, (size_t)n * sizeof(double)));
    HIP_OK(hipMalloc((void **)&rhs_d, (size_t)n * sizeof(double)));
    HIP_OK(hipMalloc((void **)&x_d, (size_t)n * sizeof(double)));
    HIP_OK(hipMemcpy(nu_d, nu, (size_t)n * sizeof(double), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(rhs_d, rhs, (size_t)n * sizeof(double), hipMemcpyHostToDevice));

    const int64_t sb = mas_op_storage_bytes(&g, MAS_FP32_REFINED);
    if (sb < 0) {
        fprintf(stderr, "storage size: %s\n", mas_last_error());
        return 1;
    }
    void *storage = NULL;
    HIP_OK(hipMalloc(&storage, (size_t)sb));
    mas_op *op = NULL;
    if (mas_op_build(&g, nu_d, 1.0, MAS_FP32_REFINED, storage, sb, NULL, &op) != MAS_OK) {
        fprintf(stderr, "build: %s\n", mas_last_error());
        return 1;
    }
    if (solve(op, rhs_d, x_d, MAS_FP64, x, n) || solve(op, rhs_d, x_d, MAS_FP32_REFINED, x + n, n))
        return 1;
    mas_op_destroy(op);
    HIP_OK(hipFree(storage));
    HIP_OK(hipFree(x_d));
    HIP_OK(hipFree(rhs_d));
    HIP_OK(hipFree(nu_d));

    FILE *f = fopen(path, "wb");
    if (!f || fwrite(rf, sizeof(double), NR + 1, f) != NR + 1 ||
        fwrite(tf, sizeof(double), NT + 1, f) != NT + 1 ||
        fwrite(rhs, sizeof(double), (size_t)n, f) != (size_t)n ||
        fwrite(x, sizeof(double), (size_t)(2 * n), f) != (size_t)(2 * n) || fclose(f)) {
        fprintf(stderr, "cannot write %s\n", path);
        return 1;
    }
    free(x);
    free(rhs);
    free(nu);
    return 0;
}

#ifdef C_API_SOLVE_MAIN
int main(int argc, char **argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s <output file>\n", argv[0]);
        return 2;
    }
    return c_api_solve_run(argv[1]);
}
#endif
