/*
 * fio_solve_file: the C ABI used from plain C (no Python, no torch).
 *
 *   fio_solve_file d n phase eps nrhs mode u.bin out.bin
 *
 * Builds the factors of the discrete FIO (phase: 1 = 1D Example 1, 2 = 2D Example 3,
 * c/16), reads u (complex128, column-major N x nrhs, interleaved re/im) from u.bin,
 * runs fio_solve on device 0 (mode 0 direct, 1 refinement with one FP64 step, 2 PCG,
 * 3 GMRES; complex64 applies) and writes fhat to out.bin in the same layout.  Device
 * memory comes from the HIP runtime's C API.  Exit status 0 on success.
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "fio.h"

#define CHECK_FIO(call)                                                                    \
    do {                                                                                   \
        fio_status s_ = (call);                                                            \
        if (s_ != FIO_OK) {                                                                \
            fprintf(stderr, "%s failed: %d (%s)\n", #call, (int)s_, fio_last_error());     \
            return 1;                                                                      \
        }                                                                                  \
    } while (0)
#define CHECK_HIP(call)                                                                    \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) {                                                            \
            fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));              \
            return 1;                                                                      \
        }                                                                                  \
    } while (0)

int main(int argc, char **argv) {
    if (argc != 9) {
        fprintf(stderr, "usage: %s d n phase eps nrhs mode u.bin out.bin\n", argv[0]);
        return 2;
    }
    fio_problem p;
    memset(&p, 0, sizeof(p));
    p.d = atoi(argv[1]);
    p.n = atoi(argv[2]);
    p.phase = (fio_phase_id)atoi(argv[3]);
    p.eps = atof(argv[4]);
    p.device = 0;
    const int64_t nrhs = atoll(argv[5]);
    const int mode = atoi(argv[6]);
    const int64_t N = p.d == 1 ? p.n : (int64_t)p.n * p.n;
    const size_t bytes = (size_t)N * nrhs * 2 * sizeof(double);

    double *host = (double *)malloc(bytes);
    FILE *f = fopen(argv[7], "rb");
    if (!host || !f || fread(host, 1, bytes, f) != bytes) {
        fprintf(stderr, "cannot read %s\n", argv[7]);
        return 1;
    }
    fclose(f);

    fio_plan plan;
    CHECK_FIO(fio_build(&p, &plan));
    void *du = NULL, *dx = NULL;
    CHECK_HIP(hipMalloc(&du, bytes));
    CHECK_HIP(hipMalloc(&dx, bytes));
    CHECK_HIP(hipMemcpy(du, host, bytes, hipMemcpyHostToDevice));

    fio_solve_opts o;
    memset(&o, 0, sizeof(o));
    o.mode = (fio_solve_mode)mode;
    o.maxit = mode == FIO_SOLVE_REFINE ? 1 : 30;
    o.tol = (mode == FIO_SOLVE_PCG || mode == FIO_SOLVE_GMRES) ? 1e-7 : 0.0;
    o.precondition = 1;
    fio_solve_info info;
    CHECK_FIO(fio_solve(plan, &o, FIO_C64, du, dx, nrhs, N, &info, NULL));
    CHECK_HIP(hipMemcpy(host, dx, bytes, hipMemcpyDeviceToHost));
    printf("solved N=%lld nrhs=%lld mode=%d: %d iterations, residual %.3e\n", (long long)N,
           (long long)nrhs, mode, info.iters, info.rel_resid);

    f = fopen(argv[8], "wb");
    if (!f || fwrite(host, 1, bytes, f) != bytes) {
        fprintf(stderr, "cannot write %s\n", argv[8]);
        return 1;
    }
    fclose(f);
    CHECK_HIP(hipFree(du));
    CHECK_HIP(hipFree(dx));
    fio_destroy(plan);
    free(host);
    return 0;
}
