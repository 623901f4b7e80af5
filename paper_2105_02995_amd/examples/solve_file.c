/*
 * fio_solve_file: the C ABI used from plain C (no Python, no torch).
 *
 *   fio_solve_file d n phase eps nrhs mode u.bin out.bin
 *
 * Builds the factors of the discrete FIO, reads u (complex128, column-major N x nrhs,
 * interleaved re/im) from u.bin, runs fio_solve on device 0 (mode 0 direct, 1
 * refinement with one FP64 step, 2 PCG, 3 GMRES; complex64 applies) and writes fhat to
 * out.bin in the same layout.  Device memory comes from the HIP runtime's C API.  Exit
 * status 0 on success.
 *
 * phase: 1 = 1D Example 1, 2 = 2D Example 3 (the library's built-in phases, c/16), or a
 * FIO this program defines itself through FIO_PHASE_CALLBACK (section 1, eq6: any
 * amplitude and phase):
 *   101  Phi = x xi + c(x)|xi|, c = (2 + sin 2 pi x)/16             (Example 1)
 *   102  Phi = x.xi + sqrt(c1^2 xi1^2 + c2^2 xi2^2)                  (Example 3)
 *   103  101's phase with a Gaussian-mixture amplitude a(x, xi)      (Example 2 shape:
 *        three terms at (x, xi/n) = (0.2, -0.2), (0.5, 0.2), (0.8, 0.0), sigma^2 = 0.1,
 *        x periodic)
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "fio.h"

static const double TWO_PI = 6.283185307179586476925286766559;

/* fio_phase_fn: the whole phase in cycles (the library reduces it mod 1). */
static double phase_ex1(const double *x, const double *xi, int d, void *user) {
    (void)d;
    (void)user;
    const double c = (2.0 + sin(TWO_PI * x[0])) / 16.0;
    return x[0] * xi[0] + c * fabs(xi[0]);
}

static double phase_radon(const double *x, const double *xi, int d, void *user) {
    (void)d;
    (void)user;
    const double c1 = (2.0 + sin(TWO_PI * x[0]) * sin(TWO_PI * x[1])) / 16.0;
    const double c2 = (2.0 + cos(TWO_PI * x[0]) * cos(TWO_PI * x[1])) / 16.0;
    return x[0] * xi[0] + x[1] * xi[1] + sqrt(c1 * c1 * xi[0] * xi[0] + c2 * c2 * xi[1] * xi[1]);
}

/* fio_amp_fn: user points at n (frequencies are scaled to xi/n). */
static void amp_mixture(const double *x, const double *xi, int d, void *user, double re_im[2]) {
    (void)d;
    static const double cx[3] = {0.2, 0.5, 0.8}, ce[3] = {-0.2, 0.2, 0.0};
    const double nu = xi[0] / (double)*(const int *)user;
    double a = 0.0;
    for (int k = 0; k < 3; ++k) {
        double dx = fabs(x[0] - cx[k]);
        if (dx > 0.5) dx = 1.0 - dx;
        const double de = nu - ce[k];
        a += exp(-(dx * dx + de * de) / 0.1);
    }
    re_im[0] = a;
    re_im[1] = 0.0;
}

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
    const int phase = atoi(argv[3]);
    p.phase = (fio_phase_id)phase;
    if (phase > 100) {
        p.phase = FIO_PHASE_CALLBACK;
        p.phi = phase == 102 ? phase_radon : phase_ex1;
        p.amp = phase == 103 ? amp_mixture : NULL;
        p.user = &p.n;
    }
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
    printf("solved N=%lld nrhs=%lld mode=%d: %d iterations, residual %.3e, estimated error %.3e\n",
           (long long)N, (long long)nrhs, mode, info.iters, info.rel_resid, info.est_rel_err);

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
