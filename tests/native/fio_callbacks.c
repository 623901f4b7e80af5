/*
 * Test-side phase and amplitude functions for FIO_PHASE_CALLBACK (fio_phase_fn and
 * fio_amp_fn of include/fio.h), written from the formulas of the paper's examples
 * (section 6): the tests build them into a shared library and pass their addresses to
 * fio_build, as a C user defining their own FIO would.
 *
 *   cb_phase_ex1    Phi = x xi + c(x)|xi|, c = (2 + sin 2 pi x)/c_div        (Example 1)
 *   cb_phase_radon  Phi = x.xi + sqrt(c1^2 xi1^2 + c2^2 xi2^2),
 *                   c1 = (2 + sin 2pi x1 sin 2pi x2)/c_div,
 *                   c2 = (2 + cos 2pi x1 cos 2pi x2)/c_div                   (Example 3)
 *   cb_amp_mixture  a = sum_k exp(-(d(x, x_k)^2 + (xi/n - eta_k)^2)/sigma2), d the
 *                   distance on the unit circle                              (Example 2)
 *   cb_phase_bad    returns NaN (error path)
 */
#include <math.h>

typedef struct {
    double c_div;
    int n;
    int terms;
    double sigma2;
    double cx[8], ce[8];
} cb_params;

static const double TWO_PI = 6.283185307179586476925286766559;

double cb_phase_ex1(const double *x, const double *xi, int d, void *user) {
    const cb_params *p = (const cb_params *)user;
    (void)d;
    const double c = (2.0 + sin(TWO_PI * x[0])) / p->c_div;
    return x[0] * xi[0] + c * fabs(xi[0]);
}

double cb_phase_radon(const double *x, const double *xi, int d, void *user) {
    const cb_params *p = (const cb_params *)user;
    (void)d;
    const double c1 = (2.0 + sin(TWO_PI * x[0]) * sin(TWO_PI * x[1])) / p->c_div;
    const double c2 = (2.0 + cos(TWO_PI * x[0]) * cos(TWO_PI * x[1])) / p->c_div;
    return x[0] * xi[0] + x[1] * xi[1] + sqrt(c1 * c1 * xi[0] * xi[0] + c2 * c2 * xi[1] * xi[1]);
}

void cb_amp_mixture(const double *x, const double *xi, int d, void *user, double re_im[2]) {
    const cb_params *p = (const cb_params *)user;
    (void)d;
    const double nu = xi[0] / (double)p->n;
    double a = 0.0;
    for (int k = 0; k < p->terms; ++k) {
        double dx = fabs(x[0] - p->cx[k]);
        dx = fmod(dx, 1.0);
        if (dx > 0.5) dx = 1.0 - dx;
        const double de = nu - p->ce[k];
        a += exp(-(dx * dx + de * de) / p->sigma2);
    }
    re_im[0] = a;
    re_im[1] = 0.0;
}

double cb_phase_bad(const double *x, const double *xi, int d, void *user) {
    (void)x;
    (void)xi;
    (void)d;
    (void)user;
    return NAN;
}
