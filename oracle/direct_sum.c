/*
 * Oracle (test infrastructure only): plain direct summation of the discrete
 * Fourier integral operator and of its adjoint, in double precision.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
 * this file.  The product library never links or calls it.
 *
 * What it computes (paper, section 1, equations eq3/eq6 and the grids
 * eq:X_domain / eq:freq_domain):
 *
 *   forward:  u(x_i)  = sum_j  a(x_i, xi_j) exp(2 pi i Phi(x_i, xi_j)) fhat(xi_j)
 *   adjoint:  v(xi_j) = sum_i  conj(a) exp(-2 pi i Phi(x_i, xi_j)) u(x_i)
 *
 * with a = 1 except for Example 2, x = (k_1..k_d)/n for 0 <= k < n and xi = (j_1..j_d) for
 * -n/2 <= j < n/2, points in lexicographic order with the first coordinate
 * slowest.  Phi = x.xi + phi(x, xi); the linear part is reduced exactly in
 * integers, ((sum_d k_d xi_d) mod n)/n, and phi is evaluated in double and
 * reduced mod 1 before the complex exponential.
 *
 * Phases (section 6):
 *   0  linear     phi = 0                                     (Phi = x.xi)
 *   1  1d_ex1     phi = c(x)|xi|, c(x) = (2 + sin 2 pi x)/param  (Example 1)
 *   2  2d_radon   phi = sqrt(c1^2 xi1^2 + c2^2 xi2^2),            (Example 3)
 *                 c1 = (2 + sin 2pi x1 sin 2pi x2)/param,
 *                 c2 = (2 + cos 2pi x1 cos 2pi x2)/param
 *   3  1d_const   phi = param |xi|   (constant c: K = N F^* diag(e^{2 pi i c|xi|}),
 *                 used only to pin this code against an FFT closed form)
 *   4  1d_ex2     Example 1's phi with the real amplitude (Example 2)
 *                 a(x, xi) = sum_k exp(-(d(x, x_k)^2 + (xi/n - eta_k)^2) / sigma2),
 *                 d the distance on the unit circle; amp = (x_0, eta_0, x_1, eta_1, ...)
 *
 * Vectors are complex, stored as interleaved (re, im) doubles, column-major
 * with leading dimension N for inputs and n_out for outputs.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double TWO_PI = 6.283185307179586476925286766559;

static double frac(double t) { return t - floor(t); }

/* Nonlinear part phi(x, xi) for point index p (X grid) and q (Omega grid). */
static double phi_nonlinear(int d, int n, int phase, double param, long long p, long long q)
{
    if (phase == 0) return 0.0;
    if (d == 1) {
        double x = (double)p / (double)n;
        double xi = (double)(q - n / 2);
        if (phase == 1 || phase == 4) return (2.0 + sin(TWO_PI * x)) / param * fabs(xi);
        if (phase == 3) return param * fabs(xi);
        return 0.0;
    }
    long long p1 = p / n, p2 = p % n;
    long long q1 = q / n, q2 = q % n;
    double x1 = (double)p1 / (double)n, x2 = (double)p2 / (double)n;
    double xi1 = (double)(q1 - n / 2), xi2 = (double)(q2 - n / 2);
    double c1 = (2.0 + sin(TWO_PI * x1) * sin(TWO_PI * x2)) / param;
    double c2 = (2.0 + cos(TWO_PI * x1) * cos(TWO_PI * x2)) / param;
    return sqrt(c1 * c1 * xi1 * xi1 + c2 * c2 * xi2 * xi2);
}

/* Exact (x.xi mod 1) * n as an integer in [0, n). */
static long long linear_mod(int d, int n, long long p, long long q)
{
    long long s;
    if (d == 1) {
        s = p * (q - n / 2);
    } else {
        long long p1 = p / n, p2 = p % n, q1 = q / n, q2 = q % n;
        s = p1 * (q1 - n / 2) + p2 * (q2 - n / 2);
    }
    s %= n;
    if (s < 0) s += n;
    return s;
}

/* Example 2's amplitude at X point p, Omega point q (1D). */
static double amplitude(int n, long long p, long long q, int nterms, const double *amp, double sigma2)
{
    double x = (double)p / (double)n, nu = (double)(q - n / 2) / (double)n, a = 0.0;
    for (int k = 0; k < nterms; ++k) {
        double dx = fmod(fabs(x - amp[2 * k]), 1.0);
        if (dx > 0.5) dx = 1.0 - dx;
        double de = nu - amp[2 * k + 1];
        a += exp(-(dx * dx + de * de) / sigma2);
    }
    return a;
}

/* Returns 0 on success, -1 on bad arguments. */
int oracle_fio_apply(int d, int n, int phase, double param, int adjoint, int nrhs,
                     const double *in, double *out, const long long *out_idx,
                     long long n_out, int nthreads, int amp_terms, const double *amp,
                     double sigma2)
{
    if ((d != 1 && d != 2) || n < 2 || (n % 2) || nrhs < 1) return -1;
    if (phase < 0 || phase > 4 || ((phase == 1 || phase == 3 || phase == 4) && d != 1) ||
        (phase == 2 && d != 2)) return -1;
    if (phase == 4 && (amp_terms < 1 || !amp || !(sigma2 > 0))) return -1;
    long long N = (d == 1) ? n : (long long)n * n;
    if (!out_idx) n_out = N;
    /* Input transposed to point-major (all right-hand sides of one point together). */
    double *tin = (double *)malloc(sizeof(double) * 2 * N * nrhs);
    if (!tin) return -1;
    for (long long j = 0; j < N; ++j)
        for (int r = 0; r < nrhs; ++r) {
            tin[2 * (j * nrhs + r)] = in[2 * (j + r * N)];
            tin[2 * (j * nrhs + r) + 1] = in[2 * (j + r * N) + 1];
        }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        double *acc = (double *)malloc(sizeof(double) * 2 * nrhs);
#pragma omp for schedule(dynamic, 4)
        for (long long o = 0; o < n_out; ++o) {
            long long a = out_idx ? out_idx[o] : o; /* output point */
            memset(acc, 0, sizeof(double) * 2 * nrhs);
            for (long long b = 0; b < N; ++b) {     /* summed point */
                long long p = adjoint ? b : a;      /* X index     */
                long long q = adjoint ? a : b;      /* Omega index */
                double theta = (double)linear_mod(d, n, p, q) / (double)n +
                               frac(phi_nonlinear(d, n, phase, param, p, q));
                theta = frac(theta);
                double c = cos(TWO_PI * theta), s = sin(TWO_PI * theta);
                if (phase == 4) {
                    double a = amplitude(n, p, q, amp_terms, amp, sigma2);
                    c *= a;
                    s *= a;
                }
                if (adjoint) s = -s;
                const double *v = tin + 2 * b * nrhs;
                for (int r = 0; r < nrhs; ++r) {
                    double vr = v[2 * r], vi = v[2 * r + 1];
                    acc[2 * r] += c * vr - s * vi;
                    acc[2 * r + 1] += c * vi + s * vr;
                }
            }
            for (int r = 0; r < nrhs; ++r) {
                out[2 * (o + r * n_out)] = acc[2 * r];
                out[2 * (o + r * n_out) + 1] = acc[2 * r + 1];
            }
        }
        free(acc);
    }
    free(tin);
    return 0;
}
