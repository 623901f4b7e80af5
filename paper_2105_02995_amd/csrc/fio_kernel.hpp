// Entries of the discrete FIO matrix K (section 1, eq6) for the phases of the
// numerical section (section 6), evaluated on the host in FP64.
//
// Points are addressed in "tree order": the order of the leaves of the dyadic
// tree (1D, identical to the natural order) or of a Z-order quadtree (2D), in
// which every tree node owns a contiguous range.  to_nat maps tree position to
// the natural (lexicographic, first coordinate slowest) index.
#pragma once

#include <cmath>
#include <vector>

#include "common.hpp"

namespace fio {

// Z-order position of (a, b) with a the slow coordinate: bits interleaved a1 b1 a0 b0.
inline int64_t morton2(int64_t a, int64_t b, int bits) {
    int64_t z = 0;
    for (int t = bits - 1; t >= 0; --t) z = (z << 2) | (((a >> t) & 1) << 1) | ((b >> t) & 1);
    return z;
}

struct FioKernel {
    int d = 1, n = 0;
    int64_t N = 0;
    fio_phase_id phase = FIO_PHASE_LINEAR;
    double c_div = 16.0;
    std::vector<int> to_nat;    // tree position -> natural index (same for X and Omega)
    std::vector<int> to_tree;   // natural index -> tree position
    std::vector<double> c1, c2; // per X point (tree order): c(x) (1D) or c1, c2 (2D)
    std::vector<int> k1, k2;    // per X point: integer coordinates
    std::vector<int> j1, j2;    // per Omega point: frequencies xi (-n/2 .. n/2-1)
    // Example 2's amplitude: each Gaussian term factors into g_k(x) h_k(xi), so
    // a(x_p, xi_q) = sum_k gx[k][p] hq[k][q] (tree order).
    std::vector<std::vector<double>> gx, hq;
    // A caller-defined FIO (FIO_PHASE_CALLBACK): the whole phase and the amplitude.
    fio_phase_fn phi_fn = nullptr;
    fio_amp_fn amp_fn = nullptr;
    void *user = nullptr;

    void init(const fio_problem &pr) {
        init(pr.d, pr.n, pr.phase, pr.c_div);
        if (pr.phase == FIO_PHASE_CALLBACK) {
            phi_fn = pr.phi;
            amp_fn = pr.amp;
            user = pr.user;
            return;
        }
        if (pr.phase != FIO_PHASE_1D_EX2) return;
        gx.assign(pr.amp_terms, std::vector<double>(N));
        hq.assign(pr.amp_terms, std::vector<double>(N));
        for (int k = 0; k < pr.amp_terms; ++k)
            for (int64_t t = 0; t < N; ++t) {
                double dx = std::fmod(std::fabs((double)k1[t] / n - pr.amp_x[k]), 1.0);
                if (dx > 0.5) dx = 1.0 - dx;
                const double de = (double)j1[t] / n - pr.amp_eta[k];
                gx[k][t] = std::exp(-dx * dx / pr.amp_sigma2);
                hq[k][t] = std::exp(-de * de / pr.amp_sigma2);
            }
    }

    void init(int d_, int n_, fio_phase_id ph, double cdiv) {
        d = d_; n = n_; phase = ph; c_div = cdiv;
        N = (d == 1) ? n : (int64_t)n * n;
        to_nat.resize(N); to_tree.resize(N);
        int bits = 0;
        while ((1 << bits) < n) ++bits;
        for (int64_t p = 0; p < N; ++p) {
            int64_t t = (d == 1) ? p : morton2(p / n, p % n, bits);
            to_tree[p] = (int)t;
            to_nat[t] = (int)p;
        }
        c1.assign(N, 0); c2.assign(N, 0);
        k1.assign(N, 0); k2.assign(N, 0); j1.assign(N, 0); j2.assign(N, 0);
        const double tp = 6.283185307179586476925286766559;
        for (int64_t t = 0; t < N; ++t) {
            int64_t p = to_nat[t];
            int a = (d == 1) ? (int)p : (int)(p / n);
            int b = (d == 1) ? 0 : (int)(p % n);
            k1[t] = a; k2[t] = b;
            j1[t] = a - n / 2; j2[t] = (d == 1) ? 0 : b - n / 2;
            double x1 = (double)a / n, x2 = (double)b / n;
            if (ph == FIO_PHASE_1D_EX1 || ph == FIO_PHASE_1D_EX2) {
                c1[t] = (2.0 + std::sin(tp * x1)) / cdiv;
            } else if (ph == FIO_PHASE_2D_RADON) {
                c1[t] = (2.0 + std::sin(tp * x1) * std::sin(tp * x2)) / cdiv;
                c2[t] = (2.0 + std::cos(tp * x1) * std::cos(tp * x2)) / cdiv;
            }
        }
    }

    // Phi(x_p, xi_q) mod 1 for tree positions p (X) and q (Omega).  The linear
    // part x.xi = (k.xi)/n is reduced exactly in integers.
    double phase_mod1(int64_t p, int64_t q) const {
        int64_t s = (int64_t)k1[p] * j1[q] + (int64_t)k2[p] * j2[q];
        s %= n;
        if (s < 0) s += n;
        double nl = 0.0;
        if (phase == FIO_PHASE_1D_EX1 || phase == FIO_PHASE_1D_EX2) {
            nl = c1[p] * std::fabs((double)j1[q]);
        } else if (phase == FIO_PHASE_2D_RADON) {
            double a = c1[p] * j1[q], b = c2[p] * j2[q];
            nl = std::sqrt(a * a + b * b);
        }
        double t = (double)s / n + (nl - std::floor(nl));
        return t - std::floor(t);
    }

    double amplitude(int64_t p, int64_t q) const {
        if (gx.empty()) return 1.0;
        double a = 0.0;
        for (size_t k = 0; k < gx.size(); ++k) a += gx[k][p] * hq[k][q];
        return a;
    }

    // K(x_p, xi_q) from the caller's functions: x = k/n, xi as given; the phase is
    // reduced mod 1 before the exponential.
    cd callback_entry(int64_t p, int64_t q) const {
        const double x[2] = {(double)k1[p] / n, (double)k2[p] / n};
        const double xi[2] = {(double)j1[q], (double)j2[q]};
        const double ph = phi_fn(x, xi, d, user);
        if (!std::isfinite(ph)) fail(FIO_ERR_ARG, "the phase callback returned a non-finite value");
        const double t = 6.283185307179586476925286766559 * (ph - std::floor(ph));
        cd e(std::cos(t), std::sin(t));
        if (amp_fn) {
            double ri[2] = {1.0, 0.0};
            amp_fn(x, xi, d, user, ri);
            if (!std::isfinite(ri[0]) || !std::isfinite(ri[1]))
                fail(FIO_ERR_ARG, "the amplitude callback returned a non-finite value");
            e *= cd(ri[0], ri[1]);
        }
        return e;
    }

    cd entry(int64_t p, int64_t q) const {
        if (phi_fn) return callback_entry(p, q);
        double t = 6.283185307179586476925286766559 * phase_mod1(p, q);
        return amplitude(p, q) * cd(std::cos(t), std::sin(t));
    }
};

}  // namespace fio
