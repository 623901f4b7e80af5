#include "la.hpp"

#include <algorithm>
#include <cmath>

namespace fio {

static inline cd opget(const Mat &A, char op, int i, int j) {
    if (op == 'N') return A(i, j);
    if (op == 'T') return A(j, i);
    return std::conj(A(j, i));
}

void gemm_acc(Mat &C, const Mat &A, const Mat &B, cd alpha, char opA, char opB) {
    const int m = (opA == 'N') ? A.m : A.n;
    const int k = (opA == 'N') ? A.n : A.m;
    const int n = (opB == 'N') ? B.n : B.m;
    const int kb = (opB == 'N') ? B.m : B.n;
    if (k != kb || C.m != m || C.n != n) fail(FIO_ERR_ARG, "gemm: shape mismatch");
    const double work = (double)m * n * k;
    if (opA == 'N' && opB == 'N') {
        par_cols(n, work, [&](int64_t j) {
            cd *c = C.col((int)j);
            for (int p = 0; p < k; ++p) {
                cd b = alpha * B(p, (int)j);
                if (b == cd(0)) continue;
                const cd *a = A.col(p);
                for (int i = 0; i < m; ++i) c[i] += a[i] * b;
            }
        });
        return;
    }
    if (opA == 'C' && opB == 'N') {
        par_cols(n, work, [&](int64_t j) {
            for (int i = 0; i < m; ++i) {
                const cd *a = A.col(i);
                const cd *b = B.col((int)j);
                cd s = 0;
                for (int p = 0; p < k; ++p) s += std::conj(a[p]) * b[p];
                C(i, (int)j) += alpha * s;
            }
        });
        return;
    }
    if (opA == 'N' && (opB == 'C' || opB == 'T')) {
        // C(:, j) += alpha * sum_p A(:, p) op(B)(p, j), op(B)(p, j) = (conj) B(j, p)
        par_cols(n, work, [&](int64_t j) {
            cd *c = C.col((int)j);
            for (int p = 0; p < k; ++p) {
                const cd bj = B((int)j, p);
                const cd b = alpha * (opB == 'C' ? std::conj(bj) : bj);
                if (b == cd(0)) continue;
                const cd *a = A.col(p);
                for (int i = 0; i < m; ++i) c[i] += a[i] * b;
            }
        });
        return;
    }
    par_cols(n, work, [&](int64_t j) {
        for (int i = 0; i < m; ++i) {
            cd s = 0;
            for (int p = 0; p < k; ++p) s += opget(A, opA, i, p) * opget(B, opB, p, (int)j);
            C(i, (int)j) += alpha * s;
        }
    });
}

Mat matmul(const Mat &A, const Mat &B, char opA, char opB) {
    const int m = (opA == 'N') ? A.m : A.n;
    const int n = (opB == 'N') ? B.n : B.m;
    Mat C(m, n);
    gemm_acc(C, A, B, 1.0, opA, opB);
    return C;
}

Mat adj(const Mat &A) {
    Mat B(A.n, A.m);
    for (int j = 0; j < A.n; ++j)
        for (int i = 0; i < A.m; ++i) B(j, i) = std::conj(A(i, j));
    return B;
}

Mat rows_of(const Mat &A, const std::vector<int> &rows) {
    Mat B((int)rows.size(), A.n);
    for (int j = 0; j < A.n; ++j)
        for (size_t i = 0; i < rows.size(); ++i) B((int)i, j) = A(rows[i], j);
    return B;
}

Mat cols_of(const Mat &A, const std::vector<int> &cols) {
    Mat B(A.m, (int)cols.size());
    for (size_t j = 0; j < cols.size(); ++j)
        std::copy(A.col(cols[j]), A.col(cols[j]) + A.m, B.col((int)j));
    return B;
}

double norm_fro(const Mat &A) {
    double s = 0;
    for (const cd &v : A.a) s += std::norm(v);
    return std::sqrt(s);
}

QRP cpqr(Mat A, double tol_abs, int max_rank) {
    QRP f;
    const int m = A.m, n = A.n;
    const int kmax = std::min({m, n, max_rank < 0 ? n : max_rank});
    f.perm.resize(n);
    for (int j = 0; j < n; ++j) f.perm[j] = j;
    std::vector<double> nrm2(n), orig2(n);
    for (int j = 0; j < n; ++j) {
        double s = 0;
        const cd *c = A.col(j);
        for (int i = 0; i < m; ++i) s += std::norm(c[i]);
        nrm2[j] = orig2[j] = s;
    }
    int k = 0;
    for (; k < kmax; ++k) {
        int p = k;
        for (int j = k + 1; j < n; ++j)
            if (nrm2[j] > nrm2[p]) p = j;
        if (std::sqrt(std::max(nrm2[p], 0.0)) <= tol_abs) break;
        if (p != k) {
            std::swap_ranges(A.col(k), A.col(k) + m, A.col(p));
            std::swap(nrm2[k], nrm2[p]);
            std::swap(orig2[k], orig2[p]);
            std::swap(f.perm[k], f.perm[p]);
        }
        // Householder reflector H = I - 2 w w^* / (w^* w) mapping A(k:m, k) to -e^{i t}|x| e_1.
        cd *x = A.col(k) + k;
        double alpha = 0;
        for (int i = 0; i < m - k; ++i) alpha += std::norm(x[i]);
        alpha = std::sqrt(alpha);
        cd ph = (std::abs(x[0]) > 0) ? x[0] / std::abs(x[0]) : cd(1.0);
        cd w0 = x[0] + ph * alpha;
        double wn2 = std::norm(w0);
        for (int i = 1; i < m - k; ++i) wn2 += std::norm(x[i]);
        f.w0.push_back(w0);
        f.wn2.push_back(wn2);
        if (wn2 > 0) {
            par_cols(n - k - 1, 2.0 * (m - k) * (n - k - 1), [&](int64_t jj) {
                cd *v = A.col(k + 1 + (int)jj) + k;
                cd s = std::conj(w0) * v[0];
                for (int i = 1; i < m - k; ++i) s += std::conj(x[i]) * v[i];
                cd t = 2.0 * s / wn2;
                v[0] -= t * w0;
                for (int i = 1; i < m - k; ++i) v[i] -= t * x[i];
            });
        }
        x[0] = -ph * alpha;  // R_kk; x[1:] keeps the reflector tail
        for (int j = k + 1; j < n; ++j) {
            nrm2[j] -= std::norm(A(k, j));
            if (nrm2[j] <= 1e-10 * orig2[j]) {  // recompute after cancellation
                double s = 0;
                for (int i = k + 1; i < m; ++i) s += std::norm(A(i, j));
                nrm2[j] = orig2[j] = s;
            }
        }
    }
    f.rank = k;
    f.A = std::move(A);
    return f;
}

Mat qr_q(const QRP &f, int k) {
    const int m = f.A.m;
    Mat Q(m, k);
    for (int c = 0; c < k; ++c) Q(c, c) = 1.0;
    // columns of Q are independent: each applies the reflectors in turn
    par_cols(k, 2.0 * m * k * k, [&](int64_t c) {
        for (int r = k - 1; r >= 0; --r) {
            if (f.wn2[r] == 0) continue;
            const cd *tail = f.A.col(r) + r;  // tail[1:] are reflector entries
            cd *v = Q.col((int)c) + r;
            cd s = std::conj(f.w0[r]) * v[0];
            for (int i = 1; i < m - r; ++i) s += std::conj(tail[i]) * v[i];
            cd t = 2.0 * s / f.wn2[r];
            v[0] -= t * f.w0[r];
            for (int i = 1; i < m - r; ++i) v[i] -= t * tail[i];
        }
    });
    return Q;
}

static double max_col_norm(const Mat &A) {
    double mx = 0;
    for (int j = 0; j < A.n; ++j) {
        double s = 0;
        const cd *c = A.col(j);
        for (int i = 0; i < A.m; ++i) s += std::norm(c[i]);
        mx = std::max(mx, s);
    }
    return std::sqrt(mx);
}

int id_rank(const Mat &A, double tol_rel, int max_rank) {
    double mx = max_col_norm(A);
    if (mx == 0) return 0;
    QRP f = cpqr(A, tol_rel * mx, max_rank);
    return f.rank;
}

ColumnID column_id(const Mat &A, double tol_rel, int fixed_rank, int max_rank) {
    ColumnID out;
    const int n = A.n;
    double mx = max_col_norm(A);
    int cap = std::min(A.m, n);
    if (max_rank >= 0) cap = std::min(cap, max_rank);
    QRP f;
    if (fixed_rank > 0) {
        f = cpqr(A, -1.0, std::min(fixed_rank, cap));
    } else {
        f = cpqr(A, mx == 0 ? 1.0 : tol_rel * mx, cap);
    }
    const int k = f.rank;
    out.skel.assign(f.perm.begin(), f.perm.begin() + k);
    out.redund.assign(f.perm.begin() + k, f.perm.end());
    out.T = Mat(k, n - k);
    // T = R11^{-1} R12 by back substitution, column by column (independent columns;
    // column operations on R11 are contiguous).
    par_cols(n - k, (double)k * k * (n - k) / 2.0, [&](int64_t jj) {
        const int j = (int)jj;
        cd *t = out.T.col(j);
        const cd *r12 = f.A.col(k + j);
        for (int i = 0; i < k; ++i) t[i] = r12[i];
        for (int p = k - 1; p >= 0; --p) {
            t[p] /= f.A(p, p);
            const cd tp = t[p];
            const cd *rp = f.A.col(p);
            for (int i = 0; i < p; ++i) t[i] -= rp[i] * tp;
        }
    });
    return out;
}

bool cholesky_lower(Mat &A) {
    // right-looking, column by column: scale column j, then update the trailing
    // columns with contiguous column operations (parallel for large matrices)
    const int n = A.n;
    for (int j = 0; j < n; ++j) {
        const double d2 = A(j, j).real();
        if (!(d2 > 0)) return false;
        const double d = std::sqrt(d2);
        cd *cj = A.col(j);
        cj[j] = d;
        for (int i = j + 1; i < n; ++i) cj[i] /= d;
        par_cols(n - j - 1, (double)(n - j) * (n - j), [&](int64_t t) {
            const int c = j + 1 + (int)t;
            const cd f = std::conj(cj[c]);
            cd *cc = A.col(c);
            for (int i = c; i < n; ++i) cc[i] -= cj[i] * f;
        });
    }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < j; ++i) A(i, j) = 0;
    return true;
}

Mat tri_lower_inverse(const Mat &L) {
    // column c of L^{-1} solves L x = e_c; columns are independent
    const int n = L.n;
    Mat X(n, n);
    par_cols(n, (double)n * n * n / 6.0, [&](int64_t cc) {
        const int c = (int)cc;
        cd *x = X.col(c);
        x[c] = 1.0;
        for (int p = c; p < n; ++p) {
            x[p] /= L(p, p);
            const cd xp = x[p];
            const cd *lp = L.col(p);
            for (int i = p + 1; i < n; ++i) x[i] -= lp[i] * xp;
        }
    });
    return X;
}

Mat orth(const Mat &Y, double tol_abs, int max_rank) {
    QRP f = cpqr(Y, tol_abs, max_rank);
    return qr_q(f, f.rank);
}

Mat pinv(const Mat &A, double tol_rel) {
    if (A.m < A.n) return adj(pinv(adj(A), tol_rel));
    double mx = max_col_norm(A);
    QRP f = cpqr(A, mx == 0 ? 1.0 : tol_rel * mx, A.n);
    const int k = f.rank, n = A.n;
    Mat Q = qr_q(f, k);
    // A P ~= Q [R11 R12]; basic pseudo-inverse P [R11^{-1} Q^*; 0].
    Mat out(n, A.m);
    Mat QH = adj(Q);  // k x m
    for (int c = 0; c < A.m; ++c) {
        std::vector<cd> y(k);
        for (int i = k - 1; i >= 0; --i) {
            cd s = QH(i, c);
            for (int p = i + 1; p < k; ++p) s -= f.A(i, p) * y[p];
            y[i] = s / f.A(i, i);
        }
        for (int i = 0; i < k; ++i) out(f.perm[i], c) = y[i];
    }
    return out;
}

double cholesky_lower_shifted(Mat &A, double delta0) {
    Mat work = A;
    if (cholesky_lower(work)) {
        A = std::move(work);
        return 0.0;
    }
    if (!(delta0 > 0)) return -1.0;
    double delta = delta0;
    for (int t = 0; t < 60; ++t, delta *= 2) {
        work = A;
        for (int i = 0; i < work.n; ++i) work(i, i) += delta;
        if (cholesky_lower(work)) {
            A = std::move(work);
            return delta;
        }
    }
    return -1.0;
}

double hpd_inverse_shifted(const Mat &A, Mat &inv, double delta0) {
    Mat L = A;
    const double sh = cholesky_lower_shifted(L, delta0);
    if (sh < 0) return sh;
    Mat Li = tri_lower_inverse(L);
    inv = matmul(Li, Li, 'C', 'N');
    return sh;
}

bool hpd_inverse(const Mat &A, Mat &inv) {
    Mat L = A;
    if (!cholesky_lower(L)) return false;
    Mat Li = tri_lower_inverse(L);
    inv = matmul(Li, Li, 'C', 'N');
    return true;
}

}  // namespace fio
