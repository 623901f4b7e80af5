// Small dense complex linear algebra for the host-side (FP64) factor construction:
// products, Householder QR with column pivoting, interpolative decomposition,
// Cholesky and triangular inverses.  Column-major storage throughout.
#pragma once

#include <vector>

#include "common.hpp"

namespace fio {

struct Mat {
    int m = 0, n = 0;
    std::vector<cd> a;
    Mat() = default;
    Mat(int m_, int n_) : m(m_), n(n_), a((size_t)m_ * n_) {}
    cd &operator()(int i, int j) { return a[i + (size_t)j * m]; }
    const cd &operator()(int i, int j) const { return a[i + (size_t)j * m]; }
    cd *col(int j) { return a.data() + (size_t)j * m; }
    const cd *col(int j) const { return a.data() + (size_t)j * m; }
    static Mat eye(int k) {
        Mat I(k, k);
        for (int i = 0; i < k; ++i) I(i, i) = 1.0;
        return I;
    }
};

// C = op(A) op(B); op is 'N' (as is), 'T' (transpose) or 'C' (conjugate transpose).
Mat matmul(const Mat &A, const Mat &B, char opA = 'N', char opB = 'N');
// C += alpha op(A) op(B)
void gemm_acc(Mat &C, const Mat &A, const Mat &B, cd alpha, char opA = 'N', char opB = 'N');
Mat adj(const Mat &A);
Mat rows_of(const Mat &A, const std::vector<int> &rows);
Mat cols_of(const Mat &A, const std::vector<int> &cols);
double norm_fro(const Mat &A);

// Householder QR with column pivoting, A P = Q R.  A is overwritten: R in the upper
// triangle, reflectors below.  perm[j] is the original column at position j.
// Stops after max_rank steps or once the largest remaining column norm is <= tol_abs.
// Returns the number of steps (the numerical rank).
struct QRP {
    Mat A;                    // R and reflectors
    std::vector<int> perm;
    std::vector<cd> w0;       // leading entry of each reflector (others stored below diag)
    std::vector<double> wn2;  // squared norm of each reflector
    int rank = 0;
};
QRP cpqr(Mat A, double tol_abs, int max_rank);

// First k columns of Q from a cpqr result.
Mat qr_q(const QRP &f, int k);

// Interpolative decomposition of the columns of A (m x n):
//   A(:, redund) ~= A(:, skel) T,   T is k x (n - k).
// The rank is fixed_rank if > 0, else the number of pivots with
// |R_jj| > tol_rel |R_00| (capped by max_rank).
struct ColumnID {
    std::vector<int> skel, redund;
    Mat T;
};
ColumnID column_id(const Mat &A, double tol_rel, int fixed_rank, int max_rank);
// Numerical rank only (same criterion as column_id).
int id_rank(const Mat &A, double tol_rel, int max_rank);

// In-place lower Cholesky A = L L^*; returns false if a pivot is not positive.
bool cholesky_lower(Mat &A);
// Inverse of a lower triangular matrix.
Mat tri_lower_inverse(const Mat &L);
// Orthonormal basis of the range of Y, truncated where the pivoted QR diagonal
// falls to tol_abs (at most max_rank columns).
Mat orth(const Mat &Y, double tol_abs, int max_rank);
// Moore-Penrose pseudo-inverse of a matrix of full column rank (m >= n) or full
// row rank (m < n), via pivoted QR (rank-truncated at tol_rel).
Mat pinv(const Mat &A, double tol_rel = 1e-14);
// Hermitian positive definite inverse via Cholesky; false if not HPD.
bool hpd_inverse(const Mat &A, Mat &inv);
// Cholesky (lower, in place) of a Hermitian matrix that should be positive definite
// but may not be, because its approximation error exceeds its smallest eigenvalue:
// on failure A + delta I is factored instead, delta doubling from delta0.  Returns
// the shift used (0 if none) or -1 (failure, or delta0 <= 0 and A not HPD).
double cholesky_lower_shifted(Mat &A, double delta0);
// inv = (A + delta I)^{-1} with the shift of cholesky_lower_shifted; returns it (or -1).
double hpd_inverse_shifted(const Mat &A, Mat &inv, double delta0);

}  // namespace fio
