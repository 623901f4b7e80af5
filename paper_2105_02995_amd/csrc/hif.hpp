// Hierarchical representation of S = Kd^* Kd and its inverse factors.
//
// 1D (section 3, "peeling algorithm for 1D HODLR matrices"; section 4, "1D case"):
//   Sd = D + sum_l Ahat_l, each Ahat_l made of sibling blocks
//   A_{l;(2p+1)(2p)} ~= U_{l;2p+1} B_{l;p} U_{l;2p}^* (0-based node numbers),
//   and Gd = R_L .. R_1 A_0^{-1} R_1^* .. R_L^* (eqAinv_1d) from recursive
//   skeletonization: per node, an interpolative decomposition of the stacked
//   bases (eq_id, eq:ID_1d), the zeroing matrix Z (eq_sk) and a block
//   Gaussian elimination E (eq_sk_3).
//
// One node factor Z_I E_I acts on the redundant DOFs r (I-tilde) and skeleton
// DOFs s (I-hat) of a node:
//   apply of (Z E)^*:  x_r -= T^* x_s;  x_r = Linv x_r;  x_s -= M x_r
//   apply of  Z E   :  x_r = Linv^* (x_r - M^* x_s);  x_s -= T x_r
// with Atilde_rr = L L^* (Cholesky), Linv = L^{-1} and M = Atilde_sr L^{-*}.
#pragma once

#include <functional>

#include "la.hpp"

namespace fio {

struct HifNode {
    std::vector<int> idx_r, idx_s;  // global DOF indices (Omega tree order)
    Mat T;                          // ns x nr
    Mat Linv;                       // nr x nr, lower triangular
    Mat M;                          // ns x nr
};

struct HifStep {
    std::vector<HifNode> nodes;     // disjoint index sets: factors commute
};

struct HifFactors {
    int64_t N = 0;
    std::vector<HifStep> steps;     // R_L first (the order of the upward sweep)
    std::vector<int> root_idx;      // S_0
    Mat A0inv;                      // inverse of the top-level block on S_0 (FP64)
    int max_rank_h = 0;             // largest off-diagonal rank of Sd
    int shifted = 0;                // pivot blocks (and root) that needed a diagonal shift
    int device_ids = 0;             // interpolative decompositions done on the device (not stored)
    int device_nodes = 0;           // node factorizations (and root inverse) done on the device (not stored)
};

// y = A x for nrhs vectors stored point-major (entry (e, b) at e*nrhs + b).
using BlockApply = std::function<void(const cd *x, cd *y, int nrhs)>;

// Column ID of one large matrix (tall stacked bases of coarse 2D nodes) on a device;
// returns false (having done nothing) if it declines the shape.  Same contract as
// column_id(A, tol_rel, 0, -1).
// The device implementation reduces a tall A to its triangular factor first (which
// keeps every pivot), then runs the pivoted Householder steps, one launch for pivot
// and reflector and one for the trailing columns per step.
using BigIdFn = std::function<bool(const Mat &A, double tol_rel, ColumnID &out)>;

// Dense algebra of one large skeletonization node (eq_sk, eq_sk_3): from the blocks
// Arr, Asr, Ass of A_II on the redundant (r) and skeleton (s) DOFs and the ID's T,
// forms Atr = Arr - T^* Asr - Asr^* T + T^* Ass T (made Hermitian), its Cholesky
// factor L, Linv = L^{-1}, M = (Asr - Ass T) Linv^* and delta = -M M^*.  Returns
// false (outputs untouched) if it declines or Atr is not numerically HPD, so that the
// host path, which may shift the diagonal, takes the node.
using BigNodeFn = std::function<bool(const Mat &Arr, const Mat &Asr, const Mat &Ass, const Mat &T, Mat &Linv,
                                     Mat &M, Mat &delta)>;
// Inverse of one large Hermitian matrix (the top-level block A_0) by Cholesky:
// A^{-1} = L^{-*} L^{-1}.  Returns false (inv untouched) if it declines or A is not
// numerically HPD (the host path may then shift the diagonal).
using HpdInverseFn = std::function<bool(const Mat &A, Mat &inv)>;

// Device hooks of the 2D skeletonization (each may be empty: host).
struct SkelHooks {
    BigIdFn big_id;
    BigNodeFn big_node;
    HpdInverseFn hpd_inverse;
};
// The device implementations (rocBLAS GEMMs, rocSOLVER QR, Cholesky and triangular
// inverse, FP64; one device lane, a stream shared by the host threads one call at a
// time, so that builds are deterministic; a hook that runs out of device memory
// declines, and the host path takes the node).
SkelHooks device_skel_hooks(int device);

struct PeelOptions {
    double eps = 1e-6;      // relative tolerance (to ||S||_2) of the low-rank blocks
    int leaf = 64;          // leaf size (1D points) / leaf side (2D)
    int oversample = 10;    // c
    int k0 = 16;            // initial rank guess k
    uint64_t seed = 7;
    int nthreads = 0;
    bool verbose = false;
    // Pivot blocks that are not positive definite (the approximation error of Sd
    // exceeds their smallest eigenvalue) get a diagonal shift, from 1e-3 eps_hif ||S||_2
    // doubled until positive definite, when true; the build fails with
    // FIO_ERR_NOT_HPD when false.
    bool allow_shift = true;
    // 1D only: Cholesky-prescaled skeletonization (section 4, the alternative after
    // the 1D case): each node's diagonal block is first factored A_II = L L^* and the
    // node scaled by L^{-1}, the ID is taken on Ubar L^{-*}, and the elimination that
    // remains acts on I + T^* T.  Each level then has two steps: the scaling (a node
    // with only redundant DOFs and Linv = L^{-1}) and the skeletonization.
    bool prescale = false;
    // 2D: large column IDs, dense algebra of large nodes and the root inverse on a
    // device (empty hooks: host).
    SkelHooks dev;
};

// 1D HODLR peeling of a Hermitian operator given only by products (section 3),
// followed by recursive skeletonization (section 4) with tolerance eps_hif.
HifFactors build_hif_1d(const BlockApply &A, int64_t N, const PeelOptions &po, double eps_hif);

// 2D H-matrix peeling with strong admissibility and periodic neighbour lists
// (section 3) followed by cell and edge skeletonization (section 4, 2D case).
// n points per side; po.leaf is the side of the leaf cells.
HifFactors build_hif_2d(const BlockApply &A, int n, const PeelOptions &po, double eps_hif);

// Largest eigenvalue estimate of a Hermitian positive operator by power iteration.
double power_norm(const BlockApply &A, int64_t N, int iters, uint64_t seed);

}  // namespace fio
