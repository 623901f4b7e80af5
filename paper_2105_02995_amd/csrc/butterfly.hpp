// Butterfly factorization of K (section 2), built on the host in FP64.
//
// Trees T_X and T_Omega of depth L (fan F = 2^d, leaves of m points).  At level l
// the pairs (i, j) couple X node i at level l with Omega node j at level L - l
// (the complementary low-rank blocks K_{l;ij}).  This construction uses
// interpolative decompositions: on the X side, K_{l;ij} ~= P_{l;ij} K(s_{l;ij}, Omega_j)
// with skeleton rows s chosen among the children's skeletons, so P is nested
// (U_l = U_{l+1} C_l of eq_BFF_nested); on the Omega side, K_{l;ij} ~= K(X_i, t_{l;ij}) W_{l;ij}
// with W nested across levels (V_l = V_{l+1} H_l).  At the middle level lm the
// coupling block is D_{ij} = K(s_ij, t_ij), so
//     Kd = U_L C_{L-1} .. C_lm D H^*_lm .. H^*_1 V^*_L
// has L + 3 block-sparse factors, each with O(N) nonzeros (eq_BFF_fact).
#pragma once

#include <functional>

#include "fio_kernel.hpp"
#include "stages.hpp"

namespace fio {

// A batch of interpolative decompositions of sampled kernel blocks, all of one shape:
// matrix b is ns x nc with entry (s, c) = K(cand[b][c], samp[b][s]) when the
// candidates are X points (row skeletons of the X side, through the transpose), else
// K(samp[b][s], cand[b][c]) (column skeletons of the Omega side).  Positions are
// tree positions.  Column-pivoted QR selects the skeleton columns:
//  * rank mode (fixed_rank = 0): pivots until the next pivot column's norm is at most
//    tol_rel times the largest column norm, at most max_rank of them;
//  * ID mode (fixed_rank > 0): exactly min(fixed_rank, ns, nc) pivots, and the
//    interpolation matrix T = R11^{-1} R12 (k x (nc - k), column-major).
struct IdBatch {
    int64_t nb = 0;
    int ns = 0, nc = 0;
    bool cand_is_x = true;
    std::vector<int> samp, cand;   // nb x ns and nb x nc, row-major by matrix
    double tol_rel = 0;
    int max_rank = 0;
    int fixed_rank = 0;
};
// Receives matrix b's result: k pivots, perm (nc entries, skeletons first) and, in ID
// mode, T.  Called from several host threads at once for different b.
using IdSink = std::function<void(int64_t b, int k, const int *perm, const cd *T)>;
// Runs a batch; returns false (having called nothing) if the shape is not supported.
using BatchedId = std::function<bool(const IdBatch &, const IdSink &)>;
// Makes a batched-ID engine for the entries of one kernel (device tables are built once).
using BatchedIdFactory = std::function<BatchedId(const FioKernel &)>;
// The device engine (FP64 on the given HIP device).
BatchedIdFactory device_id_factory(int device);

struct ButterflyOptions {
    double eps = 1e-7;    // relative tolerance of every interpolative decomposition
    int leaf = 8;         // leaf side (points per dimension)
    int nthreads = 0;
    uint64_t seed = 1;    // column/row sampling
    int rank_align = 1;   // a level's rank may be cut down to a multiple of this ...
    double rank_slack = 4;  // ... when the probes need no more at rank_slack * eps
    bool verbose = false;
    BatchedId ids;        // empty: sample and decompose on the host
};

struct Butterfly {
    int d = 1, F = 2, L = 0, Lm = 0, m = 0;
    int64_t N = 0;
    std::vector<int> rU, rV;       // ranks per level (X side l = Lm..L, Omega side l = 0..Lm)
    std::vector<Stage> fwd;        // L + 3 stages: Omega tree order in -> X tree order out
    int device_levels = 0;         // levels whose decompositions ran on the batched engine
    int64_t nnz() const {
        int64_t s = 0;
        for (auto &st : fwd) s += st.nnz();
        return s;
    }
};

Butterfly build_butterfly(const FioKernel &K, const ButterflyOptions &opt);

}  // namespace fio
