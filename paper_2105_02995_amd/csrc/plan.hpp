// The plan: host copies of the factors (for save/load) and their device images.
#pragma once

#include <string>

#include "butterfly.hpp"
#include "hif.hpp"

namespace fio {

// Host-side factor set: everything needed to reproduce the device images.
struct HostFactors {
    int d = 1, n = 0;
    int64_t N = 0;
    int L = 0, Lm = 0, m = 0;
    std::vector<int> perm;          // tree position -> natural index (X and Omega)
    std::vector<Stage> fwd;         // Kd stages (Omega tree order -> X tree order)
    HifFactors hif;                 // Gd factors (Omega tree order)
    fio_problem prob{};             // build description
    double build_seconds = 0;
    double bf_seconds = 0;          // butterfly construction (not stored in files)
    int bf_device_levels = 0;       // butterfly levels decomposed on the device
    // Probe of the butterfly error e_a: EA_VECS Gaussian vectors (Omega tree order,
    // column-major N x EA_VECS), EA_ROWS sampled X tree positions, and K v on those
    // rows summed from the entries of K in FP64.  Formed by the build (where the
    // phase is at hand) and compared with Kd v on the device.
    std::vector<int> ea_rows;
    std::vector<cd> ea_vecs, ea_ref;
    // Error estimates (0 until measured; see fio_plan_stats_t).
    double e_a_est = 0, e_s_est = 0, cond_est = 0;
};
constexpr int EA_ROWS = 64, EA_VECS = 4;

// Builds the factors; `gpu` (may be empty) replaces the host product Kd^* Kd of the
// peeling step, `ids` (may be empty) the host interpolative decompositions of the
// butterfly, `skel` (may be empty) the large dense work of the 2D skeletonization.
using PeelApplyFactory = std::function<BlockApply(const std::vector<Stage> &fwd)>;
void build_host_factors(const fio_problem &p, HostFactors &out, const PeelApplyFactory &gpu,
                        const BatchedIdFactory &ids, const SkelHooks &skel = SkelHooks());

// 64-bit fingerprints of the factors: the butterfly (permutation and every stage),
// each inverse-factor step, and the top-level inverse; equal for bit-identical factors.
std::vector<uint64_t> factor_fingerprints(const HostFactors &f);

void save_factors(const HostFactors &f, const std::string &path);
void load_factors(const std::string &path, HostFactors &f);

// Fills defaults of a problem description and validates it.
fio_problem normalized_problem(const fio_problem &p);

}  // namespace fio
