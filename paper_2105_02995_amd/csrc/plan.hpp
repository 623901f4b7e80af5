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
};

// Builds the factors; `gpu` (may be empty) replaces the host product Kd^* Kd of the
// peeling step, `ids` (may be empty) the host interpolative decompositions of the
// butterfly, `skel` (may be empty) the large dense work of the 2D skeletonization.
using PeelApplyFactory = std::function<BlockApply(const std::vector<Stage> &fwd)>;
void build_host_factors(const fio_problem &p, HostFactors &out, const PeelApplyFactory &gpu,
                        const BatchedIdFactory &ids, const SkelHooks &skel = SkelHooks());

void save_factors(const HostFactors &f, const std::string &path);
void load_factors(const std::string &path, HostFactors &f);

// Fills defaults of a problem description and validates it.
fio_problem normalized_problem(const fio_problem &p);

}  // namespace fio
