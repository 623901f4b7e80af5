// Block-sparse stage: the common form of every butterfly factor (section 2,
// eq_BFF_fact: V_L^*, H_l^*, D, C_l, U_L and their adjoints).
//
// A stage maps an input coefficient vector made of n_in blocks of r_in entries to
// an output vector of n_out blocks of r_out entries:
//     y_o = sum_{t < fan} A_{o,t} x_{in_idx[o*fan + t]}.
// The fan blocks of output o are stored side by side as one column-major
// r_out x (fan*r_in) matrix, at offset o*r_out*fan*r_in of A.
#pragma once

#include <new>
#include <utility>
#include <vector>

#include "common.hpp"

namespace fio {

// Allocator whose resize() leaves new elements unwritten: the stage arrays (up to
// several GB) are then first written by the parallel loops that fill them, instead
// of being zeroed on one thread beforehand.  Only for element types that every
// filler overwrites completely (complex entries of the factor blocks).
template <class T> struct FillLaterAlloc : std::allocator<T> {
    template <class U> struct rebind {
        using other = FillLaterAlloc<U>;
    };
    FillLaterAlloc() = default;
    template <class U> FillLaterAlloc(const FillLaterAlloc<U> &) noexcept {}
    template <class U> void construct(U *) noexcept {}
    template <class U, class... Args> void construct(U *p, Args &&...args) {
        ::new ((void *)p) U(std::forward<Args>(args)...);
    }
};
using CVec = std::vector<cd, FillLaterAlloc<cd>>;

struct Stage {
    int64_t n_out = 0, n_in = 0;
    int r_out = 0, r_in = 0, fan = 0;
    std::vector<int32_t> in_idx;  // n_out * fan
    CVec A;                       // n_out * r_out * fan * r_in (resize leaves it unwritten)
    size_t block_elems() const { return (size_t)r_out * fan * r_in; }
    int64_t nnz() const { return (int64_t)n_out * r_out * fan * r_in; }
};

// Adjoint stage: maps y (n_out blocks) back to x (n_in blocks) with blocks A^*.
// Every input block must be used by the same number of outputs.
Stage adjoint_stage(const Stage &s);
// Its index part only (sizes and in_idx; A left empty).  src_of[in*fan + sl] =
// o*s.fan + q: target slot sl of block `in` is the conjugate transpose of column
// group q of source block o.
Stage adjoint_index(const Stage &s, std::vector<int64_t> &src_of);

// Host product of a stage chain on nrhs vectors stored point-major
// (entry (e, b) of a vector block at e*nrhs + b).  Used by the factor
// construction (peeling needs products with Kd and Kd^*), never by the
// library's apply entry points, which run on the GPU.
void host_chain_apply(const std::vector<Stage> &chain, const cd *x, cd *y, int nrhs,
                      int nthreads);

}  // namespace fio
