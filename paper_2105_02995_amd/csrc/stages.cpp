#include "stages.hpp"

#include <algorithm>

namespace fio {

Stage adjoint_index(const Stage &s, std::vector<int64_t> &src_of) {
    Stage t;
    t.n_out = s.n_in;
    t.n_in = s.n_out;
    t.r_out = s.r_in;
    t.r_in = s.r_out;
    // Uses of every input block.
    std::vector<int32_t> count(s.n_in, 0);
    for (int64_t o = 0; o < s.n_out; ++o)
        for (int q = 0; q < s.fan; ++q) count[s.in_idx[o * s.fan + q]]++;
    int fan = s.n_in ? count[0] : 0;
    for (int32_t c : count)
        if (c != fan) fail(FIO_ERR_ARG, "adjoint_stage: non-uniform fan-out");
    t.fan = fan;
    t.in_idx.assign((size_t)t.n_out * fan, -1);
    // Slot sl of target block `in` takes the uses of `in` in source order.
    src_of.assign((size_t)t.n_out * fan, -1);
    std::vector<int32_t> slot(s.n_in, 0);
    for (int64_t o = 0; o < s.n_out; ++o)
        for (int q = 0; q < s.fan; ++q) {
            const int32_t in = s.in_idx[o * s.fan + q];
            const int sl = slot[in]++;
            t.in_idx[(size_t)in * fan + sl] = (int32_t)o;
            src_of[(size_t)in * fan + sl] = o * s.fan + q;
        }
    return t;
}

Stage adjoint_stage(const Stage &s) {
    std::vector<int64_t> src_of;
    Stage t = adjoint_index(s, src_of);
    const int fan = t.fan;
    t.A.resize((size_t)t.n_out * t.r_out * fan * t.r_in);
    const int64_t ldA = s.r_out;                   // leading dim of a source block
    const int64_t ldT = t.r_out;                   // leading dim of a target block
    // target blocks are disjoint: one task per block
    parallel_for(t.n_out, 0, [&](int64_t in) {
        cd *dst = t.A.data() + (size_t)in * t.block_elems();
        for (int sl = 0; sl < fan; ++sl) {
            const int64_t oq = src_of[(size_t)in * fan + sl];
            const int64_t o = oq / s.fan;
            const int q = (int)(oq - o * s.fan);
            const cd *src = s.A.data() + (size_t)o * s.block_elems();
            // target block (r_in x r_out) at column offset sl*r_out = conj transpose of
            // source block columns [q*r_in, (q+1)*r_in)
            for (int a = 0; a < s.r_out; ++a) {
                cd *d = dst + (int64_t)(sl * s.r_out + a) * ldT;
                const cd *sa = src + a + (int64_t)q * s.r_in * ldA;
                for (int b = 0; b < s.r_in; ++b) d[b] = std::conj(sa[(int64_t)b * ldA]);
            }
        }
    });
    return t;
}

void host_chain_apply(const std::vector<Stage> &chain, const cd *x, cd *y, int nrhs,
                      int nthreads) {
    std::vector<cd> cur, nxt;
    const int64_t n0 = chain.front().n_in * chain.front().r_in;
    cur.assign(x, x + n0 * nrhs);
    for (const Stage &s : chain) {
        nxt.assign((size_t)s.n_out * s.r_out * nrhs, cd(0));
        const int K = s.fan * s.r_in;
        parallel_for(s.n_out, nthreads, [&](int64_t o) {
            const cd *A = s.A.data() + (size_t)o * s.block_elems();
            cd *yo = nxt.data() + (size_t)o * s.r_out * nrhs;
            for (int kk = 0; kk < K; ++kk) {
                int q = kk / s.r_in, e = kk % s.r_in;
                const cd *xin = cur.data() +
                                ((size_t)s.in_idx[o * s.fan + q] * s.r_in + e) * nrhs;
                const cd *col = A + (size_t)kk * s.r_out;
                for (int a = 0; a < s.r_out; ++a) {
                    cd av = col[a];
                    cd *ya = yo + (size_t)a * nrhs;
                    for (int b = 0; b < nrhs; ++b) ya[b] += av * xin[b];
                }
            }
        });
        cur.swap(nxt);
    }
    std::copy(cur.begin(), cur.end(), y);
}

}  // namespace fio
