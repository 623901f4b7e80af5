#include "butterfly.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <functional>

#include "la.hpp"

namespace fio {

static int64_t ipow(int64_t b, int e) {
    int64_t r = 1;
    while (e-- > 0) r *= b;
    return r;
}

// Sorted distinct sample of `count` positions of [lo, lo + size): one uniformly
// random position per equal stratum (all positions if count >= size).
static std::vector<int> stratified(int64_t lo, int64_t size, int count, uint64_t seed) {
    std::vector<int> out;
    if (count >= size) {
        out.resize(size);
        for (int64_t i = 0; i < size; ++i) out[i] = (int)(lo + i);
        return out;
    }
    out.resize(count);
    for (int s = 0; s < count; ++s) {
        int64_t a = size * s / count, b = size * (s + 1) / count;
        uint64_t h = splitmix64(seed ^ splitmix64((uint64_t)s + 0x51ED27ULL));
        out[s] = (int)(lo + a + (int64_t)(h % (uint64_t)(b - a)));
    }
    return out;
}

static int n_samples(int ncand, int64_t size) {
    return (int)std::min<int64_t>(size, std::max(ncand + ncand / 2 + 16, 32));
}

// Pairs whose interpolative decompositions set the rank of a level: a stratified
// subset of all pairs, plus every pair whose Omega node holds xi = 0 (where the
// phase |xi| or sqrt(...) has its kink and ranks peak).
static std::vector<int64_t> rank_probe_pairs(int64_t npairs, int64_t nOm, int64_t j0, uint64_t seed) {
    const int64_t want = 256;
    std::vector<int64_t> out;
    if (npairs <= 2 * want) {
        for (int64_t p = 0; p < npairs; ++p) out.push_back(p);
        return out;
    }
    for (int64_t s = 0; s < want; ++s) {
        int64_t a = npairs * s / want, b = npairs * (s + 1) / want;
        out.push_back(a + (int64_t)(splitmix64(seed + s) % (uint64_t)(b - a)));
    }
    for (int64_t i = 0; i < npairs / nOm; ++i) out.push_back(i * nOm + j0);
    std::sort(out.begin(), out.end());
    out.erase(std::unique(out.begin(), out.end()), out.end());
    return out;
}

// Sampled block of K: entry (s, c) = K(cand[c], samp[s]) if the candidates are X
// points (the transpose of the X-side block), else K(samp[s], cand[c]).
static Mat sample_block(const FioKernel &K, bool cand_is_x, const std::vector<int> &cand,
                        const std::vector<int> &samp) {
    Mat M((int)samp.size(), (int)cand.size());
    for (size_t c = 0; c < cand.size(); ++c)
        for (size_t s = 0; s < samp.size(); ++s)
            M((int)s, (int)c) = cand_is_x ? K.entry(cand[c], samp[s]) : K.entry(samp[s], cand[c]);
    return M;
}

// Interpolative decompositions of one level: the rank is the largest numerical rank
// over the probe pairs, then every pair is decomposed at that rank and handed to
// sink(pair, id).  Runs through the batched engine when there is one (which may
// decline a shape), else on the host.  on_rank(r) is called once the rank is known,
// before the first sink call.  Returns the rank; *dev tells where it ran.
template <class CandFn, class SampFn, class Sink, class RankFn>
static int level_ids(const FioKernel &K, const ButterflyOptions &opt, bool cand_is_x, int64_t npairs,
                     int ncand, int ns, const std::vector<int64_t> &probe, CandFn cand_of,
                     SampFn samp_of, Sink sink, bool *dev, RankFn on_rank) {
    const int nt = opt.nthreads;
    auto fill = [&](IdBatch &bt, int64_t nb, const std::function<int64_t(int64_t)> &pair_of) {
        bt.nb = nb;
        bt.ns = ns;
        bt.nc = ncand;
        bt.cand_is_x = cand_is_x;
        bt.samp.resize((size_t)nb * ns);
        bt.cand.resize((size_t)nb * ncand);
        parallel_for(nb, nt, [&](int64_t t) {
            const int64_t pr = pair_of(t);
            std::vector<int> c = cand_of(pr), sp = samp_of(pr);
            std::copy(c.begin(), c.end(), bt.cand.begin() + t * ncand);
            std::copy(sp.begin(), sp.end(), bt.samp.begin() + t * ns);
        });
    };
    // Largest numerical rank over the probe pairs at relative tolerance tol.
    auto probe_rank = [&](double tol) {
        int r = 0;
        if (*dev) {
            IdBatch bt;
            fill(bt, (int64_t)probe.size(), [&](int64_t t) { return probe[t]; });
            bt.tol_rel = tol;
            bt.max_rank = ncand;
            std::atomic<int> mx(0);
            *dev = opt.ids(bt, [&](int64_t, int k, const int *, const cd *) {
                int cur = mx.load();
                while (k > cur && !mx.compare_exchange_weak(cur, k)) {
                }
            });
            r = mx.load();
        }
        if (!*dev) {
            std::vector<int> ranks(probe.size());
            parallel_for((int64_t)probe.size(), nt, [&](int64_t t) {
                ranks[t] = id_rank(sample_block(K, cand_is_x, cand_of(probe[t]), samp_of(probe[t])), tol, ncand);
            });
            r = *std::max_element(ranks.begin(), ranks.end());
        }
        return std::min(ncand, std::max(1, r));
    };
    *dev = (bool)opt.ids;
    int r = probe_rank(opt.eps);
    // Rank alignment: a rank just above a multiple of the alignment leaves the last
    // matrix-core tile of every block mostly padding.  The rank is cut down to that
    // multiple when the probes need no more than it at rank_slack times the
    // tolerance, so the cut costs at most that factor in the level's ID residual.
    const int a = opt.rank_align;
    if (a > 1 && r > a && r % a) {
        const int ra = r / a * a;
        if (probe_rank(opt.eps * opt.rank_slack) <= ra) r = ra;
    }
    progress(opt.verbose, "  rank probe: %zu pairs, %d candidates, %d samples, rank %d", probe.size(), ncand, ns, r);
    on_rank(r);
    if (*dev) {
        IdBatch bt;
        fill(bt, npairs, [](int64_t t) { return t; });
        bt.fixed_rank = r;
        bt.max_rank = ncand;
        *dev = opt.ids(bt, [&](int64_t pr, int k, const int *perm, const cd *T) {
            ColumnID id;
            id.skel.assign(perm, perm + k);
            id.redund.assign(perm + k, perm + ncand);
            id.T = Mat(k, ncand - k);
            std::copy(T, T + (size_t)k * (ncand - k), id.T.a.begin());
            sink(pr, id);
        });
        progress(opt.verbose, "  IDs of %lld pairs done", (long long)npairs);
        if (*dev) return r;
    }
    parallel_for(npairs, nt, [&](int64_t pr) {
        sink(pr, column_id(sample_block(K, cand_is_x, cand_of(pr), samp_of(pr)), opt.eps, r, ncand));
    });
    return r;
}

Butterfly build_butterfly(const FioKernel &K, const ButterflyOptions &opt) {
    Butterfly B;
    B.d = K.d;
    B.F = 1 << K.d;
    B.N = K.N;
    const int F = B.F;
    B.m = (int)ipow(opt.leaf, K.d);
    if (B.m > B.N || B.N % B.m) fail(FIO_ERR_ARG, "butterfly leaf larger than the grid");
    int L = 0;
    while (ipow(F, L) * B.m < B.N) ++L;
    if (ipow(F, L) * B.m != B.N) fail(FIO_ERR_ARG, "grid is not a power of the tree fan");
    B.L = L;
    B.Lm = L / 2;
    const int Lm = B.Lm;
    const int64_t N = B.N;
    const int64_t npairs = ipow(F, L);
    B.rU.assign(L + 1, 0);
    B.rV.assign(L + 1, 0);
    B.fwd.assign(L + 3, Stage());
    const int nt = opt.nthreads;
    // tree position of xi = 0 (the Omega point with j = 0 in every coordinate)
    const int64_t xi0 = K.to_tree[(K.d == 1) ? K.n / 2 : (int64_t)(K.n / 2) * K.n + K.n / 2];

    // ---------------- X side: row skeletons, levels L down to Lm ----------------
    std::vector<std::vector<int>> skelU(L + 1);
    for (int l = L; l >= Lm; --l) {
        const int64_t nOm = ipow(F, L - l);       // Omega nodes at level L - l
        const int64_t szX = N / ipow(F, l);
        const int64_t szOm = N / nOm;
        const int rnext = (l < L) ? B.rU[l + 1] : 0;
        const int ncand = (l == L) ? (int)szX : F * rnext;
        auto candidates = [&](int64_t pr) {
            int64_t i = pr / nOm, j = pr % nOm;
            std::vector<int> c(ncand);
            if (l == L) {
                for (int t = 0; t < ncand; ++t) c[t] = (int)(i * szX + t);
            } else {
                const int64_t nOmN = nOm / F;
                for (int q = 0; q < F; ++q) {
                    const int *s = &skelU[l + 1][((F * i + q) * nOmN + j / F) * rnext];
                    std::copy(s, s + rnext, c.begin() + q * rnext);
                }
            }
            return c;
        };
        const int ns = (int)std::min<int64_t>(n_samples(ncand, N), szOm);
        auto samples = [&](int64_t pr) {
            int64_t j = pr % nOm;
            return stratified(j * szOm, szOm, ns, opt.seed ^ splitmix64(0xA000 + l) ^ (uint64_t)pr * 7919ULL);
        };
        const std::vector<int64_t> probe = rank_probe_pairs(npairs, nOm, xi0 / szOm, opt.seed ^ (0xC00 + l));
        std::vector<Mat> Q(npairs);
        std::vector<int> &sk = skelU[l];
        bool dev = false;
        const int r = level_ids(K, opt, true, npairs, ncand, ns, probe, candidates, samples,
                                [&](int64_t pr, const ColumnID &id) {
            // K(cand, :) ~= Q K(skel, :) with Q(skel_k, k) = 1 and Q(redund_t, k) = T(k, t).
            const int rr = B.rU[l];
            if ((int)id.skel.size() != rr) fail(FIO_ERR_ARG, "interpolative decomposition below the level rank");
            const std::vector<int> cand = candidates(pr);
            Mat q(ncand, rr);
            for (int k = 0; k < rr; ++k) {
                q(id.skel[k], k) = 1.0;
                sk[pr * rr + k] = cand[id.skel[k]];
            }
            for (size_t t = 0; t < id.redund.size(); ++t)
                for (int k = 0; k < rr; ++k) q(id.redund[t], k) = id.T(k, (int)t);
            Q[pr] = std::move(q);
        }, &dev, [&](int rank) { B.rU[l] = rank; sk.assign((size_t)npairs * rank, 0); });
        B.device_levels += dev ? 1 : 0;
        progress(opt.verbose, "butterfly X side level %d: rank %d (%s)", l, r, dev ? "device" : "host");
        if (l < L) skelU[l + 1].clear();
        Stage st;
        if (l == L) {
            // U_L: X leaf i <- pair (i, 0), an m x r block.
            st.n_out = npairs; st.n_in = npairs;
            st.r_out = (int)szX; st.r_in = r; st.fan = 1;
            st.in_idx.resize(npairs);
            st.A.resize((size_t)npairs * szX * r);
            parallel_for(npairs, nt, [&](int64_t i) {
                st.in_idx[i] = (int32_t)i;
                std::copy(Q[i].a.begin(), Q[i].a.end(), st.A.begin() + (size_t)i * szX * r);
            });
            B.fwd[L + 2] = std::move(st);
        } else {
            // C_l: pair (ih, jh) at level l+1 <- pairs (ih/F, F jh + q) at level l.
            const int64_t nOmN = nOm / F;
            st.n_out = npairs; st.n_in = npairs;
            st.r_out = rnext; st.r_in = r; st.fan = F;
            st.in_idx.resize(npairs * F);
            st.A.resize((size_t)npairs * rnext * F * r);  // every entry written below
            parallel_for(npairs, nt, [&](int64_t o) {
                int64_t ih = o / nOmN, jh = o % nOmN;
                int64_t i = ih / F, c = ih % F;
                cd *blk = st.A.data() + (size_t)o * rnext * F * r;
                for (int q = 0; q < F; ++q) {
                    int64_t in = i * nOm + F * jh + q;
                    st.in_idx[o * F + q] = (int32_t)in;
                    const Mat &Qi = Q[in];
                    for (int k = 0; k < r; ++k)
                        for (int a = 0; a < rnext; ++a)
                            blk[a + (size_t)(q * r + k) * rnext] = Qi((int)(c * rnext + a), k);
                }
            });
            B.fwd[l + 2] = std::move(st);
        }
    }

    // ---------------- Omega side: column skeletons, levels 0 up to Lm ----------------
    std::vector<std::vector<int>> skelV(L + 1);
    for (int l = 0; l <= Lm; ++l) {
        const int64_t nOm = ipow(F, L - l);
        const int64_t szX = N / ipow(F, l);
        const int rprev = (l > 0) ? B.rV[l - 1] : 0;
        const int ncand = (l == 0) ? B.m : F * rprev;
        auto candidates = [&](int64_t pr) {
            int64_t i = pr / nOm, j = pr % nOm;
            std::vector<int> c(ncand);
            if (l == 0) {
                for (int t = 0; t < ncand; ++t) c[t] = (int)(j * B.m + t);
            } else {
                const int64_t nOmP = nOm * F;
                for (int q = 0; q < F; ++q) {
                    const int *s = &skelV[l - 1][((i / F) * nOmP + F * j + q) * rprev];
                    std::copy(s, s + rprev, c.begin() + q * rprev);
                }
            }
            return c;
        };
        const int ns = (int)std::min<int64_t>(n_samples(ncand, N), szX);
        auto samples = [&](int64_t pr) {
            int64_t i = pr / nOm;
            return stratified(i * szX, szX, ns, opt.seed ^ splitmix64(0xB000 + l) ^ (uint64_t)pr * 104729ULL);
        };
        const int64_t szOmV = N / nOm;
        const std::vector<int64_t> probe = rank_probe_pairs(npairs, nOm, xi0 / szOmV, opt.seed ^ (0xD00 + l));
        std::vector<Mat> G(npairs);
        std::vector<int> &sk = skelV[l];
        bool dev = false;
        const int r = level_ids(K, opt, false, npairs, ncand, ns, probe, candidates, samples,
                                [&](int64_t pr, const ColumnID &id) {
            // K(:, cand) ~= K(:, skel) G with G(k, skel_k) = 1 and G(k, redund_t) = T(k, t).
            const int rr = B.rV[l];
            if ((int)id.skel.size() != rr) fail(FIO_ERR_ARG, "interpolative decomposition below the level rank");
            const std::vector<int> cand = candidates(pr);
            Mat g(rr, ncand);
            for (int k = 0; k < rr; ++k) {
                g(k, id.skel[k]) = 1.0;
                sk[pr * rr + k] = cand[id.skel[k]];
            }
            for (size_t t = 0; t < id.redund.size(); ++t)
                for (int k = 0; k < rr; ++k) g(k, id.redund[t]) = id.T(k, (int)t);
            G[pr] = std::move(g);
        }, &dev, [&](int rank) { B.rV[l] = rank; sk.assign((size_t)npairs * rank, 0); });
        B.device_levels += dev ? 1 : 0;
        progress(opt.verbose, "butterfly Omega side level %d: rank %d (%s)", l, r, dev ? "device" : "host");
        if (l > 0) skelV[l - 1].clear();
        Stage st;
        st.n_out = npairs; st.n_in = npairs;
        st.r_out = r;
        st.fan = (l == 0) ? 1 : F;
        st.r_in = (l == 0) ? B.m : rprev;
        st.in_idx.resize(npairs * st.fan);
        st.A.resize((size_t)npairs * r * ncand);
        const int64_t nOmP = nOm * F;
        parallel_for(npairs, nt, [&](int64_t o) {
            int64_t i = o / nOm, j = o % nOm;
            if (l == 0) {
                st.in_idx[o] = (int32_t)j;  // Omega leaf j
            } else {
                for (int q = 0; q < F; ++q)
                    st.in_idx[o * F + q] = (int32_t)((i / F) * nOmP + F * j + q);
            }
            std::copy(G[o].a.begin(), G[o].a.end(), st.A.begin() + (size_t)o * r * ncand);
        });
        B.fwd[l] = std::move(st);
    }

    // ---------------- middle level: D_ij = K(s_ij, t_ij) ----------------
    {
        const int ru = B.rU[Lm], rv = B.rV[Lm];
        Stage st;
        st.n_out = npairs; st.n_in = npairs;
        st.r_out = ru; st.r_in = rv; st.fan = 1;
        st.in_idx.resize(npairs);
        st.A.resize((size_t)npairs * ru * rv);
        parallel_for(npairs, nt, [&](int64_t o) {
            st.in_idx[o] = (int32_t)o;
            cd *blk = st.A.data() + (size_t)o * ru * rv;
            for (int b = 0; b < rv; ++b)
                for (int a = 0; a < ru; ++a)
                    blk[a + (size_t)b * ru] = K.entry(skelU[Lm][o * ru + a], skelV[Lm][o * rv + b]);
        });
        B.fwd[Lm + 1] = std::move(st);
    }
    return B;
}

}  // namespace fio
