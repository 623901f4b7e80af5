// 2D: H-matrix peeling with strong admissibility (section 3, "peeling algorithm
// for 2D H-matrix") and the hierarchical interpolative inverse with cell and edge
// skeletonization (section 4, "2D case", eq_sk_2d, ID_2d_bases, eqAinv_2d).
//
// DOFs are the Omega points in Z-order ("tree order"), so every quadtree cell at
// level l is a contiguous range and its Morton index is the prefix of the DOF index.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <map>
#include <cstring>
#include <mutex>
#include <set>
#include <unordered_map>

#include "hif.hpp"

namespace fio {

namespace {

struct Geo {
    int n = 0, bits = 0;  // n = 2^bits points per side
    int64_t N = 0;
    int Lh = 0;           // leaf level of the cell tree
    static int64_t inter(int64_t a, int64_t b, int nb) {
        int64_t z = 0;
        for (int t = nb - 1; t >= 0; --t) z = (z << 2) | (((a >> t) & 1) << 1) | ((b >> t) & 1);
        return z;
    }
    static void deinter(int64_t z, int nb, int &a, int &b) {
        a = b = 0;
        for (int t = 0; t < nb; ++t) {
            b |= (int)((z >> (2 * t)) & 1) << t;
            a |= (int)((z >> (2 * t + 1)) & 1) << t;
        }
    }
    int64_t cell_of(int64_t dof, int l) const { return dof >> (2 * (bits - l)); }
    int64_t cell_size(int l) const { return N >> (2 * l); }
    int64_t cell_id(int l, int ci, int cj) const {
        const int s = 1 << l;
        return inter(((ci % s) + s) % s, ((cj % s) + s) % s, l);
    }
    void cell_xy(int l, int64_t c, int &ci, int &cj) const { deinter(c, l, ci, cj); }
    void dof_xy(int64_t dof, int &a, int &b) const { deinter(dof, bits, a, b); }
    // neighbour list NL (periodic, including the cell itself)
    std::vector<int64_t> NL(int l, int64_t c) const {
        int ci, cj;
        cell_xy(l, c, ci, cj);
        std::set<int64_t> s;
        for (int di = -1; di <= 1; ++di)
            for (int dj = -1; dj <= 1; ++dj) s.insert(cell_id(l, ci + di, cj + dj));
        return std::vector<int64_t>(s.begin(), s.end());
    }
    bool adjacent(int l, int64_t a, int64_t b) const {
        int ai, aj, bi, bj;
        cell_xy(l, a, ai, aj);
        cell_xy(l, b, bi, bj);
        const int s = 1 << l;
        int di = ((ai - bi) % s + s) % s, dj = ((aj - bj) % s + s) % s;
        return (di <= 1 || di == s - 1) && (dj <= 1 || dj == s - 1);
    }
    // interaction list IL: children of NL(parent) that are not in NL(c)
    std::vector<int64_t> IL(int l, int64_t c) const {
        std::vector<int64_t> out;
        if (l < 1) return out;
        std::set<int64_t> kids;
        for (int64_t p : NL(l - 1, c >> 2))
            for (int q = 0; q < 4; ++q) kids.insert(p * 4 + q);
        for (int64_t k : kids)
            if (!adjacent(l, c, k)) out.push_back(k);
        return out;
    }
};

// A(J, I) ~= UJ B UI^*  for an admissible pair (I, J), J in IL(I), stored once with I < J.
struct LR {
    int64_t I = 0, J = 0;
    Mat UI, UJ, B;
};

struct Hmat2D {
    Geo g;
    std::vector<std::vector<LR>> lr;                        // per level
    std::vector<std::unordered_map<int64_t, int>> pairidx;  // per level: key I*ncells+J -> index
    std::map<std::pair<int64_t, int64_t>, Mat> near;        // leaf level: (J, I) -> A(J, I), J in NL(I)
    int max_rank = 0;

    const LR *find(int l, int64_t a, int64_t b, bool &swapped) const {
        const int64_t nc = (int64_t)1 << (2 * l);
        auto it = pairidx[l].find(std::min(a, b) * nc + std::max(a, b));
        if (it == pairidx[l].end()) return nullptr;
        const LR &p = lr[l][it->second];
        swapped = (p.I != b);  // stored A(p.J, p.I); requested A(a rows, b cols)
        return &p;
    }

    // Dense A_H(rows, cols) of the H-matrix representation.
    Mat sub(const std::vector<int> &rows, const std::vector<int> &cols) const {
        Mat out((int)rows.size(), (int)cols.size());
        if (rows.empty() || cols.empty()) return out;
        const int L = g.Lh;
        // group by leaf cells
        std::map<int64_t, std::vector<int>> rg, cg;
        for (size_t i = 0; i < rows.size(); ++i) rg[g.cell_of(rows[i], L)].push_back((int)i);
        for (size_t j = 0; j < cols.size(); ++j) cg[g.cell_of(cols[j], L)].push_back((int)j);
        const int64_t leafsz = g.cell_size(L);
        for (auto &rc : rg) {
            for (auto &cc : cg) {
                const int64_t a = rc.first, b = cc.first;
                if (g.adjacent(L, a, b)) {
                    const Mat &blk = near.at({a, b});
                    for (int i : rc.second)
                        for (int j : cc.second)
                            out(i, j) = blk((int)(rows[i] - a * leafsz), (int)(cols[j] - b * leafsz));
                    continue;
                }
                // coarsest level at which the ancestors are not adjacent
                int l = L;
                while (l > 1 && !g.adjacent(l - 1, a >> (2 * (L - l + 1)), b >> (2 * (L - l + 1)))) --l;
                const int64_t A_ = a >> (2 * (L - l)), B_ = b >> (2 * (L - l));
                bool sw = false;
                const LR *p = find(l, A_, B_, sw);
                if (!p) fail(FIO_ERR_ARG, "H-matrix: missing admissible block");
                const int64_t csz = g.cell_size(l);
                // rows live in cell A_, columns in cell B_
                const Mat &Ur = sw ? p->UI : p->UJ;  // basis on the row cell
                const Mat &Uc = sw ? p->UJ : p->UI;  // basis on the column cell
                std::vector<int> rr, cc2;
                for (int i : rc.second) rr.push_back((int)(rows[i] - A_ * csz));
                for (int j : cc.second) cc2.push_back((int)(cols[j] - B_ * csz));
                Mat Ursub = rows_of(Ur, rr), Ucsub = rows_of(Uc, cc2);
                Mat mid = sw ? adj(p->B) : p->B;
                Mat blk = matmul(matmul(Ursub, mid), Ucsub, 'N', 'C');
                for (size_t i = 0; i < rc.second.size(); ++i)
                    for (size_t j = 0; j < cc.second.size(); ++j) out(rc.second[i], cc.second[j]) = blk((int)i, (int)j);
            }
        }
        return out;
    }
};

// Point-major N x s block helpers.
Mat take(const std::vector<cd> &X, int s, int64_t start, int64_t sz, int c0, int nc) {
    Mat R((int)sz, nc);
    for (int64_t i = 0; i < sz; ++i)
        for (int c = 0; c < nc; ++c) R((int)i, c) = X[(start + i) * s + c0 + c];
    return R;
}

// out -= sum over levels < upto of the admissible blocks applied to X (all columns).
void subtract_lr(const Hmat2D &H, int upto, const std::vector<cd> &X, std::vector<cd> &out, int s,
                 int nthreads) {
    std::mutex mu;
    for (int l = 1; l < upto; ++l) {
        const int64_t csz = H.g.cell_size(l);
        const auto &pairs = H.lr[l];
        // accumulate per cell to avoid races: collect contributions then add under a lock per level
        std::vector<std::vector<std::pair<int64_t, Mat>>> contrib(pairs.size());
        parallel_for((int64_t)pairs.size(), nthreads, [&](int64_t k) {
            const LR &p = pairs[k];
            if (p.UI.n == 0 || p.UJ.n == 0) return;
            Mat XI = take(X, s, p.I * csz, csz, 0, s), XJ = take(X, s, p.J * csz, csz, 0, s);
            Mat yJ = matmul(p.UJ, matmul(p.B, matmul(p.UI, XI, 'C', 'N')));
            Mat yI = matmul(p.UI, matmul(p.B, matmul(p.UJ, XJ, 'C', 'N'), 'C', 'N'));
            contrib[k].emplace_back(p.J, std::move(yJ));
            contrib[k].emplace_back(p.I, std::move(yI));
        });
        for (auto &cv : contrib)
            for (auto &pr : cv) {
                const int64_t st = pr.first * csz;
                for (int64_t i = 0; i < csz; ++i)
                    for (int c = 0; c < s; ++c) out[(st + i) * s + c] -= pr.second((int)i, c);
            }
    }
}

Hmat2D peel_2d(const BlockApply &A, const Geo &g, const PeelOptions &po, double normS) {
    Hmat2D H;
    H.g = g;
    const int L = g.Lh;
    H.lr.resize(L + 1);
    H.pairidx.resize(L + 1);
    const int c = po.oversample;
    const int64_t N = g.N;
    for (int l = 2; l <= L; ++l) {
        const int side = 1 << l;
        const int stride = std::min(8, side);  // 64 probe classes P_pq (eq_spq)
        const int64_t ncell = (int64_t)side * side;
        const int64_t csz = g.cell_size(l);
        // admissible pairs of this level, stored once (I < J)
        std::vector<LR> pairs;
        for (int64_t I = 0; I < ncell; ++I)
            for (int64_t J : g.IL(l, I))
                if (I < J) {
                    LR p;
                    p.I = I;
                    p.J = J;
                    pairs.push_back(std::move(p));
                }
        int k = (int)std::min<int64_t>(po.k0, csz);
        for (int attempt = 0;; ++attempt) {
            const int s = (int)std::min<int64_t>(k + c, csz);
            // Y[(I -> J)] = A(J, I) R_I for every ordered admissible pair
            std::map<std::pair<int64_t, int64_t>, Mat> Ysamp;
            std::vector<Mat> Rcell(ncell);
            const uint64_t sd = po.seed ^ splitmix64(0x2D00 + 64 * l + attempt);
            parallel_for(ncell, po.nthreads, [&](int64_t I) {
                Mat R((int)csz, s);
                for (int64_t i = 0; i < csz; ++i)
                    for (int q = 0; q < s; ++q) {
                        uint64_t ctr = (((uint64_t)I * csz + i) * s + q) * 2;
                        R((int)i, q) = cd(gauss(sd, ctr), gauss(sd, ctr + 1));
                    }
                Rcell[I] = std::move(R);
            });
            // classes batched into applies of at most ~512 columns
            std::vector<std::pair<int, int>> classes;
            for (int p = 0; p < stride; ++p)
                for (int q = 0; q < stride; ++q) classes.push_back({p, q});
            const int per_apply = std::max(1, 512 / s);
            for (size_t c0 = 0; c0 < classes.size(); c0 += per_apply) {
                const int nclass = (int)std::min<size_t>(per_apply, classes.size() - c0);
                const int S = nclass * s;
                std::vector<cd> R((size_t)N * S, cd(0)), Y((size_t)N * S);
                std::vector<std::vector<int64_t>> members(nclass);
                std::vector<std::pair<int, int64_t>> tI;  // (class, cell) pairs of this apply
                for (int t = 0; t < nclass; ++t) {
                    auto [p, q] = classes[c0 + t];
                    for (int ci = p; ci < side; ci += stride)
                        for (int cj = q; cj < side; cj += stride) {
                            members[t].push_back(g.cell_id(l, ci, cj));
                            tI.push_back({t, members[t].back()});
                        }
                }
                // the cells of one apply are distinct: disjoint rows of R
                parallel_for((int64_t)tI.size(), po.nthreads, [&](int64_t x) {
                    const int t = tI[x].first;
                    const int64_t I = tI[x].second;
                    for (int64_t i = 0; i < csz; ++i)
                        for (int u = 0; u < s; ++u) R[(I * csz + i) * S + t * s + u] = Rcell[I]((int)i, u);
                });
                A(R.data(), Y.data(), S);
                subtract_lr(H, l, R, Y, S, po.nthreads);
                std::vector<std::pair<std::pair<int64_t, int64_t>, std::pair<int, int64_t>>> want;  // (I,J) <- (t, J)
                for (int t = 0; t < nclass; ++t)
                    for (int64_t I : members[t])
                        for (int64_t J : g.IL(l, I)) want.push_back({{I, J}, {t, J}});
                std::vector<Mat> got(want.size());
                parallel_for((int64_t)want.size(), po.nthreads, [&](int64_t x) {
                    got[x] = take(Y, S, want[x].second.second * csz, csz, want[x].second.first * s, s);
                });
                for (size_t x = 0; x < want.size(); ++x) Ysamp[want[x].first] = std::move(got[x]);
            }
            const double tol = po.eps * normS * std::sqrt(2.0 * s);
            std::atomic<bool> saturated(false);
            parallel_for((int64_t)pairs.size(), po.nthreads, [&](int64_t pi) {
                LR &p = pairs[pi];
                const Mat &YJ = Ysamp.at({p.I, p.J});  // A(J, I) R_I
                const Mat &YI = Ysamp.at({p.J, p.I});  // A(I, J) R_J = A(J, I)^* R_J
                Mat uj = orth(YJ, tol, s), ui = orth(YI, tol, s);
                if (s < csz && (uj.n > s - c / 2 || ui.n > s - c / 2)) saturated = true;
                // A(J,I) ~= UJ (R_J^* UJ)^+ (R_J^* A(J,I) R_I) (UI^* R_I)^+ UI^*
                const Mat &RI = Rcell[p.I], &RJ = Rcell[p.J];
                Mat left = pinv(matmul(RJ, uj, 'C', 'N'));
                Mat mid = matmul(RJ, YJ, 'C', 'N');
                Mat right = pinv(matmul(ui, RI, 'C', 'N'));
                p.B = matmul(matmul(left, mid), right);
                p.UJ = std::move(uj);
                p.UI = std::move(ui);
            });
            if (saturated && k < csz && attempt < 5) {
                k = (int)std::min<int64_t>(2 * k, csz);
                continue;
            }
            if (po.verbose) {
                int mr = 0;
                for (const LR &p : pairs) mr = std::max({mr, p.UI.n, p.UJ.n});
                progress(true, "  peeling level %d: %d samples per cell (attempt %d), largest rank %d%s", l, s,
                         attempt, mr, saturated ? " (saturated)" : "");
            }
            break;
        }
        progress(po.verbose, "peeling level %d: %zu admissible pairs", l, pairs.size());
        for (size_t i = 0; i < pairs.size(); ++i) {
            H.max_rank = std::max({H.max_rank, pairs[i].UI.n, pairs[i].UJ.n});
            const int64_t nc = (int64_t)1 << (2 * l);
            H.pairidx[l][pairs[i].I * nc + pairs[i].J] = (int)i;
        }
        H.lr[l] = std::move(pairs);
    }
    // Leaf near field: identity probes on classes of cells 4 apart (NL regions disjoint).
    {
        const int side = 1 << L;
        const int stride = std::min(4, side);
        const int64_t csz = g.cell_size(L);
        const int m = (int)csz;
        std::vector<std::pair<int, int>> classes;
        for (int p = 0; p < stride; ++p)
            for (int q = 0; q < stride; ++q) classes.push_back({p, q});
        const int per_apply = std::max(1, 512 / m);
        for (size_t c0 = 0; c0 < classes.size(); c0 += per_apply) {
            const int nclass = (int)std::min<size_t>(per_apply, classes.size() - c0);
            const int S = nclass * m;
            std::vector<cd> R((size_t)N * S, cd(0)), Y((size_t)N * S);
            std::vector<std::vector<int64_t>> members(nclass);
            for (int t = 0; t < nclass; ++t) {
                auto [p, q] = classes[c0 + t];
                for (int ci = p; ci < side; ci += stride)
                    for (int cj = q; cj < side; cj += stride) {
                        const int64_t I = g.cell_id(L, ci, cj);
                        members[t].push_back(I);
                        for (int i = 0; i < m; ++i) R[(I * csz + i) * S + t * m + i] = 1.0;
                    }
            }
            A(R.data(), Y.data(), S);
            subtract_lr(H, L + 1, R, Y, S, po.nthreads);
            std::vector<std::pair<std::pair<int64_t, int64_t>, int>> want;  // (J, I) <- class t
            for (int t = 0; t < nclass; ++t)
                for (int64_t I : members[t])
                    for (int64_t J : g.NL(L, I)) want.push_back({{J, I}, t});
            std::vector<Mat> got(want.size());
            parallel_for((int64_t)want.size(), po.nthreads, [&](int64_t x) {
                got[x] = take(Y, S, want[x].first.first * csz, csz, want[x].second * m, m);
            });
            for (size_t x = 0; x < want.size(); ++x) H.near[want[x].first] = std::move(got[x]);
        }
        // Hermitian symmetrisation of the near field
        for (auto &kv : H.near) {
            auto [J, I] = kv.first;
            if (J > I) continue;
            Mat &a = kv.second;
            Mat &b = H.near.at({I, J});
            for (int j = 0; j < m; ++j)
                for (int i = 0; i < m; ++i) {
                    cd v = 0.5 * (a(i, j) + std::conj(b(j, i)));
                    a(i, j) = v;
                    b(j, i) = std::conj(v);
                }
        }
    }
    return H;
}

// Current active matrix = H-matrix + accumulated Schur-complement updates, the
// latter kept as dense blocks per (leaf cell, leaf cell) pair.
struct Active2D {
    const Hmat2D &H;
    std::map<std::pair<int64_t, int64_t>, Mat> mod;
    explicit Active2D(const Hmat2D &h) : H(h) {}
    Mat sub(const std::vector<int> &rows, const std::vector<int> &cols) const {
        Mat out = H.sub(rows, cols);
        if (mod.empty() || rows.empty() || cols.empty()) return out;
        const int L = H.g.Lh;
        const int64_t leafsz = H.g.cell_size(L);
        std::map<int64_t, std::vector<int>> rg, cg;
        for (size_t i = 0; i < rows.size(); ++i) rg[H.g.cell_of(rows[i], L)].push_back((int)i);
        for (size_t j = 0; j < cols.size(); ++j) cg[H.g.cell_of(cols[j], L)].push_back((int)j);
        for (auto &rc : rg)
            for (auto &cc : cg) {
                auto it = mod.find({rc.first, cc.first});
                if (it == mod.end()) continue;
                for (int i : rc.second)
                    for (int j : cc.second)
                        out(i, j) += it->second((int)(rows[i] - rc.first * leafsz), (int)(cols[j] - cc.first * leafsz));
            }
        return out;
    }
    void add(const std::vector<int> &idx, const Mat &D) {
        const int L = H.g.Lh;
        const int64_t leafsz = H.g.cell_size(L);
        for (size_t j = 0; j < idx.size(); ++j) {
            const int64_t cb = H.g.cell_of(idx[j], L);
            for (size_t i = 0; i < idx.size(); ++i) {
                const int64_t ca = H.g.cell_of(idx[i], L);
                Mat &blk = mod[{ca, cb}];
                if (blk.m == 0) blk = Mat((int)leafsz, (int)leafsz);
                blk((int)(idx[i] - ca * leafsz), (int)(idx[j] - cb * leafsz)) += D((int)i, (int)j);
            }
        }
    }
};

// Far-field rows of a set D of DOFs inside cell c (level l): for every admissible
// pair of c and of its ancestors, the rows B U(D,:)^* (eq:2d_bases).
void far_rows(const Hmat2D &H, int l, int64_t c, const std::vector<int> &D, std::vector<Mat> &out) {
    const Geo &g = H.g;
    for (int lp = l; lp >= 2; --lp) {
        const int64_t a = c >> (2 * (l - lp));
        const int64_t csz = g.cell_size(lp);
        std::vector<int> loc;
        for (int d : D) loc.push_back((int)(d - a * csz));
        for (int64_t J : g.IL(lp, a)) {
            bool sw = false;
            const LR *p = H.find(lp, J, a, sw);  // want A(J rows, a cols)
            if (!p) continue;
            // stored A(pJ, pI) ~= UJ B UI^*; requested A(J, a)
            const Mat &Ua = sw ? p->UJ : p->UI;
            Mat mid = sw ? adj(p->B) : p->B;  // rows: basis of J side
            if (Ua.n == 0 || mid.m == 0) continue;
            out.push_back(matmul(mid, rows_of(Ua, loc), 'N', 'C'));
        }
    }
}

// Wall time per phase of a skeletonization level, summed over the node loop's threads
// (verbose builds report it).
struct PhaseTimes {
    std::atomic<int64_t> ns[8] = {};
    static int64_t now() {
        return std::chrono::duration_cast<std::chrono::nanoseconds>(
                   std::chrono::steady_clock::now().time_since_epoch())
            .count();
    }
    // largest interpolation coefficient |T_ij| of the level's IDs (the bit pattern of
    // a non-negative double orders like the value)
    std::atomic<uint64_t> tmax{0};
    void add(int k, int64_t t0) { ns[k].fetch_add(now() - t0); }
    void see_T(const Mat &T) {
        double m = 0;
        for (const cd &v : T.a) m = std::max(m, std::abs(v));
        uint64_t b;
        std::memcpy(&b, &m, 8);
        uint64_t cur = tmax.load();
        while (b > cur && !tmax.compare_exchange_weak(cur, b)) {
        }
    }
    void report(bool on, const char *what, int l) {
        double tm;
        const uint64_t b = tmax.load();
        std::memcpy(&tm, &b, 8);
        progress(on,
                 "  %s level %d thread-seconds: near %.2f far %.2f stack %.2f diag %.2f node %.2f (ID %.2f, "
                 "elimination %.2f); merge %.2f; largest |T| %.2e",
                 what, l, ns[0] * 1e-9, ns[1] * 1e-9, ns[2] * 1e-9, ns[3] * 1e-9, ns[4] * 1e-9, ns[6] * 1e-9,
                 ns[7] * 1e-9, ns[5] * 1e-9, tm);
        for (auto &v : ns) v.store(0);
        tmax.store(0);
    }
};

struct NodeOut {
    HifNode nd;
    Mat delta;  // Schur update on the skeleton DOFs (added to the active matrix)
};

// Skeletonize the DOFs I given the stacked row block Ubar and the current
// diagonal block A_II; same algebra as the 1D case (eq_sk, eq_sk_3).
// Large IDs (coarse cells and edges) go to the device when the plan has one.
constexpr int64_t BIG_ID_ENTRIES = 1 << 18;
// ... and so does the dense algebra of nodes with at least this many multiply-adds
// (nr^2 (nr + ns), the Schur update and Cholesky scale).
constexpr double BIG_NODE_WORK = 1 << 25;

NodeOut skel2d(const std::vector<int> &I, const Mat &Ubar, const Mat &AII, double eps, double shift0,
               std::atomic<int> &nshift, const PeelOptions &po, std::atomic<int> &ndev,
               std::atomic<int> &nnode, PhaseTimes &pt) {
    NodeOut out;
    const int n = (int)I.size();
    std::vector<int> sk, rd;
    Mat T;
    if (Ubar.m == 0 || n == 0) {
        for (int i = 0; i < n; ++i) rd.push_back(i);
        T = Mat(0, n);
    } else {
        const int64_t t0 = PhaseTimes::now();
        ColumnID id;
        if (po.dev.big_id && (int64_t)Ubar.m * Ubar.n >= BIG_ID_ENTRIES && po.dev.big_id(Ubar, eps, id))
            ndev.fetch_add(1);
        else
            id = column_id(Ubar, eps, 0, -1);
        sk = id.skel;
        rd = id.redund;
        T = std::move(id.T);
        if (po.verbose) pt.see_T(T);
        pt.add(6, t0);
    }
    const int64_t t1 = PhaseTimes::now();
    const int ns = (int)sk.size(), nr = (int)rd.size();
    Mat Arr(nr, nr), Asr(ns, nr), Ass(ns, ns);
    for (int j = 0; j < nr; ++j) {
        for (int i = 0; i < nr; ++i) Arr(i, j) = AII(rd[i], rd[j]);
        for (int i = 0; i < ns; ++i) Asr(i, j) = AII(sk[i], rd[j]);
    }
    for (int j = 0; j < ns; ++j)
        for (int i = 0; i < ns; ++i) Ass(i, j) = AII(sk[i], sk[j]);
    const auto finish = [&]() {
        out.nd.T = std::move(T);
        for (int i : rd) out.nd.idx_r.push_back(I[i]);
        for (int i : sk) out.nd.idx_s.push_back(I[i]);
    };
    if (po.dev.big_node && nr > 0 && ns > 0 && (double)nr * nr * (nr + ns) >= BIG_NODE_WORK &&
        po.dev.big_node(Arr, Asr, Ass, T, out.nd.Linv, out.nd.M, out.delta)) {
        nnode.fetch_add(1);
        finish();
        pt.add(7, t1);
        return out;
    }
    Mat AssT = matmul(Ass, T);
    Mat Atr = Arr;
    gemm_acc(Atr, T, Asr, -1.0, 'C', 'N');
    gemm_acc(Atr, Asr, T, -1.0, 'C', 'N');
    gemm_acc(Atr, T, AssT, 1.0, 'C', 'N');
    for (int j = 0; j < nr; ++j)
        for (int i = 0; i < j; ++i) {
            cd v = 0.5 * (Atr(i, j) + std::conj(Atr(j, i)));
            Atr(i, j) = v;
            Atr(j, i) = std::conj(v);
        }
    Mat Ats = Asr;
    gemm_acc(Ats, Ass, T, -1.0);
    Mat Lf = Atr;
    const double sh = cholesky_lower_shifted(Lf, shift0);
    if (sh < 0) fail(FIO_ERR_NOT_HPD, "2D skeletonization pivot block is not HPD");
    if (sh > 0) nshift.fetch_add(1);
    out.nd.Linv = tri_lower_inverse(Lf);
    out.nd.M = matmul(Ats, out.nd.Linv, 'N', 'C');
    out.delta = Mat(ns, ns);
    gemm_acc(out.delta, out.nd.M, out.nd.M, -1.0, 'N', 'C');
    finish();
    pt.add(7, t1);
    return out;
}

Mat stack_rows(const std::vector<Mat> &blocks, int ncols) {
    int rows = 0;
    for (auto &b : blocks) rows += b.m;
    Mat U(rows, ncols);
    int r0 = 0;
    for (auto &b : blocks) {
        for (int j = 0; j < ncols; ++j)
            for (int i = 0; i < b.m; ++i) U(r0 + i, j) = b(i, j);
        r0 += b.m;
    }
    return U;
}

}  // namespace

HifFactors build_hif_2d(const BlockApply &A, int n, const PeelOptions &po, double eps_hif) {
    Geo g;
    g.n = n;
    while ((1 << g.bits) < n) ++g.bits;
    g.N = (int64_t)n * n;
    const int leaf = std::min(po.leaf, n / 2);
    g.Lh = 0;
    while ((n >> g.Lh) > leaf) ++g.Lh;
    if (g.Lh < 1) fail(FIO_ERR_ARG, "2D grid too small for the cell tree");
    HifFactors F;
    F.N = g.N;
    const double normS = power_norm(A, g.N, 12, po.seed ^ 0x5EEDULL);
    Hmat2D H = peel_2d(A, g, po, normS);
    if (po.verbose) {
        uint64_t f = 0xCBF29CE484222325ULL;
        f = fingerprint(f, &normS, 8);
        for (const auto &lv : H.lr)
            for (const LR &p : lv) {
                f = fingerprint(f, p.UI.a.data(), p.UI.a.size() * 16);
                f = fingerprint(f, p.UJ.a.data(), p.UJ.a.size() * 16);
                f = fingerprint(f, p.B.a.data(), p.B.a.size() * 16);
            }
        for (const auto &kv : H.near) f = fingerprint(f, kv.second.a.data(), kv.second.a.size() * 16);
        progress(true, "  fingerprint of the peeled matrix: %016llx (norm %.17g)", (unsigned long long)f, normS);
    }
    const double shift0 = po.allow_shift ? 1e-3 * eps_hif * normS : 0.0;
    std::atomic<int> nshift(0), ndev(0), nnode(0);
    PhaseTimes pt;
    F.max_rank_h = H.max_rank;
    Active2D act(H);
    // active DOFs per cell at the current level
    const int L = g.Lh;
    std::vector<std::vector<int>> cells((size_t)1 << (2 * L));
    for (int64_t d = 0; d < g.N; ++d) cells[g.cell_of(d, L)].push_back((int)d);
    for (int l = L; l >= 1; --l) {
        const int side = 1 << l;
        const int64_t ncell = (int64_t)side * side;
        // ---- cell skeletonization (eq_sk_2d) ----
        {
            std::vector<NodeOut> res(ncell);
            parallel_for(ncell, po.nthreads, [&](int64_t c) {
                const std::vector<int> &I = cells[c];
                std::vector<int> Bnear;
                for (int64_t J : g.NL(l, c))
                    if (J != c) Bnear.insert(Bnear.end(), cells[J].begin(), cells[J].end());
                std::vector<Mat> blocks;
                int64_t t0 = PhaseTimes::now();
                if (!Bnear.empty()) blocks.push_back(act.sub(Bnear, I));
                pt.add(0, t0);
                t0 = PhaseTimes::now();
                far_rows(H, l, c, I, blocks);
                pt.add(1, t0);
                t0 = PhaseTimes::now();
                Mat Ubar = stack_rows(blocks, (int)I.size());
                pt.add(2, t0);
                t0 = PhaseTimes::now();
                Mat AII = act.sub(I, I);
                pt.add(3, t0);
                t0 = PhaseTimes::now();
                res[c] = skel2d(I, Ubar, AII, eps_hif, shift0, nshift, po, ndev, nnode, pt);
                pt.add(4, t0);
            });
            HifStep step;
            const int64_t tm = PhaseTimes::now();
            for (int64_t c = 0; c < ncell; ++c) {
                act.add(res[c].nd.idx_s, res[c].delta);
                cells[c] = res[c].nd.idx_s;
                step.nodes.push_back(std::move(res[c].nd));
            }
            pt.add(5, tm);
            F.steps.push_back(std::move(step));
            pt.report(po.verbose, "cells", l);
            progress(po.verbose, "cell skeletonization level %d done", l);
        }
        // ---- edge skeletonization (ID_2d_bases, eq_edge_sk_2d) ----
        {
            const int S = n >> l;  // cell side in points
            // edge e: 0..ncell-1 lower a-boundary of cell c; ncell..2ncell-1 lower b-boundary
            std::vector<std::vector<int>> edofs(2 * ncell);
            std::vector<std::vector<int>> ecell(2 * ncell);  // owning cell of each edge DOF
            for (int64_t c = 0; c < ncell; ++c) {
                int ci, cj;
                g.cell_xy(l, c, ci, cj);
                for (int d : cells[c]) {
                    int a, b;
                    g.dof_xy(d, a, b);
                    const int u = a - ci * S, v = b - cj * S;
                    // distances to the four boundaries; ties: a-boundaries first, lower first
                    const double dist[4] = {u + 0.5, S - u - 0.5, v + 0.5, S - v - 0.5};
                    int best = 0;
                    for (int t = 1; t < 4; ++t)
                        if (dist[t] < dist[best]) best = t;
                    int64_t e;
                    if (best == 0) e = g.cell_id(l, ci, cj);
                    else if (best == 1) e = g.cell_id(l, ci + 1, cj);
                    else if (best == 2) e = ncell + g.cell_id(l, ci, cj);
                    else e = ncell + g.cell_id(l, ci, cj + 1);
                    edofs[e].push_back(d);
                    ecell[e].push_back((int)c);
                }
            }
            std::vector<NodeOut> res(2 * ncell);
            std::vector<char> used(2 * ncell, 0);
            parallel_for(2 * ncell, po.nthreads, [&](int64_t e) {
                const std::vector<int> &I = edofs[e];
                if (I.empty()) return;
                used[e] = 1;
                // the two cells adjacent to the edge
                int64_t c2 = (e < ncell) ? e : e - ncell;
                int ci, cj;
                g.cell_xy(l, c2, ci, cj);
                int64_t c1 = (e < ncell) ? g.cell_id(l, ci - 1, cj) : g.cell_id(l, ci, cj - 1);
                std::set<int> inE(I.begin(), I.end());
                std::set<int64_t> ncells;
                for (int64_t J : g.NL(l, c1)) ncells.insert(J);
                for (int64_t J : g.NL(l, c2)) ncells.insert(J);
                std::vector<int> Bnear;
                for (int64_t J : ncells)
                    for (int d : cells[J])
                        if (!inE.count(d)) Bnear.push_back(d);
                std::vector<Mat> blocks;
                int64_t t0 = PhaseTimes::now();
                if (!Bnear.empty()) blocks.push_back(act.sub(Bnear, I));
                pt.add(0, t0);
                t0 = PhaseTimes::now();
                // far-field bases of each side, placed in the columns of that side
                for (int64_t side_cell : {c1, c2}) {
                    std::vector<int> D, pos;
                    for (size_t t = 0; t < I.size(); ++t)
                        if (ecell[e][t] == (int)side_cell) {
                            D.push_back(I[t]);
                            pos.push_back((int)t);
                        }
                    if (D.empty()) continue;
                    std::vector<Mat> fr;
                    far_rows(H, l, side_cell, D, fr);
                    for (Mat &f : fr) {
                        Mat full(f.m, (int)I.size());
                        for (int j = 0; j < f.n; ++j)
                            for (int i = 0; i < f.m; ++i) full(i, pos[j]) = f(i, j);
                        blocks.push_back(std::move(full));
                    }
                    if (c1 == c2) break;
                }
                pt.add(1, t0);
                t0 = PhaseTimes::now();
                Mat Ubar = stack_rows(blocks, (int)I.size());
                pt.add(2, t0);
                t0 = PhaseTimes::now();
                Mat AII = act.sub(I, I);
                pt.add(3, t0);
                t0 = PhaseTimes::now();
                res[e] = skel2d(I, Ubar, AII, eps_hif, shift0, nshift, po, ndev, nnode, pt);
                pt.add(4, t0);
            });
            HifStep step;
            std::vector<std::vector<int>> remain(ncell);
            const int64_t tm = PhaseTimes::now();
            for (int64_t e = 0; e < 2 * ncell; ++e) {
                if (!used[e]) continue;
                act.add(res[e].nd.idx_s, res[e].delta);
                for (int d : res[e].nd.idx_s) remain[g.cell_of(d, l)].push_back(d);
                step.nodes.push_back(std::move(res[e].nd));
            }
            pt.add(5, tm);
            pt.report(po.verbose, "edges", l);
            F.steps.push_back(std::move(step));
            // merge child cells into their parents (level l-1)
            const int64_t npar = ncell / 4;
            std::vector<std::vector<int>> up(std::max<int64_t>(npar, 1));
            for (int64_t c = 0; c < ncell; ++c) {
                std::sort(remain[c].begin(), remain[c].end());
                auto &dst = up[l >= 1 ? (c >> 2) : 0];
                dst.insert(dst.end(), remain[c].begin(), remain[c].end());
            }
            cells.swap(up);
            progress(po.verbose, "edge skeletonization level %d done", l);
        }
    }
    // Root: the remaining DOFs (one cell at level 0).
    std::vector<int> root;
    for (auto &c : cells) root.insert(root.end(), c.begin(), c.end());
    std::sort(root.begin(), root.end());
    F.root_idx = root;
    if (!root.empty()) {
        Mat A0 = act.sub(root, root);
        for (int j = 0; j < A0.n; ++j)
            for (int i = 0; i < j; ++i) {
                cd v = 0.5 * (A0(i, j) + std::conj(A0(j, i)));
                A0(i, j) = v;
                A0(j, i) = std::conj(v);
            }
        if (po.dev.hpd_inverse && (double)A0.n * A0.n * A0.n >= BIG_NODE_WORK && po.dev.hpd_inverse(A0, F.A0inv)) {
            nnode.fetch_add(1);
        } else {
            const double sh = hpd_inverse_shifted(A0, F.A0inv, shift0);
            if (sh < 0) fail(FIO_ERR_NOT_HPD, "2D top-level block is not HPD");
            if (sh > 0) nshift.fetch_add(1);
        }
    }
    F.shifted = nshift.load();
    F.device_ids = ndev.load();
    F.device_nodes = nnode.load();
    return F;
}

}  // namespace fio
