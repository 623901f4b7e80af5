// 1D: HODLR peeling (section 3) and recursive-skeletonization inverse (section 4).
#include <atomic>
#include <algorithm>
#include <cmath>

#include "hif.hpp"

namespace fio {

namespace {

struct Hodlr1D {
    int Lh = 0;
    int64_t N = 0, mh = 0;
    std::vector<std::vector<Mat>> U;  // U[l][node]: basis on the node's points
    std::vector<std::vector<Mat>> B;  // B[l][p]: A(2p+1, 2p) ~= U[l][2p+1] B U[l][2p]^*
    std::vector<Mat> D;               // leaf diagonal blocks
};

// Rows [start, start+sz) of a point-major N x s block, as a column-major sz x s matrix.
Mat take_rows(const std::vector<cd> &X, int s, int64_t start, int64_t sz) {
    Mat R((int)sz, s);
    for (int64_t i = 0; i < sz; ++i)
        for (int c = 0; c < s; ++c) R((int)i, c) = X[(start + i) * s + c];
    return R;
}

void add_rows(std::vector<cd> &X, int s, int64_t start, const Mat &Y, cd alpha) {
    for (int64_t i = 0; i < Y.m; ++i)
        for (int c = 0; c < s; ++c) X[(start + i) * s + c] += alpha * Y((int)i, c);
}

// out -= sum_{l < upto} Ahat_l X  (both point-major N x s)
void subtract_lowrank(const Hodlr1D &H, int upto, const std::vector<cd> &X,
                      std::vector<cd> &out, int s, int nthreads) {
    for (int l = 1; l < upto; ++l) {
        const int64_t sz = H.N >> l;
        const int64_t np = (int64_t)1 << (l - 1);
        parallel_for(np, nthreads, [&](int64_t p) {
            const Mat &Ua = H.U[l][2 * p], &Ub = H.U[l][2 * p + 1], &Bp = H.B[l][p];
            if (Ua.n == 0 || Ub.n == 0) return;
            Mat Xa = take_rows(X, s, 2 * p * sz, sz), Xb = take_rows(X, s, (2 * p + 1) * sz, sz);
            Mat ta = matmul(Ua, Xa, 'C', 'N');                 // k2 x s
            Mat yb = matmul(Ub, matmul(Bp, ta));               // rows of node 2p+1
            Mat tb = matmul(Ub, Xb, 'C', 'N');
            Mat ya = matmul(Ua, matmul(Bp, tb, 'C', 'N'));     // rows of node 2p
            add_rows(out, s, (2 * p + 1) * sz, yb, -1.0);
            add_rows(out, s, 2 * p * sz, ya, -1.0);
        });
    }
}

Hodlr1D peel_1d(const BlockApply &A, int64_t N, const PeelOptions &po, double normS,
                int &max_rank) {
    Hodlr1D H;
    H.N = N;
    H.mh = std::min<int64_t>(po.leaf, N);
    while ((H.mh << H.Lh) < N) ++H.Lh;
    if ((H.mh << H.Lh) != N) fail(FIO_ERR_ARG, "HODLR leaf must divide N into a power of two");
    H.U.resize(H.Lh + 1);
    H.B.resize(H.Lh + 1);
    max_rank = 0;
    const int c = po.oversample;
    for (int l = 1; l <= H.Lh; ++l) {
        const int64_t sz = N >> l;
        const int64_t np = (int64_t)1 << (l - 1);
        int k = std::min<int64_t>(po.k0, sz);
        for (int attempt = 0;; ++attempt) {
            const int s = (int)std::min<int64_t>(k + c, sz);
            // Probes: columns [0, s) nonzero on even nodes (R1), [s, 2s) on odd nodes (R2).
            const int s2 = 2 * s;
            std::vector<cd> R((size_t)N * s2, cd(0)), Y((size_t)N * s2);
            const uint64_t sd = po.seed ^ splitmix64(0x9E00 + l * 64 + attempt);
            parallel_for(N, po.nthreads, [&](int64_t i) {
                int64_t node = i / sz;
                int off = (node % 2 == 0) ? 0 : s;
                for (int q = 0; q < s; ++q) {
                    uint64_t ctr = ((uint64_t)i * s + q) * 2;
                    R[i * s2 + off + q] = cd(gauss(sd, ctr), gauss(sd, ctr + 1));
                }
            });
            A(R.data(), Y.data(), s2);
            subtract_lowrank(H, l, R, Y, s2, po.nthreads);
            std::vector<Mat> Ua(np), Ub(np), Bp(np);
            std::atomic<bool> saturated(false);
            const double tol = po.eps * normS * std::sqrt(2.0 * s);
            parallel_for(np, po.nthreads, [&](int64_t p) {
                const int64_t sa = 2 * p * sz, sb = (2 * p + 1) * sz;
                // Y1 on node 2p+1 = A(2p+1, 2p) R1(2p); Y2 on node 2p = A(2p+1, 2p)^* R2(2p+1).
                Mat Yall_b = take_rows(Y, s2, sb, sz), Yall_a = take_rows(Y, s2, sa, sz);
                Mat Rall_b = take_rows(R, s2, sb, sz), Rall_a = take_rows(R, s2, sa, sz);
                Mat Y1(sz, s), Y2(sz, s), R1a(sz, s), R2b(sz, s);
                for (int q = 0; q < s; ++q)
                    for (int64_t i = 0; i < sz; ++i) {
                        Y1((int)i, q) = Yall_b((int)i, q);
                        Y2((int)i, q) = Yall_a((int)i, s + q);
                        R1a((int)i, q) = Rall_a((int)i, q);
                        R2b((int)i, q) = Rall_b((int)i, s + q);
                    }
                Mat ub = orth(Y1, tol, s), ua = orth(Y2, tol, s);
                if (s < sz && (ub.n > s - c / 2 || ua.n > s - c / 2)) saturated = true;
                // A21 ~= U1 (R2^* U1)^+ (R2^* A21 R1) (U2^* R1)^+ U2^*   (eqn:lvl1_LR)
                Mat left = pinv(matmul(R2b, ub, 'C', 'N'));
                Mat mid = matmul(R2b, Y1, 'C', 'N');
                Mat right = pinv(matmul(ua, R1a, 'C', 'N'));
                Bp[p] = matmul(matmul(left, mid), right);
                Ua[p] = std::move(ua);
                Ub[p] = std::move(ub);
            });
            if (saturated && k < sz && attempt < 6) {
                k = (int)std::min<int64_t>(2 * k, sz);
                continue;
            }
            progress(po.verbose, "peeling level %d: rank <= %d", l, k + c);
            H.U[l].resize(2 * np);
            H.B[l] = std::move(Bp);
            for (int64_t p = 0; p < np; ++p) {
                max_rank = std::max({max_rank, Ua[p].n, Ub[p].n});
                H.U[l][2 * p] = std::move(Ua[p]);
                H.U[l][2 * p + 1] = std::move(Ub[p]);
            }
            break;
        }
    }
    // Leaf diagonal blocks: probe with an identity block on every leaf.
    {
        const int s = (int)H.mh;
        std::vector<cd> R((size_t)N * s, cd(0)), Y((size_t)N * s);
        for (int64_t i = 0; i < N; ++i) R[i * s + (i % s)] = 1.0;
        A(R.data(), Y.data(), s);
        subtract_lowrank(H, H.Lh + 1, R, Y, s, po.nthreads);
        const int64_t nl = N / H.mh;
        H.D.resize(nl);
        for (int64_t b = 0; b < nl; ++b) {
            Mat Db = take_rows(Y, s, b * H.mh, H.mh);
            Mat Ds(s, s);
            for (int j = 0; j < s; ++j)
                for (int i = 0; i < s; ++i) Ds(i, j) = 0.5 * (Db(i, j) + std::conj(Db(j, i)));
            H.D[b] = std::move(Ds);
        }
    }
    return H;
}

struct Active {
    std::vector<int> I;  // global DOFs
    Mat A;               // current diagonal block on I
};

// Skeletonize one node: returns its factor and replaces st by its skeleton part.
HifNode skeletonize(Active &st, const Mat &Ubar, double eps, double shift0, std::atomic<int> &nshift) {
    const int n = (int)st.I.size();
    HifNode nd;
    std::vector<int> sk, rd;
    Mat T;
    if (Ubar.m == 0 || n == 0) {
        for (int i = 0; i < n; ++i) rd.push_back(i);
        T = Mat(0, n);
    } else {
        ColumnID id = column_id(Ubar, eps, 0, -1);
        sk = id.skel;
        rd = id.redund;
        T = std::move(id.T);
    }
    const int ns = (int)sk.size(), nr = (int)rd.size();
    Mat Arr(nr, nr), Asr(ns, nr), Ass(ns, ns);
    for (int j = 0; j < nr; ++j) {
        for (int i = 0; i < nr; ++i) Arr(i, j) = st.A(rd[i], rd[j]);
        for (int i = 0; i < ns; ++i) Asr(i, j) = st.A(sk[i], rd[j]);
    }
    for (int j = 0; j < ns; ++j)
        for (int i = 0; i < ns; ++i) Ass(i, j) = st.A(sk[i], sk[j]);
    // Z^* A Z (eq_sk): Atilde_rr = Arr - T^* Asr - Asr^* T + T^* Ass T; Atilde_sr = Asr - Ass T.
    Mat AssT = matmul(Ass, T);
    Mat Atr = Arr;
    gemm_acc(Atr, T, Asr, -1.0, 'C', 'N');
    gemm_acc(Atr, Asr, T, -1.0, 'C', 'N');
    gemm_acc(Atr, T, AssT, 1.0, 'C', 'N');
    for (int j = 0; j < nr; ++j)  // keep exactly Hermitian
        for (int i = 0; i < j; ++i) {
            cd v = 0.5 * (Atr(i, j) + std::conj(Atr(j, i)));
            Atr(i, j) = v;
            Atr(j, i) = std::conj(v);
        }
    Mat Ats = Asr;
    gemm_acc(Ats, Ass, T, -1.0);
    // Gaussian elimination (eq_sk_3) with Atilde_rr = L L^*.
    Mat Lf = Atr;
    const double sh = cholesky_lower_shifted(Lf, shift0);
    if (sh < 0) fail(FIO_ERR_NOT_HPD, "skeletonization pivot block is not HPD");
    if (sh > 0) nshift.fetch_add(1);
    nd.Linv = tri_lower_inverse(Lf);
    nd.M = matmul(Ats, nd.Linv, 'N', 'C');  // Atilde_sr L^{-*}
    Mat Abar = Ass;
    gemm_acc(Abar, nd.M, nd.M, -1.0, 'N', 'C');
    nd.T = std::move(T);
    for (int i : rd) nd.idx_r.push_back(st.I[i]);
    for (int i : sk) nd.idx_s.push_back(st.I[i]);
    st.I = nd.idx_s;
    st.A = std::move(Abar);
    return nd;
}

// Diagonal block of two merged siblings (section 4, "merge child blocks").
Active merge(const Active &a, const Active &b, const Mat &Ua, const Mat &Ub, const Mat &Bp,
             int64_t start_a, int64_t start_b) {
    Active m;
    const int na = (int)a.I.size(), nb = (int)b.I.size();
    m.I = a.I;
    m.I.insert(m.I.end(), b.I.begin(), b.I.end());
    m.A = Mat(na + nb, na + nb);
    for (int j = 0; j < na; ++j)
        for (int i = 0; i < na; ++i) m.A(i, j) = a.A(i, j);
    for (int j = 0; j < nb; ++j)
        for (int i = 0; i < nb; ++i) m.A(na + i, na + j) = b.A(i, j);
    if (Ua.n > 0 && Ub.n > 0 && na > 0 && nb > 0) {
        std::vector<int> ra, rb;
        for (int g : a.I) ra.push_back((int)(g - start_a));
        for (int g : b.I) rb.push_back((int)(g - start_b));
        Mat Sba = matmul(matmul(rows_of(Ub, rb), Bp), rows_of(Ua, ra), 'N', 'C');  // nb x na
        for (int j = 0; j < na; ++j)
            for (int i = 0; i < nb; ++i) {
                m.A(na + i, j) = Sba(i, j);
                m.A(j, na + i) = std::conj(Sba(i, j));
            }
    }
    return m;
}

// ---- Cholesky-prescaled variant (section 4, the alternative to eq_sk_3) ----
// The active state of a node also carries its bases in the scaled coordinates:
// P[lp] (k_lp x n) stands for U_{lp;I}^* at every ancestor level lp, multiplied on the
// right by the inverse-adjoint Cholesky factors of the scalings applied so far and
// restricted to the surviving coordinates.  Coordinates live in the storage slots I.
struct ActiveP {
    std::vector<int> I;
    Mat A;
    std::vector<Mat> P;  // index lp = 1..l (P[0] unused)
};

// Scale, decompose, eliminate: returns the two node factors (scaling first).
void skeletonize_prescaled(ActiveP &st, int l, double eps, double shift0, std::atomic<int> &nshift,
                           HifNode &pre, HifNode &skn) {
    const int n = (int)st.I.size();
    // A_II = L L^* (the scaling); Hermitian part first
    Mat Lf = st.A;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < j; ++i) {
            const cd v = 0.5 * (Lf(i, j) + std::conj(Lf(j, i)));
            Lf(i, j) = v;
            Lf(j, i) = std::conj(v);
        }
    const double sh = cholesky_lower_shifted(Lf, shift0);
    if (sh < 0) fail(FIO_ERR_NOT_HPD, "prescaled skeletonization: diagonal block is not HPD");
    if (sh > 0) nshift.fetch_add(1);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < j; ++i) Lf(i, j) = 0.0;
    const Mat Linv = tri_lower_inverse(Lf);
    // scaled bases: P[lp] L^{-*}, stacked from level l down to 1 for the ID
    int rows = 0;
    for (int lp = l; lp >= 1; --lp) {
        st.P[lp] = matmul(st.P[lp], Linv, 'N', 'C');
        rows += st.P[lp].m;
    }
    Mat Ubar(rows, n);
    int r0 = 0;
    for (int lp = l; lp >= 1; --lp) {
        for (int c = 0; c < n; ++c)
            for (int k = 0; k < st.P[lp].m; ++k) Ubar(r0 + k, c) = st.P[lp](k, c);
        r0 += st.P[lp].m;
    }
    std::vector<int> sk, rd;
    Mat T;
    if (rows == 0 || n == 0) {
        for (int i = 0; i < n; ++i) rd.push_back(i);
        T = Mat(0, n);
    } else {
        ColumnID id = column_id(Ubar, eps, 0, -1);
        sk = id.skel;
        rd = id.redund;
        T = std::move(id.T);
    }
    const int ns = (int)sk.size(), nr = (int)rd.size();
    // In the scaled coordinates A_II = I, so Z^* A Z (eq_sk) has Atilde_rr = I + T^* T
    // (eigenvalues >= 1) and Atilde_sr = -T.
    Mat Atr = Mat::eye(nr);
    gemm_acc(Atr, T, T, 1.0, 'C', 'N');
    Mat L2 = Atr;
    if (!cholesky_lower(L2)) fail(FIO_ERR_NOT_HPD, "prescaled skeletonization: I + T^*T not HPD");
    skn.Linv = tri_lower_inverse(L2);
    Mat Ats(ns, nr);
    for (int j = 0; j < nr; ++j)
        for (int i = 0; i < ns; ++i) Ats(i, j) = -T(i, j);
    skn.M = matmul(Ats, skn.Linv, 'N', 'C');
    Mat Abar = Mat::eye(ns);
    gemm_acc(Abar, skn.M, skn.M, -1.0, 'N', 'C');
    skn.T = std::move(T);
    for (int i : rd) skn.idx_r.push_back(st.I[i]);
    for (int i : sk) skn.idx_s.push_back(st.I[i]);
    pre.idx_r = st.I;
    pre.T = Mat(0, n);
    pre.Linv = Linv;
    pre.M = Mat(0, n);
    // surviving coordinates: the skeletons, with their scaled bases
    for (int lp = l; lp >= 1; --lp) st.P[lp] = cols_of(st.P[lp], sk);
    st.I = skn.idx_s;
    st.A = std::move(Abar);
}

// Merge two scaled siblings at level l: the coupling is P_b[l]^* B P_a[l].
ActiveP merge_prescaled(const ActiveP &a, const ActiveP &b, const Mat &Bp, int l) {
    ActiveP m;
    const int na = (int)a.I.size(), nb = (int)b.I.size();
    m.I = a.I;
    m.I.insert(m.I.end(), b.I.begin(), b.I.end());
    m.A = Mat(na + nb, na + nb);
    for (int j = 0; j < na; ++j)
        for (int i = 0; i < na; ++i) m.A(i, j) = a.A(i, j);
    for (int j = 0; j < nb; ++j)
        for (int i = 0; i < nb; ++i) m.A(na + i, na + j) = b.A(i, j);
    if (a.P[l].m > 0 && b.P[l].m > 0 && na > 0 && nb > 0) {
        Mat Sba = matmul(matmul(b.P[l], Bp, 'C', 'N'), a.P[l]);  // nb x na
        for (int j = 0; j < na; ++j)
            for (int i = 0; i < nb; ++i) {
                m.A(na + i, j) = Sba(i, j);
                m.A(j, na + i) = std::conj(Sba(i, j));
            }
    }
    m.P.assign(l, Mat());
    for (int lp = 1; lp < l; ++lp) {
        const Mat &pa = a.P[lp], &pb = b.P[lp];
        Mat c(std::max(pa.m, pb.m), na + nb);
        for (int j = 0; j < na; ++j)
            for (int k = 0; k < pa.m; ++k) c(k, j) = pa(k, j);
        for (int j = 0; j < nb; ++j)
            for (int k = 0; k < pb.m; ++k) c(k, na + j) = pb(k, j);
        m.P[lp] = std::move(c);
    }
    return m;
}

}  // namespace

double power_norm(const BlockApply &A, int64_t N, int iters, uint64_t seed) {
    std::vector<cd> x(N), y(N);
    for (int64_t i = 0; i < N; ++i) x[i] = cd(gauss(seed, 2 * i), gauss(seed, 2 * i + 1));
    double lam = 0;
    for (int it = 0; it < iters; ++it) {
        double nx = 0;
        for (auto &v : x) nx += std::norm(v);
        nx = std::sqrt(nx);
        for (auto &v : x) v /= nx;
        A(x.data(), y.data(), 1);
        double ny = 0;
        for (auto &v : y) ny += std::norm(v);
        lam = std::sqrt(ny);
        x.swap(y);
    }
    return lam;
}

HifFactors build_hif_1d(const BlockApply &A, int64_t N, const PeelOptions &po, double eps_hif) {
    HifFactors F;
    F.N = N;
    const double normS = power_norm(A, N, 12, po.seed ^ 0x5EEDULL);
    Hodlr1D H = peel_1d(A, N, po, normS, F.max_rank_h);
    const double shift0 = po.allow_shift ? 1e-3 * eps_hif * normS : 0.0;
    std::atomic<int> nshift(0);
    const int64_t nleaf = N / H.mh;
    if (po.prescale) {
        std::vector<ActiveP> sp(nleaf);
        for (int64_t b = 0; b < nleaf; ++b) {
            ActiveP &a = sp[b];
            a.I.resize(H.mh);
            for (int64_t i = 0; i < H.mh; ++i) a.I[i] = (int)(b * H.mh + i);
            a.A = H.D[b];
            a.P.assign(H.Lh + 1, Mat());
            for (int lp = 1; lp <= H.Lh; ++lp) {
                const int64_t an = b >> (H.Lh - lp);
                const Mat &Ua = H.U[lp][an];
                const int64_t start = an * (N >> lp);
                Mat P(Ua.n, (int)H.mh);
                for (int64_t c = 0; c < H.mh; ++c)
                    for (int k = 0; k < Ua.n; ++k) P(k, (int)c) = std::conj(Ua((int)(b * H.mh + c - start), k));
                a.P[lp] = std::move(P);
            }
        }
        for (int l = H.Lh; l >= 1; --l) {
            const int64_t nn = (int64_t)1 << l;
            HifStep pre, skl;
            pre.nodes.resize(nn);
            skl.nodes.resize(nn);
            parallel_for(nn, po.nthreads, [&](int64_t v) {
                skeletonize_prescaled(sp[v], l, eps_hif, shift0, nshift, pre.nodes[v], skl.nodes[v]);
            });
            F.steps.push_back(std::move(pre));
            F.steps.push_back(std::move(skl));
            std::vector<ActiveP> up(nn / 2);
            parallel_for(nn / 2, po.nthreads, [&](int64_t p) {
                up[p] = merge_prescaled(sp[2 * p], sp[2 * p + 1], H.B[l][p], l);
            });
            sp.swap(up);
        }
        F.root_idx = sp[0].I;
        if (!F.root_idx.empty()) {
            const double sh = hpd_inverse_shifted(sp[0].A, F.A0inv, shift0);
            if (sh < 0) fail(FIO_ERR_NOT_HPD, "top-level block is not HPD");
            if (sh > 0) nshift.fetch_add(1);
        }
        F.shifted = nshift.load();
        return F;
    }
    std::vector<Active> st(nleaf);
    for (int64_t b = 0; b < nleaf; ++b) {
        st[b].I.resize(H.mh);
        for (int64_t i = 0; i < H.mh; ++i) st[b].I[i] = (int)(b * H.mh + i);
        st[b].A = H.D[b];
    }
    for (int l = H.Lh; l >= 1; --l) {
        const int64_t nn = (int64_t)1 << l;
        HifStep step;
        step.nodes.resize(nn);
        parallel_for(nn, po.nthreads, [&](int64_t v) {
            // Ubar = [U_{l;I}^*; U_{l-1;I}^*; ...; U_{1;I}^*] (section 4, 1D case)
            const std::vector<int> &I = st[v].I;
            int rows = 0;
            for (int lp = l; lp >= 1; --lp) rows += H.U[lp][v >> (l - lp)].n;
            Mat Ubar(rows, (int)I.size());
            int r0 = 0;
            for (int lp = l; lp >= 1; --lp) {
                int64_t a = v >> (l - lp);
                const Mat &Ua = H.U[lp][a];
                int64_t start = a * (N >> lp);
                for (size_t c = 0; c < I.size(); ++c)
                    for (int k = 0; k < Ua.n; ++k)
                        Ubar(r0 + k, (int)c) = std::conj(Ua((int)(I[c] - start), k));
                r0 += Ua.n;
            }
            step.nodes[v] = skeletonize(st[v], Ubar, eps_hif, shift0, nshift);
        });
        F.steps.push_back(std::move(step));
        std::vector<Active> up(nn / 2);
        parallel_for(nn / 2, po.nthreads, [&](int64_t p) {
            const int64_t sz = N >> l;
            up[p] = merge(st[2 * p], st[2 * p + 1], H.U[l][2 * p], H.U[l][2 * p + 1], H.B[l][p],
                          2 * p * sz, (2 * p + 1) * sz);
        });
        st.swap(up);
    }
    // Root: the remaining active DOFs S_0 (st has one entry after the merge of level 1).
    F.root_idx = st[0].I;
    if (!F.root_idx.empty()) {
        const double sh = hpd_inverse_shifted(st[0].A, F.A0inv, shift0);
        if (sh < 0) fail(FIO_ERR_NOT_HPD, "top-level block is not HPD");
        if (sh > 0) nshift.fetch_add(1);
    }
    F.shifted = nshift.load();
    return F;
}

}  // namespace fio
