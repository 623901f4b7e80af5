// Host construction of all factors (Algorithm "alg", section 5) and their file format.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>

#include "plan.hpp"

namespace fio {

// Progress line on stderr, prefixed with the seconds since the first line.
void progress(bool on, const char *fmt, ...) {
    if (!on) return;
    static const auto t0 = std::chrono::steady_clock::now();
    const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    va_list ap;
    va_start(ap, fmt);
    std::fprintf(stderr, "[fio_build %8.2fs] ", el);
    std::vfprintf(stderr, fmt, ap);
    std::fprintf(stderr, "\n");
    std::fflush(stderr);
    va_end(ap);
}

static bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

fio_problem normalized_problem(const fio_problem &in) {
    fio_problem p = in;
    if (p.d != 1 && p.d != 2) fail(FIO_ERR_ARG, "d must be 1 or 2");
    if (!is_pow2(p.n) || p.n % 2) fail(FIO_ERR_ARG, "n must be an even power of two");
    if (!(p.eps > 0 && p.eps < 1)) fail(FIO_ERR_ARG, "eps must lie in (0, 1)");
    if (p.phase == FIO_PHASE_1D_EX1 && p.d != 1) fail(FIO_ERR_ARG, "phase 1D_EX1 needs d = 1");
    if (p.phase == FIO_PHASE_2D_RADON && p.d != 2) fail(FIO_ERR_ARG, "phase 2D_RADON needs d = 2");
    if (p.phase == FIO_PHASE_1D_EX2 && p.d != 1) fail(FIO_ERR_ARG, "phase 1D_EX2 needs d = 1");
    if (p.phase < FIO_PHASE_LINEAR || p.phase > FIO_PHASE_CALLBACK) fail(FIO_ERR_ARG, "unknown phase");
    if (p.phase == FIO_PHASE_CALLBACK && !p.phi) fail(FIO_ERR_ARG, "FIO_PHASE_CALLBACK needs a phase function phi");
    if (p.phase != FIO_PHASE_CALLBACK) {  // the callbacks belong to FIO_PHASE_CALLBACK only
        p.phi = nullptr;
        p.amp = nullptr;
        p.user = nullptr;
    }
    if (p.amp_terms < 0 || p.amp_terms > FIO_MAX_AMP_TERMS) fail(FIO_ERR_ARG, "amp_terms out of range");
    if (p.amp_sigma2 == 0) p.amp_sigma2 = 0.1;
    if (!(p.amp_sigma2 > 0)) fail(FIO_ERR_ARG, "amp_sigma2 must be positive");
    if (p.phase == FIO_PHASE_1D_EX2 && p.amp_terms == 0) {
        const double cx[3] = {0.2, 0.5, 0.8}, ce[3] = {-0.2, 0.2, 0.0};
        p.amp_terms = 3;
        for (int k = 0; k < 3; ++k) { p.amp_x[k] = cx[k]; p.amp_eta[k] = ce[k]; }
    }
    if (p.c_div == 0) p.c_div = 16.0;
    if (!(p.c_div > 0)) fail(FIO_ERR_ARG, "c_div must be positive");
    if (p.eps_bf == 0) p.eps_bf = p.eps / 10;
    if (p.eps_peel == 0) p.eps_peel = p.eps;
    if (p.eps_hif == 0) p.eps_hif = p.eps;
    if (!(p.eps_bf > 0 && p.eps_peel > 0 && p.eps_hif > 0)) fail(FIO_ERR_ARG, "tolerances must be positive");
    if (p.leaf_bf == 0) p.leaf_bf = (p.d == 1) ? 8 : 4;
    if (p.leaf_h == 0) p.leaf_h = (p.d == 1) ? 64 : 8;
    if (p.oversample == 0) p.oversample = 10;
    if (!is_pow2(p.leaf_bf) || p.leaf_bf > p.n / 2) fail(FIO_ERR_ARG, "leaf_bf must be a power of two <= n/2");
    if (!is_pow2(p.leaf_h)) fail(FIO_ERR_ARG, "leaf_h must be a power of two");
    if (p.d == 1 && p.leaf_h > p.n / 2) p.leaf_h = p.n / 2;
    if (p.d == 2 && p.leaf_h > p.n / 2) p.leaf_h = p.n / 2;
    if (p.oversample < 1) fail(FIO_ERR_ARG, "oversample must be positive");
    if (p.prescale_skel && p.d != 1) fail(FIO_ERR_ARG, "prescaled skeletonization is built for 1D only");
    if (p.bf_rank_align == 0) p.bf_rank_align = 8;
    if (p.bf_rank_align < 1) fail(FIO_ERR_ARG, "bf_rank_align must be positive");
    return p;
}

std::vector<uint64_t> factor_fingerprints(const HostFactors &f) {
    std::vector<uint64_t> out;
    uint64_t h = fingerprint(0xCBF29CE484222325ULL, f.perm.data(), f.perm.size() * 4);
    for (const Stage &s : f.fwd) {
        const int64_t dims[5] = {s.n_out, s.n_in, s.r_out, s.r_in, s.fan};
        h = fingerprint(h, dims, sizeof(dims));
        h = fingerprint(h, s.in_idx.data(), s.in_idx.size() * 4);
        h = fingerprint(h, s.A.data(), s.A.size() * sizeof(cd));
    }
    out.push_back(h);
    for (const HifStep &st : f.hif.steps) {
        h = 0xCBF29CE484222325ULL;
        for (const HifNode &nd : st.nodes) {
            h = fingerprint(h, nd.idx_r.data(), nd.idx_r.size() * 4);
            h = fingerprint(h, nd.idx_s.data(), nd.idx_s.size() * 4);
            h = fingerprint(h, nd.T.a.data(), nd.T.a.size() * 16);
            h = fingerprint(h, nd.Linv.a.data(), nd.Linv.a.size() * 16);
            h = fingerprint(h, nd.M.a.data(), nd.M.a.size() * 16);
        }
        out.push_back(h);
    }
    h = fingerprint(0xCBF29CE484222325ULL, f.hif.root_idx.data(), f.hif.root_idx.size() * 4);
    out.push_back(fingerprint(h, f.hif.A0inv.a.data(), f.hif.A0inv.a.size() * 16));
    return out;
}

void build_host_factors(const fio_problem &pin, HostFactors &out, const PeelApplyFactory &gpu,
                        const BatchedIdFactory &ids, const SkelHooks &skel) {
    auto t0 = std::chrono::steady_clock::now();
    fio_problem p = normalized_problem(pin);
    FioKernel K;
    K.init(p);
    ButterflyOptions bo;
    bo.eps = p.eps_bf;
    bo.leaf = p.leaf_bf;
    bo.nthreads = p.nthreads;
    bo.seed = p.seed ^ 0xB0F1ULL;
    bo.rank_align = p.bf_rank_align;
    const bool vb = p.verbose != 0;
    bo.verbose = vb;
    if (ids) bo.ids = ids(K);
    progress(vb, "d=%d n=%d: butterfly (eps_bf=%.1e)", p.d, p.n, p.eps_bf);
    Butterfly B = build_butterfly(K, bo);
    bo.ids = nullptr;  // frees the engine's device tables
    out.bf_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    out.bf_device_levels = B.device_levels;
    progress(vb, "butterfly done: L=%d nnz=%lld, %d levels on the device (%.1fs)", B.L, (long long)B.nnz(),
             B.device_levels, out.bf_seconds);
    out.d = p.d; out.n = p.n; out.N = B.N; out.L = B.L; out.Lm = B.Lm; out.m = B.m;
    out.perm = K.to_nat;
    out.prob = p;
    // e_a probe: K v on sampled rows, from the entries of K (the phase is only at hand
    // here for a caller-defined FIO)
    {
        const int64_t N = B.N;
        const int nr = (int)std::min<int64_t>(EA_ROWS, N);
        std::vector<int> rows;
        for (uint64_t t = 0; (int)rows.size() < nr; ++t) {
            const int r = (int)(splitmix64(p.seed ^ 0xEA0ULL ^ splitmix64(t)) % (uint64_t)N);
            if (std::find(rows.begin(), rows.end(), r) == rows.end()) rows.push_back(r);
        }
        std::sort(rows.begin(), rows.end());
        out.ea_rows = rows;
        out.ea_vecs.resize((size_t)N * EA_VECS);
        for (int64_t i = 0; i < N * EA_VECS; ++i)
            out.ea_vecs[i] = cd(gauss(p.seed ^ 0xEA1ULL, 2 * (uint64_t)i), gauss(p.seed ^ 0xEA1ULL, 2 * (uint64_t)i + 1));
        out.ea_ref.assign((size_t)nr * EA_VECS, cd(0));
        parallel_for(nr, p.nthreads, [&](int64_t i) {
            cd acc[EA_VECS] = {};
            for (int64_t q = 0; q < N; ++q) {
                const cd k = K.entry(rows[i], q);
                for (int v = 0; v < EA_VECS; ++v) acc[v] += k * out.ea_vecs[(size_t)v * N + q];
            }
            for (int v = 0; v < EA_VECS; ++v) out.ea_ref[(size_t)v * nr + i] = acc[v];
        });
    }
    // Peeling needs products with A = Kd^* Kd (section 5): on the GPU when available
    // (which forms the adjoint stages itself), else on the host.
    std::vector<Stage> adj;
    BlockApply A;
    if (gpu) {
        A = gpu(B.fwd);
    } else {
        for (int s = (int)B.fwd.size() - 1; s >= 0; --s) adj.push_back(adjoint_stage(B.fwd[s]));
        const int64_t N = B.N;
        const int nt = p.nthreads;
        // N and nt by value: the product outlives this block
        A = [&B, &adj, N, nt](const cd *x, cd *y, int nr) {
            std::vector<cd> t((size_t)N * nr);
            host_chain_apply(B.fwd, x, t.data(), nr, nt);
            host_chain_apply(adj, t.data(), y, nr, nt);
        };
    }
    PeelOptions po;
    po.eps = p.eps_peel;
    po.leaf = p.leaf_h;
    po.oversample = p.oversample;
    po.seed = p.seed ^ 0x9EE1ULL;
    po.nthreads = p.nthreads;
    po.verbose = vb;
    po.allow_shift = p.strict_hpd == 0;
    po.prescale = p.prescale_skel != 0;
    po.dev = skel;
    out.hif = (p.d == 1) ? build_hif_1d(A, B.N, po, p.eps_hif) : build_hif_2d(A, p.n, po, p.eps_hif);
    progress(vb,
             "inverse factors done: %zu steps, root %zu, %d shifted pivot blocks, %d IDs and %d nodes on the device "
             "(%.1fs)",
             out.hif.steps.size(), out.hif.root_idx.size(), out.hif.shifted, out.hif.device_ids, out.hif.device_nodes,
             std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
    out.fwd = std::move(B.fwd);
    out.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (vb) {
        const std::vector<uint64_t> fp = factor_fingerprints(out);
        progress(true, "  fingerprint of the butterfly: %016llx", (unsigned long long)fp.front());
        for (size_t k = 1; k + 1 < fp.size(); ++k)
            progress(true, "  fingerprint of inverse-factor step %zu: %016llx", k - 1, (unsigned long long)fp[k]);
        progress(true, "  fingerprint of the top-level inverse: %016llx", (unsigned long long)fp.back());
    }
}

// ---------------------------------------------------------------- file format
namespace {
const char MAGIC[8] = {'F', 'I', 'O', 'P', 'L', 'A', 'N', '1'};
const char EST_TAG[4] = {'E', 'S', 'T', '1'};

struct W {
    std::ofstream f;
    template <class T> void v(const T &x) { f.write((const char *)&x, sizeof(T)); }
    template <class T, class Al> void arr(const std::vector<T, Al> &a) {
        int64_t n = (int64_t)a.size();
        v(n);
        if (n) f.write((const char *)a.data(), sizeof(T) * n);
    }
    void mat(const Mat &M) {
        v(M.m); v(M.n);
        if (!M.a.empty()) f.write((const char *)M.a.data(), sizeof(cd) * M.a.size());
    }
};
struct R {
    std::ifstream f;
    template <class T> void v(T &x) {
        f.read((char *)&x, sizeof(T));
        if (!f) fail(FIO_ERR_IO, "truncated plan file");
    }
    template <class T, class Al> void arr(std::vector<T, Al> &a) {
        int64_t n = 0;
        v(n);
        if (n < 0 || n > (int64_t)1 << 40) fail(FIO_ERR_IO, "corrupt plan file");
        a.resize(n);
        if (n) f.read((char *)a.data(), sizeof(T) * n);
        if (!f) fail(FIO_ERR_IO, "truncated plan file");
    }
    void mat(Mat &M) {
        int m = 0, n = 0;
        v(m); v(n);
        if (m < 0 || n < 0) fail(FIO_ERR_IO, "corrupt plan file");
        M = Mat(m, n);
        if (!M.a.empty()) f.read((char *)M.a.data(), sizeof(cd) * M.a.size());
        if (!f) fail(FIO_ERR_IO, "truncated plan file");
    }
};
}  // namespace

void save_factors(const HostFactors &h, const std::string &path) {
    W w;
    w.f.open(path, std::ios::binary);
    if (!w.f) fail(FIO_ERR_IO, "cannot open " + path + " for writing");
    w.f.write(MAGIC, 8);
    const fio_problem &p = h.prob;
    w.v(p.d); w.v(p.n); w.v((int)p.phase); w.v(p.c_div); w.v(p.eps); w.v(p.eps_bf);
    w.v(p.eps_peel); w.v(p.eps_hif); w.v(p.leaf_bf); w.v(p.leaf_h); w.v(p.oversample);
    w.v(p.seed);
    w.v(h.N); w.v(h.L); w.v(h.Lm); w.v(h.m);
    w.arr(h.perm);
    w.v((int)h.fwd.size());
    for (const Stage &s : h.fwd) {
        w.v(s.n_out); w.v(s.n_in); w.v(s.r_out); w.v(s.r_in); w.v(s.fan);
        w.arr(s.in_idx);
        w.arr(s.A);
    }
    w.v(h.hif.N);
    w.v((int)h.hif.steps.size());
    for (const HifStep &st : h.hif.steps) {
        w.v((int)st.nodes.size());
        for (const HifNode &nd : st.nodes) {
            w.arr(nd.idx_r); w.arr(nd.idx_s);
            w.mat(nd.T); w.mat(nd.Linv); w.mat(nd.M);
        }
    }
    w.arr(h.hif.root_idx);
    w.mat(h.hif.A0inv);
    w.v(h.hif.max_rank_h);
    w.v(h.build_seconds);
    // trailer (absent in files written before it): error estimates and the e_a probe
    w.f.write(EST_TAG, 4);
    w.v(h.e_a_est); w.v(h.e_s_est); w.v(h.cond_est);
    w.arr(h.ea_rows); w.arr(h.ea_vecs); w.arr(h.ea_ref);
    if (!w.f) fail(FIO_ERR_IO, "write failed: " + path);
}

void load_factors(const std::string &path, HostFactors &h) {
    R r;
    r.f.open(path, std::ios::binary);
    if (!r.f) fail(FIO_ERR_IO, "cannot open " + path);
    char mg[8];
    r.f.read(mg, 8);
    if (!r.f || std::memcmp(mg, MAGIC, 8) != 0) fail(FIO_ERR_IO, "not a plan file: " + path);
    fio_problem &p = h.prob;
    std::memset(&p, 0, sizeof(p));
    int ph = 0;
    r.v(p.d); r.v(p.n); r.v(ph); p.phase = (fio_phase_id)ph;
    r.v(p.c_div); r.v(p.eps); r.v(p.eps_bf); r.v(p.eps_peel); r.v(p.eps_hif);
    r.v(p.leaf_bf); r.v(p.leaf_h); r.v(p.oversample); r.v(p.seed);
    h.d = p.d; h.n = p.n;
    r.v(h.N); r.v(h.L); r.v(h.Lm); r.v(h.m);
    r.arr(h.perm);
    if ((int64_t)h.perm.size() != h.N) fail(FIO_ERR_IO, "corrupt plan file (perm)");
    int ns = 0;
    r.v(ns);
    if (ns < 0 || ns > 4096) fail(FIO_ERR_IO, "corrupt plan file (stages)");
    h.fwd.resize(ns);
    for (Stage &s : h.fwd) {
        r.v(s.n_out); r.v(s.n_in); r.v(s.r_out); r.v(s.r_in); r.v(s.fan);
        r.arr(s.in_idx);
        r.arr(s.A);
        if ((int64_t)s.in_idx.size() != s.n_out * s.fan || (int64_t)s.A.size() != s.nnz())
            fail(FIO_ERR_IO, "corrupt plan file (stage sizes)");
        for (int32_t v : s.in_idx)
            if (v < 0 || v >= s.n_in) fail(FIO_ERR_IO, "corrupt plan file (stage index)");
    }
    r.v(h.hif.N);
    int nst = 0;
    r.v(nst);
    if (nst < 0 || nst > 4096) fail(FIO_ERR_IO, "corrupt plan file (hif)");
    h.hif.steps.resize(nst);
    for (HifStep &st : h.hif.steps) {
        int nn = 0;
        r.v(nn);
        if (nn < 0) fail(FIO_ERR_IO, "corrupt plan file (hif nodes)");
        st.nodes.resize(nn);
        for (HifNode &nd : st.nodes) {
            r.arr(nd.idx_r); r.arr(nd.idx_s);
            r.mat(nd.T); r.mat(nd.Linv); r.mat(nd.M);
            const int nr = (int)nd.idx_r.size(), nsk = (int)nd.idx_s.size();
            if (nd.T.m != nsk || nd.T.n != nr || nd.Linv.m != nr || nd.Linv.n != nr ||
                nd.M.m != nsk || nd.M.n != nr)
                fail(FIO_ERR_IO, "corrupt plan file (hif blocks)");
            for (int v : nd.idx_r) if (v < 0 || v >= h.N) fail(FIO_ERR_IO, "corrupt plan file (idx)");
            for (int v : nd.idx_s) if (v < 0 || v >= h.N) fail(FIO_ERR_IO, "corrupt plan file (idx)");
        }
    }
    r.arr(h.hif.root_idx);
    r.mat(h.hif.A0inv);
    for (int v : h.hif.root_idx) if (v < 0 || v >= h.N) fail(FIO_ERR_IO, "corrupt plan file (root)");
    if (h.hif.A0inv.m != (int)h.hif.root_idx.size()) fail(FIO_ERR_IO, "corrupt plan file (root)");
    r.v(h.hif.max_rank_h);
    r.v(h.build_seconds);
    char tag[4];
    r.f.read(tag, 4);
    if (r.f.gcount() == 0 && r.f.eof()) return;  // no trailer
    if (r.f.gcount() != 4 || std::memcmp(tag, EST_TAG, 4) != 0) fail(FIO_ERR_IO, "corrupt plan file (trailer)");
    r.v(h.e_a_est); r.v(h.e_s_est); r.v(h.cond_est);
    r.arr(h.ea_rows); r.arr(h.ea_vecs); r.arr(h.ea_ref);
    for (int v : h.ea_rows) if (v < 0 || v >= h.N) fail(FIO_ERR_IO, "corrupt plan file (probe rows)");
    if ((int64_t)h.ea_vecs.size() != (h.ea_rows.empty() ? 0 : h.N * EA_VECS) ||
        h.ea_ref.size() != h.ea_rows.size() * EA_VECS)
        fail(FIO_ERR_IO, "corrupt plan file (probe sizes)");
}

}  // namespace fio
