// Host-only exercise of the construction code for sanitizer builds (address and
// undefined-behaviour checks of the host C++): small problems of every phase are
// built with the host decompositions and host products, their factors applied,
// written to a plan file, read back and compared, and corrupt files rejected.
// Prints one line per case and "host check ok" at the end; exits non-zero on a
// mismatch or an unexpected error.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <string>
#include <vector>

#include "plan.hpp"

using namespace fio;

static double rel_diff(const std::vector<cd> &a, const std::vector<cd> &b) {
    double num = 0, den = 0;
    for (size_t i = 0; i < a.size(); ++i) {
        num += std::norm(a[i] - b[i]);
        den += std::norm(b[i]);
    }
    return std::sqrt(num / (den > 0 ? den : 1));
}

static std::vector<cd> probe(int64_t N, int nrhs) {
    std::vector<cd> x((size_t)N * nrhs);
    for (size_t i = 0; i < x.size(); ++i) x[i] = cd(gauss(7, 2 * i), gauss(7, 2 * i + 1));
    return x;
}

// Kd x through the stages (tree order, point-major, nrhs columns).
static std::vector<cd> apply_fwd(const HostFactors &h, const std::vector<cd> &x, int nrhs) {
    std::vector<cd> y((size_t)h.N * nrhs);
    host_chain_apply(h.fwd, x.data(), y.data(), nrhs, 2);
    return y;
}

static int check_case(const char *name, fio_problem p, const std::string &dir) {
    HostFactors h;
    build_host_factors(p, h, PeelApplyFactory(), BatchedIdFactory());
    const int nrhs = 3;
    const std::vector<cd> x = probe(h.N, nrhs);
    const std::vector<cd> y = apply_fwd(h, x, nrhs);
    const std::string path = dir + "/" + name + ".fio";
    save_factors(h, path);
    HostFactors g;
    load_factors(path, g);
    const double d = rel_diff(apply_fwd(g, x, nrhs), y);
    size_t nodes = 0;
    for (const HifStep &st : g.hif.steps) nodes += st.nodes.size();
    std::printf("%s: N=%lld stages=%zu hif steps=%zu nodes=%zu root=%zu reload diff %.1e\n", name,
                (long long)h.N, h.fwd.size(), g.hif.steps.size(), nodes, g.hif.root_idx.size(), d);
    if (d != 0.0 || g.hif.steps.size() != h.hif.steps.size() || g.hif.root_idx != h.hif.root_idx) {
        std::printf("%s: reloaded factors differ\n", name);
        return 1;
    }
    // a truncated copy must be rejected with an I/O error
    std::ifstream in(path, std::ios::binary);
    std::string bytes((std::istreambuf_iterator<char>(in)), std::istreambuf_iterator<char>());
    const std::string cut = dir + "/" + name + "_cut.fio";
    std::ofstream(cut, std::ios::binary).write(bytes.data(), (std::streamsize)(bytes.size() / 2));
    try {
        HostFactors bad;
        load_factors(cut, bad);
        std::printf("%s: truncated plan file accepted\n", name);
        return 1;
    } catch (const Error &e) {
        if (e.status != FIO_ERR_IO) {
            std::printf("%s: truncated plan file gave status %d\n", name, (int)e.status);
            return 1;
        }
    }
    return 0;
}

int main(int argc, char **argv) {
    const std::string dir = argc > 1 ? argv[1] : ".";
    int bad = 0;
    fio_problem p;
    std::memset(&p, 0, sizeof(p));
    p.device = -1;
    p.nthreads = 4;
    p.seed = 11;

    p.d = 1; p.n = 256; p.phase = FIO_PHASE_1D_EX1; p.eps = 1e-6;
    bad += check_case("ex1_n256", p, dir);
    p.n = 128; p.phase = FIO_PHASE_LINEAR;
    bad += check_case("linear_n128", p, dir);
    p.n = 512; p.phase = FIO_PHASE_1D_EX2; p.eps = 1e-5;
    bad += check_case("ex2_n512", p, dir);
    p.d = 2; p.n = 16; p.phase = FIO_PHASE_2D_RADON; p.eps = 1e-4;
    bad += check_case("radon_n16", p, dir);

    // argument errors surface as FIO_ERR_ARG, not as undefined behaviour
    fio_problem q = p;
    q.n = 12;
    try {
        HostFactors h;
        build_host_factors(q, h, PeelApplyFactory(), BatchedIdFactory());
        std::printf("n=12 accepted\n");
        ++bad;
    } catch (const Error &e) {
        if (e.status != FIO_ERR_ARG) ++bad;
    }
    if (bad) return 1;
    std::printf("host check ok\n");
    return 0;
}
