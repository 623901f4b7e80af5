// C ABI: plan lifetime, device images of the factors, and the apply/solve drivers.
// Every floating-point step of an apply runs in the kernels of kernels.hip; the
// host only enqueues work on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <complex>
#include <cmath>
#include <map>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "fio.h"
#include "kernels.hpp"
#include "plan.hpp"

using namespace fio;

namespace {

thread_local std::string g_err;
void forget_multi_tunes(fio_plan p);  // drops the multi-instance tunes that name a plan

// Named ranges of the host-side phases (solve, chains, Gd sweeps and steps,
// iterations) for a profiler's marker trace, when switched on by fio_set_trace.
std::atomic<int> g_trace(0);
struct TraceRange {
    bool on;
    explicit TraceRange(const char *fmt, ...) : on(g_trace.load(std::memory_order_relaxed) != 0) {
        if (!on) return;
        char buf[96];
        va_list ap;
        va_start(ap, fmt);
        std::vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        roctxRangePushA(buf);
    }
    ~TraceRange() {
        if (on) roctxRangePop();
    }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

#define HIPC(x)                                                                          \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess)                                                            \
            fail(e_ == hipErrorOutOfMemory ? FIO_ERR_NOMEM : FIO_ERR_DEVICE,             \
                 std::string(#x) + ": " + hipGetErrorString(e_));                        \
    } while (0)

// Device allocation owned by a plan.
struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;  // owns its device memory: moved, never copied
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), bytes(o.bytes) {
        o.p = nullptr;
        o.bytes = 0;
    }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) {
            if (p) (void)hipFree(p);
            p = o.p;
            bytes = o.bytes;
            o.p = nullptr;
            o.bytes = 0;
        }
        return *this;
    }
    ~DBuf() {
        if (p) (void)hipFree(p);
    }
    void alloc(size_t b) {
        if (p) { (void)hipFree(p); p = nullptr; bytes = 0; }
        if (b == 0) return;
        HIPC(hipMalloc(&p, b));
        bytes = b;
    }
    void upload(const void *src, size_t b) {
        alloc(b);
        if (b) HIPC(hipMemcpy(p, src, b, hipMemcpyHostToDevice));
    }
};

template <class T> struct DStageStore {
    DBuf idx, A64, A128;
    bool gone64 = false, gone128 = false;  // released by fio_plan_trim
    StageDev view(bool dbl, const Stage &s) const {
        StageDev v;
        v.n_out = s.n_out; v.n_in = s.n_in; v.r_out = s.r_out; v.r_in = s.r_in; v.fan = s.fan;
        v.idx = (const int32_t *)idx.p;
        v.A = dbl ? A128.p : A64.p;
        if (dbl ? gone128 : gone64)
            fail(FIO_ERR_UNSUPPORTED, std::string("the ") + (dbl ? "complex128" : "complex64") +
                                          " image of this chain was released by fio_plan_trim");
        return v;
    }
    bool has(bool dbl) const { return !(dbl ? gone128 : gone64); }
};

struct DHifStore {
    DBuf desc, idx, m64, m128, h64, h128, tr, ts, tr2, ts2, tr4, ts4;
    bool gone128 = false;  // released by fio_plan_trim
    HifStepDev view(bool dbl) const {
        HifStepDev v = base;
        v.desc = (const int64_t *)desc.p;
        v.idx = (const int32_t *)idx.p;
        v.mat = dbl ? m128.p : m64.p;
        v.matH = dbl ? h128.p : h64.p;
        v.tiles_r = (const int32_t *)tr.p;
        v.tiles_s = (const int32_t *)ts.p;
        v.tiles_r2 = (const int32_t *)tr2.p;
        v.tiles_s2 = (const int32_t *)ts2.p;
        v.tiles_r4 = (const int32_t *)tr4.p;
        v.tiles_s4 = (const int32_t *)ts4.p;
        if (dbl && gone128) fail(FIO_ERR_UNSUPPORTED, "the complex128 image of Gd was released by fio_plan_trim");
        return v;
    }
    bool has(bool dbl) const { return !(dbl && gone128); }
    HifStepDev base;
};

// Workgroup table of a fused stage pair (a, b), or nothing when the pair cannot
// be fused.  Stage-a blocks are grouped with the stage-b blocks that read them and
// with the stage-a blocks that share their inputs; in a butterfly these closed
// groups hold at most fan^2 blocks.  Whole groups are packed into workgroups of at
// most four stage-a and four stage-b blocks.
struct DPair {
    DBuf tab, tab_s;
    int64_t n_wg = 0, n_wg_s = 0;
    bool ok = false;
    DBuf tab3;           // stages (s, s+1, s+2) fused (StageTripleDev), if they form stacked groups
    int64_t n_wg3 = 0;
};

// Table of the stacked variant: one closed group per workgroup, whose stage-a blocks
// and stage-b blocks each split into two pairs of siblings (equal input lists).
// Returns false if some group does not.
bool build_stacked_table(const Stage &a, const Stage &b, const std::vector<int32_t> &tab,
                         std::vector<int32_t> &out) {
    out.clear();
    if (!stage_pair_stackable(a.r_out, b.r_out) || b.fan > 2) return false;
    auto same_in = [](const Stage &s, int32_t x, int32_t y) {
        for (int q = 0; q < s.fan; ++q)
            if (s.in_idx[(int64_t)x * s.fan + q] != s.in_idx[(int64_t)y * s.fan + q]) return false;
        return true;
    };
    // pair up four blocks (p[0..3]) into sibling pairs; false if impossible
    auto pairs = [&](const Stage &s, const int32_t *p, int32_t *o) {
        for (int i = 0; i < 4; ++i)
            if (p[i] < 0) return false;
        const int other[3][2] = {{2, 3}, {1, 3}, {1, 2}};
        for (int j = 1; j < 4; ++j) {
            if (!same_in(s, p[0], p[j])) continue;
            const int u = other[j - 1][0], v = other[j - 1][1];
            if (!same_in(s, p[u], p[v])) continue;
            o[0] = p[0]; o[1] = p[j]; o[2] = p[u]; o[3] = p[v];
            return true;
        }
        return false;
    };
    for (size_t g = 0; g < tab.size(); g += 16) {
        const int32_t *t = tab.data() + g;
        int32_t w[16];
        for (int i = 0; i < 16; ++i) w[i] = -1;
        if (!pairs(a, t, w) || !pairs(b, t + 4, w + 4)) return false;
        for (int pr = 0; pr < 2; ++pr) {
            const int32_t o = w[4 + 2 * pr];
            for (int q = 0; q < b.fan; ++q) {
                const int32_t m = b.in_idx[(int64_t)o * b.fan + q];
                int slot = -1;
                for (int i = 0; i < 4; ++i)
                    if (w[i] == m) slot = i;
                if (slot < 0) return false;
                w[8 + 2 * pr + q] = slot;
            }
        }
        out.insert(out.end(), w, w + 16);
    }
    return true;
}

bool build_pair_table(const Stage &a, const Stage &b, std::vector<int32_t> &tab) {
    tab.clear();
    if (b.n_in != a.n_out || b.r_in != a.r_out || !stage_pair_fusable(a.r_out, b.r_out, b.fan) || a.fan > 4 ||
        a.r_in < 1)
        return false;
    const int64_t nm = a.n_out;
    std::vector<int64_t> par(nm);
    for (int64_t i = 0; i < nm; ++i) par[i] = i;
    auto find = [&](int64_t x) {
        while (par[x] != x) { par[x] = par[par[x]]; x = par[x]; }
        return x;
    };
    auto unite = [&](int64_t x, int64_t y) { x = find(x); y = find(y); if (x != y) par[x] = y; };
    for (int64_t o = 0; o < b.n_out; ++o)
        for (int q = 1; q < b.fan; ++q) unite(b.in_idx[o * b.fan], b.in_idx[o * b.fan + q]);
    std::vector<int64_t> first_user(a.n_in, -1);
    for (int64_t o = 0; o < nm; ++o)
        for (int q = 0; q < a.fan; ++q) {
            const int32_t i = a.in_idx[o * a.fan + q];
            if (first_user[i] < 0) first_user[i] = o;
            else unite(first_user[i], o);
        }
    // members of each group, in block order
    std::map<int64_t, std::pair<std::vector<int32_t>, std::vector<int32_t>>> groups;
    for (int64_t m = 0; m < nm; ++m) groups[find(m)].first.push_back((int32_t)m);
    for (int64_t o = 0; o < b.n_out; ++o) groups[find(b.in_idx[o * b.fan])].second.push_back((int32_t)o);
    std::vector<std::pair<std::vector<int32_t>, std::vector<int32_t>>> ordered;
    for (auto &g : groups) {
        if (g.second.first.size() > 4 || g.second.second.size() > 4) return false;
        ordered.push_back(std::move(g.second));
    }
    std::sort(ordered.begin(), ordered.end(),
              [](const auto &x, const auto &y) { return x.first[0] < y.first[0]; });
    std::vector<int32_t> mids, outs;
    auto flush = [&] {
        if (mids.empty() && outs.empty()) return;
        int32_t w[16];
        for (int i = 0; i < 16; ++i) w[i] = -1;
        for (size_t i = 0; i < mids.size(); ++i) w[i] = mids[i];
        for (size_t i = 0; i < outs.size(); ++i) {
            w[4 + i] = outs[i];
            for (int q = 0; q < b.fan; ++q) {
                const int32_t m = b.in_idx[(int64_t)outs[i] * b.fan + q];
                const auto it = std::find(mids.begin(), mids.end(), m);
                if (it == mids.end()) fail(FIO_ERR_DEVICE, "fused stage table: group is not closed");
                w[8 + 2 * i + q] = (int32_t)(it - mids.begin());
            }
        }
        tab.insert(tab.end(), w, w + 16);
        mids.clear();
        outs.clear();
    };
    for (auto &g : ordered) {
        if (mids.size() + g.first.size() > 4 || outs.size() + g.second.size() > 4) flush();
        mids.insert(mids.end(), g.first.begin(), g.first.end());
        outs.insert(outs.end(), g.second.begin(), g.second.end());
    }
    flush();
    return true;
}

// Table of three consecutive stages a, b, c fused (StageTripleDev): the closed groups
// of the three stages (stage-c outputs read only stage-b outputs of the group, which
// read only its stage-a outputs), each of exactly four blocks per stage, whose
// stage-b and stage-c blocks split into two sibling pairs (equal input lists).
// Returns false if some group does not.
bool build_triple_table(const Stage &a, const Stage &b, const Stage &c, std::vector<int32_t> &out) {
    out.clear();
    if (b.n_in != a.n_out || c.n_in != b.n_out || b.r_in != a.r_out || c.r_in != b.r_out) return false;
    if (std::max({a.r_out, b.r_out, c.r_out}) > 32 || a.r_out < 1 || b.r_out < 1 || c.r_out < 1 || a.r_in < 1)
        return false;
    if (a.fan < 1 || a.fan > 4 || b.fan < 1 || b.fan > 2 || c.fan < 1 || c.fan > 2) return false;
    const int64_t na = a.n_out, nb = b.n_out, nc = c.n_out;
    std::vector<int64_t> par(na + nb + nc);
    for (size_t i = 0; i < par.size(); ++i) par[i] = (int64_t)i;
    auto find = [&](int64_t x) {
        while (par[x] != x) { par[x] = par[par[x]]; x = par[x]; }
        return x;
    };
    auto unite = [&](int64_t x, int64_t y) { x = find(x); y = find(y); if (x != y) par[x] = y; };
    for (int64_t m = 0; m < nb; ++m)
        for (int q = 0; q < b.fan; ++q) unite(na + m, b.in_idx[m * b.fan + q]);
    for (int64_t o = 0; o < nc; ++o)
        for (int q = 0; q < c.fan; ++q) unite(na + nb + o, na + c.in_idx[o * c.fan + q]);
    struct Group {
        std::vector<int32_t> a, b, c;
    };
    std::map<int64_t, Group> groups;
    for (int64_t i = 0; i < na; ++i) groups[find(i)].a.push_back((int32_t)i);
    for (int64_t i = 0; i < nb; ++i) groups[find(na + i)].b.push_back((int32_t)i);
    for (int64_t i = 0; i < nc; ++i) groups[find(na + nb + i)].c.push_back((int32_t)i);
    auto same_in = [](const Stage &st, int32_t x, int32_t y) {
        for (int q = 0; q < st.fan; ++q)
            if (st.in_idx[(int64_t)x * st.fan + q] != st.in_idx[(int64_t)y * st.fan + q]) return false;
        return true;
    };
    // four blocks into two sibling pairs, adjacent in the returned order
    auto pairs = [&](const Stage &st, const std::vector<int32_t> &v, std::vector<int32_t> &o) {
        o.clear();
        for (size_t j = 1; j < 4; ++j) {
            if (!same_in(st, v[0], v[j])) continue;
            const size_t u = j == 1 ? 2 : 1, w = j == 3 ? 2 : 3;
            if (!same_in(st, v[u], v[w])) continue;
            o = {v[0], v[j], v[u], v[w]};
            return true;
        }
        return false;
    };
    // slots of each pair's inputs (positions in the previous stage's list)
    auto slots = [](const Stage &st, const std::vector<int32_t> &blocks, const std::vector<int32_t> &prev,
                    int32_t *w) {
        for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q) {
                w[2 * p + q] = -1;
                if (q >= st.fan) continue;
                const int32_t m = st.in_idx[(int64_t)blocks[2 * p] * st.fan + q];
                const auto it = std::find(prev.begin(), prev.end(), m);
                if (it == prev.end()) return false;
                w[2 * p + q] = (int32_t)(it - prev.begin());
            }
        return true;
    };
    std::vector<std::pair<int32_t, std::vector<int32_t>>> rows;
    for (auto &kv : groups) {
        const Group &gr = kv.second;
        if (gr.a.size() != 4 || gr.b.size() != 4 || gr.c.size() != 4) return false;
        std::vector<int32_t> pa, pb, pc;
        pa = gr.a;  // the stage-a blocks run one by one
        if (!pairs(b, gr.b, pb) || !pairs(c, gr.c, pc)) return false;
        std::vector<int32_t> w(STAGE_TRIPLE_TAB, -1);
        std::copy(pa.begin(), pa.end(), w.begin());
        std::copy(pb.begin(), pb.end(), w.begin() + 4);
        if (!slots(b, pb, pa, w.data() + 8)) return false;
        std::copy(pc.begin(), pc.end(), w.begin() + 12);
        if (!slots(c, pc, pb, w.data() + 16)) return false;
        rows.push_back({pa[0], std::move(w)});
    }
    std::sort(rows.begin(), rows.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
    for (auto &r : rows) out.insert(out.end(), r.second.begin(), r.second.end());
    return true;
}

// b = a rounded to complex FP32 (round to nearest, as the host conversion).
__global__ __launch_bounds__(256) void k_to_c64(const double2 *a, float2 *b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double2 v = a[i];
        b[i] = make_float2((float)v.x, (float)v.y);
    }
}

unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1 << 16)); }

// Complex FP32 copy of a complex FP64 device array (synchronous).
void to_c64(const DBuf &b128, DBuf &b64) {
    const int64_t n = (int64_t)(b128.bytes / sizeof(cd));
    b64.alloc((size_t)n * 8);
    if (n == 0) return;
    hipLaunchKernelGGL(k_to_c64, dim3(grid_for(n)), dim3(256), 0, 0, (const double2 *)b128.p, (float2 *)b64.p, n);
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(0));
}

// FP64 array to the device, with its complex FP32 copy formed there.
template <class Al> void upload_complex(DBuf &b64, DBuf &b128, const std::vector<cd, Al> &a) {
    b128.upload(a.data(), a.size() * sizeof(cd));
    to_c64(b128, b64);
}

// Blocks of the adjoint stage (see adjoint_index): element (b, sl*r_out_s + a) of
// target block `in` is conj of element (a, q*r_in_s + b) of source block o, where
// src_of[in*fan_t + sl] = o*fan_s + q.  One thread per target element.
__global__ __launch_bounds__(256) void k_adjoint_blocks(const double2 *src, double2 *dst, const int64_t *src_of,
                                                        int64_t n_tgt, int fan_t, int r_out_s, int r_in_s,
                                                        int fan_s) {
    const int64_t cols = (int64_t)fan_t * r_out_s, per = cols * r_in_s, total = n_tgt * per;
    const int64_t blk_s = (int64_t)r_out_s * fan_s * r_in_s;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t in = e / per, rem = e - in * per;
        const int64_t c = rem / r_in_s;
        const int b = (int)(rem - c * r_in_s);
        const int sl = (int)(c / r_out_s), a = (int)(c - (int64_t)sl * r_out_s);
        const int64_t oq = src_of[in * fan_t + sl];
        const int64_t o = oq / fan_s;
        const int q = (int)(oq - o * fan_s);
        const double2 v = src[o * blk_s + a + ((int64_t)q * r_in_s + b) * r_out_s];
        dst[e] = make_double2(v.x, -v.y);
    }
}

}  // namespace

struct fio_plan_s {
    HostFactors host;
    int device = -1;
    std::vector<Stage> adj;                   // host adjoint stages (Kd^*)
    std::vector<DStageStore<int>> dfwd, dadj;
    std::vector<DPair> pfwd, padj;            // fused pairs (s, s+1) of each chain
    std::vector<DHifStore> dhif;
    DBuf root_idx, A0inv, perm, root_stage_idx;
    int s0 = 0;
    int64_t max_coef = 0;                     // longest coefficient vector between stages
    int64_t device_bytes = 0;
    // workspace (grown on demand)
    int ws_nrhs = 0;
    bool ws_captured = false;                 // a call ran under stream capture
    DBuf P, Q, V1, V2, V3, W, U, X, R, Z, Pv, red, scal, HT, RI, RO;
    DBuf GV, GH;                              // GMRES basis ((m+1) vectors) and Hessenberg entries
    int64_t gv_vecs = 0, gv_cnt = 0;
    std::mutex mu;
    // Autotuned choices keyed by (dtype, nrhs): stage kernel variant per stage of the
    // forward and adjoint chains, which consecutive stages run fused, and per
    // skeletonization step 0 = LDS kernel, 1 = matrix-core GEMMs.
    // fwd_pair/adj_pair[s] > 0: stages s and s+1 run fused with that variant;
    // fwd_triple/adj_triple[s] > 0: stages s, s+1 and s+2 run fused; hif[k]: the
    // choice of hif_step.
    struct Tune {
        std::vector<int> fwd, adj, hif, fwd_pair, adj_pair, fwd_triple, adj_triple;
        int root = -1;  // stage variant of the FP64 top-level block
    };
    std::map<std::pair<int, int>, Tune> tune;
    const Tune *tuned(bool dbl, int nrhs) const {
        auto it = tune.find({dbl ? 1 : 0, nrhs});
        return it == tune.end() ? nullptr : &it->second;
    }
};

namespace {

void count_bytes(fio_plan p) {
    int64_t b = 0;
    for (auto &s : p->dfwd) b += s.idx.bytes + s.A64.bytes + s.A128.bytes;
    for (auto &s : p->dadj) b += s.idx.bytes + s.A64.bytes + s.A128.bytes;
    for (auto &q : p->pfwd) b += q.tab.bytes + q.tab_s.bytes + q.tab3.bytes;
    for (auto &q : p->padj) b += q.tab.bytes + q.tab_s.bytes + q.tab3.bytes;
    for (auto &h : p->dhif) b += h.desc.bytes + h.idx.bytes + h.m64.bytes + h.m128.bytes + h.h64.bytes + h.h128.bytes +
                                   h.tr.bytes + h.ts.bytes + h.tr2.bytes + h.ts2.bytes + h.tr4.bytes + h.ts4.bytes;
    b += p->root_idx.bytes + p->A0inv.bytes + p->perm.bytes;
    p->device_bytes = b;
}

void upload_stages(const std::vector<Stage> &st, std::vector<DStageStore<int>> &d) {
    d.resize(st.size());
    for (size_t i = 0; i < st.size(); ++i) {
        d[i].idx.upload(st[i].in_idx.data(), st[i].in_idx.size() * sizeof(int32_t));
        upload_complex(d[i].A64, d[i].A128, st[i].A);
    }
}

// The adjoint chain formed on the device from the forward one: host index parts
// (sizes and in_idx, no blocks) in `adj`, device blocks in `dadj` (adj[k] is the
// adjoint of fwd[S-1-k]).
void device_adjoints(const std::vector<Stage> &fwd, const std::vector<DStageStore<int>> &dfwd,
                     std::vector<Stage> &adj, std::vector<DStageStore<int>> &dadj) {
    const size_t S = fwd.size();
    adj.assign(S, Stage());
    dadj.resize(S);
    std::vector<int64_t> src_of;
    for (size_t k = 0; k < S; ++k) {
        const Stage &f = fwd[S - 1 - k];
        Stage &t = adj[k];
        t = adjoint_index(f, src_of);
        DStageStore<int> &d = dadj[k];
        d.idx.upload(t.in_idx.data(), t.in_idx.size() * sizeof(int32_t));
        DBuf so;
        so.upload(src_of.data(), src_of.size() * sizeof(int64_t));
        const int64_t total = t.nnz();
        d.A128.alloc((size_t)total * sizeof(cd));
        if (total > 0) {
            hipLaunchKernelGGL(k_adjoint_blocks, dim3(grid_for(total)), dim3(256), 0, 0,
                               (const double2 *)dfwd[S - 1 - k].A128.p, (double2 *)d.A128.p,
                               (const int64_t *)so.p, t.n_out, t.fan, f.r_out, f.r_in, f.fan);
            HIPC(hipGetLastError());
            HIPC(hipStreamSynchronize(0));
        }
        to_c64(d.A128, d.A64);
    }
}

// Host index parts of the adjoint chain (a plan without a device, or one whose
// device chains are formed later).
std::vector<Stage> adjoint_indexes(const std::vector<Stage> &fwd) {
    std::vector<Stage> adj;
    std::vector<int64_t> src_of;
    for (int s = (int)fwd.size() - 1; s >= 0; --s) adj.push_back(adjoint_index(fwd[s], src_of));
    return adj;
}

// Both chains on the device (the plan's images, also used by the peeling products).
struct DeviceChains {
    std::vector<Stage> adj;                   // index parts of the adjoint stages
    std::vector<DStageStore<int>> dfwd, dadj;
};

void upload_chains(const std::vector<Stage> &fwd, DeviceChains &c) {
    upload_stages(fwd, c.dfwd);
    device_adjoints(fwd, c.dfwd, c.adj, c.dadj);
}

void upload_pairs(const std::vector<Stage> &st, std::vector<DPair> &d) {
    d.clear();  // default-constructed entries: DBuf is not copied
    d.resize(st.empty() ? 0 : st.size() - 1);
    std::vector<int32_t> tab;
    for (size_t s = 0; s + 1 < st.size(); ++s) {
        if (!build_pair_table(st[s], st[s + 1], tab)) continue;
        d[s].tab.upload(tab.data(), tab.size() * sizeof(int32_t));
        d[s].n_wg = (int64_t)tab.size() / 16;
        d[s].ok = true;
        std::vector<int32_t> ts;
        if (build_stacked_table(st[s], st[s + 1], tab, ts)) {
            d[s].tab_s.upload(ts.data(), ts.size() * sizeof(int32_t));
            d[s].n_wg_s = (int64_t)ts.size() / 16;
        }
    }
    std::vector<int32_t> t3;
    for (size_t s = 0; s + 2 < st.size(); ++s) {
        if (!build_triple_table(st[s], st[s + 1], st[s + 2], t3)) continue;
        d[s].tab3.upload(t3.data(), t3.size() * sizeof(int32_t));
        d[s].n_wg3 = (int64_t)t3.size() / STAGE_TRIPLE_TAB;
    }
}

void upload_plan(fio_plan p) {
    HIPC(hipSetDevice(p->device));
    const HostFactors &h = p->host;
    if (p->dfwd.empty()) {  // not formed by the build already
        DeviceChains c;
        upload_chains(h.fwd, c);
        p->adj.swap(c.adj);
        p->dfwd.swap(c.dfwd);
        p->dadj.swap(c.dadj);
    }
    upload_pairs(h.fwd, p->pfwd);
    upload_pairs(p->adj, p->padj);
    p->max_coef = h.N;
    for (auto &s : h.fwd) {
        p->max_coef = std::max<int64_t>(p->max_coef, s.n_out * s.r_out);
        p->max_coef = std::max<int64_t>(p->max_coef, s.n_in * s.r_in);
    }
    p->dhif.resize(h.hif.steps.size());
    for (size_t k = 0; k < h.hif.steps.size(); ++k) {
        const HifStep &st = h.hif.steps[k];
        std::vector<int64_t> desc;
        std::vector<int32_t> idx;
        std::vector<cd> mat, matH;
        int mr = 0, ms = 0, mv = 0, mm = 0;
        // row tiles of 16, 32 and 64 rows: pairs (node, first row)
        std::vector<int32_t> tr, ts, tr2, ts2, tr4, ts4;
        for (size_t v = 0; v < st.nodes.size(); ++v) {
            const int nr = (int)st.nodes[v].idx_r.size(), ns = (int)st.nodes[v].idx_s.size();
            for (int w : {16, 32, 64}) {
                auto &lr = w == 16 ? tr : (w == 32 ? tr2 : tr4);
                auto &ls = w == 16 ? ts : (w == 32 ? ts2 : ts4);
                for (int r0 = 0; r0 < nr; r0 += w) { lr.push_back((int32_t)v); lr.push_back(r0); }
                for (int r0 = 0; r0 < ns; r0 += w) { ls.push_back((int32_t)v); ls.push_back(r0); }
            }
        }
        for (const HifNode &nd : st.nodes) {
            const int nr = (int)nd.idx_r.size(), ns = (int)nd.idx_s.size();
            mr = std::max(mr, nr);
            ms = std::max(ms, ns);
            mv = std::max(mv, 2 * nr + ns);
            mm = std::max(mm, 2 * ns * nr + nr * nr);
            desc.push_back(nr);
            desc.push_back(ns);
            desc.push_back((int64_t)idx.size());
            desc.push_back((int64_t)mat.size());
            idx.insert(idx.end(), nd.idx_r.begin(), nd.idx_r.end());
            idx.insert(idx.end(), nd.idx_s.begin(), nd.idx_s.end());
            mat.insert(mat.end(), nd.T.a.begin(), nd.T.a.end());
            mat.insert(mat.end(), nd.Linv.a.begin(), nd.Linv.a.end());
            mat.insert(mat.end(), nd.M.a.begin(), nd.M.a.end());
            // conjugate transposes, same offsets: T^* and M^* are nr x ns, Linv^* nr x nr
            for (const Mat *B : {&nd.T, &nd.Linv, &nd.M})
                for (int j = 0; j < B->m; ++j)
                    for (int i = 0; i < B->n; ++i) matH.push_back(std::conj((*B)(j, i)));
        }
        DHifStore &d = p->dhif[k];
        d.base.n_nodes = (int64_t)st.nodes.size();
        d.base.max_nr = mr;
        d.base.max_ns = ms;
        d.base.max_vec = mv;
        d.base.max_mat = mm;
        d.tr.upload(tr.data(), tr.size() * sizeof(int32_t));
        d.ts.upload(ts.data(), ts.size() * sizeof(int32_t));
        d.tr2.upload(tr2.data(), tr2.size() * sizeof(int32_t));
        d.ts2.upload(ts2.data(), ts2.size() * sizeof(int32_t));
        d.tr4.upload(tr4.data(), tr4.size() * sizeof(int32_t));
        d.ts4.upload(ts4.data(), ts4.size() * sizeof(int32_t));
        d.base.n_tiles_r = (int64_t)tr.size() / 2;
        d.base.n_tiles_s = (int64_t)ts.size() / 2;
        d.base.n_tiles_r2 = (int64_t)tr2.size() / 2;
        d.base.n_tiles_s2 = (int64_t)ts2.size() / 2;
        d.base.n_tiles_r4 = (int64_t)tr4.size() / 2;
        d.base.n_tiles_s4 = (int64_t)ts4.size() / 2;
        d.desc.upload(desc.data(), desc.size() * sizeof(int64_t));
        d.idx.upload(idx.data(), idx.size() * sizeof(int32_t));
        upload_complex(d.m64, d.m128, mat);
        upload_complex(d.h64, d.h128, matH);
    }
    p->s0 = (int)h.hif.root_idx.size();
    p->root_idx.upload(h.hif.root_idx.data(), h.hif.root_idx.size() * sizeof(int32_t));
    p->A0inv.upload(h.hif.A0inv.a.data(), h.hif.A0inv.a.size() * sizeof(cd));
    p->perm.upload(h.perm.data(), h.perm.size() * sizeof(int32_t));
    const int32_t zero = 0;
    p->root_stage_idx.upload(&zero, sizeof(int32_t));
    count_bytes(p);
}

// Workspace for nrhs columns.  A graph captured from a call keeps the workspace's
// addresses, so once any call has run under stream capture the workspace never
// moves again: a later call that would need more fails instead.
void ensure_ws(fio_plan p, int nrhs, hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (st) HIPC(hipStreamIsCapturing(st, &cs));
    if (cs != hipStreamCaptureStatusNone) p->ws_captured = true;
    if (nrhs <= p->ws_nrhs) return;
    if (p->ws_captured)
        fail(FIO_ERR_ARG, "nrhs = " + std::to_string(nrhs) + " needs a larger workspace than the " +
                              std::to_string(p->ws_nrhs) + " columns a captured graph of this plan uses; "
                              "make the widest call before capturing");
    const size_t coef = (size_t)p->max_coef * nrhs * 16;
    const size_t vec = (size_t)p->host.N * nrhs * 16;
    p->P.alloc(coef); p->Q.alloc(coef);
    p->V1.alloc(vec); p->V2.alloc(vec); p->V3.alloc(vec); p->W.alloc(vec);
    p->U.alloc(vec); p->X.alloc(vec); p->R.alloc(vec); p->Z.alloc(vec); p->Pv.alloc(vec);
    p->red.alloc((size_t)reduce_partial_cap(p->host.N, nrhs) * sizeof(double));
    p->scal.alloc((size_t)nrhs * 8 * sizeof(double));
    p->HT.alloc(vec);
    p->RI.alloc((size_t)std::max(1, p->s0) * nrhs * 16);
    p->RO.alloc((size_t)std::max(1, p->s0) * nrhs * 16);
    p->ws_nrhs = nrhs;
}

// Launch schedule of a chain: (first stage, number of stages, variant) per launch.
// Tuned choices when the plan has them for (dtype, nrhs); otherwise consecutive
// fusable stages run in pairs for batches of 16 or more columns.
struct Launch {
    int first, count, variant;
};

std::vector<Launch> chain_schedule(fio_plan p, bool fwd, bool dbl, int nrhs) {
    const auto &ds = fwd ? p->dfwd : p->dadj;
    const auto &pr = fwd ? p->pfwd : p->padj;
    const auto *t = p->tuned(dbl, nrhs);
    const std::vector<int> *var = t ? (fwd ? &t->fwd : &t->adj) : nullptr;
    const std::vector<int> *pv = t ? (fwd ? &t->fwd_pair : &t->adj_pair) : nullptr;
    const std::vector<int> *tv = t ? (fwd ? &t->fwd_triple : &t->adj_triple) : nullptr;
    std::vector<Launch> out;
    const int S = (int)ds.size();
    for (int s = 0; s < S;) {
        if (tv && (size_t)s < tv->size() && (*tv)[s] > 0 && s + 2 < S && pr[s].n_wg3 > 0) {
            out.push_back({s, 3, (*tv)[s]});
            s += 3;
            continue;
        }
        int fuse = 0;
        if (s + 1 < S && pr[s].ok) {
            if (pv && (size_t)s < pv->size()) fuse = (*pv)[s];
            else if (!pv && nrhs >= 16) fuse = 2;
        }
        if (fuse > 0) {
            out.push_back({s, 2, fuse});
            s += 2;
        } else {
            out.push_back({s, 1, (var && (size_t)s < var->size()) ? (*var)[s] : -1});
            s += 1;
        }
    }
    return out;
}

StagePairDev pair_view(fio_plan p, bool fwd, bool dbl, int s) {
    const auto &hs = fwd ? p->host.fwd : p->adj;
    const auto &ds = fwd ? p->dfwd : p->dadj;
    const auto &pr = fwd ? p->pfwd : p->padj;
    StagePairDev v;
    v.a = ds[s].view(dbl, hs[s]);
    v.b = ds[s + 1].view(dbl, hs[s + 1]);
    v.tab = (const int32_t *)pr[s].tab.p;
    v.n_wg = pr[s].n_wg;
    v.tab_s = (const int32_t *)pr[s].tab_s.p;
    v.n_wg_s = pr[s].n_wg_s;
    return v;
}

StageTripleDev triple_view(fio_plan p, bool fwd, bool dbl, int s) {
    const auto &hs = fwd ? p->host.fwd : p->adj;
    const auto &ds = fwd ? p->dfwd : p->dadj;
    const auto &pr = fwd ? p->pfwd : p->padj;
    StageTripleDev v;
    v.a = ds[s].view(dbl, hs[s]);
    v.b = ds[s + 1].view(dbl, hs[s + 1]);
    v.c = ds[s + 2].view(dbl, hs[s + 2]);
    v.tab = (const int32_t *)pr[s].tab3.p;
    v.n_wg = pr[s].n_wg3;
    return v;
}

// Device temporaries of the chain and Gd drivers: the stage ping-pong buffers P, Q
// (max_coef x nrhs), the GEMM path's temporary HT (N x nrhs) and the FP64 root's
// gathered rows RI, RO (s0 x nrhs).  The plan's own workspace by default; the
// no-allocation entry point passes parts of its static scratch array instead.
struct Ws {
    void *P, *Q, *HT, *RI, *RO;
};
Ws plan_ws(fio_plan p) { return Ws{p->P.p, p->Q.p, p->HT.p, p->RI.p, p->RO.p}; }
void run_chain(fio_plan p, bool fwd, bool dbl, const void *in, void *out, int nrhs, hipStream_t st, const Ws &ws);

// Run a stage chain: in (first stage's input) -> out (last stage's output).
void run_chain(fio_plan p, bool fwd, bool dbl, const void *in, void *out, int nrhs, hipStream_t st) {
    run_chain(p, fwd, dbl, in, out, nrhs, st, plan_ws(p));
}
void run_chain(fio_plan p, bool fwd, bool dbl, const void *in, void *out, int nrhs, hipStream_t st, const Ws &ws) {
    TraceRange tr("fio %s chain %s B=%d", fwd ? "Kd" : "Kd*", dbl ? "c128" : "c64", nrhs);
    const auto &hs = fwd ? p->host.fwd : p->adj;
    const auto &ds = fwd ? p->dfwd : p->dadj;
    const std::vector<Launch> sched = chain_schedule(p, fwd, dbl, nrhs);
    const void *cur = in;
    for (size_t j = 0; j < sched.size(); ++j) {
        void *dst = (j + 1 == sched.size()) ? out : ((j % 2 == 0) ? ws.P : ws.Q);
        const Launch &l = sched[j];
        if (l.count == 3) {
            launch_stage_triple(triple_view(p, fwd, dbl, l.first), dbl, cur, dst, nrhs, st);
        } else if (l.count == 2) {
            launch_stage_pair(pair_view(p, fwd, dbl, l.first), dbl, l.variant, cur, dst, nrhs, st);
        } else {
            StageDev v = ds[l.first].view(dbl, hs[l.first]);
            v.variant = l.variant;
            launch_stage(v, dbl, cur, dst, nrhs, st);
        }
        cur = dst;
    }
}

// One skeletonization step: LDS-staged kernel for small nodes (choice 0), gathered
// GEMMs on matrix cores when a node's blocks exceed LDS (large 2D cells and edges),
// in tiles of 16 rows by 64, 32 or 16 right-hand sides (choices 1, 2, 3) or of 32
// rows by 32 (6) and 64 rows by 16 or 32 (7, 8), or the fused per-node matrix-core
// kernel for nodes of at most 64 redundant and 64 skeleton DOFs, 64 or 32
// right-hand sides per workgroup (choices 4, 5), or gathered matrix-vector products
// for small batches (choice 12).  `force` overrides the tuned choice where it applies.
constexpr int HIF_CHOICES = 13;
constexpr int HIF_GEMV = 12;
// Tiling of a gathered-GEMM choice: rows per wave in 16-row tiles, columns per wave,
// and whether a complex k-step takes three real products instead of four (9-11).
bool hif_gemm_tiling(int choice, int &mt, int &cols, bool &m3) {
    m3 = choice >= 9;
    switch (choice) {
        case 1: mt = 1; cols = 64; return true;
        case 2: mt = 1; cols = 32; return true;
        case 3: mt = 1; cols = 16; return true;
        case 6: mt = 2; cols = 32; return true;
        case 7: mt = 4; cols = 16; return true;
        case 8: mt = 4; cols = 32; return true;
        case 9: mt = 1; cols = 64; return true;
        case 10: mt = 1; cols = 32; return true;
        case 11: mt = 2; cols = 32; return true;
        default: return false;
    }
}
void hif_step(fio_plan p, size_t k, bool dbl, bool up, void *x, int nrhs, hipStream_t st, const Ws &ws,
              int force = -1) {
    const HifStepDev h = p->dhif[k].view(dbl);
    if (h.max_nr == 0) return;  // no redundant DOFs in any node: the step is the identity
    int choice = force;
    if ((choice == 4 || choice == 5) && !hif_fused_fits(h)) choice = -1;
    if (choice < 0) {
        const auto *t = p->tuned(dbl, nrhs);
        if (t && k < t->hif.size()) choice = t->hif[k];
    }
    if (choice < 0) {
        if (nrhs >= 16 && hif_fused_fits(h)) choice = 5;
        else if (hif_step_fits_lds(h, dbl)) choice = 0;
        else if (nrhs < 16) choice = HIF_GEMV;  // large nodes, small batches: matrix-vector products
        else choice = nrhs >= 64 ? 1 : 3;  // large nodes: gathered GEMMs over all nodes' row tiles
    }
    int mt = 1, cols = 16;
    bool m3 = false;
    if (choice == 4 || choice == 5) launch_hif_fused_step(h, dbl, up, x, nrhs, st, choice == 4 ? 64 : 32);
    else if (choice == HIF_GEMV)  // partial sums in the chain buffer P (idle during Gd)
        launch_hif_gemv_step(h, dbl, up, x, ws.HT, nrhs, ws.P, (size_t)p->max_coef * nrhs * (dbl ? 16 : 8), st);
    else if (hif_gemm_tiling(choice, mt, cols, m3)) launch_hif_gemm_step(h, dbl, up, x, ws.HT, nrhs, cols, st, mt, m3);
    else launch_hif_step(h, dbl, up, x, nrhs, st);
}

// A_0^{-1} on the remaining DOFs, always in FP64: a block of 64 or more DOFs as a
// one-block FP64 stage (matrix cores for batches, the small-batch kernel for fewer
// than 16 columns), a smaller one with the direct kernel.
void root_apply(fio_plan p, bool dbl, void *x, int nrhs, hipStream_t st, const Ws &ws) {
    if (p->s0 == 0) return;
    if (p->s0 < 64) {
        launch_root((const int32_t *)p->root_idx.p, p->A0inv.p, p->s0, dbl, x, nrhs, st);
        return;
    }
    launch_rows_gather(x, dbl, (const int32_t *)p->root_idx.p, p->s0, nrhs, ws.RI, true, st);
    StageDev s;
    s.n_out = 1; s.n_in = 1; s.r_out = p->s0; s.r_in = p->s0; s.fan = 1;
    s.idx = (const int32_t *)p->root_stage_idx.p;
    s.A = p->A0inv.p;
    const auto *t = p->tuned(dbl, nrhs);
    if (t) s.variant = t->root;
    if (nrhs < 16 && (s.variant < 0 || s.variant == STAGE_SMALL_BATCH)) {
        // one block of s0/64 row chunks leaves most of the device idle: split its k range
        // too (at least 64 columns per wave), partial sums in the GEMM temporary
        // (N x nrhs of the working precision), added by the scatter
        const int64_t rch = (p->s0 + 63) / 64, cch = (nrhs + 7) / 8;
        const int64_t cap = p->host.N * (dbl ? 16 : 8) / (16 * (int64_t)p->s0);
        const int ks = (int)std::min<int64_t>({16, std::max<int64_t>(1, 1024 / (rch * cch)), p->s0 / 256, cap});
        if (ks >= 2) {
            launch_stage_nb_split(s, true, ws.RI, ws.HT, nrhs, ks, st);
            launch_rows_scatter_sum(ws.HT, ks, (const int32_t *)p->root_idx.p, p->s0, nrhs, x, dbl, st);
            return;
        }
    }
    launch_stage(s, true, ws.RI, ws.RO, nrhs, st);
    launch_rows_scatter(ws.RO, true, (const int32_t *)p->root_idx.p, p->s0, nrhs, x, dbl, st);
}

void gd_inplace(fio_plan p, bool dbl, void *x, int nrhs, hipStream_t st, const Ws &ws, int force = -1) {
    TraceRange tr("fio Gd %s B=%d", dbl ? "c128" : "c64", nrhs);
    for (size_t k = 0; k < p->dhif.size(); ++k) {
        TraceRange ts("fio Gd step %zu up", k);
        hif_step(p, k, dbl, true, x, nrhs, st, ws, force);
    }
    {
        TraceRange tr0("fio Gd root");
        root_apply(p, dbl, x, nrhs, st, ws);
    }
    for (size_t k = p->dhif.size(); k-- > 0;) {
        TraceRange ts("fio Gd step %zu down", k);
        hif_step(p, k, dbl, false, x, nrhs, st, ws, force);
    }
}
void gd_inplace(fio_plan p, bool dbl, void *x, int nrhs, hipStream_t st, int force = -1) {
    gd_inplace(p, dbl, x, nrhs, st, plan_ws(p), force);
}

// worst = max(worst, v), where a NaN v (a non-finite column) wins, so that the
// convergence tests below fail for it instead of skipping it.
inline void worse(double &worst, double v) {
    if (!(v <= worst)) worst = v;
}

// Error estimates of a device plan (section 6's e_a and e_s, and cond(Kd)), in FP64
// on EA_VECS columns in the library's internal layout:
//   e_a   relative error of Kd v against K v on the probe rows the build summed;
//   e_s   spectral radius of E = I - Gd Kd^* Kd by power iteration (E is similar
//         to the Hermitian I - Sd^{1/2} Gd Sd^{1/2}, so the iteration converges to it);
//   cond  sqrt(lambda_max(Sd) lambda_max(Gd)), with Gd ~ Sd^{-1}.
// Skipped where the plan already carries them (a loaded plan file).
void estimate_errors(fio_plan p) {
    HostFactors &h = p->host;
    if (h.e_s_est > 0 || h.cond_est > 0) return;
    const int nr = EA_VECS;
    const int64_t N = h.N, cnt = N * nr;
    hipStream_t st = 0;
    ensure_ws(p, nr, st);
    double *scal = (double *)p->scal.p, *red = (double *)p->red.p;
    const int64_t cap = reduce_partial_cap(N, nr);
    std::vector<cd> pm((size_t)cnt);
    std::vector<double> nrm(nr);
    auto norms = [&](const void *v) {  // squared column norms to the host
        launch_colnorm2(v, N, nr, red, cap, scal, st);
        HIPC(hipMemcpyAsync(nrm.data(), scal, nr * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
    };
    auto start = [&](uint64_t salt) {  // Gaussian unit columns in X
        for (int64_t i = 0; i < cnt; ++i)
            pm[i] = cd(gauss(0xE57ULL ^ salt, 2 * (uint64_t)i), gauss(0xE57ULL ^ salt, 2 * (uint64_t)i + 1));
        HIPC(hipMemcpy(p->X.p, pm.data(), (size_t)cnt * 16, hipMemcpyHostToDevice));
        launch_colnorm2(p->X.p, N, nr, red, cap, scal, st);
        launch_col_unit(p->X.p, p->X.p, scal, N, nr, st);
    };
    auto sd = [&](const void *in, void *out) {  // out = Kd^* Kd in
        run_chain(p, true, true, in, p->V1.p, nr, st);
        run_chain(p, false, true, p->V1.p, out, nr, st);
    };
    auto gd = [&](const void *in, void *out) {  // out = Gd in
        HIPC(hipMemcpyAsync(out, in, (size_t)cnt * 16, hipMemcpyDeviceToDevice, st));
        gd_inplace(p, true, out, nr, st);
    };
    constexpr int ITS = 12;
    // e_a on the probe rows
    if (!h.ea_rows.empty() && h.e_a_est == 0) {
        const int rows = (int)h.ea_rows.size();
        for (int64_t q = 0; q < N; ++q)
            for (int v = 0; v < nr; ++v) pm[q * nr + v] = h.ea_vecs[(size_t)v * N + q];
        HIPC(hipMemcpy(p->X.p, pm.data(), (size_t)cnt * 16, hipMemcpyHostToDevice));
        run_chain(p, true, true, p->X.p, p->V2.p, nr, st);
        HIPC(hipMemcpy(pm.data(), p->V2.p, (size_t)cnt * 16, hipMemcpyDeviceToHost));
        double worst = 0;
        for (int v = 0; v < nr; ++v) {
            double num = 0, den = 0;
            for (int i = 0; i < rows; ++i) {
                const cd ref = h.ea_ref[(size_t)v * rows + i];
                num += std::norm(pm[(size_t)h.ea_rows[i] * nr + v] - ref);
                den += std::norm(ref);
            }
            worse(worst, std::sqrt(num / std::max(den, 1e-300)));
        }
        h.e_a_est = worst;
    }
    // e_s: power iteration on I - Gd Sd
    start(1);
    double es = 0;
    for (int it = 0; it < ITS; ++it) {
        sd(p->X.p, p->V2.p);
        gd(p->V2.p, p->V3.p);
        launch_residual(p->X.p, p->V3.p, p->R.p, true, cnt, st);  // R = (I - Gd Sd) x, ||x|| = 1
        norms(p->R.p);
        es = 0;
        for (int b = 0; b < nr; ++b) worse(es, std::sqrt(nrm[b]));
        launch_col_unit(p->X.p, p->R.p, scal, N, nr, st);
    }
    // lambda_max of Sd and of Gd
    auto lmax = [&](bool of_sd, uint64_t salt) {
        start(salt);
        double l = 0;
        for (int it = 0; it < ITS; ++it) {
            if (of_sd) sd(p->X.p, p->V2.p);
            else gd(p->X.p, p->V2.p);
            norms(p->V2.p);
            l = 0;
            for (int b = 0; b < nr; ++b) worse(l, std::sqrt(nrm[b]));
            launch_col_unit(p->X.p, p->V2.p, scal, N, nr, st);
        }
        return l;
    };
    const double ls = lmax(true, 2), lg = lmax(false, 3);
    HIPC(hipStreamSynchronize(st));
    h.e_s_est = es;
    h.cond_est = std::sqrt(std::max(ls * lg, 1.0));
}

void check_apply_args(fio_plan p, int64_t nrhs, int64_t ld, const void *a, const void *b) {
    if (!p) fail(FIO_ERR_ARG, "null plan");
    if (p->device < 0) fail(FIO_ERR_UNSUPPORTED, "plan is host-only (built or loaded with device = -1)");
    if (nrhs < 0 || nrhs > (1 << 20)) fail(FIO_ERR_ARG, "nrhs out of range");
    if (nrhs > 0 && ld < p->host.N) fail(FIO_ERR_ARG, "ld must be >= N");
    if (nrhs > 0 && (!a || !b)) fail(FIO_ERR_ARG, "null vector buffer");
}

template <class F> fio_status guard(F &&f) {
    try {
        f();
        return FIO_OK;
    } catch (const Error &e) {
        g_err = e.what();
        return e.status;
    } catch (const std::bad_alloc &) {
        g_err = "host allocation failed";
        return FIO_ERR_NOMEM;
    } catch (const std::exception &e) {
        g_err = e.what();
        return FIO_ERR_DEVICE;
    }
}

// Builder hook: products with Kd^* Kd for the peeling step on the plan's GPU (FP64).
// The device chains it forms are kept in `c` for the plan.
PeelApplyFactory gpu_peel_factory(int device, std::shared_ptr<DeviceChains> c) {
    return [device, c](const std::vector<Stage> &fwd) -> BlockApply {
        HIPC(hipSetDevice(device));
        if (c->dfwd.empty()) upload_chains(fwd, *c);
        int64_t maxc = 0;
        for (auto &s : fwd) maxc = std::max<int64_t>(maxc, std::max(s.n_out * s.r_out, s.n_in * s.r_in));
        const int64_t N = fwd.front().n_in * fwd.front().r_in;
        return [c, maxc, N, device, &fwd](const cd *x, cd *y, int nr) {
            HIPC(hipSetDevice(device));
            DBuf in, out, P, Q;
            in.alloc((size_t)N * nr * 16);
            out.alloc((size_t)N * nr * 16);
            P.alloc((size_t)maxc * nr * 16);
            Q.alloc((size_t)maxc * nr * 16);
            HIPC(hipMemcpy(in.p, x, (size_t)N * nr * 16, hipMemcpyHostToDevice));
            auto chain = [&](const std::vector<Stage> &h, const std::vector<DStageStore<int>> &d,
                             const void *src, void *dst) {
                const void *cur = src;
                for (size_t s = 0; s < d.size(); ++s) {
                    void *t = (s + 1 == d.size()) ? dst : ((s % 2 == 0) ? P.p : Q.p);
                    launch_stage(d[s].view(true, h[s]), true, cur, t, nr, 0);
                    cur = t;
                }
            };
            chain(fwd, c->dfwd, in.p, out.p);
            chain(c->adj, c->dadj, out.p, in.p);
            HIPC(hipMemcpy(y, in.p, (size_t)N * nr * 16, hipMemcpyDeviceToHost));
        };
    };
}

}  // namespace

// ------------------------------------------------- static scratch (no-allocation path)
// Device memory of fio_inverse_apply_noalloc: one file-scope array per device (every
// device that loads this code object holds its own copy until the process ends).
// In host code `scratch` names a host-side stand-in, not device memory: its device
// address comes from hipGetSymbolAddress, once per device, and only that address is
// ever handed to kernels or copies.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;  // device ordinal -> address of that device's scratch

// Address of the current device's scratch array (dev must be current).
void *scratch_on(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIPC(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) fail(FIO_ERR_DEVICE, "no device address for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

// Bytes of scratch an inverse apply of nrhs columns needs: the gathered input and
// the chain output (N x nrhs), the stage ping-pong buffers (max_coef x nrhs) and the
// GEMM path's temporary (N x nrhs), all of the working precision, and the FP64 root
// rows (s0 x nrhs, twice); each part starts on a 256-byte boundary.
struct ScratchLayout {
    size_t v1, v2, p, q, ht, ri, ro, total;
};
ScratchLayout scratch_layout(fio_plan p, bool dbl, int64_t nrhs) {
    const size_t elt = dbl ? 16 : 8;
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t vec = up((size_t)p->host.N * nrhs * elt), coef = up((size_t)p->max_coef * nrhs * elt);
    const size_t root = up((size_t)std::max(1, p->s0) * nrhs * 16);
    ScratchLayout L;
    L.v1 = 0;
    L.v2 = L.v1 + vec;
    L.p = L.v2 + vec;
    L.q = L.p + coef;
    L.ht = L.q + coef;
    L.ri = L.ht + vec;
    L.ro = L.ri + root;
    L.total = L.ro + root;
    return L;
}

}  // namespace

// ============================================================================ C ABI
extern "C" {

const char *fio_last_error(void) { return g_err.c_str(); }

void fio_set_trace(int on) { g_trace.store(on ? 1 : 0); }

fio_status fio_build(const fio_problem *prob, fio_plan *out) {
    return guard([&] {
        if (!prob || !out) fail(FIO_ERR_ARG, "null argument");
        *out = nullptr;
        std::unique_ptr<fio_plan_s> p(new fio_plan_s());
        p->device = prob->device;
        if (p->device >= 0) {
            int cnt = 0;
            HIPC(hipGetDeviceCount(&cnt));
            if (p->device >= cnt) fail(FIO_ERR_ARG, "device ordinal out of range");
            HIPC(hipSetDevice(p->device));
        }
        // Peeling products on the GPU when the plan has one (host otherwise).
        PeelApplyFactory f;
        BatchedIdFactory ids;
        auto chains = std::make_shared<DeviceChains>();
        if (p->device >= 0) f = gpu_peel_factory(p->device, chains);
        SkelHooks skel;
        if (p->device >= 0 && !prob->host_construction) {
            ids = device_id_factory(p->device);
            skel = device_skel_hooks(p->device);
        }
        build_host_factors(*prob, p->host, f, ids, skel);
        skel = SkelHooks();
        f = nullptr;
        if (!chains->dfwd.empty()) {  // the chains the peeling products used
            p->adj.swap(chains->adj);
            p->dfwd.swap(chains->dfwd);
            p->dadj.swap(chains->dadj);
        } else if (p->device < 0) {
            p->adj = adjoint_indexes(p->host.fwd);
        }
        if (p->device >= 0) {
            upload_plan(p.get());
            estimate_errors(p.get());
        }
        *out = p.release();
    });
}

fio_status fio_load(const char *path, int device, fio_plan *out) {
    return guard([&] {
        if (!path || !out) fail(FIO_ERR_ARG, "null argument");
        *out = nullptr;
        std::unique_ptr<fio_plan_s> p(new fio_plan_s());
        load_factors(path, p->host);
        p->host.prob.device = device;
        p->device = device;
        if (device >= 0) {
            upload_plan(p.get());
            estimate_errors(p.get());
        } else {
            p->adj = adjoint_indexes(p->host.fwd);
        }
        *out = p.release();
    });
}

fio_status fio_plan_trim(fio_plan p, int keep) {
    return guard([&] {
        if (!p) fail(FIO_ERR_ARG, "null plan");
        if (keep != FIO_KEEP_ALL && keep != FIO_KEEP_REFINE_C64) fail(FIO_ERR_ARG, "bad keep");
        if (p->device < 0) fail(FIO_ERR_UNSUPPORTED, "plan is host-only");
        if (keep == FIO_KEEP_ALL) return;
        std::lock_guard<std::mutex> lk(p->mu);
        HIPC(hipSetDevice(p->device));
        HIPC(hipDeviceSynchronize());  // no launch in flight may still read what goes
        for (auto &d : p->dfwd) {
            d.A64.alloc(0);
            d.gone64 = true;
        }
        for (auto &d : p->dadj) {
            d.A128.alloc(0);
            d.gone128 = true;
        }
        for (auto &h : p->dhif) {
            h.m128.alloc(0);
            h.h128.alloc(0);
            h.gone128 = true;
        }
        count_bytes(p);
    });
}

fio_status fio_save(fio_plan p, const char *path) {
    return guard([&] {
        if (!p || !path) fail(FIO_ERR_ARG, "null argument");
        save_factors(p->host, path);
    });
}

void fio_destroy(fio_plan p) {
    if (!p) return;
    forget_multi_tunes(p);
    delete p;
}

fio_status fio_plan_stats(fio_plan p, fio_plan_stats_t *o) {
    return guard([&] {
        if (!p || !o) fail(FIO_ERR_ARG, "null argument");
        std::memset(o, 0, sizeof(*o));
        const HostFactors &h = p->host;
        o->d = h.d; o->n = h.n; o->L = h.L; o->L_mid = h.Lm;
        o->n_stages = (int)h.fwd.size();
        for (auto &s : h.fwd) {
            o->bf_nnz += s.nnz();
            o->max_rank_bf = std::max({o->max_rank_bf, s.fan > 1 ? s.r_out : 0, s.fan > 1 ? s.r_in : 0});
        }
        o->hif_levels = (int)h.hif.steps.size();
        for (auto &st : h.hif.steps)
            for (auto &nd : st.nodes) {
                const int64_t r = (int64_t)nd.idx_r.size();
                o->hif_nnz += (int64_t)nd.T.a.size() + nd.Linv.a.size() + nd.M.a.size();
                o->hif_sweep_nnz += (int64_t)nd.T.a.size() + nd.M.a.size() + r * (r + 1) / 2;
            }
        o->root_size = (int)h.hif.root_idx.size();
        o->max_rank_h = h.hif.max_rank_h;
        o->hif_shifted = h.hif.shifted;
        o->device_bytes = p->device_bytes;
        o->workspace_bytes = (int64_t)(2 * p->max_coef + 12 * h.N + 2 * (int64_t)h.hif.root_idx.size()) * 16;
        o->build_seconds = h.build_seconds;
        o->bf_seconds = h.bf_seconds;
        o->bf_device_levels = h.bf_device_levels;
        o->hif_device_ids = h.hif.device_ids;
        o->hif_device_nodes = h.hif.device_nodes;
        o->e_a_est = h.e_a_est;
        o->e_s_est = h.e_s_est;
        o->cond_est = h.cond_est;
    });
}

fio_status fio_stage_info(fio_plan p, int stage, int64_t *nnz, int64_t *nob, int *r_out, int *r_in, int *fan) {
    return guard([&] {
        if (!p) fail(FIO_ERR_ARG, "null plan");
        if (stage < 0 || stage >= (int)p->host.fwd.size()) fail(FIO_ERR_ARG, "stage out of range");
        const Stage &s = p->host.fwd[stage];
        if (nnz) *nnz = s.nnz();
        if (nob) *nob = s.n_out;
        if (r_out) *r_out = s.r_out;
        if (r_in) *r_in = s.r_in;
        if (fan) *fan = s.fan;
    });
}

fio_status fio_apply(fio_plan p, fio_op op, fio_dtype dt, const void *x, void *y, int64_t nrhs, int64_t ld,
                     void *stream) {
    return guard([&] {
        check_apply_args(p, nrhs, ld, x, y);
        if (op != FIO_OP_K && op != FIO_OP_KH) fail(FIO_ERR_ARG, "bad op");
        if (dt != FIO_C64 && dt != FIO_C128) fail(FIO_ERR_ARG, "bad dtype");
        if (nrhs == 0) return;
        std::lock_guard<std::mutex> lk(p->mu);
        HIPC(hipSetDevice(p->device));
        hipStream_t st = (hipStream_t)stream;
        const bool dbl = dt == FIO_C128;
        const int nr = (int)nrhs;
        ensure_ws(p, nr, st);
        const int32_t *perm = (const int32_t *)p->perm.p;
        const int64_t N = p->host.N;
        launch_gather(x, dbl, ld, perm, p->V1.p, dbl, N, nr, st);
        if (op == FIO_OP_K) run_chain(p, true, dbl, p->V1.p, p->V2.p, nr, st);
        else run_chain(p, false, dbl, p->V1.p, p->V2.p, nr, st);
        launch_scatter(p->V2.p, dbl, perm, y, dbl, ld, N, nr, st);
    });
}

fio_status fio_stage_apply_variant(fio_plan p, fio_op op, int stage, fio_dtype dt, int variant, const void *x,
                                   void *y, int64_t nrhs, void *stream) {
    return guard([&] {
        check_apply_args(p, nrhs, p ? p->host.N : 0, x, y);
        if (op != FIO_OP_K && op != FIO_OP_KH) fail(FIO_ERR_ARG, "bad op");
        if (dt != FIO_C64 && dt != FIO_C128) fail(FIO_ERR_ARG, "bad dtype");
        if (variant < -1 || variant >= STAGE_VARIANTS) fail(FIO_ERR_ARG, "stage kernel variant out of range");
        const auto &hs = (op == FIO_OP_K) ? p->host.fwd : p->adj;
        const auto &ds = (op == FIO_OP_K) ? p->dfwd : p->dadj;
        if (stage < 0 || stage >= (int)hs.size()) fail(FIO_ERR_ARG, "stage out of range");
        if (nrhs == 0) return;
        HIPC(hipSetDevice(p->device));
        const bool dbl = dt == FIO_C128;
        StageDev v = ds[stage].view(dbl, hs[stage]);
        if (variant >= 0) {
            v.variant = variant;
        } else {
            const auto *t = p->tuned(dbl, (int)nrhs);
            if (t) v.variant = (op == FIO_OP_K) ? t->fwd[stage] : t->adj[stage];
        }
        launch_stage(v, dbl, x, y, (int)nrhs, (hipStream_t)stream);
    });
}

fio_status fio_stage_apply(fio_plan p, fio_op op, int stage, fio_dtype dt, const void *x, void *y,
                           int64_t nrhs, void *stream) {
    return fio_stage_apply_variant(p, op, stage, dt, -1, x, y, nrhs, stream);
}

fio_status fio_stage_pair_apply(fio_plan p, fio_op op, int stage, fio_dtype dt, const void *x, void *y,
                                int64_t nrhs, void *stream) {
    return guard([&] {
        check_apply_args(p, nrhs, p ? p->host.N : 0, x, y);
        if (op != FIO_OP_K && op != FIO_OP_KH) fail(FIO_ERR_ARG, "bad op");
        if (dt != FIO_C64 && dt != FIO_C128) fail(FIO_ERR_ARG, "bad dtype");
        const bool fwd = op == FIO_OP_K;
        const auto &pr = fwd ? p->pfwd : p->padj;
        if (stage < 0 || stage >= (int)pr.size()) fail(FIO_ERR_ARG, "stage out of range");
        if (!pr[stage].ok) fail(FIO_ERR_UNSUPPORTED, "these two stages cannot run fused");
        if (nrhs == 0) return;
        HIPC(hipSetDevice(p->device));
        const bool dbl = dt == FIO_C128;
        int v = 2;
        for (const Launch &l : chain_schedule(p, fwd, dbl, (int)nrhs))
            if (l.first == stage && l.count == 2) v = l.variant;
        launch_stage_pair(pair_view(p, fwd, dbl, stage), dbl, v, x, y, (int)nrhs, (hipStream_t)stream);
    });
}

fio_status fio_stage_pair_apply_variant(fio_plan p, fio_op op, int stage, fio_dtype dt, int variant, const void *x,
                                        void *y, int64_t nrhs, void *stream) {
    return guard([&] {
        check_apply_args(p, nrhs, p ? p->host.N : 0, x, y);
        if (op != FIO_OP_K && op != FIO_OP_KH) fail(FIO_ERR_ARG, "bad op");
        if (dt != FIO_C64 && dt != FIO_C128) fail(FIO_ERR_ARG, "bad dtype");
        const bool fwd = op == FIO_OP_K;
        const bool dbl = dt == FIO_C128;
        const auto &pr = fwd ? p->pfwd : p->padj;
        if (stage < 0 || stage >= (int)pr.size()) fail(FIO_ERR_ARG, "stage out of range");
        if (variant < 1 || (variant > stage_pair_variants(dbl) && variant != STAGE_PAIR_STACKED))
            fail(FIO_ERR_ARG, "fused pair variant out of range");
        if (!pr[stage].ok) fail(FIO_ERR_UNSUPPORTED, "these two stages cannot run fused");
        const StagePairDev pv = pair_view(p, fwd, dbl, stage);
        if (variant == STAGE_PAIR_STACKED && !(pv.tab_s && stage_pair_stackable(pv.a.r_out, pv.b.r_out)))
            fail(FIO_ERR_UNSUPPORTED, "these two stages cannot run stacked");
        if (nrhs == 0) return;
        HIPC(hipSetDevice(p->device));
        launch_stage_pair(pv, dbl, variant, x, y, (int)nrhs, (hipStream_t)stream);
    });
}

fio_status fio_stage_triple_apply(fio_plan p, fio_op op, int stage, fio_dtype dt, const void *x, void *y,
                                  int64_t nrhs, void *stream) {
    return guard([&] {
        check_apply_args(p, nrhs, p ? p->host.N : 0, x, y);
        if (op != FIO_OP_K && op != FIO_OP_KH) fail(FIO_ERR_ARG, "bad op");
        if (dt != FIO_C64 && dt != FIO_C128) fail(FIO_ERR_ARG, "bad dtype");
        const bool fwd = op == FIO_OP_K;
        const bool dbl = dt == FIO_C128;
        const auto &pr = fwd ? p->pfwd : p->padj;
        const int S = (int)(fwd ? p->dfwd : p->dadj).size();
        if (stage < 0 || stage + 2 >= S) fail(FIO_ERR_ARG, "stage out of range");
        if (pr[stage].n_wg3 <= 0) fail(FIO_ERR_UNSUPPORTED, "these three stages cannot run fused");
        if (!(fwd ? p->dfwd : p->dadj)[stage].has(dbl)) fail(FIO_ERR_UNSUPPORTED, "factor image released");
        if (nrhs == 0) return;
        HIPC(hipSetDevice(p->device));
        launch_stage_triple(triple_view(p, fwd, dbl, stage), dbl, x, y, (int)nrhs, (hipStream_t)stream);
    });
}

fio_status fio_column_id(int device, int64_t m, int64_t n, const void *A, int64_t lda, double tol_rel, int *rank,
                         int *perm, void *T, int64_t t_cap) {
    return guard([&] {
        if (!A || !rank || !perm || !T) fail(FIO_ERR_ARG, "null argument");
        if (m < 1 || n < 1 || n > INT32_MAX || lda < m) fail(FIO_ERR_ARG, "bad matrix shape");
        if (!(tol_rel >= 0)) fail(FIO_ERR_ARG, "tol_rel must be non-negative");
        int cnt = 0;
        HIPC(hipGetDeviceCount(&cnt));
        if (device < 0 || device >= cnt) fail(FIO_ERR_ARG, "device ordinal out of range");
        if (m > INT32_MAX) fail(FIO_ERR_UNSUPPORTED, "more than 2^31 - 1 rows");
        Mat Ah((int)m, (int)n);
        const cd *a = (const cd *)A;
        for (int64_t j = 0; j < n; ++j) std::copy(a + j * lda, a + j * lda + m, Ah.col((int)j));
        ColumnID id;
        if (!device_skel_hooks(device).big_id(Ah, tol_rel, id)) fail(FIO_ERR_UNSUPPORTED, "matrix declined (not enough device memory)");
        const int k = (int)id.skel.size();
        *rank = k;
        if ((int64_t)k * (n - k) > t_cap) fail(FIO_ERR_ARG, "T buffer too small for the rank");
        for (int q = 0; q < k; ++q) perm[q] = id.skel[q];
        for (int64_t q = k; q < n; ++q) perm[q] = id.redund[q - k];
        std::copy(id.T.a.begin(), id.T.a.end(), (cd *)T);
    });
}

fio_status fio_chain_schedule(fio_plan p, fio_op op, fio_dtype dt, int64_t nrhs, int cap, int *n_launch,
                              int *first_stage, int *n_stages, int *variant) {
    return guard([&] {
        if (!p || !n_launch) fail(FIO_ERR_ARG, "null argument");
        if (op != FIO_OP_K && op != FIO_OP_KH) fail(FIO_ERR_ARG, "bad op");
        if (dt != FIO_C64 && dt != FIO_C128) fail(FIO_ERR_ARG, "bad dtype");
        if (nrhs < 1) fail(FIO_ERR_ARG, "nrhs must be positive");
        const bool dbl = dt == FIO_C128;
        const std::vector<Launch> s = chain_schedule(p, op == FIO_OP_K, dbl, (int)nrhs);
        *n_launch = (int)s.size();
        if (cap < (int)s.size()) {
            if (cap > 0) fail(FIO_ERR_ARG, "cap smaller than the number of launches");
            return;
        }
        if (!first_stage || !n_stages || !variant) fail(FIO_ERR_ARG, "null output arrays");
        for (size_t j = 0; j < s.size(); ++j) {
            first_stage[j] = s[j].first;
            n_stages[j] = s[j].count;
            const int v = s[j].variant;
            variant[j] = (s[j].count == 1 && v < 0)
                             ? stage_default_variant((op == FIO_OP_K ? p->dfwd : p->dadj)[s[j].first].view(
                                                         dbl, (op == FIO_OP_K ? p->host.fwd : p->adj)[s[j].first]),
                                                     dbl, (int)nrhs)
                             : v;
        }
    });
}

fio_status fio_autotune(fio_plan p, fio_dtype dt, int64_t nrhs, int reps, void *stream) {
    return guard([&] {
        if (!p) fail(FIO_ERR_ARG, "null plan");
        if (p->device < 0) fail(FIO_ERR_UNSUPPORTED, "plan is host-only");
        if (dt != FIO_C64 && dt != FIO_C128) fail(FIO_ERR_ARG, "bad dtype");
        if (nrhs < 1 || nrhs > (1 << 16)) fail(FIO_ERR_ARG, "nrhs out of range");
        if (reps < 1) reps = 3;
        std::lock_guard<std::mutex> lk(p->mu);
        HIPC(hipSetDevice(p->device));
        hipStream_t st = (hipStream_t)stream;
        const bool dbl = dt == FIO_C128;
        const int nr = (int)nrhs;
        ensure_ws(p, nr, st);
        launch_scale_zero(p->P.p, p->max_coef * nr, st);
        launch_scale_zero(p->Q.p, p->max_coef * nr, st);
        launch_scale_zero(p->V2.p, p->host.N * nr, st);
        hipEvent_t e0, e1;
        HIPC(hipEventCreate(&e0));
        HIPC(hipEventCreate(&e1));
        auto timeit = [&](auto &&fn) {
            fn();  // warm-up (also sets kernel attributes outside the timed region)
            HIPC(hipEventRecord(e0, st));
            for (int r = 0; r < reps; ++r) fn();
            HIPC(hipEventRecord(e1, st));
            HIPC(hipEventSynchronize(e1));
            float ms = 0;
            HIPC(hipEventElapsedTime(&ms, e0, e1));
            return ms;
        };
        const bool vb = p->host.prob.verbose != 0;
        fio_plan_s::Tune t;
        for (int chain = 0; chain < 2; ++chain) {
            const bool fwd = chain == 0;
            const auto &hs = fwd ? p->host.fwd : p->adj;
            const auto &ds = fwd ? p->dfwd : p->dadj;
            const auto &pr = fwd ? p->pfwd : p->padj;
            std::vector<int> &out = fwd ? t.fwd : t.adj;
            std::vector<int> &pout = fwd ? t.fwd_pair : t.adj_pair;
            const int S = (int)ds.size();
            if (S > 0 && !ds[0].has(dbl)) {  // released by fio_plan_trim: nothing to tune
                out.assign(S, -1);
                pout.assign(S, 0);
                continue;
            }
            std::vector<float> one_ms(S, 0.f), two_ms(S, 1e30f), three_ms(S, 1e30f);
            std::vector<int> two_v(S, 0);
            std::vector<int> &tout = fwd ? t.fwd_triple : t.adj_triple;
            for (int s = 0; s < S; ++s) {
                int best = -1;
                float best_ms = 1e30f;
                for (int v = 0; v < STAGE_VARIANTS; ++v) {
                    if (v > 0 && v != STAGE_SMALL_BATCH && nr < 8) continue;  // matrix cores need a few columns
                    if (v == STAGE_SMALL_BATCH && nr >= 16) continue;         // for small batches only
                    StageDev sd = ds[s].view(dbl, hs[s]);
                    sd.variant = v;
                    const float ms = timeit([&] { launch_stage(sd, dbl, p->P.p, p->Q.p, nr, st); });
                    if (ms < best_ms) { best_ms = ms; best = v; }
                }
                out.push_back(best);
                one_ms[s] = best_ms;
                if (s + 1 < S && pr[s].ok && nr >= 8) {
                    const StagePairDev pv = pair_view(p, fwd, dbl, s);
                    std::vector<int> vs;
                    for (int v = 1; v <= stage_pair_variants(dbl); ++v) vs.push_back(v);
                    if (pv.tab_s && stage_pair_stackable(pv.a.r_out, pv.b.r_out)) vs.push_back(STAGE_PAIR_STACKED);
                    for (int v : vs) {
                        const float ms = timeit([&] { launch_stage_pair(pv, dbl, v, p->P.p, p->Q.p, nr, st); });
                        progress(vb, "tune %s %s pair (%d,%d) variant %d: %.4f ms", dbl ? "c128" : "c64",
                                 fwd ? "K" : "KH", s, s + 1, v, ms / reps);
                        if (ms < two_ms[s]) { two_ms[s] = ms; two_v[s] = v; }
                    }
                }
                progress(vb, "tune %s %s stage %d (r_out %d, r_in %d, fan %d): variant %d %.4f ms",
                         dbl ? "c128" : "c64", fwd ? "K" : "KH", s, hs[s].r_out, hs[s].r_in, hs[s].fan,
                         best, best_ms / reps);
            }
            // three consecutive stages in one launch, where they form stacked groups
            for (int s = 0; s + 2 < S && nr >= 8; ++s) {
                if (pr[s].n_wg3 <= 0) continue;
                const StageTripleDev tv = triple_view(p, fwd, dbl, s);
                three_ms[s] = timeit([&] { launch_stage_triple(tv, dbl, p->P.p, p->Q.p, nr, st); });
                progress(vb, "tune %s %s triple (%d,%d,%d): %.4f ms", dbl ? "c128" : "c64", fwd ? "K" : "KH", s,
                         s + 1, s + 2, three_ms[s] / reps);
            }
            // fastest split of the chain into single and fused launches
            std::vector<float> best(S + 1, 0.f);
            std::vector<int> take(S, 1);
            for (int s = S - 1; s >= 0; --s) {
                best[s] = one_ms[s] + best[s + 1];
                if (s + 1 < S && two_v[s] > 0 && two_ms[s] + best[s + 2] < best[s]) {
                    best[s] = two_ms[s] + best[s + 2];
                    take[s] = 2;
                }
                if (s + 2 < S && three_ms[s] < 1e29f && three_ms[s] + best[s + 3] < best[s]) {
                    best[s] = three_ms[s] + best[s + 3];
                    take[s] = 3;
                }
            }
            pout.assign(S, 0);
            tout.assign(S, 0);
            for (int s = 0; s < S;) {
                if (take[s] == 3) { tout[s] = 1; s += 3; }
                else if (take[s] == 2) { pout[s] = two_v[s]; s += 2; }
                else s += 1;
            }
        }
        for (size_t k = 0; k < p->dhif.size(); ++k) {
            if (!p->dhif[k].has(dbl)) {  // released by fio_plan_trim
                t.hif.push_back(-1);
                continue;
            }
            const HifStepDev h = p->dhif[k].view(dbl);
            int best = 0;
            {
                float best_ms = 1e30f;
                if (hif_step_fits_lds(h, dbl) || nr < 16) {
                    best_ms = timeit([&] {
                        launch_hif_step(h, dbl, true, p->V2.p, nr, st);
                        launch_hif_step(h, dbl, false, p->V2.p, nr, st);
                    });
                }
                for (int c : {1, 2, 3, 6, 7, 8, 9, 10, 11}) {
                    int mt = 1, cols = 16;
                    bool m3 = false;
                    hif_gemm_tiling(c, mt, cols, m3);
                    if (nr <= 16 && cols > 16) continue;  // one 16-column tile covers the batch
                    if (mt > 1 && std::max(h.max_nr, h.max_ns) < 16 * mt) continue;  // rows would be padding
                    const float ms = timeit([&] {
                        launch_hif_gemm_step(h, dbl, true, p->V2.p, p->HT.p, nr, cols, st, mt, m3);
                        launch_hif_gemm_step(h, dbl, false, p->V2.p, p->HT.p, nr, cols, st, mt, m3);
                    });
                    if (ms < best_ms) { best_ms = ms; best = c; }
                }
                if (nr < 16) {
                    const size_t pbytes = (size_t)p->max_coef * nr * (dbl ? 16 : 8);
                    const float ms = timeit([&] {
                        launch_hif_gemv_step(h, dbl, true, p->V2.p, p->HT.p, nr, p->P.p, pbytes, st);
                        launch_hif_gemv_step(h, dbl, false, p->V2.p, p->HT.p, nr, p->P.p, pbytes, st);
                    });
                    if (ms < best_ms) { best_ms = ms; best = HIF_GEMV; }
                }
                if (hif_fused_fits(h)) {
                    for (int c = 4; c <= 5; ++c) {
                        const int cw = c == 4 ? 64 : 32;
                        const float ms = timeit([&] {
                            launch_hif_fused_step(h, dbl, true, p->V2.p, nr, st, cw);
                            launch_hif_fused_step(h, dbl, false, p->V2.p, nr, st, cw);
                        });
                        if (ms < best_ms) { best_ms = ms; best = c; }
                    }
                }
                if (vb) {
                    // complex multiply-adds of the step's up and down sweeps per column:
                    // T and M products (ns nr each) and the triangular L^-1 (nr (nr+1)/2)
                    double macs = 0;
                    int mr = 0, ms = 0;
                    for (const HifNode &nd : p->host.hif.steps[k].nodes) {
                        const double r = (double)nd.idx_r.size(), q = (double)nd.idx_s.size();
                        macs += 2.0 * (2.0 * q * r + r * (r + 1) / 2);
                        mr = std::max(mr, (int)nd.idx_r.size());
                        ms = std::max(ms, (int)nd.idx_s.size());
                    }
                    const double sec = best_ms / reps * 1e-3;
                    progress(true,
                             "tune %s skeletonization step %zu (%lld nodes, largest nr %d ns %d): choice %d %.4f ms, "
                             "%.1f TFLOP/s",
                             dbl ? "c128" : "c64", k, (long long)h.n_nodes, mr, ms, best, best_ms / reps,
                             8.0 * macs * nr / sec / 1e12);
                }
            }
            t.hif.push_back(best);
        }
        if (p->s0 >= 64) {
            StageDev sr;
            sr.n_out = 1; sr.n_in = 1; sr.r_out = p->s0; sr.r_in = p->s0; sr.fan = 1;
            sr.idx = (const int32_t *)p->root_stage_idx.p;
            sr.A = p->A0inv.p;
            float best_ms = 1e30f;
            launch_scale_zero(p->RI.p, (int64_t)p->s0 * nr, st);
            for (int v = 1; v < STAGE_VARIANTS; ++v) {
                if ((v == STAGE_SMALL_BATCH) != (nr < 16)) continue;  // matrix cores from 16 columns
                if (v == STAGE_LDS4 || v == STAGE_LDS2) continue;      // blocks of up to 192 rows only
                if (v >= 12) continue;                                    // four-product tilings for FP64
                sr.variant = v;
                const float ms = timeit([&] { launch_stage(sr, true, p->RI.p, p->RO.p, nr, st); });
                if (ms < best_ms) { best_ms = ms; t.root = v; }
            }
            progress(vb, "tune top-level block (%d DOFs): variant %d %.4f ms", p->s0, t.root, best_ms / reps);
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        p->tune[{dbl ? 1 : 0, nr}] = std::move(t);
    });
}

fio_status fio_tune_query(fio_plan p, fio_op op, int stage, fio_dtype dt, int64_t nrhs, int *variant) {
    return guard([&] {
        if (!p || !variant) fail(FIO_ERR_ARG, "null argument");
        const bool dbl = dt == FIO_C128;
        const auto &hs = (op == FIO_OP_K) ? p->host.fwd : p->adj;
        if (stage < 0 || stage >= (int)hs.size()) fail(FIO_ERR_ARG, "stage out of range");
        const auto *t = p->tuned(dbl, (int)nrhs);
        if (t) {
            *variant = (op == FIO_OP_K) ? t->fwd[stage] : t->adj[stage];
        } else {
            StageDev sd;
            sd.r_out = hs[stage].r_out;
            *variant = stage_default_variant(sd, dbl, (int)nrhs);
        }
    });
}

fio_status fio_gd_apply(fio_plan p, fio_dtype dt, const void *x, void *y, int64_t nrhs, int64_t ld, void *stream) {
    return fio_gd_apply_variant(p, dt, -1, x, y, nrhs, ld, stream);
}

fio_status fio_gd_apply_variant(fio_plan p, fio_dtype dt, int variant, const void *x, void *y, int64_t nrhs,
                                int64_t ld, void *stream) {
    return guard([&] {
        check_apply_args(p, nrhs, ld, x, y);
        if (dt != FIO_C64 && dt != FIO_C128) fail(FIO_ERR_ARG, "bad dtype");
        if (variant < -1 || variant >= HIF_CHOICES) fail(FIO_ERR_ARG, "skeletonization kernel variant out of range");
        if (nrhs == 0) return;
        std::lock_guard<std::mutex> lk(p->mu);
        HIPC(hipSetDevice(p->device));
        hipStream_t st = (hipStream_t)stream;
        const bool dbl = dt == FIO_C128;
        const int nr = (int)nrhs;
        ensure_ws(p, nr, st);
        const int32_t *perm = (const int32_t *)p->perm.p;
        launch_gather(x, dbl, ld, perm, p->V2.p, dbl, p->host.N, nr, st);
        gd_inplace(p, dbl, p->V2.p, nr, st, variant);
        launch_scatter(p->V2.p, dbl, perm, y, dbl, ld, p->host.N, nr, st);
    });
}

fio_status fio_plan_fingerprints(fio_plan p, uint64_t *fp, int cap, int *count) {
    return guard([&] {
        if (!p || !count || (cap > 0 && !fp)) fail(FIO_ERR_ARG, "null argument");
        const std::vector<uint64_t> f = factor_fingerprints(p->host);
        for (int i = 0; i < cap && i < (int)f.size(); ++i) fp[i] = f[i];
        *count = (int)f.size();
    });
}

fio_status fio_inverse_apply_noalloc(fio_plan p, fio_dtype dt, const void *u, void *fh, int64_t nrhs,
                                     int64_t ld, void *stream) {
    return guard([&] {
        check_apply_args(p, nrhs, ld, u, fh);
        if (dt != FIO_C64 && dt != FIO_C128) fail(FIO_ERR_ARG, "bad dtype");
        if (nrhs == 0) return;
        const bool dbl = dt == FIO_C128;
        const ScratchLayout L = scratch_layout(p, dbl, nrhs);
        if (L.total > NOALLOC_SCRATCH_BYTES)
            fail(FIO_ERR_ARG, "nrhs = " + std::to_string(nrhs) + " needs " + std::to_string(L.total) +
                                  " bytes of scratch; the no-allocation path has " +
                                  std::to_string(NOALLOC_SCRATCH_BYTES));
        std::lock_guard<std::mutex> lk(p->mu);
        HIPC(hipSetDevice(p->device));
        char *base = (char *)scratch_on(p->device);
        hipStream_t st = (hipStream_t)stream;
        const int nr = (int)nrhs;
        const Ws ws{base + L.p, base + L.q, base + L.ht, base + L.ri, base + L.ro};
        void *v1 = base + L.v1, *v2 = base + L.v2;
        const int32_t *perm = (const int32_t *)p->perm.p;
        launch_gather(u, dbl, ld, perm, v1, dbl, p->host.N, nr, st);
        run_chain(p, false, dbl, v1, v2, nr, st, ws);
        gd_inplace(p, dbl, v2, nr, st, ws);
        launch_scatter(v2, dbl, perm, fh, dbl, ld, p->host.N, nr, st);
    });
}

fio_status fio_inverse_apply(fio_plan p, fio_dtype dt, const void *u, void *fh, int64_t nrhs, int64_t ld,
                             void *stream) {
    return guard([&] {
        check_apply_args(p, nrhs, ld, u, fh);
        if (dt != FIO_C64 && dt != FIO_C128) fail(FIO_ERR_ARG, "bad dtype");
        if (nrhs == 0) return;
        std::lock_guard<std::mutex> lk(p->mu);
        HIPC(hipSetDevice(p->device));
        hipStream_t st = (hipStream_t)stream;
        const bool dbl = dt == FIO_C128;
        const int nr = (int)nrhs;
        ensure_ws(p, nr, st);
        const int32_t *perm = (const int32_t *)p->perm.p;
        const int64_t N = p->host.N;
        launch_gather(u, dbl, ld, perm, p->V1.p, dbl, N, nr, st);
        run_chain(p, false, dbl, p->V1.p, p->V2.p, nr, st);
        gd_inplace(p, dbl, p->V2.p, nr, st);
        launch_scatter(p->V2.p, dbl, perm, fh, dbl, ld, N, nr, st);
    });
}

}  // extern "C"

namespace {

// Restarted GMRES on Kd x = u with the right preconditioner M = Gd Kd^* (or M = I),
// one Krylov space per column: x = M V y minimises ||u - Kd x|| over the space.
// Arnoldi with modified Gram-Schmidt runs on the device with per-column scalars;
// the Hessenberg columns come to the host after every step, where complex Givens
// rotations keep the least-squares residual |g_{j+1}| of every column.  At the end
// of a cycle y solves the triangular system, x += M (V y), and the next cycle
// starts from the true residual.  Expects p->U = u, leaves x in p->X (complex128).
template <class AC, class GD>
int gmres(fio_plan p, const fio_solve_opts *opts, int nr, AC &apply_chain, GD &gd128, hipStream_t st,
          double &worst, bool &converged) {
    using cdd = std::complex<double>;
    const int64_t N = p->host.N, cnt = N * nr;
    const int m = opts->restart > 0 ? std::min(opts->restart, 64) : 20;
    if (p->gv_vecs < m + 1 || p->gv_cnt < cnt) {
        p->GV.alloc((size_t)(m + 1) * cnt * 16);
        p->GH.alloc((size_t)(m + 1) * m * 2 * nr * sizeof(double) + (size_t)(m + 1) * 2 * nr * sizeof(double));
        p->gv_vecs = m + 1;
        p->gv_cnt = cnt;
    }
    auto V = [&](int j) { return (void *)((char *)p->GV.p + (size_t)j * cnt * 16); };
    double *H = (double *)p->GH.p;                        // column j of the Hessenberg: H + j*(m+1)*2*nr
    double *Yd = H + (size_t)(m + 1) * m * 2 * nr;       // y per column
    auto Hc = [&](int j, int i) { return H + ((size_t)j * (m + 1) + i) * 2 * nr; };
    double *scal = (double *)p->scal.p;
    double *nrm = scal + 6 * nr;
    double *red = (double *)p->red.p;
    const int64_t cap = reduce_partial_cap(N, nr);
    const bool pre = opts->precondition != 0;
    auto applyM = [&](const void *in128, void *out128) {  // out = Gd Kd^* in (complex128)
        apply_chain(false, in128, out128);
        gd128(out128, out128);
    };
    // unorm
    std::vector<double> hb(2 * (size_t)(m + 1) * nr), h2(nr), unorm(nr), beta(nr);
    launch_colnorm2(p->U.p, N, nr, red, cap, nrm, st);
    HIPC(hipMemcpyAsync(h2.data(), nrm, nr * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    for (int b = 0; b < nr; ++b) unorm[b] = std::max(std::sqrt(h2[b]), 1e-300);
    launch_scale_zero(p->X.p, cnt, st);
    std::vector<cdd> R((size_t)m * m * nr), g((size_t)(m + 1) * nr), cs((size_t)m * nr), sn((size_t)m * nr);
    std::vector<double> yh(2 * (size_t)m * nr);
    const int maxit = std::max(1, opts->maxit);
    int total = 0;
    converged = false;
    worst = 1.0;
    bool first = true;
    while (total < maxit) {
        // r = u - Kd x (x = 0 in the first cycle)
        if (first) {
            HIPC(hipMemcpyAsync(p->R.p, p->U.p, cnt * 16, hipMemcpyDeviceToDevice, st));
        } else {
            apply_chain(true, p->X.p, p->V1.p);
            launch_residual(p->U.p, p->V1.p, p->R.p, true, cnt, st);
        }
        first = false;
        launch_colnorm2(p->R.p, N, nr, red, cap, nrm, st);
        launch_col_unit(V(0), p->R.p, nrm, N, nr, st);
        HIPC(hipMemcpyAsync(h2.data(), nrm, nr * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
        worst = 0;
        for (int b = 0; b < nr; ++b) {
            beta[b] = std::sqrt(h2[b]);
            worse(worst, beta[b] / unorm[b]);
        }
        if (opts->tol > 0 && worst <= opts->tol) { converged = true; break; }
        std::fill(g.begin(), g.end(), cdd(0));
        for (int b = 0; b < nr; ++b) g[b] = beta[b];
        int j = 0;
        for (; j < m && total < maxit; ++j) {
            ++total;
            // w = Kd M v_j
            if (pre) {
                applyM(V(j), p->Z.p);
            } else {
                HIPC(hipMemcpyAsync(p->Z.p, V(j), cnt * 16, hipMemcpyDeviceToDevice, st));
            }
            apply_chain(true, p->Z.p, p->V1.p);
            for (int i = 0; i <= j; ++i) {
                launch_coldot(V(i), p->V1.p, N, nr, red, cap, Hc(j, i), st);
                launch_col_axpy(p->V1.p, V(i), Hc(j, i), -1.0, N, nr, st);
            }
            launch_colnorm2(p->V1.p, N, nr, red, cap, nrm, st);
            launch_col_unit(V(j + 1), p->V1.p, nrm, N, nr, st);
            HIPC(hipMemcpyAsync(hb.data(), Hc(j, 0), (size_t)(j + 1) * 2 * nr * sizeof(double),
                                hipMemcpyDeviceToHost, st));
            HIPC(hipMemcpyAsync(h2.data(), nrm, nr * sizeof(double), hipMemcpyDeviceToHost, st));
            HIPC(hipStreamSynchronize(st));
            worst = 0;
            for (int b = 0; b < nr; ++b) {
                std::vector<cdd> h(j + 2);
                for (int i = 0; i <= j; ++i) h[i] = cdd(hb[(size_t)i * 2 * nr + 2 * b], hb[(size_t)i * 2 * nr + 2 * b + 1]);
                h[j + 1] = std::sqrt(h2[b]);
                for (int i = 0; i < j; ++i) {  // earlier rotations
                    const cdd c = cs[(size_t)i * nr + b], s = sn[(size_t)i * nr + b];
                    const cdd a0 = h[i], a1 = h[i + 1];
                    h[i] = c * a0 + s * a1;
                    h[i + 1] = -std::conj(s) * a0 + c * a1;
                }
                const double aa = std::abs(h[j]), bb = std::abs(h[j + 1]);
                const double t = std::hypot(aa, bb);
                cdd c = 1.0, s = 0.0;
                if (t > 0) {
                    if (aa == 0) { c = 0.0; s = std::conj(h[j + 1]) / bb; }
                    else { c = aa / t; s = (h[j] / aa) * std::conj(h[j + 1]) / t; }
                }
                cs[(size_t)j * nr + b] = c;
                sn[(size_t)j * nr + b] = s;
                h[j] = c * h[j] + s * h[j + 1];
                for (int i = 0; i <= j; ++i) R[((size_t)j * m + i) * nr + b] = h[i];
                const cdd gj = g[(size_t)j * nr + b];
                g[(size_t)j * nr + b] = c * gj;
                g[(size_t)(j + 1) * nr + b] = -std::conj(s) * gj;
                worse(worst, std::abs(g[(size_t)(j + 1) * nr + b]) / unorm[b]);
            }
            if (opts->tol > 0 && worst <= opts->tol) { ++j; break; }
        }
        // y = R^{-1} g (upper triangular, j x j) per column; x += M (V y)
        for (int b = 0; b < nr; ++b) {
            std::vector<cdd> y(j);
            for (int i = j - 1; i >= 0; --i) {
                cdd acc = g[(size_t)i * nr + b];
                for (int k = i + 1; k < j; ++k) acc -= R[((size_t)k * m + i) * nr + b] * y[k];
                const cdd d = R[((size_t)i * m + i) * nr + b];
                y[i] = std::abs(d) > 0 ? acc / d : cdd(0);
            }
            for (int i = 0; i < j; ++i) {
                yh[(size_t)i * 2 * nr + 2 * b] = y[i].real();
                yh[(size_t)i * 2 * nr + 2 * b + 1] = y[i].imag();
            }
        }
        HIPC(hipMemcpyAsync(Yd, yh.data(), (size_t)j * 2 * nr * sizeof(double), hipMemcpyHostToDevice, st));
        launch_scale_zero(p->Pv.p, cnt, st);
        for (int i = 0; i < j; ++i) launch_col_axpy(p->Pv.p, V(i), Yd + (size_t)i * 2 * nr, 1.0, N, nr, st);
        if (pre) {
            applyM(p->Pv.p, p->Z.p);
            launch_axpy_update(p->X.p, p->Z.p, true, cnt, st);
        } else {
            launch_axpy_update(p->X.p, p->Pv.p, true, cnt, st);
        }
        HIPC(hipStreamSynchronize(st));  // the host copy of y is reused by the next cycle
        if (opts->tol > 0 && worst <= opts->tol) { converged = true; break; }
        if (opts->tol == 0 && total >= maxit) { converged = true; break; }
    }
    if (opts->tol == 0) converged = true;
    return total;
}

}  // namespace

// ============================================================ multi-instance solves
namespace {

// One instance of a multi-instance solve: its plan, batch width and user buffers.
struct Inst {
    fio_plan p;
    int nr;
    const void *u;
    void *out;
    int64_t ld;
};

// Per-level launch choices of a group of instances (autotuned, else heuristic):
// chain levels of Kd^* (in the solve's dtype) and Kd (complex128), and Gd steps.
// variant: stage kernel variant (0 vector, 1..6 matrix cores); kind: 0 LDS node
// kernel, 4/5 fused node kernel; cap: persistent grid cap (0 = full grid).
struct LevelChoice {
    int variant = -1, cap = 0;
};
struct MultiTune {
    std::vector<LevelChoice> adj, fwd, hif;
};
std::mutex g_multi_mu;
std::map<std::vector<int64_t>, MultiTune> g_multi_tune;  // key: dtype, (plan id, nrhs)...

std::vector<int64_t> multi_key(const std::vector<Inst> &I, bool dbl) {
    std::vector<int64_t> k{dbl ? 1 : 0};
    for (const Inst &i : I) {
        k.push_back((int64_t)(intptr_t)i.p);
        k.push_back(i.nr);
    }
    return k;
}

const MultiTune *multi_tuned(const std::vector<Inst> &I, bool dbl) {
    std::lock_guard<std::mutex> lk(g_multi_mu);
    auto it = g_multi_tune.find(multi_key(I, dbl));
    return it == g_multi_tune.end() ? nullptr : &it->second;
}

void forget_multi_tunes(fio_plan p) {
    std::lock_guard<std::mutex> lk(g_multi_mu);
    for (auto it = g_multi_tune.begin(); it != g_multi_tune.end();) {
        bool has = false;
        for (size_t j = 1; j < it->first.size(); j += 2) has |= it->first[j] == (int64_t)(intptr_t)p;
        it = has ? g_multi_tune.erase(it) : std::next(it);
    }
}

// Stage level j of every instance's chain (Kd if fwd, else Kd^*): one launch for the
// instances with at least 16 columns (matrix cores), one for the others (vector
// kernel).  in[i] / out[i]: the chain's input and output of instance i; the
// instance's own P/Q buffers carry the levels in between.
void multi_chain(const std::vector<Inst> &I, bool fwd, bool dbl, const std::vector<const void *> &in,
                 const std::vector<void *> &out, const std::vector<LevelChoice> *tune, hipStream_t st) {
    int S = 0;
    for (const Inst &i : I) S = std::max(S, (int)(fwd ? i.p->dfwd : i.p->dadj).size());
    for (int j = 0; j < S; ++j) {
        StageDev sv[MULTI_MAX], sm[MULTI_MAX];
        const void *xv[MULTI_MAX], *xm[MULTI_MAX];
        void *yv[MULTI_MAX], *ym[MULTI_MAX];
        int nv[MULTI_MAX], nm[MULTI_MAX], cv = 0, cm = 0;
        for (size_t k = 0; k < I.size(); ++k) {
            fio_plan p = I[k].p;
            const auto &hs = fwd ? p->host.fwd : p->adj;
            const auto &ds = fwd ? p->dfwd : p->dadj;
            const int Si = (int)ds.size();
            if (j >= Si) continue;
            const void *src = j == 0 ? in[k] : ((j - 1) % 2 == 0 ? p->P.p : p->Q.p);
            void *dst = j == Si - 1 ? out[k] : (j % 2 == 0 ? p->P.p : p->Q.p);
            const StageDev v = ds[j].view(dbl, hs[j]);
            if (I[k].nr >= 16 && v.fan <= 4) { sm[cm] = v; xm[cm] = src; ym[cm] = dst; nm[cm++] = I[k].nr; }
            else { sv[cv] = v; xv[cv] = src; yv[cv] = dst; nv[cv++] = I[k].nr; }
        }
        LevelChoice c;
        if (tune && j < (int)tune->size()) c = (*tune)[j];
        if (cm > 0) launch_stage_multi(sm, xm, ym, nm, cm, dbl, c.variant > 0 ? c.variant : (dbl ? 1 : 2), c.cap, st);
        if (cv > 0) launch_stage_multi(sv, xv, yv, nv, cv, dbl, 0, 0, st);
    }
}

// Gd in place on x[i] for every instance: step k of all instances whose sweep has a
// step k (counted from the finest level) in one launch per node kernel (the fused
// matrix-core kernel where every node fits it and the instance has 16 or more
// columns, else the LDS kernel; the gathered-GEMM path, for nodes that fit neither,
// runs per instance), then the top-level blocks, then the downward steps.
void multi_gd(const std::vector<Inst> &I, bool dbl, const std::vector<void *> &x, const std::vector<LevelChoice> *tune,
              hipStream_t st) {
    int K = 0;
    for (const Inst &i : I) K = std::max(K, (int)i.p->dhif.size());
    auto step = [&](int k, bool up) {
        HifStepDev hf[MULTI_MAX], hl[MULTI_MAX];
        void *xf[MULTI_MAX], *xl[MULTI_MAX];
        int nf[MULTI_MAX], nl[MULTI_MAX], cf = 0, cl = 0;
        LevelChoice c;
        if (tune && k < (int)tune->size()) c = (*tune)[k];
        const int fkind = c.variant == 4 ? 4 : 5;
        for (size_t i = 0; i < I.size(); ++i) {
            fio_plan p = I[i].p;
            if (k >= (int)p->dhif.size()) continue;
            const HifStepDev h = p->dhif[k].view(dbl);
            if (h.n_nodes == 0 || h.max_nr == 0) continue;  // empty or identity step
            const bool fused_ok = I[i].nr >= 16 && hif_fused_fits(h) && c.variant != 0;
            if (fused_ok) {
                hf[cf] = h; xf[cf] = x[i]; nf[cf++] = I[i].nr;
            } else if (hif_step_fits_lds(h, dbl)) {
                hl[cl] = h; xl[cl] = x[i]; nl[cl++] = I[i].nr;
            } else if (I[i].nr >= 16) {  // large nodes: the instance's own gathered-GEMM launches
                const auto *tn = p->tuned(dbl, I[i].nr);
                int mt = 1, cols = 64;
                bool m3 = false;
                if (!(tn && k < (int)tn->hif.size() && hif_gemm_tiling(tn->hif[k], mt, cols, m3))) {
                    mt = 1;
                    cols = 64;
                    m3 = false;
                }
                launch_hif_gemm_step(h, dbl, up, x[i], p->HT.p, I[i].nr, cols, st, mt, m3);
            } else {  // large nodes, small batches: matrix-vector products
                launch_hif_gemv_step(h, dbl, up, x[i], p->HT.p, I[i].nr, p->P.p,
                                     (size_t)p->max_coef * I[i].nr * (dbl ? 16 : 8), st);
            }
        }
        if (cf > 0) launch_hif_multi(hf, xf, nf, cf, dbl, up, fkind, c.cap, st);
        if (cl > 0) launch_hif_multi(hl, xl, nl, cl, dbl, up, 0, c.cap, st);
    };
    for (int k = 0; k < K; ++k) step(k, true);
    // top-level blocks: large ones as one-block FP64 stages (per instance), the small
    // ones with the direct kernel (one launch)
    const int32_t *ri[MULTI_MAX];
    const void *ra[MULTI_MAX];
    int rs[MULTI_MAX], rn[MULTI_MAX], cr = 0;
    void *rx[MULTI_MAX];
    for (size_t i = 0; i < I.size(); ++i) {
        fio_plan p = I[i].p;
        if (p->s0 == 0) continue;
        if (p->s0 >= 64) {
            root_apply(p, dbl, x[i], I[i].nr, st, plan_ws(p));
        } else {
            ri[cr] = (const int32_t *)p->root_idx.p; ra[cr] = p->A0inv.p; rs[cr] = p->s0; rx[cr] = x[i];
            rn[cr++] = I[i].nr;
        }
    }
    if (cr > 0) launch_root_multi(ri, ra, rs, rx, rn, cr, dbl, st);
    for (int k = K - 1; k >= 0; --k) step(k, false);
}

// The direct or refined solve of every instance, level by level (see fio_solve).
void multi_solve(const std::vector<Inst> &I, bool dbl, int refine, hipStream_t st) {
    const size_t n = I.size();
    const MultiTune *t = multi_tuned(I, dbl);
    std::vector<const void *> in(n);
    std::vector<void *> outv(n), xv(n);
    for (size_t i = 0; i < n; ++i) {
        fio_plan p = I[i].p;
        const int32_t *perm = (const int32_t *)p->perm.p;
        launch_gather(I[i].u, true, I[i].ld, perm, p->U.p, true, p->host.N, I[i].nr, st);
    }
    // d = Gd Kd^* r for r (complex128) in `src` of each instance, into V2 (dtype)
    auto gd_kh = [&](DBuf fio_plan_s::*src) {
        for (size_t i = 0; i < n; ++i) {
            fio_plan p = I[i].p;
            const int64_t cnt = p->host.N * I[i].nr;
            if (!dbl) launch_convert((p->*src).p, true, p->V3.p, false, cnt, st);
            in[i] = dbl ? (p->*src).p : p->V3.p;
            outv[i] = p->V2.p;
        }
        multi_chain(I, false, dbl, in, outv, t ? &t->adj : nullptr, st);
        multi_gd(I, dbl, outv, t ? &t->hif : nullptr, st);
    };
    gd_kh(&fio_plan_s::U);
    for (size_t i = 0; i < n; ++i)
        launch_convert(I[i].p->V2.p, dbl, I[i].p->X.p, true, I[i].p->host.N * I[i].nr, st);  // x0
    for (int it = 0; it < refine; ++it) {
        for (size_t i = 0; i < n; ++i) {
            in[i] = I[i].p->X.p;
            xv[i] = I[i].p->V1.p;
        }
        multi_chain(I, true, true, in, xv, t ? &t->fwd : nullptr, st);  // Kd x, FP64
        for (size_t i = 0; i < n; ++i)
            launch_residual(I[i].p->U.p, I[i].p->V1.p, I[i].p->R.p, true, I[i].p->host.N * I[i].nr, st);
        gd_kh(&fio_plan_s::R);
        for (size_t i = 0; i < n; ++i)
            launch_axpy_update(I[i].p->X.p, I[i].p->V2.p, dbl, I[i].p->host.N * I[i].nr, st);
    }
    for (size_t i = 0; i < n; ++i) {
        fio_plan p = I[i].p;
        launch_scatter(p->X.p, true, (const int32_t *)p->perm.p, I[i].out, true, I[i].ld, p->host.N, I[i].nr, st);
    }
}

// Validates a multi-instance call, takes every plan's lock (in address order) and
// sizes the workspaces.
struct MultiLock {
    std::vector<std::unique_lock<std::mutex>> locks;
};
std::vector<Inst> multi_setup(int n_inst, const fio_plan *plans, const void *const *u, void *const *out,
                              const int64_t *nrhs, const int64_t *ld, hipStream_t st, MultiLock &ml) {
    if (n_inst < 1 || n_inst > MULTI_MAX) fail(FIO_ERR_ARG, "n_inst must be 1.." + std::to_string(MULTI_MAX));
    if (!plans || !nrhs || !ld || (u == nullptr) != (out == nullptr)) fail(FIO_ERR_ARG, "null argument");
    std::vector<Inst> I;
    for (int i = 0; i < n_inst; ++i) {
        fio_plan p = plans[i];
        check_apply_args(p, nrhs[i], ld[i], u ? u[i] : (const void *)1, out ? out[i] : (void *)1);
        if (nrhs[i] < 1) fail(FIO_ERR_ARG, "every instance needs at least one column");
        if (p->device != plans[0]->device) fail(FIO_ERR_ARG, "all plans must be on one device");
        for (int j = 0; j < i; ++j)
            if (plans[j] == p) fail(FIO_ERR_ARG, "a plan appears twice (each instance uses its plan's workspace)");
        I.push_back(Inst{p, (int)nrhs[i], u ? u[i] : nullptr, out ? out[i] : nullptr, ld[i]});
    }
    std::vector<fio_plan> order(plans, plans + n_inst);
    std::sort(order.begin(), order.end());
    for (fio_plan p : order) ml.locks.emplace_back(p->mu);
    HIPC(hipSetDevice(plans[0]->device));
    for (const Inst &i : I) ensure_ws(i.p, i.nr, st);
    return I;
}

}  // namespace

extern "C" {

fio_status fio_solve_multi(int n_inst, const fio_plan *plans, const fio_solve_opts *opts, fio_dtype dt,
                           const void *const *u, void *const *out, const int64_t *nrhs, const int64_t *ld,
                           void *stream) {
    return guard([&] {
        TraceRange tr("fio solve multi %d", n_inst);
        if (!opts || !u || !out) fail(FIO_ERR_ARG, "null argument");
        if (dt != FIO_C64 && dt != FIO_C128) fail(FIO_ERR_ARG, "bad dtype");
        if (opts->mode != FIO_SOLVE_DIRECT && opts->mode != FIO_SOLVE_REFINE)
            fail(FIO_ERR_UNSUPPORTED, "multi-instance solves run DIRECT or REFINE");
        if (opts->tol != 0 || opts->spatial)
            fail(FIO_ERR_UNSUPPORTED, "multi-instance solves run a fixed number of steps (tol = 0), fhat output");
        if (opts->maxit < 0) fail(FIO_ERR_ARG, "bad iteration settings");
        hipStream_t st = (hipStream_t)stream;
        MultiLock ml;
        const std::vector<Inst> I = multi_setup(n_inst, plans, u, out, nrhs, ld, st, ml);
        multi_solve(I, dt == FIO_C128, opts->mode == FIO_SOLVE_REFINE ? opts->maxit : 0, st);
    });
}

fio_status fio_multi_autotune(int n_inst, const fio_plan *plans, fio_dtype dt, const int64_t *nrhs, int reps,
                              void *stream) {
    return guard([&] {
        if (dt != FIO_C64 && dt != FIO_C128) fail(FIO_ERR_ARG, "bad dtype");
        if (reps < 1) reps = 3;
        hipStream_t st = (hipStream_t)stream;
        std::vector<int64_t> ld(n_inst > 0 ? n_inst : 1);
        for (int i = 0; i < n_inst && plans; ++i) ld[i] = plans[i] ? plans[i]->host.N : 0;
        MultiLock ml;
        const std::vector<Inst> I = multi_setup(n_inst, plans, nullptr, nullptr, nrhs, ld.data(), st, ml);
        const bool dbl = dt == FIO_C128;
        const bool vb = I[0].p->host.prob.verbose != 0;
        for (const Inst &i : I) {  // defined inputs for the timed launches
            launch_scale_zero(i.p->P.p, i.p->max_coef * i.nr, st);
            launch_scale_zero(i.p->Q.p, i.p->max_coef * i.nr, st);
            launch_scale_zero(i.p->V2.p, i.p->host.N * i.nr, st);
            launch_scale_zero(i.p->X.p, i.p->host.N * i.nr, st);
        }
        hipEvent_t e0, e1;
        HIPC(hipEventCreate(&e0));
        HIPC(hipEventCreate(&e1));
        auto timeit = [&](auto &&fn) {
            fn();
            HIPC(hipEventRecord(e0, st));
            for (int r = 0; r < reps; ++r) fn();
            HIPC(hipEventRecord(e1, st));
            HIPC(hipEventSynchronize(e1));
            float ms = 0;
            HIPC(hipEventElapsedTime(&ms, e0, e1));
            return ms;
        };
        const int caps[] = {0, 4096, 2048, 1024};
        MultiTune t;
        // chain levels: every matrix-core tiling and grid cap, one level at a time
        for (int chain = 0; chain < 2; ++chain) {
            const bool fwd = chain == 0;
            const bool cdbl = fwd ? true : dbl;  // Kd runs in FP64 (the residual), Kd^* in dtype
            std::vector<LevelChoice> &out = fwd ? t.fwd : t.adj;
            int S = 0;
            for (const Inst &i : I) S = std::max(S, (int)(fwd ? i.p->dfwd : i.p->dadj).size());
            std::vector<const void *> in(I.size());
            std::vector<void *> ov(I.size());
            for (int j = 0; j < S; ++j) {
                LevelChoice best;
                float best_ms = 1e30f;
                for (int v = 1; v < STAGE_VARIANTS; ++v)
                    for (int cap : caps) {
                        if (!stage_multi_variant_ok(v)) continue;
                        std::vector<LevelChoice> one(S);
                        one[j] = LevelChoice{v, cap};
                        // the level alone: instances whose chain has it, P -> Q
                        const float ms = timeit([&] {
                            StageDev sm[MULTI_MAX];
                            const void *xm[MULTI_MAX];
                            void *ym[MULTI_MAX];
                            int nm[MULTI_MAX], cm = 0;
                            for (const Inst &i : I) {
                                const auto &hs = fwd ? i.p->host.fwd : i.p->adj;
                                const auto &ds = fwd ? i.p->dfwd : i.p->dadj;
                                if (j >= (int)ds.size() || i.nr < 16) continue;
                                sm[cm] = ds[j].view(cdbl, hs[j]);
                                xm[cm] = i.p->P.p; ym[cm] = i.p->Q.p; nm[cm++] = i.nr;
                            }
                            if (cm > 0) launch_stage_multi(sm, xm, ym, nm, cm, cdbl, v, cap, st);
                        });
                        if (ms < best_ms) { best_ms = ms; best = LevelChoice{v, cap}; }
                    }
                out.push_back(best);
                progress(vb, "multi tune %s level %d: variant %d cap %d %.4f ms", fwd ? "Kd c128" : "Kd^*", j,
                         best.variant, best.cap, best_ms / reps);
            }
        }
        // Gd steps: the fused kernel (64 or 32 columns) or the LDS kernel, grid caps
        int K = 0;
        for (const Inst &i : I) K = std::max(K, (int)i.p->dhif.size());
        for (int k = 0; k < K; ++k) {
            LevelChoice best{5, 0};
            float best_ms = 1e30f;
            for (int kind : {4, 5, 0})
                for (int cap : caps) {
                    HifStepDev hs[MULTI_MAX];
                    void *xs[MULTI_MAX];
                    int ns[MULTI_MAX], c = 0;
                    bool ok = true;
                    for (const Inst &i : I) {
                        if (k >= (int)i.p->dhif.size() || i.p->dhif[k].base.n_nodes == 0) continue;
                        hs[c] = i.p->dhif[k].view(dbl);
                        if (kind != 0 && (i.nr < 16 || !hif_fused_fits(hs[c]))) { ok = false; break; }
                        if (kind == 0 && !hif_step_fits_lds(hs[c], dbl)) { ok = false; break; }
                        xs[c] = i.p->V2.p; ns[c++] = i.nr;
                    }
                    if (!ok || c == 0) continue;
                    const float ms = timeit([&] {
                        launch_hif_multi(hs, xs, ns, c, dbl, true, kind, cap, st);
                        launch_hif_multi(hs, xs, ns, c, dbl, false, kind, cap, st);
                    });
                    if (ms < best_ms) { best_ms = ms; best = LevelChoice{kind, cap}; }
                }
            t.hif.push_back(best);
            progress(vb, "multi tune Gd step %d: kind %d cap %d %.4f ms", k, best.variant, best.cap,
                     best_ms < 1e29f ? best_ms / reps : 0.f);
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        std::lock_guard<std::mutex> lk(g_multi_mu);
        g_multi_tune[multi_key(I, dbl)] = std::move(t);
    });
}

}  // extern "C"

extern "C" {

fio_status fio_solve(fio_plan p, const fio_solve_opts *opts, fio_dtype dt, const void *u, void *out,
                     int64_t nrhs, int64_t ld, fio_solve_info *info, void *stream) {
    return guard([&] {
        TraceRange tr("fio solve mode %d %s", opts ? (int)opts->mode : -1, dt == FIO_C128 ? "c128" : "c64");
        check_apply_args(p, nrhs, ld, u, out);
        if (!opts) fail(FIO_ERR_ARG, "null options");
        if (dt != FIO_C64 && dt != FIO_C128) fail(FIO_ERR_ARG, "bad dtype");
        if (opts->mode < FIO_SOLVE_DIRECT || opts->mode > FIO_SOLVE_GMRES) fail(FIO_ERR_ARG, "bad mode");
        if (opts->restart < 0) fail(FIO_ERR_ARG, "bad restart length");
        if (opts->maxit < 0 || opts->tol < 0) fail(FIO_ERR_ARG, "bad iteration settings");
        if (nrhs == 0) return;
        std::lock_guard<std::mutex> lk(p->mu);
        HIPC(hipSetDevice(p->device));
        hipStream_t st = (hipStream_t)stream;
        const bool dbl = dt == FIO_C128;
        const int nr = (int)nrhs;
        ensure_ws(p, nr, st);
        const int32_t *perm = (const int32_t *)p->perm.p;
        const int64_t N = p->host.N;
        const int64_t cnt = N * nr;
        double *scal = (double *)p->scal.p;
        std::vector<double> hs(8 * (size_t)nr);
        int iters = 0;
        double worst = 0;
        bool converged = true;
        // U: u in X tree order (complex128).  X: solution in Omega tree order (complex128).
        launch_gather(u, true, ld, perm, p->U.p, true, N, nr, st);
        auto gd_kh = [&](const void *r128, void *d_out) {
            // d_out (dtype) = Gd Kd^* r
            const void *src = r128;
            if (!dbl) {
                launch_convert(r128, true, p->V3.p, false, cnt, st);
                src = p->V3.p;
            }
            run_chain(p, false, dbl, src, d_out, nr, st);
            gd_inplace(p, dbl, d_out, nr, st);
        };
        // Operator applies on complex128 vectors, computed in dtype (V3, W: conversions).
        auto apply_chain = [&](bool fwd, const void *in128, void *out128) {
            if (dbl) {
                run_chain(p, fwd, true, in128, out128, nr, st);
            } else {
                launch_convert(in128, true, p->V3.p, false, cnt, st);
                run_chain(p, fwd, false, p->V3.p, p->W.p, nr, st);
                launch_convert(p->W.p, false, out128, true, cnt, st);
            }
        };
        // z = Gd r on complex128 vectors, computed in dtype (z may alias r).
        auto gd128 = [&](const void *r128, void *z128) {
            if (dbl) {
                if (z128 != r128) HIPC(hipMemcpyAsync(z128, r128, cnt * 16, hipMemcpyDeviceToDevice, st));
                gd_inplace(p, true, z128, nr, st);
            } else {
                launch_convert(r128, true, p->V3.p, false, cnt, st);
                gd_inplace(p, false, p->V3.p, nr, st);
                launch_convert(p->V3.p, false, z128, true, cnt, st);
            }
        };
        // PCG preconditioner: Gd, or the identity without preconditioning.
        auto precond = [&](const void *r128, void *z128) {
            if (!opts->precondition) HIPC(hipMemcpyAsync(z128, r128, cnt * 16, hipMemcpyDeviceToDevice, st));
            else gd128(r128, z128);
        };
        if (opts->mode == FIO_SOLVE_GMRES) {
            iters = gmres(p, opts, nr, apply_chain, gd128, st, worst, converged);
        } else if (opts->mode == FIO_SOLVE_DIRECT || opts->mode == FIO_SOLVE_REFINE) {
            gd_kh(p->U.p, p->V2.p);
            launch_convert(p->V2.p, dbl, p->X.p, true, cnt, st);  // x0 = Gd Kd^* u
            if (opts->mode == FIO_SOLVE_REFINE) {
                for (int it = 0; it < opts->maxit; ++it) {
                    TraceRange ti("fio refine iteration %d", it);
                    // r = u - Kd x with complex128 factors and FP64 accumulation
                    run_chain(p, true, true, p->X.p, p->V1.p, nr, st);
                    launch_residual(p->U.p, p->V1.p, p->R.p, true, cnt, st);
                    gd_kh(p->R.p, p->V2.p);
                    launch_axpy_update(p->X.p, p->V2.p, dbl, cnt, st);
                    ++iters;
                    if (opts->tol > 0 || (info && it + 1 == opts->maxit)) {
                        // ||dx|| / ||x|| per column
                        if (!dbl) launch_convert(p->V2.p, false, p->V1.p, true, cnt, st);
                        const void *dx = dbl ? p->V2.p : p->V1.p;
                        launch_colnorm2(dx, N, nr, (double *)p->red.p, reduce_partial_cap(N, nr), scal, st);
                        launch_colnorm2(p->X.p, N, nr, (double *)p->red.p, reduce_partial_cap(N, nr), scal + nr, st);
                        HIPC(hipMemcpyAsync(hs.data(), scal, 2 * nr * sizeof(double), hipMemcpyDeviceToHost, st));
                        HIPC(hipStreamSynchronize(st));
                        worst = 0;
                        for (int b = 0; b < nr; ++b)
                            worse(worst, std::sqrt(hs[b] / std::max(hs[nr + b], 1e-300)));
                        if (opts->tol > 0 && worst <= opts->tol) break;
                    }
                }
                if (opts->tol > 0 && worst > opts->tol) converged = false;
            }
        } else {
            // PCG on Kd^* Kd x = Kd^* u preconditioned by Gd (section 5).  Vectors are
            // complex128; the operator applies run in dtype.
            double *rz = scal, *rzn = scal + 2 * nr, *pAp = scal + 4 * nr, *nrm = scal + 6 * nr;
            const int64_t cap = reduce_partial_cap(N, nr);
            apply_chain(false, p->U.p, p->R.p);  // r = b = Kd^* u (x0 = 0)
            launch_colnorm2(p->R.p, N, nr, (double *)p->red.p, cap, nrm, st);
            std::vector<double> bnorm(nr);
            HIPC(hipMemcpyAsync(bnorm.data(), nrm, nr * sizeof(double), hipMemcpyDeviceToHost, st));
            launch_scale_zero(p->X.p, cnt, st);
            precond(p->R.p, p->Z.p);
            HIPC(hipMemcpyAsync(p->Pv.p, p->Z.p, cnt * 16, hipMemcpyDeviceToDevice, st));
            launch_coldot(p->R.p, p->Z.p, N, nr, (double *)p->red.p, cap, rz, st);
            HIPC(hipStreamSynchronize(st));
            converged = false;
            for (int it = 0; it < std::max(1, opts->maxit); ++it) {
                TraceRange ti("fio pcg iteration %d", it);
                apply_chain(true, p->Pv.p, p->V2.p);
                apply_chain(false, p->V2.p, p->V1.p);  // Ap (complex128 in V1)
                launch_coldot(p->Pv.p, p->V1.p, N, nr, (double *)p->red.p, cap, pAp, st);
                launch_pcg_xr(p->X.p, p->R.p, p->Pv.p, p->V1.p, rz, pAp, N, nr, st);
                ++iters;
                launch_colnorm2(p->R.p, N, nr, (double *)p->red.p, cap, nrm, st);
                HIPC(hipMemcpyAsync(hs.data(), nrm, nr * sizeof(double), hipMemcpyDeviceToHost, st));
                HIPC(hipStreamSynchronize(st));
                worst = 0;
                for (int b = 0; b < nr; ++b) worse(worst, std::sqrt(hs[b] / std::max(bnorm[b], 1e-300)));
                if (opts->tol > 0 && worst <= opts->tol) { converged = true; break; }
                if (opts->tol == 0 && it + 1 == opts->maxit) { converged = true; break; }
                precond(p->R.p, p->Z.p);
                launch_coldot(p->R.p, p->Z.p, N, nr, (double *)p->red.p, cap, rzn, st);
                launch_pcg_p(p->Pv.p, p->Z.p, rzn, rz, N, nr, st);
                HIPC(hipMemcpyAsync(rz, rzn, 2 * nr * sizeof(double), hipMemcpyDeviceToDevice, st));
            }
        }
        launch_scatter(p->X.p, true, perm, out, true, ld, N, nr, st);
        if (opts->spatial)
            launch_inverse_dft(out, ld, out, p->host.d, p->host.n, nr, p->V1.p, p->V2.p, st);
        if (info) {
            HIPC(hipStreamSynchronize(st));
            info->iters = iters;
            info->rel_resid = worst;
            // error against the exact solve: the iteration's part, plus cond e_a for the
            // fixed point Kd^{-1} u (or the normal-equation solution) against K^{-1} u
            const HostFactors &h = p->host;
            const double kap = std::max(1.0, h.cond_est), fixed = kap * h.e_a_est;
            const bool direct = opts->mode == FIO_SOLVE_DIRECT || (opts->mode == FIO_SOLVE_REFINE && iters == 0);
            double est;
            if (direct) {
                // FP32 applies add rounding of about 2^-24 per factor, compounded over the steps
                const double steps = (double)(h.fwd.size() + 2 * h.hif.steps.size() + 1);
                est = h.e_s_est + fixed + (dbl ? 0.0 : kap * 6e-8 * std::sqrt(steps));
            } else if (opts->mode == FIO_SOLVE_REFINE) {
                est = h.e_s_est * worst + fixed + kap * 1e-15;
            } else if (opts->mode == FIO_SOLVE_PCG) {
                est = kap * kap * worst + fixed;
            } else {
                est = kap * worst + fixed;
            }
            info->est_rel_err = est;
        }
        if (!converged) fail(FIO_ERR_NOT_CONVERGED, "tolerance not reached within maxit");
        if (std::isnan(worst)) fail(FIO_ERR_NOT_CONVERGED, "a column of the iteration is not finite");
    });
}

fio_status fio_inverse_dft(fio_plan p, const void *fhat, void *f, int64_t nrhs, int64_t ld, void *stream) {
    return guard([&] {
        check_apply_args(p, nrhs, ld, fhat, f);
        if (nrhs == 0) return;
        std::lock_guard<std::mutex> lk(p->mu);
        HIPC(hipSetDevice(p->device));
        ensure_ws(p, (int)nrhs, (hipStream_t)stream);
        launch_inverse_dft(fhat, ld, f, p->host.d, p->host.n, (int)nrhs, p->V1.p, p->V2.p, (hipStream_t)stream);
    });
}

}  // extern "C"
