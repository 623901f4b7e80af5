// Device side of the butterfly construction (section 2): the interpolative
// decompositions of the sampled low-rank blocks K_{l;ij}, batched over all pairs of
// a level.  Three FP64 kernels per batch:
//   k_id_sample  evaluates the sampled entries of K (section 1, eq6; the phases of
//                section 6) straight into device memory,
//   k_id_cpqr    column-pivoted Householder QR of each sample matrix, one workgroup
//                per matrix, until the rank criterion or the fixed rank is reached,
//   k_id_solve   the interpolation matrix T = R11^{-1} R12 by back substitution.
// The host keeps the bookkeeping (candidates, samples, assembly of the stages).
//
// Also the large dense work of the 2D skeletonization (section 4): the column ID of
// one tall stacked basis (k_lq_* kernels, one pivot step at a time, columns in
// parallel) and the Schur update, Cholesky factor and inverse of one large node
// (rocBLAS and rocSOLVER).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "butterfly.hpp"
#include "hif.hpp"

namespace fio {
namespace {

#define CHK(x)                                                                           \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess)                                                            \
            fail(e_ == hipErrorOutOfMemory ? FIO_ERR_NOMEM : FIO_ERR_DEVICE,             \
                 std::string(#x) + ": " + hipGetErrorString(e_));                        \
    } while (0)

constexpr int ID_THREADS = 256;   // four waves per matrix
constexpr int ID_NC_MAX = 1024;   // candidates per matrix (LDS norms and order)
constexpr int ID_NS_MAX = 1024;   // samples per matrix (16 rows per lane)

// Kernel tables in tree order (the device image of FioKernel).
struct KTab {
    int n = 0, phase = 0, amp_terms = 0;
    int64_t N = 0;
    const int *k1 = nullptr, *k2 = nullptr, *j1 = nullptr, *j2 = nullptr;
    const double *c1 = nullptr, *c2 = nullptr;
    const double *gx = nullptr, *hq = nullptr;   // amp_terms x N
};

// K(x_p, xi_q): the linear part of the phase reduced exactly in integers, the
// non-linear part in FP64, then a * exp(2 pi i Phi).
__device__ double2 k_entry(const KTab &t, int p, int q) {
    int64_t s = (int64_t)t.k1[p] * t.j1[q] + (int64_t)t.k2[p] * t.j2[q];
    s %= t.n;
    if (s < 0) s += t.n;
    double nl = 0.0;
    if (t.phase == FIO_PHASE_1D_EX1 || t.phase == FIO_PHASE_1D_EX2) {
        nl = t.c1[p] * fabs((double)t.j1[q]);
    } else if (t.phase == FIO_PHASE_2D_RADON) {
        const double a = t.c1[p] * t.j1[q], b = t.c2[p] * t.j2[q];
        nl = sqrt(a * a + b * b);
    }
    double ph = (double)s / t.n + (nl - floor(nl));
    ph -= floor(ph);
    double amp = 1.0;
    if (t.amp_terms > 0) {
        amp = 0.0;
        for (int k = 0; k < t.amp_terms; ++k) amp += t.gx[(int64_t)k * t.N + p] * t.hq[(int64_t)k * t.N + q];
    }
    double sn, cs;
    sincospi(2.0 * ph, &sn, &cs);
    return make_double2(amp * cs, amp * sn);
}

// W[b] (ns x nc, column-major): (s, c) = K(cand_c, samp_s) or K(samp_s, cand_c).
__global__ void k_id_sample(KTab t, const int *samp, const int *cand, int ns, int nc, int64_t nb,
                            int cand_is_x, double2 *W) {
    const int64_t per = (int64_t)ns * nc, total = per * nb;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = e / per, rem = e - b * per;
        const int c = (int)(rem / ns), s = (int)(rem - (int64_t)c * ns);
        const int pc = cand[b * nc + c], ps = samp[b * ns + s];
        W[e] = cand_is_x ? k_entry(t, pc, ps) : k_entry(t, ps, pc);
    }
}

// Sums over the 64 lanes; the xor butterfly leaves the same bits in every lane.
__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ double2 cjmul(double2 a, double2 b) {
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// Column-pivoted Householder QR of W[b] in place, one workgroup per matrix.  Wave w
// owns the trailing columns j = k+1+w (mod 4); lane l holds rows l + 64c (c < RPL).
// Column norms of the trailing rows are recomputed exactly after every step.  The
// pivot is the largest norm, the first position among equals.  Stops before step k
// if the pivot norm is at most tol_rel times the largest initial column norm
// (tol_rel > 0), and after kmax steps.  Upper triangle of the first k rows: R.
template <int RPL>
__global__ __launch_bounds__(ID_THREADS) void k_id_cpqr(double2 *W, int ns, int nc, int kmax, double tol_rel,
                                                      int *rank_out, int *perm_out) {
    __shared__ double nrm[ID_NC_MAX];
    __shared__ int ord[ID_NC_MAX];
    __shared__ double red_v[ID_THREADS / 64];
    __shared__ int red_i[ID_THREADS / 64];
    __shared__ double s_tol, s_pmax;
    __shared__ int s_piv;
    const int b = blockIdx.x;
    double2 *A = W + (int64_t)b * ns * nc;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    constexpr int NW = ID_THREADS / 64;

    for (int j = wv; j < nc; j += NW) {
        const double2 *cj = A + (int64_t)j * ns;
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < RPL; ++c) {
            const int i = lane + 64 * c;
            if (i < ns) s += cabs2(cj[i]);
        }
        s = wsum(s);
        if (lane == 0) { nrm[j] = s; ord[j] = j; }
    }
    __syncthreads();

    int k = 0;
    for (; k < kmax; ++k) {
        // pivot: largest remaining norm, first position among equals
        double bv = -1.0;
        int bi = nc;
        for (int j = k + (int)threadIdx.x; j < nc; j += ID_THREADS) {
            const double v = nrm[j];
            if (v > bv) { bv = v; bi = j; }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(bv, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        if (lane == 0) { red_v[wv] = bv; red_i[wv] = bi; }
        __syncthreads();
        if (threadIdx.x == 0) {
            double v = red_v[0];
            int i = red_i[0];
            for (int w = 1; w < NW; ++w)
                if (red_v[w] > v || (red_v[w] == v && red_i[w] < i)) { v = red_v[w]; i = red_i[w]; }
            s_piv = i;
            s_pmax = v;
            if (k == 0) s_tol = (tol_rel > 0) ? tol_rel * sqrt(fmax(v, 0.0)) : -1.0;
        }
        __syncthreads();
        const int p = s_piv;
        if (sqrt(fmax(s_pmax, 0.0)) <= s_tol) break;   // the same decision in every thread
        if (p != k) {
            double2 *ck = A + (int64_t)k * ns, *cp = A + (int64_t)p * ns;
            for (int i = threadIdx.x; i < ns; i += ID_THREADS) {
                const double2 t = ck[i];
                ck[i] = cp[i];
                cp[i] = t;
            }
            if (threadIdx.x == 0) {
                const double tv = nrm[k]; nrm[k] = nrm[p]; nrm[p] = tv;
                const int ti = ord[k]; ord[k] = ord[p]; ord[p] = ti;
            }
        }
        __syncthreads();

        // Householder reflector H = I - 2 w w^* / (w^* w) with w = x + e^{i arg x0} |x| e_k,
        // x = column k below row k - 1; H x = -e^{i arg x0} |x| e_k.
        const double2 *ck = A + (int64_t)k * ns;
        double2 w[RPL];
        double tail = 0.0;
#pragma unroll
        for (int c = 0; c < RPL; ++c) {
            const int i = lane + 64 * c;
            w[c] = (i >= k && i < ns) ? ck[i] : make_double2(0.0, 0.0);
            if (i > k) tail += cabs2(w[c]);
        }
        tail = wsum(tail);
        const double2 x0 = ck[k];
        const double ax0 = hypot(x0.x, x0.y);
        const double alpha = sqrt(ax0 * ax0 + tail);
        const double2 ph = (ax0 > 0) ? make_double2(x0.x / ax0, x0.y / ax0) : make_double2(1.0, 0.0);
        const double2 w0 = make_double2(x0.x + ph.x * alpha, x0.y + ph.y * alpha);
        const double wn2 = cabs2(w0) + tail;
#pragma unroll
        for (int c = 0; c < RPL; ++c)
            if (lane + 64 * c == k) w[c] = w0;

        for (int j = k + 1 + wv; j < nc; j += NW) {
            double2 *cj = A + (int64_t)j * ns;
            double2 v[RPL];
            double sr = 0.0, si = 0.0;
#pragma unroll
            for (int c = 0; c < RPL; ++c) {
                const int i = lane + 64 * c;
                v[c] = (i >= k && i < ns) ? cj[i] : make_double2(0.0, 0.0);
                const double2 t = cjmul(w[c], v[c]);
                sr += t.x;
                si += t.y;
            }
            double nn = 0.0;
            if (wn2 > 0) {
                sr = wsum(sr);
                si = wsum(si);
                const double2 tau = make_double2(2.0 * sr / wn2, 2.0 * si / wn2);
#pragma unroll
                for (int c = 0; c < RPL; ++c) {
                    const int i = lane + 64 * c;
                    if (i >= k && i < ns) {
                        const double2 d = cmul(tau, w[c]);
                        v[c].x -= d.x;
                        v[c].y -= d.y;
                        cj[i] = v[c];
                        if (i > k) nn += cabs2(v[c]);
                    }
                }
            } else {
#pragma unroll
                for (int c = 0; c < RPL; ++c)
                    if (lane + 64 * c > k) nn += cabs2(v[c]);
            }
            nn = wsum(nn);
            if (lane == 0) nrm[j] = nn;
        }
        __syncthreads();
        // R_kk (every wave has read column k; nothing below reads it again)
        if (threadIdx.x == 0) A[(int64_t)k * ns + k] = make_double2(-ph.x * alpha, -ph.y * alpha);
    }
    if (threadIdx.x == 0) rank_out[b] = k;
    for (int j = threadIdx.x; j < nc; j += ID_THREADS) perm_out[(int64_t)b * nc + j] = ord[j];
}

// T[b] = R11^{-1} R12 (k x (nc - k), column-major) from the factored W[b]; one wave
// per column of R12, lane l holding rows l + 64c.  A zero pivot gives a zero row.
template <int RPL>
__global__ __launch_bounds__(ID_THREADS) void k_id_solve(const double2 *W, int ns, int nc, int k, double2 *T) {
    const int b = blockIdx.x;
    const double2 *A = W + (int64_t)b * ns * nc;
    double2 *Tb = T + (int64_t)b * k * (nc - k);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int j = wv; j < nc - k; j += ID_THREADS / 64) {
        const double2 *r12 = A + (int64_t)(k + j) * ns;
        double2 t[RPL];
#pragma unroll
        for (int c = 0; c < RPL; ++c) {
            const int i = lane + 64 * c;
            t[c] = (i < k) ? r12[i] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int c = RPL - 1; c >= 0; --c) {
            for (int l = 63; l >= 0; --l) {
                const int p = 64 * c + l;
                if (p >= k) continue;
                const double2 *rp = A + (int64_t)p * ns;
                const double2 d = rp[p];
                const double2 tv = make_double2(__shfl(t[c].x, l, 64), __shfl(t[c].y, l, 64));
                const double dd = cabs2(d);
                const double2 tp = (dd > 0) ? make_double2((tv.x * d.x + tv.y * d.y) / dd, (tv.y * d.x - tv.x * d.y) / dd)
                                            : make_double2(0.0, 0.0);
                if (lane == l) t[c] = tp;
#pragma unroll
                for (int c2 = 0; c2 < RPL; ++c2) {
                    if (c2 > c) continue;
                    const int i = lane + 64 * c2;
                    if (i < p) {
                        const double2 u = cmul(rp[i], tp);
                        t[c2].x -= u.x;
                        t[c2].y -= u.y;
                    }
                }
            }
        }
#pragma unroll
        for (int c = 0; c < RPL; ++c) {
            const int i = lane + 64 * c;
            if (i < k) Tb[(int64_t)j * k + i] = t[c];
        }
    }
}

template <int RPL>
void launch_qr(int64_t nb, double2 *W, int ns, int nc, int kmax, double tol, int *rank, int *perm) {
    hipLaunchKernelGGL(k_id_cpqr<RPL>, dim3((unsigned)nb), dim3(ID_THREADS), 0, 0, W, ns, nc, kmax, tol, rank, perm);
}
template <int RPL>
void launch_solve(int64_t nb, const double2 *W, int ns, int nc, int k, double2 *T) {
    hipLaunchKernelGGL(k_id_solve<RPL>, dim3((unsigned)nb), dim3(ID_THREADS), 0, 0, W, ns, nc, k, T);
}
// Rows per lane for a column of `rows` entries: 1, 2, 4, 8 or 16.
int rows_per_lane(int rows) {
    int r = 1;
    while (64 * r < rows) r *= 2;
    return r;
}

struct DevMem {
    void *p = nullptr;
    ~DevMem() {
        if (p) (void)hipFree(p);
    }
    void alloc(size_t b) {
        if (p) { (void)hipFree(p); p = nullptr; }
        if (b) CHK(hipMalloc(&p, b));
    }
};

// Device copies of the kernel tables, alive as long as the engine.
// A caller-defined FIO (FIO_PHASE_CALLBACK) has no device image: its entries are
// evaluated on the host (host points at the builder's kernel table, which outlives
// the engine) and copied to the device for the decompositions.
struct Tables {
    int device = 0;
    KTab view;
    DevMem k1, k2, j1, j2, c1, c2, gx, hq;
    const FioKernel *host = nullptr;
    Tables(int dev, const FioKernel &K) : device(dev) {
        CHK(hipSetDevice(dev));
        if (K.phi_fn) {
            host = &K;
            view.N = K.N;
            return;
        }
        auto up = [](DevMem &m, const void *src, size_t bytes) {
            m.alloc(bytes);
            if (bytes) CHK(hipMemcpy(m.p, src, bytes, hipMemcpyHostToDevice));
        };
        const size_t N = (size_t)K.N;
        up(k1, K.k1.data(), N * 4); up(k2, K.k2.data(), N * 4);
        up(j1, K.j1.data(), N * 4); up(j2, K.j2.data(), N * 4);
        up(c1, K.c1.data(), N * 8); up(c2, K.c2.data(), N * 8);
        const int nt = (int)K.gx.size();
        if (nt > 0) {
            std::vector<double> g(N * nt), h(N * nt);
            for (int k = 0; k < nt; ++k) {
                std::copy(K.gx[k].begin(), K.gx[k].end(), g.begin() + k * N);
                std::copy(K.hq[k].begin(), K.hq[k].end(), h.begin() + k * N);
            }
            up(gx, g.data(), g.size() * 8);
            up(hq, h.data(), h.size() * 8);
        }
        view.n = K.n; view.phase = (int)K.phase; view.amp_terms = nt; view.N = K.N;
        view.k1 = (const int *)k1.p; view.k2 = (const int *)k2.p;
        view.j1 = (const int *)j1.p; view.j2 = (const int *)j2.p;
        view.c1 = (const double *)c1.p; view.c2 = (const double *)c2.p;
        view.gx = (const double *)gx.p; view.hq = (const double *)hq.p;
    }
};

bool run_batch(const Tables &tb, const IdBatch &bt, const IdSink &sink, int nthreads) {
    if (bt.nb <= 0) return true;
    const int ns = bt.ns, nc = bt.nc;
    if (ns < 1 || nc < 1 || ns > ID_NS_MAX || nc > ID_NC_MAX) return false;
    if ((int64_t)bt.samp.size() != bt.nb * ns || (int64_t)bt.cand.size() != bt.nb * nc)
        fail(FIO_ERR_ARG, "batched ID: index arrays do not match the batch shape");
    for (int v : bt.samp) if (v < 0 || v >= tb.view.N) fail(FIO_ERR_ARG, "batched ID: sample out of range");
    for (int v : bt.cand) if (v < 0 || v >= tb.view.N) fail(FIO_ERR_ARG, "batched ID: candidate out of range");
    CHK(hipSetDevice(tb.device));
    const bool fixed = bt.fixed_rank > 0;
    const int kfix = fixed ? std::min({bt.fixed_rank, ns, nc}) : 0;
    const int kmax = fixed ? kfix : std::min({ns, nc, bt.max_rank > 0 ? bt.max_rank : nc});
    const int64_t nT = (int64_t)kfix * (nc - kfix);
    const size_t per = (size_t)ns * nc * 16 + (size_t)nT * 16 + (size_t)(ns + 2 * nc + 1) * 4;
    size_t freeb = 0, totalb = 0;
    CHK(hipMemGetInfo(&freeb, &totalb));
    const size_t budget = std::min<size_t>(freeb / 2, (size_t)8 << 30);
    const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(bt.nb, (int64_t)(budget / per)));
    DevMem W, T, S, C, R, P;
    W.alloc((size_t)chunk * ns * nc * 16);
    if (nT > 0) T.alloc((size_t)chunk * nT * 16);
    S.alloc((size_t)chunk * ns * 4);
    C.alloc((size_t)chunk * nc * 4);
    R.alloc((size_t)chunk * 4);
    P.alloc((size_t)chunk * nc * 4);
    std::vector<int> rank(chunk), perm((size_t)chunk * nc);
    std::vector<cd> Th((size_t)chunk * nT);
    const int rq = rows_per_lane(ns), rk = rows_per_lane(std::max(kfix, 1));
    for (int64_t b0 = 0; b0 < bt.nb; b0 += chunk) {
        const int64_t nbc = std::min(chunk, bt.nb - b0);
        CHK(hipMemcpy(S.p, bt.samp.data() + b0 * ns, (size_t)nbc * ns * 4, hipMemcpyHostToDevice));
        CHK(hipMemcpy(C.p, bt.cand.data() + b0 * nc, (size_t)nbc * nc * 4, hipMemcpyHostToDevice));
        const int64_t total = nbc * ns * nc;
        if (tb.host) {
            // caller's phase and amplitude: sample on the host, then upload
            std::vector<cd> Wh((size_t)total);
            const int *sp = bt.samp.data() + b0 * ns, *cp = bt.cand.data() + b0 * nc;
            const bool cx = bt.cand_is_x;
            parallel_for(nbc * nc, nthreads, [&](int64_t bc) {
                const int64_t b = bc / nc;
                const int c = (int)(bc - b * nc);
                const int pc = cp[b * nc + c];
                cd *col = Wh.data() + (size_t)bc * ns;
                for (int s2 = 0; s2 < ns; ++s2) {
                    const int ps = sp[b * ns + s2];
                    col[s2] = cx ? tb.host->entry(pc, ps) : tb.host->entry(ps, pc);
                }
            });
            CHK(hipMemcpy(W.p, Wh.data(), (size_t)total * 16, hipMemcpyHostToDevice));
        } else {
            const unsigned grid = (unsigned)std::min<int64_t>((total + 255) / 256, 1 << 20);
            hipLaunchKernelGGL(k_id_sample, dim3(grid), dim3(256), 0, 0, tb.view, (const int *)S.p,
                               (const int *)C.p, ns, nc, nbc, bt.cand_is_x ? 1 : 0, (double2 *)W.p);
            CHK(hipGetLastError());
        }
        double2 *w = (double2 *)W.p;
        const double tol = fixed ? 0.0 : bt.tol_rel;
        int *rp = (int *)R.p, *pp = (int *)P.p;
        switch (rq) {
            case 1: launch_qr<1>(nbc, w, ns, nc, kmax, tol, rp, pp); break;
            case 2: launch_qr<2>(nbc, w, ns, nc, kmax, tol, rp, pp); break;
            case 4: launch_qr<4>(nbc, w, ns, nc, kmax, tol, rp, pp); break;
            case 8: launch_qr<8>(nbc, w, ns, nc, kmax, tol, rp, pp); break;
            default: launch_qr<16>(nbc, w, ns, nc, kmax, tol, rp, pp); break;
        }
        CHK(hipGetLastError());
        if (nT > 0) {
            double2 *t = (double2 *)T.p;
            switch (rk) {
                case 1: launch_solve<1>(nbc, w, ns, nc, kfix, t); break;
                case 2: launch_solve<2>(nbc, w, ns, nc, kfix, t); break;
                case 4: launch_solve<4>(nbc, w, ns, nc, kfix, t); break;
                case 8: launch_solve<8>(nbc, w, ns, nc, kfix, t); break;
                default: launch_solve<16>(nbc, w, ns, nc, kfix, t); break;
            }
            CHK(hipGetLastError());
        }
        CHK(hipMemcpy(rank.data(), R.p, (size_t)nbc * 4, hipMemcpyDeviceToHost));
        CHK(hipMemcpy(perm.data(), P.p, (size_t)nbc * nc * 4, hipMemcpyDeviceToHost));
        if (nT > 0) CHK(hipMemcpy(Th.data(), T.p, (size_t)nbc * nT * 16, hipMemcpyDeviceToHost));
        for (int64_t t = 0; t < nbc; ++t)
            if (fixed && rank[t] != kfix) fail(FIO_ERR_DEVICE, "batched ID: pivot count differs from the fixed rank");
        parallel_for(nbc, nthreads, [&](int64_t t) {
            sink(b0 + t, rank[t], perm.data() + t * nc, nT > 0 ? Th.data() + t * nT : nullptr);
        });
    }
    return true;
}

#define RB(x)                                                                                 \
    do {                                                                                      \
        rocblas_status s_ = (x);                                                              \
        if (s_ != rocblas_status_success)                                                     \
            fail(FIO_ERR_DEVICE, std::string(#x) + ": " + rocblas_status_to_string(s_));      \
    } while (0)

// One lane of device work for the skeletonization hooks: its own stream, library
// handle and grow-only buffers (no frees between calls, so lanes do not wait on each
// other), used by one host thread at a time.
struct NodeEngine {
    int device = 0;
    hipStream_t st = nullptr;
    rocblas_handle h = nullptr;
    std::mutex mu;
    struct Buf {
        void *p = nullptr;
        size_t cap = 0;
    };
    Buf buf[10];
    ~NodeEngine() {
        (void)hipSetDevice(device);
        if (h) (void)rocblas_destroy_handle(h);
        for (Buf &b : buf)
            if (b.p) (void)hipFree(b.p);
        if (st) (void)hipStreamDestroy(st);
    }
    // Called with mu held: current device, stream and handle ready.
    void begin() {
        CHK(hipSetDevice(device));
        if (!st) CHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        if (!h) {
            RB(rocblas_create_handle(&h));
            RB(rocblas_set_stream(h, st));
            // no atomics: the same factors from the same inputs on every build
            RB(rocblas_set_atomics_mode(h, rocblas_atomics_not_allowed));
        }
        RB(rocblas_set_pointer_mode(h, rocblas_pointer_mode_host));
    }
    void *get(int slot, size_t bytes) {
        Buf &b = buf[slot];
        if (b.cap < bytes) {
            CHK(hipStreamSynchronize(st));
            if (b.p) CHK(hipFree(b.p));
            b.p = nullptr;
            b.cap = 0;
            CHK(hipMalloc(&b.p, std::max<size_t>(bytes, 256)));
            b.cap = std::max<size_t>(bytes, 256);
        }
        return b.p;
    }
    // Copies ordered on the lane's stream, complete on return.
    void copy(void *dst, const void *src, size_t bytes, hipMemcpyKind kind) {
        if (bytes == 0) return;
        CHK(hipMemcpyAsync(dst, src, bytes, kind, st));
        CHK(hipStreamSynchronize(st));
    }
};

// Lanes handed out round robin (one in use: see device_skel_hooks).
struct EnginePool {
    std::vector<std::unique_ptr<NodeEngine>> lanes;
    std::atomic<unsigned> next{0};
    EnginePool(int device, int n) {
        for (int i = 0; i < n; ++i) {
            lanes.emplace_back(new NodeEngine());
            lanes.back()->device = device;
        }
    }
    NodeEngine &pick() { return *lanes[next.fetch_add(1) % lanes.size()]; }
};

unsigned grid256(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1 << 16)); }

// ---- one large matrix: column-pivoted QR with column-parallel updates ----
// state[0]: set once the next pivot is below the tolerance; state[1]: pivots done.
// dstate[0]: absolute tolerance (from the largest initial column norm), dstate[1]:
// w^* w of the current reflector.  hh[0]: reflector head w_k, hh[1]: R_kk.

// nrm[j] = |A(:, j)|^2, one wave per column.
__global__ __launch_bounds__(256) void k_lq_norms(const double2 *A, int64_t m, int n, double *nrm) {
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= n) return;  // wave-uniform
    const double2 *c = A + j * m;
    double s = 0.0;
    for (int64_t i = lane; i < m; i += 64) s += cabs2(c[i]);
    s = wsum(s);
    if (lane == 0) nrm[j] = s;
}

// Block-wide sum over 256 threads (the same bits in every thread).
__device__ double bsum(double v, double *red) {
    v = wsum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

// Step k, one workgroup: previous R_kk, pivot (largest remaining norm, first among
// equals), tolerance test, column swap, reflector of column k.
__global__ __launch_bounds__(256) void k_lq_pivot(double2 *A, int64_t m, int n, int k, double *nrm, int *perm,
                                                  double tol_rel, int *state, double *dstate, double2 *hh) {
    __shared__ double red_v[4], red[4];
    __shared__ int red_i[4];
    __shared__ int s_p;
    __shared__ double s_v, s_tol;
    if (state[0]) return;  // the same value in every thread
    if (k > 0 && threadIdx.x == 0) A[(int64_t)(k - 1) * m + (k - 1)] = hh[1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double bv = -1.0;
    int bi = n;
    for (int j = k + (int)threadIdx.x; j < n; j += 256) {
        const double v = nrm[j];
        if (v > bv) { bv = v; bi = j; }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    if (lane == 0) { red_v[wv] = bv; red_i[wv] = bi; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = red_v[0];
        int i = red_i[0];
        for (int w = 1; w < 4; ++w)
            if (red_v[w] > v || (red_v[w] == v && red_i[w] < i)) { v = red_v[w]; i = red_i[w]; }
        s_p = i;
        s_v = v;
        if (k == 0) dstate[0] = (tol_rel > 0) ? tol_rel * sqrt(fmax(v, 0.0)) : -1.0;
        s_tol = dstate[0];
    }
    __syncthreads();
    const int p = s_p;
    if (sqrt(fmax(s_v, 0.0)) <= s_tol) {
        if (threadIdx.x == 0) state[0] = 1;
        return;
    }
    if (p != k) {
        double2 *ck = A + (int64_t)k * m, *cp = A + (int64_t)p * m;
        for (int64_t i = threadIdx.x; i < m; i += 256) {
            const double2 t = ck[i];
            ck[i] = cp[i];
            cp[i] = t;
        }
        if (threadIdx.x == 0) {
            const double tv = nrm[k]; nrm[k] = nrm[p]; nrm[p] = tv;
            const int ti = perm[k]; perm[k] = perm[p]; perm[p] = ti;
        }
    }
    __syncthreads();
    const double2 *ck = A + (int64_t)k * m;
    double tail = 0.0;
    for (int64_t i = k + 1 + threadIdx.x; i < m; i += 256) tail += cabs2(ck[i]);
    tail = bsum(tail, red);
    if (threadIdx.x == 0) {
        const double2 x0 = ck[k];
        const double ax0 = hypot(x0.x, x0.y);
        const double alpha = sqrt(ax0 * ax0 + tail);
        const double2 ph = (ax0 > 0) ? make_double2(x0.x / ax0, x0.y / ax0) : make_double2(1.0, 0.0);
        const double2 w0 = make_double2(x0.x + ph.x * alpha, x0.y + ph.y * alpha);
        hh[0] = w0;
        hh[1] = make_double2(-ph.x * alpha, -ph.y * alpha);
        dstate[1] = cabs2(w0) + tail;
        state[1] = k + 1;
    }
}

// Step k, trailing columns j > k, one wave per column: v -= (2 w^* v / w^* w) w with
// w = column k below row k - 1 (head hh[0]), then the exact norm of rows > k.
__global__ __launch_bounds__(256) void k_lq_update(double2 *A, int64_t m, int n, int k, double *nrm,
                                                   const int *state, const double *dstate, const double2 *hh) {
    if (state[0]) return;
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * 4;
    const double wn2 = dstate[1];
    const double2 w0 = hh[0];
    const double2 *wk = A + (int64_t)k * m;
    for (int64_t j = k + 1 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); j < n; j += nw) {
        double2 *v = A + j * m;
        double nn = 0.0;
        if (wn2 > 0) {
            double sr = 0.0, si = 0.0;
            for (int64_t i = k + lane; i < m; i += 64) {
                const double2 w = (i == k) ? w0 : wk[i];
                const double2 t = cjmul(w, v[i]);
                sr += t.x;
                si += t.y;
            }
            sr = wsum(sr);
            si = wsum(si);
            const double2 tau = make_double2(2.0 * sr / wn2, 2.0 * si / wn2);
            for (int64_t i = k + lane; i < m; i += 64) {
                const double2 w = (i == k) ? w0 : wk[i];
                const double2 d = cmul(tau, w);
                double2 x = v[i];
                x.x -= d.x;
                x.y -= d.y;
                v[i] = x;
                if (i > k) nn += cabs2(x);
            }
        } else {
            for (int64_t i = k + 1 + lane; i < m; i += 64) nn += cabs2(v[i]);
        }
        nn = wsum(nn);
        if (lane == 0) nrm[j] = nn;
    }
}

// R_kk of the last step when the loop ended without reaching the tolerance.
__global__ void k_lq_finish(double2 *A, int64_t m, const int *state, const double2 *hh) {
    if (threadIdx.x == 0 && state[0] == 0 && state[1] > 0)
        A[(int64_t)(state[1] - 1) * m + (state[1] - 1)] = hh[1];
}

// R (n x n, zero below the diagonal) from the upper triangle of A (lda rows).
__global__ __launch_bounds__(256) void k_upper_copy(const double2 *A, int64_t lda, int n, double2 *R) {
    const int64_t total = (int64_t)n * n;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t j = e / n, i = e - j * n;
        R[e] = (i <= j) ? A[j * lda + i] : make_double2(0.0, 0.0);
    }
}

// flags[b] = 1 if block b saw a non-finite entry of A (total entries).
__global__ __launch_bounds__(256) void k_nonfinite(const double2 *A, int64_t total, int *flags) {
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    int bad = 0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const double2 v = A[e];
        bad |= !(isfinite(v.x) && isfinite(v.y));
    }
    if (bad) any = 1;  // benign race: every writer stores 1
    __syncthreads();
    if (threadIdx.x == 0) flags[blockIdx.x] = any;
}

// Pivoted QR steps on the device (a: mrows x n, column-major, overwritten): rank k,
// the pivot order and the top k rows of R (k x n).
void device_cpqr_steps(NodeEngine &E, double2 *a, int64_t mrows, int n, double tol_rel, int &k,
                       std::vector<int> &order, Mat &R) {
    double *nrm = (double *)E.get(4, (size_t)n * 8);
    int *perm = (int *)E.get(5, (size_t)n * 4);
    int *st = (int *)E.get(6, 4 * sizeof(int));
    double *dst = (double *)E.get(7, 4 * sizeof(double));
    double2 *hh = (double2 *)E.get(8, 2 * 16);
    order.resize(n);
    for (int j = 0; j < n; ++j) order[j] = j;
    E.copy(perm, order.data(), (size_t)n * 4, hipMemcpyHostToDevice);
    const int zero[4] = {0, 0, 0, 0};
    E.copy(st, zero, sizeof(zero), hipMemcpyHostToDevice);
    hipLaunchKernelGGL(k_lq_norms, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, E.st, (const double2 *)a, mrows, n,
                       nrm);
    CHK(hipGetLastError());
    const int kmax = (int)std::min<int64_t>(mrows, n);
    int hs[4] = {0, 0, 0, 0};
    for (int s = 0; s < kmax; ++s) {
        hipLaunchKernelGGL(k_lq_pivot, dim3(1), dim3(256), 0, E.st, a, mrows, n, s, nrm, perm, tol_rel, st, dst, hh);
        const int cols = n - s - 1;
        if (cols > 0) {
            const unsigned g = (unsigned)std::min<int64_t>((cols + 3) / 4, 4096);
            hipLaunchKernelGGL(k_lq_update, dim3(g), dim3(256), 0, E.st, a, mrows, n, s, nrm, (const int *)st,
                               (const double *)dst, (const double2 *)hh);
        }
        if ((s & 31) == 31) {  // early exit once the tolerance has been reached
            E.copy(hs, st, sizeof(hs), hipMemcpyDeviceToHost);
            if (hs[0]) break;
        }
    }
    hipLaunchKernelGGL(k_lq_finish, dim3(1), dim3(64), 0, E.st, a, mrows, (const int *)st, (const double2 *)hh);
    CHK(hipGetLastError());
    E.copy(hs, st, sizeof(hs), hipMemcpyDeviceToHost);
    k = hs[1];
    E.copy(order.data(), perm, (size_t)n * 4, hipMemcpyDeviceToHost);
    R = Mat(k, n);
    if (k > 0) {
        CHK(hipMemcpy2DAsync(R.a.data(), (size_t)k * 16, a, (size_t)mrows * 16, (size_t)k * 16, (size_t)n,
                             hipMemcpyDeviceToHost, E.st));
        CHK(hipStreamSynchronize(E.st));
    }
}

bool big_column_id(NodeEngine &E, const Mat &Ah, double tol_rel, ColumnID &out) {
    const int64_t m0 = Ah.m;
    const int n0 = Ah.n;
    if (m0 < 1 || n0 < 1 || m0 > INT32_MAX) return false;
    // Exactly zero columns are redundant with zero interpolation coefficients; they
    // are left out of the factorization (the library QR turns them into NaNs).
    std::vector<int> nz, zc;
    for (int j = 0; j < n0; ++j) {
        const cd *c = Ah.col(j);
        bool any = false;
        for (int64_t i = 0; i < m0 && !any; ++i) any = c[i] != cd(0);
        (any ? nz : zc).push_back(j);
    }
    const int n = (int)nz.size();
    int k = 0;
    std::vector<int> order;
    Mat R;
    if (n > 0) {
        const Mat Ac = zc.empty() ? Mat() : cols_of(Ah, nz);
        const Mat &A = zc.empty() ? Ah : Ac;
        std::lock_guard<std::mutex> lk(E.mu);  // one host thread per lane
        E.begin();
        double2 *A0 = (double2 *)E.get(0, (size_t)m0 * n * 16);
        E.copy(A0, A.a.data(), (size_t)m0 * n * 16, hipMemcpyHostToDevice);
        // A tall matrix is first reduced to its triangular factor R (A = QR, Householder,
        // rocSOLVER): Q has orthonormal columns, so every column norm of every trailing
        // block, hence every pivot and R11^{-1} R12, is that of A, and the pivoted
        // steps touch n rows instead of m.  If that R holds a non-finite value the
        // steps run on A itself.
        bool qr = false;
        double2 *Rt = nullptr;
        if (m0 > n) {
            double2 *tau = (double2 *)E.get(2, (size_t)n * 16);
            RB(rocsolver_zgeqrf(E.h, (rocblas_int)m0, n, (rocblas_double_complex *)A0, (rocblas_int)m0,
                                (rocblas_double_complex *)tau));
            const int64_t nn = (int64_t)n * n;
            Rt = (double2 *)E.get(1, (size_t)nn * 16);
            hipLaunchKernelGGL(k_upper_copy, dim3(grid256(nn)), dim3(256), 0, E.st, (const double2 *)A0, m0, n, Rt);
            CHK(hipGetLastError());
            const unsigned G = std::min(grid256(nn), 1024u);
            int *flags = (int *)E.get(3, (size_t)G * sizeof(int));
            hipLaunchKernelGGL(k_nonfinite, dim3(G), dim3(256), 0, E.st, (const double2 *)Rt, nn, flags);
            CHK(hipGetLastError());
            std::vector<int> fl(G);
            E.copy(fl.data(), flags, (size_t)G * sizeof(int), hipMemcpyDeviceToHost);
            qr = std::find(fl.begin(), fl.end(), 1) == fl.end();
            if (!qr) E.copy(A0, A.a.data(), (size_t)m0 * n * 16, hipMemcpyHostToDevice);
        }
        if (qr) {
            device_cpqr_steps(E, Rt, n, n, tol_rel, k, order, R);
        } else {
            device_cpqr_steps(E, A0, m0, n, tol_rel, k, order, R);
        }
    }
    // map back to the columns of Ah; zero columns close the redundant set
    out.skel.resize(k);
    out.redund.clear();
    for (int q = 0; q < k; ++q) out.skel[q] = nz[order[q]];
    for (int q = k; q < n; ++q) out.redund.push_back(nz[order[q]]);
    out.redund.insert(out.redund.end(), zc.begin(), zc.end());
    out.T = Mat(k, n0 - k);
    // T = R11^{-1} R12 by back substitution, column by column (host)
    par_cols(n - k, (double)k * k * (n - k) / 2.0, [&](int64_t jj) {
        const int j = (int)jj;
        cd *t = out.T.col(j);
        const cd *r12 = R.col(k + j);
        for (int i = 0; i < k; ++i) t[i] = r12[i];
        for (int q = k - 1; q >= 0; --q) {
            const cd d = R(q, q);
            t[q] = (std::abs(d) > 0) ? t[q] / d : cd(0);
            const cd tq = t[q];
            const cd *rq = R.col(q);
            for (int i = 0; i < q; ++i) t[i] -= rq[i] * tq;
        }
    });
    return true;
}

// ---- dense algebra of one large skeletonization node ----

// Lower triangle of A (n x n, leading dimension n) := Hermitian part (A + A^*)/2.
__global__ __launch_bounds__(256) void k_herm_lower(double2 *A, int n) {
    const int64_t total = (int64_t)n * n;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t j = e / n;
        const int64_t i = e - j * n;
        if (i <= j) continue;
        const double2 l = A[e], u = A[i * n + j];
        A[e] = make_double2(0.5 * (l.x + u.x), 0.5 * (l.y - u.y));
    }
}

// Strict upper triangle of A (n x n) := 0.
__global__ __launch_bounds__(256) void k_zero_upper(double2 *A, int n) {
    const int64_t total = (int64_t)n * n;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t j = e / n;
        if (e - j * n < j) A[e] = make_double2(0.0, 0.0);
    }
}

bool big_node_device(NodeEngine &E, const Mat &Arr, const Mat &Asr, const Mat &Ass, const Mat &T, Mat &Linv, Mat &M,
                     Mat &delta) {
    const int nr = Arr.m, ns = Ass.m;
    if (nr < 1 || ns < 1 || Arr.n != nr || Asr.m != ns || Asr.n != nr || Ass.n != ns || T.m != ns || T.n != nr)
        return false;
    std::lock_guard<std::mutex> lk(E.mu);  // one host thread per lane
    E.begin();
    const size_t bR = (size_t)nr * nr * 16, bSR = (size_t)ns * nr * 16, bS = (size_t)ns * ns * 16;
    auto A = (rocblas_double_complex *)E.get(0, bR);   // Arr -> Atr -> L -> L^{-1}
    auto S = (rocblas_double_complex *)E.get(1, bSR);  // Asr -> Ats = Asr - Ass T
    auto Q = (rocblas_double_complex *)E.get(2, bS);   // Ass
    auto Tm = (rocblas_double_complex *)E.get(3, bSR); // T
    auto U = (rocblas_double_complex *)E.get(4, bSR);  // Ass T
    auto Mm = (rocblas_double_complex *)E.get(5, bSR);
    auto D = (rocblas_double_complex *)E.get(6, bS);
    auto dinfo = (rocblas_int *)E.get(7, sizeof(rocblas_int));
    E.copy(A, Arr.a.data(), bR, hipMemcpyHostToDevice);
    E.copy(S, Asr.a.data(), bSR, hipMemcpyHostToDevice);
    E.copy(Q, Ass.a.data(), bS, hipMemcpyHostToDevice);
    E.copy(Tm, T.a.data(), bSR, hipMemcpyHostToDevice);
    const rocblas_double_complex one(1.0, 0.0), mone(-1.0, 0.0), zero(0.0, 0.0);
    const auto N = rocblas_operation_none, C = rocblas_operation_conjugate_transpose;
    // U = Ass T; Atr = Arr - T^* Asr - Asr^* T + T^* U
    RB(rocblas_zgemm(E.h, N, N, ns, nr, ns, &one, Q, ns, Tm, ns, &zero, U, ns));
    RB(rocblas_zgemm(E.h, C, N, nr, nr, ns, &mone, Tm, ns, S, ns, &one, A, nr));
    RB(rocblas_zgemm(E.h, C, N, nr, nr, ns, &mone, S, ns, Tm, ns, &one, A, nr));
    RB(rocblas_zgemm(E.h, C, N, nr, nr, ns, &one, Tm, ns, U, ns, &one, A, nr));
    hipLaunchKernelGGL(k_herm_lower, dim3(grid256((int64_t)nr * nr)), dim3(256), 0, E.st, (double2 *)A, nr);
    CHK(hipGetLastError());
    // Ats = Asr - Ass T (in place of Asr, whose uses are done)
    RB(rocblas_zgemm(E.h, N, N, ns, nr, ns, &mone, Q, ns, Tm, ns, &one, S, ns));
    // L L^* = Atr, then L^{-1}
    rocblas_int info = 0;
    RB(rocsolver_zpotrf(E.h, rocblas_fill_lower, nr, A, nr, dinfo));
    E.copy(&info, dinfo, sizeof(info), hipMemcpyDeviceToHost);
    if (info != 0) return false;  // not numerically HPD: the host path decides
    RB(rocsolver_ztrtri(E.h, rocblas_fill_lower, rocblas_diagonal_non_unit, nr, A, nr, dinfo));
    E.copy(&info, dinfo, sizeof(info), hipMemcpyDeviceToHost);
    if (info != 0) return false;
    hipLaunchKernelGGL(k_zero_upper, dim3(grid256((int64_t)nr * nr)), dim3(256), 0, E.st, (double2 *)A, nr);
    CHK(hipGetLastError());
    // M = Ats L^{-*}; delta = -M M^*
    RB(rocblas_zgemm(E.h, N, C, ns, nr, nr, &one, S, ns, A, nr, &zero, Mm, ns));
    RB(rocblas_zgemm(E.h, N, C, ns, ns, nr, &mone, Mm, ns, Mm, ns, &zero, D, ns));
    Mat L(nr, nr), Mo(ns, nr), Do(ns, ns);
    E.copy(L.a.data(), A, bR, hipMemcpyDeviceToHost);
    E.copy(Mo.a.data(), Mm, bSR, hipMemcpyDeviceToHost);
    E.copy(Do.a.data(), D, bS, hipMemcpyDeviceToHost);
    Linv = std::move(L);
    M = std::move(Mo);
    delta = std::move(Do);
    return true;
}

bool hpd_inverse_device(NodeEngine &E, const Mat &Ah, Mat &inv) {
    const int n = Ah.n;
    if (n < 1 || Ah.m != n) return false;
    std::lock_guard<std::mutex> lk(E.mu);  // one host thread per lane
    E.begin();
    const size_t b = (size_t)n * n * 16;
    auto A = (rocblas_double_complex *)E.get(0, b);
    auto X = (rocblas_double_complex *)E.get(1, b);
    auto dinfo = (rocblas_int *)E.get(2, sizeof(rocblas_int));
    E.copy(A, Ah.a.data(), b, hipMemcpyHostToDevice);
    rocblas_int info = 0;
    RB(rocsolver_zpotrf(E.h, rocblas_fill_lower, n, A, n, dinfo));
    E.copy(&info, dinfo, sizeof(info), hipMemcpyDeviceToHost);
    if (info != 0) return false;
    RB(rocsolver_ztrtri(E.h, rocblas_fill_lower, rocblas_diagonal_non_unit, n, A, n, dinfo));
    E.copy(&info, dinfo, sizeof(info), hipMemcpyDeviceToHost);
    if (info != 0) return false;
    hipLaunchKernelGGL(k_zero_upper, dim3(grid256((int64_t)n * n)), dim3(256), 0, E.st, (double2 *)A, n);
    CHK(hipGetLastError());
    const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
    // A^{-1} = L^{-*} L^{-1}
    RB(rocblas_zgemm(E.h, rocblas_operation_conjugate_transpose, rocblas_operation_none, n, n, n, &one, A, n, A, n,
                     &zero, X, n));
    Mat out(n, n);
    E.copy(out.a.data(), X, b, hipMemcpyDeviceToHost);
    inv = std::move(out);
    return true;
}

}  // namespace

BatchedIdFactory device_id_factory(int device) {
    return [device](const FioKernel &K) -> BatchedId {
        auto tb = std::make_shared<Tables>(device, K);
        return [tb](const IdBatch &bt, const IdSink &sink) { return run_batch(*tb, bt, sink, 0); };
    };
}

// Runs a hook; when the device is out of memory the hook declines and the host path
// takes the node (the runtime's last-error state is cleared first).
template <class Fn> bool or_host(Fn &&fn) {
    try {
        return fn();
    } catch (const Error &e) {
        if (e.status != FIO_ERR_NOMEM) throw;
        (void)hipGetLastError();
        return false;
    }
}

SkelHooks device_skel_hooks(int device) {
    SkelHooks h;
    // One lane (stream) shared by the node loop's host threads.  With several lanes
    // the library's dense routines (zgemm, potrf, trtri) running concurrently on
    // several streams gave results that differed between identical builds, at times
    // badly (the coarse cells' Schur updates), while every lane only touches its own
    // buffers; on one lane repeated builds give identical factors.
    auto pool = std::make_shared<EnginePool>(device, 1);
    h.big_id = [pool](const Mat &A, double tol_rel, ColumnID &out) {
        return or_host([&] { return big_column_id(pool->pick(), A, tol_rel, out); });
    };
    h.big_node = [pool](const Mat &Arr, const Mat &Asr, const Mat &Ass, const Mat &T, Mat &Linv, Mat &M,
                        Mat &delta) {
        return or_host([&] { return big_node_device(pool->pick(), Arr, Asr, Ass, T, Linv, M, delta); });
    };
    h.hpd_inverse = [pool](const Mat &A, Mat &inv) {
        return or_host([&] { return hpd_inverse_device(pool->pick(), A, inv); });
    };
    return h;
}

}  // namespace fio
