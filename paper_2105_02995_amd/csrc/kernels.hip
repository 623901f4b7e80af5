// gfx950 kernels of the factor applies: butterfly stages, skeletonization steps,
// the top-level FP64 block, layout conversions and the FP64 vector updates of
// iterative refinement and preconditioned CG.
#include "kernels.hpp"

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <stdexcept>
#include <string>

namespace fio {

// ------------------------------------------------------------------ complex helpers
__device__ __forceinline__ float2 cz(float2) { return make_float2(0.f, 0.f); }
__device__ __forceinline__ double2 cz(double2) { return make_double2(0.0, 0.0); }

// acc + a*b
__device__ __forceinline__ float2 cfma(float2 acc, float2 a, float2 b) {
    acc.x = fmaf(a.x, b.x, acc.x);
    acc.x = fmaf(-a.y, b.y, acc.x);
    acc.y = fmaf(a.x, b.y, acc.y);
    acc.y = fmaf(a.y, b.x, acc.y);
    return acc;
}
__device__ __forceinline__ double2 cfma(double2 acc, double2 a, double2 b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}
// acc + conj(a)*b
__device__ __forceinline__ float2 cfmac(float2 acc, float2 a, float2 b) {
    acc.x = fmaf(a.x, b.x, acc.x);
    acc.x = fmaf(a.y, b.y, acc.x);
    acc.y = fmaf(a.x, b.y, acc.y);
    acc.y = fmaf(-a.y, b.x, acc.y);
    return acc;
}
__device__ __forceinline__ double2 cfmac(double2 acc, double2 a, double2 b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
    return acc;
}
template <class T> __device__ __forceinline__ T csub(T a, T b) {
    a.x -= b.x;
    a.y -= b.y;
    return a;
}
template <class To, class Ti> __device__ __forceinline__ To cvt(Ti v);
template <> __device__ __forceinline__ float2 cvt<float2, float2>(float2 v) { return v; }
template <> __device__ __forceinline__ double2 cvt<double2, double2>(double2 v) { return v; }
template <> __device__ __forceinline__ float2 cvt<float2, double2>(double2 v) {
    return make_float2((float)v.x, (float)v.y);
}
template <> __device__ __forceinline__ double2 cvt<double2, float2>(float2 v) {
    return make_double2((double)v.x, (double)v.y);
}

static void check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

static unsigned grid_for(int64_t work, int block) {
    int64_t g = (work + block - 1) / block;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 1 << 30));
}

// ------------------------------------------------------------------ butterfly stage
// One thread per output entry (o, a, b), b fastest: the factor entry is shared by
// the nrhs lanes of one row and the gathered input is read coalesced across b.
// Entry t = (o, a, b) of a stage's output.  Eight k-steps of loads are issued before
// their products, so a thread keeps eight loads in flight instead of waiting for
// each one (the loads do not depend on the accumulator).
template <class T>
__device__ __forceinline__ T stage_entry(int r_out, int r_in, int fan, const int32_t *__restrict__ idx,
                                         const T *__restrict__ A, const T *__restrict__ x, int nrhs, int64_t t) {
    constexpr int U = 8;
    const int b = (int)(t % nrhs);
    const int64_t t2 = t / nrhs;
    const int a = (int)(t2 % r_out);
    const int64_t o = t2 / r_out;
    const T *Ao = A + o * (int64_t)r_out * fan * r_in + a;
    T acc = cz(T());
    for (int q = 0; q < fan; ++q) {
        const T *xin = x + (int64_t)idx[o * fan + q] * r_in * nrhs + b;
        const T *Aq = Ao + (int64_t)q * r_in * r_out;
        int e = 0;
        for (; e + U <= r_in; e += U) {
            T av[U], xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                av[u] = Aq[(int64_t)(e + u) * r_out];
                xv[u] = xin[(int64_t)(e + u) * nrhs];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) acc = cfma(acc, av[u], xv[u]);
        }
        for (; e < r_in; ++e) acc = cfma(acc, Aq[(int64_t)e * r_out], xin[(int64_t)e * nrhs]);
    }
    return acc;
}

template <class T>
__global__ void __launch_bounds__(256) k_stage(int64_t n_out, int r_out, int r_in, int fan,
                                               const int32_t *__restrict__ idx,
                                               const T *__restrict__ A, const T *__restrict__ x,
                                               T *__restrict__ y, int nrhs) {
    const int64_t total = n_out * r_out * (int64_t)nrhs;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x)
        y[t] = stage_entry(r_out, r_in, fan, idx, A, x, nrhs, t);
}

// Small batches (fewer than 16 right-hand sides), bound by the factor bytes: a
// workgroup takes 64 rows of one output block (one row per lane) and NB right-hand
// sides; its four waves split the block's k range in four, so every wave streams a
// quarter of the block's columns with coalesced 64-row loads, U k-steps of loads
// issued before their products (the gathered input entries are the same for all
// lanes: one broadcast load each), and the four partial sums meet in LDS.  With
// ksplit > 1 (few output blocks, e.g. the one dense top-level block) the k range is
// also split over gridDim.z workgroups, each writing its partial sum to its own
// slice y + z * zstride, for the caller to add.
template <class T, int NB>
__global__ void __launch_bounds__(256) k_stage_nb(int64_t n_out, int r_out, int r_in, int fan,
                                                  const int32_t *__restrict__ idx, const T *__restrict__ A,
                                                  const T *__restrict__ x, T *__restrict__ y, int nrhs,
                                                  int rchunks, int ksplit, int64_t zstride) {
    constexpr int U = NB <= 2 ? 8 : (NB == 4 ? 4 : 2);
    __shared__ T red[3 * 64 * NB];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t o = blockIdx.x / rchunks;
    const int a = (int)(blockIdx.x - o * rchunks) * 64 + lane;
    const int ac = min(a, r_out - 1);
    const int c0 = blockIdx.y * NB;
    const int K = fan * r_in;
    const int ka = (int)((int64_t)K * blockIdx.z / ksplit), kz = (int)((int64_t)K * (blockIdx.z + 1) / ksplit);
    const int kb = ka + (((kz - ka) * w) >> 2), ke = ka + (((kz - ka) * (w + 1)) >> 2);
    y += blockIdx.z * zstride;
    int cj[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) cj[j] = min(c0 + j, nrhs - 1);
    T acc[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j] = cz(T());
    const T *Ao = A + o * (int64_t)r_out * K + ac;
    for (int k = kb; k < ke;) {
        const int q = k / r_in;
        const int kq = min(ke, (q + 1) * r_in);   // end of input block q in this wave's range
        // row of x for column k of the block: idx[q] * r_in + (k - q * r_in)
        const T *xr = x + ((int64_t)idx[o * fan + q] * r_in - (int64_t)q * r_in) * nrhs;
        for (; k + U <= kq; k += U) {
            T av[U], xv[U][NB];
#pragma unroll
            for (int u = 0; u < U; ++u) av[u] = Ao[(int64_t)(k + u) * r_out];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int j = 0; j < NB; ++j) xv[u][j] = xr[(int64_t)(k + u) * nrhs + cj[j]];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int j = 0; j < NB; ++j) acc[j] = cfma(acc[j], av[u], xv[u][j]);
        }
        for (; k < kq; ++k) {
            const T av = Ao[(int64_t)k * r_out];
#pragma unroll
            for (int j = 0; j < NB; ++j) acc[j] = cfma(acc[j], av, xr[(int64_t)k * nrhs + cj[j]]);
        }
    }
    if (w > 0) {
#pragma unroll
        for (int j = 0; j < NB; ++j) red[((w - 1) * 64 + lane) * NB + j] = acc[j];
    }
    __syncthreads();
    if (w == 0 && a < r_out) {
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            T s = acc[j];
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                const T t = red[(v * 64 + lane) * NB + j];
                s.x += t.x;
                s.y += t.y;
            }
            if (c0 + j < nrhs) y[(o * r_out + a) * (int64_t)nrhs + c0 + j] = s;
        }
    }
}

template <class T, int NB>
static void stage_nb_go(const StageDev &s, const void *x, void *y, int nrhs, hipStream_t st, int ksplit) {
    const int rchunks = (s.r_out + 63) / 64;
    const int64_t nb = s.n_out * rchunks;
    if (nb >= ((int64_t)1 << 31)) throw std::runtime_error("stage launch exceeds the grid limit");
    const dim3 g((unsigned)nb, (unsigned)((nrhs + NB - 1) / NB), (unsigned)ksplit);
    hipLaunchKernelGGL((k_stage_nb<T, NB>), g, dim3(256), 0, st, s.n_out, s.r_out, s.r_in, s.fan, s.idx,
                       (const T *)s.A, (const T *)x, (T *)y, nrhs, rchunks, ksplit,
                       s.n_out * (int64_t)s.r_out * nrhs);
}

template <class T>
static void launch_stage_nb(const StageDev &s, const void *x, void *y, int nrhs, hipStream_t st, int ksplit = 1) {
    if (nrhs <= 1) stage_nb_go<T, 1>(s, x, y, nrhs, st, ksplit);
    else if (nrhs <= 2) stage_nb_go<T, 2>(s, x, y, nrhs, st, ksplit);
    else if (nrhs <= 4) stage_nb_go<T, 4>(s, x, y, nrhs, st, ksplit);
    else stage_nb_go<T, 8>(s, x, y, nrhs, st, ksplit);
}

void launch_stage_nb_split(const StageDev &s, bool dbl, const void *x, void *y, int nrhs, int ksplit,
                           hipStream_t st) {
    if (ksplit < 1 || ksplit > 65535 || ksplit > s.fan * s.r_in)
        throw std::runtime_error("stage: k split out of range");
    if (dbl) launch_stage_nb<double2>(s, x, y, nrhs, st, ksplit);
    else launch_stage_nb<float2>(s, x, y, nrhs, st, ksplit);
    check_launch("stage (small batch, split k)");
}

// Batched stage on matrix cores.  One wave computes 16*MT rows of one output
// block for a chunk of 64 right-hand sides as four 16x16 tiles; the complex
// product uses four real MFMAs per k-step (Yr += Ar Xr - Ai Xi, Yi += Ar Xi + Ai Xr),
// accumulating in the working precision (FP32 for complex64, FP64 for complex128).
// MFMA 16x16x4 lane layout: A[l%16][l/16], B[l/16][l%16]; the accumulator entry v
// of lane l is D[4*(l/16)+v][l%16] for FP32 and D[l/16+4*v][l%16] for FP64.
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <class R> struct MF;
template <> struct MF<float> {
    using C = float2;
    using V4 = floatx4;
    static __device__ __forceinline__ V4 mma(float a, float b, V4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int drow(int lk, int v) { return 4 * lk + v; }
};
template <> struct MF<double> {
    using C = double2;
    using V4 = doublex4;
    static __device__ __forceinline__ V4 mma(double a, double b, V4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int drow(int lk, int v) { return lk + 4 * v; }
};

// Product of one block's factor A (r_out x K, column-major) with its gathered
// input, for the wave's 16*MT rows (first row mrow0) and 16*NT columns.  Input
// block q (q < fan <= 4) starts at xb + off[q] and its row e at + e*ld; this
// lane reads columns 16*nt + (lane % 16) of it.
// The k loop is software-pipelined: the loads of k-step i + STAGE_PF - 1 are
// issued before the MFMAs of k-step i, into STAGE_PF register buffers used in
// turn, so every wave keeps loads in flight while its matrix cores run.
// Loads are unconditional, from clamped (always valid) addresses: loads under a
// branch make the compiler wait for every load in flight before the next MFMAs.
// Rows at or beyond r_out and columns at or beyond ncols then hold finite
// duplicates of valid entries; they only feed output rows and columns that are
// never stored (each output column depends on its own input column only).  Past
// the last k the factor entry is replaced by zero, so those steps add nothing.
#ifndef FIO_STAGE_PF
#define FIO_STAGE_PF 2
#endif
constexpr int STAGE_PF = FIO_STAGE_PF;  // k-steps of loads in flight per wave, plus one

template <class R, int MT, int NT> struct Frag {
    typename MF<R>::C x[NT], a[MT];
};

// Start offsets of the (up to four) input blocks of one output block.  Four named
// members rather than an array: a lane-dependent index into an array would be
// lowered to a private-memory load.
struct Off4 {
    int64_t o0, o1, o2, o3;
    __device__ __forceinline__ int64_t operator()(int q) const {
        return q <= 0 ? o0 : q == 1 ? o1 : q == 2 ? o2 : o3;
    }
};

// Per-lane walk over k = lk, lk + 4, ...: input row pointer, factor column
// pointer and (block, entry) of the lane's next k.
template <class R, class P> struct KWalk {
    const P *xp;
    const typename MF<R>::C *ap;
    int q, e, k;
};

// Zero-filled device memory (static storage is zero-initialised): past the last k
// the factor operand is loaded from here, so it is exactly zero without any select
// on a loaded value.  64 double2 cover the 32 rows of the widest tile.
__device__ double2 g_zero_rows[64];

template <class R, int MT, int NT, class P>
__device__ __forceinline__ void frag_load(Frag<R, MT, NT> &f, KWalk<R, P> &w, int K, int r_in,
                                          const P *__restrict__ xb, const Off4 &off, int64_t ld,
                                          int r_out, const int (&colc)[NT], const int (&rowc)[MT]) {
    using C = typename MF<R>::C;
    const bool kv = w.k < K;
    // past the last k: input from a valid row (finite values), factor from zeros
    const P *xrow = kv ? w.xp : xb + off.o0;
    const C *acol = kv ? w.ap : reinterpret_cast<const C *>(g_zero_rows);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) f.x[nt] = xrow[colc[nt]];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) f.a[mt] = acol[kv ? rowc[mt] : mt * 16 + (threadIdx.x & 15)];
    w.k += 4;
    w.ap += 4 * (int64_t)r_out;
    w.e += 4;
    w.xp += 4 * ld;
    if (w.e >= r_in) {
        do { w.e -= r_in; ++w.q; } while (w.e >= r_in);
        w.xp = xb + off(w.q) + (int64_t)w.e * ld;
    }
}

// Accumulators of a wave's 16*MT x 16*NT complex tile: Yr = Ar Xr - Ai Xi and
// Yi = Ar Xi + Ai Xr as four real products per k-step (the three-product form is
// Acc3 below; its third accumulator set costs occupancy, so the tuner decides).
template <class R, int MT, int NT> struct Acc {
    using V4 = typename MF<R>::V4;
    using C = typename MF<R>::C;
    V4 re[MT][NT], im[MT][NT];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                re[mt][nt] = V4{0, 0, 0, 0};
                im[mt][nt] = V4{0, 0, 0, 0};
            }
    }
    __device__ __forceinline__ void mma(const Frag<R, MT, NT> &f) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const R ar = f.a[mt].x, ai = f.a[mt].y, nai = -f.a[mt].y;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                re[mt][nt] = MF<R>::mma(ar, f.x[nt].x, re[mt][nt]);
                im[mt][nt] = MF<R>::mma(ar, f.x[nt].y, im[mt][nt]);
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                re[mt][nt] = MF<R>::mma(nai, f.x[nt].y, re[mt][nt]);
                im[mt][nt] = MF<R>::mma(ai, f.x[nt].x, im[mt][nt]);
            }
        }
    }
    // entry v of this lane's part of tile (mt, nt)
    __device__ __forceinline__ C get(int mt, int nt, int v) const { return C{re[mt][nt][v], im[mt][nt][v]}; }
};

// The same tile with three real products per complex k-step (the 3M form):
// t1 = Ar Xr, t2 = Ai Xi, t3 = (Ar + Ai)(Xr + Xi); Yr = t1 - t2, Yi = t3 - t1 - t2.
// A quarter fewer matrix-core operations for a third more accumulators and two
// vector additions per operand; the imaginary part loses some relative accuracy
// where it is small against |Ar Xr| + |Ai Xi| (a few ulps in complex64, within what
// the FP64 refinement recovers).  Selected per stage by the autotuner.
template <class R, int MT, int NT> struct Acc3 {
    using V4 = typename MF<R>::V4;
    using C = typename MF<R>::C;
    V4 t1[MT][NT], t2[MT][NT], t3[MT][NT];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                t1[mt][nt] = V4{0, 0, 0, 0};
                t2[mt][nt] = V4{0, 0, 0, 0};
                t3[mt][nt] = V4{0, 0, 0, 0};
            }
    }
    __device__ __forceinline__ void mma(const Frag<R, MT, NT> &f) {
        R xs[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) xs[nt] = f.x[nt].x + f.x[nt].y;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const R ar = f.a[mt].x, ai = f.a[mt].y, as = ar + ai;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                t1[mt][nt] = MF<R>::mma(ar, f.x[nt].x, t1[mt][nt]);
                t2[mt][nt] = MF<R>::mma(ai, f.x[nt].y, t2[mt][nt]);
                t3[mt][nt] = MF<R>::mma(as, xs[nt], t3[mt][nt]);
            }
        }
    }
    __device__ __forceinline__ C get(int mt, int nt, int v) const {
        const R a = t1[mt][nt][v], b = t2[mt][nt][v];
        return C{a - b, t3[mt][nt][v] - a - b};
    }
};

// k-steps of loads in flight for an accumulator form: STAGE_PF, except for the
// complex64 three-product tiles, which measured fastest with 4 (2D n = 256 complex64
// chain 18.4 against 19.4 ms); deeper rings cost the FP64 and four-product tilings
// occupancy.
template <class ACC> struct PfOf { static constexpr int value = STAGE_PF; };
template <int MT, int NT> struct PfOf<Acc3<float, MT, NT>> { static constexpr int value = 4; };

// The product with explicit per-lane row offsets: row tile mt of this lane reads
// the factor at Ao + rowc[mt] + k * lda (column-major, leading dimension lda).
template <class R, int MT, int NT, class P, class ACC>
__device__ __forceinline__ void mfma_rows(ACC &acc, const typename MF<R>::C *__restrict__ Ao, int lda,
                                          int r_in, int K, const int (&rowc)[MT], int ncols,
                                          const P *__restrict__ xb, const Off4 &off, int64_t ld) {
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    acc.zero();
    int colc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) colc[nt] = min(nt * 16 + li, ncols - 1);
    KWalk<R, P> w;
    w.k = lk;
    w.q = lk / r_in;
    w.e = lk - w.q * r_in;
    w.ap = Ao + (int64_t)lk * lda;
    w.xp = xb + off(w.q) + (int64_t)w.e * ld;
    constexpr int PF = PfOf<ACC>::value;
    Frag<R, MT, NT> f[PF];
#pragma unroll
    for (int j = 0; j + 1 < PF; ++j) frag_load(f[j], w, K, r_in, xb, off, ld, lda, colc, rowc);
    for (int k0 = 0; k0 < K; k0 += 4 * PF) {
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            if (k0 + 4 * j >= K) break;  // wave-uniform
            frag_load(f[(j + PF - 1) % PF], w, K, r_in, xb, off, ld, lda, colc, rowc);
            acc.mma(f[j]);
        }
    }
}

template <class R, int MT, int NT, class P, class ACC>
__device__ __forceinline__ void mfma_block(ACC &acc, const typename MF<R>::C *__restrict__ Ao, int r_out,
                                           int r_in, int K, int mrow0, int ncols, const P *__restrict__ xb,
                                           const Off4 &off, int64_t ld) {
    const int li = threadIdx.x & 15;
    int rowc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) rowc[mt] = min(mrow0 + mt * 16 + li, r_out - 1);
    mfma_rows<R, MT, NT>(acc, Ao, r_out, r_in, K, rowc, ncols, xb, off, ld);
}

// XCD-aware workgroup order.  Workgroups of a launch are dispatched to the eight
// XCDs in turn (id % 8), each XCD with its own L2.  Logical id xcd*per + id/8
// gives every XCD a contiguous range of (block row, column chunk) pairs, chunk
// fastest, so the chunks of one block row run on one XCD one after the other
// and the factor blocks they share are read from HBM once.  The grid has
// 8*per >= nb*nch workgroups; those past the end get b >= nb.
constexpr int N_XCD = 8;
__device__ __forceinline__ void xcd_order(int64_t nb, int nch, int64_t &b, int &c) {
    const int64_t per = (nb * nch + N_XCD - 1) / N_XCD;
    const int64_t id = blockIdx.x;
    const int64_t lid = (id % N_XCD) * per + id / N_XCD;
    b = lid / nch;
    c = (int)(lid % nch);
}
static unsigned xcd_grid(int64_t nb, int nch) {
    const int64_t per = (nb * nch + N_XCD - 1) / N_XCD;
    if (per * N_XCD * 256 >= (int64_t(1) << 32))
        throw std::runtime_error("stage launch exceeds the grid limit (too many blocks x right-hand sides)");
    return (unsigned)(per * N_XCD);
}

// One workgroup's work of a stage launch: workgroup wg of the (output block, row
// chunk) waves, column chunk `chunk`.  Shared by the single-instance kernel and the
// multi-instance one.
template <class R, int MT, int NT, bool M3 = false>
__device__ __forceinline__ void stage_mfma_wg(int64_t n_out, int r_out, int r_in, int fan,
                                              const int32_t *__restrict__ idx,
                                              const typename MF<R>::C *__restrict__ A,
                                              const typename MF<R>::C *__restrict__ x,
                                              typename MF<R>::C *__restrict__ y, int nrhs, int mchunks,
                                              int64_t wg, int chunk) {
    using C = typename MF<R>::C;
    using V4 = typename MF<R>::V4;
    const int lane = threadIdx.x & 63;
    const int64_t wave = wg * 4 + (threadIdx.x >> 6);
    if (wave >= n_out * mchunks) return;  // wave-uniform
    const int64_t o = wave / mchunks;
    const int mc = (int)(wave % mchunks);
    const int n0 = chunk * (16 * NT);
    const int K = fan * r_in;
    const int li = lane & 15, lk = lane >> 4;
    typename std::conditional<M3, Acc3<R, MT, NT>, Acc<R, MT, NT>>::type acc;
    const int32_t *io = idx + o * fan;
    const int64_t bs = (int64_t)r_in * nrhs;
    const Off4 off{io[0] * bs, fan > 1 ? io[1] * bs : 0, fan > 2 ? io[2] * bs : 0, fan > 3 ? io[3] * bs : 0};
    mfma_block<R, MT, NT>(acc, A + o * (int64_t)r_out * K, r_out, r_in, K, mc * MT * 16, nrhs - n0,
                          x + n0, off, (int64_t)nrhs);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = (mc * MT + mt) * 16 + MF<R>::drow(lk, v);
                const int col = n0 + nt * 16 + li;
                if (row < r_out && col < nrhs)
                    y[(o * r_out + row) * (int64_t)nrhs + col] = acc.get(mt, nt, v);
            }
}

template <class R, int MT, int NT, bool M3 = false>
__global__ void __launch_bounds__(256) k_stage_mfma(int64_t n_out, int r_out, int r_in, int fan,
                                                    const int32_t *__restrict__ idx,
                                                    const typename MF<R>::C *__restrict__ A,
                                                    const typename MF<R>::C *__restrict__ x,
                                                    typename MF<R>::C *__restrict__ y, int nrhs,
                                                    int mchunks, int nchunks) {
    int64_t wg;
    int chunk;
    xcd_order((n_out * mchunks + 3) / 4, nchunks, wg, chunk);
    stage_mfma_wg<R, MT, NT, M3>(n_out, r_out, r_in, fan, idx, A, x, y, nrhs, mchunks, wg, chunk);
}

// Two consecutive stages a, b in one launch.  The blocks of two consecutive
// butterfly stages fall into closed groups: the stage-b outputs of a group read
// only stage-a outputs of that group.  A workgroup of four waves owns up to four
// stage-a blocks and four stage-b blocks of whole groups (table tab, 16 entries
// per workgroup: stage-a blocks, stage-b blocks, then for each stage-b block the
// workgroup slot of each of its fan_b <= 2 inputs; -1 pads).  Wave w computes
// stage-a block w of the workgroup into LDS, then stage-b block w from LDS, so
// the intermediate coefficients never leave the compute unit.  LDS holds only the
// r_mid valid rows of each block (dynamic size 4 * r_mid * 16*NT entries), which
// at ranks 22-25 lets three workgroups share a compute unit instead of two.
template <class R, int MT, int NT>
__global__ void __launch_bounds__(256) k_stage2_mfma(const int32_t *__restrict__ tab, int r_mid,
                                                     int r_in_a, int fan_a,
                                                     const int32_t *__restrict__ idx_a,
                                                     const typename MF<R>::C *__restrict__ A_a,
                                                     int r_out_b, int fan_b,
                                                     const typename MF<R>::C *__restrict__ A_b,
                                                     const typename MF<R>::C *__restrict__ x,
                                                     typename MF<R>::C *__restrict__ y, int nrhs,
                                                     int64_t n_wg, int nchunks) {
    using C = typename MF<R>::C;
    using V4 = typename MF<R>::V4;
    constexpr int COLS = 16 * NT;
    extern __shared__ char smem_raw[];
    C *mid = reinterpret_cast<C *>(smem_raw);   // [4][r_mid][COLS]
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    int64_t g;
    int chunk;
    xcd_order(n_wg, nchunks, g, chunk);
    if (g >= n_wg) return;  // workgroup-uniform, before the barrier
    const int32_t *t = tab + g * 16;
    const int n0 = chunk * COLS;
    const int ncols = nrhs - n0;
    Acc<R, MT, NT> acc;
    const int ba = t[w];
    if (ba >= 0) {  // wave-uniform
        const int Ka = fan_a * r_in_a;
        const int32_t *io = idx_a + (int64_t)ba * fan_a;
        const int64_t bs = (int64_t)r_in_a * nrhs;
        const Off4 off{io[0] * bs, fan_a > 1 ? io[1] * bs : 0, fan_a > 2 ? io[2] * bs : 0,
                       fan_a > 3 ? io[3] * bs : 0};
        mfma_block<R, MT, NT>(acc, A_a + (int64_t)ba * r_mid * Ka, r_mid, r_in_a, Ka, 0, ncols, x + n0,
                              off, (int64_t)nrhs);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = mt * 16 + MF<R>::drow(lk, v);
                if (row >= r_mid) continue;
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) mid[((int64_t)w * r_mid + row) * COLS + nt * 16 + li] = acc.get(mt, nt, v);
            }
    }
    __syncthreads();
    const int bb = t[4 + w];
    if (bb < 0) return;  // wave-uniform, after the only barrier
    const int Kb = fan_b * r_mid;
    const Off4 off{(int64_t)t[8 + 2 * w] * r_mid * COLS, fan_b > 1 ? (int64_t)t[9 + 2 * w] * r_mid * COLS : 0, 0, 0};
    mfma_block<R, MT, NT>(acc, A_b + (int64_t)bb * r_out_b * Kb, r_out_b, r_mid, Kb, 0, ncols,
                          mid, off, (int64_t)COLS);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = mt * 16 + MF<R>::drow(lk, v);
                const int col = n0 + nt * 16 + li;
                if (row < r_out_b && col < nrhs)
                    y[((int64_t)bb * r_out_b + row) * nrhs + col] = acc.get(mt, nt, v);
            }
}

// Stacked variant of the fused pair.  Two sibling blocks of one stage read the same
// inputs, so their rows are stacked into one 2r-row operand of MTS 16-row tiles
// (three for r <= 24: at r = 24 no padding, against 2 x 32 rows for the blocks
// apart, 25% fewer MFMAs; four for r <= 32).  Table (16 int32 per workgroup, one closed group): the
// two stage-a sibling pairs, the two stage-b sibling pairs, then for each stage-b
// pair the workgroup slots (0..3, position in the stage-a list) of its fan_b inputs.
// Wave w takes sibling pair w & 1 and the column half w >> 1 (16*NT columns each).
template <class R, int NT, int MTS>
__global__ void __launch_bounds__(256) k_stage2s_mfma(const int32_t *__restrict__ tab, int r_mid,
                                                      int r_in_a, int fan_a,
                                                      const int32_t *__restrict__ idx_a,
                                                      const typename MF<R>::C *__restrict__ A_a,
                                                      int r_out_b, int fan_b,
                                                      const typename MF<R>::C *__restrict__ A_b,
                                                      const typename MF<R>::C *__restrict__ x,
                                                      typename MF<R>::C *__restrict__ y, int nrhs,
                                                      int64_t n_wg, int nchunks) {
    using C = typename MF<R>::C;
    constexpr int HC = 16 * NT, COLS = 2 * HC;
    extern __shared__ char smem_raw[];
    C *mid = reinterpret_cast<C *>(smem_raw);   // [4][r_mid][COLS]
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int pr = w & 1, half = w >> 1;
    int64_t g;
    int chunk;
    xcd_order(n_wg, nchunks, g, chunk);
    if (g >= n_wg) return;  // workgroup-uniform, before the barrier
    const int32_t *t = tab + g * 16;
    const int c0 = half * HC;
    const int n0 = chunk * COLS + c0;
    const int ncols = nrhs - n0;
    Acc<R, MTS, NT> acc;
    const int a0 = t[2 * pr], a1 = t[2 * pr + 1];
    if (a0 >= 0 && ncols > 0) {  // wave-uniform
        const int Ka = fan_a * r_in_a;
        int rowc[MTS];
#pragma unroll
        for (int mt = 0; mt < MTS; ++mt) {
            const int row = min(mt * 16 + li, 2 * r_mid - 1);
            rowc[mt] = (row < r_mid) ? row : (a1 - a0) * r_mid * Ka + row - r_mid;
        }
        const int32_t *io = idx_a + (int64_t)a0 * fan_a;
        const int64_t bs = (int64_t)r_in_a * nrhs;
        const Off4 off{io[0] * bs, fan_a > 1 ? io[1] * bs : 0, fan_a > 2 ? io[2] * bs : 0,
                       fan_a > 3 ? io[3] * bs : 0};
        mfma_rows<R, MTS, NT>(acc, A_a + (int64_t)a0 * r_mid * Ka, r_mid, r_in_a, Ka, rowc, ncols, x + n0, off,
                              (int64_t)nrhs);
#pragma unroll
        for (int mt = 0; mt < MTS; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = mt * 16 + MF<R>::drow(lk, v);
                if (row >= 2 * r_mid) continue;
                const int slot = 2 * pr + (row >= r_mid ? 1 : 0);
                const int rr = row >= r_mid ? row - r_mid : row;
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    mid[((int64_t)slot * r_mid + rr) * COLS + c0 + nt * 16 + li] = acc.get(mt, nt, v);
            }
    }
    __syncthreads();
    const int b0 = t[4 + 2 * pr], b1 = t[5 + 2 * pr];
    if (b0 < 0 || ncols <= 0) return;  // wave-uniform, after the only barrier
    const int Kb = fan_b * r_mid;
    int rowc[MTS];
#pragma unroll
    for (int mt = 0; mt < MTS; ++mt) {
        const int row = min(mt * 16 + li, 2 * r_out_b - 1);
        rowc[mt] = (row < r_out_b) ? row : (b1 - b0) * r_out_b * Kb + row - r_out_b;
    }
    const Off4 off{(int64_t)t[8 + 2 * pr] * r_mid * COLS, fan_b > 1 ? (int64_t)t[9 + 2 * pr] * r_mid * COLS : 0, 0, 0};
    mfma_rows<R, MTS, NT>(acc, A_b + (int64_t)b0 * r_out_b * Kb, r_out_b, r_mid, Kb, rowc, ncols, mid + c0, off,
                          (int64_t)COLS);
#pragma unroll
    for (int mt = 0; mt < MTS; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = mt * 16 + MF<R>::drow(lk, v);
            if (row >= 2 * r_out_b) continue;
            const int blk = row >= r_out_b ? b1 : b0;
            const int rr = row >= r_out_b ? row - r_out_b : row;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int col = n0 + nt * 16 + li;
                if (col < nrhs) y[((int64_t)blk * r_out_b + rr) * nrhs + col] = acc.get(mt, nt, v);
            }
        }
}

// Three consecutive stages in one launch (the stacked form of k_stage2s_mfma carried
// one stage further).  In the 1D butterfly three consecutive stages still fall into
// closed groups of four blocks per stage; those of the second and third stage form
// two sibling pairs (blocks with equal input lists), the first stage's four read four
// different input pairs.  Wave w computes, on the column half w >> 1 (16*NT columns
// each), stage-a blocks 2 (w & 1) and 2 (w & 1) + 1 in 16-row tiles, then sibling
// pair w & 1 of stages b and c as one operand of MTS 16-row tiles.  The stage-a and
// stage-b outputs of the group stay in one LDS buffer of four block slots: stage b
// reads it, every wave passes a barrier, then stage b's results replace it.  Waves
// whose column half lies past the batch compute nothing but pass every barrier.
// Table: STAGE_TRIPLE_TAB int32 per workgroup (see StageTripleDev).
template <class R, int NT, int MTS>
__global__ void __launch_bounds__(256) k_stage3s_mfma(const int32_t *__restrict__ tab, int r_a, int r_in_a,
                                                      int fan_a, const int32_t *__restrict__ idx_a,
                                                      const typename MF<R>::C *__restrict__ A_a, int r_b, int fan_b,
                                                      const typename MF<R>::C *__restrict__ A_b, int r_c, int fan_c,
                                                      const typename MF<R>::C *__restrict__ A_c,
                                                      const typename MF<R>::C *__restrict__ x,
                                                      typename MF<R>::C *__restrict__ y, int nrhs, int64_t n_wg,
                                                      int nchunks) {
    using C = typename MF<R>::C;
    constexpr int HC = 16 * NT, COLS = 2 * HC;
    extern __shared__ char smem_raw[];
    C *mid = reinterpret_cast<C *>(smem_raw);   // [4][max(r_a, r_b)][COLS]
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int pr = w & 1, half = w >> 1;
    int64_t g;
    int chunk;
    xcd_order(n_wg, nchunks, g, chunk);
    if (g >= n_wg) return;  // workgroup-uniform, before the barriers
    const int32_t *t = tab + g * STAGE_TRIPLE_TAB;
    const int c0 = half * HC;
    const int n0 = chunk * COLS + c0;
    const int ncols = nrhs - n0;
    const bool live = ncols > 0;  // wave-uniform
    Acc<R, MTS, NT> acc;
    int rowc[MTS];
    // stage a: blocks 2 pr and 2 pr + 1 of the group, one after the other (their input
    // lists differ, so they do not stack), from the gathered global input
    if (live) {
        const int Ka = fan_a * r_in_a;
        const int64_t bs = (int64_t)r_in_a * nrhs;
        int rowa[2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) rowa[mt] = min(mt * 16 + li, r_a - 1);
        for (int j = 0; j < 2; ++j) {
            const int slot = 2 * pr + j;
            const int ab = t[slot];
            const int32_t *io = idx_a + (int64_t)ab * fan_a;
            const Off4 off{io[0] * bs, fan_a > 1 ? io[1] * bs : 0, fan_a > 2 ? io[2] * bs : 0,
                           fan_a > 3 ? io[3] * bs : 0};
            Acc<R, 2, NT> acca;
            mfma_rows<R, 2, NT>(acca, A_a + (int64_t)ab * r_a * Ka, r_a, r_in_a, Ka, rowa, ncols, x + n0, off,
                                (int64_t)nrhs);
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = mt * 16 + MF<R>::drow(lk, v);
                    if (row >= r_a) continue;
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
                        mid[((int64_t)slot * r_a + row) * COLS + c0 + nt * 16 + li] = acca.get(mt, nt, v);
                }
        }
    }
    __syncthreads();
    // stage b: sibling pair pr from the stage-a slots
    if (live) {
        const int b0 = t[4 + 2 * pr], b1 = t[5 + 2 * pr];
        const int Kb = fan_b * r_a;
#pragma unroll
        for (int mt = 0; mt < MTS; ++mt) {
            const int row = min(mt * 16 + li, 2 * r_b - 1);
            rowc[mt] = (row < r_b) ? row : (b1 - b0) * r_b * Kb + row - r_b;
        }
        const Off4 off{(int64_t)t[8 + 2 * pr] * r_a * COLS, fan_b > 1 ? (int64_t)t[9 + 2 * pr] * r_a * COLS : 0, 0, 0};
        mfma_rows<R, MTS, NT>(acc, A_b + (int64_t)b0 * r_b * Kb, r_b, r_a, Kb, rowc, ncols, mid + c0, off,
                              (int64_t)COLS);
    }
    __syncthreads();  // every wave has read its stage-b inputs: the slots can be replaced
    if (live) {
#pragma unroll
        for (int mt = 0; mt < MTS; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = mt * 16 + MF<R>::drow(lk, v);
                if (row >= 2 * r_b) continue;
                const int slot = 2 * pr + (row >= r_b ? 1 : 0);
                const int rr = row >= r_b ? row - r_b : row;
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    mid[((int64_t)slot * r_b + rr) * COLS + c0 + nt * 16 + li] = acc.get(mt, nt, v);
            }
    }
    __syncthreads();
    if (!live) return;  // after the last barrier
    // stage c: sibling pair pr from the stage-b slots, to global memory
    const int cb0 = t[12 + 2 * pr], cb1 = t[13 + 2 * pr];
    const int Kc = fan_c * r_b;
#pragma unroll
    for (int mt = 0; mt < MTS; ++mt) {
        const int row = min(mt * 16 + li, 2 * r_c - 1);
        rowc[mt] = (row < r_c) ? row : (cb1 - cb0) * r_c * Kc + row - r_c;
    }
    const Off4 off{(int64_t)t[16 + 2 * pr] * r_b * COLS, fan_c > 1 ? (int64_t)t[17 + 2 * pr] * r_b * COLS : 0, 0, 0};
    mfma_rows<R, MTS, NT>(acc, A_c + (int64_t)cb0 * r_c * Kc, r_c, r_b, Kc, rowc, ncols, mid + c0, off,
                          (int64_t)COLS);
#pragma unroll
    for (int mt = 0; mt < MTS; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = mt * 16 + MF<R>::drow(lk, v);
            if (row >= 2 * r_c) continue;
            const int blk = row >= r_c ? cb1 : cb0;
            const int rr = row >= r_c ? row - r_c : row;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int col = n0 + nt * 16 + li;
                if (col < nrhs) y[((int64_t)blk * r_c + rr) * nrhs + col] = acc.get(mt, nt, v);
            }
        }
}

template <class R, int NT, int MTS>
static void launch_triple_go(const StageTripleDev &t, const void *x, void *y, int nrhs, hipStream_t st) {
    using C = typename MF<R>::C;
    constexpr int COLS = 32 * NT;
    const int nch = (nrhs + COLS - 1) / COLS;
    const size_t lds = (size_t)4 * std::max(t.a.r_out, t.b.r_out) * COLS * sizeof(C);
    hipLaunchKernelGGL((k_stage3s_mfma<R, NT, MTS>), dim3(xcd_grid(t.n_wg, nch)), dim3(256), lds, st, t.tab,
                       t.a.r_out, t.a.r_in, t.a.fan, t.a.idx, (const C *)t.a.A, t.b.r_out, t.b.fan, (const C *)t.b.A,
                       t.c.r_out, t.c.fan, (const C *)t.c.A, (const C *)x, (C *)y, nrhs, t.n_wg, nch);
}

// 64 columns per workgroup for complex64, 32 for complex128 (one LDS buffer of four
// slots: 48 KiB at rank 24); three row tiles per sibling pair up to rank 24, four up
// to 32.
void launch_stage_triple(const StageTripleDev &t, bool dbl, const void *x, void *y, int nrhs, hipStream_t st) {
    const int rmax = std::max({t.a.r_out, t.b.r_out, t.c.r_out});
    if (!t.tab || t.n_wg <= 0 || rmax > 32 || t.a.fan > 4 || t.b.fan > 2 || t.c.fan > 2 || t.a.r_in < 1 ||
        t.b.r_in != t.a.r_out || t.c.r_in != t.b.r_out)
        throw std::runtime_error("stage triple cannot be fused");
    if (dbl) { if (rmax <= 24) launch_triple_go<double, 1, 3>(t, x, y, nrhs, st); else launch_triple_go<double, 1, 4>(t, x, y, nrhs, st); }
    else { if (rmax <= 24) launch_triple_go<float, 2, 3>(t, x, y, nrhs, st); else launch_triple_go<float, 2, 4>(t, x, y, nrhs, st); }
    check_launch("fused stage triple");
}

template <class R, int MT, int NT, bool M3 = false>
static void launch_mfma(const StageDev &s, const void *x, void *y, int nrhs, hipStream_t st) {
    using C = typename MF<R>::C;
    const int mtiles = (s.r_out + 15) / 16;
    const int mchunks = (mtiles + MT - 1) / MT;
    const int64_t waves = s.n_out * mchunks;
    const int nch = (nrhs + 16 * NT - 1) / (16 * NT);
    hipLaunchKernelGGL((k_stage_mfma<R, MT, NT, M3>), dim3(xcd_grid((waves + 3) / 4, nch)), dim3(256), 0, st,
                       s.n_out, s.r_out, s.r_in, s.fan, s.idx, (const C *)s.A, (const C *)x, (C *)y, nrhs, mchunks,
                       nch);
}

// Stage with the gathered input staged in LDS: one workgroup per (output block,
// column chunk of 16*NT right-hand sides); its four waves split the block's rows
// (16*MT each, so 64*MT >= r_out) and share the input, which is brought into LDS
// in chunks of LDS_KC k-rows, double buffered: the next chunk's global loads are in
// flight while the current chunk's products run, and every input entry is read
// from L2 once per workgroup instead of once per wave.  The factor rows stream
// from memory per wave with the same register prefetch as k_stage_mfma (past the
// last k the factor operand is zero).
constexpr int LDS_KC = 32;
template <class R, int NT> struct LdsTile {
    static constexpr int CW = 16 * NT, LDX = CW + 2;
    static constexpr int LPT = LDS_KC * CW / 256;  // staged entries per thread per chunk
};

template <class R, int MT, int NT>
__global__ void __launch_bounds__(256) k_stage_lds(int64_t n_out, int r_out, int r_in, int fan,
                                                   const int32_t *__restrict__ idx,
                                                   const typename MF<R>::C *__restrict__ A,
                                                   const typename MF<R>::C *__restrict__ x,
                                                   typename MF<R>::C *__restrict__ y, int nrhs, int nch) {
    using C = typename MF<R>::C;
    using T = LdsTile<R, NT>;
    constexpr int CW = T::CW, LDX = T::LDX, LPT = T::LPT, RSTEP = 256 / CW;
    extern __shared__ char smem_raw[];
    C *Xs = reinterpret_cast<C *>(smem_raw);  // 2 buffers of LDS_KC x LDX
    int64_t o;
    int chunk;
    xcd_order(n_out, nch, o, chunk);
    if (o >= n_out) return;  // workgroup-uniform
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    const int K = fan * r_in;
    const int n0 = chunk * CW;
    const int ncols = nrhs - n0;
    const int32_t *io = idx + o * fan;
    // staging: thread t loads column t % CW of rows t / CW + j * RSTEP of each chunk
    const int lcol = threadIdx.x % CW, lrow = threadIdx.x / CW;
    const C *xg = x + n0 + min(lcol, ncols - 1);
    R xre[LPT], xim[LPT];  // real and imaginary parts kept apart: plain registers
    // global loads of the chunk starting at k-row kc0 (past K: a valid row, which
    // meets a zero factor entry)
#define LDS_GLOAD(kc0)                                                                   \
    _Pragma("unroll") for (int j = 0; j < LPT; ++j) {                                    \
        const int k_ = min((kc0) + lrow + j * RSTEP, K - 1);                             \
        const int q_ = k_ / r_in;                                                        \
        const C v_ = xg[((int64_t)io[q_] * r_in + (k_ - q_ * r_in)) * nrhs];             \
        xre[j] = v_.x;                                                                   \
        xim[j] = v_.y;                                                                   \
    }
#define LDS_STORE(buf)                                                                   \
    _Pragma("unroll") for (int j = 0; j < LPT; ++j)                                      \
        Xs[((buf) * LDS_KC + lrow + j * RSTEP) * LDX + lcol] = C{xre[j], xim[j]};
    // this lane's factor rows; k-step s reads column k = 4 s + lk (zero past K)
    int rowc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) rowc[mt] = min(w * 16 * MT + mt * 16 + li, r_out - 1);
    const C *Ao = A + o * (int64_t)r_out * K;
#define LDS_ALOAD(slot, step)                                                            \
    {                                                                                    \
        const int k_ = 4 * (step) + lk;                                                  \
        const bool kv_ = k_ < K;                                                         \
        const C *acol_ = kv_ ? Ao + (int64_t)k_ * r_out : reinterpret_cast<const C *>(g_zero_rows); \
        _Pragma("unroll") for (int mt = 0; mt < MT; ++mt) ar[slot][mt] = acol_[kv_ ? rowc[mt] : mt * 16 + li]; \
    }
    Acc<R, MT, NT> acc;
    acc.zero();
    LDS_GLOAD(0)
    LDS_STORE(0)
    C ar[STAGE_PF][MT];
#pragma unroll
    for (int j = 0; j + 1 < STAGE_PF; ++j) LDS_ALOAD(j, j)
    __syncthreads();
    const int nchunks = (K + LDS_KC - 1) / LDS_KC;
    static_assert((LDS_KC / 4) % STAGE_PF == 0, "ring index must be a compile-time constant");
    for (int c = 0; c < nchunks; ++c) {
        const int buf = c & 1;
        const bool more = c + 1 < nchunks;
        if (more) { LDS_GLOAD((c + 1) * LDS_KC) }  // in flight during this chunk's products
        const C *Xb = Xs + buf * LDS_KC * LDX;
        const int step0 = c * (LDS_KC / 4);
        // every chunk runs all its k-steps: past K the factor operand is zero, so the
        // last chunk's extra steps add nothing, and the loop has no exit to unroll around
#pragma unroll
        for (int ks = 0; ks < LDS_KC / 4; ++ks) {
            // step0 is a multiple of STAGE_PF, so the ring slots are compile-time indices
            LDS_ALOAD((ks + STAGE_PF - 1) % STAGE_PF, step0 + ks + STAGE_PF - 1)
            Frag<R, MT, NT> f;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) f.a[mt] = ar[ks % STAGE_PF][mt];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) f.x[nt] = Xb[(4 * ks + lk) * LDX + nt * 16 + li];
            acc.mma(f);
        }
        if (more) { LDS_STORE(buf ^ 1) }  // that buffer was last read before the previous barrier
        __syncthreads();
    }
#undef LDS_GLOAD
#undef LDS_STORE
#undef LDS_ALOAD
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = w * 16 * MT + mt * 16 + MF<R>::drow(lk, v);
                const int col = n0 + nt * 16 + li;
                if (row < r_out && col < nrhs) y[(o * r_out + row) * (int64_t)nrhs + col] = acc.get(mt, nt, v);
            }
}

template <class R, int MT, int NT>
static void lds_go(const StageDev &s, const void *x, void *y, int nrhs, hipStream_t st) {
    using C = typename MF<R>::C;
    using T = LdsTile<R, NT>;
    const int nch = (nrhs + T::CW - 1) / T::CW;
    const size_t lds = (size_t)2 * LDS_KC * T::LDX * sizeof(C);
    hipLaunchKernelGGL((k_stage_lds<R, MT, NT>), dim3(xcd_grid(s.n_out, nch)), dim3(256), lds, st, s.n_out, s.r_out,
                       s.r_in, s.fan, s.idx, (const C *)s.A, (const C *)x, (C *)y, nrhs, nch);
}

// Whether the LDS-staged kernel applies: blocks of at most 192 rows (four waves of
// up to three 16-row tiles), at most four input blocks.
bool stage_lds_fits(const StageDev &s) { return s.r_out <= 192 && s.fan <= 4 && s.r_in >= 1 && s.r_out >= 1; }

template <class R, int NT>
static void launch_lds(const StageDev &s, const void *x, void *y, int nrhs, hipStream_t st) {
    if (s.r_out <= 64) lds_go<R, 1, NT>(s, x, y, nrhs, st);
    else if (s.r_out <= 128) lds_go<R, 2, NT>(s, x, y, nrhs, st);
    else lds_go<R, 3, NT>(s, x, y, nrhs, st);
}

// Right-hand-side counts from which the matrix-core path is used by default.
static const int MFMA_MIN_RHS = 16;

// Kernel variants of a stage launch (chosen by heuristics or by the autotuner):
//   0 vector kernel; 1..6 matrix cores with MT row tiles and NT 16-column tiles
//   (1: MT1 NT4, 2: MT2 NT4, 3: MT1 NT2, 4: MT2 NT2, 5: MT1 NT1, 6: MT2 NT1).
int stage_default_variant(const StageDev &s, bool dbl, int nrhs) {
    if (nrhs < MFMA_MIN_RHS) return s.r_out >= 48 ? STAGE_SMALL_BATCH : 0;
    const int mtiles = (s.r_out + 15) / 16;
    if (dbl || mtiles < 2) return 1;
    return 2;
}

template <class R>
static void launch_variant(int v, const StageDev &s, const void *x, void *y, int nrhs, hipStream_t st) {
    switch (v) {
        case 1: launch_mfma<R, 1, 4>(s, x, y, nrhs, st); break;
        case 2: launch_mfma<R, 2, 4>(s, x, y, nrhs, st); break;
        case 3: launch_mfma<R, 1, 2>(s, x, y, nrhs, st); break;
        case 4: launch_mfma<R, 2, 2>(s, x, y, nrhs, st); break;
        case 5: launch_mfma<R, 1, 1>(s, x, y, nrhs, st); break;
        case 8: launch_mfma<R, 4, 4>(s, x, y, nrhs, st); break;
        case 9: launch_mfma<R, 4, 2>(s, x, y, nrhs, st); break;
        case 12: launch_mfma<R, 2, 4, true>(s, x, y, nrhs, st); break;
        case 13: launch_mfma<R, 4, 2, true>(s, x, y, nrhs, st); break;
        case 14: launch_mfma<R, 2, 2, true>(s, x, y, nrhs, st); break;
        default: launch_mfma<R, 2, 1>(s, x, y, nrhs, st); break;
    }
}


void launch_stage(const StageDev &s, bool dbl, const void *x, void *y, int nrhs, hipStream_t st) {
    int v = (s.variant >= 0) ? s.variant : stage_default_variant(s, dbl, nrhs);
    // the matrix-core kernels walk at most four input blocks of at least one row
    if ((s.fan > 4 || s.r_in < 1 || s.r_out < 1) && v != STAGE_SMALL_BATCH) v = 0;
    if (s.r_in < 1 || s.r_out < 1) v = 0;
    if (v == STAGE_SMALL_BATCH) {
        if (dbl) launch_stage_nb<double2>(s, x, y, nrhs, st);
        else launch_stage_nb<float2>(s, x, y, nrhs, st);
        check_launch("stage (small batch)");
        return;
    }
    if (v == STAGE_LDS4 || v == STAGE_LDS2) {
        if (!stage_lds_fits(s)) v = 0;
        else {
            if (dbl) { if (v == STAGE_LDS4) launch_lds<double, 4>(s, x, y, nrhs, st); else launch_lds<double, 2>(s, x, y, nrhs, st); }
            else { if (v == STAGE_LDS4) launch_lds<float, 4>(s, x, y, nrhs, st); else launch_lds<float, 2>(s, x, y, nrhs, st); }
            check_launch("stage (LDS-staged input)");
            return;
        }
    }
    if (v > 0) {
        if (dbl) launch_variant<double>(v, s, x, y, nrhs, st);
        else launch_variant<float>(v, s, x, y, nrhs, st);
        check_launch("stage (matrix cores)");
        return;
    }
    const int64_t work = s.n_out * s.r_out * (int64_t)nrhs;
    const unsigned g = grid_for(work, 256);
    if (dbl)
        hipLaunchKernelGGL(k_stage<double2>, dim3(g), dim3(256), 0, st, s.n_out, s.r_out, s.r_in,
                           s.fan, s.idx, (const double2 *)s.A, (const double2 *)x, (double2 *)y, nrhs);
    else
        hipLaunchKernelGGL(k_stage<float2>, dim3(g), dim3(256), 0, st, s.n_out, s.r_out, s.r_in,
                           s.fan, s.idx, (const float2 *)s.A, (const float2 *)x, (float2 *)y, nrhs);
    check_launch("stage");
}

template <class R, int MT, int NT>
static void launch_pair(const StagePairDev &p, const void *x, void *y, int nrhs, hipStream_t st) {
    using C = typename MF<R>::C;
    const int nch = (nrhs + 16 * NT - 1) / (16 * NT);
    const size_t lds = (size_t)4 * p.a.r_out * 16 * NT * sizeof(C);
    hipLaunchKernelGGL((k_stage2_mfma<R, MT, NT>), dim3(xcd_grid(p.n_wg, nch)), dim3(256), lds, st, p.tab,
                       p.a.r_out, p.a.r_in, p.a.fan, p.a.idx, (const C *)p.a.A, p.b.r_out, p.b.fan,
                       (const C *)p.b.A, (const C *)x, (C *)y, nrhs, p.n_wg, nch);
}

bool stage_pair_fusable(int r_mid, int r_out_b, int fan_b) {
    return r_mid >= 1 && r_mid <= 32 && r_out_b >= 1 && r_out_b <= 32 && fan_b >= 1 && fan_b <= 2;
}

int stage_pair_variants(bool dbl) { return dbl ? 2 : 3; }

bool stage_pair_stackable(int r_mid, int r_out_b) { return r_mid >= 1 && r_mid <= 32 && r_out_b >= 1 && r_out_b <= 32; }

template <class R, int NT, int MTS>
static void launch_pair_stacked(const StagePairDev &p, const void *x, void *y, int nrhs, hipStream_t st) {
    using C = typename MF<R>::C;
    constexpr int COLS = 32 * NT;
    const int nch = (nrhs + COLS - 1) / COLS;
    const size_t lds = (size_t)4 * p.a.r_out * COLS * sizeof(C);
    hipLaunchKernelGGL((k_stage2s_mfma<R, NT, MTS>), dim3(xcd_grid(p.n_wg_s, nch)), dim3(256), lds, st, p.tab_s,
                       p.a.r_out, p.a.r_in, p.a.fan, p.a.idx, (const C *)p.a.A, p.b.r_out, p.b.fan,
                       (const C *)p.b.A, (const C *)x, (C *)y, nrhs, p.n_wg_s, nch);
}

void launch_stage_pair(const StagePairDev &p, bool dbl, int variant, const void *x, void *y, int nrhs,
                       hipStream_t st) {
    if (!stage_pair_fusable(p.a.r_out, p.b.r_out, p.b.fan) || p.b.r_in != p.a.r_out || p.a.fan > 4 ||
        p.a.r_in < 1)
        throw std::runtime_error("stage pair cannot be fused");
    if (variant == STAGE_PAIR_STACKED) {
        if (!p.tab_s || !stage_pair_stackable(p.a.r_out, p.b.r_out))
            throw std::runtime_error("stage pair cannot run stacked");
        // 64 columns per workgroup for complex64, 32 for complex128 (LDS); three row
        // tiles per sibling pair up to rank 24, four up to 32
        const bool m3 = std::max(p.a.r_out, p.b.r_out) <= 24;
        if (dbl) { if (m3) launch_pair_stacked<double, 1, 3>(p, x, y, nrhs, st); else launch_pair_stacked<double, 1, 4>(p, x, y, nrhs, st); }
        else { if (m3) launch_pair_stacked<float, 2, 3>(p, x, y, nrhs, st); else launch_pair_stacked<float, 2, 4>(p, x, y, nrhs, st); }
        check_launch("fused stage pair (stacked)");
        return;
    }
    const bool m2 = std::max(p.a.r_out, p.b.r_out) > 16;
    if (variant < 1 || variant > stage_pair_variants(dbl)) variant = 2;
    if (dbl) {
        // FP64 tiles of 16 x 64 columns would need 128 KiB of LDS: up to 32 columns.
        if (variant == 1) { if (m2) launch_pair<double, 2, 1>(p, x, y, nrhs, st); else launch_pair<double, 1, 1>(p, x, y, nrhs, st); }
        else { if (m2) launch_pair<double, 2, 2>(p, x, y, nrhs, st); else launch_pair<double, 1, 2>(p, x, y, nrhs, st); }
    } else {
        if (variant == 1) { if (m2) launch_pair<float, 2, 1>(p, x, y, nrhs, st); else launch_pair<float, 1, 1>(p, x, y, nrhs, st); }
        else if (variant == 2) { if (m2) launch_pair<float, 2, 2>(p, x, y, nrhs, st); else launch_pair<float, 1, 2>(p, x, y, nrhs, st); }
        else { if (m2) launch_pair<float, 2, 4>(p, x, y, nrhs, st); else launch_pair<float, 1, 4>(p, x, y, nrhs, st); }
    }
    check_launch("fused stage pair");
}

// ------------------------------------------------------------------ skeletonization steps
// One workgroup per node.  The node's blocks T (ns x nr), Linv (nr x nr) and
// M (ns x nr) are first copied into LDS with coalesced loads (when they fit),
// then its entries of x are gathered into LDS for a chunk of right-hand sides,
// transformed, and scattered back.  Nodes of one step own disjoint index sets,
// so workgroups never touch the same entries of x.
template <class T, bool UP, bool STAGED>
__device__ __forceinline__ void hif_node(const int64_t *__restrict__ desc, const int32_t *__restrict__ idx,
                                         const T *__restrict__ mat, T *__restrict__ x, int nrhs, int bchunk,
                                         int64_t v, int ychunk) {
    extern __shared__ char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);
    const int nr = (int)desc[4 * v], ns = (int)desc[4 * v + 1];
    const int32_t *ir = idx + desc[4 * v + 2];
    const int32_t *is = ir + nr;
    const T *gm = mat + desc[4 * v + 3];
    const int nmat = 2 * ns * nr + nr * nr;
    const T *Tm, *Li, *Mm;
    T *work = sm;
    if (STAGED) {
        for (int e = threadIdx.x; e < nmat; e += blockDim.x) sm[e] = gm[e];
        Tm = sm;
        work = sm + nmat;
        __syncthreads();
    } else {
        Tm = gm;
    }
    Li = Tm + (int64_t)ns * nr;  // nr x nr (lower)
    Mm = Li + (int64_t)nr * nr;  // ns x nr
    {
        const int b0 = ychunk * bchunk;
        const int bc = min(bchunk, nrhs - b0);
        T *xr = work, *xs = work + nr * bc, *y = xs + ns * bc;
        for (int e = threadIdx.x; e < (nr + ns) * bc; e += blockDim.x) {
            const int i = e / bc, b = e % bc;
            const int64_t g = (i < nr) ? ir[i] : is[i - nr];
            xr[e] = x[g * nrhs + b0 + b];  // xr and xs are contiguous in LDS
        }
        __syncthreads();
        if (UP) {
            // x_r -= T^* x_s
            for (int e = threadIdx.x; e < nr * bc; e += blockDim.x) {
                const int i = e / bc, b = e % bc;
                T acc = cz(T());
                const T *tc = Tm + (int64_t)i * ns;
                for (int k = 0; k < ns; ++k) acc = cfmac(acc, tc[k], xs[k * bc + b]);
                xr[e] = csub(xr[e], acc);
            }
            __syncthreads();
            // y = Linv x_r
            for (int e = threadIdx.x; e < nr * bc; e += blockDim.x) {
                const int i = e / bc, b = e % bc;
                T acc = cz(T());
                for (int k = 0; k <= i; ++k) acc = cfma(acc, Li[i + (int64_t)k * nr], xr[k * bc + b]);
                y[e] = acc;
            }
            __syncthreads();
            // x_s -= M y
            for (int e = threadIdx.x; e < ns * bc; e += blockDim.x) {
                const int k = e / bc, b = e % bc;
                T acc = cz(T());
                for (int i = 0; i < nr; ++i) acc = cfma(acc, Mm[k + (int64_t)i * ns], y[i * bc + b]);
                xs[e] = csub(xs[e], acc);
            }
            __syncthreads();
            for (int e = threadIdx.x; e < (nr + ns) * bc; e += blockDim.x) {
                const int i = e / bc, b = e % bc;
                if (i < nr) x[(int64_t)ir[i] * nrhs + b0 + b] = y[e];
                else x[(int64_t)is[i - nr] * nrhs + b0 + b] = xs[e - nr * bc];
            }
        } else {
            // y = x_r - M^* x_s
            for (int e = threadIdx.x; e < nr * bc; e += blockDim.x) {
                const int i = e / bc, b = e % bc;
                T acc = cz(T());
                const T *mc = Mm + (int64_t)i * ns;
                for (int k = 0; k < ns; ++k) acc = cfmac(acc, mc[k], xs[k * bc + b]);
                y[e] = csub(xr[e], acc);
            }
            __syncthreads();
            // x_r = Linv^* y
            for (int e = threadIdx.x; e < nr * bc; e += blockDim.x) {
                const int i = e / bc, b = e % bc;
                T acc = cz(T());
                const T *lc = Li + (int64_t)i * nr;
                for (int k = i; k < nr; ++k) acc = cfmac(acc, lc[k], y[k * bc + b]);
                xr[e] = acc;
            }
            __syncthreads();
            // x_s -= T x_r
            for (int e = threadIdx.x; e < ns * bc; e += blockDim.x) {
                const int k = e / bc, b = e % bc;
                T acc = cz(T());
                for (int i = 0; i < nr; ++i) acc = cfma(acc, Tm[k + (int64_t)i * ns], xr[i * bc + b]);
                xs[e] = csub(xs[e], acc);
            }
            __syncthreads();
            for (int e = threadIdx.x; e < (nr + ns) * bc; e += blockDim.x) {
                const int i = e / bc, b = e % bc;
                if (i < nr) x[(int64_t)ir[i] * nrhs + b0 + b] = xr[e];
                else x[(int64_t)is[i - nr] * nrhs + b0 + b] = xs[e - nr * bc];
            }
        }
        __syncthreads();
    }
}

template <class T, bool UP, bool STAGED>
__global__ void __launch_bounds__(256) k_hif(const int64_t *__restrict__ desc,
                                             const int32_t *__restrict__ idx,
                                             const T *__restrict__ mat, T *__restrict__ x,
                                             int nrhs, int bchunk, int64_t n_nodes, int nch) {
    int64_t v;
    int c;
    xcd_order(n_nodes, nch, v, c);   // the chunks of one node on one XCD, one after the other
    if (v >= n_nodes) return;
    hif_node<T, UP, STAGED>(desc, idx, mat, x, nrhs, bchunk, v, c);
}

// LDS one workgroup may use: the device's opt-in limit (160 KiB per CU on
// gfx950), capped with a margin; 64 KiB if the runtime does not report it.
static int hif_lds_budget() {
    static const int budget = [] {  // initialised once, thread-safe
        int dev = 0, v = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess || v <= 0)
            v = 64 * 1024;
        (void)hipGetLastError();
        return std::min(v, 144 * 1024);
    }();
    return budget;
}

template <class T, bool UP, bool ST>
static void hif_go(const HifStepDev &h, size_t lds, void *x, int nrhs, int bchunk, hipStream_t st) {
    static std::once_flag attr_once;  // plans may be used from several host threads
    std::call_once(attr_once, [] {
        (void)hipFuncSetAttribute((const void *)k_hif<T, UP, ST>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, hif_lds_budget());
    });
    const unsigned nch = (unsigned)((nrhs + bchunk - 1) / bchunk);
    hipLaunchKernelGGL((k_hif<T, UP, ST>), dim3(xcd_grid(h.n_nodes, (int)nch)), dim3(256), lds, st, h.desc,
                       h.idx, (const T *)h.mat, (T *)x, nrhs, bchunk, h.n_nodes, (int)nch);
}

void launch_hif_step(const HifStepDev &h, bool dbl, bool up, void *x, int nrhs, hipStream_t st) {
    if (h.n_nodes == 0) return;
    const int elt = dbl ? 16 : 8;
    const int64_t HIF_LDS = hif_lds_budget();
    const int per = std::max(1, h.max_vec);         // max over nodes of 2*nr + ns
    const int64_t matb = (int64_t)h.max_mat * elt;   // max over nodes of 2*ns*nr + nr*nr
    const bool staged = matb + (int64_t)per * elt <= HIF_LDS;
    const int64_t avail = staged ? HIF_LDS - matb : HIF_LDS;
    int bchunk = (int)std::max<int64_t>(1, std::min<int64_t>(nrhs, avail / ((int64_t)per * elt)));
    if (bchunk >= 64) bchunk = (bchunk / 64) * 64;
    // spread steps with few nodes over right-hand-side chunks (at least 16 columns each)
    const int64_t want = (int64_t)nrhs * h.n_nodes / 1024;
    if (want < bchunk) bchunk = (int)std::max<int64_t>(std::min<int64_t>(16, bchunk), want);
    const size_t lds = (size_t)(staged ? matb : 0) + (size_t)per * elt * bchunk;
    if ((int64_t)lds > HIF_LDS) throw std::runtime_error("skeletonization node exceeds LDS");
    if (dbl) {
        if (staged) { if (up) hif_go<double2, true, true>(h, lds, x, nrhs, bchunk, st); else hif_go<double2, false, true>(h, lds, x, nrhs, bchunk, st); }
        else { if (up) hif_go<double2, true, false>(h, lds, x, nrhs, bchunk, st); else hif_go<double2, false, false>(h, lds, x, nrhs, bchunk, st); }
    } else {
        if (staged) { if (up) hif_go<float2, true, true>(h, lds, x, nrhs, bchunk, st); else hif_go<float2, false, true>(h, lds, x, nrhs, bchunk, st); }
        else { if (up) hif_go<float2, true, false>(h, lds, x, nrhs, bchunk, st); else hif_go<float2, false, false>(h, lds, x, nrhs, bchunk, st); }
    }
    check_launch("hif step");
}

// ------------------------------------------------------------------ large skeletonization nodes
// Nodes whose blocks do not fit LDS run as gathered complex GEMMs on matrix
// cores, all nodes of a step in one launch per phase.  A tile is 16*MT rows of
// one node's output times 16*NT right-hand sides; its input rows are gathered
// from x (or the temporary t) through the node's index lists.
//   up:   0) x_r -= T^* x_s      1) t_r = Linv x_r      2) x_s -= M t_r; x_r = t_r
//   down: 3) t_r = x_r - M^* x_s 4) x_r = Linv^* t_r    5) x_s -= T x_r
// Every phase reads its factor column-major (the conjugate transposes are stored),
// so the loads of a tile's rows are coalesced.  Linv is lower triangular: phase 1
// stops at the tile's last row, phase 4 starts at its first.  The k loop is the
// pipelined one of the stage kernels.  Each wave first copies its tile's gathered
// row indices to LDS (one coalesced pass), so the loads of the gathered rows in the
// k loop do not wait on index loads from global memory.
template <class R, int MT, int NT> struct GWalk {
    const typename MF<R>::C *ap;
    int k, gnext;  // this lane's next k; gathered row of that k (already loaded)
};

template <class R, int MT, int NT>
__device__ __forceinline__ void gfrag_load(Frag<R, MT, NT> &f, GWalk<R, MT, NT> &w, int kend,
                                           const typename MF<R>::C *__restrict__ xb, int64_t ldx,
                                           const int32_t *__restrict__ kin, int ld,
                                           const int (&colc)[NT], const int (&rowc)[MT]) {
    using C = typename MF<R>::C;
    const bool kv = w.k < kend;
    const C *xrow = xb + (int64_t)w.gnext * ldx;
    const C *acol = kv ? w.ap : reinterpret_cast<const C *>(g_zero_rows);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) f.x[nt] = xrow[colc[nt]];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) f.a[mt] = acol[kv ? rowc[mt] : mt * 16 + (threadIdx.x & 15)];
    w.k += 4;
    w.ap += 4 * (int64_t)ld;
    w.gnext = kin[min(w.k, kend - 1)];
}

// k-steps of loads in flight in the skeletonization GEMMs: their tiles are narrow
// (few MFMAs per k-step), so more steps are kept in flight than in the stage kernels
// (measured best: 8 for complex64, 4 for complex128)
template <class R> struct HgPf { static constexpr int value = sizeof(R) == 4 ? 8 : 4; };

template <class R, int PH, int MT, int NT, bool M3 = false>
__global__ void __launch_bounds__(256) k_hgemm(const int64_t *__restrict__ desc,
                                               const int32_t *__restrict__ idx,
                                               const int32_t *__restrict__ tiles,
                                               int64_t ntiles,
                                               const typename MF<R>::C *__restrict__ mat,
                                               const typename MF<R>::C *__restrict__ matH,
                                               typename MF<R>::C *__restrict__ x,
                                               typename MF<R>::C *__restrict__ t, int nrhs, int nchunks, int maxk) {
    using C = typename MF<R>::C;
    const int lane = threadIdx.x & 63;
    int64_t wg;
    int chunk;
    xcd_order((ntiles + 3) / 4, nchunks, wg, chunk);
    const int64_t wave = wg * 4 + (threadIdx.x >> 6);
    if (wave >= ntiles) return;  // wave-uniform
    const int v = tiles[2 * wave], row0 = tiles[2 * wave + 1];
    const int nr = (int)desc[4 * v], ns = (int)desc[4 * v + 1];
    const int32_t *ir = idx + desc[4 * v + 2];
    const int32_t *is = ir + nr;
    const int64_t mo = desc[4 * v + 3];
    // factor block of the phase, column-major m x K with leading dimension ld
    constexpr bool SUB = (PH == 0 || PH == 2 || PH == 3 || PH == 5);
    const int m = (PH == 2 || PH == 5) ? ns : nr;
    const int K = (PH == 0 || PH == 3) ? ns : nr;
    const int ld = (PH == 2 || PH == 5) ? ns : nr;
    const int64_t off = (PH == 0 || PH == 5) ? 0 : ((PH == 1 || PH == 4) ? (int64_t)ns * nr : (int64_t)ns * nr + (int64_t)nr * nr);
    const C *S = ((PH == 0 || PH == 3 || PH == 4) ? matH : mat) + mo + off;
    const int32_t *kin = (PH == 0 || PH == 3) ? is : ir;      // input rows (global, then LDS)
    const C *src = (PH == 2 || PH == 4) ? t : x;              // input vector
    const int32_t *oout = (PH == 2 || PH == 5) ? is : ir;     // output rows
    C *dst = (PH == 1 || PH == 3) ? t : x;                    // output vector
    const C *yin = (PH == 3) ? x : dst;                       // subtracted-from vector
    const int kbeg = (PH == 4) ? row0 : 0;
    const int kend = (PH == 1) ? min(K, row0 + 16 * MT) : K;
    const int n0 = chunk * (16 * NT);
    const int ncols = nrhs - n0;
    const int li = lane & 15, lk = lane >> 4;
    typename std::conditional<M3, Acc3<R, MT, NT>, Acc<R, MT, NT>>::type acc;
    acc.zero();
    if (kbeg < kend && m > 0) {  // wave-uniform
        // this wave's gathered row indices kin[0..kend) in LDS (wave-local: LDS
        // operations of one wave complete in order, no barrier needed)
        extern __shared__ int32_t sidx[];
        int32_t *lidx = sidx + (threadIdx.x >> 6) * maxk;
        for (int i0 = 0; i0 < kend; i0 += 512) {  // eight loads in flight per lane
            int32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = kin[min(i0 + 64 * u + lane, kend - 1)];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (i0 + 64 * u + lane < kend) lidx[i0 + 64 * u + lane] = v[u];
        }
        kin = lidx;
        int colc[NT], rowc[MT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) colc[nt] = min(nt * 16 + li, ncols - 1);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) rowc[mt] = min(row0 + mt * 16 + li, m - 1);
        const C *xb = src + n0;
        GWalk<R, MT, NT> w;
        w.k = kbeg + lk;
        w.ap = S + (int64_t)w.k * ld;
        w.gnext = kin[min(w.k, kend - 1)];
        constexpr int HG_PF = HgPf<R>::value;
        Frag<R, MT, NT> f[HG_PF];
#pragma unroll
        for (int j = 0; j + 1 < HG_PF; ++j) gfrag_load(f[j], w, kend, xb, nrhs, kin, ld, colc, rowc);
        for (int k0 = kbeg; k0 < kend; k0 += 4 * HG_PF) {
#pragma unroll
            for (int j = 0; j < HG_PF; ++j) {
                if (k0 + 4 * j >= kend) break;  // wave-uniform
                gfrag_load(f[(j + HG_PF - 1) % HG_PF], w, kend, xb, nrhs, kin, ld, colc, rowc);
                acc.mma(f[j]);
            }
        }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) {
            const int row = row0 + mt * 16 + MF<R>::drow(lk, vv);
            if (row >= m) continue;
            const int64_t orow = (int64_t)oout[row] * nrhs;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int col = n0 + nt * 16 + li;
                if (col >= nrhs) continue;
                C a = acc.get(mt, nt, vv);
                if (SUB) {
                    const C b = yin[orow + col];
                    a = C{b.x - a.x, b.y - a.y};
                }
                dst[orow + col] = a;
            }
        }
}

// x_r = t_r for every node of a step (end of the upward pass): one workgroup per
// tile of 16 redundant rows, all right-hand sides.
template <class C>
__global__ void __launch_bounds__(256) k_hcopy(const int64_t *__restrict__ desc, const int32_t *__restrict__ idx,
                                               const int32_t *__restrict__ tiles, const C *__restrict__ t,
                                               C *__restrict__ x, int nrhs) {
    const int64_t tile = blockIdx.x;
    const int v = tiles[2 * tile], row0 = tiles[2 * tile + 1];
    const int nr = (int)desc[4 * v];
    const int32_t *ir = idx + desc[4 * v + 2];
    const int rows = min(16, nr - row0);
    for (int e = threadIdx.x; e < rows * nrhs; e += blockDim.x) {
        const int64_t g = (int64_t)ir[row0 + e / nrhs] * nrhs + e % nrhs;
        x[g] = t[g];
    }
}

template <class R, int MT, int NT, bool M3>
static void hgemm_phase(int ph, const HifStepDev &h, const int32_t *tiles, int64_t ntiles, void *x, void *t,
                        int nrhs, hipStream_t st) {
    using C = typename MF<R>::C;
    if (ntiles == 0) return;
    const int nch = (nrhs + 16 * NT - 1) / (16 * NT);
    const dim3 g(xcd_grid((ntiles + 3) / 4, nch));
    const C *mat = (const C *)h.mat, *matH = (const C *)h.matH;
    const int maxk = std::max(1, std::max(h.max_nr, h.max_ns));
    const size_t lds = (size_t)4 * maxk * sizeof(int32_t);
    if ((int64_t)lds > hif_lds_budget()) throw std::runtime_error("hif step: index lists exceed LDS");
    static std::once_flag attr_once[6];  // plans may be used from several host threads
    if (lds > 65536) {
        std::call_once(attr_once[ph], [ph] {
            const void *fn[6] = {(const void *)k_hgemm<R, 0, MT, NT, M3>, (const void *)k_hgemm<R, 1, MT, NT, M3>,
                                 (const void *)k_hgemm<R, 2, MT, NT, M3>, (const void *)k_hgemm<R, 3, MT, NT, M3>,
                                 (const void *)k_hgemm<R, 4, MT, NT, M3>, (const void *)k_hgemm<R, 5, MT, NT, M3>};
            (void)hipFuncSetAttribute(fn[ph], hipFuncAttributeMaxDynamicSharedMemorySize, hif_lds_budget());
        });
    }
#define HG(P) hipLaunchKernelGGL((k_hgemm<R, P, MT, NT, M3>), g, dim3(256), lds, st, h.desc, h.idx, tiles, ntiles, mat, \
                                 matH, (C *)x, (C *)t, nrhs, nch, maxk)
    switch (ph) {
        case 0: HG(0); break;
        case 1: HG(1); break;
        case 2: HG(2); break;
        case 3: HG(3); break;
        case 4: HG(4); break;
        default: HG(5); break;
    }
#undef HG
}

// The register tilings of the gathered GEMMs: 16*MT rows x 16*NT columns per wave,
// four or three (m3) real products per complex k-step.
template <class R>
static void hgemm_phase_tile(int mt, int nt, bool m3, int ph, const HifStepDev &h, const int32_t *tiles,
                             int64_t ntiles, void *x, void *t, int nrhs, hipStream_t st) {
    if (m3) {
        if (mt == 2) hgemm_phase<R, 2, 2, true>(ph, h, tiles, ntiles, x, t, nrhs, st);
        else if (nt == 2) hgemm_phase<R, 1, 2, true>(ph, h, tiles, ntiles, x, t, nrhs, st);
        else hgemm_phase<R, 1, 4, true>(ph, h, tiles, ntiles, x, t, nrhs, st);
    } else if (mt == 4) {
        if (nt == 1) hgemm_phase<R, 4, 1, false>(ph, h, tiles, ntiles, x, t, nrhs, st);
        else hgemm_phase<R, 4, 2, false>(ph, h, tiles, ntiles, x, t, nrhs, st);
    } else if (mt == 2) {
        hgemm_phase<R, 2, 2, false>(ph, h, tiles, ntiles, x, t, nrhs, st);
    } else {
        if (nt == 1) hgemm_phase<R, 1, 1, false>(ph, h, tiles, ntiles, x, t, nrhs, st);
        else if (nt == 2) hgemm_phase<R, 1, 2, false>(ph, h, tiles, ntiles, x, t, nrhs, st);
        else hgemm_phase<R, 1, 4, false>(ph, h, tiles, ntiles, x, t, nrhs, st);
    }
}

void launch_hif_gemm_step(const HifStepDev &h, bool dbl, bool up, void *x, void *t, int nrhs, int cols,
                          hipStream_t st, int mt, bool m3) {
    if (h.n_nodes == 0) return;
    const int nt = cols <= 16 ? 1 : (cols <= 32 ? 2 : 4);
    if (mt != 1 && mt != 2 && mt != 4) throw std::runtime_error("hif step: 1, 2 or 4 row tiles per wave");
    if ((mt == 4 && nt > 2) || (mt == 2 && nt != 2) || (m3 && (mt == 4 || nt == 1)))
        throw std::runtime_error("hif step: tiling not built");
    const int p0 = up ? 0 : 3;
    for (int k = 0; k < 3; ++k) {
        const int ph = p0 + k;
        // phases 2 and 5 produce the skeleton rows (ns), the others the redundant rows (nr)
        const bool srows = (ph == 2 || ph == 5);
        const int32_t *tiles = mt == 4 ? (srows ? h.tiles_s4 : h.tiles_r4)
                             : mt == 2 ? (srows ? h.tiles_s2 : h.tiles_r2)
                                       : (srows ? h.tiles_s : h.tiles_r);
        const int64_t ntl = mt == 4 ? (srows ? h.n_tiles_s4 : h.n_tiles_r4)
                          : mt == 2 ? (srows ? h.n_tiles_s2 : h.n_tiles_r2)
                                    : (srows ? h.n_tiles_s : h.n_tiles_r);
        if (ntl > 0 && !tiles) throw std::runtime_error("hif step: tile list missing");
        if (dbl) hgemm_phase_tile<double>(mt, nt, m3, ph, h, tiles, ntl, x, t, nrhs, st);
        else hgemm_phase_tile<float>(mt, nt, m3, ph, h, tiles, ntl, x, t, nrhs, st);
        check_launch("hif step (matrix cores)");
    }
    if (up && h.n_tiles_r > 0) {
        const dim3 g((unsigned)h.n_tiles_r);
        if (dbl) hipLaunchKernelGGL(k_hcopy<double2>, g, dim3(256), 0, st, h.desc, h.idx, h.tiles_r, (const double2 *)t, (double2 *)x, nrhs);
        else hipLaunchKernelGGL(k_hcopy<float2>, g, dim3(256), 0, st, h.desc, h.idx, h.tiles_r, (const float2 *)t, (float2 *)x, nrhs);
        check_launch("hif copy");
    }
}

// ------------------------------------------------------------------ skeletonization, small batches
// Fewer than 16 right-hand sides: the six phases above as gathered matrix-vector
// products, bound by the factor bytes.  A workgroup takes 64 output rows of one node
// (one row per lane; the 64-row tile lists) and NB right-hand sides; its W waves
// split the phase's k range and stream their share of the factor's columns with
// coalesced 64-row loads (every phase reads a column-major factor), U k-steps of
// loads issued before their products.  The gathered input entry of a k-step is the
// same for all lanes of a wave (its row index a wave-uniform load, the entry one
// broadcast load); the W partial sums meet in LDS.  Phases with few tiles take 16
// waves per workgroup, so that the device holds enough loads in flight; phases whose
// tiles have long k ranges (nodes of thousands of DOFs: one workgroup would stream
// megabytes alone) also split each tile's k range over gridDim.z workgroups, which
// write their partial sums to `part` for k_hgemv_sum to add in a fixed order.  The
// launch of phase 2 also carries the end of the up sweep, x_r = t_r, in extra
// workgroups over the 64-row tiles of the redundant rows (phase 2 reads t_r and
// writes x_s only).
template <class T, int PH, int NB, int W>
__global__ void __launch_bounds__(64 * W) k_hgemv(const int64_t *__restrict__ desc, const int32_t *__restrict__ idx,
                                                  const int32_t *__restrict__ tiles, int64_t ntiles,
                                                  const int32_t *__restrict__ ctiles, const T *__restrict__ mat,
                                                  const T *__restrict__ matH, T *__restrict__ x, T *__restrict__ t,
                                                  int nrhs, T *__restrict__ part) {
    constexpr int U = NB <= 2 ? 8 : (NB == 4 ? 4 : 2);
    __shared__ T red[(W - 1) * 64 * NB];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c0 = blockIdx.y * NB;
    if (PH == 2 && (int64_t)blockIdx.x >= ntiles) {  // workgroup-uniform: x_r = t_r
        if (blockIdx.z != 0) return;
        const int64_t ct = blockIdx.x - ntiles;
        const int v = ctiles[2 * ct], row0 = ctiles[2 * ct + 1];
        const int nr = (int)desc[4 * v];
        const int32_t *ir = idx + desc[4 * v + 2];
        for (int e = threadIdx.x; e < 64 * NB; e += 64 * W) {
            const int row = row0 + e / NB, col = c0 + e % NB;
            if (row < nr && col < nrhs) {
                const int64_t g = (int64_t)ir[row] * nrhs + col;
                x[g] = t[g];
            }
        }
        return;
    }
    const int64_t tile = blockIdx.x;
    const int v = tiles[2 * tile], row0 = tiles[2 * tile + 1];
    const int nr = (int)desc[4 * v], ns = (int)desc[4 * v + 1];
    const int32_t *ir = idx + desc[4 * v + 2];
    const int32_t *is = ir + nr;
    const int64_t mo = desc[4 * v + 3];
    constexpr bool SUB = (PH == 0 || PH == 2 || PH == 3 || PH == 5);
    const int m = (PH == 2 || PH == 5) ? ns : nr;
    const int K = (PH == 0 || PH == 3) ? ns : nr;
    const int ld = m;
    const int64_t off = (PH == 0 || PH == 5) ? 0 : ((PH == 1 || PH == 4) ? (int64_t)ns * nr : (int64_t)ns * nr + (int64_t)nr * nr);
    const T *S = ((PH == 0 || PH == 3 || PH == 4) ? matH : mat) + mo + off;
    const int32_t *kin = (PH == 0 || PH == 3) ? is : ir;
    const T *src = (PH == 2 || PH == 4) ? t : x;
    const int32_t *oout = (PH == 2 || PH == 5) ? is : ir;
    T *dst = (PH == 1 || PH == 3) ? t : x;
    const T *yin = (PH == 3) ? x : dst;
    // L^-1 is lower triangular: phase 1 stops at the tile's last row, phase 4 starts at its first
    const int kbeg = (PH == 4) ? row0 : 0;
    const int kend = (PH == 1) ? min(K, row0 + 64) : K;
    const int span = max(kend - kbeg, 0);
    const int za = kbeg + (int)((int64_t)span * blockIdx.z / gridDim.z);
    const int zspan = kbeg + (int)((int64_t)span * (blockIdx.z + 1) / gridDim.z) - za;
    const int kb = za + (zspan * w) / W, ke = za + (zspan * (w + 1)) / W;
    const int row = row0 + lane;
    const T *Sp = S + min(row, m - 1);
    int cj[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) cj[j] = min(c0 + j, nrhs - 1);
    T acc[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j] = cz(T());
    int k = kb;
    for (; k + U <= ke; k += U) {
        T av[U], xv[U][NB];
#pragma unroll
        for (int u = 0; u < U; ++u) av[u] = Sp[(int64_t)(k + u) * ld];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const T *xr = src + (int64_t)kin[k + u] * nrhs;
#pragma unroll
            for (int j = 0; j < NB; ++j) xv[u][j] = xr[cj[j]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < NB; ++j) acc[j] = cfma(acc[j], av[u], xv[u][j]);
    }
    for (; k < ke; ++k) {
        const T av = Sp[(int64_t)k * ld];
        const T *xr = src + (int64_t)kin[k] * nrhs;
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[j] = cfma(acc[j], av, xr[cj[j]]);
    }
    if (w > 0) {
#pragma unroll
        for (int j = 0; j < NB; ++j) red[((w - 1) * 64 + lane) * NB + j] = acc[j];
    }
    __syncthreads();
    if (w == 0 && gridDim.z > 1) {  // partial sum of this k slice
        T *pp = part + (((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * ntiles + tile) * 64 * NB;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            T s = acc[j];
#pragma unroll
            for (int q = 0; q < W - 1; ++q) {
                const T r = red[(q * 64 + lane) * NB + j];
                s.x += r.x;
                s.y += r.y;
            }
            pp[lane * NB + j] = s;
        }
    } else if (w == 0 && row < m) {
        const int64_t orow = (int64_t)oout[row] * nrhs;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            T s = acc[j];
#pragma unroll
            for (int q = 0; q < W - 1; ++q) {
                const T r = red[(q * 64 + lane) * NB + j];
                s.x += r.x;
                s.y += r.y;
            }
            if (c0 + j >= nrhs) continue;
            if (SUB) {
                const T b = yin[orow + c0 + j];
                s = T{b.x - s.x, b.y - s.y};
            }
            dst[orow + c0 + j] = s;
        }
    }
}

// Output of a split phase: the gridDim.z partial sums of each tile row, added in
// slice order, then stored (or subtracted) as k_hgemv stores its sums.
template <class T, int PH, int NB>
__global__ void __launch_bounds__(64) k_hgemv_sum(const int64_t *__restrict__ desc, const int32_t *__restrict__ idx,
                                                  const int32_t *__restrict__ tiles, int64_t ntiles, int ks,
                                                  const T *__restrict__ part, T *__restrict__ x, T *__restrict__ t,
                                                  int nrhs) {
    const int64_t tile = blockIdx.x;
    const int lane = threadIdx.x;
    const int v = tiles[2 * tile], row0 = tiles[2 * tile + 1];
    const int nr = (int)desc[4 * v], ns = (int)desc[4 * v + 1];
    const int32_t *ir = idx + desc[4 * v + 2];
    const int32_t *is = ir + nr;
    constexpr bool SUB = (PH == 0 || PH == 2 || PH == 3 || PH == 5);
    const int m = (PH == 2 || PH == 5) ? ns : nr;
    const int32_t *oout = (PH == 2 || PH == 5) ? is : ir;
    T *dst = (PH == 1 || PH == 3) ? t : x;
    const T *yin = (PH == 3) ? x : dst;
    const int row = row0 + lane;
    if (row >= m) return;
    const int c0 = blockIdx.y * NB;
    const int64_t orow = (int64_t)oout[row] * nrhs;
    const int64_t zs = (int64_t)gridDim.y * ntiles * 64 * NB;
    const T *pp = part + ((int64_t)blockIdx.y * ntiles + tile) * 64 * NB + lane * NB;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (c0 + j >= nrhs) continue;
        T r[16];  // ks <= 16: every load issued before the first sum
#pragma unroll
        for (int z = 0; z < 16; ++z)
            if (z < ks) r[z] = pp[z * zs + j];
        T s = r[0];
#pragma unroll
        for (int z = 1; z < 16; ++z)
            if (z < ks) {
                s.x += r[z].x;
                s.y += r[z].y;
            }
        if (SUB) {
            const T b = yin[orow + c0 + j];
            s = T{b.x - s.x, b.y - s.y};
        }
        dst[orow + c0 + j] = s;
    }
}

template <class T, int NB, int W>
static void hgemv_phase_w(int ph, const HifStepDev &h, const int32_t *tiles, int64_t ntiles, int64_t ncopy,
                          int ks, void *part, void *x, void *t, int nrhs, hipStream_t st) {
    const dim3 g((unsigned)(ntiles + ncopy), (unsigned)((nrhs + NB - 1) / NB), (unsigned)ks);
    const dim3 gs((unsigned)ntiles, g.y);
#define HV(P) hipLaunchKernelGGL((k_hgemv<T, P, NB, W>), g, dim3(64 * W), 0, st, h.desc, h.idx, tiles, ntiles, \
                                 h.tiles_r4, (const T *)h.mat, (const T *)h.matH, (T *)x, (T *)t, nrhs, (T *)part)
#define HS(P) hipLaunchKernelGGL((k_hgemv_sum<T, P, NB>), gs, dim3(64), 0, st, h.desc, h.idx, tiles, ntiles, ks, \
                                 (const T *)part, (T *)x, (T *)t, nrhs)
    switch (ph) {
        case 0: HV(0); break;
        case 1: HV(1); break;
        case 2: HV(2); break;
        case 3: HV(3); break;
        case 4: HV(4); break;
        default: HV(5); break;
    }
    if (ks > 1 && ntiles > 0) {
        switch (ph) {
            case 0: HS(0); break;
            case 1: HS(1); break;
            case 2: HS(2); break;
            case 3: HS(3); break;
            case 4: HS(4); break;
            default: HS(5); break;
        }
    }
#undef HS
#undef HV
}

// Launch shape of a phase: with fewer tiles than compute units and long k ranges
// (K >= 512), the k range of each tile is split into ks slices (at most K / 256, 16,
// about 1024 workgroups in all, and as many as `part` holds) on workgroups of 4
// waves; else, with fewer tiles than four per compute unit, whole tiles on
// workgroups of 16 waves (NB <= 2, so that the LDS of the partial sums stays small);
// otherwise 4 waves.
template <class T, int NB>
static void hgemv_phase(int ph, const HifStepDev &h, const int32_t *tiles, int64_t ntiles, int64_t ncopy,
                        void *part, size_t part_bytes, void *x, void *t, int nrhs, hipStream_t st) {
    if (ntiles + ncopy == 0) return;
    if (ntiles + ncopy >= ((int64_t)1 << 31)) throw std::runtime_error("hif step: tile count exceeds the grid limit");
    const int K = (ph == 0 || ph == 3) ? h.max_ns : h.max_nr;
    int ks = 1;
    if (ntiles > 0 && ntiles < 256 && part) {
        const int64_t slice = (int64_t)((nrhs + NB - 1) / NB) * ntiles * 64 * NB * sizeof(T);
        ks = (int)std::min<int64_t>({16, K / 256, (1024 + ntiles - 1) / ntiles,
                                     (int64_t)(part_bytes / std::max<int64_t>(1, slice))});
        ks = std::max(ks, 1);
    }
    if (ks > 1) hgemv_phase_w<T, NB, 4>(ph, h, tiles, ntiles, ncopy, ks, part, x, t, nrhs, st);
    else if (NB <= 2 && ntiles < 1024) hgemv_phase_w<T, NB, (NB <= 2 ? 16 : 4)>(ph, h, tiles, ntiles, ncopy, 1, part, x, t, nrhs, st);
    else hgemv_phase_w<T, NB, 4>(ph, h, tiles, ntiles, ncopy, 1, part, x, t, nrhs, st);
}

template <class T>
static void hgemv_phase_nb(int ph, const HifStepDev &h, const int32_t *tiles, int64_t ntiles, int64_t ncopy,
                           void *part, size_t part_bytes, void *x, void *t, int nrhs, hipStream_t st) {
    if (nrhs <= 1) hgemv_phase<T, 1>(ph, h, tiles, ntiles, ncopy, part, part_bytes, x, t, nrhs, st);
    else if (nrhs <= 2) hgemv_phase<T, 2>(ph, h, tiles, ntiles, ncopy, part, part_bytes, x, t, nrhs, st);
    else if (nrhs <= 4) hgemv_phase<T, 4>(ph, h, tiles, ntiles, ncopy, part, part_bytes, x, t, nrhs, st);
    else hgemv_phase<T, 8>(ph, h, tiles, ntiles, ncopy, part, part_bytes, x, t, nrhs, st);
}

void launch_hif_gemv_step(const HifStepDev &h, bool dbl, bool up, void *x, void *t, int nrhs, void *part,
                          size_t part_bytes, hipStream_t st) {
    if (h.n_nodes == 0) return;
    if (h.n_tiles_r4 > 0 && !h.tiles_r4) throw std::runtime_error("hif step: tile list missing");
    const int p0 = up ? 0 : 3;
    for (int k = 0; k < 3; ++k) {
        const int ph = p0 + k;
        const bool srows = (ph == 2 || ph == 5);
        const int32_t *tiles = srows ? h.tiles_s4 : h.tiles_r4;
        const int64_t ntl = srows ? h.n_tiles_s4 : h.n_tiles_r4;
        const int64_t ncopy = (ph == 2) ? h.n_tiles_r4 : 0;  // x_r = t_r with phase 2
        if (ntl > 0 && !tiles) throw std::runtime_error("hif step: tile list missing");
        if (dbl) hgemv_phase_nb<double2>(ph, h, tiles, ntl, ncopy, part, part_bytes, x, t, nrhs, st);
        else hgemv_phase_nb<float2>(ph, h, tiles, ntl, ncopy, part, part_bytes, x, t, nrhs, st);
        check_launch("hif step (small batch)");
    }
}

bool hif_step_fits_lds(const HifStepDev &h, bool dbl) {
    const int elt = dbl ? 16 : 8;
    const int64_t budget = hif_lds_budget();
    return (int64_t)h.max_mat * elt + (int64_t)std::max(1, h.max_vec) * elt <= budget;
}

// ------------------------------------------------------------------ fused skeletonization step
// Nodes with nr, ns <= 64, one workgroup per (node, 64 right-hand sides): the
// node's entries of x are staged in LDS once, the step's three products run on
// matrix cores (factor from global memory as the A operand, the staged vectors as
// B), and the results are written back once.
//   up:   x_r -= T^* x_s;  x_r <- Linv x_r;   x_s -= M x_r
//   down: x_r -= M^* x_s;  x_r <- Linv^* x_r; x_s -= T x_r
// The two products with nr output rows split their rows over the waves (wave w:
// rows 16w..16w+15, all 64 columns), so each factor entry is loaded once per
// workgroup, with a barrier where a wave reads rows another wave wrote.  The
// product with ns output rows splits its columns (wave w: columns 16w..16w+15).
// k-steps in which a triangular factor's tile is zero are skipped.  Staged rows
// past nr (ns) are zero, so clamped factor entries of k beyond the product's K
// (finite duplicates) add nothing.
constexpr int HF_PF = 4;    // k-steps of loads in flight (register ring)

template <class R> struct HfFragR {   // row split: one factor entry, four vector entries
    typename MF<R>::C a, b[4];
};
template <class R> struct HfFragC {   // column split: four factor entries, one vector entry
    typename MF<R>::C a[4], b;
};

template <class R>
__device__ __forceinline__ void cmma(typename MF<R>::V4 &re, typename MF<R>::V4 &im, typename MF<R>::C a,
                                     typename MF<R>::C b) {
    re = MF<R>::mma(a.x, b.x, re);
    im = MF<R>::mma(a.x, b.y, im);
    re = MF<R>::mma(-a.y, b.y, re);
    im = MF<R>::mma(a.y, b.x, im);
}

// Row split: acc[nt] = A(rows 16mt.., :) B(:, 16nt..) for the NTW column tiles of
// the workgroup (B has row stride ld).
template <class R, int NTW>
__device__ __forceinline__ void hf_rows(typename MF<R>::V4 (&re)[4], typename MF<R>::V4 (&im)[4],
                                        const typename MF<R>::C *__restrict__ A, int lda, int rows, int K, int tri,
                                        const typename MF<R>::C *B, int ld, int mt) {
    using C = typename MF<R>::C;
    using V4 = typename MF<R>::V4;
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) { re[nt] = V4{0, 0, 0, 0}; im[nt] = V4{0, 0, 0, 0}; }
    int sb = 0, se = (K + 3) >> 2;
    if (tri == 1) se = min(se, (16 * mt + 15) / 4 + 1);   // lower: k <= last row of the tile
    if (tri == 2) sb = (16 * mt) / 4;                      // upper: k >= first row of the tile
    if (16 * mt >= rows || sb >= se) return;               // wave-uniform
    const C *arow = A + min(16 * mt + li, rows - 1);
    // unconditional loads (a clamped k-step past the end loads valid, unused data):
    // a load under a branch would make the compiler wait for every load in flight
    auto load = [&](HfFragR<R> &f, int s) {
        s = min(s, se - 1);
        const int k = 4 * s + lk;
        f.a = arow[(int64_t)min(k, K - 1) * lda];
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt) f.b[nt] = B[k * ld + 16 * nt + li];
    };
    HfFragR<R> f[HF_PF];
#pragma unroll
    for (int j = 0; j + 1 < HF_PF; ++j) load(f[j], sb + j);
    for (int s0 = sb; s0 < se; s0 += HF_PF) {
#pragma unroll
        for (int j = 0; j < HF_PF; ++j) {
            if (s0 + j >= se) break;  // wave-uniform
            load(f[(j + HF_PF - 1) % HF_PF], s0 + j + HF_PF - 1);
#pragma unroll
            for (int nt = 0; nt < NTW; ++nt) cmma<R>(re[nt], im[nt], f[j].a, f[j].b[nt]);
        }
    }
}

// Column split: acc[mt] = A(rows 16mt.., :) B(:, col0..col0+15) for all row tiles.
template <class R>
__device__ __forceinline__ void hf_cols(typename MF<R>::V4 (&re)[4], typename MF<R>::V4 (&im)[4],
                                        const typename MF<R>::C *__restrict__ A, int lda, int rows, int K,
                                        const typename MF<R>::C *B, int ld, int col0) {
    using C = typename MF<R>::C;
    using V4 = typename MF<R>::V4;
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) { re[mt] = V4{0, 0, 0, 0}; im[mt] = V4{0, 0, 0, 0}; }
    const int nks = (K + 3) >> 2;
    const int mtl = (rows + 15) >> 4;
    if (nks == 0) return;  // wave-uniform
    auto load = [&](HfFragC<R> &f, int s) {   // unconditional, clamped (as in hf_rows)
        s = min(s, nks - 1);
        const int k = 4 * s + lk;
        const C *acol = A + (int64_t)min(k, K - 1) * lda;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) f.a[mt] = acol[min(16 * mt + li, rows - 1)];
        f.b = B[k * ld + col0 + li];
    };
    HfFragC<R> f[HF_PF];
#pragma unroll
    for (int j = 0; j + 1 < HF_PF; ++j) load(f[j], j);
    for (int s0 = 0; s0 < nks; s0 += HF_PF) {
#pragma unroll
        for (int j = 0; j < HF_PF; ++j) {
            if (s0 + j >= nks) break;  // wave-uniform
            load(f[(j + HF_PF - 1) % HF_PF], s0 + j + HF_PF - 1);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
                if (mt < mtl) cmma<R>(re[mt], im[mt], f[j].a[mt], f[j].b);
        }
    }
}

// Row-split result into Y (SET) or subtracted from it: rows 16mt.., columns 16nt + li.
template <class R, bool SET>
__device__ __forceinline__ void hf_store_rows(const typename MF<R>::V4 (&re)[4], const typename MF<R>::V4 (&im)[4],
                                              typename MF<R>::C *Y, int ld, int rows, int mt, int ntl) {
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    if (16 * mt >= rows) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int row = 16 * mt + MF<R>::drow(lk, v);
        if (row >= rows) continue;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            if (nt >= ntl) continue;
            typename MF<R>::C &y = Y[row * ld + 16 * nt + li];
            if (SET) y = typename MF<R>::C{re[nt][v], im[nt][v]};
            else y = typename MF<R>::C{y.x - re[nt][v], y.y - im[nt][v]};
        }
    }
}

// Column-split result subtracted from Y: rows 16mt + .., columns col0 + li.
template <class R>
__device__ __forceinline__ void hf_sub_cols(const typename MF<R>::V4 (&re)[4], const typename MF<R>::V4 (&im)[4],
                                            typename MF<R>::C *Y, int ld, int rows, int col0) {
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        if (16 * mt >= rows) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * mt + MF<R>::drow(lk, v);
            if (row >= rows) continue;
            typename MF<R>::C &y = Y[row * ld + col0 + li];
            y = typename MF<R>::C{y.x - re[mt][v], y.y - im[mt][v]};
        }
    }
}

template <class R, bool UP, int NTW>
__device__ __forceinline__ void hif_fused_node(const int64_t *__restrict__ desc, const int32_t *__restrict__ idx,
                                               const typename MF<R>::C *__restrict__ mat,
                                               const typename MF<R>::C *__restrict__ matH,
                                               typename MF<R>::C *__restrict__ x, int nrhs, int rows_r, int rows_s,
                                               int64_t v, int ychunk) {
    using C = typename MF<R>::C;
    using V4 = typename MF<R>::V4;
    constexpr int CW = 16 * NTW, LD = CW + 4;   // columns per workgroup, LDS row stride
    extern __shared__ char smem_raw[];
    C *Xr = reinterpret_cast<C *>(smem_raw);   // rows_r x LD
    C *Xs = Xr + (int64_t)rows_r * LD;         // rows_s x LD
    const int nr = (int)desc[4 * v], ns = (int)desc[4 * v + 1];
    const int32_t *ir = idx + desc[4 * v + 2];
    const int32_t *is = ir + nr;
    const int64_t mo = desc[4 * v + 3];
    const C *Tm = mat + mo, *Li = Tm + (int64_t)ns * nr, *Mm = Li + (int64_t)nr * nr;
    const C *TH = matH + mo, *LH = TH + (int64_t)ns * nr, *MH = LH + (int64_t)nr * nr;
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int w = threadIdx.x >> 6, col0 = 16 * w;
    const int b0 = ychunk * CW;
    const int bc = min(CW, nrhs - b0);
    const int ntl = (bc + 15) >> 4;   // column tiles holding columns
    // the node's row indices (x_r rows, then x_s rows) in LDS, one load per thread
    int32_t *gidx = reinterpret_cast<int32_t *>(Xr + (int64_t)(rows_r + rows_s) * LD);
    const int32_t g0 = (nr > 0) ? ir[0] : ((ns > 0) ? is[0] : 0);
    for (int i = threadIdx.x; i < rows_r + rows_s; i += blockDim.x) {
        const int ii = (i < rows_r) ? i : i - rows_r;
        const int cnt = (i < rows_r) ? nr : ns;
        gidx[i] = (ii < cnt) ? ((i < rows_r) ? ir[ii] : is[ii]) : -1;
    }
    __syncthreads();
    // stage: each wave its 16 columns, four rows per instruction; all loads of the
    // wave are issued (from valid rows and columns) before the first store, and
    // entries outside the node or the batch are then replaced by zero
    const bool cv = col0 + li < bc;
    const int64_t cc = b0 + min(col0 + li, bc - 1);
    for (int i0 = 0; w < NTW && i0 < rows_r + rows_s; i0 += 64) {
        C t[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int i = min(i0 + 4 * u + lk, rows_r + rows_s - 1);
            const int32_t g = gidx[i];
            t[u] = x[(int64_t)(g >= 0 ? g : g0) * nrhs + cc];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int i = i0 + 4 * u + lk;
            if (i < rows_r + rows_s) Xr[i * LD + col0 + li] = (cv && gidx[i] >= 0) ? t[u] : C{0, 0};
        }
    }
    __syncthreads();
    V4 re[4], im[4];
    // first product: x_r -= (T^* or M^*) x_s, row split
    if (ns > 0) {
        hf_rows<R, NTW>(re, im, UP ? TH : MH, nr, nr, ns, 0, Xs, LD, w);
        hf_store_rows<R, false>(re, im, Xr, LD, nr, w, ntl);
    }
    __syncthreads();
    // x_r <- (Linv or Linv^*) x_r, row split; every wave reads all rows first
    hf_rows<R, NTW>(re, im, UP ? Li : LH, nr, nr, nr, UP ? 1 : 2, Xr, LD, w);
    __syncthreads();
    hf_store_rows<R, true>(re, im, Xr, LD, nr, w, ntl);
    __syncthreads();
    // x_s -= (M or T) x_r, column split
    if (ns > 0 && col0 < bc) {
        hf_cols<R>(re, im, UP ? Mm : Tm, ns, ns, nr, Xr, LD, col0);
        hf_sub_cols<R>(re, im, Xs, LD, ns, col0);
    }
    // write back this wave's columns (x_s was last written by this wave, x_r before
    // the last barrier)
    if (cv) {
        for (int i = lk; i < nr; i += 4) x[(int64_t)gidx[i] * nrhs + cc] = Xr[i * LD + col0 + li];
        for (int i = lk; i < ns; i += 4) x[(int64_t)gidx[rows_r + i] * nrhs + cc] = Xs[i * LD + col0 + li];
    }
}

template <class R, bool UP, int NTW>
__global__ void __launch_bounds__(256) k_hif_fused(const int64_t *__restrict__ desc, const int32_t *__restrict__ idx,
                                                   const typename MF<R>::C *__restrict__ mat,
                                                   const typename MF<R>::C *__restrict__ matH,
                                                   typename MF<R>::C *__restrict__ x, int nrhs, int rows_r,
                                                   int rows_s, int64_t n_nodes, int nch) {
    int64_t v;
    int c;
    xcd_order(n_nodes, nch, v, c);   // the column chunks of one node share its factors in one L2
    if (v >= n_nodes) return;
    hif_fused_node<R, UP, NTW>(desc, idx, mat, matH, x, nrhs, rows_r, rows_s, v, c);
}

bool hif_fused_fits(const HifStepDev &h) { return h.max_nr <= 64 && h.max_ns <= 64; }

template <class R, bool UP, int NTW>
static void hif_fused_go(const HifStepDev &h, int rr, int rs, void *x, int nrhs, hipStream_t st) {
    using C = typename MF<R>::C;
    constexpr int CW = 16 * NTW, LD = CW + 4;
    const size_t lds = (size_t)(rr + rs) * LD * sizeof(C) + (size_t)(rr + rs) * sizeof(int32_t);
    static std::once_flag attr_once;  // plans may be used from several host threads
    std::call_once(attr_once, [] {
        (void)hipFuncSetAttribute((const void *)k_hif_fused<R, UP, NTW>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  hif_lds_budget());
    });
    if ((int64_t)lds > hif_lds_budget()) throw std::runtime_error("fused skeletonization step exceeds LDS");
    const int nch = (nrhs + CW - 1) / CW;
    hipLaunchKernelGGL((k_hif_fused<R, UP, NTW>), dim3(xcd_grid(h.n_nodes, nch)), dim3(256), lds, st, h.desc,
                       h.idx, (const C *)h.mat, (const C *)h.matH, (C *)x, nrhs, rr, rs, h.n_nodes, nch);
}

void launch_hif_fused_step(const HifStepDev &h, bool dbl, bool up, void *x, int nrhs, hipStream_t st, int cols) {
    if (h.n_nodes == 0) return;
    if (!hif_fused_fits(h)) throw std::runtime_error("fused skeletonization step needs nr, ns <= 64");
    // staged rows: whole 16-row tiles (the k loops read up to the next multiple of 4)
    const int rr = std::max(16, (h.max_nr + 15) / 16 * 16), rs = std::max(16, (h.max_ns + 15) / 16 * 16);
    const bool w64 = cols > 32;
    if (dbl) {
        if (w64) { if (up) hif_fused_go<double, true, 4>(h, rr, rs, x, nrhs, st); else hif_fused_go<double, false, 4>(h, rr, rs, x, nrhs, st); }
        else { if (up) hif_fused_go<double, true, 2>(h, rr, rs, x, nrhs, st); else hif_fused_go<double, false, 2>(h, rr, rs, x, nrhs, st); }
    } else {
        if (w64) { if (up) hif_fused_go<float, true, 4>(h, rr, rs, x, nrhs, st); else hif_fused_go<float, false, 4>(h, rr, rs, x, nrhs, st); }
        else { if (up) hif_fused_go<float, true, 2>(h, rr, rs, x, nrhs, st); else hif_fused_go<float, false, 2>(h, rr, rs, x, nrhs, st); }
    }
    check_launch("hif step (fused)");
}

// Rows of a point-major block: out[i*nrhs + b] = x[idx[i]*nrhs + b] (with conversion), and back.
template <class Ti, class To>
__global__ void __launch_bounds__(256) k_rows_gather(const Ti *__restrict__ x, const int32_t *__restrict__ idx,
                                                     int64_t rows, int nrhs, To *__restrict__ out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < rows * nrhs; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = cvt<To, Ti>(x[(int64_t)idx[e / nrhs] * nrhs + e % nrhs]);
}
template <class Ti, class To>
__global__ void __launch_bounds__(256) k_rows_scatter(const Ti *__restrict__ in, const int32_t *__restrict__ idx,
                                                      int64_t rows, int nrhs, To *__restrict__ x) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < rows * nrhs; e += (int64_t)gridDim.x * blockDim.x)
        x[(int64_t)idx[e / nrhs] * nrhs + e % nrhs] = cvt<To, Ti>(in[e]);
}

// x[idx[r] * nrhs + b] = sum over z < parts of in[z * rows * nrhs + r * nrhs + b]
// (complex128 partial sums, summed in order), with conversion.
template <class To>
__global__ void __launch_bounds__(256) k_rows_scatter_sum(const double2 *__restrict__ in, int parts,
                                                          const int32_t *__restrict__ idx, int64_t rows, int nrhs,
                                                          To *__restrict__ x) {
    const int64_t n = rows * nrhs;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        double2 v[16];  // parts <= 16: every load issued before the first sum
#pragma unroll
        for (int z = 0; z < 16; ++z)
            if (z < parts) v[z] = in[z * n + e];
        double2 s = v[0];
#pragma unroll
        for (int z = 1; z < 16; ++z)
            if (z < parts) {
                s.x += v[z].x;
                s.y += v[z].y;
            }
        x[(int64_t)idx[e / nrhs] * nrhs + e % nrhs] = cvt<To, double2>(s);
    }
}

void launch_rows_scatter_sum(const void *in, int parts, const int32_t *idx, int64_t rows, int nrhs, void *x,
                             bool xd, hipStream_t st) {
    if (parts < 1 || parts > 16) throw std::runtime_error("rows scatter: 1 to 16 parts");
    const unsigned g = grid_for(rows * nrhs, 256);
    if (xd) hipLaunchKernelGGL(k_rows_scatter_sum<double2>, dim3(g), dim3(256), 0, st, (const double2 *)in, parts, idx, rows, nrhs, (double2 *)x);
    else hipLaunchKernelGGL(k_rows_scatter_sum<float2>, dim3(g), dim3(256), 0, st, (const double2 *)in, parts, idx, rows, nrhs, (float2 *)x);
    check_launch("rows scatter (sum of parts)");
}

void launch_rows_gather(const void *x, bool xd, const int32_t *idx, int64_t rows, int nrhs, void *out, bool od,
                        hipStream_t st) {
    const unsigned g = grid_for(rows * nrhs, 256);
    if (xd && od) hipLaunchKernelGGL((k_rows_gather<double2, double2>), dim3(g), dim3(256), 0, st, (const double2 *)x, idx, rows, nrhs, (double2 *)out);
    else if (xd) hipLaunchKernelGGL((k_rows_gather<double2, float2>), dim3(g), dim3(256), 0, st, (const double2 *)x, idx, rows, nrhs, (float2 *)out);
    else if (od) hipLaunchKernelGGL((k_rows_gather<float2, double2>), dim3(g), dim3(256), 0, st, (const float2 *)x, idx, rows, nrhs, (double2 *)out);
    else hipLaunchKernelGGL((k_rows_gather<float2, float2>), dim3(g), dim3(256), 0, st, (const float2 *)x, idx, rows, nrhs, (float2 *)out);
    check_launch("rows gather");
}

void launch_rows_scatter(const void *in, bool id, const int32_t *idx, int64_t rows, int nrhs, void *x, bool xd,
                         hipStream_t st) {
    const unsigned g = grid_for(rows * nrhs, 256);
    if (id && xd) hipLaunchKernelGGL((k_rows_scatter<double2, double2>), dim3(g), dim3(256), 0, st, (const double2 *)in, idx, rows, nrhs, (double2 *)x);
    else if (id) hipLaunchKernelGGL((k_rows_scatter<double2, float2>), dim3(g), dim3(256), 0, st, (const double2 *)in, idx, rows, nrhs, (float2 *)x);
    else if (xd) hipLaunchKernelGGL((k_rows_scatter<float2, double2>), dim3(g), dim3(256), 0, st, (const float2 *)in, idx, rows, nrhs, (double2 *)x);
    else hipLaunchKernelGGL((k_rows_scatter<float2, float2>), dim3(g), dim3(256), 0, st, (const float2 *)in, idx, rows, nrhs, (float2 *)x);
    check_launch("rows scatter");
}

// ------------------------------------------------------------------ top-level block (FP64)
template <class T>
__global__ void __launch_bounds__(256) k_root(const int32_t *__restrict__ idx,
                                              const double2 *__restrict__ A, int s0,
                                              T *__restrict__ x, int nrhs) {
    extern __shared__ char smem_raw[];
    double2 *v = reinterpret_cast<double2 *>(smem_raw);
    const int b = blockIdx.x;
    for (int i = threadIdx.x; i < s0; i += blockDim.x) v[i] = cvt<double2, T>(x[(int64_t)idx[i] * nrhs + b]);
    __syncthreads();
    for (int i = threadIdx.x; i < s0; i += blockDim.x) {
        double2 acc = make_double2(0.0, 0.0);
        for (int k = 0; k < s0; ++k) acc = cfma(acc, A[i + (int64_t)k * s0], v[k]);
        x[(int64_t)idx[i] * nrhs + b] = cvt<T, double2>(acc);
    }
}

void launch_root(const int32_t *idx, const void *A0inv, int s0, bool dbl, void *x, int nrhs,
                 hipStream_t st) {
    if (s0 == 0) return;
    if ((size_t)s0 * 16 > 64 * 1024) throw std::runtime_error("top-level block exceeds LDS");
    const size_t lds = (size_t)s0 * 16;
    if (dbl) hipLaunchKernelGGL(k_root<double2>, dim3(nrhs), dim3(256), lds, st, idx, (const double2 *)A0inv, s0, (double2 *)x, nrhs);
    else hipLaunchKernelGGL(k_root<float2>, dim3(nrhs), dim3(256), lds, st, idx, (const double2 *)A0inv, s0, (float2 *)x, nrhs);
    check_launch("root");
}

// ------------------------------------------------------------------ layout conversion
template <class Tu, class Ti>
__global__ void __launch_bounds__(256) k_gather(const Tu *__restrict__ user, int64_t ld,
                                                const int32_t *__restrict__ perm,
                                                Ti *__restrict__ out, int64_t n, int nrhs) {
    const int64_t total = n * nrhs;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(t % nrhs);
        const int64_t p = t / nrhs;
        const int64_t src = perm ? perm[p] : p;
        out[t] = cvt<Ti, Tu>(user[src + b * ld]);
    }
}
template <class Ti, class Tu>
__global__ void __launch_bounds__(256) k_scatter(const Ti *__restrict__ in,
                                                 const int32_t *__restrict__ perm,
                                                 Tu *__restrict__ user, int64_t ld, int64_t n,
                                                 int nrhs) {
    const int64_t total = n * nrhs;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(t % nrhs);
        const int64_t p = t / nrhs;
        const int64_t dst = perm ? perm[p] : p;
        user[dst + b * ld] = cvt<Tu, Ti>(in[t]);
    }
}

void launch_gather(const void *user, bool ud, int64_t ld, const int32_t *perm, void *internal,
                   bool id, int64_t n, int nrhs, hipStream_t st) {
    const unsigned g = grid_for(n * nrhs, 256);
    if (ud && id) hipLaunchKernelGGL((k_gather<double2, double2>), dim3(g), dim3(256), 0, st, (const double2 *)user, ld, perm, (double2 *)internal, n, nrhs);
    else if (ud && !id) hipLaunchKernelGGL((k_gather<double2, float2>), dim3(g), dim3(256), 0, st, (const double2 *)user, ld, perm, (float2 *)internal, n, nrhs);
    else if (!ud && id) hipLaunchKernelGGL((k_gather<float2, double2>), dim3(g), dim3(256), 0, st, (const float2 *)user, ld, perm, (double2 *)internal, n, nrhs);
    else hipLaunchKernelGGL((k_gather<float2, float2>), dim3(g), dim3(256), 0, st, (const float2 *)user, ld, perm, (float2 *)internal, n, nrhs);
    check_launch("gather");
}

void launch_scatter(const void *internal, bool id, const int32_t *perm, void *user, bool ud,
                    int64_t ld, int64_t n, int nrhs, hipStream_t st) {
    const unsigned g = grid_for(n * nrhs, 256);
    if (ud && id) hipLaunchKernelGGL((k_scatter<double2, double2>), dim3(g), dim3(256), 0, st, (const double2 *)internal, perm, (double2 *)user, ld, n, nrhs);
    else if (ud && !id) hipLaunchKernelGGL((k_scatter<float2, double2>), dim3(g), dim3(256), 0, st, (const float2 *)internal, perm, (double2 *)user, ld, n, nrhs);
    else if (!ud && id) hipLaunchKernelGGL((k_scatter<double2, float2>), dim3(g), dim3(256), 0, st, (const double2 *)internal, perm, (float2 *)user, ld, n, nrhs);
    else hipLaunchKernelGGL((k_scatter<float2, float2>), dim3(g), dim3(256), 0, st, (const float2 *)internal, perm, (float2 *)user, ld, n, nrhs);
    check_launch("scatter");
}

template <class Ts, class Td>
__global__ void __launch_bounds__(256) k_convert(const Ts *__restrict__ s, Td *__restrict__ d, int64_t n) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        d[t] = cvt<Td, Ts>(s[t]);
}

void launch_convert(const void *src, bool sd, void *dst, bool dd, int64_t count, hipStream_t st) {
    const unsigned g = grid_for(count, 256);
    if (sd && dd) hipLaunchKernelGGL((k_convert<double2, double2>), dim3(g), dim3(256), 0, st, (const double2 *)src, (double2 *)dst, count);
    else if (sd) hipLaunchKernelGGL((k_convert<double2, float2>), dim3(g), dim3(256), 0, st, (const double2 *)src, (float2 *)dst, count);
    else if (dd) hipLaunchKernelGGL((k_convert<float2, double2>), dim3(g), dim3(256), 0, st, (const float2 *)src, (double2 *)dst, count);
    else hipLaunchKernelGGL((k_convert<float2, float2>), dim3(g), dim3(256), 0, st, (const float2 *)src, (float2 *)dst, count);
    check_launch("convert");
}

// ------------------------------------------------------------------ FP64 vector updates
template <class Td>
__global__ void __launch_bounds__(256) k_residual(const double2 *__restrict__ u, const double2 *__restrict__ y,
                                                  Td *__restrict__ d, int64_t n) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        d[t] = cvt<Td, double2>(csub(u[t], y[t]));
}

void launch_residual(const void *u, const void *y, void *dst, bool dd, int64_t count, hipStream_t st) {
    const unsigned g = grid_for(count, 256);
    if (dd) hipLaunchKernelGGL(k_residual<double2>, dim3(g), dim3(256), 0, st, (const double2 *)u, (const double2 *)y, (double2 *)dst, count);
    else hipLaunchKernelGGL(k_residual<float2>, dim3(g), dim3(256), 0, st, (const double2 *)u, (const double2 *)y, (float2 *)dst, count);
    check_launch("residual");
}

template <class Ts>
__global__ void __launch_bounds__(256) k_axpy(double2 *__restrict__ x, const Ts *__restrict__ d, int64_t n) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        double2 v = cvt<double2, Ts>(d[t]);
        double2 a = x[t];
        a.x += v.x;
        a.y += v.y;
        x[t] = a;
    }
}

void launch_axpy_update(void *x, const void *d, bool dd, int64_t count, hipStream_t st) {
    const unsigned g = grid_for(count, 256);
    if (dd) hipLaunchKernelGGL(k_axpy<double2>, dim3(g), dim3(256), 0, st, (double2 *)x, (const double2 *)d, count);
    else hipLaunchKernelGGL(k_axpy<float2>, dim3(g), dim3(256), 0, st, (double2 *)x, (const float2 *)d, count);
    check_launch("axpy");
}

// Deterministic two-pass per-column reductions.  Pass 1: workgroup (g, bt) sums
// rows [g*chunk, (g+1)*chunk) for columns [bt*bw, bt*bw + bw) into partial[col][g];
// pass 2 adds the partials of each column in a fixed order.
static const int RED_G = 64;

int64_t reduce_partial_cap(int64_t n, int nrhs) { return (int64_t)RED_G * nrhs * 2; }

template <bool DOT>
__global__ void __launch_bounds__(256) k_colred1(const double2 *__restrict__ a, const double2 *__restrict__ c,
                                                 int64_t n, int nrhs, double *__restrict__ partial) {
    __shared__ double sre[256], sim[256];
    const int bw = min(nrhs, 256);
    const int col0 = blockIdx.y * bw;
    const int lanes = min(bw, nrhs - col0);
    const int rows_per = 256 / bw;
    const int tb = threadIdx.x % bw, tr = threadIdx.x / bw;
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = blockIdx.x * chunk, r1 = min(n, r0 + chunk);
    double s_re = 0, s_im = 0;
    if (tb < lanes && tr < rows_per) {
        const int col = col0 + tb;
        for (int64_t r = r0 + tr; r < r1; r += rows_per) {
            const double2 va = a[r * nrhs + col];
            if (DOT) {
                const double2 vc = c[r * nrhs + col];
                s_re += va.x * vc.x + va.y * vc.y;
                s_im += va.x * vc.y - va.y * vc.x;
            } else {
                s_re += va.x * va.x + va.y * va.y;
            }
        }
    }
    sre[threadIdx.x] = s_re;
    sim[threadIdx.x] = s_im;
    __syncthreads();
    if (tr == 0 && tb < lanes) {
        double tre = 0, tim = 0;
        for (int q = 0; q < rows_per; ++q) {
            tre += sre[q * bw + tb];
            tim += sim[q * bw + tb];
        }
        const int col = col0 + tb;
        partial[((int64_t)col * gridDim.x + blockIdx.x) * 2] = tre;
        partial[((int64_t)col * gridDim.x + blockIdx.x) * 2 + 1] = tim;
    }
}

template <bool DOT>
__global__ void k_colred2(const double *__restrict__ partial, int G, int nrhs, double *__restrict__ out) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= nrhs) return;
    double re = 0, im = 0;
    for (int g = 0; g < G; ++g) {
        re += partial[((int64_t)col * G + g) * 2];
        im += partial[((int64_t)col * G + g) * 2 + 1];
    }
    if (DOT) {
        out[2 * col] = re;
        out[2 * col + 1] = im;
    } else {
        out[col] = re;
    }
}

static void colred(bool dot, const void *a, const void *c, int64_t n, int nrhs, double *partial,
                   int64_t cap, double *out, hipStream_t st) {
    const int G = (int)std::max<int64_t>(1, std::min<int64_t>(RED_G, (n + 1023) / 1024));
    if ((int64_t)G * nrhs * 2 > cap) throw std::runtime_error("reduction workspace too small");
    const int bw = std::min(nrhs, 256);
    const dim3 g1(G, (nrhs + bw - 1) / bw);
    if (dot) hipLaunchKernelGGL(k_colred1<true>, g1, dim3(256), 0, st, (const double2 *)a, (const double2 *)c, n, nrhs, partial);
    else hipLaunchKernelGGL(k_colred1<false>, g1, dim3(256), 0, st, (const double2 *)a, (const double2 *)a, n, nrhs, partial);
    const dim3 g2((nrhs + 63) / 64);
    if (dot) hipLaunchKernelGGL(k_colred2<true>, g2, dim3(64), 0, st, partial, G, nrhs, out);
    else hipLaunchKernelGGL(k_colred2<false>, g2, dim3(64), 0, st, partial, G, nrhs, out);
    check_launch("column reduction");
}

void launch_colnorm2(const void *v, int64_t n, int nrhs, double *partial, int64_t cap, double *out,
                     hipStream_t st) {
    colred(false, v, v, n, nrhs, partial, cap, out, st);
}

void launch_coldot(const void *a, const void *c, int64_t n, int nrhs, double *partial, int64_t cap,
                   double *out, hipStream_t st) {
    colred(true, a, c, n, nrhs, partial, cap, out, st);
}

// a / b, and 0 where b is 0: a column whose right-hand side is zero has r = p = 0,
// so both PCG ratios are 0/0 there; a zero step keeps its exact solution x = 0.
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    const double den = b.x * b.x + b.y * b.y;
    if (!(den > 0.0)) return make_double2(0.0, 0.0);
    return make_double2((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}

__global__ void __launch_bounds__(256) k_pcg_xr(double2 *__restrict__ x, double2 *__restrict__ r,
                                                const double2 *__restrict__ p, const double2 *__restrict__ Ap,
                                                const double *__restrict__ rz, const double *__restrict__ pAp,
                                                int64_t n, int nrhs) {
    const int64_t total = n * nrhs;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(t % nrhs);
        const double2 al = cdiv(make_double2(rz[2 * b], rz[2 * b + 1]), make_double2(pAp[2 * b], pAp[2 * b + 1]));
        const double2 pv = p[t], av = Ap[t];
        double2 xv = x[t], rv = r[t];
        xv.x += al.x * pv.x - al.y * pv.y;
        xv.y += al.x * pv.y + al.y * pv.x;
        rv.x -= al.x * av.x - al.y * av.y;
        rv.y -= al.x * av.y + al.y * av.x;
        x[t] = xv;
        r[t] = rv;
    }
}

__global__ void __launch_bounds__(256) k_pcg_p(double2 *__restrict__ p, const double2 *__restrict__ z,
                                               const double *__restrict__ rzn, const double *__restrict__ rzo,
                                               int64_t n, int nrhs) {
    const int64_t total = n * nrhs;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(t % nrhs);
        const double2 be = cdiv(make_double2(rzn[2 * b], rzn[2 * b + 1]), make_double2(rzo[2 * b], rzo[2 * b + 1]));
        const double2 pv = p[t], zv = z[t];
        p[t] = make_double2(zv.x + be.x * pv.x - be.y * pv.y, zv.y + be.x * pv.y + be.y * pv.x);
    }
}

__global__ void __launch_bounds__(256) k_zero(double2 *__restrict__ x, int64_t n) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        x[t] = make_double2(0.0, 0.0);
}

void launch_scale_zero(void *x, int64_t count, hipStream_t st) {
    hipLaunchKernelGGL(k_zero, dim3(grid_for(count, 256)), dim3(256), 0, st, (double2 *)x, count);
    check_launch("zero");
}

void launch_pcg_xr(void *x, void *r, const void *p, const void *Ap, const double *rz, const double *pAp,
                   int64_t n, int nrhs, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_xr, dim3(grid_for(n * nrhs, 256)), dim3(256), 0, st, (double2 *)x, (double2 *)r,
                       (const double2 *)p, (const double2 *)Ap, rz, pAp, n, nrhs);
    check_launch("pcg x/r update");
}

void launch_pcg_p(void *p, const void *z, const double *rzn, const double *rzo, int64_t n, int nrhs,
                  hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_p, dim3(grid_for(n * nrhs, 256)), dim3(256), 0, st, (double2 *)p,
                       (const double2 *)z, rzn, rzo, n, nrhs);
    check_launch("pcg p update");
}

// y_b += sign * alpha_b * x_b per column b (complex128, alpha on the device as re, im pairs).
__global__ void __launch_bounds__(256) k_col_axpy(double2 *__restrict__ y, const double2 *__restrict__ x,
                                                  const double *__restrict__ alpha, double sign, int64_t n,
                                                  int nrhs) {
    const int64_t total = n * nrhs;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(t % nrhs);
        const double ar = sign * alpha[2 * b], ai = sign * alpha[2 * b + 1];
        const double2 xv = x[t];
        double2 yv = y[t];
        yv.x += ar * xv.x - ai * xv.y;
        yv.y += ar * xv.y + ai * xv.x;
        y[t] = yv;
    }
}

// y_b = x_b / sqrt(nrm2_b) per column (zero where nrm2_b is zero).
__global__ void __launch_bounds__(256) k_col_unit(double2 *__restrict__ y, const double2 *__restrict__ x,
                                                  const double *__restrict__ nrm2, int64_t n, int nrhs) {
    const int64_t total = n * nrhs;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(t % nrhs);
        const double s = nrm2[b] > 0 ? 1.0 / sqrt(nrm2[b]) : 0.0;
        const double2 xv = x[t];
        y[t] = make_double2(s * xv.x, s * xv.y);
    }
}

void launch_col_axpy(void *y, const void *x, const double *alpha, double sign, int64_t n, int nrhs, hipStream_t st) {
    hipLaunchKernelGGL(k_col_axpy, dim3(grid_for(n * nrhs, 256)), dim3(256), 0, st, (double2 *)y, (const double2 *)x,
                       alpha, sign, n, nrhs);
    check_launch("column axpy");
}

void launch_col_unit(void *y, const void *x, const double *nrm2, int64_t n, int nrhs, hipStream_t st) {
    hipLaunchKernelGGL(k_col_unit, dim3(grid_for(n * nrhs, 256)), dim3(256), 0, st, (double2 *)y, (const double2 *)x,
                       nrm2, n, nrhs);
    check_launch("column normalise");
}

// ------------------------------------------------------------------ inverse DFT (layout out)
// f = F^-1 fhat = n^d F* fhat (section 1: F_jk = n^-d exp(-2 pi i x_k . xi_j)).  With
// x_k = k/n and xi_j = j - n/2 per coordinate,
//   f_k = sum_j exp(2 pi i k (j - n/2) / n) fhat_j = sum_j' exp(2 pi i k j' / n) fhat_{j' + n/2},
// j' = j - n/2 mod n: an unnormalised inverse DFT of fhat rotated by n/2 in every
// coordinate.  k_dft_in gathers the user's column-major block into the point-major
// layout with that rotation; Stockham passes (radix 4, and radix 2 once when log2 n is
// odd) transform one coordinate at a time with the right-hand sides as the contiguous
// batch, so every load and store is coalesced; the plain scatter writes the result.
// Everything runs in FP64.
__global__ void __launch_bounds__(256) k_dft_in(const double2 *__restrict__ user, int64_t ld,
                                                double2 *__restrict__ x, int d, int n, int nrhs) {
    const int64_t N = d == 1 ? (int64_t)n : (int64_t)n * n;
    const int64_t total = N * nrhs;
    const int h = n / 2;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(t % nrhs);
        const int64_t p = t / nrhs;
        int64_t src;
        if (d == 1) {
            src = (p + h) % n;
        } else {
            const int64_t k1 = p / n, k2 = p % n;
            src = ((k1 + h) % n) * n + (k2 + h) % n;
        }
        x[t] = user[src + b * ld];
    }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

// One Stockham pass of radix R (2 or 4) over a length-n transform (sign +).  Element
// (o, p, i) of the data sits at (o*n + p)*inner + i; Ns is the length of the
// sub-transforms already done.  One thread per (o, j, i), j < n/R.
template <int R>
__global__ void __launch_bounds__(256) k_dft_pass(const double2 *__restrict__ in, double2 *__restrict__ out,
                                                  int64_t n, int64_t inner, int64_t outer, int64_t Ns) {
    const int64_t m = n / R;
    const int64_t total = outer * m * inner;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t % inner;
        const int64_t t2 = t / inner;
        const int64_t j = t2 % m, o = t2 / m;
        const int64_t k = j % Ns;
        const double2 *src = in + (o * n + j) * inner + i;
        double2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = src[(int64_t)r * m * inner];
#pragma unroll
        for (int r = 1; r < R; ++r) {
            double sn, cs;
            sincospi(2.0 * (double)(r * k) / (double)(Ns * R), &sn, &cs);
            v[r] = cmul(v[r], make_double2(cs, sn));
        }
        double2 w[R];
        if (R == 2) {
            w[0] = make_double2(v[0].x + v[1].x, v[0].y + v[1].y);
            w[1] = make_double2(v[0].x - v[1].x, v[0].y - v[1].y);
        } else {
            const double2 a0 = make_double2(v[0].x + v[2].x, v[0].y + v[2].y);
            const double2 a1 = make_double2(v[0].x - v[2].x, v[0].y - v[2].y);
            const double2 a2 = make_double2(v[1].x + v[3].x, v[1].y + v[3].y);
            const double2 a3 = make_double2(v[1].x - v[3].x, v[1].y - v[3].y);
            w[0] = make_double2(a0.x + a2.x, a0.y + a2.y);
            w[2] = make_double2(a0.x - a2.x, a0.y - a2.y);
            w[1] = make_double2(a1.x - a3.y, a1.y + a3.x);  // a1 + i a3
            w[3] = make_double2(a1.x + a3.y, a1.y - a3.x);  // a1 - i a3
        }
        double2 *dst = out + (o * n + (j / Ns) * Ns * R + k) * inner + i;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[(int64_t)r * Ns * inner] = w[r];
    }
}

void launch_inverse_dft(const void *fhat, int64_t ld, void *f, int d, int n, int nrhs, void *w0, void *w1,
                        hipStream_t st) {
    if (n < 2 || (n & (n - 1))) throw std::runtime_error("inverse DFT needs n a power of two");
    const int64_t N = d == 1 ? (int64_t)n : (int64_t)n * n;
    double2 *a = (double2 *)w0, *b = (double2 *)w1;
    hipLaunchKernelGGL(k_dft_in, dim3(grid_for(N * nrhs, 256)), dim3(256), 0, st, (const double2 *)fhat, ld, a,
                       d, n, nrhs);
    check_launch("inverse DFT gather");
    int lg = 0;
    while ((1 << lg) < n) ++lg;
    for (int dim = d - 1; dim >= 0; --dim) {
        // dim = d-1: the last (fastest) coordinate; dim 0 in 2D: the first
        const int64_t inner = (d == 2 && dim == 0) ? (int64_t)n * nrhs : nrhs;
        const int64_t outer = (d == 2 && dim == 1) ? n : 1;
        int64_t Ns = 1;
        for (int pass = 0; pass < lg / 2; ++pass) {
            hipLaunchKernelGGL(k_dft_pass<4>, dim3(grid_for(N * nrhs / 4, 256)), dim3(256), 0, st, a, b, (int64_t)n,
                               inner, outer, Ns);
            std::swap(a, b);
            Ns *= 4;
        }
        if (lg % 2) {
            hipLaunchKernelGGL(k_dft_pass<2>, dim3(grid_for(N * nrhs / 2, 256)), dim3(256), 0, st, a, b, (int64_t)n,
                               inner, outer, Ns);
            std::swap(a, b);
        }
        check_launch("inverse DFT pass");
    }
    launch_scatter(a, true, nullptr, f, true, ld, N, nrhs, st);
}


// ------------------------------------------------------------------ multi-instance launches
// One launch runs the same factor level of several instances (plans of different
// sizes, ranks and batch widths): stage s of each instance's chain, or step k of
// each instance's Gd sweep.  The instances travel by value in the kernel arguments;
// a workgroup finds its instance from the prefix of workgroup counts (`wg0`).  With
// a grid cap the launch is persistent: a fixed grid (a multiple of the eight XCDs)
// walks the whole work list, each workgroup staying on its XCD.
//
// Instance fields are read with compile-time indices (a select over the unrolled
// list), so the argument block is never copied to private memory.
template <class A> __device__ __forceinline__ A pick_inst(const A (&in)[MULTI_MAX], int n, int64_t lid) {
    A r = in[0];
#pragma unroll
    for (int j = 1; j < MULTI_MAX; ++j)
        if (j < n && lid >= in[j].wg0) r = in[j];
    return r;
}

// Logical workgroup ids of a (possibly persistent) launch over `total` workgroups,
// in the XCD-contiguous order of xcd_order: the loop visits this workgroup's ids.
#define FOR_EACH_WG(total, lid)                                                            \
    for (int64_t id_ = blockIdx.x, per_ = ((total) + N_XCD - 1) / N_XCD; id_ < per_ * N_XCD; \
         id_ += gridDim.x)                                                                 \
        for (int64_t lid = (id_ % N_XCD) * per_ + id_ / N_XCD; lid < (total); lid = (total))

template <class R, int MT, int NT>
__global__ void __launch_bounds__(256) k_stage_mfma_multi(const StageMultiArgs a) {
    using C = typename MF<R>::C;
    FOR_EACH_WG(a.total, lid) {
        const StageInstDev s = pick_inst(a.in, a.n, lid);
        const int64_t l = lid - s.wg0;
        stage_mfma_wg<R, MT, NT>(s.n_out, s.r_out, s.r_in, s.fan, s.idx, (const C *)s.A, (const C *)s.x,
                                 (C *)s.y, s.nrhs, s.mchunks, l / s.nch, (int)(l % s.nch));
    }
}

// Vector kernel: wg0 counts output entries (n_out * r_out * nrhs per instance).
template <class T>
__global__ void __launch_bounds__(256) k_stage_vec_multi(const StageMultiArgs a) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < a.total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const StageInstDev s = pick_inst(a.in, a.n, t);
        const int64_t l = t - s.wg0;
        ((T *)s.y)[l] = stage_entry(s.r_out, s.r_in, s.fan, s.idx, (const T *)s.A, (const T *)s.x, s.nrhs, l);
    }
}

template <class T, bool UP, bool STAGED>
__global__ void __launch_bounds__(256) k_hif_multi(const HifMultiArgs a) {
    FOR_EACH_WG(a.total, lid) {
        const HifInstDev s = pick_inst(a.in, a.n, lid);
        const int64_t l = lid - s.wg0;
        hif_node<T, UP, STAGED>(s.desc, s.idx, (const T *)s.mat, (T *)s.x, s.nrhs, s.bchunk, l / s.nch,
                                (int)(l % s.nch));  // ends with a barrier
    }
}

template <class R, bool UP, int NTW>
__global__ void __launch_bounds__(256) k_hif_fused_multi(const HifMultiArgs a) {
    using C = typename MF<R>::C;
    FOR_EACH_WG(a.total, lid) {
        const HifInstDev s = pick_inst(a.in, a.n, lid);
        const int64_t l = lid - s.wg0;
        hif_fused_node<R, UP, NTW>(s.desc, s.idx, (const C *)s.mat, (const C *)s.matH, (C *)s.x, s.nrhs, s.rows_r,
                                   s.rows_s, l / s.nch, (int)(l % s.nch));
        __syncthreads();  // the next node's staging overwrites this one's LDS
    }
}

// Top-level blocks: one workgroup per (instance, right-hand side), as k_root.
template <class T>
__global__ void __launch_bounds__(256) k_root_multi(const RootMultiArgs a) {
    extern __shared__ char smem_raw[];
    double2 *v = reinterpret_cast<double2 *>(smem_raw);
    for (int64_t lid = blockIdx.x; lid < a.total; lid += gridDim.x) {
        const RootInstDev s = pick_inst(a.in, a.n, lid);
        const int b = (int)(lid - s.wg0);
        T *x = (T *)s.x;
        for (int i = threadIdx.x; i < s.s0; i += blockDim.x) v[i] = cvt<double2, T>(x[(int64_t)s.idx[i] * s.nrhs + b]);
        __syncthreads();
        for (int i = threadIdx.x; i < s.s0; i += blockDim.x) {
            double2 acc = make_double2(0.0, 0.0);
            for (int k = 0; k < s.s0; ++k) acc = cfma(acc, s.A[i + (int64_t)k * s.s0], v[k]);
            x[(int64_t)s.idx[i] * s.nrhs + b] = cvt<T, double2>(acc);
        }
        __syncthreads();
    }
}

static unsigned multi_grid(int64_t total, int grid_cap) {
    const int64_t per = (total + N_XCD - 1) / N_XCD;
    int64_t g = per * N_XCD;
    if (grid_cap > 0) g = std::min<int64_t>(g, std::max(N_XCD, grid_cap / N_XCD * N_XCD));
    if (g >= ((int64_t)1 << 31)) throw std::runtime_error("multi-instance launch exceeds the grid limit");
    return (unsigned)std::max<int64_t>(1, g);
}

template <class R, int MT, int NT>
static void stage_multi_go(StageMultiArgs &a, const StageDev *s, int grid_cap, hipStream_t st) {
    int64_t wg = 0;
    for (int i = 0; i < a.n; ++i) {
        StageInstDev &d = a.in[i];
        d.mchunks = ((s[i].r_out + 15) / 16 + MT - 1) / MT;
        d.nch = (d.nrhs + 16 * NT - 1) / (16 * NT);
        d.wg0 = wg;
        wg += (d.n_out * d.mchunks + 3) / 4 * d.nch;
    }
    a.total = wg;
    hipLaunchKernelGGL((k_stage_mfma_multi<R, MT, NT>), dim3(multi_grid(wg, grid_cap)), dim3(256), 0, st, a);
}

template <class R>
static void stage_multi_variant(int v, StageMultiArgs &a, const StageDev *s, int cap, hipStream_t st) {
    switch (v) {
        case 1: stage_multi_go<R, 1, 4>(a, s, cap, st); break;
        case 2: stage_multi_go<R, 2, 4>(a, s, cap, st); break;
        case 3: stage_multi_go<R, 1, 2>(a, s, cap, st); break;
        case 4: stage_multi_go<R, 2, 2>(a, s, cap, st); break;
        case 5: stage_multi_go<R, 1, 1>(a, s, cap, st); break;
        case 8: stage_multi_go<R, 4, 4>(a, s, cap, st); break;
        case 9: stage_multi_go<R, 4, 2>(a, s, cap, st); break;
        default: stage_multi_go<R, 2, 1>(a, s, cap, st); break;
    }
}

void launch_stage_multi(const StageDev *s, const void *const *x, void *const *y, const int *nrhs, int n, bool dbl,
                        int variant, int grid_cap, hipStream_t st) {
    if (n < 1 || n > MULTI_MAX) throw std::runtime_error("multi-instance stage: 1..MULTI_MAX instances");
    StageMultiArgs a{};
    a.n = n;
    bool mfma_ok = variant > 0;
    for (int i = 0; i < n; ++i) {
        StageInstDev &d = a.in[i];
        d.idx = s[i].idx; d.A = s[i].A; d.x = x[i]; d.y = y[i];
        d.n_out = s[i].n_out; d.r_out = s[i].r_out; d.r_in = s[i].r_in; d.fan = s[i].fan; d.nrhs = nrhs[i];
        if (s[i].fan > 4 || s[i].r_in < 1 || s[i].r_out < 1) mfma_ok = false;
    }
    if (mfma_ok) {
        if (dbl) stage_multi_variant<double>(variant, a, s, grid_cap, st);
        else stage_multi_variant<float>(variant, a, s, grid_cap, st);
        check_launch("multi-instance stage (matrix cores)");
        return;
    }
    int64_t e = 0;
    for (int i = 0; i < n; ++i) {
        a.in[i].wg0 = e;
        e += s[i].n_out * s[i].r_out * (int64_t)nrhs[i];
    }
    a.total = e;
    const unsigned g = grid_for(e, 256);
    if (dbl) hipLaunchKernelGGL(k_stage_vec_multi<double2>, dim3(g), dim3(256), 0, st, a);
    else hipLaunchKernelGGL(k_stage_vec_multi<float2>, dim3(g), dim3(256), 0, st, a);
    check_launch("multi-instance stage");
}

template <class T, bool UP, bool ST>
static void hif_multi_go(const HifMultiArgs &a, size_t lds, int grid_cap, hipStream_t st) {
    static std::once_flag attr_once;  // plans may be used from several host threads
    std::call_once(attr_once, [] {
        (void)hipFuncSetAttribute((const void *)k_hif_multi<T, UP, ST>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  hif_lds_budget());
    });
    hipLaunchKernelGGL((k_hif_multi<T, UP, ST>), dim3(multi_grid(a.total, grid_cap)), dim3(256), lds, st, a);
}

template <class R, bool UP, int NTW>
static void hif_fused_multi_go(const HifMultiArgs &a, size_t lds, int grid_cap, hipStream_t st) {
    static std::once_flag attr_once;  // plans may be used from several host threads
    std::call_once(attr_once, [] {
        (void)hipFuncSetAttribute((const void *)k_hif_fused_multi<R, UP, NTW>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, hif_lds_budget());
    });
    hipLaunchKernelGGL((k_hif_fused_multi<R, UP, NTW>), dim3(multi_grid(a.total, grid_cap)), dim3(256), lds, st, a);
}

bool hif_multi_fits(const HifStepDev *h, int n, bool dbl, int kind) {
    for (int i = 0; i < n; ++i) {
        if (h[i].n_nodes == 0) continue;
        if (kind == 0 ? !hif_step_fits_lds(h[i], dbl) : !hif_fused_fits(h[i])) return false;
    }
    return true;
}

void launch_hif_multi(const HifStepDev *h, void *const *x, const int *nrhs, int n, bool dbl, bool up, int kind,
                      int grid_cap, hipStream_t st) {
    if (n < 1 || n > MULTI_MAX) throw std::runtime_error("multi-instance step: 1..MULTI_MAX instances");
    if (!hif_multi_fits(h, n, dbl, kind)) throw std::runtime_error("multi-instance step: a node does not fit");
    HifMultiArgs a{};
    a.n = n;
    const int elt = dbl ? 16 : 8;
    const int64_t HIF_LDS = hif_lds_budget();
    int64_t wg = 0;
    size_t lds = 0;
    if (kind == 0) {
        // LDS kernel: staged factor blocks only if every instance's fit beside one column
        bool staged = true;
        for (int i = 0; i < n; ++i)
            if ((int64_t)h[i].max_mat * elt + (int64_t)std::max(1, h[i].max_vec) * elt > HIF_LDS) staged = false;
        for (int i = 0; i < n; ++i) {
            HifInstDev &d = a.in[i];
            const int per = std::max(1, h[i].max_vec);
            const int64_t matb = staged ? (int64_t)h[i].max_mat * elt : 0;
            int bchunk = (int)std::max<int64_t>(1, std::min<int64_t>(nrhs[i], (HIF_LDS - matb) / ((int64_t)per * elt)));
            if (bchunk >= 64) bchunk = (bchunk / 64) * 64;
            const int64_t want = (int64_t)nrhs[i] * h[i].n_nodes / 1024;
            if (want < bchunk) bchunk = (int)std::max<int64_t>(std::min<int64_t>(16, bchunk), want);
            d.desc = h[i].desc; d.idx = h[i].idx; d.mat = h[i].mat; d.matH = h[i].matH; d.x = x[i];
            d.nrhs = nrhs[i]; d.bchunk = bchunk;
            d.nch = (nrhs[i] + bchunk - 1) / bchunk;
            d.wg0 = wg;
            wg += h[i].n_nodes * d.nch;
            lds = std::max(lds, (size_t)matb + (size_t)per * elt * bchunk);
        }
        a.total = wg;
        if ((int64_t)lds > HIF_LDS) throw std::runtime_error("multi-instance step exceeds LDS");
        if (dbl) {
            if (staged) { if (up) hif_multi_go<double2, true, true>(a, lds, grid_cap, st); else hif_multi_go<double2, false, true>(a, lds, grid_cap, st); }
            else { if (up) hif_multi_go<double2, true, false>(a, lds, grid_cap, st); else hif_multi_go<double2, false, false>(a, lds, grid_cap, st); }
        } else {
            if (staged) { if (up) hif_multi_go<float2, true, true>(a, lds, grid_cap, st); else hif_multi_go<float2, false, true>(a, lds, grid_cap, st); }
            else { if (up) hif_multi_go<float2, true, false>(a, lds, grid_cap, st); else hif_multi_go<float2, false, false>(a, lds, grid_cap, st); }
        }
        check_launch("multi-instance hif step");
        return;
    }
    // fused kernel, 64 (kind 4) or 32 (kind 5) right-hand sides per workgroup
    const int CW = kind == 4 ? 64 : 32, LD = CW + 4;
    const size_t celt = dbl ? sizeof(double2) : sizeof(float2);
    for (int i = 0; i < n; ++i) {
        HifInstDev &d = a.in[i];
        d.desc = h[i].desc; d.idx = h[i].idx; d.mat = h[i].mat; d.matH = h[i].matH; d.x = x[i];
        d.nrhs = nrhs[i];
        d.rows_r = std::max(16, (h[i].max_nr + 15) / 16 * 16);
        d.rows_s = std::max(16, (h[i].max_ns + 15) / 16 * 16);
        d.nch = (nrhs[i] + CW - 1) / CW;
        d.wg0 = wg;
        wg += h[i].n_nodes * d.nch;
        lds = std::max(lds, (size_t)(d.rows_r + d.rows_s) * LD * celt + (size_t)(d.rows_r + d.rows_s) * sizeof(int32_t));
    }
    a.total = wg;
    if ((int64_t)lds > HIF_LDS) throw std::runtime_error("multi-instance fused step exceeds LDS");
    if (dbl) {
        if (CW == 64) { if (up) hif_fused_multi_go<double, true, 4>(a, lds, grid_cap, st); else hif_fused_multi_go<double, false, 4>(a, lds, grid_cap, st); }
        else { if (up) hif_fused_multi_go<double, true, 2>(a, lds, grid_cap, st); else hif_fused_multi_go<double, false, 2>(a, lds, grid_cap, st); }
    } else {
        if (CW == 64) { if (up) hif_fused_multi_go<float, true, 4>(a, lds, grid_cap, st); else hif_fused_multi_go<float, false, 4>(a, lds, grid_cap, st); }
        else { if (up) hif_fused_multi_go<float, true, 2>(a, lds, grid_cap, st); else hif_fused_multi_go<float, false, 2>(a, lds, grid_cap, st); }
    }
    check_launch("multi-instance hif step (fused)");
}

void launch_root_multi(const int32_t *const *idx, const void *const *A0inv, const int *s0, void *const *x,
                       const int *nrhs, int n, bool dbl, hipStream_t st) {
    if (n < 1 || n > MULTI_MAX) throw std::runtime_error("multi-instance root: 1..MULTI_MAX instances");
    RootMultiArgs a{};
    a.n = n;
    int64_t wg = 0;
    int smax = 0;
    for (int i = 0; i < n; ++i) {
        RootInstDev &d = a.in[i];
        d.idx = idx[i]; d.A = (const double2 *)A0inv[i]; d.x = x[i]; d.s0 = s0[i]; d.nrhs = nrhs[i];
        d.wg0 = wg;
        wg += s0[i] > 0 ? nrhs[i] : 0;
        smax = std::max(smax, s0[i]);
    }
    a.total = wg;
    if (wg == 0) return;
    if ((size_t)smax * 16 > 64 * 1024) throw std::runtime_error("top-level block exceeds LDS");
    const size_t lds = (size_t)smax * 16;
    const unsigned g = (unsigned)std::min<int64_t>(wg, 1 << 20);
    if (dbl) hipLaunchKernelGGL(k_root_multi<double2>, dim3(g), dim3(256), lds, st, a);
    else hipLaunchKernelGGL(k_root_multi<float2>, dim3(g), dim3(256), lds, st, a);
    check_launch("multi-instance root");
}

}  // namespace fio
