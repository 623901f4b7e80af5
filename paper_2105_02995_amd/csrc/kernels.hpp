// Device kernels (gfx950) of the factor applies and their launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fio {

// One butterfly stage on nrhs vectors stored point-major ([block][row][rhs]):
//   y_o = sum_t A_{o,t} x_{in_idx[o*fan+t]}   (blocks column-major r_out x fan*r_in).
struct StageDev {
    int64_t n_out = 0, n_in = 0;
    int r_out = 0, r_in = 0, fan = 0;
    const int32_t *idx = nullptr;
    const void *A = nullptr;   // float2 (c64) or double2 (c128)
    int variant = -1;          // kernel variant (see stage_default_variant); -1: heuristic
};

// Number of stage kernel variants and the heuristic choice for a launch: 0 the
// vector kernel (one thread per output entry), 1..6 and 8, 9 matrix-core tilings
// (16*MT rows x 16*NT columns per wave: 1 MT1 NT4, 2 MT2 NT4, 3 MT1 NT2, 4 MT2 NT2,
// 5 MT1 NT1, 6 MT2 NT1, 8 MT4 NT4, 9 MT4 NT2), 7 the small-batch kernel (64 rows x 4
// k-slices per workgroup, for fewer than 16 columns), 10 and 11 the matrix-core
// kernel with the input staged in LDS and shared by a workgroup's four waves (one
// block of up to 192 rows per workgroup, 64 or 32 columns), 12..14 the register
// tilings MT2 NT4, MT4 NT2, MT2 NT2 with three real products per complex k-step.
constexpr int STAGE_VARIANTS = 15;
constexpr int STAGE_SMALL_BATCH = 7;
constexpr int STAGE_LDS4 = 10, STAGE_LDS2 = 11;
// Whether the multi-instance stage kernel has this variant (the four-product
// register tilings only).
inline bool stage_multi_variant_ok(int v) { return (v >= 1 && v <= 6) || v == 8 || v == 9; }
int stage_default_variant(const StageDev &s, bool dbl, int nrhs);

// Two consecutive stages a, b fused in one launch (the intermediate stays in LDS).
// tab: 16 int32 per workgroup (4 stage-a blocks, 4 stage-b blocks, 2 input slots
// per stage-b block; -1 pads), built from the closed groups of the two stages.
struct StagePairDev {
    StageDev a, b;
    const int32_t *tab = nullptr;
    int64_t n_wg = 0;
    // stacked variant: one closed group of two sibling pairs per stage per workgroup
    // (16 int32: stage-a pairs, stage-b pairs, input slots of each stage-b pair)
    const int32_t *tab_s = nullptr;
    int64_t n_wg_s = 0;
};
// Whether two stages with these shapes can run fused (ranks <= 32, fan of b <= 2).
bool stage_pair_fusable(int r_mid, int r_out_b, int fan_b);
// Fused kernel variants: 1: 16 columns per wave, 2: 32, 3: 64 (complex64 only).
int stage_pair_variants(bool dbl);
// Variant number of the stacked fused pair (sibling blocks sharing their inputs
// stacked into one operand of 16-row tiles; ranks <= 32 and a stacked table).
constexpr int STAGE_PAIR_STACKED = 4;
bool stage_pair_stackable(int r_mid, int r_out_b);
void launch_stage_pair(const StagePairDev &p, bool dbl, int variant, const void *x, void *y, int nrhs,
                       hipStream_t st);

// Three consecutive stages a, b, c in one launch: closed groups of four blocks per
// stage; the stage-b and stage-c blocks of a group split into two sibling pairs
// (blocks with equal input lists).  tab: 20 int32 per workgroup: the four stage-a
// blocks, the four stage-b blocks (sibling pairs adjacent), for each stage-b pair the
// workgroup slots (0..3, position in the stage-a list) of its fan_b <= 2 inputs (-1
// pads), the four stage-c blocks and the slots (positions in the stage-b list) of each
// stage-c pair's inputs.  Ranks up to 32, fan_a <= 4.
struct StageTripleDev {
    StageDev a, b, c;
    const int32_t *tab = nullptr;
    int64_t n_wg = 0;
};
constexpr int STAGE_TRIPLE_TAB = 20;
void launch_stage_triple(const StageTripleDev &t, bool dbl, const void *x, void *y, int nrhs, hipStream_t st);

// Node factor table of one skeletonization step: per node
// {nr, ns, idx_off, mat_off}; idx holds idx_r then idx_s; mat holds T (ns x nr),
// Linv (nr x nr), M (ns x nr), column-major, one after the other.
struct HifStepDev {
    int64_t n_nodes = 0;
    int max_nr = 0, max_ns = 0;
    int max_vec = 0;   // max over nodes of 2*nr + ns (LDS entries per right-hand side)
    int max_mat = 0;   // max over nodes of 2*ns*nr + nr*nr (entries of the node's blocks)
    // Tiles of 16 output rows for the matrix-core path: pairs (node, first row)
    // over the redundant rows (nr) and over the skeleton rows (ns).
    const int32_t *tiles_r = nullptr, *tiles_s = nullptr;
    int64_t n_tiles_r = 0, n_tiles_s = 0;
    // The same over tiles of 32 and of 64 rows (two and four matrix-core row tiles
    // per wave, for large nodes: each gathered input row then serves more rows).
    const int32_t *tiles_r2 = nullptr, *tiles_s2 = nullptr, *tiles_r4 = nullptr, *tiles_s4 = nullptr;
    int64_t n_tiles_r2 = 0, n_tiles_s2 = 0, n_tiles_r4 = 0, n_tiles_s4 = 0;
    const int64_t *desc = nullptr;
    const int32_t *idx = nullptr;
    const void *mat = nullptr;
    // Conjugate transposes T^* (nr x ns), Linv^* (nr x nr), M^* (nr x ns) at the
    // offsets of T, Linv, M, column-major (read by the matrix-core path).
    const void *matH = nullptr;
};

void launch_stage(const StageDev &s, bool dbl, const void *x, void *y, int nrhs, hipStream_t st);
void launch_hif_step(const HifStepDev &h, bool dbl, bool up, void *x, int nrhs, hipStream_t st);
// Large-node variant of launch_hif_step (gathered GEMMs on matrix cores, tiles of
// 16*mt rows by `cols` right-hand sides: mt 1 with cols 16, 32 or 64, mt 2 with 32,
// mt 4 with 16 or 32; m3: three real products per complex k-step, mt 1 with 32 or 64
// columns or mt 2 with 32); t is an N x nrhs temporary of the same dtype.
void launch_hif_gemm_step(const HifStepDev &h, bool dbl, bool up, void *x, void *t, int nrhs, int cols,
                          hipStream_t st, int mt = 1, bool m3 = false);
// Small-batch variant (fewer than 16 right-hand sides): each phase as gathered
// matrix-vector products over the 64-row tiles, bound by the factor bytes; t as above;
// part (part_bytes, may be null) holds the partial sums of phases whose k ranges are
// split over workgroups (fewer slices, or none, where it is too small).
void launch_hif_gemv_step(const HifStepDev &h, bool dbl, bool up, void *x, void *t, int nrhs, void *part,
                          size_t part_bytes, hipStream_t st);
// Whether a step's largest node fits the LDS-staged kernel.
bool hif_step_fits_lds(const HifStepDev &h, bool dbl);
// One skeletonization step in a single launch for nodes with nr, ns <= 64: per
// (node, 64 or 32 right-hand sides) the node's entries of x are staged in LDS and
// the step's three products run on matrix cores.
bool hif_fused_fits(const HifStepDev &h);
// cols: right-hand sides per workgroup, 64 or 32.
void launch_hif_fused_step(const HifStepDev &h, bool dbl, bool up, void *x, int nrhs, hipStream_t st,
                           int cols = 64);
void launch_rows_gather(const void *x, bool xd, const int32_t *idx, int64_t rows, int nrhs, void *out, bool od,
                        hipStream_t st);
// The small-batch stage kernel with its k range split over ksplit workgroups: y
// receives ksplit partial results, slice z at y + z * n_out * r_out * nrhs.
void launch_stage_nb_split(const StageDev &s, bool dbl, const void *x, void *y, int nrhs, int ksplit,
                           hipStream_t st);
// x[idx[r] * nrhs + b] = sum over z < parts of in[(z * rows + r) * nrhs + b] (in
// complex128), converted to x's dtype.
void launch_rows_scatter_sum(const void *in, int parts, const int32_t *idx, int64_t rows, int nrhs, void *x,
                             bool xd, hipStream_t st);
void launch_rows_scatter(const void *in, bool id, const int32_t *idx, int64_t rows, int nrhs, void *x, bool xd,
                         hipStream_t st);
void launch_root(const int32_t *idx, const void *A0inv, int s0, bool dbl, void *x, int nrhs,
                 hipStream_t st);
// internal[t*nrhs + b] = user[perm[t] + b*ld] (perm may be null), with conversion.
void launch_gather(const void *user, bool user_dbl, int64_t ld, const int32_t *perm, void *internal,
                   bool int_dbl, int64_t n, int nrhs, hipStream_t st);
void launch_scatter(const void *internal, bool int_dbl, const int32_t *perm, void *user,
                    bool user_dbl, int64_t ld, int64_t n, int nrhs, hipStream_t st);
// dst = src (contiguous), with conversion.
void launch_convert(const void *src, bool src_dbl, void *dst, bool dst_dbl, int64_t count,
                    hipStream_t st);
// r = u - y (complex128 u, y) written as dst dtype.
void launch_residual(const void *u, const void *y, void *dst, bool dst_dbl, int64_t count,
                     hipStream_t st);
// x += d (x complex128, d of dtype).
void launch_axpy_update(void *x, const void *d, bool d_dbl, int64_t count, hipStream_t st);
// Per-column squared norms of an n x nrhs point-major complex128 block: out[b] (double).
void launch_colnorm2(const void *v, int64_t n, int nrhs, double *partial, int64_t partial_cap,
                     double *out, hipStream_t st);
// Per-column dots <a_b, c_b> (conj(a) c) of complex128 blocks: out[2b], out[2b+1] = re, im.
void launch_coldot(const void *a, const void *c, int64_t n, int nrhs, double *partial,
                   int64_t partial_cap, double *out, hipStream_t st);
// PCG vector updates (complex128, per-column scalars on the device).
void launch_pcg_xr(void *x, void *r, const void *p, const void *Ap, const double *rz,
                   const double *pAp, int64_t n, int nrhs, hipStream_t st);
void launch_pcg_p(void *p, const void *z, const double *rz_new, const double *rz_old, int64_t n,
                  int nrhs, hipStream_t st);

// GMRES vector updates (complex128, per-column scalars on the device):
// y_b += sign * alpha_b x_b (alpha as re, im pairs); y_b = x_b / sqrt(nrm2_b).
void launch_col_axpy(void *y, const void *x, const double *alpha, double sign, int64_t n, int nrhs,
                     hipStream_t st);
void launch_col_unit(void *y, const void *x, const double *nrm2, int64_t n, int nrhs, hipStream_t st);

int64_t reduce_partial_cap(int64_t n, int nrhs);
// f = n^d F* fhat (section 1) for user-layout complex128 blocks (column-major N x nrhs,
// leading dimension ld; f may alias fhat).  w0, w1: N x nrhs complex128 temporaries.
void launch_inverse_dft(const void *fhat, int64_t ld, void *f, int d, int n, int nrhs, void *w0, void *w1,
                        hipStream_t st);
// x = 0 (complex128), by a fill kernel (no memset node if the stream is captured).
void launch_scale_zero(void *x, int64_t count, hipStream_t st);

// ------------------------------------------------------------------ multi-instance launches
// One launch for the same factor level of up to MULTI_MAX instances (different
// plans, sizes and batch widths).  The instance lists travel by value as kernel
// arguments (no device memory, nothing to copy: a captured graph keeps them).
constexpr int MULTI_MAX = 8;
struct StageInstDev {
    const int32_t *idx;
    const void *A, *x;
    void *y;
    int64_t n_out, wg0;
    int r_out, r_in, fan, nrhs, mchunks, nch;
};
struct StageMultiArgs {
    StageInstDev in[MULTI_MAX];
    int n;
    int64_t total;
};
struct HifInstDev {
    const int64_t *desc;
    const int32_t *idx;
    const void *mat, *matH;
    void *x;
    int64_t wg0;
    int nrhs, bchunk, nch, rows_r, rows_s;
};
struct HifMultiArgs {
    HifInstDev in[MULTI_MAX];
    int n;
    int64_t total;
};
struct RootInstDev {
    const int32_t *idx;
    const double2 *A;
    void *x;
    int64_t wg0;
    int s0, nrhs;
};
struct RootMultiArgs {
    RootInstDev in[MULTI_MAX];
    int n;
    int64_t total;
};
// Stage s[i] of instance i applied to x[i] (nrhs[i] columns) into y[i], all in one
// launch: matrix cores with the variant's tiles (1..6 as launch_stage) when every
// instance allows them (fan <= 4), else the vector kernel.  grid_cap > 0: persistent
// grid of at most grid_cap workgroups (rounded to the eight XCDs).
void launch_stage_multi(const StageDev *s, const void *const *x, void *const *y, const int *nrhs, int n, bool dbl,
                        int variant, int grid_cap, hipStream_t st);
// Whether every instance's step fits kind 0 (LDS kernel) or 4/5 (fused kernel).
bool hif_multi_fits(const HifStepDev *h, int n, bool dbl, int kind);
// Skeletonization step h[i] of every instance on x[i], in one launch: kind 0 the
// LDS-staged node kernel, 4/5 the fused matrix-core node kernel with 64/32 columns
// per workgroup.
void launch_hif_multi(const HifStepDev *h, void *const *x, const int *nrhs, int n, bool dbl, bool up, int kind,
                      int grid_cap, hipStream_t st);
// Top-level blocks A0inv[i] (FP64, s0[i] x s0[i]) on the rows idx[i] of x[i], one launch.
void launch_root_multi(const int32_t *const *idx, const void *const *A0inv, const int *s0, void *const *x,
                       const int *nrhs, int n, bool dbl, hipStream_t st);

}  // namespace fio
