/*
 * fio.h -- C ABI of the MI355X (gfx950) approximate-inverse library for discrete
 * Fourier integral operators (Feliu-Faba and Ying, "Approximate inversion of
 * discrete Fourier integral operators").
 *
 * Problem (section 1, equations eq:X_domain, eq:freq_domain, eq3, eq6): grids
 *   X     = { x = (k_1..k_d)/n : 0 <= k_i < n },
 *   Omega = { xi = (j_1..j_d)   : -n/2 <= j_i < n/2 },   n even, N = n^d,
 * and the dense N x N matrix K with K_ij = a(x_i, xi_j) exp(2 pi i Phi(x_i, xi_j)),
 * so that u = K fhat with fhat = F f the normalised DFT.  Points are numbered
 * lexicographically with the first coordinate slowest ("natural order").
 *
 * The library builds, on the host in FP64, the butterfly factorization
 * Kd = U_L C_{L-1}..C_{lm} D H*_{lm}..H*_{1} V*_L of K (section 2, eq_BFF_fact),
 * a hierarchical representation Sd of S = Kd^* Kd by peeling (section 3), and the
 * inverse factors Gd = R_L..R_1 A_0^{-1} R_1^*..R_L^* of Sd (section 4,
 * eqAinv_1d / eqAinv_2d).  The factors are uploaded to one GPU, and every apply
 * (Kd, Kd^*, Gd Kd^* ~ K^{-1}, eq:pseudoinv, section 5) runs in HIP kernels.
 *
 * Conventions shared by every entry point:
 *  - Vectors are complex, interleaved (re, im): FIO_C64 = two floats, FIO_C128 =
 *    two doubles.  A block of nrhs vectors is column-major N x nrhs with leading
 *    dimension ld >= N (in elements), in natural order.  Vector buffers are
 *    device pointers owned by the caller.
 *  - hip_stream is a hipStream_t (NULL = the default stream).  Applies are
 *    asynchronous on that stream; they may use library-owned device workspace
 *    that is sized for the largest nrhs seen (grown on demand), so calls on one
 *    plan must not run concurrently on different streams.
 *  - Graph capture: a call made while hip_stream is being captured records the
 *    plan's workspace addresses into the graph.  From then on the workspace of
 *    that plan never moves: a later call (captured or not) that needs more
 *    columns than the workspace holds fails with FIO_ERR_ARG.  Make the widest
 *    call once, eagerly, before capturing.
 *  - Every call returns an fio_status; nothing throws across the ABI.  On error
 *    the outputs are unspecified, fio_last_error() gives a message (thread
 *    local), and the plan stays valid unless the status is FIO_ERR_DEVICE.
 */
#ifndef FIO_H
#define FIO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fio_plan_s *fio_plan;

typedef enum {
    FIO_OK = 0,
    FIO_ERR_ARG = 1,            /* invalid argument                               */
    FIO_ERR_NOMEM = 2,          /* host or device allocation failed               */
    FIO_ERR_DEVICE = 3,         /* HIP runtime error                              */
    FIO_ERR_NOT_HPD = 4,        /* a pivot block of the inverse was not HPD       */
    FIO_ERR_NOT_CONVERGED = 5,  /* iterative solve did not reach its tolerance    */
    FIO_ERR_UNSUPPORTED = 6,    /* request not supported by this plan             */
    FIO_ERR_IO = 7              /* save/load failure                              */
} fio_status;

typedef enum { FIO_C64 = 0, FIO_C128 = 1 } fio_dtype;

/* Operator selector of fio_apply: Kd (frequency -> space) or its adjoint. */
typedef enum { FIO_OP_K = 0, FIO_OP_KH = 1 } fio_op;

/* Phase functions (and amplitudes) of the paper's numerical section (section 6);
 * a = 1 except for Example 2. */
typedef enum {
    FIO_PHASE_LINEAR = 0,   /* Phi = x.xi (K = N F^*: exact identity checks)                */
    FIO_PHASE_1D_EX1 = 1,   /* Phi = x xi + c(x)|xi|, c(x) = (2 + sin 2 pi x)/c_div  (Ex. 1) */
    FIO_PHASE_2D_RADON = 2, /* Phi = x.xi + sqrt(c1^2 xi1^2 + c2^2 xi2^2),          (Ex. 3)
                               c1 = (2 + sin 2pi x1 sin 2pi x2)/c_div,
                               c2 = (2 + cos 2pi x1 cos 2pi x2)/c_div                     */
    FIO_PHASE_1D_EX2 = 3,   /* Example 1's phase with the variable amplitude of Ex. 2:
                               a(x, xi) = sum_k exp(-(d(x, x_k)^2 + (xi/n - eta_k)^2)/sigma2),
                               d the distance on the unit circle (periodic in x); the
                               centres come from amp_x/amp_eta (see fio_problem)          */
    FIO_PHASE_CALLBACK = 4  /* any FIO of section 1 (eq3, eq6): the phase Phi(x, xi) and
                               the amplitude a(x, xi) come from the caller's functions
                               phi and amp of fio_problem                                 */
} fio_phase_id;

/* Phase of a caller-defined FIO (FIO_PHASE_CALLBACK): returns Phi(x, xi) in cycles,
 * so that K_ij = a(x_i, xi_j) exp(2 pi i Phi(x_i, xi_j)) (section 1, eq6).  x holds the
 * d coordinates of a point of X (each k/n in [0, 1)), xi the d frequencies of a point
 * of Omega (integers -n/2 .. n/2 - 1, as doubles).  The whole phase is returned,
 * including the linear part x.xi; the library reduces it mod 1 in FP64 (so the phase
 * must be accurate to a small fraction of a cycle, far below eps, at |xi| up to n/2).
 * Called on the host during fio_build only, concurrently from several threads, so it
 * must be thread-safe; user is fio_problem.user. */
typedef double (*fio_phase_fn)(const double *x, const double *xi, int d, void *user);

/* Amplitude a(x, xi) of a caller-defined FIO: writes its real and imaginary parts to
 * re_im[0], re_im[1].  Same arguments and rules as fio_phase_fn.  a must be smooth in
 * both variables (the butterfly compresses K; section 1 assumes a symbol). */
typedef void (*fio_amp_fn)(const double *x, const double *xi, int d, void *user, double re_im[2]);

#define FIO_MAX_AMP_TERMS 8

/* Build description.  Zero means "default" for every tuning field. */
typedef struct {
    int d;                  /* dimension, 1 or 2                                       */
    int n;                  /* points per dimension: even power of two, N = n^d        */
    fio_phase_id phase;
    double c_div;           /* divisor of c(x) (Examples 1 and 3); 0 -> 16             */
    double eps;             /* tolerance: peeling and inverse tolerances default to it */
    double eps_bf;          /* butterfly tolerance; 0 -> eps/10                        */
    double eps_peel;        /* peeling tolerance;   0 -> eps                           */
    double eps_hif;         /* skeletonization tolerance; 0 -> eps                     */
    int leaf_bf;            /* butterfly leaf side (points per dim); 0 -> 8 (1D), 4 (2D) */
    int leaf_h;             /* hierarchical-matrix leaf side; 0 -> 64 (1D), 8 (2D)     */
    int oversample;         /* peeling oversampling c; 0 -> 10                         */
    uint64_t seed;          /* seed of the peeling probes                              */
    int device;             /* HIP device ordinal, or -1 for a host-only plan that can
                               be saved and loaded later but not applied              */
    int nthreads;           /* host threads for the build; 0 -> OMP_NUM_THREADS, else
                               the CPUs of the process's affinity mask                */
    int verbose;            /* nonzero: fio_build prints one progress line per phase
                               and per tree level to stderr                           */
    /* Example 2 amplitude (FIO_PHASE_1D_EX2 only; not stored by fio_save).  The paper
     * gives neither the number of Gaussian terms nor their centres; amp_terms = 0
     * selects three terms at (x, xi/n) = (0.2, -0.2), (0.5, 0.2), (0.8, 0.0).     */
    double amp_sigma2;      /* width sigma^2 of every term; 0 -> 0.1                   */
    int amp_terms;          /* number of terms, 0..FIO_MAX_AMP_TERMS                   */
    double amp_x[FIO_MAX_AMP_TERMS];    /* centres in x, in [0, 1)                     */
    double amp_eta[FIO_MAX_AMP_TERMS];  /* centres in xi/n, in [-1/2, 1/2)             */
    /* A skeletonization pivot block (or the top-level block) that is not positive
     * definite, because the approximation error of Sd exceeds its smallest eigenvalue
     * (ill-conditioned K), is factored with a diagonal shift (from 1e-3 eps_hif ||S||_2,
     * doubled until it is), which keeps Gd Hermitian positive definite: a
     * preconditioner-quality inverse on those nodes.  strict_hpd = 1 makes the build
     * fail with FIO_ERR_NOT_HPD instead.                                           */
    int strict_hpd;
    /* The butterfly's interpolative decompositions (sampling K, pivoted QR, the
     * interpolation matrices) run on the plan's device unless this is nonzero or the
     * plan is host-only; both give factors of the same accuracy.                    */
    int host_construction;
    /* 1D only (FIO_ERR_ARG for d = 2): Cholesky-prescaled skeletonization, the
     * paper's alternative to the elimination step (section 4, 1D case): every node is
     * first scaled by the inverse Cholesky factor of its diagonal block, the ID is
     * taken on the scaled bases, and the elimination that remains acts on I + T^*T
     * (always positive definite).  Gd then has two steps per level (the scaling, a
     * node with redundant DOFs only, then the skeletonization).  Not stored by
     * fio_save (the factors are).                                                  */
    int prescale_skel;
    /* FIO_PHASE_CALLBACK only (ignored otherwise): the caller's phase (required) and
     * amplitude (NULL means a = 1), both evaluated on the host during fio_build, and the
     * pointer passed to them.  The butterfly then samples K on the host and hands the
     * samples to the device decompositions.  Neither function is stored by fio_save:
     * a saved plan holds the factors, which is all an apply needs.                  */
    fio_phase_fn phi;
    fio_amp_fn amp;
    void *user;
    /* Butterfly rank alignment; 0 -> 8, 1 keeps every level at its tolerance rank.
     * A level whose rank r (the largest numerical rank of the probe blocks at eps_bf,
     * section 2's interpolative decompositions) is not a multiple of bf_rank_align is
     * given rank floor(r / bf_rank_align) * bf_rank_align when the probe blocks need
     * no more at 4 eps_bf: whole matrix-core tiles for at most 4x the level's ID
     * residual.  Not stored by fio_save (the ranks are, in the factors).           */
    int bf_rank_align;
} fio_problem;

/* Build the factors of K and of the approximate inverse (Algorithm "alg",
 * section 5: butterfly factorization, peeling, hierarchical inversion).
 * Synchronous.  On success *out is a library-owned plan (free with fio_destroy).
 * Errors: FIO_ERR_ARG (d, n, eps out of range), FIO_ERR_NOT_HPD, FIO_ERR_NOMEM,
 * FIO_ERR_DEVICE. */
fio_status fio_build(const fio_problem *p, fio_plan *out);

/* Tracing: with on != 0 every solve, chain apply, Gd sweep and step, and refinement
 * or PCG iteration pushes a named range for a profiler's marker trace (roctx; e.g.
 * rocprofv3 --marker-trace); 0 (the default) switches it off.  Process-wide; host
 * overhead only (about a microsecond per range) and no effect on results. */
void fio_set_trace(int on);

/* y = Kd x (op = FIO_OP_K, eq_BFF_fact) or y = Kd^* x (op = FIO_OP_KH).
 * x, y: device buffers of dtype, N x nrhs, leading dimension ld; x and y must
 * not overlap.  Asynchronous on hip_stream. */
fio_status fio_apply(fio_plan plan, fio_op op, fio_dtype dtype, const void *x, void *y,
                     int64_t nrhs, int64_t ld, void *hip_stream);

/* fhat = Gd Kd^* u, the approximate inverse of K (section 5, eq:pseudoinv).
 * The small top-level block A_0^{-1} is applied in FP64 for both dtypes.
 * u, fhat: device buffers of dtype, N x nrhs, leading dimension ld, no overlap.
 * Asynchronous. */
fio_status fio_inverse_apply(fio_plan plan, fio_dtype dtype, const void *u, void *fhat,
                             int64_t nrhs, int64_t ld, void *hip_stream);

/* fhat = Gd Kd^* u as fio_inverse_apply (same kernels, same launches, the same
 * result bit for bit), for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  The call
 * allocates nothing (no hipMalloc or hipFree, no allocating library routine): its
 * temporaries live in one static device array of 256 MiB per GPU, reserved when the
 * library's code object is loaded on that GPU and held until the process ends.  The
 * plan's factors were allocated by fio_build; the caller passes u and fhat as for
 * fio_inverse_apply.  The temporaries need
 *   (3 N + 2 C) nrhs e + 2 s0 nrhs 16 bytes (each part rounded up to 256 bytes),
 * e = 8 (FIO_C64) or 16 (FIO_C128), C the longest coefficient vector between butterfly
 * stages, s0 the top-level block (fio_plan_stats_t.root_size); e.g. 1D N = 65536 takes
 * about 5 MB per complex64 right-hand side.  Errors: FIO_ERR_ARG when nrhs needs more
 * than 256 MiB (the message states the bytes), as fio_inverse_apply otherwise.
 * Every call on one GPU uses that GPU's one array, for every plan: calls that overlap
 * on one GPU (different streams or host threads) race and give wrong results; the
 * array keeps the last call's contents, and no part of it has to start at zero.
 * Asynchronous. */
fio_status fio_inverse_apply_noalloc(fio_plan plan, fio_dtype dtype, const void *u, void *fhat,
                                     int64_t nrhs, int64_t ld, void *hip_stream);

/* y = Gd x, the approximate inverse of Kd^* Kd alone (section 4). */
fio_status fio_gd_apply(fio_plan plan, fio_dtype dtype, const void *x, void *y,
                        int64_t nrhs, int64_t ld, void *hip_stream);

/* y = Gd x as fio_gd_apply, with every skeletonization step on one kernel:
 * 0 the LDS-staged per-node kernel, 1/2/3 gathered GEMMs on matrix cores in tiles of
 * 16 rows by 64/32/16 right-hand sides, 6 the same in tiles of 32 rows by 32, 7/8 of
 * 64 rows by 16/32, 9/10/11 as 1/2/6 with three real products per complex
 * multiply-add instead of four, 4/5 the fused per-node matrix-core kernel with 64/32
 * right-hand sides per workgroup (a step whose nodes exceed 64 redundant or 64
 * skeleton DOFs keeps its tuned choice), 12 gathered matrix-vector products for
 * small batches (64 rows per workgroup, any nrhs; the factor bytes bound it), -1 the
 * tuned (else default) choice per step, which is what fio_gd_apply runs.  For tests
 * and measurement: all variants agree to rounding.  Asynchronous.  Errors:
 * FIO_ERR_ARG (variant out of range, as fio_gd_apply otherwise). */
fio_status fio_gd_apply_variant(fio_plan plan, fio_dtype dtype, int variant, const void *x, void *y,
                                int64_t nrhs, int64_t ld, void *hip_stream);

typedef enum {
    FIO_SOLVE_DIRECT = 0,   /* fhat = Gd Kd^* u                                        */
    FIO_SOLVE_REFINE = 1,   /* direct solve, then x += Gd Kd^*(u - Kd x) with the
                               residual in FP64 (complex128 factors)                  */
    FIO_SOLVE_PCG = 2,      /* CG on Kd^* Kd x = Kd^* u preconditioned by Gd (section 5) */
    FIO_SOLVE_GMRES = 3     /* restarted GMRES on Kd fhat = u with the right preconditioner
                               Gd Kd^* (sections 1 and 7 name GMRES with the factorization
                               as preconditioner; unlike CG on the normal equations it
                               does not square cond(K)); vectors and Gram-Schmidt in FP64,
                               operator applies in dtype                                  */
} fio_solve_mode;

typedef struct {
    fio_solve_mode mode;
    double tol;             /* REFINE: stop when ||dx|| <= tol ||x|| for every column;
                               PCG: stop when ||r|| <= tol ||Kd^* u||;
                               GMRES: stop when ||u - Kd x|| <= tol ||u||; 0 -> run maxit */
    int maxit;              /* iteration cap (REFINE steps, PCG or GMRES iterations)   */
    int precondition;       /* PCG only: 1 -> Gd, 0 -> none (the paper's "Kd^* only") */
    int spatial;            /* 1 -> return f = F^{-1} fhat (see fio_inverse_dft) instead of fhat */
    int restart;            /* GMRES only: Krylov dimension per cycle (0 -> 20, at most 64) */
} fio_solve_opts;

typedef struct {
    int iters;              /* iterations performed                                    */
    double rel_resid;       /* max over columns of the last relative residual/correction */
    double est_rel_err;     /* estimate of max over columns of ||x - K^{-1}u|| / ||K^{-1}u||,
                               the error against the exact solve (the method's error, not
                               only the iteration's): from the plan's estimates e_a, e_s
                               and cond(Kd) (fio_plan_stats_t) and this solve's rel_resid:
                                 DIRECT  e_s + cond e_a (+ the FP32 rounding for FIO_C64)
                                 REFINE  e_s rel_resid + cond e_a (+ FP64 rounding)
                                 PCG     cond^2 rel_resid + cond e_a
                                 GMRES   cond rel_resid + cond e_a                        */
} fio_solve_info;

/* Solve K fhat = u for nrhs columns.  u and out are complex128 device buffers
 * (N x nrhs, leading dimension ld) for every mode; dtype selects the precision
 * of the bulk factor applies: FIO_C64 (complex FP32 with FP32 accumulation,
 * accuracy won back by the FP64 residual of REFINE) or FIO_C128 (FP64 throughout).
 * If info is non-NULL the call synchronises hip_stream and fills it; with
 * tol > 0 the call synchronises once per iteration to test convergence.
 * Returns FIO_ERR_NOT_CONVERGED if tol > 0 was not met within maxit. */
fio_status fio_solve(fio_plan plan, const fio_solve_opts *opts, fio_dtype dtype,
                     const void *u, void *out, int64_t nrhs, int64_t ld,
                     fio_solve_info *info, void *hip_stream);

/* Several independent solves in one pass: instance i solves K_i fhat = u_i with
 * plans[i] (plans of any size, dimension and ranks) for nrhs[i] columns; u[i] and
 * out[i] are complex128 device buffers, column-major N_i x nrhs[i] with leading
 * dimension ld[i], as for fio_solve.  Every factor level runs as ONE launch for all
 * instances (section 7: the nodes of a tree level are independent, and so are the
 * instances): butterfly stage s of every instance's chain, skeletonization step k
 * of every instance's Gd sweep (counted from the finest level), the top-level
 * blocks; instances without that level sit it out.  Matrix-core tiles and
 * persistent-grid caps per level come from fio_multi_autotune for this group (plans
 * and batch widths), else from heuristics.  The results equal fio_solve's to
 * rounding (single-stage launches; no fused stage pairs).
 * opts: FIO_SOLVE_DIRECT, or FIO_SOLVE_REFINE with tol = 0 (maxit steps, no
 * synchronisation); spatial = 0.  1 <= n_inst <= 8; the plans must be distinct
 * (each instance uses its plan's workspace) and on one device.  Asynchronous; takes
 * every plan's lock for the call; capturable in a HIP graph (no allocation when
 * the workspaces are already sized, see the graph-capture rule above).
 * Errors: FIO_ERR_ARG, FIO_ERR_UNSUPPORTED (other modes or options). */
fio_status fio_solve_multi(int n_inst, const fio_plan *plans, const fio_solve_opts *opts, fio_dtype dtype,
                           const void *const *u, void *const *out, const int64_t *nrhs, const int64_t *ld,
                           void *hip_stream);

/* Autotuner of a multi-instance group (the plans and batch widths of a
 * fio_solve_multi call): per butterfly level of Kd^* (dtype) and Kd (complex128) the
 * matrix-core tiling and the grid (full, or persistent with 1024/2048/4096
 * workgroups), per skeletonization step the node kernel (fused with 64 or 32
 * columns, or LDS-staged) and the grid, each timed with HIP events (reps
 * repetitions) on hip_stream.  Later fio_solve_multi calls with the same plans (in
 * the same order), widths and dtype use the choices.  Synchronous; uses the plans'
 * workspaces as scratch.  Errors as fio_solve_multi. */
fio_status fio_multi_autotune(int n_inst, const fio_plan *plans, fio_dtype dtype, const int64_t *nrhs, int reps,
                              void *hip_stream);

typedef struct {
    int d, n, L, L_mid;            /* butterfly depth and middle level                 */
    int n_stages;                  /* butterfly stages of one apply (L + 3)            */
    int64_t bf_nnz;                /* nonzeros of all butterfly factors of Kd          */
    int max_rank_bf;               /* largest butterfly rank                           */
    int hif_levels;                /* skeletonization steps of Gd                      */
    int64_t hif_nnz;               /* nonzeros of all T, L^{-1}, M blocks of Gd        */
    int root_size;                 /* DOFs of the top-level block A_0                  */
    int max_rank_h;                /* largest off-diagonal rank of Sd                  */
    int64_t device_bytes;          /* device memory held by the factors                */
    int64_t workspace_bytes;       /* device workspace per right-hand side             */
    double build_seconds;          /* wall time of fio_build                           */
    int hif_shifted;               /* pivot blocks given a diagonal shift (see strict_hpd;
                                      not stored by fio_save)                          */
    double bf_seconds;             /* wall time of the butterfly construction (not stored) */
    int bf_device_levels;          /* butterfly levels decomposed on the device (not stored) */
    int hif_device_ids;            /* skeletonization IDs (large 2D cells and edges) computed
                                      on the device (not stored)                       */
    int hif_device_nodes;          /* large 2D skeletonization nodes whose Schur update,
                                      Cholesky factor, L^{-1} and M were formed on the
                                      device, plus 1 if A_0^{-1} was (not stored)      */
    /* Error estimates, measured on the device when the plan is built (and stored in
     * the plan file); 0 for a host-only plan.  The paper's e_a and e_s (section 6): */
    double e_a_est;                /* butterfly error ||K - Kd|| / ||K||: relative error of
                                      Kd v against K v (K summed directly from its entries)
                                      on 64 sampled rows, max over 4 Gaussian vectors       */
    double e_s_est;                /* inverse error: spectral radius of I - Gd Kd^* Kd by 12
                                      power iterations (4 Gaussian start vectors, FP64)     */
    double cond_est;               /* cond(Kd) = sqrt(lambda_max(Kd^* Kd) lambda_max(Gd)),
                                      each by 12 power iterations (Gd ~ (Kd^* Kd)^{-1})     */
    int64_t hif_sweep_nnz;         /* entries one sweep of Gd reads: T, M and the lower
                                      triangle of L^{-1} of every node (an apply of Gd makes
                                      two sweeps, up with T^*, L^{-1}, M and down with M^*,
                                      L^{-*}, T)                                          */
} fio_plan_stats_t;

fio_status fio_plan_stats(fio_plan plan, fio_plan_stats_t *out);

/* f = F^{-1} fhat = n^d F^* fhat (section 1: the normalised DFT F_jk =
 * n^{-d} exp(-2 pi i x_k . xi_j) with x_k = k/n and xi_j = j - n/2 per coordinate),
 * i.e. the spatial function whose Fourier coefficients a solve returns.  fhat and f
 * are device buffers of complex128, column-major N x nrhs with leading dimension ld,
 * natural lexicographic order of Omega (fhat) and X (f); f may alias fhat.  Computed
 * in FP64 by radix-4/2 passes on the GPU; the plan supplies d, n and workspace.
 * Asynchronous.  Errors: FIO_ERR_ARG, FIO_ERR_UNSUPPORTED (host-only plan). */
fio_status fio_inverse_dft(fio_plan plan, const void *fhat, void *f, int64_t nrhs, int64_t ld,
                           void *hip_stream);

/* Per-stage layout of the butterfly apply (for measurement): for stage s of the
 * forward apply, nnz of its blocks and the number of output blocks. */
fio_status fio_stage_info(fio_plan plan, int stage, int64_t *nnz, int64_t *n_out_blocks,
                          int *r_out, int *r_in, int *fan);

/* Apply the single factor `stage` of Kd (op = FIO_OP_K: stage s of eq_BFF_fact,
 * counted from V_L^* = 0 to U_L = L + 2) or of Kd^* (op = FIO_OP_KH: the adjoint
 * chain, V_L^*'s adjoint last) to coefficient vectors.  x and y are device
 * buffers in the library's internal layout: point-major, entry (e, b) of the
 * stage's input (n_in*r_in entries) or output (n_out*r_out entries) at
 * e*nrhs + b.  This is the kernel every apply runs, exposed for measurement.
 * Asynchronous; errors: FIO_ERR_ARG (stage or op out of range). */
fio_status fio_stage_apply(fio_plan plan, fio_op op, int stage, fio_dtype dtype, const void *x,
                           void *y, int64_t nrhs, void *hip_stream);

/* fio_stage_apply with one kernel variant forced (the codes of fio_tune_query;
 * -1: the tuned or default choice).  For tests and measurement: every variant
 * computes the same product (to rounding).  A matrix-core variant on a factor
 * whose blocks read more than four input blocks runs the vector kernel.
 * Asynchronous.  Errors: FIO_ERR_ARG (variant, stage or op out of range). */
fio_status fio_stage_apply_variant(fio_plan plan, fio_op op, int stage, fio_dtype dtype, int variant,
                                   const void *x, void *y, int64_t nrhs, void *hip_stream);

/* Apply the factors `stage` and `stage + 1` of Kd (FIO_OP_K) or Kd^* (FIO_OP_KH)
 * in one fused launch: consecutive butterfly factors of eq_BFF_fact couple closed
 * groups of at most fan^2 blocks, so one workgroup computes a group's
 * intermediate coefficients in LDS and applies the next factor to them.  x is
 * stage `stage`'s input and y stage `stage + 1`'s output, in the layout of
 * fio_stage_apply.  Uses the tuned column tiling for (dtype, nrhs) if there is
 * one.  Asynchronous.  Errors: FIO_ERR_ARG (stage out of range),
 * FIO_ERR_UNSUPPORTED (the pair's ranks exceed 32, the second factor's fan
 * exceeds 2, or its blocks do not form closed groups of at most four). */
fio_status fio_stage_pair_apply(fio_plan plan, fio_op op, int stage, fio_dtype dtype, const void *x,
                                void *y, int64_t nrhs, void *hip_stream);

/* The same two stages with one kernel variant forced: 1/2/3 the fused pair with
 * 16/32/64 columns per wave (3 for FIO_C64 only), 4 the stacked form (two sibling
 * blocks that read the same inputs computed as one operand of 16-row tiles: three
 * up to rank 24, four up to rank 32).  For tests and measurement.  Asynchronous.  Errors:
 * FIO_ERR_ARG (variant or stage out of range), FIO_ERR_UNSUPPORTED (the stages
 * cannot run fused, or not stacked). */
fio_status fio_stage_pair_apply_variant(fio_plan plan, fio_op op, int stage, fio_dtype dtype, int variant,
                                        const void *x, void *y, int64_t nrhs, void *hip_stream);

/* Apply the factors `stage`, `stage + 1` and `stage + 2` of Kd (FIO_OP_K) or Kd^*
 * (FIO_OP_KH) in one fused launch: three consecutive butterfly factors of eq_BFF_fact
 * (1D) couple closed groups of four blocks per factor; one workgroup computes a group's
 * two intermediate coefficient sets in LDS, the later two factors two sibling blocks
 * (equal input lists) at a time as one matrix-core operand.  x is stage `stage`'s input and y stage
 * `stage + 2`'s output, in the layout of fio_stage_apply.  For tests and
 * measurement; the autotuner uses it where it is faster.  Asynchronous.  Errors:
 * FIO_ERR_ARG (stage or op out of range), FIO_ERR_UNSUPPORTED (ranks above 32, a fan
 * of the later factors above 2, or groups that are not four blocks per factor with
 * two sibling pairs in the later two). */
fio_status fio_stage_triple_apply(fio_plan plan, fio_op op, int stage, fio_dtype dtype, const void *x, void *y,
                                  int64_t nrhs, void *hip_stream);

/* Column interpolative decomposition of one dense matrix on a device: the routine
 * the 2D skeletonization runs for its large stacked bases (section 4, the ID of
 * eq. ID_2d_bases), exposed for tests and measurement.  A(:, redund) ~= A(:, skel) T
 * where skel are the first rank pivots of a column-pivoted Householder QR that stops
 * before the first pivot whose trailing column norm is at most tol_rel times the
 * largest column norm of A (pivot: largest trailing norm, first among equals; a tall
 * A is first reduced to its triangular factor, which leaves every pivot unchanged up
 * to rounding;
 * exactly zero columns are redundant with zero coefficients).  A: host, complex128,
 * column-major m x n, leading dimension lda >= m, not modified.  Outputs, host: *rank;
 * perm[n] with skel = perm[0..rank) and redund = perm[rank..n); T complex128,
 * rank x (n - rank), column-major with leading dimension rank, in a buffer of t_cap
 * elements.  Synchronous.  Errors: FIO_ERR_ARG (sizes, null pointers, device
 * ordinal, t_cap < rank*(n - rank), with *rank set), FIO_ERR_UNSUPPORTED (m above
 * 2^31 - 1, or not enough device memory for A), FIO_ERR_DEVICE. */
fio_status fio_column_id(int device, int64_t m, int64_t n, const void *A, int64_t lda, double tol_rel, int *rank,
                         int *perm, void *T, int64_t t_cap);

/* The launches that an apply of Kd (FIO_OP_K) or Kd^* (FIO_OP_KH) makes at this
 * dtype and nrhs: launch j runs n_stages[j] (1, 2 or 3) consecutive factors from
 * first_stage[j] with kernel variant variant[j] (single factor: the codes of
 * fio_tune_query; fused pair: 1, 2, 3 for 16, 32, 64 columns per wave, 4 the stacked
 * form; three fused factors: 1).
 * *n_launch is always set; with cap = 0 only the count is returned, otherwise
 * the arrays (cap entries each, host memory) are filled.  Errors: FIO_ERR_ARG
 * (cap too small, null pointers). */
fio_status fio_chain_schedule(fio_plan plan, fio_op op, fio_dtype dtype, int64_t nrhs, int cap,
                              int *n_launch, int *first_stage, int *n_stages, int *variant);

/* Autotuner: for this dtype and batch width, time every kernel variant of every
 * butterfly stage (vector kernel; matrix-core tiles of 16 or 32 rows by 16, 32 or
 * 64 columns), of every fusable pair of consecutive stages (16, 32 or 64 columns per
 * wave, and the stacked form of sibling blocks), per skeletonization step the
 * LDS-staged kernel, the matrix-core GEMM path (16, 32 or 64 columns per tile) and
 * the fused per-node kernel (64 or 32 columns per workgroup), and the tiling of the
 * FP64 top-level block, with `reps` timed
 * repetitions each (HIP events on hip_stream); keep the fastest choices in the
 * plan, with the chain split into single and fused launches that minimises the
 * summed time.  Later applies with the same dtype and nrhs use them (other widths
 * use built-in heuristics).
 * Synchronous; the plan's workspace is used as scratch, so no other call on the
 * plan may run concurrently.  Errors: FIO_ERR_ARG, FIO_ERR_UNSUPPORTED (host-only). */
fio_status fio_autotune(fio_plan plan, fio_dtype dtype, int64_t nrhs, int reps, void *hip_stream);

/* Kernel variant used for stage `stage` of Kd (FIO_OP_K) or Kd^* (FIO_OP_KH) at
 * this dtype and nrhs: 0 vector kernel, 1..6 matrix-core tilings (16*MT rows x
 * 16*NT columns per wave: 1 MT1xNT4, 2 MT2xNT4, 3 MT1xNT2, 4 MT2xNT2, 5 MT1xNT1,
 * 6 MT2xNT1, 8 MT4xNT4, 9 MT4xNT2), 7 the small-batch kernel (fewer than 16
 * columns: 64 rows per workgroup, the k range split over its four waves), 10/11
 * matrix cores with the gathered input staged in LDS and shared by a workgroup's
 * four waves (one output block of up to 192 rows per workgroup, 64/32 columns),
 * 12/13/14 the tilings MT2xNT4, MT4xNT2, MT2xNT2 with three real products per
 * complex multiply-add instead of four. */
fio_status fio_tune_query(fio_plan plan, fio_op op, int stage, fio_dtype dtype, int64_t nrhs,
                          int *variant);

/* Device images a plan keeps (fio_plan_trim). */
typedef enum {
    FIO_KEEP_ALL = 0,          /* Kd and Kd^* in complex64 and complex128, Gd in both   */
    FIO_KEEP_REFINE_C64 = 1    /* what DIRECT and REFINE solves in complex64 use: Kd^* and
                                  Gd in complex64, Kd in complex128 (the residual)       */
} fio_keep;

/* Release the device images of the factors that `keep` does not list, to admit more
 * plans into HBM (FIO_KEEP_REFINE_C64 halves the factor memory: at 2D n = 256 from
 * 61 GB to about 30 GB).  One-way: later calls that need a released image (fio_apply
 * of Kd in complex64, complex128 solves, PCG or GMRES in complex64, ...) fail with
 * FIO_ERR_UNSUPPORTED; the error estimates, the host factors and fio_save are kept.
 * Synchronises the device.  Errors: FIO_ERR_ARG, FIO_ERR_UNSUPPORTED (host-only plan). */
fio_status fio_plan_trim(fio_plan plan, int keep);

/* 64-bit fingerprints of the plan's factors (its host copy, the source of every
 * device image and of fio_save): fp[0] the butterfly Kd (tree permutation and every
 * stage's sizes, indices and blocks, section 2), fp[1..K] the K skeletonization steps
 * of Gd (each node's index sets, T, L^-1 and M, section 4), fp[K+1] the top-level
 * block's indices and inverse.  Up to cap values are written; *count receives K + 2.
 * Builds are deterministic: the same problem built again on the same device gives
 * the same fingerprints, and a fingerprint that differs names the part of the
 * factors that does.
 * Synchronous, host only.  Errors: FIO_ERR_ARG (null plan or count, fp NULL with
 * cap > 0). */
fio_status fio_plan_fingerprints(fio_plan plan, uint64_t *fp, int cap, int *count);

/* Save the factors to a file / load them onto a device (device = -1: host only). */
fio_status fio_save(fio_plan plan, const char *path);
fio_status fio_load(const char *path, int device, fio_plan *out);

void fio_destroy(fio_plan plan);

/* Message of the last error on this thread ("" if none). */
const char *fio_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FIO_H */
