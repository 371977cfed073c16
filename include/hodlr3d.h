/*
 * hodlr3d.h -- C ABI of the MI355X HODLR3D matrix-vector library (libhodlr3d.so).
 *
 * The operator is the kernel matrix of an N-body problem in three dimensions,
 * K(i,j) = f(|r_i - r_j|) with K(i,i) = 0 (Kandappan, Gujjula, Ambikasaran,
 * "HODLR3D: Hierarchical matrices for N-body problems in three dimensions",
 * arXiv 2307.16303, Sec. 3.1, eq. (Laplace3D)), held in the HODLR3D format:
 * a balanced octree (Sec. 2.1), low-rank factors U V^T for every pair of
 * same-level boxes in each other's interaction list (Sec. 4, Definition of
 * HODLR3D admissibility and notation table), compressed by ACA (Sec. 4.1,
 * eq. (prank), Algorithm 1), and dense near-field leaf blocks evaluated on
 * the fly (Algorithm 2).
 *
 * Conventions shared by every entry point:
 *  - Every function returns an h3d_status; nothing throws across the ABI.
 *    On failure h3d_last_error() returns a message for the calling thread.
 *  - "device" pointers are HIP device memory of the current device; "host"
 *    pointers are ordinary process memory.  The caller owns every pointer it
 *    passes; the library owns the plan and everything reachable from it.
 *  - All device work is ordered on the hip_stream argument (a hipStream_t,
 *    NULL = the legacy default stream).  h3d_build synchronises that stream to
 *    read sizes back; the mat-vec calls are asynchronous and never synchronise.
 *  - A plan may be used by one stream at a time.
 */
#ifndef HODLR3D_H
#define HODLR3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define H3D_VERSION 1
#define H3D_MAX_LEVELS 11 /* levels 0..10 */

typedef struct h3d_plan h3d_plan;

typedef enum {
    H3D_OK = 0,
    H3D_EINVAL = 1,    /* bad argument (checked before any device work where possible) */
    H3D_ENOMEM = 2,    /* device or host allocation failed */
    H3D_EDEVICE = 3,   /* a HIP call failed */
    H3D_ENOTBUILT = 4, /* plan is NULL or was not built */
    H3D_EDEPTH = 5,    /* no depth <= max_depth gives leaves of at most leaf_size points */
    H3D_ENOTIMPL = 6   /* combination not provided by this build */
} h3d_status;

/* f(r); K(i,i) = 0 and f(0) := 0 for distinct coincident points. */
typedef enum {
    H3D_LAPLACE = 0, /* 1/(4 pi r): Green's function of the 3D Laplace equation */
    H3D_YUKAWA = 1,  /* exp(-kappa r)/r, kappa = kernel_param */
    H3D_INV_R4 = 2,  /* 1/r^4 (Sec. 5.1) */
    H3D_COS_R = 3    /* cos(kappa r)/r, kappa = kernel_param (Sec. 5.1 uses kappa = 1) */
} h3d_kernel;

/* Storage type of the low-rank factors.  ACA always runs in FP64. */
typedef enum {
    H3D_F64 = 0,
    H3D_F32 = 1,
    H3D_BF16_SCALED = 2 /* bfloat16 with one FP32 scale per factor of each block */
} h3d_dtype;

/* Optional device allocator (e.g. a framework's caching allocator).  alloc
 * returns NULL on failure; both are called on the build/mat-vec stream. */
typedef struct {
    void *(*alloc)(size_t bytes, void *hip_stream, void *ctx);
    void (*free)(void *ptr, size_t bytes, void *hip_stream, void *ctx);
    void *ctx;
} h3d_allocator;

enum {
    H3D_FLAG_KEEP_PIVOTS = 1, /* keep ACA pivots for h3d_export(H3D_EXPORT_PIVOTS) */
    H3D_FLAG_NO_AUTOTUNE = 2, /* keep the default launch shapes (no timing at build) */
    /* recompress every block's ACA factors in FP64 to the smallest rank r with
     * ||(s_{r+1}, ..., s_k)||_2 <= tol ||s||_2, s the singular values of U V^T
     * (QR of U and V, SVD of the small core); blocks of rank above 256 and
     * boxes of more than 4096 points are kept.  Excludes H3D_FLAG_KEEP_PIVOTS. */
    H3D_FLAG_TRUNCATE = 4,
    /* the paper's storage form (Sec. 4.1, eqs. (prank) and (LR); the low-rank
     * step of Algorithm 2): every block keeps only its ACA pivots sigma, tau
     * and the LU factors of K(sigma, tau), k^2 + 2k values instead of
     * (m + n) k; every product regenerates the entries of K(sigma, Y) and
     * K(X, tau) and applies K(X,tau) R^-1 L^-1 K(sigma,Y) x(Y).  Needs
     * factor_dtype H3D_F64 and ranks of at most 256 (H3D_ENOTIMPL otherwise;
     * max_rank caps them); excludes H3D_FLAG_TRUNCATE; not for batches.
     * h3d_export gives H3D_EXPORT_LU (and H3D_EXPORT_PIVOTS with
     * H3D_FLAG_KEEP_PIVOTS), not the explicit factors. */
    H3D_FLAG_LU_FORM = 8
};

typedef struct {
    int32_t kernel;        /* h3d_kernel */
    double kernel_param;   /* kappa for H3D_YUKAWA / H3D_COS_R */
    int32_t leaf_size;     /* N_max: a leaf holds at most this many points (>= 1) */
    double tol;            /* ACA tolerance eps, 0 < tol < 1 */
    int32_t factor_dtype;  /* h3d_dtype */
    int32_t max_rank;      /* rank cap per block; <= 0 means min(m, n) */
    int32_t max_depth;     /* deepest octree level allowed, 0..10 */
    double box_lo[3];      /* lower corner of the cube B ... */
    double box_side;       /* ... and its side; <= 0 selects the smallest enclosing cube */
    int64_t workspace_bytes; /* FP64 ACA workspace budget; <= 0 selects 4 GiB */
    int32_t flags;         /* H3D_FLAG_* */
} h3d_config;

typedef struct {
    int64_t n;
    int32_t depth;        /* L */
    int32_t factor_dtype;
    double box_lo[3];
    double box_side;
    int64_t n_far;                            /* admissible (V and W) blocks */
    int64_t n_near;                           /* ordered leaf pairs: self, E, F */
    int64_t far_per_level[H3D_MAX_LEVELS];
    int64_t rank_sum;                         /* = number of factor columns */
    int32_t rank_max;
    int64_t n_rank_capped;                    /* blocks stopped by max_rank */
    int64_t factor_entries;                   /* sum over blocks of (m + n) k */
    int64_t factor_bytes;                     /* stored bytes of U and V (+ scales); LU form:
                                                 LU factors, pivot rows, adjoint order */
    int64_t factor_bytes_per_level[H3D_MAX_LEVELS];
    int64_t near_pair_evals;                  /* sum over near leaf pairs of m n */
    int64_t device_bytes;                     /* all device memory held by the plan */
    double build_ms;                          /* wall time of h3d_build */
    double aca_ms;                            /* part of it spent in ACA kernels */
    int32_t tune_source;                      /* launch shapes: 0 defaults, 1 timed by the
                                                 tuner, 2 read from H3D_TUNE_CACHE */
} h3d_stats;

/* Fills *cfg with defaults: Laplace, leaf_size 64, tol 1e-8, FP64 factors, no
 * rank cap, max_depth 10, smallest enclosing cube, 4 GiB workspace. */
void h3d_config_init(h3d_config *cfg);

/*
 * Builds the HODLR3D representation of K on n points.
 *   points : device, n x 3 FP64, row-major (x, y, z per point); read only
 *            during the call, not retained.
 *   cfg    : host; validated before any device work.
 *   alloc  : host, may be NULL (then hipMalloc/hipFree are used).
 *   out    : receives the plan; NULL on any failure (nothing leaks).
 * Errors: H3D_EINVAL for n < 1, leaf_size < 1, tol outside (0,1), max_depth
 * outside 0..10, a bad dtype/kernel, non-finite coordinates or points outside
 * a given box; H3D_EDEPTH when max_depth levels cannot separate the points;
 * H3D_ENOMEM / H3D_EDEVICE from the device.
 */
h3d_status h3d_build(const double *points, int64_t n, const h3d_config *cfg,
                     const h3d_allocator *alloc, void *hip_stream, h3d_plan **out);

/*
 * y = K~ x (Algorithm 2): near-field leaf blocks plus the low-rank blocks of
 * every level.  x, y: device, n x nrhs column-major with leading dimensions
 * ldx, ldy >= n, in the caller's original point order; y is overwritten.
 * io_dtype is H3D_F64 or H3D_F32 (x and y share it).  x and y must not
 * overlap.  Deterministic: the same plan, input and nrhs give bitwise the same
 * output.
 */
h3d_status h3d_matvec(h3d_plan *plan, const void *x, void *y, int64_t nrhs, int64_t ldx,
                      int64_t ldy, int32_t io_dtype, void *hip_stream);

/* y = K~^T x with the same stored blocks: far blocks apply V (U^T x_t) to the
 * source box, near blocks are applied transposed.  Arguments as h3d_matvec. */
h3d_status h3d_matvec_adjoint(h3d_plan *plan, const void *x, void *y, int64_t nrhs,
                              int64_t ldx, int64_t ldy, int32_t io_dtype, void *hip_stream);

/*
 * Chooses the launch shapes of the factor streams for products with nrhs
 * right-hand sides (nrhs == 1, or any nrhs > 1 for the multi-column kernels)
 * by timing candidates on the plan's own factors on hip_stream.  h3d_build
 * runs it for nrhs == 1 unless H3D_FLAG_NO_AUTOTUNE is set.  With the
 * environment variable H3D_TUNE_CACHE naming a file, the choices are kept
 * there as JSON under a key made of the GPU architecture, the factor type,
 * one or several right-hand sides, the depth and per level the half-octave
 * buckets of the mean box size and mean rank; a plan with a stored key takes
 * the stored shapes (checked against its candidates) without timing
 * (h3d_stats.tune_source tells which happened).  The shapes only
 * change the order of floating-point sums inside a product, never which
 * entries are summed; a plan's products stay bitwise reproducible.
 */
h3d_status h3d_autotune(h3d_plan *plan, int64_t nrhs, void *hip_stream);

/*
 * A product captured once into a HIP graph and replayed.  h3d_graph_create
 * runs the product once eagerly on hip_stream (allocating the plan's scratch
 * and tables), then captures the same launch sequence, with these x and y
 * (device pointers, kept by the graph, owned by the caller) and sizes, on a
 * private capture stream.  h3d_graph_launch replays it on hip_stream: same
 * results, bitwise, as h3d_matvec / h3d_matvec_adjoint with the same
 * arguments.  The graph shares the plan's scratch and work tables: replays
 * and other products of the same plan must not overlap in time.  While a
 * graph of a plan exists, nothing it holds may move, so every call that would
 * reallocate them returns H3D_EINVAL and changes nothing: h3d_matvec,
 * h3d_matvec_adjoint, h3d_graph_create or h3d_matvec_batch (for a batch
 * member) with more right-hand sides than the plan's scratch was sized for,
 * h3d_autotune, and h3d_destroy of the plan (or of its batch).  Destroy the
 * graphs first.  h3d_graph_launch and h3d_graph_destroy on a destroyed graph
 * return H3D_EINVAL.
 */
typedef struct h3d_graph h3d_graph;
h3d_status h3d_graph_create(h3d_plan *plan, const void *x, void *y, int64_t nrhs, int64_t ldx,
                            int64_t ldy, int32_t io_dtype, int32_t adjoint, void *hip_stream,
                            h3d_graph **out);
/*
 * The same for a batch plan: the product of h3d_matvec_batch with these x
 * and y (host arrays of nprob device pointers, copied into the graph; the
 * buffers stay owned by the caller) captured once and replayed by
 * h3d_graph_launch.  The graph pins the scratch of every problem and the
 * batch's device tables: while it exists, h3d_matvec_batch with another nrhs,
 * products of a member with more right-hand sides and h3d_destroy of the
 * batch return H3D_EINVAL.  Replays give bitwise the eager result.
 */
h3d_status h3d_graph_create_batch(h3d_plan *batch, const void *const *x, void *const *y,
                                  int64_t nrhs, int32_t io_dtype, void *hip_stream,
                                  h3d_graph **out);
h3d_status h3d_graph_launch(h3d_graph *graph, void *hip_stream);
h3d_status h3d_graph_destroy(h3d_graph *graph);

/*
 * Multi-problem batching: independent operators, one per point cloud, all
 * with the same configuration, whose products run together: one launch per
 * phase of the product (gather, near field, stage 1 per launch shape, the
 * sums of split stage-1 columns, stage 2), each over the work items of every
 * problem.
 *   nprob  : number of problems (>= 1).
 *   points : host array of nprob device pointers; points[i] is n[i] x 3
 *            FP64 row-major, read only during the call.
 *   n      : host array of the nprob sizes (each >= 1).
 * cfg, alloc, hip_stream and the errors are those of h3d_build (a failure of
 * any problem fails the call and frees everything).  Every problem is built
 * as h3d_build builds it, tuned on its own factors unless
 * H3D_FLAG_NO_AUTOTUNE is set, except that its finest level is not fused
 * (the batch launches do not carry that form).  *out receives the batch
 * plan, which
 * accepts h3d_matvec_batch, h3d_batch_plan, h3d_batch_check, h3d_get_stats
 * (sums over the problems; depth and rank_max are maxima), the profiling
 * calls and h3d_destroy; other calls return H3D_EINVAL.
 */
h3d_status h3d_build_batch(int32_t nprob, const double *const *points, const int64_t *n,
                           const h3d_config *cfg, const h3d_allocator *alloc, void *hip_stream,
                           h3d_plan **out);

/*
 * y_i = K~_i x_i for every problem i of a batch plan (Algorithm 2 per
 * problem), in one launch per phase over all problems plus one small launch
 * per 32 problems that hands over the pointers.  x, y: host arrays of nprob device pointers;
 * x[i] and y[i] are n[i] x nrhs column-major with leading dimension n[i], in
 * problem i's original point order, of io_dtype (H3D_F64 or H3D_F32); y[i]
 * is overwritten and must not overlap x[i].  Asynchronous on hip_stream.
 * Each y[i] is bitwise the output of h3d_matvec on h3d_batch_plan(batch, i)
 * with the same x[i].  With nrhs >= 8 every problem's product is a set of
 * dense GEMMs on the matrix cores that fills the GPU by itself, so the
 * problems run back to back on the stream (the matrix-core path of
 * h3d_matvec) instead of in the phase launches.  Products of one batch
 * plan must not overlap in time.
 */
h3d_status h3d_matvec_batch(h3d_plan *batch, const void *const *x, void *const *y, int64_t nrhs,
                            int32_t io_dtype, void *hip_stream);

/* The plan of problem i (0 <= i < nprob) of a batch.  It belongs to the batch
 * (valid until h3d_destroy(batch); never pass it to h3d_destroy) and accepts
 * every single-operator call except h3d_autotune, which would change the
 * launch shapes the batch relies on (H3D_EINVAL). */
h3d_status h3d_batch_plan(h3d_plan *batch, int32_t i, h3d_plan **out);

/* Synchronises hip_stream and returns H3D_OK: the phases of a batch product
 * are ordered by the stream, with no waits inside a launch that could give
 * up.  (Kept so that callers written for a launch with device-side waits
 * stay valid; errors of the launches themselves are reported by the calls.) */
h3d_status h3d_batch_check(h3d_plan *batch, void *hip_stream);

h3d_status h3d_get_stats(const h3d_plan *plan, h3d_stats *out);

/* What h3d_export copies to host memory. */
typedef enum {
    H3D_EXPORT_PERM = 0,      /* int64[n]: sorted position -> original index */
    H3D_EXPORT_LEAF_OFF = 1,  /* int64[8^L + 1]: first sorted position of each leaf */
    H3D_EXPORT_FAR = 2,       /* int64[6][n_far]: level, t, s, m, n, rank */
    H3D_EXPORT_NEAR = 3,      /* int64[3][n_near]: t, s, relation (0 self, 1 F, 2 E) */
    H3D_EXPORT_FACTORS_U = 4, /* double[sum m k]: U_b (m x k, column-major), block order */
    H3D_EXPORT_FACTORS_V = 5, /* double[sum n k]: V_b (n x k, column-major), block order */
    H3D_EXPORT_PIVOTS = 6,    /* int64[2][sum k]: row then column pivots (box-local) */
    H3D_EXPORT_LU = 7         /* double[sum k^2], H3D_FLAG_LU_FORM plans: per block the
                               * k x k column-major LU of K(sigma, tau), L on and below
                               * the diagonal, the unit-diagonal R above it */
} h3d_export_what;

/* Copies one structure to host_buf.  With host_buf == NULL only *bytes is set
 * to the size needed; otherwise *bytes must hold the buffer size on entry and
 * receives the bytes written.  Factors are returned in FP64 (scales applied). */
h3d_status h3d_export(const h3d_plan *plan, int32_t what, void *host_buf, size_t *bytes);

/* Releases the plan (NULL is accepted).  H3D_EINVAL, with nothing released,
 * for a handle that is not a live plan (already destroyed), for a problem of
 * a batch (destroy the batch) and for a plan with live graphs.  Every other
 * entry point returns H3D_ENOTBUILT for a destroyed plan. */
h3d_status h3d_destroy(h3d_plan *plan);

/* Message of the last failure on the calling thread ("" if none). */
const char *h3d_last_error(void);

/*
 * Per-kernel timing of the mat-vec calls.  With profiling on, every kernel
 * launch of h3d_matvec / h3d_matvec_adjoint is bracketed by HIP events on the
 * stream it runs on.  h3d_profile_read synchronises those events and returns,
 * per kernel name, the launch count, the summed event time and the
 * algorithmic bytes and flops of one launch (the last one recorded).
 * enable >= 2 additionally launches each factor stream level by level (names
 * suffixed _L<level>), so that every level's stream rate can be read; the
 * result of the product is the same up to the summation order of stage 2.
 */
typedef struct {
    char name[48];
    int64_t launches;
    double total_ms;
    double bytes_per_launch;
    double flops_per_launch;
} h3d_kernel_profile;

h3d_status h3d_profile_enable(h3d_plan *plan, int32_t enable);
h3d_status h3d_profile_read(h3d_plan *plan, h3d_kernel_profile *out, int32_t capacity,
                            int32_t *count);
h3d_status h3d_profile_reset(h3d_plan *plan);

int32_t h3d_version(void);

/*
 * Iterative solve with the operator (Sec. 5.2, eqs. (IE) and (ILDiscrete)):
 * restarted GMRES(restart) for (diag I + scale K~) x = f, the form of the
 * collocation system of a second-kind integral equation (diag = 1 plus the
 * self-cell integral, scale = the cell volume, for the Laplace kernel times
 * 4 pi to turn 1/(4 pi r) into 1/r).  f, x: device, n doubles in the caller's
 * point order; x holds the initial guess on entry and the solution on exit.
 * Stops when the true relative residual |f - A x| / |f| falls below rtol
 * (checked at the end of every cycle; the Givens estimate ends a cycle early)
 * or after max_iter products.  Each iteration is one h3d_matvec plus
 * classical Gram-Schmidt with one reorthogonalisation; the Krylov basis (n x
 * (restart + 1) doubles) comes from the plan's allocator for the duration of
 * the call.  Dot products reduce in a fixed order: the same call gives
 * bitwise the same x.  info (host, may be NULL) receives the iterations, the
 * cycles, whether rtol was met and the final residuals.  Errors: H3D_EINVAL
 * for NULL or overlapping f and x, rtol outside (0, 1), restart outside
 * 1..256, max_iter < 1, non-finite diag or scale; those of h3d_matvec.
 * Synchronises hip_stream.
 */
typedef struct {
    int32_t iterations;   /* operator products inside the Arnoldi steps */
    int32_t cycles;       /* restart cycles completed */
    int32_t converged;    /* 1 when the true relative residual < rtol */
    double rel_residual;  /* true |f - A x| / |f| at exit */
    double est_residual;  /* last Givens estimate */
} h3d_solve_info;
h3d_status h3d_solve_gmres(h3d_plan *plan, double diag, double scale, const double *f, double *x,
                           double rtol, int32_t restart, int32_t max_iter, void *hip_stream,
                           h3d_solve_info *info);

/*
 * The exact dense product y_i = sum_{j != i} f(|p_i - p_j|) x_j over all n
 * points (eq. (Laplace3D) and the other kernels of h3d_kernel): the
 * right-hand side "exact up to roundoff" of the solve experiment, and a
 * reference for the compressed product.  points: device n x 3 FP64
 * row-major; x, y: device n doubles, same order as the points, not
 * overlapping.  O(n^2) kernel evaluations, one thread per row.  Errors:
 * H3D_EINVAL for n < 1, NULL pointers, overlap or an unknown kernel.
 */
h3d_status h3d_dense_matvec(const double *points, int64_t n, int32_t kernel,
                            double kernel_param, const double *x, double *y, void *hip_stream);

/*
 * For callers that cannot allocate device memory during a product (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * y = K~ x exactly as h3d_matvec computes it (bitwise the same result), with
 * every scratch buffer of the product taken from one static device array of
 * H3D_NOALLOC_SCRATCH_BYTES per GPU instead of plan memory.  The call makes no
 * hipMalloc, hipFree or other allocating call (profiling is off for it).
 * Arguments as h3d_matvec, with nrhs < 8 (one to seven right-hand sides).
 * The product needs 16 n nrhs bytes plus 8 bytes per stage-1 factor column
 * and right-hand side (each part rounded up to 256 bytes); more than the array
 * holds, or nrhs >= 8, gives H3D_EINVAL and launches nothing.  The array of a
 * GPU is held from the library's first use of that GPU until the process
 * ends.  Every call on one GPU shares it, whatever the plan: calls that
 * overlap in time on one GPU (other streams, other threads) race and give
 * wrong results; serialise them.  Nothing of one call's scratch is read by
 * the next (every value is written before it is read).
 */
#define H3D_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
h3d_status h3d_matvec_noalloc(h3d_plan *plan, const void *x, void *y, int64_t nrhs,
                              int64_t ldx, int64_t ldy, int32_t io_dtype, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* HODLR3D_H */
