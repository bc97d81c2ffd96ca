/*
 * pixelsne.h -- C ABI of the MI355X (gfx950) PixelSNE library.
 *
 * PixelSNE (Kim et al., arXiv:1611.02568) is Barnes-Hut t-SNE whose quadtree
 * is aligned to the pixels of the output screen (Section 4.1): positions are
 * kept in the pixel frame z with 0 <= z < r (Eq. 1-2), the tree has a fixed
 * depth L = log2 r with unit-pixel leaves, and after every gradient step the
 * positions are rescaled to fill the screen (Section 4.2) while a per-axis
 * scale factor keeps q identical to the unscaled embedding (Eq. 12-13).
 *
 * Conventions for every function below
 *   - Pointers documented as "device" must point to device memory of the
 *     current HIP device (hipMalloc or a torch CUDA tensor); "host" pointers to
 *     ordinary host memory.  All arrays are dense, row-major, C-contiguous.
 *   - The library never retains caller pointers beyond the call.
 *   - Work is enqueued on the context's stream (params.stream, or the null
 *     stream).  Functions that return values on the host synchronise that
 *     stream; the others are asynchronous unless stated.
 *   - Functions return a psne_status (0 = success) and never abort.  The
 *     init functions return NULL on failure.  pixelsne_last_error() gives a
 *     thread-local message for the last failure on the calling thread.
 *   - Arguments are validated on the host before any device work.
 *   - A context must be used from one host thread at a time.
 *
 * Precision paths (params.precision)
 *   PSNE_FP32: positions, velocities, gains, P values, the force
 *              arithmetic and the Barnes-Hut opening test are FP32 (the test
 *              optionally FP64, params.opening_fp64); the Z normaliser and
 *              the centre-of-mass sums are FP64.
 *   PSNE_FP64: everything FP64 (the paper keeps z in double, Section 4.1).
 */
#ifndef PIXELSNE_H
#define PIXELSNE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pixelsne_ctx pixelsne_ctx;

typedef enum {
    PSNE_OK = 0,
    PSNE_E_INVAL = -1,        /* bad argument (nothing was enqueued) */
    PSNE_E_NOMEM = -2,        /* device allocation failed */
    PSNE_E_DEVICE = -3,       /* HIP runtime error; the context is unusable */
    PSNE_E_NUMERIC = -4,      /* a non-finite value appeared */
    PSNE_E_STATE = -5,        /* context unusable after an earlier device error */
    PSNE_E_UNSUPPORTED = -6   /* valid request outside what the library supports */
} psne_status;

enum { PSNE_FP32 = 0, PSNE_FP64 = 1 };
/* Representative point of a cell: centre of mass of its members (Eq. 8), or
 * the geometric centre of the cell (Section 4.1, iteration-independent). */
enum { PSNE_COM_MASS = 0, PSNE_COM_CELL_CENTER = 1 };
/* The Barnes-Hut tree: the pixel-aligned P-Quadtree of PixelSNE (Section 4.1:
 * fixed depth log2 r, unit-pixel leaves), or Barnes-Hut-SNE's data-driven
 * D-Quadtree (Section 3.3, Eq. 9-10: the root spans the data, cells split
 * until each leaf holds one point; here on a 2^32 x 2^32 grid over the root,
 * levels 0..32, so points in one grid cell share a leaf), rebuilt every
 * iteration, walked by the same traversal.  PSNE_TREE_DATA requires
 * PSNE_COM_MASS. */
enum { PSNE_TREE_PIXEL = 0, PSNE_TREE_DATA = 1 };
/* Element type of the input matrix X. */
enum { PSNE_X_F32 = 0, PSNE_X_F64 = 1, PSNE_X_U8 = 2 };
/* Output frames of pixelsne_get_Y. */
enum {
    PSNE_FRAME_PIXEL = 0,   /* z, 0 <= z < r, float64 [n][2]            (Eq. 1-2) */
    PSNE_FRAME_SCREEN = 1,  /* clamp(floor(z), 0, r-1), int32 [n][2]     (Eq. 1)   */
    PSNE_FRAME_Y = 2        /* y = s * z per axis, float64 [n][2]        (Eq. 12)  */
};

typedef struct {
    uint32_t struct_size;     /* sizeof(pixelsne_params); set by pixelsne_default_params */
    int32_t k;                /* neighbours per row; 0 => floor(3 * perplexity) */
    double theta;             /* opening threshold of Eq. 11, 0 <= theta <= 0.99 [0.5] */
    int32_t exag_iters;       /* iterations with exaggerated P [250] */
    double exaggeration;      /* factor on P during those iterations [12] */
    double eta;               /* step size [200] */
    double mom0, mom1;        /* momentum before / after mom_switch [0.5, 0.8] */
    int32_t mom_switch;       /* [250] */
    double min_gain;          /* gain floor [0.01] */
    double eps;               /* screen-scaling epsilon of Section 4.2 [1e-6] */
    double init_sigma;        /* std of the generated initial embedding [1e-4] */
    uint64_t seed;            /* seed of the generated initial embedding [0] */
    int32_t precision;        /* PSNE_FP32 | PSNE_FP64 [PSNE_FP32] */
    int32_t com_mode;         /* PSNE_COM_MASS | PSNE_COM_CELL_CENTER [MASS] */
    int32_t x_dtype;          /* element type of X for pixelsne_init_ex [F32] */
    const double* Y_init;     /* optional device float64 [n][2] initial embedding
                                 (y frame); NULL => N(0, init_sigma^2) from seed */
    void* stream;             /* hipStream_t for all work; NULL => null stream */
    int32_t reorder_every;    /* renumber points internally by their Morton order after the
                                 first iteration and then after intervals that start at
                                 this many iterations and grow by reorder_growth (memory
                                 locality of the sparse attraction); 0 = never [100].
                                 Results are reported in the caller's numbering either
                                 way. */
    int32_t data_order;       /* pixelsne_init_ex only.  1: number the points internally by
                                 a Morton code of three random projections of X, so that
                                 neighbours in P sit close in memory before the embedding
                                 has formed; the first renumbering by the embedding then
                                 follows the early exaggeration.  0: start from the
                                 caller's order [1].  Results are reported in the caller's
                                 numbering either way. */
    int32_t graphs;           /* 1: pixelsne_step / _async replay one iteration as a HIP
                                 graph (captured on first use; no launch overhead per
                                 kernel); 0: launch the kernels one by one [1].  Results
                                 are identical. */
    double reorder_growth;    /* factor by which the interval between renumberings grows
                                 after each one, >= 1 (1: a fixed period) [2].  The layout
                                 moves less and less per iteration as the embedding
                                 settles, so the locality a renumbering restores decays
                                 more slowly the later it is made. */
    int32_t opening_fp64;     /* PSNE_FP32 path only.  0: the Barnes-Hut opening test of
                                 Eq. 11 and the distances run in FP32, operands rounded to
                                 FP32, each axis scaled by r_d = sqrt(b_d) rounded to FP32,
                                 and each operation rounded in the order
                                 (w*w)*(b1+b2) < th2*(dx*dx + dy*dy) with
                                 dx = z1*r1 - c1*r1, dy = z2*r2 - c2*r2, no fused
                                 multiply-add [0].  1: the test and the distances in FP64
                                 (the FP64 path always does this). */
    int32_t tree;             /* PSNE_TREE_PIXEL | PSNE_TREE_DATA [PIXEL] */
    int32_t knn_trees;        /* pixelsne_init_ex: 0 = exact brute-force kNN [0]; > 0 =
                                 the approximate kNN of pixelsne_knn_approx with this many
                                 random-projection trees (Section 4.3) */
    int32_t knn_leaf;         /* its leaf size, >= 2k + 2; 0 => 2k + 2 [0] */
    int32_t knn_explore;      /* its rounds of neighbour exploring [1] */
    int32_t attract_blocks_per_cu; /* blocks per compute unit of the persistent grid that
                                 runs the attraction's row sums on the second stream beside
                                 the tree and the traversal, 0..16 [2]; 0: none (the
                                 helper below then does all of them, after Z) */
    int32_t attract_help_blocks_per_cu; /* blocks per compute unit of the helper that
                                 joins the row sums on the context's stream once the
                                 traversal and Z are done, taking whatever row chunks the
                                 second stream has not started, 0..16 [3]; 0: no helper.
                                 At least one of the two is >= 1.  Results are identical
                                 for every setting. */
    int32_t attract_fork;     /* where the row sums fork onto the second stream:
                                 PSNE_FORK_SNAP after the snap pass (beside the sort, the
                                 cells and the walk), PSNE_FORK_CELLS after the cells (beside
                                 the walk only), PSNE_FORK_AUTO chosen on the device from
                                 measured iteration times: it starts after the cells, runs
                                 one iteration in 16 at the other point and keeps the
                                 faster of the last two [AUTO].  Results are identical for
                                 every setting. */
} pixelsne_params;

enum { PSNE_FORK_SNAP = 0, PSNE_FORK_CELLS = 1, PSNE_FORK_AUTO = 2 };

/* Fill *p with the defaults shown in brackets above. */
void pixelsne_default_params(pixelsne_params* p);

/*
 * Create a context: brute-force kNN of the rows of X (k = floor(3u) nearest by
 * squared Euclidean distance, self excluded, ties to the smaller index),
 * per-row Gaussian calibration to perplexity u (Section 3.2), the symmetric
 * sparse P = (P_cond + P_cond^T) / 2n in CSR (Section 3.3), an initial
 * embedding and its first screen scaling (Section 4.2).
 *   X          device, [n][D], float32 (pixelsne_init) or params.x_dtype
 *   n          number of points, 2 <= n < 2^27, k <= n - 1
 *   D          input dimension >= 1
 *   perplexity u > 0
 *   screen_w/h square power of two, 2 <= r <= 65536 (else PSNE_E_UNSUPPORTED)
 * X is read during the call only.  Returns NULL on failure.
 */
pixelsne_ctx* pixelsne_init(const float* X, int64_t n, int32_t D, double perplexity,
                            int32_t screen_w, int32_t screen_h);
pixelsne_ctx* pixelsne_init_ex(const void* X, int64_t n, int32_t D, double perplexity,
                               int32_t screen_w, int32_t screen_h, const pixelsne_params* p);

/*
 * Create a context from a caller-built P instead of X (Section 3.3 CSR):
 *   row_ptr device int64 [n+1], col device int32 [nnz] (each row ascending,
 *   no diagonal), val device float64 [nnz] (sums to 1).  Copied into the
 *   context; offsets and column ranges are checked on the device (NULL with
 *   PSNE_E_INVAL if they are not a CSR of n rows).  2 <= n < 2^27.  The
 *   initial embedding comes from params as for pixelsne_init_ex.
 */
pixelsne_ctx* pixelsne_init_with_P(int64_t n, int64_t nnz, const int64_t* row_ptr,
                                   const int32_t* col, const double* val, int32_t screen_w,
                                   int32_t screen_h, const pixelsne_params* p);

/*
 * Run n_iter >= 0 optimisation iterations.  Each iteration: snap to pixels and
 * Morton keys (Eq. 1-2), sort, build the P-Quadtree (Section 4.1), Barnes-Hut
 * repulsion and Z (Eq. 5, 11, 12), sparse attraction (Eq. 5), gains/momentum
 * step, screen-driven scaling (Section 4.2).  Enqueues the work and then
 * synchronises once to check for non-finite values (PSNE_E_NUMERIC).
 * The work is ordered on the context's stream (params.stream).  Inside an
 * iteration the attraction's row sums run on a second, non-blocking stream
 * that the context owns: it waits for the snap pass on the context's stream
 * and the update waits for it, so callers see one stream-ordered iteration.
 */
psne_status pixelsne_step(pixelsne_ctx* c, int32_t n_iter);

/* Enqueue the iterations without the final check (returns after enqueueing). */
psne_status pixelsne_step_async(pixelsne_ctx* c, int32_t n_iter);

/* Time spent in each pass, summed over the iterations of one call (ms),
 * measured with HIP events recorded between passes.  The attraction's row sums
 * run on a second stream of the context, at the same time as sort, tree,
 * traversal and Z; their time is measured on that stream, so the passes add
 * up to more than the iteration's wall time. */
typedef struct {
    double snap_ms;       /* pending screen scaling + pixel + Morton key */
    double sort_ms;       /* radix sort of (key, index) */
    double tree_ms;       /* cell numbering, counts and FP64 sums */
    double traverse_ms;   /* Barnes-Hut repulsion */
    double zsum_ms;       /* Z reduction */
    double attract_ms;    /* attraction row sums on the second stream, overlapping the
                             above (its launches after the snap pass and after the cells
                             added; one of them leaves at once) */
    double finalize_ms;   /* gains/momentum step and screen scaling factors, after the
                             attraction has finished */
    double reorder_ms;    /* internal renumbering (on the params.reorder_every /
                             reorder_growth schedule) */
    int32_t iterations;
} pixelsne_pass_times;

/* As pixelsne_step, also returning per-pass times.  Synchronises. */
psne_status pixelsne_step_profiled(pixelsne_ctx* c, int32_t n_iter, pixelsne_pass_times* out);

/* Write the current embedding to device memory `out` in the given frame
 * (types per PSNE_FRAME_*; [n][2], caller-owned).  Asynchronous. */
psne_status pixelsne_get_Y(const pixelsne_ctx* c, void* out, int32_t frame);

void pixelsne_destroy(pixelsne_ctx* c);
const char* pixelsne_last_error(void);

/* ---------------------------------------------------------------------- */
/* Introspection, state and parity hooks                                   */
/* ---------------------------------------------------------------------- */
typedef struct {
    int64_t n, nnz, n_nodes;  /* points, nonzeros of P, occupied cells (last tree) */
    int32_t r, L, k;          /* screen side, tree depth, neighbours per row */
    int32_t precision, com_mode;
    int32_t iteration;        /* iterations done */
    double s[2];              /* y units per pixel, per axis (beta_d = s_d^2, Eq. 13) */
    double Z;                 /* last Barnes-Hut normaliser */
    int64_t level_size[17];   /* occupied cells per level 0..L of the last tree */
    int32_t renumberings;     /* scheduled internal renumberings so far */
    int32_t fork_cells;       /* where the next iteration's row sums fork (attract_fork):
                                 1 after the cells, 0 after the snap pass */
    double fork_ms[2];        /* the fork-point tuner's iteration times, from the second
                                 stream's first launch to the end of the update, in ms:
                                 [0] forked after the snap pass, [1] after the cells
                                 (a moving average; under PSNE_FORK_AUTO the point not
                                 in use holds its last probe's mean); 0 = not measured
                                 since the context's start or the last set_state */
} pixelsne_stats;

/* Synchronises the stream. */
psne_status pixelsne_get_stats(const pixelsne_ctx* c, pixelsne_stats* out);

/*
 * Replace the optimiser state.  z, u, g: device [n][2] of the state type
 * (float32 for PSNE_FP32, float64 for PSNE_FP64), z in the pixel frame
 * (0 <= z < r), u the velocity in that frame, g the gains; u or g NULL =>
 * zeros / ones.  s: host double[2].  The iteration counter becomes
 * `iteration`, which sets the schedule (exaggeration, momentum) and the
 * internal renumbering schedule as they stand after that many iterations.
 * Synchronises.
 */
psne_status pixelsne_set_state(pixelsne_ctx* c, const void* z, const void* u, const void* g,
                               const double* s, int32_t iteration);
/* Read the state in the same layout (pending screen scaling applied). */
psne_status pixelsne_get_state(const pixelsne_ctx* c, void* z, void* u, void* g, double* s,
                               int32_t* iteration);

/*
 * Evaluate the pixel-frame gradient at the current state without stepping:
 *   B = alpha * A - R / Z  with A_i = sum_j p_ij w_ij (z_i - z_j),
 *   R_i = Barnes-Hut sum of m w^2 (z_i - c), Z = sum_i Z_i   (Eq. 5, 11, 12),
 * so that dC/dy_i,d = 4 s_d B_i,d.  Outputs are device arrays of the state type
 * ([n][2] for B, A, R) and may be NULL; Zi device float64 [n]; visits device
 * uint32 [n] (cells reached by each point's traversal); used device uint32 [n]
 * (cells that entered R_i and Z_i); Z host double.
 * Also leaves the tree of the current state for pixelsne_export_tree.
 * Synchronises the stream.
 */
psne_status pixelsne_gradient(pixelsne_ctx* c, double alpha, void* B, void* A, void* R,
                              double* Zi, uint32_t* visits, uint32_t* used, double* Z);

/*
 * Export the tree built by the last pixelsne_gradient / iteration.
 *   level_size host int64 [L+1] (always written)
 *   keys   device uint32 [n]   Morton keys in sorted order
 *   perm   device uint32 [n]   point index at each sorted position
 *   prefix device uint32 [n_nodes], count device uint32 [n_nodes],
 *   sum    device float64 [n_nodes][2]: cells of level 0, then 1, ..., L, each
 *          level ascending by Morton prefix (key >> 2(L - level)).
 * Pass NULL device pointers to query level_size only.  Synchronises.
 */
psne_status pixelsne_export_tree(const pixelsne_ctx* c, int64_t* level_size, uint32_t* keys,
                                 uint32_t* perm, uint32_t* prefix, uint32_t* count,
                                 double* sum);

/*
 * Export the data-driven tree (PSNE_TREE_DATA) built by the last
 * pixelsne_gradient / iteration; PSNE_E_INVAL for the pixel tree.
 *   level_size host int64 [33] (always written), levels 0..32
 *   keys   device uint64 [n]   64-bit grid Morton keys in sorted order
 *   perm   device uint32 [n]   point index at each sorted position
 *   prefix device uint64 [n_nodes] (key >> 2 (32 - level)), count device
 *   uint32 [n_nodes], sum device float64 [n_nodes][2]: cells of level 0, 1,
 *   ..., 32, each level ascending by prefix.
 * Pass NULL device pointers to query level_size only.  Synchronises.
 */
psne_status pixelsne_export_tree64(const pixelsne_ctx* c, int64_t* level_size, uint64_t* keys,
                                   uint32_t* perm, uint64_t* prefix, uint32_t* count,
                                   double* sum);

/* Export P: *nnz (host) always; row_ptr int64 [n+1], col int32 [nnz],
 * val float64 [nnz] device pointers may be NULL.  Synchronises. */
psne_status pixelsne_export_P(const pixelsne_ctx* c, int64_t* nnz, int64_t* row_ptr,
                              int32_t* col, double* val);

/*
 * KL(P || Q) of Eq. (4) for the current embedding with the exact normaliser
 * Z = sum over ordered pairs i != j of w_ij (O(n^2) pairs on the GPU; pair
 * terms in FP32 summed in FP64) and sum over the nonzeros of p (ln p - ln w_ij)
 * in FP64; P as stored (un-exaggerated).  *kl host double.  Synchronises.
 */
psne_status pixelsne_kl(const pixelsne_ctx* c, double* kl);

/*
 * pixelsne_kl for callers that cannot allocate device memory (serving loops
 * and harnesses that forbid hipMalloc between steps): the same kernels and the
 * same result, with the per-block partial sums in a fixed array of the library
 * (73,731 doubles, 576 KiB, one copy per device, held until the process ends)
 * instead of a buffer allocated for the call.  No device or host allocation.
 * Supports n <= 2^24 (PSNE_E_UNSUPPORTED above).  The context's device must be
 * current.  All calls on one device share the array, so calls that overlap on
 * a device (several host threads, or several streams) race; calls in
 * sequence do not.  *kl host double.  Synchronises the context's stream.
 */
psne_status pixelsne_kl_noalloc(const pixelsne_ctx* c, double* kl);

/*
 * Refinement of a warm-started embedding with the plain method as fallback
 * (the learned placement's last stage; an addition to the method).  Runs
 * ordinary iterations (pixelsne_step) of the context in chunks of check_every
 * and evaluates the exact-Z KL of Eq. (4) (pixelsne_kl) after each chunk;
 * stops as soon as KL <= kl_target or after max_iters iterations.
 * refine_iters is the refinement budget: when the target is not met within
 * it, the iterations simply continue as the plain method's (fallback = 1).
 * The context is typically created with Y_init from pixelsne_mlp_place,
 * exag_iters = 0 and mom_switch = 0.
 *   kl_target    finite; check_every >= 1; 0 <= refine_iters <= max_iters.
 *   out          host; iterations run, whether the target was reached,
 *                whether the fallback was taken, KL before and after, and the
 *                GPU time of the iterations alone (HIP events; the KL checks
 *                are not included).
 * Synchronises after every chunk.  PSNE_E_NUMERIC on non-finite positions.
 */
typedef struct {
    int32_t iterations;
    int32_t reached;          /* 1: KL <= kl_target at return */
    int32_t fallback;         /* 1: more than refine_iters iterations were needed, or the
                                 target was not reached */
    double kl_start, kl;      /* exact-Z KL before the first and after the last chunk */
    double iter_ms;           /* GPU time of the iterations (ms) */
} pixelsne_refine_result;

psne_status pixelsne_refine(pixelsne_ctx* c, double kl_target, int32_t check_every,
                            int32_t refine_iters, int32_t max_iters,
                            pixelsne_refine_result* out);

/*
 * The 32 nearest neighbours of every point in the current 2-D embedding
 * y = s * z (distance b1 dz1^2 + b2 dz2^2 with b = s^2, FP64, self excluded,
 * ties to the smaller index), by brute force on the GPU.
 *   idx device int32 [n][32], caller order, ascending by distance.
 * Requires n > 32.  Synchronises.
 */
psne_status pixelsne_knn2d(const pixelsne_ctx* c, int32_t* idx);

/*
 * Neighbourhood precision of Eq. (14) for each k in ks:
 *   out[q] = (1 / (k N)) sum_i |N_D^(k)(i) intersect N_d^(k)(i)|,
 * where N_D^(k)(i) is the first k entries of row i of hi_knn (the caller's
 * high-dimensional neighbours, device int32 [n][k_hi], caller order, distinct
 * entries, nearest first, e.g. from pixelsne_knn) and N_d^(k)(i) the first k
 * of pixelsne_knn2d.  ks host int32 [nk] with 1 <= ks[q] <= min(k_hi, 32),
 * 1 <= nk <= 64; out host double [nk].  Allocates scratch of 128 n bytes for
 * the call.  Requires n > 32.  Synchronises.
 */
psne_status pixelsne_neighborhood_precision(const pixelsne_ctx* c, const int32_t* hi_knn,
                                            int32_t k_hi, const int32_t* ks, int32_t nk,
                                            double* out);

/* ---------------------------------------------------------------------- */
/* Setup stages as standalone calls (all device pointers, stream-ordered)  */
/* ---------------------------------------------------------------------- */
/*
 * Brute-force k nearest neighbours of every row of X among all rows
 * (squared Euclidean, self excluded, ties to the smaller index).
 *   X device [n][D] of x_dtype; idx device int32 [n][k], d2 device float64
 *   [n][k] ascending (exact distances recomputed in FP64).  Requires
 *   1 <= k <= min(n - 1, 256).  Synchronises (returns after completion).
 */
psne_status pixelsne_knn(const void* X, int64_t n, int32_t D, int32_t x_dtype, int32_t k,
                         int32_t* idx, double* d2, void* stream);

/*
 * Approximate k nearest neighbours (Section 4.3, the K-NNG of LargeVis):
 * `trees` random-projection trees (a range of more than leaf_size points
 * splits by the hyperplane halfway between two of its points drawn from the
 * seed; cut in the middle when a side would get fewer than k + 1 points)
 * give each point its leaf mates as candidates; then `explore` rounds
 * replace each point's list by the best k of its list and its neighbours'
 * lists.  Lists keep the best k by (squared distance in FP64, index),
 * distinct, self excluded; all decisions in FP64, so the result is a
 * deterministic function of X and the seed.
 *   X device [n][D] of x_dtype; idx device int32 [n][k], d2 device float64
 *   [n][k] ascending.  1 <= k <= min(n - 1, 256), trees >= 1, explore >= 0,
 *   leaf_size >= 2k + 2 (0 => 2k + 2), n < 2^31.  Allocates its work
 *   buffers (about 24 n k bytes).  Synchronises.
 */
psne_status pixelsne_knn_approx(const void* X, int64_t n, int32_t D, int32_t x_dtype, int32_t k,
                                int32_t trees, int32_t leaf_size, int32_t explore,
                                uint64_t seed, int32_t* idx, double* d2, void* stream);

/*
 * Per-row Gaussian calibration (Section 3.2): for each row find b_i with
 * entropy of p_{j|i} = exp(-b_i (d2_ij - min_j d2_ij)) / sum equal to ln(u)
 * (|H - ln u| < 1e-5, at most 200 evaluations, start b = 1, double/halve
 * until bracketed, then bisect).
 *   d2 device float64 [n][k]; P device float64 [n][k]; beta device float64 [n]
 *   (may be NULL).  Asynchronous.
 */
psne_status pixelsne_perplexity(const double* d2, int64_t n, int32_t k, double perplexity,
                                double* P, double* beta, void* stream);

/* ---------------------------------------------------------------------- */
/* Learned placement network                                               */
/* ---------------------------------------------------------------------- */
/*
 * A small MLP maps a point x (dimension d_in) to its screen position z / r in
 * [0,1)^2 of a converged embedding: Linear(d_in,h1) - GELU - Linear(h1,h2) -
 * GELU - Linear(h2,2), GELU(x) = x Phi(x).  It places new points, or all
 * points of a new run, before a few ordinary iterations refine them.  Matrix
 * products take bfloat16 operands (inputs, weights and activations rounded to
 * nearest even) on the MFMA units and accumulate in FP32; master weights and
 * the Adam moments are FP32.  Inputs are standardised per feature first.
 * Parameters and gradients are flat FP32 vectors laid out as
 * W1 [d_in][h1], b1 [h1], W2 [h1][h2], b2 [h2], W3 [h2][2], b3 [2] (row-major).
 * X device float32 [n][d_in]; Y01 device float32 [n][2].  All calls are
 * stream-ordered on the stream given at creation and synchronise it before
 * returning.  Weights start He-normal from the seed, biases at zero.
 */
typedef struct pixelsne_mlp pixelsne_mlp;

pixelsne_mlp* pixelsne_mlp_create(int32_t d_in, int32_t h1, int32_t h2, uint64_t seed,
                                  void* stream);
void pixelsne_mlp_destroy(pixelsne_mlp* m);
int64_t pixelsne_mlp_num_params(const pixelsne_mlp* m);
/* theta: device float32 [num_params] */
psne_status pixelsne_mlp_set_params(pixelsne_mlp* m, const float* theta);
psne_status pixelsne_mlp_get_params(const pixelsne_mlp* m, float* theta);
/* standardisation x^ = (x - mean) * inv_std; device float32 [d_in] each */
psne_status pixelsne_mlp_set_norm(pixelsne_mlp* m, const float* mean, const float* inv_std);
/* mean and 1 / population std of each feature of X (FP64 accumulation) */
psne_status pixelsne_mlp_fit_norm(pixelsne_mlp* m, const float* X, int64_t n);
/* loss = (1/n) sum_i |MLP(x_i) - y_i|^2 over one batch of n <= 2^20 rows and its
 * gradient (device float32 [num_params], may be NULL); loss host double. */
psne_status pixelsne_mlp_grad(pixelsne_mlp* m, const float* X, const float* Y01, int64_t n,
                              float* grads_out, double* loss);
/* Adam (beta 0.9 / 0.999, eps 1e-8) over `epochs` passes of shuffled full
 * batches; the mean loss of the last epoch goes to *last_epoch_loss. */
psne_status pixelsne_mlp_train(pixelsne_mlp* m, const float* X, const float* Y01, int64_t n,
                               int32_t epochs, int32_t batch, float lr, double* last_epoch_loss);
/* Y01_out device float32 [n][2] */
psne_status pixelsne_mlp_forward(pixelsne_mlp* m, const float* X, int64_t n, float* Y01_out);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected with the
 * network's own step count, which pixelsne_mlp_train advances too) with a
 * caller-supplied gradient: device float32 [num_params] in the flat layout
 * above, e.g. a gradient averaged over several devices. */
psne_status pixelsne_mlp_adam_step(pixelsne_mlp* m, const float* grad, float lr);
/* Initial embedding for pixelsne_init_ex's Y_init: y = clamp(MLP(x), 0,
 * 1 - 2^-24) * screen * s per axis, s = y units per pixel of the run the
 * network was trained on (host double[2]).  Y_out device float64 [n][2]. */
psne_status pixelsne_mlp_place(pixelsne_mlp* m, const float* X, int64_t n, int32_t screen,
                               const double* s, double* Y_out);

/* ---------------------------------------------------------------------- */
/* 3-D embeddings                                                          */
/* ---------------------------------------------------------------------- */
/*
 * PixelSNE in three dimensions (Section 1 notes that the method carries over
 * to 3-D embeddings): the screen becomes a cube of r x r x r voxels, the
 * P-Quadtree an octree of fixed depth L = log2 r whose leaves are single
 * voxels, the Morton key interleaves the voxel coordinates x, y, z in bits
 * 3b, 3b+1, 3b+2 (3L bits), and every per-axis step of Sections 4.1-4.2 and
 * Eq. 12-13 runs over three axes: the opening test of Eq. 11 compares
 * w^2 (b1 + b2 + b3) with theta^2 (b1 dz1^2 + b2 dz2^2 + b3 dz3^2),
 * b_d = s_d^2, and the screen scaling rescales each axis to [0, r).
 * Everything is FP64 (positions, velocities, gains, P, forces and the
 * opening test) and cells are represented by their centre of mass (Eq. 8).
 * Positions and all [n][3] arrays are float64, row-major, in the caller's
 * numbering.
 *
 * pixelsne_params fields read: k, theta, exag_iters, exaggeration, eta, mom0,
 * mom1, mom_switch, min_gain, eps, init_sigma, seed, x_dtype, Y_init (device
 * float64 [n][3] in the y frame, or NULL => N(0, init_sigma^2 I) from seed),
 * stream, knn_trees, knn_leaf, knn_explore.  precision must be PSNE_FP64,
 * com_mode PSNE_COM_MASS and tree PSNE_TREE_PIXEL (else PSNE_E_UNSUPPORTED);
 * the layout fields (reorder_*, data_order, graphs, opening_fp64,
 * attract_blocks_per_cu, attract_help_blocks_per_cu) are not read.
 * r is a power of two in [2, 1024]; 2 <= n <= 2^25.
 */
typedef struct pixelsne3_ctx pixelsne3_ctx;

/* P from X exactly as pixelsne_init_ex (kNN, perplexity, symmetrisation),
 * then the initial 3-D embedding and its first scaling.  NULL on failure. */
pixelsne3_ctx* pixelsne3_init_ex(const void* X, int64_t n, int32_t D, double perplexity,
                                 int32_t r, const pixelsne_params* p);
/* From a caller-built P, as pixelsne_init_with_P (copied and checked). */
pixelsne3_ctx* pixelsne3_init_with_P(int64_t n, int64_t nnz, const int64_t* row_ptr,
                                     const int32_t* col, const double* val, int32_t r,
                                     const pixelsne_params* p);
void pixelsne3_destroy(pixelsne3_ctx* c);

/* n_iter >= 0 iterations: voxel keys, sort, octree, Barnes-Hut repulsion and
 * Z, sparse attraction, gains/momentum step, per-axis screen scaling.
 * Synchronises at the end and checks for non-finite positions
 * (PSNE_E_NUMERIC). */
psne_status pixelsne3_step(pixelsne3_ctx* c, int32_t n_iter);

/* The embedding in a PSNE_FRAME_*: z (float64 [n][3]), voxels
 * clamp(floor(z), 0, r-1) (int32 [n][3]) or y = s * z (float64 [n][3]);
 * device, caller-owned.  Asynchronous. */
psne_status pixelsne3_get_Y(const pixelsne3_ctx* c, void* out, int32_t frame);

/* Replace / read the optimiser state: z, u, g device float64 [n][3] (z in the
 * voxel frame, 0 <= z < r; u or g NULL on set => zeros / ones), s host
 * double[3], the iteration counter (sets the exaggeration and momentum
 * schedule).  Both synchronise. */
psne_status pixelsne3_set_state(pixelsne3_ctx* c, const double* z, const double* u,
                                const double* g, const double* s, int32_t iteration);
psne_status pixelsne3_get_state(const pixelsne3_ctx* c, double* z, double* u, double* g,
                                double* s, int32_t* iteration);

/* The voxel-frame gradient at the current state without stepping, as
 * pixelsne_gradient in three dimensions: B = alpha A - R / Z, outputs device
 * float64 [n][3] (B, A, R), Zi float64 [n], visits uint32 [n] (cells reached
 * by each point's walk), Z host; any may be NULL.  Leaves the octree for
 * pixelsne3_export_tree.  Synchronises. */
psne_status pixelsne3_gradient(pixelsne3_ctx* c, double alpha, double* B, double* A, double* R,
                               double* Zi, uint32_t* visits, double* Z);

/* The octree of the last gradient / iteration: level_size host int64 [L+1]
 * (always written); keys device uint32 [n] (Morton keys in sorted order),
 * perm uint32 [n] (point at each sorted position), prefix uint32 [n_nodes]
 * (key >> 3 (L - level)), count uint32 [n_nodes], sum float64 [n_nodes][3]:
 * level 0, then 1, ..., L, each ascending by prefix.  NULL device pointers =>
 * level sizes only.  Synchronises. */
psne_status pixelsne3_export_tree(const pixelsne3_ctx* c, int64_t* level_size, uint32_t* keys,
                                  uint32_t* perm, uint32_t* prefix, uint32_t* count,
                                  double* sum);

/* KL(P || Q) of Eq. 4 for the current 3-D embedding with the exact normaliser
 * (O(n^2) pairs; pair terms in FP32 summed in FP64; the P terms in FP64).
 * Allocates partial sums for the call.  *kl host.  Synchronises. */
psne_status pixelsne3_kl(const pixelsne3_ctx* c, double* kl);

#ifdef __cplusplus
}
#endif
#endif /* PIXELSNE_H */
