/*
 * sigkernel.h -- C ABI of the MI355X (gfx950) PDE signature kernel library.
 *
 * Paper: Salvi, Cass, Foster, Lyons, Yang, "The Signature Kernel is the
 * solution of a Goursat PDE", arXiv 2006.14794.
 *
 * The library evaluates, for pairs of piecewise-linear paths x (lx points) and
 * y (ly points) in R^d, the explicit finite-difference scheme of Section 3.1,
 * eq. (explicit_finite_diff), on the dyadic grid P_lambda of definition
 * (fintite_diff): the coarse increment inner products <x_{p+1}-x_p,
 * y_{q+1}-y_q> (Section 3.1, piecewise-linear case), refined by the factor
 * 2^{-2 lambda} (remark after eq. (explicit_finite_diff)), and swept from the
 * boundary values 1 (eq. (PDE), Theorem thm:PDE) to the terminal corner.
 * Rows of the fine grid follow x, columns follow y; the fine grid has
 * (2^lambda (lx-1) + 1) x (2^lambda (ly-1) + 1) nodes.
 *
 * Dyadic order: any lambda >= 0 with 2^lambda (len - 1) <= 2^20 for every
 * path of both batches (else SK_ERR_ORDER); the lifted calls and the
 * corrector's fallback take lambda <= 3.  The sweeps are compiled for orders
 * 0..3; a higher order runs at order 3 on the increments split into
 * 2^(lambda - 3) equal parts, whose fine cells and coefficients are exactly
 * those of P_lambda (each part is the increment times a power of two).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All point and output buffers are DEVICE memory owned by the caller.  The
 *    library allocates no device memory: scratch space comes from the caller's
 *    workspace (size from sigkernel_workspace_bytes).  Nothing is retained
 *    after a call returns.
 *  - Calls enqueue work on `stream` (a hipStream_t, NULL = default stream) and
 *    return immediately.  The status reports argument validation and launch
 *    only; kernel faults surface at the next synchronisation.
 *  - On any error nothing is enqueued and outputs are left untouched.
 *  - NaN/Inf inputs are not scanned: they propagate into the outputs of the
 *    pairs that contain them and into no other pair.
 *  - A path with one point has no increments: its kernel with any path is 1
 *    (the boundary value) and its gradient is 0.
 *  - Entry points are reentrant; calls that write the same output or
 *    workspace concurrently race.
 */
#ifndef SIGKERNEL_H
#define SIGKERNEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sk_status;
enum {
    SK_OK = 0,
    SK_ERR_NULL = -1,        /* a required pointer is NULL                         */
    SK_ERR_SHAPE = -2,       /* d < 1, a length < 1, dims or counts inconsistent   */
    SK_ERR_ORDER = -3,       /* dyadic order < 0, or 2^lambda (len - 1) > 2^20      */
    SK_ERR_WORKSPACE = -4,   /* workspace NULL or smaller than required             */
    SK_ERR_FLAGS = -5,       /* unknown or incompatible flag bits                   */
    SK_ERR_HIP = -6,         /* a HIP launch failed                                 */
    SK_ERR_UNSUPPORTED = -7, /* shape outside the compiled kernel configurations    */
    SK_ERR_STATE = -8,       /* not allowed in the stream's current state (a call
                                that synchronises, issued under graph capture)      */
    SK_ERR_VALUE = -9        /* a parameter outside its domain (an unknown static
                                kernel, a bandwidth that is not positive and finite) */
};

/*
 * A batch of paths in R^dim, float32, row-major.
 *  - Uniform batch (offsets == NULL): points is [n_paths][len][dim].
 *  - Ragged batch (offsets != NULL): offsets is a DEVICE array of n_paths+1
 *    int64, offsets[0] == 0, non-decreasing; path k is points
 *    [offsets[k], offsets[k+1]) of points [offsets[n_paths]][dim].  `len`
 *    must then be an upper bound of every path length; a pair whose path
 *    breaks that bound or has length < 1 gets a NaN output.
 */
typedef struct sk_paths {
    const float *points;
    const int64_t *offsets;
    int64_t n_paths;
    int32_t len;
    int32_t dim;
} sk_paths;

/*
 * Precision: path points and outputs are float32; the increments and their
 * inner products are formed in float32 (FMA), and the sweep state -- every
 * node value of the scheme -- is IEEE double.
 *
 * Channels: any dim >= 1 for sigkernel_pair / sigkernel_gram / sigkernel_mmd2
 * values.  Up to 16 channels the sweeps form the inner products on the fly
 * from increments held in registers; wider batches form the increment Gram
 * on the matrix cores first (float32 sums) and sweep from it, with x paths
 * of at most 2048 fine rows (2^lambda (x.len - 1) <= 2048; else
 * SK_ERR_UNSUPPORTED).  Gradients (sigkernel_gram_backward, the MMD
 * gradient), the lifted kernels and the corrector take at most 16 channels.
 */

/* flags */
enum {
    SK_SYMMETRIC = 1u << 0,   /* gram only: X and Y are the same batch; solve a <= b and mirror */
    SK_NO_DIAG   = 1u << 1,   /* gram only, with SK_SYMMETRIC: write 0 on the diagonal         */
    SK_MMD2_GRAD = 1u << 2,   /* mmd2 only: also write the gradient with respect to X          */
    SK_GRAM_BF16 = 1u << 3,   /* pair / gram: increments rounded to bfloat16 before the inner
                                 products (16-bit inputs, float32 accumulation)                */
    SK_GRAM_F16  = 1u << 4,   /* pair / gram: the same with IEEE half                          */
    SK_IMPLICIT  = 1u << 5    /* pair / gram: the implicit scheme of the remark after eq.
                                 (explicit_finite_diff) -- the cell integral estimated with all
                                 four corners, solved for the new corner:
                                 K11 = (K10 + K01)(1 + c/4)/(1 - c/4) - K00, c the fine cell's
                                 coefficient.  A cell with c = 4 has no solution (inf/NaN).  No
                                 gradient (sigkernel_gram_backward rejects the flag)          */
};

/*
 * sigkernel_pair -- independent pairs (Section 3.1, eq. (explicit_finite_diff)).
 *   out[k] = k_hat(x_k, y_k) at the terminal corner of P_lambda, k < n_paths.
 * x->n_paths must equal y->n_paths and x->dim == y->dim.
 * out: DEVICE float[n_paths].  ws: DEVICE workspace of at least
 * sigkernel_workspace_bytes(SK_OP_PAIR, ...) bytes.
 */
sk_status sigkernel_pair(const sk_paths *x, const sk_paths *y, int32_t dyadic_order,
                         uint32_t flags, float *out, void *ws, size_t ws_bytes,
                         void *stream);

/*
 * sigkernel_gram -- Gram matrix of two batches (Section 3.1 scheme applied to
 * every pair; the Gram matrices are what the applications of Section 5 consume).
 *   K[a * Y->n_paths + b] = k_hat(X_a, Y_b).
 * K: DEVICE float[X->n_paths * Y->n_paths], row-major.
 */
sk_status sigkernel_gram(const sk_paths *X, const sk_paths *Y, int32_t dyadic_order,
                         uint32_t flags, float *K, void *ws, size_t ws_bytes,
                         void *stream);

/*
 * sigkernel_gram_noalloc -- sigkernel_gram (same batches, flags, output and
 * errors) for callers that cannot allocate device memory or provide a
 * workspace: code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation.  The workspace is a static device array of
 * sigkernel_gram_noalloc_max_bytes() bytes (64 MiB) inside the library, one
 * per GPU, held until the process ends; the call allocates nothing.
 *  - A problem whose workspace (sigkernel_workspace_bytes(SK_OP_GRAM, ...))
 *    exceeds that size gives SK_ERR_WORKSPACE, with nothing enqueued.
 *  - stream must belong to the current device; the array's address on the
 *    device is looked up on the first call there (SK_ERR_HIP on failure).
 *  - Every call on one GPU uses the same array: calls that overlap on one
 *    GPU (concurrent streams, or threads sharing a device) race.  Nothing in
 *    the array needs to start at zero; each call overwrites what it reads.
 */
sk_status sigkernel_gram_noalloc(const sk_paths *X, const sk_paths *Y, int32_t dyadic_order,
                                 uint32_t flags, float *K, void *stream);
size_t sigkernel_gram_noalloc_max_bytes(void);

/*
 * sigkernel_gram_backward -- gradient of a weighted sum of Gram entries,
 *   L = sum_{a,b} dK[a][b] k_hat(X_a, Y_b),
 * with respect to every point of X and of Y:
 *   dX[a] = sum_b dK[a][b] d k_hat(X_a, Y_b) / d X_a   (overwritten),
 *   dY[b] = sum_a dK[a][b] d k_hat(X_a, Y_b) / d Y_b   (overwritten).
 * The derivative is that of the discrete scheme (eq. (explicit_finite_diff)
 * on P_lambda, the paper gives none): reverse accumulation through the cell
 * recurrence, then through the increment inner products of Section 3.1 and
 * the increments x_{p+1} - x_p.
 *  - dK: DEVICE float[X->n_paths * Y->n_paths], row-major; dX / dY: DEVICE
 *    float shaped like the points; either may be NULL (not wanted).
 *  - SK_SYMMETRIC: Y is X and the Gram is symmetric; the gradient of
 *    sum dK[a][b] K[a][b] over all (a, b) goes to dX and dY must be NULL.
 *    With SK_NO_DIAG as well, the diagonal entries (the constant 0 of the
 *    forward) carry no gradient.
 *  - Uniform or ragged batches (dX / dY then [offsets[n_paths]][dim], like
 *    the points).  A pair with a broken path (see sk_paths) contributes NaN
 *    to the gradient of its paths; point rows of a ragged batch that belong
 *    to no valid path receive NaN.
 *  - Any x length within the order limit: x paths taller than one band of
 *    256 fine rows are swept in bands.
 *  - Method: the forward pass saves the wavefront state every few steps
 *    (checkpoints, about 0.9 bytes per fine cell at order 1) and the adjoint
 *    recomputes each stretch of forward values from its checkpoint, bitwise
 *    as the forward computed them, instead of storing them.
 *  - Workspace: sigkernel_workspace_bytes(SK_OP_GRAM_BACKWARD, ...): the
 *    checkpoints of at most 2048 tasks in flight (a task is a run of pairs
 *    sharing one x path, or one pair of a ragged batch) and the increment
 *    gradients of every pair, in double.
 */
sk_status sigkernel_gram_backward(const sk_paths *X, const sk_paths *Y, int32_t dyadic_order,
                                  uint32_t flags, const float *dK, float *dX, float *dY,
                                  void *ws, size_t ws_bytes, void *stream);

/*
 * sigkernel_increment_gram -- the coarse increment inner products of Section
 * 3.1 (piecewise-linear case): up to 16 channels on the vector ALUs with rows
 * written in order (the contraction is too short to pay for the matrix cores;
 * the writes bound it), 17 to 64 channels on the matrix cores in 32 x 32
 * tiles:
 *   G0[pair][p][q] = <x_{p+1} - x_p, y_{q+1} - y_q>,  p < x.len - 1, q < y.len - 1,
 * written to HBM for every pair: gram = 1 enumerates (a, b) as a * Y->n_paths
 * + b, gram = 0 the pairs (x_k, y_k) (equal batch sizes).
 *  - Uniform batches of at most 64 channels (more: SK_ERR_UNSUPPORTED); G0: DEVICE
 *    float[pairs][X->len - 1][ldg], of which columns q < Y->len - 1 are
 *    written (the rest of each row is left as it was).  ldg = 0 means the
 *    dense layout, ldg = Y->len - 1; a nonzero ldg below that gives
 *    SK_ERR_SHAPE (nothing is enqueued).  A padded stride lets the caller
 *    align rows; the dense layout is the fastest to write, since the
 *    untouched padding leaves the last cache line of every row partly
 *    written.
 *  - flags: SK_GRAM_BF16 / SK_GRAM_F16 round the increments to 16 bits (the
 *    products and sums stay float32); otherwise float32 throughout.  Up to 16
 *    channels each entry is summed channel by channel in order with fused
 *    multiply-adds; above that the matrix cores choose the summation order.
 *  - No workspace.  Paths with one point give an empty G0 (nothing written).
 * The sweeps of sigkernel_pair / sigkernel_gram do not read G0 from memory:
 * they form the same inner products on the fly in registers, which avoids
 * writing and re-reading 4 bytes per coarse cell; this entry point serves
 * callers that need the coarse Gram itself.
 */
sk_status sigkernel_increment_gram(const sk_paths *X, const sk_paths *Y, int32_t gram,
                                   uint32_t flags, float *G0, int64_t ldg, void *stream);

/*
 * sigkernel_mmd2 -- unbiased MMD^2 between the laws of two batches of paths
 * under the signature kernel (the unbiased estimator mentioned at the end of
 * Section 3.1.1, used there to train generative models of paths):
 *   MMD^2 = sum_{a != b} k(X_a, X_b) / (n (n - 1)) + sum_{a != b} k(Y_a, Y_b) / (m (m - 1))
 *           - 2 sum_{a, b} k(X_a, Y_b) / (n m),     n, m >= 2,
 * with k the explicit scheme on P_lambda.  mmd2: DEVICE float[1].  With
 * SK_MMD2_GRAD, dX (DEVICE, shaped like X's points) receives d MMD^2 / d X;
 * Y is treated as fixed data.  Uniform or ragged batches.  Workspace:
 * sigkernel_workspace_bytes(SK_OP_MMD2, X, Y, dyadic_order, flags).
 */
sk_status sigkernel_mmd2(const sk_paths *X, const sk_paths *Y, int32_t dyadic_order,
                         uint32_t flags, float *mmd2, float *dX, void *ws, size_t ws_bytes,
                         void *stream);

/*
 * Signature kernels of lifted paths (the static-kernel lift, eq. (PDE_lifted)
 * and the finite-difference form that follows it).  A static kernel kappa on
 * R^d lifts x and y to paths X = phi(x), Y = psi(y) in a feature space; the
 * PDE for their signature kernel has, on the coarse cell between nodes p, p+1
 * of x and q, q+1 of y, the coefficient
 *   G[p][q] = kappa(x_{p+1}, y_{q+1}) - kappa(x_p, y_{q+1})
 *             - kappa(x_{p+1}, y_q) + kappa(x_p, y_q)
 * (the printed second term reads kappa(x_{s-1}, x_t); the pairing of X with Y
 * makes it kappa(x_{s-1}, y_t)), which replaces <dx_p, dy_q> in the scheme on
 * P_lambda (explicit, or implicit with SK_IMPLICIT).  Static kernels:
 *   SK_STATIC_LINEAR  kappa(a, b) = <a, b>: its lift is the path itself, and
 *                     the calls run the plain scheme (sigkernel_pair / _gram,
 *                     whose flags they then accept);
 *   SK_STATIC_RBF     kappa(a, b) = exp(-|a - b|^2 / (2 sigma^2)), sigma > 0
 *                     (the RBF-lifted kernel of the paper's experiments,
 *                     Section 5).  kappa and G are formed in double from the
 *                     float32 points (their coordinate differences are exact
 *                     in double), the sweep state is double, outputs float32.
 */
enum { SK_STATIC_LINEAR = 0, SK_STATIC_RBF = 1 };
typedef struct sk_static_kernel {
    int32_t kind;      /* SK_STATIC_LINEAR or SK_STATIC_RBF                     */
    int32_t reserved;  /* 0                                                     */
    double sigma;      /* SK_STATIC_RBF: the bandwidth (> 0, finite)            */
} sk_static_kernel;

/*
 * sigkernel_pair_lifted / sigkernel_gram_lifted -- as sigkernel_pair /
 * sigkernel_gram (same batches, outputs, modes and errors) for the lifted
 * kernel of `kernel` (HOST pointer, read during the call only).
 *  - flags: SK_IMPLICIT; the Gram also SK_SYMMETRIC / SK_NO_DIAG.  The 16-bit
 *    increment flags only with SK_STATIC_LINEAR.
 *  - SK_STATIC_RBF: the x paths must fit one wave's rows (2^lambda (x.len - 1)
 *    fine rows within the compiled rows-per-lane limits, at most 2048);
 *    taller x paths give SK_ERR_UNSUPPORTED (swap the arguments: the kernel
 *    is symmetric in the pair).  No gradient.
 *  - Workspace: sigkernel_workspace_bytes(SK_OP_PAIR_LIFTED / SK_OP_GRAM_LIFTED,
 *    ...), enough for either static kernel.
 *  - SK_ERR_VALUE: unknown kind, or sigma not positive and finite (or so small
 *    that 1 / (2 sigma^2) overflows).
 */
sk_status sigkernel_pair_lifted(const sk_paths *x, const sk_paths *y, int32_t dyadic_order,
                                uint32_t flags, const sk_static_kernel *kernel, float *out,
                                void *ws, size_t ws_bytes, void *stream);
sk_status sigkernel_gram_lifted(const sk_paths *X, const sk_paths *Y, int32_t dyadic_order,
                                uint32_t flags, const sk_static_kernel *kernel, float *K,
                                void *ws, size_t ws_bytes, void *stream);

/*
 * Reduced measures (Section "Moments-matching reduction algorithm for the
 * support of a discrete measure on paths").  For a measure
 * mu = sum_i alpha_i delta_{x_i} and the signature-kernel Gram
 * K[i][j] = k(x_i, x_j) (e.g. from sigkernel_gram with SK_SYMMETRIC), the
 * weights beta of the reduced measure minimise eq. (min_lasso),
 *   f(beta) = (alpha - beta)^T K (alpha - beta) + lam |beta|_1,
 * by the proximal-gradient iteration of eq. (fixed_point) started at
 * beta = alpha:
 *   beta <- A_t(beta - step 2 K (beta - alpha)),  A_t soft-thresholding,
 * with t = step * lam (the proximal map of step lam |.|_1; the printed
 * iteration writes the threshold as the step itself).
 *  - K: DEVICE float[n][n] (symmetric), alpha: DEVICE float[n]; 1 <= n <= 4096.
 *  - step > 0: used as given; step == 0: 1 / (2 * 1.05 * rho), rho the
 *    largest |eigenvalue| of K by power iteration (200 steps).  step_out:
 *    DEVICE double[1] receiving the step used, or NULL.
 *  - beta: DEVICE double[n] (overwritten).  One workgroup; iterations are
 *    matrix-vector products summed in double.
 *  - SK_ERR_VALUE: lam < 0, step < 0 or not finite.
 */
/* Fixed penalty: `iters` iterations; loss (DEVICE double[iters + 1] or NULL)
 * receives f before each iteration and after the last. */
sk_status sigkernel_reduced_measure(const float *K, const float *alpha, int32_t n, double lam,
                                    double step, int32_t iters, double *beta, double *loss,
                                    double *step_out, void *stream);
/* Support size: `rounds` bisection steps on lam over [0, 2 max_i |(K alpha)_i|]
 * (beyond that beta = 0 is optimal); each round runs `iters` iterations from
 * the previous round's beta; more non-zeros than `support` raises the lower
 * end, otherwise the upper.  beta and lam_out (DEVICE double[1]) receive the
 * last round whose support size equals `support`, else the last round. */
sk_status sigkernel_reduced_measure_support(const float *K, const float *alpha, int32_t n,
                                            int32_t support, int32_t iters, int32_t rounds,
                                            double step, double *beta, double *lam_out,
                                            double *step_out, void *stream);

/* Workspace sizing.  op is one of the SK_OP_* values. */
enum { SK_OP_PAIR = 0, SK_OP_GRAM = 1, SK_OP_GRAM_BACKWARD = 2, SK_OP_MMD2 = 3,
       SK_OP_CORRECTOR_FEATURES = 4,  /* X, Y: the pairs                              */
       SK_OP_CORRECTOR_BACKWARD = 5,  /* X->n_paths: the batch size (Y unused)        */
       SK_OP_CORRECTOR_PREDICT = 6,   /* X, Y: the pairs; dyadic_order: the fallback  */
       SK_OP_PAIR_LIFTED = 7,         /* sigkernel_pair_lifted                        */
       SK_OP_GRAM_LIFTED = 8          /* sigkernel_gram_lifted                        */
};
size_t sigkernel_workspace_bytes(int32_t op, const sk_paths *X, const sk_paths *Y,
                                 int32_t dyadic_order, uint32_t flags);

/*
 * Launch tuning (batching of pairs onto waves; no effect on any result).
 *
 * The Gram and pair calls map pairs onto one-wave sweeps.  Four launch
 * parameters change only how that work is spread over the chip, never the
 * arithmetic of a pair, so the forward outputs are bit-identical under every
 * tuning (a Gram backward sums its per-pair gradients in an order that
 * follows `run`: float32 rounding differences only):
 *  - run: pairs (a, b), (a, b+1), ... streamed back to back through one wave
 *    in a uniform Gram (the next pair's columns follow the previous pair's
 *    without draining the wavefront);
 *  - waves_per_block: one-wave sweeps per workgroup (1, 2 or 4);
 *  - pair_blocks_per_cu: resident 4-wave workgroups per CU of the persistent
 *    pair kernel (independent pairs, ragged batches, tall paths);
 *  - pair_bands: how the persistent pair kernel sweeps a grid taller than one
 *    wave's rows: 0 (built-in) as pipelined band tasks, one wave per band, all
 *    bands of a pair at once, when their hand-over slots fit a 1 GiB budget
 *    (else as 1); 1 with one wave per pair, band after band.  The workspace
 *    size does not depend on it.
 * A value of 0 keeps the built-in rule.  The library holds a table from
 * problem keys to tunings; calls whose key is in the table use its entry.
 * The workspace size of a Gram backward depends on `run`: query
 * sigkernel_workspace_bytes after changing the table.  Table updates are
 * serialised internally, but a call that runs while its entry changes may
 * use either version: set the table before concurrent use.
 */
typedef struct sk_tune_key {
    int32_t op;            /* SK_OP_PAIR, SK_OP_GRAM or SK_OP_GRAM_BACKWARD           */
    int32_t dyadic_order;
    int32_t symmetric;     /* 1 if SK_SYMMETRIC is set                                 */
    int32_t ragged;        /* 1 if either batch has offsets                            */
    int64_t nx, ny;        /* n_paths of X and Y                                       */
    int32_t x_len, y_len;  /* len of X and Y (upper bounds when ragged)                */
    int32_t dim;
    int32_t reserved;      /* 0                                                        */
} sk_tune_key;

typedef struct sk_tune {
    int32_t run;                 /* 1 .. 1024, 0 = built-in rule                       */
    int32_t waves_per_block;     /* 1, 2 or 4, 0 = 4                                   */
    int32_t pair_blocks_per_cu;  /* 1 .. 64, 0 = occupancy limit                       */
    int32_t pair_bands;          /* 0 = built-in rule (pipelined), 1 = sequential      */
} sk_tune;

/* The key of a call (op, batches, order and flags as the call receives them). */
sk_status sigkernel_tune_key(int32_t op, const sk_paths *X, const sk_paths *Y,
                             int32_t dyadic_order, uint32_t flags, sk_tune_key *key);
/* Insert or replace the entry of `key`; tune == NULL removes it.  Out-of-range
 * fields give SK_ERR_FLAGS (the table is then unchanged). */
sk_status sigkernel_tune_set(const sk_tune_key *key, const sk_tune *tune);
/* 1 and *tune filled if `key` has an entry, 0 if not, < 0 on a NULL argument. */
int32_t sigkernel_tune_get(const sk_tune_key *key, sk_tune *tune);
/* Copies up to `capacity` entries into keys / tunes (either may be NULL when
 * capacity is 0) and returns the number of entries in the table. */
int64_t sigkernel_tune_list(sk_tune_key *keys, sk_tune *tunes, int64_t capacity);
void sigkernel_tune_clear(void);

/*
 * sigkernel_autotune -- time the candidate tunings of one forward call and
 * keep the fastest in the table.
 *   op: SK_OP_PAIR or SK_OP_GRAM, with the arguments that call takes (out is
 *   its output: DEVICE float[n] or [nx * ny]; it is overwritten).
 * Each candidate runs once untimed and then `reps` (>= 1) times between HIP
 * events on `stream`; its time is the fastest repetition.  The call
 * synchronises `stream` (SK_ERR_STATE under graph capture).  On success
 * *best receives the chosen tuning, *best_ms (if not NULL) its time, and the
 * table holds it under the call's key.  Candidates that the workspace cannot
 * hold are skipped.
 */
sk_status sigkernel_autotune(int32_t op, const sk_paths *X, const sk_paths *Y,
                             int32_t dyadic_order, uint32_t flags, float *out, void *ws,
                             size_t ws_bytes, int32_t reps, void *stream, sk_tune *best,
                             float *best_ms);

/*
 * HIP graphs of library calls (launch-bound loops: replay a whole call, or a
 * sequence of calls, as one graph launch).
 *   sigkernel_graph_begin(stream): start capturing `stream` (a created stream,
 *   not the NULL stream; capture mode thread-local).  Library calls issued on
 *   it until sigkernel_graph_end are recorded, not run.
 *   sigkernel_graph_end(stream, &graph): stop capturing and instantiate.
 *   SK_ERR_HIP if the capture was invalidated (a failed launch, a
 *   synchronising call).
 *   sigkernel_graph_launch(graph, stream): replay on any stream.
 *   sigkernel_graph_destroy(graph).
 * The library calls record only kernel launches (no memset or copy nodes),
 * with every pointer and size fixed at capture: inputs, outputs and
 * workspace must stay allocated while the graph lives, and a replay reads
 * the inputs' contents at replay time.  Replays of one graph, or of graphs
 * sharing a workspace, must not overlap.
 */
typedef struct sk_graph_s *sk_graph;
sk_status sigkernel_graph_begin(void *stream);
sk_status sigkernel_graph_end(void *stream, sk_graph *graph);
sk_status sigkernel_graph_launch(sk_graph graph, void *stream);
sk_status sigkernel_graph_destroy(sk_graph graph);

/*
 * Learned corrector (this library's extension; the paper has no learned
 * component).  For pairs (x_k, y_k) of two uniform batches with at most 257
 * points and 16 channels, a small convolutional network reads the
 * dyadic-order-0 solve of the explicit scheme (Section 3.1, eq.
 * (explicit_finite_diff) with lambda = 0) and predicts the order-3 terminal
 * value and the size of its own error; pairs whose predicted error is too
 * large are solved by the plain scheme at the fallback order instead, which
 * is also what the network is trained against.
 *
 * Features: the order-0 grid of pair k has (m+1) x (n+1) nodes K and coarse
 * coefficients c[p][q] = <x_{p+1} - x_p, y_{q+1} - y_q>.  Every 4 x 4 block
 * (P, Q) of cells (64 x 64 blocks, NHWC) gets eight channels: the sums over its
 * cells of c, c^2 (A + B) / 2, c (A + B), C - 1, c^2 C, c (B - A) (C = K[p][q],
 * A = K[p+1][q], B = K[p][q+1]), then P / 63 and Q / 63; cells and blocks
 * outside the grid contribute 0.  With norm != NULL each channel is
 * normalised as (v - norm[c]) * norm[8 + c].
 *
 * Network: four layers of 3 x 3 convolution, stride 2, zero padding 1, 32
 * output channels, bias and ReLU (64 -> 32 -> 16 -> 8 -> 4 blocks a side),
 * weights and input activations rounded to bfloat16 (nearest even) before the
 * products, float32 accumulation; then a dense head 512 -> 2 in float32 over
 * the [4][4][32] map in NHWC order.  Flat float32 parameter vector of
 * sigkernel_corrector_param_count() entries: per layer weights
 * [32][3][3][Cin] (Cin = 8, 32, 32, 32) then 32 biases, then the head
 * [2][512] and 2 biases.  Output y = (y0, y1): with target_norm = (mu,
 * sigma), the corrected value is k_hat = k0 + mu + sigma y0 and the predicted
 * error sigma exp(y1).
 *
 * Features and activations are stored as bfloat16 (uint16_t bit patterns):
 * every consumer reads them as bf16 anyway, so the storage loses nothing.
 * Every buffer is DEVICE memory owned by the caller; per-pair buffers are
 * contiguous in pair order.
 */
int64_t sigkernel_corrector_param_count(void);
/* bf16 activations per pair kept by the forward for the backward */
int64_t sigkernel_corrector_act_elems(void);

/* feats: bf16[n][64][64][8]; k0: float[n] (the order-0 terminal values).
 * Workspace: sigkernel_workspace_bytes(SK_OP_CORRECTOR_FEATURES, X, Y, 0, 0).
 * SK_ERR_UNSUPPORTED beyond 257 points or 16 channels, or for ragged batches. */
sk_status sigkernel_corrector_features(const sk_paths *X, const sk_paths *Y, const float *norm,
                                       uint16_t *feats, float *k0, void *ws, size_t ws_bytes,
                                       void *stream);
/* y: float[n][2]; acts: bf16[n * sigkernel_corrector_act_elems()] (the four
 * layer outputs, layer-major: all pairs of layer 1, then of layer 2, ...). */
sk_status sigkernel_corrector_forward(const float *params, const uint16_t *feats, int64_t n,
                                      uint16_t *acts, float *y, void *stream);
/* grads (overwritten) = d sum(dy * y) / d params, through the bf16 roundings
 * as identities; the sums over pairs and positions run in a fixed order
 * (deterministic).  Workspace: sigkernel_workspace_bytes(
 * SK_OP_CORRECTOR_BACKWARD, X with n_paths = n, X, 0, 0). */
sk_status sigkernel_corrector_backward(const float *params, const uint16_t *feats,
                                       const uint16_t *acts, const float *dy, int64_t n,
                                       float *grads, void *ws, size_t ws_bytes, void *stream);
/* Training loss over n >= 1 pairs with targets t = (k_target - k0 - mu) / sigma:
 *   loss = mean(r^2 + r^2 exp(-2 y1) / 2 + y1),  r = y0 - t,
 * the second term's residual held constant for the gradient (a Gaussian
 * likelihood of the residual, which teaches y1 the error size).
 * loss: float[1]; dy: float[n][2] = d loss / d y. */
sk_status sigkernel_corrector_loss(const float *y, const float *k_target, const float *k0,
                                   const float *target_norm, int64_t n, float *loss, float *dy,
                                   void *stream);
/* Adam with bias correction; *step (DEVICE int32) is incremented first and
 * the update uses the new value t: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
sk_status sigkernel_adam_step(float *params, const float *grads, float *m, float *v, int64_t n,
                              int32_t *step, float lr, float beta1, float beta2, float eps,
                              void *stream);
/* Per-channel mean and 1 / (population) standard deviation of v = x - sub
 * (sub nullable: v = x), both [rows][channels] (channels <= 8; a constant
 * channel gets 1), summed in a fixed order in double (the normalisation
 * constants of the features and of the training targets).  x_dtype: 0
 * float32, 1 bf16 (sub is float32).  ws: SK_CHANNEL_STATS_WORKSPACE_BYTES. */
#define SK_CHANNEL_STATS_WORKSPACE_BYTES 32832
sk_status sigkernel_channel_stats(const void *x, int32_t x_dtype, const float *sub, int64_t rows,
                                  int32_t channels, float *mean, float *rstd, void *ws,
                                  size_t ws_bytes, void *stream);
/* Corrected order-3 values of the pairs: features, then the whole network
 * per pair on chip (one workgroup per pair, activations in LDS; the same
 * arithmetic as sigkernel_corrector_forward, bit for bit), then
 *   k_hat = k0 + mu + sigma y0,  e = sigma exp(y1);
 * a pair falls back unless kappa e <= tol |k_hat| and then receives the
 * plain scheme at `fallback_order` (out), computed on the device for exactly
 * those pairs (no host synchronisation).  out: float[n]; err (nullable):
 * float[n] predicted errors; fallback (nullable): int32[n], 1 where the plain
 * solve was used.  Workspace: sigkernel_workspace_bytes(
 * SK_OP_CORRECTOR_PREDICT, X, Y, fallback_order, 0). */
sk_status sigkernel_corrector_predict(const sk_paths *X, const sk_paths *Y, int32_t fallback_order,
                                      const float *params, const float *norm,
                                      const float *target_norm, float kappa, float tol, float *out,
                                      float *err, int32_t *fallback, void *ws, size_t ws_bytes,
                                      void *stream);

/* Human-readable name of a status code (static storage). */
const char *sigkernel_status_string(sk_status status);

/* Library version, "major.minor.patch" (static storage). */
const char *sigkernel_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SIGKERNEL_H */
