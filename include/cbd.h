/* cbd.h - C ABI of the MI355X (gfx950) implementation of the coloring-based
 * overlapping domain-decomposition (CBD) preconditioner with recursive-
 * skeletonization (RS) subdomain solvers for SPD first-kind integral equations
 * (Chen & Biros, "Overlapping domain decomposition preconditioner for integral
 * equations", arXiv 2108.12574).
 *
 * Conventions shared by every call:
 *  - Grid points of the n^d grid are numbered g = j1 + n*j2 (+ n^2*j3), 0-based,
 *    x fastest.  N = n^d.
 *  - Vectors with several right-hand sides are N x nrhs, column-major: column r
 *    (right-hand side r) is contiguous, i.e. a row-major (nrhs, N) array.  All
 *    vectors are FP64 device memory.
 *  - "device" pointers are HIP device allocations owned by the caller; the
 *    library keeps no reference to them after the call returns, except where a
 *    handle documents that it views them (cbd_problem views its four arrays and
 *    the FFT workspace; cbd_factor views its workspace).  The library allocates
 *    no device memory: every device array, workspaces included, comes from the
 *    caller, and *_workspace* calls give the sizes.
 *  - Handles are host objects owned by the library and released with the
 *    matching *_free call.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue work
 *    on it and return; calls that return host results (ranks, iteration counts,
 *    statistics) synchronize the stream first.
 *  - Return value: 0 = success, < 0 = error (nothing usable was produced; the
 *    message is in cbd_last_error(), which holds the last failure of the
 *    calling thread), > 0 = warning (result produced).
 */
#ifndef CBD_H
#define CBD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CBD_OK 0
#define CBD_EARG (-1)        /* invalid argument (sizes, modes, NULL pointers) */
#define CBD_EHIP (-2)        /* a HIP runtime call failed */
#define CBD_ENOTSPD (-3)     /* a Cholesky factorization met a non-positive pivot */
#define CBD_ENOMEM (-4)      /* a host allocation failed */
#define CBD_EWORKSPACE (-5)  /* the caller's workspace is too small (the message and, where the
                                call has one, an out-parameter give the bytes needed) */
#define CBD_EREPLAN (-6)     /* a replayed factorization read something other than its recording
                                (rs_factor_replay): factor again with rs_factor_batched */
#define CBD_WNOTCONV 1       /* PCG stopped at maxit before reaching tol */

#define CBD_GRID_CELL 0      /* x_t = (j_t + 1/2)/n (Section 2.1) */
#define CBD_GRID_NODE 1      /* 2D only: x_t = j_t/(n-1), weight and diagonal at h = 1/n */

#define CBD_MODE_JACOBI 0    /* Omega_i = P_i (non-overlapping), table t:dd */
#define CBD_MODE_SCHWARZ 1   /* Omega_i = extended P_i, (e:first) */
#define CBD_MODE_CBD 2       /* Omega_i = union of same-color extended P_k, (e:cbd) */

#define CBD_PREC_FP64 0      /* factors built, stored and applied in FP64 */
#define CBD_PREC_FP32 1      /* factors built, stored and applied in FP32; apply input/output FP64 */
#define CBD_PREC_BF16GEMM 2  /* as FP32, with the Schur-complement products (B_sr, B_rr, E, B_ss) on
                                bfloat16 operands with FP32 accumulation */

#define CBD_ROWS_AUTO 0      /* cbd_rs_opts.row_compression: see below */
#define CBD_ROWS_NEVER 1
#define CBD_ROWS_ALWAYS 2

#define CBD_ID_QR 0          /* cbd_rs_opts.id_method: see below */
#define CBD_ID_GRAM 1

typedef struct cbd_problem_s* cbd_problem;
typedef struct cbd_partition_s* cbd_partition;
typedef struct cbd_factor_s* cbd_factor;

/* Options of the RS factorization (Section 4.2). */
typedef struct {
    double tol;          /* relative accuracy eps of every ID, (e:id_err) */
    int n_pxy;           /* proxy points on the circle (2D) / sphere (3D) around a box */
    double proxy_ratio;  /* proxy radius / box side (1.5 in the paper's footnote to Section 5) */
    int precision;       /* CBD_PREC_FP64, CBD_PREC_FP32 or CBD_PREC_BF16GEMM */
    int exact;           /* 1: no compression; every A_i is factored by dense Cholesky
                            (the naive CBD of Section 5.1) */
    const float* mlp;    /* device parameters of the rank predictor (rank_mlp_*), or NULL.
                            Used only to schedule the pivoted QR; ranks and factors are
                            decided by the QR and do not depend on it. */
    int row_compression; /* levels of the stepped pivoted QR: reduce each proxy matrix to
                            its triangular factor R by an unpivoted Householder QR first
                            (equal column norms, pivots and ID in exact arithmetic, fewer
                            rows to stream per pivot step).  CBD_ROWS_AUTO (0): on levels
                            whose matrices are at least twice as tall as wide and hold at
                            least 32 MB together; CBD_ROWS_NEVER; CBD_ROWS_ALWAYS */
    int id_sketch;       /* 1: randomized IDs.  A box with n_p active DOFs and m proxy rows
                            takes the truncated CPQR of Z = Omega Y, Omega ell x m of random
                            signs, ell = ceil(3 n_p / 5) + 8, when ell < min(m, n_p); a sketch
                            whose rank exceeds ell - 8 is discarded for the deterministic ID.
                            With a predicted rank k_p (rank predictor or rank_hint), a first
                            sketch of 4 k_p + 32 rows is tried when smaller, and kept when its
                            rank k <= rows / 4.  0: deterministic IDs everywhere */
    unsigned long long sketch_seed;  /* seed of the random signs: the splitmix64 output
                            function of seed + key G1 + i G2 + rowkey G3 (mod 2^64), sign
                            from its top bit; key = (subdomain << 40) | (level << 32) | box,
                            rowkey = grid index of a near-field point or N + q for proxy
                            point q; G1 = 0x9E3779B97F4A7C15, G2 = 0xD1B54A32D192ED03,
                            G3 = 0x8CB92BA72F3D8DD7 */
    size_t workspace_bytes;  /* bound on the factorization's scratch per level (proxy
                            matrices, elimination work, FP64 T, box matrices): a level's boxes
                            are processed in chunks of consecutive boxes within it whose scratch
                            fits this bound and what is left of the workspace; 0: no bound
                            beyond the workspace.  Factor storage is not counted */
    int apply_rhs;       /* right-hand sides one pass of rs_apply handles (the factor's apply
                            buffers hold this many columns; more columns are applied in blocks
                            of this size); 0: 64 */
    int id_method;       /* how every ID is computed.  CBD_ID_QR (0): truncated
                            column-pivoted Householder QR, as (e:id) states it.  CBD_ID_GRAM
                            (1): truncated pivoted Cholesky of the Gram matrix G = Y^T Y (FP64
                            matrix cores for G and the trailing updates, panels of 32 pivots):
                            the Schur-complement diagonal is the squared trailing column norm,
                            so pivots, ranks and T = R11^{-1} R12 equal the QR's in exact
                            arithmetic; in FP64 the squared norms carry a rounding floor near
                            1e-16 |Y|^2, so it is meant for tol >= 1e-7 (the ID's residual then
                            stays within the tolerance) and is refused for smaller tol.  Boxes
                            with more active DOFs than the pivot kernel's LDS holds (16 bytes
                            each: about 10000 on gfx950) use the QR in both modes */
    int record;          /* 1: keep what the factorization uploads to and reads from the
                            device, in order, so that rs_factor_capture can turn it into a
                            graph (host memory of the order of the factor's index lists);
                            0: nothing kept */
} cbd_rs_opts;

/* Message of the last failed call on this thread ("" if none). */
const char* cbd_last_error(void);

/* ie_assemble - discretize the integral equation of Section 2.1, (e:ie)/(e:int)
 * with a = 0, on the n^d grid: A_ij = b_i h^d K(x_i - x_j) c_j (i != j),
 * A_ii = b_i c_i * (exact integral of K over the h-cell), K of (e:k).
 *  d: 2 or 3; n >= 2; grid: CBD_GRID_*.
 *  b, c: device, N values each, or NULL for 1.  SPD requires b = c > 0.
 *  pts (device, d*N, SoA: pts[t*N + g]), diag (device, N), w (device, N: column
 *  scale h^d c_j), rowscale (device, N: b_i): outputs, caller-owned; the
 *  returned problem views them, so they must outlive it.
 *  On success *out holds a new problem handle. */
int ie_assemble(int d, int n, int grid, const double* b, const double* c,
                double* pts, double* diag, double* w, double* rowscale,
                void* stream, cbd_problem* out);
int cbd_problem_free(cbd_problem p);

/* dd_partition - build the domain decomposition of Sections 2.2-2.3 and the
 * box hierarchy RS uses inside every subdomain (Section 4.2) for the n^d grid.
 * Host only: needs no GPU.
 *  d: 2 or 3; n: points per axis;
 *  m: partitions per axis (n % m == 0); delta: extension layers per side
 *  (ignored for JACOBI; CBD with m > 2 needs 2*delta <= n/m); mode: CBD_MODE_*;
 *  leaf_side: 0 = every extended partition is one leaf box, else leaf boxes are
 *  leaf_side-wide tiles of it.  The coloring is c(k) = sum_t (k_t mod 2) 2^(t-1).
 *  On success *out holds a new partition handle. */
int dd_partition(int d, int n, int m, int delta, int mode, int leaf_side, cbd_partition* out);
int cbd_partition_free(cbd_partition q);

/* Introspection of a partition (host arrays, caller-allocated).
 *  dd_partition_info: number of subdomains D, tile levels Lt, region levels Lr,
 *    total local DOFs sum_i |I_i|.
 *  dd_subdomain_info: |I_i|, number of leaf boxes, root level.
 *  dd_subdomain_index: I_i (|I_i| ints) in local order.
 *  dd_level_boxes: boxes of subdomain i at `level`: count; if lohi != NULL the
 *    cell bounding boxes (2*d ints per box: lo[0..d), hi[0..d)); if parent != NULL
 *    the index of each box's parent at level+1 (-1 at the root level). */
int dd_partition_info(cbd_partition q, int* D, int* Lt, int* Lr, long* total);
int dd_subdomain_info(cbd_partition q, int i, int* size, int* n_leaves, int* root_level);
int dd_subdomain_index(cbd_partition q, int i, int* index);
int dd_level_boxes(cbd_partition q, int i, int level, int* n_boxes, int* lohi, int* parent);

/* rs_factor_rank_count - number of compressed boxes of a factorization of this
 * partition with these options: the length of rank_hint and ranks_out below.  Boxes
 * are counted level by level (leaves first); within a level subdomain by subdomain,
 * and within a subdomain in the partition's box order (dd_level_boxes).  A
 * subdomain contributes at level l when its root level is above l.  Host only. */
int rs_factor_rank_count(cbd_partition q, const cbd_rs_opts* opts, int* count);

/* rs_factor_workspace - bytes of workspace to pass to rs_factor_batched.  With
 * rank_hint (host, rs_factor_rank_count ints: ranks of an earlier factorization of
 * the same layout, e.g. its ranks_out) the factor storage is exact for those ranks;
 * without, a box of n_p DOFs is guessed to keep a log10(1/tol) n_p^((d-1)/d)
 * skeletons (a = 0.55 in 2D, 0.4 in 3D).  Scratch is estimated for the largest
 * level, capped by opts->workspace_bytes.  A workspace that turns out
 * too small makes rs_factor_batched fail with CBD_EWORKSPACE and report what it
 * needed; more scratch than the estimate only means fewer chunks.  Host only. */
int rs_factor_workspace(cbd_problem p, cbd_partition q, const cbd_rs_opts* opts,
                        const int* rank_hint, size_t* bytes);

/* rs_factor_batched - RS factorization of every subdomain matrix A_i = R_i A R_i^T
 * (e:ai) of the partition, level by level (Section 4.2): at each level every box of
 * every subdomain is compressed with an ID of its proxy/near-field matrix ((e:id), the
 * proxy trick) and eliminated ((e:al), (e:alu), (e:b)); the last Schur complement
 * (e:schur) of each subdomain is factored by Cholesky.  All boxes of one level,
 * across all subdomains, are processed by the same kernel launches.
 * The factor keeps (per box) skeleton/redundant index lists, T, E = B_sr G^{-1},
 * G^{-1} (B_rr = G^T G) and B_ss, in opts->precision.
 *  rank_hint: host, rs_factor_rank_count ints, or NULL: expected ranks (for example
 *    ranks_out of an earlier factorization); they schedule the pivoted QR (its first
 *    run of steps without host checks, the row-compression choice) and override the
 *    rank predictor for that purpose.  Ranks are decided by the QR alone.
 *  ws, ws_bytes: device workspace, 256-byte aligned, caller-owned; the factor views
 *    it (factor arrays, the partition's index maps, the apply's buffers), so it must
 *    outlive the factor.  Its contents on entry do not matter.
 *  ranks_out: device, rs_factor_rank_count ints, or NULL: the rank of every
 *    compressed box.
 *  ws_used: host, or NULL: bytes of ws the factorization used (its high-water mark);
 *    on CBD_EWORKSPACE, that plus the request that did not fit (a lower bound on the
 *    bytes needed).
 * Synchronizes `stream` once per level to read the ranks.  The partition must be of
 * the problem's grid (same d and n, cell-centred points).  Errors: CBD_ENOTSPD names
 * the level and box; CBD_EWORKSPACE when ws is too small. */
int rs_factor_batched(cbd_problem p, cbd_partition q, const cbd_rs_opts* opts,
                      const int* rank_hint, void* ws, size_t ws_bytes, int* ranks_out,
                      size_t* ws_used, void* stream, cbd_factor* out);
int rs_factor_free(cbd_factor f);

/* Statistics of a factor: per subdomain DOFs at the last level (S_i, array of D
 * ints, may be NULL), the number of compressed levels, the bytes of factor
 * storage, and the algorithmic flops of the factorization (ID by truncated CPQR,
 * elimination and root Cholesky).  Per box with m proxy+near rows, n_p active
 * DOFs, rank k and n_r = n_p - k: ID 4 m n_p k - 2 (m + n_p) k^2 + 4 k^3 / 3;
 * elimination 4 k^2 n_r + 3 k n_r^2 + n_r^3 / 3 (the method's operations, with E
 * from a triangular solve; the explicit inverse the factor stores is not counted);
 * the root box counts as an elimination with k = 0. */
int rs_factor_stats(cbd_factor f, int* S, int* n_levels, size_t* bytes, double* flops);

/* Per-level ranks: number of boxes at `level` (all subdomains, in batch order)
 * and, if ranks != NULL, k per box; if np != NULL, active DOFs per box; if sub
 * != NULL, the subdomain of each box. */
int rs_factor_level(cbd_factor f, int level, int* n_boxes, int* ranks, int* np, int* sub);

/* Copy one box's factor to the host as FP64 (tests).  box is the index within
 * subdomain i at `level` (the partition's order).  sk (k ints), rd (n_r ints):
 * local indices of skeleton / redundant DOFs; T, E: k x n_r column-major;
 * Ginv: n_r x n_r column-major upper triangular; Bss: k x k.  Any output may be
 * NULL.  *k and *nr are always written. */
int rs_factor_box(cbd_factor f, int i, int level, int box, int* k, int* nr,
                  int* sk, int* rd, double* T, double* E, double* Ginv, double* Bss);
/* Root of subdomain i: S, local indices (S ints), G^{-1} of S = G^T G (S x S). */
int rs_factor_root(cbd_factor f, int i, int* S, int* idx, double* Ginv);

/* Skeleton-rank predictor (not in the paper: the project's learned part).  A
 * 3-layer MLP (width CBD_MLP_WIDTH, ReLU) maps CBD_MLP_FEATURES features of a box,
 * known before its ID, to log2(k + 1), k the rank its pivoted QR finds ((e:id)).
 * Weights are used rounded to bfloat16; activations and sums are FP32.  The
 * factorization uses the predictions to size the first, unchecked run of the
 * stepped QR of a level; the QR's stopping rule still decides every rank.
 *  params: device, rank_mlp_params() floats, layout W1 (64 x 6, row-major), b1 (64),
 *  W2 (64 x 64), b2 (64), W3 (64), b3 (1).  X: device, n x 6 row-major.
 *  Features: level/4, log2(box side in cells)/4, log2(active DOFs)/8,
 *  log2(near-field DOFs + 1)/8, -log10(tol)/8, d/3.
 *  rank_mlp_forward: y (device, n) = predictions.
 *  rank_mlp_loss_grad: mean squared error against t (device, n) into loss (device, 1,
 *  may be NULL) and its gradient into grad (device, like params); the weight
 *  gradient is taken at the rounded weights; ws: device, rank_mlp_workspace_bytes(n).
 *  rank_mlp_adam: one Adam step (beta 0.9 / 0.999, eps 1e-8) on params with moment
 *  buffers m, v (device, like params, zero before step 1); step counts from 1.
 *  rs_factor_features: training pairs of a factor's level: features (host, nbox x 6)
 *  and ranks (host, nbox), either may be NULL.
 *  rs_factor_schedule: stream synchronizations of the factorization, launch pairs of
 *  the stepped QR, boxes whose rank exceeded the predicted budget, the mean
 *  absolute rank prediction error (0 without a predictor), the number of batches
 *  whose proxy matrices were row-compressed before the pivoted QR, the boxes whose
 *  ID came from a sketch and those whose sketch saturated, the number of level
 *  chunks processed (the number of levels when no level was split), and, of the
 *  sketched boxes, those whose ID came from the rank-sized first sketch (4 k_p + 32
 *  rows for a predicted rank k_p, kept when k <= rows / 4) and those whose rank-sized
 *  sketch was not kept, and the kernel launches of the factorization (copies not
 *  counted).  Any output may be NULL. */
#define CBD_MLP_FEATURES 6
#define CBD_MLP_WIDTH 64
int rank_mlp_params(void);
size_t rank_mlp_workspace_bytes(int n);
int rank_mlp_forward(const float* params, int n, const float* X, float* y, void* stream);
int rank_mlp_loss_grad(const float* params, int n, const float* X, const float* t, float* grad,
                       float* loss, void* ws, size_t ws_bytes, void* stream);
int rank_mlp_adam(float* params, const float* grad, float* m, float* v, int step, float lr,
                  void* stream);
/* rank_mlp_loss_grad_noalloc - rank_mlp_loss_grad for callers that cannot allocate
 * device memory (code under HIP graph capture, tight training loops, harnesses that
 * forbid allocation): the same kernels and results, with the per-sample scratch in an
 * array the library holds on each device until the process ends, so no ws argument.
 *  n: 1 .. 16384 samples (more: CBD_EARG); other arguments as rank_mlp_loss_grad.
 * Every call on one device shares that array, and each call overwrites what it needs
 * before reading it: calls that overlap in time on one device race. */
int rank_mlp_loss_grad_noalloc(const float* params, int n, const float* X, const float* t, float* grad,
                               float* loss, void* stream);
int rs_factor_features(cbd_factor f, int level, int* n_boxes, float* X, int* k);
int rs_factor_schedule(cbd_factor f, int* host_syncs, int* qr_steps, int* mispredicted,
                       double* mean_abs_err, int* row_compressed, int* sketched, int* sketch_fallbacks,
                       int* chunks, int* sketched_pred, int* sketch_pred_rejected, long* launches);

/* Graph replay of a factorization (the factorization of Section 4.2, re-run whole).
 * An eager rs_factor_batched with opts.record = 1 leaves a recording of its host side:
 * every upload (box lists, near fields, metadata) and every read (ranks, skeleton
 * lists, stop flags of the pivoted QR or Cholesky, rank predictions, breakdown slots).
 * rs_factor_capture re-plays that host side without running anything and captures the
 * same kernel sequence, on the same workspace addresses, into one executable graph:
 * uploads become copies from gws, and each read (but the breakdown slots, which the
 * replay reads back itself) becomes a check of the device value against the recorded
 * one.  rs_factor_replay launches the graph on `stream`, so every
 * kernel of the factorization runs again on the problem's current device data (pts,
 * diag, w, rowscale), and synchronizes once to read the checks.  When every read
 * matches, every decision of the host is the one an eager factorization of that data
 * would take, so the factor is that factorization's (CBD_OK; the factor's host-side
 * statistics are unchanged).  Otherwise it returns CBD_EREPLAN and the factor is
 * marked stale (rs_apply refuses it) until it is freed: factor again with
 * rs_factor_batched.  With every read matching, a breakdown returns CBD_ENOTSPD (the
 * factor also stale); after a read that differs, CBD_EREPLAN is returned whatever
 * followed.
 *  rs_factor_graph_bytes: bytes of gws for a factor made with opts.record = 1 (0
 *    otherwise).
 *  rs_factor_capture: gws device, 256-byte aligned, caller-owned, at least
 *    rs_factor_graph_bytes; it must outlive the factor and stay untouched.  The
 *    factor's workspace, the problem's arrays and opts.mlp must stay where they are.
 *    Does not write ranks_out.  Synchronizes `stream` once (the upload of gws); the
 *    capture itself runs on a stream of its own.  Capturing again replaces the graph.
 *  rs_factor_replay: calls on one factor, and any other use of its workspace
 *    (rs_apply), must not overlap in time.  CBD_EARG without a captured graph. */
size_t rs_factor_graph_bytes(cbd_factor f);
int rs_factor_capture(cbd_factor f, void* gws, size_t gws_bytes, void* stream);
int rs_factor_replay(cbd_factor f, void* stream);

/* rs_apply - z = T^{-1} r = sum_i R_i^T A_i^{-1} R_i r, (e:ad), with every A_i^{-1}
 * applied through its RS factor: gather, forward sweep over levels, root solve,
 * backward sweep, and a deterministic scatter-add over overlapping subdomains.
 * Columns are processed in blocks of opts.apply_rhs.  Uses the factor's workspace:
 * calls on one factor must not overlap in time.
 *  r, z: device, N x nrhs column-major FP64 (may not alias). */
int rs_apply(cbd_factor f, int nrhs, const double* r, double* z, void* stream);

/* rs_apply_sub - one term of that sum: z = R_i^T A_i^{-1} R_i r for subdomain i
 * ((e:ai), (e:ad)); z is zero outside Omega_i.  With A_i^{-1} exact, P_i = R_i^T
 * A_i^{-1} R_i A fixes every vector supported in Omega_i (lemma l:subdomain of
 * Section 3.2); with the RS factor, up to its accuracy.  Arguments as rs_apply;
 * 0 <= i < number of subdomains. */
int rs_apply_sub(cbd_factor f, int i, int nrhs, const double* r, double* z, void* stream);

/* cbd_autotune_apply - choose, level by level, the shape of the apply's level sweep:
 * the right-hand-side columns one workgroup takes (8, 16, 32 or 64; default 16, fewer
 * where a box's local vectors would pass 64 KB of LDS) and its threads (256, 512 or
 * 1024, the product tiles spread over 4, 8 or 16 waves; default 1024 for boxes of 256
 * or more DOFs, else 256), by timing each candidate's forward and backward sweep of that level with HIP
 * events on `stream`; later rs_apply calls on this factor use the choices.  The result
 * does not depend on them (from 8 columns on, every column's sums run in the same
 * order).  r: device, N x nrhs FP64, a sample right-hand side (read only);
 * 1 <= nrhs <= opts.apply_rhs.  choices: host, 2 (levels + 1) ints (levels: rs_factor_stats'
 * n_levels), or NULL: columns and threads per level (0, 0 for a root level applied by
 * GEMMs).  Uses the factor's apply buffers: must not overlap in time with rs_apply on
 * this factor.  cbd_apply_set_shape fixes a level's shape (0: the default), for example
 * on a factor of the same layout as a tuned one.  Host only. */
int cbd_autotune_apply(cbd_factor f, int nrhs, const double* r, void* stream, int* choices);
int cbd_apply_set_shape(cbd_factor f, int level, int cols, int threads);

/* kernel_matvec - y = A x with A of ie_assemble, entries generated on the fly in
 * FP64 (the dense product; the paper uses FFTs for it, Section 5).
 *  x, y: device, N x nrhs column-major FP64 (may not alias). */
int kernel_matvec(cbd_problem p, int nrhs, const double* x, double* y, void* stream);

/* cbd_fft_prepare / kernel_matvec_fft - y = A x by FFT, the paper's matvec on the
 * uniform grid (Section 5): the kernel part is the aperiodic convolution of w o x
 * with g[delta] = K(spacing |delta|) (g[0] = 0), computed by circulant embedding
 * in a P^d grid (P the smallest power of two >= 2n - 1, at most 4096); the
 * diagonal term is added exactly.  Two right-hand sides share one complex
 * transform.  cbd_fft_prepare lays out, in ws (device, 256-byte aligned, at least
 * cbd_fft_workspace_bytes(d, n, max_pairs) bytes, caller-owned; the problem views
 * it until the next cbd_fft_prepare or cbd_problem_free), the embedded kernel's
 * transform, the twiddle factors and max_pairs complex P^d work arrays, and
 * synchronizes `stream`; kernel_matvec_fft then takes the same x, y as
 * kernel_matvec (N x nrhs column-major, FP64, no aliasing).  Calls of
 * kernel_matvec_fft on one problem must not overlap in time (shared work arrays). */
size_t cbd_fft_workspace_bytes(int d, int n, int max_pairs);
int cbd_fft_prepare(cbd_problem p, int max_pairs, void* ws, size_t ws_bytes, void* stream);
int kernel_matvec_fft(cbd_problem p, int nrhs, const double* x, double* y, void* stream);

/* cbd_autotune_matvec - choose the matvec's tile shape (rows per wave: 16, 32 or
 * 64) for this problem and nrhs by timing each candidate with HIP events on
 * `stream`; later kernel_matvec calls with the
 * same number of 16-column right-hand-side blocks use it.  Each candidate runs on
 * the first min(grid, 1024) workgroups.  x, y: device scratch of N x min(nrhs, 64)
 * doubles each (overwritten; distinct).  On 2D grids the candidates include
 * workgroups of 8 waves.  Times within 1% of the best count as ties, which go to
 * the shape with more rows per workgroup (it reads x fewer times).  *choice (may be
 * NULL) receives the shape, coded as for cbd_matvec_set_shape. */
int cbd_autotune_matvec(cbd_problem p, int nrhs, double* x, double* y, void* stream, int* choice);
/* cbd_matvec_set_shape - fix the matvec's tile shape for nrhs (as chosen by
 * cbd_autotune_matvec): shape = row blocks of 16 per wave (1, 2 or 4) with 4 waves per
 * workgroup, or 8 + that (9, 10, 12) with 8 waves per workgroup, the latter only on 2D
 * grids whose side is a multiple of the workgroup's rows.  Host only. */
int cbd_matvec_set_shape(cbd_problem p, int nrhs, int shape);

/* pcg_solve - preconditioned CG (Section 5) on A u = f for nrhs independent
 * right-hand sides: u0 = 0, stop a column when ||r||_2/||f||_2 <= tol (the
 * recurrence residual); beta = r+.z+/r.z, or r+.(z+ - z)/r.z with
 * CBD_PCG_FLEXIBLE.  With CBD_PCG_GRAPH the two launch sequences of an iteration
 * (matvec through ||r||, and preconditioner through the new direction) are
 * captured once into HIP graphs and replayed; this needs a non-default stream,
 * gives bitwise the same result, and records no kernel timers.  CBD_PCG_FFT uses
 * kernel_matvec_fft for the products with A (after cbd_fft_prepare).
 *  f (device, N x nrhs), u (device, N x nrhs, output).  fac = NULL: no
 *  preconditioner.  ws: device workspace of at least pcg_workspace_bytes(N, nrhs)
 *  bytes.  iters, relres: host arrays of nrhs (matvec count, final recurrence
 *  residual).  Returns CBD_WNOTCONV if a column did not converge within maxit. */
#define CBD_PCG_FLEXIBLE 1
#define CBD_PCG_GRAPH 2
#define CBD_PCG_FFT 4
size_t pcg_workspace_bytes(long N, int nrhs);
int pcg_solve(cbd_problem p, cbd_factor fac, int nrhs, const double* f, double* u,
              double tol, int maxit, int flags, void* ws, size_t ws_bytes,
              int* iters, double* relres, void* stream);

/* Kernel timing with HIP events recorded on the launching stream around every
 * launch of the named kernel family ("matvec", "apply", "factor"): enable,
 * read (total milliseconds and launch count since the last reset), reset. */
int cbd_timing_enable(int on);
int cbd_timing_get(const char* name, double* total_ms, long* launches);
int cbd_timing_reset(void);

#ifdef __cplusplus
}
#endif
#endif
