/*
 * dcrf.h -- C ABI of the MI355X (gfx950) library for energy minimisation in
 * dense CRFs with Gaussian pairwise potentials by continuous relaxations
 * (Desmaison, Bunel, Kohli, Torr, Kumar, "Efficient Continuous Relaxations
 * for Dense CRF", ECCV 2016).
 *
 * Problem (Sec. 3): N = H*W pixels, L labels, unaries phi (N x L), a label
 * compatibility mu (L x L) and a pixel compatibility that is a mixture of
 * Gaussian kernels sum_m w_m exp(-|f_a^m - f_b^m|^2 / 2) (eq. pairwise,
 * eq. gaussiankernel). Kernel m's features are the pixel position divided by
 * theta_pos and, when use_rgb, the RGB colour divided by theta_rgb (App. G):
 * f = (x/theta_pos, y/theta_pos[, R/theta_rgb, G/theta_rgb, B/theta_rgb]),
 * x = column, y = row.
 *
 * Conventions for every call below:
 *  - Layout: pixel-major. Pixel a = row*W + col. An N x C array holds
 *    element (a, c) at [a*C + c]. mu is row-major L x L. rgb is float32
 *    N x 3 with values in [0, 255].
 *  - Memory: every array argument marked (dev) is DEVICE memory on the
 *    context's device, owned by the caller, contiguous, 16-byte aligned (as
 *    device allocations are), in the context's floating type (float for
 *    DCRF_F32, double for DCRF_F64) unless stated.
 *    Arguments marked (host) are host memory. The context's own device
 *    memory (lattice tables, solver state) is either allocated by the
 *    library as calls need it, or carved from a workspace the caller hands
 *    to dcrf_set_image / dcrf_set_images (see dcrf_workspace_size); with a
 *    workspace the library calls neither hipMalloc nor hipFree. It never
 *    frees caller memory.
 *  - Device-detected errors: the solvers check their unaries and marginals
 *    for non-finite values on the device; a raised flag is reported as
 *    DCRF_EINVAL by the next call that waits for the stream (dcrf_sync
 *    waits and reports), and is then cleared.
 *  - Streams: all device work is enqueued on the context's stream. Calls
 *    that return host values (energies, traces, objective values) wait for
 *    the stream; the others are asynchronous.
 *  - Errors: every call returns a dcrf_status. It never aborts or exits. On
 *    failure dcrf_last_error() returns a message; the context stays usable.
 *  - Label compatibility: every mu argument may be NULL, which stands for
 *    the Potts compatibility mu(i, j) = [i != j] of Sec. 3. The library then
 *    uses its own device copy and knows the closed form without reading mu
 *    back; a non-NULL mu that happens to be Potts is recognised by one
 *    device-to-host copy per call.
 */
#ifndef DCRF_H
#define DCRF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dcrf_ctx dcrf_ctx;

typedef enum {
    DCRF_OK = 0,
    DCRF_EINVAL = -1,        /* bad argument (null, size, value)            */
    DCRF_ENOMEM = -2,        /* device allocation failed                    */
    DCRF_ERANGE = -3,        /* lattice coordinates exceed the key range    */
    DCRF_ECAPACITY = -4,     /* hash table overflow                          */
    DCRF_EHIP = -5,          /* a HIP runtime call failed                    */
    DCRF_EUNSUPPORTED = -6,  /* unsupported size or combination             */
    DCRF_ESTATE = -7         /* call out of order (e.g. no image set)       */
} dcrf_status;

typedef enum { DCRF_F32 = 0, DCRF_F64 = 1 } dcrf_dtype;

/* How the solvers apply the pixel compatibility. */
typedef enum {
    DCRF_FILTER_LATTICE = 0, /* permutohedral lattice, O(N) (Sec. 3, App. A) */
    DCRF_FILTER_EXACT = 1,   /* exact O(N^2) Gaussian sum (eq. fb)           */
    DCRF_FILTER_SEPARABLE = 2 /* position-only kernels exact by two 1-D
                                 convolutions, the others by the lattice */
} dcrf_filter_mode;

/* Flags of dcrf_filter. */
#define DCRF_ADJOINT 1u      /* apply the transpose (blur directions reversed) */
#define DCRF_EXACT 2u        /* use the exact O(N^2) sum for this call        */
#define DCRF_SEPARABLE 4u    /* the separable filter mode for this call       */
#define DCRF_KEEP_SELF 8u    /* keep the b = a term: out = Kbar in            */
#define DCRF_PER_KERNEL 16u  /* one output block per kernel (see dcrf_filter)  */

/* One Gaussian kernel of the pixel compatibility (eq. pairwise, App. G). */
typedef struct {
    int use_rgb;             /* 1: features (x, y, R, G, B); 0: (x, y)       */
    double theta_pos;        /* > 0, in pixels                               */
    double theta_rgb;        /* > 0 when use_rgb, in colour units             */
    double weight;           /* w_m >= 0                                      */
} dcrf_kernel;

/* Per-iteration record of a Frank-Wolfe run (Sec. 4, Alg. fw). */
typedef struct {
    double objective;        /* f(y_t) = c^T y_t + y_t^T (Psi + D) y_t        */
    double gap;              /* <g_t, y_t - s_t>, g_t = c + 2 (Psi + D) y_t   */
    double alpha;            /* step taken from y_t                           */
    double changed;          /* pixels whose conditional gradient changed     */
} dcrf_iter_trace;

/* Launch shapes chosen by dcrf_autotune. */
typedef struct {
    int splat_chunk;              /* entries per chunk of the one-hot splat   */
    int dense_chunk;              /* entries per chunk of the dense splat     */
    int splat_stage;              /* 1: the dense splat stages the pairs of a
                                     block's chunks in LDS; 0: each lane
                                     reads them from global memory          */
    int blur_vectors_per_thread;  /* 16-byte vectors per thread in the blur   */
    int blur_block;               /* threads per block of the blur            */
    int blur_group;               /* blur directions applied per launch       */
    int tiles;                    /* 1: splats and slices by 16x16 pixel tiles */
    int fw_splat;                 /* 0 (default): the Frank-Wolfe step splats
                                     its one-hot s in a launch of its own
                                     (vertex by vertex, over the inverse
                                     index); 1: from the kernel that picks s,
                                     pixel by pixel (runs of lanes with the
                                     same vertex and label summed in the wave
                                     first, one atomic per run) */
    int fw_persistent;            /* 0 (default): one launch per stage of each
                                     Frank-Wolfe iteration; 1: every iteration
                                     of a solve in one cooperative launch with
                                     grid barriers between the stages (the
                                     row kernels' lattice path with the staged
                                     one-hot splat and blur_group 2; other
                                     settings keep the per-stage launches) */
    double ms;                    /* time of the tuned filter paths, ms       */
} dcrf_tune;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device`; `hip_stream` is a hipStream_t
 * (NULL = the null stream). *out receives the context. */
int dcrf_create(dcrf_ctx **out, int device, void *hip_stream);
int dcrf_destroy(dcrf_ctx *ctx);
/* Message of the last failed call on this context (never NULL). */
const char *dcrf_last_error(const dcrf_ctx *ctx);
/* Enqueue later work on another hipStream_t. */
int dcrf_set_stream(dcrf_ctx *ctx, void *hip_stream);
/* Library version string. */
const char *dcrf_version(void);

/* ---- image and lattices ------------------------------------------------ */

/* An upper bound of the device memory a context needs for one H x W image
 * with these kernels, for every call of this header on it with at most L
 * labels or channels (the reverse sweep's workspace included, its
 * checkpoint buffer not: that is the caller's). The bound takes the largest
 * lattices the image size allows (N (d+1) vertices per kernel), so it holds
 * for any colours. It assumes dense splat chunks of at most 64 entries
 * (dcrf_set_tune refuses more while a workspace is attached), traces and S
 * histories of at most 4096 steps and at most 4096 unrolled iterations.
 * *bytes (host). No device is touched. */
int dcrf_workspace_size(int H, int W, int L, const dcrf_kernel *kernels,
                        int nk, int dtype, size_t *bytes);

/* The same for a batch of B images of sizes H[j] x W[j] (dcrf_set_images). */
int dcrf_workspace_size_images(int B, const int *H, const int *W, int L,
                               const dcrf_kernel *kernels, int nk, int dtype,
                               size_t *bytes);

/* Set the image and kernels (1 <= nk <= 4) and build one permutohedral
 * lattice per kernel on the device: lattice coordinates in FP64, a device
 * hash table of vertices, per-pixel vertex ids and barycentric weights and a
 * neighbour table along the d+1 blur directions. Also computes the row sums
 * r = K'1 used by d (eq. RL-diagonal). rgb: (dev) float32 N x 3.
 * dtype: DCRF_F32 or DCRF_F64 for every later floating argument.
 * workspace: (dev, caller-owned, 256-byte aligned, >= 4096 bytes) or NULL.
 * With a workspace of ws_bytes (dcrf_workspace_size gives enough) every
 * device buffer of the context is taken from it until the next
 * dcrf_set_image / dcrf_set_images or dcrf_destroy, which hand it back; the
 * caller keeps it alive until then. A call that would need more returns
 * DCRF_ENOMEM and leaves the context usable. NULL: the library allocates.
 * Errors: DCRF_EINVAL (sizes, thetas, a non-finite colour), DCRF_ERANGE
 * (coordinates too large for the 64-bit vertex key: theta too small for the
 * image), DCRF_ECAPACITY (a lattice has more vertices than hash slots: only
 * with dcrf_set_hash_capacity), DCRF_ENOMEM. */
int dcrf_set_image(dcrf_ctx *ctx, int H, int W, const float *rgb,
                   const dcrf_kernel *kernels, int nk, int dtype, void *workspace,
                   size_t ws_bytes);

/* Bytes of the context's workspace in use now and at most since it was
 * attached (DCRF_EINVAL without a workspace). Either pointer may be NULL. */
int dcrf_workspace_used(dcrf_ctx *ctx, size_t *in_use, size_t *peak);

/* Force the hash table of every lattice built by later dcrf_set_image /
 * dcrf_set_images calls to `slots` slots (a power of two in [16, 2^32]);
 * 0 restores the default (a power of two of at least 2 N (d+1), which never
 * overflows). A lattice with more vertices than slots fails its build with
 * DCRF_ECAPACITY. For testing the capacity path and for bounding the
 * table's memory. */
int dcrf_set_hash_capacity(dcrf_ctx *ctx, size_t slots);

/* Wait for the context's stream and report device-detected errors raised
 * since the last report (DCRF_EINVAL for a non-finite unary or marginal). */
int dcrf_sync(dcrf_ctx *ctx);

/* A batch of B images of their own sizes in one context (the batched
 * extension of the QP solver; the model of Sec. 3 per image). Image j has
 * H[j] x W[j] pixels and colours rgb[j] (host array of B device pointers to
 * float32 H[j] W[j] x 3); the kernels and dtype are shared. Each image gets
 * its own lattices, concatenated so that one launch per filter stage covers
 * the batch; the filter never couples two images.
 *
 * Layout: every N x C argument of the later calls is one packed array whose
 * rows [seg[2j], seg[2j+1]) are image j's pixels in row-major order
 * (dcrf_image_layout gives seg and the total row count N). Images start at
 * multiples of 64 rows; the rows between images are ignored on input by the
 * solvers, and their content in outputs is unspecified.
 * Per-image results: Frank-Wolfe steps, traces (record t * B + j) and the
 * step checkpoints are per image; dcrf_fw_backward writes B x nk weight
 * gradients (image-major); dcrf_energy returns the sum over the images.
 * Not available on a batch (DCRF_EUNSUPPORTED): the exact filter mode and
 * the LP calls. B = 1 is the same as dcrf_set_image. workspace, ws_bytes: as
 * for dcrf_set_image, sized by dcrf_workspace_size_images. */
int dcrf_set_images(dcrf_ctx *ctx, int B, const int *H, const int *W,
                    const float *const *rgb, const dcrf_kernel *kernels, int nk,
                    int dtype, void *workspace, size_t ws_bytes);

/* dcrf_set_images under the name of the batch calls below. */
int dcrf_batch_set_images(dcrf_ctx *ctx, int B, const int *H, const int *W,
                          const float *const *rgb, const dcrf_kernel *kernels, int nk,
                          int dtype, void *workspace, size_t ws_bytes);

/* dcrf_fw_forward and dcrf_fw_backward with one array per image instead of
 * the packed layout: unary[j], y_out[j], grad_y[j] and grad_unary[j] (host
 * arrays of B device pointers) each hold image j's H[j] W[j] x L values,
 * row-major. The library copies them to and from packed arrays of its own
 * (device-to-device copies on the context's stream), so the results are
 * those of the packed calls; saved, grad_w (B x nk, image-major) and
 * grad_w_total (nk) as there. One launch per stage covers every image. */
int dcrf_batch_fw_forward(dcrf_ctx *ctx, const void *const *unary, const void *mu, int L,
                          const double *w, int iters, void *const *y_out, void *saved);
int dcrf_batch_fw_backward(dcrf_ctx *ctx, const void *const *unary, const void *mu, int L,
                           int iters, const void *saved, const void *const *grad_y,
                           void *const *grad_unary, double *grad_w, double *grad_w_total);

/* *nimg = images held (1 after dcrf_set_image), *rows = N, the rows of every
 * N x C argument; seg (host, 2 nimg ints, may be NULL) = first and one past
 * the last row of each image. Any pointer may be NULL. */
int dcrf_image_layout(dcrf_ctx *ctx, int *nimg, int *rows, int *seg);

/* Pick the launch shapes of the filter by timing, for each candidate, `reps`
 * (1..1000) runs of a dense L-channel filter plus the one-hot splat, blur and
 * slice of a Frank-Wolfe iteration on the context's own lattices, in two
 * rounds: first splats and slices by inverse-index chunks and pixel rows or
 * by 16x16 pixel tiles, one-hot chunks of 32, 64 or 128 entries, and in the
 * blur 1, 2 or 3 directions per launch, 1 or 2 16-byte vectors per thread and
 * 128 or 256 threads per block; then (without tiles) dense chunks of 16, 32
 * or 64 entries, with or without staging in LDS. Keeps the fastest.
 * *out (host, may be NULL) receives the choice. Results of every call are the
 * same for every choice up to floating-point summation order. */
int dcrf_autotune(dcrf_ctx *ctx, int L, int reps, dcrf_tune *out);

/* Set the launch shapes directly (the `ms` field is ignored): splat_chunk and
 * dense_chunk in {16, 32, 64, 128, 256}, splat_stage 0 or 1,
 * blur_vectors_per_thread in 1..4, blur_block in {64, 128, 256}, blur_group
 * in 1..3, tiles 0 or 1, fw_splat 0 or 1, fw_persistent 0 or 1;
 * DCRF_EINVAL otherwise.
 * Results are the same for every choice up to floating-point summation
 * order. */
int dcrf_set_tune(dcrf_ctx *ctx, const dcrf_tune *tune);

/* Replace the kernel weights w_m (host, nk values) without rebuilding the
 * lattices; recomputes r. */
int dcrf_set_weights(dcrf_ctx *ctx, const double *w, int nk);

/* Choose how the solvers filter (default DCRF_FILTER_LATTICE).
 * DCRF_FILTER_SEPARABLE applies every kernel on position alone (no colour
 * features) exactly: its Gaussian factors into one along x and one along y
 * (eq. gaussiankernel with App. G's scaling), so K Y is a convolution of
 * each channel along the rows and then along the columns with taps
 * exp(-t^2 / (2 theta^2)), |t| <= min(ceil(theta sqrt(120 ln 2)), max(H, W) - 1)
 * (the dropped taps lie below 2^-60 of the centre); the other kernels stay on
 * the lattice. The QP apply, Frank-Wolfe, DC_gen, DC_neg and the energy then
 * take a dense K'Y per filter (as in the exact mode). The LP, the
 * differentiation, the allocation-free solve, the autotuner and batch
 * contexts give DCRF_EUNSUPPORTED in the exact and separable modes (the LP
 * accepts the exact mode). */
int dcrf_set_filter_mode(dcrf_ctx *ctx, int mode);

/* Lattice of kernel m: feature dimension d and number of vertices. */
int dcrf_lattice_info(dcrf_ctx *ctx, int m, int *d, int *nvert);

/* Copy lattice m to the host: keys (host, nvert x d int32) = the first d
 * integer coordinates of each vertex in the scaled lattice (d+1)A*_d;
 * vid (host, N x (d+1) int32) = the vertex of each pixel's simplex, -1 where
 * the barycentric weight is 0; w (host, N x (d+1) double) = the weights.
 * Any pointer may be NULL. For tests and inspection. */
int dcrf_lattice_export(dcrf_ctx *ctx, int m, int32_t *keys, int32_t *vid,
                        double *w);

/* ---- the pairwise filter ----------------------------------------------- */

/* out = K' in, where K' = sum_m w_m K_m - (sum_m w_m) I, i.e.
 * out_a = sum_{b != a} sum_m w_m k_m(a, b) in_b  (eq. fb summed over the
 * kernels without the b = a term of eq. labelling-energy). By default each
 * K_m is its permutohedral approximation gamma_d * slice . blur . splat;
 * DCRF_EXACT uses the O(N^2) sum, DCRF_SEPARABLE the separable mode of
 * dcrf_set_filter_mode (the two exclude each other), DCRF_ADJOINT the
 * transpose. DCRF_KEEP_SELF keeps the b = a term: out = Kbar in =
 * K' in + (sum w) in (with the lattice, each kernel's own approximate self
 * response). DCRF_PER_KERNEL writes nk blocks of N x C to out (out holds
 * nk N C values): block m = w_m K_m in - w_m in, kernel m's share of K' in
 * (the blocks add up to it), or w_m K_m in with DCRF_KEEP_SELF; the
 * per-kernel pieces of the weight gradient of eq. pairwise.
 * in, out: (dev) N x C, 1 <= C <= 256, not aliased. */
int dcrf_filter(dcrf_ctx *ctx, const void *in, void *out, int C,
                unsigned flags);

/* out = (Psi + D) y = (K'Y) mu^T + d * y  (eq. pairwise-matrix,
 * eq. RL-diagonal with d_a(i) = sum_j |mu_ij| (K'1)_a). y, out: (dev) N x L;
 * mu: (dev) L x L. Uses the filter mode of the context. */
int dcrf_qp_apply(dcrf_ctx *ctx, const void *y, const void *mu, int L,
                  void *out);

/* ---- solvers ------------------------------------------------------------ */

/* Frank-Wolfe on the convex QP relaxation (Sec. 4, Alg. fw, App. B):
 * minimise (phi - d)^T y + y^T (Psi + D) y over the product of simplices.
 * unary: (dev) N x L; mu: (dev) L x L; y_inout: (dev) N x L, the starting
 * point on input (must lie in the feasible set), the result on output.
 * trace: (host) `iters` records or NULL (iters x B for a batch, record
 * t * B + j). One filter call per iteration; the step size is solved on the
 * device, per image for a batch. */
int dcrf_qp_frank_wolfe(dcrf_ctx *ctx, const void *unary, const void *mu,
                        int L, void *y_inout, int iters,
                        dcrf_iter_trace *trace);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that keep the allocator out of their steady state):
 * dcrf_qp_frank_wolfe with the same arguments and results, which allocates
 * nothing. The solve's per-call buffers (linear term, P_y, P_s, conditional
 * gradients, partial sums, step accumulators, trace, the Potts copy of mu
 * and each lattice's vertex values) live in one fixed device array of the
 * library, dcrf_noalloc_scratch_bytes() bytes (64 MiB) per device, held
 * until the process ends; everything else it reads was built by
 * dcrf_set_image. Limits: lattice filter mode, L <= 32, iters <= 4096, and
 * a solve that fits the array (about 3 N L values plus the vertex values:
 * 500 x 375 with 21 labels in FP32 fits); otherwise DCRF_EINVAL or
 * DCRF_EUNSUPPORTED, with nothing allocated. A launch shape whose blur tables
 * were never built (a dcrf_set_tune without a later filter call) gives
 * DCRF_ENOMEM instead of allocating them. Every call on one device shares
 * the array, so calls that overlap on a device (other streams or threads)
 * race; consecutive calls on one stream are safe. */
int dcrf_qp_frank_wolfe_noalloc(dcrf_ctx *ctx, const void *unary, const void *mu,
                                int L, void *y_inout, int iters,
                                dcrf_iter_trace *trace);

/* *bytes = the size of the allocation-free solve's device array. */
int dcrf_noalloc_scratch_bytes(size_t *bytes);

/* Generic DC relaxation by CCCP (Sec. 5.1, Alg. cccp, eq. cccp-qp): `outer`
 * steps, each minimising phi^T y - 2 (d * y^k)^T y + y^T (Psi + D) y with
 * `inner` warm-started Frank-Wolfe iterations. S_hist: (host) outer+1 values
 * of S(y) = phi^T y + y^T Psi y (before the first and after each step) or
 * NULL. The history stays on the device until the end of the call, which
 * then waits for the stream once; without S_hist (and with mu NULL) the
 * call is asynchronous. */
int dcrf_dc_gen(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
                void *y_inout, int outer, int inner, double *S_hist);

/* DC relaxation for negative semi-definite label compatibilities by CCCP
 * (Sec. 5.2, eq. QP-concave-CCCP; App. C, eq. convexpb-concavecccp and
 * eq. convexpb-onevar). S(y) = phi^T y + y^T Psi y is split into
 * phi^T y - wsum y^T (mu (x) I) y (convex) and y^T (mu (x) Kbar) y (concave),
 * Kbar = sum_m w_m K_m, wsum = sum_m w_m. Each of the `outer` steps makes one
 * filter call for the concave part's gradient 2 (Kbar Y) mu^T and then
 * solves N independent L-variable problems
 *     min over the simplex of c_a^T y_a - wsum y_a^T mu y_a,
 *     c_a = phi_a + 2 (Kbar Y)_a mu^T.
 * mu NULL or Potts: the exact minimiser, the projection of -c_a / (2 wsum)
 * onto the simplex (the vertex of the smallest c_a(i) when wsum = 0);
 * `inner` is then unused. Another mu (dev L x L, symmetric, negative
 * semi-definite on the vectors that sum to zero; not checked): `inner` >= 1
 * per-pixel Frank-Wolfe iterations with exact steps from y_a (App. C).
 * unary: (dev) N x L; y_inout: (dev) N x L, start (in the feasible set) and
 * result. S_hist: (host) outer + 1 values of S(y) (before the first and
 * after each step; for a batch, the sum over its images) or NULL; asking
 * for it costs one more filter call and one wait for the stream at the end.
 * L <= 32 (DCRF_EUNSUPPORTED otherwise). */
int dcrf_dc_neg(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
                void *y_inout, int outer, int inner, double *S_hist);

/* argmax labelling of marginals y (dev, N x L) into labels (dev int32 N),
 * lowest label on ties. */
int dcrf_round(dcrf_ctx *ctx, const void *y, int L, int32_t *labels);

/* Energy E(x) = sum_a phi_a(x_a) + sum_a sum_{b != a} mu(x_a, x_b) Kbar_ab
 * (eq. labelling-energy) of labels (dev int32 N, values in [0, L)), with the
 * context's filter mode; *energy (host). */
int dcrf_energy(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
                const int32_t *labels, double *energy);

/* ---- LP relaxation (Potts) --------------------------------------------- */

/* Leaf-exact divide and conquer for the LP calls below (App. E): from the
 * first level whose nodes all hold at most `leaf` sorted positions
 * (ceil(N / 2^l) <= leaf), the pairs inside each node are summed exactly
 * (the Gaussian sum, one block per node) instead of being filtered level by
 * level further down: ceil(log2(N / leaf)) lattice levels instead of
 * ceil(log2 N). leaf in [0, 256]; 0 or 1 (the default 0) keeps the plain
 * recursion. The exact filter mode ignores it. */
int dcrf_set_lp_leaf(dcrf_ctx *ctx, int leaf);

/* One subgradient of the LP relaxation of the Potts model (Sec. 6,
 * eq. potts-lp) at y: g_c(i) = phi_c(i) + sum_{a after c} Kbar_ac
 * - sum_{a before c} Kbar_ac, the order being y(:, i) descending with ties by
 * ascending pixel index (eq. simple_S, eq. grad_lp). The two sums are computed
 * by the divide and conquer of App. E (nodes split at floor((2n+1) N / 2^(l+1))
 * at level l), each node's filter on a permutohedral lattice built on the
 * node's points; with DCRF_FILTER_EXACT they are summed exactly, O(N^2) per
 * label. unary, y: (dev) N x L (y in the feasible set); g: (dev) N x L out;
 * *S_lp (host) = <g, y>, the LP objective at y. Waits for the stream. The
 * label compatibility is Potts; no mu argument is taken. Lattice mode keeps
 * one sub-lattice table per kernel of 2 N (d+1) slots: DCRF_ERANGE if that
 * exceeds 2^31 - 1 (about 179 M pixels with the bilateral kernel); a batch
 * context gives DCRF_EUNSUPPORTED. */
int dcrf_lp_subgradient(dcrf_ctx *ctx, const void *unary, int L, const void *y,
                        void *g, double *S_lp);

/* Projected subgradient descent on the LP (Alg. lp_subgrad): `steps` steps
 * y <- Pi(y - beta_t g), beta_t = beta0 / (1 + t) for t = 0, 1, ..., Pi the
 * Euclidean projection onto the product of simplices. y_inout (dev N x L):
 * start and result. best_obj (host, may be NULL): the smallest S_LP met;
 * best_y (dev N x L, may be NULL, not aliasing y): the iterate that had it;
 * hist (host, `steps` values, may be NULL): S_LP(y_t). */
int dcrf_lp_descent(dcrf_ctx *ctx, const void *unary, int L, void *y_inout,
                    int steps, double beta0, double *best_obj, void *best_y,
                    double *hist);

/* ---- LP relaxation for an r-HST metric (App. F) ----------------------- */

/* One subgradient of the LP for a tree metric (App. F, eq. rHST-LP,
 * Alg. rHST). The tree has n_nodes nodes: node k < L is label k's leaf,
 * parent[t] (host int32) is t's parent or -1 for the root (one root, no
 * cycles, labels are leaves), c[t] (host, >= 0) the weight c_T of subtree t.
 * With y_a(T) the sum of y_a(i) over the labels under T (added in increasing
 * label order), g = phi plus, for every subtree with c_T > 0,
 * c_T (sum_{a after c} Kbar_ac - sum_{a before c} Kbar_ac) in the order of
 * y(T) (descending, ties by pixel index) on the column of every label under
 * T; *S_lp (host) = <g, y>, the objective of eq. rHST-LP. The pair sums are
 * those of dcrf_lp_subgradient (divide and conquer, or exact), one pass per
 * weighted subtree. For an r-HST with edge length l_T above subtree T,
 * c_T = 2 l_T makes the objective at integral y the energy with
 * mu(i, j) = the tree's path length between i and j. n_nodes <= 1024.
 * DCRF_EINVAL for a malformed tree or a negative or non-finite weight; a
 * batch context gives DCRF_EUNSUPPORTED. Waits for the stream. */
int dcrf_lp_subgradient_tree(dcrf_ctx *ctx, const void *unary, int L, const void *y,
                             int n_nodes, const int32_t *parent, const double *c, void *g,
                             double *S_lp);

/* Projected subgradient descent on eq. rHST-LP (Alg. rHST's loop), with the
 * tree as for dcrf_lp_subgradient_tree and the steps, outputs and limits of
 * dcrf_lp_descent. */
int dcrf_lp_descent_tree(dcrf_ctx *ctx, const void *unary, int L, void *y_inout,
                         int n_nodes, const int32_t *parent, const double *c, int steps,
                         double beta0, double *best_obj, void *best_y, double *hist);

/* Kleinberg and Tardos's rounding of marginals y (dev N x L) for the
 * uniform metric, the Potts model (Sec. 6 cites it for the LP relaxation's
 * factor-2 bound): round r = 0..R-1 carries a label round_label[r] (dev int32
 * R, in [0, L)) and a threshold round_theta[r] (dev R, context dtype),
 * which the caller draws uniform in [0, 1); each pixel takes the label of
 * the first round with y_a(label) > theta (compared in the context's
 * precision). So P(x_a = i) = y_a(i), and the expected energy is at most
 * phi^T y plus twice the LP's pairwise term. Pixels that no round reaches
 * take the argmax of y (lowest label on ties); *left (host, may be NULL)
 * receives their number (about N (1 - 1/L)^R). labels: (dev int32 N) out.
 * Waits for the stream. DCRF_EINVAL for a round label outside [0, L). */
int dcrf_round_kt(dcrf_ctx *ctx, const void *y, int L, const int32_t *round_label,
                  const void *round_theta, int R, int32_t *labels, int *left);

/* The labels with y_a(i) > tau at some pixel (y dev N x L), in increasing
 * order, into labels (host, L ints); *count (host) their number. The labels
 * "present in the solutions provided by other methods" of Sec. 7, to which
 * the LP can be restricted (App. I drops labels of small probability the
 * same way). Waits for the stream. */
int dcrf_present_labels(dcrf_ctx *ctx, const void *y, int L, double tau,
                        int32_t *labels, int *count);

/* The labels that a labelling uses (labels: dev int32 N, values in [0, L)),
 * in increasing order, into used (host, L ints); *count (host) their number:
 * the labels present in another method's solution, to which Sec. 7
 * restricts the LP. Waits for the stream. DCRF_EINVAL for a label outside
 * [0, L). */
int dcrf_labels_used(dcrf_ctx *ctx, const int32_t *labels, int L, int32_t *used,
                     int *count);

/* dcrf_lp_descent restricted to the labels subset[0..nsub-1] (host, distinct,
 * in [0, L)) (Sec. 7): the other labels are held at 0, which leaves their
 * terms of eq. potts-lp at 0, so the objective is the full S_LP of the
 * scattered point. The start is the Euclidean projection of y_inout's subset
 * columns onto the simplex; y_inout (dev N x L) receives the result with 0 in
 * the other columns; best_obj, best_y, hist as for dcrf_lp_descent. Each
 * step sorts and runs the divide and conquer for nsub labels instead of L.
 * A batch context gives DCRF_EUNSUPPORTED. */
int dcrf_lp_descent_subset(dcrf_ctx *ctx, const void *unary, int L, void *y_inout,
                           const int32_t *subset, int nsub, int steps, double beta0,
                           double *best_obj, void *best_y, double *hist);

/* y = Euclidean projection of each row of v onto the simplex (sort-based
 * rule). v, y: (dev) N x L; may be the same array. */
int dcrf_project_simplex(dcrf_ctx *ctx, const void *v, int L, void *y);

/* ---- differentiation of unrolled Frank-Wolfe ---------------------------- */

/* The pipeline y_T = FW^T(softmax(-phi)): T = `iters` >= 1 Frank-Wolfe
 * iterations on the QP (Sec. 4, App. B) started from y_0 = softmax(-phi)
 * row by row, made differentiable in phi and in the kernel weights w_m by a
 * reverse sweep over checkpoints (the step size alpha_t = -b1 / (2 a2) of the
 * exact line search is differentiated where it is interior to (0, 1); a
 * clipped step and the conditional gradient s_t are piecewise constant).
 * Lattice filter mode only (DCRF_EUNSUPPORTED in exact mode); L <= 32.
 *
 * *bytes (host) = the size of the checkpoint buffer for (L, iters) at the
 * context's image and precision: y_t and P_t = (Psi + D) y_t (T x N x L
 * values each), s_t (T x N int32), per lattice the blurred vertex values of
 * y_0 and of each one-hot s_t (T + 1 blocks of sum_m M_m x ld values, ld = L
 * rounded up to 16 bytes), and four doubles per iteration and image, each
 * part 256-byte aligned. L <= 32. */
int dcrf_fw_saved_size(dcrf_ctx *ctx, int L, int iters, size_t *bytes);

/* Forward: unary (dev N x L), mu (dev L x L or NULL); w (host, nk doubles,
 * >= 0, or NULL to keep the context's weights): the kernel weights w_m of
 * eq. pairwise, which stay set on the context afterwards (changing them
 * recomputes K'1, one filter call; the lattices do not depend on them);
 * y_out (dev N x L) = y_T; saved (dev, dcrf_fw_saved_size bytes,
 * caller-owned) receives the checkpoints that dcrf_fw_backward reads. */
int dcrf_fw_forward(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
                    const double *w, int iters, void *y_out, void *saved);

/* Backward: given dl/dy_T in grad_y (dev N x L), writes dl/dphi to
 * grad_unary (dev N x L); grad_w (host, nk doubles; B x nk for a batch,
 * image-major; may be NULL) receives each image's dl/dw_m, and grad_w_total
 * (host, nk doubles, may be NULL) their sum over the images, the gradient of
 * weights that the images share (equal to grad_w for one image). unary, mu,
 * L, iters and saved must be those of the forward call, and neither the
 * image nor the weights may have changed in between. The step adjoints are
 * formed on the device; the call waits for the stream once, at its end. */
int dcrf_fw_backward(dcrf_ctx *ctx, const void *unary, const void *mu, int L,
                     int iters, const void *saved, const void *grad_y,
                     void *grad_unary, double *grad_w, double *grad_w_total);

/* ---- benchmarking support ---------------------------------------------- */

/* Turn per-kernel timing on or off (and reset the counters). While on, the
 * launches of the hot kernels carry a pair of HIP events in their dispatch
 * (hipExtLaunchKernelGGL on the context's stream), so each interval is the
 * kernel's own execution time. */
int dcrf_set_profiling(dcrf_ctx *ctx, int enable);

/* Totals of kernel class k (0 <= k < 9): *name (static string, the kernel's
 * name), *total_ms (summed event time) and *launches. Waits for the stream.
 * Any output pointer may be NULL. */
int dcrf_get_profile(dcrf_ctx *ctx, int k, const char **name, double *total_ms,
                     long long *launches);

#ifdef __cplusplus
}
#endif

#endif /* DCRF_H */
