/*
 * fepll.h -- C ABI of the MI355X (gfx950) EPLL denoising library.
 *
 * The library restores an image y = x + w (white Gaussian noise of standard
 * deviation sigma, A = identity) under a zero-mean Gaussian-mixture prior on
 * DC-removed 8x8 patches, by half-quadratic splitting: every iteration runs
 * the five steps of Algorithm 1 of Parameswaran, Deledalle, Denis & Nguyen,
 * "Accelerating GMM-based patch priors for image restoration: three
 * ingredients for a 100x speed-up" (arXiv 1710.08124) -- patch extraction,
 * Gaussian selection, patch estimation, patch reprojection, image
 * estimation -- with selection and estimation in each component's
 * eigenbasis (Sec. 2.1, Eq. (7) / Eq. (8)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - A patch is the 8x8 block whose top-left pixel is (r, c); its vector index
 *   is 8*dy + dx.  The patch set is every block fully inside the image,
 *   Np = (H-7)*(W-7) patches, numbered r*(W-7) + c.
 * - Images are float32, row-major, `row_stride` elements between rows.
 * - GMM parameters come in float64 (they are set up once); the hot path runs
 *   in float32 (or bf16 / fp8 for the projections, see fepll_options).
 * - The "cost" of component k for a patch is the selection objective of
 *   Alg. 1, iota_k + sum_j (log nu_kj + c_j^2 / nu_kj), c = U_k^t z~,
 *   iota_k = -2 log w_k, nu_kj = lambda_kj + 1/beta.  The chosen component is
 *   the smallest cost, ties going to the lowest index.
 * - Every call returns a fepll_status; on failure nothing the caller owns has
 *   been written unless stated, and fepll_last_error() gives a message
 *   (thread-local, valid until the next call on the same thread).
 * - Calls on the same fepll_gmm handle must not run concurrently (the handle
 *   owns the scratch memory the restoration uses).
 * - Device work is enqueued on fepll_options.stream (a hipStream_t; NULL =
 *   the default stream).  Entry points that take host buffers synchronise the
 *   stream before returning; entry points that take only device buffers do
 *   not, unless stated.
 */
#ifndef FEPLL_H
#define FEPLL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fepll_gmm fepll_gmm; /* opaque; owns its device copies */

typedef enum {
  FEPLL_OK = 0,
  FEPLL_EINVAL = -1,       /* an argument is out of its documented range   */
  FEPLL_ENOMEM = -2,       /* a device or host allocation failed            */
  FEPLL_EDEVICE = -3,      /* a HIP runtime call failed                     */
  FEPLL_EUNSUPPORTED = -4, /* a valid request the library does not implement */
  FEPLL_ECHECKSUM = -5     /* a serialized blob failed its integrity check  */
} fepll_status;

enum { FEPLL_FP32 = 0, FEPLL_BF16 = 1, FEPLL_FP8 = 2 };

typedef struct {
  float* data;         /* first pixel                                   */
  int32_t height;      /* H >= 8                                        */
  int32_t width;       /* W >= 8                                        */
  int64_t row_stride;  /* elements between rows, >= width               */
  int32_t on_device;   /* 1: data is device memory, 0: host memory      */
} fepll_image;

typedef struct {
  /* Arithmetic of the projection c = U_k^t z~ in the selection step:
   * FEPLL_FP32 (default), FEPLL_BF16, or FEPLL_FP8 (OCP e4m3 operands with a
   * power-of-two scale per component and per patch that brings the largest
   * magnitude to at most 448), always with float32 accumulation;
   * log-determinant terms, patch estimation, reprojection and image
   * estimation stay float32.  The proposal path needs FEPLL_BF16.         */
  int32_t precision;
  /* FEPLL_FP32 only: every patch whose float32 selection is not certified
   * by the rounding-error bound of its costs is re-selected in float64, so
   * the labels equal those of an exact evaluation (default 1).             */
  int32_t recheck;
  /* Learned proposal (needs fepll_gmm_load_proposal): score only the top_m
   * components proposed by the network, fall back to all K when half the
   * exact gap between the two best proposed costs is below margin_nats.    */
  int32_t use_proposal;
  int32_t top_m;          /* 1..K, default 8                                */
  double margin_nats;     /* default 0.5; +inf = always fall back           */
  /* Start of the iterations; NULL = y (Alg. 1 starts from x = y).          */
  const fepll_image* init;
  void* stream;           /* hipStream_t; NULL = default stream             */
  /* Stage timing (forces an eager run, no graph): bracket kernel stages
   * with HIP events on `stream` and accumulate their times in the handle
   * (read with fepll_profile).  0 = off; 1 (bit 0) = every stage; else bit
   * s + 1 set = stage s timed (the stages of fepll_profile), so that a
   * run can time one stage with two events per launch.  EINVAL when
   * negative or above bit 9.                                               */
  int32_t profile;
  /* Jittered stochastic patch subsampling (Sec. 3.3): 0 (default) = every
   * patch; s in 1..8 = each iteration runs on the patches of a grid of
   * spacing s, shifted as a whole at random and each point moved uniformly
   * by at most floor((8 - s) / 2) pixels per direction, clamped so that
   * every pixel stays covered, drawn again at every iteration; the
   * reprojection averages the chosen patches only.  Random numbers:
   * Philox4x32-10 keyed by `seed` (low word, high word), counter
   * (t, grid row, grid column, 0) for a point's offsets (word 0 rows, word 1
   * columns) and (t, 0xffffffff, 0xffffffff, 0) for the shift; uniform
   * integers as a word modulo their range.  Every image of a batch uses the
   * same seed.  Not with use_proposal (EUNSUPPORTED), nor in fepll_select.
   * labels_out gives K for the patches not chosen.                        */
  int32_t jitter;
  uint64_t seed;
  /* Nonzero: Gaussian selection by the search tree of fepll_gmm_set_tree
   * (Sec. 3.2): from the root, each patch follows the child of smallest
   * selection cost down to a leaf.  Needs FEPLL_BF16 (the costs are those of
   * the bfloat16 selection, flat-tailed with the mixture); not with
   * use_proposal or jitter (EUNSUPPORTED).                                 */
  int32_t use_tree;
} fepll_options;

/* Fill *opt with the defaults above. */
void fepll_options_default(fepll_options* opt);

/*
 * Create a GMM handle from the eigendecomposition Sigma_k = U_k S_k U_k^t
 * (Sec. 2.1, computed offline in the paper).
 *   U:      K x d x d float64, host, row-major: U[(k*d + p)*d + j] is entry p
 *           of the j-th eigenvector of Sigma_k (columns are eigenvectors);
 *           each U_k must be orthonormal (max |U^t U - I| <= 1e-8).
 *   lambda: K x d float64, host, the diagonal of S_k, finite and >= 0.
 *   w:      K float64, host, the mixture weights (Eq. (2)): w_k > 0 and
 *           |sum w - 1| <= 1e-6 (never renormalised).
 *   K:      1..1024.   d: must be 64 (8x8 patches).
 * The library copies what it keeps.  EINVAL on any violated condition,
 * ENOMEM / EDEVICE on allocation or copy failure; *out is set only on OK.
 */
fepll_status fepll_gmm_create(const double* U, const double* lambda, const double* w,
                              int32_t K, int32_t d, fepll_gmm** out);

/*
 * Create a GMM handle from the covariances (the eigendecomposition of
 * Sec. 2.1 is done here, in float64, by the cyclic Jacobi method).
 *   Sigma: K x d x d float64, host, row-major, each symmetric (1e-9 of its
 *          largest entry) and positive semidefinite (eigenvalues below
 *          -1e-10 of the largest rejected; smaller negative ones set to 0).
 *   w, K, d: as fepll_gmm_create.
 * EINVAL on a violated condition, otherwise as fepll_gmm_create.
 */
fepll_status fepll_gmm_create_from_cov(const double* Sigma, const double* w, int32_t K,
                                       int32_t d, fepll_gmm** out);

/*
 * The float64 eigendecomposition used by fepll_gmm_create_from_cov, on the
 * host only (no device is touched): U (K x d x d, column j of U_k the j-th
 * eigenvector) and lambda (K x d, decreasing) receive Sigma_k = U_k
 * diag(lambda_k) U_k^t.  d in 1..1024.  Same conditions as above.
 */
fepll_status fepll_cov_eig(const double* Sigma, int32_t K, int32_t d, double* U,
                           double* lambda);

/*
 * Flat-tail spectrum approximation (Sec. 3.1) of the mixture, for every
 * later call on the handle.  In each component, r_k is the smallest rank
 * whose r_k largest eigenvalues hold at least rho of the trace (sums taken
 * in index order), and the 64 - r_k smaller eigenvalues are replaced by
 * their average.  Restoration is then EPLL with these spectra: the FEPLL_FP32
 * selection stays exact (certified) for them; the FEPLL_BF16 / FEPLL_FP8
 * selections and the proposal's rescoring take Sec. 3.1's rewritten cost,
 * projecting each patch on only the r_k leading eigenvectors plus one
 * squared norm of the DC-removed patch, |z~|^2 / nu_P.  rho = 1 restores the
 * spectra as created (no approximation).  Each call starts from the
 * spectra as created (calls do not compound).
 *   rho:   in (0, 1]; anything else (NaN included) returns EINVAL.
 *   ranks: NULL or K int32 (host) receiving r_k (64 for every component
 *          when rho = 1).
 * Synchronises the device (tables and captured work of earlier calls read
 * the spectra).  EDEVICE / ENOMEM on a device failure.
 */
fepll_status fepll_gmm_flat_tail(fepll_gmm* g, double rho, int32_t* ranks);

/*
 * Search tree of the mixture (Sec. 3.2), for options.use_tree.
 *   nlevels: levels of the tree, 2..16, the root first; 0 removes the tree.
 *   sizes:   nlevels node counts: sizes[0] = 1 (the root), sizes[nlevels-1]
 *            = K (the leaves are the mixture's components, in order).
 *   parents: for each level n = 1..nlevels-1 in turn, sizes[n] int32 giving
 *            the node of level n-1 that each node of level n belongs to;
 *            every node above the leaves has 1..8 children.
 * The nodes above the leaves are zero-mean Gaussians made from the leaves
 * by moment matching (weights summed, covariances averaged with the
 * weights), level by level, and eigendecomposed in float64 on the host; the
 * flat tail of fepll_gmm_flat_tail applies to them as to the leaves.  A
 * balanced tree is built offline (e.g. by paper_1710_08124_amd.tree).
 * EINVAL on a malformed tree.  Synchronises the device.
 */
fepll_status fepll_gmm_set_tree(fepll_gmm* g, int32_t nlevels, const int32_t* sizes,
                                const int32_t* parents);

/* Release a handle (NULL is a no-op).  Synchronises the device first. */
void fepll_gmm_destroy(fepll_gmm* g);

/* Degradation operator A of the restoration problem (Sec. 2: y = A x + n). */
enum { FEPLL_OP_IDENTITY = 0, FEPLL_OP_CONVOLUTION = 1 };
typedef struct {
  int32_t kind;         /* FEPLL_OP_IDENTITY or FEPLL_OP_CONVOLUTION          */
  /* FEPLL_OP_CONVOLUTION: periodic convolution with a centred kernel,
   * (A x)[i, j] = sum_{u,v} kernel[u * kw + v] x[i - (u - kh/2), j - (v - kw/2)]
   * (indices modulo the image size); kh, kw odd, at most the image's
   * height and width; kernel: host float32, finite.                        */
  int32_t kh, kw;
  const float* kernel;
} fepll_operator;

/*
 * Restore y by T iterations of Alg. 1.
 *   y:      degraded image (host or device).  Finite values only (EINVAL).
 *   H:      the degradation operator A: NULL or FEPLL_OP_IDENTITY for
 *           denoising; FEPLL_OP_CONVOLUTION for deblurring, where the image
 *           estimation (A^t A + beta sigma^2 I)^-1 (A^t y + beta sigma^2 x~)
 *           is solved with float64 FFTs, the default schedule is
 *           beta = lambda sigma^-2 {1, 4, 8, 16, 32} with lambda =
 *           min(|A^t A|_F^2 / (N |A|_2^2), 250 sigma^2) and the default
 *           start (options.init NULL) is (A^t A + 0.2 sigma^2 / lambda Lap)^-1
 *           A^t y, Lap the periodic 5-point Laplacian (Sec. 5, "Parameter
 *           settings"); runs without graph capture.
 *   sigma:  noise standard deviation on the image's scale, > 0.
 *   beta_schedule: T absolute values of beta (the HQS coupling weight of
 *           Eq. (3)), each > 0; NULL = {1, 4, 8, 16, 32} / sigma^2 (denoising,
 *           lambda = 1) with T = 5 (T must then be 5 or 0, where 0 means 5).
 *   T:      1..16 iterations.
 *   out:    H x W output (host or device); may alias y.
 *   opt:    NULL = defaults.
 *   labels_out: optional int32 buffer of T * Np entries, iteration-major; in
 *           the same memory space as y; receives the chosen component of
 *           every patch at every iteration.
 * Host images are copied in and out and the call returns after the result
 * is in `out`.  Device images: the work is enqueued and the call returns.
 */
fepll_status fepll_restore(fepll_gmm* g, const fepll_image* y, const fepll_operator* H,
                           double sigma, const double* beta_schedule, int32_t T,
                           fepll_image* out, const fepll_options* opt, int32_t* labels_out);

/*
 * Restore n independent images, each by the default schedule (T = 5,
 * beta = {1, 4, 8, 16, 32} / sigma[i]^2, start x = y) of Alg. 1 with A =
 * identity -- the same result per image as fepll_restore.
 *   n:      1..65536 images, of any sizes (each >= 8 x 8).
 *   y:      n noisy images (host or device, finite values).
 *   sigma:  n noise levels (host), each > 0: every image has its own betas.
 *   out:    n outputs, each of the shape of its y; out[i] may alias y[i].
 *   opt:    NULL = defaults; options.init must be NULL.
 * The images are packed one after the other in device memory and every
 * stage of an iteration is one launch over all of them (the all-K
 * bfloat16 / e4m3 selection as a persistent launch over the selection
 * tiles of the batch; float32 and proposal selection image by image).
 * Without options.profile the launch sequence of the 5 iterations is
 * captured once as a HIP graph and replayed by later calls with the same
 * sizes, noise levels and options.  Host images: the call returns after
 * every result is in out.  Device images: the work is enqueued.
 */
fepll_status fepll_restore_batch(fepll_gmm* g, int32_t n, const fepll_image* y,
                                 const double* sigma, fepll_image* out,
                                 const fepll_options* opt);

/* Launch shapes of the restoration kernels (per handle). */
typedef struct {
  int32_t est_blocks;    /* workgroups of the persistent selection launch;
                            0 = one per tile (default 768: 3 per CU)       */
  int32_t wiener_blocks; /* cap on the patch-estimation workgroups, a
                            multiple of 8 (default 4096)                   */
  int32_t ola_rows;      /* rows of a reprojection tile: 16 (default), 32
                            or 64                                          */
  int32_t reserved;      /* 0                                              */
} fepll_tuning;

/* Set the launch shapes (NULL = defaults).  EINVAL when out of range. */
fepll_status fepll_set_tuning(fepll_gmm* g, const fepll_tuning* t);
fepll_status fepll_get_tuning(fepll_gmm* g, fepll_tuning* t);

/*
 * Autotuner: time every candidate launch shape of each stage (selection
 * workgroups 0 / 512 / 768 / 1024, patch-estimation workgroups 1024 / 2048 /
 * 4096 / 8192, reprojection rows 16 / 32 / 64) on a restoration of the given
 * batch (arguments as fepll_restore_batch; the results are discarded), keep
 * the fastest of each stage in the handle and return them in *best (may be
 * NULL).  Synchronises.
 * Tuning cache: when the environment variable FEPLL_TUNING_CACHE names a
 * file, a result found there for the same device, precision and selection
 * path, K, flat tail and batch shape class (image count, total and largest
 * image size, each rounded down to a power of two) is applied without any
 * trial, and a new result is appended to it (one text line per workload; a
 * file that cannot be read or written is no error).
 */
fepll_status fepll_autotune(fepll_gmm* g, int32_t n, const fepll_image* y,
                            const double* sigma, const fepll_options* opt,
                            fepll_tuning* best);

/*
 * One Gaussian-selection step (Alg. 1, "Gaussian selection", eigenspace
 * form) on every patch of the device image x for one beta, without
 * estimation or reprojection.  Device buffers of Np entries each:
 *   labels (int32, required), best and second (float32, optional: the two
 *   smallest costs scored), flags (int32, optional: FEPLL_FP32 -- 1 where the
 *   float32 selection was not certified and, with recheck on, was redone in
 *   float64; with options.use_proposal -- 1 where the patch fell back to the
 *   full-K search; otherwise 0).
 * Used to check the selection against an exact evaluation and to record
 * the labels the proposal network is trained on.
 */
fepll_status fepll_select(fepll_gmm* g, const fepll_image* x, double beta,
                          int32_t* labels, float* best, float* second, int32_t* flags,
                          const fepll_options* opt);

/*
 * fepll_select in float32 (options: FEPLL_FP32, recheck on, the other
 * defaults), allocating no device memory: for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * it).  Same labels, costs and flags as fepll_select, bit for bit.
 * x: a device image, contiguous (row_stride 0 or width), on the handle's
 * device, which must be current.  labels / best / second / flags: device
 * buffers of Np = (H - 7)(W - 7) entries as in fepll_select (best, second,
 * flags optional).  Asynchronous on stream (NULL: the default stream).
 * Scratch: one 32 MiB device array per GPU inside the library, held until
 * the process ends; a call takes the per-beta tables, 33 300 bytes per
 * component (6.7 MB at K = 200), and 16 bytes per patch for the list of
 * uncertified patches (16.5 MB at 1024 x 1024), each region rounded up to
 * 256 bytes; a call that needs more returns EINVAL.  Every call on a GPU uses that
 * GPU's one array: calls that overlap on one GPU (other streams or threads)
 * race, the caller serialises them.
 * Errors: EINVAL (NULL handle or buffers, host or strided image, size < 8,
 * beta <= 0, not the handle's device, scratch exceeded), EDEVICE.
 */
fepll_status fepll_select_static(fepll_gmm* g, const fepll_image* x, double beta,
                                 int32_t* labels, float* best, float* second, int32_t* flags,
                                 void* stream);

/*
 * Stage timing of the calls made with options.profile set since the last
 * read.  Stages: 0 selection (E-step; with the proposal: exact rescoring of
 * the candidates), 1 float64 re-selection, 2 bucketing, 3 patch
 * estimation, 4 reprojection + image estimation, 5 per-beta constants,
 * 6 proposal network, 7 full-K selection of the fallback patches, 8 the
 * jittered patch subset (positions, list, and the merge of a selection
 * split over components).  ms[s] receives the summed event time of stage s
 * in milliseconds and launches[s] the number of timed launches (either
 * pointer may be NULL); n is the number of entries provided (at most 9 are
 * written).
 * Synchronises with the recorded events, then clears the accumulators.
 */
fepll_status fepll_profile(fepll_gmm* g, double* ms, int32_t* launches, int32_t n);

/* ------------------------------------------------------------------------
 * Component-proposal network.  Not part of the paper: the paper limits the
 * components scored by a search tree (Sec. 3.2) and reviews a gating network
 * that approximates the selection score (Sec. 4); here a network
 * [z~/128, log sigma_beta] (65) -> 256 -> 256 -> K, tanh-form GELU after the
 * hidden layers, proposes components that the selection step then rescores
 * with the exact cost.  Parameters are one float32 vector
 * W1 (256x65) b1 (256) W2 (256x256) b2 (256) W3 (Kx256) b3 (K), every W
 * stored (out, in) row-major.  All buffers below are device memory unless
 * stated; work is enqueued on `stream` (hipStream_t, NULL = default).
 * ---------------------------------------------------------------------- */
typedef struct fepll_mlp fepll_mlp;

typedef struct {
  double lr, beta1, beta2, eps, weight_decay; /* AdamW, decoupled decay */
} fepll_adamw;

/* Number of float32 parameters of the network for K components. */
int64_t fepll_mlp_param_count(int32_t K);

/* Create a network with K outputs (1..1024) from `params` (host,
 * fepll_mlp_param_count(K) floats); max_batch (>= 1) bounds the rows of
 * one loss/gradient evaluation (forward passes are chunked). */
fepll_status fepll_mlp_create(int32_t K, const float* params, int32_t max_batch,
                              fepll_mlp** out);
void fepll_mlp_destroy(fepll_mlp* m);

/* Copy the current parameters to host memory (synchronises). */
fepll_status fepll_mlp_get_params(fepll_mlp* m, float* params);

/* logits (n x K, float32) of the n feature rows X (n x 65, float32). */
fepll_status fepll_mlp_forward(fepll_mlp* m, const float* X, int32_t n, float* logits,
                               void* stream);

/* Mean softmax cross-entropy of X against labels (n <= max_batch rows,
 * int32 in 0..K-1) into *loss (device float, optional) and its gradient
 * into grads (device, param_count floats, optional). */
fepll_status fepll_mlp_loss_grad(fepll_mlp* m, const float* X, const int32_t* labels,
                                 int32_t n, float* grads, float* loss, void* stream);

/* One AdamW step on a minibatch of n <= max_batch rows; *loss as above.
 * rows == NULL: the first n rows of X / labels; otherwise rows (device,
 * n int32) lists the rows of X / labels that form the minibatch. */
fepll_status fepll_mlp_train_step(fepll_mlp* m, const float* X, const int32_t* labels,
                                  const int32_t* rows, int32_t n, const fepll_adamw* hp,
                                  float* loss, void* stream);

/* Network input of every patch of the device image x at coupling beta:
 * X (Np x 65 float32) row i = [z~_i / 128, -0.5 log beta], z~_i the
 * DC-removed patch i (numbered as in fepll_restore). */
fepll_status fepll_features(const fepll_image* x, double beta, float* X, void* stream);

/* Serialize the parameters into buf (host): a 64-byte header (magic
 * "FEPLLMLP", version, K, widths, input scale, GELU variant, parameter
 * count, FNV-1a-64 checksum of the parameter bytes) followed by the
 * parameters.  With buf = NULL only *nbytes is set.  Synchronises. */
fepll_status fepll_mlp_serialize(fepll_mlp* m, void* buf, size_t cap, size_t* nbytes);

/* Attach a serialized network to a mixture for options.use_proposal.
 * EINVAL on a malformed header or a K different from the mixture's,
 * ECHECKSUM when the checksum does not match. */
fepll_status fepll_gmm_load_proposal(fepll_gmm* g, const void* blob, size_t nbytes);

/* The top_m (1..8) components the attached network proposes for every
 * patch of the device image x at coupling beta: cand (device, Np x 8
 * uint16) row i lists them by decreasing logit (ties to the lower index),
 * 0xffff after the top_m-th.  EINVAL without a loaded network. */
fepll_status fepll_propose(fepll_gmm* g, const fepll_image* x, double beta, int32_t top_m,
                           uint16_t* cand, void* stream);

/* Message of the last failed call on this thread ("" if none). */
const char* fepll_last_error(void);

/* Library version string. */
const char* fepll_version(void);

/*
 * Device memory the library holds (every handle's buffers and scratch, in
 * bytes), and a cap on it for testing the out-of-memory paths: once set
 * (limit_bytes > 0; 0 removes it), an allocation that would take the
 * holdings past the cap fails as on a full device: the call returns
 * FEPLL_ENOMEM and leaves its outputs unwritten; the handle stays usable
 * (buffers it grew before the failure stay with it until a later call or
 * fepll_gmm_destroy frees them).  Process-wide.
 */
fepll_status fepll_set_memory_limit(size_t limit_bytes);
size_t fepll_memory_in_use(void);

#ifdef __cplusplus
}
#endif

#endif /* FEPLL_H */
