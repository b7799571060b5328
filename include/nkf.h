/*
 * nkf.h -- C ABI of the Nystrom kernel filtering library (MI355X / gfx950).
 *
 * The library computes the fast kernel filter of Nair & Chaudhury, "Fast
 * High-Dimensional Kernel Filtering": the bilateral / nonlocal-means filter of
 * Eq. (num) (Section II) with the range kernel replaced by its Nystrom
 * approximation K_hat = B^T A^{-1} B (Eqs. (hatK), (defA), (eigA), (defB),
 * (vk), Section III), evaluated as r_eff * (C + 1) spatial convolutions and a
 * per-pixel contraction and normalisation (Eqs. (finalnum), (finalden),
 * Algorithm 1).  Landmarks are k-means centroids of the guide values
 * (Section III).
 *
 * Notation: image f is [H, W, C] (C = n of the paper), guide p is [H, W, D]
 * (D = rho of the paper), N = H * W pixels, r landmarks (m0 of the paper).
 * Spatial kernel w(z) = w1(z1) w1(z2) on |z1|, |z2| <= S with
 * w1(t) = exp(-t^2 / (2 sigma_s^2)) (Gaussian) or w1 = 1 (box) -- Section IV.
 * Range kernel k(s, t) = exp(-|s - t|^2 / (2 sigma_r^2)).
 *
 * Conventions for every call:
 *  - Array pointers are DEVICE pointers owned by the caller unless the name
 *    ends in _host.  Layout is row-major, pixel-major, channel-contiguous:
 *    element (y, x, c) of an [H, W, C] array is at (y * W + x) * C + c.
 *    Images and guides are float32; host matrices are float64.
 *  - No pointer is retained after a call returns.
 *  - Device work is enqueued on the context's stream.  Unless stated
 *    otherwise a call returns as soon as its work is enqueued.
 *  - Errors are returned as nkf_status; nkf_last_error() gives a message.
 *    Arguments are validated before any work is enqueued; a call that fails
 *    validation has no effect.  No call aborts the process.
 *  - Sizes: H * W <= 2^31 (else NKF_ERR_INVALID_ARG), W <= 2^21 and
 *    C <= 1024 (else NKF_ERR_UNSUPPORTED).
 *  - Non-finite input pixels give unspecified output (not checked).
 *  - The image border is handled by intersecting the window with the image
 *    (zero extension of numerator and denominator alike).
 */
#ifndef NKF_H
#define NKF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nkf_ctx nkf_ctx;

typedef enum {
  NKF_OK = 0,
  NKF_ERR_INVALID_ARG = 1,   /* a size, pointer or parameter is out of range       */
  NKF_ERR_OUT_OF_MEMORY = 2, /* device/host allocation failed or workspace limit hit */
  NKF_ERR_HIP = 3,           /* a HIP runtime call failed                           */
  NKF_ERR_NUMERICAL = 4,     /* an eigensolver did not converge, or every eigenvalue
                                of A was truncated (r_eff == 0)                      */
  NKF_ERR_UNSUPPORTED = 5    /* valid request outside what this build implements    */
} nkf_status;

/* Spatial kernels.  GAUSSIAN and BOX are the truncated windows of radius S.
 * RECURSIVE is the O(1) recursive Gaussian of Young and van Vliet (Signal
 * Processing 44, 1995) that Section IV uses for the Gaussian window: their
 * third-order recursion run forwards and then backwards along each row and
 * column, with their fit of the scale q to sigma_s (0.5 <= sigma_s <= 200,
 * else NKF_ERR_INVALID_ARG).  Its response is not truncated (radius is
 * ignored) and approximates the Gaussian to within a few percent of its peak
 * (about 10% wider in variance).  The image is extended by zeros, so each
 * filtered line is that response convolved with the line.  Up to three
 * channels (else NKF_ERR_UNSUPPORTED).  nkf_filter_backward gives df, dp and
 * the sigma_r gradient through it (the filter is symmetric, so the adjoint
 * runs the same passes); its sigma_s gradient is NKF_ERR_UNSUPPORTED.  Work
 * and memory do not grow with sigma_s: the filtered planes take
 * r_eff (C + 1) H (W' + 32) floats of workspace
 * (W' = W rounded up to 64), plus the recursion's states at every 24 rows or
 * 32 columns and a copy of f. */
enum { NKF_SPATIAL_GAUSSIAN = 0, NKF_SPATIAL_BOX = 1, NKF_SPATIAL_RECURSIVE = 2 };
/* Guide kinds: EXPLICIT = caller passes p [H, W, D]; SELF = p is f (D == C);
 * PATCH = nonlocal-means guide, the (2pr+1)^2 * C patch of f around each pixel
 * in (dy, dx, c) order, read from a symmetrically padded f (Section II, NLM). */
enum { NKF_GUIDE_EXPLICIT = 0, NKF_GUIDE_SELF = 1, NKF_GUIDE_PATCH = 2 };
/* Input precision of the distance / embedding contraction (k-means assignment
 * and the cross kernel B).  FP32 is the plain form; BF16 and FP16 round the
 * centred guide and landmarks to 16 bits and accumulate in FP32, with the
 * squared norms kept in FP32/FP64 (the embedding's products as 16-bit hi + lo
 * pairs).  On up to three channels the Gaussian-window convolutions store
 * FP32 and accumulate each pass in FP64 in every form; on more channels the
 * plain form does the same per channel, and the 16-bit forms evaluate each
 * window as K_hat(x, y) = u(x).u(y) on the matrix cores (Eq. (num1) with
 * K_hat, 16-bit hi + lo embedding operands, FP32 sums) when r <= 64, and
 * like the plain form otherwise.  The box window on up to three channels keeps its window sums and
 * the contraction in FP64, with the embedding planes stored in FP64 in the
 * plain form and FP32 in the 16-bit forms. */
enum { NKF_PREC_FP32 = 0, NKF_PREC_BF16 = 1, NKF_PREC_FP16 = 2 };

typedef struct {
  double sigma_s;          /* spatial Gaussian width, > 0 (ignored by BOX except for radius = -1;
                              RECURSIVE: 0.5 .. 200)                                              */
  double sigma_r;          /* range kernel width, > 0; +INFINITY means k == 1                     */
  int r;                   /* landmarks, 1 <= r <= min(N, 256)                                  */
  int radius;              /* window radius S, 0 <= S <= 16; -1 means ceil(3 sigma_s); unused by
                              RECURSIVE                                                          */
  int spatial;             /* NKF_SPATIAL_*                                                      */
  int guide;               /* NKF_GUIDE_*                                                        */
  int patch_radius;        /* PATCH guide only: pr >= 0, D must equal C (2pr+1)^2                */
  int prec;                /* NKF_PREC_*                                                         */
  int kmeans_iters;        /* Lloyd iterations, >= 0                                             */
  uint64_t seed;           /* SplitMix64 seed of the k-means initialisation                      */
  double eig_rel_tol;      /* tau: eigenvalues alpha <= tau * max(alpha) are dropped (>= 0)      */
  double center;           /* f0 subtracted before and added after the filter (exact by affine
                              equivariance); NAN means per-channel (min + max) / 2 of f.  The
                              box window on C <= 3 sums in FP64 and needs no centring        */
} nkf_params;

/* Fills defaults: sigma_s 3, sigma_r 30, r 16, radius -1, Gaussian, SELF
 * guide, pr 3, FP32, 10 iterations, seed 0, tau 1e-10, center NAN. */
void nkf_params_default(nkf_params *p);

/* Library version string (static storage). */
const char *nkf_version(void);

/* Create a context bound to `hip_stream` (a hipStream_t; NULL = default stream)
 * on the current device.  The context owns a growable device workspace. */
nkf_status nkf_create(nkf_ctx **out, void *hip_stream);
nkf_status nkf_set_stream(nkf_ctx *ctx, void *hip_stream);
/* Waits for the context's stream, frees the workspace and the context. */
nkf_status nkf_destroy(nkf_ctx *ctx);
/* Message of the last failing call on `ctx` (or of the last failing
 * nkf_create / host-only call when ctx is NULL).  Valid until the next call. */
const char *nkf_last_error(const nkf_ctx *ctx);
/* Cap on the workspace size in bytes (0 = no cap).  A call that would need
 * more fails with NKF_ERR_OUT_OF_MEMORY before enqueuing work. */
nkf_status nkf_set_workspace_limit(nkf_ctx *ctx, size_t bytes);
/* Tile geometry of the Gaussian-window convolution kernels (forward and
 * backward; the box-window kernel has fixed tiles): each
 * block streams its output tile in chunks of rows, and by default the number
 * of chunks per tile is the largest that still gives enough blocks to fill
 * the GPU, so small images run one chunk per tile.  nch > 0 requests nch
 * chunks per tile (capped by each kernel's register budget and by the rows
 * the image has), e.g. to exercise the multi-chunk row ring of large images
 * on small ones; 0 restores the automatic choice.  Results are the same up to
 * rounding order.  NKF_ERR_INVALID_ARG for nch < 0. */
nkf_status nkf_set_conv_chunks(nkf_ctx *ctx, int nch);
/* Bytes of workspace currently held by the context. */
size_t nkf_workspace_bytes(const nkf_ctx *ctx);

/* ---------------------------------------------------------------------------
 * One-shot forward (Algorithm 1): k-means landmarks -> landmark factor ->
 * embedding -> r_eff (C+1) convolutions -> contraction and normalisation.
 * f [H, W, C]; p [H, W, D] for EXPLICIT, NULL for SELF / PATCH.
 * out [H, W, C] receives g_hat; eta_out (nullable) [H, W] receives eta_hat.
 * Pixels with eta_hat <= 0 or non-finite output f (the paper leaves this case
 * open).  Synchronises the stream once: the landmarks are copied to the host
 * for the FP64 eigendecomposition of A.  r_eff_out (nullable, host) receives
 * the number of kept eigenpairs.
 */
nkf_status nkf_filter(nkf_ctx *ctx, int H, int W, int C, const float *f, int D, const float *p,
                      const nkf_params *prm, float *out, float *eta_out, int *r_eff_out);

/* k-means landmarks (Section III): r distinct pixels drawn by SplitMix64
 * (prm->seed) give the initial centroids, then prm->kmeans_iters Lloyd
 * iterations (ties to the lowest index; an empty cluster keeps its centroid).
 * centroids [r, D] float32 (output); labels (nullable) [N] int32 receives the
 * assignment of the last iteration (left untouched when kmeans_iters == 0).
 * Asynchronous. */
nkf_status nkf_kmeans(nkf_ctx *ctx, int H, int W, int C, const float *f, int D, const float *p,
                      const nkf_params *prm, float *centroids, int *labels);

/* `iters` Lloyd iterations starting from the centroids already in
 * `centroids` [r, D] (in/out).  labels as in nkf_kmeans.  Asynchronous. */
nkf_status nkf_kmeans_iterate(nkf_ctx *ctx, int H, int W, int C, const float *f, int D,
                              const float *p, const nkf_params *prm, float *centroids, int iters,
                              int *labels);

/* PCA patch guide of PCA-NLM (Section IV: the NLM experiments reduce the
 * (2pr+1)^2 C patch values by PCA, e.g. 147 -> 25, before the range kernel).
 * f: device [H, W, C] float32.  The basis is estimated from the patches
 * ((dy, dx, channel) order, symmetric padding) of min(H*W, 65536) pixels: a
 * SplitMix64 partial Fisher-Yates draw from `seed` (as in nkf_seed_indices)
 * when H*W is larger, all pixels in order otherwise.  FP64 mean and
 * mean-centred covariance (1/n); the `dim` eigenvectors of the largest
 * eigenvalues, in descending order, each with its largest-magnitude entry
 * positive (the first on ties).  guide_out: device [H, W, dim] float32,
 * g(x)_k = (p(x) - mean) . v_k evaluated in FP64; pass it to nkf_filter as an
 * explicit guide with D = dim.  eigvals_host (nullable, host [dim]): the kept
 * eigenvalues.  Limits: (2pr+1)^2 C <= 256 (else NKF_ERR_UNSUPPORTED) and
 * 1 <= dim <= min((2pr+1)^2 C, 32) (else NKF_ERR_INVALID_ARG).  Synchronises
 * the stream once: the covariance is decomposed on the host (Householder
 * tridiagonalisation, its eigenvalues by implicit QR, the `dim` leading
 * eigenvectors by inverse iteration); NKF_ERR_NUMERICAL if that does not
 * converge. */
nkf_status nkf_patch_pca(nkf_ctx *ctx, int H, int W, int C, const float *f, int patch_radius, int dim,
                         uint64_t seed, float *guide_out, double *eigvals_host);

/* Host-only, synchronous, FP64.  Landmark Gram matrix A(i,j) = k(c_i, c_j)
 * (Eq. (defA)), its eigendecomposition A = Q diag(alpha) Q^T (Eq. (eigA)) by
 * Householder tridiagonalisation and implicit symmetric QR steps, truncation
 * of alpha <= tau * max(alpha), and the factor
 * F = Q_keep diag(alpha_keep^{-1/2}) so that u(x) = F^T b(x) gives
 * u(x).u(y) = b(x)^T A^+ b(y) = K_hat(x, y) (Eqs. (hatK), (vk)).
 * centroids_host [r, D]; eigvecs_host (nullable) [r, r], column j = q_j;
 * eigvals_host (nullable) [r] ascending; F_host [r, r] of which the first
 * *r_eff columns are written (columns follow ascending kept alpha).
 * Returns NKF_ERR_NUMERICAL when r_eff would be 0 or the eigensolver does not
 * converge. */
nkf_status nkf_landmark_factor(int r, int D, const double *centroids_host, double sigma_r,
                               double tau, double *eigvecs_host, double *eigvals_host,
                               double *F_host, int *r_eff);

/* Forward with given landmarks: embedding, convolutions, contraction.
 * centroids [r, D] float32 device; F [r, r_eff] float64 device (row-major, the
 * F of nkf_landmark_factor restricted to its first r_eff columns).
 * Fully asynchronous.  Other arguments as in nkf_filter. */
nkf_status nkf_filter_landmarks(nkf_ctx *ctx, int H, int W, int C, const float *f, int D,
                                const float *p, const nkf_params *prm, const float *centroids,
                                const double *F, int r_eff, float *out, float *eta_out);

/* nkf_filter_landmarks for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Same arguments, kernels and results as nkf_filter_landmarks,
 * but its scratch (the embedding planes, centring offsets, staged landmarks)
 * lives in a fixed 64 MiB device array that the library holds on each GPU it
 * runs on until the process ends; the call allocates nothing and never uses
 * the context's workspace.  The context supplies the stream and the device
 * (the array's address on that device is taken by nkf_create).  A problem
 * whose scratch exceeds 64 MiB (about r_eff * H * W * 4 bytes plus a few
 * hundred KiB) returns NKF_ERR_OUT_OF_MEMORY before any work is enqueued.
 * Every call on one GPU shares that GPU's array, whatever the context: calls
 * that overlap in time on one GPU (different streams, threads or contexts)
 * race on it and give undefined results; calls ordered on one stream are
 * safe.  Stage timing is not recorded for this call. */
nkf_status nkf_filter_landmarks_noalloc(nkf_ctx *ctx, int H, int W, int C, const float *f, int D,
                                        const float *p, const nkf_params *prm, const float *centroids,
                                        const double *F, int r_eff, float *out, float *eta_out);

/* Backward of nkf_filter_landmarks for L with dL/dg_hat = grad_out [H, W, C],
 * landmarks held fixed and the window radius S held fixed.
 * eigvecs_host [r, r] / eigvals_host [r] as returned by nkf_landmark_factor
 * for the same centroids and sigma_r; r_eff must equal r when
 * grad_sigma_r_host is requested (else NKF_ERR_UNSUPPORTED).
 * Outputs (each nullable): grad_f [H, W, C], grad_p [H, W, D] (EXPLICIT or
 * SELF guide; for SELF the caller adds grad_f and grad_p to get the total),
 * grad_sigma_r_host, grad_sigma_s_host (host doubles; sigma_s only for the
 * truncated Gaussian window).  Recomputes the embedding instead of storing
 * r_eff (C+1) planes.  out_fwd [H, W, C] and eta_fwd [H, W] (both nullable,
 * device) are the out and eta_out of the nkf_filter_landmarks call with the
 * same arguments; when both are given the forward convolutions are not
 * repeated (the caller guarantees they match), otherwise they are recomputed
 * (always for the recursive Gaussian, whose backward reads the forward's
 * filtered planes).
 * Synchronises the stream (the r x r_eff reduction for the sigma_r gradient
 * is finished on the host in FP64). */
nkf_status nkf_filter_backward(nkf_ctx *ctx, int H, int W, int C, const float *f, int D,
                               const float *p, const nkf_params *prm, const float *centroids,
                               const double *eigvecs_host, const double *eigvals_host, int r_eff,
                               const float *grad_out, float *grad_f, float *grad_p,
                               double *grad_sigma_r_host, double *grad_sigma_s_host,
                               const float *out_fwd, const float *eta_fwd);

/* Stage timing.  When enabled, every stage a call enqueues is bracketed by
 * HIP events on the context's stream (host-side stages by the host clock).
 * Stages: 0 seeding, 1 k-means iterations, 2 landmark factor (host FP64,
 * from the landmarks' arrival on the host to the queued copy of F; nkf_filter
 * runs the centring on the device meanwhile), 3 embedding (with the centring
 * in nkf_filter_landmarks), 4 convolutions + contraction, 5 backward.  Timing
 * adds no synchronisation to a call. */
enum { NKF_STAGE_SEED = 0, NKF_STAGE_KMEANS = 1, NKF_STAGE_FACTOR = 2, NKF_STAGE_EMBED = 3,
       NKF_STAGE_CONV = 4, NKF_STAGE_BACKWARD = 5, NKF_STAGE_COUNT = 6 };
nkf_status nkf_enable_timing(nkf_ctx *ctx, int enable);
/* Waits for the stream, then writes the summed milliseconds per stage to
 * ms_host[NKF_STAGE_COUNT] and (nullable) the number of timed intervals to
 * count_host[NKF_STAGE_COUNT] since the last reset; reset != 0 clears them. */
nkf_status nkf_stage_times(nkf_ctx *ctx, double *ms_host, int *count_host, int reset);

/* Statistics of the last forward call on a context (nkf_filter or
 * nkf_filter_landmarks; not the allocation-free call nor the backward's
 * recompute), for diagnosing the cases the paper leaves open: the number of
 * kept eigenpairs of A and its conditioning (Section III: A may be
 * ill-conditioned; eigenvalues at or below tau * alpha_max are dropped), and
 * the pixels whose eta_hat was <= 0 or not finite, where the output is f.
 * Off by default; with it on, each forward call adds one small reduction over
 * eta_hat (and keeps its own eta_hat copy when eta_out is NULL).  Setting the
 * environment variable NKF_LOG (non-empty, not "0") when a context is created
 * turns it on and prints the record of every forward call to stderr (each
 * call then waits for its stream). */
typedef struct {
  int valid;               /* 1 when a forward call has been recorded since the last enable */
  int r, r_eff;            /* landmarks and kept eigenpairs                                     */
  double alpha_max;        /* largest eigenvalue of A (NAN: the caller supplied F)              */
  double alpha_min_kept;   /* smallest kept eigenvalue (NAN as above)                           */
  double cond_kept;        /* alpha_max / alpha_min_kept                                         */
  long long pixels;        /* H * W                                                              */
  long long guarded;       /* pixels with eta_hat <= 0 or not finite (output = f)               */
  double min_eta;          /* smallest positive finite eta_hat (NAN if none)                    */
} nkf_stats;
/* enable != 0 turns the statistics on (allocates an 8-byte device buffer
 * once), 0 turns them off; either clears the record. */
nkf_status nkf_enable_stats(nkf_ctx *ctx, int enable);
/* Copies the record of the last forward call to *out, waiting for the stream
 * for the eta_hat part.  out->valid == 0 when none has been recorded. */
nkf_status nkf_get_stats(nkf_ctx *ctx, nkf_stats *out);

/* Host-only: the r distinct pixel indices (draw order) that initialise
 * k-means for (N, r, seed): partial Fisher-Yates over [0, N) driven by
 * SplitMix64.  idx_host [r].  Exposed so the draw can be checked. */
nkf_status nkf_seed_indices(int64_t N, int r, uint64_t seed, int64_t *idx_host);

/* Host-only: the window radius the library uses for (radius, sigma_s) and
 * the one-dimensional taps w1[0 .. 2S] (float32, as uploaded).  taps_host
 * nullable; returns S via *S_out.  NKF_ERR_UNSUPPORTED for RECURSIVE, which
 * has no taps. */
nkf_status nkf_spatial_taps(int radius, double sigma_s, int spatial, int *S_out, float *taps_host);

#ifdef __cplusplus
}
#endif

#endif /* NKF_H */
