// Internal declarations shared by the host runtime and the HIP kernels of the
// Nystrom kernel filtering library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nkf {

enum GuideKind { GUIDE_EXPLICIT = 0, GUIDE_SELF = 1, GUIDE_PATCH = 2 };

// Where the guide value p(x)[d] comes from: an explicit [N, D] array, the
// image itself (D == C), or the (2pr+1)^2 C patch of f read with symmetric
// padding in (dy, dx, c) order.
struct Guide {
  int kind;
  const float *p;   // EXPLICIT
  const float *f;   // SELF / PATCH
  int H, W, C, D, pr;
};

// Window radius limit of the convolution kernels (T = 2S+1 <= 33 taps).
constexpr int kMaxRadius = 16;
constexpr int kMaxLandmarks = 256;
constexpr int kMaxGuideDim = 256;  // D

struct Taps {
  float w[2 * kMaxRadius + 1];
};

// ---- kernels_kmeans.hip -----------------------------------------------------
hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t s);
hipError_t launch_gather_landmarks(const Guide &g, const int64_t *idx, int r, float *c,
                                   hipStream_t s);
// Size (doubles) of the per-block partial-sum buffer of one Lloyd step.
size_t kmeans_partials_doubles(int r, int D);
// Size (floats) of the landmark scratch of the FP32 assignment: the transposed
// copy [D][r rounded up to 8] of the VALU kernel, or the prepared FP32 tile of
// the matrix-core kernel, whichever is larger.
size_t kmeans_transposed_floats(const Guide &g, int r);
// One Lloyd iteration in place on c [r, D]: assignment (labels nullable),
// per-block cluster sums into `partials`, ordered reduction and mean update;
// ct is scratch of kmeans_transposed_floats(g, r) floats.
hipError_t launch_kmeans_step(const Guide &g, float *c, int r, double *partials, int *labels,
                              int *label_scratch, float *ct, hipStream_t s);

// ---- kernels_mfma.hip -------------------------------------------------------
// FP32 form, D > 32: labels of every pixel from the FP32 products on the matrix
// cores (v_mfma_f32_16x16x4f32), when the FP32 landmark tile fits in LDS;
// scratch holds assign_mfma32_scratch_floats(g, r) floats.
bool assign_mfma32_supported(const Guide &g, int r);
size_t assign_mfma32_scratch_floats(const Guide &g, int r);
hipError_t launch_assign_mfma32(const Guide &g, const float *c, int r, int *labels, float *scratch,
                                hipStream_t s);
// Distance step on MFMA with 16-bit centred operands (prec 1 = BF16, 2 = FP16).
// Whether the LDS plan of the 16-bit path fits this guide and landmark count.
bool mfma_path_supported(const Guide &g, int r, int prec);
// Centring offsets mu ([C] for patch guides, else [D]); scratch holds
// guide_mean_scratch_doubles(g) doubles.
size_t guide_mean_scratch_doubles(const Guide &g);
hipError_t launch_guide_mean(const Guide &g, float *mu, double *scratch, hipStream_t s);
// Device scratch (bytes) for the prepared 16-bit landmarks of one launch.
size_t mfma_landmark_scratch_bytes(const Guide &g, int r);
// Assignment fused with the per-cluster sums of the centred guide values:
// per-block FP64 partials [*nparts][r][D+1] (at most 256 blocks); labels nullable.
hipError_t launch_lloyd_mfma(const Guide &g, const float *c, int r, const float *mu, int prec, double *partials,
                             int *labels, int *nparts, void *lm_scratch, hipStream_t s);
hipError_t launch_embed_mfma(const Guide &g, const float *c, int r, const float *mu, const double *F,
                             float *F32, int r_eff, double sigma_r, int prec, float *u, void *lm_scratch,
                             hipStream_t s);
// The 16-bit embedding in two launches: the cross-kernel tiles b (landmarks
// only; they can run while the host decomposes A) into bbuf, then the mix
// u = F^T b from them.  bbuf holds embed_split_floats(g, r, prec) floats.
size_t embed_split_floats(const Guide &g, int r, int prec);
hipError_t launch_embed_mfma_b(const Guide &g, const float *c, int r, const float *mu, double sigma_r, int prec,
                               float *bbuf, void *lm_scratch, hipStream_t s);
hipError_t launch_embed_mfma_mix(const Guide &g, int r, const double *F, float *F32, int r_eff, int prec, float *u,
                                 const float *bbuf, hipStream_t s);
// One Lloyd step whose assignment runs on MFMA (labels nullable).
hipError_t launch_kmeans_step_mfma(const Guide &g, float *c, int r, const float *mu, int prec, double *partials,
                                   int *labels, void *lm_scratch, hipStream_t s);
// Whether the 16-bit MFMA distance path serves this guide / precision.
inline bool use_mfma_distance(const Guide &g, int prec) { return prec != 0 && g.D > 8; }
// The 16-bit forms' k-means takes the matrix cores from D > 32; below, one
// 32-wide K step and half-empty landmark tiles make the FP32 VALU assignment
// (also the more exact one) the faster.
inline bool use_mfma_kmeans(const Guide &g, int prec) { return prec != 0 && g.D > 32; }

// ---- kernels_embed.hip ------------------------------------------------------
// f0[c] = center (finite) or (min_c + max_c) / 2 over f.
// words of the mm scratch that launch_center needs
size_t center_scratch_words(int C);
hipError_t launch_center(const float *f, int64_t N, int C, double center, float *f0,
                         unsigned *scratch /*[2C]*/, hipStream_t s);
// eta_hat statistics into st[2] (device): the count of pixels that took the
// eta_hat <= 0 / non-finite guard, and the order-preserving code of the
// smallest positive eta_hat (decoded by eta_stats_min; NAN if none).
hipError_t launch_eta_stats(const float *eta, int64_t N, unsigned *st, hipStream_t s);
// A [r][r] FP64 = exp(-|c_i - c_j|^2 / (2 sigma_r^2)) from FP32 landmarks c [r][D].
hipError_t launch_landmark_gram(const float *c, int r, int D, double sigma_r, double *A, hipStream_t s);
double eta_stats_min(unsigned code);
// u[k][x] = sum_j F[j][k] exp(-|p(x) - c_j|^2 / (2 sigma_r^2)), planar [r_eff][N] float32.
// ct64 is scratch of embed_scratch_doubles(g, r) doubles (transposed FP64 landmarks).
size_t embed_scratch_doubles(const Guide &g, int r);
// u64 (nullable): write the planes as FP64 [r_eff][N] there instead of u.
hipError_t launch_embed(const Guide &g, const float *c, int r, const double *F, int r_eff,
                        double sigma_r, float *u, double *ct64, hipStream_t s, double *u64 = nullptr);

// ---- kernels_conv.hip -------------------------------------------------------
struct ConvProblem {
  int H, W, C, S, r_eff;
  const float *f;     // [H, W, C]
  const float *f0;    // [C] centring offsets
  const float *u;     // [r_eff][N]
  Taps taps;
  float *out;         // [H, W, C]
  float *eta_out;     // nullable [N]
  float *eta_buf;     // [N] scratch used when C > 3 (eta pass, then channel chunks)
  float *f_planar;    // [C][N] scratch used when C > 3 (f transposed to planes)
  int box;            // box spatial kernel (all taps 1): sliding sums for C <= 3
  int force_nch;      // > 0: row chunks per tile (tile-geometry control); 0: automatic
};
hipError_t launch_conv_contract(const ConvProblem &pb, hipStream_t s);

// ---- kernels_box.hip --------------------------------------------------------
// Box-window convolutions + contraction + normalisation for C <= 3 with FP64
// sums throughout; u is FP64 (u_fp64) or FP32 planes [r_eff][N].
struct BoxProblem {
  int H, W, C, S, r_eff;
  const float *f;     // [H, W, C]
  const void *u;      // [r_eff][N], double when u_fp64 else float
  int u_fp64;
  float *out;         // [H, W, C]
  float *eta_out;     // nullable [N]
  double *part;       // box_partials_doubles(...) doubles (unused when that is 0)
  int num_cu;         // compute units of the device (0: 256)
};
// k ranges per tile and the partial-sum scratch they need.
int box_splits(int H, int W, int S, int r_eff, int num_cu, int u_fp64);
size_t box_partials_doubles(int H, int W, int S, int r_eff, int num_cu, int u_fp64);
hipError_t launch_box(const BoxProblem &pb, hipStream_t s);

// ---- kernels_rec.hip --------------------------------------------------------
// Recursive-Gaussian (Young and van Vliet) convolutions + contraction +
// normalisation for C <= 3: parallel-form coefficients of the cascade.
struct RecCoef {
  double n0, n1, n2, n3;  // numerator of the causal half
  double a1, a2, a3;      // feedback of the cascade's recursion
};
constexpr double kRecSigmaMin = 0.5, kRecSigmaMax = 200.0;
// False when sigma_s is outside [kRecSigmaMin, kRecSigmaMax].
bool rec_coefficients(double sigma_s, RecCoef *c);
struct RecProblem {
  int H, W, C, r_eff;
  RecCoef coef;
  const float *f;     // [H, W, C]
  const float *f0;    // [C] centring offsets
  const float *u;     // [r_eff][N]
  float *out;         // [H, W, C]
  float *eta_out;     // nullable [N]
  float *planes;      // rec_plane_floats(...) floats: the filtered planes
  // backward only (launch_rec_bwd, after launch_rec on the same planes)
  const float *G;     // dL/dg [H, W, C]
  const float *eta;   // the forward's eta_hat [N]
  const float *ab;    // (beta, a_c) [N][4] of launch_bwd_ab
  float *dud, *du;    // [r_eff][N] outputs for the reduction
  float *df;          // [H, W, C]
};
size_t rec_plane_floats(int H, int W, int C, int r_eff);
hipError_t launch_rec(const RecProblem &pb, hipStream_t s);
hipError_t launch_rec_bwd(const RecProblem &pb, hipStream_t s);

// ---- kernels_wk.hip ---------------------------------------------------------
// Windowed Nystrom-kernel evaluation on MFMA for many channels (16-bit forms):
// K_hat = U_keys U_queries^T per window, then zeta = (w K_hat)^T (f - f0).
constexpr int kWkMaxRank = 64;
struct WkProblem {
  int H, W, C, S, r_eff, prec;  // prec 1 = BF16, 2 = FP16
  const float *f;     // [H, W, C]
  const float *f0;    // [C] centring offsets
  const float *u;     // [r_eff][N] FP32 planes
  Taps taps;
  float *out;         // [H, W, C]
  float *eta_out;     // nullable [N]
  void *scratch;      // wk_scratch_bytes(H, W, C, r_eff or more)
};
// The centred 16-bit image the windowed kernel reads (landmark-independent:
// enqueue it before the landmark factor); launch_wk expects it in scratch.
hipError_t launch_wk_prep_f(const WkProblem &pb, hipStream_t s);
// Whether the windowed form serves C channels, up to r landmarks, radius S.
bool wk_supported(int C, int r, int S, int prec);
size_t wk_scratch_bytes(int H, int W, int C, int r);
hipError_t launch_wk(const WkProblem &pb, hipStream_t s);

// ---- kernels_bwd.hip --------------------------------------------------------
// Backward passes (C <= 3).  mode 1: du_dir planes; 2: sigma_s partial sums
// (one double per block, with row taps wr and column taps wc); 3: adjoint
// convolutions -> du planes and df; 4: modes 1 and 2 in one pass.
struct BwdConvProblem {
  int mode, H, W, C, S, r_eff;
  const float *f, *f0, *u, *ab, *plane_in, *G, *eta;
  float *plane_out, *df;
  double *partials;
  Taps wr, wc;
  int *nblocks_out;
  int force_nch;      // as in ConvProblem
};
int bwd_conv_max_blocks(int H, int W);
hipError_t launch_bwd_ab(int64_t N, int C, const float *G, const float *out, const float *eta,
                         const float *f0, float *ab, hipStream_t s);
hipError_t launch_bwd_conv(const BwdConvProblem &pb, hipStream_t s);
int bwd_reduce_blocks(int64_t N);
size_t bwd_reduce_lds(int r, int r_eff, int D, int want_R);
// db = F du, dp (nullable), and per-block partials [blocks][1 + r*r_eff]:
// the sigma_r-through-b sum, then R = sum_x b du_dir^T (when want_R).
hipError_t launch_bwd_reduce(const Guide &g, const float *c, int r, const double *F, int r_eff,
                             double sigma_r, const float *du, const float *dud, float *dp, int want_R,
                             double *partials, hipStream_t s);
// Column sums of partials [nrows][width] on the device: groups of 32 rows in
// row order, then the groups in order.  Returns the device pointer of the
// width sums inside scratch (bwd_sum_scratch_doubles(nrows, width) doubles).
size_t bwd_sum_scratch_doubles(int nrows, int width);
const double *launch_bwd_sum_partials(const double *partials, int nrows, int width, double *scratch,
                                      hipStream_t s, hipError_t *err);


// ---- static_scratch.hip ------------------------------------------------------
// Fixed-size device array of the allocation-free forward entry point.
size_t static_scratch_bytes();
// Takes the device address of `device`'s copy (once per device; `device` must
// be current).  Returns the lookup's status on every later call.
hipError_t static_scratch_init(int device);
// The address found by static_scratch_init (hipErrorNotInitialized before it).
hipError_t static_scratch_ptr(int device, void **out);

// ---- kernels_pca.hip ---------------------------------------------------------
// PCA patch guide: sample moments (FP64), projection of every pixel's patch.
int pca_max_dim();
size_t pca_sample_floats(int D, int ns);
hipError_t launch_pca_moments(const Guide &g, const int64_t *idx, int ns, int mean_blocks, int cov_chunks,
                              float *S, double *partials, double *mu, double *cpart, double *cov, hipStream_t s);
hipError_t launch_pca_project(const Guide &g, const double *mu, const double *V, int dim, float *out,
                              hipStream_t s);

}  // namespace nkf
