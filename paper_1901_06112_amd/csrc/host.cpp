// Host runtime of the Nystrom kernel filtering library: the C ABI of
// include/nkf.h, argument validation, the device workspace, the k-means
// seeding draw, the FP64 landmark factor and the stream-ordered launch
// sequence of Algorithm 1.
#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <string>
#include <algorithm>
#include <vector>

#include "../../include/nkf.h"
#include "nkf_internal.h"

namespace nkf {
int sym_eig(int n, const double *A, double *w, double *V);
int sym_eig_top(int n, const double *A, int k, double *w, double *V);
}

using namespace nkf;

struct nkf_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  char *ws = nullptr;
  size_t ws_bytes = 0;
  size_t ws_limit = 0;
  char *pinned = nullptr;  // host staging for landmarks / factor
  size_t pinned_bytes = 0;
  std::string err;
  // stage timing
  bool timing = false;
  struct Interval {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Interval> pending;
  std::vector<hipEvent_t> event_pool;
  double host_ms[NKF_STAGE_COUNT] = {0};
  int host_count[NKF_STAGE_COUNT] = {0};
  hipEvent_t copy_done = nullptr;  // the landmark copy of nkf_filter
  hipEvent_t pinned_free = nullptr;  // after the last queued copy through `pinned`
  // the last PCA sample draw (it depends on N and the seed only)
  int conv_chunks = 0;  // nkf_set_conv_chunks
  // statistics of the last forward call (nkf_enable_stats, NKF_LOG)
  bool stats = false;
  bool log = false;          // NKF_LOG set: print them after each forward call
  unsigned *dstat = nullptr; // device [2]: guarded-pixel count, min eta_hat code
  nkf_stats last{};
  int num_cu = 0;       // compute units of the device
  int64_t pca_draw_N = -1;
  uint64_t pca_draw_seed = 0;
  std::vector<int64_t> pca_draw;
};

namespace {

// roctx ranges (rocprofv3 --marker-trace) around every stage, when the roctx
// library can be loaded; otherwise the ranges are no-ops.
struct Roctx {
  int (*push)(const char *) = nullptr;
  int (*pop)() = nullptr;
  Roctx() {
    void *h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
    if (!h) h = dlopen("librocprofiler-sdk-roctx.so", RTLD_NOW | RTLD_LOCAL);
    if (!h) return;
    push = reinterpret_cast<int (*)(const char *)>(dlsym(h, "roctxRangePushA"));
    pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
    if (!push || !pop) push = nullptr, pop = nullptr;
  }
};
const Roctx &roctx() {
  static const Roctx r;
  return r;
}
struct Range {
  bool on;
  explicit Range(const char *name) : on(roctx().push != nullptr) {
    if (on) roctx().push(name);
  }
  ~Range() {
    if (on) roctx().pop();
  }
};
const char *const kStageRange[NKF_STAGE_COUNT] = {"nkf:seed", "nkf:kmeans", "nkf:factor",
                                                  "nkf:embed", "nkf:conv", "nkf:backward"};

hipEvent_t take_event(nkf_ctx *ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets the device work enqueued during its lifetime with two events.
struct StageTimer {
  nkf_ctx *ctx;
  int stage;
  Range range;
  hipEvent_t a = nullptr;
  StageTimer(nkf_ctx *c, int s) : ctx(c), stage(s), range(kStageRange[s]) {
    if (ctx->timing && (a = take_event(ctx))) (void)hipEventRecord(a, ctx->stream);
  }
  ~StageTimer() {
    if (!a) return;
    hipEvent_t b = take_event(ctx);
    if (!b) return;
    (void)hipEventRecord(b, ctx->stream);
    ctx->pending.push_back({stage, a, b});
  }
};

struct HostTimer {
  nkf_ctx *ctx;
  int stage;
  Range range;
  std::chrono::steady_clock::time_point t0;
  HostTimer(nkf_ctx *c, int s) : ctx(c), stage(s), range(kStageRange[s]), t0(std::chrono::steady_clock::now()) {}
  ~HostTimer() {
    if (!ctx || !ctx->timing) return;
    ctx->host_ms[stage] += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    ctx->host_count[stage] += 1;
  }
};

}  // namespace

namespace {

thread_local std::string g_err;

nkf_status fail(nkf_ctx *ctx, nkf_status st, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
nkf_status fail(nkf_ctx *ctx, nkf_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx)
    ctx->err = buf;
  else
    g_err = buf;
  return st;
}

#define HIP_TRY(ctx, expr)                                                              \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(ctx, NKF_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

// Sub-allocation of the workspace: the same sequence of take() calls is run
// once to size the arena and once to hand out pointers.
struct Carve {
  char *base;
  size_t off = 0;
  template <class T>
  T *take(size_t n) {
    off = (off + 255) & ~(size_t)255;
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

nkf_status ensure_workspace(nkf_ctx *ctx, size_t bytes) {
  if (bytes <= ctx->ws_bytes) return NKF_OK;
  if (ctx->ws_limit && bytes > ctx->ws_limit)
    return fail(ctx, NKF_ERR_OUT_OF_MEMORY, "workspace of %zu bytes exceeds the limit of %zu", bytes,
                ctx->ws_limit);
  if (ctx->ws) {
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    HIP_TRY(ctx, hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  size_t want = bytes + bytes / 8;
  if (ctx->ws_limit && want > ctx->ws_limit) want = ctx->ws_limit;
  void *p = nullptr;
  if (hipMalloc(&p, want) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, NKF_ERR_OUT_OF_MEMORY, "hipMalloc of %zu workspace bytes failed", want);
  }
  ctx->ws = static_cast<char *>(p);
  ctx->ws_bytes = want;
  return NKF_OK;
}

nkf_status ensure_pinned(nkf_ctx *ctx, size_t bytes) {
  if (bytes <= ctx->pinned_bytes) return NKF_OK;
  if (ctx->pinned) {
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    HIP_TRY(ctx, hipHostFree(ctx->pinned));
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
  }
  void *p = nullptr;
  if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, NKF_ERR_OUT_OF_MEMORY, "hipHostMalloc of %zu bytes failed", bytes);
  }
  ctx->pinned = static_cast<char *>(p);
  ctx->pinned_bytes = bytes;
  return NKF_OK;
}

// The pinned staging buffer is shared by the entry points of a context: each
// records pinned_free after its last queued copy through it, and a call about
// to write it from the host waits for that event, not for the whole stream,
// so a call's host work can start while the previous call's kernels run.
nkf_status pinned_acquire(nkf_ctx *ctx) {
  if (ctx->pinned_free) HIP_TRY(ctx, hipEventSynchronize(ctx->pinned_free));
  return NKF_OK;
}

nkf_status pinned_release(nkf_ctx *ctx) {
  if (!ctx->pinned_free) HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->pinned_free, hipEventDisableTiming));
  HIP_TRY(ctx, hipEventRecord(ctx->pinned_free, ctx->stream));
  return NKF_OK;
}

uint64_t splitmix_next(uint64_t &s) {
  s += 0x9E3779B97F4A7C15ull;
  uint64_t z = s;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// The swaps of a partial Fisher-Yates shuffle of the virtual identity array
// [0, N), kept in an open-addressing table (linear probing, at most 2r keys in
// a power-of-two table of >= 4r slots): entry k of the array is map[k] when
// present, else k.
class SwapMap {
 public:
  explicit SwapMap(int r) {
    size_t cap = 16;
    int bits = 4;
    while (cap < 4 * (size_t)r) cap <<= 1, ++bits;
    keys_.assign(cap, -1);
    vals_.resize(cap);
    mask_ = cap - 1;
    shift_ = 64 - bits;
  }
  int64_t get(int64_t k) const {
    for (size_t h = slot(k);; h = (h + 1) & mask_) {
      if (keys_[h] == k) return vals_[h];
      if (keys_[h] < 0) return k;
    }
  }
  void set(int64_t k, int64_t v) {
    size_t h = slot(k);
    while (keys_[h] >= 0 && keys_[h] != k) h = (h + 1) & mask_;
    keys_[h] = k;
    vals_[h] = v;
  }

 private:
  size_t slot(int64_t k) const { return (size_t)(((uint64_t)k * 0x9E3779B97F4A7C15ull) >> shift_); }
  std::vector<int64_t> keys_, vals_;
  size_t mask_;
  int shift_;
};

void draw_indices(int64_t N, int r, uint64_t seed, int64_t *idx) {
  uint64_t s = seed;
  SwapMap sw(r);
  for (int i = 0; i < r; ++i) {
    const int64_t j = i + (int64_t)(splitmix_next(s) % (uint64_t)(N - i));
    const int64_t vi = sw.get(i), vj = sw.get(j);
    sw.set(i, vj);
    sw.set(j, vi);
    idx[i] = vj;
  }
}

int resolve_radius(int radius, double sigma_s) {
  if (radius >= 0) return radius;
  return (int)ceil(3.0 * sigma_s);
}

struct Resolved {
  int H, W, C, D, S;
  int64_t N;
  Guide g;
  Taps taps;
  int box;  // spatial kernel is the box
  int rec;  // spatial kernel is the recursive Gaussian
  RecCoef rc;
};

// Validation shared by every device entry point.
nkf_status validate(nkf_ctx *ctx, int H, int W, int C, const float *f, int D, const float *p,
                    const nkf_params *prm, Resolved &rs) {
  if (!ctx) return fail(nullptr, NKF_ERR_INVALID_ARG, "ctx is NULL");
  if (!prm) return fail(ctx, NKF_ERR_INVALID_ARG, "params is NULL");
  if (H < 1 || W < 1 || C < 1 || D < 1)
    return fail(ctx, NKF_ERR_INVALID_ARG, "sizes must be >= 1 (H=%d W=%d C=%d D=%d)", H, W, C, D);
  if ((int64_t)H * W > (int64_t)1 << 31)
    return fail(ctx, NKF_ERR_INVALID_ARG, "H*W exceeds 2^31");
  // the convolution kernels address a chunk of rows with 32-bit byte offsets
  if (W > (1 << 21)) return fail(ctx, NKF_ERR_UNSUPPORTED, "W=%d exceeds 2^21", W);
  if (!f) return fail(ctx, NKF_ERR_INVALID_ARG, "f is NULL");
  if (D > kMaxGuideDim) return fail(ctx, NKF_ERR_UNSUPPORTED, "guide dimension D=%d exceeds %d", D, kMaxGuideDim);
  if (C > 1024) return fail(ctx, NKF_ERR_UNSUPPORTED, "C=%d exceeds 1024", C);
  if (!(prm->sigma_r > 0.0) || isnan(prm->sigma_r))
    return fail(ctx, NKF_ERR_INVALID_ARG, "sigma_r must be > 0 (got %g)", prm->sigma_r);
  if (prm->spatial != NKF_SPATIAL_GAUSSIAN && prm->spatial != NKF_SPATIAL_BOX &&
      prm->spatial != NKF_SPATIAL_RECURSIVE)
    return fail(ctx, NKF_ERR_INVALID_ARG, "unknown spatial kernel %d", prm->spatial);
  const bool rec = prm->spatial == NKF_SPATIAL_RECURSIVE;
  RecCoef rc{};
  if (rec) {
    if (!rec_coefficients(prm->sigma_s, &rc))
      return fail(ctx, NKF_ERR_INVALID_ARG, "the recursive Gaussian needs %g <= sigma_s <= %g (got %g)",
                  kRecSigmaMin, kRecSigmaMax, prm->sigma_s);
    if (C > 3) return fail(ctx, NKF_ERR_UNSUPPORTED, "the recursive Gaussian supports C <= 3 (got %d)", C);
  } else if (prm->spatial == NKF_SPATIAL_GAUSSIAN || prm->radius < 0) {
    if (!(prm->sigma_s > 0.0) || !isfinite(prm->sigma_s))
      return fail(ctx, NKF_ERR_INVALID_ARG, "sigma_s must be finite and > 0 (got %g)", prm->sigma_s);
  }
  if (prm->radius < -1) return fail(ctx, NKF_ERR_INVALID_ARG, "radius must be >= -1");
  // the recursive filter has no window: radius is unused
  const int S = rec ? 0 : resolve_radius(prm->radius, prm->sigma_s);
  if (S > kMaxRadius)
    return fail(ctx, NKF_ERR_UNSUPPORTED, "window radius %d exceeds %d", S, kMaxRadius);
  const int64_t N = (int64_t)H * W;
  if (prm->r < 1 || prm->r > kMaxLandmarks || prm->r > N)
    return fail(ctx, NKF_ERR_INVALID_ARG, "r=%d must satisfy 1 <= r <= min(N, %d)", prm->r,
                kMaxLandmarks);
  if (prm->kmeans_iters < 0) return fail(ctx, NKF_ERR_INVALID_ARG, "kmeans_iters must be >= 0");
  if (!(prm->eig_rel_tol >= 0.0)) return fail(ctx, NKF_ERR_INVALID_ARG, "eig_rel_tol must be >= 0");
  if (prm->prec != NKF_PREC_FP32 && prm->prec != NKF_PREC_BF16 && prm->prec != NKF_PREC_FP16)
    return fail(ctx, NKF_ERR_INVALID_ARG, "unknown precision %d", prm->prec);
  Guide g{};
  g.H = H;
  g.W = W;
  g.C = C;
  g.D = D;
  g.f = f;
  switch (prm->guide) {
    case NKF_GUIDE_EXPLICIT:
      if (!p) return fail(ctx, NKF_ERR_INVALID_ARG, "explicit guide needs p");
      g.kind = GUIDE_EXPLICIT;
      g.p = p;
      break;
    case NKF_GUIDE_SELF:
      if (D != C) return fail(ctx, NKF_ERR_INVALID_ARG, "self guide needs D == C (D=%d C=%d)", D, C);
      g.kind = GUIDE_SELF;
      break;
    case NKF_GUIDE_PATCH: {
      const int pr = prm->patch_radius;
      if (pr < 0) return fail(ctx, NKF_ERR_INVALID_ARG, "patch_radius must be >= 0");
      if (pr > H || pr > W) return fail(ctx, NKF_ERR_INVALID_ARG, "patch_radius exceeds the image");
      if (D != C * (2 * pr + 1) * (2 * pr + 1))
        return fail(ctx, NKF_ERR_INVALID_ARG, "patch guide needs D == C (2pr+1)^2 (D=%d)", D);
      g.kind = GUIDE_PATCH;
      g.pr = pr;
      break;
    }
    default:
      return fail(ctx, NKF_ERR_INVALID_ARG, "unknown guide kind %d", prm->guide);
  }
  if (use_mfma_distance(g, prm->prec) && !mfma_path_supported(g, prm->r, prm->prec))
    return fail(ctx, NKF_ERR_UNSUPPORTED,
                "16-bit distance form: r=%d landmarks of dimension D=%d exceed the LDS plan", prm->r, D);
  rs.H = H;
  rs.W = W;
  rs.C = C;
  rs.D = D;
  rs.S = S;
  rs.N = N;
  rs.g = g;
  rs.box = prm->spatial == NKF_SPATIAL_BOX;
  rs.rec = rec;
  rs.rc = rc;
  for (int t = 0; t < 2 * kMaxRadius + 1; ++t) rs.taps.w[t] = 0.0f;
  for (int t = -S; t <= S; ++t)
    rs.taps.w[t + S] = prm->spatial == NKF_SPATIAL_BOX
                           ? 1.0f
                           : (float)exp(-(double)t * t / (2.0 * prm->sigma_s * prm->sigma_s));
  return NKF_OK;
}

// ---- host FP64 landmark factor ----------------------------------------------
nkf_status factor_from_gram(nkf_ctx *ctx, int r, std::vector<double> &A, double tau, double *Q, double *alpha,
                            double *F, int *r_eff);

nkf_status factor(nkf_ctx *ctx, int r, int D, const double *c, double sigma_r, double tau, double *Q,
                  double *alpha, double *F, int *r_eff) {
  std::vector<double> A((size_t)r * r);
  const double inv = isinf(sigma_r) ? 0.0 : 1.0 / (2.0 * sigma_r * sigma_r);
  for (int i = 0; i < r; ++i) {
    A[i * r + i] = 1.0;
    for (int j = 0; j < i; ++j) {
      // four partial sums in a fixed order: independent chains, same result every call
      double d4[4] = {0.0, 0.0, 0.0, 0.0};
      int k = 0;
      for (; k + 4 <= D; k += 4)
        for (int q = 0; q < 4; ++q) {
          const double t = c[i * D + k + q] - c[j * D + k + q];
          d4[q] += t * t;
        }
      for (; k < D; ++k) {
        const double t = c[i * D + k] - c[j * D + k];
        d4[0] += t * t;
      }
      const double d2 = (d4[0] + d4[1]) + (d4[2] + d4[3]);
      A[i * r + j] = A[j * r + i] = exp(-d2 * inv);
    }
  }
  return factor_from_gram(ctx, r, A, tau, Q, alpha, F, r_eff);
}

// The eigendecomposition of A (Eq. (eigA)) and F = Q_keep diag(alpha_keep^{-1/2}).
nkf_status factor_from_gram(nkf_ctx *ctx, int r, std::vector<double> &A, double tau, double *Q, double *alpha,
                            double *F, int *r_eff) {
  std::vector<double> Qv((size_t)r * r), al(r);
  if (sym_eig(r, A.data(), al.data(), Qv.data()) != 0)
    return fail(ctx, NKF_ERR_NUMERICAL, "eigendecomposition of A did not converge");
  const double amax = al[r - 1];
  int keep = 0;
  for (int j = 0; j < r; ++j)
    if (al[j] > tau * amax && al[j] > 0.0) ++keep;
  if (Q) memcpy(Q, Qv.data(), sizeof(double) * r * r);
  if (alpha) memcpy(alpha, al.data(), sizeof(double) * r);
  if (keep == 0) {
    if (r_eff) *r_eff = 0;
    return fail(ctx, NKF_ERR_NUMERICAL, "every eigenvalue of A was truncated");
  }
  // kept eigenvalues are the largest ones; columns in ascending order
  const int first = r - keep;
  if (F) {
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < r; ++j) F[i * r + j] = 0.0;
    for (int j = 0; j < keep; ++j) {
      const double s = 1.0 / sqrt(al[first + j]);
      for (int i = 0; i < r; ++i) F[i * r + j] = Qv[i * r + first + j] * s;
    }
  }
  if (r_eff) *r_eff = keep;
  return NKF_OK;
}

// The box window on up to three channels runs the FP64 box kernel; its plain
// form (FP32 distances) keeps the embedding planes in FP64 as well.  The
// backward's conv modes read FP32 planes, so it never asks for them.
bool box_path(const Resolved &rs) { return rs.box && rs.C <= 3; }
bool fwd_u64(const Resolved &rs, int prec) { return box_path(rs) && !use_mfma_distance(rs.g, prec); }

// Partial-sum scratch of the box kernel for any r_eff <= r (its split count
// depends on r_eff only through min(r_eff, 8)).
size_t box_part_doubles(const Resolved &rs, int r, int num_cu, bool u64) {
  if (!box_path(rs)) return 0;
  size_t m = 0;
  for (int re = 1; re <= (r < 8 ? r : 8); ++re) {
    const size_t v = box_partials_doubles(rs.H, rs.W, rs.S, re, num_cu, u64 ? 1 : 0);
    if (v > m) m = v;
  }
  return m;
}

// Workspace of the forward path after the landmarks are known.
struct FwdBufs {
  float *f0;
  unsigned *mm;
  float *u;      // FP32 planes, or
  double *u64;   // FP64 planes (box kernel, plain form)
  double *box_part;
  float *eta_buf;
  float *f_planar;  // [C][N] when C > 3
  float *mu;     // [D] centring of the 16-bit distance path
  float *F32;    // [r][r_eff] FP32 factor for the MFMA mix
  double *mpart; // partial sums of the centring offsets
  void *lm;      // prepared 16-bit landmarks
  double *ct64;  // transposed FP64 landmarks of the FP32 embedding
  float *eta_stat;  // eta_hat for the statistics when the caller passes no eta_out
  void *wk;         // operands of the windowed MFMA form (16-bit forms, C > 3), else null
  float *bsplit;    // cross-kernel tiles of the split 16-bit embedding (nkf_filter), else null
  float *rec;       // filtered planes of the recursive Gaussian, else null
};

// The 16-bit forms on more than three channels evaluate the windows on MFMA
// (kernels_wk.hip) instead of convolving r_eff (C + 1) planes; wk_r bounds
// r_eff (the landmark count), 0 when the windowed form is not used.
int fwd_wk_r(const Resolved &rs, const nkf_params *prm, int r) {
  return wk_supported(rs.C, r, rs.S, prm->prec) ? r : 0;
}

void carve_fwd(Carve &cv, const Resolved &rs, int r_eff, FwdBufs &b, int r, bool u64, int num_cu,
               bool stats = false, int wk_r = 0, int split_prec = 0) {
  b.f0 = cv.take<float>(rs.C);
  b.mm = cv.take<unsigned>(center_scratch_words(rs.C));
  b.u = u64 ? nullptr : cv.take<float>((size_t)r_eff * rs.N);
  b.u64 = u64 ? cv.take<double>((size_t)r_eff * rs.N) : nullptr;
  b.box_part = cv.take<double>(box_part_doubles(rs, r_eff, num_cu, u64));
  b.eta_buf = cv.take<float>(rs.C > 3 && !wk_r ? rs.N : 1);
  b.f_planar = cv.take<float>(rs.C > 3 && !wk_r ? (size_t)rs.C * rs.N : 1);
  b.mu = cv.take<float>(rs.D);
  b.F32 = cv.take<float>((size_t)r * r_eff);
  b.mpart = cv.take<double>(guide_mean_scratch_doubles(rs.g));
  b.lm = cv.take<unsigned char>(mfma_landmark_scratch_bytes(rs.g, r));
  b.ct64 = cv.take<double>(embed_scratch_doubles(rs.g, r));
  b.eta_stat = cv.take<float>(stats ? rs.N : 1);
  b.wk = wk_r ? static_cast<void *>(cv.take<unsigned char>(wk_scratch_bytes(rs.H, rs.W, rs.C, wk_r))) : nullptr;
  b.bsplit = split_prec ? cv.take<float>(embed_split_floats(rs.g, r_eff, split_prec)) : nullptr;
  b.rec = rs.rec ? cv.take<float>(rec_plane_floats(rs.H, rs.W, rs.C, r_eff)) : nullptr;
}

// The landmark-independent part of the forward: the centring offsets f0,
// for the 16-bit distance path the guide mean, and for the windowed form its
// centred 16-bit image.
// mu_ready: the guide mean the k-means of this call already formed (copied
// instead of recomputed), or null.
nkf_status run_pre(nkf_ctx *ctx, const Resolved &rs, const nkf_params *prm, const FwdBufs &b,
                   const float *mu_ready = nullptr) {
  HIP_TRY(ctx, launch_center(rs.g.f, rs.N, rs.C, prm->center, b.f0, b.mm, ctx->stream));
  if (use_mfma_distance(rs.g, prm->prec)) {
    if (mu_ready)
      HIP_TRY(ctx, hipMemcpyAsync(b.mu, mu_ready, sizeof(float) * rs.D, hipMemcpyDeviceToDevice, ctx->stream));
    else
      HIP_TRY(ctx, launch_guide_mean(rs.g, b.mu, b.mpart, ctx->stream));
  }
  if (b.wk) {
    WkProblem wp{};
    wp.H = rs.H;
    wp.W = rs.W;
    wp.C = rs.C;
    wp.prec = prm->prec;
    wp.f = rs.g.f;
    wp.f0 = b.f0;
    wp.scratch = b.wk;
    HIP_TRY(ctx, launch_wk_prep_f(wp, ctx->stream));
  }
  return NKF_OK;
}

// pre_done: run_pre has been enqueued already
// stats_ok: a forward entry point whose statistics are recorded (not the
// backward's recompute, nor the allocation-free call)
// embed_b_done: the cross-kernel tiles of the split 16-bit embedding are in
// b.bsplit already (enqueued before the landmark factor), only the mix is left
nkf_status run_fwd(nkf_ctx *ctx, const Resolved &rs, const nkf_params *prm, const float *c, const double *F,
                   int r_eff, float *out, float *eta_out, const FwdBufs &b, bool conv = true, bool pre_done = false,
                   bool stats_ok = false, bool embed_b_done = false) {
  {
    StageTimer tm(ctx, NKF_STAGE_EMBED);
    if (!pre_done) {
      nkf_status st = run_pre(ctx, rs, prm, b);
      if (st != NKF_OK) return st;
    }
    if (use_mfma_distance(rs.g, prm->prec) && embed_b_done && b.bsplit) {
      HIP_TRY(ctx, launch_embed_mfma_mix(rs.g, prm->r, F, b.F32, r_eff, prm->prec, b.u, b.bsplit, ctx->stream));
    } else if (use_mfma_distance(rs.g, prm->prec)) {
      HIP_TRY(ctx, launch_embed_mfma(rs.g, c, prm->r, b.mu, F, b.F32, r_eff, prm->sigma_r, prm->prec, b.u,
                                     b.lm, ctx->stream));
    } else {
      HIP_TRY(ctx, launch_embed(rs.g, c, prm->r, F, r_eff, prm->sigma_r, b.u, b.ct64, ctx->stream, b.u64));
    }
  }
  if (!conv) return NKF_OK;
  // eta_hat for the statistics: the caller's, else the library's copy
  const bool want_stats = ctx->stats && ctx->dstat && stats_ok;
  if (want_stats && !eta_out) eta_out = b.eta_stat;
  if (rs.rec) {
    RecProblem rp{};
    rp.H = rs.H;
    rp.W = rs.W;
    rp.C = rs.C;
    rp.r_eff = r_eff;
    rp.coef = rs.rc;
    rp.f = rs.g.f;
    rp.f0 = b.f0;
    rp.u = b.u;
    rp.out = out;
    rp.eta_out = eta_out;
    rp.planes = b.rec;
    {
      StageTimer tm(ctx, NKF_STAGE_CONV);
      HIP_TRY(ctx, launch_rec(rp, ctx->stream));
    }
    if (want_stats) HIP_TRY(ctx, launch_eta_stats(eta_out, rs.N, ctx->dstat, ctx->stream));
    return NKF_OK;
  }
  if (box_path(rs)) {
    BoxProblem bx{};
    bx.H = rs.H;
    bx.W = rs.W;
    bx.C = rs.C;
    bx.S = rs.S;
    bx.r_eff = r_eff;
    bx.f = rs.g.f;
    bx.u = b.u64 ? static_cast<const void *>(b.u64) : static_cast<const void *>(b.u);
    bx.u_fp64 = b.u64 != nullptr;
    bx.out = out;
    bx.eta_out = eta_out;
    bx.part = b.box_part;
    bx.num_cu = ctx->num_cu;
    {
      StageTimer tm(ctx, NKF_STAGE_CONV);
      HIP_TRY(ctx, launch_box(bx, ctx->stream));
    }
    if (want_stats) HIP_TRY(ctx, launch_eta_stats(eta_out, rs.N, ctx->dstat, ctx->stream));
    return NKF_OK;
  }
  if (b.wk) {
    WkProblem wp{};
    wp.H = rs.H;
    wp.W = rs.W;
    wp.C = rs.C;
    wp.S = rs.S;
    wp.r_eff = r_eff;
    wp.prec = prm->prec;
    wp.f = rs.g.f;
    wp.f0 = b.f0;
    wp.u = b.u;
    wp.taps = rs.taps;
    wp.out = out;
    wp.eta_out = eta_out;
    wp.scratch = b.wk;
    {
      StageTimer tm(ctx, NKF_STAGE_CONV);
      HIP_TRY(ctx, launch_wk(wp, ctx->stream));
    }
    if (want_stats) HIP_TRY(ctx, launch_eta_stats(eta_out, rs.N, ctx->dstat, ctx->stream));
    return NKF_OK;
  }
  ConvProblem pb{};
  pb.H = rs.H;
  pb.W = rs.W;
  pb.C = rs.C;
  pb.S = rs.S;
  pb.r_eff = r_eff;
  pb.f = rs.g.f;
  pb.f0 = b.f0;
  pb.u = b.u;
  pb.taps = rs.taps;
  pb.box = rs.box;
  pb.out = out;
  pb.eta_out = eta_out;
  pb.eta_buf = b.eta_buf;
  pb.f_planar = b.f_planar;
  pb.force_nch = ctx->conv_chunks;
  {
    StageTimer tm(ctx, NKF_STAGE_CONV);
    HIP_TRY(ctx, launch_conv_contract(pb, ctx->stream));
  }
  if (want_stats) HIP_TRY(ctx, launch_eta_stats(eta_out, rs.N, ctx->dstat, ctx->stream));
  return NKF_OK;
}

struct KmBufs {
  double *sums;
  int *lab_scratch;
  float *mu;
  void *lm;  // prepared 16-bit landmarks
  float *ct; // transposed landmarks of the FP32 assignment
};

void carve_km(Carve &cv, const Resolved &rs, int r, KmBufs &b) {
  // the partial sums double as the scratch of the guide mean
  b.sums = cv.take<double>(std::max(kmeans_partials_doubles(r, rs.D), guide_mean_scratch_doubles(rs.g)));
  b.lab_scratch = cv.take<int>(rs.N);
  b.mu = cv.take<float>(rs.D);
  b.lm = cv.take<unsigned char>(mfma_landmark_scratch_bytes(rs.g, r));
  b.ct = cv.take<float>(kmeans_transposed_floats(rs.g, r));
}

nkf_status run_lloyd(nkf_ctx *ctx, const Resolved &rs, int r, float *c, int iters, int *labels,
                     const KmBufs &b, int prec) {
  StageTimer tm(ctx, NKF_STAGE_KMEANS);
  if (use_mfma_kmeans(rs.g, prec)) {
    // the partial-sum buffer doubles as the scratch of the centring offsets
    if (iters > 0) HIP_TRY(ctx, launch_guide_mean(rs.g, b.mu, b.sums, ctx->stream));
    for (int it = 0; it < iters; ++it)
      HIP_TRY(ctx, launch_kmeans_step_mfma(rs.g, c, r, b.mu, prec, b.sums, it + 1 == iters ? labels : nullptr,
                                           b.lm, ctx->stream));
    return NKF_OK;
  }
  for (int it = 0; it < iters; ++it)
    HIP_TRY(ctx, launch_kmeans_step(rs.g, c, r, b.sums, it + 1 == iters ? labels : nullptr, b.lab_scratch,
                                    b.ct, ctx->stream));
  return NKF_OK;
}

nkf_status run_seed(nkf_ctx *ctx, const Resolved &rs, const nkf_params *prm, float *c, int64_t *idx_dev) {
  const int r = prm->r;
  nkf_status st = ensure_pinned(ctx, 64 * 1024 + sizeof(int64_t) * r);
  if (st != NKF_OK) return st;
  if ((st = pinned_acquire(ctx)) != NKF_OK) return st;
  int64_t *idx = reinterpret_cast<int64_t *>(ctx->pinned);
  draw_indices(rs.N, r, prm->seed, idx);
  StageTimer tm(ctx, NKF_STAGE_SEED);
  HIP_TRY(ctx, hipMemcpyAsync(idx_dev, idx, sizeof(int64_t) * r, hipMemcpyHostToDevice, ctx->stream));
  if ((st = pinned_release(ctx)) != NKF_OK) return st;
  HIP_TRY(ctx, launch_gather_landmarks(rs.g, idx_dev, r, c, ctx->stream));
  return NKF_OK;
}

// Host part of the statistics of one forward call (the eta_hat part is
// reduced on the device and read by nkf_get_stats).
void record_stats(nkf_ctx *ctx, const Resolved &rs, const nkf_params *prm, int r_eff, double alpha_max,
                  double alpha_min_kept) {
  if (!ctx->stats) return;
  nkf_stats &t = ctx->last;
  t = nkf_stats{};
  t.valid = 1;
  t.pixels = rs.N;
  t.r = prm->r;
  t.r_eff = r_eff;
  t.alpha_max = alpha_max;
  t.alpha_min_kept = alpha_min_kept;
  t.cond_kept = alpha_max / alpha_min_kept;
  t.guarded = -1;
  t.min_eta = NAN;
}

nkf_status log_stats(nkf_ctx *ctx, const char *call, const Resolved &rs, const nkf_params *prm) {
  if (!ctx->log) return NKF_OK;
  nkf_stats t;
  const nkf_status st = nkf_get_stats(ctx, &t);
  if (st != NKF_OK) return st;
  fprintf(stderr,
          "nkf: %s %dx%dx%d D=%d S=%d %s %s r=%d r_eff=%d cond(A_kept)=%.3g alpha_max=%.6g "
          "guarded=%lld min_eta=%.6g\n",
          call, rs.H, rs.W, rs.C, rs.D, rs.S, rs.box ? "box" : "gaussian",
          prm->prec == NKF_PREC_FP32 ? "fp32" : prm->prec == NKF_PREC_BF16 ? "bf16" : "fp16", t.r, t.r_eff,
          t.cond_kept, t.alpha_max, t.guarded, t.min_eta);
  return NKF_OK;
}

}  // namespace

// =============================================================================
extern "C" {

void nkf_params_default(nkf_params *p) {
  if (!p) return;
  p->sigma_s = 3.0;
  p->sigma_r = 30.0;
  p->r = 16;
  p->radius = -1;
  p->spatial = NKF_SPATIAL_GAUSSIAN;
  p->guide = NKF_GUIDE_SELF;
  p->patch_radius = 3;
  p->prec = NKF_PREC_FP32;
  p->kmeans_iters = 10;
  p->seed = 0;
  p->eig_rel_tol = 1e-10;
  p->center = NAN;
}

const char *nkf_version(void) { return "nkf 0.1 (gfx950)"; }

nkf_status nkf_create(nkf_ctx **out, void *hip_stream) {
  if (!out) return fail(nullptr, NKF_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  nkf_ctx *c = new (std::nothrow) nkf_ctx();
  if (!c) return fail(nullptr, NKF_ERR_OUT_OF_MEMORY, "context allocation failed");
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&c->device) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return fail(nullptr, NKF_ERR_HIP, "hipGetDevice failed (no GPU?)");
  }
  // device address of this device's static scratch (allocation-free entry
  // point); a failed lookup only disables that entry point
  (void)static_scratch_init(c->device);
  if (hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) {
    (void)hipGetLastError();
    c->num_cu = 0;
  }
  // NKF_LOG (non-empty, not "0"): statistics of every forward call on stderr
  const char *lg = getenv("NKF_LOG");
  if (lg && *lg && strcmp(lg, "0") != 0) {
    c->log = true;
    if (nkf_enable_stats(c, 1) != NKF_OK) c->log = false;
  }
  *out = c;
  return NKF_OK;
}

nkf_status nkf_set_stream(nkf_ctx *ctx, void *hip_stream) {
  if (!ctx) return fail(nullptr, NKF_ERR_INVALID_ARG, "ctx is NULL");
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return NKF_OK;
}

nkf_status nkf_enable_timing(nkf_ctx *ctx, int enable) {
  if (!ctx) return fail(nullptr, NKF_ERR_INVALID_ARG, "ctx is NULL");
  ctx->timing = enable != 0;
  return NKF_OK;
}

nkf_status nkf_stage_times(nkf_ctx *ctx, double *ms_host, int *count_host, int reset) {
  if (!ctx) return fail(nullptr, NKF_ERR_INVALID_ARG, "ctx is NULL");
  if (!ms_host) return fail(ctx, NKF_ERR_INVALID_ARG, "ms_host is NULL");
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  double ms[NKF_STAGE_COUNT];
  int cnt[NKF_STAGE_COUNT];
  for (int i = 0; i < NKF_STAGE_COUNT; ++i) {
    ms[i] = ctx->host_ms[i];
    cnt[i] = ctx->host_count[i];
  }
  for (auto &iv : ctx->pending) {
    float e = 0.0f;
    HIP_TRY(ctx, hipEventElapsedTime(&e, iv.a, iv.b));
    ms[iv.stage] += e;
    cnt[iv.stage] += 1;
  }
  for (int i = 0; i < NKF_STAGE_COUNT; ++i) {
    ms_host[i] = ms[i];
    if (count_host) count_host[i] = cnt[i];
  }
  if (reset) {
    for (auto &iv : ctx->pending) {
      ctx->event_pool.push_back(iv.a);
      ctx->event_pool.push_back(iv.b);
    }
    ctx->pending.clear();
    for (int i = 0; i < NKF_STAGE_COUNT; ++i) {
      ctx->host_ms[i] = 0.0;
      ctx->host_count[i] = 0;
    }
  }
  return NKF_OK;
}

nkf_status nkf_destroy(nkf_ctx *ctx) {
  if (!ctx) return NKF_OK;
  nkf_status st = NKF_OK;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) st = NKF_ERR_HIP;
  for (auto &iv : ctx->pending) {
    (void)hipEventDestroy(iv.a);
    (void)hipEventDestroy(iv.b);
  }
  for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
  if (ctx->copy_done) (void)hipEventDestroy(ctx->copy_done);
  if (ctx->pinned_free) (void)hipEventDestroy(ctx->pinned_free);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->dstat) (void)hipFree(ctx->dstat);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  delete ctx;
  return st;
}

const char *nkf_last_error(const nkf_ctx *ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

nkf_status nkf_enable_stats(nkf_ctx *ctx, int enable) {
  if (!ctx) return fail(nullptr, NKF_ERR_INVALID_ARG, "ctx is NULL");
  if (enable && !ctx->dstat) {
    void *p = nullptr;
    if (hipMalloc(&p, 2 * sizeof(unsigned)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, NKF_ERR_OUT_OF_MEMORY, "hipMalloc of the statistics buffer failed");
    }
    ctx->dstat = static_cast<unsigned *>(p);
  }
  ctx->stats = enable != 0;
  ctx->last = nkf_stats{};
  return NKF_OK;
}

nkf_status nkf_get_stats(nkf_ctx *ctx, nkf_stats *out) {
  if (!ctx || !out) return fail(ctx, NKF_ERR_INVALID_ARG, "ctx and out are required");
  *out = ctx->last;
  if (!ctx->last.valid || !ctx->dstat) return NKF_OK;
  unsigned h[2] = {0u, 0u};
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  HIP_TRY(ctx, hipMemcpy(h, ctx->dstat, sizeof h, hipMemcpyDeviceToHost));
  out->guarded = (long long)h[0];
  out->min_eta = eta_stats_min(h[1]);
  return NKF_OK;
}

nkf_status nkf_set_conv_chunks(nkf_ctx *ctx, int nch) {
  if (!ctx) return fail(nullptr, NKF_ERR_INVALID_ARG, "ctx is NULL");
  if (nch < 0) return fail(ctx, NKF_ERR_INVALID_ARG, "nch must be >= 0 (got %d)", nch);
  ctx->conv_chunks = nch;
  return NKF_OK;
}

nkf_status nkf_set_workspace_limit(nkf_ctx *ctx, size_t bytes) {
  if (!ctx) return fail(nullptr, NKF_ERR_INVALID_ARG, "ctx is NULL");
  ctx->ws_limit = bytes;
  return NKF_OK;
}

size_t nkf_workspace_bytes(const nkf_ctx *ctx) { return ctx ? ctx->ws_bytes : 0; }

nkf_status nkf_seed_indices(int64_t N, int r, uint64_t seed, int64_t *idx_host) {
  if (!idx_host) return fail(nullptr, NKF_ERR_INVALID_ARG, "idx_host is NULL");
  if (N < 1 || r < 1 || r > N) return fail(nullptr, NKF_ERR_INVALID_ARG, "need 1 <= r <= N");
  draw_indices(N, r, seed, idx_host);
  return NKF_OK;
}

nkf_status nkf_spatial_taps(int radius, double sigma_s, int spatial, int *S_out, float *taps_host) {
  if (!S_out) return fail(nullptr, NKF_ERR_INVALID_ARG, "S_out is NULL");
  if (radius < -1) return fail(nullptr, NKF_ERR_INVALID_ARG, "radius must be >= -1");
  if ((spatial == NKF_SPATIAL_GAUSSIAN || radius < 0) && !(sigma_s > 0.0 && isfinite(sigma_s)))
    return fail(nullptr, NKF_ERR_INVALID_ARG, "sigma_s must be finite and > 0");
  if (spatial == NKF_SPATIAL_RECURSIVE)
    return fail(nullptr, NKF_ERR_UNSUPPORTED, "the recursive Gaussian has no taps");
  if (spatial != NKF_SPATIAL_GAUSSIAN && spatial != NKF_SPATIAL_BOX)
    return fail(nullptr, NKF_ERR_INVALID_ARG, "unknown spatial kernel");
  const int S = resolve_radius(radius, sigma_s);
  if (S > kMaxRadius) return fail(nullptr, NKF_ERR_UNSUPPORTED, "window radius %d exceeds %d", S, kMaxRadius);
  *S_out = S;
  if (taps_host)
    for (int t = -S; t <= S; ++t)
      taps_host[t + S] = spatial == NKF_SPATIAL_BOX ? 1.0f : (float)exp(-(double)t * t / (2.0 * sigma_s * sigma_s));
  return NKF_OK;
}

nkf_status nkf_landmark_factor(int r, int D, const double *centroids_host, double sigma_r, double tau,
                               double *eigvecs_host, double *eigvals_host, double *F_host, int *r_eff) {
  if (r < 1 || r > kMaxLandmarks || D < 1) return fail(nullptr, NKF_ERR_INVALID_ARG, "need 1 <= r <= 256, D >= 1");
  if (!centroids_host || !F_host || !r_eff) return fail(nullptr, NKF_ERR_INVALID_ARG, "NULL pointer");
  if (!(sigma_r > 0.0)) return fail(nullptr, NKF_ERR_INVALID_ARG, "sigma_r must be > 0");
  if (!(tau >= 0.0)) return fail(nullptr, NKF_ERR_INVALID_ARG, "tau must be >= 0");
  return factor(nullptr, r, D, centroids_host, sigma_r, tau, eigvecs_host, eigvals_host, F_host, r_eff);
}

nkf_status nkf_kmeans_iterate(nkf_ctx *ctx, int H, int W, int C, const float *f, int D, const float *p,
                              const nkf_params *prm, float *centroids, int iters, int *labels) {
  Resolved rs;
  nkf_status st = validate(ctx, H, W, C, f, D, p, prm, rs);
  if (st != NKF_OK) return st;
  if (!centroids) return fail(ctx, NKF_ERR_INVALID_ARG, "centroids is NULL");
  if (iters < 0) return fail(ctx, NKF_ERR_INVALID_ARG, "iters must be >= 0");
  Carve dry{nullptr};
  KmBufs kb;
  carve_km(dry, rs, prm->r, kb);
  if ((st = ensure_workspace(ctx, dry.off)) != NKF_OK) return st;
  Carve cv{ctx->ws};
  carve_km(cv, rs, prm->r, kb);
  return run_lloyd(ctx, rs, prm->r, centroids, iters, labels, kb, prm->prec);
}

nkf_status nkf_kmeans(nkf_ctx *ctx, int H, int W, int C, const float *f, int D, const float *p,
                      const nkf_params *prm, float *centroids, int *labels) {
  Resolved rs;
  nkf_status st = validate(ctx, H, W, C, f, D, p, prm, rs);
  if (st != NKF_OK) return st;
  if (!centroids) return fail(ctx, NKF_ERR_INVALID_ARG, "centroids is NULL");
  Carve dry{nullptr};
  KmBufs kb;
  carve_km(dry, rs, prm->r, kb);
  int64_t *idx = dry.take<int64_t>(prm->r);
  if ((st = ensure_workspace(ctx, dry.off)) != NKF_OK) return st;
  Carve cv{ctx->ws};
  carve_km(cv, rs, prm->r, kb);
  idx = cv.take<int64_t>(prm->r);
  if ((st = run_seed(ctx, rs, prm, centroids, idx)) != NKF_OK) return st;
  return run_lloyd(ctx, rs, prm->r, centroids, prm->kmeans_iters, labels, kb, prm->prec);
}

// PCA patch guide (PCA-NLM, Section IV).  Basis from the patches of
// min(N, kPcaSample) pixels (a seeded draw when N is larger), FP64 moments on
// the device, the D x D eigenproblem on the host, projection on the device.
constexpr int kPcaSample = 65536;

nkf_status nkf_patch_pca(nkf_ctx *ctx, int H, int W, int C, const float *f, int patch_radius, int dim,
                         uint64_t seed, float *guide_out, double *eigvals_host) {
  if (!ctx) return fail(nullptr, NKF_ERR_INVALID_ARG, "ctx is NULL");
  if (H < 1 || W < 1 || C < 1) return fail(ctx, NKF_ERR_INVALID_ARG, "sizes must be >= 1 (H=%d W=%d C=%d)", H, W, C);
  if ((int64_t)H * W > (int64_t)1 << 31) return fail(ctx, NKF_ERR_INVALID_ARG, "H*W exceeds 2^31");
  if (!f || !guide_out) return fail(ctx, NKF_ERR_INVALID_ARG, "f and guide_out are required");
  const int pr = patch_radius;
  if (pr < 0) return fail(ctx, NKF_ERR_INVALID_ARG, "patch_radius must be >= 0");
  if (pr > H || pr > W) return fail(ctx, NKF_ERR_INVALID_ARG, "patch_radius exceeds the image");
  const int64_t D64 = (int64_t)(2 * pr + 1) * (2 * pr + 1) * C;
  if (D64 > kMaxGuideDim)
    return fail(ctx, NKF_ERR_UNSUPPORTED, "patch dimension %lld exceeds %d", (long long)D64, kMaxGuideDim);
  const int D = (int)D64;
  if (dim < 1 || dim > D || dim > pca_max_dim())
    return fail(ctx, NKF_ERR_INVALID_ARG, "need 1 <= dim <= min(D = %d, %d) (got %d)", D, pca_max_dim(), dim);
  const int64_t N = (int64_t)H * W;
  const int ns = N > kPcaSample ? kPcaSample : (int)N;
  const int mb = ns < 256 ? ns : 256;
  const int cc = std::max(1, std::min(64, (ns + 63) / 64));
  Guide g{GUIDE_PATCH, nullptr, f, H, W, C, D, pr};
  float *S;
  auto carve = [&](Carve &cv, int64_t *&idx, double *&part, double *&mu, double *&cpart, double *&cov, double *&V) {
    idx = cv.take<int64_t>(ns);
    S = cv.take<float>(pca_sample_floats(D, ns));
    part = cv.take<double>((size_t)mb * D);
    mu = cv.take<double>(D);
    cpart = cv.take<double>((size_t)cc * D * D);
    cov = cv.take<double>((size_t)D * D);
    V = cv.take<double>((size_t)D * dim);
  };
  int64_t *idx;
  double *part, *mu, *cpart, *cov, *V;
  Carve dry{nullptr};
  carve(dry, idx, part, mu, cpart, cov, V);
  nkf_status st;
  if ((st = ensure_workspace(ctx, dry.off)) != NKF_OK) return st;
  const size_t h_idx = (sizeof(int64_t) * ns + 255) & ~(size_t)255;
  const size_t h_cov = (sizeof(double) * D * D + 255) & ~(size_t)255;
  if ((st = ensure_pinned(ctx, h_idx + h_cov + sizeof(double) * D * dim)) != NKF_OK) return st;
  Carve cv{ctx->ws};
  carve(cv, idx, part, mu, cpart, cov, V);
  int64_t *idx_host = reinterpret_cast<int64_t *>(ctx->pinned);
  double *cov_host = reinterpret_cast<double *>(ctx->pinned + h_idx);
  double *V_host = reinterpret_cast<double *>(ctx->pinned + h_idx + h_cov);
  const int64_t *idx_dev = nullptr;
  if (N > ns) {
    if (ctx->pca_draw_N != N || ctx->pca_draw_seed != seed) {
      ctx->pca_draw.resize(ns);
      draw_indices(N, ns, seed, ctx->pca_draw.data());
      ctx->pca_draw_N = N;
      ctx->pca_draw_seed = seed;
    }
    // an earlier call's copy may still read the pinned buffer
    if ((st = pinned_acquire(ctx)) != NKF_OK) return st;
    memcpy(idx_host, ctx->pca_draw.data(), sizeof(int64_t) * ns);
    HIP_TRY(ctx, hipMemcpyAsync(idx, idx_host, sizeof(int64_t) * ns, hipMemcpyHostToDevice, ctx->stream));
    idx_dev = idx;
  }
  HIP_TRY(ctx, launch_pca_moments(g, idx_dev, ns, mb, cc, S, part, mu, cpart, cov, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(cov_host, cov, sizeof(double) * D * D, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  // the dim largest eigenpairs (ascending in w, Q: D x dim)
  std::vector<double> w(dim), Q((size_t)D * dim);
  if (sym_eig_top(D, cov_host, dim, w.data(), Q.data()) != 0)
    return fail(ctx, NKF_ERR_NUMERICAL, "eigendecomposition of the patch covariance did not converge");
  // descending; each vector's largest-magnitude entry (the first on ties) made positive
  for (int k = 0; k < dim; ++k) {
    const int col = dim - 1 - k;
    int jm = 0;
    for (int j = 1; j < D; ++j)
      if (fabs(Q[(size_t)j * dim + col]) > fabs(Q[(size_t)jm * dim + col])) jm = j;
    const double sg = Q[(size_t)jm * dim + col] < 0.0 ? -1.0 : 1.0;
    for (int j = 0; j < D; ++j) V_host[(size_t)j * dim + k] = sg * Q[(size_t)j * dim + col];
    if (eigvals_host) eigvals_host[k] = w[col];
  }
  HIP_TRY(ctx, hipMemcpyAsync(V, V_host, sizeof(double) * D * dim, hipMemcpyHostToDevice, ctx->stream));
  if ((st = pinned_release(ctx)) != NKF_OK) return st;
  HIP_TRY(ctx, launch_pca_project(g, mu, V, dim, guide_out, ctx->stream));
  return NKF_OK;
}

nkf_status nkf_filter_landmarks(nkf_ctx *ctx, int H, int W, int C, const float *f, int D, const float *p,
                                const nkf_params *prm, const float *centroids, const double *F, int r_eff,
                                float *out, float *eta_out) {
  Resolved rs;
  nkf_status st = validate(ctx, H, W, C, f, D, p, prm, rs);
  if (st != NKF_OK) return st;
  if (!centroids || !F || !out) return fail(ctx, NKF_ERR_INVALID_ARG, "centroids, F and out are required");
  if (r_eff < 1 || r_eff > prm->r) return fail(ctx, NKF_ERR_INVALID_ARG, "need 1 <= r_eff <= r");
  Carve dry{nullptr};
  FwdBufs fb;
  const bool u64 = fwd_u64(rs, prm->prec);
  const int wk_r = fwd_wk_r(rs, prm, r_eff);
  carve_fwd(dry, rs, r_eff, fb, kMaxLandmarks, u64, ctx->num_cu, ctx->stats, wk_r);
  if ((st = ensure_workspace(ctx, dry.off)) != NKF_OK) return st;
  Carve cv{ctx->ws};
  carve_fwd(cv, rs, r_eff, fb, kMaxLandmarks, u64, ctx->num_cu, ctx->stats, wk_r);
  // the factor was formed by the caller: no eigenvalues to report
  record_stats(ctx, rs, prm, r_eff, NAN, NAN);
  if ((st = run_fwd(ctx, rs, prm, centroids, F, r_eff, out, eta_out, fb, true, false, true)) != NKF_OK) return st;
  return log_stats(ctx, "filter_landmarks", rs, prm);
}

nkf_status nkf_filter_landmarks_noalloc(nkf_ctx *ctx, int H, int W, int C, const float *f, int D,
                                        const float *p, const nkf_params *prm, const float *centroids,
                                        const double *F, int r_eff, float *out, float *eta_out) {
  Resolved rs;
  nkf_status st = validate(ctx, H, W, C, f, D, p, prm, rs);
  if (st != NKF_OK) return st;
  if (!centroids || !F || !out) return fail(ctx, NKF_ERR_INVALID_ARG, "centroids, F and out are required");
  if (r_eff < 1 || r_eff > prm->r) return fail(ctx, NKF_ERR_INVALID_ARG, "need 1 <= r_eff <= r");
  Carve dry{nullptr};
  FwdBufs fb;
  const bool u64 = fwd_u64(rs, prm->prec);
  const int wk_r = fwd_wk_r(rs, prm, r_eff);
  carve_fwd(dry, rs, r_eff, fb, prm->r, u64, ctx->num_cu, false, wk_r);
  if (dry.off > static_scratch_bytes())
    return fail(ctx, NKF_ERR_OUT_OF_MEMORY,
                "this problem needs %zu bytes of scratch; the static scratch holds %zu (use nkf_filter_landmarks)",
                dry.off, static_scratch_bytes());
  void *base = nullptr;
  const hipError_t e = static_scratch_ptr(ctx->device, &base);
  if (e != hipSuccess)
    return fail(ctx, NKF_ERR_HIP, "static scratch of device %d unavailable: %s", ctx->device, hipGetErrorString(e));
  Carve cv{static_cast<char *>(base)};
  carve_fwd(cv, rs, r_eff, fb, prm->r, u64, ctx->num_cu, false, wk_r);
  // no stage events either: the call enqueues kernels only
  const bool timing = ctx->timing;
  ctx->timing = false;
  st = run_fwd(ctx, rs, prm, centroids, F, r_eff, out, eta_out, fb);
  ctx->timing = timing;
  return st;
}

nkf_status nkf_filter(nkf_ctx *ctx, int H, int W, int C, const float *f, int D, const float *p,
                      const nkf_params *prm, float *out, float *eta_out, int *r_eff_out) {
  Resolved rs;
  nkf_status st = validate(ctx, H, W, C, f, D, p, prm, rs);
  if (st != NKF_OK) return st;
  if (!out) return fail(ctx, NKF_ERR_INVALID_ARG, "out is NULL");
  const int r = prm->r;
  // workspace: k-means buffers and landmark state first, forward buffers sized for r_eff = r
  auto carve_all = [&](Carve &cv, KmBufs &kb, float *&c, int64_t *&idx, double *&Fd, double *&Ad, FwdBufs &fb) {
    carve_km(cv, rs, r, kb);
    c = cv.take<float>((size_t)r * rs.D);
    idx = cv.take<int64_t>(r);
    Fd = cv.take<double>((size_t)r * r);
    Ad = cv.take<double>((size_t)r * r);
    // the 16-bit embedding runs split: its cross-kernel part overlaps the host factor
    carve_fwd(cv, rs, r, fb, kMaxLandmarks, fwd_u64(rs, prm->prec), ctx->num_cu, ctx->stats, fwd_wk_r(rs, prm, r),
              use_mfma_distance(rs.g, prm->prec) ? prm->prec : 0);
  };
  KmBufs kb;
  FwdBufs fb;
  float *c;
  int64_t *idx;
  double *Fd, *Ad;
  Carve dry{nullptr};
  carve_all(dry, kb, c, idx, Fd, Ad, fb);
  if ((st = ensure_workspace(ctx, dry.off)) != NKF_OK) return st;
  const size_t host_bytes = sizeof(double) * ((size_t)r * rs.D + 3 * (size_t)r * r + r) + sizeof(float) * r * rs.D;
  if ((st = ensure_pinned(ctx, 64 * 1024 + host_bytes)) != NKF_OK) return st;
  Carve cv{ctx->ws};
  carve_all(cv, kb, c, idx, Fd, Ad, fb);

  if ((st = run_seed(ctx, rs, prm, c, idx)) != NKF_OK) return st;
  if ((st = run_lloyd(ctx, rs, r, c, prm->kmeans_iters, nullptr, kb, prm->prec)) != NKF_OK) return st;
  // the one host round trip: the landmark Gram matrix A (formed on the
  // device in FP64) to the host for the FP64 eigendecomposition
  int r_eff = 0;
  {
    HIP_TRY(ctx, launch_landmark_gram(c, r, rs.D, prm->sigma_r, Ad, ctx->stream));
    double *A_host = reinterpret_cast<double *>(ctx->pinned);
    HIP_TRY(ctx, hipMemcpyAsync(A_host, Ad, sizeof(double) * r * r, hipMemcpyDeviceToHost, ctx->stream));
    if (!ctx->copy_done) HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->copy_done, hipEventDisableTiming));
    HIP_TRY(ctx, hipEventRecord(ctx->copy_done, ctx->stream));
    // landmark-independent work runs on the device while the host factors A
    const bool mean_ready = prm->kmeans_iters > 0 && use_mfma_kmeans(rs.g, prm->prec);
    if ((st = run_pre(ctx, rs, prm, fb, mean_ready ? kb.mu : nullptr)) != NKF_OK) return st;
    if (fb.bsplit)
      HIP_TRY(ctx, launch_embed_mfma_b(rs.g, c, r, fb.mu, prm->sigma_r, prm->prec, fb.bsplit, fb.lm, ctx->stream));
    HIP_TRY(ctx, hipEventSynchronize(ctx->copy_done));
    // the factor stage is the host's work once the landmarks have arrived, so
    // timing it needs no extra synchronisation
    HostTimer ht(ctx, NKF_STAGE_FACTOR);
    std::vector<double> A(A_host, A_host + (size_t)r * r);
    double *F_host = reinterpret_cast<double *>(ctx->pinned + ((sizeof(double) * r * r + 255) & ~(size_t)255));
    std::vector<double> Fr((size_t)r * r), al(r);
    if ((st = factor_from_gram(ctx, r, A, prm->eig_rel_tol, nullptr, al.data(), Fr.data(), &r_eff)) != NKF_OK)
      return st;
    record_stats(ctx, rs, prm, r_eff, al[r - 1], al[r - r_eff]);
    // pack F [r, r_eff]
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < r_eff; ++j) F_host[i * r_eff + j] = Fr[i * r + j];
    HIP_TRY(ctx, hipMemcpyAsync(Fd, F_host, sizeof(double) * r * r_eff, hipMemcpyHostToDevice, ctx->stream));
    if ((st = pinned_release(ctx)) != NKF_OK) return st;
  }
  if (r_eff_out) *r_eff_out = r_eff;
  if ((st = run_fwd(ctx, rs, prm, c, Fd, r_eff, out, eta_out, fb, true, true, true, fb.bsplit != nullptr)) !=
      NKF_OK)
    return st;
  return log_stats(ctx, "filter", rs, prm);
}

nkf_status nkf_filter_backward(nkf_ctx *ctx, int H, int W, int C, const float *f, int D, const float *p,
                               const nkf_params *prm, const float *centroids, const double *eigvecs_host,
                               const double *eigvals_host, int r_eff, const float *grad_out, float *grad_f,
                               float *grad_p, double *grad_sigma_r_host, double *grad_sigma_s_host,
                               const float *out_fwd, const float *eta_fwd) {
  Resolved rs;
  nkf_status st = validate(ctx, H, W, C, f, D, p, prm, rs);
  if (st != NKF_OK) return st;
  const int r = prm->r;
  if (!centroids || !eigvecs_host || !eigvals_host || !grad_out)
    return fail(ctx, NKF_ERR_INVALID_ARG, "centroids, eigvecs_host, eigvals_host and grad_out are required");
  if (r_eff < 1 || r_eff > r) return fail(ctx, NKF_ERR_INVALID_ARG, "need 1 <= r_eff <= r");
  if (C > 3) return fail(ctx, NKF_ERR_UNSUPPORTED, "backward supports C <= 3 (got %d)", C);
  if (rs.rec && grad_sigma_s_host)
    return fail(ctx, NKF_ERR_UNSUPPORTED, "sigma_s gradient of the recursive Gaussian is not implemented");
  if (r > 64) return fail(ctx, NKF_ERR_UNSUPPORTED, "backward supports r <= 64 (got %d)", r);
  if (grad_p && rs.g.kind == GUIDE_PATCH)
    return fail(ctx, NKF_ERR_UNSUPPORTED, "guide gradient of the patch guide is not implemented");
  if (grad_sigma_r_host && (r_eff != r || isinf(prm->sigma_r)))
    return fail(ctx, NKF_ERR_UNSUPPORTED, "sigma_r gradient needs r_eff == r and finite sigma_r");
  if (grad_sigma_s_host && prm->spatial != NKF_SPATIAL_GAUSSIAN)
    return fail(ctx, NKF_ERR_UNSUPPORTED, "sigma_s gradient needs the Gaussian window");
  // F = Q_keep diag(alpha_keep^{-1/2}), kept = the r_eff largest eigenvalues
  std::vector<double> Fh((size_t)r * r_eff);
  for (int k = 0; k < r_eff; ++k) {
    const int idx = r - r_eff + k;
    const double al = eigvals_host[idx];
    if (!(al > 0.0)) return fail(ctx, NKF_ERR_NUMERICAL, "kept eigenvalue %d is not positive", idx);
    for (int j = 0; j < r; ++j) Fh[(size_t)j * r_eff + k] = eigvecs_host[(size_t)j * r + idx] / sqrt(al);
  }
  const bool want_R = grad_sigma_r_host != nullptr;
  const bool want_S = grad_sigma_s_host != nullptr;
  const int nR = want_R ? r * r_eff : 0;
  const int nred = bwd_reduce_blocks(rs.N);
  const int nsig = bwd_conv_max_blocks(H, W);
  if (bwd_reduce_lds(r, r_eff, rs.D, want_R) > 160 * 1024)
    return fail(ctx, NKF_ERR_UNSUPPORTED, "backward reduction tile does not fit in LDS (r=%d, D=%d)", r, rs.D);

  FwdBufs fb;
  float *out_s, *eta_s, *ab, *dud, *du, *df_s;
  double *Fd, *red, *red2, *sig;
  auto carve_all = [&](Carve &cv) {
    carve_fwd(cv, rs, r_eff, fb, kMaxLandmarks, false, ctx->num_cu);
    out_s = cv.take<float>((size_t)rs.N * C);
    eta_s = cv.take<float>(rs.N);
    ab = cv.take<float>((size_t)rs.N * 4);
    dud = cv.take<float>((size_t)r_eff * rs.N);
    du = cv.take<float>((size_t)r_eff * rs.N);
    df_s = cv.take<float>(grad_f ? 1 : (size_t)rs.N * C);
    Fd = cv.take<double>((size_t)r * r_eff);
    red = cv.take<double>((size_t)nred * (nR + 1));
    red2 = cv.take<double>(bwd_sum_scratch_doubles(nred, nR + 1));
    sig = cv.take<double>(2 * (size_t)nsig);
  };
  Carve dry{nullptr};
  carve_all(dry);
  if ((st = ensure_workspace(ctx, dry.off)) != NKF_OK) return st;
  const size_t host_doubles = (size_t)r * r_eff + (size_t)nred * (nR + 1) + 2 * (size_t)nsig + (size_t)r * rs.D;
  if ((st = ensure_pinned(ctx, 64 * 1024 + sizeof(double) * host_doubles)) != NKF_OK) return st;
  Carve cv{ctx->ws};
  carve_all(cv);
  if ((st = pinned_acquire(ctx)) != NKF_OK) return st;
  double *hF = reinterpret_cast<double *>(ctx->pinned);
  double *hred = hF + (size_t)r * r_eff;
  double *hsig = hred + (size_t)nred * (nR + 1);
  float *hc = reinterpret_cast<float *>(hsig + 2 * (size_t)nsig);
  memcpy(hF, Fh.data(), sizeof(double) * Fh.size());
  int nb1 = 0;
  {
    StageTimer tm(ctx, NKF_STAGE_BACKWARD);
    HIP_TRY(ctx, hipMemcpyAsync(Fd, hF, sizeof(double) * r * r_eff, hipMemcpyHostToDevice, ctx->stream));
    if ((st = pinned_release(ctx)) != NKF_OK) return st;
    // the recursive filter's backward reads the forward's filtered planes, so
    // its forward always runs
    const bool have_fwd = out_fwd && eta_fwd && !rs.rec;
    if ((st = run_fwd(ctx, rs, prm, centroids, Fd, r_eff, out_s, eta_s, fb, !have_fwd)) != NKF_OK) return st;
    const float *outv = have_fwd ? out_fwd : out_s, *etav = have_fwd ? eta_fwd : eta_s;
    HIP_TRY(ctx, launch_bwd_ab(rs.N, C, grad_out, outv, etav, fb.f0, ab, ctx->stream));
    if (rs.rec) {
      RecProblem rp{};
      rp.H = H;
      rp.W = W;
      rp.C = C;
      rp.r_eff = r_eff;
      rp.coef = rs.rc;
      rp.f = f;
      rp.f0 = fb.f0;
      rp.u = fb.u;
      rp.planes = fb.rec;
      rp.G = grad_out;
      rp.eta = etav;
      rp.ab = ab;
      rp.dud = dud;
      rp.du = du;
      rp.df = grad_f ? grad_f : df_s;
      HIP_TRY(ctx, launch_rec_bwd(rp, ctx->stream));
    } else {
      BwdConvProblem bp{};
      bp.H = H;
      bp.W = W;
      bp.C = C;
      bp.S = rs.S;
      bp.r_eff = r_eff;
      bp.f = f;
      bp.f0 = fb.f0;
      bp.u = fb.u;
      bp.ab = ab;
      bp.G = grad_out;
      bp.eta = etav;
      bp.wr = rs.taps;
      bp.wc = rs.taps;
      bp.force_nch = ctx->conv_chunks;
      bp.plane_out = dud;
      if (want_S) {
        // du_dir and the sigma_s terms in one pass over the same planes:
        // dw/dsigma_s = w1' (x) w1 + w1 (x) w1', w1'(t) = w1(t) t^2 / sigma_s^3
        Taps dt = rs.taps;
        const double s3 = prm->sigma_s * prm->sigma_s * prm->sigma_s;
        for (int t = -rs.S; t <= rs.S; ++t)
          dt.w[t + rs.S] = (float)(exp(-(double)t * t / (2.0 * prm->sigma_s * prm->sigma_s)) * t * t / s3);
        bp.mode = 4;  // w1 in wr, w1' in wc
        bp.partials = sig;
        bp.wr = rs.taps;
        bp.wc = dt;
        bp.nblocks_out = &nb1;
        HIP_TRY(ctx, launch_bwd_conv(bp, ctx->stream));
        bp.wr = bp.wc = rs.taps;
        bp.nblocks_out = nullptr;
        bp.partials = nullptr;
      } else {
        bp.mode = 1;
        HIP_TRY(ctx, launch_bwd_conv(bp, ctx->stream));
      }
      bp.mode = 3;
      bp.plane_in = dud;
      bp.plane_out = du;
      bp.df = grad_f ? grad_f : df_s;
      HIP_TRY(ctx, launch_bwd_conv(bp, ctx->stream));
    }
    HIP_TRY(ctx, launch_bwd_reduce(rs.g, centroids, r, Fd, r_eff, prm->sigma_r, du, dud, grad_p, want_R ? 1 : 0,
                                   red, ctx->stream));
  }
  if (!want_R && !want_S) return NKF_OK;
  // the blocks' partials summed on the device; only the sums cross to the host
  hipError_t serr = hipSuccess;
  const double *red_sum = launch_bwd_sum_partials(red, nred, nR + 1, red2, ctx->stream, &serr);
  HIP_TRY(ctx, serr);
  HIP_TRY(ctx, hipMemcpyAsync(hred, red_sum, sizeof(double) * (nR + 1), hipMemcpyDeviceToHost, ctx->stream));
  if (want_S) {
    HIP_TRY(ctx, hipMemcpyAsync(hsig, sig, sizeof(double) * nb1, hipMemcpyDeviceToHost, ctx->stream));
  }
  if (want_R)
    HIP_TRY(ctx, hipMemcpyAsync(hc, centroids, sizeof(float) * r * rs.D, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (want_S) {
    double s = 0.0;
    for (int b = 0; b < nb1; ++b) s += hsig[b];
    *grad_sigma_s_host = s;
  }
  if (want_R) {
    // sigma_r through b, and through M = A^{-1}:  dL/dM = R diag(alpha^{1/2}) Q^T,
    // dL/dA = -M (dL/dM) M,  dA_ij/dsigma_r = A_ij D_ij / sigma_r^3
    double sr_b = 0.0;
    std::vector<double> R((size_t)r * r, 0.0);
    sr_b = hred[0];
    for (int e = 0; e < nR; ++e) R[e] = hred[1 + e];
    const double *Q = eigvecs_host, *al = eigvals_host;
    std::vector<double> GM((size_t)r * r, 0.0), M((size_t)r * r, 0.0), T1((size_t)r * r, 0.0);
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < r; ++j) {
        double gm = 0.0, m = 0.0;
        for (int k = 0; k < r; ++k) {
          gm += R[(size_t)i * r + k] * sqrt(al[k]) * Q[(size_t)j * r + k];
          m += Q[(size_t)i * r + k] * Q[(size_t)j * r + k] / al[k];
        }
        GM[(size_t)i * r + j] = gm;
        M[(size_t)i * r + j] = m;
      }
    for (int i = 0; i < r; ++i)  // T1 = M GM
      for (int j = 0; j < r; ++j) {
        double s = 0.0;
        for (int k = 0; k < r; ++k) s += M[(size_t)i * r + k] * GM[(size_t)k * r + j];
        T1[(size_t)i * r + j] = s;
      }
    double sr_a = 0.0;
    const double inv2 = 1.0 / (2.0 * prm->sigma_r * prm->sigma_r);
    const double s3 = prm->sigma_r * prm->sigma_r * prm->sigma_r;
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < r; ++j) {
        double ga = 0.0;  // (M GM M)_ij
        for (int k = 0; k < r; ++k) ga += T1[(size_t)i * r + k] * M[(size_t)k * r + j];
        double d2 = 0.0;
        for (int d = 0; d < rs.D; ++d) {
          const double t = (double)hc[i * rs.D + d] - (double)hc[j * rs.D + d];
          d2 += t * t;
        }
        sr_a += -ga * exp(-d2 * inv2) * d2 / s3;
      }
    *grad_sigma_r_host = sr_b + sr_a;
  }
  return NKF_OK;
}

}  // extern "C"
