// Forward convolutions + contraction + normalisation for the box spatial
// kernel (Section IV: the box window of the nonlocal-means experiments) on
// images with up to three channels: the same fused kernel as for the
// Gaussian, with sliding FP64 window sums in place of the FIR passes.
#include <hip/hip_runtime.h>

#include "conv_core.h"

namespace nkf {

namespace {

using namespace conv;

template <int S>
hipError_t launch_box_S(ConvArgs a, hipStream_t s) {
  if (a.C == 1) return launch_one<S, 2, true, 32, MODE_FWD, kBlock, true>(a, s, 1, 1);
  return launch_one<S, 4, true, 32, MODE_FWD, 512, true>(a, s, 3, 1);
}

}  // namespace

hipError_t launch_conv_contract_box(const ConvProblem &pb, hipStream_t s) {
  if (pb.C > 3) return hipErrorInvalidValue;
  ConvArgs a{};
  a.H = pb.H;
  a.W = pb.W;
  a.C = pb.C;
  a.r_eff = pb.r_eff;
  a.f = pb.f;
  a.f0 = pb.f0;
  a.u = pb.u;
  a.out = pb.out;
  a.eta_out = pb.eta_out;
  a.eta_buf = pb.eta_buf;
  a.force_nch = pb.force_nch;
  for (int t = 0; t < 2 * kMaxRadius + 1; ++t) a.wr[t] = a.wc[t] = 1.0;
  switch (pb.S) {
#define NKF_CASE(SV) \
  case SV:           \
    return launch_box_S<SV>(a, s);
    NKF_CASE(0) NKF_CASE(1) NKF_CASE(2) NKF_CASE(3) NKF_CASE(4) NKF_CASE(5) NKF_CASE(6) NKF_CASE(7)
    NKF_CASE(8) NKF_CASE(9) NKF_CASE(10) NKF_CASE(11) NKF_CASE(12) NKF_CASE(13) NKF_CASE(14)
    NKF_CASE(15) NKF_CASE(16)
#undef NKF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace nkf
