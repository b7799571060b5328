// Forward convolutions + contraction + normalisation (Section III,
// Eqs. (finalnum), (finalden); Algorithm 1 accumulation loop).  The kernel
// body is in conv_core.h; this file instantiates it for every window radius
// and picks the plane grouping from the channel count.
#include <hip/hip_runtime.h>

#include "conv_core.h"

namespace nkf {

namespace {

using namespace conv;

template <int S>
hipError_t launch_S(ConvArgs a, hipStream_t s) {
  const int C = a.C;
  if (C == 1) return launch_one<S, 2, true, 32, MODE_FWD>(a, s, 1, 1);
  if (C <= 3) return launch_one<S, 4, true, 32, MODE_FWD, 512>(a, s, 3, 1);
  // eta pass, then channel chunks that read eta
  hipError_t e = launch_one<S, 1, true, 32, MODE_FWD>(a, s, 0, 1);
  if (e != hipSuccess) return e;
  ConvArgs b = a;
  b.eta_out = nullptr;
  return launch_one<S, 4, false, 32, MODE_FWD, 512>(b, s, 4, (C + 3) / 4);
}

}  // namespace

hipError_t launch_conv_contract(const ConvProblem &pb, hipStream_t s) {
  if (pb.box && pb.C <= 3) return launch_conv_contract_box(pb, s);
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
  for (int t = 0; t < 2 * kMaxRadius + 1; ++t) a.wr[t] = a.wc[t] = (double)pb.taps.w[t];
  switch (pb.S) {
#define NKF_CASE(SV) \
  case SV:           \
    return launch_S<SV>(a, s);
    NKF_CASE(0) NKF_CASE(1) NKF_CASE(2) NKF_CASE(3) NKF_CASE(4) NKF_CASE(5) NKF_CASE(6) NKF_CASE(7)
    NKF_CASE(8) NKF_CASE(9) NKF_CASE(10) NKF_CASE(11) NKF_CASE(12) NKF_CASE(13) NKF_CASE(14)
    NKF_CASE(15) NKF_CASE(16)
#undef NKF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace nkf
