// Fused GW (Remark, Entropic algorithm for FGW).  The fused objective is
// (1 - theta) sum c_ip^2 T_ip + theta E(T); its gradient is
// (1 - theta) C o C + theta grad E (the Remark's C_2 - 4 theta D_X T D_Y).  The
// feature cost here is c_ip = fa_i - fb_p.  The library works with half
// gradients (G = grad E / 2), so
//   * a solve's Sinkhorn cost 2 G_fgw needs G_fgw = theta G + (1 - theta)/2 c^2;
//   * the fused objective is sum_ip T_ip (theta G' + (1 - theta) c_ip^2), G' the
//     half gradient with T's own marginals.
// Both are one elementwise step on a computed G:  G <- a G + b (fa_i - fb_p)^2.
// The FAST kernels that write G (1D tile sweep, separable 2D write) apply it
// as they store; this standalone pass serves the paths whose output kernel
// does not (dense, generic 2D).
#include "common.h"
#include "runtime.h"

namespace {

constexpr int FB_NT = 256;

// One block per row of G; the row's feature value is read once.
__global__ __launch_bounds__(FB_NT) void k_fgw_blend(double* __restrict__ G, int64_t ldG, int N,
                                                      const double* __restrict__ fa,
                                                      const double* __restrict__ fb, double a,
                                                      double b) {
  const int64_t i = blockIdx.x;
  const double fai = fa[i];
  double* row = G + i * ldG;
#pragma unroll 4
  for (int p = threadIdx.x; p < N; p += FB_NT) {
    const double d = fai - fb[p];
    row[p] = fma(a, row[p], b * (d * d));
  }
}

}  // namespace

namespace gwl {

gw_status fgw_blend(double* G, int64_t ldG, int64_t M, int64_t N, const double* fa,
                    const double* fb, double a, double b, hipStream_t s) {
  gwr::ProfScope ps(gwr::kFamOther, s);
  k_fgw_blend<<<(unsigned)M, FB_NT, 0, s>>>(G, ldG, (int)N, fa, fb, a, b);
  return gwr::last_launch_status();
}

}  // namespace gwl
