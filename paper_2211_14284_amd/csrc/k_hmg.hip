// HIP kernels (gfx950) of the geometric h-multigrid V(1,1) cycle on the Q_1 space
// (the h-coarse solver below p = 1, Sec. 5.1) with damped point Jacobi relaxation,
// and on the lowest-order H(curl)/H(div) spaces its Hiptmair form (Jacobi in the
// space, then in the potential space): one matrix row per lane, FP64.  Each level
// of the cycle is four launches (ten with the potential steps); the
// coarsest level's dense inverse is applied by the symmetric product of the
// H(curl)/H(div) coarse solve.  Every sum runs in the order of the row's entries
// (deterministic, no atomics).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace rz {

namespace {

constexpr int kRowBS = 64;  // one wavefront per block: the small levels still spread over the CUs

// Matrices in ELL form, entry k of row i at k * n + i (the loads of a wavefront's
// rows are contiguous), padded rows with column i and value 0.  W > 0 fixes the
// width at compile time (the host pads every matrix to one of the widths the
// launcher lists, e.g. 27 for the Q_1 operators), so that every column index, then
// every gathered value, of a row is loaded at once instead of as a chain of
// dependent loads.
// mode HMG_RES0:  out = b - A (w D^{-1} b)          (pre-relaxation from zero, then residual)
// mode HMG_PROD:  out = M x                          (restriction)
// mode HMG_PROL:  out = w D^{-1} b + P x             (pre-relaxed iterate plus the correction)
// mode HMG_POST:  out = x + w D^{-1} (b - A x)       (post-relaxation)
// mode HMG_RES:   out = b - A x                      (residual)
// mode HMG_ADD:   out = b + M x                      (interpolated correction added to b)
// mode HMG_JPROD: out = w D^{-1} (M x)               (Jacobi step on a restricted residual)
template <int W>
__global__ void __launch_bounds__(kRowBS) k_hmg_row(int mode, int n, int width, const int *__restrict__ col,
                                                    const double *__restrict__ val, const double *__restrict__ x,
                                                    const double *__restrict__ b, const double *__restrict__ dinv,
                                                    double w, double *__restrict__ out) {
  const int i = blockIdx.x * kRowBS + threadIdx.x;
  if (i >= n) return;
  const int wd = W > 0 ? W : width;
  double s = 0.0;
  if (mode == HMG_RES0) {
#pragma unroll
    for (int k = 0; k < wd; ++k) {
      const long e = (long)k * n + i;
      const int j = col[e];
      s += val[e] * (w * dinv[j] * b[j]);
    }
    out[i] = b[i] - s;
    return;
  }
#pragma unroll
  for (int k = 0; k < wd; ++k) {
    const long e = (long)k * n + i;
    s += val[e] * x[col[e]];
  }
  if (mode == HMG_PROD) out[i] = s;
  else if (mode == HMG_PROL) out[i] = w * dinv[i] * b[i] + s;
  else if (mode == HMG_RES) out[i] = b[i] - s;
  else if (mode == HMG_ADD) out[i] = b[i] + s;
  else if (mode == HMG_JPROD) out[i] = w * dinv[i] * s;
  else out[i] = x[i] + w * dinv[i] * (b[i] - s);
}

}  // namespace

void launch_hmg_row(int mode, int n, int width, const int *col, const double *val, const double *x,
                    const double *b, const double *dinv, double w, double *out, hipStream_t s) {
  if (n <= 0) return;
  const unsigned g = (unsigned)((n + kRowBS - 1) / kRowBS);
#define RZ_HMG_W(W) \
  case W: k_hmg_row<W><<<g, kRowBS, 0, s>>>(mode, n, width, col, val, x, b, dinv, w, out); break;
  switch (width) {
    RZ_HMG_W(2) RZ_HMG_W(4) RZ_HMG_W(6) RZ_HMG_W(8) RZ_HMG_W(12) RZ_HMG_W(16) RZ_HMG_W(18) RZ_HMG_W(20)
    RZ_HMG_W(24) RZ_HMG_W(27) RZ_HMG_W(28) RZ_HMG_W(32) RZ_HMG_W(36) RZ_HMG_W(40) RZ_HMG_W(48) RZ_HMG_W(64)
    default: k_hmg_row<0><<<g, kRowBS, 0, s>>>(mode, n, width, col, val, x, b, dinv, w, out); break;
  }
#undef RZ_HMG_W
}

}  // namespace rz
