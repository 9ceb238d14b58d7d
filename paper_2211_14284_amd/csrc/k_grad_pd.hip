// HIP kernels (gfx950) of the H(grad) relaxation with the paper's auxiliary operator
// on trilinear cells (eq. sum-factorization_approx: the weighted mass matrices
// replaced by their diagonals in the broken bases), steps 1 and 4 of eq. schur:
//   condensation   rt_G = r_G - P_GI P_II^{-1} r_I
//   extension      z_I  = P_II^{-1} (r_I - P_IG z_G)
// P_II is diagonal (the interior FDM functions are unchanged by the broken
// transformation, and D has one entry in each interior column), and an interior DoF
// t couples only to the face DoFs at the two ends of its lines, with
//   P(t, u) = D[t_d][e] w_d(t),   w_d(t) = sqrt(lambda_{t_d}) da_d(t),
// for the face DoF u at local end e along axis d.  pii and w_d are lattice arrays
// (entries at cell-interior points; every such point belongs to one cell).  The patch
// solves between the two steps are those of the separable path.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace rz {

namespace {

__device__ __forceinline__ bool pd_dirichlet(const LatDev &L, int X, int Y, int Z) {
  return ((L.dir & 1u) && X == 0) || ((L.dir & 2u) && X == L.Nx - 1) || ((L.dir & 4u) && Y == 0) ||
         ((L.dir & 8u) && Y == L.Ny - 1) || ((L.dir & 16u) && Z == 0) || ((L.dir & 32u) && Z == L.Nz - 1);
}

__device__ __forceinline__ long pd_index(const LatDev &L, const int C[3]) {
  return (long)C[0] + (long)L.Nx * ((long)C[1] + (long)L.Ny * (long)C[2]);
}

// Condensation, one thread per lattice point: rt = 0 on Dirichlet points, r at
// points with two or more coordinates on vertex planes, and at a face point (one
// coordinate on a vertex plane, axis d) r minus the interior points of its normal
// line in the (up to two) cells that share the face.  Interior points of rt are
// not written.
template <typename T>
__global__ void k_condense_pd(LatDev L, PdSolve<T> S, const T *__restrict__ r, T *__restrict__ rt, long n) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const int p = L.p;
  const int C[3] = {(int)(g % L.Nx), (int)((g / L.Nx) % L.Ny), (int)(g / ((long)L.Nx * L.Ny))};
  const int on = (C[0] % p == 0) + (C[1] % p == 0) + (C[2] % p == 0);
  if (on == 0) return;
  if (pd_dirichlet(L, C[0], C[1], C[2])) {
    rt[g] = T(0);
    return;
  }
  T val = r[g];
  if (on == 1) {
    const int d = C[0] % p == 0 ? 0 : (C[1] % p == 0 ? 1 : 2);
    const int nc = d == 0 ? L.nx : (d == 1 ? L.ny : L.nz);
    const int k = C[d] / p;
    const T *w = d == 0 ? S.w0 : (d == 1 ? S.w1 : S.w2);
    const int n1 = p + 1;
    // the cell below (its local end p), then the cell above (local end 0)
    for (int side = 0; side < 2; ++side) {
      const int cell = side == 0 ? k - 1 : k;
      if (cell < 0 || cell >= nc) continue;
      const int e = side == 0 ? p : 0;
      T acc = 0;
      for (int i = 1; i < p; ++i) {
        int t[3] = {C[0], C[1], C[2]};
        t[d] = cell * p + i;
        const long gt = pd_index(L, t);
        acc += S.D[i * n1 + e] * w[gt] * (r[gt] / S.pii[gt]);
      }
      val -= acc;
    }
  }
  rt[g] = val;
}

// Extension, one thread per cell-interior point t:
//   z_t = (scale r_t - sum_d sum_e D[t_d][e] w_d(t) z_e) / pii(t)
// with z_e the (already scaled) plane values at the ends of t's lines (Dirichlet ends
// count as 0); with acc: acc_t += w z_t instead of storing z_t.
template <typename T>
__global__ void k_expand_interior_pd(LatDev L, PdSolve<T> S, const T *__restrict__ r, T *__restrict__ z, T scale,
                                     T wgt, T *__restrict__ acc, long n) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const int p = L.p, n1 = p + 1;
  const int C[3] = {(int)(g % L.Nx), (int)((g / L.Nx) % L.Ny), (int)(g / ((long)L.Nx * L.Ny))};
  if (C[0] % p == 0 || C[1] % p == 0 || C[2] % p == 0) return;
  T val = scale * r[g];
  for (int d = 0; d < 3; ++d) {
    const T *w = d == 0 ? S.w0 : (d == 1 ? S.w1 : S.w2);
    const int lt = C[d] % p, base = C[d] - lt;
    T s = 0;
    for (int side = 0; side < 2; ++side) {
      int u[3] = {C[0], C[1], C[2]};
      u[d] = base + (side ? p : 0);
      const T zu = pd_dirichlet(L, u[0], u[1], u[2]) ? T(0) : z[pd_index(L, u)];
      s += S.D[lt * n1 + (side ? p : 0)] * zu;
    }
    val -= w[g] * s;
  }
  const T out = val / S.pii[g];
  if (acc) acc[g] += wgt * out;
  else z[g] = out;
}

inline unsigned pd_blocks(long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

template <typename T>
void launch_condense_pd(const LatDev &L, const PdSolve<T> &S, const T *r, T *rt, hipStream_t s) {
  const long n = (long)L.Nx * L.Ny * L.Nz;
  k_condense_pd<T><<<pd_blocks(n), 256, 0, s>>>(L, S, r, rt, n);
}

template <typename T>
void launch_expand_interior_pd(const LatDev &L, const PdSolve<T> &S, const T *r, T *z, T scale, T w, T *acc,
                               hipStream_t s) {
  const long n = (long)L.Nx * L.Ny * L.Nz;
  k_expand_interior_pd<T><<<pd_blocks(n), 256, 0, s>>>(L, S, r, z, scale, w, acc, n);
}

template void launch_condense_pd<double>(const LatDev &, const PdSolve<double> &, const double *, double *,
                                         hipStream_t);
template void launch_condense_pd<float>(const LatDev &, const PdSolve<float> &, const float *, float *, hipStream_t);
template void launch_expand_interior_pd<double>(const LatDev &, const PdSolve<double> &, const double *, double *,
                                                double, double, double *, hipStream_t);
template void launch_expand_interior_pd<float>(const LatDev &, const PdSolve<float> &, const float *, float *, float,
                                               float, float *, hipStream_t);

}  // namespace rz
