// HIP kernels (gfx950) of the operator apply in H(curl) (NCE_p) and H(div) (NCF_p)
// on axis-aligned cells with cellwise-constant coefficients (eq. sum-factorization
// with the exact 1-D integrals; Sec. 2.4 bases, eqs. curlbasis / divbasis):
//   curl: y_K = sum_m mu_m ME_m u_m + sum_n sigma_n C_n^T MF_n C_n u,
//         ME_m = I along m, B along the other axes;  MF_n = B along n, I elsewhere;
//         (C u)_0 = D_y u_2 - D_z u_1, (C u)_1 = D_z u_0 - D_x u_2, (C u)_2 = D_x u_1 - D_y u_0;
//   div:  y_K = sum_m mu_m MF_m u_m + sigma D_m^T (sum_n D_n u_n).
// In the FDM bases every 1-D factor is sparse (B: diagonal plus (0,p); D: at most
// three entries per row), so each line costs O(p).  A few cells per block; tiles of
// the three components and of the intermediate fields live in LDS.  Interior rows
// of a component (no continuous axis at an end) are stored, the others go to a
// per-cell buffer summed by the gather kernel in a fixed cell order.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace rz {

namespace {

constexpr int kMaxP = 9;

// component m of a space: kind along each axis (true = continuous P, false = DP)
__device__ __forceinline__ bool is_P(int space, int m, int a) { return space == 1 ? a != m : a == m; }

__device__ __forceinline__ bool comp_dirichlet(const VecDev &V, int m, const int C[3]) {
  for (int a = 0; a < 3; ++a) {
    if (!is_P(V.space, m, a)) continue;
    if ((V.dir & (1u << (2 * a))) && C[a] == 0) return true;
    if ((V.dir & (1u << (2 * a + 1))) && C[a] == V.ext[m][a] - 1) return true;
  }
  return false;
}

__device__ __forceinline__ long comp_index(const VecDev &V, int m, const int C[3]) {
  return V.off[m] + (long)C[0] + (long)V.ext[m][0] * ((long)C[1] + (long)V.ext[m][1] * (long)C[2]);
}

enum { OP_B = 0, OP_D = 1, OP_DT = 2 };

// ---- the apply, degree P known at compile time ----------------------------------------
// CPB cells per block, every tile sized for P in dynamic LDS; in each pass one thread
// per line of one cell applies a 1-D factor (B: diagonal plus (0,p); D: at most three
// entries per row) with unrolled loops, values held in registers; the cell weights
// scale whole tiles between passes.
template <int P>
struct TileP {
  int e[3];
  __device__ int size() const { return e[0] * e[1] * e[2]; }
};

template <int P, typename T>
__device__ __forceinline__ void line_op_p(const T *in, int csi, TileP<P> ti, T *out, int cso, TileP<P> to, int ax,
                                          int op, const T *sB, const T *sD, T scale, bool acc, int ncells) {
  constexpr int n1 = P + 1;
  const int b = ax == 0 ? 1 : 0, c = ax == 2 ? 1 : 2;
  const int nl = ti.e[b] * ti.e[c];
  const int sti = ax == 0 ? 1 : (ax == 1 ? ti.e[0] : ti.e[0] * ti.e[1]);
  const int sto = ax == 0 ? 1 : (ax == 1 ? to.e[0] : to.e[0] * to.e[1]);
  const int nin = ti.e[ax], nout = to.e[ax];
  for (int t = threadIdx.x; t < nl * ncells; t += blockDim.x) {
    const int cl = t / nl, l = t % nl;
    const int u = l % ti.e[b], w = l / ti.e[b];
    int ci[3], co[3];
    ci[ax] = co[ax] = 0;
    ci[b] = co[b] = u;
    ci[c] = co[c] = w;
    const T *ip = in + cl * csi + ci[0] + ti.e[0] * (ci[1] + ti.e[1] * ci[2]);
    T *op_ = out + cl * cso + co[0] + to.e[0] * (co[1] + to.e[1] * co[2]);
    T v[n1], r[n1];
#pragma unroll
    for (int i = 0; i < n1; ++i) v[i] = i < nin ? ip[i * sti] : T(0);
    if (op == OP_B) {
#pragma unroll
      for (int i = 0; i <= P; ++i) r[i] = sB[i * n1 + i] * v[i];
      r[0] += sB[P] * v[P];
      r[P] += sB[P * n1] * v[0];
    } else if (op == OP_D) {
#pragma unroll
      for (int i = 0; i < P; ++i) {
        T s = sD[i * n1] * v[0] + sD[i * n1 + P] * v[P];
        if (i >= 1) s += sD[i * n1 + i] * v[i];
        r[i] = s;
      }
      r[P] = 0;
    } else {
      T r0 = 0, rp = 0;
#pragma unroll
      for (int i = 0; i < P; ++i) {
        r0 += sD[i * n1] * v[i];
        rp += sD[i * n1 + P] * v[i];
      }
#pragma unroll
      for (int j = 1; j < P; ++j) r[j] = sD[j * n1 + j] * v[j];
      r[0] = r0;
      r[P] = rp;
    }
#pragma unroll
    for (int i = 0; i < n1; ++i)
      if (i < nout) {
        const T val = scale * r[i];
        op_[i * sto] = acc ? op_[i * sto] + val : val;
      }
  }
}

template <int P>
__device__ __forceinline__ TileP<P> tile_p(int space, int m) {
  TileP<P> t;
  for (int a = 0; a < 3; ++a) t.e[a] = is_P(space, m, a) ? P + 1 : P;
  return t;
}

template <int P, typename T, int CPB>
__global__ void __launch_bounds__(256) k_apply_vec_p(VecDev V, const T *__restrict__ coef, const T *__restrict__ Bg,
                                                      const T *__restrict__ Dg, const T *__restrict__ x,
                                                      T *__restrict__ y, T *__restrict__ ebuf, long ncells) {
  // TS: a component tile (the largest, NCE: p(p+1)^2); TF: a tile of the derived field
  // (NCF for the curl, DQ for the divergence).  F also holds the mass pass's
  // intermediate component tile, so it takes TS values per cell.
  constexpr int TS = P * (P + 1) * (P + 1), TF = (P + 1) * P * P;
  extern __shared__ unsigned char vsm[];
  T *U = reinterpret_cast<T *>(vsm);         // [CPB][3][TS]
  T *Y = U + CPB * 3 * TS;                    // [CPB][3][TS]
  T *F = Y + CPB * 3 * TS;                    // [CPB][TS]
  T *G = F + CPB * TS;                        // [CPB][TF]
  T *sB = G + CPB * TF;
  T *sD = sB + (P + 1) * (P + 1);
  const int space = V.space;
  const long c0 = (long)blockIdx.x * CPB;
  const int nc = (int)min((long)CPB, ncells - c0);
  for (int k = threadIdx.x; k < (P + 1) * (P + 1); k += blockDim.x) sB[k] = Bg[k];
  for (int k = threadIdx.x; k < P * (P + 1); k += blockDim.x) sD[k] = Dg[k];
  TileP<P> tc[3];
  for (int m = 0; m < 3; ++m) tc[m] = tile_p<P>(space, m);
  for (int m = 0; m < 3; ++m) {
    const int ts = tc[m].size();
    for (int t = threadIdx.x; t < ts * nc; t += blockDim.x) {
      const int cl = t / ts, k = t % ts;
      const long cell = c0 + cl;
      const int cc[3] = {(int)(cell % V.nx), (int)((cell / V.nx) % V.ny), (int)(cell / ((long)V.nx * V.ny))};
      const int l[3] = {k % tc[m].e[0], (k / tc[m].e[0]) % tc[m].e[1], k / (tc[m].e[0] * tc[m].e[1])};
      const int C[3] = {cc[0] * P + l[0], cc[1] * P + l[1], cc[2] * P + l[2]};
      U[(cl * 3 + m) * TS + k] = comp_dirichlet(V, m, C) ? T(0) : x[comp_index(V, m, C)];
    }
  }
  __syncthreads();
  // per-cell weights in registers of the thread's cell are read from global per pass
  if (space == 1) {
    for (int m = 0; m < 3; ++m) {
      const int b = m == 0 ? 1 : 0, c = m == 2 ? 1 : 2;
      line_op_p<P>(U + m * TS, 3 * TS, tc[m], F, TS, tc[m], b, OP_B, sB, sD, T(1), false, nc);
      __syncthreads();
      // scale per cell: mu_m; a pass per cell-weight would split the lines, so scale
      // after the second factor below
      line_op_p<P>(F, TS, tc[m], Y + m * TS, 3 * TS, tc[m], c, OP_B, sB, sD, T(1), false, nc);
      __syncthreads();
      for (int t = threadIdx.x; t < tc[m].size() * nc; t += blockDim.x) {
        const int cl = t / tc[m].size(), k = t % tc[m].size();
        Y[(cl * 3 + m) * TS + k] *= coef[6 * (c0 + cl) + 3 + m];
      }
      __syncthreads();
    }
    for (int n = 0; n < 3; ++n) {
      const int a1 = (n + 1) % 3, a2 = (n + 2) % 3;
      TileP<P> tf;
      for (int a = 0; a < 3; ++a) tf.e[a] = a == n ? P + 1 : P;
      line_op_p<P>(U + a2 * TS, 3 * TS, tc[a2], F, TS, tf, a1, OP_D, sB, sD, T(1), false, nc);
      __syncthreads();
      line_op_p<P>(U + a1 * TS, 3 * TS, tc[a1], F, TS, tf, a2, OP_D, sB, sD, T(-1), true, nc);
      __syncthreads();
      line_op_p<P>(F, TS, tf, G, TF, tf, n, OP_B, sB, sD, T(1), false, nc);
      __syncthreads();
      for (int t = threadIdx.x; t < tf.size() * nc; t += blockDim.x) {
        const int cl = t / tf.size(), k = t % tf.size();
        G[cl * TF + k] *= coef[6 * (c0 + cl) + n];
      }
      __syncthreads();
      line_op_p<P>(G, TF, tf, Y + a2 * TS, 3 * TS, tc[a2], a1, OP_DT, sB, sD, T(1), true, nc);
      __syncthreads();
      line_op_p<P>(G, TF, tf, Y + a1 * TS, 3 * TS, tc[a1], a2, OP_DT, sB, sD, T(-1), true, nc);
      __syncthreads();
    }
  } else {
    for (int m = 0; m < 3; ++m) line_op_p<P>(U + m * TS, 3 * TS, tc[m], Y + m * TS, 3 * TS, tc[m], m, OP_B, sB, sD,
                                             T(1), false, nc);
    __syncthreads();
    for (int m = 0; m < 3; ++m)
      for (int t = threadIdx.x; t < tc[m].size() * nc; t += blockDim.x) {
        const int cl = t / tc[m].size(), k = t % tc[m].size();
        Y[(cl * 3 + m) * TS + k] *= coef[6 * (c0 + cl) + 3 + m];
      }
    TileP<P> tq;
    tq.e[0] = tq.e[1] = tq.e[2] = P;
    for (int m = 0; m < 3; ++m) {
      line_op_p<P>(U + m * TS, 3 * TS, tc[m], F, TS, tq, m, OP_D, sB, sD, T(1), m > 0, nc);
      __syncthreads();
    }
    for (int t = threadIdx.x; t < tq.size() * nc; t += blockDim.x) {
      const int cl = t / tq.size(), k = t % tq.size();
      F[cl * TS + k] *= coef[6 * (c0 + cl)];
    }
    __syncthreads();
    for (int m = 0; m < 3; ++m) line_op_p<P>(F, TS, tq, Y + m * TS, 3 * TS, tc[m], m, OP_DT, sB, sD, T(1), true, nc);
    __syncthreads();
  }
  for (int m = 0; m < 3; ++m) {
    int coff = 0;
    for (int k = 0; k < m; ++k) coff += tc[k].size();
    const int ts = tc[m].size();
    for (int t = threadIdx.x; t < ts * nc; t += blockDim.x) {
      const int cl = t / ts, k = t % ts;
      const long cell = c0 + cl;
      const int cc[3] = {(int)(cell % V.nx), (int)((cell / V.nx) % V.ny), (int)(cell / ((long)V.nx * V.ny))};
      const int l[3] = {k % tc[m].e[0], (k / tc[m].e[0]) % tc[m].e[1], k / (tc[m].e[0] * tc[m].e[1])};
      bool owned = true;
      for (int a = 0; a < 3; ++a)
        if (is_P(space, m, a) && (l[a] == 0 || l[a] == P)) owned = false;
      const T val = Y[(cl * 3 + m) * TS + k];
      if (owned) {
        const int C[3] = {cc[0] * P + l[0], cc[1] * P + l[1], cc[2] * P + l[2]};
        y[comp_index(V, m, C)] = val;
      } else {
        ebuf[cell * (long)V.cell_dofs + coff + k] = val;
      }
    }
  }
}

// Shared rows: sum of the contributions of the cells holding the DoF (fixed order:
// z, y, x of the cells); Dirichlet rows copy x.
template <typename T>
__global__ void k_apply_vec_gather(VecDev V, const T *__restrict__ x, const T *__restrict__ ebuf,
                                   T *__restrict__ y, long n) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  int m = 0;
  while (m < 2 && g >= V.off[m + 1]) ++m;
  const long r = g - V.off[m];
  const int C[3] = {(int)(r % V.ext[m][0]), (int)((r / V.ext[m][0]) % V.ext[m][1]),
                    (int)(r / ((long)V.ext[m][0] * V.ext[m][1]))};
  const int p = V.p, space = V.space;
  bool shared = false;
  for (int a = 0; a < 3; ++a)
    if (is_P(space, m, a) && C[a] % p == 0) shared = true;
  if (!shared) return;
  if (comp_dirichlet(V, m, C)) {
    y[g] = x[g];
    return;
  }
  const int nc[3] = {V.nx, V.ny, V.nz};
  int cl[3][2], lo[3][2], cnt[3];
  for (int a = 0; a < 3; ++a) {
    cnt[a] = 0;
    if (is_P(space, m, a) && C[a] % p == 0) {
      const int c = C[a] / p;
      if (c - 1 >= 0) {
        cl[a][cnt[a]] = c - 1;
        lo[a][cnt[a]++] = p;
      }
      if (c < nc[a]) {
        cl[a][cnt[a]] = c;
        lo[a][cnt[a]++] = 0;
      }
    } else {
      cl[a][0] = C[a] / p;
      lo[a][0] = C[a] % p;
      cnt[a] = 1;
    }
  }
  int coff = 0, e[3];
  for (int k = 0; k < m; ++k) {
    int s = 1;
    for (int a = 0; a < 3; ++a) s *= is_P(space, k, a) ? p + 1 : p;
    coff += s;
  }
  for (int a = 0; a < 3; ++a) e[a] = is_P(space, m, a) ? p + 1 : p;
  T acc = 0;
  for (int k = 0; k < cnt[2]; ++k)
    for (int j = 0; j < cnt[1]; ++j)
      for (int i = 0; i < cnt[0]; ++i) {
        const long cell = cl[0][i] + (long)V.nx * (cl[1][j] + (long)V.ny * cl[2][k]);
        acc += ebuf[cell * V.cell_dofs + coff + lo[0][i] + e[0] * (lo[1][j] + e[1] * lo[2][k])];
      }
  y[g] = acc;
}

}  // namespace

template <int P, typename T>
void apply_vec_p(const VecDev &V, const T *coef, const T *B, const T *D, const T *x, T *y, T *ebuf, long nc,
                 hipStream_t s) {
  constexpr int TS = P * (P + 1) * (P + 1), TF = (P + 1) * P * P;
  constexpr size_t per_cell = (7 * (size_t)TS + (size_t)TF) * sizeof(T);
  constexpr int CPB = per_cell * 4 <= 64 * 1024 ? 4 : (per_cell * 2 <= 64 * 1024 ? 2 : 1);
  const size_t shm = CPB * per_cell + ((P + 1) * (P + 1) + P * (P + 1)) * sizeof(T);
  if (shm > 64 * 1024)
    hipFuncSetAttribute((const void *)k_apply_vec_p<P, T, CPB>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  k_apply_vec_p<P, T, CPB><<<(unsigned)((nc + CPB - 1) / CPB), 256, shm, s>>>(V, coef, B, D, x, y, ebuf, nc);
}

template <typename T>
int launch_apply_vec(const VecDev &V, const T *coef, const T *B, const T *D, const T *x, T *y, T *ebuf,
                     hipStream_t s) {
  if (V.p < 1 || V.p > kMaxP) return -1;
  const long nc = (long)V.nx * V.ny * V.nz;
  switch (V.p) {
    case 1: apply_vec_p<1, T>(V, coef, B, D, x, y, ebuf, nc, s); break;
    case 2: apply_vec_p<2, T>(V, coef, B, D, x, y, ebuf, nc, s); break;
    case 3: apply_vec_p<3, T>(V, coef, B, D, x, y, ebuf, nc, s); break;
    case 4: apply_vec_p<4, T>(V, coef, B, D, x, y, ebuf, nc, s); break;
    case 5: apply_vec_p<5, T>(V, coef, B, D, x, y, ebuf, nc, s); break;
    case 6: apply_vec_p<6, T>(V, coef, B, D, x, y, ebuf, nc, s); break;
    case 7: apply_vec_p<7, T>(V, coef, B, D, x, y, ebuf, nc, s); break;
    case 8: apply_vec_p<8, T>(V, coef, B, D, x, y, ebuf, nc, s); break;
    default: apply_vec_p<9, T>(V, coef, B, D, x, y, ebuf, nc, s); break;
  }
  const long n = V.off[3];
  k_apply_vec_gather<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(V, x, ebuf, y, n);
  return 0;
}

template int launch_apply_vec<double>(const VecDev &, const double *, const double *, const double *,
                                      const double *, double *, double *, hipStream_t);
template int launch_apply_vec<float>(const VecDev &, const float *, const float *, const float *, const float *,
                                     float *, float *, hipStream_t);

}  // namespace rz
