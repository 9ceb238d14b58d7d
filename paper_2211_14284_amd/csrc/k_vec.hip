// HIP kernels (gfx950) of the operator apply in H(curl) (NCE_p) and H(div) (NCF_p)
// on axis-aligned cells with cellwise-constant coefficients (eq. sum-factorization
// with the exact 1-D integrals; Sec. 2.4 bases, eqs. curlbasis / divbasis):
//   curl: y_K = sum_m mu_m ME_m u_m + sum_n sigma_n C_n^T MF_n C_n u,
//         ME_m = I along m, B along the other axes;  MF_n = B along n, I elsewhere;
//         (C u)_0 = D_y u_2 - D_z u_1, (C u)_1 = D_z u_0 - D_x u_2, (C u)_2 = D_x u_1 - D_y u_0;
//   div:  y_K = sum_m mu_m MF_m u_m + sigma D_m^T (sum_n D_n u_n).
// In the FDM bases every 1-D factor is sparse (B: diagonal plus (0,p); D: at most
// three entries per row), so each line costs O(p).  One block per cell; tiles of
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

struct Tile {
  int e[3];  // local extents (x, y, z)
  __device__ int size() const { return e[0] * e[1] * e[2]; }
};

__device__ __forceinline__ Tile comp_tile(int space, int m, int p) {
  Tile t;
  for (int a = 0; a < 3; ++a) t.e[a] = is_P(space, m, a) ? p + 1 : p;
  return t;
}

enum { OP_B = 0, OP_D = 1, OP_DT = 2 };

// out (+)= scale * op along axis `ax` of in; in/out tiles differ only along ax.
// B: (p+1) -> (p+1); D: (p+1) -> p; D^T: p -> (p+1).  Tables in LDS.
template <typename T>
__device__ void line_op(const T *in, Tile ti, T *out, Tile to, int ax, int op, const T *sB, const T *sD, int p,
                        T scale, bool acc) {
  const int b = ax == 0 ? 1 : 0, c = ax == 2 ? 1 : 2;
  const int nl = ti.e[b] * ti.e[c];
  const int sti = ax == 0 ? 1 : (ax == 1 ? ti.e[0] : ti.e[0] * ti.e[1]);
  const int sto = ax == 0 ? 1 : (ax == 1 ? to.e[0] : to.e[0] * to.e[1]);
  const int n1 = p + 1;
  for (int l = threadIdx.x; l < nl; l += blockDim.x) {
    const int u = l % ti.e[b], w = l / ti.e[b];
    int ci[3], co[3];
    ci[ax] = co[ax] = 0;
    ci[b] = co[b] = u;
    ci[c] = co[c] = w;
    const int bi = ci[0] + ti.e[0] * (ci[1] + ti.e[1] * ci[2]);
    const int bo = co[0] + to.e[0] * (co[1] + to.e[1] * co[2]);
    T v[kMaxP + 1], r[kMaxP + 1];
    for (int i = 0; i < ti.e[ax]; ++i) v[i] = in[bi + i * sti];
    if (op == OP_B) {
      for (int i = 0; i <= p; ++i) r[i] = sB[i * n1 + i] * v[i];
      r[0] += sB[p] * v[p];
      r[p] += sB[p * n1] * v[0];
    } else if (op == OP_D) {  // r_i = sum_j D[i][j] v_j, D row i: columns 0, p and i (i >= 1)
      for (int i = 0; i < p; ++i) {
        T s = sD[i * n1] * v[0] + sD[i * n1 + p] * v[p];
        if (i >= 1) s += sD[i * n1 + i] * v[i];
        r[i] = s;
      }
    } else {  // r_j = sum_i D[i][j] v_i
      T r0 = 0, rp = 0;
      for (int i = 0; i < p; ++i) {
        r0 += sD[i * n1] * v[i];
        rp += sD[i * n1 + p] * v[i];
      }
      for (int j = 1; j < p; ++j) r[j] = sD[j * n1 + j] * v[j];
      r[0] = r0;
      r[p] = rp;
    }
    for (int i = 0; i < to.e[ax]; ++i) {
      const T val = scale * r[i];
      out[bo + i * sto] = acc ? out[bo + i * sto] + val : val;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_apply_vec(VecDev V, const T *__restrict__ coef, const T *__restrict__ Bg,
                                                    const T *__restrict__ Dg, const T *__restrict__ x,
                                                    T *__restrict__ y, T *__restrict__ ebuf) {
  constexpr int TS = (kMaxP + 1) * (kMaxP + 1) * (kMaxP + 1);
  __shared__ T U[3][TS], Y[3][TS], F[TS], G[TS];
  __shared__ T sB[(kMaxP + 1) * (kMaxP + 1)], sD[kMaxP * (kMaxP + 1)];
  const int p = V.p, n1 = p + 1, space = V.space;
  const long cell = blockIdx.x;
  const int cc[3] = {(int)(cell % V.nx), (int)((cell / V.nx) % V.ny), (int)(cell / ((long)V.nx * V.ny))};
  for (int k = threadIdx.x; k < n1 * n1; k += blockDim.x) sB[k] = Bg[k];
  for (int k = threadIdx.x; k < p * n1; k += blockDim.x) sD[k] = Dg[k];
  Tile tc[3];
  for (int m = 0; m < 3; ++m) tc[m] = comp_tile(space, m, p);
  for (int m = 0; m < 3; ++m)
    for (int k = threadIdx.x; k < tc[m].size(); k += blockDim.x) {
      const int l[3] = {k % tc[m].e[0], (k / tc[m].e[0]) % tc[m].e[1], k / (tc[m].e[0] * tc[m].e[1])};
      const int C[3] = {cc[0] * p + l[0], cc[1] * p + l[1], cc[2] * p + l[2]};
      U[m][k] = comp_dirichlet(V, m, C) ? T(0) : x[comp_index(V, m, C)];
    }
  __syncthreads();
  const T *cf = coef + 6 * cell;
  if (space == 1) {
    // mass: Y_m = mu_m B_b B_c U_m (b, c: the continuous axes of component m)
    for (int m = 0; m < 3; ++m) {
      const int b = m == 0 ? 1 : 0, c = m == 2 ? 1 : 2;
      line_op(U[m], tc[m], F, tc[m], b, OP_B, sB, sD, p, T(1), false);
      __syncthreads();
      line_op(F, tc[m], Y[m], tc[m], c, OP_B, sB, sD, p, cf[3 + m], false);
      __syncthreads();
    }
    // curl: F_n (P along n, DP elsewhere), G_n = sigma_n B_n F_n, then C_n^T G_n
    for (int n = 0; n < 3; ++n) {
      const int a1 = (n + 1) % 3, a2 = (n + 2) % 3;  // F_n = D_{a1} U_{a2} - D_{a2} U_{a1}
      Tile tf;
      for (int a = 0; a < 3; ++a) tf.e[a] = a == n ? p + 1 : p;
      line_op(U[a2], tc[a2], F, tf, a1, OP_D, sB, sD, p, T(1), false);
      __syncthreads();
      line_op(U[a1], tc[a1], F, tf, a2, OP_D, sB, sD, p, T(-1), true);
      __syncthreads();
      line_op(F, tf, G, tf, n, OP_B, sB, sD, p, cf[n], false);
      __syncthreads();
      line_op(G, tf, Y[a2], tc[a2], a1, OP_DT, sB, sD, p, T(1), true);
      __syncthreads();
      line_op(G, tf, Y[a1], tc[a1], a2, OP_DT, sB, sD, p, T(-1), true);
      __syncthreads();
    }
  } else {
    // mass: Y_m = mu_m B_m U_m
    for (int m = 0; m < 3; ++m) line_op(U[m], tc[m], Y[m], tc[m], m, OP_B, sB, sD, p, cf[3 + m], false);
    __syncthreads();
    // divergence F = sum_m D_m U_m (DP in all axes), then Y_m += sigma D_m^T F
    Tile tq;
    tq.e[0] = tq.e[1] = tq.e[2] = p;
    for (int m = 0; m < 3; ++m) {
      line_op(U[m], tc[m], F, tq, m, OP_D, sB, sD, p, T(1), m > 0);
      __syncthreads();
    }
    for (int m = 0; m < 3; ++m) line_op(F, tq, Y[m], tc[m], m, OP_DT, sB, sD, p, cf[0], true);
    __syncthreads();
  }
  // store: rows with no continuous axis at an end are owned by the cell
  long eo = cell * (long)V.cell_dofs;
  for (int m = 0; m < 3; ++m) {
    for (int k = threadIdx.x; k < tc[m].size(); k += blockDim.x) {
      const int l[3] = {k % tc[m].e[0], (k / tc[m].e[0]) % tc[m].e[1], k / (tc[m].e[0] * tc[m].e[1])};
      bool owned = true;
      for (int a = 0; a < 3; ++a)
        if (is_P(space, m, a) && (l[a] == 0 || l[a] == p)) owned = false;
      if (owned) {
        const int C[3] = {cc[0] * p + l[0], cc[1] * p + l[1], cc[2] * p + l[2]};
        y[comp_index(V, m, C)] = Y[m][k];
      } else {
        ebuf[eo + k] = Y[m][k];
      }
    }
    eo += tc[m].size();
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

template <typename T>
int launch_apply_vec(const VecDev &V, const T *coef, const T *B, const T *D, const T *x, T *y, T *ebuf,
                     hipStream_t s) {
  if (V.p < 1 || V.p > kMaxP) return -1;
  const long nc = (long)V.nx * V.ny * V.nz;
  k_apply_vec<T><<<(unsigned)nc, 256, 0, s>>>(V, coef, B, D, x, y, ebuf);
  const long n = V.off[3];
  k_apply_vec_gather<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(V, x, ebuf, y, n);
  return 0;
}

template int launch_apply_vec<double>(const VecDev &, const double *, const double *, const double *,
                                      const double *, double *, double *, hipStream_t);
template int launch_apply_vec<float>(const VecDev &, const float *, const float *, const float *, const float *,
                                     float *, float *, hipStream_t);

}  // namespace rz
