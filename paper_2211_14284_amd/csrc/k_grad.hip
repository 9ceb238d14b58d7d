// HIP kernels (gfx950) of the H(grad) hot path: sum-factorised operator apply,
// statically condensed vertex-star Schwarz relaxation (condense / patch solve /
// expand), incomplete Cholesky of the patch Schur complements, p-transfer.
//
// Data layout in HBM:
//   * vectors: one value per Q_p lattice point, x fastest (coalesced along x);
//   * per-cell separable weights: 6 values per cell (sigma_1..3, mu_1..3), cells
//     x fastest;
//   * patch factors: one contiguous block of nnz values per vertex slot (vertex
//     lattice order), lower CSR of the symbolic pattern shared by every slot;
//   * patch solution buffer: nrows values per vertex slot in patch order.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "lattice.hpp"

namespace rz {

namespace {

__device__ __forceinline__ bool lat_dirichlet(const LatDev &L, int X, int Y, int Z) {
  return ((L.dir & 1u) && X == 0) || ((L.dir & 2u) && X == L.Nx - 1) ||
         ((L.dir & 4u) && Y == 0) || ((L.dir & 8u) && Y == L.Ny - 1) ||
         ((L.dir & 16u) && Z == 0) || ((L.dir & 32u) && Z == L.Nz - 1);
}

__device__ __forceinline__ long lat_index(const LatDev &L, int X, int Y, int Z) {
  return (long)X + (long)L.Nx * ((long)Y + (long)L.Ny * (long)Z);
}

__device__ __forceinline__ int ncells_axis(const LatDev &L, int a) {
  return a == 0 ? L.nx : (a == 1 ? L.ny : L.nz);
}

// 1-D FDM mass (diagonal + (0,p)) applied along one axis of a tile.
template <typename T>
__device__ __forceinline__ T mass1d(const T *B, int p, int m, const T *f, int stride) {
  const int n1 = p + 1;
  T v = B[m * n1 + m] * f[m * stride];
  if (m == 0) v += B[p] * f[p * stride];
  else if (m == p) v += B[p * n1] * f[0];
  return v;
}

// 1-D FDM stiffness (diagonal + rows/columns 0, p) applied along one axis.
template <typename T>
__device__ __forceinline__ T stiff1d(const T *A, int p, int m, const T *f, int stride) {
  const int n1 = p + 1;
  if (m != 0 && m != p)
    return A[m * n1 + m] * f[m * stride] + A[m * n1] * f[0] + A[m * n1 + p] * f[p * stride];
  T v = 0;
  for (int i = 0; i <= p; ++i) v += A[m * n1 + i] * f[i * stride];
  return v;
}

template <typename T>
__device__ __forceinline__ void atomic_add(T *addr, T v) {
  atomicAdd(addr, v);
}

// ------------------------------------------------------------------------------------
// y = A x: per cell, y_K = s1 (A x B x B) + s2 (B x A x B) + s3 (B x B x A) + mu (B x B x B)
// applied as per-axis contractions of the (p+1)^3 tile staged in LDS (eq.
// sum-factorization with the exact 1-D integrals of an axis-aligned cell).
// Interface contributions are summed with atomics; cell-interior rows are owned.
// ------------------------------------------------------------------------------------
template <typename T>
__global__ void k_apply_grad(LatDev L, const T *__restrict__ coef, const T *__restrict__ Bg,
                             const T *__restrict__ Ag, const T *__restrict__ x, T *__restrict__ y) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *sm = reinterpret_cast<T *>(smem_raw);
  const int p = L.p, n1 = p + 1, n2 = n1 * n1, n3 = n2 * n1;
  T *sB = sm, *sA = sB + n2, *xs = sA + n2, *t1 = xs + n3, *v = t1 + n3, *u = v + n3, *w = u + n3;
  const int cell = blockIdx.x;
  const int cx = cell % L.nx, cy = (cell / L.nx) % L.ny, cz = cell / (L.nx * L.ny);
  for (int k = threadIdx.x; k < n2; k += blockDim.x) {
    sB[k] = Bg[k];
    sA[k] = Ag[k];
  }
  const T s1 = coef[6 * cell + 0], s2 = coef[6 * cell + 1], s3 = coef[6 * cell + 2];
  const T mu = coef[6 * cell + 3];
  for (int k = threadIdx.x; k < n3; k += blockDim.x) {
    int a = k % n1, b = (k / n1) % n1, c = k / n2;
    int X = cx * p + a, Y = cy * p + b, Z = cz * p + c;
    xs[k] = lat_dirichlet(L, X, Y, Z) ? T(0) : x[lat_index(L, X, Y, Z)];
  }
  __syncthreads();
  for (int k = threadIdx.x; k < n3; k += blockDim.x) {  // along z
    int ab = k % n2, c = k / n2;
    t1[k] = mass1d(sB, p, c, xs + ab, n2);
    v[k] = stiff1d(sA, p, c, xs + ab, n2);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < n3; k += blockDim.x) {  // along y
    int a = k % n1, b = (k / n1) % n1, c = k / n2;
    int base = a + n2 * c;
    T uu = mass1d(sB, p, b, t1 + base, n1);
    u[k] = uu;
    w[k] = mu * uu + s2 * stiff1d(sA, p, b, t1 + base, n1) + s3 * mass1d(sB, p, b, v + base, n1);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < n3; k += blockDim.x) {  // along x, scatter
    int a = k % n1, b = (k / n1) % n1, c = k / n2;
    int base = n1 * (b + n1 * c);
    T val = s1 * stiff1d(sA, p, a, u + base, 1) + mass1d(sB, p, a, w + base, 1);
    int X = cx * p + a, Y = cy * p + b, Z = cz * p + c;
    if (lat_dirichlet(L, X, Y, Z)) continue;
    long g = lat_index(L, X, Y, Z);
    bool own = (a != 0 && a != p && b != 0 && b != p && c != 0 && c != p);
    if (own) y[g] = val;
    else atomic_add(y + g, val);
  }
}

template <typename T>
__global__ void k_apply_init(LatDev L, const T *__restrict__ x, T *__restrict__ y, long n) {
  long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  int X = g % L.Nx, Y = (g / L.Nx) % L.Ny, Z = g / ((long)L.Nx * L.Ny);
  y[g] = lat_dirichlet(L, X, Y, Z) ? x[g] : T(0);
}

// ------------------------------------------------------------------------------------
// Relaxation step 1 (eq. schur, R_Gamma r): rt_G = r_G - P_GI P_II^{-1} r_I.  Only
// face DoFs (exactly one lattice coordinate on a vertex plane) couple to cell
// interiors: along their normal line in each of the two cells.
// ------------------------------------------------------------------------------------
template <typename T>
__global__ void k_condense_grad(LatDev L, const T *__restrict__ coef, const T *__restrict__ Ag,
                                const T *__restrict__ lam, const T *__restrict__ r, T *__restrict__ rt,
                                long n) {
  long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const int p = L.p, n1 = p + 1;
  int C[3] = {(int)(g % L.Nx), (int)((g / L.Nx) % L.Ny), (int)(g / ((long)L.Nx * L.Ny))};
  int onv[3] = {C[0] % p == 0, C[1] % p == 0, C[2] % p == 0};
  int nb = onv[0] + onv[1] + onv[2];
  if (nb == 0) return;
  if (lat_dirichlet(L, C[0], C[1], C[2])) {
    rt[g] = T(0);
    return;
  }
  T val = r[g];
  if (nb == 1 && p >= 2) {
    int a = onv[0] ? 0 : (onv[1] ? 1 : 2);
    long stride = a == 0 ? 1 : (a == 1 ? (long)L.Nx : (long)L.Nx * L.Ny);
    for (int side = 0; side < 2; ++side) {
      int cell[3];
      for (int d = 0; d < 3; ++d) cell[d] = C[d] / p;
      cell[a] = C[a] / p - 1 + side;
      if (cell[a] < 0 || cell[a] >= ncells_axis(L, a)) continue;
      int e = side == 0 ? p : 0;
      int cid = cell[0] + L.nx * (cell[1] + L.ny * cell[2]);
      T s[3] = {coef[6 * cid], coef[6 * cid + 1], coef[6 * cid + 2]};
      T mu = coef[6 * cid + 3];
      int loc[3];
      for (int d = 0; d < 3; ++d) loc[d] = C[d] - cell[d] * p;
      T part = 0;
      T base = mu;
      for (int d = 0; d < 3; ++d)
        if (d != a) base += s[d] * lam[loc[d]];
      long g0 = g - (long)loc[a] * stride;  // lattice index of local coordinate 0 on axis a
      for (int i = 1; i < p; ++i) {
        T dd = base + s[a] * lam[i];
        part += Ag[e * n1 + i] * r[g0 + i * stride] / dd;
      }
      val -= s[a] * part;
    }
  }
  rt[g] = val;
}

// ------------------------------------------------------------------------------------
// Relaxation step 2 (eq. sc-asm-afw): one workgroup per vertex slot; the IC factor
// of the slot is staged in LDS, forward and backward substitution by level sets.
// ------------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_patch_solve(LatDev L, PatchDev P, const T *__restrict__ factor,
                                                      const T *__restrict__ rt, T *__restrict__ zbuf) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *Ls = reinterpret_cast<T *>(smem_raw);
  T *xs = Ls + P.nnz;
  const int p = L.p;
  const long vid = blockIdx.x;
  const int nvx = L.nx + 1, nvy = L.ny + 1;
  const int vx = vid % nvx, vy = (vid / nvx) % nvy, vz = vid / ((long)nvx * nvy);
  const T *f = factor + vid * (long)P.nnz;
  for (int k = threadIdx.x; k < P.nnz; k += blockDim.x) Ls[k] = f[k];
  for (int k = threadIdx.x; k < P.nrows; k += blockDim.x) {
    int X = vx * p + P.off[3 * k], Y = vy * p + P.off[3 * k + 1], Z = vz * p + P.off[3 * k + 2];
    bool in = X >= 0 && X < L.Nx && Y >= 0 && Y < L.Ny && Z >= 0 && Z < L.Nz;
    xs[k] = (in && !lat_dirichlet(L, X, Y, Z)) ? rt[lat_index(L, X, Y, Z)] : T(0);
  }
  __syncthreads();
  for (int lv = 0; lv < P.nflev; ++lv) {
    const int b = P.flev_ptr[lv], e = P.flev_ptr[lv + 1];
    for (int t = b + threadIdx.x; t < e; t += blockDim.x) {
      int i = P.flev_rows[t];
      int rs = P.rowptr[i], re = P.rowptr[i + 1] - 1;
      T s = xs[i];
      for (int k = rs; k < re; ++k) s -= Ls[k] * xs[P.col[k]];
      xs[i] = s / Ls[re];
    }
    __syncthreads();
  }
  for (int lv = 0; lv < P.nblev; ++lv) {
    const int b = P.blev_ptr[lv], e = P.blev_ptr[lv + 1];
    for (int t = b + threadIdx.x; t < e; t += blockDim.x) {
      int i = P.blev_rows[t];
      T s = xs[i];
      for (int k = P.uptr[i]; k < P.uptr[i + 1]; ++k) s -= Ls[P.upos[k]] * xs[P.urow[k]];
      xs[i] = s / Ls[P.rowptr[i + 1] - 1];
    }
    __syncthreads();
  }
  T *zo = zbuf + vid * (long)P.nrows;
  for (int k = threadIdx.x; k < P.nrows; k += blockDim.x) zo[k] = xs[k];
}

// ------------------------------------------------------------------------------------
// Relaxation step 3: z_G = sum over the vertex patches containing the DoF (ascending
// vertex id) of the patch solutions; Dirichlet rows copy r.
// Step 4 (harmonic extension, R_Gamma^T): z_I = P_II^{-1} (r_I - P_IG z_G).
// ------------------------------------------------------------------------------------
template <typename T>
__global__ void k_expand_iface(LatDev L, int nrows, const T *__restrict__ r, const T *__restrict__ zbuf,
                               T *__restrict__ z, long n) {
  long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const int p = L.p;
  int C[3] = {(int)(g % L.Nx), (int)((g / L.Nx) % L.Ny), (int)(g / ((long)L.Nx * L.Ny))};
  int lo[3], hi[3], nb = 0;
  for (int d = 0; d < 3; ++d) {
    if (C[d] % p == 0) {
      lo[d] = hi[d] = C[d] / p;
      ++nb;
    } else {
      lo[d] = C[d] / p;
      hi[d] = lo[d] + 1;
    }
  }
  if (nb == 0) return;
  if (lat_dirichlet(L, C[0], C[1], C[2])) {
    z[g] = r[g];
    return;
  }
  const int nvx = L.nx + 1, nvy = L.ny + 1;
  T acc = 0;
  for (int vz = lo[2]; vz <= hi[2]; ++vz)
    for (int vy = lo[1]; vy <= hi[1]; ++vy)
      for (int vx = lo[0]; vx <= hi[0]; ++vx) {
        int k = patch_local_index(p, C[0] - vx * p, C[1] - vy * p, C[2] - vz * p);
        long vid = vx + (long)nvx * (vy + (long)nvy * vz);
        acc += zbuf[vid * nrows + k];
      }
  z[g] = acc;
}

template <typename T>
__global__ void k_expand_interior(LatDev L, const T *__restrict__ coef, const T *__restrict__ Ag,
                                  const T *__restrict__ lam, const T *__restrict__ r, T *__restrict__ z,
                                  long n) {
  long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const int p = L.p, n1 = p + 1;
  int C[3] = {(int)(g % L.Nx), (int)((g / L.Nx) % L.Ny), (int)(g / ((long)L.Nx * L.Ny))};
  if (C[0] % p == 0 || C[1] % p == 0 || C[2] % p == 0) return;
  int cell[3], loc[3];
  for (int d = 0; d < 3; ++d) {
    cell[d] = C[d] / p;
    loc[d] = C[d] - cell[d] * p;
  }
  int cid = cell[0] + L.nx * (cell[1] + L.ny * cell[2]);
  T s[3] = {coef[6 * cid], coef[6 * cid + 1], coef[6 * cid + 2]};
  T dd = coef[6 * cid + 3];
  T val = r[g];
  for (int a = 0; a < 3; ++a) {
    dd += s[a] * lam[loc[a]];
    for (int side = 0; side < 2; ++side) {
      int e = side ? p : 0;
      int F[3] = {C[0], C[1], C[2]};
      F[a] = cell[a] * p + e;
      T zf = lat_dirichlet(L, F[0], F[1], F[2]) ? T(0) : z[lat_index(L, F[0], F[1], F[2])];
      val -= s[a] * Ag[loc[a] * n1 + e] * zf;
    }
  }
  z[g] = val / dd;
}

// ------------------------------------------------------------------------------------
// Setup: S_v on the symbolic pattern from the per-cell separable weights, then
// incomplete Cholesky restricted to the pattern (Sec. 4.5), rows processed by
// level sets (a row only depends on rows of earlier levels).  Slots whose rows
// fall outside the domain or on Dirichlet faces get identity rows.
// ------------------------------------------------------------------------------------
__device__ double cell_schur_value(int p, const double *B, const double *A, const double *lam,
                                   const double s[3], double mu, const int u[3], const int w[3]) {
  const int n1 = p + 1;
  double Bv[3], Av[3];
  for (int d = 0; d < 3; ++d) {
    Bv[d] = B[u[d] * n1 + w[d]];
    Av[d] = A[u[d] * n1 + w[d]];
  }
  double v = s[0] * Av[0] * Bv[1] * Bv[2] + s[1] * Bv[0] * Av[1] * Bv[2] + s[2] * Bv[0] * Bv[1] * Av[2] +
             mu * Bv[0] * Bv[1] * Bv[2];
  if (p < 2) return v;
  int nu = on_end(p, u[0]) + on_end(p, u[1]) + on_end(p, u[2]);
  int nw = on_end(p, w[0]) + on_end(p, w[1]) + on_end(p, w[2]);
  if (nu != 1 || nw != 1) return v;
  int du = on_end(p, u[0]) ? 0 : (on_end(p, u[1]) ? 1 : 2);
  int dw = on_end(p, w[0]) ? 0 : (on_end(p, w[1]) ? 1 : 2);
  if (du == dw) {
    for (int e = 0; e < 3; ++e)
      if (e != du && u[e] != w[e]) return v;
    double base = mu;
    for (int e = 0; e < 3; ++e)
      if (e != du) base += s[e] * lam[u[e]];
    double acc = 0.0;
    for (int i = 1; i < p; ++i) acc += A[u[du] * n1 + i] * A[i * n1 + w[du]] / (base + s[du] * lam[i]);
    return v - s[du] * s[du] * acc;
  }
  int e = 3 - du - dw;
  if (u[e] != w[e]) return v;
  int t[3];
  t[du] = w[du];
  t[dw] = u[dw];
  t[e] = u[e];
  double dd = mu + s[0] * lam[t[0]] + s[1] * lam[t[1]] + s[2] * lam[t[2]];
  return v - s[du] * A[u[du] * n1 + t[du]] * s[dw] * A[t[dw] * n1 + w[dw]] / dd;
}

__global__ void __launch_bounds__(256) k_patch_factor(LatDev L, PatchDev P, const int *__restrict__ erow,
                                                       const double *__restrict__ coef,
                                                       const double *__restrict__ Bg, const double *__restrict__ Ag,
                                                       const double *__restrict__ lamg, double *__restrict__ f64,
                                                       float *__restrict__ f32, int *status) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *S = reinterpret_cast<double *>(smem_raw);
  const int p = L.p, n1 = p + 1;
  double *sB = S + P.nnz, *sA = sB + n1 * n1, *sl = sA + n1 * n1;
  unsigned char *allowed = reinterpret_cast<unsigned char *>(sl + n1);
  const long vid = blockIdx.x;
  const int nvx = L.nx + 1, nvy = L.ny + 1;
  const int V[3] = {(int)(vid % nvx), (int)((vid / nvx) % nvy), (int)(vid / ((long)nvx * nvy))};
  for (int k = threadIdx.x; k < n1 * n1; k += blockDim.x) {
    sB[k] = Bg[k];
    sA[k] = Ag[k];
  }
  for (int k = threadIdx.x; k < n1; k += blockDim.x) sl[k] = lamg[k];
  __syncthreads();
  for (int k = threadIdx.x; k < P.nnz; k += blockDim.x) {
    int r = erow[k], c = P.col[k];
    int Gr[3], Gc[3];
    bool pr = true, pc = true;
    for (int d = 0; d < 3; ++d) {
      Gr[d] = V[d] * p + P.off[3 * r + d];
      Gc[d] = V[d] * p + P.off[3 * c + d];
    }
    const int Nd[3] = {L.Nx, L.Ny, L.Nz};
    for (int d = 0; d < 3; ++d) {
      pr = pr && Gr[d] >= 0 && Gr[d] < Nd[d];
      pc = pc && Gc[d] >= 0 && Gc[d] < Nd[d];
    }
    pr = pr && !lat_dirichlet(L, Gr[0], Gr[1], Gr[2]);
    pc = pc && !lat_dirichlet(L, Gc[0], Gc[1], Gc[2]);
    double val = 0.0;
    bool ok = false;
    if (!pr || !pc) {
      val = (r == c) ? 1.0 : 0.0;
      ok = (r == c);
    } else {
      for (int cell = 0; cell < 8; ++cell) {
        int cc[3], u[3], w[3];
        bool in = true;
        for (int d = 0; d < 3; ++d) {
          cc[d] = V[d] - 1 + ((cell >> d) & 1);
          u[d] = Gr[d] - cc[d] * p;
          w[d] = Gc[d] - cc[d] * p;
          in = in && cc[d] >= 0 && cc[d] < ncells_axis(L, d) && u[d] >= 0 && u[d] <= p && w[d] >= 0 &&
               w[d] <= p;
        }
        if (!in) continue;
        if (!cell_schur_coupled(p, u, w)) continue;
        ok = true;
        int cid = cc[0] + L.nx * (cc[1] + L.ny * cc[2]);
        double s[3] = {coef[6 * cid], coef[6 * cid + 1], coef[6 * cid + 2]};
        val += cell_schur_value(p, sB, sA, sl, s, coef[6 * cid + 3], u, w);
      }
    }
    S[k] = ok ? val : 0.0;
    allowed[k] = ok ? 1 : 0;
  }
  __syncthreads();
  for (int lv = 0; lv < P.nflev; ++lv) {
    const int b = P.flev_ptr[lv], e = P.flev_ptr[lv + 1];
    for (int t = b + threadIdx.x; t < e; t += blockDim.x) {
      int i = P.flev_rows[t];
      int rs = P.rowptr[i], re = P.rowptr[i + 1] - 1;
      for (int k = rs; k < re; ++k) {
        if (!allowed[k]) {
          S[k] = 0.0;
          continue;
        }
        int j = P.col[k];
        double s = S[k];
        int pi = rs, pj = P.rowptr[j], pje = P.rowptr[j + 1] - 1;
        while (pi < k && pj < pje) {
          int ci = P.col[pi], cj = P.col[pj];
          if (ci == cj) {
            s -= S[pi] * S[pj];
            ++pi;
            ++pj;
          } else if (ci < cj) {
            ++pi;
          } else {
            ++pj;
          }
        }
        S[k] = s / S[pje];
      }
      double d = S[re];
      for (int k = rs; k < re; ++k) d -= S[k] * S[k];
      if (!(d > 0.0)) {
        atomicCAS(status, 0, (int)vid + 1);
        d = 1.0;
      }
      S[re] = sqrt(d);
    }
    __syncthreads();
  }
  double *o64 = f64 + vid * (long)P.nnz;
  float *o32 = f32 + vid * (long)P.nnz;
  for (int k = threadIdx.x; k < P.nnz; k += blockDim.x) {
    o64[k] = S[k];
    o32[k] = (float)S[k];
  }
}

// ------------------------------------------------------------------------------------
// p-transfer: the embedding of Q_1 in Q_p in FDM coefficients is the Kronecker
// product of the (p+1)x2 hat matrix E per axis; restriction is its transpose.
// ------------------------------------------------------------------------------------
__global__ void k_prolong_add_grad(LatDev L, const double *__restrict__ E, const double *__restrict__ xc,
                                   double *__restrict__ xf, long n) {
  long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const int p = L.p;
  int C[3] = {(int)(g % L.Nx), (int)((g / L.Nx) % L.Ny), (int)(g / ((long)L.Nx * L.Ny))};
  if (lat_dirichlet(L, C[0], C[1], C[2])) return;
  const int NC[3] = {L.nx + 1, L.ny + 1, L.nz + 1};
  int c0[3];
  double w[3][2];
  for (int d = 0; d < 3; ++d) {
    int c = C[d] / p;
    if (c >= NC[d] - 1) c = NC[d] - 2;
    int a = C[d] - c * p;
    c0[d] = c;
    w[d][0] = E[2 * a];
    w[d][1] = E[2 * a + 1];
  }
  double acc = 0.0;
  for (int k = 0; k < 8; ++k) {
    int kx = k & 1, ky = (k >> 1) & 1, kz = k >> 2;
    double wt = w[0][kx] * w[1][ky] * w[2][kz];
    if (wt == 0.0) continue;
    int X = c0[0] + kx, Y = c0[1] + ky, Z = c0[2] + kz;
    bool dir = ((L.dir & 1u) && X == 0) || ((L.dir & 2u) && X == NC[0] - 1) || ((L.dir & 4u) && Y == 0) ||
               ((L.dir & 8u) && Y == NC[1] - 1) || ((L.dir & 16u) && Z == 0) || ((L.dir & 32u) && Z == NC[2] - 1);
    if (dir) continue;
    acc += wt * xc[X + (long)NC[0] * (Y + (long)NC[1] * Z)];
  }
  xf[g] += acc;
}

__global__ void __launch_bounds__(256) k_restrict_grad(LatDev L, const double *__restrict__ E,
                                                        const double *__restrict__ rf, double *__restrict__ rc) {
  __shared__ double red[256];
  const int p = L.p;
  const int NC[3] = {L.nx + 1, L.ny + 1, L.nz + 1};
  const long V = blockIdx.x;
  const int VC[3] = {(int)(V % NC[0]), (int)((V / NC[0]) % NC[1]), (int)(V / ((long)NC[0] * NC[1]))};
  bool dir = ((L.dir & 1u) && VC[0] == 0) || ((L.dir & 2u) && VC[0] == NC[0] - 1) ||
             ((L.dir & 4u) && VC[1] == 0) || ((L.dir & 8u) && VC[1] == NC[1] - 1) ||
             ((L.dir & 16u) && VC[2] == 0) || ((L.dir & 32u) && VC[2] == NC[2] - 1);
  if (dir) {
    if (threadIdx.x == 0) rc[V] = 0.0;
    return;
  }
  const int Nd[3] = {L.Nx, L.Ny, L.Nz};
  int lo[3], ext[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = VC[d] * p - (p - 1);
    int hi = VC[d] * p + (p - 1);
    if (lo[d] < 0) lo[d] = 0;
    if (hi > Nd[d] - 1) hi = Nd[d] - 1;
    ext[d] = hi - lo[d] + 1;
  }
  const int tot = ext[0] * ext[1] * ext[2];
  double acc = 0.0;
  for (int k = threadIdx.x; k < tot; k += blockDim.x) {
    int G[3] = {lo[0] + k % ext[0], lo[1] + (k / ext[0]) % ext[1], lo[2] + k / (ext[0] * ext[1])};
    if (lat_dirichlet(L, G[0], G[1], G[2])) continue;
    double wt = 1.0;
    for (int d = 0; d < 3; ++d) {
      int off = G[d] - VC[d] * p;
      if (off < 0) wt *= E[2 * (off + p) + 1];
      else if (off > 0) wt *= E[2 * off];
    }
    acc += wt * rf[G[0] + (long)L.Nx * (G[1] + (long)L.Ny * G[2])];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) rc[V] = red[0];
}

__global__ void k_dirichlet_copy(LatDev L, const double *__restrict__ r, double *__restrict__ z, long n) {
  long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  int X = g % L.Nx, Y = (g / L.Nx) % L.Ny, Z = g / ((long)L.Nx * L.Ny);
  if (lat_dirichlet(L, X, Y, Z)) z[g] = r ? r[g] : 0.0;
}

inline unsigned nblocks(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------
template <typename T>
void launch_apply_grad(const LatDev &L, const T *coef, const T *B, const T *A, const T *x, T *y,
                       hipStream_t s) {
  long n = (long)L.Nx * L.Ny * L.Nz;
  k_apply_init<T><<<nblocks(n, 256), 256, 0, s>>>(L, x, y, n);
  const int n1 = L.p + 1, n3 = n1 * n1 * n1;
  int bs = n3 >= 256 ? 256 : (n3 >= 128 ? 128 : 64);
  size_t shm = sizeof(T) * (2 * n1 * n1 + 5 * n3);
  k_apply_grad<T><<<L.nx * L.ny * L.nz, bs, shm, s>>>(L, coef, B, A, x, y);
}

template <typename T>
void launch_condense_grad(const LatDev &L, const T *coef, const T *A, const T *lam, const T *r, T *rt,
                          hipStream_t s) {
  long n = (long)L.Nx * L.Ny * L.Nz;
  k_condense_grad<T><<<nblocks(n, 256), 256, 0, s>>>(L, coef, A, lam, r, rt, n);
}

template <typename T>
void launch_patch_solve(const LatDev &L, const PatchDev &P, const T *factor, const T *rt, T *zbuf,
                        hipStream_t s) {
  long nv = (long)(L.nx + 1) * (L.ny + 1) * (L.nz + 1);
  size_t shm = sizeof(T) * (P.nnz + P.nrows);
  if (shm > 65536) hipFuncSetAttribute((const void *)k_patch_solve<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  k_patch_solve<T><<<(unsigned)nv, 256, shm, s>>>(L, P, factor, rt, zbuf);
}

template <typename T>
void launch_expand_grad(const LatDev &L, const PatchDev &P, const T *coef, const T *A, const T *lam,
                        const T *r, const T *zbuf, T *z, hipStream_t s) {
  long n = (long)L.Nx * L.Ny * L.Nz;
  k_expand_iface<T><<<nblocks(n, 256), 256, 0, s>>>(L, P.nrows, r, zbuf, z, n);
  k_expand_interior<T><<<nblocks(n, 256), 256, 0, s>>>(L, coef, A, lam, r, z, n);
}

void launch_patch_factor(const LatDev &L, const PatchDev &P, const double *coef, const double *B,
                         const double *A, const double *lam, double *f64, float *f32, int *status,
                         hipStream_t s) {
  long nv = (long)(L.nx + 1) * (L.ny + 1) * (L.nz + 1);
  const int n1 = L.p + 1;
  size_t shm = sizeof(double) * (P.nnz + 2 * n1 * n1 + n1) + P.nnz;
  if (shm > 65536) hipFuncSetAttribute((const void *)k_patch_factor, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  k_patch_factor<<<(unsigned)nv, 256, shm, s>>>(L, P, P.erow, coef, B, A, lam, f64, f32, status);
}

void launch_dirichlet_copy(const LatDev &L, const double *r, double *z, hipStream_t s) {
  long n = (long)L.Nx * L.Ny * L.Nz;
  k_dirichlet_copy<<<nblocks(n, 256), 256, 0, s>>>(L, r, z, n);
}

void launch_prolong_add_grad(const LatDev &L, const double *E, const double *xc, double *xf,
                             hipStream_t s) {
  long n = (long)L.Nx * L.Ny * L.Nz;
  k_prolong_add_grad<<<nblocks(n, 256), 256, 0, s>>>(L, E, xc, xf, n);
}

void launch_restrict_grad(const LatDev &L, const double *E, const double *rf, double *rc, hipStream_t s) {
  long nc = (long)(L.nx + 1) * (L.ny + 1) * (L.nz + 1);
  k_restrict_grad<<<(unsigned)nc, 256, 0, s>>>(L, E, rf, rc);
}

template void launch_apply_grad<double>(const LatDev &, const double *, const double *, const double *,
                                        const double *, double *, hipStream_t);
template void launch_apply_grad<float>(const LatDev &, const float *, const float *, const float *,
                                       const float *, float *, hipStream_t);
template void launch_condense_grad<double>(const LatDev &, const double *, const double *, const double *,
                                           const double *, double *, hipStream_t);
template void launch_condense_grad<float>(const LatDev &, const float *, const float *, const float *,
                                          const float *, float *, hipStream_t);
template void launch_patch_solve<double>(const LatDev &, const PatchDev &, const double *, const double *,
                                         double *, hipStream_t);
template void launch_patch_solve<float>(const LatDev &, const PatchDev &, const float *, const float *,
                                        float *, hipStream_t);
template void launch_expand_grad<double>(const LatDev &, const PatchDev &, const double *, const double *,
                                         const double *, const double *, const double *, double *,
                                         hipStream_t);
template void launch_expand_grad<float>(const LatDev &, const PatchDev &, const float *, const float *,
                                        const float *, const float *, const float *, float *, hipStream_t);

}  // namespace rz
