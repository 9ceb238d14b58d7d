// HIP kernels (gfx950) of the statically condensed Pavarino-Hiptmair relaxation
// for H(curl) and H(div) (Sec. 4.3-4.5; eq. schur for the cell interiors, eq.
// sc-asm-hiptmair for the interface): per-cell condensation and harmonic extension
// with the exact block factors of P_II, edge-star Cholesky solves, sums back to
// the interface in a fixed order, and the sparse products with the exterior
// derivative and the p-transfer.  Every result is deterministic (no atomics).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace rz {

namespace {

constexpr int kBS = 256;

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBS - 1) / kBS); }

__device__ __forceinline__ bool vr_is_P(int space, int m, int a) { return space == 1 ? a != m : a == m; }

// global index and Dirichlet flag of local DoF l of cell (cx, cy, cz)
template <typename T>
__device__ __forceinline__ long vr_global(const VecDev &V, const VecCellDev<T> &C, const int cc[3], int l,
                                          bool &dir) {
  const int m = C.lcomp[l];
  int X[3];
  dir = false;
  for (int a = 0; a < 3; ++a) {
    X[a] = cc[a] * V.p + C.lcrd[3 * l + a];
    if (vr_is_P(V.space, m, a)) {
      if ((V.dir & (1u << (2 * a))) && X[a] == 0) dir = true;
      if ((V.dir & (1u << (2 * a + 1))) && X[a] == V.ext[m][a] - 1) dir = true;
    }
  }
  return V.off[m] + (long)X[0] + (long)V.ext[m][0] * ((long)X[1] + (long)V.ext[m][1] * (long)X[2]);
}

// u = L^{-T} L^{-1} v on one interior block (3 x 3 lower L^{-1}, zero padded)
template <typename T>
__device__ __forceinline__ void block_solve(const T *Li, const T v[3], T u[3]) {
  T w[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    T s = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) s += Li[3 * r + c] * v[c];
    w[r] = s;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T s = 0;
#pragma unroll
    for (int r = 0; r < 3; ++r) s += Li[3 * r + c] * w[r];
    u[c] = s;
  }
}

// Condensation: z_I = P_II^{-1} r_I (stored), eb[cell] = P_GI z_I per interface row.
template <typename T>
__global__ void __launch_bounds__(kBS) k_vc_condense(VecDev V, VecCellDev<T> C, const T *__restrict__ r,
                                                     T *__restrict__ z, T *__restrict__ eb) {
  extern __shared__ unsigned char vr_smem[];
  T *sr = reinterpret_cast<T *>(vr_smem), *sz = sr + C.nI;
  const long cell = blockIdx.x;
  const int cc[3] = {(int)(cell % V.nx), (int)((cell / V.nx) % V.ny), (int)(cell / ((long)V.nx * V.ny))};
  const int key = C.key[cell];
  for (int t = threadIdx.x; t < C.nI; t += blockDim.x) {
    bool d;
    sr[t] = r[vr_global(V, C, cc, C.il[t], d)];
  }
  __syncthreads();
  const T *Lk = C.linv + (size_t)key * C.nblk * 9;
  for (int b = threadIdx.x; b < C.nblk; b += blockDim.x) {
    const int *rows = C.blk + 3 * b;
    T v[3], u[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = rows[k] >= 0 ? sr[rows[k]] : T(0);
    block_solve(Lk + 9 * b, v, u);
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (rows[k] >= 0) {
        sz[rows[k]] = u[k];
        bool d;
        z[vr_global(V, C, cc, C.il[rows[k]], d)] = u[k];
      }
  }
  __syncthreads();
  const T *gv = C.gi_val + (size_t)key * C.nnz_gi;
  for (int g = threadIdx.x; g < C.nG; g += blockDim.x) {
    T acc = 0;
    for (int k = C.gi_ptr[g]; k < C.gi_ptr[g + 1]; ++k) acc += gv[k] * sz[C.gi_col[k]];
    eb[cell * C.nG + g] = acc;
  }
}

// Harmonic extension: z_I -= P_II^{-1} P_IG z_G (z_G read at the cell's free
// interface DoFs, Dirichlet ones as zero).
template <typename T>
__global__ void __launch_bounds__(kBS) k_vc_expand(VecDev V, VecCellDev<T> C, T *__restrict__ z) {
  extern __shared__ unsigned char vr_smem[];
  T *sg = reinterpret_cast<T *>(vr_smem), *st = sg + C.nG;
  const long cell = blockIdx.x;
  const int cc[3] = {(int)(cell % V.nx), (int)((cell / V.nx) % V.ny), (int)(cell / ((long)V.nx * V.ny))};
  const int key = C.key[cell];
  for (int t = threadIdx.x; t < C.nG; t += blockDim.x) {
    bool d;
    const long g = vr_global(V, C, cc, C.gl[t], d);
    sg[t] = d ? T(0) : z[g];
  }
  __syncthreads();
  const T *iv = C.ig_val + (size_t)key * C.nnz_ig;
  for (int i = threadIdx.x; i < C.nI; i += blockDim.x) {
    T acc = 0;
    for (int k = C.ig_ptr[i]; k < C.ig_ptr[i + 1]; ++k) acc += iv[k] * sg[C.ig_col[k]];
    st[i] = acc;
  }
  __syncthreads();
  const T *Lk = C.linv + (size_t)key * C.nblk * 9;
  for (int b = threadIdx.x; b < C.nblk; b += blockDim.x) {
    const int *rows = C.blk + 3 * b;
    T v[3], u[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = rows[k] >= 0 ? st[rows[k]] : T(0);
    block_solve(Lk + 9 * b, v, u);
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (rows[k] >= 0) {
        bool d;
        const long g = vr_global(V, C, cc, C.il[rows[k]], d);
        z[g] -= u[k];
      }
  }
}

// y[rows[t]] = (x ? x[rows[t]] : 0) + sign * sum of buf over the positions of row t
template <typename T>
__global__ void k_list_gather(int n, const int *__restrict__ rows, const int *__restrict__ ptr,
                              const int *__restrict__ pos, const T *__restrict__ buf, const T *__restrict__ x,
                              T *__restrict__ y, T sign) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int g = rows[t];
  T acc = 0;
  for (int k = ptr[t]; k < ptr[t + 1]; ++k) acc += buf[pos[k]];
  y[g] = (x ? x[g] : T(0)) + sign * acc;
}

// y[rows[t]] = d[t] * x[rows[t]]
template <typename T>
__global__ void k_rows_scale(int n, const int *__restrict__ rows, const T *__restrict__ d, const T *__restrict__ x,
                             T *__restrict__ y) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int g = rows[t];
  y[g] = d[t] * x[g];
}

// y[row(t)] (+)= sum_k val[k] x[col[k]]; row(t) = rows ? rows[t] : t
template <typename TV, typename TX, typename TY>
__global__ void k_csr(int n, const int *__restrict__ rows, const int *__restrict__ ptr, const int *__restrict__ col,
                      const TV *__restrict__ val, const TX *__restrict__ x, TY *__restrict__ y, int add) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int g = rows ? rows[t] : t;
  TV acc = 0;
  for (int k = ptr[t]; k < ptr[t + 1]; ++k) acc += val[k] * (TV)x[col[k]];
  y[g] = add ? (TY)((TV)y[g] + acc) : (TY)acc;
}

// Edge-star patch solves: one wavefront per (patch, mode block); z = W^T (W b) with W
// = L^{-1} of the block's Cholesky factor (the patch type's, computed at setup in
// FP64), packed by columns for W b and by rows for W^T y.  The gathered right-hand
// side and the intermediate y are broadcast from LDS; lane l forms rows l and l + 64
// with coalesced loads, and no row waits for another (unlike two triangular sweeps).
template <typename T>
__global__ void __launch_bounds__(kBS) k_edge_solve(EdgeDev E, const T *__restrict__ fac, const T *__restrict__ rt,
                                                    T *__restrict__ zb) {
  __shared__ T sb[kBS / 64][128];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long w = (long)blockIdx.x * (blockDim.x >> 6) + wv;
  if (w >= (long)E.npatch * E.p) return;
  const int patch = (int)(w / E.p), blk = (int)(w % E.p);
  const int nb = E.blk_n[blk], s0 = E.blk_slot[blk];
  const int *ix = E.idx + (size_t)patch * E.nslot + s0;
  const T *Wc = fac + (size_t)E.type[patch] * E.fac_stride + E.blk_fac[blk];  // by columns
  const T *Wr = Wc + nb * (nb + 1) / 2;                                         // by rows
  const int r0 = lane, r1 = lane + 64;
  const int g0 = r0 < nb ? ix[r0] : -1, g1 = r1 < nb ? ix[r1] : -1;
  T *b = sb[wv];
  b[r0] = g0 >= 0 ? rt[g0] : T(0);
  b[r1] = g1 >= 0 ? rt[g1] : T(0);
  // LDS of this wavefront only: its own writes are visible after the wave-level fence
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // y = W b: y_r = sum_{c <= r} W_rc b_c, column c holds W_{c..n-1, c}
  T y0 = 0, y1 = 0;
  for (int c = 0; c < nb; ++c) {
    const T bc = b[c];
    const T *col = Wc + c * nb - (c * (c - 1)) / 2 - c;  // col[r] = W_rc for r >= c
    if (r0 >= c && r0 < nb) y0 += col[r0] * bc;
    if (r1 >= c && r1 < nb) y1 += col[r1] * bc;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  b[r0] = y0;
  b[r1] = y1;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // z = W^T y: z_r = sum_{c >= r} W_cr y_c, row c holds W_{c, 0..c}
  T z0 = 0, z1 = 0;
  for (int c = 0; c < nb; ++c) {
    const T yc = b[c];
    const T *row = Wr + (c * (c + 1)) / 2;  // row[r] = W_cr for r <= c
    if (r0 <= c) z0 += row[r0] * yc;
    if (r1 <= c) z1 += row[r1] * yc;
  }
  T *zo = zb + (size_t)patch * E.nslot + s0;
  if (r0 < nb) zo[r0] = z0;
  if (r1 < nb) zo[r1] = z1;
}

// y = M x for a dense m x m matrix (row-major), one wavefront per row, FP64 sums
template <typename TM>
__global__ void __launch_bounds__(kBS) k_gemv(int m, const TM *__restrict__ M, const double *__restrict__ x,
                                              double *__restrict__ y) {
  const int lane = threadIdx.x & 63;
  const long row = (long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= m) return;
  const TM *Mr = M + row * (long)m;
  double acc = 0.0;
  for (int c = lane; c < m; c += 64) acc += (double)Mr[c] * x[c];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if (lane == 0) y[row] = acc;
}

// z[list[t]] = r ? r[list[t]] : 0
template <typename T>
__global__ void k_list_copy(int n, const int *__restrict__ list, const T *__restrict__ r, T *__restrict__ z) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int g = list[t];
  z[g] = r ? r[g] : T(0);
}

}  // namespace

template <typename T>
void launch_vc_condense(const VecDev &V, const VecCellDev<T> &C, const T *r, T *z, T *eb, hipStream_t s) {
  const long nc = (long)V.nx * V.ny * V.nz;
  const size_t shm = 2 * (size_t)C.nI * sizeof(T);
  k_vc_condense<T><<<(unsigned)nc, kBS, shm, s>>>(V, C, r, z, eb);
}

template <typename T>
void launch_vc_expand(const VecDev &V, const VecCellDev<T> &C, T *z, hipStream_t s) {
  const long nc = (long)V.nx * V.ny * V.nz;
  const size_t shm = ((size_t)C.nI + C.nG) * sizeof(T);
  k_vc_expand<T><<<(unsigned)nc, kBS, shm, s>>>(V, C, z);
}

template <typename T>
void launch_list_gather(int n, const int *rows, const int *ptr, const int *pos, const T *buf, const T *x, T *y,
                        T sign, hipStream_t s) {
  if (n > 0) k_list_gather<T><<<nblk(n), kBS, 0, s>>>(n, rows, ptr, pos, buf, x, y, sign);
}

template <typename T>
void launch_rows_scale(int n, const int *rows, const T *d, const T *x, T *y, hipStream_t s) {
  if (n > 0) k_rows_scale<T><<<nblk(n), kBS, 0, s>>>(n, rows, d, x, y);
}

template <typename TV, typename TX, typename TY>
void launch_csr(int n, const int *rows, const int *ptr, const int *col, const TV *val, const TX *x, TY *y, int add,
                hipStream_t s) {
  if (n > 0) k_csr<TV, TX, TY><<<nblk(n), kBS, 0, s>>>(n, rows, ptr, col, val, x, y, add);
}

template <typename T>
void launch_edge_solve(const EdgeDev &E, const T *fac, const T *rt, T *zb, hipStream_t s) {
  const long nw = (long)E.npatch * E.p;
  if (nw > 0) k_edge_solve<T><<<(unsigned)((nw + 3) / 4), kBS, 0, s>>>(E, fac, rt, zb);
}

template <typename TM>
void launch_gemv(int m, const TM *M, const double *x, double *y, hipStream_t s) {
  if (m > 0) k_gemv<TM><<<(unsigned)((m + 3) / 4), kBS, 0, s>>>(m, M, x, y);
}

template <typename T>
void launch_list_copy(int n, const int *list, const T *r, T *z, hipStream_t s) {
  if (n > 0) k_list_copy<T><<<nblk(n), kBS, 0, s>>>(n, list, r, z);
}

template void launch_vc_condense<double>(const VecDev &, const VecCellDev<double> &, const double *, double *,
                                         double *, hipStream_t);
template void launch_vc_condense<float>(const VecDev &, const VecCellDev<float> &, const float *, float *, float *,
                                        hipStream_t);
template void launch_vc_expand<double>(const VecDev &, const VecCellDev<double> &, double *, hipStream_t);
template void launch_vc_expand<float>(const VecDev &, const VecCellDev<float> &, float *, hipStream_t);
template void launch_list_gather<double>(int, const int *, const int *, const int *, const double *,
                                         const double *, double *, double, hipStream_t);
template void launch_list_gather<float>(int, const int *, const int *, const int *, const float *, const float *,
                                        float *, float, hipStream_t);
template void launch_rows_scale<double>(int, const int *, const double *, const double *, double *, hipStream_t);
template void launch_rows_scale<float>(int, const int *, const float *, const float *, float *, hipStream_t);
template void launch_csr<double, double, double>(int, const int *, const int *, const int *, const double *,
                                                 const double *, double *, int, hipStream_t);
template void launch_csr<float, float, float>(int, const int *, const int *, const int *, const float *,
                                              const float *, float *, int, hipStream_t);
template void launch_csr<double, float, double>(int, const int *, const int *, const int *, const double *,
                                                const float *, double *, int, hipStream_t);
template void launch_csr<double, double, float>(int, const int *, const int *, const int *, const double *,
                                                const double *, float *, int, hipStream_t);
template void launch_edge_solve<double>(const EdgeDev &, const double *, const double *, double *, hipStream_t);
template void launch_edge_solve<float>(const EdgeDev &, const float *, const float *, float *, hipStream_t);
template void launch_gemv<double>(int, const double *, const double *, double *, hipStream_t);
template void launch_gemv<float>(int, const float *, const double *, double *, hipStream_t);
template void launch_list_copy<double>(int, const int *, const double *, double *, hipStream_t);
template void launch_list_copy<float>(int, const int *, const float *, float *, hipStream_t);

}  // namespace rz
