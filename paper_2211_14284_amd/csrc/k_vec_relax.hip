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

// The same product with one wavefront per row (rows of hundreds of entries: the
// restriction to the p = 1 space): lanes stride over the row, then a fixed-order
// shuffle reduction.
template <typename TV, typename TX, typename TY>
__global__ void __launch_bounds__(kBS) k_csr_wave(int n, const int *__restrict__ rows, const int *__restrict__ ptr,
                                                  const int *__restrict__ col, const TV *__restrict__ val,
                                                  const TX *__restrict__ x, TY *__restrict__ y, int add) {
  const int lane = threadIdx.x & 63;
  const long t = (long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (t >= n) return;
  TV acc = 0;
  for (int k = ptr[t] + lane; k < ptr[t + 1]; k += 64) acc += val[k] * (TV)x[col[k]];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if (lane == 0) {
    const int g = rows ? rows[t] : (int)t;
    y[g] = add ? (TY)((TV)y[g] + acc) : (TY)acc;
  }
}

// Edge-star patch solves, z = W^T (W b) per (patch, mode block) with W = L^{-1} of the
// block's Cholesky factor (the patch type's, computed at setup in FP64).  A block of
// the kernel takes one mode block of up to 256 patches of one type: W goes to LDS once
// (by rows), and each lane solves one patch with its n values in registers (n fixed
// per degree and mode: 4p - 3 for mode 0, 8p - 3 for the others): y = W b bottom-up
// and z = W^T y top-down in place (y_r needs b_0..b_r, z_r needs y_r..y_{n-1}), every
// W entry read by all lanes at once.  Sums run over ascending column index.
// (the empty asm with a memory clobber after each row keeps the compiler from holding
// the LDS values of W in registers across rows and phases: only v stays live)
template <typename T, int N>
__device__ __forceinline__ void edge_block_solve(const T *W, T (&v)[N]) {
#pragma unroll
  for (int r = N - 1; r >= 0; --r) {
    T acc = 0;
#pragma unroll
    for (int c = 0; c <= r; ++c) acc += W[r * (r + 1) / 2 + c] * v[c];
    v[r] = acc;
    asm volatile("" ::: "memory");
  }
#pragma unroll
  for (int r = 0; r < N; ++r) {
    T acc = 0;
#pragma unroll
    for (int c = r; c < N; ++c) acc += W[c * (c + 1) / 2 + r] * v[c];
    v[r] = acc;
    asm volatile("" ::: "memory");
  }
}

template <typename T, int N>
__device__ __forceinline__ void edge_chunk(const EdgeDev &E, const T *__restrict__ fac, const T *__restrict__ rt,
                                           T *__restrict__ zb, T *sW, int blk) {
  const int c0 = E.chunk[3 * blockIdx.x], c1 = E.chunk[3 * blockIdx.x + 1], type = E.chunk[3 * blockIdx.x + 2];
  const int s0 = E.blk_slot[blk];
  // the block's W by rows: it follows the by-columns copy in the factor set
  const T *Wr = fac + (size_t)type * E.fac_stride + E.blk_fac[blk] + N * (N + 1) / 2;
  for (int k = threadIdx.x; k < N * (N + 1) / 2; k += blockDim.x) sW[k] = Wr[k];
  __syncthreads();
  const int q = c0 + (int)threadIdx.x;
  if (q >= c1) return;
  const int patch = E.plist[q];
  const int *ix = E.idx + (size_t)patch * E.nslot + s0;
  T v[N];
#pragma unroll
  for (int r = 0; r < N; ++r) {
    const int g = ix[r];
    v[r] = g >= 0 ? rt[g] : T(0);
  }
  edge_block_solve<T, N>(sW, v);
  T *zo = zb + (size_t)patch * E.nslot + s0;
#pragma unroll
  for (int r = 0; r < N; ++r) zo[r] = v[r];
}

template <typename T, int P>
__global__ void __launch_bounds__(256) k_edge_solve(EdgeDev E, const T *__restrict__ fac, const T *__restrict__ rt,
                                                    T *__restrict__ zb) {
  constexpr int N0 = 4 * P - 3, N1 = 8 * P - 3;
  __shared__ T sW[N1 * (N1 + 1) / 2];
  const int blk = blockIdx.y;
  if (blk == 0) edge_chunk<T, N0>(E, fac, rt, zb, sW, 0);
  else if constexpr (P > 1) edge_chunk<T, N1>(E, fac, rt, zb, sW, blk);
}

// y = M x for a dense symmetric m x m matrix (row-major) reading only its lower
// triangle: one block per 64 x 64 tile (ti, tj), ti >= tj, adds M_ij x_j to row block
// ti and, below the diagonal, M_ij^T x_i to row block tj, each as a partial vector in
// part[(row block) * nt + (other tile index)] (one partial per pair, no atomics);
// k_symv_reduce sums the nt partials of every row in a fixed order.  FP64 sums.
template <typename TM>
__global__ void __launch_bounds__(256) k_symv_tile(int m, int nt, const TM *__restrict__ M,
                                                   const double *__restrict__ x, double *__restrict__ part) {
  // the tile in LDS, rows padded by one entry so that a lane-per-row read of one
  // column touches distinct banks
  __shared__ TM tile[64][65];
  __shared__ double xi[64], xj[64], red[4][64];
  const long b = blockIdx.x;
  int ti = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
  while ((long)(ti + 1) * (ti + 2) / 2 <= b) ++ti;
  while ((long)ti * (ti + 1) / 2 > b) --ti;
  const int tj = (int)(b - (long)ti * (ti + 1) / 2);
  const int r0 = 64 * ti, c0 = 64 * tj, tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  if (tid < 64) {
    xi[tid] = r0 + tid < m ? x[r0 + tid] : 0.0;
    xj[tid] = c0 + tid < m ? x[c0 + tid] : 0.0;
  }
  // wave wv loads rows 16 wv .. 16 wv + 15, lane = column (one contiguous row segment
  // per load); column partial sums of M^T x_i over those rows stay in the lane
  TM v[16];
  const int c = c0 + lane;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int row = r0 + 16 * wv + k;
    v[k] = row < m && c < m ? M[(long)row * m + c] : TM(0);
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) tile[16 * wv + k][lane] = v[k];
  __syncthreads();
  if (ti != tj) {  // uniform over the block
    double cs = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) cs += (double)v[k] * xi[16 * wv + k];
    red[wv][lane] = cs;
  }
  __syncthreads();
  if (ti != tj && tid < 64) part[((long)tj * nt + ti) * 64 + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
  // row partial sums of M x_j: lane = row, wave wv takes columns 16 wv .. 16 wv + 15
  double rs = 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) rs += (double)tile[lane][16 * wv + k] * xj[16 * wv + k];
  __syncthreads();
  red[wv][lane] = rs;
  __syncthreads();
  if (tid < 64) part[((long)ti * nt + tj) * 64 + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
}

// one block per row block: y = sum over the nt partials, four waves over a quarter of
// them each, combined in a fixed order
__global__ void __launch_bounds__(256) k_symv_reduce(int m, int nt, const double *__restrict__ part,
                                                     double *__restrict__ y) {
  __shared__ double red[4][64];
  const int bi = blockIdx.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double acc = 0.0;
  for (int k = wv; k < nt; k += 4) acc += part[((long)bi * nt + k) * 64 + lane];
  red[wv][lane] = acc;
  __syncthreads();
  const int i = 64 * bi + threadIdx.x;
  if (threadIdx.x < 64 && i < m) y[i] = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
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

// Dense patch solves z_v = W_v^T (W_v b_v), W_v = L_v^{-1} packed by rows, on patches
// given by index lists (nr entries per patch, -1 for the padding rows, whose W rows
// are those of the identity): one block per patch; y = W b with one wavefront per
// row, z = W^T y with one thread per column reading the rows in order.
template <typename T>
__global__ void __launch_bounds__(256) k_dense_patch_solve(int nr, const int *__restrict__ idx,
                                                            const T *__restrict__ W, const T *__restrict__ r,
                                                            T *__restrict__ zb) {
  extern __shared__ __align__(16) unsigned char dps_smem[];
  double *sb = reinterpret_cast<double *>(dps_smem), *sy = sb + nr;
  const long pt = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int i = tid; i < nr; i += blockDim.x) {
    const int g = idx[pt * nr + i];
    sb[i] = g >= 0 ? (double)r[g] : 0.0;
  }
  __syncthreads();
  const T *Ws = W + pt * ((long)nr * (nr + 1) / 2);
  for (int i = wv; i < nr; i += blockDim.x >> 6) {
    const T *row = Ws + (long)i * (i + 1) / 2;
    double acc = 0.0;
    for (int j = lane; j <= i; j += 64) acc += (double)row[j] * sb[j];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) sy[i] = acc;
  }
  __syncthreads();
  for (int j0 = 0; j0 < nr; j0 += blockDim.x) {
    const int j = j0 + tid;
    double acc = 0.0;
    for (int i = j0; i < nr; ++i)
      if (j <= i) acc += (double)Ws[(long)i * (i + 1) / 2 + j] * sy[i];
    if (j < nr) zb[pt * nr + j] = (T)acc;
  }
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

template <typename TV, typename TX, typename TY>
void launch_csr_wave(int n, const int *rows, const int *ptr, const int *col, const TV *val, const TX *x, TY *y,
                     int add, hipStream_t s) {
  if (n > 0) k_csr_wave<TV, TX, TY><<<(unsigned)((n + 3) / 4), kBS, 0, s>>>(n, rows, ptr, col, val, x, y, add);
}
template void launch_csr_wave<double, double, double>(int, const int *, const int *, const int *, const double *,
                                                      const double *, double *, int, hipStream_t);

template <typename T>
void launch_edge_solve(const EdgeDev &E, const T *fac, const T *rt, T *zb, hipStream_t s) {
  if (E.nchunk <= 0) return;
  const dim3 grid((unsigned)E.nchunk, (unsigned)E.p);
  switch (E.p) {
    case 1: k_edge_solve<T, 1><<<grid, 256, 0, s>>>(E, fac, rt, zb); break;
    case 2: k_edge_solve<T, 2><<<grid, 256, 0, s>>>(E, fac, rt, zb); break;
    case 3: k_edge_solve<T, 3><<<grid, 256, 0, s>>>(E, fac, rt, zb); break;
    case 4: k_edge_solve<T, 4><<<grid, 256, 0, s>>>(E, fac, rt, zb); break;
    case 5: k_edge_solve<T, 5><<<grid, 256, 0, s>>>(E, fac, rt, zb); break;
    case 6: k_edge_solve<T, 6><<<grid, 256, 0, s>>>(E, fac, rt, zb); break;
    case 7: k_edge_solve<T, 7><<<grid, 256, 0, s>>>(E, fac, rt, zb); break;
    case 8: k_edge_solve<T, 8><<<grid, 256, 0, s>>>(E, fac, rt, zb); break;
    case 9: k_edge_solve<T, 9><<<grid, 256, 0, s>>>(E, fac, rt, zb); break;
    default: break;
  }
}

template <typename TM>
void launch_symv(int m, const TM *M, const double *x, double *y, double *work, hipStream_t s) {
  if (m <= 0) return;
  const int nt = (m + 63) / 64;
  k_symv_tile<TM><<<(unsigned)((long)nt * (nt + 1) / 2), 256, 0, s>>>(m, nt, M, x, work);
  k_symv_reduce<<<nt, 256, 0, s>>>(m, nt, work, y);
}
template void launch_symv<double>(int, const double *, const double *, double *, double *, hipStream_t);
template void launch_symv<float>(int, const float *, const double *, double *, double *, hipStream_t);

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

template <typename T>
void launch_dense_patch_solve(int npatch, int nr, const int *idx, const T *W, const T *r, T *zb, hipStream_t s) {
  if (npatch <= 0) return;
  k_dense_patch_solve<T><<<(unsigned)npatch, 256, 2 * sizeof(double) * nr, s>>>(nr, idx, W, r, zb);
}
template void launch_dense_patch_solve<double>(int, int, const int *, const double *, const double *, double *,
                                               hipStream_t);
template void launch_dense_patch_solve<float>(int, int, const int *, const float *, const float *, float *,
                                              hipStream_t);

}  // namespace rz
