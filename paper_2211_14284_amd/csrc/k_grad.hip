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

#include <algorithm>

#include "bf16.hpp"
#include "kernels.hpp"
#include "lattice.hpp"

namespace rz {

namespace {

__device__ __forceinline__ bool lat_dirichlet(const LatDev &L, int X, int Y, int Z) {
  return ((L.dir & 1u) && X == 0) || ((L.dir & 2u) && X == L.Nx - 1) ||
         ((L.dir & 4u) && Y == 0) || ((L.dir & 8u) && Y == L.Ny - 1) ||
         ((L.dir & 16u) && Z == 0) || ((L.dir & 32u) && Z == L.Nz - 1);
}

// Dirichlet test of one lattice coordinate along axis a (0: x, 1: y, 2: z)
__device__ __forceinline__ bool lat_dirichlet_axis(const LatDev &L, int a, int v) {
  const int N = a == 0 ? L.Nx : (a == 1 ? L.Ny : L.Nz);
  return ((L.dir & (1u << (2 * a))) && v == 0) || ((L.dir & (2u << (2 * a))) && v == N - 1);
}

__device__ __forceinline__ long lat_index(const LatDev &L, int X, int Y, int Z) {
  return (long)X + (long)L.Nx * ((long)Y + (long)L.Ny * (long)Z);
}

__device__ __forceinline__ int ncells_axis(const LatDev &L, int a) {
  return a == 0 ? L.nx : (a == 1 ? L.ny : L.nz);
}

// Workgroups are dispatched to the 8 XCDs in turn (block b to XCD b mod 8), each
// with its own L2.  Row kernels read neighbouring rows, so block b is mapped to a
// logical index such that every XCD works through one contiguous range of rows.
__device__ __forceinline__ long xcd_block(long b, long nblk) {
  constexpr int kXcd = 8;
  const long q = nblk / kXcd, rem = nblk % kXcd;
  const int x = b % kXcd;
  return x * q + min((long)x, rem) + b / kXcd;
}

// Lattice rows (Y, Z) along x, enumerated as: rows on a y- or z-vertex plane first
// (Y on a vertex plane with any Z, then Z on a vertex plane with Y off them), then
// the rows strictly inside a cell's y-z cross section.
template <int P>
__device__ __forceinline__ void plane_row(const LatDev &L, long line, int &Y, int &Z) {
  const long n1 = (long)(L.ny + 1) * L.Nz;
  if (line < n1) {
    Y = (int)(line / L.Nz) * P;
    Z = line % L.Nz;
  } else if constexpr (P > 1) {
    const long m = line - n1, off = (long)L.ny * (P - 1);
    Z = (int)(m / off) * P;
    const int yn = m % off;
    Y = (yn / (P - 1)) * P + 1 + yn % (P - 1);
  } else {
    Y = Z = 0;
  }
}

template <int P>
__device__ __forceinline__ void interior_row(const LatDev &L, long i, int &Y, int &Z) {
  if constexpr (P > 1) {
    const long my = (long)L.ny * (P - 1);
    const int iy = i % my, iz = i / my;
    Y = (iy / (P - 1)) * P + 1 + iy % (P - 1);
    Z = (iz / (P - 1)) * P + 1 + iz % (P - 1);
  } else {
    Y = Z = 0;  // P = 1 has no interior rows
  }
}

// ------------------------------------------------------------------------------------
// y = A x: per cell, y_K = s1 (A x B x B) + s2 (B x A x B) + s3 (B x B x A) + mu (B x B x B)
// (eq. sum-factorization with the exact 1-D integrals of an axis-aligned cell),
// applied as per-axis contractions.  In the FDM basis B is diagonal plus the (0,p)
// pair and A an arrowhead, so each 1-D factor costs O(p) per line.
//
// Pencil decomposition: one block per x-row of cells (fixed cell indices ey, ez),
// walked in chunks of CPC cells.  Per chunk: one thread per tensor line of a cell,
// lines exchanged through LDS (x to z, z to y, y to x).  The x-faces shared by two
// cells of the row are summed in the block (the last cell's x = P face carries to
// the next chunk), so every lattice row (Y, Z) strictly inside the row's y-z cross
// section is complete when stored and goes to y directly, coalesced along x.  The
// 4p rows of the cross section on its y- or z-faces go to a face-line buffer, one
// x-line per (row of cells, face row), summed by k_apply_faces.  The next chunk's
// x tile is loaded into registers while the current chunk computes.  With bsub
// given the kernels store bsub - A x instead (the residual of the V-cycle).
// ------------------------------------------------------------------------------------
template <int P, typename T>
struct Tab1D {
  T B[(P + 1) * (P + 1)];
  T A[(P + 1) * (P + 1)];
};

template <int P, typename T>
__device__ __forceinline__ void mass_line(const Tab1D<P, T> &t, const T *in, T *out) {
  constexpr int N1 = P + 1;
#pragma unroll
  for (int m = 0; m <= P; ++m) out[m] = t.B[m * N1 + m] * in[m];
  out[0] += t.B[P] * in[P];
  out[P] += t.B[P * N1] * in[0];
}

template <int P, typename T>
__device__ __forceinline__ void stiff_line(const Tab1D<P, T> &t, const T *in, T *out) {
  constexpr int N1 = P + 1;
#pragma unroll
  for (int m = 1; m < P; ++m) out[m] = t.A[m * N1 + m] * in[m] + t.A[m * N1] * in[0] + t.A[m * N1 + P] * in[P];
  T a0 = 0, aP = 0;
#pragma unroll
  for (int i = 0; i <= P; ++i) {
    a0 += t.A[i] * in[i];
    aP += t.A[P * N1 + i] * in[i];
  }
  out[0] = a0;
  out[P] = aP;
}

// face-row index of (b, c) in a cell's y-z cross section (b or c on {0, P})
template <int P>
__device__ __forceinline__ int face_row(int b, int c) {
  return c == 0 ? b : (c == P ? P + 1 + b : 2 * (P + 1) + 2 * (c - 1) + (b == P));
}

template <int P, typename T, int CPC, typename S = T>
__global__ void __launch_bounds__(CPC *(P + 1) * (P + 1), 4)
    k_apply_pencil(LatDev L, Tab1D<P, T> tb, const T *__restrict__ coef, const S *__restrict__ x,
                   const S *__restrict__ bsub, S *__restrict__ y, T *__restrict__ fb) {
  constexpr int N1 = P + 1, NL = N1 * N1, NT = CPC * NL, W = CPC * P + 1;
  // LDS tile of a cell: element (a, b, c) at a + SB b + SC c, cells CS apart; the
  // padding spreads the lanes of the z-, y- and x-line passes over the banks
  constexpr int SB = N1 + 1, SC = SB * N1, CS = SC * N1 + 8;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *S0 = reinterpret_cast<T *>(smem_raw), *S1 = S0 + CPC * CS;
  T(*CR)[NL] = reinterpret_cast<T(*)[NL]>(S1 + CPC * CS);  // x = P face carried between chunks
  const int tid = threadIdx.x, lc = tid / NL, l = tid % NL;
  const int pen = xcd_block(blockIdx.x, gridDim.x);
  const int ey = pen % L.ny, ez = pen / L.ny;
  const int nch = (L.nx + CPC - 1) / CPC;
  T *s0 = S0 + lc * CS, *s1 = S1 + lc * CS;
  // x tile of chunk j: thread tid loads the z-column (a, lk, b) of the chunk's cells,
  // a = tid % N1, lk = (tid / N1) % CPC, b = tid / (N1 CPC), c = 0..P (lanes along x);
  // the loads stay in flight until the values go to LDS at the top of the next chunk
  const int la = tid % N1, llk = (tid / N1) % CPC, lb = tid / (N1 * CPC);
  const int Yl = ey * P + lb;
  const long zst = (long)L.Nx * L.Ny;
  unsigned zmask = 0;  // bit c: the point at Z = ez P + c is not on a Dirichlet z-face
#pragma unroll
  for (int i = 0; i < N1; ++i) zmask |= (unsigned)!lat_dirichlet_axis(L, 2, ez * P + i) << i;
  if (lat_dirichlet_axis(L, 1, Yl)) zmask = 0;
  T xv[N1];
  unsigned okm = 0;  // bit c: xv[c] is a free DoF of the chunk (else it counts as 0)
  auto load = [&](int j) {
    const int X = (j * CPC + llk) * P + la;
    const bool okx = j * CPC + llk < L.nx && !lat_dirichlet_axis(L, 0, X);
    okm = okx ? zmask : 0u;
    // always in bounds (x clamped to the lattice); masked values are never used
    const S *xc = x + lat_index(L, min(X, L.Nx - 1), Yl, ez * P);
#pragma unroll
    for (int i = 0; i < N1; ++i) xv[i] = st_load<T, S>(xc[i * zst]);
  };
  load(0);
  T *sx = S0 + llk * CS + la + SB * lb;
  for (int j = 0; j < nch; ++j) {
    const int nc = min(CPC, L.nx - j * CPC);
#pragma unroll
    for (int i = 0; i < N1; ++i) sx[SC * i] = ((okm >> i) & 1u) ? xv[i] : T(0);
    // this chunk's weights first: the compute waits on them, not on the prefetch
    const long cell = (j * CPC + min(lc, nc - 1)) + (long)L.nx * (ey + (long)L.ny * ez);
    const T s1c = coef[6 * cell], s2c = coef[6 * cell + 1], s3c = coef[6 * cell + 2], mu = coef[6 * cell + 3];
    load(min(j + 1, nch - 1));  // unconditional, so no branch merges the wait counts
    T r0[N1], r1[N1], r2[N1];
    __syncthreads();
    const int lz = l % N1 + SB * (l / N1);  // z-line (a, b) = (l % N1, l / N1)
    {  // z-line (a, b): t1 = B_z x, v = A_z x
#pragma unroll
      for (int c = 0; c <= P; ++c) r0[c] = s0[lz + SC * c];
      mass_line<P, T>(tb, r0, r1);
      stiff_line<P, T>(tb, r0, r2);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c <= P; ++c) {
      s0[lz + SC * c] = r1[c];
      s1[lz + SC * c] = r2[c];
    }
    __syncthreads();
    {  // y-line (a, c): u = B_y t1, w = mu u + s2 A_y t1 + s3 B_y v
      const int a = l % N1, c = l / N1;
#pragma unroll
      for (int b = 0; b <= P; ++b) {
        r0[b] = s0[a + SB * b + SC * c];
        r1[b] = s1[a + SB * b + SC * c];
      }
      T u[N1], t[N1];
      mass_line<P, T>(tb, r0, u);
      stiff_line<P, T>(tb, r0, t);
      mass_line<P, T>(tb, r1, r2);
      __syncthreads();
#pragma unroll
      for (int b = 0; b <= P; ++b) {
        s0[a + SB * b + SC * c] = u[b];
        s1[a + SB * b + SC * c] = mu * u[b] + s2c * t[b] + s3c * r2[b];
      }
    }
    __syncthreads();
    {  // x-line (b, c): y = s1 A_x u + B_x w
      const int b = l % N1, c = l / N1;
#pragma unroll
      for (int a = 0; a <= P; ++a) {
        r0[a] = s0[a + SB * b + SC * c];
        r1[a] = s1[a + SB * b + SC * c];
      }
      stiff_line<P, T>(tb, r0, r2);
      mass_line<P, T>(tb, r1, r0);
      __syncthreads();
#pragma unroll
      for (int a = 0; a <= P; ++a) s0[a + SB * b + SC * c] = s1c * r2[a] + r0[a];
    }
    __syncthreads();
    // rows of the chunk, lanes along x: point xo of row (b, c) is local a = xo % P of
    // cell xo / P plus, at a = 0, the x = P face of the cell before it
    const bool last = j + 1 == nch;
    for (int k = tid; k < NL * W; k += NT) {
      const int xo = k % W, row = k / W, b = row % N1, c = row / N1, ro = SB * b + SC * c;
      T val;
      if (xo < nc * P) {
        const int lk = xo / P, a = xo % P;
        val = S0[lk * CS + a + ro];
        if (a == 0) val += lk > 0 ? S0[(lk - 1) * CS + P + ro] : (j > 0 ? CR[(j - 1) & 1][row] : T(0));
      } else if (last && xo == nc * P) {
        val = S0[(nc - 1) * CS + P + ro];
      } else {
        continue;
      }
      const int X = j * CPC * P + xo;
      if (b > 0 && b < P && c > 0 && c < P) {
        const long g = lat_index(L, X, ey * P + b, ez * P + c);
        if (lat_dirichlet(L, X, ey * P + b, ez * P + c)) val = st_load<T, S>(x[g]);
        y[g] = st_store<S, T>(bsub ? st_load<T, S>(bsub[g]) - val : val);
      } else {
        fb[((long)pen * 4 * P + face_row<P>(b, c)) * L.Nx + X] = val;
      }
    }
    if (tid < NL) CR[j & 1][tid] = S0[(nc - 1) * CS + P + SB * (tid % N1) + SC * (tid / N1)];
    __syncthreads();
  }
}

// Lattice rows (Y, Z) on a y- or z-vertex plane: the sum of the face-line buffer
// rows of the (up to 4) rows of cells that hold them, in a fixed order (cell z, then
// y, lower first); Dirichlet points take x.
template <int P, typename T, typename S = T>
__global__ void __launch_bounds__(256) k_apply_faces(LatDev L, const S *__restrict__ x, const T *__restrict__ fb,
                                                     const S *__restrict__ bsub, S *__restrict__ y, long n) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const int X = g % L.Nx;
  int Y, Z;
  plane_row<P>(L, g / L.Nx, Y, Z);
  const long gi = lat_index(L, X, Y, Z);
  const bool dir = lat_dirichlet(L, X, Y, Z);
  // the (up to 2 x 2) rows of cells holding the point along y and z: candidate j is
  // the cell below (j = 0, local coordinate P) or above (j = 1, local 0) on a vertex
  // plane, the cell itself (j = 0) off it; the loads of all candidates go out
  // together, then sum in the fixed order (z cells outer, y cells inner)
  const int qy = Y / P, qz = Z / P;
  const bool ony = Y % P == 0, onz = Z % P == 0;
  T f[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int i = c & 1, k = c >> 1;
    int cyc, byc, czc, bzc;
    bool ok = !dir;
    if (ony) {
      cyc = i ? qy : qy - 1;
      byc = i ? 0 : P;
      ok = ok && cyc >= 0 && cyc < L.ny;
    } else {
      cyc = qy;
      byc = Y % P;
      ok = ok && i == 0;
    }
    if (onz) {
      czc = k ? qz : qz - 1;
      bzc = k ? 0 : P;
      ok = ok && czc >= 0 && czc < L.nz;
    } else {
      czc = qz;
      bzc = Z % P;
      ok = ok && k == 0;
    }
    f[c] = ok ? fb[(((long)cyc + (long)L.ny * czc) * 4 * P + face_row<P>(byc, bzc)) * L.Nx + X] : T(0);
  }
  const T bs = bsub ? st_load<T, S>(bsub[gi]) : T(0);
  T val = 0;
  if (dir) {
    val = st_load<T, S>(x[gi]);
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) val += f[c];
  }
  y[gi] = st_store<S, T>(bsub ? bs - val : val);
}

// Interface rows of y: sum of the contributions of the (up to 8) cells that hold the
// DoF, read from the per-cell buffer in a fixed order (z, y, x of the cells);
// Dirichlet rows copy x.  Rows interior to a cell were written by the cell kernel.
template <typename S, typename T>
__global__ void k_apply_gather(LatDev L, const S *__restrict__ x, const T *__restrict__ ebuf, S *__restrict__ y,
                               long n, const S *__restrict__ bsub) {
  long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const int p = L.p, n1 = p + 1, n3 = n1 * n1 * n1;
  const int C[3] = {(int)(g % L.Nx), (int)((g / L.Nx) % L.Ny), (int)(g / ((long)L.Nx * L.Ny))};
  if (C[0] % p != 0 && C[1] % p != 0 && C[2] % p != 0) return;
  if (lat_dirichlet(L, C[0], C[1], C[2])) {
    y[g] = bsub ? st_store<S, T>(st_load<T, S>(bsub[g]) - st_load<T, S>(x[g])) : x[g];
    return;
  }
  // per axis the (1 or 2) cells holding the coordinate: candidate 0 is the cell below
  // (local p) on a vertex plane, else the cell itself; candidate 1 the cell above
  // (local 0).  All (up to 8) loads go out together, then sum in the fixed order
  // (z cells outer, x cells inner; absent cells add zero).
  int c0[3], l0[3];
  bool has0[3], has1[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int nc = ncells_axis(L, d), c = C[d] / p;
    if (C[d] % p == 0) {
      has0[d] = c - 1 >= 0;
      has1[d] = c < nc;
      c0[d] = c - 1;
      l0[d] = p;
    } else {
      has0[d] = true;
      has1[d] = false;
      c0[d] = c;
      l0[d] = C[d] % p;
    }
  }
  T v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int i = q & 1, j = (q >> 1) & 1, k = q >> 2;
    const bool ok = (i ? has1[0] : has0[0]) && (j ? has1[1] : has0[1]) && (k ? has1[2] : has0[2]);
    const int cx = i ? c0[0] + 1 : c0[0], cy = j ? c0[1] + 1 : c0[1], cz = k ? c0[2] + 1 : c0[2];
    const int lx = i ? 0 : l0[0], ly = j ? 0 : l0[1], lz = k ? 0 : l0[2];
    const long cell = cx + (long)L.nx * (cy + (long)L.ny * cz);
    v[q] = ok ? ebuf[cell * n3 + lx + n1 * (ly + n1 * lz)] : T(0);
  }
  T acc = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) acc += v[q];
  y[g] = st_store<S, T>(bsub ? st_load<T, S>(bsub[g]) - acc : acc);
}

// ------------------------------------------------------------------------------------
// Relaxation step 1 (eq. schur, R_Gamma r): rt_G = r_G - P_GI P_II^{-1} r_I.  Only
// face DoFs (exactly one lattice coordinate on a vertex plane) couple to cell
// interiors: along their normal line in each of the two cells.
// ------------------------------------------------------------------------------------
// t = r / dd at an interior point of cell ce with local coordinates l (P_II is
// diagonal: dd = mu + sum_d sigma_d lambda_{l_d})
template <typename T>
__device__ __forceinline__ T interior_scaled(const T *coef, long ce, const T *lam, int l0, int l1, int l2, T rv) {
  const T *cf = coef + 6 * ce;
  const T dd = cf[3] + cf[0] * lam[l0] + cf[1] * lam[l1] + cf[2] * lam[l2];
  return rv / dd;
}

// One block per lattice row, lanes along x.  For a face DoF with normal axis a the
// two cells sharing the face contribute sigma_a sum_i A_{e,i} t_i over the cell's
// interior line through the DoF (e = P for the cell below, 0 for the cell above).
// Rows on a y- or z-vertex plane: every point is a plane point; the normal lines
// run across rows (coalesced over the lanes).  Rows inside a cross section: only
// the x-face points (X on an x-vertex plane) are plane points; the row of r is
// handled by extra blocks of the same launch.  Interior points of rt are not written.
template <int P, typename T>
__device__ void condense_xface(const LatDev &L, const T *__restrict__ coef, const T *__restrict__ Ag,
                               const T *__restrict__ lam, const T *__restrict__ r, T *__restrict__ rt, long t,
                               long n);

template <int P, typename T>
__global__ void __launch_bounds__(256) k_condense_rows(LatDev L, const T *__restrict__ coef,
                                                       const T *__restrict__ Ag, const T *__restrict__ lam,
                                                       const T *__restrict__ r, T *__restrict__ rt, long nplane,
                                                       long nxf) {
  constexpr int N1 = P + 1;
  const long sz = (long)L.Nx * L.Ny;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (blockIdx.x >= nplane) {  // the x-face points of the other rows, one lane each
    condense_xface<P, T>(L, coef, Ag, lam, r, rt, (blockIdx.x - nplane) * (long)blockDim.x + threadIdx.x, nxf);
    return;
  }
  const long blk = xcd_block(blockIdx.x, nplane);
  {
    int Y, Z;
    plane_row<P>(L, blk, Y, Z);
    const bool ony = Y % P == 0, onz = Z % P == 0;
    const long row = (long)L.Nx * (Y + (long)L.Ny * Z);
    // face rows (normal y or z): the weights of the row's cells below and above the
    // face, staged in LDS (4 per cell: sigma_1..3, mu)
    const bool face = P >= 2 && ony != onz;
    const int a = ony ? 1 : 2, Ca = ony ? Y : Z, ka = Ca / P, na = ony ? L.ny : L.nz;
    const int co = ony ? Z / P : Y / P, lo_ = ony ? Z % P : Y % P;  // the remaining axis
    T *cw = reinterpret_cast<T *>(smem_raw);  // [2][nx][4]: below, above
    if (face) {
      for (int t = threadIdx.x; t < 2 * L.nx; t += blockDim.x) {
        const int side = t / L.nx, cx = t % L.nx, kc = ka - 1 + side;
        T v[4] = {0, 0, 0, 0};
        if (kc >= 0 && kc < na) {
          const long ce = ony ? cx + (long)L.nx * (kc + (long)L.ny * co) : cx + (long)L.nx * (co + (long)L.ny * kc);
#pragma unroll
          for (int j = 0; j < 4; ++j) v[j] = coef[6 * ce + j];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) cw[4 * t + j] = v[j];
      }
      __syncthreads();
    }
    const long st = ony ? (long)L.Nx : sz;
    const T llo = lam[lo_];
    for (int X = threadIdx.x; X < L.Nx; X += blockDim.x) {
      const long g = row + X;
      if (lat_dirichlet(L, X, Y, Z)) {
        rt[g] = T(0);
        continue;
      }
      T val = r[g];
      if (face && X % P != 0) {  // face point
        const int cx = X / P, lx = X % P;
        const T llx = lam[lx];
        const T *ra = r + g;
        // the interior values on the normal line in both cells, all loads in flight
        // together before either sum
        T vb[P > 1 ? P - 1 : 1], va[P > 1 ? P - 1 : 1];
#pragma unroll
        for (int i = 1; i < P; ++i) {
          vb[i - 1] = ka > 0 ? ra[(long)(i - P) * st] : T(0);
          va[i - 1] = ka < na ? ra[(long)i * st] : T(0);
        }
        // the cell's diagonal at (lx, i, lo_) with the normal axis at i: the
        // weights of the normal and of the remaining in-face axis
        const int an = ony ? 1 : 2, at = ony ? 2 : 1;
        if (ka > 0) {  // the cell below: its face at local coordinate P
          const T *cf = cw + 4 * cx;
          const T e = cf[3] + cf[0] * llx, cn = cf[an], ct = cf[at] * llo;
          T hi = 0;
#pragma unroll
          for (int i = 1; i < P; ++i) hi += Ag[P * N1 + i] * (vb[i - 1] / (e + cn * lam[i] + ct));
          val -= cf[a] * hi;
        }
        if (ka < na) {  // the cell above: its face at local coordinate 0
          const T *cf = cw + 4 * (L.nx + cx);
          const T e = cf[3] + cf[0] * llx, cn = cf[an], ct = cf[at] * llo;
          T lo = 0;
#pragma unroll
          for (int i = 1; i < P; ++i) lo += Ag[i] * (va[i - 1] / (e + cn * lam[i] + ct));
          val -= cf[a] * lo;
        }
      }
      rt[g] = val;
    }
  }
}

// The x-face points of the rows inside the cells' y-z cross sections, one lane per
// point (consecutive lanes along x, nx + 1 points per row); their x-lines lie in
// the same lattice row.  Run by the blocks appended to the k_condense_rows launch.
template <int P, typename T>
__device__ void condense_xface(const LatDev &L, const T *__restrict__ coef, const T *__restrict__ Ag,
                               const T *__restrict__ lam, const T *__restrict__ r, T *__restrict__ rt, long t,
                               long n) {
  constexpr int N1 = P + 1;
  if (t >= n) return;
  const int k = t % (L.nx + 1);
  int Y, Z;
  interior_row<P>(L, t / (L.nx + 1), Y, Z);
  const int X = k * P;
  const long g = lat_index(L, X, Y, Z);
  if (lat_dirichlet_axis(L, 0, X)) {
    rt[g] = T(0);
    return;
  }
  const int ly = Y % P, lz = Z % P;
  const long cyz = (long)L.nx * (Y / P + (long)L.ny * (Z / P));
  const T ly_ = lam[ly], lz_ = lam[lz];
  T val = r[g];
  if (k > 0) {
    const T *cf = coef + 6 * ((k - 1) + cyz);
    T hi = 0;
#pragma unroll
    for (int i = 1; i < P; ++i)
      hi += Ag[P * N1 + i] * (r[g - P + i] / (cf[3] + cf[0] * lam[i] + cf[1] * ly_ + cf[2] * lz_));
    val -= cf[0] * hi;
  }
  if (k < L.nx) {
    const T *cf = coef + 6 * (k + cyz);
    T lo = 0;
#pragma unroll
    for (int i = 1; i < P; ++i) lo += Ag[i] * (r[g + i] / (cf[3] + cf[0] * lam[i] + cf[1] * ly_ + cf[2] * lz_));
    val -= cf[0] * lo;
  }
  rt[g] = val;
}

// ------------------------------------------------------------------------------------
// Relaxation step 2 (eq. sc-asm-afw): L_v L_v^T z_v = rt|_v for every vertex slot.
// One wavefront per slot, no block barriers: the passes of the wavefront schedule
// (levels of the forward sweep) run in program order on the slot's vector in LDS,
// which only this wavefront touches, each row gathering its entries; then the same
// passes run in reverse for the transposed solve, each row finishing its value and
// pushing it to its columns with LDS atomic adds (rows of one pass may share a
// column; rows of one level never depend on each other).  The block shares the
// schedule's index tables in LDS, and the slot's vector is kept in FP64 in LDS for
// both precisions (the FP32 factor is widened on use).
// Two kernels: k_patch_solve_r (below) holds a slot's off-diagonals in registers
// between the sweeps; k_patch_solve_w, for the degrees and precisions whose values do
// not fit, streams them in both sweeps into two register buffers used in turn (pass
// u + 1 loads while pass u computes) through a buffer resource spanning the slot.
// ------------------------------------------------------------------------------------
// sum over the K steps of one lane in a pass of buf[s] * x[col(s)], K uniform: one
// straight-line body per K so that the LDS reads batch without per-step branches
template <int KM, typename T, int K = KM>
__device__ __forceinline__ double pass_dot(int k, const T (&buf)[KM], const unsigned short *ec, const double *xw) {
  if (k == K) {
    int ix[K];
#pragma unroll
    for (int s = 0; s < K; ++s) ix[s] = ec[64 * s];
    double acc = 0;
#pragma unroll
    for (int s = 0; s < K; ++s) acc += (double)buf[s] * xw[ix[s]];
    return acc;
  }
  if constexpr (K > 1) {
    return pass_dot<KM, T, K - 1>(k, buf, ec, xw);
  } else {
    return 0.0;
  }
}

// w[col(s)] -= buf[s] * xr over the K steps of one lane in a backward pass (the
// rows of a pass may share columns: LDS atomic adds; zero values, which include
// the padding, are skipped)
template <int KM, typename T, int K = KM>
__device__ __forceinline__ void pass_push(int k, const T (&buf)[KM], const unsigned short *ec, double *xw, double xr) {
  if (k == K) {
    int ix[K];
#pragma unroll
    for (int s = 0; s < K; ++s) ix[s] = ec[64 * s];
#pragma unroll
    for (int s = 0; s < K; ++s)
      if (buf[s] != T(0)) atomicAdd(&xw[ix[s]], -(double)buf[s] * xr);
    return;
  }
  if constexpr (K > 1) pass_push<KM, T, K - 1>(k, buf, ec, xw, xr);
}

// raw buffer loads (offsets in bytes, per-lane voff plus wave-uniform soff;
// out-of-range offsets read 0)
template <typename T>
__device__ __forceinline__ T buffer_load(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff = 0);
template <>
__device__ __forceinline__ double buffer_load<double>(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff) {
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  const u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0);
  return __builtin_bit_cast(double, v);
}
template <>
__device__ __forceinline__ float buffer_load<float>(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
}

// two adjacent values per lane: one 16-byte (FP64) or 8-byte (FP32) load
template <typename T>
__device__ __forceinline__ void buffer_load2(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff, T &a, T &b);
template <>
__device__ __forceinline__ void buffer_load2<double>(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff, double &a,
                                                     double &b) {
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  const u4 v = __builtin_amdgcn_raw_buffer_load_b128(r, off, soff, 0);
  a = __builtin_bit_cast(double, u2{v.x, v.y});
  b = __builtin_bit_cast(double, u2{v.z, v.w});
}
template <>
__device__ __forceinline__ void buffer_load2<float>(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff, float &a,
                                                    float &b) {
  // split through a 64-bit integer: taking the two elements of the returned
  // 2 x u32 vector directly compiles (hipcc of ROCm 7.2) into a single 4-byte load
  // whose value serves both
  const unsigned long long v =
      __builtin_bit_cast(unsigned long long, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
  a = __builtin_bit_cast(float, (unsigned)v);
  b = __builtin_bit_cast(float, (unsigned)(v >> 32));
}

template <typename T>
__device__ __forceinline__ T group_sum(T s, int G) {
  for (int o = G >> 1; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  return s;
}

template <typename T, int KM>
__global__ void __launch_bounds__(1024) k_patch_solve_w(LatDev L, PatchEllDev E, const T *__restrict__ factor,
                                                         const T *__restrict__ rt, T *__restrict__ zbuf,
                                                         long nslots) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nrows = E.nrows, ne = E.ne, np = E.npass, p = L.p;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
  // LDS: the wavefronts' vectors (FP64 whatever T is: the sweeps accumulate in FP64,
  // which also keeps the backward pushes on the FP64 LDS atomic add, several times
  // faster than the FP32 one), then their diagonals (T), then the shared tables
  double *xw = reinterpret_cast<double *>(smem_raw) + (size_t)w * nrows;  // this wavefront's vector
  T *dw = reinterpret_cast<T *>(reinterpret_cast<double *>(smem_raw) + (size_t)nw * nrows) + (size_t)w * nrows;
  int *off = reinterpret_cast<int *>(reinterpret_cast<T *>(reinterpret_cast<double *>(smem_raw) + (size_t)nw * nrows) +
                                     (size_t)nw * nrows);
  unsigned short *ecol = reinterpret_cast<unsigned short *>(off + nrows);
  unsigned short *erow = ecol + ne;
  for (int i = tid; i < ne; i += blockDim.x) ecol[i] = (unsigned short)E.ecol[i];
  for (int i = tid; i < np * 64; i += blockDim.x) erow[i] = (unsigned short)(E.erow[i] & 0xFFFF);
  for (int i = tid; i < nrows; i += blockDim.x)
    off[i] = (E.off[3 * i] + 64) | ((E.off[3 * i + 1] + 64) << 8) | ((E.off[3 * i + 2] + 64) << 16);
  __syncthreads();
  const int nvx = L.nx + 1, nvy = L.ny + 1;
  // the wavefront index as a wave-uniform (scalar) value, so that slot addresses
  // and the slot's buffer resource live in scalar registers
  const int wu = __builtin_amdgcn_readfirstlane(w);
  for (long sl = (long)blockIdx.x * nw + wu; sl < nslots; sl += (long)gridDim.x * nw) {
    const T *f = factor + sl * (long)E.stride;
    const int vx = sl % nvx, vy = (sl / nvx) % nvy, vz = sl / ((long)nvx * nvy);
    for (int i = lane; i < nrows; i += 64) {
      const int o = off[i];
      const int X = vx * p + (o & 255) - 64, Y = vy * p + ((o >> 8) & 255) - 64, Z = vz * p + ((o >> 16) & 255) - 64;
      const bool in = X >= 0 && X < L.Nx && Y >= 0 && Y < L.Ny && Z >= 0 && Z < L.Nz;
      xw[i] = (in && !lat_dirichlet(L, X, Y, Z)) ? (double)rt[lat_index(L, X, Y, Z)] : 0.0;
      dw[i] = f[i];
    }
    // Factor values of pass t through a buffer resource spanning this slot: steps
    // past K take an offset beyond the range, which reads 0 without a memory access,
    // so the loads carry no branch and stay in flight across the other buffer's pass.
    const __amdgpu_buffer_rsrc_t fr =
        __builtin_amdgcn_make_buffer_rsrc((void *)f, (short)0, E.stride * (int)sizeof(T), 0x00020000);
    // FP64: bit t set when the lane's row in pass t is real (boundary slots: trivial
    // rows are identity rows with zero columns, their values are not loaded)
    unsigned real = 0xFFFFFFFFu;
    const bool inner = vx >= 1 && vx < L.nx && vy >= 1 && vy < L.ny && vz >= 1 && vz < L.nz;
    if (sizeof(T) == 8 && !inner && np <= 32) {
      real = 0;
      for (int t = 0; t < np; ++t) {
        const unsigned row = erow[64 * t + lane];
        if (row >= (unsigned)nrows) continue;
        const int o = off[row];
        const int X = vx * p + (o & 255) - 64, Y = vy * p + ((o >> 8) & 255) - 64, Z = vz * p + ((o >> 16) & 255) - 64;
        if (X >= 0 && X < L.Nx && Y >= 0 && Y < L.Ny && Z >= 0 && Z < L.Nz && !lat_dirichlet(L, X, Y, Z))
          real |= 1u << t;
      }
    }
    auto load_pass = [&](T (&buf)[KM], int t) {
      const int K = E.pass[3 * t + 1], base = E.ell0 + E.pass[3 * t + 2];
      const int K2 = K & ~1;
      const bool on = (real >> t) & 1u;
#pragma unroll
      for (int s = 0; s < KM; ++s) {
        // value position of step s (steps in lane-adjacent pairs, an odd last step alone)
        const int pos = s < K2 ? base + 128 * (s >> 1) + 2 * lane + (s & 1) : base + 64 * s + lane;
        buf[s] = buffer_load<T>(fr, s < K && on ? (unsigned)pos * sizeof(T) : 0x80000000u);
      }
    };
    // pass sequence u = 0 .. 2 np - 1: the passes forward (gather), then the same in
    // reverse (push form of the transposed solve)
    const int nu = 2 * np;
    auto pass_of = [&](int u) { return u < np ? u : 2 * np - 1 - u; };
    auto run_pass = [&](const T (&buf)[KM], int u) {
      const int t = pass_of(u);
      const int G = E.pass[3 * t], K = E.pass[3 * t + 1], base = E.pass[3 * t + 2];
      const unsigned row = erow[64 * t + lane];
      const bool lead = (lane & (G - 1)) == 0 && row != 0xFFFFu;
      if (u < np) {
        double acc = 0;
        if (K > 0) {
          acc = pass_dot<KM, T>(K, buf, ecol + base + lane, xw);
          acc = group_sum(acc, G);
        }
        if (lead) xw[row] = (xw[row] - acc) / (double)dw[row];
      } else {
        if (lead) xw[row] = xw[row] / (double)dw[row];
        if (K > 0 && row != 0xFFFFu) pass_push<KM, T>(K, buf, ecol + base + lane, xw, xw[row]);
      }
    };
    // two register buffers in turn: pass u computes while pass u + 1 loads
    T ba[KM], bb[KM];
    load_pass(ba, pass_of(0));
    for (int u = 0; u < nu; u += 2) {
      load_pass(bb, pass_of(min(u + 1, nu - 1)));
      run_pass(ba, u);
      load_pass(ba, pass_of(min(u + 2, nu - 1)));
      if (u + 1 < nu) run_pass(bb, u + 1);
    }
    T *zo = zbuf + sl * (long)nrows;
    for (int i = lane; i < nrows; i += 64) zo[i] = (T)xw[i];
  }
}

// Register-resident variant for the degrees whose factor values fit a wavefront's
// registers (KT steps per lane: 97 at p = 7, so 194 VGPRs in FP64).  The schedule
// is compiled in (PassTable, generated from the same routine the setup runs), so
// every pass's steps sit at fixed register indices: a slot's off-diagonals are
// loaded once (two steps of a pass per load, fully coalesced across the lanes),
// used by the forward sweep and again from registers by the backward sweep, which
// reloads each pass's registers with the next slot's values as soon as the pass
// is done, so the next slot's factor streams in while this one finishes.  The
// diagonals are kept inverted in LDS.
template <int P>
struct PassTable {
  static constexpr int NR = 0, NP = 0, KT = 0;
};
#include "pass_tables.inc"

// one DPP move of a double (both halves; every lane reads a lane of its own row)
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// sum over aligned groups of G lanes, the same value on every lane of a group:
// lane swaps within quads, then the mirror images within 8 and 16 lanes (DPP),
// then cross-lane shuffles for 32 and 64
template <int G>
__device__ __forceinline__ double group_sum_c(double s) {
  if constexpr (G >= 2) s += dpp_move<0xB1>(s);   // quad_perm 1,0,3,2
  if constexpr (G >= 4) s += dpp_move<0x4E>(s);   // quad_perm 2,3,0,1
  if constexpr (G >= 8) s += dpp_move<0x141>(s);  // row_half_mirror
  if constexpr (G >= 16) s += dpp_move<0x140>(s); // row_mirror
  if constexpr (G >= 32) s += __shfl_xor(s, 16, 64);
  if constexpr (G >= 64) s += __shfl_xor(s, 32, 64);
  return s;
}

// pass t's values of a slot into their registers: the lane-adjacent step pairs
// with one load each, an odd last step alone.  A lane whose row is trivial (outside
// the domain or on a Dirichlet face: an identity row, and a zero column in every
// other row) takes an offset past the slot's range, which reads zeros without a
// memory access.
template <typename T, int P, int t>
__device__ __forceinline__ void load_pass_regs(T (&v)[PassTable<P>::KT], __amdgpu_buffer_rsrc_t r, int lane,
                                               bool on) {
  using S = PassTable<P>;
  constexpr int K = S::K[t], c0 = S::C[t], base = S::E0 + 64 * c0;
  constexpr unsigned kOut = 0x80000000u;
  const unsigned o2 = on ? 2 * lane * (unsigned)sizeof(T) : kOut, o1 = on ? lane * (unsigned)sizeof(T) : kOut;
#pragma unroll
  for (int g = 0; g < K / 2; ++g)
    buffer_load2<T>(r, o2, (base + 128 * g) * (unsigned)sizeof(T), v[c0 + 2 * g], v[c0 + 2 * g + 1]);
  if constexpr (K & 1) v[c0 + K - 1] = buffer_load<T>(r, o1, (base + 64 * (K - 1)) * sizeof(T));
}

// the vertex of a slot and whether its patch lies inside the domain away from the
// boundary (then no row of it is trivial)
struct SlotPos {
  int vx, vy, vz;
  bool inner;
};

__device__ __forceinline__ SlotPos slot_pos(const LatDev &L, long sl) {
  const int nvx = L.nx + 1, nvy = L.ny + 1;
  SlotPos s;
  s.vx = sl % nvx;
  s.vy = (sl / nvx) % nvy;
  s.vz = sl / ((long)nvx * nvy);
  s.inner = s.vx >= 1 && s.vx < L.nx && s.vy >= 1 && s.vy < L.ny && s.vz >= 1 && s.vz < L.nz;
  return s;
}

// bit t set when the lane's row in pass t is a real row of the slot at s (inside the
// domain and not on a Dirichlet face; the dummy row NR is not); all set for inner
// slots.  One short loop per boundary slot (at most 32 passes).
template <typename T, int P>
__device__ __forceinline__ unsigned real_row_mask(const LatDev &L, const int *off, const unsigned short *erow,
                                                  int lane, const SlotPos &s) {
  static_assert(PassTable<P>::NP <= 32, "one bit per pass");
  // FP32 launches are bound by the latency of the passes rather than by HBM, so they
  // load every row
  if (sizeof(T) == 4 || s.inner) return 0xFFFFFFFFu;
  unsigned m = 0;
#pragma unroll 1
  for (int t = 0; t < PassTable<P>::NP; ++t) {
    const unsigned row = erow[64 * t + lane];
    if (row >= (unsigned)PassTable<P>::NR) continue;
    const int o = off[row];
    const int X = s.vx * P + (o & 255) - 64, Y = s.vy * P + ((o >> 8) & 255) - 64,
              Z = s.vz * P + ((o >> 16) & 255) - 64;
    if (X >= 0 && X < L.Nx && Y >= 0 && Y < L.Ny && Z >= 0 && Z < L.Nz && !lat_dirichlet(L, X, Y, Z)) m |= 1u << t;
  }
  return m;
}

template <typename T, int P, int t = 0>
__device__ __forceinline__ void load_all_regs(T (&v)[PassTable<P>::KT], __amdgpu_buffer_rsrc_t r, int lane,
                                              unsigned mask) {
  if constexpr (t < PassTable<P>::NP) {
    load_pass_regs<T, P, t>(v, r, lane, (mask >> t) & 1u);
    load_all_regs<T, P, t + 1>(v, r, lane, mask);
  }
}

// indices of one pass read ahead of it: the lane's row, its columns, and (forward)
// the row's right-hand sides (one per vector) and inverted diagonal
template <int K, int NV>
struct PassIdx {
  unsigned row;
  int ix[K > 0 ? K : 1];
  double b[NV], d;
};

template <int P, int NV, int t>
__device__ __forceinline__ void read_idx(PassIdx<PassTable<P>::K[t], NV> &q, const unsigned short *ecol,
                                         const unsigned short *erow, int lane) {
  constexpr int K = PassTable<P>::K[t], c0 = PassTable<P>::C[t];
  q.row = erow[64 * t + lane];
#pragma unroll
  for (int s = 0; s < K; ++s) q.ix[s] = ecol[64 * (c0 + s) + lane];
}

// forward pass t (gather): x_row = (w_row - sum_s L[row, col(s)] x_col(s)) / L_row,row,
// for each of the NV vectors, which sit interleaved in LDS (row-major, NV values
// per row), so every factor value in registers serves all of them.  Every lane of
// a row's group holds the same sum and writes the same value, and lanes without a
// row use the dummy entry NR (zero vector values and diagonal), so the sweeps run
// without lane masks.  Pass t + 1's indices are read while pass t computes, and its
// row's right-hand sides before pass t writes (rows of different passes are
// distinct).
template <typename T, int P, int NV, int t>
__device__ __forceinline__ void fwd_passes(const T (&v)[PassTable<P>::KT], double *xw, const double *iw,
                                           const unsigned short *ecol, const unsigned short *erow, int lane,
                                           const PassIdx<PassTable<P>::K[t], NV> &q) {
  using S = PassTable<P>;
  constexpr int G = S::G[t], K = S::K[t], c0 = S::C[t];
  double xg[K > 0 ? K : 1][NV];
#pragma unroll
  for (int s = 0; s < K; ++s)
#pragma unroll
    for (int r = 0; r < NV; ++r) xg[s][r] = xw[q.ix[s] * NV + r];
  PassIdx<S::K[t + 1 < S::NP ? t + 1 : t], NV> n;
  if constexpr (t + 1 < S::NP) read_idx<P, NV, t + 1>(n, ecol, erow, lane);
  double acc[NV];
#pragma unroll
  for (int r = 0; r < NV; ++r) {
    acc[r] = 0;
    if constexpr (K > 0) {
      // two interleaved partial sums halve the dependent chain
      double a0 = 0, a1 = 0;
#pragma unroll
      for (int s = 0; s < K; s += 2) a0 += (double)v[c0 + s] * xg[s][r];
#pragma unroll
      for (int s = 1; s < K; s += 2) a1 += (double)v[c0 + s] * xg[s][r];
      acc[r] = group_sum_c<G>(a0 + a1);
    }
  }
  if constexpr (t + 1 < S::NP) {
#pragma unroll
    for (int r = 0; r < NV; ++r) n.b[r] = xw[n.row * NV + r];
    n.d = iw[n.row];
  }
#pragma unroll
  for (int r = 0; r < NV; ++r) xw[q.row * NV + r] = (q.b[r] - acc[r]) * q.d;
  if constexpr (t + 1 < S::NP) fwd_passes<T, P, NV, t + 1>(v, xw, iw, ecol, erow, lane, n);
}

// backward pass t (push form of L^T x = z): x_row = w_row / L_row,row, then
// w_col(s) -= L[row, col(s)] x_row, for each vector.  Padding values are zero, and
// their adds of -0 leave every value as it is (the dummy row's values are zero too).
// Pass t - 1's indices and inverted diagonal are read while pass t computes (the
// diagonals never change).  Once pass t has pushed, its registers load the next
// slot's values of pass t (through nr, which reads zeros without memory access past
// the last slot).
template <typename T, int P, int NV, int t>
__device__ __forceinline__ void bwd_passes(T (&v)[PassTable<P>::KT], double *xw, const double *iw,
                                           const unsigned short *ecol, const unsigned short *erow, int lane,
                                           const PassIdx<PassTable<P>::K[t], NV> &q, __amdgpu_buffer_rsrc_t nr,
                                           unsigned nmask) {
  using S = PassTable<P>;
  constexpr int K = S::K[t], c0 = S::C[t];
  double x[NV];
#pragma unroll
  for (int r = 0; r < NV; ++r) x[r] = xw[q.row * NV + r];
  PassIdx<S::K[t > 0 ? t - 1 : 0], NV> n;
  if constexpr (t > 0) read_idx<P, NV, t - 1>(n, ecol, erow, lane);
#pragma unroll
  for (int r = 0; r < NV; ++r) {
    x[r] *= q.d;
    xw[q.row * NV + r] = x[r];
  }
#pragma unroll
  for (int s = 0; s < K; ++s) {
    T vs = v[c0 + s];
    // an empty asm marks vs as redefined, so the FP32 factor is widened again here
    // instead of the forward sweep's widened copies staying live in registers
    if constexpr (sizeof(T) == 4) asm("" : "+v"(vs));
#pragma unroll
    for (int r = 0; r < NV; ++r) atomicAdd(&xw[q.ix[s] * NV + r], -(double)vs * x[r]);
  }
  load_pass_regs<T, P, t>(v, nr, lane, (nmask >> t) & 1u);
  if constexpr (t > 0) {
    n.d = iw[n.row];
    bwd_passes<T, P, NV, t - 1>(v, xw, iw, ecol, erow, lane, n, nr, nmask);
  }
}

template <typename T, int P, int NV>
__global__ void __launch_bounds__(256) k_patch_solve_r(LatDev L, PatchEllDev E, const T *__restrict__ factor,
                                                        PatchVecs<T> V, long nslots) {
  using S = PassTable<P>;
  constexpr int NR = S::NR, NP = S::NP, KT = S::KT;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int ne = E.ne;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
  // LDS: the wavefronts' vectors (NV interleaved, FP64, NR + 1 rows: the last is the
  // dummy row of lanes without a row), their inverted diagonals (FP64), the shared
  // tables
  constexpr int NR1 = NR + 1;
  double *xw = reinterpret_cast<double *>(smem_raw) + (size_t)w * NR1 * NV;
  double *iw = reinterpret_cast<double *>(smem_raw) + (size_t)nw * NR1 * NV + (size_t)w * NR1;
  int *off = reinterpret_cast<int *>(reinterpret_cast<double *>(smem_raw) + (size_t)nw * NR1 * (NV + 1));
  unsigned short *ecol = reinterpret_cast<unsigned short *>(off + NR);
  unsigned short *erow = ecol + ne;
  for (int i = tid; i < ne; i += blockDim.x) ecol[i] = (unsigned short)E.ecol[i];
  for (int i = tid; i < NP * 64; i += blockDim.x) erow[i] = (unsigned short)(E.erow[i] < 0 ? NR : E.erow[i]);
  for (int i = tid; i < NR; i += blockDim.x)
    off[i] = (E.off[3 * i] + 64) | ((E.off[3 * i + 1] + 64) << 8) | ((E.off[3 * i + 2] + 64) << 16);
  __syncthreads();
  const int nvx = L.nx + 1, nvy = L.ny + 1;
  const int wu = __builtin_amdgcn_readfirstlane(w);
  const long step = (long)gridDim.x * nw;
  // a slot's factor through a buffer resource; past the last slot its range is
  // empty, so that loads read zeros without touching memory
  auto slot_rsrc = [&](long s) {
    const bool ok = s < nslots;
    return __builtin_amdgcn_make_buffer_rsrc((void *)(factor + (ok ? s : 0) * (long)E.stride), (short)0,
                                             ok ? E.stride * (int)sizeof(T) : 0, 0x00020000);
  };
  long sl = (long)blockIdx.x * nw + wu;
  T v[KT];  // the current slot's off-diagonals (step s of the slot's passes in v[s])
  if (sl < nslots) load_all_regs<T, P>(v, slot_rsrc(sl), lane, real_row_mask<T, P>(L, off, erow, lane, slot_pos(L, sl)));
  for (; sl < nslots; sl += step) {
    const T *f = factor + sl * (long)E.stride;
    const int vx = sl % nvx, vy = (sl / nvx) % nvy, vz = sl / ((long)nvx * nvy);
    // right-hand sides and diagonals (the off-diagonals are loaded already)
    constexpr int NI = (NR + 63) / 64;
    T rhs[NI][NV], dia[NI];
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int i = lane + 64 * j;
#pragma unroll
      for (int r = 0; r < NV; ++r) rhs[j][r] = T(0);
      dia[j] = T(1);
      if (i < NR) {
        const int o = off[i];
        const int X = vx * P + (o & 255) - 64, Y = vy * P + ((o >> 8) & 255) - 64, Z = vz * P + ((o >> 16) & 255) - 64;
        const bool in = X >= 0 && X < L.Nx && Y >= 0 && Y < L.Ny && Z >= 0 && Z < L.Nz;
        if (in && !lat_dirichlet(L, X, Y, Z)) {
          const long g = lat_index(L, X, Y, Z);
#pragma unroll
          for (int r = 0; r < NV; ++r) rhs[j][r] = V.rt[r][g];
        }
        dia[j] = f[i];
      }
    }
    // the next slot's real rows (while this slot's right-hand sides are in flight)
    const unsigned nmask = real_row_mask<T, P>(L, off, erow, lane, slot_pos(L, sl + step));
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int i = lane + 64 * j;
      if (i < NR) {
#pragma unroll
        for (int r = 0; r < NV; ++r) xw[i * NV + r] = (double)rhs[j][r];
        iw[i] = 1.0 / (double)dia[j];
      }
    }
    if (lane == 0) {  // the dummy row
#pragma unroll
      for (int r = 0; r < NV; ++r) xw[NR * NV + r] = 0.0;
      iw[NR] = 0.0;
    }
    {
      PassIdx<S::K[0], NV> q;
      read_idx<P, NV, 0>(q, ecol, erow, lane);
#pragma unroll
      for (int r = 0; r < NV; ++r) q.b[r] = xw[q.row * NV + r];
      q.d = iw[q.row];
      fwd_passes<T, P, NV, 0>(v, xw, iw, ecol, erow, lane, q);
    }
    {
      PassIdx<S::K[NP - 1], NV> q;
      read_idx<P, NV, NP - 1>(q, ecol, erow, lane);
      q.d = iw[q.row];
      bwd_passes<T, P, NV, NP - 1>(v, xw, iw, ecol, erow, lane, q, slot_rsrc(sl + step), nmask);
    }
#pragma unroll
    for (int r = 0; r < NV; ++r) {
      T *zo = V.zb[r] + sl * (long)NR;
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        const int i = lane + 64 * j;
        if (i < NR) zo[i] = (T)xw[i * NV + r];
      }
    }
  }
}

// ------------------------------------------------------------------------------------
// Relaxation step 3: z_G = sum over the vertex patches containing the DoF (ascending
// vertex id) of the patch solutions; Dirichlet rows copy r.
// Step 4 (harmonic extension, R_Gamma^T): z_I = P_II^{-1} (r_I - P_IG z_G).
// ------------------------------------------------------------------------------------
// Sum of the patch solutions at plane point C (ascending vertex id).
template <int P, typename T>
__device__ __forceinline__ T patch_sum(const LatDev &L, const int C[3], const T *zbuf) {
  constexpr int NR = 1 + 6 * (P - 1) + 12 * (P - 1) * (P - 1);
  // the point's vertices: lo, and lo + 1 along the axes where the point is off the
  // vertex planes; the (up to 8) loads are issued together, then summed in
  // ascending vertex id (absent vertices add zero)
  int lo[3];
  bool two[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = C[d] / P;
    two[d] = C[d] % P != 0;
  }
  const int nvx = L.nx + 1, nvy = L.ny + 1;
  T val[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int ix = c & 1, iy = (c >> 1) & 1, iz = c >> 2;
    val[c] = T(0);
    if ((ix == 0 || two[0]) && (iy == 0 || two[1]) && (iz == 0 || two[2])) {
      const int vx = lo[0] + ix, vy = lo[1] + iy, vz = lo[2] + iz;
      const int k = patch_local_index(P, C[0] - vx * P, C[1] - vy * P, C[2] - vz * P);
      val[c] = zbuf[(vx + (long)nvx * (vy + (long)nvy * vz)) * NR + k];
    }
  }
  T acc = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) acc += val[c];
  return acc;
}

// Output of the expansion: z = scale * (M r) (plane values stored scaled; the
// interior solve is linear in (r, z_G), so it takes scale * r against them), and,
// when acc is given, acc += w * (M r) at every point (then scale is 1 and only the
// plane values of z, needed by the interior solve, are written).
template <typename T>
struct ExpandOut {
  T scale, w;
  T *acc;
};

// Step 3 on the rows of the y- and z-vertex planes (every point a plane point).
template <int P, typename T>
__device__ void expand_xface(const LatDev &L, const T *__restrict__ r, const T *__restrict__ zbuf, T *__restrict__ z,
                             const ExpandOut<T> &o, long t, long n);

template <int P, typename T>
__global__ void __launch_bounds__(256) k_expand_plane_rows(LatDev L, const T *__restrict__ r,
                                                           const T *__restrict__ zbuf, T *__restrict__ z,
                                                           ExpandOut<T> o, long nplane, long nxf) {
  if (blockIdx.x >= nplane) {  // the x-face points of the other rows, one lane each
    expand_xface<P, T>(L, r, zbuf, z, o, (blockIdx.x - nplane) * (long)blockDim.x + threadIdx.x, nxf);
    return;
  }
  int Y, Z;
  plane_row<P>(L, xcd_block(blockIdx.x, nplane), Y, Z);
  const long row = (long)L.Nx * (Y + (long)L.Ny * Z);
  for (int X = threadIdx.x; X < L.Nx; X += blockDim.x) {
    const int C[3] = {X, Y, Z};
    const T v = o.scale * (lat_dirichlet(L, X, Y, Z) ? r[row + X] : patch_sum<P, T>(L, C, zbuf));
    z[row + X] = v;
    if (o.acc) o.acc[row + X] += o.w * v;
  }
}

// Step 3 on the x-face points of the rows inside the cells' y-z cross sections,
// one lane per point (nx + 1 per row); run by the blocks appended to the
// k_expand_plane_rows launch.
template <int P, typename T>
__device__ void expand_xface(const LatDev &L, const T *__restrict__ r, const T *__restrict__ zbuf, T *__restrict__ z,
                             const ExpandOut<T> &o, long t, long n) {
  if (t >= n) return;
  const int k = t % (L.nx + 1);
  int Y, Z;
  interior_row<P>(L, t / (L.nx + 1), Y, Z);
  const int C[3] = {k * P, Y, Z};
  const long g = lat_index(L, C[0], Y, Z);
  const T v = o.scale * (lat_dirichlet_axis(L, 0, C[0]) ? r[g] : patch_sum<P, T>(L, C, zbuf));
  z[g] = v;
  if (o.acc) o.acc[g] += o.w * v;
}

// Step 4 on the rows inside a cell's y-z cross section: every interior point
//   z_I = (r_I - sum_d sigma_d (A_{l,0} z_lo + A_{l,P} z_hi)) / dd
// with z_lo, z_hi the plane values at the ends of its line along axis d (written by
// k_expand_plane_rows, x-face points included; Dirichlet ends count as 0).
template <int P, typename T>
__global__ void __launch_bounds__(256) k_expand_interior_rows(LatDev L, const T *__restrict__ coef,
                                                              const T *__restrict__ Ag, const T *__restrict__ lam,
                                                              const T *__restrict__ r, T *__restrict__ z,
                                                              ExpandOut<T> o) {
  // block: the P - 1 interior rows Y = cy P + ly (ly = 1 .. P - 1) of one y-layer of
  // cells at one interior z-coordinate Z; a thread takes one x for all of them, so
  // the y-face values at the layer's two ends and the cell weights are loaded once,
  // and every load of the thread's P - 1 points is in flight before the first sum
  constexpr int N1 = P + 1;
  const long b = xcd_block(blockIdx.x, gridDim.x);
  const int cy = b % L.ny;
  constexpr int PI = P > 1 ? P - 1 : 1;  // interior coordinates per cell (P = 1 has none)
  const int iz = b / L.ny, cz = iz / PI, lz = 1 + iz % PI, Z = cz * P + lz;
  const long sy = L.Nx, sz = (long)L.Nx * L.Ny;
  const long base = sy * ((long)cy * P + (long)L.Ny * Z);  // lattice row Y = cy P
  const long cyz = (long)L.nx * (cy + (long)L.ny * cz);
  const bool dyl = lat_dirichlet_axis(L, 1, cy * P), dyh = lat_dirichlet_axis(L, 1, cy * P + P);
  const bool dzl = lat_dirichlet_axis(L, 2, cz * P), dzh = lat_dirichlet_axis(L, 2, cz * P + P);
  const T a0z = Ag[lz * N1], aPz = Ag[lz * N1 + P], lmz = lam[lz];
  // the x-dependent table entries (A_{lx,0}, A_{lx,P}, lambda_lx) in LDS
  __shared__ T tx[3 * N1];
  for (int i = threadIdx.x; i < N1; i += blockDim.x) {
    tx[3 * i] = Ag[i * N1];
    tx[3 * i + 1] = Ag[i * N1 + P];
    tx[3 * i + 2] = lam[i];
  }
  __syncthreads();
  for (int X = threadIdx.x; X < L.Nx; X += blockDim.x) {
    const int cx = X / P, lx = X % P;
    if (lx == 0) continue;  // x-face point, written by the previous launch
    const T *cf = coef + 6 * (cx + cyz);
    const bool dxl = lat_dirichlet_axis(L, 0, cx * P), dxh = lat_dirichlet_axis(L, 0, cx * P + P);
    const long g0 = base + X;
    const T c0 = cf[0], c1 = cf[1], c2 = cf[2], c3 = cf[3];
    const T zly = dyl ? T(0) : z[g0];
    const T zhy = dyh ? T(0) : z[g0 + P * sy];
    constexpr int NI = P > 1 ? P - 1 : 1;
    T rv[NI], av[NI], zlx[NI], zhx[NI], zlz[NI], zhz[NI];
#pragma unroll
    for (int k = 0; k < P - 1; ++k) {
      const long g = g0 + (k + 1) * sy;
      rv[k] = r[g];
      av[k] = o.acc ? o.acc[g] : T(0);
      zlx[k] = dxl ? T(0) : z[g - lx];
      zhx[k] = dxh ? T(0) : z[g + (P - lx)];
      zlz[k] = dzl ? T(0) : z[g - (long)lz * sz];
      zhz[k] = dzh ? T(0) : z[g + (long)(P - lz) * sz];
    }
    const T a0x = tx[3 * lx], aPx = tx[3 * lx + 1], lmx = tx[3 * lx + 2];
#pragma unroll
    for (int k = 0; k < P - 1; ++k) {
      const int ly = k + 1;
      const long g = g0 + ly * sy;
      T dd = c3;
      T val = o.scale * rv[k];
      dd += c0 * lmx;
      val -= c0 * (a0x * zlx[k] + aPx * zhx[k]);
      dd += c1 * lam[ly];
      val -= c1 * (Ag[ly * N1] * zly + Ag[ly * N1 + P] * zhy);
      dd += c2 * lmz;
      val -= c2 * (a0z * zlz[k] + aPz * zhz[k]);
      if (o.acc) o.acc[g] = av[k] + o.w * (val / dd);
      else z[g] = val / dd;
    }
  }
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

// The paper's auxiliary (eq. sum-factorization_approx) on one cell from its broken
// diagonals: P_K(u, w) = sum over broken indices of dm Gbar Gbar (x3) + sum_m sum_r
// D[r][u_m] D[r][w_m] da_m (Gbar Gbar along the other two axes).  Gbar is the
// identity on interior indices and mixes the two end functions, so along an axis
// the broken indices are u_d (interior, w_d = u_d) or both ends (u_d and w_d ends);
// along the DP axis of component m the row r is u_m or w_m where one is interior,
// every row when both are ends.
struct PdCell {
  const double *dm, *da;  // this cell's (p+1)^3 and 3 p (p+1)^2 diagonals
  const double *G, *D;    // (p+1)^2 broken transformation, p x (p+1) D-hat
};

// broken indices along one axis for local coordinates (a, b) and their G G factors
__device__ __forceinline__ int pd_axis(int p, const double *G, int a, int b, int idx[2], double f[2]) {
  const int n1 = p + 1;
  if (!on_end(p, a) || !on_end(p, b)) {
    if (a != b) return 0;
    idx[0] = a;
    f[0] = 1.0;
    return 1;
  }
  idx[0] = 0;
  f[0] = G[a] * G[b];
  idx[1] = p;
  f[1] = G[p * n1 + a] * G[p * n1 + b];
  return 2;
}

__device__ double pd_entry(int p, const PdCell &C, const int u[3], const int w[3]) {
  const int n1 = p + 1;
  int ix[3][2];
  double fx[3][2];
  int nb[3];
  for (int d = 0; d < 3; ++d) nb[d] = pd_axis(p, C.G, u[d], w[d], ix[d], fx[d]);
  double v = 0.0;
  if (nb[0] && nb[1] && nb[2])
    for (int c = 0; c < nb[2]; ++c)
      for (int b = 0; b < nb[1]; ++b)
        for (int a = 0; a < nb[0]; ++a)
          v += C.dm[ix[0][a] + n1 * (ix[1][b] + n1 * ix[2][c])] * fx[0][a] * fx[1][b] * fx[2][c];
  const long nc = (long)p * n1 * n1;
  for (int m = 0; m < 3; ++m) {
    const int e1 = (m + 1) % 3, e2 = (m + 2) % 3;
    if (!nb[e1] || !nb[e2]) continue;
    int r0, r1;
    if (!on_end(p, u[m])) {
      r0 = r1 = u[m];
    } else if (!on_end(p, w[m])) {
      r0 = r1 = w[m];
    } else {
      r0 = 0;
      r1 = p - 1;
    }
    const double *da = C.da + m * nc;
    for (int r = r0; r <= r1; ++r) {
      const double dd = C.D[r * n1 + u[m]] * C.D[r * n1 + w[m]];
      if (dd == 0.0) continue;
      for (int b2 = 0; b2 < nb[e2]; ++b2)
        for (int b1 = 0; b1 < nb[e1]; ++b1) {
          int t[3];
          t[m] = r;
          t[e1] = ix[e1][b1];
          t[e2] = ix[e2][b2];
          // component m: extent p along m, p + 1 along the others, x fastest
          const int ex = m == 0 ? p : n1, ey = m == 1 ? p : n1;
          v += da[t[0] + ex * (t[1] + ey * t[2])] * dd * fx[e1][b1] * fx[e2][b2];
        }
    }
  }
  return v;
}

// one cell's Schur-complement entry of interface DoFs u, w (cell_schur_value with
// the paper's auxiliary): P_GG(u, w) minus the interior DoFs coupled to both
__device__ double pd_cell_schur(int p, const PdCell &C, const int u[3], const int w[3]) {
  double v = pd_entry(p, C, u, w);
  if (p < 2) return v;
  int nu = on_end(p, u[0]) + on_end(p, u[1]) + on_end(p, u[2]);
  int nw = on_end(p, w[0]) + on_end(p, w[1]) + on_end(p, w[2]);
  if (nu != 1 || nw != 1) return v;
  int du = on_end(p, u[0]) ? 0 : (on_end(p, u[1]) ? 1 : 2);
  int dw = on_end(p, w[0]) ? 0 : (on_end(p, w[1]) ? 1 : 2);
  if (du == dw) {
    for (int e = 0; e < 3; ++e)
      if (e != du && u[e] != w[e]) return v;
    for (int i = 1; i < p; ++i) {
      int t[3] = {u[0], u[1], u[2]};
      t[du] = i;
      v -= pd_entry(p, C, u, t) * pd_entry(p, C, t, w) / pd_entry(p, C, t, t);
    }
    return v;
  }
  int e = 3 - du - dw;
  if (u[e] != w[e]) return v;
  int t[3];
  t[du] = w[du];
  t[dw] = u[dw];
  t[e] = u[e];
  return v - pd_entry(p, C, u, t) * pd_entry(p, C, t, w) / pd_entry(p, C, t, t);
}

__global__ void __launch_bounds__(256) k_patch_factor(LatDev L, PatchDev P, const int *__restrict__ erow,
                                                       const double *__restrict__ coef,
                                                       const double *__restrict__ Bg, const double *__restrict__ Ag,
                                                       const double *__restrict__ lamg, PdDev pd,
                                                       double *__restrict__ f64, float *__restrict__ f32,
                                                       int *status, int ic) {
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
        if (pd.dm) {
          const PdCell C{pd.dm + (long)cid * n1 * n1 * n1, pd.da + (long)cid * 3 * p * n1 * n1, pd.G, pd.D};
          val += pd_cell_schur(p, C, u, w);
        } else {
          double s[3] = {coef[6 * cid], coef[6 * cid + 1], coef[6 * cid + 2]};
          val += cell_schur_value(p, sB, sA, sl, s, coef[6 * cid + 3], u, w);
        }
      }
    }
    S[k] = ok ? val : 0.0;
    allowed[k] = ok ? 1 : 0;
  }
  __syncthreads();
  // ic = 0: store the assembled S_v on its pattern, unfactored
  for (int lv = 0; ic && lv < P.nflev; ++lv) {
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
  double *o64 = f64 + vid * (long)P.stride;
  float *o32 = f32 + vid * (long)P.stride;
  for (int k = threadIdx.x; k < P.nnz; k += blockDim.x) {
    const int q = P.perm[k], q2 = P.perm2[k];
    o64[q] = S[k];
    o32[q] = (float)S[k];
    if (q2 >= 0) {
      o64[q2] = S[k];
      o32[q2] = (float)S[k];
    }
  }
}

// ------------------------------------------------------------------------------------
// p-transfer: the embedding of Q_1 in Q_p in FDM coefficients is the Kronecker
// product of the (p+1)x2 hat matrix E per axis; restriction is its transpose.
// ------------------------------------------------------------------------------------
// One block per lattice row (Y, Z), lanes along x.  The y and z weights are
// uniform over the row, so the block first combines the four coarse x-lines
// around the row into one line in LDS (coarse Dirichlet vertices excluded); each
// fine point then interpolates between two entries of that line.
template <int P>
__global__ void __launch_bounds__(256) k_prolong_add_p(LatDev L, const double *__restrict__ E,
                                                       const double *__restrict__ xc, double *__restrict__ xf) {
  extern __shared__ double cl[];
  const int Y = blockIdx.x % L.Ny, Z = blockIdx.x / L.Ny;
  const int cy = min(Y / P, L.ny - 1), cz = min(Z / P, L.nz - 1);
  const int ay = Y - cy * P, az = Z - cz * P;
  const double wy[2] = {((L.dir & 4u) && cy == 0) ? 0.0 : E[2 * ay],
                        ((L.dir & 8u) && cy + 1 == L.ny) ? 0.0 : E[2 * ay + 1]};
  const double wz[2] = {((L.dir & 16u) && cz == 0) ? 0.0 : E[2 * az],
                        ((L.dir & 32u) && cz + 1 == L.nz) ? 0.0 : E[2 * az + 1]};
  const long sy = L.nx + 1, sz = sy * (L.ny + 1);
  const double *q = xc + sy * cy + sz * cz;
  for (int v = threadIdx.x; v <= L.nx; v += blockDim.x) {
    const bool dv = ((L.dir & 1u) && v == 0) || ((L.dir & 2u) && v == L.nx);
    const double a0 = (wy[0] != 0.0 ? wy[0] * q[v] : 0.0) + (wy[1] != 0.0 ? wy[1] * q[v + sy] : 0.0);
    const double a1 = (wy[0] != 0.0 ? wy[0] * q[v + sz] : 0.0) + (wy[1] != 0.0 ? wy[1] * q[v + sz + sy] : 0.0);
    cl[v] = dv ? 0.0 : (wz[0] != 0.0 ? wz[0] * a0 : 0.0) + (wz[1] != 0.0 ? wz[1] * a1 : 0.0);
  }
  __syncthreads();
  const long row = (long)L.Nx * blockIdx.x;
  const bool rowdir = lat_dirichlet_axis(L, 1, Y) || lat_dirichlet_axis(L, 2, Z);
  if (rowdir) return;
  for (int X = threadIdx.x; X < L.Nx; X += blockDim.x) {
    if (lat_dirichlet_axis(L, 0, X)) continue;
    const int cx = min(X / P, L.nx - 1), ax = X - cx * P;
    xf[row + X] += E[2 * ax] * cl[cx] + E[2 * ax + 1] * cl[cx + 1];
  }
}

// Coarse correction and the residual after it, in one pass per lattice row:
//   z += P xc,   r -= A P xc   (r holds r - A z_old on entry, r - A z_new on exit).
// P xc is trilinear in each cell, so (A P xc)_K = s1 (AE x BE x BE) c + s2 (BE x AE x BE) c
// + s3 (BE x BE x AE) c + mu (BE x BE x BE) c with c the cell's 8 coarse corner
// values and AE = A E, BE = B E the (p+1) x 2 products of the 1-D tables with the
// hat embedding E (cellwise-constant weights on Cartesian cells).  Coarse Dirichlet
// vertices count as 0, which also makes P xc vanish on fine Dirichlet points; fine
// Dirichlet rows keep z and r.  The block stages the (up to 9) coarse x-lines around
// the row and the weights of the row's cells in LDS.
template <int P, typename TV>
__global__ void __launch_bounds__(256) k_prolong_residual_p(LatDev L, const double *__restrict__ E,
                                                            const double *__restrict__ T2, const double *__restrict__ coef,
                                                            const double *__restrict__ xc, TV *__restrict__ z,
                                                            TV *__restrict__ r) {
  // block: the lattice rows Y = cy P .. cy P + P - 1 (and Y = ny P in the last layer)
  // of one z-coordinate Z; they share the coarse lines at vertices cy - 1 .. cy + 1
  // along y and the weights of the cells cy - 1, cy
  extern __shared__ double sm[];
  const int nv = L.nx + 1;
  double *lines = sm;                 // [3 (vy = cy-1+d)][3 (vz = vz0+d)][nv]
  double *cw = lines + 9 * nv;        // [2 (cy-1, cy)][2 (z cells)][nx][4]
  double *tb = cw + 16 * L.nx;        // [2][P+1][2]: AE, BE
  const int cy = blockIdx.x % L.ny, Z = blockIdx.x / L.ny;
  // the cells containing the coordinate along one axis: (cell, local coordinate)
  // for up to two cells, written without run-time array indices (registers)
  auto cells_of = [](int C, int nc, int (&cv)[2], int (&bv)[2]) {
    const int c = C / P;
    if (C % P != 0) {
      cv[0] = cv[1] = c;
      bv[0] = bv[1] = C % P;
      return 1;
    }
    const bool below = c > 0, above = c < nc;
    cv[0] = below ? c - 1 : c;
    bv[0] = below ? P : 0;
    cv[1] = c;
    bv[1] = 0;
    return (below ? 1 : 0) + (above && below ? 1 : 0) + (!below && above ? 1 : 0);
  };
  int czv[2], bzv[2];
  const int nz = cells_of(Z, L.nz, czv, bzv);
  const int vz0 = czv[0];
  const long sy = nv, sz = (long)nv * (L.ny + 1);
  // staging of lines, cw and tb (contiguous in LDS) as one index range, four
  // entries per thread per round with their loads in flight together
  const int n_ln = 9 * nv, n_cw = 16 * L.nx, n_st = n_ln + n_cw + 4 * (P + 1);
  auto stage_value = [&](int t) -> double {
    if (t < n_ln) {
      const int v = t % nv, d = t / nv, vy = cy - 1 + d % 3, vz = vz0 + d / 3;
      if (vy < 0 || vy > L.ny || vz > L.nz) return 0.0;
      const bool dir = ((L.dir & 1u) && v == 0) || ((L.dir & 2u) && v == L.nx) || ((L.dir & 4u) && vy == 0) ||
                       ((L.dir & 8u) && vy == L.ny) || ((L.dir & 16u) && vz == 0) || ((L.dir & 32u) && vz == L.nz);
      return dir ? 0.0 : xc[v + sy * vy + sz * vz];
    }
    if (t < n_ln + n_cw) {
      const int u = t - n_ln;
      const int q = u % 4, cx = (u / 4) % L.nx, iy = (u / (4 * L.nx)) % 2, iz = u / (8 * L.nx);
      const int ccy = cy - 1 + iy;
      return (ccy >= 0 && iz < nz) ? coef[6 * (cx + (long)L.nx * (ccy + (long)L.ny * (iz ? czv[1] : czv[0]))) + q]
                                   : 0.0;
    }
    return T2[t - n_ln - n_cw];
  };
  for (int t0 = threadIdx.x; t0 < n_st; t0 += 4 * blockDim.x) {
    double sv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int t = t0 + k * blockDim.x;
      sv[k] = t < n_st ? stage_value(t) : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int t = t0 + k * blockDim.x;
      if (t < n_st) sm[t] = sv[k];
    }
  }
  __syncthreads();
  if (lat_dirichlet_axis(L, 2, Z)) return;
  const double *AE = tb, *BE = tb + 2 * (P + 1);
  const int pz = min(Z / P, L.nz - 1), az = Z - pz * P;
  const double wz[2] = {E[2 * az], E[2 * az + 1]};
  const int nrow = cy + 1 == L.ny ? P + 1 : P;
  // four points per thread per round: their z and r loads first, then the sums
  const int npt = nrow * L.Nx;
  for (int t0 = threadIdx.x; t0 < npt; t0 += 4 * blockDim.x) {
    double zv[4], rv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int t = t0 + k * blockDim.x;
      zv[k] = rv[k] = 0.0;
      if (t < npt) {
        const long g = (long)(t % L.Nx) + (long)L.Nx * (cy * P + t / L.Nx + (long)L.Ny * Z);
        zv[k] = (double)z[g];
        rv[k] = (double)r[g];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
    const int t = t0 + k * blockDim.x;
    if (t >= npt) continue;
    const int X = t % L.Nx, Y = cy * P + t / L.Nx;
    if (lat_dirichlet_axis(L, 0, X) || lat_dirichlet_axis(L, 1, Y)) continue;
    // the cells containing the point along y (index into the staged cells: cy - 1 + iy)
    int iyv[2], byv[2];
    const int ny = cells_of(Y, L.ny, iyv, byv);
    iyv[0] -= cy - 1;
    iyv[1] -= cy - 1;
    // z += P xc (cell cy along y, the last cell for the last vertex plane)
    const int ay = Y - cy * P;
    const int px = min(X / P, L.nx - 1), ax = X - px * P;
    double pacc = 0.0;
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const double *ln = lines + nv * ((1 + j) + 3 * (pz + k - vz0));
        pacc += wz[k] * E[2 * ay + j] * (E[2 * ax] * ln[px] + E[2 * ax + 1] * ln[px + 1]);
      }
    // r -= A P xc, summed over the cells containing the point
    int cxv[2], bxv[2];
    const int nx = cells_of(X, L.nx, cxv, bxv);
    double acc = 0.0;
    // fixed trip counts with guards, so that the short index arrays stay in registers
#pragma unroll
    for (int iz = 0; iz < 2; ++iz)
#pragma unroll
      for (int i2 = 0; i2 < 2; ++i2) {
        if (iz >= nz || i2 >= ny) continue;
        const int iy = iyv[i2], b = byv[i2];
        const double By[2] = {BE[2 * b], BE[2 * b + 1]}, Ay[2] = {AE[2 * b], AE[2 * b + 1]};
        const double Bz[2] = {BE[2 * bzv[iz]], BE[2 * bzv[iz] + 1]}, Az[2] = {AE[2 * bzv[iz]], AE[2 * bzv[iz] + 1]};
#pragma unroll
        for (int ix = 0; ix < 2; ++ix) {
          if (ix >= nx) continue;
          const int cx = cxv[ix], a = bxv[ix];
          const double *s = cw + 4 * (cx + L.nx * (iy + 2 * iz));
          const double Ax0 = AE[2 * a], Ax1 = AE[2 * a + 1], Bx0 = BE[2 * a], Bx1 = BE[2 * a + 1];
#pragma unroll
          for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
              // cell (cy - 1 + iy) spans the vertex lines iy + j (= vy - (cy - 1))
              const double *ln = lines + nv * ((iy + j) + 3 * (czv[iz] + k - vz0));
              const double c0 = ln[cx], c1 = ln[cx + 1];
              const double ax_ = Ax0 * c0 + Ax1 * c1, bx_ = Bx0 * c0 + Bx1 * c1;
              acc += s[0] * ax_ * By[j] * Bz[k] + bx_ * (s[1] * Ay[j] * Bz[k] + s[2] * By[j] * Az[k] + s[3] * By[j] * Bz[k]);
            }
        }
      }
    const long g = (long)X + (long)L.Nx * (Y + (long)L.Ny * Z);
    z[g] = (TV)(zv[k] + pacc);
    r[g] = (TV)(rv[k] - acc);
    }
  }
}

// Restriction rc = P^T rf as three 1-D passes (x, then y, then z); the weight of a
// fine coordinate X for coarse vertex V is E[X - (V-1)p][1] left of V p, 1 at V p,
// E[X - V p][0] right of it.  Fine Dirichlet entries are read as zero, coarse
// Dirichlet outputs are zero.
__device__ __forceinline__ double hat_weight(const double *E, int p, int off) {
  return off < 0 ? E[2 * (off + p) + 1] : (off > 0 ? E[2 * off] : 1.0);
}

// x pass: R lattice rows per block (64 lanes each), each row staged in LDS with
// its Dirichlet entries zeroed, then one lane per coarse vertex sums its 2P - 1
// fine neighbours (weights uniform over the lanes).
template <int P>
__global__ void __launch_bounds__(256) k_restrict_x_p(LatDev L, const double *__restrict__ E,
                                                      const double *__restrict__ rf, double *__restrict__ t1,
                                                      long nrows) {
  extern __shared__ double srow[];
  const int R = blockDim.x >> 6, r = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long row = (long)blockIdx.x * R + r;
  const bool active = row < nrows;
  const int Y = active ? row % L.Ny : 0, Z = active ? row / L.Ny : 0;
  const bool rowdir = lat_dirichlet_axis(L, 1, Y) || lat_dirichlet_axis(L, 2, Z);
  double *s = srow + (size_t)r * L.Nx;
  for (int X = lane; X < L.Nx; X += 64)
    s[X] = (active && !rowdir && !lat_dirichlet_axis(L, 0, X)) ? rf[X + (long)L.Nx * row] : 0.0;
  __syncthreads();
  if (!active) return;
  for (int V = lane; V <= L.nx; V += 64) {
    double acc = 0.0;
#pragma unroll
    for (int o = -(P - 1); o <= P - 1; ++o) {
      const int X = V * P + o;
      const double wt = o < 0 ? E[2 * (o + P) + 1] : (o > 0 ? E[2 * o] : 1.0);
      if (X >= 0 && X < L.Nx) acc += wt * s[X];
    }
    t1[V + (long)(L.nx + 1) * row] = acc;
  }
}

// x pass for rows too long to stage in LDS: one thread per (coarse vertex, row)
__global__ void k_restrict_x(LatDev L, const double *__restrict__ E, const double *__restrict__ rf,
                             double *__restrict__ t1, long n) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p = L.p, NCX = L.nx + 1;
  const int VX = i % NCX;
  const long yz = i / NCX;
  const int Y = yz % L.Ny, Z = yz / L.Ny;
  const int lo = max(0, VX * p - (p - 1)), hi = min(L.Nx - 1, VX * p + (p - 1));
  double acc = 0.0;
  for (int X = lo; X <= hi; ++X)
    if (!lat_dirichlet(L, X, Y, Z)) acc += hat_weight(E, p, X - VX * p) * rf[X + (long)L.Nx * yz];
  t1[i] = acc;
}

// y and z passes: the 2P - 1 taps of a coarse vertex as one unrolled body (loads of
// all taps in flight together), summed in ascending fine coordinate; taps outside the
// lattice add zero
template <int P>
__global__ void k_restrict_y(LatDev L, const double *__restrict__ E, const double *__restrict__ t1,
                             double *__restrict__ t2, long n) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int NCX = L.nx + 1, NCY = L.ny + 1;
  const int VX = i % NCX, VY = (i / NCX) % NCY;
  const int Z = i / ((long)NCX * NCY);
  double v[2 * P - 1];
#pragma unroll
  for (int o = -(P - 1); o <= P - 1; ++o) {
    const int Y = VY * P + o;
    v[o + P - 1] = Y >= 0 && Y < L.Ny ? t1[VX + (long)NCX * (Y + (long)L.Ny * Z)] : 0.0;
  }
  double acc = 0.0;
#pragma unroll
  for (int o = -(P - 1); o <= P - 1; ++o) acc += hat_weight(E, P, o) * v[o + P - 1];
  t2[i] = acc;
}

template <int P>
__global__ void k_restrict_z(LatDev L, const double *__restrict__ E, const double *__restrict__ t2,
                             double *__restrict__ rc, long n) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int NC[3] = {L.nx + 1, L.ny + 1, L.nz + 1};
  const int VX = i % NC[0], VY = (i / NC[0]) % NC[1], VZ = i / ((long)NC[0] * NC[1]);
  const bool dir = ((L.dir & 1u) && VX == 0) || ((L.dir & 2u) && VX == NC[0] - 1) ||
                   ((L.dir & 4u) && VY == 0) || ((L.dir & 8u) && VY == NC[1] - 1) ||
                   ((L.dir & 16u) && VZ == 0) || ((L.dir & 32u) && VZ == NC[2] - 1);
  double v[2 * P - 1];
#pragma unroll
  for (int o = -(P - 1); o <= P - 1; ++o) {
    const int Z = VZ * P + o;
    v[o + P - 1] = !dir && Z >= 0 && Z < L.Nz ? t2[VX + (long)NC[0] * (VY + (long)NC[1] * Z)] : 0.0;
  }
  double acc = 0.0;
#pragma unroll
  for (int o = -(P - 1); o <= P - 1; ++o) acc += hat_weight(E, P, o) * v[o + P - 1];
  rc[i] = dir ? 0.0 : acc;
}

// Dirichlet rows only: the points of the six boundary faces of the lattice (face f:
// axis f / 2, side f % 2), one thread per face point; faces without a Dirichlet
// condition return at once.  Edge and corner points are visited by each of their
// faces and receive the same value.
template <typename T>
__global__ void k_dirichlet_copy(LatDev L, const T *__restrict__ r, T *__restrict__ z) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int f = blockIdx.y;
  if (!(L.dir & (1u << f))) return;
  const int a = f >> 1, b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
  const int Nd[3] = {L.Nx, L.Ny, L.Nz};
  if (t >= (long)Nd[b] * Nd[c]) return;
  int C[3];
  C[a] = (f & 1) ? Nd[a] - 1 : 0;
  C[b] = t % Nd[b];
  C[c] = t / Nd[b];
  const long g = lat_index(L, C[0], C[1], C[2]);
  z[g] = r ? r[g] : T(0);
}

inline unsigned nblocks(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------
#define RZ_DISPATCH_P(p, call) \
  switch (p) {                 \
    case 1: call(1); break;    \
    case 2: call(2); break;    \
    case 3: call(3); break;    \
    case 4: call(4); break;    \
    case 5: call(5); break;    \
    case 6: call(6); break;    \
    case 7: call(7); break;    \
    case 8: call(8); break;    \
    case 9: call(9); break;    \
    default: break;            \
  }

template <int P, typename T, typename S = T>
static void apply_pencil(const LatDev &L, const T *coef, const double *Bh, const double *Ah, const S *x,
                         const S *bsub, S *y, T *fb, hipStream_t s) {
  constexpr int NL = (P + 1) * (P + 1);
  // cells per chunk: 512 threads for P = 6, 7 (fewer, larger chunks per row of cells;
  // two blocks per CU), 256 otherwise
  constexpr int CPC = (P == 6 || P == 7) ? 512 / NL : (NL >= 256 ? 1 : 256 / NL);
  constexpr int N1 = P + 1, CS = (N1 + 1) * N1 * N1 + 8;
  const size_t shm = (2 * (size_t)CPC * CS + 2 * NL) * sizeof(T);
  if (shm > 64 * 1024)
    hipFuncSetAttribute((const void *)k_apply_pencil<P, T, CPC, S>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)shm);
  Tab1D<P, T> tb;
  for (int i = 0; i < (P + 1) * (P + 1); ++i) {
    tb.B[i] = (T)Bh[i];
    tb.A[i] = (T)Ah[i];
  }
  k_apply_pencil<P, T, CPC, S><<<(unsigned)(L.ny * L.nz), CPC * NL, shm, s>>>(L, tb, coef, x, bsub, y, fb);
  const long nlines = (long)(L.ny + 1) * L.Nz + (long)(L.nz + 1) * (L.Ny - L.ny - 1);
  const long n = nlines * L.Nx;
  k_apply_faces<P, T, S><<<nblocks(n, 256), 256, 0, s>>>(L, x, fb, bsub, y, n);
}

template <typename T>
void launch_apply_grad(const LatDev &L, const T *coef, const double *Bh, const double *Ah, const T *x,
                       const T *bsub, T *y, T *fbuf, hipStream_t s) {
#define RZ_CALL(Q) apply_pencil<Q, T>(L, coef, Bh, Ah, x, bsub, y, fbuf, s)
  RZ_DISPATCH_P(L.p, RZ_CALL)
#undef RZ_CALL
}

// BF16 vectors: FP32 weights, arithmetic and face-line buffer
void launch_apply_grad_bf16(const LatDev &L, const float *coef, const double *Bh, const double *Ah, const bf16_t *x,
                            bf16_t *y, float *fbuf, hipStream_t s) {
#define RZ_CALL(Q) apply_pencil<Q, float, bf16_t>(L, coef, Bh, Ah, x, nullptr, y, fbuf, s)
  RZ_DISPATCH_P(L.p, RZ_CALL)
#undef RZ_CALL
}

template <typename T>
void launch_apply_gather(const LatDev &L, const T *x, const T *ebuf, T *y, hipStream_t s, const T *bsub) {
  long n = (long)L.Nx * L.Ny * L.Nz;
  k_apply_gather<T, T><<<nblocks(n, 256), 256, 0, s>>>(L, x, ebuf, y, n, bsub);
}

// BF16 vectors, FP32 per-cell buffer (the matrix-core apply)
void launch_apply_gather_bf16(const LatDev &L, const bf16_t *x, const float *ebuf, bf16_t *y, hipStream_t s) {
  long n = (long)L.Nx * L.Ny * L.Nz;
  k_apply_gather<bf16_t, float><<<nblocks(n, 256), 256, 0, s>>>(L, x, ebuf, y, n, nullptr);
}

template <int P, typename T>
static void condense_p(const LatDev &L, const T *coef, const T *A, const T *lam, const T *r, T *rt, hipStream_t s) {
  const long np = (long)(L.ny + 1) * L.Nz + (long)(L.nz + 1) * (L.Ny - L.ny - 1);
  const long ni = (long)L.ny * (P - 1) * L.nz * (P - 1);
  const int bs = L.Nx >= 256 ? 256 : ((L.Nx + 63) / 64) * 64;
  const long nxf = ni * (L.nx + 1);
  const long nb = np + (long)nblocks(nxf, bs);
  k_condense_rows<P, T><<<(unsigned)nb, bs, 8 * L.nx * sizeof(T), s>>>(L, coef, A, lam, r, rt, np, nxf);
}

template <int P, typename T>
static void expand_p(const LatDev &L, const T *coef, const T *A, const T *lam, const T *r, const T *zbuf, T *z,
                     ExpandOut<T> o, hipStream_t s) {
  const long np = (long)(L.ny + 1) * L.Nz + (long)(L.nz + 1) * (L.Ny - L.ny - 1);
  const long ni = (long)L.ny * (P - 1) * L.nz * (P - 1);
  const int bs = L.Nx >= 256 ? 256 : ((L.Nx + 63) / 64) * 64;
  const long nxf = ni * (L.nx + 1);
  k_expand_plane_rows<P, T><<<(unsigned)(np + (long)nblocks(nxf, bs)), bs, 0, s>>>(L, r, zbuf, z, o, np, nxf);
  if (ni > 0) k_expand_interior_rows<P, T><<<(unsigned)(ni / (P > 1 ? P - 1 : 1)), bs, 0, s>>>(L, coef, A, lam, r, z, o);
}

template <int P, typename T>
static void expand_plane_p(const LatDev &L, const T *r, const T *zbuf, T *z, ExpandOut<T> o, hipStream_t s) {
  const long np = (long)(L.ny + 1) * L.Nz + (long)(L.nz + 1) * (L.Ny - L.ny - 1);
  const long ni = (long)L.ny * (P - 1) * L.nz * (P - 1);
  const int bs = L.Nx >= 256 ? 256 : ((L.Nx + 63) / 64) * 64;
  const long nxf = ni * (L.nx + 1);
  k_expand_plane_rows<P, T><<<(unsigned)(np + (long)nblocks(nxf, bs)), bs, 0, s>>>(L, r, zbuf, z, o, np, nxf);
}

template <typename T>
void launch_expand_plane_grad(const LatDev &L, const T *r, const T *zbuf, T *z, T scale, T w, T *acc, hipStream_t s) {
  const ExpandOut<T> o{scale, w, acc};
#define RZ_CALL(Q) expand_plane_p<Q, T>(L, r, zbuf, z, o, s)
  RZ_DISPATCH_P(L.p, RZ_CALL)
#undef RZ_CALL
}
template void launch_expand_plane_grad<double>(const LatDev &, const double *, const double *, double *, double,
                                               double, double *, hipStream_t);
template void launch_expand_plane_grad<float>(const LatDev &, const float *, const float *, float *, float, float,
                                              float *, hipStream_t);

template <typename T>
void launch_condense_grad(const LatDev &L, const T *coef, const T *A, const T *lam, const T *r, T *rt,
                          hipStream_t s) {
#define RZ_CALL(P) condense_p<P, T>(L, coef, A, lam, r, rt, s)
  RZ_DISPATCH_P(L.p, RZ_CALL)
#undef RZ_CALL
}

int device_cu_count() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    if (cus <= 0) cus = 256;
  }
  return cus;
}

// LDS of a patch-solve block: per wavefront row_bytes per patch row, plus the shared
// schedule tables (row offsets, ELL columns, pass rows)
static size_t patch_solve_lds(const PatchEllDev &E, size_t row_bytes, int waves) {
  return (size_t)waves * E.nrows * row_bytes + 4 * (size_t)E.nrows + 2 * (size_t)E.ne + 2 * 64 * (size_t)E.npass;
}

size_t patch_solve_lds_bytes(const PatchEllDev &E, size_t elem, int waves) {
  return patch_solve_lds(E, 2 * elem, waves);
}

// wavefronts per block and blocks per CU for row_bytes of LDS per patch row: the
// block size with the most resident wavefronts per CU, at most cap (ties: larger
// blocks)
static bool patch_solve_shape(const PatchEllDev &E, size_t row_bytes, int cap, int &waves, int &per_cu) {
  constexpr size_t kLds = 160 * 1024;
  waves = per_cu = 0;
  int best = 0;
  for (int w = 16; w >= 1; --w) {
    const size_t need = patch_solve_lds(E, row_bytes, w);
    if (need > kLds) continue;
    int b = (int)(kLds / need);
    if (b * w > cap) b = cap / w;
    if (b * w > best) {
      best = b * w;
      waves = w;
      per_cu = b;
    }
  }
  return waves > 0;
}

bool patch_solve_stream_shape(const PatchEllDev &E, size_t elem, int cap, int &waves, int &per_cu) {
  return patch_solve_shape(E, sizeof(double) + elem, cap, waves, per_cu);
}

template <int P>
static bool pass_table_matches(const int *pass, int np, int nrows, int ne, int ell0) {
  using S = PassTable<P>;
  if (S::NP != np || S::NR != nrows || 64 * S::KT != ne || S::E0 != ell0) return false;
  for (int t = 0; t < np; ++t)
    if (pass[3 * t] != S::G[t] || pass[3 * t + 1] != S::K[t] || pass[3 * t + 2] != 64 * S::C[t]) return false;
  return true;
}

bool patch_regs_table_matches(int p, const int *pass, int np, int nrows, int ne, int ell0) {
  switch (p) {
    case 2: return pass_table_matches<2>(pass, np, nrows, ne, ell0);
    case 3: return pass_table_matches<3>(pass, np, nrows, ne, ell0);
    case 4: return pass_table_matches<4>(pass, np, nrows, ne, ell0);
    case 5: return pass_table_matches<5>(pass, np, nrows, ne, ell0);
    case 6: return pass_table_matches<6>(pass, np, nrows, ne, ell0);
    case 7: return pass_table_matches<7>(pass, np, nrows, ne, ell0);
    case 8: return pass_table_matches<8>(pass, np, nrows, ne, ell0);
    default: return false;
  }
}

// the register kernel: four wavefronts per block, as many blocks per CU as the
// registers (2 at p = 7 in FP64) and the LDS allow
template <typename T, int P, int NV>
static int launch_patch_solve_r(const LatDev &L, const PatchEllDev &E, const T *factor, const PatchVecs<T> &V,
                                hipStream_t s) {
  using S = PassTable<P>;
  constexpr int waves = 4;
  const long nv = (long)(L.nx + 1) * (L.ny + 1) * (L.nz + 1);
  const size_t shm = (size_t)waves * (NV + 1) * (S::NR + 1) * sizeof(double) + 4 * (size_t)S::NR +
                     2 * (size_t)E.ne + 2 * 64 * S::NP;
  // the LDS attribute on every launch (it belongs to the current device); the
  // occupancy once (one device type)
  if (hipFuncSetAttribute((const void *)k_patch_solve_r<T, P, NV>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)shm) != hipSuccess)
    return -1;
  static const int per_cu = [&] {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_patch_solve_r<T, P, NV>, 64 * waves, shm) != hipSuccess)
      b = 0;
    return b;
  }();
  if (per_cu <= 0) return -1;
  long grid = (long)device_cu_count() * per_cu;
  const long need = (nv + waves - 1) / waves;
  if (grid > need) grid = need;
  k_patch_solve_r<T, P, NV><<<(unsigned)grid, 64 * waves, shm, s>>>(L, E, factor, V, nv);
  return 0;
}

// one register-kernel launch over NV vectors (NV = 1, 2 or 4)
template <typename T, int NV>
static int launch_patch_solve_r_nv(const LatDev &L, const PatchEllDev &E, const T *factor, const PatchVecs<T> &V,
                                   hipStream_t s) {
  switch (L.p) {
    case 2: return launch_patch_solve_r<T, 2, NV>(L, E, factor, V, s);
    case 3: return launch_patch_solve_r<T, 3, NV>(L, E, factor, V, s);
    case 4: return launch_patch_solve_r<T, 4, NV>(L, E, factor, V, s);
    case 5: return launch_patch_solve_r<T, 5, NV>(L, E, factor, V, s);
    case 6: return launch_patch_solve_r<T, 6, NV>(L, E, factor, V, s);
    case 7: return launch_patch_solve_r<T, 7, NV>(L, E, factor, V, s);
    case 8:
      if constexpr (sizeof(T) == 4) return launch_patch_solve_r<T, 8, NV>(L, E, factor, V, s);
      return -1;
    default: return -1;
  }
}

// the register kernel's range: the compiled schedule matches, p >= 2, and the slot's
// values fit the registers (FP64 up to p = 7, FP32 up to p = 8)
bool patch_solve_uses_regs(const PatchEllDev &E, int p, size_t elem) {
  return E.regs && p >= 2 && p <= (elem == 8 ? 7 : 8);
}

template <typename T>
int launch_patch_solve(const LatDev &L, const PatchEllDev &E, const T *factor, const T *rt, T *zbuf, hipStream_t s) {
  const long nv = (long)(L.nx + 1) * (L.ny + 1) * (L.nz + 1);
  if (patch_solve_uses_regs(E, L.p, sizeof(T))) {
    PatchVecs<T> V{};
    V.rt[0] = rt;
    V.zb[0] = zbuf;
    return launch_patch_solve_r_nv<T, 1>(L, E, factor, V, s);
  }
  auto grid_of = [&](int waves, int per_cu) {
    long grid = (long)device_cu_count() * per_cu;
    const long need = (nv + waves - 1) / waves;
    return (unsigned)(grid > need ? need : grid);
  };
  // vectors in FP64 and diagonals in T in LDS; the resident wavefronts per CU as the
  // setup's autotuner chose them, else at most 12 for FP64 (measured at p = 7: 12 ->
  // 0.70 ms, 16 -> 0.73 ms, 8 -> 0.77 ms per launch; fewer slots in flight keep more
  // of the factor cached between the two sweeps) and as many as fit for FP32 (18 at
  // p = 7: 0.42 ms; 12: 0.57 ms)
  int waves, per_cu;
  const int tuned = E.cap[sizeof(T) == 8 ? 0 : 1];
  if (!patch_solve_shape(E, sizeof(double) + sizeof(T), tuned > 0 ? tuned : (sizeof(T) == 8 ? 12 : 32), waves,
                         per_cu))
    return -1;
  const size_t shm = patch_solve_lds(E, sizeof(double) + sizeof(T), waves);
  const unsigned grid = grid_of(waves, per_cu);
#define RZ_CALL(KM)                                                                                          \
  hipFuncSetAttribute((const void *)k_patch_solve_w<T, KM>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                      (int)shm);                                                                             \
  k_patch_solve_w<T, KM><<<grid, 64 * waves, shm, s>>>(L, E, factor, rt, zbuf, nv)
  switch (E.kmax) {
    case 1: RZ_CALL(1); break;
    case 2: RZ_CALL(2); break;
    case 3: RZ_CALL(3); break;
    case 4: RZ_CALL(4); break;
    case 5: RZ_CALL(5); break;
    case 6: RZ_CALL(6); break;
    case 7: RZ_CALL(7); break;
    case 8: RZ_CALL(8); break;
    default: return -1;
  }
#undef RZ_CALL
  return 0;
}

template <typename T>
void launch_expand_grad(const LatDev &L, const PatchDev &P, const T *coef, const T *A, const T *lam,
                        const T *r, const T *zbuf, T *z, T scale, T w, T *acc, hipStream_t s) {
  const ExpandOut<T> o{scale, w, acc};
#define RZ_CALL(Q) expand_p<Q, T>(L, coef, A, lam, r, zbuf, z, o, s)
  RZ_DISPATCH_P(L.p, RZ_CALL)
#undef RZ_CALL
}

void launch_patch_factor(const LatDev &L, const PatchDev &P, const double *coef, const double *B,
                         const double *A, const double *lam, const PdDev &pd, double *f64, float *f32, int *status,
                         hipStream_t s, int ic) {
  long nv = (long)(L.nx + 1) * (L.ny + 1) * (L.nz + 1);
  const int n1 = L.p + 1;
  size_t shm = sizeof(double) * (P.nnz + 2 * n1 * n1 + n1) + P.nnz;
  if (shm > 65536) hipFuncSetAttribute((const void *)k_patch_factor, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  k_patch_factor<<<(unsigned)nv, 256, shm, s>>>(L, P, P.erow, coef, B, A, lam, pd, f64, f32, status, ic);
}

namespace {

// Vertex-patch solves with exact Cholesky factors (eq. sc-asm-afw with
// S_v^{-1} = L_v^{-T} L_v^{-1}): z_v = W_v^T (W_v b_v) with W_v = L_v^{-1} stored dense,
// lower, packed by rows (row i at i (i + 1) / 2).  One block per vertex slot: the
// right-hand side gathered as by the IC solve (rows outside the domain or on a
// Dirichlet face read 0; their W rows are those of the identity); y = W b with one
// wavefront per row; z = W^T y with one thread per column reading the rows in order
// (coalesced); z to the slot's rows of zb.
template <typename T>
__global__ void __launch_bounds__(256) k_patch_chol_solve(LatDev L, const int *__restrict__ off, int nr,
                                                           const T *__restrict__ W, const T *__restrict__ rt,
                                                           T *__restrict__ zb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *sb = reinterpret_cast<double *>(smem_raw), *sy = sb + nr;
  const long slot = blockIdx.x;
  const int nvx = L.nx + 1, nvy = L.ny + 1, p = L.p;
  const int V[3] = {(int)(slot % nvx), (int)((slot / nvx) % nvy), (int)(slot / ((long)nvx * nvy))};
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int i = tid; i < nr; i += blockDim.x) {
    const int X = V[0] * p + off[3 * i], Y = V[1] * p + off[3 * i + 1], Z = V[2] * p + off[3 * i + 2];
    const bool in = X >= 0 && X < L.Nx && Y >= 0 && Y < L.Ny && Z >= 0 && Z < L.Nz;
    sb[i] = in && !lat_dirichlet(L, X, Y, Z) ? (double)rt[lat_index(L, X, Y, Z)] : 0.0;
  }
  __syncthreads();
  const T *Ws = W + slot * ((long)nr * (nr + 1) / 2);
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
    if (j < nr) zb[slot * nr + j] = (T)acc;
  }
}

}  // namespace

namespace {

// Sum over the full vertex stars holding each lattice point (vertex v holds X iff
// |X - v p| < p on every axis: one vertex per axis on a vertex plane, two off it) of
// their solutions, in a fixed order (z, y, x of the vertices); Dirichlet points take
// r.  v = scale * (that); z = v, or with acc: acc += w v.
template <typename T>
__global__ void k_full_star_sum(LatDev L, int nrf, const T *__restrict__ zb, const T *__restrict__ r,
                                T *__restrict__ z, T scale, T w, T *__restrict__ acc, long n) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const int p = L.p, q = 2 * p - 1;
  const int X[3] = {(int)(g % L.Nx), (int)((g / L.Nx) % L.Ny), (int)(g / ((long)L.Nx * L.Ny))};
  T v;
  if (lat_dirichlet(L, X[0], X[1], X[2])) {
    v = r[g];
  } else {
    int v0[3], nv[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      v0[d] = X[d] / p;
      nv[d] = X[d] - v0[d] * p == 0 ? 1 : 2;
    }
    const int nvx = L.nx + 1, nvy = L.ny + 1;
    T sum = 0;
    for (int k = 0; k < nv[2]; ++k)
      for (int j = 0; j < nv[1]; ++j)
        for (int i = 0; i < nv[0]; ++i) {
          const int V[3] = {v0[0] + i, v0[1] + j, v0[2] + k};
          const long slot = V[0] + (long)nvx * (V[1] + (long)nvy * V[2]);
          const int o = (X[0] - V[0] * p + p - 1) + q * ((X[1] - V[1] * p + p - 1) + q * (X[2] - V[2] * p + p - 1));
          sum += zb[slot * nrf + o];
        }
    v = sum;
  }
  v *= scale;
  if (acc) acc[g] += w * v;
  else z[g] = v;
}

}  // namespace

template <typename T>
void launch_full_star_sum(const LatDev &L, int nrf, const T *zb, const T *r, T *z, T scale, T w, T *acc,
                          hipStream_t s) {
  const long n = (long)L.Nx * L.Ny * L.Nz;
  k_full_star_sum<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(L, nrf, zb, r, z, scale, w, acc, n);
}
template void launch_full_star_sum<double>(const LatDev &, int, const double *, const double *, double *, double,
                                           double, double *, hipStream_t);
template void launch_full_star_sum<float>(const LatDev &, int, const float *, const float *, float *, float, float,
                                          float *, hipStream_t);

template <typename T>
void launch_patch_chol_solve(const LatDev &L, const PatchDev &P, const T *W, const T *rt, T *zb, hipStream_t s) {
  const long nv = (long)(L.nx + 1) * (L.ny + 1) * (L.nz + 1);
  k_patch_chol_solve<T><<<(unsigned)nv, 256, 2 * sizeof(double) * P.nrows, s>>>(L, P.off, P.nrows, W, rt, zb);
}
template void launch_patch_chol_solve<double>(const LatDev &, const PatchDev &, const double *, const double *,
                                              double *, hipStream_t);
template void launch_patch_chol_solve<float>(const LatDev &, const PatchDev &, const float *, const float *, float *,
                                             hipStream_t);

static long max_face_points(const LatDev &L) {
  return std::max({(long)L.Ny * L.Nz, (long)L.Nx * L.Nz, (long)L.Nx * L.Ny});
}

void launch_dirichlet_copy(const LatDev &L, const double *r, double *z, hipStream_t s) {
  const long nf = max_face_points(L);
  k_dirichlet_copy<double><<<dim3(nblocks(nf, 256), 6), 256, 0, s>>>(L, r, z);
}

void launch_dirichlet_copy_f(const LatDev &L, const float *r, float *z, hipStream_t s) {
  const long nf = max_face_points(L);
  k_dirichlet_copy<float><<<dim3(nblocks(nf, 256), 6), 256, 0, s>>>(L, r, z);
}

void launch_prolong_add_grad(const LatDev &L, const double *E, const double *xc, double *xf,
                             hipStream_t s) {
  const unsigned grid = (unsigned)((long)L.Ny * L.Nz);
  const int bs = L.Nx >= 256 ? 256 : ((L.Nx + 63) / 64) * 64;
  const size_t shm = (L.nx + 1) * sizeof(double);
#define RZ_CALL(Q) k_prolong_add_p<Q><<<grid, bs, shm, s>>>(L, E, xc, xf)
  RZ_DISPATCH_P(L.p, RZ_CALL)
#undef RZ_CALL
}

template <typename TV>
static void prolong_residual(const LatDev &L, const double *E, const double *T2, const double *coef,
                             const double *xc, TV *z, TV *r, hipStream_t s) {
  const unsigned grid = (unsigned)((long)L.ny * L.Nz);
  const size_t shm = (9 * (size_t)(L.nx + 1) + 16 * (size_t)L.nx + 4 * (size_t)(L.p + 1)) * sizeof(double);
#define RZ_CALL(Q) k_prolong_residual_p<Q, TV><<<grid, 256, shm, s>>>(L, E, T2, coef, xc, z, r)
  RZ_DISPATCH_P(L.p, RZ_CALL)
#undef RZ_CALL
}

void launch_prolong_residual_grad(const LatDev &L, const double *E, const double *T2, const double *coef,
                                  const double *xc, double *z, double *r, hipStream_t s) {
  prolong_residual<double>(L, E, T2, coef, xc, z, r, s);
}

void launch_prolong_residual_grad_f(const LatDev &L, const double *E, const double *T2, const double *coef,
                                    const double *xc, float *z, float *r, hipStream_t s) {
  prolong_residual<float>(L, E, T2, coef, xc, z, r, s);
}

void launch_restrict_grad(const LatDev &L, const double *E, const double *rf, double *rc, double *t1, double *t2,
                          hipStream_t s) {
  const long n1 = (long)(L.nx + 1) * L.Ny * L.Nz, n2 = (long)(L.nx + 1) * (L.ny + 1) * L.Nz,
             n3 = (long)(L.nx + 1) * (L.ny + 1) * (L.nz + 1);
  const long rows = (long)L.Ny * L.Nz;
  int R = 4;
  while (R > 1 && (size_t)R * L.Nx * sizeof(double) > 64 * 1024) R >>= 1;
  const size_t shm = (size_t)R * L.Nx * sizeof(double);
  if (shm <= 64 * 1024) {
    const unsigned grid = (unsigned)((rows + R - 1) / R);
#define RZ_CALL(Q) k_restrict_x_p<Q><<<grid, 64 * R, shm, s>>>(L, E, rf, t1, rows)
    RZ_DISPATCH_P(L.p, RZ_CALL)
#undef RZ_CALL
  } else {
    k_restrict_x<<<nblocks(n1, 256), 256, 0, s>>>(L, E, rf, t1, n1);
  }
#define RZ_CALL(Q)                                                          \
  k_restrict_y<Q><<<nblocks(n2, 256), 256, 0, s>>>(L, E, t1, t2, n2); \
  k_restrict_z<Q><<<nblocks(n3, 256), 256, 0, s>>>(L, E, t2, rc, n3)
  RZ_DISPATCH_P(L.p, RZ_CALL)
#undef RZ_CALL
}

template void launch_apply_grad<double>(const LatDev &, const double *, const double *, const double *,
                                        const double *, const double *, double *, double *, hipStream_t);
template void launch_apply_grad<float>(const LatDev &, const float *, const double *, const double *,
                                       const float *, const float *, float *, float *, hipStream_t);
template void launch_apply_gather<double>(const LatDev &, const double *, const double *, double *, hipStream_t,
                                          const double *);
template void launch_apply_gather<float>(const LatDev &, const float *, const float *, float *, hipStream_t,
                                         const float *);
template void launch_condense_grad<double>(const LatDev &, const double *, const double *, const double *,
                                           const double *, double *, hipStream_t);
template void launch_condense_grad<float>(const LatDev &, const float *, const float *, const float *,
                                          const float *, float *, hipStream_t);
// The patch solve of nvec right-hand sides rt[r] into zb[r].  The register kernel
// takes two vectors per launch, each slot's factor loaded once for both (measured at
// p = 7 in FP64: 0.351 ms per vector with two per launch, 0.403 with four, whose
// extra registers leave one wavefront per SIMD, 0.450 alone); the streaming kernel
// runs once per vector.
template <typename T>
int launch_patch_solve_multi(const LatDev &L, const PatchEllDev &E, const T *factor, int nvec, const T *const *rt,
                             T *const *zb, hipStream_t s) {
  if (nvec < 1) return 0;
  if (!patch_solve_uses_regs(E, L.p, sizeof(T))) {
    for (int r = 0; r < nvec; ++r)
      if (int e = launch_patch_solve<T>(L, E, factor, rt[r], zb[r], s)) return e;
    return 0;
  }
  for (int r0 = 0; r0 < nvec;) {
    const int nv = nvec - r0 >= 2 ? 2 : 1;
    PatchVecs<T> V{};
    for (int r = 0; r < nv; ++r) {
      V.rt[r] = rt[r0 + r];
      V.zb[r] = zb[r0 + r];
    }
    const int e = nv == 2 ? launch_patch_solve_r_nv<T, 2>(L, E, factor, V, s)
                          : launch_patch_solve_r_nv<T, 1>(L, E, factor, V, s);
    if (e) return e;
    r0 += nv;
  }
  return 0;
}

template int launch_patch_solve_multi<double>(const LatDev &, const PatchEllDev &, const double *, int,
                                              const double *const *, double *const *, hipStream_t);
template int launch_patch_solve_multi<float>(const LatDev &, const PatchEllDev &, const float *, int,
                                             const float *const *, float *const *, hipStream_t);
template int launch_patch_solve<double>(const LatDev &, const PatchEllDev &, const double *,
                                         const double *, double *, hipStream_t);
template int launch_patch_solve<float>(const LatDev &, const PatchEllDev &, const float *,
                                        const float *, float *, hipStream_t);
template void launch_expand_grad<double>(const LatDev &, const PatchDev &, const double *, const double *,
                                         const double *, const double *, const double *, double *, double,
                                         double, double *, hipStream_t);
template void launch_expand_grad<float>(const LatDev &, const PatchDev &, const float *, const float *,
                                        const float *, const float *, const float *, float *, float, float,
                                        float *, hipStream_t);

}  // namespace rz
