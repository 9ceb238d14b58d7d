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

#include <algorithm>

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

// vectors are below 2^31 entries (checked at setup), so 32-bit offsets within a component
__device__ __forceinline__ long comp_index(const VecDev &V, int m, const int C[3]) {
  return V.off[m] + (long)(C[0] + V.ext[m][0] * (C[1] + V.ext[m][1] * C[2]));
}

// ---- the apply, degree P and space known at compile time --------------------------------
// In the FDM bases every 1-D factor has at most three entries per row (B: diagonal
// plus the (0,P), (P,0) pair; D, P x (P+1): columns 0, P and i in row i >= 1), so
// every entry of a composite such as B_n (D_a1 u_a2 - D_a2 u_a1) is a short stencil
// of the input tile.  The apply works on CPB cells per block in two passes over
// lines of the cell tiles, one thread per line, the 1-D coefficients of the line's
// fixed coordinates in registers and the tile strides known at compile time:
//   1. the derived field into LDS: G_n = sigma_n B_n (C u)_n along lines of axis n
//      (curl) or Q = sigma sum_n D_n u_n along x lines (div);
//   2. every component entry along lines of its own axis m:
//      curl y_m = mu_m (B x B) u_m + D_{m+2}^T G_{m+1} - D_{m+1}^T G_{m+2},
//      div  y_m = mu_m B_m u_m + D_m^T Q,
//      stored from registers (owned rows to y, shared rows to the cell buffer).

// extents and strides of the cell tiles: component m of the space, and component n
// of the derived field (curl: NCF, P + 1 along n and P elsewhere; div: P^3)
template <int P, bool CURL>
struct VT {
  static constexpr int ext(int m, int a) { return (CURL ? a != m : a == m) ? P + 1 : P; }
  static constexpr int str(int m, int a) { return a == 0 ? 1 : (a == 1 ? ext(m, 0) : ext(m, 0) * ext(m, 1)); }
  static constexpr int size(int m) { return ext(m, 0) * ext(m, 1) * ext(m, 2); }
  static constexpr int coff(int m) { return m == 0 ? 0 : (m == 1 ? size(0) : size(0) + size(1)); }
  static constexpr int fext(int n, int a) { return CURL && a == n ? P + 1 : P; }
  static constexpr int fstr(int n, int a) { return a == 0 ? 1 : (a == 1 ? fext(n, 0) : fext(n, 0) * fext(n, 1)); }
  static constexpr int TS = P * (P + 1) * (P + 1);              // pitch of the component tiles
  static constexpr int TF = CURL ? (P + 1) * P * P : P * P * P;  // pitch of the field tiles
  static constexpr int NF = CURL ? 3 : 1;
  // lines per cell of the two passes
  static constexpr int L1 = CURL ? 3 * P * P : P * P;
  static constexpr int L2 = CURL ? 3 * (P + 1) * (P + 1) : 3 * P * P;
};

// pass 1, curl: the line of G_N along N at (a1, a2) = (i, j), a1 = N + 1, a2 = N + 2
template <int P, typename T, int N>
__device__ __forceinline__ void curl_field_line(const T *Uc, T *Gc, const T *sB, const T *sD, T sigma, int i, int j) {
  using S = VT<P, true>;
  constexpr int n1 = P + 1, A1 = (N + 1) % 3, A2 = (N + 2) % 3;
  constexpr int an = S::str(A2, N), aa = S::str(A2, A1), bn = S::str(A1, N), bb = S::str(A1, A2);
  const T *pa = Uc + A2 * S::TS + j * S::str(A2, A2);  // u_a2 at a2 = j: lines along a1
  const T *pb = Uc + A1 * S::TS + i * S::str(A1, A1);  // u_a1 at a1 = i: lines along a2
  const T d0 = sD[i * n1], dP = sD[i * n1 + P], di = i ? sD[i * n1 + i] : T(0);
  const T e0 = sD[j * n1], eP = sD[j * n1 + P], ej = j ? sD[j * n1 + j] : T(0);
  T F[n1];
#pragma unroll
  for (int q = 0; q <= P; ++q) {
    const T *ra = pa + q * an, *rb = pb + q * bn;
    F[q] = (d0 * ra[0] + dP * ra[P * aa] + di * ra[i * aa]) - (e0 * rb[0] + eP * rb[P * bb] + ej * rb[j * bb]);
  }
  T *g = Gc + N * S::TF + i * S::fstr(N, A1) + j * S::fstr(N, A2);
#pragma unroll
  for (int q = 0; q <= P; ++q) {
    T v = sB[q * n1 + q] * F[q];
    if (q == 0) v += sB[P] * F[P];
    if (q == P) v += sB[P * n1] * F[0];
    g[q * S::fstr(N, N)] = sigma * v;
  }
}

// pass 1, div: the x line of Q at (y, z) = (q1, q2)
template <int P, typename T>
__device__ __forceinline__ void div_field_line(const T *Uc, T *Gc, const T *sD, T sigma, int q1, int q2) {
  using S = VT<P, false>;
  constexpr int n1 = P + 1, s1 = S::str(1, 1), s2 = S::str(2, 2);
  const T *u0 = Uc + q1 * S::str(0, 1) + q2 * S::str(0, 2);
  const T *u1 = Uc + S::TS + q2 * S::str(1, 2);      // u_1 at z = q2: lines along y
  const T *u2 = Uc + 2 * S::TS + q1 * S::str(2, 1);  // u_2 at y = q1: lines along z
  T v[n1];
#pragma unroll
  for (int q = 0; q <= P; ++q) v[q] = u0[q];
  const T d0 = sD[q1 * n1], dP = sD[q1 * n1 + P], di = q1 ? sD[q1 * n1 + q1] : T(0);
  const T e0 = sD[q2 * n1], eP = sD[q2 * n1 + P], ej = q2 ? sD[q2 * n1 + q2] : T(0);
  T *g = Gc + q1 * P + q2 * P * P;
#pragma unroll
  for (int q = 0; q < P; ++q) {
    T dx = sD[q * n1] * v[0] + sD[q * n1 + P] * v[P];
    if (q >= 1) dx += sD[q * n1 + q] * v[q];
    const T *r1 = u1 + q, *r2 = u2 + q;
    const T dy = d0 * r1[0] + dP * r1[P * s1] + di * r1[q1 * s1];
    const T dz = e0 * r2[0] + eP * r2[P * s2] + ej * r2[q2 * s2];
    g[q] = sigma * (dx + dy + dz);
  }
}

// pass 2, curl: the line of y_M along M at (b, c) = (lb, lc), b < c the other axes
template <int P, typename T, int M>
__device__ __forceinline__ void curl_out_line(const T *Uc, const T *Gc, const T *sB, const T *sD, T mu, int lb,
                                              int lc, T *out) {
  using S = VT<P, true>;
  constexpr int n1 = P + 1, Bx = M == 0 ? 1 : 0, Cx = M == 2 ? 1 : 2, NA = (M + 1) % 3, NB = (M + 2) % 3;
  constexpr int sm = S::str(M, M), sb = S::str(M, Bx), sc = S::str(M, Cx);
  const T *u = Uc + M * S::TS;
  const bool eb = lb == 0 || lb == P, ec = lc == 0 || lc == P;
  const int jb = eb ? P - lb : lb, jc = ec ? P - lc : lc;
  const T wb0 = sB[lb * n1 + lb], wb1 = eb ? sB[lb * n1 + jb] : T(0);
  const T wc0 = sB[lc * n1 + lc], wc1 = ec ? sB[lc * n1 + jc] : T(0);
  const int o00 = lb * sb + lc * sc, o10 = jb * sb + lc * sc, o01 = lb * sb + jc * sc, o11 = jb * sb + jc * sc;
  // + D_NB^T G_NA (G_NA at M = q, NA = lna, NB = i; row lnb of D^T)
  // - D_NA^T G_NB (G_NB at M = q, NB = lnb, NA = i; row lna of D^T)
  const int lna = NA == Bx ? lb : lc, lnb = NB == Bx ? lb : lc;
  const T *ga = Gc + NA * S::TF + lna * S::fstr(NA, NA);
  const T *gb = Gc + NB * S::TF + lnb * S::fstr(NB, NB);
  const bool fa = lnb == 0 || lnb == P, fb = lna == 0 || lna == P;
  T ca[P], cb[P];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    ca[i] = fa || i == lnb ? sD[i * n1 + lnb] : T(0);
    cb[i] = fb || i == lna ? sD[i * n1 + lna] : T(0);
  }
#pragma unroll
  for (int q = 0; q < P; ++q) {
    const T *uq = u + q * sm;
    const T mass = wc0 * (wb0 * uq[o00] + wb1 * uq[o10]) + wc1 * (wb0 * uq[o01] + wb1 * uq[o11]);
    T ta = 0, tb = 0;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      ta += ca[i] * ga[q * S::fstr(NA, M) + i * S::fstr(NA, NB)];
      tb += cb[i] * gb[q * S::fstr(NB, M) + i * S::fstr(NB, NA)];
    }
    out[q] = mu * mass + ta - tb;
  }
}

// pass 2, div: the line of y_M along M at (a, b) = (la, lb), a < b the other axes
template <int P, typename T, int M>
__device__ __forceinline__ void div_out_line(const T *Uc, const T *Gc, const T *sB, const T *sD, T mu, int la,
                                             int lb, T *out) {
  using S = VT<P, false>;
  constexpr int n1 = P + 1, Ax = M == 0 ? 1 : 0, Bx = M == 2 ? 1 : 2;
  const T *u = Uc + M * S::TS + la * S::str(M, Ax) + lb * S::str(M, Bx);
  const T *g = Gc + la * S::fstr(0, Ax) + lb * S::fstr(0, Bx);
  T v[n1], w[P];
#pragma unroll
  for (int q = 0; q <= P; ++q) v[q] = u[q * S::str(M, M)];
#pragma unroll
  for (int i = 0; i < P; ++i) w[i] = g[i * S::fstr(0, M)];
#pragma unroll
  for (int q = 0; q <= P; ++q) {
    T mass = sB[q * n1 + q] * v[q];
    if (q == 0) mass += sB[P] * v[P];
    if (q == P) mass += sB[P * n1] * v[0];
    T dt;
    if (q == 0 || q == P) {
      dt = 0;
#pragma unroll
      for (int i = 0; i < P; ++i) dt += sD[i * n1 + q] * w[i];
    } else {
      dt = sD[q * n1 + q] * w[q];
    }
    out[q] = mu * mass + dt;
  }
}

// the vector entry of point k of component M's tile in the cell with per-cell data
// o (origin, boundary flag, component origins); -1 past the tile and on Dirichlet points
template <int P, bool CURL, int M>
__device__ __forceinline__ int tile_entry(const VecDev &V, const int *o, int k) {
  using S = VT<P, CURL>;
  constexpr int e0 = S::ext(M, 0), e1 = S::ext(M, 1);
  if (k >= S::size(M)) return -1;
  const int l0 = k % e0, l1 = (k / e0) % e1, l2 = k / (e0 * e1);
  if (o[3]) {
    const int C[3] = {o[0] + l0, o[1] + l1, o[2] + l2};
    if (comp_dirichlet(V, M, C)) return -1;
  }
  return o[4 + M] + l0 + V.ext[M][0] * (l1 + V.ext[M][1] * l2);
}

// pass 2, curl, a line with both other coordinates strictly inside the cell: one
// entry of each 1-D factor per point
template <int P, typename T, int M>
__device__ __forceinline__ void curl_out_line_int(const T *Uc, const T *Gc, const T *sB, const T *sD, T mu, int lb,
                                                  int lc, T *out) {
  using S = VT<P, true>;
  constexpr int n1 = P + 1, Bx = M == 0 ? 1 : 0, Cx = M == 2 ? 1 : 2, NA = (M + 1) % 3, NB = (M + 2) % 3;
  const T *u = Uc + M * S::TS + lb * S::str(M, Bx) + lc * S::str(M, Cx);
  const int lna = NA == Bx ? lb : lc, lnb = NB == Bx ? lb : lc;
  const T *ga = Gc + NA * S::TF + lna * S::fstr(NA, NA) + lnb * S::fstr(NA, NB);
  const T *gb = Gc + NB * S::TF + lnb * S::fstr(NB, NB) + lna * S::fstr(NB, NA);
  const T wb0 = sB[lb * n1 + lb], wc0 = sB[lc * n1 + lc];
  const T ca = sD[lnb * n1 + lnb], cb = sD[lna * n1 + lna];
#pragma unroll
  for (int q = 0; q < P; ++q)
    out[q] = mu * (wc0 * (wb0 * u[q * S::str(M, M)])) + ca * ga[q * S::fstr(NA, M)] - cb * gb[q * S::fstr(NB, M)];
}

template <int P, typename T, int CPB, bool CURL>
__global__ void __launch_bounds__(256) k_apply_vec_p(VecDev V, const T *__restrict__ coef, const T *__restrict__ Bg,
                                                      const T *__restrict__ Dg, const T *__restrict__ x,
                                                      T *__restrict__ y, T *__restrict__ ebuf, long ncells,
                                                      const T *__restrict__ bsub) {
  using S = VT<P, CURL>;
  constexpr int n1 = P + 1, TS = S::TS, TF = S::TF, NF = S::NF;
  extern __shared__ unsigned char vsm[];
  T *U = reinterpret_cast<T *>(vsm);  // [CPB][3][TS]
  T *G = U + CPB * 3 * TS;            // [CPB][NF][TF]
  T *sB = G + CPB * NF * TF;
  T *sD = sB + n1 * n1;
  T *sC = sD + P * n1;                                       // [CPB][6]
  // per cell: lattice origin, whether the cell touches the domain boundary, and the
  // index of its origin in each component
  int(*sO)[8] = reinterpret_cast<int(*)[8]>(sC + 6 * CPB);
  // fixed trip counts of the per-thread loops (every block but the last holds CPB cells)
  constexpr int NLU = (3 * TS * CPB + 255) / 256, NL1 = (S::L1 * CPB + 255) / 256, NL2 = (S::L2 * CPB + 255) / 256;
  const int c0 = blockIdx.x * CPB;
  const int nc = (int)min((long)CPB, ncells - c0);
  for (int k = threadIdx.x; k < n1 * n1; k += blockDim.x) sB[k] = Bg[k];
  for (int k = threadIdx.x; k < P * n1; k += blockDim.x) sD[k] = Dg[k];
  for (int k = threadIdx.x; k < 6 * nc; k += blockDim.x) sC[k] = coef[6 * (long)c0 + k];
  for (int k = threadIdx.x; k < nc; k += blockDim.x) {
    const int cell = c0 + k, cy = cell / V.nx;
    const int cc[3] = {cell - cy * V.nx, cy % V.ny, cy / V.ny};
    const int O[3] = {P * cc[0], P * cc[1], P * cc[2]};
    sO[k][0] = O[0];
    sO[k][1] = O[1];
    sO[k][2] = O[2];
    sO[k][3] = cc[0] == 0 || cc[0] == V.nx - 1 || cc[1] == 0 || cc[1] == V.ny - 1 || cc[2] == 0 ||
               cc[2] == V.nz - 1;
    for (int m = 0; m < 3; ++m) sO[k][4 + m] = (int)comp_index(V, m, O);
  }
  __syncthreads();
  {
    // one thread per tile point, all loads of the thread in flight before the first
    // LDS store (consecutive threads read consecutive x entries)
    T v[NLU];
#pragma unroll
    for (int it = 0; it < NLU; ++it) {
      const int t = threadIdx.x + 256 * it;
      const int cl = t / (3 * TS), m = (t / TS) % 3, k = t % TS;
      v[it] = T(0);
      if (t < 3 * TS * nc) {
        const int g = m == 0 ? tile_entry<P, CURL, 0>(V, sO[cl], k)
                              : (m == 1 ? tile_entry<P, CURL, 1>(V, sO[cl], k) : tile_entry<P, CURL, 2>(V, sO[cl], k));
        if (g >= 0) v[it] = x[g];
      }
    }
#pragma unroll
    for (int it = 0; it < NLU; ++it) {
      const int t = threadIdx.x + 256 * it;
      if (t < 3 * TS * CPB) U[t] = v[it];
    }
  }
  __syncthreads();
  for (int it = 0; it < NL1; ++it) {
    const int t = threadIdx.x + 256 * it;
    if (t >= S::L1 * nc) break;
    const int cl = t / S::L1, r = t % S::L1;
    const T *Uc = U + cl * 3 * TS;
    T *Gc = G + cl * NF * TF;
    if constexpr (CURL) {
      const int n = r / (P * P), w = r % (P * P), i = w % P, j = w / P;
      const T sg = sC[6 * cl + n];
      if (n == 0) curl_field_line<P, T, 0>(Uc, Gc, sB, sD, sg, i, j);
      else if (n == 1) curl_field_line<P, T, 1>(Uc, Gc, sB, sD, sg, i, j);
      else curl_field_line<P, T, 2>(Uc, Gc, sB, sD, sg, i, j);
    } else {
      div_field_line<P, T>(Uc, Gc, sD, sC[6 * cl], r % P, r / P);
    }
  }
  __syncthreads();
  for (int it = 0; it < NL2; ++it) {
    const int t = threadIdx.x + 256 * it;
    if (t >= S::L2 * nc) break;
    // the line's points: l[m] = q, the other two axes (in increasing order) la, lb
    int cl, m, la, lb;
    T out[n1];
    bool inner = false;  // curl: both other coordinates inside the cell (no shared entry)
    if constexpr (CURL) {
      // the (P-1)^2 lines of a component with both other coordinates inside the
      // cell first (cheap, and whole wavefronts of them), then the 4P others
      constexpr int NI = (P - 1) * (P - 1), NE = 4 * P;
      inner = t < 3 * NI * nc;
      if (inner) {
        cl = t / (3 * NI);
        const int r = t % (3 * NI), w = r % NI;
        m = r / NI;
        la = 1 + w % (P - 1 > 0 ? P - 1 : 1);
        lb = 1 + w / (P - 1 > 0 ? P - 1 : 1);
      } else {
        const int t2 = t - 3 * NI * nc;
        cl = t2 / (3 * NE);
        const int r = t2 % (3 * NE), k = r % NE;
        m = r / NE;
        if (k < 2 * n1) {
          la = k < n1 ? k : k - n1;
          lb = k < n1 ? 0 : P;
        } else {
          const int k2 = k - 2 * n1;
          la = k2 < P - 1 ? 0 : P;
          lb = 1 + (k2 < P - 1 ? k2 : k2 - (P - 1));
        }
      }
      const T *Uc = U + cl * 3 * TS;
      const T *Gc = G + cl * NF * TF;
      const T mu = sC[6 * cl + 3 + m];
      if (inner) {
        if (m == 0) curl_out_line_int<P, T, 0>(Uc, Gc, sB, sD, mu, la, lb, out);
        else if (m == 1) curl_out_line_int<P, T, 1>(Uc, Gc, sB, sD, mu, la, lb, out);
        else curl_out_line_int<P, T, 2>(Uc, Gc, sB, sD, mu, la, lb, out);
      } else {
        if (m == 0) curl_out_line<P, T, 0>(Uc, Gc, sB, sD, mu, la, lb, out);
        else if (m == 1) curl_out_line<P, T, 1>(Uc, Gc, sB, sD, mu, la, lb, out);
        else curl_out_line<P, T, 2>(Uc, Gc, sB, sD, mu, la, lb, out);
      }
    } else {
      cl = t / S::L2;
      const int r = t % S::L2, w = r % (P * P);
      m = r / (P * P);
      la = w % P;
      lb = w / P;
      const T *Uc = U + cl * 3 * TS;
      const T *Gc = G + cl * NF * TF;
      const T mu = sC[6 * cl + 3 + m];
      if (m == 0) div_out_line<P, T, 0>(Uc, Gc, sB, sD, mu, la, lb, out);
      else if (m == 1) div_out_line<P, T, 1>(Uc, Gc, sB, sD, mu, la, lb, out);
      else div_out_line<P, T, 2>(Uc, Gc, sB, sD, mu, la, lb, out);
    }
    // tile coordinates of the line's first point (la, lb on the other axes in order)
    const int l[3] = {m == 0 ? 0 : la, m == 0 ? la : (m == 1 ? 0 : lb), m == 2 ? 0 : lb};
    const long gbase = sO[cl][4 + m] + l[0] + V.ext[m][0] * (l[1] + V.ext[m][1] * l[2]);
    const long gstr = m == 0 ? 1 : (m == 1 ? (long)V.ext[m][0] : (long)V.ext[m][0] * V.ext[m][1]);
    const long n = V.off[3];
    // with bsub (the residual b - A x): an entry held by this cell alone is complete
    // here and stores b - value; shared entries store their partial sums, and the
    // gather subtracts their totals
    if constexpr (CURL) {
      // continuous along the two other axes: slot (la == P) + 2 (lb == P) of every point
      const int sl = (la == P) + 2 * (lb == P);
      T *dst = sl == 0 ? y + gbase : ebuf + (sl - 1) * n + gbase;
      if (bsub && inner) {
#pragma unroll
        for (int q = 0; q < P; ++q) y[gbase + q * gstr] = bsub[gbase + q * gstr] - out[q];
      } else {
#pragma unroll
        for (int q = 0; q < P; ++q) dst[q * gstr] = out[q];
      }
    } else {
      // continuous along m only: the end q = P of the line goes to slot 1
#pragma unroll
      for (int q = 0; q < P; ++q)
        y[gbase + q * gstr] = (bsub && q > 0) ? bsub[gbase + q * gstr] - out[q] : out[q];
      ebuf[gbase + P * gstr] = out[P];
    }
  }
}

// Shared rows.  An entry on the vertex planes of its continuous axes receives one
// contribution per cell holding it, identified by its side along those axes (side 1:
// the entry is at the cell's local end P); with s = side_b + 2 side_c (curl, b < c
// the continuous axes) or s = side_m (div), the cell with s = 0 stored its
// contribution in y, the others in ebuf[(s - 1) n + g].  The gather sums the
// existing contributions in the order of s; Dirichlet rows copy x.  One block per
// (GL consecutive x lines of the components, chunk of 128 entries), one thread per
// entry of each of its lines, all loads issued before the stores.  With bsub the
// stores are b - sum (b - x on Dirichlet rows).
constexpr int GL = 4;

template <int P, typename T, bool CURL>
__global__ void __launch_bounds__(128) k_apply_vec_gather(VecDev V, const T *__restrict__ x,
                                                          const T *__restrict__ ebuf, T *__restrict__ y,
                                                          int chunks, const T *__restrict__ bsub) {
  using S = VT<P, CURL>;
  int line = (blockIdx.x / chunks) * GL;
  const int ch = blockIdx.x % chunks, C0 = ch * 128 + (int)threadIdx.x;
  int m = 0;
  for (; m < 2; ++m) {
    const int nl = V.ext[m][1] * V.ext[m][2];
    if (line < nl) break;
    line -= nl;
  }
  int C1 = line % V.ext[m][1], C2 = line / V.ext[m][1];
  const int nc[3] = {V.nx, V.ny, V.nz};
  const long n = V.off[3];
  long g[GL];
  T acc[GL];
  int what[GL];  // 0: nothing, 1: sum, 2: Dirichlet copy
#pragma unroll
  for (int q = 0; q < GL; ++q) {
    what[q] = 0;
    acc[q] = T(0);
    g[q] = 0;
    if (m < 3 && C0 < V.ext[m][0]) {
      const int C[3] = {C0, C1, C2};
      bool lo_ok[2] = {false, false}, hi_ok[2] = {false, false}, shared = false;
      int k = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (S::ext(m, a) != P + 1) continue;
        const int c = C[a] / P;
        const bool on = C[a] - c * P == 0;
        shared |= on;
        hi_ok[k] = on && c > 0;  // side 1: the cell below
        lo_ok[k] = c < nc[a];    // side 0: the cell holding the entry at local index < P
        ++k;
      }
      if (shared) {
        g[q] = V.off[m] + C0 + (long)V.ext[m][0] * (C1 + (long)V.ext[m][1] * C2);
        if (comp_dirichlet(V, m, C)) {
          what[q] = 2;
          acc[q] = x[g[q]];
        } else {
          what[q] = 1;
          if (lo_ok[0] && (!CURL || lo_ok[1])) acc[q] = y[g[q]];
          if (hi_ok[0] && (!CURL || lo_ok[1])) acc[q] += ebuf[g[q]];
          if constexpr (CURL) {
            if (lo_ok[0] && hi_ok[1]) acc[q] += ebuf[n + g[q]];
            if (hi_ok[0] && hi_ok[1]) acc[q] += ebuf[2 * n + g[q]];
          }
        }
      }
    }
    // the next line (uniform over the block)
    if (m < 3 && ++C1 == V.ext[m][1]) {
      C1 = 0;
      if (++C2 == V.ext[m][2]) {
        C2 = 0;
        ++m;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < GL; ++q)
    if (what[q]) y[g[q]] = bsub ? bsub[g[q]] - acc[q] : acc[q];
}

}  // namespace

template <int P, typename T, bool CURL>
void apply_vec_pc(const VecDev &V, const T *coef, const T *B, const T *D, const T *x, T *y, T *ebuf, long nc,
                  hipStream_t s, const T *bsub) {
  using S = VT<P, CURL>;
  constexpr size_t per_cell = (3 * (size_t)S::TS + (size_t)S::NF * S::TF + 6) * sizeof(T) + 8 * sizeof(int);
  // about 2048 tile points per block of 256 threads, at most 48 KB of LDS
  constexpr int want = (2048 + 3 * S::TS - 1) / (3 * S::TS);
  constexpr int fit = (int)(48 * 1024 / per_cell) > 0 ? (int)(48 * 1024 / per_cell) : 1;
  constexpr int CPB = want < fit ? want : fit;
  const size_t shm = CPB * per_cell + ((P + 1) * (P + 1) + P * (P + 1)) * sizeof(T);
  k_apply_vec_p<P, T, CPB, CURL><<<(unsigned)((nc + CPB - 1) / CPB), 256, shm, s>>>(V, coef, B, D, x, y, ebuf, nc, bsub);
  long lines = 0;
  int emax = 0;
  for (int m = 0; m < 3; ++m) {
    lines += (long)V.ext[m][1] * V.ext[m][2];
    emax = std::max(emax, V.ext[m][0]);
  }
  const int chunks = (emax + 127) / 128;
  k_apply_vec_gather<P, T, CURL><<<(unsigned)((lines + GL - 1) / GL * chunks), 128, 0, s>>>(V, x, ebuf, y, chunks, bsub);
}

template <int P, typename T>
void apply_vec_p(const VecDev &V, const T *coef, const T *B, const T *D, const T *x, T *y, T *ebuf, long nc,
                 hipStream_t s, const T *bsub) {
  if (V.space == 1) apply_vec_pc<P, T, true>(V, coef, B, D, x, y, ebuf, nc, s, bsub);
  else apply_vec_pc<P, T, false>(V, coef, B, D, x, y, ebuf, nc, s, bsub);
}

template <typename T>
int launch_apply_vec(const VecDev &V, const T *coef, const T *B, const T *D, const T *x, T *y, T *ebuf,
                     hipStream_t s, const T *bsub) {
  if (V.p < 1 || V.p > kMaxP) return -1;
  const long nc = (long)V.nx * V.ny * V.nz;
  switch (V.p) {
    case 1: apply_vec_p<1, T>(V, coef, B, D, x, y, ebuf, nc, s, bsub); break;
    case 2: apply_vec_p<2, T>(V, coef, B, D, x, y, ebuf, nc, s, bsub); break;
    case 3: apply_vec_p<3, T>(V, coef, B, D, x, y, ebuf, nc, s, bsub); break;
    case 4: apply_vec_p<4, T>(V, coef, B, D, x, y, ebuf, nc, s, bsub); break;
    case 5: apply_vec_p<5, T>(V, coef, B, D, x, y, ebuf, nc, s, bsub); break;
    case 6: apply_vec_p<6, T>(V, coef, B, D, x, y, ebuf, nc, s, bsub); break;
    case 7: apply_vec_p<7, T>(V, coef, B, D, x, y, ebuf, nc, s, bsub); break;
    case 8: apply_vec_p<8, T>(V, coef, B, D, x, y, ebuf, nc, s, bsub); break;
    default: apply_vec_p<9, T>(V, coef, B, D, x, y, ebuf, nc, s, bsub); break;
  }
  return 0;
}

template int launch_apply_vec<double>(const VecDev &, const double *, const double *, const double *,
                                      const double *, double *, double *, hipStream_t, const double *);
template int launch_apply_vec<float>(const VecDev &, const float *, const float *, const float *, const float *,
                                     float *, float *, hipStream_t, const float *);

}  // namespace rz
