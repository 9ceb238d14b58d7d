// HIP kernel (gfx950) of the operator apply on trilinear cells with variable
// coefficients (eq. form-reference-values, eq. sum-factorization, Sec. 3.1
// pullbacks): y_K = sum over quadrature points of w det(J) [alpha (J^-1 J^-T grad u)
// . grad v + beta u v] in reference coordinates, with u interpolated from the FDM
// coefficients of the cell by 1-D contractions along x, y, z and the result
// contracted back.  One cell per block, P+1 <= Q; Q*Q threads.  Stages:
//   A  x-contraction of the tile (lines b,c): XB = B_x x, XD = D_x x
//   B  y-contraction (lines i,c): W0 = B_y XB, W1 = D_y XB, W2 = B_y XD
//   C  z-contraction (lines i,j) to u, d_z u, d_y u, d_x u at the Q points of the
//      line, the pointwise pullback, and the transposed z-contraction back into
//      W0..W2 (the Jacobian along a z-line is affine in xi_z)
//   F  transposed y-contraction into XB, XD;  G  transposed x-contraction.
// Interior rows of the cell are stored, interface rows go to the per-cell buffer
// summed by the gather kernel of the Cartesian path.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace rz {

namespace {

__device__ __forceinline__ bool qlat_dirichlet(const LatDev &L, int X, int Y, int Z) {
  return ((L.dir & 1u) && X == 0) || ((L.dir & 2u) && X == L.Nx - 1) || ((L.dir & 4u) && Y == 0) ||
         ((L.dir & 8u) && Y == L.Ny - 1) || ((L.dir & 16u) && Z == 0) || ((L.dir & 32u) && Z == L.Nz - 1);
}

__device__ __forceinline__ long qlat_index(const LatDev &L, int X, int Y, int Z) {
  return (long)X + (long)L.Nx * ((long)Y + (long)L.Ny * (long)Z);
}

template <int P, int Q, typename T>
__global__ void __launch_bounds__(Q *Q) k_apply_quad(LatDev L, QuadDev<T> G, const T *__restrict__ x,
                                                     T *__restrict__ y, T *__restrict__ ebuf,
                                                     const T *__restrict__ bsub) {
  constexpr int N1 = P + 1, N2 = N1 * N1, N3 = N2 * N1, QQ = Q * Q;
  __shared__ T tile[N3];
  __shared__ T XB[N2 * Q], XD[N2 * Q];
  __shared__ T W0[N1 * QQ], W1[N1 * QQ], W2[N1 * QQ];
  __shared__ T sB[Q * N1], sD[Q * N1], sw[Q], sx[Q], sL[3 * Q];
  __shared__ T cr[24], sa[27], sb[27];
  const int tid = threadIdx.x;
  const long cell = blockIdx.x;
  const int cx = cell % L.nx, cy = (cell / L.nx) % L.ny, cz = cell / ((long)L.nx * L.ny);
  for (int k = tid; k < Q * N1; k += QQ) {
    sB[k] = G.Bq[k];
    sD[k] = G.Dq[k];
  }
  if (tid < Q) {
    sw[tid] = G.wq[tid];
    sx[tid] = G.xq[tid];
  }
  // small blocks (Q*Q may be below 27) load the per-cell data in strides
  for (int t = tid; t < 3 * Q; t += QQ) sL[t] = G.Lq[t];
  for (int t = tid; t < 24; t += QQ) {
    const int k = t / 3, r = t % 3;
    const long vid = (cx + (k & 1)) + (long)(L.nx + 1) * ((cy + ((k >> 1) & 1)) + (long)(L.ny + 1) * (cz + (k >> 2)));
    cr[t] = (T)G.vert[3 * vid + r];
  }
  for (int t = tid; t < 27; t += QQ) {
    sa[t] = G.as[27 * cell + t];
    sb[t] = G.bs[27 * cell + t];
  }
  for (int k = tid; k < N3; k += QQ) {
    const int a = k % N1, b = (k / N1) % N1, c = k / N2;
    const int X = cx * P + a, Y = cy * P + b, Z = cz * P + c;
    tile[k] = qlat_dirichlet(L, X, Y, Z) ? T(0) : x[qlat_index(L, X, Y, Z)];
  }
  __syncthreads();
  // A: lines (b,c) along x
  if (tid < N2) {
    T r[N1];
#pragma unroll
    for (int a = 0; a < N1; ++a) r[a] = tile[tid * N1 + a];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      T vb = 0, vd = 0;
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        vb += sB[i * N1 + a] * r[a];
        vd += sD[i * N1 + a] * r[a];
      }
      XB[tid * Q + i] = vb;
      XD[tid * Q + i] = vd;
    }
  }
  __syncthreads();
  // B: lines (i,c) along y
  if (tid < Q * N1) {
    const int i = tid % Q, c = tid / Q;
    T rb[N1], rd[N1];
#pragma unroll
    for (int b = 0; b < N1; ++b) {
      rb[b] = XB[(b + N1 * c) * Q + i];
      rd[b] = XD[(b + N1 * c) * Q + i];
    }
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      T v0 = 0, v1 = 0, v2 = 0;
#pragma unroll
      for (int b = 0; b < N1; ++b) {
        v0 += sB[j * N1 + b] * rb[b];
        v1 += sD[j * N1 + b] * rb[b];
        v2 += sB[j * N1 + b] * rd[b];
      }
      W0[(c * Q + j) * Q + i] = v0;
      W1[(c * Q + j) * Q + i] = v1;
      W2[(c * Q + j) * Q + i] = v2;
    }
  }
  __syncthreads();
  // C: lines (i,j) along z
  const int i = tid % Q, j = tid / Q;
  T bb[N1], bd[N1], db[N1];
#pragma unroll
  for (int c = 0; c < N1; ++c) {
    bb[c] = W0[(c * Q + j) * Q + i];
    bd[c] = W1[(c * Q + j) * Q + i];
    db[c] = W2[(c * Q + j) * Q + i];
  }
  __syncthreads();
  {
    // Jacobian along the line: J(xi_z) = J0 + xi_z J1 (column 2 constant)
    const T xi = sx[i], eta = sx[j];
    T J0[9], J1[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) J0[e] = J1[e] = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const T s0 = (k & 1) ? 1 : -1, s1 = ((k >> 1) & 1) ? 1 : -1, s2 = (k >> 2) ? 1 : -1;
      const T f0 = T(0.5) * (1 + s0 * xi), f1 = T(0.5) * (1 + s1 * eta);
      // d/dxi_x: 0.5 s0 f1 fz, d/dxi_y: 0.5 s1 f0 fz with fz = 0.5 (1 + s2 xi_z); d/dxi_z: 0.5 s2 f0 f1
      const T gx0 = T(0.25) * s0 * f1, gy0 = T(0.25) * s1 * f0;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const T X = cr[3 * k + r];
        J0[3 * r] += gx0 * X;
        J1[3 * r] += gx0 * s2 * X;
        J0[3 * r + 1] += gy0 * X;
        J1[3 * r + 1] += gy0 * s2 * X;
        J0[3 * r + 2] += T(0.5) * s2 * f0 * f1 * X;
      }
    }
    // coefficient samples reduced to the line: ca[c] = sum_ab s[a,b,c] L_a(xi) L_b(eta)
    T ca[3], cb[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      ca[c] = cb[c] = 0;
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const T l = sL[3 * i + a] * sL[3 * j + b];
          ca[c] += sa[a + 3 * b + 9 * c] * l;
          cb[c] += sb[a + 3 * b + 9 * c] * l;
        }
    }
    const T wij = sw[i] * sw[j];
    T t1[N1], t2[N1], t3[N1];
#pragma unroll
    for (int c = 0; c < N1; ++c) t1[c] = t2[c] = t3[c] = 0;
    for (int k = 0; k < Q; ++k) {
      T u = 0, uz = 0, uy = 0, ux = 0;
#pragma unroll
      for (int c = 0; c < N1; ++c) {
        const T bk = sB[k * N1 + c], dk = sD[k * N1 + c];
        u += bk * bb[c];
        uz += dk * bb[c];
        uy += bk * bd[c];
        ux += bk * db[c];
      }
      const T z = sx[k];
      T J[9];
#pragma unroll
      for (int e = 0; e < 9; ++e) J[e] = J0[e] + z * J1[e];
      // cofactors: J^-1 = adj / det; G = J^-1 J^-T = adj adj^T / det^2
      const T a00 = J[4] * J[8] - J[5] * J[7], a01 = J[2] * J[7] - J[1] * J[8], a02 = J[1] * J[5] - J[2] * J[4];
      const T a10 = J[5] * J[6] - J[3] * J[8], a11 = J[0] * J[8] - J[2] * J[6], a12 = J[2] * J[3] - J[0] * J[5];
      const T a20 = J[3] * J[7] - J[4] * J[6], a21 = J[1] * J[6] - J[0] * J[7], a22 = J[0] * J[4] - J[1] * J[3];
      const T det = J[0] * a00 + J[1] * a10 + J[2] * a20;
      const T al = ca[0] * sL[3 * k] + ca[1] * sL[3 * k + 1] + ca[2] * sL[3 * k + 2];
      const T be = cb[0] * sL[3 * k] + cb[1] * sL[3 * k + 1] + cb[2] * sL[3 * k + 2];
      const T w = wij * sw[k];
      const T ka = w * al / det;  // w det alpha / det^2
      // flux = w det alpha J^-1 J^-T grad_ref u = ka * adj (adj^T grad_ref u), adj = a
      const T g0 = a00 * ux + a10 * uy + a20 * uz;
      const T g1 = a01 * ux + a11 * uy + a21 * uz;
      const T g2 = a02 * ux + a12 * uy + a22 * uz;
      const T fx = ka * (a00 * g0 + a01 * g1 + a02 * g2);
      const T fy = ka * (a10 * g0 + a11 * g1 + a12 * g2);
      const T fz = ka * (a20 * g0 + a21 * g1 + a22 * g2);
      const T m = w * det * be * u;
#pragma unroll
      for (int c = 0; c < N1; ++c) {
        const T bk = sB[k * N1 + c], dk = sD[k * N1 + c];
        t1[c] += bk * m + dk * fz;
        t2[c] += bk * fy;
        t3[c] += bk * fx;
      }
    }
#pragma unroll
    for (int c = 0; c < N1; ++c) {
      W0[(c * Q + j) * Q + i] = t1[c];
      W1[(c * Q + j) * Q + i] = t2[c];
      W2[(c * Q + j) * Q + i] = t3[c];
    }
  }
  __syncthreads();
  // F: lines (i,c) along y, transposed
  if (tid < Q * N1) {
    const int ii = tid % Q, c = tid / Q;
    T s1[N1], s2[N1];
#pragma unroll
    for (int b = 0; b < N1; ++b) s1[b] = s2[b] = 0;
    for (int jj = 0; jj < Q; ++jj) {
      const T v0 = W0[(c * Q + jj) * Q + ii], v1 = W1[(c * Q + jj) * Q + ii], v2 = W2[(c * Q + jj) * Q + ii];
#pragma unroll
      for (int b = 0; b < N1; ++b) {
        s1[b] += sB[jj * N1 + b] * v0 + sD[jj * N1 + b] * v1;
        s2[b] += sB[jj * N1 + b] * v2;
      }
    }
#pragma unroll
    for (int b = 0; b < N1; ++b) {
      XB[(b + N1 * c) * Q + ii] = s1[b];
      XD[(b + N1 * c) * Q + ii] = s2[b];
    }
  }
  __syncthreads();
  // G: lines (b,c) along x, transposed
  if (tid < N2) {
    T o[N1];
#pragma unroll
    for (int a = 0; a < N1; ++a) o[a] = 0;
    for (int ii = 0; ii < Q; ++ii) {
      const T v1 = XB[tid * Q + ii], v2 = XD[tid * Q + ii];
#pragma unroll
      for (int a = 0; a < N1; ++a) o[a] += sB[ii * N1 + a] * v1 + sD[ii * N1 + a] * v2;
    }
#pragma unroll
    for (int a = 0; a < N1; ++a) tile[tid * N1 + a] = o[a];
  }
  __syncthreads();
  for (int k = tid; k < N3; k += QQ) {
    const int a = k % N1, b = (k / N1) % N1, c = k / N2;
    const T val = tile[k];
    if (a != 0 && a != P && b != 0 && b != P && c != 0 && c != P) {  // held by this cell alone
      const long g = qlat_index(L, cx * P + a, cy * P + b, cz * P + c);
      y[g] = bsub ? bsub[g] - val : val;
    } else {
      ebuf[cell * N3 + k] = val;
    }
  }
}

template <int P, int Q, typename T>
void apply_quad_pq(const LatDev &L, const QuadDev<T> &G, const T *x, T *y, T *ebuf, hipStream_t s, const T *bsub) {
  const long nc = (long)L.nx * L.ny * L.nz;
  k_apply_quad<P, Q, T><<<(unsigned)nc, Q * Q, 0, s>>>(L, G, x, y, ebuf, bsub);
}

}  // namespace

template <typename T>
int launch_apply_quad_cells(const LatDev &L, const QuadDev<T> &G, const T *x, T *y, T *ebuf, hipStream_t s,
                            const T *bsub) {
  switch (L.p) {
    case 1: apply_quad_pq<1, 3, T>(L, G, x, y, ebuf, s, bsub); break;
    case 2: apply_quad_pq<2, 5, T>(L, G, x, y, ebuf, s, bsub); break;
    case 3: apply_quad_pq<3, 6, T>(L, G, x, y, ebuf, s, bsub); break;
    case 4: apply_quad_pq<4, 8, T>(L, G, x, y, ebuf, s, bsub); break;
    case 5: apply_quad_pq<5, 9, T>(L, G, x, y, ebuf, s, bsub); break;
    case 6: apply_quad_pq<6, 11, T>(L, G, x, y, ebuf, s, bsub); break;
    case 7: apply_quad_pq<7, 12, T>(L, G, x, y, ebuf, s, bsub); break;
    case 8: apply_quad_pq<8, 14, T>(L, G, x, y, ebuf, s, bsub); break;
    case 9: apply_quad_pq<9, 15, T>(L, G, x, y, ebuf, s, bsub); break;
    default: return -1;
  }
  return 0;
}

template int launch_apply_quad_cells<double>(const LatDev &, const QuadDev<double> &, const double *, double *,
                                             double *, hipStream_t, const double *);
template int launch_apply_quad_cells<float>(const LatDev &, const QuadDev<float> &, const float *, float *,
                                            float *, hipStream_t, const float *);

}  // namespace rz
