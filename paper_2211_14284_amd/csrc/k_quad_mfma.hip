// HIP kernel (gfx950) of the operator apply on trilinear cells with the 1-D
// contractions of the sum factorisation on the matrix cores: BF16 operands, FP32
// accumulation (v_mfma_f32_16x16x16_bf16), the pointwise pullback in FP32 (eq.
// sum-factorization with the quadrature of Sec. 5 and the pullbacks of Sec. 3.1:
// y_K = sum over quadrature points of w det(J) [alpha (J^-1 J^-T grad u) . grad v
// + beta u v]).  BF16 input x and output y; the interface rows of a cell go to the
// FP32 per-cell buffer summed by the gather kernel.
//
// Every 1-D factor (B_q, D_q: Q x (p+1), and their transposes) fits one 16 x 16
// MFMA operand (p <= 9, Q <= 16), held in registers for the whole cell.  A
// contraction along one axis is a product of that operand with the tile viewed as a
// (16 x columns) matrix whose rows are the contracted index; the columns (the other
// two indices) go 16 per MFMA.  One cell per block of four wavefronts, the column
// tiles of each stage split over the wavefronts:
//   A  x-contraction:  XB = B_x x, XD = D_x x                 (rows a, columns (b, c))
//   B  y-contraction:  W0 = B_y XB, W1 = D_y XB, W2 = B_y XD  (rows b, columns (i, c))
//   C  per column tile (j, i): z-contraction to u, d_z u, d_y u, d_x u at the Q
//      points of the line (rows k), the pullback on the accumulators, and the
//      transposed z-contraction of the results, which sit in the accumulator layout
//      that the next product takes as its operand (no LDS round trip)
//   F  transposed y-contraction:  S1 = B_y^T T1 + D_y^T T2, S2 = B_y^T T3
//   G  transposed x-contraction:  o = B_x^T S1 + D_x^T S2
// Between the stages the results go through LDS as BF16, stored [column][RS] with
// the next contraction's index fastest, so that a lane reads its four operand values
// with one 8-byte load.  Operand positions past the true sizes read zeros (the LDS
// is cleared before they are read and those positions are never written).  The
// affine Jacobian J0 + xi_z J1 of each z-line is computed once per line into LDS
// before stage C, in the space of XB, XD (free between stages B and F), not once per
// lane group that shares the line; the LDS of a block (53 KB at p = 8) leaves room
// for three blocks per CU.
//
// Operand layout of the 16 x 16 x 16 BF16 MFMA (wave64; lane l, g = l / 16, r = l % 16):
// A[r][4g + j], B[4g + j][r] for j = 0..3; the result D[4g + j][r].
#include <hip/hip_runtime.h>

#include "bf16.hpp"
#include "kernels.hpp"

namespace rz {

namespace {

typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mma(bf4 a, bf4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }

// row stride (BF16 elements) of the operand buffers: 16 operand rows padded to 10
// dwords, so that the 16 columns of a lane group's stores and loads fall in 16
// different banks (a stride of 8 dwords put every fourth row on the same banks)
constexpr int RS = 20;

// operand B of column col of a [column][RS] buffer for lane group g
__device__ __forceinline__ bf4 opnd(const bf16_t *buf, int col, int g) {
  return *reinterpret_cast<const bf4 *>(buf + col * RS + 4 * g);
}

constexpr int LN = 16;  // floats per z-line: J0 (9), J1 columns 0, 1 (6), pad

__device__ __forceinline__ bool mlat_dirichlet(const LatDev &L, int X, int Y, int Z) {
  return ((L.dir & 1u) && X == 0) || ((L.dir & 2u) && X == L.Nx - 1) || ((L.dir & 4u) && Y == 0) ||
         ((L.dir & 8u) && Y == L.Ny - 1) || ((L.dir & 16u) && Z == 0) || ((L.dir & 32u) && Z == L.Nz - 1);
}

__device__ __forceinline__ long mlat_index(const LatDev &L, int X, int Y, int Z) {
  return (long)X + (long)L.Nx * ((long)Y + (long)L.Ny * (long)Z);
}

template <int P, int Q>
__global__ void __launch_bounds__(256) k_apply_quad_mfma(LatDev L, QuadDev<float> G, const bf16_t *__restrict__ x,
                                                         bf16_t *__restrict__ y, float *__restrict__ ebuf) {
  constexpr int N1 = P + 1, N2 = N1 * N1, N3 = N2 * N1;
  static_assert(N1 <= 16 && Q <= 16 && Q >= N1, "one 16 x 16 operand per 1-D factor");
  constexpr int CA = (N2 + 15) / 16;     // column tiles of stages A and G: (b, c)
  constexpr int CB = (Q * N1 + 15) / 16; // stages B and F: (i, c)
  constexpr int CC = (Q * Q + 15) / 16;  // stage C: (j, i)
  constexpr int TB = 16 * RS;             // elements per column tile
  constexpr int UB = 2 * CB * TB * 2 > Q * Q * LN * 4 ? 2 * CB * TB * 2 : Q * Q * LN * 4;  // bytes
  static_assert(UB % 16 == 0, "aligned regions");
  __shared__ __align__(16) unsigned char smem[UB + 2 * (3 * CC * TB + 3 * CB * TB)];
  // XB, XD (later S1, S2; CA <= CB) share their space with the line geometry lg;
  // T1 first holds the x tile
  bf16_t *const XB = reinterpret_cast<bf16_t *>(smem), *const XD = XB + CB * TB;
  float *const lg = reinterpret_cast<float *>(smem);
  bf16_t *const W0 = reinterpret_cast<bf16_t *>(smem + UB), *const W1 = W0 + CC * TB, *const W2 = W1 + CC * TB;
  bf16_t *const T1 = W2 + CC * TB, *const T2 = T1 + CB * TB, *const T3 = T2 + CB * TB;
  __shared__ float sw[16], sx[16], sL[48], cr[24], sa[27], sb[27];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, g = lane >> 4, r = lane & 15;
  const long cell = blockIdx.x;
  const int cx = cell % L.nx, cy = (cell / L.nx) % L.ny, cz = cell / ((long)L.nx * L.ny);
  // clear n BF16 elements (a multiple of 8) at buf, 16 bytes per store
  auto clear = [&](bf16_t *buf, int n) {
    uint4 *w = reinterpret_cast<uint4 *>(buf);
    for (int k = tid; k < n / 8; k += 256) w[k] = uint4{0u, 0u, 0u, 0u};
  };
  clear(XB, (UB / 2 + 3 * CC * TB + 3 * CB * TB));
  if (tid < Q) {
    sw[tid] = G.wq[tid];
    sx[tid] = G.xq[tid];
  }
  if (tid < 3 * Q) sL[tid] = G.Lq[tid];
  if (tid < 24) {
    const int k = tid / 3, c = tid % 3;
    const long vid = (cx + (k & 1)) + (long)(L.nx + 1) * ((cy + ((k >> 1) & 1)) + (long)(L.ny + 1) * (cz + (k >> 2)));
    cr[tid] = (float)G.vert[3 * vid + c];
  }
  if (tid < 27) {
    sa[tid] = G.as[27 * cell + tid];
    sb[tid] = G.bs[27 * cell + tid];
  }
  // the 1-D factors as MFMA operands: aB[r][k] = B_q[r][k] (contraction over the
  // polynomial index), tB[r][k] = B_q[k][r] (over the quadrature index)
  bf4 aB, aD, tB, tD;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int k = 4 * g + j;
    aB[j] = (short)((r < Q && k < N1) ? f_to_bf16(G.Bq[r * N1 + k]) : 0);
    aD[j] = (short)((r < Q && k < N1) ? f_to_bf16(G.Dq[r * N1 + k]) : 0);
    tB[j] = (short)((k < Q && r < N1) ? f_to_bf16(G.Bq[k * N1 + r]) : 0);
    tD[j] = (short)((k < Q && r < N1) ? f_to_bf16(G.Dq[k * N1 + r]) : 0);
  }
  __syncthreads();
  // the x tile into T1 as [(b, c)][a]
  for (int k = tid; k < N3; k += 256) {
    const int a = k % N1, b = (k / N1) % N1, c = k / N2;
    const int X = cx * P + a, Y = cy * P + b, Z = cz * P + c;
    T1[(b + N1 * c) * RS + a] = mlat_dirichlet(L, X, Y, Z) ? bf16_t(0) : x[mlat_index(L, X, Y, Z)];
  }
  __syncthreads();
  const f4 zero = {0.f, 0.f, 0.f, 0.f};
  // A: rows i, columns (b, c)
  for (int task = wv; task < 2 * CA; task += 4) {
    const int t = task % CA, m = task / CA, col = 16 * t + r;
    const f4 acc = mma(m ? aD : aB, opnd(T1, col, g), zero);
    bf16_t *out = m ? XD : XB;
    if (col < N2) {
      const int b = col % N1, c = col / N1;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = 4 * g + j;
        if (i < Q) out[(i + Q * c) * RS + b] = f_to_bf16(acc[j]);
      }
    }
  }
  __syncthreads();
  // B: rows j, columns (i, c)
  for (int task = wv; task < 3 * CB; task += 4) {
    const int t = task % CB, o = task / CB, col = 16 * t + r;
    const f4 acc = mma(o == 1 ? aD : aB, opnd(o == 2 ? XD : XB, col, g), zero);
    bf16_t *out = o == 0 ? W0 : (o == 1 ? W1 : W2);
    if (col < Q * N1) {
      const int i = col % Q, c = col / Q;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int jj = 4 * g + j;
        if (jj < Q) out[(i + Q * jj) * RS + c] = f_to_bf16(acc[j]);
      }
    }
  }
  __syncthreads();
  // the Jacobian of every z-line (i, j): J(xi_z) = J0 + xi_z J1 (column 2 of J1 is
  // zero)
  for (int line = tid; line < Q * Q; line += 256) {
    const int i = line % Q, j = line / Q;
    const float xi = sx[i], eta = sx[j];
    float J0[9], J1[6];
#pragma unroll
    for (int e = 0; e < 9; ++e) J0[e] = 0.f;
#pragma unroll
    for (int e = 0; e < 6; ++e) J1[e] = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float s0 = (k & 1) ? 1.f : -1.f, s1 = ((k >> 1) & 1) ? 1.f : -1.f, s2 = (k >> 2) ? 1.f : -1.f;
      const float f0 = 0.5f * (1.f + s0 * xi), f1 = 0.5f * (1.f + s1 * eta);
      const float gx0 = 0.25f * s0 * f1, gy0 = 0.25f * s1 * f0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float X = cr[3 * k + c];
        J0[3 * c] += gx0 * X;
        J1[2 * c] += gx0 * s2 * X;
        J0[3 * c + 1] += gy0 * X;
        J1[2 * c + 1] += gy0 * s2 * X;
        J0[3 * c + 2] += 0.5f * s2 * f0 * f1 * X;
      }
    }
    float *o = lg + line * LN;
#pragma unroll
    for (int e = 0; e < 9; ++e) o[e] = J0[e];
#pragma unroll
    for (int e = 0; e < 6; ++e) o[9 + e] = J1[e];
  }
  __syncthreads();
  // C: per column tile (j, i) of the z-lines
  bf4 n0, n1, n2;  // the operands of the wavefront's next tile, loaded ahead
  if (wv < CC) {
    n0 = opnd(W0, 16 * wv + r, g);
    n1 = opnd(W1, 16 * wv + r, g);
    n2 = opnd(W2, 16 * wv + r, g);
  }
  for (int t = wv; t < CC; t += 4) {
    const int col = 16 * t + r;
    const bool ok = col < Q * Q;
    const int i = ok ? col % Q : 0, j = ok ? col / Q : 0;
    const bf4 w0 = n0, w1 = n1, w2 = n2;
    if (t + 4 < CC) {
      n0 = opnd(W0, col + 64, g);
      n1 = opnd(W1, col + 64, g);
      n2 = opnd(W2, col + 64, g);
    }
    const f4 u4 = mma(aB, w0, zero), uz4 = mma(aD, w0, zero), uy4 = mma(aB, w1, zero), ux4 = mma(aB, w2, zero);
    // the line's Jacobian (J1 column 2 is zero)
    const float4 *lq = reinterpret_cast<const float4 *>(lg + (i + Q * j) * LN);
    const float4 q0 = lq[0], q1 = lq[1], q2 = lq[2], q3 = lq[3];
    const float J0[9] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, q2.x};
    const float J1[9] = {q2.y, q2.z, 0.f, q2.w, q3.x, 0.f, q3.y, q3.z, 0.f};
    // coefficient samples reduced to the line: ca[c] = sum_ab s[a,b,c] L_a(xi) L_b(eta)
    float ca[3], cb[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      ca[c] = cb[c] = 0.f;
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float l = sL[3 * i + a] * sL[3 * j + b];
          ca[c] += sa[a + 3 * b + 9 * c] * l;
          cb[c] += sb[a + 3 * b + 9 * c] * l;
        }
    }
    const float wij = sw[i] * sw[j];
    bf4 m4, fz4, fy4, fx4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = 4 * g + q;
      float m = 0.f, fx = 0.f, fy = 0.f, fz = 0.f;
      if (ok && k < Q) {
        const float z = sx[k];
        float J[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) J[e] = J0[e] + z * J1[e];
        // cofactors: J^-1 = adj / det; G = J^-1 J^-T = adj adj^T / det^2
        const float a00 = J[4] * J[8] - J[5] * J[7], a01 = J[2] * J[7] - J[1] * J[8], a02 = J[1] * J[5] - J[2] * J[4];
        const float a10 = J[5] * J[6] - J[3] * J[8], a11 = J[0] * J[8] - J[2] * J[6], a12 = J[2] * J[3] - J[0] * J[5];
        const float a20 = J[3] * J[7] - J[4] * J[6], a21 = J[1] * J[6] - J[0] * J[7], a22 = J[0] * J[4] - J[1] * J[3];
        const float det = J[0] * a00 + J[1] * a10 + J[2] * a20;
        const float al = ca[0] * sL[3 * k] + ca[1] * sL[3 * k + 1] + ca[2] * sL[3 * k + 2];
        const float be = cb[0] * sL[3 * k] + cb[1] * sL[3 * k + 1] + cb[2] * sL[3 * k + 2];
        const float w = wij * sw[k];
        const float ka = w * al * __builtin_amdgcn_rcpf(det);  // w det alpha / det^2 (BF16 output: 1 ulp rcp)
        const float ux = ux4[q], uy = uy4[q], uz = uz4[q];
        const float g0 = a00 * ux + a10 * uy + a20 * uz;
        const float g1 = a01 * ux + a11 * uy + a21 * uz;
        const float g2 = a02 * ux + a12 * uy + a22 * uz;
        fx = ka * (a00 * g0 + a01 * g1 + a02 * g2);
        fy = ka * (a10 * g0 + a11 * g1 + a12 * g2);
        fz = ka * (a20 * g0 + a21 * g1 + a22 * g2);
        m = w * det * be * u4[q];
      }
      m4[q] = (short)f_to_bf16(m);
      fz4[q] = (short)f_to_bf16(fz);
      fy4[q] = (short)f_to_bf16(fy);
      fx4[q] = (short)f_to_bf16(fx);
    }
    // transposed z-contraction: rows c; the pointwise values are in operand layout
    const f4 t1 = mma(tD, fz4, mma(tB, m4, zero)), t2 = mma(tB, fy4, zero), t3 = mma(tB, fx4, zero);
    if (ok) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = 4 * g + q;
        if (c < N1) {
          const int o = (i + Q * c) * RS + j;
          T1[o] = f_to_bf16(t1[q]);
          T2[o] = f_to_bf16(t2[q]);
          T3[o] = f_to_bf16(t3[q]);
        }
      }
    }
  }
  __syncthreads();
  clear(XB, UB / 2);  // the line geometry out, zeros in for the operand padding of stage G
  __syncthreads();
  // F: rows b, columns (i, c); S1, S2 into XB, XD as [(b, c)][i]
  for (int task = wv; task < 2 * CB; task += 4) {
    const int t = task % CB, o = task / CB, col = 16 * t + r;
    const f4 acc = o == 0 ? mma(tD, opnd(T2, col, g), mma(tB, opnd(T1, col, g), zero)) : mma(tB, opnd(T3, col, g), zero);
    bf16_t *out = o == 0 ? XB : XD;
    if (col < Q * N1) {
      const int i = col % Q, c = col / Q;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int b = 4 * g + q;
        if (b < N1) out[(b + N1 * c) * RS + i] = f_to_bf16(acc[q]);
      }
    }
  }
  __syncthreads();
  // G: rows a, columns (b, c); interior rows of the cell to y, interface rows to ebuf
  for (int t = wv; t < CA; t += 4) {
    const int col = 16 * t + r;
    const f4 acc = mma(tD, opnd(XD, col, g), mma(tB, opnd(XB, col, g), zero));
    if (col < N2) {
      const int b = col % N1, c = col / N1;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int a = 4 * g + q;
        if (a < N1) {
          if (a != 0 && a != P && b != 0 && b != P && c != 0 && c != P)
            y[mlat_index(L, cx * P + a, cy * P + b, cz * P + c)] = f_to_bf16(acc[q]);
          else
            ebuf[cell * N3 + a + N1 * (b + N1 * c)] = acc[q];
        }
      }
    }
  }
}

template <int P, int Q>
void apply_quad_mfma_pq(const LatDev &L, const QuadDev<float> &G, const bf16_t *x, bf16_t *y, float *ebuf,
                        hipStream_t s) {
  const long nc = (long)L.nx * L.ny * L.nz;
  k_apply_quad_mfma<P, Q><<<(unsigned)nc, 256, 0, s>>>(L, G, x, y, ebuf);
}

}  // namespace

int launch_apply_quad_cells_bf16(const LatDev &L, const QuadDev<float> &G, const bf16_t *x, bf16_t *y, float *ebuf,
                                 hipStream_t s) {
  switch (L.p) {
    case 1: apply_quad_mfma_pq<1, 3>(L, G, x, y, ebuf, s); break;
    case 2: apply_quad_mfma_pq<2, 5>(L, G, x, y, ebuf, s); break;
    case 3: apply_quad_mfma_pq<3, 6>(L, G, x, y, ebuf, s); break;
    case 4: apply_quad_mfma_pq<4, 8>(L, G, x, y, ebuf, s); break;
    case 5: apply_quad_mfma_pq<5, 9>(L, G, x, y, ebuf, s); break;
    case 6: apply_quad_mfma_pq<6, 11>(L, G, x, y, ebuf, s); break;
    case 7: apply_quad_mfma_pq<7, 12>(L, G, x, y, ebuf, s); break;
    case 8: apply_quad_mfma_pq<8, 14>(L, G, x, y, ebuf, s); break;
    case 9: apply_quad_mfma_pq<9, 15>(L, G, x, y, ebuf, s); break;
    default: return -1;
  }
  return 0;
}

}  // namespace rz
