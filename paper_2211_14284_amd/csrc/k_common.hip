// HIP kernels (gfx950): vector updates, deterministic FP64 dot products, and the
// coarse (p = 1) block-tridiagonal LDL^T factorisation and solve.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace rz {

namespace {

constexpr int kDotBlocks = 1024;
constexpr int kBS = 256;

inline unsigned nblk(int64_t n, int bs = kBS) {
  int64_t b = (n + bs - 1) / bs;
  if (b > 65535 * 64) b = 65535 * 64;
  return (unsigned)(b < 1 ? 1 : b);
}

__global__ void k_fill(double *y, double v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = v;
}
__global__ void k_d2f(const double *x, float *y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}
__global__ void k_f2d(const float *x, double *y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (double)x[i];
}

__global__ void k_f2d_scale(double a, const float *__restrict__ x, double *__restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * (double)x[i];
}

__global__ void k_f2d_axpy(double a, const float *__restrict__ x, double *__restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] += a * (double)x[i];
}
__global__ void k_axpy(double a, const double *x, double *y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] += a * x[i];
}
__global__ void k_xpby(const double *x, double b, double *y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i] + b * y[i];
}

// Multi-vector layouts: interleaved (value r of DoF g at u[g * nv + r]) and planar
// (vector r contiguous at v + r * ld).  One thread per DoF moves its nv values.
template <typename T>
__global__ void k_deinterleave(const T *__restrict__ u, T *__restrict__ v, int nv, int64_t ld, int64_t n) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x)
    for (int r = 0; r < nv; ++r) v[r * ld + g] = u[g * nv + r];
}
template <typename T>
__global__ void k_interleave(const T *__restrict__ v, T *__restrict__ u, int nv, int64_t ld, int64_t n) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x)
    for (int r = 0; r < nv; ++r) u[g * nv + r] = v[r * ld + g];
}

// y = x + b y with b = (num - cross) / den read from device memory (cross optional)
__global__ void k_xpby_dev(const double *__restrict__ x, const double *__restrict__ num,
                           const double *__restrict__ cross, const double *__restrict__ den, double *__restrict__ y,
                           int64_t n) {
  const double b = (*num - (cross ? *cross : 0.0)) / *den;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i] + b * y[i];
}
__global__ void k_sub(const double *x, const double *y, double *z, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    z[i] = x[i] - y[i];
}
__global__ void k_scale_copy(double a, const double *x, double *y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}

struct DotArgs {
  const double *x[3];
  const double *y[3];
};

// wavefront (64 lanes) sum by shuffles, then across the 4 waves of the block
// FP32 vectors of the inner solve of the defect-correction protocol (scalars and
// inner products in FP64)
__global__ void k_axpy_f(float a, const float *x, float *y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] += a * x[i];
}
__global__ void k_xpby_f(const float *x, float b, float *y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i] + b * y[i];
}
__global__ void k_sub_f(const float *x, const float *y, float *z, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    z[i] = x[i] - y[i];
}
__global__ void k_scale_copy_f(float a, const float *x, float *y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}
__global__ void k_fill_f(float *y, float v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = v;
}
// y64 += x32 ; z32 += t64
__global__ void k_add_f2d(const float *x, double *y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] += (double)x[i];
}
__global__ void k_add_d2f(const double *t, float *z, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    z[i] += (float)t[i];
}

__device__ __forceinline__ double block_sum(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
  __syncthreads();
  return t;
}

__global__ void __launch_bounds__(kBS) k_dot_partial(int np, DotArgs a, int64_t n, double *partials) {
  __shared__ double red[16];
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    for (int k = 0; k < np; ++k) acc[k] += a.x[k][i] * a.y[k][i];
  for (int k = 0; k < np; ++k) {
    double t = block_sum(acc[k], red);
    if (threadIdx.x == 0) partials[k * gridDim.x + blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(kBS) k_dot_final(int np, int nb, const double *partials, double *out) {
  __shared__ double red[16];
  for (int k = 0; k < np; ++k) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += partials[k * nb + i];
    double t = block_sum(acc, red);
    if (threadIdx.x == 0) out[k] = t;
  }
}

// CG update fused with the next inner product: x += a p; (ro = r); r -= a Ap;
// partial sums of r.r (same two-pass reduction as the dots)
// x += a p, r -= a Ap (ro = r before the update when given), partial sums of r.r;
// a = num / den read from device memory (0 when den <= 0: the host reports the
// breakdown from the den it reads back)
__global__ void __launch_bounds__(kBS) k_cg_update(const double *__restrict__ num, const double *__restrict__ den,
                                                    const double *__restrict__ p,
                                                    const double *__restrict__ Ap, double *__restrict__ x,
                                                    double *__restrict__ r, double *__restrict__ ro, int64_t n,
                                                    double *partials) {
  __shared__ double red[16];
  const double dn = *den;
  const double a = dn > 0.0 ? *num / dn : 0.0;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    x[i] += a * p[i];
    const double ri = r[i];
    if (ro) ro[i] = ri;
    const double rn = ri - a * Ap[i];
    r[i] = rn;
    acc += rn * rn;
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

struct DotArgsF {
  const float *x[3];
  const float *y[3];
};

__global__ void __launch_bounds__(kBS) k_dot_partial_f(int np, DotArgsF a, int64_t n, double *partials) {
  __shared__ double red[16];
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    for (int k = 0; k < np; ++k) acc[k] += (double)a.x[k][i] * (double)a.y[k][i];
  for (int k = 0; k < np; ++k) {
    double t = block_sum(acc[k], red);
    if (threadIdx.x == 0) partials[k * gridDim.x + blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(kBS) k_cg_update_f(float a, const float *__restrict__ p,
                                                      const float *__restrict__ Ap, float *__restrict__ x,
                                                      float *__restrict__ r, float *__restrict__ ro, int64_t n,
                                                      double *partials) {
  __shared__ double red[16];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    x[i] += a * p[i];
    const float ri = r[i];
    if (ro) ro[i] = ri;
    const float rn = ri - a * Ap[i];
    r[i] = rn;
    acc += (double)rn * (double)rn;
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// ---- coarse block-tridiagonal LDL^T ------------------------------------------------
__device__ __forceinline__ int nbr(int a, int j, int mx, int my) {
  int ax = a % mx + (j % 3) - 1, ay = a / mx + (j / 3) - 1;
  if (ax < 0 || ax >= mx || ay < 0 || ay >= my) return -1;
  return ax + mx * ay;
}

// D = Akk - C W C^T  (C has <= 9 entries per row)
__global__ void k_schur_update(int m, int mx, const double *__restrict__ W, const double *__restrict__ C,
                               const double *__restrict__ Akk, double *__restrict__ D) {
  int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * m) return;
  int a = idx / m, b = idx % m;
  int my = m / mx;
  double acc = 0.0;
  for (int i = 0; i < 9; ++i) {
    int c = nbr(a, i, mx, my);
    double ca = C[a * 9 + i];
    if (c < 0 || ca == 0.0) continue;
    for (int j = 0; j < 9; ++j) {
      int d = nbr(b, j, mx, my);
      double cb = C[b * 9 + j];
      if (d < 0 || cb == 0.0) continue;
      acc += ca * cb * W[(int64_t)c * m + d];
    }
  }
  D[idx] = Akk[idx] - acc;
}

// one pivot of the symmetric sweep operator (Goodnight): after sweeping every
// pivot of an SPD matrix the array holds -A^{-1}.  Reads `in`, writes `out`.
__global__ void k_sweep(int m, int k, const double *__restrict__ in, double *__restrict__ out, int *status) {
  int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * m) return;
  int i = idx / m, j = idx % m;
  double d = in[(int64_t)k * m + k];
  if (!(d > 0.0)) {
    if (idx == 0) atomicCAS(status, 0, k + 1);
    d = 1.0;
  }
  double v;
  if (i == k && j == k) v = -1.0 / d;
  else if (i == k) v = in[(int64_t)k * m + j] / d;
  else if (j == k) v = in[(int64_t)i * m + k] / d;
  else v = in[idx] - in[(int64_t)i * m + k] * in[(int64_t)k * m + j] / d;
  out[idx] = v;
}

__global__ void k_negate(double *W, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    W[i] = -W[i];
}

// Cross-block data of the coarse sweeps (v, x) is written once per solve with
// agent-scope relaxed atomic stores and read with agent-scope atomic loads (both
// bypass the per-XCD L2 incoherence).  Before the launch every entry holds the
// signalling-NaN pattern kEmpty, which no arithmetic result can take (computed NaNs
// are quiet), so a reader polls each entry until it differs from kEmpty: the data
// itself is the synchronisation and no grid barrier is needed.  An aligned 64-bit
// store is single-copy atomic, so a reader sees either kEmpty or the final value.
// The wait is bounded: after ~2^26 polls the thread records status = -1 and goes on.
constexpr unsigned long long kEmpty = 0xFFF5A5A5A5A5A5A5ull;

__device__ __forceinline__ void st_agent(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_agent_bits(const double *p) {
  return __hip_atomic_load(reinterpret_cast<unsigned long long *>(const_cast<double *>(p)), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}


// Coupling products of the block LDL^T: out = W_k Cs with Cs the 9-point in-plane
// coupling of plane k to a neighbouring plane (C[a][j]: row a, neighbour j of a), so
// out[i][b] = sum_j W_k[i][nbr_j(b)] C[nbr_j(b)][8 - j] (the offset of b seen from
// nbr_j(b) is the reverse one, index 8 - j).
__global__ void k_coarse_wc(int m, int mx, int my, const double *__restrict__ W, const double *__restrict__ C,
                            double *__restrict__ out) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * m) return;
  const int i = idx / m, b = idx % m;
  double s = 0.0;
  for (int j = 0; j < 9; ++j) {
    const int a = nbr(b, j, mx, my);
    if (a >= 0) s += W[(int64_t)i * m + a] * C[(int64_t)a * 9 + (8 - j)];
  }
  out[idx] = s;
}

// Whole coarse solve, one persistent cooperative launch, on the twisted block
// factorisation (middle plane q; Inv_k is W_k above q, Z_k below q, G at q):
//   u_k = Inv_k r_k (all planes, no waiting),
//   top:    v_0 = u_0,       v_k = u_k - M_k v_{k-1}   (k = 1 .. q-1),
//   bottom: v_{nb-1} = u_{nb-1}, v_k = u_k - M_k v_{k+1} (k = nb-2 .. q+1),
//   middle: x_q = u_q - M_q v_{q-1} - N_q v_{q+1},
//   top:    x_k = v_k - N_k x_{k+1} (k = q-1 .. 0),
//   bottom: x_k = v_k - N_k x_{k-1} (k = q+1 .. nb-1),
// with M, N as set up (above q: W_k C_k, W_k Ct_k; below q: Z_k Ct_k, Z_k C_k; at q:
// G C_q, G Ct_q).  The first nbt blocks work on the top planes and the middle, the
// rest on the bottom planes, so the two halves advance together.  One matrix row per
// wavefront (RPB rows per block); the neighbouring plane's vector is staged in LDS
// once per block; the next matrix row is requested before the wait for that vector,
// so its loads overlap the wait.
// TM: element type of the stored dense blocks (FP64, or FP32 for the mixed
// protocols); vectors and sums are FP64 either way
template <typename TM>
struct CoarseArgs2 {
  int m, nb, q, nbt;
  const TM *W, *M, *N;
  const double *r;
  double *u, *v, *x;
  int *status;
};

template <int MPL, int RPB, typename TM>
__global__ void __launch_bounds__(64 * RPB) k_coarse_mn(CoarseArgs2<TM> a) {
  extern __shared__ double vl[];
  const int m = a.m, nb = a.nb, q = a.q;
  const bool top = blockIdx.x < a.nbt;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int row = (top ? blockIdx.x : blockIdx.x - a.nbt) * RPB + wid;
  const bool has_row = row < m;
  const size_t mm = (size_t)m * m;
  TM wr[MPL];
  // this wavefront's matrix row: loads without branches (column index clamped; the
  // entries past m are never used), left in flight until the next row_dot
  auto load_row = [&](const TM *mat) {
    const TM *Wr = mat + (size_t)(has_row ? row : 0) * m;
#pragma unroll
    for (int j = 0; j < MPL; ++j) wr[j] = Wr[min(lane + 64 * j, m - 1)];
  };
  // r_k into LDS: each thread's (at most 4) entries loaded together
  auto stage = [&](const double *vp) {
    double t[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) t[j] = vp[min((int)(threadIdx.x + blockDim.x * j), m - 1)];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = threadIdx.x + blockDim.x * j;
      if (i < m) vl[i] = t[j];
    }
    __syncthreads();
  };
  // a vector produced by other blocks in this launch into LDS: each entry polled
  // until it is no longer kEmpty
  auto stage_wait = [&](const double *vp) {
    unsigned long long t[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) t[j] = ld_agent_bits(vp + min((int)(threadIdx.x + blockDim.x * j), m - 1));
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = threadIdx.x + blockDim.x * j;
      if (i < m) {
        long spins = 0;
        while (t[j] == kEmpty) {
          __builtin_amdgcn_s_sleep(1);
          t[j] = ld_agent_bits(vp + i);
          if (++spins > (1l << 26)) {
            atomicCAS(a.status, 0, -1);
            break;
          }
        }
        vl[i] = __builtin_bit_cast(double, t[j]);
      }
    }
    __syncthreads();
  };
  auto row_dot = [&]() {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < MPL; ++j) {
      const int c = lane + 64 * j;
      if (c < m) acc += (double)wr[j] * vl[c];
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    return acc;
  };
  auto own = [&](double *arr, int k) { return arr + (size_t)k * m + row; };
  auto put = [&](double *arr, int k, double val) {
    if (has_row && lane == 0) st_agent(own(arr, k), val);
  };
  auto own_v = [&](int k) { return __builtin_bit_cast(double, ld_agent_bits(own(a.v, k))); };
  // phase 0: u_k = Inv_k r_k over this side's planes (top: 0 .. q, bottom: q+1 .. nb-1)
  const int k0 = top ? 0 : q + 1, k1 = top ? q : nb - 1;
  load_row(a.W + k0 * mm);
  for (int k = k0; k <= k1; ++k) {
    stage(a.r + (size_t)k * m);
    const double acc = row_dot();
    if (k < k1) load_row(a.W + (k + 1) * mm);
    if (has_row && lane == 0) a.u[(size_t)k * m + row] = acc;
    __syncthreads();
  }
  auto own_u = [&](int k) { return a.u[(size_t)k * m + row]; };
  if (top) {
    // forward sweep down to q - 1, then the middle plane
    if (q >= 1) put(a.v, 0, own_u(0));
    if (q >= 2) load_row(a.M + mm);
    for (int k = 1; k <= q - 1; ++k) {
      stage_wait(a.v + (size_t)(k - 1) * m);
      const double acc = row_dot();
      load_row(a.M + (k + 1 <= q - 1 ? k + 1 : q) * mm);
      put(a.v, k, own_u(k) - acc);
      __syncthreads();
    }
    double xq = own_u(q);
    if (q >= 1) {
      if (q == 1) load_row(a.M + q * mm);
      stage_wait(a.v + (size_t)(q - 1) * m);
      xq -= row_dot();
      __syncthreads();
    }
    if (q + 1 < nb) {
      load_row(a.N + q * mm);
      stage_wait(a.v + (size_t)(q + 1) * m);
      xq -= row_dot();
      __syncthreads();
    }
    put(a.x, q, xq);
    // back substitution upwards: x_k = v_k - N_k x_{k+1}
    if (q >= 1) load_row(a.N + (q - 1) * mm);
    for (int k = q - 1; k >= 0; --k) {
      stage_wait(a.x + (size_t)(k + 1) * m);
      const double acc = row_dot();
      if (k > 0) load_row(a.N + (k - 1) * mm);
      put(a.x, k, own_v(k) - acc);
      __syncthreads();
    }
  } else {
    // forward sweep up to q + 1
    put(a.v, nb - 1, own_u(nb - 1));
    if (nb - 2 >= q + 1) load_row(a.M + (nb - 2) * mm);
    for (int k = nb - 2; k >= q + 1; --k) {
      stage_wait(a.v + (size_t)(k + 1) * m);
      const double acc = row_dot();
      put(a.v, k, own_u(k) - acc);
      if (k > q + 1) load_row(a.M + (k - 1) * mm);
      __syncthreads();
    }
    // back substitution downwards: x_k = v_k - N_k x_{k-1}
    load_row(a.N + (q + 1) * mm);
    for (int k = q + 1; k <= nb - 1; ++k) {
      stage_wait(a.x + (size_t)(k - 1) * m);
      const double acc = row_dot();
      if (k < nb - 1) load_row(a.N + (k + 1) * mm);
      put(a.x, k, own_v(k) - acc);
      __syncthreads();
    }
  }
}

// the free coarse values into the plane-blocked order of the coarse solve, and
// its sweep vectors v, x (as many entries) set to kEmpty for the solve that follows
__global__ void k_coarse_gather(int nfree, int bx0, int by0, int bz0, int mx, int my, int NX, int NY,
                                const double *rc, double *blk, double *v, double *xv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nfree) return;
  int x = i % mx, y = (i / mx) % my, z = i / (mx * my);
  blk[i] = rc[(bx0 + x) + (int64_t)NX * ((by0 + y) + (int64_t)NY * (bz0 + z))];
  v[i] = __builtin_bit_cast(double, kEmpty);
  xv[i] = __builtin_bit_cast(double, kEmpty);
}

__global__ void k_coarse_scatter(int ncoarse, int bx0, int by0, int bz0, int mx, int my, int mz, int NX, int NY,
                                 const double *blk, double *xc) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ncoarse) return;
  int X = g % NX - bx0, Y = (g / NX) % NY - by0, Z = g / (NX * NY) - bz0;
  bool in = X >= 0 && X < mx && Y >= 0 && Y < my && Z >= 0 && Z < mz;
  xc[g] = in ? blk[X + mx * (Y + my * Z)] : 0.0;
}

}  // namespace

void launch_fill(double *y, double v, int64_t n, hipStream_t s) { k_fill<<<nblk(n), kBS, 0, s>>>(y, v, n); }
void launch_cast_d2f(const double *x, float *y, int64_t n, hipStream_t s) { k_d2f<<<nblk(n), kBS, 0, s>>>(x, y, n); }
void launch_cast_f2d(const float *x, double *y, int64_t n, hipStream_t s) { k_f2d<<<nblk(n), kBS, 0, s>>>(x, y, n); }
void launch_f2d_scale(double a, const float *x, double *y, int64_t n, hipStream_t s) {
  k_f2d_scale<<<nblk(n), kBS, 0, s>>>(a, x, y, n);
}
void launch_f2d_axpy(double a, const float *x, double *y, int64_t n, hipStream_t s) {
  k_f2d_axpy<<<nblk(n), kBS, 0, s>>>(a, x, y, n);
}
void launch_axpy(double a, const double *x, double *y, int64_t n, hipStream_t s) {
  k_axpy<<<nblk(n), kBS, 0, s>>>(a, x, y, n);
}
void launch_xpby(const double *x, double b, double *y, int64_t n, hipStream_t s) {
  k_xpby<<<nblk(n), kBS, 0, s>>>(x, b, y, n);
}
void launch_xpby_dev(const double *x, const double *num, const double *cross, const double *den, double *y,
                     int64_t n, hipStream_t s) {
  k_xpby_dev<<<nblk(n), kBS, 0, s>>>(x, num, cross, den, y, n);
}
void launch_sub(const double *x, const double *y, double *z, int64_t n, hipStream_t s) {
  k_sub<<<nblk(n), kBS, 0, s>>>(x, y, z, n);
}
template <typename T>
void launch_deinterleave(const T *u, T *v, int nv, int64_t ld, int64_t n, hipStream_t s) {
  k_deinterleave<T><<<nblk(n), kBS, 0, s>>>(u, v, nv, ld, n);
}
template <typename T>
void launch_interleave(const T *v, T *u, int nv, int64_t ld, int64_t n, hipStream_t s) {
  k_interleave<T><<<nblk(n), kBS, 0, s>>>(v, u, nv, ld, n);
}
template void launch_deinterleave<double>(const double *, double *, int, int64_t, int64_t, hipStream_t);
template void launch_deinterleave<float>(const float *, float *, int, int64_t, int64_t, hipStream_t);
template void launch_interleave<double>(const double *, double *, int, int64_t, int64_t, hipStream_t);
template void launch_interleave<float>(const float *, float *, int, int64_t, int64_t, hipStream_t);
template void launch_deinterleave<unsigned short>(const unsigned short *, unsigned short *, int, int64_t, int64_t,
                                                  hipStream_t);
template void launch_interleave<unsigned short>(const unsigned short *, unsigned short *, int, int64_t, int64_t,
                                                hipStream_t);

void launch_scale_copy(double a, const double *x, double *y, int64_t n, hipStream_t s) {
  k_scale_copy<<<nblk(n), kBS, 0, s>>>(a, x, y, n);
}

int dots_partials_size() { return 3 * kDotBlocks; }
void launch_axpy_f(float a, const float *x, float *y, int64_t n, hipStream_t s) {
  k_axpy_f<<<nblk(n), kBS, 0, s>>>(a, x, y, n);
}
void launch_xpby_f(const float *x, float b, float *y, int64_t n, hipStream_t s) {
  k_xpby_f<<<nblk(n), kBS, 0, s>>>(x, b, y, n);
}
void launch_sub_f(const float *x, const float *y, float *z, int64_t n, hipStream_t s) {
  k_sub_f<<<nblk(n), kBS, 0, s>>>(x, y, z, n);
}
void launch_scale_copy_f(float a, const float *x, float *y, int64_t n, hipStream_t s) {
  k_scale_copy_f<<<nblk(n), kBS, 0, s>>>(a, x, y, n);
}
void launch_fill_f(float *y, float v, int64_t n, hipStream_t s) { k_fill_f<<<nblk(n), kBS, 0, s>>>(y, v, n); }
void launch_add_f2d(const float *x, double *y, int64_t n, hipStream_t s) {
  k_add_f2d<<<nblk(n), kBS, 0, s>>>(x, y, n);
}
void launch_add_d2f(const double *t, float *z, int64_t n, hipStream_t s) {
  k_add_d2f<<<nblk(n), kBS, 0, s>>>(t, z, n);
}
void launch_dots_f(int npairs, const float *const *xs, const float *const *ys, int64_t n, double *partials,
                   double *out, hipStream_t s) {
  DotArgsF a{};
  for (int k = 0; k < npairs; ++k) {
    a.x[k] = xs[k];
    a.y[k] = ys[k];
  }
  k_dot_partial_f<<<kDotBlocks, kBS, 0, s>>>(npairs, a, n, partials);
  k_dot_final<<<1, kBS, 0, s>>>(npairs, kDotBlocks, partials, out);
}
void launch_cg_update_f(float a, const float *p, const float *Ap, float *x, float *r, float *ro, int64_t n,
                        double *partials, double *out, hipStream_t s) {
  k_cg_update_f<<<kDotBlocks, kBS, 0, s>>>(a, p, Ap, x, r, ro, n, partials);
  k_dot_final<<<1, kBS, 0, s>>>(1, kDotBlocks, partials, out);
}

void launch_cg_update(const double *num, const double *den, const double *p, const double *Ap, double *x,
                      double *r, double *ro, int64_t n, double *partials, double *out, hipStream_t s) {
  k_cg_update<<<kDotBlocks, kBS, 0, s>>>(num, den, p, Ap, x, r, ro, n, partials);
  k_dot_final<<<1, kBS, 0, s>>>(1, kDotBlocks, partials, out);
}

void launch_dots(int npairs, const double *const *xs, const double *const *ys, int64_t n, double *partials,
                 double *out, hipStream_t s) {
  DotArgs a{};
  for (int k = 0; k < npairs; ++k) {
    a.x[k] = xs[k];
    a.y[k] = ys[k];
  }
  k_dot_partial<<<kDotBlocks, kBS, 0, s>>>(npairs, a, n, partials);
  k_dot_final<<<1, kBS, 0, s>>>(npairs, kDotBlocks, partials, out);
}

void launch_schur_update(int m, int mx, const double *Wprev, const double *C, const double *Akk, double *Dk,
                         hipStream_t s) {
  int64_t n = (int64_t)m * m;
  k_schur_update<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(m, mx, Wprev, C, Akk, Dk);
}

void launch_sweep_inverse(int m, double *W, double *tmp, int *status, hipStream_t s) {
  int64_t n = (int64_t)m * m;
  unsigned nb = (unsigned)((n + 255) / 256);
  double *a = W, *b = tmp;
  for (int k = 0; k < m; ++k) {
    k_sweep<<<nb, 256, 0, s>>>(m, k, a, b, status);
    double *t = a;
    a = b;
    b = t;
  }
  // a holds -A^{-1}; bring it to W with the sign flipped
  if (a != W) {
    hipMemcpyAsync(W, a, sizeof(double) * n, hipMemcpyDeviceToDevice, s);
  }
  k_negate<<<nblk(n), kBS, 0, s>>>(W, n);
}

void launch_coarse_wc(int m, int mx, int my, const double *W, const double *C, double *out, hipStream_t s) {
  const int64_t n = (int64_t)m * m;
  k_coarse_wc<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(m, mx, my, W, C, out);
}

int coarse_blocks(int m) { return m <= 1024 ? (m + 3) / 4 : (m + 15) / 16; }

template <typename TM>
static int coarse_solve(int m, int nb, int q, const TM *W, const TM *M, const TM *N, const double *r, double *u,
                        double *v, double *x, int *status, hipStream_t s) {
  const bool small = m <= 1024;
  const int nbt = coarse_blocks(m);
  const int blocks = q + 1 < nb ? 2 * nbt : nbt;
  const int64_t nv = (int64_t)m * nb;
  CoarseArgs2<TM> a{m, nb, q, nbt, W, M, N, r, u, v, x, status};
  void *args[] = {&a};
  const void *fn;
  const int mpl = (m + 63) / 64;
  if (small) {
    if (mpl <= 4) fn = (const void *)k_coarse_mn<4, 4, TM>;
    else if (mpl <= 8) fn = (const void *)k_coarse_mn<8, 4, TM>;
    else fn = (const void *)k_coarse_mn<16, 4, TM>;
  } else {
    if (mpl <= 32) fn = (const void *)k_coarse_mn<32, 16, TM>;
    else if (mpl <= 64) fn = (const void *)k_coarse_mn<64, 16, TM>;
    else return -1;
  }
  hipError_t e = hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(small ? 256 : 1024), args, sizeof(double) * m, s);
  return e == hipSuccess ? 0 : -1;
}

int launch_coarse_solve(int m, int nb, int q, const double *W, const double *M, const double *N, const double *r,
                        double *u, double *v, double *x, int *status, hipStream_t s) {
  return coarse_solve<double>(m, nb, q, W, M, N, r, u, v, x, status, s);
}

int launch_coarse_solve_f(int m, int nb, int q, const float *W, const float *M, const float *N, const double *r,
                          double *u, double *v, double *x, int *status, hipStream_t s) {
  return coarse_solve<float>(m, nb, q, W, M, N, r, u, v, x, status, s);
}

void launch_coarse_gather(int nfree, int bx0, int by0, int bz0, int mx, int my, int NX, int NY, const double *rc,
                          double *blk, double *v, double *x, hipStream_t s) {
  k_coarse_gather<<<(nfree + 255) / 256, 256, 0, s>>>(nfree, bx0, by0, bz0, mx, my, NX, NY, rc, blk, v, x);
}

void launch_coarse_scatter(int ncoarse, int bx0, int by0, int bz0, int mx, int my, int mz, int NX, int NY,
                           const double *blk, double *xc, hipStream_t s) {
  k_coarse_scatter<<<(ncoarse + 255) / 256, 256, 0, s>>>(ncoarse, bx0, by0, bz0, mx, my, mz, NX, NY, blk, xc);
}

}  // namespace rz
