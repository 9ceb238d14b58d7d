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
__global__ void k_axpy(double a, const double *x, double *y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] += a * x[i];
}
__global__ void k_xpby(const double *x, double b, double *y, int64_t n) {
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

// v = W (r - C vprev): every block rebuilds w in LDS, then each wavefront computes
// whole rows of the dense matrix-vector product.
constexpr int kRowsPerBlock = 16;
__global__ void __launch_bounds__(256) k_coarse_fwd(int m, int mx, const double *__restrict__ W,
                                                    const double *__restrict__ C, const double *__restrict__ r,
                                                    const double *__restrict__ vprev, double *__restrict__ v) {
  extern __shared__ double w[];
  int my = m / mx;
  for (int a = threadIdx.x; a < m; a += blockDim.x) {
    double t = r[a];
    if (vprev)
      for (int j = 0; j < 9; ++j) {
        int c = nbr(a, j, mx, my);
        if (c >= 0) t -= C[a * 9 + j] * vprev[c];
      }
    w[a] = t;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int rr = wid; rr < kRowsPerBlock; rr += 4) {
    int row = blockIdx.x * kRowsPerBlock + rr;
    if (row >= m) break;
    const double *Wr = W + (int64_t)row * m;
    double acc = 0.0;
    for (int c = lane; c < m; c += 64) acc += Wr[c] * w[c];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if (lane == 0) v[row] = acc;
  }
}

// x = v - W (C^T xnext)   (xnext == nullptr: x = v)
__global__ void __launch_bounds__(256) k_coarse_bwd(int m, int mx, const double *__restrict__ W,
                                                    const double *__restrict__ Ct, const double *__restrict__ v,
                                                    const double *__restrict__ xnext, double *__restrict__ x) {
  extern __shared__ double w[];
  int my = m / mx;
  if (!xnext) {
    for (int a = blockIdx.x * kRowsPerBlock + threadIdx.x; a < min(m, (int)(blockIdx.x + 1) * kRowsPerBlock);
         a += blockDim.x)
      x[a] = v[a];
    return;
  }
  for (int a = threadIdx.x; a < m; a += blockDim.x) {
    double t = 0.0;
    for (int j = 0; j < 9; ++j) {
      int c = nbr(a, j, mx, my);
      if (c >= 0) t += Ct[a * 9 + j] * xnext[c];
    }
    w[a] = t;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int rr = wid; rr < kRowsPerBlock; rr += 4) {
    int row = blockIdx.x * kRowsPerBlock + rr;
    if (row >= m) break;
    const double *Wr = W + (int64_t)row * m;
    double acc = 0.0;
    for (int c = lane; c < m; c += 64) acc += Wr[c] * w[c];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if (lane == 0) x[row] = v[row] - acc;
  }
}

__global__ void k_coarse_gather(int nfree, int bx0, int by0, int bz0, int mx, int my, int NX, int NY,
                                const double *rc, double *blk) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nfree) return;
  int x = i % mx, y = (i / mx) % my, z = i / (mx * my);
  blk[i] = rc[(bx0 + x) + (int64_t)NX * ((by0 + y) + (int64_t)NY * (bz0 + z))];
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
void launch_axpy(double a, const double *x, double *y, int64_t n, hipStream_t s) {
  k_axpy<<<nblk(n), kBS, 0, s>>>(a, x, y, n);
}
void launch_xpby(const double *x, double b, double *y, int64_t n, hipStream_t s) {
  k_xpby<<<nblk(n), kBS, 0, s>>>(x, b, y, n);
}
void launch_sub(const double *x, const double *y, double *z, int64_t n, hipStream_t s) {
  k_sub<<<nblk(n), kBS, 0, s>>>(x, y, z, n);
}
void launch_scale_copy(double a, const double *x, double *y, int64_t n, hipStream_t s) {
  k_scale_copy<<<nblk(n), kBS, 0, s>>>(a, x, y, n);
}

int dots_partials_size() { return 3 * kDotBlocks; }

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

void launch_coarse_fwd(int m, int mx, const double *W, const double *C, const double *r, const double *vprev,
                       double *v, hipStream_t s) {
  unsigned nb = (unsigned)((m + kRowsPerBlock - 1) / kRowsPerBlock);
  k_coarse_fwd<<<nb, 256, sizeof(double) * m, s>>>(m, mx, W, C, r, vprev, v);
}

void launch_coarse_bwd(int m, int mx, const double *W, const double *Ct, const double *v, const double *xnext,
                       double *x, hipStream_t s) {
  unsigned nb = (unsigned)((m + kRowsPerBlock - 1) / kRowsPerBlock);
  k_coarse_bwd<<<nb, 256, sizeof(double) * m, s>>>(m, mx, W, Ct, v, xnext, x);
}

void launch_coarse_gather(int nfree, int bx0, int by0, int bz0, int mx, int my, int NX, int NY, const double *rc,
                          double *blk, hipStream_t s) {
  k_coarse_gather<<<(nfree + 255) / 256, 256, 0, s>>>(nfree, bx0, by0, bz0, mx, my, NX, NY, rc, blk);
}

void launch_coarse_scatter(int ncoarse, int bx0, int by0, int bz0, int mx, int my, int mz, int NX, int NY,
                           const double *blk, double *xc, hipStream_t s) {
  k_coarse_scatter<<<(ncoarse + 255) / 256, 256, 0, s>>>(ncoarse, bx0, by0, bz0, mx, my, mz, NX, NY, blk, xc);
}

}  // namespace rz
