// Small MLP (FP32) that predicts the separable auxiliary weights of a cell from
// its features: nin -> nhid (tanh) -> nhid (tanh) -> nout, mean-squared-error loss,
// Adam.  Hand-written HIP kernels for inference, backward pass and update; every
// reduction runs in a fixed order (deterministic).  Parameters are packed as
// W1 (nhid x nin), b1, W2 (nhid x nhid), b2, W3 (nout x nhid), b3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/rz.h"

namespace rz {
void *ctx_stream(const rz_ctx *ctx);        // the context's HIP stream (rz_api.cpp)
void ctx_retain(rz_ctx *ctx, int delta);   // count of live objects on a context
}

struct rz_mlp {
  rz_ctx *ctx = nullptr;
  int nin = 0, nhid = 0, nout = 0;
  hipStream_t stream = nullptr;
  size_t nparam = 0;
  float *param = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  int64_t step = 0;
  // activations of the last forward pass (capacity cap rows)
  int64_t cap = 0;
  float *a1 = nullptr, *a2 = nullptr, *y = nullptr, *g2 = nullptr, *g1 = nullptr, *gy = nullptr, *lossbuf = nullptr;
  int *perm = nullptr;  // one epoch's row permutation (capacity pcap)
  int64_t pcap = 0;
  float *xb = nullptr, *yb = nullptr;
  std::string err;
};

namespace {

constexpr int kBS = 256;

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBS - 1) / kBS); }

// out[i, o] = act(sum_k in[i, k] W[o, k] + b[o]); act = tanh if tanh_act
__global__ void k_dense_fwd(const float *__restrict__ in, const float *__restrict__ W, const float *__restrict__ b,
                            float *__restrict__ out, int64_t nb, int nin, int nout, int tanh_act) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb * nout) return;
  const int64_t i = t / nout;
  const int o = t % nout;
  float s = b[o];
  for (int k = 0; k < nin; ++k) s += in[i * nin + k] * W[o * nin + k];
  out[t] = tanh_act ? tanhf(s) : s;
}

// gy = 2 (y - Y) / (nb * nout); lossbuf[i] = sum_o (y - Y)^2 for row i
__global__ void k_mse(const float *__restrict__ y, const float *__restrict__ Y, float *__restrict__ gy,
                      float *__restrict__ lossbuf, int64_t nb, int nout, float scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  float s = 0;
  for (int o = 0; o < nout; ++o) {
    const float d = y[i * nout + o] - Y[i * nout + o];
    gy[i * nout + o] = 2.0f * d * scale;
    s += d * d;
  }
  lossbuf[i] = s;
}

// gin[i, k] = (sum_o gout[i, o] W[o, k]) * (1 - a[i, k]^2)
__global__ void k_dense_bwd_in(const float *__restrict__ gout, const float *__restrict__ W, const float *__restrict__ a,
                               float *__restrict__ gin, int64_t nb, int nin, int nout) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb * nin) return;
  const int64_t i = t / nin;
  const int k = t % nin;
  float s = 0;
  for (int o = 0; o < nout; ++o) s += gout[i * nout + o] * W[o * nin + k];
  gin[t] = s * (1.0f - a[t] * a[t]);
}

// gW[o, k] = sum_i gout[i, o] in[i, k]; gb[o] = sum_i gout[i, o] (thread per (o, k), k = nin -> bias)
__global__ void k_dense_bwd_w(const float *__restrict__ gout, const float *__restrict__ in, float *__restrict__ gW,
                              float *__restrict__ gb, int64_t nb, int nin, int nout) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nout * (nin + 1)) return;
  const int o = t / (nin + 1), k = t % (nin + 1);
  float s = 0;
  if (k < nin) {
    for (int64_t i = 0; i < nb; ++i) s += gout[i * nout + o] * in[i * nin + k];
    gW[o * nin + k] = s;
  } else {
    for (int64_t i = 0; i < nb; ++i) s += gout[i * nout + o];
    gb[o] = s;
  }
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       int64_t n, float lr, float b1, float b2, float c1, float c2, float eps) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float gt = g[t];
  const float mt = b1 * m[t] + (1.0f - b1) * gt;
  const float vt = b2 * v[t] + (1.0f - b2) * gt * gt;
  m[t] = mt;
  v[t] = vt;
  p[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
}

__global__ void k_gather_rows(const float *__restrict__ src, const int *__restrict__ idx, float *__restrict__ dst,
                              int64_t nb, int w) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb * w) return;
  dst[t] = src[(int64_t)idx[t / w] * w + t % w];
}

struct Views {
  const float *W1, *b1, *W2, *b2, *W3, *b3;
};

Views views(const rz_mlp *h, const float *base) {
  const int a = h->nin, H = h->nhid, o = h->nout;
  Views v;
  v.W1 = base;
  v.b1 = v.W1 + (size_t)H * a;
  v.W2 = v.b1 + H;
  v.b2 = v.W2 + (size_t)H * H;
  v.W3 = v.b2 + H;
  v.b3 = v.W3 + (size_t)o * H;
  return v;
}

rz_status mfail(rz_mlp *h, rz_status st, const std::string &msg) {
  if (h) h->err = msg;
  return st;
}

rz_status ensure_cap(rz_mlp *h, int64_t nb) {
  if (nb <= h->cap) return RZ_OK;
  hipFree(h->a1);
  hipFree(h->a2);
  hipFree(h->y);
  hipFree(h->g2);
  hipFree(h->g1);
  hipFree(h->gy);
  hipFree(h->lossbuf);
  hipFree(h->xb);
  hipFree(h->yb);
  h->cap = 0;
  const size_t H = h->nhid, o = h->nout;
  if (hipMalloc(&h->a1, sizeof(float) * nb * H) || hipMalloc(&h->a2, sizeof(float) * nb * H) ||
      hipMalloc(&h->y, sizeof(float) * nb * o) || hipMalloc(&h->g2, sizeof(float) * nb * H) ||
      hipMalloc(&h->g1, sizeof(float) * nb * H) || hipMalloc(&h->gy, sizeof(float) * nb * o) ||
      hipMalloc(&h->lossbuf, sizeof(float) * nb) || hipMalloc(&h->xb, sizeof(float) * nb * h->nin) ||
      hipMalloc(&h->yb, sizeof(float) * nb * o))
    return mfail(h, RZ_ERR_OOM, "hipMalloc of MLP workspace");
  h->cap = nb;
  return RZ_OK;
}

void forward(rz_mlp *h, const float *X, int64_t nb) {
  const Views p = views(h, h->param);
  hipStream_t s = h->stream;
  k_dense_fwd<<<nblk(nb * h->nhid), kBS, 0, s>>>(X, p.W1, p.b1, h->a1, nb, h->nin, h->nhid, 1);
  k_dense_fwd<<<nblk(nb * h->nhid), kBS, 0, s>>>(h->a1, p.W2, p.b2, h->a2, nb, h->nhid, h->nhid, 1);
  k_dense_fwd<<<nblk(nb * h->nout), kBS, 0, s>>>(h->a2, p.W3, p.b3, h->y, nb, h->nhid, h->nout, 0);
}

// gradient of the mean squared error into h->grad (after forward on the same rows)
void backward(rz_mlp *h, const float *X, const float *Y, int64_t nb) {
  const Views p = views(h, h->param);
  Views g = views(h, h->grad);
  hipStream_t s = h->stream;
  const int a = h->nin, H = h->nhid, o = h->nout;
  k_mse<<<nblk(nb), kBS, 0, s>>>(h->y, Y, h->gy, h->lossbuf, nb, o, 1.0f / (float)(nb * o));
  k_dense_bwd_w<<<nblk(o * (H + 1)), kBS, 0, s>>>(h->gy, h->a2, (float *)g.W3, (float *)g.b3, nb, H, o);
  k_dense_bwd_in<<<nblk(nb * H), kBS, 0, s>>>(h->gy, p.W3, h->a2, h->g2, nb, H, o);
  k_dense_bwd_w<<<nblk(H * (H + 1)), kBS, 0, s>>>(h->g2, h->a1, (float *)g.W2, (float *)g.b2, nb, H, H);
  k_dense_bwd_in<<<nblk(nb * H), kBS, 0, s>>>(h->g2, p.W2, h->a1, h->g1, nb, H, H);
  k_dense_bwd_w<<<nblk(H * (a + 1)), kBS, 0, s>>>(h->g1, X, (float *)g.W1, (float *)g.b1, nb, a, H);
}

double read_loss(rz_mlp *h, int64_t nb) {
  std::vector<float> l(nb);
  hipMemcpyAsync(l.data(), h->lossbuf, sizeof(float) * nb, hipMemcpyDeviceToHost, h->stream);
  hipStreamSynchronize(h->stream);
  double s = 0;
  for (float v : l) s += v;
  return s / ((double)nb * h->nout);
}

// SplitMix64 (Steele, Lea & Flood 2014): uniform doubles in [-1, 1)
uint64_t splitmix_next(uint64_t &state) {
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

extern "C" {

rz_status rz_mlp_create(rz_ctx *ctx, int32_t nin, int32_t nhid, int32_t nout, uint64_t seed, rz_mlp **out) {
  if (!out || nin < 1 || nhid < 1 || nout < 1) return RZ_ERR_ARG;
  *out = nullptr;
  rz_mlp *h = new rz_mlp();
  h->nin = nin;
  h->nhid = nhid;
  h->nout = nout;
  h->stream = ctx ? (hipStream_t)rz::ctx_stream(ctx) : nullptr;
  h->nparam = (size_t)nhid * nin + nhid + (size_t)nhid * nhid + nhid + (size_t)nout * nhid + nout;
  // Glorot-uniform weights from the SplitMix64 stream `seed` (W1, W2, W3 in turn,
  // row-major), zero biases
  std::vector<float> p(h->nparam, 0.0f);
  uint64_t st = seed;
  const int fo[3] = {nhid, nhid, nout}, fi[3] = {nin, nhid, nhid};
  size_t o = 0;
  for (int l = 0; l < 3; ++l) {
    const double lim = std::sqrt(6.0 / (fi[l] + fo[l]));
    for (size_t k = 0; k < (size_t)fo[l] * fi[l]; ++k) {
      const double u = (double)(splitmix_next(st) >> 11) * 0x1.0p-53;
      p[o + k] = (float)(lim * (2.0 * u - 1.0));
    }
    o += (size_t)fo[l] * fi[l] + fo[l];
  }
  if (hipMalloc(&h->param, sizeof(float) * h->nparam) || hipMalloc(&h->grad, sizeof(float) * h->nparam) ||
      hipMalloc(&h->m, sizeof(float) * h->nparam) || hipMalloc(&h->v, sizeof(float) * h->nparam)) {
    rz_mlp_free(h);
    return RZ_ERR_OOM;
  }
  hipMemcpyAsync(h->param, p.data(), sizeof(float) * h->nparam, hipMemcpyHostToDevice, h->stream);
  hipMemsetAsync(h->m, 0, sizeof(float) * h->nparam, h->stream);
  hipMemsetAsync(h->v, 0, sizeof(float) * h->nparam, h->stream);
  hipMemsetAsync(h->grad, 0, sizeof(float) * h->nparam, h->stream);
  if (hipStreamSynchronize(h->stream) != hipSuccess) {
    rz_mlp_free(h);
    return RZ_ERR_HIP;
  }
  h->ctx = ctx;
  rz::ctx_retain(ctx, 1);
  *out = h;
  return RZ_OK;
}

rz_status rz_mlp_free(rz_mlp *h) {
  if (!h) return RZ_OK;
  hipStreamSynchronize(h->stream);
  rz::ctx_retain(h->ctx, -1);
  for (void *p : {(void *)h->param, (void *)h->grad, (void *)h->m, (void *)h->v, (void *)h->a1, (void *)h->a2,
                  (void *)h->y, (void *)h->g2, (void *)h->g1, (void *)h->gy, (void *)h->lossbuf, (void *)h->xb,
                  (void *)h->yb, (void *)h->perm})
    if (p) hipFree(p);
  delete h;
  return RZ_OK;
}

const char *rz_mlp_last_error(const rz_mlp *h) { return h ? h->err.c_str() : "null MLP"; }

int64_t rz_mlp_nparams(const rz_mlp *h) { return h ? (int64_t)h->nparam : 0; }

rz_status rz_mlp_params(rz_mlp *h, float *host, int32_t set) {
  if (!h || !host) return RZ_ERR_ARG;
  hipError_t e = set ? hipMemcpyAsync(h->param, host, sizeof(float) * h->nparam, hipMemcpyHostToDevice, h->stream)
                     : hipMemcpyAsync(host, h->param, sizeof(float) * h->nparam, hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess) return mfail(h, RZ_ERR_HIP, "params copy");
  if (set) h->step = 0;
  return RZ_OK;
}

rz_status rz_mlp_predict(rz_mlp *h, const float *X, float *Y, int64_t n) {
  if (!h || !X || !Y || n < 0) return RZ_ERR_ARG;
  const int64_t chunk = 1 << 16;
  for (int64_t s = 0; s < n; s += chunk) {
    const int64_t nb = n - s < chunk ? n - s : chunk;
    rz_status st = ensure_cap(h, nb);
    if (st) return st;
    forward(h, X + s * h->nin, nb);
    if (hipMemcpyAsync(Y + s * h->nout, h->y, sizeof(float) * nb * h->nout, hipMemcpyDeviceToDevice, h->stream))
      return mfail(h, RZ_ERR_HIP, "copy of predictions");
  }
  return RZ_OK;
}

rz_status rz_mlp_loss_grad(rz_mlp *h, const float *X, const float *Y, int64_t n, double *loss, float *grad_host) {
  if (!h || !X || !Y || n < 1) return RZ_ERR_ARG;
  rz_status st = ensure_cap(h, n);
  if (st) return st;
  forward(h, X, n);
  backward(h, X, Y, n);
  if (loss) *loss = read_loss(h, n);
  if (grad_host) {
    if (hipMemcpyAsync(grad_host, h->grad, sizeof(float) * h->nparam, hipMemcpyDeviceToHost, h->stream) ||
        hipStreamSynchronize(h->stream))
      return mfail(h, RZ_ERR_HIP, "gradient copy");
  }
  return RZ_OK;
}

rz_status rz_mlp_train(rz_mlp *h, const float *X, const float *Y, int64_t n, int32_t epochs, int32_t batch,
                       float lr, uint64_t seed, double *final_loss) {
  if (!h || !X || !Y || n < 1 || epochs < 0 || batch < 1) return RZ_ERR_ARG;
  const int64_t nb = batch < n ? batch : n;
  rz_status st = ensure_cap(h, nb);
  if (st) return st;
  if (n > h->pcap) {
    if (h->perm) hipFree(h->perm);
    h->perm = nullptr;
    h->pcap = 0;
    if (hipMalloc(&h->perm, sizeof(int) * n)) return mfail(h, RZ_ERR_OOM, "hipMalloc of the permutation");
    h->pcap = n;
  }
  std::vector<int> perm(n);
  uint64_t rs = seed;
  double last = 0.0;
  for (int ep = 0; ep < epochs; ++ep) {
    // Fisher-Yates shuffle of the rows from the SplitMix64 stream
    for (int64_t i = 0; i < n; ++i) perm[i] = (int)i;
    for (int64_t i = n - 1; i > 0; --i) {
      const int64_t j = (int64_t)(splitmix_next(rs) % (uint64_t)(i + 1));
      std::swap(perm[i], perm[j]);
    }
    // the host array changes in the next epoch: wait for the upload
    if (hipMemcpyAsync(h->perm, perm.data(), sizeof(int) * n, hipMemcpyHostToDevice, h->stream) ||
        hipStreamSynchronize(h->stream))
      return mfail(h, RZ_ERR_HIP, "permutation upload");
    for (int64_t s0 = 0; s0 + nb <= n; s0 += nb) {
      k_gather_rows<<<nblk(nb * h->nin), kBS, 0, h->stream>>>(X, h->perm + s0, h->xb, nb, h->nin);
      k_gather_rows<<<nblk(nb * h->nout), kBS, 0, h->stream>>>(Y, h->perm + s0, h->yb, nb, h->nout);
      forward(h, h->xb, nb);
      backward(h, h->xb, h->yb, nb);
      ++h->step;
      const float b1 = 0.9f, b2 = 0.999f;
      const float c1 = 1.0f - std::pow(b1, (float)h->step), c2 = 1.0f - std::pow(b2, (float)h->step);
      k_adam<<<nblk(h->nparam), kBS, 0, h->stream>>>(h->param, h->grad, h->m, h->v, h->nparam, lr, b1, b2, c1, c2,
                                                   1e-8f);
    }
    last = read_loss(h, nb);
  }
  if (final_loss) *final_loss = last;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return mfail(h, RZ_ERR_HIP, "training failed");
  return RZ_OK;
}

rz_status rz_mlp_adam_step(rz_mlp *h, const float *X, const float *Y, int64_t n, float lr) {
  if (!h || !X || !Y || n < 1) return RZ_ERR_ARG;
  rz_status st = ensure_cap(h, n);
  if (st) return st;
  forward(h, X, n);
  backward(h, X, Y, n);
  ++h->step;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - std::pow(b1, (float)h->step), c2 = 1.0f - std::pow(b2, (float)h->step);
  k_adam<<<nblk(h->nparam), kBS, 0, h->stream>>>(h->param, h->grad, h->m, h->v, h->nparam, lr, b1, b2, c1, c2, 1e-8f);
  if (hipStreamSynchronize(h->stream) != hipSuccess) return mfail(h, RZ_ERR_HIP, "Adam step failed");
  return RZ_OK;
}

}  // extern "C"
