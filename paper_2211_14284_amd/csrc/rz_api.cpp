// C ABI (include/rz.h): problem setup on the host and the device, and the
// stream-ordered compute calls that drive the HIP kernels.
#include "../../include/rz.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "kernels.hpp"
#include "lattice.hpp"
#include "geom.hpp"
#include "patch.hpp"
#include "tables1d.hpp"

struct rz_ctx {
  int device = -1;
  hipStream_t stream = nullptr;
  std::string err;
  int nlive = 0;  // problems and MLPs created on this context and not yet freed
};

namespace rz {
void *ctx_stream(const rz_ctx *ctx) { return ctx ? (void *)ctx->stream : nullptr; }
void ctx_retain(rz_ctx *ctx, int delta) {
  if (ctx) ctx->nlive += delta;
}
}  // namespace rz

namespace {

// Workspace of rz_apply_noalloc: one static device array per GPU (each device that
// loads the library holds its own copy until the process ends).  Host code never
// passes `scratch` itself to a kernel; it uses the device address taken once per
// device by scratch_init.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

// With `device` current: record the device address of `scratch` (once per device).
hipError_t scratch_init(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (g_scratch_ptr[device]) return hipSuccess;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void *scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
}

using namespace rz;

struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct rz_problem {
  rz_ctx *ctx = nullptr;
  rz_opts opts{};
  int p = 0, nx = 0, ny = 0, nz = 0;
  unsigned dir = 0;
  int Nx = 0, Ny = 0, Nz = 0;
  int64_t ndofs = 0, nfree = 0, ncells = 0, nvert = 0, ncoarse = 0;
  Tables1D t, t1;
  PatchSymbolic ps;
  std::vector<double> coef;       // ncells * 6
  std::vector<int> erow;          // row of every pattern entry
  std::vector<int64_t> patch_vids;  // non-empty patches (vertex ids)
  double omega = 0.0;
  // device
  LatDev L{};
  PatchDev P{};
  PatchEllDev PE{};
  std::vector<void *> allocs;
  double *coef64 = nullptr, *B64 = nullptr, *A64 = nullptr, *lam64 = nullptr, *E64 = nullptr;
  double *T2_64 = nullptr;  // (p+1) x 2 products A E, then B E (fused coarse correction and residual)
  float *coef32 = nullptr, *B32 = nullptr, *A32 = nullptr, *lam32 = nullptr;
  // H(curl) / H(div): apply only
  int space = RZ_GRAD;
  VecDev V{};
  double *D64 = nullptr;
  float *D32 = nullptr;
  // trilinear / sampled-coefficient path
  bool quad = false;
  QuadTables qt;
  std::vector<double> vert, asmp, bsmp;  // vertices (nvert x 3), 27 samples per cell
  std::vector<double> cellA1;            // p=1 cell matrices (ncells x 64)
  QuadDev<double> Q64{};
  QuadDev<float> Q32{};
  double *f64 = nullptr, *eb64 = nullptr;
  float *f32 = nullptr, *eb32 = nullptr;
  double *rt64 = nullptr, *zb64 = nullptr;
  float *rt32 = nullptr, *zb32 = nullptr, *r32 = nullptr, *z32 = nullptr;
  // inner FP32 solve of the defect-correction protocol
  float *kp32 = nullptr, *kAp32 = nullptr, *ko32 = nullptr, *ke32 = nullptr, *t32 = nullptr, *az32 = nullptr,
        *vr32 = nullptr;
  double *vt = nullptr, *vaz = nullptr, *vr = nullptr, *rc = nullptr, *xc = nullptr, *rt1 = nullptr, *rt2 = nullptr;
  // coarse
  int cm = 0, cmx = 0, cmy = 0, cmz = 0, cbx0 = 0, cby0 = 0, cbz0 = 0, cNX = 0, cNY = 0, cNZ = 0;
  int cq = 0;  // middle plane of the twisted coarse factorisation
  double *cW = nullptr, *cC = nullptr, *cCt = nullptr, *cr = nullptr, *cv = nullptr, *cx = nullptr;
  double *cM = nullptr, *cN = nullptr, *cu = nullptr;
  // FP32 copies of the dense blocks W, M, N (mixed and defect-correction protocols)
  float *cW32 = nullptr, *cM32 = nullptr, *cN32 = nullptr;
  // krylov
  double *kr = nullptr, *kz = nullptr, *kp = nullptr, *kAp = nullptr, *kro = nullptr;
  double *partials = nullptr, *dots = nullptr;
  double *hdots = nullptr;  // pinned host copy of the dot products (8 values)
  int *status = nullptr;
  // per-kernel timing
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
  std::vector<std::pair<int, size_t>> ev_used;  // (kernel id, pool index)
};

namespace {

rz_status fail(rz_ctx *ctx, rz_status st, const std::string &msg) {
  if (ctx) ctx->err = msg;
  return st;
}

rz_status take_device_status(rz_problem *h);

#define HIPCALL(h, expr)                                                                   \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail((h)->ctx, RZ_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
rz_status dalloc(rz_problem *h, T **ptr, size_t count) {
  void *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(&p, sizeof(T) * count);
  if (e != hipSuccess) return fail(h->ctx, RZ_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  h->allocs.push_back(p);
  *ptr = static_cast<T *>(p);
  return RZ_OK;
}

template <typename T>
rz_status upload(rz_problem *h, T **ptr, const std::vector<T> &v) {
  rz_status st = dalloc(h, ptr, v.size());
  if (st != RZ_OK) return st;
  HIPCALL(h, hipMemcpyAsync(*ptr, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, h->ctx->stream));
  return RZ_OK;
}

bool lat_dirichlet_h(const rz_problem *h, int X, int Y, int Z) {
  return ((h->dir & 1u) && X == 0) || ((h->dir & 2u) && X == h->Nx - 1) || ((h->dir & 4u) && Y == 0) ||
         ((h->dir & 8u) && Y == h->Ny - 1) || ((h->dir & 16u) && Z == 0) || ((h->dir & 32u) && Z == h->Nz - 1);
}

bool patch_row_present(const rz_problem *h, int64_t vid, int k, int G[3]) {
  const int nvx = h->nx + 1, nvy = h->ny + 1;
  const int V[3] = {(int)(vid % nvx), (int)((vid / nvx) % nvy), (int)(vid / ((int64_t)nvx * nvy))};
  const int Nd[3] = {h->Nx, h->Ny, h->Nz};
  for (int d = 0; d < 3; ++d) {
    G[d] = V[d] * h->p + h->ps.off[3 * k + d];
    if (G[d] < 0 || G[d] >= Nd[d]) return false;
  }
  return !lat_dirichlet_h(h, G[0], G[1], G[2]);
}

// Entry (r, c) of a patch pattern is kept for slot vid iff some existing cell of the
// star holds both DoFs and couples them (same rule as the device factorisation).
bool patch_entry_allowed(const rz_problem *h, int64_t vid, const int Gr[3], const int Gc[3]) {
  const int nvx = h->nx + 1, nvy = h->ny + 1;
  const int V[3] = {(int)(vid % nvx), (int)((vid / nvx) % nvy), (int)(vid / ((int64_t)nvx * nvy))};
  const int nc[3] = {h->nx, h->ny, h->nz};
  for (int cell = 0; cell < 8; ++cell) {
    int u[3], w[3];
    bool in = true;
    for (int d = 0; d < 3; ++d) {
      int cc = V[d] - 1 + ((cell >> d) & 1);
      u[d] = Gr[d] - cc * h->p;
      w[d] = Gc[d] - cc * h->p;
      in = in && cc >= 0 && cc < nc[d] && u[d] >= 0 && u[d] <= h->p && w[d] >= 0 && w[d] <= h->p;
    }
    if (in && cell_schur_coupled(h->p, u, w)) return true;
  }
  return false;
}

uint64_t splitmix_next(uint64_t &s) {
  s += 0x9E3779B97F4A7C15ull;
  uint64_t z = s;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------------------
// per-kernel timing: events around launches while enabled
// ---------------------------------------------------------------------------------------
struct Timed {
  rz_problem *h;
  int id;
  size_t slot = 0;
  Timed(rz_problem *h_, int id_) : h(h_), id(id_) {
    if (!h->timing) return;
    slot = h->ev_used.size();
    if (slot >= h->ev_pool.size()) {
      hipEvent_t a, b;
      hipEventCreate(&a);
      hipEventCreate(&b);
      h->ev_pool.push_back({a, b});
    }
    h->ev_used.push_back({id, slot});
    hipEventRecord(h->ev_pool[slot].first, h->ctx->stream);
  }
  ~Timed() {
    if (h->timing) hipEventRecord(h->ev_pool[slot].second, h->ctx->stream);
  }
};


// vector updates of the Krylov method and the V-cycle (timed as one group)
void v_axpy(rz_problem *h, double a, const double *x, double *y) {
  Timed t(h, RZ_K_KRYLOV);
  launch_axpy(a, x, y, h->ndofs, h->ctx->stream);
}
void v_xpby(rz_problem *h, const double *x, double b, double *y) {
  Timed t(h, RZ_K_KRYLOV);
  launch_xpby(x, b, y, h->ndofs, h->ctx->stream);
}
void v_sub(rz_problem *h, const double *x, const double *y, double *z) {
  Timed t(h, RZ_K_KRYLOV);
  launch_sub(x, y, z, h->ndofs, h->ctx->stream);
}
void v_scale_copy(rz_problem *h, double a, const double *x, double *y) {
  Timed t(h, RZ_K_KRYLOV);
  launch_scale_copy(a, x, y, h->ndofs, h->ctx->stream);
}

// ---------------------------------------------------------------------------------------
// operator pieces on the device
// ---------------------------------------------------------------------------------------
rz_status do_apply64(rz_problem *h, const double *x, double *y) {
  Timed t(h, RZ_K_APPLY);
  if (h->space != RZ_GRAD) {
    if (launch_apply_vec<double>(h->V, h->coef64, h->B64, h->D64, x, y, h->eb64, h->ctx->stream))
      return fail(h->ctx, RZ_ERR_ARG, "unsupported degree");
  } else if (h->quad) {
    launch_apply_quad_cells<double>(h->L, h->Q64, x, y, h->eb64, h->ctx->stream);
    launch_apply_gather<double>(h->L, x, h->eb64, y, h->ctx->stream);
  } else {
    launch_apply_grad<double>(h->L, h->coef64, h->t.B.data(), h->t.A.data(), x, nullptr, y, h->eb64,
                              h->ctx->stream);
  }
  return RZ_OK;
}

// out = b - A x (fused into the apply's stores for the sum-factorised H(grad) operator)
rz_status do_residual64(rz_problem *h, const double *b, const double *x, double *out) {
  if (h->space == RZ_GRAD && !h->quad) {
    Timed t(h, RZ_K_APPLY);
    launch_apply_grad<double>(h->L, h->coef64, h->t.B.data(), h->t.A.data(), x, b, out, h->eb64, h->ctx->stream);
    return RZ_OK;
  }
  rz_status e = do_apply64(h, x, h->vaz);
  if (e) return e;
  v_sub(h, b, h->vaz, out);
  return RZ_OK;
}

// z = scale * M r; with acc: acc += w * M r (z then holds only the plane values)
template <typename T>
rz_status relax_steps(rz_problem *h, const T *coef, const T *A, const T *lam, const T *f, T *rt, T *zb,
                      const T *r, T *z, T scale = T(1), T w = T(0), T *acc = nullptr) {
  hipStream_t s = h->ctx->stream;
  {
    Timed t(h, RZ_K_CONDENSE);
    launch_condense_grad<T>(h->L, coef, A, lam, r, rt, s);
  }
  {
    Timed t(h, RZ_K_PATCH);
    if (launch_patch_solve<T>(h->L, h->PE, f, rt, zb, s)) return fail(h->ctx, RZ_ERR_HIP, "patch solve launch failed");
  }
  {
    Timed t(h, RZ_K_EXPAND);
    launch_expand_grad<T>(h->L, h->P, coef, A, lam, r, zb, z, scale, w, acc, s);
  }
  return RZ_OK;
}

rz_status do_relax64(rz_problem *h, const double *r, double *z, double scale = 1.0, double w = 0.0,
                     double *acc = nullptr) {
  return relax_steps<double>(h, h->coef64, h->A64, h->lam64, h->f64, h->rt64, h->zb64, r, z, scale, w, acc);
}

rz_status do_relax32(rz_problem *h, const float *r, float *z, float scale = 1.0f, float w = 0.0f,
                     float *acc = nullptr) {
  return relax_steps<float>(h, h->coef32, h->A32, h->lam32, h->f32, h->rt32, h->zb32, r, z, scale, w, acc);
}

// fine relaxation on FP64 vectors in the precision of the problem's protocol
// (FP32 relaxation for the mixed and defect-correction protocols):
// z = scale * M r, or with acc: acc += w * M r (z is then scratch)
rz_status do_relax_prec(rz_problem *h, const double *r, double *z, double scale = 1.0, double w = 0.0,
                        double *acc = nullptr) {
  if (h->opts.precision != RZ_PREC_F64) {
    launch_cast_d2f(r, h->r32, h->ndofs, h->ctx->stream);
    if (rz_status e = do_relax32(h, h->r32, h->z32)) return e;
    if (acc) launch_f2d_axpy(w, h->z32, acc, h->ndofs, h->ctx->stream);
    else launch_f2d_scale(scale, h->z32, z, h->ndofs, h->ctx->stream);
    return RZ_OK;
  }
  return do_relax64(h, r, z, scale, w, acc);
}

// Coarse solve; f32 selects the FP32 copies of the dense blocks (V-cycles of the
// mixed protocols), otherwise FP64 throughout.
rz_status do_coarse(rz_problem *h, const double *rcv, double *xcv, bool f32 = false) {
  Timed tm(h, RZ_K_COARSE);
  hipStream_t s = h->ctx->stream;
  const int m = h->cm, nb = h->cmz;
  launch_coarse_gather(m * nb, h->cbx0, h->cby0, h->cbz0, h->cmx, h->cmy, h->cNX, h->cNY, rcv, h->cr, h->cv, h->cx,
                       s);
  const int rc = f32 && h->cW32
                     ? launch_coarse_solve_f(m, nb, h->cq, h->cW32, h->cM32, h->cN32, h->cr, h->cu, h->cv, h->cx,
                                             h->status, s)
                     : launch_coarse_solve(m, nb, h->cq, h->cW, h->cM, h->cN, h->cr, h->cu, h->cv, h->cx, h->status, s);
  if (rc) return fail(h->ctx, RZ_ERR_HIP, "cooperative launch of the coarse solve failed");
  launch_coarse_scatter((int)h->ncoarse, h->cbx0, h->cby0, h->cbz0, h->cmx, h->cmy, h->cmz, h->cNX, h->cNY,
                        h->cx, xcv, s);
  return RZ_OK;
}

rz_status do_vcycle(rz_problem *h, const double *r, double *z) {
  hipStream_t s = h->ctx->stream;
  const int64_t n = h->ndofs;
  const double w = h->omega;
  if (rz_status e = do_relax_prec(h, r, z, w)) return e;  // z = w M r
  do_residual64(h, r, z, h->vr);           // r1 = r - A z
  {
    Timed tm(h, RZ_K_TRANSFER);
    launch_restrict_grad(h->L, h->E64, h->vr, h->rc, h->rt1, h->rt2, s);
  }
  do_coarse(h, h->rc, h->xc, h->opts.precision != RZ_PREC_F64);
  if (h->T2_64) {  // z += P xc and r2 = r1 - A P xc in one pass
    Timed tm(h, RZ_K_TRANSFER);
    launch_prolong_residual_grad(h->L, h->E64, h->T2_64, h->coef64, h->xc, z, h->vr, s);
  } else {
    {
      Timed tm(h, RZ_K_TRANSFER);
      launch_prolong_add_grad(h->L, h->E64, h->xc, z, s);   // z += P A0^{-1} P^T r1
    }
    do_residual64(h, r, z, h->vr);           // r2 = r - A z
  }
  if (rz_status e = do_relax_prec(h, h->vr, h->vt, 1.0, w, z)) return e;  // z += w M r2
  launch_dirichlet_copy(h->L, r, z, s);
  return RZ_OK;
}

rz_status do_apply32(rz_problem *h, const float *x, float *y) {
  Timed t(h, RZ_K_APPLY);
  hipStream_t s = h->ctx->stream;
  if (h->space != RZ_GRAD) {
    if (launch_apply_vec<float>(h->V, h->coef32, h->B32, h->D32, x, y, h->eb32, s))
      return fail(h->ctx, RZ_ERR_ARG, "unsupported degree");
  } else if (h->quad) {
    launch_apply_quad_cells<float>(h->L, h->Q32, x, y, h->eb32, s);
    launch_apply_gather<float>(h->L, x, h->eb32, y, s);
  } else {
    launch_apply_grad<float>(h->L, h->coef32, h->t.B.data(), h->t.A.data(), x, nullptr, y, h->eb32, s);
  }
  return RZ_OK;
}

rz_status do_residual32(rz_problem *h, const float *b, const float *x, float *out) {
  if (h->space == RZ_GRAD && !h->quad) {
    Timed t(h, RZ_K_APPLY);
    launch_apply_grad<float>(h->L, h->coef32, h->t.B.data(), h->t.A.data(), x, b, out, h->eb32, h->ctx->stream);
    return RZ_OK;
  }
  rz_status e = do_apply32(h, x, h->az32);
  if (e) return e;
  launch_sub_f(b, h->az32, out, h->ndofs, h->ctx->stream);
  return RZ_OK;
}

// The V(1,1) cycle on FP32 vectors (inner solve of the defect-correction
// protocol): FP32 apply and relaxation, the coarse correction in FP64.
rz_status do_vcycle32(rz_problem *h, const float *r, float *z) {
  hipStream_t s = h->ctx->stream;
  const int64_t n = h->ndofs;
  const float w = (float)h->omega;
  if (rz_status e = do_relax32(h, r, z, w)) return e;  // z = w M r
  do_residual32(h, r, z, h->vr32);              // r1 = r - A z
  launch_cast_f2d(h->vr32, h->vr, n, s);
  {
    Timed tm(h, RZ_K_TRANSFER);
    launch_restrict_grad(h->L, h->E64, h->vr, h->rc, h->rt1, h->rt2, s);
  }
  rz_status e = do_coarse(h, h->rc, h->xc, true);
  if (e) return e;
  if (h->T2_64) {  // z += P A0^{-1} P^T r1 and r2 = r1 - A P A0^{-1} P^T r1 = r - A z in one pass
    Timed tm(h, RZ_K_TRANSFER);
    launch_prolong_residual_grad_f(h->L, h->E64, h->T2_64, h->coef64, h->xc, z, h->vr32, s);
  } else {
    launch_fill(h->vt, 0.0, n, s);
    {
      Timed tm(h, RZ_K_TRANSFER);
      launch_prolong_add_grad(h->L, h->E64, h->xc, h->vt, s);
    }
    launch_add_d2f(h->vt, z, n, s);              // z += P A0^{-1} P^T r1
    do_residual32(h, r, z, h->vr32);            // r2 = r - A z
  }
  if (rz_status e2 = do_relax32(h, h->vr32, h->t32, 1.0f, w, z)) return e2;  // z += w M r2
  launch_dirichlet_copy_f(h->L, r, z, s);
  return RZ_OK;
}

rz_status dots_host(rz_problem *h, int np, const double *const *xs, const double *const *ys, double *out) {
  {
    Timed tm(h, RZ_K_KRYLOV);
    launch_dots(np, xs, ys, h->ndofs, h->partials, h->dots, h->ctx->stream);
  }
  HIPCALL(h, hipMemcpyAsync(out, h->dots, sizeof(double) * np, hipMemcpyDeviceToHost, h->ctx->stream));
  HIPCALL(h, hipStreamSynchronize(h->ctx->stream));
  return RZ_OK;
}

rz_status dots_host_f(rz_problem *h, int np, const float *const *xs, const float *const *ys, double *out) {
  {
    Timed tm(h, RZ_K_KRYLOV);
    launch_dots_f(np, xs, ys, h->ndofs, h->partials, h->dots, h->ctx->stream);
  }
  HIPCALL(h, hipMemcpyAsync(out, h->dots, sizeof(double) * np, hipMemcpyDeviceToHost, h->ctx->stream));
  HIPCALL(h, hipStreamSynchronize(h->ctx->stream));
  return RZ_OK;
}

// Defect correction (not in the paper; the FP32 operator protocol): the outer loop
// forms the true residual r = b - A x in FP64 and stops at ||r|| <= rtol ||b||; each
// correction solves A e = r with FP32 flexible CG (FP32 apply, FP32 V-cycle,
// Polak-Ribiere) to 1e-4 relative, and x += e in FP64.  iters counts the inner
// iterations.
rz_status defect_solve(rz_problem *h, const double *b, double *x, rz_solve_info *info) {
  hipStream_t s = h->ctx->stream;
  const int64_t n = h->ndofs;
  rz_status e;
  struct EventPair {  // destroyed on every return path
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
      if (a) hipEventDestroy(a);
      if (b) hipEventDestroy(b);
    }
  } ev;
  HIPCALL(h, hipEventCreate(&ev.a));
  HIPCALL(h, hipEventCreate(&ev.b));
  HIPCALL(h, hipEventRecord(ev.a, s));
  launch_fill(x, 0.0, n, s);
  v_scale_copy(h, 1.0, b, h->kr);
  launch_dirichlet_copy(h->L, nullptr, h->kr, s);
  double bb;
  {
    const double *xs[1] = {h->kr};
    if ((e = dots_host(h, 1, xs, xs, &bb))) return e;
  }
  const double nb = std::sqrt(bb), tol = h->opts.rtol * nb;
  int it = 0;
  rz_status result = RZ_ERR_NOT_CONVERGED;
  double rr = bb;
  for (int outer = 0; outer < 64; ++outer) {
    if (outer > 0) {  // true residual of the current iterate
      do_residual64(h, b, x, h->kr);
      launch_dirichlet_copy(h->L, nullptr, h->kr, s);
      const double *xs[1] = {h->kr};
      if ((e = dots_host(h, 1, xs, xs, &rr))) return e;
    }
    if (std::sqrt(rr) <= tol) {
      result = RZ_OK;
      break;
    }
    if (it >= h->opts.maxit) break;
    // inner FP32 flexible CG from e = 0
    launch_cast_d2f(h->kr, h->r32, n, s);
    launch_fill_f(h->ke32, 0.0f, n, s);
    if ((e = do_vcycle32(h, h->r32, h->z32))) return e;
    launch_scale_copy_f(1.0f, h->z32, h->kp32, n, s);
    double rz;
    {
      const float *xs[1] = {h->r32}, *ys[1] = {h->z32};
      if ((e = dots_host_f(h, 1, xs, ys, &rz))) return e;
    }
    const double tol_in = 1e-4 * std::sqrt(rr);
    while (it < h->opts.maxit) {
      if ((e = do_apply32(h, h->kp32, h->kAp32))) return e;
      double pAp;
      {
        const float *xs[1] = {h->kp32}, *ys[1] = {h->kAp32};
        if ((e = dots_host_f(h, 1, xs, ys, &pAp))) return e;
      }
      if (!(pAp > 0)) break;  // the FP64 outer loop decides
      const double a = rz / pAp;
      double rin;
      {
        Timed tm(h, RZ_K_KRYLOV);
        launch_cg_update_f((float)a, h->kp32, h->kAp32, h->ke32, h->r32, h->ko32, n, h->partials, h->dots, s);
      }
      HIPCALL(h, hipMemcpyAsync(&rin, h->dots, sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCALL(h, hipStreamSynchronize(s));
      ++it;
      if (std::sqrt(rin) <= tol_in) break;
      if ((e = do_vcycle32(h, h->r32, h->z32))) return e;
      double d[2];
      {
        const float *xs[2] = {h->r32, h->ko32}, *ys[2] = {h->z32, h->z32};
        if ((e = dots_host_f(h, 2, xs, ys, d))) return e;
      }
      const double beta = (d[0] - d[1]) / rz;
      rz = d[0];
      launch_xpby_f(h->z32, (float)beta, h->kp32, n, s);
    }
    launch_add_f2d(h->ke32, x, n, s);
  }
  HIPCALL(h, hipEventRecord(ev.b, s));
  HIPCALL(h, hipEventSynchronize(ev.b));
  float ms = 0;
  hipEventElapsedTime(&ms, ev.a, ev.b);
  if (result == RZ_OK) result = take_device_status(h);
  if (info) {
    info->iters = it;
    info->status = result;
    info->rel_res = nb > 0 ? std::sqrt(rr) / nb : 0.0;
    info->omega = h->omega;
    info->t_solve_ms = ms;
  }
  return result;
}

// largest eigenvalue of T (k x k symmetric tridiagonal) by bisection on Sturm counts
double tridiag_max_eig(const std::vector<double> &a, const std::vector<double> &b) {
  const int k = (int)a.size();
  double lo = 0, hi = 0;
  for (int i = 0; i < k; ++i) {
    double r = std::fabs(i > 0 ? b[i - 1] : 0.0) + std::fabs(i + 1 < k ? b[i] : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  auto count_below = [&](double x) {
    int c = 0;
    double d = 1.0;
    for (int i = 0; i < k; ++i) {
      d = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (count_below(mid) >= k) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// 10 preconditioned CG steps on A x = v0 with M = fine relaxation; Lanczos estimate
rz_status estimate_lambda(rz_problem *h, double *lam_out) {
  hipStream_t s = h->ctx->stream;
  const int64_t n = h->ndofs;
  std::vector<double> v0(n);
  uint64_t st = h->opts.lanczos_seed;
  for (int64_t g = 0; g < n; ++g) {
    double u = (double)(splitmix_next(st) >> 11) * 0x1.0p-53;
    int X = g % h->Nx, Y = (g / h->Nx) % h->Ny, Z = g / ((int64_t)h->Nx * h->Ny);
    v0[g] = lat_dirichlet_h(h, X, Y, Z) ? 0.0 : 2.0 * u - 1.0;
  }
  HIPCALL(h, hipMemcpyAsync(h->kr, v0.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
  if (rz_status e = do_relax_prec(h, h->kr, h->kz)) return e;
  HIPCALL(h, hipMemcpyAsync(h->kp, h->kz, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  double rz_;
  {
    const double *xs[1] = {h->kr}, *ys[1] = {h->kz};
    rz_status e = dots_host(h, 1, xs, ys, &rz_);
    if (e) return e;
  }
  std::vector<double> al, be;
  for (int it = 0; it < 10; ++it) {
    do_apply64(h, h->kp, h->kAp);
    double pAp;
    const double *xs[1] = {h->kp}, *ys[1] = {h->kAp};
    rz_status e = dots_host(h, 1, xs, ys, &pAp);
    if (e) return e;
    if (!(pAp > 0)) break;
    double a = rz_ / pAp;
    v_axpy(h, -a, h->kAp, h->kr);
    if ((e = do_relax_prec(h, h->kr, h->kz))) return e;
    double rzn;
    const double *xs2[1] = {h->kr}, *ys2[1] = {h->kz};
    e = dots_host(h, 1, xs2, ys2, &rzn);
    if (e) return e;
    double b = rzn / rz_;
    al.push_back(a);
    be.push_back(b);
    rz_ = rzn;
    v_xpby(h, h->kz, b, h->kp);
    if (!(rzn > 0)) break;
  }
  const int k = (int)al.size();
  if (k == 0) return fail(h->ctx, RZ_ERR_BREAKDOWN, "Lanczos estimate failed");
  std::vector<double> d(k), off(k > 1 ? k - 1 : 1, 0.0);
  for (int j = 0; j < k; ++j) {
    d[j] = 1.0 / al[j] + (j > 0 ? be[j - 1] / al[j - 1] : 0.0);
    if (j + 1 < k) off[j] = std::sqrt(be[j]) / al[j];
  }
  *lam_out = tridiag_max_eig(d, off);
  return RZ_OK;
}

// ---------------------------------------------------------------------------------------
// coarse problem: Q_1 rediscretisation with the same per-cell weights; plane-wise
// block-tridiagonal LDL^T with dense inverse diagonal blocks.
// ---------------------------------------------------------------------------------------
rz_status setup_coarse(rz_problem *h) {
  hipStream_t s = h->ctx->stream;
  const int NX = h->nx + 1, NY = h->ny + 1, NZ = h->nz + 1;
  h->cNX = NX;
  h->cNY = NY;
  h->cNZ = NZ;
  h->ncoarse = (int64_t)NX * NY * NZ;
  int lo[3], hi[3];
  const int Nd[3] = {NX, NY, NZ};
  for (int d = 0; d < 3; ++d) {
    lo[d] = (h->dir & (1u << (2 * d))) ? 1 : 0;
    hi[d] = (h->dir & (1u << (2 * d + 1))) ? Nd[d] - 2 : Nd[d] - 1;
    if (hi[d] < lo[d]) return fail(h->ctx, RZ_ERR_ARG, "coarse problem has no free DoF along an axis");
  }
  h->cbx0 = lo[0];
  h->cby0 = lo[1];
  h->cbz0 = lo[2];
  h->cmx = hi[0] - lo[0] + 1;
  h->cmy = hi[1] - lo[1] + 1;
  h->cmz = hi[2] - lo[2] + 1;
  const int m = h->cmx * h->cmy, nb = h->cmz;
  h->cm = m;
  if (m > 4096) return fail(h->ctx, RZ_ERR_ARG, "coarse plane too large for the dense-block coarse solver");
  // 27-point stencil of every free coarse DoF from the p=1 cell matrices
  const Tables1D &t1 = h->t1;
  auto B1 = [&](int a, int b) { return t1.B[a * 2 + b]; };
  auto A1 = [&](int a, int b) { return t1.A[a * 2 + b]; };
  const int64_t nfree = (int64_t)m * nb;
  std::vector<double> st(nfree * 27, 0.0);
  for (int64_t c = 0; c < h->ncells; ++c) {
    int cx = c % h->nx, cy = (c / h->nx) % h->ny, cz = c / ((int64_t)h->nx * h->ny);
    const double *w = &h->coef[6 * c];
    for (int i = 0; i < 8; ++i) {
      int ia[3] = {i & 1, (i >> 1) & 1, i >> 2};
      int Vi[3] = {cx + ia[0], cy + ia[1], cz + ia[2]};
      bool fi = true;
      for (int d = 0; d < 3; ++d) fi = fi && Vi[d] >= lo[d] && Vi[d] <= hi[d];
      if (!fi) continue;
      int64_t row = (Vi[0] - lo[0]) + h->cmx * ((Vi[1] - lo[1]) + (int64_t)h->cmy * (Vi[2] - lo[2]));
      for (int j = 0; j < 8; ++j) {
        int ja[3] = {j & 1, (j >> 1) & 1, j >> 2};
        double v = h->quad ? h->cellA1[64 * c + 8 * i + j]
                           : w[0] * A1(ia[0], ja[0]) * B1(ia[1], ja[1]) * B1(ia[2], ja[2]) +
                                 w[1] * B1(ia[0], ja[0]) * A1(ia[1], ja[1]) * B1(ia[2], ja[2]) +
                                 w[2] * B1(ia[0], ja[0]) * B1(ia[1], ja[1]) * A1(ia[2], ja[2]) +
                                 w[3] * B1(ia[0], ja[0]) * B1(ia[1], ja[1]) * B1(ia[2], ja[2]);
        int off = (ja[0] - ia[0] + 1) + 3 * (ja[1] - ia[1] + 1) + 9 * (ja[2] - ia[2] + 1);
        st[row * 27 + off] += v;
      }
    }
  }
  // device blocks
  rz_status e;
  if ((e = dalloc(h, &h->cW, (size_t)nb * m * m))) return e;
  std::vector<double> C((size_t)nb * m * 9, 0.0), Ct((size_t)nb * m * 9, 0.0);
  for (int k = 0; k < nb; ++k)
    for (int a = 0; a < m; ++a)
      for (int j = 0; j < 9; ++j) {
        C[((size_t)k * m + a) * 9 + j] = k > 0 ? st[((int64_t)k * m + a) * 27 + j] : 0.0;
        Ct[((size_t)k * m + a) * 9 + j] = k < nb - 1 ? st[((int64_t)k * m + a) * 27 + 18 + j] : 0.0;
      }
  if ((e = upload(h, &h->cC, C))) return e;
  if ((e = upload(h, &h->cCt, Ct))) return e;
  double *Akk = nullptr, *tmp = nullptr;
  if ((e = dalloc(h, &Akk, (size_t)m * m))) return e;
  if ((e = dalloc(h, &tmp, (size_t)m * m))) return e;
  // Twisted block factorisation: top-down (W_k, k < q), bottom-up (Z_k, k > q), and
  // the middle plane q with both Schur terms; plane k's inverse block goes to cW[k].
  // Planes larger than 1024 use q = nb - 1 (the top-down factorisation alone).
  const int q = m <= 1024 ? (nb - 1) / 2 : nb - 1;
  h->cq = q;
  std::vector<double> Ah((size_t)m * m);
  auto plane_matrix = [&](int k) -> rz_status {
    std::fill(Ah.begin(), Ah.end(), 0.0);
    for (int a = 0; a < m; ++a) {
      int ax = a % h->cmx, ay = a / h->cmx;
      for (int j = 0; j < 9; ++j) {
        int bx = ax + j % 3 - 1, by = ay + j / 3 - 1;
        if (bx < 0 || bx >= h->cmx || by < 0 || by >= h->cmy) continue;
        Ah[(size_t)a * m + bx + h->cmx * by] = st[((int64_t)k * m + a) * 27 + 9 + j];
      }
    }
    HIPCALL(h, hipMemcpyAsync(Akk, Ah.data(), sizeof(double) * m * m, hipMemcpyHostToDevice, s));
    return RZ_OK;
  };
  auto block = [&](int k) { return h->cW + (size_t)k * m * m; };
  for (int k = 0; k <= q; ++k) {  // top-down; at k = q only the upper Schur term so far
    if ((e = plane_matrix(k))) return e;
    if (k == 0) HIPCALL(h, hipMemcpyAsync(block(k), Akk, sizeof(double) * m * m, hipMemcpyDeviceToDevice, s));
    else launch_schur_update(m, h->cmx, block(k - 1), h->cC + (size_t)k * m * 9, Akk, block(k), s);
    if (k < q) launch_sweep_inverse(m, block(k), tmp, h->status, s);
    HIPCALL(h, hipStreamSynchronize(s));  // Ah is reused for the next plane
  }
  for (int k = nb - 1; k > q; --k) {  // bottom-up
    if ((e = plane_matrix(k))) return e;
    if (k == nb - 1) HIPCALL(h, hipMemcpyAsync(block(k), Akk, sizeof(double) * m * m, hipMemcpyDeviceToDevice, s));
    else launch_schur_update(m, h->cmx, block(k + 1), h->cCt + (size_t)k * m * 9, Akk, block(k), s);
    launch_sweep_inverse(m, block(k), tmp, h->status, s);
    HIPCALL(h, hipStreamSynchronize(s));
  }
  if (q + 1 < nb) {  // the middle plane's lower Schur term
    HIPCALL(h, hipMemcpyAsync(Akk, block(q), sizeof(double) * m * m, hipMemcpyDeviceToDevice, s));
    launch_schur_update(m, h->cmx, block(q + 1), h->cCt + (size_t)q * m * 9, Akk, block(q), s);
  }
  launch_sweep_inverse(m, block(q), tmp, h->status, s);
  HIPCALL(h, hipStreamSynchronize(s));
  int stv = 0;
  HIPCALL(h, hipMemcpy(&stv, h->status, sizeof(int), hipMemcpyDeviceToHost));
  if (stv) return fail(h->ctx, RZ_ERR_SINGULAR, "coarse factorisation: non-positive pivot");
  // coupling products for the solve (C_k: coupling of plane k to plane k-1, Ct_k: to
  // plane k+1): k < q: M_k = W_k C_k, N_k = W_k Ct_k; k > q: M_k = Z_k Ct_k, N_k =
  // Z_k C_k; k = q: M_q = G C_q, N_q = G Ct_q
  if ((e = dalloc(h, &h->cM, (size_t)nb * m * m)) || (e = dalloc(h, &h->cN, (size_t)nb * m * m))) return e;
  for (int k = 0; k < nb; ++k) {
    const double *Ck = h->cC + (size_t)k * m * 9, *Ctk = h->cCt + (size_t)k * m * 9;
    const bool down = k > q;
    const double *cm = down ? Ctk : Ck, *cn = down ? Ck : Ctk;
    const bool hm = down ? k + 1 < nb : k > 0, hn = down ? true : k + 1 < nb;
    if (hm) launch_coarse_wc(m, h->cmx, h->cmy, block(k), cm, h->cM + (size_t)k * m * m, s);
    if (hn) launch_coarse_wc(m, h->cmx, h->cmy, block(k), cn, h->cN + (size_t)k * m * m, s);
  }
  if ((e = dalloc(h, &h->cu, nfree))) return e;
  if ((e = dalloc(h, &h->cr, nfree))) return e;
  if ((e = dalloc(h, &h->cv, nfree))) return e;
  if ((e = dalloc(h, &h->cx, nfree))) return e;
  if (h->opts.precision != RZ_PREC_F64) {
    // the V-cycle of the mixed protocols streams the blocks in FP32 (half the bytes of
    // the coarse solve; its vectors and sums stay FP64)
    const size_t nbm = (size_t)nb * m * m;
    if ((e = dalloc(h, &h->cW32, nbm)) || (e = dalloc(h, &h->cM32, nbm)) || (e = dalloc(h, &h->cN32, nbm))) return e;
    launch_cast_d2f(h->cW, h->cW32, (int64_t)nbm, s);
    launch_cast_d2f(h->cM, h->cM32, (int64_t)nbm, s);
    launch_cast_d2f(h->cN, h->cN32, (int64_t)nbm, s);
  }
  HIPCALL(h, hipStreamSynchronize(s));
  return RZ_OK;
}

void release(rz_problem *h) {
  for (void *p : h->allocs) hipFree(p);
  h->allocs.clear();
  if (h->hdots) hipHostFree(h->hdots);
  h->hdots = nullptr;
  for (auto &e : h->ev_pool) {
    hipEventDestroy(e.first);
    hipEventDestroy(e.second);
  }
  h->ev_pool.clear();
  h->ev_used.clear();
}

// The coarse solve's bounded waits record -1 in the problem's status word when a
// wait gives up (its result is then garbage).  Synchronises the stream, reads and
// clears the word.
rz_status take_device_status(rz_problem *h) {
  if (!h->status) return RZ_OK;
  int stv = 0;
  HIPCALL(h, hipMemcpyAsync(&stv, h->status, sizeof(int), hipMemcpyDeviceToHost, h->ctx->stream));
  HIPCALL(h, hipStreamSynchronize(h->ctx->stream));
  if (stv == 0) return RZ_OK;
  const int zero = 0;
  HIPCALL(h, hipMemcpyAsync(h->status, &zero, sizeof(int), hipMemcpyHostToDevice, h->ctx->stream));
  HIPCALL(h, hipStreamSynchronize(h->ctx->stream));
  return fail(h->ctx, RZ_ERR_HIP, "a bounded wait of the coarse solve gave up (device status word set)");
}

rz_status require_device(const rz_problem *h) {
  if (!h) return RZ_ERR_ARG;
  if (h->ctx->device < 0) return fail(h->ctx, RZ_ERR_NODEVICE, "host-only context");
  return RZ_OK;
}

}  // namespace

// =========================================================================================
// public API
// =========================================================================================
namespace {

// H(curl) / H(div) problems: the cellwise-constant Cartesian cell matrices of the
// closed form (Sec. 3.2 with the pullbacks of Sec. 3.1 on boxes), apply only.
//   curl: stiffness weight of curl component n: alpha 2 h_n^2 / V, mass weight of
//         component m: beta V / (2 h_m^2);
//   div:  stiffness weight alpha 8 / V, mass weight of component m: beta 2 h_m^2 / V.
rz_status setup_vector(rz_problem *h, const rz_coef *cf, rz_problem **out) {
  rz_ctx *ctx = h->ctx;
  const int p = h->p;
  h->space = h->opts.space;
  if (h->quad) {
    delete h;
    return fail(ctx, RZ_ERR_ARG, "H(curl)/H(div) need axis-aligned cells and cellwise-constant coefficients");
  }
  const int nvx = h->nx + 1, nvy = h->ny + 1;
  for (int64_t c = 0; c < h->ncells; ++c) {
    int cx = c % h->nx, cy = (c / h->nx) % h->ny, cz = c / ((int64_t)h->nx * h->ny);
    const double hs[3] = {h->vert[3 * (cx + 1)] - h->vert[3 * cx],
                          h->vert[3 * ((cy + 1) * nvx) + 1] - h->vert[3 * (cy * nvx) + 1],
                          h->vert[3 * ((int64_t)(cz + 1) * nvx * nvy) + 2] - h->vert[3 * ((int64_t)cz * nvx * nvy) + 2]};
    const double al = cf->kind == RZ_COEF_CONST ? cf->alpha[0] : cf->alpha[c];
    const double be = cf->kind == RZ_COEF_CONST ? cf->beta[0] : cf->beta[c];
    const double V = hs[0] * hs[1] * hs[2];
    for (int d = 0; d < 3; ++d) {
      if (h->space == RZ_CURL) {
        h->coef[6 * c + d] = al * 2.0 * hs[d] * hs[d] / V;
        h->coef[6 * c + 3 + d] = be * V / (2.0 * hs[d] * hs[d]);
      } else {
        h->coef[6 * c + d] = al * 8.0 / V;
        h->coef[6 * c + 3 + d] = be * 2.0 * hs[d] * hs[d] / V;
      }
    }
  }
  VecDev &Vd = h->V;
  Vd.p = p;
  Vd.nx = h->nx;
  Vd.ny = h->ny;
  Vd.nz = h->nz;
  Vd.dir = h->dir;
  Vd.space = h->space;
  const int nd[3] = {h->nx, h->ny, h->nz};
  long off = 0;
  Vd.cell_dofs = 0;
  int64_t ndir = 0;
  for (int m = 0; m < 3; ++m) {
    int tile = 1;
    bool P[3];
    for (int a = 0; a < 3; ++a) {
      P[a] = h->space == RZ_CURL ? a != m : a == m;
      Vd.ext[m][a] = nd[a] * p + (P[a] ? 1 : 0);
      tile *= P[a] ? p + 1 : p;
    }
    Vd.off[m] = off;
    off += (long)Vd.ext[m][0] * Vd.ext[m][1] * Vd.ext[m][2];
    Vd.cell_dofs += tile;
    for (int64_t g = 0; g < (int64_t)Vd.ext[m][0] * Vd.ext[m][1] * Vd.ext[m][2]; ++g) {
      const int C[3] = {(int)(g % Vd.ext[m][0]), (int)((g / Vd.ext[m][0]) % Vd.ext[m][1]),
                        (int)(g / ((int64_t)Vd.ext[m][0] * Vd.ext[m][1]))};
      bool d = false;
      for (int a = 0; a < 3; ++a)
        if (P[a] && (((h->dir >> (2 * a)) & 1u) && C[a] == 0 || ((h->dir >> (2 * a + 1)) & 1u) && C[a] == Vd.ext[m][a] - 1))
          d = true;
      ndir += d;
    }
  }
  Vd.off[3] = off;
  h->ndofs = off;
  h->nfree = off - ndir;
  if (ctx->device < 0) {
    *out = h;
    return RZ_OK;
  }
  hipStream_t s = ctx->stream;
  rz_status e;
  auto bail = [&](rz_status st) {
    hipStreamSynchronize(s);
    release(h);
    delete h;
    return st;
  };
  std::vector<float> c32(h->coef.begin(), h->coef.end()), B32(h->t.B.begin(), h->t.B.end()),
      D32(h->t.D.begin(), h->t.D.end());
  const size_t neb = (size_t)h->ncells * Vd.cell_dofs;
  if ((e = upload(h, &h->coef64, h->coef)) || (e = upload(h, &h->coef32, c32)) || (e = upload(h, &h->B64, h->t.B)) ||
      (e = upload(h, &h->B32, B32)) || (e = upload(h, &h->D64, h->t.D)) || (e = upload(h, &h->D32, D32)) ||
      (e = dalloc(h, &h->eb64, neb)) || (e = dalloc(h, &h->eb32, neb)))
    return bail(e);
  if (hipStreamSynchronize(s) != hipSuccess) return bail(fail(ctx, RZ_ERR_HIP, "setup failed"));
  *out = h;
  return RZ_OK;
}

rz_status require_grad(const rz_problem *h) {
  if (h->space != RZ_GRAD)
    return fail(h->ctx, RZ_ERR_ARG, "this call is available for H(grad) only (H(curl)/H(div): apply)");
  return RZ_OK;
}

}  // namespace

namespace {

// PCG (Sec. 5) as a state machine: each step enqueues stream-ordered work and the
// dot products it needs (copied asynchronously to pinned host memory); the caller
// waits for the stream and hands the values to the next step.  rz_solve runs one
// instance; rz_solve_batched advances instances of several problems in lockstep,
// so their streams overlap on the device.  Both issue the same kernels in the same
// order, so their results are identical.
// PCG as a step machine: each step enqueues work and the read-back of the scalars
// the host needs next; the caller synchronises the stream between steps.  The CG
// coefficients are formed on the device (alpha in the update kernel, beta in the
// direction update), so one host round trip per iteration remains: the convergence
// test on r.r, which decides whether the next V-cycle runs.
// Device scalar slots (h->dots): [2q], [2q+1]: r.z and (mixed) r_old.z of the
// iterations with parity q; [4]: p.Ap; [5]: r.r after the update; [6]: other norms.
struct PcgRun {
  rz_problem *h = nullptr;
  const double *b = nullptr;
  double *x = nullptr;
  enum Phase { INIT, GOT_BB, GOT_RR, GOT_TR, GOT_FINAL, DONE } phase = INIT;
  int it = 0;
  double nb = 0, tol = 0, relres = 0;
  rz_status result = RZ_OK;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

enum { kSlotPap = 4, kSlotRr = 5, kSlotNorm = 6 };

// one norm (x.x) into slot kSlotNorm and its host copy hdots[0]
rz_status pcg_norm(PcgRun &R, const double *v) {
  rz_problem *h = R.h;
  const double *xs[1] = {v};
  {
    Timed tm(h, RZ_K_KRYLOV);
    launch_dots(1, xs, xs, h->ndofs, h->partials, h->dots + kSlotNorm, h->ctx->stream);
  }
  HIPCALL(h, hipMemcpyAsync(h->hdots, h->dots + kSlotNorm, sizeof(double), hipMemcpyDeviceToHost, h->ctx->stream));
  return RZ_OK;
}

rz_status pcg_final(PcgRun &R) {
  rz_problem *h = R.h;
  do_residual64(h, R.b, R.x, h->vr);
  launch_dirichlet_copy(h->L, nullptr, h->vr, h->ctx->stream);
  R.phase = PcgRun::GOT_FINAL;
  return pcg_norm(R, h->vr);
}

// One iteration from the current residual r: z = V r, rz (+ cross), p = z + beta p
// (p = z on the first iteration), Ap, p.Ap, x += alpha p, r -= alpha Ap, r.r; then
// p.Ap and r.r go back to the host.
rz_status pcg_iteration(PcgRun &R, bool first) {
  rz_problem *h = R.h;
  hipStream_t s = h->ctx->stream;
  const int64_t n = h->ndofs;
  const bool mixed = h->opts.precision == RZ_PREC_MIXED;
  const int q = R.it & 1;
  double *rz = h->dots + 2 * q, *rz_old = h->dots + 2 * (1 - q);
  if (rz_status e = do_vcycle(h, h->kr, h->kz)) return e;
  {
    Timed tm(h, RZ_K_KRYLOV);
    if (first) {
      const double *xs[1] = {h->kr}, *ys[1] = {h->kz};
      launch_dots(1, xs, ys, n, h->partials, rz, s);
      launch_scale_copy(1.0, h->kz, h->kp, n, s);
    } else if (mixed) {
      const double *xs[2] = {h->kr, h->kro}, *ys[2] = {h->kz, h->kz};
      launch_dots(2, xs, ys, n, h->partials, rz, s);
      launch_xpby_dev(h->kz, rz, rz + 1, rz_old, h->kp, n, s);
    } else {
      const double *xs[1] = {h->kr}, *ys[1] = {h->kz};
      launch_dots(1, xs, ys, n, h->partials, rz, s);
      launch_xpby_dev(h->kz, rz, nullptr, rz_old, h->kp, n, s);
    }
  }
  do_apply64(h, h->kp, h->kAp);
  {
    Timed tm(h, RZ_K_KRYLOV);
    const double *xs[1] = {h->kp}, *ys[1] = {h->kAp};
    launch_dots(1, xs, ys, n, h->partials, h->dots + kSlotPap, s);
    launch_cg_update(rz, h->dots + kSlotPap, h->kp, h->kAp, R.x, h->kr, mixed ? h->kro : nullptr, n, h->partials,
                     h->dots + kSlotRr, s);
  }
  HIPCALL(h, hipMemcpyAsync(h->hdots, h->dots + kSlotPap, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  ++R.it;
  R.phase = PcgRun::GOT_RR;
  return RZ_OK;
}

// Advance one step with the scalars of the previous step in h->hdots.
rz_status pcg_step(PcgRun &R) {
  rz_problem *h = R.h;
  hipStream_t s = h->ctx->stream;
  const int64_t n = h->ndofs;
  const double *d = h->hdots;
  switch (R.phase) {
    case PcgRun::INIT: {
      HIPCALL(h, hipEventCreate(&R.ev0));
      HIPCALL(h, hipEventCreate(&R.ev1));
      HIPCALL(h, hipEventRecord(R.ev0, s));
      launch_fill(R.x, 0.0, n, s);  // x = 0, r = b with Dirichlet rows zero
      v_scale_copy(h, 1.0, R.b, h->kr);
      launch_dirichlet_copy(h->L, nullptr, h->kr, s);
      R.phase = PcgRun::GOT_BB;
      return pcg_norm(R, h->kr);
    }
    case PcgRun::GOT_BB: {
      R.nb = std::sqrt(d[0]);
      R.tol = h->opts.rtol * R.nb;
      if (!(R.nb > 0)) return pcg_final(R);
      if (h->opts.maxit < 1) {
        R.result = RZ_ERR_NOT_CONVERGED;
        return pcg_final(R);
      }
      return pcg_iteration(R, true);
    }
    case PcgRun::GOT_RR: {
      const double pAp = d[0], rr = d[1];
      if (!(pAp > 0)) {
        R.result = fail(h->ctx, RZ_ERR_BREAKDOWN, "CG breakdown: p.Ap <= 0");
        return pcg_final(R);
      }
      if (std::sqrt(rr) <= R.tol) {  // recurrence converged: check the true residual
        do_residual64(h, R.b, R.x, h->vr);
        launch_dirichlet_copy(h->L, nullptr, h->vr, s);
        R.phase = PcgRun::GOT_TR;
        return pcg_norm(R, h->vr);
      }
      if (R.it >= h->opts.maxit) {
        R.result = RZ_ERR_NOT_CONVERGED;
        return pcg_final(R);
      }
      return pcg_iteration(R, false);
    }
    case PcgRun::GOT_TR: {
      if (std::sqrt(d[0]) <= R.tol) {
        R.result = RZ_OK;
        R.relres = R.nb > 0 ? std::sqrt(d[0]) / R.nb : 0.0;
        R.phase = PcgRun::DONE;
        return RZ_OK;
      }
      if (R.it >= h->opts.maxit) {
        R.result = RZ_ERR_NOT_CONVERGED;
        R.relres = R.nb > 0 ? std::sqrt(d[0]) / R.nb : 0.0;
        R.phase = PcgRun::DONE;
        return RZ_OK;
      }
      v_scale_copy(h, 1.0, h->vr, h->kr);  // continue from the true residual
      return pcg_iteration(R, false);
    }
    case PcgRun::GOT_FINAL:
      R.relres = R.nb > 0 ? std::sqrt(d[0]) / R.nb : 0.0;
      R.phase = PcgRun::DONE;
      return RZ_OK;
    case PcgRun::DONE:
      return RZ_OK;
  }
  return RZ_OK;
}

void pcg_release(PcgRun &R) {
  if (R.ev0) hipEventDestroy(R.ev0);
  if (R.ev1) hipEventDestroy(R.ev1);
  R.ev0 = R.ev1 = nullptr;
}

rz_status pcg_finish(PcgRun &R, rz_solve_info *info) {
  rz_problem *h = R.h;
  float ms = 0;
  if (R.ev0) {
    const bool ok = hipEventRecord(R.ev1, h->ctx->stream) == hipSuccess && hipEventSynchronize(R.ev1) == hipSuccess;
    if (ok) hipEventElapsedTime(&ms, R.ev0, R.ev1);
    pcg_release(R);
    if (!ok) return fail(h->ctx, RZ_ERR_HIP, "stream execution failed during the solve");
  }
  if (R.result == RZ_OK) R.result = take_device_status(h);
  if (info) {
    info->iters = R.it;
    info->status = R.result;
    info->rel_res = R.relres;
    info->omega = h->omega;
    info->t_solve_ms = ms;
  }
  return R.result;
}

}  // namespace

extern "C" {

void rz_opts_default(rz_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->space = RZ_GRAD;
  o->p = 4;
  o->precision = RZ_PREC_F64;
  o->maxit = 200;
  o->rtol = 1e-8;
  o->omega = 0.0;
  o->lanczos_seed = 99;
}

rz_status rz_create(rz_ctx **ctx, int device, void *stream) {
  if (!ctx) return RZ_ERR_ARG;
  rz_ctx *c = new rz_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  if (device >= 0) {
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = scratch_init(device);
    if (e != hipSuccess) {
      delete c;
      return RZ_ERR_HIP;
    }
  }
  *ctx = c;
  return RZ_OK;
}

rz_status rz_destroy(rz_ctx *ctx) {
  if (!ctx) return RZ_OK;
  if (ctx->nlive > 0) {
    ctx->err = "rz_destroy: " + std::to_string(ctx->nlive) + " problem(s) or MLP(s) on this context are not freed";
    return RZ_ERR_ARG;
  }
  if (ctx->device >= 0) hipStreamSynchronize(ctx->stream);
  delete ctx;
  return RZ_OK;
}

const char *rz_last_error(const rz_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

static rz_status setup_impl(rz_ctx *ctx, const rz_mesh *mesh, const rz_coef *cf, const rz_opts *opts,
                            rz_problem **out) {
  if (!ctx || !mesh || !cf || !opts || !out) return RZ_ERR_ARG;
  *out = nullptr;
  if (opts->space != RZ_GRAD && opts->space != RZ_CURL && opts->space != RZ_DIV)
    return fail(ctx, RZ_ERR_ARG, "bad space");
  if (opts->p < 1 || opts->p > 9) return fail(ctx, RZ_ERR_ARG, "p must be in 1..9");
  if (mesh->nx < 1 || mesh->ny < 1 || mesh->nz < 1) return fail(ctx, RZ_ERR_ARG, "bad mesh size");
  if (mesh->dirichlet_faces > 0x3F) return fail(ctx, RZ_ERR_ARG, "bad Dirichlet mask");
  if (cf->kind != RZ_COEF_CONST && cf->kind != RZ_COEF_CELL && cf->kind != RZ_COEF_SAMPLES)
    return fail(ctx, RZ_ERR_ARG, "bad coefficient kind");
  if (!cf->alpha || !cf->beta) return fail(ctx, RZ_ERR_ARG, "missing coefficients");
  if (opts->precision != RZ_PREC_F64 && opts->precision != RZ_PREC_MIXED && opts->precision != RZ_PREC_DEFECT)
    return fail(ctx, RZ_ERR_ARG, "bad precision");
  rz_problem *h = new rz_problem();
  h->ctx = ctx;
  h->opts = *opts;
  if (h->opts.maxit <= 0) h->opts.maxit = 200;
  if (!(h->opts.rtol > 0)) h->opts.rtol = 1e-8;
  const int p = opts->p;
  h->p = p;
  h->nx = mesh->nx;
  h->ny = mesh->ny;
  h->nz = mesh->nz;
  h->dir = mesh->dirichlet_faces;
  h->Nx = h->nx * p + 1;
  h->Ny = h->ny * p + 1;
  h->Nz = h->nz * p + 1;
  h->ndofs = (int64_t)h->Nx * h->Ny * h->Nz;
  h->ncells = (int64_t)h->nx * h->ny * h->nz;
  h->nvert = (int64_t)(h->nx + 1) * (h->ny + 1) * (h->nz + 1);
  if (!build_tables1d(p, h->t) || !build_tables1d(1, h->t1)) {
    delete h;
    return fail(ctx, RZ_ERR_ARG, "1-D tables failed");
  }
  // geometry: vertices (uniform unit cube by default); a tensor grid of
  // axis-aligned boxes with cellwise-constant coefficients takes the Kronecker path
  const int nvx = h->nx + 1, nvy = h->ny + 1, nvz = h->nz + 1;
  h->vert.resize(3 * h->nvert);
  for (int64_t k = 0; k < h->nvert; ++k) {
    const int vx = k % nvx, vy = (k / nvx) % nvy, vz = k / ((int64_t)nvx * nvy);
    if (mesh->vertex_xyz) {
      for (int r = 0; r < 3; ++r) h->vert[3 * k + r] = mesh->vertex_xyz[3 * k + r];
    } else {
      h->vert[3 * k] = (double)vx / h->nx;
      h->vert[3 * k + 1] = (double)vy / h->ny;
      h->vert[3 * k + 2] = (double)vz / h->nz;
    }
  }
  bool cartesian = true;
  for (int64_t k = 0; k < h->nvert && cartesian; ++k) {
    const int vx = k % nvx, vy = (k / nvx) % nvy, vz = k / ((int64_t)nvx * nvy);
    cartesian = h->vert[3 * k] == h->vert[3 * vx] && h->vert[3 * k + 1] == h->vert[3 * (vy * nvx) + 1] &&
                h->vert[3 * k + 2] == h->vert[3 * (vz * nvx * nvy) + 2];
  }
  h->quad = !cartesian || cf->kind == RZ_COEF_SAMPLES;
  h->coef.assign(6 * h->ncells, 0.0);
  if (!h->quad) {
    for (int64_t c = 0; c < h->ncells; ++c) {
      int cx = c % h->nx, cy = (c / h->nx) % h->ny, cz = c / ((int64_t)h->nx * h->ny);
      // axis-aligned boxes: extents from the first row of vertices along each axis
      const double hs[3] = {h->vert[3 * (cx + 1)] - h->vert[3 * cx],
                            h->vert[3 * ((cy + 1) * nvx) + 1] - h->vert[3 * (cy * nvx) + 1],
                            h->vert[3 * ((int64_t)(cz + 1) * nvx * nvy) + 2] -
                                h->vert[3 * ((int64_t)cz * nvx * nvy) + 2]};
      if (!(hs[0] > 0 && hs[1] > 0 && hs[2] > 0)) {
        delete h;
        return fail(ctx, RZ_ERR_ARG, "cells must have positive extent");
      }
      double al = cf->kind == RZ_COEF_CONST ? cf->alpha[0] : cf->alpha[c];
      double be = cf->kind == RZ_COEF_CONST ? cf->beta[0] : cf->beta[c];
      if (!(al > 0 && be > 0)) {
        delete h;
        return fail(ctx, RZ_ERR_ARG, "alpha and beta must be positive");
      }
      double V = hs[0] * hs[1] * hs[2];
      for (int d = 0; d < 3; ++d) h->coef[6 * c + d] = al * V / (2.0 * hs[d] * hs[d]);
      for (int d = 0; d < 3; ++d) h->coef[6 * c + 3 + d] = be * V / 8.0;
    }
  } else {
    h->asmp.resize(27 * h->ncells);
    h->bsmp.resize(27 * h->ncells);
    for (int64_t c = 0; c < h->ncells; ++c)
      for (int k = 0; k < 27; ++k) {
        h->asmp[27 * c + k] = cf->kind == RZ_COEF_CONST ? cf->alpha[0]
                              : cf->kind == RZ_COEF_CELL ? cf->alpha[c] : cf->alpha[27 * c + k];
        h->bsmp[27 * c + k] = cf->kind == RZ_COEF_CONST ? cf->beta[0]
                              : cf->kind == RZ_COEF_CELL ? cf->beta[c] : cf->beta[27 * c + k];
        if (!(h->asmp[27 * c + k] > 0 && h->bsmp[27 * c + k] > 0)) {
          delete h;
          return fail(ctx, RZ_ERR_ARG, "coefficient samples must be positive");
        }
      }
    build_quad_tables(h->t, default_quad_points(p), h->qt);
    QuadTables q1;
    build_quad_tables(h->t1, default_quad_points(1), q1);
    h->cellA1.resize(64 * h->ncells);
    for (int64_t c = 0; c < h->ncells; ++c) {
      int cx = c % h->nx, cy = (c / h->nx) % h->ny, cz = c / ((int64_t)h->nx * h->ny);
      double corners[24];
      for (int k = 0; k < 8; ++k) {
        const int64_t vid = (cx + (k & 1)) + nvx * ((cy + ((k >> 1) & 1)) + (int64_t)nvy * (cz + (k >> 2)));
        for (int r = 0; r < 3; ++r) corners[3 * k + r] = h->vert[3 * vid + r];
      }
      if (!averaged_weights(corners, &h->asmp[27 * c], &h->bsmp[27 * c], h->qt, &h->coef[6 * c]) ||
          !q1_cell_matrix(corners, &h->asmp[27 * c], &h->bsmp[27 * c], q1, &h->cellA1[64 * c])) {
        delete h;
        return fail(ctx, RZ_ERR_ARG, "non-positive Jacobian determinant or coefficient at a quadrature point");
      }
    }
  }
  if (opts->space != RZ_GRAD) return setup_vector(h, cf, out);
  build_patch_symbolic(p, h->ps);
  h->erow.resize(h->ps.nnz);
  for (int r = 0; r < h->ps.nrows; ++r)
    for (int k = h->ps.rowptr[r]; k < h->ps.rowptr[r + 1]; ++k) h->erow[k] = r;
  // free DoFs and non-empty patches
  int64_t nd = 0;
  for (int64_t g = 0; g < h->ndofs; ++g) {
    int X = g % h->Nx, Y = (g / h->Nx) % h->Ny, Z = g / ((int64_t)h->Nx * h->Ny);
    nd += lat_dirichlet_h(h, X, Y, Z);
  }
  h->nfree = h->ndofs - nd;
  for (int64_t v = 0; v < h->nvert; ++v) {
    int G[3];
    for (int k = 0; k < h->ps.nrows; ++k)
      if (patch_row_present(h, v, k, G)) {
        h->patch_vids.push_back(v);
        break;
      }
  }
  h->L = LatDev{p, h->nx, h->ny, h->nz, h->Nx, h->Ny, h->Nz, h->dir};
  if (ctx->device < 0) {
    *out = h;
    return RZ_OK;
  }
  // ---- device data ----------------------------------------------------------------------
  hipStream_t s = ctx->stream;
  rz_status e;
  auto bail = [&](rz_status st) {
    hipStreamSynchronize(s);
    release(h);
    delete h;
    return st;
  };
  const int n1 = p + 1;
  std::vector<double> lamf(n1, 0.0);
  for (int i = 1; i < p; ++i) lamf[i] = h->t.lam[i - 1];
  std::vector<float> c32(h->coef.begin(), h->coef.end()), B32(h->t.B.begin(), h->t.B.end()),
      A32(h->t.A.begin(), h->t.A.end()), l32(lamf.begin(), lamf.end());
  if ((e = dalloc(h, &h->status, 1))) return bail(e);
  if (hipMemsetAsync(h->status, 0, sizeof(int), s) != hipSuccess) return bail(fail(ctx, RZ_ERR_HIP, "memset"));
  if ((e = upload(h, &h->coef64, h->coef)) || (e = upload(h, &h->B64, h->t.B)) || (e = upload(h, &h->A64, h->t.A)) ||
      (e = upload(h, &h->lam64, lamf)) || (e = upload(h, &h->E64, h->t.E)) || (e = upload(h, &h->coef32, c32)) ||
      (e = upload(h, &h->B32, B32)) || (e = upload(h, &h->A32, A32)) || (e = upload(h, &h->lam32, l32)))
    return bail(e);
  if (!h->quad) {  // A E and B E for the fused coarse correction and residual
    std::vector<double> T2(4 * (size_t)n1, 0.0);
    for (int a = 0; a < n1; ++a)
      for (int i = 0; i < 2; ++i)
        for (int m = 0; m < n1; ++m) {
          T2[2 * a + i] += h->t.A[a * n1 + m] * h->t.E[2 * m + i];
          T2[2 * n1 + 2 * a + i] += h->t.B[a * n1 + m] * h->t.E[2 * m + i];
        }
    if ((e = upload(h, &h->T2_64, T2))) return bail(e);
  }
  if (h->quad) {
    auto to32 = [](const std::vector<double> &v) { return std::vector<float>(v.begin(), v.end()); };
    const QuadTables &qt = h->qt;
    double *dv = nullptr, *a64 = nullptr, *b64 = nullptr, *qB = nullptr, *qD = nullptr, *qw = nullptr, *qx = nullptr,
           *qL = nullptr;
    float *a32 = nullptr, *b32 = nullptr, *fB = nullptr, *fD = nullptr, *fw = nullptr, *fx = nullptr, *fL = nullptr;
    if ((e = upload(h, &dv, h->vert)) || (e = upload(h, &a64, h->asmp)) || (e = upload(h, &b64, h->bsmp)) ||
        (e = upload(h, &qB, qt.Bq)) || (e = upload(h, &qD, qt.Dq)) || (e = upload(h, &qw, qt.wq)) ||
        (e = upload(h, &qx, qt.xq)) || (e = upload(h, &qL, qt.Lq)) || (e = upload(h, &a32, to32(h->asmp))) ||
        (e = upload(h, &b32, to32(h->bsmp))) || (e = upload(h, &fB, to32(qt.Bq))) || (e = upload(h, &fD, to32(qt.Dq))) ||
        (e = upload(h, &fw, to32(qt.wq))) || (e = upload(h, &fx, to32(qt.xq))) || (e = upload(h, &fL, to32(qt.Lq))))
      return bail(e);
    h->Q64 = QuadDev<double>{dv, a64, b64, qB, qD, qw, qx, qL};
    h->Q32 = QuadDev<float>{dv, a32, b32, fB, fD, fw, fx, fL};
  }
  // symbolic patch arrays
  const PatchSymbolic &ps = h->ps;
  std::vector<int> sym;
  auto push = [&](const std::vector<int> &v) {
    size_t o = sym.size();
    sym.insert(sym.end(), v.begin(), v.end());
    return o;
  };
  std::vector<int> passes;
  for (int t = 0; t < ps.npass; ++t) {
    passes.push_back(ps.pass_g[t]);
    passes.push_back(ps.pass_k[t]);
    passes.push_back(ps.pass_base[t]);
  }
  size_t o_off = push(ps.off), o_rp = push(ps.rowptr), o_col = push(ps.col), o_er = push(h->erow),
         o_up = push(ps.uptr), o_ur = push(ps.urow), o_upos = push(ps.upos), o_fp = push(ps.flev_ptr),
         o_fr = push(ps.flev_rows), o_bp = push(ps.blev_ptr), o_br = push(ps.blev_rows), o_p1 = push(ps.pos1),
         o_p2 = push(ps.pos2), o_pass = push(passes), o_ecol = push(ps.ecol), o_erow = push(ps.erow);
  int *dsym = nullptr;
  if ((e = upload(h, &dsym, sym))) return bail(e);
  h->P = PatchDev{ps.nrows, ps.nnz, (int)ps.flev_ptr.size() - 1, (int)ps.blev_ptr.size() - 1,
                  dsym + o_off, dsym + o_rp, dsym + o_col, dsym + o_er, dsym + o_up, dsym + o_ur, dsym + o_upos,
                  dsym + o_fp, dsym + o_fr, dsym + o_bp, dsym + o_br, ps.stride, dsym + o_p1, dsym + o_p2};
  int kmax = 1;
  for (int k : ps.pass_k) kmax = std::max(kmax, k);
  h->PE = PatchEllDev{ps.nrows, ps.npass, ps.ef + ps.eb, ps.stride, kmax, dsym + o_pass, dsym + o_ecol,
                      dsym + o_erow, dsym + o_off,
                      patch_regs_table_matches(p, passes.data(), ps.npass, ps.nrows, ps.ef + ps.eb, ps.ell0) ? 1 : 0,
                      ps.ell0};
  if (patch_solve_lds_bytes(h->PE, sizeof(double), 1) > 160 * 1024)
    return bail(fail(ctx, RZ_ERR_ARG, "patch schedule does not fit the LDS"));
  const size_t nf = (size_t)h->nvert * ps.stride, nzb = (size_t)h->nvert * ps.nrows;
  const size_t neb = (size_t)h->ncells * (p + 1) * (p + 1) * (p + 1);
  if ((e = dalloc(h, &h->eb64, neb)) || (e = dalloc(h, &h->eb32, neb)) || (e = dalloc(h, &h->f64, nf)) ||
      (e = dalloc(h, &h->f32, nf)) || (e = dalloc(h, &h->zb64, nzb)) ||
      (e = dalloc(h, &h->zb32, nzb)) || (e = dalloc(h, &h->rt64, h->ndofs)) || (e = dalloc(h, &h->rt32, h->ndofs)) ||
      (e = dalloc(h, &h->r32, h->ndofs)) || (e = dalloc(h, &h->z32, h->ndofs)) || (e = dalloc(h, &h->vt, h->ndofs)) ||
      (e = dalloc(h, &h->vaz, h->ndofs)) || (e = dalloc(h, &h->vr, h->ndofs)) || (e = dalloc(h, &h->kr, h->ndofs)) ||
      (e = dalloc(h, &h->kz, h->ndofs)) || (e = dalloc(h, &h->kp, h->ndofs)) || (e = dalloc(h, &h->kAp, h->ndofs)) ||
      (e = dalloc(h, &h->kro, h->ndofs)) || (e = dalloc(h, &h->partials, dots_partials_size())) ||
      (e = dalloc(h, &h->dots, 8)))
    return bail(e);
  if (hipHostMalloc((void **)&h->hdots, 8 * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return bail(fail(ctx, RZ_ERR_OOM, "pinned host buffer"));
  if (opts->precision == RZ_PREC_DEFECT &&
      ((e = dalloc(h, &h->kp32, h->ndofs)) || (e = dalloc(h, &h->kAp32, h->ndofs)) ||
       (e = dalloc(h, &h->ko32, h->ndofs)) || (e = dalloc(h, &h->ke32, h->ndofs)) ||
       (e = dalloc(h, &h->t32, h->ndofs)) || (e = dalloc(h, &h->az32, h->ndofs)) ||
       (e = dalloc(h, &h->vr32, h->ndofs))))
    return bail(e);
  // the workspace of the vertex patches: keep rows of empty slots well defined
  launch_fill(h->zb64, 0.0, (int64_t)nzb, s);
  // ELL padding of the factors must read as zero
  if (hipMemsetAsync(h->f64, 0, nf * sizeof(double), s) != hipSuccess ||
      hipMemsetAsync(h->f32, 0, nf * sizeof(float), s) != hipSuccess)
    return bail(fail(ctx, RZ_ERR_HIP, "memset"));
  launch_patch_factor(h->L, h->P, h->coef64, h->B64, h->A64, h->lam64, h->f64, h->f32, h->status, s);
  if (hipStreamSynchronize(s) != hipSuccess) return bail(fail(ctx, RZ_ERR_HIP, "patch factorisation failed"));
  int stv = 0;
  if (hipMemcpy(&stv, h->status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return bail(fail(ctx, RZ_ERR_HIP, "status read"));
  if (stv) {
    char msg[128];
    std::snprintf(msg, sizeof msg, "incomplete Cholesky breakdown in vertex patch %d", stv - 1);
    return bail(fail(ctx, RZ_ERR_BREAKDOWN, msg));
  }
  if ((e = dalloc(h, &h->rt1, (size_t)(h->nx + 1) * h->Ny * h->Nz)) ||
      (e = dalloc(h, &h->rt2, (size_t)(h->nx + 1) * (h->ny + 1) * h->Nz)) ||
      (e = dalloc(h, &h->rc, (size_t)(h->nx + 1) * (h->ny + 1) * (h->nz + 1))) ||
      (e = dalloc(h, &h->xc, (size_t)(h->nx + 1) * (h->ny + 1) * (h->nz + 1))))
    return bail(e);
  if ((e = setup_coarse(h))) return bail(e);
  if (opts->omega > 0) {
    h->omega = opts->omega;
  } else {
    double lam = 0;
    if ((e = estimate_lambda(h, &lam))) return bail(e);
    h->omega = 2.0 / (1.2 * lam);
  }
  if (hipStreamSynchronize(s) != hipSuccess) return bail(fail(ctx, RZ_ERR_HIP, "setup failed"));
  *out = h;
  return RZ_OK;
}

rz_status rz_setup(rz_ctx *ctx, const rz_mesh *mesh, const rz_coef *cf, const rz_opts *opts, rz_problem **out) {
  const rz_status e = setup_impl(ctx, mesh, cf, opts, out);
  if (e == RZ_OK) ctx->nlive += 1;
  return e;
}

rz_status rz_free(rz_problem *h) {
  if (!h) return RZ_OK;
  if (h->ctx && h->ctx->device >= 0) hipStreamSynchronize(h->ctx->stream);
  release(h);
  if (h->ctx) h->ctx->nlive -= 1;
  delete h;
  return RZ_OK;
}

rz_status rz_sizes(const rz_problem *h, int64_t sizes[8]) {
  if (!h || !sizes) return RZ_ERR_ARG;
  sizes[0] = h->ndofs;
  sizes[1] = h->nfree;
  sizes[2] = h->ncells;
  sizes[3] = h->nvert;
  sizes[4] = (int64_t)(h->nx + 1) * (h->ny + 1) * (h->nz + 1);
  sizes[5] = h->ps.nnz;
  sizes[6] = h->ps.nrows;
  sizes[7] = (int64_t)h->patch_vids.size();
  return RZ_OK;
}

rz_status rz_apply(rz_problem *h, const void *x, void *y, rz_dtype t) {
  rz_status e = require_device(h);
  if (e) return e;
  if (!x || !y || x == y) return fail(h->ctx, RZ_ERR_ARG, "rz_apply: bad vectors");
  if (t == RZ_F64) return do_apply64(h, static_cast<const double *>(x), static_cast<double *>(y));
  if (t == RZ_F32) return do_apply32(h, static_cast<const float *>(x), static_cast<float *>(y));
  return fail(h->ctx, RZ_ERR_ARG, "rz_apply: bad dtype");
}

// Bytes of the apply's workspace (face-line buffer of the Cartesian H(grad) path,
// per-cell outputs of the quadrature and vector-space paths) for element size sz.
static size_t apply_workspace_bytes(const rz_problem *h, size_t sz) {
  if (h->space != RZ_GRAD) return (size_t)h->ncells * h->V.cell_dofs * sz;
  const size_t n1 = (size_t)h->p + 1;
  if (h->quad) return (size_t)h->ncells * n1 * n1 * n1 * sz;
  return (size_t)h->ny * h->nz * 4 * h->p * h->Nx * sz;
}

rz_status rz_apply_noalloc(rz_problem *h, const void *x, void *y, rz_dtype t) {
  rz_status e = require_device(h);
  if (e) return e;
  if (!x || !y || x == y) return fail(h->ctx, RZ_ERR_ARG, "rz_apply_noalloc: bad vectors");
  if (t != RZ_F64 && t != RZ_F32) return fail(h->ctx, RZ_ERR_ARG, "rz_apply_noalloc: bad dtype");
  const size_t need = apply_workspace_bytes(h, t == RZ_F64 ? 8 : 4);
  if (need > kScratchBytes) {
    char msg[160];
    std::snprintf(msg, sizeof msg, "rz_apply_noalloc: this problem needs %zu bytes of workspace, more than the %zu "
                  "bytes of the static scratch (use rz_apply)", need, kScratchBytes);
    return fail(h->ctx, RZ_ERR_ARG, msg);
  }
  void *ws = scratch_ptr(h->ctx->device);
  if (!ws) return fail(h->ctx, RZ_ERR_HIP, "rz_apply_noalloc: no scratch address for this device");
  hipStream_t s = h->ctx->stream;
  if (t == RZ_F64) {
    const double *xd = static_cast<const double *>(x);
    double *yd = static_cast<double *>(y), *wd = static_cast<double *>(ws);
    if (h->space != RZ_GRAD) {
      if (launch_apply_vec<double>(h->V, h->coef64, h->B64, h->D64, xd, yd, wd, s))
        return fail(h->ctx, RZ_ERR_ARG, "unsupported degree");
    } else if (h->quad) {
      launch_apply_quad_cells<double>(h->L, h->Q64, xd, yd, wd, s);
      launch_apply_gather<double>(h->L, xd, wd, yd, s);
    } else {
      launch_apply_grad<double>(h->L, h->coef64, h->t.B.data(), h->t.A.data(), xd, nullptr, yd, wd, s);
    }
  } else {
    const float *xf = static_cast<const float *>(x);
    float *yf = static_cast<float *>(y), *wf = static_cast<float *>(ws);
    if (h->space != RZ_GRAD) {
      if (launch_apply_vec<float>(h->V, h->coef32, h->B32, h->D32, xf, yf, wf, s))
        return fail(h->ctx, RZ_ERR_ARG, "unsupported degree");
    } else if (h->quad) {
      launch_apply_quad_cells<float>(h->L, h->Q32, xf, yf, wf, s);
      launch_apply_gather<float>(h->L, xf, wf, yf, s);
    } else {
      launch_apply_grad<float>(h->L, h->coef32, h->t.B.data(), h->t.A.data(), xf, nullptr, yf, wf, s);
    }
  }
  return RZ_OK;
}

rz_status rz_relax(rz_problem *h, const void *r, void *z, rz_dtype t) {
  rz_status e = require_device(h);
  if (e) return e;
  if ((e = require_grad(h))) return e;
  if (!r || !z || r == z) return fail(h->ctx, RZ_ERR_ARG, "rz_relax: bad vectors");
  if (t == RZ_F64) return do_relax64(h, static_cast<const double *>(r), static_cast<double *>(z));
  if (t == RZ_F32) return do_relax32(h, static_cast<const float *>(r), static_cast<float *>(z));
  return fail(h->ctx, RZ_ERR_ARG, "rz_relax: bad dtype");
}

rz_status rz_prolong_add(rz_problem *h, const double *xc, double *xf) {
  rz_status e = require_device(h);
  if (e) return e;
  if ((e = require_grad(h))) return e;
  if (!xc || !xf) return fail(h->ctx, RZ_ERR_ARG, "rz_prolong_add: bad vectors");
  launch_prolong_add_grad(h->L, h->E64, xc, xf, h->ctx->stream);
  return RZ_OK;
}

rz_status rz_restrict(rz_problem *h, const double *rf, double *rcv) {
  rz_status e = require_device(h);
  if (e) return e;
  if ((e = require_grad(h))) return e;
  if (!rf || !rcv) return fail(h->ctx, RZ_ERR_ARG, "rz_restrict: bad vectors");
  launch_restrict_grad(h->L, h->E64, rf, rcv, h->rt1, h->rt2, h->ctx->stream);
  return RZ_OK;
}

rz_status rz_coarse_solve(rz_problem *h, const double *rcv, double *xcv) {
  rz_status e = require_device(h);
  if (e) return e;
  if ((e = require_grad(h))) return e;
  if (!rcv || !xcv || rcv == xcv) return fail(h->ctx, RZ_ERR_ARG, "rz_coarse_solve: bad vectors");
  return do_coarse(h, rcv, xcv);
}

rz_status rz_vcycle(rz_problem *h, const double *r, double *z) {
  rz_status e = require_device(h);
  if (e) return e;
  if ((e = require_grad(h))) return e;
  if (!r || !z || r == z) return fail(h->ctx, RZ_ERR_ARG, "rz_vcycle: bad vectors");
  return do_vcycle(h, r, z);
}

rz_status rz_solve(rz_problem *h, const double *b, double *x, rz_solve_info *info) {
  rz_status e = require_device(h);
  if (e) return e;
  if ((e = require_grad(h))) return e;
  if (!b || !x || b == x) return fail(h->ctx, RZ_ERR_ARG, "rz_solve: bad vectors");
  if (h->opts.precision == RZ_PREC_DEFECT) return defect_solve(h, b, x, info);
  PcgRun R;
  R.h = h;
  R.b = b;
  R.x = x;
  while (R.phase != PcgRun::DONE) {
    if ((e = pcg_step(R))) {
      pcg_release(R);
      return e;
    }
    if (R.phase != PcgRun::DONE && hipStreamSynchronize(h->ctx->stream) != hipSuccess) {
      pcg_release(R);
      return fail(h->ctx, RZ_ERR_HIP, "stream execution failed during the solve");
    }
  }
  return pcg_finish(R, info);
}

rz_status rz_solve_batched(rz_problem *const *hs, int32_t n, const double *const *b, double *const *x, int32_t nrhs,
                           rz_solve_info *infos) {
  if (!hs || !b || !x || n < 0 || nrhs < 1) return RZ_ERR_ARG;
  for (int i = 0; i < n; ++i) {
    if (!hs[i] || !b[i] || !x[i]) return RZ_ERR_ARG;
    rz_status e = require_device(hs[i]);
    if (e || (e = require_grad(hs[i]))) return e;
    if (hs[i]->opts.precision == RZ_PREC_DEFECT)
      return fail(hs[i]->ctx, RZ_ERR_ARG, "rz_solve_batched: the defect-correction protocol is not batched");
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(hs[i]->ctx, RZ_ERR_ARG, "rz_solve_batched: a problem appears twice");
  }
  // One running instance per problem (its right-hand sides one after another).  Each
  // enqueued step ends with an event; the host advances every instance whose event
  // has completed, so problems on different streams progress independently and the
  // device works on one while the host serves another.
  std::vector<PcgRun> run(n);
  std::vector<int> rhs(n, 0);
  std::vector<rz_status> st(n, RZ_OK);
  std::vector<hipEvent_t> ev(n, nullptr);
  std::vector<char> pending(n, 0);
  rz_status first_fail = RZ_OK;  // first non-OK result of a finished solve
  auto start = [&](int i) {
    run[i] = PcgRun();
    run[i].h = hs[i];
    run[i].b = b[i] + (int64_t)rhs[i] * hs[i]->ndofs;
    run[i].x = x[i] + (int64_t)rhs[i] * hs[i]->ndofs;
  };
  for (int i = 0; i < n; ++i) {
    start(i);
    if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess) {
      for (int j = 0; j < i; ++j) hipEventDestroy(ev[j]);
      return fail(hs[i]->ctx, RZ_ERR_HIP, "rz_solve_batched: event creation");
    }
  }
  auto live = [&](int i) { return rhs[i] < nrhs && st[i] == RZ_OK; };
  int active = n;
  while (active > 0) {
    bool progressed = false;
    for (int i = 0; i < n; ++i) {
      if (!live(i)) continue;
      if (pending[i]) {
        const hipError_t q = hipEventQuery(ev[i]);
        if (q == hipErrorNotReady) continue;
        pending[i] = 0;
        if (q != hipSuccess) {
          st[i] = fail(hs[i]->ctx, RZ_ERR_HIP, "stream execution");
          continue;
        }
      }
      progressed = true;
      if (run[i].phase == PcgRun::DONE) {
        rz_solve_info inf{};
        const rz_status r = pcg_finish(run[i], &inf);
        if (infos) infos[(int64_t)i * nrhs + rhs[i]] = inf;
        if (r != RZ_OK && first_fail == RZ_OK) first_fail = r;  // keep solving the others
        if (++rhs[i] >= nrhs) continue;
        start(i);
      }
      rz_status e = pcg_step(run[i]);
      if (e) {
        st[i] = e;
        continue;
      }
      if (run[i].phase != PcgRun::DONE) {
        if (hipEventRecord(ev[i], hs[i]->ctx->stream) != hipSuccess) {
          st[i] = fail(hs[i]->ctx, RZ_ERR_HIP, "event record");
          continue;
        }
        pending[i] = 1;
      }
    }
    active = 0;
    for (int i = 0; i < n; ++i) active += live(i);
    if (!progressed && active > 0) std::this_thread::yield();
  }
  for (int i = 0; i < n; ++i) {
    hipEventDestroy(ev[i]);
    pcg_release(run[i]);  // instances stopped by an error still hold their events
  }
  for (int i = 0; i < n; ++i)
    if (st[i]) return st[i];
  return first_fail;
}

rz_status rz_aux_data(const rz_problem *h, double *targets, double *features, double *base) {
  if (!h) return RZ_ERR_ARG;
  if (!h->quad) return fail(h->ctx, RZ_ERR_ARG, "rz_aux_data: needs trilinear cells or sampled coefficients");
  std::vector<double> kP, kD;
  christoffel(h->t, h->qt, kP, kD);
  const int nvx = h->nx + 1, nvy = h->ny + 1;
  for (int64_t c = 0; c < h->ncells; ++c) {
    int cx = c % h->nx, cy = (c / h->nx) % h->ny, cz = c / ((int64_t)h->nx * h->ny);
    double corners[24];
    for (int k = 0; k < 8; ++k) {
      const int64_t vid = (cx + (k & 1)) + nvx * ((cy + ((k >> 1) & 1)) + (int64_t)nvy * (cz + (k >> 2)));
      for (int r = 0; r < 3; ++r) corners[3 * k + r] = h->vert[3 * vid + r];
    }
    if (targets && !fit_targets(corners, &h->asmp[27 * c], &h->bsmp[27 * c], h->qt, kP, kD, targets + 6 * c))
      return fail(h->ctx, RZ_ERR_ARG, "non-positive Jacobian determinant");
    if (features) cell_features(corners, &h->asmp[27 * c], features + 51 * c);
    if (base)
      for (int k = 0; k < 6; ++k) base[6 * c + k] = h->coef[6 * c + k];
  }
  return RZ_OK;
}

// Upload per-cell auxiliary weights and refactor the vertex patches with them.
// Returns 0, or the 1-based index of the patch slot whose IC broke down.
namespace {
rz_status refactor_patches(rz_problem *h, int *breakdown) {
  hipStream_t s = h->ctx->stream;
  std::vector<float> c32(h->coef.begin(), h->coef.end());
  HIPCALL(h, hipMemcpyAsync(h->coef64, h->coef.data(), sizeof(double) * h->coef.size(), hipMemcpyHostToDevice, s));
  HIPCALL(h, hipMemcpyAsync(h->coef32, c32.data(), sizeof(float) * c32.size(), hipMemcpyHostToDevice, s));
  const size_t nf = (size_t)h->nvert * h->ps.stride;
  HIPCALL(h, hipMemsetAsync(h->f64, 0, nf * sizeof(double), s));
  HIPCALL(h, hipMemsetAsync(h->f32, 0, nf * sizeof(float), s));
  HIPCALL(h, hipMemsetAsync(h->status, 0, sizeof(int), s));
  launch_patch_factor(h->L, h->P, h->coef64, h->B64, h->A64, h->lam64, h->f64, h->f32, h->status, s);
  HIPCALL(h, hipMemcpyAsync(breakdown, h->status, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCALL(h, hipStreamSynchronize(s));
  return RZ_OK;
}
}  // namespace

rz_status rz_set_aux(rz_problem *h, const double *coef6) {
  rz_status e = require_device(h);
  if (e) return e;
  if ((e = require_grad(h))) return e;
  // On Cartesian cells with cellwise-constant coefficients the six weights are the
  // operator's own (P = A there): replacing them would change the matrix solved.
  if (!h->quad)
    return fail(h->ctx, RZ_ERR_ARG, "rz_set_aux: needs trilinear cells or sampled coefficients (the weights of a "
                                    "Cartesian problem define its operator)");
  if (!coef6) return fail(h->ctx, RZ_ERR_ARG, "rz_set_aux: null weights");
  for (int64_t k = 0; k < 6 * h->ncells; ++k)
    if (!(coef6[k] > 0)) return fail(h->ctx, RZ_ERR_ARG, "rz_set_aux: weights must be positive");
  std::vector<double> old = h->coef;
  h->coef.assign(coef6, coef6 + 6 * h->ncells);
  int stv = 0;
  if ((e = refactor_patches(h, &stv))) return e;
  if (stv) {  // restore the previous weights and their factors
    h->coef.swap(old);
    int st2 = 0;
    if ((e = refactor_patches(h, &st2))) return e;
    return fail(h->ctx, RZ_ERR_BREAKDOWN,
                "incomplete Cholesky breakdown with the new weights (previous weights restored)");
  }
  if (!(h->opts.omega > 0)) {
    double lam = 0;
    if ((e = estimate_lambda(h, &lam))) return e;
    h->omega = 2.0 / (1.2 * lam);
  }
  HIPCALL(h, hipStreamSynchronize(h->ctx->stream));
  return RZ_OK;
}

rz_status rz_export(rz_problem *h, int what, int64_t index, void *buf, int64_t *bytes) {
  if (!h || !bytes) return RZ_ERR_ARG;
  const int p = h->p, n1 = p + 1;
  std::vector<unsigned char> out;
  auto put = [&](const void *src, size_t nb) {
    size_t o = out.size();
    out.resize(o + nb);
    std::memcpy(out.data() + o, src, nb);
  };
  switch (what) {
    case RZ_EXPORT_DOFMAP: {
      if (h->space != RZ_GRAD) {
        const VecDev &Vd = h->V;
        for (int64_t c = 0; c < h->ncells; ++c) {
          const int cc[3] = {(int)(c % h->nx), (int)((c / h->nx) % h->ny), (int)(c / ((int64_t)h->nx * h->ny))};
          for (int m = 0; m < 3; ++m) {
            int e3[3];
            for (int a = 0; a < 3; ++a) e3[a] = (h->space == RZ_CURL ? a != m : a == m) ? p + 1 : p;
            for (int l = 0; l < e3[2]; ++l)
              for (int j = 0; j < e3[1]; ++j)
                for (int i = 0; i < e3[0]; ++i) {
                  const int64_t g = Vd.off[m] + (int64_t)(cc[0] * p + i) +
                                    (int64_t)Vd.ext[m][0] * ((cc[1] * p + j) + (int64_t)Vd.ext[m][1] * (cc[2] * p + l));
                  put(&g, sizeof g);
                }
          }
        }
        break;
      }
      for (int64_t c = 0; c < h->ncells; ++c) {
        int cx = c % h->nx, cy = (c / h->nx) % h->ny, cz = c / ((int64_t)h->nx * h->ny);
        for (int l = 0; l < n1; ++l)
          for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n1; ++i) {
              int64_t g = (int64_t)(cx * p + i) + (int64_t)h->Nx * ((cy * p + j) + (int64_t)h->Ny * (cz * p + l));
              put(&g, sizeof g);
            }
      }
      break;
    }
    case RZ_EXPORT_PATCH:
    case RZ_EXPORT_IC_PATTERN:
    case RZ_EXPORT_IC_FACTOR: {
      if (index < 0 || index >= (int64_t)h->patch_vids.size()) return fail(h->ctx, RZ_ERR_ARG, "bad patch index");
      const int64_t vid = h->patch_vids[index];
      std::vector<int> loc(h->ps.nrows, -1);
      std::vector<std::array<int, 3>> G(h->ps.nrows);
      int cnt = 0;
      for (int k = 0; k < h->ps.nrows; ++k) {
        int g3[3];
        if (patch_row_present(h, vid, k, g3)) {
          loc[k] = cnt++;
          G[k] = {g3[0], g3[1], g3[2]};
        }
      }
      if (what == RZ_EXPORT_PATCH) {
        put(&vid, sizeof vid);
        for (int k = 0; k < h->ps.nrows; ++k)
          if (loc[k] >= 0) {
            int64_t g = (int64_t)G[k][0] + (int64_t)h->Nx * (G[k][1] + (int64_t)h->Ny * G[k][2]);
            put(&g, sizeof g);
          }
        break;
      }
      std::vector<double> vals;
      if (what == RZ_EXPORT_IC_FACTOR) {
        rz_status e = require_device(h);
        if (e) return e;
        vals.resize(h->ps.stride);
        HIPCALL(h, hipStreamSynchronize(h->ctx->stream));
        HIPCALL(h, hipMemcpy(vals.data(), h->f64 + vid * (int64_t)h->ps.stride, sizeof(double) * h->ps.stride,
                             hipMemcpyDeviceToHost));
      }
      for (int r = 0; r < h->ps.nrows; ++r) {
        if (loc[r] < 0) continue;
        for (int k = h->ps.rowptr[r]; k < h->ps.rowptr[r + 1]; ++k) {
          int c = h->ps.col[k];
          if (loc[c] < 0) continue;
          if (r != c && !patch_entry_allowed(h, vid, G[r].data(), G[c].data())) continue;
          if (what == RZ_EXPORT_IC_PATTERN) {
            int pr[2] = {loc[r], loc[c]};
            put(pr, sizeof pr);
          } else {
            put(&vals[h->ps.pos1[k]], sizeof(double));
          }
        }
      }
      break;
    }
    case RZ_EXPORT_TABLES1D: {
      std::vector<double> v(h->t.lam);
      v.insert(v.end(), h->t.B.begin(), h->t.B.end());
      v.insert(v.end(), h->t.A.begin(), h->t.A.end());
      v.insert(v.end(), h->t.D.begin(), h->t.D.end());
      v.insert(v.end(), h->t.E.begin(), h->t.E.end());
      put(v.data(), sizeof(double) * v.size());
      break;
    }
    case RZ_EXPORT_AUXCOEF:
      put(h->coef.data(), sizeof(double) * h->coef.size());
      break;
    case RZ_EXPORT_OMEGA:
      put(&h->omega, sizeof(double));
      break;
    case RZ_EXPORT_PATCH_KERNEL: {
      const int32_t v[2] = {patch_solve_uses_regs(h->PE, h->p, 8) ? 1 : 0, patch_solve_uses_regs(h->PE, h->p, 4) ? 1 : 0};
      put(v, sizeof v);
      break;
    }
    default:
      return fail(h->ctx, RZ_ERR_ARG, "bad export kind");
  }
  if (!buf) {
    *bytes = (int64_t)out.size();
    return RZ_OK;
  }
  if (*bytes < (int64_t)out.size()) return fail(h->ctx, RZ_ERR_ARG, "export buffer too small");
  std::memcpy(buf, out.data(), out.size());
  *bytes = (int64_t)out.size();
  return RZ_OK;
}

rz_status rz_sync(rz_problem *h) {
  rz_status e = require_device(h);
  if (e) return e;
  HIPCALL(h, hipStreamSynchronize(h->ctx->stream));
  return take_device_status(h);
}

rz_status rz_timing_enable(rz_problem *h, int on) {
  rz_status e = require_device(h);
  if (e) return e;
  h->timing = on != 0;
  return RZ_OK;
}

rz_status rz_timing_read(rz_problem *h, double ms[RZ_NKERNELS], int64_t count[RZ_NKERNELS]) {
  rz_status e = require_device(h);
  if (e) return e;
  HIPCALL(h, hipStreamSynchronize(h->ctx->stream));
  for (int k = 0; k < RZ_NKERNELS; ++k) {
    if (ms) ms[k] = 0.0;
    if (count) count[k] = 0;
  }
  for (auto &u : h->ev_used) {
    float t = 0;
    hipEventElapsedTime(&t, h->ev_pool[u.second].first, h->ev_pool[u.second].second);
    if (ms) ms[u.first] += t;
    if (count) count[u.first] += 1;
  }
  h->ev_used.clear();
  return RZ_OK;
}

}  // extern "C"
