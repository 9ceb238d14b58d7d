// C ABI (include/rz.h): problem setup on the host and the device, and the
// stream-ordered compute calls that drive the HIP kernels.
#include "../../include/rz.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "kernels.hpp"
#include "lattice.hpp"
#include "geom.hpp"
#include "hmg.hpp"
#include "patch.hpp"
#include "tables1d.hpp"
#include "vec_local.hpp"

struct rz_ctx {
  int device = -1;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream on which PCG iterations are captured
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
  // ---- H(curl) / H(div): statically condensed Pavarino-Hiptmair relaxation --------
  VecCellDev<double> vc64{};
  VecCellDev<float> vc32{};
  int nGam = 0;
  int *gam = nullptr;                       // free interface DoFs, ascending
  int *cg_ptr = nullptr, *cg_pos = nullptr; // condensation sums (positions in veb)
  double *veb64 = nullptr;
  float *veb32 = nullptr;                   // ncells * nG per-cell P_GI z_I
  double *vrt64 = nullptr;
  float *vrt32 = nullptr;                   // condensed right-hand side (all DoFs)
  EdgeDev ed{};                             // curl: edge stars of the problem
  double *efac64 = nullptr, *ezb64 = nullptr;
  float *efac32 = nullptr, *ezb32 = nullptr;
  int *eg_ptr = nullptr, *eg_pos = nullptr; // sums back (rows = gam)
  std::vector<int64_t> edge_ids;            // curl: edge of every patch; div: of the potential's
  std::vector<int> edge_idx;                // slot DoFs (host copy, for exports)
  int edge_nslot = 0;
  double *dinv64 = nullptr;
  float *dinv32 = nullptr;                  // div: face stars (diagonal)
  rz_problem *pot = nullptr;                // curl: Q_p potential problem (vertex-star IC)
  EdgeDev ped{};                            // div: edge stars of the NCE potential problem
  double *pfac64 = nullptr, *pzb64 = nullptr;
  float *pfac32 = nullptr, *pzb32 = nullptr;
  int npg = 0;
  int *pg_rows = nullptr, *pg_ptr = nullptr, *pg_pos = nullptr;
  int ndt = 0;                              // Dt^T: rows = free interface DoFs of the potential
  int *dt_rows = nullptr, *dt_ptr = nullptr, *dt_col = nullptr;
  double *dt_val64 = nullptr;
  float *dt_val32 = nullptr;
  int *d_ptr = nullptr, *d_col = nullptr;   // Dt: rows = gam
  double *d_val64 = nullptr;
  float *d_val32 = nullptr;
  int64_t pndofs = 0;
  double *vq64 = nullptr, *vy64 = nullptr;
  float *vq32 = nullptr, *vy32 = nullptr;   // potential vectors
  int ncf = 0;                              // free DoFs of the p = 1 space
  double *cinv64 = nullptr;
  float *cinv32 = nullptr;                  // dense A_0^{-1}
  double *csym = nullptr;                   // partial products of the symmetric product
  int *pr_ptr = nullptr, *pr_col = nullptr; // restriction (rows: coarse free, compact)
  double *pr_val = nullptr;
  int npf = 0;
  int *pp_rows = nullptr, *pp_ptr = nullptr, *pp_col = nullptr;  // prolongation
  double *pp_val = nullptr;
  double *vcr = nullptr, *vcx = nullptr;
  int nDir = 0;
  int *dlist = nullptr;
  std::vector<char> dmask;                  // host: Dirichlet rows
  // several right-hand sides: planar copies of the caller's interleaved
  // multi-vectors (mcap vectors each) and the per-vector buffers of right-hand
  // sides 1 .. mcap-1 (right-hand side 0 uses the buffers above)
  int mcap = 0;
  size_t mnzb = 0;
  std::vector<void *> mallocs;
  double *mb = nullptr, *mx = nullptr, *mvec = nullptr, *mzb64 = nullptr, *mdots = nullptr, *mhdots = nullptr;
  float *mf32 = nullptr, *mzb32 = nullptr;
  // the paper's auxiliary on trilinear cells (broken diagonals, eq.
  // sum-factorization_approx) instead of the separable per-cell weights
  bool pd = false;
  std::vector<double> pd_host_dm, pd_host_da;   // per cell, until uploaded
  double *pd_dm = nullptr, *pd_da = nullptr, *pd_G = nullptr, *pd_D64 = nullptr;
  PdSolve<double> pds64{};
  PdSolve<float> pds32{};
  // autotuned streaming patch solve: per precision (FP64, FP32) the candidates' caps
  // and their times (ms per launch), the chosen cap
  std::vector<std::pair<int, double>> tune[2];
  // per-kernel timing
  bool timing = false;
  // PCG iterations captured as HIP graphs (opts.graph), one set per parity of the
  // iteration count (the CG scalars alternate between two slots): the segments
  // between the cooperative Q_1 coarse solves, which run between their replays, and
  // the vectors and buffer generation they were captured for
  struct IterGraph {
    std::vector<hipGraphExec_t> seg;
    std::vector<double *> xs;
    int nv = 0;
    uint64_t gen = 0;
    bool f32 = false, ok = false;
  } ig[2];
  uint64_t graph_gen = 1;                  // bumped when buffers named by the graphs change
  int64_t graph_stat[3] = {0, 0, 0};       // captures, replayed iterations, segments
  // geometric h-multigrid on the Q_1 space (rz_opts.coarse = RZ_COARSE_HMG): levels
  // with a coarser one below (n rows; A, D^{-1}, P to and R from the next level; the
  // level's input b and output o, unused on level 0; residual t and iterate x), then
  // the coarsest level's dense inverse
  struct HmgLevel {
    int n = 0, nnext = 0, aw = 0, pw = 0, rw = 0;  // rows; ELL widths of A, P, R
    int *a_col = nullptr, *p_col = nullptr, *r_col = nullptr;
    double *a_val = nullptr, *dinv = nullptr, *p_val = nullptr, *r_val = nullptr;
    double *b = nullptr, *o = nullptr, *t = nullptr, *x = nullptr;
    double w = 0.0;                               // Jacobi weight on A
    // H(curl)/H(div): potential space (np DoFs), G and G^T in ELL, its Jacobi data
    int np = 0, gw = 0, gtw = 0;
    int *g_col = nullptr, *gt_col = nullptr;
    double *g_val = nullptr, *gt_val = nullptr, *dpinv = nullptr, *x2 = nullptr, *y = nullptr;
    double wp = 0.0;
  };
  bool hmg_on = false;
  std::vector<HmgLevel> hmg;
  std::vector<int64_t> hmg_sizes;           // rows of levels 0..L
  int hmg_nc = 0;
  double *hmg_cinv = nullptr, *hmg_cb = nullptr, *hmg_co = nullptr, *hmg_work = nullptr;
  // exact Cholesky vertex-star solves (opts.patch_solver): W = L^{-1} per slot,
  // dense lower packed by rows
  double *cw64 = nullptr;
  float *cw32 = nullptr;
  // full vertex stars (opts.decomposition): rows per star, the star's offsets (in PF),
  // and the per-slot solutions
  int nrf = 0;
  PatchDev PF{};
  // H(curl)/H(div) vertex stars (opts.decomposition): patches, their index lists
  // (nrf entries each), and per free DoF the positions of its star solutions
  int nvs = 0, nvfree = 0;
  bool vs_sc = false;                       // vertex stars on the condensed interface (SC-PAFW)
  // PH without static condensation (RZ_DECOMP_FULL_PH): the edge / face stars of the
  // space, the NCE_p edge stars of the H(div) potential (the H(curl) potential uses the
  // full vertex stars of its Q_p problem), the full exterior derivative D and D^T
  struct StarSet {
    int np = 0, nr = 0, nfree = 0;
    int *idx = nullptr, *rows = nullptr, *ptr = nullptr, *pos = nullptr;
    double *w64 = nullptr, *zb64 = nullptr;
    float *w32 = nullptr, *zb32 = nullptr;
  };
  StarSet ph_s, ph_p;
  int nphd = 0, nphdt = 0;
  int *phd_rows = nullptr, *phd_ptr = nullptr, *phd_col = nullptr;
  int *phdt_rows = nullptr, *phdt_ptr = nullptr, *phdt_col = nullptr;
  double *phd_val64 = nullptr, *phdt_val64 = nullptr;
  float *phd_val32 = nullptr, *phdt_val32 = nullptr;
  int *vs_idx = nullptr, *vs_rows = nullptr, *vs_ptr = nullptr, *vs_pos = nullptr;
  double *fzb64 = nullptr;
  float *fzb32 = nullptr;
  std::vector<hipGraph_t> *cap = nullptr;  // capture in progress: the closed segments
  bool cap_bad = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
  std::vector<std::pair<int, size_t>> ev_used;  // (kernel id, pool index)
};

namespace {

rz_status fail(rz_ctx *ctx, rz_status st, const std::string &msg) {
  if (ctx) ctx->err = msg;
  return st;
}

rz_status take_device_status(rz_problem *h);
rz_status setup_vec_relax(rz_problem *h, const std::vector<double> &al, const std::vector<double> &be,
                          const std::vector<std::array<double, 3>> &hs);
rz_status alloc_krylov(rz_problem *h);
rz_status estimate_lambda(rz_problem *h, double *lam_out);

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

// The workspace of calls on several right-hand sides (grown on first use with more
// vectors than it holds, kept until rz_free).
void free_multi(rz_problem *h) {
  for (void *p : h->mallocs) hipFree(p);
  h->mallocs.clear();
  if (h->mhdots) hipHostFree(h->mhdots);
  h->mb = h->mx = h->mvec = h->mzb64 = h->mdots = h->mhdots = nullptr;
  h->mf32 = h->mzb32 = nullptr;
  h->mcap = 0;
  h->mnzb = 0;
}

constexpr int kRhsVecs = 7;  // FP64 vectors per extra right-hand side: r, z, p, Ap, r_old, V-cycle residual, rt
constexpr int kRhsVecs32 = 2;  // FP32: rt, r

rz_status ensure_multi(rz_problem *h, int nv) {
  if (nv <= h->mcap) return RZ_OK;
  HIPCALL(h, hipStreamSynchronize(h->ctx->stream));
  free_multi(h);
  ++h->graph_gen;  // captured iterations name the buffers being replaced
  const size_t n = (size_t)h->ndofs, extra = (size_t)nv - 1;
  const size_t nzb = h->space == RZ_GRAD ? (size_t)h->nvert * h->ps.nrows : 0;
  auto al = [&](auto **ptr, size_t count) -> rz_status {
    void *q = nullptr;
    const hipError_t e = hipMalloc(&q, sizeof(**ptr) * (count ? count : 1));
    if (e != hipSuccess) return fail(h->ctx, RZ_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
    h->mallocs.push_back(q);
    *ptr = static_cast<std::remove_reference_t<decltype(*ptr)>>(q);
    return RZ_OK;
  };
  rz_status e;
  if ((e = al(&h->mb, nv * n)) || (e = al(&h->mx, nv * n))) return e;
  if (extra) {
    if ((e = al(&h->mvec, extra * kRhsVecs * n)) || (e = al(&h->mf32, extra * kRhsVecs32 * n)) ||
        (e = al(&h->mdots, 8 * extra)))
      return e;
    if (nzb) {
      if ((e = al(&h->mzb64, extra * nzb)) || (e = al(&h->mzb32, extra * nzb))) return e;
      launch_fill(h->mzb64, 0.0, (int64_t)(extra * nzb), h->ctx->stream);
      launch_fill_f(h->mzb32, 0.0f, (int64_t)(extra * nzb), h->ctx->stream);
    }
    if (hipHostMalloc((void **)&h->mhdots, 8 * extra * sizeof(double), hipHostMallocDefault) != hipSuccess)
      return fail(h->ctx, RZ_ERR_OOM, "pinned host buffer");
  }
  h->mcap = nv;
  h->mnzb = nzb;
  return RZ_OK;
}

// Buffers of right-hand side i of a multi-vector call.
struct RhsBufs {
  double *r, *z, *p, *Ap, *ro, *vr, *rt64, *zb64, *dots, *hdots;
  float *rt32, *zb32, *r32;
};

RhsBufs rhs_bufs(rz_problem *h, int i) {
  if (i == 0)
    return {h->kr, h->kz, h->kp, h->kAp, h->kro, h->vr, h->rt64, h->zb64, h->dots, h->hdots, h->rt32, h->zb32, h->r32};
  const size_t n = (size_t)h->ndofs, k = (size_t)i - 1;
  double *v = h->mvec + k * kRhsVecs * n;
  float *f = h->mf32 + k * kRhsVecs32 * n;
  return {v,         v + n,     v + 2 * n, v + 3 * n, v + 4 * n, v + 5 * n, v + 6 * n,
          h->mzb64 ? h->mzb64 + k * h->mnzb : nullptr,         h->mdots + 8 * k, h->mhdots + 8 * k,
          f,         h->mzb32 ? h->mzb32 + k * h->mnzb : nullptr,          f + n};
}

template <typename T>
std::vector<T> as_type(const std::vector<double> &v) {
  return std::vector<T>(v.begin(), v.end());
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

// z_D = r_D (r == nullptr: z_D = 0) on the Dirichlet rows of the problem's space
void dir_copy(rz_problem *h, const double *r, double *z, hipStream_t s) {
  if (h->space == RZ_GRAD) launch_dirichlet_copy(h->L, r, z, s);
  else launch_list_copy<double>(h->nDir, h->dlist, r, z, s);
}
void dir_copy_f(rz_problem *h, const float *r, float *z, hipStream_t s) {
  if (h->space == RZ_GRAD) launch_dirichlet_copy_f(h->L, r, z, s);
  else launch_list_copy<float>(h->nDir, h->dlist, r, z, s);
}

// z = M^{-1} r for H(curl) / H(div): statically condensed Pavarino-Hiptmair
// relaxation (eq. schur for the interiors, eq. sc-asm-hiptmair on the interface
// without the coarse term):
//   z_I = P_II^{-1} r_I;  rt = r_G - P_GI z_I;
//   z_G = sum_i R_i^T S_i^{-1} R_i rt + Dt (sum_j R_j^T Bt_j^{-1} R_j) Dt^T rt;
//   z_I -= P_II^{-1} P_IG z_G;  z_D = r_D.
// T selects the precision of vectors, factors and sums.
template <typename T>
struct VecRelaxPtrs {
  const VecCellDev<T> *vc;
  T *veb, *vrt, *ezb, *vq, *vy, *pzb;
  const T *efac, *dinv, *dtv, *dv, *pfac;
  const T *fq, *coefq, *Aq, *lamq;  // curl: the Q_p potential problem
  T *zbq;
};

VecRelaxPtrs<double> vec_ptrs64(rz_problem *h) {
  const rz_problem *q = h->pot;
  return {&h->vc64, h->veb64, h->vrt64, h->ezb64, h->vq64, h->vy64, h->pzb64, h->efac64, h->dinv64,
          h->dt_val64, h->d_val64, h->pfac64, q ? q->f64 : nullptr, q ? q->coef64 : nullptr,
          q ? q->A64 : nullptr, q ? q->lam64 : nullptr, q ? q->zb64 : nullptr};
}
VecRelaxPtrs<float> vec_ptrs32(rz_problem *h) {
  const rz_problem *q = h->pot;
  return {&h->vc32, h->veb32, h->vrt32, h->ezb32, h->vq32, h->vy32, h->pzb32, h->efac32, h->dinv32,
          h->dt_val32, h->d_val32, h->pfac32, q ? q->f32 : nullptr, q ? q->coef32 : nullptr,
          q ? q->A32 : nullptr, q ? q->lam32 : nullptr, q ? q->zb32 : nullptr};
}

double *full_zb(rz_problem *h, double *);
float *full_zb(rz_problem *h, float *);
const double *chol_w(rz_problem *h, const double *);
const float *chol_w(rz_problem *h, const float *);
const double *ph_w(const rz_problem::StarSet &S, const double *) { return S.w64; }
const float *ph_w(const rz_problem::StarSet &S, const float *) { return S.w32; }
double *ph_zb(const rz_problem::StarSet &S, double *) { return S.zb64; }
float *ph_zb(const rz_problem::StarSet &S, float *) { return S.zb32; }
const double *ph_d(const rz_problem *h, const double *) { return h->phd_val64; }
const float *ph_d(const rz_problem *h, const float *) { return h->phd_val32; }
const double *ph_dt(const rz_problem *h, const double *) { return h->phdt_val64; }
const float *ph_dt(const rz_problem *h, const float *) { return h->phdt_val32; }
void fill_any(double *y, int64_t n, hipStream_t s) { launch_fill(y, 0.0, n, s); }
void fill_any(float *y, int64_t n, hipStream_t s) { launch_fill_f(y, 0.0f, n, s); }
template <typename T>
void relax_full(rz_problem *h, const T *r, T *z, T scale, T w, T *acc);

template <typename T>
rz_status relax_vec(rz_problem *h, const VecRelaxPtrs<T> &X, const T *r, T *z) {
  hipStream_t s = h->ctx->stream;
  if (h->ph_s.np) {  // PH without condensation: the space's stars + D (potential stars) D^T
    Timed t(h, RZ_K_PATCH);
    const rz_problem::StarSet &S = h->ph_s;
    T *zb = ph_zb(S, (T *)nullptr);
    launch_dense_patch_solve<T>(S.np, S.nr, S.idx, ph_w(S, (const T *)nullptr), r, zb, s);
    launch_list_gather<T>(S.nfree, S.rows, S.ptr, S.pos, zb, (const T *)nullptr, z, T(1), s);
    fill_any(X.vq, h->pndofs, s);
    launch_csr<T, T, T>(h->nphdt, h->phdt_rows, h->phdt_ptr, h->phdt_col, ph_dt(h, (const T *)nullptr), r, X.vq, 0,
                        s);
    if (h->space == RZ_CURL) {
      relax_full<T>(h->pot, X.vq, X.vy, T(1), T(0), (T *)nullptr);
    } else {
      const rz_problem::StarSet &Q = h->ph_p;
      T *zq = ph_zb(Q, (T *)nullptr);
      launch_dense_patch_solve<T>(Q.np, Q.nr, Q.idx, ph_w(Q, (const T *)nullptr), X.vq, zq, s);
      launch_list_gather<T>(Q.nfree, Q.rows, Q.ptr, Q.pos, zq, (const T *)nullptr, X.vy, T(1), s);
    }
    launch_csr<T, T, T>(h->nphd, h->phd_rows, h->phd_ptr, h->phd_col, ph_d(h, (const T *)nullptr), X.vy, z, 1, s);
    launch_list_copy<T>(h->nDir, h->dlist, r, z, s);
    return RZ_OK;
  }
  if (h->nvs && h->vs_sc) {  // SC-PAFW: condense, vertex stars on the interface, expand
    {
      Timed t(h, RZ_K_CONDENSE);
      launch_vc_condense<T>(h->V, *X.vc, r, z, X.veb, s);
      launch_list_gather<T>(h->nGam, h->gam, h->cg_ptr, h->cg_pos, X.veb, r, X.vrt, T(-1), s);
    }
    {
      Timed t(h, RZ_K_PATCH);
      T *zb = full_zb(h, (T *)nullptr);
      launch_dense_patch_solve<T>(h->nvs, h->nrf, h->vs_idx, chol_w(h, (const T *)nullptr), X.vrt, zb, s);
      launch_list_gather<T>(h->nvfree, h->vs_rows, h->vs_ptr, h->vs_pos, zb, (const T *)nullptr, z, T(1), s);
    }
    {
      Timed t(h, RZ_K_EXPAND);
      launch_vc_expand<T>(h->V, *X.vc, z, s);
      launch_list_copy<T>(h->nDir, h->dlist, r, z, s);
    }
    return RZ_OK;
  }
  if (h->nvs) {  // vertex stars without static condensation (PAFW)
    Timed t(h, RZ_K_PATCH);
    T *zb = full_zb(h, (T *)nullptr);
    launch_dense_patch_solve<T>(h->nvs, h->nrf, h->vs_idx, chol_w(h, (const T *)nullptr), r, zb, s);
    launch_list_gather<T>(h->nvfree, h->vs_rows, h->vs_ptr, h->vs_pos, zb, (const T *)nullptr, z, T(1), s);
    launch_list_copy<T>(h->nDir, h->dlist, r, z, s);
    return RZ_OK;
  }
  {
    Timed t(h, RZ_K_CONDENSE);
    launch_vc_condense<T>(h->V, *X.vc, r, z, X.veb, s);
    launch_list_gather<T>(h->nGam, h->gam, h->cg_ptr, h->cg_pos, X.veb, r, X.vrt, T(-1), s);
  }
  {
    Timed t(h, RZ_K_PATCH);
    if (h->space == RZ_CURL) {  // edge stars (exact Cholesky)
      launch_edge_solve<T>(h->ed, X.efac, X.vrt, X.ezb, s);
      launch_list_gather<T>(h->nGam, h->gam, h->eg_ptr, h->eg_pos, X.ezb, (const T *)nullptr, z, T(1), s);
    } else {  // face stars: the interface Schur complement is diagonal on a face
      launch_rows_scale<T>(h->nGam, h->gam, X.dinv, X.vrt, z, s);
    }
    // potential term: Dt (sum_j R_j^T Bt_j^{-1} R_j) Dt^T rt
    launch_csr<T, T, T>(h->ndt, h->dt_rows, h->dt_ptr, h->dt_col, X.dtv, X.vrt, X.vq, 0, s);
    if (h->space == RZ_CURL) {
      rz_problem *q = h->pot;
      if (launch_patch_solve<T>(q->L, q->PE, X.fq, X.vq, X.zbq, s))
        return fail(h->ctx, RZ_ERR_HIP, "potential patch solve launch failed");
      launch_expand_grad<T>(q->L, q->P, X.coefq, X.Aq, X.lamq, X.vq, X.zbq, X.vy, T(1), T(0), (T *)nullptr, s);
    } else {
      launch_edge_solve<T>(h->ped, X.pfac, X.vq, X.pzb, s);
      launch_list_gather<T>(h->npg, h->pg_rows, h->pg_ptr, h->pg_pos, X.pzb, (const T *)nullptr, X.vy, T(1), s);
    }
    launch_csr<T, T, T>(h->nGam, h->gam, h->d_ptr, h->d_col, X.dv, X.vy, z, 1, s);
  }
  {
    Timed t(h, RZ_K_EXPAND);
    launch_vc_expand<T>(h->V, *X.vc, z, s);
    launch_list_copy<T>(h->nDir, h->dlist, r, z, s);
  }
  return RZ_OK;
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
  if (h->space != RZ_GRAD) {  // b - A x fused into the apply's stores
    Timed t(h, RZ_K_APPLY);
    if (launch_apply_vec<double>(h->V, h->coef64, h->B64, h->D64, x, out, h->eb64, h->ctx->stream, b))
      return fail(h->ctx, RZ_ERR_ARG, "unsupported degree");
    return RZ_OK;
  }
  if (h->quad) {  // trilinear cells: the same fusion in the cell kernel and the gather
    Timed t(h, RZ_K_APPLY);
    launch_apply_quad_cells<double>(h->L, h->Q64, x, out, h->eb64, h->ctx->stream, b);
    launch_apply_gather<double>(h->L, x, h->eb64, out, h->ctx->stream, b);
    return RZ_OK;
  }
  rz_status e = do_apply64(h, x, h->vaz);
  if (e) return e;
  v_sub(h, b, h->vaz, out);
  return RZ_OK;
}

// z = scale * M r; with acc: acc += w * M r (z then holds only the plane values)
const PdSolve<double> &pd_solve(const rz_problem *h, double *) { return h->pds64; }
const PdSolve<float> &pd_solve(const rz_problem *h, float *) { return h->pds32; }

// relaxation steps 1 and 4 of the H(grad) path: the separable weights, or the
// paper's auxiliary (per-point data)
template <typename T>
void condense_any(rz_problem *h, const T *coef, const T *A, const T *lam, const T *r, T *rt) {
  if (h->pd) launch_condense_pd<T>(h->L, pd_solve(h, (T *)nullptr), r, rt, h->ctx->stream);
  else launch_condense_grad<T>(h->L, coef, A, lam, r, rt, h->ctx->stream);
}
template <typename T>
void expand_any(rz_problem *h, const T *coef, const T *A, const T *lam, const T *r, const T *zb, T *z, T scale, T w,
                T *acc) {
  hipStream_t s = h->ctx->stream;
  if (h->pd) {
    launch_expand_plane_grad<T>(h->L, r, zb, z, scale, w, acc, s);
    launch_expand_interior_pd<T>(h->L, pd_solve(h, (T *)nullptr), r, z, scale, w, acc, s);
  } else {
    launch_expand_grad<T>(h->L, h->P, coef, A, lam, r, zb, z, scale, w, acc, s);
  }
}

// The vertex-patch solves of the H(grad) relaxation: incomplete factors through the
// compiled pass schedule, or the exact factors (RZ_PATCH_CHOLESKY) as dense W = L^{-1}
const double *chol_w(rz_problem *h, const double *) { return h->cw64; }
const float *chol_w(rz_problem *h, const float *) { return h->cw32; }

template <typename T>
rz_status patch_solve_any(rz_problem *h, const T *f, const T *rt, T *zb) {
  if (h->cw64) {
    launch_patch_chol_solve<T>(h->L, h->P, chol_w(h, (const T *)nullptr), rt, zb, h->ctx->stream);
    return RZ_OK;
  }
  if (launch_patch_solve<T>(h->L, h->PE, f, rt, zb, h->ctx->stream))
    return fail(h->ctx, RZ_ERR_HIP, "patch solve launch failed");
  return RZ_OK;
}

double *full_zb(rz_problem *h, double *) { return h->fzb64; }
float *full_zb(rz_problem *h, float *) { return h->fzb32; }

// The relaxation with full vertex stars (no static condensation): the star solves on
// r, then their sum at every point
template <typename T>
void relax_full(rz_problem *h, const T *r, T *z, T scale, T w, T *acc) {
  Timed t(h, RZ_K_PATCH);
  T *zb = full_zb(h, (T *)nullptr);
  launch_patch_chol_solve<T>(h->L, h->PF, chol_w(h, (const T *)nullptr), r, zb, h->ctx->stream);
  launch_full_star_sum<T>(h->L, h->nrf, zb, r, z, scale, w, acc, h->ctx->stream);
}

template <typename T>
rz_status relax_steps(rz_problem *h, const T *coef, const T *A, const T *lam, const T *f, T *rt, T *zb,
                      const T *r, T *z, T scale = T(1), T w = T(0), T *acc = nullptr) {
  hipStream_t s = h->ctx->stream;
  if (h->nrf) {
    relax_full<T>(h, r, z, scale, w, acc);
    return RZ_OK;
  }
  {
    Timed t(h, RZ_K_CONDENSE);
    condense_any<T>(h, coef, A, lam, r, rt);
  }
  {
    Timed t(h, RZ_K_PATCH);
    if (rz_status e = patch_solve_any<T>(h, f, rt, zb)) return e;
  }
  {
    Timed t(h, RZ_K_EXPAND);
    expand_any<T>(h, coef, A, lam, r, zb, z, scale, w, acc);
  }
  return RZ_OK;
}

rz_status do_relax64(rz_problem *h, const double *r, double *z, double scale = 1.0, double w = 0.0,
                     double *acc = nullptr) {
  if (h->space != RZ_GRAD) {
    if (rz_status e = relax_vec<double>(h, vec_ptrs64(h), r, z)) return e;
    if (acc) launch_axpy(w, z, acc, h->ndofs, h->ctx->stream);
    else if (scale != 1.0) launch_scale_copy(scale, z, z, h->ndofs, h->ctx->stream);
    return RZ_OK;
  }
  return relax_steps<double>(h, h->coef64, h->A64, h->lam64, h->f64, h->rt64, h->zb64, r, z, scale, w, acc);
}

rz_status do_relax32(rz_problem *h, const float *r, float *z, float scale = 1.0f, float w = 0.0f,
                     float *acc = nullptr) {
  if (h->space != RZ_GRAD) {
    if (rz_status e = relax_vec<float>(h, vec_ptrs32(h), r, z)) return e;
    if (acc) launch_axpy_f(w, z, acc, h->ndofs, h->ctx->stream);
    else if (scale != 1.0f) launch_scale_copy_f(scale, z, z, h->ndofs, h->ctx->stream);
    return RZ_OK;
  }
  return relax_steps<float>(h, h->coef32, h->A32, h->lam32, h->f32, h->rt32, h->zb32, r, z, scale, w, acc);
}

// fine relaxation on FP64 vectors in the precision of the problem's protocol
// (FP32 relaxation for the mixed and defect-correction protocols):
// z = scale * M r, or with acc: acc += w * M r (z is then scratch)
rz_status do_relax_prec(rz_problem *h, const double *r, double *z, double scale = 1.0, double w = 0.0,
                        double *acc = nullptr);
rz_status do_relax_prec(rz_problem *h, const double *r, double *z, double scale, double w, double *acc) {
  if (h->opts.precision != RZ_PREC_F64) {
    launch_cast_d2f(r, h->r32, h->ndofs, h->ctx->stream);
    if (rz_status e = do_relax32(h, h->r32, h->z32)) return e;
    if (acc) launch_f2d_axpy(w, h->z32, acc, h->ndofs, h->ctx->stream);
    else launch_f2d_scale(scale, h->z32, z, h->ndofs, h->ctx->stream);
    return RZ_OK;
  }
  return do_relax64(h, r, z, scale, w, acc);
}

// The cooperative launch of the Q_1 coarse solve on the gathered right-hand side.
int coarse_coop(rz_problem *h, bool f32) {
  const int m = h->cm, nb = h->cmz;
  hipStream_t s = h->ctx->stream;
  return f32 && h->cW32
             ? launch_coarse_solve_f(m, nb, h->cq, h->cW32, h->cM32, h->cN32, h->cr, h->cu, h->cv, h->cx, h->status, s)
             : launch_coarse_solve(m, nb, h->cq, h->cW, h->cM, h->cN, h->cr, h->cu, h->cv, h->cx, h->status, s);
}

void hmg_cycle(rz_problem *h, const double *b0, double *o0);
rz_status setup_ph_full(rz_problem *h, const std::vector<double> &coefe);

// Coarse solve; f32 selects the FP32 copies of the dense blocks (V-cycles of the
// mixed protocols), otherwise FP64 throughout.
rz_status do_coarse(rz_problem *h, const double *rcv, double *xcv, bool f32 = false) {
  Timed tm(h, RZ_K_COARSE);
  hipStream_t s = h->ctx->stream;
  const int m = h->cm, nb = h->cmz;
  launch_coarse_gather(m * nb, h->cbx0, h->cby0, h->cbz0, h->cmx, h->cmy, h->cNX, h->cNY, rcv, h->cr, h->cv, h->cx,
                       s);
  if (h->hmg_on) {
    hmg_cycle(h, h->cr, h->cx);  // ordinary launches: captured with the rest of the iteration
  } else if (h->cap) {
    // capturing a PCG iteration: the cooperative launch stays outside the graphs, so
    // the segment closes here and the next one starts; the replay runs the solve
    // between the two segments
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(s, &g) != hipSuccess || !g) h->cap_bad = true;
    else h->cap->push_back(g);
    if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) {
      h->cap_bad = true;
      return fail(h->ctx, RZ_ERR_HIP, "capture of the PCG iteration failed at the coarse solve");
    }
  } else if (coarse_coop(h, f32)) {
    return fail(h->ctx, RZ_ERR_HIP, "cooperative launch of the coarse solve failed");
  }
  launch_coarse_scatter((int)h->ncoarse, h->cbx0, h->cby0, h->cbz0, h->cmx, h->cmy, h->cmz, h->cNX, h->cNY,
                        h->cx, xcv, s);
  return RZ_OK;
}

// coarse correction of the H(curl) / H(div) cycle: z += P A_0^{-1} P^T r1 (FP64
// coarse vectors; the dense inverse in FP32 for the mixed protocols)
template <typename T>
void coarse_correction_vec(rz_problem *h, const double *r1, T *z, bool f32) {
  hipStream_t s = h->ctx->stream;
  if (h->ncf == 0) return;
  {
    Timed tm(h, RZ_K_TRANSFER);
    launch_csr_wave<double, double, double>(h->ncf, nullptr, h->pr_ptr, h->pr_col, h->pr_val, r1, h->vcr, 0, s);
  }
  {
    Timed tm(h, RZ_K_COARSE);
    if (h->hmg_on) hmg_cycle(h, h->vcr, h->vcx);
    else if (f32 && h->cinv32) launch_symv<float>(h->ncf, h->cinv32, h->vcr, h->vcx, h->csym, s);
    else launch_symv<double>(h->ncf, h->cinv64, h->vcr, h->vcx, h->csym, s);
  }
  {
    Timed tm(h, RZ_K_TRANSFER);
    launch_csr<double, double, T>(h->npf, h->pp_rows, h->pp_ptr, h->pp_col, h->pp_val, h->vcx, z, 1, s);
  }
}

rz_status do_residual64(rz_problem *h, const double *b, const double *x, double *out);
rz_status do_residual32(rz_problem *h, const float *b, const float *x, float *out);

// hybrid V(1,1) for H(curl) / H(div), FP64 vectors
rz_status do_vcycle_vec(rz_problem *h, const double *r, double *z) {
  const double w = h->omega;
  if (rz_status e = do_relax_prec(h, r, z, w, 0.0, nullptr)) return e;  // z = w M r
  if (rz_status e = do_residual64(h, r, z, h->vr)) return e;            // r1 = r - A z
  coarse_correction_vec<double>(h, h->vr, z, h->opts.precision != RZ_PREC_F64);
  if (rz_status e = do_residual64(h, r, z, h->vr)) return e;            // r2 = r - A z
  if (rz_status e = do_relax_prec(h, h->vr, h->vt, 1.0, w, z)) return e;  // z += w M r2
  dir_copy(h, r, z, h->ctx->stream);
  return RZ_OK;
}

rz_status do_vcycle(rz_problem *h, const double *r, double *z) {
  if (h->space != RZ_GRAD) return do_vcycle_vec(h, r, z);
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

// y = A x on BF16 vectors (H(grad)): matrix-core contractions on trilinear cells or
// sampled coefficients, FP32 line operators with BF16 loads and stores on Cartesian
// cells
rz_status do_apply_bf16(rz_problem *h, const uint16_t *x, uint16_t *y) {
  Timed t(h, RZ_K_APPLY);
  hipStream_t s = h->ctx->stream;
  if (h->quad) {
    if (launch_apply_quad_cells_bf16(h->L, h->Q32, x, y, h->eb32, s))
      return fail(h->ctx, RZ_ERR_ARG, "unsupported degree");
    launch_apply_gather_bf16(h->L, x, h->eb32, y, s);
  } else {
    launch_apply_grad_bf16(h->L, h->coef32, h->t.B.data(), h->t.A.data(), x, y, h->eb32, s);
  }
  return RZ_OK;
}

rz_status do_residual32(rz_problem *h, const float *b, const float *x, float *out) {
  if (h->space == RZ_GRAD && !h->quad) {
    Timed t(h, RZ_K_APPLY);
    launch_apply_grad<float>(h->L, h->coef32, h->t.B.data(), h->t.A.data(), x, b, out, h->eb32, h->ctx->stream);
    return RZ_OK;
  }
  if (h->space != RZ_GRAD) {  // b - A x fused into the apply's stores
    Timed t(h, RZ_K_APPLY);
    if (launch_apply_vec<float>(h->V, h->coef32, h->B32, h->D32, x, out, h->eb32, h->ctx->stream, b))
      return fail(h->ctx, RZ_ERR_ARG, "unsupported degree");
    return RZ_OK;
  }
  if (h->quad) {
    Timed t(h, RZ_K_APPLY);
    launch_apply_quad_cells<float>(h->L, h->Q32, x, out, h->eb32, h->ctx->stream, b);
    launch_apply_gather<float>(h->L, x, h->eb32, out, h->ctx->stream, b);
    return RZ_OK;
  }
  rz_status e = do_apply32(h, x, h->az32);
  if (e) return e;
  launch_sub_f(b, h->az32, out, h->ndofs, h->ctx->stream);
  return RZ_OK;
}

// The same cycle on FP32 vectors for H(curl) / H(div) (coarse correction in FP64)
rz_status do_vcycle32_vec(rz_problem *h, const float *r, float *z) {
  hipStream_t s = h->ctx->stream;
  const float w = (float)h->omega;
  if (rz_status e = do_relax32(h, r, z, w)) return e;       // z = w M r
  if (rz_status e = do_residual32(h, r, z, h->vr32)) return e;  // r1 = r - A z
  launch_cast_f2d(h->vr32, h->vr, h->ndofs, s);
  coarse_correction_vec<float>(h, h->vr, z, true);
  if (rz_status e = do_residual32(h, r, z, h->vr32)) return e;  // r2 = r - A z
  if (rz_status e = do_relax32(h, h->vr32, h->t32, 1.0f, w, z)) return e;  // z += w M r2
  dir_copy_f(h, r, z, s);
  return RZ_OK;
}

// The V(1,1) cycle on FP32 vectors (inner solve of the defect-correction
// protocol): FP32 apply and relaxation, the coarse correction in FP64.
rz_status do_vcycle32(rz_problem *h, const float *r, float *z) {
  if (h->space != RZ_GRAD) return do_vcycle32_vec(h, r, z);
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

// ---------------------------------------------------------------------------------------
// Several right-hand sides at once (planar vectors; ids name the right-hand sides,
// which select their per-vector buffers).  The H(grad) vertex-patch solve runs on two
// vectors per launch, each slot's factor loaded once for both
// (launch_patch_solve_multi); the other steps run per vector, in the same order and
// arithmetic as for one vector.
// ---------------------------------------------------------------------------------------
VecRelaxPtrs<double> vec_ptrs(rz_problem *h, double *) { return vec_ptrs64(h); }
VecRelaxPtrs<float> vec_ptrs(rz_problem *h, float *) { return vec_ptrs32(h); }

void axpy_t(double a, const double *x, double *y, int64_t n, hipStream_t s) { launch_axpy(a, x, y, n, s); }
void axpy_t(float a, const float *x, float *y, int64_t n, hipStream_t s) { launch_axpy_f(a, x, y, n, s); }
void scale_copy_t(double a, const double *x, double *y, int64_t n, hipStream_t s) { launch_scale_copy(a, x, y, n, s); }
void scale_copy_t(float a, const float *x, float *y, int64_t n, hipStream_t s) { launch_scale_copy_f(a, x, y, n, s); }

// z_j = scale M r_j, or with acc: acc_j += w M r_j (z_j is then scratch, and may be
// one buffer for all j); post(j) runs once vector j's result is complete.
template <typename T, typename Post>
rz_status relax_multi(rz_problem *h, int nv, const int *ids, const T *const *r, T *const *z, T scale, T w,
                      T *const *acc, Post post) {
  hipStream_t s = h->ctx->stream;
  if (h->space != RZ_GRAD) {
    for (int j = 0; j < nv; ++j) {
      if (rz_status e = relax_vec<T>(h, vec_ptrs(h, (T *)nullptr), r[j], z[j])) return e;
      if (acc) axpy_t(w, z[j], acc[j], h->ndofs, s);
      else if (scale != T(1)) scale_copy_t(scale, z[j], z[j], h->ndofs, s);
      post(j);
    }
    return RZ_OK;
  }
  if (h->nrf) {
    for (int j = 0; j < nv; ++j) {
      relax_full<T>(h, r[j], z[j], scale, w, acc ? acc[j] : nullptr);
      post(j);
    }
    return RZ_OK;
  }
  constexpr bool f64 = sizeof(T) == 8;
  const T *coef, *A, *lam, *f;
  if constexpr (f64) {
    coef = h->coef64, A = h->A64, lam = h->lam64, f = h->f64;
  } else {
    coef = h->coef32, A = h->A32, lam = h->lam32, f = h->f32;
  }
  std::vector<T *> rt(nv), zb(nv);
  for (int j = 0; j < nv; ++j) {
    const RhsBufs B = rhs_bufs(h, ids[j]);
    if constexpr (f64) {
      rt[j] = B.rt64, zb[j] = B.zb64;
    } else {
      rt[j] = B.rt32, zb[j] = B.zb32;
    }
  }
  {
    Timed t(h, RZ_K_CONDENSE);
    for (int j = 0; j < nv; ++j) condense_any<T>(h, coef, A, lam, r[j], rt[j]);
  }
  {
    Timed t(h, RZ_K_PATCH);
    if (h->cw64) {
      for (int j = 0; j < nv; ++j)
        if (rz_status e = patch_solve_any<T>(h, f, rt[j], zb[j])) return e;
    } else if (launch_patch_solve_multi<T>(h->L, h->PE, f, nv, rt.data(), zb.data(), s)) {
      return fail(h->ctx, RZ_ERR_HIP, "patch solve launch failed");
    }
  }
  {
    Timed t(h, RZ_K_EXPAND);
    for (int j = 0; j < nv; ++j) {
      expand_any<T>(h, coef, A, lam, r[j], zb[j], z[j], scale, w, acc ? acc[j] : nullptr);
      post(j);
    }
  }
  return RZ_OK;
}

// relax_multi on FP64 vectors in the precision of the problem's protocol (as
// do_relax_prec): z_j = scale M r_j, or acc_j += w M r_j
rz_status relax_prec_multi(rz_problem *h, int nv, const int *ids, const double *const *r, double *const *z,
                           double scale, double w, double *const *acc) {
  hipStream_t s = h->ctx->stream;
  const int64_t n = h->ndofs;
  if (h->opts.precision == RZ_PREC_F64) return relax_multi<double>(h, nv, ids, r, z, scale, w, acc, [](int) {});
  std::vector<const float *> r32(nv);
  std::vector<float *> z32(nv, h->z32);
  for (int j = 0; j < nv; ++j) {
    float *b = rhs_bufs(h, ids[j]).r32;
    launch_cast_d2f(r[j], b, n, s);
    r32[j] = b;
  }
  return relax_multi<float>(h, nv, ids, r32.data(), z32.data(), 1.0f, 0.0f, nullptr, [&](int j) {
    if (acc) launch_f2d_axpy(w, h->z32, acc[j], n, s);
    else launch_f2d_scale(scale, h->z32, z[j], n, s);
  });
}

// z_j = V(r_j) for nv vectors (the cycle of do_vcycle; FP64 vectors)
rz_status vcycle_multi(rz_problem *h, int nv, const int *ids, const double *const *r, double *const *z) {
  if (h->space != RZ_GRAD) {
    for (int j = 0; j < nv; ++j)
      if (rz_status e = do_vcycle_vec(h, r[j], z[j])) return e;
    return RZ_OK;
  }
  hipStream_t s = h->ctx->stream;
  const double w = h->omega;
  const bool f32c = h->opts.precision != RZ_PREC_F64;
  if (rz_status e = relax_prec_multi(h, nv, ids, r, z, w, 0.0, nullptr)) return e;  // z = w M r
  std::vector<double *> vr(nv), vt(nv, h->vt);
  for (int j = 0; j < nv; ++j) {
    vr[j] = rhs_bufs(h, ids[j]).vr;
    do_residual64(h, r[j], z[j], vr[j]);  // r1 = r - A z
    {
      Timed tm(h, RZ_K_TRANSFER);
      launch_restrict_grad(h->L, h->E64, vr[j], h->rc, h->rt1, h->rt2, s);
    }
    if (rz_status e = do_coarse(h, h->rc, h->xc, f32c)) return e;
    if (h->T2_64) {  // z += P xc and r2 = r1 - A P xc in one pass
      Timed tm(h, RZ_K_TRANSFER);
      launch_prolong_residual_grad(h->L, h->E64, h->T2_64, h->coef64, h->xc, z[j], vr[j], s);
    } else {
      {
        Timed tm(h, RZ_K_TRANSFER);
        launch_prolong_add_grad(h->L, h->E64, h->xc, z[j], s);
      }
      do_residual64(h, r[j], z[j], vr[j]);  // r2 = r - A z
    }
  }
  if (rz_status e = relax_prec_multi(h, nv, ids, vr.data(), vt.data(), 1.0, w, z)) return e;  // z += w M r2
  for (int j = 0; j < nv; ++j) launch_dirichlet_copy(h->L, r[j], z[j], s);
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
  dir_copy(h, nullptr, h->kr, s);
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
      dir_copy(h, nullptr, h->kr, s);
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
    info->iters_natural = -1;
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

// Autotuner of the streaming vertex-patch solve (the degrees and precisions whose
// factor does not fit the registers): for each candidate number of resident
// wavefronts per CU that gives a distinct block shape, one warm-up and three timed
// launches on the problem's own factors (right-hand side zero: the work does not
// depend on its values), and the fastest is kept in the problem's patch data.  The
// block shape does not change the arithmetic of a patch (one wavefront per slot), so
// results are the same for every choice.
template <typename T>
rz_status autotune_patch_solve(rz_problem *h, const T *f, T *rt, T *zb, int which) {
  hipStream_t s = h->ctx->stream;
  static const int kCaps[] = {4, 8, 12, 16, 20, 24, 32, 40};
  std::vector<std::pair<int, int>> seen;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCALL(h, hipEventCreate(&e0));
  HIPCALL(h, hipEventCreate(&e1));
  struct Ev {
    hipEvent_t &a, &b;
    ~Ev() {
      if (a) hipEventDestroy(a);
      if (b) hipEventDestroy(b);
    }
  } guard{e0, e1};
  if (sizeof(T) == 8) launch_fill(reinterpret_cast<double *>(rt), 0.0, h->ndofs, s);
  else launch_fill_f(reinterpret_cast<float *>(rt), 0.0f, h->ndofs, s);
  h->tune[which].clear();
  double best = 0;
  int best_cap = 0;
  for (int cap : kCaps) {
    int w = 0, b = 0;
    if (!patch_solve_stream_shape(h->PE, sizeof(T), cap, w, b)) continue;
    bool dup = false;
    for (auto &q : seen) dup |= q.first == w && q.second == b;
    if (dup) continue;
    seen.push_back({w, b});
    h->PE.cap[which] = cap;
    if (launch_patch_solve<T>(h->L, h->PE, f, rt, zb, s)) return fail(h->ctx, RZ_ERR_HIP, "patch solve launch failed");
    HIPCALL(h, hipEventRecord(e0, s));
    for (int k = 0; k < 3; ++k) launch_patch_solve<T>(h->L, h->PE, f, rt, zb, s);
    HIPCALL(h, hipEventRecord(e1, s));
    HIPCALL(h, hipEventSynchronize(e1));
    float ms = 0;
    HIPCALL(h, hipEventElapsedTime(&ms, e0, e1));
    const double t = ms / 3.0;
    h->tune[which].push_back({cap, t});
    if (best_cap == 0 || t < best) {
      best = t;
      best_cap = cap;
    }
  }
  h->PE.cap[which] = best_cap;
  return RZ_OK;
}

// rz_opts.lanczos_steps (default 10, 40 for RZ_DECOMP_SC_VERTEX) preconditioned CG steps on A x = v0 with M = the
// FP64 fine relaxation (for every precision protocol, so the damping does not depend
// on it); Lanczos estimate
rz_status estimate_lambda(rz_problem *h, double *lam_out) {
  hipStream_t s = h->ctx->stream;
  const int64_t n = h->ndofs;
  std::vector<double> v0(n);
  uint64_t st = h->opts.lanczos_seed;
  for (int64_t g = 0; g < n; ++g) {
    double u = (double)(splitmix_next(st) >> 11) * 0x1.0p-53;
    bool d;
    if (h->space == RZ_GRAD) {
      int X = g % h->Nx, Y = (g / h->Nx) % h->Ny, Z = g / ((int64_t)h->Nx * h->Ny);
      d = lat_dirichlet_h(h, X, Y, Z);
    } else {
      d = h->dmask[g] != 0;
    }
    v0[g] = d ? 0.0 : 2.0 * u - 1.0;
  }
  HIPCALL(h, hipMemcpyAsync(h->kr, v0.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
  if (rz_status e = do_relax64(h, h->kr, h->kz)) return e;
  HIPCALL(h, hipMemcpyAsync(h->kp, h->kz, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  double rz_;
  {
    const double *xs[1] = {h->kr}, *ys[1] = {h->kz};
    rz_status e = dots_host(h, 1, xs, ys, &rz_);
    if (e) return e;
  }
  std::vector<double> al, be;
  // default: 10 steps; 40 for the condensed vector vertex stars, whose spectrum has an
  // outlying top that 10 steps underestimate by about 30 % at small beta
  const int steps = h->opts.lanczos_steps > 0 ? h->opts.lanczos_steps
                                              : (h->opts.decomposition == RZ_DECOMP_SC_VERTEX ? 40 : 10);
  for (int it = 0; it < steps; ++it) {
    do_apply64(h, h->kp, h->kAp);
    double pAp;
    const double *xs[1] = {h->kp}, *ys[1] = {h->kAp};
    rz_status e = dots_host(h, 1, xs, ys, &pAp);
    if (e) return e;
    if (!(pAp > 0)) break;
    double a = rz_ / pAp;
    v_axpy(h, -a, h->kAp, h->kr);
    if ((e = do_relax64(h, h->kr, h->kz))) return e;
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
// Geometric h-multigrid on the Q_1 space: the level-0 operator is the 27-point
// stencil st of the free box (neighbours outside the box dropped: Dirichlet
// vertices), the hierarchy and its Galerkin operators are built on the host, the
// coarsest level is inverted densely on the device.
constexpr int64_t kHmgMinFree = 512, kHmgMaxCoarsest = 4096;
constexpr double kHmgJacobiC = 1.5;

// Damping of point Jacobi on the SPD matrix M: 1.5 over the largest row sum of
// |D^{-1/2} M D^{-1/2}| (Gershgorin), an upper bound of the spectrum of D^{-1} M, so
// the weighted spectrum stays in (0, 1.5] and the relaxation contracts on any mesh
// and for any positive coefficients.  Also D^{-1} into dinv; false on a non-positive
// diagonal.
bool jacobi_weight(const HostCsr &M, std::vector<double> &dinv, double &w) {
  std::vector<double> d(M.n, 0.0);
  for (int i = 0; i < M.n; ++i)
    for (int k = M.ptr[i]; k < M.ptr[i + 1]; ++k)
      if (M.col[k] == i) d[i] = M.val[k];
  dinv.resize(M.n);
  double g = 0.0;
  for (int i = 0; i < M.n; ++i) {
    if (!(d[i] > 0.0)) return false;
    dinv[i] = 1.0 / d[i];
    double r = 0.0;
    for (int k = M.ptr[i]; k < M.ptr[i + 1]; ++k) r += std::fabs(M.val[k]) / std::sqrt(d[i] * d[M.col[k]]);
    g = std::max(g, r);
  }
  w = kHmgJacobiC / g;
  return true;
}

// Device copies of the hierarchy: operators A[l], interpolations P[l] and
// restrictions R[l] = P[l]^T; for H(curl)/H(div) also the exterior derivative G[l]
// from the potential space and the potential operators Ap[l] = G^T A G (empty for
// H(grad)).  Matrices in ELL form, the coarsest level inverted densely.
rz_status hmg_upload(rz_problem *h, const std::vector<HostCsr> &A, const std::vector<HostCsr> &P,
                     const std::vector<HostCsr> &R, const std::vector<HostCsr> &G, const std::vector<HostCsr> &Ap) {
  hipStream_t s = h->ctx->stream;
  const int L = (int)P.size();
  h->hmg_sizes.clear();
  for (auto &M : A) h->hmg_sizes.push_back(M.n);
  if (A[L].n > kHmgMaxCoarsest)
    return fail(h->ctx, RZ_ERR_ARG,
                "h-multigrid coarse solver: the coarsest level (cell counts halved while all even) exceeds 4096 "
                "free DoFs");
  // ELL form: entry k of row i at k * n + i, short rows padded with (min(i, m-1), 0)
  auto ell = [&](const HostCsr &M, int &width, int **dcol, double **dval) -> rz_status {
    width = 1;
    for (int i = 0; i < M.n; ++i) width = std::max(width, M.ptr[i + 1] - M.ptr[i]);
    width = hmg_ell_width(width);
    std::vector<int> cc((size_t)width * M.n);
    std::vector<double> v((size_t)width * M.n, 0.0);
    for (int i = 0; i < M.n; ++i)
      for (int k = 0; k < width; ++k) {
        const int q = M.ptr[i] + k;
        const bool in = q < M.ptr[i + 1];
        cc[(size_t)k * M.n + i] = in ? M.col[q] : std::min(i, M.m - 1);
        v[(size_t)k * M.n + i] = in ? M.val[q] : 0.0;
      }
    rz_status r;
    if ((r = upload(h, dcol, cc)) || (r = upload(h, dval, v))) return r;
    return RZ_OK;
  };
  rz_status e;
  h->hmg.assign(L, rz_problem::HmgLevel());
  for (int l = 0; l < L; ++l) {
    auto &V = h->hmg[l];
    V.n = A[l].n;
    V.nnext = A[l + 1].n;
    std::vector<double> dinv;
    if (!jacobi_weight(A[l], dinv, V.w)) return fail(h->ctx, RZ_ERR_SINGULAR, "h-multigrid: non-positive diagonal");
    if ((e = ell(A[l], V.aw, &V.a_col, &V.a_val)) || (e = ell(P[l], V.pw, &V.p_col, &V.p_val)) ||
        (e = ell(R[l], V.rw, &V.r_col, &V.r_val)) || (e = upload(h, &V.dinv, dinv)) || (e = dalloc(h, &V.t, V.n)) ||
        (e = dalloc(h, &V.x, V.n)))
      return e;
    if (l > 0 && ((e = dalloc(h, &V.b, V.n)) || (e = dalloc(h, &V.o, V.n)))) return e;
    if (!G.empty()) {
      V.np = G[l].m;
      std::vector<double> dpinv;
      if (!jacobi_weight(Ap[l], dpinv, V.wp))
        return fail(h->ctx, RZ_ERR_SINGULAR, "h-multigrid: non-positive diagonal of the potential operator");
      const HostCsr GT = csr_transpose(G[l]);
      if ((e = ell(G[l], V.gw, &V.g_col, &V.g_val)) || (e = ell(GT, V.gtw, &V.gt_col, &V.gt_val)) ||
          (e = upload(h, &V.dpinv, dpinv)) || (e = dalloc(h, &V.x2, V.n)) || (e = dalloc(h, &V.y, std::max(V.np, 1))))
        return e;
    }
  }
  const int nc = A[L].n;
  h->hmg_nc = nc;
  std::vector<double> D((size_t)nc * nc, 0.0);
  for (int i = 0; i < nc; ++i)
    for (int k = A[L].ptr[i]; k < A[L].ptr[i + 1]; ++k) D[(size_t)i * nc + A[L].col[k]] = A[L].val[k];
  if ((e = upload(h, &h->hmg_cinv, D))) return e;
  double *tmp = nullptr;
  if (hipMalloc(&tmp, sizeof(double) * (size_t)nc * nc) != hipSuccess)
    return fail(h->ctx, RZ_ERR_OOM, "h-multigrid coarsest inverse workspace");
  launch_sweep_inverse(nc, h->hmg_cinv, tmp, h->status, s);
  const hipError_t se = hipStreamSynchronize(s);
  hipFree(tmp);
  if (se != hipSuccess) return fail(h->ctx, RZ_ERR_HIP, "h-multigrid coarsest inverse failed");
  int stv = 0;
  HIPCALL(h, hipMemcpy(&stv, h->status, sizeof(int), hipMemcpyDeviceToHost));
  if (stv) return fail(h->ctx, RZ_ERR_SINGULAR, "h-multigrid coarsest level: non-positive pivot");
  const size_t nt = ((size_t)nc + 63) / 64;
  if ((e = dalloc(h, &h->hmg_work, nt * nt * 64))) return e;
  if (L > 0 && ((e = dalloc(h, &h->hmg_cb, nc)) || (e = dalloc(h, &h->hmg_co, nc)))) return e;
  h->hmg_on = true;
  return RZ_OK;
}

// H(grad): the level-0 operator is the 27-point stencil st of the free box
// (neighbours outside the box dropped: Dirichlet vertices), the hierarchy of
// hmg_hierarchy.
rz_status setup_hmg(rz_problem *h, const std::vector<double> &st) {
  const int mx = h->cmx, my = h->cmy, mz = h->cmz;
  HostCsr A0;
  A0.n = A0.m = mx * my * mz;
  A0.ptr.assign(A0.n + 1, 0);
  for (int z = 0; z < mz; ++z)
    for (int y = 0; y < my; ++y)
      for (int x = 0; x < mx; ++x) {
        const int64_t row = x + (int64_t)mx * (y + (int64_t)my * z);
        for (int off = 0; off < 27; ++off) {  // ascending column order: z, then y, then x offset
          const int X = x + off % 3 - 1, Y = y + (off / 3) % 3 - 1, Z = z + off / 9 - 1;
          if (X < 0 || X >= mx || Y < 0 || Y >= my || Z < 0 || Z >= mz) continue;
          A0.col.push_back(X + mx * (Y + my * Z));
          A0.val.push_back(st[row * 27 + off]);
        }
        A0.ptr[row + 1] = (int)A0.col.size();
      }
  const int n[3] = {h->nx, h->ny, h->nz};
  std::vector<HostCsr> A, P, R;
  hmg_hierarchy(std::move(A0), n, h->dir, kHmgMinFree, A, P, R);
  return hmg_upload(h, A, P, R, {}, {});
}

// One V(1,1) cycle of the h-multigrid from a zero guess on the free-DoF vectors,
// o0 = B b0.  H(grad), per level: the residual after the pre-relaxation, its
// restriction; after the coarser level, the pre-relaxed iterate plus the
// interpolated correction, and the post-relaxation.  H(curl)/H(div) (Hiptmair): the
// pre-relaxation is Jacobi on A, then Jacobi on the potential operator through G;
// the post-relaxation the same two steps in the reverse order.
void hmg_cycle(rz_problem *h, const double *b0, double *o0) {
  hipStream_t s = h->ctx->stream;
  const int L = (int)h->hmg.size();
  auto bin = [&](int l) -> const double * { return l == 0 ? b0 : l < L ? h->hmg[l].b : h->hmg_cb; };
  auto bout = [&](int l) -> double * { return l == 0 ? o0 : l < L ? h->hmg[l].o : h->hmg_co; };
  for (int l = 0; l < L; ++l) {
    auto &V = h->hmg[l];
    const double *b = bin(l);
    launch_hmg_row(HMG_RES0, V.n, V.aw, V.a_col, V.a_val, nullptr, b, V.dinv, V.w, V.t, s);  // t = b - A x0
    if (V.np) {
      launch_hmg_row(HMG_JPROD, V.np, V.gtw, V.gt_col, V.gt_val, V.t, nullptr, V.dpinv, V.wp, V.y, s);
      launch_hmg_row(HMG_PROL, V.n, V.gw, V.g_col, V.g_val, V.y, b, V.dinv, V.w, V.x, s);  // x1 = x0 + G y
      launch_hmg_row(HMG_RES, V.n, V.aw, V.a_col, V.a_val, V.x, b, nullptr, 0.0, V.t, s);  // t = b - A x1
    }
    launch_hmg_row(HMG_PROD, V.nnext, V.rw, V.r_col, V.r_val, V.t, nullptr, nullptr, 0.0,
                   const_cast<double *>(bin(l + 1)), s);
  }
  launch_symv<double>(h->hmg_nc, h->hmg_cinv, bin(L), bout(L), h->hmg_work, s);
  for (int l = L - 1; l >= 0; --l) {
    auto &V = h->hmg[l];
    const double *b = bin(l);
    if (V.np) {
      launch_hmg_row(HMG_ADD, V.n, V.pw, V.p_col, V.p_val, bout(l + 1), V.x, nullptr, 0.0, V.x2, s);  // x2 = x1 + P xc
      launch_hmg_row(HMG_RES, V.n, V.aw, V.a_col, V.a_val, V.x2, b, nullptr, 0.0, V.t, s);
      launch_hmg_row(HMG_JPROD, V.np, V.gtw, V.gt_col, V.gt_val, V.t, nullptr, V.dpinv, V.wp, V.y, s);
      launch_hmg_row(HMG_ADD, V.n, V.gw, V.g_col, V.g_val, V.y, V.x2, nullptr, 0.0, V.x, s);  // x3 = x2 + G y
    } else {
      launch_hmg_row(HMG_PROL, V.n, V.pw, V.p_col, V.p_val, bout(l + 1), b, V.dinv, V.w, V.x, s);
    }
    launch_hmg_row(HMG_POST, V.n, V.aw, V.a_col, V.a_val, V.x, b, V.dinv, V.w, bout(l), s);
  }
}

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
  rz_status e;
  if (h->opts.coarse == RZ_COARSE_HMG) {
    if ((e = dalloc(h, &h->cr, nfree)) || (e = dalloc(h, &h->cv, nfree)) || (e = dalloc(h, &h->cx, nfree))) return e;
    return setup_hmg(h, st);
  }
  if (m > 4096) return fail(h->ctx, RZ_ERR_ARG, "coarse plane too large for the dense-block coarse solver");
  // device blocks
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

void graphs_release(rz_problem *h) {
  for (auto &G : h->ig) {
    for (hipGraphExec_t e : G.seg) hipGraphExecDestroy(e);
    G.seg.clear();
    G.ok = false;
  }
}

void release(rz_problem *h) {
  graphs_release(h);
  if (h->pot) {
    release(h->pot);
    delete h->pot;
    h->pot = nullptr;
  }
  for (void *p : h->allocs) hipFree(p);
  h->allocs.clear();
  free_multi(h);
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

// ---------------------------------------------------------------------------------------
// pieces of the H(grad) setup shared by problems and the internal Q_p potential problem
// of the H(curl) relaxation
// ---------------------------------------------------------------------------------------
namespace {

// symbolic patch pattern, free DoFs, non-empty patches, lattice description
PdDev pd_dev(const rz_problem *h) {
  if (!h->pd) return PdDev{nullptr, nullptr, nullptr, nullptr};
  return PdDev{h->pd_dm, h->pd_da, h->pd_G, h->pd_D64};
}

// The broken diagonals of every cell (host, FP64, cells split over the host's
// threads): (p+1)^3 + 3 p (p+1)^2 values per cell.
bool paper_diagonals_all(rz_problem *h) {
  const int p = h->p, n1 = p + 1;
  const size_t nm = (size_t)n1 * n1 * n1, na = 3 * (size_t)p * n1 * n1;
  h->pd_host_dm.assign(nm * h->ncells, 0.0);
  h->pd_host_da.assign(na * h->ncells, 0.0);
  const PaperDiagTables T(h->t, h->qt);
  const int nvx = h->nx + 1, nvy = h->ny + 1;
  unsigned nt = std::thread::hardware_concurrency();
  nt = std::max(1u, std::min(nt, 32u));
  std::vector<char> ok(nt, 1);
  std::vector<std::thread> pool;
  for (unsigned w = 0; w < nt; ++w)
    pool.emplace_back([&, w] {
      for (int64_t c = w; c < h->ncells; c += nt) {
        const int cx = c % h->nx, cy = (c / h->nx) % h->ny, cz = c / ((int64_t)h->nx * h->ny);
        double corners[24];
        for (int k = 0; k < 8; ++k) {
          const int64_t vid = (cx + (k & 1)) + nvx * ((cy + ((k >> 1) & 1)) + (int64_t)nvy * (cz + (k >> 2)));
          for (int r = 0; r < 3; ++r) corners[3 * k + r] = h->vert[3 * vid + r];
        }
        if (!paper_diagonals(corners, &h->asmp[27 * c], &h->bsmp[27 * c], h->qt, T, &h->pd_host_dm[nm * c],
                             &h->pd_host_da[na * c]))
          ok[w] = 0;
      }
    });
  for (auto &t : pool) t.join();
  for (char o : ok)
    if (!o) return false;
  return true;
}

// Device data of the paper's auxiliary: the per-cell diagonals and 1-D tables (for
// the patch factorisation), and at every cell-interior lattice point t the P_II
// diagonal dm + sum_d lambda_{t_d} da_d and w_d = sqrt(lambda_{t_d}) da_d (for the
// condensation and extension), FP64 and FP32.
rz_status upload_paper_diagonals(rz_problem *h) {
  const int p = h->p, n1 = p + 1;
  const size_t nm = (size_t)n1 * n1 * n1, na = 3 * (size_t)p * n1 * n1, nc = (size_t)p * n1 * n1;
  const int64_t N = h->ndofs;
  std::vector<double> pii(N, 1.0), w[3] = {std::vector<double>(N, 0.0), std::vector<double>(N, 0.0),
                                            std::vector<double>(N, 0.0)};
  for (int64_t c = 0; c < h->ncells; ++c) {
    const int cx = c % h->nx, cy = (c / h->nx) % h->ny, cz = c / ((int64_t)h->nx * h->ny);
    const double *dm = &h->pd_host_dm[nm * c], *da = &h->pd_host_da[na * c];
    for (int k = 1; k < p; ++k)
      for (int j = 1; j < p; ++j)
        for (int i = 1; i < p; ++i) {
          const int64_t g = (int64_t)(cx * p + i) + h->Nx * ((int64_t)(cy * p + j) + (int64_t)h->Ny * (cz * p + k));
          const double dx = da[i + p * (j + n1 * k)], dy = da[nc + i + n1 * (j + p * k)],
                       dz = da[2 * nc + i + n1 * (j + n1 * k)];
          const double li = h->t.lam[i - 1], lj = h->t.lam[j - 1], lk = h->t.lam[k - 1];
          pii[g] = dm[i + n1 * (j + n1 * k)] + li * dx + lj * dy + lk * dz;
          w[0][g] = std::sqrt(li) * dx;
          w[1][g] = std::sqrt(lj) * dy;
          w[2][g] = std::sqrt(lk) * dz;
        }
  }
  rz_status e;
  double *pii64, *w64[3], *D64;
  float *pii32, *w32[3], *D32;
  if ((e = upload(h, &h->pd_dm, h->pd_host_dm)) || (e = upload(h, &h->pd_da, h->pd_host_da)) ||
      (e = upload(h, &h->pd_G, h->t.G)) || (e = upload(h, &D64, h->t.D)) || (e = upload(h, &pii64, pii)) ||
      (e = upload(h, &w64[0], w[0])) || (e = upload(h, &w64[1], w[1])) || (e = upload(h, &w64[2], w[2])) ||
      (e = upload(h, &D32, as_type<float>(h->t.D))) || (e = upload(h, &pii32, as_type<float>(pii))) ||
      (e = upload(h, &w32[0], as_type<float>(w[0]))) || (e = upload(h, &w32[1], as_type<float>(w[1]))) ||
      (e = upload(h, &w32[2], as_type<float>(w[2]))))
    return e;
  h->pd_D64 = D64;
  h->pds64 = PdSolve<double>{pii64, w64[0], w64[1], w64[2], D64};
  h->pds32 = PdSolve<float>{pii32, w32[0], w32[1], w32[2], D32};
  h->pd_host_dm = std::vector<double>();
  h->pd_host_da = std::vector<double>();
  return RZ_OK;
}

void grad_symbolic(rz_problem *h) {
  const int p = h->p;
  build_patch_symbolic(p, h->ps);
  h->erow.resize(h->ps.nnz);
  for (int r = 0; r < h->ps.nrows; ++r)
    for (int k = h->ps.rowptr[r]; k < h->ps.rowptr[r + 1]; ++k) h->erow[k] = r;
  int64_t nd = 0;
  for (int64_t g = 0; g < h->ndofs; ++g) {
    int X = g % h->Nx, Y = (g / h->Nx) % h->Ny, Z = g / ((int64_t)h->Nx * h->Ny);
    nd += lat_dirichlet_h(h, X, Y, Z);
  }
  h->nfree = h->ndofs - nd;
  h->patch_vids.clear();
  for (int64_t v = 0; v < h->nvert; ++v) {
    int G[3];
    for (int k = 0; k < h->ps.nrows; ++k)
      if (patch_row_present(h, v, k, G)) {
        h->patch_vids.push_back(v);
        break;
      }
  }
  h->L = LatDev{p, h->nx, h->ny, h->nz, h->Nx, h->Ny, h->Nz, h->dir};
}

// status word, weights and 1-D tables on the device, the patch schedule, and the IC
// factors of every vertex patch (FP64 pivots, FP32 copy)
rz_status grad_patch_device(rz_problem *h) {
  rz_ctx *ctx = h->ctx;
  hipStream_t s = ctx->stream;
  rz_status e;
  const int p = h->p, n1 = p + 1;
  std::vector<double> lamf(n1, 0.0);
  for (int i = 1; i < p; ++i) lamf[i] = h->t.lam[i - 1];
  std::vector<float> c32(h->coef.begin(), h->coef.end()), B32(h->t.B.begin(), h->t.B.end()),
      A32(h->t.A.begin(), h->t.A.end()), l32(lamf.begin(), lamf.end());
  if ((e = dalloc(h, &h->status, 1))) return e;
  HIPCALL(h, hipMemsetAsync(h->status, 0, sizeof(int), s));
  if ((e = upload(h, &h->coef64, h->coef)) || (e = upload(h, &h->B64, h->t.B)) || (e = upload(h, &h->A64, h->t.A)) ||
      (e = upload(h, &h->lam64, lamf)) || (e = upload(h, &h->coef32, c32)) || (e = upload(h, &h->B32, B32)) ||
      (e = upload(h, &h->A32, A32)) || (e = upload(h, &h->lam32, l32)))
    return e;
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
  if ((e = upload(h, &dsym, sym))) return e;
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
    return fail(ctx, RZ_ERR_ARG, "patch schedule does not fit the LDS");
  const size_t nf = (size_t)h->nvert * ps.stride, nzb = (size_t)h->nvert * ps.nrows;
  if ((e = dalloc(h, &h->f64, nf)) || (e = dalloc(h, &h->f32, nf)) || (e = dalloc(h, &h->zb64, nzb)) ||
      (e = dalloc(h, &h->zb32, nzb)))
    return e;
  // the workspace of the vertex patches: keep rows of empty slots well defined
  launch_fill(h->zb64, 0.0, (int64_t)nzb, s);
  launch_fill_f(h->zb32, 0.0f, (int64_t)nzb, s);
  // ELL padding of the factors must read as zero
  HIPCALL(h, hipMemsetAsync(h->f64, 0, nf * sizeof(double), s));
  HIPCALL(h, hipMemsetAsync(h->f32, 0, nf * sizeof(float), s));
  launch_patch_factor(h->L, h->P, h->coef64, h->B64, h->A64, h->lam64, pd_dev(h), h->f64, h->f32, h->status, s);
  if (hipStreamSynchronize(s) != hipSuccess) return fail(ctx, RZ_ERR_HIP, "patch factorisation failed");
  int stv = 0;
  HIPCALL(h, hipMemcpy(&stv, h->status, sizeof(int), hipMemcpyDeviceToHost));
  if (stv) {
    char msg[128];
    std::snprintf(msg, sizeof msg, "incomplete Cholesky breakdown in vertex patch %d", stv - 1);
    return fail(ctx, RZ_ERR_BREAKDOWN, msg);
  }
  return RZ_OK;
}

// Dense lower factor of a symmetric matrix A (n x n, row-major; overwritten by L),
// row-oriented: for each row i the entries j < i in ascending order, then the pivot;
// with pat (n x n flags) the entries off the pattern are dropped (incomplete
// Cholesky on the pattern), without it the factor is exact.  False on a pivot <= 0.
bool dense_factor(std::vector<double> &A, int n, const std::vector<unsigned char> *pat) {
  for (int i = 0; i < n; ++i) {
    double *ri = &A[(size_t)i * n];
    for (int j = 0; j < i; ++j) {
      if (pat && !(*pat)[(size_t)i * n + j]) {
        ri[j] = 0.0;
        continue;
      }
      const double *rj = &A[(size_t)j * n];
      double v = ri[j];
      for (int k = 0; k < j; ++k) v -= ri[k] * rj[k];
      ri[j] = v / rj[j];
    }
    double d = ri[i];
    for (int k = 0; k < i; ++k) d -= ri[k] * ri[k];
    if (!(d > 0.0)) return false;
    ri[i] = std::sqrt(d);
    for (int j = i + 1; j < n; ++j) ri[j] = 0.0;
  }
  return true;
}

// W = L^{-1} of a dense lower L (n x n, row-major), column by column:
// W[c][c] = 1 / L[c][c], W[i][c] = -(sum_{c<=k<i} L[i][k] W[k][c]) / L[i][i]; written
// packed by rows (row i at i (i + 1) / 2) to out.
void dense_inverse_packed(const std::vector<double> &L, int n, std::vector<double> &Wc, double *out) {
  Wc.assign((size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c) {
    Wc[(size_t)c * n + c] = 1.0 / L[(size_t)c * n + c];
    for (int i = c + 1; i < n; ++i) {
      double v = 0.0;
      const double *ri = &L[(size_t)i * n];
      for (int k = c; k < i; ++k) v += ri[k] * Wc[(size_t)k * n + c];
      Wc[(size_t)i * n + c] = -v / ri[i];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) out[(size_t)i * (i + 1) / 2 + j] = Wc[(size_t)i * n + j];
}

// Per slot on host threads: fill(slot, A) builds the dense patch matrix, then the
// exact (pat == nullptr) or incomplete factor and W = L^{-1}, packed by rows, into W;
// the first slot with a pivot <= 0, or -1.
template <typename Fill>
long factor_slots(size_t nslot, int n, const std::vector<unsigned char> *(*patf)(size_t, const std::vector<double> &,
                                                                                 std::vector<unsigned char> &),
                  Fill fill, std::vector<double> &W) {
  const size_t tri = (size_t)n * (n + 1) / 2;
  W.assign(nslot * tri, 0.0);
  std::atomic<long> bad(-1);
  auto work = [&](size_t s0, size_t s1) {
    std::vector<double> A((size_t)n * n), Wc;
    std::vector<unsigned char> pat;
    for (size_t sl = s0; sl < s1; ++sl) {
      std::fill(A.begin(), A.end(), 0.0);
      fill(sl, A);
      const std::vector<unsigned char> *pp = patf ? patf(sl, A, pat) : nullptr;
      if (!dense_factor(A, n, pp)) {
        long exp = -1;
        bad.compare_exchange_strong(exp, (long)sl);
        continue;
      }
      dense_inverse_packed(A, n, Wc, W.data() + sl * tri);
    }
  };
  const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t) th.emplace_back(work, nslot * t / nt, nslot * (t + 1) / nt);
  for (auto &t : th) t.join();
  return bad.load();
}

// the pattern of a dense patch matrix: its nonzero entries
const std::vector<unsigned char> *nonzero_pattern(size_t, const std::vector<double> &A,
                                                  std::vector<unsigned char> &pat) {
  pat.resize(A.size());
  for (size_t k = 0; k < A.size(); ++k) pat[k] = A[k] != 0.0;
  return &pat;
}

rz_status upload_patch_inverse(rz_problem *h, const std::vector<double> &W) {
  rz_status e;
  if (!h->cw64 && ((e = dalloc(h, &h->cw64, W.size())) || (e = dalloc(h, &h->cw32, W.size())))) return e;
  HIPCALL(h, hipMemcpyAsync(h->cw64, W.data(), W.size() * sizeof(double), hipMemcpyHostToDevice, h->ctx->stream));
  launch_cast_d2f(h->cw64, h->cw32, (int64_t)W.size(), h->ctx->stream);
  HIPCALL(h, hipStreamSynchronize(h->ctx->stream));
  return RZ_OK;
}

// Exact Cholesky factors of the statically condensed vertex-star matrices S_v
// (rz_opts.patch_solver = RZ_PATCH_CHOLESKY): S_v assembled on the device on its
// pattern (the setup kernel without its incomplete factorisation), then per slot on
// host threads: S_v dense, S_v = L L^T, W = L^{-1}, packed by rows; W uploaded in FP64
// and FP32; the incomplete factors are formed again so that their export is unchanged.
rz_status setup_patch_cholesky(rz_problem *h) {
  const PatchSymbolic &ps = h->ps;
  const int nr = ps.nrows;
  const size_t tri = (size_t)nr * (nr + 1) / 2, nslot = (size_t)h->nvert;
  if ((double)nslot * tri * 12.0 > 16.0 * (1ull << 30))
    return fail(h->ctx, RZ_ERR_ARG, "RZ_PATCH_CHOLESKY: the dense patch factors would exceed 16 GiB (small meshes only)");
  hipStream_t s = h->ctx->stream;
  const size_t nf = nslot * ps.stride;
  HIPCALL(h, hipMemsetAsync(h->f64, 0, nf * sizeof(double), s));
  launch_patch_factor(h->L, h->P, h->coef64, h->B64, h->A64, h->lam64, pd_dev(h), h->f64, h->f32, h->status, s, 0);
  std::vector<double> fh(nf);
  HIPCALL(h, hipMemcpyAsync(fh.data(), h->f64, nf * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCALL(h, hipStreamSynchronize(s));
  std::vector<double> W;
  const long bad = factor_slots(nslot, nr, nullptr, [&](size_t sl, std::vector<double> &A) {
    const double *f = fh.data() + sl * ps.stride;
    for (int r = 0; r < nr; ++r)
      for (int k = ps.rowptr[r]; k < ps.rowptr[r + 1]; ++k) A[(size_t)r * nr + ps.col[k]] = f[ps.pos1[k]];
    for (int r = 0; r < nr; ++r)  // symmetric: the upper triangle from the lower
      for (int c = 0; c < r; ++c) A[(size_t)c * nr + r] = A[(size_t)r * nr + c];
  }, W);
  if (bad >= 0) {
    char msg[128];
    std::snprintf(msg, sizeof msg, "Cholesky breakdown in vertex patch %ld", bad);
    return fail(h->ctx, RZ_ERR_BREAKDOWN, msg);
  }
  if (rz_status e = upload_patch_inverse(h, W)) return e;
  // the incomplete factors again (their export and the ELL padding as before)
  HIPCALL(h, hipMemsetAsync(h->f64, 0, nf * sizeof(double), s));
  HIPCALL(h, hipMemsetAsync(h->f32, 0, nf * sizeof(float), s));
  launch_patch_factor(h->L, h->P, h->coef64, h->B64, h->A64, h->lam64, pd_dev(h), h->f64, h->f32, h->status, s);
  HIPCALL(h, hipStreamSynchronize(s));
  return RZ_OK;
}

// Full vertex stars (rz_opts.decomposition = RZ_DECOMP_FULL, PAFW without static
// condensation, eq. pafw): every lattice point strictly inside the 8 cells around a
// vertex, rows in the (2p-1)^3 box of offsets with x fastest (points outside the
// domain or on a Dirichlet face are identity rows).  P_v assembled on host threads
// from the separable cell weights and the 1-D tables (P_K(u, w) = s_0 A B B + s_1 B A B
// + s_2 B B A + mu B B B over the cells holding both points), factored exactly or by IC
// on its pattern, W = L^{-1} uploaded.
rz_status setup_full_stars(rz_problem *h) {
  const int p = h->p, q = 2 * p - 1, n1 = p + 1;
  const int nrf = q * q * q;
  const size_t tri = (size_t)nrf * (nrf + 1) / 2, nslot = (size_t)h->nvert;
  if ((double)nslot * tri * 12.0 > 16.0 * (1ull << 30) || (double)nslot * nrf * nrf * (double)nrf > 5e11)
    return fail(h->ctx, RZ_ERR_ARG, "RZ_DECOMP_FULL: the dense full-star factors are for small meshes and degrees");
  std::vector<int> off(3 * (size_t)nrf);
  for (int i = 0; i < nrf; ++i) {
    off[3 * i] = i % q - (p - 1);
    off[3 * i + 1] = (i / q) % q - (p - 1);
    off[3 * i + 2] = i / (q * q) - (p - 1);
  }
  const int nvx = h->nx + 1, nvy = h->ny + 1;
  const int N[3] = {h->nx * p + 1, h->ny * p + 1, h->nz * p + 1}, nc[3] = {h->nx, h->ny, h->nz};
  const std::vector<double> &B = h->t.B, &A = h->t.A;
  auto dir = [&](const int X[3]) {
    for (int d = 0; d < 3; ++d) {
      if (((h->dir >> (2 * d)) & 1u) && X[d] == 0) return true;
      if (((h->dir >> (2 * d + 1)) & 1u) && X[d] == N[d] - 1) return true;
    }
    return false;
  };
  std::vector<double> W;
  const bool ic = h->opts.patch_solver == RZ_PATCH_IC;
  const long bad = factor_slots(nslot, nrf, ic ? nonzero_pattern : nullptr, [&](size_t sl, std::vector<double> &M) {
    const int V[3] = {(int)(sl % nvx), (int)((sl / nvx) % nvy), (int)(sl / ((size_t)nvx * nvy))};
    std::vector<char> live(nrf);
    for (int i = 0; i < nrf; ++i) {
      int X[3];
      bool in = true;
      for (int d = 0; d < 3; ++d) {
        X[d] = V[d] * p + off[3 * i + d];
        in = in && X[d] >= 0 && X[d] < N[d];
      }
      live[i] = in && !dir(X);
    }
    for (int i = 0; i < nrf; ++i) {
      if (!live[i]) {
        M[(size_t)i * nrf + i] = 1.0;
        continue;
      }
      for (int j = 0; j < nrf; ++j) {
        if (!live[j]) continue;
        double v = 0.0;
        for (int cell = 0; cell < 8; ++cell) {
          int cc[3], u[3], w[3];
          bool ok = true;
          for (int d = 0; d < 3; ++d) {
            cc[d] = V[d] - 1 + ((cell >> d) & 1);
            u[d] = V[d] * p + off[3 * i + d] - cc[d] * p;
            w[d] = V[d] * p + off[3 * j + d] - cc[d] * p;
            ok = ok && cc[d] >= 0 && cc[d] < nc[d] && u[d] >= 0 && u[d] <= p && w[d] >= 0 && w[d] <= p;
          }
          if (!ok) continue;
          const double *cf = &h->coef[6 * ((size_t)cc[0] + (size_t)h->nx * (cc[1] + (size_t)h->ny * cc[2]))];
          double Bv[3], Av[3];
          for (int d = 0; d < 3; ++d) {
            Bv[d] = B[u[d] * n1 + w[d]];
            Av[d] = A[u[d] * n1 + w[d]];
          }
          v += cf[0] * Av[0] * Bv[1] * Bv[2] + cf[1] * Bv[0] * Av[1] * Bv[2] + cf[2] * Bv[0] * Bv[1] * Av[2] +
               cf[3] * Bv[0] * Bv[1] * Bv[2];
        }
        M[(size_t)i * nrf + j] = v;
      }
    }
  }, W);
  if (bad >= 0) {
    char msg[128];
    std::snprintf(msg, sizeof msg, "%s breakdown in full vertex star %ld", ic ? "incomplete Cholesky" : "Cholesky", bad);
    return fail(h->ctx, RZ_ERR_BREAKDOWN, msg);
  }
  if (!h->nrf) {
    rz_status e;
    int *doff = nullptr;
    if ((e = upload(h, &doff, off))) return e;
    if ((e = dalloc(h, &h->fzb64, nslot * nrf)) || (e = dalloc(h, &h->fzb32, nslot * nrf))) return e;
    h->PF = h->P;
    h->PF.nrows = nrf;
    h->PF.off = doff;
    h->nrf = nrf;
  }
  return upload_patch_inverse(h, W);
}

// Vertex stars of H(curl) / H(div) without static condensation (rz_opts.decomposition
// = RZ_DECOMP_FULL, PAFW, eq. pafw): a free DoF belongs to the star of vertex v when
// every cell holding it is one of the cells around v.  Per non-empty star on host
// threads: its DoFs ascending, P_v assembled dense from the cells' six weighted basis
// matrices, exact Cholesky and W = L^{-1}; the stars padded to one size with identity
// rows; per free DoF the positions of its star solutions, in ascending star order.
void cell_keys(const std::vector<double> &w6, int64_t ncells, std::vector<int> &key,
               std::vector<std::array<double, 6>> &keyw);
bool condense_keys(const VecLocal &L, const SpRows basis[6], const std::vector<std::array<double, 6>> &keyw,
                   bool want_S, std::vector<CellCondensed> &conds, std::string &err);

rz_status setup_vertex_stars_vec(rz_problem *h, bool sc) {
  const int p = h->p, space = h->space == RZ_CURL ? 1 : 2;
  VecLocal VL;
  vec_local_layout(space, p, VL);
  SpRows basis[6];
  vec_basis_matrices(h->t, VL, basis);
  // SC-PAFW: the star matrices are assembled from the cells' interface Schur
  // complements (the interior DoFs of a cell belong to that cell alone)
  std::vector<int> key;
  std::vector<std::array<double, 6>> keyw;
  std::vector<CellCondensed> conds;
  if (sc) {
    std::string err;
    cell_keys(h->coef, h->ncells, key, keyw);
    if (!condense_keys(VL, basis, keyw, true, conds, err)) return fail(h->ctx, RZ_ERR_BREAKDOWN, err);
  }
  const VecDev &V = h->V;
  const int nc[3] = {h->nx, h->ny, h->nz};
  const int nvx = nc[0] + 1, nvy = nc[1] + 1, nvz = nc[2] + 1;
  const size_t nvert = (size_t)nvx * nvy * nvz;
  std::vector<char> dirm((size_t)h->ndofs, 0);
  {
    std::vector<int> dl(h->nDir);
    HIPCALL(h, hipMemcpy(dl.data(), h->dlist, sizeof(int) * dl.size(), hipMemcpyDeviceToHost));
    for (int g : dl) dirm[g] = 1;
  }
  auto global = [&](int cx, int cy, int cz, int l, int &m, int C[3]) {
    m = VL.comp[l];
    const int cc[3] = {cx, cy, cz};
    for (int a = 0; a < 3; ++a) C[a] = cc[a] * p + VL.crd[3 * l + a];
    return V.off[m] + C[0] + (int64_t)V.ext[m][0] * (C[1] + (int64_t)V.ext[m][1] * C[2]);
  };
  // star membership: along every axis the cells holding the DoF lie in {v - 1, v}
  auto in_star = [&](int m, const int C[3], const int v[3]) {
    for (int a = 0; a < 3; ++a) {
      const int c = C[a] / p;
      int lo = std::min(c, nc[a] - 1), hi = lo;
      if (vec_is_P(space, m, a) && C[a] % p == 0) {
        lo = std::max(c - 1, 0);
        hi = std::min(c, nc[a] - 1);
      }
      if (lo < v[a] - 1 || hi > v[a]) return false;
    }
    return true;
  };
  std::vector<std::vector<int64_t>> stars(nvert);
  for (size_t vid = 0; vid < nvert; ++vid) {
    const int v[3] = {(int)(vid % nvx), (int)((vid / nvx) % nvy), (int)(vid / ((size_t)nvx * nvy))};
    std::vector<int64_t> &S = stars[vid];
    for (int cz = v[2] - 1; cz <= v[2]; ++cz)
      for (int cy = v[1] - 1; cy <= v[1]; ++cy)
        for (int cx = v[0] - 1; cx <= v[0]; ++cx) {
          if (cx < 0 || cy < 0 || cz < 0 || cx >= nc[0] || cy >= nc[1] || cz >= nc[2]) continue;
          for (int l = 0; l < VL.nloc; ++l) {
            int m, C[3];
            const int64_t g = global(cx, cy, cz, l, m, C);
            if (!dirm[g] && in_star(m, C, v) && !(sc && VL.interior[l])) S.push_back(g);
          }
        }
    std::sort(S.begin(), S.end());
    S.erase(std::unique(S.begin(), S.end()), S.end());
  }
  std::vector<size_t> live;
  int nr = 0;
  for (size_t vid = 0; vid < nvert; ++vid)
    if (!stars[vid].empty()) {
      live.push_back(vid);
      nr = std::max(nr, (int)stars[vid].size());
    }
  const size_t np = live.size(), tri = (size_t)nr * (nr + 1) / 2;
  if ((double)np * tri * 12.0 > 16.0 * (1ull << 30) || (double)np * nr * nr * (double)nr > 5e11)
    return fail(h->ctx, RZ_ERR_ARG, "RZ_DECOMP_FULL / RZ_DECOMP_SC_VERTEX: the dense vertex-star factors are for small "
                                    "meshes and degrees");
  std::vector<double> W;
  const long bad = factor_slots(np, nr, nullptr, [&](size_t k, std::vector<double> &M) {
    const size_t vid = live[k];
    const int v[3] = {(int)(vid % nvx), (int)((vid / nvx) % nvy), (int)(vid / ((size_t)nvx * nvy))};
    const std::vector<int64_t> &S = stars[vid];
    const int ns = (int)S.size();
    for (int i = ns; i < nr; ++i) M[(size_t)i * nr + i] = 1.0;
    std::vector<int> pos(VL.nloc);
    for (int cz = v[2] - 1; cz <= v[2]; ++cz)
      for (int cy = v[1] - 1; cy <= v[1]; ++cy)
        for (int cx = v[0] - 1; cx <= v[0]; ++cx) {
          if (cx < 0 || cy < 0 || cz < 0 || cx >= nc[0] || cy >= nc[1] || cz >= nc[2]) continue;
          for (int l = 0; l < VL.nloc; ++l) {
            int m, C[3];
            const int64_t g = global(cx, cy, cz, l, m, C);
            const auto it = std::lower_bound(S.begin(), S.end(), g);
            pos[l] = (it != S.end() && *it == g) ? (int)(it - S.begin()) : -1;
          }
          const size_t cell = (size_t)cx + (size_t)nc[0] * (cy + (size_t)nc[1] * cz);
          if (sc) {
            const CellCondensed &cd = conds[key[cell]];
            const int nG = (int)cd.G.size();
            for (int i = 0; i < nG; ++i) {
              const int pi = pos[cd.G[i]];
              if (pi < 0) continue;
              for (int j = 0; j < nG; ++j) {
                const int pj = pos[cd.G[j]];
                if (pj >= 0) M[(size_t)pi * nr + pj] += cd.S[(size_t)i * nG + j];
              }
            }
            continue;
          }
          const double *w = &h->coef[6 * cell];
          for (int kb = 0; kb < 6; ++kb)
            for (int l1 = 0; l1 < VL.nloc; ++l1) {
              if (pos[l1] < 0) continue;
              for (const auto &e : basis[kb][l1])
                if (pos[e.first] >= 0) M[(size_t)pos[l1] * nr + pos[e.first]] += w[kb] * e.second;
            }
        }
  }, W);
  if (bad >= 0) {
    char msg[128];
    std::snprintf(msg, sizeof msg, "Cholesky breakdown in vertex star %ld", bad);
    return fail(h->ctx, RZ_ERR_BREAKDOWN, msg);
  }
  // index lists and, per free DoF, its star positions (ascending star order)
  std::vector<int> idx(np * nr, -1);
  std::vector<std::vector<int>> where((size_t)h->ndofs);
  for (size_t k = 0; k < np; ++k) {
    const std::vector<int64_t> &S = stars[live[k]];
    for (size_t i = 0; i < S.size(); ++i) {
      idx[k * nr + i] = (int)S[i];
      where[S[i]].push_back((int)(k * nr + i));
    }
  }
  std::vector<int> rows, ptr{0}, pos;
  for (int64_t g = 0; g < h->ndofs; ++g)
    if (!where[g].empty()) {
      rows.push_back((int)g);
      pos.insert(pos.end(), where[g].begin(), where[g].end());
      ptr.push_back((int)pos.size());
    }
  rz_status e;
  if ((e = upload(h, &h->vs_idx, idx)) || (e = upload(h, &h->vs_rows, rows)) || (e = upload(h, &h->vs_ptr, ptr)) ||
      (e = upload(h, &h->vs_pos, pos)) || (e = dalloc(h, &h->fzb64, np * nr)) || (e = dalloc(h, &h->fzb32, np * nr)))
    return e;
  h->nvs = (int)np;
  h->vs_sc = sc;
  h->nvfree = (int)rows.size();
  h->nrf = nr;
  return upload_patch_inverse(h, W);
}

// vectors of the V-cycle and of the Krylov methods (ndofs each), dot-product
// scratch and the pinned host copy of the scalars
rz_status alloc_krylov(rz_problem *h) {
  rz_status e;
  const int64_t n = h->ndofs;
  if ((e = dalloc(h, &h->r32, n)) || (e = dalloc(h, &h->z32, n)) || (e = dalloc(h, &h->vt, n)) ||
      (e = dalloc(h, &h->vaz, n)) || (e = dalloc(h, &h->vr, n)) || (e = dalloc(h, &h->kr, n)) ||
      (e = dalloc(h, &h->kz, n)) || (e = dalloc(h, &h->kp, n)) || (e = dalloc(h, &h->kAp, n)) ||
      (e = dalloc(h, &h->kro, n)) || (e = dalloc(h, &h->partials, dots_partials_size())) ||
      (e = dalloc(h, &h->dots, 8)))
    return e;
  if (hipHostMalloc((void **)&h->hdots, 8 * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return fail(h->ctx, RZ_ERR_OOM, "pinned host buffer");
  if (h->opts.precision == RZ_PREC_DEFECT &&
      ((e = dalloc(h, &h->kp32, n)) || (e = dalloc(h, &h->kAp32, n)) || (e = dalloc(h, &h->ko32, n)) ||
       (e = dalloc(h, &h->ke32, n)) || (e = dalloc(h, &h->t32, n)) || (e = dalloc(h, &h->az32, n)) ||
       (e = dalloc(h, &h->vr32, n))))
    return e;
  return RZ_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------------
// H(curl) / H(div): setup of the statically condensed Pavarino-Hiptmair relaxation
// (Sec. 4.3-4.5), the p = 1 coarse problem and the transfers (Sec. 4.3, 5)
// ---------------------------------------------------------------------------------------
namespace {

// lattice of NCE_p (space 1) / NCF_p (space 2) on an n[0] x n[1] x n[2] mesh
void vec_lattice(int space, int p, const int n[3], int ext[3][3], int64_t off[4]) {
  int64_t o = 0;
  for (int m = 0; m < 3; ++m) {
    off[m] = o;
    int64_t sz = 1;
    for (int a = 0; a < 3; ++a) {
      ext[m][a] = n[a] * p + (vec_is_P(space, m, a) ? 1 : 0);
      sz *= ext[m][a];
    }
    o += sz;
  }
  off[3] = o;
}

void vec_coords(const int64_t off[4], const int ext[3][3], int64_t g, int &m, int X[3]) {
  m = 0;
  while (m < 2 && g >= off[m + 1]) ++m;
  const int64_t r = g - off[m];
  X[0] = (int)(r % ext[m][0]);
  X[1] = (int)((r / ext[m][0]) % ext[m][1]);
  X[2] = (int)(r / ((int64_t)ext[m][0] * ext[m][1]));
}

int64_t vec_index(const int64_t off[4], const int ext[3][3], int m, const int X[3]) {
  return off[m] + X[0] + (int64_t)ext[m][0] * (X[1] + (int64_t)ext[m][1] * X[2]);
}

// trace condition on a Dirichlet face: a continuous coordinate on that face's plane
bool vec_dirichlet(int space, unsigned dir, const int ext[3][3], int m, const int X[3]) {
  for (int a = 0; a < 3; ++a) {
    if (!vec_is_P(space, m, a)) continue;
    if ((dir & (1u << (2 * a))) && X[a] == 0) return true;
    if ((dir & (1u << (2 * a + 1))) && X[a] == ext[m][a] - 1) return true;
  }
  return false;
}

bool vec_interior(int space, int p, int m, const int X[3]) {
  for (int a = 0; a < 3; ++a)
    if (vec_is_P(space, m, a) && X[a] % p == 0) return false;
  return true;
}

// Free numbering of the lowest-order lattice of `space` (RZ_GRAD: the Q_1 vertices)
// on a mesh of n cells: map[g] = free index or -1.
int p1_free_map(int space, const int n[3], unsigned dir, int ext[3][3], int64_t off[4], std::vector<int> &map) {
  if (space == RZ_GRAD) {
    off[0] = 0;
    off[1] = off[2] = off[3] = (int64_t)(n[0] + 1) * (n[1] + 1) * (n[2] + 1);
    for (int m = 0; m < 3; ++m)
      for (int a = 0; a < 3; ++a) ext[m][a] = n[a] + 1;
  } else {
    vec_lattice(space, 1, n, ext, off);
  }
  map.assign(off[3], -1);
  int nf = 0;
  for (int64_t g = 0; g < off[3]; ++g) {
    int m, X[3];
    vec_coords(off, ext, g, m, X);
    bool d = false;
    if (space == RZ_GRAD) {
      for (int a = 0; a < 3; ++a)
        d = d || ((dir & (1u << (2 * a))) && X[a] == 0) || ((dir & (1u << (2 * a + 1))) && X[a] == n[a]);
    } else {
      d = vec_dirichlet(space, dir, ext, m, X);
    }
    if (!d) map[g] = nf++;
  }
  return nf;
}

// Geometric h-multigrid with Hiptmair relaxation on the lowest-order H(curl) / H(div)
// space (Sec. 5.1, the p-coarse solver of Fig. hcurl_solver_diagram).  Levels: the
// mesh with half the cells per axis while every count is even and the level holds
// more than 512 free DoFs.  Interpolation per component and axis: the hats
// (weights 1 and 1/2) along a continuous axis; along a broken axis each fine half of
// a coarse cell gets 1/2 of its r_0 (in reference coefficients the Piola factor of
// that axis scales with the cell size).  A_{l+1} = P^T A_l P.  Potential space:
// Q_1 (H(curl)) or NCE_1 (H(div)) on the level's mesh with the same Dirichlet faces,
// G the exterior derivative from the 1-D derivative table of degree 1 (the rule of
// the relaxation's potential term at p = 1), its operator G^T A_l G.
rz_status setup_hmg_vec(rz_problem *h, HostCsr A0) {
  const int space = h->space, pspace = space == RZ_CURL ? RZ_GRAD : RZ_CURL;
  const double *D1 = h->t1.D.data();  // 1 x 2: derivative of the two hats in r_0
  const unsigned dir = h->dir;
  int n[3] = {h->nx, h->ny, h->nz};
  std::vector<HostCsr> A, P, R, G, Ap;
  A.push_back(std::move(A0));
  int ext[3][3], pext[3][3];
  int64_t off[4], poff[4];
  std::vector<int> map, pmap;
  for (;;) {
    const int nf = p1_free_map(space, n, dir, ext, off, map);
    const int npf = p1_free_map(pspace, n, dir, pext, poff, pmap);
    if (nf != A.back().n) return fail(h->ctx, RZ_ERR_ARG, "h-multigrid: level numbering mismatch");
    // exterior derivative, rows the free DoFs of the space, columns the free potential DoFs
    HostCsr Gl;
    Gl.n = nf;
    Gl.m = npf;
    Gl.ptr.assign(nf + 1, 0);
    for (int64_t g = 0; g < off[3]; ++g) {
      if (map[g] < 0) continue;
      int m, X[3];
      vec_coords(off, ext, g, m, X);
      std::vector<std::pair<int, double>> row;
      // (sign, potential component, derivative axis): grad of Q_1 along m for NCE
      // component m; curl of NCE for NCF component k
      int terms[2][3], nt = 0;
      if (space == RZ_CURL) {
        terms[nt][0] = 1, terms[nt][1] = 0, terms[nt][2] = m, ++nt;
      } else {
        const int a1 = (m + 1) % 3, a2 = (m + 2) % 3;
        terms[nt][0] = 1, terms[nt][1] = a2, terms[nt][2] = a1, ++nt;
        terms[nt][0] = -1, terms[nt][1] = a1, terms[nt][2] = a2, ++nt;
      }
      for (int q = 0; q < nt; ++q)
        for (int a = 0; a <= 1; ++a) {
          int Y[3] = {X[0], X[1], X[2]};
          Y[terms[q][2]] += a;
          const int col = pmap[vec_index(poff, pext, terms[q][1], Y)];
          if (col >= 0 && D1[a] != 0.0) row.push_back({col, terms[q][0] * D1[a]});
        }
      std::sort(row.begin(), row.end());
      for (auto &cv : row) {
        Gl.col.push_back(cv.first);
        Gl.val.push_back(cv.second);
      }
      Gl.ptr[map[g] + 1] = (int)Gl.col.size();
    }
    for (int i = 0; i < nf; ++i) Gl.ptr[i + 1] = std::max(Gl.ptr[i + 1], Gl.ptr[i]);
    Ap.push_back(csr_product(csr_transpose(Gl), csr_product(A.back(), Gl)));
    G.push_back(std::move(Gl));
    if (!(n[0] % 2 == 0 && n[1] % 2 == 0 && n[2] % 2 == 0) || nf <= kHmgMinFree) break;
    const int nc[3] = {n[0] / 2, n[1] / 2, n[2] / 2};
    int cext[3][3];
    int64_t coff[4];
    std::vector<int> cmap;
    const int ncf = p1_free_map(space, nc, dir, cext, coff, cmap);
    if (ncf == 0) break;
    HostCsr Pl;
    Pl.n = nf;
    Pl.m = ncf;
    Pl.ptr.assign(nf + 1, 0);
    for (int64_t g = 0; g < off[3]; ++g) {
      if (map[g] < 0) continue;
      int m, X[3];
      vec_coords(off, ext, g, m, X);
      int cnt[3], ci[3][2];
      double cw[3][2];
      for (int a = 0; a < 3; ++a) {
        cnt[a] = 0;
        if (vec_is_P(space, m, a)) {
          for (int d = -1; d <= 1; ++d) {
            const int t = X[a] + d;
            if (t < 0 || t % 2 != 0 || t / 2 > nc[a]) continue;
            ci[a][cnt[a]] = t / 2;
            cw[a][cnt[a]++] = d == 0 ? 1.0 : 0.5;
          }
        } else {
          ci[a][0] = X[a] / 2;
          cw[a][0] = 0.5;
          cnt[a] = 1;
        }
      }
      std::vector<std::pair<int, double>> row;
      for (int k = 0; k < cnt[2]; ++k)
        for (int j = 0; j < cnt[1]; ++j)
          for (int i = 0; i < cnt[0]; ++i) {
            const int Y[3] = {ci[0][i], ci[1][j], ci[2][k]};
            const int col = cmap[vec_index(coff, cext, m, Y)];
            if (col >= 0) row.push_back({col, cw[0][i] * cw[1][j] * cw[2][k]});
          }
      std::sort(row.begin(), row.end());
      for (auto &cv : row) {
        Pl.col.push_back(cv.first);
        Pl.val.push_back(cv.second);
      }
      Pl.ptr[map[g] + 1] = (int)Pl.col.size();
    }
    for (int i = 0; i < nf; ++i) Pl.ptr[i + 1] = std::max(Pl.ptr[i + 1], Pl.ptr[i]);
    R.push_back(csr_transpose(Pl));
    A.push_back(csr_product(R.back(), csr_product(A.back(), Pl)));
    P.push_back(std::move(Pl));
    for (int a = 0; a < 3; ++a) n[a] = nc[a];
  }
  return hmg_upload(h, A, P, R, G, Ap);
}

// keys: cells with bitwise equal weights share one
void cell_keys(const std::vector<double> &w6, int64_t ncells, std::vector<int> &key,
               std::vector<std::array<double, 6>> &keyw) {
  std::map<std::array<double, 6>, int> km;
  key.resize(ncells);
  keyw.clear();
  for (int64_t c = 0; c < ncells; ++c) {
    std::array<double, 6> w;
    for (int k = 0; k < 6; ++k) w[k] = w6[6 * c + k];
    auto it = km.find(w);
    if (it == km.end()) {
      it = km.emplace(w, (int)keyw.size()).first;
      keyw.push_back(w);
    }
    key[c] = it->second;
  }
}

bool condense_keys(const VecLocal &L, const SpRows basis[6], const std::vector<std::array<double, 6>> &keyw,
                   bool want_S, std::vector<CellCondensed> &conds, std::string &err) {
  conds.assign(keyw.size(), CellCondensed());
  for (size_t k = 0; k < keyw.size(); ++k)
    if (!vec_condense(L, basis, keyw[k].data(), want_S, conds[k], err)) return false;
  for (size_t k = 1; k < conds.size(); ++k)
    if (conds[k].blocks.size() != conds[0].blocks.size() || conds[k].gi_col != conds[0].gi_col ||
        conds[k].ig_col != conds[0].ig_col) {
      err = "cell operators of one problem differ in structure";
      return false;
    }
  return true;
}


// CSR transpose: (rows r_ids with ptr/col/val) -> rows = distinct columns ascending
void csr_transpose(const std::vector<int> &rid, const std::vector<int> &ptr, const std::vector<int> &col,
                   const std::vector<double> &val, int64_t ncols, std::vector<int> &trid, std::vector<int> &tptr,
                   std::vector<int> &tcol, std::vector<double> &tval) {
  std::vector<int> cnt(ncols, 0);
  for (int c : col) cnt[c] += 1;
  std::vector<int64_t> start(ncols, -1);
  trid.clear();
  tptr.assign(1, 0);
  for (int64_t c = 0; c < ncols; ++c)
    if (cnt[c]) {
      start[c] = tptr.back();
      trid.push_back((int)c);
      tptr.push_back(tptr.back() + cnt[c]);
    }
  tcol.assign(tptr.back(), 0);
  tval.assign(tptr.back(), 0.0);
  std::vector<int> fill(ncols, 0);
  for (size_t t = 0; t < rid.size(); ++t)
    for (int k = ptr[t]; k < ptr[t + 1]; ++k) {
      const int c = col[k];
      const int64_t o = start[c] + fill[c]++;
      tcol[o] = rid[t];
      tval[o] = val[k];
    }
}

rz_status upload_cells(rz_problem *h, const VecLocal &L, const std::vector<CellCondensed> &conds,
                       const std::vector<int> &key) {
  rz_status e;
  const CellCondensed &c0 = conds[0];
  std::vector<int> blk;
  for (auto &b : c0.blocks) blk.insert(blk.end(), b.begin(), b.end());
  std::vector<double> linv, giv, igv;
  for (const CellCondensed &c : conds) {
    linv.insert(linv.end(), c.linv.begin(), c.linv.end());
    giv.insert(giv.end(), c.gi_val.begin(), c.gi_val.end());
    igv.insert(igv.end(), c.ig_val.begin(), c.ig_val.end());
  }
  int *il = nullptr, *gl = nullptr, *lc = nullptr, *lx = nullptr, *db = nullptr, *dk = nullptr, *gp = nullptr,
      *gc = nullptr, *ip = nullptr, *ic = nullptr;
  double *l64 = nullptr, *g64 = nullptr, *i64 = nullptr;
  float *l32 = nullptr, *g32 = nullptr, *i32 = nullptr;
  if ((e = upload(h, &il, c0.I)) || (e = upload(h, &gl, c0.G)) || (e = upload(h, &lc, L.comp)) ||
      (e = upload(h, &lx, L.crd)) || (e = upload(h, &db, blk)) || (e = upload(h, &dk, key)) ||
      (e = upload(h, &gp, c0.gi_ptr)) || (e = upload(h, &gc, c0.gi_col)) || (e = upload(h, &ip, c0.ig_ptr)) ||
      (e = upload(h, &ic, c0.ig_col)) || (e = upload(h, &l64, linv)) || (e = upload(h, &g64, giv)) ||
      (e = upload(h, &i64, igv)) || (e = upload(h, &l32, as_type<float>(linv))) ||
      (e = upload(h, &g32, as_type<float>(giv))) || (e = upload(h, &i32, as_type<float>(igv))))
    return e;
  const int nI = (int)c0.I.size(), nG = (int)c0.G.size(), nb = (int)c0.blocks.size();
  const int ngi = (int)c0.gi_col.size(), nig = (int)c0.ig_col.size();
  h->vc64 = VecCellDev<double>{nI, nG, nb, ngi, nig, il, gl, lc, lx, db, dk, l64, gp, gc, g64, ip, ic, i64};
  h->vc32 = VecCellDev<float>{nI, nG, nb, ngi, nig, il, gl, lc, lx, db, dk, l32, gp, gc, g32, ip, ic, i32};
  return RZ_OK;
}

rz_status upload_edges(rz_problem *h, const EdgePatches &ep, EdgeDev &ed, double **f64, float **f32, double **zb64,
                       float **zb32) {
  rz_status e;
  int *idx = nullptr, *typ = nullptr;
  if ((e = upload(h, &idx, ep.idx)) || (e = upload(h, &typ, ep.type)) || (e = upload(h, f64, ep.fac)) ||
      (e = upload(h, f32, as_type<float>(ep.fac))))
    return e;
  const size_t nz = ep.edge_id.size() * (size_t)ep.lay.nslot;
  if ((e = dalloc(h, zb64, nz)) || (e = dalloc(h, zb32, nz))) return e;
  ed = EdgeDev{};
  ed.p = ep.lay.p;
  ed.nslot = ep.lay.nslot;
  ed.fac_stride = ep.lay.fac_stride;
  ed.npatch = (int)ep.edge_id.size();
  for (int i = 0; i < ep.lay.p; ++i) {
    ed.blk_n[i] = ep.lay.blk_n[i];
    ed.blk_slot[i] = ep.lay.blk_slot[i];
    ed.blk_fac[i] = ep.lay.blk_fac[i];
  }
  ed.idx = idx;
  ed.type = typ;
  // the patches grouped by type, in chunks of at most 256 (one block of the solve
  // kernel each: one factor set in LDS for all its patches)
  const int np = ed.npatch;
  std::vector<int> plist(np), chunk;
  for (int i = 0; i < np; ++i) plist[i] = i;
  std::stable_sort(plist.begin(), plist.end(), [&](int a, int b) { return ep.type[a] < ep.type[b]; });
  for (int i = 0; i < np;) {
    int j = i;
    while (j < np && ep.type[plist[j]] == ep.type[plist[i]] && j - i < 256) ++j;
    chunk.push_back(i);
    chunk.push_back(j);
    chunk.push_back(ep.type[plist[i]]);
    i = j;
  }
  int *dpl = nullptr, *dch = nullptr;
  if ((e = upload(h, &dpl, plist)) || (e = upload(h, &dch, chunk))) return e;
  ed.nchunk = (int)chunk.size() / 3;
  ed.chunk = dch;
  ed.plist = dpl;
  return RZ_OK;
}

// the Q_p potential problem of the H(curl) relaxation: B = (grad phi, beta grad psi)
// with the problem's mesh and Dirichlet faces; its vertex-star patches factored by
// incomplete Cholesky on the static-condensation pattern (as an H(grad) problem)
rz_status build_grad_potential(rz_problem *h, const std::vector<double> &coefq) {
  rz_problem *q = new rz_problem();
  h->pot = q;
  q->ctx = h->ctx;
  q->opts = h->opts;
  q->opts.space = RZ_GRAD;
  q->space = RZ_GRAD;
  q->p = h->p;
  q->nx = h->nx;
  q->ny = h->ny;
  q->nz = h->nz;
  q->dir = h->dir;
  q->Nx = h->nx * h->p + 1;
  q->Ny = h->ny * h->p + 1;
  q->Nz = h->nz * h->p + 1;
  q->ndofs = (int64_t)q->Nx * q->Ny * q->Nz;
  q->ncells = h->ncells;
  q->nvert = h->nvert;
  q->t = h->t;
  q->t1 = h->t1;
  q->coef = coefq;
  grad_symbolic(q);
  return grad_patch_device(q);
}

rz_status setup_vec_relax(rz_problem *h, const std::vector<double> &al, const std::vector<double> &be,
                          const std::vector<std::array<double, 3>> &hs) {
  rz_ctx *ctx = h->ctx;
  hipStream_t s = ctx->stream;
  rz_status e;
  std::string err;
  const int p = h->p, space = h->space;
  const int n[3] = {h->nx, h->ny, h->nz};
  const int64_t nc = h->ncells;
  int ext[3][3];
  int64_t off[4];
  vec_lattice(space, p, n, ext, off);
  // ---- cell algebra of the operator --------------------------------------------------
  VecLocal Lp;
  vec_local_layout(space, p, Lp);
  SpRows basis[6];
  vec_basis_matrices(h->t, Lp, basis);
  std::vector<int> key;
  std::vector<std::array<double, 6>> keyw;
  cell_keys(h->coef, nc, key, keyw);
  std::vector<CellCondensed> conds;
  if (!condense_keys(Lp, basis, keyw, true, conds, err)) return fail(ctx, RZ_ERR_BREAKDOWN, err);
  if ((e = upload_cells(h, Lp, conds, key))) return e;
  const int nG = (int)conds[0].G.size();
  // ---- free interface DoFs and the condensation sums -------------------------------
  std::vector<int> cnt(h->ndofs, 0);
  for (int64_t c = 0; c < nc; ++c) {
    const int cc[3] = {(int)(c % n[0]), (int)((c / n[0]) % n[1]), (int)(c / ((int64_t)n[0] * n[1]))};
    for (int g = 0; g < nG; ++g) {
      const int l = conds[0].G[g], m = Lp.comp[l];
      int X[3];
      for (int a = 0; a < 3; ++a) X[a] = cc[a] * p + Lp.crd[3 * l + a];
      if (!vec_dirichlet(space, h->dir, ext, m, X)) cnt[vec_index(off, ext, m, X)] += 1;
    }
  }
  std::vector<int> gam, cptr(1, 0), cpos;
  std::vector<int64_t> start(h->ndofs, -1);
  for (int64_t g = 0; g < h->ndofs; ++g)
    if (cnt[g]) {
      start[g] = cptr.back();
      gam.push_back((int)g);
      cptr.push_back(cptr.back() + cnt[g]);
    }
  cpos.assign(cptr.back(), 0);
  std::fill(cnt.begin(), cnt.end(), 0);
  for (int64_t c = 0; c < nc; ++c) {
    const int cc[3] = {(int)(c % n[0]), (int)((c / n[0]) % n[1]), (int)(c / ((int64_t)n[0] * n[1]))};
    for (int g = 0; g < nG; ++g) {
      const int l = conds[0].G[g], m = Lp.comp[l];
      int X[3];
      for (int a = 0; a < 3; ++a) X[a] = cc[a] * p + Lp.crd[3 * l + a];
      if (vec_dirichlet(space, h->dir, ext, m, X)) continue;
      const int64_t gi = vec_index(off, ext, m, X);
      cpos[start[gi] + cnt[gi]++] = (int)(c * nG + g);
    }
  }
  h->nGam = (int)gam.size();
  if ((e = upload(h, &h->gam, gam)) || (e = upload(h, &h->cg_ptr, cptr)) || (e = upload(h, &h->cg_pos, cpos)) ||
      (e = dalloc(h, &h->veb64, (size_t)nc * nG)) || (e = dalloc(h, &h->veb32, (size_t)nc * nG)) ||
      (e = dalloc(h, &h->vrt64, h->ndofs)) || (e = dalloc(h, &h->vrt32, h->ndofs)))
    return e;
  // ---- local solves: edge stars (curl) or face stars (div, diagonal) ----------------
  if (space == RZ_CURL) {
    EdgePatches ep;
    if (!edge_patches_build(p, n, h->dir, ext, off, Lp, key, conds, ep, err)) return fail(ctx, RZ_ERR_BREAKDOWN, err);
    if (ep.rows != gam) return fail(ctx, RZ_ERR_ARG, "edge patches do not cover the interface DoFs");
    if ((e = upload_edges(h, ep, h->ed, &h->efac64, &h->efac32, &h->ezb64, &h->ezb32)) ||
        (e = upload(h, &h->eg_ptr, ep.ptr)) || (e = upload(h, &h->eg_pos, ep.pos)))
      return e;
    h->edge_ids = ep.edge_id;
    h->edge_idx = ep.idx;
    h->edge_nslot = ep.lay.nslot;
  } else {
    std::vector<double> dsum(gam.size(), 0.0);
    for (size_t t = 0; t < gam.size(); ++t)
      for (int k = cptr[t]; k < cptr[t + 1]; ++k) {
        const int c = cpos[k] / nG, g = cpos[k] % nG;
        dsum[t] += conds[key[c]].S[(size_t)g * nG + g];
      }
    for (double &d : dsum) {
      if (!(d > 0)) return fail(ctx, RZ_ERR_BREAKDOWN, "face-star pivot is not positive");
      d = 1.0 / d;
    }
    if ((e = upload(h, &h->dinv64, dsum)) || (e = upload(h, &h->dinv32, as_type<float>(dsum)))) return e;
  }
  // ---- the potential problem and D_GG -------------------------------------------------
  const Tables1D &t = h->t;
  const int n1 = p + 1;
  std::vector<int> drow, dptr(1, 0), dcol;
  std::vector<double> dval;
  int64_t pndofs = 0;
  std::vector<double> coefe_pot;  // H(div): the NCE_p potential's weights
  if (space == RZ_CURL) {
    std::vector<double> coefq(6 * nc, 0.0);
    for (int64_t c = 0; c < nc; ++c) {
      const double V = hs[c][0] * hs[c][1] * hs[c][2];
      for (int d = 0; d < 3; ++d) coefq[6 * c + d] = be[c] * V / (2.0 * hs[c][d] * hs[c][d]);
    }
    if ((e = build_grad_potential(h, coefq))) return e;
    const rz_problem *q = h->pot;
    pndofs = q->ndofs;
    auto q_free_iface = [&](const int Y[3]) {
      if (Y[0] % p && Y[1] % p && Y[2] % p) return false;
      return !lat_dirichlet_h(q, Y[0], Y[1], Y[2]);
    };
    for (int g : gam) {  // grad: NCE component m at X <- Q_p points along m
      int m, X[3];
      vec_coords(off, ext, g, m, X);
      const int c = X[m] / p, j = X[m] % p;
      for (int a = 0; a <= p; ++a) {
        const double v = t.D[j * n1 + a];
        if (v == 0.0) continue;
        int Y[3] = {X[0], X[1], X[2]};
        Y[m] = c * p + a;
        if (!q_free_iface(Y)) continue;
        dcol.push_back((int)(Y[0] + (int64_t)q->Nx * (Y[1] + (int64_t)q->Ny * Y[2])));
        dval.push_back(v);
      }
      dptr.push_back((int)dcol.size());
    }
  } else {
    // NCE_p potential: B = (curl phi, beta curl psi) + eps (phi, beta psi)
    const double eps = h->opts.hdiv_eps > 0 ? h->opts.hdiv_eps : 1e-3;
    std::vector<double> coefe(6 * nc, 0.0);
    for (int64_t c = 0; c < nc; ++c) {
      const double V = hs[c][0] * hs[c][1] * hs[c][2];
      for (int d = 0; d < 3; ++d) {
        coefe[6 * c + d] = be[c] * 2.0 * hs[c][d] * hs[c][d] / V;
        coefe[6 * c + 3 + d] = eps * be[c] * V / (2.0 * hs[c][d] * hs[c][d]);
      }
    }
    coefe_pot = coefe;
    int exte[3][3];
    int64_t offe[4];
    vec_lattice(RZ_CURL, p, n, exte, offe);
    pndofs = offe[3];
    VecLocal Le;
    vec_local_layout(RZ_CURL, p, Le);
    SpRows basise[6];
    vec_basis_matrices(t, Le, basise);
    std::vector<int> keye;
    std::vector<std::array<double, 6>> keywe;
    cell_keys(coefe, nc, keye, keywe);
    std::vector<CellCondensed> condse;
    if (!condense_keys(Le, basise, keywe, true, condse, err)) return fail(ctx, RZ_ERR_BREAKDOWN, err);
    EdgePatches ep;
    if (!edge_patches_build(p, n, h->dir, exte, offe, Le, keye, condse, ep, err))
      return fail(ctx, RZ_ERR_BREAKDOWN, err);
    if ((e = upload_edges(h, ep, h->ped, &h->pfac64, &h->pfac32, &h->pzb64, &h->pzb32)) ||
        (e = upload(h, &h->pg_rows, ep.rows)) || (e = upload(h, &h->pg_ptr, ep.ptr)) ||
        (e = upload(h, &h->pg_pos, ep.pos)))
      return e;
    h->npg = (int)ep.rows.size();
    h->edge_ids = ep.edge_id;
    h->edge_idx = ep.idx;
    h->edge_nslot = ep.lay.nslot;
    auto e_free_iface = [&](int c, const int Y[3]) {
      return !vec_interior(RZ_CURL, p, c, Y) && !vec_dirichlet(RZ_CURL, h->dir, exte, c, Y);
    };
    for (int g : gam) {  // curl: NCF component k at X <- NCE d_{a1} u_{a2} - d_{a2} u_{a1}
      int k, X[3];
      vec_coords(off, ext, g, k, X);
      const int a1 = (k + 1) % 3, a2 = (k + 2) % 3;
      const int terms[2][3] = {{1, a2, a1}, {-1, a1, a2}};  // sign, component, derivative axis
      std::vector<std::pair<int, double>> row;
      for (auto &tm : terms) {
        const int c = tm[1], d = tm[2];
        const int cd = X[d] / p, j = X[d] % p;
        for (int a = 0; a <= p; ++a) {
          const double v = tm[0] * t.D[j * n1 + a];
          if (v == 0.0) continue;
          int Y[3] = {X[0], X[1], X[2]};
          Y[d] = cd * p + a;
          if (!e_free_iface(c, Y)) continue;
          row.push_back({(int)vec_index(offe, exte, c, Y), v});
        }
      }
      std::sort(row.begin(), row.end());
      for (auto &rv : row) {
        dcol.push_back(rv.first);
        dval.push_back(rv.second);
      }
      dptr.push_back((int)dcol.size());
    }
  }
  drow = gam;
  std::vector<int> trid, tptr, tcol;
  std::vector<double> tval;
  csr_transpose(drow, dptr, dcol, dval, pndofs, trid, tptr, tcol, tval);
  h->pndofs = pndofs;
  h->ndt = (int)trid.size();
  if ((e = upload(h, &h->d_ptr, dptr)) || (e = upload(h, &h->d_col, dcol)) || (e = upload(h, &h->d_val64, dval)) ||
      (e = upload(h, &h->d_val32, as_type<float>(dval))) || (e = upload(h, &h->dt_rows, trid)) ||
      (e = upload(h, &h->dt_ptr, tptr)) || (e = upload(h, &h->dt_col, tcol)) ||
      (e = upload(h, &h->dt_val64, tval)) || (e = upload(h, &h->dt_val32, as_type<float>(tval))) ||
      (e = dalloc(h, &h->vq64, pndofs)) || (e = dalloc(h, &h->vq32, pndofs)) || (e = dalloc(h, &h->vy64, pndofs)) ||
      (e = dalloc(h, &h->vy32, pndofs)))
    return e;
  // entries of the potential vectors outside the rows written stay zero
  launch_fill(h->vq64, 0.0, pndofs, s);
  launch_fill_f(h->vq32, 0.0f, pndofs, s);
  launch_fill(h->vy64, 0.0, pndofs, s);
  launch_fill_f(h->vy32, 0.0f, pndofs, s);
  if (h->opts.decomposition == RZ_DECOMP_FULL_PH && (e = setup_ph_full(h, coefe_pot))) return e;
  // ---- Dirichlet rows --------------------------------------------------------------------
  std::vector<int> dl;
  h->dmask.assign(h->ndofs, 0);
  for (int64_t g = 0; g < h->ndofs; ++g) {
    int m, X[3];
    vec_coords(off, ext, g, m, X);
    if (vec_dirichlet(space, h->dir, ext, m, X)) {
      dl.push_back((int)g);
      h->dmask[g] = 1;
    }
  }
  h->nDir = (int)dl.size();
  if ((e = upload(h, &h->dlist, dl))) return e;
  // ---- the p = 1 coarse problem: dense inverse on its free DoFs ---------------------
  int ext1[3][3];
  int64_t off1[4];
  vec_lattice(space, 1, n, ext1, off1);
  std::vector<int> cmap(off1[3], -1);
  int ncf = 0;
  for (int64_t g = 0; g < off1[3]; ++g) {
    int m, X[3];
    vec_coords(off1, ext1, g, m, X);
    if (!vec_dirichlet(space, h->dir, ext1, m, X)) cmap[g] = ncf++;
  }
  h->ncf = ncf;
  if (ncf > 0) {
    VecLocal L1;
    vec_local_layout(space, 1, L1);
    SpRows basis1[6];
    vec_basis_matrices(h->t1, L1, basis1);
    std::vector<int> lg(L1.nloc);
    // the cells' entries in a fixed order (cell, weight, row, column) into per-row maps
    auto for_entries = [&](auto &&add) {
      for (int64_t c = 0; c < nc; ++c) {
        const int cc[3] = {(int)(c % n[0]), (int)((c / n[0]) % n[1]), (int)(c / ((int64_t)n[0] * n[1]))};
        for (int l = 0; l < L1.nloc; ++l) {
          int X[3];
          for (int a = 0; a < 3; ++a) X[a] = cc[a] + L1.crd[3 * l + a];
          lg[l] = cmap[vec_index(off1, ext1, L1.comp[l], X)];
        }
        for (int k = 0; k < 6; ++k) {
          const double w = h->coef[6 * c + k];
          for (int r = 0; r < L1.nloc; ++r) {
            if (lg[r] < 0) continue;
            for (auto &ev : basis1[k][r])
              if (lg[ev.first] >= 0) add(lg[r], lg[ev.first], w * ev.second);
          }
        }
      }
    };
    if (h->opts.coarse == RZ_COARSE_HMG) {
      std::vector<std::map<int, double>> rows(ncf);
      for_entries([&](int r, int c, double v) { rows[r][c] += v; });
      HostCsr A0;
      A0.n = A0.m = ncf;
      A0.ptr.assign(ncf + 1, 0);
      for (int r = 0; r < ncf; ++r) {
        for (auto &cv : rows[r]) {
          A0.col.push_back(cv.first);
          A0.val.push_back(cv.second);
        }
        A0.ptr[r + 1] = (int)A0.col.size();
      }
      std::vector<std::map<int, double>>().swap(rows);
      if ((e = setup_hmg_vec(h, std::move(A0)))) return e;
    } else {
      std::vector<double> A0((size_t)ncf * ncf, 0.0);
      for_entries([&](int r, int c, double v) { A0[(size_t)r * ncf + c] += v; });
      if ((e = upload(h, &h->cinv64, A0))) return e;
      std::vector<double>().swap(A0);
      double *tmp = nullptr;
      if (hipMalloc(&tmp, sizeof(double) * (size_t)ncf * ncf) != hipSuccess)
        return fail(ctx, RZ_ERR_OOM, "coarse inverse workspace");
      launch_sweep_inverse(ncf, h->cinv64, tmp, h->status, s);
      const hipError_t se = hipStreamSynchronize(s);
      hipFree(tmp);
      if (se != hipSuccess) return fail(ctx, RZ_ERR_HIP, "coarse inverse failed");
      int stv = 0;
      HIPCALL(h, hipMemcpy(&stv, h->status, sizeof(int), hipMemcpyDeviceToHost));
      if (stv) return fail(ctx, RZ_ERR_SINGULAR, "coarse factorisation: non-positive pivot");
      if (h->opts.precision != RZ_PREC_F64) {
        if ((e = dalloc(h, &h->cinv32, (size_t)ncf * ncf))) return e;
        launch_cast_d2f(h->cinv64, h->cinv32, (int64_t)ncf * ncf, s);
      }
      const size_t nt = ((size_t)ncf + 63) / 64;
      if ((e = dalloc(h, &h->csym, nt * nt * 64))) return e;
    }
    // prolongation (the embedding of the p = 1 space, per axis: hats on continuous
    // axes, the constant r_0 on broken ones) and restriction = its transpose
    std::vector<int> prow, pptr(1, 0), pcol;
    std::vector<double> pval;
    for (int64_t g = 0; g < h->ndofs; ++g) {
      if (h->dmask[g]) continue;
      int m, X[3];
      vec_coords(off, ext, g, m, X);
      int cnum[3], cix[3][2];
      double cw[3][2];
      bool empty = false;
      for (int a = 0; a < 3; ++a) {
        const int c = X[a] / p, i = X[a] % p;
        if (vec_is_P(space, m, a)) {
          if (i == 0) {
            cnum[a] = 1;
            cix[a][0] = c;
            cw[a][0] = 1.0;
          } else {
            cnum[a] = 2;
            cix[a][0] = c;
            cw[a][0] = t.E[2 * i];
            cix[a][1] = c + 1;
            cw[a][1] = t.E[2 * i + 1];
          }
        } else {
          cnum[a] = 1;
          cix[a][0] = c;
          cw[a][0] = i == 0 ? 1.0 : 0.0;
          empty = empty || i != 0;
        }
      }
      if (empty) continue;
      std::vector<std::pair<int, double>> row;
      for (int k = 0; k < cnum[2]; ++k)
        for (int j = 0; j < cnum[1]; ++j)
          for (int i = 0; i < cnum[0]; ++i) {
            const double w = cw[0][i] * cw[1][j] * cw[2][k];
            if (w == 0.0) continue;
            const int Y[3] = {cix[0][i], cix[1][j], cix[2][k]};
            const int ci = cmap[vec_index(off1, ext1, m, Y)];
            if (ci >= 0) row.push_back({ci, w});
          }
      if (row.empty()) continue;
      std::sort(row.begin(), row.end());
      prow.push_back((int)g);
      for (auto &rv : row) {
        pcol.push_back(rv.first);
        pval.push_back(rv.second);
      }
      pptr.push_back((int)pcol.size());
    }
    std::vector<int> rrid, rptr, rcol;
    std::vector<double> rval;
    csr_transpose(prow, pptr, pcol, pval, ncf, rrid, rptr, rcol, rval);
    if ((int)rrid.size() != ncf) return fail(ctx, RZ_ERR_ARG, "a coarse DoF has no fine counterpart");
    h->npf = (int)prow.size();
    if ((e = upload(h, &h->pp_rows, prow)) || (e = upload(h, &h->pp_ptr, pptr)) || (e = upload(h, &h->pp_col, pcol)) ||
        (e = upload(h, &h->pp_val, pval)) || (e = upload(h, &h->pr_ptr, rptr)) || (e = upload(h, &h->pr_col, rcol)) ||
        (e = upload(h, &h->pr_val, rval)) || (e = dalloc(h, &h->vcr, ncf)) || (e = dalloc(h, &h->vcx, ncf)))
      return e;
  }
  HIPCALL(h, hipStreamSynchronize(s));
  return RZ_OK;
}

}  // namespace

// =========================================================================================
// public API
// =========================================================================================
namespace {

// Stars of the k-dimensional entities of NCE_p (space 1) or NCF_p (space 2) without
// static condensation (PH, Sec. 4.3 eq. ph): kind 1 the edges (the cell along the edge,
// up to two cells across each of its vertex coordinates), kind 2 the faces (up to two
// cells across the face's vertex plane).  A free DoF belongs to a star when every
// cell holding it is among the entity's cells.  Entities by axis (of the edge, of the
// face normal), then lattice order; empty stars dropped.  Each star matrix is
// assembled from the cells' weighted basis matrices (weights coef6, six per cell),
// factored exactly on host threads and applied as W = L^{-1} (FP64 and FP32).
rz_status build_entity_stars(rz_problem *h, int space, const double *coef6, int kind, rz_problem::StarSet &S) {
  const int p = h->p;
  VecLocal VL;
  vec_local_layout(space, p, VL);
  SpRows basis[6];
  vec_basis_matrices(h->t, VL, basis);
  const int n[3] = {h->nx, h->ny, h->nz};
  int ext[3][3];
  int64_t off[4];
  vec_lattice(space, p, n, ext, off);
  auto global = [&](const int cc[3], int l, int &m, int C[3]) {
    m = VL.comp[l];
    for (int a = 0; a < 3; ++a) C[a] = cc[a] * p + VL.crd[3 * l + a];
    return vec_index(off, ext, m, C);
  };
  struct Ent {
    int lo[3], hi[3];
  };
  std::vector<Ent> ents;
  for (int m = 0; m < 3; ++m) {
    bool cell_axis[3];
    int ee[3];
    for (int a = 0; a < 3; ++a) {
      cell_axis[a] = kind == 1 ? a == m : a != m;
      ee[a] = cell_axis[a] ? n[a] : n[a] + 1;
    }
    for (int k2 = 0; k2 < ee[2]; ++k2)
      for (int k1 = 0; k1 < ee[1]; ++k1)
        for (int k0 = 0; k0 < ee[0]; ++k0) {
          const int c[3] = {k0, k1, k2};
          Ent E;
          for (int a = 0; a < 3; ++a) {
            E.lo[a] = cell_axis[a] ? c[a] : c[a] - 1;
            E.hi[a] = c[a];
          }
          ents.push_back(E);
        }
  }
  auto inside = [&](int m, const int C[3], const Ent &E) {
    for (int a = 0; a < 3; ++a) {
      const int c = C[a] / p;
      int lo = std::min(c, n[a] - 1), hi = lo;
      if (vec_is_P(space, m, a) && C[a] % p == 0) {
        lo = std::max(c - 1, 0);
        hi = std::min(c, n[a] - 1);
      }
      if (lo < E.lo[a] || hi > E.hi[a]) return false;
    }
    return true;
  };
  auto for_cells = [&](const Ent &E, auto &&f) {
    for (int cz = std::max(E.lo[2], 0); cz <= std::min(E.hi[2], n[2] - 1); ++cz)
      for (int cy = std::max(E.lo[1], 0); cy <= std::min(E.hi[1], n[1] - 1); ++cy)
        for (int cx = std::max(E.lo[0], 0); cx <= std::min(E.hi[0], n[0] - 1); ++cx) {
          const int cc[3] = {cx, cy, cz};
          f(cc);
        }
  };
  std::vector<std::vector<int64_t>> stars(ents.size());
  for (size_t k = 0; k < ents.size(); ++k) {
    std::vector<int64_t> &St = stars[k];
    for_cells(ents[k], [&](const int cc[3]) {
      for (int l = 0; l < VL.nloc; ++l) {
        int m, C[3];
        const int64_t g = global(cc, l, m, C);
        if (!vec_dirichlet(space, h->dir, ext, m, C) && inside(m, C, ents[k])) St.push_back(g);
      }
    });
    std::sort(St.begin(), St.end());
    St.erase(std::unique(St.begin(), St.end()), St.end());
  }
  std::vector<size_t> live;
  int nr = 0;
  for (size_t k = 0; k < ents.size(); ++k)
    if (!stars[k].empty()) {
      live.push_back(k);
      nr = std::max(nr, (int)stars[k].size());
    }
  const size_t np = live.size(), tri = (size_t)nr * (nr + 1) / 2;
  if ((double)np * tri * 12.0 > 16.0 * (1ull << 30) || (double)np * nr * nr * (double)nr > 5e11)
    return fail(h->ctx, RZ_ERR_ARG, "RZ_DECOMP_FULL_PH: the dense star factors are for small meshes and degrees");
  std::vector<double> W;
  const long bad = factor_slots(np, nr, nullptr, [&](size_t k, std::vector<double> &M) {
    const std::vector<int64_t> &St = stars[live[k]];
    const int ns = (int)St.size();
    for (int i = ns; i < nr; ++i) M[(size_t)i * nr + i] = 1.0;
    std::vector<int> pos(VL.nloc);
    for_cells(ents[live[k]], [&](const int cc[3]) {
      for (int l = 0; l < VL.nloc; ++l) {
        int m, C[3];
        const int64_t g = global(cc, l, m, C);
        const auto it = std::lower_bound(St.begin(), St.end(), g);
        pos[l] = (it != St.end() && *it == g) ? (int)(it - St.begin()) : -1;
      }
      const double *w = coef6 + 6 * ((size_t)cc[0] + (size_t)n[0] * (cc[1] + (size_t)n[1] * cc[2]));
      for (int kb = 0; kb < 6; ++kb)
        for (int l1 = 0; l1 < VL.nloc; ++l1) {
          if (pos[l1] < 0) continue;
          for (const auto &ev : basis[kb][l1])
            if (pos[ev.first] >= 0) M[(size_t)pos[l1] * nr + pos[ev.first]] += w[kb] * ev.second;
        }
    });
  }, W);
  if (bad >= 0) {
    char msg[128];
    std::snprintf(msg, sizeof msg, "Cholesky breakdown in star %ld", bad);
    return fail(h->ctx, RZ_ERR_BREAKDOWN, msg);
  }
  std::vector<int> idx(np * nr, -1);
  std::vector<std::vector<int>> where((size_t)off[3]);
  for (size_t k = 0; k < np; ++k) {
    const std::vector<int64_t> &St = stars[live[k]];
    for (size_t i = 0; i < St.size(); ++i) {
      idx[k * nr + i] = (int)St[i];
      where[St[i]].push_back((int)(k * nr + i));
    }
  }
  std::vector<int> rows, ptr{0}, pos;
  for (int64_t g = 0; g < off[3]; ++g)
    if (!where[g].empty()) {
      rows.push_back((int)g);
      pos.insert(pos.end(), where[g].begin(), where[g].end());
      ptr.push_back((int)pos.size());
    }
  rz_status e;
  if ((e = upload(h, &S.idx, idx)) || (e = upload(h, &S.rows, rows)) || (e = upload(h, &S.ptr, ptr)) ||
      (e = upload(h, &S.pos, pos)) || (e = upload(h, &S.w64, W)) || (e = dalloc(h, &S.w32, W.size())) ||
      (e = dalloc(h, &S.zb64, np * nr)) || (e = dalloc(h, &S.zb32, np * nr)))
    return e;
  launch_cast_d2f(S.w64, S.w32, (int64_t)W.size(), h->ctx->stream);
  S.np = (int)np;
  S.nr = nr;
  S.nfree = (int)rows.size();
  return RZ_OK;
}

// PH without static condensation: the stars of the space, the potential's stars (H(curl):
// the full vertex stars of the Q_p problem h->pot; H(div): NCE_p edge stars with the
// weights coefe), and the full exterior derivative between the free DoFs of the
// potential space and of the space (the 1-D derivative table of degree p), with its
// transpose.
rz_status setup_ph_full(rz_problem *h, const std::vector<double> &coefe) {
  const int p = h->p, space = h->space, n1 = p + 1;
  const int n[3] = {h->nx, h->ny, h->nz};
  rz_status e;
  if ((e = build_entity_stars(h, space, h->coef.data(), space == RZ_CURL ? 1 : 2, h->ph_s))) return e;
  if (space == RZ_CURL) {
    if ((e = setup_full_stars(h->pot))) return e;
  } else if ((e = build_entity_stars(h, RZ_CURL, coefe.data(), 1, h->ph_p))) {
    return e;
  }
  int ext[3][3], exte[3][3];
  int64_t off[4], offe[4];
  vec_lattice(space, p, n, ext, off);
  vec_lattice(RZ_CURL, p, n, exte, offe);
  const rz_problem *q = h->pot;
  const Tables1D &t = h->t;
  std::vector<int> drow, dptr(1, 0), dcol;
  std::vector<double> dval;
  for (int64_t g = 0; g < off[3]; ++g) {
    int m, X[3];
    vec_coords(off, ext, g, m, X);
    if (vec_dirichlet(space, h->dir, ext, m, X)) continue;
    std::vector<std::pair<int, double>> row;
    if (space == RZ_CURL) {  // NCE component m at X <- Q_p points along m
      const int c = X[m] / p, j = X[m] % p;
      for (int a = 0; a <= p; ++a) {
        const double v = t.D[j * n1 + a];
        if (v == 0.0) continue;
        int Y[3] = {X[0], X[1], X[2]};
        Y[m] = c * p + a;
        if (lat_dirichlet_h(q, Y[0], Y[1], Y[2])) continue;
        row.push_back({(int)(Y[0] + (int64_t)q->Nx * (Y[1] + (int64_t)q->Ny * Y[2])), v});
      }
    } else {  // NCF component m at X <- NCE d_{a1} u_{a2} - d_{a2} u_{a1}
      const int a1 = (m + 1) % 3, a2 = (m + 2) % 3;
      const int terms[2][3] = {{1, a2, a1}, {-1, a1, a2}};
      for (auto &tm : terms) {
        const int c = tm[1], d = tm[2];
        const int cd = X[d] / p, j = X[d] % p;
        for (int a = 0; a <= p; ++a) {
          const double v = tm[0] * t.D[j * n1 + a];
          if (v == 0.0) continue;
          int Y[3] = {X[0], X[1], X[2]};
          Y[d] = cd * p + a;
          if (vec_dirichlet(RZ_CURL, h->dir, exte, c, Y)) continue;
          row.push_back({(int)vec_index(offe, exte, c, Y), v});
        }
      }
    }
    if (row.empty()) continue;
    std::sort(row.begin(), row.end());
    drow.push_back((int)g);
    for (auto &cv : row) {
      dcol.push_back(cv.first);
      dval.push_back(cv.second);
    }
    dptr.push_back((int)dcol.size());
  }
  std::vector<int> trid, tptr, tcol;
  std::vector<double> tval;
  csr_transpose(drow, dptr, dcol, dval, h->pndofs, trid, tptr, tcol, tval);
  h->nphd = (int)drow.size();
  h->nphdt = (int)trid.size();
  if ((e = upload(h, &h->phd_rows, drow)) || (e = upload(h, &h->phd_ptr, dptr)) || (e = upload(h, &h->phd_col, dcol)) ||
      (e = upload(h, &h->phd_val64, dval)) || (e = upload(h, &h->phd_val32, as_type<float>(dval))) ||
      (e = upload(h, &h->phdt_rows, trid)) || (e = upload(h, &h->phdt_ptr, tptr)) ||
      (e = upload(h, &h->phdt_col, tcol)) || (e = upload(h, &h->phdt_val64, tval)) ||
      (e = upload(h, &h->phdt_val32, as_type<float>(tval))))
    return e;
  HIPCALL(h, hipStreamSynchronize(h->ctx->stream));
  return RZ_OK;
}

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
  std::vector<double> alc(h->ncells), bec(h->ncells);
  std::vector<std::array<double, 3>> hsc(h->ncells);
  for (int64_t c = 0; c < h->ncells; ++c) {
    int cx = c % h->nx, cy = (c / h->nx) % h->ny, cz = c / ((int64_t)h->nx * h->ny);
    const double hs[3] = {h->vert[3 * (cx + 1)] - h->vert[3 * cx],
                          h->vert[3 * ((cy + 1) * nvx) + 1] - h->vert[3 * (cy * nvx) + 1],
                          h->vert[3 * ((int64_t)(cz + 1) * nvx * nvy) + 2] - h->vert[3 * ((int64_t)cz * nvx * nvy) + 2]};
    const double al = cf->kind == RZ_COEF_CONST ? cf->alpha[0] : cf->alpha[c];
    const double be = cf->kind == RZ_COEF_CONST ? cf->beta[0] : cf->beta[c];
    alc[c] = al;
    bec[c] = be;
    hsc[c] = {hs[0], hs[1], hs[2]};
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
  if (off > 0x7fffffffL) {
    delete h;
    return fail(ctx, RZ_ERR_ARG, "H(curl)/H(div) vectors are limited to 2^31 - 1 entries");
  }
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
  const size_t neb = (size_t)h->ndofs * (h->space == RZ_CURL ? 3 : 1);
  if ((e = upload(h, &h->coef64, h->coef)) || (e = upload(h, &h->coef32, c32)) || (e = upload(h, &h->B64, h->t.B)) ||
      (e = upload(h, &h->B32, B32)) || (e = upload(h, &h->D64, h->t.D)) || (e = upload(h, &h->D32, D32)) ||
      (e = dalloc(h, &h->eb64, neb)) || (e = dalloc(h, &h->eb32, neb)) || (e = dalloc(h, &h->status, 1)))
    return bail(e);
  if (hipMemsetAsync(h->status, 0, sizeof(int), s) != hipSuccess) return bail(fail(ctx, RZ_ERR_HIP, "memset"));
  // the relaxation, coarse problem and transfers of the solver
  if ((e = setup_vec_relax(h, alc, bec, hsc)) || (e = alloc_krylov(h))) return bail(e);
  if ((h->opts.decomposition == RZ_DECOMP_FULL || h->opts.decomposition == RZ_DECOMP_SC_VERTEX) &&
      (e = setup_vertex_stars_vec(h, h->opts.decomposition == RZ_DECOMP_SC_VERTEX)))
    return bail(e);
  if (h->opts.omega > 0) {
    h->omega = h->opts.omega;
  } else {
    double lam = 0;
    if ((e = estimate_lambda(h, &lam))) return bail(e);
    h->omega = 2.0 / (1.2 * lam);
  }
  if (hipStreamSynchronize(s) != hipSuccess) return bail(fail(ctx, RZ_ERR_HIP, "setup failed"));
  *out = h;
  return RZ_OK;
}

rz_status require_grad(const rz_problem *h) {
  if (h->space != RZ_GRAD)
    return fail(h->ctx, RZ_ERR_ARG, "this call is available for H(grad) only");
  return RZ_OK;
}

}  // namespace

namespace {

// PCG (Sec. 5) on nv right-hand sides of one problem as a step machine.  Each step
// enqueues stream-ordered work for every right-hand side that is still running,
// and the read-back of the scalars the host needs next (copied asynchronously to
// pinned memory); the caller waits for the stream (or an event) and calls the next
// step.  The right-hand sides iterate in lockstep: their V-cycles run together
// (vcycle_multi: the patch solves of a relaxation take two vectors per launch), every other step
// per vector.  A right-hand side that has converged drops out of the later steps.
// The CG coefficients are formed on the device (alpha in the update kernel, beta in
// the direction update), so one host round trip per iteration remains: the
// convergence test on r.r, which decides whether the next V-cycle runs.
// Device scalar slots (dots of each right-hand side): [2q], [2q+1]: r.z and (mixed)
// r_old.z of the iterations with parity q; [4]: p.Ap; [5]: r.r after the update;
// [6]: other norms.
struct BlockRun {
  rz_problem *h = nullptr;
  int nv = 0;
  const double *bu = nullptr;  // caller's vectors (interleaved when nv > 1)
  double *xu = nullptr;
  // per right-hand side: what the last step enqueued, and what comes next
  enum Kind { NONE, NORM_B, ITER, TRUE_RES, FINAL, DONE };
  struct Rhs {
    const double *b = nullptr;
    double *x = nullptr;
    Kind enq = NONE, next = NONE;
    bool restart = false;     // continue from the true residual (stored in Ap)
    int it = 0;
    double rz0 = 0;           // r.z of the first iteration (natural norm squared)
    int it_natural = -1;      // first iteration count at which the natural norm had dropped by rtol
    double nb = 0, tol = 0, relres = 0;
    rz_status result = RZ_OK;
  };
  std::vector<Rhs> s;
  bool started = false, done = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

enum { kSlotPap = 4, kSlotRr = 5, kSlotNorm = 6 };

// v.v into slot kSlotNorm of right-hand side i
void block_norm(rz_problem *h, int i, const double *v) {
  const double *xs[1] = {v};
  Timed tm(h, RZ_K_KRYLOV);
  launch_dots(1, xs, xs, h->ndofs, h->partials, rhs_bufs(h, i).dots + kSlotNorm, h->ctx->stream);
}

// one CG iteration of right-hand side i after its V-cycle z = V r: r.z (+ cross),
// p = z + beta p (p = z on the first iteration), Ap, p.Ap, x += alpha p,
// r -= alpha Ap, r.r
rz_status block_iteration_tail(rz_problem *h, int i, BlockRun::Rhs &R) {
  hipStream_t s = h->ctx->stream;
  const int64_t n = h->ndofs;
  const RhsBufs B = rhs_bufs(h, i);
  const bool mixed = h->opts.precision == RZ_PREC_MIXED;
  const int q = R.it & 1;
  double *rz = B.dots + 2 * q, *rz_old = B.dots + 2 * (1 - q);
  {
    Timed tm(h, RZ_K_KRYLOV);
    if (R.it == 0) {
      const double *xs[1] = {B.r}, *ys[1] = {B.z};
      launch_dots(1, xs, ys, n, h->partials, rz, s);
      launch_scale_copy(1.0, B.z, B.p, n, s);
    } else if (mixed) {
      const double *xs[2] = {B.r, B.ro}, *ys[2] = {B.z, B.z};
      launch_dots(2, xs, ys, n, h->partials, rz, s);
      launch_xpby_dev(B.z, rz, rz + 1, rz_old, B.p, n, s);
    } else {
      const double *xs[1] = {B.r}, *ys[1] = {B.z};
      launch_dots(1, xs, ys, n, h->partials, rz, s);
      launch_xpby_dev(B.z, rz, nullptr, rz_old, B.p, n, s);
    }
  }
  if (rz_status e = do_apply64(h, B.p, B.Ap)) return e;
  {
    Timed tm(h, RZ_K_KRYLOV);
    const double *xs[1] = {B.p}, *ys[1] = {B.Ap};
    launch_dots(1, xs, ys, n, h->partials, B.dots + kSlotPap, s);
    launch_cg_update(rz, B.dots + kSlotPap, B.p, B.Ap, R.x, B.r, mixed ? B.ro : nullptr, n, h->partials,
                     B.dots + kSlotRr, s);
  }
  ++R.it;
  return RZ_OK;
}

// Decide what right-hand side i does next from the scalars of the last step.
void block_decide(rz_problem *h, int i, BlockRun::Rhs &R) {
  const double *d = rhs_bufs(h, i).hdots;
  switch (R.enq) {
    case BlockRun::NORM_B:
      R.nb = std::sqrt(d[kSlotNorm]);
      R.tol = h->opts.rtol * R.nb;
      if (!(R.nb > 0)) {
        R.next = BlockRun::FINAL;
      } else if (h->opts.maxit < 1) {
        R.result = RZ_ERR_NOT_CONVERGED;
        R.next = BlockRun::FINAL;
      } else {
        R.next = BlockRun::ITER;
      }
      break;
    case BlockRun::ITER: {
      const double pAp = d[kSlotPap], rr = d[kSlotRr], rzv = d[2 * ((R.it - 1) & 1)];
      // the paper's criterion (Sec. 5.1): the natural norm (r^T M^{-1} r)^{1/2} of the
      // residual that started this iteration, against the first one
      if (R.it == 1) R.rz0 = rzv;
      if (R.it_natural < 0 && R.it > 1 && std::sqrt(std::fabs(rzv)) <= h->opts.rtol * std::sqrt(std::fabs(R.rz0)))
        R.it_natural = R.it - 1;
      if (!(pAp > 0)) {
        R.result = fail(h->ctx, RZ_ERR_BREAKDOWN, "CG breakdown: p.Ap <= 0");
        R.next = BlockRun::FINAL;
      } else if (rzv < 0) {  // CG needs a positive definite preconditioner
        R.result = fail(h->ctx, RZ_ERR_BREAKDOWN, "CG breakdown: r.Mr < 0 (the preconditioner is not positive definite)");
        R.next = BlockRun::FINAL;
      } else if (h->opts.norm == RZ_NORM_NATURAL && R.it_natural >= 0) {  // the paper's criterion
        R.result = RZ_OK;
        R.next = BlockRun::FINAL;
      } else if (h->opts.norm != RZ_NORM_NATURAL && std::sqrt(rr) <= R.tol) {  // check the true residual
        R.next = BlockRun::TRUE_RES;
      } else if (R.it >= h->opts.maxit) {
        R.result = RZ_ERR_NOT_CONVERGED;
        R.next = BlockRun::FINAL;
      } else {
        R.next = BlockRun::ITER;
      }
      break;
    }
    case BlockRun::TRUE_RES: {
      const double tr = std::sqrt(d[kSlotNorm]);
      R.relres = R.nb > 0 ? tr / R.nb : 0.0;
      if (tr <= R.tol) {
        R.result = RZ_OK;
        R.next = BlockRun::DONE;
      } else if (R.it >= h->opts.maxit) {
        R.result = RZ_ERR_NOT_CONVERGED;
        R.next = BlockRun::DONE;
      } else {
        R.restart = true;  // continue from the true residual
        R.next = BlockRun::ITER;
      }
      break;
    }
    case BlockRun::FINAL:
      R.relres = R.nb > 0 ? std::sqrt(d[kSlotNorm]) / R.nb : 0.0;
      R.next = BlockRun::DONE;
      break;
    default:
      break;
  }
  R.enq = BlockRun::NONE;
}

// One CG iteration of the right-hand sides ids (all of the run's, at one iteration
// count it >= 1) from captured HIP graphs: on first use for this parity, vector count,
// set of x vectors and buffer generation, the V-cycle and the iteration tails are
// captured on the context's private stream (nothing runs while capturing), the
// segments are instantiated, and the host counters are put back; then the segments
// are launched on the problem's stream with the cooperative coarse solves between
// them.  done = false (and nothing enqueued) if the capture cannot start.
rz_status graph_iteration(rz_problem *h, BlockRun &B, const std::vector<int> &ids,
                          const std::vector<const double *> &rs, const std::vector<double *> &zs, bool &done) {
  done = false;
  const int nv = (int)ids.size();
  const int par = B.s[ids[0]].it & 1;
  rz_problem::IterGraph &G = h->ig[par];
  std::vector<double *> xs;
  for (int i : ids) xs.push_back(B.s[i].x);
  if (!(G.ok && G.gen == h->graph_gen && G.nv == nv && G.xs == xs)) {
    for (hipGraphExec_t e : G.seg) hipGraphExecDestroy(e);
    G.seg.clear();
    G.ok = false;
    rz_ctx *c = h->ctx;
    if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
      c->cap_stream = nullptr;
      return RZ_OK;
    }
    if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) return RZ_OK;
    const hipStream_t user = c->stream;
    std::vector<int> its;
    for (int i : ids) its.push_back(B.s[i].it);
    std::vector<hipGraph_t> graphs;
    c->stream = c->cap_stream;
    h->cap = &graphs;
    h->cap_bad = false;
    rz_status e = vcycle_multi(h, nv, ids.data(), rs.data(), zs.data());
    for (size_t k = 0; k < ids.size() && !e; ++k) e = block_iteration_tail(h, ids[k], B.s[ids[k]]);
    hipGraph_t last = nullptr;
    const hipError_t ee = hipStreamEndCapture(c->cap_stream, &last);
    c->stream = user;
    h->cap = nullptr;
    for (size_t k = 0; k < ids.size(); ++k) B.s[ids[k]].it = its[k];
    bool ok = !e && ee == hipSuccess && last && !h->cap_bad;
    if (last) graphs.push_back(last);
    for (hipGraph_t g : graphs) {
      hipGraphExec_t x = nullptr;
      if (ok && hipGraphInstantiate(&x, g, nullptr, nullptr, 0) == hipSuccess) G.seg.push_back(x);
      else ok = false;
      hipGraphDestroy(g);
    }
    if (!ok) {
      for (hipGraphExec_t x : G.seg) hipGraphExecDestroy(x);
      G.seg.clear();
      if (e) return e;
      return fail(h->ctx, RZ_ERR_HIP, "capture of the PCG iteration failed");
    }
    G.xs = xs;
    G.nv = nv;
    G.gen = h->graph_gen;
    G.f32 = h->opts.precision != RZ_PREC_F64;
    G.ok = true;
    ++h->graph_stat[0];
    h->graph_stat[2] = (int64_t)G.seg.size();
  }
  hipStream_t s = h->ctx->stream;
  for (size_t k = 0; k < G.seg.size(); ++k) {
    HIPCALL(h, hipGraphLaunch(G.seg[k], s));
    if (k + 1 < G.seg.size() && coarse_coop(h, G.f32))
      return fail(h->ctx, RZ_ERR_HIP, "cooperative launch of the coarse solve failed");
  }
  for (int i : ids) ++B.s[i].it;
  ++h->graph_stat[1];
  done = true;
  return RZ_OK;
}

// Advance every right-hand side by one step (the caller has waited for the
// previous step's work).
rz_status block_step(BlockRun &B) {
  rz_problem *h = B.h;
  hipStream_t s = h->ctx->stream;
  const int64_t n = h->ndofs;
  const int nv = B.nv;
  if (!B.started) {
    B.started = true;
    HIPCALL(h, hipEventCreate(&B.ev0));
    HIPCALL(h, hipEventCreate(&B.ev1));
    HIPCALL(h, hipEventRecord(B.ev0, s));
    B.s.assign(nv, BlockRun::Rhs());
    if (nv > 1) {
      if (rz_status e = ensure_multi(h, nv)) return e;
      launch_deinterleave<double>(B.bu, h->mb, nv, n, n, s);
      for (int i = 0; i < nv; ++i) {
        B.s[i].b = h->mb + (size_t)i * n;
        B.s[i].x = h->mx + (size_t)i * n;
      }
    } else {
      B.s[0].b = B.bu;
      B.s[0].x = B.xu;
    }
    for (int i = 0; i < nv; ++i) {  // x = 0, r = b with Dirichlet rows zero
      const RhsBufs R = rhs_bufs(h, i);
      launch_fill(B.s[i].x, 0.0, n, s);
      v_scale_copy(h, 1.0, B.s[i].b, R.r);
      dir_copy(h, nullptr, R.r, s);
      block_norm(h, i, R.r);
      B.s[i].enq = BlockRun::NORM_B;
    }
  } else {
    for (int i = 0; i < nv; ++i) block_decide(h, i, B.s[i]);
    std::vector<int> ids;
    std::vector<const double *> rs;
    std::vector<double *> zs;
    for (int i = 0; i < nv; ++i) {
      BlockRun::Rhs &R = B.s[i];
      if (R.next != BlockRun::ITER) continue;
      const RhsBufs Bi = rhs_bufs(h, i);
      if (R.restart) v_scale_copy(h, 1.0, Bi.Ap, Bi.r);
      R.restart = false;
      ids.push_back(i);
      rs.push_back(Bi.r);
      zs.push_back(Bi.z);
    }
    if (!ids.empty()) {
      // captured iterations: every right-hand side of the run at one count it >= 1
      bool graph = h->opts.graph && !h->timing && (int)ids.size() == nv && B.s[ids[0]].it >= 1;
      for (int i : ids) graph = graph && B.s[i].it == B.s[ids[0]].it;
      bool done = false;
      if (graph)
        if (rz_status e = graph_iteration(h, B, ids, rs, zs, done)) return e;
      if (!done) {
        if (rz_status e = vcycle_multi(h, (int)ids.size(), ids.data(), rs.data(), zs.data())) return e;
        for (int i : ids)
          if (rz_status e = block_iteration_tail(h, i, B.s[i])) return e;
      }
      for (int i : ids) B.s[i].enq = BlockRun::ITER;
    }
    for (int i = 0; i < nv; ++i) {
      BlockRun::Rhs &R = B.s[i];
      if (R.next != BlockRun::TRUE_RES && R.next != BlockRun::FINAL) continue;
      const RhsBufs Bi = rhs_bufs(h, i);  // the true residual goes to Ap
      if (rz_status e = do_residual64(h, R.b, R.x, Bi.Ap)) return e;
      dir_copy(h, nullptr, Bi.Ap, s);
      block_norm(h, i, Bi.Ap);
      R.enq = R.next;
    }
  }
  bool any = false;
  for (const BlockRun::Rhs &R : B.s) any |= R.enq != BlockRun::NONE;
  if (!any) {
    if (nv > 1) launch_interleave<double>(h->mx, B.xu, nv, n, n, s);
    B.done = true;
    return RZ_OK;
  }
  HIPCALL(h, hipMemcpyAsync(h->hdots, h->dots, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
  if (nv > 1)
    HIPCALL(h, hipMemcpyAsync(h->mhdots, h->mdots, 8 * (size_t)(nv - 1) * sizeof(double), hipMemcpyDeviceToHost, s));
  return RZ_OK;
}

void block_release(BlockRun &B) {
  if (B.ev0) hipEventDestroy(B.ev0);
  if (B.ev1) hipEventDestroy(B.ev1);
  B.ev0 = B.ev1 = nullptr;
}

// Wait for the solve, fill infos (nv entries, may be null) and return the first
// failing status of the right-hand sides.
rz_status block_finish(BlockRun &B, rz_solve_info *infos) {
  rz_problem *h = B.h;
  float ms = 0;
  if (B.ev0) {
    const bool ok = hipEventRecord(B.ev1, h->ctx->stream) == hipSuccess && hipEventSynchronize(B.ev1) == hipSuccess;
    if (ok) hipEventElapsedTime(&ms, B.ev0, B.ev1);
    block_release(B);
    if (!ok) return fail(h->ctx, RZ_ERR_HIP, "stream execution failed during the solve");
  }
  const rz_status dev = take_device_status(h);
  rz_status first = RZ_OK;
  for (int i = 0; i < B.nv; ++i) {
    BlockRun::Rhs &R = B.s[i];
    if (R.result == RZ_OK) R.result = dev;
    if (R.result != RZ_OK && first == RZ_OK) first = R.result;
    if (infos) {
      infos[i].iters = R.it;
      infos[i].status = R.result;
      infos[i].rel_res = R.relres;
      infos[i].omega = h->omega;
      infos[i].t_solve_ms = ms;
      infos[i].iters_natural = R.it_natural;
    }
  }
  return first;
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
  o->aux = RZ_AUX_CELL_AVG;
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
  if (ctx->cap_stream) hipStreamDestroy(ctx->cap_stream);
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
  if (opts->aux != RZ_AUX_CELL_AVG && opts->aux != RZ_AUX_PAPER_DIAG) return fail(ctx, RZ_ERR_ARG, "bad aux");
  if (opts->patch_solver != RZ_PATCH_IC && opts->patch_solver != RZ_PATCH_CHOLESKY)
    return fail(ctx, RZ_ERR_ARG, "bad patch_solver");
  if (opts->norm != RZ_NORM_2 && opts->norm != RZ_NORM_NATURAL) return fail(ctx, RZ_ERR_ARG, "bad norm");
  if (opts->coarse != RZ_COARSE_DIRECT && opts->coarse != RZ_COARSE_HMG) return fail(ctx, RZ_ERR_ARG, "bad coarse");
  if (opts->lanczos_steps < 0 || opts->lanczos_steps > 200) return fail(ctx, RZ_ERR_ARG, "bad lanczos_steps");
  if (opts->coarse == RZ_COARSE_HMG && opts->space != RZ_GRAD && opts->decomposition == RZ_DECOMP_FULL)
    return fail(ctx, RZ_ERR_ARG, "the h-multigrid coarse solver goes with the statically condensed relaxation");
  if (opts->decomposition != RZ_DECOMP_SC && opts->decomposition != RZ_DECOMP_FULL &&
      opts->decomposition != RZ_DECOMP_SC_VERTEX && opts->decomposition != RZ_DECOMP_FULL_PH)
    return fail(ctx, RZ_ERR_ARG, "bad decomposition");
  if (opts->decomposition == RZ_DECOMP_FULL_PH && (opts->space == RZ_GRAD || opts->patch_solver != RZ_PATCH_CHOLESKY))
    return fail(ctx, RZ_ERR_ARG, "RZ_DECOMP_FULL_PH: H(curl)/H(div) with exact star solves (RZ_PATCH_CHOLESKY)");
  if (opts->decomposition == RZ_DECOMP_SC_VERTEX &&
      (opts->space == RZ_GRAD || opts->patch_solver != RZ_PATCH_CHOLESKY))
    return fail(ctx, RZ_ERR_ARG,
                "RZ_DECOMP_SC_VERTEX: H(curl)/H(div) with exact vertex-star solves (RZ_PATCH_CHOLESKY); for H(grad) "
                "RZ_DECOMP_SC is already the condensed vertex-star decomposition");
  if (opts->decomposition == RZ_DECOMP_FULL && opts->space == RZ_GRAD && opts->aux == RZ_AUX_PAPER_DIAG)
    return fail(ctx, RZ_ERR_ARG, "RZ_DECOMP_FULL: H(grad) with the separable auxiliary only");
  if (opts->decomposition == RZ_DECOMP_FULL && opts->space != RZ_GRAD && opts->patch_solver != RZ_PATCH_CHOLESKY)
    return fail(ctx, RZ_ERR_ARG, "RZ_DECOMP_FULL on H(curl)/H(div): exact vertex-star solves (RZ_PATCH_CHOLESKY) only");
  if (opts->patch_solver == RZ_PATCH_CHOLESKY && opts->space != RZ_GRAD && opts->decomposition == RZ_DECOMP_SC)
    return fail(ctx, RZ_ERR_ARG,
                "RZ_PATCH_CHOLESKY: H(grad) vertex stars, or the H(curl)/H(div) stars (RZ_DECOMP_FULL, "
                "RZ_DECOMP_SC_VERTEX, RZ_DECOMP_FULL_PH)");
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
    if (opts->aux == RZ_AUX_PAPER_DIAG && opts->space == RZ_GRAD) {
      if (!paper_diagonals_all(h)) {
        delete h;
        return fail(ctx, RZ_ERR_ARG, "non-positive Jacobian determinant or coefficient at a quadrature point");
      }
      h->pd = true;
    }
  }
  if (opts->space != RZ_GRAD) return setup_vector(h, cf, out);
  grad_symbolic(h);
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
  if (h->pd && (e = upload_paper_diagonals(h))) return bail(e);
  if ((e = grad_patch_device(h))) return bail(e);
  if (h->opts.decomposition == RZ_DECOMP_FULL) {
    if ((e = setup_full_stars(h))) return bail(e);
  } else if (h->opts.patch_solver == RZ_PATCH_CHOLESKY && (e = setup_patch_cholesky(h))) {
    return bail(e);
  }
  const int n1 = p + 1;
  if ((e = upload(h, &h->E64, h->t.E))) return bail(e);
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
  const size_t neb = (size_t)h->ncells * (p + 1) * (p + 1) * (p + 1);
  if ((e = dalloc(h, &h->eb64, neb)) || (e = dalloc(h, &h->eb32, neb)) || (e = dalloc(h, &h->rt64, h->ndofs)) ||
      (e = dalloc(h, &h->rt32, h->ndofs)) || (e = alloc_krylov(h)))
    return bail(e);
  if ((e = dalloc(h, &h->rt1, (size_t)(h->nx + 1) * h->Ny * h->Nz)) ||
      (e = dalloc(h, &h->rt2, (size_t)(h->nx + 1) * (h->ny + 1) * h->Nz)) ||
      (e = dalloc(h, &h->rc, (size_t)(h->nx + 1) * (h->ny + 1) * (h->nz + 1))) ||
      (e = dalloc(h, &h->xc, (size_t)(h->nx + 1) * (h->ny + 1) * (h->nz + 1))))
    return bail(e);
  if ((e = setup_coarse(h))) return bail(e);
  if (!patch_solve_uses_regs(h->PE, p, 8) && (e = autotune_patch_solve<double>(h, h->f64, h->rt64, h->zb64, 0)))
    return bail(e);
  if (!patch_solve_uses_regs(h->PE, p, 4) && (e = autotune_patch_solve<float>(h, h->f32, h->rt32, h->zb32, 1)))
    return bail(e);
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
  if (h->space != RZ_GRAD) {
    const int nx = h->nx, ny = h->ny, nz = h->nz;
    sizes[0] = h->ndofs;
    sizes[1] = h->nfree;
    sizes[2] = h->ncells;
    // star patches of the relaxation: edges (curl) or faces (div)
    sizes[3] = h->space == RZ_CURL ? (int64_t)nx * (ny + 1) * (nz + 1) + (int64_t)(nx + 1) * ny * (nz + 1) +
                                         (int64_t)(nx + 1) * (ny + 1) * nz
                                   : (int64_t)(nx + 1) * ny * nz + (int64_t)nx * (ny + 1) * nz +
                                         (int64_t)nx * ny * (nz + 1);
    // p = 1 lattice DoFs
    sizes[4] = h->space == RZ_CURL ? sizes[3] : sizes[3];
    sizes[5] = h->ed.fac_stride;     // curl: factor values of one edge patch
    sizes[6] = h->edge_nslot;        // slots of one edge patch (curl; div: its potential)
    sizes[7] = (int64_t)h->edge_ids.size();  // non-empty edge patches
    return RZ_OK;
  }
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

rz_status rz_apply(rz_problem *h, const void *x, void *y, rz_dtype t, int32_t nrhs) {
  rz_status e = require_device(h);
  if (e) return e;
  if (!x || !y || x == y || nrhs < 1) return fail(h->ctx, RZ_ERR_ARG, "rz_apply: bad vectors");
  if (t != RZ_F64 && t != RZ_F32 && t != RZ_BF16) return fail(h->ctx, RZ_ERR_ARG, "rz_apply: bad dtype");
  if (t == RZ_BF16 && h->space != RZ_GRAD) return fail(h->ctx, RZ_ERR_ARG, "rz_apply: BF16 vectors are H(grad) only");
  if (nrhs == 1) {
    if (t == RZ_F64) return do_apply64(h, static_cast<const double *>(x), static_cast<double *>(y));
    if (t == RZ_BF16) return do_apply_bf16(h, static_cast<const uint16_t *>(x), static_cast<uint16_t *>(y));
    return do_apply32(h, static_cast<const float *>(x), static_cast<float *>(y));
  }
  if ((e = ensure_multi(h, nrhs))) return e;
  hipStream_t s = h->ctx->stream;
  const int64_t n = h->ndofs;
  if (t == RZ_BF16) {
    uint16_t *xb = reinterpret_cast<uint16_t *>(h->mb), *yb = reinterpret_cast<uint16_t *>(h->mx);
    launch_deinterleave<unsigned short>(static_cast<const uint16_t *>(x), xb, nrhs, n, n, s);
    for (int r = 0; r < nrhs; ++r)
      if ((e = do_apply_bf16(h, xb + (size_t)r * n, yb + (size_t)r * n))) return e;
    launch_interleave<unsigned short>(yb, static_cast<uint16_t *>(y), nrhs, n, n, s);
  } else if (t == RZ_F64) {
    launch_deinterleave<double>(static_cast<const double *>(x), h->mb, nrhs, n, n, s);
    for (int r = 0; r < nrhs; ++r)
      if ((e = do_apply64(h, h->mb + (size_t)r * n, h->mx + (size_t)r * n))) return e;
    launch_interleave<double>(h->mx, static_cast<double *>(y), nrhs, n, n, s);
  } else {
    float *xb = reinterpret_cast<float *>(h->mb), *yb = reinterpret_cast<float *>(h->mx);
    launch_deinterleave<float>(static_cast<const float *>(x), xb, nrhs, n, n, s);
    for (int r = 0; r < nrhs; ++r)
      if ((e = do_apply32(h, xb + (size_t)r * n, yb + (size_t)r * n))) return e;
    launch_interleave<float>(yb, static_cast<float *>(y), nrhs, n, n, s);
  }
  return RZ_OK;
}

// Bytes of the apply's workspace (face-line buffer of the Cartesian H(grad) path,
// per-cell outputs of the quadrature path, per-entry contributions of the other
// cells sharing an entry in the vector-space paths: three per entry for H(curl),
// one for H(div)) for element size sz.
static size_t apply_workspace_bytes(const rz_problem *h, size_t sz) {
  if (h->space != RZ_GRAD) return (size_t)h->ndofs * (h->space == RZ_CURL ? 3 : 1) * sz;
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

rz_status rz_relax(rz_problem *h, const void *r, void *z, rz_dtype t, int32_t nrhs) {
  rz_status e = require_device(h);
  if (e) return e;
  if (!r || !z || r == z || nrhs < 1) return fail(h->ctx, RZ_ERR_ARG, "rz_relax: bad vectors");
  if (t != RZ_F64 && t != RZ_F32) return fail(h->ctx, RZ_ERR_ARG, "rz_relax: bad dtype");
  if (nrhs == 1) {
    if (t == RZ_F64) return do_relax64(h, static_cast<const double *>(r), static_cast<double *>(z));
    return do_relax32(h, static_cast<const float *>(r), static_cast<float *>(z));
  }
  if ((e = ensure_multi(h, nrhs))) return e;
  hipStream_t s = h->ctx->stream;
  const int64_t n = h->ndofs;
  std::vector<int> ids(nrhs);
  for (int i = 0; i < nrhs; ++i) ids[i] = i;
  auto run = [&](auto *rb, auto *zb) -> rz_status {
    using T = std::remove_pointer_t<decltype(rb)>;
    launch_deinterleave<T>(static_cast<const T *>(r), rb, nrhs, n, n, s);
    std::vector<const T *> rs(nrhs);
    std::vector<T *> zs(nrhs);
    for (int i = 0; i < nrhs; ++i) {
      rs[i] = rb + (size_t)i * n;
      zs[i] = zb + (size_t)i * n;
    }
    if (rz_status e2 = relax_multi<T>(h, nrhs, ids.data(), rs.data(), zs.data(), T(1), T(0), nullptr, [](int) {}))
      return e2;
    launch_interleave<T>(zb, static_cast<T *>(z), nrhs, n, n, s);
    return RZ_OK;
  };
  if (t == RZ_F64) return run(h->mb, h->mx);
  return run(reinterpret_cast<float *>(h->mb), reinterpret_cast<float *>(h->mx));
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

rz_status rz_vcycle(rz_problem *h, const double *r, double *z, int32_t nrhs) {
  rz_status e = require_device(h);
  if (e) return e;
  if (!r || !z || r == z || nrhs < 1) return fail(h->ctx, RZ_ERR_ARG, "rz_vcycle: bad vectors");
  if (nrhs == 1) return do_vcycle(h, r, z);
  if ((e = ensure_multi(h, nrhs))) return e;
  hipStream_t s = h->ctx->stream;
  const int64_t n = h->ndofs;
  launch_deinterleave<double>(r, h->mb, nrhs, n, n, s);
  std::vector<int> ids(nrhs);
  std::vector<const double *> rs(nrhs);
  std::vector<double *> zs(nrhs);
  for (int i = 0; i < nrhs; ++i) {
    ids[i] = i;
    rs[i] = h->mb + (size_t)i * n;
    zs[i] = h->mx + (size_t)i * n;
  }
  if ((e = vcycle_multi(h, nrhs, ids.data(), rs.data(), zs.data()))) return e;
  launch_interleave<double>(h->mx, z, nrhs, n, n, s);
  return RZ_OK;
}

rz_status rz_solve(rz_problem *h, const double *b, double *x, int32_t nrhs, rz_solve_info *info) {
  rz_status e = require_device(h);
  if (e) return e;
  if (!b || !x || b == x || nrhs < 1) return fail(h->ctx, RZ_ERR_ARG, "rz_solve: bad vectors");
  if (h->opts.precision == RZ_PREC_DEFECT) {
    if (nrhs == 1) return defect_solve(h, b, x, info);
    // one right-hand side after another (planar copies)
    if ((e = ensure_multi(h, nrhs))) return e;
    hipStream_t s = h->ctx->stream;
    const int64_t n = h->ndofs;
    launch_deinterleave<double>(b, h->mb, nrhs, n, n, s);
    rz_status first = RZ_OK;
    for (int i = 0; i < nrhs; ++i) {
      rz_status r = defect_solve(h, h->mb + (size_t)i * n, h->mx + (size_t)i * n, info ? info + i : nullptr);
      if (r == RZ_ERR_HIP || r == RZ_ERR_ARG || r == RZ_ERR_OOM) return r;
      if (r != RZ_OK && first == RZ_OK) first = r;
    }
    launch_interleave<double>(h->mx, x, nrhs, n, n, s);
    HIPCALL(h, hipStreamSynchronize(s));
    return first;
  }
  BlockRun B;
  B.h = h;
  B.nv = nrhs;
  B.bu = b;
  B.xu = x;
  while (!B.done) {
    if ((e = block_step(B))) {
      block_release(B);
      return e;
    }
    if (hipStreamSynchronize(h->ctx->stream) != hipSuccess) {
      block_release(B);
      return fail(h->ctx, RZ_ERR_HIP, "stream execution failed during the solve");
    }
  }
  return block_finish(B, info);
}

rz_status rz_solve_batched(rz_problem *const *hs, int32_t n, const double *const *b, double *const *x, int32_t nrhs,
                           rz_solve_info *infos) {
  if (!hs || !b || !x || n < 0 || nrhs < 1) return RZ_ERR_ARG;
  for (int i = 0; i < n; ++i) {
    if (!hs[i] || !b[i] || !x[i] || b[i] == x[i]) return RZ_ERR_ARG;
    rz_status e = require_device(hs[i]);
    if (e) return e;
    if (hs[i]->opts.precision == RZ_PREC_DEFECT)
      return fail(hs[i]->ctx, RZ_ERR_ARG, "rz_solve_batched: the defect-correction protocol is not batched");
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(hs[i]->ctx, RZ_ERR_ARG, "rz_solve_batched: a problem appears twice");
  }
  // One block run per problem (its right-hand sides in lockstep).  Each enqueued
  // step ends with an event; the host advances every run whose event has completed,
  // so problems on different streams progress independently and the device works
  // on one while the host serves another.
  std::vector<BlockRun> run(n);
  std::vector<rz_status> st(n, RZ_OK);
  std::vector<hipEvent_t> ev(n, nullptr);
  std::vector<char> pending(n, 0), finished(n, 0);
  rz_status first_fail = RZ_OK;  // first non-OK result of a finished solve
  for (int i = 0; i < n; ++i) {
    run[i].h = hs[i];
    run[i].nv = nrhs;
    run[i].bu = b[i];
    run[i].xu = x[i];
    if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess) {
      for (int j = 0; j < i; ++j) hipEventDestroy(ev[j]);
      return fail(hs[i]->ctx, RZ_ERR_HIP, "rz_solve_batched: event creation");
    }
  }
  auto live = [&](int i) { return !finished[i] && st[i] == RZ_OK; };
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
      if (run[i].done) {
        const rz_status r = block_finish(run[i], infos ? infos + (int64_t)i * nrhs : nullptr);
        if (r != RZ_OK && first_fail == RZ_OK) first_fail = r;  // keep solving the others
        finished[i] = 1;
        continue;
      }
      if (rz_status e = block_step(run[i])) {
        st[i] = e;
        continue;
      }
      if (hipEventRecord(ev[i], hs[i]->ctx->stream) != hipSuccess) {
        st[i] = fail(hs[i]->ctx, RZ_ERR_HIP, "event record");
        continue;
      }
      pending[i] = 1;
    }
    active = 0;
    for (int i = 0; i < n; ++i) active += live(i);
    if (!progressed && active > 0) std::this_thread::yield();
  }
  for (int i = 0; i < n; ++i) {
    hipEventDestroy(ev[i]);
    block_release(run[i]);  // runs stopped by an error still hold their events
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
  launch_patch_factor(h->L, h->P, h->coef64, h->B64, h->A64, h->lam64, pd_dev(h), h->f64, h->f32, h->status, s);
  HIPCALL(h, hipMemcpyAsync(breakdown, h->status, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCALL(h, hipStreamSynchronize(s));
  if (!*breakdown && h->nrf) return setup_full_stars(h);
  if (!*breakdown && h->cw64) return setup_patch_cholesky(h);
  return RZ_OK;
}
}  // namespace

rz_status rz_set_aux(rz_problem *h, const double *coef6) {
  if (h) ++h->graph_gen;  // the graphs of captured iterations may name replaced buffers
  if (h && h->pd) return fail(h->ctx, RZ_ERR_ARG, "rz_set_aux: the problem uses the paper's auxiliary (RZ_AUX_PAPER_DIAG)");
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
    case RZ_EXPORT_GRAPHS:
      put(h->graph_stat, sizeof h->graph_stat);
      break;
    case RZ_EXPORT_HMG:
      if (!h->hmg_on) return fail(h->ctx, RZ_ERR_ARG, "no h-multigrid coarse solver on this problem");
      put(h->hmg_sizes.data(), sizeof(int64_t) * h->hmg_sizes.size());
      break;
    case RZ_EXPORT_AUTOTUNE: {
      for (int w = 0; w < 2; ++w) {
        const double n = (double)h->tune[w].size();
        put(&n, sizeof n);
        for (auto &q : h->tune[w]) {
          const double c = q.first, t = q.second;
          put(&c, sizeof c);
          put(&t, sizeof t);
        }
        const double chosen = h->PE.cap[w];
        put(&chosen, sizeof chosen);
      }
      break;
    }
    case RZ_EXPORT_PAPER_DIAG: {
      if (!h->pd) return fail(h->ctx, RZ_ERR_ARG, "rz_export: the problem does not use RZ_AUX_PAPER_DIAG");
      if (index < 0 || index >= h->ncells) return fail(h->ctx, RZ_ERR_ARG, "rz_export: bad cell");
      const size_t nm = (size_t)n1 * n1 * n1, na = 3 * (size_t)p * n1 * n1;
      std::vector<double> v(nm + na);
      HIPCALL(h, hipStreamSynchronize(h->ctx->stream));
      HIPCALL(h, hipMemcpy(v.data(), h->pd_dm + nm * index, nm * sizeof(double), hipMemcpyDeviceToHost));
      HIPCALL(h, hipMemcpy(v.data() + nm, h->pd_da + na * index, na * sizeof(double), hipMemcpyDeviceToHost));
      put(v.data(), v.size() * sizeof(double));
      break;
    }
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
    case RZ_EXPORT_STATS: {
      // H(grad): lower non-zeros (diagonal included) and rows of the IC factors of all
      // non-empty vertex patches, without padding or the identity rows of absent DoFs
      if (h->space != RZ_GRAD) return fail(h->ctx, RZ_ERR_ARG, "statistics of vertex patches: H(grad) only");
      int64_t nnz = 0, rows = 0;
      const int nvx = h->nx + 1, nvy = h->ny + 1;
      for (int64_t vid : h->patch_vids) {
        const int V[3] = {(int)(vid % nvx), (int)((vid / nvx) % nvy), (int)(vid / ((int64_t)nvx * nvy))};
        const int nc[3] = {h->nx, h->ny, h->nz};
        bool inner = true;
        for (int d = 0; d < 3; ++d) inner = inner && V[d] >= 1 && V[d] <= nc[d] - 1;
        if (inner) {  // a full star away from the boundary: every row, the whole pattern
          nnz += h->ps.nnz;
          rows += h->ps.nrows;
          continue;
        }
        std::vector<int> pres(h->ps.nrows, 0);
        std::vector<std::array<int, 3>> G(h->ps.nrows);
        for (int k = 0; k < h->ps.nrows; ++k) {
          int g3[3];
          if (patch_row_present(h, vid, k, g3)) {
            pres[k] = 1;
            G[k] = {g3[0], g3[1], g3[2]};
            ++rows;
          }
        }
        for (int r = 0; r < h->ps.nrows; ++r) {
          if (!pres[r]) continue;
          for (int k = h->ps.rowptr[r]; k < h->ps.rowptr[r + 1]; ++k) {
            const int c = h->ps.col[k];
            if (!pres[c]) continue;
            if (r == c || patch_entry_allowed(h, vid, G[r].data(), G[c].data())) ++nnz;
          }
        }
      }
      const int64_t v[2] = {nnz, rows};
      put(v, sizeof v);
      break;
    }
    case RZ_EXPORT_EDGE_PATCH: {
      if (h->space == RZ_GRAD) return fail(h->ctx, RZ_ERR_ARG, "edge patches exist for H(curl) / H(div) only");
      if (index < 0 || index >= (int64_t)h->edge_ids.size()) return fail(h->ctx, RZ_ERR_ARG, "bad patch index");
      std::vector<int64_t> v;
      for (int k = 0; k < h->edge_nslot; ++k) {
        const int g = h->edge_idx[(size_t)index * h->edge_nslot + k];
        if (g >= 0) v.push_back(g);
      }
      std::sort(v.begin(), v.end());
      put(&h->edge_ids[index], sizeof(int64_t));
      put(v.data(), sizeof(int64_t) * v.size());
      break;
    }
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

rz_status rz_set_graph(rz_problem *h, int on) {
  rz_status e = require_device(h);
  if (e) return e;
  h->opts.graph = on != 0;
  if (!on) {
    HIPCALL(h, hipStreamSynchronize(h->ctx->stream));
    graphs_release(h);
  }
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

// ---------------------------------------------------------------------------------------
// Mixed Hodge Laplacians (Sec. 5.3): find (sigma, u) in V^{k-1} x V^k, no essential
// boundary, with the block operator
//   K = [ -M_{k-1}  D^T M_k ; M_k D  S_k ]
// (M_j the beta-weighted mass of V^j, S_k the alpha-weighted (d v, d u), D = d^{k-1}
// in FDM coefficients), preconditioned by blockdiag(C_{k-1}, C_k), C_j a fixed number
// of Chebyshev steps on the Riesz map A_j = M_j + S_j preconditioned by its V-cycle
// (for V^3 = DQ_{p-1}: by point Jacobi of its diagonal mass), and solved by MINRES.
// ---------------------------------------------------------------------------------------
struct rz_hodge {
  rz_ctx *ctx = nullptr;
  int k = 0, steps = 4;
  rz_problem *lo = nullptr, *hi = nullptr;  // hi == nullptr for k = 3
  int64_t nlo = 0, nhi = 0;
  double eig_lo[2] = {0, 0}, eig_hi[2] = {1, 1};
  std::vector<void *> allocs;
  // mass-only and stiffness-only cell weights of the two problems
  double *cm_lo = nullptr, *cm_hi = nullptr, *cs_hi = nullptr;
  // D and D^T in CSR (int32 offsets)
  int *d_ptr = nullptr, *d_col = nullptr, *dt_ptr = nullptr, *dt_col = nullptr;
  double *d_val = nullptr, *dt_val = nullptr;
  // DQ_{p-1}: mass diagonal, Chebyshev-scaled inverse, identity row list
  double *m3 = nullptr, *m3c = nullptr;
  int *rows3 = nullptr;
  double *partials = nullptr, *dots = nullptr;
  // block temporaries and the MINRES vectors (length nlo + nhi)
  double *tlo = nullptr, *thi = nullptr, *shi = nullptr;
  double *cr = nullptr, *cd = nullptr, *ct = nullptr, *cz = nullptr;  // Chebyshev (max block length)
  double *mv[10] = {};
};

namespace {

template <typename T>
rz_status hg_alloc(rz_hodge *g, T **ptr, size_t count) {
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, sizeof(T) * (count ? count : 1));
  if (e != hipSuccess) return fail(g->ctx, RZ_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  g->allocs.push_back(p);
  *ptr = static_cast<T *>(p);
  return RZ_OK;
}

template <typename T>
rz_status hg_upload(rz_hodge *g, T **ptr, const std::vector<T> &v) {
  if (rz_status e = hg_alloc(g, ptr, v.size())) return e;
  hipError_t e = hipMemcpyAsync(*ptr, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, g->ctx->stream);
  if (e != hipSuccess) return fail(g->ctx, RZ_ERR_HIP, hipGetErrorString(e));
  return RZ_OK;
}

// Per-axis kinds of component m of the space of form degree k (k = 3: DQ_{p-1}):
// true = continuous (p n + 1 points), false = broken (p n values)
bool hg_cont(int k, int m, int a) {
  if (k == 0) return true;
  if (k == 1) return a != m;
  if (k == 2) return a == m;
  return false;
}
int hg_ncomp(int k) { return (k == 0 || k == 3) ? 1 : 3; }

struct HgLat {
  int k, p, n[3];
  int64_t off[3], ext[3][3];
  int64_t ndofs;
  HgLat(int k_, int p_, const int nn[3]) : k(k_), p(p_) {
    for (int a = 0; a < 3; ++a) n[a] = nn[a];
    int64_t o = 0;
    for (int m = 0; m < hg_ncomp(k); ++m) {
      off[m] = o;
      int64_t sz = 1;
      for (int a = 0; a < 3; ++a) {
        ext[m][a] = (int64_t)n[a] * p + (hg_cont(k, m, a) ? 1 : 0);
        sz *= ext[m][a];
      }
      o += sz;
    }
    ndofs = o;
  }
  int64_t index(int m, const int64_t X[3]) const { return off[m] + X[0] + ext[m][0] * (X[1] + ext[m][1] * X[2]); }
};

// d^{k-1}: V^{k-1} -> V^k on the lattice.  A derivative along axis a takes the
// continuous index of the source to the broken index X_a = c p + i of the target
// with the 1-D weights D[i][j] (the FDM derivative table); the other axes keep
// their index.  grad: component m = d_m u; curl: component m = d_{m+1} u_{m+2} -
// d_{m+2} u_{m+1} (indices mod 3); div: sum_m d_m u_m.
void hg_derivative(int k, int p, const int nn[3], const std::vector<double> &Dt, std::vector<int> &ptr,
                   std::vector<int> &col, std::vector<double> &val) {
  HgLat src(k - 1, p, nn), dst(k, p, nn);
  ptr.assign(1, 0);
  col.clear();
  val.clear();
  for (int m = 0; m < hg_ncomp(k); ++m) {
    // terms (sign, derivative axis, source component)
    struct Term { double sign; int axis, comp; };
    std::vector<Term> terms;
    if (k == 1) terms = {{1.0, m, 0}};
    else if (k == 2) terms = {{1.0, (m + 1) % 3, (m + 2) % 3}, {-1.0, (m + 2) % 3, (m + 1) % 3}};
    else terms = {{1.0, 0, 0}, {1.0, 1, 1}, {1.0, 2, 2}};
    int64_t X[3];
    for (X[2] = 0; X[2] < dst.ext[m][2]; ++X[2])
      for (X[1] = 0; X[1] < dst.ext[m][1]; ++X[1])
        for (X[0] = 0; X[0] < dst.ext[m][0]; ++X[0]) {
          for (const Term &t : terms) {
            const int64_t c = X[t.axis] / p, i = X[t.axis] % p;
            int64_t Y[3] = {X[0], X[1], X[2]};
            for (int j = 0; j <= p; ++j) {
              const double w = Dt[i * (p + 1) + j];
              if (w == 0.0) continue;
              Y[t.axis] = c * p + j;
              col.push_back((int)src.index(t.comp, Y));
              val.push_back(t.sign * w);
            }
          }
          ptr.push_back((int)col.size());
        }
  }
}

void hg_transpose(int64_t nrows, int64_t ncols, const std::vector<int> &ptr, const std::vector<int> &col,
                  const std::vector<double> &val, std::vector<int> &tp, std::vector<int> &tc, std::vector<double> &tv) {
  tp.assign(ncols + 1, 0);
  for (int c : col) tp[c + 1]++;
  for (int64_t i = 0; i < ncols; ++i) tp[i + 1] += tp[i];
  tc.resize(col.size());
  tv.resize(val.size());
  std::vector<int> pos(tp.begin(), tp.end() - 1);
  for (int64_t r = 0; r < nrows; ++r)
    for (int q = ptr[r]; q < ptr[r + 1]; ++q) {
      tc[pos[col[q]]] = (int)r;
      tv[pos[col[q]]++] = val[q];
    }
}

// y = M x (mass) or S x (stiffness) of problem h with the weights w
void hg_apply_w(rz_problem *h, const double *w, const double *x, double *y) {
  Timed t(h, RZ_K_APPLY);
  if (h->space != RZ_GRAD)
    launch_apply_vec<double>(h->V, w, h->B64, h->D64, x, y, h->eb64, h->ctx->stream);
  else
    launch_apply_grad<double>(h->L, w, h->t.B.data(), h->t.A.data(), x, nullptr, y, h->eb64, h->ctx->stream);
}

rz_status hg_dot(rz_hodge *g, const double *x, const double *y, int64_t n, double *out) {
  hipStream_t s = g->ctx->stream;
  const double *xs[1] = {x}, *ys[1] = {y};
  launch_dots(1, xs, ys, n, g->partials, g->dots, s);
  hipError_t e = hipMemcpyAsync(out, g->dots, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(g->ctx, RZ_ERR_HIP, hipGetErrorString(e));
  return RZ_OK;
}

// y = K x on [sigma; u]
rz_status hg_apply(rz_hodge *g, const double *x, double *y) {
  hipStream_t s = g->ctx->stream;
  const double *xs = x, *xu = x + g->nlo;
  double *ys = y, *yu = y + g->nlo;
  const int nlo = (int)g->nlo, nhi = (int)g->nhi;
  // t_hi = M_k u ; y_sigma = D^T t_hi - M_{k-1} sigma
  if (g->hi) hg_apply_w(g->hi, g->cm_hi, xu, g->thi);
  else launch_rows_scale<double>(nhi, g->rows3, g->m3, xu, g->thi, s);
  launch_csr<double, double, double>(nlo, nullptr, g->dt_ptr, g->dt_col, g->dt_val, g->thi, ys, 0, s);
  hg_apply_w(g->lo, g->cm_lo, xs, g->tlo);
  launch_axpy(-1.0, g->tlo, ys, g->nlo, s);
  // y_u = M_k D sigma + S_k u
  launch_csr<double, double, double>(nhi, nullptr, g->d_ptr, g->d_col, g->d_val, xs, g->shi, 0, s);
  if (g->hi) {
    hg_apply_w(g->hi, g->cm_hi, g->shi, yu);
    hg_apply_w(g->hi, g->cs_hi, xu, g->thi);
    launch_axpy(1.0, g->thi, yu, g->nhi, s);
  } else {
    launch_rows_scale<double>(nhi, g->rows3, g->m3, g->shi, yu, s);
  }
  return RZ_OK;
}

// x = steps Chebyshev iterations on A x = f (problem h's Riesz map, its V-cycle as
// the preconditioner) for the spectrum [lmin, lmax] of B A, from x = 0
rz_status hg_cheb(rz_hodge *g, rz_problem *h, double lmin, double lmax, const double *f, double *x) {
  hipStream_t s = g->ctx->stream;
  const int64_t n = h->ndofs;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
  double rho = 1.0 / sigma;
  if (rz_status e = do_vcycle(h, f, g->cz)) return e;
  launch_scale_copy(1.0 / theta, g->cz, g->cd, n, s);  // d = B f / theta
  hipError_t he = hipMemcpyAsync(g->cr, f, sizeof(double) * n, hipMemcpyDeviceToDevice, s);
  if (he != hipSuccess) return fail(g->ctx, RZ_ERR_HIP, hipGetErrorString(he));
  for (int j = 0; j < g->steps; ++j) {
    if (j == 0) launch_scale_copy(1.0, g->cd, x, n, s);
    else launch_axpy(1.0, g->cd, x, n, s);
    if (j + 1 == g->steps) break;
    // r <- r - A d, fused into the apply's stores (into the spare buffer, then swapped)
    if (rz_status e = do_residual64(h, g->cr, g->cd, g->ct)) return e;
    std::swap(g->cr, g->ct);
    const double rho_next = 1.0 / (2.0 * sigma - rho);
    if (rz_status e = do_vcycle(h, g->cr, g->cz)) return e;
    launch_scale_copy(rho_next * rho, g->cd, g->cd, n, s);
    launch_axpy(2.0 * rho_next / delta, g->cz, g->cd, n, s);
    rho = rho_next;
  }
  return RZ_OK;
}

// z = blockdiag(C_{k-1}, C_k) r
rz_status hg_precond(rz_hodge *g, const double *r, double *z) {
  if (rz_status e = hg_cheb(g, g->lo, 0.9 * g->eig_lo[0], 1.1 * g->eig_lo[1], r, z)) return e;
  if (g->hi) return hg_cheb(g, g->hi, 0.9 * g->eig_hi[0], 1.1 * g->eig_hi[1], r + g->nlo, z + g->nlo);
  // L^2: B A = I, so the steps reduce to z = q M^{-1} r with q = 1 - p(1) for the
  // Chebyshev polynomial p of the interval [0.9, 1.1] (m3c holds q / diag)
  launch_rows_scale<double>((int)g->nhi, g->rows3, g->m3c, r + g->nlo, z + g->nlo, g->ctx->stream);
  return RZ_OK;
}

// extreme eigenvalues of (V-cycle) A from the Lanczos tridiagonal of 10 preconditioned CG
// steps from the SplitMix64 start vector of the problem's lanczos_seed
rz_status hg_extremes(rz_hodge *g, rz_problem *h, double out[2]) {
  hipStream_t s = g->ctx->stream;
  const int64_t n = h->ndofs;
  std::vector<double> v0(n);
  uint64_t st = h->opts.lanczos_seed;
  for (int64_t i = 0; i < n; ++i) v0[i] = 2.0 * ((double)(splitmix_next(st) >> 11) * 0x1.0p-53) - 1.0;
  double *r = g->cr, *z = g->cz, *d = g->cd, *Ad = g->ct;
  hipError_t he = hipMemcpyAsync(r, v0.data(), sizeof(double) * n, hipMemcpyHostToDevice, s);
  if (he != hipSuccess) return fail(g->ctx, RZ_ERR_HIP, hipGetErrorString(he));
  if (rz_status e = do_vcycle(h, r, z)) return e;
  launch_scale_copy(1.0, z, d, n, s);
  double rz_;
  if (rz_status e = hg_dot(g, r, z, n, &rz_)) return e;
  std::vector<double> diag, off;
  double a_prev = 0, b_prev = 0;
  for (int it = 0; it < 10; ++it) {
    if (rz_status e = do_apply64(h, d, Ad)) return e;
    double dAd;
    if (rz_status e = hg_dot(g, d, Ad, n, &dAd)) return e;
    if (!(dAd > 0)) break;
    const double a = rz_ / dAd;
    launch_axpy(-a, Ad, r, n, s);
    if (rz_status e = do_vcycle(h, r, z)) return e;
    double rzn;
    if (rz_status e = hg_dot(g, r, z, n, &rzn)) return e;
    const double b = rzn / rz_;
    diag.push_back(1.0 / a + (it > 0 ? b_prev / a_prev : 0.0));
    off.push_back(std::sqrt(b) / a);
    a_prev = a;
    b_prev = b;
    rz_ = rzn;
    launch_xpby(z, b, d, n, s);
    if (!(rzn > 0)) break;
  }
  if (diag.empty()) return fail(g->ctx, RZ_ERR_BREAKDOWN, "rz_hodge: Lanczos estimate failed");
  off.resize(diag.size() > 1 ? diag.size() - 1 : 1, 0.0);
  if (diag.size() == 1) off[0] = 0.0;
  std::vector<double> neg(diag.size());
  for (size_t i = 0; i < diag.size(); ++i) neg[i] = -diag[i];
  out[1] = tridiag_max_eig(diag, off);
  out[0] = -tridiag_max_eig(neg, off);
  return RZ_OK;
}

}  // namespace

extern "C" {

rz_status rz_hodge_create(int32_t k, rz_problem *lo, rz_problem *hi, int32_t cheb_steps, rz_hodge **out) {
  if (!out) return RZ_ERR_ARG;
  *out = nullptr;
  rz_status e = require_device(lo);
  if (e) return e;
  rz_ctx *ctx = lo->ctx;
  if (k < 1 || k > 3) return fail(ctx, RZ_ERR_ARG, "rz_hodge_create: k must be 1, 2 or 3");
  if (cheb_steps < 1 || cheb_steps > 64) return fail(ctx, RZ_ERR_ARG, "rz_hodge_create: cheb_steps in 1..64");
  if ((k == 3) != (hi == nullptr)) return fail(ctx, RZ_ERR_ARG, "rz_hodge_create: hi is null exactly for k = 3");
  if (lo->space != k - 1 || (hi && hi->space != k))
    return fail(ctx, RZ_ERR_ARG, "rz_hodge_create: lo must be the space of form degree k-1, hi of degree k");
  for (rz_problem *h : {lo, hi}) {
    if (!h) continue;
    if (h->ctx != ctx) return fail(ctx, RZ_ERR_ARG, "rz_hodge_create: problems on different contexts");
    if (h->dir != 0) return fail(ctx, RZ_ERR_ARG, "rz_hodge_create: no essential boundary (dirichlet = 0) expected");
    if (h->quad) return fail(ctx, RZ_ERR_ARG, "rz_hodge_create: Cartesian cells with cellwise coefficients only");
    if (h->opts.precision == RZ_PREC_DEFECT || h->opts.decomposition != RZ_DECOMP_SC)
      return fail(ctx, RZ_ERR_ARG,
                  "rz_hodge_create: FP64 or mixed-protocol problems with the condensed decomposition expected");
    if (h->p != lo->p || h->nx != lo->nx || h->ny != lo->ny || h->nz != lo->nz)
      return fail(ctx, RZ_ERR_ARG, "rz_hodge_create: lo and hi on different meshes or degrees");
  }
  if (lo->p < 1) return fail(ctx, RZ_ERR_ARG, "rz_hodge_create: degree");
  auto *g = new rz_hodge;
  g->ctx = ctx;
  g->k = k;
  g->steps = cheb_steps;
  g->lo = lo;
  g->hi = hi;
  g->nlo = lo->ndofs;
  const int nn[3] = {lo->nx, lo->ny, lo->nz};
  g->nhi = hi ? hi->ndofs : (int64_t)lo->ncells * lo->p * lo->p * lo->p;
  auto bail = [&](rz_status st) { rz_hodge_free(g); return st; };
  if (g->nlo + g->nhi >= (int64_t)1 << 31) return bail(fail(ctx, RZ_ERR_ARG, "rz_hodge_create: too many DoFs"));
  hipStream_t s = ctx->stream;
  // cell weights: [alpha-part x3, beta-part x3] per cell; mass keeps beta, stiffness alpha
  auto split = [&](rz_problem *h, bool mass) {
    std::vector<double> w(h->coef);
    for (size_t c = 0; c < w.size(); c += 6)
      for (int d = 0; d < 3; ++d) w[c + (mass ? d : 3 + d)] = 0.0;
    return w;
  };
  if ((e = hg_upload(g, &g->cm_lo, split(lo, true)))) return bail(e);
  if (hi && ((e = hg_upload(g, &g->cm_hi, split(hi, true))) || (e = hg_upload(g, &g->cs_hi, split(hi, false)))))
    return bail(e);
  // D and D^T
  std::vector<int> ptr, col, tp, tc;
  std::vector<double> val, tv;
  hg_derivative(k, lo->p, nn, lo->t.D, ptr, col, val);
  if ((int64_t)ptr.size() != g->nhi + 1) return bail(fail(ctx, RZ_ERR_ARG, "rz_hodge_create: D rows"));
  hg_transpose(g->nhi, g->nlo, ptr, col, val, tp, tc, tv);
  if ((e = hg_upload(g, &g->d_ptr, ptr)) || (e = hg_upload(g, &g->d_col, col)) || (e = hg_upload(g, &g->d_val, val)) ||
      (e = hg_upload(g, &g->dt_ptr, tp)) || (e = hg_upload(g, &g->dt_col, tc)) || (e = hg_upload(g, &g->dt_val, tv)))
    return bail(e);
  if (!hi) {
    // DQ_{p-1} mass: 8 / V per value (3-form Piola map, L^2-orthonormal broken basis)
    const int p = lo->p;
    HgLat l3(3, p, nn);
    std::vector<double> m3(g->nhi), m3c(g->nhi);
    std::vector<int> rows(g->nhi);
    const double th = 1.0, dl = 0.1, sg = th / dl;  // interval [0.9, 1.1]
    // q = 1 - p(1) evaluated by running the scalar recurrence itself (A = B = 1)
    {
      double x = 0, r = 1, d = 1.0 / th, rh = 1.0 / sg;
      for (int j = 0; j < g->steps; ++j) {
        x += d;
        if (j + 1 == g->steps) break;
        r -= d;
        const double rn = 1.0 / (2.0 * sg - rh);
        d = rn * rh * d + (2.0 * rn / dl) * r;
        rh = rn;
      }
      for (int64_t c = 0; c < lo->ncells; ++c) {
        const int cx = c % lo->nx, cy = (c / lo->nx) % lo->ny, cz = c / ((int64_t)lo->nx * lo->ny);
        const int nvx = lo->nx + 1, nvy = lo->ny + 1;
        const double hs[3] = {lo->vert[3 * (cx + 1)] - lo->vert[3 * cx],
                              lo->vert[3 * ((cy + 1) * nvx) + 1] - lo->vert[3 * (cy * nvx) + 1],
                              lo->vert[3 * ((int64_t)(cz + 1) * nvx * nvy) + 2] -
                                  lo->vert[3 * ((int64_t)cz * nvx * nvy) + 2]};
        const double w = 8.0 / (hs[0] * hs[1] * hs[2]);
        for (int zc = 0; zc < p; ++zc)
          for (int yc = 0; yc < p; ++yc)
            for (int xc = 0; xc < p; ++xc) {
              const int64_t X[3] = {(int64_t)cx * p + xc, (int64_t)cy * p + yc, (int64_t)cz * p + zc};
              const int64_t gi = l3.index(0, X);
              m3[gi] = w;
              m3c[gi] = x / w;
            }
      }
    }
    for (int64_t i = 0; i < g->nhi; ++i) rows[i] = (int)i;
    if ((e = hg_upload(g, &g->m3, m3)) || (e = hg_upload(g, &g->m3c, m3c)) || (e = hg_upload(g, &g->rows3, rows)))
      return bail(e);
  }
  const int64_t nmax = std::max(g->nlo, g->nhi), N = g->nlo + g->nhi;
  if ((e = hg_alloc(g, &g->partials, dots_partials_size())) || (e = hg_alloc(g, &g->dots, 4)) ||
      (e = hg_alloc(g, &g->tlo, g->nlo)) || (e = hg_alloc(g, &g->thi, g->nhi)) || (e = hg_alloc(g, &g->shi, g->nhi)) ||
      (e = hg_alloc(g, &g->cr, nmax)) || (e = hg_alloc(g, &g->cd, nmax)) || (e = hg_alloc(g, &g->ct, nmax)) ||
      (e = hg_alloc(g, &g->cz, nmax)))
    return bail(e);
  for (double *&v : g->mv)
    if ((e = hg_alloc(g, &v, N))) return bail(e);
  if ((e = hg_extremes(g, lo, g->eig_lo))) return bail(e);
  if (hi && (e = hg_extremes(g, hi, g->eig_hi))) return bail(e);
  if (hipStreamSynchronize(s) != hipSuccess) return bail(fail(ctx, RZ_ERR_HIP, "rz_hodge_create: stream"));
  *out = g;
  return RZ_OK;
}

rz_status rz_hodge_free(rz_hodge *g) {
  if (!g) return RZ_OK;
  hipStreamSynchronize(g->ctx->stream);
  for (void *p : g->allocs) hipFree(p);
  delete g;
  return RZ_OK;
}

rz_status rz_hodge_sizes(const rz_hodge *g, int64_t sizes[2], double eig[4]) {
  if (!g || !sizes) return RZ_ERR_ARG;
  sizes[0] = g->nlo;
  sizes[1] = g->nhi;
  if (eig) {
    eig[0] = g->eig_lo[0];
    eig[1] = g->eig_lo[1];
    eig[2] = g->eig_hi[0];
    eig[3] = g->eig_hi[1];
  }
  return RZ_OK;
}

rz_status rz_hodge_apply(rz_hodge *g, const double *x, double *y) {
  if (!g || !x || !y || x == y) return g ? fail(g->ctx, RZ_ERR_ARG, "rz_hodge_apply: bad vectors") : RZ_ERR_ARG;
  return hg_apply(g, x, y);
}

rz_status rz_hodge_precond(rz_hodge *g, const double *r, double *z) {
  if (!g || !r || !z || r == z) return g ? fail(g->ctx, RZ_ERR_ARG, "rz_hodge_precond: bad vectors") : RZ_ERR_ARG;
  return hg_precond(g, r, z);
}

rz_status rz_hodge_solve(rz_hodge *g, const double *b, double *x, double rtol, int32_t maxit, rz_solve_info *info) {
  if (!g || !b || !x || b == x || !(rtol > 0) || maxit < 1)
    return g ? fail(g->ctx, RZ_ERR_ARG, "rz_hodge_solve: bad arguments") : RZ_ERR_ARG;
  rz_ctx *ctx = g->ctx;
  hipStream_t s = ctx->stream;
  const int64_t N = g->nlo + g->nhi;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  hipEventRecord(e0, s);
  double *v_prev = g->mv[0], *v = g->mv[1], *kz = g->mv[2], *z = g->mv[3], *z_next = g->mv[4];
  double *w_prev = g->mv[5], *w = g->mv[6], *tmp = g->mv[7];
  rz_status st = RZ_OK;
  int it = 0;
  double eta = 0, phi0 = 0;
  auto run = [&]() -> rz_status {
    hipError_t he;
    if ((he = hipMemsetAsync(x, 0, sizeof(double) * N, s)) != hipSuccess ||
        (he = hipMemsetAsync(v_prev, 0, sizeof(double) * N, s)) != hipSuccess ||
        (he = hipMemsetAsync(w_prev, 0, sizeof(double) * N, s)) != hipSuccess ||
        (he = hipMemsetAsync(w, 0, sizeof(double) * N, s)) != hipSuccess ||
        (he = hipMemcpyAsync(v, b, sizeof(double) * N, hipMemcpyDeviceToDevice, s)) != hipSuccess)
      return fail(ctx, RZ_ERR_HIP, hipGetErrorString(he));
    rz_status e;
    if ((e = hg_precond(g, v, z))) return e;
    double g2;
    if ((e = hg_dot(g, v, z, N, &g2))) return e;
    if (!(g2 > 0)) return g2 == 0 ? RZ_OK : fail(ctx, RZ_ERR_BREAKDOWN, "rz_hodge_solve: indefinite preconditioner");
    double gamma = std::sqrt(g2), gamma_prev = 1.0;
    double c = 1, c_prev = 1, sn = 0, s_prev = 0;
    eta = phi0 = gamma;
    while (it < maxit && std::fabs(eta) > rtol * phi0) {
      ++it;
      launch_scale_copy(1.0 / gamma, z, z, N, s);
      if ((e = hg_apply(g, z, kz))) return e;
      double delta;
      if ((e = hg_dot(g, kz, z, N, &delta))) return e;
      launch_axpy(-delta / gamma, v, kz, N, s);
      launch_axpy(-gamma / gamma_prev, v_prev, kz, N, s);  // kz now holds v_next
      if ((e = hg_precond(g, kz, z_next))) return e;
      double gn2;
      if ((e = hg_dot(g, kz, z_next, N, &gn2))) return e;
      if (gn2 < 0) return fail(ctx, RZ_ERR_BREAKDOWN, "rz_hodge_solve: indefinite preconditioner");
      const double gamma_next = std::sqrt(gn2);
      const double a0 = c * delta - c_prev * sn * gamma;
      const double a1 = std::hypot(a0, gamma_next);
      const double a2 = sn * delta + c_prev * c * gamma;
      const double a3 = s_prev * gamma;
      c_prev = c;
      c = a0 / a1;
      s_prev = sn;
      sn = gamma_next / a1;
      // w_next = (z - a3 w_prev - a2 w) / a1, written over w_prev
      launch_scale_copy(-a3 / a1, w_prev, w_prev, N, s);
      launch_axpy(1.0 / a1, z, w_prev, N, s);
      launch_axpy(-a2 / a1, w, w_prev, N, s);
      std::swap(w_prev, w);  // w = w_next, w_prev = old w
      launch_axpy(c * eta, w, x, N, s);
      eta = -sn * eta;
      // rotate: v_prev <- v, v <- v_next (in kz); the old v_prev buffer takes the next A z
      double *old = v_prev;
      v_prev = v;
      v = kz;
      kz = old;
      std::swap(z, z_next);
      gamma_prev = gamma;
      gamma = gamma_next;
      if (gamma == 0) break;
    }
    return RZ_OK;
  };
  st = run();
  double rel = -1;
  if (st == RZ_OK) {
    // true residual ||b - K x|| / ||b||
    rz_status e = hg_apply(g, x, tmp);
    if (!e) {
      launch_axpy(-1.0, b, tmp, N, s);
      double rr = 0, bb = 0;
      if (!(e = hg_dot(g, tmp, tmp, N, &rr)) && !(e = hg_dot(g, b, b, N, &bb))) rel = bb > 0 ? std::sqrt(rr / bb) : 0;
    }
    st = e;
  }
  hipEventRecord(e1, s);
  hipEventSynchronize(e1);
  float ms = 0;
  hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st == RZ_OK && std::fabs(eta) > rtol * phi0) st = RZ_ERR_NOT_CONVERGED;
  if (info) {
    info->iters = it;
    info->status = st;
    info->rel_res = rel;
    info->omega = 0.0;
    info->t_solve_ms = ms;
    info->iters_natural = it;
  }
  return st;
}

}  // extern "C"
