// Host-side launchers of the HIP kernels (gfx950).  All launches are
// asynchronous on the given stream; pointers are device pointers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace rz {

// Lattice description passed to kernels by value.
struct LatDev {
  int p, nx, ny, nz;   // degree and cells per axis
  int Nx, Ny, Nz;      // Q_p lattice extents (n*p + 1)
  unsigned dir;        // Dirichlet face bits
};

// H(curl) / H(div) lattice (space 1 / 2): component m has extents ext[m][a] and
// starts at off[m] (off[3] = all DoFs); cell_dofs = sum of the per-cell tile sizes.
struct VecDev {
  int p, nx, ny, nz;
  unsigned dir;
  int space;
  int ext[3][3];
  long off[4];
  int cell_dofs;
};

// Per-cell algebra of the H(curl) / H(div) relaxation (device): the local numbering
// (component and tile coordinates of every local DoF), the interior / interface
// split, the interior blocks (at most 3 x 3) with their inverse Cholesky factors,
// and P_GI, P_IG in CSR with one value set per key (cells with equal weights share
// a key).
template <typename T>
struct VecCellDev {
  int nI, nG, nblk, nnz_gi, nnz_ig;
  const int *il, *gl;        // local DoF of each interior / interface position
  const int *lcomp, *lcrd;   // per local DoF: component, 3 tile coordinates
  const int *blk;            // 3 interior positions per block (-1 padded)
  const int *key;            // key of every cell
  const T *linv;             // per key: 9 values per block (L^{-1}, row-major, lower)
  const int *gi_ptr, *gi_col;
  const T *gi_val;           // per key: nnz_gi values
  const int *ig_ptr, *ig_col;
  const T *ig_val;           // per key: nnz_ig values
};

// Edge-star patch layout (fixed per degree: p mode blocks) and the patches.
struct EdgeDev {
  int p, nslot, fac_stride, npatch;
  int blk_n[9], blk_slot[9], blk_fac[9];
  const int *idx;   // npatch * nslot global DoFs (-1: absent slot)
  const int *type;  // npatch: factor set of each patch
  int nchunk;       // groups of at most 256 patches of one type
  const int *chunk; // nchunk x 3: first and end position in plist, type
  const int *plist; // npatch: the patches ordered by type
};

// Symbolic patch data on the device.
struct PatchDev {
  int nrows, nnz;
  int nflev, nblev;
  const int *off;                  // 3*nrows offsets
  const int *rowptr, *col;         // lower CSR (diagonal last)
  const int *erow;                 // row of every CSR entry
  const int *uptr, *urow, *upos;   // column access of the lower factor
  const int *flev_ptr, *flev_rows, *blev_ptr, *blev_rows;
  // slot layout of the factor values (see PatchSymbolic): stride values per slot,
  // CSR entry k at perm[k] and, for off-diagonal entries, also at perm2[k]
  int stride;
  const int *perm, *perm2;
};

// Wavefront schedule of the patch triangular solves (see PatchSymbolic).
struct PatchEllDev {
  int nrows, npass, ne, stride;
  int kmax;                        // largest step count K over the passes (1..8)
  const int *pass;                 // 3*npass: lanes per row G, steps K, ELL offset
  const int *ecol;                 // ne: x index read at every ELL position
  const int *erow;                 // 64*npass: row solved by each lane's group (-1 none)
  const int *off;                  // 3*nrows: lattice offsets of the patch rows
  int regs;                        // 1: the schedule equals the one compiled into the register kernel
  int ell0;                        // offset of the ELL values in a slot (values at ell0 + ell_pos)
  int cap[2];                      // streaming kernel: resident wavefronts per CU (FP64, FP32),
                                   // chosen by the setup's autotuner; 0 = the built-in default
};

// Trilinear cells with sampled coefficients: vertex coordinates (nvertices x 3,
// FP64), 27 coefficient samples per cell, and the quadrature tabulations of
// QuadTables (Bq, Dq: Q x (p+1); wq, xq: Q; Lq: Q x 3) in the compute precision.
template <typename T>
struct QuadDev {
  const double *vert;
  const T *as, *bs;
  const T *Bq, *Dq, *wq, *xq, *Lq;
};

// ---- vectors ------------------------------------------------------------------
void launch_fill(double *y, double v, int64_t n, hipStream_t s);
void launch_cast_d2f(const double *x, float *y, int64_t n, hipStream_t s);
void launch_cast_f2d(const float *x, double *y, int64_t n, hipStream_t s);
// y = a * x (a = 1: plain widening), and y += a * x, x in FP32
void launch_f2d_scale(double a, const float *x, double *y, int64_t n, hipStream_t s);
void launch_f2d_axpy(double a, const float *x, double *y, int64_t n, hipStream_t s);
// y = a*x + y ; y = x + b*y ; z = x - y
void launch_axpy(double a, const double *x, double *y, int64_t n, hipStream_t s);
void launch_xpby(const double *x, double b, double *y, int64_t n, hipStream_t s);
void launch_sub(const double *x, const double *y, double *z, int64_t n, hipStream_t s);
void launch_scale_copy(double a, const double *x, double *y, int64_t n, hipStream_t s);
// Multi-vector layouts: interleaved u (value r of DoF g at u[g * nv + r]) to planar v
// (vector r at v + r * ld, n values each), and back.
template <typename T>
void launch_deinterleave(const T *u, T *v, int nv, int64_t ld, int64_t n, hipStream_t s);
template <typename T>
void launch_interleave(const T *v, T *u, int nv, int64_t ld, int64_t n, hipStream_t s);
// Deterministic two-pass dot products: out[k] = <x_k, y_k> for up to 3 pairs.
void launch_dots(int npairs, const double *const *xs, const double *const *ys, int64_t n,
                 double *partials, double *out, hipStream_t s);
int dots_partials_size();
// x += a p; ro = r (if ro != nullptr); r -= a Ap; out[0] = r.r (two-pass, like
// launch_dots); a = *num / *den from device memory (0 if *den <= 0)
void launch_cg_update(const double *num, const double *den, const double *p, const double *Ap, double *x,
                      double *r, double *ro, int64_t n, double *partials, double *out, hipStream_t s);
// y = x + b y, b = (*num - *cross) / *den from device memory (cross may be null)
void launch_xpby_dev(const double *x, const double *num, const double *cross, const double *den, double *y,
                     int64_t n, hipStream_t s);

// FP32 vectors (inner solve of the defect-correction protocol); inner products
// accumulate in FP64 into out[k] like launch_dots
void launch_axpy_f(float a, const float *x, float *y, int64_t n, hipStream_t s);
void launch_xpby_f(const float *x, float b, float *y, int64_t n, hipStream_t s);
void launch_sub_f(const float *x, const float *y, float *z, int64_t n, hipStream_t s);
void launch_scale_copy_f(float a, const float *x, float *y, int64_t n, hipStream_t s);
void launch_fill_f(float *y, float v, int64_t n, hipStream_t s);
void launch_add_f2d(const float *x, double *y, int64_t n, hipStream_t s);  // y += x
void launch_add_d2f(const double *t, float *z, int64_t n, hipStream_t s);  // z += t
void launch_dots_f(int npairs, const float *const *xs, const float *const *ys, int64_t n, double *partials,
                   double *out, hipStream_t s);
void launch_cg_update_f(float a, const float *p, const float *Ap, float *x, float *r, float *ro, int64_t n,
                        double *partials, double *out, hipStream_t s);

// ---- H(grad) operator and relaxation ----------------------------------------------
// Bh, Ah: host copies of the 1-D FDM mass and stiffness ((p+1)^2, row-major);
// y = A x, or y = bsub - A x when bsub is not null (y must not alias x or bsub);
// fbuf: scratch of ny*nz*4p*Nx values (the face-line buffer)
template <typename T>
void launch_apply_grad(const LatDev &L, const T *coef, const double *Bh, const double *Ah, const T *x,
                       const T *bsub, T *y, T *fbuf, hipStream_t s);
// rt at every plane point (interior points of rt are left unwritten)
template <typename T>
void launch_condense_grad(const LatDev &L, const T *coef, const T *A, const T *lam, const T *r, T *rt,
                          hipStream_t s);
// Returns non-zero when the schedule does not fit the LDS of one block.
// true when the host pass table (G, K, ELL offset per pass; ne ELL values) of
// degree p equals the schedule compiled into the register-resident patch solve
bool patch_regs_table_matches(int p, const int *pass, int np, int nrows, int ne, int ell0);
// whether the patch solve of degree p in elements of elem bytes runs the
// register-resident kernel (else the streaming one)
bool patch_solve_uses_regs(const PatchEllDev &E, int p, size_t elem);
size_t patch_solve_lds_bytes(const PatchEllDev &E, size_t elem, int waves);
// the streaming kernel's block shape (wavefronts per block, blocks per CU) for at
// most cap resident wavefronts per CU; false if no block fits the LDS
bool patch_solve_stream_shape(const PatchEllDev &E, size_t elem, int cap, int &waves, int &per_cu);
// Right-hand sides and outputs of one patch-solve launch over several vectors.
constexpr int kPatchMaxVecs = 2;
template <typename T>
struct PatchVecs {
  const T *rt[kPatchMaxVecs];
  T *zb[kPatchMaxVecs];
};
template <typename T>
int launch_patch_solve(const LatDev &L, const PatchEllDev &E, const T *factor, const T *rt, T *zbuf, hipStream_t s);
template <typename T>
int launch_patch_solve_multi(const LatDev &L, const PatchEllDev &E, const T *factor, int nvec, const T *const *rt,
                             T *const *zb, hipStream_t s);
// y = A x on BF16 vectors (Cartesian H(grad)): FP32 weights, arithmetic and face-line
// buffer, BF16 loads of x and stores of y.
void launch_apply_grad_bf16(const LatDev &L, const float *coef, const double *Bh, const double *Ah,
                            const unsigned short *x, unsigned short *y, float *fbuf, hipStream_t s);
// The same on BF16 vectors x, y (FP32 per-cell buffer): the 1-D contractions on the
// matrix cores (BF16 operands, FP32 accumulation), the pullback in FP32; then the
// gather of the interface rows.  Returns non-zero for an unsupported degree.
int launch_apply_quad_cells_bf16(const LatDev &L, const QuadDev<float> &G, const unsigned short *x,
                                 unsigned short *y, float *ebuf, hipStream_t s);
void launch_apply_gather_bf16(const LatDev &L, const unsigned short *x, const float *ebuf, unsigned short *y,
                              hipStream_t s);
// Cell phase of y = A x on trilinear cells (interior rows to y, interface rows to
// ebuf); the interface rows are then summed by launch_apply_gather.  Returns
// non-zero for an unsupported degree.
template <typename T>
int launch_apply_quad_cells(const LatDev &L, const QuadDev<T> &G, const T *x, T *y, T *ebuf, hipStream_t s,
                            const T *bsub = nullptr);  // bsub: interior rows store bsub - A x
template <typename T>
void launch_apply_gather(const LatDev &L, const T *x, const T *ebuf, T *y, hipStream_t s,
                         const T *bsub = nullptr);  // bsub: y = bsub - A x (bsub - x on Dirichlet rows)
// y = A x in H(curl) / H(div) on axis-aligned cells (weights: 6 per cell, stiffness
// part 0..2, mass part 3..5); ebuf: ncells * cell_dofs.  Non-zero for unsupported p.
template <typename T>
int launch_apply_vec(const VecDev &V, const T *coef, const T *B, const T *D, const T *x, T *y, T *ebuf,
                     hipStream_t s, const T *bsub = nullptr);  // bsub: y = bsub - A x
// ---- H(curl) / H(div) relaxation ---------------------------------------------------
// z_I = P_II^{-1} r_I at the interior DoFs; eb (ncells * nG) = P_GI z_I per cell
template <typename T>
void launch_vc_condense(const VecDev &V, const VecCellDev<T> &C, const T *r, T *z, T *eb, hipStream_t s);
// z_I -= P_II^{-1} P_IG z_G
template <typename T>
void launch_vc_expand(const VecDev &V, const VecCellDev<T> &C, T *z, hipStream_t s);
// y[rows[t]] = (x ? x[rows[t]] : 0) + sign * sum_{k in ptr[t]..ptr[t+1]} buf[pos[k]]
template <typename T>
void launch_list_gather(int n, const int *rows, const int *ptr, const int *pos, const T *buf, const T *x, T *y,
                        T sign, hipStream_t s);
// y[rows[t]] = d[t] * x[rows[t]]
template <typename T>
void launch_rows_scale(int n, const int *rows, const T *d, const T *x, T *y, hipStream_t s);
// y[row t] (+= if add) sum_k val[k] x[col[k]], row t = rows ? rows[t] : t (sums in TV)
template <typename TV, typename TX, typename TY>
void launch_csr(int n, const int *rows, const int *ptr, const int *col, const TV *val, const TX *x, TY *y, int add,
                hipStream_t s);
// the same with one wavefront per row (long rows)
template <typename TV, typename TX, typename TY>
void launch_csr_wave(int n, const int *rows, const int *ptr, const int *col, const TV *val, const TX *x, TY *y,
                     int add, hipStream_t s);
// edge-star Cholesky solves: zb (npatch * nslot) from rt
template <typename T>
void launch_edge_solve(const EdgeDev &E, const T *fac, const T *rt, T *zb, hipStream_t s);
// y = M x, dense m x m row-major matrix in TM, FP64 vectors
template <typename TM>
void launch_gemv(int m, const TM *M, const double *x, double *y, hipStream_t s);
// y = M x for a dense symmetric m x m matrix (row-major) from its lower triangle;
// work: ceil(m/64)^2 * 64 doubles
// One matrix row per lane of the h-multigrid cycle on the Q_1 space (FP64), the
// matrix in ELL form (n rows, width entries each, entry k of row i at k * n + i;
// hmg_ell_width lists the widths compiled for):
// HMG_RES0 out = b - A (w D^{-1} b); HMG_PROD out = M x; HMG_PROL out = w D^{-1} b + P x;
// HMG_POST out = x + w D^{-1} (b - A x); HMG_RES out = b - A x; HMG_ADD out = b + M x;
// HMG_JPROD out = w D^{-1} (M x).  out aliases none of the inputs.
enum { HMG_RES0 = 0, HMG_PROD = 1, HMG_PROL = 2, HMG_POST = 3, HMG_RES = 4, HMG_ADD = 5, HMG_JPROD = 6 };
// the smallest compiled ELL width >= w (w itself past 64: a loop without a fixed count)
inline int hmg_ell_width(int w) {
  static const int kW[] = {2, 4, 6, 8, 12, 16, 18, 20, 24, 27, 28, 32, 36, 40, 48, 64};
  for (int v : kW)
    if (v >= w) return v;
  return w;
}
void launch_hmg_row(int mode, int n, int width, const int *col, const double *val, const double *x,
                    const double *b, const double *dinv, double w, double *out, hipStream_t s);
template <typename TM>
void launch_symv(int m, const TM *M, const double *x, double *y, double *work, hipStream_t s);
// z[list[t]] = r ? r[list[t]] : 0
template <typename T>
void launch_list_copy(int n, const int *list, const T *r, T *z, hipStream_t s);

// number of compute units of the current device (cached), for persistent grids
int device_cu_count();
// z = scale * (relaxation output); with acc: acc += w * output at every point (scale
// must then be 1; z receives the plane values only, as scratch)
template <typename T>
void launch_expand_grad(const LatDev &L, const PatchDev &P, const T *coef, const T *A,
                        const T *lam, const T *r, const T *zbuf, T *z, T scale, T w, T *acc, hipStream_t s);

// The paper's auxiliary on trilinear cells (eq. sum-factorization_approx): per-cell
// broken diagonals (FP64, setup) -- dm (p+1)^3 and da 3 p (p+1)^2 per cell -- with the
// 1-D broken transformation G ((p+1)^2) and D-hat (p x (p+1)); dm == nullptr selects
// the separable per-cell weights.
struct PdDev {
  const double *dm, *da, *G, *D;
};
// Solve-time data of that auxiliary: P_II diagonal and w_d(t) = sqrt(lambda_{t_d})
// da_d(t) at cell-interior lattice points, D-hat in the compute precision.
template <typename T>
struct PdSolve {
  const T *pii, *w0, *w1, *w2, *D;
};
template <typename T>
void launch_condense_pd(const LatDev &L, const PdSolve<T> &S, const T *r, T *rt, hipStream_t s);
template <typename T>
void launch_expand_interior_pd(const LatDev &L, const PdSolve<T> &S, const T *r, T *z, T scale, T w, T *acc,
                               hipStream_t s);
// the plane part of launch_expand_grad alone (patch sums at plane points, Dirichlet
// rows copy r; z = scale * value, or acc += w * value as well)
template <typename T>
void launch_expand_plane_grad(const LatDev &L, const T *r, const T *zbuf, T *z, T scale, T w, T *acc, hipStream_t s);

// IC factorisation of every vertex patch (FP64) on the static-condensation
// pattern; writes the FP64 factor and an FP32 copy; *status = 0 or the first
// failing patch + 1 (pivot <= 0).
void launch_patch_factor(const LatDev &L, const PatchDev &P, const double *coef, const double *B,
                         const double *A, const double *lam, const PdDev &pd, double *f64, float *f32, int *status,
                         hipStream_t s, int ic = 1);
// Vertex-patch solves with exact Cholesky factors: z_v = W_v^T (W_v b_v), W_v = L_v^{-1}
// dense lower packed by rows, nrows (nrows + 1) / 2 values per slot
template <typename T>
void launch_patch_chol_solve(const LatDev &L, const PatchDev &P, const T *W, const T *rt, T *zb, hipStream_t s);
// Sum of the full vertex stars' solutions at every lattice point (Dirichlet points take
// r), times scale, to z, or with acc: acc += w times that
// Dense patch solves z_v = W_v^T (W_v b_v) on npatch patches given by index lists (nr
// entries each, -1 padding), W_v packed by rows
template <typename T>
void launch_dense_patch_solve(int npatch, int nr, const int *idx, const T *W, const T *r, T *zb, hipStream_t s);
template <typename T>
void launch_full_star_sum(const LatDev &L, int nrf, const T *zb, const T *r, T *z, T scale, T w, T *acc,
                          hipStream_t s);

// z_D = r_D on Dirichlet rows of the Q_p lattice (r == nullptr: z_D = 0).
void launch_dirichlet_copy_f(const LatDev &L, const float *r, float *z, hipStream_t s);
void launch_dirichlet_copy(const LatDev &L, const double *r, double *z, hipStream_t s);

// ---- p-transfer (Q_1 <-> Q_p) -------------------------------------------------------
void launch_prolong_add_grad(const LatDev &L, const double *E, const double *xc, double *xf,
                             hipStream_t s);
// z += P xc and r -= A P xc in one pass (Cartesian cells, cellwise-constant weights);
// T2: the (p+1) x 2 products A E then B E of the 1-D tables with the hat embedding
void launch_prolong_residual_grad(const LatDev &L, const double *E, const double *T2, const double *coef,
                                  const double *xc, double *z, double *r, hipStream_t s);
// the same on FP32 vectors z and r (sums in FP64)
void launch_prolong_residual_grad_f(const LatDev &L, const double *E, const double *T2, const double *coef,
                                    const double *xc, float *z, float *r, hipStream_t s);
// t1: (nx+1)*Ny*Nz and t2: (nx+1)*(ny+1)*Nz scratch arrays
void launch_restrict_grad(const LatDev &L, const double *E, const double *rf, double *rc, double *t1,
                          double *t2, hipStream_t s);

// ---- coarse block-tridiagonal LDL^T ---------------------------------------------------
// Dense m x m blocks, row-major; C and Ct are m x 9 stencil couplings to the
// previous / next plane (entry j couples to in-plane offset (j%3-1, j/3-1)).
void launch_schur_update(int m, int mx, const double *Wprev, const double *C, const double *Akk,
                         double *Dk, hipStream_t s);
void launch_sweep_inverse(int m, double *W, double *tmp, int *status, hipStream_t s);
// out = W Cs for the 9-point coupling Cs (m*9, see launch_coarse_solve)
void launch_coarse_wc(int m, int mx, int my, const double *W, const double *C, double *out, hipStream_t s);
// cooperative blocks of the coarse solve for plane size m
int coarse_blocks(int m);
// Whole block-tridiagonal solve in one cooperative launch, on the twisted block
// factorisation with middle plane q (q = nb - 1: top-down only).  W: nb inverse
// blocks (m*m each); M, N: nb coupling products each (see k_coarse_mn); u: nb*m
// scratch; v, x: nb*m each, overwritten; on entry they must hold the not-yet-written
// pattern (launch_coarse_gather sets it, earlier in the same stream); returns 0 on a
// successful launch.
int launch_coarse_solve(int m, int nb, int q, const double *W, const double *M, const double *N, const double *r,
                        double *u, double *v, double *x, int *status, hipStream_t s);
// the same with the dense blocks stored in FP32 (vectors and sums in FP64)
int launch_coarse_solve_f(int m, int nb, int q, const float *W, const float *M, const float *N, const double *r,
                          double *u, double *v, double *x, int *status, hipStream_t s);
// gather / scatter between the coarse lattice and the free-box block vector; the
// gather also sets the sweep vectors v, x (nfree entries each) to the empty pattern
// that launch_coarse_solve(_f) expects (call it before each solve)
void launch_coarse_gather(int nfree, int bx0, int by0, int bz0, int mx, int my, int NX, int NY,
                          const double *rc, double *blk, double *v, double *x, hipStream_t s);
void launch_coarse_scatter(int ncoarse, int bx0, int by0, int bz0, int mx, int my, int mz, int NX,
                           int NY, const double *blk, double *xc, hipStream_t s);

}  // namespace rz
