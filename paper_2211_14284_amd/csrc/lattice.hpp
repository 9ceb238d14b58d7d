// Index arithmetic of the lattice numbering and of the vertex-star interface
// patch layout, shared by host code and HIP kernels.
//
// Q_p lattice: X = c*p + a (a in 0..p), index X + Nx*(Y + Ny*Z), Nx = nx*p + 1.
//
// Vertex-star interface patch of a vertex at lattice (Xv, Yv, Zv) (Sec. 4.1: the
// star of v; Sec. 4.4: its interface DoFs).  Patch DoFs are the lattice points
// with offsets d in (-p, p)^3 with at least one zero offset.  Patch order: the 12
// faces (normal axis a = x, y, z; side along the lower remaining axis b, then
// along the higher one c; inside a face ascending lattice index = offset along b
// fastest), then the 6 edges (axis, side, ascending), then the vertex.
#pragma once

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define RZ_HD __host__ __device__ inline
#else
#define RZ_HD inline
#endif

namespace rz {

RZ_HD int patch_nrows(int p) { return 1 + 6 * (p - 1) + 12 * (p - 1) * (p - 1); }

// Local index of the patch DoF with offsets (dx, dy, dz); -1 if not a patch DoF.
RZ_HD int patch_local_index(int p, int dx, int dy, int dz) {
  const int q = p - 1;
  int d[3] = {dx, dy, dz};
  int nz = (dx == 0) + (dy == 0) + (dz == 0);
  for (int k = 0; k < 3; ++k)
    if (d[k] <= -p || d[k] >= p) return -1;
  if (nz == 0) return -1;
  if (nz == 3) return 12 * q * q + 6 * q;
  if (nz == 1) {
    int a = dx == 0 ? 0 : (dy == 0 ? 1 : 2);
    int b = a == 0 ? 1 : 0;
    int c = a == 2 ? 1 : 2;
    int sb = d[b] > 0, sc = d[c] > 0;
    int u = sb ? d[b] - 1 : d[b] + q;
    int w = sc ? d[c] - 1 : d[c] + q;
    return (a * 4 + sb * 2 + sc) * q * q + u + q * w;
  }
  int a = dx != 0 ? 0 : (dy != 0 ? 1 : 2);
  int s = d[a] > 0;
  int u = s ? d[a] - 1 : d[a] + q;
  return 12 * q * q + (a * 2 + s) * q + u;
}

// Offsets of patch DoF k (inverse of patch_local_index).
RZ_HD void patch_offsets(int p, int k, int &dx, int &dy, int &dz) {
  const int q = p - 1;
  int d[3] = {0, 0, 0};
  if (k < 12 * q * q) {
    int f = k / (q * q), r = k % (q * q);
    int a = f / 4, sb = (f >> 1) & 1, sc = f & 1;
    int b = a == 0 ? 1 : 0;
    int c = a == 2 ? 1 : 2;
    int u = r % q, w = r / q;
    d[b] = sb ? u + 1 : u - q;
    d[c] = sc ? w + 1 : w - q;
  } else if (k < 12 * q * q + 6 * q) {
    int e = (k - 12 * q * q) / q, u = (k - 12 * q * q) % q;
    int a = e / 2, s = e & 1;
    d[a] = s ? u + 1 : u - q;
  }
  dx = d[0];
  dy = d[1];
  dz = d[2];
}

// 1-D structural patterns of the FDM mass (diagonal + (0,p)) and stiffness
// (diagonal + full rows/columns 0 and p).
RZ_HD bool pat_mass(int p, int a, int b) { return a == b || (a == 0 && b == p) || (a == p && b == 0); }
RZ_HD bool pat_stiff(int p, int a, int b) { return a == b || a == 0 || a == p || b == 0 || b == p; }

RZ_HD bool on_end(int p, int a) { return a == 0 || a == p; }

// Structural coupling of two local cell DoFs u, w (coordinates 0..p) in the
// Schur complement of one cell: P_GG pattern, or a common interior neighbour.
RZ_HD bool cell_schur_coupled(int p, const int u[3], const int w[3]) {
  for (int d = 0; d < 3; ++d) {
    bool ok = pat_stiff(p, u[d], w[d]);
    for (int e = 0; e < 3 && ok; ++e)
      if (e != d) ok = pat_mass(p, u[e], w[e]);
    if (ok) return true;
  }
  int nu = on_end(p, u[0]) + on_end(p, u[1]) + on_end(p, u[2]);
  int nw = on_end(p, w[0]) + on_end(p, w[1]) + on_end(p, w[2]);
  if (nu != 1 || nw != 1 || p < 2) return false;
  int du = on_end(p, u[0]) ? 0 : (on_end(p, u[1]) ? 1 : 2);
  int dw = on_end(p, w[0]) ? 0 : (on_end(p, w[1]) ? 1 : 2);
  if (du == dw) {
    for (int e = 0; e < 3; ++e)
      if (e != du && u[e] != w[e]) return false;
    return true;
  }
  int e = 3 - du - dw;
  return u[e] == w[e];
}

}  // namespace rz
