// Host side of the geometric h-multigrid on the Q_1 space (Sec. 5.1).
#include "hmg.hpp"

#include <algorithm>
#include <utility>

namespace rz {

HostCsr csr_product(const HostCsr &A, const HostCsr &B) {
  HostCsr C;
  C.n = A.n;
  C.m = B.m;
  C.ptr.assign(A.n + 1, 0);
  std::vector<double> acc(B.m, 0.0);
  std::vector<int> mark(B.m, -1), cols;
  for (int i = 0; i < A.n; ++i) {
    cols.clear();
    for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      const int j = A.col[k];
      const double a = A.val[k];
      for (int q = B.ptr[j]; q < B.ptr[j + 1]; ++q) {
        const int c = B.col[q];
        if (mark[c] != i) {
          mark[c] = i;
          acc[c] = 0.0;
          cols.push_back(c);
        }
        acc[c] += a * B.val[q];
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int c : cols) {
      C.col.push_back(c);
      C.val.push_back(acc[c]);
    }
    C.ptr[i + 1] = (int)C.col.size();
  }
  return C;
}

HostCsr csr_transpose(const HostCsr &A) {
  HostCsr T;
  T.n = A.m;
  T.m = A.n;
  T.ptr.assign(A.m + 1, 0);
  for (int c : A.col) ++T.ptr[c + 1];
  for (int j = 0; j < A.m; ++j) T.ptr[j + 1] += T.ptr[j];
  T.col.resize(A.col.size());
  T.val.resize(A.val.size());
  std::vector<int> next(T.ptr.begin(), T.ptr.end() - 1);
  for (int i = 0; i < A.n; ++i)  // rows in ascending order: T's columns come out sorted
    for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      const int q = next[A.col[k]]++;
      T.col[q] = i;
      T.val[q] = A.val[k];
    }
  return T;
}

FreeBox free_box(const int n[3], unsigned dir) {
  FreeBox b;
  for (int a = 0; a < 3; ++a) {
    b.n[a] = n[a];
    b.lo[a] = (dir & (1u << (2 * a))) ? 1 : 0;
    b.hi[a] = (dir & (1u << (2 * a + 1))) ? n[a] - 1 : n[a];
  }
  return b;
}

HostCsr trilinear_interpolation(const FreeBox &f, const FreeBox &c) {
  HostCsr P;
  P.n = (int)f.size();
  P.m = (int)c.size();
  P.ptr.assign(P.n + 1, 0);
  // per axis: the coarse parents (free ones only) of fine vertex v, with weights
  auto parents = [](const FreeBox &c, int a, int v, int *cc, double *w) {
    int k = 0;
    for (int d = -1; d <= 1; ++d) {
      const int t = v + d;
      if (t % 2 != 0 || t / 2 < c.lo[a] || t / 2 > c.hi[a]) continue;
      cc[k] = t / 2 - c.lo[a];
      w[k++] = d == 0 ? 1.0 : 0.5;
    }
    return k;
  };
  int cx[2], cy[2], cz[2];
  double wx[2], wy[2], wz[2];
  int64_t row = 0;
  for (int z = f.lo[2]; z <= f.hi[2]; ++z) {
    const int nz = parents(c, 2, z, cz, wz);
    for (int y = f.lo[1]; y <= f.hi[1]; ++y) {
      const int ny = parents(c, 1, y, cy, wy);
      for (int x = f.lo[0]; x <= f.hi[0]; ++x, ++row) {
        const int nx = parents(c, 0, x, cx, wx);
        for (int k = 0; k < nz; ++k)
          for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
              P.col.push_back(cx[i] + c.ext(0) * (cy[j] + c.ext(1) * cz[k]));
              P.val.push_back(wx[i] * wy[j] * wz[k]);
            }
        P.ptr[row + 1] = (int)P.col.size();
      }
    }
  }
  return P;
}

void hmg_hierarchy(HostCsr A0, const int n0[3], unsigned dir, int64_t min_free, std::vector<HostCsr> &A,
                   std::vector<HostCsr> &P, std::vector<HostCsr> &R) {
  A.clear();
  P.clear();
  R.clear();
  int n[3] = {n0[0], n0[1], n0[2]};
  FreeBox fb = free_box(n, dir);
  A.push_back(std::move(A0));
  while (n[0] % 2 == 0 && n[1] % 2 == 0 && n[2] % 2 == 0 && fb.size() > min_free) {
    const int nc[3] = {n[0] / 2, n[1] / 2, n[2] / 2};
    const FreeBox cb = free_box(nc, dir);
    if (cb.ext(0) < 1 || cb.ext(1) < 1 || cb.ext(2) < 1) break;
    P.push_back(trilinear_interpolation(fb, cb));
    R.push_back(csr_transpose(P.back()));
    A.push_back(csr_product(R.back(), csr_product(A.back(), P.back())));
    for (int a = 0; a < 3; ++a) n[a] = nc[a];
    fb = cb;
  }
}

}  // namespace rz
