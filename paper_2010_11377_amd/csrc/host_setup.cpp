// Host-side setup; see host_setup.hpp.
#include "host_setup.hpp"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdio>

namespace irk {

void Stencil9::resize(int nx_, int ny_) {
  nx = nx_;
  ny = ny_;
  for (int k = 0; k < 9; ++k) c[k].assign((size_t)nx * ny, 0.0);
}

int ldu_factor(int s, const double *A, double *L, double *d, double *U) {
  if (s < 1 || s > 8 || !A) return -1;
  double amax = 0.0;
  for (int i = 0; i < s * s; ++i) amax = std::max(amax, std::fabs(A[i]));
  double W[64], Lw[64];
  for (int i = 0; i < s * s; ++i) W[i] = A[i];
  for (int i = 0; i < s * s; ++i) Lw[i] = 0.0;
  for (int i = 0; i < s; ++i) Lw[i * s + i] = 1.0;
  const double piv_tol = 64.0 * DBL_EPSILON * (amax > 0 ? amax : 1.0);
  // Doolittle elimination without row exchanges: row i -= l_ik * row k.
  for (int k = 0; k < s; ++k) {
    double p = W[k * s + k];
    if (!(std::fabs(p) > piv_tol)) return -2;
    for (int i = k + 1; i < s; ++i) {
      double l = W[i * s + k] / p;
      Lw[i * s + k] = l;
      for (int j = k; j < s; ++j) W[i * s + j] -= l * W[k * s + j];
    }
  }
  for (int i = 0; i < s; ++i) {
    if (d) d[i] = W[i * s + i];
    for (int j = 0; j < s; ++j) {
      if (L) L[i * s + j] = Lw[i * s + j];
      if (U) U[i * s + j] = (j < i) ? 0.0 : (j == i ? 1.0 : W[i * s + j] / W[i * s + i]);
    }
  }
  return 0;
}

int coefficient_matrix(int s, const double *A, int kind, double *At) {
  for (int i = 0; i < s * s; ++i) At[i] = 0.0;
  if (kind == 2 || kind == 3) {
    if (s < 1 || s > 8) return -1;
    for (int i = 0; i < s; ++i)
      for (int j = 0; j <= i; ++j)
        if (kind == 2 || i == j) At[i * s + j] = A[i * s + j];
    return 0;
  }
  double L[64], d[8], U[64];
  int rc = ldu_factor(s, A, L, d, U);
  if (rc) return rc;
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < s; ++j)
      At[i * s + j] = (kind == 0) ? L[i * s + j] * d[j] : d[i] * U[i * s + j];
  return 0;
}

bool csr_to_stencil(int n, const int *rowptr, const int *colind, const double *val, int nx,
                    int ny, Stencil9 &out, std::string &err) {
  char buf[256];
  if (nx <= 0 || ny <= 0 || (long long)nx * ny != n) {
    err = "grid nx*ny does not match the matrix size";
    return false;
  }
  if (!rowptr || !colind || !val) {
    err = "null CSR array";
    return false;
  }
  if (rowptr[0] != 0) {
    err = "CSR rowptr[0] must be 0";
    return false;
  }
  out.resize(nx, ny);
  for (int r = 0; r < n; ++r) {
    if (rowptr[r + 1] < rowptr[r]) {
      err = "CSR rowptr is decreasing";
      return false;
    }
    int i = r % nx, j = r / nx;
    int prev = -1;
    for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) {
      int col = colind[e];
      if (col < 0 || col >= n) {
        snprintf(buf, sizeof buf, "CSR column %d out of range in row %d", col, r);
        err = buf;
        return false;
      }
      if (col <= prev) {
        snprintf(buf, sizeof buf, "CSR columns not sorted/unique in row %d", r);
        err = buf;
        return false;
      }
      prev = col;
      double v = val[e];
      if (!std::isfinite(v)) {
        snprintf(buf, sizeof buf, "non-finite CSR value in row %d", r);
        err = buf;
        return false;
      }
      int ci = col % nx, cj = col / nx;
      int dx = ci - i, dy = cj - j;
      if (dx < -1 || dx > 1 || dy < -1 || dy > 1) {
        snprintf(buf, sizeof buf, "row %d couples (%d,%d) to (%d,%d): not a 3x3 stencil", r, i, j,
                 ci, cj);
        err = buf;
        return false;
      }
      out.c[(dy + 1) * 3 + (dx + 1)][r] += v;
    }
  }
  if (rowptr[n] < 0) {
    err = "bad CSR nnz";
    return false;
  }
  return true;
}

Stencil9 identity_stencil(int nx, int ny) {
  Stencil9 s;
  s.resize(nx, ny);
  std::fill(s.c[4].begin(), s.c[4].end(), 1.0);
  return s;
}

double boundary_weight(int level) {
  const double p = std::ldexp(1.0, level);
  return (p + 1.0) / (2.0 * p + 1.0);
}

Interp linear_interp(int level) { return Interp{0.75, 0.25, boundary_weight(level)}; }
Interp constant_interp() { return Interp{1.0, 0.0, 1.0}; }

// 1-D interpolation weights of fine point f onto coarse points: returns the
// number of parents (1 at the ends of the grid or without neighbour weight).
static int interp1d(int f, int nc, const Interp &ip, int *J, double *w) {
  int I = f / 2;
  int nb = (f % 2 == 0) ? I - 1 : I + 1;
  J[0] = I;
  if (nb >= 0 && nb < nc) {
    w[0] = ip.own;
    if (ip.nb == 0.0) return 1;
    J[1] = nb;
    w[1] = ip.nb;
    return 2;
  }
  w[0] = ip.wb;
  return 1;
}

Stencil9 galerkin(const Stencil9 &A, double wb) { return galerkin(A, Interp{0.75, 0.25, wb}); }

Stencil9 galerkin(const Stencil9 &A, const Interp &ip) {
  const int nx = A.nx, ny = A.ny, ncx = nx / 2, ncy = ny / 2;
  Stencil9 C;
  C.resize(ncx, ncy);
  for (int Iy = 0; Iy < ncy; ++Iy)
    for (int Ix = 0; Ix < ncx; ++Ix) {
      double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          int px = 2 * Ix + a, py = 2 * Iy + b;
          size_t p = (size_t)py * nx + px;
          for (int k = 0; k < 9; ++k) {
            double v = A.c[k][p];
            if (v == 0.0) continue;
            int qx = px + kdx(k), qy = py + kdy(k);
            if (qx < 0 || qx >= nx || qy < 0 || qy >= ny) continue;
            int Jx[2], Jy[2];
            double wx[2], wy[2];
            int mx = interp1d(qx, ncx, ip, Jx, wx), my = interp1d(qy, ncy, ip, Jy, wy);
            for (int t = 0; t < my; ++t)
              for (int u = 0; u < mx; ++u) {
                int ox = Jx[u] - Ix, oy = Jy[t] - Iy;  // in [-1, 1]
                acc[(oy + 1) * 3 + (ox + 1)] += v * wx[u] * wy[t];
              }
          }
        }
      size_t I = (size_t)Iy * ncx + Ix;
      for (int k = 0; k < 9; ++k) C.c[k][I] = acc[k];
    }
  return C;
}

Stencil9 axpy_stencil(const Stencil9 &a, double t, const Stencil9 &b) {
  Stencil9 r;
  r.resize(a.nx, a.ny);
  for (int k = 0; k < 9; ++k)
    for (size_t p = 0; p < a.size(); ++p) r.c[k][p] = a.c[k][p] + t * b.c[k][p];
  return r;
}

bool classify(const Stencil9 &A, double tol, double cls[9][9]) {
  bool seen[9] = {false, false, false, false, false, false, false, false, false};
  for (int q = 0; q < 9; ++q)
    for (int k = 0; k < 9; ++k) cls[q][k] = 0.0;
  double scale = 0.0;
  for (int k = 0; k < 9; ++k)
    for (double v : A.c[k]) scale = std::max(scale, std::fabs(v));
  if (scale == 0.0) scale = 1.0;
  for (int j = 0; j < A.ny; ++j)
    for (int i = 0; i < A.nx; ++i) {
      int q = node_class(i, j, A.nx, A.ny);
      size_t p = (size_t)j * A.nx + i;
      if (!seen[q]) {
        seen[q] = true;
        for (int k = 0; k < 9; ++k) cls[q][k] = A.c[k][p];
      } else {
        for (int k = 0; k < 9; ++k)
          if (std::fabs(cls[q][k] - A.c[k][p]) > tol * scale) return false;
      }
    }
  return true;
}

bool is_symmetric(const Stencil9 &A, double tol) {
  double scale = 0.0;
  for (int k = 0; k < 9; ++k)
    for (double v : A.c[k]) scale = std::max(scale, std::fabs(v));
  for (int j = 0; j < A.ny; ++j)
    for (int i = 0; i < A.nx; ++i)
      for (int k = 0; k < 9; ++k) {
        int qi = i + kdx(k), qj = j + kdy(k);
        if (qi < 0 || qi >= A.nx || qj < 0 || qj >= A.ny) continue;
        double a = A.c[k][(size_t)j * A.nx + i];
        double b = A.c[8 - k][(size_t)qj * A.nx + qi];
        if (std::fabs(a - b) > tol * scale) return false;
      }
  return true;
}

bool dense_inverse(const Stencil9 &A, std::vector<double> &inv) {
  const int n = A.nx * A.ny;
  std::vector<double> M((size_t)n * n, 0.0);
  for (int j = 0; j < A.ny; ++j)
    for (int i = 0; i < A.nx; ++i) {
      int r = j * A.nx + i;
      for (int k = 0; k < 9; ++k) {
        int qi = i + kdx(k), qj = j + kdy(k);
        if (qi < 0 || qi >= A.nx || qj < 0 || qj >= A.ny) continue;
        M[(size_t)r * n + qj * A.nx + qi] += A.c[k][r];
      }
    }
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    double best = std::fabs(M[(size_t)col * n + col]);
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(M[(size_t)r * n + col]) > best) {
        best = std::fabs(M[(size_t)r * n + col]);
        piv = r;
      }
    if (!(best > 0.0)) return false;
    if (piv != col)
      for (int c = 0; c < n; ++c) {
        std::swap(M[(size_t)piv * n + c], M[(size_t)col * n + c]);
        std::swap(inv[(size_t)piv * n + c], inv[(size_t)col * n + c]);
      }
    double p = M[(size_t)col * n + col];
    for (int c = 0; c < n; ++c) {
      M[(size_t)col * n + c] /= p;
      inv[(size_t)col * n + c] /= p;
    }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      double f = M[(size_t)r * n + col];
      if (f == 0.0) continue;
      for (int c = 0; c < n; ++c) {
        M[(size_t)r * n + c] -= f * M[(size_t)col * n + c];
        inv[(size_t)r * n + c] -= f * inv[(size_t)col * n + c];
      }
    }
  }
  return true;
}

}  // namespace irk
