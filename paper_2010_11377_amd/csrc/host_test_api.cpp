// C entry points into the host-side setup code, built with g++ into
// libirk_host_test.so so that the CPU test suite can check the host logic
// (stencil extraction, Galerkin coarsening, boundary classes, LDU) without a
// GPU.  Not part of libirk.so.
#include <cstring>
#include <string>

#include "host_setup.hpp"

using irk::Stencil9;

namespace {
void to_flat(const Stencil9 &S, double *out) {
  const size_t n = S.size();
  for (int k = 0; k < 9; ++k) std::memcpy(out + (size_t)k * n, S.c[k].data(), n * sizeof(double));
}
Stencil9 from_flat(int nx, int ny, const double *in) {
  Stencil9 S;
  S.resize(nx, ny);
  const size_t n = S.size();
  for (int k = 0; k < 9; ++k) std::memcpy(S.c[k].data(), in + (size_t)k * n, n * sizeof(double));
  return S;
}
thread_local std::string g_err;
}  // namespace

extern "C" {

// CSR -> 9 coefficient arrays (k-major, 9 * nx * ny doubles).  0 on success.
int irkh_csr_to_stencil(int n, const int *rowptr, const int *colind, const double *val, int nx,
                        int ny, double *out) {
  Stencil9 S;
  if (!irk::csr_to_stencil(n, rowptr, colind, val, nx, ny, S, g_err)) return -1;
  to_flat(S, out);
  return 0;
}

const char *irkh_last_error() { return g_err.c_str(); }

// Galerkin coarse operator of a 9-point stencil (nx, ny even) on hierarchy
// level `level` (which fixes the boundary interpolation weight).
int irkh_galerkin(int nx, int ny, int level, const double *in, double *out) {
  if (nx % 2 || ny % 2 || level < 0) return -1;
  Stencil9 C = irk::galerkin(from_flat(nx, ny, in), irk::boundary_weight(level));
  to_flat(C, out);
  return 0;
}

// The same with piecewise-constant interpolation (P = R^T).
int irkh_galerkin_constant(int nx, int ny, const double *in, double *out) {
  if (nx % 2 || ny % 2) return -1;
  Stencil9 C = irk::galerkin(from_flat(nx, ny, in), irk::constant_interp());
  to_flat(C, out);
  return 0;
}

// 1 if the operator has one coefficient set per boundary class (cls: 81).
int irkh_classify(int nx, int ny, const double *in, double tol, double *cls) {
  double c[9][9];
  bool ok = irk::classify(from_flat(nx, ny, in), tol, c);
  for (int q = 0; q < 9; ++q)
    for (int k = 0; k < 9; ++k) cls[q * 9 + k] = c[q][k];
  return ok ? 1 : 0;
}

int irkh_is_symmetric(int nx, int ny, const double *in, double tol) {
  return irk::is_symmetric(from_flat(nx, ny, in), tol) ? 1 : 0;
}

// dense inverse (n x n, n = nx*ny) of the stencil operator.
int irkh_dense_inverse(int nx, int ny, const double *in, double *out) {
  std::vector<double> inv;
  if (!irk::dense_inverse(from_flat(nx, ny, in), inv)) return -1;
  std::memcpy(out, inv.data(), inv.size() * sizeof(double));
  return 0;
}

int irkh_coefficient_matrix(int s, const double *A, int kind, double *At) {
  return irk::coefficient_matrix(s, A, kind, At);
}

}  // extern "C"
