// Host-side setup of the IRK stage solver: tableau factorisation, stencil
// extraction from CSR, the Galerkin AMG hierarchy and the coarse inverse.
// Plain C++17 (no HIP), so it also builds with g++ for CPU tests.
#pragma once
#include <string>
#include <vector>

namespace irk {

// 9-point stencil on an nx x ny grid: (A x)_P = sum_k c[k][P] x[P + off_k]
// with off_k = (dx, dy), k = (dy + 1) * 3 + (dx + 1), and x = 0 outside the
// grid.  Coefficients that would reach outside the grid are zero.
struct Stencil9 {
  int nx = 0, ny = 0;
  std::vector<double> c[9];
  void resize(int nx_, int ny_);
  size_t size() const { return (size_t)nx * ny; }
};

inline int kdx(int k) { return k % 3 - 1; }
inline int kdy(int k) { return k / 3 - 1; }

// Boundary class of a node: 3 * cy + cx with cx = 0 (first column),
// 1 (interior), 2 (last column); likewise cy for rows.
inline int node_class(int i, int j, int nx, int ny) {
  int cx = (i == 0) ? 0 : (i == nx - 1 ? 2 : 1);
  int cy = (j == 0) ? 0 : (j == ny - 1 ? 2 : 1);
  return 3 * cy + cx;
}

// LDU factorisation without pivoting (Sec. 4.1).  Returns 0, -1 (bad s) or
// -2 (pivot |d_k| <= 64 eps max|a|).
int ldu_factor(int s, const double *A, double *L, double *d, double *U);

// Preconditioner coefficient matrix A~ for kind 0 = LD, 1 = DU, 2 = GSL (tril),
// 3 = J (diag) (Sec. 4, (4.2); Sec. 4.1, (4.3)).  Returns the ldu_factor code.
int coefficient_matrix(int s, const double *A, int kind, double *At);

// CSR (0-based) on an nx x ny grid into a 9-point stencil.  Fails on a
// coupling outside the 3 x 3 neighbourhood or a malformed CSR.
bool csr_to_stencil(int n, const int *rowptr, const int *colind, const double *val, int nx,
                    int ny, Stencil9 &out, std::string &err);

// Identity stencil.
Stencil9 identity_stencil(int nx, int ny);

// Interpolation weight of the outermost coarse node at the outermost fine
// node of level `level` (0 = finest): the grids are interior nodes of a
// Dirichlet problem, the boundary one fine spacing beyond the outermost
// finest node, and each 2 x 2 coarsening moves the outermost node half a
// spacing inwards, so the weight is the distance ratio
// (2^l + 1) / (2^(l+1) + 1).
double boundary_weight(int level);

// Galerkin coarse operator R A P for 2 x 2 coarsening (nx, ny even):
// P is the tensor product of the 1-D linear interpolation between cell
// centres (fine 2I gets 3/4 of coarse I and 1/4 of I-1, fine 2I+1 gets 3/4
// of I and 1/4 of I+1; the outermost fine node gets wb of its coarse node
// and nothing from beyond the grid) and R = P0^T is the sum over the 2 x 2
// aggregate.
Stencil9 galerkin(const Stencil9 &A, double wb);

// Prolongation weights of one level: a fine node takes `own` of its coarse
// parent and `nb` of the next coarse node on its side, per direction; an
// outermost fine node (no such coarse node) takes `wb` of its parent.
// Restriction is the transpose of the piecewise-constant prolongation (the
// sum over the 2 x 2 cell) in both cases.
struct Interp {
  double own, nb, wb;
};
Interp linear_interp(int level);  // 3/4, 1/4, boundary_weight(level)
Interp constant_interp();         // 1, 0, 1: P = R^T
Stencil9 galerkin(const Stencil9 &A, const Interp &ip);

// a + t * b, entrywise.
Stencil9 axpy_stencil(const Stencil9 &a, double t, const Stencil9 &b);

// True if every node of each boundary class carries the same 9 coefficients
// (relative tolerance tol); fills cls[9][9] (class, coefficient).
bool classify(const Stencil9 &A, double tol, double cls[9][9]);

// True if the operator is symmetric: c[k][P] == c[8-k][P + off_k].
bool is_symmetric(const Stencil9 &A, double tol);

// Dense inverse (row-major n x n) of the stencil operator, by Gauss-Jordan
// with partial pivoting.  Returns false if singular.
bool dense_inverse(const Stencil9 &A, std::vector<double> &inv);

}  // namespace irk
