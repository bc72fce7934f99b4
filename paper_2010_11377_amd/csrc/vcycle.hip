// Fused AMG V-cycle kernels (gfx950).
//
// One V(nu, nu) cycle on a stage block D = S_l + tau K_l (Sec. 4.2: one
// V-cycle per diagonal block) with red-black Gauss-Seidel smoothing (or, with
// OpView::jw > 0, damped Jacobi: x += jw D^-1 (b - A x), every node from the
// old values, nu sweeps before and after the coarse correction), from a
// zero initial guess.  The smoother is the memory-bound part, so several
// sweeps are fused into one pass over HBM with LDS temporal blocking: a tile
// of the grid plus a halo is staged in LDS, every sweep shrinks the region
// where values are exact by one node, and only the tile interior is
// written.  Per level and V-cycle this gives two passes:
//
//   down: x = nu pre-sweeps from 0 (in LDS), rc = R (b - D x)
//         reads b, writes rc                          (1 + 1/4 words/node)
//   up:   recompute x from b (cheaper than storing it), x += P ec,
//         nu post-sweeps, write x
//         reads b and ec, writes x                    (2 + 1/4 words/node)
//
// The smoother colours nodes by (i + j) mod 2; every sweep loop enumerates
// only the nodes of its colour.  For a 9-point coarse operator nodes of one
// colour also couple diagonally; their new values are computed from the old
// ones (Jacobi within a colour), staged in registers and written after a
// barrier, so the result does not depend on thread order.
//
// Constant-coefficient operators (9 boundary classes x 9 coefficients) are
// staged in LDS once per workgroup; per-node operators are read through the
// cache.
//
// All levels with at most kTailMax nodes run in one workgroup (k_vtail),
// which keeps the whole remaining hierarchy in LDS, including the dense
// coarsest-level solve.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace irk {
namespace {

struct Row8 {
  double c[8];
};

__device__ __forceinline__ int cls_of(int i, int j, int nx, int ny) {
  const int cx = (i == 0) ? 0 : (i == nx - 1 ? 2 : 1);
  const int cy = (j == 0) ? 0 : (j == ny - 1 ? 2 : 1);
  return 3 * cy + cx;
}

__device__ __forceinline__ constexpr bool used(int npt, int k) {
  return npt == 9 || k == 1 || k == 3 || k == 4 || k == 5 || k == 7;
}

// The coefficients of node (gx, gy) into a[9] (entries not in the stencil
// are left unset).
template <typename T, int NPT, bool CLS>
__device__ __forceinline__ void node_coefs(const T *cls_lds, const T *ci, const OpView<T> &D,
                                           int gx, int gy, T *a) {
  if (CLS) {
    // interior nodes (almost all) take the interior class from registers
    const bool inner = gx > 0 && gy > 0 && gx < D.nx - 1 && gy < D.ny - 1;
    const T *c = cls_lds + 9 * cls_of(gx, gy, D.nx, D.ny);
#pragma unroll
    for (int k = 0; k < 9; ++k)
      if (used(NPT, k)) a[k] = inner ? ci[k] : c[k];
  } else {
    const size_t N = (size_t)D.nx * D.ny, p = (size_t)gy * D.nx + gx;
#pragma unroll
    for (int k = 0; k < 9; ++k)
      if (used(NPT, k)) a[k] = D.arr[(size_t)k * N + p];
  }
}

// b - sum_{k != centre} a_k x_k at LDS position (lx, ly), row pitch W.
template <typename T, int NPT, int W>
__device__ __forceinline__ T offdiag_rhs(const T *a, const T *sx, const T *sb, int lx, int ly) {
  T acc = sb[ly * W + lx];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if (k == 4 || !used(NPT, k)) continue;
    acc -= a[k] * sx[(ly + k / 3 - 1) * W + lx + k % 3 - 1];
  }
  return acc;
}

template <typename T>
__device__ __forceinline__ void stage_cls(const T *__restrict__ g, T *lds) {
  if (threadIdx.x < 81) lds[threadIdx.x] = g[threadIdx.x];
}

// interior-class coefficients into registers (after the staging barrier)
template <typename T, bool CLS>
__device__ __forceinline__ void interior_coefs(const T *lds, T *ci) {
#pragma unroll
  for (int k = 0; k < 9; ++k) ci[k] = CLS ? lds[36 + k] : T(0);
}

// One colour sweep over the LDS region [m, W-m) x [m, HH-m) (grid nodes only).
template <typename T, int NPT, bool CLS, int W, int HH, int NT>
__device__ __forceinline__ void tile_sweep(const OpView<T> &D, const T *cls_lds, const T *ci, T *sx,
                                           const T *sb, int X0, int Y0, int color, int m) {
  const int w = W - 2 * m, hgt = HH - 2 * m, half = (w + 1) / 2;
  const int par0 = X0 + m;
  if (NPT == 5) {
    // nodes of one colour do not couple: update in place
    for (int q = threadIdx.x; q < half * hgt; q += NT) {
      const int ly = m + q / half;
      const int gy = Y0 + ly;
      const int lx = m + 2 * (q % half) + ((color - par0 - gy) & 1);
      const int gx = X0 + lx;
      if (lx >= W - m || gx < 0 || gy < 0 || gx >= D.nx || gy >= D.ny) continue;
      T a[9];
      node_coefs<T, NPT, CLS>(cls_lds, ci, D, gx, gy, a);
      sx[ly * W + lx] = offdiag_rhs<T, NPT, W>(a, sx, sb, lx, ly) / a[4];
    }
    __syncthreads();
  } else {
    constexpr int MAXP = (((W + 1) / 2) * HH + NT - 1) / NT;
    T nv[MAXP];
#pragma unroll
    for (int it = 0; it < MAXP; ++it) {
      const int q = threadIdx.x + it * NT;
      nv[it] = T(0);
      if (q >= half * hgt) continue;
      const int ly = m + q / half;
      const int gy = Y0 + ly;
      const int lx = m + 2 * (q % half) + ((color - par0 - gy) & 1);
      const int gx = X0 + lx;
      if (lx >= W - m || gx < 0 || gy < 0 || gx >= D.nx || gy >= D.ny) continue;
      T a[9];
      node_coefs<T, NPT, CLS>(cls_lds, ci, D, gx, gy, a);
      nv[it] = offdiag_rhs<T, NPT, W>(a, sx, sb, lx, ly) / a[4];
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < MAXP; ++it) {
      const int q = threadIdx.x + it * NT;
      if (q >= half * hgt) continue;
      const int ly = m + q / half;
      const int gy = Y0 + ly;
      const int lx = m + 2 * (q % half) + ((color - par0 - gy) & 1);
      const int gx = X0 + lx;
      if (lx >= W - m || gx < 0 || gy < 0 || gx >= D.nx || gy >= D.ny) continue;
      sx[ly * W + lx] = nv[it];
    }
    __syncthreads();
  }
}

// One damped Jacobi sweep over the LDS region [m, W-m) x [m, HH-m): every
// grid node takes x + jw (b - A x) / d from the old values (computed into
// registers, written after a barrier).
template <typename T, int NPT, bool CLS, int W, int HH, int NT>
__device__ __forceinline__ void tile_jsweep(const OpView<T> &D, const T *cls_lds, const T *ci,
                                            T *sx, const T *sb, int X0, int Y0, int m) {
  const int w = W - 2 * m, hgt = HH - 2 * m;
  constexpr int MAXP = (W * HH + NT - 1) / NT;
  T nv[MAXP];
#pragma unroll
  for (int it = 0; it < MAXP; ++it) {
    const int q = threadIdx.x + it * NT;
    nv[it] = T(0);
    if (q >= w * hgt) continue;
    const int lx = m + q % w, ly = m + q / w;
    const int gx = X0 + lx, gy = Y0 + ly;
    if (gx < 0 || gy < 0 || gx >= D.nx || gy >= D.ny) continue;
    T a[9];
    node_coefs<T, NPT, CLS>(cls_lds, ci, D, gx, gy, a);
    const T xo = sx[ly * W + lx];
    nv[it] = xo + D.jw * ((offdiag_rhs<T, NPT, W>(a, sx, sb, lx, ly) - a[4] * xo) / a[4]);
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < MAXP; ++it) {
    const int q = threadIdx.x + it * NT;
    if (q >= w * hgt) continue;
    const int lx = m + q % w, ly = m + q / w;
    const int gx = X0 + lx, gy = Y0 + ly;
    if (gx < 0 || gy < 0 || gx >= D.nx || gy >= D.ny) continue;
    sx[ly * W + lx] = nv[it];
  }
  __syncthreads();
}

// Stage a grid vector on the LDS region whose origin is grid node (X0, Y0),
// zero outside the grid.  A plain copy loop, so that many loads are in flight.
template <typename T, int W, int HH, int NT>
__device__ __forceinline__ void tile_load(const T *__restrict__ g, T *lds, int X0, int Y0, int nx,
                                          int ny) {
#pragma unroll 4
  for (int q = threadIdx.x; q < W * HH; q += NT) {
    const int gx = X0 + q % W, gy = Y0 + q / W;
    lds[q] = (gx >= 0 && gy >= 0 && gx < nx && gy < ny) ? g[(size_t)gy * nx + gx] : T(0);
  }
}

// x = 0 followed by the first half sweep (colour 0 gets b / d), then the
// remaining 2 nu - 1 half sweeps.  Afterwards x is exact on margin >= 2nu-1.
template <typename T, int NPT, bool CLS, int NU, int W, int HH, int NT, bool JAC = false>
__device__ __forceinline__ void tile_presmooth(const OpView<T> &D, const T *cls_lds, const T *ci, T *sx,
                                               const T *sb, int X0, int Y0) {
  if constexpr (JAC) {
    // Jacobi from x = 0: nu sweeps, exact on margin nu afterwards
    for (int q = threadIdx.x; q < W * HH; q += NT) sx[q] = T(0);
    __syncthreads();
    for (int k = 1; k <= NU; ++k) tile_jsweep<T, NPT, CLS, W, HH, NT>(D, cls_lds, ci, sx, sb, X0, Y0, k);
    return;
  }
  for (int q = threadIdx.x; q < W * HH; q += NT) {
    const int gx = X0 + q % W, gy = Y0 + q / W;
    T xv = T(0);
    if (((gx + gy) & 1) == 0 && gx >= 0 && gy >= 0 && gx < D.nx && gy < D.ny) {
      T a[9];
      node_coefs<T, NPT, CLS>(cls_lds, ci, D, gx, gy, a);
      xv = sb[q] / a[4];
    }
    sx[q] = xv;
  }
  __syncthreads();
#pragma unroll
  for (int k = 1; k < 2 * NU; ++k)
    tile_sweep<T, NPT, CLS, W, HH, NT>(D, cls_lds, ci, sx, sb, X0, Y0, k & 1, k);
}

// rc = R (b - D x) for the coarse nodes of the tile (output region at margin H).
template <typename T, int NPT, bool CLS, int TX, int TY, int H, int W, int NT>
__device__ __forceinline__ void tile_restrict(const OpView<T> &D, const T *cls_lds, const T *ci,
                                              const T *sx,
                                              const T *sb, int X0, int Y0, T *__restrict__ rc) {
  const int ncx = D.nx / 2, ncy = D.ny / 2;
  for (int q = threadIdx.x; q < (TX / 2) * (TY / 2); q += NT) {
    const int qi = q % (TX / 2), qj = q / (TX / 2);
    const int I = (X0 + H) / 2 + qi, J = (Y0 + H) / 2 + qj;  // tile origin / 2
    if (I >= ncx || J >= ncy) continue;
    T acc = T(0);
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int a2 = 0; a2 < 2; ++a2) {
        const int lx = H + 2 * qi + a2, ly = H + 2 * qj + bb;
        T a[9];
        node_coefs<T, NPT, CLS>(cls_lds, ci, D, X0 + lx, Y0 + ly, a);
        acc += offdiag_rhs<T, NPT, W>(a, sx, sb, lx, ly) - a[4] * sx[ly * W + lx];
      }
    rc[(size_t)J * ncx + I] = acc;
  }
}

constexpr int kNT = 256;

template <typename T, int NPT, bool CLS, int NU, int TX, int TY, bool JAC>
__global__ void __launch_bounds__(kNT)
    k_vdown(OpView<T> D, const T *__restrict__ b, T *__restrict__ rc) {
  constexpr int H = 2 * NU;
  constexpr int W = TX + 2 * H, HH = TY + 2 * H;
  __shared__ T sb[W * HH];
  __shared__ T sx[W * HH];
  __shared__ T scls[81];
  if (CLS) stage_cls(D.cls, scls);
  const Tile2 tile = xcd_tile();
  const int X0 = tile.x * TX - H, Y0 = tile.y * TY - H;
  tile_load<T, W, HH, kNT>(b, sb, X0, Y0, D.nx, D.ny);
  __syncthreads();
  T ci[9];
  interior_coefs<T, CLS>(scls, ci);
  tile_presmooth<T, NPT, CLS, NU, W, HH, kNT, JAC>(D, scls, ci, sx, sb, X0, Y0);
  tile_restrict<T, NPT, CLS, TX, TY, H, W, kNT>(D, scls, ci, sx, sb, X0, Y0, rc);
}

// The finest-level down pass fused with the block-substitution coupling of
// stage i (Sec. 4.2): b = scale_j v_i - K (sum_k C_ik z_k) is formed in LDS
// from v and the earlier stage vectors (the combination on the region plus
// one node, K applied from LDS), written out for the up pass, and smoothed.
template <typename T, int NPT, bool CLS, int NPTK, int NU, int TX, int TY>
__global__ void __launch_bounds__(kNT)
    k_vdown_couple(OpView<T> D, OpView<T> K, const double *__restrict__ v,
                   const double *__restrict__ scale_j, const T *__restrict__ z, Row8 crow, int s,
                   int i, T *__restrict__ b_out, T *__restrict__ rc) {
  constexpr int H = 2 * NU;
  constexpr int W = TX + 2 * H, HH = TY + 2 * H;
  constexpr int WE = W + 2, HE = HH + 2;
  __shared__ T sb[W * HH];
  __shared__ T sx[W * HH];
  __shared__ T sc[WE * HE];
  __shared__ T scls[81];
  __shared__ T sclk[81];
  if (CLS) {
    stage_cls(D.cls, scls);
    stage_cls(K.cls, sclk);
  }
  const Tile2 tile = xcd_tile();
  const int X0 = tile.x * TX - H, Y0 = tile.y * TY - H;
  const size_t N = (size_t)D.nx * D.ny;
  const double sc_j = *scale_j;
  bool any = false;
#pragma unroll
  for (int k = 0; k < kMaxStages; ++k)
    if (k < s && crow.c[k] != 0.0) any = true;
  // v_i on the region
#pragma unroll 4
  for (int q = threadIdx.x; q < W * HH; q += kNT) {
    const int gx = X0 + q % W, gy = Y0 + q / W;
    sb[q] = (gx >= 0 && gy >= 0 && gx < D.nx && gy < D.ny)
                ? T(sc_j * v[(size_t)i * N + (size_t)gy * D.nx + gx])
                : T(0);
  }
  __syncthreads();  // class tables staged
  T ci[9], cik[9];
  interior_coefs<T, CLS>(scls, ci);
  interior_coefs<T, CLS>(sclk, cik);
  if (any) {
    // the combination sum_k C_ik z_k on the region plus one node
    for (int q = threadIdx.x; q < WE * HE; q += kNT) {
      const int gx = X0 - 1 + q % WE, gy = Y0 - 1 + q / WE;
      T c = T(0);
      if (gx >= 0 && gy >= 0 && gx < D.nx && gy < D.ny) {
        const size_t p = (size_t)gy * D.nx + gx;
#pragma unroll
        for (int k = 0; k < kMaxStages; ++k)
          if (k < s && crow.c[k] != 0.0) c += T(crow.c[k]) * z[(size_t)k * N + p];
      }
      sc[q] = c;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < W * HH; q += kNT) {
      const int lx = q % W, ly = q / W;
      const int gx = X0 + lx, gy = Y0 + ly;
      if (gx < 0 || gy < 0 || gx >= D.nx || gy >= D.ny) continue;
      T a[9];
      node_coefs<T, NPTK, CLS>(sclk, cik, K, gx, gy, a);
      T kc = T(0);
#pragma unroll
      for (int k = 0; k < 9; ++k)
        if (used(NPTK, k)) kc += a[k] * sc[(ly + 1 + k / 3 - 1) * WE + lx + 1 + k % 3 - 1];
      sb[q] -= kc;
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < TX * TY; q += kNT) {
    const int lx = H + q % TX, ly = H + q / TX;
    const int gx = X0 + lx, gy = Y0 + ly;
    if (gx >= D.nx || gy >= D.ny) continue;
    b_out[(size_t)gy * D.nx + gx] = sb[ly * W + lx];
  }
  tile_presmooth<T, NPT, CLS, NU, W, HH, kNT>(D, scls, ci, sx, sb, X0, Y0);
  tile_restrict<T, NPT, CLS, TX, TY, H, W, kNT>(D, scls, ci, sx, sb, X0, Y0, rc);
}

// P ec at fine node (fx, fy) from a staged coarse tile with origin (CX0, CY0)
// and pitch CW: per direction pa of the own coarse node and pn of the next
// one (3/4 and 1/4 for linear, 1 and 0 for piecewise-constant interpolation);
// an outermost fine node (no next coarse node) takes pw of its own.
template <typename T>
__device__ __forceinline__ T prolong_value(const T *ec, int CW, int CX0, int CY0, int fx, int fy,
                                           int ncx, int ncy, T pw, T pa, T pn) {
  const int Ix = fx / 2, Iy = fy / 2;
  const int nbx = (fx & 1) ? Ix + 1 : Ix - 1;
  const int nby = (fy & 1) ? Iy + 1 : Iy - 1;
  const bool hx = nbx >= 0 && nbx < ncx && pn != T(0), hy = nby >= 0 && nby < ncy && pn != T(0);
  const T wx = (nbx >= 0 && nbx < ncx) ? pa : pw, wy = (nby >= 0 && nby < ncy) ? pa : pw;
  const int lx = Ix - CX0, ly = Iy - CY0, nlx = nbx - CX0, nly = nby - CY0;
  T v = wx * wy * ec[ly * CW + lx];
  if (hx) v += pn * wy * ec[ly * CW + nlx];
  if (hy) v += wx * pn * ec[nly * CW + lx];
  if (hx && hy) v += pn * pn * ec[nly * CW + nlx];
  return v;
}

template <typename T, int NPT, bool CLS, int NU, int TX, int TY, bool JAC>
__global__ void __launch_bounds__(kNT)
    k_vup(OpView<T> D, const T *__restrict__ b, const T *__restrict__ ec, T *__restrict__ x) {
  constexpr int H = 4 * NU - 1;
  constexpr int W = TX + 2 * H, HH = TY + 2 * H;
  constexpr int m = 2 * NU - 1;  // margin where the pre-smoothed x is exact
  constexpr int CW = (W - 2 * m) / 2 + 4, CH = (HH - 2 * m) / 2 + 4;
  __shared__ T sb[W * HH];
  __shared__ T sx[W * HH];
  __shared__ T se[CW * CH];
  __shared__ T scls[81];
  if (CLS) stage_cls(D.cls, scls);
  const Tile2 tile = xcd_tile();
  const int X0 = tile.x * TX - H, Y0 = tile.y * TY - H;
  const int ncx = D.nx / 2, ncy = D.ny / 2;
  // coarse nodes that interpolate onto the fine region at margin m
  const int CX0 = ((X0 + m) >> 1) - 1, CY0 = ((Y0 + m) >> 1) - 1;
  tile_load<T, W, HH, kNT>(b, sb, X0, Y0, D.nx, D.ny);
  tile_load<T, CW, CH, kNT>(ec, se, CX0, CY0, ncx, ncy);
  __syncthreads();
  T ci[9];
  interior_coefs<T, CLS>(scls, ci);
  tile_presmooth<T, NPT, CLS, NU, W, HH, kNT, JAC>(D, scls, ci, sx, sb, X0, Y0);
  {
    constexpr int w = W - 2 * m, hgt = HH - 2 * m;
    for (int q = threadIdx.x; q < w * hgt; q += kNT) {
      const int lx = m + q % w, ly = m + q / w;
      const int gx = X0 + lx, gy = Y0 + ly;
      if (gx < 0 || gy < 0 || gx >= D.nx || gy >= D.ny) continue;
      sx[ly * W + lx] += prolong_value(se, CW, CX0, CY0, gx, gy, ncx, ncy, D.pw, D.pa, D.pn);
    }
    __syncthreads();
  }
  if constexpr (JAC) {
    for (int k = 0; k < NU; ++k)
      tile_jsweep<T, NPT, CLS, W, HH, kNT>(D, scls, ci, sx, sb, X0, Y0, 2 * NU + k);
  } else {
#pragma unroll
    for (int k = 0; k < 2 * NU; ++k)
      tile_sweep<T, NPT, CLS, W, HH, kNT>(D, scls, ci, sx, sb, X0, Y0, (k & 1) ^ 1, 2 * NU + k);
  }
  for (int q = threadIdx.x; q < TX * TY; q += kNT) {
    const int lx = H + q % TX, ly = H + q / TX;
    const int gx = X0 + lx, gy = Y0 + ly;
    if (gx >= D.nx || gy >= D.ny) continue;
    x[(size_t)gy * D.nx + gx] = sx[ly * W + lx];
  }
}

// ---------------------------------------------------------------------------
// the coarse tail of the V-cycle in one workgroup

constexpr int kTailThreads = 1024;
constexpr int kTailPer = (kTailMax / 2 + kTailThreads - 1) / kTailThreads;  // per colour

// x_p of a tail level after one colour sweep (resid = false) or the residual
// b_p - (D x)_p (resid = true).
template <typename T, bool CLS>
__device__ __forceinline__ T tail_node(const TailDesc<T> &td, const T *cls_lds, int l,
                                       const T *sx, const T *sb, int i, int j, bool resid) {
  const int nx = td.nx[l], ny = td.ny[l];
  const size_t N = (size_t)nx * ny, p = (size_t)j * nx + i;
  const T *c = CLS ? cls_lds + 81 * l + 9 * cls_of(i, j, nx, ny) : nullptr;
  const T *arr = td.arr[l];
  T acc = sb[p];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if (k == 4 && !resid) continue;
    const int ii = i + k % 3 - 1, jj = j + k / 3 - 1;
    if (ii < 0 || jj < 0 || ii >= nx || jj >= ny) continue;
    const T a = CLS ? c[k] : arr[(size_t)k * N + p];
    acc -= a * sx[(size_t)jj * nx + ii];
  }
  if (resid) return acc;
  return acc / (CLS ? c[4] : arr[(size_t)4 * N + p]);
}

template <typename T, bool CLS>
__device__ void tail_sweep(const TailDesc<T> &td, const T *cls_lds, int l, T *sx, const T *sb,
                           int color) {
  const int nx = td.nx[l], ny = td.ny[l], half = (nx + 1) / 2;
  T nv[kTailPer];
#pragma unroll
  for (int it = 0; it < kTailPer; ++it) {
    const int q = threadIdx.x + it * kTailThreads;
    nv[it] = T(0);
    if (q >= half * ny) continue;
    const int j = q / half, i = 2 * (q % half) + ((color - j) & 1);
    if (i >= nx) continue;
    nv[it] = tail_node<T, CLS>(td, cls_lds, l, sx, sb, i, j, false);
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kTailPer; ++it) {
    const int q = threadIdx.x + it * kTailThreads;
    if (q >= half * ny) continue;
    const int j = q / half, i = 2 * (q % half) + ((color - j) & 1);
    if (i >= nx) continue;
    sx[(size_t)j * nx + i] = nv[it];
  }
  __syncthreads();
}

// One damped Jacobi sweep of a tail level (every node from the old values).
template <typename T, bool CLS>
__device__ void tail_jsweep(const TailDesc<T> &td, const T *cls_lds, int l, T *sx, const T *sb) {
  const int nx = td.nx[l], ny = td.ny[l], n = nx * ny;
  T nv[2 * kTailPer];
#pragma unroll
  for (int it = 0; it < 2 * kTailPer; ++it) {
    const int p = threadIdx.x + it * kTailThreads;
    nv[it] = T(0);
    if (p >= n) continue;
    const int i = p % nx, j = p / nx;
    // x + jw (b - D x) / d = x + jw ((b - offdiag x) / d - x)
    nv[it] = sx[p] + td.jw * (tail_node<T, CLS>(td, cls_lds, l, sx, sb, i, j, false) - sx[p]);
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < 2 * kTailPer; ++it) {
    const int p = threadIdx.x + it * kTailThreads;
    if (p < n) sx[p] = nv[it];
  }
  __syncthreads();
}

template <typename T, bool CLS, bool JAC>
__global__ void __launch_bounds__(kTailThreads)
    k_vtail(TailDesc<T> td, const T *__restrict__ b_top, T *__restrict__ x_top, int nu) {
  extern __shared__ unsigned char smem_raw[];
  T *sm = reinterpret_cast<T *>(smem_raw);
  const int L = td.nlev;
  // LDS: level arrays (b then x per level), the reduction buffer of the
  // dense solve (kTailThreads), then the class tables (81 per level)
  T *red = sm + td.off[L];
  T *cls_lds = red + kTailThreads;
  if (CLS)
    for (int q = threadIdx.x; q < 81 * (L - 1); q += kTailThreads) cls_lds[q] = td.cls[q / 81][q % 81];
  {
    const int n = td.nx[0] * td.ny[0];
    for (int p = threadIdx.x; p < n; p += kTailThreads) sm[td.off[0] + p] = b_top[p];
  }
  __syncthreads();
  // down
  for (int l = 0; l + 1 < L; ++l) {
    T *sb = sm + td.off[l];
    const int nx = td.nx[l], ny = td.ny[l], n = nx * ny;
    T *sx = sb + n;
    for (int p = threadIdx.x; p < n; p += kTailThreads) sx[p] = T(0);
    __syncthreads();
    for (int sw = 0; sw < nu; ++sw) {
      if constexpr (JAC) {
        tail_jsweep<T, CLS>(td, cls_lds, l, sx, sb);
      } else {
        tail_sweep<T, CLS>(td, cls_lds, l, sx, sb, 0);
        tail_sweep<T, CLS>(td, cls_lds, l, sx, sb, 1);
      }
    }
    const int ncx = td.nx[l + 1], ncy = td.ny[l + 1];
    T *sbc = sm + td.off[l + 1];
    for (int I = threadIdx.x; I < ncx * ncy; I += kTailThreads) {
      const int Ix = I % ncx, Iy = I / ncx;
      T acc = T(0);
      for (int bb = 0; bb < 2; ++bb)
        for (int a = 0; a < 2; ++a)
          acc += tail_node<T, CLS>(td, cls_lds, l, sx, sb, 2 * Ix + a, 2 * Iy + bb, true);
      sbc[I] = acc;
    }
    __syncthreads();
  }
  // coarsest: x = Cinv b with the inverse stored transposed (column c at
  // CinvT + c * n); nb column blocks per row, partial sums reduced in LDS
  {
    const int n = td.nx[L - 1] * td.ny[L - 1];
    const T *sb = sm + td.off[L - 1];
    T *sx = sm + td.off[L - 1] + n;
    const int nb = kTailThreads / n;  // n <= kTailMaxCoarse = kTailThreads
    for (int t = threadIdx.x; t < nb * n; t += kTailThreads) {
      const int r = t % n, cb = t / n;
      T acc = T(0);
      if (td.CinvT)
        for (int c = cb; c < n; c += nb) acc += td.CinvT[(size_t)c * n + r] * sb[c];
      red[t] = acc;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += kTailThreads) {
      T acc = T(0);
      for (int cb = 0; cb < nb; ++cb) acc += red[cb * n + r];
      sx[r] = acc;
    }
    __syncthreads();
  }
  // up
  for (int l = L - 2; l >= 0; --l) {
    T *sb = sm + td.off[l];
    const int nx = td.nx[l], ny = td.ny[l], n = nx * ny;
    T *sx = sb + n;
    const int ncx = td.nx[l + 1], ncy = td.ny[l + 1];
    const T *sxc = sm + td.off[l + 1] + (size_t)ncx * ncy;
    for (int p = threadIdx.x; p < n; p += kTailThreads)
      sx[p] += prolong_value(sxc, ncx, 0, 0, p % nx, p / nx, ncx, ncy, td.pw[l], td.pa, td.pn);
    __syncthreads();
    for (int sw = 0; sw < nu; ++sw) {
      if constexpr (JAC) {
        tail_jsweep<T, CLS>(td, cls_lds, l, sx, sb);
      } else {
        tail_sweep<T, CLS>(td, cls_lds, l, sx, sb, 1);
        tail_sweep<T, CLS>(td, cls_lds, l, sx, sb, 0);
      }
    }
  }
  {
    const int n = td.nx[0] * td.ny[0];
    const T *sx = sm + td.off[0] + n;
    for (int p = threadIdx.x; p < n; p += kTailThreads) x_top[p] = sx[p];
  }
}

// Tile shape: large tiles on big grids, small ones when the large tiles
// would leave most compute units idle.
bool small_tiles(int nx, int ny) {
  return (long long)((nx + 63) / 64) * ((ny + 31) / 32) < 512;
}

}  // namespace

namespace kern {

template <typename T, int NPT, bool CLS, int NU, bool JAC>
void vdown_tj(const OpView<T> &D, const T *b, T *rc, hipStream_t st) {
  if (small_tiles(D.nx, D.ny)) {
    dim3 grid((D.nx + 31) / 32, (D.ny + 15) / 16);
    k_vdown<T, NPT, CLS, NU, 32, 16, JAC><<<grid, kNT, 0, st>>>(D, b, rc);
  } else {
    dim3 grid((D.nx + 63) / 64, (D.ny + 31) / 32);
    k_vdown<T, NPT, CLS, NU, 64, 32, JAC><<<grid, kNT, 0, st>>>(D, b, rc);
  }
}

template <typename T, int NPT, bool CLS, int NU>
void vdown_t(const OpView<T> &D, const T *b, T *rc, hipStream_t st) {
  if (D.jw > T(0))
    vdown_tj<T, NPT, CLS, NU, true>(D, b, rc, st);
  else
    vdown_tj<T, NPT, CLS, NU, false>(D, b, rc, st);
}

template <typename T, int NPT, bool CLS, int NU, bool JAC>
void vup_tj(const OpView<T> &D, const T *b, const T *ec, T *x, hipStream_t st) {
  if (small_tiles(D.nx, D.ny)) {
    dim3 grid((D.nx + 31) / 32, (D.ny + 15) / 16);
    k_vup<T, NPT, CLS, NU, 32, 16, JAC><<<grid, kNT, 0, st>>>(D, b, ec, x);
  } else {
    dim3 grid((D.nx + 63) / 64, (D.ny + 31) / 32);
    k_vup<T, NPT, CLS, NU, 64, 32, JAC><<<grid, kNT, 0, st>>>(D, b, ec, x);
  }
}

template <typename T, int NPT, bool CLS, int NU>
void vup_t(const OpView<T> &D, const T *b, const T *ec, T *x, hipStream_t st) {
  if (D.jw > T(0))
    vup_tj<T, NPT, CLS, NU, true>(D, b, ec, x, st);
  else
    vup_tj<T, NPT, CLS, NU, false>(D, b, ec, x, st);
}

#define IRK_V_DISPATCH(FN, ...)                                                   \
  do {                                                                            \
    const bool cl = D.cls != nullptr;                                             \
    if (D.npt == 5) {                                                             \
      if (cl) {                                                                   \
        if (nu == 1) FN<T, 5, true, 1>(__VA_ARGS__);                              \
        else if (nu == 2) FN<T, 5, true, 2>(__VA_ARGS__);                         \
        else FN<T, 5, true, 3>(__VA_ARGS__);                                      \
      } else {                                                                    \
        if (nu == 1) FN<T, 5, false, 1>(__VA_ARGS__);                             \
        else if (nu == 2) FN<T, 5, false, 2>(__VA_ARGS__);                        \
        else FN<T, 5, false, 3>(__VA_ARGS__);                                     \
      }                                                                           \
    } else {                                                                      \
      if (cl) {                                                                   \
        if (nu == 1) FN<T, 9, true, 1>(__VA_ARGS__);                              \
        else if (nu == 2) FN<T, 9, true, 2>(__VA_ARGS__);                         \
        else FN<T, 9, true, 3>(__VA_ARGS__);                                      \
      } else {                                                                    \
        if (nu == 1) FN<T, 9, false, 1>(__VA_ARGS__);                             \
        else if (nu == 2) FN<T, 9, false, 2>(__VA_ARGS__);                        \
        else FN<T, 9, false, 3>(__VA_ARGS__);                                     \
      }                                                                           \
    }                                                                             \
  } while (0)

template <typename T>
void vdown(const OpView<T> &D, int nu, const T *b, T *rc, hipStream_t st) {
  IRK_V_DISPATCH(vdown_t, D, b, rc, st);
}

template <typename T, int NPT, bool CLS, int NU>
void vdown_couple_t(const OpView<T> &D, const OpView<T> &K, const double *v, const double *scale_j,
                    const T *z, const Row8 &crow, int s, int i, T *b_out, T *rc,
                    hipStream_t st) {
  // the finest level is large: always the large tiles
  dim3 grid((D.nx + 63) / 64, (D.ny + 31) / 32);
  if (K.npt == 5)
    k_vdown_couple<T, NPT, CLS, 5, NU, 64, 32><<<grid, kNT, 0, st>>>(D, K, v, scale_j, z, crow, s,
                                                                     i, b_out, rc);
  else
    k_vdown_couple<T, NPT, CLS, 9, NU, 64, 32><<<grid, kNT, 0, st>>>(D, K, v, scale_j, z, crow, s,
                                                                     i, b_out, rc);
}

template <typename T>
void vdown_couple(const OpView<T> &D, const OpView<T> &K, int nu, const double *v,
                  const double *scale_j, const T *z, const double *C, int s, int i, T *b_out,
                  T *rc, hipStream_t st) {
  Row8 crow{};
  for (int k = 0; k < s; ++k) crow.c[k] = C[k];
  IRK_V_DISPATCH(vdown_couple_t, D, K, v, scale_j, z, crow, s, i, b_out, rc, st);
}

template <typename T>
void vup(const OpView<T> &D, int nu, const T *b, const T *ec, T *x, hipStream_t st) {
  IRK_V_DISPATCH(vup_t, D, b, ec, x, st);
}

template <typename T>
size_t vtail_lds_bytes(const TailDesc<T> &td) {
  size_t n = 0;
  for (int l = 0; l < td.nlev; ++l) n += 2 * (size_t)td.nx[l] * td.ny[l];
  n += kTailThreads + 81 * (size_t)td.nlev;
  return n * sizeof(T);
}

template <typename T, bool JAC>
void vtail_j(const TailDesc<T> &td, int nu, const T *b, T *x, hipStream_t st) {
  if (td.cls[0] || td.nlev == 1)
    k_vtail<T, true, JAC><<<1, kTailThreads, vtail_lds_bytes(td), st>>>(td, b, x, nu);
  else
    k_vtail<T, false, JAC><<<1, kTailThreads, vtail_lds_bytes(td), st>>>(td, b, x, nu);
}

template <typename T>
void vtail(const TailDesc<T> &td, int nu, const T *b, T *x, hipStream_t st) {
  if (td.jw > T(0))
    vtail_j<T, true>(td, nu, b, x, st);
  else
    vtail_j<T, false>(td, nu, b, x, st);
}

template void vdown<float>(const OpView<float> &, int, const float *, float *, hipStream_t);
template void vdown<double>(const OpView<double> &, int, const double *, double *, hipStream_t);
template void vdown_couple<float>(const OpView<float> &, const OpView<float> &, int,
                                  const double *, const double *, const float *, const double *,
                                  int, int, float *, float *, hipStream_t);
template void vdown_couple<double>(const OpView<double> &, const OpView<double> &, int,
                                   const double *, const double *, const double *,
                                   const double *, int, int, double *, double *, hipStream_t);
template void vup<float>(const OpView<float> &, int, const float *, const float *, float *,
                         hipStream_t);
template void vup<double>(const OpView<double> &, int, const double *, const double *, double *,
                          hipStream_t);
template size_t vtail_lds_bytes<float>(const TailDesc<float> &);
template size_t vtail_lds_bytes<double>(const TailDesc<double> &);
template void vtail<float>(const TailDesc<float> &, int, const float *, float *, hipStream_t);
template void vtail<double>(const TailDesc<double> &, int, const double *, double *, hipStream_t);

}  // namespace kern
}  // namespace irk
