// Register-tiled V-cycle passes (gfx950, wave64).
//
// Same operations as the LDS-tiled passes (one fused pass down, one up per
// level; see vcycle.hip) but organised for the CDNA issue model: every
// wavefront owns an independent tile of 64 grid columns (one per lane) and R
// grid rows held in registers.  North/south neighbours are registers of the
// same lane, east/west neighbours come from the adjacent lanes through DPP
// wave shifts, so a red-black half sweep over a row costs a handful of VALU
// instructions, with no LDS traffic and no barriers.  Tiles overlap by a halo
// that shrinks by one node per dependent sweep (temporal blocking); only the
// tile interior is written.
//
//   lanes 0..63  <->  grid columns X0 .. X0+63,  X0 = OX - HX
//   rows  0..R-1 <->  grid rows    Y0 .. Y0+R-1, Y0 = OY - HY
//   output: lanes [HX, 64-HX) x rows [HY, R-HY)
//
// Coefficients: an operator whose boundary rows equal the interior stencil
// with the couplings to outside nodes dropped (five-point constant
// coefficients, e.g. the heat operator and its stage blocks) is applied with
// the interior stencil from registers everywhere, since x is zero outside the
// grid; per-node operators are loaded per row through the cache.  Other
// operators use the LDS-tiled passes.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace irk {
namespace {

struct Row8w {
  double c[8];
};

constexpr int kWaves = 4;  // independent wave tiles per workgroup

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// DPP wave shifts: value of lane+1 (wave_shl1) and of lane-1 (wave_shr1); the
// lanes shifted in from outside the wave read 0.
__device__ __forceinline__ float from_next(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ float from_prev(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ double from_next(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), 0x130, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double from_prev(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), 0x138, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ int wcls(int i, int j, int nx, int ny) {
  const int cx = (i == 0) ? 0 : (i == nx - 1 ? 2 : 1);
  const int cy = (j == 0) ? 0 : (j == ny - 1 ? 2 : 1);
  return 3 * cy + cx;
}

__device__ __forceinline__ constexpr bool wused(int npt, int k) {
  return npt == 9 || k == 1 || k == 3 || k == 4 || k == 5 || k == 7;
}

// Coefficient source of one operator for one wave tile.
//  MODE 0: uniform interior class (registers)
//  MODE 1: boundary classes looked up per node
//  MODE 2: per-node arrays
template <typename T>
struct WOp {
  int nx, ny;
  const T *cls;
  const T *arr;
  T u[9];    // interior class (MODE 0)
  T inv_d;   // 1 / u[4]
  T pw;      // prolongation weight of the outermost fine node
  T pa, pn;  // prolongation weights from the own and the next coarse node
};

template <typename T, int NPT, int MODE>
__device__ __forceinline__ void wcoefs(const WOp<T> &o, int gx, int gy, bool inside, T *a) {
  if (MODE == 0) {
#pragma unroll
    for (int k = 0; k < 9; ++k)
      if (wused(NPT, k)) a[k] = o.u[k];
  } else if (MODE == 1) {
    const int q = inside ? wcls(gx, gy, o.nx, o.ny) : 4;
#pragma unroll
    for (int k = 0; k < 9; ++k)
      if (wused(NPT, k)) a[k] = o.cls[q * 9 + k];
  } else {
    const size_t N = (size_t)o.nx * o.ny;
    const size_t p = inside ? (size_t)gy * o.nx + gx : 0;
#pragma unroll
    for (int k = 0; k < 9; ++k)
      if (wused(NPT, k)) a[k] = inside ? o.arr[(size_t)k * N + p] : (k == 4 ? T(1) : T(0));
  }
}

// b - sum_{k != centre} a_k x_k for the node of this lane in row r.
// xs / xn: old values of rows r-1 / r+1 in this lane's column.
template <typename T, int NPT>
__device__ __forceinline__ T wrhs(const T *a, T b, T xc, T xs, T xn) {
  T acc = b - a[7] * xn - a[1] * xs - a[5] * from_next(xc) - a[3] * from_prev(xc);
  if (NPT == 9)
    acc -= a[8] * from_next(xn) + a[6] * from_prev(xn) + a[2] * from_next(xs) + a[0] * from_prev(xs);
  return acc;
}

// One colour half sweep on rows [M, R-M) (lanes: all; the halo lanes hold
// values that are never written out).
template <typename T, int NPT, int MODE, int R, int M>
__device__ __forceinline__ void wsweep(const WOp<T> &o, T (&x)[R], const T (&b)[R], int X0, int Y0,
                                       int color) {
  const int gx = X0 + lane_id();
  const bool in_x = gx >= 0 && gx < o.nx;
  T prev_old = T(0);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r < M || r >= R - M) {
      prev_old = x[r];
      continue;
    }
    const int gy = Y0 + r;
    const bool inside = in_x && gy >= 0 && gy < o.ny;
    const bool upd = (((gx + gy) & 1) == color) && inside;
    T a[9];
    wcoefs<T, NPT, MODE>(o, gx, gy, inside, a);
    // old value of row r-1 (saved before its update): keeps the rows of one
    // half sweep independent, so their instructions interleave
    const T xs = prev_old;
    const T xn = (r + 1 < R) ? x[r + 1] : T(0);
    const T t = wrhs<T, NPT>(a, b[r], x[r], xs, xn);
    const T xnew = (MODE == 0) ? t * o.inv_d : t / a[4];
    prev_old = x[r];
    x[r] = upd ? xnew : x[r];
  }
}

// x = 0 and the first half sweep (colour 0 gets b / d), then 2 nu - 1 sweeps.
template <typename T, int NPT, int MODE, int R, int NU>
__device__ __forceinline__ void wpresmooth(const WOp<T> &o, T (&x)[R], const T (&b)[R], int X0,
                                           int Y0) {
  const int gx = X0 + lane_id();
  const bool in_x = gx >= 0 && gx < o.nx;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int gy = Y0 + r;
    const bool inside = in_x && gy >= 0 && gy < o.ny;
    T a[9];
    wcoefs<T, NPT, MODE>(o, gx, gy, inside, a);
    const T xv = (MODE == 0) ? b[r] * o.inv_d : b[r] / a[4];
    x[r] = ((((gx + gy) & 1) == 0) && inside) ? xv : T(0);
  }
  wsweep<T, NPT, MODE, R, 1>(o, x, b, X0, Y0, 1);
  if (NU >= 2) {
    wsweep<T, NPT, MODE, R, 2>(o, x, b, X0, Y0, 0);
    wsweep<T, NPT, MODE, R, 3>(o, x, b, X0, Y0, 1);
  }
  if (NU >= 3) {
    wsweep<T, NPT, MODE, R, 4>(o, x, b, X0, Y0, 0);
    wsweep<T, NPT, MODE, R, 5>(o, x, b, X0, Y0, 1);
  }
}

template <typename T, int NPT, int MODE, int R, int NU>
__device__ __forceinline__ void wpostsmooth(const WOp<T> &o, T (&x)[R], const T (&b)[R], int X0,
                                            int Y0) {
  constexpr int M0 = 2 * NU;
  wsweep<T, NPT, MODE, R, M0>(o, x, b, X0, Y0, 1);
  wsweep<T, NPT, MODE, R, M0 + 1>(o, x, b, X0, Y0, 0);
  if (NU >= 2) {
    wsweep<T, NPT, MODE, R, M0 + 2>(o, x, b, X0, Y0, 1);
    wsweep<T, NPT, MODE, R, M0 + 3>(o, x, b, X0, Y0, 0);
  }
  if (NU >= 3) {
    wsweep<T, NPT, MODE, R, M0 + 4>(o, x, b, X0, Y0, 1);
    wsweep<T, NPT, MODE, R, M0 + 5>(o, x, b, X0, Y0, 0);
  }
}

// rc = R (b - D x) on the coarse nodes of the output region.
template <typename T, int NPT, int MODE, int R, int HX, int HY>
__device__ __forceinline__ void wrestrict(const WOp<T> &o, const T (&x)[R], const T (&b)[R], int X0,
                                          int Y0, T *__restrict__ rc) {
  const int lane = lane_id();
  const int gx = X0 + lane;
  const bool in_x = gx >= 0 && gx < o.nx;
  const int ncx = o.nx / 2, ncy = o.ny / 2;
#pragma unroll
  for (int r = HY; r + 1 < R - HY + 1; r += 2) {
    T s = T(0);
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int rr = r + d, gy = Y0 + rr;
      const bool inside = in_x && gy >= 0 && gy < o.ny;
      T a[9];
      wcoefs<T, NPT, MODE>(o, gx, gy, inside, a);
      const T xs = rr > 0 ? x[rr - 1] : T(0);
      const T xn = rr + 1 < R ? x[rr + 1] : T(0);
      const T res = wrhs<T, NPT>(a, b[rr], x[rr], xs, xn) - a[4] * x[rr];
      s += inside ? res : T(0);
    }
    const T t = s + from_next(s);  // this lane (even column) + the next one
    const int gy = Y0 + r;
    const int I = gx >> 1, J = gy >> 1;
    if (((lane - HX) & 1) == 0 && lane >= HX && lane < 64 - HX && I < ncx && J < ncy && gx >= 0)
      rc[(size_t)J * ncx + I] = t;
  }
}

template <typename T, int R>
__device__ __forceinline__ void wload(const T *__restrict__ g, T (&v)[R], int X0, int Y0, int nx,
                                      int ny) {
  const int gx = X0 + lane_id();
  const bool in_x = gx >= 0 && gx < nx;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int gy = Y0 + r;
    v[r] = (in_x && gy >= 0 && gy < ny) ? g[(size_t)gy * nx + gx] : T(0);
  }
}

template <typename T>
__device__ __forceinline__ WOp<T> make_wop(const OpView<T> &D) {
  WOp<T> o;
  o.nx = D.nx;
  o.ny = D.ny;
  o.cls = D.cls;
  o.arr = D.arr;
#pragma unroll
  for (int k = 0; k < 9; ++k) o.u[k] = D.cls ? D.cls[36 + k] : T(0);
  o.inv_d = D.cls ? T(1) / o.u[4] : T(0);
  o.pw = D.pw;
  o.pa = D.pa;
  o.pn = D.pn;
  return o;
}

// Geometry per (type, nu): halo and rows (registers hold 2 rows per value
// array, so doubles get fewer rows).
template <typename T, int NU>
struct WGeom {
  static constexpr int HD = 2 * NU;      // down halo
  static constexpr int HU = 4 * NU - 1;  // up halo
  static constexpr int TYD = sizeof(T) == 4 ? 32 : 16;
  static constexpr int TYU = sizeof(T) == 4 ? (NU == 3 ? 16 : 32) : (NU == 3 ? 8 : 16);
};

template <typename T, int NPT, int NU, bool COUPLE, int NPTK, int MODE>
__global__ void __launch_bounds__(64 * kWaves)
    k_wdown(OpView<T> D, OpView<T> K, const double *__restrict__ v, const double *__restrict__ scale_j,
            const T *__restrict__ z, Row8w crow, int s, int i, const T *__restrict__ bin,
            T *__restrict__ b_out, T *__restrict__ rc) {
  constexpr int HY = WGeom<T, NU>::HD;
  constexpr int HX = COUPLE ? HY + 1 : HY;
  constexpr int TY = WGeom<T, NU>::TYD;
  constexpr int R = TY + 2 * HY;
  constexpr int TXO = 64 - 2 * HX;
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const Tile2 tile = xcd_tile();
  const int OX = tile.x * TXO, OY = (tile.y * kWaves + wave) * TY;
  if (OY >= D.ny) return;  // whole wave leaves together
  const int X0 = OX - HX, Y0 = OY - HY;
  T b[R], x[R];
  if (COUPLE) {
    // b = scale_j v_i - K (sum_k C_k z_k) on the region (the lanes at the
    // region's edge lack a neighbour column and stay halo)
    const size_t N = (size_t)D.nx * D.ny;
    const double sc = *scale_j;
    const int gx = X0 + lane;
    const bool in_x = gx >= 0 && gx < D.nx;
    bool any = false;
#pragma unroll
    for (int k = 0; k < kMaxStages; ++k)
      if (k < s && crow.c[k] != 0.0) any = true;
    T c[R + 2];
#pragma unroll
    for (int r = 0; r < R + 2; ++r) {
      const int gy = Y0 - 1 + r;
      T acc = T(0);
      if (any && in_x && gy >= 0 && gy < D.ny) {
        const size_t p = (size_t)gy * D.nx + gx;
#pragma unroll
        for (int k = 0; k < kMaxStages; ++k)
          if (k < s && crow.c[k] != 0.0) acc += T(crow.c[k]) * z[(size_t)k * N + p];
      }
      c[r] = acc;
    }
    WOp<T> ko = make_wop(K);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int gy = Y0 + r;
      const bool inside = in_x && gy >= 0 && gy < D.ny;
      T vv = inside ? T(sc * v[(size_t)i * N + (size_t)gy * D.nx + gx]) : T(0);
      if (any) {
        T a[9];
        wcoefs<T, NPTK, MODE>(ko, gx, gy, inside, a);
        // K c = a_c c + (sum of neighbours): reuse wrhs with b = 0
        const T kc = a[4] * c[r + 1] - wrhs<T, NPTK>(a, T(0), c[r + 1], c[r], c[r + 2]);
        vv -= inside ? kc : T(0);
      }
      b[r] = vv;
    }
    // the right-hand side of the output region, for the up pass
#pragma unroll
    for (int r = HY; r < R - HY; ++r) {
      const int gy = Y0 + r;
      if (lane >= HX && lane < 64 - HX && gx < D.nx && gy < D.ny)
        b_out[(size_t)gy * D.nx + gx] = b[r];
    }
  } else {
    wload<T, R>(bin, b, X0, Y0, D.nx, D.ny);
  }
  WOp<T> o = make_wop(D);
  wpresmooth<T, NPT, MODE, R, NU>(o, x, b, X0, Y0);
  wrestrict<T, NPT, MODE, R, HX, HY>(o, x, b, X0, Y0, rc);
}

// LIN: linear interpolation (weights 3/4 and 1/4 built in, pw at the
// boundary); otherwise the weights pa, pn, pw of the operator.
template <typename T, int NPT, int MODE, int R, int NU, int H, bool LIN>
__device__ __forceinline__ void wup_body(const WOp<T> &o, T (&x)[R], const T (&b)[R], int X0,
                                         int Y0, const T *se, int CW, int CX0, int CY0) {
  wpresmooth<T, NPT, MODE, R, NU>(o, x, b, X0, Y0);
  // x += P ec where the pre-smoothed x is exact (rows/lanes at margin 2nu-1)
  constexpr int M = 2 * NU - 1;
  const int lane = lane_id();
  const int gx = X0 + lane;
  const int ncx = o.nx / 2, ncy = o.ny / 2;
  const int Ix = gx >> 1;
  const int nbx = (gx & 1) ? Ix + 1 : Ix - 1;
  const bool ix = nbx >= 0 && nbx < ncx;
  const T pa = LIN ? T(0.75) : o.pa, pn = LIN ? T(0.25) : o.pn;
  const bool hx = ix && (LIN || pn != T(0));
  const bool in_x = gx >= 0 && gx < o.nx && lane >= M && lane < 64 - M;
#pragma unroll
  for (int r = M; r < R - M; ++r) {
    const int gy = Y0 + r;
    const int Iy = gy >> 1;
    const int nby = (gy & 1) ? Iy + 1 : Iy - 1;
    const bool iy = nby >= 0 && nby < ncy;
    const bool hy = iy && (LIN || pn != T(0));
    if (in_x && gy >= 0 && gy < o.ny) {
      const T *row = se + (Iy - CY0) * CW;
      const T *nrow = se + (nby - CY0) * CW;
      const T wx = ix ? pa : o.pw, wy = iy ? pa : o.pw;
      T pv = wx * wy * row[Ix - CX0];
      if (hx) pv += pn * wy * row[nbx - CX0];
      if (hy) pv += wx * pn * nrow[Ix - CX0];
      if (hx && hy) pv += (LIN ? T(0.0625) : pn * pn) * nrow[nbx - CX0];
      x[r] += pv;
    }
  }
  wpostsmooth<T, NPT, MODE, R, NU>(o, x, b, X0, Y0);
}

template <typename T, int NPT, int NU, int MODE, bool LIN>
__global__ void __launch_bounds__(64 * kWaves)
    k_wup(OpView<T> D, const T *__restrict__ bin, const T *__restrict__ ec, T *__restrict__ xout) {
  constexpr int H = WGeom<T, NU>::HU;
  constexpr int TY = WGeom<T, NU>::TYU;
  constexpr int R = TY + 2 * H;
  constexpr int TXO = 64 - 2 * H;
  constexpr int M = 2 * NU - 1;
  constexpr int CW = (64 - 2 * M) / 2 + 4, CH = (R - 2 * M) / 2 + 4;
  __shared__ T se_all[kWaves][CW * CH];
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const Tile2 tile = xcd_tile();
  const int OX = tile.x * TXO, OY = (tile.y * kWaves + wave) * TY;
  const int X0 = OX - H, Y0 = OY - H;
  const int ncx = D.nx / 2, ncy = D.ny / 2;
  const int CX0 = ((X0 + M) >> 1) - 1, CY0 = ((Y0 + M) >> 1) - 1;
  T *se = se_all[wave];
  // stage the coarse correction this wave interpolates from
  for (int q = lane; q < CW * CH; q += 64) {
    const int I = CX0 + q % CW, J = CY0 + q / CW;
    se[q] = (I >= 0 && J >= 0 && I < ncx && J < ncy) ? ec[(size_t)J * ncx + I] : T(0);
  }
  T b[R], x[R];
  wload<T, R>(bin, b, X0, Y0, D.nx, D.ny);
  __syncthreads();
  if (OY >= D.ny) return;
  WOp<T> o = make_wop(D);
  wup_body<T, NPT, MODE, R, NU, H, LIN>(o, x, b, X0, Y0, se, CW, CX0, CY0);
  const int gx = X0 + lane;
  if (lane >= H && lane < 64 - H && gx < D.nx) {
#pragma unroll
    for (int r = H; r < R - H; ++r) {
      const int gy = Y0 + r;
      if (gy < D.ny) xout[(size_t)gy * D.nx + gx] = x[r];
    }
  }
}

template <typename T, int NPT, int NU, bool COUPLE, int NPTK, int MODE>
void launch_wdown(const OpView<T> &D, const OpView<T> &K, const double *v, const double *scale_j,
                  const T *z, const Row8w &crow, int s, int i, const T *bin, T *b_out, T *rc,
                  hipStream_t st) {
  constexpr int HY = WGeom<T, NU>::HD;
  constexpr int HX = COUPLE ? HY + 1 : HY;
  constexpr int TY = WGeom<T, NU>::TYD;
  constexpr int TXO = 64 - 2 * HX;
  dim3 grid((D.nx + TXO - 1) / TXO, (D.ny + TY * kWaves - 1) / (TY * kWaves));
  k_wdown<T, NPT, NU, COUPLE, NPTK, MODE><<<grid, 64 * kWaves, 0, st>>>(D, K, v, scale_j, z, crow,
                                                                        s, i, bin, b_out, rc);
}

template <typename T, int NPT, int NU, int MODE>
void launch_wup(const OpView<T> &D, const T *b, const T *ec, T *x, hipStream_t st) {
  constexpr int H = WGeom<T, NU>::HU;
  constexpr int TY = WGeom<T, NU>::TYU;
  constexpr int TXO = 64 - 2 * H;
  dim3 grid((D.nx + TXO - 1) / TXO, (D.ny + TY * kWaves - 1) / (TY * kWaves));
  if (D.pa == T(0.75) && D.pn == T(0.25))
    k_wup<T, NPT, NU, MODE, true><<<grid, 64 * kWaves, 0, st>>>(D, b, ec, x);
  else
    k_wup<T, NPT, NU, MODE, false><<<grid, 64 * kWaves, 0, st>>>(D, b, ec, x);
}

}  // namespace

namespace kern {

// Only five-point operators, uniform (constant coefficients) or per node.
template <typename T>
bool wtile_ok(const OpView<T> &D) {
  return D.npt == 5 && (D.uniform || D.arr);
}
template bool wtile_ok<float>(const OpView<float> &);
template bool wtile_ok<double>(const OpView<double> &);

#define IRK_W_NU(FN, MODE_, ...)                         \
  do {                                                   \
    if (nu == 1) FN<T, 5, 1, MODE_>(__VA_ARGS__);        \
    else if (nu == 2) FN<T, 5, 2, MODE_>(__VA_ARGS__);   \
    else FN<T, 5, 3, MODE_>(__VA_ARGS__);                \
  } while (0)

template <typename T, int NPT, int NU, int MODE>
void wdown_plain(const OpView<T> &D, const T *b, T *rc, hipStream_t st) {
  const Row8w none{};
  const OpView<T> K0{};
  launch_wdown<T, NPT, NU, false, 5, MODE>(D, K0, nullptr, nullptr, nullptr, none, 0, 0, b, nullptr,
                                          rc, st);
}

template <typename T, int NPT, int NU, int MODE>
void wdown_cpl(const OpView<T> &D, const OpView<T> &K, const double *v, const double *scale_j,
               const T *z, const Row8w &crow, int s, int i, T *b_out, T *rc, hipStream_t st) {
  launch_wdown<T, NPT, NU, true, 5, MODE>(D, K, v, scale_j, z, crow, s, i, nullptr, b_out, rc, st);
}

template <typename T>
void wdown(const OpView<T> &D, int nu, const T *b, T *rc, hipStream_t st) {
  if (D.arr)
    IRK_W_NU(wdown_plain, 2, D, b, rc, st);
  else
    IRK_W_NU(wdown_plain, 0, D, b, rc, st);
}

template <typename T>
void wdown_couple(const OpView<T> &D, const OpView<T> &K, int nu, const double *v,
                  const double *scale_j, const T *z, const double *C, int s, int i, T *b_out,
                  T *rc, hipStream_t st) {
  Row8w crow{};
  for (int k = 0; k < s; ++k) crow.c[k] = C[k];
  if (D.arr)
    IRK_W_NU(wdown_cpl, 2, D, K, v, scale_j, z, crow, s, i, b_out, rc, st);
  else
    IRK_W_NU(wdown_cpl, 0, D, K, v, scale_j, z, crow, s, i, b_out, rc, st);
}

template <typename T>
void wup(const OpView<T> &D, int nu, const T *b, const T *ec, T *x, hipStream_t st) {
  if (D.arr)
    IRK_W_NU(launch_wup, 2, D, b, ec, x, st);
  else
    IRK_W_NU(launch_wup, 0, D, b, ec, x, st);
}

template void wdown<float>(const OpView<float> &, int, const float *, float *, hipStream_t);
template void wdown<double>(const OpView<double> &, int, const double *, double *, hipStream_t);
template void wdown_couple<float>(const OpView<float> &, const OpView<float> &, int,
                                  const double *, const double *, const float *, const double *,
                                  int, int, float *, float *, hipStream_t);
template void wdown_couple<double>(const OpView<double> &, const OpView<double> &, int,
                                   const double *, const double *, const double *,
                                   const double *, int, int, double *, double *, hipStream_t);
template void wup<float>(const OpView<float> &, int, const float *, const float *, float *,
                         hipStream_t);
template void wup<double>(const OpView<double> &, int, const double *, const double *, double *,
                          hipStream_t);

}  // namespace kern
}  // namespace irk
