// Finest-level V-cycle passes with the pre-smoothed x kept in memory.
//
// Layout as in the split-column kernels: lane l of a wave holds grid columns
// X0 + 2l (slot a) and X0 + 2l + 1 (slot b) of R consecutive grid rows in
// registers, X0 and Y0 even, so slot a of tile row r has red-black colour
// r mod 2 and every lane updates exactly one of its two nodes per row in a
// half sweep.  West/east neighbours across the slot pair come from the
// adjacent lane through DPP wave shifts.
//
// Down pass: x = 0, 2 nu half sweeps (colours 0, 1, ...), residual and its
// 2 x 2 sum onto the coarse grid, and the pre-smoothed x of the output
// region stored for the up pass.  Up pass: x = stored pre-smoothed x plus
// the prolongated coarse correction, then 2 nu half sweeps in the reverse
// colour order.  Both run as row pipelines: stage k (the k-th operation on a
// row) reaches row r at step r + 2k, which reads exactly the values the
// stage-by-stage order reads (a half sweep reads the other colour, which
// only the previous stage wrote; see the down pass of the split kernels), so
// a wave computes on its first rows while the later ones are still loading.
// Storing the pre-smoothed x costs one vector write and one read per level
// and spares the up pass the repeated pre-smoothing and its wider halo.
//
// Operators (five-point, M = I on the finest level):
//  VAR = false: a uniform constant-coefficient stencil (interior
//               coefficients as kernel arguments; boundary rows are the
//               interior stencil without the couplings that leave the grid);
//  VAR = true:  D = I + tau K with K per node, packed as (S, W, E, N) and the
//               centre, in the pass's precision; the block's coefficients are
//               formed in registers, so one packed K serves every stage.
// Nodes outside the grid are held at zero: their rows are skipped (a
// wave-uniform branch) and their lanes relax with 1/d = 0.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace irk {
namespace {

constexpr int kFW = 4;  // waves per workgroup, stacked in y

__device__ __forceinline__ int f_lane() { return threadIdx.x & 63; }

// Value of lane + 1 / lane - 1 (zero shifted in at the wave's ends).
__device__ __forceinline__ float f_next(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ float f_prev(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ double f_next(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), 0x130, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double f_prev(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), 0x138, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ float f_rcp(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double f_rcp(double v) { return 1.0 / v; }

template <typename T>
struct V2T;
template <>
struct V2T<float> {
  using V = float2;
};
template <>
struct V2T<double> {
  using V = double2;
};
template <typename T>
struct V4T;
template <>
struct V4T<float> {
  using V = float4;
};
template <>
struct V4T<double> {
  using V = double4;
};

// The finest level's operator as the kernels see it.
template <typename T>
struct FOp {
  int nx, ny;
  T s, w, c, e, n, inv;            // constant mode: interior stencil and 1 / centre
  const typename V4T<T>::V *kq;    // variable mode: K's (S, W, E, N) per node
  const T *kc;                     // variable mode: K's centre per node
  T tau;                           // variable mode: D = I + tau K
  T pw;                            // prolongation weight of the outermost fine node
};

// Coefficients of one node of D.
template <typename T>
struct FCo {
  T s, w, e, n, c, inv;
};

// Both slots' coefficients in tile row r (grid row gy); zero outside the grid.
template <typename T, bool VAR>
__device__ __forceinline__ void f_coefs(const FOp<T> &o, int gy, int gxa, bool inx, FCo<T> &ca,
                                        FCo<T> &cb) {
  if (!VAR) {
    const T inv = inx ? o.inv : T(0);
    ca = FCo<T>{o.s, o.w, o.e, o.n, o.c, inv};
    cb = ca;
    return;
  }
  if (!inx || gy < 0 || gy >= o.ny) {
    ca = FCo<T>{T(0), T(0), T(0), T(0), T(0), T(0)};
    cb = ca;
    return;
  }
  const size_t p = (size_t)gy * o.nx + gxa;  // even
  const typename V4T<T>::V qa = o.kq[p], qb = o.kq[p + 1];
  const typename V2T<T>::V cc = *reinterpret_cast<const typename V2T<T>::V *>(o.kc + p);
  const T t = o.tau;
  ca.s = t * qa.x;
  ca.w = t * qa.y;
  ca.e = t * qa.z;
  ca.n = t * qa.w;
  ca.c = T(1) + t * cc.x;
  ca.inv = f_rcp(ca.c);
  cb.s = t * qb.x;
  cb.w = t * qb.y;
  cb.e = t * qb.z;
  cb.n = t * qb.w;
  cb.c = T(1) + t * cc.y;
  cb.inv = f_rcp(cb.c);
}

// Tile rows of one wave: x, b and the coefficients of both slots.
template <typename T, int R>
struct FTile {
  T xa[R], xb[R], ba[R], bb[R];
  FCo<T> ca[R], cb[R];
};

// Relaxation of row r in colour `color` (slot a has colour r mod 2).
template <typename T, int R>
__device__ __forceinline__ void f_relax(FTile<T, R> &t, int r, int color) {
  if ((r & 1) == color) {
    const FCo<T> &c = t.ca[r];
    t.xa[r] = (t.ba[r] - c.s * t.xa[r - 1] - c.n * t.xa[r + 1] - c.w * f_prev(t.xb[r]) -
               c.e * t.xb[r]) * c.inv;
  } else {
    const FCo<T> &c = t.cb[r];
    t.xb[r] = (t.bb[r] - c.s * t.xb[r - 1] - c.n * t.xb[r + 1] - c.w * t.xa[r] -
               c.e * f_next(t.xa[r])) * c.inv;
  }
}

// Residual b - D x of row r, summed over the lane's two slots.
template <typename T, int R>
__device__ __forceinline__ T f_resid_pair(const FTile<T, R> &t, int r) {
  const FCo<T> &a = t.ca[r], &b = t.cb[r];
  const T ra = t.ba[r] - a.c * t.xa[r] - a.s * t.xa[r - 1] - a.n * t.xa[r + 1] -
               a.w * f_prev(t.xb[r]) - a.e * t.xb[r];
  const T rb = t.bb[r] - b.c * t.xb[r] - b.s * t.xb[r - 1] - b.n * t.xb[r + 1] - b.w * t.xa[r] -
               b.e * f_next(t.xa[r]);
  return ra + rb;
}

// Rows Y0..Y0+R-1 of a grid vector at columns X0+2l, X0+2l+1 (zero outside).
template <typename T, int R>
__device__ __forceinline__ void f_load(const T *__restrict__ g, T (&a)[R], T (&b)[R], int X0,
                                       int Y0, int nx, int ny) {
  const int gx = X0 + 2 * f_lane();
  const bool inx = gx >= 0 && gx < nx;  // nx and gx even: gx + 1 < nx too
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int gy = Y0 + r;
    typename V2T<T>::V v{};
    if (inx && gy >= 0 && gy < ny)
      v = *reinterpret_cast<const typename V2T<T>::V *>(g + (size_t)gy * nx + gx);
    a[r] = v.x;
    b[r] = v.y;
  }
}

template <typename T>
__device__ __forceinline__ void f_store2(T *p, T a, T b) {
  typename V2T<T>::V v;
  v.x = a;
  v.y = b;
  *reinterpret_cast<typename V2T<T>::V *>(p) = v;
}

__host__ __device__ constexpr int f_even(int h) { return (h + 1) & ~1; }

// Tile geometry.  Down: TY output rows, row and column halo H = 2 nu (the
// residual needs x exact one node beyond the output).  Up: row halo 2 nu
// (the post-smoothing), column halo 2 nu + 2 (the outermost lanes lack the
// coarse column beyond the tile, so their correction is wrong).
// Tile heights keep the registers of x, b (and, VAR, the coefficients of
// the rows in flight) within about 200 per lane.  With K per node the FP32
// tiles are 4 rows high: the grids these passes serve (1024^2) then give
// every CU workgroups and each wave a short row chain (double glazing
// 1024^2: 5.25 ms per step with 16-row tiles, 4.83 with 8, 4.72 with 4).
// SMALL: 4-row tiles, taken when the usual ones would leave CUs without a
// workgroup (fewer than 256).
template <typename T, int NU, bool VAR, bool SMALL = false>
struct FGeomD {
  static constexpr int K = 2 * NU;
  static constexpr int H = f_even(2 * NU);
  static constexpr int TY = SMALL ? 4 : (sizeof(T) == 4 ? (VAR ? 4 : 16) : 8);
  static constexpr int R = TY + 2 * H;
  static constexpr int TXO = 128 - 2 * H;
};
template <typename T, int NU, bool VAR, bool SMALL = false>
struct FGeomU {
  static constexpr int K = 2 * NU;
  static constexpr int H = f_even(2 * NU);
  static constexpr int HC = H + 2;
  static constexpr int TY = SMALL ? 4 : (sizeof(T) == 4 ? (VAR ? 4 : 24) : 8);
  static constexpr int R = TY + 2 * H;
  static constexpr int TXO = 128 - 2 * HC;
};

// Down pass of one tile.  BOUND: the tile reaches past the grid.
template <typename T, bool VAR, bool BOUND, int NU, bool SMALL>
__device__ __forceinline__ void f_down_tile(const FOp<T> &o,
                                            FTile<T, FGeomD<T, NU, VAR, SMALL>::R> &t, int X0,
                                            int Y0, T *__restrict__ rc, T *__restrict__ xpre) {
  using G = FGeomD<T, NU, VAR, SMALL>;
  constexpr int K = G::K, H = G::H, R = G::R;
  const int lane = f_lane();
  const int gxa = X0 + 2 * lane;
  const bool inx = gxa >= 0 && gxa < o.nx;  // nx even: slot b is inside iff slot a is
  const int ncx = o.nx / 2, ncy = o.ny / 2;
  const int I = gxa >> 1;
  const bool lane_out = lane >= H / 2 && lane < 64 - H / 2 && gxa < o.nx;
  auto row_in = [&](int r) { return !BOUND || (unsigned)(Y0 + r) < (unsigned)o.ny; };
#pragma unroll
  for (int step = 0; step < R + 2 * K + 2; ++step) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int r = step - 2 * k;
      if (k == 0 && r < R) {
        // coefficients of row r, then x = b / d on colour 0 and 0 on colour 1
        f_coefs<T, VAR>(o, Y0 + r, gxa, BOUND ? inx : true, t.ca[r], t.cb[r]);
        if ((r & 1) == 0) {
          t.xa[r] = t.ba[r] * t.ca[r].inv;
          t.xb[r] = T(0);
        } else {
          t.xb[r] = t.bb[r] * t.cb[r].inv;
          t.xa[r] = T(0);
        }
      } else if (k > 0 && r >= k && r < R - k) {
        if (row_in(r)) f_relax<T, R>(t, r, k & 1);
      }
    }
    // row rx is final once the last stage has passed it
    const int rx = step - 2 * (K - 1);
    if (rx >= H && rx < R - H) {
      const int gy = Y0 + rx;
      if (lane_out && gy < o.ny) f_store2(xpre + (size_t)gy * o.nx + gxa, t.xa[rx], t.xb[rx]);
    }
    // the pair r0, r0 + 1 once row r0 + 2 is final
    const int r0 = step - 2 - 2 * (K - 1);
    if (r0 >= H && r0 < R - H && ((r0 - H) & 1) == 0) {
      T sum = T(0);
      if (row_in(r0)) sum += f_resid_pair<T, R>(t, r0);
      if (row_in(r0 + 1)) sum += f_resid_pair<T, R>(t, r0 + 1);
      if (BOUND && !inx) sum = T(0);
      const int J = (Y0 + r0) >> 1;
      if (lane_out && I < ncx && J < ncy) rc[(size_t)J * ncx + I] = sum;
    }
  }
}

// The right-hand side of a block without coupling terms, formed on load:
// rows of *vscale times the FP64 vector v, multiplied in FP64 and rounded to
// T (the same bits the coupling pass would write).
template <typename T, int R>
__device__ __forceinline__ void f_load_v(const double *__restrict__ v,
                                         const double *__restrict__ vscale, T (&a)[R], T (&b)[R],
                                         int X0, int Y0, int nx, int ny) {
  const double sc = *vscale;
  const int gx = X0 + 2 * f_lane();
  const bool inx = gx >= 0 && gx < nx;  // nx and gx even: gx + 1 < nx too
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int gy = Y0 + r;
    double2 w = make_double2(0.0, 0.0);
    if (inx && gy >= 0 && gy < ny) w = *reinterpret_cast<const double2 *>(v + (size_t)gy * nx + gx);
    a[r] = (T)(sc * w.x);
    b[r] = (T)(sc * w.y);
  }
}

template <typename T, bool VAR, int NU, bool SMALL>
__global__ void __launch_bounds__(64 * kFW)
    k_fdown(FOp<T> o, const T *__restrict__ bin, const double *__restrict__ vin,
            const double *__restrict__ vscale, T *__restrict__ rc, T *__restrict__ xpre) {
  using G = FGeomD<T, NU, VAR, SMALL>;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const Tile2 tile = xcd_tile();
  const int OX = tile.x * G::TXO, OY = (tile.y * kFW + wave) * G::TY;
  if (OY >= o.ny) return;
  const int X0 = OX - G::H, Y0 = OY - G::H;
  FTile<T, G::R> t;
  if (vin)
    f_load_v<T, G::R>(vin, vscale, t.ba, t.bb, X0, Y0, o.nx, o.ny);
  else
    f_load<T, G::R>(bin, t.ba, t.bb, X0, Y0, o.nx, o.ny);
  if (X0 >= 0 && Y0 >= 0 && X0 + 128 <= o.nx && Y0 + G::R <= o.ny)
    f_down_tile<T, VAR, false, NU, SMALL>(o, t, X0, Y0, rc, xpre);
  else
    f_down_tile<T, VAR, true, NU, SMALL>(o, t, X0, Y0, rc, xpre);
}

// Up pass of one tile: stage 0 adds the prolongated correction to row r,
// stages 1..K relax in colours 1, 0, 1, ...; row r is written once stage K
// has passed it.  cr[q]: coarse correction of this lane's coarse column in
// coarse row Y0/2 - 1 + q.
template <typename T, bool VAR, bool BOUND, int NU, bool SMALL>
__device__ __forceinline__ void f_up_tile(const FOp<T> &o,
                                          FTile<T, FGeomU<T, NU, VAR, SMALL>::R> &t,
                                          const T (&cr)[FGeomU<T, NU, VAR, SMALL>::R / 2 + 3],
                                          int X0, int Y0, T *__restrict__ xout) {
  using G = FGeomU<T, NU, VAR, SMALL>;
  constexpr int K = G::K, H = G::H, R = G::R, HC = G::HC;
  const int lane = f_lane();
  const int gxa = X0 + 2 * lane;
  const bool inx = gxa >= 0 && gxa < o.nx;
  const bool lane_out = lane >= HC / 2 && lane < 64 - HC / 2 && gxa < o.nx;
  const T q = T(0.25);
  const T wxa = gxa == 0 ? o.pw : T(0.75);
  const T wxb = gxa + 2 == o.nx ? o.pw : T(0.75);
  auto row_in = [&](int r) { return !BOUND || (unsigned)(Y0 + r) < (unsigned)o.ny; };
#pragma unroll
  for (int step = 0; step < R + 2 * K + 1; ++step) {
#pragma unroll
    for (int k = 0; k <= K; ++k) {
      const int r = step - 2 * k;
      if (k == 0 && r < R) {
        f_coefs<T, VAR>(o, Y0 + r, gxa, BOUND ? inx : true, t.ca[r], t.cb[r]);
        const int gy = Y0 + r;
        const T wy = (gy == 0 || gy == o.ny - 1) ? o.pw : T(0.75);
        const T cj = cr[r / 2 + 1];
        const T cn = cr[(r & 1) ? r / 2 + 2 : r / 2];
        const T ya = wy * cj + q * cn;
        const T yp = wy * f_prev(cj) + q * f_prev(cn);
        const T yn = wy * f_next(cj) + q * f_next(cn);
        const bool in = !BOUND || (inx && row_in(r));
        t.xa[r] += in ? wxa * ya + q * yp : T(0);
        t.xb[r] += in ? wxb * ya + q * yn : T(0);
      } else if (k > 0 && r >= k && r < R - k) {
        if (row_in(r)) f_relax<T, R>(t, r, k & 1);
      }
    }
    const int rs = step - 2 * K;
    if (rs >= H && rs < R - H) {
      const int gy = Y0 + rs;
      if (lane_out && gy < o.ny) f_store2(xout + (size_t)gy * o.nx + gxa, t.xa[rs], t.xb[rs]);
    }
  }
}

template <typename T, bool VAR, int NU, bool SMALL>
__global__ void __launch_bounds__(64 * kFW)
    k_fup(FOp<T> o, const T *__restrict__ bin, const double *__restrict__ vin,
          const double *__restrict__ vscale, const T *__restrict__ xpre, const T *__restrict__ ec,
          T *__restrict__ xout) {
  using G = FGeomU<T, NU, VAR, SMALL>;
  constexpr int R = G::R;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = f_lane();
  const Tile2 tile = xcd_tile();
  const int OX = tile.x * G::TXO, OY = (tile.y * kFW + wave) * G::TY;
  if (OY >= o.ny) return;
  const int X0 = OX - G::HC, Y0 = OY - G::H;
  const int ncx = o.nx / 2, ncy = o.ny / 2;
  FTile<T, R> t;
  if (vin)
    f_load_v<T, R>(vin, vscale, t.ba, t.bb, X0, Y0, o.nx, o.ny);
  else
    f_load<T, R>(bin, t.ba, t.bb, X0, Y0, o.nx, o.ny);
  f_load<T, R>(xpre, t.xa, t.xb, X0, Y0, o.nx, o.ny);
  T cr[R / 2 + 3];
  {
    const int I = (X0 >> 1) + lane;
#pragma unroll
    for (int qq = 0; qq < R / 2 + 3; ++qq) {
      const int J = (Y0 >> 1) - 1 + qq;
      cr[qq] = (I >= 0 && I < ncx && J >= 0 && J < ncy) ? ec[(size_t)J * ncx + I] : T(0);
    }
  }
  if (X0 >= 0 && Y0 >= 0 && X0 + 128 <= o.nx && Y0 + R <= o.ny)
    f_up_tile<T, VAR, false, NU, SMALL>(o, t, cr, X0, Y0, xout);
  else
    f_up_tile<T, VAR, true, NU, SMALL>(o, t, cr, X0, Y0, xout);
}

template <typename G>
dim3 f_grid(int nx, int ny) {
  return dim3((nx + G::TXO - 1) / G::TXO, (ny + G::TY * kFW - 1) / (G::TY * kFW));
}

template <typename T>
FOp<T> make_fop(const FineOp<T> &F, int stage) {
  FOp<T> o{};
  o.nx = F.nx;
  o.ny = F.ny;
  o.pw = F.pw;
  if (F.kq) {
    o.kq = reinterpret_cast<const typename V4T<T>::V *>(F.kq);
    o.kc = F.kc;
    o.tau = F.tau[stage];
  } else {
    o.s = F.cs[stage][0];
    o.w = F.cs[stage][1];
    o.c = F.cs[stage][2];
    o.e = F.cs[stage][3];
    o.n = F.cs[stage][4];
    o.inv = T(1) / o.c;
  }
  return o;
}

template <typename G>
bool f_fills(int nx, int ny) {
  const dim3 g = f_grid<G>(nx, ny);
  return g.x * g.y >= 256;
}

template <typename T, bool VAR, int NU>
void fdown_launch(const FOp<T> &o, const T *b, const double *v0, const double *vs, T *rc, T *xpre,
                  hipStream_t st) {
  if (f_fills<FGeomD<T, NU, VAR>>(o.nx, o.ny))
    k_fdown<T, VAR, NU, false><<<f_grid<FGeomD<T, NU, VAR>>(o.nx, o.ny), 64 * kFW, 0, st>>>(
        o, b, v0, vs, rc, xpre);
  else
    k_fdown<T, VAR, NU, true><<<f_grid<FGeomD<T, NU, VAR, true>>(o.nx, o.ny), 64 * kFW, 0, st>>>(
        o, b, v0, vs, rc, xpre);
}
template <typename T, bool VAR, int NU>
void fup_launch(const FOp<T> &o, const T *b, const double *v0, const double *vs, const T *xpre,
                const T *ec, T *x, hipStream_t st) {
  if (f_fills<FGeomU<T, NU, VAR>>(o.nx, o.ny))
    k_fup<T, VAR, NU, false><<<f_grid<FGeomU<T, NU, VAR>>(o.nx, o.ny), 64 * kFW, 0, st>>>(
        o, b, v0, vs, xpre, ec, x);
  else
    k_fup<T, VAR, NU, true><<<f_grid<FGeomU<T, NU, VAR, true>>(o.nx, o.ny), 64 * kFW, 0, st>>>(
        o, b, v0, vs, xpre, ec, x);
}

}  // namespace

namespace kern {

template <typename T>
void fdown(const FineOp<T> &F, int stage, int nu, const T *b, T *rc, T *xpre, hipStream_t st,
           const double *v0, const double *v0scale) {
  const FOp<T> o = make_fop(F, stage);
  if (F.kq) {
    if (nu == 1) fdown_launch<T, true, 1>(o, b, v0, v0scale, rc, xpre, st);
    else if (nu == 2) fdown_launch<T, true, 2>(o, b, v0, v0scale, rc, xpre, st);
    else fdown_launch<T, true, 3>(o, b, v0, v0scale, rc, xpre, st);
  } else {
    if (nu == 1) fdown_launch<T, false, 1>(o, b, v0, v0scale, rc, xpre, st);
    else if (nu == 2) fdown_launch<T, false, 2>(o, b, v0, v0scale, rc, xpre, st);
    else fdown_launch<T, false, 3>(o, b, v0, v0scale, rc, xpre, st);
  }
}

template <typename T>
void fup(const FineOp<T> &F, int stage, int nu, const T *b, const T *xpre, const T *ec, T *x,
         hipStream_t st, const double *v0, const double *v0scale) {
  const FOp<T> o = make_fop(F, stage);
  if (F.kq) {
    if (nu == 1) fup_launch<T, true, 1>(o, b, v0, v0scale, xpre, ec, x, st);
    else if (nu == 2) fup_launch<T, true, 2>(o, b, v0, v0scale, xpre, ec, x, st);
    else fup_launch<T, true, 3>(o, b, v0, v0scale, xpre, ec, x, st);
  } else {
    if (nu == 1) fup_launch<T, false, 1>(o, b, v0, v0scale, xpre, ec, x, st);
    else if (nu == 2) fup_launch<T, false, 2>(o, b, v0, v0scale, xpre, ec, x, st);
    else fup_launch<T, false, 3>(o, b, v0, v0scale, xpre, ec, x, st);
  }
}

template void fdown<float>(const FineOp<float> &, int, int, const float *, float *, float *,
                           hipStream_t, const double *, const double *);
template void fup<float>(const FineOp<float> &, int, int, const float *, const float *,
                         const float *, float *, hipStream_t, const double *, const double *);
template void fdown<double>(const FineOp<double> &, int, int, const double *, double *, double *,
                            hipStream_t, const double *, const double *);
template void fup<double>(const FineOp<double> &, int, int, const double *, const double *,
                          const double *, double *, hipStream_t, const double *, const double *);

}  // namespace kern
}  // namespace irk

// ---------------------------------------------------------------------------
// Block-substitution coupling for stage i (Sec. 4.2) with a five-point K
// stored per node (FP64 arrays, coefficient k of node p at k * N + p):
//   b = scale_j v_i - K c,   c = sum_k C[k] z_k,
// FP64 arithmetic, b rounded once to the V-cycle's precision (as the
// constant-coefficient coupling pass).  Each wave covers 124 output columns
// (one halo column pair per side) and kVRows rows, with c on kVRows + 2 rows
// in registers.
namespace irk {
namespace {

// 4 rows per wave: v's and K's rows are loaded before the z rows, all in
// flight at once (8 rows with the K loads up front: 0.85 -> 1.00 ms per step
// for the coupling on double glazing 1024^2; 4 rows: 0.81).
constexpr int kVRows = 4;
constexpr int kVTXO = 124;

struct VCoupleList {
  double c[kMaxStages];
  int k[kMaxStages];
};

template <typename T>
struct VPair;
template <>
struct VPair<float> {
  using V = float2;
  __device__ static V make(double a, double b) { return make_float2((float)a, (float)b); }
};
template <>
struct VPair<double> {
  using V = double2;
  __device__ static V make(double a, double b) { return make_double2(a, b); }
};

template <int NK, typename T>
__global__ void __launch_bounds__(64 * kFW)
    k_scouple_v(int nx, int ny, const double *__restrict__ karr, const double *__restrict__ v,
                const double *__restrict__ scale_j, const T *__restrict__ z, VCoupleList cl,
                int i, T *__restrict__ b) {
  using P = VPair<T>;
  const int wave = threadIdx.x >> 6, lane = f_lane();
  const Tile2 tile = xcd_tile();
  const int OX = tile.x * kVTXO, OY = (tile.y * kFW + wave) * kVRows;
  if (OY >= ny) return;
  const int X0 = OX - 2, gxa = X0 + 2 * lane;
  const size_t N = (size_t)nx * ny;
  const bool inx = gxa >= 0 && gxa < nx;
  const bool out = lane >= 1 && lane < 63 && inx;
  const double sc = *scale_j;
  // v's rows first: their loads are in flight while the z rows arrive
  double2 vr[kVRows];
#pragma unroll
  for (int r = 0; r < kVRows; ++r) {
    const int gy = OY + r;
    vr[r] = make_double2(0.0, 0.0);
    if (inx && gy < ny) vr[r] = *reinterpret_cast<const double2 *>(v + (size_t)i * N + (size_t)gy * nx + gxa);
  }
  // K's rows next (five FP64 coefficient arrays; centre at 4)
  double2 kr[NK > 0 ? kVRows : 1][5];
  if (NK > 0) {
#pragma unroll
    for (int r = 0; r < kVRows; ++r) {
      const int gy = OY + r;
      const size_t p = (size_t)gy * nx + gxa;
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        constexpr int kk[5] = {1, 3, 4, 5, 7};
        kr[r][c] = make_double2(0.0, 0.0);
        if (inx && gy < ny) kr[r][c] = *reinterpret_cast<const double2 *>(karr + (size_t)kk[c] * N + p);
      }
    }
  }
  double ca[kVRows + 2], cb[kVRows + 2];
#pragma unroll
  for (int r = 0; r < kVRows + 2; ++r) {
    const int gy = OY - 1 + r;
    double ax = 0.0, ay = 0.0;
    if (inx && gy >= 0 && gy < ny) {
      const size_t p = (size_t)gy * nx + gxa;
#pragma unroll
      for (int m = 0; m < NK; ++m) {
        const typename P::V zz = *reinterpret_cast<const typename P::V *>(z + (size_t)cl.k[m] * N + p);
        ax += cl.c[m] * (double)zz.x;
        ay += cl.c[m] * (double)zz.y;
      }
    }
    ca[r] = ax;
    cb[r] = ay;
  }
#pragma unroll
  for (int r = 0; r < kVRows; ++r) {
    const int gy = OY + r;
    if (gy >= ny) break;
    const size_t p = (size_t)gy * nx + gxa;
    const double2 vv = vr[r];
    double va = sc * vv.x, vb = sc * vv.y;
    if (NK > 0) {
      const double2 ks = kr[r][0], kw = kr[r][1], kcn = kr[r][2], ke = kr[r][3], kn = kr[r][4];
      va -= kcn.x * ca[r + 1] + ks.x * ca[r] + kn.x * ca[r + 2] + kw.x * f_prev(cb[r + 1]) +
            ke.x * cb[r + 1];
      vb -= kcn.y * cb[r + 1] + ks.y * cb[r] + kn.y * cb[r + 2] + kw.y * ca[r + 1] +
            ke.y * f_next(ca[r + 1]);
    }
    if (out) *reinterpret_cast<typename P::V *>(b + p) = P::make(va, vb);
  }
}

}  // namespace

namespace kern {

template <typename T>
void scouple_var(int nx, int ny, const double *karr, const double *v, const double *scale_j,
                 const T *z, const double *C, int s, int i, T *b, hipStream_t st) {
  VCoupleList cl{};
  int nk = 0;
  for (int k = 0; k < s; ++k)
    if (C[k] != 0.0) {
      cl.c[nk] = C[k];
      cl.k[nk] = k;
      ++nk;
    }
  const dim3 grid((nx + kVTXO - 1) / kVTXO, (ny + kVRows * kFW - 1) / (kVRows * kFW));
#define L_VCOUPLE(NK_) \
  k_scouple_v<NK_, T><<<grid, 64 * kFW, 0, st>>>(nx, ny, karr, v, scale_j, z, cl, i, b)
  switch (nk) {
    case 0: L_VCOUPLE(0); break;
    case 1: L_VCOUPLE(1); break;
    case 2: L_VCOUPLE(2); break;
    case 3: L_VCOUPLE(3); break;
    case 4: L_VCOUPLE(4); break;
    case 5: L_VCOUPLE(5); break;
    case 6: L_VCOUPLE(6); break;
    default: L_VCOUPLE(7); break;
  }
#undef L_VCOUPLE
}
template void scouple_var<float>(int, int, const double *, const double *, const double *,
                                 const float *, const double *, int, int, float *, hipStream_t);
template void scouple_var<double>(int, int, const double *, const double *, const double *,
                                  const double *, const double *, int, int, double *, hipStream_t);

}  // namespace kern
}  // namespace irk
