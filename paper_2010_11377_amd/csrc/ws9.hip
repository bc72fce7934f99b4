// Split-column register tiles for nine-point levels with constant
// coefficients per boundary class (the Galerkin coarse levels of the heat
// hierarchy), in FP32 (the mixed form) or FP64.  Same layout as the five-point split kernels: lane l holds grid
// columns X0 + 2l (slot a) and X0 + 2l + 1 (slot b) of R rows; slot a of row
// r has colour r mod 2.
//
// Nine-point red-black relaxation is Jacobi within a colour: the diagonal
// neighbours of a node have its colour, so every update of a half sweep must
// read old values.  Row r's update reads rows r-1, r, r+1 and only rows r-1
// and r+1 hold same-colour nodes, so the new value of row r-1 is committed
// right after row r has been computed: one pending register, no copies.
//
// Boundary classes without per-row coefficient sets: the grid height is a
// multiple of the tile height, and the last tile column is shifted back so
// that it ends exactly on the grid (it writes only the outputs no other tile
// writes).  Then the grid's first row can only sit at tile row H, its last
// row at tile row H + TY - 1, its first column at lane H/2 (slot a) and its
// last column at lane 63 - H/2 (slot b): compile-time positions.  Other
// tiles may hold a boundary row or column only at their very edge (distance
// 0, when TY = H), where the halo has one row of slack; the host refuses
// grids where a boundary column would fall deeper into a neighbour's halo.
// Every other row uses the middle-row classes, whose coefficients each lane
// selects once (first-column, interior or last-column class); only the two
// boundary rows select their row class at the point of use.  Interior tiles
// use class 4 from scalar registers.  Nodes outside the grid are held at
// zero.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.hpp"

namespace irk {
namespace {

constexpr int kW9 = 4;  // waves per workgroup, stacked in y

__device__ __forceinline__ int l9() { return threadIdx.x & 63; }

__device__ __forceinline__ float nx9(float v) {  // value of lane + 1 (0 in lane 63)
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ float pv9(float v) {  // value of lane - 1 (0 in lane 0)
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ double nx9(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), 0x130, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double pv9(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), 0x138, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename T>
struct P9;  // two adjacent elements
template <>
struct P9<float> {
  using V = float2;
};
template <>
struct P9<double> {
  using V = double2;
};

// Class q = 3 cy + cx (cx, cy: 0 first, 1 inside, 2 last), coefficient
// k = 3 (dy + 1) + (dx + 1).  Only compile-time indices are used on the
// device, so the table stays in the kernel-argument segment.
template <typename T>
struct S9Op {
  int nx, ny;
  T c[9][9];
  T inv[9];  // 1 / c[q][4]
  T pw;      // prolongation weight of the outermost fine node
};

template <typename T>
S9Op<T> make_s9op(const OpView<T> &D, const T *classes) {
  S9Op<T> o;
  o.nx = D.nx;
  o.ny = D.ny;
  for (int q = 0; q < 9; ++q) {
    for (int k = 0; k < 9; ++k) o.c[q][k] = classes[q * 9 + k];
    o.inv[q] = T(1) / o.c[q][4];
  }
  o.pw = D.pw;
  return o;
}

template <typename T, int R>
struct T9 {
  T xa[R], xb[R], ba[R], bb[R];
};

template <typename T>
struct Co {
  T c[9];
  T inv;
  __device__ __forceinline__ T operator[](int k) const { return c[k]; }
};

// Per-wave tile placement and boundary flags.
struct Place {
  int X0, Y0;       // tile origin (halo included)
  int OXn, OYn;     // first output column / row this wave writes
  int lo, hi;       // output lanes [lo, hi) (before the shifted-tile cut)
  bool top, bot;    // grid row 0 at tile row H / row ny-1 at tile row H+TY-1
  bool fcol, lcol;  // this lane's slot a is column 0 / slot b is column nx-1
};

// The coefficients of slot a (side 0: first-column class when edge) or slot
// b (side 2: last-column class when edge) for row class CY.
template <int CY, int SIDE, typename T>
__device__ __forceinline__ Co<T> side_coefs(const S9Op<T> &o, bool edge) {
  constexpr int qe = 3 * CY + SIDE, qm = 3 * CY + 1;
  Co<T> r;
#pragma unroll
  for (int k = 0; k < 9; ++k) r.c[k] = edge ? o.c[qe][k] : o.c[qm][k];
  r.inv = edge ? o.inv[qe] : o.inv[qm];
  return r;
}

// Lane coefficients of a boundary tile, selected once per wave: the grid's
// first row (tile row H when the tile holds it), its last row (tile row
// H + TY - 1) and every other row.  Selecting them up front keeps the class
// table out of the registers for the rest of the kernel.
template <typename T>
struct RowCo {
  Co<T> a, b;
};
template <typename T>
struct MidCo {
  RowCo<T> top, mid, bot;
};

template <typename T>
__device__ __forceinline__ MidCo<T> mid_coefs(const S9Op<T> &o, const Place &p) {
  MidCo<T> m;
  m.mid.a = side_coefs<1, 0>(o, p.fcol);
  m.mid.b = side_coefs<1, 2>(o, p.lcol);
  m.top = m.mid;
  m.bot = m.mid;
  if (p.top) {
    m.top.a = side_coefs<0, 0>(o, p.fcol);
    m.top.b = side_coefs<0, 2>(o, p.lcol);
  }
  if (p.bot) {
    m.bot.a = side_coefs<2, 0>(o, p.fcol);
    m.bot.b = side_coefs<2, 2>(o, p.lcol);
  }
  // lanes outside the grid relax with 1 / d = 0, which keeps them at zero
  const int gxa = p.X0 + 2 * l9();
  if (gxa < 0 || gxa >= o.nx) {
    m.mid.a.inv = m.mid.b.inv = m.top.a.inv = m.top.b.inv = m.bot.a.inv = m.bot.b.inv = T(0);
  }
  return m;
}

// sum over the eight neighbours of slot a / slot b in row r
template <typename T, int R, typename C>
__device__ __forceinline__ T offdiag_a(const C &c, const T9<T, R> &t, int r) {
  return c[0] * pv9(t.xb[r - 1]) + c[1] * t.xa[r - 1] + c[2] * t.xb[r - 1] +
         c[3] * pv9(t.xb[r]) + c[5] * t.xb[r] +
         c[6] * pv9(t.xb[r + 1]) + c[7] * t.xa[r + 1] + c[8] * t.xb[r + 1];
}
template <typename T, int R, typename C>
__device__ __forceinline__ T offdiag_b(const C &c, const T9<T, R> &t, int r) {
  return c[0] * t.xa[r - 1] + c[1] * t.xb[r - 1] + c[2] * nx9(t.xa[r - 1]) +
         c[3] * t.xa[r] + c[5] * nx9(t.xa[r]) +
         c[6] * t.xa[r + 1] + c[7] * t.xb[r + 1] + c[8] * nx9(t.xa[r + 1]);
}

// Coefficients of slot a / b in tile row r.  YB: which tile rows lie
// outside the grid (0 none, 1 the rows above the grid's first row, tile rows
// < H, 2 those below its last row, tile rows >= H + TY): the grid height is a
// multiple of TY, so these are the only cases, known at compile time; 3 is
// both, a single tile row covering the grid).
template <typename T, bool BOUND, int R, int H, int TY, int YB = 0>
struct Ctx {
  const S9Op<T> &o;
  const Place &p;
  const MidCo<T> &m;
  // r is a compile-time row index after unrolling, so these fold to one set
  __device__ __forceinline__ Co<T> a(int r) const {
    if (!BOUND) return side_coefs<1, 1>(o, false);
    return r == H ? m.top.a : (r == H + TY - 1 ? m.bot.a : m.mid.a);
  }
  __device__ __forceinline__ Co<T> b(int r) const {
    if (!BOUND) return side_coefs<1, 1>(o, false);
    return r == H ? m.top.b : (r == H + TY - 1 ? m.bot.b : m.mid.b);
  }
  // tile row r lies in the grid; rows outside are never updated and stay zero
  __device__ __forceinline__ bool row_in(int r) const {
    return (YB & 1 ? r >= H : true) && (YB & 2 ? r < H + TY : true);
  }
  __device__ __forceinline__ bool lane_in() const {
    const int gxa = p.X0 + 2 * l9();
    return !BOUND || (gxa >= 0 && gxa < o.nx);
  }
};

// One colour half sweep over rows [M, R-M), Jacobi within the colour.
template <typename T, bool BOUND, int R, int H, int TY, int YB, int M>
__device__ __forceinline__ void s9_sweep(const Ctx<T, BOUND, R, H, TY, YB> &cx, T9<T, R> &t,
                                         int color) {
  T pend = T(0);
#pragma unroll
  for (int r = M; r < R - M; ++r) {
    T v = T(0);
    if (cx.row_in(r)) {
      if ((r & 1) == color) {
        const Co<T> c = cx.a(r);
        v = (t.ba[r] - offdiag_a<T, R>(c, t, r)) * c.inv;
      } else {
        const Co<T> c = cx.b(r);
        v = (t.bb[r] - offdiag_b<T, R>(c, t, r)) * c.inv;
      }
    }
    if (r > M) {  // row r-1 is no longer read by this half sweep
      if (((r - 1) & 1) == color)
        t.xa[r - 1] = pend;
      else
        t.xb[r - 1] = pend;
    }
    pend = v;
  }
  constexpr int rl = R - M - 1;
  if ((rl & 1) == color)
    t.xa[rl] = pend;
  else
    t.xb[rl] = pend;
}

template <typename T, bool BOUND, int R, int H, int TY, int YB, int NU>
__device__ __forceinline__ void s9_pre(const Ctx<T, BOUND, R, H, TY, YB> &cx, T9<T, R> &t) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    // from x = 0 the first colour-0 half sweep is x = b / d (b is zero
    // outside the grid, so this x is too)
    if ((r & 1) == 0) {
      t.xa[r] = t.ba[r] * cx.a(r).inv;
      t.xb[r] = T(0);
    } else {
      t.xb[r] = t.bb[r] * cx.b(r).inv;
      t.xa[r] = T(0);
    }
  }
  s9_sweep<T, BOUND, R, H, TY, YB, 1>(cx, t, 1);
  if (NU >= 2) {
    s9_sweep<T, BOUND, R, H, TY, YB, 2>(cx, t, 0);
    s9_sweep<T, BOUND, R, H, TY, YB, 3>(cx, t, 1);
  }
  if (NU >= 3) {
    s9_sweep<T, BOUND, R, H, TY, YB, 4>(cx, t, 0);
    s9_sweep<T, BOUND, R, H, TY, YB, 5>(cx, t, 1);
  }
}

// Post-smoothing in the reverse colour order (colour 1 first), from x exact
// on the whole tile (the stored pre-smoothed x plus the coarse correction).
template <typename T, bool BOUND, int R, int H, int TY, int YB, int NU>
__device__ __forceinline__ void s9_post(const Ctx<T, BOUND, R, H, TY, YB> &cx, T9<T, R> &t) {
  s9_sweep<T, BOUND, R, H, TY, YB, 1>(cx, t, 1);
  s9_sweep<T, BOUND, R, H, TY, YB, 2>(cx, t, 0);
  if (NU >= 2) {
    s9_sweep<T, BOUND, R, H, TY, YB, 3>(cx, t, 1);
    s9_sweep<T, BOUND, R, H, TY, YB, 4>(cx, t, 0);
  }
  if (NU >= 3) {
    s9_sweep<T, BOUND, R, H, TY, YB, 5>(cx, t, 1);
    s9_sweep<T, BOUND, R, H, TY, YB, 6>(cx, t, 0);
  }
}

// rc = R (b - D x), sum over 2 x 2 cells: both slots of one lane, two rows.
// Writes the coarse nodes of this wave's output rows and lanes.
template <typename T, bool BOUND, int R, int H, int TY, int YB>
__device__ __forceinline__ void s9_restrict(const Ctx<T, BOUND, R, H, TY, YB> &cx,
                                            const T9<T, R> &t, T *__restrict__ rcoarse) {
  const S9Op<T> &o = cx.o;
  const Place &p = cx.p;
  const int lane = l9();
  const int gxa = p.X0 + 2 * lane;
  const int ncx = o.nx / 2, ncy = o.ny / 2;
  const int I = gxa >> 1;
  const bool inx = cx.lane_in();
  const bool lane_out = lane >= p.lo && lane < p.hi && gxa >= p.OXn && I < ncx;
#pragma unroll
  for (int r = H; r < R - H; r += 2) {
    T sum = T(0);
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int rr = r + d;
      if (!cx.row_in(rr)) continue;
      const Co<T> ca = cx.a(rr), cb = cx.b(rr);
      const T ra = t.ba[rr] - ca.c[4] * t.xa[rr] - offdiag_a<T, R>(ca, t, rr);
      const T rb = t.bb[rr] - cb.c[4] * t.xb[rr] - offdiag_b<T, R>(cb, t, rr);
      sum += ra + rb;
    }
    // an outside node next to an inside one has a nonzero residual
    if (!inx) sum = T(0);
    const int gy0 = p.Y0 + r, J = gy0 >> 1;
    if (lane_out && gy0 >= p.OYn && J < ncy) rcoarse[(size_t)J * ncx + I] = sum;
  }
}

template <typename T, int R>
__device__ __forceinline__ void s9_load(const T *__restrict__ g, T (&a)[R], T (&b)[R], int X0,
                                        int Y0, int nx, int ny) {
  using V = typename P9<T>::V;
  const int gx = X0 + 2 * l9();
  const bool inx = gx >= 0 && gx < nx;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int gy = Y0 + r;
    V v{};
    if (inx && gy >= 0 && gy < ny) v = *reinterpret_cast<const V *>(g + (size_t)gy * nx + gx);
    a[r] = v.x;
    b[r] = v.y;
  }
}

__host__ __device__ constexpr int ev9(int h) { return (h + 1) & ~1; }

// Tile geometry: the down pass needs x exact on margin 2 nu for its
// residual, the up pass (which starts from the stored pre-smoothed x) needs
// 2 nu post half sweeps: row halo H = 2 nu either way.  In x the up pass
// needs one more column: the coarse correction of the outermost lanes lacks
// the coarse column beyond the tile, so its column halo is HX = H + 2.
// Short tiles (TY rows), so that many waves share a level and each wave's
// chain of sweeps stays short; TY must exceed H, or a boundary row would sit
// inside the second tile's halo with interior coefficients.
template <int NU_, int TY_, bool UP_>
struct G9 {
  static constexpr int NU = NU_, TY = TY_, H = ev9(2 * NU_);
  static constexpr int HX = H + (UP_ ? 2 : 0);
  static constexpr int R = TY + 2 * H;
  static constexpr int TXO = 128 - 2 * HX;
};
constexpr int kTY9 = 8;
static_assert(kTY9 > ev9(2 * 3), "tile height must exceed the row halo for nu <= 3");

// Placement of this wave's tile; false if the wave has no rows.  Needs
// nx >= TXO and ny a multiple of TY.
template <typename G, typename T>
__device__ __forceinline__ bool place(const S9Op<T> &o, Place &p) {
  const int wave = threadIdx.x >> 6;
  const Tile2 tile = xcd_tile();
  p.OXn = tile.x * G::TXO;
  p.OYn = (tile.y * kW9 + wave) * G::TY;
  if (p.OYn >= o.ny) return false;
  const int OX = min(p.OXn, o.nx - G::TXO), OY = p.OYn;
  p.X0 = OX - G::HX;
  p.Y0 = OY - G::H;
  p.lo = G::HX / 2;
  p.hi = 64 - G::HX / 2;
  p.top = OY == 0;
  p.bot = OY == o.ny - G::TY;
  const int lane = l9();
  p.fcol = OX == 0 && lane == G::HX / 2;
  p.lcol = OX == o.nx - G::TXO && lane == 63 - G::HX / 2;
  return true;
}

__device__ __forceinline__ bool boundary_tile(const Place &p, int R, int nx, int ny) {
  return !(p.X0 >= 1 && p.Y0 >= 1 && p.X0 + 128 <= nx - 1 && p.Y0 + R <= ny - 1);
}

template <typename T, bool BOUND, int R, int H, int TY, int YB, int NU>
__device__ __forceinline__ void s9_down_tile(const S9Op<T> &o, const Place &p, const MidCo<T> &m,
                                             T9<T, R> &t, T *__restrict__ rc) {
  const Ctx<T, BOUND, R, H, TY, YB> cx{o, p, m};
  s9_pre<T, BOUND, R, H, TY, YB, NU>(cx, t);
  s9_restrict<T, BOUND, R, H, TY, YB>(cx, t, rc);
}

// Pre-smoothing from zero and rc = R (b - D x); the pre-smoothed x of the
// output region goes to xpre for the up pass.
template <typename T, int NU, int TY>
__global__ void __launch_bounds__(64 * kW9)
    k_s9down(S9Op<T> o, const T *__restrict__ bin, T *__restrict__ rc, T *__restrict__ xpre) {
  using G = G9<NU, TY, false>;
  using V = typename P9<T>::V;
  constexpr int H = G::H, R = G::R;
  Place p;
  if (!place<G>(o, p)) return;
  T9<T, R> t;
  s9_load<T, R>(bin, t.ba, t.bb, p.X0, p.Y0, o.nx, o.ny);
  if (!boundary_tile(p, R, o.nx, o.ny)) {
    s9_down_tile<T, false, R, H, TY, 0, NU>(o, p, MidCo<T>{}, t, rc);
  } else {
    const MidCo<T> m = mid_coefs(o, p);
    if (p.top && p.bot)
      s9_down_tile<T, true, R, H, TY, 3, NU>(o, p, m, t, rc);
    else if (p.top)
      s9_down_tile<T, true, R, H, TY, 1, NU>(o, p, m, t, rc);
    else if (p.bot)
      s9_down_tile<T, true, R, H, TY, 2, NU>(o, p, m, t, rc);
    else
      s9_down_tile<T, true, R, H, TY, 0, NU>(o, p, m, t, rc);
  }
  const int lane = l9(), gxa = p.X0 + 2 * lane;
  if (lane >= p.lo && lane < p.hi && gxa >= p.OXn && gxa < o.nx) {
#pragma unroll
    for (int r = H; r < R - H; ++r) {
      const int gy = p.Y0 + r;
      if (gy < o.ny) {
        V v;
        v.x = t.xa[r];
        v.y = t.xb[r];
        *reinterpret_cast<V *>(xpre + (size_t)gy * o.nx + gxa) = v;
      }
    }
  }
}

// x = xpre + P e_c, then the post-smoothing.
template <typename T, bool BOUND, int R, int H, int TY, int YB, int NU>
__device__ __forceinline__ void s9_up_body(const Ctx<T, BOUND, R, H, TY, YB> &cx, T9<T, R> &t,
                                           const T (&cr)[R / 2 + 3]) {
  const S9Op<T> &o = cx.o;
  // fine column 2I takes 3/4 of coarse column I and 1/4 of I-1, column 2I+1
  // 3/4 of I and 1/4 of I+1, likewise in y; the outermost fine column / row
  // takes pw of its coarse node (its second coarse node is outside the grid,
  // where cr and the neighbour lanes hold zero)
  const int gxa = cx.p.X0 + 2 * l9();
  const bool inx = cx.lane_in();
  // lanes outside the grid take no correction
  const T wxa = !inx ? T(0) : (gxa == 0 ? o.pw : T(0.75));
  const T wxb = !inx ? T(0) : (gxa + 2 == o.nx ? o.pw : T(0.75));
  const T wq = !inx ? T(0) : T(0.25);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (!cx.row_in(r)) continue;
    const int gy = cx.p.Y0 + r;
    const T wy = (gy == 0 || gy == o.ny - 1) ? o.pw : T(0.75);
    const T cj = cr[r / 2 + 1];
    const T cn = cr[(r & 1) ? r / 2 + 2 : r / 2];
    const T ya = wy * cj + T(0.25) * cn;
    const T yp = wy * pv9(cj) + T(0.25) * pv9(cn);
    const T yn = wy * nx9(cj) + T(0.25) * nx9(cn);
    t.xa[r] += wxa * ya + wq * yp;
    t.xb[r] += wxb * ya + wq * yn;
  }
  s9_post<T, BOUND, R, H, TY, YB, NU>(cx, t);
}

template <typename T, bool BOUND, int R, int H, int TY, int YB, int NU>
__device__ __forceinline__ void s9_up_tile(const S9Op<T> &o, const Place &p, const MidCo<T> &m,
                                           T9<T, R> &t, const T (&cr)[R / 2 + 3]) {
  const Ctx<T, BOUND, R, H, TY, YB> cx{o, p, m};
  s9_up_body<T, BOUND, R, H, TY, YB, NU>(cx, t, cr);
}

template <typename T, int NU, int TY>
__global__ void __launch_bounds__(64 * kW9)
    k_s9up(S9Op<T> o, const T *__restrict__ bin, const T *__restrict__ ec,
           const T *__restrict__ xpre, T *__restrict__ xout) {
  using G = G9<NU, TY, true>;
  using V = typename P9<T>::V;
  constexpr int H = G::H, R = G::R;
  Place p;
  if (!place<G>(o, p)) return;
  const int lane = l9();
  const int ncx = o.nx / 2, ncy = o.ny / 2;
  T9<T, R> t;
  s9_load<T, R>(bin, t.ba, t.bb, p.X0, p.Y0, o.nx, o.ny);
  s9_load<T, R>(xpre, t.xa, t.xb, p.X0, p.Y0, o.nx, o.ny);
  T cr[R / 2 + 3];
  {
    const int I = (p.X0 >> 1) + lane;
#pragma unroll
    for (int q = 0; q < R / 2 + 3; ++q) {
      const int J = (p.Y0 >> 1) - 1 + q;
      cr[q] = (I >= 0 && I < ncx && J >= 0 && J < ncy) ? ec[(size_t)J * ncx + I] : T(0);
    }
  }
  if (!boundary_tile(p, R, o.nx, o.ny)) {
    s9_up_tile<T, false, R, H, TY, 0, NU>(o, p, MidCo<T>{}, t, cr);
  } else {
    const MidCo<T> m = mid_coefs(o, p);
    if (p.top && p.bot)
      s9_up_tile<T, true, R, H, TY, 3, NU>(o, p, m, t, cr);
    else if (p.top)
      s9_up_tile<T, true, R, H, TY, 1, NU>(o, p, m, t, cr);
    else if (p.bot)
      s9_up_tile<T, true, R, H, TY, 2, NU>(o, p, m, t, cr);
    else
      s9_up_tile<T, true, R, H, TY, 0, NU>(o, p, m, t, cr);
  }
  const int gxa = p.X0 + 2 * lane;
  if (lane >= p.lo && lane < p.hi && gxa >= p.OXn && gxa < o.nx) {
#pragma unroll
    for (int r = H; r < R - H; ++r) {
      const int gy = p.Y0 + r;
      if (gy < o.ny) {
        V v;
        v.x = t.xa[r];
        v.y = t.xb[r];
        *reinterpret_cast<V *>(xout + (size_t)gy * o.nx + gxa) = v;
      }
    }
  }
}

template <typename G>
dim3 grid9(int nx, int ny) {
  return dim3((nx + G::TXO - 1) / G::TXO, (ny + G::TY * kW9 - 1) / (G::TY * kW9));
}

// ===========================================================================
// The last level of a cycle that ends above the coarsest level: its V(nu, nu)
// with a zero coarse correction is the pre-smoothing from x = 0 followed by
// the post-smoothing, 4 nu - 1 half sweeps after the first, in one pass with
// a halo of that depth.  Tiles of 8 rows with a halo of 8: a boundary row can
// sit in another tile only on its never-relaxed edge row, whose wrong class
// reaches 7 rows in.  Column classes per lane from the global column, so any
// width works (a single tile column when the grid is narrower than one).
template <int NU_>
struct G9S {
  static constexpr int NU = NU_, TY = 8, H = ev9(4 * NU_ - 1), HX = H;
  static constexpr int R = TY + 2 * H;
  static constexpr int TXO = 128 - 2 * HX;
};

template <typename T, bool BOUND, int R, int H, int TY, int YB, int NU>
__device__ __forceinline__ void s9_smooth_tile(const S9Op<T> &o, const Place &p,
                                               const MidCo<T> &m, T9<T, R> &t) {
  const Ctx<T, BOUND, R, H, TY, YB> cx{o, p, m};
  s9_pre<T, BOUND, R, H, TY, YB, NU>(cx, t);
  s9_post<T, BOUND, R, H, TY, YB, NU>(cx, t);
}

template <typename T, int NU>
__global__ void __launch_bounds__(64 * kW9)
    k_s9smooth(S9Op<T> o, const T *__restrict__ bin, T *__restrict__ xout) {
  using G = G9S<NU>;
  using V = typename P9<T>::V;
  constexpr int H = G::H, R = G::R, TY = G::TY;
  const int wave = threadIdx.x >> 6, lane = l9();
  const Tile2 tile = xcd_tile();
  Place p;
  p.OXn = tile.x * G::TXO;
  p.OYn = (tile.y * kW9 + wave) * TY;
  if (p.OYn >= o.ny) return;
  const int OX = max(0, min(p.OXn, o.nx - G::TXO));
  p.X0 = OX - G::HX;
  p.Y0 = p.OYn - H;
  p.lo = G::HX / 2;
  p.hi = 64 - G::HX / 2;
  p.top = p.OYn == 0;
  p.bot = p.OYn == o.ny - TY;
  p.fcol = p.X0 + 2 * lane == 0;
  p.lcol = p.X0 + 2 * lane + 1 == o.nx - 1;
  T9<T, R> t;
  s9_load<T, R>(bin, t.ba, t.bb, p.X0, p.Y0, o.nx, o.ny);
  if (!boundary_tile(p, R, o.nx, o.ny)) {
    s9_smooth_tile<T, false, R, H, TY, 0, NU>(o, p, MidCo<T>{}, t);
  } else {
    const MidCo<T> m = mid_coefs(o, p);
    if (p.top && p.bot)
      s9_smooth_tile<T, true, R, H, TY, 3, NU>(o, p, m, t);
    else if (p.top)
      s9_smooth_tile<T, true, R, H, TY, 1, NU>(o, p, m, t);
    else if (p.bot)
      s9_smooth_tile<T, true, R, H, TY, 2, NU>(o, p, m, t);
    else
      s9_smooth_tile<T, true, R, H, TY, 0, NU>(o, p, m, t);
  }
  const int gxa = p.X0 + 2 * lane;
  if (lane >= p.lo && lane < p.hi && gxa >= p.OXn && gxa < o.nx) {
#pragma unroll
    for (int r = H; r < H + TY; ++r) {
      V v;
      v.x = t.xa[r];
      v.y = t.xb[r];
      *reinterpret_cast<V *>(xout + (size_t)(p.Y0 + r) * o.nx + gxa) = v;
    }
  }
}

// ===========================================================================
// Two adjacent levels in one launch (nu = 2), the fine level F and its coarse
// level C = F + 1, both nine-point with constant coefficients per class.
//
// Down: a workgroup owns a block of C of kD2TYC x kD2TXC nodes.  Its kD2W
// waves pre-smooth F on overlapping tiles that cover the 2 x 2 cells of that
// block widened by the halo H of C, restrict the residual into LDS, and store
// the pre-smoothed x of the F nodes inside the block; then wave 0 pre-smooths
// C on the LDS right-hand side (one register tile of 16 rows, 60 of its 128
// columns filled: the outputs lie at least H nodes inside the filled part, so
// the unfilled columns cannot reach them), stores C's x and b, and restricts
// C's residual to the next level.
//
// Up: a workgroup owns kU2W tiles of F of the single-level up pass (the same
// placement).  Its two waves first correct and post-smooth C on two register
// tiles of 16 rows that together cover every C node those tiles read, H nodes
// deeper, and park the needed part in LDS; then every wave post-smooths its
// tile of F with its C values taken from LDS.
//
// Row classes stay compile-time: a boundary row of C lies at a fixed tile row
// in the first and last workgroup rows and otherwise only at a tile's outer
// edge row, which is never relaxed.  Column classes are chosen per lane from
// the global column.  Each node goes through the same arithmetic as in the
// one-level passes, so the results are the same bits.
constexpr int kD2W = 4, kD2TYC = 8, kD2TXC = 52;
constexpr int kD2BC = kD2TXC + 8;  // coarse columns filled from LDS (outputs + 2 H)
constexpr int kU2W = 2;
constexpr int kU2XR = 4 * kU2W + 7;  // coarse rows the fine tiles read

__device__ __forceinline__ bool interior_w(int X0, int Y0, int w, int R, int nx, int ny) {
  return X0 >= 1 && Y0 >= 1 && X0 + w <= nx - 1 && Y0 + R <= ny - 1;
}

// Coarse right-hand sides of the 2 x 2 cells of a pre-smoothed tile's output
// rows (sums of the residual; zero outside the grid), one per lane and row pair.
template <typename T, bool BOUND, int R, int H, int TY, int YB>
__device__ __forceinline__ void s9_sums(const Ctx<T, BOUND, R, H, TY, YB> &cx, const T9<T, R> &t,
                                        T (&cs)[TY / 2]) {
  const bool inx = cx.lane_in();
#pragma unroll
  for (int r = H, k = 0; r < H + TY; r += 2, ++k) {
    T sum = T(0);
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int rr = r + d;
      if (!cx.row_in(rr)) continue;
      const Co<T> ca = cx.a(rr), cb = cx.b(rr);
      const T ra = t.ba[rr] - ca.c[4] * t.xa[rr] - offdiag_a<T, R>(ca, t, rr);
      const T rb = t.bb[rr] - cb.c[4] * t.xb[rr] - offdiag_b<T, R>(cb, t, rr);
      sum += ra + rb;
    }
    cs[k] = inx ? sum : T(0);
  }
}

template <typename T, bool BOUND, int R, int H, int TY, int YB>
__device__ __forceinline__ void s9_pre_sums(const S9Op<T> &o, const Place &p, const MidCo<T> &m,
                                            T9<T, R> &t, T (&cs)[TY / 2]) {
  const Ctx<T, BOUND, R, H, TY, YB> cx{o, p, m};
  s9_pre<T, BOUND, R, H, TY, YB, 2>(cx, t);
  s9_sums<T, BOUND, R, H, TY, YB>(cx, t, cs);
}

template <typename T>
__global__ void __launch_bounds__(64 * kD2W)
    k_s9down2(S9Op<T> of, S9Op<T> oc, const T *__restrict__ bin, T *__restrict__ xpre_f,
              T *__restrict__ b_c, T *__restrict__ xpre_c, T *__restrict__ rcc) {
  using V = typename P9<T>::V;
  constexpr int TY = 8, H = 4, HX = 4, R = 16;
  static_assert(2 * (kD2TYC + 2 * H) == kD2W * TY, "the fine tiles cover the coarse region");
  __shared__ T bc[kD2TYC + 2 * H][kD2BC];
  const int ncx = of.nx / 2, ncy = of.ny / 2;
  const Tile2 tile = xcd_tile();
  const int OXn = tile.x * kD2TXC;  // first coarse column this workgroup writes
  const int OXc = min(OXn, ncx - kD2TXC), OYc = tile.y * kD2TYC;
  const int Xc0 = OXc - H, Yc0 = OYc - H;  // origin of the coarse region
  const int wave = threadIdx.x >> 6, lane = l9();

  // ---- F: wave w pre-smooths rows OYf .. OYf + TY - 1 (halo H)
  {
    const int OYf = 2 * Yc0 + TY * wave;
    T cs[TY / 2];
#pragma unroll
    for (int k = 0; k < TY / 2; ++k) cs[k] = T(0);
    if (OYf >= 0 && OYf < of.ny) {
      Place p;
      p.X0 = 2 * Xc0 - HX;
      p.Y0 = OYf - H;
      p.OXn = 2 * OXn;
      p.OYn = OYf;
      p.lo = HX / 2;
      p.hi = 64 - HX / 2;
      p.top = OYf == 0;
      p.bot = OYf == of.ny - TY;
      p.fcol = p.X0 + 2 * lane == 0;
      p.lcol = p.X0 + 2 * lane + 1 == of.nx - 1;
      T9<T, R> t;
      s9_load<T, R>(bin, t.ba, t.bb, p.X0, p.Y0, of.nx, of.ny);
      if (interior_w(p.X0, p.Y0, 128, R, of.nx, of.ny)) {
        s9_pre_sums<T, false, R, H, TY, 0>(of, p, MidCo<T>{}, t, cs);
      } else {
        const MidCo<T> m = mid_coefs(of, p);
        if (p.top && p.bot)
          s9_pre_sums<T, true, R, H, TY, 3>(of, p, m, t, cs);
        else if (p.top)
          s9_pre_sums<T, true, R, H, TY, 1>(of, p, m, t, cs);
        else if (p.bot)
          s9_pre_sums<T, true, R, H, TY, 2>(of, p, m, t, cs);
        else
          s9_pre_sums<T, true, R, H, TY, 0>(of, p, m, t, cs);
      }
      // the pre-smoothed x of the fine nodes of this workgroup's coarse block
      const int gxa = p.X0 + 2 * lane;
      if (OYf >= 2 * OYc && OYf < 2 * (OYc + kD2TYC) && gxa >= 2 * OXn &&
          gxa < 2 * (OXc + kD2TXC) && gxa < of.nx) {
#pragma unroll
        for (int r = H; r < H + TY; ++r) {
          V v;
          v.x = t.xa[r];
          v.y = t.xb[r];
          *reinterpret_cast<V *>(xpre_f + (size_t)(p.Y0 + r) * of.nx + gxa) = v;
        }
      }
    }
    const int c = lane - HX / 2;
    if (c >= 0 && c < kD2BC) {
#pragma unroll
      for (int k = 0; k < TY / 2; ++k) bc[TY / 2 * wave + k][c] = cs[k];
    }
  }
  __syncthreads();
  if (wave != 0) return;

  // ---- C: one tile of R = 16 rows on the coarse region
  Place p;
  p.X0 = Xc0;
  p.Y0 = Yc0;
  p.OXn = OXn;
  p.OYn = OYc;
  p.lo = H / 2;
  p.hi = H / 2 + kD2TXC / 2;
  p.top = OYc == 0;
  p.bot = OYc == ncy - kD2TYC;
  p.fcol = p.X0 + 2 * lane == 0;
  p.lcol = p.X0 + 2 * lane + 1 == ncx - 1;
  T9<T, R> t;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    T a = T(0), b = T(0);
    if (lane < kD2BC / 2) {
      a = bc[r][2 * lane];
      b = bc[r][2 * lane + 1];
    }
    t.ba[r] = a;
    t.bb[r] = b;
  }
  if (interior_w(p.X0, p.Y0, kD2BC, R, ncx, ncy)) {
    s9_down_tile<T, false, R, H, TY, 0, 2>(oc, p, MidCo<T>{}, t, rcc);
  } else {
    const MidCo<T> m = mid_coefs(oc, p);
    if (p.top && p.bot)
      s9_down_tile<T, true, R, H, TY, 3, 2>(oc, p, m, t, rcc);
    else if (p.top)
      s9_down_tile<T, true, R, H, TY, 1, 2>(oc, p, m, t, rcc);
    else if (p.bot)
      s9_down_tile<T, true, R, H, TY, 2, 2>(oc, p, m, t, rcc);
    else
      s9_down_tile<T, true, R, H, TY, 0, 2>(oc, p, m, t, rcc);
  }
  const int gxa = p.X0 + 2 * lane;
  if (lane >= p.lo && lane < p.hi && gxa >= OXn && gxa < ncx) {
#pragma unroll
    for (int r = H; r < H + TY; ++r) {
      const size_t q = (size_t)(p.Y0 + r) * ncx + gxa;
      V v;
      v.x = t.xa[r];
      v.y = t.xb[r];
      *reinterpret_cast<V *>(xpre_c + q) = v;
      v.x = t.ba[r];
      v.y = t.bb[r];
      *reinterpret_cast<V *>(b_c + q) = v;
    }
  }
}

template <typename T, bool BOUND, int HC, int YB>
__device__ __forceinline__ void s9_up_coarse(const S9Op<T> &o, const Place &p, T9<T, 16> &t,
                                             const T (&cr)[11]) {
  const MidCo<T> m = BOUND ? mid_coefs(o, p) : MidCo<T>{};
  s9_up_tile<T, BOUND, 16, HC, 8, YB, 2>(o, p, m, t, cr);
}

// One of the two coarse tiles of the up pair: rows Y0 .. Y0 + 15, where the
// grid's first row can only sit at tile row HC and its last at HC + 7.
template <typename T, int HC>
__device__ __forceinline__ void s9_up_coarse_any(const S9Op<T> &o, const Place &p, T9<T, 16> &t,
                                                 const T (&cr)[11], bool interior) {
  if (interior)
    s9_up_coarse<T, false, HC, 0>(o, p, t, cr);
  else if (p.top && p.bot)
    s9_up_coarse<T, true, HC, 3>(o, p, t, cr);
  else if (p.top)
    s9_up_coarse<T, true, HC, 1>(o, p, t, cr);
  else if (p.bot)
    s9_up_coarse<T, true, HC, 2>(o, p, t, cr);
  else
    s9_up_coarse<T, true, HC, 0>(o, p, t, cr);
}

template <typename T>
__global__ void __launch_bounds__(64 * kU2W)
    k_s9up2(S9Op<T> of, S9Op<T> oc, const T *__restrict__ bf, const T *__restrict__ xpre_f,
            const T *__restrict__ b_c, const T *__restrict__ xpre_c, const T *__restrict__ ecc,
            T *__restrict__ xf) {
  using G = G9<2, 8, true>;
  using V = typename P9<T>::V;
  constexpr int H = G::H, R = G::R, TY = G::TY;
  static_assert(kU2W == 2 && kU2XR == 15, "two coarse tiles of 16 rows cover the rows read");
  __shared__ T xs[kU2XR][64];
  const int ncx = of.nx / 2, ncy = of.ny / 2;
  const Tile2 tile = xcd_tile();
  const int OXn = tile.x * G::TXO, OX = min(OXn, of.nx - G::TXO);
  const int OY = tile.y * TY * kU2W;
  const int X0f = OX - G::HX;
  const int Ic = X0f >> 1;              // coarse column of lane 0 in the fine tiles
  const int Jlo = ((OY - H) >> 1) - 1;  // first coarse row the fine tiles read
  const int wave = threadIdx.x >> 6, lane = l9();

  // in FP32 the fine tile's inputs are read first, so that their latency
  // overlaps the coarse work; in FP64 they are read after it (register room)
  constexpr bool kEarly = std::is_same_v<T, float>;
  Place p;
  p.OXn = OXn;
  p.OYn = OY + TY * wave;
  p.X0 = X0f;
  p.Y0 = p.OYn - H;
  p.lo = G::HX / 2;
  p.hi = 64 - G::HX / 2;
  p.top = p.OYn == 0;
  p.bot = p.OYn == of.ny - TY;
  p.fcol = OX == 0 && lane == G::HX / 2;
  p.lcol = OX == of.nx - G::TXO && lane == 63 - G::HX / 2;
  T9<T, R> t;
  if (kEarly) {
    s9_load<T, R>(bf, t.ba, t.bb, p.X0, p.Y0, of.nx, of.ny);
    s9_load<T, R>(xpre_f, t.xa, t.xb, p.X0, p.Y0, of.nx, of.ny);
  }

  // ---- C: the rows read are Jlo .. Jlo + 14; wave 0 corrects and
  // post-smooths coarse rows Y0c .. Y0c + 15 (valid 4 .. 11), wave 1 rows
  // Y0c + 8 .. Y0c + 23 (valid 12 .. 19), with Y0c = Jlo - 5.  The correction
  // leaves a tile's outermost columns without their outer coarse neighbour,
  // so the columns read lie H + 1 inside the tile.
  {
    const int X0c = (Ic - H - 1) & ~1, Y0c = (Jlo - H) & ~1;
    Place pc;
    pc.X0 = X0c;
    pc.Y0 = Y0c + 8 * wave;
    pc.OXn = pc.OYn = 0;
    pc.lo = 0;
    pc.hi = 64;
    pc.top = OY == 0;
    pc.bot = OY == of.ny - TY * kU2W;
    pc.fcol = X0c + 2 * lane == 0;
    pc.lcol = X0c + 2 * lane + 1 == ncx - 1;
    T9<T, 16> tc;
    s9_load<T, 16>(b_c, tc.ba, tc.bb, pc.X0, pc.Y0, ncx, ncy);
    s9_load<T, 16>(xpre_c, tc.xa, tc.xb, pc.X0, pc.Y0, ncx, ncy);
    T cr[11];
    {
      const int ncx2 = ncx / 2, ncy2 = ncy / 2;
      const int I = (X0c >> 1) + lane;
#pragma unroll
      for (int q = 0; q < 11; ++q) {
        const int J = (pc.Y0 >> 1) - 1 + q;
        cr[q] = (I >= 0 && I < ncx2 && J >= 0 && J < ncy2) ? ecc[(size_t)J * ncx2 + I] : T(0);
      }
    }
    const bool interior = interior_w(X0c, Y0c, 2 * 40, 24, ncx, ncy);
    // the grid's first row sits at row 8 of the first tile (row 0 of the
    // second, its never-relaxed edge); the last at row 15 of the first tile
    // (its edge) and row 7 of the second
    if (wave == 0)
      s9_up_coarse_any<T, 8>(oc, pc, tc, cr, interior);
    else
      s9_up_coarse_any<T, 0>(oc, pc, tc, cr, interior);
    // park rows 4 .. 11 of the tile that are read, columns Ic .. Ic + 63
    const int dc = Ic - X0c;
    const int ca = 2 * lane - dc, cb = ca + 1;
    const int q0 = pc.Y0 - Jlo;  // row of tile row 0 in xs
#pragma unroll
    for (int r = 4; r < 12; ++r) {
      const int q = q0 + r;
      if (q >= 0 && q < kU2XR) {
        if (ca >= 0 && ca < 64) xs[q][ca] = tc.xa[r];
        if (cb >= 0 && cb < 64) xs[q][cb] = tc.xb[r];
      }
    }
  }
  __syncthreads();

  // ---- F: the single-level up tile of wave w, C values from LDS
  if (!kEarly) {
    s9_load<T, R>(bf, t.ba, t.bb, p.X0, p.Y0, of.nx, of.ny);
    s9_load<T, R>(xpre_f, t.xa, t.xb, p.X0, p.Y0, of.nx, of.ny);
  }
  T cr[R / 2 + 3];
#pragma unroll
  for (int q = 0; q < R / 2 + 3; ++q) cr[q] = xs[TY / 2 * wave + q][lane];
  if (!boundary_tile(p, R, of.nx, of.ny)) {
    s9_up_tile<T, false, R, H, TY, 0, 2>(of, p, MidCo<T>{}, t, cr);
  } else {
    const MidCo<T> m = mid_coefs(of, p);
    if (p.top && p.bot)
      s9_up_tile<T, true, R, H, TY, 3, 2>(of, p, m, t, cr);
    else if (p.top)
      s9_up_tile<T, true, R, H, TY, 1, 2>(of, p, m, t, cr);
    else if (p.bot)
      s9_up_tile<T, true, R, H, TY, 2, 2>(of, p, m, t, cr);
    else
      s9_up_tile<T, true, R, H, TY, 0, 2>(of, p, m, t, cr);
  }
  const int gxa = p.X0 + 2 * lane;
  if (lane >= p.lo && lane < p.hi && gxa >= p.OXn && gxa < of.nx) {
#pragma unroll
    for (int r = H; r < R - H; ++r) {
      V v;
      v.x = t.xa[r];
      v.y = t.xb[r];
      *reinterpret_cast<V *>(xf + (size_t)(p.Y0 + r) * of.nx + gxa) = v;
    }
  }
}

// Grid shapes the tiling takes: even dimensions, nx >= 128, ny a multiple of
// TY, and the grid's last column not inside the halo of the second-to-last
// tile column (nx mod TXO zero or beyond the halo width H).
template <typename G>
bool geometry_ok(int nx, int ny) {
  const int rx = nx % G::TXO;
  return nx % 2 == 0 && ny % 2 == 0 && nx >= 128 && ny % G::TY == 0 && (rx == 0 || rx > G::HX);
}

}  // namespace

namespace kern {

template <int NU>
bool level_ok(int nx, int ny) {
  return geometry_ok<G9<NU, kTY9, false>>(nx, ny) && geometry_ok<G9<NU, kTY9, true>>(nx, ny);
}

template <typename T>
bool ws9_ok(const OpView<T> &D, int nu) {
  if (D.npt != 9 || !D.cls || D.arr) return false;
  if (nu == 1) return level_ok<1>(D.nx, D.ny);
  if (nu == 2) return level_ok<2>(D.nx, D.ny);
  return level_ok<3>(D.nx, D.ny);
}

template bool ws9_ok<float>(const OpView<float> &, int);
template bool ws9_ok<double>(const OpView<double> &, int);

#define IRK_S9_NU(KERNEL, UP, ...)                                                             \
  do {                                                                                         \
    if (nu == 1)                                                                               \
      KERNEL<T, 1, kTY9><<<grid9<G9<1, kTY9, UP>>(o.nx, o.ny), 64 * kW9, 0, st>>>(__VA_ARGS__); \
    else if (nu == 2)                                                                          \
      KERNEL<T, 2, kTY9><<<grid9<G9<2, kTY9, UP>>(o.nx, o.ny), 64 * kW9, 0, st>>>(__VA_ARGS__); \
    else                                                                                       \
      KERNEL<T, 3, kTY9><<<grid9<G9<3, kTY9, UP>>(o.nx, o.ny), 64 * kW9, 0, st>>>(__VA_ARGS__); \
  } while (0)

template <typename T>
void s9down(const OpView<T> &D, const T *classes, int nu, const T *b, T *rc, T *xpre,
            hipStream_t st) {
  const S9Op<T> o = make_s9op(D, classes);
  IRK_S9_NU(k_s9down, false, o, b, rc, xpre);
}

template <typename T>
void s9up(const OpView<T> &D, const T *classes, int nu, const T *b, const T *ec, const T *xpre,
          T *x, hipStream_t st) {
  const S9Op<T> o = make_s9op(D, classes);
  IRK_S9_NU(k_s9up, true, o, b, ec, xpre, x);
}

template void s9down<float>(const OpView<float> &, const float *, int, const float *, float *,
                            float *, hipStream_t);
template void s9down<double>(const OpView<double> &, const double *, int, const double *,
                             double *, double *, hipStream_t);
template void s9up<float>(const OpView<float> &, const float *, int, const float *, const float *,
                          const float *, float *, hipStream_t);

// Pairs: nu = 2, both levels on the register tiling, C = F / 2 exactly, F's
// height a multiple of 16 (C's a multiple of the coarse block height) and
// C's width at least one coarse block.
template <typename T>
bool s9pair_ok(const OpView<T> &Df, const OpView<T> &Dc, int nu) {
  if (nu != 2 || !ws9_ok<T>(Df, nu) || !ws9_ok<T>(Dc, nu)) return false;
  if (Dc.nx * 2 != Df.nx || Dc.ny * 2 != Df.ny) return false;
  return Df.nx % 4 == 0 && Df.ny % (2 * kD2TYC) == 0 && Dc.nx >= kD2TXC &&
         Df.nx >= G9<2, kTY9, true>::TXO;
}

template <typename T>
void s9down2(const OpView<T> &Df, const T *cls_f, const OpView<T> &Dc, const T *cls_c,
             const T *b, T *xpre_f, T *b_c, T *xpre_c, T *rcc, hipStream_t st) {
  const S9Op<T> of = make_s9op(Df, cls_f), oc = make_s9op(Dc, cls_c);
  const dim3 grid((Dc.nx + kD2TXC - 1) / kD2TXC, Dc.ny / kD2TYC);
  k_s9down2<T><<<grid, 64 * kD2W, 0, st>>>(of, oc, b, xpre_f, b_c, xpre_c, rcc);
}

template <typename T>
void s9up2(const OpView<T> &Df, const T *cls_f, const OpView<T> &Dc, const T *cls_c, const T *b,
           const T *xpre_f, const T *b_c, const T *xpre_c, const T *ecc, T *x, hipStream_t st) {
  using G = G9<2, kTY9, true>;
  const S9Op<T> of = make_s9op(Df, cls_f), oc = make_s9op(Dc, cls_c);
  const dim3 grid((Df.nx + G::TXO - 1) / G::TXO, Df.ny / (G::TY * kU2W));
  k_s9up2<T><<<grid, 64 * kU2W, 0, st>>>(of, oc, b, xpre_f, b_c, xpre_c, ecc, x);
}

// The end-level pass: nine-point classes, linear interpolation, nu = 2, even
// width, height a multiple of the tile height.
template <typename T>
bool s9smooth_ok(const OpView<T> &D, int nu) {
  return nu == 2 && D.npt == 9 && D.cls && !D.arr && D.nx % 2 == 0 && D.nx >= 2 &&
         D.ny % G9S<2>::TY == 0;
}

template <typename T>
void s9smooth(const OpView<T> &D, const T *classes, const T *b, T *x, hipStream_t st) {
  using G = G9S<2>;
  const S9Op<T> o = make_s9op(D, classes);
  const dim3 grid((D.nx + G::TXO - 1) / G::TXO, (D.ny + G::TY * kW9 - 1) / (G::TY * kW9));
  k_s9smooth<T, 2><<<grid, 64 * kW9, 0, st>>>(o, b, x);
}

template bool s9smooth_ok<float>(const OpView<float> &, int);
template bool s9smooth_ok<double>(const OpView<double> &, int);
template void s9smooth<float>(const OpView<float> &, const float *, const float *, float *,
                              hipStream_t);
template void s9smooth<double>(const OpView<double> &, const double *, const double *, double *,
                               hipStream_t);

template bool s9pair_ok<float>(const OpView<float> &, const OpView<float> &, int);
template bool s9pair_ok<double>(const OpView<double> &, const OpView<double> &, int);
template void s9down2<float>(const OpView<float> &, const float *, const OpView<float> &,
                             const float *, const float *, float *, float *, float *, float *,
                             hipStream_t);
template void s9down2<double>(const OpView<double> &, const double *, const OpView<double> &,
                              const double *, const double *, double *, double *, double *,
                              double *, hipStream_t);
template void s9up2<float>(const OpView<float> &, const float *, const OpView<float> &,
                           const float *, const float *, const float *, const float *,
                           const float *, const float *, float *, hipStream_t);
template void s9up2<double>(const OpView<double> &, const double *, const OpView<double> &,
                            const double *, const double *, const double *, const double *,
                            const double *, const double *, double *, hipStream_t);
template void s9up<double>(const OpView<double> &, const double *, int, const double *,
                           const double *, const double *, double *, hipStream_t);

}  // namespace kern
}  // namespace irk
