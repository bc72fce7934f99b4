// Split-column register tiles for the finest-level V-cycle passes in FP32.
//
// Lane l of a wavefront holds grid columns X0 + 2l ("slot a") and X0 + 2l + 1
// ("slot b") of R consecutive grid rows in registers; X0 and Y0 are even.
// For the red-black colouring (i + j) mod 2 the colour of slot a in row r is
// r mod 2 and slot b has the other one, so every lane of a half sweep updates
// exactly one of its two columns and which one is fixed at compile time for
// each row: no idle lanes and no per-lane colour masks.  West/east
// neighbours across the lane pair come from the adjacent lane through DPP
// wave shifts; north/south neighbours are registers of the same lane.  The
// 2 x 2 restriction sums the two slots of two rows in one lane, and the
// bilinear prolongation takes the neighbouring coarse column from the next or
// previous lane.
//
// Five-point constant-coefficient operators whose boundary rows are the
// interior stencil without the couplings that leave the grid (the heat
// operator and the shifted operators I + tau K built from it), on grids with
// even nx and ny.  Nodes outside the grid are held at zero.  The interior
// coefficients travel as kernel arguments.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace irk {
namespace {

constexpr int kSW = 4;  // waves per workgroup, stacked in y

__device__ __forceinline__ int s_lane() { return threadIdx.x & 63; }

__device__ __forceinline__ float s_next(float v) {  // value of lane + 1 (0 in lane 63)
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ float s_prev(float v) {  // value of lane - 1 (0 in lane 0)
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}

// Interior five-point coefficients: south (k=1), west (3), centre (4),
// east (5), north (7), and 1 / centre.
struct SOp {
  int nx, ny;
  float s, w, c, e, n, inv;
  float pw;  // prolongation weight of the outermost fine node
};

SOp make_sop(const OpView<float> &D, const float *interior) {
  SOp o;
  o.nx = D.nx;
  o.ny = D.ny;
  o.s = interior[1];
  o.w = interior[3];
  o.c = interior[4];
  o.e = interior[5];
  o.n = interior[7];
  o.inv = 1.0f / o.c;
  o.pw = D.pw;
  return o;
}

template <int R>
struct STile {
  float xa[R], xb[R], ba[R], bb[R];
};

// Row pipeline of the down pass.  The pass is a sequence of stages (the
// first colour-0 half sweep from x = 0, the red-black half sweeps, the
// restriction), each over a range of tile rows.  Stage k touches row r at
// step r + kSkew k.  Every stage reads rows r - 1 .. r + 1 as the previous
// stage left them (a five-point half sweep reads the other colour, which
// only the previous half sweep wrote): with kSkew = 2, at step r + 2k row
// r + 1 has been through stage k - 1 (step r + 2k - 1) but not k, and row
// r - 1 through stage k but not k + 1 (step r + 2k + 1), which are exactly
// the values a stage-by-stage order reads; the stages of one step are
// independent of each other, so the wave has several row updates in flight.
// Row by row, it works on the first rows while the later ones are still
// loading, and writes its outputs while it is still computing.  The down
// pass is latency bound (a few hundred instructions per wave after long
// loads), so this overlap is what counts; the up pass, bound by its
// arithmetic, keeps the stage-by-stage order below.
constexpr int kSkew = 2;

// Stage 0: x = b / d on colour 0 (slot a of even rows, slot b of odd rows)
// and zero on colour 1; b is zero outside the grid, so this x is too.
template <int R>
__device__ __forceinline__ void s_init_row(const SOp &o, STile<R> &t, int r) {
  if ((r & 1) == 0) {
    t.xa[r] = t.ba[r] * o.inv;
    t.xb[r] = 0.0f;
  } else {
    t.xb[r] = t.bb[r] * o.inv;
    t.xa[r] = 0.0f;
  }
}

// One row of a colour half sweep with 1 / centre = inv: the lanes outside
// the grid take inv = 0, which keeps them at zero (rows outside the grid are
// skipped altogether).
template <int R>
__device__ __forceinline__ void s_relax_row(const SOp &o, STile<R> &t, int r, int color,
                                            float inv) {
  if ((r & 1) == color) {  // slot a has colour r mod 2
    t.xa[r] = (t.ba[r] - o.s * t.xa[r - 1] - o.n * t.xa[r + 1] - o.w * s_prev(t.xb[r]) -
               o.e * t.xb[r]) * inv;
  } else {
    t.xb[r] = (t.bb[r] - o.s * t.xb[r - 1] - o.n * t.xb[r + 1] - o.w * t.xa[r] -
               o.e * s_next(t.xa[r])) * inv;
  }
}

// Residual b - D x of row r, summed over the lane's two slots.
template <int R>
__device__ __forceinline__ float s_resid_pair(const SOp &o, const STile<R> &t, int r) {
  const float ra = t.ba[r] - o.c * t.xa[r] - o.s * t.xa[r - 1] - o.n * t.xa[r + 1] -
                   o.w * s_prev(t.xb[r]) - o.e * t.xb[r];
  const float rb = t.bb[r] - o.c * t.xb[r] - o.s * t.xb[r - 1] - o.n * t.xb[r + 1] -
                   o.w * t.xa[r] - o.e * s_next(t.xa[r]);
  return ra + rb;
}

// Rows Y0..Y0+R-1 of a grid vector, columns X0+2l and X0+2l+1, zero outside.
template <int R>
__device__ __forceinline__ void s_load(const float *__restrict__ g, float (&a)[R], float (&b)[R],
                                       int X0, int Y0, int nx, int ny) {
  const int gx = X0 + 2 * s_lane();
  const bool inx = gx >= 0 && gx < nx;  // nx and gx even: gx + 1 < nx too
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int gy = Y0 + r;
    float2 v = make_float2(0.0f, 0.0f);
    if (inx && gy >= 0 && gy < ny) v = *reinterpret_cast<const float2 *>(g + (size_t)gy * nx + gx);
    a[r] = v.x;
    b[r] = v.y;
  }
}

// The right-hand side of a block without coupling terms is scale_j v_i
// rounded to FP32, formed here on load from the FP64 Krylov vector (the same
// bits the coupling pass would write), so that block needs no pass of its own.
template <int R>
__device__ __forceinline__ void s_load_scaled(const double *__restrict__ g, double sc,
                                              float (&a)[R], float (&b)[R], int X0, int Y0,
                                              int nx, int ny) {
  const int gx = X0 + 2 * s_lane();
  const bool inx = gx >= 0 && gx < nx;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int gy = Y0 + r;
    double2 v = make_double2(0.0, 0.0);
    if (inx && gy >= 0 && gy < ny) v = *reinterpret_cast<const double2 *>(g + (size_t)gy * nx + gx);
    a[r] = (float)(sc * v.x);
    b[r] = (float)(sc * v.y);
  }
}

// Right-hand side source of the finest-level passes: FP32 b, or (VIN) FP64 v
// scaled by *vscale.
struct BIn {
  const float *b;
  const double *v;
  const double *vscale;
};

template <bool VIN, int R>
__device__ __forceinline__ void s_load_b(const BIn &in, float (&a)[R], float (&b)[R], int X0,
                                         int Y0, int nx, int ny) {
  if (VIN)
    s_load_scaled<R>(in.v, *in.vscale, a, b, X0, Y0, nx, ny);
  else
    s_load<R>(in.b, a, b, X0, Y0, nx, ny);
}

__device__ __forceinline__ bool s_interior(int X0, int Y0, int R, int nx, int ny) {
  return X0 >= 0 && Y0 >= 0 && X0 + 128 <= nx && Y0 + R <= ny;
}

__host__ __device__ constexpr int even_up(int h) { return (h + 1) & ~1; }

// Tile geometry: TY output rows per wave, R = TY + 2H register rows, TXO
// output columns.  The down pass needs x exact on margin 2 nu + 1 for its
// residual; the up pass repeats the 2 nu pre-sweeps and adds 2 nu
// post-sweeps.  Halos are even so that the tile origin stays even.  Short
// down tiles: the latency-bound down pass runs best with many short waves
// (two or three per SIMD hide each other's load latency); the up pass is
// bound by its arithmetic, where the halo's share of the work decides.
// SMALL: 4-row tiles for grids whose tall tiles would leave CUs without a
// workgroup (below 256 of them): more, shorter row chains.
template <int NU, bool SMALL = false>
struct SGeomD {
  static constexpr int H = even_up(2 * NU);
  static constexpr int TY = SMALL ? 4 : 16;
  static constexpr int R = TY + 2 * H;
  static constexpr int TXO = 128 - 2 * H;
};
template <int NU, bool SMALL = false>
struct SGeomU {
  static constexpr int H = even_up(4 * NU - 1);
  static constexpr int TY = SMALL ? 4 : (NU == 1 ? 32 : (NU == 2 ? 24 : 16));
  static constexpr int R = TY + 2 * H;
  static constexpr int TXO = 128 - 2 * H;
};

// Pre-smoothing from x = 0 (stage 0, then 2 nu - 1 half sweeps; sweep k
// covers rows [k, R - k) in colour k mod 2) and rc = R (b - D x) with R the
// sum over 2 x 2 cells: coarse node (I, J) takes fine columns 2I, 2I+1 of
// rows 2J, 2J+1, i.e. both slots of one lane in two rows.  Written for output
// rows [H, R-H) and lanes [H/2, 64-H/2); the pair of rows r0, r0 + 1 is
// restricted once rows r0 - 1 .. r0 + 2 are final.
//
// BOUND: the tile reaches past the grid.  Its nodes outside stay zero: rows
// outside (Y0 is the same for the whole wave, so the test is a scalar
// branch) are never updated, lanes outside relax with inv = 0, and the
// residual of an outside node (nonzero next to a nonzero inside one) is left
// out of the sums.
template <bool BOUND, int R, int NU, int H>
__device__ __forceinline__ void s_down_rows(const SOp &o, STile<R> &t, int X0, int Y0,
                                            float *__restrict__ rc) {
  constexpr int K = 2 * NU;
  const int lane = s_lane();
  const int gxa = X0 + 2 * lane;
  const int ncx = o.nx / 2, ncy = o.ny / 2;
  const int I = gxa >> 1;
  const bool inx = gxa >= 0 && gxa < o.nx;  // nx even: slot b is inside iff slot a is
  const bool lane_out = lane >= H / 2 && lane < 64 - H / 2 && I < ncx;
  const float inv = BOUND && !inx ? 0.0f : o.inv;
  auto row_in = [&](int r) { return !BOUND || (unsigned)(Y0 + r) < (unsigned)o.ny; };
#pragma unroll
  for (int step = 0; step < R + kSkew * K; ++step) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int r = step - kSkew * k;
      if (k == 0 && r < R) {
        s_init_row<R>(o, t, r);
      } else if (k > 0 && r >= k && r < R - k) {
        if (row_in(r)) s_relax_row<R>(o, t, r, k & 1, inv);
      }
    }
    // the pair r0, r0 + 1 once stage K - 1 has passed row r0 + 2
    const int r0 = step - 2 - kSkew * (K - 1);
    if (r0 >= H && r0 < R - H && ((r0 - H) & 1) == 0) {
      float sum = 0.0f;
      if (row_in(r0)) sum += s_resid_pair<R>(o, t, r0);
      if (row_in(r0 + 1)) sum += s_resid_pair<R>(o, t, r0 + 1);
      if (BOUND && !inx) sum = 0.0f;
      const int J = (Y0 + r0) >> 1;
      if (lane_out && J < ncy) rc[(size_t)J * ncx + I] = sum;
    }
  }
}

template <int NU, bool VIN, bool SMALL>
__global__ void __launch_bounds__(64 * kSW)
    k_sdown(SOp o, BIn bin, float *__restrict__ rc) {
  using G = SGeomD<NU, SMALL>;
  constexpr int H = G::H, TY = G::TY, R = G::R;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // Y0 uniform
  const Tile2 tile = xcd_tile();
  const int OX = tile.x * G::TXO, OY = (tile.y * kSW + wave) * TY;
  if (OY >= o.ny) return;
  const int X0 = OX - H, Y0 = OY - H;
  STile<R> t;
  s_load_b<VIN, R>(bin, t.ba, t.bb, X0, Y0, o.nx, o.ny);
  if (s_interior(X0, Y0, R, o.nx, o.ny))
    s_down_rows<false, R, NU, H>(o, t, X0, Y0, rc);
  else
    s_down_rows<true, R, NU, H>(o, t, X0, Y0, rc);
}

// One colour half sweep over rows [M, R-M).  BOUND: the tile reaches past the
// grid, whose outside nodes are kept at zero.
template <bool BOUND, int R, int M>
__device__ __forceinline__ void s_sweep(const SOp &o, STile<R> &t, int X0, int Y0, int color) {
  const int gxa = X0 + 2 * s_lane();
  const bool inx = gxa >= 0 && gxa < o.nx;  // nx even: slot b is inside iff slot a is
#pragma unroll
  for (int r = M; r < R - M; ++r) {
    const int gy = Y0 + r;
    const bool in = !BOUND || (inx && gy >= 0 && gy < o.ny);
    if ((r & 1) == color) {  // slot a has colour r mod 2
      const float v = (t.ba[r] - o.s * t.xa[r - 1] - o.n * t.xa[r + 1] - o.w * s_prev(t.xb[r]) -
                       o.e * t.xb[r]) * o.inv;
      t.xa[r] = in ? v : 0.0f;
    } else {
      const float v = (t.bb[r] - o.s * t.xb[r - 1] - o.n * t.xb[r + 1] - o.w * t.xa[r] -
                       o.e * s_next(t.xa[r])) * o.inv;
      t.xb[r] = in ? v : 0.0f;
    }
  }
}

// Pre-smoothing from x = 0: the first colour-0 half sweep is x = b / d on
// colour 0 (zero on colour 1), then 2 nu - 1 half sweeps.  Afterwards x is
// exact on margin 2 nu - 1.
template <bool BOUND, int R, int NU>
__device__ __forceinline__ void s_pre(const SOp &o, STile<R> &t, int X0, int Y0) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    // b is zero outside the grid, so this x is too
    if ((r & 1) == 0) {
      t.xa[r] = t.ba[r] * o.inv;
      t.xb[r] = 0.0f;
    } else {
      t.xb[r] = t.bb[r] * o.inv;
      t.xa[r] = 0.0f;
    }
  }
  s_sweep<BOUND, R, 1>(o, t, X0, Y0, 1);
  if (NU >= 2) {
    s_sweep<BOUND, R, 2>(o, t, X0, Y0, 0);
    s_sweep<BOUND, R, 3>(o, t, X0, Y0, 1);
  }
  if (NU >= 3) {
    s_sweep<BOUND, R, 4>(o, t, X0, Y0, 0);
    s_sweep<BOUND, R, 5>(o, t, X0, Y0, 1);
  }
}

// Post-smoothing in the reverse colour order (colour 1 first), starting from
// x exact on margin 2 nu - 1.
template <bool BOUND, int R, int NU>
__device__ __forceinline__ void s_post(const SOp &o, STile<R> &t, int X0, int Y0) {
  constexpr int M0 = 2 * NU;
  s_sweep<BOUND, R, M0>(o, t, X0, Y0, 1);
  s_sweep<BOUND, R, M0 + 1>(o, t, X0, Y0, 0);
  if (NU >= 2) {
    s_sweep<BOUND, R, M0 + 2>(o, t, X0, Y0, 1);
    s_sweep<BOUND, R, M0 + 3>(o, t, X0, Y0, 0);
  }
  if (NU >= 3) {
    s_sweep<BOUND, R, M0 + 4>(o, t, X0, Y0, 1);
    s_sweep<BOUND, R, M0 + 5>(o, t, X0, Y0, 0);
  }
}

// cr[q] = coarse correction of this lane's coarse column I = X0/2 + lane in
// coarse row Y0/2 - 1 + q (zero outside the coarse grid).
template <bool BOUND, int R, int NU>
__device__ __forceinline__ void s_up_body(const SOp &o, STile<R> &t, const float (&cr)[R / 2 + 3],
                                          int X0, int Y0) {
  s_pre<BOUND, R, NU>(o, t, X0, Y0);
  // x += P e_c on margin 2 nu - 1: fine column 2I takes 3/4 of coarse column
  // I and 1/4 of I-1, column 2I+1 3/4 of I and 1/4 of I+1, likewise in y;
  // the outermost fine column / row takes pw of its coarse node instead (its
  // second coarse node lies outside the grid, where cr and the neighbour
  // lanes hold zero)
  constexpr int M = 2 * NU - 1;
  const int gxa = X0 + 2 * s_lane();
  const bool inx = gxa >= 0 && gxa < o.nx;
  const float wxa = gxa == 0 ? o.pw : 0.75f;
  const float wxb = gxa + 2 == o.nx ? o.pw : 0.75f;
#pragma unroll
  for (int r = M; r < R - M; ++r) {
    const int gy = Y0 + r;
    const bool in = !BOUND || (inx && gy >= 0 && gy < o.ny);
    const float wy = (gy == 0 || gy == o.ny - 1) ? o.pw : 0.75f;
    const float cj = cr[r / 2 + 1];
    const float cn = cr[(r & 1) ? r / 2 + 2 : r / 2];
    const float ya = wy * cj + 0.25f * cn;                      // own coarse column
    const float yp = wy * s_prev(cj) + 0.25f * s_prev(cn);      // column I-1
    const float yn = wy * s_next(cj) + 0.25f * s_next(cn);      // column I+1
    const float pa = wxa * ya + 0.25f * yp;
    const float pb = wxb * ya + 0.25f * yn;
    t.xa[r] += in ? pa : 0.0f;
    t.xb[r] += in ? pb : 0.0f;
  }
  s_post<BOUND, R, NU>(o, t, X0, Y0);
}

template <int NU, bool VIN, bool SMALL>
__global__ void __launch_bounds__(64 * kSW)
    k_sup(SOp o, BIn bin, const float *__restrict__ ec, float *__restrict__ xout) {
  using G = SGeomU<NU, SMALL>;
  constexpr int H = G::H, TY = G::TY, R = G::R;
  const int wave = threadIdx.x >> 6, lane = s_lane();
  const Tile2 tile = xcd_tile();
  const int OX = tile.x * G::TXO, OY = (tile.y * kSW + wave) * TY;
  if (OY >= o.ny) return;
  const int X0 = OX - H, Y0 = OY - H;
  const int ncx = o.nx / 2, ncy = o.ny / 2;
  STile<R> t;
  s_load_b<VIN, R>(bin, t.ba, t.bb, X0, Y0, o.nx, o.ny);
  float cr[R / 2 + 3];
  {
    const int I = (X0 >> 1) + lane;
#pragma unroll
    for (int q = 0; q < R / 2 + 3; ++q) {
      const int J = (Y0 >> 1) - 1 + q;
      cr[q] = (I >= 0 && I < ncx && J >= 0 && J < ncy) ? ec[(size_t)J * ncx + I] : 0.0f;
    }
  }
  if (s_interior(X0, Y0, R, o.nx, o.ny))
    s_up_body<false, R, NU>(o, t, cr, X0, Y0);
  else
    s_up_body<true, R, NU>(o, t, cr, X0, Y0);
  const int gxa = X0 + 2 * lane;
  if (lane >= H / 2 && lane < 64 - H / 2 && gxa < o.nx) {
#pragma unroll
    for (int r = H; r < R - H; ++r) {
      const int gy = Y0 + r;
      if (gy < o.ny)
        *reinterpret_cast<float2 *>(xout + (size_t)gy * o.nx + gxa) = make_float2(t.xa[r], t.xb[r]);
    }
  }
}

// Block-substitution coupling for stage i (Sec. 4.2) as a streaming pass:
//   b = scale_j v_i - K c,   c = sum_k C[k] z_k,
// K uniform five-point.  The arithmetic is FP64 (z may be FP32) and only b is
// rounded to the V-cycle's precision: for smooth stage vectors K c nearly
// cancels v_i, and forming the difference in FP32 would leave FP32 noise of
// the size of v_i in b, which costs the outer FGMRES iterations.  Each wave covers 124 output
// columns (two halo columns per side for the east/west couplings of c) and
// kCRows rows, with c on kCRows + 2 rows in registers.  Every z, v and b
// element is read or written about once: the pass streams.
constexpr int kCRows = 8;
constexpr int kCTXO = 124;

// Interior five-point coefficients of K in FP64.
struct KOpD {
  int nx, ny;
  double s, w, c, e, n;
};

// The nonzero coupling coefficients of one stage row, compacted on the host:
// c[m] multiplies z_{k[m]}, m < NK.
struct CoupleList {
  double c[kMaxStages];
  int k[kMaxStages];
};

__device__ __forceinline__ double s_next_d(double v) {  // lane + 1 (0 in lane 63)
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), 0x130, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double s_prev_d(double v) {  // lane - 1 (0 in lane 0)
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), 0x138, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Two adjacent elements of a float or double vector.
template <typename T>
struct Pair2;
template <>
struct Pair2<float> {
  using V = float2;
  __device__ static V make(double a, double b) { return make_float2((float)a, (float)b); }
};
template <>
struct Pair2<double> {
  using V = double2;
  __device__ static V make(double a, double b) { return make_double2(a, b); }
};

// T: the type of z and b (float for the FP32 V-cycles, double for the FP64 path).
template <int NK, typename T>
__global__ void __launch_bounds__(64 * kSW)
    k_scouple(KOpD ko, const double *__restrict__ v, const double *__restrict__ scale_j,
              const T *__restrict__ z, CoupleList cl, int i, T *__restrict__ b) {
  using P = Pair2<T>;
  const int wave = threadIdx.x >> 6, lane = s_lane();
  const Tile2 tile = xcd_tile();
  const int OX = tile.x * kCTXO, OY = (tile.y * kSW + wave) * kCRows;
  if (OY >= ko.ny) return;
  const int X0 = OX - 2, gxa = X0 + 2 * lane;
  const size_t N = (size_t)ko.nx * ko.ny;
  const bool inx = gxa >= 0 && gxa < ko.nx;
  const bool out = lane >= 1 && lane < 63 && inx;
  const double sc = *scale_j;
  // v's rows first: their loads are in flight while the z rows arrive
  double2 vr[kCRows];
#pragma unroll
  for (int r = 0; r < kCRows; ++r) {
    const int gy = OY + r;
    vr[r] = make_double2(0.0, 0.0);
    if (inx && gy < ko.ny)
      vr[r] = *reinterpret_cast<const double2 *>(v + (size_t)i * N + (size_t)gy * ko.nx + gxa);
  }
  double ca[kCRows + 2], cb[kCRows + 2];
#pragma unroll
  for (int r = 0; r < kCRows + 2; ++r) {
    const int gy = OY - 1 + r;
    double ax = 0.0, ay = 0.0;
    if (inx && gy >= 0 && gy < ko.ny) {
      const size_t p = (size_t)gy * ko.nx + gxa;
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
  for (int r = 0; r < kCRows; ++r) {
    const int gy = OY + r;
    if (gy >= ko.ny) break;
    const double2 vv = vr[r];
    double va = sc * vv.x, vb = sc * vv.y;
    if (NK > 0) {
      va -= ko.c * ca[r + 1] + ko.s * ca[r] + ko.n * ca[r + 2] + ko.w * s_prev_d(cb[r + 1]) +
            ko.e * cb[r + 1];
      vb -= ko.c * cb[r + 1] + ko.s * cb[r] + ko.n * cb[r + 2] + ko.w * ca[r + 1] +
            ko.e * s_next_d(ca[r + 1]);
    }
    if (out) *reinterpret_cast<typename P::V *>(b + (size_t)gy * ko.nx + gxa) = P::make(va, vb);
  }
}

template <typename G>
dim3 s_grid(int nx, int ny) {
  return dim3((nx + G::TXO - 1) / G::TXO, (ny + G::TY * kSW - 1) / (G::TY * kSW));
}

template <typename G>
bool s_fills(int nx, int ny) {
  const dim3 g = s_grid<G>(nx, ny);
  return g.x * g.y >= 256;
}

template <int NU, bool SMALL>
void sdown_geo(const SOp &o, const BIn &b, float *rc, hipStream_t st) {
  const dim3 g = s_grid<SGeomD<NU, SMALL>>(o.nx, o.ny);
  if (b.v)
    k_sdown<NU, true, SMALL><<<g, 64 * kSW, 0, st>>>(o, b, rc);
  else
    k_sdown<NU, false, SMALL><<<g, 64 * kSW, 0, st>>>(o, b, rc);
}
template <int NU>
void sdown_nu(const SOp &o, const BIn &b, float *rc, hipStream_t st) {
  if (s_fills<SGeomD<NU>>(o.nx, o.ny))
    sdown_geo<NU, false>(o, b, rc, st);
  else
    sdown_geo<NU, true>(o, b, rc, st);
}
template <int NU, bool SMALL>
void sup_geo(const SOp &o, const BIn &b, const float *ec, float *x, hipStream_t st) {
  const dim3 g = s_grid<SGeomU<NU, SMALL>>(o.nx, o.ny);
  if (b.v)
    k_sup<NU, true, SMALL><<<g, 64 * kSW, 0, st>>>(o, b, ec, x);
  else
    k_sup<NU, false, SMALL><<<g, 64 * kSW, 0, st>>>(o, b, ec, x);
}
template <int NU>
void sup_nu(const SOp &o, const BIn &b, const float *ec, float *x, hipStream_t st) {
  if (s_fills<SGeomU<NU>>(o.nx, o.ny))
    sup_geo<NU, false>(o, b, ec, x, st);
  else
    sup_geo<NU, true>(o, b, ec, x, st);
}

template <typename T>
void scouple_launch(const KOpD &ko, const double *v, const double *scale_j, const T *z,
                    const CoupleList &cl, int nk, int i, T *b, hipStream_t st) {
  const dim3 grid((ko.nx + kCTXO - 1) / kCTXO, (ko.ny + kCRows * kSW - 1) / (kCRows * kSW));
#define L_SCOUPLE(NK_) \
  k_scouple<NK_, T><<<grid, 64 * kSW, 0, st>>>(ko, v, scale_j, z, cl, i, b)
  switch (nk) {
    case 0: L_SCOUPLE(0); break;
    case 1: L_SCOUPLE(1); break;
    case 2: L_SCOUPLE(2); break;
    case 3: L_SCOUPLE(3); break;
    case 4: L_SCOUPLE(4); break;
    case 5: L_SCOUPLE(5); break;
    case 6: L_SCOUPLE(6); break;
    default: L_SCOUPLE(7); break;
  }
#undef L_SCOUPLE
}

// The true residual r = 1 (x) f - (I (x) I + hA (x) K) x of the stage system
// for a uniform five-point K and M = I, streamed like the coupling pass: two
// adjacent columns per lane, kRRows output rows per wave, K x_st of every
// stage from its rows in registers (east/west neighbours by DPP), all in
// FP64.  Optionally V0 = r and u_out = u_in + sum_i wts_i x_i (summed in
// stage order from u_in, as the combining pass does).  One block sum of |r|^2
// per workgroup into partial[block].
constexpr int kRRows = 2;  // 4 rows: 116 us (256 VGPRs + AGPRs, one wave per SIMD), 2 rows: 93 us

struct RMat {
  double a[kMaxStages][kMaxStages];  // a[q][st]: hA row q
  double w[kMaxStages];              // state weights h b_i
};

__device__ __forceinline__ double s_block_sum(double v) {
  __shared__ double red[kSW];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < kSW; ++q) r += red[q];
  }
  return r;
}

template <int S>
__global__ void __launch_bounds__(64 * kSW)
    k_resid_split(KOpD ko, const double *__restrict__ x, RMat m, const double *__restrict__ f,
                  double *__restrict__ V0, double *__restrict__ partial,
                  const double *__restrict__ u_in, double *__restrict__ u_out) {
  const int wave = threadIdx.x >> 6, lane = s_lane();
  const Tile2 tile = xcd_tile();
  const int OX = tile.x * kCTXO, OY = (tile.y * kSW + wave) * kRRows;
  double val = 0.0;
  if (OY < ko.ny) {
    const int X0 = OX - 2, gxa = X0 + 2 * lane;
    const size_t N = (size_t)ko.nx * ko.ny;
    const bool inx = gxa >= 0 && gxa < ko.nx;
    const bool out = lane >= 1 && lane < 63 && inx;
    double wa[S][kRRows], wb[S][kRRows], ua[kRRows], ub[kRRows];
#pragma unroll
    for (int r = 0; r < kRRows; ++r) {
      const int gy = OY + r;
      double2 u = make_double2(0.0, 0.0);
      if (u_out && inx && gy < ko.ny)
        u = *reinterpret_cast<const double2 *>(u_in + (size_t)gy * ko.nx + gxa);
      ua[r] = u.x;
      ub[r] = u.y;
#pragma unroll
      for (int q = 0; q < S; ++q) wa[q][r] = wb[q][r] = 0.0;
    }
#pragma unroll
    for (int st = 0; st < S; ++st) {
      const double *xs = x + (size_t)st * N;
      double ra[kRRows + 2], rb[kRRows + 2];
#pragma unroll
      for (int r = 0; r < kRRows + 2; ++r) {
        const int gy = OY - 1 + r;
        double2 v = make_double2(0.0, 0.0);
        if (inx && gy >= 0 && gy < ko.ny)
          v = *reinterpret_cast<const double2 *>(xs + (size_t)gy * ko.nx + gxa);
        ra[r] = v.x;
        rb[r] = v.y;
      }
#pragma unroll
      for (int r = 0; r < kRRows; ++r) {
        const double ka = ko.c * ra[r + 1] + ko.s * ra[r] + ko.n * ra[r + 2] +
                          ko.w * s_prev_d(rb[r + 1]) + ko.e * rb[r + 1];
        const double kb = ko.c * rb[r + 1] + ko.s * rb[r] + ko.n * rb[r + 2] + ko.w * ra[r + 1] +
                          ko.e * s_next_d(ra[r + 1]);
#pragma unroll
        for (int q = 0; q < S; ++q) {
          wa[q][r] += m.a[q][st] * ka;
          wb[q][r] += m.a[q][st] * kb;
        }
        wa[st][r] += ra[r + 1];
        wb[st][r] += rb[r + 1];
        ua[r] += m.w[st] * ra[r + 1];
        ub[r] += m.w[st] * rb[r + 1];
      }
    }
#pragma unroll
    for (int r = 0; r < kRRows; ++r) {
      const int gy = OY + r;
      if (gy >= ko.ny) break;
      const size_t p = (size_t)gy * ko.nx + gxa;
      double2 fv = make_double2(0.0, 0.0);
      if (inx) fv = *reinterpret_cast<const double2 *>(f + p);
#pragma unroll
      for (int q = 0; q < S; ++q) {
        const double resa = fv.x - wa[q][r], resb = fv.y - wb[q][r];
        if (out) {
          val += resa * resa + resb * resb;
          if (V0) *reinterpret_cast<double2 *>(V0 + (size_t)q * N + p) = make_double2(resa, resb);
        }
      }
      if (u_out && out) *reinterpret_cast<double2 *>(u_out + p) = make_double2(ua[r], ub[r]);
    }
  }
  const double t = s_block_sum(val);
  if (threadIdx.x == 0) partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
}

}  // namespace

namespace kern {

int residual_split(int nx, int ny, const double *k_interior, const double *x, const double *hA,
                   int s, const double *f, double *V0, double *partial, hipStream_t st,
                   const double *u_in, const double *wts, double *u_out) {
  RMat m{};
  for (int q = 0; q < s; ++q)
    for (int k = 0; k < s; ++k) m.a[q][k] = hA[(size_t)q * s + k];
  if (u_out)
    for (int k = 0; k < s; ++k) m.w[k] = wts[k];
  const KOpD ko{nx, ny, k_interior[1], k_interior[3], k_interior[4], k_interior[5], k_interior[7]};
  const dim3 grid((nx + kCTXO - 1) / kCTXO, (ny + kRRows * kSW - 1) / (kRRows * kSW));
#define L_RESID(S_)                                                                        \
  k_resid_split<S_><<<grid, 64 * kSW, 0, st>>>(ko, x, m, f, V0, partial, u_in, u_out)
  switch (s) {
    case 1: L_RESID(1); break;
    case 2: L_RESID(2); break;
    case 3: L_RESID(3); break;
    case 4: L_RESID(4); break;
    case 5: L_RESID(5); break;
    case 6: L_RESID(6); break;
    case 7: L_RESID(7); break;
    default: L_RESID(8); break;
  }
#undef L_RESID
  return (int)(grid.x * grid.y);
}

bool wsplit_ok(const OpView<float> &D) {
  return D.npt == 5 && D.uniform && D.cls && D.nx % 2 == 0 && D.ny % 2 == 0;
}

#define IRK_S_NU(FN, ...)                 \
  do {                                    \
    if (nu == 1) FN<1>(__VA_ARGS__);      \
    else if (nu == 2) FN<2>(__VA_ARGS__); \
    else FN<3>(__VA_ARGS__);              \
  } while (0)

void sdown(const OpView<float> &D, const float *interior, int nu, const float *b, float *rc,
           hipStream_t st) {
  IRK_S_NU(sdown_nu, make_sop(D, interior), BIn{b, nullptr, nullptr}, rc, st);
}

void sdown_v(const OpView<float> &D, const float *interior, int nu, const double *v,
             const double *vscale, float *rc, hipStream_t st) {
  IRK_S_NU(sdown_nu, make_sop(D, interior), BIn{nullptr, v, vscale}, rc, st);
}

template <typename T>
void scouple(int nx, int ny, const double *k_interior, const double *v, const double *scale_j,
             const T *z, const double *C, int s, int i, T *b, hipStream_t st) {
  CoupleList cl{};
  int nk = 0;
  for (int k = 0; k < s; ++k)
    if (C[k] != 0.0) {
      cl.c[nk] = C[k];
      cl.k[nk] = k;
      ++nk;
    }
  const KOpD ko{nx, ny, k_interior[1], k_interior[3], k_interior[4], k_interior[5], k_interior[7]};
  scouple_launch<T>(ko, v, scale_j, z, cl, nk, i, b, st);
}
template void scouple<float>(int, int, const double *, const double *, const double *,
                             const float *, const double *, int, int, float *, hipStream_t);
template void scouple<double>(int, int, const double *, const double *, const double *,
                              const double *, const double *, int, int, double *, hipStream_t);

void sup(const OpView<float> &D, const float *interior, int nu, const float *b, const float *ec,
         float *x, hipStream_t st) {
  IRK_S_NU(sup_nu, make_sop(D, interior), BIn{b, nullptr, nullptr}, ec, x, st);
}

void sup_v(const OpView<float> &D, const float *interior, int nu, const double *v,
           const double *vscale, const float *ec, float *x, hipStream_t st) {
  IRK_S_NU(sup_nu, make_sop(D, interior), BIn{nullptr, v, vscale}, ec, x, st);
}

}  // namespace kern
}  // namespace irk
