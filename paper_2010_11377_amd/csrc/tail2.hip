// The coarse tail of the FP32 V-cycle in one workgroup, rows in registers.
//
// Levels of the tail are at most 64 x 64.  Two layouts:
//
// * workgroup levels (wider or taller than 16): each lane holds two adjacent
//   grid columns 2i, 2i+1 of four consecutive rows, a unit of 32 lanes (16
//   for levels at most 32 wide) covers a row segment, and the units of the
//   eight waves stack the rows.  In a red-black half sweep every lane then
//   updates exactly one node per row (no lane computes a node of the other
//   colour), east/west neighbours come from the adjacent lane through DPP,
//   and the 2 x 2 cells of the restriction are lane-local.  Each unit
//   publishes its first and last row in LDS after every half sweep, double
//   buffered, so one barrier per half sweep suffices;
// * wave levels (at most 16 x 16) above a dense coarsest level of at most 64
//   unknowns run in wave 0 alone: one column per lane, 16 lanes per row of
//   columns, four row groups of up to four rows each, the same publish/read
//   scheme with wave-scope ordering instead of workgroup barriers.  The other
//   waves meanwhile copy the coarsest inverse into LDS and wait at one
//   barrier.
//
// The relaxation is Jacobi within a colour (all updates of a half sweep read
// old values), which for five-point operators is Gauss-Seidel.
//
// During the descent the pre-smoothed x of every level (and b below the top
// level) is parked in LDS and picked up again on the way back.  Coarse
// right-hand sides and the coarse x handed up a level go through LDS areas of
// their own (the level array and two alternating hand-over areas), so no
// barrier is spent on freeing shared space.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace irk {
namespace {

constexpr int kT2Threads = 512;
constexpr int kT2Waves = kT2Threads / 64;
constexpr int kT2Rows = 4;     // rows per unit
constexpr int kT2A = 4096;     // exchange area (floats)
constexpr int kT2R = 64 * 64;  // level array
// Offsets inside the level array of areas used while it holds at most a
// 32 x 32 level: the wave layout's exchange slots (256 floats), the coarsest
// right-hand side (64) and the two hand-over areas (1024 each).
constexpr int kT2SEx = 1024, kT2Bc = 1536, kT2X0 = 2048, kT2X1 = 3072;
constexpr int kT2SUnits = 4, kT2SCols = 16;
constexpr int kT2SSide = 16;    // wave levels: at most 16 x 16
constexpr int kT2SCoarse = 64;  // dense coarsest level solved by one wave
constexpr int kT2CiPer =        // inverse entries copied per thread of waves 1..7
    (kT2SCoarse * kT2SCoarse + kT2Threads - 64 - 1) / (kT2Threads - 64);
// Class tables in LDS: 9 classes per level, each padded to 12 floats so that a
// node's nine coefficients are three 16-byte reads.
constexpr int kT2ClsPad = 12, kT2ClsLevel = 9 * kT2ClsPad;

// The nine coefficients of class q from a padded table.
__device__ __forceinline__ void class_coefs(const float *tab, int q, float *c) {
  const float4 *p = reinterpret_cast<const float4 *>(tab + q * kT2ClsPad);
  const float4 v0 = p[0], v1 = p[1], v2 = p[2];
  c[0] = v0.x; c[1] = v0.y; c[2] = v0.z; c[3] = v0.w;
  c[4] = v1.x; c[5] = v1.y; c[6] = v1.z; c[7] = v1.w;
  c[8] = v2.x;
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Orders the LDS accesses of one wave (its LDS instructions execute in order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int t2_cls(int i, int j, int nx, int ny) {
  const int cx = (i == 0) ? 0 : (i == nx - 1 ? 2 : 1);
  const int cy = (j == 0) ? 0 : (j == ny - 1 ? 2 : 1);
  return 3 * cy + cx;
}

struct T2Desc {
  int nlev;
  int ls;  // first level run by wave 0 alone (nlev: none)
  int nx[kTailLevels], ny[kTailLevels];
  const float *cls[kTailLevels];
  const float *arr[kTailLevels];
  float pw[kTailLevels];
  float pa, pn;  // prolongation weights from the own and the next coarse node
  const float *CinvT;  // null: the coarsest level returns x = 0
  int store_off[kTailLevels];  // LDS offset of level l's parked x (and b for l > 0)
};

// ===========================================================================
// workgroup levels: two columns per lane
// ===========================================================================

// Units of CW lanes; lane i of a unit holds columns 2i, 2i+1 of rows
// r0 .. r0 + nr - 1 (r0 = 4 u is even, so a row's colour pattern is fixed).
template <int CW>
struct Pair {
  static constexpr int upw = 64 / CW;           // units per wave
  static constexpr int units = kT2Waves * upw;  // units of the workgroup
};

struct PShare {
  int nx, ny, r0, nr, i, u;
  bool col;  // the lane holds grid columns
};

template <int CW>
__device__ __forceinline__ PShare pshare(int nx, int ny) {
  PShare s;
  s.u = (threadIdx.x >> 6) * Pair<CW>::upw + (threadIdx.x & 63) / CW;
  s.i = threadIdx.x & (CW - 1);
  s.nx = nx;
  s.ny = ny;
  s.r0 = kT2Rows * s.u;
  s.nr = max(0, min(kT2Rows, ny - s.r0));
  s.col = 2 * s.i < nx;
  return s;
}

// Value of the lane holding the previous / next column pair (0 past the
// unit's ends).  16-lane units use row shifts (zero at row ends); 32-lane
// units use wave shifts and clear the lanes at the unit's ends.
template <int CW>
__device__ __forceinline__ float p_prev(float v, int i) {
  if (CW == 16) return dpp<0x111>(v);
  const float w = dpp<0x138>(v);
  return i == 0 ? 0.0f : w;
}
template <int CW>
__device__ __forceinline__ float p_next(float v, int i) {
  if (CW == 16) return dpp<0x101>(v);
  const float w = dpp<0x130>(v);
  return i == CW - 1 ? 0.0f : w;
}

template <int CW>
__device__ __forceinline__ float2 *pslot(float *ex, int buf, int u, int side) {
  return reinterpret_cast<float2 *>(ex + ((buf * Pair<CW>::units + u) * 2 + side) * (2 * CW));
}

// Coefficients of the lane's eight nodes (9 each) and 1 / centre.
struct PCo {
  float a[kT2Rows][9], b[kT2Rows][9];
  float ia[kT2Rows], ib[kT2Rows];
};

template <bool CLS>
__device__ __forceinline__ void pload_co(const PShare &s, const float *cls_lds, const float *arr,
                                         PCo &co) {
  const size_t N = (size_t)s.nx * s.ny;
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) {
    const int j = s.r0 + t, ca = 2 * s.i, cb = 2 * s.i + 1;
    const bool ok = t < s.nr && s.col;
    if (CLS) {
      // the classes are read for every lane (valid table rows), then masked
      class_coefs(cls_lds, t2_cls(ca, j, s.nx, s.ny), co.a[t]);
      class_coefs(cls_lds, t2_cls(cb, j, s.nx, s.ny), co.b[t]);
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        co.a[t][k] = ok ? co.a[t][k] : 0.0f;
        co.b[t][k] = ok ? co.b[t][k] : 0.0f;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        float va = 0.0f, vb = 0.0f;
        if (ok) {
          va = arr[(size_t)k * N + (size_t)j * s.nx + ca];
          vb = arr[(size_t)k * N + (size_t)j * s.nx + cb];
        }
        co.a[t][k] = va;
        co.b[t][k] = vb;
      }
    }
    co.ia[t] = ok ? 1.0f / co.a[t][4] : 0.0f;
    co.ib[t] = ok ? 1.0f / co.b[t][4] : 0.0f;
  }
}

template <int CW>
__device__ __forceinline__ void ppublish(const PShare &s, const float (&xa)[kT2Rows],
                                         const float (&xb)[kT2Rows], float *ex, int buf) {
  if (s.nr == 0) return;
  float la = xa[0], lb = xb[0];
#pragma unroll
  for (int t = 1; t < kT2Rows; ++t)
    if (t == s.nr - 1) {
      la = xa[t];
      lb = xb[t];
    }
  pslot<CW>(ex, buf, s.u, 0)[s.i] = make_float2(xa[0], xb[0]);
  pslot<CW>(ex, buf, s.u, 1)[s.i] = make_float2(la, lb);
}

// Rows above (u*) and below (d*) each of the unit's rows: own registers
// inside the block, the neighbouring units' published rows at its ends
// (read unconditionally from clamped slots; zero outside the grid).
template <int CW>
__device__ __forceinline__ void pneigh(const PShare &s, const float (&xa)[kT2Rows],
                                       const float (&xb)[kT2Rows], float *ex, int buf,
                                       float (&ua)[kT2Rows], float (&ub)[kT2Rows],
                                       float (&da)[kT2Rows], float (&db)[kT2Rows]) {
  const int uu = max(s.u - 1, 0), ud = min(s.u + 1, Pair<CW>::units - 1);
  const float2 t2 = pslot<CW>(ex, buf, uu, 1)[s.i], b2 = pslot<CW>(ex, buf, ud, 0)[s.i];
  const bool ht = s.r0 > 0 && s.col, hb = s.r0 + s.nr < s.ny && s.col;
  const float ta = ht ? t2.x : 0.0f, tb = ht ? t2.y : 0.0f;
  const float ba = hb ? b2.x : 0.0f, bb = hb ? b2.y : 0.0f;
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) {
    ua[t] = (t == 0) ? ta : xa[t > 0 ? t - 1 : 0];
    ub[t] = (t == 0) ? tb : xb[t > 0 ? t - 1 : 0];
    const bool in = t + 1 < kT2Rows && t + 1 < s.nr;
    da[t] = in ? xa[t + 1 < kT2Rows ? t + 1 : t] : ba;
    db[t] = in ? xb[t + 1 < kT2Rows ? t + 1 : t] : bb;
  }
}

// Off-centre part of the stencil at column 2i (node a) and at column 2i+1
// (node b) of a row, from the rows above (ua, ub), the row itself (ma, mb)
// and below (da, db); summed as a tree of pairs.
template <int CW>
__device__ __forceinline__ float sum_a(const float *c, float ua, float ub, float ma, float mb,
                                       float da, float db, int i) {
  const float s0 = c[0] * p_prev<CW>(ub, i) + c[1] * ua;
  const float s1 = c[2] * ub + c[3] * p_prev<CW>(mb, i);
  const float s2 = c[5] * mb + c[6] * p_prev<CW>(db, i);
  const float s3 = c[7] * da + c[8] * db;
  return (s0 + s1) + (s2 + s3);
}
template <int CW>
__device__ __forceinline__ float sum_b(const float *c, float ua, float ub, float ma, float mb,
                                       float da, float db, int i) {
  const float s0 = c[0] * ua + c[1] * ub;
  const float s1 = c[2] * p_next<CW>(ua, i) + c[3] * ma;
  const float s2 = c[5] * p_next<CW>(ma, i) + c[6] * da;
  const float s3 = c[7] * db + c[8] * p_next<CW>(da, i);
  return (s0 + s1) + (s2 + s3);
}

// One colour half sweep reading the rows published in buffer rb, then
// publishing into rb ^ 1 (and the whole level into `full` when given) and
// waiting for the workgroup.  In row t (parity t) node a has colour t & 1.
template <int CW>
__device__ __forceinline__ void phalf(const PShare &s, const PCo &co, float (&xa)[kT2Rows],
                                      float (&xb)[kT2Rows], const float (&ba)[kT2Rows],
                                      const float (&bb)[kT2Rows], float *ex, int rb, int color,
                                      float *full) {
  float ua[kT2Rows], ub[kT2Rows], da[kT2Rows], db[kT2Rows];
  pneigh<CW>(s, xa, xb, ex, rb, ua, ub, da, db);
  float na[kT2Rows], nb[kT2Rows];
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) {
    na[t] = xa[t];
    nb[t] = xb[t];
    if (t < s.nr) {
      if ((t & 1) == color)
        na[t] = (ba[t] - sum_a<CW>(co.a[t], ua[t], ub[t], xa[t], xb[t], da[t], db[t], s.i)) *
                co.ia[t];
      else
        nb[t] = (bb[t] - sum_b<CW>(co.b[t], ua[t], ub[t], xa[t], xb[t], da[t], db[t], s.i)) *
                co.ib[t];
    }
  }
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) {
    xa[t] = na[t];
    xb[t] = nb[t];
  }
  ppublish<CW>(s, xa, xb, ex, rb ^ 1);
  if (full) {
#pragma unroll
    for (int t = 0; t < kT2Rows; ++t)
      if (t < s.nr && s.col)
        *reinterpret_cast<float2 *>(full + (s.r0 + t) * s.nx + 2 * s.i) = make_float2(xa[t], xb[t]);
  }
  __syncthreads();
}

// b of a level in the pair layout from a row-major array (global or LDS).
template <int CW>
__device__ __forceinline__ void pload_b(const PShare &s, const float *src, float (&ba)[kT2Rows],
                                        float (&bb)[kT2Rows]) {
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) {
    float2 v = make_float2(0.0f, 0.0f);
    if (t < s.nr && s.col)
      v = *reinterpret_cast<const float2 *>(src + (size_t)(s.r0 + t) * s.nx + 2 * s.i);
    ba[t] = v.x;
    bb[t] = v.y;
  }
}

// Pre-smoothing of level l from x = 0 with b read from bsrc (or given in
// b_in when have_b); the coarse right-hand side (sums of the residual over
// 2 x 2 cells) goes to R in row-major order, x (and b) are parked.
template <int CW, bool CLS>
__device__ __forceinline__ void pdescend(const T2Desc &td, int l, const float *bsrc, bool have_b,
                                         const float (&ba_in)[kT2Rows],
                                         const float (&bb_in)[kT2Rows], float *ex, float *R,
                                         float *store, const float *cls_lds, int nu) {
  const PShare s = pshare<CW>(td.nx[l], td.ny[l]);
  float ba[kT2Rows], bb[kT2Rows];
  if (have_b) {
#pragma unroll
    for (int t = 0; t < kT2Rows; ++t) {
      ba[t] = ba_in[t];
      bb[t] = bb_in[t];
    }
  } else {
    pload_b<CW>(s, bsrc, ba, bb);
  }
  PCo co;
  pload_co<CLS>(s, cls_lds + kT2ClsLevel * l, td.arr[l], co);
  float xa[kT2Rows], xb[kT2Rows];
  // x = 0, then colour 0 takes b / d: node a in even rows, node b in odd rows
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) {
    xa[t] = (t & 1) == 0 ? ba[t] * co.ia[t] : 0.0f;
    xb[t] = (t & 1) == 1 ? bb[t] * co.ib[t] : 0.0f;
  }
  ppublish<CW>(s, xa, xb, ex, 0);
  __syncthreads();
  int buf = 0;
  for (int h = 1; h < 2 * nu; ++h) {
    phalf<CW>(s, co, xa, xb, ba, bb, ex, buf, h & 1, nullptr);
    buf ^= 1;
  }
  float ua[kT2Rows], ub[kT2Rows], da[kT2Rows], db[kT2Rows];
  pneigh<CW>(s, xa, xb, ex, buf, ua, ub, da, db);
  float ra[kT2Rows], rb[kT2Rows];
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) {
    ra[t] = ba[t] - (sum_a<CW>(co.a[t], ua[t], ub[t], xa[t], xb[t], da[t], db[t], s.i) +
                     co.a[t][4] * xa[t]);
    rb[t] = bb[t] - (sum_b<CW>(co.b[t], ua[t], ub[t], xa[t], xb[t], da[t], db[t], s.i) +
                     co.b[t][4] * xb[t]);
  }
  float *px = store + td.store_off[l];
  float *pb = px + s.nx * s.ny;
  const int ncx = s.nx / 2;
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t)
    if (t < s.nr && s.col) {
      const int p = (s.r0 + t) * s.nx + 2 * s.i;
      *reinterpret_cast<float2 *>(px + p) = make_float2(xa[t], xb[t]);
      if (l > 0) *reinterpret_cast<float2 *>(pb + p) = make_float2(ba[t], bb[t]);
      if (t & 1)
        R[((s.r0 + t) >> 1) * ncx + s.i] =
            (ra[t > 0 ? t - 1 : 0] + rb[t > 0 ? t - 1 : 0]) + (ra[t] + rb[t]);
    }
  __syncthreads();
}

// Coarse correction of level l from the coarse x in xc, then post-smoothing;
// the result goes to xo (l > 0) or to x_top (l == 0).
template <int CW, bool CLS>
__device__ __forceinline__ void pascend(const T2Desc &td, int l, const float *xc, float *xo,
                                        const float *b_top, float *x_top, float *ex,
                                        const float *store, const float *cls_lds, int nu) {
  const PShare s = pshare<CW>(td.nx[l], td.ny[l]);
  const int ncx = td.nx[l + 1], ncy = td.ny[l + 1];
  const float pw = td.pw[l], pa = td.pa, pn = td.pn;
  const float *px = store + td.store_off[l];
  float xa[kT2Rows], xb[kT2Rows], ba[kT2Rows], bb[kT2Rows];
  pload_b<CW>(s, l > 0 ? px + s.nx * s.ny : b_top, ba, bb);
  // x = parked x + P x_c; both nodes of the lane lie in coarse column i
  const int I = s.col ? s.i : 0;
  const bool hxa = I - 1 >= 0, hxb = I + 1 < ncx;
  const int nxa = hxa ? I - 1 : I, nxb = hxb ? I + 1 : I;
  const float wxa = hxa ? pa : pw, wxb = hxb ? pa : pw;
  const float axa = hxa ? pn : 0.0f, axb = hxb ? pn : 0.0f;
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) {
    const bool ok = t < s.nr && s.col;
    const int fy = ok ? s.r0 + t : 0;
    const int Iy = fy >> 1, nby = (t & 1) ? Iy + 1 : Iy - 1;
    const bool hy = nby >= 0 && nby < ncy;
    const int nbyc = hy ? nby : Iy;
    const float wy = hy ? pa : pw, ay = hy ? pn : 0.0f;
    const float c00 = xc[Iy * ncx + I], c0a = xc[Iy * ncx + nxa], c0b = xc[Iy * ncx + nxb];
    const float c10 = xc[nbyc * ncx + I], c1a = xc[nbyc * ncx + nxa], c1b = xc[nbyc * ncx + nxb];
    const float va = (wxa * wy * c00 + axa * wy * c0a) + (wxa * ay * c10 + axa * ay * c1a);
    const float vb = (wxb * wy * c00 + axb * wy * c0b) + (wxb * ay * c10 + axb * ay * c1b);
    const float2 p = ok ? *reinterpret_cast<const float2 *>(px + fy * s.nx + 2 * s.i)
                        : make_float2(0.0f, 0.0f);
    xa[t] = ok ? p.x + va : 0.0f;
    xb[t] = ok ? p.y + vb : 0.0f;
  }
  PCo co;
  pload_co<CLS>(s, cls_lds + kT2ClsLevel * l, td.arr[l], co);
  ppublish<CW>(s, xa, xb, ex, 0);
  __syncthreads();
  int buf = 0;
  for (int h = 0; h < 2 * nu; ++h) {  // colour 1 first
    phalf<CW>(s, co, xa, xb, ba, bb, ex, buf, (h & 1) ^ 1,
              (h == 2 * nu - 1 && l > 0) ? xo : nullptr);
    buf ^= 1;
  }
  if (l == 0) {
#pragma unroll
    for (int t = 0; t < kT2Rows; ++t)
      if (t < s.nr && s.col)
        *reinterpret_cast<float2 *>(x_top + (size_t)(s.r0 + t) * s.nx + 2 * s.i) =
            make_float2(xa[t], xb[t]);
  }
}

// ===========================================================================
// wave levels: one column per lane, wave 0 alone
// ===========================================================================

// Lane i of row group g (16 lanes each) holds column i of rows r0 .. r0 + nr - 1.
struct WShare {
  int nx, ny, r0, nr, i, g;
  bool col;
};

__device__ __forceinline__ WShare wshare(int nx, int ny) {
  WShare s;
  const int rpg = (ny + kT2SUnits - 1) / kT2SUnits;
  s.g = (threadIdx.x & 63) >> 4;
  s.nx = nx;
  s.ny = ny;
  s.r0 = s.g * rpg;
  s.nr = max(0, min(rpg, ny - s.r0));
  s.i = threadIdx.x & 15;
  s.col = s.i < nx;
  return s;
}

__device__ __forceinline__ float w_next(float v) { return dpp<0x101>(v); }  // lane + 1 in the row
__device__ __forceinline__ float w_prev(float v) { return dpp<0x111>(v); }  // lane - 1 in the row

__device__ __forceinline__ float *wslot(float *ex, int buf, int g, int side) {
  return ex + ((buf * kT2SUnits + g) * 2 + side) * kT2SCols;
}

struct WCo {
  float c[kT2Rows][9];
  float inv[kT2Rows];
};

template <bool CLS>
__device__ __forceinline__ void wload_co(const WShare &s, const float *cls_lds, const float *arr,
                                         WCo &co) {
  const size_t N = (size_t)s.nx * s.ny;
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) {
    const int j = s.r0 + t;
    const bool ok = t < s.nr && s.col;
    if (CLS) {
      class_coefs(cls_lds, t2_cls(s.i, j, s.nx, s.ny), co.c[t]);
#pragma unroll
      for (int k = 0; k < 9; ++k) co.c[t][k] = ok ? co.c[t][k] : 0.0f;
    } else {
#pragma unroll
      for (int k = 0; k < 9; ++k)
        co.c[t][k] = ok ? arr[(size_t)k * N + (size_t)j * s.nx + s.i] : 0.0f;
    }
    co.inv[t] = ok ? 1.0f / co.c[t][4] : 0.0f;
  }
}

__device__ __forceinline__ void wneigh(const WShare &s, const float (&x)[kT2Rows], float *ex,
                                       int buf, float (&up)[kT2Rows], float (&dn)[kT2Rows]) {
  const int gu = max(s.g - 1, 0), gd = min(s.g + 1, kT2SUnits - 1);
  const float ta = wslot(ex, buf, gu, 1)[s.i], tb = wslot(ex, buf, gd, 0)[s.i];
  const float top = (s.r0 > 0 && s.col) ? ta : 0.0f;
  const float bot = (s.r0 + s.nr < s.ny && s.col) ? tb : 0.0f;
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) {
    up[t] = (t == 0) ? top : x[t > 0 ? t - 1 : 0];
    dn[t] = (t + 1 < kT2Rows && t + 1 < s.nr) ? x[t + 1 < kT2Rows ? t + 1 : t] : bot;
  }
}

template <bool CENTRE>
__device__ __forceinline__ float wsum(const float *a, float up, float mid, float dn) {
  const float s0 = a[0] * w_prev(up) + a[1] * up;
  const float s1 = a[2] * w_next(up) + a[3] * w_prev(mid);
  const float s2 = a[5] * w_next(mid) + a[6] * w_prev(dn);
  const float s3 = a[7] * dn + a[8] * w_next(dn);
  float acc = (s0 + s1) + (s2 + s3);
  if (CENTRE) acc += a[4] * mid;
  return acc;
}

__device__ __forceinline__ void wpublish(const WShare &s, const float (&x)[kT2Rows], float *ex,
                                         int buf) {
  if (s.nr == 0) return;
  float last = x[0];
#pragma unroll
  for (int t = 1; t < kT2Rows; ++t)
    if (t == s.nr - 1) last = x[t];
  wslot(ex, buf, s.g, 0)[s.i] = x[0];
  wslot(ex, buf, s.g, 1)[s.i] = last;
}

__device__ __forceinline__ void whalf(const WShare &s, const WCo &co, float (&x)[kT2Rows],
                                      const float (&b)[kT2Rows], float *ex, int rb, int color,
                                      float *full) {
  float up[kT2Rows], dn[kT2Rows], nv[kT2Rows];
  wneigh(s, x, ex, rb, up, dn);
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) {
    nv[t] = x[t];
    if (t < s.nr) {
      const float v = (b[t] - wsum<false>(co.c[t], up[t], x[t], dn[t])) * co.inv[t];
      // m v + (1 - m) x with m in {0, 1}: exact, and computed on every lane
      const float m = (s.col && ((s.i + s.r0 + t) & 1) == color) ? 1.0f : 0.0f;
      nv[t] = m * v + (1.0f - m) * x[t];
    }
  }
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) x[t] = nv[t];
  wpublish(s, x, ex, rb ^ 1);
  if (full) {
#pragma unroll
    for (int t = 0; t < kT2Rows; ++t)
      if (t < s.nr && s.col) full[(s.r0 + t) * s.nx + s.i] = x[t];
  }
  wave_sync();
}

__device__ __forceinline__ void wload_b(const WShare &s, const float *src, float (&b)[kT2Rows]) {
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t)
    b[t] = (t < s.nr && s.col) ? src[(size_t)(s.r0 + t) * s.nx + s.i] : 0.0f;
}

// Pre-smoothing of wave level l from x = 0 (b given); the coarse
// right-hand side replaces b (registers, the next wave level's layout).
template <bool CLS>
__device__ __forceinline__ void wdescend(const T2Desc &td, int l, float (&b)[kT2Rows], float *ex,
                                         float *R, float *store, const float *cls_lds, int nu) {
  const WShare s = wshare(td.nx[l], td.ny[l]);
  WCo co;
  wload_co<CLS>(s, cls_lds + kT2ClsLevel * l, td.arr[l], co);
  float x[kT2Rows];
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t)
    x[t] = (t < s.nr && s.col && ((s.i + s.r0 + t) & 1) == 0) ? b[t] * co.inv[t] : 0.0f;
  wpublish(s, x, ex, 0);
  wave_sync();
  int buf = 0;
  for (int h = 1; h < 2 * nu; ++h) {
    whalf(s, co, x, b, ex, buf, h & 1, nullptr);
    buf ^= 1;
  }
  float *px = store + td.store_off[l];
  float *pb = px + s.nx * s.ny;
  float up[kT2Rows], dn[kT2Rows];
  wneigh(s, x, ex, buf, up, dn);
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) {
    const float r = b[t] - wsum<true>(co.c[t], up[t], x[t], dn[t]);
    if (t < s.nr && s.col) {
      const int p = (s.r0 + t) * s.nx + s.i;
      px[p] = x[t];
      if (l > 0) pb[p] = b[t];
      R[p] = r;
    }
  }
  wave_sync();
  // restriction: sums over the 2 x 2 cells, into the next level's layout
  const WShare c = wshare(td.nx[l + 1], td.ny[l + 1]);
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) {
    float v = 0.0f;
    if (t < c.nr && c.col) {
      const int J = c.r0 + t, I = c.i;
      const float *row0 = R + (2 * J) * s.nx, *row1 = row0 + s.nx;
      v = row0[2 * I] + row0[2 * I + 1] + row1[2 * I] + row1[2 * I + 1];
    }
    b[t] = v;
  }
}

template <bool CLS>
__device__ __forceinline__ void wascend(const T2Desc &td, int l, const float *xc, float *xo,
                                        const float *b_top, float *x_top, float *ex,
                                        const float *store, const float *cls_lds, int nu) {
  const WShare s = wshare(td.nx[l], td.ny[l]);
  const int ncx = td.nx[l + 1], ncy = td.ny[l + 1];
  const float pw = td.pw[l], pa = td.pa, pn = td.pn;
  const float *px = store + td.store_off[l];
  const float *pb = px + s.nx * s.ny;
  float x[kT2Rows], b[kT2Rows];
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) {
    const bool ok = t < s.nr && s.col;
    const int fx = ok ? s.i : 0, fy = ok ? s.r0 + t : 0, p = fy * s.nx + fx;
    const int Ix = fx >> 1, Iy = fy >> 1;
    const int nbx = (fx & 1) ? Ix + 1 : Ix - 1, nby = (fy & 1) ? Iy + 1 : Iy - 1;
    const bool hx = nbx >= 0 && nbx < ncx, hy = nby >= 0 && nby < ncy;
    const int nbxc = hx ? nbx : Ix, nbyc = hy ? nby : Iy;
    const float wx = hx ? pa : pw, wy = hy ? pa : pw;
    const float ax = hx ? pn : 0.0f, ay = hy ? pn : 0.0f;
    const float cv = (wx * wy * xc[Iy * ncx + Ix] + ax * wy * xc[Iy * ncx + nbxc]) +
                     (wx * ay * xc[nbyc * ncx + Ix] + ax * ay * xc[nbyc * ncx + nbxc]);
    const float pv = px[p];
    float bv = 0.0f;
    if (ok) bv = (l > 0) ? pb[p] : b_top[p];
    x[t] = ok ? pv + cv : 0.0f;
    b[t] = bv;
  }
  WCo co;
  wload_co<CLS>(s, cls_lds + kT2ClsLevel * l, td.arr[l], co);
  wpublish(s, x, ex, 0);
  wave_sync();
  int buf = 0;
  for (int h = 0; h < 2 * nu; ++h) {  // colour 1 first
    whalf(s, co, x, b, ex, buf, (h & 1) ^ 1, (h == 2 * nu - 1 && l > 0) ? xo : nullptr);
    buf ^= 1;
  }
  if (l == 0) {
#pragma unroll
    for (int t = 0; t < kT2Rows; ++t)
      if (t < s.nr && s.col) x_top[(size_t)(s.r0 + t) * s.nx + s.i] = x[t];
  }
}

// ===========================================================================

template <bool CLS>
__device__ __forceinline__ void descend_pair(const T2Desc &td, int l, const float *bsrc,
                                             bool have_b, const float (&ba)[kT2Rows],
                                             const float (&bb)[kT2Rows], float *A, float *R,
                                             float *store, const float *cls_lds, int nu) {
  if (td.nx[l] <= 32)
    pdescend<16, CLS>(td, l, bsrc, have_b, ba, bb, A, R, store, cls_lds, nu);
  else
    pdescend<32, CLS>(td, l, bsrc, have_b, ba, bb, A, R, store, cls_lds, nu);
}

template <bool CLS>
__device__ __forceinline__ void ascend_pair(const T2Desc &td, int l, const float *xc, float *xo,
                                            const float *b_top, float *x_top, float *A,
                                            const float *store, const float *cls_lds, int nu) {
  if (td.nx[l] <= 32)
    pascend<16, CLS>(td, l, xc, xo, b_top, x_top, A, store, cls_lds, nu);
  else
    pascend<32, CLS>(td, l, xc, xo, b_top, x_top, A, store, cls_lds, nu);
}

template <bool CLS>
__global__ void __launch_bounds__(kT2Threads)
    k_vtail2(T2Desc td, const float *__restrict__ b_top, float *__restrict__ x_top, int nu) {
  extern __shared__ float sm[];
  float *A = sm;            // workgroup exchange buffers; coarsest inverse or its scratch
  float *R = sm + kT2A;     // coarse right-hand sides and the areas placed at kT2SEx ...
  float *store = R + kT2R;  // parked x, b
  float *cls_lds = store + td.store_off[td.nlev - 1];  // padded class tables per level
  const int L = td.nlev, ls = td.ls;
  const bool wave_tail = ls < L;
  const int wave = threadIdx.x >> 6;
  const int lm = min(ls, L - 1);
  // level 0's right-hand side is read from global memory while the class
  // tables travel to LDS (the two load latencies overlap)
  float ba0[kT2Rows], bb0[kT2Rows];
  if (lm > 0) {
    if (td.nx[0] <= 32)
      pload_b<16>(pshare<16>(td.nx[0], td.ny[0]), b_top, ba0, bb0);
    else
      pload_b<32>(pshare<32>(td.nx[0], td.ny[0]), b_top, ba0, bb0);
  }
  if (CLS)
    for (int q = threadIdx.x; q < 81 * (L - 1); q += kT2Threads)
      cls_lds[(q / 81) * kT2ClsLevel + ((q % 81) / 9) * kT2ClsPad + q % 9] = td.cls[q / 81][q % 81];
  __syncthreads();

  // ---- descent through the workgroup levels: level l takes b from the top
  // right-hand side (level 0, already in registers) or from R, and leaves
  // the coarse b in R
  for (int l = 0; l < lm; ++l) descend_pair<CLS>(td, l, R, l == 0, ba0, bb0, A, R, store, cls_lds, nu);

  const int nc = td.nx[L - 1] * td.ny[L - 1];
  int cur = 0;  // hand-over area holding the x of the level below the next one up
  if (wave_tail) {
    if (wave == 0) {
      float b[kT2Rows];
      wload_b(wshare(td.nx[ls], td.ny[ls]), ls == 0 ? b_top : R, b);
      for (int l = ls; l + 1 < L; ++l) wdescend<CLS>(td, l, b, R + kT2SEx, R, store, cls_lds, nu);
      // the coarsest right-hand side, row-major at kT2Bc
      const WShare c = wshare(td.nx[L - 1], td.ny[L - 1]);
      float *bc = R + kT2Bc;
#pragma unroll
      for (int t = 0; t < kT2Rows; ++t)
        if (t < c.nr && c.col) bc[(c.r0 + t) * c.nx + c.i] = b[t];
    } else {
      float v[kT2CiPer];
      const int q0 = threadIdx.x - 64;
#pragma unroll
      for (int k = 0; k < kT2CiPer; ++k) {
        const int q = q0 + k * (kT2Threads - 64);
        v[k] = q < nc * nc && td.CinvT ? td.CinvT[q] : 0.0f;
      }
#pragma unroll
      for (int k = 0; k < kT2CiPer; ++k) {
        const int q = q0 + k * (kT2Threads - 64);
        if (q < nc * nc) A[q] = v[k];
      }
    }
    __syncthreads();
    if (wave == 0) {
      // coarsest: x = C^-1 b with C^-1 stored transposed, one row per lane
      const float *bc = R + kT2Bc;
      const int row = threadIdx.x;
      if (row < nc) {
        float acc = 0.0f;
        if (td.CinvT)
          for (int col = 0; col < nc; ++col) acc += A[col * nc + row] * bc[col];
        if (L == 1)
          x_top[row] = acc;
        else
          R[kT2X0 + row] = acc;
      }
      wave_sync();
      int k = 0;
      for (int l = L - 2; l >= ls; --l, k ^= 1)
        wascend<CLS>(td, l, R + (k ? kT2X1 : kT2X0), R + (k ? kT2X0 : kT2X1), b_top, x_top,
                     R + kT2SEx, store, cls_lds, nu);
    }
    __syncthreads();
    if (ls == 0) return;
    cur = (L - 1 - ls) & 1;
  } else {
    // coarsest by the whole workgroup: its b is the top b (one level) or in R
    const float *bc = R;
    if (L == 1) {
      for (int q = threadIdx.x; q < nc; q += kT2Threads) A[q] = b_top[q];
      __syncthreads();
      bc = A;
    }
    float *red = A + 2048;
    const int nb = max(1, kT2Threads / nc);  // column blocks; nc <= kTailMaxCoarse
    for (int q = threadIdx.x; q < nb * nc; q += kT2Threads) {
      const int row = q % nc, cb = q / nc;
      float acc = 0.0f;
      if (td.CinvT)
        for (int col = cb; col < nc; col += nb) acc += td.CinvT[(size_t)col * nc + row] * bc[col];
      red[q] = acc;
    }
    __syncthreads();
    for (int row = threadIdx.x; row < nc; row += kT2Threads) {
      float acc = 0.0f;
      for (int cb = 0; cb < nb; ++cb) acc += red[cb * nc + row];
      if (L == 1)
        x_top[row] = acc;
      else
        R[kT2X0 + row] = acc;
    }
    __syncthreads();
    if (L == 1) return;
  }

  // ---- ascent through the workgroup levels
  for (int l = lm - 1; l >= 0; --l, cur ^= 1)
    ascend_pair<CLS>(td, l, R + (cur ? kT2X1 : kT2X0), R + (cur ? kT2X0 : kT2X1), b_top, x_top,
                     A, store, cls_lds, nu);
}

}  // namespace

namespace kern {

static size_t park_words(const TailDesc<float> &td) {
  size_t off = 0;
  for (int l = 0; l + 1 < td.nlev; ++l) off += (l == 0 ? 1 : 2) * (size_t)td.nx[l] * td.ny[l];
  return off;
}

size_t vtail2_lds_bytes(const TailDesc<float> &td) {
  return (kT2A + kT2R + park_words(td) + kT2ClsLevel * (size_t)td.nlev) * sizeof(float);
}

// The register tail takes levels of at most 64 x 64 nodes, even dimensions
// on every level that is smoothed, up to kTailLevels levels; the coarsest
// level has at most kTailMaxCoarse nodes, and everything fits 64 KiB of LDS.
bool vtail2_ok(const TailDesc<float> &td) {
  if (td.nlev < 1 || td.nlev > kTailLevels) return false;
  for (int l = 0; l < td.nlev; ++l) {
    if (td.nx[l] > 64 || td.ny[l] > 64) return false;
    if (l + 1 < td.nlev && (td.nx[l] % 2 || td.ny[l] % 2)) return false;
  }
  const int nc = td.nx[td.nlev - 1] * td.ny[td.nlev - 1];
  return nc <= kTailMaxCoarse && vtail2_lds_bytes(td) <= 65536;
}

// First level run by wave 0 alone: the wave levels (at most 16 x 16) end in a
// dense coarsest level of at most kT2SCoarse unknowns; nlev when there are none.
static int wave_levels_start(const TailDesc<float> &td) {
  const int L = td.nlev;
  const int nxc = td.nx[L - 1], nyc = td.ny[L - 1];
  if (nxc * nyc > kT2SCoarse || nxc > kT2SSide || nyc > kT2SSide) return L;
  int ls = L - 1;
  while (ls > 0 && td.nx[ls - 1] <= kT2SSide && td.ny[ls - 1] <= kT2SSide) --ls;
  return ls;
}

void vtail2(const TailDesc<float> &td, int nu, const float *b, float *x, hipStream_t st) {
  T2Desc d{};
  d.nlev = td.nlev;
  d.ls = wave_levels_start(td);
  int off = 0;
  for (int l = 0; l < td.nlev; ++l) {
    d.nx[l] = td.nx[l];
    d.ny[l] = td.ny[l];
    d.cls[l] = td.cls[l];
    d.arr[l] = td.arr[l];
    d.pw[l] = td.pw[l];
    d.store_off[l] = off;
    if (l + 1 < td.nlev) off += (l == 0 ? 1 : 2) * td.nx[l] * td.ny[l];
  }
  d.pa = td.pa;
  d.pn = td.pn;
  d.CinvT = td.CinvT;
  const size_t bytes = vtail2_lds_bytes(td);
  const bool cls = td.cls[0] || td.nlev == 1;
  if (cls)
    k_vtail2<true><<<1, kT2Threads, bytes, st>>>(d, b, x, nu);
  else
    k_vtail2<false><<<1, kT2Threads, bytes, st>>>(d, b, x, nu);
}

}  // namespace kern
}  // namespace irk
