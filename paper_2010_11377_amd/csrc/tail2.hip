// The coarse tail of the FP32 V-cycle in one workgroup, rows in registers.
//
// Levels of the tail are at most 64 x 64.  Two layouts:
//
// * workgroup levels (wider or taller than 16): lane i of every wave holds
//   grid column i and the 16 waves split the rows (up to four rows per wave,
//   in registers).  A red-black half sweep needs only the rows just above and
//   below a wave's block from other waves: each wave publishes its first and
//   last row in LDS after every half sweep, double buffered, so one barrier
//   per half sweep suffices;
// * wave levels (at most 16 x 16) above a dense coarsest level of at most 64
//   unknowns run in wave 0 alone: 16 lanes per row of columns, four row
//   groups of up to four rows each, the same publish/read scheme between row
//   groups with wave-scope ordering instead of workgroup barriers.  The other
//   waves meanwhile copy the coarsest inverse into LDS and wait at one
//   barrier.
//
// East/west neighbours come from adjacent lanes through DPP (wave shifts for
// the workgroup layout, row shifts within 16 lanes for the wave layout).  The
// relaxation is Jacobi within a colour (all updates of a half sweep read old
// values), which for five-point operators is Gauss-Seidel.
//
// During the descent the pre-smoothed x of every level (and b below the top
// level) is parked in LDS and picked up again on the way back.  Residuals go
// through a level array in LDS of their own, and each ascending level hands
// its x to the next finer one through one of two alternating areas, so no
// barrier is spent on freeing shared space.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace irk {
namespace {

constexpr int kT2Threads = 1024;
constexpr int kT2Waves = kT2Threads / 64;
constexpr int kT2Rows = 4;   // rows per wave (workgroup layout) or row group (wave layout)
constexpr int kT2Cols = 64;  // one column per lane
constexpr int kT2A = 2 * kT2Waves * 2 * kT2Cols;  // exchange area = 4096 floats
constexpr int kT2R = 64 * 64;                      // level array
// Offsets inside the level array of areas used while it holds at most the
// residual of a 32 x 32 level: the wave layout's exchange slots (256 floats),
// the coarsest right-hand side (64) and the two hand-over areas (1024 each).
constexpr int kT2SEx = 1024, kT2Bc = 1536, kT2X0 = 2048, kT2X1 = 3072;
constexpr int kT2SUnits = 4, kT2SCols = 16;
constexpr int kT2SSide = 16;    // wave levels: at most 16 x 16
constexpr int kT2SCoarse = 64;  // dense coarsest level solved by one wave
constexpr int kT2CiPer =        // inverse entries copied per thread of waves 1..15
    (kT2SCoarse * kT2SCoarse + kT2Threads - 64 - 1) / (kT2Threads - 64);

template <bool W>
struct Lay {
  static constexpr int units = W ? kT2SUnits : kT2Waves;
  static constexpr int cols = W ? kT2SCols : kT2Cols;
  // the wave index is made explicitly uniform, so row counts live in scalar
  // registers and loops over rows branch on the scalar unit
  __device__ static int unit() {
    return W ? ((threadIdx.x & 63) >> 4) : __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  }
  __device__ static int lane() { return W ? (threadIdx.x & 15) : (threadIdx.x & 63); }
};

// lane + 1 / lane - 1 within the layout's row of columns (0 past its end)
template <bool W>
__device__ __forceinline__ float t2_next(float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(v), W ? 0x101 : 0x130, 0xF, 0xF, true));
}
template <bool W>
__device__ __forceinline__ float t2_prev(float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(v), W ? 0x111 : 0x138, 0xF, 0xF, true));
}

// Orders the LDS accesses of one wave (its LDS instructions execute in order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
template <bool W>
__device__ __forceinline__ void t2_sync() {
  if (W)
    wave_sync();
  else
    __syncthreads();
}

__device__ __forceinline__ int t2_cls(int i, int j, int nx, int ny) {
  const int cx = (i == 0) ? 0 : (i == nx - 1 ? 2 : 1);
  const int cy = (j == 0) ? 0 : (j == ny - 1 ? 2 : 1);
  return 3 * cy + cx;
}

// This thread's share of a level: rows [r0, r0 + nr) of unit u, column i.
struct Share {
  int nx, ny, r0, nr, i, u;
  bool col;  // the lane holds a grid column
};

template <bool W>
__device__ __forceinline__ Share share_of(int nx, int ny) {
  Share s;
  const int rpu = (ny + Lay<W>::units - 1) / Lay<W>::units;
  s.u = Lay<W>::unit();
  s.nx = nx;
  s.ny = ny;
  s.r0 = s.u * rpu;
  s.nr = max(0, min(rpu, ny - s.r0));
  s.i = Lay<W>::lane();
  s.col = s.i < nx;
  return s;
}

// Exchange slot of unit u, side 0 (first row) or 1 (last row), buffer buf.
template <bool W>
__device__ __forceinline__ float *xslot(float *ex, int buf, int u, int side) {
  return ex + ((buf * Lay<W>::units + u) * 2 + side) * Lay<W>::cols;
}

// Coefficients of this thread's nodes (9 per node and 1 / centre).
struct RowCo {
  float c[kT2Rows][9];
  float inv[kT2Rows];
};

template <bool CLS>
__device__ __forceinline__ void load_co(const Share &s, const float *cls_lds, const float *arr,
                                        RowCo &co) {
  const size_t N = (size_t)s.nx * s.ny;
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) {
    const int j = s.r0 + t;
    const bool ok = t < s.nr && s.col;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      float v = 0.0f;
      if (ok) v = CLS ? cls_lds[9 * t2_cls(s.i, j, s.nx, s.ny) + k]
                      : arr[(size_t)k * N + (size_t)j * s.nx + s.i];
      co.c[t][k] = v;
    }
    co.inv[t] = ok ? 1.0f / co.c[t][4] : 0.0f;
  }
}

// The rows above and below each of this unit's rows: own registers inside
// the block, the neighbouring units' rows published in buffer buf at its
// ends (zero outside the grid).  Both published rows are read at once, from
// clamped slots, so the reads are unconditional.
template <bool W>
__device__ __forceinline__ void neighbours(const Share &s, const float (&x)[kT2Rows], float *ex,
                                           int buf, float (&up)[kT2Rows], float (&dn)[kT2Rows]) {
  const int ua = max(s.u - 1, 0), ub = min(s.u + 1, Lay<W>::units - 1);
  const float ta = xslot<W>(ex, buf, ua, 1)[s.i], tb = xslot<W>(ex, buf, ub, 0)[s.i];
  const float top = (s.r0 > 0 && s.col) ? ta : 0.0f;
  const float bot = (s.r0 + s.nr < s.ny && s.col) ? tb : 0.0f;
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) {
    up[t] = (t == 0) ? top : x[t > 0 ? t - 1 : 0];
    dn[t] = (t + 1 < kT2Rows && t + 1 < s.nr) ? x[t + 1 < kT2Rows ? t + 1 : t] : bot;
  }
}

// sum_k a_k x_k over the stencil of a row (centre included when CENTRE),
// summed as a tree of four pairs.
template <bool W, bool CENTRE>
__device__ __forceinline__ float stencil_sum(const float *a, float up, float mid, float dn) {
  const float s0 = a[0] * t2_prev<W>(up) + a[1] * up;
  const float s1 = a[2] * t2_next<W>(up) + a[3] * t2_prev<W>(mid);
  const float s2 = a[5] * t2_next<W>(mid) + a[6] * t2_prev<W>(dn);
  const float s3 = a[7] * dn + a[8] * t2_next<W>(dn);
  float acc = (s0 + s1) + (s2 + s3);
  if (CENTRE) acc += a[4] * mid;
  return acc;
}

// Publish this unit's first and last row in exchange buffer buf.
template <bool W>
__device__ __forceinline__ void publish(const Share &s, const float (&x)[kT2Rows], float *ex,
                                        int buf) {
  if (s.nr == 0) return;
  float last = x[0];
#pragma unroll
  for (int t = 1; t < kT2Rows; ++t)
    if (t == s.nr - 1) last = x[t];
  xslot<W>(ex, buf, s.u, 0)[s.i] = x[0];
  xslot<W>(ex, buf, s.u, 1)[s.i] = last;
}

// One colour half sweep reading the rows published in buffer rb, then
// publishing into rb ^ 1 (and the whole level into `full` when given) and
// synchronising.
template <bool W>
__device__ __forceinline__ void half_sweep(const Share &s, const RowCo &co, float (&x)[kT2Rows],
                                           const float (&b)[kT2Rows], float *ex, int rb,
                                           int color, float *full) {
  float up[kT2Rows], dn[kT2Rows], nv[kT2Rows];
  neighbours<W>(s, x, ex, rb, up, dn);
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) {
    nv[t] = x[t];
    if (t < s.nr) {
      const float v = (b[t] - stencil_sum<W, false>(co.c[t], up[t], x[t], dn[t])) * co.inv[t];
      // m v + (1 - m) x with m in {0, 1}: exact, and computed on every lane
      // (a select lets the compiler branch around the stencil per lane)
      const float m = (s.col && ((s.i + s.r0 + t) & 1) == color) ? 1.0f : 0.0f;
      nv[t] = m * v + (1.0f - m) * x[t];
    }
  }
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) x[t] = nv[t];
  publish<W>(s, x, ex, rb ^ 1);
  if (full) {
#pragma unroll
    for (int t = 0; t < kT2Rows; ++t)
      if (t < s.nr && s.col) full[(s.r0 + t) * s.nx + s.i] = x[t];
  }
  t2_sync<W>();
}

struct T2Desc {
  int nlev;
  int ls;  // first level run by wave 0 alone (nlev: none)
  int nx[kTailLevels], ny[kTailLevels];
  const float *cls[kTailLevels];
  const float *arr[kTailLevels];
  float pw[kTailLevels];
  float pa, pn;  // prolongation weights from the own and the next coarse node
  const float *CinvT;
  int store_off[kTailLevels];  // LDS offset of level l's parked x (and b for l > 0)
};

// Pre-smoothing of level l from x = 0; residual into R, x (and b) parked.
template <bool W, bool CLS>
__device__ __forceinline__ void descend(const T2Desc &td, int l, const float (&b)[kT2Rows],
                                        float *ex, float *R, float *store, const float *cls_lds,
                                        int nu) {
  const Share s = share_of<W>(td.nx[l], td.ny[l]);
  RowCo co;
  load_co<CLS>(s, cls_lds + 81 * l, td.arr[l], co);
  float x[kT2Rows];
  // x = 0, then colour 0 takes b / d
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t)
    x[t] = (t < s.nr && s.col && ((s.i + s.r0 + t) & 1) == 0) ? b[t] * co.inv[t] : 0.0f;
  publish<W>(s, x, ex, 0);
  t2_sync<W>();
  int buf = 0;
  for (int h = 1; h < 2 * nu; ++h) {
    half_sweep<W>(s, co, x, b, ex, buf, h & 1, nullptr);
    buf ^= 1;
  }
  float *px = store + td.store_off[l];
  float *pb = px + s.nx * s.ny;
  float up[kT2Rows], dn[kT2Rows];
  neighbours<W>(s, x, ex, buf, up, dn);
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) {
    const float r = b[t] - stencil_sum<W, true>(co.c[t], up[t], x[t], dn[t]);
    if (t < s.nr && s.col) {
      const int p = (s.r0 + t) * s.nx + s.i;
      px[p] = x[t];
      if (l > 0) pb[p] = b[t];
      R[p] = r;
    }
  }
  t2_sync<W>();
}

// Right-hand side of level l + 1: sums of level l's residual over 2 x 2 cells.
template <bool W>
__device__ __forceinline__ void restrict_to(const T2Desc &td, int l, const float *R,
                                            float (&b)[kT2Rows]) {
  const Share c = share_of<W>(td.nx[l + 1], td.ny[l + 1]);
  const int fnx = td.nx[l];
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) {
    float v = 0.0f;
    if (t < c.nr && c.col) {
      const int J = c.r0 + t, I = c.i;
      const float *row0 = R + (2 * J) * fnx, *row1 = row0 + fnx;
      v = row0[2 * I] + row0[2 * I + 1] + row1[2 * I] + row1[2 * I + 1];
    }
    b[t] = v;
  }
}

// Coarse correction of level l from the coarse x in xc, then post-smoothing;
// the result goes to xo (l > 0) or to x_top (l == 0).
template <bool W, bool CLS>
__device__ __forceinline__ void ascend(const T2Desc &td, int l, const float *xc, float *xo,
                                       const float *b_top, float *x_top, float *ex,
                                       const float *store, const float *cls_lds, int nu) {
  const Share s = share_of<W>(td.nx[l], td.ny[l]);
  const int ncx = td.nx[l + 1], ncy = td.ny[l + 1];
  const float pw = td.pw[l];
  const float *px = store + td.store_off[l];
  const float *pb = px + s.nx * s.ny;
  float x[kT2Rows], b[kT2Rows];
  // x = parked x + P x_c; b back from the park (level 0: from global)
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) {
    const bool ok = t < s.nr && s.col;
    // out-of-range neighbours get weight 0 and a clamped (valid) address
    const int fx = ok ? s.i : 0, fy = ok ? s.r0 + t : 0, p = fy * s.nx + fx;
    const int Ix = fx >> 1, Iy = fy >> 1;
    const int nbx = (fx & 1) ? Ix + 1 : Ix - 1, nby = (fy & 1) ? Iy + 1 : Iy - 1;
    const bool hx = nbx >= 0 && nbx < ncx, hy = nby >= 0 && nby < ncy;
    const int nbxc = hx ? nbx : Ix, nbyc = hy ? nby : Iy;
    const float wx = hx ? td.pa : pw, wy = hy ? td.pa : pw;
    const float ax = hx ? td.pn : 0.0f, ay = hy ? td.pn : 0.0f;
    const float cv = (wx * wy * xc[Iy * ncx + Ix] + ax * wy * xc[Iy * ncx + nbxc]) +
                     (wx * ay * xc[nbyc * ncx + Ix] + ax * ay * xc[nbyc * ncx + nbxc]);
    const float pv = px[p];
    float bv = 0.0f;
    if (ok) bv = (l > 0) ? pb[p] : b_top[p];
    x[t] = ok ? pv + cv : 0.0f;
    b[t] = bv;
  }
  RowCo co;
  load_co<CLS>(s, cls_lds + 81 * l, td.arr[l], co);
  publish<W>(s, x, ex, 0);
  t2_sync<W>();
  int buf = 0;
  for (int h = 0; h < 2 * nu; ++h) {  // colour 1 first
    half_sweep<W>(s, co, x, b, ex, buf, (h & 1) ^ 1, (h == 2 * nu - 1 && l > 0) ? xo : nullptr);
    buf ^= 1;
  }
  if (l == 0) {
#pragma unroll
    for (int t = 0; t < kT2Rows; ++t)
      if (t < s.nr && s.col) x_top[(size_t)(s.r0 + t) * s.nx + s.i] = x[t];
  }
}

template <bool W>
__device__ __forceinline__ void load_top_b(const T2Desc &td, const float *b_top,
                                           float (&b)[kT2Rows]) {
  const Share s = share_of<W>(td.nx[0], td.ny[0]);
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t)
    b[t] = (t < s.nr && s.col) ? b_top[(size_t)(s.r0 + t) * s.nx + s.i] : 0.0f;
}

template <bool CLS>
__global__ void __launch_bounds__(kT2Threads)
    k_vtail2(T2Desc td, const float *__restrict__ b_top, float *__restrict__ x_top, int nu) {
  extern __shared__ float sm[];
  float *A = sm;            // workgroup exchange buffers; coarsest inverse or its scratch
  float *R = sm + kT2A;     // level array and the areas placed at kT2SEx ...
  float *store = R + kT2R;  // parked x, b
  float *cls_lds = store + td.store_off[td.nlev - 1];  // class tables, 81 per level
  const int L = td.nlev, ls = td.ls;
  const bool wave_tail = ls < L;
  const int wave = threadIdx.x >> 6;
  if (CLS)
    for (int q = threadIdx.x; q < 81 * (L - 1); q += kT2Threads) cls_lds[q] = td.cls[q / 81][q % 81];
  __syncthreads();

  float b[kT2Rows] = {0.0f, 0.0f, 0.0f, 0.0f};
  if (ls > 0)
    load_top_b<false>(td, b_top, b);
  else if (wave == 0)
    load_top_b<true>(td, b_top, b);

  // ---- descent through the workgroup levels
  const int lm = min(ls, L - 1);
  for (int l = 0; l < lm; ++l) {
    descend<false, CLS>(td, l, b, A, R, store, cls_lds, nu);
    if (l + 1 < ls)
      restrict_to<false>(td, l, R, b);
    else if (wave == 0)
      restrict_to<true>(td, l, R, b);
  }

  const int nc = td.nx[L - 1] * td.ny[L - 1];
  int cur = 0;  // hand-over area holding the x of the level below the next one up
  if (wave_tail) {
    if (wave == 0) {
      for (int l = ls; l + 1 < L; ++l) {
        descend<true, CLS>(td, l, b, R + kT2SEx, R, store, cls_lds, nu);
        restrict_to<true>(td, l, R, b);
      }
    } else {
      float v[kT2CiPer];
      const int q0 = threadIdx.x - 64;
#pragma unroll
      for (int k = 0; k < kT2CiPer; ++k) {
        const int q = q0 + k * (kT2Threads - 64);
        v[k] = q < nc * nc ? td.CinvT[q] : 0.0f;
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
      const Share c = share_of<true>(td.nx[L - 1], td.ny[L - 1]);
      float *bc = R + kT2Bc;
#pragma unroll
      for (int t = 0; t < kT2Rows; ++t)
        if (t < c.nr && c.col) bc[(c.r0 + t) * c.nx + c.i] = b[t];
      wave_sync();
      const int row = threadIdx.x;
      if (row < nc) {
        float acc = 0.0f;
        for (int col = 0; col < nc; ++col) acc += A[col * nc + row] * bc[col];
        if (L == 1)
          x_top[row] = acc;
        else
          R[kT2X0 + row] = acc;
      }
      wave_sync();
      int k = 0;
      for (int l = L - 2; l >= ls; --l, k ^= 1)
        ascend<true, CLS>(td, l, R + (k ? kT2X1 : kT2X0), R + (k ? kT2X0 : kT2X1), b_top, x_top,
                          R + kT2SEx, store, cls_lds, nu);
    }
    __syncthreads();
    if (ls == 0) return;
    cur = (L - 1 - ls) & 1;
  } else {
    // coarsest by the whole workgroup: partial products over column blocks
    const Share c = share_of<false>(td.nx[L - 1], td.ny[L - 1]);
    float *bc = A, *red = A + kTailMaxCoarse;
#pragma unroll
    for (int t = 0; t < kT2Rows; ++t)
      if (t < c.nr && c.col) bc[(c.r0 + t) * c.nx + c.i] = b[t];
    __syncthreads();
    const int nb = kT2Threads / nc;  // nc <= kTailMaxCoarse = kT2Threads
    for (int q = threadIdx.x; q < nb * nc; q += kT2Threads) {
      const int row = q % nc, cb = q / nc;
      float acc = 0.0f;
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
    ascend<false, CLS>(td, l, R + (cur ? kT2X1 : kT2X0), R + (cur ? kT2X0 : kT2X1), b_top, x_top,
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
  return (kT2A + kT2R + park_words(td) + 81 * (size_t)td.nlev) * sizeof(float);
}

// The register tail takes levels of at most 64 x 64 nodes and up to
// kTailLevels levels; the coarsest level has at most kTailMaxCoarse nodes,
// and everything fits 64 KiB of LDS.
bool vtail2_ok(const TailDesc<float> &td) {
  if (td.nlev < 1 || td.nlev > kTailLevels) return false;
  for (int l = 0; l < td.nlev; ++l)
    if (td.nx[l] > kT2Cols || td.ny[l] > kT2Waves * kT2Rows) return false;
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
