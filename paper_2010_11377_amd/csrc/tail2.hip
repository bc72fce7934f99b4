// The coarse tail of the FP32 V-cycle in one workgroup, rows in registers.
//
// Levels of the tail are at most 64 x 64: lane i of every wave holds grid
// column i, and the 16 waves split the rows (up to four rows per wave, in
// registers).  A red-black half sweep needs only the rows just above and
// below a wave's block from other waves: each wave publishes its first and
// last row in LDS after every half sweep, double buffered, so one barrier per
// half sweep suffices (the old kernel keeps the whole level in LDS and needs
// two).  East/west neighbours come from adjacent lanes through DPP.  The
// relaxation is Jacobi within a colour (all updates of a half sweep read old
// values), which for five-point operators is Gauss-Seidel.
//
// During the descent the pre-smoothed x of every level (and b below the top
// level) is parked in LDS and picked up again on the way back.  The restricted
// residual and the coarse correction travel through a level-sized LDS array
// that shares space with the exchange buffers.  The coarsest level is the
// dense product with the stored inverse.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace irk {
namespace {

constexpr int kT2Threads = 1024;
constexpr int kT2Waves = kT2Threads / 64;
constexpr int kT2Rows = 4;   // rows per wave at most
constexpr int kT2Cols = 64;  // one column per lane
constexpr int kT2A = 2 * kT2Waves * 2 * kT2Cols;  // exchange area = 4096 floats

__device__ __forceinline__ float t2_next(float v) {  // lane + 1 (0 in lane 63)
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ float t2_prev(float v) {  // lane - 1 (0 in lane 0)
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}

__device__ __forceinline__ int t2_cls(int i, int j, int nx, int ny) {
  const int cx = (i == 0) ? 0 : (i == nx - 1 ? 2 : 1);
  const int cy = (j == 0) ? 0 : (j == ny - 1 ? 2 : 1);
  return 3 * cy + cx;
}

// This wave's share of a level: rows [r0, r0 + nr), column i = lane.
struct Share {
  int nx, ny, r0, nr, i;
  bool col;  // lane holds a grid column
};

__device__ __forceinline__ Share share_of(int nx, int ny) {
  Share s;
  const int rpw = (ny + kT2Waves - 1) / kT2Waves;
  const int w = threadIdx.x >> 6;
  s.nx = nx;
  s.ny = ny;
  s.r0 = w * rpw;
  s.nr = max(0, min(rpw, ny - s.r0));
  s.i = threadIdx.x & 63;
  s.col = s.i < nx;
  return s;
}

// Exchange slot of wave w, side 0 (first row) or 1 (last row), buffer buf.
__device__ __forceinline__ float *xslot(float *A, int buf, int w, int side) {
  return A + ((buf * kT2Waves + w) * 2 + side) * kT2Cols;
}

// Coefficients of this wave's nodes (9 per node and 1 / centre).
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

// The row above / below row t of this wave: own registers inside the block,
// the neighbour waves' published rows at its ends (zero outside the grid).
__device__ __forceinline__ float row_above(const Share &s, const float (&x)[kT2Rows], int t,
                                           const float *A, int buf) {
  if (t > 0) return x[t - 1];
  const int w = threadIdx.x >> 6;
  return (s.r0 > 0 && s.col) ? xslot(const_cast<float *>(A), buf, w - 1, 1)[s.i] : 0.0f;
}
__device__ __forceinline__ float row_below(const Share &s, const float (&x)[kT2Rows], int t,
                                           const float *A, int buf) {
  if (t + 1 < s.nr) return x[t + 1];
  const int w = threadIdx.x >> 6;
  return (s.r0 + t + 1 < s.ny && s.col) ? xslot(const_cast<float *>(A), buf, w + 1, 0)[s.i]
                                        : 0.0f;
}

// sum_k a_k x_k over the stencil of row t (centre included when CENTRE).
template <bool CENTRE>
__device__ __forceinline__ float stencil_sum(const float *a, float up, float mid, float dn) {
  float acc = a[0] * t2_prev(up) + a[1] * up + a[2] * t2_next(up) + a[3] * t2_prev(mid) +
              a[5] * t2_next(mid) + a[6] * t2_prev(dn) + a[7] * dn + a[8] * t2_next(dn);
  if (CENTRE) acc += a[4] * mid;
  return acc;
}

// Publish this wave's first and last row in exchange buffer buf.
__device__ __forceinline__ void publish(const Share &s, const float (&x)[kT2Rows], float *A,
                                        int buf) {
  if (s.nr == 0) return;
  const int w = threadIdx.x >> 6;
  float last = x[0];
#pragma unroll
  for (int t = 1; t < kT2Rows; ++t)
    if (t == s.nr - 1) last = x[t];
  xslot(A, buf, w, 0)[s.i] = x[0];
  xslot(A, buf, w, 1)[s.i] = last;
}

// One colour half sweep reading the rows published in buffer rb, then
// publishing into rb ^ 1 and waiting for everyone.
__device__ __forceinline__ void half_sweep(const Share &s, const RowCo &co, float (&x)[kT2Rows],
                                           const float (&b)[kT2Rows], float *A, int rb,
                                           int color) {
  float nv[kT2Rows];
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) {
    const float up = row_above(s, x, t, A, rb), dn = row_below(s, x, t, A, rb);
    const float v = (b[t] - stencil_sum<false>(co.c[t], up, x[t], dn)) * co.inv[t];
    const int j = s.r0 + t;
    nv[t] = (t < s.nr && s.col && ((s.i + j) & 1) == color) ? v : x[t];
  }
#pragma unroll
  for (int t = 0; t < kT2Rows; ++t) x[t] = nv[t];
  publish(s, x, A, rb ^ 1);
  __syncthreads();
}

struct T2Desc {
  int nlev;
  int nx[kTailLevels], ny[kTailLevels];
  const float *cls[kTailLevels];
  const float *arr[kTailLevels];
  float pw[kTailLevels];
  const float *CinvT;
  int store_off[kTailLevels];  // LDS offset of level l's parked x (and b for l > 0)
};

template <bool CLS>
__global__ void __launch_bounds__(kT2Threads)
    k_vtail2(T2Desc td, const float *__restrict__ b_top, float *__restrict__ x_top, int nu) {
  extern __shared__ float sm[];
  float *A = sm;                              // exchange buffers / level array
  float *store = sm + kT2A;                   // parked x, b
  float *cls_lds = store + td.store_off[td.nlev - 1];  // class tables, 81 per level
  const int L = td.nlev;
  if (CLS)
    for (int q = threadIdx.x; q < 81 * (L - 1); q += kT2Threads) cls_lds[q] = td.cls[q / 81][q % 81];
  __syncthreads();

  float x[kT2Rows], b[kT2Rows];
  // level 0 right-hand side from global memory
  {
    const Share s = share_of(td.nx[0], td.ny[0]);
#pragma unroll
    for (int t = 0; t < kT2Rows; ++t)
      b[t] = (t < s.nr && s.col) ? b_top[(size_t)(s.r0 + t) * s.nx + s.i] : 0.0f;
  }

  // ---- descent
  for (int l = 0; l + 1 < L; ++l) {
    const Share s = share_of(td.nx[l], td.ny[l]);
    RowCo co;
    load_co<CLS>(s, cls_lds + 81 * l, td.arr[l], co);
    // x = 0, then colour 0 takes b / d
#pragma unroll
    for (int t = 0; t < kT2Rows; ++t)
      x[t] = (t < s.nr && s.col && ((s.i + s.r0 + t) & 1) == 0) ? b[t] * co.inv[t] : 0.0f;
    publish(s, x, A, 0);
    __syncthreads();
    int buf = 0;
    for (int h = 1; h < 2 * nu; ++h) {
      half_sweep(s, co, x, b, A, buf, h & 1);
      buf ^= 1;
    }
    // residual from the last published rows
    float r[kT2Rows];
#pragma unroll
    for (int t = 0; t < kT2Rows; ++t) {
      const float up = row_above(s, x, t, A, buf), dn = row_below(s, x, t, A, buf);
      r[t] = b[t] - stencil_sum<true>(co.c[t], up, x[t], dn);
    }
    // park x (and b) of this level
    float *px = store + td.store_off[l];
    float *pb = px + s.nx * s.ny;
#pragma unroll
    for (int t = 0; t < kT2Rows; ++t)
      if (t < s.nr && s.col) {
        const int p = (s.r0 + t) * s.nx + s.i;
        px[p] = x[t];
        if (l > 0) pb[p] = b[t];
      }
    __syncthreads();  // exchange buffers free: the level array may overwrite them
#pragma unroll
    for (int t = 0; t < kT2Rows; ++t)
      if (t < s.nr && s.col) A[(s.r0 + t) * s.nx + s.i] = r[t];
    __syncthreads();
    // coarse b = sum over 2 x 2 cells
    const Share c = share_of(td.nx[l + 1], td.ny[l + 1]);
#pragma unroll
    for (int t = 0; t < kT2Rows; ++t) {
      float v = 0.0f;
      if (t < c.nr && c.col) {
        const int J = c.r0 + t, I = c.i;
        const float *row0 = A + (2 * J) * s.nx, *row1 = row0 + s.nx;
        v = row0[2 * I] + row0[2 * I + 1] + row1[2 * I] + row1[2 * I + 1];
      }
      b[t] = v;
    }
    __syncthreads();
  }

  // ---- coarsest level: x = C^-1 b with C^-1 stored transposed
  {
    const Share c = share_of(td.nx[L - 1], td.ny[L - 1]);
    const int n = c.nx * c.ny;
    float *bc = A, *red = A + kTailMaxCoarse, *xc = A + 2 * kTailMaxCoarse;
#pragma unroll
    for (int t = 0; t < kT2Rows; ++t)
      if (t < c.nr && c.col) bc[(c.r0 + t) * c.nx + c.i] = b[t];
    __syncthreads();
    const int nb = kT2Threads / n;  // n <= kTailMaxCoarse = kT2Threads
    for (int q = threadIdx.x; q < nb * n; q += kT2Threads) {
      const int row = q % n, cb = q / n;
      float acc = 0.0f;
      for (int col = cb; col < n; col += nb) acc += td.CinvT[(size_t)col * n + row] * bc[col];
      red[q] = acc;
    }
    __syncthreads();
    for (int row = threadIdx.x; row < n; row += kT2Threads) {
      float acc = 0.0f;
      for (int cb = 0; cb < nb; ++cb) acc += red[cb * n + row];
      xc[row] = acc;
    }
    __syncthreads();
    if (L == 1) {
      for (int row = threadIdx.x; row < n; row += kT2Threads) x_top[row] = xc[row];
      return;
    }
  }

  // ---- ascent: the coarse x of level l+1 is in A (at offset xoff)
  int xoff = 2 * kTailMaxCoarse;
  for (int l = L - 2; l >= 0; --l) {
    const Share s = share_of(td.nx[l], td.ny[l]);
    const int ncx = td.nx[l + 1], ncy = td.ny[l + 1];
    const float pw = td.pw[l];
    const float *xc = A + xoff;
    const float *px = store + td.store_off[l];
    const float *pb = px + s.nx * s.ny;
    // x = parked x + P x_c; b back from the park (level 0: from global)
#pragma unroll
    for (int t = 0; t < kT2Rows; ++t) {
      float xv = 0.0f, bv = 0.0f;
      if (t < s.nr && s.col) {
        const int fx = s.i, fy = s.r0 + t, p = fy * s.nx + fx;
        const int Ix = fx >> 1, Iy = fy >> 1;
        const int nbx = (fx & 1) ? Ix + 1 : Ix - 1, nby = (fy & 1) ? Iy + 1 : Iy - 1;
        const bool hx = nbx >= 0 && nbx < ncx, hy = nby >= 0 && nby < ncy;
        const float wx = hx ? 0.75f : pw, wy = hy ? 0.75f : pw;
        float cv = wx * wy * xc[Iy * ncx + Ix];
        if (hx) cv += 0.25f * wy * xc[Iy * ncx + nbx];
        if (hy) cv += wx * 0.25f * xc[nby * ncx + Ix];
        if (hx && hy) cv += 0.0625f * xc[nby * ncx + nbx];
        xv = px[p] + cv;
        bv = (l > 0) ? pb[p] : b_top[p];
      }
      x[t] = xv;
      b[t] = bv;
    }
    __syncthreads();  // the coarse x is read: exchange buffers free
    RowCo co;
    load_co<CLS>(s, cls_lds + 81 * l, td.arr[l], co);
    publish(s, x, A, 0);
    __syncthreads();
    int buf = 0;
    for (int h = 0; h < 2 * nu; ++h) {  // colour 1 first
      half_sweep(s, co, x, b, A, buf, (h & 1) ^ 1);
      buf ^= 1;
    }
    if (l > 0) {
      // hand x to the next finer level through the level array (after the
      // barrier that closed the last half sweep nobody reads the buffers)
      xoff = 2 * kTailMaxCoarse;
#pragma unroll
      for (int t = 0; t < kT2Rows; ++t)
        if (t < s.nr && s.col) A[xoff + (s.r0 + t) * s.nx + s.i] = x[t];
      __syncthreads();
    } else {
#pragma unroll
      for (int t = 0; t < kT2Rows; ++t)
        if (t < s.nr && s.col) x_top[(size_t)(s.r0 + t) * s.nx + s.i] = x[t];
    }
  }
}

}  // namespace

namespace kern {

// The register tail takes levels of at most 64 x 64 nodes and up to
// kTailLevels levels; the coarsest level has at most kTailMaxCoarse nodes.
bool vtail2_ok(const TailDesc<float> &td) {
  if (td.nlev < 1 || td.nlev > kTailLevels) return false;
  for (int l = 0; l < td.nlev; ++l)
    if (td.nx[l] > kT2Cols || td.ny[l] > kT2Waves * kT2Rows) return false;
  const int nc = td.nx[td.nlev - 1] * td.ny[td.nlev - 1];
  return nc <= kTailMaxCoarse;
}

void vtail2(const TailDesc<float> &td, int nu, const float *b, float *x, hipStream_t st) {
  T2Desc d{};
  d.nlev = td.nlev;
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
  d.CinvT = td.CinvT;
  // the level array holds the coarse x at offset 2 * kTailMaxCoarse
  const size_t words = kT2A + off + 81 * (size_t)td.nlev;
  const bool cls = td.cls[0] || td.nlev == 1;
  if (cls)
    k_vtail2<true><<<1, kT2Threads, words * sizeof(float), st>>>(d, b, x, nu);
  else
    k_vtail2<false><<<1, kT2Threads, words * sizeof(float), st>>>(d, b, x, nu);
}

size_t vtail2_lds_bytes(const TailDesc<float> &td) {
  size_t off = 0;
  for (int l = 0; l + 1 < td.nlev; ++l) off += (l == 0 ? 1 : 2) * (size_t)td.nx[l] * td.ny[l];
  return (kT2A + off + 81 * (size_t)td.nlev) * sizeof(float);
}

}  // namespace kern
}  // namespace irk
