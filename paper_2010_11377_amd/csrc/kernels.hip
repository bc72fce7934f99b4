// Device kernels of the IRK stage solver for gfx950 (CDNA4, wave64).
//
// Layout: every grid vector is x-fastest (p = j * nx + i); stage vectors are
// stage-major (element (i, p) at i * N + p); a Krylov column of the stage
// system is s * N contiguous doubles.
//
// The kernels are HBM-bound sparse/vector passes (<= ~1 flop per byte), so
// they are organised around coalesced loads and few passes over the data:
//  * the Kronecker SpMM reads every stage vector once and mixes the s values
//    of K z at a node through the s x s matrix h A held in scalar registers;
//  * the Gram-Schmidt dot products are fused into the SpMM (the SpMM result
//    is never written), and the update pass recomputes it instead of reading
//    it back;
//  * every reduction is a fixed-order two-stage (block, then single-block)
//    sum, so results are bitwise reproducible run to run.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.hpp"

namespace irk {
namespace {

struct Mat8 {
  double a[64];
};
struct Row8 {
  double c[8];
};

__device__ __forceinline__ int node_class_d(int i, int j, int nx, int ny) {
  int cx = (i == 0) ? 0 : (i == nx - 1 ? 2 : 1);
  int cy = (j == 0) ? 0 : (j == ny - 1 ? 2 : 1);
  return 3 * cy + cx;
}

// Sum over the block, valid on thread 0.  Fixed order: wave shuffle tree,
// then the 4 wave results in order.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kBlock / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) r += red[q];
  }
  return r;
}

// Single-workgroup sums of the per-block partials of a reduction (up to
// tens of thousands of doubles): 1024 threads with eight independent loads in
// flight each, so the pass is not a chain of dependent memory latencies.  The
// summation order is fixed for a given n (deterministic).
constexpr int kRed = 1024;

__device__ __forceinline__ double red_block_sum(double v) {
  __shared__ double red[kRed / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < kRed / 64; ++q) r += red[q];
  }
  return r;
}

__device__ __forceinline__ double sum_partials(const double *__restrict__ p, int n) {
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int b = threadIdx.x;
  for (; b + 7 * kRed < n; b += 8 * kRed) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += p[b + u * kRed];
  }
  for (; b < n; b += kRed) a[0] += p[b];
  const double t = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  return red_block_sum(t);
}

// Coefficient k at node p (boundary class q).  A constant-coefficient table
// has 81 entries and is read through the cache (nearly every lane of a wave
// reads the same interior entry).
template <typename T>
__device__ __forceinline__ T coef(const OpView<T> &op, int q, int k, size_t p, size_t N) {
  return op.cls ? op.cls[q * 9 + k] : op.arr[(size_t)k * N + p];
}

// (A x)_p without the diagonal term; also returns the diagonal coefficient.
template <typename T, typename TX>
__device__ __forceinline__ T offdiag_apply(const OpView<T> &op, const TX *x, int i,
                                           int j, size_t p, size_t N, T &diag) {
  const int nx = op.nx, ny = op.ny;
  const int q = node_class_d(i, j, nx, ny);
  T acc = T(0);
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if (k == 4) continue;
    if (op.npt == 5 && (k == 0 || k == 2 || k == 6 || k == 8)) continue;
    const int dx = k % 3 - 1, dy = k / 3 - 1;
    const int ii = i + dx, jj = j + dy;
    if (ii < 0 || ii >= nx || jj < 0 || jj >= ny) continue;
    acc += coef(op, q, k, p, N) * T(x[(size_t)jj * nx + ii]);
  }
  diag = coef(op, q, 4, p, N);
  return acc;
}

// ---------------------------------------------------------------------------
// right-hand sides and norms

__global__ void __launch_bounds__(kBlock)
    k_rhs_forward(OpView<double> K, const double *__restrict__ u, const double *__restrict__ g,
                  int s, double *__restrict__ f, double *__restrict__ V0,
                  double *__restrict__ partial) {
  const size_t N = (size_t)K.nx * K.ny;
  const size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x;
  double val = 0.0;
  if (p < N) {
    const int i = (int)(p % K.nx), j = (int)(p / K.nx);
    double d;
    double Ku = offdiag_apply(K, u, i, j, p, N, d);
    Ku += d * u[p];
    const double fv = (g ? g[p] : 0.0) - Ku;
    f[p] = fv;
    for (int st = 0; st < s; ++st) V0[(size_t)st * N + p] = fv;
    val = fv * fv * s;
  }
  const double r = block_sum(val);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

__global__ void __launch_bounds__(kBlock)
    k_rhs_copy(const double *__restrict__ rhs, size_t n, double *__restrict__ V0,
               double *__restrict__ partial) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  double val = 0.0;
  if (e < n) {
    const double v = rhs[e];
    V0[e] = v;
    val = v * v;
  }
  const double r = block_sum(val);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

__global__ void __launch_bounds__(kRed)
    k_finalize_norm(const double *__restrict__ partial, int nblk, double *__restrict__ scale,
                    int col, double *__restrict__ norm_out) {
  const double r = sum_partials(partial, nblk);
  if (threadIdx.x == 0) {
    const double nrm = sqrt(r);
    scale[col] = (nrm > 0.0 && isfinite(nrm)) ? 1.0 / nrm : 0.0;
    if (norm_out) *norm_out = nrm;
  }
}

// ---------------------------------------------------------------------------
// block substitution coupling (Sec. 4.2)

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_couple(OpView<T> K, const double *__restrict__ v, const double *__restrict__ scale_j,
             const T *__restrict__ z, Row8 crow, int s, int i, T *__restrict__ b) {
  const size_t N = (size_t)K.nx * K.ny;
  const size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= N) return;
  const int ii = (int)(p % K.nx), jj = (int)(p / K.nx);
  const double sc = *scale_j;
  T acc = T(sc * v[(size_t)i * N + p]);
  bool any = false;
#pragma unroll
  for (int k = 0; k < kMaxStages; ++k)
    if (k < s && crow.c[k] != 0.0) any = true;
  if (any) {
    const int q = node_class_d(ii, jj, K.nx, K.ny);
    T kc = T(0);
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      if (K.npt == 5 && (t == 0 || t == 2 || t == 6 || t == 8)) continue;
      const int dx = t % 3 - 1, dy = t / 3 - 1;
      const int xi = ii + dx, yj = jj + dy;
      if (xi < 0 || xi >= K.nx || yj < 0 || yj >= K.ny) continue;
      const size_t pn = (size_t)yj * K.nx + xi;
      T comb = T(0);
#pragma unroll
      for (int k = 0; k < kMaxStages; ++k)
        if (k < s && crow.c[k] != 0.0) comb += T(crow.c[k]) * z[(size_t)k * N + pn];
      kc += coef(K, q, t, p, N) * comb;
    }
    acc -= kc;
  }
  b[p] = acc;
}

// ---------------------------------------------------------------------------
// Kronecker SpMM with fused Gram-Schmidt

// w_i(p) = (M z_i)(p) + sum_k hA[i][k] (K z_k)(p) for all s stages at node p
// (Sec. 4: the stage matrix I_s (x) M + h A (x) K); M = I unless MASS.
template <typename TZ, int S, bool MASS>
__device__ __forceinline__ void kron_apply(const OpView<double> &K, const OpView<double> &M,
                                           const TZ *__restrict__ z, const Mat8 &hA, size_t p,
                                           size_t N, double *w) {
  const int i = (int)(p % K.nx), j = (int)(p / K.nx);
  const int q = node_class_d(i, j, K.nx, K.ny);
  double kz[S], mz[S];
#pragma unroll
  for (int st = 0; st < S; ++st) kz[st] = mz[st] = 0.0;
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const bool corner = t == 0 || t == 2 || t == 6 || t == 8;
    const bool kt = !(K.npt == 5 && corner);
    const bool mt = MASS && !(M.npt == 5 && corner);
    if (!kt && !mt) continue;
    const int dx = t % 3 - 1, dy = t / 3 - 1;
    const int xi = i + dx, yj = j + dy;
    if (xi < 0 || xi >= K.nx || yj < 0 || yj >= K.ny) continue;
    const size_t pn = (size_t)yj * K.nx + xi;
    const double a = kt ? coef(K, q, t, p, N) : 0.0;
    const double m = mt ? coef(M, q, t, p, N) : 0.0;
#pragma unroll
    for (int st = 0; st < S; ++st) {
      const double zv = double(z[(size_t)st * N + pn]);
      kz[st] += a * zv;
      if (MASS) mz[st] += m * zv;
    }
  }
#pragma unroll
  for (int r = 0; r < S; ++r) {
    double acc = MASS ? mz[r] : double(z[(size_t)r * N + p]);
#pragma unroll
    for (int st = 0; st < S; ++st) acc += hA.a[r * 8 + st] * kz[st];
    w[r] = acc;
  }
}

// Block sums of NV values at once (one pair of barriers); each value is
// summed in the order block_sum uses.
template <int NV>
__device__ __forceinline__ void block_sums(double (&v)[NV]) {
  __shared__ double red[NV][kBlock / 64];
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k][w] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double r = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
      for (int q = 0; q < kBlock / 64; ++q) r += red[k][q];
    }
    v[k] = r;
  }
}

// The basis columns are read once per pass and the new column is not read
// again before the next pass: non-temporal loads and stores keep them from
// displacing the stencil's z rows in the caches (measured at 2048^2, seven
// stages: update 341 -> 299 us, dots 274 -> 239 us with four columns per
// block reduction).
//
// bc0 != 0: the s stage blocks of V_0 are equal (the first restart cycle of
// a forward stage system starts from 1 (x) f, block system (3.2)), so block 0 is read
// once and stands for all of them; the arithmetic is unchanged.
template <typename TZ, int S, bool MASS>
__global__ void __launch_bounds__(kBlock)
    k_spmm_dots(OpView<double> K, OpView<double> M, const TZ *__restrict__ z, Mat8 hA,
                const double *__restrict__ V,
                const double *__restrict__ scale, const KrylovState *__restrict__ ks,
                double *__restrict__ partial, int bc0) {
  constexpr int NV = 4;  // columns per block reduction
  const size_t N = (size_t)K.nx * K.ny;
  const size_t sN = (size_t)S * N;
  const size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x;
  const int nblk = gridDim.x;
  const int jj = ks->j;
  double w[S];
  const bool live = p < N;
  if (live) kron_apply<TZ, S, MASS>(K, M, z + (size_t)jj * sN, hA, p, N, w);
  for (int m0 = 0; m0 <= jj; m0 += NV) {
    double acc[NV];
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int m = m0 + u;
      acc[u] = 0.0;
      if (live && m <= jj) {
        const double *Vm = V + (size_t)m * sN;
        if (m == 0 && bc0) {
          const double v0 = __builtin_nontemporal_load(Vm + p);
#pragma unroll
          for (int r = 0; r < S; ++r) acc[u] += v0 * w[r];
        } else {
#pragma unroll
          for (int r = 0; r < S; ++r)
            acc[u] += __builtin_nontemporal_load(Vm + (size_t)r * N + p) * w[r];
        }
        acc[u] *= scale[m];
      }
    }
    block_sums<NV>(acc);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int u = 0; u < NV; ++u)
        if (m0 + u <= jj) partial[(size_t)(m0 + u) * nblk + blockIdx.x] = acc[u];
    }
  }
  // ||w||^2 as column j+1: lets the device decide on a second Gram-Schmidt pass
  double ww = 0.0;
  if (live) {
#pragma unroll
    for (int r = 0; r < S; ++r) ww += w[r] * w[r];
  }
  const double t = block_sum(ww);
  if (threadIdx.x == 0) partial[(size_t)(jj + 1) * nblk + blockIdx.x] = t;
}

template <typename TZ, int S, bool MASS>
__global__ void __launch_bounds__(kBlock)
    k_spmm_update(OpView<double> K, OpView<double> M, const TZ *__restrict__ z, Mat8 hA,
                  const double *__restrict__ V, const double *__restrict__ scale,
                  const double *__restrict__ hcol, const KrylovState *__restrict__ ks,
                  double *__restrict__ Vall, double *__restrict__ partial, int bc0) {
  const size_t N = (size_t)K.nx * K.ny;
  const size_t sN = (size_t)S * N;
  const size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x;
  const int jj = ks->j;
  double val = 0.0;
  if (p < N) {
    double w[S];
    kron_apply<TZ, S, MASS>(K, M, z + (size_t)jj * sN, hA, p, N, w);
    int m = 0;
    if (bc0) {
      const double c = hcol[0] * scale[0];
      const double v0 = __builtin_nontemporal_load(V + p);
#pragma unroll
      for (int r = 0; r < S; ++r) w[r] -= c * v0;
      m = 1;
    }
    for (; m <= jj; ++m) {
      const double c = hcol[m] * scale[m];
      const double *Vm = V + (size_t)m * sN;
#pragma unroll
      for (int r = 0; r < S; ++r) w[r] -= c * __builtin_nontemporal_load(Vm + (size_t)r * N + p);
    }
    double *vout = Vall + (size_t)(jj + 1) * sN;
#pragma unroll
    for (int r = 0; r < S; ++r) {
      __builtin_nontemporal_store(w[r], vout + (size_t)r * N + p);
      val += w[r] * w[r];
    }
  }
  const double t = block_sum(val);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// Second Gram-Schmidt pass on the new column V_{j+1} (elements EPT per thread).
constexpr int kEPT = 4;

__global__ void __launch_bounds__(kBlock)
    k_vec_dots(const double *__restrict__ V, size_t n, const double *__restrict__ scale,
               const KrylovState *__restrict__ ks, double *__restrict__ partial) {
  if (ks->skip_reorth) return;  // uniform over the grid
  const int jj = ks->j;
  const double *vin = V + (size_t)(jj + 1) * n;
  const size_t e0 = ((size_t)blockIdx.x * kBlock + threadIdx.x) * kEPT;
  double x[kEPT];
#pragma unroll
  for (int q = 0; q < kEPT; ++q) x[q] = (e0 + q < n) ? vin[e0 + q] : 0.0;
  const int nblk = gridDim.x;
  for (int m = 0; m <= jj; ++m) {
    const double *Vm = V + (size_t)m * n;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < kEPT; ++q)
      if (e0 + q < n) acc += x[q] * Vm[e0 + q];
    acc *= scale[m];
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partial[(size_t)m * nblk + blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(kBlock)
    k_vec_update(double *__restrict__ V, size_t n, const double *__restrict__ scale,
                 const double *__restrict__ h2, const KrylovState *__restrict__ ks,
                 double *__restrict__ partial) {
  if (ks->skip_reorth) return;
  const int jj = ks->j;
  double *vin = V + (size_t)(jj + 1) * n;
  const size_t e0 = ((size_t)blockIdx.x * kBlock + threadIdx.x) * kEPT;
  double x[kEPT];
#pragma unroll
  for (int q = 0; q < kEPT; ++q) x[q] = (e0 + q < n) ? vin[e0 + q] : 0.0;
  for (int m = 0; m <= jj; ++m) {
    const double c = h2[m] * scale[m];
    const double *Vm = V + (size_t)m * n;
#pragma unroll
    for (int q = 0; q < kEPT; ++q)
      if (e0 + q < n) x[q] -= c * Vm[e0 + q];
  }
  double val = 0.0;
#pragma unroll
  for (int q = 0; q < kEPT; ++q)
    if (e0 + q < n) {
      vin[e0 + q] = x[q];
      val += x[q] * x[q];
    }
  const double t = block_sum(val);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kRed)
    k_reduce_cols(const double *__restrict__ partial, int nblk,
                  const KrylovState *__restrict__ ks, int extra, int honor_skip,
                  double *__restrict__ out) {
  const int m = blockIdx.x;
  if (m > ks->j + extra || (honor_skip && ks->skip_reorth)) return;  // uniform per block
  const double t = sum_partials(partial + (size_t)m * nblk, nblk);
  if (threadIdx.x == 0) out[m] = t;
}

// Decide on the second Gram-Schmidt pass (DGKS criterion): mode 0 never,
// 1 always, 2 when the first pass removed more than half of ||w||^2, i.e.
// ||v|| < ||w|| / sqrt(2).  Also keeps ||v||^2 of the first pass.
__global__ void __launch_bounds__(kRed)
    k_reorth_decide(const double *__restrict__ partial_norm, int nblk,
                    const double *__restrict__ h1, KrylovState *__restrict__ ks, int mode,
                    double *__restrict__ norm_sq) {
  const double nrm2 = sum_partials(partial_norm, nblk);
  if (threadIdx.x != 0) return;
  const double ww = h1[ks->j + 1];
  const bool skip = (mode == 0) || (mode == 2 && nrm2 > 0.5 * ww);
  ks->skip_reorth = skip ? 1 : 0;
  norm_sq[0] = nrm2;
}

// Hessenberg column j: H[:, j] = h1 (+ h2), H[j+1, j] = ||v_{j+1}||, rotate
// with the stored Givens rotations, form the new one, update g and the
// residual estimate |g_{j+1}|, set the lazy scale of V_{j+1}, advance j.
// FIRST_ONLY: no second Gram-Schmidt pass exists, partial_norm holds the
// first pass's partial sums of ||v_{j+1}||^2 and h2 is not read.
static_assert(kMaxKrylov < kRed, "one lane per Krylov column in k_givens");

template <bool FIRST_ONLY>
__global__ void __launch_bounds__(kRed)
    k_givens(const double *__restrict__ h1, const double *__restrict__ h2,
             const double *__restrict__ partial_norm, int nblk,
             const double *__restrict__ norm_sq_first, double *__restrict__ H, int ldh,
             double *__restrict__ cs, double *__restrict__ sn, double *__restrict__ g,
             double *__restrict__ scale, KrylovState *__restrict__ ks, double beta, double rtol,
             double *__restrict__ host_resid) {
  // column inputs are loaded by all lanes at once into LDS, so the serial
  // rotation chain below runs on LDS values instead of dependent global loads
  __shared__ double hc[kMaxKrylov + 1], csl[kMaxKrylov], snl[kMaxKrylov];
  const bool second = !FIRST_ONLY && !ks->skip_reorth;
  const bool sum = FIRST_ONLY || second;
  const int j = ks->j;  // j < kMaxKrylov <= kRed
  const int t = threadIdx.x;
  if (t <= j) {
    hc[t] = h1[t] + (second ? h2[t] : 0.0);
    if (t < j) {
      csl[t] = cs[t];
      snl[t] = sn[t];
    }
  }
  const double nrm2s = sum ? sum_partials(partial_norm, nblk) : 0.0;  // uniform branch
  __syncthreads();
  if (t != 0) return;
  const double nrm2 = sum ? nrm2s : norm_sq_first[0];
  double *Hc = H + (size_t)j * ldh;
  const double nrm = sqrt(nrm2);
  double bb = nrm;  // H[j+1, j] before the rotations
  for (int m = 0; m < j; ++m) {
    const double a = hc[m], b1 = hc[m + 1];
    Hc[m] = csl[m] * a + snl[m] * b1;
    hc[m + 1] = -snl[m] * a + csl[m] * b1;
  }
  const double a = hc[j];
  const double r = hypot(a, bb);
  double c = 1.0, sv = 0.0;
  if (r > 0.0) {
    c = a / r;
    sv = bb / r;
  }
  cs[j] = c;
  sn[j] = sv;
  Hc[j] = r;
  Hc[j + 1] = 0.0;
  const double gj = g[j];
  g[j + 1] = -sv * gj;
  g[j] = c * gj;
  const double res = fabs(g[j + 1]);
  scale[j + 1] = (nrm > 0.0 && isfinite(nrm)) ? 1.0 / nrm : 0.0;
  const bool bad = !isfinite(nrm) || !isfinite(res) || !(r > 0.0);
  ks->breakdown = bad ? 1 : (nrm == 0.0 ? 2 : 0);
  ks->converged = (res <= rtol * beta) ? 1 : 0;
  ks->j = j + 1;
  host_resid[0] = res;
  host_resid[1] = (double)ks->breakdown;
}

__global__ void k_solve_upper(const double *__restrict__ H, int ldh, const double *__restrict__ g,
                              int k, double *__restrict__ y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int r = k - 1; r >= 0; --r) {
    double acc = g[r];
    for (int c = r + 1; c < k; ++c) acc -= H[(size_t)c * ldh + r] * y[c];
    y[r] = acc / H[(size_t)r * ldh + r];
  }
}

template <typename TZ, bool FIRST>
__global__ void __launch_bounds__(kBlock)
    k_accumulate(const TZ *__restrict__ Z, size_t zs, const double *__restrict__ y, int k,
                 size_t n, double *__restrict__ acc) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  double a = FIRST ? 0.0 : acc[e];
  for (int j = 0; j < k; ++j) a += y[j] * double(Z[(size_t)j * zs + e]);
  acc[e] = a;
}

// The same for four consecutive elements per thread (16-byte loads of Z and
// acc): n and zs multiples of 4, Z and acc 16-byte aligned.
template <typename TZ>
struct Vec4;
typedef float NtF4 __attribute__((ext_vector_type(4)));
typedef double NtD2 __attribute__((ext_vector_type(2)));
template <>
struct Vec4<float> {
  __device__ static void load(const float *p, double (&v)[4]) {
    const float4 q = *reinterpret_cast<const float4 *>(p);
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
  }
  // non-temporal: data read once and not again soon
  __device__ static void load_nt(const float *p, double (&v)[4]) {
    const NtF4 q = __builtin_nontemporal_load(reinterpret_cast<const NtF4 *>(p));
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
  }
};
template <>
struct Vec4<double> {
  __device__ static void load(const double *p, double (&v)[4]) {
    const double2 q0 = *reinterpret_cast<const double2 *>(p);
    const double2 q1 = *reinterpret_cast<const double2 *>(p + 2);
    v[0] = q0.x;
    v[1] = q0.y;
    v[2] = q1.x;
    v[3] = q1.y;
  }
  __device__ static void load_nt(const double *p, double (&v)[4]) {
    const NtD2 q0 = __builtin_nontemporal_load(reinterpret_cast<const NtD2 *>(p));
    const NtD2 q1 = __builtin_nontemporal_load(reinterpret_cast<const NtD2 *>(p + 2));
    v[0] = q0.x;
    v[1] = q0.y;
    v[2] = q1.x;
    v[3] = q1.y;
  }
};

template <typename TZ, bool FIRST>
__global__ void __launch_bounds__(kBlock)
    k_accumulate4(const TZ *__restrict__ Z, size_t zs, const double *__restrict__ y, int k,
                  size_t n4, double *__restrict__ acc) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n4) return;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  if (!FIRST) Vec4<double>::load(acc + 4 * e, a);
  for (int j = 0; j < k; ++j) {
    double z[4];
    Vec4<TZ>::load_nt(Z + (size_t)j * zs + 4 * e, z);  // each column read once
    const double yj = y[j];
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] += yj * z[q];
  }
  double2 *out = reinterpret_cast<double2 *>(acc + 4 * e);
  out[0] = make_double2(a[0], a[1]);
  out[1] = make_double2(a[2], a[3]);
}

__global__ void __launch_bounds__(kBlock)
    k_combine(const double *__restrict__ u_in, const double *__restrict__ x, Row8 wts, int s,
              size_t N, double *__restrict__ u_out) {
  const size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= N) return;
  double a = u_in[p];
#pragma unroll
  for (int i = 0; i < kMaxStages; ++i)
    if (i < s) a += wts.c[i] * x[(size_t)i * N + p];
  u_out[p] = a;
}

// u_out (may be null): also u_out = u_in + sum_i wts_i x_i at every node, in
// k_combine's order (the new state, should this residual pass the test).
template <int S, bool MASS>
__global__ void __launch_bounds__(kBlock)
    k_residual_full(OpView<double> K, OpView<double> M, const double *__restrict__ x, Mat8 hA,
                    const double *__restrict__ rhs, const double *__restrict__ f,
                    double *__restrict__ V0, double *__restrict__ partial,
                    const double *__restrict__ u_in, Row8 wts, double *__restrict__ u_out) {
  const size_t N = (size_t)K.nx * K.ny;
  const size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x;
  double val = 0.0;
  if (p < N) {
    double w[S];
    kron_apply<double, S, MASS>(K, M, x, hA, p, N, w);
#pragma unroll
    for (int r = 0; r < S; ++r) {
      const double b = rhs ? rhs[(size_t)r * N + p] : f[p];
      const double res = b - w[r];
      if (V0) V0[(size_t)r * N + p] = res;
      val += res * res;
    }
    if (u_out) {
      double a = u_in[p];
#pragma unroll
      for (int i = 0; i < S; ++i) a += wts.c[i] * x[(size_t)i * N + p];
      u_out[p] = a;
    }
  }
  const double t = block_sum(val);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

template <int S, bool MASS>
__global__ void __launch_bounds__(kBlock)
    k_kron_out(OpView<double> K, OpView<double> M, const double *__restrict__ x, Mat8 hA,
               double *__restrict__ y) {
  const size_t N = (size_t)K.nx * K.ny;
  const size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= N) return;
  double w[S];
  kron_apply<double, S, MASS>(K, M, x, hA, p, N, w);
#pragma unroll
  for (int r = 0; r < S; ++r) y[(size_t)r * N + p] = w[r];
}

__global__ void __launch_bounds__(kBlock)
    k_stage_values(const double *__restrict__ u, const double *__restrict__ k, Mat8 hA, int s,
                   size_t N, double *__restrict__ U) {
  const size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= N) return;
  double kv[kMaxStages];
#pragma unroll
  for (int i = 0; i < kMaxStages; ++i) kv[i] = (i < s) ? k[(size_t)i * N + p] : 0.0;
  const double up = u[p];
#pragma unroll
  for (int i = 0; i < kMaxStages; ++i) {
    if (i >= s) break;
    double a = up;
#pragma unroll
    for (int jx = 0; jx < kMaxStages; ++jx)
      if (jx < s) a += hA.a[i * 8 + jx] * kv[jx];
    U[(size_t)i * N + p] = a;
  }
}

__global__ void __launch_bounds__(kBlock)
    k_adjoint_lambda(OpView<double> K, const double *__restrict__ lam_in,
                     const double *__restrict__ psi, int s, double *__restrict__ lam_out) {
  const size_t N = (size_t)K.nx * K.ny;
  const size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= N) return;
  const int i = (int)(p % K.nx), j = (int)(p / K.nx);
  const int q = node_class_d(i, j, K.nx, K.ny);
  double acc = 0.0;
  for (int t = 0; t < 9; ++t) {
    if (K.npt == 5 && (t == 0 || t == 2 || t == 6 || t == 8)) continue;
    const int xi = i + t % 3 - 1, yj = j + t / 3 - 1;
    if (xi < 0 || xi >= K.nx || yj < 0 || yj >= K.ny) continue;
    const size_t pn = (size_t)yj * K.nx + xi;
    double sp = 0.0;
    for (int st = 0; st < s; ++st) sp += psi[(size_t)st * N + pn];
    acc += coef(K, q, t, p, N) * sp;
  }
  lam_out[p] = lam_in[p] - acc;
}

__global__ void __launch_bounds__(kBlock)
    k_scaled_broadcast(const double *__restrict__ lam, Row8 wts, int s, size_t N,
                       double *__restrict__ rhs) {
  const size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= N) return;
  const double l = lam[p];
  for (int i = 0; i < s; ++i) rhs[(size_t)i * N + p] = wts.c[i] * l;
}

// value of a stage vector at full-grid node (I, J); zero on the boundary.
__device__ __forceinline__ double full_val(const double *v, int I, int J, int nx, int ny) {
  if (I < 1 || I > nx || J < 1 || J > ny) return 0.0;
  return v[(size_t)(J - 1) * nx + (I - 1)];
}

__global__ void __launch_bounds__(kBlock)
    k_grad_nodes(const double *__restrict__ psi, const double *__restrict__ U, int s, int nx,
                 int ny, double inv_h2, double *__restrict__ gnode) {
  const int NX = nx + 2, NY = ny + 2;
  const size_t P = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (P >= (size_t)NX * NY) return;
  const int I = (int)(P % NX), J = (int)(P / NX);
  const size_t N = (size_t)nx * ny;
  double acc = 0.0;
  // faces: east (I,J)-(I+1,J), west (I-1,J)-(I,J) on rows 1..ny;
  //        north (I,J)-(I,J+1), south (I,J-1)-(I,J) on columns 1..nx.
  const int nb[4][2] = {{I + 1, J}, {I - 1, J}, {I, J + 1}, {I, J - 1}};
  for (int f = 0; f < 4; ++f) {
    const int QI = nb[f][0], QJ = nb[f][1];
    const bool horizontal = f < 2;
    if (horizontal) {
      if (J < 1 || J > ny || QI < 0 || QI > nx + 1) continue;
    } else {
      if (I < 1 || I > nx || QJ < 0 || QJ > ny + 1) continue;
    }
    double face = 0.0;
    for (int st = 0; st < s; ++st) {
      const double *ps = psi + (size_t)st * N;
      const double *us = U + (size_t)st * N;
      face += (full_val(ps, I, J, nx, ny) - full_val(ps, QI, QJ, nx, ny)) *
              (full_val(us, I, J, nx, ny) - full_val(us, QI, QJ, nx, ny));
    }
    acc += face;
  }
  gnode[P] += -0.5 * inv_h2 * acc;
}

// One thread per face.  x faces come first (ny rows of nx + 1), then y faces
// (ny + 1 rows of nx); P is the face's node with the smaller full-grid index.
__global__ void __launch_bounds__(kBlock)
    k_grad_faces(const double *__restrict__ psi, const double *__restrict__ U, int s, int nx,
                 int ny, double inv_h2, double *__restrict__ gface) {
  const size_t nfx = (size_t)ny * (nx + 1), nfy = (size_t)(ny + 1) * nx;
  const size_t f = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (f >= nfx + nfy) return;
  int PI, PJ, QI, QJ;
  if (f < nfx) {
    const int i = (int)(f % (nx + 1)), j = (int)(f / (nx + 1));
    PI = i;
    PJ = j + 1;
    QI = i + 1;
    QJ = j + 1;
  } else {
    const size_t g = f - nfx;
    const int i = (int)(g % nx), j = (int)(g / nx);
    PI = i + 1;
    PJ = j;
    QI = i + 1;
    QJ = j + 1;
  }
  const size_t N = (size_t)nx * ny;
  double acc = 0.0;
  for (int st = 0; st < s; ++st) {
    const double *ps = psi + (size_t)st * N;
    const double *us = U + (size_t)st * N;
    acc += (full_val(ps, PI, PJ, nx, ny) - full_val(ps, QI, QJ, nx, ny)) *
           (full_val(us, PI, PJ, nx, ny) - full_val(us, QI, QJ, nx, ny));
  }
  gface[f] += -inv_h2 * acc;
}

__global__ void __launch_bounds__(kBlock)
    k_nonfinite(const double *__restrict__ x, size_t n, double *__restrict__ partial) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  double bad = 0.0;
  if (e < n && !isfinite(x[e])) bad = 1.0;
  const double t = block_sum(bad);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

inline unsigned nblocks(size_t n, size_t per = kBlock) { return (unsigned)((n + per - 1) / per); }

Mat8 pack_mat(const double *hA, int s) {
  Mat8 m{};
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < s; ++j) m.a[i * 8 + j] = hA[i * s + j];
  return m;
}

Row8 pack_row(const double *c, int s) {
  Row8 r{};
  for (int i = 0; i < s; ++i) r.c[i] = c[i];
  return r;
}

}  // namespace

namespace kern {

void rhs_forward(const OpView<double> &K, const double *u, const double *g, int s, double *f,
                 double *V0, double *partial, hipStream_t st) {
  const size_t N = (size_t)K.nx * K.ny;
  k_rhs_forward<<<nblocks(N), kBlock, 0, st>>>(K, u, g, s, f, V0, partial);
}

void rhs_copy(const double *rhs, size_t n, double *V0, double *partial, hipStream_t st) {
  k_rhs_copy<<<nblocks(n), kBlock, 0, st>>>(rhs, n, V0, partial);
}

void finalize_norm(const double *partial, int nblk, double *scale, int col, double *norm_out,
                   hipStream_t st) {
  k_finalize_norm<<<1, kRed, 0, st>>>(partial, nblk, scale, col, norm_out);
}

template <typename T>
void couple(const OpView<T> &K, const double *v, const double *scale_j, const T *z,
            const double *C, int s, int i, T *b, hipStream_t st) {
  const size_t N = (size_t)K.nx * K.ny;
  k_couple<T><<<nblocks(N), kBlock, 0, st>>>(K, v, scale_j, z, pack_row(C, s), s, i, b);
}

#define IRK_DISPATCH_S(s, KERNEL, ...)                     \
  switch (s) {                                             \
    case 1: KERNEL(1, __VA_ARGS__); break;                 \
    case 2: KERNEL(2, __VA_ARGS__); break;                 \
    case 3: KERNEL(3, __VA_ARGS__); break;                 \
    case 4: KERNEL(4, __VA_ARGS__); break;                 \
    case 5: KERNEL(5, __VA_ARGS__); break;                 \
    case 6: KERNEL(6, __VA_ARGS__); break;                 \
    case 7: KERNEL(7, __VA_ARGS__); break;                 \
    default: KERNEL(8, __VA_ARGS__); break;                \
  }

// M == nullptr: the identity mass matrix.
template <typename TZ>
void spmm_dots(const OpView<double> &K, const OpView<double> *M, const TZ *z, const double *hA,
               int s, const double *V, const double *scale, const KrylovState *ks, int jmax,
               double *partial, bool v0_bcast, hipStream_t st) {
  (void)jmax;
  const size_t N = (size_t)K.nx * K.ny;
  const Mat8 m = pack_mat(hA, s);
  const OpView<double> Mv = M ? *M : K;
#define L_SPMM_DOTS(S_, MS_)                                                          \
  k_spmm_dots<TZ, S_, MS_><<<nblocks(N), kBlock, 0, st>>>(K, Mv, z, m, V, scale, ks, \
                                                          partial, v0_bcast ? 1 : 0)
  if (M) {
    IRK_DISPATCH_S(s, L_SPMM_DOTS, true)
  } else {
    IRK_DISPATCH_S(s, L_SPMM_DOTS, false)
  }
#undef L_SPMM_DOTS
}

template <typename TZ>
void spmm_update(const OpView<double> &K, const OpView<double> *M, const TZ *z, const double *hA,
                 int s, const double *V, const double *scale, const double *hcol,
                 const KrylovState *ks, double *vout, double *partial, bool v0_bcast,
                 hipStream_t st) {
  const size_t N = (size_t)K.nx * K.ny;
  const Mat8 m = pack_mat(hA, s);
  const OpView<double> Mv = M ? *M : K;
#define L_SPMM_UPD(S_, MS_)                                                              \
  k_spmm_update<TZ, S_, MS_><<<nblocks(N), kBlock, 0, st>>>(K, Mv, z, m, V, scale, hcol, ks, \
                                                            vout, partial, v0_bcast ? 1 : 0)
  if (M) {
    IRK_DISPATCH_S(s, L_SPMM_UPD, true)
  } else {
    IRK_DISPATCH_S(s, L_SPMM_UPD, false)
  }
#undef L_SPMM_UPD
}

void vec_dots(const double *vin, size_t n, const double *V, const double *scale,
              const KrylovState *ks, int jmax, double *partial, hipStream_t st) {
  (void)vin;
  (void)jmax;
  k_vec_dots<<<nblocks(n, (size_t)kBlock * kEPT), kBlock, 0, st>>>(V, n, scale, ks, partial);
}

void vec_update(double *vin, size_t n, const double *V, const double *scale, const double *h2,
                const KrylovState *ks, double *partial, hipStream_t st) {
  (void)vin;
  k_vec_update<<<nblocks(n, (size_t)kBlock * kEPT), kBlock, 0, st>>>(const_cast<double *>(V), n,
                                                                     scale, h2, ks, partial);
}

void reduce_cols(const double *partial, int nblk, const KrylovState *ks, int jmax, int extra,
                 int honor_skip, double *out, hipStream_t st) {
  k_reduce_cols<<<jmax + 1 + extra, kRed, 0, st>>>(partial, nblk, ks, extra, honor_skip, out);
}

void reorth_decide(const double *partial_norm, int nblk, const double *h1, KrylovState *ks,
                   int mode, double *norm_sq, hipStream_t st) {
  k_reorth_decide<<<1, kRed, 0, st>>>(partial_norm, nblk, h1, ks, mode, norm_sq);
}

void givens(const double *h1, const double *h2, const double *partial_norm, int nblk,
            const double *norm_sq_first, double *H, int ldh, double *cs, double *sn, double *g,
            double *scale, KrylovState *ks, double beta, double rtol, double *host_resid,
            bool first_only, hipStream_t st) {
  if (first_only)
    k_givens<true><<<1, kRed, 0, st>>>(h1, h2, partial_norm, nblk, norm_sq_first, H, ldh, cs,
                                       sn, g, scale, ks, beta, rtol, host_resid);
  else
    k_givens<false><<<1, kRed, 0, st>>>(h1, h2, partial_norm, nblk, norm_sq_first, H, ldh, cs,
                                        sn, g, scale, ks, beta, rtol, host_resid);
}

void solve_upper(const double *H, int ldh, const double *g, int k, double *y, hipStream_t st) {
  k_solve_upper<<<1, 64, 0, st>>>(H, ldh, g, k, y);
}

template <typename TZ>
void accumulate_solution(const TZ *Z, size_t zs, const double *y, int k, size_t n, double *acc,
                         bool first, hipStream_t st) {
  const bool vec = n % 4 == 0 && zs % 4 == 0 && reinterpret_cast<uintptr_t>(Z) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(acc) % 16 == 0;
  if (vec) {
    const size_t n4 = n / 4;
    if (first)
      k_accumulate4<TZ, true><<<nblocks(n4), kBlock, 0, st>>>(Z, zs, y, k, n4, acc);
    else
      k_accumulate4<TZ, false><<<nblocks(n4), kBlock, 0, st>>>(Z, zs, y, k, n4, acc);
  } else if (first) {
    k_accumulate<TZ, true><<<nblocks(n), kBlock, 0, st>>>(Z, zs, y, k, n, acc);
  } else {
    k_accumulate<TZ, false><<<nblocks(n), kBlock, 0, st>>>(Z, zs, y, k, n, acc);
  }
}

void combine_stages(const double *u_in, const double *x, const double *wts, int s, size_t N,
                    double *u_out, hipStream_t st) {
  k_combine<<<nblocks(N), kBlock, 0, st>>>(u_in, x, pack_row(wts, s), s, N, u_out);
}

void residual_full(const OpView<double> &K, const OpView<double> *M, const double *x,
                   const double *hA, int s, const double *rhs, const double *f, double *V0,
                   double *partial, hipStream_t st, const double *u_in, const double *wts,
                   double *u_out) {
  const size_t N = (size_t)K.nx * K.ny;
  const Mat8 m = pack_mat(hA, s);
  const OpView<double> Mv = M ? *M : K;
  const Row8 w = u_out ? pack_row(wts, s) : Row8{};
#define L_RES(S_, MS_)                                                                  \
  k_residual_full<S_, MS_><<<nblocks(N), kBlock, 0, st>>>(K, Mv, x, m, rhs, f, V0, partial, \
                                                          u_in, w, u_out)
  if (M) {
    IRK_DISPATCH_S(s, L_RES, true)
  } else {
    IRK_DISPATCH_S(s, L_RES, false)
  }
#undef L_RES
}

void kron_apply(const OpView<double> &K, const OpView<double> *M, const double *x,
                const double *hA, int s, double *y, hipStream_t st) {
  const size_t N = (size_t)K.nx * K.ny;
  const Mat8 m = pack_mat(hA, s);
  const OpView<double> Mv = M ? *M : K;
#define L_KRON(S_, MS_) k_kron_out<S_, MS_><<<nblocks(N), kBlock, 0, st>>>(K, Mv, x, m, y)
  if (M) {
    IRK_DISPATCH_S(s, L_KRON, true)
  } else {
    IRK_DISPATCH_S(s, L_KRON, false)
  }
#undef L_KRON
}

void stage_values(const double *u, const double *k, const double *hA, int s, size_t N, double *U,
                  hipStream_t st) {
  k_stage_values<<<nblocks(N), kBlock, 0, st>>>(u, k, pack_mat(hA, s), s, N, U);
}

void adjoint_lambda(const OpView<double> &K, const double *lam_in, const double *psi, int s,
                    double *lam_out, hipStream_t st) {
  const size_t N = (size_t)K.nx * K.ny;
  k_adjoint_lambda<<<nblocks(N), kBlock, 0, st>>>(K, lam_in, psi, s, lam_out);
}

void scaled_broadcast(const double *lam, const double *wts, int s, size_t N, double *rhs,
                      hipStream_t st) {
  k_scaled_broadcast<<<nblocks(N), kBlock, 0, st>>>(lam, pack_row(wts, s), s, N, rhs);
}

void grad_nodes(const double *psi, const double *U, int s, int nx, int ny, double inv_h2,
                double *gnode, hipStream_t st) {
  k_grad_nodes<<<nblocks((size_t)(nx + 2) * (ny + 2)), kBlock, 0, st>>>(psi, U, s, nx, ny, inv_h2,
                                                                         gnode);
}

void grad_faces(const double *psi, const double *U, int s, int nx, int ny, double inv_h2,
                double *gface, hipStream_t st) {
  const size_t nf = (size_t)ny * (nx + 1) + (size_t)(ny + 1) * nx;
  k_grad_faces<<<nblocks(nf), kBlock, 0, st>>>(psi, U, s, nx, ny, inv_h2, gface);
}

void nonfinite_check(const double *x, size_t n, double *partial, hipStream_t st) {
  k_nonfinite<<<nblocks(n), kBlock, 0, st>>>(x, n, partial);
}

// explicit instantiations
template void couple<float>(const OpView<float> &, const double *, const double *, const float *,
                            const double *, int, int, float *, hipStream_t);
template void couple<double>(const OpView<double> &, const double *, const double *,
                             const double *, const double *, int, int, double *, hipStream_t);
template void spmm_dots<float>(const OpView<double> &, const OpView<double> *, const float *,
                               const double *, int, const double *, const double *,
                               const KrylovState *, int, double *, bool, hipStream_t);
template void spmm_dots<double>(const OpView<double> &, const OpView<double> *, const double *,
                                const double *, int, const double *, const double *,
                                const KrylovState *, int, double *, bool, hipStream_t);
template void spmm_update<float>(const OpView<double> &, const OpView<double> *, const float *,
                                 const double *, int, const double *, const double *,
                                 const double *, const KrylovState *, double *, double *,
                                 bool, hipStream_t);
template void spmm_update<double>(const OpView<double> &, const OpView<double> *, const double *,
                                  const double *, int, const double *, const double *,
                                  const double *, const KrylovState *, double *, double *,
                                  bool, hipStream_t);
template void accumulate_solution<float>(const float *, size_t, const double *, int, size_t,
                                         double *, bool, hipStream_t);
template void accumulate_solution<double>(const double *, size_t, const double *, int, size_t,
                                          double *, bool, hipStream_t);

}  // namespace kern
}  // namespace irk
