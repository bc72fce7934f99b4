// Host runtime of libirk: setup of the block preconditioner and its AMG
// hierarchy, the flexible GMRES loop, and the C ABI of include/irk.h.
//
// Per Krylov iteration j (right preconditioning, flexible):
//   z_j = P^-1 v_j                 block substitution over the stages
//                                  (Sec. 4.2), one V-cycle per stage block
//   w   = (I + hA (x) K) z_j       Kronecker SpMM, dots with V_0..V_j fused
//   v_{j+1} = w - sum h_mj v_m     classical Gram-Schmidt (+ optional second
//                                  pass), recomputing w instead of storing it
//   Givens update of the Hessenberg column and |g_{j+1}| (single block)
// The residual estimate is read on the host once per iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/irk.h"
#include "host_setup.hpp"
#include "kernels.hpp"

using irk::KrylovState;
using irk::OpView;
using irk::Stencil9;

namespace {

template <typename T>
struct DevOp {
  int nx = 0, ny = 0, npt = 9;
  T *cls = nullptr;
  T *arr = nullptr;
  int uniform = 0;
  T interior[9] = {};  // host copy of the interior class (constant coefficients)
  T classes[81] = {};  // host copy of all nine classes (q * 9 + k)
  T pw = T(0);         // prolongation boundary weight of this level
  T pa = T(0.75), pn = T(0.25);  // parent and next-node weights (linear interpolation)
  T jw = T(0);                   // smoother: 0 red-black Gauss-Seidel, > 0 damped Jacobi weight
  OpView<T> view() const { return OpView<T>{nx, ny, npt, cls, arr, uniform, pw, pa, pn, jw}; }
};

// A constant-coefficient operator is uniform when every boundary class equals
// the interior stencil except for the couplings that leave the grid.
bool classes_uniform(const double cls[9][9]) {
  for (int q = 0; q < 9; ++q)
    for (int k = 0; k < 9; ++k) {
      const int cx = q % 3, cy = q / 3, dx = k % 3 - 1, dy = k / 3 - 1;
      const bool outside =
          (cx == 0 && dx < 0) || (cx == 2 && dx > 0) || (cy == 0 && dy < 0) || (cy == 2 && dy > 0);
      if (!outside && std::fabs(cls[q][k] - cls[4][k]) > 1e-14 * std::fabs(cls[4][4])) return false;
    }
  return true;
}

struct HipError {
  hipError_t e;
  const char *what;
};

#define HIP_TRY(expr)                            \
  do {                                           \
    hipError_t _e = (expr);                      \
    if (_e != hipSuccess) throw HipError{_e, #expr}; \
  } while (0)

}  // namespace

struct irk_solver {
  hipStream_t stream = nullptr;
  int device = 0;  // the HIP device current at setup
  int s = 0, nx = 0, ny = 0;
  size_t N = 0, sN = 0;
  double h = 0.0;
  double A[64] = {}, b[8] = {}, At[64] = {};
  double hA[64] = {}, hAT[64] = {};
  double Cfwd[64] = {}, Cadj[64] = {};
  int ord_fwd[8] = {}, ord_adj[8] = {};
  double tau[8] = {}, hb[8] = {};
  irk_options opt{};
  bool const_mode = false, symmetric = false;
  int nlev = 0, ncoarse = 0;
  int lt = 0;  // first level handled by the single-workgroup tail kernel
  // per stage: the level that ends its V-cycle (pre- and post-smoothing, no
  // coarse correction); nlev - 1 when the cycle reaches the coarsest level
  std::vector<int> cycle_end;
  std::vector<int> lnx, lny;

  // mass matrix (Sec. 3.1: M_kl = integral of phi_k phi_l); none means M = I
  bool has_mass = false;
  Stencil9 Mst;
  DevOp<double> M64;
  OpView<double> Mview{};

  // operators (rebuilt by irk_update_operator)
  Stencil9 Kst;  // host copy of K, kept when the adjoint needs K^T (K not symmetric or M given)
  // the transposed stage system (I (x) M^T + h A^T (x) K^T) psi = r as a stage
  // system of its own (tableau A^T, operators K^T and M^T), set up on the first
  // adjoint step that needs it and dropped when K changes
  irk_solver *adj = nullptr;
  DevOp<double> K64;
  DevOp<float> K32;
  std::vector<std::vector<DevOp<double>>> D64;  // [stage][level]
  std::vector<std::vector<DevOp<float>>> D32;
  std::vector<double *> Cinv64;
  std::vector<float *> Cinv32;
  std::vector<void *> op_allocs;
  // finest level of the blocks for the passes that keep the pre-smoothed x
  // (M = I, five-point K, linear interpolation); fine_mode 0: not used,
  // 1: constant coefficients, 2: K per node
  int fine_mode = 0;
  irk::FineOp<float> fine32;
  irk::FineOp<double> fine64;

  // workspace
  double *V = nullptr, *acc = nullptr, *f = nullptr, *g = nullptr, *rhs = nullptr;
  double *Ubuf = nullptr, *zero = nullptr, *gbuf = nullptr;
  double *partial = nullptr, *pnorm = nullptr, *pnorm2 = nullptr;
  double *H = nullptr, *cs = nullptr, *sn = nullptr, *gv = nullptr, *y = nullptr;
  double *scale = nullptr, *h1 = nullptr, *h2 = nullptr, *norm_dev = nullptr;
  // coherent pinned host memory: {residual estimate, breakdown flag} written
  // by the Givens kernel through host_resid_dev, read by the host after sync
  double *host_resid = nullptr;
  double *host_resid_dev = nullptr;
  void *Z = nullptr;             // m * sN elements of float or double
  void *b0 = nullptr;            // level-0 right-hand side, N elements
  // levels 1.. of b, x and the stored pre-smoothed x (level 0: b0, z and xp0)
  void *levb = nullptr, *levx = nullptr, *levp = nullptr, *xp0 = nullptr;
  double *one = nullptr;  // device constant 1.0
  std::vector<size_t> lev_off;
  KrylovState *ks = nullptr;
  size_t partial_len = 0;
  std::vector<void *> ws_allocs;

  // measurement hook (irk_profile_select / irk_profile_read)
  struct ProfTok {
    hipEvent_t a = nullptr, b = nullptr;
    double bytes = 0.0;
  };
  int prof_sel = -1;
  std::vector<hipEvent_t> prof_pool;
  std::vector<ProfTok> prof_pending;
  long long prof_launches = 0;
  double prof_ms = 0.0, prof_bytes = 0.0;

  // preconditioner applications captured as HIP graphs, one per argument set
  // (Krylov column j of a system); dropped when the operators change
  struct PrecGraph {
    const void *v, *scale, *z, *C, *ord;
    hipGraphExec_t exec;
  };
  std::vector<PrecGraph> graphs;
  hipStream_t cap_stream = nullptr;  // capture only; replays go to `stream`
  long long graph_replays = 0;
  hipEvent_t resid_ev = nullptr;  // recorded after an iteration's residual estimate reaches the host
  bool u_written = false;  // the last converged true-residual pass wrote the step's output

  std::string err;
};

namespace {

size_t elem_size(const irk_solver *S) { return S->opt.precision == IRK_MIXED ? 4 : 8; }

// The V-cycles smooth with damped Jacobi (else red-black Gauss-Seidel).
bool jacobi(const irk_solver *S) { return S->opt.smoother == IRK_SMOOTH_JACOBI; }

using ProfTok = irk_solver::ProfTok;

hipEvent_t prof_event(irk_solver *S) {
  if (!S->prof_pool.empty()) {
    hipEvent_t e = S->prof_pool.back();
    S->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIP_TRY(hipEventCreate(&e));
  return e;
}

// Start timing a launch of kernel class kc (no-op unless kc is selected).
ProfTok prof_begin(irk_solver *S, int kc, double bytes) {
  ProfTok t;
  if (S->prof_sel != kc) return t;
  t.a = prof_event(S);
  t.b = prof_event(S);
  t.bytes = bytes;
  HIP_TRY(hipEventRecord(t.a, S->stream));
  return t;
}

void prof_end(irk_solver *S, const ProfTok &t) {
  if (!t.a) return;
  HIP_TRY(hipEventRecord(t.b, S->stream));
  S->prof_pending.push_back(t);
}

// Resolve the recorded events; call only after the stream has synchronised.
void prof_collect(irk_solver *S) {
  std::vector<ProfTok> keep;
  for (const ProfTok &t : S->prof_pending) {
    if (hipEventQuery(t.b) != hipSuccess) {  // still queued (work enqueued ahead)
      keep.push_back(t);
      continue;
    }
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, t.a, t.b));
    S->prof_ms += ms;
    S->prof_bytes += t.bytes;
    S->prof_launches += 1;
    S->prof_pool.push_back(t.a);
    S->prof_pool.push_back(t.b);
  }
  S->prof_pending.swap(keep);
}

// Coefficient bytes of one pass over a stored operator (0 for a constant one).
double op_bytes(const irk_solver *S, size_t n, int npt, size_t es) {
  return S->const_mode ? 0.0 : (double)n * npt * es;
}

template <typename T>
T *dalloc(std::vector<void *> &list, size_t n) {
  void *p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess) throw HipError{e, "hipMalloc"};
  list.push_back(p);
  return static_cast<T *>(p);
}

template <typename T>
DevOp<T> upload_op(irk_solver *S, const Stencil9 &op, bool use_classes, int npt) {
  DevOp<T> d;
  d.nx = op.nx;
  d.ny = op.ny;
  d.npt = npt;
  if (use_classes) {
    double cls[9][9];
    irk::classify(op, 1e-12, cls);
    d.uniform = classes_uniform(cls) ? 1 : 0;
    std::vector<T> h(81);
    for (int q = 0; q < 9; ++q)
      for (int k = 0; k < 9; ++k) h[q * 9 + k] = (T)cls[q][k];
    for (int k = 0; k < 9; ++k) d.interior[k] = h[4 * 9 + k];
    for (int q = 0; q < 81; ++q) d.classes[q] = h[q];
    d.cls = dalloc<T>(S->op_allocs, 81);
    HIP_TRY(hipMemcpy(d.cls, h.data(), 81 * sizeof(T), hipMemcpyHostToDevice));
  } else {
    const size_t n = op.size();
    std::vector<T> h(9 * n);
    for (int k = 0; k < 9; ++k)
      for (size_t p = 0; p < n; ++p) h[(size_t)k * n + p] = (T)op.c[k][p];
    d.arr = dalloc<T>(S->op_allocs, 9 * n);
    HIP_TRY(hipMemcpy(d.arr, h.data(), 9 * n * sizeof(T), hipMemcpyHostToDevice));
  }
  return d;
}

int stencil_npt(const Stencil9 &op) {
  for (int k : {0, 2, 6, 8})
    for (double v : op.c[k])
      if (v != 0.0) return 9;
  return 5;
}

void free_list(std::vector<void *> &list) {
  for (void *p : list) (void)hipFree(p);
  list.clear();
}

// Transfer weights between level l and l + 1 for the configured interpolation.
irk::Interp interp_of(const irk_solver *S, int l) {
  return S->opt.interp == IRK_INTERP_CONSTANT ? irk::constant_interp() : irk::linear_interp(l);
}

// Build the operators: K (and M) on the fine grid and, for every stage block
// D_i = M + tau_i K (Sec. 4.2), the Galerkin hierarchy S_l + tau_i K_l and the
// dense inverse on the coarsest level.
// Destroy the captured preconditioner graphs (their kernel arguments point at
// the operators being replaced).
void drop_graphs(irk_solver *S) {
  if (S->graphs.empty()) return;
  HIP_TRY(hipStreamSynchronize(S->stream));
  for (const auto &g : S->graphs) (void)hipGraphExecDestroy(g.exec);
  S->graphs.clear();
}

// The finest level for the passes that keep the pre-smoothed x: M = I, a
// five-point K on an even grid, linear interpolation, and a finest level
// handled by the fused passes (not the one-workgroup tail).  Uniform blocks
// keep their interior stencil (FP64 only); otherwise K is packed per node
// (S, W, E, N; centre) in the V-cycle's precision and each block is
// I + tau_i K.
template <typename T>
void fill_fine(irk_solver *S, const Stencil9 &K0, irk::FineOp<T> &F,
               const std::vector<std::vector<DevOp<T>>> &D) {
  F = irk::FineOp<T>{};
  F.nx = S->nx;
  F.ny = S->ny;
  F.pw = (T)interp_of(S, 0).wb;
  if (S->fine_mode == 1) {
    for (int i = 0; i < S->s; ++i) {
      const T *c = D[i][0].interior;
      F.cs[i][0] = c[1];
      F.cs[i][1] = c[3];
      F.cs[i][2] = c[4];
      F.cs[i][3] = c[5];
      F.cs[i][4] = c[7];
    }
    return;
  }
  const size_t n = (size_t)S->nx * S->ny;
  std::vector<T> q(4 * n), c(n);
  for (size_t p = 0; p < n; ++p) {
    q[4 * p + 0] = (T)K0.c[1][p];
    q[4 * p + 1] = (T)K0.c[3][p];
    q[4 * p + 2] = (T)K0.c[5][p];
    q[4 * p + 3] = (T)K0.c[7][p];
    c[p] = (T)K0.c[4][p];
  }
  T *dq = dalloc<T>(S->op_allocs, 4 * n);
  T *dc = dalloc<T>(S->op_allocs, n);
  HIP_TRY(hipMemcpy(dq, q.data(), 4 * n * sizeof(T), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(dc, c.data(), n * sizeof(T), hipMemcpyHostToDevice));
  F.kq = dq;
  F.kc = dc;
  for (int i = 0; i < S->s; ++i) F.tau[i] = (T)S->tau[i];
}

void build_fine(irk_solver *S, const Stencil9 &K0, int npt0) {
  S->fine_mode = 0;
  const bool mixed = S->opt.precision == IRK_MIXED;
  if (S->has_mass || npt0 != 5 || S->nx % 2 || S->ny % 2 || S->lt < 1 ||
      S->opt.interp != IRK_INTERP_LINEAR)
    return;
  const bool uniform = mixed ? (S->D32[0][0].uniform && S->D32[0][0].cls)
                             : (S->D64[0][0].uniform && S->D64[0][0].cls);
  if (uniform && S->K64.uniform && S->K64.cls) {
    // FP32 constant coefficients: the split kernels that repeat the
    // pre-smoothing in the up pass move fewer bytes and are faster there
    // (2048^2 heat, seven stages, event-timed per step: down 0.93 against
    // 1.11 ms, up 1.22 against 1.44 ms)
    if (mixed) return;
    S->fine_mode = 1;
  } else if (S->K64.arr) {
    S->fine_mode = 2;
  } else {
    return;
  }
  if (mixed)
    fill_fine<float>(S, K0, S->fine32, S->D32);
  else
    fill_fine<double>(S, K0, S->fine64, S->D64);
}

irk_status build_operators(irk_solver *S, const irk_csr *K) {
  drop_graphs(S);
  Stencil9 K0;
  if (!irk::csr_to_stencil(K->n, K->rowptr, K->colind, K->val, S->nx, S->ny, K0, S->err))
    return IRK_E_INVALID;
  S->symmetric = irk::is_symmetric(K0, 1e-13);
  S->Kst = (S->symmetric && !S->has_mass) ? Stencil9{} : K0;
  // hierarchy of S_l = R S_{l-1} P (S_0 = M) and K_l = R K_{l-1} P
  std::vector<Stencil9> Sl, Kl;
  Sl.push_back(S->has_mass ? S->Mst : irk::identity_stencil(S->nx, S->ny));
  Kl.push_back(K0);
  while ((long long)Sl.back().nx * Sl.back().ny > S->opt.coarse_max && Sl.back().nx % 2 == 0 &&
         Sl.back().ny % 2 == 0 && Sl.back().nx >= 2 && Sl.back().ny >= 2) {
    const irk::Interp ip = interp_of(S, (int)Sl.size() - 1);
    Sl.push_back(irk::galerkin(Sl.back(), ip));
    Kl.push_back(irk::galerkin(Kl.back(), ip));
  }
  const int L = (int)Sl.size();
  const long long ncoarse = (long long)Sl.back().nx * Sl.back().ny;
  if (ncoarse > irk::kTailMaxCoarse) {
    S->err = "the grid does not coarsen to at most 1024 unknowns by halving (nx, ny must stay "
             "even down to coarse_max)";
    return IRK_E_INVALID;
  }
  bool cm = true;
  double tmp[9][9];
  for (int l = 0; l < L && cm; ++l) cm = irk::classify(Sl[l], 1e-12, tmp) && irk::classify(Kl[l], 1e-12, tmp);
  S->const_mode = cm;
  S->nlev = L;
  // end of each block's cycle: the first level with tau_i max_p (K_l)_pp /
  // (S_l)_pp <= coarse_ratio
  S->cycle_end.assign(S->s, L - 1);
  if (S->opt.coarse_ratio > 0.0) {
    std::vector<double> ratio(L, 0.0);
    for (int l = 0; l + 1 < L; ++l) {
      const size_t n = (size_t)Sl[l].nx * Sl[l].ny;
      for (size_t q = 0; q < n; ++q) {
        const double sd = Sl[l].c[4][q], kd = Kl[l].c[4][q];
        ratio[l] = sd > 0.0 ? std::max(ratio[l], kd / sd) : INFINITY;
      }
    }
    for (int i = 0; i < S->s; ++i) {
      if (!(S->tau[i] > 0.0)) continue;
      for (int l = 0; l + 1 < L; ++l)
        if (S->tau[i] * ratio[l] <= S->opt.coarse_ratio) {
          S->cycle_end[i] = l;
          break;
        }
    }
  }
  S->ncoarse = (int)ncoarse;
  S->lnx.clear();
  S->lny.clear();
  for (int l = 0; l < L; ++l) {
    S->lnx.push_back(Sl[l].nx);
    S->lny.push_back(Sl[l].ny);
  }
  // the tail starts at the first level that fits one workgroup's LDS (the
  // device's limit per workgroup: 160 KiB on gfx950; 64 KiB if unknown)
  {
    const size_t es = (S->opt.precision == IRK_MIXED) ? 4 : 8;
    int dev = 0, lds = 0;
    size_t lds_max = 65536;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        lds > 65536)
      lds_max = (size_t)lds;
    S->lt = L - 1;
    for (int l = 0; l < L; ++l) {
      size_t words = 1024 + 81 * (size_t)(L - l);  // reduction buffer + class tables
      for (int m = l; m < L; ++m) words += 2 * (size_t)Sl[m].nx * Sl[m].ny;
      if ((size_t)Sl[l].nx * Sl[l].ny <= (size_t)irk::kTailMax && words * es <= lds_max &&
          L - l <= irk::kTailLevels) {
        S->lt = l;
        break;
      }
    }
  }
  free_list(S->op_allocs);
  S->D64.assign(S->s, {});
  S->D32.assign(S->s, {});
  S->Cinv64.assign(S->s, nullptr);
  S->Cinv32.assign(S->s, nullptr);
  const bool mixed = S->opt.precision == IRK_MIXED;
  const int npt0 = stencil_npt(K0);
  S->K64 = upload_op<double>(S, K0, cm, npt0);
  if (S->has_mass) {
    double tmpm[9][9];
    S->M64 = upload_op<double>(S, S->Mst, irk::classify(S->Mst, 1e-12, tmpm),
                               stencil_npt(S->Mst));
    S->Mview = S->M64.view();
  }
  if (mixed) S->K32 = upload_op<float>(S, K0, cm, npt0);
  for (int i = 0; i < S->s; ++i) {
    for (int l = 0; l + 1 < L; ++l) {
      Stencil9 D = irk::axpy_stencil(Sl[l], S->tau[i], Kl[l]);
      const int npt = stencil_npt(D);
      const irk::Interp ip = interp_of(S, l);
      const double jw = S->opt.smoother == IRK_SMOOTH_JACOBI ? S->opt.jacobi_omega : 0.0;
      if (mixed) {
        S->D32[i].push_back(upload_op<float>(S, D, cm, npt));
        DevOp<float> &d = S->D32[i].back();
        d.pw = (float)ip.wb;
        d.pa = (float)ip.own;
        d.pn = (float)ip.nb;
        d.jw = (float)jw;
      } else {
        S->D64[i].push_back(upload_op<double>(S, D, cm, npt));
        DevOp<double> &d = S->D64[i].back();
        d.pw = ip.wb;
        d.pa = ip.own;
        d.pn = ip.nb;
        d.jw = jw;
      }
    }
    Stencil9 Dc = irk::axpy_stencil(Sl[L - 1], S->tau[i], Kl[L - 1]);
    std::vector<double> inv;
    if (!irk::dense_inverse(Dc, inv)) {
      S->err = "singular coarsest-level block";
      return IRK_E_INVALID;
    }
    // stored transposed: the tail kernel reads column c of the inverse contiguously
    const size_t nn = inv.size();
    const size_t nc = (size_t)ncoarse;
    for (size_t r = 0; r < nc; ++r)
      for (size_t c = r + 1; c < nc; ++c) std::swap(inv[r * nc + c], inv[c * nc + r]);
    if (mixed) {
      std::vector<float> hf(inv.begin(), inv.end());
      S->Cinv32[i] = dalloc<float>(S->op_allocs, nn);
      HIP_TRY(hipMemcpy(S->Cinv32[i], hf.data(), nn * sizeof(float), hipMemcpyHostToDevice));
    } else {
      S->Cinv64[i] = dalloc<double>(S->op_allocs, nn);
      HIP_TRY(hipMemcpy(S->Cinv64[i], inv.data(), nn * sizeof(double), hipMemcpyHostToDevice));
    }
  }
  build_fine(S, K0, npt0);
  return IRK_OK;
}

void alloc_workspace(irk_solver *S) {
  const int m = S->opt.restart;
  const size_t N = S->N, sN = S->sN;
  auto &L = S->ws_allocs;
  S->V = dalloc<double>(L, (size_t)(m + 1) * sN);
  S->Z = (S->opt.precision == IRK_MIXED) ? (void *)dalloc<float>(L, (size_t)m * sN)
                                         : (void *)dalloc<double>(L, (size_t)m * sN);
  S->acc = dalloc<double>(L, sN);
  S->rhs = dalloc<double>(L, sN);
  S->f = dalloc<double>(L, N);
  S->g = nullptr;
  S->zero = dalloc<double>(L, sN);
  {
    S->one = dalloc<double>(L, 1);
    const double one = 1.0;
    HIP_TRY(hipMemcpy(S->one, &one, sizeof one, hipMemcpyHostToDevice));
  }
  HIP_TRY(hipMemset(S->zero, 0, sN * sizeof(double)));
  const size_t nblk_pt = (N + irk::kBlock - 1) / irk::kBlock;
  const size_t nblk_vec = (sN + irk::kBlock * 4 - 1) / (irk::kBlock * 4);
  const size_t nblk_full = (sN + irk::kBlock - 1) / irk::kBlock;
  S->partial_len = std::max({(size_t)(m + 2) * std::max(nblk_pt, nblk_vec), nblk_full,
                             (size_t)((S->nx + 2) * (size_t)(S->ny + 2) / irk::kBlock + 2)});
  S->partial = dalloc<double>(L, S->partial_len);
  S->pnorm = dalloc<double>(L, std::max({nblk_pt, nblk_vec, nblk_full}));
  S->pnorm2 = dalloc<double>(L, std::max({nblk_pt, nblk_vec, nblk_full}));
  S->H = dalloc<double>(L, (size_t)(m + 1) * m);
  S->cs = dalloc<double>(L, m + 1);
  S->sn = dalloc<double>(L, m + 1);
  S->gv = dalloc<double>(L, m + 2);
  S->y = dalloc<double>(L, m + 1);
  S->scale = dalloc<double>(L, m + 2);
  S->h1 = dalloc<double>(L, m + 2);
  S->h2 = dalloc<double>(L, m + 2);
  S->norm_dev = dalloc<double>(L, 2);
  S->ks = dalloc<KrylovState>(L, 1);
  const size_t es = elem_size(S);
  S->b0 = dalloc<char>(L, N * es);
  size_t tot = 0;
  S->lev_off.assign(S->nlev + 1, 0);
  for (int l = 1; l < S->nlev; ++l) {
    S->lev_off[l] = tot;
    tot += (size_t)S->lnx[l] * S->lny[l];
  }
  S->levb = dalloc<char>(L, (tot + 1) * es);
  S->levx = dalloc<char>(L, (tot + 1) * es);
  S->levp = dalloc<char>(L, (tot + 1) * es);
  S->xp0 = dalloc<char>(L, N * es);  // level 0 is not in the level buffers
  void *hp = nullptr;
  HIP_TRY(hipHostMalloc(&hp, 4 * sizeof(double), hipHostMallocCoherent | hipHostMallocMapped));
  S->host_resid = static_cast<double *>(hp);
  void *dp = nullptr;
  HIP_TRY(hipHostGetDevicePointer(&dp, hp, 0));
  S->host_resid_dev = static_cast<double *>(dp);
  HIP_TRY(hipEventCreateWithFlags(&S->resid_ev, hipEventDisableTiming));
}

template <typename T>
const std::vector<std::vector<DevOp<T>>> &Dops(const irk_solver *S);
template <>
const std::vector<std::vector<DevOp<double>>> &Dops<double>(const irk_solver *S) {
  return S->D64;
}
template <>
const std::vector<std::vector<DevOp<float>>> &Dops<float>(const irk_solver *S) {
  return S->D32;
}
template <typename T>
const T *Cinv(const irk_solver *S, int i);
template <>
const double *Cinv<double>(const irk_solver *S, int i) {
  return S->Cinv64[i];
}
template <>
const float *Cinv<float>(const irk_solver *S, int i) {
  return S->Cinv32[i];
}
template <typename T>
OpView<T> Kview(const irk_solver *S);
template <>
OpView<double> Kview<double>(const irk_solver *S) {
  return S->K64.view();
}

// The mass operator for the Kronecker products, or nullptr for M = I.
const OpView<double> *mass(const irk_solver *S) { return S->has_mass ? &S->Mview : nullptr; }
template <>
OpView<float> Kview<float>(const irk_solver *S) {
  return S->K32.view();
}

template <typename T>
const DevOp<T> &Kdev(const irk_solver *S);
template <>
const DevOp<double> &Kdev<double>(const irk_solver *S) {
  return S->K64;
}
template <>
const DevOp<float> &Kdev<float>(const irk_solver *S) {
  return S->K32;
}

template <typename T>
T *lev_b(irk_solver *S, int l) {
  return static_cast<T *>(S->levb) + S->lev_off[l];
}
template <typename T>
T *lev_x(irk_solver *S, int l) {
  return static_cast<T *>(S->levx) + S->lev_off[l];
}
template <typename T>
T *lev_p(irk_solver *S, int l) {
  return l == 0 ? static_cast<T *>(S->xp0) : static_cast<T *>(S->levp) + S->lev_off[l];
}

template <typename T>
const irk::FineOp<T> &fine_op(const irk_solver *S);
template <>
const irk::FineOp<float> &fine_op<float>(const irk_solver *S) {
  return S->fine32;
}
template <>
const irk::FineOp<double> &fine_op<double>(const irk_solver *S) {
  return S->fine64;
}

// Fused down / up passes of one level: two columns per lane for FP32 uniform
// five-point and FP32 constant-coefficient nine-point operators, one column
// per lane for other five-point operators, LDS tiles for the rest.
template <typename T>
bool linear_p(const DevOp<T> &D) {
  return D.pa == T(0.75) && D.pn == T(0.25);
}

template <typename T>
bool split_ok(const DevOp<T> &D) {
  if constexpr (std::is_same_v<T, float>)
    return linear_p(D) && irk::kern::wsplit_ok(D.view());
  else
    return false;
}

// The nine-point register kernels have the linear interpolation built in.
template <typename T>
bool ws9_usable(const DevOp<T> &D, int nu) {
  return linear_p(D) && irk::kern::ws9_ok<T>(D.view(), nu);
}

// Levels l and l + 1 (both intermediate: the finest level and the tail have
// kernels of their own) run as one pair in each direction.
// In FP64 a pair whose fine level is large runs slower than its two levels
// apart (the pair kernels spill, and the fine tiles of a pair overlap more):
// 1024^2 + 512^2 takes 23.0 + 21.1 us against about 16.5 + 18.5, while
// 256^2 + 128^2 takes 8.9 + 15.1 against about 15.5 + 17.5.
constexpr long long kPairMaxFine64 = 256 * 256;

template <typename T>
bool pair_ok(const irk_solver *S, int i, int l) {
  if (!S->opt.fuse_levels || jacobi(S) || l < 1) return false;
  const DevOp<T> &Df = Dops<T>(S)[i][l];
  const DevOp<T> &Dc = Dops<T>(S)[i][l + 1];
  if (std::is_same_v<T, double> && (long long)Df.nx * Df.ny > kPairMaxFine64) return false;
  return linear_p(Df) && linear_p(Dc) &&
         irk::kern::s9pair_ok<T>(Df.view(), Dc.view(), S->opt.nu_pre);
}

// The one-pass smoothing of a cycle's last level (red-black, linear
// interpolation, nine-point classes).
template <typename T>
bool smooth_ok(const irk_solver *S, int i, int l) {
  if (!S->opt.fuse_levels || jacobi(S) || l < 1) return false;
  const DevOp<T> &D = Dops<T>(S)[i][l];
  return linear_p(D) && irk::kern::s9smooth_ok<T>(D.view(), S->opt.nu_pre);
}

template <typename T>
void down_pass(const DevOp<T> &D, int nu, const T *b, T *rc, T *xpre, hipStream_t st) {
  if (D.jw > T(0)) return irk::kern::vdown<T>(D.view(), nu, b, rc, st);  // damped Jacobi
  if constexpr (std::is_same_v<T, float>) {
    if (split_ok(D)) return irk::kern::sdown(D.view(), D.interior, nu, b, rc, st);
  }
  if (ws9_usable<T>(D, nu)) return irk::kern::s9down<T>(D.view(), D.classes, nu, b, rc, xpre, st);
  if (irk::kern::wtile_ok<T>(D.view()))
    irk::kern::wdown<T>(D.view(), nu, b, rc, st);
  else
    irk::kern::vdown<T>(D.view(), nu, b, rc, st);
}

template <typename T>
void up_pass(const DevOp<T> &D, int nu, const T *b, const T *ec, const T *xpre, T *x,
             hipStream_t st) {
  if (D.jw > T(0)) return irk::kern::vup<T>(D.view(), nu, b, ec, x, st);  // damped Jacobi
  if constexpr (std::is_same_v<T, float>) {
    if (split_ok(D)) return irk::kern::sup(D.view(), D.interior, nu, b, ec, x, st);
  }
  if (ws9_usable<T>(D, nu))
    return irk::kern::s9up<T>(D.view(), D.classes, nu, b, ec, xpre, x, st);
  if (irk::kern::wtile_ok<T>(D.view()))
    irk::kern::wup<T>(D.view(), nu, b, ec, x, st);
  else
    irk::kern::vup<T>(D.view(), nu, b, ec, x, st);
}

// One V(nu, nu)-cycle for the stage-i block, x ~= D_i^-1 b on the finest
// level (Sec. 4.2): fused down passes to the tail level, the tail in one
// workgroup, fused up passes back.  The cycle ends at level E = cycle_end[i]:
// E takes its smoothing with a zero coarse correction (an up pass from the
// zero vector, or a tail whose coarsest level returns zero).
// v0 (a block without coupling terms, finest level on the FP32 split passes
// or on the passes that keep the pre-smoothed x: FP64 constant coefficients,
// or K per node in either precision): the finest level's right-hand side is
// *v0scale * v0 rounded to T, formed by its passes on load.
template <typename T>
void vcycle(irk_solver *S, int i, const T *b, T *x, bool finest_down_done,
            const double *v0 = nullptr, const double *v0scale = nullptr) {
  hipStream_t st = S->stream;
  const int nu = S->opt.nu_pre, L = S->nlev;
  const int E = S->cycle_end[i];
  const bool ends = E < L - 1;          // the cycle stops above the coarsest level
  const bool tail = E >= S->lt;         // ... at or below the tail's first level
  const int lt = tail ? S->lt : E + 1;  // levels run by the fused passes: 0 .. lt-1
  const int Lt = ends ? E + 2 : L;      // tail levels lt .. Lt-1; if ends, Lt-1 returns zero
  const size_t es = sizeof(T);
  auto bl = [&](int l) -> const T * { return l == 0 ? b : lev_b<T>(S, l); };
  auto xl = [&](int l) -> T * { return l == 0 ? x : lev_x<T>(S, l); };
  const T *zero = reinterpret_cast<const T *>(S->zero);
  for (int l = finest_down_done ? 1 : 0; l < lt; ++l) {
    const DevOp<T> &D = Dops<T>(S)[i][l];
    const size_t n = (size_t)D.nx * D.ny;
    if (l > 0 && l + 1 < lt && pair_ok<T>(S, i, l)) {
      // levels l and l + 1 in one launch
      const DevOp<T> &Dc = Dops<T>(S)[i][l + 1];
      const size_t nc = (size_t)Dc.nx * Dc.ny;
      ProfTok t = prof_begin(S, IRK_KC_VMID_DOWN, (double)(n + nc) * es * 1.25);
      irk::kern::s9down2<T>(D.view(), D.classes, Dc.view(), Dc.classes, bl(l), lev_p<T>(S, l),
                            lev_b<T>(S, l + 1), lev_p<T>(S, l + 1), lev_b<T>(S, l + 2), st);
      prof_end(S, t);
      ++l;
      continue;
    }
    if (l == 0 && S->fine_mode && !jacobi(S)) {
      // b (or v_0 in FP64) and K per node (read) in, the coarse residual and
      // the pre-smoothed x out
      const double kb = S->fine_mode == 2 ? (double)n * 5 * es : 0.0;
      ProfTok t = prof_begin(S, IRK_KC_VDOWN_L0,
                             (double)n * (v0 ? 8.0 + es * 1.25 : es * 2.25) + kb);
      irk::kern::fdown<T>(fine_op<T>(S), i, nu, b, lev_b<T>(S, 1), lev_p<T>(S, 0), st, v0,
                          v0scale);
      prof_end(S, t);
      continue;
    }
    ProfTok t = prof_begin(S, l == 0 ? IRK_KC_VDOWN_L0 : IRK_KC_VMID_DOWN,
                           (double)n * (l == 0 && v0 ? 8.0 + es * 0.25 : es * 1.25) +
                               op_bytes(S, n, D.npt, es));
    if constexpr (std::is_same_v<T, float>) {
      if (l == 0 && v0)
        irk::kern::sdown_v(D.view(), D.interior, nu, v0, v0scale, lev_b<T>(S, 1), st);
      else
        down_pass<T>(D, nu, bl(l), lev_b<T>(S, l + 1), lev_p<T>(S, l), st);
    } else {
      down_pass<T>(D, nu, bl(l), lev_b<T>(S, l + 1), lev_p<T>(S, l), st);
    }
    prof_end(S, t);
  }
  if (tail && ends && E == S->lt && smooth_ok<T>(S, i, E)) {
    // the cycle ends on the tail's first level: its smoothing alone, on many
    // workgroups instead of the one-workgroup tail
    const DevOp<T> &D = Dops<T>(S)[i][E];
    const size_t n = (size_t)D.nx * D.ny;
    ProfTok t = prof_begin(S, IRK_KC_VTAIL, (double)n * es * 2.0);
    irk::kern::s9smooth<T>(D.view(), D.classes, bl(E), xl(E), st);
    prof_end(S, t);
  } else if (tail) {
    irk::TailDesc<T> td{};
    td.nlev = Lt - lt;
    size_t off = 0, words = 0;
    for (int k = 0; k < td.nlev; ++k) {
      const int l = lt + k;
      td.nx[k] = S->lnx[l];
      td.ny[k] = S->lny[l];
      td.off[k] = off;
      off += 2 * (size_t)S->lnx[l] * S->lny[l];
      if (l < Lt - 1) {
        const DevOp<T> &D = Dops<T>(S)[i][l];
        td.cls[k] = D.cls;
        td.arr[k] = D.arr;
        td.pw[k] = D.pw;
        td.pa = D.pa;
        td.pn = D.pn;
        if (D.arr) words += 9 * (size_t)D.nx * D.ny;
      }
    }
    td.off[td.nlev] = off;
    // a cycle that ends inside the tail: its coarsest level returns zero
    td.CinvT = ends ? nullptr : Cinv<T>(S, i);
    td.jw = jacobi(S) ? (T)S->opt.jacobi_omega : T(0);
    const size_t ntop = (size_t)S->lnx[lt] * S->lny[lt];
    words += 2 * ntop + (ends ? 0 : (size_t)S->ncoarse * S->ncoarse);
    ProfTok t = prof_begin(S, IRK_KC_VTAIL, (double)words * es);
    bool done = false;
    if constexpr (std::is_same_v<T, float>) {
      if (!jacobi(S) && irk::kern::vtail2_ok(td)) {
        irk::kern::vtail2(td, nu, bl(lt), xl(lt), st);
        done = true;
      }
    }
    if (!done) irk::kern::vtail<T>(td, nu, bl(lt), xl(lt), st);
    prof_end(S, t);
  }
  for (int l = lt - 1; l >= 0; --l) {
    const DevOp<T> &D = Dops<T>(S)[i][l];
    const size_t n = (size_t)D.nx * D.ny;
    if (l > 1 && pair_ok<T>(S, i, l - 1)) {
      // levels l and l - 1 in one launch: l's x stays on chip
      const DevOp<T> &Df = Dops<T>(S)[i][l - 1];
      const size_t nf = (size_t)Df.nx * Df.ny;
      ProfTok t = prof_begin(S, IRK_KC_VMID_UP, (double)(n + nf) * es * 2.25);
      irk::kern::s9up2<T>(Df.view(), Df.classes, D.view(), D.classes, bl(l - 1),
                          lev_p<T>(S, l - 1), bl(l), lev_p<T>(S, l),
                          l == E ? zero : lev_x<T>(S, l + 1), xl(l - 1), st);
      prof_end(S, t);
      --l;
      continue;
    }
    if (l == 0 && S->fine_mode && !jacobi(S)) {
      // b (or v_0 in FP64), the pre-smoothed x, K per node and the coarse
      // correction in, x out
      const double kb = S->fine_mode == 2 ? (double)n * 5 * es : 0.0;
      ProfTok t = prof_begin(S, IRK_KC_VUP_L0,
                             (double)n * (v0 ? 8.0 + es * 2.25 : es * 3.25) + kb);
      const T *ec0 = l == E ? zero : lev_x<T>(S, 1);
      irk::kern::fup<T>(fine_op<T>(S), i, nu, b, lev_p<T>(S, 0), ec0, x, st, v0, v0scale);
      prof_end(S, t);
      continue;
    }
    ProfTok t = prof_begin(S, l == 0 ? IRK_KC_VUP_L0 : IRK_KC_VMID_UP,
                           (double)n * (l == 0 && v0 ? 8.0 + es * 1.25 : es * 2.25) +
                               op_bytes(S, n, D.npt, es));
    const T *ec = l == E ? zero : lev_x<T>(S, l + 1);
    if constexpr (std::is_same_v<T, float>) {
      if (l == 0 && v0)
        irk::kern::sup_v(D.view(), D.interior, nu, v0, v0scale, ec, xl(l), st);
      else
        up_pass<T>(D, nu, bl(l), ec, lev_p<T>(S, l), xl(l), st);
    } else {
      up_pass<T>(D, nu, bl(l), ec, lev_p<T>(S, l), xl(l), st);
    }
    prof_end(S, t);
  }
}

// The stage coupling as a streaming pass of its own (uniform five-point K,
// FP64 arithmetic): b0 = scale_j v_i - K (sum_k C[k] z_k).
template <typename T>
void couple_split(irk_solver *S, const double *v, const double *scale_j, const T *z,
                  const double *Crow, int i) {
  irk::kern::scouple<T>(S->nx, S->ny, S->K64.interior, v, scale_j, z, Crow, S->s, i,
                        static_cast<T *>(S->b0), S->stream);
}

// K suits the streaming coupling pass: uniform five-point, even dimensions.
bool kcouple_ok(const irk_solver *S) {
  const OpView<double> k = S->K64.view();
  return k.npt == 5 && k.uniform && k.cls && k.nx % 2 == 0 && k.ny % 2 == 0;
}

// z = P^-1 v by block substitution (Sec. 4.2).  v = V_j (lazy scale
// scale[j]), z = Z_j.  C holds h A~ without its diagonal, ord the stage order.
template <typename T>
void apply_precond(irk_solver *S, const double *v, const double *scale_j, T *z, const double *C,
                   const int *ord) {
  T *b0 = static_cast<T *>(S->b0);
  const size_t N = S->N, es = sizeof(T);
  for (int t = 0; t < S->s; ++t) {
    const int i = ord[t];
    int ncoup = 0;
    for (int k = 0; k < S->s; ++k) ncoup += (C[(size_t)i * S->s + k] != 0.0);
    // v_i (double), the coupled z_k and the right-hand side b
    const double cbytes = (double)N * (8.0 + es * (ncoup + 1)) +
                          (ncoup ? op_bytes(S, N, S->K64.npt, es) : 0.0);
    const DevOp<T> *D0 = S->lt > 0 ? &Dops<T>(S)[i][0] : nullptr;
    bool ws9_0 = false;  // FP32 nine-point constant-coefficient finest level (M != I)
    if constexpr (std::is_same_v<T, float>)
      ws9_0 = D0 && !split_ok<T>(*D0) && ws9_usable<T>(*D0, S->opt.nu_pre);
    const bool split64 = std::is_same_v<T, double> && D0 && kcouple_ok(S);
    if (ncoup == 0 && D0 && !jacobi(S) && S->fine_mode == 2) {
      // no coupling terms: the finest passes (K per node) form scale_j v_i
      // on load
      vcycle<T>(S, i, nullptr, z + (size_t)i * N, false, v + (size_t)i * N, scale_j);
    } else if (S->fine_mode == 2) {
      // K per node: the streaming coupling pass reads K's FP64 arrays
      const double vbytes = (double)N * (8.0 + es * (ncoup + 1)) + (ncoup ? (double)N * 5 * 8 : 0.0);
      ProfTok tk = prof_begin(S, IRK_KC_COUPLE, vbytes);
      irk::kern::scouple_var<T>(S->nx, S->ny, S->K64.arr, v, scale_j, z, C + (size_t)i * S->s,
                                S->s, i, b0, S->stream);
      prof_end(S, tk);
      vcycle<T>(S, i, b0, z + (size_t)i * N, false);
    } else if (ncoup == 0 && D0 && !jacobi(S) &&
               ((std::is_same_v<T, float> && split_ok<T>(*D0) && !S->fine_mode) ||
                (std::is_same_v<T, double> && S->fine_mode == 1))) {
      // no coupling terms: the finest passes form scale_j v_i (rounded to the
      // V-cycle's precision) on load
      vcycle<T>(S, i, nullptr, z + (size_t)i * N, false, v + (size_t)i * N, scale_j);
    } else if ((S->fine_mode == 1 && kcouple_ok(S)) ||
               (D0 && split_ok<T>(*D0) && split_ok<T>(Kdev<T>(S))) || split64) {
      // streaming coupling pass, then the plain V-cycle (FP32: two columns per
      // lane on the finest level)
      ProfTok tk = prof_begin(S, IRK_KC_COUPLE, cbytes);
      couple_split<T>(S, v, scale_j, z, C + (size_t)i * S->s, i);
      prof_end(S, tk);
      vcycle<T>(S, i, b0, z + (size_t)i * N, false);
    } else if (D0 && !ws9_0 && !std::is_same_v<T, double> && !jacobi(S)) {
      // coupling fused into the finest-level down pass (+ rc = R(b - D x))
      const DevOp<T> &D = *D0;
      ProfTok tk = prof_begin(S, IRK_KC_VDOWN_L0,
                              cbytes + (double)N * es * 0.25 + op_bytes(S, N, D.npt, es));
      if (irk::kern::wtile_ok<T>(D.view()) && irk::kern::wtile_ok<T>(Kview<T>(S)))
        irk::kern::wdown_couple<T>(D.view(), Kview<T>(S), S->opt.nu_pre, v, scale_j, z,
                                   C + (size_t)i * S->s, S->s, i, b0, lev_b<T>(S, 1), S->stream);
      else
        irk::kern::vdown_couple<T>(D.view(), Kview<T>(S), S->opt.nu_pre, v, scale_j, z,
                                   C + (size_t)i * S->s, S->s, i, b0, lev_b<T>(S, 1), S->stream);
      prof_end(S, tk);
      vcycle<T>(S, i, b0, z + (size_t)i * N, true);
    } else {
      ProfTok tk = prof_begin(S, IRK_KC_COUPLE, cbytes);
      irk::kern::couple<T>(Kview<T>(S), v, scale_j, z, C + (size_t)i * S->s, S->s, i, b0,
                           S->stream);
      prof_end(S, tk);
      vcycle<T>(S, i, b0, z + (size_t)i * N, false);
    }
  }
}

// Kernel classes launched inside apply_precond: timing one of them needs the
// direct launches (events between kernels).
bool prof_in_precond(const irk_solver *S) {
  switch (S->prof_sel) {
    case IRK_KC_COUPLE:
    case IRK_KC_VDOWN_L0:
    case IRK_KC_VMID_DOWN:
    case IRK_KC_VTAIL:
    case IRK_KC_VMID_UP:
    case IRK_KC_VUP_L0:
      return true;
    default:
      return false;
  }
}

// apply_precond through a HIP graph: the kernel sequence of one argument set
// is captured on a private stream the first time (capture records, it does
// not run) and replayed on the solver's stream after that.  The sequence
// holds kernel launches only (no memory set or copy nodes).
template <typename T>
void precondition(irk_solver *S, const double *v, const double *scale_j, T *z, const double *C,
                  const int *ord) {
  if (!S->opt.graphs || prof_in_precond(S)) return apply_precond<T>(S, v, scale_j, z, C, ord);
  const irk_solver::PrecGraph *hit = nullptr;
  for (const auto &g : S->graphs)
    if (g.v == v && g.scale == scale_j && g.z == z && g.C == C && g.ord == ord) {
      hit = &g;
      break;
    }
  if (!hit) {
    if (S->graphs.size() >= 256) drop_graphs(S);
    if (!S->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&S->cap_stream, hipStreamNonBlocking));
    const hipStream_t run = S->stream;
    HIP_TRY(hipStreamBeginCapture(S->cap_stream, hipStreamCaptureModeThreadLocal));
    S->stream = S->cap_stream;
    hipGraph_t g = nullptr;
    try {
      apply_precond<T>(S, v, scale_j, z, C, ord);
    } catch (...) {
      S->stream = run;
      (void)hipStreamEndCapture(S->cap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    S->stream = run;
    HIP_TRY(hipStreamEndCapture(S->cap_stream, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) throw HipError{e, "hipGraphInstantiate"};
    S->graphs.push_back({v, scale_j, z, C, ord, ex});
    hit = &S->graphs.back();
  }
  HIP_TRY(hipGraphLaunch(hit->exec, S->stream));
  ++S->graph_replays;
}

struct SystemDesc {
  const double *hA;  // s x s matrix of the SpMM (h A or h A^T)
  const double *C;   // coupling h A~ without diagonal (row i = stage i)
  const int *ord;    // substitution order
  // right-hand side: forward = 1 (x) (g - K u); otherwise rhs (s*N) given
  const double *u;
  bool forward;
  // forward steps whose output does not overlap u: the true-residual pass
  // also writes u + sum_i h b_i k_i here; a converged check then leaves
  // S->u_written set and the step skips its combining pass
  double *u_out = nullptr;
};

// The true residual 1 (x) f - A k (forward systems) or rhs - A k of the
// accumulated k into V0 (may be null) with block partials of its squared norm;
// returns their count.  Uniform five-point K with M = I: the streaming pass.
int true_residual(irk_solver *S, const SystemDesc &sys, int nblk_pt, double *V0, double *u_out,
                  hipStream_t st) {
  if (sys.forward && !mass(S) && kcouple_ok(S))
    return irk::kern::residual_split(S->nx, S->ny, S->K64.interior, S->acc, sys.hA, S->s, S->f,
                                     V0, S->partial, st, sys.u, S->hb, u_out);
  irk::kern::residual_full(S->K64.view(), mass(S), S->acc, sys.hA, S->s,
                           sys.forward ? nullptr : S->rhs, S->f, V0, S->partial, st, sys.u,
                           S->hb, u_out);
  return nblk_pt;
}

template <typename T>
irk_status fgmres(irk_solver *S, const SystemDesc &sys, irk_stats *stats) {
  using namespace irk::kern;
  hipStream_t st = S->stream;
  const int s = S->s, m = S->opt.restart;
  const size_t N = S->N, sN = S->sN;
  const int nblk_pt = (int)((N + irk::kBlock - 1) / irk::kBlock);
  const int nblk_vec = (int)((sN + irk::kBlock * 4 - 1) / (irk::kBlock * 4));
  const int nblk_full = (int)((sN + irk::kBlock - 1) / irk::kBlock);
  const OpView<double> K = S->K64.view();
  T *Z = static_cast<T *>(S->Z);

  // initial residual = rhs (x0 = 0; the first cycle writes acc outright)
  if (sys.forward) {
    rhs_forward(K, sys.u, S->g, s, S->f, S->V, S->partial, st);
    finalize_norm(S->partial, nblk_pt, S->scale, 0, S->norm_dev, st);
  } else {
    rhs_copy(S->rhs, sN, S->V, S->partial, st);
    finalize_norm(S->partial, nblk_full, S->scale, 0, S->norm_dev, st);
  }
  HIP_TRY(hipMemcpyAsync(S->host_resid, S->norm_dev, sizeof(double), hipMemcpyDeviceToHost, st));
  // the first column's preconditioner depends only on the right-hand side:
  // enqueued before the host reads ||rhs|| (unused if that is zero or not finite)
  HIP_TRY(hipEventRecord(S->resid_ev, st));
  precondition<T>(S, S->V, S->scale, Z, sys.C, sys.ord);
  HIP_TRY(hipEventSynchronize(S->resid_ev));
  const double beta0 = S->host_resid[0];
  if (stats) {
    stats->iters = 0;
    stats->restarts = 0;
    stats->rel_resid_est = 0.0;
    stats->rel_resid_true = -1.0;
  }
  if (!std::isfinite(beta0) || beta0 == 0.0) {
    HIP_TRY(hipMemsetAsync(S->acc, 0, sN * sizeof(double), st));
    if (beta0 == 0.0) return IRK_OK;  // k = 0 solves the system exactly
    S->err = "non-finite right-hand side";
    return IRK_E_NONFINITE;
  }

  double beta = beta0;
  int total = 0, restarts = 0;
  irk_status status = IRK_E_NOT_CONVERGED;
  double est = 1.0, true_rel = -1.0;
  while (true) {
    KrylovState ks0{0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(S->ks, &ks0, sizeof ks0, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(S->gv, &beta, sizeof(double), hipMemcpyHostToDevice, st));
    int j = 0;
    bool stop = false;
    bool pre_next = restarts == 0;  // column j's preconditioner is already enqueued
    double res_last = beta, rate = 0.5;
    for (; j < m; ++j) {
      const double *Vj = S->V + (size_t)j * sN;
      T *Zj = Z + (size_t)j * sN;
      if (!pre_next) precondition<T>(S, Vj, S->scale + j, Zj, sys.C, sys.ord);
      pre_next = false;
      const double kb = op_bytes(S, N, S->K64.npt, 8);
      const double zb = (double)sN * sizeof(T), vb = (double)sN * 8.0;
      // the first cycle of a forward system starts from 1 (x) f: the SpMM
      // passes read one stage block of V_0
      const bool v0b = sys.forward && restarts == 0;
      const double v0save = v0b ? (double)(sN - N) * 8.0 : 0.0;
      ProfTok t1 = prof_begin(S, IRK_KC_SPMM_DOTS, zb + vb * (j + 1) + kb - v0save);
      spmm_dots<T>(K, mass(S), Z, sys.hA, s, S->V, S->scale, S->ks, j, S->partial, v0b, st);
      prof_end(S, t1);
      reduce_cols(S->partial, nblk_pt, S->ks, j, 1, 0, S->h1, st);
      ProfTok t2 = prof_begin(S, IRK_KC_SPMM_UPDATE, zb + vb * (j + 2) + kb - v0save);
      spmm_update<T>(K, mass(S), Z, sys.hA, s, S->V, S->scale, S->h1, S->ks, S->V, S->pnorm,
                     v0b, st);
      prof_end(S, t2);
      // second classical Gram-Schmidt pass, skipped on the device when the
      // first one kept most of ||w|| (reorth = 2) or never run (reorth = 0:
      // then the Givens step sums the first pass's norm itself)
      const bool first_only = S->opt.reorth == 0;
      if (!first_only) {
        reorth_decide(S->pnorm, nblk_pt, S->h1, S->ks, S->opt.reorth, S->norm_dev + 1, st);
        ProfTok t3 = prof_begin(S, IRK_KC_VEC_DOTS, vb * (j + 2));
        vec_dots(nullptr, sN, S->V, S->scale, S->ks, j, S->partial, st);
        prof_end(S, t3);
        reduce_cols(S->partial, nblk_vec, S->ks, j, 0, 1, S->h2, st);
        ProfTok t4 = prof_begin(S, IRK_KC_VEC_UPDATE, vb * (j + 3));
        vec_update(nullptr, sN, S->V, S->scale, S->h2, S->ks, S->pnorm2, st);
        prof_end(S, t4);
      }
      givens(S->h1, S->h2, first_only ? S->pnorm : S->pnorm2, first_only ? nblk_pt : nblk_vec,
             S->norm_dev + 1, S->H, m + 1, S->cs, S->sn, S->gv, S->scale, S->ks, beta0,
             S->opt.rtol, S->host_resid_dev, first_only, st);
      // Column j+1's preconditioner needs V_{j+1} (written above), not the
      // convergence decision.  When the estimate will almost surely stay above
      // the tolerance (even at twice the last rate of decrease it would be 10x
      // above), it is enqueued before the host waits for this estimate, so the
      // GPU does not idle through the round trip; a misprediction leaves one
      // unused column (results unchanged).
      const bool spec = j + 1 < m && total + 1 < S->opt.max_iter &&
                        res_last * rate * rate > 10.0 * S->opt.rtol * beta0;
      if (spec) {
        HIP_TRY(hipEventRecord(S->resid_ev, st));
        precondition<T>(S, S->V + (size_t)(j + 1) * sN, S->scale + j + 1,
                        Z + (size_t)(j + 1) * sN, sys.C, sys.ord);
        pre_next = true;
        HIP_TRY(hipEventSynchronize(S->resid_ev));
      } else {
        HIP_TRY(hipStreamSynchronize(st));
      }
      prof_collect(S);
      ++total;
      const double res = S->host_resid[0];
      const int brk = (int)S->host_resid[1];
      est = res / beta0;
      if (res > 0.0 && res_last > 0.0) rate = std::min(1.0, res / res_last);
      res_last = res;
      if (brk == 1 || !std::isfinite(res)) {
        status = IRK_E_BREAKDOWN;
        S->err = "Krylov breakdown (non-finite or zero Hessenberg entry)";
        stop = true;
        ++j;
        break;
      }
      if (res <= S->opt.rtol * beta0 || brk == 2) {
        status = IRK_OK;
        stop = true;
        ++j;
        break;
      }
      if (total >= S->opt.max_iter) {
        status = IRK_E_NOT_CONVERGED;
        stop = true;
        ++j;
        break;
      }
    }
    // x += Z y over the j columns of this cycle (a column that broke down is dropped)
    if (status == IRK_E_BREAKDOWN) --j;
    solve_upper(S->H, m + 1, S->gv, j, S->y, st);
    accumulate_solution<T>(Z, sN, S->y, j, sN, S->acc, restarts == 0, st);
    if (status == IRK_E_BREAKDOWN || (stop && status == IRK_E_NOT_CONVERGED)) break;
    if (status == IRK_OK && !S->opt.true_resid) break;  // trust the estimate
    // true residual of the accumulated solution: verifies a converged estimate
    // (single-pass Gram-Schmidt can make the estimate optimistic) or starts
    // the next restart cycle.  A converged estimate usually passes, so the
    // residual vector itself is only stored when a next cycle needs it.
    const bool need_v0 = status != IRK_OK;
    double *u_out = sys.forward ? sys.u_out : nullptr;
    const int nres = true_residual(S, sys, nblk_pt, need_v0 ? S->V : nullptr, u_out, st);
    finalize_norm(S->partial, nres, S->scale, 0, S->norm_dev, st);
    HIP_TRY(hipMemcpyAsync(S->host_resid, S->norm_dev, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    beta = S->host_resid[0];
    true_rel = beta / beta0;
    if (!std::isfinite(beta)) {
      status = IRK_E_NONFINITE;
      S->err = "non-finite residual";
      break;
    }
    if (beta <= S->opt.rtol * beta0) {
      status = IRK_OK;
      S->u_written = u_out != nullptr;
      break;
    }
    if (total >= S->opt.max_iter) {
      status = IRK_E_NOT_CONVERGED;
      S->u_written = u_out != nullptr;  // the best iterate, as the combining pass would write
      break;
    }
    if (!need_v0) {  // the estimate was optimistic: store the residual for the restart
      const int nr = true_residual(S, sys, nblk_pt, S->V, nullptr, st);
      finalize_norm(S->partial, nr, S->scale, 0, S->norm_dev, st);
    }
    status = IRK_E_NOT_CONVERGED;
    ++restarts;
  }
  if (stats) {
    stats->iters = total;
    stats->restarts = restarts;
    stats->rel_resid_est = est;
    stats->rel_resid_true = true_rel;
  }
  return status;
}

// Left-preconditioned GMRES on P^-1 A k = P^-1 rhs (FP64, forward solves):
// stops when the preconditioned residual estimate |g_{j+1}| <= rtol
// ||P^-1 rhs|| (the paper's criterion for its left-preconditioned runs,
// Sec. 5.1, Tables 7-10) and checks the same quantity from the accumulated solution.
// Each iteration: u = A v_j (into the rhs buffer, unused by forward solves),
// z = P^-1 u (into Z_j), then two classical Gram-Schmidt passes of z against
// the basis; the solution is the basis combination V y.
irk_status gmres_left(irk_solver *S, const SystemDesc &sys, irk_stats *stats) {
  using namespace irk::kern;
  hipStream_t st = S->stream;
  const int s = S->s, m = S->opt.restart;
  const size_t sN = S->sN;
  const int nblk_vec = (int)((sN + irk::kBlock * 4 - 1) / (irk::kBlock * 4));
  const int nblk_full = (int)((sN + irk::kBlock - 1) / irk::kBlock);
  const OpView<double> K = S->K64.view();
  double *Z = static_cast<double *>(S->Z);
  double *u = S->rhs;

  HIP_TRY(hipMemsetAsync(S->acc, 0, sN * sizeof(double), st));
  rhs_forward(K, sys.u, S->g, s, S->f, S->V, S->partial, st);
  // V_0 = P^-1 (1 (x) f), lazily normalised
  precondition<double>(S, S->V, S->one, Z, sys.C, sys.ord);
  rhs_copy(Z, sN, S->V, S->partial, st);
  finalize_norm(S->partial, nblk_full, S->scale, 0, S->norm_dev, st);
  HIP_TRY(hipMemcpyAsync(S->host_resid, S->norm_dev, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const double beta0 = S->host_resid[0];
  if (stats) {
    stats->iters = 0;
    stats->restarts = 0;
    stats->rel_resid_est = 0.0;
    stats->rel_resid_true = -1.0;
  }
  if (!std::isfinite(beta0)) {
    S->err = "non-finite right-hand side";
    return IRK_E_NONFINITE;
  }
  if (beta0 == 0.0) return IRK_OK;

  double beta = beta0, est = 1.0, true_rel = -1.0;
  int total = 0, restarts = 0;
  irk_status status = IRK_E_NOT_CONVERGED;
  while (true) {
    KrylovState ks0{0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(S->ks, &ks0, sizeof ks0, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(S->gv, &beta, sizeof(double), hipMemcpyHostToDevice, st));
    int j = 0;
    bool stop = false;
    for (; j < m; ++j) {
      const double *Vj = S->V + (size_t)j * sN;
      double *Zj = Z + (size_t)j * sN;
      double *Vn = S->V + (size_t)(j + 1) * sN;
      kron_apply(K, mass(S), Vj, sys.hA, s, u, st);
      precondition<double>(S, u, S->scale + j, Zj, sys.C, sys.ord);
      rhs_copy(Zj, sN, Vn, S->partial, st);
      // two classical Gram-Schmidt passes (h1, then h2)
      vec_dots(nullptr, sN, S->V, S->scale, S->ks, j, S->partial, st);
      reduce_cols(S->partial, nblk_vec, S->ks, j, 0, 0, S->h1, st);
      vec_update(nullptr, sN, S->V, S->scale, S->h1, S->ks, S->pnorm, st);
      reorth_decide(S->pnorm, nblk_vec, S->h1, S->ks, 1, S->norm_dev + 1, st);
      vec_dots(nullptr, sN, S->V, S->scale, S->ks, j, S->partial, st);
      reduce_cols(S->partial, nblk_vec, S->ks, j, 0, 1, S->h2, st);
      vec_update(nullptr, sN, S->V, S->scale, S->h2, S->ks, S->pnorm2, st);
      givens(S->h1, S->h2, S->pnorm2, nblk_vec, S->norm_dev + 1, S->H, m + 1, S->cs, S->sn,
             S->gv, S->scale, S->ks, beta0, S->opt.rtol, S->host_resid_dev, false, st);
      HIP_TRY(hipStreamSynchronize(st));
      ++total;
      const double res = S->host_resid[0];
      const int brk = (int)S->host_resid[1];
      est = res / beta0;
      if (brk == 1 || !std::isfinite(res)) {
        status = IRK_E_BREAKDOWN;
        S->err = "Krylov breakdown (non-finite or zero Hessenberg entry)";
        stop = true;
        ++j;
        break;
      }
      if (res <= S->opt.rtol * beta0 || brk == 2) {
        status = IRK_OK;
        stop = true;
        ++j;
        break;
      }
      if (total >= S->opt.max_iter) {
        status = IRK_E_NOT_CONVERGED;
        stop = true;
        ++j;
        break;
      }
    }
    if (status == IRK_E_BREAKDOWN) --j;
    solve_upper(S->H, m + 1, S->gv, j, S->y, st);
    scale_by(S->y, S->scale, j, st);
    accumulate_solution<double>(S->V, sN, S->y, j, sN, S->acc, false, st);
    if (status == IRK_E_BREAKDOWN || (stop && status == IRK_E_NOT_CONVERGED)) break;
    if (status == IRK_OK && !S->opt.true_resid) break;
    // preconditioned residual of the accumulated solution: P^-1 (rhs - A k)
    residual_full(K, mass(S), S->acc, sys.hA, s, nullptr, S->f, S->V, S->partial, st);
    precondition<double>(S, S->V, S->one, Z, sys.C, sys.ord);
    rhs_copy(Z, sN, S->V, S->partial, st);
    finalize_norm(S->partial, nblk_full, S->scale, 0, S->norm_dev, st);
    HIP_TRY(hipMemcpyAsync(S->host_resid, S->norm_dev, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    beta = S->host_resid[0];
    true_rel = beta / beta0;
    if (!std::isfinite(beta)) {
      status = IRK_E_NONFINITE;
      S->err = "non-finite residual";
      break;
    }
    if (beta <= S->opt.rtol * beta0) {
      status = IRK_OK;
      break;
    }
    if (total >= S->opt.max_iter) {
      status = IRK_E_NOT_CONVERGED;
      break;
    }
    status = IRK_E_NOT_CONVERGED;
    ++restarts;
  }
  if (stats) {
    stats->iters = total;
    stats->restarts = restarts;
    stats->rel_resid_est = est;
    stats->rel_resid_true = true_rel;
  }
  return status;
}

irk_status run_system(irk_solver *S, const SystemDesc &sys, irk_stats *st) {
  if (S->opt.side == IRK_LEFT && sys.forward) return gmres_left(S, sys, st);
  if (S->opt.precision == IRK_MIXED) return fgmres<float>(S, sys, st);
  return fgmres<double>(S, sys, st);
}

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

bool valid_options(const irk_options &o, std::string &err) {
  if (o.precision != IRK_FP64 && o.precision != IRK_MIXED) return err = "bad precision", false;
  if (o.precond < IRK_PREC_LD || o.precond > IRK_PREC_J) return err = "bad precond", false;
  if (o.restart < 1 || o.restart > irk::kMaxKrylov) return err = "restart must be in 1..200", false;
  if (o.max_iter < 1) return err = "max_iter must be >= 1", false;
  if (o.nu_pre < 1 || o.nu_pre > 3 || o.nu_post != o.nu_pre)
    return err = "nu_pre = nu_post in 1..3 is required", false;
  if (o.coarse_max < 1) return err = "coarse_max must be >= 1", false;
  if (o.vcycles != 1) return err = "only one V-cycle per subsolve is implemented", false;
  if (!(o.rtol > 0.0) || !(o.rtol < 1.0)) return err = "rtol must be in (0, 1)", false;
  if (o.reorth < 0 || o.reorth > 2) return err = "reorth must be 0, 1 or 2", false;
  if (o.side != IRK_RIGHT && o.side != IRK_LEFT) return err = "side must be IRK_RIGHT or IRK_LEFT", false;
  if (o.interp != IRK_INTERP_LINEAR && o.interp != IRK_INTERP_CONSTANT)
    return err = "interp must be IRK_INTERP_LINEAR or IRK_INTERP_CONSTANT", false;
  if (o.graphs != 0 && o.graphs != 1) return err = "graphs must be 0 or 1", false;
  if (!(o.coarse_ratio >= 0.0) || !std::isfinite(o.coarse_ratio))
    return err = "coarse_ratio must be finite and >= 0", false;
  if (o.side == IRK_LEFT && o.precision != IRK_FP64)
    return err = "left preconditioning needs precision IRK_FP64", false;
  if (o.smoother != IRK_SMOOTH_RBGS && o.smoother != IRK_SMOOTH_JACOBI)
    return err = "smoother must be IRK_SMOOTH_RBGS or IRK_SMOOTH_JACOBI", false;
  if (o.smoother == IRK_SMOOTH_JACOBI && !(o.jacobi_omega > 0.0 && o.jacobi_omega <= 1.0))
    return err = "jacobi_omega must be in (0, 1]", false;
  if (o.fuse_levels != 0 && o.fuse_levels != 1) return err = "fuse_levels must be 0 or 1", false;
  return true;
}

thread_local std::string g_setup_error;

template <typename F>
irk_status guarded(irk_solver *S, F &&fn) {
  try {
    return fn();
  } catch (const HipError &e) {
    if (S) {
      S->err = std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e);
    }
    return e.e == hipErrorOutOfMemory ? IRK_E_OOM : IRK_E_HIP;
  } catch (const std::bad_alloc &) {
    if (S) S->err = "host allocation failed";
    return IRK_E_OOM;
  } catch (...) {
    if (S) S->err = "unexpected exception";
    return IRK_E_INVALID;
  }
}

// ---------------------------------------------------------------------------
// Static scratch of the allocation-free step (irk_step_noalloc).  One copy per
// GPU, held from module load to process end.  Host code never uses the name
// `scratch` as an address: each device's address comes from
// hipGetSymbolAddress, taken once per device at setup with that device
// current, and only that address reaches kernels and copies.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
bool g_scratch_done[kScratchDevices] = {};
void *g_scratch_ptr[kScratchDevices] = {};
hipError_t g_scratch_err[kScratchDevices] = {};

// Record the device address of `scratch` on the current device (first call
// per device only).  A failure is kept and reported by irk_step_noalloc.
void init_scratch(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev < 0 || dev >= kScratchDevices || g_scratch_done[dev]) return;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_scratch_done[dev] = true;
  g_scratch_err[dev] = e;
  g_scratch_ptr[dev] = (e == hipSuccess) ? p : nullptr;
}

__global__ void __launch_bounds__(256) k_fill_zero(double *__restrict__ p, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// The per-step buffers of a solver (everything a step writes besides its
// output; the operators and the pinned host word stay the solver's).
struct StepBuffers {
  double *V, *acc, *rhs, *f, *zero, *partial, *pnorm, *pnorm2, *H, *cs, *sn, *gv, *y, *scale, *h1,
      *h2, *norm_dev;
  void *Z, *b0, *levb, *levx, *levp, *xp0;
  KrylovState *ks;
};

StepBuffers get_buffers(const irk_solver *S) {
  return StepBuffers{S->V,  S->acc, S->rhs,   S->f,     S->zero, S->partial, S->pnorm, S->pnorm2,
                     S->H,  S->cs,  S->sn,    S->gv,    S->y,    S->scale,   S->h1,    S->h2,
                     S->norm_dev, S->Z, S->b0, S->levb, S->levx, S->levp, S->xp0, S->ks};
}

void set_buffers(irk_solver *S, const StepBuffers &b) {
  S->V = b.V;
  S->acc = b.acc;
  S->rhs = b.rhs;
  S->f = b.f;
  S->zero = b.zero;
  S->partial = b.partial;
  S->pnorm = b.pnorm;
  S->pnorm2 = b.pnorm2;
  S->H = b.H;
  S->cs = b.cs;
  S->sn = b.sn;
  S->gv = b.gv;
  S->y = b.y;
  S->scale = b.scale;
  S->h1 = b.h1;
  S->h2 = b.h2;
  S->norm_dev = b.norm_dev;
  S->Z = b.Z;
  S->b0 = b.b0;
  S->levb = b.levb;
  S->levx = b.levx;
  S->levp = b.levp;
  S->xp0 = b.xp0;
  S->ks = b.ks;
}

// Lay the step buffers of S out from `base` (256-byte aligned pieces); with
// base == nullptr only the size is computed.  `zero` has N elements here:
// it only serves as the zero coarse correction (levels >= 1).
size_t carve_buffers(const irk_solver *S, unsigned char *base, StepBuffers &b) {
  const size_t m = (size_t)S->opt.restart, N = S->N, sN = S->sN, es = elem_size(S);
  const size_t nblk_pt = (N + irk::kBlock - 1) / irk::kBlock;
  const size_t nblk_vec = (sN + irk::kBlock * 4 - 1) / (irk::kBlock * 4);
  const size_t nblk_full = (sN + irk::kBlock - 1) / irk::kBlock;
  const size_t npn = std::max({nblk_pt, nblk_vec, nblk_full});
  size_t tot = 0;
  for (int l = 1; l < S->nlev; ++l) tot += (size_t)S->lnx[l] * S->lny[l];
  size_t off = 0;
  auto take = [&](size_t bytes) -> void * {
    void *p = base ? static_cast<void *>(base + off) : nullptr;
    off += (bytes + 255) & ~size_t(255);
    return p;
  };
  b.V = static_cast<double *>(take((m + 1) * sN * 8));
  b.Z = take(m * sN * es);
  b.acc = static_cast<double *>(take(sN * 8));
  b.rhs = static_cast<double *>(take(sN * 8));
  b.f = static_cast<double *>(take(N * 8));
  b.zero = static_cast<double *>(take(N * 8));
  b.partial = static_cast<double *>(take(S->partial_len * 8));
  b.pnorm = static_cast<double *>(take(npn * 8));
  b.pnorm2 = static_cast<double *>(take(npn * 8));
  b.H = static_cast<double *>(take((m + 1) * m * 8));
  b.cs = static_cast<double *>(take((m + 1) * 8));
  b.sn = static_cast<double *>(take((m + 1) * 8));
  b.gv = static_cast<double *>(take((m + 2) * 8));
  b.y = static_cast<double *>(take((m + 1) * 8));
  b.scale = static_cast<double *>(take((m + 2) * 8));
  b.h1 = static_cast<double *>(take((m + 2) * 8));
  b.h2 = static_cast<double *>(take((m + 2) * 8));
  b.norm_dev = static_cast<double *>(take(2 * 8));
  b.ks = static_cast<KrylovState *>(take(sizeof(KrylovState)));
  b.b0 = take(N * es);
  b.levb = take((tot + 1) * es);
  b.levx = take((tot + 1) * es);
  b.levp = take((tot + 1) * es);
  b.xp0 = take(N * es);
  return off;
}

}  // namespace

extern "C" {

void irk_default_options(irk_options *o) {
  if (!o) return;
  o->precision = IRK_FP64;
  o->precond = IRK_PREC_LD;
  o->restart = 40;
  o->max_iter = 200;
  o->nu_pre = 2;
  o->nu_post = 2;
  o->coarse_max = 64;
  o->vcycles = 1;
  o->true_resid = 1;
  o->reorth = 0;
  o->rtol = 1e-8;
  o->side = IRK_RIGHT;
  o->interp = IRK_INTERP_LINEAR;
  o->graphs = 0;
  o->coarse_ratio = 8.0;
  o->smoother = IRK_SMOOTH_RBGS;
  o->jacobi_omega = 0.8;
  o->fuse_levels = 1;
}

irk_status irk_ldu(int s, const double *A, double *L, double *d, double *U) {
  int rc = irk::ldu_factor(s, A, L, d, U);
  return rc == 0 ? IRK_OK : (rc == -2 ? IRK_E_SINGULAR_PIVOT : IRK_E_INVALID);
}

irk_status irk_setup(irk_solver **out, const irk_butcher *tab, const irk_csr *M, const irk_csr *K,
                     double h_t, const irk_grid *grid, const irk_options *opt, void *hip_stream) {
  if (!out) return IRK_E_INVALID;
  *out = nullptr;
  irk_solver *S = new (std::nothrow) irk_solver();
  if (!S) return IRK_E_OOM;
  irk_status rc = guarded(S, [&]() -> irk_status {
    if (!tab || !tab->A || !tab->b || tab->s < 1 || tab->s > 8) {
      S->err = "bad Butcher tableau (need 1 <= s <= 8 and non-null A, b)";
      return IRK_E_INVALID;
    }
    if (!K || !grid) {
      S->err = "K and the structured grid are required";
      return IRK_E_INVALID;
    }
    if (!(h_t > 0.0) || !std::isfinite(h_t)) {
      S->err = "h_t must be positive and finite";
      return IRK_E_INVALID;
    }
    irk_options o;
    irk_default_options(&o);
    if (opt) o = *opt;
    if (!valid_options(o, S->err)) return IRK_E_INVALID;
    S->opt = o;
    S->stream = static_cast<hipStream_t>(hip_stream);
    S->s = tab->s;
    S->nx = grid->nx;
    S->ny = grid->ny;
    if (S->nx < 1 || S->ny < 1 || (long long)S->nx * S->ny != K->n) {
      S->err = "grid size does not match K";
      return IRK_E_INVALID;
    }
    S->N = (size_t)S->nx * S->ny;
    S->sN = S->N * S->s;
    if (M) {
      if (M->n != K->n) {
        S->err = "M and K differ in size";
        return IRK_E_INVALID;
      }
      std::string merr;
      if (!irk::csr_to_stencil(M->n, M->rowptr, M->colind, M->val, S->nx, S->ny, S->Mst, merr)) {
        S->err = "M: " + merr;
        return IRK_E_INVALID;
      }
      for (size_t p = 0; p < S->N; ++p)
        if (!(S->Mst.c[4][p] > 0.0)) {
          S->err = "M needs a positive diagonal";
          return IRK_E_INVALID;
        }
      S->has_mass = true;
    }
    S->h = h_t;
    const int s = S->s;
    for (int i = 0; i < s * s; ++i) {
      S->A[i] = tab->A[i];
      if (!std::isfinite(S->A[i])) {
        S->err = "non-finite Butcher coefficient";
        return IRK_E_INVALID;
      }
    }
    for (int i = 0; i < s; ++i) S->b[i] = tab->b[i];
    // A~ and its LDU (Sec. 4.1): pivot check for every choice
    if (irk::ldu_factor(s, S->A, nullptr, nullptr, nullptr) == -2) {
      S->err = "A has a zero leading principal minor: no LDU factorisation without pivoting";
      return IRK_E_SINGULAR_PIVOT;
    }
    const int kind = o.precond;  // 0 LD, 1 DU, 2 GSL, 3 J
    if (irk::coefficient_matrix(s, S->A, kind, S->At) != 0) {
      S->err = "LDU factorisation failed";
      return IRK_E_SINGULAR_PIVOT;
    }
    const bool upper = (kind == IRK_PREC_DU);
    for (int i = 0; i < s; ++i) {
      S->tau[i] = h_t * S->At[i * s + i];
      S->hb[i] = h_t * S->b[i];
      if (!(S->tau[i] > 0.0)) {
        S->err = "a diagonal block I + h A~_ii K has A~_ii <= 0";
        return IRK_E_INVALID;
      }
      for (int j = 0; j < s; ++j) {
        S->hA[i * s + j] = h_t * S->A[i * s + j];
        S->hAT[i * s + j] = h_t * S->A[j * s + i];
        S->Cfwd[i * s + j] = (i == j) ? 0.0 : h_t * S->At[i * s + j];
        S->Cadj[i * s + j] = (i == j) ? 0.0 : h_t * S->At[j * s + i];
      }
    }
    for (int t = 0; t < s; ++t) {
      S->ord_fwd[t] = upper ? s - 1 - t : t;  // lower: forward substitution
      S->ord_adj[t] = upper ? t : s - 1 - t;  // transposed: the other direction
    }
    irk_status r = build_operators(S, K);
    if (r != IRK_OK) return r;
    // the device that holds the operators (and the workspace below)
    HIP_TRY(hipGetDevice(&S->device));
    init_scratch(S->device);
    alloc_workspace(S);
    return IRK_OK;
  });
  if (rc != IRK_OK) {
    // the solver is gone; its message stays readable through irk_last_error(NULL)
    g_setup_error = S->err;
    irk_destroy(S);
    return rc;
  }
  g_setup_error.clear();
  *out = S;
  return IRK_OK;
}

irk_status irk_set_source(irk_solver *S, const double *g_dev) {
  if (!S) return IRK_E_INVALID;
  return guarded(S, [&]() -> irk_status {
    if (!g_dev) {
      S->g = nullptr;
      return IRK_OK;
    }
    // the source lives in a buffer of its own, allocated on first use
    if (!S->gbuf) S->gbuf = dalloc<double>(S->ws_allocs, S->N);
    HIP_TRY(hipMemcpyAsync(S->gbuf, g_dev, S->N * sizeof(double), hipMemcpyDeviceToDevice,
                           S->stream));
    HIP_TRY(hipStreamSynchronize(S->stream));
    S->g = S->gbuf;
    return IRK_OK;
  });
}

irk_status irk_update_operator(irk_solver *S, const irk_csr *K) {
  if (!S || !K) return IRK_E_INVALID;
  return guarded(S, [&]() -> irk_status {
    if (K->n != (int)S->N) {
      S->err = "K size changed";
      return IRK_E_INVALID;
    }
    const int old_levels = S->nlev;
    irk_destroy(S->adj);  // its K^T is stale; set up again when needed
    S->adj = nullptr;
    irk_status r = build_operators(S, K);
    if (r == IRK_OK && S->nlev != old_levels) {
      S->err = "hierarchy depth changed";
      return IRK_E_INVALID;
    }
    return r;
  });
}

static irk_status step_impl(irk_solver *S, const double *u_n, double *u_np1, double *k_out,
                            irk_stats *st) {
  if (!S || !u_n || !u_np1) return IRK_E_INVALID;
  return guarded(S, [&]() -> irk_status {
    const double t0 = now_s();
    SystemDesc sys{S->hA, S->Cfwd, S->ord_fwd, u_n, true};
    // the true-residual pass may write the output only if it does not
    // overlap u_n: a restart after a failed check reads u_n again
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(u_n), a1 = reinterpret_cast<uintptr_t>(u_np1);
    const uintptr_t nb = S->N * sizeof(double);
    const bool apart = a1 + nb <= a0 || a0 + nb <= a1;
    sys.u_out = apart ? u_np1 : nullptr;
    S->u_written = false;
    irk_stats local{};
    irk_status r = run_system(S, sys, st ? st : &local);
    if (r == IRK_OK || r == IRK_E_NOT_CONVERGED) {
      if (!S->u_written)
        irk::kern::combine_stages(u_n, S->acc, S->hb, S->s, S->N, u_np1, S->stream);
      if (k_out)
        HIP_TRY(hipMemcpyAsync(k_out, S->acc, S->sN * sizeof(double), hipMemcpyDeviceToDevice,
                               S->stream));
      HIP_TRY(hipStreamSynchronize(S->stream));
    }
    if (st) st->seconds = now_s() - t0;
    return r;
  });
}

irk_status irk_step(irk_solver *S, const double *u_n_dev, double *u_np1_dev, irk_stats *st) {
  return step_impl(S, u_n_dev, u_np1_dev, nullptr, st);
}

irk_status irk_step_stages(irk_solver *S, const double *u_n_dev, double *u_np1_dev, double *k_dev,
                           irk_stats *st) {
  if (!k_dev) return IRK_E_INVALID;
  return step_impl(S, u_n_dev, u_np1_dev, k_dev, st);
}

irk_status irk_step_noalloc(irk_solver *S, const double *u_n_dev, double *u_np1_dev,
                            irk_stats *st) {
  if (!S || !u_n_dev || !u_np1_dev) return IRK_E_INVALID;
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (S->device < 0 || S->device >= kScratchDevices || !g_scratch_done[S->device]) {
      S->err = "irk_step_noalloc: no static scratch address for this device";
      return IRK_E_HIP;
    }
    if (!g_scratch_ptr[S->device]) {
      S->err = std::string("irk_step_noalloc: hipGetSymbolAddress failed: ") +
               hipGetErrorString(g_scratch_err[S->device]);
      return IRK_E_HIP;
    }
    base = g_scratch_ptr[S->device];
  }
  StepBuffers mine{};
  const size_t need = carve_buffers(S, nullptr, mine);
  if (need > kScratchBytes) {
    char msg[200];
    std::snprintf(msg, sizeof msg,
                  "irk_step_noalloc: this solver's step needs %zu bytes of scratch, more than the "
                  "static %zu bytes (use irk_step)",
                  need, kScratchBytes);
    S->err = msg;
    return IRK_E_INVALID;
  }
  carve_buffers(S, static_cast<unsigned char *>(base), mine);
  // run the ordinary step on the static buffers: no graph capture (it would
  // allocate), no event timing; the solver's own buffers come back afterwards
  const StepBuffers own = get_buffers(S);
  const int graphs = S->opt.graphs, prof = S->prof_sel;
  set_buffers(S, mine);
  S->opt.graphs = 0;
  S->prof_sel = -1;
  irk_status r = guarded(S, [&]() -> irk_status {
    k_fill_zero<<<(unsigned)((S->N + 255) / 256), 256, 0, S->stream>>>(S->zero, S->N);
    HIP_TRY(hipGetLastError());
    return IRK_OK;
  });
  if (r == IRK_OK) r = step_impl(S, u_n_dev, u_np1_dev, nullptr, st);
  set_buffers(S, own);
  S->opt.graphs = graphs;
  S->prof_sel = prof;
  return r;
}

// K^T (and M^T) as a stencil: the coefficient of node p towards neighbour
// p + d is the coefficient of p + d towards p.
static Stencil9 transposed(const Stencil9 &A) {
  Stencil9 T;
  T.resize(A.nx, A.ny);
  for (int j = 0; j < A.ny; ++j)
    for (int i = 0; i < A.nx; ++i)
      for (int k = 0; k < 9; ++k) {
        const int qi = i + irk::kdx(k), qj = j + irk::kdy(k);
        double v = 0.0;
        if (qi >= 0 && qi < A.nx && qj >= 0 && qj < A.ny)
          v = A.c[8 - k][(size_t)qj * A.nx + qi];
        T.c[k][(size_t)j * A.nx + i] = v;
      }
  return T;
}

struct HostCsr {
  std::vector<int> rowptr, colind;
  std::vector<double> val;
  irk_csr view() const {
    return irk_csr{(int)rowptr.size() - 1, (int)colind.size(), rowptr.data(), colind.data(),
                   val.data()};
  }
};

// Row-major CSR of a stencil (the diagonal always, other entries when nonzero).
static HostCsr to_csr(const Stencil9 &A) {
  HostCsr c;
  c.rowptr.push_back(0);
  for (int j = 0; j < A.ny; ++j)
    for (int i = 0; i < A.nx; ++i) {
      const size_t p = (size_t)j * A.nx + i;
      for (int k = 0; k < 9; ++k) {
        const int qi = i + irk::kdx(k), qj = j + irk::kdy(k);
        if (qi < 0 || qi >= A.nx || qj < 0 || qj >= A.ny) continue;
        const double v = A.c[k][p];
        if (v == 0.0 && k != 4) continue;
        c.colind.push_back(qj * A.nx + qi);
        c.val.push_back(v);
      }
      c.rowptr.push_back((int)c.colind.size());
    }
  return c;
}

// The solver of the transposed stage system: tableau A^T, K^T, M^T, the
// same grid, h_t, options and stream.
static irk_status adjoint_solver(irk_solver *S) {
  if (S->adj) return IRK_OK;
  const int s = S->s;
  double AT[64], c[8] = {};
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < s; ++j) AT[i * s + j] = S->A[j * s + i];
  const irk_butcher tab{s, AT, S->b, c};
  const HostCsr kt = to_csr(transposed(S->Kst));
  HostCsr mt;
  if (S->has_mass) mt = to_csr(transposed(S->Mst));
  const irk_csr kv = kt.view(), mv = mt.view();
  const irk_grid grid{S->nx, S->ny};
  irk_status r = irk_setup(&S->adj, &tab, S->has_mass ? &mv : nullptr, &kv, S->h, &grid, &S->opt,
                           S->stream);
  if (r != IRK_OK) {
    S->err = std::string("transposed stage system: ") + irk_last_error(nullptr);
    S->adj = nullptr;
  }
  return r;
}

irk_status irk_adjoint_step(irk_solver *S, const double *u_n_dev, const double *lam_np1_dev,
                            double *lam_n_dev, double *psi_dev, double *U_dev, irk_stats *st) {
  if (!S || !u_n_dev || !lam_np1_dev || !lam_n_dev) return IRK_E_INVALID;
  return guarded(S, [&]() -> irk_status {
    const double t0 = now_s();
    irk_stats fst{}, ast{};
    // 1. forward stages from the checkpoint u_n
    SystemDesc fwd{S->hA, S->Cfwd, S->ord_fwd, u_n_dev, true};
    irk_status r = run_system(S, fwd, &fst);
    if (r != IRK_OK) return r;
    if (!S->Ubuf) S->Ubuf = dalloc<double>(S->ws_allocs, S->sN);
    irk::kern::stage_values(u_n_dev, S->acc, S->hA, S->s, S->N, S->Ubuf, S->stream);
    // 2. transposed stage system with rhs h (b (x) lam_{n+1}): for a
    // symmetric K and M = I this solver's own operators with A^T and the
    // transposed preconditioner; otherwise the solver of the transposed system
    irk_solver *T = S;
    if (S->symmetric && !S->has_mass) {
      irk::kern::scaled_broadcast(lam_np1_dev, S->hb, S->s, S->N, S->rhs, S->stream);
      SystemDesc adj{S->hAT, S->Cadj, S->ord_adj, nullptr, false};
      r = run_system(S, adj, &ast);
    } else {
      r = adjoint_solver(S);
      if (r != IRK_OK) return r;
      T = S->adj;
      irk::kern::scaled_broadcast(lam_np1_dev, S->hb, S->s, S->N, T->rhs, S->stream);
      SystemDesc adj{T->hA, T->Cfwd, T->ord_fwd, nullptr, false};
      r = run_system(T, adj, &ast);
      if (r != IRK_OK && r != IRK_E_NOT_CONVERGED) S->err = "transposed stage system: " + T->err;
    }
    if (r != IRK_OK && r != IRK_E_NOT_CONVERGED) return r;
    // 3. lam_n = lam_{n+1} - K^T sum_i psi_i (T's K is K^T, or K when symmetric)
    irk::kern::adjoint_lambda(T->K64.view(), lam_np1_dev, T->acc, S->s, lam_n_dev, S->stream);
    if (psi_dev)
      HIP_TRY(hipMemcpyAsync(psi_dev, T->acc, S->sN * sizeof(double), hipMemcpyDeviceToDevice,
                             S->stream));
    if (U_dev)
      HIP_TRY(hipMemcpyAsync(U_dev, S->Ubuf, S->sN * sizeof(double), hipMemcpyDeviceToDevice,
                             S->stream));
    HIP_TRY(hipStreamSynchronize(S->stream));
    if (st) {
      *st = ast;
      st->iters = fst.iters + ast.iters;
      st->seconds = now_s() - t0;
    }
    return r;
  });
}

irk_status irk_grad_diffusion_nodes(irk_solver *S, const double *psi_dev, const double *U_dev,
                                    double h_x, double *gnode_dev) {
  if (!S || !psi_dev || !U_dev || !gnode_dev || !(h_x > 0.0)) return IRK_E_INVALID;
  return guarded(S, [&]() -> irk_status {
    irk::kern::grad_nodes(psi_dev, U_dev, S->s, S->nx, S->ny, 1.0 / (h_x * h_x), gnode_dev,
                          S->stream);
    HIP_TRY(hipStreamSynchronize(S->stream));
    return IRK_OK;
  });
}

irk_status irk_grad_diffusion_faces(irk_solver *S, const double *psi_dev, const double *U_dev,
                                    double h_x, double *gface_dev) {
  if (!S || !psi_dev || !U_dev || !gface_dev || !(h_x > 0.0)) return IRK_E_INVALID;
  return guarded(S, [&]() -> irk_status {
    irk::kern::grad_faces(psi_dev, U_dev, S->s, S->nx, S->ny, 1.0 / (h_x * h_x), gface_dev,
                          S->stream);
    HIP_TRY(hipStreamSynchronize(S->stream));
    return IRK_OK;
  });
}

irk_status irk_apply_operator(irk_solver *S, const double *x_dev, double *y_dev) {
  if (!S || !x_dev || !y_dev) return IRK_E_INVALID;
  return guarded(S, [&]() -> irk_status {
    irk::kern::kron_apply(S->K64.view(), mass(S), x_dev, S->hA, S->s, y_dev, S->stream);
    HIP_TRY(hipStreamSynchronize(S->stream));
    return IRK_OK;
  });
}

irk_status irk_apply_preconditioner(irk_solver *S, const double *v_dev, double *z_dev) {
  if (!S || !v_dev || !z_dev) return IRK_E_INVALID;
  return guarded(S, [&]() -> irk_status {
    const double one = 1.0;
    HIP_TRY(hipMemcpyAsync(S->scale, &one, sizeof(double), hipMemcpyHostToDevice, S->stream));
    HIP_TRY(hipMemcpyAsync(S->V, v_dev, S->sN * sizeof(double), hipMemcpyDeviceToDevice, S->stream));
    HIP_TRY(hipMemcpyAsync(S->y, &one, sizeof(double), hipMemcpyHostToDevice, S->stream));
    if (S->opt.precision == IRK_MIXED) {
      precondition<float>(S, S->V, S->scale, static_cast<float *>(S->Z), S->Cfwd, S->ord_fwd);
      irk::kern::accumulate_solution<float>(static_cast<float *>(S->Z), S->sN, S->y, 1, S->sN,
                                            z_dev, true, S->stream);
    } else {
      precondition<double>(S, S->V, S->scale, static_cast<double *>(S->Z), S->Cfwd, S->ord_fwd);
      irk::kern::accumulate_solution<double>(static_cast<double *>(S->Z), S->sN, S->y, 1, S->sN,
                                             z_dev, true, S->stream);
    }
    HIP_TRY(hipStreamSynchronize(S->stream));
    return IRK_OK;
  });
}

void irk_destroy(irk_solver *S) {
  if (!S) return;
  (void)hipStreamSynchronize(S->stream);
  irk_destroy(S->adj);
  for (const auto &t : S->prof_pending) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (hipEvent_t e : S->prof_pool) (void)hipEventDestroy(e);
  for (const auto &g : S->graphs) (void)hipGraphExecDestroy(g.exec);
  if (S->cap_stream) (void)hipStreamDestroy(S->cap_stream);
  if (S->resid_ev) (void)hipEventDestroy(S->resid_ev);
  free_list(S->op_allocs);
  free_list(S->ws_allocs);
  if (S->host_resid) (void)hipHostFree(S->host_resid);
  delete S;
}

const char *irk_status_string(irk_status st) {
  switch (st) {
    case IRK_OK: return "IRK_OK";
    case IRK_E_INVALID: return "IRK_E_INVALID";
    case IRK_E_SINGULAR_PIVOT: return "IRK_E_SINGULAR_PIVOT";
    case IRK_E_NOT_CONVERGED: return "IRK_E_NOT_CONVERGED";
    case IRK_E_BREAKDOWN: return "IRK_E_BREAKDOWN";
    case IRK_E_NONFINITE: return "IRK_E_NONFINITE";
    case IRK_E_HIP: return "IRK_E_HIP";
    case IRK_E_OOM: return "IRK_E_OOM";
  }
  return "unknown irk_status";
}

const char *irk_last_error(const irk_solver *S) {
  return S ? S->err.c_str() : g_setup_error.c_str();
}

irk_status irk_profile_select(irk_solver *S, int kc) {
  if (!S || kc < -1 || kc >= IRK_KC_COUNT) return IRK_E_INVALID;
  return guarded(S, [&]() -> irk_status {
    HIP_TRY(hipStreamSynchronize(S->stream));
    prof_collect(S);
    S->prof_sel = kc;
    S->prof_launches = 0;
    S->prof_ms = 0.0;
    S->prof_bytes = 0.0;
    return IRK_OK;
  });
}

irk_status irk_profile_read(const irk_solver *S, long long *launches, double *total_ms,
                            double *total_bytes) {
  if (!S) return IRK_E_INVALID;
  if (launches) *launches = S->prof_launches;
  if (total_ms) *total_ms = S->prof_ms;
  if (total_bytes) *total_bytes = S->prof_bytes;
  return IRK_OK;
}

irk_status irk_graph_stats(const irk_solver *S, int *graphs, long long *replays) {
  if (!S) return IRK_E_INVALID;
  if (graphs) *graphs = (int)S->graphs.size();
  if (replays) *replays = S->graph_replays;
  return IRK_OK;
}

irk_status irk_info(const irk_solver *S, int *N, int *s, int *levels, int *constant_coeff) {
  if (!S) return IRK_E_INVALID;
  if (N) *N = (int)S->N;
  if (s) *s = S->s;
  if (levels) *levels = S->nlev;
  if (constant_coeff) *constant_coeff = S->const_mode ? 1 : 0;
  return IRK_OK;
}

}  // extern "C"
