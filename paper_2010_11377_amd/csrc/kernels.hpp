// Device kernels of the IRK stage solver (gfx950, wave64) and their host
// launchers.  All launches go to the stream passed in; nothing synchronises.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace irk {

constexpr int kBlock = 256;  // threads per block for point kernels (4 waves)
constexpr int kMaxStages = 8;
constexpr int kMaxKrylov = 200;  // longest FGMRES restart cycle (Krylov columns)

#ifdef __HIPCC__
// Workgroups go to the eight XCDs (each with its own L2) in turn, so the
// neighbouring tiles of a 2-D launch would sit on different XCDs and fetch
// their shared halo rows and partial cache lines twice.  Tile of this
// workgroup when each XCD takes a contiguous band of tiles (row-major over
// the launch grid; the last total mod 8 workgroups keep their own tile).
struct Tile2 {
  int x, y;
};
__device__ __forceinline__ Tile2 xcd_tile() {
  constexpr int kXcds = 8;
  const int nx = gridDim.x, total = gridDim.x * gridDim.y;
  const int id = blockIdx.y * nx + blockIdx.x;
  const int per = total / kXcds;
  const int t = id < per * kXcds ? (id % kXcds) * per + id / kXcds : id;
  return {t % nx, t / nx};
}
#endif

// A stencil operator on one grid level, as seen by the kernels.
//  cls != nullptr: constant-coefficient operator; cls[q * 9 + k] is
//                  coefficient k of boundary class q (see node_class).
//  arr != nullptr: per-node coefficients, arr[k * N + p].
//  npt = 5: only the centre and the four edge neighbours are nonzero.
//  uniform: constant coefficients whose boundary rows are the interior
//           stencil without the couplings that leave the grid.
//  pw:      prolongation weight of the outermost fine node of this level
//           (linear interpolation towards the zero Dirichlet boundary; the
//           other fine nodes take 3/4 and 1/4 per direction).
template <typename T>
struct OpView {
  int nx, ny;
  int npt;
  const T *cls;
  const T *arr;
  int uniform;
  T pw;            // prolongation weight of an outermost fine node from its parent
  T pa = T(0.75);  // prolongation weight from the parent (other fine nodes)
  T pn = T(0.25);  // prolongation weight from the next coarse node (0: piecewise constant)
  T jw = T(0);     // smoother: 0 red-black Gauss-Seidel; > 0 damped Jacobi with this weight
};

// The coarse end of the hierarchy, solved by one workgroup in LDS: levels
// 0..nlev-1 of the tail (level 0 = the finest tail level, at most kTailMax
// nodes), operators of every level but the last, and the transposed dense
// inverse of the last.
constexpr int kTailMax = 4096;
constexpr int kTailLevels = 8;
constexpr int kTailMaxCoarse = 1024;  // largest dense coarsest level
template <typename T>
struct TailDesc {
  int nlev;
  int nx[kTailLevels], ny[kTailLevels];
  size_t off[kTailLevels + 1];  // LDS offset (elements) of level l: b then x; off[nlev] = end
  const T *cls[kTailLevels];
  const T *arr[kTailLevels];
  T pw[kTailLevels];  // prolongation boundary weight of level l (see OpView)
  T pa = T(0.75), pn = T(0.25);  // parent / next-node prolongation weights (see OpView)
  const T *CinvT;  // null: the coarsest level returns x = 0 (the cycle ends one level up)
  T jw = T(0);     // smoother (see OpView)
};

// The finest level of the stage blocks D_i = I + tau_i K (M = I) for the
// passes that keep the pre-smoothed x (wfine.hip): either K per node, packed
// in the passes' precision (kq: S, W, E, N of node p at 4p..4p+3; kc: centre),
// with tau_i per stage, or (kq == nullptr) a uniform constant-coefficient
// five-point stencil per stage, cs[i] = (S, W, C, E, N) of D_i.
template <typename T>
struct FineOp {
  int nx = 0, ny = 0;
  T pw = T(0);  // prolongation weight of the outermost fine node
  const T *kq = nullptr;
  const T *kc = nullptr;
  T tau[kMaxStages] = {};
  T cs[kMaxStages][5] = {};
};

// Scalars the Krylov kernels read from device memory so that a whole
// iteration can be replayed without host arguments changing.
struct KrylovState {
  int j;            // current iteration (column) index within the cycle
  int converged;    // set by the Givens kernel
  int breakdown;    // set by the Givens kernel
  int skip_reorth;  // set by the reorthogonalisation decision
};

namespace kern {

// f = g - K u (g may be null); V0[i*N + p] = f[p] for every stage i; per-block
// partial sums of f^2 into partial[blk].  nblk = ceil(N / kBlock).
void rhs_forward(const OpView<double> &K, const double *u, const double *g, int s, double *f,
                 double *V0, double *partial, hipStream_t st);

// V0 = given stage-major rhs (copy), partial sums of rhs^2.
void rhs_copy(const double *rhs, size_t n, double *V0, double *partial, hipStream_t st);

// scale[col] = 1 / sqrt(sum partial) (and norm_out = sqrt(sum) if non-null);
// single block.
void finalize_norm(const double *partial, int nblk, double *scale, int col, double *norm_out,
                   hipStream_t st);

// Block-substitution coupling for stage i of the preconditioner (Sec. 4.2):
//   b = scale_j * v_i - K( sum_{k in done} C[i*s+k] z_k )
// v = V_j (double, stage-major, lazily scaled by *scale_j); z = Z_j (T).
template <typename T>
void couple(const OpView<T> &K, const double *v, const double *scale_j, const T *z,
            const double *C, int s, int i, T *b, hipStream_t st);

// Fused V-cycle passes on one level (vcycle.hip): nu red-black Gauss-Seidel
// sweeps from zero, then rc = R (b - D x) (down); the same sweeps, x += P ec
// and nu post-sweeps (up).  nu in 1..3.
template <typename T>
void vdown(const OpView<T> &D, int nu, const T *b, T *rc, hipStream_t st);
template <typename T>
void vup(const OpView<T> &D, int nu, const T *b, const T *ec, T *x, hipStream_t st);
// The finest-level down pass with the stage coupling of Sec. 4.2 fused in:
// b = scale_j v_i - K (sum_k C[k] z_k) is formed in LDS, written to b_out for
// the up pass, smoothed and restricted.  v = V_j (double), z = Z_j (T).
template <typename T>
void vdown_couple(const OpView<T> &D, const OpView<T> &K, int nu, const double *v,
                  const double *scale_j, const T *z, const double *C, int s, int i, T *b_out,
                  T *rc, hipStream_t st);
// The same passes register-tiled per wavefront (wtile.hip): rows in
// registers, east/west neighbours through DPP lane shifts.
template <typename T>
bool wtile_ok(const OpView<T> &D);
template <typename T>
void wdown(const OpView<T> &D, int nu, const T *b, T *rc, hipStream_t st);
template <typename T>
void wdown_couple(const OpView<T> &D, const OpView<T> &K, int nu, const double *v,
                  const double *scale_j, const T *z, const double *C, int s, int i, T *b_out,
                  T *rc, hipStream_t st);
template <typename T>
void wup(const OpView<T> &D, int nu, const T *b, const T *ec, T *x, hipStream_t st);
// FP32 finest-level passes with two adjacent columns per lane (wsplit.hip):
// every lane updates one node per row in each colour half sweep.  Uniform
// five-point operators on grids with even nx and ny; `interior` is a host
// copy of the interior-class coefficients (9 entries) of D.
bool wsplit_ok(const OpView<float> &D);
void sdown(const OpView<float> &D, const float *interior, int nu, const float *b, float *rc,
           hipStream_t st);
void sup(const OpView<float> &D, const float *interior, int nu, const float *b, const float *ec,
         float *x, hipStream_t st);
// The same passes for a block without coupling terms: the right-hand side is
// float(*vscale * v) formed on load from the FP64 vector v.
void sdown_v(const OpView<float> &D, const float *interior, int nu, const double *v,
             const double *vscale, float *rc, hipStream_t st);
void sup_v(const OpView<float> &D, const float *interior, int nu, const double *v,
           const double *vscale, const float *ec, float *x, hipStream_t st);
// Nine-point constant-coefficient levels, two columns per lane, FP32 or
// FP64 (ws9.hip); `classes` is a host copy of the 81 class coefficients.
// The down pass stores its pre-smoothed x in xpre (a level-sized buffer),
// which the up pass starts from.  ws9_ok tells whether the level's grid
// shape fits the tiling (both passes must run these kernels).
template <typename T>
bool ws9_ok(const OpView<T> &D, int nu);
template <typename T>
void s9down(const OpView<T> &D, const T *classes, int nu, const T *b, T *rc, T *xpre,
            hipStream_t st);
template <typename T>
void s9up(const OpView<T> &D, const T *classes, int nu, const T *b, const T *ec, const T *xpre,
          T *x, hipStream_t st);
// Two adjacent nine-point levels F and C = F + 1 in one launch per direction
// (nu = 2, FP32 or FP64): s9down2 pre-smooths F from b, stores F's
// pre-smoothed x, C's right-hand side b_c and pre-smoothed x, and C's
// restricted residual rcc (the right-hand side of C + 1); s9up2 corrects C by
// ecc (the x of C + 1), post-smooths it and then F, writing F's x.  The same
// operations per node as s9down / s9up on F then C (and C then F).
// s9pair_ok tells whether the pair fits the tiling.
template <typename T>
bool s9pair_ok(const OpView<T> &Df, const OpView<T> &Dc, int nu);
// The last level of a cycle that ends above the coarsest level (nine-point
// classes, nu = 2): x = post-smoothing of the pre-smoothing from zero of b,
// the level's V-cycle with a zero coarse correction, in one pass.
template <typename T>
bool s9smooth_ok(const OpView<T> &D, int nu);
template <typename T>
void s9smooth(const OpView<T> &D, const T *classes, const T *b, T *x, hipStream_t st);
template <typename T>
void s9down2(const OpView<T> &Df, const T *cls_f, const OpView<T> &Dc, const T *cls_c,
             const T *b, T *xpre_f, T *b_c, T *xpre_c, T *rcc, hipStream_t st);
template <typename T>
void s9up2(const OpView<T> &Df, const T *cls_f, const OpView<T> &Dc, const T *cls_c, const T *b,
           const T *xpre_f, const T *b_c, const T *xpre_c, const T *ecc, T *x, hipStream_t st);
// b = scale_j v_i - K (sum_k C[k] z_k) for a uniform five-point K on an
// nx x ny grid with even nx (z and b float or double, FP64 arithmetic);
// k_interior is a host copy of K's interior coefficients.
template <typename T>
void scouple(int nx, int ny, const double *k_interior, const double *v, const double *scale_j,
             const T *z, const double *C, int s, int i, T *b, hipStream_t st);
// The true residual pass of residual_full for a uniform five-point K with
// even nx and M = I (hA: s x s row-major, host; k_interior as for scouple),
// in the coupling pass's streaming layout; V0, u_in/wts/u_out as there.
// Returns the number of block partials written to partial.
int residual_split(int nx, int ny, const double *k_interior, const double *x, const double *hA,
                   int s, const double *f, double *V0, double *partial, hipStream_t st,
                   const double *u_in, const double *wts, double *u_out);
// The same coupling with K stored per node (FP64 arrays, karr[k * N + p],
// five-point), wfine.hip.
template <typename T>
void scouple_var(int nx, int ny, const double *karr, const double *v, const double *scale_j,
                 const T *z, const double *C, int s, int i, T *b, hipStream_t st);
// Finest-level down pass of stage block `stage`: pre-smoothing from x = 0,
// rc = R (b - D x), and the pre-smoothed x of every node into xpre.  nx, ny
// even.  Up pass: x = xpre + P ec, then the post-smoothing (wfine.hip).
// v0 (device, may be null; b is then unused): the right-hand side is
// *v0scale times the FP64 vector v0, multiplied in FP64 and rounded to T on
// load (a block without coupling terms).
template <typename T>
void fdown(const FineOp<T> &F, int stage, int nu, const T *b, T *rc, T *xpre, hipStream_t st,
           const double *v0 = nullptr, const double *v0scale = nullptr);
template <typename T>
void fup(const FineOp<T> &F, int stage, int nu, const T *b, const T *xpre, const T *ec, T *x,
         hipStream_t st, const double *v0 = nullptr, const double *v0scale = nullptr);
// y[j] *= scale[j], j < k (left.hip).
void scale_by(double *y, const double *scale, int k, hipStream_t st);
// The FP32 tail with rows in registers (tail2.hip): levels of at most 64 x 64
// nodes; vtail2_ok tells whether td fits.
bool vtail2_ok(const TailDesc<float> &td);
void vtail2(const TailDesc<float> &td, int nu, const float *b, float *x, hipStream_t st);
size_t vtail2_lds_bytes(const TailDesc<float> &td);
// The whole V-cycle below (and including) the first tail level, one workgroup.
template <typename T>
size_t vtail_lds_bytes(const TailDesc<T> &td);
template <typename T>
void vtail(const TailDesc<T> &td, int nu, const T *b, T *x, hipStream_t st);

// Kronecker SpMM with fused classical Gram-Schmidt dots:
//   w = (I (x) M) z + (hA (x) K) z, z = Z_j (TZ, stage-major); M == nullptr: M = I
//   partial[m * nblk + blk] = block sum of <V_m, w> * scale_m, m = 0..j
// v0_bcast: V_0's s stage blocks are equal and only block 0 is read.
template <typename TZ>
void spmm_dots(const OpView<double> &K, const OpView<double> *M, const TZ *z, const double *hA,
               int s, const double *V, const double *scale, const KrylovState *ks, int jmax,
               double *partial, bool v0_bcast, hipStream_t st);

// w = (I (x) M) z + (hA (x) K) z recomputed; vout = w - sum_{m<=j} hcol[m] scale_m V_m;
// partial[blk] = block sum of vout^2.  v0_bcast as for spmm_dots.
template <typename TZ>
void spmm_update(const OpView<double> &K, const OpView<double> *M, const TZ *z, const double *hA,
                 int s, const double *V, const double *scale, const double *hcol,
                 const KrylovState *ks, double *vout, double *partial, bool v0_bcast,
                 hipStream_t st);

// Second Gram-Schmidt pass: partial dots of vin with V_0..V_j.
void vec_dots(const double *vin, size_t n, const double *V, const double *scale,
              const KrylovState *ks, int jmax, double *partial, hipStream_t st);
// vin -= sum_m h2[m] scale_m V_m; partial norms.
void vec_update(double *vin, size_t n, const double *V, const double *scale, const double *h2,
                const KrylovState *ks, double *partial, hipStream_t st);

// out[m] = sum_b partial[m * nblk + b] for m = 0..j+extra (one block per
// column); with honor_skip, nothing when the second pass is skipped.
void reduce_cols(const double *partial, int nblk, const KrylovState *ks, int jmax, int extra,
                 int honor_skip, double *out, hipStream_t st);

// Second-pass decision (0 never, 1 always, 2 DGKS) from the first pass's
// partial norms and ||w||^2 = h1[j+1]; stores ||v||^2 in norm_sq[0].
void reorth_decide(const double *partial_norm, int nblk, const double *h1, KrylovState *ks,
                   int mode, double *norm_sq, hipStream_t st);

// Single-block Hessenberg/Givens step for column j (see solver).  With
// first_only there is no second Gram-Schmidt pass: partial_norm/nblk are the
// first pass's partial norms and neither h2 nor norm_sq_first is read.
// host_resid receives {|g_{j+1}|, breakdown flag}: a device-accessible address
// of coherent pinned host memory, read by the host after the kernel completes.
void givens(const double *h1, const double *h2, const double *partial_norm, int nblk,
            const double *norm_sq_first, double *H, int ldh, double *cs, double *sn, double *g,
            double *scale, KrylovState *ks, double beta, double rtol, double *host_resid,
            bool first_only, hipStream_t st);

// Back substitution H y = g for the leading k x k block, single block.
void solve_upper(const double *H, int ldh, const double *g, int k, double *y, hipStream_t st);

// acc (double, s*N) += sum_{j<k} y_j Z_j  (Z stride zs elements per column);
// first: acc = sum_{j<k} y_j Z_j (acc is not read).
template <typename TZ>
void accumulate_solution(const TZ *Z, size_t zs, const double *y, int k, size_t n, double *acc,
                         bool first, hipStream_t st);

// u_out = u_in + sum_i wts[i] * x_i   (x stage-major double, wts = h b).
void combine_stages(const double *u_in, const double *x, const double *wts, int s, size_t N,
                    double *u_out, hipStream_t st);

// r = rhs - (I (x) M + hA (x) K) x; V0 = r (unless V0 == nullptr); partial
// norms.  rhs == nullptr with f given means rhs = 1 (x) f; M == nullptr means
// M = I.  u_out != nullptr: also u_out = u_in + sum_i wts[i] x_i, bit for bit
// what combine_stages writes (u_out must not overlap u_in or x).
void residual_full(const OpView<double> &K, const OpView<double> *M, const double *x,
                   const double *hA, int s, const double *rhs, const double *f, double *V0,
                   double *partial, hipStream_t st, const double *u_in = nullptr,
                   const double *wts = nullptr, double *u_out = nullptr);

// y = (I (x) M + hA (x) K) x for a double stage-major x (the Kronecker SpMM
// alone); M == nullptr means M = I.
void kron_apply(const OpView<double> &K, const OpView<double> *M, const double *x,
                const double *hA, int s, double *y, hipStream_t st);

// Stage values U_i = u + sum_j hA[i][j] k_j.
void stage_values(const double *u, const double *k, const double *hA, int s, size_t N, double *U,
                  hipStream_t st);

// lam_out = lam_in - K^T sum_i psi_i (K symmetric: K^T = K).
void adjoint_lambda(const OpView<double> &K, const double *lam_in, const double *psi, int s,
                    double *lam_out, hipStream_t st);

// rhs = wts (x) lam  (wts = h b), stage-major.
void scaled_broadcast(const double *lam, const double *wts, int s, size_t N, double *rhs,
                      hipStream_t st);

// Nodal gradient of the face-diffusion operator, accumulated into gnode
// ((nx+2) x (ny+2)): every face (P,Q) adds -1/2 h^-2 sum_i (psi_iP -
// psi_iQ)(U_iP - U_iQ) to both nodes.
void grad_nodes(const double *psi, const double *U, int s, int nx, int ny, double inv_h2,
                double *gnode, hipStream_t st);

// Face gradient of the face-diffusion operator, accumulated into gface:
// the x faces (ny rows of nx+1, face (i, j) between full-grid nodes (i, j+1)
// and (i+1, j+1)) followed by the y faces (ny+1 rows of nx, face (i, j)
// between (i+1, j) and (i+1, j+1)); each adds -h^-2 sum_i (psi_iP -
// psi_iQ)(U_iP - U_iQ).
void grad_faces(const double *psi, const double *U, int s, int nx, int ny, double inv_h2,
                double *gface, hipStream_t st);

// Count of non-finite entries (nonzero result = bad), via partial sums.
void nonfinite_check(const double *x, size_t n, double *partial, hipStream_t st);

}  // namespace kern
}  // namespace irk
