// Launchers for the gfx950 kernels (all FP64).  Each launcher enqueues on `st`.
#pragma once

#include "common.h"

namespace rom {

// Scalar state of one deflated-CG solve (one per member of a batch of right-hand sides;
// device memory, read back by the host at its convergence polls).
struct CGState {
  double gamma[2];     // s^T s by step parity (exact from the operator step; the update
                       // writes its recurrence estimate of the next one first)
  double pw;           // p^T A p of the latest direction
  double tol2;         // (tol * ||b||)^2
  double rscale;       // the right-hand side is read as rscale * r
  double alpha, beta;  // of the latest update
  double cGc;          // c^T (U^T A U) c of the latest direction (p = q - U c)
  double gcur;         // gamma of the latest operator step (read by the update)
  double t[NJ_MAX];    // U_j^T r (unscaled) for the start
  int nj;              // columns of U_j
  int its;             // updates done: written by the update, read by the operator step
  int maxit;
  int done;            // 1: stop (converged, maxit, breakdown, or inactive member)
  int flag;            // 0 ok, 1 non-positive curvature, 2 non-finite
  int kcur;            // index of the latest operator step: written by it, read by the
                       // update (no kernel reads a field that another block of the same
                       // launch may already have rewritten)
  // one-launch step only, by step parity (written by launch j at j & 1, read by launch
  // j + 1): updates done after the launch and c^T G c of its direction
  int its2[2];
  double cGc2[2];
};

// Per-member vectors of the deflated-CG recurrences (device memory beside the state).
// The direction is kept split as p_k = q_k - U c_k, and the correction as g = g_q - U e.
struct CGVec {
  double ts[NJ_MAX];     // (A U)^T s_k of the latest operator step
  double tw[NJ_MAX];     // (A U)^T w_k of the latest operator step
  double c[2][NJ_MAX];   // c_k by step parity
  double e[NJ_MAX];      // sum over the updates of alpha_k c_k
};

// Most right-hand sides solved together (members of one batch).
constexpr int G_MAX = 16;

// Per-member parameters of a batched CG start (members >= nb are ignored).
struct CgSetup {
  double tol2[G_MAX];
  double rscale[G_MAX];
  int maxit[G_MAX];
  int nj[G_MAX];
  int active[G_MAX];
};

// Launch shape of the stencil products: blocks of 256 plane nodes x zc planes.
struct StencilShape {
  dim3 grid;
  int zc;
  int blocks;
  int pairs = 0;   // CG operator step with two x-nodes per thread (grid.x counts pairs)
  int quads = 0;   // FP32 operator step with four x-nodes per thread (grid.x counts quads)
};
StencilShape stencil_shape(const Stencil& S, int target_blocks);
// Launch shape of the CG operator step (launch_dcg_op) for these buffers: the two-node
// walk when nx is even and every array is aligned for it (then grid.x and blocks count
// node pairs: the partials per member are `blocks`, at stride `blocks`); with quads (FP32
// only), the four-node walk where nx, the leading dimension and the alignment allow it
// (grid.x and blocks count groups of four nodes).
template <typename T>
StencilShape cg_apply_shape(const Stencil& S, int target_blocks, const T* diag, const T* p,
                            const T* w, int64_t vstride, const T* AW = nullptr,
                            bool quads = false);

// Absorption bumps of one parameter point, passed by value as a kernel argument.
struct Bumps {
  int nb;
  int dim;
  double mu0;
  double p[ROM_MAX_BUMPS * 5];  // per bump: centre (dim), radius, amplitude
};

// ---- operator -------------------------------------------------------------------
// D == NULL: constant D_const.  fx/fy/fz (per-node +face coefficients) may be NULL.
void launch_assemble(const rom_grid& g, double D_const, const double* D, double* diag_star,
                     double* fx, double* fy, double* fz, hipStream_t st);
// mu_i = mu0 + sum of bumps; diag_i = diag_star + mu_i (if diag_i); dmu = mu_i - mu0.
void launch_mu_eval(const Stencil& S, const Bumps& bumps, const double* diag_star,
                    double* diag_i, double* dmu, hipStream_t st);
// w[j ld + i] = -d mu(x_i) / d p_j for the dim + 2 parameters of bump b (amplitude,
// radius, centre coordinates), i < n.
void launch_mu_grad(const Stencil& S, const Bumps& bumps, int b, double* w, int64_t ld,
                    hipStream_t st);

// y = A x with A = stencil(S) + diag (diag holds the full diagonal).
void launch_spmv(const Stencil& S, const double* diag, const double* x, double* y,
                 hipStream_t st);
// out[:, v] = a A X[:, v] + b X[:, v] + c prev[:, v] for v < k (prev may be NULL; out may
// alias prev but not X): one fused step of a three-term recurrence.
void launch_cheb_step(const Stencil& S, const double* diag, const double* X, int64_t ld, int k,
                      double a, double b, double c, const double* prev, double* out,
                      hipStream_t st);
// Y[:, c] = A X[:, c] for c < k (contiguous, leading dimension ld).
void launch_spmm(const Stencil& S, const double* diag, const double* X, int64_t ld, int k,
                 double* Y, hipStream_t st);
// r = scale * e_idx - A x (b is a scaled unit column) and nrm2[0] = ||r||^2.
void launch_resid_unit(const Stencil& S, const double* diag, const double* x, int64_t idx,
                       double scale, double* r, double* nrm2, double* partials,
                       hipStream_t st);
// Columns z < nb at once: R[:, z] = scale[z] e_{idx[z]} - A X[:, z] (idx, scale on the
// device) and nrm2[z * nstride] = ||R[:, z]||^2.  partials: >= nb * stencil_shape(S,
// 512).blocks doubles.
void launch_resid_cols(const Stencil& S, const double* diag, const double* X, int64_t ldx, int nb,
                       const int64_t* idx, const double* scale, double* R, int64_t ldr,
                       double* nrm2, int64_t nstride, double* partials, hipStream_t st);
// out[r] = sum_b partials[b*R + r] for r < R (R = 1 or 2), one block, fixed order.
void launch_reduce_finish(const double* partials, int P, int R, double* out, hipStream_t st,
                          Skip skip = Skip());

// ---- tall-skinny products ---------------------------------------------------------
// out[v * cols + c] = sum_{r < rows} M[r + c * ld] * V[r + v * vstride], v < nv (nv <= 2).
// partials: >= gemvt_partials(rows, cols, nv) doubles.
size_t gemvt_partials(int64_t rows, int cols, int nv);
// max of gemvt_partials over every column count <= maxcols
size_t gemvt_partials_max(int64_t rows, int maxcols, int nv);
void launch_gemvt(const double* M, int64_t ld, int64_t rows, int cols, const double* V,
                  int64_t vstride, int nv, double* out, double* partials, hipStream_t st,
                  Skip skip = Skip());
// out[r] = alpha * in[r] + beta * sum_{c < cols} M[r + c * ld] coef[c]  (in may be NULL)
// and, if nrm2 != NULL, nrm2[0] = ||out||^2.  partials: >= 1024 doubles.
void launch_gemvn(const double* M, int64_t ld, int64_t rows, int cols, const double* coef,
                  double alpha, const double* in, double beta, double* out, double* nrm2,
                  double* partials, hipStream_t st, Skip skip = Skip());

// One basis pass for three products: out0 = in - M t (||out0||^2 into nrm2, device),
// out1 = M c1, out2 = M c2.  Needs gemvn_fused_ok (ld % 4 == 0, M 16-byte aligned,
// 3 cols doubles of LDS <= 64 KiB).  partials: >= 256 doubles.
bool gemvn_fused_ok(const double* M, int64_t ld, int cols);
void launch_gemvn_fused(const double* M, int64_t ld, int64_t rows, int cols, const double* t,
                        const double* c1, const double* c2, const double* in, double* out0,
                        double* out1, double* out2, double* nrm2, double* partials,
                        hipStream_t st);
// out = a + (u - w) * (cm[0] * s) (cm on the device).
void launch_fused_start(int64_t n, const double* a, const double* u, const double* w,
                        const double* cm, double s, double* out, hipStream_t st);
// Several right-hand sides at once: out[r + v*ldo] = alpha * in[r + v*ldi]
//   + beta * sum_{c < cols} M[r + c*ld] coef[c + v*ldc], v < nv <= 16 (in may be NULL).
void launch_gemvn_multi(const double* M, int64_t ld, int64_t rows, int cols, const double* coef,
                        int64_t ldc, int nv, double alpha, const double* in, int64_t ldi,
                        double beta, double* out, int64_t ldo, hipStream_t st);
// out[r + v*ldo] = a x[r + v*ldx] + b y[r + v*ldy] for r < n, v < nv (y may be NULL).
void launch_axpby_cols(int64_t n, int nv, double a, const double* x, int64_t ldx, double b,
                       const double* y, int64_t ldy, double* out, int64_t ldo, hipStream_t st);

// out[c] = ||X[:, c]||^2 for c < s (device).  partials: >= 256 * s doubles.
void launch_col_norms(int64_t n, int s, const double* X, int64_t ld, double* out,
                      double* partials, hipStream_t st);
// Gram borders of k new columns m .. m+k-1 from B = [V^T A_* Q_new | V^T A_i Q_new]
// ((m + k) x 2k, column-major, ld ldb), written to both triangles of G_* and G_i.
void launch_border_fill_block(const double* B, int64_t ldb, int m, int k, double* Gs, double* Gi,
                              int64_t ldg, hipStream_t st);

// ---- vector helpers ---------------------------------------------------------------
// out = a*x + b*y (y may be NULL); if nrm2: nrm2[0] = ||out||^2, nrm2[1] = ||y||^2.
// partials: >= 2048 doubles.
void launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* out,
                  double* nrm2, double* partials, hipStream_t st);
// x *= 1/sqrt(*nrm2)
void launch_normalize(int64_t n, double* x, const double* nrm2, hipStream_t st);
// bytes (a multiple of 8, at most 16 KiB) from device memory src into coherent pinned host
// memory dst, then seq stored at *flag (host memory) once every byte is visible to the host.
void launch_publish(const void* src, void* dst, size_t bytes, unsigned* flag, unsigned seq,
                    hipStream_t st);
// dst[:, c] = src[c] columns (pointer table) for c < k.
void launch_pack_cols(int64_t n, const ColPtrs& src, int k, double* dst, int64_t ld,
                      hipStream_t st);
// out[c] = scale * M[idx + c * ld] for c < cols (rows of a tall matrix at a node).
void launch_gather_row(const double* M, int64_t ld, int cols, int64_t idx, double scale,
                       double* out, hipStream_t st);
// Out[c + r*ldo] for c < cols, r < nidx: scale[r] * M[idx[r] + c * ld] (B_r = V^T B~).
void launch_gather_rows(const double* M, int64_t ld, int cols, const int64_t* idx,
                        const double* scale, int nidx, double* out, int64_t ldo,
                        hipStream_t st);

// ---- Gram matrices (FP64 MFMA) ----------------------------------------------------
// C = X^T diag(w) Y (w may be NULL = identity) for X: rows x a, Y: rows x b, contiguous
// column-major.  sym: X == Y, only the lower tiles are computed and mirrored.
// The result is written as C[i + j*ldc] = base[i + j*ldb] + shift*(i==j) + (X^T W Y)[i,j]
// (base may be NULL).  Rows whose weight is zero in a whole 32-row chunk are skipped.
size_t gram_partials(int a, int b, int64_t rows, bool sym);
// max of gram_partials over a' <= a (b' = a' when sym) -- the split count depends on a.
size_t gram_partials_max(int a, int b, int64_t rows, bool sym);
// C[i + v*ldc] = sum_r X[r + i*ldx] V[r + v*ldv] for i < a, v < nv <= 16 (MFMA).
// partials: >= proj_partials(a, nv, rows) doubles.
size_t proj_partials(int a, int nv, int64_t rows);
size_t proj_partials_max(int maxa, int nv, int64_t rows);
void launch_proj(const double* X, int64_t ldx, int a, const double* V, int64_t ldv, int nv,
                 int64_t rows, double* C, int64_t ldc, double* partials, hipStream_t st);
void launch_gram(const double* X, int64_t ldx, int a, const double* Y, int64_t ldy, int b,
                 int64_t rows, const double* w, bool sym, const double* base, int64_t ldb,
                 double shift, double* C, int64_t ldc, double* partials, hipStream_t st);

// ---- nonzero frequency: multi-shift CG for (A + i sigma I) X = B ---------------------
constexpr int MS_MAX = 8;   // shifts per call
struct MsShifts {
  int ns;
  double sigma[MS_MAX];
};
// Per right-hand side: the seed CG scalars and, per shift (complex, interleaved re/im),
// pi = R_k(-i sigma) (previous, current, next), zeta = 1/pi_cur and zeta_next = 1/pi_next,
// rho = pi_cur/pi_next, the shifted step alpha(s) and direction weight beta(s).  sdone[s]:
// shift converged (frozen).
struct MsState {
  double rr, bb, tol2, a_prev, b_prev, alpha, beta;
  double pi_prev[2 * MS_MAX], pi_cur[2 * MS_MAX], pi_next[2 * MS_MAX];
  double zeta[2 * MS_MAX], zeta_next[2 * MS_MAX], rho[2 * MS_MAX], as[2 * MS_MAX],
      bs[2 * MS_MAX];
  int sdone[MS_MAX];
  int its, maxit, flag, done;   // flag: 0 ok, 1 non-positive curvature, 2 non-finite
};
// Blocks of the vector kernels below (their partials: that many per column).
int ms_vec_blocks(int64_t n);
// r = p = B[:, j], P(s, j) = B[:, j] (imaginary part 0), X = 0; partials of b^T b.
void launch_ms_init(int64_t n, const double* B, int64_t ldb, int nb, int ns, double* r, double* p,
                    int64_t ld, double* Pr, double* Pi, double* Xr, double* Xi, int64_t ldx,
                    double* partials, hipStream_t st);
void launch_ms_start(const double* partials, int P, MsState* state, int nb, int ns, double tol,
                     int maxit, hipStream_t st);
// w = A p per live column, partials of p^T w; returns the partials per column (at most
// sh.blocks), which is what launch_ms_alpha must sum.
int launch_ms_apply(const Stencil& S, const StencilShape& sh, const double* diag, const double* p,
                    int64_t ld, double* w, int nb, const MsState* state, double* partials,
                    hipStream_t st);
void launch_ms_alpha(const double* partials, int P, MsState* state, int nb, const MsShifts& sh,
                     hipStream_t st);
void launch_ms_update(int64_t n, int nb, int ns, const double* w, double* r, int64_t ld,
                      double* Pr, double* Pi, double* Xr, double* Xi, int64_t ldx,
                      const MsState* state, double* partials, hipStream_t st);
void launch_ms_beta(const double* partials, int P, MsState* state, int nb, int ns,
                    hipStream_t st);
void launch_ms_dir(int64_t n, int nb, const double* r, double* p, int64_t ld,
                   const MsState* state, hipStream_t st);
// out[c] (c = s * nb + j) = ||Re(b_j - (A + i sigma_s) X_c)||^2 and out[nb*ns + c] the
// imaginary part's.  partials: >= 2 * nb * ns * shp.blocks doubles.
void launch_ms_resid(const Stencil& S, const StencilShape& shp, const double* diag,
                     const double* Xr, const double* Xi, int64_t ldx, const double* B, int64_t ldb,
                     int nb, const MsShifts& sh, double* partials, double* out, hipStream_t st);

// ---- lowest eigenpairs (U_0) ----------------------------------------------------------
// Eigenpairs of the symmetric m x m H (ld), m <= 32, by parallel-order Jacobi in one
// workgroup: lam ascending, Z (m x m, column-major) the matching unit eigenvectors.
void launch_sym_eig(const double* H, int64_t ld, int m, double* lam, double* Z, hipStream_t st);
// out[:, v] = a AY[:, v] + b Y[:, v] + c Y2[:, v] (Y2 may be NULL; out may alias Y or Y2).
void launch_comb3(int64_t n, int k, double a, const double* AY, double b, const double* Y,
                  double c, const double* Y2, int64_t ld, double* out, hipStream_t st);
// R[:, v] = AY[:, v] - lam[v] Y[:, v].
void launch_ritz_resid(int64_t n, int k, const double* AY, const double* Y, const double* lam,
                       int64_t ld, double* R, hipStream_t st);
// out[0] = max_i (2 diag_i - a1_i), with a1 = A 1: the Gershgorin bound of an operator whose
// off-diagonal entries are non-positive.  partials: >= 1024 doubles.
void launch_gersh(int64_t n, const double* diag, const double* a1, double* partials, double* out,
                  hipStream_t st);
void launch_transpose_small(int m, const double* in, double* out, hipStream_t st);
void launch_fill(int64_t n, double v, double* x, hipStream_t st);

// ---- inverse Cholesky factor -------------------------------------------------------
// Linv (lower, inverse of the Cholesky factor of G) kept in two layouts, Lc
// (column-major, ld) and Lr (its transpose, column-major, ld).  Border step k: with
// g = G[0:k, k] and d = G[k, k]: l = Linv g, delta^2 = d - l^T l,
// Linv[k, 0:k] = -(Linv^T l)^T / delta, Linv[k, k] = 1/delta.  status[0] is set to 1
// if delta^2 <= 0 (not SPD); the first such border also stores (k, d, l^T l) in info.
void launch_linv_border(double* Lc, double* Lr, int64_t ld, int k, const double* gcol,
                        double* tmp_l, double* tmp_r, int* status, double* partials,
                        hipStream_t st, double* info = nullptr);
// Rebuild Linv (both layouts, the whole m x m matrix including the zeros above the
// diagonal) from the m x m SPD matrix G in 64-column blocks: per block
// L21 = G21 Linv11^T, S = G22 - L21 L21^T, Linv22 = chol(S)^{-1},
// Linv21 = -Linv22 (L21 Linv11).  work: >= linv_rebuild_work(m) doubles (the last part
// holds the K-split slices of its products).
constexpr int GEMM_KSPLIT = 16;
inline size_t linv_rebuild_work(int m) {
  return 3 * 64 * 64 + 3 * 64 * (size_t)m + (size_t)GEMM_KSPLIT * 64 * (size_t)(m > 64 ? m : 64);
}
void launch_linv_rebuild(const double* G, int64_t ldg, int m, double* Lc, double* Lr,
                         double* work, int* status, hipStream_t st);
// C = alpha op(A) op(B) + beta D, column-major, op(A) M x K, op(B) K x N.  part
// (part_elems doubles, may be NULL): room for K-split slices of M x N; with it an output of
// few tiles and a long K is summed over K chunks in parallel, then the slices in order.
void launch_gemm(int M, int N, int K, double alpha, const double* A, int64_t lda, bool ta,
                 const double* B, int64_t ldb, bool tb, double beta, const double* D, int64_t ldd,
                 double* C, int64_t ldc, hipStream_t st, double* part = nullptr,
                 size_t part_elems = 0);
// c = Linv^T (Linv t), for m x m Linv.
void launch_linv_solve(const double* Lc, const double* Lr, int64_t ld, int m, const double* t,
                       double* u, double* c, double* partials, hipStream_t st);
// C[:, v] = Linv^T (Linv T[:, v]) for v < nv <= 3 (T at stride tstride; U and C at stride m).
void launch_linv_solve_multi(const double* Lc, const double* Lr, int64_t ld, int m, const double* T,
                             int64_t tstride, int nv, double* U, double* C, double* partials,
                             hipStream_t st);
// Rows r < n with w[r] != 0, ascending: idx[t] = r and wc[t] = w[r] for the first cap of
// them; *total = how many there are (device int, all of them).  work: ceil(n / 256) ints.
void launch_nz_rows(int64_t n, const double* w, int64_t* idx, double* wc, int64_t cap, int* total,
                    int* work, hipStream_t st);
// Vb[t + c ldb] = M[idx[t] + c ld] for t < cnt, c0 <= c < c1 (rows of a basis at given
// indices).
void launch_gather_idx(const double* M, int64_t ld, const int64_t* idx, int64_t cnt, int c0,
                       int c1, double* Vb, int64_t ldb, hipStream_t st);
// qb[t] = q[idx[t]] (qb may be NULL), zb[t] = wc[t] q[idx[t]] for t < cnt.
void launch_gather_scale(const double* q, const int64_t* idx, const double* wc, int64_t cnt,
                         double* qb, double* zb, hipStream_t st);
// The rest of a symmetric m x m Gram matrix G (col-major, ld = m, m <= NJ_MAX) whose
// columns k..m-1 are computed: G[0:k, 0:k] = Gs[0:k, 0:k] (ld lds), and the block below it
// G[k:m, 0:k] the transpose of G[0:k, k:m].
void launch_gram_assemble(const double* Gs, int lds, int k, double* G, int m, hipStream_t st);
// Small SPD m x m (m <= NJ_MAX) in one workgroup: Linv (inverse of its Cholesky factor)
// and Ginv (its inverse), col-major, ld = m.  status[0] = 1 if not SPD.
void launch_small_chol_inv(const double* G, int m, double* Linv, double* Ginv, int* status,
                           hipStream_t st);

// Symmetric border of the outer Gram matrices: for c <= k,
// Gs[c,k] = Gs[k,c] = vals[c] and Gi[c,k] = Gi[k,c] = vals[k+1+c].
void launch_border_fill(const double* vals, int k, double* Gs, double* Gi, int64_t ldg,
                        hipStream_t st);

// vals[c] = (h[c] - u[c]) / sqrt(nrm2[0]) and vals[k+1+c] = vals[c] + w[c] for c < k;
// vals[k] = d2[0], vals[2k+1] = d2[1] (the Gram border of a new basis column).
void launch_border_from_proj(const double* h, const double* u, const double* w,
                             const double* nrm2, const double* d2, int k, double* vals,
                             hipStream_t st);
// out2 = [x^T a, x^T b]; z = dmu o x.  partials: >= 2048 doubles.
void launch_dot2_scale(int64_t n, const double* x, const double* a, const double* b,
                       const double* dmu, double* z, double* out2, double* partials,
                       hipStream_t st);

// ---- deflated CG --------------------------------------------------------------------
// T = double (plain form) or float (inner sweeps of the mixed form).  A batch of nb
// members runs together; member y uses cg[y] / cv[y] (its nj, rscale, tol2, maxit), the
// recycle-space columns of slot y (Slots), Ginv / Gm + y*gstride (stride 0: one recycle
// space for every member), the FP64 right-hand side r + y*rstride (read as rscale * r) and
// its CG vectors at + y*vstride.  W, AW: n x nj column-major; Ginv, Gm: nj x nj FP64
// (W^T A W)^{-1} and W^T A W.  Inactive members (done set at setup) return at once from
// every kernel.
//
// Where column c of member y's W and AW sits: W + (c < ns ? soff : y*wstride) + c*ld.  The
// first ns columns (U_0 and A_i U_0 after the first point: the same in every member's
// recycle space) are read from one slot for all members, so that the members' blocks of
// one tile, which run on the same XCD, share them in its L2 instead of each reading its
// own copy from HBM.  ns = 0 (or soff = y*wstride) reads each member's own slot.
struct Slots {
  int64_t wstride;   // elements between members' slots (0: one slot for every member)
  int64_t ld;        // elements between columns
  int64_t soff;      // elements from the base to the slot holding the shared columns
  int ns;            // leading columns read from there
};
//
// A solve is: setup; start (g = U y0, s = q = r - AU y0, y0 = Ginv U^T r with U^T r in
// cg[y].t); then per step the operator kernel (the start's or the previous update's
// partials give gamma = s^T s, the stopping test, and c; w = A q - AU c with every dot
// product the update needs) and the update kernel (alpha, beta, s, g, q); finally
// g -= U e.  The step kernels take the step index from the state, so chunks of steps
// can be captured once and replayed.
int dcg_blocks(int64_t n);
// the width class (8, 16, 32 or 64 columns) the kernels are compiled for
int njt_of(int nj);
// values per block of the operator step's partials for width class njt
inline int dcg_op_values(int njt) { return 4 + 2 * njt; }
inline int dcg_iter_values(int njt) { return 5 + 2 * njt; }
void launch_cg_setup(CGState* cg, CGVec* cv, const CgSetup& su, int nb, hipStream_t st);
// P blocks per member; partials ps (NJ_MAX + 1 values per block, transposed) at stride
// psstride per member.
template <typename T>
void launch_dcg_start(const T* W, const T* AW, const Slots& sl, int64_t n, int njmax,
                      const double* Ginv, int64_t gstride, const double* r, int64_t rstride, T* g,
                      T* s, T* q, int64_t vstride, const CGState* cg, T* ps, int64_t psstride,
                      int nb, int P, hipStream_t st);
// The operator step on the launch shape sh (cg_apply_shape; sh.blocks partial rows of
// dcg_op_values(njt_of(njmax)) values per member at stride postride).  Ps: blocks of the
// start (its partials are read at the first step), Pu: blocks of the update kernel.
template <typename T>
void launch_dcg_op(const Stencil& S, const StencilShape& sh, const T* diag, const T* q,
                   const T* s, T* w, int64_t vstride, const T* AW, const Slots& sl,
                   int njmax, const double* Ginv, const double* Gm, int64_t gstride, CGState* cg,
                   CGVec* cv, const T* ps, int Ps, int64_t psstride, const T* pu, int Pu,
                   int64_t pustride, T* po, int64_t postride, int nb, hipStream_t st);
// The update on P blocks per member (1 <= P <= dcg_blocks(n)); P1 = the operator step's
// blocks.  narrow: half the rows per thread.
template <typename T>
void launch_dcg_update(T* q, const T* w, T* g, T* s, int64_t vstride, int64_t n, int njmax,
                       CGState* cg, CGVec* cv, const T* po, int P1, int64_t postride, T* pu,
                       int64_t pustride, int nb, int P, hipStream_t st, int narrow = 0);
// One whole CG step per launch (update of step j-1 and operator step j) on the operator
// step's shape sh.  s, q, w: two buffers each, parity p at + p pstride (the start writes
// s_0, q_0 into parity 0); step j (par = j & 1) reads parity 1 - par and writes par, and
// its partials (dcg_iter_values(njt_of(njmax)) values per member at stride postride) at
// po + par pohalf.  first: step 0 (par 0, reads the start's Ps partial rows); else Pprev
// = the previous step's blocks (sh.blocks).  g: the q part of the correction.
template <typename T>
void launch_dcg_iter(const Stencil& S, const StencilShape& sh, const T* diag, T* s, T* q, T* w,
                     int64_t pstride, int64_t vstride, T* g, const T* AW, const Slots& sl,
                     int njmax, const double* Ginv, const double* Gm,
                     int64_t gstride, CGState* cg, CGVec* cv, const T* ps, int Ps,
                     int64_t psstride, T* po, int64_t postride, int64_t pohalf, int Pprev,
                     int par, int first, int nb, hipStream_t st);
// g -= U e for every member (the U part of the split correction).
template <typename T>
void launch_dcg_finish(const T* W, const Slots& sl, int64_t n, int njmax, T* g,
                       int64_t vstride, const CGState* cg, const CGVec* cv, int nb,
                       hipStream_t st);

// Error reporting shared by the entry points of every subsystem (sets rom_last_error).
rom_status report(const Error& e);
void report_message(const std::string& m);

// ---- learned seed (3D convolutional network, BF16 with FP32 accumulation) -----------
// Activations: voxel-major BF16 with Cp channels (Cp a multiple of 8, pads zero); GEMM
// weights: BF16 [rows = round_up(cout, 16)][Kp = round_up(27 Cpi, 32)].
int seed_round8(int c);
int seed_kp(int cp);
// up != 0: X is on the grid of half the size (even nx, ny, nz) and the layer reads its
// 2x nearest-neighbour upsampling.
void launch_seed_conv(int nx, int ny, int nz, int batch, const void* X, int Cpi, const void* W,
                      int Kp, int Cout, int rows, const float* bias, const void* skip, int relu,
                      void* Y, int Cpo, hipStream_t st, int up = 0);
size_t seed_wgrad_partials(int nx, int ny, int nz, int batch, int rows, int Kp);
void launch_seed_wgrad(int nx, int ny, int nz, int batch, const void* X, int Cpi, const void* dZ,
                       int Cpo, int Cout, int rows, int Kp, float* P, float* dWg, float* Pb,
                       float* db, hipStream_t st, int up = 0);
void launch_seed_pool(int nx, int ny, int nz, int batch, const void* X, void* Y, int C,
                      hipStream_t st);
void launch_seed_pool_bwd(int nx, int ny, int nz, int batch, const void* dY, void* dX, int C,
                          int acc, hipStream_t st);
void launch_seed_up_bwd(int nx, int ny, int nz, int batch, const void* dY, void* dX, int C,
                        hipStream_t st);
void launch_seed_relu_bwd(int64_t ne, void* dY, const void* Y, hipStream_t st);
void launch_seed_add(int64_t ne, void* out, const void* in, hipStream_t st);
void launch_seed_pack_input(int64_t nvox, int batch, int cin, const float* in, void* X, int Cp,
                            hipStream_t st);
void launch_seed_unpack_output(int64_t nvox, int batch, int cout, const void* Y, int Cp,
                               float* out, hipStream_t st);
void launch_seed_mse(int64_t ne, const void* Y, int Cp, const float* tgt, void* dY,
                     double* partials, double* loss, hipStream_t st);
void launch_seed_adam(int64_t n, float* p, const float* g, float* m, float* v, float lr, float b1,
                      float b2, float c1, float c2, float eps, hipStream_t st);
void launch_seed_pack_weights(const float* w, int cout, int cin, int Cpi, int Kp, int rows,
                              void* Wb, int Cpo, int Ktp, int rowst, void* Wt, hipStream_t st);
void launch_seed_unpack_wgrad(const float* dWg, int Kp, int cout, int cin, int Cpi, float* dw,
                              hipStream_t st);

// Seed-network inputs [dmu/mu_scale, log(D/Dref), indicator of idx[b]] for count
// right-hand sides (out: FP32 [count][3][n]; D NULL: constant Dc; idx on the device).
void launch_seed_inputs(int64_t n, int count, const double* dmu, double mu_scale, const double* D,
                        double Dc, double Dref, const int64_t* idx, float* out, hipStream_t st);
// Training targets out[b][v] = X[v + b ldx] / max |X[:, b]|.  part: >= 64 count doubles.
void launch_seed_targets(int64_t n, int count, const double* X, int64_t ldx, double* part,
                         float* out, hipStream_t st);
// d = xg - x0 (guess direction; xg FP32)
void launch_guess_dir(int64_t n, const float* xg, const double* x0, double* d, hipStream_t st);

// ---- mixed form -----------------------------------------------------------------------
// out[i] = (float) in[i], i < n.
void launch_cast_f32(int64_t n, const double* in, float* out, hipStream_t st);
// out[i + c*ldo] = in[i + c*ldi] converted, for i < n, c < k.
void launch_convert_cols(int64_t n, int k, const float* in, int64_t ldi, double* out, int64_t ldo,
                         hipStream_t st);
void launch_convert_cols(int64_t n, int k, const double* in, int64_t ldi, float* out, int64_t ldo,
                         hipStream_t st);
// out[:, c] = in[:, c] / sqrt(norm2[c]) for c < k (norm2 on the device; 0 gives 0).
void launch_scale_cols(int64_t n, int k, const double* in, int64_t ldi, const double* norm2,
                       double* out, int64_t ldo, hipStream_t st);
// out[i + c*ld] = (float) in[i + c*ld] for i < n, c < k.
void launch_cast_cols_f32(int64_t n, int k, const double* in, int64_t ld, float* out,
                          hipStream_t st);
// Batched refinement step, columns y < nb: g[:, y] += coef.c[y] d[:, y] (d of type T;
// c = 0 leaves g), x[:, y] = x0[:, y] + g[:, y].  g, x0 at stride ld, d at ldd, x at ldx.
struct Coefs {
  double c[G_MAX];
};
template <typename T>
void launch_refine_cols(int64_t n, int nb, const Coefs& coef, const T* d, int64_t ldd, double* g,
                        const double* x0, int64_t ld, double* x, int64_t ldx, hipStream_t st);
// One refinement step: g += sigma * d (d FP32), x = x0 + g (FP64).
void launch_refine_update(int64_t n, double sigma, const float* d, double* g, const double* x0,
                          double* x, hipStream_t st);

}  // namespace rom
