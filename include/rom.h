/*
 * rom.h -- C ABI of the MI355X (gfx950) library for inner-outer Krylov recycling in
 * diffuse optical tomography (O'Connell, Kilmer, de Sturler, Gugercin, arXiv:1602.00138).
 *
 * The three calls follow the paper's statement of the problem:
 *   rom_assemble_operator  -- the SPD zero-frequency operator A(p) = A_* + diag(mu(p))
 *                             of Sec. 3 / eq. (sum): finite differences of
 *                             -div(D grad eta) + mu eta with the Robin boundary
 *                             unknowns eliminated (Schur complement of eq. (block1)).
 *   rom_solve_sequence     -- Algorithm 2 (Sec. 4.3): solves A(p_i) X_i = [B~, C~]
 *                             (eq. (blkeqn)) for a sequence of parameter points with
 *                             recycled CG and grows the global basis V.
 *   rom_reduced_transfer   -- the reduced matrices of eq. (newreduced):
 *                             E_r = V^T V, A_r(p) = V^T A(p) V, B_r = V^T B~, C_r = V^T C~.
 *
 * Conventions
 *   - Grid: unit square (dim 2) or cube (dim 3), n[a] interior nodes on axis a at
 *     (i+1) h_a, h_a = 1/(n[a]+1); unknowns in x-fastest lexicographic order;
 *     N = n[0]*n[1]*n[2] (n[2] = 1 in 2D).
 *   - Faces -x,+x,-y,+y,-z,+z carry bc[] = 0 (Dirichlet, eq. (ModelPDE3)) or
 *     1 (Robin eta + 2 A D d(eta)/d(xi) = 0, eq. (ModelPDE2), first-order difference,
 *     eliminated: the face adds (D/h^2) h/(h + 2 A D) to the diagonal).
 *   - mu(x; p) = mu0 + sum_b amps[b] * psi(|x - centers[b]| / radii[b]),
 *     psi(t) = (1-t)^4 (4t+1) for t < 1 (compactly supported RBFs, Sec. 2.1, Sec. 5).
 *   - Sources B~ and detectors C~ are scaled identity columns (Sec. 3.1): column j
 *     is scale[j] * e_{idx[j]}.  The right-hand side block is [B~, C~], sources first.
 *   - All dense device matrices are column-major with leading dimension N.
 *
 * Memory: the library never allocates device memory.  The caller provides device
 * buffers (sizes from rom_operator_bytes / rom_sequence_bytes) and keeps them alive
 * for as long as a handle that refers to them is in use.  Handles themselves are
 * small host objects owned by the library and released with the *_destroy calls.
 *
 * Streams: every call enqueues its work on `stream` (a hipStream_t, NULL = default
 * stream).  rom_solve_sequence synchronises that stream at its decision points
 * (the skip test of Algorithm 2, CG convergence polls, the truncation test) and
 * returns when all its work is complete.  rom_assemble_operator and
 * rom_reduced_transfer return with their work enqueued (asynchronous).
 *
 * Errors: a call returns ROM_OK (0) or a negative status; rom_last_error() gives a
 * message for the calling thread.  Invalid arguments are rejected before any work is
 * enqueued.
 */
#ifndef ROM_H
#define ROM_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define ROM_API __attribute__((visibility("default")))
#else
#define ROM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef int rom_status;
#define ROM_OK 0
#define ROM_EINVAL (-1)     /* bad argument (shape, pointer, size) */
#define ROM_ENOTSPD (-2)    /* CG or Cholesky met a non-positive curvature / pivot */
#define ROM_ENONFINITE (-3) /* NaN or Inf in the iteration */
#define ROM_ENOCONV (-4)    /* some solve hit maxit (per-solve flags in the records) */
#define ROM_ECAPACITY (-5)  /* workspace too small */
#define ROM_EHIP (-6)       /* HIP runtime error */

#define ROM_NJ_MAX 64       /* max columns of a per-RHS recycle space U_j */
#define ROM_MAX_BUMPS 64

/* Arithmetic of the inner solves (rom_opts.precision).
 *   ROM_PREC_FP64:  Algorithm 2 entirely in FP64.
 *   ROM_PREC_MIXED: the inner recycled CG of each solve runs in FP32 (stencil products,
 *     projections onto U_j and all CG vectors in FP32 with FP32 sums) inside an FP64
 *     iterative refinement on the true residual: r = b - A x in FP64, an FP32 sweep
 *     solves A d = r / ||r|| to inner_tol, x += ||r|| d in FP64, until the FP64 residual
 *     meets tol.  A sweep that fails to halve the residual hands the solve to the FP64
 *     solver.  The outer projection, the skip test, the basis append, the truncation
 *     test, the Gram matrices and (U_j^T A U_j)^{-1} stay FP64, so every returned
 *     solution meets the same FP64 tolerance as in ROM_PREC_FP64. */
#define ROM_PREC_FP64 0
#define ROM_PREC_MIXED 1

typedef struct rom_operator rom_operator;
typedef struct rom_basis rom_basis;

typedef struct {
  int dim;          /* 2 or 3 */
  int n[3];         /* interior nodes per axis; n[2] = 1 when dim == 2 */
  int bc[6];        /* per face -x,+x,-y,+y,-z,+z: 0 Dirichlet, 1 Robin */
  double robin_A;   /* the constant A of eq. (ModelPDE2) */
} rom_grid;

typedef struct {
  int nb;                 /* number of RBF bumps (0 .. ROM_MAX_BUMPS) */
  const double* centers;  /* host, nb x dim, row-major */
  const double* radii;    /* host, nb */
  const double* amps;     /* host, nb */
  double mu0;             /* background absorption */
} rom_mu;

typedef struct {
  double tol;       /* relative residual tolerance ||b - A x|| <= tol ||b|| (Alg. 2 skip test and CG stop) */
  double trunc;     /* keep a new basis direction iff its norm outside range(V) > trunc (unit input) */
  double inner_tol; /* mixed precision: residual reduction asked of each FP32 sweep
                       (0: 1e-5; values below 1e-6 act as 1e-6) */
  int cap;          /* max basis columns (0: k_u + n_rhs * K) */
  int maxit;        /* max inner CG iterations per solve (0: N) */
  int check_every;  /* CG iterations between host convergence polls (0: 16) */
  int timing;       /* bit mask over ROM_K_* classes: time every launch of those classes with
                       HIP events (0: no events; algorithmic bytes are always counted) */
  int precision;    /* ROM_PREC_FP64 or ROM_PREC_MIXED */
  int group;        /* right-hand sides per batch, 1..16 (0: 1, the paper's order): the
                       members of a group are projected on V as it stands at the group
                       start, solved together, and appended in order afterwards */
  int tune;         /* 1: the first batch of each kind in the process times a few launch
                       shapes of the CG kernels and keeps the fastest (results then depend on
                       the chosen shape up to rounding); 0: fixed shape */
  int graph;        /* 1: the CG iterations run as replays of a captured HIP graph of 8 steps
                       (same kernels, same results; not used while a CG class is timed) */
  const float* guess; /* device, or NULL: an initial guess per (point i, RHS j), N values at
                       column (i (n_src + n_det) + j), any scale (e.g. the seed network's
                       output).  A solve that the outer test does not skip first moves to the
                       A(p_i)-optimal point of x0 + span(guess - x0) when that lowers the
                       residual; the correction appended to V and U_j is still x - x0.
                       With groups each member takes this step from the group's start. */
  const float* recycle; /* device, or NULL: n_recycle learned recycle vectors per point i, N
                       values each at column (i n_recycle + c).  At each point they are made
                       A(p_i)-orthogonal to V as it stands at the point start (the part the
                       outer projection cannot supply) and orthonormal among themselves, and
                       join the recycle space U_j of every right-hand side solved at that
                       point (not V); a vector with less than 1e-6 of its norm left is
                       dropped. */
  int n_recycle;    /* 1..16 when recycle is set */
  int cg_step;      /* launches per CG step: 0 chosen by the tuner when tune is set (else 1),
                       1 two (operator step, update), 2 one (the update of each step folded
                       into the next operator step; same recurrences, s, q and w then kept
                       in two buffers by step parity) */
} rom_opts;

/* One record per (point i, right-hand side j), in solve order. */
typedef struct {
  int point, rhs;
  double rho0;      /* relative residual after the outer projection on V */
  int its;          /* inner CG iterations (0 when skipped) */
  int solved;       /* 1 if the inner recycled CG ran */
  int kept;         /* 1 if the correction was appended to V */
  double rho;       /* norm of the normalised correction outside range(V) (-1 if not solved) */
  double final_res; /* true relative residual of the returned solution */
  int m;            /* basis size after this right-hand side */
  int restarts;     /* CG restarts from the true residual */
  int converged;    /* 1 if final_res <= tol */
  int fp64_sweeps;  /* mixed precision: refinement sweeps that fell back to the FP64 solver */
  double rho_guess; /* relative residual of the start after an initial guess (-1: none) */
} rom_record;

/* Instrumented kernel classes (event timing for the classes set in opts.timing). */
#define ROM_K_DCG_OP 0      /* CG operator step: w = A q - (A U_j) c and its dot products */
#define ROM_K_DCG_UPDATE 1  /* CG update: s -= a w, g += a q, q = s + b q, s^T s */
#define ROM_K_DCG_ENDS 2    /* start and end of each inner solve (g = U_j y0, g -= U_j e) */
#define ROM_K_GEMVT 3       /* V^T x (tall-skinny transposed products) */
#define ROM_K_GEMVN 4       /* V c (tall-skinny products) */
#define ROM_K_GRAM 5        /* V^T diag(w) V (FP64 MFMA) */
#define ROM_K_OUTER 6       /* outer projection x0 = V c (one per right-hand side) */
#define ROM_K_OTHER 7
#define ROM_K_DCG_STEP 8    /* one-launch CG step: update of step k-1 and operator step k */
#define ROM_NK 9

typedef struct {
  int m;                 /* final basis size */
  int k_u;               /* columns of U_0 kept after orthonormalisation */
  int n_solved, n_kept, n_dropped_trunc, n_dropped_cap, n_nonconv;
  long long total_its;
  double seconds;        /* host wall time of the call */
  double kernel_ms[ROM_NK];      /* summed event time per class (timed classes only) */
  double kernel_bytes[ROM_NK];   /* summed algorithmic bytes per class */
  double kernel_flops[ROM_NK];   /* summed algorithmic flops per class */
  long long kernel_launches[ROM_NK];
  int n_uj_capped;       /* kept corrections that did not join U_j because U_j already had
                            ROM_NJ_MAX columns (the paper's U_j grows without bound) */
} rom_stats;

/* Device bytes needed by rom_assemble_operator (variable_D = 1 for a per-node D). */
ROM_API rom_status rom_operator_bytes(const rom_grid* grid, int variable_D, size_t* bytes);

/* Assemble A_* (Sec. 3, eq. (sum)) into caller memory `op_mem` (device, >= bytes).
 * D_field == NULL: constant diffusion D_const (> 0).  Otherwise D_field is a device
 * array of N per-node values (> 0): an interior face takes the harmonic mean of its
 * two nodes, a boundary face the node value.  *op receives a host handle referring
 * to op_mem (and to D_field's values copied into op_mem). */
ROM_API rom_status rom_assemble_operator(const rom_grid* grid, double D_const, const double* D_field,
                                 void* op_mem, size_t op_bytes, rom_operator** op,
                                 void* stream);

/* Y[:, c] = A(p) X[:, c] for c < k, A(p) = A_* + diag(mu(p)) (eq. (sum)).
 * X, Y: device N x k, column-major (ld = N), must not overlap.  scratch: device,
 * >= 8*N bytes (holds the diagonal of A(p)).  Asynchronous on `stream`. */
ROM_API rom_status rom_apply_operator(const rom_operator* op, const rom_mu* p, const double* X,
                                      double* Y, int k, void* scratch, size_t scratch_bytes,
                                      void* stream);

/* Allocation-free form of rom_apply_operator, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same product Y[:, c] = A(p) X[:, c], c < k, with the
 * diagonal of A(p) kept in a device array owned by the library instead of caller scratch.
 * That array holds ROM_STATIC_MAX_N doubles (16 MiB) on every GPU the library runs on and
 * stays allocated until the process ends; its address is looked up once per device on
 * the first call there.  N > ROM_STATIC_MAX_N: ROM_ECAPACITY, before any work is enqueued.
 * Every call on one GPU uses that GPU's array, so calls that overlap on one GPU (other
 * streams or host threads) race on it: the caller serialises them.  X, Y as in
 * rom_apply_operator; asynchronous on `stream`; allocates nothing. */
#define ROM_STATIC_MAX_N (1 << 21)
ROM_API rom_status rom_apply_operator_static(const rom_operator* op, const rom_mu* p,
                                             const double* X, double* Y, int k, void* stream);

/* Device bytes of the workspace of rom_solve_sequence. */
ROM_API rom_status rom_sequence_bytes(const rom_operator* op, int n_src, int n_det, int k_u, int K,
                              const rom_opts* opts, size_t* bytes);

/* Algorithm 2 (CG form) over K parameter points params[0..K-1] (p_0 first).
 *   src_idx/src_scale, det_idx/det_scale: host arrays (n_src, n_det) describing B~, C~.
 *   U0: device N x k_u (offline estimates of the low eigenvectors of A(p_0); may be
 *       NULL when k_u == 0).  It is copied; the caller may reuse it.
 *   workspace: device, >= rom_sequence_bytes(...).  The returned basis refers to it.
 *   X_out: device N x (n_src+n_det) x K (column (i*(n_src+n_det) + j)), or NULL.
 *   records: host array of K*(n_src+n_det) entries, or NULL.
 *   stats: host, or NULL.
 * Returns ROM_OK, or ROM_ENOCONV if some solve reached maxit (its record says which),
 * or an error.  On success *basis receives the global basis handle. */
ROM_API rom_status rom_solve_sequence(rom_operator* op, const rom_mu* params, int K,
                              const int64_t* src_idx, const double* src_scale, int n_src,
                              const int64_t* det_idx, const double* det_scale, int n_det,
                              const double* U0, int k_u, const rom_opts* opts,
                              void* workspace, size_t ws_bytes, rom_basis** basis,
                              double* X_out, rom_record* records, rom_stats* stats,
                              void* stream);

/* Algorithm 2 one parameter point at a time, for callers whose points arrive one by one
 * (the iterates of an optimiser): the same method and results as rom_solve_sequence,
 * whose K points are rom_sequence_point calls in order.
 *   rom_sequence_begin: arguments as rom_solve_sequence; K is the most points the
 *     sequence will take (it sizes the workspace through rom_sequence_bytes and sets the
 *     default basis cap k_u + n_rhs K).  U0 is read during the first point (keep it alive
 *     until then).  All later work runs on `stream`.  *seq receives the handle.
 *   rom_sequence_point: the next point p (host); X_out (device, N x n_rhs, ld N, or NULL)
 *     receives its solutions, records (host, n_rhs entries, or NULL) its records.
 *     Returns when the point's work is complete: ROM_OK, ROM_ENOCONV (a solve of this point
 *     reached maxit), ROM_EINVAL past K points, or an error that stops the sequence (later
 *     calls other than rom_sequence_end then return ROM_EINVAL).
 *   rom_sequence_basis: the basis as it stands (a view into the workspace, for
 *     rom_reduced_transfer and the other basis calls; valid until the next call on seq).
 *   rom_sequence_stats: the totals so far (as rom_stats; seconds since begin).
 *   rom_sequence_end: releases seq; *basis (if not NULL) receives the global basis (as
 *     from rom_solve_sequence; NULL after an error) and *stats (if not NULL) the totals. */
typedef struct rom_sequence rom_sequence;
ROM_API rom_status rom_sequence_begin(rom_operator* op, int K, const int64_t* src_idx,
                                      const double* src_scale, int n_src, const int64_t* det_idx,
                                      const double* det_scale, int n_det, const double* U0,
                                      int k_u, const rom_opts* opts, void* workspace,
                                      size_t ws_bytes, rom_sequence** seq, void* stream);
ROM_API rom_status rom_sequence_point(rom_sequence* seq, const rom_mu* p, double* X_out,
                                      rom_record* records);
ROM_API rom_status rom_sequence_basis(rom_sequence* seq, const rom_basis** V);
ROM_API rom_status rom_sequence_stats(rom_sequence* seq, rom_stats* stats);
ROM_API rom_status rom_sequence_end(rom_sequence* seq, rom_basis** basis, rom_stats* stats);

/* Several independent sequences at once (e.g. one per grid of a set of uneven grids):
 * each job holds the arguments of one rom_solve_sequence call; every job runs on its own
 * host thread on its own stream (give each a different stream for the kernels of the
 * sequences to overlap on the GPU), on the device current for the calling thread.
 * job.status receives that job's status and job.message its error text.  Returns
 * ROM_OK, ROM_ENOCONV if some job reported it, or the first (in job order) other error
 * status.  Returns when every job has finished. */
typedef struct {
  rom_operator* op;
  const rom_mu* params;
  int K;
  const int64_t* src_idx;
  const double* src_scale;
  int n_src;
  const int64_t* det_idx;
  const double* det_scale;
  int n_det;
  const double* U0;
  int k_u;
  const rom_opts* opts;
  void* workspace;
  size_t ws_bytes;
  rom_basis** basis;
  double* X_out;
  rom_record* records;
  rom_stats* stats;
  void* stream;
  rom_status status;      /* out */
  char message[192];      /* out: error text of this job ("" if none) */
} rom_sequence_job;

ROM_API rom_status rom_solve_sequences(rom_sequence_job* jobs, int count);

/* Reduced matrices of eq. (newreduced) at parameter p for the basis V (m columns):
 *   Ar (m x m), Er (m x m), Br (m x n_src), Cr (m x n_det): device, column-major.
 * Any output pointer may be NULL to skip it.  scratch: device, >= rom_reduced_bytes. */
ROM_API rom_status rom_reduced_bytes(const rom_basis* V, size_t* bytes);
ROM_API rom_status rom_reduced_transfer(const rom_basis* V, const rom_mu* p, double* Ar, double* Br,
                                double* Cr, double* Er, void* scratch, size_t scratch_bytes,
                                void* stream);

/* Reduced Jacobian (eq. (newjac) with A~ and Delta_k replaced by their projections on V,
 * the derivative the interpolation theorem of Sec. 4 matches at the sample points):
 *   J_k = -C_r^T A_r(p)^{-1} (V^T diag(d mu / d p_k) V) A_r(p)^{-1} B_r
 * for every parameter of the bumps of p, per bump b in the order (amplitude a_b, radius
 * r_b, centre c_b[0] .. c_b[dim-1]): k = b (dim + 2) + j.  J: device, nb (dim + 2) blocks
 * of n_det x n_src (column-major, block k at J + k n_det n_src).  Computed as
 * -Z^T diag(d mu / d p_k) U with U = V A_r^{-1} B_r, Z = V A_r^{-1} C_r (the products in
 * a different order; each weighted product only reads the rows of one bump's support).
 * scratch: device, >= rom_reduced_jacobian_bytes.  Synchronises the stream on return
 * (it reports ROM_ENOTSPD if A_r(p) is not positive definite). */
ROM_API rom_status rom_reduced_jacobian_bytes(const rom_basis* V, size_t* bytes);
ROM_API rom_status rom_reduced_jacobian(const rom_basis* V, const rom_mu* p, double* J, void* scratch,
                                        size_t scratch_bytes, void* stream);

/* The k smallest eigenpairs of A(p) (the U_0 of Algorithm 2, Sec. 4.2.2, which the paper
 * computes offline), by Chebyshev-filtered subspace iteration on a block of kx >= k
 * columns (the extra ones are guards):
 *   X0: device N x kx (ld N), the starting block (e.g. smooth modes of the background);
 *   each sweep: Rayleigh-Ritz on the orthonormal block (a one-workgroup Jacobi
 *   eigensolver), then a degree-24 Chebyshev filter damping [largest Ritz value,
 *   Gershgorin bound b], then Cholesky QR twice;
 *   stops when every ||A u_i - lambda_i u_i|| <= tol * b (i < k), or after maxit sweeps.
 * U: device N x k (ld N), orthonormal; lambda: host, k values ascending; *sweeps: host
 * (may be NULL).  1 <= k <= kx <= 32; the filter's lower edge is the largest Ritz value of
 * the block, so column k converges at the rate of lambda_k / lambda_{kx+1}: give kx - k >= 2
 * guard columns (k == kx is accepted but its last column converges slowly).
 * Returns ROM_ENOCONV (U, lambda and *sweeps still written) if the residual test did not
 * pass within maxit sweeps.
 * scratch: device, >= rom_lowest_modes_bytes.
 * Synchronises the stream (it decides on the host after every sweep). */
ROM_API rom_status rom_lowest_modes_bytes(const rom_operator* op, int kx, size_t* bytes);
ROM_API rom_status rom_lowest_modes(const rom_operator* op, const rom_mu* p, int k,
                                    const double* X0, int kx, double tol, int maxit, double* U,
                                    double* lambda, int* sweeps, void* scratch,
                                    size_t scratch_bytes, void* stream);

/* Nonzero modulation frequency.  The systems of eq. (solves), (A(p) + i sigma I) X = B with
 * sigma = omega/nu, for ns shifts at once by multi-shift CG (one real CG on A(p) whose
 * residuals every shifted system shares up to a complex factor; each shift stops when its
 * residual <= tol ||b_j||, checked again on the FP64 true residual at exit):
 *   B: device N x nb (ld N), real right-hand sides; sigma: host, ns values (1 <= ns <= 8);
 *   Xr, Xi: device N x (nb * ns) (ld N), real and imaginary parts, column s * nb + j;
 *   its: host nb (may be NULL), iterations of the shared CG per right-hand side;
 *   resid: host nb * ns (may be NULL), true relative residuals, index s * nb + j.
 * Returns ROM_ENOCONV if some shift reached maxit (X then holds the last iterate),
 * ROM_ENOTSPD / ROM_ENONFINITE on breakdown.  scratch: >= rom_shifted_solve_bytes. */
ROM_API rom_status rom_shifted_solve_bytes(const rom_operator* op, int nb, int ns, size_t* bytes);
ROM_API rom_status rom_shifted_solve(const rom_operator* op, const rom_mu* p, const double* B,
                                     int nb, const double* sigma, int ns, double tol, int maxit,
                                     double* Xr, double* Xi, int* its, double* resid,
                                     void* scratch, size_t scratch_bytes, void* stream);
/* The reduced frequency response of the basis (the transfer function that follows eq.
 * (newreduced)), Psi_r(sigma) = C_r^T (i sigma E_r + A_r(p))^{-1} B_r with E_r = I (V has
 * orthonormal columns), for ns shifts (host array sigma).  Computed in real arithmetic:
 * y_r solves the SPD system (A_r + sigma^2 A_r^{-1}) y_r = B_r, y_i = -sigma A_r^{-1} y_r.
 * Psi_re, Psi_im: device n_det x n_src per shift (column-major), shift s at s*n_det*n_src.
 * scratch: >= rom_reduced_response_bytes. */
ROM_API rom_status rom_reduced_response_bytes(const rom_basis* V, size_t* bytes);
ROM_API rom_status rom_reduced_response(const rom_basis* V, const rom_mu* p, const double* sigma,
                                        int ns, double* Psi_re, double* Psi_im, void* scratch,
                                        size_t scratch_bytes, void* stream);

/* Basis queries: N, m, and a device copy of V (N x m, column-major, ld = N). */
ROM_API rom_status rom_basis_dims(const rom_basis* V, int64_t* N, int* m);
ROM_API rom_status rom_basis_copy(const rom_basis* V, double* dst, void* stream);

/* ---- Learned seed (not in the paper) -------------------------------------------------
 * A small 3D convolutional network on an nx x ny x nz grid (each a positive multiple of
 * 8): 4 levels (16, 32, 48, 64 channels), 3x3x3 convolutions with zero padding, 2x2x2
 * average pooling, 2x nearest upsampling, additive skips, ReLU:
 *   e0 = relu(conv(x; 3->16)), e1 = relu(conv(pool(e0); 16->32)),
 *   e2 = relu(conv(pool(e1); 32->48)), e3 = relu(conv(pool(e2); 48->64)),
 *   d2 = relu(conv(up(e3); 64->48) + e2), d1 = relu(conv(up(d2); 48->32) + e1),
 *   d0 = relu(conv(up(d1); 32->16) + e0), y = conv(d0; 16->outputs).
 * outputs = 1 for the initial-guess network, up to 16 for the recycle-vector network (one
 * output channel per vector).
 * Weights and activations are BF16 with FP32 accumulation (matrix cores); the master
 * parameters, gradients and Adam moments are FP32.  Parameters (host or device arrays
 * of nparams floats): per layer in the order e0 e1 e2 e3 d2 d1 d0 y, the weights
 * w[o][i][a][b][c] (multiplying input channel i at offset (a-1, b-1, c-1) in (z, y, x))
 * then the biases b[o].
 * Inputs: device FP32 [batch][3][N] (fields in the grid's x-fastest order); outputs (and
 * output gradients): device FP32 [batch][outputs][N]; targets (one-output networks):
 * device FP32 [batch][N], with the loss the mean over batch and voxels of (y - target)^2.  Memory is caller-owned: param_mem (>= param_bytes) and work_mem
 * (>= work_bytes, sized for up to `batch` samples per call), 256-byte aligned. */
typedef struct rom_seednet rom_seednet;
ROM_API rom_status rom_seednet_bytes(int nx, int ny, int nz, int batch, int outputs,
                             int64_t* nparams, size_t* param_bytes, size_t* work_bytes);
ROM_API rom_status rom_seednet_create(int nx, int ny, int nz, int batch, int outputs,
                              const float* params,
                              void* param_mem, size_t param_bytes, void* work_mem,
                              size_t work_bytes, rom_seednet** net, void* stream);
ROM_API rom_status rom_seednet_forward(rom_seednet* net, const float* in, float* out, int batch,
                               void* stream);
/* MSE loss and gradient (host array of nparams floats, or NULL) at the current parameters
 * (one-output networks; ROM_EINVAL otherwise). */
ROM_API rom_status rom_seednet_gradients(rom_seednet* net, const float* in, const float* target,
                                 int batch, float* grads, double* loss, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the batch; *loss (if not NULL)
 * receives the loss before the step. */
ROM_API rom_status rom_seednet_train_step(rom_seednet* net, const float* in, const float* target,
                                  int batch, float lr, double* loss, void* stream);
/* Gradient of any loss of the outputs: dy = d loss / d y (device FP32, [batch][outputs][N])
 * at the outputs of `in` is propagated back through the network; the parameter gradient
 * is kept for rom_seednet_adam and copied to grads (host, nparams floats) if not NULL. */
ROM_API rom_status rom_seednet_backward(rom_seednet* net, const float* in, const float* dy,
                                        int batch, float* grads, void* stream);
/* One Adam step with the gradient of the last rom_seednet_backward. */
ROM_API rom_status rom_seednet_adam(rom_seednet* net, float lr, void* stream);
ROM_API rom_status rom_seednet_params(const rom_seednet* net, float* params, void* stream);
/* Network inputs for `count` right-hand sides (unit columns at nodes idx[], host) at the
 * parameter point p of operator op: out (device FP32 [count][3][N]) receives
 * (mu(p) - mu0) / 0.03, log(D / 0.03) and the indicator of node idx[b] (all zero for
 * idx[b] = -1: the point-only input of the recycle-vector network).
 * scratch: device, >= 8 (N + count) bytes. */
ROM_API rom_status rom_seednet_inputs(const rom_operator* op, const rom_mu* p, const int64_t* idx,
                              int count, float* out, void* scratch, size_t scratch_bytes,
                              void* stream);
/* Subspace loss of the recycle-vector network for one parameter point: with N the k <= 16
 * outputs (device FP32 [k][N], i.e. N x k column-major), X the s solutions of that point
 * (device FP64, N x s, ld ldx) and x^_c = x_c / ||x_c||,
 *   loss = (1/s) sum_c ||x^_c - N (N^T N)^{-1} N^T x^_c||^2
 * (the share of the solutions outside span(N), invariant to N -> N S), and if dY is not
 * NULL its gradient -(2/s) R (N^T X^)^T (N^T N)^{-1}, R the residual block, into dY (device
 * FP32 [k][N]).  *loss: host.  ROM_ENOTSPD if the outputs are linearly dependent.
 * scratch: device, >= rom_subspace_loss_bytes. */
ROM_API rom_status rom_subspace_loss_bytes(int64_t N, int k, int s, size_t* bytes);
ROM_API rom_status rom_subspace_loss(const float* Y, int k, const double* X, int64_t N,
                                     int64_t ldx, int s, double* loss, float* dY, void* scratch,
                                     size_t scratch_bytes, void* stream);
/* Training targets: out[b][v] = X[v + b ldx] / max_v |X[v + b ldx]| (device; X FP64, out
 * FP32 [count][N]).  scratch: device, >= 512 count bytes. */
ROM_API rom_status rom_seednet_targets(const double* X, int64_t N, int64_t ldx, int count,
                               float* out, void* scratch, size_t scratch_bytes, void* stream);
ROM_API void rom_seednet_destroy(rom_seednet* net);

ROM_API void rom_operator_destroy(rom_operator* op);
ROM_API void rom_basis_destroy(rom_basis* V);
ROM_API const char* rom_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ROM_H */
