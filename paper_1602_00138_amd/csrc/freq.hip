// Nonzero modulation frequency: the shifted systems (A(p) + i sigma I) X = B of eq.
// (solves), sigma = omega/nu, for several sigma at once by multi-shift CG.
//
// A is real SPD and the shift is a multiple of I, so every shifted system has the same
// Krylov space as the seed A x = b, and its CG residuals are scalar multiples of the
// seed's: r_k(sigma) = zeta_k r_k with zeta_k = 1 / R_k(-i sigma), R_k the seed's residual
// polynomial.  R_k(-i sigma) follows the seed's three-term recurrence evaluated at
// t = -i sigma, and the shifted step lengths and direction weights follow from it:
// alpha_k(s) = alpha_k R_k(-s) / R_{k+1}(-s), beta_k(s) = (R_k(-s) / R_{k+1}(-s))^2 beta_k
// (the multi-shift CG of Frommer and Maass / Jegerlehner).  One real stencil product per
// iteration serves every shift; each shift costs a complex solution and a complex
// direction (four real vectors).  A shift stops updating once its residual meets the
// tolerance, which also keeps R_k(-s) bounded by about 1/tol.
//
// Per iteration k and column: k_ms_apply (w = A p and p^T w), k_ms_alpha (seed step and
// the shifted scalars), k_ms_update (the shifted direction P(s)_k = zeta_k r_k +
// beta(s)_{k-1} P(s)_{k-1} formed where r_k is read anyway, X(s) += alpha(s)_k P(s)_k, then
// r -= alpha w and r^T r), k_ms_beta (beta, per-shift convergence), k_ms_dir (the seed's
// p).  Columns (right-hand sides) ride on the grid's last dimension, each with its own
// scalars in MsState.
#include "kernels.h"

namespace rom {

namespace {

constexpr int BS = 256;

struct Cx {
  double re, im;
};
__device__ __forceinline__ Cx cmul(Cx a, Cx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ Cx cinv(Cx a) {
  // 1/a scaled to avoid overflow of |a|^2
  const double s = fmax(fabs(a.re), fabs(a.im));
  const double ar = a.re / s, ai = a.im / s;
  const double d = s * (ar * ar + ai * ai);
  return {ar / d, -ai / d};
}

__global__ void k_ms_init(int64_t n, const double* __restrict__ B, int64_t ldb, int nb, int ns,
                          double* __restrict__ r, double* __restrict__ p, int64_t ld,
                          double* __restrict__ Pr, double* __restrict__ Pi,
                          double* __restrict__ Xr, double* __restrict__ Xi, int64_t ldx,
                          double* __restrict__ partials) {
  const int j = blockIdx.y;
  double acc[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    const double v = B[i + j * ldb];
    r[i + j * ld] = v;
    p[i + j * ld] = v;
    for (int s = 0; s < ns; ++s) {
      const int64_t c = (int64_t)s * nb + j;
      Pr[i + c * ld] = 0.0;   // P(s)_{-1}: weighted by beta(s)_{-1} = 0 in the first update
      Pi[i + c * ld] = 0.0;
      Xr[i + c * ldx] = 0.0;
      Xi[i + c * ldx] = 0.0;
    }
    acc[0] += v * v;
  }
  write_partials<1, BS>(acc, partials + (int64_t)j * gridDim.x, blockIdx.x);
}

__global__ void k_ms_start(const double* __restrict__ partials, int P, MsState* st, int ns,
                           double tol, int maxit) {
  __shared__ double tot[1];
  sum_partials<1, BS>(partials + (int64_t)blockIdx.x * P, P, tot);
  if (threadIdx.x == 0) {
    MsState& m = st[blockIdx.x];
    const double rr = tot[0];
    m.rr = rr;
    m.bb = rr;
    m.tol2 = tol * tol * rr;
    m.a_prev = 1.0;
    m.b_prev = 0.0;
    m.alpha = 0.0;
    m.beta = 0.0;
    for (int s = 0; s < MS_MAX; ++s) {
      m.pi_prev[2 * s] = m.pi_cur[2 * s] = 1.0;
      m.pi_prev[2 * s + 1] = m.pi_cur[2 * s + 1] = 0.0;
      m.zeta[2 * s] = 1.0;   // zeta_0
      m.zeta[2 * s + 1] = 0.0;
      m.bs[2 * s] = m.bs[2 * s + 1] = 0.0;
      m.sdone[s] = s < ns ? (rr > 0.0 ? 0 : 1) : 1;
    }
    m.its = 0;
    m.maxit = maxit;
    m.flag = rr == rr ? 0 : 2;
    m.done = (rr > 0.0 && m.flag == 0) ? 0 : 1;
  }
}

// w = A p; partial p^T w per block.  Threads outside the plane still join the block sum.
template <bool VAR>
__global__ __launch_bounds__(BS) void k_ms_apply(Stencil S, const double* __restrict__ diag,
                                                  const double* __restrict__ p0, int64_t ld,
                                                  double* __restrict__ w0, int zc,
                                                  const MsState* __restrict__ st,
                                                  double* __restrict__ partials) {
  if (st[blockIdx.z].done) return;
  const double* __restrict__ p = p0 + (int64_t)blockIdx.z * ld;
  double* __restrict__ w = w0 + (int64_t)blockIdx.z * ld;
  const int q = blockIdx.x * BS + threadIdx.x;
  const int z0 = blockIdx.y * zc;
  const int z1 = min(z0 + zc, S.nz);
  double acc[1] = {0.0};
  if (q < S.nx * S.ny && z0 < z1)
    stencil_walk<VAR>(S, diag, p, q, z0, z1, [&](int64_t i, double ax, double xi) {
      w[i] = ax;
      acc[0] += xi * ax;
    });
  write_partials<1, BS>(acc, partials + (int64_t)blockIdx.z * gridDim.x * gridDim.y,
                        blockIdx.x + gridDim.x * blockIdx.y);
}

// k_ms_apply with two x-nodes per thread (even nx, 16-byte aligned columns).
template <bool VAR>
__global__ __launch_bounds__(BS) void k_ms_apply2(Stencil S, const double* __restrict__ diag,
                                                   const double* __restrict__ p0, int64_t ld,
                                                   double* __restrict__ w0, int zc,
                                                   const MsState* __restrict__ st,
                                                   double* __restrict__ partials) {
  if (st[blockIdx.z].done) return;
  const double* __restrict__ p = p0 + (int64_t)blockIdx.z * ld;
  double* __restrict__ w = w0 + (int64_t)blockIdx.z * ld;
  const int q = blockIdx.x * BS + threadIdx.x;
  const int z0 = blockIdx.y * zc;
  const int z1 = min(z0 + zc, S.nz);
  double acc[1] = {0.0};
  if (q < (S.nx / 2) * S.ny && z0 < z1)
    stencil_walk2<VAR>(S, diag, p, q, z0, z1,
                       [&](int64_t i, double v0, double v1, double x0i, double x1i) {
                         *reinterpret_cast<double2*>(w + i) = double2{v0, v1};
                         acc[0] += x0i * v0 + x1i * v1;
                       });
  write_partials<1, BS>(acc, partials + (int64_t)blockIdx.z * gridDim.x * gridDim.y,
                        blockIdx.x + gridDim.x * blockIdx.y);
}

// Seed step length, then per live shift: pi_next = (1 + c + i alpha sigma) pi_cur - c pi_prev
// with c = alpha beta_prev / alpha_prev; rho = pi_cur / pi_next; alpha(s) = alpha rho;
// zeta_next = 1 / pi_next (zeta, the current one, is still read by the update).
__global__ void k_ms_alpha(const double* __restrict__ partials, int P, MsState* st,
                           MsShifts sh) {
  MsState& m = st[blockIdx.x];
  if (m.done) return;
  __shared__ double tot[1];
  sum_partials<1, BS>(partials + (int64_t)blockIdx.x * P, P, tot);
  if (threadIdx.x != 0) return;
  const double pw = tot[0];
  if (!(pw > 0.0)) {
    m.flag = pw == pw ? 1 : 2;
    m.done = 1;
    return;
  }
  const double alpha = m.rr / pw;
  const double c = alpha * m.b_prev / m.a_prev;
  m.alpha = alpha;
  for (int s = 0; s < sh.ns; ++s) {
    if (m.sdone[s]) continue;
    const Cx cur = {m.pi_cur[2 * s], m.pi_cur[2 * s + 1]};
    const Cx prev = {m.pi_prev[2 * s], m.pi_prev[2 * s + 1]};
    const Cx z = {1.0 + c, alpha * sh.sigma[s]};
    Cx nxt = cmul(z, cur);
    nxt.re -= c * prev.re;
    nxt.im -= c * prev.im;
    const Cx zeta = cinv(nxt);
    const Cx rho = cmul(cur, zeta);
    m.pi_next[2 * s] = nxt.re;
    m.pi_next[2 * s + 1] = nxt.im;
    m.zeta_next[2 * s] = zeta.re;
    m.zeta_next[2 * s + 1] = zeta.im;
    m.rho[2 * s] = rho.re;
    m.rho[2 * s + 1] = rho.im;
    m.as[2 * s] = alpha * rho.re;
    m.as[2 * s + 1] = alpha * rho.im;
  }
}

// For the live shifts P(s) = zeta r + beta(s) P(s) and X(s) += alpha(s) P(s); then
// r -= alpha w (partial r^T r).
__global__ void k_ms_update(int64_t n, int nb, const double* __restrict__ w,
                            double* __restrict__ r, int64_t ld, double* __restrict__ Pr,
                            double* __restrict__ Pi, double* __restrict__ Xr,
                            double* __restrict__ Xi, int64_t ldx, const MsState* __restrict__ st,
                            int ns, double* __restrict__ partials) {
  const int j = blockIdx.y;
  const MsState& m = st[j];
  if (m.done) return;
  const double alpha = m.alpha;
  double acc[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    const double r0 = r[i + j * ld];
    for (int s = 0; s < ns; ++s) {
      if (m.sdone[s]) continue;
      const int64_t c = (int64_t)s * nb + j;
      const double zr = m.zeta[2 * s], zi = m.zeta[2 * s + 1];
      const double br = m.bs[2 * s], bi = m.bs[2 * s + 1];
      const double qr = Pr[i + c * ld], qi = Pi[i + c * ld];
      const double pr = zr * r0 + br * qr - bi * qi;
      const double pi = zi * r0 + br * qi + bi * qr;
      Pr[i + c * ld] = pr;
      Pi[i + c * ld] = pi;
      const double ar = m.as[2 * s], ai = m.as[2 * s + 1];
      Xr[i + c * ldx] += ar * pr - ai * pi;
      Xi[i + c * ldx] += ar * pi + ai * pr;
    }
    const double rv = r0 - alpha * w[i + j * ld];
    r[i + j * ld] = rv;
    acc[0] += rv * rv;
  }
  write_partials<1, BS>(acc, partials + (int64_t)j * gridDim.x, blockIdx.x);
}

// beta = r'^T r' / r^T r; per live shift beta(s) = rho^2 beta and the convergence test
// |zeta|^2 r'^T r' <= tol^2 b^T b; then the recurrence history moves one step.
__global__ void k_ms_beta(const double* __restrict__ partials, int P, MsState* st, int ns) {
  MsState& m = st[blockIdx.x];
  if (m.done) return;
  __shared__ double tot[1];
  sum_partials<1, BS>(partials + (int64_t)blockIdx.x * P, P, tot);
  if (threadIdx.x != 0) return;
  const double rr = tot[0];
  if (!(rr == rr) || !(rr < INFINITY)) {
    m.flag = 2;
    m.done = 1;
    return;
  }
  const double beta = rr / m.rr;
  m.beta = beta;
  int live = 0;
  for (int s = 0; s < ns; ++s) {
    if (m.sdone[s]) continue;
    const Cx rho = {m.rho[2 * s], m.rho[2 * s + 1]};
    const Cx r2 = cmul(rho, rho);
    m.bs[2 * s] = r2.re * beta;
    m.bs[2 * s + 1] = r2.im * beta;
    const double zr = m.zeta_next[2 * s], zi = m.zeta_next[2 * s + 1];
    if ((zr * zr + zi * zi) * rr <= m.tol2) m.sdone[s] = 1;
    else ++live;
    m.zeta[2 * s] = zr;
    m.zeta[2 * s + 1] = zi;
    m.pi_prev[2 * s] = m.pi_cur[2 * s];
    m.pi_prev[2 * s + 1] = m.pi_cur[2 * s + 1];
    m.pi_cur[2 * s] = m.pi_next[2 * s];
    m.pi_cur[2 * s + 1] = m.pi_next[2 * s + 1];
  }
  m.rr = rr;
  m.a_prev = m.alpha;
  m.b_prev = beta;
  m.its += 1;
  if (live == 0 || m.its >= m.maxit) m.done = 1;
}

// The seed's direction p = r + beta p.
__global__ void k_ms_dir(int64_t n, int nb, const double* __restrict__ r, double* __restrict__ p,
                         int64_t ld, const MsState* __restrict__ st) {
  const int j = blockIdx.y;
  const MsState& m = st[j];
  if (m.done) return;
  const double beta = m.beta;
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
    p[i + j * ld] = r[i + j * ld] + beta * p[i + j * ld];
}

// True residual of column c = s * nb + j, one plane at a time:
//   PLANE 0: t = b_j - A Xr + sigma_s Xi,   PLANE 1: t = -(A Xi) - sigma_s Xr,
// partial sum of t^2 at partials[(PLANE * gridDim.z + c) * P + block].
template <bool VAR, int PLANE>
__global__ __launch_bounds__(BS) void k_ms_resid(Stencil S, const double* __restrict__ diag,
                                                  const double* __restrict__ Xr,
                                                  const double* __restrict__ Xi, int64_t ldx,
                                                  const double* __restrict__ B, int64_t ldb,
                                                  int nb, MsShifts sh, int zc,
                                                  double* __restrict__ partials) {
  const int c = blockIdx.z;
  const int j = c % nb, s = c / nb;
  const double sigma = sh.sigma[s];
  const double* __restrict__ xr = Xr + (int64_t)c * ldx;
  const double* __restrict__ xi = Xi + (int64_t)c * ldx;
  const double* __restrict__ b = B + (int64_t)j * ldb;
  const int q = blockIdx.x * BS + threadIdx.x;
  const int z0 = blockIdx.y * zc;
  const int z1 = min(z0 + zc, S.nz);
  double acc[1] = {0.0};
  if (q < S.nx * S.ny && z0 < z1) {
    if (PLANE == 0)
      stencil_walk<VAR>(S, diag, xr, q, z0, z1, [&](int64_t i, double ax, double) {
        const double t = b[i] - ax + sigma * xi[i];
        acc[0] += t * t;
      });
    else
      stencil_walk<VAR>(S, diag, xi, q, z0, z1, [&](int64_t i, double ax, double) {
        const double t = ax + sigma * xr[i];
        acc[0] += t * t;
      });
  }
  const int P = gridDim.x * gridDim.y;
  write_partials<1, BS>(acc, partials + ((int64_t)PLANE * gridDim.z + c) * P,
                        blockIdx.x + gridDim.x * blockIdx.y);
}

// out[c] = sum_b partials[c * P + b], one block per row c.
__global__ void k_ms_sum_rows(const double* __restrict__ partials, int P, double* out) {
  __shared__ double tot[1];
  sum_partials<1, BS>(partials + (int64_t)blockIdx.x * P, P, tot);
  if (threadIdx.x == 0) out[blockIdx.x] = tot[0];
}

int vec_grid(int64_t n) {
  const int64_t g = (n + BS - 1) / BS;
  return (int)std::min<int64_t>(g, 1024);
}

}  // namespace

int ms_vec_blocks(int64_t n) { return vec_grid(n); }

void launch_ms_init(int64_t n, const double* B, int64_t ldb, int nb, int ns, double* r, double* p,
                    int64_t ld, double* Pr, double* Pi, double* Xr, double* Xi, int64_t ldx,
                    double* partials, hipStream_t st) {
  ROM_LAUNCH(k_ms_init, dim3(vec_grid(n), nb), dim3(BS), 0, st, n, B, ldb, nb, ns, r, p, ld, Pr,
             Pi, Xr, Xi, ldx, partials);
}

void launch_ms_start(const double* partials, int P, MsState* state, int nb, int ns, double tol,
                     int maxit, hipStream_t st) {
  ROM_LAUNCH(k_ms_start, dim3(nb), dim3(BS), 0, st, partials, P, state, ns, tol, maxit);
}

int launch_ms_apply(const Stencil& S, const StencilShape& sh, const double* diag, const double* p,
                    int64_t ld, double* w, int nb, const MsState* state, double* partials,
                    hipStream_t st) {
  if (stencil_pairs_ok(S, ld, {diag, p, w})) {
    // half the x-blocks of sh (at most sh.blocks partials per column)
    const dim3 grid2(ceil_div((int64_t)(S.nx / 2) * S.ny, BS), sh.grid.y, nb);
    if (S.var)
      ROM_LAUNCH(k_ms_apply2<true>, grid2, dim3(BS), 0, st, S, diag, p, ld, w, sh.zc, state,
                 partials);
    else
      ROM_LAUNCH(k_ms_apply2<false>, grid2, dim3(BS), 0, st, S, diag, p, ld, w, sh.zc, state,
                 partials);
    return (int)(grid2.x * grid2.y);
  }
  const dim3 grid(sh.grid.x, sh.grid.y, nb);
  if (S.var)
    ROM_LAUNCH(k_ms_apply<true>, grid, dim3(BS), 0, st, S, diag, p, ld, w, sh.zc, state,
               partials);
  else
    ROM_LAUNCH(k_ms_apply<false>, grid, dim3(BS), 0, st, S, diag, p, ld, w, sh.zc, state,
               partials);
  return (int)(grid.x * grid.y);
}

void launch_ms_alpha(const double* partials, int P, MsState* state, int nb, const MsShifts& sh,
                     hipStream_t st) {
  ROM_LAUNCH(k_ms_alpha, dim3(nb), dim3(BS), 0, st, partials, P, state, sh);
}

void launch_ms_update(int64_t n, int nb, int ns, const double* w, double* r, int64_t ld,
                      double* Pr, double* Pi, double* Xr, double* Xi, int64_t ldx,
                      const MsState* state, double* partials, hipStream_t st) {
  ROM_LAUNCH(k_ms_update, dim3(vec_grid(n), nb), dim3(BS), 0, st, n, nb, w, r, ld, Pr, Pi, Xr, Xi,
             ldx, state, ns, partials);
}

void launch_ms_beta(const double* partials, int P, MsState* state, int nb, int ns,
                    hipStream_t st) {
  ROM_LAUNCH(k_ms_beta, dim3(nb), dim3(BS), 0, st, partials, P, state, ns);
}

void launch_ms_dir(int64_t n, int nb, const double* r, double* p, int64_t ld,
                   const MsState* state, hipStream_t st) {
  ROM_LAUNCH(k_ms_dir, dim3(vec_grid(n), nb), dim3(BS), 0, st, n, nb, r, p, ld, state);
}

void launch_ms_resid(const Stencil& S, const StencilShape& shp, const double* diag,
                     const double* Xr, const double* Xi, int64_t ldx, const double* B, int64_t ldb,
                     int nb, const MsShifts& sh, double* partials, double* out, hipStream_t st) {
  const int cols = nb * sh.ns;
  const dim3 grid(shp.grid.x, shp.grid.y, cols);
  if (S.var) {
    ROM_LAUNCH((k_ms_resid<true, 0>), grid, dim3(BS), 0, st, S, diag, Xr, Xi, ldx, B, ldb, nb, sh,
               shp.zc, partials);
    ROM_LAUNCH((k_ms_resid<true, 1>), grid, dim3(BS), 0, st, S, diag, Xr, Xi, ldx, B, ldb, nb, sh,
               shp.zc, partials);
  } else {
    ROM_LAUNCH((k_ms_resid<false, 0>), grid, dim3(BS), 0, st, S, diag, Xr, Xi, ldx, B, ldb, nb, sh,
               shp.zc, partials);
    ROM_LAUNCH((k_ms_resid<false, 1>), grid, dim3(BS), 0, st, S, diag, Xr, Xi, ldx, B, ldb, nb, sh,
               shp.zc, partials);
  }
  ROM_LAUNCH(k_ms_sum_rows, dim3(2 * cols), dim3(BS), 0, st, partials, shp.blocks, out);
}

}  // namespace rom
