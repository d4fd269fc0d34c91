// Gram matrices X^T diag(w) Y of tall-skinny FP64 matrices on the matrix cores
// (v_mfma_f64_16x16x4f64).  Used for the per-point outer Gram Q^T A(p) Q (only the
// rows inside the absorption bumps contribute beyond Q^T A_* Q + mu0 I), for the
// recycle-space Gram U_j^T A U_j, and for the reduced matrices of eq. (newreduced).
#include <algorithm>

#include "kernels.h"

namespace rom {

namespace {

constexpr int BS = 256;    // 4 waves
constexpr int TT = 64;     // output tile (TT x TT), each wave owns a 32 x 32 quarter
constexpr int KC = 32;     // rows staged in LDS per step
constexpr int PAD = 1;

typedef double double4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void tile_of(int p, bool sym, int ntb, int& ti, int& tj) {
  if (!sym) {
    ti = p % ntb;  // ntb = number of X tiles here
    tj = p / ntb;
    return;
  }
  // lower-triangle pair index p -> (ti >= tj)
  int t = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
  while ((t + 1) * (t + 2) / 2 <= p) ++t;
  while (t * (t + 1) / 2 > p) --t;
  ti = t;
  tj = p - t * (t + 1) / 2;
}

// partials[s][i + j*a] = sum over the rows of split s of w[r] X[r,i] Y[r,j]
// for the tile pair of this block.
__global__ __launch_bounds__(BS) void k_gram(const double* __restrict__ X, int64_t ldx, int a,
                                              const double* __restrict__ Y, int64_t ldy, int b,
                                              int64_t rows, int64_t rows_per_split,
                                              const double* __restrict__ w, int sym, int ntx,
                                              double* __restrict__ partials) {
  __shared__ double Xs[KC][TT + PAD];
  __shared__ double Ys[KC][TT + PAD];
  int ti, tj;
  tile_of(blockIdx.x, sym != 0, ntx, ti, tj);
  const int x0 = ti * TT, y0 = tj * TT;
  const int64_t rbeg = (int64_t)blockIdx.y * rows_per_split;
  int64_t rend = rbeg + rows_per_split;
  if (rend > rows) rend = rows;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  double4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (double4_t){0.0, 0.0, 0.0, 0.0};

  // staging map: thread -> row (t % 32) and columns (t / 32) + 8 q
  const int srow = threadIdx.x % KC;
  const int scol = threadIdx.x / KC;
  for (int64_t r0 = rbeg; r0 < rend; r0 += KC) {
    const int64_t r = r0 + srow;
    double wr_ = 0.0;
    if (r < rend) wr_ = w ? w[r] : 1.0;
    if (!__syncthreads_or(wr_ != 0.0)) continue;
#pragma unroll
    for (int q = 0; q < TT / (BS / KC); ++q) {
      const int c = scol + (BS / KC) * q;
      const int xc = x0 + c, yc = y0 + c;
      Xs[srow][c] = (wr_ != 0.0 && xc < a) ? wr_ * X[r + (int64_t)xc * ldx] : 0.0;
      Ys[srow][c] = (r < rend && yc < b) ? Y[r + (int64_t)yc * ldy] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const int kr = kk + (lane >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = Xs[kr][wr * 32 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = Ys[kr][wc * 32 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // D layout of the 16x16x4 f64 MFMA: register v of a lane holds row (lane/16) + 4 v,
  // column lane % 16.
  double* P = partials + (int64_t)blockIdx.y * a * b;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int xi = x0 + wr * 32 + i * 16 + (lane >> 4) + 4 * v;
        const int yj = y0 + wc * 32 + j * 16 + (lane & 15);
        if (xi < a && yj < b) P[xi + (int64_t)yj * a] = acc[i][j][v];
      }
}

// C = base + shift I + sum over splits: one thread per element when there are few
// splits, one wave per element otherwise (fixed summation order either way).
template <bool WAVE_PER_ELEM>
__global__ void k_gram_finish(const double* __restrict__ partials, int nsplit, int a, int b,
                              int sym, const double* __restrict__ base, int64_t ldb, double shift,
                              double* __restrict__ C, int64_t ldc) {
  const int64_t ne = (int64_t)a * b;
  int64_t e;
  int lane = 0;
  if (WAVE_PER_ELEM) {
    e = (int64_t)blockIdx.x * (BS / WAVE) + (threadIdx.x >> 6);
    lane = threadIdx.x & 63;
  } else {
    e = (int64_t)blockIdx.x * BS + threadIdx.x;
  }
  if (e >= ne) return;
  const int i = (int)(e % a), j = (int)(e / a);
  int pi = i, pj = j;
  if (sym && j > i) {
    pi = j;
    pj = i;
  }
  const int64_t off = pi + (int64_t)pj * a;
  double s = 0.0;
  if (WAVE_PER_ELEM) {
    for (int q = lane; q < nsplit; q += WAVE) s += partials[(int64_t)q * ne + off];
    s = wave_sum(s);
    if (lane != 0) return;
  } else {
    for (int q = 0; q < nsplit; ++q) s += partials[(int64_t)q * ne + off];
  }
  if (base) s += base[i + j * ldb];
  if (i == j) s += shift;
  C[i + j * ldc] = s;
}

// Projections onto a tall basis: partials[s][i + v*a] = sum over the rows of split s of
// X[r, i] V[r, v] for v < nv <= 16 (a block of right-hand sides against the basis).
// Each wave owns 16 columns of X and all 16 vector slots (one 16x16 MFMA tile); the
// block stages KC rows of its 64 columns of X and of V through LDS.
__global__ __launch_bounds__(BS) void k_proj(const double* __restrict__ X, int64_t ldx, int a,
                                              const double* __restrict__ V, int64_t ldv, int nv,
                                              int64_t rows, int64_t rows_per_split,
                                              double* __restrict__ partials) {
  __shared__ double Xs[KC][TT + PAD];
  __shared__ double Vs[KC][16 + PAD];
  const int x0 = blockIdx.x * TT;
  const int64_t rbeg = (int64_t)blockIdx.y * rows_per_split;
  int64_t rend = rbeg + rows_per_split;
  if (rend > rows) rend = rows;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double4_t acc = (double4_t){0.0, 0.0, 0.0, 0.0};
  const int srow = threadIdx.x % KC;
  const int scol = threadIdx.x / KC;   // 0..7
  for (int64_t r0 = rbeg; r0 < rend; r0 += KC) {
    const int64_t r = r0 + srow;
    const bool in = r < rend;
#pragma unroll
    for (int q = 0; q < TT / (BS / KC); ++q) {
      const int c = scol + (BS / KC) * q;
      Xs[srow][c] = (in && x0 + c < a) ? X[r + (int64_t)(x0 + c) * ldx] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 16 / (BS / KC); ++q) {
      const int v = scol + (BS / KC) * q;
      Vs[srow][v] = (in && v < nv) ? V[r + (int64_t)v * ldv] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const int kr = kk + (lane >> 4);
      const double av = Xs[kr][wid * 16 + (lane & 15)];
      const double bv = Vs[kr][lane & 15];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  double* P = partials + (int64_t)blockIdx.y * a * nv;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int xi = x0 + wid * 16 + (lane >> 4) + 4 * v;
    const int vj = lane & 15;
    if (xi < a && vj < nv) P[xi + (int64_t)vj * a] = acc[v];
  }
}

void proj_shape(int a, int64_t rows, int& ntile, int& nsplit, int64_t& rps) {
  ntile = (a + TT - 1) / TT;
  nsplit = 2048 / (ntile > 0 ? ntile : 1);
  if (nsplit < 1) nsplit = 1;
  int64_t maxs = (rows + 8 * KC - 1) / (8 * KC);
  if (nsplit > maxs) nsplit = (int)(maxs > 0 ? maxs : 1);
  rps = (rows + nsplit - 1) / nsplit;
  rps = (rps + KC - 1) / KC * KC;
  nsplit = (int)((rows + rps - 1) / rps);
  if (nsplit < 1) nsplit = 1;
}

void gram_shape(int a, int b, int64_t rows, bool sym, int& npairs, int& nsplit, int64_t& rps) {
  const int ta = (a + TT - 1) / TT, tb = (b + TT - 1) / TT;
  npairs = sym ? ta * (ta + 1) / 2 : ta * tb;
  nsplit = 2048 / (npairs > 0 ? npairs : 1);
  if (nsplit < 1) nsplit = 1;
  if (nsplit > 1024) nsplit = 1024;
  int64_t maxs = (rows + 8 * KC - 1) / (8 * KC);   // at least 8 staged chunks per split
  if (nsplit > maxs) nsplit = (int)(maxs > 0 ? maxs : 1);
  rps = (rows + nsplit - 1) / nsplit;
  rps = (rps + KC - 1) / KC * KC;
  nsplit = (int)((rows + rps - 1) / rps);
  if (nsplit < 1) nsplit = 1;
}

}  // namespace

size_t gram_partials(int a, int b, int64_t rows, bool sym) {
  int np, ns;
  int64_t rps;
  gram_shape(a, b, rows, sym, np, ns, rps);
  return (size_t)ns * a * b;
}

size_t gram_partials_max(int a, int b, int64_t rows, bool sym) {
  size_t best = 0;
  for (int ta = 1; ta <= (a + TT - 1) / TT; ++ta) {
    const int aa = std::min(a, ta * TT);
    const int bb = sym ? aa : b;
    best = std::max(best, gram_partials(aa, bb, rows, sym));
  }
  return best;
}

size_t proj_partials(int a, int nv, int64_t rows) {
  int nt, ns;
  int64_t rps;
  proj_shape(a, rows, nt, ns, rps);
  return (size_t)ns * a * nv;
}

size_t proj_partials_max(int maxa, int nv, int64_t rows) {
  size_t best = 0;
  for (int t = 1; t <= (maxa + TT - 1) / TT; ++t)
    best = std::max(best, proj_partials(std::min(maxa, t * TT), nv, rows));
  return best;
}

void launch_proj(const double* X, int64_t ldx, int a, const double* V, int64_t ldv, int nv,
                 int64_t rows, double* C, int64_t ldc, double* partials, hipStream_t st) {
  if (a <= 0 || nv <= 0) return;
  if (nv > 16) throw Error(ROM_EINVAL, "launch_proj: at most 16 vectors");
  int nt, ns;
  int64_t rps;
  proj_shape(a, rows, nt, ns, rps);
  ROM_LAUNCH(k_proj, dim3(nt, ns), dim3(BS), 0, st, X, ldx, a, V, ldv, nv, rows, rps, partials);
  ROM_CHECK_LAUNCH();
  const int64_t ne = (int64_t)a * nv;
  if (ns >= 32)
    ROM_LAUNCH(k_gram_finish<true>, dim3(ceil_div(ne, BS / WAVE)), dim3(BS), 0, st, partials, ns,
               a, nv, 0, (const double*)nullptr, (int64_t)0, 0.0, C, ldc);
  else
    ROM_LAUNCH(k_gram_finish<false>, dim3(ceil_div(ne, BS)), dim3(BS), 0, st, partials, ns, a,
               nv, 0, (const double*)nullptr, (int64_t)0, 0.0, C, ldc);
  ROM_CHECK_LAUNCH();
}

void launch_gram(const double* X, int64_t ldx, int a, const double* Y, int64_t ldy, int b,
                 int64_t rows, const double* w, bool sym, const double* base, int64_t ldb,
                 double shift, double* C, int64_t ldc, double* partials, hipStream_t st) {
  if (a <= 0 || b <= 0) return;
  int np, ns;
  int64_t rps;
  gram_shape(a, b, rows, sym, np, ns, rps);
  const int ntx = (a + TT - 1) / TT;
  ROM_LAUNCH(k_gram, dim3(np, ns), dim3(BS), 0, st, X, ldx, a, Y, ldy, b, rows, rps, w,
                     sym ? 1 : 0, ntx, partials);
  ROM_CHECK_LAUNCH();
  const int64_t ne = (int64_t)a * b;
  if (ns >= 32)
    ROM_LAUNCH(k_gram_finish<true>, dim3(ceil_div(ne, BS / WAVE)), dim3(BS), 0, st,
                       partials, ns, a, b, sym ? 1 : 0, base, ldb, shift, C, ldc);
  else
    ROM_LAUNCH(k_gram_finish<false>, dim3(ceil_div(ne, BS)), dim3(BS), 0, st, partials,
                       ns, a, b, sym ? 1 : 0, base, ldb, shift, C, ldc);
  ROM_CHECK_LAUNCH();
}

}  // namespace rom
