// Gram matrices X^T diag(w) Y of tall-skinny FP64 matrices on the matrix cores
// (v_mfma_f64_16x16x4f64).  Used for the per-point outer Gram Q^T A(p) Q (only the
// rows inside the absorption bumps contribute beyond Q^T A_* Q + mu0 I), for the
// recycle-space Gram U_j^T A U_j, and for the reduced matrices of eq. (newreduced).
#include <algorithm>

#include "kernels.h"

namespace rom {

namespace {

constexpr int BS = 256;    // 4 waves
constexpr int TT = 64;     // output tile (TT x TT) of one wave

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

// Four consecutive rows of one column: two 16-byte loads when the whole row group is in
// range, guarded scalar loads in the ragged tail.
__device__ __forceinline__ void load4(const double* __restrict__ p, int64_t r, int64_t rend,
                                      bool full, double (&v)[4]) {
  if (full) {
    const double2 u0 = *reinterpret_cast<const double2*>(p + r);
    const double2 u1 = *reinterpret_cast<const double2*>(p + r + 2);
    v[0] = u0.x;
    v[1] = u0.y;
    v[2] = u1.x;
    v[3] = u1.y;
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = r + s < rend ? p[r + s] : 0.0;
  }
}

constexpr int ROWG = 16;   // rows per MFMA group: four k-steps of four k-slots

// partials[s][i + j*a] = sum over the rows of block s of w[r] X[r,i] Y[r,j] for the tile
// pair of this block.  Every wave works alone on its own rows and on the whole 64 x 64
// pair (4 x 4 MFMA tiles of 16 x 16).  A lane reads four consecutive rows of one column,
// so the 16 rows of a group reach the matrix core as four k-steps: step s takes, in
// k-slot q, row 4 q + s of the group (a reordering of the sum over rows).  A group whose
// weights are all zero is skipped.  On a diagonal pair of a symmetric Gram only the tiles
// on or below the diagonal are formed.  The waves' tiles are added in a fixed order.
// The unweighted form prefetches the next row group into registers while the matrix
// cores work on the current one (one wave per SIMD fits, so the overlap has to come from
// within the wave).  The weighted form (a few rows of bump support) loads a group only
// after its weights show a non-zero.
template <bool WEIGHTED>
__global__ __launch_bounds__(BS) void k_gram(const double* __restrict__ X, int64_t ldx, int a,
                                              const double* __restrict__ Y, int64_t ldy, int b,
                                              int64_t rows, int64_t rows_per_wave,
                                              const double* __restrict__ w, int sym, int ntx,
                                              double* __restrict__ partials) {
  __shared__ double red[16][4][WAVE];
  int ti, tj;
  tile_of(blockIdx.x, sym != 0, ntx, ti, tj);
  const int x0 = ti * TT, y0 = tj * TT;
  const bool diag = sym && ti == tj;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int ci = lane & 15, kq = lane >> 4;
  const int64_t rbeg = ((int64_t)blockIdx.y * (BS / WAVE) + wid) * rows_per_wave;
  int64_t rend = rbeg + rows_per_wave;
  if (rend > rows) rend = rows;
  const double *xp[4], *yp[4];
  bool xin[4], yin[4];
  int ntlx = 0, ntly = 0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int cx = x0 + 16 * t + ci, cy = y0 + 16 * t + ci;
    xin[t] = cx < a;
    yin[t] = cy < b;
    xp[t] = X + (int64_t)(xin[t] ? cx : a - 1) * ldx;
    yp[t] = Y + (int64_t)(yin[t] ? cy : b - 1) * ldy;
    if (x0 + 16 * t < a) ntlx = t + 1;
    if (y0 + 16 * t < b) ntly = t + 1;
  }
  double4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (double4_t){0.0, 0.0, 0.0, 0.0};

  auto load_group = [&](int64_t r0, double (&xv)[4][4], double (&yv)[4][4]) {
    const bool full = r0 + ROWG <= rend;
    const int64_t r = r0 + 4 * kq;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t < ntlx) load4(xp[t], r, rend, full, xv[t]);
      if (t < ntly) load4(yp[t], r, rend, full, yv[t]);
    }
  };
  auto mma_group = [&](double (&xv)[4][4], double (&yv)[4][4], const double (&wv)[4]) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        xv[t][s] = xin[t] ? xv[t][s] * wv[s] : 0.0;
        yv[t][s] = yin[t] ? yv[t][s] : 0.0;
      }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (i >= ntlx || j >= ntly || (diag && i < j)) continue;
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xv[i][s], yv[j][s], acc[i][j], 0, 0, 0);
        }
  };

  if (WEIGHTED) {
    // scan the weights 256 rows (16 groups) at a time: lane l checks rows 4 l .. 4 l + 3,
    // so lanes 4 g .. 4 g + 3 cover group g; only groups with a non-zero weight are loaded
    for (int64_t rs = rbeg; rs < rend; rs += 16 * ROWG) {
      double ws[4];
      load4(w, rs + 4 * lane, rend, rs + 4 * lane + 4 <= rend, ws);
      uint64_t nz = __ballot(ws[0] != 0.0 || ws[1] != 0.0 || ws[2] != 0.0 || ws[3] != 0.0);
      while (nz) {
        const int g = __builtin_ctzll(nz) >> 2;
        nz &= ~(0xFull << (4 * g));
        const int64_t r0 = rs + (int64_t)g * ROWG;
        double wv[4];
        load4(w, r0 + 4 * kq, rend, r0 + ROWG <= rend, wv);
        double xv[4][4], yv[4][4];
        load_group(r0, xv, yv);
        mma_group(xv, yv, wv);
      }
    }
  } else {
    const double one[4] = {1.0, 1.0, 1.0, 1.0};
    double xc[4][4], yc[4][4];
    if (rbeg < rend) load_group(rbeg, xc, yc);
    for (int64_t r0 = rbeg; r0 < rend; r0 += ROWG) {
      double xn[4][4], yn[4][4];
      if (r0 + ROWG < rend) load_group(r0 + ROWG, xn, yn);
      mma_group(xc, yc, one);
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          xc[t][s] = xn[t][s];
          yc[t][s] = yn[t][s];
        }
    }
  }
  // waves 3, 2, 1 pass their running sum down through LDS; wave 0 adds its own last
#pragma unroll
  for (int src = BS / WAVE - 1; src >= 1; --src) {
    if (wid == src) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double t = acc[i][j][v];
            if (src < BS / WAVE - 1) t += red[i * 4 + j][v][lane];
            red[i * 4 + j][v][lane] = t;
          }
    }
    __syncthreads();
  }
  if (wid != 0) return;
  // D layout of the 16x16x4 f64 MFMA: register v of a lane holds row (lane/16) + 4 v,
  // column lane % 16.
  double* P = partials + (int64_t)blockIdx.y * a * b;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int xi = x0 + 16 * i + (lane >> 4) + 4 * v;
        const int yj = y0 + 16 * j + (lane & 15);
        if (xi < a && yj < b) P[xi + (int64_t)yj * a] = acc[i][j][v] + red[i * 4 + j][v][lane];
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

// Projections onto a tall basis: partials[s][i + v*a] = sum over the rows of block s of
// X[r, i] V[r, v] for v < nv <= 16 (a block of right-hand sides against the basis).
// Every wave works alone on its own rows and on the block's 64 columns of X (four 16 x 16
// MFMA tiles against the 16 vector slots).  A lane reads four consecutive rows of one
// column (two 16-byte loads), so the 16 rows of a group reach the matrix core as four
// k-steps: step s takes, in k-slot q, row 4 q + s of the group -- a reordering of the
// sum over rows.  The four waves' tiles are added in wave order at the end.
__global__ __launch_bounds__(BS) void k_proj(const double* __restrict__ X, int64_t ldx, int a,
                                              const double* __restrict__ V, int64_t ldv, int nv,
                                              int64_t rows, int64_t rows_per_wave,
                                              double* __restrict__ partials) {
  __shared__ double red[BS / WAVE - 1][4][4][WAVE];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int ci = lane & 15, kq = lane >> 4;
  const int x0 = blockIdx.x * TT;
  const int64_t rbeg = ((int64_t)blockIdx.y * (BS / WAVE) + wid) * rows_per_wave;
  int64_t rend = rbeg + rows_per_wave;
  if (rend > rows) rend = rows;
  // lanes past the last column read a valid neighbour and drop the value
  const double* xp[4];
  bool xin[4];
  int ntl = 0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int c = x0 + 16 * t + ci;
    xin[t] = c < a;
    xp[t] = X + (int64_t)(xin[t] ? c : a - 1) * ldx;
    if (x0 + 16 * t < a) ntl = t + 1;
  }
  const bool vin = ci < nv;
  const double* vp = V + (int64_t)(vin ? ci : nv - 1) * ldv;
  double4_t acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = (double4_t){0.0, 0.0, 0.0, 0.0};
  for (int64_t r0 = rbeg; r0 < rend; r0 += ROWG) {
    const bool full = r0 + ROWG <= rend;
    const int64_t r = r0 + 4 * kq;
    double vv[4], xv[4][4];
    load4(vp, r, rend, full, vv);
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (t < ntl) load4(xp[t], r, rend, full, xv[t]);
#pragma unroll
    for (int s = 0; s < 4; ++s) vv[s] = vin ? vv[s] : 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t >= ntl) continue;
#pragma unroll
      for (int s = 0; s < 4; ++s)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(xin[t] ? xv[t][s] : 0.0, vv[s], acc[t],
                                                      0, 0, 0);
    }
  }
  if (wid > 0) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[wid - 1][t][v][lane] = acc[t][v];
  }
  __syncthreads();
  if (wid != 0) return;
  // D layout of the 16x16x4 f64 MFMA: register v of a lane holds row (lane/16) + 4 v,
  // column lane % 16.
  double* P = partials + (int64_t)blockIdx.y * a * nv;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double sum = acc[t][v];
#pragma unroll
      for (int w = 0; w < BS / WAVE - 1; ++w) sum += red[w][t][v][lane];
      const int xi = x0 + 16 * t + (lane >> 4) + 4 * v;
      const int vj = lane & 15;
      if (xi < a && vj < nv) P[xi + (int64_t)vj * a] = sum;
    }
}

// About 1024 blocks of four waves (four blocks per CU, one round), each wave at least
// four row groups; rps is the rows of one wave, a multiple of the row group.
void proj_shape(int a, int64_t rows, int& ntile, int& nsplit, int64_t& rps) {
  constexpr int64_t WPB = BS / WAVE;
  ntile = (a + TT - 1) / TT;
  if (ntile < 1) ntile = 1;
  int64_t ns = 1024 / ntile;
  if (ns < 1) ns = 1;
  const int64_t maxs = (rows + WPB * 4 * ROWG - 1) / (WPB * 4 * ROWG);
  if (ns > maxs) ns = maxs > 0 ? maxs : 1;
  rps = (rows + ns * WPB - 1) / (ns * WPB);
  rps = (rps + ROWG - 1) / ROWG * ROWG;
  if (rps < ROWG) rps = ROWG;
  nsplit = (int)((rows + rps * WPB - 1) / (rps * WPB));
  if (nsplit < 1) nsplit = 1;
}

// About 256 blocks of four waves (one block per CU, one round), each wave at least four
// row groups; rps is the rows of one wave, a multiple of 256 rows (the weight scan).  A
// weighted Gram (rows of bump support only) gets four times as many blocks: most of its
// rows are skipped, and the scan itself is what has to be spread.
void gram_shape(int a, int b, int64_t rows, bool sym, bool weighted, int& npairs, int& nsplit,
                int64_t& rps) {
  constexpr int64_t WPB = BS / WAVE, SCAN = 16 * ROWG;
  const int ta = (a + TT - 1) / TT, tb = (b + TT - 1) / TT;
  npairs = sym ? ta * (ta + 1) / 2 : ta * tb;
  if (npairs < 1) npairs = 1;
  int64_t ns = (weighted ? 1024 : 256) / npairs;
  if (ns < 1) ns = 1;
  const int64_t maxs = (rows + WPB * SCAN - 1) / (WPB * SCAN);
  if (ns > maxs) ns = maxs > 0 ? maxs : 1;
  rps = (rows + ns * WPB - 1) / (ns * WPB);
  rps = (rps + SCAN - 1) / SCAN * SCAN;
  nsplit = (int)((rows + rps * WPB - 1) / (rps * WPB));
  if (nsplit < 1) nsplit = 1;
}

}  // namespace

size_t gram_partials(int a, int b, int64_t rows, bool sym) {
  int np, ns, nsw;
  int64_t rps;
  gram_shape(a, b, rows, sym, false, np, ns, rps);
  gram_shape(a, b, rows, sym, true, np, nsw, rps);
  return (size_t)std::max(ns, nsw) * a * b;
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
  if ((ldx | ldv) & 1 || ((uintptr_t)X | (uintptr_t)V) & 15)
    throw Error(ROM_EINVAL, "launch_proj: X and V need 16-byte aligned columns");
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
  if ((ldx | ldy) & 1 || ((uintptr_t)X | (uintptr_t)Y | (uintptr_t)w) & 15)
    throw Error(ROM_EINVAL, "launch_gram: X, Y and w need 16-byte aligned columns");
  int np, ns;
  int64_t rps;
  gram_shape(a, b, rows, sym, w != nullptr, np, ns, rps);
  const int ntx = (a + TT - 1) / TT;
  if (w)
    ROM_LAUNCH(k_gram<true>, dim3(np, ns), dim3(BS), 0, st, X, ldx, a, Y, ldy, b, rows, rps, w,
               sym ? 1 : 0, ntx, partials);
  else
    ROM_LAUNCH(k_gram<false>, dim3(np, ns), dim3(BS), 0, st, X, ldx, a, Y, ldy, b, rows, rps,
               w, sym ? 1 : 0, ntx, partials);
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
