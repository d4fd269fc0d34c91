// Deflated (recycled) CG on A g = r with the recycle space U_j (Sec. 4.2.1, CG form):
// directions are kept A-orthogonal to U_j by p = s + beta p - U_j (U_j^T A U_j)^{-1}
// (A U_j)^T s.  Every step is three launches (operator, update, direction).  No kernel
// synchronises across blocks: each writes per-block partial sums and the next launch
// reduces them; the scalar state lives in device memory (s^T s double-buffered by
// step parity), so chunks of steps run without host round trips.  Each thread loads
// its first row before reducing the previous launch's partials, so the reduction
// latency hides behind the loads.  T is the vector type: double for the plain form,
// float for the inner sweeps of the mixed form (FP32 vectors and FP32 sums); the CG
// scalars, the tolerance and (U^T A U)^{-1} stay FP64 in either case.
#include "kernels.h"

namespace rom {

namespace {

// Step kernels: blocks of 256 threads, each thread RPT rows of a 256 * RPT-row chunk
// (rows b * chunk + t + 256 q), a block's chunks strided by the grid.  A thread issues
// every load of its first chunk (the rows of U_j or A U_j and the vectors) before it
// reduces the previous launch's partials, so the reduction hides behind the loads.  RPT
// is as large as keeps those values and the NJT + 1 running sums in registers without
// spilling; at 64 columns nothing is preloaded (RPT 0: one row per thread per pass,
// U_j read as it is used).
constexpr int CG_BS = 256;
template <typename T, int NJT>
struct CgRows {
  static constexpr int value =
      sizeof(T) == 8 ? (NJT <= 16 ? 4 : NJT <= 32 ? 2 : 0) : (NJT <= 32 ? 4 : 0);
  // the narrow variant: half the rows per thread, more waves per SIMD (batches of
  // members, where a block walks several chunks, can prefer it; the tuner decides)
  static constexpr int narrow = value >= 2 ? value / 2 : value;
};
constexpr int CG_GRID = 256;
constexpr int START_BS = 256;

__global__ void k_cg_setup(CGState* cg, CgSetup su, int nb) {
  const int y = threadIdx.x;
  if (y >= nb) return;
  CGState* c = cg + y;
  c->tol2 = su.tol2[y];
  c->rscale = su.rscale[y];
  c->maxit = su.maxit[y];
  c->nj = su.nj[y];
  c->its = 0;
  c->done = su.active[y] ? 0 : 1;
  c->flag = 0;
  c->gamma[0] = 0.0;
  c->gamma[1] = 0.0;
  c->pw = 0.0;
  c->kcur = 0;
}

// Row j = threadIdx.x < nj of Ginv = (U^T A U)^{-1} (symmetric, FP64) is loaded early
// into registers, where it fits (NJT <= 16), so that its latency hides behind other loads.
template <int NJT>
struct GramPf {
  static constexpr bool value = NJT <= 16;
};

template <int NJT, bool PF>
__device__ __forceinline__ void gram_row(const double* __restrict__ Ginv, int nj,
                                         double (&gr)[PF ? NJT : 1]) {
  if (!PF) return;
  const int j = threadIdx.x;
#pragma unroll
  for (int c = 0; c < NJT; ++c)
    if (j < nj && c < nj) gr[PF ? c : 0] = Ginv[j + c * nj];
}

// ys[j] = scale * sum_c Ginv[j + c nj] t[c], evaluated in FP64 (the loop is unrolled to
// NJT so that the row loads, where not prefetched, issue together) and stored as T in
// shared memory.
template <int NJT, bool PF, typename T, typename S>
__device__ __forceinline__ void gram_apply(const double* __restrict__ Ginv,
                                           const double (&gr)[PF ? NJT : 1], int nj, const S* t,
                                           double scale, T* ys) {
  if (threadIdx.x < nj) {
    const int j = threadIdx.x;
    double y = 0.0;
#pragma unroll
    for (int c = 0; c < NJT; ++c)
      if (c < nj) y += (PF ? gr[PF ? c : 0] : Ginv[j + c * nj]) * (double)t[c];
    ys[j] = (T)(scale * y);
  }
  __syncthreads();
}

// Rows per thread of the start kernel (it reads both U_j and A U_j): as for the steps, as
// many as keep the loaded rows and the running sums in registers.
template <typename T, int NJT>
struct StartRows {
  static constexpr int value = sizeof(T) == 8 ? (NJT <= 8 ? 4 : NJT <= 16 ? 2 : 0)
                                              : (NJT <= 16 ? 4 : 0);
};

// Start: y0 = G^{-1} U^T r (U^T r in cg->t), g = U y0, s = r - AU y0; partials of
// (AU)^T s (values 0..nj-1) and s^T s (value NJT).  The right-hand side is FP64 and is
// read as rscale * r (the mixed form solves for a unit-norm residual in FP32).  Rows as
// in the step kernels: a thread loads its first chunk's rows before y0 is formed.
template <typename T, int NJT, int RPT = StartRows<T, NJT>::value>
__global__ __launch_bounds__(START_BS) void k_dcg_start(const T* __restrict__ W,
                                                         const T* __restrict__ AW,
                                                         int64_t wstride, int64_t ld, int64_t n,
                                                         const double* __restrict__ Ginv,
                                                         int64_t gstride,
                                                         const double* __restrict__ r,
                                                         int64_t rstride, T* __restrict__ g,
                                                         T* __restrict__ s, int64_t vstride,
                                                         const CGState* cgs,
                                                         T* __restrict__ part2,
                                                         int64_t p2stride) {
  const int y = blockIdx.y;
  const CGState* cg = cgs + y;
  if (cg->done) return;
  W += y * wstride;
  AW += y * wstride;
  Ginv += y * gstride;
  r += y * rstride;
  g += y * vstride;
  s += y * vstride;
  part2 += y * p2stride;
  const int nj = cg->nj;
  const double rscale = cg->rscale;
  constexpr bool PRE = RPT > 0;
  constexpr int R = PRE ? RPT : 1;
  constexpr int64_t CH = (int64_t)START_BS * R;
  int64_t base = (int64_t)blockIdx.x * CH + threadIdx.x;
  T wr[R][PRE ? NJT : 1], ar[R][PRE ? NJT : 1], rv[R];
  auto load = [&](int64_t b0) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int64_t i = b0 + (int64_t)q * START_BS;
      const bool in = i < n;
      rv[q] = in ? (T)r[i] : T(0);
      if (PRE) {
#pragma unroll
        for (int c = 0; c < NJT; ++c) {
          wr[q][PRE ? c : 0] = (in && c < nj) ? W[i + c * ld] : T(0);
          ar[q][PRE ? c : 0] = (in && c < nj) ? AW[i + c * ld] : T(0);
        }
      }
    }
  };
  load(base);
  __shared__ T ys[NJ_MAX];
  constexpr bool GPF = GramPf<NJT>::value;
  double gr[GPF ? NJT : 1];
  gram_row<NJT, GPF>(Ginv, nj, gr);
  gram_apply<NJT, GPF>(Ginv, gr, nj, cg->t, rscale, ys);
  const T rs = (T)rscale;
  T acc[NJT + 1];
#pragma unroll
  for (int c = 0; c <= NJT; ++c) acc[c] = T(0);
  for (;;) {
    // without a preload the row of A U is still kept between its two uses when it fits
    constexpr bool KEEP = !PRE && NJT * sizeof(T) <= 256;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int64_t i = base + (int64_t)q * START_BS;
      const bool in = i < n;
      T gi = T(0), si = rs * rv[q];
      T kept[KEEP ? NJT : 1];
#pragma unroll
      for (int c = 0; c < NJT; ++c)
        if (c < nj) {
          const T wv = PRE ? wr[q][PRE ? c : 0] : (in ? W[i + c * ld] : T(0));
          const T av = PRE ? ar[q][PRE ? c : 0] : (in ? AW[i + c * ld] : T(0));
          if (KEEP) kept[KEEP ? c : 0] = av;
          gi += wv * ys[c];
          si -= av * ys[c];
        }
      if (in) {
        g[i] = gi;
        s[i] = si;
      }
      acc[NJT] += si * si;   // 0 past the end (rv and the rows are 0 there)
#pragma unroll
      for (int c = 0; c < NJT; ++c)
        if (c < nj)
          acc[c] += (PRE ? ar[q][PRE ? c : 0]
                         : KEEP ? kept[KEEP ? c : 0] : (in ? AW[i + c * ld] : T(0))) * si;
    }
    base += (int64_t)gridDim.x * CH;
    if (base - threadIdx.x >= n) break;
    load(base);
  }
  write_partials_t<NJT + 1, START_BS>(acc, part2, blockIdx.x, gridDim.x);
}

// Reduce the step's partials (s^T s, (AU)^T s); record s^T s for the next step, count
// the step, stop on convergence / maxit / non-finite values; else the new direction
// p = s + beta p - U G^{-1} (AU)^T s.  iter = -1 for the direction after the start.
template <typename T, int NJT, int RPT = CgRows<T, NJT>::value>
__global__ __launch_bounds__(CG_BS) void k_dcg_dir(const T* __restrict__ W, int64_t wstride,
                                                    int64_t ld, int64_t n,
                                                    const double* __restrict__ Ginv,
                                                    int64_t gstride, const T* __restrict__ s,
                                                    T* __restrict__ p, int64_t vstride, int iter,
                                                    CGState* cgs, const T* __restrict__ part2,
                                                    int64_t p2stride, int P2) {
  const int y = blockIdx.y;
  CGState* cg = cgs + y;
  if (cg->done) return;
  W += y * wstride;
  Ginv += y * gstride;
  s += y * vstride;
  p += y * vstride;
  part2 += y * p2stride;
  const int nj = cg->nj;
  if (iter == ITER_STATE) iter = cg->kcur;
  const bool first = iter < 0;
  constexpr bool PRE = RPT > 0;
  constexpr int R = PRE ? RPT : 1;
  constexpr int64_t CH = (int64_t)CG_BS * R;
  int64_t base = (int64_t)blockIdx.x * CH + threadIdx.x;
  T wr[R][PRE ? NJT : 1], sv[R], pv[R];
  auto load = [&](int64_t b0) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int64_t i = b0 + (int64_t)q * CG_BS;
      const bool in = i < n;
      sv[q] = in ? s[i] : T(0);
      pv[q] = (in && !first) ? p[i] : T(0);
      if (PRE) {
#pragma unroll
        for (int c = 0; c < NJT; ++c)
          wr[q][PRE ? c : 0] = (in && c < nj) ? W[i + c * ld] : T(0);
      }
    }
  };
  load(base);
  constexpr bool GPF = GramPf<NJT>::value;
  double gr[GPF ? NJT : 1];
  gram_row<NJT, GPF>(Ginv, nj, gr);
  // the state's scalars are read with the rows, ahead of the partial sums
  const double g0 = cg->gamma[0], g1 = cg->gamma[1], tol2 = cg->tol2;
  const int maxit = cg->maxit;
  __shared__ T tot[NJT + 1];
  __shared__ T ys[NJ_MAX];
  sum_partials_t<NJT + 1, CG_BS>(part2, P2, tot);
  const double gnew = (double)tot[NJT];
  const double gold = first ? 1.0 : ((iter & 1) ? g1 : g0);
  const bool nonfinite = !isfinite(gnew);
  const bool conv = gnew <= tol2;
  const bool hit = !first && iter + 1 >= maxit;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    cg->gamma[(iter + 1) & 1] = gnew;
    if (!first) cg->its = iter + 1;
    if (nonfinite) {
      cg->flag = 2;
      cg->done = 1;
    } else if (conv || hit) {
      cg->done = 1;
    }
  }
  if (nonfinite || conv || hit) return;
  gram_apply<NJT, GPF>(Ginv, gr, nj, tot, 1.0, ys);
  const T beta = first ? T(0) : (T)(gnew / gold);
  for (;;) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int64_t i = base + (int64_t)q * CG_BS;
      T pi = sv[q] + beta * pv[q];
#pragma unroll
      for (int c = 0; c < NJT; ++c)
        if (c < nj) pi -= (PRE ? wr[q][PRE ? c : 0] : (i < n ? W[i + c * ld] : T(0))) * ys[c];
      if (i < n) p[i] = pi;
    }
    base += (int64_t)gridDim.x * CH;
    if (base - threadIdx.x >= n) break;
    load(base);
  }
}

// alpha = s^T s / p^T A p; g += alpha p; s -= alpha w; partials of (AU)^T s and s^T s.
template <typename T, int NJT, int RPT = CgRows<T, NJT>::value>
__global__ __launch_bounds__(CG_BS) void k_dcg_update(const T* __restrict__ AW, int64_t wstride,
                                                       int64_t ld, int64_t n,
                                                       const T* __restrict__ p,
                                                       const T* __restrict__ w,
                                                       T* __restrict__ g, T* __restrict__ s,
                                                       int64_t vstride, int iter, CGState* cgs,
                                                       const T* __restrict__ part1, int P1,
                                                       int64_t p1stride, T* __restrict__ part2,
                                                       int64_t p2stride) {
  const int y = blockIdx.y;
  CGState* cg = cgs + y;
  if (cg->done) return;
  AW += y * wstride;
  p += y * vstride;
  w += y * vstride;
  g += y * vstride;
  s += y * vstride;
  part1 += y * p1stride;
  part2 += y * p2stride;
  const int nj = cg->nj;
  if (iter == ITER_STATE) iter = cg->its;
  constexpr bool PRE = RPT > 0;
  constexpr int R = PRE ? RPT : 1;
  constexpr int64_t CH = (int64_t)CG_BS * R;
  int64_t base = (int64_t)blockIdx.x * CH + threadIdx.x;
  T a[R][PRE ? NJT : 1], pv[R], wv[R], gv[R], sv[R];
  auto load = [&](int64_t b0) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int64_t i = b0 + (int64_t)q * CG_BS;
      const bool in = i < n;
      pv[q] = in ? p[i] : T(0);
      wv[q] = in ? w[i] : T(0);
      gv[q] = in ? g[i] : T(0);
      sv[q] = in ? s[i] : T(0);
      if (PRE) {
#pragma unroll
        for (int c = 0; c < NJT; ++c)
          a[q][PRE ? c : 0] = (in && c < nj) ? AW[i + c * ld] : T(0);
      }
    }
  };
  const double g0 = cg->gamma[0], g1 = cg->gamma[1];   // read with the rows, used after the sum
  load(base);
  __shared__ T pwt[1];
  sum_partials_t<1, CG_BS>(part1, P1, pwt);
  const double pw = (double)pwt[0];
  if (!(pw > 0.0) || !isfinite(pw)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      cg->flag = isfinite(pw) ? 1 : 2;
      cg->done = 1;
    }
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    cg->pw = pw;
    cg->kcur = iter;
  }
  const T alpha = (T)(((iter & 1) ? g1 : g0) / pw);
  T acc[NJT + 1];
#pragma unroll
  for (int c = 0; c <= NJT; ++c) acc[c] = T(0);
  for (;;) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int64_t i = base + (int64_t)q * CG_BS;
      const T si = sv[q] - alpha * wv[q];   // 0 past the end (sv = wv = 0 there)
      if (i < n) {
        g[i] = gv[q] + alpha * pv[q];
        s[i] = si;
      }
      acc[NJT] += si * si;
#pragma unroll
      for (int c = 0; c < NJT; ++c)
        if (c < nj)
          acc[c] += (PRE ? a[q][PRE ? c : 0] : (i < n ? AW[i + c * ld] : T(0))) * si;
    }
    base += (int64_t)gridDim.x * CH;
    if (base - threadIdx.x >= n) break;
    load(base);
  }
  write_partials_t<NJT + 1, CG_BS>(acc, part2, blockIdx.x, gridDim.x);
}

}  // namespace

int njt_of(int nj) { return nj <= 8 ? 8 : nj <= 16 ? 16 : nj <= 32 ? 32 : 64; }

int dcg_blocks(int64_t n) {
  const int b = ceil_div(n, 512);
  return b < CG_GRID ? (b < 1 ? 1 : b) : CG_GRID;
}

void launch_cg_setup(CGState* cg, const CgSetup& su, int nb, hipStream_t st) {
  if (nb < 1 || nb > G_MAX) throw Error(ROM_EINVAL, "cg_setup: batch size out of range");
  ROM_LAUNCH(k_cg_setup, dim3(1), dim3(64), 0, st, cg, su, nb);
  ROM_CHECK_LAUNCH();
}

template <typename T>
void launch_dcg_start(const T* W, const T* AW, int64_t wstride, int64_t ld, int64_t n, int njmax,
                      const double* Ginv, int64_t gstride, const double* r, int64_t rstride, T* g,
                      T* s, int64_t vstride, const CGState* cg, T* part2, int64_t p2stride, int nb,
                      int P, hipStream_t st) {
  const dim3 grid(P, nb);
  switch (njt_of(njmax)) {
#define C(J) case J: ROM_LAUNCH((k_dcg_start<T, J>), grid, dim3(START_BS), 0, st, W, AW, wstride, ld, n, Ginv, gstride, r, rstride, g, s, vstride, cg, part2, p2stride); break;
    C(8) C(16) C(32) C(64)
#undef C
  }
  ROM_CHECK_LAUNCH();
}

template <typename T>
void launch_dcg_dir(const T* W, int64_t wstride, int64_t ld, int64_t n, int njmax,
                    const double* Ginv, int64_t gstride, const T* s, T* p, int64_t vstride,
                    int iter, CGState* cg, const T* part2, int64_t p2stride, int nb, int P,
                    hipStream_t st, int P2, int narrow) {
  const dim3 grid(P, nb);
  if (P2 <= 0) P2 = P;
  switch (njt_of(njmax)) {
#define C(J)                                                                                    \
  case J:                                                                                       \
    if (narrow)                                                                                 \
      ROM_LAUNCH((k_dcg_dir<T, J, CgRows<T, J>::narrow>), grid, dim3(CG_BS), 0, st, W, wstride,  \
                 ld, n, Ginv, gstride, s, p, vstride, iter, cg, part2, p2stride, P2);           \
    else                                                                                        \
      ROM_LAUNCH((k_dcg_dir<T, J>), grid, dim3(CG_BS), 0, st, W, wstride, ld, n, Ginv, gstride,  \
                 s, p, vstride, iter, cg, part2, p2stride, P2);                                 \
    break;
    C(8) C(16) C(32) C(64)
#undef C
  }
  ROM_CHECK_LAUNCH();
}

template <typename T>
void launch_dcg_update(const T* AW, int64_t wstride, int64_t ld, int64_t n, int njmax, const T* p,
                       const T* w, T* g, T* s, int64_t vstride, int iter, CGState* cg,
                       const T* part1, int P1, int64_t p1stride, T* part2, int64_t p2stride,
                       int nb, int P, hipStream_t st, int narrow) {
  const dim3 grid(P, nb);
  switch (njt_of(njmax)) {
#define C(J)                                                                                     \
  case J:                                                                                        \
    if (narrow)                                                                                  \
      ROM_LAUNCH((k_dcg_update<T, J, CgRows<T, J>::narrow>), grid, dim3(CG_BS), 0, st, AW,        \
                 wstride, ld, n, p, w, g, s, vstride, iter, cg, part1, P1, p1stride, part2,      \
                 p2stride);                                                                      \
    else                                                                                         \
      ROM_LAUNCH((k_dcg_update<T, J>), grid, dim3(CG_BS), 0, st, AW, wstride, ld, n, p, w, g, s,  \
                 vstride, iter, cg, part1, P1, p1stride, part2, p2stride);                       \
    break;
    C(8) C(16) C(32) C(64)
#undef C
  }
  ROM_CHECK_LAUNCH();
}

#define INSTANTIATE(T)                                                                          \
  template void launch_dcg_start<T>(const T*, const T*, int64_t, int64_t, int64_t, int,          \
                                    const double*, int64_t, const double*, int64_t, T*, T*,      \
                                    int64_t, const CGState*, T*, int64_t, int, int,              \
                                    hipStream_t);                                                \
  template void launch_dcg_dir<T>(const T*, int64_t, int64_t, int64_t, int, const double*,       \
                                  int64_t, const T*, T*, int64_t, int, CGState*, const T*,       \
                                  int64_t, int, int, hipStream_t, int, int);                     \
  template void launch_dcg_update<T>(const T*, int64_t, int64_t, int64_t, int, const T*,         \
                                     const T*, T*, T*, int64_t, int, CGState*, const T*, int,    \
                                     int64_t, T*, int64_t, int, int, hipStream_t, int);
INSTANTIATE(double)
INSTANTIATE(float)
#undef INSTANTIATE

}  // namespace rom
