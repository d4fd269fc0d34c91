// Deflated (recycled) CG on A g = r with the recycle space U = U_j (Sec. 4.2.1, CG form):
// the directions are kept A-orthogonal to U, p_k = s_k + beta p_{k-1} - U G^{-1} (AU)^T s_k
// with G = U^T A U.
//
// Two launches per step.  The direction is carried split as p_k = q_k - U c_k, with
// q_k = s_k + beta q_{k-1} and c_k = G^{-1} (AU)^T s_k + beta c_{k-1}, so that U itself is
// only read once per solve (g = g_q - U e at the end, e = sum of alpha_k c_k):
//   operator step: gamma_k = s_k^T s_k (from the previous launch's partials), the stopping
//     test, c_k; w_k = A p_k = A q_k - AU c_k, and in the same pass over the rows of AU the
//     partial sums of q^T w, q^T (AU c), s^T w, w^T w, (AU)^T w and (AU)^T s;
//   update: p^T w = q^T w - q^T (AU c) + c^T G c (U^T w = (AU)^T q - G c), alpha, the next
//     s^T s = gamma - 2 alpha s^T w + alpha^2 w^T w (for beta only; the next operator step
//     sums the exact value), s -= alpha w, g_q += alpha q, q = s + beta q, and the totals
//     (AU)^T s_k, (AU)^T w_k, from which the next operator step forms
//     (AU)^T s_{k+1} = (AU)^T s_k - alpha (AU)^T w_k.
// Per step the rows of AU are read once and those of U not at all, against twice (AU and
// U) for the unsplit recurrence.  No kernel synchronises across blocks: each writes
// per-block partial sums and the next launch reduces them; the scalar state and the small
// vectors live in device memory, so chunks of steps run without host round trips.
// T is the vector type: double for the plain form, float for the inner sweeps of the
// mixed form (FP32 vectors and FP32 sums); the CG scalars, c, e, the tolerance and
// G, G^{-1} stay FP64 in either case.
#include "kernels.h"

namespace rom {

namespace {

constexpr int CG_BS = 256;
constexpr int CG_GRID = 256;
constexpr int START_BS = 256;
constexpr int OP_BS = 256;

__global__ void k_cg_setup(CGState* cg, CGVec* cv, CgSetup su, int nb) {
  const int y = threadIdx.x;
  if (y < nb) {
    CGState* c = cg + y;
    c->tol2 = su.tol2[y];
    c->rscale = su.rscale[y];
    c->maxit = su.maxit[y];
    c->nj = su.nj[y];
    c->its = 0;
    c->kcur = 0;
    c->done = su.active[y] ? 0 : 1;
    c->flag = 0;
    c->gamma[0] = 0.0;
    c->gamma[1] = 0.0;
    c->pw = 0.0;
    c->alpha = 0.0;
    c->beta = 0.0;
    c->cGc = 0.0;
    c->gcur = 0.0;
    c->its2[0] = c->its2[1] = 0;
    c->cGc2[0] = c->cGc2[1] = 0.0;
  }
  for (int k = threadIdx.x; k < nb * NJ_MAX; k += blockDim.x) cv[k / NJ_MAX].e[k % NJ_MAX] = 0.0;
}

// Column c of a member's W or AW: the shared slot for the first ns columns, else the
// member's own (see Slots).  c is a compile-time index in the unrolled column loops, so
// the choice is one scalar select per column.
template <typename T>
__device__ __forceinline__ const T* col_of(const T* own, const T* shared, int ns, int c,
                                           int64_t ld) {
  return (c < ns ? shared : own) + (int64_t)c * ld;
}

// NP consecutive values at index i (vector loads for NP = 2 and 4: i a multiple of NP and
// the array aligned, as the two- and four-node walks require).
template <typename T>
__device__ __forceinline__ void ldn(const T* __restrict__ p, int64_t i, T (&v)[1]) {
  v[0] = p[i];
}
template <typename T>
__device__ __forceinline__ void ldn(const T* __restrict__ p, int64_t i, T (&v)[2]) {
  const typename Vec2<T>::type t = *reinterpret_cast<const typename Vec2<T>::type*>(p + i);
  v[0] = t.x;
  v[1] = t.y;
}
template <typename T>
__device__ __forceinline__ void ldn(const T* __restrict__ p, int64_t i, T (&v)[4]) {
  const typename Vec4<T>::type t = *reinterpret_cast<const typename Vec4<T>::type*>(p + i);
  v[0] = t.x;
  v[1] = t.y;
  v[2] = t.z;
  v[3] = t.w;
}
template <typename T>
__device__ __forceinline__ void stn(T* __restrict__ p, int64_t i, const T (&v)[1]) {
  p[i] = v[0];
}
template <typename T>
__device__ __forceinline__ void stn(T* __restrict__ p, int64_t i, const T (&v)[2]) {
  *reinterpret_cast<typename Vec2<T>::type*>(p + i) = typename Vec2<T>::type{v[0], v[1]};
}
template <typename T>
__device__ __forceinline__ void stn(T* __restrict__ p, int64_t i, const T (&v)[4]) {
  *reinterpret_cast<typename Vec4<T>::type*>(p + i) = typename Vec4<T>::type{v[0], v[1], v[2], v[3]};
}

// Block order of the CG kernels that read the members' shared data (one-dimensional grid
// of round_up(ntiles, NXCD) * nb blocks): the nb members' blocks of one tile are handed out
// one after another to the same XCD, so the data they share (the shared columns of U and
// AU; in the operator step also the diagonal and face coefficients) is fetched from HBM
// once into that XCD's L2 whatever the grid size.  In the operator step tile t is
// x-position block t % gx of z chunk t / gx; in the start and finish (gx = ntiles) it is
// the row chunk.  Blocks past the last tile (t >= ntiles) have no work.
struct StepBlock {
  int y, t, tx, tz;
  bool valid;
};
__device__ __forceinline__ StepBlock step_block(int gx, int ntiles, int nb) {
  const int L = blockIdx.x;
  const int r = L / NXCD;
  StepBlock b;
  b.y = r % nb;
  b.t = (r / nb) * NXCD + L % NXCD;
  b.valid = b.t < ntiles;
  b.tx = b.t % gx;
  b.tz = b.t / gx;
  return b;
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

// y[j] = scale * sum_c Ginv[j + c nj] t[c] for threads j < nj, in FP64 (the loop is
// unrolled to NJT so that the row loads, where not prefetched, issue together).
template <int NJT, bool PF, typename S>
__device__ __forceinline__ double gram_row_apply(const double* __restrict__ Ginv,
                                                 const double (&gr)[PF ? NJT : 1], int nj,
                                                 const S* t, double scale) {
  const int j = threadIdx.x;
  double y = 0.0;
  if (j < nj) {
#pragma unroll
    for (int c = 0; c < NJT; ++c)
      if (c < nj) y += (PF ? gr[PF ? c : 0] : Ginv[j + c * nj]) * (double)t[c];
  }
  return scale * y;
}

// Rows per thread of the start kernel (it reads both U and AU): as many as keep the loaded
// rows and the running sums in registers.
template <typename T, int NJT>
struct StartRows {
  static constexpr int value = sizeof(T) == 8 ? (NJT <= 8 ? 4 : NJT <= 16 ? 2 : 0)
                                              : (NJT <= 16 ? 4 : 0);
};

// Start: y0 = G^{-1} U^T r (U^T r in cg->t), g = U y0, s = q = r - AU y0; partials of
// (AU)^T s (values 0..nj-1) and s^T s (value NJT).  The right-hand side is FP64 and is
// read as rscale * r (the mixed form solves for a unit-norm residual in FP32).  A thread
// loads its first chunk's rows before y0 is formed.  V: values per access (16-byte
// accesses where the launcher finds n, the strides and the arrays aligned for them; the
// kernel is bound by its load instructions), RPT / V accesses per thread and pass.
template <typename T, int NJT, int RPT = StartRows<T, NJT>::value, int V = 1>
__global__ __launch_bounds__(START_BS) void k_dcg_start(const T* __restrict__ W0,
                                                         const T* __restrict__ AW0,
                                                         Slots sl, int64_t n,
                                                         const double* __restrict__ Ginv,
                                                         int64_t gstride,
                                                         const double* __restrict__ r,
                                                         int64_t rstride, T* __restrict__ g,
                                                         T* __restrict__ s, T* __restrict__ qv,
                                                         int64_t vstride, const CGState* cgs,
                                                         T* __restrict__ ps, int64_t psstride,
                                                         int P, int nb) {
  const StepBlock bk = step_block(P, P, nb);
  if (!bk.valid) return;
  const int y = bk.y;
  const CGState* cg = cgs + y;
  if (cg->done) return;
  const int64_t ld = sl.ld;
  const int ns = sl.ns;
  const T* __restrict__ W = W0 + y * sl.wstride;
  const T* __restrict__ AW = AW0 + y * sl.wstride;
  const T* __restrict__ Ws = W0 + sl.soff;
  const T* __restrict__ AWs = AW0 + sl.soff;
  Ginv += y * gstride;
  r += y * rstride;
  g += y * vstride;
  s += y * vstride;
  qv += y * vstride;
  ps += y * psstride;
  const int nj = cg->nj;
  const double rscale = cg->rscale;
  constexpr bool PRE = RPT > 0;
  static_assert(V == 1 || (PRE && RPT % V == 0), "vector accesses need the preloaded rows");
  constexpr int R = PRE ? RPT / V : 1;
  constexpr int64_t STEP = (int64_t)START_BS * V;   // elements between a thread's accesses
  constexpr int64_t CH = STEP * R;
  int64_t base = (int64_t)bk.t * CH + (int64_t)threadIdx.x * V;
  T wr[R][PRE ? NJT : 1][V], ar[R][PRE ? NJT : 1][V], rv[R][V];
  auto zero = [](T (&v)[V]) {
#pragma unroll
    for (int e = 0; e < V; ++e) v[e] = T(0);
  };
  // V FP64 values of r at i (16-byte loads for V > 1)
  auto ldr = [&](int64_t i, T (&v)[V]) {
    if (V == 1) {
      v[0] = (T)r[i];
    } else {
#pragma unroll
      for (int h = 0; h < V; h += 2) {
        const double2 t = *reinterpret_cast<const double2*>(r + i + h);
        v[h] = (T)t.x;
        v[h + 1] = (T)t.y;
      }
    }
  };
  // with V > 1, n is a multiple of V: an access's values are all in range or all past it
  auto load = [&](int64_t b0) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int64_t i = b0 + (int64_t)q * STEP;
      const bool in = i < n;
      if (in) ldr(i, rv[q]); else zero(rv[q]);
      if (PRE) {
#pragma unroll
        for (int c = 0; c < NJT; ++c) {
          if (in && c < nj) {
            ldn(col_of(W, Ws, ns, c, ld), i, wr[q][PRE ? c : 0]);
            ldn(col_of(AW, AWs, ns, c, ld), i, ar[q][PRE ? c : 0]);
          } else {
            zero(wr[q][PRE ? c : 0]);
            zero(ar[q][PRE ? c : 0]);
          }
        }
      }
    }
  };
  load(base);
  __shared__ T ys[NJ_MAX];
  constexpr bool GPF = GramPf<NJT>::value;
  double gr[GPF ? NJT : 1];
  gram_row<NJT, GPF>(Ginv, nj, gr);
  const double y0 = gram_row_apply<NJT, GPF>(Ginv, gr, nj, cg->t, rscale);
  if (threadIdx.x < nj) ys[threadIdx.x] = (T)y0;
  __syncthreads();
  const T rs = (T)rscale;
  T acc[NJT + 1];
#pragma unroll
  for (int c = 0; c <= NJT; ++c) acc[c] = T(0);
  for (;;) {
    // without a preload the row of A U is still kept between its two uses when it fits
    constexpr bool KEEP = !PRE && NJT * sizeof(T) <= 256;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int64_t i = base + (int64_t)q * STEP;
      const bool in = i < n;
      T gi[V], si[V];
#pragma unroll
      for (int e = 0; e < V; ++e) {
        gi[e] = T(0);
        si[e] = rs * rv[q][e];
      }
      T kept[KEEP ? NJT : 1];
#pragma unroll
      for (int c = 0; c < NJT; ++c)
        if (c < nj) {
          const T yc = ys[c];
#pragma unroll
          for (int e = 0; e < V; ++e) {
            const T wv = PRE ? wr[q][PRE ? c : 0][e]
                             : (in ? col_of(W, Ws, ns, c, ld)[i] : T(0));
            const T av = PRE ? ar[q][PRE ? c : 0][e]
                             : (in ? col_of(AW, AWs, ns, c, ld)[i] : T(0));
            if (KEEP) kept[KEEP ? c : 0] = av;
            gi[e] += wv * yc;
            si[e] -= av * yc;
          }
        }
      if (in) {
        stn(g, i, gi);
        stn(s, i, si);
        stn(qv, i, si);
      }
#pragma unroll
      for (int e = 0; e < V; ++e) acc[NJT] += si[e] * si[e];   // 0 past the end
#pragma unroll
      for (int c = 0; c < NJT; ++c)
        if (c < nj) {
#pragma unroll
          for (int e = 0; e < V; ++e)
            acc[c] += (PRE ? ar[q][PRE ? c : 0][e]
                           : KEEP ? kept[KEEP ? c : 0]
                                  : (in ? col_of(AW, AWs, ns, c, ld)[i] : T(0))) * si[e];
        }
    }
    base += (int64_t)P * CH;
    if (base - (int64_t)threadIdx.x * V >= n) break;
    load(base);
  }
  write_partials_t<NJT + 1, START_BS>(acc, ps, bk.t, P);
}

// The same loads and stores at byte offset bo from an array's base p (wave-uniform).  The
// step kernels keep one 32-bit offset per lane, so each access is an SGPR base plus a
// VGPR offset rather than a 64-bit address per array and lane; the launchers check that
// every offset fits in 32 bits.
template <typename T, int N>
__device__ __forceinline__ void ldb(const T* p, uint32_t bo, T (&v)[N]) {
  ldn(reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + bo), 0, v);
}
// one value OFF elements past offset bo (the constant shift goes into the instruction)
template <int OFF, typename T>
__device__ __forceinline__ T ld1(const T* p, uint32_t bo) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + bo)[OFF];
}
template <typename T, int N>
__device__ __forceinline__ void stb(T* p, uint32_t bo, const T (&v)[N]) {
  stn(reinterpret_cast<T*>(reinterpret_cast<char*>(p) + bo), 0, v);
}

// How the operator step sums its 2 NJT vector dot products.  Up to 8 FP64 or 16 FP32
// columns every thread keeps running sums in registers over its z planes and the block
// reduces them once at the end.  Wider (up to 128 sums) each plane's values are reduced
// over the wave at once and
// accumulated in LDS by the wave's first lane (every lane of the block then walks every
// plane, lanes past the plane with zero values, so the wave reductions see full waves).
// pre: the rows of AU are loaded with the rest of a plane (before the first plane's
// prologue reductions, so their latency hides behind them) where they fit in registers.
template <typename T, int NJT>
struct OpMode {
  static constexpr bool imm = NJT * sizeof(T) >= 128;
  static constexpr bool pre = NJT * sizeof(T) <= 128;
  // without pre, the rows are kept between their two uses where they fit, else reloaded
  static constexpr bool keep = !imm && !pre && NJT * sizeof(T) <= 128;
};

// Everything one z plane of the operator step reads for NP consecutive x-nodes at i: the
// next plane of q (the current and previous ones are carried), the lateral neighbours of q,
// the diagonal, the face coefficients (D field), s and, with pre, the rows of AU.
template <typename T, bool VAR, int NP, int NJT, bool PRE>
struct OpPlane {
  T xp[NP], xl, xr, yd[NP], yu[NP], d[NP], s[NP];
  T fxl, fx[NP], fyd[NP], fyu[NP], fp[NP];
  T a[PRE ? NJT : 1][NP];
};

// The operator step of member y over the z planes [tz zc, + zc) of the x-y positions of
// block tx (NP consecutive x-nodes per thread; see step_block).  See the file comment.
// LY (four-node walk, a block's positions whole rows of the plane): each plane's q and
// y-face coefficients are staged in LDS (two buffers, one barrier per plane), and a
// position's y-neighbours inside the block's rows are read from there; only the block's
// first and last rows load theirs.
template <typename T, bool VAR, int NP, int NJT, bool LY = false>
__global__ __launch_bounds__(OP_BS) void k_dcg_op(Stencil S, const T* __restrict__ diag,
                                                   const T* __restrict__ q0,
                                                   const T* __restrict__ s0, T* __restrict__ w0,
                                                   int64_t vstride, const T* __restrict__ AW0,
                                                   Slots sl, const double* __restrict__ Ginv0,
                                                   const double* __restrict__ Gm0,
                                                   int64_t gstride, int zc, int gx, int ntiles,
                                                   int nb, CGState* cgs,
                                                   CGVec* cvs, const T* __restrict__ ps0, int Ps,
                                                   int64_t psstride, const T* __restrict__ pu0,
                                                   int Pu, int64_t pustride, T* __restrict__ po0,
                                                   int64_t postride) {
  constexpr bool IMM = OpMode<T, NJT>::imm;
  constexpr bool PRE = OpMode<T, NJT>::pre;
  constexpr bool KEEP = OpMode<T, NJT>::keep;
  // the column walk without a branch per column (the rows past nj are 0 and their sums
  // unused) where the sums stay in registers; with per-plane wave reductions the columns
  // past nj are skipped
  constexpr bool FREE = PRE && !IMM;
  const StepBlock bk = step_block(gx, ntiles, nb);
  if (!bk.valid) return;
  const int y = bk.y;
  CGState* cg = cgs + y;
  if (cg->done) return;
  CGVec* cv = cvs + y;
  const T* __restrict__ q = q0 + y * vstride;
  const T* __restrict__ s = s0 + y * vstride;
  T* __restrict__ w = w0 + y * vstride;
  const int64_t ld = sl.ld;
  const int ns = sl.ns;
  const T* __restrict__ AW = AW0 + y * sl.wstride;
  const T* __restrict__ AWs = AW0 + sl.soff;
  const double* __restrict__ Ginv = Ginv0 + y * gstride;
  const int nj = cg->nj;
  const int k = cg->its;

  // ---- this thread's nodes, and the first plane's loads (issued before the reductions)
  const T *Fx, *Fy, *Fz;
  walk_faces(S, T(0), Fx, Fy, Fz);
  const int nxy = S.nx * S.ny;
  const int rowp = S.nx / NP;       // positions (groups of NP x-nodes) per row
  const int npos = rowp * S.ny;
  const int qpos = bk.tx * OP_BS + threadIdx.x;
  const bool act = qpos < npos;
  const int qq = act ? qpos : 0;   // lanes past the plane read position 0 (zero weight)
  const int ix = NP * (qq % rowp);
  const int iy = qq / rowp;
  const bool hl = ix > 0, hr = ix + NP < S.nx, hd = iy > 0, hu = iy < S.ny - 1;
  const int z0 = bk.tz * zc;
  const int z1 = min(z0 + zc, S.nz);
  const bool walk = z0 < z1 && (act || IMM);
  // byte offset of this thread's first node: every load below is an array's base plus
  // this offset, shifted by a row (bx) or a plane (bplane) where it reads a neighbour
  uint32_t bi = (uint32_t)(((int64_t)z0 * nxy + (int64_t)iy * S.nx + ix) * (int64_t)sizeof(T));
  const uint32_t bplane = (uint32_t)nxy * (uint32_t)sizeof(T);
  const uint32_t bx = (uint32_t)S.nx * (uint32_t)sizeof(T);
  auto zero = [](T (&v)[NP]) {
#pragma unroll
    for (int u = 0; u < NP; ++u) v[u] = T(0);
  };
  OpPlane<T, VAR, NP, NJT, PRE> P;
  if (PRE) {
#pragma unroll
    for (int c = 0; c < NJT; ++c) zero(P.a[PRE ? c : 0]);
  }
  T xm[NP], xc[NP], fm[NP];
  // XS (the four-node walk): a wave holds consecutive positions, so the x-neighbours of a
  // position are the adjacent lanes' end values (moved across the wave below); only the
  // wave's first and last lanes load theirs
  constexpr bool XS = NP == 4;
  static_assert(!LY || XS, "the LDS y-neighbours need the four-node walk");
  const int xln = threadIdx.x % WAVE;
  const int lrw = LY ? threadIdx.x / rowp : 0;   // row within the block's rows
  const bool frow = !LY || lrw == 0, lrow = !LY || lrw == OP_BS / rowp - 1;
  __shared__ __align__(16) T lyq[LY ? 2 * OP_BS * NP : 1];
  __shared__ __align__(16) T lyf[(LY && VAR) ? 2 * OP_BS * NP : 1];
  auto load_plane = [&](uint32_t bj, int z) {
    if (z < S.nz - 1) ldb(q, bj + bplane, P.xp); else zero(P.xp);
    P.xl = (hl && (!XS || xln == 0)) ? ld1<-1>(q, bj) : T(0);
    P.xr = (hr && (!XS || xln == WAVE - 1)) ? ld1<NP>(q, bj) : T(0);
    if (hd && frow) ldb(q, bj - bx, P.yd); else zero(P.yd);
    if (hu && lrow) ldb(q, bj + bx, P.yu); else zero(P.yu);
    ldb(diag, bj, P.d);
    if (VAR) {
      P.fxl = (hl && (!XS || xln == 0)) ? ld1<-1>(Fx, bj) : T(0);
      ldb(Fx, bj, P.fx);
      if (hd && frow) ldb(Fy, bj - bx, P.fyd); else zero(P.fyd);
      ldb(Fy, bj, P.fyu);
      if (S.dim == 3) ldb(Fz, bj, P.fp); else zero(P.fp);
    }
    if (act) ldb(s, bj, P.s); else zero(P.s);
    if (PRE) {
      // the loads are the kernel's limit (address processing per load instruction), so the
      // columns past nj are not loaded (a uniform branch per column, without an else: their
      // registers keep the 0 they start with, their coefficient is 0 and their sums unused);
      // lanes past the plane read position 0 and add nothing (their s and w are 0)
#pragma unroll
      for (int c = 0; c < NJT; ++c)
        if (c < nj) ldb(col_of(AW, AWs, ns, c, ld), bj, P.a[PRE ? c : 0]);
    }
  };
  if (walk) {
    if (z0 > 0) ldb(q, bi - bplane, xm); else zero(xm);
    if (VAR && z0 > 0) ldb(Fz, bi - bplane, fm); else zero(fm);
    ldb(q, bi, xc);
    load_plane(bi, z0);
  }

  // ---- gamma_k = s_k^T s_k and t = (AU)^T s_k: from the start's partials at the first step,
  // else gamma from the update's partials and t by the recurrence
  const bool first = k == 0;
  const double tol2 = cg->tol2;
  const int maxit = cg->maxit;
  const double alpha = cg->alpha, beta = cg->beta;
  constexpr bool GPF = GramPf<NJT>::value;
  double gr[GPF ? NJT : 1];
  gram_row<NJT, GPF>(Ginv, nj, gr);
  __shared__ T tot[NJT + 1];
  __shared__ double tv[NJ_MAX];
  double gam;
  if (first) {
    sum_partials_t<NJT + 1, OP_BS>(ps0 + y * psstride, Ps, tot);
    gam = (double)tot[NJT];
    if (threadIdx.x < nj) tv[threadIdx.x] = (double)tot[threadIdx.x];
  } else {
    if (threadIdx.x < nj) tv[threadIdx.x] = cv->ts[threadIdx.x] - alpha * cv->tw[threadIdx.x];
    sum_partials_t<1, OP_BS>(pu0 + y * pustride, Pu, tot);
    gam = (double)tot[0];
  }
  const bool lead = bk.t == 0;
  const bool nonfinite = !isfinite(gam);
  const bool stop = nonfinite || gam <= tol2 || k >= maxit;
  if (lead && threadIdx.x == 0) {
    cg->gamma[k & 1] = gam;
    cg->gcur = gam;
    cg->kcur = k;
    if (nonfinite) cg->flag = 2;
    if (stop) cg->done = 1;
  }
  if (stop) return;
  __syncthreads();
  // c_k = G^{-1} t + beta c_{k-1} (c_0 = G^{-1} t)
  __shared__ T cs[NJ_MAX];
  __shared__ double cd[NJ_MAX];
  {
    const int j = threadIdx.x;
    double cj = gram_row_apply<NJT, GPF>(Ginv, gr, nj, tv, 1.0);
    if (j < nj) {
      if (!first) cj += beta * cv->c[(k - 1) & 1][j];
      cs[j] = (T)cj;
      cd[j] = cj;
      if (lead) cv->c[k & 1][j] = cj;
    } else if (j < NJT) {
      cs[j] = T(0);   // the padding columns of the branch-free walk
    }
  }
  __syncthreads();
  if (lead && threadIdx.x < WAVE) {
    // c^T G c for the update's p^T w (one wave; lanes past nj add zero)
    const double* __restrict__ Gm = Gm0 + y * gstride;
    const int j = threadIdx.x;
    double v = 0.0;
    if (j < nj) {
      double gc = 0.0;
      for (int c = 0; c < nj; ++c) gc += Gm[j + c * nj] * cd[c];
      v = cd[j] * gc;
    }
    v = wave_sum(v);
    if (j == 0) cg->cGc = v;
  }

  // ---- the planes
  constexpr int RV = 4 + (IMM ? 0 : 2 * NJT);
  T acc[RV];
#pragma unroll
  for (int r = 0; r < RV; ++r) acc[r] = T(0);
  __shared__ T imm[IMM ? (OP_BS / WAVE) * 2 * NJT : 1];
  const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
  if (IMM) {
    for (int r = threadIdx.x; r < (OP_BS / WAVE) * 2 * NJT; r += OP_BS) imm[r] = T(0);
    __syncthreads();
  }
  // vector sum r of x^T y over this thread's nodes: in registers, or reduced over the wave
  // and added to the wave's LDS slot
  auto vadd = [&](int r, const T (&x)[NP], const T (&y)[NP]) {
    if (IMM) {
      T v = T(0);
#pragma unroll
      for (int u = 0; u < NP; ++u) v += x[u] * y[u];
      v = wave_sum(v);
      if (lane == 0) imm[wid * 2 * NJT + r] += v;
    } else {
#pragma unroll
      for (int u = 0; u < NP; ++u) acc[4 + r] += x[u] * y[u];
    }
  };
  const T cx = (T)S.cx, cy = (T)S.cy, cz = (T)S.cz;
  const T m = act ? T(1) : T(0);
  // one plane; more: load the next one (the last plane of the chunk is peeled off below, so
  // that the loop's loads need no branch: under one, the registers of the plane would be
  // merged and copied every plane)
  auto plane = [&](int z, bool more) __attribute__((always_inline)) {
    // y-neighbours: loaded, or with LY from the plane's rows staged in LDS
    T yd[NP], yu[NP], fyd[NP];
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      yd[u] = P.yd[u];
      yu[u] = P.yu[u];
      fyd[u] = VAR ? P.fyd[u] : T(0);
    }
    if (LY) {
      const int bo = ((z - z0) & 1) * OP_BS * NP;
      T* tq = lyq + bo;
      T* tf = lyf + ((LY && VAR) ? bo : 0);
      const int me = threadIdx.x * NP;
      stn(tq, me, xc);
      if (VAR) stn(tf, me, P.fyu);
      __syncthreads();
      // inside the block's rows the neighbour rows exist (hd, hu hold there)
      if (!frow) {
        ldn(tq, me - rowp * NP, yd);
        if (VAR) ldn(tf, me - rowp * NP, fyd);
      }
      if (!lrow) ldn(tq, me + rowp * NP, yu);
    }
    // (A q) at the NP nodes
    T xl = P.xl, xr = P.xr, fxl = P.fxl;
    if (XS) {
      // whole-wave shifts by one lane: lane l takes lane l - 1's last and lane l + 1's
      // first value (the first and last lanes keep their loaded ones); 0 off the grid
      const T sl = wave_shr1(xc[NP - 1]), sr = wave_shl1(xc[0]);
      xl = hl ? (xln == 0 ? P.xl : sl) : T(0);
      xr = hr ? (xln == WAVE - 1 ? P.xr : sr) : T(0);
      if (VAR) {
        const T sf = wave_shr1(P.fx[NP - 1]);
        fxl = hl ? (xln == 0 ? P.fxl : sf) : T(0);
      }
    }
    T av[NP], xq[NP];
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const T left = u == 0 ? xl : xc[u - 1];
      const T right = u == NP - 1 ? xr : xc[u + 1];
      T v = P.d[u] * xc[u];
      if (!VAR) {
        v -= cx * (left + right) + cy * (yd[u] + yu[u]) + cz * (xm[u] + P.xp[u]);
      } else {
        const T fl = u == 0 ? fxl : P.fx[u - 1];
        v -= fl * left + P.fx[u] * right;
        v -= fyd[u] * yd[u] + P.fyu[u] * yu[u];
        if (S.dim == 3) v -= fm[u] * xm[u] + P.fp[u] * P.xp[u];
      }
      av[u] = v;   // masked in w below
      xq[u] = m * xc[u];
    }
    // pass 1 over the rows of AU: AU c, (AU)^T s
    T au[NP], wv[NP];
    zero(au);
    T keep[KEEP ? NJT : 1][NP];
#pragma unroll
    for (int c = 0; c < NJT; ++c)
      if (FREE || c < nj) {
        T a[NP];
        if (PRE) {
#pragma unroll
          for (int u = 0; u < NP; ++u) a[u] = P.a[PRE ? c : 0][u];
        } else if (act) {
          ldb(col_of(AW, AWs, ns, c, ld), bi, a);
        } else {
          zero(a);
        }
        if (KEEP) {
#pragma unroll
          for (int u = 0; u < NP; ++u) keep[KEEP ? c : 0][u] = a[u];
        }
        const T cc = cs[c];
#pragma unroll
        for (int u = 0; u < NP; ++u) au[u] += a[u] * cc;
        vadd(NJT + c, a, P.s);
      }
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      wv[u] = m * (av[u] - au[u]);
      acc[0] += xq[u] * wv[u];
      acc[1] += xq[u] * au[u];
      acc[2] += P.s[u] * wv[u];
      acc[3] += wv[u] * wv[u];
    }
    if (act) stb(w, bi, wv);
    // pass 2: (AU)^T w
#pragma unroll
    for (int c = 0; c < NJT; ++c)
      if (FREE || c < nj) {
        T a[NP];
        if (PRE) {
#pragma unroll
          for (int u = 0; u < NP; ++u) a[u] = P.a[PRE ? c : 0][u];
        } else if (KEEP) {
#pragma unroll
          for (int u = 0; u < NP; ++u) a[u] = keep[KEEP ? c : 0][u];
        } else if (act) {
          ldb(col_of(AW, AWs, ns, c, ld), bi, a);
        } else {
          zero(a);
        }
        vadd(c, a, wv);
      }
    // next plane
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      xm[u] = xc[u];
      xc[u] = P.xp[u];
      if (VAR) fm[u] = P.fp[u];
    }
    if (more) load_plane(bi + bplane, z + 1);
  };
  int z = z0;
  for (; walk && z < z1 - 1; ++z, bi += bplane) plane(z, true);
  if (walk) plane(z, false);
  T* __restrict__ po = po0 + y * postride;
  const int P1 = ntiles;
  const int bid = bk.t;
  if (!IMM) {
    write_partials_t<RV, OP_BS>(acc, po, bid, P1);
  } else {
    T a4[4] = {acc[0], acc[1], acc[2], acc[3]};
    write_partials_t<4, OP_BS>(a4, po, bid, P1);
    __syncthreads();
    for (int r = threadIdx.x; r < 2 * NJT; r += OP_BS) {
      T t = T(0);
#pragma unroll
      for (int v = 0; v < OP_BS / WAVE; ++v) t += imm[v * 2 * NJT + r];
      po[(size_t)(4 + r) * P1 + bid] = t;
    }
  }
}

// Totals of R transposed partial rows of P blocks, every row's loads issued before any
// reduction: wave w sums rows w, w + NW, ... (NW waves), each lane a strided share of the P
// blocks, so a block waits one memory latency for all R totals instead of one per row.
// tot[] (shared) is visible to every thread on return.
template <int R, int BS, typename T>
__device__ __forceinline__ void sum_rows_wide(const T* __restrict__ partials, int P, T* tot) {
  constexpr int NW = BS / WAVE;
  constexpr int RPW = (R + NW - 1) / NW;
  const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
  T a[RPW];
#pragma unroll
  for (int k = 0; k < RPW; ++k) a[k] = T(0);
  for (int b = lane; b < P; b += WAVE) {
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const int r = wid + k * NW;
      if (r < R) a[k] += partials[(size_t)r * P + b];
    }
  }
#pragma unroll
  for (int k = 0; k < RPW; ++k) {
    const int r = wid + k * NW;
    const T v = wave_sum(a[k]);
    if (lane == 0 && r < R) tot[r] = v;
  }
  __syncthreads();
}

// One whole step in one launch (member y; see step_block), for latency-bound sizes: launch j
// applies update j-1 at this block's nodes and then operator step j.  s, q and w are kept
// in two buffers by step parity (par = j & 1, at + par pstride): launch j reads s_{j-1},
// q_{j-1}, w_{j-1} from the other buffer and writes s_j, q_j, w_j; q_j at a node's
// neighbours is formed there from s_{j-1}, w_{j-1}, q_{j-1}
// (q_j = s_{j-1} - alpha w_{j-1} + beta q_{j-1}), so no launch waits for another's update.
// Every block sums the previous launch's partial rows itself (5 scalars q^T w, q^T (AU c),
// s^T w, w^T w, s^T s and the 2 NJT totals (AU)^T w, (AU)^T s): alpha, beta, c_j and the
// stopping test on the exact s_{j-1}^T s_{j-1} follow.  The scalars the lead block writes
// for the next launch (updates done, c, c^T G c, gamma) sit in parity slots, so no block
// reads a value another block of the same launch rewrites.  first: the launch right after
// the start (par 0): no update, q_0 = s_0 read directly, gamma_0 and (AU)^T s_0 from the
// start's partials.  Pprev: the previous launch's block count (its partial rows).
template <typename T, bool VAR, int NP, int NJT>
__global__ __launch_bounds__(OP_BS) void k_dcg_iter(Stencil S, const T* __restrict__ diag,
                                                     T* __restrict__ sb, T* __restrict__ qb,
                                                     T* __restrict__ wb, int64_t pstride,
                                                     int64_t vstride, T* __restrict__ g0,
                                                     const T* __restrict__ AW0, Slots sl,
                                                     const double* __restrict__ Ginv0,
                                                     const double* __restrict__ Gm0,
                                                     int64_t gstride, int zc, int gx, int ntiles,
                                                     int nb, CGState* cgs,
                                                     CGVec* cvs, const T* __restrict__ ps0, int Ps,
                                                     int64_t psstride, T* __restrict__ po0,
                                                     int64_t postride, int64_t pohalf, int Pprev,
                                                     int par, int first) {
  constexpr bool IMM = OpMode<T, NJT>::imm;
  constexpr bool PRE = OpMode<T, NJT>::pre;
  constexpr bool KEEP = OpMode<T, NJT>::keep;
  constexpr int RS = 5;                      // scalar partials
  const StepBlock bk = step_block(gx, ntiles, nb);
  if (!bk.valid) return;
  const int y = bk.y;
  CGState* cg = cgs + y;
  if (cg->done) return;
  CGVec* cv = cvs + y;
  const int rp = first ? 0 : 1 - par;        // parity of the buffers read
  const T* __restrict__ sr = sb + rp * pstride + y * vstride;
  const T* __restrict__ qr = qb + rp * pstride + y * vstride;
  // step 0 reads no w: its loads then read s (finite values, weight 0), so that no load
  // depends on the step
  const T* __restrict__ wr = first ? sr : wb + rp * pstride + y * vstride;
  T* __restrict__ sw_ = sb + par * pstride + y * vstride;
  T* __restrict__ qw_ = qb + par * pstride + y * vstride;
  T* __restrict__ ww_ = wb + par * pstride + y * vstride;
  T* __restrict__ g = g0 + y * vstride;
  const int64_t ld = sl.ld;
  const int ns = sl.ns;
  const T* __restrict__ AW = AW0 + y * sl.wstride;
  const T* __restrict__ AWs = AW0 + sl.soff;
  const double* __restrict__ Ginv = Ginv0 + y * gstride;
  const int nj = cg->nj;

  // ---- this thread's nodes, and the first plane's raw loads (before the reductions)
  const T *Fx, *Fy, *Fz;
  walk_faces(S, T(0), Fx, Fy, Fz);
  const int nxy = S.nx * S.ny;
  const int npos = NP == 2 ? (S.nx / 2) * S.ny : nxy;
  const int qpos = bk.tx * OP_BS + threadIdx.x;
  const bool act = qpos < npos;
  const int qq = act ? qpos : 0;
  const int ix = NP == 2 ? 2 * (qq % (S.nx / 2)) : qq % S.nx;
  const int iy = NP == 2 ? qq / (S.nx / 2) : qq / S.nx;
  const bool hl = ix > 0, hr = ix + NP < S.nx, hd = iy > 0, hu = iy < S.ny - 1;
  const int z0 = bk.tz * zc;
  const int z1 = min(z0 + zc, S.nz);
  const bool walk = z0 < z1 && (act || IMM);
  int64_t i = (int64_t)z0 * nxy + (int64_t)iy * S.nx + ix;
  auto ldv = [&] __attribute__((always_inline)) (const T* p, int64_t j, T (&v)[NP]) { ldn(p, j, v); };
  auto zero = [] __attribute__((always_inline)) (T (&v)[NP]) {
#pragma unroll
    for (int u = 0; u < NP; ++u) v[u] = T(0);
  };
  // raw (s, w, q) of the previous step at a position: NP values or one scalar
  struct Tri {
    T s[NP], w[NP], q[NP];
  };
  struct Tri1 {
    T s, w, q;
  };
  auto ld3 = [&] __attribute__((always_inline)) (int64_t j, Tri& r) {
    ldv(sr, j, r.s);
    ldv(qr, j, r.q);
    ldv(wr, j, r.w);
  };
  auto z3 = [&] __attribute__((always_inline)) (Tri& r) {
    zero(r.s);
    zero(r.w);
    zero(r.q);
  };
  struct Plane {
    Tri own, xp, yd, yu;
    Tri1 xl, xr;
    T gv[NP], d[NP];
    T fxl, fx[NP], fyd[NP], fyu[NP], fp[NP];
    T a[PRE ? NJT : 1][NP];
    T mxp;   // 0 on the top plane (whose upper neighbours are read from the plane itself)
  } P;
  Tri xm3;           // raw values of the plane below the chunk (its q_j is formed later)
  T fm[NP];
  auto load_plane = [&] __attribute__((always_inline)) (int64_t j, int z) {
    if (act) ld3(j, P.own); else z3(P.own);
    if (act) ldv(g, j, P.gv); else zero(P.gv);
    const bool zin = z < S.nz - 1;
    ld3(j + (zin ? nxy : 0), P.xp);
    P.mxp = zin ? T(1) : T(0);
    P.xl.s = hl ? sr[j - 1] : T(0);
    P.xl.q = hl ? qr[j - 1] : T(0);
    P.xl.w = hl ? wr[j - 1] : T(0);
    P.xr.s = hr ? sr[j + NP] : T(0);
    P.xr.q = hr ? qr[j + NP] : T(0);
    P.xr.w = hr ? wr[j + NP] : T(0);
    if (hd) ld3(j - S.nx, P.yd); else z3(P.yd);
    if (hu) ld3(j + S.nx, P.yu); else z3(P.yu);
    ldv(diag, j, P.d);
    if (VAR) {
      P.fxl = hl ? Fx[j - 1] : T(0);
      ldv(Fx, j, P.fx);
      if (hd) ldv(Fy, j - S.nx, P.fyd); else zero(P.fyd);
      ldv(Fy, j, P.fyu);
      if (S.dim == 3) ldv(Fz, j, P.fp); else zero(P.fp);
    }
    if (PRE) {
#pragma unroll
      for (int c = 0; c < NJT; ++c)
        if (c < nj) {
          if (act) ldv(col_of(AW, AWs, ns, c, ld), j, P.a[PRE ? c : 0]);
          else zero(P.a[PRE ? c : 0]);
        }
    }
  };
  if (walk) {
    if (z0 > 0) ld3(i - nxy, xm3); else z3(xm3);
    if (VAR && z0 > 0) ldv(Fz, i - nxy, fm); else zero(fm);
    load_plane(i, z0);
  }

  // ---- the previous launch's (or the start's) sums
  const double tol2 = cg->tol2;
  const int maxit = cg->maxit;
  const int done_its = first ? 0 : cg->its2[rp];
  const double cGc_prev = first ? 0.0 : cg->cGc2[rp];
  constexpr bool GPF = GramPf<NJT>::value;
  double gr[GPF ? NJT : 1];
  gram_row<NJT, GPF>(Ginv, nj, gr);
  __shared__ T tot[RS + 2 * NJT];
  __shared__ double tv[NJ_MAX];
  __shared__ double cprev[NJ_MAX];
  if (threadIdx.x < NJT) cprev[threadIdx.x] = first ? 0.0 : cv->c[rp][threadIdx.x];
  double gam, al = 0.0, be = 0.0, pw = 1.0;
  if (first) {
    sum_rows_wide<NJT + 1, OP_BS>(ps0 + y * psstride, Ps, tot);
    gam = (double)tot[NJT];
    if (threadIdx.x < NJT) tv[threadIdx.x] = (double)tot[threadIdx.x];
  } else {
    sum_rows_wide<RS + 2 * NJT, OP_BS>(po0 + y * postride + rp * pohalf, Pprev, tot);
    gam = (double)tot[4];
    pw = (double)tot[0] - (double)tot[1] + cGc_prev;
    al = gam / pw;
    double gnext = gam - 2.0 * al * (double)tot[2] + al * al * (double)tot[3];
    if (!(gnext > 0.0)) gnext = 0.0;
    be = gnext / gam;
    if (threadIdx.x < NJT)
      tv[threadIdx.x] = (double)tot[RS + NJT + threadIdx.x] - al * (double)tot[RS + threadIdx.x];
  }
  const bool lead = bk.t == 0;
  const bool nonfinite = !isfinite(gam);
  const bool conv = gam <= tol2;
  const bool hit = done_its >= maxit;
  const bool breakdown = !first && !nonfinite && !conv && !hit && (!(pw > 0.0) || !isfinite(pw));
  const bool stop = nonfinite || conv || hit || breakdown;
  if (lead && threadIdx.x == 0) {
    cg->gamma[done_its & 1] = gam;   // s^T s after done_its updates, as the two-launch step
    cg->gcur = gam;
    if (nonfinite) cg->flag = 2;
    if (breakdown) cg->flag = isfinite(pw) ? 1 : 2;
    if (stop) {
      cg->its = done_its;
      cg->done = 1;
    }
  }
  if (stop) return;
  __syncthreads();
  // c_j = G^{-1} t + beta c_{j-1}
  __shared__ T cs[NJ_MAX];
  __shared__ double cd[NJ_MAX];
  {
    const int j = threadIdx.x;
    double cj = gram_row_apply<NJT, GPF>(Ginv, gr, nj, tv, 1.0);
    if (j < nj) {
      cj += be * cprev[j];
      cs[j] = (T)cj;
      cd[j] = cj;
      if (lead) {
        cv->c[par][j] = cj;
        if (!first) cv->e[j] += al * cprev[j];
      }
    }
  }
  __syncthreads();
  if (lead && threadIdx.x < WAVE) {
    const double* __restrict__ Gm = Gm0 + y * gstride;
    const int j = threadIdx.x;
    double v = 0.0;
    if (j < nj) {
      double gc = 0.0;
      for (int c = 0; c < nj; ++c) gc += Gm[j + c * nj] * cd[c];
      v = cd[j] * gc;
    }
    v = wave_sum(v);
    if (j == 0) {
      cg->cGc2[par] = v;
      cg->its2[par] = first ? 0 : done_its + 1;
      cg->its = first ? 0 : done_its + 1;
      cg->alpha = al;
      cg->beta = be;
    }
  }

  // ---- the planes
  constexpr int RV = RS + (IMM ? 0 : 2 * NJT);
  T acc[RV];
#pragma unroll
  for (int r = 0; r < RV; ++r) acc[r] = T(0);
  __shared__ T imm[IMM ? (OP_BS / WAVE) * 2 * NJT : 1];
  const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
  if (IMM) {
    for (int r = threadIdx.x; r < (OP_BS / WAVE) * 2 * NJT; r += OP_BS) imm[r] = T(0);
    __syncthreads();
  }
  auto vadd = [&] __attribute__((always_inline)) (int r, T v) {
    if (IMM) {
      v = wave_sum(v);
      if (lane == 0) imm[wid * 2 * NJT + r] += v;
    } else {
      acc[RS + r] += v;
    }
  };
  // q_j from raw values: q_0 = q (first), else s - alpha w + beta q
  const T ks = first ? T(0) : T(1), kw = (T)(-al), kq = first ? T(1) : (T)be;
  auto qj = [&] __attribute__((always_inline)) (T s_, T w_, T q_) { return ks * s_ + kw * w_ + kq * q_; };
  const T cx = (T)S.cx, cy = (T)S.cy, cz = (T)S.cz;
  const T a_ = (T)al;
  const T m = act ? T(1) : T(0);
  T xm[NP], xc[NP];
#pragma unroll
  for (int u = 0; u < NP; ++u) {
    xm[u] = qj(xm3.s[u], xm3.w[u], xm3.q[u]);
    xc[u] = qj(P.own.s[u], P.own.w[u], P.own.q[u]);
  }
  for (int z = z0; walk && z < z1; ++z, i += nxy) {
    T xp[NP], yd[NP], yu[NP], sj[NP];
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      xp[u] = P.mxp * qj(P.xp.s[u], P.xp.w[u], P.xp.q[u]);
      yd[u] = qj(P.yd.s[u], P.yd.w[u], P.yd.q[u]);
      yu[u] = qj(P.yu.s[u], P.yu.w[u], P.yu.q[u]);
      sj[u] = P.own.s[u] - a_ * P.own.w[u];
    }
    const T xl = qj(P.xl.s, P.xl.w, P.xl.q), xr = qj(P.xr.s, P.xr.w, P.xr.q);
    // the update of step j-1 at this thread's nodes
    if (act) {
      if (!first) {
        T gn[NP];
#pragma unroll
        for (int u = 0; u < NP; ++u) gn[u] = P.gv[u] + a_ * P.own.q[u];
        stn(g, i, gn);
        stn(sw_, i, sj);
        stn(qw_, i, xc);
      }
    }
    // (A q_j) at the NP nodes
    T av[NP], xq[NP];
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const T left = u == 0 ? xl : xc[u - 1];
      const T right = u == NP - 1 ? xr : xc[u + 1];
      T v = P.d[u] * xc[u];
      if (!VAR) {
        v -= cx * (left + right) + cy * (yd[u] + yu[u]) + cz * (xm[u] + xp[u]);
      } else {
        const T fl = u == 0 ? P.fxl : P.fx[u - 1];
        v -= fl * left + P.fx[u] * right;
        v -= P.fyd[u] * yd[u] + P.fyu[u] * yu[u];
        if (S.dim == 3) v -= fm[u] * xm[u] + P.fp[u] * xp[u];
      }
      av[u] = m * v;
      xq[u] = m * xc[u];
      sj[u] = m * sj[u];
    }
    // pass 1 over the rows of AU: AU c_j, (AU)^T s_j
    T au[NP], wv[NP];
    zero(au);
    T keep[KEEP ? NJT : 1][NP];
#pragma unroll
    for (int c = 0; c < NJT; ++c)
      if (c < nj) {
        T a[NP];
        if (PRE) {
#pragma unroll
          for (int u = 0; u < NP; ++u) a[u] = P.a[PRE ? c : 0][u];
        } else if (act) {
          ldv(col_of(AW, AWs, ns, c, ld), i, a);
        } else {
          zero(a);
        }
        if (KEEP) {
#pragma unroll
          for (int u = 0; u < NP; ++u) keep[KEEP ? c : 0][u] = a[u];
        }
        T t = T(0);
#pragma unroll
        for (int u = 0; u < NP; ++u) {
          au[u] += a[u] * cs[c];
          t += a[u] * sj[u];
        }
        vadd(NJT + c, t);
      }
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      wv[u] = av[u] - au[u];
      acc[0] += xq[u] * wv[u];
      acc[1] += xq[u] * au[u];
      acc[2] += sj[u] * wv[u];
      acc[3] += wv[u] * wv[u];
      acc[4] += sj[u] * sj[u];
    }
    if (act) stn(ww_, i, wv);
    // pass 2: (AU)^T w_j
#pragma unroll
    for (int c = 0; c < NJT; ++c)
      if (c < nj) {
        T a[NP];
        if (PRE) {
#pragma unroll
          for (int u = 0; u < NP; ++u) a[u] = P.a[PRE ? c : 0][u];
        } else if (KEEP) {
#pragma unroll
          for (int u = 0; u < NP; ++u) a[u] = keep[KEEP ? c : 0][u];
        } else if (act) {
          ldv(col_of(AW, AWs, ns, c, ld), i, a);
        } else {
          zero(a);
        }
        T t = T(0);
#pragma unroll
        for (int u = 0; u < NP; ++u) t += a[u] * wv[u];
        vadd(c, t);
      }
    // next plane
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      xm[u] = xc[u];
      xc[u] = xp[u];
      if (VAR) fm[u] = P.fp[u];
    }
    if (z + 1 < z1) load_plane(i + nxy, z + 1);
  }
  T* __restrict__ po = po0 + y * postride + par * pohalf;
  const int P1 = ntiles;
  const int bid = bk.t;
  if (!IMM) {
    write_partials_t<RV, OP_BS>(acc, po, bid, P1);
  } else {
    T a5[RS] = {acc[0], acc[1], acc[2], acc[3], acc[4]};
    write_partials_t<RS, OP_BS>(a5, po, bid, P1);
    __syncthreads();
    for (int r = threadIdx.x; r < 2 * NJT; r += OP_BS) {
      T t = T(0);
#pragma unroll
      for (int v = 0; v < OP_BS / WAVE; ++v) t += imm[v * 2 * NJT + r];
      po[(size_t)(RS + r) * P1 + bid] = t;
    }
  }
}

// Rows per thread of the update (five vectors, no U rows): 4, or 2 in the narrow variant.
template <int NARROW>
struct UpdRows {
  static constexpr int value = NARROW ? 2 : 4;
};

// The update of member y = blockIdx.y (see the file comment).  Block b also reduces the
// operator step's vector totals r = b, b + P, ... < 2 nj into cv (tw first, then ts).
// Each access moves V consecutive values (V = 16 / sizeof(T) where the vectors are
// aligned, else 1): the kernel is bound by the number of load and store instructions, not
// by their bytes.  Values past n are read as 0 (the vectors' storage runs to a multiple of
// 64 elements) and not written.
template <typename T, int RPT, int V>
__global__ __launch_bounds__(CG_BS) void k_dcg_update(T* __restrict__ q0, const T* __restrict__ w0,
                                                       T* __restrict__ g0, T* __restrict__ s0,
                                                       int64_t vstride, int64_t n, int njt,
                                                       CGState* cgs, CGVec* cvs,
                                                       const T* __restrict__ po0, int P1,
                                                       int64_t postride, T* __restrict__ pu0,
                                                       int64_t pustride) {
  const int y = blockIdx.y;
  CGState* cg = cgs + y;
  if (cg->done) return;
  CGVec* cv = cvs + y;
  T* __restrict__ q = q0 + y * vstride;
  const T* __restrict__ w = w0 + y * vstride;
  T* __restrict__ g = g0 + y * vstride;
  T* __restrict__ s = s0 + y * vstride;
  const T* __restrict__ po = po0 + y * postride;
  const int nj = cg->nj;
  const int k = cg->kcur;
  const double gam = cg->gcur, cGc = cg->cGc;
  constexpr int R = RPT;
  constexpr int64_t CH = (int64_t)CG_BS * R;   // accesses (of V values) per block and pass
  const int64_t nv = (n + V - 1) / V;
  int64_t base = (int64_t)blockIdx.x * CH + threadIdx.x;
  T qv[R][V], wv[R][V], gv[R][V], sv[R][V];
  auto load = [&](int64_t b0) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int64_t vi = b0 + (int64_t)u * CG_BS, i = vi * V;
      if (vi < nv) {
        ldn(q, i, qv[u]);
        ldn(w, i, wv[u]);
        ldn(g, i, gv[u]);
        ldn(s, i, sv[u]);
#pragma unroll
        for (int e = 0; e < V; ++e)
          if (i + e >= n) qv[u][e] = wv[u][e] = gv[u][e] = sv[u][e] = T(0);
      } else {
#pragma unroll
        for (int e = 0; e < V; ++e) qv[u][e] = wv[u][e] = gv[u][e] = sv[u][e] = T(0);
      }
    }
  };
  load(base);
  // wave w sums the operator step's scalar w (one of q^T w, q^T (AU c), s^T w, w^T w) and,
  // in the same loop, the vector total this block owns for that wave (value b + P w, if
  // any, of the 2 nj totals), so that both sets of loads are in flight together
  __shared__ T tot[4];
  {
    const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
    const int v = blockIdx.x + gridDim.x * wid;
    const bool own = v < 2 * nj;
    const int r = v < nj ? 4 + v : 4 + njt + (v - nj);
    T a = T(0), o = T(0);
#pragma unroll 4
    for (int b = lane; b < P1; b += WAVE) {
      a += po[(size_t)wid * P1 + b];
      if (own) o += po[(size_t)r * P1 + b];
    }
    a = wave_sum(a);
    if (lane == 0) tot[wid] = a;
    if (own) {
      o = wave_sum(o);
      if (lane == 0) {
        if (v < nj) cv->tw[v] = (double)o;
        else cv->ts[v - nj] = (double)o;
      }
    }
    // totals past the first P * 4 (when 2 nj exceeds the update's waves)
    for (int u = v + gridDim.x * (CG_BS / WAVE); u < 2 * nj; u += gridDim.x * (CG_BS / WAVE)) {
      const int ru = u < nj ? 4 + u : 4 + njt + (u - nj);
      T e = T(0);
      for (int b = lane; b < P1; b += WAVE) e += po[(size_t)ru * P1 + b];
      e = wave_sum(e);
      if (lane == 0) {
        if (u < nj) cv->tw[u] = (double)e;
        else cv->ts[u - nj] = (double)e;
      }
    }
  }
  __syncthreads();
  const double qw = tot[0], qau = tot[1], sw = tot[2], ww = tot[3];
  const double pw = qw - qau + cGc;
  if (!(pw > 0.0) || !isfinite(pw)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      cg->flag = isfinite(pw) ? 1 : 2;
      cg->done = 1;
    }
    return;
  }
  const double al = gam / pw;
  double gnext = gam - 2.0 * al * sw + al * al * ww;
  if (!(gnext > 0.0)) gnext = 0.0;
  const double be = gnext / gam;
  if (blockIdx.x == 0) {
    if (threadIdx.x < nj) cv->e[threadIdx.x] += al * cv->c[k & 1][threadIdx.x];
    if (threadIdx.x == 0) {
      cg->pw = pw;
      cg->alpha = al;
      cg->beta = be;
      cg->gamma[(k + 1) & 1] = gnext;
      cg->its = k + 1;
    }
  }
  const T a = (T)al, b = (T)be;
  T acc[1] = {T(0)};
  for (;;) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int64_t i = (base + (int64_t)u * CG_BS) * V;
      T sn[V], gn[V], qn[V];
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const T si = sv[u][e] - a * wv[u][e];   // 0 past the end (sv = wv = 0 there)
        sn[e] = si;
        gn[e] = gv[u][e] + a * qv[u][e];
        qn[e] = si + b * qv[u][e];
        acc[0] += si * si;
      }
      if (i + V <= n) {
        stn(s, i, sn);
        stn(g, i, gn);
        stn(q, i, qn);
      } else if (i < n) {
#pragma unroll
        for (int e = 0; e < V; ++e)
          if (i + e < n) {
            s[i + e] = sn[e];
            g[i + e] = gn[e];
            q[i + e] = qn[e];
          }
      }
    }
    base += (int64_t)gridDim.x * CH;
    if (base - threadIdx.x >= nv) break;
    load(base);
  }
  write_partials_t<1, CG_BS>(acc, pu0 + y * pustride, blockIdx.x, gridDim.x);
}

// g -= U e (member y; see step_block): the U part of the split correction.  V values per
// access (16-byte accesses where the launcher finds n and the layout aligned for them).
template <typename T, int NJT, int V = 1>
__global__ __launch_bounds__(CG_BS) void k_dcg_finish(const T* __restrict__ W0, Slots sl,
                                                       int64_t n,
                                                       T* __restrict__ g0, int64_t vstride,
                                                       const CGState* cgs, const CGVec* cvs,
                                                       int P, int nb) {
  const StepBlock bk = step_block(P, P, nb);
  if (!bk.valid) return;
  const int y = bk.y;
  const CGState* cg = cgs + y;
  const int nj = cg->nj;
  if (nj == 0) return;
  __shared__ T es[NJ_MAX];
  if (threadIdx.x < nj) es[threadIdx.x] = (T)cvs[y].e[threadIdx.x];
  __syncthreads();
  const T* __restrict__ W = W0 + y * sl.wstride;
  const T* __restrict__ Ws = W0 + sl.soff;
  T* __restrict__ g = g0 + y * vstride;
  // with V > 1, n is a multiple of V
  for (int64_t i = ((int64_t)bk.t * CG_BS + threadIdx.x) * V; i < n;
       i += (int64_t)P * CG_BS * V) {
    T v[V];
    ldn(g, i, v);
#pragma unroll
    for (int c = 0; c < NJT; ++c)
      if (c < nj) {
        T w[V];
        ldn(col_of(W, Ws, sl.ns, c, sl.ld), i, w);
        const T ec = es[c];
#pragma unroll
        for (int e = 0; e < V; ++e) v[e] -= w[e] * ec;
      }
    stn(g, i, v);
  }
}

}  // namespace

int njt_of(int nj) { return nj <= 8 ? 8 : nj <= 16 ? 16 : nj <= 32 ? 32 : 64; }

int dcg_blocks(int64_t n) {
  const int b = ceil_div(n, 512);
  return b < CG_GRID ? (b < 1 ? 1 : b) : CG_GRID;
}

void launch_cg_setup(CGState* cg, CGVec* cv, const CgSetup& su, int nb, hipStream_t st) {
  if (nb < 1 || nb > G_MAX) throw Error(ROM_EINVAL, "cg_setup: batch size out of range");
  ROM_LAUNCH(k_cg_setup, dim3(1), dim3(256), 0, st, cg, cv, su, nb);
  ROM_CHECK_LAUNCH();
}

template <typename T>
void launch_dcg_start(const T* W, const T* AW, const Slots& sl, int64_t n, int njmax,
                      const double* Ginv, int64_t gstride, const double* r, int64_t rstride, T* g,
                      T* s, T* q, int64_t vstride, const CGState* cg, T* ps, int64_t psstride,
                      int nb, int P, hipStream_t st) {
  if (nb < 1 || nb > G_MAX || P < 1) throw Error(ROM_EINVAL, "dcg_start: bad batch or grid");
  const dim3 grid(ceil_div(P, NXCD) * NXCD * nb);
  // 16-byte accesses where n, the strides and every array allow them (the widths whose
  // rows are preloaded)
  constexpr int V = 16 / sizeof(T);
  const uintptr_t al = (uintptr_t)W | (uintptr_t)AW | (uintptr_t)(W + sl.soff) |
                       (uintptr_t)(AW + sl.soff) | (uintptr_t)g | (uintptr_t)s | (uintptr_t)q |
                       (uintptr_t)r;
  const bool vec = n % V == 0 && sl.ld % V == 0 && sl.wstride % V == 0 && vstride % V == 0 &&
                   rstride % 2 == 0 && (al & 15) == 0;
#define C(J)                                                                                  \
  case J:                                                                                     \
    if (vec && StartRows<T, J>::value > 0)                                                    \
      ROM_LAUNCH((k_dcg_start<T, J, StartRows<T, J>::value, (StartRows<T, J>::value > 0 ? V : 1)>), \
                 grid, dim3(START_BS), 0, st, W, AW, sl, n, Ginv, gstride, r, rstride, g, s, q,  \
                 vstride, cg, ps, psstride, P, nb);                                             \
    else                                                                                      \
      ROM_LAUNCH((k_dcg_start<T, J>), grid, dim3(START_BS), 0, st, W, AW, sl, n, Ginv, gstride, \
                 r, rstride, g, s, q, vstride, cg, ps, psstride, P, nb);                        \
    break;
  switch (njt_of(njmax)) {
    C(8) C(16) C(32) C(64)
  }
#undef C
  ROM_CHECK_LAUNCH();
}

template <typename T>
void launch_dcg_op(const Stencil& S, const StencilShape& sh, const T* diag, const T* q,
                   const T* s, T* w, int64_t vstride, const T* AW, const Slots& sl,
                   int njmax, const double* Ginv, const double* Gm, int64_t gstride, CGState* cg,
                   CGVec* cv, const T* ps, int Ps, int64_t psstride, const T* pu, int Pu,
                   int64_t pustride, T* po, int64_t postride, int nb, hipStream_t st) {
  const int gx = sh.grid.x, ntiles = sh.blocks;
  if (nb < 1 || nb > G_MAX || ntiles != gx * (int)sh.grid.y)
    throw Error(ROM_EINVAL, "dcg_op: launch shape and batch size do not match");
  // the kernel addresses a vector's nodes by 32-bit byte offsets
  if ((uint64_t)S.n * sizeof(T) > 0xffffffffull)
    throw Error(ROM_EINVAL, "dcg_op: grid too large for 32-bit node offsets");
  const dim3 grid(ceil_div(ntiles, NXCD) * NXCD * nb);
#define OPL(VAR, NP, J)                                                                       \
  ROM_LAUNCH((k_dcg_op<T, VAR, NP, J>), grid, dim3(OP_BS), 0, st, S, diag, q, s, w, vstride,  \
             AW, sl, Ginv, Gm, gstride, sh.zc, gx, ntiles, nb, cg, cv, ps, Ps, psstride, pu,   \
             Pu, pustride, po, postride)
#define OPJ(VAR, NP)                      \
  switch (njt_of(njmax)) {                \
    case 8: OPL(VAR, NP, 8); break;       \
    case 16: OPL(VAR, NP, 16); break;     \
    case 32: OPL(VAR, NP, 32); break;     \
    default: OPL(VAR, NP, 64); break;     \
  }
#define OPLY(VAR, J)                                                                          \
  ROM_LAUNCH((k_dcg_op<T, VAR, 4, J, true>), grid, dim3(OP_BS), 0, st, S, diag, q, s, w,      \
             vstride, AW, sl, Ginv, Gm, gstride, sh.zc, gx, ntiles, nb, cg, cv, ps, Ps,       \
             psstride, pu, Pu, pustride, po, postride)
#define OPJY(VAR)                         \
  switch (njt_of(njmax)) {                \
    case 8: OPLY(VAR, 8); break;          \
    case 16: OPLY(VAR, 16); break;        \
    case 32: OPLY(VAR, 32); break;        \
    default: OPLY(VAR, 64); break;        \
  }
  if (sh.quads) {
    // FP32 only (16-byte loads of four nodes); the LDS y-neighbours where a block's
    // positions are whole rows and every block is full
    if constexpr (sizeof(T) == 4) {
      const int rowp = S.nx / 4;
      if (OP_BS % rowp == 0 && ((int64_t)rowp * S.ny) % OP_BS == 0) {
        if (S.var) { OPJY(true) } else { OPJY(false) }
      } else {
        if (S.var) { OPJ(true, 4) } else { OPJ(false, 4) }
      }
    } else {
      throw Error(ROM_EINVAL, "dcg_op: the four-node walk is FP32 only");
    }
  } else if (sh.pairs) {
    if (S.var) { OPJ(true, 2) } else { OPJ(false, 2) }
  } else {
    if (S.var) { OPJ(true, 1) } else { OPJ(false, 1) }
  }
#undef OPJY
#undef OPLY
#undef OPJ
#undef OPL
  ROM_CHECK_LAUNCH();
}

template <typename T>
void launch_dcg_iter(const Stencil& S, const StencilShape& sh, const T* diag, T* s, T* q, T* w,
                     int64_t pstride, int64_t vstride, T* g, const T* AW, const Slots& sl,
                     int njmax, const double* Ginv, const double* Gm,
                     int64_t gstride, CGState* cg, CGVec* cv, const T* ps, int Ps,
                     int64_t psstride, T* po, int64_t postride, int64_t pohalf, int Pprev,
                     int par, int first, int nb, hipStream_t st) {
  if (par != 0 && par != 1) throw Error(ROM_EINVAL, "dcg_iter: parity must be 0 or 1");
  if (sh.quads) throw Error(ROM_EINVAL, "dcg_iter: no four-node walk for the one-launch step");
  if (first && par != 0) throw Error(ROM_EINVAL, "dcg_iter: the first step has parity 0");
  if (sh.pairs) {
    // the two-node walk reads and writes s, q, w and g two values at a time
    const uintptr_t m = 2 * sizeof(T) - 1;
    if ((((uintptr_t)s | (uintptr_t)q | (uintptr_t)w | (uintptr_t)g) & m) || pstride % 2 ||
        vstride % 2)
      throw Error(ROM_EINVAL, "dcg_iter: vectors not aligned for the two-node walk");
  }
  const int gx = sh.grid.x, ntiles = sh.blocks;
  if (nb < 1 || nb > G_MAX || ntiles != gx * (int)sh.grid.y)
    throw Error(ROM_EINVAL, "dcg_iter: launch shape and batch size do not match");
  const dim3 grid(ceil_div(ntiles, NXCD) * NXCD * nb);
#define ITL(VAR, NP, J)                                                                        \
  ROM_LAUNCH((k_dcg_iter<T, VAR, NP, J>), grid, dim3(OP_BS), 0, st, S, diag, s, q, w, pstride,  \
             vstride, g, AW, sl, Ginv, Gm, gstride, sh.zc, gx, ntiles, nb, cg, cv, ps, Ps,      \
             psstride, po, postride, pohalf, Pprev, par, first)
#define ITJ(VAR, NP)                      \
  switch (njt_of(njmax)) {                \
    case 8: ITL(VAR, NP, 8); break;       \
    case 16: ITL(VAR, NP, 16); break;     \
    case 32: ITL(VAR, NP, 32); break;     \
    default: ITL(VAR, NP, 64); break;     \
  }
  if (sh.pairs) {
    if (S.var) { ITJ(true, 2) } else { ITJ(false, 2) }
  } else {
    if (S.var) { ITJ(true, 1) } else { ITJ(false, 1) }
  }
#undef ITJ
#undef ITL
  ROM_CHECK_LAUNCH();
}

template <typename T>
void launch_dcg_update(T* q, const T* w, T* g, T* s, int64_t vstride, int64_t n, int njmax,
                       CGState* cg, CGVec* cv, const T* po, int P1, int64_t postride, T* pu,
                       int64_t pustride, int nb, int P, hipStream_t st, int narrow) {
  const dim3 grid(P, nb);
  const int njt = njt_of(njmax);
  // 16-byte accesses where every vector is aligned for them and long enough that the
  // instruction count, not the latency of fewer threads, bounds the kernel (at 64^3 the
  // one-value form measured faster, at 128^3 the 16-byte form)
  constexpr int V = 16 / sizeof(T);
  const bool vec = n >= (int64_t(1) << 20) &&
                   !((((uintptr_t)q | (uintptr_t)w | (uintptr_t)g | (uintptr_t)s) & 15) ||
                     vstride % V);
#define UPL(RR, VV)                                                                         \
  ROM_LAUNCH((k_dcg_update<T, RR, VV>), grid, dim3(CG_BS), 0, st, q, w, g, s, vstride, n, njt, \
             cg, cv, po, P1, postride, pu, pustride)
  if (vec) {
    if (narrow) UPL(UpdRows<1>::value, V); else UPL(UpdRows<0>::value, V);
  } else {
    if (narrow) UPL(UpdRows<1>::value, 1); else UPL(UpdRows<0>::value, 1);
  }
#undef UPL
  ROM_CHECK_LAUNCH();
}

template <typename T>
void launch_dcg_finish(const T* W, const Slots& sl, int64_t n, int njmax, T* g,
                       int64_t vstride, const CGState* cg, const CGVec* cv, int nb,
                       hipStream_t st) {
  if (njmax <= 0) return;
  if (nb < 1 || nb > G_MAX) throw Error(ROM_EINVAL, "dcg_finish: bad batch");
  const int P = dcg_blocks(n);
  const dim3 grid(ceil_div(P, NXCD) * NXCD * nb);
  constexpr int V = 16 / sizeof(T);
  const bool vec = n % V == 0 && sl.ld % V == 0 && sl.wstride % V == 0 && vstride % V == 0 &&
                   (((uintptr_t)W | (uintptr_t)(W + sl.soff) | (uintptr_t)g) & 15) == 0;
#define C(J)                                                                                  \
  case J:                                                                                     \
    if (vec)                                                                                  \
      ROM_LAUNCH((k_dcg_finish<T, J, V>), grid, dim3(CG_BS), 0, st, W, sl, n, g, vstride, cg, cv, \
                 P, nb);                                                                      \
    else                                                                                      \
      ROM_LAUNCH((k_dcg_finish<T, J>), grid, dim3(CG_BS), 0, st, W, sl, n, g, vstride, cg, cv, P, \
                 nb);                                                                         \
    break;
  switch (njt_of(njmax)) {
    C(8) C(16) C(32) C(64)
  }
#undef C
  ROM_CHECK_LAUNCH();
}

#define INSTANTIATE(T)                                                                          \
  template void launch_dcg_start<T>(const T*, const T*, const Slots&, int64_t, int,              \
                                    const double*, int64_t, const double*, int64_t, T*, T*, T*,  \
                                    int64_t, const CGState*, T*, int64_t, int, int,              \
                                    hipStream_t);                                                \
  template void launch_dcg_op<T>(const Stencil&, const StencilShape&, const T*, const T*,        \
                                 const T*, T*, int64_t, const T*, const Slots&, int,             \
                                 const double*, const double*, int64_t, CGState*, CGVec*,        \
                                 const T*, int, int64_t, const T*, int, int64_t, T*, int64_t,    \
                                 int, hipStream_t);                                              \
  template void launch_dcg_iter<T>(const Stencil&, const StencilShape&, const T*, T*, T*, T*,     \
                                   int64_t, int64_t, T*, const T*, const Slots&, int,            \
                                   const double*, const double*, int64_t, CGState*, CGVec*,      \
                                   const T*, int, int64_t, T*, int64_t, int64_t, int, int, int,  \
                                   int, hipStream_t);                                            \
  template void launch_dcg_update<T>(T*, const T*, T*, T*, int64_t, int64_t, int, CGState*,      \
                                     CGVec*, const T*, int, int64_t, T*, int64_t, int, int,      \
                                     hipStream_t, int);                                          \
  template void launch_dcg_finish<T>(const T*, const Slots&, int64_t, int, T*, int64_t,          \
                                     const CGState*, const CGVec*, int, hipStream_t);
INSTANTIATE(double)
INSTANTIATE(float)
#undef INSTANTIATE

}  // namespace rom
