// Tall-skinny products against the basis, vector helpers, and the inverse Cholesky
// factor of the outer Gram matrix Q^T A(p) Q.
#include <algorithm>

#include "kernels.h"

namespace rom {

namespace {

constexpr int BS = 256;
constexpr int GT_COLS = 32;   // columns per block of the transposed product

int reduce_grid(int64_t n) {
  int b = ceil_div(n, BS);
  return b < 1024 ? (b < 1 ? 1 : b) : 1024;
}

// Transposed product, lanes over rows, waves over columns; one block covers
// 64*CPL rows x gcols columns (GT_COLS, or one column per wave when that would leave the
// chip mostly idle).  When several row chunks exist, k_gemvt_reduce sums the chunk
// partials of each output in chunk order.
//
// Q4: a lane takes four consecutive rows per 256-row slice of its chunk (two 16-byte loads
// per column instead of four 8-byte ones); needs M and V 16-byte aligned at even leading
// dimensions.  The chunk and the partials are the same as without it.
template <int CPL, int NV, bool Q4 = false>
__global__ __launch_bounds__(BS) void k_gemvt(const double* __restrict__ M, int64_t ld,
                                               int64_t rows, int cols,
                                               const double* __restrict__ V, int64_t vstride,
                                               double* __restrict__ out,
                                               double* __restrict__ partials, Skip skip,
                                               int gcols) {
  if (skip.on()) return;
  const int64_t r0 = (int64_t)blockIdx.x * (64 * CPL);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double vr[NV][CPL];
  // four rows of a slice: two 16-byte loads when all four exist, else guarded scalars
  auto quad = [rows](const double* __restrict__ p, int64_t base, double (&o)[4]) {
    if (base + 3 < rows) {
      const double2 a = *reinterpret_cast<const double2*>(p + base);
      const double2 b = *reinterpret_cast<const double2*>(p + base + 2);
      o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) o[e] = base + e < rows ? p[base + e] : 0.0;
    }
  };
  if (Q4) {
#pragma unroll
    for (int qq = 0; qq < CPL / 4; ++qq) {
      const int64_t base = r0 + 256 * qq + 4 * lane;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double o[4];
        quad(V + v * vstride, base, o);
#pragma unroll
        for (int e = 0; e < 4; ++e) vr[v][4 * qq + e] = o[e];
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int64_t r = r0 + lane + 64 * q;
#pragma unroll
      for (int v = 0; v < NV; ++v) vr[v][q] = r < rows ? V[r + v * vstride] : 0.0;
    }
  }
  const int c0 = blockIdx.y * gcols;
  const bool single = gridDim.x == 1;
  if (NV == 1) {
    // a row chunk whose vector entries are all zero contributes nothing: skip its reads of M
    bool nz = false;
#pragma unroll
    for (int q = 0; q < CPL; ++q) nz |= vr[0][q] != 0.0;
    if (!__syncthreads_or(nz)) {
      for (int cc = wid; cc < gcols; cc += BS / 64) {
        const int c = c0 + cc;
        if (c < cols && lane == 0) {
          if (single)
            out[c] = 0.0;
          else
            partials[(int64_t)c * gridDim.x + blockIdx.x] = 0.0;
        }
      }
      return;
    }
  }
  for (int cc = wid; cc < gcols; cc += BS / 64) {
    const int c = c0 + cc;
    if (c >= cols) break;
    const double* col = M + (int64_t)c * ld;
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    if (Q4) {
#pragma unroll
      for (int qq = 0; qq < CPL / 4; ++qq) {
        double o[4];
        quad(col, r0 + 256 * qq + 4 * lane, o);
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int v = 0; v < NV; ++v) acc[v] += o[e] * vr[v][4 * qq + e];
      }
    } else {
#pragma unroll
      for (int q = 0; q < CPL; ++q) {
        const int64_t r = r0 + lane + 64 * q;
        const double mv = r < rows ? col[r] : 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] += mv * vr[v][q];
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double s = wave_sum(acc[v]);
      if (lane == 0) {
        if (single)
          out[v * cols + c] = s;
        else
          partials[((int64_t)v * cols + c) * gridDim.x + blockIdx.x] = s;
      }
    }
  }
}

// out[e] = sum over chunks b of partials[e * nch + b]: one wave per output, fixed order.
__global__ void k_gemvt_reduce(const double* __restrict__ partials, int nch, int ne,
                               double* __restrict__ out, Skip skip) {
  if (skip.on()) return;
  const int e = blockIdx.x * (BS / WAVE) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (e >= ne) return;
  const double* p = partials + (int64_t)e * nch;
  double a = 0.0;
  for (int b = lane; b < nch; b += WAVE) a += p[b];
  a = wave_sum(a);
  if (lane == 0) out[e] = a;
}

int gemvt_cpl(int cols) { return cols > 64 ? 16 : 4; }

template <bool NRM>
__global__ __launch_bounds__(BS) void k_gemvn(const double* __restrict__ M, int64_t ld,
                                               int64_t rows, int cols,
                                               const double* __restrict__ coef, double alpha,
                                               const double* __restrict__ in, double beta,
                                               double* __restrict__ out,
                                               double* partials, Skip skip) {
  if (skip.on()) return;
  extern __shared__ double cs[];
  for (int c = threadIdx.x; c < cols; c += BS) cs[c] = coef[c];
  __syncthreads();
  double nv[1] = {0.0};
  for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < rows;
       r += (int64_t)gridDim.x * BS) {
    const double* p = M + r;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int c = 0;
    for (; c + 8 <= cols; c += 8) {
      a0 += p[(int64_t)(c + 0) * ld] * cs[c + 0];
      a1 += p[(int64_t)(c + 1) * ld] * cs[c + 1];
      a2 += p[(int64_t)(c + 2) * ld] * cs[c + 2];
      a3 += p[(int64_t)(c + 3) * ld] * cs[c + 3];
      a0 += p[(int64_t)(c + 4) * ld] * cs[c + 4];
      a1 += p[(int64_t)(c + 5) * ld] * cs[c + 5];
      a2 += p[(int64_t)(c + 6) * ld] * cs[c + 6];
      a3 += p[(int64_t)(c + 7) * ld] * cs[c + 7];
    }
    for (; c < cols; ++c) a0 += p[(int64_t)c * ld] * cs[c];
    const double acc = (a0 + a1) + (a2 + a3);
    const double o = beta * acc + (in ? alpha * in[r] : 0.0);
    out[r] = o;
    nv[0] += o * o;
  }
  if (NRM) write_partials<1, BS>(nv, partials, blockIdx.x);
}

// The same product with four consecutive rows per thread: two 16-byte loads per column,
// four columns per step, one block per CU at 64^3 (the loop is strided by the grid).
// Rows are read in groups of four up to round_up(rows, 4) <= ld (the column padding);
// `in` and `out` are touched only below `rows`.  Needs ld % 4 == 0 and M 16-byte aligned.
template <bool NRM>
__global__ __launch_bounds__(BS) void k_gemvn4(const double* __restrict__ M, int64_t ld,
                                                int64_t rows, int cols,
                                                const double* __restrict__ coef, double alpha,
                                                const double* __restrict__ in, double beta,
                                                double* __restrict__ out, double* partials,
                                                Skip skip) {
  if (skip.on()) return;
  extern __shared__ double cs[];
  for (int c = threadIdx.x; c < cols; c += BS) cs[c] = coef[c];
  __syncthreads();
  double nv[1] = {0.0};
  for (int64_t r0 = ((int64_t)blockIdx.x * BS + threadIdx.x) * 4; r0 < rows;
       r0 += (int64_t)gridDim.x * BS * 4) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const double* p = M + r0;
    int c = 0;
    for (; c + 4 <= cols; c += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double w = cs[c + u];
        const double2 v0 = *reinterpret_cast<const double2*>(p + (int64_t)(c + u) * ld);
        const double2 v1 = *reinterpret_cast<const double2*>(p + (int64_t)(c + u) * ld + 2);
        acc[0] += v0.x * w;
        acc[1] += v0.y * w;
        acc[2] += v1.x * w;
        acc[3] += v1.y * w;
      }
    }
    for (; c < cols; ++c) {
      const double w = cs[c];
      const double2 v0 = *reinterpret_cast<const double2*>(p + (int64_t)c * ld);
      const double2 v1 = *reinterpret_cast<const double2*>(p + (int64_t)c * ld + 2);
      acc[0] += v0.x * w;
      acc[1] += v0.y * w;
      acc[2] += v1.x * w;
      acc[3] += v1.y * w;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t r = r0 + q;
      if (r < rows) {
        const double o = beta * acc[q] + (in ? alpha * in[r] : 0.0);
        out[r] = o;
        nv[0] += o * o;
      }
    }
  }
  if (NRM) write_partials<1, BS>(nv, partials, blockIdx.x);
}

// One pass over the basis for three products (the Gram-Schmidt subtraction of one right-hand
// side fused with the next right-hand side's start): out0 = in - M t (and partial sums of
// out0^2), out1 = M c1, out2 = M c2.  Same row layout as k_gemvn4 (four consecutive rows
// per thread, two 16-byte loads per column); the three coefficient vectors sit in LDS.
__global__ __launch_bounds__(BS) void k_gemvn4x3(const double* __restrict__ M, int64_t ld,
                                                 int64_t rows, int cols,
                                                 const double* __restrict__ t,
                                                 const double* __restrict__ c1,
                                                 const double* __restrict__ c2,
                                                 const double* __restrict__ in,
                                                 double* __restrict__ out0,
                                                 double* __restrict__ out1,
                                                 double* __restrict__ out2, double* partials) {
  extern __shared__ double cs[];   // [t | c1 | c2]
  for (int c = threadIdx.x; c < cols; c += BS) {
    cs[c] = t[c];
    cs[cols + c] = c1[c];
    cs[2 * cols + c] = c2[c];
  }
  __syncthreads();
  double nv[1] = {0.0};
  for (int64_t r0 = ((int64_t)blockIdx.x * BS + threadIdx.x) * 4; r0 < rows;
       r0 += (int64_t)gridDim.x * BS * 4) {
    double a0[4] = {0.0, 0.0, 0.0, 0.0}, a1[4] = {0.0, 0.0, 0.0, 0.0},
           a2[4] = {0.0, 0.0, 0.0, 0.0};
    const double* p = M + r0;
    for (int c = 0; c < cols; ++c) {
      const double w0 = cs[c], w1 = cs[cols + c], w2 = cs[2 * cols + c];
      const double2 v0 = *reinterpret_cast<const double2*>(p + (int64_t)c * ld);
      const double2 v1 = *reinterpret_cast<const double2*>(p + (int64_t)c * ld + 2);
      const double v[4] = {v0.x, v0.y, v1.x, v1.y};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a0[q] += v[q] * w0;
        a1[q] += v[q] * w1;
        a2[q] += v[q] * w2;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t r = r0 + q;
      if (r < rows) {
        const double o = in[r] - a0[q];
        out0[r] = o;
        out1[r] = a1[q];
        out2[r] = a2[q];
        nv[0] += o * o;
      }
    }
  }
  write_partials<1, BS>(nv, partials, blockIdx.x);
}

// out = a + (u - w) * (cm[0] * s): the next right-hand side's start from the fused pass.
__global__ void k_fused_start(int64_t n, const double* __restrict__ a, const double* __restrict__ u,
                              const double* __restrict__ w, const double* __restrict__ cm,
                              double s, double* __restrict__ out) {
  const double f = cm[0] * s;
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
    out[i] = a[i] + (u[i] - w[i]) * f;
}

// Several coefficient vectors against one basis pass: each thread owns RPT rows and
// NV accumulators per row; coefficients are staged through LDS in chunks of CCH columns.
template <int NV, int RPT>
__global__ __launch_bounds__(BS) void k_gemvn_multi(const double* __restrict__ M, int64_t ld,
                                                     int64_t rows, int cols,
                                                     const double* __restrict__ coef,
                                                     int64_t ldc, int nv, double alpha,
                                                     const double* __restrict__ in, int64_t ldi,
                                                     double beta, double* __restrict__ out,
                                                     int64_t ldo) {
  constexpr int CCH = 128;
  __shared__ double cs[CCH][NV];
  const int64_t rbase = (int64_t)blockIdx.x * (BS * RPT) + threadIdx.x;
  double acc[RPT][NV];
#pragma unroll
  for (int q = 0; q < RPT; ++q)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[q][v] = 0.0;
  for (int c0 = 0; c0 < cols; c0 += CCH) {
    const int cn = min(CCH, cols - c0);
    __syncthreads();
    for (int e = threadIdx.x; e < CCH * NV; e += BS) {
      const int c = e % CCH, v = e / CCH;
      cs[c][v] = (c < cn && v < nv) ? coef[(int64_t)(c0 + c) + (int64_t)v * ldc] : 0.0;
    }
    __syncthreads();
    for (int c = 0; c < cn; ++c) {
      const double* col = M + (int64_t)(c0 + c) * ld;
      double mv[RPT];
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int64_t r = rbase + (int64_t)q * BS;
        mv[q] = r < rows ? col[r] : 0.0;
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double cv = cs[c][v];
#pragma unroll
        for (int q = 0; q < RPT; ++q) acc[q][v] += mv[q] * cv;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t r = rbase + (int64_t)q * BS;
    if (r >= rows) continue;
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (v < nv) {
        const double o = beta * acc[q][v] + (in ? alpha * in[r + (int64_t)v * ldi] : 0.0);
        out[r + (int64_t)v * ldo] = o;
      }
  }
}

__global__ void k_axpby_cols(int64_t n, double a, const double* __restrict__ x, int64_t ldx,
                             double b, const double* __restrict__ y, int64_t ldy,
                             double* __restrict__ out, int64_t ldo) {
  const int v = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    const double yi = y ? y[i + v * ldy] : 0.0;
    out[i + v * ldo] = a * x[i + v * ldx] + b * yi;
  }
}

__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b,
                        const double* __restrict__ y, double* __restrict__ out, int want,
                        double* partials) {
  double v[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    const double yi = y ? y[i] : 0.0;
    const double o = a * x[i] + b * yi;
    out[i] = o;
    v[0] += o * o;
    v[1] += yi * yi;
  }
  if (want) write_partials<2, BS>(v, partials, blockIdx.x);
}

// Copies nwords (<= 64 PUBLISH_WORDS) 8-byte words from device memory into coherent pinned
// host memory, then stores seq at *flag with system-scope release: one wave, so the
// release (which waits for this wave's own stores) also covers every word the wave wrote.
// All loads are issued before the stores.  The host spins on the flag instead of blocking
// on the stream.
constexpr int PUBLISH_WORDS = 32;
__global__ __launch_bounds__(64) void k_publish(const double* __restrict__ src,
                                                double* dst, int nwords, unsigned* flag,
                                                unsigned seq) {
  double v[PUBLISH_WORDS];
#pragma unroll
  for (int k = 0; k < PUBLISH_WORDS; ++k) {
    const int i = threadIdx.x + 64 * k;
    v[k] = i < nwords ? src[i] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < PUBLISH_WORDS; ++k) {
    const int i = threadIdx.x + 64 * k;
    if (i < nwords) __hip_atomic_store(dst + i, v[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  if (threadIdx.x == 0) __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void k_normalize(int64_t n, double* __restrict__ x, const double* nrm2) {
  const double s = 1.0 / sqrt(nrm2[0]);
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
    x[i] *= s;
}

// Mixed form: FP32 copies of FP64 columns (blockIdx.y = column).
__global__ void k_cast_cols_f32(int64_t n, const double* __restrict__ in, int64_t ld,
                                float* __restrict__ out) {
  const int64_t off = (int64_t)blockIdx.y * ld;
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
    out[off + i] = (float)in[off + i];
}

// out[i + c*ldo] = (Tout) in[i + c*ldi] for i < n, c = blockIdx.y.
template <typename Tin, typename Tout>
__global__ void k_convert_cols(int64_t n, const Tin* __restrict__ in, int64_t ldi,
                               Tout* __restrict__ out, int64_t ldo) {
  const Tin* a = in + (int64_t)blockIdx.y * ldi;
  Tout* b = out + (int64_t)blockIdx.y * ldo;
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
    b[i] = (Tout)a[i];
}

// out[:, c] = in[:, c] / sqrt(norm2[c]) (0 where norm2[c] == 0), c = blockIdx.y.
__global__ void k_scale_cols(int64_t n, const double* __restrict__ in, int64_t ldi,
                             const double* __restrict__ norm2, double* __restrict__ out,
                             int64_t ldo) {
  const double q = norm2[blockIdx.y];
  const double f = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
  const double* a = in + (int64_t)blockIdx.y * ldi;
  double* b = out + (int64_t)blockIdx.y * ldo;
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
    b[i] = f * a[i];
}

// Mixed form, end of an FP32 sweep: g += sigma d; x = x0 + g (FP64).
__global__ void k_refine_update(int64_t n, double sigma, const float* __restrict__ d,
                                double* __restrict__ g, const double* __restrict__ x0,
                                double* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    const double gi = g[i] + sigma * (double)d[i];
    g[i] = gi;
    x[i] = x0[i] + gi;
  }
}

// End of a refinement sweep for a batch: g[:, y] += coef.c[y] d[:, y] (d of type T),
// x[:, y] = x0[:, y] + g[:, y] (blockIdx.y = y).
template <typename T>
__global__ void k_refine_cols(int64_t n, Coefs coef, const T* __restrict__ d, int64_t ldd,
                              double* __restrict__ g, const double* __restrict__ x0, int64_t ld,
                              double* __restrict__ x, int64_t ldx) {
  const int y = blockIdx.y;
  const double c = coef.c[y];
  d += y * ldd;
  g += y * ld;
  x0 += y * ld;
  x += y * ldx;
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    const double gi = c != 0.0 ? g[i] + c * (double)d[i] : g[i];
    g[i] = gi;
    x[i] = x0[i] + gi;
  }
}

// Squared norms of s columns: partials[c * gridDim.x + b] (column c = blockIdx.y).
__global__ void k_colnorm2(int64_t n, const double* __restrict__ X, int64_t ld,
                           double* __restrict__ partials) {
  const double* x = X + (int64_t)blockIdx.y * ld;
  double v[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
    v[0] += x[i] * x[i];
  write_partials<1, BS>(v, partials + (int64_t)blockIdx.y * gridDim.x, blockIdx.x);
}

__global__ void k_sum_cols(const double* __restrict__ partials, int P, double* out) {
  __shared__ double tot[1];
  sum_partials<1, BS>(partials + (int64_t)blockIdx.x * P, P, tot);
  if (threadIdx.x == 0) out[blockIdx.x] = tot[0];
}

// Gram borders of k new basis columns m .. m+k-1 from B = [V^T A_* Q_new | V^T A_i Q_new]
// ((m + k) x 2k, ld ldb): column m + c of G_* and G_i gets rows 0 .. m + c, mirrored.
__global__ void k_border_fill_block(const double* __restrict__ B, int64_t ldb, int m, int k,
                                    double* Gs, double* Gi, int64_t ldg) {
  const int c = blockIdx.y;
  const int r = blockIdx.x * BS + threadIdx.x;
  const int col = m + c;
  if (r > col) return;
  const double a = B[r + (int64_t)c * ldb], b = B[r + (int64_t)(k + c) * ldb];
  Gs[r + (int64_t)col * ldg] = a;
  Gs[col + (int64_t)r * ldg] = a;
  Gi[r + (int64_t)col * ldg] = b;
  Gi[col + (int64_t)r * ldg] = b;
}

__global__ void k_pack_cols(int64_t n, ColPtrs src, int k, double* __restrict__ dst, int64_t ld) {
  const int c = blockIdx.y;
  const double* s = src.p[c];
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
    dst[i + c * ld] = s[i];
}

__global__ void k_gather_row(const double* __restrict__ M, int64_t ld, int cols, int64_t idx,
                             double scale, double* __restrict__ out) {
  const int c = blockIdx.x * BS + threadIdx.x;
  if (c < cols) out[c] = scale * M[idx + (int64_t)c * ld];
}

__global__ void k_gather_rows(const double* __restrict__ M, int64_t ld, int cols,
                              const int64_t* __restrict__ idx, const double* __restrict__ scale,
                              int nidx, double* __restrict__ out, int64_t ldo) {
  const int c = blockIdx.x * BS + threadIdx.x;
  const int r = blockIdx.y;
  if (c < cols && r < nidx) out[c + r * ldo] = scale[r] * M[idx[r] + (int64_t)c * ld];
}

// Border step finalisation (one block): delta^2 = d - l^T l, new row of Linv.
__global__ void k_linv_finish(double* Lc, double* Lr, int64_t ld, int k,
                              const double* __restrict__ gcol, const double* __restrict__ l,
                              const double* __restrict__ r, int* status, double* info) {
  __shared__ double sh[BS / WAVE];
  double s = 0.0;
  for (int i = threadIdx.x; i < k; i += BS) s += l[i] * l[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  double ll = 0.0;
#pragma unroll
  for (int w = 0; w < BS / WAVE; ++w) ll += sh[w];
  const double d2 = gcol[k] - ll;
  const bool bad = !(d2 > 0.0) || !isfinite(d2);
  const double inv = bad ? 0.0 : 1.0 / sqrt(d2);
  for (int c = threadIdx.x; c < k; c += BS) {
    const double v = -r[c] * inv;
    Lr[c + (int64_t)k * ld] = v;
    Lc[k + (int64_t)c * ld] = v;
  }
  if (threadIdx.x == 0) {
    Lr[k + (int64_t)k * ld] = inv;
    Lc[k + (int64_t)k * ld] = inv;
    if (bad && status[0] == 0) {
      status[0] = 1;
      // the first failing border: column, diagonal entry, squared norm of its projection
      if (info) {
        info[0] = k;
        info[1] = gcol[k];
        info[2] = ll;
      }
    }
  }
}

// Cholesky factor of a small SPD matrix in one workgroup (m <= 64), the inverse of the
// factor (Linv) and the inverse of the matrix (Ginv = Linv^T Linv).
__global__ __launch_bounds__(BS) void k_small_chol_inv(const double* __restrict__ G, int m,
                                                       double* __restrict__ Linv,
                                                       double* __restrict__ Ginv, int* status) {
  // A holds the symmetrised G.  Elimination in the square-root-free form: after step k the
  // lower column k holds sqrt(d_k) L[:, k] and A[k][k] the pivot d_k, so one barrier per
  // step suffices; the columns are scaled at the end.  A pivot that is not positive is
  // replaced by 1 and reported.  The strict upper triangle then holds R = L^{-1} before
  // its row scaling, transposed (R[i][j] at A[j][i], j < i); the diagonal of R is 1, and
  // Z = L^{-1} is R with row i divided by L[i][i].
  __shared__ double A[NJ_MAX][NJ_MAX + 1];
  __shared__ double rl[NJ_MAX];   // 1 / L[i][i]
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  for (int e = t; e < m * m; e += BS) {
    const int i = e % m, j = e / m;
    A[i][j] = i >= j ? 0.5 * (G[i + j * m] + G[j + i * m]) : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    const double d = A[k][k];
    const bool ok = d > 0.0 && isfinite(d);
    const double rd = ok ? 1.0 / d : 1.0;
    if (t == 0 && !ok) {
      A[k][k] = 1.0;   // every reader of this step takes the same replacement
      bad = 1;
    }
    const int w = m - k - 1;
    for (int e = t; e < w * (w + 1) / 2; e += BS) {
      // e -> (i, j) with k < j <= i < m, packed by rows of the trailing lower triangle
      int r = (int)((sqrtf(8.0f * e + 1.0f) - 1.0f) * 0.5f);
      if ((r + 1) * (r + 2) / 2 <= e) ++r;
      if (r * (r + 1) / 2 > e) --r;
      const int i = k + 1 + r, j = k + 1 + (e - r * (r + 1) / 2);
      A[i][j] -= A[i][k] * A[j][k] * rd;
    }
    __syncthreads();
  }
  for (int k = t; k < m; k += BS) {
    const double d = A[k][k];
    const double l = sqrt(d);
    rl[k] = 1.0 / l;
    A[k][k] = l;
  }
  __syncthreads();
  for (int e = t; e < m * m; e += BS) {
    const int i = e % m, k = e / m;
    if (i > k) A[i][k] *= rl[k];
  }
  __syncthreads();
  // R by right-looking substitution: after column c is final, R[i][j] -= L[i][c] Z[c][j]
  // for every i > c, j <= c, where Z[c][j] = R[c][j] / L[c][c].
  for (int c = 0; c + 1 < m; ++c) {
    const double sc = rl[c];
    const int rows = m - c - 1, cols = c + 1;
    for (int e = t; e < rows * cols; e += BS) {
      const int i = c + 1 + e % rows, j = e / rows;
      const double zcj = (j == c ? 1.0 : A[j][c]) * sc;
      A[j][i] -= A[i][c] * zcj;
    }
    __syncthreads();
  }
  // Z in place (row i scaled by 1 / L[i][i]); the diagonal is rl
  for (int e = t; e < m * m; e += BS) {
    const int i = e % m, j = e / m;
    if (j < i) A[j][i] *= rl[i];
  }
  __syncthreads();
  // Linv = Z (column-major), Ginv = Z^T Z: Ginv[i][j] = sum_{k >= max(i,j)} Z[k][i] Z[k][j]
  for (int e = t; e < m * m; e += BS) {
    const int i = e % m, j = e / m;
    Linv[e] = i > j ? A[j][i] : (i == j ? rl[i] : 0.0);
    const int k0 = i > j ? i : j;
    double s = (k0 == i ? rl[i] : A[i][k0]) * (k0 == j ? rl[j] : A[j][k0]);
    for (int k = k0 + 1; k < m; ++k) s += A[i][k] * A[j][k];
    Ginv[e] = s;
  }
  if (t == 0 && bad) status[0] = 1;
}

// C = alpha op(A) op(B) + beta D (all column-major; D may be NULL).  op(A) is M x K,
// op(B) is K x N.  64 x 64 output tiles, 256 threads with 4 x 4 outputs each.  With
// gridDim.z > 1 the K range is split in chunks of kc: block z sums its chunk into the
// M x N slice C + z ldc N (the caller passes alpha 1, beta 0 and sums the slices).
__global__ __launch_bounds__(BS) void k_gemm(int M, int N, int K, int kc, double alpha,
                                             const double* __restrict__ A, int64_t lda, int ta,
                                             const double* __restrict__ B, int64_t ldb, int tb,
                                             double beta, const double* __restrict__ D,
                                             int64_t ldd, double* __restrict__ C, int64_t ldc) {
  __shared__ double As[16][64 + 1];
  __shared__ double Bs[16][64 + 1];
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  const int kb = blockIdx.z * kc, ke = min(K, kb + kc);
  C += (int64_t)blockIdx.z * ldc * N;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int k0 = kb; k0 < ke; k0 += 16) {
    // stage op(A)[m0:m0+64, k0:k0+16] and op(B)[k0:k0+16, n0:n0+64]
    for (int e = threadIdx.x; e < 16 * 64; e += BS) {
      const int kk = e / 64, r = e % 64;
      const int k = k0 + kk, mi = m0 + r, ni = n0 + r;
      double a = 0.0, b = 0.0;
      if (k < ke && mi < M) a = ta ? A[k + (int64_t)mi * lda] : A[mi + (int64_t)k * lda];
      if (k < ke && ni < N) b = tb ? B[ni + (int64_t)k * ldb] : B[k + (int64_t)ni * ldb];
      As[kk][r] = a;
      Bs[kk][r] = b;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[kk][tx + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[kk][ty + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += av[i] * bv[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int mi = m0 + tx + 16 * i, ni = n0 + ty + 16 * j;
      if (mi < M && ni < N) {
        double v = alpha * acc[i][j];
        if (D) v += beta * D[mi + (int64_t)ni * ldd];
        C[mi + (int64_t)ni * ldc] = v;
      }
    }
}

// C = alpha sum_z P[z] + beta D over ks slices P[z] = P + z M N (leading dimension M),
// summed in slice order.
__global__ void k_gemm_sum(int M, int N, int ks, const double* __restrict__ P, double alpha,
                           double beta, const double* __restrict__ D, int64_t ldd,
                           double* __restrict__ C, int64_t ldc) {
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (e >= (int64_t)M * N) return;
  const int i = (int)(e % M), j = (int)(e / M);
  double s = 0.0;
  for (int z = 0; z < ks; ++z) s += P[(int64_t)z * M * N + e];
  double v = alpha * s;
  if (D) v += beta * D[i + (int64_t)j * ldd];
  C[i + (int64_t)j * ldc] = v;
}

// Scatter one block row of the inverse Cholesky factor: rows k0..k0+nb of Linv get
// T21 (nb x k0, ld nb) left of the diagonal block and T22 (nb x nb lower, ld nb).
// Rows k0 .. k0+nb-1 of Linv (all m columns: the strict upper part is written as zeros, so
// the factor is complete whatever the buffers held) into both layouts.
__global__ void k_linv_scatter(double* Lc, double* Lr, int64_t ld, int k0, int nb, int m,
                               const double* __restrict__ T21, const double* __restrict__ T22) {
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  const int64_t tot = (int64_t)nb * m;
  if (e >= tot) return;
  const int r = (int)(e % nb);
  const int c = (int)(e / nb);   // 0 .. m-1
  double v;
  if (c < k0)
    v = T21[r + (int64_t)c * nb];
  else if (c < k0 + nb)
    v = (c - k0 <= r) ? T22[r + (int64_t)(c - k0) * nb] : 0.0;
  else
    v = 0.0;
  Lc[(k0 + r) + (int64_t)c * ld] = v;
  Lr[c + (int64_t)(k0 + r) * ld] = v;
}

// Gram border from the Gram-Schmidt projections: with q = (v - Q t)/rho,
// Q^T A_* q = (h - G_* t)/rho and Q^T A_i q = Q^T A_* q + w (w = Q^T (dmu o q)).
// vals[c] = (h[c] - u[c]) / rho, vals[k+1+c] = vals[c] + w[c] for c < k; the diagonal
// entries (c = k) come from d2[0] = q^T A_* q, d2[1] = q^T A_i q.
__global__ void k_border_from_proj(const double* __restrict__ h, const double* __restrict__ u,
                                   const double* __restrict__ w, const double* __restrict__ nrm2,
                                   const double* __restrict__ d2, int k,
                                   double* __restrict__ vals) {
  const int c = blockIdx.x * BS + threadIdx.x;
  if (c > k) return;
  if (c == k) {
    vals[k] = d2[0];
    vals[2 * k + 1] = d2[1];
    return;
  }
  const double inv = 1.0 / sqrt(nrm2[0]);
  const double gs = (h[c] - u[c]) * inv;
  vals[c] = gs;
  vals[k + 1 + c] = gs + w[c];
}

// out[0] = x^T a, out[1] = x^T b (partials; finished by k_reduce_finish<2>); also
// z = dmu o x.
__global__ void k_dot2_scale(int64_t n, const double* __restrict__ x, const double* __restrict__ a,
                             const double* __restrict__ b, const double* __restrict__ dmu,
                             double* __restrict__ z, double* partials) {
  double v[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    const double xi = x[i];
    v[0] += xi * a[i];
    v[1] += xi * b[i];
    if (z) z[i] = dmu[i] * xi;
  }
  write_partials<2, BS>(v, partials, blockIdx.x);
}

// ---- rows of bump support, compacted once per parameter point ----------------------
// counts[b] = rows r of block b (256 rows) with w[r] != 0.
__global__ __launch_bounds__(BS) void k_nz_count(int64_t n, const double* __restrict__ w,
                                                 int* __restrict__ counts) {
  __shared__ int sh[BS / WAVE];
  const int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x;
  const uint64_t b = __ballot(r < n && w[r] != 0.0);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = __popcll(b);
  __syncthreads();
  if (threadIdx.x == 0) {
    int c = 0;
#pragma unroll
    for (int k = 0; k < BS / WAVE; ++k) c += sh[k];
    counts[blockIdx.x] = c;
  }
}

// Exclusive prefix sums of counts[0..nb) in place (one block: each thread a run of
// consecutive counts, then a scan of the run totals in LDS); the total goes to *total.
__global__ __launch_bounds__(1024) void k_nz_scan(int nb, int* __restrict__ counts,
                                                  int* __restrict__ total) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int per = (nb + 1023) / 1024;
  const int b0 = t * per, b1 = min(nb, b0 + per);
  int s = 0;
  for (int b = b0; b < b1; ++b) s += counts[b];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = t > 0 ? part[t - 1] : 0;
  for (int b = b0; b < b1; ++b) {
    const int c = counts[b];
    counts[b] = run;
    run += c;
  }
  if (t == 1023) *total = part[1023];
}

// idx[pos] = r and wc[pos] = w[r] for every row with w[r] != 0, in ascending row order
// (pos = the block's offset + the non-zero rows before r in the block); positions past
// cap are not written.
__global__ __launch_bounds__(BS) void k_nz_scatter(int64_t n, const double* __restrict__ w,
                                                   const int* __restrict__ offs, int64_t cap,
                                                   int64_t* __restrict__ idx,
                                                   double* __restrict__ wc) {
  __shared__ int sh[BS / WAVE];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x;
  const double v = r < n ? w[r] : 0.0;
  const bool nz = v != 0.0;
  const uint64_t b = __ballot(nz);
  if (lane == 0) sh[wid] = __popcll(b);
  __syncthreads();
  int before = 0;
  for (int k = 0; k < wid; ++k) before += sh[k];
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t pos = (int64_t)offs[blockIdx.x] + before + __popcll(b & lt);
  if (nz && pos < cap) {
    idx[pos] = r;
    wc[pos] = v;
  }
}

// Vb[t + c ldb] = M[idx[t] + c ld] for t < cnt, column c = c0 + blockIdx.y.
__global__ void k_gather_idx(const double* __restrict__ M, int64_t ld,
                             const int64_t* __restrict__ idx, int64_t cnt, int c0,
                             double* __restrict__ Vb, int64_t ldb) {
  const int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x;
  const int64_t c = c0 + blockIdx.y;
  if (t < cnt) Vb[t + c * ldb] = M[idx[t] + c * ld];
}

// qb[t] = q[idx[t]] (if qb), zb[t] = wc[t] q[idx[t]] for t < cnt.
__global__ void k_gather_scale(const double* __restrict__ q, const int64_t* __restrict__ idx,
                               const double* __restrict__ wc, int64_t cnt,
                               double* __restrict__ qb, double* __restrict__ zb) {
  const int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (t < cnt) {
    const double v = q[idx[t]];
    if (qb) qb[t] = v;
    zb[t] = wc[t] * v;
  }
}

__global__ void k_border_fill(const double* __restrict__ vals, int k, double* Gs, double* Gi,
                              int64_t ldg) {
  const int c = blockIdx.x * BS + threadIdx.x;
  if (c > k) return;
  const double a = vals[c], b = vals[k + 1 + c];
  Gs[c + k * ldg] = a;
  Gs[k + c * ldg] = a;
  Gi[c + k * ldg] = b;
  Gi[k + c * ldg] = b;
}

}  // namespace

void launch_gemm(int M, int N, int K, double alpha, const double* A, int64_t lda, bool ta,
                 const double* B, int64_t ldb, bool tb, double beta, const double* D, int64_t ldd,
                 double* C, int64_t ldc, hipStream_t st, double* part, size_t part_elems) {
  if (M <= 0 || N <= 0) return;
  const int tiles = ceil_div(M, 64) * ceil_div(N, 64);
  // split K when the output has few tiles and K is long: chunks of >= 64, ~128 blocks
  int ks = 1;
  if (part && tiles < 64 && K >= 128) {
    ks = std::min(ceil_div(K, 64), std::max(1, 128 / tiles));
    ks = (int)std::min<int64_t>(ks, (int64_t)(part_elems / ((size_t)M * N)));
  }
  if (ks <= 1) {
    ROM_LAUNCH(k_gemm, dim3(ceil_div(M, 64), ceil_div(N, 64)), dim3(BS), 0, st, M, N, K, K,
               alpha, A, lda, ta ? 1 : 0, B, ldb, tb ? 1 : 0, beta, D, ldd, C, ldc);
    return;
  }
  const int kc = (ceil_div(K, ks) + 15) / 16 * 16;
  ks = ceil_div(K, kc);
  ROM_LAUNCH(k_gemm, dim3(ceil_div(M, 64), ceil_div(N, 64), ks), dim3(BS), 0, st, M, N, K, kc,
             1.0, A, lda, ta ? 1 : 0, B, ldb, tb ? 1 : 0, 0.0, (const double*)nullptr,
             (int64_t)0, part, (int64_t)M);
  ROM_LAUNCH(k_gemm_sum, dim3(ceil_div((int64_t)M * N, BS)), dim3(BS), 0, st, M, N, ks,
             (const double*)part, alpha, beta, D, ldd, C, ldc);
}

void launch_linv_rebuild(const double* G, int64_t ldg, int m, double* Lc, double* Lr,
                         double* work, int* status, hipStream_t st) {
  // work: 3 nb^2 (S, Linv22, Ginv22) + 3 nb m + the K-split slices (linv_rebuild_work)
  constexpr int NB = 64;
  double* S = work;
  double* L22 = S + NB * NB;
  double* G22i = L22 + NB * NB;
  double* T1 = G22i + NB * NB;
  double* T2 = T1 + (int64_t)NB * m;
  double* T3 = T2 + (int64_t)NB * m;
  double* SK = T3 + (int64_t)NB * m;
  const size_t sk = (size_t)GEMM_KSPLIT * NB * std::max(m, NB);
  for (int k0 = 0; k0 < m; k0 += NB) {
    const int nb = std::min(NB, m - k0);
    if (k0 == 0) {
      launch_gemm(nb, nb, 0, 0.0, nullptr, 1, false, nullptr, 1, false, 1.0, G, ldg, S, nb, st);
    } else {
      // L21 = G21 Linv11^T  (nb x k0); Linv11^T is Lr in column-major form
      launch_gemm(nb, k0, k0, 1.0, G + k0, ldg, false, Lr, ldg, false, 0.0, nullptr, 0,
                  T1, nb, st, SK, sk);
      // S = G22 - L21 L21^T
      launch_gemm(nb, nb, k0, -1.0, T1, nb, false, T1, nb, true, 1.0, G + k0 + k0 * ldg, ldg,
                  S, nb, st, SK, sk);
    }
    launch_small_chol_inv(S, nb, L22, G22i, status, st);
    if (k0 > 0) {
      // M = L21 Linv11 (nb x k0), Linv21 = -Linv22 M
      launch_gemm(nb, k0, k0, 1.0, T1, nb, false, Lc, ldg, false, 0.0, nullptr, 0, T2, nb,
                  st, SK, sk);
      launch_gemm(nb, k0, nb, -1.0, L22, nb, false, T2, nb, false, 0.0, nullptr, 0, T3, nb, st);
    }
    const int64_t tot = (int64_t)nb * m;
    ROM_LAUNCH(k_linv_scatter, dim3(ceil_div(tot, BS)), dim3(BS), 0, st, Lc, Lr, ldg, k0, nb, m, T3,
               L22);
  }
}

void launch_border_from_proj(const double* h, const double* u, const double* w,
                             const double* nrm2, const double* d2, int k, double* vals,
                             hipStream_t st) {
  ROM_LAUNCH(k_border_from_proj, dim3(ceil_div(k + 1, BS)), dim3(BS), 0, st, h, u, w, nrm2, d2, k,
             vals);
}

void launch_dot2_scale(int64_t n, const double* x, const double* a, const double* b,
                       const double* dmu, double* z, double* out2, double* partials,
                       hipStream_t st) {
  const int grid = reduce_grid(n);
  ROM_LAUNCH(k_dot2_scale, dim3(grid), dim3(BS), 0, st, n, x, a, b, dmu, z, partials);
  launch_reduce_finish(partials, grid, 2, out2, st);
}

void launch_border_fill(const double* vals, int k, double* Gs, double* Gi, int64_t ldg,
                        hipStream_t st) {
  ROM_LAUNCH(k_border_fill, dim3(ceil_div(k + 1, BS)), dim3(BS), 0, st, vals, k, Gs, Gi,
                     ldg);
  ROM_CHECK_LAUNCH();
}

size_t gemvt_partials(int64_t rows, int cols, int nv) {
  const int chunk = 64 * gemvt_cpl(cols);
  const int64_t nch = (rows + chunk - 1) / chunk;
  return nch <= 1 ? 0 : (size_t)nch * nv * cols;
}

size_t gemvt_partials_max(int64_t rows, int maxcols, int nv) {
  // the chunk height switches at 64 columns; within each regime the size grows with cols
  return std::max(gemvt_partials(rows, std::min(maxcols, 64), nv),
                  gemvt_partials(rows, maxcols, nv));
}

void launch_gemvt(const double* M, int64_t ld, int64_t rows, int cols, const double* V,
                  int64_t vstride, int nv, double* out, double* partials, hipStream_t st,
                  Skip skip) {
  if (cols <= 0) return;
  const int cpl = gemvt_cpl(cols);
  const int chunk = 64 * cpl;
  const int64_t nch = std::max<int64_t>(1, ceil_div(rows, chunk));
  // GT_COLS columns per block; a product that would not fill the chip that way (the
  // m x m triangular solves, short tall-skinny ones) takes one column per wave instead
  const int gcols = nch * ceil_div(cols, GT_COLS) < 512 ? BS / 64 : GT_COLS;
  dim3 grid((unsigned)nch, ceil_div(cols, gcols));
#define GT_LAUNCH(C, N, Q) \
  ROM_LAUNCH((k_gemvt<C, N, Q>), grid, dim3(BS), 0, st, M, ld, rows, cols, V, vstride, out, \
             partials, skip, gcols)
  if (nv < 1 || nv > 3) throw Error(ROM_EINVAL, "gemvt: 1 to 3 vectors");
  const bool q4 = ld % 2 == 0 && ((uintptr_t)M & 15) == 0 && ((uintptr_t)V & 15) == 0 &&
                  (nv == 1 || vstride % 2 == 0);
  if (cpl == 16 && q4) {
    if (nv == 1) GT_LAUNCH(16, 1, true); else if (nv == 2) GT_LAUNCH(16, 2, true);
    else GT_LAUNCH(16, 3, true);
  } else if (cpl == 16) {
    if (nv == 1) GT_LAUNCH(16, 1, false); else if (nv == 2) GT_LAUNCH(16, 2, false);
    else GT_LAUNCH(16, 3, false);
  } else {
    if (nv == 1) GT_LAUNCH(4, 1, false); else if (nv == 2) GT_LAUNCH(4, 2, false);
    else GT_LAUNCH(4, 3, false);
  }
#undef GT_LAUNCH
  ROM_CHECK_LAUNCH();
  if (grid.x > 1) {
    const int ne = nv * cols;
    ROM_LAUNCH(k_gemvt_reduce, dim3(ceil_div(ne, BS / WAVE)), dim3(BS), 0, st, partials,
                       (int)grid.x, ne, out, skip);
    ROM_CHECK_LAUNCH();
  }
}

void launch_gemvn(const double* M, int64_t ld, int64_t rows, int cols, const double* coef,
                  double alpha, const double* in, double beta, double* out, double* nrm2,
                  double* partials, hipStream_t st, Skip skip) {
  const size_t shm = (size_t)(cols > 0 ? cols : 1) * sizeof(double);
  // four rows per thread where the basis allows it (the usual case: columns padded to 64)
  const bool four = ld % 4 == 0 && ((uintptr_t)M & 15) == 0;
  const int grid = four ? std::min(256, std::max(1, ceil_div(rows, 4 * BS))) : reduce_grid(rows);
  if (nrm2) {
    if (four)
      ROM_LAUNCH(k_gemvn4<true>, dim3(grid), dim3(BS), shm, st, M, ld, rows, cols, coef, alpha,
                 in, beta, out, partials, skip);
    else
      ROM_LAUNCH(k_gemvn<true>, dim3(grid), dim3(BS), shm, st, M, ld, rows, cols, coef, alpha,
                 in, beta, out, partials, skip);
    ROM_CHECK_LAUNCH();
    launch_reduce_finish(partials, grid, 1, nrm2, st, skip);
  } else {
    if (four)
      ROM_LAUNCH(k_gemvn4<false>, dim3(grid), dim3(BS), shm, st, M, ld, rows, cols, coef, alpha,
                 in, beta, out, partials, skip);
    else
      ROM_LAUNCH(k_gemvn<false>, dim3(grid), dim3(BS), shm, st, M, ld, rows, cols, coef, alpha,
                 in, beta, out, partials, skip);
    ROM_CHECK_LAUNCH();
  }
}

bool gemvn_fused_ok(const double* M, int64_t ld, int cols) {
  return cols > 0 && ld % 4 == 0 && ((uintptr_t)M & 15) == 0 &&
         (size_t)3 * cols * sizeof(double) <= 64 * 1024;
}

void launch_gemvn_fused(const double* M, int64_t ld, int64_t rows, int cols, const double* t,
                        const double* c1, const double* c2, const double* in, double* out0,
                        double* out1, double* out2, double* nrm2, double* partials,
                        hipStream_t st) {
  if (!gemvn_fused_ok(M, ld, cols)) throw Error(ROM_EINVAL, "gemvn_fused: layout not supported");
  // one block per CU, as for k_gemvn4 (its streaming rate was measured with this shape)
  const int grid = std::min(256, std::max(1, ceil_div(rows, 4 * BS)));
  const size_t shm = (size_t)3 * cols * sizeof(double);
  ROM_LAUNCH(k_gemvn4x3, dim3(grid), dim3(BS), shm, st, M, ld, rows, cols, t, c1, c2, in, out0,
             out1, out2, partials);
  ROM_CHECK_LAUNCH();
  launch_reduce_finish(partials, grid, 1, nrm2, st);
}

void launch_fused_start(int64_t n, const double* a, const double* u, const double* w,
                        const double* cm, double s, double* out, hipStream_t st) {
  if (n <= 0) return;
  const int gx = std::min(ceil_div(n, BS), 1024);
  ROM_LAUNCH(k_fused_start, dim3(gx), dim3(BS), 0, st, n, a, u, w, cm, s, out);
  ROM_CHECK_LAUNCH();
}

void launch_gemvn_multi(const double* M, int64_t ld, int64_t rows, int cols, const double* coef,
                        int64_t ldc, int nv, double alpha, const double* in, int64_t ldi,
                        double beta, double* out, int64_t ldo, hipStream_t st) {
  if (nv <= 0 || rows <= 0) return;
  if (nv > 16) throw Error(ROM_EINVAL, "gemvn_multi: at most 16 vectors");
#define GM_LAUNCH(NV, RPT)                                                                   \
  ROM_LAUNCH((k_gemvn_multi<NV, RPT>), dim3(ceil_div(rows, BS * RPT)), dim3(BS), 0, st, M, ld, \
             rows, cols, coef, ldc, nv, alpha, in, ldi, beta, out, ldo)
  if (nv <= 2)
    GM_LAUNCH(2, 4);
  else if (nv <= 4)
    GM_LAUNCH(4, 4);
  else if (nv <= 8)
    GM_LAUNCH(8, 2);
  else
    GM_LAUNCH(16, 1);
#undef GM_LAUNCH
  ROM_CHECK_LAUNCH();
}

void launch_axpby_cols(int64_t n, int nv, double a, const double* x, int64_t ldx, double b,
                       const double* y, int64_t ldy, double* out, int64_t ldo, hipStream_t st) {
  if (nv <= 0 || n <= 0) return;
  int gx = ceil_div(n, BS);
  if (gx > 512) gx = 512;
  ROM_LAUNCH(k_axpby_cols, dim3(gx, nv), dim3(BS), 0, st, n, a, x, ldx, b, y, ldy, out, ldo);
  ROM_CHECK_LAUNCH();
}

void launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* out,
                  double* nrm2, double* partials, hipStream_t st) {
  const int grid = reduce_grid(n);
  ROM_LAUNCH(k_axpby, dim3(grid), dim3(BS), 0, st, n, a, x, b, y, out, nrm2 ? 1 : 0,
                     partials);
  ROM_CHECK_LAUNCH();
  if (nrm2) launch_reduce_finish(partials, grid, 2, nrm2, st);
}

void launch_publish(const void* src, void* dst, size_t bytes, unsigned* flag, unsigned seq,
                    hipStream_t st) {
  if (bytes % sizeof(double) != 0 || bytes / sizeof(double) > (size_t)64 * PUBLISH_WORDS)
    throw Error(ROM_EINVAL, "publish: size must be a multiple of 8 bytes, at most 16 KiB");
  ROM_LAUNCH(k_publish, dim3(1), dim3(64), 0, st, static_cast<const double*>(src),
             static_cast<double*>(dst), (int)(bytes / sizeof(double)), flag, seq);
  ROM_CHECK_LAUNCH();
}

void launch_normalize(int64_t n, double* x, const double* nrm2, hipStream_t st) {
  ROM_LAUNCH(k_normalize, dim3(reduce_grid(n)), dim3(BS), 0, st, n, x, nrm2);
  ROM_CHECK_LAUNCH();
}

void launch_cast_cols_f32(int64_t n, int k, const double* in, int64_t ld, float* out,
                          hipStream_t st) {
  if (k <= 0 || n <= 0) return;
  int gx = ceil_div(n, BS);
  if (gx > 512) gx = 512;
  ROM_LAUNCH(k_cast_cols_f32, dim3(gx, k), dim3(BS), 0, st, n, in, ld, out);
  ROM_CHECK_LAUNCH();
}

void launch_convert_cols(int64_t n, int k, const float* in, int64_t ldi, double* out, int64_t ldo,
                         hipStream_t st) {
  if (k <= 0 || n <= 0) return;
  const int gx = std::min(ceil_div(n, BS), 512);
  ROM_LAUNCH((k_convert_cols<float, double>), dim3(gx, k), dim3(BS), 0, st, n, in, ldi, out, ldo);
  ROM_CHECK_LAUNCH();
}

void launch_convert_cols(int64_t n, int k, const double* in, int64_t ldi, float* out, int64_t ldo,
                         hipStream_t st) {
  if (k <= 0 || n <= 0) return;
  const int gx = std::min(ceil_div(n, BS), 512);
  ROM_LAUNCH((k_convert_cols<double, float>), dim3(gx, k), dim3(BS), 0, st, n, in, ldi, out, ldo);
  ROM_CHECK_LAUNCH();
}

void launch_scale_cols(int64_t n, int k, const double* in, int64_t ldi, const double* norm2,
                       double* out, int64_t ldo, hipStream_t st) {
  if (k <= 0 || n <= 0) return;
  const int gx = std::min(ceil_div(n, BS), 512);
  ROM_LAUNCH(k_scale_cols, dim3(gx, k), dim3(BS), 0, st, n, in, ldi, norm2, out, ldo);
  ROM_CHECK_LAUNCH();
}

void launch_cast_f32(int64_t n, const double* in, float* out, hipStream_t st) {
  launch_cast_cols_f32(n, 1, in, n, out, st);
}

void launch_refine_update(int64_t n, double sigma, const float* d, double* g, const double* x0,
                          double* x, hipStream_t st) {
  if (n <= 0) return;
  ROM_LAUNCH(k_refine_update, dim3(reduce_grid(n)), dim3(BS), 0, st, n, sigma, d, g, x0, x);
  ROM_CHECK_LAUNCH();
}

template <typename T>
void launch_refine_cols(int64_t n, int nb, const Coefs& coef, const T* d, int64_t ldd, double* g,
                        const double* x0, int64_t ld, double* x, int64_t ldx, hipStream_t st) {
  if (n <= 0 || nb <= 0) return;
  int gx = ceil_div(n, BS);
  if (gx > 512) gx = 512;
  ROM_LAUNCH((k_refine_cols<T>), dim3(gx, nb), dim3(BS), 0, st, n, coef, d, ldd, g, x0, ld, x, ldx);
  ROM_CHECK_LAUNCH();
}
template void launch_refine_cols<double>(int64_t, int, const Coefs&, const double*, int64_t,
                                         double*, const double*, int64_t, double*, int64_t,
                                         hipStream_t);
template void launch_refine_cols<float>(int64_t, int, const Coefs&, const float*, int64_t, double*,
                                        const double*, int64_t, double*, int64_t, hipStream_t);

void launch_col_norms(int64_t n, int s, const double* X, int64_t ld, double* out,
                      double* partials, hipStream_t st) {
  if (s <= 0) return;
  const int P = std::min(256, std::max(1, ceil_div(n, BS * 4)));
  ROM_LAUNCH(k_colnorm2, dim3(P, s), dim3(BS), 0, st, n, X, ld, partials);
  ROM_CHECK_LAUNCH();
  ROM_LAUNCH(k_sum_cols, dim3(s), dim3(BS), 0, st, partials, P, out);
  ROM_CHECK_LAUNCH();
}

void launch_border_fill_block(const double* B, int64_t ldb, int m, int k, double* Gs, double* Gi,
                              int64_t ldg, hipStream_t st) {
  if (k <= 0) return;
  ROM_LAUNCH(k_border_fill_block, dim3(ceil_div(m + k, BS), k), dim3(BS), 0, st, B, ldb, m, k, Gs,
             Gi, ldg);
  ROM_CHECK_LAUNCH();
}

void launch_pack_cols(int64_t n, const ColPtrs& src, int k, double* dst, int64_t ld,
                      hipStream_t st) {
  if (k <= 0) return;
  int gx = ceil_div(n, BS);
  if (gx > 256) gx = 256;
  ROM_LAUNCH(k_pack_cols, dim3(gx, k), dim3(BS), 0, st, n, src, k, dst, ld);
  ROM_CHECK_LAUNCH();
}

void launch_gather_row(const double* M, int64_t ld, int cols, int64_t idx, double scale,
                       double* out, hipStream_t st) {
  if (cols <= 0) return;
  ROM_LAUNCH(k_gather_row, dim3(ceil_div(cols, BS)), dim3(BS), 0, st, M, ld, cols, idx,
                     scale, out);
  ROM_CHECK_LAUNCH();
}

void launch_gather_rows(const double* M, int64_t ld, int cols, const int64_t* idx,
                        const double* scale, int nidx, double* out, int64_t ldo,
                        hipStream_t st) {
  if (cols <= 0 || nidx <= 0) return;
  ROM_LAUNCH(k_gather_rows, dim3(ceil_div(cols, BS), nidx), dim3(BS), 0, st, M, ld, cols,
                     idx, scale, nidx, out, ldo);
  ROM_CHECK_LAUNCH();
}

void launch_linv_border(double* Lc, double* Lr, int64_t ld, int k, const double* gcol,
                        double* tmp_l, double* tmp_r, int* status, double* partials,
                        hipStream_t st, double* info) {
  if (k > 0) {
    // l = Linv g: row i of Linv is column i of Lr.
    launch_gemvt(Lr, ld, k, k, gcol, 0, 1, tmp_l, partials, st);
    // r = Linv^T l: column j of Linv is column j of Lc.
    launch_gemvt(Lc, ld, k, k, tmp_l, 0, 1, tmp_r, partials, st);
  }
  ROM_LAUNCH(k_linv_finish, dim3(1), dim3(BS), 0, st, Lc, Lr, ld, k, gcol, tmp_l, tmp_r,
                     status, info);
  ROM_CHECK_LAUNCH();
}

void launch_linv_solve(const double* Lc, const double* Lr, int64_t ld, int m, const double* t,
                       double* u, double* c, double* partials, hipStream_t st) {
  if (m <= 0) return;
  launch_gemvt(Lr, ld, m, m, t, 0, 1, u, partials, st);
  launch_gemvt(Lc, ld, m, m, u, 0, 1, c, partials, st);
}

void launch_linv_solve_multi(const double* Lc, const double* Lr, int64_t ld, int m, const double* T,
                             int64_t tstride, int nv, double* U, double* C, double* partials,
                             hipStream_t st) {
  if (m <= 0) return;
  launch_gemvt(Lr, ld, m, m, T, tstride, nv, U, partials, st);
  launch_gemvt(Lc, ld, m, m, U, m, nv, C, partials, st);
}

void launch_nz_rows(int64_t n, const double* w, int64_t* idx, double* wc, int64_t cap, int* total,
                    int* work, hipStream_t st) {
  const int nb = ceil_div(n, BS);
  if (nb < 1) return;
  ROM_LAUNCH(k_nz_count, dim3(nb), dim3(BS), 0, st, n, w, work);
  ROM_LAUNCH(k_nz_scan, dim3(1), dim3(1024), 0, st, nb, work, total);
  ROM_LAUNCH(k_nz_scatter, dim3(nb), dim3(BS), 0, st, n, w, (const int*)work, cap, idx, wc);
}

void launch_gather_idx(const double* M, int64_t ld, const int64_t* idx, int64_t cnt, int c0,
                       int c1, double* Vb, int64_t ldb, hipStream_t st) {
  if (cnt <= 0 || c1 <= c0) return;
  ROM_LAUNCH(k_gather_idx, dim3(ceil_div(cnt, BS), c1 - c0), dim3(BS), 0, st, M, ld, idx, cnt, c0,
             Vb, ldb);
}

void launch_gather_scale(const double* q, const int64_t* idx, const double* wc, int64_t cnt,
                         double* qb, double* zb, hipStream_t st) {
  if (cnt <= 0) return;
  ROM_LAUNCH(k_gather_scale, dim3(ceil_div(cnt, BS)), dim3(BS), 0, st, q, idx, wc, cnt, qb, zb);
}

void launch_small_chol_inv(const double* G, int m, double* Linv, double* Ginv, int* status,
                           hipStream_t st) {
  if (m <= 0) return;
  ROM_LAUNCH(k_small_chol_inv, dim3(1), dim3(BS), 0, st, G, m, Linv, Ginv, status);
  ROM_CHECK_LAUNCH();
}

namespace {
__global__ void k_gram_assemble(const double* __restrict__ Gs, int lds, int k,
                                double* __restrict__ G, int m) {
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
    const int i = e % m, j = e / m;
    if (i < k && j < k) G[i + j * m] = Gs[i + j * lds];
    else if (j < k) G[i + j * m] = G[j + i * m];   // i >= k: mirror of the computed border
  }
}
}  // namespace

void launch_gram_assemble(const double* Gs, int lds, int k, double* G, int m, hipStream_t st) {
  if (m <= 0 || k < 0 || k > m || m > NJ_MAX) throw Error(ROM_EINVAL, "gram_assemble: bad sizes");
  ROM_LAUNCH(k_gram_assemble, dim3(1), dim3(BS), 0, st, Gs, lds, k, G, m);
  ROM_CHECK_LAUNCH();
}

}  // namespace rom
