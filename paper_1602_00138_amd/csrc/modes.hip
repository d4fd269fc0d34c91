// Kernels of the lowest-eigenpair solver for U_0 (the block of eigenvectors of the
// operator for its smallest eigenvalues that seeds Algorithm 2, Sec. 4.2.2; the paper
// computes it offline): Chebyshev-filtered subspace iteration.  The SpMM, the Gram and
// the small Cholesky inverse are the path's own kernels; here are the pieces only this
// solver needs: a small symmetric eigensolver for the Rayleigh-Ritz step, the filter's
// three-term combination, the Ritz residuals and the Gershgorin bound.
#include <algorithm>

#include "kernels.h"

namespace rom {

namespace {

constexpr int BS = 256;
constexpr int EIG_MAX = 32;

// Eigenpairs of the symmetric m x m matrix H (column-major, ld): Jacobi rotations in the
// parallel (round-robin) order: each round rotates m/2 disjoint index pairs at once, first
// the rows, then the columns (H <- J^T H J), and accumulates Z <- Z J; the players move
// one seat round the table after every round (index 0 fixed).  Sweeps until the
// off-diagonal Frobenius norm is below 1e-15 of the whole (at most 40 sweeps).  Outputs
// the eigenvalues ascending in lam and the matching unit eigenvectors as columns of Z
// (column-major, m x m).  One workgroup, m <= EIG_MAX.
__global__ __launch_bounds__(BS) void k_sym_eig(const double* __restrict__ H, int64_t ld, int m,
                                                double* __restrict__ lam,
                                                double* __restrict__ Z) {
  __shared__ double A[EIG_MAX][EIG_MAX + 1];
  __shared__ double V[EIG_MAX][EIG_MAX + 1];
  __shared__ double cs[EIG_MAX / 2], sn[EIG_MAX / 2];
  __shared__ int pp[EIG_MAX / 2], qq[EIG_MAX / 2];
  __shared__ int order[EIG_MAX + 1];
  __shared__ double off2, tot2;
  __shared__ double red[(BS / WAVE) * 2];
  const int t = threadIdx.x;
  const int mp = m + (m & 1);   // players (an odd m sits one out per round)
  for (int e = t; e < m * m; e += BS) {
    const int i = e % m, j = e / m;
    A[i][j] = 0.5 * (H[i + j * ld] + H[j + i * ld]);
    V[i][j] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  // player at seat k of round r: seat 0 keeps player 0, the others rotate one seat a round
  auto seat = [&](int k, int r) {
    return k == 0 ? 0 : 1 + ((k - 1 - r) % (mp - 1) + (mp - 1)) % (mp - 1);
  };
  for (int sweep = 0; sweep < 40; ++sweep) {
    {
      double v2[2] = {0.0, 0.0};   // off-diagonal, whole
      for (int e = t; e < m * m; e += BS) {
        const int i = e % m, j = e / m;
        const double v = A[i][j] * A[i][j];
        v2[1] += v;
        if (i != j) v2[0] += v;
      }
      double s2;
      block_sum<2, BS>(v2, red, s2);
      if (t == 0) off2 = s2;
      if (t == 1) tot2 = s2;
      __syncthreads();
    }
    if (!(off2 > 1e-30 * tot2)) break;
    for (int round = 0; round < mp - 1; ++round) {
      // pair i: the players at seats i and mp - 1 - i
      if (t < mp / 2) {
        int p = seat(t, round), q = seat(mp - 1 - t, round);
        if (p > q) {
          const int s = p;
          p = q;
          q = s;
        }
        double c = 1.0, s = 0.0;
        if (q < m) {
          const double apq = A[p][q];
          if (apq != 0.0) {
            const double th = (A[q][q] - A[p][p]) / (2.0 * apq);
            const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(tt * tt + 1.0);
            s = tt * c;
          }
        }
        pp[t] = p;
        qq[t] = q;
        cs[t] = c;
        sn[t] = s;
      }
      __syncthreads();
      // rows p, q of A (pairs disjoint)
      for (int e = t; e < (mp / 2) * m; e += BS) {
        const int r = e / m, k = e % m;
        const int p = pp[r], q = qq[r];
        if (q < m) {
          const double c = cs[r], s = sn[r];
          const double ap = A[p][k], aq = A[q][k];
          A[p][k] = c * ap - s * aq;
          A[q][k] = s * ap + c * aq;
        }
      }
      __syncthreads();
      // columns p, q of A and of V
      for (int e = t; e < (mp / 2) * m; e += BS) {
        const int r = e / m, k = e % m;
        const int p = pp[r], q = qq[r];
        if (q < m) {
          const double c = cs[r], s = sn[r];
          const double ap = A[k][p], aq = A[k][q];
          A[k][p] = c * ap - s * aq;
          A[k][q] = s * ap + c * aq;
          const double vp = V[k][p], vq = V[k][q];
          V[k][p] = c * vp - s * vq;
          V[k][q] = s * vp + c * vq;
        }
      }
      __syncthreads();
    }
  }
  // sort ascending (m <= 32: a selection by thread 0), then write
  if (t == 0) {
    for (int i = 0; i < m; ++i) order[i] = i;
    for (int i = 0; i < m; ++i) {
      int b = i;
      for (int j = i + 1; j < m; ++j)
        if (A[order[j]][order[j]] < A[order[b]][order[b]]) b = j;
      const int s = order[i];
      order[i] = order[b];
      order[b] = s;
    }
  }
  __syncthreads();
  for (int e = t; e < m * m; e += BS) {
    const int i = e % m, j = e / m;
    Z[i + (int64_t)j * m] = V[i][order[j]];
  }
  for (int j = t; j < m; j += BS) lam[j] = A[order[j]][order[j]];
}

// out[:, v] = a AY[:, v] + b Y[:, v] + c Y2[:, v] for v < k (Y2 may be NULL).
__global__ void k_comb3(int64_t n, int k, double a, const double* __restrict__ AY, double b,
                        const double* __restrict__ Y, double c, const double* __restrict__ Y2,
                        int64_t ld, double* __restrict__ out) {
  const int v = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    const int64_t e = i + v * ld;
    double o = a * AY[e] + b * Y[e];
    if (Y2) o += c * Y2[e];
    out[e] = o;
  }
}

// R[:, v] = AY[:, v] - lam[v] Y[:, v] for v < k.
__global__ void k_ritz_resid(int64_t n, int k, const double* __restrict__ AY,
                             const double* __restrict__ Y, const double* __restrict__ lam,
                             int64_t ld, double* __restrict__ R) {
  const int v = blockIdx.y;
  const double l = lam[v];
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    const int64_t e = i + v * ld;
    R[e] = AY[e] - l * Y[e];
  }
}

// Block maxima of 2 diag_i - (A 1)_i = a_ii + sum_{j != i} |a_ij| (off-diagonals of the
// operator are non-positive), then their maximum: the Gershgorin bound of the spectrum.
__global__ void k_gersh(int64_t n, const double* __restrict__ diag, const double* __restrict__ a1,
                        double* __restrict__ partials) {
  __shared__ double sh[BS];
  double v = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
    v = fmax(v, 2.0 * diag[i] - a1[i]);
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = BS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

__global__ void k_max_finish(int P, const double* __restrict__ partials, double* out) {
  __shared__ double sh[BS];
  double v = 0.0;
  for (int b = threadIdx.x; b < P; b += BS) v = fmax(v, partials[b]);
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = BS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// out (column-major, m x m) = in^T
__global__ void k_transpose_small(int m, const double* __restrict__ in, double* __restrict__ out) {
  for (int e = threadIdx.x; e < m * m; e += BS) {
    const int i = e % m, j = e / m;
    out[j + i * m] = in[i + j * m];
  }
}

__global__ void k_fill(int64_t n, double v, double* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
    x[i] = v;
}

int grid1(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>((n + BS - 1) / BS, 1), 1024); }

}  // namespace

void launch_sym_eig(const double* H, int64_t ld, int m, double* lam, double* Z, hipStream_t st) {
  if (m < 1 || m > EIG_MAX) throw Error(ROM_EINVAL, "sym_eig: order out of range");
  ROM_LAUNCH(k_sym_eig, dim3(1), dim3(BS), 0, st, H, ld, m, lam, Z);
  ROM_CHECK_LAUNCH();
}

void launch_comb3(int64_t n, int k, double a, const double* AY, double b, const double* Y,
                  double c, const double* Y2, int64_t ld, double* out, hipStream_t st) {
  if (k <= 0 || n <= 0) return;
  ROM_LAUNCH(k_comb3, dim3(std::min(grid1(n), 256), k), dim3(BS), 0, st, n, k, a, AY, b, Y, c,
             Y2, ld, out);
  ROM_CHECK_LAUNCH();
}

void launch_ritz_resid(int64_t n, int k, const double* AY, const double* Y, const double* lam,
                       int64_t ld, double* R, hipStream_t st) {
  if (k <= 0 || n <= 0) return;
  ROM_LAUNCH(k_ritz_resid, dim3(std::min(grid1(n), 256), k), dim3(BS), 0, st, n, k, AY, Y, lam, ld,
             R);
  ROM_CHECK_LAUNCH();
}

void launch_gersh(int64_t n, const double* diag, const double* a1, double* partials, double* out,
                  hipStream_t st) {
  const int P = grid1(n);
  ROM_LAUNCH(k_gersh, dim3(P), dim3(BS), 0, st, n, diag, a1, partials);
  ROM_LAUNCH(k_max_finish, dim3(1), dim3(BS), 0, st, P, (const double*)partials, out);
  ROM_CHECK_LAUNCH();
}

void launch_transpose_small(int m, const double* in, double* out, hipStream_t st) {
  ROM_LAUNCH(k_transpose_small, dim3(1), dim3(BS), 0, st, m, in, out);
  ROM_CHECK_LAUNCH();
}

void launch_fill(int64_t n, double v, double* x, hipStream_t st) {
  ROM_LAUNCH(k_fill, dim3(grid1(n)), dim3(BS), 0, st, n, v, x);
  ROM_CHECK_LAUNCH();
}

}  // namespace rom
