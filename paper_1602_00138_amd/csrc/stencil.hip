// Stencil kernels: assembly of A_* (Sec. 3, eq. (sum)), RBF absorption, and the
// 5/7-point operator products used throughout the solve.
//
// Launch shape of the products: a block owns 256 consecutive nodes of an x-y plane
// (coalesced along x) and walks a chunk of z planes, carrying the z neighbours in
// registers, so each node value is fetched from HBM about once per product.
#include <algorithm>

#include "kernels.h"

namespace rom {

namespace {

constexpr int BS = 256;
// Columns per thread of the two-node SpMM: with a D field the diagonal and the three face
// arrays are shared by all columns, and 8 columns per thread took 64 columns at 96^3 from
// 2.0 to 3.1 TB/s; with constant D only the diagonal is shared and one column per thread
// is fastest (2 and 4 measured 1% and 13% slower at 64^3).
constexpr int SPMM_CPT_VAR = 8;
constexpr int SPMM_CPT_CONST = 1;
// The LDS-tiled SpMM: columns per block and the block count its z chunks aim at.  With a D
// field 4 columns share the diagonal and face loads (96 columns at 128^3: 3.0 TB/s with one
// column per block, 4.4 with four, against 3.2 for the register-walk k_spmm2c); with
// constant D one column per block over about 16k blocks was fastest at 64^3 (4.8 TB/s
// against 4.6 and 4.7 for 2 and 4 columns).  Fewer columns where their staged tiles would
// pass SPMM_LDS_MAX bytes of LDS.
constexpr int SPMM_LDS_C_VAR = 4;
constexpr int SPMM_LDS_C_CONST = 1;
constexpr int64_t SPMM_LDS_BLOCKS_VAR = 1024;
constexpr int64_t SPMM_LDS_BLOCKS_CONST = 16384;
constexpr size_t SPMM_LDS_MAX = 48 * 1024;

__global__ void k_assemble(rom_grid g, double Dc, const double* __restrict__ D, int64_t n,
                           double* __restrict__ diag, double* __restrict__ fx,
                           double* __restrict__ fy, double* __restrict__ fz) {
  int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= n) return;
  const int N[3] = {g.n[0], g.n[1], g.n[2]};
  int c[3];
  c[0] = (int)(i % N[0]);
  c[1] = (int)((i / N[0]) % N[1]);
  c[2] = (int)(i / ((int64_t)N[0] * N[1]));
  const int64_t st[3] = {1, N[0], (int64_t)N[0] * N[1]};
  double* F[3] = {fx, fy, fz};
  const bool cst = D == nullptr;
  const double Di = cst ? Dc : D[i];
  double d = 0.0;
  for (int a = 0; a < g.dim; ++a) {
    const double h = 1.0 / (N[a] + 1);
    const double ih2 = 1.0 / (h * h);
    // minus face
    if (c[a] > 0) {
      const double Dn = cst ? Di : D[i - st[a]];
      d += (cst ? Di : 2.0 * Di * Dn / (Di + Dn)) * ih2;
    } else {
      const double beta = g.bc[2 * a] == 1 ? h / (h + 2.0 * g.robin_A * Di) : 1.0;
      d += Di * ih2 * beta;
    }
    // plus face
    if (c[a] < N[a] - 1) {
      const double Dn = cst ? Di : D[i + st[a]];
      const double cf = (cst ? Di : 2.0 * Di * Dn / (Di + Dn)) * ih2;
      d += cf;
      if (F[a]) F[a][i] = cf;
    } else {
      const double beta = g.bc[2 * a + 1] == 1 ? h / (h + 2.0 * g.robin_A * Di) : 1.0;
      d += Di * ih2 * beta;
      if (F[a]) F[a][i] = 0.0;
    }
  }
  diag[i] = d;
}

// mu(p) - mu0 at every node, and diag_i = diag_* + mu(p).  A block's nodes are consecutive
// (a few grid rows of one or two planes): the bump parameters are staged in LDS and each
// bump is first tested against the block's bounding box, so a node only evaluates the
// bumps whose support can reach its block.
__global__ __launch_bounds__(BS) void k_mu_eval(Stencil S, Bumps B,
                                                const double* __restrict__ diag_star,
                                                double* __restrict__ diag_i,
                                                double* __restrict__ dmu) {
  __shared__ double bp[ROM_MAX_BUMPS * 5];
  __shared__ int live[ROM_MAX_BUMPS];
  const int stride = S.dim + 2;
  const int nb = B.nb;
  for (int t = threadIdx.x; t < nb * stride; t += BS) bp[t] = B.p[t];
  const int64_t i0 = (int64_t)blockIdx.x * BS;
  const int64_t i = i0 + threadIdx.x;
  const int64_t nxy = (int64_t)S.nx * S.ny;
  __syncthreads();
  if (threadIdx.x < nb) {
    // the block's bounding box in grid indices: all of x, its rows of y, its planes of z
    const int64_t i1 = min(i0 + BS, S.n) - 1;
    const int64_t z0 = i0 / nxy, z1 = i1 / nxy;
    int64_t y0 = 0, y1 = S.ny - 1;
    if (z0 == z1) {
      y0 = (i0 % nxy) / S.nx;
      y1 = (i1 % nxy) / S.nx;
    }
    const int64_t lo[3] = {0, y0, z0}, hi[3] = {S.nx - 1, y1, z1};
    const int n[3] = {S.nx, S.ny, S.nz};
    const double* pb = bp + threadIdx.x * stride;
    double d2 = 0.0;
    for (int c = 0; c < S.dim; ++c) {
      const double a = (lo[c] + 1.0) / (n[c] + 1), e = (hi[c] + 1.0) / (n[c] + 1);
      const double d = pb[c] < a ? a - pb[c] : pb[c] > e ? pb[c] - e : 0.0;
      d2 += d * d;
    }
    // conservative: a bump stays when its support may touch the box
    live[threadIdx.x] = d2 < pb[S.dim] * pb[S.dim] * (1.0 + 1e-9) ? 1 : 0;
  }
  __syncthreads();
  if (i >= S.n) return;
  int ix, iy, iz;
  if (S.n <= INT32_MAX) {     // 32-bit index arithmetic where the grid allows it
    const unsigned u = (unsigned)i, q = u / (unsigned)S.nx;
    ix = (int)(u - q * (unsigned)S.nx);
    iy = (int)(q % (unsigned)S.ny);
    iz = (int)(q / (unsigned)S.ny);
  } else {
    const int64_t q = i / S.nx;
    ix = (int)(i % S.nx);
    iy = (int)(q % S.ny);
    iz = (int)(q / S.ny);
  }
  const double x[3] = {(ix + 1.0) / (S.nx + 1), (iy + 1.0) / (S.ny + 1),
                       (iz + 1.0) / (S.nz + 1)};
  double m = 0.0;
  for (int b = 0; b < nb; ++b) {
    if (!live[b]) continue;
    const double* pb = bp + b * stride;
    double d2 = 0.0;
    for (int a = 0; a < S.dim; ++a) {
      const double e = x[a] - pb[a];
      d2 += e * e;
    }
    // outside the support (|x - c| >= r) the bump contributes nothing: skip the square
    // root and the division there
    if (d2 >= pb[S.dim] * pb[S.dim]) continue;
    const double t = sqrt(d2) / pb[S.dim];
    if (t < 1.0) {
      const double u = 1.0 - t;
      const double u2 = u * u;
      m += pb[S.dim + 1] * (u2 * u2) * (4.0 * t + 1.0);
    }
  }
  dmu[i] = m;
  if (diag_i) diag_i[i] = diag_star[i] + B.mu0 + m;
}

// w[j ld + i] = -d mu(x_i) / d p for the parameters of bump b in the order (a, r, c_0 ..
// c_{dim-1}), negated (the Jacobian column is -Z^T diag(d mu / d p) U).  With
// t = |x - c| / r and psi'(t) = -20 t (1-t)^3: d/da = psi(t), d/dr = 20 a t^2 (1-t)^3 / r,
// d/dc_d = 20 a (1-t)^3 (x_d - c_d) / r^2, all zero for t >= 1.
__global__ void k_mu_grad(Stencil S, Bumps B, int b, double* __restrict__ w, int64_t ld) {
  int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= S.n) return;
  const int ix = (int)(i % S.nx);
  const int64_t q = i / S.nx;
  const int iy = (int)(q % S.ny);
  const int iz = (int)(q / S.ny);
  const double x[3] = {(ix + 1.0) / (S.nx + 1), (iy + 1.0) / (S.ny + 1),
                       (iz + 1.0) / (S.nz + 1)};
  const double* pb = B.p + b * (S.dim + 2);
  const double r = pb[S.dim], a = pb[S.dim + 1];
  double d2 = 0.0;
  for (int k = 0; k < S.dim; ++k) {
    const double e = x[k] - pb[k];
    d2 += e * e;
  }
  const double t = sqrt(d2) / r;
  double u3 = 0.0, psi = 0.0;
  if (t < 1.0) {
    const double u = 1.0 - t;
    u3 = u * u * u;
    psi = u3 * u * (4.0 * t + 1.0);
  }
  w[i] = -psi;
  w[i + ld] = -20.0 * a * t * t * u3 / r;
  for (int k = 0; k < S.dim; ++k) w[i + (2 + k) * ld] = -20.0 * a * u3 * (x[k] - pb[k]) / (r * r);
}

template <typename T>
struct Faces {
  const T *fx, *fy, *fz;
};
__device__ __forceinline__ Faces<double> faces(const Stencil& S, double) {
  return {S.fx, S.fy, S.fz};
}
__device__ __forceinline__ Faces<float> faces(const Stencil& S, float) {
  return {S.fx32, S.fy32, S.fz32};
}

// MODE 0: y = A x.
// MODE 2: y = b - A x with b = bscale e_bidx (or bscale_arr[z] e_{bidx_arr[z]}), partial
// y^T y.  blockIdx.z selects a column (x + z*ldx, y + z*ldy; partials of column z at
// + z * gridDim.x * gridDim.y).  T is the arithmetic type.
template <typename T, bool VAR, int MODE>
__global__ __launch_bounds__(BS) void k_stencil(Stencil S, const T* __restrict__ diag,
                                                 const T* __restrict__ x0, int64_t ldx,
                                                 T* __restrict__ y0, int64_t ldy, int zc,
                                                 int64_t bidx, double bscale,
                                                 const int64_t* __restrict__ bidx_arr,
                                                 const double* __restrict__ bscale_arr,
                                                 T* __restrict__ partials, const CGState* cg) {
  if (MODE == 2 && bidx_arr) {
    bidx = bidx_arr[blockIdx.z];
    bscale = bscale_arr[blockIdx.z];
  }
  const T* __restrict__ x = x0 + (int64_t)blockIdx.z * ldx;
  T* __restrict__ y = y0 + (int64_t)blockIdx.z * ldy;
  const Faces<T> F = faces(S, T(0));
  const T cx = (T)S.cx, cy = (T)S.cy, cz = (T)S.cz;
  const int nxy = S.nx * S.ny;
  const int q = blockIdx.x * BS + threadIdx.x;
  const bool active = q < nxy;
  const int ix = active ? q % S.nx : 0;
  const int iy = active ? q / S.nx : 0;
  const int z0 = blockIdx.y * zc;
  const int z1 = min(z0 + zc, S.nz);
  T acc[1] = {T(0)};
  if (active && z0 < z1) {
    const bool hl = ix > 0, hr = ix < S.nx - 1, hd = iy > 0, hu = iy < S.ny - 1;
    int64_t i = (int64_t)z0 * nxy + q;
    T xm = z0 > 0 ? x[i - nxy] : T(0);
    T fm = T(0);
    if (VAR && z0 > 0) fm = F.fz[i - nxy];
    T xc = x[i];
    for (int z = z0; z < z1; ++z, i += nxy) {
      const T xp = z < S.nz - 1 ? x[i + nxy] : T(0);
      T v = diag[i] * xc;
      if (!VAR) {
        const T sx = (hl ? x[i - 1] : T(0)) + (hr ? x[i + 1] : T(0));
        const T sy = (hd ? x[i - S.nx] : T(0)) + (hu ? x[i + S.nx] : T(0));
        v -= cx * sx + cy * sy + cz * (xm + xp);
      } else {
        if (hl) v -= F.fx[i - 1] * x[i - 1];
        if (hr) v -= F.fx[i] * x[i + 1];
        if (hd) v -= F.fy[i - S.nx] * x[i - S.nx];
        if (hu) v -= F.fy[i] * x[i + S.nx];
        if (S.dim == 3) {
          const T fp = F.fz[i];
          v -= fm * xm + fp * xp;
          fm = fp;
        }
      }
      if (MODE == 2) {
        v = -v;
        if (i == bidx) v += (T)bscale;
        acc[0] += v * v;
      }
      y[i] = v;
      xm = xc;
      xc = xp;
    }
  }
  if (MODE != 0)
    write_partials<1, BS>(acc, partials + (int64_t)blockIdx.z * gridDim.x * gridDim.y,
                          blockIdx.x + gridDim.x * blockIdx.y);
}

// One step of a three-term (Chebyshev) recurrence on k columns, fused with the product:
// out[:, v] = a (A x[:, v]) + b x[:, v] + c prev[:, v] (prev may be NULL).  out may alias
// prev (each element of prev is read by the thread that then writes it); neither may alias
// x.  Same launch shape as k_stencil (blockIdx.z = column), so x is fetched about once.
template <bool VAR>
__global__ __launch_bounds__(BS) void k_cheb_step(Stencil S, const double* __restrict__ diag,
                                                   const double* __restrict__ x0, int64_t ld,
                                                   double a, double b, double c,
                                                   const double* prev0, double* out0, int zc) {
  const double* __restrict__ x = x0 + (int64_t)blockIdx.z * ld;
  const double* prev = prev0 ? prev0 + (int64_t)blockIdx.z * ld : nullptr;
  double* out = out0 + (int64_t)blockIdx.z * ld;
  const int q = blockIdx.x * BS + threadIdx.x;
  if (q >= S.nx * S.ny) return;
  const int z0 = blockIdx.y * zc;
  const int z1 = min(z0 + zc, S.nz);
  stencil_walk<VAR>(S, diag, x, q, z0, z1, [&](int64_t i, double ax, double xi) {
    double r = a * ax + b * xi;
    if (prev) r += c * prev[i];
    out[i] = r;
  });
}

// Y = A X for several columns with two consecutive x-nodes per thread (stencil_walk2: even
// nx, 16-byte aligned columns), which halves the memory instructions per node of the
// one-node walk.  Columns on blockIdx.z; z planes in chunks of zc.
template <bool VAR>
__global__ __launch_bounds__(BS) void k_spmm2(Stencil S, const double* __restrict__ diag,
                                               const double* __restrict__ x0, int64_t ld,
                                               double* __restrict__ y0, int zc) {
  const double* __restrict__ x = x0 + (int64_t)blockIdx.z * ld;
  double* __restrict__ y = y0 + (int64_t)blockIdx.z * ld;
  const int q = blockIdx.x * BS + threadIdx.x;
  if (q >= (S.nx / 2) * S.ny) return;
  const int z0 = blockIdx.y * zc, z1 = min(z0 + zc, S.nz);
  if (z0 >= z1) return;
  stencil_walk2<VAR>(S, diag, x, q, z0, z1, [&](int64_t i, double v0, double v1, double, double) {
    *reinterpret_cast<double2*>(y + i) = double2{v0, v1};
  });
}

// Y = A X with LDS-staged x-y tiles (2.5D blocking): a block owns TY = 256 / (nx / 2) full
// rows of the grid (two x-nodes per thread, nx even, nx <= 512) over a chunk of zc planes,
// for C columns, and walks the planes; each plane's tile rows and the two rows next to the
// tile are staged in LDS for every column (two buffers, one barrier per plane), so the
// lateral neighbours come from LDS, the z neighbours stay in registers, and the diagonal and
// the face coefficients (D field) are read once per node for all C columns.  The launch is
// one-dimensional: block b takes tile b % ntiles, z chunk (b / ntiles) % nzc and column
// group b / (ntiles nzc).  (Giving each XCD a contiguous run of tiles, so that its own L2
// would serve the rows two tiles share, measured no faster.)
template <bool VAR, int C>
__global__ __launch_bounds__(BS) void k_spmm_lds(Stencil S, const double* __restrict__ diag,
                                                  const double* __restrict__ x0, int64_t ld,
                                                  int k, double* __restrict__ y0, int zc,
                                                  int ntiles, int nzc) {
  extern __shared__ double2 smem[];
  const int PR = S.nx / 2;            // pairs per row
  const int TY = BS / PR;             // rows per tile
  const int TT = (TY + 2) * PR;       // pairs of one staged plane tile
  const int lg = blockIdx.x;
  const int tile = lg % ntiles;
  const int zch = (lg / ntiles) % nzc;
  const int c0 = (lg / ntiles / nzc) * C;
  const int nc = min(C, k - c0);
  const int t = threadIdx.x;
  const int px = t % PR, ry = t / PR;
  const int y0r = tile * TY;          // first row of the tile
  const int iy = y0r + ry;
  const bool own = ry < TY && iy < S.ny;
  const int z0 = zch * zc, z1 = min(z0 + zc, S.nz);
  if (z0 >= z1 || nc <= 0) return;
  const int nxy = S.nx * S.ny;
  auto ld2 = [](const double* p, int64_t j) { return *reinterpret_cast<const double2*>(p + j); };
  const double2 zero = {0.0, 0.0};
  const double* x[C];
  double* y[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int64_t col = c0 + (c < nc ? c : 0);   // columns past k alias the first (never stored)
    x[c] = x0 + col * ld;
    y[c] = y0 + col * ld;
  }
  int64_t i = (int64_t)z0 * nxy + (int64_t)iy * S.nx + 2 * px;
  double2 xm[C], xc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    xm[c] = (own && z0 > 0) ? ld2(x[c], i - nxy) : zero;
    xc[c] = own ? ld2(x[c], i) : zero;
  }
  double2 fm = (VAR && own && z0 > 0) ? ld2(S.fz, i - nxy) : zero;
  const bool hl = px > 0, hd = iy > 0;
  const double cx = S.cx, cy = S.cy, cz = S.cz;
  int buf = 0;
  for (int z = z0; z < z1; ++z, i += nxy) {
    double2* T = smem + (size_t)buf * C * TT;
#pragma unroll
    for (int c = 0; c < C; ++c)
      if (ry < TY) T[c * TT + (ry + 1) * PR + px] = xc[c];   // zero for rows past the grid
    // the rows below and above the tile (zero outside the grid)
    for (int h = t; h < 2 * PR; h += BS) {
      const int hr = h / PR, hx = h % PR;
      const int hy = hr == 0 ? y0r - 1 : y0r + TY;
      const bool in = hy >= 0 && hy < S.ny;
      const int64_t j = (int64_t)z * nxy + (int64_t)hy * S.nx + 2 * hx;
#pragma unroll
      for (int c = 0; c < C; ++c)
        T[c * TT + (hr == 0 ? 0 : TY + 1) * PR + hx] = in ? ld2(x[c], j) : zero;
    }
    double2 xp[C];
#pragma unroll
    for (int c = 0; c < C; ++c) xp[c] = (own && z < S.nz - 1) ? ld2(x[c], i + nxy) : zero;
    const double2 d = own ? ld2(diag, i) : zero;
    double fxl = 0.0;
    double2 fx = zero, fyd = zero, fyu = zero, fp = zero;
    if (VAR && own) {
      fxl = hl ? S.fx[i - 1] : 0.0;
      fx = ld2(S.fx, i);
      fyd = hd ? ld2(S.fy, i - S.nx) : zero;
      fyu = ld2(S.fy, i);
      fp = ld2(S.fz, i);
    }
    __syncthreads();
    if (own) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        if (c >= nc) break;
        const double2* Tc = T + c * TT;
        const double2 yd = Tc[ry * PR + px], yu = Tc[(ry + 2) * PR + px];
        const double xl = hl ? Tc[(ry + 1) * PR + px - 1].y : 0.0;
        const double xr = px < PR - 1 ? Tc[(ry + 1) * PR + px + 1].x : 0.0;
        double v0 = d.x * xc[c].x, v1 = d.y * xc[c].y;
        if (!VAR) {
          v0 -= cx * (xl + xc[c].y) + cy * (yd.x + yu.x) + cz * (xm[c].x + xp[c].x);
          v1 -= cx * (xc[c].x + xr) + cy * (yd.y + yu.y) + cz * (xm[c].y + xp[c].y);
        } else {
          v0 -= fxl * xl + fx.x * xc[c].y;
          v1 -= fx.x * xc[c].x + fx.y * xr;
          v0 -= fyd.x * yd.x + fyu.x * yu.x;
          v1 -= fyd.y * yd.y + fyu.y * yu.y;
          v0 -= fm.x * xm[c].x + fp.x * xp[c].x;
          v1 -= fm.y * xm[c].y + fp.y * xp[c].y;
        }
        *reinterpret_cast<double2*>(y[c] + i) = double2{v0, v1};
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      xm[c] = xc[c];
      xc[c] = xp[c];
    }
    if (VAR) fm = fp;
    buf ^= 1;
  }
}

// k_spmm2 with C columns per thread (blockIdx.z = group of C columns, the last group
// possibly partial): the diagonal and, with a D field, the face coefficients are loaded once
// per node pair for all C columns instead of once per column.  Same arithmetic per column
// as stencil_walk2.
template <bool VAR, int C>
__global__ __launch_bounds__(BS) void k_spmm2c(Stencil S, const double* __restrict__ diag,
                                                const double* __restrict__ x0, int64_t ld, int k,
                                                double* __restrict__ y0, int zc) {
  const int hx = S.nx / 2;
  const int q = blockIdx.x * BS + threadIdx.x;
  if (q >= hx * S.ny) return;
  const int z0 = blockIdx.y * zc, z1 = min(z0 + zc, S.nz);
  if (z0 >= z1) return;
  const int c0 = blockIdx.z * C;
  const int nc = min(C, k - c0);
  const int ix = 2 * (q % hx), iy = q / hx;
  const int nxy = S.nx * S.ny;
  const bool hl = ix > 0, hr = ix + 2 < S.nx, hd = iy > 0, hu = iy < S.ny - 1;
  const double2 zero = {0.0, 0.0};
  auto ld2 = [](const double* p, int64_t j) { return *reinterpret_cast<const double2*>(p + j); };
  const double* x[C];
  double* y[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int64_t col = c0 + (c < nc ? c : 0);   // columns past k alias the first (never stored)
    x[c] = x0 + col * ld;
    y[c] = y0 + col * ld;
  }
  int64_t i = (int64_t)z0 * nxy + (int64_t)iy * S.nx + ix;
  double2 xm[C], xc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    xm[c] = z0 > 0 ? ld2(x[c], i - nxy) : zero;
    xc[c] = ld2(x[c], i);
  }
  double2 fm = (VAR && z0 > 0) ? ld2(S.fz, i - nxy) : zero;
  for (int z = z0; z < z1; ++z, i += nxy) {
    const double2 d = ld2(diag, i);
    double fxl = 0.0;
    double2 fx = zero, fyd = zero, fyu = zero, fp = zero;
    if (VAR) {
      fxl = hl ? S.fx[i - 1] : 0.0;
      fx = ld2(S.fx, i);
      fyd = hd ? ld2(S.fy, i - S.nx) : zero;
      fyu = ld2(S.fy, i);
      if (S.dim == 3) fp = ld2(S.fz, i);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (c >= nc) break;
      const double2 xp = z < S.nz - 1 ? ld2(x[c], i + nxy) : zero;
      const double xl = hl ? x[c][i - 1] : 0.0;
      const double xr = hr ? x[c][i + 2] : 0.0;
      const double2 yd = hd ? ld2(x[c], i - S.nx) : zero;
      const double2 yu = hu ? ld2(x[c], i + S.nx) : zero;
      double v0 = d.x * xc[c].x, v1 = d.y * xc[c].y;
      if (!VAR) {
        v0 -= S.cx * (xl + xc[c].y) + S.cy * (yd.x + yu.x) + S.cz * (xm[c].x + xp.x);
        v1 -= S.cx * (xc[c].x + xr) + S.cy * (yd.y + yu.y) + S.cz * (xm[c].y + xp.y);
      } else {
        v0 -= fxl * xl + fx.x * xc[c].y;
        v1 -= fx.x * xc[c].x + fx.y * xr;
        v0 -= fyd.x * yd.x + fyu.x * yu.x;
        v1 -= fyd.y * yd.y + fyu.y * yu.y;
        if (S.dim == 3) {
          v0 -= fm.x * xm[c].x + fp.x * xp.x;
          v1 -= fm.y * xm[c].y + fp.y * xp.y;
        }
      }
      *reinterpret_cast<double2*>(y[c] + i) = double2{v0, v1};
      xm[c] = xc[c];
      xc[c] = xp;
    }
    if (VAR) fm = fp;
  }
}

// k_cheb_step with two x-nodes per thread (the same conditions as k_spmm2).
template <bool VAR>
__global__ __launch_bounds__(BS) void k_cheb_step2(Stencil S, const double* __restrict__ diag,
                                                    const double* __restrict__ x0, int64_t ld,
                                                    double a, double b, double c,
                                                    const double* prev0, double* out0, int zc) {
  const double* __restrict__ x = x0 + (int64_t)blockIdx.z * ld;
  const double* prev = prev0 ? prev0 + (int64_t)blockIdx.z * ld : nullptr;
  double* out = out0 + (int64_t)blockIdx.z * ld;
  const int q = blockIdx.x * BS + threadIdx.x;
  if (q >= (S.nx / 2) * S.ny) return;
  const int z0 = blockIdx.y * zc, z1 = min(z0 + zc, S.nz);
  if (z0 >= z1) return;
  stencil_walk2<VAR>(S, diag, x, q, z0, z1,
                     [&](int64_t i, double v0, double v1, double x0i, double x1i) {
                       double r0 = a * v0 + b * x0i, r1 = a * v1 + b * x1i;
                       if (prev) {
                         const double2 pv = *reinterpret_cast<const double2*>(prev + i);
                         r0 += c * pv.x;
                         r1 += c * pv.y;
                       }
                       *reinterpret_cast<double2*>(out + i) = double2{r0, r1};
                     });
}

// out[z * ostride] = sum_b partials[z * P + b], one block per column z.
__global__ void k_reduce_cols(const double* __restrict__ partials, int P, double* out,
                              int64_t ostride) {
  __shared__ double tot[1];
  sum_partials<1, BS>(partials + (int64_t)blockIdx.x * P, P, tot);
  if (threadIdx.x == 0) out[blockIdx.x * ostride] = tot[0];
}

template <int R>
__global__ void k_reduce_finish(const double* __restrict__ partials, int P, double* out,
                                Skip skip) {
  if (skip.on()) return;
  __shared__ double tot[R];
  sum_partials<R, BS>(partials, P, tot);
  if (threadIdx.x < R) out[threadIdx.x] = tot[threadIdx.x];
}

}  // namespace

StencilShape stencil_shape(const Stencil& S, int target_blocks) {
  StencilShape sh;
  const int nxy = S.nx * S.ny;
  const int gx = ceil_div(nxy, BS);
  int nzc = (target_blocks + gx - 1) / gx;
  if (nzc < 1) nzc = 1;
  if (nzc > S.nz) nzc = S.nz;
  sh.zc = (S.nz + nzc - 1) / nzc;
  nzc = (S.nz + sh.zc - 1) / sh.zc;
  sh.grid = dim3(gx, nzc, 1);
  sh.blocks = gx * nzc;
  return sh;
}

void launch_assemble(const rom_grid& g, double D_const, const double* D, double* diag_star,
                     double* fx, double* fy, double* fz, hipStream_t st) {
  int64_t n = (int64_t)g.n[0] * g.n[1] * g.n[2];
  ROM_LAUNCH(k_assemble, dim3(ceil_div(n, BS)), dim3(BS), 0, st, g, D_const, D, n,
                     diag_star, fx, fy, fz);
  ROM_CHECK_LAUNCH();
}

void launch_mu_eval(const Stencil& S, const Bumps& bumps, const double* diag_star,
                    double* diag_i, double* dmu, hipStream_t st) {
  ROM_LAUNCH(k_mu_eval, dim3(ceil_div(S.n, BS)), dim3(BS), 0, st, S, bumps, diag_star,
                     diag_i, dmu);
  ROM_CHECK_LAUNCH();
}

#define STENCIL_LAUNCH(T, MODE, grid, ...)                                                     \
  do {                                                                                         \
    if (S.var)                                                                                 \
      ROM_LAUNCH((k_stencil<T, true, MODE>), grid, dim3(BS), 0, st, S, __VA_ARGS__);           \
    else                                                                                       \
      ROM_LAUNCH((k_stencil<T, false, MODE>), grid, dim3(BS), 0, st, S, __VA_ARGS__);          \
  } while (0)

void launch_mu_grad(const Stencil& S, const Bumps& bumps, int b, double* w, int64_t ld,
                    hipStream_t st) {
  ROM_LAUNCH(k_mu_grad, dim3(ceil_div(S.n, BS)), dim3(BS), 0, st, S, bumps, b, w, ld);
  ROM_CHECK_LAUNCH();
}

void launch_spmv(const Stencil& S, const double* diag, const double* x, double* y,
                 hipStream_t st) {
  const StencilShape sh = stencil_shape(S, 1024);
  STENCIL_LAUNCH(double, 0, sh.grid, diag, x, 0, y, 0, sh.zc, (int64_t)-1, 0.0,
                 (const int64_t*)nullptr, (const double*)nullptr, (double*)nullptr,
                 (const CGState*)nullptr);
}

// Columns per thread of the two-node SpMM (1, 2, 4 or 8), at most k.
static int spmm_cols_per_thread(const Stencil& S, int k) {
  int c = S.var ? SPMM_CPT_VAR : SPMM_CPT_CONST;
  while (c > 1 && c > k) c /= 2;
  return c;
}

void launch_spmm(const Stencil& S, const double* diag, const double* X, int64_t ld, int k,
                 double* Y, hipStream_t st) {
  if (k <= 0) return;
  StencilShape sh = stencil_shape(S, 512);
  dim3 grid = sh.grid;
  grid.z = k;
  if (S.dim == 3 && S.nx <= 2 * BS && stencil_pairs_ok(S, ld, {X, Y, diag})) {
    // LDS tiles of full rows, C columns per block; z chunks so that the launch has about
    // `target` blocks
    const int ty = BS / (S.nx / 2);
    const size_t tile = sizeof(double2) * 2 * (size_t)(ty + 2) * (S.nx / 2);   // per column
    int C = S.var ? SPMM_LDS_C_VAR : SPMM_LDS_C_CONST;
    while (C > 1 && tile * C > SPMM_LDS_MAX) C /= 2;
    const int64_t target = S.var ? SPMM_LDS_BLOCKS_VAR : SPMM_LDS_BLOCKS_CONST;
    if (tile * C <= SPMM_LDS_MAX) {
      const int ntiles = ceil_div(S.ny, ty);
      const int ncg = ceil_div(k, C);
      const int64_t base = (int64_t)ntiles * ncg;
      int nzc = (int)std::min<int64_t>(S.nz,
                                       std::max<int64_t>(1, (target + base - 1) / base));
      const int zc = ceil_div(S.nz, nzc);
      nzc = ceil_div(S.nz, zc);
      const int64_t blocks = base * nzc;
      if (blocks > 2147483647LL) throw Error(ROM_EINVAL, "spmm: grid too large");
      const dim3 g((unsigned)blocks);
#define SPL(V, CC)                                                                             \
  ROM_LAUNCH((k_spmm_lds<V, CC>), g, dim3(BS), tile * CC, st, S, diag, X, ld, k, Y, zc, ntiles, \
             nzc)
      if (S.var) {
        if (C == 4) SPL(true, 4); else if (C == 2) SPL(true, 2); else SPL(true, 1);
      } else {
        if (C == 4) SPL(false, 4); else if (C == 2) SPL(false, 2); else SPL(false, 1);
      }
#undef SPL
      ROM_CHECK_LAUNCH();
      return;
    }
  }
  if (stencil_pairs_ok(S, ld, {X, Y, diag})) {
    grid.x = ceil_div((int64_t)(S.nx / 2) * S.ny, BS);
    const int C = spmm_cols_per_thread(S, k);   // > 1 only with a D field
    if (C > 1) {
      grid.z = ceil_div(k, C);
#define SPMMC(CC) ROM_LAUNCH((k_spmm2c<true, CC>), grid, dim3(BS), 0, st, S, diag, X, ld, k, Y, sh.zc)
      if (C == 8) SPMMC(8); else if (C == 4) SPMMC(4); else SPMMC(2);
#undef SPMMC
    } else if (S.var) {
      ROM_LAUNCH(k_spmm2<true>, grid, dim3(BS), 0, st, S, diag, X, ld, Y, sh.zc);
    } else {
      ROM_LAUNCH(k_spmm2<false>, grid, dim3(BS), 0, st, S, diag, X, ld, Y, sh.zc);
    }
    ROM_CHECK_LAUNCH();
    return;
  }
  STENCIL_LAUNCH(double, 0, grid, diag, X, ld, Y, ld, sh.zc, (int64_t)-1, 0.0,
                 (const int64_t*)nullptr, (const double*)nullptr, (double*)nullptr,
                 (const CGState*)nullptr);
}

void launch_cheb_step(const Stencil& S, const double* diag, const double* X, int64_t ld, int k,
                      double a, double b, double c, const double* prev, double* out,
                      hipStream_t st) {
  if (k <= 0) return;
  StencilShape sh = stencil_shape(S, 512);
  dim3 grid = sh.grid;
  grid.z = k;
  if (stencil_pairs_ok(S, ld, {X, diag, prev, out})) {
    grid.x = ceil_div((int64_t)(S.nx / 2) * S.ny, BS);
    if (S.var)
      ROM_LAUNCH(k_cheb_step2<true>, grid, dim3(BS), 0, st, S, diag, X, ld, a, b, c, prev, out,
                 sh.zc);
    else
      ROM_LAUNCH(k_cheb_step2<false>, grid, dim3(BS), 0, st, S, diag, X, ld, a, b, c, prev, out,
                 sh.zc);
    ROM_CHECK_LAUNCH();
    return;
  }
  if (S.var)
    ROM_LAUNCH(k_cheb_step<true>, grid, dim3(BS), 0, st, S, diag, X, ld, a, b, c, prev, out,
               sh.zc);
  else
    ROM_LAUNCH(k_cheb_step<false>, grid, dim3(BS), 0, st, S, diag, X, ld, a, b, c, prev, out,
               sh.zc);
  ROM_CHECK_LAUNCH();
}

void launch_resid_unit(const Stencil& S, const double* diag, const double* x, int64_t idx,
                       double scale, double* r, double* nrm2, double* partials,
                       hipStream_t st) {
  const StencilShape sh = stencil_shape(S, 512);
  STENCIL_LAUNCH(double, 2, sh.grid, diag, x, 0, r, 0, sh.zc, idx, scale,
                 (const int64_t*)nullptr, (const double*)nullptr, partials,
                 (const CGState*)nullptr);
  launch_reduce_finish(partials, sh.blocks, 1, nrm2, st);
}

template <typename T>
StencilShape cg_apply_shape(const Stencil& S, int target_blocks, const T* diag, const T* p,
                            const T* w, int64_t vstride, const T* AW, bool quads) {
  StencilShape sh = stencil_shape(S, target_blocks);
  if (quads && sizeof(T) == 4 && stencil_quads_ok(S, vstride, {diag, p, w, AW})) {
    sh.grid.x = ceil_div((int64_t)(S.nx / 4) * S.ny, BS);
    sh.blocks = (int)(sh.grid.x * sh.grid.y);
    sh.quads = 1;
  } else if (stencil_pairs_ok(S, vstride, {diag, p, w, AW}, sizeof(T) == 4)) {
    sh.grid.x = ceil_div((int64_t)(S.nx / 2) * S.ny, BS);
    sh.blocks = (int)(sh.grid.x * sh.grid.y);
    sh.pairs = 1;
  }
  return sh;
}
template StencilShape cg_apply_shape<double>(const Stencil&, int, const double*, const double*,
                                             const double*, int64_t, const double*, bool);
template StencilShape cg_apply_shape<float>(const Stencil&, int, const float*, const float*,
                                            const float*, int64_t, const float*, bool);

void launch_resid_cols(const Stencil& S, const double* diag, const double* X, int64_t ldx, int nb,
                       const int64_t* idx, const double* scale, double* R, int64_t ldr,
                       double* nrm2, int64_t nstride, double* partials, hipStream_t st) {
  if (nb <= 0) return;
  const StencilShape sh = stencil_shape(S, 512);
  const dim3 grid(sh.grid.x, sh.grid.y, nb);
  STENCIL_LAUNCH(double, 2, grid, diag, X, ldx, R, ldr, sh.zc, (int64_t)-1, 0.0, idx, scale,
                 partials, (const CGState*)nullptr);
  ROM_LAUNCH(k_reduce_cols, dim3(nb), dim3(BS), 0, st, partials, sh.blocks, nrm2, nstride);
  ROM_CHECK_LAUNCH();
}

void launch_reduce_finish(const double* partials, int P, int R, double* out, hipStream_t st,
                          Skip skip) {
  if (R == 1)
    ROM_LAUNCH(k_reduce_finish<1>, dim3(1), dim3(BS), 0, st, partials, P, out, skip);
  else if (R == 2)
    ROM_LAUNCH(k_reduce_finish<2>, dim3(1), dim3(BS), 0, st, partials, P, out, skip);
  else
    throw Error(ROM_EINVAL, "reduce_finish: R must be 1 or 2");
  ROM_CHECK_LAUNCH();
}

}  // namespace rom
