// Kernels of the learned-seed network (a small 3D convolutional network in BF16 with
// FP32 accumulation; not part of the paper).  Activations are stored voxel-major with
// the channels contiguous: X[v][c], v = x + nx (y + ny (z + nz b)) over a batch of grids,
// c < Cp (Cp a multiple of 8; padded channels hold zeros).  A 3x3x3 convolution with zero
// padding is an implicit GEMM
//     Y[v][o] = sum_k A[v][k] W[o][k],   k = tap * Cp_in + c,  A[v][k] = X[nbr(v, tap)][c],
// evaluated on the matrix cores (v_mfma_f32_16x16x32_bf16: a wave owns 16 voxels and
// 16-channel output tiles; the 8 consecutive k a lane supplies lie in one tap, so its A
// operand is one 16-byte load of a neighbour's channels).  The data gradient is the same
// convolution with the weights flipped in space and transposed in channels; the weight
// gradient reduces over voxels in LDS-staged 32-voxel steps, split over voxel chunks.
#include <algorithm>

#include "kernels.h"

namespace rom {

namespace {

constexpr int BS = 256;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

struct Grid3 {
  int nx, ny, nz, batch;
};

// Convolution: Y = act(conv(X; W) + bias + skip).  W: [cop16][Kp] BF16 (zero beyond K =
// 27 Cpi and beyond Cout), NT = cop16 / 16 output tiles.  Writes channels < Cpo of Y
// (zeros for Cout <= c < Cpo).  A wave owns VT tiles of 16 voxels, so each weight load
// feeds VT MFMAs; a lane decomposes its voxels into (x, y, z) once and follows its tap
// and channel through the k loop by increments (no divisions inside the loop).  up != 0:
// X lives on the grid of half the size and the convolution reads its 2x nearest-neighbour
// upsampling (fine voxel (x, y, z) takes coarse voxel (x/2, y/2, z/2)) without forming it.
template <int NT, int VT>
__global__ __launch_bounds__(BS) void k_conv(Grid3 g, const __bf16* __restrict__ X, int Cpi,
                                             const __bf16* __restrict__ W, int Kp, int Cout,
                                             const float* __restrict__ bias,
                                             const __bf16* __restrict__ skip, int relu,
                                             __bf16* __restrict__ Y, int Cpo, int up) {
  const int64_t nv = (int64_t)g.nx * g.ny * g.nz * g.batch;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t v0 = ((int64_t)blockIdx.x * (BS / WAVE) + wid) * (16 * VT);
  const int kg = lane >> 4;              // which 8 of the 32 k of a step
  const int K = 27 * Cpi;
  const int64_t sy = g.nx, sz = (int64_t)g.nx * g.ny;
  const int cx = g.nx >> 1, cy = g.ny >> 1, cz = g.nz >> 1;   // the coarse grid (up)
  int64_t va[VT], cb[VT];
  int vx[VT], vy[VT], vz[VT];
  bool rowok[VT];
#pragma unroll
  for (int u = 0; u < VT; ++u) {
    va[u] = v0 + 16 * u + (lane & 15);
    rowok[u] = va[u] < nv;
    const int64_t v = rowok[u] ? va[u] : 0;
    vx[u] = (int)(v % g.nx);
    const int64_t r = v / g.nx;
    vy[u] = (int)(r % g.ny);
    const int64_t r2 = r / g.ny;
    vz[u] = (int)(r2 % g.nz);
    cb[u] = (r2 / g.nz) * cz;   // batch offset in coarse planes
  }
  float4_t acc[VT][NT];
#pragma unroll
  for (int u = 0; u < VT; ++u)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[u][t] = (float4_t){0.f, 0.f, 0.f, 0.f};
  int tap = (8 * kg) / Cpi, c = (8 * kg) % Cpi;
  for (int k0 = 0; k0 < Kp; k0 += 32) {
    const int k = k0 + 8 * kg;
    const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
    const int64_t off = dx + sy * dy + sz * dz;
    bf16x8 a[VT];
#pragma unroll
    for (int u = 0; u < VT; ++u) {
#pragma unroll
      for (int q = 0; q < 8; ++q) a[u][q] = (__bf16)0.f;
      const int xx = vx[u] + dx, yy = vy[u] + dy, zz = vz[u] + dz;
      if (rowok[u] && k < K && xx >= 0 && xx < g.nx && yy >= 0 && yy < g.ny && zz >= 0 &&
          zz < g.nz) {
        const int64_t src =
            up ? (((cb[u] + (zz >> 1)) * cy + (yy >> 1)) * cx + (xx >> 1)) : va[u] + off;
        a[u] = *reinterpret_cast<const bf16x8*>(X + src * Cpi + c);
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(W + (int64_t)(16 * t + (lane & 15)) * Kp + k);
#pragma unroll
      for (int u = 0; u < VT; ++u)
        acc[u][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u], b, acc[u][t], 0, 0, 0);
    }
    c += 32;
    while (c >= Cpi) {
      c -= Cpi;
      ++tap;
    }
  }
  // D layout: register r of a lane holds row 4 (lane / 16) + r, column lane % 16
#pragma unroll
  for (int u = 0; u < VT; ++u)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int o = 16 * t + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t v = v0 + 16 * u + 4 * kg + r;
        if (v >= nv || o >= Cpo) continue;
        float val = 0.f;
        if (o < Cout) {
          val = acc[u][t][r] + (bias ? bias[o] : 0.f);
          if (skip) val += (float)skip[v * Cpo + o];
          if (relu) val = fmaxf(val, 0.f);
        }
        Y[v * Cpo + o] = (__bf16)val;
      }
    }
}

// k_conv with the input staged in LDS: a block owns a box of 16 x 4 x BZ voxels (4 BZ tiles
// of 16 consecutive x; wave w computes tiles BZ w .. BZ w + BZ - 1 for all NT output tiles)
// and first stages the box with its one-voxel halo (18 x 6 x (BZ + 2) voxels, all Cpi
// channels, each voxel's channels padded by 8 to spread the LDS banks; zeros outside the
// grid; with up the coarse voxel each fine halo voxel takes).  The 27 taps then read their
// A operands from LDS instead of gathering them through the caches; each step's LDS and
// weight loads are issued one step ahead.  Needs nx % 16 == 0, ny % 4 == 0, nz % BZ == 0
// (boxes stay inside one grid of the batch).
constexpr int CB_X = 16, CB_Y = 4;
constexpr int CH_X = CB_X + 2, CH_Y = CB_Y + 2;
constexpr int conv_halo_vox(int bz) { return CH_X * CH_Y * (bz + 2); }
template <int NT, int BZ>
__global__ __launch_bounds__(BS) void k_conv_lds(Grid3 g, const __bf16* __restrict__ X, int Cpi,
                                                 const __bf16* __restrict__ W, int Kp, int Cout,
                                                 const float* __restrict__ bias,
                                                 const __bf16* __restrict__ skip, int relu,
                                                 __bf16* __restrict__ Y, int Cpo, int up) {
  extern __shared__ __bf16 halo[];
  const int cs = Cpi + 8;   // LDS stride of one voxel (elements)
  const int bxn = g.nx / CB_X, byn = g.ny / CB_Y;
  const int bx = blockIdx.x % bxn, by = (blockIdx.x / bxn) % byn;
  const int bzb = blockIdx.x / (bxn * byn);           // box along z over the batch
  constexpr int CB_Z = BZ, CH_Z = BZ + 2, CH_VOX = CH_X * CH_Y * CH_Z;
  const int zpb = g.nz / CB_Z;                        // boxes per grid along z
  const int b = bzb / zpb;                            // grid of the batch
  const int X0 = bx * CB_X, Y0 = by * CB_Y, Z0 = (bzb % zpb) * CB_Z;
  const int64_t sy = g.nx, sz = (int64_t)g.nx * g.ny;
  const int64_t gbase = (int64_t)b * g.nz * sz;       // first voxel of grid b
  const int cx = g.nx >> 1, cy = g.ny >> 1, cz = g.nz >> 1;
  // stage the halo box: Cpi / 8 16-byte chunks per voxel
  const int chunks = Cpi / 8;
  for (int e = threadIdx.x; e < CH_VOX * chunks; e += BS) {
    const int h = e / chunks, q = e % chunks;
    const int hx = h % CH_X, hy = (h / CH_X) % CH_Y, hz = h / (CH_X * CH_Y);
    const int xx = X0 + hx - 1, yy = Y0 + hy - 1, zz = Z0 + hz - 1;
    bf16x8 v;
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = (__bf16)0.f;
    if (xx >= 0 && xx < g.nx && yy >= 0 && yy < g.ny && zz >= 0 && zz < g.nz) {
      const int64_t src = up ? ((((int64_t)b * cz + (zz >> 1)) * cy + (yy >> 1)) * cx + (xx >> 1))
                             : gbase + xx + sy * yy + sz * zz;
      v = *reinterpret_cast<const bf16x8*>(X + src * Cpi + 8 * q);
    }
    *reinterpret_cast<bf16x8*>(halo + h * cs + 8 * q) = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int kg = lane >> 4;
  const int K = 27 * Cpi;
  constexpr int VT = BZ;
  int hv[VT];   // halo index of this lane's voxel in each of its tiles (tap 0, 0, 0)
#pragma unroll
  for (int u = 0; u < VT; ++u) {
    const int t = VT * wid + u;
    const int vx = lane & 15, vy = t % CB_Y, vz = t / CB_Y;
    hv[u] = (vx + 1) + CH_X * ((vy + 1) + CH_Y * (vz + 1));
  }
  float4_t acc[VT][NT];
#pragma unroll
  for (int u = 0; u < VT; ++u)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[u][t] = (float4_t){0.f, 0.f, 0.f, 0.f};
  // the operands of step k0 (this lane's 8 k from tap, channel c), loaded one step ahead
  // so that the next step's LDS and weight loads are in flight during this step's MFMAs
  auto load_step = [&](int k0, int tp, int cc, bf16x8 (&a)[VT], bf16x8 (&bw)[NT]) {
    const int k = k0 + 8 * kg;
    const int dz = tp / 9 - 1, dy = (tp / 3) % 3 - 1, dx = tp % 3 - 1;
    const int off = dx + CH_X * (dy + CH_Y * dz);
#pragma unroll
    for (int u = 0; u < VT; ++u) {
      if (k < K) {
        a[u] = *reinterpret_cast<const bf16x8*>(halo + (hv[u] + off) * cs + cc);
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) a[u][q] = (__bf16)0.f;
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
      bw[t] = *reinterpret_cast<const bf16x8*>(W + (int64_t)(16 * t + (lane & 15)) * Kp + k);
  };
  int tap = (8 * kg) / Cpi, c = (8 * kg) % Cpi;
  bf16x8 a[VT], bw[NT];
  load_step(0, tap, c, a, bw);
  for (int k0 = 0; k0 < Kp; k0 += 32) {
    c += 32;
    while (c >= Cpi) {
      c -= Cpi;
      ++tap;
    }
    bf16x8 an[VT], bn[NT];
    if (k0 + 32 < Kp) load_step(k0 + 32, tap, c, an, bn);
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int u = 0; u < VT; ++u)
        acc[u][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u], bw[t], acc[u][t], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < VT; ++u) a[u] = an[u];
#pragma unroll
    for (int t = 0; t < NT; ++t) bw[t] = bn[t];
  }
  // D layout: register r of a lane holds row 4 (lane / 16) + r (the voxel's x in its
  // tile), column lane % 16 (the output channel in its tile)
#pragma unroll
  for (int u = 0; u < VT; ++u) {
    const int t = VT * wid + u;
    const int64_t rowbase = gbase + X0 + sy * (Y0 + t % CB_Y) + sz * (Z0 + t / CB_Y);
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
      const int o = 16 * tt + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t v = rowbase + 4 * kg + r;
        if (o >= Cpo) continue;
        float val = 0.f;
        if (o < Cout) {
          val = acc[u][tt][r] + (bias ? bias[o] : 0.f);
          if (skip) val += (float)skip[v * Cpo + o];
          if (relu) val = fmaxf(val, 0.f);
        }
        Y[v * Cpo + o] = (__bf16)val;
      }
    }
  }
}

// Weight gradient partials: P[chunk][o][k] = sum over the chunk's voxels of
// dZ[v][o] A[v][k] for o in the block's 16-channel tile and k in its 64-wide slice (one
// 16-wide tile per wave); 32 voxels are staged in LDS per step.
constexpr int WG_VOX = 2048;   // voxels per chunk
__global__ __launch_bounds__(BS) void k_conv_wgrad(Grid3 g, const __bf16* __restrict__ X,
                                                   int Cpi, const __bf16* __restrict__ dZ,
                                                   int Cpo, int Kp, float* __restrict__ P,
                                                   int up) {
  __shared__ __bf16 Zs[32][16 + 2];
  __shared__ __bf16 As[32][64 + 8];
  const int64_t nv = (int64_t)g.nx * g.ny * g.nz * g.batch;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int o0 = blockIdx.z * 16;
  const int kb = blockIdx.y * 64;
  const int K = 27 * Cpi;
  const int64_t vbeg = (int64_t)blockIdx.x * WG_VOX;
  const int64_t vend = min<int64_t>(vbeg + WG_VOX, nv);
  float4_t acc = (float4_t){0.f, 0.f, 0.f, 0.f};
  // staging maps: dZ: thread -> (voxel t/8, channels 2 (t%8) .. +1); A: thread -> (voxel
  // t/8, k 8 (t%8) .. +7)
  const int zr = threadIdx.x >> 3, zc = 2 * (threadIdx.x & 7);
  const int ar = threadIdx.x >> 3, ac = 8 * (threadIdx.x & 7);
  // this thread's k (fixed: tap and channel once) and its staged voxel, decomposed once
  // and then advanced by 32 per step
  const int ka = kb + ac;
  const bool kin = ka < K;
  const int tap = kin ? ka / Cpi : 0, ca = kin ? ka % Cpi : 0;
  const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
  const int64_t off = dx + (int64_t)g.nx * (dy + (int64_t)g.ny * dz);
  const int cx = g.nx >> 1, cy = g.ny >> 1, cz = g.nz >> 1;   // the coarse grid (up)
  int ax, ay, az;
  int64_t ab;
  {
    const int64_t v = vbeg + ar;
    ax = (int)(v % g.nx);
    const int64_t r = v / g.nx;
    ay = (int)(r % g.ny);
    const int64_t r2 = r / g.ny;
    az = (int)(r2 % g.nz);
    ab = r2 / g.nz;
  }
  for (int64_t vs = vbeg; vs < vend; vs += 32) {
    {
      const int64_t v = vs + zr;
      __bf16 z0 = (__bf16)0.f, z1 = (__bf16)0.f;
      if (v < vend) {
        if (o0 + zc < Cpo) z0 = dZ[v * Cpo + o0 + zc];
        if (o0 + zc + 1 < Cpo) z1 = dZ[v * Cpo + o0 + zc + 1];
      }
      Zs[zr][zc] = z0;
      Zs[zr][zc + 1] = z1;
    }
    {
      const int64_t v = vs + ar;
      bf16x8 a;
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] = (__bf16)0.f;
      const int xx = ax + dx, yy = ay + dy, zz = az + dz;
      if (v < vend && kin && xx >= 0 && xx < g.nx && yy >= 0 && yy < g.ny && zz >= 0 &&
          zz < g.nz) {
        const int64_t src =
            up ? (((ab * cz + (zz >> 1)) * cy + (yy >> 1)) * cx + (xx >> 1)) : v + off;
        a = *reinterpret_cast<const bf16x8*>(X + src * Cpi + ca);
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) As[ar][ac + q] = a[q];
      ax += 32;
      while (ax >= g.nx) {
        ax -= g.nx;
        if (++ay == g.ny) {
          ay = 0;
          if (++az == g.nz) {
            az = 0;
            ++ab;
          }
        }
      }
    }
    __syncthreads();
    // A operand: A[i = o][kk = voxel]; B operand: B[kk = voxel][j = k]
    bf16x8 am, bm;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      am[q] = Zs[8 * (lane >> 4) + q][lane & 15];
      bm[q] = As[8 * (lane >> 4) + q][16 * wid + (lane & 15)];
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm, acc, 0, 0, 0);
    __syncthreads();
  }
  float* Pc = P + (int64_t)blockIdx.x * (gridDim.z * 16) * Kp;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int o = o0 + 4 * (lane >> 4) + r;
    const int k = kb + 16 * wid + (lane & 15);
    if (k < Kp) Pc[(int64_t)o * Kp + k] = acc[r];
  }
}

// dW[o][k] (+)= sum over chunks of P[chunk][o][k]; bias partials likewise.
__global__ void k_wgrad_reduce(const float* __restrict__ P, int nchunk, int rows, int Kp,
                               float* __restrict__ dW, int accumulate) {
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  const int64_t ne = (int64_t)rows * Kp;
  if (e >= ne) return;
  float s = 0.f;
  for (int c = 0; c < nchunk; ++c) s += P[(int64_t)c * ne + e];
  dW[e] = accumulate ? dW[e] + s : s;
}

// Bias gradient partials: Pb[chunk][o] = sum over the chunk's voxels of dZ[v][o].
__global__ void k_bias_grad(int64_t nv, const __bf16* __restrict__ dZ, int Cpo, int Cout,
                            float* __restrict__ Pb) {
  __shared__ float sh[BS];
  const int o = blockIdx.y;
  float s = 0.f;
  const int64_t vbeg = (int64_t)blockIdx.x * WG_VOX;
  const int64_t vend = min<int64_t>(vbeg + WG_VOX, nv);
  for (int64_t v = vbeg + threadIdx.x; v < vend; v += BS) s += (float)dZ[v * Cpo + o];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = BS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) Pb[(int64_t)blockIdx.x * Cout + o] = sh[0];
}

// 2x2x2 average pooling and its adjoint; 2x nearest upsampling and its adjoint.
// g: the fine grid.  acc: add into the output instead of overwriting.
__global__ void k_pool(Grid3 g, const __bf16* __restrict__ X, __bf16* __restrict__ Y, int C) {
  const int cx = g.nx / 2, cy = g.ny / 2, cz = g.nz / 2;
  const int64_t nc = (int64_t)cx * cy * cz * g.batch;
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (e >= nc * C) return;
  const int c = (int)(e % C);
  const int64_t vc = e / C;
  const int x = (int)(vc % cx);
  const int y = (int)((vc / cx) % cy);
  const int64_t zb = vc / ((int64_t)cx * cy);   // z + cz * b
  const int z = (int)(zb % cz);
  const int64_t b = zb / cz;
  float s = 0.f;
  for (int d = 0; d < 8; ++d) {
    const int64_t v = (2 * x + (d & 1)) +
                      (int64_t)g.nx * ((2 * y + ((d >> 1) & 1)) +
                                       (int64_t)g.ny * ((2 * z + (d >> 2)) + (int64_t)g.nz * b));
    s += (float)X[v * C + c];
  }
  Y[vc * C + c] = (__bf16)(0.125f * s);
}

__global__ void k_pool_bwd(Grid3 g, const __bf16* __restrict__ dY, __bf16* __restrict__ dX, int C,
                           int acc) {
  const int64_t nv = (int64_t)g.nx * g.ny * g.nz * g.batch;
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (e >= nv * C) return;
  const int c = (int)(e % C);
  const int64_t v = e / C;
  const int x = (int)(v % g.nx);
  const int y = (int)((v / g.nx) % g.ny);
  const int64_t zb = v / ((int64_t)g.nx * g.ny);
  const int z = (int)(zb % g.nz);
  const int64_t b = zb / g.nz;
  const int cx = g.nx / 2, cy = g.ny / 2, cz = g.nz / 2;
  const int64_t vc = (x / 2) + (int64_t)cx * ((y / 2) + (int64_t)cy * ((z / 2) + (int64_t)cz * b));
  float val = 0.125f * (float)dY[vc * C + c];
  if (acc) val += (float)dX[e];
  dX[e] = (__bf16)val;
}

__global__ void k_up_bwd(Grid3 g, const __bf16* __restrict__ dY, __bf16* __restrict__ dX, int C) {
  const int cx = g.nx / 2, cy = g.ny / 2, cz = g.nz / 2;
  const int64_t nc = (int64_t)cx * cy * cz * g.batch;
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (e >= nc * C) return;
  const int c = (int)(e % C);
  const int64_t vc = e / C;
  const int x = (int)(vc % cx);
  const int y = (int)((vc / cx) % cy);
  const int64_t zb = vc / ((int64_t)cx * cy);
  const int z = (int)(zb % cz);
  const int64_t b = zb / cz;
  float s = 0.f;
  for (int d = 0; d < 8; ++d) {
    const int64_t v = (2 * x + (d & 1)) +
                      (int64_t)g.nx * ((2 * y + ((d >> 1) & 1)) +
                                       (int64_t)g.ny * ((2 * z + (d >> 2)) + (int64_t)g.nz * b));
    s += (float)dY[v * C + c];
  }
  dX[e] = (__bf16)s;
}

// dZ = dY * (Y > 0) in place on dY
__global__ void k_relu_bwd(int64_t ne, __bf16* __restrict__ dY, const __bf16* __restrict__ Y) {
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (e < ne && !((float)Y[e] > 0.f)) dY[e] = (__bf16)0.f;
}

// out += in (elementwise, bf16 storage, FP32 add)
__global__ void k_add(int64_t ne, __bf16* __restrict__ out, const __bf16* __restrict__ in) {
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (e < ne) out[e] = (__bf16)((float)out[e] + (float)in[e]);
}

// Input fields (FP32, [b][c][v], c < cin) -> BF16 activations [b v][Cp] (pads zero).
__global__ void k_pack_input(int64_t nvox, int batch, int cin, const float* __restrict__ in,
                             __bf16* __restrict__ X, int Cp) {
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (e >= nvox * batch * Cp) return;
  const int c = (int)(e % Cp);
  const int64_t vb = e / Cp;
  const int64_t b = vb / nvox, v = vb % nvox;
  X[e] = (__bf16)(c < cin ? in[(b * cin + c) * nvox + v] : 0.f);
}

// Output channels c < cout of [b v][Cp] -> FP32 [b][c][v]
__global__ void k_unpack_output(int64_t nvox, int batch, int cout, const __bf16* __restrict__ Y,
                                int Cp, float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (e >= nvox * batch * cout) return;
  const int64_t v = e % nvox;
  const int64_t bc = e / nvox;
  const int c = (int)(bc % cout);
  const int64_t b = bc / cout;
  out[e] = (float)Y[(b * nvox + v) * Cp + c];
}

// MSE on channel 0: partial sums of (y - t)^2 / count per block, dY = 2 (y - t) / count.
__global__ void k_mse(int64_t ne, const __bf16* __restrict__ Y, int Cp,
                      const float* __restrict__ tgt, double inv_count, __bf16* __restrict__ dY,
                      double* __restrict__ partials) {
  double v[1] = {0.0};
  for (int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x; e < ne; e += (int64_t)gridDim.x * BS) {
    const double d = (double)(float)Y[e * Cp] - (double)tgt[e];
    v[0] += d * d * inv_count;
    dY[e * Cp] = (__bf16)(float)(2.0 * d * inv_count);
    for (int c = 1; c < Cp; ++c) dY[e * Cp + c] = (__bf16)0.f;
  }
  write_partials<1, BS>(v, partials, blockIdx.x);
}

// Adam (Kingma & Ba) on FP32 master parameters; c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void k_adam(int64_t n, float* __restrict__ p, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2,
                       float c1, float c2, float eps) {
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.f - b1) * gi;
  const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  p[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// FP32 layer weights (oracle order w[o][i][a][b][c]) -> BF16 GEMM weights
// Wb[o][tap Cpi + i] (zeros beyond) and the data-gradient weights
// Wt[i][tap' Cpo + o] = w[o][i][26 - tap'] (spatially flipped, channels transposed).
__global__ void k_pack_weights(const float* __restrict__ w, int cout, int cin, int Cpi, int Kp,
                               int rows, __bf16* __restrict__ Wb, int Cpo, int Ktp, int rowst,
                               __bf16* __restrict__ Wt) {
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  const int64_t n1 = (int64_t)rows * Kp, n2 = (int64_t)rowst * Ktp;
  if (e < n1) {
    const int o = (int)(e / Kp), k = (int)(e % Kp);
    float val = 0.f;
    if (o < cout && k < 27 * Cpi) {
      const int tap = k / Cpi, i = k % Cpi;
      if (i < cin) val = w[((int64_t)o * cin + i) * 27 + tap];
    }
    Wb[e] = (__bf16)val;
  } else if (e < n1 + n2) {
    const int64_t f = e - n1;
    const int i = (int)(f / Ktp), k = (int)(f % Ktp);
    float val = 0.f;
    if (i < cin && k < 27 * Cpo) {
      const int tap = k / Cpo, o = k % Cpo;
      if (o < cout) val = w[((int64_t)o * cin + i) * 27 + (26 - tap)];
    }
    Wt[f] = (__bf16)val;
  }
}

// GEMM-layout weight gradient dWg[o][tap Cpi + i] -> oracle order dw[o][i][tap] (added).
__global__ void k_unpack_wgrad(const float* __restrict__ dWg, int Kp, int cout, int cin, int Cpi,
                               float* __restrict__ dw) {
  const int64_t e = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (e >= (int64_t)cout * cin * 27) return;
  const int tap = (int)(e % 27);
  const int i = (int)((e / 27) % cin);
  const int o = (int)(e / (27 * cin));
  dw[e] += dWg[(int64_t)o * Kp + tap * Cpi + i];
}

// Network inputs for `count` right-hand sides: [dmu / mu_scale, log(D / D_ref), e_idx[b]].
__global__ void k_seed_inputs(int64_t n, int count, const double* __restrict__ dmu,
                              double mu_scale, const double* __restrict__ D, double Dc,
                              double Dref, const int64_t* __restrict__ idx,
                              float* __restrict__ out) {
  const int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x;
  const int b = blockIdx.y;
  if (v >= n || b >= count) return;
  float* o = out + (int64_t)b * 3 * n;
  o[v] = (float)(dmu[v] / mu_scale);
  o[n + v] = (float)log((D ? D[v] : Dc) / Dref);
  o[2 * n + v] = v == idx[b] ? 1.f : 0.f;
}

// Per-column max |X| partials (blockIdx.y = column).
__global__ void k_colmaxabs(int64_t n, const double* __restrict__ X, int64_t ldx,
                            double* __restrict__ part) {
  __shared__ double sh[BS];
  const double* x = X + (int64_t)blockIdx.y * ldx;
  double m = 0.0;
  for (int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x; v < n; v += (int64_t)gridDim.x * BS)
    m = fmax(m, fabs(x[v]));
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = BS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = sh[0];
}

// out[b][v] = X[v + b ldx] / max over the column's partials
__global__ void k_scale_targets(int64_t n, const double* __restrict__ X, int64_t ldx,
                                const double* __restrict__ part, int P, float* __restrict__ out) {
  const int b = blockIdx.y;
  double m = 0.0;
  for (int q = 0; q < P; ++q) m = fmax(m, part[(int64_t)b * P + q]);
  const double s = m > 0.0 ? 1.0 / m : 0.0;
  for (int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x; v < n; v += (int64_t)gridDim.x * BS)
    out[(int64_t)b * n + v] = (float)(X[(int64_t)b * ldx + v] * s);
}

// Guess direction d = xg - x0 (xg FP32).
__global__ void k_guess_dir(int64_t n, const float* __restrict__ xg, const double* __restrict__ x0,
                            double* __restrict__ d) {
  for (int64_t v = (int64_t)blockIdx.x * BS + threadIdx.x; v < n; v += (int64_t)gridDim.x * BS)
    d[v] = (double)xg[v] - x0[v];
}

int gridn(int64_t n) { return (int)ceil_div(n, BS); }

}  // namespace

// LDS budget of the staged convolution (larger input widths take the gathering kernel)
constexpr size_t CONV_LDS_MAX = 64 * 1024;

int seed_round8(int c) { return (c + 7) / 8 * 8; }
int seed_kp(int cp) { return (27 * cp + 31) / 32 * 32; }

void launch_seed_conv(int nx, int ny, int nz, int batch, const void* X, int Cpi, const void* W,
                      int Kp, int Cout, int rows, const float* bias, const void* skip, int relu,
                      void* Y, int Cpo, hipStream_t st, int up) {
  if (up && ((nx | ny | nz) & 1)) throw Error(ROM_EINVAL, "seed conv: upsampled input needs even sizes");
  const Grid3 g{nx, ny, nz, batch};
  const int64_t nv = (int64_t)nx * ny * nz * batch;
  // the deepest box whose staged halo fits the LDS budget
  int bz = 0;
  for (int c : {4, 2})
    if (!bz && nx % CB_X == 0 && ny % CB_Y == 0 && nz % c == 0 &&
        sizeof(__bf16) * (size_t)conv_halo_vox(c) * (Cpi + 8) <= CONV_LDS_MAX)
      bz = c;
  if (bz) {
    const size_t lds = sizeof(__bf16) * (size_t)conv_halo_vox(bz) * (Cpi + 8);
    const dim3 grid((unsigned)(nv / (CB_X * CB_Y * bz)));
    const __bf16* x = (const __bf16*)X;
    const __bf16* w = (const __bf16*)W;
    const __bf16* sk = (const __bf16*)skip;
    __bf16* y = (__bf16*)Y;
    if (rows / 16 < 1 || rows / 16 > 4) throw Error(ROM_EINVAL, "seed conv: at most 64 output channels");
#define C(N, Z) ROM_LAUNCH((k_conv_lds<N, Z>), grid, dim3(BS), lds, st, g, x, Cpi, w, Kp, Cout, bias, sk, relu, y, Cpo, up)
    if (bz == 4) {
      switch (rows / 16) { case 1: C(1, 4); break; case 2: C(2, 4); break; case 3: C(3, 4); break; default: C(4, 4); break; }
    } else {
      switch (rows / 16) { case 1: C(1, 2); break; case 2: C(2, 2); break; case 3: C(3, 2); break; default: C(4, 2); break; }
    }
#undef C
    ROM_CHECK_LAUNCH();
    return;
  }
  constexpr int VT = 2;
  const dim3 grid(ceil_div(nv, 64 * VT));
  const __bf16* x = (const __bf16*)X;
  const __bf16* w = (const __bf16*)W;
  const __bf16* sk = (const __bf16*)skip;
  __bf16* y = (__bf16*)Y;
  switch (rows / 16) {
#define C(N) case N: ROM_LAUNCH((k_conv<N, VT>), grid, dim3(BS), 0, st, g, x, Cpi, w, Kp, Cout, bias, sk, relu, y, Cpo, up); break;
    C(1) C(2) C(3) C(4)
#undef C
    default: throw Error(ROM_EINVAL, "seed conv: at most 64 output channels");
  }
  ROM_CHECK_LAUNCH();
}

size_t seed_wgrad_partials(int nx, int ny, int nz, int batch, int rows, int Kp) {
  const int64_t nv = (int64_t)nx * ny * nz * batch;
  return (size_t)ceil_div(nv, WG_VOX) * rows * Kp;
}

void launch_seed_wgrad(int nx, int ny, int nz, int batch, const void* X, int Cpi, const void* dZ,
                       int Cpo, int Cout, int rows, int Kp, float* P, float* dWg, float* Pb,
                       float* db, hipStream_t st, int up) {
  if (up && ((nx | ny | nz) & 1)) throw Error(ROM_EINVAL, "seed wgrad: upsampled input needs even sizes");
  const Grid3 g{nx, ny, nz, batch};
  const int64_t nv = (int64_t)nx * ny * nz * batch;
  const int nch = (int)ceil_div(nv, WG_VOX);
  ROM_LAUNCH(k_conv_wgrad, dim3(nch, ceil_div(Kp, 64), rows / 16), dim3(BS), 0, st, g,
             (const __bf16*)X, Cpi, (const __bf16*)dZ, Cpo, Kp, P, up);
  ROM_CHECK_LAUNCH();
  ROM_LAUNCH(k_wgrad_reduce, dim3(gridn((int64_t)rows * Kp)), dim3(BS), 0, st, P, nch, rows, Kp,
             dWg, 0);
  ROM_CHECK_LAUNCH();
  ROM_LAUNCH(k_bias_grad, dim3(nch, Cout), dim3(BS), 0, st, nv, (const __bf16*)dZ, Cpo, Cout, Pb);
  ROM_CHECK_LAUNCH();
  // db[o] += sum over chunks
  ROM_LAUNCH(k_wgrad_reduce, dim3(gridn(Cout)), dim3(BS), 0, st, Pb, nch, 1, Cout, db, 1);
  ROM_CHECK_LAUNCH();
}

void launch_seed_pool(int nx, int ny, int nz, int batch, const void* X, void* Y, int C,
                      hipStream_t st) {
  const Grid3 g{nx, ny, nz, batch};
  const int64_t n = (int64_t)(nx / 2) * (ny / 2) * (nz / 2) * batch * C;
  ROM_LAUNCH(k_pool, dim3(gridn(n)), dim3(BS), 0, st, g, (const __bf16*)X, (__bf16*)Y, C);
  ROM_CHECK_LAUNCH();
}

void launch_seed_pool_bwd(int nx, int ny, int nz, int batch, const void* dY, void* dX, int C,
                          int acc, hipStream_t st) {
  const Grid3 g{nx, ny, nz, batch};
  const int64_t n = (int64_t)nx * ny * nz * batch * C;
  ROM_LAUNCH(k_pool_bwd, dim3(gridn(n)), dim3(BS), 0, st, g, (const __bf16*)dY, (__bf16*)dX, C,
             acc);
  ROM_CHECK_LAUNCH();
}

void launch_seed_up_bwd(int nx, int ny, int nz, int batch, const void* dY, void* dX, int C,
                        hipStream_t st) {
  const Grid3 g{nx, ny, nz, batch};
  const int64_t n = (int64_t)(nx / 2) * (ny / 2) * (nz / 2) * batch * C;
  ROM_LAUNCH(k_up_bwd, dim3(gridn(n)), dim3(BS), 0, st, g, (const __bf16*)dY, (__bf16*)dX, C);
  ROM_CHECK_LAUNCH();
}

void launch_seed_relu_bwd(int64_t ne, void* dY, const void* Y, hipStream_t st) {
  ROM_LAUNCH(k_relu_bwd, dim3(gridn(ne)), dim3(BS), 0, st, ne, (__bf16*)dY, (const __bf16*)Y);
  ROM_CHECK_LAUNCH();
}

void launch_seed_add(int64_t ne, void* out, const void* in, hipStream_t st) {
  ROM_LAUNCH(k_add, dim3(gridn(ne)), dim3(BS), 0, st, ne, (__bf16*)out, (const __bf16*)in);
  ROM_CHECK_LAUNCH();
}

void launch_seed_pack_input(int64_t nvox, int batch, int cin, const float* in, void* X, int Cp,
                            hipStream_t st) {
  ROM_LAUNCH(k_pack_input, dim3(gridn(nvox * batch * Cp)), dim3(BS), 0, st, nvox, batch, cin, in,
             (__bf16*)X, Cp);
  ROM_CHECK_LAUNCH();
}

void launch_seed_unpack_output(int64_t nvox, int batch, int cout, const void* Y, int Cp,
                               float* out, hipStream_t st) {
  ROM_LAUNCH(k_unpack_output, dim3(gridn(nvox * batch * cout)), dim3(BS), 0, st, nvox, batch, cout,
             (const __bf16*)Y, Cp, out);
  ROM_CHECK_LAUNCH();
}

void launch_seed_mse(int64_t ne, const void* Y, int Cp, const float* tgt, void* dY,
                     double* partials, double* loss, hipStream_t st) {
  int grid = gridn(ne);
  if (grid > 1024) grid = 1024;
  ROM_LAUNCH(k_mse, dim3(grid), dim3(BS), 0, st, ne, (const __bf16*)Y, Cp, tgt, 1.0 / (double)ne,
             (__bf16*)dY, partials);
  ROM_CHECK_LAUNCH();
  launch_reduce_finish(partials, grid, 1, loss, st);
}

void launch_seed_adam(int64_t n, float* p, const float* g, float* m, float* v, float lr, float b1,
                      float b2, float c1, float c2, float eps, hipStream_t st) {
  ROM_LAUNCH(k_adam, dim3(gridn(n)), dim3(BS), 0, st, n, p, g, m, v, lr, b1, b2, c1, c2, eps);
  ROM_CHECK_LAUNCH();
}

void launch_seed_pack_weights(const float* w, int cout, int cin, int Cpi, int Kp, int rows,
                              void* Wb, int Cpo, int Ktp, int rowst, void* Wt, hipStream_t st) {
  const int64_t n = (int64_t)rows * Kp + (int64_t)rowst * Ktp;
  ROM_LAUNCH(k_pack_weights, dim3(gridn(n)), dim3(BS), 0, st, w, cout, cin, Cpi, Kp, rows,
             (__bf16*)Wb, Cpo, Ktp, rowst, (__bf16*)Wt);
  ROM_CHECK_LAUNCH();
}

void launch_seed_unpack_wgrad(const float* dWg, int Kp, int cout, int cin, int Cpi, float* dw,
                              hipStream_t st) {
  ROM_LAUNCH(k_unpack_wgrad, dim3(gridn((int64_t)cout * cin * 27)), dim3(BS), 0, st, dWg, Kp, cout,
             cin, Cpi, dw);
  ROM_CHECK_LAUNCH();
}

void launch_seed_inputs(int64_t n, int count, const double* dmu, double mu_scale, const double* D,
                        double Dc, double Dref, const int64_t* idx, float* out, hipStream_t st) {
  if (count <= 0) return;
  ROM_LAUNCH(k_seed_inputs, dim3(gridn(n), count), dim3(BS), 0, st, n, count, dmu, mu_scale, D, Dc,
             Dref, idx, out);
  ROM_CHECK_LAUNCH();
}

void launch_seed_targets(int64_t n, int count, const double* X, int64_t ldx, double* part,
                         float* out, hipStream_t st) {
  if (count <= 0) return;
  const int P = std::min(64, gridn(n));
  ROM_LAUNCH(k_colmaxabs, dim3(P, count), dim3(BS), 0, st, n, X, ldx, part);
  ROM_CHECK_LAUNCH();
  ROM_LAUNCH(k_scale_targets, dim3(std::min(256, gridn(n)), count), dim3(BS), 0, st, n, X, ldx,
             part, P, out);
  ROM_CHECK_LAUNCH();
}

void launch_guess_dir(int64_t n, const float* xg, const double* x0, double* d, hipStream_t st) {
  ROM_LAUNCH(k_guess_dir, dim3(std::min(1024, gridn(n))), dim3(BS), 0, st, n, xg, x0, d);
  ROM_CHECK_LAUNCH();
}

}  // namespace rom
