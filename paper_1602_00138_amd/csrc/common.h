// Internal helpers shared by the HIP kernels and the host runtime.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <initializer_list>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>

#include "../../include/rom.h"

namespace rom {

constexpr int WAVE = 64;
constexpr int NJ_MAX = ROM_NJ_MAX;
// XCDs of the part: workgroup b of a launch runs on XCD b % NXCD, each XCD with its own L2
constexpr int NXCD = 8;

// Error carried from the runtime to the C ABI layer.
struct Error : std::runtime_error {
  rom_status code;
  Error(rom_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define ROM_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::rom::Error(ROM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define ROM_CHECK_LAUNCH() ROM_HIP(hipGetLastError())

// Start/stop events for the next kernel launch of this thread (set by the kernel
// timer).  A launch through ROM_LAUNCH consumes them: the events are recorded by the
// dispatch of that kernel itself, so their interval is the kernel's execution.
struct LaunchEvents {
  hipEvent_t a = nullptr, b = nullptr;
};
inline LaunchEvents& pending_events() {
  thread_local LaunchEvents e;
  return e;
}

#define ROM_LAUNCH(K, G, B, S, ST, ...)                                                 \
  do {                                                                                  \
    ::rom::LaunchEvents& pe_ = ::rom::pending_events();                                \
    if (pe_.a) {                                                                        \
      hipExtLaunchKernelGGL(K, G, B, S, ST, pe_.a, pe_.b, 0, __VA_ARGS__);              \
      pe_.a = pe_.b = nullptr;                                                          \
    } else {                                                                            \
      hipLaunchKernelGGL(K, G, B, S, ST, __VA_ARGS__);                                  \
    }                                                                                   \
    ROM_CHECK_LAUNCH();                                                                 \
  } while (0)

// Column pointer table passed by value as a kernel argument (U_j columns live in
// different buffers: the first columns of V and a per-RHS pool).
struct ColPtrs {
  const double* p[NJ_MAX];
};

// Device-side skip condition: a kernel given Skip{v, thr} returns at once when
// v[0] > thr * v[1] (both read from device memory); Skip{} never skips.
struct Skip {
  const double* v = nullptr;
  double thr = 0.0;
  __device__ __forceinline__ bool on() const { return v && v[0] > thr * v[1]; }
};

// Stencil description handed to kernels.
struct Stencil {
  int nx, ny, nz;        // interior nodes per axis (nz = 1 in 2D)
  int dim;
  double cx, cy, cz;     // constant-D face coefficients D/h^2 (used when var == 0)
  const double* fx;      // per-node coefficient of the +x face (var D), 0 at the boundary
  const double* fy;
  const double* fz;
  const float* fx32;     // FP32 copies of the face coefficients (var D), for the FP32 solver
  const float* fy32;
  const float* fz32;
  int var;               // 1: per-node face coefficients
  int64_t n;
};

// Walk one x-y position q of the FP64 operator through the z planes [z0, z1): calls
// f(i, (A x)_i, x_i) per node i, with the z neighbours carried in registers (the lateral
// ones come from the caches), so x is fetched from HBM about once.  diag holds A's
// diagonal (A_* plus mu); the off-diagonal entries are minus the face coefficients.
template <bool VAR, class F>
__device__ __forceinline__ void stencil_walk(const Stencil& S, const double* __restrict__ diag,
                                             const double* __restrict__ x, int q, int z0,
                                             int z1, F&& f) {
  const int nxy = S.nx * S.ny;
  const int ix = q % S.nx, iy = q / S.nx;
  const bool hl = ix > 0, hr = ix < S.nx - 1, hd = iy > 0, hu = iy < S.ny - 1;
  int64_t i = (int64_t)z0 * nxy + q;
  double xm = z0 > 0 ? x[i - nxy] : 0.0;
  double fm = (VAR && z0 > 0) ? S.fz[i - nxy] : 0.0;
  double xc = x[i];
  for (int z = z0; z < z1; ++z, i += nxy) {
    const double xp = z < S.nz - 1 ? x[i + nxy] : 0.0;
    double v = diag[i] * xc;
    if (!VAR) {
      const double sx = (hl ? x[i - 1] : 0.0) + (hr ? x[i + 1] : 0.0);
      const double sy = (hd ? x[i - S.nx] : 0.0) + (hu ? x[i + S.nx] : 0.0);
      v -= S.cx * sx + S.cy * sy + S.cz * (xm + xp);
    } else {
      if (hl) v -= S.fx[i - 1] * x[i - 1];
      if (hr) v -= S.fx[i] * x[i + 1];
      if (hd) v -= S.fy[i - S.nx] * x[i - S.nx];
      if (hu) v -= S.fy[i] * x[i + S.nx];
      if (S.dim == 3) {
        const double fp = S.fz[i];
        v -= fm * xm + fp * xp;
        fm = fp;
      }
    }
    f(i, v, xc);
    xm = xc;
    xc = xp;
  }
}

// The walk of stencil_walk for two consecutive x-nodes (i even, nx even, every array
// aligned for two-element vector loads at even indices), in arithmetic T (double, or float
// with the FP32 face coefficients): calls f(i, (A x)_i, (A x)_{i+1}, x_i, x_{i+1}) per
// z-plane.  Vector loads for the pair, its y-neighbour pairs, the diagonal, the face
// coefficients and the next plane; one scalar load per outer x-neighbour.
template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };
template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
__device__ __forceinline__ void walk_faces(const Stencil& S, double, const double*& fx,
                                           const double*& fy, const double*& fz) {
  fx = S.fx; fy = S.fy; fz = S.fz;
}
__device__ __forceinline__ void walk_faces(const Stencil& S, float, const float*& fx,
                                           const float*& fy, const float*& fz) {
  fx = S.fx32; fy = S.fy32; fz = S.fz32;
}
template <typename T, bool VAR, class F>
__device__ __forceinline__ void stencil_walk2t(const Stencil& S, const T* __restrict__ diag,
                                               const T* __restrict__ x, int q, int z0, int z1,
                                               F&& f) {
  using V = typename Vec2<T>::type;
  const T *Fx, *Fy, *Fz;
  walk_faces(S, T(0), Fx, Fy, Fz);
  const T cx = (T)S.cx, cy = (T)S.cy, cz = (T)S.cz;
  const int hx = S.nx / 2;
  const int ix = 2 * (q % hx), iy = q / hx;
  const int nxy = S.nx * S.ny;
  const bool hl = ix > 0, hr = ix + 2 < S.nx, hd = iy > 0, hu = iy < S.ny - 1;
  const V zero = {T(0), T(0)};
  auto ld2 = [](const T* p, int64_t k) { return *reinterpret_cast<const V*>(p + k); };
  int64_t i = (int64_t)z0 * nxy + (int64_t)iy * S.nx + ix;
  V xm = z0 > 0 ? ld2(x, i - nxy) : zero;
  V fm = (VAR && z0 > 0) ? ld2(Fz, i - nxy) : zero;
  V xc = ld2(x, i);
  for (int z = z0; z < z1; ++z, i += nxy) {
    const V xp = z < S.nz - 1 ? ld2(x, i + nxy) : zero;
    const V d = ld2(diag, i);
    const T xl = hl ? x[i - 1] : T(0);
    const T xr = hr ? x[i + 2] : T(0);
    const V yd = hd ? ld2(x, i - S.nx) : zero;
    const V yu = hu ? ld2(x, i + S.nx) : zero;
    T v0 = d.x * xc.x, v1 = d.y * xc.y;
    if (!VAR) {
      v0 -= cx * (xl + xc.y) + cy * (yd.x + yu.x) + cz * (xm.x + xp.x);
      v1 -= cx * (xc.x + xr) + cy * (yd.y + yu.y) + cz * (xm.y + xp.y);
    } else {
      // +x faces: node i-1 (left of the pair), i (inside the pair), i+1 (right)
      const T fxl = hl ? Fx[i - 1] : T(0);
      const V fx = ld2(Fx, i);
      v0 -= fxl * xl + fx.x * xc.y;
      v1 -= fx.x * xc.x + fx.y * xr;
      const V fyd = hd ? ld2(Fy, i - S.nx) : zero;
      const V fyu = ld2(Fy, i);
      v0 -= fyd.x * yd.x + fyu.x * yu.x;
      v1 -= fyd.y * yd.y + fyu.y * yu.y;
      if (S.dim == 3) {
        const V fp = ld2(Fz, i);
        v0 -= fm.x * xm.x + fp.x * xp.x;
        v1 -= fm.y * xm.y + fp.y * xp.y;
        fm = fp;
      }
    }
    f(i, v0, v1, xc.x, xc.y);
    xm = xc;
    xc = xp;
  }
}
template <bool VAR, class F>
__device__ __forceinline__ void stencil_walk2(const Stencil& S, const double* __restrict__ diag,
                                              const double* __restrict__ x, int q, int z0,
                                              int z1, F&& f) {
  stencil_walk2t<double, VAR>(S, diag, x, q, z0, z1, static_cast<F&&>(f));
}

// stencil_walk in arithmetic T (double, or float with the FP32 face coefficients): one
// x-y position q through the z planes [z0, z1), f(i, (A x)_i, x_i) per node.
template <typename T, bool VAR, class F>
__device__ __forceinline__ void stencil_walk1t(const Stencil& S, const T* __restrict__ diag,
                                               const T* __restrict__ x, int q, int z0, int z1,
                                               F&& f) {
  const T *Fx, *Fy, *Fz;
  walk_faces(S, T(0), Fx, Fy, Fz);
  const T cx = (T)S.cx, cy = (T)S.cy, cz = (T)S.cz;
  const int nxy = S.nx * S.ny;
  const int ix = q % S.nx, iy = q / S.nx;
  const bool hl = ix > 0, hr = ix < S.nx - 1, hd = iy > 0, hu = iy < S.ny - 1;
  int64_t i = (int64_t)z0 * nxy + q;
  T xm = z0 > 0 ? x[i - nxy] : T(0);
  T fm = (VAR && z0 > 0) ? Fz[i - nxy] : T(0);
  T xc = x[i];
  for (int z = z0; z < z1; ++z, i += nxy) {
    const T xp = z < S.nz - 1 ? x[i + nxy] : T(0);
    T v = diag[i] * xc;
    if (!VAR) {
      const T sx = (hl ? x[i - 1] : T(0)) + (hr ? x[i + 1] : T(0));
      const T sy = (hd ? x[i - S.nx] : T(0)) + (hu ? x[i + S.nx] : T(0));
      v -= cx * sx + cy * sy + cz * (xm + xp);
    } else {
      if (hl) v -= Fx[i - 1] * x[i - 1];
      if (hr) v -= Fx[i] * x[i + 1];
      if (hd) v -= Fy[i - S.nx] * x[i - S.nx];
      if (hu) v -= Fy[i] * x[i + S.nx];
      if (S.dim == 3) {
        const T fp = Fz[i];
        v -= fm * xm + fp * xp;
        fm = fp;
      }
    }
    f(i, v, xc);
    xm = xc;
    xc = xp;
  }
}

// Whether the two-node walk applies: even nx and 16-byte aligned arrays at even leading
// dimensions (ld of every column array passed in `ld`).
inline bool stencil_pairs_ok(const Stencil& S, int64_t ld, std::initializer_list<const void*> ptrs,
                             bool fp32 = false) {
  const uintptr_t m = fp32 ? 7 : 15;
  if (S.nx % 2 != 0 || ld % 2 != 0) return false;
  for (const void* p : ptrs)
    if (p && ((uintptr_t)p & m)) return false;
  if (S.var) {
    const uintptr_t f = fp32 ? ((uintptr_t)S.fx32 | (uintptr_t)S.fy32 |
                                (S.dim == 3 ? (uintptr_t)S.fz32 : 0))
                             : ((uintptr_t)S.fx | (uintptr_t)S.fy |
                                (S.dim == 3 ? (uintptr_t)S.fz : 0));
    if (f & m) return false;
  }
  return true;
}

// Whether the four-node walk of the FP32 CG operator step applies: nx and every leading
// dimension a multiple of 4 and every FP32 array 16-byte aligned.
inline bool stencil_quads_ok(const Stencil& S, int64_t ld, std::initializer_list<const void*> ptrs) {
  if (S.nx % 4 != 0 || ld % 4 != 0) return false;
  for (const void* p : ptrs)
    if (p && ((uintptr_t)p & 15)) return false;
  if (S.var &&
      (((uintptr_t)S.fx32 | (uintptr_t)S.fy32 | (S.dim == 3 ? (uintptr_t)S.fz32 : 0)) & 15))
    return false;
  return true;
}

// One DPP move of a 32-bit or 64-bit value (lanes whose source is outside the pattern,
// or whose row is masked off, receive 0).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf,
                                                    false));
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Whole-wave shifts by one lane (DPP wave_shr:1 / wave_shl:1): lane l receives lane l - 1's
// (shr) or lane l + 1's (shl) value; lane 0 (shr) and lane 63 (shl) receive 0.
__device__ __forceinline__ float wave_shr1(float v) { return dpp_move<0x138, 0xf>(v); }
__device__ __forceinline__ float wave_shl1(float v) { return dpp_move<0x130, 0xf>(v); }
__device__ __forceinline__ double wave_shr1(double v) { return dpp_move<0x138, 0xf>(v); }
__device__ __forceinline__ double wave_shl1(double v) { return dpp_move<0x130, 0xf>(v); }
__device__ __forceinline__ float lane63(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ double lane63(double v) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                          __builtin_amdgcn_readlane(__double2loint(v), 63));
}

// Sum over the 64 lanes of a wave, returned to every lane.  Row shifts by 1, 2, 4 and 8
// leave each 16-lane row's sum in its last lane; the row broadcasts of lanes 15 and 31
// carry the row sums up so that lane 63 holds the total.  All on the vector ALU (no LDS
// traffic, unlike a butterfly of lane permutes).  Every lane of the wave must be active.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  v += dpp_move<0x111, 0xf>(v);   // row_shr:1
  v += dpp_move<0x112, 0xf>(v);   // row_shr:2
  v += dpp_move<0x114, 0xf>(v);   // row_shr:4
  v += dpp_move<0x118, 0xf>(v);   // row_shr:8
  v += dpp_move<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return lane63(v);
}

// Sum R per-thread values over the block; thread r < R of the returned block gets
// the block total of value r in `out` (other threads get garbage).
template <int R, int BS, typename T>
__device__ __forceinline__ void block_sum(const T (&v)[R], T* sh /* [BS/WAVE][R] */, T& out) {
  const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    T s = wave_sum(v[r]);
    if (lane == 0) sh[wid * R + r] = s;
  }
  __syncthreads();
  out = T(0);
  if (threadIdx.x < R) {
#pragma unroll
    for (int w = 0; w < BS / WAVE; ++w) out += sh[w * R + threadIdx.x];
  }
}

// Block partials: thread r < R of the block writes the block total of value r to
// partials[bid * R + r] (plain stores; a later kernel launch reads them).
template <int R, int BS, typename T>
__device__ __forceinline__ void write_partials(const T (&v)[R], T* partials, int bid) {
  __shared__ T sh[(BS / WAVE) * R];
  T bs;
  block_sum<R, BS>(v, sh, bs);
  if (threadIdx.x < R) partials[(size_t)bid * R + threadIdx.x] = bs;
}

// Sum P rows of R partials (row b = partials[b*R .. b*R+R)) in a fixed order; the totals
// land in tot[0..R) (shared memory) and are visible to every thread on return.
template <int R, int BS, typename T>
__device__ __forceinline__ void sum_partials(const T* __restrict__ partials, int P, T* tot) {
  __shared__ T sh[(BS / WAVE) * R];
  T acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = T(0);
  for (int b = threadIdx.x; b < P; b += BS) {
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] += partials[(size_t)b * R + r];
  }
  T t;
  block_sum<R, BS>(acc, sh, t);
  if (threadIdx.x < R) tot[threadIdx.x] = t;
  __syncthreads();
}

// Transposed partials for many values: value r of block bid goes to partials[r * P + bid]
// so that the consumer's loads are coalesced across blocks.
template <int R, int BS, typename T>
__device__ __forceinline__ void write_partials_t(const T (&v)[R], T* partials, int bid, int P) {
  __shared__ T sh[(BS / WAVE) * R];
  T bs;
  block_sum<R, BS>(v, sh, bs);
  if (threadIdx.x < R) partials[(size_t)threadIdx.x * P + bid] = bs;
}

// Totals of R transposed partial rows: a single value is summed by the whole block; with
// several, wave w sums values w, w + BS/64, ... (one wave reduction per value, not R
// reductions per wave).  tot[] (shared) is visible to every thread on return.
template <int R, int BS, typename T>
__device__ __forceinline__ void sum_partials_t(const T* __restrict__ partials, int P, T* tot) {
  const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
  if (R == 1) {
    __shared__ T sh[BS / WAVE];
    T a = T(0);
#pragma unroll 4
    for (int b = threadIdx.x; b < P; b += BS) a += partials[b];
    a = wave_sum(a);
    if (lane == 0) sh[wid] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
      T t = T(0);
#pragma unroll
      for (int w = 0; w < BS / WAVE; ++w) t += sh[w];
      tot[0] = t;
    }
  } else {
    for (int r = wid; r < R; r += BS / WAVE) {
      T a = T(0);
#pragma unroll 4
      for (int b = lane; b < P; b += WAVE) a += partials[(size_t)r * P + b];
      a = wave_sum(a);
      if (lane == 0) tot[r] = a;
    }
  }
  __syncthreads();
}

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace rom
