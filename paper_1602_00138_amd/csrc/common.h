// Internal helpers shared by the HIP kernels and the host runtime.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>

#include "../../include/rom.h"

namespace rom {

constexpr int WAVE = 64;
constexpr int NJ_MAX = ROM_NJ_MAX;

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

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
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

template <int R, int BS, typename T>
__device__ __forceinline__ void sum_partials_t(const T* __restrict__ partials, int P, T* tot) {
  __shared__ T sh[(BS / WAVE) * R];
  T acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = T(0);
  for (int b = threadIdx.x; b < P; b += BS) {
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] += partials[(size_t)r * P + b];
  }
  T t;
  block_sum<R, BS>(acc, sh, t);
  if (threadIdx.x < R) tot[threadIdx.x] = t;
  __syncthreads();
}

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace rom
