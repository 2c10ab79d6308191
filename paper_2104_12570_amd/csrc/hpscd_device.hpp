// Device-side building blocks shared by the HPSCD kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hpscd {

constexpr int WAVE = 64;

// Column storage formats.  A "chunk" is the 16 bytes one lane loads with a
// single 128-bit load: 4 FP32 rows or 8 BF16 rows of one column.
struct F32 {
  static constexpr int VEC = 4;
  using raw_t = float4;
  __device__ static inline float get(const raw_t& r, int i) {
    return i == 0 ? r.x : i == 1 ? r.y : i == 2 ? r.z : r.w;
  }
  __device__ static inline raw_t zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
};

struct BF16 {
  static constexpr int VEC = 8;
  using raw_t = uint4;
  // bfloat16 -> float is exact: the 16 stored bits are the top of the binary32 word.
  __device__ static inline float get(const raw_t& r, int i) {
    const uint32_t w = (i >> 1) == 0 ? r.x : (i >> 1) == 1 ? r.y : (i >> 1) == 2 ? r.z : r.w;
    const uint32_t b = (i & 1) ? (w & 0xFFFF0000u) : (w << 16);
    return __uint_as_float(b);
  }
  __device__ static inline raw_t zero() { return make_uint4(0u, 0u, 0u, 0u); }
};

template <class S>
__device__ inline typename S::raw_t load_chunk(const void* base, int64_t elem_off) {
  return *reinterpret_cast<const typename S::raw_t*>(
      reinterpret_cast<const char*>(base) + elem_off * (int64_t)(16 / S::VEC));
}

// Zero the entries of a chunk at or beyond row limit `lim` (0 <= lim < VEC).
template <class S>
__device__ inline typename S::raw_t mask_chunk(typename S::raw_t r, int lim);

template <>
__device__ inline float4 mask_chunk<F32>(float4 r, int lim) {
  if (lim <= 0) return F32::zero();
  if (lim < 2) r.y = 0.f;
  if (lim < 3) r.z = 0.f;
  if (lim < 4) r.w = 0.f;
  return r;
}

template <>
__device__ inline uint4 mask_chunk<BF16>(uint4 r, int lim) {
  uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (lim <= 2 * k) w[k] = 0u;
    else if (lim == 2 * k + 1) w[k] &= 0x0000FFFFu;
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// ---------------------------------------------------------------- reductions
// Sum over the 64 lanes of a wave; every lane receives the same value and the
// order of additions is fixed (results are bitwise reproducible).
template <int CTRL>
__device__ inline float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

__device__ inline float wave_sum(float v) {
  v += dpp_f32<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f32<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f32<0x141>(v);  // row_half_mirror
  v += dpp_f32<0x140>(v);  // row_mirror: each row of 16 now holds its sum
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
  return (r0 + r1) + (r2 + r3);
}

// Wave sums of 16 values at once, scattered: lane L returns the total of
// value (L >> 2) & 15 (the four lanes of a quad hold the same total).  Each
// stage pairs every lane with a partner across one lane bit and halves the
// values a lane holds (it keeps its half, adds the partner's copy of it), so
// the 16 totals take 8 + 4 + 2 + 1 + 2 additions instead of 16 full sums.
// Partners: lane xor 32 and xor 16 (LDS permute), then the row mirror (xor 15
// within a row of 16), the half-row mirror (xor 7 within 8), xor 2 and xor 1.
// The six masks are linearly independent over GF(2), so every lane's
// contribution enters each total exactly once.  Fixed order.
__device__ inline float wave_sum16_scatter(const float (&p)[16]) {
  const int L = (int)__lane_id();
  float q[8], r[4], s[2];
  const bool h5 = (L & 32) != 0, h4 = (L & 16) != 0, h3 = (L & 8) != 0, h2 = (L & 4) != 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float keep = h5 ? p[i + 8] : p[i], send = h5 ? p[i] : p[i + 8];
    q[i] = keep + __shfl_xor(send, 32);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float keep = h4 ? q[i + 4] : q[i], send = h4 ? q[i] : q[i + 4];
    r[i] = keep + __shfl_xor(send, 16);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float keep = h3 ? r[i + 2] : r[i], send = h3 ? r[i] : r[i + 2];
    s[i] = keep + dpp_f32<0x140>(send);  // row_mirror
  }
  const float keep = h2 ? s[1] : s[0], send = h2 ? s[0] : s[1];
  float t = keep + dpp_f32<0x141>(send);  // row_half_mirror
  t += dpp_f32<0x4E>(t);                  // quad_perm [2,3,0,1]
  t += dpp_f32<0xB1>(t);                  // quad_perm [1,0,3,2]
  return t;
}

template <int CTRL>
__device__ inline double dpp_f64(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

__device__ inline double readlane_f64(double v, int lane) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ inline double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x141>(v);
  v += dpp_f64<0x140>(v);
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

__device__ inline int lane_id() { return (int)__lane_id(); }

// A value known to be equal in every lane, moved to scalar registers.
__device__ inline double uniform_f64(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// ---------------------------------------------------------------- grid words
// A published value is one 64-bit word {seq (high 32 bits), FP32 bits (low)}
// stored and loaded as a relaxed atomic at agent scope: the value and its
// sequence number arrive together, so no fence is needed, and the access is
// coherent across the XCDs' separate L2 caches.
__device__ inline void publish(uint64_t* p, uint32_t seq, float v) {
  const uint64_t w = ((uint64_t)seq << 32) | (uint64_t)__float_as_uint(v);
  __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline uint64_t peek(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int32_t load_flag(const int32_t* p) {
  return __hip_atomic_load(const_cast<int32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The cancel word lives in pinned host memory mapped into the device: the
// host writes it directly, so a request needs no GPU work of its own (a copy
// could not start while a persistent kernel fills every CU).  The load
// crosses to host memory (about a microsecond), so kernels issue it early.
__device__ inline int32_t load_cancel(const int32_t* p) {
  return __hip_atomic_load(const_cast<int32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ inline void store_flag(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Constant 100 MHz wall clock, used to bound every spin-wait.
__device__ inline uint64_t now_ticks() { return wall_clock64(); }

// Control-word layout shared by the kernels and the host.
enum Ctl : int {
  CTL_ABORT = 0,      // (unused: the cancel word is in host memory, SolveArgs::cancel)
  CTL_ERR = 1,        // kernel-reported error (status code)
  CTL_SWEEPS = 2,     // complete sweeps performed
  CTL_CONVERGED = 3,  // a stop test fired
  CTL_NONFINITE = 4,  // prep found a non-finite norm or right-hand side
  CTL_DONE = 5,       // the solve has finished (later segments return at once)
  CTL_COUNT = 8
};
enum Ctl64 : int { C64_COLS = 0, C64_ZERO_COLS = 1, C64_FINAL_NORM2 = 2, C64_COUNT = 4 };

constexpr int ERR_TIMEOUT = 6;
constexpr int ERR_ABORTED = 5;
constexpr int ERR_NONFINITE = 4;

// Stop rules.
enum StopRule : int { STOP_NONE = 0, STOP_REL_CHANGE = 1, STOP_REL_RESID = 2 };

}  // namespace hpscd
