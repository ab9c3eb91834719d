// km_device.hpp -- device-side building blocks shared by the gfx950 kernels:
// low-precision formats with their matrix-core instructions, the FP64 direct
// squared distance, and wavefront helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace km {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kWave = 64;

// Pointers to device memory held in problem descriptors are generic (flat)
// pointers.  Flat loads count against the LDS wait counter as well, so an LDS
// wait would also wait for every outstanding flat load: a prefetch from
// global memory would complete before the next LDS read could be used.
// Kernels therefore access device memory through global-address-space views.
#define KM_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const KM_GLOBAL T* as_global(const T* p) {
  return (const KM_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ KM_GLOBAL T* as_global(T* p) {
  return (KM_GLOBAL T*)p;
}


// ---------------------------------------------------------------------------
// Low-precision formats.  Each provides: the storage type S; the matrix-core
// fragment of one lane for a 32x32 output block (KV consecutive K elements),
// the K extent KS of one instruction, the round-to-nearest-even conversion
// from FP32, the overflow threshold (inputs at or above it round to inf),
// and the 32x32 MFMA D = A*B + C with FP32 accumulation.
//
// Operand layout of the 32x32xKS instructions (lane l = 0..63):
//   A: row (l % 32), K elements [(l/32)*KV, (l/32)*KV + KV)
//   B: column (l % 32), same K elements
//   D: column (l % 32), rows 8*(r/4) + 4*(l/32) + (r%4) for r = 0..15
// ---------------------------------------------------------------------------
struct LowF16 {
  static constexpr int kFmt = 0;
  using S = _Float16;
  using frag = f16x8;
  static constexpr int KS = 16, KV = 8;
  static constexpr bool kHasRange = true;
  // binary16: the largest finite value is 65504; halfway to 2^16 is 65520.
  static constexpr float kOverflow = 65520.0f;
  __device__ static inline S cvt(float x) { return (S)x; }
  __device__ static inline float tof(S v) { return (float)v; }
  __device__ static inline uint16_t bits(S v) { return __builtin_bit_cast(uint16_t, v); }
  __device__ static inline f32x16 mfma(frag a, frag b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

struct LowBF16 {
  static constexpr int kFmt = 1;
  using S = __bf16;
  using frag = bf16x8;
  static constexpr int KS = 16, KV = 8;
  static constexpr bool kHasRange = false;  // same exponent range as FP32
  static constexpr float kOverflow = 0.0f;
  __device__ static inline S cvt(float x) { return (S)x; }
  __device__ static inline float tof(S v) { return (float)v; }
  __device__ static inline uint16_t bits(S v) { return __builtin_bit_cast(uint16_t, v); }
  __device__ static inline f32x16 mfma(frag a, frag b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

struct LowF32 {
  static constexpr int kFmt = 2;
  using S = float;
  using frag = float;
  static constexpr int KS = 2, KV = 1;
  static constexpr bool kHasRange = false;
  static constexpr float kOverflow = 0.0f;
  __device__ static inline S cvt(float x) { return x; }
  __device__ static inline float tof(S v) { return v; }
  __device__ static inline uint16_t bits(S) { return 0; }
  __device__ static inline f32x16 mfma(frag a, frag b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
};

// Row of the 32x32 output block held in accumulator register r by lane l.
__device__ __host__ constexpr int acc_row(int r, int lane) {
  return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

// ---------------------------------------------------------------------------
// Direct formula eq:dist-direct in FP64 from FP32 data: differences and the
// running sum in FP64, coordinates in index order (fused multiply-add).
// ---------------------------------------------------------------------------
__device__ inline double sqdist64(const float* __restrict__ xp,
                                  const float* __restrict__ cp, int d) {
  const KM_GLOBAL float* x = as_global(xp);
  const KM_GLOBAL float* c = as_global(cp);
  double s = 0.0;
  int l = 0;
  if ((((uintptr_t)xp | (uintptr_t)cp) & 15) == 0 && (d & 3) == 0) {
    for (; l < d; l += 4) {
      f32x4 a = *reinterpret_cast<const KM_GLOBAL f32x4*>(x + l);
      f32x4 b = *reinterpret_cast<const KM_GLOBAL f32x4*>(c + l);
      double e0 = (double)a.x - (double)b.x;
      double e1 = (double)a.y - (double)b.y;
      double e2 = (double)a.z - (double)b.z;
      double e3 = (double)a.w - (double)b.w;
      s = __builtin_fma(e0, e0, s);
      s = __builtin_fma(e1, e1, s);
      s = __builtin_fma(e2, e2, s);
      s = __builtin_fma(e3, e3, s);
    }
  } else {
    for (; l < d; ++l) {
      double e = (double)x[l] - (double)c[l];
      s = __builtin_fma(e, e, s);
    }
  }
  return s;
}

// Out-of-line copy for rare paths (keeps the hot loops compact).
__device__ __noinline__ double sqdist64_call(const float* __restrict__ x,
                                            const float* __restrict__ c, int d);

// ---------------------------------------------------------------------------
// Other correction precisions of a flagged pair (the fallback rules
// eq:fallback-rule and eq:fallback-rule-mp with another precision u):
//   kHigh64  -- the FP64 direct formula on the FP32 inputs (default);
//   kHigh32  -- the FP32 direct formula on the FP32 inputs;
//   kHighLow -- the direct formula in the low format itself, on the
//               quantised inputs x~, c~ (the uniform rule eq:fallback-rule).
// Every operation is one correctly rounded operation of the format
// (round to nearest even): differences, then a fused multiply-add per
// coordinate in index order.
// ---------------------------------------------------------------------------
constexpr int kHigh64 = 0, kHigh32 = 1, kHighLow = 2;

// f(x_l, c_l) for l = 0 .. d-1 in index order; the rows are read four
// coordinates per 16-byte load when both are 16-byte aligned and d is a
// multiple of 4 (rows in global memory or in LDS).
template <class F>
__device__ __forceinline__ void for_coords(const float* x, const float* c, int d, F&& f) {
  int l = 0;
  if ((((uintptr_t)x | (uintptr_t)c) & 15) == 0 && (d & 3) == 0) {
    for (; l < d; l += 4) {
      const f32x4 a = *reinterpret_cast<const f32x4*>(x + l);
      const f32x4 b = *reinterpret_cast<const f32x4*>(c + l);
      f(a.x, b.x);
      f(a.y, b.y);
      f(a.z, b.z);
      f(a.w, b.w);
    }
  }
  for (; l < d; ++l) f(x[l], c[l]);
}

// FP32 direct formula, coordinates in index order.
__device__ inline float sqdist32(const float* x, const float* c, int d) {
  float s = 0.0f;
  for_coords(x, c, d, [&](float a, float b) {
    const float t = a - b;
    s = __builtin_fmaf(t, t, s);
  });
  return s;
}

// binary16 direct formula on x~ = RNE16(x), c~ = RNE16(c): the hardware's
// half-precision subtraction and fused multiply-add round once each.
__device__ inline float sqdist16(const float* x, const float* c, int d) {
  _Float16 s = (_Float16)0.0f;
  for_coords(x, c, d, [&](float a, float b) {
    const _Float16 t = (_Float16)a - (_Float16)b;
    s = __builtin_fmaf16(t, t, s);
  });
  return (float)s;
}

// One rounding of the exact value hi + lo to bfloat16 (returned as FP32),
// where hi = RN64(hi + lo).  hi is first rounded to FP32; that can land on a
// bfloat16 midpoint that the exact value does not lie on, and only then does
// the remainder (hi - f) + lo decide the direction.
__device__ inline float bf16_round(double hi, double lo) {
  const float f = (float)hi;
  uint32_t b = __float_as_uint(f);
  if ((b & 0xffffu) == 0x8000u && (b & 0x7f800000u) != 0x7f800000u) {
    const double rem = (hi - (double)f) + lo;  // hi - f is exact
    if (rem != 0.0) {
      const bool up = (rem > 0.0) == (f > 0.0);  // away from zero
      return __uint_as_float(up ? (b + 0x8000u) : (b & 0xffff0000u));
    }
  }
  if ((b & 0x7f800000u) == 0x7f800000u) return f;  // inf (no NaN arises here)
  b += 0x7fffu + ((b >> 16) & 1u);
  return __uint_as_float(b & 0xffff0000u);
}

// bfloat16 a - b and a * b + c for bfloat16 operands held in FP32: the exact
// result as an unevaluated FP64 sum (two-sum; a * b is exact in FP64), one
// rounding.
__device__ inline float bf16_sub(float a, float b) {
  const double x = (double)a, y = -(double)b;
  const double s = x + y;
  const double yv = s - x;
  const double e = (x - (s - yv)) + (y - yv);
  return bf16_round(s, e);
}
__device__ inline float bf16_fma(float a, float b, float c) {
  const double x = (double)a * (double)b, y = (double)c;
  const double s = x + y;
  const double yv = s - x;
  const double e = (x - (s - yv)) + (y - yv);
  return bf16_round(s, e);
}

// bfloat16 direct formula on x~ = RNE_bf16(x), c~ = RNE_bf16(c).
__device__ inline float sqdistbf16(const float* x, const float* c, int d) {
  float s = 0.0f;
  for_coords(x, c, d, [&](float a, float b) {
    const float t = bf16_sub((float)(__bf16)a, (float)(__bf16)b);
    s = bf16_fma(t, t, s);
  });
  return s;
}

// Corrected squared distance in the requested precision (fmt: 0 FP16,
// 1 BF16, 2 FP32 low format).  The FP32 and low-format values are exact in
// FP64.
__device__ inline double corr_dist(int high, int fmt, const float* x, const float* c, int d) {
  if (high == kHigh32 || (high == kHighLow && fmt == 2)) return (double)sqdist32(x, c, d);
  if (high == kHighLow) return (double)(fmt == 0 ? sqdist16(x, c, d) : sqdistbf16(x, c, d));
  double s = 0.0;
  for (int l = 0; l < d; ++l) {
    const double e = (double)x[l] - (double)c[l];
    s = __builtin_fma(e, e, s);
  }
  return s;
}
// Out-of-line, for x and c in global memory (FP64 through sqdist64).
__device__ __noinline__ double corr_dist_call(int high, int fmt, const float* x, const float* c, int d);

// Wavefront sum of a double in a fixed butterfly order (deterministic).
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

}  // namespace km
