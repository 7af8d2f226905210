// Minimal complex arithmetic for device code (FP32 and FP64), interleaved
// (re, im) like bf_c64 / bf_c128.
#pragma once
#include <hip/hip_runtime.h>

namespace bf {

struct cf { float re, im; };
struct cd { double re, im; };

__device__ __forceinline__ cf cf_make(float r, float i) { return cf{r, i}; }
__device__ __forceinline__ cd cd_make(double r, double i) { return cd{r, i}; }
__device__ __forceinline__ cd cd_add(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd cd_sub(cd a, cd b) { return cd{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd cd_mul(cd a, cd b) {
  return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
__device__ __forceinline__ cd cd_cmul(cd a, cd b) {
  return cd{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
__device__ __forceinline__ cd cd_conj(cd a) { return cd{a.re, -a.im}; }
__device__ __forceinline__ cd cd_scale(cd a, double s) { return cd{a.re * s, a.im * s}; }
__device__ __forceinline__ double cd_abs2(cd a) { return a.re * a.re + a.im * a.im; }
// acc += a * b
__device__ __forceinline__ void cd_fma(cd& acc, cd a, cd b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
// acc += conj(a) * b
__device__ __forceinline__ void cd_cfma(cd& acc, cd a, cd b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
}
__device__ __forceinline__ void cf_fma(cf& acc, cf a, cf b) {
  acc.re = fmaf(a.re, b.re, acc.re);
  acc.re = fmaf(-a.im, b.im, acc.re);
  acc.im = fmaf(a.re, b.im, acc.im);
  acc.im = fmaf(a.im, b.re, acc.im);
}

// Lane exchanges by DPP (data-parallel primitives: a VALU source modifier,
// no trip through the LDS crossbar that __shfl's ds_bpermute takes).  CTRL:
// 0xB1 / 0x4E swap lanes at distance 1 / 2 within each group of four,
// 0x141 mirrors each half row of 8 lanes, 0x140 each row of 16.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum over each row of 16 lanes, left in every lane of the row: pairs at
// distance 1 and 2, then mirrored half rows and rows (each step adds two
// equal-shaped partial sums, so every lane of the row ends with the same
// bits).  All lanes of the row must be active.
template <typename T>
__device__ __forceinline__ T row16_sum(T v);
template <>
__device__ __forceinline__ float row16_sum<float>(float v) {
  v += dpp_f32<0xB1>(v);
  v += dpp_f32<0x4E>(v);
  v += dpp_f32<0x141>(v);
  v += dpp_f32<0x140>(v);
  return v;
}
template <>
__device__ __forceinline__ double row16_sum<double>(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x141>(v);
  v += dpp_f64<0x140>(v);
  return v;
}

// The same over each group of 8 lanes (the first three steps).
template <typename T>
__device__ __forceinline__ T row8_sum(T v);
template <>
__device__ __forceinline__ float row8_sum<float>(float v) {
  v += dpp_f32<0xB1>(v);
  v += dpp_f32<0x4E>(v);
  v += dpp_f32<0x141>(v);
  return v;
}
template <>
__device__ __forceinline__ double row8_sum<double>(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x141>(v);
  return v;
}

// Wavefront (64 lanes) sum, every lane gets the result: row sums as above,
// then (row 0 + row 1) + (row 2 + row 3) from lanes 0, 16, 32, 48.  Fixed
// order, so results are deterministic.  All 64 lanes must be active.
__device__ __forceinline__ double wave_sum(double v) {
  v = row16_sum(v);
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}
__device__ __forceinline__ cd wave_sum(cd v) {
  v.re = wave_sum(v.re);
  v.im = wave_sum(v.im);
  return v;
}

}  // namespace bf
