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

// Wavefront (64 lanes) reductions by butterfly shuffles; every lane gets the
// result.  Fixed order, so results are deterministic.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ cd wave_sum(cd v) {
  v.re = wave_sum(v.re);
  v.im = wave_sum(v.im);
  return v;
}

}  // namespace bf
