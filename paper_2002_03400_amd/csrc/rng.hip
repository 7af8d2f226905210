// Counter-based complex Gaussians for the random matrices of Alg. 2
// (structured samples of Sec. 4.1).
//
// Each entry is a pure function of (seed, tag, row, col):
//   o = Philox4x64-10(counter = (row, col, tag, 0), key = (seed, 0))
//   u_q = ((o_q >> 12) + 1/2) 2^-52 in (0, 1),  q = 0, 1
//   g = sqrt(-2 ln u_0) (cos 2 pi u_1 + i sin 2 pi u_1) / sqrt(2)
// Philox4x64-10 follows Salmon et al., SC'11 (published multipliers and Weyl
// key increments).  The draw is therefore independent of launch order, grid
// shape and of which other requests share the device.  The random matrices
// of the construction round each part of g to the nearest BF16 value (ties
// to even), so the black-box products can take them as exact BF16 operands.
#include "bf_internal.h"
#include "cplx.h"

namespace bf {

__device__ __forceinline__ void philox_round(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
  uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
  uint64_t n0 = hi1 ^ c[1] ^ k0;
  uint64_t n2 = hi0 ^ c[3] ^ k1;
  c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
}

__device__ cd gauss_entry(uint64_t seed, uint64_t tag, uint64_t row, uint64_t col) {
  uint64_t c[4] = {row, col, tag, 0};
  uint64_t k0 = seed, k1 = 0;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B97F4A7C15ull; k1 += 0xBB67AE8584CAA73Bull; }
    philox_round(c, k0, k1);
  }
  const double two52 = 2.220446049250313080847e-16;  // 2^-52
  double u0 = ((double)(c[0] >> 12) + 0.5) * two52;
  double u1 = ((double)(c[1] >> 12) + 0.5) * two52;
  double rad = sqrt(-2.0 * log(u0)) * 0.70710678118654752440;
  double s, co;
  sincospi(2.0 * u1, &s, &co);
  return cd{rad * co, rad * s};
}

// Nearest BF16 value of an FP64 value (8 significant bits, ties to even),
// by integer rounding of the 52-bit fraction to 7 bits.
__device__ __forceinline__ double round_bf16(double x) {
  const uint64_t drop = (uint64_t(1) << 45) - 1, half = (uint64_t(1) << 44) - 1;
  uint64_t b = (uint64_t)__double_as_longlong(x);
  b = (b + half + ((b >> 45) & 1)) & ~drop;
  return __longlong_as_double((long long)b);
}

// One thread per entry of a column: grid (ceil(rows/256), ncols).
__global__ void gauss_samples_kernel(bf_c64* X, int64_t rows, int64_t /*ncols: grid y*/,
                                     int32_t level, const uint64_t* tags, const int32_t* widths,
                                     uint64_t seed) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t c = blockIdx.y;
  if (r >= rows) return;
  // node of row r at `level`: i = ceil((r+1) 2^level / rows) - 1
  int64_t g = ((((r + 1) << level) + rows - 1) / rows) - 1;
  bf_c64 out = {0.f, 0.f};
  if (c < widths[g]) {
    cd v = gauss_entry(seed, tags[g], (uint64_t)r, (uint64_t)c);
    out.re = (float)round_bf16(v.re);   // exact: 8 significant bits
    out.im = (float)round_bf16(v.im);
  }
  X[c * rows + r] = out;
}

__global__ void gauss_f64_kernel(bf_c128* X, int64_t rows, int64_t row0, uint64_t tag,
                                 uint64_t seed) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t c = blockIdx.y;
  if (r >= rows) return;
  cd v = gauss_entry(seed, tag, (uint64_t)(row0 + r), (uint64_t)c);
  X[c * rows + r] = bf_c128{v.re, v.im};
}

void launch_gauss_samples(bf_c64* X, int64_t rows, int64_t ncols, int32_t level,
                          const uint64_t* tags_dev, const int32_t* widths_dev, uint64_t seed,
                          hipStream_t s) {
  if (rows <= 0 || ncols <= 0) return;
  BF_CHECK(ncols <= 65535, BF_ERANK, "sample width too large");
  dim3 grid((unsigned)((rows + 255) / 256), (unsigned)ncols);
  ProfScope ps(BF_KC_OTHER, s, 0.0, 8.0 * rows * ncols);
  hipLaunchKernelGGL(gauss_samples_kernel, grid, dim3(256), 0, s, X, rows, ncols, level,
                     tags_dev, widths_dev, seed);
  BF_HIP(hipGetLastError());
}

void launch_gauss_f64(bf_c128* X, int64_t rows, int64_t ncols, int64_t row0, uint64_t tag,
                      uint64_t seed, hipStream_t s) {
  if (rows <= 0 || ncols <= 0) return;
  dim3 grid((unsigned)((rows + 255) / 256), (unsigned)ncols);
  hipLaunchKernelGGL(gauss_f64_kernel, grid, dim3(256), 0, s, X, rows, row0, tag, seed);
  BF_HIP(hipGetLastError());
}

}  // namespace bf
