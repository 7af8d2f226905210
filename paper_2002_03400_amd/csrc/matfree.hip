// Black-box products for the built-in test operators: entries of op(A) are
// produced on the fly (never stored) and multiplied into a block of columns.
//
// Y[i, g*ncols + c] = sum_{j in seg_g} E(i, j) X[j, c]    (Sec. 4.1 structured
// samples: group g is the product with the random block living on node g).
//
// Layout: one workgroup of 8 waves owns 128 output rows of one group, up to
// 48 columns, and one slice of the group's inner range (split-K when there
// are too few row tiles to fill 256 CUs); chunks of TK inner points (their
// coordinates and the TK x 64 block of X) are staged in LDS.  Split-K
// partials go to an FP64 scratch buffer and are summed in a fixed order
// (deterministic).
//
// Precision: entries are FP32-accurate (FP64 phase reduction, FP32 sin/cos
// and 1/r) and the inputs are complex64.  A recursive FP32 sum over the
// 10^4..10^5 terms of one output would carry a relative rounding error of
// order 1e-6..1e-5 -- the size of the tolerances of interest, inflating every
// sampled rank -- so products are accumulated in FP64 on the matrix cores.
#include "bf_internal.h"
#include "cplx.h"

namespace bf {

constexpr int MF_THREADS = 512;   // 8 waves share each staged chunk of X
constexpr int MF_TK = 64;
// inner length of the product being launched (for the profiler's accounting)
static thread_local int64_t g_matfree_nin = 0;

// ---- entry functors ------------------------------------------------------

// sin and cos of 2 pi t for a phase t given in revolutions (FP64, |t| < 2^29).
// The phase is reduced in FP64 to the nearest quarter revolution,
// t = q/4 + y with |y| <= 1/8, so x = 2 pi y lies in [-pi/4, pi/4] and only
// its FP32 rounding (< 3e-8 rad) enters; sin x and cos x are the Taylor
// polynomials through x^9 and x^10 (truncation below 2e-9 on that interval),
// then rotated by q quarter turns.
__device__ __forceinline__ void sincos_rev(double t, float* s, float* c) {
  const double q = rint(4.0 * t);
  const double y = fma(-0.25, q, t);
  const float x = (float)(y * 6.283185307179586477);
  const float x2 = x * x;
  float sp = fmaf(x2, 2.75573192e-6f, -1.98412698e-4f);   // 1/9!, -1/7!
  sp = fmaf(x2, sp, 8.33333333e-3f);                       // 1/5!
  sp = fmaf(x2, sp, -1.66666667e-1f);                      // -1/3!
  sp = x * fmaf(x2, sp, 1.0f);
  float cp = fmaf(x2, -2.75573192e-7f, 2.48015873e-5f);    // -1/10!, 1/8!
  cp = fmaf(x2, cp, -1.38888889e-3f);                      // -1/6!
  cp = fmaf(x2, cp, 4.16666667e-2f);                       // 1/4!
  cp = fmaf(x2, cp, -0.5f);                                // -1/2!
  cp = fmaf(x2, cp, 1.0f);
  const int n = (int)q & 3;
  const float sv = (n & 1) ? cp : sp;
  const float cv = (n & 1) ? sp : cp;
  *s = (n & 2) ? -sv : sv;
  *c = ((n ^ (n >> 1)) & 1) ? -cv : cv;
}

// exp(i k r)/r, r = |p - q|: r from an FP32 square root refined by one
// FP64 Newton step (relative error ~1e-14, so the phase k r / 2pi stays
// accurate to ~1e-9 revolutions for k r up to 1e5), 1/r from the FP32
// reciprocal.  sign = -1 gives the conjugate (entries of A^H with the point
// roles swapped).
struct SegEntry {
  PointSet out, in;
  double kk;   // k / (2 pi)
  float sign;
  struct Row { double x, y; };
  struct Col { double x, y; };
  __device__ Row row(int64_t i) const { return Row{out.x[i], out.y[i]}; }
  __device__ Col col(int64_t j) const { return Col{in.x[j], in.y[j]}; }
  __device__ cf entry(const Row& r, const Col& c) const {
    const double dx = r.x - c.x, dy = r.y - c.y;
    const double r2 = fma(dx, dx, dy * dy);
    const float rf = __builtin_amdgcn_sqrtf((float)r2);
    const float inv = __builtin_amdgcn_rcpf(rf);
    const double rd = (double)rf;
    const double rr = fma(fma(-rd, rd, r2), 0.5 * (double)inv, rd);
    float s, co;
    sincos_rev(rr * kk, &s, &co);
    return cf{co * inv, sign * s * inv};
  }
};

// exp(2 pi i (j xi / n + c_j |xi|)).  j * xi is an exact integer (< 2^53),
// so j xi / n is formed in FP64 with one rounding before the reduction.
// Forward: output index j (row), inner index k (xi = k - n/2).
struct FioEntry {
  int64_t n;
  double inv_n;
  const double* cx;  // c(x_j), FP64
  struct Row { double j; double c; };
  struct Col { double xi; };
  __device__ Row row(int64_t j) const { return Row{(double)j, cx[j]}; }
  __device__ Col col(int64_t k) const { return Col{(double)(k - n / 2)}; }
  __device__ cf entry(const Row& r, const Col& c) const {
    const double ph = fma(r.j * c.xi, inv_n, r.c * fabs(c.xi));
    float s, co;
    sincos_rev(ph, &s, &co);
    return cf{co, s};
  }
};
// Adjoint: output index k, inner index j: conj(A_jk).
struct FioAdjEntry {
  int64_t n;
  double inv_n;
  const double* cx;
  struct Row { double xi; };
  struct Col { double j; double c; };
  __device__ Row row(int64_t k) const { return Row{(double)(k - n / 2)}; }
  __device__ Col col(int64_t j) const { return Col{(double)j, cx[j]}; }
  __device__ cf entry(const Row& r, const Col& c) const {
    const double ph = fma(c.j * r.xi, inv_n, c.c * fabs(r.xi));
    float s, co;
    sincos_rev(ph, &s, &co);
    return cf{co, -s};
  }
};

struct DenseEntry {
  const bf_c64* A;
  int64_t lda;
  int adjoint;
  struct Row { int64_t i; };
  struct Col { int64_t j; };
  __device__ Row row(int64_t i) const { return Row{i}; }
  __device__ Col col(int64_t j) const { return Col{j}; }
  __device__ cf entry(const Row& r, const Col& c) const {
    if (!adjoint) {
      bf_c64 a = A[c.j * lda + r.i];
      return cf{a.re, a.im};
    }
    bf_c64 a = A[r.i * lda + c.j];
    return cf{a.re, -a.im};
  }
};

// ---- kernel ----------------------------------------------------------------
//
// Complex products on the matrix cores in FP64 (v_mfma_f64_16x16x4f64; on
// gfx950 the FP64 matrix rate equals the FP64 vector rate, but the matrix
// cores run beside the vector ALUs that evaluate the entries).  A wave owns
// 16*MF_H output rows x 16*NT columns; per step of 4 inner points lane l
// evaluates the entries (row l % 16 of each 16-row tile, inner point l / 16)
// -- its own slots of the A operand -- and reads its B slots (inner point l / 16,
// column l % 16) from the X chunk staged in LDS.  Complex products use three
// real products (Gauss):  P1 = Re a Re x, P2 = Im a Im x,
// P3 = (Re a + Im a)(Re x + Im x);  Re y = P1 - P2, Im y = P3 - P1 - P2.
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int MF_H = 1;                                  // 16-row tiles per wave
constexpr int MF_ROWS = (MF_THREADS / 64) * 16 * MF_H;   // output rows per workgroup

template <class E, int NT, typename Tout>
__global__ __launch_bounds__(MF_THREADS) void matfree_kernel(
    E e, int64_t nout, const bf_c64* __restrict__ X, int64_t ldx, int32_t ncols, int32_t c0,
    int32_t width, Tout* __restrict__ Y, int64_t ldy, int64_t ycols,
    const int64_t* __restrict__ seg, int32_t nsplit) {
  constexpr int NC = 16 * NT;
  __shared__ typename E::Col cols[MF_TK];
  // row stride NC + 1: consecutive inner points (the staging write pattern)
  // land in distinct banks
  __shared__ cf xs[MF_TK][NC + 1];
  const int g = blockIdx.y;
  const int z = blockIdx.z;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t row0 = (int64_t)blockIdx.x * MF_ROWS + wave * 16 * MF_H;
  const int kq = lane >> 4;       // inner point of the step held by this lane
  const int lc = lane & 15;       // A row / B column within a 16-wide tile
  const int64_t j0 = seg[g], j1 = seg[g + 1];
  const int64_t len = j1 - j0;
  const int64_t chunk = (len + nsplit - 1) / nsplit;
  const int64_t a = j0 + (int64_t)z * chunk;
  const int64_t b = (a + chunk < j1) ? a + chunk : j1;
  const int nc = width < NC ? width : NC;

  doublex4 p1[MF_H][NT], p2[MF_H][NT], p3[MF_H][NT];
#pragma unroll
  for (int h = 0; h < MF_H; ++h)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) { p1[h][t][v] = 0.0; p2[h][t][v] = 0.0; p3[h][t][v] = 0.0; }
  typename E::Row rw[MF_H];
#pragma unroll
  for (int h = 0; h < MF_H; ++h) {
    const int64_t r = row0 + 16 * h + lc;
    rw[h] = e.row(r < nout ? r : nout - 1);
  }

  for (int64_t jb = a; jb < b; jb += MF_TK) {
    const int tk = (b - jb < MF_TK) ? (int)(b - jb) : MF_TK;
    __syncthreads();
    for (int idx = threadIdx.x; idx < MF_TK * NC; idx += MF_THREADS) {
      const int jj = idx % MF_TK, c = idx / MF_TK;
      bf_c64 v = {0.f, 0.f};
      if (jj < tk && c < nc) v = X[(int64_t)(c0 + c) * ldx + jb + jj];
      xs[jj][c] = cf{v.re, v.im};
    }
    if (threadIdx.x < tk) cols[threadIdx.x] = e.col(jb + threadIdx.x);
    __syncthreads();
    const int nsteps = (tk + 3) >> 2;
    for (int q = 0; q < nsteps; ++q) {
      const int jj = 4 * q + kq;
      double ar[MF_H], ai[MF_H], as[MF_H];
#pragma unroll
      for (int h = 0; h < MF_H; ++h) {
        cf ev = cf{0.f, 0.f};
        if (jj < tk) ev = e.entry(rw[h], cols[jj]);
        ar[h] = ev.re;
        ai[h] = ev.im;
        as[h] = (double)ev.re + (double)ev.im;
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const cf xv = xs[jj][t * 16 + lc];
        const double xr = xv.re, xi = xv.im, xsum = (double)xv.re + (double)xv.im;
#pragma unroll
        for (int h = 0; h < MF_H; ++h) {
          p1[h][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[h], xr, p1[h][t], 0, 0, 0);
          p2[h][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[h], xi, p2[h][t], 0, 0, 0);
          p3[h][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(as[h], xsum, p3[h][t], 0, 0, 0);
        }
      }
    }
  }
  // accumulator layout of a 16x16 f64 MFMA tile on gfx950: lane l, register
  // v holds row l / 16 + 4 v, column l % 16 (A[i][k] sits in lane i + 16 k,
  // B[k][j] in lane j + 16 k)
  Tout* yz = Y + (int64_t)z * ycols * ldy + ((int64_t)g * ncols + c0) * ldy;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int c = t * 16 + lc;
    if (c < nc) {
#pragma unroll
      for (int h = 0; h < MF_H; ++h)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t r = row0 + 16 * h + kq + 4 * v;
          if (r < nout) {
            Tout o;
            o.re = p1[h][t][v] - p2[h][t][v];
            o.im = p3[h][t][v] - p1[h][t][v] - p2[h][t][v];
            yz[(int64_t)c * ldy + r] = o;
          }
        }
    }
  }
}

// ---- split-BF16 kernel --------------------------------------------------
//
// The same product on the BF16 matrix cores (v_mfma_f32_32x32x16_bf16), which
// on gfx950 run concurrently with the vector ALUs that evaluate the entries
// (the FP32/FP64 matrix instructions do not).  Every entry a and input x is
// split into three BF16 terms, a = a1 + a2 + a3 (a1 = bf16(a),
// a2 = bf16(a - a1), a3 = bf16(a - a1 - a2)), and the products keep every
// term down to 2^-24 relative:  a x ~ a1x1 + a1x2 + a2x1 + a1x3 + a3x1 + a2x2
// -- six MFMAs per real product, 24 per complex tile step
// (Re += ar xr - ai xi, Im += ar xi + ai xr).  A wave owns 32 rows x 32 NT
// columns; per step of 16 inner points lane l evaluates its 8 A-operand
// entries (row l % 32, inner points 8 (l / 32) .. +7) and reads its B operands
// (8 inner points of column l % 32) from the split planes staged in LDS.
// Each step's FP32 tile sums (16 terms) are added into FP64 registers, so the
// only FP32 summation error is that of 16-term sums.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ void split3(float x, __bf16& h, __bf16& m, __bf16& l) {
  h = (__bf16)x;
  const float r1 = x - (float)h;
  m = (__bf16)r1;
  l = (__bf16)(r1 - (float)m);
}

constexpr int BF_TK = 64;            // inner points per staged chunk (4 MFMA steps)
constexpr int BF_KP = BF_TK + 8;     // padded k stride of the split planes (bank spread)
constexpr int BF_WAVES = 4;
constexpr int BF_ROWS = 32 * BF_WAVES;

template <class E, int NT, typename Tout>
__global__ __launch_bounds__(64 * BF_WAVES) void matfree_bf16_kernel(
    E e, int64_t nout, const bf_c64* __restrict__ X, int64_t ldx, int32_t ncols, int32_t c0,
    int32_t width, Tout* __restrict__ Y, int64_t ldy, int64_t ycols,
    const int64_t* __restrict__ seg, int32_t nsplit) {
  constexpr int NC = 32 * NT;
  __shared__ typename E::Col cols[BF_TK];
  // split planes: [term 0..2][re/im][column][k], 16 bytes = 8 consecutive k
  __shared__ __attribute__((aligned(16))) __bf16 xs[3][2][NC][BF_KP];
  const int g = blockIdx.y;
  const int z = blockIdx.z;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t row0 = (int64_t)blockIdx.x * BF_ROWS + wave * 32;
  const int64_t myrow = row0 + (lane & 31);
  const int kh = lane >> 5;       // which 8 of the step's 16 inner points
  const int lc = lane & 31;
  const int64_t j0 = seg[g], j1 = seg[g + 1];
  const int64_t len = j1 - j0;
  const int64_t chunk = (len + nsplit - 1) / nsplit;
  const int64_t a = j0 + (int64_t)z * chunk;
  const int64_t b = (a + chunk < j1) ? a + chunk : j1;
  const int nc = width < NC ? width : NC;

  double fr[NT][16], fi[NT][16];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) { fr[t][v] = 0.0; fi[t][v] = 0.0; }
  const typename E::Row rw = e.row(myrow < nout ? myrow : nout - 1);

  for (int64_t jb = a; jb < b; jb += BF_TK) {
    const int tk = (b - jb < BF_TK) ? (int)(b - jb) : BF_TK;
    __syncthreads();
    for (int idx = threadIdx.x; idx < BF_TK * NC; idx += 64 * BF_WAVES) {
      const int kk = idx % BF_TK, c = idx / BF_TK;
      bf_c64 v = {0.f, 0.f};
      if (kk < tk && c < nc) v = X[(int64_t)(c0 + c) * ldx + jb + kk];
      split3(v.re, xs[0][0][c][kk], xs[1][0][c][kk], xs[2][0][c][kk]);
      split3(v.im, xs[0][1][c][kk], xs[1][1][c][kk], xs[2][1][c][kk]);
    }
    if (threadIdx.x < tk) cols[threadIdx.x] = e.col(jb + threadIdx.x);
    __syncthreads();
    const int nsteps = (tk + 15) >> 4;
    for (int q = 0; q < nsteps; ++q) {
      const int kb = 16 * q + 8 * kh;
      bf16x8 ar[3], ai[3], an[3];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        cf ev = cf{0.f, 0.f};
        if (kb + u < tk) ev = e.entry(rw, cols[kb + u]);
        __bf16 h, m, l;
        split3(ev.re, h, m, l);
        ar[0][u] = h; ar[1][u] = m; ar[2][u] = l;
        split3(ev.im, h, m, l);
        ai[0][u] = h; ai[1][u] = m; ai[2][u] = l;
        an[0][u] = -h; an[1][u] = -m; an[2][u] = -l;
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        bf16x8 xr[3], xi[3];
#pragma unroll
        for (int p = 0; p < 3; ++p) {
          xr[p] = *reinterpret_cast<const bf16x8*>(&xs[p][0][t * 32 + lc][kb]);
          xi[p] = *reinterpret_cast<const bf16x8*>(&xs[p][1][t * 32 + lc][kb]);
        }
        floatx16 R = {}, I = {};
        // term pairs (p, q) with p + q <= 2 (0-based): 00 01 10 02 20 11
#define BF_PAIR(P, Q)                                                              \
        R = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar[P], xr[Q], R, 0, 0, 0);      \
        R = __builtin_amdgcn_mfma_f32_32x32x16_bf16(an[P], xi[Q], R, 0, 0, 0);      \
        I = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar[P], xi[Q], I, 0, 0, 0);      \
        I = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ai[P], xr[Q], I, 0, 0, 0);
        BF_PAIR(2, 0) BF_PAIR(0, 2) BF_PAIR(1, 1) BF_PAIR(1, 0) BF_PAIR(0, 1) BF_PAIR(0, 0)
#undef BF_PAIR
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          fr[t][v] += (double)R[v];
          fi[t][v] += (double)I[v];
        }
      }
    }
  }
  // accumulator layout of a 32x32 MFMA tile on gfx950: lane l, register v
  // holds row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32
  Tout* yz = Y + (int64_t)z * ycols * ldy + ((int64_t)g * ncols + c0) * ldy;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int c = t * 32 + lc;
    if (c < nc) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t r = row0 + 8 * (v >> 2) + 4 * kh + (v & 3);
        if (r < nout) {
          Tout o;
          o.re = fr[t][v];
          o.im = fi[t][v];
          yz[(int64_t)c * ldy + r] = o;
        }
      }
    }
  }
}

// Y(:, col) = sum_z P[z](:, col) over the FP64 split planes (fixed order).
__global__ void split_reduce_kernel(const bf_c128* __restrict__ P, int64_t nout, int64_t ycols,
                                    int32_t nsplit, bf_c64* __restrict__ Y, int64_t ldy) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nout * ycols) return;
  int64_t r = idx % nout, c = idx / nout;
  double re = 0.0, im = 0.0;
  for (int z = 0; z < nsplit; ++z) {
    bf_c128 v = P[((int64_t)z * ycols + c) * nout + r];
    re += v.re;
    im += v.im;
  }
  Y[c * ldy + r] = bf_c64{(float)re, (float)im};
}

template <class E, int NT, typename Tout>
static void launch_nt(const E& e, int64_t nout, const bf_c64* X, int64_t ldx, int32_t ncols,
                      int32_t c0, int32_t width, Tout* Y, int64_t ldy, int64_t ycols,
                      const int64_t* seg_dev, int32_t nseg, int32_t nsplit, hipStream_t s) {
  dim3 grid((unsigned)((nout + MF_ROWS - 1) / MF_ROWS), (unsigned)nseg, (unsigned)nsplit);
  // algorithmic work of this launch: every (output row, inner point) pair
  // once per column of the chunk; bytes = the X chunk read and Y written once
  const double nc = (double)std::min<int32_t>(16 * NT, width);
  const double nin = (double)g_matfree_nin;
  ProfScope ps(BF_KC_MATFREE, s, 8.0 * (double)nout * nin * nc,
               8.0 * nc * (nin + (double)nout * nseg));
  hipLaunchKernelGGL((matfree_kernel<E, NT, Tout>), grid, dim3(MF_THREADS), 0, s, e, nout, X, ldx,
                     ncols, c0, width, Y, ldy, ycols, seg_dev, nsplit);
  BF_HIP(hipGetLastError());
}

template <class E, int NT, typename Tout>
static void launch_bf16(const E& e, int64_t nout, const bf_c64* X, int64_t ldx, int32_t ncols,
                        int32_t c0, int32_t width, Tout* Y, int64_t ldy, int64_t ycols,
                        const int64_t* seg_dev, int32_t nseg, int32_t nsplit, hipStream_t s) {
  dim3 grid((unsigned)((nout + BF_ROWS - 1) / BF_ROWS), (unsigned)nseg, (unsigned)nsplit);
  const double nc = (double)std::min<int32_t>(32 * NT, width);
  const double nin = (double)g_matfree_nin;
  ProfScope ps(BF_KC_MATFREE, s, 8.0 * (double)nout * nin * nc,
               8.0 * nc * (nin + (double)nout * nseg));
  hipLaunchKernelGGL((matfree_bf16_kernel<E, NT, Tout>), grid, dim3(64 * BF_WAVES), 0, s, e, nout,
                     X, ldx, ncols, c0, width, Y, ldy, ycols, seg_dev, nsplit);
  BF_HIP(hipGetLastError());
}

template <class E, typename Tout>
static void launch_chunk(const E& e, int64_t nout, const bf_c64* X, int64_t ldx, int32_t ncols,
                         int32_t c0, int32_t width, Tout* Y, int64_t ldy, int64_t ycols,
                         const int64_t* seg_dev, int32_t nseg, int32_t nsplit, hipStream_t s) {
  if (width <= 16)
    launch_nt<E, 1>(e, nout, X, ldx, ncols, c0, width, Y, ldy, ycols, seg_dev, nseg, nsplit, s);
  else if (width <= 32)
    launch_nt<E, 2>(e, nout, X, ldx, ncols, c0, width, Y, ldy, ycols, seg_dev, nseg, nsplit, s);
  else
    launch_nt<E, 3>(e, nout, X, ldx, ncols, c0, width, Y, ldy, ycols, seg_dev, nseg, nsplit, s);
}

template <class E, typename Tout>
static void launch_chunk_prec(int prec, const E& e, int64_t nout, const bf_c64* X, int64_t ldx,
                              int32_t ncols, int32_t c0, int32_t width, Tout* Y, int64_t ldy,
                              int64_t ycols, const int64_t* seg_dev, int32_t nseg, int32_t nsplit,
                              hipStream_t s) {
  if (prec == BF_PREC_BF16X3) {
    if (width <= 32)
      launch_bf16<E, 1>(e, nout, X, ldx, ncols, c0, width, Y, ldy, ycols, seg_dev, nseg, nsplit, s);
    else
      launch_bf16<E, 2>(e, nout, X, ldx, ncols, c0, width, Y, ldy, ycols, seg_dev, nseg, nsplit, s);
  } else {
    launch_chunk(e, nout, X, ldx, ncols, c0, width, Y, ldy, ycols, seg_dev, nseg, nsplit, s);
  }
}

template <class E>
static void run_matfree(int prec, const E& e, int64_t nout, int64_t nin, const bf_c64* X,
                        int64_t ldx, int64_t ncols, bf_c64* Y, int64_t ldy,
                        const int64_t* seg_host, int32_t nseg, hipStream_t s) {
  if (nout <= 0 || ncols <= 0) return;
  std::vector<int64_t> segv;
  if (seg_host) {
    segv.assign(seg_host, seg_host + nseg + 1);
  } else {
    nseg = 1;
    segv = {0, nin};
  }
  BF_CHECK(nseg >= 1 && nseg <= 65535, BF_EINVAL, "bad segment count");
  int64_t maxlen = 0;
  for (int g = 0; g < nseg; ++g) {
    BF_CHECK(segv[g] <= segv[g + 1] && segv[g] >= 0 && segv[g + 1] <= nin, BF_EINVAL,
             "segments must partition the input rows");
    maxlen = std::max(maxlen, segv[g + 1] - segv[g]);
  }
  // split-K so that row tiles x groups x splits reaches ~2048 workgroups,
  // keeping at least 512 inner points per split.
  const int64_t rows_per_wg = prec == BF_PREC_BF16X3 ? BF_ROWS : MF_ROWS;
  int64_t tiles = ((nout + rows_per_wg - 1) / rows_per_wg) * nseg;
  int64_t want = (2048 + tiles - 1) / tiles;
  int64_t cap = std::max<int64_t>(1, maxlen / 512);
  int32_t nsplit = (int32_t)std::max<int64_t>(1, std::min<int64_t>({want, cap, 64}));

  DevBuf<int64_t> seg_dev(segv.size(), s);
  BF_HIP(hipMemcpyAsync(seg_dev.p, segv.data(), segv.size() * sizeof(int64_t),
                        hipMemcpyHostToDevice, s));
  const int64_t ycols = (int64_t)nseg * ncols;
  g_matfree_nin = segv[nseg] - segv[0];
  DevBuf<bf_c128> part;
  if (nsplit > 1) part = DevBuf<bf_c128>((size_t)nsplit * ycols * nout, s);
  const int64_t maxw = prec == BF_PREC_BF16X3 ? 64 : 48;
  const int64_t nchunk = (ncols + maxw - 1) / maxw;
  const int64_t cw = (ncols + nchunk - 1) / nchunk;   // balanced widths <= maxw
  for (int64_t c0 = 0; c0 < ncols; c0 += cw) {
    const int32_t w = (int32_t)std::min<int64_t>(cw, ncols - c0);
    if (nsplit > 1)
      launch_chunk_prec(prec, e, nout, X, ldx, (int32_t)ncols, (int32_t)c0, w, part.p, nout, ycols,
                        seg_dev.p, nseg, nsplit, s);
    else
      launch_chunk_prec(prec, e, nout, X, ldx, (int32_t)ncols, (int32_t)c0, w, Y, ldy, ycols,
                        seg_dev.p, nseg, nsplit, s);
  }
  if (nsplit > 1) {
    int64_t tot = nout * ycols;
    ProfScope ps(BF_KC_OTHER, s, 0.0, 16.0 * nsplit * tot + 8.0 * tot);
    hipLaunchKernelGGL(split_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                       part.p, nout, ycols, nsplit, Y, ldy);
    BF_HIP(hipGetLastError());
  }
}

void launch_segkernel(int prec, PointSet out_pts, int64_t nout, PointSet in_pts, int64_t nin,
                      double k_over_2pi, int sign, const bf_c64* X, int64_t ldx, int64_t ncols,
                      bf_c64* Y, int64_t ldy, const int64_t* seg_host, int32_t nseg,
                      hipStream_t s) {
  SegEntry e{out_pts, in_pts, k_over_2pi, (float)sign};
  run_matfree(prec, e, nout, nin, X, ldx, ncols, Y, ldy, seg_host, nseg, s);
}

void launch_fio(int prec, int64_t n, const double* cx_dev, int adjoint, const bf_c64* X,
                int64_t ldx, int64_t ncols, bf_c64* Y, int64_t ldy, const int64_t* seg_host,
                int32_t nseg, hipStream_t s) {
  if (!adjoint) {
    FioEntry e{n, 1.0 / (double)n, cx_dev};
    run_matfree(prec, e, n, n, X, ldx, ncols, Y, ldy, seg_host, nseg, s);
  } else {
    FioAdjEntry e{n, 1.0 / (double)n, cx_dev};
    run_matfree(prec, e, n, n, X, ldx, ncols, Y, ldy, seg_host, nseg, s);
  }
}

void launch_dense(int prec, const bf_c64* A, int64_t m, int64_t n, int64_t lda, int adjoint,
                  const bf_c64* X, int64_t ldx, int64_t ncols, bf_c64* Y, int64_t ldy,
                  const int64_t* seg_host, int32_t nseg, hipStream_t s) {
  DenseEntry e{A, lda, adjoint};
  if (!adjoint)
    run_matfree(prec, e, m, n, X, ldx, ncols, Y, ldy, seg_host, nseg, s);
  else
    run_matfree(prec, e, n, m, X, ldx, ncols, Y, ldy, seg_host, nseg, s);
}

}  // namespace bf
