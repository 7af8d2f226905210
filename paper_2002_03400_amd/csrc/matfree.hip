// Black-box products for the built-in test operators: entries of op(A) are
// produced on the fly (never stored) and multiplied into a block of columns.
//
// Y[i, g*ncols + c] = sum_{j in seg_g} E(i, j) X[j, c]    (Sec. 4.1 structured
// samples: group g is the product with the random block living on node g).
//
// Layout: one workgroup of 8 waves owns 128 output rows of one group, up to
// 48 (FP64 path) or 80 (split-BF16 path) columns, every matrix entry being
// evaluated once for all of them, and one slice of the group's inner range
// (split-K when there
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
#include <array>
#include <atomic>
#include <map>
#include <mutex>

#include "bf_internal.h"
#include "cplx.h"

namespace bf {

constexpr int MF_THREADS = 512;   // 8 waves share each staged chunk of X
constexpr int MF_TK = 64;
// inner length of the product being launched (for the profiler's accounting)
static thread_local int64_t g_matfree_nin = 0;

// ---- entry functors ------------------------------------------------------

// amp * exp(i pi a b) for a phase t = a b given in half revolutions (FP64,
// |t| < 2^51; a b is never rounded on its own).  The phase is reduced in FP64
// to the nearest half revolution q by adding 1.5 * 2^52 (the sum rounds to
// q + 1.5 * 2^52, whose low word holds q mod 2^32, so q's parity is its low
// bit); y = t - q, |y| <= 1/2, is then formed with one rounding, and only the
// FP32 rounding of y (< 2^-26 half revolutions, 4.7e-8 rad) enters.  sin(pi y)
// and cos(pi y) are minimax polynomials in y on [-1/2, 1/2]
// (linear-programming fit, coefficients rounded to FP32 one at a time from the
// lowest order, each rounding compensated by refitting the higher ones;
// errors before FP32 evaluation 2.8e-8 relative -- the FP32 rounding of pi --
// and 1.2e-9 absolute), and (-1)^q is applied as a sign flip of amp.  An FP32
// emulation against exp(i theta) in FP64 over 2e6 phases up to 2e4 rad stays
// within 1.7e-7 (rms 4.3e-8); csrc/fit_cispi.py refits and rechecks.
__device__ __forceinline__ cf cis_pi(double a, double b, float amp) {
  constexpr double kRound = 0x1.8p52;
  const double v = fma(a, b, kRound);
  const float y = (float)fma(a, b, kRound - v);
  const uint32_t flip = (uint32_t)__double2loint(v) << 31;
  const float y2 = y * y;
  float sp = fmaf(y2, 0x1.3b9a6ep-4f, -0x1.323be0p-1f);
  sp = fmaf(y2, sp, 0x1.46690ap+1f);
  sp = fmaf(y2, sp, -0x1.4abbd0p+2f);
  sp = fmaf(y2, sp, 0x1.921fb6p+1f);
  float cp = fmaf(y2, -0x1.88bf7ap-6f, 0x1.e0a362p-3f);
  cp = fmaf(y2, cp, -0x1.55cd2ap+0f);
  cp = fmaf(y2, cp, 0x1.03c1d4p+2f);
  cp = fmaf(y2, cp, -0x1.3bd3ccp+2f);
  const float am = __uint_as_float(__float_as_uint(amp) ^ flip);
  return cf{fmaf(y2, cp, 1.0f) * am, (y * sp) * am};
}

// exp(i k r)/r, r = |p - q|: y = 1/r from the FP32 reciprocal square root
// (the amplitude), and the phase k r = k h (1 + e / 2) with h = r^2 y and
// e = 1 - r^2 y^2 in FP64 -- one Newton step for 1/sqrt(r^2) folded into the
// phase scale, relative error ~1.5 (2^-23)^2 ~ 1e-14, so k r stays accurate
// to ~1e-9 revolutions for k r / 2pi up to 1e5.  The conjugate (entries of
// A^H with the point roles swapped) uses the negated phase scale: sin is odd,
// cos even, and every rounding here and in cis_pi is symmetric (q = -q'
// exactly, ties to even), so it is exactly the conjugate.
struct SegEntry {
  static constexpr int kKind = 1;
  PointSet out, in;
  double k2;   // +-k / pi: k r in half revolutions, the sign selecting A or conj
  double k2h;  // k2 / 2
  struct Row { double x, y; };
  struct Col { double x, y; };
  __device__ Row row(int64_t i) const { return Row{out.x[i], out.y[i]}; }
  __device__ Col col(int64_t j) const { return Col{in.x[j], in.y[j]}; }
  __device__ cf entry(const Row& r, const Col& c) const {
    const double dx = r.x - c.x, dy = r.y - c.y;
    const double r2 = fma(dx, dx, dy * dy);
    const float inv = __builtin_amdgcn_rsqf((float)r2);
    const double y = (double)inv, h = r2 * y;
    return cis_pi(h, fma(fma(-h, y, 1.0), k2h, k2), inv);
  }
};

// The same kernel on 3D points (eq. 3dkernel: the two semi-spheres).
struct Seg3Entry {
  static constexpr int kKind = 2;
  PointSet out, in;
  double k2, k2h;
  struct Row { double x, y, z; };
  struct Col { double x, y, z; };
  __device__ Row row(int64_t i) const { return Row{out.x[i], out.y[i], out.z[i]}; }
  __device__ Col col(int64_t j) const { return Col{in.x[j], in.y[j], in.z[j]}; }
  __device__ cf entry(const Row& r, const Col& c) const {
    const double dx = r.x - c.x, dy = r.y - c.y, dz = r.z - c.z;
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const float inv = __builtin_amdgcn_rsqf((float)r2);
    const double y = (double)inv, h = r2 * y;
    return cis_pi(h, fma(fma(-h, y, 1.0), k2h, k2), inv);
  }
};

// exp(2 pi i (j xi / n + c_j |xi|)).  j * xi is an exact integer (< 2^53),
// so the phase (in half revolutions: the exact scalings 2/n and 2 c_j) is
// formed in FP64 with one rounding before the reduction.
// Forward: output index j (row), inner index k (xi = k - n/2).
struct FioEntry {
  static constexpr int kKind = 3;
  int64_t n;
  double inv_n2;     // 2 / n
  const double* cx;  // c(x_j), FP64
  struct Row { double j; double c2; };
  struct Col { double xi; };
  __device__ Row row(int64_t j) const { return Row{(double)j, 2.0 * cx[j]}; }
  __device__ Col col(int64_t k) const { return Col{(double)(k - n / 2)}; }
  __device__ cf entry(const Row& r, const Col& c) const {
    return cis_pi(fma(r.j * c.xi, inv_n2, r.c2 * fabs(c.xi)), 1.0, 1.0f);
  }
};
// Adjoint: output index k, inner index j: conj(A_jk), from the negated phase
// (exact, as for SegEntry).
struct FioAdjEntry {
  static constexpr int kKind = 4;
  int64_t n;
  double inv_n2;
  const double* cx;
  struct Row { double xi; };
  struct Col { double j; double c2; };
  __device__ Row row(int64_t k) const { return Row{(double)(k - n / 2)}; }
  __device__ Col col(int64_t j) const { return Col{(double)j, 2.0 * cx[j]}; }
  __device__ cf entry(const Row& r, const Col& c) const {
    return cis_pi(fma(c.j * r.xi, inv_n2, c.c2 * fabs(r.xi)), -1.0, 1.0f);
  }
};

struct DenseEntry {
  static constexpr int kKind = 5;
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
    // points past the chunk's end repeat its last point (their X rows are zero)
    if (threadIdx.x < MF_TK) cols[threadIdx.x] = e.col(jb + min((int)threadIdx.x, tk - 1));
    __syncthreads();
    const int nsteps = (tk + 3) >> 2;
    for (int q = 0; q < nsteps; ++q) {
      const int jj = 4 * q + kq;
      double ar[MF_H], ai[MF_H], as[MF_H];
#pragma unroll
      for (int h = 0; h < MF_H; ++h) {
        const cf ev = e.entry(rw[h], cols[jj]);
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
// The same product on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16), which
// on gfx950 run concurrently with the vector ALUs that evaluate the entries
// (the FP32/FP64 matrix instructions do not).  Every entry a and input x is
// split into three BF16 terms, a = a1 + a2 + a3 (a1 = bf16(a),
// a2 = bf16(a - a1), a3 = bf16(a - a1 - a2)), and the products keep every
// term down to 2^-24 relative:  a x ~ a1x1 + a1x2 + a2x1 + a1x3 + a3x1 + a2x2
// -- six MFMAs per real product, 24 per complex tile step
// (Re += ar xr - ai xi, Im += ar xi + ai xr).  A wave owns 16 rows x 16 NT
// columns; per step of 32 inner points lane l evaluates its 8 A-operand
// entries (row l % 16, inner points 8 (l / 16) .. +7) and reads its B operands
// (the same 8 inner points of column l % 16 of each 16-column tile) from the
// split planes staged in LDS.  Each step's FP32 tile sums (32 terms) are
// added into FP64 registers, so the only FP32 summation error is that of
// 32-term sums.  Sixteen-column tiles keep the padding of odd sample widths
// (the adaptive passes use r + p columns) to less than 16 columns.
//
// X is split once per call (split_planes_kernel) into six BF16 planes laid
// out per column along the inner index, each segment padded with zeros to a
// multiple of the 64-point chunk, so a workgroup stages a chunk with 16-byte
// copies and a ragged tail needs no masking: its X terms are zero and its
// entries are evaluated at a clamped (valid) inner point.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// bf16(x0) in the low half, bf16(x1) in the high half (round to nearest even)
__device__ __forceinline__ uint32_t pk_bf16(float x0, float x1) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){x0, x1}, bf16x2));
}

// three-term split of two values at once: h + m + l = x to 2^-24 relative
// (x - bf16(x) and the next difference are exact in FP32)
__device__ __forceinline__ void split3_pk(float x0, float x1, uint32_t& h, uint32_t& m,
                                          uint32_t& l) {
  h = pk_bf16(x0, x1);
  const float r0 = x0 - __uint_as_float(h << 16);
  const float r1 = x1 - __uint_as_float(h & 0xffff0000u);
  m = pk_bf16(r0, r1);
  l = pk_bf16(r0 - __uint_as_float(m << 16), r1 - __uint_as_float(m & 0xffff0000u));
}

// Inner points per staged chunk: 128 (four MFMA steps between barriers) when
// X is exact in BF16 and only its first term is staged, 64 for the three
// terms of a general X (keeps two eight-wave workgroups per CU).  Segments
// of the split planes are padded to the larger one.
constexpr int BF_TK = 128;
template <bool EXACT> constexpr int bf_tk() { return EXACT ? 128 : 64; }
constexpr int BF_WAVES = 8;
constexpr int BF_ROWS = 16 * BF_WAVES;
// The 80-column tile runs four waves per workgroup (64 rows) so that three of
// its ~160-register workgroups fit on a CU (the split-K slicing still follows
// BF_ROWS, so results do not depend on the tile width).
template <int NT> constexpr int bf_waves() { return NT > 4 ? 4 : BF_WAVES; }
constexpr int BF_PLANES = 6;         // (term 0..2) x (re, im)

// Xp[(c * 6 + 2 term + part) * kpad + pofs[g] + (j - seg[g])] = term of
// X[j, c] (part 0 real, 1 imaginary); zero from seg[g+1] to pofs[g+1].
// One thread splits 8 consecutive inner points of one column.  *inexact
// (zero on entry) becomes nonzero if any value needs more than its first
// term, i.e. if X is not exactly representable in BF16.
__global__ void split_planes_kernel(const bf_c64* __restrict__ X, int64_t ldx,
                                    const int64_t* __restrict__ seg,
                                    const int64_t* __restrict__ pofs, int64_t kpad,
                                    uint16_t* __restrict__ Xp,
                                    unsigned long long* __restrict__ inexact) {
  const int g = blockIdx.y, c = blockIdx.z;
  const int64_t kk = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 8;
  const bool live = kk < pofs[g + 1] - pofs[g];
  uint32_t rest = 0;
  if (live) {
    const int64_t j0 = seg[g] + kk, j1 = seg[g + 1];
    const bf_c64* xc = X + (int64_t)c * ldx;
    u32x4 t[BF_PLANES];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      bf_c64 x0 = {0.f, 0.f}, x1 = {0.f, 0.f};
      if (j0 + 2 * d < j1) x0 = xc[j0 + 2 * d];
      if (j0 + 2 * d + 1 < j1) x1 = xc[j0 + 2 * d + 1];
      uint32_t h, m, l;
      split3_pk(x0.re, x1.re, h, m, l);
      t[0][d] = h; t[2][d] = m; t[4][d] = l;
      split3_pk(x0.im, x1.im, h, m, l);
      t[1][d] = h; t[3][d] = m; t[5][d] = l;
    }
    uint16_t* dst = Xp + (int64_t)c * BF_PLANES * kpad + pofs[g] + kk;
#pragma unroll
    for (int p = 0; p < BF_PLANES; ++p) *reinterpret_cast<u32x4*>(dst + p * kpad) = t[p];
#pragma unroll
    for (int p = 2; p < BF_PLANES; ++p) rest |= t[p][0] | t[p][1] | t[p][2] | t[p][3];
  }
  // one vector atomic per wave that saw a nonzero lower term
  const unsigned long long any = __ballot(rest != 0u);
  if (any != 0ull && (threadIdx.x & 63) == __ffsll((long long)any) - 1) atomicOr(inexact, 1ull);
}

// Two instantiations per shape: EXACT (X exact in BF16, e.g. the random
// blocks of Alg. 2, so x = x1 and a real product needs the three MFMAs
// a1x1 + a2x1 + a3x1) and general (six).  Both are launched; the one that
// does not match the flag written by split_planes_kernel exits at once.  When
// the construction driver marks the input as one of its random blocks
// (input_known_exact), only the EXACT variant is launched.
// Four waves per SIMD (at most 128 VGPRs) up to 64 columns: for the 48- and
// 64-column tiles of the general path this costs a few spilled registers
// outside the inner loop and is still ~25% faster than the two waves their
// unconstrained register count allows.  The 80-column tile (NT = 5) keeps its
// ~160 registers in four-wave workgroups (three waves per SIMD; two on the
// general path, whose three staged terms need ~250): its entries serve 25%
// more columns, so one call replaces the two a 68-column block would
// otherwise need.
template <class E, int NT, typename Tout, bool EXACT>
__global__ __launch_bounds__(64 * bf_waves<NT>())
__attribute__((amdgpu_waves_per_eu(NT > 4 ? (EXACT ? 3 : 2) : 4, 8)))
void matfree_bf16_kernel(
    E e, int64_t nout, const uint16_t* __restrict__ Xp, int64_t kpad, int32_t ncols, int32_t c0,
    int32_t width, Tout* __restrict__ Y, int64_t ldy, int64_t ycols,
    const int64_t* __restrict__ seg, const int64_t* __restrict__ pofs, int32_t nsplit,
    const unsigned long long* __restrict__ inexact) {
  if ((*inexact == 0ull) != EXACT) return;
  constexpr int NC = 16 * NT;
  constexpr int NTERM = EXACT ? 1 : 3;      // staged terms of X
  constexpr int TK = bf_tk<EXACT>();
  constexpr int KP = TK + 8;                // padded k stride (bank spread)
  __shared__ typename E::Col cols[TK];
  // split planes: [term][re/im][column][k], 16 bytes = 8 consecutive k
  __shared__ __attribute__((aligned(16))) uint16_t xs[NTERM][2][NC][KP];
  const int g = blockIdx.y;
  const int z = blockIdx.z;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  constexpr int NW = bf_waves<NT>();
  const int64_t row0 = (int64_t)blockIdx.x * (16 * NW) + wave * 16;
  const int64_t myrow = row0 + (lane & 15);
  const int kq = lane >> 4;       // which 8 of the step's 32 inner points
  const int lc = lane & 15;
  const int64_t j0 = seg[g], j1 = seg[g + 1];
  const int64_t len = j1 - j0;
  // split-K slices are whole chunks, so only a segment's last chunk is ragged
  const int64_t chunk = ((len + nsplit - 1) / nsplit + TK - 1) / TK * TK;
  const int64_t a = j0 + (int64_t)z * chunk;
  const int64_t b = (a + chunk < j1) ? a + chunk : j1;
  const int nc = width < NC ? width : NC;
  const uint16_t* xg = Xp + (int64_t)c0 * BF_PLANES * kpad + pofs[g] - j0;

  double fr[NT][4], fi[NT][4];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) { fr[t][v] = 0.0; fi[t][v] = 0.0; }
  const typename E::Row rw = e.row(myrow < nout ? myrow : nout - 1);

  for (int64_t jb = a; jb < b; jb += TK) {
    __syncthreads();
    // NC columns x (2 NTERM) planes x TK/8 copies of 16 bytes
    constexpr int NQ = TK / 8;
    for (int idx = threadIdx.x; idx < NC * 2 * NTERM * NQ; idx += 64 * NW) {
      const int q8 = idx % NQ, pl = (idx / NQ) % (2 * NTERM), c = (idx / NQ) / (2 * NTERM);
      u32x4 v = {0u, 0u, 0u, 0u};
      if (c < nc)
        v = *reinterpret_cast<const u32x4*>(xg + ((int64_t)c * BF_PLANES + pl) * kpad + jb + 8 * q8);
      *reinterpret_cast<u32x4*>(&xs[pl >> 1][pl & 1][c][8 * q8]) = v;
    }
    if (threadIdx.x < TK) {
      const int64_t j = jb + threadIdx.x;
      cols[threadIdx.x] = e.col(j < j1 ? j : j1 - 1);
    }
    __syncthreads();
    const int nsteps = (int)((b - jb < TK ? b - jb : TK) + 31) >> 5;
    for (int q = 0; q < nsteps; ++q) {
      const int kb = 32 * q + 8 * kq;
      cf ev[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) ev[u] = e.entry(rw, cols[kb + u]);
      u32x4 ar[3], ai[3], an[3];
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        uint32_t h, m, l;
        split3_pk(ev[2 * d].re, ev[2 * d + 1].re, h, m, l);
        ar[0][d] = h; ar[1][d] = m; ar[2][d] = l;
        split3_pk(ev[2 * d].im, ev[2 * d + 1].im, h, m, l);
        ai[0][d] = h; ai[1][d] = m; ai[2][d] = l;
      }
#pragma unroll
      for (int p = 0; p < 3; ++p) an[p] = ai[p] ^ 0x80008000u;   // -ai, both halves
      __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        u32x4 xr[NTERM], xi[NTERM];
#pragma unroll
        for (int p = 0; p < NTERM; ++p) {
          xr[p] = *reinterpret_cast<const u32x4*>(&xs[p][0][t * 16 + lc][kb]);
          xi[p] = *reinterpret_cast<const u32x4*>(&xs[p][1][t * 16 + lc][kb]);
        }
        floatx4 R = {}, I = {};
#define BF_MM(A, B, C) \
  C = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, A), \
                                              __builtin_bit_cast(bf16x8, B), C, 0, 0, 0);
#define BF_PAIR(P, Q) BF_MM(ar[P], xr[Q], R) BF_MM(an[P], xi[Q], R) \
                      BF_MM(ar[P], xi[Q], I) BF_MM(ai[P], xr[Q], I)
        if constexpr (EXACT) {
          // x = x1: a1x1 + a2x1 + a3x1, smallest first
          BF_PAIR(2, 0) BF_PAIR(1, 0) BF_PAIR(0, 0)
        } else {
          // term pairs (p, q) with p + q <= 2 (0-based): 20 02 11 10 01 00
          BF_PAIR(2, 0) BF_PAIR(0, 2) BF_PAIR(1, 1) BF_PAIR(1, 0) BF_PAIR(0, 1) BF_PAIR(0, 0)
        }
#undef BF_PAIR
#undef BF_MM
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          fr[t][v] += (double)R[v];
          fi[t][v] += (double)I[v];
        }
      }
      __builtin_amdgcn_s_setprio(0);
    }
  }
  // accumulator layout of a 16x16 MFMA tile on gfx950: lane l, register v
  // holds row 4 (l / 16) + v, column l % 16
  Tout* yz = Y + (int64_t)z * ycols * ldy + ((int64_t)g * ncols + c0) * ldy;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int c = t * 16 + lc;
    if (c < nc) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = row0 + 4 * kq + v;
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

template <class E, int NT, typename Tout>
static void launch_bf16(const E& e, int64_t nout, const uint16_t* Xp, int64_t kpad, int32_t ncols,
                        int32_t c0, int32_t width, Tout* Y, int64_t ldy, int64_t ycols,
                        const int64_t* seg_dev, const int64_t* pofs_dev, int32_t nseg,
                        int32_t nsplit, const unsigned long long* inexact, bool known_exact,
                        hipStream_t s) {
  constexpr int NW = bf_waves<NT>();
  dim3 grid((unsigned)((nout + 16 * NW - 1) / (16 * NW)), (unsigned)nseg, (unsigned)nsplit);
  const double nc = (double)std::min<int32_t>(16 * NT, width);
  const double nin = (double)g_matfree_nin;
  ProfScope ps(BF_KC_MATFREE, s, 8.0 * (double)nout * nin * nc,
               8.0 * nc * (nin + (double)nout * nseg));
  hipLaunchKernelGGL((matfree_bf16_kernel<E, NT, Tout, true>), grid, dim3(64 * NW), 0, s, e,
                     nout, Xp, kpad, ncols, c0, width, Y, ldy, ycols, seg_dev, pofs_dev, nsplit,
                     inexact);
  if (!known_exact)
    hipLaunchKernelGGL((matfree_bf16_kernel<E, NT, Tout, false>), grid, dim3(64 * NW), 0, s, e,
                       nout, Xp, kpad, ncols, c0, width, Y, ldy, ycols, seg_dev, pofs_dev, nsplit,
                       inexact);
  BF_HIP(hipGetLastError());
}

template <class E, typename Tout>
static void launch_chunk_bf16(const E& e, int64_t nout, const uint16_t* Xp, int64_t kpad,
                              int32_t ncols, int32_t c0, int32_t width, Tout* Y, int64_t ldy,
                              int64_t ycols, const int64_t* seg_dev, const int64_t* pofs_dev,
                              int32_t nseg, int32_t nsplit, const unsigned long long* inexact,
                              bool known_exact, hipStream_t s) {
  if (width <= 16)
    launch_bf16<E, 1>(e, nout, Xp, kpad, ncols, c0, width, Y, ldy, ycols, seg_dev, pofs_dev, nseg,
                      nsplit, inexact, known_exact, s);
  else if (width <= 32)
    launch_bf16<E, 2>(e, nout, Xp, kpad, ncols, c0, width, Y, ldy, ycols, seg_dev, pofs_dev, nseg,
                      nsplit, inexact, known_exact, s);
  else if (width <= 48)
    launch_bf16<E, 3>(e, nout, Xp, kpad, ncols, c0, width, Y, ldy, ycols, seg_dev, pofs_dev, nseg,
                      nsplit, inexact, known_exact, s);
  else if (width <= 64)
    launch_bf16<E, 4>(e, nout, Xp, kpad, ncols, c0, width, Y, ldy, ycols, seg_dev, pofs_dev, nseg,
                      nsplit, inexact, known_exact, s);
  else
    launch_bf16<E, 5>(e, nout, Xp, kpad, ncols, c0, width, Y, ldy, ycols, seg_dev, pofs_dev, nseg,
                      nsplit, inexact, known_exact, s);
}

// Column tiles of a product: with more than 48 split-BF16 columns the 48-,
// 64- and 80-column tiles are all usable and the autotuner picks per shape
// class (operator kind, column count, and the powers of two at or above the
// output rows, input points and segment count).  Every chunking gives bitwise
// the same products: a column's sums do not depend on the other columns of
// its tile, and split-K follows the row tiles only.

template <class E>
static void run_matfree(int prec, const E& e, int64_t nout, int64_t nin, const bf_c64* X,
                        int64_t ldx, int64_t ncols, bf_c64* Y, int64_t ldy,
                        const int64_t* seg_host, int32_t nseg, hipStream_t s) {
  if (nout <= 0 || ncols <= 0) return;
  const bool bf16 = prec == BF_PREC_BF16X3;
  const bool known_exact = bf16 && input_known_exact(X);
  std::vector<int64_t> segv;
  if (seg_host) {
    segv.assign(seg_host, seg_host + nseg + 1);
  } else {
    nseg = 1;
    segv = {0, nin};
  }
  BF_CHECK(nseg >= 1 && nseg <= 65535, BF_EINVAL, "bad segment count");
  BF_CHECK(ncols <= 65535, BF_EINVAL, "too many columns");
  int64_t maxlen = 0;
  for (int g = 0; g < nseg; ++g) {
    BF_CHECK(segv[g] <= segv[g + 1] && segv[g] >= 0 && segv[g + 1] <= nin, BF_EINVAL,
             "segments must partition the input rows");
    maxlen = std::max(maxlen, segv[g + 1] - segv[g]);
  }
  // split-K so that row tiles x groups x splits reaches ~2048 workgroups,
  // keeping at least 512 inner points per split.
  const int64_t rows_per_wg = bf16 ? BF_ROWS : MF_ROWS;
  int64_t tiles = ((nout + rows_per_wg - 1) / rows_per_wg) * nseg;
  int64_t want = (2048 + tiles - 1) / tiles;
  int64_t cap = std::max<int64_t>(1, maxlen / 512);
  int32_t nsplit = (int32_t)std::max<int64_t>(1, std::min<int64_t>({want, cap, 64}));

  // segment offsets (and, for the split planes, their chunk-padded offsets)
  // travel in one upload
  std::vector<int64_t> offs(segv);
  int64_t kpad = 0, maxpad = 0;
  if (bf16) {
    offs.resize(2 * (size_t)(nseg + 1));
    offs[nseg + 1] = 0;
    for (int g = 0; g < nseg; ++g) {
      const int64_t padded = (segv[g + 1] - segv[g] + BF_TK - 1) / BF_TK * BF_TK;
      offs[nseg + 2 + g] = offs[nseg + 1 + g] + padded;
      maxpad = std::max(maxpad, padded);
    }
    kpad = offs[2 * (size_t)nseg + 1];
    offs.push_back(0);   // the inexact flag of split_planes_kernel
  }
  DevBuf<int64_t> seg_dev(offs.size(), s);
  if (Staging* st = scope_staging(s)) {
    // pinned source: the copy does not wait for the stream to drain
    void* h = st->alloc(offs.size() * sizeof(int64_t), s);
    std::memcpy(h, offs.data(), offs.size() * sizeof(int64_t));
    BF_HIP(hipMemcpyAsync(seg_dev.p, h, offs.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
  } else {
    BF_HIP(hipMemcpyAsync(seg_dev.p, offs.data(), offs.size() * sizeof(int64_t),
                          hipMemcpyHostToDevice, s));
  }
  const int64_t* pofs_dev = seg_dev.p + nseg + 1;
  auto* inexact = bf16 ? reinterpret_cast<unsigned long long*>(seg_dev.p + offs.size() - 1) : nullptr;
  const int64_t ycols = (int64_t)nseg * ncols;
  g_matfree_nin = segv[nseg] - segv[0];

  DevBuf<uint16_t> planes;
  if (bf16) planes = DevBuf<uint16_t>(std::max<size_t>((size_t)ncols * BF_PLANES * kpad, 8), s);
  if (bf16 && kpad > 0) {
    ProfScope ps(BF_KC_OTHER, s, 0.0, 8.0 * ncols * (double)g_matfree_nin + 12.0 * ncols * kpad);
    dim3 grid((unsigned)((maxpad / 8 + 255) / 256), (unsigned)nseg, (unsigned)ncols);
    hipLaunchKernelGGL(split_planes_kernel, grid, dim3(256), 0, s, X, ldx, seg_dev.p, pofs_dev,
                       kpad, planes.p, inexact);
    BF_HIP(hipGetLastError());
  }

  DevBuf<bf_c128> part;
  if (nsplit > 1) part = DevBuf<bf_c128>((size_t)nsplit * ycols * nout, s);
  // one product, in column chunks of at most maxw columns (balanced widths)
  auto run_chunks = [&](int64_t maxw) {
    const int64_t nchunk = (ncols + maxw - 1) / maxw;
    const int64_t cw = (ncols + nchunk - 1) / nchunk;
    for (int64_t c0 = 0; c0 < ncols; c0 += cw) {
      const int32_t w = (int32_t)std::min<int64_t>(cw, ncols - c0);
      if (bf16) {
        if (nsplit > 1)
          launch_chunk_bf16(e, nout, planes.p, kpad, (int32_t)ncols, (int32_t)c0, w, part.p, nout,
                            ycols, seg_dev.p, pofs_dev, nseg, nsplit, inexact, known_exact, s);
        else
          launch_chunk_bf16(e, nout, planes.p, kpad, (int32_t)ncols, (int32_t)c0, w, Y, ldy,
                            ycols, seg_dev.p, pofs_dev, nseg, nsplit, inexact, known_exact, s);
      } else {
        if (nsplit > 1)
          launch_chunk(e, nout, X, ldx, (int32_t)ncols, (int32_t)c0, w, part.p, nout, ycols,
                       seg_dev.p, nseg, nsplit, s);
        else
          launch_chunk(e, nout, X, ldx, (int32_t)ncols, (int32_t)c0, w, Y, ldy, ycols,
                       seg_dev.p, nseg, nsplit, s);
      }
    }
  };
  if (bf16 && ncols > 48) {
    const TuneKey key{kTuneMatfreeWidth, E::kKind, ncols, pow2_ceil(nout),
                      pow2_ceil(g_matfree_nin), pow2_ceil(nseg)};
    tune_choose(key, {48, 64, 80}, 80, s, [&](int64_t w) { run_chunks(w); });
  } else {
    run_chunks(bf16 ? 80 : 48);
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
  if (out_pts.z && in_pts.z) {
    Seg3Entry e{out_pts, in_pts, 2.0 * (double)sign * k_over_2pi, (double)sign * k_over_2pi};
    run_matfree(prec, e, nout, nin, X, ldx, ncols, Y, ldy, seg_host, nseg, s);
  } else {
    SegEntry e{out_pts, in_pts, 2.0 * (double)sign * k_over_2pi, (double)sign * k_over_2pi};
    run_matfree(prec, e, nout, nin, X, ldx, ncols, Y, ldy, seg_host, nseg, s);
  }
}

void launch_fio(int prec, int64_t n, const double* cx_dev, int adjoint, const bf_c64* X,
                int64_t ldx, int64_t ncols, bf_c64* Y, int64_t ldy, const int64_t* seg_host,
                int32_t nseg, hipStream_t s) {
  if (!adjoint) {
    FioEntry e{n, 2.0 / (double)n, cx_dev};
    run_matfree(prec, e, n, n, X, ldx, ncols, Y, ldy, seg_host, nseg, s);
  } else {
    FioAdjEntry e{n, 2.0 / (double)n, cx_dev};
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
