// One stage of the hybrid butterfly apply (eq. hybrid_butterfly_mat): every
// output block is  out = sum_t G_t in_t  with at most two terms, where G_t is
// the factor block already put in the orientation this stage needs (W^H, R,
// B, U, V^H ... for the forward apply; their adjoints for A^H) and stored
// column-major (ld = M) contiguously in the order the stage reads it.
//
// Buffers are addressed by id (0: caller input, 1/2: ping-pong intermediates,
// 3: caller output) so descriptors built once per factorization serve any
// column count and any caller leading dimension.
#include "bf_internal.h"
#include "cplx.h"

namespace bf {

// Work mappings, by right-hand-side count and arithmetic:
//  * ncols <= 4 (streaming): a group of 16 lanes per output row splits the
//    inner dimension, so each row of the packed block is read as contiguous
//    bytes; partial sums are combined with shuffles inside the group.
//  * ncols > 4, split-BF16 (default): BF16 matrix-core tiles per (output
//    block, 64-column chunk), operands split into three BF16 terms; one wave
//    per block when every block of the stage has at most 16 rows, else one
//    workgroup per block with the operands staged in LDS.
//  * ncols > 4, FP32: one workgroup per (output block, 64-column chunk); the
//    packed block and the input chunk are staged in LDS and each thread
//    accumulates 4 rows of one column.
// Element (row r, column c) of buffer i is p[i][r * rs[i] + c * ld[i]]: the
// caller's buffers are column-major (rs = 1, ld = leading dimension); with
// more than AP_SMALL columns the intermediates are row-major (rs = ncols,
// ld = 1), so a block's rows for a 64-column chunk are contiguous 512-byte
// runs instead of 64 scattered columns.
struct ApplyBufs {
  bf_c64* p[4];
  int64_t ld[4];
  int64_t rs[4];
};

constexpr int AP_SMALL = kApplyFewCols;

// ncols <= 4: a group of AP_LPR = 8 lanes per output row (32 rows per
// workgroup); the row's record holds every address it needs (one dependent
// load), the inner loop is unrolled so the factor and input loads of a row
// issue together.  With one or two columns each lane loads two consecutive
// entries per 16-byte load.  At n = 262144, one column: 1.31 ms with 16 lanes
// and 8-byte loads, 1.06 ms with pairs, 0.84 ms with pairs on 8 lanes (FP64
// sums); four columns 1.88 -> 1.52 ms on 8 lanes.  Sums are FP32 (Acc = cf):
// FP64 sums of the FP32 products, once the default for one column, held a
// stage at 3.6-3.9 TB/s where FP32 sums reach 5.3 (the block kernel below).
template <typename Acc>
__device__ __forceinline__ void acc_fma(Acc& a, bf_c64 g, bf_c64 x);
template <>
__device__ __forceinline__ void acc_fma<cf>(cf& a, bf_c64 g, bf_c64 x) {
  cf_fma(a, cf{g.re, g.im}, cf{x.re, x.im});
}

typedef float f32x4u __attribute__((ext_vector_type(4)));
// two consecutive complex64 values in one 16-byte load (8-byte alignment is
// enough for global loads on gfx950)
__device__ __forceinline__ void load_pair(const bf_c64* p, bf_c64& a, bf_c64& b) {
  f32x4u v;
  __builtin_memcpy(&v, p, sizeof(v));
  a = bf_c64{v.x, v.y};
  b = bf_c64{v.z, v.w};
}

constexpr int AP_LPR = 8;   // lanes per output row of the few-column kernel

template <typename Acc, int NC>
__global__ __launch_bounds__(256) void apply_stream_kernel(const ApplyRowRec* __restrict__ rows,
                                                           int32_t nrows,
                                                           const bf_c64* __restrict__ G,
                                                           ApplyBufs B, int32_t ncols) {
  const int q = threadIdx.x & (AP_LPR - 1);
  const int64_t R = (int64_t)blockIdx.x * (256 / AP_LPR) + (threadIdx.x / AP_LPR);
  const bool live = R < nrows;
  const ApplyRowRec rr = rows[live ? R : 0];
  const int KK = live ? rr.KK : 0;
  const bf_c64* g = G + rr.g;
  const bf_c64* in0 = B.p[rr.in_buf0] + rr.in0;
  const bf_c64* in1 = B.p[rr.in_buf1] + rr.in1;
  const int64_t ld0 = B.ld[rr.in_buf0], ld1 = B.ld[rr.in_buf1];
  Acc acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = Acc{0, 0};
  if constexpr (NC <= 2) {
    const int K0 = rr.K0;
    for (int kb = 0; kb < KK; kb += 4 * AP_LPR) {
      // lane q takes entries k, k + 1 (k = kb + 2q + 16u): one 16-byte load per
      // pair of factor entries and, inside one input segment, per pair of inputs
      bf_c64 gv[4], xv[4][NC];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int k = kb + 2 * q + 2 * AP_LPR * u;
        const bool k0v = k < KK, k1v = k + 1 < KK;
        if (k1v) {
          load_pair(g + k, gv[2 * u], gv[2 * u + 1]);
        } else {
          gv[2 * u] = k0v ? g[k] : bf_c64{0.f, 0.f};
          gv[2 * u + 1] = bf_c64{0.f, 0.f};
        }
        const bool seg0 = k < K0, seg1 = k + 1 < K0;
        const bf_c64* base = seg0 ? in0 : in1;
        const int64_t ldk = seg0 ? ld0 : ld1;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          if (c < ncols && k1v && seg0 == seg1) {
            load_pair(base + k + (int64_t)c * ldk, xv[2 * u][c], xv[2 * u + 1][c]);
          } else {
            xv[2 * u][c] = (c < ncols && k0v) ? base[k + (int64_t)c * ldk] : bf_c64{0.f, 0.f};
            xv[2 * u + 1][c] = (c < ncols && k1v)
                                   ? (seg1 ? in0 : in1)[k + 1 + (int64_t)c * (seg1 ? ld0 : ld1)]
                                   : bf_c64{0.f, 0.f};
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc_fma(acc[c], gv[u], xv[u][c]);
    }
  } else {
    // four columns: one entry per lane and load (pairs measured 8% slower)
    for (int kb = 0; kb < KK; kb += 4 * AP_LPR) {
      bf_c64 gv[4], xv[4][NC];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = kb + q + AP_LPR * u;
        const bool kv = k < KK;
        gv[u] = kv ? g[k] : bf_c64{0.f, 0.f};
        const bf_c64* inp = k < rr.K0 ? in0 + k : in1 + k;
        const int64_t ldk = k < rr.K0 ? ld0 : ld1;
#pragma unroll
        for (int c = 0; c < NC; ++c)
          xv[u][c] = (kv && c < ncols) ? inp[(int64_t)c * ldk] : bf_c64{0.f, 0.f};
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc_fma(acc[c], gv[u], xv[u][c]);
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    acc[c].re = row8_sum(acc[c].re);
    acc[c].im = row8_sum(acc[c].im);
  }
  if (live && q == 0) {
    bf_c64* out = B.p[rr.out_buf] + rr.out;
    const int64_t ldo = B.ld[rr.out_buf];
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (c < ncols) out[(int64_t)c * ldo] = bf_c64{(float)acc[c].re, (float)acc[c].im};
  }
}

// Slot j of lane q in a row of the few-column kernels: pairs 2q, 2q + 1 in
// steps of 16 for one or two columns, q in steps of 8 otherwise -- the order
// of apply_stream_kernel, which every few-column path keeps so that all of
// them sum a row's terms in the same order.
template <int NC>
__device__ __forceinline__ int fused_k(int q, int j) {
  if constexpr (NC <= 2)
    return 2 * q + (j & 1) + 16 * (j >> 1);
  else
    return q + 8 * j;
}

// ncols <= 4 on stages whose rows have at most 32 * IT terms: one wave per
// block, no row records.  The wave reads its block's descriptor once; each
// lane holds the inputs of its slots (the same slots in every row of the
// block) in registers and streams the factor rows RG groups of 8 rows at a
// time.  Slots and summation order are apply_stream_kernel's, so both give
// the same bits.  Dropping the 48-byte records and the per-row input loads
// took one 200 MB stage of the n = 262144 FIO butterfly from 4.2-4.5 to
// 5.3-5.4 TB/s of factor bytes in a stand-alone probe that kept the factors
// out of the last-level cache (a read-only sum of the same bytes: 6.0 TB/s).
template <int NC, int IT, int RG, bool XL, bool MW>
__global__ __launch_bounds__(256) void apply_blockrows_kernel(const ApplyBlk* __restrict__ blks,
                                                              int32_t nblk,
                                                              const bf_c64* __restrict__ G,
                                                              ApplyBufs B, int32_t ncols,
                                                              int32_t wpb) {
  constexpr int S = 4 * IT;   // slots per lane
  // XL: the block's inputs in LDS (32 IT rows x NC columns per wave), read
  // per slot, instead of S x NC registers per lane
  __shared__ __attribute__((aligned(16))) bf_c64 xsh[XL ? 4 : 1][XL ? 32 * IT * NC : 1];
  const int wave = threadIdx.x >> 6;
  // MW: wpb waves per block, wave `part` taking row groups part, part + wpb,
  // ... (a separate instantiation: the runtime stride costs the one-wave
  // kernel a fifth of its speed on the streaming stages)
  const int wid = (int)(blockIdx.x * 4 + wave);
  const int b = __builtin_amdgcn_readfirstlane(MW ? wid / wpb : wid);
  const int part = MW ? __builtin_amdgcn_readfirstlane(wid % wpb) : 0;
  const int rstep = MW ? wpb * AP_LPR * RG : AP_LPR * RG;
  if (b >= nblk) return;
  const int lane = threadIdx.x & 63, q = lane & (AP_LPR - 1), rs = lane / AP_LPR;
  const ApplyBlk bk = blks[b];
  const int KK = bk.K0 + bk.K1, K0 = bk.K0;
  const bf_c64* in0 = B.p[bk.in_buf0] + bk.in_row0;
  const bf_c64* in1 = B.p[bk.in_buf1] + bk.in_row1 - K0;
  const int64_t ld0 = B.ld[bk.in_buf0], ld1 = B.ld[bk.in_buf1];
  bf_c64 xv[XL ? 1 : S][NC];
  if constexpr (XL) {
    bf_c64* xw = xsh[wave];
    for (int e = lane; e < 32 * IT * NC; e += 64) {
      const int k = e / NC, c = e % NC;
      bf_c64 x = {0.f, 0.f};
      if (k < KK && c < ncols) x = k < K0 ? in0[k + (int64_t)c * ld0] : in1[k + (int64_t)c * ld1];
      xw[e] = x;
    }
    // the wave's own LDS writes, read back by its other lanes
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const int k = fused_k<NC>(q, j);
      if constexpr (NC <= 2) {
        if (j & 1) continue;   // pairs: slot j + 1 is entry k + 1
        const bool k0v = k < KK, k1v = k + 1 < KK;
        const bool seg0 = k < K0, seg1 = k + 1 < K0;
        const bf_c64* base = seg0 ? in0 : in1;
        const int64_t ldk = seg0 ? ld0 : ld1;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          if (c < ncols && k1v && seg0 == seg1) {
            load_pair(base + k + (int64_t)c * ldk, xv[j][c], xv[j + 1][c]);
          } else {
            xv[j][c] = (c < ncols && k0v) ? base[k + (int64_t)c * ldk] : bf_c64{0.f, 0.f};
            xv[j + 1][c] = (c < ncols && k1v)
                               ? (seg1 ? in0 : in1)[k + 1 + (int64_t)c * (seg1 ? ld0 : ld1)]
                               : bf_c64{0.f, 0.f};
          }
        }
      } else {
        const bool kv = k < KK;
        const bf_c64* inp = k < K0 ? in0 + k : in1 + k;
        const int64_t ldk = k < K0 ? ld0 : ld1;
#pragma unroll
        for (int c = 0; c < NC; ++c)
          xv[j][c] = (kv && c < ncols) ? inp[(int64_t)c * ldk] : bf_c64{0.f, 0.f};
      }
    }
  }
  bf_c64* out = B.p[bk.out_buf] + bk.out_row;
  const int64_t ldo = B.ld[bk.out_buf];
  for (int r0 = part * AP_LPR * RG; r0 < bk.M; r0 += rstep) {
    // an offset the compiler cannot see through (an empty asm statement), so
    // that the LDS reads stay inside the loop instead of being hoisted into
    // registers
    int xo = 0;
    if constexpr (XL) asm volatile("" : "+s"(xo));
    bf_c64 gv[RG][S];
#pragma unroll
    for (int i = 0; i < RG; ++i) {
      const int r = r0 + AP_LPR * i + rs;
      const bf_c64* g = G + bk.g_off + (int64_t)r * KK;
#pragma unroll
      for (int j = 0; j < S; ++j) {
        const int k = fused_k<NC>(q, j);
        if constexpr (NC <= 2) {
          if (j & 1) continue;
          const bool k0v = r < bk.M && k < KK, k1v = r < bk.M && k + 1 < KK;
          if (k1v) {
            load_pair(g + k, gv[i][j], gv[i][j + 1]);
          } else {
            gv[i][j] = k0v ? g[k] : bf_c64{0.f, 0.f};
            gv[i][j + 1] = bf_c64{0.f, 0.f};
          }
        } else {
          gv[i][j] = (r < bk.M && k < KK) ? g[k] : bf_c64{0.f, 0.f};
        }
      }
    }
#pragma unroll
    for (int i = 0; i < RG; ++i) {
      cf acc[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] = cf{0.f, 0.f};
#pragma unroll
      for (int j = 0; j < S; ++j) {
        if constexpr (XL) {
          const bf_c64* xr = xsh[wave] + xo + fused_k<NC>(q, j) * NC;
#pragma unroll
          for (int c = 0; c < NC; ++c) acc_fma(acc[c], gv[i][j], xr[c]);
        } else {
#pragma unroll
          for (int c = 0; c < NC; ++c) acc_fma(acc[c], gv[i][j], xv[j][c]);
        }
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        acc[c].re = row8_sum(acc[c].re);
        acc[c].im = row8_sum(acc[c].im);
      }
      const int r = r0 + AP_LPR * i + rs;
      if (q == 0 && r < bk.M) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
          if (c < ncols) out[r + (int64_t)c * ldo] = bf_c64{acc[c].re, acc[c].im};
      }
    }
  }
}

constexpr int AP_CW = 64;   // columns per workgroup in the blocked mapping

__global__ __launch_bounds__(256) void apply_blocked_kernel(const ApplyBlk* __restrict__ blks,
                                                            const bf_c64* __restrict__ G,
                                                            ApplyBufs B, int64_t ncols) {
  extern __shared__ cf lds_ap[];
  const ApplyBlk bk = blks[blockIdx.x];
  const int64_t c0 = (int64_t)blockIdx.y * AP_CW;
  const int cw = (int)((ncols - c0 < AP_CW) ? ncols - c0 : AP_CW);
  const int M = bk.M, KK = bk.K0 + bk.K1;
  cf* Gs = lds_ap;                 // M x KK, row-major
  cf* Xs = lds_ap + M * KK;        // KK x AP_CW
  const bf_c64* gsrc = G + bk.g_off;
  for (int idx = threadIdx.x; idx < M * KK; idx += 256) {
    const bf_c64 v = gsrc[idx];
    Gs[idx] = cf{v.re, v.im};
  }
  for (int idx = threadIdx.x; idx < KK * AP_CW; idx += 256) {
    const int k = idx % KK, c = idx / KK;
    bf_c64 v = {0.f, 0.f};
    if (c < cw) {
      if (k < bk.K0)
        v = B.p[bk.in_buf0][(c0 + c) * B.ld[bk.in_buf0] + (bk.in_row0 + k) * B.rs[bk.in_buf0]];
      else
        v = B.p[bk.in_buf1][(c0 + c) * B.ld[bk.in_buf1] +
                            (bk.in_row1 + (k - bk.K0)) * B.rs[bk.in_buf1]];
    }
    Xs[k * AP_CW + c] = cf{v.re, v.im};
  }
  __syncthreads();
  const int c = threadIdx.x % AP_CW;
  const int rg = threadIdx.x / AP_CW;    // 0..3
  const int64_t rso = B.rs[bk.out_buf];
  bf_c64* out = B.p[bk.out_buf] + (c0 + c) * B.ld[bk.out_buf] + bk.out_row * rso;
  for (int rb = rg; rb < M; rb += 16) {  // rows rb, rb+4, rb+8, rb+12
    cf acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = cf{0.f, 0.f};
    for (int k = 0; k < KK; ++k) {
      const cf x = Xs[k * AP_CW + c];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = rb + 4 * j;
        if (r < M) cf_fma(acc[j], Gs[r * KK + k], x);
      }
    }
    if (c < cw) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = rb + 4 * j;
        if (r < M) out[r * rso] = bf_c64{acc[j].re, acc[j].im};
      }
    }
  }
}

// ---- split-BF16 stage (more than AP_SMALL right-hand sides) --------------
//
// Same stage as apply_blocked_kernel on the BF16 matrix cores: every factor
// entry and input value is split into three BF16 terms, g = g1 + g2 + g3,
// x = x1 + x2 + x3 (g2 = bf16(g - g1), ...), and the six products with
// p + q <= 2 keep every term down to 2^-24 relative, so the result matches
// the FP32 stage.  One workgroup (4 waves) per (output block, 64 columns);
// the inner dimension (both terms' inputs, one after the other) goes through
// LDS in chunks of 32, split while staged, as planes [term][re/im][row or
// column][k].  Wave w owns the 16-column tile w and every 16-row tile of the
// block (row blocks of 64): per tile and chunk 24 v_mfma_f32_16x16x32_bf16
// (Re += gr xr - gi xi, Im += gr xi + gi xr), FP32 accumulation.
typedef __bf16 abf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int au32x4 __attribute__((ext_vector_type(4)));
typedef float afloatx4 __attribute__((ext_vector_type(4)));
typedef float af32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 abf16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t apk_bf16(float x0, float x1) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((af32x2){x0, x1}, abf16x2));
}
__device__ __forceinline__ void asplit3(float x0, float x1, uint32_t& h, uint32_t& m, uint32_t& l) {
  h = apk_bf16(x0, x1);
  const float r0 = x0 - __uint_as_float(h << 16);
  const float r1 = x1 - __uint_as_float(h & 0xffff0000u);
  m = apk_bf16(r0, r1);
  l = apk_bf16(r0 - __uint_as_float(m << 16), r1 - __uint_as_float(m & 0xffff0000u));
}

constexpr int AM_KT = 32;            // inner indices per staged chunk
constexpr int AM_KP = AM_KT + 8;     // padded k stride of a plane row
constexpr int AM_R = 64;             // rows per row block
constexpr int AM_MIN_COLS = AP_SMALL + 1;

__global__ __launch_bounds__(256) void apply_mfma_kernel(const ApplyBlk* __restrict__ blks,
                                                         const bf_c64* __restrict__ G,
                                                         ApplyBufs B, int64_t ncols) {
  __shared__ __attribute__((aligned(16))) uint16_t gs[6][AM_R][AM_KP];
  __shared__ __attribute__((aligned(16))) uint16_t xs[6][AP_CW][AM_KP];
  const ApplyBlk bk = blks[blockIdx.x];
  const int64_t c0 = (int64_t)blockIdx.y * AP_CW;
  const int cw = (int)((ncols - c0 < AP_CW) ? ncols - c0 : AP_CW);
  const int M = bk.M, K0 = bk.K0, KK = bk.K0 + bk.K1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lc = lane & 15, kq = lane >> 4;
  const bf_c64* gsrc = G + bk.g_off;
  const int64_t rs0 = B.rs[bk.in_buf0], rs1 = B.rs[bk.in_buf1];
  const bf_c64* in0 = B.p[bk.in_buf0] + bk.in_row0 * rs0;
  const bf_c64* in1 = B.p[bk.in_buf1] + bk.in_row1 * rs1;
  const int64_t ld0 = B.ld[bk.in_buf0], ld1 = B.ld[bk.in_buf1];
  for (int rb = 0; rb < M; rb += AM_R) {
    const int mr = (M - rb < AM_R) ? M - rb : AM_R;
    const int rt_n = (mr + 15) >> 4;
    afloatx4 R[4], I[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) { R[t] = afloatx4{0.f, 0.f, 0.f, 0.f}; I[t] = R[t]; }
    for (int k0 = 0; k0 < KK; k0 += AM_KT) {
      __syncthreads();
      // factor chunk: rows rb..rb+63, two consecutive k per thread step
      for (int idx = threadIdx.x; idx < AM_R * (AM_KT / 2); idx += 256) {
        const int r = idx / (AM_KT / 2), k = 2 * (idx % (AM_KT / 2));
        bf_c64 v0 = {0.f, 0.f}, v1 = {0.f, 0.f};
        if (r < mr) {
          const bf_c64* gr = gsrc + (int64_t)(rb + r) * KK + k0;
          if (k0 + k < KK) v0 = gr[k];
          if (k0 + k + 1 < KK) v1 = gr[k + 1];
        }
        uint32_t h, m, l;
        asplit3(v0.re, v1.re, h, m, l);
        *reinterpret_cast<uint32_t*>(&gs[0][r][k]) = h;
        *reinterpret_cast<uint32_t*>(&gs[2][r][k]) = m;
        *reinterpret_cast<uint32_t*>(&gs[4][r][k]) = l;
        asplit3(v0.im, v1.im, h, m, l);
        *reinterpret_cast<uint32_t*>(&gs[1][r][k]) = h;
        *reinterpret_cast<uint32_t*>(&gs[3][r][k]) = m;
        *reinterpret_cast<uint32_t*>(&gs[5][r][k]) = l;
      }
      // input chunk: inner rows k0..k0+31 (term 0 rows, then term 1 rows)
      for (int idx = threadIdx.x; idx < AP_CW * (AM_KT / 2); idx += 256) {
        const int c = idx / (AM_KT / 2), k = 2 * (idx % (AM_KT / 2));
        bf_c64 v[2] = {{0.f, 0.f}, {0.f, 0.f}};
        if (c < cw) {
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const int kk = k0 + k + u;
            if (kk < K0)
              v[u] = in0[(c0 + c) * ld0 + kk * rs0];
            else if (kk < KK)
              v[u] = in1[(c0 + c) * ld1 + (kk - K0) * rs1];
          }
        }
        uint32_t h, m, l;
        asplit3(v[0].re, v[1].re, h, m, l);
        *reinterpret_cast<uint32_t*>(&xs[0][c][k]) = h;
        *reinterpret_cast<uint32_t*>(&xs[2][c][k]) = m;
        *reinterpret_cast<uint32_t*>(&xs[4][c][k]) = l;
        asplit3(v[0].im, v[1].im, h, m, l);
        *reinterpret_cast<uint32_t*>(&xs[1][c][k]) = h;
        *reinterpret_cast<uint32_t*>(&xs[3][c][k]) = m;
        *reinterpret_cast<uint32_t*>(&xs[5][c][k]) = l;
      }
      __syncthreads();
      au32x4 xb[6];
#pragma unroll
      for (int p = 0; p < 6; ++p)
        xb[p] = *reinterpret_cast<const au32x4*>(&xs[p][wave * 16 + lc][8 * kq]);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t < rt_n) {
          au32x4 ga[6], gn[3];
#pragma unroll
          for (int p = 0; p < 6; ++p)
            ga[p] = *reinterpret_cast<const au32x4*>(&gs[p][t * 16 + lc][8 * kq]);
#pragma unroll
          for (int q = 0; q < 3; ++q) gn[q] = ga[2 * q + 1] ^ 0x80008000u;
#define AM_MM(A, Bv, C) \
  C = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(abf16x8, A), \
                                              __builtin_bit_cast(abf16x8, Bv), C, 0, 0, 0);
#define AM_PAIR(P, Q) AM_MM(ga[2 * P], xb[2 * Q], R[t]) AM_MM(gn[P], xb[2 * Q + 1], R[t]) \
                      AM_MM(ga[2 * P], xb[2 * Q + 1], I[t]) AM_MM(ga[2 * P + 1], xb[2 * Q], I[t])
          AM_PAIR(2, 0) AM_PAIR(0, 2) AM_PAIR(1, 1) AM_PAIR(1, 0) AM_PAIR(0, 1) AM_PAIR(0, 0)
#undef AM_PAIR
#undef AM_MM
        }
      }
    }
    // accumulator layout of a 16x16 tile: lane l, register v -> row
    // 4 (l / 16) + v, column l % 16
    const int c = wave * 16 + lc;
    if (c < cw) {
      const int64_t rso = B.rs[bk.out_buf];
      bf_c64* out = B.p[bk.out_buf] + (c0 + c) * B.ld[bk.out_buf] + (bk.out_row + rb) * rso;
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = t * 16 + 4 * kq + v;
          if (t < rt_n && r < mr) out[r * rso] = bf_c64{R[t][v], I[t][v]};
        }
    }
  }
}

// Small blocks (every block of the stage has M <= 16): one wave per block
// (its single 16-row tile) and 64 columns, four waves per workgroup.  The
// wave loads its A operands (8 consecutive k of one factor row per lane) and
// B operands (8 consecutive k of one input column per lane) straight into
// registers and splits them there: no LDS, no barriers, so the per-block cost
// is a few loads and 24 MFMAs per 16-column tile instead of a workgroup's
// staging passes.
__device__ __forceinline__ void am_split8(const bf_c64 (&v)[8], au32x4 (&pl)[6]) {
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    uint32_t h, m, l;
    asplit3(v[2 * d].re, v[2 * d + 1].re, h, m, l);
    pl[0][d] = h; pl[2][d] = m; pl[4][d] = l;
    asplit3(v[2 * d].im, v[2 * d + 1].im, h, m, l);
    pl[1][d] = h; pl[3][d] = m; pl[5][d] = l;
  }
}

__global__ __launch_bounds__(256) void apply_mfma_small_kernel(const ApplyBlk* __restrict__ blks,
                                                               int32_t nblk,
                                                               const bf_c64* __restrict__ G,
                                                               ApplyBufs B, int64_t ncols) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t bi = (int64_t)blockIdx.x * 4 + wave;
  if (bi >= nblk) return;
  const ApplyBlk bk = blks[bi];
  const int64_t c0 = (int64_t)blockIdx.y * AP_CW;
  const int cw = (int)((ncols - c0 < AP_CW) ? ncols - c0 : AP_CW);
  const int M = bk.M, K0 = bk.K0, KK = bk.K0 + bk.K1;
  const int lc = lane & 15, kq = lane >> 4;
  const bf_c64* grow = G + bk.g_off + (int64_t)lc * KK;   // factor row lc (row-major M x KK)
  const int64_t rs0 = B.rs[bk.in_buf0], rs1 = B.rs[bk.in_buf1];
  const bf_c64* in0 = B.p[bk.in_buf0] + bk.in_row0 * rs0;
  const bf_c64* in1 = B.p[bk.in_buf1] + (bk.in_row1 - K0) * rs1;   // indexed by k >= K0
  const int64_t ld0 = B.ld[bk.in_buf0], ld1 = B.ld[bk.in_buf1];
  const int nct = (cw + 15) >> 4;
  afloatx4 R[4], I[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) { R[t] = afloatx4{0.f, 0.f, 0.f, 0.f}; I[t] = R[t]; }
  for (int k0 = 0; k0 < KK; k0 += 32) {
    const int kb = k0 + 8 * kq;
    bf_c64 v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e)
      v[e] = (lc < M && kb + e < KK) ? grow[kb + e] : bf_c64{0.f, 0.f};
    au32x4 ga[6], gn[3];
    am_split8(v, ga);
#pragma unroll
    for (int q = 0; q < 3; ++q) gn[q] = ga[2 * q + 1] ^ 0x80008000u;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t < nct) {
        const int c = t * 16 + lc;
        const int64_t col = c0 + (c < cw ? c : 0);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int k = kb + e;
          bf_c64 x = {0.f, 0.f};
          if (c < cw && k < KK) x = k < K0 ? in0[col * ld0 + k * rs0] : in1[col * ld1 + k * rs1];
          v[e] = x;
        }
        au32x4 xb[6];
        am_split8(v, xb);
#define AM_MM(A, Bv, C) \
  C = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(abf16x8, A), \
                                              __builtin_bit_cast(abf16x8, Bv), C, 0, 0, 0);
#define AM_PAIR(P, Q) AM_MM(ga[2 * P], xb[2 * Q], R[t]) AM_MM(gn[P], xb[2 * Q + 1], R[t]) \
                      AM_MM(ga[2 * P], xb[2 * Q + 1], I[t]) AM_MM(ga[2 * P + 1], xb[2 * Q], I[t])
        AM_PAIR(2, 0) AM_PAIR(0, 2) AM_PAIR(1, 1) AM_PAIR(1, 0) AM_PAIR(0, 1) AM_PAIR(0, 0)
#undef AM_PAIR
#undef AM_MM
      }
    }
  }
  // 16x16 tile layout: lane l, register v -> row 4 (l / 16) + v, column l % 16
  const int64_t rso = B.rs[bk.out_buf];
  bf_c64* ob = B.p[bk.out_buf] + bk.out_row * rso;
  const int64_t ldo = B.ld[bk.out_buf];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int c = t * 16 + lc;
    if (t < nct && c < cw) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 4 * kq + v;
        if (r < M) ob[(c0 + c) * ldo + r * rso] = bf_c64{R[t][v], I[t][v]};
      }
    }
  }
}

// Blocks of up to 64 rows: one wave per block and ctw 16-column tiles, the
// tiles one after another (stages of few blocks take one tile per wave, so
// that the device fills; stages of many blocks all tiles per wave, so that a
// block's factor rows are read from memory once and from the cache for its
// further tiles).  Per tile and 32-term chunk the wave loads and splits its
// B operands once, then each 16-row tile's A operands straight from the
// factor rows, and runs the 24 MFMAs of that row tile: the operands, products
// and their order are apply_mfma_kernel's (same bits) without its LDS passes
// and barriers.
__global__ __launch_bounds__(256) void apply_mfma_wave_kernel(const ApplyBlk* __restrict__ blks,
                                                              int32_t nblk,
                                                              const bf_c64* __restrict__ G,
                                                              ApplyBufs B, int64_t ncols,
                                                              int32_t ctw) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t bi = (int64_t)blockIdx.x * 4 + wave;
  if (bi >= nblk) return;
  const ApplyBlk bk = blks[bi];
  const int M = bk.M, K0 = bk.K0, KK = bk.K0 + bk.K1;
  const int lc = lane & 15, kq = lane >> 4;
  const int rt_n = (M + 15) >> 4;   // at most 4
  const bf_c64* gb = G + bk.g_off;
  const int64_t rs0 = B.rs[bk.in_buf0], rs1 = B.rs[bk.in_buf1];
  const bf_c64* in0 = B.p[bk.in_buf0] + bk.in_row0 * rs0;
  const bf_c64* in1 = B.p[bk.in_buf1] + (bk.in_row1 - K0) * rs1;   // indexed by k >= K0
  const int64_t ld0 = B.ld[bk.in_buf0], ld1 = B.ld[bk.in_buf1];
  const int64_t rso = B.rs[bk.out_buf], ldo = B.ld[bk.out_buf];
  bf_c64* ob = B.p[bk.out_buf] + bk.out_row * rso;
  // column tiles [blockIdx.y * ctw, (blockIdx.y + 1) * ctw) of this block
  const int64_t cbeg = (int64_t)blockIdx.y * ctw * 16;
  const int64_t cend = cbeg + (int64_t)ctw * 16 < ncols ? cbeg + (int64_t)ctw * 16 : ncols;
  for (int64_t c0 = cbeg; c0 < cend; c0 += 16) {
    const int64_t col = c0 + lc;
    const bool cv = col < ncols;
    afloatx4 R[4], I[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) { R[t] = afloatx4{0.f, 0.f, 0.f, 0.f}; I[t] = R[t]; }
    for (int k0 = 0; k0 < KK; k0 += AM_KT) {
      const int kb = k0 + 8 * kq;
      bf_c64 v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = kb + e;
        bf_c64 x = {0.f, 0.f};
        if (cv && k < KK) x = k < K0 ? in0[col * ld0 + k * rs0] : in1[col * ld1 + k * rs1];
        v[e] = x;
      }
      au32x4 xb[6];
      am_split8(v, xb);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t < rt_n) {
          const int r = t * 16 + lc;
          const bf_c64* grow = gb + (int64_t)r * KK;
#pragma unroll
          for (int e = 0; e < 8; ++e)
            v[e] = (r < M && kb + e < KK) ? grow[kb + e] : bf_c64{0.f, 0.f};
          au32x4 ga[6], gn[3];
          am_split8(v, ga);
#pragma unroll
          for (int q = 0; q < 3; ++q) gn[q] = ga[2 * q + 1] ^ 0x80008000u;
#define AM_MM(A, Bv, C) \
  C = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(abf16x8, A), \
                                              __builtin_bit_cast(abf16x8, Bv), C, 0, 0, 0);
#define AM_PAIR(P, Q) AM_MM(ga[2 * P], xb[2 * Q], R[t]) AM_MM(gn[P], xb[2 * Q + 1], R[t]) \
                      AM_MM(ga[2 * P], xb[2 * Q + 1], I[t]) AM_MM(ga[2 * P + 1], xb[2 * Q], I[t])
          AM_PAIR(2, 0) AM_PAIR(0, 2) AM_PAIR(1, 1) AM_PAIR(1, 0) AM_PAIR(0, 1) AM_PAIR(0, 0)
#undef AM_PAIR
#undef AM_MM
        }
      }
    }
    // 16x16 tile layout: lane l, register v -> row 4 (l / 16) + v, column l % 16
    if (cv) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = t * 16 + 4 * kq + v;
          if (t < rt_n && r < M) ob[col * ldo + r * rso] = bf_c64{R[t][v], I[t][v]};
        }
    }
  }
}

// The same work for stages of few blocks (every wave of the stage resident at
// once, so the stage lasts one wave's chain of memory trips): each 32-term
// chunk issues its B-operand loads and the A-operand loads of all RT row
// tiles before any arithmetic, one trip per chunk instead of one per row
// tile.  The extra live registers cost a wave per SIMD, which stages of
// many blocks need more.  Same operands, products and order: same bits.
template <int RT>
__global__ __launch_bounds__(256) void apply_mfma_wave_lf_kernel(const ApplyBlk* __restrict__ blks,
                                                                 int32_t nblk,
                                                                 const bf_c64* __restrict__ G,
                                                                 ApplyBufs B, int64_t ncols,
                                                                 int32_t ctw) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t bi = (int64_t)blockIdx.x * 4 + wave;
  if (bi >= nblk) return;
  const ApplyBlk bk = blks[bi];
  const int M = bk.M, K0 = bk.K0, KK = bk.K0 + bk.K1;
  const int lc = lane & 15, kq = lane >> 4;
  const int rt_n = (M + 15) >> 4;   // at most RT
  const bf_c64* gb = G + bk.g_off;
  const int64_t rs0 = B.rs[bk.in_buf0], rs1 = B.rs[bk.in_buf1];
  const bf_c64* in0 = B.p[bk.in_buf0] + bk.in_row0 * rs0;
  const bf_c64* in1 = B.p[bk.in_buf1] + (bk.in_row1 - K0) * rs1;   // indexed by k >= K0
  const int64_t ld0 = B.ld[bk.in_buf0], ld1 = B.ld[bk.in_buf1];
  const int64_t rso = B.rs[bk.out_buf], ldo = B.ld[bk.out_buf];
  bf_c64* ob = B.p[bk.out_buf] + bk.out_row * rso;
  const int64_t cbeg = (int64_t)blockIdx.y * ctw * 16;
  const int64_t cend = cbeg + (int64_t)ctw * 16 < ncols ? cbeg + (int64_t)ctw * 16 : ncols;
  for (int64_t c0 = cbeg; c0 < cend; c0 += 16) {
    const int64_t col = c0 + lc;
    const bool cv = col < ncols;
    afloatx4 R[RT], I[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) { R[t] = afloatx4{0.f, 0.f, 0.f, 0.f}; I[t] = R[t]; }
    for (int k0 = 0; k0 < KK; k0 += AM_KT) {
      const int kb = k0 + 8 * kq;
      bf_c64 xv[8], gv[RT][8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = kb + e;
        bf_c64 x = {0.f, 0.f};
        if (cv && k < KK) x = k < K0 ? in0[col * ld0 + k * rs0] : in1[col * ld1 + k * rs1];
        xv[e] = x;
      }
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int r = t * 16 + lc;
        const bf_c64* grow = gb + (int64_t)r * KK;
#pragma unroll
        for (int e = 0; e < 8; ++e)
          gv[t][e] = (r < M && kb + e < KK) ? grow[kb + e] : bf_c64{0.f, 0.f};
      }
      au32x4 xb[6];
      am_split8(xv, xb);
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        if (t < rt_n) {
          au32x4 ga[6], gn[3];
          am_split8(gv[t], ga);
#pragma unroll
          for (int q = 0; q < 3; ++q) gn[q] = ga[2 * q + 1] ^ 0x80008000u;
#define AM_MM(A, Bv, C) \
  C = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(abf16x8, A), \
                                              __builtin_bit_cast(abf16x8, Bv), C, 0, 0, 0);
#define AM_PAIR(P, Q) AM_MM(ga[2 * P], xb[2 * Q], R[t]) AM_MM(gn[P], xb[2 * Q + 1], R[t]) \
                      AM_MM(ga[2 * P], xb[2 * Q + 1], I[t]) AM_MM(ga[2 * P + 1], xb[2 * Q], I[t])
          AM_PAIR(2, 0) AM_PAIR(0, 2) AM_PAIR(1, 1) AM_PAIR(1, 0) AM_PAIR(0, 1) AM_PAIR(0, 0)
#undef AM_PAIR
#undef AM_MM
        }
      }
    }
    if (cv) {
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = t * 16 + 4 * kq + v;
          if (t < rt_n && r < M) ob[col * ldo + r * rso] = bf_c64{R[t][v], I[t][v]};
        }
    }
  }
}

template <int RT>
static void launch_wave_lf(dim3 grid, hipStream_t s, const ApplyBlk* blks, int32_t nblk,
                           const bf_c64* G, const ApplyBufs& B, int64_t ncols, int32_t ctw) {
  hipLaunchKernelGGL((apply_mfma_wave_lf_kernel<RT>), grid, dim3(256), 0, s, blks, nblk, G, B,
                     ncols, ctw);
}

// A merging stage of a structured sample's windows (see apply_structured):
// every intermediate row holds only the columns of the segments below its
// node, so an output row's window is its two children's windows side by
// side -- the first `win` columns come from term 0 (inputs k < K0, the first
// child) and the rest from term 1 (the second child).  Each lane takes the
// term of its own column (the B operand is per column); chunks of 32 inner
// indices that only the other term touches are skipped.  The products are
// those of the block-diagonal expansion, whose other entries are zeros, in
// the same order: same bits.  One wave per block and 16-column tile.
template <int RT>
__global__ __launch_bounds__(256) void apply_mfma_window_kernel(const ApplyBlk* __restrict__ blks,
                                                                int32_t nblk,
                                                                const bf_c64* __restrict__ G,
                                                                ApplyBufs B, int64_t ncols,
                                                                int64_t win) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t bi = (int64_t)blockIdx.x * 4 + wave;
  if (bi >= nblk) return;
  const ApplyBlk bk = blks[bi];
  const int M = bk.M, K0 = bk.K0, KK = bk.K0 + bk.K1;
  const int lc = lane & 15, kq = lane >> 4;
  const int rt_n = (M + 15) >> 4;   // at most RT
  const bf_c64* gb = G + bk.g_off;
  const int64_t rs0 = B.rs[bk.in_buf0], rs1 = B.rs[bk.in_buf1];
  const bf_c64* in0 = B.p[bk.in_buf0] + bk.in_row0 * rs0;
  const bf_c64* in1 = B.p[bk.in_buf1] + (bk.in_row1 - K0) * rs1;   // indexed by k >= K0
  const int64_t ld0 = B.ld[bk.in_buf0], ld1 = B.ld[bk.in_buf1];
  const int64_t rso = B.rs[bk.out_buf], ldo = B.ld[bk.out_buf];
  bf_c64* ob = B.p[bk.out_buf] + bk.out_row * rso;
  const int64_t c0 = (int64_t)blockIdx.y * 16;
  const int64_t col = c0 + lc;
  const bool cv = col < ncols;
  const bool second = col >= win;   // this lane's column belongs to term 1
  const int kbeg = c0 >= win ? (K0 / AM_KT) * AM_KT : 0;
  const int kend = c0 + 15 < win ? K0 : KK;
  afloatx4 R[RT], I[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) { R[t] = afloatx4{0.f, 0.f, 0.f, 0.f}; I[t] = R[t]; }
  for (int k0 = kbeg; k0 < kend; k0 += AM_KT) {
    const int kb = k0 + 8 * kq;
    bf_c64 v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = kb + e;
      bf_c64 x = {0.f, 0.f};
      if (cv && k < KK) {
        if (k < K0) {
          if (!second) x = in0[col * ld0 + k * rs0];
        } else if (second) {
          x = in1[(col - win) * ld1 + k * rs1];
        }
      }
      v[e] = x;
    }
    au32x4 xb[6];
    am_split8(v, xb);
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      if (t < rt_n) {
        const int r = t * 16 + lc;
        const bf_c64* grow = gb + (int64_t)r * KK;
#pragma unroll
        for (int e = 0; e < 8; ++e)
          v[e] = (r < M && kb + e < KK) ? grow[kb + e] : bf_c64{0.f, 0.f};
        au32x4 ga[6], gn[3];
        am_split8(v, ga);
#pragma unroll
        for (int q = 0; q < 3; ++q) gn[q] = ga[2 * q + 1] ^ 0x80008000u;
#define AM_MM(A, Bv, C) \
  C = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(abf16x8, A), \
                                              __builtin_bit_cast(abf16x8, Bv), C, 0, 0, 0);
#define AM_PAIR(P, Q) AM_MM(ga[2 * P], xb[2 * Q], R[t]) AM_MM(gn[P], xb[2 * Q + 1], R[t]) \
                      AM_MM(ga[2 * P], xb[2 * Q + 1], I[t]) AM_MM(ga[2 * P + 1], xb[2 * Q], I[t])
        AM_PAIR(2, 0) AM_PAIR(0, 2) AM_PAIR(1, 1) AM_PAIR(1, 0) AM_PAIR(0, 1) AM_PAIR(0, 0)
#undef AM_PAIR
#undef AM_MM
      }
    }
  }
  if (cv) {
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = t * 16 + 4 * kq + v;
        if (t < rt_n && r < M) ob[col * ldo + r * rso] = bf_c64{R[t][v], I[t][v]};
      }
  }
}

void launch_apply_window_stage(const ApplyBlk* blks_dev, int32_t nblk, int32_t maxM,
                               const bf_c64* G, const bf_c64* const bufs[4],
                               const int64_t lds[4], const int64_t rss[4], int64_t ncols,
                               int64_t win, hipStream_t s) {
  if (nblk <= 0 || ncols <= 0) return;
  BF_CHECK(maxM <= 64 && win > 0 && win < ncols, BF_EINVAL, "window stage: bad shape");
  ApplyBufs B;
  for (int i = 0; i < 4; ++i) {
    B.p[i] = const_cast<bf_c64*>(bufs[i]);
    B.ld[i] = lds[i];
    B.rs[i] = rss[i];
  }
  const int64_t gy = (ncols + 15) / 16;
  BF_CHECK(gy <= 65535, BF_EINVAL, "window stage: too many columns");
  const dim3 grid((unsigned)((nblk + 3) / 4), (unsigned)gy);
  const int rt = (maxM + 15) / 16;
  if (rt <= 1)
    hipLaunchKernelGGL((apply_mfma_window_kernel<1>), grid, dim3(256), 0, s, blks_dev, nblk, G, B, ncols, win);
  else if (rt == 2)
    hipLaunchKernelGGL((apply_mfma_window_kernel<2>), grid, dim3(256), 0, s, blks_dev, nblk, G, B, ncols, win);
  else if (rt == 3)
    hipLaunchKernelGGL((apply_mfma_window_kernel<3>), grid, dim3(256), 0, s, blks_dev, nblk, G, B, ncols, win);
  else
    hipLaunchKernelGGL((apply_mfma_window_kernel<4>), grid, dim3(256), 0, s, blks_dev, nblk, G, B, ncols, win);
  BF_HIP(hipGetLastError());
}

// ---- fused stages (few right-hand sides) ---------------------------------
//
// One launch runs several consecutive stages.  The blocks of those stages
// split into groups that depend only on each other (each block's inputs are
// produced inside its group, or come from the launch's input buffer), and
// workgroup w runs group w stage after stage, with a barrier between stages:
// an apply of 13 stages becomes 4 launches instead of 13 dependent ones.
// Rows follow the few-column kernels above (8 lanes per output row, same
// slots and summation order, so 1 to 4 columns give their results bit for
// bit).  Inside a launch a group's intermediates stay in its workgroup's
// LDS (a stage writes one half, the next stage reads it after the barrier
// and writes the other); the last stage of a launch writes global memory,
// each launch its own rows of the tall intermediate, so workgroups never
// overwrite what another still reads.

// Inputs of a fused row: LI, from the workgroup's LDS matrix of
// 2 kFusedLdsRows rows per column (records with buffer kFusedLdsBuf), else
// from the caller's buffers.  A row's two input ranges are both in LDS or
// both in global memory, and so are all rows of a group's stage: callers
// pick the instantiation per row, a uniform branch, so that every access
// has a known address space (LDS or global, never flat).
template <bool LI>
__device__ __forceinline__ const bf_c64* fused_in(const ApplyBufs& B, const bf_c64* lds, int i,
                                                  int64_t off) {
  if constexpr (LI) return lds + off;
  else return B.p[i] + off;
}
template <bool LI>
__device__ __forceinline__ int64_t fused_in_ld(const ApplyBufs& B, int i) {
  if constexpr (LI) return 2 * kFusedLdsRows;
  else return B.ld[i];
}
// The row's sums (lane q = 0 of the row) to LDS or to the caller's buffer.
template <typename Acc, int NC>
__device__ __forceinline__ void fused_store(const ApplyRowRec& rr, const ApplyBufs& B, bf_c64* lds,
                                            const Acc (&acc)[NC], int ncols) {
  if (rr.out_buf == kFusedLdsBuf) {
    // relaxed workgroup-scope atomic stores (plain LDS writes): unlike ordinary
    // stores they are never merged with the global branch's into one flat
    // store through a selected pointer
    uint64_t* out = reinterpret_cast<uint64_t*>(lds + rr.out);
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (c < ncols) {
        const bf_c64 v{(float)acc[c].re, (float)acc[c].im};
        uint64_t bits;
        __builtin_memcpy(&bits, &v, sizeof(bits));
        __hip_atomic_store(out + (int64_t)c * 2 * kFusedLdsRows, bits, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
      }
  } else {
    bf_c64* out = B.p[rr.out_buf] + rr.out;
    const int64_t ldo = B.ld[rr.out_buf];
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (c < ncols) out[(int64_t)c * ldo] = bf_c64{(float)acc[c].re, (float)acc[c].im};
  }
}

template <typename Acc, int NC, bool LI>
__device__ __forceinline__ void fused_row(const ApplyRowRec& rr, int q, const bf_c64* __restrict__ G,
                                          const ApplyBufs& B, bf_c64* lds, int ncols) {
  const int KK = rr.KK;
  const bf_c64* g = G + rr.g;
  const bf_c64* in0 = fused_in<LI>(B, lds, rr.in_buf0, rr.in0);
  const bf_c64* in1 = fused_in<LI>(B, lds, rr.in_buf1, rr.in1);
  const int64_t ld0 = fused_in_ld<LI>(B, rr.in_buf0), ld1 = fused_in_ld<LI>(B, rr.in_buf1);
  // 16-byte input loads from global memory only (LDS rows are 8-byte aligned)
  constexpr bool pair_in = !LI;
  Acc acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = Acc{0, 0};
  if constexpr (NC <= 2) {
    const int K0 = rr.K0;
    for (int kb = 0; kb < KK; kb += 4 * AP_LPR) {
      bf_c64 gv[4], xv[4][NC];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int k = kb + 2 * q + 2 * AP_LPR * u;
        const bool k0v = k < KK, k1v = k + 1 < KK;
        if (k1v) {
          load_pair(g + k, gv[2 * u], gv[2 * u + 1]);
        } else {
          gv[2 * u] = k0v ? g[k] : bf_c64{0.f, 0.f};
          gv[2 * u + 1] = bf_c64{0.f, 0.f};
        }
        const bool seg0 = k < K0, seg1 = k + 1 < K0;
        const bf_c64* base = seg0 ? in0 : in1;
        const int64_t ldk = seg0 ? ld0 : ld1;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          if (c < ncols && k1v && seg0 == seg1 && pair_in) {
            load_pair(base + k + (int64_t)c * ldk, xv[2 * u][c], xv[2 * u + 1][c]);
          } else {
            xv[2 * u][c] = (c < ncols && k0v) ? base[k + (int64_t)c * ldk] : bf_c64{0.f, 0.f};
            xv[2 * u + 1][c] = (c < ncols && k1v)
                                   ? (seg1 ? in0 : in1)[k + 1 + (int64_t)c * (seg1 ? ld0 : ld1)]
                                   : bf_c64{0.f, 0.f};
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc_fma(acc[c], gv[u], xv[u][c]);
    }
  } else {
    // one entry per lane and load, 4 per lane and step
    constexpr int U = 4;
    for (int kb = 0; kb < KK; kb += U * AP_LPR) {
      bf_c64 gv[U], xv[U][NC];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = kb + q + AP_LPR * u;
        const bool kv = k < KK;
        gv[u] = kv ? g[k] : bf_c64{0.f, 0.f};
        const bf_c64* inp = k < rr.K0 ? in0 + k : in1 + k;
        const int64_t ldk = k < rr.K0 ? ld0 : ld1;
#pragma unroll
        for (int c = 0; c < NC; ++c)
          xv[u][c] = (kv && c < ncols) ? inp[(int64_t)c * ldk] : bf_c64{0.f, 0.f};
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc_fma(acc[c], gv[u], xv[u][c]);
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    acc[c].re = row8_sum(acc[c].re);
    acc[c].im = row8_sum(acc[c].im);
  }
  if (q == 0) fused_store<Acc, NC>(rr, B, lds, acc, ncols);
}

constexpr int AF_PF = 8;   // factor entries per lane fetched ahead (rows of up to 64 terms)

__device__ __forceinline__ void fused_fetch_g(const ApplyRowRec& rr, bool has, int q,
                                              const bf_c64* __restrict__ G, bf_c64 (&g)[AF_PF],
                                              int nc_small) {
#pragma unroll
  for (int j = 0; j < AF_PF; ++j) {
    const int k = nc_small ? 2 * q + (j & 1) + 16 * (j >> 1) : q + 8 * j;
    g[j] = (has && k < rr.KK) ? G[rr.g + k] : bf_c64{0.f, 0.f};
  }
}

// One output row whose first AF_PF factor entries per lane are in g: the
// inputs of those slots are loaded together (in chunks of 4 columns), then
// further slots (rows of more than 64 terms) stream from memory.  Same
// slots, same order as fused_row.
template <typename Acc, int NC, bool LI>
__device__ __forceinline__ void fused_row_pre(const ApplyRowRec& rr, const bf_c64 (&g)[AF_PF], int q,
                                              const bf_c64* __restrict__ G, const ApplyBufs& B,
                                              bf_c64* lds, int ncols) {
  const int KK = rr.KK, K0 = rr.K0;
  const bf_c64* in0 = fused_in<LI>(B, lds, rr.in_buf0, rr.in0);
  const bf_c64* in1 = fused_in<LI>(B, lds, rr.in_buf1, rr.in1);
  const int64_t ld0 = fused_in_ld<LI>(B, rr.in_buf0), ld1 = fused_in_ld<LI>(B, rr.in_buf1);
  constexpr int CH = NC < 4 ? NC : 4;
  Acc acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = Acc{0, 0};
  // slots j < AF_PF: factor entries already in registers
#pragma unroll
  for (int c0 = 0; c0 < NC; c0 += CH) {
    bf_c64 xv[AF_PF][CH];
#pragma unroll
    for (int j = 0; j < AF_PF; ++j) {
      const int k = fused_k<NC>(q, j);
      const bool kv = k < KK;
      const bf_c64* inp = k < K0 ? in0 + k : in1 + k;
      const int64_t ldk = k < K0 ? ld0 : ld1;
#pragma unroll
      for (int c = 0; c < CH; ++c)
        xv[j][c] = (kv && c0 + c < ncols) ? inp[(int64_t)(c0 + c) * ldk] : bf_c64{0.f, 0.f};
    }
#pragma unroll
    for (int j = 0; j < AF_PF; ++j)
#pragma unroll
      for (int c = 0; c < CH; ++c) acc_fma(acc[c0 + c], g[j], xv[j][c]);
  }
  // further slots
  for (int j0 = AF_PF; fused_k<NC>(0, j0) < KK; j0 += AF_PF) {
#pragma unroll
    for (int jj = 0; jj < AF_PF; ++jj) {
      const int k = fused_k<NC>(q, j0 + jj);
      const bool kv = k < KK;
      const bf_c64 gk = kv ? G[rr.g + k] : bf_c64{0.f, 0.f};
      const bf_c64* inp = k < K0 ? in0 + k : in1 + k;
      const int64_t ldk = k < K0 ? ld0 : ld1;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const bf_c64 x = (kv && c < ncols) ? inp[(int64_t)c * ldk] : bf_c64{0.f, 0.f};
        acc_fma(acc[c], gk, x);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    acc[c].re = row8_sum(acc[c].re);
    acc[c].im = row8_sum(acc[c].im);
  }
  if (q == 0) fused_store<Acc, NC>(rr, B, lds, acc, ncols);
}

// fused_row_pre in two halves, so that a stage's input loads can be issued
// before the next stage's fetches (memory results return in issue order: a
// wait for the inputs would otherwise wait for those fetches too).
template <int NC, bool LI>
__device__ __forceinline__ void fused_in_load(const ApplyRowRec& rr, int q, const ApplyBufs& B,
                                              bf_c64* lds, int ncols, bf_c64 (&xv)[AF_PF][NC]) {
  const bf_c64* in0 = fused_in<LI>(B, lds, rr.in_buf0, rr.in0);
  const bf_c64* in1 = fused_in<LI>(B, lds, rr.in_buf1, rr.in1);
  const int64_t ld0 = fused_in_ld<LI>(B, rr.in_buf0), ld1 = fused_in_ld<LI>(B, rr.in_buf1);
#pragma unroll
  for (int j = 0; j < AF_PF; ++j) {
    const int k = fused_k<NC>(q, j);
    const bool kv = k < rr.KK;
    const bf_c64* inp = k < rr.K0 ? in0 + k : in1 + k;
    const int64_t ldk = k < rr.K0 ? ld0 : ld1;
#pragma unroll
    for (int c = 0; c < NC; ++c)
      xv[j][c] = (kv && c < ncols) ? inp[(int64_t)c * ldk] : bf_c64{0.f, 0.f};
  }
}

template <typename Acc, int NC, bool LI>
__device__ __forceinline__ void fused_row_fin(const ApplyRowRec& rr, const bf_c64 (&g)[AF_PF],
                                              const bf_c64 (&xv)[AF_PF][NC], int q,
                                              const bf_c64* __restrict__ G, const ApplyBufs& B,
                                              bf_c64* lds, int ncols) {
  const int KK = rr.KK, K0 = rr.K0;
  Acc acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = Acc{0, 0};
#pragma unroll
  for (int j = 0; j < AF_PF; ++j)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc_fma(acc[c], g[j], xv[j][c]);
  // further slots (rows of more than 64 terms)
  if (fused_k<NC>(0, AF_PF) < KK) {
    const bf_c64* in0 = fused_in<LI>(B, lds, rr.in_buf0, rr.in0);
    const bf_c64* in1 = fused_in<LI>(B, lds, rr.in_buf1, rr.in1);
    const int64_t ld0 = fused_in_ld<LI>(B, rr.in_buf0), ld1 = fused_in_ld<LI>(B, rr.in_buf1);
    for (int j0 = AF_PF; fused_k<NC>(0, j0) < KK; j0 += AF_PF) {
#pragma unroll
      for (int jj = 0; jj < AF_PF; ++jj) {
        const int k = fused_k<NC>(q, j0 + jj);
        const bool kv = k < KK;
        const bf_c64 gk = kv ? G[rr.g + k] : bf_c64{0.f, 0.f};
        const bf_c64* inp = k < K0 ? in0 + k : in1 + k;
        const int64_t ldk = k < K0 ? ld0 : ld1;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const bf_c64 x = (kv && c < ncols) ? inp[(int64_t)c * ldk] : bf_c64{0.f, 0.f};
          acc_fma(acc[c], gk, x);
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    acc[c].re = row8_sum(acc[c].re);
    acc[c].im = row8_sum(acc[c].im);
  }
  if (q == 0) fused_store<Acc, NC>(rr, B, lds, acc, ncols);
}

// off[w * (nstage + 1) + t] .. off[w * (nstage + 1) + t + 1]: the row records
// of workgroup w's group in stage t (records grouped by workgroup, then
// stage).  NT threads, NT / 8 rows of a stage at a time; rows are
// independent, so NT changes the schedule only, never the results.  The
// first RPT rows of each thread in stage t + 1 (their records, then their
// factor entries) and their records of stage t + 2 are fetched while stage t
// computes: after a barrier only the inputs, just written by the workgroup
// itself (to LDS), are waited for.  Further rows of a stage take extra passes without
// fetching ahead.
template <typename Acc, int NC, int NT, int RPT>
__global__ __launch_bounds__(NT) void apply_fused_kernel(const ApplyRowRec* __restrict__ rows,
                                                         const int32_t* __restrict__ off,
                                                         int32_t nstage,
                                                         const bf_c64* __restrict__ G,
                                                         ApplyBufs B, int32_t ncols) {
  const int q = threadIdx.x & (AP_LPR - 1);
  const int rl = threadIdx.x / AP_LPR;
  constexpr int RS = NT / AP_LPR;   // rows per pass
  const int32_t* o = off + (int64_t)blockIdx.x * (nstage + 1);
  constexpr int small = NC <= 2;
  __shared__ bf_c64 lds[2 * kFusedLdsRows * NC];
  auto fetch_rec = [&](int t, int i, ApplyRowRec& r) -> bool {
    const int32_t R = o[t] + rl + i * RS;
    const bool h = R < o[t + 1];
    if (h) r = rows[R];
    return h;
  };
  ApplyRowRec rc[RPT], rn[RPT];
  bool hc[RPT], hn[RPT];
  bf_c64 gc[RPT][AF_PF], gn[RPT][AF_PF];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    hc[i] = fetch_rec(0, i, rc[i]);
    hn[i] = nstage > 1 ? fetch_rec(1, i, rn[i]) : false;
  }
#pragma unroll
  for (int i = 0; i < RPT; ++i) fused_fetch_g(rc[i], hc[i], q, G, gc[i], small);
  for (int t = 0; t < nstage; ++t) {
    // inputs of the first row first, then the next stages' fetches, then the
    // arithmetic: the first row waits for its inputs only
    constexpr int RI = NC == 1 ? RPT : 1;   // rows whose inputs go first
    bf_c64 xv0[RI][AF_PF][NC];
#pragma unroll
    for (int i = 0; i < RI; ++i)
      if (hc[i]) {
        if (rc[i].in_buf0 == kFusedLdsBuf)
          fused_in_load<NC, true>(rc[i], q, B, lds, ncols, xv0[i]);
        else
          fused_in_load<NC, false>(rc[i], q, B, lds, ncols, xv0[i]);
      }
    __builtin_amdgcn_sched_barrier(0);
    ApplyRowRec r2[RPT];
    bool h2[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      if (t + 1 < nstage) fused_fetch_g(rn[i], hn[i], q, G, gn[i], small);
      h2[i] = t + 2 < nstage ? fetch_rec(t + 2, i, r2[i]) : false;
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      if (!hc[i]) continue;
      const bool li = rc[i].in_buf0 == kFusedLdsBuf;
      if (i < RI) {
        if (li)
          fused_row_fin<Acc, NC, true>(rc[i], gc[i], xv0[i < RI ? i : 0], q, G, B, lds, ncols);
        else
          fused_row_fin<Acc, NC, false>(rc[i], gc[i], xv0[i < RI ? i : 0], q, G, B, lds, ncols);
      } else if (li) {
        fused_row_pre<Acc, NC, true>(rc[i], gc[i], q, G, B, lds, ncols);
      } else {
        fused_row_pre<Acc, NC, false>(rc[i], gc[i], q, G, B, lds, ncols);
      }
    }
    for (int32_t R = o[t] + rl + RPT * RS; R < o[t + 1]; R += RS) {
      const ApplyRowRec rr = rows[R];
      if (rr.in_buf0 == kFusedLdsBuf)
        fused_row<Acc, NC, true>(rr, q, G, B, lds, ncols);
      else
        fused_row<Acc, NC, false>(rr, q, G, B, lds, ncols);
    }
    if (t + 1 < nstage) __syncthreads();
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      rc[i] = rn[i];
      hc[i] = hn[i];
#pragma unroll
      for (int j = 0; j < AF_PF; ++j) gc[i][j] = gn[i][j];
      rn[i] = r2[i];
      hn[i] = h2[i];
    }
  }
}

// Workgroup shape of a fused launch: 8 threads per row and a stage's rows in
// one pass of up to 128 rows -- 256 threads with one row each for up to 32
// rows, else 512 threads with two rows each fetched ahead for one column
// (one row each for 2 to 4 columns, whose inputs need the registers); larger
// stages take further passes.
template <typename Acc, int NC>
static void launch_fused_nc(dim3 grid, int32_t max_rows, hipStream_t s,
                            const ApplyRowRec* rows_dev, const int32_t* off_dev, int32_t nstage,
                            const bf_c64* G, const ApplyBufs& B, int nc) {
  if (max_rows <= 32) {
    hipLaunchKernelGGL((apply_fused_kernel<Acc, NC, 256, 1>), grid, dim3(256), 0, s, rows_dev,
                       off_dev, nstage, G, B, nc);
  } else if constexpr (NC >= 2) {
    hipLaunchKernelGGL((apply_fused_kernel<Acc, NC, 512, 1>), grid, dim3(512), 0, s, rows_dev,
                       off_dev, nstage, G, B, nc);
  } else {
    hipLaunchKernelGGL((apply_fused_kernel<Acc, NC, 512, 2>), grid, dim3(512), 0, s, rows_dev,
                       off_dev, nstage, G, B, nc);
  }
}

void launch_apply_fused(const ApplyRowRec* rows_dev, const int32_t* off_dev, int32_t nwg,
                        int32_t nstage, int32_t max_rows, const bf_c64* G,
                        const bf_c64* const bufs[4], const int64_t lds[4], int64_t ncols,
                        int prec, hipStream_t s) {
  if (nwg <= 0 || ncols <= 0) return;
  BF_CHECK(ncols <= kApplyFusedCols, BF_EINVAL, "fused apply: too many right-hand sides");
  ApplyBufs B;
  for (int i = 0; i < 4; ++i) {
    B.p[i] = const_cast<bf_c64*>(bufs[i]);
    B.ld[i] = lds[i];
    B.rs[i] = 1;
  }
  const int nc = (int)ncols;
  const dim3 grid((unsigned)nwg);
  (void)prec;
  if (nc == 1) {
    launch_fused_nc<cf, 1>(grid, max_rows, s, rows_dev, off_dev, nstage, G, B, nc);
  } else if (nc == 2) {
    launch_fused_nc<cf, 2>(grid, max_rows, s, rows_dev, off_dev, nstage, G, B, nc);
  } else {
    launch_fused_nc<cf, 4>(grid, max_rows, s, rows_dev, off_dev, nstage, G, B, nc);
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs == hipStreamCaptureStatusNone)
    BF_HIP(hipGetLastError());
}

constexpr size_t AP_LDS_LIMIT = 160 * 1024;

// One workgroup per block: row r of block b multiplies packed row r of its
// factor slice by the block's input rows and writes output row out_row + r.
__global__ void expand_rows_kernel(const ApplyBlk* __restrict__ blks,
                                   ApplyRowRec* __restrict__ rows) {
  const ApplyBlk b = blks[blockIdx.x];
  const int KK = b.K0 + b.K1;
  for (int r = threadIdx.x; r < b.M; r += blockDim.x) {
    ApplyRowRec rr{};
    rr.g = b.g_off + (int64_t)r * KK;
    rr.in0 = b.in_row0;
    rr.in1 = b.in_row1 - b.K0;
    rr.out = b.out_row + r;
    rr.K0 = b.K0;
    rr.KK = KK;
    rr.out_buf = b.out_buf;
    rr.in_buf0 = b.in_buf0;
    rr.in_buf1 = b.in_buf1;
    rows[b.row_rec + r] = rr;
  }
}

void launch_expand_rows(const ApplyBlk* blks_dev, int32_t nblk, ApplyRowRec* rows_dev,
                        hipStream_t s) {
  if (nblk <= 0) return;
  hipLaunchKernelGGL(expand_rows_kernel, dim3((unsigned)nblk), dim3(64), 0, s, blks_dev, rows_dev);
  BF_HIP(hipGetLastError());
}

void launch_apply_stage(const ApplyBlk* blks_dev, int32_t nblk, const ApplyRowRec* rows_dev,
                        int32_t nrows, int32_t maxMK, int32_t maxKK, int32_t maxM, const bf_c64* G,
                        const bf_c64* const bufs[4], const int64_t lds[4], const int64_t rss[4],
                        int64_t ncols, int prec, hipStream_t s, bool may_time) {
  if (nblk <= 0 || ncols <= 0) return;
  ApplyBufs B;
  for (int i = 0; i < 4; ++i) {
    B.p[i] = const_cast<bf_c64*>(bufs[i]);
    B.ld[i] = lds[i];
    B.rs[i] = rss[i];
  }
  if (ncols <= AP_SMALL) {
    // the row records address column-major buffers
    for (int i = 0; i < 4; ++i) BF_CHECK(rss[i] == 1, BF_EINVAL, "few-column apply needs column-major buffers");
    const int nc = (int)ncols;
    const int ncl = nc == 1 ? 1 : (nc == 2 ? 2 : 4);
    auto rec = [&] {
      const dim3 grid((unsigned)((nrows + 256 / AP_LPR - 1) / (256 / AP_LPR)));
      if (ncl == 1)
        hipLaunchKernelGGL((apply_stream_kernel<cf, 1>), grid, dim3(256), 0, s, rows_dev, nrows, G, B, nc);
      else if (ncl == 2)
        hipLaunchKernelGGL((apply_stream_kernel<cf, 2>), grid, dim3(256), 0, s, rows_dev, nrows, G, B, nc);
      else
        hipLaunchKernelGGL((apply_stream_kernel<cf, 4>), grid, dim3(256), 0, s, rows_dev, nrows, G, B, nc);
    };
    // one wave per block while a block's rows fit 3 x 32 terms and 128 rows
    // (a wave walks all of its block's rows); the record kernel otherwise
    const int it = (maxKK + 31) / 32;
    if (it < 1 || it > 3 || maxM > 128) {
      rec();
    } else {
      auto run = [&](int64_t c) {
        if (!c) {
          rec();
          return;
        }
        const int wpb = (int)((c >> 4) & 3) + 1;
        const dim3 grid((unsigned)(((int64_t)nblk * wpb + 3) / 4));
#define AP_BR(N, I, R, X)                                                                      \
  hipLaunchKernelGGL((apply_blockrows_kernel<N, I, R, X, false>), grid, dim3(256), 0, s, blks_dev, \
                     nblk, G, B, nc, 1)
#define AP_BRM(N, I, X)                                                                       \
  hipLaunchKernelGGL((apply_blockrows_kernel<N, I, 1, X, true>), grid, dim3(256), 0, s, blks_dev, \
                     nblk, G, B, nc, wpb)
        const bool xl = (c >> 3) & 1;
        const int rg = (int)(c & 7);
        if (wpb > 1) {
          // one row group per load, several waves per block
          if (ncl == 1) {
            if (it == 1) AP_BRM(1, 1, false); else if (it == 2) AP_BRM(1, 2, false); else AP_BRM(1, 3, false);
          } else if (ncl == 2) {
            if (it == 1) AP_BRM(2, 1, false); else if (it == 2) AP_BRM(2, 2, false); else AP_BRM(2, 3, false);
          } else if (xl) {
            if (it == 1) AP_BRM(4, 1, true); else if (it == 2) AP_BRM(4, 2, true); else AP_BRM(4, 3, true);
          } else {
            if (it == 1) AP_BRM(4, 1, false); else if (it == 2) AP_BRM(4, 2, false); else AP_BRM(4, 3, false);
          }
          return;
        }
        if (ncl == 1) {
          if (it == 1) { if (rg == 4) AP_BR(1, 1, 4, false); else if (rg == 2) AP_BR(1, 1, 2, false); else AP_BR(1, 1, 1, false); }
          else if (it == 2) { if (rg == 2) AP_BR(1, 2, 2, false); else AP_BR(1, 2, 1, false); }
          else { if (rg == 2) AP_BR(1, 3, 2, false); else AP_BR(1, 3, 1, false); }
        } else if (ncl == 2) {
          if (it == 1) { if (rg == 4) AP_BR(2, 1, 4, false); else if (rg == 2) AP_BR(2, 1, 2, false); else AP_BR(2, 1, 1, false); }
          else if (it == 2) { if (rg == 2) AP_BR(2, 2, 2, false); else AP_BR(2, 2, 1, false); }
          else { if (rg == 2) AP_BR(2, 3, 2, false); else AP_BR(2, 3, 1, false); }
        } else if (xl) {
          if (it == 1) { if (rg == 2) AP_BR(4, 1, 2, true); else AP_BR(4, 1, 1, true); }
          else if (it == 2) { if (rg == 2) AP_BR(4, 2, 2, true); else AP_BR(4, 2, 1, true); }
          else { if (rg == 2) AP_BR(4, 3, 2, true); else AP_BR(4, 3, 1, true); }
        } else {
          if (it == 1) { if (rg == 2) AP_BR(4, 1, 2, false); else AP_BR(4, 1, 1, false); }
          else if (it == 2) AP_BR(4, 2, 1, false);
          else AP_BR(4, 3, 1, false);
        }
#undef AP_BR
#undef AP_BRM
      };
      // record kernel (0) or block kernel with rg = c & 7 groups of 8 rows
      // loaded together, its inputs in LDS when bit 3 is set, and
      // ((c >> 4) & 3) + 1 waves sharing each block's row groups (stages of
      // few blocks, which one wave per block leaves idle): all give the same
      // bits; the autotuner picks per shape class
      std::vector<int64_t> cand;
      if (ncl <= 2)
        cand = it == 1 ? std::vector<int64_t>{4, 2, 1, 0} : std::vector<int64_t>{1, 2, 0};
      else
        cand = it == 1 ? std::vector<int64_t>{2, 1, 9, 10, 0} : std::vector<int64_t>{1, 9, 10, 0};
      if (nblk < 4096) {
        for (int64_t w : {16, 48}) {
          cand.push_back(1 + w);
          if (ncl > 2) cand.push_back(9 + w);
        }
      }
      // Stages larger than the last-level cache are not timed: repeated
      // launches of one stage find part of its factors in that cache, which
      // favours other variants than the cold stream of a real apply.  They
      // take the rule measured on cold data (one row group per load, inputs
      // in registers for 1-2 columns and in LDS for 4).
      const int64_t rule = ncl > 2 ? 9 : 1;
      if ((double)nrows * (double)maxKK * sizeof(bf_c64) > 64.0 * (1 << 20))
        run(rule);
      else
        tune_choose(TuneKey{kTuneApplyRows, ncl, it, pow2_ceil(nblk), pow2_ceil(maxM), 0}, cand,
                    rule, s, run, may_time);
    }
  } else if (prec == BF_PREC_BF16X3 && ncols >= AM_MIN_COLS) {
    const int64_t ych = (ncols + AP_CW - 1) / AP_CW;
    BF_CHECK(ych <= 65535, BF_EINVAL, "too many right-hand sides");
    auto wg = [&] {
      hipLaunchKernelGGL(apply_mfma_kernel, dim3((unsigned)nblk, (unsigned)ych), dim3(256), 0, s,
                         blks_dev, G, B, ncols);
    };
    if (maxM <= 16) {
      hipLaunchKernelGGL(apply_mfma_small_kernel, dim3((unsigned)((nblk + 3) / 4), (unsigned)ych),
                         dim3(256), 0, s, blks_dev, nblk, G, B, ncols);
    } else if (maxM <= 64) {
      // one workgroup per block (0) or one wave per block and c column tiles
      // (c = 1, 2, 4, ..., all): same bits, tuned per class; the rule
      // without the tuner fills the device with one tile per wave when the
      // stage has few blocks
      const int64_t nct = (ncols + 15) / 16;
      std::vector<int64_t> cand;
      for (int64_t c = 1; c < nct; c *= 2) cand.push_back(c);
      cand.push_back(nct);
      cand.push_back(0);
      auto run = [&](int64_t c) {
        if (c) {
          const int64_t gy = (nct + c - 1) / c;
          BF_CHECK(gy <= 65535, BF_EINVAL, "too many right-hand sides");
          const dim3 grid((unsigned)((nblk + 3) / 4), (unsigned)gy);
          const int rt = (maxM + 15) / 16;
          if (nblk * gy >= 4096)
            hipLaunchKernelGGL(apply_mfma_wave_kernel, grid, dim3(256), 0, s, blks_dev, nblk, G, B,
                               ncols, (int32_t)c);
          else if (rt == 2)
            launch_wave_lf<2>(grid, s, blks_dev, nblk, G, B, ncols, (int32_t)c);
          else if (rt == 3)
            launch_wave_lf<3>(grid, s, blks_dev, nblk, G, B, ncols, (int32_t)c);
          else
            launch_wave_lf<4>(grid, s, blks_dev, nblk, G, B, ncols, (int32_t)c);
        } else {
          wg();
        }
      };
      tune_choose(TuneKey{kTuneApplyMfma, pow2_ceil(ncols), (maxM + 15) / 16, pow2_ceil(nblk),
                          pow2_ceil(maxKK), 0},
                  cand, nblk >= 4096 ? nct : 1, s, run, may_time);
    } else {
      wg();
    }
  } else {
    const size_t lds_b = sizeof(cf) * ((size_t)maxMK + (size_t)maxKK * AP_CW);
    BF_CHECK(lds_b <= AP_LDS_LIMIT, BF_ERANK, "apply block too large for LDS");
    if (lds_b > 64 * 1024)
      BF_HIP(hipFuncSetAttribute((const void*)apply_blocked_kernel,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_b));
    const int64_t ych = (ncols + AP_CW - 1) / AP_CW;
    BF_CHECK(ych <= 65535, BF_EINVAL, "too many right-hand sides");
    hipLaunchKernelGGL(apply_blocked_kernel, dim3((unsigned)nblk, (unsigned)ych), dim3(256), lds_b,
                       s, blks_dev, G, B, ncols);
  }
  // launch errors of a captured stage surface when the graph is instantiated
  // (the runtime refuses hipGetLastError on a capturing stream)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs == hipStreamCaptureStatusNone)
    BF_HIP(hipGetLastError());
}

template <typename Tout>
__global__ void pack_kernel(const PackDesc* __restrict__ descs, Tout* __restrict__ dst) {
  const PackDesc d = descs[blockIdx.x];
  const int64_t tot = (int64_t)d.M * d.K;
  for (int64_t idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int r = (int)(idx % d.M), k = (int)(idx / d.M);
    bf_c128 v;
    if (d.conjT) {
      v = d.src[(int64_t)(d.row0 + k) + (int64_t)r * d.src_ld];
      v.im = -v.im;
    } else {
      v = d.src[(int64_t)(d.row0 + r) + (int64_t)k * d.src_ld];
    }
    Tout o;
    o.re = v.re;
    o.im = v.im;
    dst[d.dst_off + (int64_t)r * d.dst_rs + (int64_t)k * d.dst_cs] = o;
  }
}

void launch_pack_c64(const PackDesc* d_dev, int32_t ndesc, bf_c64* dst, hipStream_t s) {
  if (ndesc <= 0) return;
  hipLaunchKernelGGL(pack_kernel<bf_c64>, dim3((unsigned)ndesc), dim3(256), 0, s, d_dev, dst);
  BF_HIP(hipGetLastError());
}
void launch_pack_c128(const PackDesc* d_dev, int32_t ndesc, bf_c128* dst, hipStream_t s) {
  if (ndesc <= 0) return;
  hipLaunchKernelGGL(pack_kernel<bf_c128>, dim3((unsigned)ndesc), dim3(256), 0, s, d_dev, dst);
  BF_HIP(hipGetLastError());
}

}  // namespace bf
