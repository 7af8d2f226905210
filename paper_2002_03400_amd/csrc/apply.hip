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

constexpr int AP_COLS = 64;

struct ApplyBufs {
  bf_c64* p[4];
  int64_t ld[4];
};

__global__ __launch_bounds__(256) void apply_stage_kernel(const ApplyDesc* __restrict__ descs,
                                                          const bf_c64* __restrict__ G,
                                                          ApplyBufs B, int64_t ncols) {
  const ApplyDesc d = descs[blockIdx.x];
  const int64_t c0 = (int64_t)blockIdx.y * AP_COLS;
  if (c0 >= ncols) return;
  const int cw = (int)((ncols - c0 < AP_COLS) ? ncols - c0 : AP_COLS);
  const int M = d.M;
  for (int idx = threadIdx.x; idx < M * cw; idx += blockDim.x) {
    const int r = idx % M;
    const int64_t c = c0 + idx / M;
    cf acc = {0.f, 0.f};
    for (int t = 0; t < d.nterm; ++t) {
      const ApplyTerm T = d.t[t];
      const bf_c64* g = G + T.g_off + r;
      const bf_c64* in = B.p[T.in_buf] + c * B.ld[T.in_buf] + T.in_row;
      for (int k = 0; k < T.K; ++k) {
        bf_c64 gv = g[(int64_t)k * M];
        bf_c64 xv = in[k];
        cf_fma(acc, cf{gv.re, gv.im}, cf{xv.re, xv.im});
      }
    }
    B.p[d.out_buf][c * B.ld[d.out_buf] + d.out_row + r] = bf_c64{acc.re, acc.im};
  }
}

void launch_apply_stage(const ApplyDesc* d_dev, int32_t ndesc, const bf_c64* G,
                        const bf_c64* const bufs[4], const int64_t lds[4], int64_t ncols,
                        int32_t maxM, hipStream_t s) {
  (void)maxM;
  if (ndesc <= 0 || ncols <= 0) return;
  ApplyBufs B;
  for (int i = 0; i < 4; ++i) {
    B.p[i] = const_cast<bf_c64*>(bufs[i]);
    B.ld[i] = lds[i];
  }
  int64_t ychunks = (ncols + AP_COLS - 1) / AP_COLS;
  BF_CHECK(ychunks <= 65535, BF_EINVAL, "too many right-hand sides");
  hipLaunchKernelGGL(apply_stage_kernel, dim3((unsigned)ndesc, (unsigned)ychunks), dim3(256), 0,
                     s, d_dev, G, B, ncols);
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
    dst[d.dst_off + idx] = o;
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
