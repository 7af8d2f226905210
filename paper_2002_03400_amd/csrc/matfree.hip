// Black-box products for the built-in test operators: entries of op(A) are
// produced on the fly (never stored) and multiplied into a block of columns.
//
// Y[i, g*ncols + c] = sum_{j in seg_g} E(i, j) X[j, c]    (Sec. 4.1 structured
// samples: group g is the product with the random block living on node g).
//
// Layout: one workgroup of 256 threads owns 256 output rows of one group and
// one slice of the group's inner range (split-K when there are too few row
// tiles to fill 256 CUs); each thread keeps NC complex accumulators in
// registers; a chunk of TK inner points (their coordinates and the TK x NC
// block of X) is staged in LDS and read as broadcasts.  Split-K partials go
// to a scratch buffer and are summed in a fixed order (deterministic).
#include "bf_internal.h"
#include "cplx.h"

namespace bf {

constexpr int MF_THREADS = 256;
constexpr int MF_TK = 64;

// ---- entry functors ------------------------------------------------------

// exp(i k r)/r, r = |p - q|; phase k r / 2pi reduced to [-1/2, 1/2] in FP64,
// then sin/cos of 2 pi f and 1/r in FP32.  sign = -1 gives the conjugate
// (entries of A^H with the point roles swapped).
struct SegEntry {
  PointSet out, in;
  double kk;   // k / (2 pi)
  float sign;
  struct Row { double x, y; };
  struct Col { double x, y; };
  __device__ Row row(int64_t i) const { return Row{out.x[i], out.y[i]}; }
  __device__ Col col(int64_t j) const { return Col{in.x[j], in.y[j]}; }
  __device__ cf entry(const Row& r, const Col& c) const {
    double dx = r.x - c.x, dy = r.y - c.y;
    double rr = sqrt(fma(dx, dx, dy * dy));
    double t = rr * kk;
    double f = t - rint(t);
    float s, co;
    sincospif(2.0f * (float)f, &s, &co);
    float inv = 1.0f / (float)rr;
    return cf{co * inv, sign * s * inv};
  }
};

// exp(2 pi i (j xi / n + c_j |xi|)); the linear phase is reduced modulo n in
// integers.  Forward: output index j (row), inner index k (xi = k - n/2).
struct FioEntry {
  int64_t n;
  const double* cx;  // c(x_j), FP64
  float sign;
  struct Row { int64_t j; double c; };
  struct Col { int64_t xi; };
  __device__ Row row(int64_t j) const { return Row{j, cx[j]}; }
  __device__ Col col(int64_t k) const { return Col{k - n / 2}; }
  __device__ cf entry(const Row& r, const Col& c) const {
    int64_t lin = (r.j * c.xi) % n;
    if (lin < 0) lin += n;
    double ph = (double)lin / (double)n + r.c * (double)(c.xi < 0 ? -c.xi : c.xi);
    double f = ph - rint(ph);
    float s, co;
    sincospif(2.0f * (float)f, &s, &co);
    return cf{co, sign * s};
  }
};
// Adjoint: output index k, inner index j: conj(A_jk).
struct FioAdjEntry {
  int64_t n;
  const double* cx;
  struct Row { int64_t xi; };
  struct Col { int64_t j; double c; };
  __device__ Row row(int64_t k) const { return Row{k - n / 2}; }
  __device__ Col col(int64_t j) const { return Col{j, cx[j]}; }
  __device__ cf entry(const Row& r, const Col& c) const {
    int64_t lin = (c.j * r.xi) % n;
    if (lin < 0) lin += n;
    double ph = (double)lin / (double)n + c.c * (double)(r.xi < 0 ? -r.xi : r.xi);
    double f = ph - rint(ph);
    float s, co;
    sincospif(2.0f * (float)f, &s, &co);
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

template <class E, int NC>
__global__ __launch_bounds__(MF_THREADS) void matfree_kernel(
    E e, int64_t nout, const bf_c64* __restrict__ X, int64_t ldx, int32_t ncols, int32_t c0,
    bf_c64* __restrict__ Y, int64_t ldy, int64_t ycols, const int64_t* __restrict__ seg,
    int32_t nsplit) {
  __shared__ typename E::Col cols[MF_TK];
  __shared__ cf xs[MF_TK][NC];
  const int g = blockIdx.y;
  const int z = blockIdx.z;
  const int64_t i = (int64_t)blockIdx.x * MF_THREADS + threadIdx.x;
  const int64_t j0 = seg[g], j1 = seg[g + 1];
  const int64_t len = j1 - j0;
  const int64_t chunk = (len + nsplit - 1) / nsplit;
  const int64_t a = j0 + (int64_t)z * chunk;
  const int64_t b = (a + chunk < j1) ? a + chunk : j1;
  const int nc = (ncols - c0 < NC) ? ncols - c0 : NC;

  cf acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = cf{0.f, 0.f};
  typename E::Row rw = e.row(i < nout ? i : 0);

  for (int64_t jb = a; jb < b; jb += MF_TK) {
    const int tk = (b - jb < MF_TK) ? (int)(b - jb) : MF_TK;
    __syncthreads();
    for (int idx = threadIdx.x; idx < MF_TK * NC; idx += MF_THREADS) {
      int jj = idx % MF_TK, c = idx / MF_TK;
      bf_c64 v = {0.f, 0.f};
      if (jj < tk && c < nc) v = X[(int64_t)(c0 + c) * ldx + jb + jj];
      xs[jj][c] = cf{v.re, v.im};
    }
    if (threadIdx.x < tk) cols[threadIdx.x] = e.col(jb + threadIdx.x);
    __syncthreads();
    if (i < nout) {
      for (int jj = 0; jj < tk; ++jj) {
        cf av = e.entry(rw, cols[jj]);
#pragma unroll
        for (int c = 0; c < NC; ++c) cf_fma(acc[c], av, xs[jj][c]);
      }
    }
  }
  if (i < nout) {
    bf_c64* yz = Y + (int64_t)z * ycols * ldy;   // split-K partial plane
    for (int c = 0; c < nc; ++c)
      yz[((int64_t)g * ncols + c0 + c) * ldy + i] = bf_c64{acc[c].re, acc[c].im};
  }
}

// Y(:, col) = sum_z P[z](:, col) over the split planes (fixed order).
__global__ void split_reduce_kernel(const bf_c64* __restrict__ P, int64_t nout, int64_t ycols,
                                    int32_t nsplit, bf_c64* __restrict__ Y, int64_t ldy) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nout * ycols) return;
  int64_t r = idx % nout, c = idx / nout;
  float re = 0.f, im = 0.f;
  for (int z = 0; z < nsplit; ++z) {
    bf_c64 v = P[((int64_t)z * ycols + c) * nout + r];
    re += v.re;
    im += v.im;
  }
  Y[c * ldy + r] = bf_c64{re, im};
}

template <class E, int NC>
static void launch_nc(const E& e, int64_t nout, const bf_c64* X, int64_t ldx, int32_t ncols,
                      int32_t c0, bf_c64* Y, int64_t ldy, int64_t ycols, const int64_t* seg_dev,
                      int32_t nseg, int32_t nsplit, hipStream_t s) {
  dim3 grid((unsigned)((nout + MF_THREADS - 1) / MF_THREADS), (unsigned)nseg, (unsigned)nsplit);
  hipLaunchKernelGGL((matfree_kernel<E, NC>), grid, dim3(MF_THREADS), 0, s, e, nout, X, ldx,
                     ncols, c0, Y, ldy, ycols, seg_dev, nsplit);
  BF_HIP(hipGetLastError());
}

template <class E>
static void run_matfree(const E& e, int64_t nout, int64_t nin, const bf_c64* X, int64_t ldx,
                        int64_t ncols, bf_c64* Y, int64_t ldy, const int64_t* seg_host,
                        int32_t nseg, hipStream_t s) {
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
  int64_t tiles = ((nout + MF_THREADS - 1) / MF_THREADS) * nseg;
  int64_t want = (2048 + tiles - 1) / tiles;
  int64_t cap = std::max<int64_t>(1, maxlen / 512);
  int32_t nsplit = (int32_t)std::max<int64_t>(1, std::min<int64_t>({want, cap, 64}));

  DevBuf<int64_t> seg_dev(segv.size(), s);
  BF_HIP(hipMemcpyAsync(seg_dev.p, segv.data(), segv.size() * sizeof(int64_t),
                        hipMemcpyHostToDevice, s));
  const int64_t ycols = (int64_t)nseg * ncols;
  DevBuf<bf_c64> part;
  bf_c64* Yk = Y;
  int64_t ldk = ldy;
  if (nsplit > 1) {
    part = DevBuf<bf_c64>((size_t)nsplit * ycols * nout, s);
    Yk = part.p;
    ldk = nout;
  }
  for (int64_t c0 = 0; c0 < ncols; c0 += 64) {
    int64_t rem = ncols - c0;
    if (rem <= 8)
      launch_nc<E, 8>(e, nout, X, ldx, (int32_t)ncols, (int32_t)c0, Yk, ldk, ycols, seg_dev.p, nseg, nsplit, s);
    else if (rem <= 16)
      launch_nc<E, 16>(e, nout, X, ldx, (int32_t)ncols, (int32_t)c0, Yk, ldk, ycols, seg_dev.p, nseg, nsplit, s);
    else if (rem <= 24)
      launch_nc<E, 24>(e, nout, X, ldx, (int32_t)ncols, (int32_t)c0, Yk, ldk, ycols, seg_dev.p, nseg, nsplit, s);
    else if (rem <= 32)
      launch_nc<E, 32>(e, nout, X, ldx, (int32_t)ncols, (int32_t)c0, Yk, ldk, ycols, seg_dev.p, nseg, nsplit, s);
    else if (rem <= 40)
      launch_nc<E, 40>(e, nout, X, ldx, (int32_t)ncols, (int32_t)c0, Yk, ldk, ycols, seg_dev.p, nseg, nsplit, s);
    else if (rem <= 48)
      launch_nc<E, 48>(e, nout, X, ldx, (int32_t)ncols, (int32_t)c0, Yk, ldk, ycols, seg_dev.p, nseg, nsplit, s);
    else
      launch_nc<E, 64>(e, nout, X, ldx, (int32_t)ncols, (int32_t)c0, Yk, ldk, ycols, seg_dev.p, nseg, nsplit, s);
  }
  if (nsplit > 1) {
    int64_t tot = nout * ycols;
    hipLaunchKernelGGL(split_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                       part.p, nout, ycols, nsplit, Y, ldy);
    BF_HIP(hipGetLastError());
  }
}

void launch_segkernel(PointSet out_pts, int64_t nout, PointSet in_pts, int64_t nin,
                      double k_over_2pi, int sign, const bf_c64* X, int64_t ldx, int64_t ncols,
                      bf_c64* Y, int64_t ldy, const int64_t* seg_host, int32_t nseg,
                      hipStream_t s) {
  SegEntry e{out_pts, in_pts, k_over_2pi, (float)sign};
  run_matfree(e, nout, nin, X, ldx, ncols, Y, ldy, seg_host, nseg, s);
}

void launch_fio(int64_t n, const double* cx_dev, int adjoint, const bf_c64* X, int64_t ldx,
                int64_t ncols, bf_c64* Y, int64_t ldy, const int64_t* seg_host, int32_t nseg,
                hipStream_t s) {
  if (!adjoint) {
    FioEntry e{n, cx_dev, 1.0f};
    run_matfree(e, n, n, X, ldx, ncols, Y, ldy, seg_host, nseg, s);
  } else {
    FioAdjEntry e{n, cx_dev};
    run_matfree(e, n, n, X, ldx, ncols, Y, ldy, seg_host, nseg, s);
  }
}

void launch_dense(const bf_c64* A, int64_t m, int64_t n, int64_t lda, int adjoint,
                  const bf_c64* X, int64_t ldx, int64_t ncols, bf_c64* Y, int64_t ldy,
                  const int64_t* seg_host, int32_t nseg, hipStream_t s) {
  DenseEntry e{A, lda, adjoint};
  if (!adjoint)
    run_matfree(e, m, n, X, ldx, ncols, Y, ldy, seg_host, nseg, s);
  else
    run_matfree(e, n, m, X, ldx, ncols, Y, ldy, seg_host, nseg, s);
}

}  // namespace bf
