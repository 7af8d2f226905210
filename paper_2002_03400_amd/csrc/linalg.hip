// Batched small FP64 complex linear algebra of Alg. 2:
//  * chain_gemm : products with the partially built factors (the V-chain^H,
//                 U-chain^H and X-chain products of the W/R sweeps, and
//                 R^H Z for the centre blocks);
//  * cpqr       : truncated column-pivoted Householder QR (Alg. 1 step 3);
//  * lsq        : centre blocks B = C X^+ (eq. Bij, read from its argmin).
// Blocks are ragged and described by host-built descriptor arrays; one
// workgroup per block (QR, least squares, chain products with blocks of more
// than 16 rows) or one wave per block (chain products of smaller blocks).
// All arithmetic is FP64.
#include "bf_internal.h"
#include "cplx.h"

namespace bf {

template <typename T> __device__ __forceinline__ cd load_c(const T* p);
template <> __device__ __forceinline__ cd load_c<bf_c64>(const bf_c64* p) {
  bf_c64 v = *p;
  return cd{(double)v.re, (double)v.im};
}
template <> __device__ __forceinline__ cd load_c<bf_c128>(const bf_c128* p) {
  bf_c128 v = *p;
  return cd{v.re, v.im};
}

// ---------------------------------------------------------------- gemm ----
// grid (ndesc, ceil(max_ncols / 64)); a workgroup of 4 waves computes rows
// 0..M-1 of one descriptor (in row blocks of 20, 24, 32 or 64: the smallest
// that holds the launch's largest M) for
// the 64-column chunk blockIdx.y.
// Lane l of every wave owns column l of the chunk and wave w the rows w,
// w+4, ... of the block.  op(F) is staged in LDS in chunks of 64 (or 32)
// inner indices as [k][row] and read as a broadcast; each lane reads its own input
// column straight from global memory (contiguous along k, shared by the 4
// waves through L1) and writes its results directly.  The 32 KB of LDS lets
// several workgroups per CU hide the load latency.
constexpr int CG_COLS = 64;
constexpr int CG_YMAX = 65535;

// op(F) rows [rb, rb + mr), inner indices [k0, k0 + kt) -> fs[k][r]
template <int ROWS, int KT>
__device__ __forceinline__ void cg_stage(cd (*fs)[ROWS], const GemmTerm& T, int rb, int mr,
                                         int k0, int kt) {
  if (T.op == 0) {   // F is M x K column-major: op(F)[r][k] = F[k f_ld + r]
    for (int idx = threadIdx.x; idx < KT * ROWS; idx += 256) {
      const int r = idx % ROWS, k = idx / ROWS;
      cd v = {0.0, 0.0};
      if (r < mr && k < kt) {
        const bf_c128 f = T.F[(int64_t)(k0 + k) * T.f_ld + rb + r];
        v = cd{f.re, f.im};
      }
      fs[k][r] = v;
    }
  } else {           // F is K x M column-major: op(F)[r][k] = conj(F[r f_ld + k])
    for (int idx = threadIdx.x; idx < KT * ROWS; idx += 256) {
      const int k = idx % KT, r = idx / KT;
      cd v = {0.0, 0.0};
      if (r < mr && k < kt) {
        const bf_c128 f = T.F[(int64_t)(rb + r) * T.f_ld + k0 + k];
        v = cd{f.re, -f.im};
      }
      fs[k][r] = v;
    }
  }
}

template <typename Tin, int ROWS>
__device__ __forceinline__ void cg_accum(cd* acc, const cd (*fs)[ROWS], const Tin* ip, int64_t rs,
                                         int kt, int wave, int mr) {
  int k = 0;
  for (; k + 4 <= kt; k += 4) {
    cd x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = load_c<Tin>(ip + (k + u) * rs);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int i = 0; i < ROWS / 4; ++i)
        if (wave + 4 * i < mr) cd_fma(acc[i], fs[k + u][wave + 4 * i], x[u]);
  }
  for (; k < kt; ++k) {
    const cd x = load_c<Tin>(ip + k * rs);
#pragma unroll
    for (int i = 0; i < ROWS / 4; ++i)
      if (wave + 4 * i < mr) cd_fma(acc[i], fs[k][wave + 4 * i], x);
  }
}

// ROWS x KT entries of op(F) in LDS: 20 / 24 / 32 x 64 or 40 / 48 / 64 x 32
// (at most 32 KB).  Each wave owns ROWS / 4 rows, so a ROWS close above the launch's
// largest M leaves few idle row slots (M = 19 on 20 rows instead of 32).
template <typename Tin, int ROWS>
__global__ __launch_bounds__(256) void chain_gemm_kernel(const GemmDesc* __restrict__ descs) {
  constexpr int KT = ROWS > 32 ? 32 : 64;
  __shared__ cd fs[KT][ROWS];
  const GemmDesc d = descs[blockIdx.x];
  if (d.M <= 0 || (int)blockIdx.y * CG_COLS >= d.ncols) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nchunk = (d.ncols + CG_COLS - 1) / CG_COLS;
  for (int ch = blockIdx.y; ch < nchunk; ch += gridDim.y) {
    const int c = ch * CG_COLS + lane;
    const bool live = c < d.ncols;
    for (int rb = 0; rb < d.M; rb += ROWS) {
      const int mr = (d.M - rb < ROWS) ? d.M - rb : ROWS;
      cd acc[ROWS / 4];
#pragma unroll
      for (int i = 0; i < ROWS / 4; ++i) acc[i] = cd{0.0, 0.0};
      for (int t = 0; t < d.nterm; ++t) {
        const GemmTerm T = d.t[t];
        const Tin* inp =
            static_cast<const Tin*>(T.in) + (int64_t)(live ? c : ch * CG_COLS) * T.in_ld;
        for (int k0 = 0; k0 < T.K; k0 += KT) {
          const int kt = (T.K - k0 < KT) ? T.K - k0 : KT;
          __syncthreads();
          cg_stage<ROWS, KT>(fs, T, rb, mr, k0, kt);
          __syncthreads();
          cg_accum<Tin, ROWS>(acc, fs, inp + k0 * T.in_rs, T.in_rs, kt, wave, mr);
        }
      }
      if (live) {
        const int64_t ors = d.out_rs;
        bf_c128* o = d.out + (int64_t)c * d.out_ld + rb * ors;
#pragma unroll
        for (int i = 0; i < ROWS / 4; ++i)
          if (wave + 4 * i < mr) o[(wave + 4 * i) * ors] = bf_c128{acc[i].re, acc[i].im};
      }
    }
  }
}

// Small descriptors (every M <= RM, RM = 8 or 16), such as the transfer
// blocks of rank-8 butterflies: a whole workgroup per descriptor would leave
// most lanes and most of its staged tile empty, so each wave takes one
// descriptor and a chunk of CS_TC * 64 / RM columns.  Lane l owns row l % RM
// and columns cg + (64 / RM) u (cg = l / RM, u < CS_TC): per inner index it
// loads op(F)[row][k] once and reuses it for its CS_TC columns, whose input
// entries are shared by the RM lanes of the column through L1.  Same FP64
// operation order as chain_gemm_kernel (terms, then k ascending), so the two
// give identical results.
constexpr int CS_TC = 4;

template <typename Tin, int RM>
__global__ __launch_bounds__(256) void chain_small_kernel(const GemmDesc* __restrict__ descs,
                                                          int64_t ndesc) {
  constexpr int CG = 64 / RM, CW = CG * CS_TC;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t di = (int64_t)blockIdx.x * 4 + wave;
  if (di >= ndesc) return;
  const GemmDesc& d = descs[di];
  if (d.M <= 0) return;
  const int r = lane % RM, cg = lane / RM;
  const bool rlive = r < d.M;
  for (int cb = (int)blockIdx.y * CW; cb < d.ncols; cb += (int)gridDim.y * CW) {
    const int ncc = (d.ncols - cb < CW) ? d.ncols - cb : CW;
    bool live[CS_TC];
    int col[CS_TC];
#pragma unroll
    for (int u = 0; u < CS_TC; ++u) {
      live[u] = rlive && cg + CG * u < ncc;
      col[u] = live[u] ? cb + cg + CG * u : cb;
    }
    cd acc[CS_TC];
#pragma unroll
    for (int u = 0; u < CS_TC; ++u) acc[u] = cd{0.0, 0.0};
    for (int t = 0; t < d.nterm; ++t) {
      const GemmTerm& T = d.t[t];
      const Tin* in = static_cast<const Tin*>(T.in);
      const int rr = rlive ? r : 0;
      const bf_c128* fp = T.F + (T.op == 0 ? rr : (int64_t)rr * T.f_ld);
      const int64_t fs = T.op == 0 ? T.f_ld : 1;
      const double sg = T.op == 0 ? 1.0 : -1.0;
      const Tin* ip[CS_TC];
#pragma unroll
      for (int u = 0; u < CS_TC; ++u) ip[u] = in + (int64_t)col[u] * T.in_ld;
      const int64_t rs = T.in_rs;
#pragma unroll 2
      for (int k = 0; k < T.K; ++k) {
        const bf_c128 fv = fp[(int64_t)k * fs];
        const cd f{fv.re, sg * fv.im};
#pragma unroll
        for (int u = 0; u < CS_TC; ++u)
          if (CG * u < ncc) cd_fma(acc[u], f, load_c<Tin>(ip[u] + k * rs));
      }
    }
#pragma unroll
    for (int u = 0; u < CS_TC; ++u)
      if (live[u])
        d.out[(int64_t)col[u] * d.out_ld + (int64_t)r * d.out_rs] = bf_c128{acc[u].re, acc[u].im};
  }
}

// One launch with tile height `rows`: 8 or 16 (chain_small_kernel, every
// descriptor's M at most that) or 20 / 24 / 32 / 40 / 48 / 64
// (chain_gemm_kernel, row blocks of that height: ranks of 33 to 48 leave
// fewer idle rows on 40 or 48 than on 64).  Every height gives the same FP64
// operation order.
template <typename Tin>
static void launch_chain_rows(const GemmDesc* d_dev, int32_t ndesc, int32_t max_ncols, int rows,
                              hipStream_t s) {
  if (rows <= 16) {
    const int cw = (rows <= 8 ? 8 : 4) * CS_TC;
    dim3 grid((unsigned)((ndesc + 3) / 4),
              (unsigned)std::min((max_ncols + cw - 1) / cw, CG_YMAX));
    if (rows <= 8)
      hipLaunchKernelGGL((chain_small_kernel<Tin, 8>), grid, dim3(256), 0, s, d_dev,
                         (int64_t)ndesc);
    else
      hipLaunchKernelGGL((chain_small_kernel<Tin, 16>), grid, dim3(256), 0, s, d_dev,
                         (int64_t)ndesc);
    return;
  }
  const int nchunk = (max_ncols + CG_COLS - 1) / CG_COLS;
  dim3 grid((unsigned)ndesc, (unsigned)std::min(nchunk, CG_YMAX));
  if (rows <= 20)
    hipLaunchKernelGGL((chain_gemm_kernel<Tin, 20>), grid, dim3(256), 0, s, d_dev);
  else if (rows <= 24)
    hipLaunchKernelGGL((chain_gemm_kernel<Tin, 24>), grid, dim3(256), 0, s, d_dev);
  else if (rows <= 32)
    hipLaunchKernelGGL((chain_gemm_kernel<Tin, 32>), grid, dim3(256), 0, s, d_dev);
  else if (rows <= 40)
    hipLaunchKernelGGL((chain_gemm_kernel<Tin, 40>), grid, dim3(256), 0, s, d_dev);
  else if (rows <= 48)
    hipLaunchKernelGGL((chain_gemm_kernel<Tin, 48>), grid, dim3(256), 0, s, d_dev);
  else
    hipLaunchKernelGGL((chain_gemm_kernel<Tin, 64>), grid, dim3(256), 0, s, d_dev);
}

// Tile heights at least the launch's largest M (32 and 64 above 64 rows);
// the smallest is the rule without the autotuner.
template <typename Tin>
static void launch_chain_t(const GemmDesc* d_dev, int32_t ndesc, int32_t max_ncols,
                           int32_t max_M, hipStream_t s) {
  std::vector<int64_t> cand;
  for (int h : {8, 16, 20, 24, 32, 40, 48, 64})
    if (h >= max_M) cand.push_back(h);
  if (cand.empty()) cand = {32, 64};
  const TuneKey key{kTuneChainRows, sizeof(Tin) == sizeof(bf_c64) ? 1 : 0, max_M,
                    pow2_ceil(ndesc), pow2_ceil(max_ncols), 0};
  tune_choose(key, cand, cand.front(), s, [&](int64_t h) {
    launch_chain_rows<Tin>(d_dev, ndesc, max_ncols, (int)h, s);
  });
}

void launch_chain_gemm(const GemmDesc* d_dev, int32_t ndesc, int32_t max_ncols, int32_t max_M,
                       int32_t max_Ksum, bool in_c64, hipStream_t s) {
  if (ndesc <= 0 || max_ncols <= 0 || max_M <= 0) return;
  (void)max_Ksum;
  ProfScope ps(BF_KC_CHAIN, s, 0.0, 0.0);
  if (in_c64)
    launch_chain_t<bf_c64>(d_dev, ndesc, max_ncols, max_M, s);
  else
    launch_chain_t<bf_c128>(d_dev, ndesc, max_ncols, max_M, s);
  BF_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- cpqr ----
// Businger-Golub pivoting, complex Householder reflectors
// H = I - 2 v v^H / (v^H v), v = x - alpha e1, alpha = -exp(i arg x0) ||x||;
// column norms of the trailing rows are recomputed after every update (never
// downdated).  Rank: first k >= 1 with ||A[k:, k:]||_F <= tol ||Z||_F, else
// min(M, N); an empty block has rank 0.
//
// Work mapping: 4 waves; wave w updates columns j = k+1+w, k+5+w, ...; its 64
// lanes stride over the rows and reduce the reflector dot products with
// butterfly shuffles.  The block lives in LDS (column-major, ld = M) when it
// fits, else in a global scratch slot.  After the loop the reflectors (stored
// in the dead columns of A) are accumulated backwards into Q, which overwrites
// A column by column.
constexpr int QR_THREADS = 256;        // blocks held in LDS
constexpr int QR_BIG_THREADS = 1024;   // blocks in global scratch
constexpr int64_t QR_SCRATCH_BYTES = int64_t(1) << 30;

struct QRShared {
  double tail2;
  int piv;
  int stop;
};

__device__ __forceinline__ void reflect_column(cd* A, int M, int k, int j, const cd* v, double tau,
                                               int lane, double* norm_out) {
  // w = v^H A[k:, j];  A[k:, j] -= tau v w;  optionally the new norm^2 of rows k+1..
  cd w = {0.0, 0.0};
  for (int i = k + lane; i < M; i += 64) cd_cfma(w, v[i - k], A[(int64_t)j * M + i]);
  w = wave_sum(w);
  double nn = 0.0;
  for (int i = k + lane; i < M; i += 64) {
    cd a = A[(int64_t)j * M + i];
    cd tv = cd_mul(v[i - k], w);
    a.re -= tau * tv.re;
    a.im -= tau * tv.im;
    A[(int64_t)j * M + i] = a;
    if (i > k) nn += cd_abs2(a);
  }
  if (norm_out) {
    nn = wave_sum(nn);
    if (lane == 0) *norm_out = nn;
  }
}

// One block by one workgroup of NT threads (every thread calls it with the
// same descriptor; returns together).  smem: the workgroup's dynamic LDS;
// gslot: the block's global scratch slot when use_lds == 0.
template <typename Tin, int NT>
__device__ void cpqr_block(const QRDesc& d, double tol, int32_t* __restrict__ rank_out,
                           double* smem_raw, bf_c128* gslot, int use_lds) {
  const int M = d.M, N = d.N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (M == 0 || N == 0) {
    if (tid == 0) *rank_out = 0;
    return;
  }
  // LDS layout: [norm2 N][vn2 N][tmp M (cd)][QRShared][A M*N (cd) if use_lds]
  double* norm2 = smem_raw;
  double* vn2 = norm2 + N;
  cd* tmp = reinterpret_cast<cd*>(vn2 + N);
  QRShared* sh = reinterpret_cast<QRShared*>(tmp + M);
  cd* A = use_lds ? reinterpret_cast<cd*>(reinterpret_cast<char*>(sh) + 64)
                  : reinterpret_cast<cd*>(gslot);
  const Tin* in = static_cast<const Tin*>(d.in);
  if (d.in_rs == 1) {        // column-major input: consecutive threads, consecutive rows
    for (int idx = tid; idx < M * N; idx += NT) {
      int i = idx % M, j = idx / M;
      A[idx] = load_c<Tin>(in + (int64_t)j * d.in_ld + i);
    }
  } else {                   // row-major input: consecutive threads, consecutive columns
    for (int idx = tid; idx < M * N; idx += NT) {
      int j = idx % N, i = idx / N;
      A[(int64_t)j * M + i] = load_c<Tin>(in + (int64_t)j * d.in_ld + (int64_t)i * d.in_rs);
    }
  }
  __syncthreads();
  // initial column norms (wave per column) and the total
  for (int j = wave; j < N; j += (NT / 64)) {
    double nn = 0.0;
    for (int i = lane; i < M; i += 64) nn += cd_abs2(A[(int64_t)j * M + i]);
    nn = wave_sum(nn);
    if (lane == 0) norm2[j] = nn;
  }
  __syncthreads();
  double total2 = 0.0;
  {
    double part = 0.0;
    for (int j = lane; j < N; j += 64) part += norm2[j];
    total2 = wave_sum(part);  // every wave computes the same value
  }
  const double thr2 = tol * tol * total2;
  const int kmax = M < N ? M : N;
  int rank = kmax;
  for (int k = 0; k < kmax; ++k) {
    if (wave == 0) {
      // trailing Frobenius norm^2 and first argmax of the trailing column norms
      double part = 0.0, best = -1.0;
      int bidx = N;
      for (int j = k + lane; j < N; j += 64) {
        double v = norm2[j];
        part += v;
        if (v > best) { best = v; bidx = j; }
      }
      double tail2 = wave_sum(part);
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        double ob = __shfl_xor(best, off, 64);
        int oi = __shfl_xor(bidx, off, 64);
        if (ob > best || (ob == best && oi < bidx)) { best = ob; bidx = oi; }
      }
      if (lane == 0) {
        sh->tail2 = tail2;
        sh->piv = bidx;
        sh->stop = (k >= 1 && tail2 <= thr2) ? 1 : 0;
      }
    }
    __syncthreads();
    if (sh->stop) { rank = k; break; }
    const int p = sh->piv;
    if (p != k) {
      for (int i = tid; i < M; i += NT) {
        cd a = A[(int64_t)k * M + i];
        A[(int64_t)k * M + i] = A[(int64_t)p * M + i];
        A[(int64_t)p * M + i] = a;
      }
      if (tid == 0) { double t = norm2[k]; norm2[k] = norm2[p]; norm2[p] = t; }
    }
    __syncthreads();
    // Householder vector of column k, stored in place (A[k:, k] <- v)
    if (wave == 0) {
      double xn2 = 0.0;
      for (int i = k + lane; i < M; i += 64) xn2 += cd_abs2(A[(int64_t)k * M + i]);
      xn2 = wave_sum(xn2);
      const double xn = sqrt(xn2);
      if (lane == 0) {
        cd x0 = A[(int64_t)k * M + k];
        double ax0 = sqrt(cd_abs2(x0));
        cd ph = ax0 > 0.0 ? cd{x0.re / ax0, x0.im / ax0} : cd{1.0, 0.0};
        cd alpha = cd{-ph.re * xn, -ph.im * xn};
        A[(int64_t)k * M + k] = cd_sub(x0, alpha);
        vn2[k] = 2.0 * (xn2 + ax0 * xn);
      }
    }
    __syncthreads();
    const double vv = vn2[k];
    if (vv > 0.0) {
      const double tau = 2.0 / vv;
      const cd* v = A + (int64_t)k * M + k;
      for (int j = k + 1 + wave; j < N; j += (NT / 64))
        reflect_column(A, M, k, j, v, tau, lane, &norm2[j]);
    } else {
      // x = 0: H = I; trailing norms just lose row k
      for (int j = k + 1 + wave; j < N; j += (NT / 64)) {
        double nn = 0.0;
        for (int i = k + 1 + lane; i < M; i += 64) nn += cd_abs2(A[(int64_t)j * M + i]);
        nn = wave_sum(nn);
        if (lane == 0) norm2[j] = nn;
      }
    }
    __syncthreads();
  }
  // Q = H_0 ... H_{rank-1} [I; 0], accumulated backwards; column k of Q stays
  // e_k until step k, and H_k only touches columns k..rank-1.
  for (int k = rank - 1; k >= 0; --k) {
    for (int i = tid; i < M; i += NT) {
      if (i >= k) tmp[i - k] = A[(int64_t)k * M + i];
      A[(int64_t)k * M + i] = cd{i == k ? 1.0 : 0.0, 0.0};
    }
    __syncthreads();
    const double vv = vn2[k];
    if (vv > 0.0) {
      const double tau = 2.0 / vv;
      for (int j = k + wave; j < rank; j += (NT / 64))
        reflect_column(A, M, k, j, tmp, tau, lane, nullptr);
    }
    __syncthreads();
  }
  for (int idx = tid; idx < M * rank; idx += NT) {
    cd a = A[idx];
    d.q[idx] = bf_c128{a.re, a.im};
  }
  if (tid == 0) *rank_out = rank;
}

template <typename Tin, int NT>
__global__ __launch_bounds__(NT) void cpqr_kernel(const QRDesc* __restrict__ descs,
                                                  double tol, int32_t* __restrict__ ranks,
                                                  bf_c128* __restrict__ gscratch,
                                                  int64_t scratch_slot, int use_lds) {
  extern __shared__ double smem_raw[];
  cpqr_block<Tin, NT>(descs[blockIdx.x], tol, ranks + blockIdx.x, smem_raw,
                      gscratch + (int64_t)blockIdx.x * scratch_slot, use_lds);
}

static size_t cpqr_lds_bytes(int M, int N, bool with_block) {
  size_t b = 2 * sizeof(double) * N + sizeof(cd) * M + 64;
  if (with_block) b += sizeof(cd) * (size_t)M * N;
  return b;
}

constexpr size_t LDS_LIMIT = 160 * 1024;

void launch_cpqr(const QRDesc* d_dev, int32_t nblk, int32_t maxM, int32_t maxN, double tol,
                 bool in_c64, int32_t* ranks_dev, hipStream_t s) {
  if (nblk <= 0) return;
  BF_CHECK(maxM <= BF_MAX_BLOCK_ROWS && maxN <= BF_MAX_BLOCK_COLS, BF_ERANK,
           "block exceeds BF_MAX_BLOCK_ROWS/COLS");
  ProfScope ps(BF_KC_CPQR, s, 0.0, 0.0);
  size_t lds = cpqr_lds_bytes(maxM, maxN, true);
  if (lds <= LDS_LIMIT) {
    // 256 or 512 threads: each column's updates and sums stay with one wave
    // either way, so both give the same bits
    auto run = [&](int64_t nt) {
      auto kern = nt == 512 ? (in_c64 ? cpqr_kernel<bf_c64, 512> : cpqr_kernel<bf_c128, 512>)
                            : (in_c64 ? cpqr_kernel<bf_c64, QR_THREADS>
                                      : cpqr_kernel<bf_c128, QR_THREADS>);
      if (lds > 64 * 1024)
        BF_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
      hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3((unsigned)nt), lds, s, d_dev, tol,
                         ranks_dev, (bf_c128*)nullptr, (int64_t)0, 1);
      BF_HIP(hipGetLastError());
    };
    const TuneKey key{kTuneCpqrThreads, in_c64 ? 1 : 0, pow2_ceil(maxM), pow2_ceil(maxN),
                      pow2_ceil(nblk), 0};
    tune_choose(key, {QR_THREADS, 512}, QR_THREADS, s, run);
    return;
  }
  // Blocks too large for LDS live in a global scratch slot each (L2-resident
  // working set); 16 waves per block hide the longer load latency.  Launched
  // in chunks that bound the scratch to QR_SCRATCH_BYTES.
  lds = cpqr_lds_bytes(maxM, maxN, false);
  const int64_t slot = (int64_t)maxM * maxN;
  const int64_t chunk = std::max<int64_t>(
      1, std::min<int64_t>(nblk, QR_SCRATCH_BYTES / (slot * (int64_t)sizeof(bf_c128))));
  DevBuf<bf_c128> scratch((size_t)(slot * chunk), s);
  auto kern = in_c64 ? cpqr_kernel<bf_c64, QR_BIG_THREADS> : cpqr_kernel<bf_c128, QR_BIG_THREADS>;
  if (lds > 64 * 1024)
    BF_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
  for (int64_t b0 = 0; b0 < nblk; b0 += chunk) {
    const int64_t nb = std::min<int64_t>(chunk, nblk - b0);
    hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(QR_BIG_THREADS), lds, s, d_dev + b0, tol,
                       ranks_dev + b0, scratch.p, slot, 0);
    BF_HIP(hipGetLastError());
  }
}

// ---------------------------------------------------------------- lsq -----
// B = argmin ||C - B X||_F for C (kU x s), X (kV x s), s >= kV:
//   X^H = Q_x R_x (Householder, no pivoting), then R_x B^H = Q_x^H C^H.
// Both X^H (s x kV) and C^H (s x kU) are held in LDS and reduced together.
template <int NT>
__device__ void lsq_block(const LSDesc& d, double* smem_raw, bf_c128* gslot, int use_lds) {
  const int S = d.s, KV = d.kV, KU = d.kU;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (KU == 0 || KV == 0) return;
  // LDS: [vn2 KV][diag KV (cd)][XH S*KV][CH S*KU]; XH and CH in a global
  // scratch slot instead when they do not fit
  double* vn2 = smem_raw;
  cd* diag = reinterpret_cast<cd*>(vn2 + KV);
  cd* XH = use_lds ? diag + KV                              // X^H, S x KV, ld S
                   : reinterpret_cast<cd*>(gslot);
  cd* CH = XH + (int64_t)S * KV;           // C^H, S x KU, ld S
  for (int idx = tid; idx < S * KV; idx += NT) {
    int i = idx % S, j = idx / S;          // XH[i, j] = conj(X[j, i])
    bf_c128 x = d.X[(int64_t)i * d.ldx + (int64_t)j * d.rsx];
    XH[idx] = cd{x.re, -x.im};
  }
  for (int idx = tid; idx < S * KU; idx += NT) {
    int i = idx % S, j = idx / S;
    bf_c128 c = d.C[(int64_t)i * d.ldc + j];
    CH[idx] = cd{c.re, -c.im};
  }
  __syncthreads();
  const int kmax = KV < S ? KV : S;
  for (int k = 0; k < kmax; ++k) {
    if (wave == 0) {
      double xn2 = 0.0;
      for (int i = k + lane; i < S; i += 64) xn2 += cd_abs2(XH[(int64_t)k * S + i]);
      xn2 = wave_sum(xn2);
      const double xn = sqrt(xn2);
      if (lane == 0) {
        cd x0 = XH[(int64_t)k * S + k];
        double ax0 = sqrt(cd_abs2(x0));
        cd ph = ax0 > 0.0 ? cd{x0.re / ax0, x0.im / ax0} : cd{1.0, 0.0};
        cd alpha = cd{-ph.re * xn, -ph.im * xn};
        diag[k] = alpha;                                // R_x(k, k)
        XH[(int64_t)k * S + k] = cd_sub(x0, alpha);     // v stored in place
        vn2[k] = 2.0 * (xn2 + ax0 * xn);
      }
    }
    __syncthreads();
    const double vv = vn2[k];
    if (vv > 0.0) {
      const double tau = 2.0 / vv;
      const cd* v = XH + (int64_t)k * S + k;
      for (int j = k + 1 + wave; j < KV; j += (NT / 64))
        reflect_column(XH, S, k, j, v, tau, lane, nullptr);
      for (int j = wave; j < KU; j += (NT / 64))
        reflect_column(CH, S, k, j, v, tau, lane, nullptr);
    }
    __syncthreads();
  }
  // R_x b = (Q_x^H C^H)[0:KV, c] for every column c; R_x(r, q) = XH[r, q]
  // for q > r, R_x(r, r) = diag[r].
  for (int c = tid; c < KU; c += NT) {
    cd* y = CH + (int64_t)c * S;
    for (int r = KV - 1; r >= 0; --r) {
      cd acc = y[r];
      for (int q = r + 1; q < KV; ++q) acc = cd_sub(acc, cd_mul(XH[(int64_t)q * S + r], y[q]));
      cd dg = diag[r];
      double den = cd_abs2(dg);
      y[r] = den > 0.0 ? cd{(acc.re * dg.re + acc.im * dg.im) / den,
                            (acc.im * dg.re - acc.re * dg.im) / den}
                       : cd{0.0, 0.0};
    }
    for (int r = 0; r < KV; ++r) {          // B[c, r] = conj(b[r])
      cd bv = y[r];
      d.B[(int64_t)r * KU + c] = bf_c128{bv.re, -bv.im};
    }
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void lsq_kernel(const LSDesc* __restrict__ descs,
                                                 bf_c128* __restrict__ gscratch,
                                                 int64_t scratch_slot, int use_lds) {
  extern __shared__ double smem_raw[];
  lsq_block<NT>(descs[blockIdx.x], smem_raw, gscratch + (int64_t)blockIdx.x * scratch_slot,
                use_lds);
}

void launch_lsq(const LSDesc* d_dev, int32_t nblk, int32_t maxS, int32_t maxK, hipStream_t s) {
  if (nblk <= 0) return;
  BF_CHECK(maxK <= BF_MAX_BLOCK_COLS && maxS <= 2 * BF_MAX_BLOCK_COLS, BF_ERANK,
           "centre block exceeds BF_MAX_BLOCK_COLS");
  ProfScope ps(BF_KC_LSQ, s, 0.0, 0.0);
  const size_t head = (sizeof(double) + sizeof(cd)) * maxK;
  const int64_t slot = (int64_t)maxS * (2 * maxK);
  size_t lds = head + sizeof(cd) * (size_t)slot;
  if (lds <= LDS_LIMIT) {
    if (lds > 64 * 1024)
      BF_HIP(hipFuncSetAttribute((const void*)lsq_kernel<QR_THREADS>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(lsq_kernel<QR_THREADS>, dim3((unsigned)nblk), dim3(QR_THREADS), lds, s,
                       d_dev, (bf_c128*)nullptr, (int64_t)0, 1);
    BF_HIP(hipGetLastError());
    return;
  }
  lds = head;
  BF_CHECK(lds <= LDS_LIMIT, BF_ERANK, "centre block too large for the least-squares kernel");
  const int64_t chunk = std::max<int64_t>(
      1, std::min<int64_t>(nblk, QR_SCRATCH_BYTES / (slot * (int64_t)sizeof(bf_c128))));
  DevBuf<bf_c128> scratch((size_t)(slot * chunk), s);
  if (lds > 64 * 1024)
    BF_HIP(hipFuncSetAttribute((const void*)lsq_kernel<QR_BIG_THREADS>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  for (int64_t b0 = 0; b0 < nblk; b0 += chunk) {
    const int64_t nb = std::min<int64_t>(chunk, nblk - b0);
    hipLaunchKernelGGL(lsq_kernel<QR_BIG_THREADS>, dim3((unsigned)nb), dim3(QR_BIG_THREADS), lds,
                       s, d_dev + b0, scratch.p, slot, 0);
    BF_HIP(hipGetLastError());
  }
}

// ------------------------------------------------ cross-request rounds ----
// One persistent launch for the level solves of every construction in flight
// (request engine): item i of the work list is block items[i].block of work
// items[i].work, a work being one request's batch of truncated pivoted QRs
// (Alg. 1 step 3 on a level's Z blocks) or centre-block least squares (eq.
// Bij read from its argmin).  Items come sorted by estimated cost and
// workgroup g takes items g, g + G, g + 2G, ... of the nitems[0] items.  Each
// block runs the same code as cpqr_kernel / lsq_kernel on their LDS path, so
// its result does not depend on the other requests of the round.
__global__ __launch_bounds__(QR_THREADS) void solve_round_kernel(const SolveWork* __restrict__ works,
                                                                 const SolveItem* __restrict__ items,
                                                                 const int32_t* __restrict__ nitems) {
  extern __shared__ double smem_raw[];
  const int32_t n = *nitems;
  for (int32_t it = blockIdx.x; it < n; it += gridDim.x) {
    const SolveItem item = items[it];
    const SolveWork w = works[item.work];
    if (w.kind == kSolveQR) {
      const QRDesc d = static_cast<const QRDesc*>(w.descs)[item.block];
      if (w.in_c64)
        cpqr_block<bf_c64, QR_THREADS>(d, w.tol, w.ranks + item.block, smem_raw, nullptr, 1);
      else
        cpqr_block<bf_c128, QR_THREADS>(d, w.tol, w.ranks + item.block, smem_raw, nullptr, 1);
    } else {
      const LSDesc d = static_cast<const LSDesc*>(w.descs)[item.block];
      lsq_block<QR_THREADS>(d, smem_raw, nullptr, 1);
    }
    __syncthreads();   // the next item reuses the LDS
  }
}

size_t solve_lds_qr(int32_t maxM, int32_t maxN) { return cpqr_lds_bytes(maxM, maxN, true); }
size_t solve_lds_lsq(int32_t maxS, int32_t maxK) {
  return (sizeof(double) + sizeof(cd)) * (size_t)maxK + sizeof(cd) * (size_t)maxS * (2 * maxK);
}
size_t solve_lds_limit() { return LDS_LIMIT; }

void launch_solve_round(const SolveWork* works, const SolveItem* items, const int32_t* nitems,
                        int32_t grid, size_t lds, hipStream_t s) {
  if (lds > 64 * 1024)
    BF_HIP(hipFuncSetAttribute((const void*)solve_round_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(solve_round_kernel, dim3((unsigned)grid), dim3(QR_THREADS), lds, s, works,
                     items, nitems);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs == hipStreamCaptureStatusNone)
    BF_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- misc ----
__global__ void c128_to_c64_kernel(const bf_c128* in, bf_c64* out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = bf_c64{(float)in[i].re, (float)in[i].im};
}
void launch_c128_to_c64(const bf_c128* in, bf_c64* out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(c128_to_c64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in,
                     out, n);
  BF_HIP(hipGetLastError());
}

__global__ void expand_segments_kernel(const bf_c64* X, int64_t ldx, int64_t rows, int64_t ncols,
                                       const int64_t* seg, int32_t /*nseg: grid y / ncols*/,
                                       bf_c64* out, int64_t ldo) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t col = blockIdx.y;           // 0 .. nseg*ncols-1
  if (r >= rows) return;
  int64_t g = col / ncols, c = col % ncols;
  bf_c64 v = {0.f, 0.f};
  if (r >= seg[g] && r < seg[g + 1]) v = X[c * ldx + r];
  out[col * ldo + r] = v;
}
// Y0(:, g s0 + c) = Yb(:, 2g w + off + c) + Yb(:, (2g+1) w + off + c): a
// level's products from the halves computed over its nodes' two children.
__global__ void sum_halves_kernel(const bf_c64* __restrict__ Yb, int64_t rows, int32_t w,
                                  int32_t off, int32_t s0, bf_c64* __restrict__ Y0) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t col = blockIdx.y;    // 0 .. nseg*s0-1
  if (r >= rows) return;
  const int64_t g = col / s0, c = col % s0;
  const bf_c64 a = Yb[((2 * g) * w + off + c) * rows + r];
  const bf_c64 b = Yb[((2 * g + 1) * w + off + c) * rows + r];
  Y0[col * rows + r] = bf_c64{a.re + b.re, a.im + b.im};
}
void launch_sum_halves(const bf_c64* Yb, int64_t rows, int64_t nseg, int32_t w, int32_t off,
                       int32_t s0, bf_c64* Y0, hipStream_t s) {
  if (rows <= 0 || nseg <= 0 || s0 <= 0) return;
  BF_CHECK(nseg * s0 <= 65535, BF_EINVAL, "too many summed columns");
  dim3 grid((unsigned)((rows + 255) / 256), (unsigned)(nseg * s0));
  hipLaunchKernelGGL(sum_halves_kernel, grid, dim3(256), 0, s, Yb, rows, w, off, s0, Y0);
  BF_HIP(hipGetLastError());
}

void launch_expand_segments(const bf_c64* X, int64_t ldx, int64_t rows, int64_t ncols,
                            const int64_t* seg_dev, int32_t nseg, bf_c64* out, int64_t ldo,
                            hipStream_t s) {
  if (rows <= 0 || ncols <= 0 || nseg <= 0) return;
  BF_CHECK((int64_t)nseg * ncols <= 65535, BF_EINVAL, "too many expanded columns");
  dim3 grid((unsigned)((rows + 255) / 256), (unsigned)(nseg * ncols));
  hipLaunchKernelGGL(expand_segments_kernel, grid, dim3(256), 0, s, X, ldx, rows, ncols, seg_dev,
                     nseg, out, ldo);
  BF_HIP(hipGetLastError());
}

// E(r, (g - g0) s + c) = C(r, c) for the rows r of segment g (rowseg[r] = g,
// g0 <= g < g0 + ng), zero elsewhere: the block-diagonal expansion of an
// intermediate whose rows each belong to one segment.  Element (r, c) of C is
// C[r crs + c cld], element (r, col) of E is E[r ers + col eld].  Consecutive
// threads take consecutive columns of one row (row-major E) or consecutive
// rows of one column (column-major E).
__global__ void expand_by_segment_kernel(const bf_c64* __restrict__ C, int64_t crs, int64_t cld,
                                         const int32_t* __restrict__ rowseg, int64_t rows,
                                         int32_t s, int32_t g0, int32_t ng, bf_c64* __restrict__ E,
                                         int64_t ers, int64_t eld) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t w = (int64_t)ng * s;
  if (idx >= rows * w) return;
  int64_t r, col;
  if (eld == 1) {
    r = idx / w;
    col = idx % w;
  } else {
    col = idx / rows;
    r = idx % rows;
  }
  const int64_t g = col / s, c = col % s;
  bf_c64 v = {0.f, 0.f};
  if (rowseg[r] == g0 + g) v = C[r * crs + c * cld];
  E[r * ers + col * eld] = v;
}
void launch_expand_by_segment(const bf_c64* C, int64_t crs, int64_t cld, const int32_t* rowseg,
                              int64_t rows, int32_t s, int32_t g0, int32_t ng, bf_c64* E,
                              int64_t ers, int64_t eld, hipStream_t st) {
  const int64_t tot = rows * (int64_t)ng * s;
  if (tot <= 0) return;
  hipLaunchKernelGGL(expand_by_segment_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                     st, C, crs, cld, rowseg, rows, s, g0, ng, E, ers, eld);
  BF_HIP(hipGetLastError());
}

}  // namespace bf
