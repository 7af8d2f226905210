// Apply plans of a hybrid butterfly: the L + 3 stages of eq.
// (hybrid_butterfly_mat) for Y = F X, and their conjugate-transposed stages in
// reverse order for Y = F^H X.
//
// Intermediates of a stage live in a "tall" buffer: the blocks (i, j) of one
// level stacked i-major (rows = ranks), all right-hand sides as columns.  Each
// output block of a stage is out = sum_t G_t in_t (at most two terms); G_t is
// a (sub-)block of one factor, packed at plan time into the orientation the
// stage multiplies by (e.g. W^H rows for the forward row side) and stored
// contiguously in stage order, so a stage streams its factor bytes once.
#include <algorithm>
#include <mutex>
#include <unordered_map>

#include "factors.h"

namespace bf {

namespace {

struct LevelIndex {   // row offsets of the blocks of one level in its tall buffer
  std::vector<int64_t> off;
  int64_t rows = 0;
};

LevelIndex index_level(const bf_factors* F, int l, bool col_side) {
  const int L = F->L;
  LevelIndex ix;
  const int64_t nT = int64_t(1) << l, nS = int64_t(1) << (L - l);
  ix.off.resize((size_t)(nT * nS));
  for (int64_t i = 0; i < nT; ++i)
    for (int64_t j = 0; j < nS; ++j) {
      ix.off[(size_t)((i << (L - l)) + j)] = ix.rows;
      ix.rows += col_side ? F->ku(l, i, j) : F->kv(l, i, j);
    }
  return ix;
}

// One term of an output block: rows [row0, ...) of factor block b, taken as
// is (conjT = 0, an M x K slice) or conjugate-transposed (conjT = 1, the
// K x M slice's adjoint), multiplying input rows [in_row, in_row + K).
struct TermSpec {
  const Block* b;
  int row0, M, K, conjT;
  int in_buf;
  int64_t in_row;
};

struct PlanBuilder {
  const bf_factors* F;
  std::vector<ApplyBlk> blks;
  int64_t nrows = 0;   // row records (expanded from the blocks on the device)
  std::vector<PackDesc> packs;
  std::vector<int32_t> pack_blk;   // block of each pack descriptor
  std::vector<Stage> stages;
  int64_t goff = 0;
  int cur_in = 0, cur_out = 1;
  Stage cur;

  std::vector<int64_t> node;   // input-side tree node of every block (Stage::level)

  void begin(int in, int out, int level = -1) {
    cur = Stage{};
    cur.level = level;
    cur.out_buf = out;
    cur.blk_off = (int64_t)blks.size();
    cur.row_off = nrows;
    cur_in = in;
    cur_out = out;
  }
  void end() { stages.push_back(cur); }
  TermSpec term(const Block& b, int row0, int M, int K, int conjT, int64_t in_row) {
    return TermSpec{&b, row0, M, K, conjT, cur_in, in_row};
  }
  // out rows [out_row, out_row + M) = sum of the terms; the terms' factor
  // slices are packed side by side into one row-major M x (K0 + K1) block
  void add(int64_t out_row, int M, const TermSpec* t, int nt, int64_t nd = 0) {
    if (M <= 0) return;
    node.push_back(nd);
    const int K0 = nt > 0 ? t[0].K : 0, K1 = nt > 1 ? t[1].K : 0;
    const int KK = K0 + K1;
    ApplyBlk bk{};
    bk.g_off = goff;
    bk.out_row = out_row;
    bk.M = M;
    bk.K0 = K0;
    bk.K1 = K1;
    bk.out_buf = (int8_t)cur_out;
    bk.in_buf0 = (int8_t)(nt > 0 ? t[0].in_buf : cur_in);
    bk.in_row0 = nt > 0 ? t[0].in_row : 0;
    bk.in_buf1 = (int8_t)(nt > 1 ? t[1].in_buf : bk.in_buf0);
    bk.in_row1 = nt > 1 ? t[1].in_row : bk.in_row0;
    int koff = 0;
    for (int q = 0; q < nt; ++q) {
      if (t[q].K > 0)
      {
        packs.push_back(PackDesc{t[q].b->p, goff + koff, t[q].b->rows, t[q].row0, M, t[q].K,
                                 t[q].conjT, KK, 1, 0});
        pack_blk.push_back((int32_t)blks.size());
      }
      koff += t[q].K;
    }
    goff += (int64_t)M * KK;
    bk.row_rec = nrows;
    nrows += M;
    blks.push_back(bk);
    cur.nrows += M;
    cur.nblk += 1;
    cur.maxMK = std::max(cur.maxMK, M * KK);
    cur.maxKK = std::max(cur.maxKK, KK);
    cur.maxM = std::max(cur.maxM, M);
    cur.macs += (double)M * KK;
  }
};

// A stage joins a fused launch while every group keeps at most
// kFusedMaxStageRows rows per stage (one pass of a 512-thread workgroup with
// two rows per thread, so each thread's rows of the next stage can be fetched
// ahead) and the launch keeps kFusedMinGroups workgroups.  Measured with one
// event pair around whole applies: with fewer groups (n = 16384, 64 groups)
// a workgroup's chain of dependent stages is slower than the stage kernels
// at 2 to 16 columns (80 vs 99 us at 8 columns), with 256 groups (n = 65536)
// faster at one column (57 vs 62 us).  Above 4 columns the stage-by-stage
// matrix-core apply is faster at every size measured (n = 65536, 16 columns:
// 117 vs 189 us), so only applies of up to 4 columns fuse.
constexpr int64_t kFusedMaxStageRows = kFusedLdsRows;
constexpr int64_t kFusedMinGroups = 256;
// Stages with more factor bytes than this stream at HBM rate on their own
// (each launch then fills the device); only smaller, latency-bound stages
// are fused.
constexpr double kFusedMaxStageBytes = 16.0 * (1 << 20);

struct UnionFind {
  std::vector<int32_t> p;
  explicit UnionFind(size_t n) : p(n) {
    for (size_t i = 0; i < n; ++i) p[i] = (int32_t)i;
  }
  int32_t find(int32_t x) {
    while (p[x] != x) x = p[x] = p[p[x]];
    return x;
  }
  bool unite(int32_t a, int32_t b) {
    a = find(a);
    b = find(b);
    if (a == b) return false;
    if (a < b) std::swap(a, b);
    p[a] = b;
    return true;
  }
};

// The fused schedule of a plan: consecutive stages are grouped into
// launches, each launch's blocks split into independent groups (one
// workgroup each), and the groups' blocks re-indexed as row records ordered
// by launch, group and stage.  The last stage of a launch (unless it is the
// plan's last) writes rows [base_t, base_t + rows_t) of one tall intermediate
// (buffer 1), which the next launch's first stage reads; inside a launch a
// group's stages hand their rows over in its workgroup's LDS.
struct FusedHost {
  std::vector<ApplyBlk> fb;      // blocks in fused order, fused buffers and rows
  std::vector<int32_t> off;      // per segment, group and stage: first row record
  int64_t rec = 0;
};

// Computes the schedule and lays the packed factor arena out in its order
// (group after group, stage after stage), so that a workgroup streams one
// contiguous range per stage; rewrites pb's block offsets and pack
// destinations accordingly (the arena's size is unchanged).
void fused_schedule(PlanBuilder& pb, ApplyPlan& plan, FusedHost& fh) {
  const auto& stg = pb.stages;
  const int ns = (int)stg.size();
  if (ns == 0) return;
  std::vector<int64_t> base(ns, 0);
  int64_t tot = 0;
  for (int t = 0; t + 1 < ns; ++t) {
    base[t] = tot;
    tot += stg[t].nrows;
  }
  const size_t nb = pb.blks.size();
  // producers: for each block of stage t > 0, the blocks of stage t - 1 whose
  // output rows its two input ranges read (stage blocks are sorted by row);
  // block b's are prod[poff[b] .. poff[b + 1])
  std::vector<int64_t> poff(nb + 1, 0);
  std::vector<int32_t> prod;
  prod.reserve(2 * nb);
  for (int t = 1; t < ns; ++t) {
    const int64_t p0 = stg[t - 1].blk_off, pn = stg[t - 1].nblk;
    std::vector<int64_t> starts((size_t)pn);
    for (int64_t k = 0; k < pn; ++k) starts[(size_t)k] = pb.blks[(size_t)(p0 + k)].out_row;
    for (int64_t b = stg[t].blk_off; b < stg[t].blk_off + stg[t].nblk; ++b) {
      const ApplyBlk& bk = pb.blks[(size_t)b];
      const int64_t rr[2][2] = {{bk.in_row0, bk.K0}, {bk.in_row1, bk.K1}};
      for (auto& r : rr) {
        if (r[1] <= 0) continue;
        auto it = std::upper_bound(starts.begin(), starts.end(), r[0]);
        int64_t k = (int64_t)(it - starts.begin()) - 1;
        for (; k >= 0 && k < pn && starts[(size_t)k] < r[0] + r[1]; ++k) {
          const ApplyBlk& pk = pb.blks[(size_t)(p0 + k)];
          if (pk.out_row + pk.M > r[0]) prod.push_back((int32_t)(p0 + k));
        }
      }
      poff[(size_t)b + 1] = (int64_t)prod.size();
    }
  }
  std::vector<ApplyBlk>& fb = fh.fb;
  std::vector<int32_t>& off = fh.off;
  fb.reserve(nb);
  int64_t rec = 0, gcur = 0;
  std::vector<int64_t> new_g(nb, 0), lds_row(nb, 0);
  UnionFind uf(nb);
  int a = 0;
  while (a < ns) {
    // grow the launch [a, e) while it keeps enough groups (or stays small)
    int64_t groups = stg[a].nblk;
    int e = a + 1;
    while (e < ns && 8.0 * stg[a].macs <= kFusedMaxStageBytes &&
           8.0 * stg[e].macs <= kFusedMaxStageBytes) {
      UnionFind trial = uf;
      int64_t g = groups + stg[e].nblk;
      for (int64_t b = stg[e].blk_off; b < stg[e].blk_off + stg[e].nblk; ++b)
        for (int64_t k = poff[(size_t)b]; k < poff[(size_t)b + 1]; ++k)
          if (trial.unite((int32_t)b, prod[(size_t)k])) --g;
      if (g < kFusedMinGroups) break;
      // rows per group and stage
      int64_t stage_rows_max = 0;
      for (int t = a; t <= e; ++t) {
        std::unordered_map<int32_t, int64_t> srows;
        for (int64_t b = stg[t].blk_off; b < stg[t].blk_off + stg[t].nblk; ++b)
          stage_rows_max = std::max(stage_rows_max,
                                    srows[trial.find((int32_t)b)] += pb.blks[(size_t)b].M);
      }
      if (stage_rows_max > kFusedMaxStageRows) break;
      uf = std::move(trial);
      groups = g;
      ++e;
    }
    // groups in order of their first block; records by group, then stage
    std::unordered_map<int32_t, int32_t> gid;
    std::vector<std::vector<std::vector<int32_t>>> members;
    for (int t = a; t < e; ++t)
      for (int64_t b = stg[t].blk_off; b < stg[t].blk_off + stg[t].nblk; ++b) {
        const int32_t r = uf.find((int32_t)b);
        auto it = gid.find(r);
        if (it == gid.end()) {
          it = gid.emplace(r, (int32_t)members.size()).first;
          members.emplace_back(e - a);
        }
        members[(size_t)it->second][(size_t)(t - a)].push_back((int32_t)b);
      }
    FusedSeg seg;
    seg.off_off = (int64_t)off.size();
    seg.nwg = (int32_t)members.size();
    seg.nstage = e - a;
    seg.first_stage = a;
    for (int t = a; t < e; ++t) seg.macs += stg[t].macs;
    for (auto& grp : members) {
      // Within the launch the group's stages pass their rows through LDS:
      // stage t's blocks (sorted by output row) get consecutive rows of LDS
      // half (t - a) & 1, and an input range of stage t + 1, whose producers
      // all lie in the group, maps to as many consecutive LDS rows.
      bool in_lds = e - a >= 2;
      for (int t = a; in_lds && t + 1 < e; ++t) {
        int64_t r = 0;
        for (int32_t b : grp[(size_t)(t - a)]) {
          lds_row[(size_t)b] = ((t - a) & 1) * kFusedLdsRows + r;
          r += pb.blks[(size_t)b].M;
        }
        in_lds = r <= kFusedLdsRows;
      }
      // LDS row of row x of stage t's output in the group, or -1
      auto lds_of = [&](int t, int64_t x) -> int64_t {
        const auto& pg = grp[(size_t)(t - a)];
        auto it = std::upper_bound(pg.begin(), pg.end(), x, [&](int64_t v, int32_t b) {
          return v < pb.blks[(size_t)b].out_row;
        });
        if (it == pg.begin()) return -1;
        const ApplyBlk& pk = pb.blks[(size_t)*(it - 1)];
        return x < pk.out_row + pk.M ? lds_row[(size_t)*(it - 1)] + (x - pk.out_row) : -1;
      };
      for (int t = a + 1; in_lds && t < e; ++t)
        for (int32_t b : grp[(size_t)(t - a)]) {
          const ApplyBlk& bk = pb.blks[(size_t)b];
          const int64_t rr[2][2] = {{bk.in_row0, bk.K0}, {bk.in_row1, bk.K1}};
          for (auto& r : rr) {
            if (r[1] <= 0) continue;
            const int64_t f = lds_of(t - 1, r[0]), l = lds_of(t - 1, r[0] + r[1] - 1);
            if (f < 0 || l != f + r[1] - 1) in_lds = false;
          }
        }
      for (int t = a; t < e; ++t) {
        off.push_back((int32_t)rec);
        int64_t rows_gs = 0;
        for (int32_t b : grp[(size_t)(t - a)]) rows_gs += pb.blks[(size_t)b].M;
        seg.max_rows = (int32_t)std::max<int64_t>(seg.max_rows, rows_gs);
        for (int32_t b : grp[(size_t)(t - a)]) {
          new_g[(size_t)b] = gcur;
          gcur += (int64_t)pb.blks[(size_t)b].M * (pb.blks[(size_t)b].K0 + pb.blks[(size_t)b].K1);
          ApplyBlk bk = pb.blks[(size_t)b];
          bk.g_off = new_g[(size_t)b];
          if (in_lds && t + 1 < e) {
            bk.out_buf = kFusedLdsBuf;
            bk.out_row = lds_row[(size_t)b];
          } else if (t + 1 < ns) {
            bk.out_buf = 1;
            bk.out_row += base[t];
          }
          if (in_lds && t > a) {
            bk.in_buf0 = kFusedLdsBuf;
            bk.in_buf1 = kFusedLdsBuf;
            bk.in_row0 = bk.K0 > 0 ? lds_of(t - 1, bk.in_row0) : 0;
            bk.in_row1 = bk.K1 > 0 ? lds_of(t - 1, bk.in_row1) : 0;
          } else if (t > 0) {
            bk.in_buf0 = 1;
            bk.in_buf1 = 1;
            bk.in_row0 += base[t - 1];
            bk.in_row1 += base[t - 1];
          }
          bk.row_rec = rec;
          rec += bk.M;
          fb.push_back(bk);
        }
      }
      off.push_back((int32_t)rec);
    }
    BF_CHECK(rec < INT32_MAX, BF_EINVAL, "fused apply: too many row records");
    plan.segs.push_back(seg);
    a = e;
  }
  if (plan.segs.size() == (size_t)ns) {   // nothing fused: the stage kernels serve better
    plan.segs.clear();
    fh = FusedHost{};
    return;
  }
  plan.fused_rows = std::max<int64_t>(tot, 1);
  fh.rec = rec;
  // the arena in fused order: every block's packed entries move as a whole
  for (size_t b = 0; b < nb; ++b) {
    const int64_t old = pb.blks[b].g_off;
    pb.blks[b].g_off = new_g[b];
    new_g[b] -= old;   // now the shift of block b
  }
  for (size_t k = 0; k < pb.packs.size(); ++k) pb.packs[k].dst_off += new_g[(size_t)pb.pack_blk[k]];
}

void build_fused(const FusedHost& fh, ApplyPlan& plan, Staging& st, hipStream_t s) {
  if (plan.segs.empty()) return;
  auto fbd = upload(fh.fb, s, st);
  plan.foff = upload(fh.off, s, st);
  plan.frows = DevBuf<ApplyRowRec>((size_t)std::max<int64_t>(fh.rec, 1), s);
  launch_expand_rows(fbd.p, (int32_t)fh.fb.size(), plan.frows.p, s);
  BF_HIP(hipStreamSynchronize(s));   // fbd is released at return
}

void finish(PlanBuilder& pb, ApplyPlan& plan, int64_t tmp_rows, hipStream_t s,
            int64_t rows_in, int64_t rows_out) {
  FusedHost fh;
  fused_schedule(pb, plan, fh);
  if (validating()) {
    const int64_t nr[4] = {rows_in, tmp_rows, tmp_rows, rows_out};
    for (auto& b : pb.blks) {
      BF_CHECK(b.out_row >= 0 && b.out_row + b.M <= nr[b.out_buf], BF_EINVAL,
               "bounds check failed: apply output rows");
      BF_CHECK(b.in_row0 >= 0 && b.in_row0 + b.K0 <= nr[b.in_buf0], BF_EINVAL,
               "bounds check failed: apply input rows");
      BF_CHECK(b.K1 == 0 || (b.in_row1 >= 0 && b.in_row1 + b.K1 <= nr[b.in_buf1]), BF_EINVAL,
               "bounds check failed: apply input rows");
      BF_CHECK(b.g_off + (int64_t)b.M * (b.K0 + b.K1) <= pb.goff, BF_EINVAL,
               "bounds check failed: apply factor block");
    }
    for (auto& p : pb.packs) {
      const int64_t r = p.conjT ? (int64_t)p.row0 + p.K : (int64_t)p.row0 + p.M;
      const int64_t c = p.conjT ? p.M : p.K;
      if (p.M > 0 && p.K > 0)
        check_extent(p.src, ((size_t)(c - 1) * p.src_ld + r) * sizeof(bf_c128), "pack source");
    }
  }
  Staging local;
  Staging& st = scope_staging(s) ? *scope_staging(s) : local;
  plan.G = DevBuf<bf_c64>((size_t)std::max<int64_t>(pb.goff, 1), s);
  plan.blks = upload(pb.blks, s, st);
  plan.rows = DevBuf<ApplyRowRec>((size_t)std::max<int64_t>(pb.nrows, 1), s);
  launch_expand_rows(plan.blks.p, (int32_t)pb.blks.size(), plan.rows.p, s);
  plan.stages = pb.stages;
  plan.tmp_rows = std::max<int64_t>(tmp_rows, 1);
  plan.out_row.resize(pb.blks.size());
  plan.out_m.resize(pb.blks.size());
  for (size_t b = 0; b < pb.blks.size(); ++b) {
    plan.out_row[b] = pb.blks[b].out_row;
    plan.out_m[b] = pb.blks[b].M;
  }
  plan.node = pb.node;
  for (size_t o = 0; o < pb.packs.size(); o += 60000) {
    size_t cnt = std::min<size_t>(60000, pb.packs.size() - o);
    std::vector<PackDesc> part(pb.packs.begin() + o, pb.packs.begin() + o + cnt);
    auto dd = upload(part, s, st);
    ProfScope ps(BF_KC_OTHER, s, 0.0, 0.0);
    launch_pack_c64(dd.p, (int32_t)cnt, plan.G.p, s);
  }
  build_fused(fh, plan, st, s);
  BF_HIP(hipStreamSynchronize(s));
  st.reset();
}

}  // namespace

void build_apply_plans(bf_factors* F, hipStream_t s) {
  const int L = F->L, lm = F->lm;
  const int64_t m = F->m, n = F->n;
  std::vector<LevelIndex> iv(lm + 1), iu(L + 1);
  int64_t tmp_rows = 0;
  for (int l = 0; l <= lm; ++l) { iv[l] = index_level(F, l, false); tmp_rows = std::max(tmp_rows, iv[l].rows); }
  for (int l = lm; l <= L; ++l) { iu[l] = index_level(F, l, true); tmp_rows = std::max(tmp_rows, iu[l].rows); }
  auto bidx = [&](int l, int64_t i, int64_t j) { return (size_t)((i << (L - l)) + j); };

  // ---------------- forward: V^0, W^1..W^lm, B, R^lm..R^{L-1}, U^L ----------
  {
    PlanBuilder pb{F};
    int a = 1, b = 2;
    pb.begin(0, a, L);
    for (int64_t j = 0; j < (int64_t(1) << L); ++j) {
      const Block& V = F->V[j];
      TermSpec t = pb.term(V, 0, V.cols, V.rows, 1, node_lo(n, L, j));
      pb.add(iv[0].off[j], V.cols, &t, 1, j);
    }
    pb.end();
    for (int l = 1; l <= lm; ++l) {
      pb.begin(a, b, L - l);
      for (int64_t i = 0; i < (int64_t(1) << l); ++i)
        for (int64_t j = 0; j < (int64_t(1) << (L - l)); ++j) {
          const Block& Wb = F->W[l][bidx(l, i, j)];
          const int ka = F->kv(l - 1, i >> 1, 2 * j), kb = F->kv(l - 1, i >> 1, 2 * j + 1);
          TermSpec t[2] = {pb.term(Wb, 0, Wb.cols, ka, 1, iv[l - 1].off[bidx(l - 1, i >> 1, 2 * j)]),
                            pb.term(Wb, ka, Wb.cols, kb, 1, iv[l - 1].off[bidx(l - 1, i >> 1, 2 * j + 1)])};
          pb.add(iv[l].off[bidx(l, i, j)], Wb.cols, t, 2, j);
        }
      pb.end();
      std::swap(a, b);
    }
    pb.begin(a, b, L - lm);
    for (int64_t i = 0; i < (int64_t(1) << lm); ++i)
      for (int64_t j = 0; j < (int64_t(1) << (L - lm)); ++j) {
        const Block& Bb = F->B[bidx(lm, i, j)];
        TermSpec t = pb.term(Bb, 0, Bb.rows, Bb.cols, 0, iv[lm].off[bidx(lm, i, j)]);
        pb.add(iu[lm].off[bidx(lm, i, j)], Bb.rows, &t, 1, j);
      }
    pb.end();
    std::swap(a, b);
    for (int l = lm; l < L; ++l) {
      pb.begin(a, b, L - l - 1);
      for (int64_t ic = 0; ic < (int64_t(1) << (l + 1)); ++ic)
        for (int64_t jc = 0; jc < (int64_t(1) << (L - l - 1)); ++jc) {
          const int64_t i = ic >> 1;
          const int Mo = F->ku(l + 1, ic, jc);
          TermSpec t[2];
          for (int q = 0; q < 2; ++q) {
            const int64_t j = 2 * jc + q;
            const Block& Rb = F->R[l - lm][bidx(l, i, j)];
            const int k1 = F->ku(l + 1, 2 * i, jc);
            t[q] = pb.term(Rb, (ic & 1) ? k1 : 0, Mo, Rb.cols, 0, iu[l].off[bidx(l, i, j)]);
          }
          pb.add(iu[l + 1].off[bidx(l + 1, ic, jc)], Mo, t, 2, jc);
        }
      pb.end();
      std::swap(a, b);
    }
    pb.begin(a, 3);
    for (int64_t i = 0; i < (int64_t(1) << L); ++i) {
      const Block& U = F->U[i];
      TermSpec t = pb.term(U, 0, U.rows, U.cols, 0, iu[L].off[i]);
      pb.add(node_lo(m, L, i), U.rows, &t, 1);
    }
    pb.end();
    finish(pb, F->fwd, tmp_rows, s, n, m);
  }

  // ---------------- adjoint: U^H, R^H (L-1..lm), B^H, W^H (lm..1), V ----------
  {
    PlanBuilder pb{F};
    int a = 1, b = 2;
    pb.begin(0, a, L);
    for (int64_t i = 0; i < (int64_t(1) << L); ++i) {
      const Block& U = F->U[i];
      TermSpec t = pb.term(U, 0, U.cols, U.rows, 1, node_lo(m, L, i));
      pb.add(iu[L].off[i], U.cols, &t, 1, i);
    }
    pb.end();
    for (int l = L - 1; l >= lm; --l) {
      pb.begin(a, b, l);
      for (int64_t i = 0; i < (int64_t(1) << l); ++i)
        for (int64_t j = 0; j < (int64_t(1) << (L - l)); ++j) {
          const Block& Rb = F->R[l - lm][bidx(l, i, j)];
          const int k1 = F->ku(l + 1, 2 * i, j >> 1), k2 = F->ku(l + 1, 2 * i + 1, j >> 1);
          TermSpec t[2] = {pb.term(Rb, 0, Rb.cols, k1, 1, iu[l + 1].off[bidx(l + 1, 2 * i, j >> 1)]),
                            pb.term(Rb, k1, Rb.cols, k2, 1, iu[l + 1].off[bidx(l + 1, 2 * i + 1, j >> 1)])};
          pb.add(iu[l].off[bidx(l, i, j)], Rb.cols, t, 2, i);
        }
      pb.end();
      std::swap(a, b);
    }
    pb.begin(a, b, lm);
    for (int64_t i = 0; i < (int64_t(1) << lm); ++i)
      for (int64_t j = 0; j < (int64_t(1) << (L - lm)); ++j) {
        const Block& Bb = F->B[bidx(lm, i, j)];
        TermSpec t = pb.term(Bb, 0, Bb.cols, Bb.rows, 1, iu[lm].off[bidx(lm, i, j)]);
        pb.add(iv[lm].off[bidx(lm, i, j)], Bb.cols, &t, 1, i);
      }
    pb.end();
    std::swap(a, b);
    for (int l = lm; l >= 1; --l) {
      pb.begin(a, b, l - 1);
      for (int64_t ip = 0; ip < (int64_t(1) << (l - 1)); ++ip)
        for (int64_t jp = 0; jp < (int64_t(1) << (L - l + 1)); ++jp) {
          const int64_t j = jp >> 1;
          const int Mo = F->kv(l - 1, ip, jp);
          TermSpec t[2];
          for (int q = 0; q < 2; ++q) {
            const int64_t i = 2 * ip + q;
            const Block& Wb = F->W[l][bidx(l, i, j)];
            const int ka = F->kv(l - 1, ip, 2 * j);
            t[q] = pb.term(Wb, (jp & 1) ? ka : 0, Mo, Wb.cols, 0, iv[l].off[bidx(l, i, j)]);
          }
          pb.add(iv[l - 1].off[bidx(l - 1, ip, jp)], Mo, t, 2, ip);
        }
      pb.end();
      std::swap(a, b);
    }
    pb.begin(a, 3);
    for (int64_t j = 0; j < (int64_t(1) << L); ++j) {
      const Block& V = F->V[j];
      TermSpec t = pb.term(V, 0, V.rows, V.cols, 0, iv[0].off[j]);
      pb.add(node_lo(n, L, j), V.rows, &t, 1);
    }
    pb.end();
    finish(pb, F->adj, tmp_rows, s, m, n);
  }
}

// Layout of an intermediate of an apply with ncols columns: row-major above
// the few-column path (see launch_apply_stage), else column-major.
static void tmp_layout(const ApplyPlan& P, int64_t ncols, int64_t* ld, int64_t* rs) {
  const bool rowmajor = ncols > kApplyFewCols;
  *ld = rowmajor ? 1 : P.tmp_rows;
  *rs = rowmajor ? ncols : 1;
}

// Stage launches [k0, k1) of one apply on stream s (buffers: X, two
// intermediates, Y; every intermediate in tmp_layout for ncols).
static void run_stage_range(const bf_factors* F, int trans, size_t k0, size_t k1,
                            const bf_c64* const bufs[4], int64_t ldx, int64_t ldy, int64_t ncols,
                            hipStream_t s, bool prof) {
  const ApplyPlan& P = trans ? F->adj : F->fwd;
  int64_t tld, trs;
  tmp_layout(P, ncols, &tld, &trs);
  const int64_t lds[4] = {ldx, tld, tld, ldy};
  const int64_t rss[4] = {1, trs, trs, 1};
  const int64_t rin = trans ? F->m : F->n, rout = trans ? F->n : F->m;
  for (size_t k = k0; k < k1; ++k) {
    const Stage& st = P.stages[k];
    // algorithmic bytes: this stage's factor entries once, plus the caller's
    // input (first stage) and output (last stage); intermediates excluded
    double by = 8.0 * st.macs;
    if (k == 0) by += 8.0 * (double)rin * ncols;
    if (k + 1 == P.stages.size()) by += 8.0 * (double)rout * ncols;
    auto launch = [&] {
      launch_apply_stage(P.blks.p + st.blk_off, st.nblk, P.rows.p + st.row_off, st.nrows,
                         st.maxMK, st.maxKK, st.maxM, P.G.p, bufs, lds, rss, ncols,
                         F->apply_prec, s, prof);
    };
    if (prof) {
      ProfScope ps(BF_KC_APPLY, s, 8.0 * st.macs * ncols, by);
      launch();
    } else {
      launch();
    }
  }
}

// The L+3 stage launches of one apply on stream s (buffers: X, two
// intermediates, Y).
static void run_apply_stages(const bf_factors* F, int trans, const bf_c64* X, int64_t ldx,
                      int64_t ncols, bf_c64* Y, int64_t ldy, bf_c64* t1, bf_c64* t2,
                      hipStream_t s, bool prof) {
  const ApplyPlan& P = trans ? F->adj : F->fwd;
  const bf_c64* bufs[4] = {X, t1, t2, Y};
  run_stage_range(F, trans, 0, P.stages.size(), bufs, ldx, ldy, ncols, s, prof);
}

// The fused launches of one apply (ncols <= kApplyFusedCols): intermediates
// in one column-major tall buffer T of plan.fused_rows rows.
static void run_fused(const bf_factors* F, int trans, const bf_c64* X, int64_t ldx,
                      int64_t ncols, bf_c64* Y, int64_t ldy, bf_c64* T, hipStream_t s,
                      bool prof) {
  const ApplyPlan& P = trans ? F->adj : F->fwd;
  const bf_c64* bufs[4] = {X, T, T, Y};
  const int64_t lds[4] = {ldx, P.fused_rows, P.fused_rows, ldy};
  const int64_t rin = trans ? F->m : F->n, rout = trans ? F->n : F->m;
  for (size_t k = 0; k < P.segs.size(); ++k) {
    const FusedSeg& sg = P.segs[k];
    double by = 8.0 * sg.macs;
    if (k == 0) by += 8.0 * (double)rin * ncols;
    if (k + 1 == P.segs.size()) by += 8.0 * (double)rout * ncols;
    auto launch = [&] {
      launch_apply_fused(P.frows.p, P.foff.p + sg.off_off, sg.nwg, sg.nstage, sg.max_rows,
                         P.G.p, bufs, lds, ncols, F->apply_prec, s);
    };
    if (prof) {
      ProfScope ps(BF_KC_APPLY, s, 8.0 * sg.macs * ncols, by);
      launch();
    } else {
      launch();
    }
  }
}

static bool fused_ok(const bf_factors* F, int trans, int64_t ncols) {
  const ApplyPlan& P = trans ? F->adj : F->fwd;
  return F->apply_fuse && ncols > 0 && ncols <= kApplyFusedCols && !P.segs.empty();
}

size_t apply_scratch_bytes(const bf_factors* F, int trans, int64_t ncols, bool staged) {
  const ApplyPlan& P = trans ? F->adj : F->fwd;
  if (!staged && fused_ok(F, trans, ncols))
    return (size_t)P.fused_rows * (size_t)ncols * sizeof(bf_c64);
  const size_t one = (size_t)P.tmp_rows * (size_t)std::max<int64_t>(ncols, 0) * sizeof(bf_c64);
  return ((one + 255) & ~size_t(255)) + one;
}

void run_apply(const bf_factors* F, int trans, const bf_c64* X, int64_t ldx, int64_t ncols,
               bf_c64* Y, int64_t ldy, void* scratch, size_t scratch_bytes, hipStream_t s,
               bool prof) {
  if (ncols <= 0) return;
  char* base = static_cast<char*>(scratch);
  const ApplyPlan& P = trans ? F->adj : F->fwd;
  const size_t one = (size_t)P.tmp_rows * (size_t)ncols * sizeof(bf_c64);
  const bool fused = fused_ok(F, trans, ncols) &&
                     scratch_bytes >= apply_scratch_bytes(F, trans, ncols);
  const bool staged = scratch_bytes >= apply_scratch_bytes(F, trans, ncols, true);
  BF_CHECK(fused || staged, BF_EINVAL, "apply: scratch too small for the intermediates");
  auto run = [&](int64_t f) {
    if (f)
      run_fused(F, trans, X, ldx, ncols, Y, ldy, reinterpret_cast<bf_c64*>(base), s, prof);
    else
      run_apply_stages(F, trans, X, ldx, ncols, Y, ldy, reinterpret_cast<bf_c64*>(base),
                       reinterpret_cast<bf_c64*>(base + ((one + 255) & ~size_t(255))), s, prof);
  };
  if (fused && staged && ncols <= kApplyFewCols) {
    // up to 4 columns both run the same row kernel (same bits): the autotuner
    // picks per shape class; fused is the rule without it
    const TuneKey key{kTuneApplyFused, trans, ncols, pow2_ceil(F->m), pow2_ceil(F->n),
                      F->L * 64 + F->apply_prec};
    tune_choose(key, {1, 0}, 1, s, run, prof);
    return;
  }
  run(fused ? 1 : 0);
}

// ---- applies as captured HIP graphs (bf_set_apply_graph_cols) --------------
// One graph per (direction, column count, precision, stream): the stage
// launches read a private input buffer and write a private output buffer, and
// a call copies X in, launches the graph and copies Y out.  The buffers are
// plain device allocations made before capture (nothing is allocated or
// cleared inside the graph).
struct ApplyGraph {
  int trans = 0, prec = 0;
  int64_t ncols = 0;
  hipStream_t s = nullptr;
  bf_c64 *Xs = nullptr, *Ys = nullptr;
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  hipGraphExec_t exec = nullptr;
};
struct ApplyGraphCache {
  std::mutex mu;
  std::vector<ApplyGraph> g;
  hipStream_t cap = nullptr;    // private capture stream (the default stream cannot capture)
};
constexpr size_t kMaxApplyGraphs = 16;

static void release_graph(ApplyGraph& a) {
  if (a.exec) (void)hipGraphExecDestroy(a.exec);
  for (void* p : {(void*)a.Xs, (void*)a.Ys, a.tmp})
    if (p) (void)hipFree(p);
  a = ApplyGraph{};
}

ApplyGraphCache* new_apply_graph_cache() { return new ApplyGraphCache(); }

int apply_graph_count(const bf_factors* F) {
  if (!F->graphs) return 0;
  std::lock_guard<std::mutex> lk(F->graphs->mu);
  return (int)F->graphs->g.size();
}

void free_apply_graphs(ApplyGraphCache* c) {
  if (!c) return;
  for (auto& a : c->g) release_graph(a);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  delete c;
}

// Capture the graph of one key on the cache's own stream (a graph can be
// launched on any stream); false (nothing kept) if capture fails.
static bool capture_graph(const bf_factors* F, ApplyGraphCache* c, ApplyGraph& a) {
  const ApplyPlan& P = a.trans ? F->adj : F->fwd;
  const int64_t rin = a.trans ? F->m : F->n, rout = a.trans ? F->n : F->m;
  a.tmp_bytes = std::max<size_t>(apply_scratch_bytes(F, a.trans, a.ncols), 256);
  if (hipMalloc((void**)&a.Xs, (size_t)(rin * a.ncols) * sizeof(bf_c64)) != hipSuccess ||
      hipMalloc((void**)&a.Ys, (size_t)(rout * a.ncols) * sizeof(bf_c64)) != hipSuccess ||
      hipMalloc(&a.tmp, a.tmp_bytes) != hipSuccess) {
    release_graph(a);
    return false;
  }
  if (!c->cap && hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
    c->cap = nullptr;
    (void)hipGetLastError();
    release_graph(a);
    return false;
  }
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    release_graph(a);
    return false;
  }
  bool ok = true;
  try {
    run_apply(F, a.trans, a.Xs, rin, a.ncols, a.Ys, rout, a.tmp, a.tmp_bytes, c->cap, true);
  } catch (...) {
    ok = false;
  }
  if (hipStreamEndCapture(c->cap, &g) != hipSuccess || !g) ok = false;
  if (ok && hipGraphInstantiate(&a.exec, g, nullptr, nullptr, 0) != hipSuccess) ok = false;
  if (g) (void)hipGraphDestroy(g);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(c->cap, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
    hipGraph_t dead = nullptr;    // never leave the stream capturing
    (void)hipStreamEndCapture(c->cap, &dead);
    if (dead) (void)hipGraphDestroy(dead);
    ok = false;
  }
  (void)hipGetLastError();
  if (!ok) release_graph(a);
  return ok;
}

// Runs the apply through a cached graph; false if none could be made (the
// caller then launches the stages directly).
static bool apply_graph(const bf_factors* F, int trans, const bf_c64* X, int64_t ldx,
                        int64_t ncols, bf_c64* Y, int64_t ldy, hipStream_t s) {
  ApplyGraphCache* c = F->graphs;
  if (!c) return false;
  hipGraphExec_t exec = nullptr;
  bf_c64 *Xs = nullptr, *Ys = nullptr;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    for (auto& a : c->g)
      if (a.trans == trans && a.ncols == ncols && a.prec == F->apply_prec && a.s == s) {
        exec = a.exec;
        Xs = a.Xs;
        Ys = a.Ys;
      }
    if (!exec) {
      if (c->g.size() >= kMaxApplyGraphs) return false;
      ApplyGraph a;
      a.trans = trans;
      a.ncols = ncols;
      a.prec = F->apply_prec;
      a.s = s;
      if (!capture_graph(F, c, a)) return false;
      c->g.push_back(a);
      exec = a.exec;
      Xs = a.Xs;
      Ys = a.Ys;
    }
  }
  const int64_t rin = trans ? F->m : F->n, rout = trans ? F->n : F->m;
  BF_HIP(hipMemcpy2DAsync(Xs, rin * sizeof(bf_c64), X, ldx * sizeof(bf_c64), rin * sizeof(bf_c64),
                          ncols, hipMemcpyDeviceToDevice, s));
  BF_HIP(hipGraphLaunch(exec, s));
  BF_HIP(hipMemcpy2DAsync(Y, ldy * sizeof(bf_c64), Ys, rout * sizeof(bf_c64),
                          rout * sizeof(bf_c64), ncols, hipMemcpyDeviceToDevice, s));
  return true;
}

bool apply_structured(const bf_factors* F, int trans, const bf_c64* X, int64_t ldx,
                      int64_t ncols, bf_c64* Y, int64_t ldy, const int64_t* seg, int32_t nseg,
                      int64_t max_cols, hipStream_t s) {
  const ApplyPlan& P = trans ? F->adj : F->fwd;
  const int64_t rin = trans ? F->m : F->n;
  const size_t nst = P.stages.size();
  if (ncols <= 0 || nseg < 2 || nst < 2) return false;
  // the level tl whose consecutive nodes i0, i0 + 1, ... the segments are
  int tl = -1;
  int64_t i0 = 0;
  for (int l = 1; l <= F->L && tl < 0; ++l) {
    // node_lo(rin, l, i) = floor(i rin / 2^l): seg[0]'s node is one of two
    const int64_t q = (seg[0] << l) / rin;
    for (int64_t first = q; first <= q + 1 && tl < 0; ++first) {
      bool ok = first >= 0 && first + nseg <= (int64_t(1) << l);
      for (int32_t g = 0; ok && g <= nseg; ++g) ok = seg[g] == node_lo(rin, l, first + g);
      if (ok) {
        tl = l;
        i0 = first;
      }
    }
  }
  if (tl < 0) return false;
  // stages [0, ks) keep every segment apart
  size_t ks = 0;
  while (ks < nst && P.stages[ks].level >= tl) ++ks;
  if (ks == 0 || ks == nst) return false;
  // Windowed stages [ks, kw) (down to level tl - c): every row keeps just the
  // columns of the segments below its node, 2^(tl - level) ncols of them, and a
  // merging stage puts its two children's windows side by side.  Taken when
  // the segments are a whole level (so that windows are whole subtrees), on
  // the matrix-core path with blocks of at most 64 rows, and with c such that
  // a window of 2^c ncols columns over every intermediate row fits the budget.
  int c = 0;
  size_t kw = ks;
  if (i0 == 0 && nseg == (int64_t(1) << tl) && F->apply_prec == BF_PREC_BF16X3 &&
      ncols > kApplyFewCols) {
    while (c < tl && (ncols << (c + 1)) <= max_cols) ++c;
    while (kw + 1 < nst && P.stages[kw].level >= tl - c &&
           (P.stages[kw].level == P.stages[kw - 1].level || P.stages[kw].maxM <= 64))
      ++kw;
    // the windows end at the last stage taken
    c = kw > ks ? tl - P.stages[kw - 1].level : 0;
    if (c <= 0) {
      c = 0;
      kw = ks;
    }
  }
  Staging local;
  Staging& st = scope_staging(s) ? *scope_staging(s) : local;
  // stages [0, ks) on X itself
  const size_t one = (size_t)P.tmp_rows * (size_t)ncols;
  DevBuf<bf_c64> c1(one, s), c2(one, s);
  {
    const bf_c64* bufs[4] = {X, c1.p, c2.p, nullptr};
    run_stage_range(F, trans, 0, ks, bufs, ldx, ldy, ncols, s, true);
  }
  const bf_c64* C = P.stages[ks - 1].out_buf == 1 ? c1.p : c2.p;
  int64_t cw = ncols;   // columns of C's rows
  DevBuf<bf_c64> w1, w2;
  if (kw > ks) {
    const size_t wsz = (size_t)P.tmp_rows * (size_t)(ncols << c);
    w1 = DevBuf<bf_c64>(wsz, s);
    w2 = DevBuf<bf_c64>(wsz, s);
    bf_c64* nxt = w1.p;
    for (size_t k = ks; k < kw; ++k) {
      const Stage& sk = P.stages[k];
      const bool merge = sk.level < P.stages[k - 1].level;
      const int64_t wo = merge ? 2 * cw : cw;
      const int in_idx = P.stages[k - 1].out_buf, out_idx = sk.out_buf;
      const bf_c64* bufs[4] = {X, nullptr, nullptr, nullptr};
      bufs[in_idx] = C;
      bufs[out_idx] = nxt;
      const int64_t lds[4] = {ldx, 1, 1, ldy};
      int64_t rss[4] = {1, 1, 1, 1};
      rss[in_idx] = cw;
      rss[out_idx] = wo;
      ProfScope ps(BF_KC_APPLY, s, 8.0 * sk.macs * (double)cw, 8.0 * sk.macs);
      if (merge)
        launch_apply_window_stage(P.blks.p + sk.blk_off, sk.nblk, sk.maxM, P.G.p, bufs, lds, rss,
                                  wo, cw, s);
      else
        launch_apply_stage(P.blks.p + sk.blk_off, sk.nblk, P.rows.p + sk.row_off, sk.nrows,
                           sk.maxMK, sk.maxKK, sk.maxM, P.G.p, bufs, lds, rss, wo,
                           F->apply_prec, s, true);
      C = nxt;
      nxt = nxt == w1.p ? w2.p : w1.p;
      cw = wo;
    }
  }
  // the rows written by stage kw - 1 each belong to one group of 2^c
  // segments: the block-diagonal expansion of those groups for the rest
  const int tg = tl - c;
  const int32_t ngroups = nseg >> c;
  const Stage& last = P.stages[kw - 1];
  std::vector<int32_t> rowseg((size_t)P.tmp_rows, -1);
  for (int64_t b = last.blk_off; b < last.blk_off + last.nblk; ++b) {
    const int64_t g = (P.node[(size_t)b] >> (last.level - tg)) - (i0 >> c);
    if (g < 0 || g >= ngroups) continue;
    for (int64_t r = P.out_row[(size_t)b]; r < P.out_row[(size_t)b] + P.out_m[(size_t)b]; ++r)
      rowseg[(size_t)r] = (int32_t)g;
  }
  auto rs_dev = upload(rowseg, s, st);
  int64_t cld, crs;
  tmp_layout(P, cw, &cld, &crs);
  const int32_t per = (int32_t)std::max<int64_t>(1, std::min<int64_t>(ngroups, max_cols / cw));
  const int64_t wcols = (int64_t)per * cw;
  DevBuf<bf_c64> e1((size_t)P.tmp_rows * (size_t)wcols, s), e2((size_t)P.tmp_rows * (size_t)wcols, s);
  for (int32_t g0 = 0; g0 < ngroups; g0 += per) {
    const int32_t ng = std::min(per, ngroups - g0);
    const int64_t ec = (int64_t)ng * cw;
    int64_t eld, ers;
    tmp_layout(P, ec, &eld, &ers);
    launch_expand_by_segment(C, crs, cld, rs_dev.p, P.tmp_rows, (int32_t)cw, g0, ng, e1.p, ers,
                             eld, s);
    const bf_c64* bufs[4] = {X, last.out_buf == 1 ? e1.p : e2.p, last.out_buf == 1 ? e2.p : e1.p,
                             Y + (int64_t)g0 * cw * ldy};
    run_stage_range(F, trans, kw, nst, bufs, ldx, ldy, ec, s, true);
  }
  return true;
}

void apply_factors(const bf_factors* F, int trans, const bf_c64* X, int64_t ldx, int64_t ncols,
                   bf_c64* Y, int64_t ldy, hipStream_t s) {
  if (ncols <= 0) return;
  if (F->graph_cols > 0 && ncols <= F->graph_cols && apply_graph(F, trans, X, ldx, ncols, Y, ldy, s))
    return;
  const size_t need = apply_scratch_bytes(F, trans, ncols);
  DevBuf<char> tmp(need, s);
  run_apply(F, trans, X, ldx, ncols, Y, ldy, tmp.p, need, s, true);
}

}  // namespace bf

bf_factors::~bf_factors() { bf::free_apply_graphs(graphs); }
