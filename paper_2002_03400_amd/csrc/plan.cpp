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

struct PlanBuilder {
  const bf_factors* F;
  std::vector<ApplyDesc> descs;
  std::vector<PackDesc> packs;
  std::vector<Stage> stages;
  std::vector<int> in_buf, out_buf;
  int64_t goff = 0;
  int cur_in = 0, cur_out = 1;
  Stage cur;

  void begin(int in, int out) {
    cur = Stage{(int64_t)descs.size(), 0, 0};
    cur_in = in;
    cur_out = out;
  }
  void end() {
    stages.push_back(cur);
    in_buf.push_back(cur_in);
    out_buf.push_back(cur_out);
  }
  // term with G = conjT ? (src rows [row0, row0+K))^H : src rows [row0, row0+M)
  ApplyTerm term(const Block& b, int row0, int M, int K, int conjT, int64_t in_row) {
    PackDesc p{b.p, goff, b.rows, row0, M, K, conjT, 0};
    packs.push_back(p);
    ApplyTerm t{goff, in_row, K, cur_in};
    goff += (int64_t)M * K;
    return t;
  }
  void add(int64_t out_row, int M, const ApplyTerm* t, int nt) {
    if (M <= 0) return;
    ApplyDesc d{};
    d.out_row = out_row;
    d.M = M;
    d.out_buf = cur_out;
    d.nterm = 0;
    for (int q = 0; q < nt; ++q)
      if (t[q].K > 0) d.t[d.nterm++] = t[q];
    for (int q = 0; q < d.nterm; ++q) cur.macs += (double)M * d.t[q].K;
    descs.push_back(d);
    cur.count++;
    cur.maxM = std::max(cur.maxM, M);
  }
};

void finish(PlanBuilder& pb, ApplyPlan& plan, int64_t tmp_rows, hipStream_t s,
            int64_t rows_in, int64_t rows_out) {
  if (validating()) {
    const int64_t rows[4] = {rows_in, tmp_rows, tmp_rows, rows_out};
    for (auto& d : pb.descs) {
      BF_CHECK(d.out_row >= 0 && d.out_row + d.M <= rows[d.out_buf], BF_EINVAL,
               "bounds check failed: apply output rows");
      for (int t = 0; t < d.nterm; ++t) {
        BF_CHECK(d.t[t].in_row >= 0 && d.t[t].in_row + d.t[t].K <= rows[d.t[t].in_buf], BF_EINVAL,
                 "bounds check failed: apply input rows");
        BF_CHECK(d.t[t].g_off + (int64_t)d.M * d.t[t].K <= pb.goff, BF_EINVAL,
                 "bounds check failed: apply factor block");
      }
    }
    for (auto& p : pb.packs) {
      const int64_t r = p.conjT ? (int64_t)p.row0 + p.K : (int64_t)p.row0 + p.M;
      const int64_t c = p.conjT ? p.M : p.K;
      if (p.M > 0 && p.K > 0) check_extent(p.src, ((size_t)(c - 1) * p.src_ld + r) * sizeof(bf_c128), "pack source");
    }
  }
  Staging st;
  plan.G = DevBuf<bf_c64>((size_t)std::max<int64_t>(pb.goff, 1), s);
  plan.desc = upload(pb.descs, s, st);
  plan.stages = pb.stages;
  plan.in_buf = pb.in_buf;
  plan.out_buf = pb.out_buf;
  plan.tmp_rows = std::max<int64_t>(tmp_rows, 1);
  for (size_t o = 0; o < pb.packs.size(); o += 60000) {
    size_t cnt = std::min<size_t>(60000, pb.packs.size() - o);
    std::vector<PackDesc> part(pb.packs.begin() + o, pb.packs.begin() + o + cnt);
    auto dd = upload(part, s, st);
    ProfScope ps(BF_KC_OTHER, s, 0.0, 0.0);
    launch_pack_c64(dd.p, (int32_t)cnt, plan.G.p, s);
  }
  BF_HIP(hipStreamSynchronize(s));
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
    pb.begin(0, a);
    for (int64_t j = 0; j < (int64_t(1) << L); ++j) {
      const Block& V = F->V[j];
      ApplyTerm t = pb.term(V, 0, V.cols, V.rows, 1, node_lo(n, L, j));
      pb.add(iv[0].off[j], V.cols, &t, 1);
    }
    pb.end();
    for (int l = 1; l <= lm; ++l) {
      pb.begin(a, b);
      for (int64_t i = 0; i < (int64_t(1) << l); ++i)
        for (int64_t j = 0; j < (int64_t(1) << (L - l)); ++j) {
          const Block& Wb = F->W[l][bidx(l, i, j)];
          const int ka = F->kv(l - 1, i >> 1, 2 * j), kb = F->kv(l - 1, i >> 1, 2 * j + 1);
          ApplyTerm t[2] = {pb.term(Wb, 0, Wb.cols, ka, 1, iv[l - 1].off[bidx(l - 1, i >> 1, 2 * j)]),
                            pb.term(Wb, ka, Wb.cols, kb, 1, iv[l - 1].off[bidx(l - 1, i >> 1, 2 * j + 1)])};
          pb.add(iv[l].off[bidx(l, i, j)], Wb.cols, t, 2);
        }
      pb.end();
      std::swap(a, b);
    }
    pb.begin(a, b);
    for (int64_t i = 0; i < (int64_t(1) << lm); ++i)
      for (int64_t j = 0; j < (int64_t(1) << (L - lm)); ++j) {
        const Block& Bb = F->B[bidx(lm, i, j)];
        ApplyTerm t = pb.term(Bb, 0, Bb.rows, Bb.cols, 0, iv[lm].off[bidx(lm, i, j)]);
        pb.add(iu[lm].off[bidx(lm, i, j)], Bb.rows, &t, 1);
      }
    pb.end();
    std::swap(a, b);
    for (int l = lm; l < L; ++l) {
      pb.begin(a, b);
      for (int64_t ic = 0; ic < (int64_t(1) << (l + 1)); ++ic)
        for (int64_t jc = 0; jc < (int64_t(1) << (L - l - 1)); ++jc) {
          const int64_t i = ic >> 1;
          const int Mo = F->ku(l + 1, ic, jc);
          ApplyTerm t[2];
          for (int q = 0; q < 2; ++q) {
            const int64_t j = 2 * jc + q;
            const Block& Rb = F->R[l - lm][bidx(l, i, j)];
            const int k1 = F->ku(l + 1, 2 * i, jc);
            t[q] = pb.term(Rb, (ic & 1) ? k1 : 0, Mo, Rb.cols, 0, iu[l].off[bidx(l, i, j)]);
          }
          pb.add(iu[l + 1].off[bidx(l + 1, ic, jc)], Mo, t, 2);
        }
      pb.end();
      std::swap(a, b);
    }
    pb.begin(a, 3);
    for (int64_t i = 0; i < (int64_t(1) << L); ++i) {
      const Block& U = F->U[i];
      ApplyTerm t = pb.term(U, 0, U.rows, U.cols, 0, iu[L].off[i]);
      pb.add(node_lo(m, L, i), U.rows, &t, 1);
    }
    pb.end();
    finish(pb, F->fwd, tmp_rows, s, n, m);
  }

  // ---------------- adjoint: U^H, R^H (L-1..lm), B^H, W^H (lm..1), V ----------
  {
    PlanBuilder pb{F};
    int a = 1, b = 2;
    pb.begin(0, a);
    for (int64_t i = 0; i < (int64_t(1) << L); ++i) {
      const Block& U = F->U[i];
      ApplyTerm t = pb.term(U, 0, U.cols, U.rows, 1, node_lo(m, L, i));
      pb.add(iu[L].off[i], U.cols, &t, 1);
    }
    pb.end();
    for (int l = L - 1; l >= lm; --l) {
      pb.begin(a, b);
      for (int64_t i = 0; i < (int64_t(1) << l); ++i)
        for (int64_t j = 0; j < (int64_t(1) << (L - l)); ++j) {
          const Block& Rb = F->R[l - lm][bidx(l, i, j)];
          const int k1 = F->ku(l + 1, 2 * i, j >> 1), k2 = F->ku(l + 1, 2 * i + 1, j >> 1);
          ApplyTerm t[2] = {pb.term(Rb, 0, Rb.cols, k1, 1, iu[l + 1].off[bidx(l + 1, 2 * i, j >> 1)]),
                            pb.term(Rb, k1, Rb.cols, k2, 1, iu[l + 1].off[bidx(l + 1, 2 * i + 1, j >> 1)])};
          pb.add(iu[l].off[bidx(l, i, j)], Rb.cols, t, 2);
        }
      pb.end();
      std::swap(a, b);
    }
    pb.begin(a, b);
    for (int64_t i = 0; i < (int64_t(1) << lm); ++i)
      for (int64_t j = 0; j < (int64_t(1) << (L - lm)); ++j) {
        const Block& Bb = F->B[bidx(lm, i, j)];
        ApplyTerm t = pb.term(Bb, 0, Bb.cols, Bb.rows, 1, iu[lm].off[bidx(lm, i, j)]);
        pb.add(iv[lm].off[bidx(lm, i, j)], Bb.cols, &t, 1);
      }
    pb.end();
    std::swap(a, b);
    for (int l = lm; l >= 1; --l) {
      pb.begin(a, b);
      for (int64_t ip = 0; ip < (int64_t(1) << (l - 1)); ++ip)
        for (int64_t jp = 0; jp < (int64_t(1) << (L - l + 1)); ++jp) {
          const int64_t j = jp >> 1;
          const int Mo = F->kv(l - 1, ip, jp);
          ApplyTerm t[2];
          for (int q = 0; q < 2; ++q) {
            const int64_t i = 2 * ip + q;
            const Block& Wb = F->W[l][bidx(l, i, j)];
            const int ka = F->kv(l - 1, ip, 2 * j);
            t[q] = pb.term(Wb, (jp & 1) ? ka : 0, Mo, Wb.cols, 0, iv[l].off[bidx(l, i, j)]);
          }
          pb.add(iv[l - 1].off[bidx(l - 1, ip, jp)], Mo, t, 2);
        }
      pb.end();
      std::swap(a, b);
    }
    pb.begin(a, 3);
    for (int64_t j = 0; j < (int64_t(1) << L); ++j) {
      const Block& V = F->V[j];
      ApplyTerm t = pb.term(V, 0, V.rows, V.cols, 0, iv[0].off[j]);
      pb.add(node_lo(n, L, j), V.rows, &t, 1);
    }
    pb.end();
    finish(pb, F->adj, tmp_rows, s, m, n);
  }
}

void apply_factors(const bf_factors* F, int trans, const bf_c64* X, int64_t ldx, int64_t ncols,
                   bf_c64* Y, int64_t ldy, hipStream_t s) {
  const ApplyPlan& P = trans ? F->adj : F->fwd;
  if (ncols <= 0) return;
  DevBuf<bf_c64> t1((size_t)P.tmp_rows * ncols, s), t2((size_t)P.tmp_rows * ncols, s);
  const bf_c64* bufs[4] = {X, t1.p, t2.p, Y};
  const int64_t lds[4] = {ldx, P.tmp_rows, P.tmp_rows, ldy};
  const int64_t rin = trans ? F->m : F->n, rout = trans ? F->n : F->m;
  for (size_t k = 0; k < P.stages.size(); ++k) {
    const Stage& st = P.stages[k];
    // algorithmic bytes: this stage's factor entries once, plus the caller's
    // input (first stage) and output (last stage); intermediates excluded
    double by = 8.0 * st.macs;
    if (k == 0) by += 8.0 * (double)rin * ncols;
    if (k + 1 == P.stages.size()) by += 8.0 * (double)rout * ncols;
    ProfScope ps(BF_KC_APPLY, s, 8.0 * st.macs * ncols, by);
    launch_apply_stage(P.desc.p + st.off, st.count, P.G.p, bufs, lds, ncols, st.maxM, s);
  }
}

}  // namespace bf
