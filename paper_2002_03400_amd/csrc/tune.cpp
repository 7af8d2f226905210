// Launch-shape autotuner: for each kernel family and shape class, the fastest
// of a few launch variants that give bitwise the same results, timed with
// events on the stream of the first launch of the class (that launch runs
// every candidate once to warm caches and code, then three interleaved timed
// rounds, keeping each candidate's fastest, and keeps the results of the
// last run, which equal the others').  Families and their candidates:
//   black-box column tile   48 / 64 / 80 columns (split-BF16 products of more than 48)
//   chain tile height       8 / 16 (one wave per descriptor) or 20 / 24 / 32 / 64
//                           rows, every height at least the launch's largest M
//   CPQR workgroup          256 or 512 threads (LDS-resident blocks)
//   few-column apply        fused stages or one launch per stage (1 to 4 columns)
// The table is process-wide, loaded at the first lookup from BF_TUNE_FILE or,
// when that is unset, from tune_gfx950.tsv next to libbf.so (if present), and
// written back by bf_autotune_save.  A tuning launch synchronizes its stream
// once; launches under HIP graph capture never tune.
#include <dlfcn.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>

#include "bf_internal.h"

namespace bf {

namespace {
std::atomic<int> g_on{1};
std::mutex g_mu;
std::map<TuneKey, int64_t> g_table;
std::map<TuneKey, std::vector<std::pair<int64_t, float>>> g_times;   // measured candidates
std::once_flag g_load_once;

const char* kFamily[kTuneFamilies] = {"matfree_width", "chain_rows", "cpqr_threads",
                                      "apply_fused", "apply_rows", "apply_mfma"};

std::string default_path() {
  if (const char* e = std::getenv("BF_TUNE_FILE")) return e;
  Dl_info info;
  if (dladdr((void*)&default_path, &info) && info.dli_fname) {
    std::string p = info.dli_fname;
    const size_t slash = p.rfind('/');
    return (slash == std::string::npos ? std::string(".") : p.substr(0, slash)) +
           "/tune_gfx950.tsv";
  }
  return "tune_gfx950.tsv";
}

// one entry per line: family name, the key's class fields, the choice
int load_into(const std::string& path, std::map<TuneKey, int64_t>& t) {
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return -1;
  char name[64];
  long long v[kTuneKeyFields], choice;
  int n = 0;
  while (std::fscanf(f, "%63s", name) == 1) {
    if (name[0] == '#') {
      int c;
      while ((c = std::fgetc(f)) != '\n' && c != EOF) {
      }
      continue;
    }
    bool ok = true;
    for (int i = 0; i < kTuneKeyFields && ok; ++i) ok = std::fscanf(f, "%lld", &v[i]) == 1;
    if (!ok || std::fscanf(f, "%lld", &choice) != 1) break;
    for (int fam = 0; fam < kTuneFamilies; ++fam)
      if (std::string(name) == kFamily[fam]) {
        TuneKey k{};
        k[0] = fam;
        for (int i = 0; i < kTuneKeyFields; ++i) k[1 + i] = v[i];
        t[k] = choice;
        ++n;
      }
  }
  std::fclose(f);
  return n;
}

void load_default() {
  std::call_once(g_load_once, [] {
    std::map<TuneKey, int64_t> t;
    if (load_into(default_path(), t) > 0) {
      std::lock_guard<std::mutex> lk(g_mu);
      for (auto& kv : t) g_table.emplace(kv.first, kv.second);
    }
  });
}

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}
}  // namespace

int64_t pow2_ceil(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

void set_autotune(int on) { g_on.store(on ? 1 : 0); }
bool autotune_on() { return g_on.load() != 0; }

int64_t autotune_entries() {
  load_default();
  std::lock_guard<std::mutex> lk(g_mu);
  return (int64_t)g_table.size();
}

int64_t tune_choose(const TuneKey& key, const std::vector<int64_t>& cand, int64_t fallback,
                    hipStream_t s, const std::function<void(int64_t)>& run, bool may_time) {
  if (cand.size() <= 1 || !autotune_on()) {
    run(fallback);
    return fallback;
  }
  load_default();
  // look the class up under the lock, run outside it: a candidate may itself
  // launch tuned kernels (a staged apply's stages)
  int64_t known = 0;
  bool found = false;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find(key);
    if (it != g_table.end()) {
      for (int64_t c : cand)
        if (c == it->second) {
          known = c;
          found = true;
        }
    }
  }
  if (found) {
    run(known);
    return known;
  }
  if (!may_time || capturing(s)) {
    run(fallback);
    return fallback;
  }
  // every candidate once untimed (caches and code warm alike for all), then
  // kTuneRounds interleaved timed rounds; a candidate's time is its fastest
  // round (robust to other streams' work passing through the device)
  constexpr int kTuneRounds = 3;
  for (int64_t c : cand) run(c);
  const size_t nc = cand.size();
  std::vector<hipEvent_t> ev(nc * kTuneRounds + 1, nullptr);
  for (auto& e : ev) BF_HIP(hipEventCreate(&e));
  BF_HIP(hipEventRecord(ev[0], s));
  for (int r = 0; r < kTuneRounds; ++r)
    for (size_t i = 0; i < nc; ++i) {
      run(cand[i]);
      BF_HIP(hipEventRecord(ev[r * nc + i + 1], s));
    }
  BF_HIP(hipEventSynchronize(ev.back()));
  int64_t best = cand.back();
  float best_ms = 0.f;
  std::vector<std::pair<int64_t, float>> times;
  for (size_t i = 0; i < nc; ++i) {
    float ms = 0.f;
    for (int r = 0; r < kTuneRounds; ++r) {
      float m = 0.f;
      BF_HIP(hipEventElapsedTime(&m, ev[r * nc + i], ev[r * nc + i + 1]));
      ms = r == 0 ? m : std::min(ms, m);
    }
    times.push_back({cand[i], ms});
    if (i == 0 || ms < best_ms) {
      best_ms = ms;
      best = cand[i];
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  std::lock_guard<std::mutex> lk(g_mu);
  g_table[key] = best;
  g_times[key] = times;
  return best;
}

int tune_save(const char* path) {
  load_default();
  const std::string p = path && path[0] ? std::string(path) : default_path();
  FILE* f = std::fopen(p.c_str(), "w");
  if (!f) return BF_EINVAL;
  std::fprintf(f, "# family  class fields (%d)  choice\n", kTuneKeyFields);
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_table) {
    std::fprintf(f, "%s", kFamily[kv.first[0]]);
    for (int i = 0; i < kTuneKeyFields; ++i) std::fprintf(f, " %lld", (long long)kv.first[1 + i]);
    std::fprintf(f, " %lld\n", (long long)kv.second);
    auto it = g_times.find(kv.first);
    if (it != g_times.end()) {   // the timed candidates, as a comment line
      std::fprintf(f, "#   timed:");
      for (auto& ct : it->second) std::fprintf(f, " %lld=%.4fms", (long long)ct.first, ct.second);
      std::fprintf(f, "\n");
    }
  }
  return std::fclose(f) == 0 ? BF_OK : BF_EINVAL;
}

int tune_load(const char* path) {
  std::map<TuneKey, int64_t> t;
  const int n = load_into(path && path[0] ? std::string(path) : default_path(), t);
  if (n < 0) return BF_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : t) g_table[kv.first] = kv.second;
  return BF_OK;
}

void tune_clear() {
  load_default();   // a later first lookup must not bring the file back
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
  g_times.clear();
}

}  // namespace bf
