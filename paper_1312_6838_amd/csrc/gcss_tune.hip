// Autotuner of the streaming passes' launch settings: time the selection
// call under each candidate setting with HIP events, keep the fastest, and
// remember it in a JSON file keyed by architecture, m, ceil(log2 n), storage
// type and target kind (and the block count of the batched call).
//
// The cache file is one JSON object whose members map a key to a setting:
//   {
//   "gfx950 select m=4096 n2=16 f32 gram": {"stream_pd": 1, "stream_upw": 4,
//        "batch_group": 64, "batch_wg_per_cu": 0, "ms": 2.5},
//   ...
//   }
// (each member on one line).  Members of other keys are kept when the file
// is rewritten; unknown fields of a member are ignored.
#include <hip/hip_runtime.h>
#include <unistd.h>

#include <algorithm>
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "../../include/gcss.h"
#include "gcss_internal.h"

using namespace gcss;

namespace {

struct Entry {
  std::string key;
  gcss_tuning t;
  double ms;
};

// ---- restricted JSON reader: an object of objects of numbers ----
struct Reader {
  const std::string &s;
  size_t i = 0;
  explicit Reader(const std::string &text) : s(text) {}
  void ws() {
    while (i < s.size() && isspace((unsigned char)s[i])) ++i;
  }
  bool eat(char c) {
    ws();
    if (i < s.size() && s[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
  bool str(std::string *out) {
    ws();
    if (i >= s.size() || s[i] != '"') return false;
    ++i;
    out->clear();
    while (i < s.size() && s[i] != '"') {
      if (s[i] == '\\') return false;  // keys and field names never need escapes
      out->push_back(s[i++]);
    }
    if (i >= s.size()) return false;
    ++i;
    return true;
  }
  bool num(double *out) {
    ws();
    const char *b = s.c_str() + i;
    char *e = nullptr;
    *out = strtod(b, &e);
    if (e == b) return false;
    i += (size_t)(e - b);
    return true;
  }
};

bool parse_cache(const std::string &text, std::vector<Entry> *out) {
  Reader r(text);
  if (!r.eat('{')) return false;
  if (r.eat('}')) return true;
  do {
    Entry e{};
    e.t = gcss_tuning{1, 4, 64, 0};
    if (!r.str(&e.key) || !r.eat(':') || !r.eat('{')) return false;
    if (!r.eat('}')) {
      do {
        std::string name;
        double v = 0.0;
        if (!r.str(&name) || !r.eat(':') || !r.num(&v)) return false;
        if (name == "stream_pd") e.t.stream_pd = (int32_t)v;
        else if (name == "stream_upw") e.t.stream_upw = (int32_t)v;
        else if (name == "batch_group") e.t.batch_group = (int32_t)v;
        else if (name == "batch_wg_per_cu") e.t.batch_wg_per_cu = (int32_t)v;
        else if (name == "ms") e.ms = v;
      } while (r.eat(','));
      if (!r.eat('}')) return false;
    }
    out->push_back(e);
  } while (r.eat(','));
  if (!r.eat('}')) return false;
  r.ws();
  return r.i == text.size();
}

std::string format_cache(const std::vector<Entry> &es) {
  std::string o = "{\n";
  char line[512];
  for (size_t x = 0; x < es.size(); ++x) {
    const Entry &e = es[x];
    snprintf(line, sizeof line,
             "\"%s\": {\"stream_pd\": %d, \"stream_upw\": %d, \"batch_group\": %d, "
             "\"batch_wg_per_cu\": %d, \"ms\": %.6f}%s\n",
             e.key.c_str(), e.t.stream_pd, e.t.stream_upw, e.t.batch_group, e.t.batch_wg_per_cu,
             e.ms, x + 1 < es.size() ? "," : "");
    o += line;
  }
  return o + "}\n";
}

// 0: read (or the file does not exist: empty); -1: unreadable or malformed
int load_cache(const char *path, std::vector<Entry> *out, std::string *why) {
  FILE *f = fopen(path, "rb");
  if (!f) return 0;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
  const bool bad = ferror(f) != 0;
  fclose(f);
  if (bad) {
    *why = "cannot read the tuning cache";
    return -1;
  }
  if (!parse_cache(text, out)) {
    *why = "the tuning cache is not a JSON object of settings";
    return -1;
  }
  return 0;
}

bool store_cache(const char *path, const std::vector<Entry> &es) {
  const std::string tmp = std::string(path) + ".tmp." + std::to_string((long)getpid());
  FILE *f = fopen(tmp.c_str(), "wb");
  if (!f) return false;
  const std::string text = format_cache(es);
  const bool ok = fwrite(text.data(), 1, text.size(), f) == text.size();
  if (fclose(f) != 0 || !ok) {
    remove(tmp.c_str());
    return false;
  }
  if (rename(tmp.c_str(), path) != 0) {
    remove(tmp.c_str());
    return false;
  }
  return true;
}

int ceil_log2(int64_t n) {
  int b = 0;
  while (b < 62 && ((int64_t)1 << b) < n) ++b;
  return b;
}

std::string cache_key(const CtxInfo &c, const char *what, int nblocks) {
  static const char *dt[] = {"f32", "bf16", "fp8"};
  char k[160];
  if (nblocks > 0)
    snprintf(k, sizeof k, "gfx950 %s m=%lld n2=%d %s blocks=%d", what, (long long)c.m,
             ceil_log2(c.n), dt[c.dtype], nblocks);
  else
    snprintf(k, sizeof k, "gfx950 %s m=%lld n2=%d %s %s", what, (long long)c.m, ceil_log2(c.n),
             dt[c.dtype], c.target == 2 ? "gram" : "explicit");
  return k;
}

bool same(const gcss_tuning &a, const gcss_tuning &b) {
  return a.stream_pd == b.stream_pd && a.stream_upw == b.stream_upw &&
         a.batch_group == b.batch_group && a.batch_wg_per_cu == b.batch_wg_per_cu;
}

// Median time (ms) of `reps` calls after one untimed call; each call is
// bracketed by events on the context's stream.
gcss_status time_calls(hipStream_t s, int reps, const std::function<gcss_status()> &call,
                       double *med) {
  gcss_status st = call();
  if (st < 0) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return GCSS_ERR_DEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return GCSS_ERR_DEVICE;
  }
  std::vector<double> t;
  for (int x = 0; x < reps && st >= 0; ++x) {
    if (hipEventRecord(e0, s) != hipSuccess) {
      st = GCSS_ERR_DEVICE;
      break;
    }
    st = call();
    if (st < 0) break;
    float ms = 0.f;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      st = GCSS_ERR_DEVICE;
      break;
    }
    t.push_back(ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st < 0) return st;
  std::sort(t.begin(), t.end());
  *med = t.size() % 2 ? t[t.size() / 2] : 0.5 * (t[t.size() / 2 - 1] + t[t.size() / 2]);
  return GCSS_OK;
}

// Sweep: the entry setting first, then the candidates; ties keep the earlier.
gcss_status sweep(gcss_ctx *h, const CtxInfo &c, const std::string &key, const char *cache_path,
                  int reps, const std::vector<gcss_tuning> &cands,
                  const std::function<gcss_status()> &call, gcss_tune_result *out) {
  std::vector<Entry> cache;
  if (cache_path) {
    std::string why;
    if (load_cache(cache_path, &cache, &why) != 0) {
      set_error((why + ": " + cache_path).c_str());
      return GCSS_ERR_ARG;
    }
    for (const Entry &e : cache)
      if (e.key == key) {
        gcss_status st = gcss_set_tuning(h, &e.t);
        if (st != GCSS_OK) return st;
        out->best = e.t;
        out->best_ms = e.ms;
        out->initial_ms = 0.0;
        out->candidates = 0;
        return GCSS_OK;
      }
  }
  gcss_tuning entry{};
  gcss_status st = gcss_get_tuning(h, &entry);
  if (st != GCSS_OK) return st;
  std::vector<gcss_tuning> order{entry};
  for (const gcss_tuning &t : cands)
    if (!same(t, entry)) order.push_back(t);
  gcss_tuning best = entry;
  double best_ms = 0.0, entry_ms = 0.0;
  int timed = 0;
  for (size_t x = 0; x < order.size(); ++x) {
    st = gcss_set_tuning(h, &order[x]);
    double ms = 0.0;
    if (st == GCSS_OK) st = time_calls(c.stream, reps, call, &ms);
    if (st < 0) {
      (void)gcss_set_tuning(h, &entry);
      return st;
    }
    ++timed;
    if (x == 0) entry_ms = ms;
    if (x == 0 || ms < best_ms) {
      best_ms = ms;
      best = order[x];
    }
  }
  st = gcss_set_tuning(h, &best);
  if (st != GCSS_OK) return st;
  out->best = best;
  out->best_ms = best_ms;
  out->initial_ms = entry_ms;
  out->candidates = timed;
  if (cache_path) {
    cache.push_back(Entry{key, best, best_ms});
    if (!store_cache(cache_path, cache)) {
      set_error((std::string("cannot write the tuning cache: ") + cache_path).c_str());
      return GCSS_ERR_ARG;
    }
  }
  return GCSS_OK;
}

}  // namespace

extern "C" {

gcss_status gcss_autotune_select(gcss_ctx *h, int32_t k, int32_t reps, const char *cache_path,
                                 gcss_tune_result *out) {
  CtxInfo c{};
  if (!ctx_describe(h, &c) || !out) {
    set_error("null argument");
    return GCSS_ERR_ARG;
  }
  if (k < 1 || reps < 1) {
    set_error("k and reps must be positive");
    return GCSS_ERR_ARG;
  }
  if (c.target == 0) {
    set_error("autotuning the selection needs a target");
    return GCSS_ERR_STATE;
  }
  std::vector<int64_t> idx(k);
  std::vector<double> obj(k + 1);
  int32_t ns = 0;
  auto call = [&]() { return gcss_select(h, k, idx.data(), obj.data(), &ns); };
  std::vector<gcss_tuning> cands;
  gcss_tuning base{};
  gcss_status st = gcss_get_tuning(h, &base);
  if (st != GCSS_OK) return st;
  for (int pd = 1; pd <= 2; ++pd)
    for (int upw : {2, 4, 8, 16}) {
      gcss_tuning t = base;
      t.stream_pd = pd;
      t.stream_upw = upw;
      cands.push_back(t);
    }
  return sweep(h, c, cache_key(c, "select", 0), cache_path, reps, cands, call, out);
}

gcss_status gcss_autotune_batched(gcss_ctx *h, int32_t nblocks, const int64_t *col_off,
                                  int32_t k_block, int32_t k_merge, int32_t reps,
                                  const char *cache_path, gcss_tune_result *out) {
  CtxInfo c{};
  if (!ctx_describe(h, &c) || !out || !col_off) {
    set_error("null argument");
    return GCSS_ERR_ARG;
  }
  if (nblocks < 1 || k_block < 1 || k_merge < 1 || reps < 1) {
    set_error("nblocks, k_block, k_merge and reps must be positive");
    return GCSS_ERR_ARG;
  }
  std::vector<int64_t> ib((size_t)nblocks * k_block), im(k_merge);
  std::vector<double> obj(k_merge + 1);
  int32_t nm = 0;
  auto call = [&]() {
    return gcss_select_batched(h, nblocks, col_off, k_block, k_merge, ib.data(), im.data(),
                               obj.data(), &nm);
  };
  // argument and state errors surface before any setting changes
  gcss_status st = call();
  if (st < 0) return st;
  std::vector<gcss_tuning> cands;
  gcss_tuning base{};
  st = gcss_get_tuning(h, &base);
  if (st != GCSS_OK) return st;
  for (int gsz : {16, 32, 64})
    for (int wpc : {0, 2, 4}) {
      gcss_tuning t = base;
      t.batch_group = gsz;
      t.batch_wg_per_cu = wpc;
      cands.push_back(t);
    }
  return sweep(h, c, cache_key(c, "batched", nblocks), cache_path, reps, cands, call, out);
}

}  // extern "C"
