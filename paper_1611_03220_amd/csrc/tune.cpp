// Tuning table of the kernel products: launch choices (column splits, right-hand-side pass
// width) found by timing candidates per problem shape, kept for the process and optionally
// persisted as a small JSON file keyed by the GPU architecture and a digest of the library's
// kernel sources, so a rebuilt library never reuses stale timings.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "kernels.hpp"

#ifndef KRR_CODE_DIGEST
#define KRR_CODE_DIGEST "unversioned"
#endif

namespace krr {
namespace {

typedef std::tuple<int, int, int, int, int> Key;  // prec, kind, Kp, m bucket, n bucket
std::mutex g_mu;
std::map<Key, TuneChoice> g_table;
bool g_loaded = false;

int bucket_m(int64_t m) {
  int b = 0;
  while ((int64_t(1) << b) < m) ++b;
  return b;  // ceil(log2 m)
}
int bucket_n(int64_t n) {
  int b = 0;
  while ((int64_t(1) << (b + 1)) <= n) ++b;
  return b;  // floor(log2 n)
}
Key make_key(int prec, int kind, int64_t Kp, int64_t m, int64_t n) {
  return Key(prec, kind, (int)Kp, bucket_m(m), bucket_n(n));
}

// file format: {"arch": "gfx950", "digest": "...", "entries": [[prec, kind, Kp, mb, nb,
// nsplit, pass_width, ms_default, ms_best], ...]}
bool load_file(const char* path) {
  FILE* f = fopen(path, "r");
  if (!f) return false;
  std::string txt;
  char buf[4096];
  size_t r;
  while ((r = fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, r);
  fclose(f);
  const std::string want = std::string("\"digest\": \"") + KRR_CODE_DIGEST + "\"";
  if (txt.find("\"arch\": \"gfx950\"") == std::string::npos || txt.find(want) == std::string::npos)
    return false;  // another architecture or another build of the kernels
  size_t pos = txt.find("\"entries\"");
  if (pos == std::string::npos) return false;
  pos = txt.find('[', pos);
  while (pos != std::string::npos) {
    pos = txt.find('[', pos + 1);
    if (pos == std::string::npos) break;
    int v[7];
    double ms0 = 0.0, ms1 = 0.0;
    if (sscanf(txt.c_str() + pos, "[%d, %d, %d, %d, %d, %d, %d, %lf, %lf]", &v[0], &v[1], &v[2],
               &v[3], &v[4], &v[5], &v[6], &ms0, &ms1) != 9)
      break;
    TuneChoice c;
    c.nsplit = v[5];
    c.pass_width = v[6];
    c.ms_default = ms0;
    c.ms_best = ms1;
    g_table[Key(v[0], v[1], v[2], v[3], v[4])] = c;
  }
  return true;
}

bool save_file(const char* path) {
  FILE* f = fopen(path, "w");
  if (!f) return false;
  fprintf(f, "{\"arch\": \"gfx950\", \"digest\": \"%s\", \"entries\": [", KRR_CODE_DIGEST);
  bool first = true;
  for (const auto& kv : g_table) {
    const Key& k = kv.first;
    const TuneChoice& c = kv.second;
    fprintf(f, "%s\n  [%d, %d, %d, %d, %d, %d, %d, %.6f, %.6f]", first ? "" : ",", std::get<0>(k),
            std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k), c.nsplit,
            c.pass_width, c.ms_default, c.ms_best);
    first = false;
  }
  fprintf(f, "\n]}\n");
  fclose(f);
  return true;
}

void ensure_loaded() {
  if (g_loaded) return;
  g_loaded = true;
  const char* p = getenv("KRR_TUNE_CACHE");
  if (p && *p) load_file(p);
}

}  // namespace

bool tune_lookup(int prec, int kind, int64_t Kp, int64_t m, int64_t n, TuneChoice* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  ensure_loaded();
  auto it = g_table.find(make_key(prec, kind, Kp, m, n));
  if (it == g_table.end()) return false;
  *out = it->second;
  return true;
}

void tune_store(int prec, int kind, int64_t Kp, int64_t m, int64_t n, const TuneChoice& c) {
  std::lock_guard<std::mutex> lk(g_mu);
  ensure_loaded();
  g_table[make_key(prec, kind, Kp, m, n)] = c;
  const char* p = getenv("KRR_TUNE_CACHE");
  if (p && *p) save_file(p);
}

const char* tune_digest() { return KRR_CODE_DIGEST; }

}  // namespace krr

extern "C" {

int32_t krr_tune_cache_save(const char* path) {
  std::lock_guard<std::mutex> lk(krr::g_mu);
  return path && krr::save_file(path) ? 1 : 0;
}

int32_t krr_tune_cache_load(const char* path) {
  std::lock_guard<std::mutex> lk(krr::g_mu);
  krr::g_loaded = true;
  return path && krr::load_file(path) ? 1 : 0;
}

void krr_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lk(krr::g_mu);
  krr::g_table.clear();
  krr::g_loaded = true;
}

int32_t krr_tune_cache_size(void) {
  std::lock_guard<std::mutex> lk(krr::g_mu);
  return (int32_t)krr::g_table.size();
}

const char* krr_tune_digest(void) { return krr::tune_digest(); }

}  // extern "C"
