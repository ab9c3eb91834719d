// km_tune.cpp -- persisted choices of the sweep-length tuner of the batched
// small-problem launches.
//
// A choice is keyed by the launch's shape bucket: low format, correction
// precision, threshold on/off, the largest row capacity of its kernel
// (8 / 16 / 32 coordinates), the largest padded centre count, and the
// launch's total points rounded down to a power of two.  The value is the
// number of 32-point groups per wave that timed fastest, with the measured
// times.  One cache per context; a file path makes it persistent (text, one
// entry per line: key, choice, then the times in ms).
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>

#include "km_context.hpp"

namespace km {

std::string TuneCache::key(int low, int high, bool fallback, int xd, int k_pad, int64_t points) {
  int lg = 0;
  while (lg < 62 && (int64_t(1) << (lg + 1)) <= points) ++lg;
  char b[128];
  snprintf(b, sizeof(b), "small:low=%d:high=%d:fb=%d:xd=%d:kpad=%d:pts=2^%d", low, high, fallback ? 1 : 0,
           xd, k_pad, lg);
  return b;
}

bool TuneCache::lookup(const std::string& k, int* gpw) {
  std::lock_guard<std::mutex> g(mu);
  auto it = entries.find(k);
  if (it == entries.end()) return false;
  *gpw = it->second.gpw;
  return true;
}

void TuneCache::store(const std::string& k, int gpw, const std::vector<float>& ms) {
  std::lock_guard<std::mutex> g(mu);
  entries[k] = Entry{gpw, ms};
  if (!path.empty()) save_locked();
}

int32_t TuneCache::set_path(const char* p) {
  std::lock_guard<std::mutex> g(mu);
  path = p ? p : "";
  if (path.empty()) return KM_OK;
  std::ifstream in(path);
  if (!in) return KM_OK;  // a new file: written on the first choice
  std::string line;
  while (std::getline(in, line)) {
    std::istringstream ls(line);
    std::string k;
    Entry e{};
    if (!(ls >> k >> e.gpw) || (e.gpw != 1 && e.gpw != 2 && e.gpw != 4 && e.gpw != 8 && e.gpw != 16 && e.gpw != 32))
      continue;  // malformed lines are ignored
    float t;
    while (ls >> t) e.ms.push_back(t);
    entries[k] = e;
  }
  return KM_OK;
}

void TuneCache::save_locked() {
  const std::string tmp = path + ".tmp";
  {
    std::ofstream out(tmp, std::ios::trunc);
    if (!out) return;
    for (auto& kv : entries) {
      out << kv.first << ' ' << kv.second.gpw;
      for (float t : kv.second.ms) out << ' ' << t;
      out << '\n';
    }
  }
  std::rename(tmp.c_str(), path.c_str());
}

std::string TuneCache::dump() {
  std::lock_guard<std::mutex> g(mu);
  std::ostringstream o;
  for (auto& kv : entries) {
    o << kv.first << ' ' << kv.second.gpw;
    for (float t : kv.second.ms) o << ' ' << t;
    o << '\n';
  }
  return o.str();
}

}  // namespace km

using namespace km;

extern "C" {

int32_t kmeans_tune_cache(km_context* ctx, const char* path) {
  if (!ctx) return KM_ERR_ARG;
  return ctx->tune.set_path(path);
}

int64_t kmeans_tune_dump(km_context* ctx, char* buf, int64_t cap) {
  if (!ctx || cap < 0 || (cap > 0 && !buf)) return KM_ERR_ARG;
  const std::string s = ctx->tune.dump();
  if (cap > 0) {
    const size_t n = std::min(s.size(), (size_t)cap - 1);
    memcpy(buf, s.data(), n);
    buf[n] = '\0';
  }
  return (int64_t)s.size();
}

}  // extern "C"
