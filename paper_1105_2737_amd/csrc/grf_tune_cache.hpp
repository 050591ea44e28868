// The autotuners' cache: a text file named by GRF_TUNE_CACHE, one choice per
// line, whitespace-separated fields
//   <scope> <arch> <dtype> <pass> <direction> <length> <choice...>
// scope "plan" (the runtime-radix / compile-time choice of one pass of a plan)
// or "batch" (a tile-shape variant of the uneven batch).  Lines of another
// architecture, another scope or that do not parse are skipped; the last
// valid line for a key wins.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <sstream>
#include <string>
#include <vector>

namespace grf {
namespace tune {

inline std::string cache_path() {
  const char* e = std::getenv("GRF_TUNE_CACHE");
  return e ? std::string(e) : std::string();
}

// gfx name of a device, without feature suffixes ("gfx950").
inline std::string arch_name(int dev) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

struct Line {
  std::string scope, arch, dtype, pass, dir;
  long long length = 0;
  std::vector<std::string> choice;
};

// Every line of the cache of the given scope and architecture that has the
// key fields and at least one choice field.
inline std::vector<Line> read(const std::string& scope, const std::string& arch) {
  std::vector<Line> out;
  const std::string path = cache_path();
  if (path.empty()) return out;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return out;
  char buf[512];
  while (std::fgets(buf, sizeof(buf), f)) {
    std::istringstream is(buf);
    Line l;
    std::string len;
    if (!(is >> l.scope >> l.arch >> l.dtype >> l.pass >> l.dir >> len)) continue;
    if (l.scope != scope || l.arch != arch) continue;
    char* end = nullptr;
    l.length = std::strtoll(len.c_str(), &end, 10);
    if (end == len.c_str() || *end != '\0' || l.length <= 0) continue;
    std::string w;
    while (is >> w) l.choice.push_back(w);
    if (!l.choice.empty()) out.push_back(l);
  }
  std::fclose(f);
  return out;
}

inline void append(const std::string& text) {
  const std::string path = cache_path();
  if (path.empty() || text.empty()) return;
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;
  std::fputs(text.c_str(), f);
  std::fclose(f);
}

}  // namespace tune
}  // namespace grf
