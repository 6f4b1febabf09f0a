// Autotuner cache (see tune.h).

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <sys/stat.h>
#include <unistd.h>

#include "tune.h"

namespace abddc {

namespace {

std::mutex g_mu;
std::map<std::string, int>* g_table = nullptr;
bool g_loaded = false;
std::string g_loaded_path;

std::string cache_path() {
  const char* env = std::getenv("ABDDC_TUNE_CACHE");
  if (env && std::string(env) == "off") return "";
  if (env && *env) return env;
  const char* home = std::getenv("HOME");
  if (!home || !*home) return "";
  return std::string(home) + "/.cache/abddc/tune.json";
}

// the file is one flat JSON object of "key": integer pairs
// (re)loads when the cache file named by the environment has changed
void load_locked() {
  const std::string path = cache_path();
  if (g_loaded && path == g_loaded_path) return;
  g_loaded = true;
  g_loaded_path = path;
  if (!g_table) g_table = new std::map<std::string, int>();
  g_table->clear();
  if (path.empty()) return;
  std::ifstream f(path);
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t i = 0;
  while (true) {
    const size_t a = s.find('"', i);
    if (a == std::string::npos) break;
    const size_t b = s.find('"', a + 1);
    if (b == std::string::npos) break;
    const size_t colon = s.find(':', b);
    if (colon == std::string::npos) break;
    const std::string key = s.substr(a + 1, b - a - 1);
    char* end = nullptr;
    const long v = std::strtol(s.c_str() + colon + 1, &end, 10);
    if (end != s.c_str() + colon + 1) (*g_table)[key] = (int)v;
    i = end ? (size_t)(end - s.c_str()) : colon + 1;
  }
}

void save_locked() {
  const std::string path = cache_path();
  if (path.empty()) return;
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos) {
    // create the directory chain (best effort)
    std::string dir = path.substr(0, slash);
    for (size_t p = 1; p <= dir.size(); ++p)
      if (p == dir.size() || dir[p] == '/') mkdir(dir.substr(0, p).c_str(), 0755);
  }
  const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
  {
    std::ofstream f(tmp);
    if (!f) return;
    f << "{\n";
    size_t k = 0;
    for (const auto& kv : *g_table) f << "  \"" << kv.first << "\": " << kv.second << (++k < g_table->size() ? ",\n" : "\n");
    f << "}\n";
  }
  std::rename(tmp.c_str(), path.c_str());
}

}  // namespace

std::string device_arch(int device) {
  // hipGetDeviceProperties is slow: query once per device
  static std::mutex mu;
  static std::map<int, std::string> known;
  std::lock_guard<std::mutex> g(mu);
  auto it = known.find(device);
  if (it != known.end()) return it->second;
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) != hipSuccess) return "unknown";
  std::string a = p.gcnArchName;
  const size_t colon = a.find(':');
  a = colon == std::string::npos ? a : a.substr(0, colon);
  known[device] = a;
  return a;
}

int tune_lookup(const std::string& key) {
  std::lock_guard<std::mutex> g(g_mu);
  load_locked();
  auto it = g_table->find(key);
  return it == g_table->end() ? -1 : it->second;
}

void tune_store(const std::string& key, int value) {
  std::lock_guard<std::mutex> g(g_mu);
  load_locked();
  (*g_table)[key] = value;
  save_locked();
}

int size_bucket(long long v) {
  int b = 0;
  while ((1LL << b) < v) ++b;
  return b;
}

}  // namespace abddc
