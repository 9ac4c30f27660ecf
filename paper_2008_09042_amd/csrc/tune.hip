// Persistent cache of plan-time kernel choices (host code).
//
// A plan picks some kernels per shape by timing the candidates on the device (the dense
// basis products: the streaming kernel against the tiled GEMM at each split-K factor).  The
// choices are kept for the process and in a text file keyed by shape and GPU architecture,
// so that a later process on the same kind of GPU reuses them instead of timing again.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <sys/stat.h>

#include "tune.h"

namespace mx {

namespace {

std::mutex g_mu;
std::map<std::string, int> g_mem;
bool g_loaded = false;
long long g_measured = 0, g_reused = 0;

std::string cache_path() {
  const char* env = std::getenv("MAXWELL_TUNE_CACHE");
  if (env) return std::string(env);
  const char* home = std::getenv("HOME");
  if (!home || !home[0]) return std::string();
  const std::string dir = std::string(home) + "/.cache/maxwell";
  (void)mkdir((std::string(home) + "/.cache").c_str(), 0755);
  (void)mkdir(dir.c_str(), 0755);
  return dir + "/tune.txt";
}

// Lines "key = value"; keys hold no '=' (they are built from names and numbers).
void load_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const std::string path = cache_path();
  if (path.empty()) return;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    const size_t eq = line.rfind(" = ");
    if (eq == std::string::npos) continue;
    std::istringstream v(line.substr(eq + 3));
    int value = 0;
    if (v >> value) g_mem[line.substr(0, eq)] = value;
  }
}

void append(const std::string& key, int value) {
  const std::string path = cache_path();
  if (path.empty()) return;
  if (FILE* f = std::fopen(path.c_str(), "a")) {
    std::fprintf(f, "%s = %d\n", key.c_str(), value);
    std::fclose(f);
  }
}

}  // namespace

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  return std::string(prop.gcnArchName);
}

int tuned_choice(const std::string& key, const std::function<int()>& measure) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    auto it = g_mem.find(key);
    if (it != g_mem.end()) {
      ++g_reused;
      return it->second;
    }
  }
  const int v = measure();
  std::lock_guard<std::mutex> lk(g_mu);
  ++g_measured;
  g_mem[key] = v;
  append(key, v);
  return v;
}

void tune_counts(long long* measured, long long* reused) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (measured) *measured = g_measured;
  if (reused) *reused = g_reused;
}

}  // namespace mx
