// Persistent cache of autotuned launch choices.  An entry maps a key naming
// the device architecture, the kernel and the shape class to the chosen value;
// entries are loaded once per process from a text file (one "key value" line
// each) and appended when a new choice is made, so a later process skips the
// tuning runs.  File: $GABP_TUNE_CACHE, else $XDG_CACHE_HOME/gabp-mi355x/tune.txt,
// else $HOME/.cache/gabp-mi355x/tune.txt; GABP_TUNE_CACHE=off (or an unusable
// path) keeps the choices for the life of the process only.
#include <sys/stat.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "engine.h"

namespace gabp {
namespace {

std::mutex g_mu;
std::map<std::string, int> g_entries;
bool g_loaded = false;
std::string g_path;

std::string cache_path() {
  const char *p = std::getenv("GABP_TUNE_CACHE");
  if (p && *p) return std::strcmp(p, "off") == 0 ? std::string() : std::string(p);
  std::string dir;
  if (const char *x = std::getenv("XDG_CACHE_HOME"); x && *x) dir = x;
  else if (const char *h = std::getenv("HOME"); h && *h) dir = std::string(h) + "/.cache";
  else return std::string();
  dir += "/gabp-mi355x";
  ::mkdir(dir.c_str(), 0755);  // may exist already; a failure shows at open
  return dir + "/tune.txt";
}

void load_locked() {
  if (g_loaded) return;
  g_loaded = true;
  g_path = cache_path();
  if (g_path.empty()) return;
  std::ifstream in(g_path);
  std::string line;
  while (std::getline(in, line)) {
    std::istringstream ls(line);
    std::string key;
    int v = 0;
    if (ls >> key >> v) g_entries[key] = v;
  }
}

std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown";
  }
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');  // drop feature suffixes (":sramecc+:xnack-")
  return colon == std::string::npos ? a : a.substr(0, colon);
}

}  // namespace

std::string tune_key(const std::string &kernel, const std::string &shape) {
  return arch_name() + "|" + gabp_version() + "|" + kernel + "|" + shape;
}

bool tune_lookup(const std::string &key, int *value) {
  std::lock_guard<std::mutex> lock(g_mu);
  load_locked();
  auto it = g_entries.find(key);
  if (it == g_entries.end()) return false;
  *value = it->second;
  return true;
}

void tune_store(const std::string &key, int value) {
  std::lock_guard<std::mutex> lock(g_mu);
  load_locked();
  g_entries[key] = value;
  if (g_path.empty()) return;
  if (FILE *f = std::fopen(g_path.c_str(), "a")) {
    std::fprintf(f, "%s %d\n", key.c_str(), value);
    std::fclose(f);
  }
}

}  // namespace gabp
