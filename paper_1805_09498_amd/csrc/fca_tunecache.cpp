// Persistent cache of measured launch shapes.  When the environment variable
// FASTFCA_TUNE_CACHE names a file, every shape the tuners measure is appended
// to it as one line "<key>\t<a> <b>" and later processes read it instead of
// measuring again.  The key starts with the device's architecture name, its
// compute-unit count and the build stamp of this library, so a rebuilt
// library or another GPU model never reuses an entry.  Without the variable
// the tuners keep their results for the life of the process only.
#include <hip/hip_runtime.h>

#include <sys/stat.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>

#include "fca_internal.h"

namespace {

std::mutex g_mu;
std::string g_path;        // file the map was read from
long long g_size = -1;     // its size then (re-read when it changes)
std::map<std::string, std::pair<int, int>> g_disk;

const char* cache_path() {
  const char* p = std::getenv("FASTFCA_TUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

long long file_size(const char* path) {
  struct stat st;
  return stat(path, &st) == 0 ? (long long)st.st_size : -1;
}

// (Re-)read the file when it is another file or has changed size since the
// last read (other processes append to it).
void refresh_locked(const char* path) {
  const long long size = file_size(path);
  if (g_path == path && g_size == size) return;
  g_path = path;
  g_size = size;
  g_disk.clear();
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[1024];
  while (std::fgets(line, sizeof line, f)) {
    char* tab = std::strchr(line, '\t');
    if (!tab) continue;
    *tab = '\0';
    int a = 0, b = 0;
    if (std::sscanf(tab + 1, "%d %d", &a, &b) == 2) g_disk[line] = {a, b};  // later lines win
  }
  std::fclose(f);
}

}  // namespace

namespace fca {

std::string tune_key_prefix() {
  int dev = 0;
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  int cus = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    cus = prop.multiProcessorCount;
  }
  return arch + " cu" + std::to_string(cus) + " build " + __DATE__ + " " + __TIME__;
}

bool tune_cache_get(const std::string& key, int* a, int* b) {
  const char* path = cache_path();
  if (!path) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  refresh_locked(path);
  auto it = g_disk.find(key);
  if (it == g_disk.end()) return false;
  *a = it->second.first;
  *b = it->second.second;
  return true;
}

void tune_cache_put(const std::string& key, int a, int b) {
  const char* path = cache_path();
  if (!path || key.find('\n') != std::string::npos || key.find('\t') != std::string::npos) return;
  std::lock_guard<std::mutex> lk(g_mu);
  refresh_locked(path);
  // One short line per write: appends from several processes do not interleave.
  FILE* f = std::fopen(path, "a");
  if (!f) return;  // an unwritable cache only costs a re-measurement
  std::fprintf(f, "%s\t%d %d\n", key.c_str(), a, b);
  std::fclose(f);
  g_disk[key] = {a, b};
  g_size = file_size(path);
}

}  // namespace fca
