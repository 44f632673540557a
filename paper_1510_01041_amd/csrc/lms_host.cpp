// Host-side utilities shared by the C-ABI entry points (see lms_host.h).
#include "lms_host.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

namespace lms_host {
namespace {

thread_local std::string g_err;

struct Workspace {
  void* base = nullptr;
  size_t bytes = 0;
};

std::mutex g_mu;
std::map<std::tuple<int, void*, int>, Workspace> g_ws;
int g_num_cu = 0;
bool g_prof_on = false;
std::vector<std::array<hipEvent_t, LMS_NSTAGES + 1>> g_prof_events;

// tuning table: key (arch, path, size class)
std::map<std::tuple<std::string, int, int>, lms_tuning> g_tune;
bool g_tune_loaded = false;

std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "unknown";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

// One entry per line: arch path class tile_regs tile_batches seed_pairs
// bins_log2 ms range (a JSON array of arrays, so that other tools can read it).
void load_tuning_locked() {
  g_tune_loaded = true;
  const char* path = std::getenv("LMS_TUNE_FILE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char arch[64];
  int p, c, r, b, sp, bl, rg;
  double ms;
  int ch;
  while ((ch = std::fgetc(f)) != EOF) {
    if (ch != '[') continue;
    if (std::fscanf(f, " \"%63[^\"]\" , %d , %d , %d , %d , %d , %d , %lf , %d ]", arch, &p, &c,
                    &r, &b, &sp, &bl, &ms, &rg) == 9) {
      lms_tuning t{r, b, sp, bl, ms, rg, 0};
      g_tune[{arch, p, c}] = t;
    }
  }
  std::fclose(f);
}

void save_tuning_locked() {
  const char* path = std::getenv("LMS_TUNE_FILE");
  if (!path) return;
  FILE* f = std::fopen(path, "w");
  if (!f) return;
  std::fprintf(f, "[\n");
  size_t k = 0;
  for (auto& kv : g_tune) {
    std::fprintf(f, " [\"%s\", %d, %d, %d, %d, %d, %d, %.6f, %d]%s\n",
                 std::get<0>(kv.first).c_str(), std::get<1>(kv.first), std::get<2>(kv.first),
                 kv.second.tile_regs, kv.second.tile_batches, kv.second.seed_pairs,
                 kv.second.bins_log2, kv.second.ms, kv.second.range,
                 ++k < g_tune.size() ? "," : "");
  }
  std::fprintf(f, "]\n");
  std::fclose(f);
}

}  // namespace

int size_class(int n) {
  int p = 64;
  while (p < n) p <<= 1;
  return p;
}

void clear_tuning() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_tune.clear();
  g_tune_loaded = true;  // and do not read the file again
}

bool get_tuning(int path, int cls, lms_tuning* t) {
  const std::string a = arch_name();
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_tune_loaded) load_tuning_locked();
  auto it = g_tune.find({a, path, cls});
  if (it == g_tune.end()) return false;
  *t = it->second;
  return true;
}

void set_tuning(int path, int cls, const lms_tuning& t) {
  const std::string a = arch_name();
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_tune_loaded) load_tuning_locked();
  g_tune[{a, path, cls}] = t;
  save_tuning_locked();
}

lms_status fail(lms_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

void clear_error() { g_err.clear(); }

const char* last_error() { return g_err.c_str(); }

int num_cu() {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_num_cu == 0) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      g_num_cu = prop.multiProcessorCount;
    else
      return 256;
  }
  return g_num_cu;
}

lms_status get_workspace(int tag, void* stream, size_t bytes, char** base) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(LMS_ERR_DEVICE, "hipGetDevice failed");
  (void)num_cu();
  std::lock_guard<std::mutex> lk(g_mu);
  Workspace& w = g_ws[{dev, stream, tag}];
  if (w.bytes < bytes) {
    if (w.base) {
      if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        return fail(LMS_ERR_DEVICE, "hipStreamSynchronize failed");
      (void)hipFree(w.base);
      w.base = nullptr;
      w.bytes = 0;
    }
    if (hipMalloc(&w.base, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(LMS_ERR_NOMEM, "hipMalloc of the workspace failed");
    }
    w.bytes = bytes;
  }
  *base = (char*)w.base;
  return LMS_OK;
}

void free_workspace(int tag, void* stream) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ws.find({dev, stream, tag});
  if (it != g_ws.end()) {
    (void)hipFree(it->second.base);
    g_ws.erase(it);
  }
}

void free_workspaces() {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_ws)
    if (kv.second.base) (void)hipFree(kv.second.base);
  g_ws.clear();
}

void StageEvents::start(hipStream_t stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  on = g_prof_on;
  s = stream;
  if (!on) return;
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) {
      on = false;
      return;
    }
  if (on && next <= LMS_NSTAGES) (void)hipEventRecord(ev[next++], s);
}

void StageEvents::mark() {
  if (on && next <= LMS_NSTAGES) (void)hipEventRecord(ev[next++], s);
}

void StageEvents::finish() {
  if (!on) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (next == LMS_NSTAGES + 1) {
    g_prof_events.push_back(ev);
  } else {
    for (auto& e : ev) (void)hipEventDestroy(e);
  }
  on = false;
}

void profile_begin() {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& ev : g_prof_events)
    for (auto& e : ev) (void)hipEventDestroy(e);
  g_prof_events.clear();
  g_prof_on = true;
}

int64_t profile_end(double* ms) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_prof_on = false;
  double sum[LMS_NSTAGES] = {0};
  int64_t count = 0;
  int64_t st = 0;
  for (auto& ev : g_prof_events) {
    if (st == 0 && hipEventSynchronize(ev[LMS_NSTAGES]) != hipSuccess) st = LMS_ERR_DEVICE;
    for (int k = 0; st == 0 && k < LMS_NSTAGES; ++k) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, ev[k], ev[k + 1]) != hipSuccess) st = LMS_ERR_DEVICE;
      sum[k] += t;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    ++count;
  }
  g_prof_events.clear();
  if (ms)
    for (int k = 0; k < LMS_NSTAGES; ++k) ms[k] = sum[k];
  return st != 0 ? st : count;
}

}  // namespace lms_host
