// hipGraph replay cache: a step loop (or a reverse segment) is captured once on a private stream
// and replayed on the caller's stream by every later call with identical arguments, so the host
// issues one launch per call instead of two per step.
#include <map>
#include <mutex>

#include "ts_graph.h"

namespace ts {
namespace {

struct GraphEntry {
  hipGraph_t graph;
  hipGraphExec_t exec;
  uint64_t stamp;
};

std::mutex g_mu;
std::map<std::string, GraphEntry> g_cache;
uint64_t g_clock = 0;
std::map<int, hipStream_t> g_capture_stream;
constexpr size_t kMaxGraphs = 16;

void destroy_entry(GraphEntry &e) {
  (void)hipGraphExecDestroy(e.exec);
  (void)hipGraphDestroy(e.graph);
}

int capture_stream(int device, hipStream_t *out) {
  auto it = g_capture_stream.find(device);
  if (it != g_capture_stream.end()) {
    *out = it->second;
    return TS_OK;
  }
  hipStream_t s;
  TS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  g_capture_stream[device] = s;
  *out = s;
  return TS_OK;
}

}  // namespace

int run_graph_cached(bool use_graph, std::string key, hipStream_t st, const std::function<int(hipStream_t)> &seq) {
  if (!use_graph) return seq(st);
  int device = 0;
  TS_HIP(hipGetDevice(&device));
  key_add(key, device);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_cache.find(key);
  if (it == g_cache.end()) {
    hipStream_t cap;
    int rc = capture_stream(device, &cap);
    if (rc != TS_OK) return rc;
    TS_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    rc = seq(cap);
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(cap, &graph);
    if (rc != TS_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (ce != hipSuccess || graph == nullptr) return TS_E_HIP;
    hipGraphExec_t exec;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return TS_E_HIP;
    }
    if (g_cache.size() >= kMaxGraphs) {
      auto old = g_cache.begin();
      for (auto jt = g_cache.begin(); jt != g_cache.end(); ++jt)
        if (jt->second.stamp < old->second.stamp) old = jt;
      (void)hipDeviceSynchronize();  // the evicted graph may still be running
      destroy_entry(old->second);
      g_cache.erase(old);
    }
    it = g_cache.emplace(key, GraphEntry{graph, exec, 0}).first;
  }
  it->second.stamp = ++g_clock;
  TS_HIP(hipGraphLaunch(it->second.exec, st));
  return TS_OK;
}

void release_graphs() {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_cache.empty()) (void)hipDeviceSynchronize();
  for (auto &kv : g_cache) destroy_entry(kv.second);
  g_cache.clear();
}

}  // namespace ts

extern "C" void ts_release_graphs(void) { ts::release_graphs(); }
