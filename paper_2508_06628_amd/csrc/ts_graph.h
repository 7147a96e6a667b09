// Capture-and-replay cache of hipGraphs keyed by the bytes of a call's arguments.
#pragma once

#include <functional>
#include <string>

#include "ts_internal.h"

namespace ts {

// Append the bytes of v to a key.
template <typename V>
inline void key_add(std::string &key, const V &v) {
  key.append(reinterpret_cast<const char *>(&v), sizeof(V));
}

// With use_graph, look up `key` (device-qualified) and replay its graph on `st`, capturing
// `seq` on a private stream into a new graph on a miss; otherwise run `seq` on `st` directly.
int run_graph_cached(bool use_graph, std::string key, hipStream_t st, const std::function<int(hipStream_t)> &seq);

void release_graphs();

}  // namespace ts
