// Capture of a fixed number of method steps into a HIP graph, replayed while the step inputs
// (bubble constants, bubble buffers, ping-pong parities) stay the same. The graph holds kernel
// launches only (buffers are cleared by fill kernels, never by memset nodes).
#pragma once

#include <hip/hip_runtime.h>
#include <string.h>

#include "../../include/lbm.h"

namespace lbm {

struct GraphKey {
  bubble_params p;
  bubble_soa s;
  int32_t nb, cur, flag, steps;
  uint32_t mode;  // the rest of the host step state and the launch configuration
  bool valid;

  static GraphKey of(const bubble_params* p, const bubble_soa* s, int32_t nb, int cur, int flag,
                     int steps, uint32_t mode) {
    GraphKey k;
    memset(&k, 0, sizeof(k));
    if (p) memcpy(&k.p, p, sizeof(*p));
    if (s) memcpy(&k.s, s, sizeof(*s));
    k.nb = nb;
    k.cur = cur;
    k.flag = flag;
    k.steps = steps;
    k.mode = mode;
    k.valid = true;
    return k;
  }
  bool same(const GraphKey& o) const {
    return valid && o.valid && memcmp(&p, &o.p, sizeof(p)) == 0 &&
           memcmp(&s, &o.s, sizeof(s)) == 0 && nb == o.nb && cur == o.cur && flag == o.flag &&
           steps == o.steps && mode == o.mode;
  }
};

class StepGraph {
 public:
  StepGraph() { memset(&key_, 0, sizeof(key_)); }
  ~StepGraph() { reset(); }
  StepGraph(const StepGraph&) = delete;
  StepGraph& operator=(const StepGraph&) = delete;

  void reset() {
    if (exec_) (void)hipGraphExecDestroy(exec_);
    exec_ = nullptr;
    key_.valid = false;
  }

  // Capture `enqueue` on stream s unless a graph for the same key exists.
  template <class F>
  hipError_t ensure(const GraphKey& key, hipStream_t s, F&& enqueue, bool* captured) {
    *captured = false;
    if (exec_ && key_.same(key)) return hipSuccess;
    reset();
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t ee = enqueue();
    e = hipStreamEndCapture(s, &g);
    if (ee != hipSuccess) {
      if (e == hipSuccess && g) (void)hipGraphDestroy(g);
      return ee;
    }
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&exec_, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      exec_ = nullptr;
      return e;
    }
    key_ = key;
    *captured = true;
    return hipSuccess;
  }

  hipError_t launch(hipStream_t s) { return hipGraphLaunch(exec_, s); }
  bool holds(const GraphKey& key) const { return exec_ && key_.same(key); }

 private:
  hipGraphExec_t exec_ = nullptr;
  GraphKey key_;
};

// A few captured graphs, each with the host step state its replay leaves behind (Post); a new
// key replaces the least recently used one.
template <class Post, int N = 2>
class GraphCache {
 public:
  void reset() {
    for (Slot& s : slot_) s.g.reset();
  }
  template <class F>
  hipError_t ensure(const GraphKey& key, hipStream_t s, F&& enqueue, bool* captured) {
    int k = -1;
    for (int i = 0; i < N; ++i)
      if (slot_[i].g.holds(key)) k = i;
    if (k < 0) {
      k = 0;
      for (int i = 1; i < N; ++i)
        if (slot_[i].used < slot_[k].used) k = i;
    }
    cur_ = k;
    slot_[k].used = ++clock_;
    return slot_[k].g.ensure(key, s, static_cast<F&&>(enqueue), captured);
  }
  // the graph of the last ensure()
  hipError_t launch(hipStream_t s) { return slot_[cur_].g.launch(s); }
  Post& post() { return slot_[cur_].post; }

 private:
  struct Slot {
    StepGraph g;
    Post post{};
    unsigned long long used = 0;
  };
  Slot slot_[N];
  int cur_ = 0;
  unsigned long long clock_ = 0;
};

}  // namespace lbm
