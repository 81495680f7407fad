// Optional per-launch timing, switched on by the environment variable
// LBM_TRACE=1 when a lattice is created.
//
// Each traced launch is bracketed by two HIP events recorded on the stream
// it is launched on, so the interval is the launch's own run time (from the
// moment its stream reaches it). Event pairs are resolved in batches (the
// host waits for the batch's last events), summed per label, and printed to
// stderr when the lattice is destroyed: calls, total, mean, minimum and
// maximum per label. Off (the default), every call here is a branch on a
// bool: no events, no synchronisation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

namespace lbm {

class Tracer {
 public:
  Tracer() {
    const char* v = std::getenv("LBM_TRACE");
    on_ = v != nullptr && std::strcmp(v, "1") == 0;
  }
  ~Tracer() {
    flush();
    for (hipEvent_t e : pool_) (void)hipEventDestroy(e);
  }
  Tracer(const Tracer&) = delete;
  Tracer& operator=(const Tracer&) = delete;

  bool on() const { return on_; }

  // Starts a record of `label` (a string that outlives the tracer: a literal,
  // or "name|" joined to __PRETTY_FUNCTION__ by LBM_TRACE_LABEL); tag >= 0 is
  // appended as a level index.
  void begin(hipStream_t s, const char* label, int tag = -1) {
    if (!on_) return;
    Rec r{label, tag, take(), take(), s};
    if (!r.a || !r.b || hipEventRecord(r.a, s) != hipSuccess) {
      give(r.a);
      give(r.b);
      return;
    }
    open_.push_back(r);
  }

  // Ends the most recent open record.
  void end() {
    if (!on_ || open_.empty()) return;
    Rec r = open_.back();
    open_.pop_back();
    if (hipEventRecord(r.b, r.s) != hipSuccess) {
      give(r.a);
      give(r.b);
      return;
    }
    done_.push_back(r);
    if (done_.size() >= 1024) flush();
  }

  // Resolves every finished record into the per-label sums.
  void flush() {
    for (Rec& r : done_) {
      float ms = 0.0f;
      if (hipEventSynchronize(r.b) == hipSuccess &&
          hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
        std::string key = short_label(r.label);
        if (r.tag >= 0) key += " [level " + std::to_string(r.tag) + "]";
        Stat& st = stats_[key];
        st.n += 1;
        st.total += ms;
        if (ms < st.min) st.min = ms;
        if (ms > st.max) st.max = ms;
      }
      give(r.a);
      give(r.b);
    }
    done_.clear();
  }

  // Prints the summary (what names the lattice) to stderr.
  void report(const char* what) {
    if (!on_) return;
    flush();
    std::fprintf(stderr, "lbm trace (%s): %zu labels\n", what, stats_.size());
    for (const auto& kv : stats_) {
      const Stat& st = kv.second;
      std::fprintf(stderr,
                   "lbm trace: %8lld calls %12.3f ms total %10.2f us mean %10.2f us min "
                   "%10.2f us max  %s\n",
                   st.n, st.total, 1e3 * st.total / (double)st.n, 1e3 * st.min, 1e3 * st.max,
                   kv.first.c_str());
    }
  }

 private:
  struct Rec {
    const char* label;
    int tag;
    hipEvent_t a, b;
    hipStream_t s;
  };
  struct Stat {
    long long n = 0;
    double total = 0.0, min = 1e30, max = 0.0;
  };

  hipEvent_t take() {
    if (!pool_.empty()) {
      hipEvent_t e = pool_.back();
      pool_.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void give(hipEvent_t e) {
    if (e) pool_.push_back(e);
  }
  // A label "name|signature": the name followed by the template arguments
  // that close the signature (a __PRETTY_FUNCTION__ string ends in
  // "[KIND = 2, S = float, ...]"); other labels unchanged.
  static std::string short_label(const char* s) {
    const char* bar = std::strchr(s, '|');
    if (!bar) return s;
    std::string name(s, (size_t)(bar - s));
    const char* w = std::strrchr(bar, '[');
    return w ? name + " " + std::string(w) : name;
  }

  bool on_ = false;
  std::vector<Rec> open_, done_;
  std::vector<hipEvent_t> pool_;
  std::map<std::string, Stat> stats_;
};

// A persistent "name|signature" label for the template instance that calls
// it (the instance's own static string).
#define LBM_TRACE_LABEL(name)                                       \
  ([](const char* pf) -> const char* {                              \
    static const std::string l = std::string(name) + "|" + pf;      \
    return l.c_str();                                               \
  }(__PRETTY_FUNCTION__))

// Records the launches of one scope (no-op when tracing is off).
class TraceScope {
 public:
  TraceScope(Tracer* t, hipStream_t s, const char* label, int tag = -1) : t_(t) {
    if (t_ && t_->on()) t_->begin(s, label, tag);
  }
  ~TraceScope() {
    if (t_ && t_->on()) t_->end();
  }
  TraceScope(const TraceScope&) = delete;
  TraceScope& operator=(const TraceScope&) = delete;

 private:
  Tracer* t_;
};

}  // namespace lbm
