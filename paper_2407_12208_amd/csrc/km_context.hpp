// km_context.hpp -- host-side library state: the context (device, workspace
// arena, descriptor uploader) and the planning helpers shared by the C ABI
// entry points and the server.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/kmeans.h"
#include "km_internal.hpp"

namespace km {

// Device bump allocator, reset per call; grows (after draining the device)
// when a call needs more than it holds.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  static size_t align(size_t x) { return (x + 255) & ~size_t(255); }
  hipError_t ensure(size_t bytes) {
    if (bytes <= cap) return hipSuccess;
    if (base) {
      hipError_t e = hipDeviceSynchronize();
      if (e != hipSuccess) return e;
      (void)hipFree(base);
      base = nullptr;
      cap = 0;
    }
    size_t c = bytes + bytes / 4 + (1 << 20);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&base), c);
    if (e != hipSuccess) {
      base = nullptr;
      return e;
    }
    cap = c;
    return hipSuccess;
  }
  void reset() { used = 0; }
  template <class T>
  T* take(size_t count) {
    T* p = reinterpret_cast<T*>(base + used);
    used += align(count * sizeof(T));
    return p;
  }
};

// Size accumulator used to plan an Arena before carving it.
struct Plan {
  size_t bytes = 0;
  template <class T>
  void add(size_t count) { bytes += Arena::align(count * sizeof(T)); }
};

// Pinned host ring + device ring for small descriptor uploads that are
// ordered on the caller's stream.
struct Uploader {
  char* host = nullptr;
  char* dev = nullptr;
  size_t cap = 0;
  size_t head = 0;
  hipError_t init(size_t bytes);
  void destroy();
  // Copies `bytes` from src into the ring and enqueues the H2D copy on st;
  // returns the device address (nullptr on failure).
  void* put(const void* src, size_t bytes, hipStream_t st);
};

// Persisted choices of the sweep-length tuner (km_tune.cpp).
struct TuneCache {
  struct Entry {
    int gpw;
    std::vector<float> ms;
  };
  std::mutex mu;
  std::map<std::string, Entry> entries;
  std::string path;
  static std::string key(int low, int high, bool fallback, int xd, int k_pad, int64_t points);
  bool lookup(const std::string& k, int* gpw);
  void store(const std::string& k, int gpw, const std::vector<float>& ms);
  int32_t set_path(const char* p);
  std::string dump();

 private:
  void save_locked();
};

struct km_context_impl {
  int device = 0;
  int num_cu = 0;
  Arena arena;
  Uploader up;
  char* static_scratch = nullptr; // device address of this device's fixed
                                  // workspace array (kmeans_assign_static)
  double* h_scalar = nullptr;     // pinned: shift read-back
  KResult* h_result = nullptr;    // pinned: result read-back (up to kMaxResults)
  static constexpr int kMaxResults = 4096;
  // Workspace ordering across streams: every call that uses the arena or
  // the result records waits (on its own stream) for the last such call's
  // work, whatever stream that call used, and records its own end here.
  hipEvent_t ws_event = nullptr;
  hipStream_t ws_stream = nullptr;
  bool ws_valid = false;
  TuneCache tune;
  // kernel timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;  // pairs: [2i] start, [2i+1] stop
  int ev_used = 0;                  // pairs recorded since enable
  hipEvent_t timing_event(int i);
};

// Scope of one entry point's use of the context workspace on stream st.
struct WorkspaceUse {
  km_context_impl* c;
  hipStream_t st;
  hipError_t err = hipSuccess;
  WorkspaceUse(km_context_impl* ctx, hipStream_t s) : c(ctx), st(s) {
    if (c->ws_valid && c->ws_stream != st) err = hipStreamWaitEvent(st, c->ws_event, 0);
  }
  ~WorkspaceUse() {
    if (c->ws_event && hipEventRecord(c->ws_event, st) == hipSuccess) {
      c->ws_stream = st;
      c->ws_valid = true;
    }
  }
};

// Threshold alpha for (prec, d): -1 = no fallback, +inf = always correct.
double alpha_for(const km_precision& p, int d);
km_precision precision_or_default(const km_precision* p);
int32_t validate_precision(const km_precision& p);
int32_t status_from_bits(int bits);

// How a problem's assignment pass is executed.
enum class Route { Mfma, MfmaNoFallback, Direct64Exact, Direct64All };
struct AssignPlan {
  Route route;
  int low;
  int high;         // correction precision (KM_HIGH_*)
  int DP;
  int k_pad;
  int xd;           // > 0: the small-problem kernel with this row capacity
  int gpw;          // its 32-point groups per wave (may follow a batched launch)
  int gpw_own;      // groups per wave from the problem alone: passes whose
  int nwg_own;      // SSE comes from per-workgroup partials use these, so the
                    // partition (and the FP64 sum) never depends on the batch
  int nwg;          // workgroups of the assignment kernel
  int nwg_pair;     // workgroups of the materialising kernel
  float alpha_f;    // alpha as applied (FP32)
  float oma;        // 1 - alpha (FP32)
  double alpha_used;
  bool record = false;  // the large kernel writes the flagged pairs (diagnostics)
};
AssignPlan plan_assign(const km_precision& p, int64_t n, int d, int k);
void set_small_sweep(AssignPlan& a, int64_t n, int64_t launch_points);
size_t cq_elem_bytes(int low);

// Launch helpers working on arrays of problems that share one AssignPlan
// shape (same route, low format and DP).
hipError_t run_prep(km_context_impl* ctx, int low, const std::vector<PrepProb>& probs,
                    const std::vector<int>& kpads, hipStream_t st);
hipError_t run_assign(km_context_impl* ctx, const AssignPlan& shape, int mode,
                      const std::vector<AssignProb>& probs, const std::vector<int>& nwgs, hipStream_t st);
hipError_t run_reduce(km_context_impl* ctx, const std::vector<ReduceProb>& probs, hipStream_t st);
hipError_t run_update(km_context_impl* ctx, const std::vector<UpdateProb>& probs, hipStream_t st);

// Reads the result records at src (device) into out (host): one gather
// launch and one copy per kMaxResults records, then waits for st.  Uses the
// context's arena.
hipError_t read_results(km_context_impl* ctx, const std::vector<const KResult*>& src, KResult* out,
                        hipStream_t st);

// Workspace sizes of one problem's centre update.
void plan_update(Plan& pl, int64_t n, int d, int k);
UpdateProb carve_update(Arena& a, int64_t n, int d, int k);

// Everything one assignment pass of one problem needs on the device.
struct PassBufs {
  void* Cq;
  float* cinit;
  float* ca;
  double* sse_part;
  unsigned long long* corr_part;
  int* status;
  KResult* result;
};
void plan_pass(Plan& pl, const AssignPlan& a);
PassBufs carve_pass(Arena& ar, const AssignPlan& a);
bool uses_prep(const AssignPlan& a);
int32_t check_shape(int64_t n, int32_t d, int32_t k, const km_precision& p);

// One problem inside a batched solve (device pointers in *prob).
struct BatchState {
  km_problem* prob;
  AssignPlan plan;
  PassBufs bufs;
  UpdateProb upd;
  float* cur;
  float* nxt;
  int32_t it = 0;
  bool done = false;  // update rounds finished (converged or max_iter)
};
// One assignment pass for every listed problem (final = write mindist).
hipError_t enqueue_batch_pass(km_context_impl* ctx, std::vector<BatchState*>& list, bool final_pass,
                              hipStream_t st);
// One Lloyd round (assignment pass + centre update) for every listed problem.
hipError_t enqueue_batch_round(km_context_impl* ctx, std::vector<BatchState*>& act, hipStream_t st);

}  // namespace km

struct km_context : km::km_context_impl {};
