// km_api.hip -- the C ABI declared in include/kmeans.h: argument checks,
// workspace planning and the launch sequences of one assignment pass, one
// centre update, Lloyd's loop and batched solves.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <climits>
#include <new>
#include <map>
#include <vector>

#include <cstddef>

#include "km_context.hpp"

namespace km {

// ---------------------------------------------------------------------------
// Uploader
// ---------------------------------------------------------------------------
hipError_t Uploader::init(size_t bytes) {
  hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&host), bytes, hipHostMallocDefault);
  if (e != hipSuccess) return e;
  e = hipMalloc(reinterpret_cast<void**>(&dev), bytes);
  if (e != hipSuccess) {
    (void)hipHostFree(host);
    host = nullptr;
    return e;
  }
  cap = bytes;
  head = 0;
  return hipSuccess;
}

void Uploader::destroy() {
  if (host) (void)hipHostFree(host);
  if (dev) (void)hipFree(dev);
  host = dev = nullptr;
  cap = head = 0;
}

void* Uploader::put(const void* src, size_t bytes, hipStream_t st) {
  size_t need = (bytes + 255) & ~size_t(255);
  if (need > cap) return nullptr;
  if (head + need > cap) {
    // wrap: earlier copies out of this ring must have completed before the
    // host overwrites their source bytes
    if (hipDeviceSynchronize() != hipSuccess) return nullptr;
    head = 0;
  }
  memcpy(host + head, src, bytes);
  void* d = dev + head;
  if (hipMemcpyAsync(d, host + head, bytes, hipMemcpyHostToDevice, st) != hipSuccess) return nullptr;
  head += need;
  return d;
}

// ---------------------------------------------------------------------------
// Precision and planning
// ---------------------------------------------------------------------------
static double unit_roundoff_low(int low) {
  switch (low) {
    case kLowFP16: return ldexp(1.0, -11);
    case kLowBF16: return ldexp(1.0, -8);
    case kLowFP32: return ldexp(1.0, -24);
  }
  return 0.0;
}

km_precision precision_or_default(const km_precision* p) {
  if (p) return *p;
  km_precision q;
  q.low = KM_LOW_FP16;
  q.alpha_mode = KM_ALPHA_PAPER_EQ;
  q.rho = 5.0;
  q.alpha = 0.0;
  q.high = KM_HIGH_FP64;
  q.reserved = 0;
  return q;
}

int32_t validate_precision(const km_precision& p) {
  if (p.low < KM_LOW_FP16 || p.low > KM_EXACT64) return KM_ERR_ARG;
  if (p.high < KM_HIGH_FP64 || p.high > KM_HIGH_LOW) return KM_ERR_ARG;
  if (p.low == KM_EXACT64) return p.high == KM_HIGH_FP64 ? KM_OK : KM_ERR_ARG;
  if (p.alpha_mode < KM_ALPHA_PAPER_EQ || p.alpha_mode > KM_ALPHA_HW) return KM_ERR_ARG;
  if ((p.alpha_mode == KM_ALPHA_PAPER_EQ || p.alpha_mode == KM_ALPHA_PAPER_ALG ||
       p.alpha_mode == KM_ALPHA_HW) && !(p.rho > 2.0))
    return KM_ERR_ARG;  // the relative bound needs rho~ > 2 (Section 4.3)
  if (p.alpha_mode == KM_ALPHA_EXPLICIT && !(p.alpha >= 0.0)) return KM_ERR_ARG;
  return KM_OK;
}

double alpha_for(const km_precision& p, int d) {
  if (p.low == KM_EXACT64 || p.alpha_mode == KM_ALPHA_NONE) return -1.0;
  if (p.alpha_mode == KM_ALPHA_EXPLICIT) return p.alpha;
  if (p.alpha_mode == KM_ALPHA_HW) {
    // arithmetic error of the expanded formula with FP32 accumulation
    // (rounding unit taken as 2^-23, room for any accumulator rounding)
    // plus the conversion error of the rounded inputs
    const double u32 = ldexp(1.0, -23);
    const double m32 = (double)(d + 2) * u32;
    if (!(m32 < 1.0)) return INFINITY;
    const double ul = unit_roundoff_low(p.low);
    const double conv = 2.0 * (2.0 * ul + ul * ul) * (1.0 + ul) * (1.0 + ul);
    return p.rho * (2.0 * m32 / (1.0 - m32) + conv);
  }
  const double mu = (double)(d + 2) * unit_roundoff_low(p.low);
  if (!(mu < 1.0)) return INFINITY;  // gamma undefined: correct every pair
  const double g = mu / (1.0 - mu);
  return p.alpha_mode == KM_ALPHA_PAPER_EQ ? 2.0 * p.rho * g : p.rho * g;
}

int32_t status_from_bits(int bits) {
  if (bits & kStatusNonFinite) return KM_ERR_NONFINITE;
  if (bits & kStatusRange) return KM_ERR_RANGE;
  if (bits & kStatusBadLabel) return KM_ERR_ARG;  // label out of range in an update
  if (bits & kStatusSync) return KM_ERR_DEVICE;   // persistent round kernel gave up a wait
  return KM_OK;
}

size_t cq_elem_bytes(int low) { return low == kLowFP32 ? 4 : 2; }

// Above this threshold every pair fails the test (d^ <= 2 S always), so the
// pass is run by the FP64 direct kernel instead of a fully divergent sweep.
static constexpr double kDenseAlpha = 2.5;

// Groups of 32 points per wave of the small-problem kernel: the centre
// set-up of a workgroup is amortised over more points once the launch
// (`launch_points` over all of its problems) still has >= 4096 workgroups.
void set_small_sweep(AssignPlan& a, int64_t n, int64_t launch_points) {
  if (a.xd <= 0) return;
  const int64_t q = launch_points / ((int64_t)kSmallWaves * 32 * 4096);
  a.gpw = q >= 8 ? 8 : q >= 4 ? 4 : q >= 2 ? 2 : 1;
  const int64_t ppw = (int64_t)kSmallWaves * 32 * a.gpw;
  a.nwg = (int)((n + ppw - 1) / ppw);
}

AssignPlan plan_assign(const km_precision& p, int64_t n, int d, int k) {
  AssignPlan a{};
  a.low = p.low;
  a.high = p.high;
  a.DP = padded_dim(d);
  a.k_pad = (k + 31) & ~31;
  const double alpha = alpha_for(p, d);
  a.alpha_used = alpha;
  if (p.low == KM_EXACT64) {
    a.route = Route::Direct64Exact;
  } else if (alpha < 0.0) {
    a.route = Route::MfmaNoFallback;
  } else if (!(alpha < kDenseAlpha)) {
    a.route = Route::Direct64All;
  } else {
    a.route = Route::Mfma;
  }
  a.alpha_f = alpha < 0.0 ? 0.0f : (float)std::min(alpha, 1e30);
  a.oma = 1.0f - a.alpha_f;
  if (a.route == Route::Mfma) a.alpha_used = (double)a.alpha_f;
  if (a.route == Route::Direct64Exact || a.route == Route::Direct64All) {
    a.nwg = (int)((n + kDirectPointsPerWg - 1) / kDirectPointsPerWg);
    a.nwg_pair = a.nwg;
  } else {
    a.nwg = (int)((n + assign_points_per_wg(p.low, a.DP) - 1) / assign_points_per_wg(p.low, a.DP));
    a.nwg_pair = (int)((n + mfma_points_per_wg(p.low, a.DP) - 1) / mfma_points_per_wg(p.low, a.DP));
    // few coordinates and centres: the pass is bound by memory and the
    // vector epilogue, and a lighter kernel with resident centres serves it
    if ((p.low == KM_LOW_FP16 || p.low == KM_LOW_BF16) && d <= kSmallMaxD && a.k_pad <= kSmallMaxK) {
      a.xd = small_xd(d);
      set_small_sweep(a, n, n);
    }
  }
  a.gpw_own = a.gpw;
  a.nwg_own = a.nwg;
  return a;
}

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------
// Several host arrays gathered into one upload (one H2D copy per call).
struct Pack {
  std::vector<char> buf;
  size_t add(const void* p, size_t n) {
    const size_t off = (buf.size() + 255) & ~size_t(255);
    buf.resize(off + n);
    memcpy(buf.data() + off, p, n);
    return off;
  }
  char* upload(km_context_impl* ctx, hipStream_t st) {
    return static_cast<char*>(ctx->up.put(buf.data(), buf.size(), st));
  }
};

// One clearing launch for the status word and the result record that follow
// it in the arena.
static hipError_t zero_status_result(int* status, KResult* result, hipStream_t st) {
  const size_t span = (size_t)(reinterpret_cast<char*>(result + 1) - reinterpret_cast<char*>(status));
  return launch_zero_words(status, span, st);
}

static std::vector<int32_t> prefix(const std::vector<int>& counts) {
  std::vector<int32_t> s(counts.size() + 1, 0);
  for (size_t i = 0; i < counts.size(); ++i) s[i + 1] = s[i] + counts[i];
  return s;
}

hipError_t run_prep(km_context_impl* ctx, int low, const std::vector<PrepProb>& probs,
                    const std::vector<int>& kpads, hipStream_t st) {
  std::vector<int> wgs(kpads.size());
  for (size_t i = 0; i < kpads.size(); ++i) wgs[i] = (kpads[i] + 3) / 4;  // one wave per centre
  std::vector<int32_t> pre = prefix(wgs);
  Pack pk;
  const size_t op = pk.add(probs.data(), probs.size() * sizeof(PrepProb));
  const size_t os = pk.add(pre.data(), pre.size() * sizeof(int32_t));
  char* d = pk.upload(ctx, st);
  if (!d) return hipErrorOutOfMemory;
  return launch_prep(low, (const PrepProb*)(d + op), (const int32_t*)(d + os), (int)probs.size(), pre.back(), st);
}

hipEvent_t km_context_impl::timing_event(int i) {
  while ((int)ev_pool.size() <= i) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ev_pool.push_back(e);
  }
  return ev_pool[i];
}

static hipError_t run_assign_dev(km_context_impl* ctx, const AssignPlan& shape, int mode, const void* dp,
                                 const void* ds, int nprob, int total_wg, hipStream_t st);

hipError_t run_assign(km_context_impl* ctx, const AssignPlan& shape, int mode,
                      const std::vector<AssignProb>& probs, const std::vector<int>& nwgs, hipStream_t st) {
  std::vector<int32_t> pre = prefix(nwgs);
  if (pre.back() == 0) return hipSuccess;
  Pack pk;
  const size_t op = pk.add(probs.data(), probs.size() * sizeof(AssignProb));
  const size_t os = pk.add(pre.data(), pre.size() * sizeof(int32_t));
  char* d = pk.upload(ctx, st);
  if (!d) return hipErrorOutOfMemory;
  return run_assign_dev(ctx, shape, mode, d + op, d + os, (int)probs.size(), pre.back(), st);
}

// Arithmetic of the direct-formula kernel: FP64 unless every pair of a
// mixed pass is corrected in another precision.
static int direct_arith(const AssignPlan& a) {
  if (a.route != Route::Direct64All || a.high == KM_HIGH_FP64) return 0;
  if (a.high == KM_HIGH_FP32 || a.low == KM_LOW_FP32) return 1;
  return a.low == KM_LOW_FP16 ? 2 : 3;
}

// The assignment launch of problems whose descriptors are already on the
// device, bracketed by timing events when timing is enabled.
static hipError_t run_assign_dev(km_context_impl* ctx, const AssignPlan& shape, int mode, const void* dp,
                                 const void* ds, int nprob, int total_wg, hipStream_t st) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ctx->timing) {
    e0 = ctx->timing_event(2 * ctx->ev_used);
    e1 = ctx->timing_event(2 * ctx->ev_used + 1);
    if (!e0 || !e1) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(e0, st);
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipErrorInvalidValue;
  switch (shape.route) {
    case Route::Mfma:
    case Route::MfmaNoFallback:
      if (mode == 0 && shape.xd > 0) {
        e = launch_assign_small(shape.low, shape.xd, shape.route == Route::Mfma, (const AssignProb*)dp,
                                (const int32_t*)ds, nprob, total_wg, st);
        break;
      }
      e = launch_assign_mfma(shape.low, shape.DP, mode == 0 && shape.record ? 2 : mode, shape.route == Route::Mfma,
                             (const AssignProb*)dp,
                             (const int32_t*)ds, nprob, total_wg, st);
      break;
    case Route::Direct64Exact:
    case Route::Direct64All:
      e = launch_assign_direct64(shape.route == Route::Direct64Exact, direct_arith(shape), mode,
                                 (const AssignProb*)dp, (const int32_t*)ds, nprob, total_wg, st);
      break;
  }
  if (e == hipSuccess && ctx->timing) {
    e = hipEventRecord(e1, st);
    ctx->ev_used += 1;
  }
  return e;
}

hipError_t run_reduce(km_context_impl* ctx, const std::vector<ReduceProb>& probs, hipStream_t st) {
  void* dp = ctx->up.put(probs.data(), probs.size() * sizeof(ReduceProb), st);
  if (!dp) return hipErrorOutOfMemory;
  return launch_reduce_parts((const ReduceProb*)dp, (int)probs.size(), st);
}

hipError_t read_results(km_context_impl* ctx, const std::vector<const KResult*>& src, KResult* out,
                        hipStream_t st) {
  const int cap = km_context_impl::kMaxResults;
  hipError_t e = ctx->arena.ensure(sizeof(KResult) * (size_t)cap);
  if (e != hipSuccess) return e;
  ctx->arena.reset();
  KResult* dst = ctx->arena.take<KResult>((size_t)cap);
  for (size_t s0 = 0; s0 < src.size(); s0 += (size_t)cap) {
    const int cnt = (int)std::min(src.size() - s0, (size_t)cap);
    void* dsrc = ctx->up.put(src.data() + s0, sizeof(const KResult*) * (size_t)cnt, st);
    if (!dsrc) return hipErrorOutOfMemory;
    e = launch_gather_results((const KResult* const*)dsrc, cnt, dst, st);
    if (e == hipSuccess) e = hipMemcpyAsync(ctx->h_result, dst, sizeof(KResult) * (size_t)cnt, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    memcpy(out + s0, ctx->h_result, sizeof(KResult) * (size_t)cnt);
  }
  return hipSuccess;
}

void plan_update(Plan& pl, int64_t n, int d, int k) {
  const OwnShape sh = own_shape(d, k);
  if (sh.owners > 0) {
    const int64_t cs = own_chunk(sh, own_iters(n, sh));
    const int64_t nch = (n + cs - 1) / cs;
    pl.add<double>((size_t)nch * k * d);  // chunk partials
    pl.add<int32_t>((size_t)nch * k);     // chunk counts
    pl.add<double>((size_t)nch);          // chunk SSE partials
    pl.add<double>((size_t)k);            // shift2
    return;
  }
  const int ntiles = (int)((n + kUpdTile - 1) / kUpdTile);
  pl.add<int32_t>((size_t)k * ntiles);  // hist
  pl.add<int32_t>((size_t)k * ntiles);  // offs
  pl.add<int32_t>((size_t)n);           // perm
  pl.add<int32_t>((size_t)k + 1);       // cstart
  pl.add<int32_t>((size_t)k + 1);       // chunk_start
  pl.add<double>(((size_t)(n + kUpdChunk - 1) / kUpdChunk + k) * d);  // chunk sums
  pl.add<double>((size_t)(n + kUpdChunk - 1) / kUpdChunk + k);        // chunk SSE partials
  pl.add<double>((size_t)k);            // shift2
}

UpdateProb carve_update(Arena& a, int64_t n, int d, int k) {
  UpdateProb u{};
  const OwnShape sh = own_shape(d, k);
  if (sh.owners > 0) {
    const int iters = own_iters(n, sh);
    const int64_t cs = own_chunk(sh, iters);
    const int64_t nch = (n + cs - 1) / cs;
    u.iters = iters;
    u.pacc = a.take<double>((size_t)nch * k * d);
    u.pcnt = a.take<int32_t>((size_t)nch * k);
    u.psse = a.take<double>((size_t)nch);
    u.shift2 = a.take<double>((size_t)k);
    u.owners = sh.owners;
    u.lp = sh.lp;
    u.nc = sh.nc;
    u.nchunk = (int)nch;
    u.n = n;
    u.d = d;
    u.k = k;
    return u;
  }
  const int ntiles = (int)((n + kUpdTile - 1) / kUpdTile);
  u.hist = a.take<int32_t>((size_t)k * ntiles);
  u.offs = a.take<int32_t>((size_t)k * ntiles);
  u.perm = a.take<int32_t>((size_t)n);
  u.cstart = a.take<int32_t>((size_t)k + 1);
  u.chunk_start = a.take<int32_t>((size_t)k + 1);
  u.chunk_sum = a.take<double>(((size_t)(n + kUpdChunk - 1) / kUpdChunk + k) * d);
  u.sse_chunk = a.take<double>((size_t)(n + kUpdChunk - 1) / kUpdChunk + k);
  u.shift2 = a.take<double>((size_t)k);
  u.sse_out = nullptr;
  u.n = n;
  u.d = d;
  u.k = k;
  u.ntiles = ntiles;
  u.chunk = upd_chunk(d);
  return u;
}

hipError_t run_update_sort(km_context_impl* ctx, const std::vector<UpdateProb>& probs, hipStream_t st);

// Owner-path problems: part launches grouped by coordinates per lane, SSE
// request and the workgroups per compute unit their LDS allows (a launch
// sizes its LDS for its largest problem), then one finalize and one shift
// launch over all of them.  The grouping never changes a problem's result.
static hipError_t run_update_own(km_context_impl* ctx, const std::vector<UpdateProb>& probs, hipStream_t st) {
  constexpr int kLdsPerCu = 160 * 1024;
  constexpr int kFit = 3;  // 1, 2, 3 or more workgroups per compute unit
  std::vector<UpdateProb> grp[2][2][kFit];
  for (const UpdateProb& u : probs) {
    const bool sse = u.sse_out != nullptr;
    const int need = kOwnWaves * own_wave_bytes(u.owners, u.d, u.k) + (sse ? 4 * u.k * u.d : 0);
    const int fit = std::min(kFit, std::max(1, kLdsPerCu / need));
    grp[u.nc - 1][sse][fit - 1].push_back(u);
  }
  std::vector<UpdateProb> all;
  std::vector<std::pair<size_t, size_t>> ranges;  // (first, count) per part launch
  for (auto& a : grp)
    for (auto& b : a)
      for (auto& g : b)
        if (!g.empty()) {
          ranges.emplace_back(all.size(), g.size());
          all.insert(all.end(), g.begin(), g.end());
        }
  const int np = (int)all.size();
  std::vector<int> fin(np);
  for (int i = 0; i < np; ++i) {
    const int J = own_fin_clusters(all[i].d);
    fin[i] = (all[i].k + J - 1) / J;
  }
  Pack pk;
  const size_t op = pk.add(all.data(), all.size() * sizeof(UpdateProb));
  std::vector<size_t> oc;
  for (auto& r : ranges) {
    std::vector<int> ch(r.second);
    for (size_t i = 0; i < r.second; ++i) ch[i] = all[r.first + i].nchunk;
    std::vector<int32_t> pre = prefix(ch);
    oc.push_back(pk.add(pre.data(), pre.size() * sizeof(int32_t)));
  }
  std::vector<int32_t> pf = prefix(fin);
  const size_t of = pk.add(pf.data(), pf.size() * sizeof(int32_t));
  char* d = pk.upload(ctx, st);
  if (!d) return hipErrorOutOfMemory;
  const UpdateProb* dprobs = (const UpdateProb*)(d + op);
  hipError_t e = hipSuccess;
  for (size_t g = 0; g < ranges.size() && e == hipSuccess; ++g)
    e = launch_update_own_part(dprobs + ranges[g].first, all.data() + ranges[g].first, (int)ranges[g].second,
                               (const int32_t*)(d + oc[g]), st);
  if (e == hipSuccess) e = launch_update_own_fin(dprobs, all.data(), np, (const int32_t*)(d + of), st);
  return e;
}

hipError_t run_update(km_context_impl* ctx, const std::vector<UpdateProb>& probs, hipStream_t st) {
  std::vector<UpdateProb> sorted, own;
  for (const UpdateProb& u : probs) (u.owners > 0 ? own : sorted).push_back(u);
  hipError_t e = hipSuccess;
  if (!sorted.empty()) e = run_update_sort(ctx, sorted, st);
  if (e == hipSuccess && !own.empty()) e = run_update_own(ctx, own, st);
  return e;
}

hipError_t run_update_sort(km_context_impl* ctx, const std::vector<UpdateProb>& probs, hipStream_t st) {
  const int np = (int)probs.size();
  std::vector<int> tiles(np), cl(np), chunkwg(np), clwg(np), scatwg(np);
  for (int i = 0; i < np; ++i) {
    tiles[i] = probs[i].ntiles;
    cl[i] = probs[i].k;
    chunkwg[i] = (int)(((probs[i].n + probs[i].chunk - 1) / probs[i].chunk + probs[i].k + 3) / 4);
    clwg[i] = (probs[i].k + 3) / 4;
    scatwg[i] = (probs[i].ntiles + 3) / 4;
  }
  std::vector<int32_t> pre;
  for (auto* v : {&tiles, &cl, &chunkwg, &clwg, &scatwg}) {
    std::vector<int32_t> p = prefix(*v);
    pre.insert(pre.end(), p.begin(), p.end());
  }
  Pack pk;
  const size_t op = pk.add(probs.data(), probs.size() * sizeof(UpdateProb));
  const size_t os = pk.add(pre.data(), pre.size() * sizeof(int32_t));
  char* d = pk.upload(ctx, st);
  if (!d) return hipErrorOutOfMemory;
  return launch_update((const UpdateProb*)(d + op), probs.data(), np, (const int32_t*)(d + os), st);
}

}  // namespace km

using namespace km;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
#define KM_HIP(call)                         \
  do {                                       \
    hipError_t e_ = (call);                  \
    if (e_ != hipSuccess) {                  \
      (void)hipGetLastError();               \
      return e_ == hipErrorOutOfMemory ? KM_ERR_OOM : KM_ERR_DEVICE; \
    }                                        \
  } while (0)

extern "C" {

const char* kmeans_status_string(int32_t s) {
  switch (s) {
    case KM_OK: return "ok";
    case KM_PENDING: return "pending";
    case KM_ERR_ARG: return "invalid argument";
    case KM_ERR_RANGE: return "input overflows the low-precision format";
    case KM_ERR_NONFINITE: return "non-finite input";
    case KM_ERR_OOM: return "out of device memory or over the memory budget";
    case KM_ERR_DEVICE: return "HIP runtime error";
    case KM_ERR_NOTFOUND: return "unknown ticket";
    case KM_ERR_CANCELLED: return "cancelled";
    case KM_ERR_UNSUPPORTED: return "unsupported shape";
  }
  return "unknown status";
}

int32_t kmeans_alpha(const km_precision* prec, int32_t d, double* alpha_out) {
  if (!alpha_out || d < 1) return KM_ERR_ARG;
  km_precision p = precision_or_default(prec);
  int32_t v = validate_precision(p);
  if (v != KM_OK) return v;
  double a = alpha_for(p, d);
  if (p.low != KM_EXACT64 && a >= 0.0 && a < 2.5 && p.alpha_mode != KM_ALPHA_NONE) a = (double)(float)a;
  *alpha_out = a;
  return KM_OK;
}

// Fixed workspace of kmeans_assign_static: one copy per device, held for the
// life of the process.  Host code never uses this name as an address (on
// the host it is a stand-in, not device memory); it uses the device address
// that kmeans_context_create obtains with hipGetSymbolAddress, with the
// context's device current.
static __device__ __align__(256) char scratch[KM_STATIC_SCRATCH_BYTES];

int32_t kmeans_context_create(int32_t device, km_context** out) {
  if (!out) return KM_ERR_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return KM_ERR_DEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return KM_ERR_DEVICE;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return KM_ERR_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return KM_ERR_DEVICE;
  km_context* c = new (std::nothrow) km_context();
  if (!c) return KM_ERR_OOM;
  c->device = device;
  c->num_cu = prop.multiProcessorCount;
  void* sp = nullptr;
  if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || !sp) {
    delete c;
    return KM_ERR_DEVICE;
  }
  c->static_scratch = static_cast<char*>(sp);
  if (c->up.init(8u << 20) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&c->h_scalar), 64, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&c->h_result), sizeof(KResult) * km_context_impl::kMaxResults,
                    hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&c->ws_event, hipEventDisableTiming) != hipSuccess) {
    kmeans_context_destroy(c);
    return KM_ERR_OOM;
  }
  *out = c;
  return KM_OK;
}

int32_t kmeans_timing_enable(km_context* c, int32_t enable) {
  if (!c) return KM_ERR_ARG;
  c->timing = enable != 0;
  c->ev_used = 0;
  return KM_OK;
}

int32_t kmeans_timing_read(km_context* c, float* ms_out, int32_t max, int32_t* count) {
  if (!c || (!ms_out && max > 0) || max < 0) return KM_ERR_ARG;
  const int n = c->ev_used;
  for (int i = 0; i < n && i < max; ++i) {
    if (hipEventSynchronize(c->ev_pool[2 * i + 1]) != hipSuccess) return KM_ERR_DEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev_pool[2 * i], c->ev_pool[2 * i + 1]) != hipSuccess) return KM_ERR_DEVICE;
    ms_out[i] = ms;
  }
  if (count) *count = n;
  return KM_OK;
}

int32_t kmeans_context_destroy(km_context* c) {
  if (!c) return KM_ERR_ARG;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->ws_event) (void)hipEventDestroy(c->ws_event);
  c->up.destroy();
  if (c->arena.base) (void)hipFree(c->arena.base);
  if (c->h_scalar) (void)hipHostFree(c->h_scalar);
  if (c->h_result) (void)hipHostFree(c->h_result);
  delete c;
  return KM_OK;
}

}  // extern "C"

namespace km {

int32_t check_shape(int64_t n, int32_t d, int32_t k, const km_precision& p) {
  if (n < 1 || n > (int64_t)INT32_MAX - 1024 || d < 1 || k < 1 || k > 65536) return KM_ERR_ARG;
  if (p.low != KM_EXACT64) {
    const int DP = padded_dim(d);
    if (DP < 0) return KM_ERR_UNSUPPORTED;
    if (p.low == KM_LOW_FP32 && DP > 128) return KM_ERR_UNSUPPORTED;
  }
  return KM_OK;
}

void plan_pass(Plan& pl, const AssignPlan& a) {
  const int parts = std::max(std::max(a.nwg, a.nwg_own), a.nwg_pair);
  pl.add<char>((size_t)a.k_pad * a.DP * 4);
  pl.add<float>(a.k_pad);
  pl.add<float>(a.k_pad);
  pl.add<double>(parts);
  pl.add<unsigned long long>(parts);
  pl.add<int>(1);
  pl.add<KResult>(1);
}

PassBufs carve_pass(Arena& ar, const AssignPlan& a) {
  PassBufs b;
  b.Cq = ar.take<char>((size_t)a.k_pad * a.DP * 4);
  b.cinit = ar.take<float>(a.k_pad);
  b.ca = ar.take<float>(a.k_pad);
  const int parts = std::max(std::max(a.nwg, a.nwg_own), a.nwg_pair);
  b.sse_part = ar.take<double>(parts);
  b.corr_part = ar.take<unsigned long long>(parts);
  b.status = ar.take<int>(1);
  b.result = ar.take<KResult>(1);
  return b;
}

bool uses_prep(const AssignPlan& a) { return a.route == Route::Mfma || a.route == Route::MfmaNoFallback; }

// Descriptor of one assignment pass of one problem.
static AssignProb pass_assign_prob(const AssignPlan& a, const PassBufs& b, const float* X, int64_t n, int d,
                                   const float* C, int k, int32_t* labels, float* mindist, float* D,
                                   uint8_t* flagged, bool refine, bool hint) {
  AssignProb ap{};
  ap.X = X;
  ap.C = C;
  ap.Cq = b.Cq;
  ap.cinit = b.cinit;
  ap.ca = b.ca;
  ap.labels = labels;
  ap.mindist = mindist;
  ap.D = D;
  ap.flagged = flagged;
  ap.sse_part = b.sse_part;
  ap.corr_part = b.corr_part;
  ap.status = b.status;
  ap.n = n;
  ap.d = d;
  ap.k = k;
  ap.k_pad = a.k_pad;
  ap.oma = a.oma;
  ap.refine = refine ? 1 : 0;
  ap.hint = hint ? labels : nullptr;
  ap.gpw = a.gpw;
  ap.alpha = a.alpha_f;
  ap.high = a.high;
  return ap;
}

// Reduction of a pass's per-workgroup partials into the result record.
static ReduceProb pass_reduce_prob(const PassBufs& b, int64_t n, int k, double* sse_slot, int nparts) {
  ReduceProb rp{};
  rp.sse_part = b.sse_part;
  rp.corr_part = b.corr_part;
  rp.status = b.status;
  rp.sse_out = sse_slot;
  rp.result = b.result;
  rp.pairs = n * (long long)k;
  rp.nparts = nparts;
  return rp;
}

// Enqueue one assignment pass (prep + assign + reduce) of one problem.
static hipError_t enqueue_pass(km_context_impl* ctx, const AssignPlan& a, const PassBufs& b,
                               const float* X, int64_t n, int d, const float* C, int k, int32_t* labels,
                               float* mindist, double* sse_slot, int mode, float* D, uint8_t* flagged,
                               bool refine, bool hint, hipStream_t st) {
  // every descriptor of the pass in one upload
  Pack pk;
  // the small-problem kernel prepares its centres itself
  const bool prep = uses_prep(a) && !(mode == 0 && a.xd > 0);
  size_t o_pp = 0, o_ps = 0;
  int prep_wg = 0;
  if (prep) {
    PrepProb pp{};
    pp.C = C;
    pp.Cq = b.Cq;
    pp.cinit = b.cinit;
    pp.ca = b.ca;
    pp.status = b.status;
    pp.alpha = a.alpha_f;
    pp.k = k;
    pp.k_pad = a.k_pad;
    pp.d = d;
    pp.DP = a.DP;
    prep_wg = (a.k_pad + 3) / 4;  // one wave per centre
    const int32_t pre[2] = {0, prep_wg};
    o_pp = pk.add(&pp, sizeof(pp));
    o_ps = pk.add(pre, sizeof(pre));
  }
  const AssignProb ap = pass_assign_prob(a, b, X, n, d, C, k, labels, mindist, D, flagged, refine, hint);
  const int nwg = mode == 0 ? a.nwg : a.nwg_pair;
  const int32_t apre[2] = {0, nwg};
  const size_t o_ap = pk.add(&ap, sizeof(ap));
  const size_t o_as = pk.add(apre, sizeof(apre));
  const ReduceProb rp = pass_reduce_prob(b, n, k, sse_slot, nwg);
  const size_t o_rp = pk.add(&rp, sizeof(rp));
  char* dv = pk.upload(ctx, st);
  if (!dv) return hipErrorOutOfMemory;
  hipError_t e;
  if (prep) {
    e = launch_prep(a.low, (const PrepProb*)(dv + o_pp), (const int32_t*)(dv + o_ps), 1, prep_wg, st);
    if (e != hipSuccess) return e;
  }
  e = run_assign_dev(ctx, a, mode, dv + o_ap, dv + o_as, 1, nwg, st);
  if (e != hipSuccess) return e;
  return launch_reduce_parts((const ReduceProb*)(dv + o_rp), 1, st);
}

static int32_t finish_stats(km_context_impl* ctx, const KResult* dres, km_stats* stats, const AssignPlan& a,
                            int32_t iters, hipStream_t st) {
  KM_HIP(hipMemcpyAsync(ctx->h_result, dres, sizeof(KResult), hipMemcpyDeviceToHost, st));
  KM_HIP(hipStreamSynchronize(st));
  const KResult r = *ctx->h_result;
  const int32_t ds = status_from_bits(r.status);
  if (stats) {
    stats->n_corrected = a.route == Route::Direct64Exact ? 0 : r.n_corrected;
    stats->n_pairs = r.n_pairs;
    stats->iters = iters;
    stats->data_status = ds;
    stats->sse_last = r.sse;
    stats->shift_last = r.shift;
    stats->alpha_used = a.alpha_used;
  }
  return ds;
}

}  // namespace km

extern "C" {

int32_t kmeans_assign(km_context* ctx, const float* X, int64_t n, int32_t d, const float* C, int32_t k,
                      const km_precision* prec, int32_t* labels, float* mindist, double* sse,
                      km_stats* stats, void* stream, uint32_t flags) {
  if (!ctx || !X || !C || !labels) return KM_ERR_ARG;
  km_precision p = precision_or_default(prec);
  int32_t v = validate_precision(p);
  if (v != KM_OK) return v;
  v = check_shape(n, d, k, p);
  if (v != KM_OK) return v;
  hipStream_t st = (hipStream_t)stream;
  KM_HIP(hipSetDevice(ctx->device));
  WorkspaceUse ws_use(ctx, st);
  KM_HIP(ws_use.err);
  AssignPlan a = plan_assign(p, n, d, k);
  Plan pl;
  plan_pass(pl, a);
  KM_HIP(ctx->arena.ensure(pl.bytes));
  ctx->arena.reset();
  PassBufs b = carve_pass(ctx->arena, a);
  KM_HIP(zero_status_result(b.status, b.result, st));
  // the FP64 winner refinement only when distances or the SSE are wanted
  const bool refine = mindist || sse || stats;
  KM_HIP(enqueue_pass(ctx, a, b, X, n, d, C, k, labels, mindist, sse, 0, nullptr, nullptr, refine,
                      (flags & KM_LABELS_HINT) != 0, st));
  if (stats || (flags & KM_SYNC)) return finish_stats(ctx, b.result, stats, a, 0, st);
  return KM_OK;
}

int32_t kmeans_assign_flags(km_context* ctx, const float* X, int64_t n, int32_t d, const float* C, int32_t k,
                            const km_precision* prec, int32_t* labels, uint8_t* flagged, km_stats* stats,
                            void* stream, uint32_t flags) {
  if (!ctx || !X || !C || !labels || !flagged) return KM_ERR_ARG;
  km_precision p = precision_or_default(prec);
  int32_t v = validate_precision(p);
  if (v != KM_OK) return v;
  v = check_shape(n, d, k, p);
  if (v != KM_OK) return v;
  hipStream_t st = (hipStream_t)stream;
  KM_HIP(hipSetDevice(ctx->device));
  WorkspaceUse ws_use(ctx, st);
  KM_HIP(ws_use.err);
  AssignPlan a = plan_assign(p, n, d, k);
  a.record = true;
  Plan pl;
  plan_pass(pl, a);
  KM_HIP(ctx->arena.ensure(pl.bytes));
  ctx->arena.reset();
  PassBufs b = carve_pass(ctx->arena, a);
  KM_HIP(zero_status_result(b.status, b.result, st));
  // a pass routed to the direct kernel corrects every pair; otherwise the
  // assignment kernels write a 1 for each pair their test flags
  KM_HIP(launch_fill_bytes(flagged, n * (int64_t)k, a.route == Route::Direct64All ? 1 : 0, st));
  KM_HIP(enqueue_pass(ctx, a, b, X, n, d, C, k, labels, nullptr, nullptr, 0, nullptr, flagged, stats != nullptr,
                      (flags & KM_LABELS_HINT) != 0, st));
  if (stats || (flags & KM_SYNC)) return finish_stats(ctx, b.result, stats, a, 0, st);
  return KM_OK;
}

int32_t kmeans_assign_static(km_context* ctx, const float* X, int64_t n, int32_t d, const float* C,
                             int32_t k, const km_precision* prec, int32_t* labels, float* mindist,
                             double* sse, km_stats* stats, void* stream, uint32_t flags) {
  if (!ctx || !X || !C || !labels || !ctx->static_scratch) return KM_ERR_ARG;
  km_precision p = precision_or_default(prec);
  int32_t v = validate_precision(p);
  if (v != KM_OK) return v;
  v = check_shape(n, d, k, p);
  if (v != KM_OK) return v;
  AssignPlan a = plan_assign(p, n, d, k);
  Plan pl;
  plan_pass(pl, a);
  if (pl.bytes > (size_t)KM_STATIC_SCRATCH_BYTES) return KM_ERR_UNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  KM_HIP(hipSetDevice(ctx->device));
  WorkspaceUse ws_use(ctx, st);
  KM_HIP(ws_use.err);
  // the pass's workspace is carved from the fixed array, never grown
  Arena ar;
  ar.base = ctx->static_scratch;
  ar.cap = KM_STATIC_SCRATCH_BYTES;
  PassBufs b = carve_pass(ar, a);
  // timing events would be created on first use: not recorded here
  const bool timing = ctx->timing;
  ctx->timing = false;
  // the status word and result record start at zero (a fill kernel)
  hipError_t e = zero_status_result(b.status, b.result, st);
  const bool refine = mindist || sse || stats;
  if (e == hipSuccess)
    e = enqueue_pass(ctx, a, b, X, n, d, C, k, labels, mindist, sse, 0, nullptr, nullptr, refine,
                     (flags & KM_LABELS_HINT) != 0, st);
  ctx->timing = timing;
  KM_HIP(e);
  if (stats || (flags & KM_SYNC)) return finish_stats(ctx, b.result, stats, a, 0, st);
  return KM_OK;
}

int32_t kmeans_pairwise(km_context* ctx, const float* X, int64_t m, int32_t d, const float* C, int32_t k,
                        const km_precision* prec, float* D, uint8_t* flagged, void* stream, uint32_t flags) {
  if (!ctx || !X || !C || !D) return KM_ERR_ARG;
  km_precision p = precision_or_default(prec);
  int32_t v = validate_precision(p);
  if (v != KM_OK) return v;
  v = check_shape(m, d, k, p);
  if (v != KM_OK) return v;
  hipStream_t st = (hipStream_t)stream;
  KM_HIP(hipSetDevice(ctx->device));
  WorkspaceUse ws_use(ctx, st);
  KM_HIP(ws_use.err);
  AssignPlan a = plan_assign(p, m, d, k);
  Plan pl;
  plan_pass(pl, a);
  KM_HIP(ctx->arena.ensure(pl.bytes));
  ctx->arena.reset();
  PassBufs b = carve_pass(ctx->arena, a);
  KM_HIP(zero_status_result(b.status, b.result, st));
  KM_HIP(enqueue_pass(ctx, a, b, X, m, d, C, k, nullptr, nullptr, nullptr, 1, D, flagged, true, false, st));
  if (flags & KM_SYNC) return finish_stats(ctx, b.result, nullptr, a, 0, st);
  return KM_OK;
}

int32_t kmeans_quantize(km_context* ctx, const float* in, int64_t count, int32_t low, uint16_t* out,
                        void* stream, uint32_t flags) {
  if (!ctx || !in || !out || count < 0 || (low != KM_LOW_FP16 && low != KM_LOW_BF16)) return KM_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  KM_HIP(hipSetDevice(ctx->device));
  KM_HIP(launch_quantize(low, in, count, out, st));
  if (flags & KM_SYNC) KM_HIP(hipStreamSynchronize(st));
  return KM_OK;
}

int32_t kmeans_update(km_context* ctx, const float* X, int64_t n, int32_t d, const int32_t* labels, int32_t k,
                      const float* C_old, float* C_new, int64_t* counts, double* shift, double* sse,
                      void* stream, uint32_t flags) {
  if (!ctx || !X || !labels || !C_old || !C_new || C_old == C_new) return KM_ERR_ARG;
  if (n < 1 || n > (int64_t)INT32_MAX - 1024 || d < 1 || k < 1 || k > 65536) return KM_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  KM_HIP(hipSetDevice(ctx->device));
  WorkspaceUse ws_use(ctx, st);
  KM_HIP(ws_use.err);
  Plan pl;
  plan_update(pl, n, d, k);
  pl.add<int>(1);
  pl.add<KResult>(1);
  KM_HIP(ctx->arena.ensure(pl.bytes));
  ctx->arena.reset();
  UpdateProb u = carve_update(ctx->arena, n, d, k);
  int* status = ctx->arena.take<int>(1);
  KResult* res = ctx->arena.take<KResult>(1);
  KM_HIP(zero_status_result(status, res, st));
  u.X = X;
  u.labels = labels;
  u.C_old = C_old;
  u.C_new = C_new;
  u.counts_out = reinterpret_cast<long long*>(counts);
  u.shift_out = shift;
  u.sse_out = sse;
  u.result = res;
  u.status = status;
  KM_HIP(run_update(ctx, {u}, st));
  if (flags & KM_SYNC) {
    KM_HIP(hipMemcpyAsync(ctx->h_result, status, sizeof(int), hipMemcpyDeviceToHost, st));
    KM_HIP(hipStreamSynchronize(st));
    return status_from_bits(*reinterpret_cast<int*>(ctx->h_result));
  }
  return KM_OK;
}

}  // extern "C"

namespace km {

// Descriptors of one Lloyd round, laid out for an upload of many rounds.
struct RoundDesc {
  alignas(16) PrepProb pp;
  alignas(16) AssignProb ap;
  alignas(16) ReduceProb rp;
  alignas(16) UpdateProb up;
};

// Rounds of kmeans_lloyd with one launch per phase and the descriptors of up
// to kRoundBlock rounds uploaded in one copy (one pass and one update
// uploaded separately cost two copies per round, each a few microseconds on
// the stream).  The launches and their arguments are those of enqueue_pass
// and run_update (for an owner-path update the partial reduction of the
// pass runs in the launch of the shift).  Round r goes from C0/C1 (r even/odd) to the other
// buffer; *done receives the rounds run (a positive tol reads the shift back
// after every round).
static hipError_t enqueue_phase_rounds(km_context_impl* ctx, const AssignPlan& a, const PassBufs& b,
                                       const UpdateProb& u0, const float* X, int64_t n, int d, int k, float* C0,
                                       float* C1, int32_t* labels, double* sse_hist, int max_iter, double tol,
                                       int* done, hipStream_t st) {
  constexpr int kRoundBlock = 128;
  *done = 0;
  const bool prep = uses_prep(a) && !(a.xd > 0);  // the small kernel prepares its centres itself
  const int prep_wg = (a.k_pad + 3) / 4;          // one wave per centre
  const bool own = u0.owners > 0;
  // prefixes, the same every round: assignment, preparation, update
  std::vector<int32_t> pre = {0, a.nwg, 0, prep_wg};
  const size_t upd = pre.size();
  if (own) {
    const int J = own_fin_clusters(d);
    for (int v : {u0.nchunk, (k + J - 1) / J}) pre.insert(pre.end(), {0, v});
  } else {
    const int chunkwg = (int)(((n + u0.chunk - 1) / u0.chunk + k + 3) / 4);
    for (int v : {u0.ntiles, k, chunkwg, (k + 3) / 4, (u0.ntiles + 3) / 4}) pre.insert(pre.end(), {0, v});
  }
  const int32_t* dpre = static_cast<const int32_t*>(ctx->up.put(pre.data(), sizeof(int32_t) * pre.size(), st));
  if (!dpre) return hipErrorOutOfMemory;
  for (int r0 = 0; r0 < max_iter; r0 += kRoundBlock) {
    const int r1 = std::min(max_iter, r0 + kRoundBlock);
    std::vector<RoundDesc> rd((size_t)(r1 - r0));
    for (int r = r0; r < r1; ++r) {
      float* c_old = (r & 1) ? C1 : C0;
      float* c_new = (r & 1) ? C0 : C1;
      RoundDesc& q = rd[(size_t)(r - r0)];
      q = RoundDesc{};
      if (prep) {
        q.pp.C = c_old;
        q.pp.Cq = b.Cq;
        q.pp.cinit = b.cinit;
        q.pp.ca = b.ca;
        q.pp.status = b.status;
        q.pp.alpha = a.alpha_f;
        q.pp.k = k;
        q.pp.k_pad = a.k_pad;
        q.pp.d = d;
        q.pp.DP = a.DP;
      }
      // the SSE of a round's pass comes from the update, which reads every
      // point's row against the centre it was assigned to
      q.ap = pass_assign_prob(a, b, X, n, d, c_old, k, labels, nullptr, nullptr, nullptr, false, r > 0);
      q.rp = pass_reduce_prob(b, n, k, nullptr, a.nwg);
      q.up = u0;
      q.up.C_old = c_old;
      q.up.C_new = c_new;
      q.up.sse_out = sse_hist ? sse_hist + r : nullptr;
    }
    char* dr = static_cast<char*>(ctx->up.put(rd.data(), sizeof(RoundDesc) * rd.size(), st));
    if (!dr) return hipErrorOutOfMemory;
    for (int r = r0; r < r1; ++r) {
      char* dq = dr + sizeof(RoundDesc) * (size_t)(r - r0);
      const RoundDesc& hq = rd[(size_t)(r - r0)];
      const UpdateProb* dup = reinterpret_cast<const UpdateProb*>(dq + offsetof(RoundDesc, up));
      hipError_t e = hipSuccess;
      if (prep) e = launch_prep(a.low, reinterpret_cast<const PrepProb*>(dq + offsetof(RoundDesc, pp)), dpre + 2, 1,
                                prep_wg, st);
      const ReduceProb* drp = reinterpret_cast<const ReduceProb*>(dq + offsetof(RoundDesc, rp));
      if (e == hipSuccess) e = run_assign_dev(ctx, a, 0, dq + offsetof(RoundDesc, ap), dpre, 1, a.nwg, st);
      if (e == hipSuccess) {
        if (own) {  // the partial reduction joins the shift launch at the end
          e = launch_update_own_part(dup, &hq.up, 1, dpre + upd, st);
          if (e == hipSuccess) e = launch_update_own_fin(dup, &hq.up, 1, dpre + upd + 2, st, false);
          if (e == hipSuccess) e = launch_round_tail(drp, dup, st);
        } else {
          e = launch_reduce_parts(drp, 1, st);
          if (e == hipSuccess) e = launch_update(dup, &hq.up, 1, dpre + upd, st);
        }
      }
      if (e != hipSuccess) return e;
      *done = r + 1;
      if (tol > 0.0) {
        e = hipMemcpyAsync(ctx->h_scalar, &b.result->shift, sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        if (*ctx->h_scalar < tol) return hipSuccess;
      }
    }
  }
  return hipSuccess;
}

// Polls after which a grid-wide wait of the persistent launch gives up:
// kSyncSpins, or KM_ROUND_SPIN_LIMIT from the environment (a small value
// forces the give-up path in tests; the launch still ends and the call
// reports KM_ERR_DEVICE).
static unsigned round_spin_limit() {
  const char* e = getenv("KM_ROUND_SPIN_LIMIT");
  if (!e || !*e) return kSyncSpins;
  const unsigned long v = strtoul(e, nullptr, 10);
  return v >= 1 && v <= kSyncSpins ? (unsigned)v : kSyncSpins;
}

// Lloyd rounds that one persistent launch can run: the small-problem
// assignment kernel and the owner path of the update.
static bool rounds_fit(const AssignPlan& a, const UpdateProb& u) {
  return a.xd > 0 && (a.route == Route::Mfma || a.route == Route::MfmaNoFallback) && u.owners > 0 && u.nc == 1;
}

// Enqueues every round of one problem in one persistent launch (C0 holds the
// initial centres, rounds alternate C0 -> C1 -> C0 ...).  *ran = false when
// the runtime refuses the co-resident grid: nothing ran and the caller runs
// its launch-per-phase loop.
static hipError_t enqueue_rounds(km_context_impl* ctx, const AssignPlan& a, const PassBufs& b,
                                 const UpdateProb& u0, const float* X, int64_t n, int d, int k, float* C0,
                                 float* C1, int32_t* labels, double* sse_hist, int max_iter, double tol, int* ctl,
                                 bool* ran, hipStream_t st) {
  *ran = false;
  RoundProb R{};
  for (int q = 0; q < 2; ++q) {
    float* c_old = q == 0 ? C0 : C1;
    float* c_new = q == 0 ? C1 : C0;
    R.a[q] = pass_assign_prob(a, b, X, n, d, c_old, k, labels, nullptr, nullptr, nullptr, false, false);
    R.u[q] = u0;
    R.u[q].C_old = c_old;
    R.u[q].C_new = c_new;
    R.u[q].sse_out = nullptr;
  }
  R.red = pass_reduce_prob(b, n, k, nullptr, a.nwg);
  R.sse_hist = sse_hist;
  R.tol = tol;
  R.max_iter = max_iter;
  const int J = own_fin_clusters(d);
  R.nfin = (k + J - 1) / J;
  R.wstride = std::max(16, own_wave_bytes(u0.owners, d, k));
  const int32_t tpre[2] = {0, a.nwg};
  const int32_t cpre[2] = {0, u0.nchunk};
  const int32_t fpre[2] = {0, 1 + R.nfin};
  Pack pk;
  const size_t o_r = pk.add(&R, sizeof(R));
  const size_t o_t = pk.add(tpre, sizeof(tpre));
  const size_t o_c = pk.add(cpre, sizeof(cpre));
  const size_t o_f = pk.add(fpre, sizeof(fpre));
  char* dv = pk.upload(ctx, st);
  if (!dv) return hipErrorOutOfMemory;
  hipError_t e = launch_zero_words(ctl, sizeof(int) * (size_t)round_ctl_words(1), st);
  if (e != hipSuccess) return e;
  const bool fb = a.route == Route::Mfma;
  const int lds = std::max(small_lds_bytes(a.xd, fb), kOwnWaves * R.wstride + 4 * k * d);
  // with timing on, the whole launch is one entry of the record
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ctx->timing) {
    e0 = ctx->timing_event(2 * ctx->ev_used);
    e1 = ctx->timing_event(2 * ctx->ev_used + 1);
    if (!e0 || !e1) return hipErrorOutOfMemory;
    e = hipEventRecord(e0, st);
    if (e != hipSuccess) return e;
  }
  e = launch_lloyd_rounds(a.low, a.xd, fb, (const RoundProb*)(dv + o_r), 1, (const int32_t*)(dv + o_t),
                          (const int32_t*)(dv + o_c), (const int32_t*)(dv + o_f), ctl,
                          std::max(a.nwg, u0.nchunk), lds, round_spin_limit(), st);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return hipSuccess;
  }
  *ran = true;
  if (ctx->timing) {
    e = hipEventRecord(e1, st);
    if (e != hipSuccess) return e;
    ctx->ev_used += 1;
  }
  return hipSuccess;
}

}  // namespace km

extern "C" {

int32_t kmeans_lloyd(km_context* ctx, const float* X, int64_t n, int32_t d, int32_t k, float* C_inout,
                     int32_t max_iter, double tol, const km_precision* prec, int32_t* labels, float* mindist,
                     double* sse_hist, km_stats* stats, void* stream, uint32_t flags) {
  if (!ctx || !X || !C_inout || !labels || max_iter < 0) return KM_ERR_ARG;
  km_precision p = precision_or_default(prec);
  int32_t v = validate_precision(p);
  if (v != KM_OK) return v;
  v = check_shape(n, d, k, p);
  if (v != KM_OK) return v;
  hipStream_t st = (hipStream_t)stream;
  KM_HIP(hipSetDevice(ctx->device));
  WorkspaceUse ws_use(ctx, st);
  KM_HIP(ws_use.err);
  AssignPlan a = plan_assign(p, n, d, k);
  Plan pl;
  plan_pass(pl, a);
  plan_update(pl, n, d, k);
  pl.add<float>((size_t)k * d);  // second centre buffer
  pl.add<int>((size_t)round_ctl_words(1));
  KM_HIP(ctx->arena.ensure(pl.bytes));
  ctx->arena.reset();
  PassBufs b = carve_pass(ctx->arena, a);
  UpdateProb u = carve_update(ctx->arena, n, d, k);
  float* Cw = ctx->arena.take<float>((size_t)k * d);
  int* ctl = ctx->arena.take<int>((size_t)round_ctl_words(1));
  KM_HIP(zero_status_result(b.status, b.result, st));
  u.X = X;
  u.labels = labels;
  u.result = b.result;
  u.status = b.status;
  float* cur = C_inout;
  float* nxt = Cw;
  int32_t it = 0;
  bool ran = false;
  if (max_iter > 0 && (flags & KM_ROUND_LAUNCH) && rounds_fit(a, u)) {
    KM_HIP(enqueue_rounds(ctx, a, b, u, X, n, d, k, C_inout, Cw, labels, sse_hist, max_iter, tol, ctl, &ran, st));
    if (ran) {
      it = max_iter;
      if (tol > 0.0) {  // the rounds run are known on the device only
        int* h = reinterpret_cast<int*>(ctx->h_result);
        KM_HIP(hipMemcpyAsync(h, ctl, sizeof(int) * (size_t)round_ctl_words(1), hipMemcpyDeviceToHost, st));
        KM_HIP(hipStreamSynchronize(st));
        if (h[1] != 0) return KM_ERR_DEVICE;
        it = h[3];
      }
      if (it & 1) std::swap(cur, nxt);
    }
  }
  if (!ran && max_iter > 0) {
    int done = 0;
    KM_HIP(enqueue_phase_rounds(ctx, a, b, u, X, n, d, k, C_inout, Cw, labels, sse_hist, max_iter, tol, &done, st));
    it = done;
    if (it & 1) std::swap(cur, nxt);
  }
  KM_HIP(enqueue_pass(ctx, a, b, X, n, d, cur, k, labels, mindist, sse_hist ? sse_hist + it : nullptr, 0,
                      nullptr, nullptr, true, it > 0, st));
  if (cur != C_inout)
    KM_HIP(hipMemcpyAsync(C_inout, cur, sizeof(float) * (size_t)k * d, hipMemcpyDeviceToDevice, st));
  if (stats || (flags & KM_SYNC)) return finish_stats(ctx, b.result, stats, a, it, st);
  return KM_OK;
}

int32_t kmeans_seed_pp(km_context* ctx, const float* X, int64_t n, int32_t d, int32_t k, const double* uniforms,
                       float* C_out, int32_t* idx_out, void* stream, uint32_t flags) {
  if (!ctx || !X || !uniforms || !C_out) return KM_ERR_ARG;
  if (n < 1 || n > (int64_t)INT32_MAX - 1024 || d < 1 || d > 1024 || k < 1 || k > 65536 || k > n)
    return KM_ERR_ARG;
  for (int i = 0; i < k; ++i)
    if (!(uniforms[i] >= 0.0 && uniforms[i] < 1.0)) return KM_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  KM_HIP(hipSetDevice(ctx->device));
  WorkspaceUse ws_use(ctx, st);
  KM_HIP(ws_use.err);
  const int64_t nblocks = (n + 1023) / 1024;
  Plan pl;
  pl.add<double>((size_t)n);
  pl.add<double>((size_t)nblocks);
  pl.add<int32_t>(1);
  KM_HIP(ctx->arena.ensure(pl.bytes));
  ctx->arena.reset();
  double* w = ctx->arena.take<double>((size_t)n);
  double* bsum = ctx->arena.take<double>((size_t)nblocks);
  int32_t* pick = ctx->arena.take<int32_t>(1);
  KM_HIP(launch_seed_pp(X, n, d, k, uniforms, C_out, idx_out, w, bsum, pick, st));
  if (flags & KM_SYNC) KM_HIP(hipStreamSynchronize(st));
  return KM_OK;
}

int32_t kmeans_lloyd_schedule(km_context* ctx, const float* X, int64_t n, int32_t d, int32_t k, float* C_inout,
                              int32_t max_iter, double tol, const km_precision* early, const km_precision* late,
                              double switch_rel, int32_t max_early, int32_t* labels, float* mindist,
                              double* sse_hist, km_stats* stats, int32_t* switch_round, void* stream,
                              uint32_t flags) {
  if (!ctx || !X || !C_inout || !labels || max_iter < 0 || max_early < 0 || !(switch_rel >= 0.0))
    return KM_ERR_ARG;
  const km_precision pe = precision_or_default(early), pl_ = precision_or_default(late);
  int32_t v = validate_precision(pe);
  if (v == KM_OK) v = validate_precision(pl_);
  if (v == KM_OK) v = check_shape(n, d, k, pe);
  if (v == KM_OK) v = check_shape(n, d, k, pl_);
  if (v != KM_OK) return v;
  hipStream_t st = (hipStream_t)stream;
  KM_HIP(hipSetDevice(ctx->device));
  WorkspaceUse ws_use(ctx, st);
  KM_HIP(ws_use.err);
  AssignPlan ae = plan_assign(pe, n, d, k), al = plan_assign(pl_, n, d, k);
  Plan pl;
  plan_pass(pl, ae);
  plan_pass(pl, al);
  plan_update(pl, n, d, k);
  pl.add<float>((size_t)k * d);           // second centre buffer
  pl.add<double>((size_t)max_iter + 1);   // round SSEs when the caller keeps none
  KM_HIP(ctx->arena.ensure(pl.bytes));
  ctx->arena.reset();
  PassBufs be = carve_pass(ctx->arena, ae), bl = carve_pass(ctx->arena, al);
  UpdateProb u = carve_update(ctx->arena, n, d, k);
  float* Cw = ctx->arena.take<float>((size_t)k * d);
  double* sse_dev = sse_hist ? sse_hist : ctx->arena.take<double>((size_t)max_iter + 1);
  KM_HIP(zero_status_result(be.status, be.result, st));
  KM_HIP(zero_status_result(bl.status, bl.result, st));
  u.X = X;
  u.labels = labels;
  float* cur = C_inout;
  float* nxt = Cw;
  // early rounds: the early precision while the round's relative SSE
  // decrease is at least switch_rel (and at most max_early rounds); then the
  // late precision for the remaining rounds and the final pass
  bool late_on = max_early == 0;
  int32_t switched = late_on ? 0 : -1;
  double prev_sse = 0.0;
  int32_t it = 0;
  for (; it < max_iter; ++it) {
    const AssignPlan& a = late_on ? al : ae;
    const PassBufs& b = late_on ? bl : be;
    KM_HIP(enqueue_pass(ctx, a, b, X, n, d, cur, k, labels, nullptr, nullptr, 0, nullptr, nullptr, false,
                        it > 0, st));
    u.C_old = cur;
    u.C_new = nxt;
    u.sse_out = sse_dev + it;
    u.result = b.result;
    u.status = b.status;
    KM_HIP(run_update(ctx, {u}, st));
    std::swap(cur, nxt);
    if (!late_on || tol > 0.0) {
      KM_HIP(hipMemcpyAsync(ctx->h_scalar, &b.result->shift, sizeof(double), hipMemcpyDeviceToHost, st));
      KM_HIP(hipMemcpyAsync(ctx->h_scalar + 1, sse_dev + it, sizeof(double), hipMemcpyDeviceToHost, st));
      KM_HIP(hipStreamSynchronize(st));
      const double shift = ctx->h_scalar[0], sse_t = ctx->h_scalar[1];
      if (!late_on) {
        const bool flat = it > 0 && !(prev_sse - sse_t >= switch_rel * prev_sse);
        if (flat || it + 1 >= max_early) {
          late_on = true;
          switched = it + 1;
        }
        prev_sse = sse_t;
      }
      if (tol > 0.0 && shift < tol) {
        ++it;
        break;
      }
    }
  }
  if (switched < 0) switched = it;  // the final pass is the first in the late precision
  if (switch_round) *switch_round = switched;
  KM_HIP(enqueue_pass(ctx, al, bl, X, n, d, cur, k, labels, mindist, sse_hist ? sse_hist + it : nullptr, 0,
                      nullptr, nullptr, true, it > 0, st));
  if (cur != C_inout)
    KM_HIP(hipMemcpyAsync(C_inout, cur, sizeof(float) * (size_t)k * d, hipMemcpyDeviceToDevice, st));
  if (!stats && !(flags & KM_SYNC)) return KM_OK;
  KM_HIP(hipMemcpyAsync(ctx->h_result, be.result, sizeof(KResult), hipMemcpyDeviceToHost, st));
  KM_HIP(hipMemcpyAsync(ctx->h_result + 1, bl.result, sizeof(KResult), hipMemcpyDeviceToHost, st));
  KM_HIP(hipStreamSynchronize(st));
  const KResult re = ctx->h_result[0], rl = ctx->h_result[1];
  const int32_t ds_e = status_from_bits(re.status), ds_l = status_from_bits(rl.status);
  const int32_t ds = ds_e != KM_OK ? ds_e : ds_l;
  if (stats) {
    stats->n_corrected = (ae.route == Route::Direct64Exact ? 0 : re.n_corrected) +
                         (al.route == Route::Direct64Exact ? 0 : rl.n_corrected);
    stats->n_pairs = re.n_pairs + rl.n_pairs;
    stats->iters = it;
    stats->data_status = ds;
    stats->sse_last = rl.sse;
    stats->shift_last = switched < it ? rl.shift : re.shift;
    stats->alpha_used = al.alpha_used;
  }
  return ds;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched solves
// ---------------------------------------------------------------------------
namespace km {

// Enqueue one assignment pass for every listed problem: one prep launch per
// low format, one assignment launch per (route, DP) group, one reduce launch.
hipError_t enqueue_batch_pass(km_context_impl* ctx, std::vector<BatchState*>& list, bool final_pass,
                                     hipStream_t st) {
  if (list.empty()) return hipSuccess;
  // prep
  {
    std::vector<PrepProb> pp;
    std::vector<int> kp;
    int low = -1;
    for (BatchState* s : list) {
      if (!uses_prep(s->plan) || s->plan.xd > 0) continue;  // small kernel: prepared in the pass
      PrepProb q{};
      q.C = s->cur;
      q.Cq = s->bufs.Cq;
      q.cinit = s->bufs.cinit;
      q.ca = s->bufs.ca;
      q.status = s->bufs.status;
      q.alpha = s->plan.alpha_f;
      q.k = s->prob->k;
      q.k_pad = s->plan.k_pad;
      q.d = s->prob->d;
      q.DP = s->plan.DP;
      pp.push_back(q);
      kp.push_back(s->plan.k_pad);
      low = s->plan.low;
    }
    if (!pp.empty()) {
      hipError_t e = run_prep(ctx, low, pp, kp, st);
      if (e != hipSuccess) return e;
    }
  }
  // assign, grouped by kernel shape
  std::vector<bool> taken(list.size(), false);
  for (size_t i = 0; i < list.size(); ++i) {
    if (taken[i]) continue;
    const AssignPlan& sh = list[i]->plan;
    std::vector<AssignProb> ap;
    std::vector<int> nw;
    for (size_t j = i; j < list.size(); ++j) {
      const AssignPlan& o = list[j]->plan;
      if (taken[j] || o.route != sh.route || o.DP != sh.DP || o.low != sh.low || o.xd != sh.xd ||
          o.high != sh.high)
        continue;
      // the final pass refines and sums the SSE per workgroup: the problem's
      // own partition, as when it runs alone
      const int gpw = final_pass ? o.gpw_own : o.gpw;
      const int nwg = final_pass ? o.nwg_own : o.nwg;
      taken[j] = true;
      BatchState* s = list[j];
      AssignProb a{};
      a.X = s->prob->X;
      a.C = s->cur;
      a.Cq = s->bufs.Cq;
      a.cinit = s->bufs.cinit;
      a.ca = s->bufs.ca;
      a.labels = s->prob->labels;
      a.mindist = final_pass ? s->prob->mindist : nullptr;
      a.sse_part = s->bufs.sse_part;
      a.corr_part = s->bufs.corr_part;
      a.status = s->bufs.status;
      a.n = s->prob->n;
      a.d = s->prob->d;
      a.k = s->prob->k;
      a.k_pad = o.k_pad;
      a.oma = o.oma;
      a.refine = final_pass ? 1 : 0;
      a.hint = s->it > 0 ? s->prob->labels : nullptr;  // the previous round's labels
      a.gpw = gpw;
      a.alpha = o.alpha_f;
      a.high = o.high;
      ap.push_back(a);
      nw.push_back(nwg);
    }
    hipError_t e = run_assign(ctx, sh, 0, ap, nw, st);
    if (e != hipSuccess) return e;
  }
  // reduce
  std::vector<ReduceProb> rp;
  for (BatchState* s : list) {
    ReduceProb r{};
    r.sse_part = s->bufs.sse_part;
    r.corr_part = s->bufs.corr_part;
    r.status = s->bufs.status;
    r.sse_out = (final_pass && s->prob->sse_hist) ? s->prob->sse_hist + s->it : nullptr;
    r.result = s->bufs.result;
    r.pairs = s->prob->n * (long long)s->prob->k;
    r.nparts = final_pass ? s->plan.nwg_own : s->plan.nwg;
    rp.push_back(r);
  }
  return run_reduce(ctx, rp, st);
}

hipError_t enqueue_batch_round(km_context_impl* ctx, std::vector<BatchState*>& act, hipStream_t st) {
  if (act.empty()) return hipSuccess;
  hipError_t e = enqueue_batch_pass(ctx, act, false, st);
  if (e != hipSuccess) return e;
  std::vector<UpdateProb> up;
  for (BatchState* s : act) {
    s->upd.C_old = s->cur;
    s->upd.C_new = s->nxt;
    s->upd.sse_out = s->prob->sse_hist ? s->prob->sse_hist + s->it : nullptr;
    up.push_back(s->upd);
  }
  e = run_update(ctx, up, st);
  if (e != hipSuccess) return e;
  for (BatchState* s : act) {
    std::swap(s->cur, s->nxt);
    s->it += 1;
    if (s->it >= s->prob->max_iter) s->done = true;
  }
  return hipSuccess;
}

// Every remaining round of the listed problems that one persistent launch
// can run (rounds_fit), one cooperative launch per kernel shape (row
// capacity, threshold on/off), at most kRoundMaxProbs problems each.  The
// per-round descriptors are those of enqueue_batch_round; a problem's rounds
// are its own (max_iter, tol), so each gets the bits it gets alone.  Problems
// handled are marked done with their rounds and centre buffer; a launch the
// runtime refuses leaves its problems to the caller's per-phase rounds.
static hipError_t enqueue_batch_rounds(km_context_impl* ctx, std::vector<BatchState>& S, int* ctl,
                                       hipStream_t st) {
  std::map<std::pair<int, int>, std::vector<BatchState*>> groups;
  for (auto& s : S)
    if (!s.done && s.it < s.prob->max_iter && rounds_fit(s.plan, s.upd))
      groups[{s.plan.xd, s.plan.route == Route::Mfma ? 1 : 0}].push_back(&s);
  for (auto& g : groups) {
    for (size_t g0 = 0; g0 < g.second.size(); g0 += kRoundMaxProbs) {
      const size_t g1 = std::min(g.second.size(), g0 + (size_t)kRoundMaxProbs);
      std::vector<BatchState*> list(g.second.begin() + g0, g.second.begin() + g1);
      const int np = (int)list.size();
      std::vector<RoundProb> R((size_t)np);
      std::vector<int> tiles(np), chunks(np), fins(np);
      int lds = 0, work = 0;
      bool need_tol = false;
      for (int i = 0; i < np; ++i) {
        BatchState& b = *list[i];
        const km_problem& q = *b.prob;
        RoundProb& r = R[i];
        for (int par = 0; par < 2; ++par) {
          float* c_old = par == 0 ? b.cur : b.nxt;
          float* c_new = par == 0 ? b.nxt : b.cur;
          r.a[par] = pass_assign_prob(b.plan, b.bufs, q.X, q.n, q.d, c_old, q.k, q.labels, nullptr, nullptr,
                                      nullptr, false, false);
          r.u[par] = b.upd;
          r.u[par].C_old = c_old;
          r.u[par].C_new = c_new;
          r.u[par].sse_out = nullptr;
        }
        r.red = pass_reduce_prob(b.bufs, q.n, q.k, nullptr, b.plan.nwg);
        r.sse_hist = q.sse_hist ? q.sse_hist + b.it : nullptr;
        r.tol = q.tol;
        r.max_iter = q.max_iter - b.it;
        const int J = own_fin_clusters(q.d);
        r.nfin = (q.k + J - 1) / J;
        r.wstride = std::max(16, own_wave_bytes(b.upd.owners, q.d, q.k));
        tiles[i] = b.plan.nwg;
        chunks[i] = b.upd.nchunk;
        fins[i] = 1 + r.nfin;
        lds = std::max(lds, kOwnWaves * r.wstride + 4 * q.k * q.d);
        work = std::max(work, std::max(b.plan.nwg, b.upd.nchunk));
        need_tol |= q.tol > 0.0;
      }
      std::vector<int32_t> tpre = prefix(tiles), cpre = prefix(chunks), fpre = prefix(fins);
      work = std::max(work, std::max(std::max(tpre.back(), cpre.back()), fpre.back()));
      const bool fb = g.first.second != 0;
      lds = std::max(lds, small_lds_bytes(g.first.first, fb));
      Pack pk;
      const size_t o_r = pk.add(R.data(), sizeof(RoundProb) * R.size());
      const size_t o_t = pk.add(tpre.data(), sizeof(int32_t) * tpre.size());
      const size_t o_c = pk.add(cpre.data(), sizeof(int32_t) * cpre.size());
      const size_t o_f = pk.add(fpre.data(), sizeof(int32_t) * fpre.size());
      char* dv = pk.upload(ctx, st);
      if (!dv) return hipErrorOutOfMemory;
      hipError_t e = launch_zero_words(ctl, sizeof(int) * (size_t)round_ctl_words(np), st);
      if (e != hipSuccess) return e;
      e = launch_lloyd_rounds(list[0]->plan.low, g.first.first, fb, (const RoundProb*)(dv + o_r), np,
                              (const int32_t*)(dv + o_t), (const int32_t*)(dv + o_c), (const int32_t*)(dv + o_f),
                              ctl, work, lds, round_spin_limit(), st);
      if (e != hipSuccess) {  // not co-resident: per-phase rounds instead
        (void)hipGetLastError();
        continue;
      }
      std::vector<int> rounds((size_t)np);
      if (need_tol) {  // the rounds run are known on the device only
        int* h = reinterpret_cast<int*>(ctx->h_result);
        e = hipMemcpyAsync(h, ctl, sizeof(int) * (size_t)round_ctl_words(np), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        if (h[1] != 0) return hipErrorLaunchFailure;
        for (int i = 0; i < np; ++i) rounds[i] = h[2 + np + i];
      } else {
        for (int i = 0; i < np; ++i) rounds[i] = list[i]->prob->max_iter - list[i]->it;
      }
      for (int i = 0; i < np; ++i) {
        BatchState& b = *list[i];
        b.it += rounds[i];
        if (rounds[i] & 1) std::swap(b.cur, b.nxt);
        b.done = true;
      }
    }
  }
  return hipSuccess;
}

}  // namespace km

extern "C" int32_t kmeans_solve_batch(km_context* ctx, km_problem* probs, int32_t count,
                                      const km_precision* prec, void* stream, uint32_t flags) {
  if (!ctx || (!probs && count > 0) || count < 0) return KM_ERR_ARG;
  if (count == 0) return KM_OK;
  if (count > km_context_impl::kMaxResults) return KM_ERR_ARG;
  km_precision p = precision_or_default(prec);
  int32_t v = validate_precision(p);
  if (v != KM_OK) return v;
  for (int i = 0; i < count; ++i) {
    const km_problem& q = probs[i];
    if (!q.X || !q.C_inout || !q.labels || q.max_iter < 0) return KM_ERR_ARG;
    v = check_shape(q.n, q.d, q.k, p);
    if (v != KM_OK) return v;
  }
  hipStream_t st = (hipStream_t)stream;
  KM_HIP(hipSetDevice(ctx->device));
  WorkspaceUse ws_use(ctx, st);
  KM_HIP(ws_use.err);
  std::vector<BatchState> S(count);
  Plan pl;
  for (int i = 0; i < count; ++i) {
    S[i].prob = &probs[i];
    S[i].plan = plan_assign(p, probs[i].n, probs[i].d, probs[i].k);
  }
  {  // problems sharing a small-problem launch: sweep length from their total
    std::map<int, int64_t> total;
    for (int i = 0; i < count; ++i)
      if (S[i].plan.xd > 0) total[S[i].plan.xd] += probs[i].n;
    for (int i = 0; i < count; ++i)
      if (S[i].plan.xd > 0) set_small_sweep(S[i].plan, probs[i].n, total[S[i].plan.xd]);
  }
  for (int i = 0; i < count; ++i) {
    plan_pass(pl, S[i].plan);
    plan_update(pl, probs[i].n, probs[i].d, probs[i].k);
    pl.add<float>((size_t)probs[i].k * probs[i].d);
  }
  bool round_launch = (flags & KM_ROUND_LAUNCH) != 0;
  if (round_launch) pl.add<int>((size_t)round_ctl_words(std::min(count, kRoundMaxProbs)));
  KM_HIP(ctx->arena.ensure(pl.bytes));
  ctx->arena.reset();
  KResult* results = nullptr;
  for (int i = 0; i < count; ++i) {
    BatchState& s = S[i];
    s.bufs = carve_pass(ctx->arena, s.plan);
    s.upd = carve_update(ctx->arena, s.prob->n, s.prob->d, s.prob->k);
    s.nxt = ctx->arena.take<float>((size_t)s.prob->k * s.prob->d);
    s.cur = s.prob->C_inout;
    s.upd.X = s.prob->X;
    s.upd.labels = s.prob->labels;
    s.upd.result = s.bufs.result;
    s.upd.status = s.bufs.status;
    KM_HIP(zero_status_result(s.bufs.status, s.bufs.result, st));
    s.done = s.prob->max_iter == 0;
  }
  (void)results;
  int* round_ctl = round_launch ? ctx->arena.take<int>((size_t)round_ctl_words(std::min(count, kRoundMaxProbs)))
                                : nullptr;
  bool need_tol = false;
  for (int i = 0; i < count; ++i) need_tol |= probs[i].tol > 0.0;
  // Sweep-length tuner of the small-problem launches: the first rounds run
  // with 2, 4, 8, 16 and 32 groups per wave (never fewer than a problem's own,
  // whose partials bound the workspace; timed with events around the
  // assignment launches) and the fastest is kept for the rest.  These are
  // real rounds: labels and counts do not depend on the partition and the
  // rounds' SSE comes from the update, so results are the same whatever is
  // chosen (the final pass uses each problem's own partition).
  // A choice made before for the same shape bucket (the context's tuning
  // cache, persisted when the caller gave it a file) is used without tuning.
  static constexpr int kTuneN = 5;
  static const int kTuneGpw[kTuneN] = {2, 4, 8, 16, 32};
  bool tune = false;
  std::string tune_key;
  int cached_gpw = 0;
  {
    // every problem active through the tuning rounds, so that each round
    // times the same launches
    int64_t small_pts = 0;
    int min_iter = INT32_MAX, xd = 0, k_pad = 0;
    bool fallback = false;
    for (auto& s : S) {
      if (s.plan.xd > 0) {
        small_pts += s.prob->n;
        xd = std::max(xd, s.plan.xd);
        k_pad = std::max(k_pad, s.plan.k_pad);
        fallback |= s.plan.route == Route::Mfma;
      }
      min_iter = std::min(min_iter, (int)s.prob->max_iter);
    }
    if (small_pts > 0) {
      tune_key = TuneCache::key(p.low, p.high, fallback, xd, k_pad, small_pts);
      if (!ctx->tune.lookup(tune_key, &cached_gpw)) cached_gpw = 0;
    }
    tune = cached_gpw == 0 && !ctx->timing && !need_tol &&
           small_pts >= 2 * (int64_t)kSmallWaves * 32 * 4096 && min_iter >= kTuneN + 1;
  }
  auto apply_gpw = [&](int g) {
    for (auto& s : S)
      if (s.plan.xd > 0) {
        s.plan.gpw = std::max(g, s.plan.gpw_own);
        const int64_t ppw = (int64_t)kSmallWaves * 32 * s.plan.gpw;
        s.plan.nwg = (int)((s.prob->n + ppw - 1) / ppw);
      }
  };
  int round = 0;
  int ev_mark[kTuneN + 1] = {};
  // the tuner borrows the context's launch timing; it is off again however
  // this call returns
  struct TimingOff {
    km_context_impl* c;
    bool on;
    ~TimingOff() {
      if (on) {
        c->timing = false;
        c->ev_used = 0;
      }
    }
  } timing_off{ctx, tune};
  if (tune) {
    ctx->timing = true;
    ctx->ev_used = 0;
  }
  if (cached_gpw > 0) apply_gpw(cached_gpw);
  for (;;) {
    std::vector<BatchState*> act;
    for (auto& s : S)
      if (!s.done) act.push_back(&s);
    if (act.empty()) break;
    if (round_launch && !tune) {  // the remaining rounds in persistent launches
      round_launch = false;
      KM_HIP(enqueue_batch_rounds(ctx, S, round_ctl, st));
      continue;
    }
    if (tune && round < kTuneN) apply_gpw(kTuneGpw[round]);
    KM_HIP(enqueue_batch_round(ctx, act, st));
    if (tune && round < kTuneN) ev_mark[round + 1] = ctx->ev_used;
    if (tune && round == kTuneN - 1) {
      KM_HIP(hipEventSynchronize(ctx->timing_event(2 * ev_mark[kTuneN] - 1)));
      int best = 0;
      float best_ms = 0.0f;
      std::vector<float> times;
      for (int r = 0; r < kTuneN; ++r) {
        float tot = 0.0f;
        for (int e = ev_mark[r]; e < ev_mark[r + 1]; ++e) {
          float ms = 0.0f;
          KM_HIP(hipEventElapsedTime(&ms, ctx->timing_event(2 * e), ctx->timing_event(2 * e + 1)));
          tot += ms;
        }
        times.push_back(tot);
        if (r == 0 || tot < best_ms) {
          best = r;
          best_ms = tot;
        }
      }
      apply_gpw(kTuneGpw[best]);
      ctx->tune.store(tune_key, kTuneGpw[best], times);
      ctx->timing = false;
      ctx->ev_used = 0;
      tune = false;
    }
    ++round;
    if (need_tol) {
      for (size_t i = 0; i < act.size(); ++i)
        KM_HIP(hipMemcpyAsync(ctx->h_result + i, act[i]->bufs.result, sizeof(KResult), hipMemcpyDeviceToHost, st));
      KM_HIP(hipStreamSynchronize(st));
      for (size_t i = 0; i < act.size(); ++i)
        if (act[i]->prob->tol > 0.0 && ctx->h_result[i].shift < act[i]->prob->tol) act[i]->done = true;
    }
  }
  std::vector<BatchState*> all;
  for (auto& s : S) all.push_back(&s);
  KM_HIP(enqueue_batch_pass(ctx, all, true, st));
  for (auto& s : S)
    if (s.cur != s.prob->C_inout)
      KM_HIP(hipMemcpyAsync(s.prob->C_inout, s.cur, sizeof(float) * (size_t)s.prob->k * s.prob->d,
                            hipMemcpyDeviceToDevice, st));
  bool want_stats = (flags & KM_SYNC) != 0;
  for (int i = 0; i < count; ++i) want_stats |= probs[i].stats != nullptr;
  if (!want_stats) return KM_OK;
  for (int i = 0; i < count; ++i)
    KM_HIP(hipMemcpyAsync(ctx->h_result + i, S[i].bufs.result, sizeof(KResult), hipMemcpyDeviceToHost, st));
  KM_HIP(hipStreamSynchronize(st));
  int32_t first_err = KM_OK;
  for (int i = 0; i < count; ++i) {
    const KResult r = ctx->h_result[i];
    const int32_t ds = status_from_bits(r.status);
    if (ds != KM_OK && first_err == KM_OK) first_err = ds;
    if (probs[i].stats) {
      km_stats* o = probs[i].stats;
      o->n_corrected = S[i].plan.route == Route::Direct64Exact ? 0 : r.n_corrected;
      o->n_pairs = r.n_pairs;
      o->iters = S[i].it;
      o->data_status = ds;
      o->sse_last = r.sse;
      o->shift_last = r.shift;
      o->alpha_used = S[i].plan.alpha_used;
    }
  }
  return first_err;
}
