// km_internal.hpp -- structures shared by the host-side library code and the
// kernels (problem descriptors passed to the device) and the launcher
// declarations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace km {

constexpr int kLowFP16 = 0;
constexpr int kLowBF16 = 1;
constexpr int kLowFP32 = 2;
constexpr int kExact64 = 3;

// Status bits raised by the kernels (a single int per problem).
constexpr int kStatusNonFinite = 1;
constexpr int kStatusRange = 2;
constexpr int kStatusBadLabel = 4;
constexpr int kStatusSync = 8;  // a grid-wide wait of the persistent round kernel gave up

// Padded coordinate extent of the matrix-core kernels (multiple of the K
// extent of one instruction; 16 for every format so layouts agree).
constexpr int padded_dim(int d) {
  return d <= 16 ? 16 : d <= 32 ? 32 : d <= 64 ? 64 : d <= 128 ? 128 : d <= 256 ? 256 : -1;
}

// 32-point column blocks per wave (the point fragments of all of them stay in
// registers for the whole sweep over the centres).
constexpr int mfma_nb(int low, int DP) {
  return low == kLowFP32 ? (DP <= 32 ? 2 : 1) : (DP <= 128 ? 2 : 1);
}
constexpr int mfma_points_per_wg(int low, int DP) { return 4 * 32 * mfma_nb(low, DP); }
// workgroup of the pipelined assignment kernel
constexpr int kPipeWaves = 8;
constexpr int kPipeThreads = 64 * kPipeWaves;
constexpr int pipe_points_per_wg(int low, int DP) { return kPipeWaves * 32 * mfma_nb(low, DP); }
// points per workgroup of the assignment-mode kernel
constexpr int assign_points_per_wg(int low, int DP) { return pipe_points_per_wg(low, DP); }
constexpr int kDirectPointsPerWg = 128;
// small-problem assignment kernel (d <= 32, k <= 64): four waves, each
// sweeping `gpw` groups of 32 points
constexpr int kSmallWaves = 4;
constexpr int kSmallThreads = 64 * kSmallWaves;
constexpr int kSmallMaxD = 32;
constexpr int kSmallMaxK = 64;
// register capacity of a point row in the small-problem kernel
constexpr int small_xd(int d) { return d <= 8 ? 8 : d <= 16 ? 16 : d <= 32 ? 32 : 0; }

// Accumulated per-problem results on the device.
struct KResult {
  double sse;               // SSE of the last assignment pass
  long long n_corrected;    // summed over passes
  long long n_pairs;        // summed over passes
  int status;               // OR of the status bits seen
  int pad;
  double shift;             // max centre move of the last update
};

struct PrepProb {
  const float* C;  // k x d FP32
  void* Cq;        // k_pad x DP low precision (output)
  float* cinit;    // k_pad (output)
  float* ca;       // k_pad (output)
  int* status;
  float alpha;
  int k, k_pad, d, DP;
};

struct AssignProb {
  const float* X;       // n x d
  const float* C;       // k x d (FP32 originals, for the FP64 direct formula)
  const void* Cq;       // k_pad x DP quantised centres
  const float* cinit;   // k_pad
  const float* ca;      // k_pad
  int32_t* labels;      // n
  float* mindist;       // n, nullable
  float* D;             // pairwise mode: n x k
  uint8_t* flagged;     // n x k, nullable: pairwise mode, every pair's flag; assignment
                        // mode, 1 written for each pair the test sends to the fallback
  double* sse_part;     // one per workgroup of this problem
  unsigned long long* corr_part;
  int* status;
  int64_t n;
  int d, k, k_pad;
  float oma;            // 1 - alpha (FP32)
  int refine;           // 1: FP64 winner refinement, mindist and SSE partials;
                        // 0: labels and counters only (SSE left to the update)
  const int32_t* hint;  // nullable: an earlier assignment (seeds the search)
  int gpw;              // small-problem kernel: 32-point groups per wave
  float alpha;          // small-problem kernel: alpha (FP32), for its own centre constants
  int high;             // correction precision of flagged pairs (kHigh64 / kHigh32 / kHighLow)
};

struct ReduceProb {
  const double* sse_part;
  const unsigned long long* corr_part;
  const int* status;
  double* sse_out;      // nullable (caller's scalar)
  KResult* result;      // nullable
  long long pairs;
  int nparts;
};

// Centre update, one problem.
struct UpdateProb {
  const float* X;
  const int32_t* labels;
  const float* C_old;
  float* C_new;
  long long* counts_out;   // k, nullable
  double* shift_out;       // nullable
  KResult* result;         // nullable
  // workspace
  int32_t* hist;           // k * ntiles (cluster-major)
  int32_t* offs;           // k * ntiles
  int32_t* perm;           // n
  int32_t* cstart;         // k+1 cluster starts in perm
  int32_t* chunk_start;    // k+1 chunk starts
  double* chunk_sum;       // (n/64 + k) * d
  double* sse_chunk;       // n/64 + k: per-chunk SSE partials
  double* shift2;          // k
  double* sse_out;         // nullable: SSE of the labels against C_old (FP64)
  int* status;
  int64_t n;
  int d, k, ntiles;
  int chunk;               // members per partial sum (upd_chunk(d))
  // owner path (owners > 0, small k*d): per-chunk FP64 partials
  double* pacc;            // nchunk * k * d
  int32_t* pcnt;           // nchunk * k
  double* psse;            // nchunk
  int owners, lp, nc, nchunk;
  int iters;               // points per owner per chunk (own_iters)
};

hipError_t launch_prep(int low, const PrepProb* dprobs, const int32_t* dstart, int nprob, int nwg,
                       hipStream_t st);
// mode: 0 assignment, 1 materialised pairs, 2 assignment writing P.flagged
hipError_t launch_assign_mfma(int low, int DP, int mode, bool fallback, const AssignProb* dprobs,
                              const int32_t* dstart, int nprob, int nwg, hipStream_t st);
hipError_t launch_assign_small(int low, int xd, bool fallback, const AssignProb* dprobs, const int32_t* dstart,
                               int nprob, int nwg, hipStream_t st);
// arith: 0 FP64, 1 FP32, 2 binary16, 3 bfloat16 (direct formula arithmetic)
hipError_t launch_assign_direct64(bool cmp64, int arith, int mode, const AssignProb* dprobs,
                                  const int32_t* dstart, int nprob, int nwg, hipStream_t st);
hipError_t launch_reduce_parts(const ReduceProb* dprobs, int nprob, hipStream_t st);
hipError_t launch_gather_results(const KResult* const* dsrc, int count, KResult* ddst, hipStream_t st);
hipError_t launch_zero_words(void* p, size_t bytes, hipStream_t st);  // bytes rounded up to 4
hipError_t launch_fill_bytes(void* p, int64_t count, uint8_t v, hipStream_t st);
hipError_t launch_quantize(int low, const float* in, int64_t count, uint16_t* out, hipStream_t st);

// centre update (km_update.hip)
constexpr int kUpdTile = 1024;   // points per histogram / scatter tile
constexpr int kUpdChunk = 64;    // members per partial sum (the smallest; workspace bound)
// Members per partial sum: rows of a few coordinates carry little work per
// member, so a wave takes longer runs of them.
constexpr int upd_chunk(int d) { return d <= 16 ? 8 * kUpdChunk : kUpdChunk; }
hipError_t launch_update(const UpdateProb* dprobs, const UpdateProb* hprobs, int nprob,
                         const int32_t* dscratch_i32, hipStream_t st);

// Owner path of the centre update, for small k*d: a wave's lanes are split
// into `owners` groups of `lp` lanes; each group takes every owners-th point
// of the wave's run and adds its row into its own FP64 accumulators of all k
// clusters in LDS (one lane per coordinate, `nc` coordinates per lane), so
// each accumulator has a single writer and a fixed order.
constexpr int kOwnWaves = 4;            // waves per workgroup
constexpr int kOwnIters = 256;          // points per owner per chunk (at most)
constexpr int kOwnItersMin = 32;        // (at least: two batches of 16 in flight)
constexpr int kOwnChunksWanted = 32;    // chunks a problem should have
constexpr int kOwnWaveBytes = 34816;    // LDS per wave: accumulators + counts
constexpr int kOwnCentreFloats = 4096;  // LDS staging of C_old (k*d floats)
struct OwnShape {
  int owners, lp, nc;
};
inline OwnShape own_shape(int d, int k) {
  OwnShape s{0, 0, 0};
  if (d < 1 || d > 128 || k < 1 || (int64_t)k * d > kOwnCentreFloats) return s;
  s.nc = (d + 63) / 64;
  s.lp = (d + s.nc - 1) / s.nc;
  const int64_t per_owner = (int64_t)k * d * 8 + (int64_t)k * 4;
  const int64_t fit = kOwnWaveBytes / per_owner;
  const int lanes = 64 / s.lp;
  s.owners = (int)(fit < lanes ? fit : lanes);
  if (s.owners < 1) s = OwnShape{0, 0, 0};
  return s;
}
// k-means++ seeding (km_seed.hip); u: host array of k uniforms in [0, 1);
// workspace w [n] FP64, bsum [ceil(n/1024)] FP64, pick [1] int32
hipError_t launch_seed_pp(const float* X, int64_t n, int d, int k, const double* u, float* C, int32_t* idx,
                          double* w, double* bsum, int32_t* pick, hipStream_t st);

// LDS of one wave's accumulators and counts (16-byte multiple)
inline int own_wave_bytes(int owners, int d, int k) {
  return (int)((((int64_t)owners * ((int64_t)k * d * 8 + (int64_t)k * 4)) + 15) / 16 * 16);
}
// points per chunk (one workgroup)
inline int64_t own_chunk(const OwnShape& s, int iters) { return (int64_t)kOwnWaves * s.owners * iters; }
// Points per owner per chunk: 256, halved (down to 32) while the problem has
// fewer than kOwnChunksWanted chunks.  An owner's points are a chain of
// dependent global-load batches, so a small problem cut in few long chunks
// is latency-bound on a handful of workgroups; the choice depends on (n, d,
// k) only, so results stay the same alone, batched and served.
inline int own_iters(int64_t n, const OwnShape& s) {
  int it = kOwnIters;
  while (it > kOwnItersMin && (n + own_chunk(s, it) - 1) / own_chunk(s, it) < kOwnChunksWanted) it >>= 1;
  return it;
}
// clusters per finalize workgroup
constexpr int own_fin_clusters(int d) { return d >= 256 ? 1 : 256 / d; }
// Persistent Lloyd rounds of small problems (d <= 32, k <= 64, owner-path
// update): one launch runs every round of every problem in the list --
// assignment tiles, update chunks, the reduction of the assignment partials
// and the finalize of each cluster group, then per problem shift, SSE and
// the stopping test -- with grid-wide waits between the phases.  Round r of a problem uses
// a[r & 1] and u[r & 1] (centres C_old -> C_new of that round); every body is
// the one of the one-launch-per-phase kernels, so the results are bitwise
// theirs.
struct RoundProb {
  AssignProb a[2];
  UpdateProb u[2];
  ReduceProb red;
  double* sse_hist;  // nullable: SSE of round r at [r]
  double tol;        // > 0: stop after a round whose shift is below tol
  int max_iter;      // >= 1
  int nfin;          // finalize cluster groups
  int wstride;       // LDS stride of the update's wave regions
  int pad;
};
// Control words (device, zeroed before the launch): [0] wait arrivals,
// [1] abort flag, [2, 2 + nprob) done flags, [2 + nprob, 2 + 2 nprob) rounds
// run per problem.
constexpr int round_ctl_words(int nprob) { return 2 + 2 * nprob; }
constexpr int kRoundMaxProbs = 1024;  // problems of one persistent launch
// tpre, cpre, fpre: prefixes of the problems' assignment tiles, update
// chunks and finalize items (1 + nfin each).  Returns the runtime's error
// when the grid cannot be co-resident; the caller then runs one launch per
// phase.
// max_spins: polls after which a grid-wide wait gives up (kSyncSpins unless
// the KM_ROUND_SPIN_LIMIT environment variable sets it: tests of that path).
constexpr unsigned kSyncSpins = 1u << 25;  // s_sleep(2) polls: well over a second
hipError_t launch_lloyd_rounds(int low, int xd, bool fallback, const RoundProb* dprobs, int nprob,
                               const int32_t* tpre, const int32_t* cpre, const int32_t* fpre, int* ctl,
                               int work_items, int lds_bytes, unsigned max_spins, hipStream_t st);
int small_lds_bytes(int xd, bool fallback);

hipError_t launch_update_own_part(const UpdateProb* dprobs, const UpdateProb* hprobs, int nprob,
                                  const int32_t* dpre, hipStream_t st);
// shift = false leaves the shift and SSE to the caller (launch_round_tail)
hipError_t launch_update_own_fin(const UpdateProb* dprobs, const UpdateProb* hprobs, int nprob,
                                 const int32_t* dpre, hipStream_t st, bool shift = true);
// One problem's partial reduction (as k_reduce_parts) then owner-path shift
// and SSE (as k_upd_own_shift), in one launch.
hipError_t launch_round_tail(const ReduceProb* drp, const UpdateProb* dup, hipStream_t st);

}  // namespace km
