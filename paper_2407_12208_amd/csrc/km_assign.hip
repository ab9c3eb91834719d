// km_assign.hip -- assignment-pass kernels for gfx950.
//
//  k_prep_centroids  quantises the centres (round to nearest even) into a
//                    dense [k_pad x DP] low-precision array and forms the
//                    per-centre constants of the fused epilogue.
//  k_assign_mfma     one workgroup per tile of points: each lane loads its
//                    matrix-core fragments of the FP32 points once from HBM,
//                    rounds them to the low format and keeps them in
//                    registers for the whole sweep over all centres
//                    (double-buffered LDS tiles) with 32x32 MFMAs, and fuses
//                    the expanded formula, the reliability test, the FP64
//                    direct correction of flagged pairs, the argmin, the FP64
//                    winner refinement and per-tile SSE / counter partials.
//  k_assign_direct64 every pair by the FP64 direct formula (the plain FP64
//                    baseline and the dense-fallback path when the threshold
//                    makes every pair fail the test).
//  k_reduce_parts    fixed-order sums of the per-tile partials.
//  k_quantize        element-wise conversion (tests of the rounding).
//
// All kernels take an array of problem descriptors and a prefix array of
// workgroup counts, so one launch can serve many independent problems; a
// problem's arithmetic never depends on the other problems in the launch.
#include "km_device.hpp"
#include "km_internal.hpp"
#include "km_update_dev.hpp"

namespace km {

__device__ __noinline__ double sqdist64_call(const float* __restrict__ x, const float* __restrict__ c, int d) {
  return sqdist64(x, c, d);
}

__device__ __noinline__ double corr_dist_call(int high, int fmt, const float* x, const float* c, int d) {
  return high == kHigh64 ? sqdist64(x, c, d) : corr_dist(high, fmt, x, c, d);
}

// Correction of a flagged pair in the problem's correction precision: one
// out-of-line call with the arguments of the plain FP64 one (d and the
// precision share a register; d < 2^16), so the sweep keeps its registers.
template <class L>
__device__ __noinline__ double correct_pair_call(const float* x, const float* c, int d_high) {
  const int d = d_high & 0xffff, high = d_high >> 16;
  return high == kHigh64 ? sqdist64(x, c, d) : corr_dist(high, L::kFmt, x, c, d);
}
template <class L>
__device__ inline double correct_pair(const AssignProb& P, const float* x, const float* c, int d) {
  return correct_pair_call<L>(x, c, d | (P.high << 16));
}

// Maximum of the 16 accumulator registers (a v_max3 tree).
__device__ inline float max16(const f32x16& v) {
  const float a = __builtin_fmaxf(__builtin_fmaxf(v[0], v[1]), v[2]);
  const float b = __builtin_fmaxf(__builtin_fmaxf(v[3], v[4]), v[5]);
  const float c = __builtin_fmaxf(__builtin_fmaxf(v[6], v[7]), v[8]);
  const float e = __builtin_fmaxf(__builtin_fmaxf(v[9], v[10]), v[11]);
  const float f = __builtin_fmaxf(__builtin_fmaxf(v[12], v[13]), v[14]);
  const float g = __builtin_fmaxf(__builtin_fmaxf(a, b), c);
  const float h = __builtin_fmaxf(__builtin_fmaxf(e, f), v[15]);
  return __builtin_fmaxf(g, h);
}

// Problem index of workgroup b: largest p with wg_start[p] <= b.
__device__ inline int find_problem(const int32_t* __restrict__ wg_start, int nprob, int b) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (wg_start[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ inline void raise_status(int* status, int bits) {
  // one atomic per wave that saw a problem
  unsigned long long m = __ballot(bits != 0);
  if (m) {
    int all = bits;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) all |= __shfl_xor(all, o, kWave);
    if ((threadIdx.x & 63) == (int)(__ffsll((long long)m) - 1)) atomicOr(status, all);
  }
}

// ---------------------------------------------------------------------------
// Winner refinement of a wave's points: mindist_i = fl32(sum_l (x_il -
// c_{label_i,l})^2) with the sum in FP64.  Sixteen lanes share one point:
// each reads its coordinates (8 consecutive ones per 128-coordinate pass,
// float4 loads when the rows allow it) so that a group of 16 lanes reads 512
// contiguous bytes; the lane partials are combined by a fixed butterfly.
// labs[q] is the label of point pbase+q (q < nloc).  Returns this lane's part
// of the wave's SSE (lanes 0, 16, 32, 48 hold the point sums).
// ---------------------------------------------------------------------------
__device__ inline double refine_wave(const AssignProb& P, int64_t pbase, int nloc, const int* labs,
                                     int lane) {
  const int d = P.d;
  const int sub = lane & 15;
  const bool vec = ((d & 3) == 0) && (((((uintptr_t)P.X) | ((uintptr_t)P.C)) & 15) == 0);
  double sse = 0.0;
  for (int q0 = 0; q0 < nloc; q0 += 4) {
    const int q = q0 + (lane >> 4);
    const bool on = q < nloc;
    const int lab = on ? labs[q] : 0;
    const KM_GLOBAL float* xr = as_global(P.X) + (pbase + (on ? q : 0)) * d;
    const KM_GLOBAL float* cr = as_global(P.C) + (int64_t)lab * d;
    double part = 0.0;
    for (int l0 = 8 * sub; l0 < d; l0 += 128) {
      if (vec) {
#pragma unroll
        for (int h = 0; h < 8; h += 4) {
          if (l0 + h < d) {
            const f32x4 a = *reinterpret_cast<const KM_GLOBAL f32x4*>(xr + l0 + h);
            const f32x4 b = *reinterpret_cast<const KM_GLOBAL f32x4*>(cr + l0 + h);
            const double e0 = (double)a.x - (double)b.x, e1 = (double)a.y - (double)b.y;
            const double e2 = (double)a.z - (double)b.z, e3 = (double)a.w - (double)b.w;
            part = __builtin_fma(e0, e0, part);
            part = __builtin_fma(e1, e1, part);
            part = __builtin_fma(e2, e2, part);
            part = __builtin_fma(e3, e3, part);
          }
        }
      } else {
        for (int e = 0; e < 8 && l0 + e < d; ++e) {
          const double t = (double)xr[l0 + e] - (double)cr[l0 + e];
          part = __builtin_fma(t, t, part);
        }
      }
    }
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) part += __shfl_xor(part, o, kWave);
    if (on && sub == 0) {
      if (P.mindist) as_global(P.mindist)[pbase + q] = (float)part;
      sse += part;
    }
  }
  return sse;
}

// ---------------------------------------------------------------------------
// Centre preparation.  One wave per (padded) centre row, lanes over the
// coordinates.
//   Cq[j, 0:DP]  = RNE_low(C[j, 0:d]), zero padded
//   nc_j         = sum_l Cq[j,l]^2 in FP32 (each lane sums its coordinates
//                  l = lane, lane+64, ... in order, then a fixed butterfly):
//                  the norm of the quantised centre, as the expanded formula
//                  requires
//   cinit[j]     = -nc_j / 2          (accumulator start of the cross term)
//   ca[j]        = alpha * nc_j / 2   (centre part of the reliability test)
// Padded rows j >= k: cinit = -inf, ca = 0, so they never win and never fail
// the test.
// ---------------------------------------------------------------------------
template <class L>
__global__ void __launch_bounds__(256)
k_prep_centroids(const PrepProb* __restrict__ probs, const int32_t* __restrict__ wg_start, int nprob) {
  const int pi = find_problem(wg_start, nprob, blockIdx.x);
  const PrepProb& P = probs[pi];
  const int lane = threadIdx.x & 63;
  const int j = (blockIdx.x - wg_start[pi]) * 4 + (threadIdx.x >> 6);
  if (j >= P.k_pad) return;
  KM_GLOBAL typename L::S* out = reinterpret_cast<KM_GLOBAL typename L::S*>(as_global(P.Cq)) + (int64_t)j * P.DP;
  int bad = 0;
  float s = 0.0f;
  const bool valid = j < P.k;
  for (int l = lane; l < P.DP; l += 64) {
    float v = 0.0f;
    if (valid && l < P.d) {
      v = as_global(P.C)[(int64_t)j * P.d + l];
      if (!__builtin_isfinite(v)) bad |= kStatusNonFinite;
      if (L::kHasRange && __builtin_fabsf(v) >= L::kOverflow) bad |= kStatusRange;
    }
    const typename L::S q = L::cvt(v);
    out[l] = q;
    const float f = L::tof(q);
    s = __builtin_fmaf(f, f, s);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, kWave);
  if (lane == 0) {
    if (valid) {
      const float hc = 0.5f * s;
      as_global(P.cinit)[j] = -hc;
      as_global(P.ca)[j] = P.alpha * hc;
    } else {
      as_global(P.cinit)[j] = -__builtin_inff();
      as_global(P.ca)[j] = 0.0f;
    }
  }
  raise_status(P.status, bad);
}

// ---------------------------------------------------------------------------
// Fused mixed-precision assignment.
//
// Per pair (x~ = RNE(x), c~ = RNE(c)) the accumulator holds
//     W = -nc/2 + x~^T c~                      (FP32 accumulation)
// so that the expanded distance is d^ = nx + nc - 2 x~^T c~ = nx - 2W and the
// reliability test  d^ > alpha (nx + nc)  (keep) reads
//     W + alpha nc/2 < (1 - alpha) nx / 2,
// i.e. a pair is corrected iff  W + ca_j >= hx_i.  The kept pair with the
// largest W has the smallest d^.  Corrected pairs are recomputed in FP64 by
// the direct formula from the FP32 data and rounded once to FP32.
//
// MODE 0: argmin + refinement + partials.  MODE 1: write every pair's value
// and flag (materialised distances for reports and tests).
// ---------------------------------------------------------------------------
template <class L, int DP, int NB, int WAVES = 4>
struct AssignCfg {
  static constexpr int kWaves = WAVES;
  static constexpr int kPts = kWaves * NB * 32;           // points per workgroup
  static constexpr int kLd = DP + (L::KS == 2 ? 4 : 8);   // LDS row stride (elements)
  static constexpr int kCt = 64;                          // centres per LDS tile
  static constexpr int kSteps = DP / L::KS;
  static constexpr int kBytes = 2 * kCt * kLd * (int)sizeof(typename L::S);
  // 16-byte chunks of one centre tile in global memory
  static constexpr int kChunks = kCt * DP * (int)sizeof(typename L::S) / 16;
  static constexpr int kChunksPerThread = (kChunks + kWaves * 64 - 1) / (kWaves * 64);
  static constexpr int kElemsPerChunk = 16 / (int)sizeof(typename L::S);
};

template <class L, int DP, int NB, int MODE, bool FALLBACK>
__global__ void __launch_bounds__(256, 2)
k_assign_mfma(const AssignProb* __restrict__ probs, const int32_t* __restrict__ wg_start, int nprob) {
  using Cfg = AssignCfg<L, DP, NB>;
  using S = typename L::S;
  constexpr int LD = Cfg::kLd;
  constexpr int CT = Cfg::kCt;

  __shared__ __attribute__((aligned(16))) unsigned char smem[Cfg::kBytes];
  __shared__ float s_cinit[2][CT];
  __shared__ float s_ca[2][CT];
  __shared__ double s_sse[Cfg::kWaves];
  __shared__ unsigned long long s_corr[Cfg::kWaves];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int pi = find_problem(wg_start, nprob, blockIdx.x);
  const AssignProb& P = probs[pi];
  const int tile = blockIdx.x - wg_start[pi];
  const int64_t p0 = (int64_t)tile * Cfg::kPts;
  const int64_t n = P.n;
  const int d = P.d;
  const int nvalid = (int)((n - p0) < Cfg::kPts ? (n - p0) : Cfg::kPts);

  // ---- prologue: each lane loads its matrix-core fragments of the FP32
  // points straight from HBM, rounds them (RNE) to the low format and forms
  // the squared norm of the quantised point (FP32; each lane half sums its
  // own K elements in order, the two halves are then added).
  typename L::frag bfr[NB][Cfg::kSteps];
  float nx[NB], hx[NB];
  const int pw = wave * NB * 32;  // first point of this wave within the tile
  int bad = 0;
  const bool vec4 = ((d & 3) == 0) && ((((uintptr_t)P.X) & 15) == 0);
  // full tile, no coordinate padding: unconditional streaming loads
  const bool fast = vec4 && d == DP && nvalid == Cfg::kPts;
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    const int pl = pw + cb * 32 + (lane & 31);
    const bool pv = pl < nvalid;
    const KM_GLOBAL float* xr = as_global(P.X) + (p0 + (pv ? pl : 0)) * d;
    float part = 0.0f;
#pragma unroll
    for (int s = 0; s < Cfg::kSteps; ++s) {
      const int o = s * L::KS + (lane >> 5) * L::KV;
      float v[L::KV];
      if constexpr (L::KV % 4 == 0) {
        if (fast) {
#pragma unroll
          for (int u = 0; u < L::KV; u += 4) {
            const f32x4 q = *reinterpret_cast<const KM_GLOBAL f32x4*>(xr + o + u);
            v[u] = q[0]; v[u + 1] = q[1]; v[u + 2] = q[2]; v[u + 3] = q[3];
          }
        } else if (vec4) {
#pragma unroll
          for (int u = 0; u < L::KV; u += 4) {
            f32x4 q = {0.f, 0.f, 0.f, 0.f};
            if (pv && o + u < d) q = *reinterpret_cast<const KM_GLOBAL f32x4*>(xr + o + u);
            v[u] = q[0]; v[u + 1] = q[1]; v[u + 2] = q[2]; v[u + 3] = q[3];
          }
        } else {
#pragma unroll
          for (int u = 0; u < L::KV; ++u) v[u] = (pv && o + u < d) ? xr[o + u] : 0.0f;
        }
      } else {
#pragma unroll
        for (int u = 0; u < L::KV; ++u) v[u] = (pv && o + u < d) ? xr[o + u] : 0.0f;
      }
      typename L::frag f;
#pragma unroll
      for (int u = 0; u < L::KV; ++u) {
        if (!__builtin_isfinite(v[u])) bad |= kStatusNonFinite;
        if (L::kHasRange && __builtin_fabsf(v[u]) >= L::kOverflow) bad |= kStatusRange;
        const S q = L::cvt(v[u]);
        if constexpr (L::KV == 1) f = q; else f[u] = q;
        const float qf = L::tof(q);
        part = __builtin_fmaf(qf, qf, part);
      }
      bfr[cb][s] = f;
    }
    const float other = __shfl_xor(part, 32, kWave);
    nx[cb] = (lane < 32) ? part + other : other + part;
    // points past the end never fail the test (no correction reads there)
    hx[cb] = pv ? 0.5f * (P.oma * nx[cb]) : __builtin_inff();
  }
  raise_status(P.status, bad);

  S* const sc0 = reinterpret_cast<S*>(smem);  // two buffers of CT rows

  // running state per column block: best kept value (largest W), the block
  // where it occurred and a copy of that block's 16 accumulator values (the
  // index inside the block is recovered once, after the sweep); best
  // corrected pair (smallest FP64-direct value rounded to FP32)
  float bw[NB];
  int bb[NB];
  f32x16 sv[NB];
  float cd[NB];
  int cj[NB];
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    bw[cb] = -__builtin_inff();
    bb[cb] = -1;
    cd[cb] = __builtin_inff();
    cj[cb] = -1;
#pragma unroll
    for (int r = 0; r < 16; ++r) sv[cb][r] = -__builtin_inff();
  }
  unsigned long long ncorr = 0;

  // per-lane queue of flagged pairs (centre index | column block << 24)
  constexpr int kQueue = 12;
  __shared__ int s_q[FALLBACK ? kQueue * 256 : 1];
  int qn = 0;
  auto flush_queue = [&]() {
    if constexpr (FALLBACK) {
      for (int q = 0; q < qn; ++q) {
        const int e = s_q[q * 256 + tid];
        const int j = e & 0xffffff;
        const int cbq = e >> 24;
        const int pl = pw + cbq * 32 + (lane & 31);
        const double dd = P.high == kHigh64 ? sqdist64(P.X + (p0 + pl) * d, P.C + (int64_t)j * d, d)
                                            : corr_dist_call(P.high, L::kFmt, P.X + (p0 + pl) * d,
                                                             P.C + (int64_t)j * d, d);
        const float df = (float)dd;
        ncorr += 1;
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
          if (cb != cbq) continue;
          if constexpr (MODE == 0) {
            if (df < cd[cb] || (df == cd[cb] && j < cj[cb])) {
              cd[cb] = df;
              cj[cb] = j;
            }
          } else {
            const int64_t o = (p0 + pl) * (int64_t)P.k + j;
            as_global(P.D)[o] = df;
            if (P.flagged) as_global(P.flagged)[o] = 1;
          }
        }
      }
      qn = 0;
    }
  };

  const int kpad = P.k_pad;
  const int ntile = (kpad + CT - 1) / CT;
  const KM_GLOBAL S* Cq = reinterpret_cast<const KM_GLOBAL S*>(as_global(P.Cq));

  // global -> register staging of one centre tile (16-byte chunks)
  f32x4 stage[Cfg::kChunksPerThread];
  float st_ci = 0.f, st_ca = 0.f;
  auto load_tile = [&](int t) {
    const int rows = (kpad - t * CT) < CT ? (kpad - t * CT) : CT;
    const KM_GLOBAL f32x4* g = reinterpret_cast<const KM_GLOBAL f32x4*>(Cq + (int64_t)t * CT * DP);
    const int nchunk = rows * DP / Cfg::kElemsPerChunk;
#pragma unroll
    for (int u = 0; u < Cfg::kChunksPerThread; ++u) {
      const int c = tid + u * 256;
      if (c < nchunk) stage[u] = g[c];
    }
    if (tid < rows) {
      st_ci = as_global(P.cinit)[t * CT + tid];
      st_ca = as_global(P.ca)[t * CT + tid];
    }
  };
  auto store_tile = [&](int t, int buf) {
    const int rows = (kpad - t * CT) < CT ? (kpad - t * CT) : CT;
    const int nchunk = rows * DP / Cfg::kElemsPerChunk;
    constexpr int CPR = DP / Cfg::kElemsPerChunk;  // chunks per row
#pragma unroll
    for (int u = 0; u < Cfg::kChunksPerThread; ++u) {
      const int c = tid + u * 256;
      if (c < nchunk) {
        const int row = c / CPR, col = (c % CPR) * Cfg::kElemsPerChunk;
        *reinterpret_cast<f32x4*>(sc0 + buf * CT * LD + row * LD + col) = stage[u];
      }
    }
    if (tid < rows) {
      s_cinit[buf][tid] = st_ci;
      s_ca[buf][tid] = st_ca;
    }
  };

  load_tile(0);
  store_tile(0, 0);
  __syncthreads();

  for (int t = 0; t < ntile; ++t) {
    const int buf = t & 1;
    if (t + 1 < ntile) load_tile(t + 1);
    const int rows = (kpad - t * CT) < CT ? (kpad - t * CT) : CT;
    uint32_t fmask[2][NB];
#pragma unroll
    for (int bk = 0; bk < 2; ++bk)
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) fmask[bk][cb] = 0;
    for (int bk = 0; bk < rows / 32; ++bk) {
      const int jb = t * CT + bk * 32;  // first centre of this 32-block
      // all A fragments of the block first (their LDS latency overlaps)
      typename L::frag af[Cfg::kSteps];
      const S* arow = sc0 + buf * CT * LD + (bk * 32 + (lane & 31)) * LD + (lane >> 5) * L::KV;
#pragma unroll
      for (int s = 0; s < Cfg::kSteps; ++s) {
        if constexpr (L::KV == 1) af[s] = arow[s * L::KS];
        else af[s] = *reinterpret_cast<const typename L::frag*>(arow + s * L::KS);
      }
      f32x16 acc[NB];
      {
        f32x16 ci;
#pragma unroll
        for (int r = 0; r < 16; ++r) ci[r] = s_cinit[buf][bk * 32 + acc_row(r, lane)];
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) acc[cb] = L::mfma(af[0], bfr[cb][0], ci);
      }
#pragma unroll
      for (int s = 1; s < Cfg::kSteps; ++s)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) acc[cb] = L::mfma(af[s], bfr[cb][s], acc[cb]);

      // ---- epilogue ----
      f32x16 cav;
      if constexpr (FALLBACK) {
#pragma unroll
        for (int r = 0; r < 16; ++r) cav[r] = s_ca[buf][bk * 32 + acc_row(r, lane)];
      }
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        f32x16 w = acc[cb];
        if constexpr (MODE == 0) {
          if constexpr (FALLBACK) {
            // any pair failing the test  W + ca >= hx  in this block?
            f32x16 tv = w + cav;
            const float tm = max16(tv);
            if (__ballot(tm >= hx[cb])) {  // rare: wave-uniform slow path
              uint32_t fm = 0;
#pragma unroll
              for (int r = 0; r < 16; ++r) {
                const bool f = tv[r] >= hx[cb];
                fm |= (uint32_t)f << r;
                w[r] = f ? -__builtin_inff() : w[r];
              }
              fmask[bk][cb] = fm;
            }
          }
          const float wm = max16(w);
          const bool imp = wm > bw[cb];  // strict: the earlier block keeps ties
          bw[cb] = imp ? wm : bw[cb];
          bb[cb] = imp ? jb : bb[cb];
#pragma unroll
          for (int r = 0; r < 16; ++r) sv[cb][r] = imp ? w[r] : sv[cb][r];
        } else {
          const int pl = pw + cb * 32 + (lane & 31);
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int j = jb + acc_row(r, lane);
            const bool flag = FALLBACK && (w[r] + cav[r] >= hx[cb]);
            if (flag) fmask[bk][cb] |= 1u << r;
            if (!flag && pl < nvalid && j < P.k) {
              const int64_t o = (p0 + pl) * (int64_t)P.k + j;
              as_global(P.D)[o] = __builtin_fmaxf(nx[cb] - 2.0f * w[r], 0.0f);
              if (P.flagged) as_global(P.flagged)[o] = 0;
            }
          }
        }
      }
    }
    // queue this tile's flagged pairs; they are corrected in batches (one
    // memory round trip per batch instead of one per tile)
    if constexpr (FALLBACK) {
#pragma unroll
      for (int bk = 0; bk < 2; ++bk)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
          uint32_t fm = fmask[bk][cb];
          const int pl = pw + cb * 32 + (lane & 31);
          if (pl >= nvalid) fm = 0;
          while (fm) {
            const int r = __builtin_ctz(fm);
            fm &= fm - 1;
            const int j = t * CT + bk * 32 + acc_row(r, lane);
            if (j < P.k) {
              if (qn == kQueue) {  // full: flush this lane's queue first
                flush_queue();
              }
              s_q[qn * 256 + tid] = j | (cb << 24);
              qn += 1;
            }
          }
        }
      // a lane with a full queue forces a batch for the whole wave
      if (__ballot(qn >= kQueue - 2 * NB * 2)) flush_queue();
    }
    if (t + 1 < ntile) store_tile(t + 1, buf ^ 1);
    __syncthreads();
  }

  flush_queue();

  // ---- index of the best kept pair, merge the two lanes that share a
  // point, choose between kept and corrected, refine in FP64 --------------
  double sse = 0.0;
  if constexpr (MODE == 0) {
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      // first register of the saved block holding the best value
      int rs = 16;
#pragma unroll
      for (int r = 15; r >= 0; --r) rs = (sv[cb][r] == bw[cb]) ? r : rs;
      int bj = (bb[cb] >= 0 && rs < 16) ? bb[cb] + acc_row(rs, lane) : -1;
      float ow = __shfl_xor(bw[cb], 32, kWave);
      int oj = __shfl_xor(bj, 32, kWave);
      if (ow > bw[cb] || (ow == bw[cb] && oj >= 0 && (bj < 0 || oj < bj))) {
        bw[cb] = ow;
        bj = oj;
      }
      float od = __shfl_xor(cd[cb], 32, kWave);
      int ojc = __shfl_xor(cj[cb], 32, kWave);
      if (od < cd[cb] || (od == cd[cb] && ojc >= 0 && (cj[cb] < 0 || ojc < cj[cb]))) {
        cd[cb] = od;
        cj[cb] = ojc;
      }
      bb[cb] = bj;  // now the best kept centre index
    }
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      if ((cb & 1) != (lane >> 5)) continue;  // lane half cb%2 finishes block cb
      const int pl = pw + cb * 32 + (lane & 31);
      if (pl >= nvalid) continue;
      const float dk = bb[cb] >= 0 ? __builtin_fmaxf(nx[cb] - 2.0f * bw[cb], 0.0f) : __builtin_inff();
      int lab = bb[cb];
      if (cj[cb] >= 0 && (cd[cb] < dk || (cd[cb] == dk && cj[cb] < lab) || lab < 0)) lab = cj[cb];
      if (lab < 0 || lab >= P.k) lab = 0;  // only with non-finite data (status raised)
      const int64_t p = p0 + pl;
      const double dd = sqdist64(P.X + p * d, P.C + (int64_t)lab * d, d);
      as_global(P.labels)[p] = lab;
      if (P.mindist) as_global(P.mindist)[p] = (float)dd;
      sse += dd;
    }
  }
  sse = wave_sum(sse);
  unsigned long long nc = wave_sum_u64(ncorr);
  if (lane == 0) {
    s_sse[wave] = sse;
    s_corr[wave] = nc;
  }
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    unsigned long long c = 0;
#pragma unroll
    for (int w = 0; w < Cfg::kWaves; ++w) {
      s += s_sse[w];
      c += s_corr[w];
    }
    as_global(P.sse_part)[tile] = s;
    as_global(P.corr_part)[tile] = c;
  }
}

// ---------------------------------------------------------------------------
// Fused mixed-precision assignment, software-pipelined (assignment mode).
//
// Same arithmetic as k_assign_mfma in assignment mode; the difference is the
// schedule.  The sweep over 32-centre blocks keeps two accumulator sets: the
// MFMAs of block b+1 are issued and, while the matrix core executes them, the
// wave runs the epilogue of block b (sched_group_barrier interleaves one
// MFMA with a few VALU instructions).  The saved copy of a lane's best block
// lives in LDS and is written only when the lane's best value improves.
// ---------------------------------------------------------------------------
// REC: also write a 1 into P.flagged for every flagged pair (diagnostic
// launches only: the record's stores cost the sweep registers).
template <class L, int DP, int NB, bool FALLBACK, bool REC = false>
__global__ void __launch_bounds__(kPipeThreads, 1)
k_assign_pipe(const AssignProb* __restrict__ probs, const int32_t* __restrict__ wg_start, int nprob) {
  using Cfg = AssignCfg<L, DP, NB, kPipeWaves>;
  constexpr int NT = kPipeThreads;
  using S = typename L::S;
  constexpr int LD = Cfg::kLd;
  constexpr int CT = Cfg::kCt;
  constexpr int kQueue = 8;

  // centre tiles, then the saved best blocks [wave][cb][r/4][lane]; before
  // the sweep the same bytes stage the point rows of the prologue
  // Three tile slots: tile t+1 is in LDS while tile t is processed, so the
  // fragments and accumulator starts of the next tile's first block are read
  // before the barrier that ends tile t.  The test constants keep four slots
  // (the epilogue of a tile's last block runs during the next tile).
  constexpr int kTileBytes = 3 * CT * LD * (int)sizeof(S);
  constexpr int kSvBytes = kPipeWaves * NB * 4 * 64 * 16;
  __shared__ __attribute__((aligned(16))) unsigned char lds_main[kTileBytes + kSvBytes];
  unsigned char* const smem = lds_main;
  f32x4 (*const s_sv)[NB][4][64] = reinterpret_cast<f32x4 (*)[NB][4][64]>(lds_main + kTileBytes);
  __shared__ float s_cinit[3][CT];
  __shared__ float s_ca[4][CT];
  __shared__ int s_q[FALLBACK ? kQueue * NT : 1];
  __shared__ int s_lab[kPipeWaves][NB * 32];
  __shared__ double s_sse[Cfg::kWaves];
  __shared__ unsigned long long s_corr[Cfg::kWaves];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int pi = find_problem(wg_start, nprob, blockIdx.x);
  const AssignProb& P = probs[pi];
  const int tile = blockIdx.x - wg_start[pi];
  const int64_t p0 = (int64_t)tile * Cfg::kPts;
  const int64_t n = P.n;
  const int d = P.d;
  const int nvalid = (int)((n - p0) < Cfg::kPts ? (n - p0) : Cfg::kPts);

  // ---- prologue: point fragments (RNE low precision) and quantised norms
  typename L::frag bfr[NB][Cfg::kSteps];
  float nx[NB], hx[NB];
  const int pw = wave * NB * 32;
  int bad = 0;
  const bool vec4 = ((d & 3) == 0) && ((((uintptr_t)P.X) & 15) == 0);
  const bool fast = vec4 && d == DP && nvalid == Cfg::kPts;
  // 16-bit formats with full rows: each wave reads its 32-point slices of X
  // with contiguous 1 KB loads (64 lanes x 16 B), rounds them and stages them
  // in LDS (rows padded like the centre tiles), then reads its fragments
  // back; strided 16-byte fragment loads straight from HBM would touch 32
  // cache lines per instruction.
  constexpr bool kStageable = L::KS == 16 && DP <= 128;
  const bool staged = kStageable && vec4 && d == DP;
  S* const stg = reinterpret_cast<S*>(lds_main) + wave * 32 * LD;
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    const int pl = pw + cb * 32 + (lane & 31);
    const bool pv = pl < nvalid;
    const KM_GLOBAL float* xr = as_global(P.X) + (p0 + (pv ? pl : 0)) * d;
    float part = 0.0f;
    if constexpr (kStageable) {
      if (staged) {
        constexpr int kLoads = 32 * DP / 256;  // float4 per lane and load
        f32x4 xv[kLoads];
#pragma unroll
        for (int q = 0; q < kLoads; ++q) {
          const int f = q * 256 + lane * 4;
          const int row = f / DP, col = f % DP;
          const int pr = pw + cb * 32 + row;
          xv[q] = f32x4{0.f, 0.f, 0.f, 0.f};
          if (pr < nvalid) xv[q] = *reinterpret_cast<const KM_GLOBAL f32x4*>(as_global(P.X) + (p0 + pr) * d + col);
        }
#pragma unroll
        for (int q = 0; q < kLoads; ++q) {
          const int f = q * 256 + lane * 4;
          const int row = f / DP, col = f % DP;
          typedef S s4 __attribute__((ext_vector_type(4)));
          s4 h;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const float v = xv[q][u];
            if (!__builtin_isfinite(v)) bad |= kStatusNonFinite;
            if (L::kHasRange && __builtin_fabsf(v) >= L::kOverflow) bad |= kStatusRange;
            h[u] = L::cvt(v);
          }
          *reinterpret_cast<s4*>(stg + row * LD + col) = h;
        }
#pragma unroll
        for (int s = 0; s < Cfg::kSteps; ++s) {
          const typename L::frag f =
              *reinterpret_cast<const typename L::frag*>(stg + (lane & 31) * LD + s * L::KS + (lane >> 5) * L::KV);
#pragma unroll
          for (int u = 0; u < L::KV; ++u) {
            const float qf = L::tof(f[u]);
            part = __builtin_fmaf(qf, qf, part);
          }
          bfr[cb][s] = f;
        }
        const float other = __shfl_xor(part, 32, kWave);
        nx[cb] = (lane < 32) ? part + other : other + part;
        hx[cb] = pv ? 0.5f * (P.oma * nx[cb]) : __builtin_inff();
        continue;
      }
    }
#pragma unroll
    for (int s = 0; s < Cfg::kSteps; ++s) {
      const int o = s * L::KS + (lane >> 5) * L::KV;
      float v[L::KV];
      if constexpr (L::KV % 4 == 0) {
        if (fast) {
#pragma unroll
          for (int u = 0; u < L::KV; u += 4) {
            const f32x4 q = *reinterpret_cast<const KM_GLOBAL f32x4*>(xr + o + u);
            v[u] = q[0]; v[u + 1] = q[1]; v[u + 2] = q[2]; v[u + 3] = q[3];
          }
        } else {
#pragma unroll
          for (int u = 0; u < L::KV; ++u) v[u] = (pv && o + u < d) ? xr[o + u] : 0.0f;
        }
      } else {
#pragma unroll
        for (int u = 0; u < L::KV; ++u) v[u] = (pv && o + u < d) ? xr[o + u] : 0.0f;
      }
      typename L::frag f;
#pragma unroll
      for (int u = 0; u < L::KV; ++u) {
        if (!__builtin_isfinite(v[u])) bad |= kStatusNonFinite;
        if (L::kHasRange && __builtin_fabsf(v[u]) >= L::kOverflow) bad |= kStatusRange;
        const S q = L::cvt(v[u]);
        if constexpr (L::KV == 1) f = q; else f[u] = q;
        const float qf = L::tof(q);
        part = __builtin_fmaf(qf, qf, part);
      }
      bfr[cb][s] = f;
    }
    const float other = __shfl_xor(part, 32, kWave);
    nx[cb] = (lane < 32) ? part + other : other + part;
    hx[cb] = pv ? 0.5f * (P.oma * nx[cb]) : __builtin_inff();
  }
  raise_status(P.status, bad);

  S* const sc0 = reinterpret_cast<S*>(smem);
  float bw[NB];
  int bb[NB];
  float cd[NB];
  int cj[NB];
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    bw[cb] = -__builtin_inff();
    bb[cb] = -1;
    cd[cb] = __builtin_inff();
    cj[cb] = -1;
  }
  // Seed of the running best from an earlier assignment (Lloyd rounds):
  // W of the hinted pair is recomputed on the vector ALU from the same
  // rounded operands, and the running best starts just below it, by more
  // than any difference between two FP32 evaluations of that dot product
  // (2 gamma_{d+1} at twice the unit roundoff, times the absolute sum).  The
  // block that holds the maximum still beats the seed, so the result is the
  // same as without the seed; only the copies of blocks that cannot win are
  // skipped.  A hinted pair that the reliability test might flag is not used
  // as a seed.  A hinted pair that the test surely flags (even the smallest
  // FP32 evaluation of W, plus the centre term, reaches the threshold) is
  // corrected here, once, by the lane whose accumulator rows hold it, and
  // that accumulator is set to -inf in its block before the block's test:
  // the sweep then takes its slow path only for other flagged pairs.  (In a
  // Lloyd round the previous label is often the one flagged pair of a point:
  // a point close to its centre compared with the norms.)
  unsigned long long ncorr = 0;
  // (up to 64 coordinates: at 128 the extra registers would spill)
  constexpr bool kPreCorrect = FALLBACK && DP <= 64;
  int xh[NB];  // excluded pair of the lane: block start | register, or -1
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) xh[cb] = -1;
  if (P.hint) {
    constexpr float kU2 = 1.0f / 8388608.0f;  // 2 * 2^-24
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const int pl = pw + cb * 32 + (lane & 31);
      const bool pv = pl < nvalid;
      const int h = pv ? as_global(P.hint)[p0 + pl] : -1;
      const bool hv = h >= 0 && h < P.k;
      // the hinted centre's quantised row, read in the lane's fragment layout
      const KM_GLOBAL S* cr = reinterpret_cast<const KM_GLOBAL S*>(as_global(P.Cq)) +
                              (int64_t)(hv ? h : 0) * DP + (lane >> 5) * L::KV;
      float dp = 0.0f, ap = 0.0f;
#pragma unroll
      for (int s = 0; s < Cfg::kSteps; ++s) {
        typename L::frag cf;
        if constexpr (L::KV == 1) cf = cr[s * L::KS];
        else cf = *reinterpret_cast<const KM_GLOBAL typename L::frag*>(cr + s * L::KS);
#pragma unroll
        for (int u = 0; u < L::KV; ++u) {
          float xq, cq;
          if constexpr (L::KV == 1) {
            xq = L::tof(bfr[cb][s]);
            cq = L::tof(cf);
          } else {
            xq = L::tof(bfr[cb][s][u]);
            cq = L::tof(cf[u]);
          }
          dp = __builtin_fmaf(xq, cq, dp);
          ap = __builtin_fmaf(__builtin_fabsf(xq), __builtin_fabsf(cq), ap);
        }
      }
      const float od = __shfl_xor(dp, 32, kWave), oa = __shfl_xor(ap, 32, kWave);
      const float dot = (lane < 32) ? dp + od : od + dp;
      const float abs_sum = (lane < 32) ? ap + oa : oa + ap;
      if (hv && pv) {
        const float ci = as_global(P.cinit)[h];
        const float caj = as_global(P.ca)[h];
        const float m = (float)(d + 1) * kU2;
        const float delta = 2.0f * (m / (1.0f - m)) * (abs_sum + __builtin_fabsf(ci)) * 1.0625f + 1e-30f;
        const float w = dot + ci;
        if ((w + delta) + caj + delta < hx[cb]) bw[cb] = w - 2.0f * delta;
        if constexpr (kPreCorrect) {
          if ((w - delta) + caj - delta >= hx[cb] && (lane >> 5) == ((h >> 2) & 1)) {
            if (REC && P.flagged) as_global(P.flagged)[(p0 + pl) * (int64_t)P.k + h] = 1;  // diagnostic record
            const float df = (float)correct_pair<L>(P, P.X + (p0 + pl) * d, P.C + (int64_t)h * d, d);
            ncorr += 1;
            cd[cb] = df;
            cj[cb] = h;
            xh[cb] = (h & ~31) | (4 * ((h & 31) >> 3) + (h & 3));
          }
        }
      }
    }
  }
  int qn = 0;
  auto flush_queue = [&]() {
    if constexpr (FALLBACK) {
      for (int q = 0; q < qn; ++q) {
        const int e = s_q[q * NT + tid];
        const int j = e & 0xffffff;
        const int cbq = e >> 24;
        const int pl = pw + cbq * 32 + (lane & 31);
        if (REC && P.flagged) as_global(P.flagged)[(p0 + pl) * (int64_t)P.k + j] = 1;  // diagnostic record
        const double dd = correct_pair<L>(P, P.X + (p0 + pl) * d, P.C + (int64_t)j * d, d);
        const float df = (float)dd;
        ncorr += 1;
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
          if (cb != cbq) continue;
          if (df < cd[cb] || (df == cd[cb] && j < cj[cb])) {
            cd[cb] = df;
            cj[cb] = j;
          }
        }
      }
      qn = 0;
    }
  };

  const int kpad = P.k_pad;
  const int ntile = (kpad + CT - 1) / CT;
  const KM_GLOBAL S* Cq = reinterpret_cast<const KM_GLOBAL S*>(as_global(P.Cq));
  f32x4 stage[Cfg::kChunksPerThread];
  float st_ci = 0.f, st_ca = 0.f;
  auto load_tile = [&](int t) {
    const int rows = (kpad - t * CT) < CT ? (kpad - t * CT) : CT;
    const KM_GLOBAL f32x4* g = reinterpret_cast<const KM_GLOBAL f32x4*>(Cq + (int64_t)t * CT * DP);
    const int nchunk = rows * DP / Cfg::kElemsPerChunk;
#pragma unroll
    for (int u = 0; u < Cfg::kChunksPerThread; ++u) {
      const int c = tid + u * NT;
      if (c < nchunk) stage[u] = g[c];
    }
    if (tid < rows) {
      st_ci = as_global(P.cinit)[t * CT + tid];
      st_ca = as_global(P.ca)[t * CT + tid];
    }
  };
  auto store_tile = [&](int t) {
    const int rows = (kpad - t * CT) < CT ? (kpad - t * CT) : CT;
    const int nchunk = rows * DP / Cfg::kElemsPerChunk;
    constexpr int CPR = DP / Cfg::kElemsPerChunk;
    S* dst = sc0 + (t % 3) * CT * LD;
#pragma unroll
    for (int u = 0; u < Cfg::kChunksPerThread; ++u) {
      const int c = tid + u * NT;
      if (c < nchunk) {
        const int row = c / CPR, col = (c % CPR) * Cfg::kElemsPerChunk;
        *reinterpret_cast<f32x4*>(dst + row * LD + col) = stage[u];
      }
    }
    if (tid < rows) {
      s_cinit[t % 3][tid] = st_ci;
      s_ca[t % 4][tid] = st_ca;
    }
  };

  // A fragments of one 32-centre block (8 consecutive K values per lane and
  // K step) from the LDS tile
  typename L::frag af[Cfg::kSteps];
  auto afrag_ptr = [&](int t, int bk) {
    return sc0 + (t % 3) * CT * LD + (bk * 32 + (lane & 31)) * LD + (lane >> 5) * L::KV;
  };
  auto load_af = [&](int t, int bk) {
    const S* arow = afrag_ptr(t, bk);
#pragma unroll
    for (int s = 0; s < Cfg::kSteps; ++s) {
      if constexpr (L::KV == 1) af[s] = arow[s * L::KS];
      else af[s] = *reinterpret_cast<const typename L::frag*>(arow + s * L::KS);
    }
  };
  // MFMAs of one 32-centre block: acc = -nc/2 + x~^T c~, from the fragments
  // in af; when `pre` is set, each K step's fragment register is refilled
  // with the next block's (tn, bkn) fragment right after its last use
  auto issue = [&](f32x16 (&acc)[NB], int t, int bk, bool pre, int tn, int bkn) {
    f32x16 ci;
#pragma unroll
    for (int r = 0; r < 16; ++r) ci[r] = s_cinit[t % 3][bk * 32 + acc_row(r, lane)];
    const S* nrow = afrag_ptr(tn, bkn);
#pragma unroll
    for (int s = 0; s < Cfg::kSteps; ++s) {
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) acc[cb] = L::mfma(af[s], bfr[cb][s], s == 0 ? ci : acc[cb]);
      if (pre) {
        if constexpr (L::KV == 1) af[s] = nrow[s * L::KS];
        else af[s] = *reinterpret_cast<const typename L::frag*>(nrow + s * L::KS);
      }
    }
  };
  // epilogue part 1 (overlaps the next block's MFMAs): block maxima of the
  // test quantity W + ca and of W
  auto epi1 = [&](f32x16 (&acc)[NB], int t, int bk, float (&tm)[NB], float (&wm)[NB]) {
    if constexpr (kPreCorrect) {
      // hinted pairs already corrected: out of this block's test and argmax
      const int jb = t * CT + bk * 32;
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        const bool here = (xh[cb] & ~31) == jb;
        if (__ballot(here) != 0) {
          const int rx = here ? (xh[cb] & 31) : 16;
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[cb][r] = r == rx ? -__builtin_inff() : acc[cb][r];
        }
      }
    }
    if constexpr (FALLBACK) {
      f32x16 cav;
#pragma unroll
      for (int r = 0; r < 16; ++r) cav[r] = s_ca[t % 4][bk * 32 + acc_row(r, lane)];
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) tm[cb] = max16(acc[cb] + cav);
    }
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) wm[cb] = max16(acc[cb]);
  };
  // epilogue part 2: rare slow path for flagged pairs, then the running best
  auto epi2 = [&](const f32x16 (&acc)[NB], int t, int bk, float (&tm)[NB], float (&wm)[NB]) {
    const int jb = t * CT + bk * 32;
    // the block's values go to LDS when it improves the running best; each
    // path stores from its own registers (no merged copy of the block)
    auto save = [&](int cb, const f32x16& w) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        f32x4 v = {w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]};
        s_sv[wave][cb][q][lane] = v;
      }
    };
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      if constexpr (FALLBACK) {
        if (__builtin_expect(__ballot(tm[cb] >= hx[cb]) != 0, 0)) {  // rare, wave-uniform
          f32x16 w = acc[cb];
          const int pl = pw + cb * 32 + (lane & 31);
          uint32_t fm = 0;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const bool f = w[r] + s_ca[t % 4][bk * 32 + acc_row(r, lane)] >= hx[cb];
            fm |= (uint32_t)f << r;
            w[r] = f ? -__builtin_inff() : w[r];
          }
          wm[cb] = max16(w);
          if (pl >= nvalid) fm = 0;
          while (fm) {
            const int r = __builtin_ctz(fm);
            fm &= fm - 1;
            const int j = jb + acc_row(r, lane);
            if (j >= P.k) continue;
            if (qn < kQueue) {
              s_q[qn * NT + tid] = j | (cb << 24);
              qn += 1;
            } else {  // queue full (dense flags): correct this pair now
              if (REC && P.flagged) as_global(P.flagged)[(p0 + pl) * (int64_t)P.k + j] = 1;  // diagnostic record
              const float df = (float)correct_pair<L>(P, P.X + (p0 + pl) * d, P.C + (int64_t)j * d, d);
              ncorr += 1;
              if (df < cd[cb] || (df == cd[cb] && j < cj[cb])) {
                cd[cb] = df;
                cj[cb] = j;
              }
            }
          }
          if (wm[cb] > bw[cb]) {  // strict: the earlier block keeps ties
            bw[cb] = wm[cb];
            bb[cb] = jb;
            save(cb, w);
          }
          continue;
        }
      }
      if (wm[cb] > bw[cb]) {
        bw[cb] = wm[cb];
        bb[cb] = jb;
        save(cb, acc[cb]);
      }
    }
  };

  load_tile(0);
  __syncthreads();  // the staged point rows share these LDS bytes
  store_tile(0);
  if (1 < ntile) {
    load_tile(1);
    store_tile(1);
  }
  __syncthreads();
  if (2 < ntile) load_tile(2);

  f32x16 accA[NB], accB[NB];
  float tm[NB], wm[NB];
  // one region: MFMAs of the next block interleaved with the epilogue
  // (block maxima) of the previous one
#define KM_INTERLEAVE()                                        \
  _Pragma("unroll") for (int i_ = 0; i_ < Cfg::kSteps * NB; ++i_) { \
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);         \
    __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);         \
  }
  // end of tile t: tile t+2 into its slot, barrier, tile t+3 in flight
  auto tile_end = [&](int t) {
    if (t + 2 < ntile) store_tile(t + 2);
    if constexpr (FALLBACK) {
      if (__ballot(qn >= kQueue / 2)) flush_queue();  // batch: rare flags wait to the end
    }
    __syncthreads();
    if (t + 3 < ntile) load_tile(t + 3);
  };
  // block 1 of tile t prefetches block 0 of tile t+1 (already in LDS); the
  // last tile prefetches a block of its own (unused)
  // tile 0
  const int nbk0 = (kpad < CT ? kpad : CT) / 32;
  load_af(0, 0);
  issue(accA, 0, 0, true, 0, 1);  // a tile of one block prefetches unused rows
  if (nbk0 == 2) {
    issue(accB, 0, 1, true, 1 < ntile ? 1 : 0, 0);
    epi1(accA, 0, 0, tm, wm);
    KM_INTERLEAVE();
    epi2(accA, 0, 0, tm, wm);
  }
  tile_end(0);
  // tiles 1..: every tile before the last holds two blocks
  for (int t = 1; t < ntile; ++t) {
    const int nbk = ((kpad - t * CT) < CT ? (kpad - t * CT) : CT) / 32;
    issue(accA, t, 0, true, t, 1);
    epi1(accB, t - 1, 1, tm, wm);
    KM_INTERLEAVE();
    epi2(accB, t - 1, 1, tm, wm);
    if (nbk == 2) {
      issue(accB, t, 1, true, t + 1 < ntile ? t + 1 : t, 0);
      epi1(accA, t, 0, tm, wm);
      KM_INTERLEAVE();
      epi2(accA, t, 0, tm, wm);
    }
    tile_end(t);
  }
#undef KM_INTERLEAVE
  {
    const int tl = ntile - 1;
    const int nbkl = ((kpad - tl * CT) < CT ? (kpad - tl * CT) : CT) / 32;
    if (nbkl == 2) {
      epi1(accB, tl, 1, tm, wm);
      epi2(accB, tl, 1, tm, wm);
    } else {
      epi1(accA, tl, 0, tm, wm);
      epi2(accA, tl, 0, tm, wm);
    }
  }
  flush_queue();

  // ---- index of the best kept pair, merge the two lanes that share a
  // point, choose between kept and corrected, refine in FP64
  double sse = 0.0;
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    int rs = 16;
    if (bb[cb] >= 0) {
#pragma unroll
      for (int q = 3; q >= 0; --q) {
        const f32x4 v = s_sv[wave][cb][q][lane];
#pragma unroll
        for (int e = 3; e >= 0; --e) rs = (v[e] == bw[cb]) ? 4 * q + e : rs;
      }
    }
    int bj = (bb[cb] >= 0 && rs < 16) ? bb[cb] + acc_row(rs, lane) : -1;
    float ow = __shfl_xor(bw[cb], 32, kWave);
    int oj = __shfl_xor(bj, 32, kWave);
    if (ow > bw[cb] || (ow == bw[cb] && oj >= 0 && (bj < 0 || oj < bj))) {
      bw[cb] = ow;
      bj = oj;
    }
    float od = __shfl_xor(cd[cb], 32, kWave);
    int ojc = __shfl_xor(cj[cb], 32, kWave);
    if (od < cd[cb] || (od == cd[cb] && ojc >= 0 && (cj[cb] < 0 || ojc < cj[cb]))) {
      cd[cb] = od;
      cj[cb] = ojc;
    }
    bb[cb] = bj;
  }
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    if ((cb & 1) != (lane >> 5)) continue;
    const int pl = pw + cb * 32 + (lane & 31);
    if (pl >= nvalid) continue;
    const float dk = bb[cb] >= 0 ? __builtin_fmaxf(nx[cb] - 2.0f * bw[cb], 0.0f) : __builtin_inff();
    int lab = bb[cb];
    if (cj[cb] >= 0 && (cd[cb] < dk || (cd[cb] == dk && cj[cb] < lab) || lab < 0)) lab = cj[cb];
    if (lab < 0 || lab >= P.k) lab = 0;  // only with non-finite data (status raised)
    as_global(P.labels)[p0 + pl] = lab;
    s_lab[wave][cb * 32 + (lane & 31)] = lab;
  }
  {
    int nloc = nvalid - pw;
    nloc = nloc < 0 ? 0 : (nloc > NB * 32 ? NB * 32 : nloc);
    if (P.refine) sse = refine_wave(P, p0 + pw, nloc, s_lab[wave], lane);
  }
  sse = wave_sum(sse);
  unsigned long long nc = wave_sum_u64(ncorr);
  if (lane == 0) {
    s_sse[wave] = sse;
    s_corr[wave] = nc;
  }
  __syncthreads();
  if (tid == 0) {
    double ssum = 0.0;
    unsigned long long c = 0;
#pragma unroll
    for (int w = 0; w < Cfg::kWaves; ++w) {
      ssum += s_sse[w];
      c += s_corr[w];
    }
    as_global(P.sse_part)[tile] = ssum;
    as_global(P.corr_part)[tile] = c;
  }
}

// ---------------------------------------------------------------------------
// Fused mixed-precision assignment for small problems (d <= 32, k <= 64).
//
// Same arithmetic and outputs as k_assign_pipe in assignment mode, for shapes
// that are bound by memory and the vector epilogue rather than the matrix
// cores (a few coordinates, a few dozen centres).  Each workgroup rounds the
// centres itself (no preparation launch); their fragments (at most two
// 32-centre blocks) stay in registers for the whole launch, their
// accumulator starts and test constants in LDS, and each wave sweeps `gpw`
// groups of 32 points, loading the rows of the next group before the
// epilogue of the current one.  Every
// lane holds the full FP32 row of its point (the two lanes of a point hold
// different centres of a block).  Flagged pairs can be frequent on such data
// (a tenth of all pairs on normalised image features), so they are not
// corrected by their own lane: the lanes append them to a per-wave queue in
// LDS (positions from a prefix sum of the lanes' counts) and all 64 lanes
// evaluate the FP64 direct formula on the queue, merging each result into its
// point's best corrected pair with a 64-bit LDS minimum on (FP32 value bits,
// centre index) -- smallest value, then lowest index, as in a sequential
// scan.
//   XD: register capacity of a point row (8, 16 or 32, >= d)
// The reliability test first adds the lane's block maximum of W and the
// largest centre term of its rows: FP32 addition is monotonic, so when that
// sum stays below the threshold no pair of the lane is flagged, exactly as
// the per-pair test "W + ca_j >= hx" would decide.  Otherwise the per-pair
// test masks the flagged pairs and queues them.
// ---------------------------------------------------------------------------
// Orders this wave's LDS accesses: LDS operations of one wave complete in
// issue order; the fence keeps the compiler from moving accesses across it
// and the wait makes the results of earlier ones visible to every lane.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
}

template <int XD>
__device__ inline double sqdist64_rl(const float (&x)[XD], const float* c, int d) {
  double s = 0.0;
#pragma unroll
  for (int l = 0; l < XD; ++l) {
    if (l >= d) break;
    const double e = (double)x[l] - (double)c[l];
    s = __builtin_fma(e, e, s);
  }
  return s;
}

// LDS of one workgroup of the small-problem body: FP32 centre rows, their
// accumulator starts and test constants, and per wave the correction queue of
// a 32-centre block (at most 32 x 32 pairs), the group's point rows and each
// point's best corrected pair.
template <int XD, bool FALLBACK>
struct SmallLds {
  static constexpr int CS = XD + 4;  // LDS row stride of FP32 rows (16-byte aligned)
  alignas(16) float ca[kSmallMaxK];
  alignas(16) float cinit[kSmallMaxK];
  alignas(16) float c[kSmallMaxK * CS];
  alignas(16) float x[FALLBACK ? kSmallWaves : 1][FALLBACK ? 32 * CS : 4];
  unsigned long long key[FALLBACK ? kSmallWaves : 1][32];
  double sse[kSmallWaves];
  unsigned long long corr[kSmallWaves];
  int q[FALLBACK ? kSmallWaves : 1][FALLBACK ? 32 * 32 : 1];
};

// One tile (kSmallWaves x 32 x gpw consecutive points) of a problem; writes
// the tile's labels and its SSE / corrected-pair partials.
template <class L, int XD, bool FALLBACK>
__device__ __attribute__((always_inline)) inline void
assign_small_tile(const AssignProb& P, const int tile, SmallLds<XD, FALLBACK>& sm) {
  constexpr int DP = XD < 16 ? 16 : XD;  // row extent of the quantised centres
  constexpr int STEPS = DP / L::KS;
  constexpr int CS = XD + 4;
  using S = typename L::S;
  using frag = typename L::frag;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int hi = lane >> 5;
  const int gpw = P.gpw;
  const int64_t p0 = (int64_t)tile * (kSmallWaves * 32) * gpw;
  const int64_t n = P.n;
  const int d = P.d;
  const int k = P.k;
  const int kb = P.k_pad > 32 ? 2 : 1;

  const bool vec4 = ((d & 3) == 0) && ((((uintptr_t)P.X) & 15) == 0);
  auto load_rows = [&](int q, float (&xr)[XD]) {
    const int64_t p = p0 + (int64_t)(q * kSmallWaves + wave) * 32 + (lane & 31);
    const bool pv = p < n;
    const KM_GLOBAL float* row = as_global(P.X) + (pv ? p : 0) * d;
    if (vec4) {
#pragma unroll
      for (int l = 0; l < XD; l += 4) {
        f32x4 v = {0.f, 0.f, 0.f, 0.f};
        if (l < d) v = *reinterpret_cast<const KM_GLOBAL f32x4*>(row + l);
        xr[l] = v[0]; xr[l + 1] = v[1]; xr[l + 2] = v[2]; xr[l + 3] = v[3];
      }
    } else {
#pragma unroll
      for (int l = 0; l < XD; ++l) xr[l] = l < d ? row[l] : 0.0f;
    }
#pragma unroll
    for (int l = 0; l < XD; ++l) xr[l] = pv ? xr[l] : 0.0f;
  };
  // the first group's rows are requested before the centre set-up
  float xn[XD];
  load_rows(0, xn);

  // Centres, prepared by each workgroup itself (no separate launch): FP32
  // rows to LDS (corrections, refinement), range and finiteness, then per
  // centre the rounded row's squared norm nc in FP32 (coordinates in order),
  // the accumulator start -nc/2 and the test constant alpha nc/2; rows past k
  // start at -inf and never fail the test.
  int bad = 0;
  for (int e = tid; e < kSmallMaxK * CS; e += kSmallThreads) {
    const int j = e / CS, l = e - j * CS;
    float v = 0.0f;
    if (j < k && l < d) {
      v = as_global(P.C)[(int64_t)j * d + l];
      if (!__builtin_isfinite(v)) bad |= kStatusNonFinite;
      if (L::kHasRange && __builtin_fabsf(v) >= L::kOverflow) bad |= kStatusRange;
    }
    sm.c[e] = v;
  }
  __syncthreads();
  if (tid < kSmallMaxK) {
    float nc = 0.0f;
#pragma unroll
    for (int l = 0; l < XD; ++l) {
      if (l >= d) break;
      const float f = L::tof(L::cvt(sm.c[tid * CS + l]));
      nc = __builtin_fmaf(f, f, nc);
    }
    const float hc = 0.5f * nc;
    sm.cinit[tid] = tid < k ? -hc : -__builtin_inff();
    sm.ca[tid] = tid < k ? P.alpha * hc : 0.0f;
  }
  // centre fragments in registers: RNE of the LDS rows (zero past d and k)
  frag af[2][STEPS];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
#pragma unroll
      for (int u = 0; u < L::KV; ++u) {
        const int l = s * L::KS + hi * L::KV + u;
        const float v = (b < kb && l < XD) ? sm.c[(b * 32 + (lane & 31)) * CS + (l < XD ? l : 0)] : 0.0f;
        af[b][s][u] = L::cvt(v);
      }
    }
  }
  // accumulator start of block b: -nc_j/2 of the lane's rows
  auto acc_start = [&](int b) {
    f32x16 a;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const f32x4 v = *reinterpret_cast<const f32x4*>(&sm.cinit[b * 32 + 8 * q + 4 * hi]);
      a[4 * q] = v[0]; a[4 * q + 1] = v[1]; a[4 * q + 2] = v[2]; a[4 * q + 3] = v[3];
    }
    return a;
  };
  __syncthreads();
  // rows of real centres among the lane's rows of each block
  uint32_t vmask[2];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    uint32_t v = 0;
#pragma unroll
    for (int r = 0; r < 16; ++r) v |= (uint32_t)(b * 32 + acc_row(r, lane) < k) << r;
    vmask[b] = v;
  }
  float cam[2];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    float m = -__builtin_inff();
#pragma unroll
    for (int r = 0; r < 16; ++r) m = __builtin_fmaxf(m, sm.ca[b * 32 + acc_row(r, lane)]);
    cam[b] = m;
  }

  double sse = 0.0;
  unsigned long long ncorr = 0;
  for (int q = 0; q < gpw; ++q) {
    float x[XD];
#pragma unroll
    for (int l = 0; l < XD; ++l) x[l] = xn[l];
    if (q + 1 < gpw) load_rows(q + 1, xn);
    const int64_t p = p0 + (int64_t)(q * kSmallWaves + wave) * 32 + (lane & 31);
    const bool pv = p < n;

    // range and finiteness, rounding, quantised norm (coordinates in order)
    S qx[XD];
    float nxv = 0.0f;
#pragma unroll
    for (int l = 0; l < XD; ++l) {
      qx[l] = L::cvt(x[l]);
      if (l < d) {
        if (!__builtin_isfinite(x[l])) bad |= kStatusNonFinite;
        if (L::kHasRange && __builtin_fabsf(x[l]) >= L::kOverflow) bad |= kStatusRange;
        const float f = L::tof(qx[l]);
        nxv = __builtin_fmaf(f, f, nxv);
      }
    }
    frag bf[STEPS];
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
#pragma unroll
      for (int u = 0; u < L::KV; ++u) {
        const int l0 = s * L::KS + u, l1 = s * L::KS + L::KV + u;
        const S a = l0 < XD ? qx[l0] : S(0.0f);
        const S c = l1 < XD ? qx[l1] : S(0.0f);
        bf[s][u] = hi ? c : a;
      }
    }
    const float hx = pv ? 0.5f * (P.oma * nxv) : __builtin_inff();

    // cross terms W = x~^T c~ - nc/2 of both blocks
    f32x16 acc[2];
    float m[2];
    acc[0] = acc_start(0);
#pragma unroll
    for (int s = 0; s < STEPS; ++s) acc[0] = L::mfma(af[0][s], bf[s], acc[0]);
    // a second block is always issued: without centres its fragments are
    // zero and its starts -inf, so it never wins and is never flagged
    acc[1] = acc_start(1);
#pragma unroll
    for (int s = 0; s < STEPS; ++s) acc[1] = L::mfma(af[1][s], bf[s], acc[1]);
    m[0] = max16(acc[0]);
    m[1] = max16(acc[1]);

    // reliability test; flagged pairs go to the wave's queue and are
    // corrected in FP64 by all lanes together
    bool staged = false;
    if constexpr (FALLBACK) {
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if (b >= kb) break;
        if (__ballot(m[b] + cam[b] >= hx) != 0) {
          uint32_t fm = 0;
#pragma unroll
          for (int q = 0; q < 4; ++q) {  // rows 8q + 4hi + 0..3 of the block
            const f32x4 ca4 = *reinterpret_cast<const f32x4*>(&sm.ca[b * 32 + 8 * q + 4 * hi]);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int r = 4 * q + e;
              const bool f = acc[b][r] + ca4[e] >= hx;
              fm |= (uint32_t)f << r;
              acc[b][r] = f ? -__builtin_inff() : acc[b][r];
            }
          }
          m[b] = max16(acc[b]);
          fm &= vmask[b];
          if (!staged) {  // the group's rows and best corrected pairs
            staged = true;
            if (hi == 0) {  // whole rows: the coordinates past d are zero
#pragma unroll
              for (int l = 0; l < XD; l += 4)
                *reinterpret_cast<f32x4*>(&sm.x[wave][(lane & 31) * CS + l]) =
                    f32x4{x[l], x[l + 1], x[l + 2], x[l + 3]};
              sm.key[wave][lane & 31] = ~0ull;
            }
          }
          // queue positions: exclusive prefix of the lanes' flag counts
          // (at most 16), one ballot per bit of the count
          const int cnt = __builtin_popcount(fm);
          int pos = 0, total = 0;
#pragma unroll
          for (int bit = 0; bit < 5; ++bit) {
            const unsigned long long bal = __ballot((cnt >> bit) & 1);
            const int below = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
            pos += below << bit;
            total += __popcll(bal) << bit;
          }
          while (fm) {
            const int r = __builtin_ctz(fm);
            fm &= fm - 1;
            sm.q[wave][pos++] = (lane & 31) | ((b * 32 + acc_row(r, lane)) << 5);
            if (P.flagged)  // diagnostic record of the test's decision
              as_global(P.flagged)[p * (int64_t)k + b * 32 + acc_row(r, lane)] = 1;
          }
          wave_lds_sync();
          for (int e = lane; e < total; e += 64) {
            const int code = sm.q[wave][e];
            const int pt = code & 31, j = code >> 5;
            const float* xr = &sm.x[wave][pt * CS];
            const float* cr = &sm.c[j * CS];
            // four coordinates per LDS access; both rows are zero past d,
            // and a zero term leaves the FP64 sum unchanged
            double sq = 0.0;
            if (P.high == kHigh64) {
#pragma unroll
              for (int l0 = 0; l0 < XD; l0 += 4) {
                if (l0 >= d) break;
                const f32x4 a4 = *reinterpret_cast<const f32x4*>(xr + l0);
                const f32x4 c4 = *reinterpret_cast<const f32x4*>(cr + l0);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                  const double t = (double)a4[e] - (double)c4[e];
                  sq = __builtin_fma(t, t, sq);
                }
              }
            } else {
              sq = corr_dist(P.high, L::kFmt, xr, cr, d);
            }
            // smallest value, then lowest index: FP32 bits of a
            // non-negative value order like the value
            const unsigned long long key =
                ((unsigned long long)__float_as_uint((float)sq) << 32) | (unsigned)j;
            atomicMin(&sm.key[wave][pt], key);
            ncorr += 1;
          }
          wave_lds_sync();
        }
      }
    }
    float cd = __builtin_inff();
    int cj = -1;
    if (staged) {
      const unsigned long long key = sm.key[wave][lane & 31];
      if (key != ~0ull) {
        cj = (int)(key & 0xffffffffu);
        cd = __uint_as_float((unsigned)(key >> 32));
      }
    }

    // best kept pair of the lane: block, then the lowest row holding it
    const bool sel = m[1] > m[0];
    float bw = sel ? m[1] : m[0];
    int rs = 16;
#pragma unroll
    for (int r = 15; r >= 0; --r) {
      const float v = sel ? acc[1][r] : acc[0][r];
      rs = (v == bw) ? r : rs;
    }
    int bj = (bw > -__builtin_inff() && rs < 16) ? (sel ? 32 : 0) + acc_row(rs, lane) : -1;
    // merge the two lanes of the point; choose between kept and corrected
    const float ow = __shfl_xor(bw, 32, kWave);
    const int oj = __shfl_xor(bj, 32, kWave);
    if (ow > bw || (ow == bw && oj >= 0 && (bj < 0 || oj < bj))) {
      bw = ow;
      bj = oj;
    }
    if (hi == 0 && pv) {
      const float dk = bj >= 0 ? __builtin_fmaxf(nxv - 2.0f * bw, 0.0f) : __builtin_inff();
      int lab = bj;
      if (cj >= 0 && (cd < dk || (cd == dk && cj < lab) || lab < 0)) lab = cj;
      if (lab < 0 || lab >= k) lab = 0;  // only with non-finite data (status raised)
      as_global(P.labels)[p] = lab;
      if (P.refine) {
        const double dd = sqdist64_rl<XD>(x, sm.c + lab * CS, d);
        if (P.mindist) as_global(P.mindist)[p] = (float)dd;
        sse += dd;
      }
    }
  }
  raise_status(P.status, bad);
  sse = wave_sum(sse);
  const unsigned long long nc = wave_sum_u64(ncorr);
  if (lane == 0) {
    sm.sse[wave] = sse;
    sm.corr[wave] = nc;
  }
  __syncthreads();
  if (tid == 0) {
    double ssum = 0.0;
    unsigned long long c = 0;
#pragma unroll
    for (int w = 0; w < kSmallWaves; ++w) {
      ssum += sm.sse[w];
      c += sm.corr[w];
    }
    as_global(P.sse_part)[tile] = ssum;
    as_global(P.corr_part)[tile] = c;
  }
}

template <class L, int XD, bool FALLBACK>
__global__ void __launch_bounds__(kSmallThreads, XD == 8 ? 4 : XD == 16 ? 3 : 2)
k_assign_small(const AssignProb* __restrict__ probs, const int32_t* __restrict__ wg_start, int nprob) {
  __shared__ SmallLds<XD, FALLBACK> sm;
  const int pi = find_problem(wg_start, nprob, blockIdx.x);
  assign_small_tile<L, XD, FALLBACK>(probs[pi], blockIdx.x - wg_start[pi], sm);
}

// ---------------------------------------------------------------------------
// Persistent Lloyd rounds of small problems (descriptor in km_internal.hpp).
// The grid is co-resident (cooperative launch); the phases of a round are
// separated by grid-wide waits on an arrival counter: release of the
// workgroup's writes at agent scope, one relaxed increment, then polling until
// every workgroup of the grid has arrived, and an agent-scope acquire.  The
// counter only grows (target = waits so far x grid size), so no reset is
// needed.  A wait that polls more than max_spins times (kSyncSpins by
// default, far beyond any phase) raises the abort flag; every other waiting
// workgroup sees it and leaves, so the kernel always ends, and every
// problem's status gets kStatusSync.
// ---------------------------------------------------------------------------
// Fixed-order sums of a pass's per-workgroup partials into its result record
// (ss, sc: 256 entries of LDS each)
__device__ __attribute__((always_inline)) inline void
reduce_parts_prob(const ReduceProb& P, double* ss, unsigned long long* sc) {
  const int tid = threadIdx.x;
  double s = 0.0;
  unsigned long long c = 0;
  for (int i = tid; i < P.nparts; i += 256) {
    s += as_global(P.sse_part)[i];
    c += as_global(P.corr_part)[i];
  }
  ss[tid] = s;
  sc[tid] = c;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (tid < o) {
      ss[tid] += ss[tid + o];
      sc[tid] += sc[tid + o];
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (P.sse_out) *P.sse_out = ss[0];
    if (P.result) {
      P.result->sse = ss[0];
      P.result->n_corrected += (long long)sc[0];
      P.result->n_pairs += P.pairs;
      P.result->status |= *P.status;
    }
  }
}

__device__ inline bool grid_wait(int* ctl, unsigned target, int* s_ok, unsigned max_spins) {
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned* arrivals = reinterpret_cast<unsigned*>(ctl);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(arrivals, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    unsigned spins = 0;
    while (__hip_atomic_load(arrivals, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(ctl + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || ++spins > max_spins) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    if (!ok) __hip_atomic_fetch_or(ctl + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

__device__ inline int load_agent(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Dynamic LDS: max(SmallLds, the update's wave regions and C_old), shared by
// the phases (a grid-wide wait separates them).
// (two workgroups per compute unit at most: the update's LDS rarely allows
// more, and the fused body then keeps its registers)
template <class L, int XD, bool FALLBACK>
__global__ void __launch_bounds__(kSmallThreads, 2)
k_lloyd_rounds(const RoundProb* __restrict__ probs, int nprob, const int32_t* __restrict__ tpre,
               const int32_t* __restrict__ cpre, const int32_t* __restrict__ fpre, int* ctl, unsigned max_spins) {
  extern __shared__ __attribute__((aligned(16))) char s_dyn[];
  __shared__ double s_sse[kOwnWaves];
  __shared__ double s_red[256];
  __shared__ unsigned long long s_cnt[256];
  __shared__ int s_m[256];
  __shared__ int s_ok;
  __shared__ unsigned char s_done[kRoundMaxProbs];  // this round's done flags
  SmallLds<XD, FALLBACK>& sm = *reinterpret_cast<SmallLds<XD, FALLBACK>*>(s_dyn);
  int* done = ctl + 2;
  int* rounds = ctl + 2 + nprob;
  const int G = gridDim.x;
  const int ntile = tpre[nprob], nchunk = cpre[nprob], nfin = fpre[nprob];
  unsigned waits = 0;
  for (int r = 0;; ++r) {
    const int b = r & 1;
    // done flags (written by the previous round's last phase) once per round
    int live = 0;
    for (int i = threadIdx.x; i < nprob; i += kSmallThreads) {
      const int dn = load_agent(done + i);
      s_done[i] = (unsigned char)dn;
      live |= dn == 0;
    }
    if (!__syncthreads_or(live)) return;
    // assignment of every tile of the running problems
    for (int t = blockIdx.x; t < ntile; t += G) {
      const int pi = find_problem(tpre, nprob, t);
      if (s_done[pi]) continue;
      assign_small_tile<L, XD, FALLBACK>(probs[pi].a[b], t - tpre[pi], sm);
      __syncthreads();
    }
    if (!grid_wait(ctl, ++waits * (unsigned)G, &s_ok, max_spins)) break;
    // chunk partials of the centre update
    for (int c = blockIdx.x; c < nchunk; c += G) {
      const int pi = find_problem(cpre, nprob, c);
      if (s_done[pi]) continue;
      own_part_chunk<1, true>(probs[pi].u[b], c - cpre[pi], s_dyn, probs[pi].wstride, s_sse);
      __syncthreads();
    }
    if (!grid_wait(ctl, ++waits * (unsigned)G, &s_ok, max_spins)) break;
    // per problem: counters of the pass (item 0), new centres of each
    // cluster group (items 1..nfin)
    for (int f = blockIdx.x; f < nfin; f += G) {
      const int pi = find_problem(fpre, nprob, f);
      if (s_done[pi]) continue;
      const int item = f - fpre[pi];
      if (item == 0) reduce_parts_prob(probs[pi].red, s_red, s_cnt);
      else own_fin_group(probs[pi].u[b], item - 1, s_m, s_red);
      __syncthreads();
    }
    if (!grid_wait(ctl, ++waits * (unsigned)G, &s_ok, max_spins)) break;
    // per problem: shift, SSE, stop test
    for (int pi = blockIdx.x; pi < nprob; pi += G) {
      if (s_done[pi]) continue;
      const RoundProb& R = probs[pi];
      const double shift = own_shift_prob(R.u[b], R.sse_hist ? R.sse_hist + r : nullptr, s_red);
      if (threadIdx.x == 0) {
        rounds[pi] = r + 1;
        if (r + 1 >= R.max_iter || (R.tol > 0.0 && shift < R.tol)) done[pi] = 1;
      }
      __syncthreads();
    }
    if (!grid_wait(ctl, ++waits * (unsigned)G, &s_ok, max_spins)) break;
  }
  // a wait gave up: mark every problem (the result records carry it)
  if (blockIdx.x == 0 && threadIdx.x == 0)
    for (int i = 0; i < nprob; ++i) atomicOr(probs[i].a[0].status, kStatusSync);
}

// ---------------------------------------------------------------------------
// Every pair by the direct formula (tiles described below).
// CMP64: compare the FP64 values (plain FP64 kernel); otherwise compare the
// values rounded to FP32 (mixed path with every pair corrected).
// AR: arithmetic of the formula -- 0 FP64; 1 FP32; 2 binary16 and 3 bfloat16
// on the rounded inputs (every operation rounded once, coordinates in
// order), for the other correction precisions when every pair is flagged.
// ---------------------------------------------------------------------------
template <int AR>
struct DirectArith;
template <>
struct DirectArith<0> {
  using T = double;
  __device__ static inline T in(float v) { return (double)v; }
  __device__ static inline T step(T x, T c, T s) { return acc(diff(x, c), s); }
  __device__ static inline T diff(T x, T c) { return x - c; }
  __device__ static inline T acc(T e, T s) { return __builtin_fma(e, e, s); }
};
template <>
struct DirectArith<1> {
  using T = float;
  __device__ static inline T in(float v) { return v; }
  __device__ static inline T step(T x, T c, T s) { return acc(diff(x, c), s); }
  __device__ static inline T diff(T x, T c) { return x - c; }
  __device__ static inline T acc(T e, T s) { return __builtin_fmaf(e, e, s); }
};
template <>
struct DirectArith<2> {
  using T = _Float16;
  __device__ static inline T in(float v) { return (_Float16)v; }
  __device__ static inline T step(T x, T c, T s) { return acc(diff(x, c), s); }
  __device__ static inline T diff(T x, T c) { return x - c; }
  __device__ static inline T acc(T e, T s) { return __builtin_fmaf16(e, e, s); }
};
template <>
struct DirectArith<3> {
  using T = float;  // bfloat16 values held in FP32
  __device__ static inline T in(float v) { return (float)(__bf16)v; }
  __device__ static inline T step(T x, T c, T s) { return acc(diff(x, c), s); }
  __device__ static inline T diff(T x, T c) { return bf16_sub(x, c); }
  __device__ static inline T acc(T e, T s) { return bf16_fma(e, e, s); }
};

// 128 points x 128 centres per step; thread (pg, cg) owns points pg*8.. and
// centres cg*8.. (8 x 8 pairs in registers).  Coordinate chunks of 16 are
// staged in LDS already converted to the arithmetic type, coordinate-major,
// so each thread reads its 8 points and 8 centres of a coordinate with wide
// loads; per coordinate a thread issues 64 subtractions and 64 FMAs.  The
// sum of a pair runs over the coordinates in index order.
template <bool CMP64, int MODE, int AR>
__global__ void __launch_bounds__(256, 2)  // two workgroups per CU: <= 256 VGPRs
k_assign_direct64(const AssignProb* __restrict__ probs, const int32_t* __restrict__ wg_start, int nprob) {
  using A = DirectArith<AR>;
  using T = typename A::T;
  constexpr int TP = kDirectPointsPerWg, TC = 128, DC = 16, RB = 8;
  static_assert(TP == 128, "tile");
  __shared__ __attribute__((aligned(16))) T sx[DC][TP];
  __shared__ __attribute__((aligned(16))) T sc[DC][TC];
  __shared__ double s_best[16][TP];
  __shared__ int s_bidx[16][TP];
  __shared__ double s_sse[4];
  __shared__ unsigned long long s_corr[4];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int pi = find_problem(wg_start, nprob, blockIdx.x);
  const AssignProb& P = probs[pi];
  const int tile = blockIdx.x - wg_start[pi];
  const int64_t p0 = (int64_t)tile * TP;
  const int d = P.d, k = P.k;
  const int nvalid = (int)((P.n - p0) < TP ? (P.n - p0) : TP);
  const int pg = tid & 15, cg = tid >> 4;  // points pg*8.., centres cg*8..
  const bool vec = (d & 3) == 0 && ((((uintptr_t)P.X) | ((uintptr_t)P.C)) & 15) == 0;

  int bad = 0;
  // each thread's best centre per point so far lives in its own LDS slots
  // (registers go to the 8 x 8 sums)
#pragma unroll
  for (int a = 0; a < RB; ++a) {
    s_best[cg][pg * RB + a] = __builtin_inf();
    s_bidx[cg][pg * RB + a] = -1;
  }
  // The next chunk's coordinates are loaded into registers while the
  // current chunk is computed: loads of chunk (c0, l0) are issued one chunk
  // ahead and written to LDS (converted) between two barriers.
  constexpr int NS = TP * DC / 256;  // elements per thread and chunk (8)
  static_assert(NS == 8, "two quads per thread");
  float xr[NS], cr[NS];  // vector path: quads r = 0, 1 in elements 4r..4r+3
  auto fetch = [&](int c0f, int l0f) __attribute__((always_inline)) {
    if (vec) {
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int e = tid + 256 * r, p = e >> 2, q = e & 3;
        f32x4 a = f32x4{0.f, 0.f, 0.f, 0.f}, b = f32x4{0.f, 0.f, 0.f, 0.f};
        if (p < nvalid && l0f + 4 * q < d)
          a = *reinterpret_cast<const KM_GLOBAL f32x4*>(as_global(P.X) + (p0 + p) * d + l0f + 4 * q);
        if (c0f + p < k && l0f + 4 * q < d)
          b = *reinterpret_cast<const KM_GLOBAL f32x4*>(as_global(P.C) + (int64_t)(c0f + p) * d + l0f + 4 * q);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          xr[4 * r + i] = a[i];
          cr[4 * r + i] = b[i];
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < NS; ++r) {
        const int e = tid + 256 * r, p = e / DC, l = e - p * DC;
        xr[r] = (p < nvalid && l0f + l < d) ? as_global(P.X)[(p0 + p) * d + l0f + l] : 0.f;
        cr[r] = (c0f + p < k && l0f + l < d) ? as_global(P.C)[(int64_t)(c0f + p) * d + l0f + l] : 0.f;
      }
    }
  };
  auto stage = [&](bool first_tile) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      const float v = xr[r], w = cr[r];
      if (first_tile && !__builtin_isfinite(v)) bad |= kStatusNonFinite;
      if (AR == 2 && (__builtin_fabsf(v) >= LowF16::kOverflow || __builtin_fabsf(w) >= LowF16::kOverflow))
        bad |= kStatusRange;
      int p, l;
      if (vec) {
        const int e = tid + 256 * (r >> 2);
        p = e >> 2;
        l = 4 * (e & 3) + (r & 3);
      } else {
        const int e = tid + 256 * r;
        p = e / DC;
        l = e - p * DC;
      }
      sx[l][p] = A::in(v);
      sc[l][p] = A::in(w);
    }
  };
  fetch(0, 0);
  for (int c0 = 0; c0 < k; c0 += TC) {
    T acc[RB][RB];
#pragma unroll
    for (int a = 0; a < RB; ++a)
#pragma unroll
      for (int b = 0; b < RB; ++b) acc[a][b] = (T)0.0f;
    for (int l0 = 0; l0 < d; l0 += DC) {
      // zero past the ends: a zero difference leaves a sum unchanged
      __syncthreads();
      stage(c0 == 0);
      __syncthreads();
      {
        const bool more = l0 + DC < d;
        const int c0n = more ? c0 : c0 + TC, l0n = more ? l0 + DC : 0;
        if (c0n < k) fetch(c0n, l0n);
      }
      const int lmax = (d - l0) < DC ? (d - l0) : DC;
      for (int l = 0; l < lmax; ++l) {
        T xv[RB], cv[RB];
#pragma unroll
        for (int a = 0; a < RB; ++a) xv[a] = sx[l][pg * RB + a];
#pragma unroll
        for (int b = 0; b < RB; ++b) cv[b] = sc[l][cg * RB + b];
        // eight independent differences, then their eight multiply-adds
        // (no subtraction feeds the instruction right after it)
#pragma unroll
        for (int a = 0; a < RB; ++a) {
          T e[RB];
#pragma unroll
          for (int b = 0; b < RB; ++b) e[b] = A::diff(xv[a], cv[b]);
#pragma unroll
          for (int b = 0; b < RB; ++b) acc[a][b] = A::acc(e[b], acc[a][b]);
        }
      }
    }
#pragma unroll
    for (int a = 0; a < RB; ++a)
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        const int j = c0 + cg * RB + b;
        const int p = pg * RB + a;
        if (j < k && p < nvalid) {
          if constexpr (MODE == 0) {
            const double v = CMP64 ? (double)acc[a][b] : (double)(float)acc[a][b];
            if (v < s_best[cg][p]) {  // centres visited in increasing order
              s_best[cg][p] = v;
              s_bidx[cg][p] = j;
            }
          } else {
            const int64_t o = (p0 + p) * (int64_t)k + j;
            as_global(P.D)[o] = (float)acc[a][b];
            if (P.flagged) as_global(P.flagged)[o] = 1;
          }
        }
      }
  }
  raise_status(P.status, bad);
  double sse = 0.0;
  unsigned long long nc = 0;
  if constexpr (MODE == 0) {
    __syncthreads();
    if (tid < TP && tid < nvalid) {
      double bv = __builtin_inf();
      int bi = -1;
      for (int g = 0; g < 16; ++g) {
        const double v = s_best[g][tid];
        const int i = s_bidx[g][tid];
        if (i >= 0 && (v < bv || (v == bv && i < bi))) {
          bv = v;
          bi = i;
        }
      }
      const int64_t p = p0 + tid;
      if (bi < 0) bi = 0;  // only with non-finite data (status raised)
      as_global(P.labels)[p] = bi;
      if (P.refine) {
        const double dd = sqdist64(P.X + p * d, P.C + (int64_t)bi * d, d);
        if (P.mindist) as_global(P.mindist)[p] = (float)dd;
        sse = dd;
      }
    }
  }
  if (!CMP64 && tid < TP && tid < nvalid) nc = (unsigned long long)k;
  sse = wave_sum(sse);
  nc = wave_sum_u64(nc);
  if (lane == 0) {
    s_sse[wave] = sse;
    s_corr[wave] = nc;
  }
  __syncthreads();
  if (tid == 0) {
    as_global(P.sse_part)[tile] = s_sse[0] + s_sse[1] + s_sse[2] + s_sse[3];
    as_global(P.corr_part)[tile] = s_corr[0] + s_corr[1] + s_corr[2] + s_corr[3];
  }
}

// ---------------------------------------------------------------------------
// Per-problem fixed-order sums of the per-tile partials.  One workgroup per
// problem.  Writes the SSE to the caller's scalar (if any) and the problem's
// result record (SSE, corrected pairs, status).
// ---------------------------------------------------------------------------

// End of a Lloyd round of one owner-path problem, in one launch: the
// pass's partial reduction, then the update's shift and SSE (the bodies of
// k_reduce_parts and k_upd_own_shift, in that order).
__global__ void __launch_bounds__(256) k_round_tail(const ReduceProb* __restrict__ rp,
                                                    const UpdateProb* __restrict__ up) {
  __shared__ double ss[256];
  __shared__ unsigned long long sc[256];
  reduce_parts_prob(*rp, ss, sc);
  __syncthreads();
  own_shift_prob(*up, up->sse_out, ss);
}

hipError_t launch_round_tail(const ReduceProb* drp, const UpdateProb* dup, hipStream_t st) {
  hipLaunchKernelGGL(k_round_tail, dim3(1), dim3(256), 0, st, drp, dup);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256)
k_reduce_parts(const ReduceProb* __restrict__ probs) {
  __shared__ double ss[256];
  __shared__ unsigned long long sc[256];
  reduce_parts_prob(probs[blockIdx.x], ss, sc);
}

template <class L>
__global__ void k_quantize(const float* __restrict__ in, int64_t count, uint16_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = L::bits(L::cvt(in[i]));
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
template <class L>
static hipError_t launch_prep_t(const PrepProb* dprobs, const int32_t* dstart, int nprob, int nwg,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_prep_centroids<L>, dim3(nwg), dim3(256), 0, st, dprobs, dstart, nprob);
  return hipGetLastError();
}

hipError_t launch_prep(int low, const PrepProb* dprobs, const int32_t* dstart, int nprob, int nwg,
                       hipStream_t st) {
  switch (low) {
    case kLowFP16: return launch_prep_t<LowF16>(dprobs, dstart, nprob, nwg, st);
    case kLowBF16: return launch_prep_t<LowBF16>(dprobs, dstart, nprob, nwg, st);
    case kLowFP32: return launch_prep_t<LowF32>(dprobs, dstart, nprob, nwg, st);
  }
  return hipErrorInvalidValue;
}

template <class L, int DP, int NB>
static hipError_t launch_mfma_t(int mode, bool fallback, const AssignProb* dprobs, const int32_t* dstart,
                                int nprob, int nwg, hipStream_t st) {
  if (mode == 0 || mode == 2) {  // 2: assignment recording the flagged pairs
    if (fallback && mode == 2)
      hipLaunchKernelGGL((k_assign_pipe<L, DP, NB, true, true>), dim3(nwg), dim3(kPipeThreads), 0, st, dprobs, dstart,
                         nprob);
    else if (fallback)
      hipLaunchKernelGGL((k_assign_pipe<L, DP, NB, true>), dim3(nwg), dim3(kPipeThreads), 0, st, dprobs, dstart, nprob);
    else
      hipLaunchKernelGGL((k_assign_pipe<L, DP, NB, false>), dim3(nwg), dim3(kPipeThreads), 0, st, dprobs, dstart, nprob);
  } else {
    if (fallback)
      hipLaunchKernelGGL((k_assign_mfma<L, DP, NB, 1, true>), dim3(nwg), dim3(256), 0, st, dprobs, dstart, nprob);
    else
      hipLaunchKernelGGL((k_assign_mfma<L, DP, NB, 1, false>), dim3(nwg), dim3(256), 0, st, dprobs, dstart, nprob);
  }
  return hipGetLastError();
}

template <class L>
static hipError_t launch_mfma_l(int DP, int mode, bool fallback, const AssignProb* dprobs,
                                const int32_t* dstart, int nprob, int nwg, hipStream_t st) {
  switch (DP) {
    case 16: return launch_mfma_t<L, 16, mfma_nb(kLowFP16, 16)>(mode, fallback, dprobs, dstart, nprob, nwg, st);
    case 32: return launch_mfma_t<L, 32, mfma_nb(kLowFP16, 32)>(mode, fallback, dprobs, dstart, nprob, nwg, st);
    case 64: return launch_mfma_t<L, 64, mfma_nb(kLowFP16, 64)>(mode, fallback, dprobs, dstart, nprob, nwg, st);
    case 128: return launch_mfma_t<L, 128, mfma_nb(kLowFP16, 128)>(mode, fallback, dprobs, dstart, nprob, nwg, st);
    case 256: return launch_mfma_t<L, 256, mfma_nb(kLowFP16, 256)>(mode, fallback, dprobs, dstart, nprob, nwg, st);
  }
  return hipErrorInvalidValue;
}

template <>
hipError_t launch_mfma_l<LowF32>(int DP, int mode, bool fallback, const AssignProb* dprobs,
                                 const int32_t* dstart, int nprob, int nwg, hipStream_t st) {
  switch (DP) {
    case 16: return launch_mfma_t<LowF32, 16, mfma_nb(kLowFP32, 16)>(mode, fallback, dprobs, dstart, nprob, nwg, st);
    case 32: return launch_mfma_t<LowF32, 32, mfma_nb(kLowFP32, 32)>(mode, fallback, dprobs, dstart, nprob, nwg, st);
    case 64: return launch_mfma_t<LowF32, 64, mfma_nb(kLowFP32, 64)>(mode, fallback, dprobs, dstart, nprob, nwg, st);
    case 128: return launch_mfma_t<LowF32, 128, mfma_nb(kLowFP32, 128)>(mode, fallback, dprobs, dstart, nprob, nwg, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_assign_mfma(int low, int DP, int mode, bool fallback, const AssignProb* dprobs,
                              const int32_t* dstart, int nprob, int nwg, hipStream_t st) {
  switch (low) {
    case kLowFP16: return launch_mfma_l<LowF16>(DP, mode, fallback, dprobs, dstart, nprob, nwg, st);
    case kLowBF16: return launch_mfma_l<LowBF16>(DP, mode, fallback, dprobs, dstart, nprob, nwg, st);
    case kLowFP32: return launch_mfma_l<LowF32>(DP, mode, fallback, dprobs, dstart, nprob, nwg, st);
  }
  return hipErrorInvalidValue;
}

template <class L, bool FALLBACK>
static hipError_t launch_small_t(int xd, const AssignProb* dprobs, const int32_t* dstart, int nprob, int nwg,
                                 hipStream_t st) {
  switch (xd) {
    case 8:
      hipLaunchKernelGGL((k_assign_small<L, 8, FALLBACK>), dim3(nwg), dim3(kSmallThreads), 0, st, dprobs, dstart, nprob);
      break;
    case 16:
      hipLaunchKernelGGL((k_assign_small<L, 16, FALLBACK>), dim3(nwg), dim3(kSmallThreads), 0, st, dprobs, dstart, nprob);
      break;
    case 32:
      hipLaunchKernelGGL((k_assign_small<L, 32, FALLBACK>), dim3(nwg), dim3(kSmallThreads), 0, st, dprobs, dstart, nprob);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_assign_small(int low, int xd, bool fallback, const AssignProb* dprobs, const int32_t* dstart,
                               int nprob, int nwg, hipStream_t st) {
  if (low == kLowFP16)
    return fallback ? launch_small_t<LowF16, true>(xd, dprobs, dstart, nprob, nwg, st)
                    : launch_small_t<LowF16, false>(xd, dprobs, dstart, nprob, nwg, st);
  if (low == kLowBF16)
    return fallback ? launch_small_t<LowBF16, true>(xd, dprobs, dstart, nprob, nwg, st)
                    : launch_small_t<LowBF16, false>(xd, dprobs, dstart, nprob, nwg, st);
  return hipErrorInvalidValue;
}

template <class L, bool FALLBACK>
static hipError_t launch_rounds_t(int xd, const RoundProb* dprobs, int nprob, const int32_t* tpre,
                                  const int32_t* cpre, const int32_t* fpre, int* ctl, int work_items,
                                  int lds_bytes, unsigned max_spins, hipStream_t st) {
  const void* f = nullptr;
  switch (xd) {
    case 8: f = reinterpret_cast<const void*>(&k_lloyd_rounds<L, 8, FALLBACK>); break;
    case 16: f = reinterpret_cast<const void*>(&k_lloyd_rounds<L, 16, FALLBACK>); break;
    case 32: f = reinterpret_cast<const void*>(&k_lloyd_rounds<L, 32, FALLBACK>); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
  if (e != hipSuccess) return e;
  int dev = 0, cus = 0, per_cu = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kSmallThreads, lds_bytes);
  if (e != hipSuccess) return e;
  if (per_cu < 1 || cus < 1) return hipErrorInvalidConfiguration;
  const int grid = std::max(1, std::min(per_cu * cus, work_items));
  void* args[] = {(void*)&dprobs, (void*)&nprob, (void*)&tpre, (void*)&cpre, (void*)&fpre, (void*)&ctl,
                  (void*)&max_spins};
  return hipLaunchCooperativeKernel(f, dim3(grid), dim3(kSmallThreads), args, (unsigned)lds_bytes, st);
}

hipError_t launch_lloyd_rounds(int low, int xd, bool fallback, const RoundProb* dprobs, int nprob,
                               const int32_t* tpre, const int32_t* cpre, const int32_t* fpre, int* ctl,
                               int work_items, int lds_bytes, unsigned max_spins, hipStream_t st) {
#define KM_ROUNDS(L, F) \
  launch_rounds_t<L, F>(xd, dprobs, nprob, tpre, cpre, fpre, ctl, work_items, lds_bytes, max_spins, st)
  if (low == kLowFP16) return fallback ? KM_ROUNDS(LowF16, true) : KM_ROUNDS(LowF16, false);
  if (low == kLowBF16) return fallback ? KM_ROUNDS(LowBF16, true) : KM_ROUNDS(LowBF16, false);
#undef KM_ROUNDS
  return hipErrorInvalidValue;
}

// LDS of the persistent round kernel's assignment body
int small_lds_bytes(int xd, bool fallback) {
  switch (xd) {
    case 8: return fallback ? (int)sizeof(SmallLds<8, true>) : (int)sizeof(SmallLds<8, false>);
    case 16: return fallback ? (int)sizeof(SmallLds<16, true>) : (int)sizeof(SmallLds<16, false>);
    case 32: return fallback ? (int)sizeof(SmallLds<32, true>) : (int)sizeof(SmallLds<32, false>);
  }
  return 0;
}

hipError_t launch_assign_direct64(bool cmp64, int arith, int mode, const AssignProb* dprobs,
                                  const int32_t* dstart, int nprob, int nwg, hipStream_t st) {
#define KM_DIRECT(C, M, AR) \
  hipLaunchKernelGGL((k_assign_direct64<C, M, AR>), dim3(nwg), dim3(256), 0, st, dprobs, dstart, nprob)
  if (cmp64) {
    if (arith != 0) return hipErrorInvalidValue;
    if (mode == 0) KM_DIRECT(true, 0, 0);
    else KM_DIRECT(true, 1, 0);
    return hipGetLastError();
  }
  switch (arith * 2 + (mode != 0)) {
    case 0: KM_DIRECT(false, 0, 0); break;
    case 1: KM_DIRECT(true, 1, 0); break;  // materialised values are the same
    case 2: KM_DIRECT(false, 0, 1); break;
    case 3: KM_DIRECT(true, 1, 1); break;
    case 4: KM_DIRECT(false, 0, 2); break;
    case 5: KM_DIRECT(true, 1, 2); break;
    case 6: KM_DIRECT(false, 0, 3); break;
    case 7: KM_DIRECT(true, 1, 3); break;
    default: return hipErrorInvalidValue;
  }
#undef KM_DIRECT
  return hipGetLastError();
}

// Clears a small device range (status words and result records before a
// pass): one launch, and usable where a memset node is not.
__global__ void __launch_bounds__(256) k_zero_words(uint32_t* __restrict__ p, int nwords) {
  for (int i = threadIdx.x; i < nwords; i += 256) as_global(p)[i] = 0u;
}

// Byte-exact fill of a device range (diagnostic flag maps).
__global__ void __launch_bounds__(256) k_fill_bytes(uint8_t* __restrict__ p, int64_t count, uint8_t v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256)
    as_global(p)[i] = v;
}

hipError_t launch_fill_bytes(void* p, int64_t count, uint8_t v, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((count + 255) / 256, 16384);
  hipLaunchKernelGGL(k_fill_bytes, dim3((unsigned)blocks), dim3(256), 0, st, reinterpret_cast<uint8_t*>(p), count, v);
  return hipGetLastError();
}

hipError_t launch_zero_words(void* p, size_t bytes, hipStream_t st) {
  const int nwords = (int)((bytes + 3) / 4);
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, st, reinterpret_cast<uint32_t*>(p), nwords);
  return hipGetLastError();
}

// Copies the result records of many problems into one contiguous array (one
// device-to-host copy then reads them all).
__global__ void __launch_bounds__(256) k_gather_results(const KResult* const* __restrict__ src, int count,
                                                        KResult* __restrict__ dst) {
  constexpr int W = (int)(sizeof(KResult) / 4);
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= count * W) return;
  const int r = i / W, w = i - r * W;
  as_global(reinterpret_cast<uint32_t*>(dst))[i] = as_global(reinterpret_cast<const uint32_t*>(src[r]))[w];
}

hipError_t launch_gather_results(const KResult* const* dsrc, int count, KResult* ddst, hipStream_t st) {
  const int words = count * (int)(sizeof(KResult) / 4);
  if (words == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_results, dim3((words + 255) / 256), dim3(256), 0, st, dsrc, count, ddst);
  return hipGetLastError();
}

hipError_t launch_reduce_parts(const ReduceProb* dprobs, int nprob, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_parts, dim3(nprob), dim3(256), 0, st, dprobs);
  return hipGetLastError();
}

hipError_t launch_quantize(int low, const float* in, int64_t count, uint16_t* out, hipStream_t st) {
  const int64_t nwg = (count + 255) / 256;
  if (nwg == 0) return hipSuccess;
  if (low == kLowFP16) hipLaunchKernelGGL(k_quantize<LowF16>, dim3((unsigned)nwg), dim3(256), 0, st, in, count, out);
  else if (low == kLowBF16) hipLaunchKernelGGL(k_quantize<LowBF16>, dim3((unsigned)nwg), dim3(256), 0, st, in, count, out);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace km
