// km_update.hip -- centre update of Lloyd's iteration (eq:center,
// Algorithm alg:mp-kmeans) on gfx950.
//
// c_j <- fl32( (sum_{i: label_i = j} x_i) / m_j ),  m_j = 0 keeps c_j.
//
// The sums are FP64 and their order is fixed by the data alone (never by the
// launch or by other problems sharing it), so results are bitwise
// reproducible and identical whether a problem runs alone or batched:
//   1. hist      per 1024-point tile, label counts (integer LDS atomics:
//                order-free);
//   2. scan_rel  per cluster, exclusive scan of its tile counts;
//   3. scan_cl   per problem, cluster starts and chunk starts;
//   4. scatter   stable counting sort of point indices by label: members of
//                a cluster appear in ascending point order;
//   5. chunksum  one wave per chunk of consecutive members of one cluster
//                (64, or 512 when d <= 16): FP64 sums over fixed member
//                groups, combined by a fixed butterfly;
//   6. finalize  per cluster, sum of its chunk partials in a fixed
//                lane-strided order with a fixed butterfly, division,
//                one rounding to FP32, empty clusters keep their centre,
//                squared move;
//   7. shift     per problem, max_j ||c_j^new - c_j^old|| (FP64), and, when
//                asked, the SSE of the labels against C_old: per-chunk FP64
//                partials from the chunk sums (they read every member row
//                anyway), summed per cluster by finalize, then over clusters.
// No floating-point atomics anywhere.
#include <algorithm>
#include <type_traits>

#include "km_device.hpp"
#include "km_internal.hpp"
#include "km_update_dev.hpp"

namespace km {

__device__ inline int find_prob(const int32_t* __restrict__ start, int nprob, int b) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

constexpr int kHistSlice = 8192;  // clusters counted per LDS pass

// 1. per-tile label histogram -> hist[j * ntiles + tile]
__global__ void __launch_bounds__(256)
k_upd_hist(const UpdateProb* __restrict__ probs, const int32_t* __restrict__ wg_start, int nprob) {
  __shared__ int cnt[kHistSlice];
  const int pi = find_prob(wg_start, nprob, blockIdx.x);
  const UpdateProb& P = probs[pi];
  const int tile = blockIdx.x - wg_start[pi];
  const int64_t p0 = (int64_t)tile * kUpdTile;
  const int m = (int)((P.n - p0) < kUpdTile ? (P.n - p0) : kUpdTile);
  int bad = 0;
  for (int s0 = 0; s0 < P.k; s0 += kHistSlice) {
    const int sl = (P.k - s0) < kHistSlice ? (P.k - s0) : kHistSlice;
    for (int j = threadIdx.x; j < sl; j += 256) cnt[j] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += 256) {
      const int lab = as_global(P.labels)[p0 + i];
      if (lab < 0 || lab >= P.k) bad = 1;
      else if (lab >= s0 && lab < s0 + sl) atomicAdd(&cnt[lab - s0], 1);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < sl; j += 256) as_global(P.hist)[(int64_t)(s0 + j) * P.ntiles + tile] = cnt[j];
    __syncthreads();
  }
  if (bad) atomicOr(P.status, kStatusBadLabel);
}

// 2. per cluster: exclusive scan over its tiles -> offs, total -> cstart[j]
__global__ void __launch_bounds__(256)
k_upd_scan_rel(const UpdateProb* __restrict__ probs, const int32_t* __restrict__ wg_start, int nprob) {
  __shared__ int part[256];
  const int pi = find_prob(wg_start, nprob, blockIdx.x);
  const UpdateProb& P = probs[pi];
  const int j = blockIdx.x - wg_start[pi];
  const int T = P.ntiles;
  const int per = (T + 255) / 256;
  const int t0 = threadIdx.x * per;
  const KM_GLOBAL int32_t* h = as_global(P.hist) + (int64_t)j * T;
  KM_GLOBAL int32_t* o = as_global(P.offs) + (int64_t)j * T;
  int s = 0;
  for (int t = t0; t < t0 + per && t < T; ++t) s += h[t];
  part[threadIdx.x] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan of the 256 partial sums
  for (int off = 1; off < 256; off <<= 1) {
    int v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int run = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0;
  for (int t = t0; t < t0 + per && t < T; ++t) {
    o[t] = run;
    run += h[t];
  }
  if (threadIdx.x == 255) as_global(P.cstart)[j] = part[255];  // count, scanned by k_upd_scan_cl
}

// 3. per problem: counts -> exclusive cluster starts and chunk starts
__global__ void __launch_bounds__(1024)
k_upd_scan_cl(const UpdateProb* __restrict__ probs) {
  __shared__ int a[1024];
  __shared__ int b[1024];
  __shared__ int carry[2];
  const UpdateProb& P = probs[blockIdx.x];
  const int tid = threadIdx.x;
  if (tid == 0) {
    carry[0] = 0;
    carry[1] = 0;
  }
  __syncthreads();
  for (int base = 0; base < P.k; base += 1024) {
    const int j = base + tid;
    const int mj = j < P.k ? as_global(P.cstart)[j] : 0;
    const int cj = (mj + P.chunk - 1) / P.chunk;
    a[tid] = mj;
    b[tid] = cj;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      int va = tid >= off ? a[tid - off] : 0;
      int vb = tid >= off ? b[tid - off] : 0;
      __syncthreads();
      a[tid] += va;
      b[tid] += vb;
      __syncthreads();
    }
    const int c0 = carry[0], c1 = carry[1];
    if (j < P.k) {
      as_global(P.cstart)[j] = c0 + a[tid] - mj;
      as_global(P.chunk_start)[j] = c1 + b[tid] - cj;
    }
    __syncthreads();
    if (tid == 1023) {
      carry[0] = c0 + a[1023];
      carry[1] = c1 + b[1023];
    }
    __syncthreads();
  }
  if (tid == 0) {
    as_global(P.cstart)[P.k] = carry[0];
    as_global(P.chunk_start)[P.k] = carry[1];
  }
}

// 4. stable scatter of point indices into cluster order.  One wave per
// 1024-point tile walks the tile in 16 rounds of 64 points.  In a round each
// lane finds the lanes holding its label from one ballot per label bit (the
// lanes that agree with it on every bit), ranks itself among them by lane
// order and is placed after the earlier rounds' points of that label
// (per-wave counters in LDS, advanced by the group's lowest lane).  Members
// of a cluster thus appear in ascending point order.  k > kScatterLds uses
// the brute-force rank.
constexpr int kScatterLds = 4096;

__global__ void __launch_bounds__(256)
k_upd_scatter(const UpdateProb* __restrict__ probs, const int32_t* __restrict__ wg_start, int nprob) {
  __shared__ int cnt[4][kScatterLds];
  const int pi = find_prob(wg_start, nprob, blockIdx.x);
  const UpdateProb& P = probs[pi];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tile = (blockIdx.x - wg_start[pi]) * 4 + wave;
  if (tile >= P.ntiles) return;
  const int64_t p0 = (int64_t)tile * kUpdTile;
  const int m = (int)((P.n - p0) < kUpdTile ? (P.n - p0) : kUpdTile);
  if (P.k <= kScatterLds) {
    int* c = cnt[wave];
    // running output position of each cluster for this tile
    for (int j = lane; j < P.k; j += 64) c[j] = as_global(P.cstart)[j] + as_global(P.offs)[(int64_t)j * P.ntiles + tile];
    int nbits = 0;
    while ((1 << nbits) < P.k) ++nbits;
    const unsigned long long below = (1ull << lane) - 1;
    for (int r0 = 0; r0 < m; r0 += 64) {
      const int i = r0 + lane;
      const int lab = i < m ? as_global(P.labels)[p0 + i] : -1;
      const bool ok = lab >= 0 && lab < P.k;
      unsigned long long grp = __ballot(ok);
      for (int b = 0; b < nbits; ++b) {
        const bool bit = (lab >> b) & 1;
        const unsigned long long mb = __ballot(ok && bit);
        grp &= bit ? mb : ~mb;
      }
      // grp: the valid lanes whose label equals this lane's (this lane
      // included when ok)
      if (ok) {
        const int base = c[lab];
        as_global(P.perm)[base + __popcll(grp & below)] = (int32_t)(p0 + i);
      }
      // every lane of the round has read its counter above before any
      // group leader writes it (the wave executes the reads first)
      if (ok && (grp & below) == 0) c[lab] += __popcll(grp);
    }
  } else {
    for (int i = lane; i < m; i += 64) {
      const int lab = as_global(P.labels)[p0 + i];
      if (lab < 0 || lab >= P.k) continue;
      int rank = 0;
      for (int q = 0; q < i; ++q) rank += (as_global(P.labels)[p0 + q] == lab);
      const int pos = as_global(P.cstart)[lab] + as_global(P.offs)[(int64_t)lab * P.ntiles + tile] + rank;
      as_global(P.perm)[pos] = (int32_t)(p0 + i);
    }
  }
}

// 5. one wave per chunk of members of one cluster (P.chunk at most).  Lanes are split
// into G member groups x L lanes per member row; each lane sums its group's
// members (every G-th member, ascending) in FP64 over its coordinates, then
// the groups are combined by a fixed butterfly.  The order depends only on
// the chunk.  Rows of 16-byte aligned data with d % 4 == 0 are read as float4
// (L = lanes for d/4 vectors, rounded up to a power of two), other rows one
// coordinate per lane (L = lanes for d, up to 64, several coordinates per
// lane beyond 64).
template <bool VEC>
__device__ inline void chunk_rows(const UpdateProb& P, int c, int j, int m0, int m1, int lane) {
  const int d = P.d;
  const int per = VEC ? 4 : 1;              // coordinates per load
  const int nv = (d + per - 1) / per;       // loads per row
  int L = 1;
  while (L < nv && L < 64) L <<= 1;
  const int G = 64 / L;                     // member groups
  const int g = lane / L, cl = lane % L;
  constexpr int kMaxSlots = VEC ? 1 : 4;    // VEC: d <= 256 -> <= 64 vectors
  const int nslot = (nv + 63) / 64;
  double s[kMaxSlots][4];
#pragma unroll
  for (int q = 0; q < kMaxSlots; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e) s[q][e] = 0.0;
  const KM_GLOBAL float* __restrict__ X = as_global(P.X);
  // SSE against the centre the members were assigned to: this lane's
  // coordinates of C_old[j] (zero where the lane holds none)
  const bool want_sse = P.sse_out != nullptr;
  double e2 = 0.0;
  double cv[kMaxSlots][4];
#pragma unroll
  for (int q = 0; q < kMaxSlots; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int l = per * (cl + 64 * q) + e;
      cv[q][e] = (want_sse && q < nslot && e < per && l < d) ? (double)as_global(P.C_old)[(int64_t)j * d + l] : 0.0;
    }
  auto add_sq = [&](int q, int e, float x) {
    const double t = (double)x - cv[q][e];
    e2 = __builtin_fma(t, t, e2);
  };
  auto add_row = [&](int id) {
#pragma unroll
    for (int q = 0; q < kMaxSlots; ++q) {
      if (q >= nslot) break;
      const int v = cl + 64 * q;
      if (v >= nv) continue;
      if constexpr (VEC) {
        const f32x4 x = *reinterpret_cast<const KM_GLOBAL f32x4*>(X + (int64_t)id * d + 4 * v);
        s[q][0] += (double)x.x;
        s[q][1] += (double)x.y;
        s[q][2] += (double)x.z;
        s[q][3] += (double)x.w;
        if (want_sse) {
          add_sq(q, 0, x.x);
          add_sq(q, 1, x.y);
          add_sq(q, 2, x.z);
          add_sq(q, 3, x.w);
        }
      } else {
        const float x = X[(int64_t)id * d + v];
        s[q][0] += (double)x;
        if (want_sse) add_sq(q, 0, x);
      }
    }
  };
  int mm = m0 + g;
  // 8 members per group and batch: all their loads are independent
  for (; mm + 7 * G < m1; mm += 8 * G) {
    int idx[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) idx[u] = as_global(P.perm)[mm + u * G];
    if constexpr (VEC) {
      f32x4 xv[8];
      const int v = cl;
      const bool on = v < nv;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        xv[u] = on ? *reinterpret_cast<const KM_GLOBAL f32x4*>(X + (int64_t)idx[u] * d + 4 * v) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        s[0][0] += (double)xv[u].x;
        s[0][1] += (double)xv[u].y;
        s[0][2] += (double)xv[u].z;
        s[0][3] += (double)xv[u].w;
      }
      if (want_sse && on) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          add_sq(0, 0, xv[u].x);
          add_sq(0, 1, xv[u].y);
          add_sq(0, 2, xv[u].z);
          add_sq(0, 3, xv[u].w);
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < 8; ++u) add_row(idx[u]);
    }
  }
  for (; mm < m1; mm += G) add_row(as_global(P.perm)[mm]);
  // combine the G groups (fixed butterfly over the group bits)
  for (int o = L; o < 64; o <<= 1) {
#pragma unroll
    for (int q = 0; q < kMaxSlots; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) s[q][e] += __shfl_xor(s[q][e], o, kWave);
  }
  if (g == 0) {
#pragma unroll
    for (int q = 0; q < kMaxSlots; ++q) {
      if (q >= nslot) break;
      const int v = cl + 64 * q;
      if (v >= nv) continue;
#pragma unroll
      for (int e = 0; e < per; ++e) {
        const int l = per * v + e;
        if (l < d) as_global(P.chunk_sum)[(int64_t)c * d + l] = s[q][e];
      }
    }
  }
  if (want_sse) {
    e2 = wave_sum(e2);
    if (lane == 0) as_global(P.sse_chunk)[c] = e2;
  }
}

__global__ void __launch_bounds__(256)
k_upd_chunksum(const UpdateProb* __restrict__ probs, const int32_t* __restrict__ wg_start, int nprob) {
  const int pi = find_prob(wg_start, nprob, blockIdx.x);
  const UpdateProb& P = probs[pi];
  const int c = (blockIdx.x - wg_start[pi]) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= as_global(P.chunk_start)[P.k]) return;
  // cluster owning chunk c
  int lo = 0, hi = P.k - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (as_global(P.chunk_start)[mid] <= c) lo = mid; else hi = mid - 1;
  }
  const int j = lo;
  const int m0 = as_global(P.cstart)[j] + (c - as_global(P.chunk_start)[j]) * P.chunk;
  const int m1 = (m0 + P.chunk) < as_global(P.cstart)[j + 1] ? (m0 + P.chunk) : as_global(P.cstart)[j + 1];
  if ((P.d & 3) == 0 && (((uintptr_t)P.X) & 15) == 0)
    chunk_rows<true>(P, c, j, m0, m1, lane);
  else
    chunk_rows<false>(P, c, j, m0, m1, lane);
}

// 6. per cluster: sum of its chunk partials, divide, round, keep empty.
// Lanes are split into G chunk groups x L lanes per coordinate block (L the
// coordinate count rounded up to a power of two, at most 64): group g sums
// chunks c0+g, c0+g+G, ... in ascending order and the groups are combined by
// a fixed butterfly, so the order depends only on the cluster's chunk count.
__global__ void __launch_bounds__(256)
k_upd_finalize(const UpdateProb* __restrict__ probs, const int32_t* __restrict__ wg_start, int nprob) {
  const int pi = find_prob(wg_start, nprob, blockIdx.x);
  const UpdateProb& P = probs[pi];
  const int j = (blockIdx.x - wg_start[pi]) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= P.k) return;
  const int mj = as_global(P.cstart)[j + 1] - as_global(P.cstart)[j];
  const int c0 = as_global(P.chunk_start)[j], c1 = as_global(P.chunk_start)[j + 1];
  const int d = P.d;
  int L = 1;
  while (L < d && L < 64) L <<= 1;
  const int G = 64 / L;
  const int g = lane / L, cl = lane % L;
  double mv2 = 0.0;
  for (int l0 = 0; l0 < d; l0 += L) {
    const int l = l0 + cl;
    double s = 0.0;
    if (l < d && mj > 0) {
#pragma unroll 4
      for (int c = c0 + g; c < c1; c += G) s += as_global(P.chunk_sum)[(int64_t)c * d + l];
    }
    for (int o = L; o < 64; o <<= 1) s += __shfl_xor(s, o, kWave);
    if (g == 0 && l < d) {
      const float old = as_global(P.C_old)[(int64_t)j * d + l];
      const float nv = mj > 0 ? (float)(s / (double)mj) : old;
      as_global(P.C_new)[(int64_t)j * d + l] = nv;
      const double df = (double)nv - (double)old;
      mv2 += df * df;
    }
  }
  mv2 = wave_sum(mv2);
  if (P.sse_out && c1 > c0) {  // the cluster's SSE: lane-strided chunks, fixed butterfly
    double e = 0.0;
    for (int c = c0 + lane; c < c1; c += 64) e += as_global(P.sse_chunk)[c];
    e = wave_sum(e);
    if (lane == 0) as_global(P.sse_chunk)[c0] = e;
  }
  if (lane == 0) {
    as_global(P.shift2)[j] = mv2;
    if (P.counts_out) as_global(P.counts_out)[j] = mj;
  }
}

// 7. per problem: shift = max_j sqrt(shift2[j])
__global__ void __launch_bounds__(256)
k_upd_shift(const UpdateProb* __restrict__ probs) {
  __shared__ double mx[256];
  const UpdateProb& P = probs[blockIdx.x];
  if (P.sse_out) {  // SSE: per-cluster sums (in each cluster's first chunk
                    // slot), per-thread strided sums, then a fixed tree
    double e = 0.0;
    for (int j = threadIdx.x; j < P.k; j += 256) {
      const int c0 = as_global(P.chunk_start)[j];
      if (as_global(P.chunk_start)[j + 1] > c0) e += as_global(P.sse_chunk)[c0];
    }
    mx[threadIdx.x] = e;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
      if (threadIdx.x < o) mx[threadIdx.x] += mx[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) *as_global(P.sse_out) = mx[0];
    __syncthreads();
  }
  double v = 0.0;
  for (int j = threadIdx.x; j < P.k; j += 256) v = __builtin_fmax(v, as_global(P.shift2)[j]);
  mx[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (threadIdx.x < o) mx[threadIdx.x] = __builtin_fmax(mx[threadIdx.x], mx[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double s = __builtin_sqrt(mx[0]);
    if (P.shift_out) *P.shift_out = s;
    if (P.result) P.result->shift = s;
  }
}

// dscratch_i32 layout (device): [0, nprob] tile prefix, [nprob+1, 2nprob+1]
// cluster prefix, then chunk-wave prefix and cluster-wave prefix.
hipError_t launch_update(const UpdateProb* dprobs, const UpdateProb* hprobs, int nprob,
                         const int32_t* dpre, hipStream_t st) {
  int tiles = 0, clusters = 0, chunkwg = 0, clwg = 0, scatwg = 0;
  for (int i = 0; i < nprob; ++i) {
    tiles += hprobs[i].ntiles;
    scatwg += (hprobs[i].ntiles + 3) / 4;
    clusters += hprobs[i].k;
    chunkwg += (int)((hprobs[i].n + hprobs[i].chunk - 1) / hprobs[i].chunk + hprobs[i].k + 3) / 4;
    clwg += (hprobs[i].k + 3) / 4;
  }
  const int32_t* pre_tiles = dpre;
  const int32_t* pre_cl = dpre + (nprob + 1);
  const int32_t* pre_chunk = dpre + 2 * (nprob + 1);
  const int32_t* pre_clwg = dpre + 3 * (nprob + 1);
  const int32_t* pre_scat = dpre + 4 * (nprob + 1);
  if (tiles > 0) hipLaunchKernelGGL(k_upd_hist, dim3(tiles), dim3(256), 0, st, dprobs, pre_tiles, nprob);
  hipLaunchKernelGGL(k_upd_scan_rel, dim3(clusters), dim3(256), 0, st, dprobs, pre_cl, nprob);
  hipLaunchKernelGGL(k_upd_scan_cl, dim3(nprob), dim3(1024), 0, st, dprobs);
  if (tiles > 0) hipLaunchKernelGGL(k_upd_scatter, dim3(scatwg), dim3(256), 0, st, dprobs, pre_scat, nprob);
  if (chunkwg > 0) hipLaunchKernelGGL(k_upd_chunksum, dim3(chunkwg), dim3(256), 0, st, dprobs, pre_chunk, nprob);
  hipLaunchKernelGGL(k_upd_finalize, dim3(clwg), dim3(256), 0, st, dprobs, pre_clwg, nprob);
  hipLaunchKernelGGL(k_upd_shift, dim3(nprob), dim3(256), 0, st, dprobs);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Owner-path kernels, one launch per phase (bodies in km_update_dev.hpp).
template <int NC, bool SSE>
__global__ void __launch_bounds__(256)
k_upd_own_part(const UpdateProb* __restrict__ probs, const int32_t* __restrict__ wg_start, int nprob,
               int wstride) {
  extern __shared__ __attribute__((aligned(16))) char s_dyn[];
  __shared__ double s_sse[kOwnWaves];
  const int pi = find_prob(wg_start, nprob, blockIdx.x);
  own_part_chunk<NC, SSE>(probs[pi], blockIdx.x - wg_start[pi], s_dyn, wstride, s_sse);
}

__global__ void __launch_bounds__(256)
k_upd_own_fin(const UpdateProb* __restrict__ probs, const int32_t* __restrict__ wg_start, int nprob) {
  __shared__ int s_m[256];
  __shared__ double s_sq[256];
  const int pi = find_prob(wg_start, nprob, blockIdx.x);
  own_fin_group(probs[pi], blockIdx.x - wg_start[pi], s_m, s_sq);
}

__global__ void __launch_bounds__(256)
k_upd_own_shift(const UpdateProb* __restrict__ probs) {
  __shared__ double red[256];
  const UpdateProb& P = probs[blockIdx.x];
  own_shift_prob(P, P.sse_out, red);
}

// Part launch over problems that share nc and the SSE request; dpre is the
// device chunk prefix of these problems.
hipError_t launch_update_own_part(const UpdateProb* dprobs, const UpdateProb* hprobs, int nprob,
                                  const int32_t* dpre, hipStream_t st) {
  if (nprob < 1) return hipSuccess;
  int chunks = 0, wstride = 16, kd_max = 1;
  const int nc = hprobs[0].nc;
  const bool sse = hprobs[0].sse_out != nullptr;
  for (int i = 0; i < nprob; ++i) {
    const UpdateProb& u = hprobs[i];
    if (u.nc != nc || (u.sse_out != nullptr) != sse || u.owners < 1) return hipErrorInvalidValue;
    chunks += u.nchunk;
    wstride = std::max(wstride, own_wave_bytes(u.owners, u.d, u.k));
    kd_max = std::max(kd_max, u.k * u.d);
  }
  if (chunks == 0) return hipSuccess;
  const size_t lds = (size_t)kOwnWaves * wstride + (sse ? (size_t)kd_max * 4 : 0);
  auto go = [&](auto kern) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(chunks), dim3(256), lds, st, dprobs, dpre, nprob, wstride);
    return hipGetLastError();
  };
  if (nc == 1) return sse ? go(k_upd_own_part<1, true>) : go(k_upd_own_part<1, false>);
  if (nc == 2) return sse ? go(k_upd_own_part<2, true>) : go(k_upd_own_part<2, false>);
  return hipErrorInvalidValue;
}

// Finalize and shift launches over all owner-path problems of a round; dpre
// is the device finalize prefix.
hipError_t launch_update_own_fin(const UpdateProb* dprobs, const UpdateProb* hprobs, int nprob,
                                 const int32_t* dpre, hipStream_t st, bool shift) {
  if (nprob < 1) return hipSuccess;
  int fin = 0;
  for (int i = 0; i < nprob; ++i) {
    const int J = own_fin_clusters(hprobs[i].d);
    fin += (hprobs[i].k + J - 1) / J;
  }
  hipLaunchKernelGGL(k_upd_own_fin, dim3(fin), dim3(256), 0, st, dprobs, dpre, nprob);
  if (shift) hipLaunchKernelGGL(k_upd_own_shift, dim3(nprob), dim3(256), 0, st, dprobs);
  return hipGetLastError();
}

}  // namespace km
