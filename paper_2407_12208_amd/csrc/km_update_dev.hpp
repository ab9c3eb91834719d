// km_update_dev.hpp -- device bodies of the centre update's owner path for
// small k*d (eq:center): per-chunk partials, per cluster group the cross-chunk
// sums, per problem the shift and SSE.  The one-launch-per-phase kernels of
// the update and the persistent round kernel both run these bodies, so they
// compute bitwise the same centres.
#pragma once

#include "km_device.hpp"
#include "km_internal.hpp"

namespace km {

// ---------------------------------------------------------------------------
// Owner path for small k*d (no sort): per-chunk partials, then per cluster
// group the cross-chunk sums, then per problem the shift and SSE.
//
// Chunk c of a problem is points [c*S, (c+1)*S), S = 4 waves x owners x I,
// I = P.iters points per owner (256, fewer for small n: own_iters).
// Wave w of the chunk's workgroup takes the run [c*S + w*owners*I, +owners*I)
// and owner o of the wave its points o, o+owners, o+2*owners, ... in order.
// Each lane of an owner holds one coordinate (two when d > 64) and adds the
// point's value into the owner's FP64 accumulator of the point's cluster in
// LDS.  Every accumulator has exactly one writing lane and the wave's LDS
// operations complete in issue order, so each is a sequential sum in point
// order.  The chunk partial of (j, l) is then the sum over waves (in order)
// of the sums over owners (in order); the finalize sums the chunk partials in
// chunk order.  The partition depends only on (n, d, k): a problem gets the
// same bits alone, batched or served.
__device__ inline void lds_add_f64(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// LDS (dynamic, sized per launch): 4 wave regions of `wstride` bytes, then
// C_old as FP32 rows (SSE only).  The stride only places the regions; the
// arithmetic of a problem does not depend on it.
// One chunk of a problem (s_dyn: the LDS above; s_sse: kOwnWaves doubles).
template <int NC, bool SSE>
__device__ __attribute__((always_inline)) inline void
own_part_chunk(const UpdateProb& P, const int chunk, char* s_dyn, const int wstride, double* s_sse) {
  char* s_acc = s_dyn;
  float* s_c = reinterpret_cast<float*>(s_dyn + kOwnWaves * wstride);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int k = P.k, d = P.d, O = P.owners, LP = P.lp;
  const int kd = k * d;
  const int64_t n = P.n;
  const int o = lane / LP, l = lane - o * LP;
  const bool active = o < O;
  double* acc = reinterpret_cast<double*>(s_acc + wave * wstride);  // [O][k][d]
  int* cnt = reinterpret_cast<int*>(acc + (size_t)O * kd);                 // [O][k]
  {
    const int words = (O * kd * 8 + O * k * 4 + 7) / 8;
    unsigned long long* z = reinterpret_cast<unsigned long long*>(acc);
    for (int e = lane; e < words; e += 64) z[e] = 0ull;
  }
  if constexpr (SSE) {
    for (int e = tid; e < kd; e += 256) s_c[e] = as_global(P.C_old)[e];
  }
  __syncthreads();

  const int I = P.iters;  // points per owner (32..256, a multiple of 2 x 16)
  const int64_t run0 = (int64_t)chunk * (kOwnWaves * O * I) + (int64_t)wave * O * I;
  double e2 = 0.0;
  int bad = 0;
  // lanes past the last owner load what the last owner loads and add nothing;
  // a second coordinate past d loads coordinate d-1 and adds nothing
  const int oc = active ? o : O - 1;
  int cc[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) cc[q] = (l + q * LP) < d ? (l + q * LP) : d - 1;
  auto add_point = [&](int j, const float (&xr)[NC]) __attribute__((always_inline)) {
    if ((unsigned)j >= (unsigned)k) {
      bad = 1;
      return;
    }
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      if (NC == 1 || l + q * LP < d) {
        const double x = (double)xr[q];
        lds_add_f64(&acc[(o * k + j) * d + l + q * LP], x);
        if constexpr (SSE) {
          const double t = x - (double)s_c[j * d + l + q * LP];
          e2 = __builtin_fma(t, t, e2);
        }
      }
    }
    if (l == 0) atomicAdd(&cnt[o * k + j], 1);
  };
  // the run's points inside the problem (the last run of a problem is cut)
  const int64_t lim64 = n - run0;
  const int lim = lim64 < (int64_t)O * I ? (int)lim64 : O * I;
  auto run = [&](auto tail) __attribute__((always_inline)) {
    constexpr bool TAIL = decltype(tail)::value;
    // unsigned 32-bit offsets from the run's base (a run spans at most
    // 64 x 256 points of at most 128 coordinates); in a cut run, points past
    // the problem load its last point and add nothing
    const KM_GLOBAL int32_t* __restrict__ lab_g = as_global(P.labels) + run0;
    const KM_GLOBAL float* __restrict__ X = as_global(P.X) + run0 * d;
    const unsigned ud = (unsigned)d, ulast = (unsigned)(lim - 1);
    constexpr int U = 16;  // points per owner in flight
    int lab[2][U];
    float xv[2][U][NC];
    auto fetch = [&](int buf, int i0) __attribute__((always_inline)) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        unsigned r = (unsigned)((i0 + u) * O + oc);
        if constexpr (TAIL) r = r < ulast ? r : ulast;
        lab[buf][u] = lab_g[r];
#pragma unroll
        for (int q = 0; q < NC; ++q) xv[buf][u][q] = X[r * ud + (unsigned)cc[q]];
      }
    };
    auto consume = [&](int buf, int i0) __attribute__((always_inline)) {
      if (!active) return;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (TAIL && (i0 + u) * O + o >= lim) break;
        add_point(lab[buf][u], xv[buf][u]);
      }
    };
    fetch(0, 0);
#pragma unroll 1
    for (int i0 = 0; i0 < I - 2 * U; i0 += 2 * U) {
      if (TAIL && i0 * O >= lim) return;
      fetch(1, i0 + U);
      consume(0, i0);
      fetch(0, i0 + 2 * U);
      consume(1, i0 + U);
    }
    fetch(1, I - U);
    consume(0, I - 2 * U);
    consume(1, I - U);
  };
  if (lim == O * I) run(std::false_type{});
  else if (lim > 0) run(std::true_type{});
  if (bad) atomicOr(P.status, kStatusBadLabel);
  if constexpr (SSE) {
    e2 = wave_sum(e2);
    if (lane == 0) s_sse[wave] = e2;
  }
  __syncthreads();
  // chunk partials: waves in order, owners in order
  KM_GLOBAL double* pacc = as_global(P.pacc) + (int64_t)chunk * kd;
  for (int e = tid; e < kd; e += 256) {
    double s = 0.0;
    for (int w = 0; w < kOwnWaves; ++w) {
      const double* aw = reinterpret_cast<const double*>(s_acc + w * wstride);
      for (int oo = 0; oo < O; ++oo) s += aw[oo * kd + e];
    }
    pacc[e] = s;
  }
  KM_GLOBAL int32_t* pcnt = as_global(P.pcnt) + (int64_t)chunk * k;
  for (int j = tid; j < k; j += 256) {
    int m = 0;
    for (int w = 0; w < kOwnWaves; ++w) {
      const int* cw = reinterpret_cast<const int*>(s_acc + w * wstride + (size_t)O * kd * 8);
      for (int oo = 0; oo < O; ++oo) m += cw[oo * k + j];
    }
    pcnt[j] = m;
  }
  if (SSE && tid == 0) as_global(P.psse)[chunk] = ((s_sse[0] + s_sse[1]) + s_sse[2]) + s_sse[3];
}

// Per group of clusters: chunk partials summed in chunk order, division,
// one rounding to FP32, empty clusters keep their centre, squared move.
// Cluster group `grp` of a problem (s_m: 256 ints, s_sq: 256 doubles).
__device__ __attribute__((always_inline)) inline void
own_fin_group(const UpdateProb& P, const int grp, int* s_m, double* s_sq) {
  const int k = P.k, d = P.d, kd = k * d, nch = P.nchunk;
  const int J = own_fin_clusters(d);
  const int j0 = grp * J;
  const int nj = (k - j0) < J ? (k - j0) : J;
  const int t = threadIdx.x;
  if (t < nj) {
    const KM_GLOBAL int32_t* pc = as_global(P.pcnt) + j0 + t;
    int m = 0;
#pragma unroll 8
    for (int c = 0; c < nch; ++c) m += pc[(int64_t)c * k];  // integers: any order
    s_m[t] = m;
    if (P.counts_out) as_global(P.counts_out)[j0 + t] = m;
  }
  __syncthreads();
  // J * d <= 256: one entry per thread
  double df2 = 0.0;
  if (t < nj * d) {
    const int jl = t / d;
    const int64_t g = (int64_t)j0 * d + t;
    const KM_GLOBAL double* pa = as_global(P.pacc) + g;
    // chunk c goes to partial c % 8, each partial in chunk order, then the
    // partials in a fixed tree: the order depends only on the chunk count
    double sp[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) sp[q] = 0.0;
    int c = 0;
    // 32 loads in flight, added in the same order as 8 at a time
    for (; c + 32 <= nch; c += 32) {
      double v[32];
#pragma unroll
      for (int q = 0; q < 32; ++q) v[q] = pa[(int64_t)(c + q) * kd];
#pragma unroll
      for (int q = 0; q < 32; ++q) sp[q & 7] += v[q];
    }
    for (; c + 8 <= nch; c += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = pa[(int64_t)(c + q) * kd];
#pragma unroll
      for (int q = 0; q < 8; ++q) sp[q] += v[q];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (c + q < nch) sp[q] += pa[(int64_t)(c + q) * kd];
    const double s = ((sp[0] + sp[1]) + (sp[2] + sp[3])) + ((sp[4] + sp[5]) + (sp[6] + sp[7]));
    const int m = s_m[jl];
    const float old = as_global(P.C_old)[g];
    const float nv = m > 0 ? (float)(s / (double)m) : old;
    as_global(P.C_new)[g] = nv;
    const double df = (double)nv - (double)old;
    df2 = df * df;
  }
  s_sq[t] = df2;
  __syncthreads();
  // squared move of each cluster, coordinates in order
  if (t < nj) {
    double mv = 0.0;
    for (int c = 0; c < d; ++c) mv += s_sq[t * d + c];
    as_global(P.shift2)[j0 + t] = mv;
  }
}

// Per problem: shift = max_j sqrt(shift2_j); SSE = chunk partials, each
// thread's strided ones in order, then a fixed tree.
// sse_out: where the SSE goes (nullable); red: 256 doubles of LDS.  Returns
// the shift in thread 0.
__device__ __attribute__((always_inline)) inline double
own_shift_prob(const UpdateProb& P, double* sse_out, double* red) {
  const int t = threadIdx.x;
  if (sse_out) {
    double e = 0.0;
    for (int c = t; c < P.nchunk; c += 256) e += as_global(P.psse)[c];
    red[t] = e;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
      if (t < w) red[t] += red[t + w];
      __syncthreads();
    }
    if (t == 0) *as_global(sse_out) = red[0];
    __syncthreads();
  }
  double v = 0.0;
  for (int j = t; j < P.k; j += 256) v = __builtin_fmax(v, as_global(P.shift2)[j]);
  red[t] = v;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) red[t] = __builtin_fmax(red[t], red[t + w]);
    __syncthreads();
  }
  if (t == 0) {
    const double s = __builtin_sqrt(red[0]);
    if (P.shift_out) *P.shift_out = s;
    if (P.result) P.result->shift = s;
    return s;
  }
  return 0.0;
}

}  // namespace km
