/*
 * kmeans_oracle.c -- plain, slow, CPU reference for mixed-precision Lloyd
 * k-means (Carson, Chen, Liu, "Computing k-means in Mixed Precision").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the GPU library.
 *
 * What it computes, and where each definition comes from:
 *
 *   O1  assign   -- squared distance by the direct formula eq:dist-direct,
 *                   d(x,y)^2 = (x-y)^T (x-y), accumulated in FP64 over the
 *                   coordinates in index order, from the FP32 inputs
 *                   converted exactly to FP64; label = smallest index among
 *                   the minimisers (tie rule: the paper is silent); the SSE
 *                   of eq:sse as a pairwise FP64 sum over the points.
 *                   Error <= gamma_{d+2}(u_64) d^2 (Theorem thm:dist-diff).
 *   O2  update   -- centre update of eq:center: per-cluster coordinate sums
 *                   in FP64 in ascending point order, one division, one
 *                   rounding to FP32 (centres are stored in working precision,
 *                   Algorithm alg:mp-kmeans).  An empty cluster keeps its
 *                   previous centre (the paper reinitialises empty clusters
 *                   without saying how).
 *   O3  lloyd    -- Algorithm alg:kmeans / alg:mp-kmeans without the
 *                   normalisation step: t_max rounds of assign + update,
 *                   break when max_j ||c_j^t - c_j^{t-1}|| < tau, then one
 *                   final assignment.
 *   O4  mp rows  -- emulation of the quantities that decide the mixed-precision
 *                   reliability test of eq:fallback-rule-mp / Algorithm
 *                   alg:mp-dist: round-to-nearest-even quantisation to FP16 or
 *                   BF16 written from the IEEE 754 definition, the squared
 *                   distance q of the quantised vectors, S = ||x~||^2+||c~||^2,
 *                   the margin q - alpha*S, and a per-pair classification
 *                   (surely corrected / surely kept / ambiguous) together with
 *                   an a-posteriori error bound on the value a GPU evaluation
 *                   in FP32 arithmetic may return (Theorem thm:dist-exp applied
 *                   to the quantised inputs, conversion bound C(x,y) of
 *                   Section 4.3).
 *   O5  corr     -- the value a flagged pair takes under another fallback
 *                   precision u (eq:fallback-rule with the uniform precision,
 *                   eq:fallback-rule-mp with u = FP32; Section 6.1 tests
 *                   both): the direct formula with every operation rounded
 *                   once, to nearest even, in the target format (difference,
 *                   then multiply-add of the square onto the running sum, in
 *                   coordinate order), on the FP32 inputs (u = FP32) or on
 *                   the quantised inputs (uniform FP16/BF16/FP32).  Rounding
 *                   of an exact result is written from the format's
 *                   definition (spacing of the binade, ties to even); exact
 *                   results come from exact products and error-free sums in
 *                   FP64.
 *   O6  seed     -- k-means++ seeding by D^2 weighting (Arthur and
 *                   Vassilvitskii): the first centre is point floor(u_0 n);
 *                   each further centre is the first point whose running
 *                   sum of weights (point order, FP64) exceeds u_i times
 *                   their total, the weight of a point being its O1
 *                   squared distance to the nearest centre chosen so far;
 *                   if every weight is zero, point floor(u_i n).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------- */
/* Floating-point formats (Table table:float-arith-parameter)             */
/* ---------------------------------------------------------------------- */
/* fmt: 0 = binary16, 1 = bfloat16, 2 = binary32, 3 = binary64.
 * t = significand bits including the implicit bit; emin = exponent of the
 * smallest normal number; emax = exponent of the largest finite number. */
static const int FMT_T[4] = {11, 8, 24, 53};
static const int FMT_EMIN[4] = {-14, -126, -126, -1022};
static const int FMT_EMAX[4] = {15, 127, 127, 1023};

int oracle_fmt_params(int fmt, int *t, int *emin, int *emax) {
  if (fmt < 0 || fmt > 3) return -1;
  *t = FMT_T[fmt];
  *emin = FMT_EMIN[fmt];
  *emax = FMT_EMAX[fmt];
  return 0;
}

/* unit roundoff u = 2^-t for round to nearest */
double oracle_unit_roundoff(int fmt) {
  if (fmt < 0 || fmt > 3) return NAN;
  return ldexp(1.0, -FMT_T[fmt]);
}

/* largest finite number (2 - 2^(1-t)) * 2^emax */
double oracle_fmt_max(int fmt) {
  if (fmt < 0 || fmt > 3) return NAN;
  return ldexp(2.0 - ldexp(1.0, 1 - FMT_T[fmt]), FMT_EMAX[fmt]);
}

/* smallest positive normal number 2^emin */
double oracle_fmt_min_normal(int fmt) {
  if (fmt < 0 || fmt > 3) return NAN;
  return ldexp(1.0, FMT_EMIN[fmt]);
}

/* gamma_m = m u / (1 - m u), defined for m u < 1 (Section 4, after
 * eq:fpmode-vecprod); +inf otherwise. */
double oracle_gamma(double m, double u) {
  double mu = m * u;
  if (!(mu < 1.0)) return INFINITY;
  return mu / (1.0 - mu);
}

/* Round a binary32 value to the nearest value of format fmt (0: binary16,
 * 1: bfloat16), ties to even, with gradual underflow and overflow to
 * infinity, as IEEE 754 round-to-nearest-even defines it.  The result is
 * returned as a double (every such value is exactly representable).
 *
 * Method: for |x| in [2^e, 2^(e+1)) with e >= emin the spacing of the target
 * format is 2^(e+1-t); below 2^emin the spacing is the subnormal quantum
 * 2^(emin+1-t).  x / spacing is rounded to the nearest integer, ties to even
 * (exact in double, default rounding mode), and scaled back.  A result whose
 * magnitude exceeds the largest finite number overflows to infinity; that
 * happens exactly when |x| >= (2 - 2^-t) * 2^emax. */
double oracle_round_low(float xf, int fmt) {
  double x = (double)xf;
  if (fmt != 0 && fmt != 1) return NAN;
  if (isnan(x)) return x;
  if (isinf(x)) return x;
  if (x == 0.0) return x; /* keeps the sign of zero */
  int t = FMT_T[fmt], emin = FMT_EMIN[fmt];
  double ax = fabs(x);
  int e;
  frexp(ax, &e); /* ax = f * 2^e, f in [0.5, 1): ax in [2^(e-1), 2^e) */
  int expo = e - 1;
  if (expo < emin) expo = emin;
  double spacing = ldexp(1.0, expo + 1 - t);
  double r = nearbyint(ax / spacing) * spacing;
  if (r > oracle_fmt_max(fmt)) r = INFINITY;
  return x < 0 ? -r : r;
}

void oracle_quantize(const float *in, int64_t count, int fmt, double *out) {
  for (int64_t i = 0; i < count; ++i) out[i] = oracle_round_low(in[i], fmt);
}

/* ---------------------------------------------------------------------- */
/* O5: one correctly rounded operation in FP16 / BF16 / FP32               */
/* ---------------------------------------------------------------------- */

/* The exact value v = hi + lo (hi = v rounded to FP64, so |lo| is at most
 * half an FP64 ulp of hi) rounded to the nearest value of format fmt
 * (0 binary16, 1 bfloat16, 2 binary32), ties to even.  hi alone decides,
 * except when hi lies exactly halfway between two neighbours of the format:
 * then v lies on the side of lo (a midpoint has at most t+1 significant bits,
 * so it is an FP64 number, and an FP64 number other than the midpoint is at
 * least one FP64 ulp away from it, farther than |lo|). */
double oracle_round_exact(double hi, double lo, int fmt) {
  if (fmt < 0 || fmt > 2) return NAN;
  if (isnan(hi) || isinf(hi)) return hi;
  if (hi == 0.0) return hi; /* then lo is 0 too */
  int t = FMT_T[fmt], emin = FMT_EMIN[fmt];
  double ax = fabs(hi);
  double al = hi < 0 ? -lo : lo; /* lo along the direction of |hi| */
  int e;
  frexp(ax, &e);
  int expo = e - 1;
  if (expo < emin) expo = emin;
  double spacing = ldexp(1.0, expo + 1 - t);
  double qv = ax / spacing; /* exact: division by a power of two */
  double fl = floor(qv);
  double r;
  if (qv - fl == 0.5 && al != 0.0)
    r = (al > 0.0 ? fl + 1.0 : fl) * spacing;
  else
    r = nearbyint(qv) * spacing;
  if (r > oracle_fmt_max(fmt)) r = INFINITY;
  return hi < 0 ? -r : r;
}

/* a - b and a*b + c for values a, b, c of format fmt, rounded once: a*b is
 * exact in FP64 (at most 2 x 24 significant bits) and the sum is split into
 * its FP64 rounding and the exact error (Knuth's two-sum). */
static double two_sum_round(double x, double y, int fmt) {
  double s = x + y;
  double yv = s - x;
  double err = (x - (s - yv)) + (y - yv);
  return oracle_round_exact(s, err, fmt);
}
double oracle_low_sub(double a, double b, int fmt) { return two_sum_round(a, -b, fmt); }
double oracle_low_fma(double a, double b, double c, int fmt) {
  return two_sum_round(a * b, c, fmt);
}

double oracle_sqdist(const float *x, const float *y, int d);

/* The squared distance a flagged pair takes under fallback precision high
 * (0: FP64 on the FP32 inputs, O1's sum; 1: FP32 on the FP32 inputs; 2: the
 * low format fmt itself on the quantised inputs) for the low format fmt
 * (0 FP16, 1 BF16, 2 FP32). */
double oracle_corr_dist(const float *x, const float *c, int d, int high, int fmt) {
  if (high == 0) return oracle_sqdist(x, c, d);
  int f = (high == 1) ? 2 : fmt;
  double s = 0.0;
  for (int l = 0; l < d; ++l) {
    double xv = (double)x[l], cv = (double)c[l];
    if (high == 2 && fmt != 2) {
      xv = oracle_round_low(x[l], fmt);
      cv = oracle_round_low(c[l], fmt);
    }
    double t = oracle_low_sub(xv, cv, f);
    s = oracle_low_fma(t, t, s, f);
  }
  return s;
}

/* O6: indices of the k seeds; u holds k uniforms in [0, 1). */
void oracle_seed_pp(const float *X, int64_t n, int d, int k, const double *u, int64_t *idx) {
  double *w = (double *)malloc(sizeof(double) * (size_t)n);
  int64_t first = (int64_t)(u[0] * (double)n);
  idx[0] = first < n ? first : n - 1;
  for (int i = 1; i < k; ++i) {
    const float *c = X + idx[i - 1] * (int64_t)d;
    double total = 0.0;
    for (int64_t p = 0; p < n; ++p) {
      double dist = oracle_sqdist(X + p * (int64_t)d, c, d);
      w[p] = (i == 1 || dist < w[p]) ? dist : w[p];
      total += w[p];
    }
    int64_t pick = -1;
    if (total > 0.0) {
      double target = u[i] * total, run = 0.0;
      int64_t last = -1;
      for (int64_t p = 0; p < n; ++p) {
        if (w[p] > 0.0) last = p;
        run += w[p];
        if (run > target && w[p] > 0.0) {
          pick = p;
          break;
        }
      }
      if (pick < 0) pick = last;
    }
    if (pick < 0) {
      pick = (int64_t)(u[i] * (double)n);
      if (pick >= n) pick = n - 1;
    }
    idx[i] = pick;
  }
  free(w);
}

void oracle_corr_rows(const float *X, int64_t m, int d, const float *C, int k,
                      int high, int fmt, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i)
    for (int j = 0; j < k; ++j)
      out[i * (int64_t)k + j] =
          oracle_corr_dist(X + i * (int64_t)d, C + (int64_t)j * d, d, high, fmt);
}

/* ---------------------------------------------------------------------- */
/* O1: direct-formula distances, argmin, SSE                               */
/* ---------------------------------------------------------------------- */

/* eq:dist-direct in FP64, coordinates in index order. */
double oracle_sqdist(const float *x, const float *y, int d) {
  double s = 0.0;
  for (int l = 0; l < d; ++l) {
    double diff = (double)x[l] - (double)y[l];
    s += diff * diff;
  }
  return s;
}

/* Pairwise (cascade) summation of v[0..n) in FP64. */
static double pairwise_sum(const double *v, int64_t n) {
  if (n <= 8) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += v[i];
    return s;
  }
  int64_t h = n / 2;
  return pairwise_sum(v, h) + pairwise_sum(v + h, n - h);
}

double oracle_pairwise_sum(const double *v, int64_t n) { return pairwise_sum(v, n); }

/* D[i*k + j] = d(x_i, c_j)^2 for the m rows of X. */
void oracle_dist_rows(const float *X, int64_t m, int d, const float *C, int k,
                      double *D) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i)
    for (int j = 0; j < k; ++j)
      D[i * (int64_t)k + j] = oracle_sqdist(X + i * (int64_t)d, C + (int64_t)j * d, d);
}

/* For each point: label = smallest index attaining min_j d_ij, mind = that
 * distance (FP64).  sse (nullable) receives the pairwise sum of mind. */
void oracle_assign(const float *X, int64_t n, int d, const float *C, int k,
                   int32_t *labels, double *mind, double *sse) {
  double *md = mind;
  if (md == NULL) md = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const float *x = X + i * (int64_t)d;
    int best = 0;
    double bd = oracle_sqdist(x, C, d);
    for (int j = 1; j < k; ++j) {
      double v = oracle_sqdist(x, C + (int64_t)j * d, d);
      if (v < bd) { /* strict: the first minimiser is kept */
        bd = v;
        best = j;
      }
    }
    labels[i] = best;
    md[i] = bd;
  }
  if (sse) *sse = pairwise_sum(md, n);
  if (mind == NULL) free(md);
}

/* eq:sse for a given assignment: the pairwise sum over i of the FP64 direct
 * distance d(x_i, c_{labels_i}) (the same terms and order as O1's SSE when
 * the labels are O1's).  Returns -1 on a label out of range. */
double oracle_sse_labels(const float *X, int64_t n, int d, const int32_t *labels,
                         const float *C, int k) {
  double *t = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  for (int64_t i = 0; i < n; ++i) {
    if (labels[i] < 0 || labels[i] >= k) {
      free(t);
      return -1.0;
    }
    t[i] = oracle_sqdist(X + i * (int64_t)d, C + (int64_t)labels[i] * d, d);
  }
  double s = pairwise_sum(t, n);
  free(t);
  return s;
}

/* ---------------------------------------------------------------------- */
/* O2: centre update                                                       */
/* ---------------------------------------------------------------------- */

/* C_new[j] = fl32( (sum_{i: label_i = j} x_i) / m_j ), sums in FP64 in
 * ascending i; m_j = 0 keeps C_old[j].  counts (nullable) receives m_j.
 * shift (nullable) receives max_j ||C_new[j] - C_old[j]|| (FP64).
 * Returns the number of empty clusters, or -1 on a label out of range. */
int64_t oracle_update(const float *X, int64_t n, int d, const int32_t *labels,
                      int k, const float *C_old, float *C_new, int64_t *counts,
                      double *shift) {
  double *s = (double *)calloc((size_t)k * (size_t)d, sizeof(double));
  int64_t *m = (int64_t *)calloc((size_t)k, sizeof(int64_t));
  if (!s || !m) {
    free(s);
    free(m);
    return -2;
  }
  for (int64_t i = 0; i < n; ++i) {
    int j = labels[i];
    if (j < 0 || j >= k) {
      free(s);
      free(m);
      return -1;
    }
    const float *x = X + i * (int64_t)d;
    double *sj = s + (int64_t)j * d;
    for (int l = 0; l < d; ++l) sj[l] += (double)x[l];
    m[j] += 1;
  }
  int64_t empty = 0;
  double maxshift = 0.0;
  for (int j = 0; j < k; ++j) {
    double mv2 = 0.0;
    for (int l = 0; l < d; ++l) {
      float nv;
      if (m[j] > 0)
        nv = (float)(s[(int64_t)j * d + l] / (double)m[j]);
      else
        nv = C_old[(int64_t)j * d + l];
      double diff = (double)nv - (double)C_old[(int64_t)j * d + l];
      mv2 += diff * diff;
      C_new[(int64_t)j * d + l] = nv;
    }
    if (m[j] == 0) empty += 1;
    double mv = sqrt(mv2);
    if (mv > maxshift) maxshift = mv;
    if (counts) counts[j] = m[j];
  }
  if (shift) *shift = maxshift;
  free(s);
  free(m);
  return empty;
}

/* ---------------------------------------------------------------------- */
/* O3: Lloyd's algorithm                                                   */
/* ---------------------------------------------------------------------- */

/* C (k x d) holds the initial centres on entry and the final ones on exit.
 * sse_hist (nullable, max_iter+1 entries): SSE of each assignment, the last
 * filled entry being the final assignment.  shift_hist (nullable, max_iter).
 * labels/mind receive the final assignment.  Returns the number of update
 * rounds performed (<= max_iter), or a negative value on error. */
int oracle_lloyd(const float *X, int64_t n, int d, int k, float *C, int max_iter,
                 double tol, int32_t *labels, double *mind, double *sse_hist,
                 double *shift_hist) {
  float *Cn = (float *)malloc(sizeof(float) * (size_t)k * (size_t)d);
  if (!Cn) return -2;
  int t;
  for (t = 0; t < max_iter; ++t) {
    double sse = 0.0, shift = 0.0;
    oracle_assign(X, n, d, C, k, labels, mind, &sse);
    if (sse_hist) sse_hist[t] = sse;
    if (oracle_update(X, n, d, labels, k, C, Cn, NULL, &shift) < 0) {
      free(Cn);
      return -1;
    }
    memcpy(C, Cn, sizeof(float) * (size_t)k * (size_t)d);
    if (shift_hist) shift_hist[t] = shift;
    if (shift < tol) { /* strict, as in the stopping test of alg:kmeans */
      t += 1;
      break;
    }
  }
  double sse = 0.0;
  oracle_assign(X, n, d, C, k, labels, mind, &sse);
  if (sse_hist) sse_hist[t] = sse;
  free(Cn);
  return t;
}

/* ---------------------------------------------------------------------- */
/* O4: mixed-precision reliability test, emulated                           */
/* ---------------------------------------------------------------------- */

/*
 * For the m rows of X against all k centres, with x~ = RNE_fmt(x), c~ = RNE_fmt(c)
 * (fmt 0 = FP16, 1 = BF16):
 *
 *   dist[i,j] = d(x_i, c_j)^2 from the original data (O1)
 *   q[i,j]    = d(x~_i, c~_j)^2 in FP64 (the quantised distance)
 *   S[i,j]    = ||x~_i||^2 + ||c~_j||^2
 *   P[i,j]    = |x~_i|^T |c~_j|
 *
 * The reliability test of eq:quantis-reliability-test keeps the low-precision
 * value iff  d^ > alpha * S  (alpha = rho~ * 2 gamma^l_{d+2} in the equation
 * form, rho~ gamma^l_{d+2} in the listing form -- the caller passes the value
 * the GPU uses).  A GPU evaluates d^ with inputs x~, c~ in FP32 arithmetic, so
 * by Theorem thm:dist-exp (with the FP32 unit roundoff doubled to cover any
 * rounding mode of the accumulator)
 *
 *   |d^ - q| <= A := gamma'_{d+4} (S + 2P),   gamma' = gamma(., 2 u_32),
 *
 * and the FP32 evaluation of alpha*S is off by at most alpha*A.  Hence
 *
 *   cls = -1 (surely corrected) if q - alpha S < -band,
 *   cls = +1 (surely kept)      if q - alpha S > +band,
 *   cls =  0 (ambiguous)        otherwise,          band := (1 + alpha) A.
 *
 * B[i,j] bounds |D - dist| for the value D the GPU reports for the pair:
 *   kept:      |q - dist| + A + gamma_{d+2}(u_64) dist
 *   corrected: 2 u_32 dist   (FP64 direct formula rounded once to FP32,
 *                             eq:fallback-rule-mp and alg:mp-dist)
 *   ambiguous: the larger of the two.
 * alpha < 0 means "never correct" (uniform low precision, no fallback).
 *
 * Every output pointer except dist is nullable.  Returns the number of pairs
 * whose inputs overflow the low format (those get cls = -2, B = inf).
 */
/* Quantised centres of O4: C~ (k x d, as doubles), ||c~_j||^2 and an
 * overflow flag per centre.  Returns 0, or -1 when out of memory. */
typedef struct {
  double *Ct;
  double *nc;
  int *bad;
} mp_centres;

static int mp_centres_make(const float *C, int k, int d, int fmt, mp_centres *mc) {
  mc->Ct = (double *)malloc(sizeof(double) * (size_t)k * (size_t)d);
  mc->nc = (double *)malloc(sizeof(double) * (size_t)k);
  mc->bad = (int *)calloc((size_t)k, sizeof(int));
  if (!mc->Ct || !mc->nc || !mc->bad) {
    free(mc->Ct);
    free(mc->nc);
    free(mc->bad);
    return -1;
  }
  for (int j = 0; j < k; ++j) {
    double s = 0.0;
    for (int l = 0; l < d; ++l) {
      double v = oracle_round_low(C[(int64_t)j * d + l], fmt);
      if (isinf(v) || isnan(v)) mc->bad[j] = 1;
      mc->Ct[(int64_t)j * d + l] = v;
      s += v * v;
    }
    mc->nc[j] = s;
  }
  return 0;
}

static void mp_centres_free(mp_centres *mc) {
  free(mc->Ct);
  free(mc->nc);
  free(mc->bad);
}

/* O4 quantities of one pair (x, c_j): dist, q, S, A, class and bound B as
 * described above.  xt is x~ (doubles), nx = ||x~||^2, xbad = x~ overflows. */
typedef struct {
  double dist, q, S, A, B;
  int8_t cls;
} mp_pair;

static mp_pair mp_pair_eval(const float *x, const double *xt, double nx, int xbad,
                            const float *c, const mp_centres *mc, int j, int d,
                            double alpha, double gp, double g64, double u32) {
  mp_pair r;
  const double *ct = mc->Ct + (int64_t)j * d;
  r.dist = oracle_sqdist(x, c, d);
  double q = 0.0, P = 0.0;
  for (int l = 0; l < d; ++l) {
    double diff = xt[l] - ct[l];
    q += diff * diff;
    P += fabs(xt[l]) * fabs(ct[l]);
  }
  r.q = q;
  r.S = nx + mc->nc[j];
  r.A = gp * (r.S + 2.0 * P);
  double Bk = fabs(q - r.dist) + r.A + g64 * r.dist;
  double Bc = 2.0 * u32 * r.dist;
  if (xbad || mc->bad[j]) {
    r.cls = -2;
    r.B = INFINITY;
  } else if (alpha < 0.0) {
    r.cls = 1;
    r.B = Bk;
  } else {
    double margin = q - alpha * r.S;
    double band = (1.0 + alpha) * r.A;
    if (margin < -band) {
      r.cls = -1;
      r.B = Bc;
    } else if (margin > band) {
      r.cls = 1;
      r.B = Bk;
    } else {
      r.cls = 0;
      r.B = Bk > Bc ? Bk : Bc;
    }
  }
  return r;
}

/* x~ = RNE_fmt(x) into xt; returns ||x~||^2 and sets *bad on overflow. */
static double mp_round_row(const float *x, int d, int fmt, double *xt, int *bad) {
  double nx = 0.0;
  *bad = 0;
  for (int l = 0; l < d; ++l) {
    xt[l] = oracle_round_low(x[l], fmt);
    if (isinf(xt[l]) || isnan(xt[l])) *bad = 1;
    nx += xt[l] * xt[l];
  }
  return nx;
}

int64_t oracle_mp_rows(const float *X, int64_t m, int d, const float *C, int k,
                       int fmt, double alpha, double *dist, double *q_out,
                       double *S_out, double *A_out, double *B_out,
                       int8_t *cls_out) {
  double u32 = oracle_unit_roundoff(2), u64 = oracle_unit_roundoff(3);
  double gp = oracle_gamma((double)(d + 4), 2.0 * u32);
  double g64 = oracle_gamma((double)(d + 2), u64);
  mp_centres mc;
  if (mp_centres_make(C, k, d, fmt, &mc) != 0) return -1;
  int64_t nbad = 0;
#pragma omp parallel for schedule(static) reduction(+ : nbad)
  for (int64_t i = 0; i < m; ++i) {
    const float *x = X + i * (int64_t)d;
    double *xt = (double *)malloc(sizeof(double) * (size_t)d);
    int xbad;
    double nx = mp_round_row(x, d, fmt, xt, &xbad);
    for (int j = 0; j < k; ++j) {
      int64_t o = i * (int64_t)k + j;
      mp_pair r = mp_pair_eval(x, xt, nx, xbad, C + (int64_t)j * d, &mc, j, d,
                               alpha, gp, g64, u32);
      if (r.cls == -2) nbad += 1;
      dist[o] = r.dist;
      if (q_out) q_out[o] = r.q;
      if (S_out) S_out[o] = r.S;
      if (A_out) A_out[o] = r.A;
      if (B_out) B_out[o] = r.B;
      if (cls_out) cls_out[o] = r.cls;
    }
    free(xt);
  }
  mp_centres_free(&mc);
  return nbad;
}

/* The per-row quantities of the parity contract without materialising the
 * m x k pairs (same pair arithmetic as oracle_mp_rows).  For every row i:
 *   j1[i]   = smallest index attaining min_j dist_ij (O1's label)
 *   dj1[i]  = dist_{i j1},  Bj1[i] = B_{i j1}
 *   lo[i]   = min_{j != j1} (dist_ij - B_ij)   (+inf when k = 1)
 *   d2[i]   = min_{j != j1} dist_ij            (+inf when k = 1)
 * and for each of the nlab given label arrays (labs[t*m + i], t < nlab):
 *   dlab[t*m + i] = dist_{i, lab},  Blab[t*m + i] = B_{i, lab}
 * (labels outside [0,k) give NaN).  The label gate of row i is
 * lo[i] > dj1[i] + Bj1[i].  counts[0..3] receive the class counts over all
 * pairs (surely corrected, ambiguous, surely kept, overflow).
 * fmt = 3 (no low precision: every pair is the FP64 direct value compared in
 * FP64) uses B = 2 gamma_{d+2}(u_64) dist and counts every pair as corrected.
 * Returns 0, or -1 when out of memory. */
int oracle_mp_scan(const float *X, int64_t m, int d, const float *C, int k,
                   int fmt, double alpha, int nlab, const int32_t *labs,
                   int32_t *j1_out, double *dj1_out, double *Bj1_out,
                   double *lo_out, double *d2_out, double *dlab, double *Blab,
                   int64_t *counts) {
  double u32 = oracle_unit_roundoff(2), u64 = oracle_unit_roundoff(3);
  double gp = oracle_gamma((double)(d + 4), 2.0 * u32);
  double g64 = oracle_gamma((double)(d + 2), u64);
  mp_centres mc = {NULL, NULL, NULL};
  if (fmt != 3 && mp_centres_make(C, k, d, fmt, &mc) != 0) return -1;
  int64_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
  int fail = 0;
#pragma omp parallel reduction(+ : c0, c1, c2, c3) reduction(| : fail)
  {
    double *xt = (double *)malloc(sizeof(double) * (size_t)d);
    double *dist = (double *)malloc(sizeof(double) * (size_t)k);
    double *B = (double *)malloc(sizeof(double) * (size_t)k);
    if (!xt || !dist || !B) fail = 1;
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < m; ++i) {
      if (fail) continue;
      const float *x = X + i * (int64_t)d;
      if (fmt == 3) {
        for (int j = 0; j < k; ++j) {
          dist[j] = oracle_sqdist(x, C + (int64_t)j * d, d);
          B[j] = 2.0 * g64 * dist[j];
        }
        c0 += k;
      } else {
        int xbad;
        double nx = mp_round_row(x, d, fmt, xt, &xbad);
        for (int j = 0; j < k; ++j) {
          mp_pair r = mp_pair_eval(x, xt, nx, xbad, C + (int64_t)j * d, &mc, j, d,
                                   alpha, gp, g64, u32);
          dist[j] = r.dist;
          B[j] = r.B;
          if (r.cls == -1) c0++;
          else if (r.cls == 0) c1++;
          else if (r.cls == 1) c2++;
          else c3++;
        }
      }
      int best = 0;
      for (int j = 1; j < k; ++j)
        if (dist[j] < dist[best]) best = j;
      double lo = INFINITY, d2 = INFINITY;
      for (int j = 0; j < k; ++j) {
        if (j == best) continue;
        if (dist[j] - B[j] < lo) lo = dist[j] - B[j];
        if (dist[j] < d2) d2 = dist[j];
      }
      j1_out[i] = best;
      d2_out[i] = d2;
      dj1_out[i] = dist[best];
      Bj1_out[i] = B[best];
      lo_out[i] = lo;
      for (int t = 0; t < nlab; ++t) {
        int32_t lab = labs[(int64_t)t * m + i];
        dlab[(int64_t)t * m + i] = (lab >= 0 && lab < k) ? dist[lab] : NAN;
        Blab[(int64_t)t * m + i] = (lab >= 0 && lab < k) ? B[lab] : NAN;
      }
    }
    free(xt);
    free(dist);
    free(B);
  }
  if (fmt != 3) mp_centres_free(&mc);
  counts[0] = c0;
  counts[1] = c1;
  counts[2] = c2;
  counts[3] = c3;
  return fail ? -1 : 0;
}

/* Counts of the O4 classes over all pairs, without materialising them:
 * counts[0] = surely corrected, counts[1] = ambiguous, counts[2] = surely kept,
 * counts[3] = pairs whose inputs overflow the low format. */
void oracle_mp_count(const float *X, int64_t m, int d, const float *C, int k,
                     int fmt, double alpha, int64_t *counts) {
  const int64_t rows = 64;
  int64_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
  double *dist = (double *)malloc(sizeof(double) * (size_t)rows * (size_t)k);
  int8_t *cls = (int8_t *)malloc((size_t)rows * (size_t)k);
  for (int64_t s = 0; s < m; s += rows) {
    int64_t e = s + rows < m ? s + rows : m;
    oracle_mp_rows(X + s * (int64_t)d, e - s, d, C, k, fmt, alpha, dist, NULL,
                   NULL, NULL, NULL, cls);
    for (int64_t o = 0; o < (e - s) * (int64_t)k; ++o) {
      if (cls[o] == -1) c0++;
      else if (cls[o] == 0) c1++;
      else if (cls[o] == 1) c2++;
      else c3++;
    }
  }
  free(dist);
  free(cls);
  counts[0] = c0;
  counts[1] = c1;
  counts[2] = c2;
  counts[3] = c3;
}

/* Number of threads the OpenMP runtime will use (1 without OpenMP). */
int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_num_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}
