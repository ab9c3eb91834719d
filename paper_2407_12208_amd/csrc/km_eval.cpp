// km_eval.cpp -- clustering agreement measures the paper reports (host code):
// the adjusted Rand index and adjusted mutual information of two labelings
// (Section 6.2 evaluates Lloyd's algorithm with SSE, ARI and AMI, after Vinh,
// Epps and Bailey), and the segmentation Diff of Section 6.3: the fraction
// of points whose labels differ after the one-to-one matching of cluster ids
// that agrees on the most points.
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <unordered_map>
#include <vector>

#include "../../include/kmeans.h"

namespace {

// Contingency table of two labelings: dense ids per labeling (first-seen
// order) and the nonzero cells.
struct Table {
  int ra = 0, rb = 0;
  std::vector<int64_t> a, b;                 // row and column sums
  std::vector<std::pair<int64_t, int64_t>> cells;  // (row * rb + col, count)
  int64_t n = 0;
};

Table contingency(const int32_t* x, const int32_t* y, int64_t n) {
  Table t;
  t.n = n;
  std::unordered_map<int32_t, int> ix, iy;
  std::vector<int> dx(n), dy(n);
  for (int64_t i = 0; i < n; ++i) {
    auto fx = ix.emplace(x[i], (int)ix.size());
    auto fy = iy.emplace(y[i], (int)iy.size());
    dx[i] = fx.first->second;
    dy[i] = fy.first->second;
  }
  t.ra = (int)ix.size();
  t.rb = (int)iy.size();
  t.a.assign(t.ra, 0);
  t.b.assign(t.rb, 0);
  std::unordered_map<int64_t, int64_t> cell;
  for (int64_t i = 0; i < n; ++i) {
    t.a[dx[i]] += 1;
    t.b[dy[i]] += 1;
    cell[(int64_t)dx[i] * t.rb + dy[i]] += 1;
  }
  t.cells.assign(cell.begin(), cell.end());
  std::sort(t.cells.begin(), t.cells.end());
  return t;
}

double comb2(int64_t m) { return 0.5 * (double)m * (double)(m - 1); }

}  // namespace

extern "C" {

int32_t kmeans_ari(const int32_t* labels_a, const int32_t* labels_b, int64_t n, double* ari) {
  if (!labels_a || !labels_b || !ari || n < 1) return KM_ERR_ARG;
  const Table t = contingency(labels_a, labels_b, n);
  // one cluster each, or one point per cluster each: identical partitions
  if ((t.ra == 1 && t.rb == 1) || (t.ra == n && t.rb == n)) {
    *ari = 1.0;
    return KM_OK;
  }
  double idx = 0.0, sa = 0.0, sb = 0.0;
  for (auto& c : t.cells) idx += comb2(c.second);
  for (int64_t v : t.a) sa += comb2(v);
  for (int64_t v : t.b) sb += comb2(v);
  const double expected = sa * sb / comb2(n);
  const double mx = 0.5 * (sa + sb);
  *ari = (mx - expected) == 0.0 ? 1.0 : (idx - expected) / (mx - expected);
  return KM_OK;
}

int32_t kmeans_ami(const int32_t* labels_a, const int32_t* labels_b, int64_t n, double* ami) {
  if (!labels_a || !labels_b || !ami || n < 1) return KM_ERR_ARG;
  const Table t = contingency(labels_a, labels_b, n);
  if ((t.ra == 1 && t.rb == 1) || (t.ra == n && t.rb == n)) {
    *ami = 1.0;
    return KM_OK;
  }
  const double N = (double)n;
  // mutual information and entropies (natural logarithm)
  double mi = 0.0;
  for (auto& c : t.cells) {
    const int64_t r = c.first / t.rb, s = c.first % t.rb;
    const double nij = (double)c.second;
    mi += nij / N * std::log(N * nij / ((double)t.a[r] * (double)t.b[s]));
  }
  auto entropy = [&](const std::vector<int64_t>& v) {
    double h = 0.0;
    for (int64_t m : v)
      if (m > 0) h -= (double)m / N * std::log((double)m / N);
    return h;
  };
  const double ha = entropy(t.a), hb = entropy(t.b);
  // expected mutual information under the permutation model (hypergeometric
  // cell counts with the margins fixed)
  std::vector<double> lf((size_t)n + 1, 0.0);  // log factorials
  for (int64_t m = 1; m <= n; ++m) lf[m] = lf[m - 1] + std::log((double)m);
  double emi = 0.0;
  for (int64_t ai : t.a)
    for (int64_t bj : t.b) {
      const int64_t lo = std::max<int64_t>(1, ai + bj - n), hi = std::min(ai, bj);
      for (int64_t nij = lo; nij <= hi; ++nij) {
        const double term = (double)nij / N * std::log(N * (double)nij / ((double)ai * (double)bj));
        const double lp = lf[ai] + lf[bj] + lf[n - ai] + lf[n - bj] - lf[n] - lf[nij] - lf[ai - nij] -
                          lf[bj - nij] - lf[n - ai - bj + nij];
        emi += term * std::exp(lp);
      }
    }
  const double norm = 0.5 * (ha + hb);  // arithmetic mean of the entropies
  double den = norm - emi;
  const double eps = std::numeric_limits<double>::epsilon();
  den = den < 0.0 ? std::min(den, -eps) : std::max(den, eps);
  *ami = (mi - emi) / den;
  return KM_OK;
}

// Largest agreement of two labelings under a one-to-one matching of their
// ids (Hungarian method on the contingency table, shortest augmenting
// paths with potentials); *diff = 1 - agreement / n.
int32_t kmeans_label_diff(const int32_t* labels_a, const int32_t* labels_b, int64_t n, double* diff) {
  if (!labels_a || !labels_b || !diff || n < 1) return KM_ERR_ARG;
  const Table t = contingency(labels_a, labels_b, n);
  const int K = std::max(t.ra, t.rb);
  if (K > 4096) return KM_ERR_UNSUPPORTED;
  // cost[i][j] = -count (square, padded with zeros)
  std::vector<double> cost((size_t)K * K, 0.0);
  for (auto& c : t.cells) {
    const int64_t r = c.first / t.rb, s = c.first % t.rb;
    cost[(size_t)r * K + s] = -(double)c.second;
  }
  const double INF = std::numeric_limits<double>::infinity();
  std::vector<double> u(K + 1, 0.0), v(K + 1, 0.0), minv(K + 1);
  std::vector<int> p(K + 1, 0), way(K + 1, 0);
  std::vector<char> used(K + 1);
  for (int i = 1; i <= K; ++i) {
    p[0] = i;
    int j0 = 0;
    std::fill(minv.begin(), minv.end(), INF);
    std::fill(used.begin(), used.end(), 0);
    do {
      used[j0] = 1;
      const int i0 = p[j0];
      double delta = INF;
      int j1 = 0;
      for (int j = 1; j <= K; ++j)
        if (!used[j]) {
          const double cur = cost[(size_t)(i0 - 1) * K + (j - 1)] - u[i0] - v[j];
          if (cur < minv[j]) {
            minv[j] = cur;
            way[j] = j0;
          }
          if (minv[j] < delta) {
            delta = minv[j];
            j1 = j;
          }
        }
      for (int j = 0; j <= K; ++j)
        if (used[j]) {
          u[p[j]] += delta;
          v[j] -= delta;
        } else {
          minv[j] -= delta;
        }
      j0 = j1;
    } while (p[j0] != 0);
    do {
      const int j1 = way[j0];
      p[j0] = p[j1];
      j0 = j1;
    } while (j0);
  }
  double agree = 0.0;
  for (int j = 1; j <= K; ++j)
    if (p[j] > 0) agree -= cost[(size_t)(p[j] - 1) * K + (j - 1)];
  *diff = 1.0 - agree / (double)n;
  return KM_OK;
}

}  // extern "C"
