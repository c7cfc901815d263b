// Host part of preparation: the degree-aware evidence factor and its scale
// (Section III-C, eq. 9-14) folded with eta^beta into FP32 heuristic weights,
// plus the numeric-range checks that keep every choice weight a normal FP32
// number.  This is the only place the decoder evaluates exp / log / pow; it
// runs once per instance, in FP64, with the C library, so the weights are
// reproducible bit for bit on any host.

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <vector>

#include "hac_fold.h"

namespace hac {

static double edge_length(const FoldInput& in, int32_t i, int32_t j) {
  if (in.coords) {
    const double dx = in.coords[2 * i] - in.coords[2 * j];
    const double dy = in.coords[2 * i + 1] - in.coords[2 * j + 1];
    return std::sqrt(dx * dx + dy * dy);
  }
  return in.dist[(int64_t)i * in.n + j];
}

// eta^beta; integral exponents by repeated multiplication
static double power_of_eta(double eta, double beta) {
  if (beta >= 0.0 && beta <= 64.0 && beta == std::floor(beta)) {
    double r = 1.0;
    const int times = (int)beta;
    for (int b = 0; b < times; ++b) r = r * eta;
    return r;
  }
  return std::pow(eta, beta);
}

double fold_p_x(double p_best, int32_t n) { return std::pow(p_best, 1.0 / (double)n); }

// eq. (13): tau_max / tau_min, which does not depend on the tour length
double fold_range(int32_t n, int32_t k, int32_t local_search, double p_best) {
  if (local_search) return 2.0 * (double)n;
  const double px = fold_p_x(p_best, n);
  return (((double)(k - 1) / 2.0) * px) / (1.0 - px);
}

int fold_instance(const FoldInput& in, const int32_t* cand, float* heur, FoldOutput* out) {
  const int32_t n = in.n, k = in.k;
  const int64_t nk = (int64_t)n * k;
  std::vector<double> conf(nk), evid(nk);
  std::vector<double> row_heat(n, 0.0);
  std::vector<char> row_has(n, 0);
  std::vector<double> pos;
  pos.reserve(64);

  for (int32_t i = 0; i < n; ++i) {
    // scatter heatmap row i
    for (int32_t e = in.row_ptr[i]; e < in.row_ptr[i + 1]; ++e) {
      row_heat[in.col[e]] = (double)in.val[e];
      row_has[in.col[e]] = 1;
    }
    // eq. (9): thresholded confidence on the candidate edges
    for (int32_t u = 0; u < k; ++u) {
      const int32_t j = cand[(int64_t)i * k + u];
      const double h = row_has[j] ? row_heat[j] : 0.0;
      conf[(int64_t)i * k + u] = h > in.theta_h ? h : 0.0;
    }
    // eq. (10): (d*+1)-th largest positive confidence of the row
    pos.clear();
    if (in.baseline_scope == 0) {
      for (int32_t u = 0; u < k; ++u) {
        const double c = conf[(int64_t)i * k + u];
        if (c > 0.0) pos.push_back(c);
      }
    } else {
      for (int32_t e = in.row_ptr[i]; e < in.row_ptr[i + 1]; ++e) {
        const double h = (double)in.val[e];
        if (in.col[e] != i && h > in.theta_h) pos.push_back(h);
      }
    }
    std::sort(pos.begin(), pos.end(), [](double a, double b) { return a > b; });
    const double stat = (int32_t)pos.size() > in.dstar ? pos[in.dstar] : 0.0;
    const double base = std::max(stat, in.eps);
    // eq. (11)
    for (int32_t u = 0; u < k; ++u) {
      const double c = conf[(int64_t)i * k + u];
      const double ratio = std::max(c, in.eps) / base;
      evid[(int64_t)i * k + u] = std::max(ratio, 1.0);
    }
    for (int32_t e = in.row_ptr[i]; e < in.row_ptr[i + 1]; ++e) {
      row_heat[in.col[e]] = 0.0;
      row_has[in.col[e]] = 0;
    }
  }

  if (in.evid_gt1)
    for (int64_t x = 0; x < nk; ++x) in.evid_gt1[x] = evid[x] > 1.0 ? 1 : 0;
  // eq. (12): 0.9-quantile of the positive log-margins, linear interpolation
  std::vector<double> margins;
  for (int64_t x = 0; x < nk; ++x)
    if (evid[x] > 1.0) margins.push_back(std::log(evid[x]));
  double q90 = 0.0;
  if (!margins.empty()) {
    std::sort(margins.begin(), margins.end());
    const int64_t cnt = (int64_t)margins.size();
    const double h = 0.9 * (double)(cnt - 1);
    const int64_t lo = (int64_t)std::floor(h);
    const double frac = h - (double)lo;
    q90 = lo + 1 < cnt ? margins[lo] + frac * (margins[lo + 1] - margins[lo]) : margins[lo];
  }
  // eq. (13)-(14)
  const double range = fold_range(n, k, in.local_search, in.p_best);
  const double kappa = in.kappa_fixed >= 0.0 ? in.kappa_fixed
                       : (q90 > 0.0 && range > 1.0) ? in.c_cap * in.alpha * std::log(range) / q90
                                                    : 0.0;

  // fold: S = eta^beta * exp(min(kappa log e, clip))
  float hmin = FLT_MAX, hmax = 0.0f;
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t u = 0; u < k; ++u) {
      const int64_t x = (int64_t)i * k + u;
      const double d = edge_length(in, i, cand[x]);
      if (!(d > 0.0) || !std::isfinite(d)) return FOLD_BAD_DISTANCE;
      const double eta = 1.0 / d;
      double lw = kappa * std::log(evid[x]);
      if (lw > in.clip) lw = in.clip;
      const float s = (float)(power_of_eta(eta, in.beta) * std::exp(lw));
      if (!std::isfinite(s) || s < FLT_MIN) return FOLD_RANGE;
      heur[x] = s;
      hmin = std::min(hmin, s);
      hmax = std::max(hmax, s);
    }
  }
  out->kappa = kappa;
  out->q90 = q90;
  out->r_hat = range;
  out->heur_min = hmin;
  out->heur_max = hmax;
  return FOLD_OK;
}

// The bounds a tour of length L gives (eq. 5-6); FP64, as the device does.
void fold_bounds(int32_t n, int32_t k, int32_t local_search, double rho, double p_x, double len,
                 double* tmax, double* tmin) {
  *tmax = 1.0 / (rho * len);
  if (local_search)
    *tmin = *tmax / (2.0 * (double)n);
  else
    *tmin = *tmax * (1.0 - p_x) / (((double)(k - 1) / 2.0) * p_x);
}

// Every choice weight tau * S stays a normal FP32 number for the whole
// search: tau never exceeds the tau_max of the shortest conceivable tour
// (each node leaves once: L >= sum of nearest-neighbour distances) and never
// falls below the first tau_min.
int fold_check_range(const FoldInput& in, const FoldOutput& fo, double nn_len_lower_bound,
                     double l_nn, double p_x) {
  const double lb = nn_len_lower_bound;
  if (!(lb > 0.0)) return FOLD_RANGE;
  const double top = (double)(float)(1.0 / (in.rho * lb)) * (double)fo.heur_max;
  double tmax, tmin;
  fold_bounds(in.n, in.k, in.local_search, in.rho, p_x, l_nn, &tmax, &tmin);
  const double bottom = (double)(float)tmin * (double)fo.heur_min;
  if (top >= (double)FLT_MAX / 2 || bottom < (double)FLT_MIN * 2) return FOLD_RANGE;
  return FOLD_OK;
}

}  // namespace hac
