// Host-side evidence fold (Section III-C) and numeric-range checks.
#pragma once

#include <stdint.h>

namespace hac {

enum { FOLD_OK = 0, FOLD_BAD_DISTANCE = 1, FOLD_RANGE = 2 };

struct FoldInput {
  int32_t n, k, dstar, local_search, baseline_scope;
  const double* coords;  // [n][2] or null
  const double* dist;    // [n][n] or null
  const int32_t* row_ptr;
  const int32_t* col;
  const float* val;
  double theta_h, eps, c_cap, alpha, beta, clip, p_best, rho;
  double kappa_fixed;  // >= 0 replaces eq. (14)
  uint8_t* evid_gt1;   // optional output, [n][k]: 1 where e > 1 (eq. 11)
};

struct FoldOutput {
  double kappa, q90, r_hat;
  float heur_min, heur_max;
};

double fold_p_x(double p_best, int32_t n);
double fold_range(int32_t n, int32_t k, int32_t local_search, double p_best);
// cand int32[n][k] -> heur f32[n][k]; returns FOLD_*
int fold_instance(const FoldInput& in, const int32_t* cand, float* heur, FoldOutput* out);
void fold_bounds(int32_t n, int32_t k, int32_t local_search, double rho, double p_x, double len,
                 double* tmax, double* tmin);
int fold_check_range(const FoldInput& in, const FoldOutput& fo, double nn_len_lower_bound,
                     double l_nn, double p_x);

}  // namespace hac
