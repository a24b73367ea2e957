// Host part of SP2-ACC: the polynomial schedule of Alg. 3 (Kruchinina,
// Rudberg, Rubensson 2015, sec. 4), computed once per instance from bounds
// of its homo and lumo eigenvalues before a run. The device applies it step
// by step (Alg. 4) through the finalize kernel and the square epilogues.
#include <math.h>
#include <float.h>

#include "../../include/sp2.h"
#include "sp2_device.h"

namespace sp2 {

// The schedule's decisions compare bounds that may tie exactly (the proof
// of Theorem 2 starts from such a tie); keep every product and sum rounded
// on its own, as written, so that the comparisons do not depend on whether
// the compiler fuses them.
#pragma clang fp contract(off)

int acc_schedule(double lmin, double lmax, double homo_out, double homo_in,
                 double lumo_in, double lumo_out, bool accelerate, int cap,
                 int* n_min_out, int* n_max_out, int8_t* p_out,
                 double* alpha_out) {
  const double vals[6] = {lmin, lmax, homo_out, homo_in, lumo_in, lumo_out};
  for (double v : vals)
    if (!isfinite(v)) return -1;
  // Bounds in order, intervals disjoint, nonzero upper distances (Theorem 2
  // assumes them; with a zero one the schedule never alternates).
  if (!(lmin <= homo_out && homo_out <= homo_in && homo_in < lumo_in &&
        lumo_in <= lumo_out && lumo_out <= lmax && homo_in > lmin &&
        lumo_in < lmax))
    return -1;
  const double width = lmax - lmin;
  // Distances in the spectrum of X_0 = (lmax I - F) / width: beta of the homo
  // image from 1, gamma of the lumo image from 0; 'hi' from the inner
  // bounds (upper estimates), 'lo' from the outer ones (lower estimates).
  double beta_hi = 1.0 - (lmax - homo_in) / width;
  double beta_lo = 1.0 - (lmax - homo_out) / width;
  double gamma_hi = (lmax - lumo_in) / width;
  double gamma_lo = (lmax - lumo_out) / width;
  if (!accelerate) beta_lo = gamma_lo = 0.0;   // alpha_i = 1 throughout
  const double eps = DBL_EPSILON;   // FP64 machine epsilon
  double delta = 0.01;              // switch-off threshold of the stretch
  int n_min = -1;
  int i = 0;
  int p_prev2 = -1, p_prev = -1;    // p_{i-1}, p_i (undefined before step 1)
  for (;;) {
    const bool converged = !(beta_hi - beta_hi * beta_hi > eps) &&
                           !(gamma_hi - gamma_hi * gamma_hi > eps);
    // Continue until converged and the last two steps alternate; before
    // step 2 there is no pair to compare and the loop goes on.
    const bool alternated = (i >= 2) && (p_prev != p_prev2);
    if (converged && alternated) break;
    ++i;
    if (i > kMaxIter || i > cap) return -2;
    if (beta_lo < delta && gamma_lo < delta) {
      beta_lo = 0.0;
      gamma_lo = 0.0;
      n_min = i + 1;
      delta = 0.0;
    }
    int p;
    double a;
    if (gamma_hi >= beta_hi) {
      // fold the unoccupied side towards 0 with ((1 - a) + a x)^2
      p = 1;
      a = 2.0 / (2.0 - gamma_lo);
      const double gl = (1.0 - a) + a * gamma_lo;
      const double gh = (1.0 - a) + a * gamma_hi;
      gamma_lo = gl * gl;
      gamma_hi = gh * gh;
      // the occupied side's distance from 1 under the same polynomial
      const double bl = a * beta_lo, bh = a * beta_hi;
      beta_lo = 2.0 * bl - bl * bl;
      beta_hi = 2.0 * bh - bh * bh;
    } else {
      // fold the occupied side towards 1 with 2 a x - (a x)^2
      p = 0;
      a = 2.0 / (2.0 - beta_lo);
      const double gl = a * gamma_lo, gh = a * gamma_hi;
      gamma_lo = 2.0 * gl - gl * gl;
      gamma_hi = 2.0 * gh - gh * gh;
      const double bl = (1.0 - a) + a * beta_lo;
      const double bh = (1.0 - a) + a * beta_hi;
      beta_lo = bl * bl;
      beta_hi = bh * bh;
    }
    if (p_out) p_out[i - 1] = static_cast<int8_t>(p);
    if (alpha_out) alpha_out[i - 1] = a;
    p_prev2 = p_prev;
    p_prev = p;
  }
  if (n_min < 0 || n_min > i) n_min = i;
  *n_min_out = n_min;
  *n_max_out = i;
  return 0;
}

}  // namespace sp2

extern "C" sp2_status sp2_acc_schedule(double lambda_min, double lambda_max,
                                       double homo_out, double homo_in,
                                       double lumo_in, double lumo_out,
                                       int32_t accelerate, int32_t cap,
                                       int32_t* n_min, int32_t* n_max,
                                       int8_t* p, double* alpha) {
  if (!n_min || !n_max || cap < 0) return SP2_INVALID_ARG;
  int lo = 0, hi = 0;
  // With no output arrays only the lengths are asked for.
  const int room = (p || alpha) ? cap : sp2::kMaxIter;
  const int rc = sp2::acc_schedule(lambda_min, lambda_max, homo_out, homo_in,
                                   lumo_in, lumo_out, accelerate != 0, room,
                                   &lo, &hi, p, alpha);
  if (rc != 0) return SP2_INVALID_ARG;
  *n_min = lo;
  *n_max = hi;
  return SP2_OK;
}
