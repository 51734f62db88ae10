// Device side of the Newton-Schulz stopping rule (section 3.3: the
// iteration eq. NS run to a residual tolerance, or for a fixed depth m, the
// finite-step filter p_m of eq. pm), shared by the decision kernel of the
// tiled iterations and the LDS-resident small-order iteration, so that every
// FP32 / FP64 path stops at the same step.
#pragma once
#include "common.h"
#include "launch.h"

namespace refl {

// X_m has residual r = ||X_m^2 - I||_F; s.trace already holds trace X_m.
// Records m and r in s and returns true when the iteration stops at X_m
// (then s.state and s.par are set): a non-finite residual, m reaching the
// fixed depth, r below tol, the rounding floor, or the step cap.
// The floor test is the one STAG_R (launch.h) describes.
__device__ __forceinline__ bool batch_rule(BatchStep& s, const BatchRule& ru, double r, int m,
                                           int par) {
  s.m = m;
  s.resid = r;
  if (!isfinite(r)) {
    s.state = BATCH_NONFINITE;
    return true;
  }
  bool stop = false, conv = false;
  if (ru.fixed_steps > 0) {
    if (m >= ru.fixed_steps) stop = conv = true;
  } else if (r < ru.tol) {
    stop = conv = true;
  } else if (m >= 2 && r < STAG_R && r > 0.5 * s.h2) {
    stop = true;
  } else if (m >= ru.max_iter) {
    stop = true;
  }
  s.h2 = s.h1;
  s.h1 = r;
  if (stop) {
    s.par = par;
    s.state = conv ? BATCH_CONVERGED : BATCH_STOPPED;
  }
  return stop;
}

// Index certificate (the same test as the host's index_certificate): the
// number j of negative eigenvalues of a symmetric iterate with
// b = sqrt(d) ||X^2 - I||_F < 1 is the integer with |trace - (d - 2j)| < 1;
// -1 when b >= 1 or no integer qualifies.
__device__ __forceinline__ int device_index_certificate(int d, double r, double trace) {
  const double b = sqrt((double)d) * r;
  if (!(b < 1.0)) return -1;
  const double jr = rint(((double)d - trace) / 2.0);
  return fabs(trace - ((double)d - 2.0 * jr)) < 1.0 ? (int)jr : -1;
}

// MIXED bulk rule (MixedRule in launch.h): X_m has residual r; s.trace holds
// trace X_m.  Returns true when the bulk stops at X_m.
__device__ __forceinline__ bool mixed_rule(BatchStep& s, const MixedRule& ru, double r, int m,
                                           int par) {
  s.m = m;
  s.resid = r;
  if (!isfinite(r)) {
    s.state = BATCH_NONFINITE;
    s.par = par;
    return true;
  }
  bool stop = false, conv = false;
  if (device_index_certificate(ru.d, r, s.trace) >= 0) {
    s.cert += 1;
    const bool floor = m >= 1 && r > 0.25 * s.h1;
    if (floor || s.cert > ru.extra) stop = conv = true;
  } else if (m >= 2 && r < STAG_R && r > 0.5 * s.h2) {
    stop = true;
  }
  if (!stop && m >= ru.cap) stop = true;
  s.h2 = s.h1;
  s.h1 = r;
  if (stop) {
    s.par = par;
    s.state = conv ? BATCH_CONVERGED : BATCH_STOPPED;
  }
  return stop;
}

}  // namespace refl
