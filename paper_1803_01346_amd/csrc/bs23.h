// Bogacki-Shampine 3(2) step controller (the method of Matlab's ode23, which
// the paper uses with relative tolerance 2e-4; Sec. 2, discretisation
// paragraph), written once over an abstract set of vector operations so the
// device integrator and the host test integrator run the same control logic.
//
//   k1 = f(t, y)  (first same as last)     k2 = f(t + dt/2, y + dt/2 k1)
//   k3 = f(t + 3dt/4, y + 3dt/4 k2)        y1 = y + dt (2/9 k1 + 1/3 k2 + 4/9 k3)
//   k4 = f(t + dt, y1)                     E  = dt (-5/72 k1 + 1/12 k2 + 1/9 k3 - 1/8 k4)
//   err = max_i |E_i| / max(|y_i|, |y1_i|, atol/rtol),  accept iff err <= rtol
//   accepted: dt *= min(5, max(0.2, 0.8 (rtol/err)^(1/3))), no growth right
//             after a rejection;  rejected: dt *= max(0.2, 0.8 (rtol/err)^(1/3)),
//             at most 1/2 on a repeated rejection
//   steps end exactly on breakpoints and t1; after a breakpoint k1 is
//   recomputed (the applied-field rate may jump there)
//
// Ops provides (buffers are named by the enum below; Y is the state):
//   int  rhs(double t, Buf src, Buf dst)          dst = f(t, src); < 0 = error
//                                                 (src is a state: Y or Y1)
//   int  rhs_at(double t, Buf y, Buf k, double c, Buf dst)   dst = f(t, y + c k),
//                                                 may use Y1 as scratch
//   int  combo(Buf out, Buf y, Buf a, double ca, Buf b, double cb, Buf c, double cc)
//   int  errnorm(Buf y, Buf y1, double dt, double thr, double* err)   uses K1..K4
//   int  rate(double thr, double* r)              max_i |K1_i| / max(|Y_i|, thr)
//   int  accept()                                 Y = Y1, K1 <-> K4 (may swap buffers)
//   int  observe(double t, int* stop)
#pragma once

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/scfft.h"

namespace scfft {

enum Buf : int { B_Y = 0, B_K1, B_K2, B_K3, B_K4, B_Y1, B_NONE = -1 };

// Continuation of the adaptive controller between calls.  In: if `use`, the
// run starts from it (k1 already in K1 when has_k1, step size dt, whether
// the last step was rejected) instead of computing k1 and a first step.
// Out: where the run stopped (its observer, t1 or max_steps) and what the
// next step would have started with; valid = false after a failure and in
// fixed-step mode.
struct Bs23Cont {
  bool use = false;
  bool valid = false;
  double t = 0.0;
  double dt = 0.0;
  bool rejected_last = false;
  bool has_k1 = false;
};

template <class Ops>
scfft_status bs23_run(Ops& ops, double t0, double t1, const scfft_ode_opts& o,
                      const std::vector<double>& extra_stops, scfft_ode_stats& st,
                      Bs23Cont* cont = nullptr) {
  const bool resume = cont && cont->use;
  if (cont) cont->valid = false;
  const double rtol = o.rtol, atol = o.atol;
  const double thr = atol / rtol;
  const int64_t max_steps = o.max_steps > 0 ? o.max_steps : 10000000;
  const double dt_max = o.dt_max_s > 0.0 ? o.dt_max_s : INFINITY;
  st.t_s = t0;
  int rc;

  auto step = [&](double t, double dt, double* err) -> int {
    int r;
    if ((r = ops.rhs_at(t + 0.5 * dt, B_Y, B_K1, 0.5 * dt, B_K2)) < 0) return r;
    if ((r = ops.rhs_at(t + 0.75 * dt, B_Y, B_K2, 0.75 * dt, B_K3)) < 0) return r;
    if ((r = ops.combo(B_Y1, B_Y, B_K1, dt * (2.0 / 9.0), B_K2, dt * (1.0 / 3.0), B_K3,
                       dt * (4.0 / 9.0))) < 0)
      return r;
    if ((r = ops.rhs(t + dt, B_Y1, B_K4)) < 0) return r;
    st.rhs_calls += 3;
    return ops.errnorm(B_Y, B_Y1, dt, thr, err);
  };

  if (!(t1 > t0)) return SCFFT_ERR_ARG;

  if (o.fixed_steps > 0) {
    const double dt = (t1 - t0) / o.fixed_steps;
    double t = t0;
    if ((rc = ops.rhs(t, B_Y, B_K1)) < 0) return (scfft_status)rc;
    st.rhs_calls += 1;
    for (int s = 0; s < o.fixed_steps; ++s) {
      const double tn = s + 1 < o.fixed_steps ? t0 + (s + 1) * dt : t1;
      double err = 0.0;
      if ((rc = step(t, tn - t, &err)) < 0) return (scfft_status)rc;
      if (!std::isfinite(err)) return SCFFT_ERR_NAN;
      st.dt_last_s = tn - t;
      st.err_last = err;
      if ((rc = ops.accept()) < 0) return (scfft_status)rc;
      t = tn;
      st.t_s = t;
      st.accepted += 1;
      int stop = 0;
      if ((rc = ops.observe(t, &stop)) < 0) return (scfft_status)rc;
      if (stop) break;
    }
    return SCFFT_OK;
  }

  std::vector<double> stops;
  for (double b : extra_stops)
    if (b > t0 && b < t1) stops.push_back(b);
  stops.push_back(t1);
  std::sort(stops.begin(), stops.end());
  stops.erase(std::unique(stops.begin(), stops.end()), stops.end());

  // a drive kink at t1 itself: the next run recomputes k1 there
  bool kink_at_t1 = false;
  for (double b : extra_stops)
    if (std::fabs(b - t1) <= 1e-12 * std::max(std::fabs(t1), 1.0)) kink_at_t1 = true;

  double t = t0;
  if (!(resume && cont->has_k1)) {
    if ((rc = ops.rhs(t, B_Y, B_K1)) < 0) return (scfft_status)rc;
    st.rhs_calls += 1;
  }
  double dt;
  if (resume) {
    dt = cont->dt;
  } else if (o.dt0_s > 0.0) {
    dt = o.dt0_s;
  } else {
    double r = 0.0;
    if ((rc = ops.rate(thr, &r)) < 0) return (scfft_status)rc;
    dt = (r > 0.0 && std::isfinite(r)) ? 0.8 * std::cbrt(rtol) / r : (t1 - t0);
  }
  dt = std::min(std::min(dt, dt_max), t1 - t0);
  size_t si = 0;
  bool rejected_last = resume && cont->rejected_last;
  bool nonfinite_last = false;
  auto save = [&](double tt, double dnext, bool rej, bool k1) {
    if (!cont) return;
    cont->valid = true;
    cont->t = tt;
    cont->dt = dnext;
    cont->rejected_last = rej;
    cont->has_k1 = k1;
  };
  while (t < t1 && st.accepted + st.rejected < max_steps) {
    const double stop = stops[si];
    bool hit = false;
    if (t + dt >= stop || (stop - (t + dt)) < 1e-12 * std::max(std::fabs(stop), 1.0)) {
      dt = stop - t;
      hit = true;
    }
    double err = 0.0;
    if ((rc = step(t, dt, &err)) < 0) return (scfft_status)rc;
    if (!std::isfinite(err)) err = INFINITY;
    st.err_last = err;
    if (err <= rtol) {
      if ((rc = ops.accept()) < 0) return (scfft_status)rc;
      t = hit ? stop : t + dt;
      st.t_s = t;
      st.dt_last_s = dt;
      st.accepted += 1;
      nonfinite_last = false;
      // after a drive kink (a stop before t1) k1 is recomputed: the rate may jump
      const bool kink = hit && si + 1 < stops.size() && stop < t1;
      double fac = err == 0.0 ? 5.0 : std::min(5.0, std::max(0.2, 0.8 * std::cbrt(rtol / err)));
      if (rejected_last) fac = std::min(fac, 1.0);
      const double dt_next = std::min(dt * fac, dt_max);
      save(t, dt_next, false, !kink && !(t >= t1 && kink_at_t1));
      int stop_req = 0;
      if ((rc = ops.observe(t, &stop_req)) < 0) return (scfft_status)rc;
      if (stop_req) return SCFFT_OK;
      if (hit) {
        ++si;
        if (kink) {
          if ((rc = ops.rhs(t, B_Y, B_K1)) < 0) return (scfft_status)rc;
          st.rhs_calls += 1;
          save(t, dt_next, false, true);
        }
      }
      rejected_last = false;
      dt = dt_next;
    } else {
      st.rejected += 1;
      nonfinite_last = !std::isfinite(err);
      const double fac = nonfinite_last ? 0.2 : std::max(0.2, 0.8 * std::cbrt(rtol / err));
      dt = dt * std::min(fac, rejected_last ? 0.5 : fac);
      rejected_last = true;
      if (dt < 1e-14 * std::max(std::fabs(t), 1.0)) {
        if (cont) cont->valid = false;
        return nonfinite_last ? SCFFT_ERR_NAN : SCFFT_ERR_STEP_UNDERFLOW;
      }
      save(t, dt, true, true);
    }
  }
  return SCFFT_OK;
}

}  // namespace scfft
