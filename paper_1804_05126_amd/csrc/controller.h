// Step controller of the KIOPS solver: Algorithm 4 with the acceptance test of
// Section 3.5 (Eq. (39)), the variable step size of Section 3.6.1 (Eqs. (43)-(44))
// and the variable Krylov dimension of Section 3.6.2 (Eqs. (45)-(46)).
// Plain scalar code, compiled for the device (where the solver calls it once per
// attempt) and for the host (tests).
#pragma once

#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__)
#define KIOPS_HD __host__ __device__
#else
#define KIOPS_HD
#endif

namespace kiops {

// Paper constants: delta of Section 3.5; gamma and the smaller safety factor
// used after a rejection at m_max (Section 3.6); default kappa (Section 3.6.2).
constexpr double kDelta = 1.4;
constexpr double kGamma = 0.9;
constexpr double kGammaReject = 0.6;
constexpr double kKappa0 = 2.0;

enum CtrlBranch : int32_t {
  kBranchBreakdown = 0,
  kBranchTauReject = 1,
  kBranchTauAccept = 2,
  kBranchMReject = 3,
  kBranchMAccept = 4,
  kBranchNonFinite = -1,
};

struct CtrlIn {
  double T_end, tol, T_now, tau;
  int32_t m_min, m_max, m, have_old;   // have_old: previous attempt of this substep was rejected
  double tau_old, eps_old, omega_old;  // values of that rejected attempt
  int32_t m_old, reserved;
};

struct CtrlOut {
  int32_t accept, m_new, branch, reserved;
  double tau_new, omega;
};

// Order estimate for Eq. (44).  Default m/4 - 1 (Section 3.6.1).  After a
// rejected attempt of the same substep with another tau, the model
// eps ~ C tau^(ord+1) gives ord + 1 = log(eps/eps_old) / log(tau/tau_old)
// (Eq. (43) read with the ratio of errors over the ratio of steps).
KIOPS_HD inline double ctrl_order(const CtrlIn& s, int j, double eps) {
  double dflt = 0.25 * (double)j - 1.0;
  if (s.have_old && s.tau_old != s.tau && s.eps_old > 0.0 && eps > 0.0) {
    double o = log(eps / s.eps_old) / log(s.tau / s.tau_old) - 1.0;
    if (isfinite(o) && o + 1.0 > 0.0) return o;
  }
  return dflt;
}

// Convergence-rate estimate of Eq. (45): used when this attempt and the
// previous one of the substep were both rejected at different dimensions.
KIOPS_HD inline double ctrl_kappa(const CtrlIn& s, int j, double omega) {
  if (s.have_old && omega > kDelta && s.m_old != j && s.omega_old > 0.0 && omega > 0.0) {
    double k = pow(omega / s.omega_old, 1.0 / (double)(s.m_old - j));
    if (isfinite(k) && k > 1.0) return k;
  }
  return kKappa0;
}

KIOPS_HD inline double ctrl_min(double a, double b) { return a < b ? a : b; }
KIOPS_HD inline double ctrl_max(double a, double b) { return a > b ? a : b; }

// One decision.  j = basis size reached, eps = estimate of Eq. (36).
KIOPS_HD inline CtrlOut ctrl_decide(const CtrlIn& s, int j, double eps, bool breakdown) {
  CtrlOut o;
  o.reserved = 0;
  const double tau = s.tau;
  const double omega = s.T_end * eps / (tau * s.tol);           // Eq. (39)
  o.omega = omega;
  if (!isfinite(omega)) {
    o.accept = 0; o.m_new = s.m; o.tau_new = tau; o.branch = kBranchNonFinite;
    return o;
  }
  if (breakdown || omega == 0.0) {                               // Alg. 4: breakdown
    o.accept = 1; o.tau_new = tau; o.m_new = s.m; o.branch = kBranchBreakdown;
    return o;
  }
  if (j == s.m_max) {                                            // Alg. 4: at m_max
    const double ord = ctrl_order(s, j, eps);
    if (omega > kDelta) {
      double tn = tau * pow(kGammaReject / omega, 1.0 / (ord + 1.0));
      tn = ctrl_min(s.T_end - s.T_now, ctrl_max(tau / 5.0, tn));
      o.accept = 0; o.tau_new = tn; o.m_new = j; o.branch = kBranchTauReject;
      return o;
    }
    double tn = tau * pow(kGamma / omega, 1.0 / (ord + 1.0));   // Eq. (44)
    tn = ctrl_min(5.0 * tau, ctrl_max(tau / 5.0, tn));
    o.accept = 1; o.tau_new = tn; o.m_new = s.m; o.branch = kBranchTauAccept;
    return o;
  }
  const double kap = ctrl_kappa(s, j, omega);                    // Alg. 4, Eq. (45)
  double mn = ceil((double)j + log(omega / kGamma) / log(kap));  // Eq. (46)
  double lo = ctrl_max((double)s.m_min, floor(0.75 * (double)j));
  double hi = ctrl_min((double)s.m_max, ceil(4.0 * (double)j / 3.0));
  mn = ctrl_min(hi, ctrl_max(lo, mn));
  o.tau_new = tau;
  if (omega > kDelta) {
    mn = ctrl_max(mn, (double)(j + 1));
    o.accept = 0; o.m_new = (int32_t)mn; o.branch = kBranchMReject;
    return o;
  }
  o.accept = 1; o.m_new = (int32_t)mn; o.branch = kBranchMAccept;
  return o;
}

// Bookkeeping of the "old" values (Section 3.6): kept only from the
// immediately preceding rejected attempt of the same substep.
KIOPS_HD inline void ctrl_record(CtrlIn& s, const CtrlOut& o, int j, double eps) {
  if (o.accept) {
    s.have_old = 0;
  } else {
    s.have_old = 1;
    s.tau_old = s.tau;
    s.eps_old = eps;
    s.omega_old = o.omega;
    s.m_old = j;
  }
}

}  // namespace kiops
