"""Algorithm 4 with Sections 3.5-3.6: acceptance, step size and dimension.

One decision per attempt.  Inputs: the basis size j reached, the error
estimate eps of Eq. (36), whether Algorithm 2 broke down, and the controller
state.  Output: accept?, tau_new, m_new and omega.

  omega = T_end eps / (tau tol)                         Eq. (39), accept iff omega <= delta = 1.4
  breakdown (or omega == 0): accept, tau_new = tau, m_new = m      Alg. 4
  j == m_max:
      rejected: m_new = j, tau_new = tau (0.6/omega)^(1/(ord+1)),
                clipped below by tau/5 and above by T_end - T_now    Alg. 4
      accepted: tau_new = tau (0.9/omega)^(1/(ord+1)), clipped to [tau/5, 5 tau]   Eq. (44)
  otherwise:
      m_new = ceil(j + log(omega/0.9)/log(kappa)), clipped to
      [max(m_min, floor(3j/4)), min(m_max, ceil(4j/3))], and >= j+1 after a
      rejection; tau unchanged                             Eqs. (45)-(46)
  ord  = log(eps/eps_old)/log(tau/tau_old) - 1 after a rejected attempt with a
         different tau in the same substep (the model eps ~ C tau^(ord+1) of
         Section 3.6.1 solved for ord), else j/4 - 1; the default is also used
         when the estimate is not finite or ord + 1 <= 0.
  kappa = (omega/omega_old)^(1/(m_old - j)) when this attempt and the
         previous one (same substep, different m) were both rejected, else 2;
         2 is also used when the estimate is not finite or <= 1.

The clip of tau to the remaining interval after an accepted step is applied
by the caller (Algorithm 1) once T_now has advanced.
"""

from __future__ import annotations

import dataclasses
import math

DELTA = 1.4
GAMMA = 0.9
GAMMA_MAX = 0.6   # the smaller safety factor used after a rejection at m_max
KAPPA0 = 2.0


@dataclasses.dataclass
class ControllerState:
    T_end: float
    tol: float
    m_min: int = 10
    m_max: int = 128
    T_now: float = 0.0
    tau: float = 0.0
    m: int = 10
    have_old: bool = False
    tau_old: float = 0.0
    eps_old: float = 0.0
    omega_old: float = 0.0
    m_old: int = 0


@dataclasses.dataclass
class Decision:
    accept: bool
    tau_new: float
    m_new: int
    omega: float
    branch: str


def _order(st: ControllerState, j: int, eps: float) -> float:
    default = j / 4.0 - 1.0
    if st.have_old and st.tau_old != st.tau and st.eps_old > 0.0 and eps > 0.0:
        try:
            o = math.log(eps / st.eps_old) / math.log(st.tau / st.tau_old) - 1.0
        except (ValueError, ZeroDivisionError):
            return default
        if math.isfinite(o) and o + 1.0 > 0.0:
            return o
    return default


def _kappa(st: ControllerState, j: int, omega: float) -> float:
    if st.have_old and omega > DELTA and st.m_old != j and st.omega_old > 0.0 and omega > 0.0:
        try:
            k = (omega / st.omega_old) ** (1.0 / (st.m_old - j))
        except (ValueError, ZeroDivisionError, OverflowError):
            return KAPPA0
        if math.isfinite(k) and k > 1.0:
            return k
    return KAPPA0


def decide(st: ControllerState, j: int, eps: float, breakdown: bool) -> Decision:
    tau = st.tau
    omega = st.T_end * eps / (tau * st.tol)
    if not math.isfinite(omega):
        raise FloatingPointError("non-finite error estimate")
    if breakdown or omega == 0.0:
        return Decision(True, tau, st.m, omega, "breakdown")
    if j == st.m_max:
        ord_ = _order(st, j, eps)
        if omega > DELTA:
            tn = tau * (GAMMA_MAX / omega) ** (1.0 / (ord_ + 1.0))
            tn = min(st.T_end - st.T_now, max(tau / 5.0, tn))
            return Decision(False, tn, j, omega, "tau_reject")
        tn = tau * (GAMMA / omega) ** (1.0 / (ord_ + 1.0))
        tn = min(5.0 * tau, max(tau / 5.0, tn))
        return Decision(True, tn, st.m, omega, "tau_accept")
    kap = _kappa(st, j, omega)
    mn = math.ceil(j + math.log(omega / GAMMA) / math.log(kap))
    lo = max(st.m_min, math.floor(0.75 * j))
    hi = min(st.m_max, math.ceil(4.0 * j / 3.0))
    mn = min(hi, max(lo, mn))
    if omega > DELTA:
        mn = max(mn, j + 1)
        return Decision(False, tau, mn, omega, "m_reject")
    return Decision(True, tau, mn, omega, "m_accept")


def record(st: ControllerState, d: Decision, j: int, eps: float) -> None:
    """Keep the "old" values of a rejected attempt for the next attempt of the
    same substep; an accepted attempt clears them."""
    if d.accept:
        st.have_old = False
    else:
        st.have_old = True
        st.tau_old = st.tau
        st.eps_old = eps
        st.omega_old = d.omega
        st.m_old = j
