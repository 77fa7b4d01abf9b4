// The persistent solve kernel: Algorithm 1 (Task II) on the device.
//
//   setup:   ||B||_1 -> nu, mu (Eqs. (48)-(49)); w <- b_0
//   substep: start vector [w; mu y(T_now)] (Alg. 1 lines 10-15, Eq. (47))
//   passes:  Algorithm 2, one pass per basis vector (see pass_common.h)
//   attempt: F = exp(tau H~) (Eqs. (37)-(38)), eps (Eq. (36)), Algorithm 4
//   accept:  w <- beta V(1:N, 1:j) F(1:j, 1) (Algorithm 3, Eq. (33))
//
// Every phase ends in a grid barrier whose last arriving workgroup runs the
// serial epilogue; all workgroups then read the next phase from Ctrl.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "controller.h"
#include "pass_common.h"
#include "small_expm.h"

namespace kiops {

constexpr int kLdsDoubles = 3600;   // union: pass tiles / expm staging / reductions

#define KIOPS_AGENT __HIP_MEMORY_SCOPE_AGENT

// Wait until the barrier generation moves past g.  Bounded: a wait longer than
// spin_limit ticks of the constant-rate clock raises the abort flag so that
// every workgroup leaves the kernel.
__device__ inline bool barrier_wait(Barrier* b, unsigned g, uint64_t spin_limit) {
  const uint64_t t0 = (uint64_t)wall_clock64();
  while (__hip_atomic_load(&b->gen, __ATOMIC_RELAXED, KIOPS_AGENT) == g) {
    if (__hip_atomic_load(&b->abort, __ATOMIC_RELAXED, KIOPS_AGENT)) return false;
    __builtin_amdgcn_s_sleep(2);
    if ((uint64_t)wall_clock64() - t0 > spin_limit) {
      __hip_atomic_store(&b->abort, 1u, __ATOMIC_RELAXED, KIOPS_AGENT);
      return false;
    }
  }
  return true;
}

// Grid barrier; the last workgroup to arrive runs `epi` (whole workgroup)
// before the others are released.
template <class F>
__device__ inline void grid_barrier(Barrier* b, unsigned nwg, uint64_t spin_limit, F&& epi) {
  __shared__ int s_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned g = __hip_atomic_load(&b->gen, __ATOMIC_RELAXED, KIOPS_AGENT);
    const unsigned prev = __hip_atomic_fetch_add(&b->count, 1u, __ATOMIC_ACQ_REL, KIOPS_AGENT);
    int last = (prev == nwg - 1) ? 1 : 0;
    if (!last) barrier_wait(b, g, spin_limit);
    __threadfence();
    s_last = last;
  }
  __syncthreads();
  if (s_last) {
    epi();
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
      __hip_atomic_store(&b->count, 0u, __ATOMIC_RELAXED, KIOPS_AGENT);
      __hip_atomic_fetch_add(&b->gen, 1u, __ATOMIC_RELEASE, KIOPS_AGENT);
    }
  }
  __syncthreads();
}

__device__ inline bool aborted(const KParams& P) {
  return __hip_atomic_load(&P.bar->abort, __ATOMIC_RELAXED, KIOPS_AGENT) != 0;
}

// Deterministic reduction of the per-workgroup partials: out[d] = sum_wg partials[wg][d]
// summed in workgroup order, for d < ndots.  Result in LDS `out` (all threads).
__device__ inline void reduce_partials(const KParams& P, int ndots, double* out) {
  const int t = threadIdx.x;
  if (ndots <= 16) {
    const int d = t >> 4, lane = t & 15;
    double s = 0.0;
    if (d < ndots)
      for (int wgi = lane; wgi < P.nwg; wgi += 16) s += P.partials[(int64_t)wgi * P.ndot_stride + d];
    for (int off = 8; off > 0; off >>= 1) s += __shfl_down(s, off, 16);
    if (d < ndots && lane == 0) out[d] = s;
  } else {
    for (int d = t; d < ndots; d += kThreads) {
      double s = 0.0;
      for (int wgi = 0; wgi < P.nwg; ++wgi) s += P.partials[(int64_t)wgi * P.ndot_stride + d];
      out[d] = s;
    }
  }
  __syncthreads();
}

__device__ inline double& Hel(const KParams& P, int i, int l) { return P.H[i * kLdh + l]; }
__device__ inline double& Gel(const KParams& P, int i, int l) { return P.G[i * kLdh + l]; }
__device__ inline double* Yrow(const KParams& P, int i) { return P.Y + i * kPM; }

// Start of a substep (thread 0): exact trailing entries mu [T^{p-1}/(p-1)!, ..., T, 1].
__device__ inline void start_substep(const KParams& P) {
  Ctrl& C = *P.ctrl;
  double* y1 = Yrow(P, 1);
  const int p = C.p;
  double fact = 1.0;
  for (int i = 0; i < p; ++i) {            // entry p-1-i holds T^i / i!
    if (i > 0) fact *= (double)i;
    y1[p - 1 - i] = C.mu * pow(C.T_now, (double)i) / fact;
  }
  for (int c = 0; c < kPM; ++c) C.yb_cur[c] = (c < p) ? C.nu * y1[c] : 0.0;
  C.kp = 1;
  C.flo = 1;
  C.dlo = 1;
  C.breakdown = 0;
  C.have_old = 0;
  C.phase = kPhasePass;
}

__device__ inline double pass_bytes(const KParams& P, int kp, int flo) {
  // algorithmic bytes of one pass: read R_{kp-1} and the older window
  // vectors, B and the coefficient fields; write R_kp
  const double s = P.elem_bytes;
  double reads = (kp == 1) ? 8.0 : s * (double)(kp - flo);
  reads += s * ((double)P.p + P.coef_streams);
  const double writes = (kp == 1 && !P.mixed) ? 0.0 : s;
  return (reads + writes) * (double)P.N;
}

// The small exponential and the controller for an attempt with basis size j.
// Whole workgroup.  Loops while the attempt is rejected at m_max (same basis, smaller tau).
__device__ inline void attempt_end(const KParams& P, int j, bool breakdown, double* lds) {
  Ctrl& C = *P.ctrl;
  __shared__ int s_again;
  const int n = j + 1;
  const int n16 = pad16(n);
  for (int round = 0;; ++round) {
    const double tau = C.tau;
    double* A = P.expm;
    for (int e = threadIdx.x; e < n16 * n16; e += kThreads) {
      const int r = e / n16, c = e % n16;
      double v = 0.0;
      if (r < j && c < j) v = tau * Hel(P, r + 1, c + 1);
      else if (c == j && r == 0) v = tau;
      A[r * kExpmLd + c] = v;
    }
    __syncthreads();
    const int slot = wg_expm(P.expm, n, lds);
    const double* F = P.expm + (size_t)slot * kExpmSlot;
    if (threadIdx.x == 0) {
      const double eps = breakdown ? 0.0 : C.beta * fabs(Hel(P, j + 1, j)) * fabs(F[(j - 1) * kExpmLd + j]);
      CtrlIn ci;
      ci.T_end = C.T_end; ci.tol = C.tol; ci.T_now = C.T_now; ci.tau = tau;
      ci.m_min = C.m_min; ci.m_max = C.m_max; ci.m = C.m; ci.have_old = C.have_old;
      ci.tau_old = C.tau_old; ci.eps_old = C.eps_old; ci.omega_old = C.omega_old;
      ci.m_old = C.m_old; ci.reserved = 0;
      const CtrlOut o = ctrl_decide(ci, j, eps, breakdown);
      ctrl_record(ci, o, j, eps);
      C.have_old = ci.have_old; C.tau_old = ci.tau_old; C.eps_old = ci.eps_old;
      C.omega_old = ci.omega_old; C.m_old = ci.m_old;
      C.expms += 1;
      C.last_omega = o.omega;
      if (C.attempts < kTraceMax) {
        double* tr = P.trace + (size_t)C.attempts * kTraceStride;
        tr[0] = (double)C.substeps; tr[1] = (double)j; tr[2] = tau;
        tr[3] = o.omega; tr[4] = (double)o.accept; tr[5] = (double)o.branch;
      }
      C.attempts += 1;
      int again = 0;
      if (o.branch == kBranchNonFinite) {
        C.status = KIOPS_ERR_NONFINITE;
        C.phase = kPhaseDone;
      } else if (o.accept) {
        for (int i = 1; i <= j; ++i) C.cg[i] = C.beta * F[(i - 1) * kExpmLd] * P.sinv[i];
        C.jg = j;
        C.tau_new = o.tau_new;
        C.m_new = o.m_new;
        if (breakdown) C.breakdowns += 1;
        C.phase = kPhaseGather;
      } else {
        C.rejections += 1;
        if (j == C.m_max) {
          C.tau = o.tau_new;
          again = 1;
          if (round >= 1000 || !(o.tau_new > 0.0)) {   // step size collapsed: give up
            C.status = KIOPS_ERR_NOT_CONVERGED;
            C.phase = kPhaseDone;
            again = 0;
          }
        } else {
          C.m = o.m_new;
          C.phase = kPhasePass;
        }
      }
      s_again = again;
    }
    __syncthreads();
    if (!s_again) break;
  }
}

// Epilogue after the setup phase.
__device__ inline void epilogue_setup(const KParams& P, double* lds) {
  reduce_partials(P, kPM, lds);
  if (threadIdx.x == 0) {
    Ctrl& C = *P.ctrl;
    double nb = 0.0;
    for (int k = 0; k < P.p; ++k) nb = lds[k] > nb ? lds[k] : nb;
    double nu = 1.0, mu = 1.0;
    if (P.p > 0 && nb > 0.0 && isfinite(nb)) {
      int e;
      const double f = frexp(nb, &e);          // nb = f 2^e, f in [0.5, 1)
      const int c = (f == 0.5) ? e - 1 : e;    // ceil(log2 nb)
      nu = ldexp(1.0, -c);
      mu = ldexp(1.0, c);
    }
    C.nu = nu; C.mu = mu;
    C.T_now = 0.0; C.T_end = P.T_end; C.tau = P.T_end; C.tol = P.tol;
    C.p = P.p; C.q = P.q; C.m_min = P.m_min; C.m_max = P.m_max; C.max_substeps = P.max_substeps;
    int m = P.m_init < P.m_max ? P.m_init : P.m_max;   // Alg. 1, line 3
    C.m = m > P.m_min ? m : P.m_min;
    C.m_new = C.m;
    C.status = KIOPS_OK;
    C.mode = P.mode;
    C.substeps = C.rejections = C.expms = C.breakdowns = C.attempts = 0;
    C.matvecs = 0;
    C.last_omega = 0.0;
    C.beta = 0.0;
    C.alg_bytes = (double)P.p * 8.0 * (double)P.N;   // ||B||_1
    if (!isfinite(nb)) {
      C.status = KIOPS_ERR_NONFINITE;
      C.phase = kPhaseDone;
    } else if (P.T_end == 0.0) {
      C.phase = kPhaseDone;
    } else {
      start_substep(P);
    }
  }
  __syncthreads();
}

// Epilogue after pass kp.
__device__ inline void epilogue_pass(const KParams& P, double* lds) {
  Ctrl& C = *P.ctrl;
  __shared__ int s_action;    // 0 continue, 1 attempt end, 2 attempt end with breakdown
  __shared__ int s_j;
  const int kp = C.kp;
  const int dlo = C.dlo;
  const int ngd = kp - dlo;
  reduce_partials(P, kDotSlots, lds);
  if (threadIdx.x == 0) {
    int action = 0;
    const int k = kp;
    const int p = C.p;
    const double* yk = Yrow(P, k);
    double ykr[kPM], Ky[kPM];
#pragma unroll
    for (int c = 0; c < kPM; ++c) ykr[c] = (c < p) ? yk[c] : 0.0;
#pragma unroll
    for (int c = 0; c < kPM; ++c) Ky[c] = (c + 1 < kPM) ? ykr[c + 1] : 0.0;   // K y: upper shift
    double RR = lds[kDotRR], UU = lds[kDotUU], Ck = lds[kDotCk];
#pragma unroll
    for (int c = 0; c < kPM; ++c) { RR += ykr[c] * ykr[c]; UU += Ky[c] * Ky[c]; Ck += ykr[c] * Ky[c]; }
    C.matvecs += 1;
    C.alg_bytes += pass_bytes(P, kp, C.flo);
    bool finite = isfinite(RR) && isfinite(UU) && isfinite(Ck);
    for (int d = 0; d < ngd; ++d) finite = finite && isfinite(lds[kDotG + d]) && isfinite(lds[kDotC + d]);
    const double s = sqrt(RR);
    if (!finite) {
      C.status = KIOPS_ERR_NONFINITE;
      C.phase = kPhaseDone;
      action = 3;
    } else if (k == 1 && s == 0.0) {
      // zero start vector: the solution stays zero (w == 0 already)
      C.beta = 0.0;
      C.T_now = C.T_end;
      C.phase = kPhaseDone;
      action = 3;
    } else if (k > 1 && (s == 0.0 || s <= 1e-12 * P.unorm[k - 1])) {
      Hel(P, k, k - 1) = 0.0;                 // happy breakdown (Alg. 2, lines 12-14)
      C.breakdown = 1;
      C.s_last = s;
      action = 2;
    } else {
      if (k == 1) C.beta = s;
      else Hel(P, k, k - 1) = s;
      C.s_last = s;
      const double si = 1.0 / s;
      P.sinv[k] = si;
      P.unorm[k] = sqrt(UU) * si;
      for (int d = 0; d < ngd; ++d) {
        const int i = dlo + d;
        double yd = 0.0;
        const double* yi = Yrow(P, i);
#pragma unroll
        for (int c = 0; c < kPM; ++c) yd += (c < p) ? yi[c] * ykr[c] : 0.0;
        const double g = (lds[kDotG + d] + yd) * P.sinv[i] * si;
        Gel(P, i, k) = g;
        Gel(P, k, i) = g;
      }
      Gel(P, k, k) = 1.0;
      // modified Gram-Schmidt over the window [dlo, k] (Alg. 2, lines 7-10)
      for (int i = dlo; i <= k; ++i) {
        double raw;
        if (i < k) {
          const double* yi = Yrow(P, i);
          double yd = 0.0;
#pragma unroll
          for (int c = 0; c < kPM; ++c) yd += (c < p) ? yi[c] * Ky[c] : 0.0;
          raw = lds[kDotC + (i - dlo)] + yd;
        } else {
          raw = Ck;
        }
        double h = raw * P.sinv[i] * si;
        for (int l = dlo; l < i; ++l) h -= Hel(P, l, k) * Gel(P, i, l);
        Hel(P, i, k) = h;
      }
      // coefficients of the next pass: R_{k+1} = si U_k - sum_i H(i,k) sinv[i] R_i
      double* yn = Yrow(P, k + 1);
#pragma unroll
      for (int c = 0; c < kPM; ++c) {
        double v = (c < p) ? si * Ky[c] : 0.0;
        if (c < p)
          for (int i = dlo; i <= k; ++i) v -= Hel(P, i, k) * P.sinv[i] * Yrow(P, i)[c];
        yn[c] = (c < p) ? v : 0.0;
        C.yb_prev[c] = (c < p) ? C.nu * ykr[c] : 0.0;
        C.yb_cur[c] = (c < p) ? C.nu * v : 0.0;
      }
      C.a = si;
      for (int i = dlo; i <= k; ++i) C.bw[i] = -Hel(P, i, k) * P.sinv[i];
      C.flo = dlo;
      C.kp = k + 1;
      C.dlo = (C.q == 0) ? 1 : ((k + 1 - C.q + 1) > 1 ? (k + 1 - C.q + 1) : 1);
      const int jdone = k - 1;
      if (C.mode == kModeBasis) {
        if (jdone >= C.m) { C.phase = kPhaseDone; action = 3; }
      } else if (jdone >= C.m && jdone >= 1) {
        action = 1;
      }
      C.phase = (action == 3) ? kPhaseDone : kPhasePass;
    }
    if (action == 2 && C.mode == kModeBasis) { C.phase = kPhaseDone; action = 3; }
    s_action = action;
    s_j = k - 1;
  }
  __syncthreads();
  const int action = s_action;
  if (action == 1 || action == 2) attempt_end(P, s_j, action == 2, lds);
}

// Epilogue after the gather: advance T_now (Alg. 1, line 24) and start the next substep.
__device__ inline void epilogue_gather(const KParams& P) {
  if (threadIdx.x == 0) {
    Ctrl& C = *P.ctrl;
    const double s = P.elem_bytes;
    C.alg_bytes += (8.0 + s * (double)(C.jg - 1) + 8.0) * (double)P.N;
    C.T_now = C.T_now + C.tau;
    if (C.T_end - C.T_now <= 8.0 * 2.220446049250313e-16 * C.T_end) C.T_now = C.T_end;
    const double rem = C.T_end - C.T_now;
    C.tau = C.tau_new < rem ? C.tau_new : rem;
    C.m = C.m_new;
    C.substeps += 1;
    if (C.T_now >= C.T_end) {
      C.phase = kPhaseDone;
    } else if (C.substeps >= C.max_substeps) {
      C.status = KIOPS_ERR_NOT_CONVERGED;
      C.phase = kPhaseDone;
    } else {
      start_substep(P);
    }
  }
  __syncthreads();
}

template <typename T>
__device__ inline void load_pass_ctx(const KParams& P, PassCtx<T>& c) {
  const Ctrl& C = *P.ctrl;
  if (threadIdx.x == 0) {
    c.kp = C.kp;
    c.src = C.kp - 1;
    c.flo = C.flo;
    c.dlo = C.dlo;
    c.ngd = C.kp - C.dlo;
    c.first = (C.kp == 1);
    c.write_out = !(C.kp == 1 && !P.mixed);
    c.p = C.p;
    c.a = (T)C.a;
  }
  for (int i = threadIdx.x; i < kLdh; i += kThreads) c.bw[i] = (T)C.bw[i];
  if (threadIdx.x < kPM) {
    c.ybp[threadIdx.x] = (T)C.yb_prev[threadIdx.x];
    c.ybc[threadIdx.x] = (T)C.yb_cur[threadIdx.x];
  }
  __syncthreads();
}

// Write the per-workgroup partial inner products of a pass (fixed slots kDot*).
__device__ inline void store_partials(const KParams& P, const DotAcc& acc, double* lds) {
  double packed[kDotSlots];
  packed[kDotRR] = acc.RR;
  packed[kDotUU] = acc.UU;
#pragma unroll
  for (int d = 0; d < kWinMax - 1; ++d) {
    packed[kDotG + d] = acc.G[d];
    packed[kDotC + d] = acc.C[d];
  }
  packed[kDotCk] = acc.Ck;
  block_sum(packed, kDotSlots, lds, P.partials + (int64_t)blockIdx.x * P.ndot_stride);
}

template <class Op, typename T>
__device__ inline void setup_phase(const KParams& P, const Op& op, T* bcopy, double* lds) {
  const int64_t gt = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t gs = (int64_t)gridDim.x * kThreads;
  for (int64_t e = gt; e < (int64_t)kLdh * kLdh; e += gs) { P.H[e] = 0.0; P.G[e] = 0.0; }
  double sums[kPM];
#pragma unroll
  for (int k = 0; k < kPM; ++k) sums[k] = 0.0;
  const bool copy_b0 = P.w != P.b[0];
  for (int64_t n = gt; n < P.N; n += gs) {
    if (copy_b0) P.w[n] = P.b[0][n];
#pragma unroll
    for (int k = 0; k < kPM; ++k) {
      if (k < P.p) {
        const double v = P.b[k + 1][n];
        sums[k] += fabs(v);
        if (P.mixed) bcopy[(int64_t)(P.p - 1 - k) * P.N + n] = (T)v;   // column c = p-k holds b_k
      }
    }
  }
  op.setup_coefficients(P, gt, gs);
  block_sum(sums, kPM, lds, P.partials + (int64_t)blockIdx.x * P.ndot_stride);
}

// Gather w <- sum_i cg[i] R_i (R_1 = w).
template <typename T>
__device__ inline void gather_phase(const KParams& P, const BasisPtrs<T>& bp, double* lds) {
  const Ctrl& C = *P.ctrl;
  const int jg = C.jg;
  for (int i = threadIdx.x; i <= jg; i += kThreads) lds[i] = C.cg[i];
  __syncthreads();
  const int64_t gt = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t gs = (int64_t)gridDim.x * kThreads;
  for (int64_t n = gt; n < P.N; n += gs) {
    double acc = lds[1] * P.w[n];
    int i = 2;
    for (; i + 3 <= jg; i += 4) {
      const double a0 = (double)bp.get(i)[n];
      const double a1 = (double)bp.get(i + 1)[n];
      const double a2 = (double)bp.get(i + 2)[n];
      const double a3 = (double)bp.get(i + 3)[n];
      acc = fma(lds[i], a0, acc);
      acc = fma(lds[i + 1], a1, acc);
      acc = fma(lds[i + 2], a2, acc);
      acc = fma(lds[i + 3], a3, acc);
    }
    for (; i <= jg; ++i) acc = fma(lds[i], (double)bp.get(i)[n], acc);
    P.w[n] = acc;
  }
  __syncthreads();
}

template <class Op, typename T>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 8)))
kiops_solve_kernel(KParams P, Op op) {
  __shared__ double lds[kLdsDoubles];
  __shared__ PassCtx<T> pctx;
  const unsigned nwg = gridDim.x;
  T* bcopy = reinterpret_cast<T*>(P.bcopy);
  BasisPtrs<T> bp;
  bp.R1 = P.mixed ? reinterpret_cast<const T*>(P.slots) : reinterpret_cast<const T*>(P.w);
  bp.slots = reinterpret_cast<T*>(P.slots);
  bp.N = P.N;

  setup_phase<Op, T>(P, op, bcopy, lds);
  grid_barrier(P.bar, nwg, P.spin_limit, [&] { epilogue_setup(P, lds); });

  for (int iter = 0;; ++iter) {
    if (aborted(P)) break;
    __shared__ int s_phase;
    if (threadIdx.x == 0) s_phase = __hip_atomic_load(&P.ctrl->phase, __ATOMIC_RELAXED, KIOPS_AGENT);
    __syncthreads();
    const int phase = s_phase;
    if (phase == kPhaseDone) break;
    if (phase == kPhasePass) {
      load_pass_ctx<T>(P, pctx);
      DotAcc acc;
      acc.zero();
      T* Rout = bp.get_mut(pctx.kp);
      op.pass(pctx, bp, P.w, Rout, acc, reinterpret_cast<T*>(lds));
      store_partials(P, acc, lds);
      grid_barrier(P.bar, nwg, P.spin_limit, [&] { epilogue_pass(P, lds); });
    } else {
      gather_phase<T>(P, bp, lds);
      grid_barrier(P.bar, nwg, P.spin_limit, [&] { epilogue_gather(P); });
    }
  }
}

__global__ void kiops_reset_kernel(Barrier* b, Ctrl* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    b->count = 0;
    b->gen = 0;
    b->abort = 0;
    b->pad = 0;
    c->phase = kPhaseDone;
    c->status = KIOPS_OK;
  }
}

}  // namespace kiops
