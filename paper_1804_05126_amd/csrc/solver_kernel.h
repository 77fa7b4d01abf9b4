// The persistent solve kernel: Algorithm 1 (Task II) on the device.
//
//   setup:   ||B||_1 -> nu, mu (Eqs. (48)-(49)); w <- b_0
//   substep: start vector [w; mu y(T_now)] (Alg. 1, Eq. (47))
//   passes:  Algorithm 2, one pass per basis vector (see pass_common.h)
//   attempt: F = exp(tau H~) (Eqs. (37)-(38)), eps (Eq. (36)), Algorithm 4
//   accept:  w <- beta V(1:N, 1:j) F(1:j, 1) (Algorithm 3, Eq. (33))
//
// Every phase ends in a grid barrier.  Workgroup 0 collects the arrivals,
// runs the serial epilogue and releases the grid.  The solver's small state
// (control block, normalisations, the band of H, the window of the Gram
// matrix and of the trailing parts) lives in workgroup 0's LDS for the whole
// solve; after each epilogue the control block is published to device memory,
// where the other workgroups read the next phase and its coefficients.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "controller.h"
#include "pass_common.h"
#include "small_expm.h"

namespace kiops {

constexpr int kLdsDoubles = 2600;           // union: pass tiles / expm staging
constexpr int kRingRows = kWinMax + 2;      // ring of trailing parts and Gram rows

#define KIOPS_AGENT __HIP_MEMORY_SCOPE_AGENT

// Small state of workgroup 0 (LDS).
struct SmallState {
  Ctrl C;
  double sinv[kLdh];                 // v_i = R_i * sinv[i]
  double Hb[kLdh][kWinMax + 1];      // Hb[k][d] = H(k - kWinMax + 1 + d, k)
  double Yw[kRingRows][kPM];         // y-part of R_i at row i % kRingRows
  double Gw[kRingRows][kWinMax];     // Gw[k % kRingRows][d] = G(k, k - kWinMax + 1 + d)
  double unorm_prev;                 // ||A~ v_{kp-1}||
  double fy[kPM], fky[kPM], fsi, fck;  // full-window step: y_k, K y_k, 1/s_k, <R_k, U_k>
  double red[16];                    // reduced inner products
  int action, jj, again, expired;
  uint32_t ctx_stage[kCtxWords];     // payloads of the release words (every workgroup)
  // next-pass coefficients: the serial step hands them to kPM lanes
  double nx_si, nx_hk[kWinMax], nx_ky[kPM], nx_ykr[kPM];
  int nx_k, nx_dlo, nx_p, nx_go;
  // Copy of the solve's parameter block: the epilogue's serial steps read
  // their parameters from LDS rather than from device memory, where each
  // read after the barrier's acquire is a round trip of about a microsecond.
  KParams P;
};

// Store to device memory through a global (not flat) address.  The serial
// epilogue interleaves LDS reads with stores of its diagnostics copies; a
// flat store counts against both wait counters, so every wait for an LDS
// read would also wait for the previous stores to complete.
__device__ __forceinline__ void gstore(double* p, double v) {
  *(__attribute__((address_space(1))) double*)p = v;
}

__device__ inline double h_get(const SmallState& S, int i, int k) {
  const int d = i - (k - kWinMax + 1);
  return (d >= 0 && d <= kWinMax) ? S.Hb[k][d] : 0.0;
}
__device__ inline void h_set(SmallState& S, const KParams& P, int i, int k, double v) {
  const int d = i - (k - kWinMax + 1);
  if (d >= 0 && d <= kWinMax) S.Hb[k][d] = v;   // the band kept in LDS
  gstore(&P.H[i * kLdh + k], v);                // full copy in device memory
}
__device__ inline double g_get(const SmallState& S, int i, int l) {   // |i - l| < kWinMax
  if (i < l) { const int t = i; i = l; l = t; }
  return S.Gw[i % kRingRows][l - (i - kWinMax + 1)];
}
__device__ inline double* y_row(SmallState& S, int i) { return S.Yw[i % kRingRows]; }

__device__ inline bool spin_expired(Barrier* b, uint64_t t0, uint64_t spin_limit) {
  if (__hip_atomic_load(&b->abort, __ATOMIC_RELAXED, KIOPS_AGENT)) return true;
  if ((uint64_t)wall_clock64() - t0 > spin_limit) {
    __hip_atomic_store(&b->abort, 1u, __ATOMIC_RELAXED, KIOPS_AGENT);
    return true;
  }
  return false;
}

// Payload of release word l (low 32 bits; the epoch is the high half).
__device__ inline uint32_t ctx_payload(const Ctrl& C, int phase, int l) {
  if (l == 0) return (uint32_t)phase;
  if (l == 1) return (uint32_t)C.kp;
  if (l == 2) return (uint32_t)C.flo;
  if (l == 3) return (uint32_t)C.dlo;
  const int d = (l - 4) >> 1;
  double v;
  if (d == 0) {
    v = C.a;
  } else if (d <= kWinMax) {
    const int i = C.flo + d - 1;
    v = i < kLdh ? C.bw[i] : 0.0;
  } else if (d <= kWinMax + kPM) {
    v = C.yb_prev[d - 1 - kWinMax];
  } else {
    v = C.yb_cur[d - 1 - kWinMax - kPM];
  }
  return (uint32_t)(((l - 4) & 1) ? __double2hiint(v) : __double2loint(v));
}

// Pass context from a control block (workgroup 0: its own; the others: the
// published one, for the phases and windows the release words do not carry).
template <typename T>
__device__ inline void ctx_from_ctrl(const KParams& P, const Ctrl& C, PassCtx<T>& c) {
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
    c.store_u = (C.q == 0);
    c.ranks = P.ranks;
  }
  for (int i = threadIdx.x; i < kLdh; i += kThreads) c.bw[i] = (T)C.bw[i];
  if (threadIdx.x < kPM) {
    c.ybp[threadIdx.x] = (T)C.yb_prev[threadIdx.x];
    c.ybc[threadIdx.x] = (T)C.yb_cur[threadIdx.x];
  }
}

// Pass context from the payloads of the release words (a pass whose window
// coefficients bw[flo..kp-1] are among the kWinMax carried).  Only those bw
// entries are written: the passes read no others.
template <typename T>
__device__ inline void ctx_from_words(const KParams& P, const uint32_t* st, PassCtx<T>& c) {
  auto dbl = [&](int d) { return __hiloint2double((int)st[5 + 2 * d], (int)st[4 + 2 * d]); };
  const int kp = (int)st[1], flo = (int)st[2], dlo = (int)st[3];
  const int t = threadIdx.x;
  if (t == 0) {
    c.kp = kp;
    c.src = kp - 1;
    c.flo = flo;
    c.dlo = dlo;
    c.ngd = kp - dlo;
    c.first = (kp == 1);
    c.write_out = !(kp == 1 && !P.mixed);
    c.p = P.p;
    c.a = (T)dbl(0);
    c.store_u = (P.q == 0);
    c.ranks = P.ranks;
  }
  if (t < kWinMax && flo + t < kLdh) c.bw[flo + t] = (T)dbl(1 + t);
  if (t < kPM) {
    c.ybp[t] = (T)dbl(1 + kWinMax + t);
    c.ybc[t] = (T)dbl(1 + kWinMax + kPM + t);
  }
}

// Grid barrier without contended atomics.  Workgroup w publishes its arrival
// by storing the barrier epoch into arrive[w]; workgroup 0 waits until every
// slot holds the epoch, runs `epi`, and releases the grid with the release
// words: the next phase and, for a windowed pass, its whole context, each
// 64-bit word tagged with the epoch, so that a workgroup that sees every
// word tagged has the context in hand (one round trip instead of a release
// flag followed by reads of the control block).  It also stores the epoch
// into `gen` (the sub-grid barriers wait on that).  On return s_phase holds
// the next phase and pctx its pass context.  Every wait is bounded by
// spin_limit ticks of the constant-rate clock; on expiry the abort flag is
// raised and all workgroups leave (the next phase reads as done).
//
// kWriteThrough: the barrier that ends a single-phase pass, all of whose
// stores to device memory are device-scope (write-through: buf_st and the
// partial sums).  The arrival then does not issue the agent-scope release
// fence, whose L2 write-back took 2.4 us per workgroup on average (4 us for
// the last one) at 2048^2 even with write-through outputs; instead every wave
// waits until its own stores have completed, which for device-scope stores
// means that they have reached the device's coherence point.  (The fence is
// implemented on this target as that same wait preceded by the write-back of
// dirty L2 lines, which such stores do not leave.)  Every other barrier keeps
// the fence; workgroup 0's release keeps it unless it follows such a barrier
// and the next phase is a windowed pass (then the release words are all the
// other workgroups read).
template <bool kWriteThrough = false, typename T, class F>
__device__ inline void grid_barrier(const KParams& P, SmallState& S, unsigned& epoch, PassCtx<T>& pctx,
                                    int& s_phase, F&& epi) {
  Barrier* b = P.bar;
  ++epoch;
  if constexpr (kWriteThrough) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wave's stores done
  // The workgroup's stores are ordered before wave 0's agent-scope release
  // (one L2 write-back per workgroup rather than one per wave).
  __syncthreads();
  if (vblock() != 0) {
    if (threadIdx.x < 64) {
      const int lane = threadIdx.x;
      if (lane == 0) {
        if constexpr (kWriteThrough) {
          if (P.profile) {
            __hip_atomic_store(&P.arrive_t[vblock()], (uint64_t)wall_clock64(), __ATOMIC_RELAXED, KIOPS_AGENT);
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
          }
        } else {
          if (P.profile) P.arrive_t[vblock()] = (uint64_t)wall_clock64();
          // release (the workgroup's stores, ordered before this wave by the
          // barrier above) then the arrival flag.  One-sided fences: a full
          // fence would also invalidate the XCD's L2 under the workgroups
          // still running their pass.
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        }
        __hip_atomic_store(&P.arrive[vblock()], epoch, __ATOMIC_RELAXED, KIOPS_AGENT);
      }
      uint64_t w = 0;
      int expired = 0;
      const uint64_t t0 = (uint64_t)wall_clock64();
      for (unsigned spins = 1;; ++spins) {
        if (lane < kCtxUsed) w = __hip_atomic_load(&P.tctx[lane], __ATOMIC_RELAXED, KIOPS_AGENT);
        if (__all(lane >= kCtxUsed || (uint32_t)(w >> 32) == epoch)) break;
        for (int z = 0; z < P.poll_sleep; ++z) __builtin_amdgcn_s_sleep(2);
        if ((spins & 63u) == 0) {
          int e = 0;
          if (lane == 0) e = spin_expired(b, t0, P.spin_limit) ? 1 : 0;
          if (__builtin_amdgcn_readfirstlane(e)) {
            expired = 1;
            break;
          }
        }
      }
      if (lane == 0 && P.profile) P.arrive_t[P.nwg + vblock()] = (uint64_t)wall_clock64();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      if (lane < kCtxWords) S.ctx_stage[lane] = (uint32_t)w;
      if (lane == 0 && expired) S.ctx_stage[0] = (uint32_t)kPhaseDone;
    }
    __syncthreads();
    const int ph = (int)S.ctx_stage[0];
    const int kp = (int)S.ctx_stage[1], flo = (int)S.ctx_stage[2];
    if (ph == kPhasePass && P.q != 0 && kp - 1 - flo < kWinMax) {
      ctx_from_words<T>(P, S.ctx_stage, pctx);
    } else if (ph != kPhaseDone) {
      ctx_from_ctrl<T>(P, *P.ctrl, pctx);   // published before the release words
    }
    if (threadIdx.x == 0) s_phase = ph;
    __syncthreads();
    return;
  }
  int expired = 0;
  const uint64_t t0 = (uint64_t)wall_clock64();
  for (unsigned spins = 1;; ++spins) {
    int ok = 1;
    for (unsigned w = 1 + threadIdx.x; w < (unsigned)P.nwg; w += kThreads)
      ok &= (__hip_atomic_load(&P.arrive[w], __ATOMIC_RELAXED, KIOPS_AGENT) == epoch) ? 1 : 0;
    if (__syncthreads_and(ok)) break;
    for (int z = 0; z < P.poll_sleep; ++z) __builtin_amdgcn_s_sleep(2);
    if ((spins & 15u) == 0) {
      if (threadIdx.x == 0) S.expired = spin_expired(b, t0, P.spin_limit) ? 1 : 0;   // thread 0 decides
      __syncthreads();
      if (S.expired) {
        expired = 1;
        break;
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  __syncthreads();
  const uint64_t t1 = (uint64_t)wall_clock64();
  if (P.profile) {
    // arrival spread and release delay: latest and mean, after the previous release
    uint64_t mx = 0, sum = 0, rmx = 0, rsum = 0;
    for (int w = 1 + threadIdx.x; w < P.nwg; w += kThreads) {
      const uint64_t a = P.arrive_t[w] - S.C.t_last;
      const uint64_t r = P.arrive_t[P.nwg + w] - S.C.t_last;
      if (S.C.n_barriers > 0) P.arrive_t[2 * P.nwg + w] += a;   // per-workgroup sum
      mx = a > mx ? a : mx;
      sum += a;
      rmx = r > rmx ? r : rmx;
      rsum += r;
    }
    for (int off = 32; off > 0; off >>= 1) {
      const uint64_t om = __shfl_down(mx, off, 64);
      const uint64_t os = __shfl_down(sum, off, 64);
      const uint64_t rm = __shfl_down(rmx, off, 64);
      const uint64_t rs = __shfl_down(rsum, off, 64);
      mx = om > mx ? om : mx;
      sum += os;
      rmx = rm > rmx ? rm : rmx;
      rsum += rs;
    }
    __shared__ uint64_t s_mx[kThreads / 64], s_sum[kThreads / 64], s_rmx[kThreads / 64], s_rsum[kThreads / 64];
    if ((threadIdx.x & 63) == 0) {
      s_mx[threadIdx.x >> 6] = mx;
      s_sum[threadIdx.x >> 6] = sum;
      s_rmx[threadIdx.x >> 6] = rmx;
      s_rsum[threadIdx.x >> 6] = rsum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int q = 1; q < kThreads / 64; ++q) {
        mx = s_mx[q] > mx ? s_mx[q] : mx;
        sum += s_sum[q];
        rmx = s_rmx[q] > rmx ? s_rmx[q] : rmx;
        rsum += s_rsum[q];
      }
      const uint64_t others = P.nwg > 1 ? (uint64_t)(P.nwg - 1) : 1;
      if (S.C.n_barriers > 0) {   // the first barrier has no previous release
        S.C.t_arrive_max += mx;
        S.C.t_arrive_mean += sum / others;
        S.C.t_release_max += rmx;
        S.C.t_release_mean += rsum / others;
      }
      S.C.n_barriers += 1;
    }
    __syncthreads();
  }
  epi();
  __syncthreads();   // the epilogue's stores (control block) before wave 0's release
  const int ph = expired ? (int)kPhaseDone : S.C.phase;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    if (lane == 0) {
      const uint64_t t2 = (uint64_t)wall_clock64();
      Ctrl& C = S.C;
      C.t_work += t0 - C.t_last;
      C.t_wait += t1 - t0;
      C.t_epi += t2 - t1;
      C.t_last = t2;
      if (P.profile || C.phase == kPhaseDone) {   // the timers the host reads at the end
        P.ctrl->t_work = C.t_work;
        P.ctrl->t_wait = C.t_wait;
        P.ctrl->t_epi = C.t_epi;
        P.ctrl->t_expm = C.t_expm;
        P.ctrl->t_arrive_max = C.t_arrive_max;
        P.ctrl->t_arrive_mean = C.t_arrive_mean;
        P.ctrl->t_release_max = C.t_release_max;
        P.ctrl->t_release_mean = C.t_release_mean;
        P.ctrl->n_barriers = C.n_barriers;
        P.ctrl->t_red = C.t_red;
        P.ctrl->t_pub = C.t_pub;
        P.ctrl->t_ser = C.t_ser;
        P.ctrl->t_begin = C.t_begin;
        P.ctrl->t_end = t2;
      }
    }
    // After a write-through pass barrier whose next phase is a windowed pass,
    // the other workgroups read only the release words and the pass outputs
    // (complete, device-scope); workgroup 0's plain stores of this epilogue
    // (control block, diagnostics) are read by itself or the host alone, so
    // the release needs no L2 write-back.  Every other release keeps it.
    const bool words_only = kWriteThrough && ph == kPhasePass && P.q != 0 && S.C.kp - 1 - S.C.flo < kWinMax;
    if (!words_only) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lane < kCtxUsed)
      __hip_atomic_store(&P.tctx[lane], ((uint64_t)epoch << 32) | ctx_payload(S.C, ph, lane), __ATOMIC_RELAXED,
                         KIOPS_AGENT);
    if (lane == 0) __hip_atomic_store(&b->gen, epoch, __ATOMIC_RELAXED, KIOPS_AGENT);
  }
  if (ph != kPhaseDone) ctx_from_ctrl<T>(P, S.C, pctx);
  if (threadIdx.x == 0) s_phase = ph;
  __syncthreads();
}

// Barrier among the first nw workgroups of the grid only (the others are not
// waiting on it): the same arrival slots, release word and epoch sequence as
// grid_barrier, with no epilogue.  The workgroups left out add the number of
// these barriers to their epoch before the next grid barrier, so that every
// epoch agrees there.
__device__ inline void sub_barrier(const KParams& P, SmallState& S, unsigned& epoch, int nw) {
  Barrier* b = P.bar;
  ++epoch;
  __syncthreads();
  if (vblock() != 0) {
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(&P.arrive[vblock()], epoch, __ATOMIC_RELAXED, KIOPS_AGENT);
      const uint64_t t0 = (uint64_t)wall_clock64();
      for (unsigned spins = 1;; ++spins) {
        if (__hip_atomic_load(&b->gen, __ATOMIC_RELAXED, KIOPS_AGENT) == epoch) break;
        for (int z = 0; z < P.poll_sleep; ++z) __builtin_amdgcn_s_sleep(2);
        if ((spins & 63u) == 0 && spin_expired(b, t0, P.spin_limit)) break;
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return;
  }
  const uint64_t t0 = (uint64_t)wall_clock64();
  for (unsigned spins = 1;; ++spins) {
    int ok = 1;
    for (unsigned w = 1 + threadIdx.x; w < (unsigned)nw; w += kThreads)
      ok &= (__hip_atomic_load(&P.arrive[w], __ATOMIC_RELAXED, KIOPS_AGENT) == epoch) ? 1 : 0;
    if (__syncthreads_and(ok)) break;
    for (int z = 0; z < P.poll_sleep; ++z) __builtin_amdgcn_s_sleep(2);
    if ((spins & 15u) == 0) {
      if (threadIdx.x == 0) S.expired = spin_expired(b, t0, P.spin_limit) ? 1 : 0;
      __syncthreads();
      if (S.expired) break;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  __syncthreads();   // this workgroup's stage stores before thread 0's release
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(&b->gen, epoch, __ATOMIC_RELAXED, KIOPS_AGENT);
  }
  __syncthreads();
}

__device__ inline bool aborted(const KParams& P) {
  return __hip_atomic_load(&P.bar->abort, __ATOMIC_RELAXED, KIOPS_AGENT) != 0;
}

// out[d] = sum over workgroups of partials[wg][d], d < kDotSlots, in a fixed
// order (workgroup index within a thread, a fixed tree over the lanes, then
// waves).  Loads are issued four rows
// per thread at a time.
__device__ inline void reduce_partials(const KParams& P, double* out, double* lds, int rows) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  double acc[kDotSlots];
#pragma unroll
  for (int d = 0; d < kDotSlots; ++d) acc[d] = 0.0;
  int w = t;
  for (; w + 3 * kThreads < rows; w += 4 * kThreads) {
    double v[4][kDotSlots];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int d = 0; d < kDotSlots; ++d) v[u][d] = P.partials[(int64_t)(w + u * kThreads) * P.ndot_stride + d];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int d = 0; d < kDotSlots; ++d) acc[d] += v[u][d];
  }
  if (w + kThreads < rows) {   // two rows per thread (512 workgroups): all loads in flight at once
    double v[2][kDotSlots];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int d = 0; d < kDotSlots; ++d) v[u][d] = P.partials[(int64_t)(w + u * kThreads) * P.ndot_stride + d];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int d = 0; d < kDotSlots; ++d) acc[d] += v[u][d];
    w += 2 * kThreads;
  }
  for (; w < rows; w += kThreads)
#pragma unroll
    for (int d = 0; d < kDotSlots; ++d) acc[d] += P.partials[(int64_t)w * P.ndot_stride + d];
  wave_sum(acc);
  if (lane == 63) {
#pragma unroll
    for (int d = 0; d < kDotSlots; ++d) lds[wv * 16 + d] = acc[d];
  }
  __syncthreads();
  if (t < kDotSlots) {
    double s = 0.0;
    for (int q = 0; q < kThreads / 64; ++q) s += lds[q * 16 + t];
    out[t] = s;
  }
  __syncthreads();
}

// Copy the control block to device memory (all threads).
__device__ inline void publish(const KParams& P, const SmallState& S) {
  const uint64_t* src = reinterpret_cast<const uint64_t*>(&S.C);
  uint64_t* dst = reinterpret_cast<uint64_t*>(P.ctrl);
  static_assert(sizeof(Ctrl) % 8 == 0, "control block layout");
  for (int i = threadIdx.x; i < (int)(sizeof(Ctrl) / 8); i += kThreads) dst[i] = src[i];
  __syncthreads();
}

// Start of a substep (thread 0): exact trailing entries mu [T^{p-1}/(p-1)!, ..., T, 1].
__device__ inline void start_substep(const KParams& P, SmallState& S) {
  Ctrl& C = S.C;
  double* y1 = y_row(S, 1);
  const int p = C.p;
  double fact = 1.0;
#pragma unroll
  for (int c = 0; c < kPM; ++c) y1[c] = 0.0;
  for (int i = 0; i < p; ++i) {            // entry p-1-i holds T^i / i!
    if (i > 0) fact *= (double)i;
    y1[p - 1 - i] = C.mu * pow(C.T_now, (double)i) / fact;
  }
  for (int c = 0; c < kPM; ++c) {
    C.yb_cur[c] = (c < p) ? C.nu * y1[c] : 0.0;
    C.yb_prev[c] = 0.0;
    gstore(&P.Y[1 * kPM + c], y1[c]);
  }
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

// Gather coefficients for output k inside an accepted substep (Algorithm 3):
// F2 = exp(tau_k H(1:j, 1:j)) with tau_k = T_k - T_now, c_i = beta F2(i, 1) / s_i,
// and for Task I the factor (1 / T_k)^p of Algorithm 1.  Whole workgroup.
__device__ void output_coefs(const KParams& P, SmallState& S, int j, int k, double* lds) {
  Ctrl& C = S.C;
  const double tk = P.times[k] - C.T_now;
  const int n16 = pad16(j);
  double* A = P.expm;
  const bool full = C.q == 0;
  double colmax = 0.0;
  for (int c = threadIdx.x; c < n16; c += kThreads) {
    double cs = 0.0;
    for (int r = 0; r < n16; ++r) {
      const double v =
          (r < j && c < j) ? tk * (full ? P.H[(r + 1) * kLdh + (c + 1)] : h_get(S, r + 1, c + 1)) : 0.0;
      A[r * kExpmLd + c] = v;
      cs += fabs(v);
    }
    colmax = cs > colmax ? cs : colmax;
  }
  const double eta = wg_max(colmax, lds);
  const int slot = wg_expm(P.expm, j, eta, lds);
  const double* F = P.expm + (size_t)slot * kExpmSlot;
  const double scale = P.task1 ? pow(1.0 / P.times[k], (double)C.p) : 1.0;
  for (int i = 1 + threadIdx.x; i <= j; i += kThreads) C.cg[i] = scale * C.beta * F[(i - 1) * kExpmLd] * S.sinv[i];
  if (threadIdx.x == 0) C.expms += 1;
  __syncthreads();
}

// Task I: the output at T_end is scaled by (1 / T_end)^p (Algorithm 1), folded
// into the gather of the substep that reaches T_end.  Whole workgroup.
__device__ void final_scale(const KParams& P, SmallState& S, int j) {
  Ctrl& C = S.C;
  const bool last = C.T_end - (C.T_now + C.tau) <= 8.0 * 2.220446049250313e-16 * C.T_end;
  if (P.task1 && last) {
    const double scale = pow(1.0 / C.T_end, (double)C.p);
    for (int i = 1 + threadIdx.x; i <= j; i += kThreads) C.cg[i] *= scale;
  }
  __syncthreads();
}

// After the coefficients of an accepted substep are known: the output times
// T_k (k >= l, not the last) with T_k < T_now + tau are written first, each
// by its own gather (Algorithm 3); the substep's own gather, whose
// coefficients are kept in device memory meanwhile, comes last.
__device__ void begin_outputs(const KParams& P, SmallState& S, int j, double* lds) {
  Ctrl& C = S.C;
  if (threadIdx.x == 0) {
    const double tnext = C.T_now + C.tau;
    int n = 0;
    for (int k = C.out_next; k < P.ntimes - 1; ++k)
      if (P.times[k] < tnext) ++n;
    C.pending = n;
    C.gather_to = -1;
  }
  __syncthreads();
  if (C.pending > 0) {
    for (int i = threadIdx.x; i <= j; i += kThreads) P.cgsave[i] = C.cg[i];
    __syncthreads();
    output_coefs(P, S, j, C.out_next, lds);
    if (threadIdx.x == 0) C.gather_to = C.out_next;
    __syncthreads();
  } else {
    final_scale(P, S, j);
  }
}

// Error estimate of an attempt with basis size j (Section 3.4) from F =
// exp(tau H~): the first term of Eq. (35), which is Eq. (36), or (with the
// extra row and column of the two-term exponential, F(j, j+2) =
// tau^2 e_j^T phi_2(tau H_j) e_1) the first two terms or the second alone.
// v_{j+1} is the latest normalised vector: est_c = <v, A~ v>, est_u = ||A~ v||^2.
__device__ inline double attempt_estimate(const Ctrl& C, double h, const double* F, int j) {
  const double a = F[(j - 1) * kExpmLd + j];
  if (C.estimate == KIOPS_ESTIMATE_ONE_TERM) return C.beta * fabs(h) * fabs(a);
  const double b = F[(j - 1) * kExpmLd + j + 1];
  const double u = C.est_u > 0.0 ? C.est_u : 0.0;
  if (C.estimate == KIOPS_ESTIMATE_CORRECTED) return C.beta * fabs(h) * fabs(b) * sqrt(u);
  const double q2 = a * a + 2.0 * a * b * C.est_c + b * b * u;   // ||a v + b A~ v||^2
  return C.beta * fabs(h) * sqrt(q2 > 0.0 ? q2 : 0.0);
}

// Decision for an attempt with basis size j whose exponential F = exp(tau H~)
// is in slot `slot` of the scratch: eps (Section 3.4), Algorithm 4, and on
// acceptance the gather coefficients.  Whole workgroup.  Returns true when
// the attempt is to be repeated on the same basis with a smaller tau
// (rejection at m_max).
__device__ bool attempt_decide(const KParams& P, SmallState& S, int j, bool breakdown, int slot, double* lds) {
  Ctrl& C = S.C;
  const double* F = P.expm + (size_t)slot * kExpmSlot;
  if (threadIdx.x == 0) {
    const double tau = C.tau;
    const double eps = breakdown ? 0.0 : attempt_estimate(C, h_get(S, j + 1, j), F, j);
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
        if (C.e_round >= 1000 || !(o.tau_new > 0.0)) {   // step size collapsed: give up
          C.status = KIOPS_ERR_NOT_CONVERGED;
          C.phase = kPhaseDone;
          again = 0;
        }
      } else {
        C.m = o.m_new;
        C.phase = kPhasePass;
      }
    }
    C.e_round += 1;
    S.again = again;
  }
  __syncthreads();
  if (C.phase == kPhaseGather) {
    // gather coefficients c_i = beta F(i, 1) / s_{i-1}
    for (int i = 1 + threadIdx.x; i <= j; i += kThreads) C.cg[i] = C.beta * F[(i - 1) * kExpmLd] * S.sinv[i];
    if (threadIdx.x == 0 && C.estimate == KIOPS_ESTIMATE_CORRECTED && !breakdown) {
      // corrected scheme: + beta h_{j+1,j} (tau e_j^T phi_1(tau H_j) e_1) v_{j+1}
      C.cg[j + 1] = C.beta * h_get(S, j + 1, j) * F[(j - 1) * kExpmLd + j] * S.sinv[j + 1];
      C.jg = j + 1;
    }
    __syncthreads();
    begin_outputs(P, S, C.jg, lds);
  }
  return S.again != 0;
}

// Exponentials of the attempt (X = tau H~ of Eq. (37)) and their decisions,
// until the attempt is decided or an exponential is handed to the whole grid
// (phase kPhaseExpm, continued by epilogue_expm).  Whole workgroup.
__device__ void attempt_run(const KParams& P, SmallState& S, int j, bool breakdown, double* lds) {
  Ctrl& C = S.C;
  const int extra = C.estimate != KIOPS_ESTIMATE_ONE_TERM ? 1 : 0;   // the phi_2 column of the two-term estimate
  const int n = j + 1 + extra;
  const int n16 = pad16(n);
  for (;;) {
    const double tau = C.tau;
    // X = tau H~ (Eq. (37)) by columns, with its 1-norm; with the extra row
    // and column, tau [[H, e_1, 0], [0, 0, 1], [0, 0, 0]] (Theorem 1 on H)
    double* A = P.expm;
    const bool full = C.q == 0;   // full window: H in device memory, else the band in LDS
    double colmax = 0.0;
    for (int c = threadIdx.x; c < n16; c += kThreads) {
      double cs = 0.0;
      for (int r = 0; r < n16; ++r) {
        double v = 0.0;
        if (r < j && c < j) v = tau * (full ? P.H[(r + 1) * kLdh + (c + 1)] : h_get(S, r + 1, c + 1));
        else if (c == j && r == 0) v = tau;
        else if (extra && r == j && c == j + 1) v = tau;
        A[r * kExpmLd + c] = v;
        cs += fabs(v);
      }
      colmax = cs > colmax ? cs : colmax;
    }
    const double eta = wg_max(colmax, lds);
    if (P.expm_grid > 0 && P.nwg > 1 && n16 >= P.expm_grid) {
      if (threadIdx.x == 0) {
        int d, s;
        expm_plan(eta, d, s);
        C.e_j = j;
        C.e_bd = breakdown ? 1 : 0;
        C.e_d = d;
        C.e_s = s;
        C.e_alpha = ldexp(1.0, -s);
        C.e_nst = expm_stages(d, s);
        C.phase = kPhaseExpm;
      }
      __syncthreads();
      return;
    }
    const int slot = wg_expm(P.expm, n, eta, lds);
    if (!attempt_decide(P, S, j, breakdown, slot, lds)) break;
  }
  if (threadIdx.x == 0) C.t_expm += (uint64_t)wall_clock64() - C.e_t0;
}

// The small exponential and the controller for an attempt with basis size j.
// Whole workgroup.  Repeats while the attempt is rejected at m_max (same
// basis, smaller tau).
__device__ __noinline__ void attempt_end(const KParams& P, SmallState& S, int j, bool breakdown,
                                         double* lds) {
  if (threadIdx.x == 0) {
    S.C.e_round = 0;
    S.C.e_t0 = (uint64_t)wall_clock64();
  }
  __syncthreads();
  attempt_run(P, S, j, breakdown, lds);
}

// Epilogue after a grid-wide small exponential: the attempt's decision, and
// the next exponential if the attempt is repeated with a smaller tau.
__device__ __noinline__ void epilogue_expm(const KParams& P, SmallState& S, double* lds) {
  Ctrl& C = S.C;
  const int j = C.e_j;
  const bool breakdown = C.e_bd != 0;
  if (attempt_decide(P, S, j, breakdown, expm_result_slot(C.e_d, C.e_s), lds)) {
    attempt_run(P, S, j, breakdown, lds);
  } else if (threadIdx.x == 0) {
    C.t_expm += (uint64_t)wall_clock64() - C.e_t0;
  }
  __syncthreads();
  publish(P, S);
}

// Workgroups that compute a grid-wide exponential of padded size n16: one
// tile of a product per wave (the stage of X^3 and X^4 has two).
__device__ __forceinline__ int expm_participants(int n16, int nwg) {
  const int nt = n16 >> 4;
  const int want = (nt * nt + 3) / 4;
  return want < nwg ? want : nwg;
}

// A grid-wide small exponential: its stages run on the first workgroups of the
// grid, separated by barriers among them; the others go straight to the grid
// barrier that ends the phase.
template <typename T, class F>
__device__ inline void expm_phase(const KParams& P, SmallState& S, unsigned& epoch, double* lds, PassCtx<T>& pctx,
                                  int& s_phase, F&& epi) {
  const Ctrl& C = *P.ctrl;
  const int n = uniform(C.e_j) + 1 + (uniform(C.estimate) != KIOPS_ESTIMATE_ONE_TERM ? 1 : 0);
  const int d = uniform(C.e_d), s = uniform(C.e_s), nst = uniform(C.e_nst);
  const double alpha = uniform(C.e_alpha);
  const int npart = expm_participants(pad16(n), P.nwg);
  if (vblock() < npart) {
    for (int st = 0; st < nst; ++st) {
      grid_expm_stage(P.expm, n, d, s, alpha, st, vblock(), npart, lds);
      if (st + 1 < nst) sub_barrier(P, S, epoch, npart);
    }
  } else {
    epoch += (unsigned)(nst - 1);
  }
  grid_barrier(P, S, epoch, pctx, s_phase, epi);
}

// Epilogue after the setup phase.
__device__ __noinline__ void epilogue_setup(const KParams& P, SmallState& S, double* lds) {
  reduce_partials(P, S.red, lds, P.nwg);
  for (int e = threadIdx.x; e < kLdh * (kWinMax + 1); e += kThreads) (&S.Hb[0][0])[e] = 0.0;
  for (int e = threadIdx.x; e < kRingRows * kWinMax; e += kThreads) (&S.Gw[0][0])[e] = 0.0;
  for (int e = threadIdx.x; e < kLdh; e += kThreads) S.sinv[e] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    Ctrl& C = S.C;
    double nb = 0.0;
    for (int k = 0; k < P.p; ++k) nb = S.red[k] > nb ? S.red[k] : nb;
    double nu = 1.0, mu = 1.0;
    if (P.p > 0 && nb > 0.0 && isfinite(nb)) {
      int e;
      const double f = frexp(nb, &e);          // nb = f 2^e, f in [0.5, 1)
      const int c = (f == 0.5) ? e - 1 : e;    // ceil(log2 nb)
      nu = ldexp(1.0, -c);
      mu = ldexp(1.0, c);
    }
    const uint64_t tw = C.t_work, tl = C.t_last, tb = C.t_begin;
    C = Ctrl{};
    C.t_work = tw;
    C.t_last = tl;
    C.t_begin = tb;
    C.nu = nu; C.mu = mu;
    C.gather_to = -1;
    C.T_now = 0.0; C.T_end = P.T_end; C.tau = P.T_end; C.tol = P.tol;
    C.p = P.p; C.q = P.q; C.m_min = P.m_min; C.m_max = P.m_max; C.max_substeps = P.max_substeps;
    int m = P.m_init < P.m_max ? P.m_init : P.m_max;   // Alg. 1: initial dimension
    C.m = m > P.m_min ? m : P.m_min;
    C.m_new = C.m;
    C.status = KIOPS_OK;
    C.mode = P.mode;
    C.estimate = P.estimate;
    C.alg_bytes = (double)P.p * 8.0 * (double)P.N;   // ||B||_1
    if (!isfinite(nb)) {
      C.status = KIOPS_ERR_NONFINITE;
      C.phase = kPhaseDone;
    } else if (P.T_end == 0.0) {
      C.phase = kPhaseDone;
    } else {
      start_substep(P, S);
    }
  }
  __syncthreads();
  publish(P, S);
}

// Normalisation of R_k after pass k (thread 0): its norm over N + p entries is
// s_{k-1} = h_{k,k-1}.  Returns -1 to continue with the orthogonalisation,
// else the action: 2 breakdown (end the attempt), 3 done.
__device__ inline int step_normalise(const KParams& P, SmallState& S, int k, double* ykr, double* Ky,
                                     double& Ck_out, double& si_out) {
  Ctrl& C = S.C;
  const int p = C.p;
  const double* red = S.red;
  if (C.q == 0) {   // two loops, so that the windowed form reads LDS directly
#pragma unroll
    for (int c = 0; c < kPM; ++c) ykr[c] = P.Y[k * kPM + c];
  } else {
    const double* yk = y_row(S, k);
#pragma unroll
    for (int c = 0; c < kPM; ++c) ykr[c] = yk[c];
  }
#pragma unroll
  for (int c = 0; c < kPM; ++c) Ky[c] = (c + 1 < kPM && c + 1 < p) ? ykr[c + 1] : 0.0;   // K y
  double RR = red[kDotRR], UU = red[kDotUU], Ck = red[kDotCk];
#pragma unroll
  for (int c = 0; c < kPM; ++c) { RR += ykr[c] * ykr[c]; UU += Ky[c] * Ky[c]; Ck += ykr[c] * Ky[c]; }
  C.matvecs += 1;
  C.alg_bytes += pass_bytes(P, k, C.flo);
  bool finite = isfinite(RR) && isfinite(UU) && isfinite(Ck);
  for (int d = 0; d < k - C.dlo; ++d) finite = finite && isfinite(red[kDotG + d]) && isfinite(red[kDotC + d]);
  const double s = sqrt(RR);
  if (!finite) {
    C.status = KIOPS_ERR_NONFINITE;
    C.phase = kPhaseDone;
    return 3;
  }
  if (k == 1 && s == 0.0) {
    C.beta = 0.0;                             // zero start vector: w stays zero
    C.T_now = C.T_end;
    C.phase = kPhaseDone;
    return 3;
  }
  if (k > 1 && (s == 0.0 || s <= 1e-12 * S.unorm_prev)) {
    h_set(S, P, k, k - 1, 0.0);               // happy breakdown (Alg. 2)
    C.breakdown = 1;
    C.s_last = s;
    const int action = (C.mode == kModeBasis) ? 3 : 2;
    if (action == 3) C.phase = kPhaseDone;
    return action;
  }
  if (k == 1) C.beta = s;
  else h_set(S, P, k, k - 1, s);
  C.s_last = s;
  const double si = 1.0 / s;
  S.sinv[k] = si;
  gstore(&P.sinv[k], si);
  S.unorm_prev = sqrt(UU) * si;
  C.est_c = Ck * si * si;                     // <v_k, A~ v_k>
  C.est_u = UU * si * si;                     // ||A~ v_k||^2
  Ck_out = Ck;
  si_out = si;
  return -1;
}

// Next pass and the attempt bookkeeping once column k of H is known (thread 0).
__device__ inline int step_advance(SmallState& S, int k, int flo_next) {
  Ctrl& C = S.C;
  int action = 0;
  C.flo = flo_next;
  C.kp = k + 1;
  C.dlo = (C.q == 0) ? k + 1 : ((k + 1 - C.q + 1) > 1 ? (k + 1 - C.q + 1) : 1);
  const int jdone = k - 1;
  if (C.mode == kModeBasis) {
    if (jdone >= C.m) { C.phase = kPhaseDone; action = 3; }
  } else if (jdone >= C.m && jdone >= 1) {
    action = 1;
  }
  if (action != 3) C.phase = kPhasePass;
  return action;
}

// Epilogue after pass kp: Algorithm 2's normalisation of R_kp, the window
// coefficients h_{i,kp} by modified Gram-Schmidt of Algorithm 2 reproduced
// from the inner products, the coefficients of the next pass, and the end of
// an attempt.  With a full window (q = 0) the inner products with the older
// vectors come from a separate phase first (epilogue_dots).
__device__ __noinline__ void epilogue_pass(const KParams& P, SmallState& S, double* lds) {
  Ctrl& C = S.C;
  const uint64_t tr0 = P.profile ? (uint64_t)wall_clock64() : 0;
  reduce_partials(P, S.red, lds, P.nwg);
  if (P.profile && threadIdx.x == 0) C.t_red += (uint64_t)wall_clock64() - tr0;
  if (C.q == 0 && C.kp > 1) {                 // full window: inner products first
    if (threadIdx.x == 0) C.phase = kPhaseDots;
    __syncthreads();
    publish(P, S);
    return;
  }
  const uint64_t ts0 = P.profile ? (uint64_t)wall_clock64() : 0;
  if (threadIdx.x == 0) {
    const int k = C.kp;
    const int dlo = C.dlo;
    const int p = C.p;
    const double* red = S.red;
    double ykr[kPM], Ky[kPM], Ck = 0.0, si = 0.0;
    S.nx_go = 0;
    int action = step_normalise(P, S, k, ykr, Ky, Ck, si);
    if (action < 0) {
      const int ngd = k - dlo;
      double* gk = S.Gw[k % kRingRows];
#pragma unroll
      for (int d = 0; d < kWinMax; ++d) gk[d] = 0.0;
      gk[kWinMax - 1] = 1.0;                    // G(k, k)
      for (int d = 0; d < ngd; ++d) {
        const int i = dlo + d;
        const double* yi = y_row(S, i);
        double yd = 0.0;
#pragma unroll
        for (int c = 0; c < kPM; ++c) yd += yi[c] * ykr[c];
        gk[i - (k - kWinMax + 1)] = (red[kDotG + d] + yd) * S.sinv[i] * si;
      }
      // modified Gram-Schmidt over the window [dlo, k] (Alg. 2)
      double hk[kWinMax];
      for (int i = dlo; i <= k; ++i) {
        double raw;
        if (i < k) {
          const double* yi = y_row(S, i);
          double yd = 0.0;
#pragma unroll
          for (int c = 0; c < kPM; ++c) yd += yi[c] * Ky[c];
          raw = red[kDotC + (i - dlo)] + yd;
        } else {
          raw = Ck;
        }
        double h = raw * S.sinv[i] * si;
        for (int l = dlo; l < i; ++l) h -= hk[l - dlo] * g_get(S, i, l);
        hk[i - dlo] = h;
        h_set(S, P, i, k, h);
      }
      // coefficients of the next pass: R_{k+1} = si U_k - sum_i H(i,k) sinv[i] R_i;
      // the y-parts (one entry per lane below) and a, bw here
      S.nx_si = si;
      S.nx_k = k;
      S.nx_dlo = dlo;
      S.nx_p = p;
#pragma unroll
      for (int d = 0; d < kWinMax; ++d) S.nx_hk[d] = d <= k - dlo ? hk[d] : 0.0;
#pragma unroll
      for (int c = 0; c < kPM; ++c) {
        S.nx_ky[c] = Ky[c];
        S.nx_ykr[c] = ykr[c];
      }
      S.nx_go = 1;
      C.a = si;
      for (int i = dlo; i <= k; ++i) C.bw[i] = -hk[i - dlo] * S.sinv[i];
      action = step_advance(S, k, dlo);
    }
    S.action = action;
    S.jj = k - 1;
  }
  __syncthreads();
  if (S.nx_go) {   // entry c of the y-parts: the same operations as a loop over c would do
    const int c = threadIdx.x;
    if (c < kPM) {
      const int k = S.nx_k, dlo = S.nx_dlo, p = S.nx_p;
      double v = (c < p) ? S.nx_si * S.nx_ky[c] : 0.0;
      if (c < p)
        for (int i = dlo; i <= k; ++i) v -= S.nx_hk[i - dlo] * S.sinv[i] * y_row(S, i)[c];
      const double yv = (c < p) ? v : 0.0;
      y_row(S, k + 1)[c] = yv;
      gstore(&P.Y[(k + 1) * kPM + c], yv);
      C.yb_prev[c] = (c < p) ? C.nu * S.nx_ykr[c] : 0.0;
      C.yb_cur[c] = (c < p) ? C.nu * v : 0.0;
    }
    __syncthreads();
  }
  if (P.profile && threadIdx.x == 0) C.t_ser += (uint64_t)wall_clock64() - ts0;
  const int action = S.action;
  if (action == 1 || action == 2) attempt_end(P, S, S.jj, action == 2, lds);
  const uint64_t tp0 = P.profile ? (uint64_t)wall_clock64() : 0;
  publish(P, S);
  if (P.profile && threadIdx.x == 0) S.C.t_pub += (uint64_t)wall_clock64() - tp0;
}

// Epilogue after the inner-product phase of a full-window step (q = 0): the
// orthogonalisation of A~ v_k against every earlier v_i by classical
// Gram-Schmidt with a Gram-matrix correction, from one set of inner products:
// with c_i = <v_i, A~ v_k> and the Gram matrix G of v_1..v_k,
// h = c + (c - G c) (what a second Gram-Schmidt pass would add if the
// basis's own loss of orthogonality, I - G, were the only error; it is not a
// second pass over fresh inner products).  G and c live in device memory (P.G,
// P.fullc); the sums over i run on all threads.
__device__ __noinline__ void epilogue_dots(const KParams& P, SmallState& S, double* lds) {
  Ctrl& C = S.C;
  const int k = C.kp;
  // x-parts of <R_i, R_k> and <R_i, U_k>, i < k: fixed-order sum over workgroups
  for (int i = 1 + (int)threadIdx.x; i < k; i += kThreads) {
    double g = 0.0, c = 0.0;
    for (int w = 0; w < P.nwg; ++w) {
      g += P.dpart[(int64_t)w * kDotFullStride + 2 * i];
      c += P.dpart[(int64_t)w * kDotFullStride + 2 * i + 1];
    }
    P.fullc[2 * i] = g;
    P.fullc[2 * i + 1] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ykr[kPM], Ky[kPM], Ck = 0.0, si = 0.0;
    const int action = step_normalise(P, S, k, ykr, Ky, Ck, si);
    for (int c = 0; c < kPM; ++c) { S.fy[c] = ykr[c]; S.fky[c] = Ky[c]; }
    S.fsi = si;
    S.fck = Ck;
    S.action = action;
    S.jj = k - 1;
  }
  __syncthreads();
  if (S.action < 0) {
    const double si = S.fsi;
    // G(k, i) and c_i with the trailing parts, for i < k
    for (int i = 1 + (int)threadIdx.x; i < k; i += kThreads) {
      const double* yi = P.Y + i * kPM;
      double yg = 0.0, yc = 0.0;
#pragma unroll
      for (int c = 0; c < kPM; ++c) { yg += yi[c] * S.fy[c]; yc += yi[c] * S.fky[c]; }
      const double g = (P.fullc[2 * i] + yg) * S.sinv[i] * si;
      P.G[k * kLdh + i] = g;
      P.G[i * kLdh + k] = g;
      P.coefc[i] = (P.fullc[2 * i + 1] + yc) * S.sinv[i] * si;   // c_i
    }
    if (threadIdx.x == 0) P.coefc[k] = S.fck * si * si;
    __syncthreads();
    // h_i = 2 c_i - (G c)_i, i <= k
    for (int i = 1 + (int)threadIdx.x; i <= k; i += kThreads) {
      double gc = 0.0;
      for (int l = 1; l <= k; ++l) gc += (l == i ? 1.0 : P.G[i * kLdh + l]) * P.coefc[l];
      lds[i] = 2.0 * P.coefc[i] - gc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const int p = C.p;
      for (int i = 1; i <= k; ++i) h_set(S, P, i, k, lds[i]);
      for (int c = 0; c < kPM; ++c) {
        double v = (c < p) ? si * S.fky[c] : 0.0;
        if (c < p)
          for (int i = 1; i <= k; ++i) v -= lds[i] * S.sinv[i] * P.Y[i * kPM + c];
        const double yn = (c < p) ? v : 0.0;
        P.Y[(k + 1) * kPM + c] = yn;
        y_row(S, k + 1)[c] = yn;
        C.yb_prev[c] = (c < p) ? C.nu * S.fy[c] : 0.0;
        C.yb_cur[c] = (c < p) ? C.nu * v : 0.0;
      }
      C.a = si;
      for (int i = 1; i <= k; ++i) C.bw[i] = -lds[i] * S.sinv[i];
      S.action = step_advance(S, k, 1);
    }
    __syncthreads();
  }
  const int action = S.action;
  if (action == 1 || action == 2) attempt_end(P, S, S.jj, action == 2, lds);
  const uint64_t tp0 = P.profile ? (uint64_t)wall_clock64() : 0;
  publish(P, S);
  if (P.profile && threadIdx.x == 0) S.C.t_pub += (uint64_t)wall_clock64() - tp0;
}

// Epilogue after the gather: advance T_now (Alg. 1) and start the next substep.
__device__ __noinline__ void epilogue_gather(const KParams& P, SmallState& S, double* lds) {
  if (S.C.gather_to >= 0) {   // an intermediate output was written (Algorithm 3)
    if (threadIdx.x == 0) {
      Ctrl& C = S.C;
      C.alg_bytes += (8.0 + P.elem_bytes * (double)(C.jg - 1) + 8.0) * (double)P.N;
      C.out_next = C.gather_to + 1;
      C.pending -= 1;
    }
    __syncthreads();
    if (S.C.pending > 0) {
      output_coefs(P, S, S.C.jg, S.C.out_next, lds);
      if (threadIdx.x == 0) S.C.gather_to = S.C.out_next;
    } else {
      for (int i = threadIdx.x; i <= S.C.jg; i += kThreads) S.C.cg[i] = P.cgsave[i];
      __syncthreads();
      if (threadIdx.x == 0) S.C.gather_to = -1;
      final_scale(P, S, S.C.jg);
    }
    __syncthreads();
    publish(P, S);
    return;
  }
  if (threadIdx.x == 0) {
    Ctrl& C = S.C;
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
      C.out_next = P.ntimes;
    } else if (C.substeps >= C.max_substeps) {
      C.status = KIOPS_ERR_NOT_CONVERGED;
      C.phase = kPhaseDone;
    } else {
      start_substep(P, S);
    }
  }
  __syncthreads();
  publish(P, S);
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
  block_sum(packed, lds, P.partials + (int64_t)vblock() * P.ndot_stride);
}

template <class Op, typename T>
__device__ inline void setup_phase(const KParams& P, const Op& op, T* bcopy, double* lds) {
  const int64_t gt = (int64_t)vblock() * kThreads + threadIdx.x;
  const int64_t gs = (int64_t)vgrid() * kThreads;
  for (int64_t e = gt; e < (int64_t)kLdh * kLdh; e += gs) { P.H[e] = 0.0; P.G[e] = 0.0; }
  double sums[kDotSlots];
#pragma unroll
  for (int k = 0; k < kDotSlots; ++k) sums[k] = 0.0;
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
  block_sum(sums, lds, P.partials + (int64_t)vblock() * P.ndot_stride);
}

// Gather w <- sum_i cg[i] R_i (R_1 = w).
template <typename T>
__device__ inline void gather_phase(const KParams& P, const BasisPtrs<T>& bp, double* lds) {
  const Ctrl& C = *P.ctrl;
  const int jg = C.jg;
  double* out = C.gather_to >= 0 ? P.wout[C.gather_to] : P.w;   // an output time, or the state
  for (int i = threadIdx.x; i <= jg; i += kThreads) lds[i] = C.cg[i];
  __syncthreads();
  const int64_t gt = (int64_t)vblock() * kThreads + threadIdx.x;
  const int64_t gs = (int64_t)vgrid() * kThreads;
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
    out[n] = acc;
  }
  __syncthreads();
}

// Inner products of R_kp and U_kp (the latest pass) with every earlier basis
// vector R_i, i < kp (full window).  Workgroup w owns elements
// [N w / nwg, N (w+1) / nwg); a thread holds 16 elements of R_kp and U_kp at a
// time and streams each R_i over them; wave sums accumulate in LDS per i and
// are written as the workgroup's partials (fixed order).
template <typename T>
__device__ inline void dots_phase(const KParams& P, const BasisPtrs<T>& bp, double* lds) {
  constexpr int E = 16;
  const int kp = P.ctrl->kp;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t n0 = P.N * vblock() / vgrid(), n1 = P.N * (vblock() + 1) / vgrid();
  const T* U = reinterpret_cast<const T*>(P.ubuf);
  const T* Rk = bp.get(kp);
  double* acc = lds;                          // [kLdh][4 waves][2]
  for (int e = t; e < kLdh * 8; e += kThreads) acc[e] = 0.0;
  __syncthreads();
  for (int64_t c0 = n0; c0 < n1; c0 += (int64_t)E * kThreads) {
    double xr[E], xu[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int64_t n = c0 + t + (int64_t)e * kThreads;
      const bool in = n < n1;
      xr[e] = in ? (double)Rk[n] : 0.0;
      xu[e] = in ? (double)U[n] : 0.0;
    }
    for (int i = 1; i < kp; ++i) {
      const T* Ri = bp.get(i);
      double g = 0.0, u = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int64_t n = c0 + t + (int64_t)e * kThreads;
        const double r = n < n1 ? (double)Ri[n] : 0.0;
        g = fma(r, xr[e], g);
        u = fma(r, xu[e], u);
      }
      for (int off = 32; off > 0; off >>= 1) {
        g += __shfl_xor(g, off, 64);
        u += __shfl_xor(u, off, 64);
      }
      if (lane == 0) {
        acc[i * 8 + wv * 2] += g;
        acc[i * 8 + wv * 2 + 1] += u;
      }
    }
  }
  __syncthreads();
  double* out = P.dpart + (int64_t)vblock() * kDotFullStride;
  for (int e = t; e < 2 * kp; e += kThreads) {
    const int i = e >> 1, j = e & 1;
    double v = 0.0;
    if (i >= 1 && i < kp)
      for (int q = 0; q < kThreads / 64; ++q) v += acc[i * 8 + q * 2 + j];
    out[e] = v;
  }
  __syncthreads();
}

// Entry e of a group queue: e once the host has published it, or -1 when the
// queue is closed (and drained) or nothing came within its idle limit.  Called
// by the whole first wave with wave-uniform values (one loop exit, one result).
// kScope is the scope of the tail's acquire: the agent when the queue was
// filled before the launch, the system when the host fills it while the
// launch runs (a fine-grained queue).
template <int kScope = KIOPS_AGENT>
__device__ inline long long wait_entry(GroupQueue& Q, unsigned e) {
  const uint64_t t0 = (uint64_t)wall_clock64();
  long long result = -2;
  while (result == -2) {
    const unsigned tail = __builtin_amdgcn_readfirstlane(__hip_atomic_load(&Q.tail, __ATOMIC_ACQUIRE, kScope));
    const unsigned closed =
        __builtin_amdgcn_readfirstlane(__hip_atomic_load(&Q.closed, __ATOMIC_RELAXED, kScope));
    const bool idle = (uint64_t)wall_clock64() - t0 > Q.idle_limit;
    if (tail > e) {
      result = e;
    } else if (closed || idle) {
      if (threadIdx.x == 0) {
        __hip_atomic_store(&Q.exit_reason, closed ? 1u : 2u, __ATOMIC_RELAXED, KIOPS_AGENT);
        __hip_atomic_store(&Q.exit_entry, e, __ATOMIC_RELAXED, KIOPS_AGENT);
      }
      result = -1;
    } else {
      for (unsigned z = 0; z < Q.idle_sleep; ++z) __builtin_amdgcn_s_sleep(127);
      __builtin_amdgcn_s_sleep(8);
    }
  }
  if (result >= 0) __threadfence();
  return result;
}

// One solve (Algorithm 1) on the workgroups of the current virtual grid.
// `epoch` is the grid-barrier epoch of this group of workgroups; it keeps
// counting across the solves a group runs one after another.
template <class Op, typename T>
__device__ inline void solve_instance(const KParams& P, const Op& op, SmallState& S, PassCtx<T>& pctx,
                                      double* lds, int& s_phase, unsigned& epoch) {
  T* bcopy = reinterpret_cast<T*>(P.bcopy);
  BasisPtrs<T> bp;
  bp.R1 = P.mixed ? reinterpret_cast<const T*>(P.slots) : reinterpret_cast<const T*>(P.w);
  bp.slots = reinterpret_cast<T*>(P.slots);
  bp.N = P.N;
  if (vblock() == 0 && threadIdx.x == 0) {
    S.C.t_work = S.C.t_wait = S.C.t_epi = 0;
    S.C.t_expm = S.C.t_arrive_max = S.C.t_arrive_mean = S.C.n_barriers = 0;
    S.C.t_release_max = S.C.t_release_mean = 0;
    S.C.t_red = S.C.t_pub = S.C.t_ser = 0;
    S.C.t_last = (uint64_t)wall_clock64();
    S.C.t_begin = S.C.t_last;
  }

  if (vblock() == 0) {   // workgroup 0's copy of the parameter block (ordered by the barrier below)
    static_assert(sizeof(KParams) % 8 == 0, "parameter block layout");
    const uint64_t* src = reinterpret_cast<const uint64_t*>(&P);
    uint64_t* dst = reinterpret_cast<uint64_t*>(&S.P);
    for (int i = threadIdx.x; i < (int)(sizeof(KParams) / 8); i += kThreads) dst[i] = src[i];
  }
  const KParams& Pe = S.P;   // the epilogues run on workgroup 0 only

  setup_phase<Op, T>(P, op, bcopy, lds);
  grid_barrier(P, S, epoch, pctx, s_phase, [&] { epilogue_setup(Pe, S, lds); });

  for (;;) {
    // each grid barrier leaves the next phase in s_phase and, for a pass,
    // its context in pctx
    const int phase = s_phase;
    if (phase == kPhaseDone) break;
    if (phase == kPhasePass) {
      DotAcc acc;
      acc.zero();
      T* Rout = bp.get_mut(pctx.kp);
      if constexpr (Op::kTwoPhase) {
        op.form(pctx, bp, P.w, Rout);
        grid_barrier(P, S, epoch, pctx, s_phase, [] {});   // R_kp complete before the product reads it
        op.matvec(pctx, bp, Rout, acc);
      } else {
        op.pass(pctx, bp, P.w, Rout, acc, reinterpret_cast<T*>(lds));
      }
      store_partials(P, acc, lds);
      grid_barrier<!Op::kTwoPhase>(P, S, epoch, pctx, s_phase, [&] { epilogue_pass(Pe, S, lds); });
    } else if (phase == kPhaseDots) {
      dots_phase<T>(P, bp, lds);
      grid_barrier(P, S, epoch, pctx, s_phase, [&] { epilogue_dots(Pe, S, lds); });
    } else if (phase == kPhaseExpm) {
      expm_phase(P, S, epoch, lds, pctx, s_phase, [&] { epilogue_expm(Pe, S, lds); });
    } else {
      gather_phase<T>(P, bp, lds);
      grid_barrier(P, S, epoch, pctx, s_phase, [&] { epilogue_gather(Pe, S, lds); });
    }
  }
}

// One solve on the whole grid.  Parameters live in device memory (written by
// the host before the launch) so that no by-value kernel argument has its
// address taken.
template <class Op, typename T>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(Op::kWavesPerEU, 8)))
kiops_solve_kernel(const KParams* __restrict__ Pp, const Op* __restrict__ opp) {
  // pass tiles (size set by the operator) / small-exponential and reduction staging
  constexpr int kLds = Op::kLdsDoubles > kLdsDoubles ? Op::kLdsDoubles : kLdsDoubles;
  __shared__ double lds[kLds];
  __shared__ PassCtx<T> pctx;
  __shared__ SmallState S;       // used by workgroup 0 only
  __shared__ int s_phase;
  set_vgrid((int)blockIdx.x, (int)gridDim.x);
  unsigned epoch = 0;
  solve_instance<Op, T>(*Pp, *opp, S, pctx, lds, s_phase, epoch);
}

// A solve whose parameter block and operator struct are read-only for its
// whole duration (restrict, kept through inlining), so that their fields can
// stay in scalar registers across the stores of the passes.
template <class Op, typename T>
__device__ __forceinline__ void solve_block(const KParams* __restrict__ Pp, const Op* __restrict__ opp,
                                            SmallState& S, PassCtx<T>& pctx, double* lds, int& s_phase,
                                            unsigned& epoch) {
  const Op op = load_uniform(opp);   // operator fields in scalar registers for the passes
  solve_instance<Op, T>(*Pp, op, S, pctx, lds, s_phase, epoch);
}

// Groups of workgroups, each running the solves queued for it one after
// another (batched form).  Group g is workgroups [wg0, wg0 + gsize) of its
// queue (wg_group[b] names the group of workgroup b); its queue lists parameter blocks
// (KParams, operator struct at +2048) that the host prepared for that group's
// workspace.  A group waits for entry e until the host has published it
// (queue tail > e) or has closed the queue; it reports entry e done by
// storing e + 1 into `done`.  Waiting is bounded by the queue's idle limit.
template <class Op, typename T>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(Op::kWavesPerEU, 8)))
kiops_group_kernel(GroupQueue* __restrict__ queues, const int* __restrict__ wg_group) {
  constexpr int kLds = Op::kLdsDoubles > kLdsDoubles ? Op::kLdsDoubles : kLdsDoubles;
  __shared__ double lds[kLds];
  __shared__ PassCtx<T> pctx;
  __shared__ SmallState S;
  __shared__ int s_phase;
  __shared__ long long s_entry;
  // groups are contiguous runs of workgroups of different sizes (a large
  // problem gets a larger group); wg_group maps a workgroup to its group
  const int g = uniform(wg_group[blockIdx.x]);
  GroupQueue& Q = queues[g];
  set_vgrid((int)blockIdx.x - uniform(Q.wg0), uniform(Q.gsize));
  unsigned epoch = 0;
  for (unsigned e = 0;; ++e) {
    if (threadIdx.x < 64) {
      const long long r = wait_entry(Q, e);
      if (threadIdx.x == 0) s_entry = r;
    }
    __syncthreads();
    const long long entry = s_entry;
    __syncthreads();
    if (entry < 0) {
      if (vblock() == 0 && threadIdx.x == 0) __hip_atomic_store(&Q.exited, 1u, __ATOMIC_RELEASE, KIOPS_AGENT);
      return;
    }
    // the block pointer is wave-uniform (made explicit, so that the block's
    // fields are read with scalar loads and buffer resources stay scalar)
    const unsigned char* blk = uniform(Q.blocks[uniform((int)(entry % kGroupQueueLen))]);
    solve_block<Op, T>(reinterpret_cast<const KParams*>(blk), reinterpret_cast<const Op*>(blk + 2048), S, pctx,
                       lds, s_phase, epoch);
    if (vblock() == 0 && threadIdx.x == 0) {
      __threadfence();
      __hip_atomic_store(&Q.done, e + 1, __ATOMIC_RELEASE, KIOPS_AGENT);
    }
  }
}

}  // namespace kiops
