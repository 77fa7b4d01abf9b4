// Device-side state shared by the persistent KIOPS solver kernels.
//
// One solve is one cooperative launch.  Every workgroup runs the same loop of
// phases separated by grid-wide barriers; the last workgroup to reach a
// barrier runs a serial "epilogue" (reductions, the Hessenberg bookkeeping of
// Algorithm 2, the small exponential of Section 3.3.1, the controller of
// Algorithm 4) before releasing the others.  The host sees the solve only at
// launch and at completion.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/kiops.h"

namespace kiops {

constexpr int kThreads = 256;
constexpr int kMaxBasis = KIOPS_M_MAX_LIMIT + 1;   // v_1 .. v_{m_max+1}
constexpr int kLdh = kMaxBasis + 2;                 // H, G indexed 1-based
constexpr int kPM = KIOPS_P_MAX;
constexpr int kWinMax = 4;                          // windows q <= 4 use register accumulators
constexpr int kTraceMax = 4096;
constexpr int kTraceStride = 6;
// Release words of a grid barrier: the next pass's context as 64-bit words
// that carry the barrier epoch in their high half (phase, kp, flo, dlo, then
// a, the window coefficients bw[flo..flo+kWinMax) and the trailing parts of
// the last two vectors, each double as two words).
constexpr int kCtxUsed = 4 + 2 * (1 + kWinMax + 2 * kPM);
constexpr int kCtxWords = 64;
static_assert(kCtxUsed <= kCtxWords, "release words");
constexpr int kMaxTimes = KIOPS_MAX_TIMES;            // output times of one call
constexpr int kXcds = 8;                            // accelerator complex dies of an MI355X

enum Phase : int32_t { kPhasePass = 0, kPhaseGather = 1, kPhaseDone = 2, kPhaseDots = 3, kPhaseExpm = 4 };
constexpr int kDotFullStride = 2 * kLdh;            // full-window inner products per workgroup
enum Mode : int32_t { kModeSolve = 0, kModeBasis = 1 };
// Served form: which solver body a request runs (p <= 4).
enum Family : int32_t { kFamily2D = 0, kFamily2DMixed = 1, kFamily3D = 2, kFamily3DMixed = 3 };

// The solve a workgroup works on: its index among that solve's workgroups and
// their number (the whole grid for a single solve; one group of workgroups of
// a batched or served launch).  Set once per workgroup at kernel entry.
__shared__ int kiops_vgrid[2];
__device__ __forceinline__ int vblock() { return kiops_vgrid[0]; }
__device__ __forceinline__ int vgrid() { return kiops_vgrid[1]; }
__device__ __forceinline__ void set_vgrid(int b, int n) {
  if (threadIdx.x == 0) {
    kiops_vgrid[0] = b;
    kiops_vgrid[1] = n;
  }
  __syncthreads();
}

// Small solver state, in the workspace.  Written only inside epilogues.
struct Ctrl {
  // ---- what the workgroups do next
  int32_t phase;
  int32_t kp;        // next pass produces basis vector R_kp (1-based)
  int32_t flo;       // formation window: R_i, i in [flo, kp-1] (kp >= 2)
  int32_t dlo;       // inner products of the pass: i in [dlo, kp]
  int32_t jg;        // gather: number of basis vectors
  int32_t status;
  int32_t mode;
  int32_t estimate;  // KIOPS_ESTIMATE_*
  double a;                    // R_kp = a U_{kp-1} + sum_i bw[i] R_i
  double bw[kLdh];
  double yb_prev[kPM];         // nu * y(R_{kp-1}): B term of U_{kp-1}
  double yb_cur[kPM];          // nu * y(R_kp):     B term of U_kp
  double cg[kLdh];             // gather coefficients
  // ---- solver state (Algorithm 1)
  double T_now, T_end, tau, tol, beta, nu, mu;
  double tau_new;              // decided at acceptance, applied after the gather
  int32_t m, m_new, p, q, m_min, m_max, max_substeps, breakdown;
  int32_t have_old, m_old;
  double tau_old, eps_old, omega_old;
  // ---- statistics
  int32_t substeps, rejections, expms, breakdowns, attempts;
  uint32_t epoch_end;          // served form: grid-barrier epoch when the solve ended
  // ---- several output times (Algorithms 1 and 3)
  int32_t out_next;            // first output time not yet written (l)
  int32_t pending;             // intermediate outputs of this substep still to gather
  int32_t gather_to;           // output the next gather writes: -1 = the state w
  int32_t pad2;
  // ---- the attempt's small exponential when it is spread over the grid
  int32_t e_nst, pad4;         // number of stages
  int32_t e_j, e_bd;           // basis size and breakdown flag of the attempt
  int32_t e_d, e_s;            // Taylor degree index, squarings
  int32_t e_round, pad3;       // exponentials of this attempt so far
  double e_alpha;              // 2^-s
  uint64_t e_t0;               // clock when the attempt's first exponential began
  int64_t matvecs;
  double last_omega, alg_bytes;
  double s_last;
  // phase timers of workgroup 0, in ticks of the constant-rate clock:
  // its own pass work, waiting for the other workgroups, epilogues
  uint64_t t_work, t_wait, t_epi, t_last;
  // optional profile: small exponentials, latest / mean arrival after a release
  uint64_t t_expm, t_arrive_max, t_arrive_mean, n_barriers;
  uint64_t t_release_max, t_release_mean;   // delay until a workgroup sees the release
  uint64_t t_red, t_pub, t_ser;   // epilogues of passes: partial-sum reduction, control-block copy,
                                  // serial normalisation and coefficients
  // the latest normalised vector v_k: <v_k, A~ v_k> and ||A~ v_k||^2 (the
  // two-term and corrected error estimates use them for v_{m+1})
  double est_c, est_u;
  uint64_t t_begin, t_end;      // clock at the start and at the end of the solve
};

// Release word and abort flag on separate 128-byte lines: every workgroup
// polls `gen`, and the abort flag is read far less often.
struct Barrier {
  unsigned gen;
  unsigned pad0[31];
  unsigned abort;
  unsigned pad1[31];
};

// Kernel parameters common to all operators (passed by value).
struct KParams {
  int64_t N;
  int p, q, m_min, m_max, m_init, max_substeps;
  int mode, mixed, nwg, ndot_stride;
  int profile;                 // record per-workgroup arrival times (diagnostics)
  int family;                  // served form: operator family of the request (kFamily*)
  int wg0;                     // served form: first workgroup of the gang running the solve
  unsigned epoch0;             // served form: grid-barrier epoch the solve starts from
  int poll_sleep;              // barrier polls: s_sleep(2) repeats between two reads of a flag
  int ranks;                   // workgroups per CU of a grid that fills every CU evenly, else 1
  int expm_grid;               // padded size from which the small exponential runs on the whole grid (0: never)
  int estimate;                // error estimate of an attempt: KIOPS_ESTIMATE_* (Section 3.4)
  double T_end, tol;
  double elem_bytes;           // bytes per basis element (8 or 4)
  double coef_streams;         // per-cell coefficient arrays the operator reads
  uint64_t spin_limit;         // wall-clock ticks a barrier may wait before aborting
  const double* b[kPM + 1];    // caller's b_0..b_p
  double* w;                   // result (FP64), also R_1 in FP64 mode
  void* slots;                 // basis vector storage, slot i at (i-1)*N elements
  void* bcopy;                 // mixed: float copies of B columns
  Ctrl* ctrl;
  Barrier* bar;
  unsigned* arrive;            // per-workgroup arrival epochs (grid barrier)
  uint64_t* arrive_t;          // profile only: per-workgroup arrival clocks, release-seen clocks,
                               // and per-workgroup sums of arrival after release
  double* H;                   // kLdh x kLdh
  double* G;                   // Gram matrix of the normalised basis, kLdh x kLdh
  double* Y;                   // trailing (y) parts of R_i, kLdh x kPM
  double* sinv;                // v_i = R_i * sinv[i]
  double* coefc;               // full window: c_i = <v_i, A~ v_k>
  double* fullc;               // full window: reduced <R_i, R_k>, <R_i, U_k> (interleaved)
  double* dpart;               // full window: nwg x kDotFullStride partial inner products
  void* ubuf;                  // full window: U_k = A~ R_k of the latest pass (elements of T)
  double* partials;            // nwg x ndot_stride
  double* expm;                // small-exponential scratch
  double* trace;               // kTraceMax x kTraceStride
  double* cgsave;              // several output times: the substep's own gather coefficients (kLdh)
  int ntimes;                  // output times (1: only T_end)
  int task1;                   // Task I: output l is scaled by (1 / T_l)^p (Algorithm 1)
  double times[kMaxTimes];     // T_1 < ... < T_ntimes = T_end
  double* wout[kMaxTimes];     // output l (wout[ntimes - 1] == w, the state)
  uint64_t* tctx;               // release words (kCtxWords): zero, or tagged below this solve's epochs
};

// Work queue of one group of workgroups (batched and served launches).  The
// host publishes entry e by storing its parameter block pointer at
// blocks[e % kGroupQueueLen] and then tail = e + 1; the group stores done =
// e + 1 when that solve has finished (its control block is then final).
constexpr int kGroupQueueLen = 256;
struct GroupQueue {
  unsigned tail;            // entries published (host)
  unsigned closed;          // no more entries will come (host)
  unsigned done;            // entries finished (device)
  unsigned exited;          // the group has left its loop (device)
  uint64_t idle_limit;      // wall-clock ticks a group waits for an entry
  unsigned exit_reason;     // why the group left: 1 closed, 2 idle (device)
  unsigned exit_entry;      // the entry it was waiting for then (device)
  unsigned idle_sleep;      // s_sleep(127) repeats between two polls of an idle group
  int wg0;                  // batched form: first workgroup of the group
  int gsize;                // batched form: workgroups of the group
  unsigned pad0;
  uint64_t pad1[10];        // one 128-byte line for the words above
  const unsigned char* blocks[kGroupQueueLen];
};

}  // namespace kiops
