// Small dense matrix exponential on one workgroup (256 threads), float64.
//
// Section 3.3.1 forms exp(tau H~) of the (j+1) x (j+1) projected matrix by
// scaling and squaring around a rational (diagonal Pade) approximant.  Here the
// approximant is the truncated Taylor series, still with scaling and squaring:
// a Taylor polynomial needs nothing but matrix products, and those run on the
// f64 matrix cores (v_mfma_f64_16x16x4), whereas a Pade quotient needs a
// pivoted LU solve whose column-after-column dependence leaves a workgroup
// waiting on latency for most of its run.
//
// Degree.  With X the matrix and eta = ||X||_1, the degree is the smallest m in
// {2, 4, 6, 9, 12, 16} with eta <= theta_m, where theta_m is the largest theta
// with sum_{k>m} theta^k / k! <= 2^-53 e^-theta.  Every eigenvalue of X lies in
// |z| <= eta, so ||e^X||_1 >= e^-eta and the truncation error stays below the
// unit roundoff relative to ||e^X||_1.  Beyond theta_16 the matrix is scaled by
// 2^-s (s = ceil(log2(eta / theta_16))) and the result squared s times.
//
// Evaluation (Paterson & Stockmeyer 1973).  With m = q b and c_k = 1/k!:
//   powers X^2 .. X^b,
//   Z_{q-1} = sum_{i<b} c_{(q-1)b+i} X^i + c_m X^b,
//   Z_k     = X^b Z_{k+1} + sum_{i<b} c_{kb+i} X^i,   k = q-2 .. 0,
// and T_m(X) = Z_0: (b - 1) + (q - 1) products, the sums fused into the
// products' output stage.  (m, b) = (2,2) (4,2) (6,3) (9,3) (12,4) (16,4).
//
// Matrices live in global scratch memory (at most 7 x 166 KB, resident in L2)
// with the fixed leading dimension kExpmLd; entries beyond n are kept zero, so
// products over the 16-padded size are exact.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "buffer.h"

namespace kiops {

constexpr int kExpmMaxN = 129;   // m_max + 1
constexpr int kExpmLd = 144;     // kExpmMaxN rounded up to 16
constexpr int kExpmSlot = kExpmLd * kExpmLd;
constexpr int kExpmSlots = 9;    // scratch size of the C interface; 7 are used
constexpr int kExpmLdsDoubles = 264;   // reduction buffer (256) + coefficients (5)

// theta_m for m = 2, 4, 6, 9, 12, 16 (criterion in the header comment).
__device__ constexpr double kTaylorTheta[6] = {8.733444801477513e-06, 1.6778312117956388e-03,
                                               1.7719629491983992e-02, 1.135367072544621e-01,
                                               3.269045734215958e-01, 7.873811561929019e-01};
__device__ constexpr int kTaylorDeg[6] = {2, 4, 6, 9, 12, 16};
__device__ constexpr int kTaylorBlk[6] = {2, 2, 3, 3, 4, 4};

typedef double kiops_f64x2 __attribute__((ext_vector_type(2)));
typedef double kiops_f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int pad16(int n) { return (n + 15) & ~15; }

// Maximum of one value per thread over the workgroup (lds: 256 doubles).
__device__ __forceinline__ double wg_max(double v, double* lds) {
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) lds[t] = lds[t] > lds[t + off] ? lds[t] : lds[t + off];
    __syncthreads();
  }
  const double r = lds[0];
  __syncthreads();
  return r;
}

// Output stage shared by products and plain sums: cf[0] I + sum_{k=1}^{nterms-1}
// cf[k] X^k, with X^k held in slot k-1 of `pw`.  nterms = 0 adds nothing.
__device__ __forceinline__ double power_sum(const double* __restrict__ pw, const double* cf,
                                            int nterms, int n, int row, int col) {
  double v = 0.0;
  if (nterms > 0 && row == col && row < n) v = cf[0];
  for (int k = 1; k < nterms; ++k) v = fma(cf[k], pw[(k - 1) * kExpmSlot + row * kExpmLd + col], v);
  return v;
}

// C = alpha A B + (power sum), n16 x n16, leading dimension kExpmLd.  C must
// not alias A or B.  Each wave owns 16-row strips of C in chunks of NJ <= 5
// 16 x 16 tiles; per 8-deep slice of the inner dimension a lane holds two
// entries of A and two of B per tile (the 16x16x4 f64 operand layout: A(i, k)
// in lane i + 16 k, B(k, j) in lane j + 16 k, C(i, j) in lane j + 16 (i % 4),
// element i / 4), and the next slice is loaded while the current one is
// multiplied.  Within a slice, lane group g covers inner indices 2g and 2g+1.
template <int NJ>
__device__ __forceinline__ void gemm_strip(__amdgpu_buffer_rsrc_t rC, __amdgpu_buffer_rsrc_t rA,
                                           __amdgpu_buffer_rsrc_t rB, __amdgpu_buffer_rsrc_t rP,
                                           int n, int n16, double alpha, const double* cf,
                                           int nterms, int I, int J0) {
  const int lane = threadIdx.x & 63;
  const int r16 = lane & 15, g = lane >> 4;
  constexpr uint32_t kRow = kExpmLd * 8;   // bytes per row
  const uint32_t oA = (uint32_t)((I * 16 + r16) * kExpmLd + 2 * g) * 8u;
  const uint32_t oB = (uint32_t)(2 * g * kExpmLd + J0 * 16 + r16) * 8u;
  kiops_f64x4 acc[NJ];
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) acc[jj] = kiops_f64x4{0.0, 0.0, 0.0, 0.0};
  // two register sets, X and Y, alternate between slices (n16 is a multiple of
  // 16, so slices come in pairs); a set is refilled right after its products
  // are issued, one slice ahead of its use
  double xa0, xa1, xb0[NJ], xb1[NJ], ya0, ya1, yb0[NJ], yb1[NJ];
  auto load = [&](uint32_t k, double& a0, double& a1, double* b0, double* b1) {
    buf_ld2(rA, oA + k * 8u, a0, a1);
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
      b0[jj] = buf_ld(rB, oB + k * kRow + jj * 128u, 0.0);
      b1[jj] = buf_ld(rB, oB + k * kRow + kRow + jj * 128u, 0.0);
    }
  };
  auto mma = [&](double a0, double a1, const double* b0, const double* b1) {
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) acc[jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0[jj], acc[jj], 0, 0, 0);
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) acc[jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1[jj], acc[jj], 0, 0, 0);
  };
  load(0, xa0, xa1, xb0, xb1);
  for (int k0 = 0; k0 < n16; k0 += 16) {
    load((uint32_t)(k0 + 8), ya0, ya1, yb0, yb1);
    mma(xa0, xa1, xb0, xb1);
    // the last pair reloads its own second slice instead of branching
    load((uint32_t)(k0 + 16 < n16 ? k0 + 16 : k0 + 8), xa0, xa1, xb0, xb1);
    mma(ya0, ya1, yb0, yb1);
  }
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) {
    const int col = (J0 + jj) * 16 + r16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = I * 16 + g + 4 * i;
      const uint32_t o = (uint32_t)(row * kExpmLd + col);
      double v = (nterms > 0 && row == col && row < n) ? cf[0] : 0.0;
      for (int k = 1; k < nterms; ++k) v = fma(cf[k], buf_ld(rP, (o + (uint32_t)(k - 1) * kExpmSlot) * 8u, 0.0), v);
      buf_st(rC, o * 8u, fma(alpha, acc[jj][i], v));
    }
  }
}

// One product on the whole workgroup; every argument is the same on all lanes.
__device__ __noinline__ void wg_gemm(double* C, const double* A, const double* B, int n, int n16,
                                     double alpha, const double* pw, const double* cf, int nterms) {
  n = uniform(n);
  n16 = uniform(n16);
  alpha = uniform(alpha);
  nterms = uniform(nterms);
  constexpr uint64_t kSlotBytes = (uint64_t)kExpmSlot * 8;
  const __amdgpu_buffer_rsrc_t rC = make_rsrc(uniform(C), kSlotBytes);
  const __amdgpu_buffer_rsrc_t rA = make_rsrc(uniform(A), kSlotBytes);
  const __amdgpu_buffer_rsrc_t rB = make_rsrc(uniform(B), kSlotBytes);
  const __amdgpu_buffer_rsrc_t rP = make_rsrc(uniform(pw), 4 * kSlotBytes);
  const int wv = uniform((int)(threadIdx.x >> 6));
  const int nt = n16 >> 4;
  const int nch = nt > 5 ? 2 : 1;
  const int wch = (nt + nch - 1) / nch;
  for (int u = wv; u < nt * nch; u += 4) {
    const int I = u / nch;
    const int J0 = (u - I * nch) * wch;
    const int nj = (nt - J0) < wch ? (nt - J0) : wch;
    switch (nj) {
      case 1: gemm_strip<1>(rC, rA, rB, rP, n, n16, alpha, cf, nterms, I, J0); break;
      case 2: gemm_strip<2>(rC, rA, rB, rP, n, n16, alpha, cf, nterms, I, J0); break;
      case 3: gemm_strip<3>(rC, rA, rB, rP, n, n16, alpha, cf, nterms, I, J0); break;
      case 4: gemm_strip<4>(rC, rA, rB, rP, n, n16, alpha, cf, nterms, I, J0); break;
      default: gemm_strip<5>(rC, rA, rB, rP, n, n16, alpha, cf, nterms, I, J0); break;
    }
  }
  __syncthreads();
}

// C = (power sum) over the n16 x n16 block.
__device__ __forceinline__ void wg_power_sum(double* __restrict__ C, int n, int n16,
                                             const double* __restrict__ pw, const double* cf,
                                             int nterms) {
  for (int e = threadIdx.x; e < n16 * n16; e += 256) {
    const int r = e / n16, c = e - r * n16;
    C[r * kExpmLd + c] = power_sum(pw, cf, nterms, n, r, c);
  }
  __syncthreads();
}

// Degree index d (Taylor degree kTaylorDeg[d]) and number of squarings s for
// a matrix with ||X||_1 = eta (criterion in the header comment).
__device__ __forceinline__ void expm_plan(double eta, int& d, int& s) {
  d = 5;
  s = 0;
  if (eta <= kTaylorTheta[5]) {
    d = 0;
    while (eta > kTaylorTheta[d]) ++d;
  } else if (eta < 1e300) {
    s = (int)ceil(log2(eta / kTaylorTheta[5]));
    if (s > 1000) s = 1000;
  }
  // eta non-finite: no scaling; the result carries the NaN / Inf onward
}

// Coefficients of Paterson-Stockmeyer block k (one thread): cf[i] = c_{kb+i}
// for i < b, cf[1] carrying alpha since slot 0 holds the unscaled X; the top
// block also takes cf[b] = c_m (the coefficient of X^b).
__device__ inline void expm_block_coefs(double* cf, int k, int b, double alpha, bool top) {
  double c = 1.0;
  for (int i = 1; i <= k * b; ++i) c /= (double)i;   // c_{kb}
  for (int i = 0; i < b; ++i) {
    cf[i] = (i == 1) ? c * alpha : c;
    c /= (double)(k * b + i + 1);
  }
  cf[b] = top ? c : 0.0;                               // c_{(k+1)b} = c_m when top
}

// exp(X) for the n x n matrix X held in slot 0 of `scratch` (zero-padded to a
// multiple of 16), eta = ||X||_1 (computed by the caller while it writes X).
// Returns the slot (4 or 5) holding the result.  Slots 0..5 are used; slot 0
// is left unchanged (the scaling is folded into the products).
// lds: kExpmLdsDoubles doubles.
__device__ __forceinline__ int wg_expm(double* scratch, int n, double eta, double* lds) {
  const int n16 = pad16(n);
  double* X = scratch;                          // slots 0..3: X, X^2, X^3, X^4
  double* Z[2] = {scratch + 4 * kExpmSlot, scratch + 5 * kExpmSlot};
  double* cf = lds + 256;

  int d, s;
  expm_plan(eta, d, s);
  const int m = kTaylorDeg[d], b = kTaylorBlk[d], q = m / b;
  const double alpha = ldexp(1.0, -s);

  // powers of the scaled matrix: (alpha X)^k = alpha^k X^k
  if (b >= 2) wg_gemm(X + kExpmSlot, X, X, n, n16, alpha * alpha, nullptr, nullptr, 0);
  if (b >= 3) wg_gemm(X + 2 * kExpmSlot, X + kExpmSlot, X, n, n16, alpha, nullptr, nullptr, 0);
  if (b >= 4) wg_gemm(X + 3 * kExpmSlot, X + kExpmSlot, X + kExpmSlot, n, n16, 1.0, nullptr, nullptr, 0);

  auto set_block = [&](int k, bool top) {
    if (threadIdx.x == 0) expm_block_coefs(cf, k, b, alpha, top);
    __syncthreads();
  };
  set_block(q - 1, true);
  int cur = 0;
  wg_power_sum(Z[cur], n, n16, X, cf, b + 1);
  for (int k = q - 2; k >= 0; --k) {
    set_block(k, false);
    wg_gemm(Z[cur ^ 1], X + (b - 1) * kExpmSlot, Z[cur], n, n16, 1.0, X, cf, b);
    cur ^= 1;
  }
  for (int i = 0; i < s; ++i) {
    wg_gemm(Z[cur ^ 1], Z[cur], Z[cur], n, n16, 1.0, nullptr, nullptr, 0);
    cur ^= 1;
  }
  return 4 + cur;
}

// ---- The same exponential spread over the workgroups of a grid.
//
// The products of wg_expm run as stages separated by grid barriers:
//   X^2;  then X^3 and X^4 together;  the top block's power sum (elementwise);
//   the q - 1 block products;  the s squarings.
// Each product tile is computed by one wave with the same products in the
// same order as in wg_expm, so the result is bitwise the same.

// Number of stages for degree index d and s squarings.
__device__ __forceinline__ int expm_stages(int d, int s) {
  const int b = kTaylorBlk[d], q = kTaylorDeg[d] / b;
  return (b >= 2 ? 1 : 0) + (b >= 3 ? 1 : 0) + 1 + (q - 1) + s;
}

// Slot holding the result after the last stage.
__device__ __forceinline__ int expm_result_slot(int d, int s) {
  const int q = kTaylorDeg[d] / kTaylorBlk[d];
  return 4 + ((q - 1 + s) & 1);
}

// One 16 x 16 tile (I, J) of C = alpha A B + (power sum) by one wave, with
// the same products in the same order as gemm_strip<1>, but with the operand
// loads issued kB 8-deep slices at a time, one batch ahead: the operands
// were written by other workgroups just before, so each load is a full
// memory round trip, and a one-slice lookahead would pay one per slice.
template <int kB>
__device__ __forceinline__ void gemm_tile_deep(__amdgpu_buffer_rsrc_t rC, __amdgpu_buffer_rsrc_t rA,
                                               __amdgpu_buffer_rsrc_t rB, __amdgpu_buffer_rsrc_t rP, int n,
                                               int n16, double alpha, const double* cf, int nterms, int I,
                                               int J) {
  const int lane = threadIdx.x & 63;
  const int r16 = lane & 15, g = lane >> 4;
  constexpr uint32_t kRow = kExpmLd * 8;   // bytes per row
  const uint32_t oA = (uint32_t)((I * 16 + r16) * kExpmLd + 2 * g) * 8u;
  const uint32_t oB = (uint32_t)(2 * g * kExpmLd + J * 16 + r16) * 8u;
  const int nsl = n16 >> 3;                // 8-deep slices
  kiops_f64x4 acc = kiops_f64x4{0.0, 0.0, 0.0, 0.0};
  double xa0[kB], xa1[kB], xb0[kB], xb1[kB], ya0[kB], ya1[kB], yb0[kB], yb1[kB];
  auto load = [&](int s0, double* a0, double* a1, double* b0, double* b1) {
#pragma unroll
    for (int i = 0; i < kB; ++i) {
      if (s0 + i < nsl) {
        const uint32_t k = (uint32_t)(s0 + i) * 8u;
        buf_ld2(rA, oA + k * 8u, a0[i], a1[i]);
        b0[i] = buf_ld(rB, oB + k * kRow, 0.0);
        b1[i] = buf_ld(rB, oB + k * kRow + kRow, 0.0);
      }
    }
  };
  auto mma = [&](int s0, const double* a0, const double* a1, const double* b0, const double* b1) {
#pragma unroll
    for (int i = 0; i < kB; ++i) {
      if (s0 + i < nsl) {
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[i], b0[i], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[i], b1[i], acc, 0, 0, 0);
      }
    }
  };
  load(0, xa0, xa1, xb0, xb1);
  for (int s0 = 0; s0 < nsl; s0 += 2 * kB) {
    load(s0 + kB, ya0, ya1, yb0, yb1);
    mma(s0, xa0, xa1, xb0, xb1);
    load(s0 + 2 * kB, xa0, xa1, xb0, xb1);
    mma(s0 + kB, ya0, ya1, yb0, yb1);
  }
  const int col = J * 16 + r16;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = I * 16 + g + 4 * i;
    const uint32_t o = (uint32_t)(row * kExpmLd + col);
    double v = (nterms > 0 && row == col && row < n) ? cf[0] : 0.0;
    for (int k = 1; k < nterms; ++k) v = fma(cf[k], buf_ld(rP, (o + (uint32_t)(k - 1) * kExpmSlot) * 8u, 0.0), v);
    buf_st(rC, o * 8u, fma(alpha, acc[i], v));
  }
}

// Stage st of exp(X) (X in slot 0 of `scratch`, n x n, degree index d,
// s squarings, alpha = 2^-s) by workgroup wg of nwg.  The 16 x 16 tiles of a
// stage's products are dealt to the waves of the grid: wave w of workgroup v
// takes tiles v + nwg (w + 4 r), r = 0, 1, ...; the power-sum stage is dealt
// element by element to all threads.  Every workgroup calls this (whole
// workgroup); cf: 8 doubles of the workgroup's LDS.
__device__ __noinline__ void grid_expm_stage(double* scratch, int n, int d, int s, double alpha, int st,
                                             int wg, int nwg, double* cf) {
  n = uniform(n);
  d = uniform(d);
  s = uniform(s);
  alpha = uniform(alpha);
  st = uniform(st);
  wg = uniform(wg);
  nwg = uniform(nwg);
  const int n16 = pad16(n);
  const int nt = n16 >> 4;
  const int b = kTaylorBlk[d], q = kTaylorDeg[d] / b;
  const int npow = (b >= 2 ? 1 : 0) + (b >= 3 ? 1 : 0);
  double* X = uniform(scratch);
  if (st == npow) {   // Z_{q-1}: the top block's power sum into slot 4
    if (threadIdx.x == 0) expm_block_coefs(cf, q - 1, b, alpha, true);
    __syncthreads();
    double* Z = X + 4 * kExpmSlot;
    for (int e = wg * kThreads + (int)threadIdx.x; e < n16 * n16; e += nwg * kThreads) {
      const int r = e / n16, c = e - r * n16;
      Z[r * kExpmLd + c] = power_sum(X, cf, b + 1, n, r, c);
    }
    return;
  }
  // one or two products C = alpha A B + (power sum of X); slots by stage
  int ng = 1, c0 = 0, a0 = 0, b0 = 0, c1 = 0, a1 = 0, b1 = 0, nterms = 0;
  double al0 = 1.0, al1 = 1.0;
  if (st < npow) {
    if (st == 0) {                       // X^2
      c0 = 1; a0 = 0; b0 = 0; al0 = alpha * alpha;
    } else {                             // X^3 = X^2 X, and X^4 = X^2 X^2
      c0 = 2; a0 = 1; b0 = 0; al0 = alpha;
      if (b >= 4) { ng = 2; c1 = 3; a1 = 1; b1 = 1; al1 = 1.0; }
    }
  } else if (st < npow + q) {            // block k: Z <- X^b Z + sum_{i<b} c_{kb+i} X^i
    const int i = st - npow - 1;
    const int cur = i & 1;
    if (threadIdx.x == 0) expm_block_coefs(cf, q - 2 - i, b, alpha, false);
    __syncthreads();
    c0 = 4 + (cur ^ 1); a0 = b - 1; b0 = 4 + cur; nterms = b;
  } else {                               // squaring i: Z <- Z Z
    const int cur = (q - 1 + (st - npow - q)) & 1;
    c0 = 4 + (cur ^ 1); a0 = 4 + cur; b0 = 4 + cur;
  }
  constexpr uint64_t kSlotBytes = (uint64_t)kExpmSlot * 8;
  const __amdgpu_buffer_rsrc_t rP = make_rsrc(X, 4 * kSlotBytes);
  const int tiles = nt * nt;
  const int wv = uniform((int)(threadIdx.x >> 6));
  for (int u = wg + nwg * wv; u < ng * tiles; u += 4 * nwg) {
    const int g = u >= tiles ? 1 : 0;
    const int t = u - g * tiles;
    const int I = t / nt, J = t - I * nt;
    const __amdgpu_buffer_rsrc_t rC = make_rsrc(X + (size_t)(g ? c1 : c0) * kExpmSlot, kSlotBytes);
    const __amdgpu_buffer_rsrc_t rA = make_rsrc(X + (size_t)(g ? a1 : a0) * kExpmSlot, kSlotBytes);
    const __amdgpu_buffer_rsrc_t rB = make_rsrc(X + (size_t)(g ? b1 : b0) * kExpmSlot, kSlotBytes);
    gemm_tile_deep<6>(rC, rA, rB, rP, n, n16, g ? al1 : al0, cf, nterms, I, J);
  }
}

}  // namespace kiops
