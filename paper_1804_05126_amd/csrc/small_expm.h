// Small dense matrix exponential on one workgroup (256 threads), float64.
//
// Section 3.3.1 computes exp(tau H~) of the (j+1) x (j+1) projected matrix
// with "a diagonal Pade approximation combined with scaling and squaring".
// This is that method in the form of N. J. Higham, "The scaling and squaring
// method for the matrix exponential revisited", SIAM J. Matrix Anal. Appl. 26
// (2005): choose the Pade degree m in {3, 5, 7, 9, 13} from ||A||_1 and the
// published thresholds theta_m; for degree 13 scale A by 2^-s so that
// ||A/2^s||_1 <= theta_13; evaluate r_m = q_m(A)^-1 p_m(A) with p_m(A) = V + U,
// q_m(A) = V - U (U odd part, V even part), solve by LU with partial pivoting;
// square s times.
//
// Matrices live in global scratch memory (they stay in L2: at most 9 x 166 KB)
// with a fixed leading dimension; entries beyond n are kept zero so that the
// 16-padded products are exact.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace kiops {

constexpr int kExpmMaxN = 129;   // m_max + 1
constexpr int kExpmLd = 144;     // kExpmMaxN rounded up to 16
constexpr int kExpmSlot = kExpmLd * kExpmLd;
constexpr int kExpmSlots = 9;
constexpr int kExpmLdsDoubles = 48 * 17 + 16 * 49 + 16;   // gemm staging + Pade coefficients

// theta_m for m = 3, 5, 7, 9, 13 (Higham 2005, Table 2.3, double precision).
__device__ constexpr double kTheta[5] = {1.495585217958292e-2, 2.539398330063230e-1,
                                         9.504178996162932e-1, 2.097847961257068e0,
                                         5.371920351148152e0};

// Coefficients of the [m/m] Pade approximant of e^x, numerator p_m(x) = sum c_i x^i,
// c_i = (2m-i)! m! / ((2m)! i! (m-i)!), by the ratio c_{i+1}/c_i = (m-i)/((2m-i)(i+1)).
__device__ inline void pade_coeffs(int m, double* c) {
  c[0] = 1.0;
  for (int i = 0; i < m; ++i) c[i + 1] = c[i] * (double)(m - i) / ((double)(2 * m - i) * (double)(i + 1));
}

__device__ inline int pad16(int n) { return (n + 15) & ~15; }

// C = A * B for n16 x n16 matrices with leading dimension kExpmLd (C must not alias A or B).
// Output in 48 x 48 blocks; thread (tr, tc) of a 16 x 16 layout owns rows
// tr + 16 a and columns tc + 16 b (a, b < 3) of a block: 9 accumulators.
__device__ inline void wg_gemm(double* __restrict__ C, const double* __restrict__ A,
                               const double* __restrict__ B, int n16, double* lds) {
  const int t = threadIdx.x;
  const int tr = t >> 4, tc = t & 15;
  double* sA = lds;                 // [48][17]
  double* sB = lds + 48 * 17;       // [16][49]
  for (int r0 = 0; r0 < n16; r0 += 48) {
    const int nr = (n16 - r0) < 48 ? (n16 - r0) : 48;
    for (int c0 = 0; c0 < n16; c0 += 48) {
      const int nc = (n16 - c0) < 48 ? (n16 - c0) : 48;
      double acc[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) acc[a][b] = 0.0;
      for (int kk = 0; kk < n16; kk += 16) {
        for (int e = t; e < 48 * 16; e += 256) {
          const int r = e >> 4, k = e & 15;
          sA[r * 17 + k] = (r < nr) ? A[(r0 + r) * kExpmLd + kk + k] : 0.0;
        }
        for (int e = t; e < 16 * 48; e += 256) {
          const int k = e / 48, c = e - k * 48;
          sB[k * 49 + c] = (c < nc) ? B[(kk + k) * kExpmLd + c0 + c] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int k = 0; k < 16; ++k) {
          const double b0 = sB[k * 49 + tc], b1 = sB[k * 49 + 16 + tc], b2 = sB[k * 49 + 32 + tc];
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const double av = sA[(a * 16 + tr) * 17 + k];
            acc[a][0] = fma(av, b0, acc[a][0]);
            acc[a][1] = fma(av, b1, acc[a][1]);
            acc[a][2] = fma(av, b2, acc[a][2]);
          }
        }
        __syncthreads();
      }
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          if (a * 16 + tr < nr && b * 16 + tc < nc)
            C[(r0 + a * 16 + tr) * kExpmLd + c0 + b * 16 + tc] = acc[a][b];
    }
  }
  __syncthreads();
}

// ||A||_1 of the leading n x n block (maximum absolute column sum).
__device__ inline double wg_norm1(const double* A, int n, double* lds) {
  const int t = threadIdx.x;
  double best = 0.0;
  for (int c = t; c < n; c += 256) {
    double s = 0.0;
    for (int r = 0; r < n; ++r) s += fabs(A[r * kExpmLd + c]);
    best = s > best ? s : best;
  }
  lds[t] = best;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) lds[t] = lds[t] > lds[t + off] ? lds[t] : lds[t + off];
    __syncthreads();
  }
  const double r = lds[0];
  __syncthreads();
  return r;
}

// D = w0 M0 + w1 M1 + w2 M2 + w3 M3 + wI I over the n16 x n16 block (null M ignored).
__device__ inline void wg_lincomb(double* D, int n, int n16, const double* M0, double w0,
                                  const double* M1, double w1, const double* M2, double w2,
                                  const double* M3, double w3, double wI) {
  for (int e = threadIdx.x; e < n16 * n16; e += 256) {
    const int r = e / n16, c = e - r * n16;
    const int o = r * kExpmLd + c;
    double v = (r == c && r < n) ? wI : 0.0;
    if (M0) v = fma(w0, M0[o], v);
    if (M1) v = fma(w1, M1[o], v);
    if (M2) v = fma(w2, M2[o], v);
    if (M3) v = fma(w3, M3[o], v);
    D[o] = v;
  }
  __syncthreads();
}

// Solve P X = R (n x n, n right-hand sides) in place: on return R holds X.
// Gaussian elimination with partial pivoting; P is destroyed.
__device__ inline void wg_lu_solve(double* P, double* R, int n, double* lds) {
  const int t = threadIdx.x;
  __shared__ int s_piv;
  for (int k = 0; k < n; ++k) {
    // pivot: argmax |P[i][k]|, i >= k (first wave, shuffle reduction)
    if (t < 64) {
      double best = -1.0;
      int bi = k;
      for (int i = k + t; i < n; i += 64) {
        const double v = fabs(P[i * kExpmLd + k]);
        if (v > best) { best = v; bi = i; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_down(best, off, 64);
        const int oi = __shfl_down(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (t == 0) s_piv = bi;
    }
    __syncthreads();
    const int piv = s_piv;
    if (piv != k) {
      for (int c = t; c < 2 * n; c += 256) {
        double* a = (c < n) ? &P[k * kExpmLd + c] : &R[k * kExpmLd + (c - n)];
        double* b = (c < n) ? &P[piv * kExpmLd + c] : &R[piv * kExpmLd + (c - n)];
        const double tmp = *a;
        *a = *b;
        *b = tmp;
      }
      __syncthreads();
    }
    const double inv = 1.0 / P[k * kExpmLd + k];
    // multipliers kept in column k below the diagonal
    for (int i = k + 1 + t; i < n; i += 256) P[i * kExpmLd + k] *= inv;
    __syncthreads();
    const int rows = n - k - 1;
    const int cols = (n - k - 1) + n;   // trailing part of P, then all of R
    for (int e = t; e < rows * cols; e += 256) {
      const int i = k + 1 + e / cols;
      const int cc = e % cols;
      const double l = P[i * kExpmLd + k];
      if (cc < n - k - 1) {
        const int c = k + 1 + cc;
        P[i * kExpmLd + c] = fma(-l, P[k * kExpmLd + c], P[i * kExpmLd + c]);
      } else {
        const int c = cc - (n - k - 1);
        R[i * kExpmLd + c] = fma(-l, R[k * kExpmLd + c], R[i * kExpmLd + c]);
      }
    }
    __syncthreads();
  }
  // back substitution, one right-hand side column per thread
  for (int c = t; c < n; c += 256) {
    for (int k = n - 1; k >= 0; --k) {
      double v = R[k * kExpmLd + c];
      for (int q = k + 1; q < n; ++q) v = fma(-P[k * kExpmLd + q], R[q * kExpmLd + c], v);
      R[k * kExpmLd + c] = v / P[k * kExpmLd + k];
    }
  }
  __syncthreads();
  (void)lds;
}

// exp(A) for the n x n matrix held in slot 0 of `scratch` (zero-padded to 16).
// Returns the slot index holding the result.  Uses slots 0..8.
__device__ inline int wg_expm(double* scratch, int n, double* lds) {
  const int n16 = pad16(n);
  double* A = scratch;
  double* A2 = scratch + 1 * kExpmSlot;
  double* A4 = scratch + 2 * kExpmSlot;
  double* A6 = scratch + 3 * kExpmSlot;
  double* A8 = scratch + 4 * kExpmSlot;
  double* T = scratch + 5 * kExpmSlot;
  double* U = scratch + 6 * kExpmSlot;
  double* V = scratch + 7 * kExpmSlot;
  double* W = scratch + 8 * kExpmSlot;
  double* c = lds + 48 * 17 + 16 * 49;   // Pade coefficients (14 doubles)

  const double eta = wg_norm1(A, n, lds);
  int m = 13;
  int s = 0;
  if (eta <= kTheta[0]) m = 3;
  else if (eta <= kTheta[1]) m = 5;
  else if (eta <= kTheta[2]) m = 7;
  else if (eta <= kTheta[3]) m = 9;
  else if (eta > kTheta[4]) s = (int)ceil(log2(eta / kTheta[4]));
  if (s > 0) {
    const double sc = ldexp(1.0, -s);
    for (int e = threadIdx.x; e < n16 * n16; e += 256) {
      const int r = e / n16, cc = e - r * n16;
      A[r * kExpmLd + cc] *= sc;
    }
  }
  if (threadIdx.x == 0) pade_coeffs(m, c);
  __syncthreads();

  wg_gemm(A2, A, A, n16, lds);
  if (m >= 5) wg_gemm(A4, A2, A2, n16, lds);
  if (m >= 7) wg_gemm(A6, A4, A2, n16, lds);
  if (m == 9) wg_gemm(A8, A4, A4, n16, lds);

  if (m == 13) {
    // U = A [A6 (c13 A6 + c11 A4 + c9 A2) + c7 A6 + c5 A4 + c3 A2 + c1 I]
    wg_lincomb(T, n, n16, A6, c[13], A4, c[11], A2, c[9], nullptr, 0.0, 0.0);
    wg_gemm(W, A6, T, n16, lds);
    wg_lincomb(T, n, n16, W, 1.0, A6, c[7], A4, c[5], A2, c[3], c[1]);
    wg_gemm(U, A, T, n16, lds);
    // V = A6 (c12 A6 + c10 A4 + c8 A2) + c6 A6 + c4 A4 + c2 A2 + c0 I
    wg_lincomb(T, n, n16, A6, c[12], A4, c[10], A2, c[8], nullptr, 0.0, 0.0);
    wg_gemm(W, A6, T, n16, lds);
    wg_lincomb(V, n, n16, W, 1.0, A6, c[6], A4, c[4], A2, c[2], c[0]);
  } else {
    // odd part U = A (c1 I + c3 A2 + c5 A4 + ...), even part V = c0 I + c2 A2 + ...
    const double* P4 = (m >= 5) ? A4 : nullptr;
    const double* P6 = (m >= 7) ? A6 : nullptr;
    const double* P8 = (m >= 9) ? A8 : nullptr;
    wg_lincomb(T, n, n16, A2, c[3], P4, (m >= 5) ? c[5] : 0.0, P6, (m >= 7) ? c[7] : 0.0, P8,
               (m >= 9) ? c[9] : 0.0, c[1]);
    wg_gemm(U, A, T, n16, lds);
    wg_lincomb(V, n, n16, A2, c[2], P4, (m >= 5) ? c[4] : 0.0, P6, (m >= 7) ? c[6] : 0.0, P8,
               (m >= 9) ? c[8] : 0.0, c[0]);
  }
  // P = V - U (slot T), R = V + U (slot W); solve P X = R
  wg_lincomb(T, n, n16, V, 1.0, U, -1.0, nullptr, 0.0, nullptr, 0.0, 0.0);
  wg_lincomb(W, n, n16, V, 1.0, U, 1.0, nullptr, 0.0, nullptr, 0.0, 0.0);
  wg_lu_solve(T, W, n, lds);
  // square s times, ping-pong between W and U
  double* cur = W;
  double* nxt = U;
  for (int i = 0; i < s; ++i) {
    wg_gemm(nxt, cur, cur, n16, lds);
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  return cur == W ? 8 : 6;
}

}  // namespace kiops
