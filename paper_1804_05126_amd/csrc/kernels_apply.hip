// Product y = A x of an operator outside a solve (FP64): the periodic stencils
// of the operator description and CSR, one thread per row.  A plain kernel for
// callers that need A x itself, e.g. the nonlinear right-hand side f(u) = A u
// + g(u) of an exponential integrator (Section 2) or a residual; the solves
// never call it (their passes fuse the product with the basis update).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/kiops.h"
#include "kernel_table.h"

namespace kiops {

namespace {

constexpr int kApplyThreads = 256;

struct ApplyStencil {
  int64_t nx, ny, nz;
  double h2inv, half_hinv, diff;
  double adv[3];
  const double* kappa;
  const double* r;
};

// (A u)_i = sum_d [kf+ (u_{i+e_d} - u_i) - kf- (u_i - u_{i-e_d})] / h^2
//           - adv_d (u_{i+e_d} - u_{i-e_d}) / (2 h) + r_i u_i,
// kf+- = diff, or the mean of kappa at i and at the neighbour; periodic.
__global__ void __launch_bounds__(kApplyThreads) apply_stencil_kernel(ApplyStencil s, const double* __restrict__ x,
                                                                     double* __restrict__ y, int64_t N) {
  const int64_t stride = (int64_t)gridDim.x * kApplyThreads;
  for (int64_t i = (int64_t)blockIdx.x * kApplyThreads + threadIdx.x; i < N; i += stride) {
    const int64_t ix = i % s.nx;
    const int64_t rest = i / s.nx;
    const int64_t iy = rest % s.ny;
    const int64_t iz = rest / s.ny;
    const int64_t len[3] = {s.nx, s.ny, s.nz};
    const int64_t pos[3] = {ix, iy, iz};
    const int64_t step[3] = {1, s.nx, s.nx * s.ny};
    const double c = x[i];
    const double kc = s.kappa ? s.kappa[i] : 0.0;
    double acc = s.r ? s.r[i] * c : 0.0;
    for (int d = 0; d < 3; ++d) {
      const int64_t ip = i + (pos[d] + 1 < len[d] ? step[d] : (1 - len[d]) * step[d]);
      const int64_t im = i + (pos[d] > 0 ? -step[d] : (len[d] - 1) * step[d]);
      const double up = x[ip], um = x[im];
      const double kp = s.kappa ? 0.5 * (kc + s.kappa[ip]) : s.diff;
      const double km = s.kappa ? 0.5 * (kc + s.kappa[im]) : s.diff;
      acc += (kp * (up - c) - km * (c - um)) * s.h2inv;
      acc -= s.adv[d] * (up - um) * s.half_hinv;
    }
    y[i] = acc;
  }
}

// CSR rows; a row pointer outside [0, nnz] or a column outside [0, n) reads as
// a zero entry, as in the solver's CSR pass.
__global__ void __launch_bounds__(kApplyThreads) apply_csr_kernel(const int32_t* __restrict__ rowptr,
                                                                 const int32_t* __restrict__ col,
                                                                 const double* __restrict__ val, int64_t nnz,
                                                                 const double* __restrict__ x,
                                                                 double* __restrict__ y, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kApplyThreads;
  for (int64_t i = (int64_t)blockIdx.x * kApplyThreads + threadIdx.x; i < n; i += stride) {
    int64_t a = rowptr[i], b = rowptr[i + 1];
    a = a < 0 ? 0 : (a > nnz ? nnz : a);
    b = b < a ? a : (b > nnz ? nnz : b);
    double acc = 0.0;
    for (int64_t k = a; k < b; ++k) {
      const int32_t j = col[k];
      if (j >= 0 && (int64_t)j < n) acc = fma(val[k], x[j], acc);
    }
    y[i] = acc;
  }
}

// general form: per-cell weights [nw][N] of (centre, +x, -x, +y, -y, +z, -z)
__global__ void __launch_bounds__(kApplyThreads) apply_weights_kernel(int64_t nx, int64_t ny, int64_t nz, int nw,
                                                                     const double* __restrict__ W,
                                                                     const double* __restrict__ x,
                                                                     double* __restrict__ y, int64_t N) {
  const int64_t stride = (int64_t)gridDim.x * kApplyThreads;
  for (int64_t i = (int64_t)blockIdx.x * kApplyThreads + threadIdx.x; i < N; i += stride) {
    const int64_t ix = i % nx;
    const int64_t rest = i / nx;
    const int64_t pos[3] = {ix, rest % ny, rest / ny};
    const int64_t len[3] = {nx, ny, nz};
    const int64_t step[3] = {1, nx, nx * ny};
    double acc = W[i] * x[i];
    for (int d = 0; 2 * d + 1 < nw; ++d) {
      const int64_t ip = i + (pos[d] + 1 < len[d] ? step[d] : (1 - len[d]) * step[d]);
      const int64_t im = i + (pos[d] > 0 ? -step[d] : (len[d] - 1) * step[d]);
      acc = fma(W[(2 * d + 1) * N + i], x[ip], acc);
      acc = fma(W[(2 * d + 2) * N + i], x[im], acc);
    }
    y[i] = acc;
  }
}

int apply_blocks(int64_t n) {
  const int64_t b = (n + kApplyThreads - 1) / kApplyThreads;
  return (int)(b < 65536 ? b : 65536);
}

}  // namespace

hipError_t launch_apply(const kiops_operator_desc& d, int64_t N, const double* x, double* y, hipStream_t st) {
  if (d.weights) {
    const int nw = d.kind == KIOPS_OP_STENCIL2D_5PT ? 5 : 7;
    hipLaunchKernelGGL(apply_weights_kernel, dim3(apply_blocks(N)), dim3(kApplyThreads), 0, st, (int64_t)d.nx,
                       (int64_t)d.ny, (int64_t)d.nz, nw, d.weights, x, y, N);
  } else if (d.kind == KIOPS_OP_CSR) {
    hipLaunchKernelGGL(apply_csr_kernel, dim3(apply_blocks(N)), dim3(kApplyThreads), 0, st, d.rowptr, d.col, d.val,
                       (int64_t)d.nnz, x, y, N);
  } else {
    ApplyStencil s;
    s.nx = d.nx;
    s.ny = d.ny;
    s.nz = d.nz;
    s.h2inv = 1.0 / (d.h * d.h);
    s.half_hinv = 0.5 / d.h;
    s.diff = d.diff;
    for (int k = 0; k < 3; ++k) s.adv[k] = d.adv[k];
    s.kappa = d.kappa;
    s.r = d.reaction;
    hipLaunchKernelGGL(apply_stencil_kernel, dim3(apply_blocks(N)), dim3(kApplyThreads), 0, st, s, x, y, N);
  }
  return hipGetLastError();
}

}  // namespace kiops
