// Host side of the C ABI declared in include/kiops.h: argument checks,
// workspace layout, the cooperative launch of the persistent solve kernel,
// and the diagnostics entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <new>
#include <deque>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "../../include/kiops.h"
#include "controller.h"
#include "op_stencil2d.h"
#include "op_stencil2d_march.h"
#include "op_stencil3d.h"
#include "op_csr.h"
#include "op_weights.h"
#include "kernel_table.h"
#include "solver_kernel.h"

using namespace kiops;

struct kiops_operator {
  kiops_operator_desc d;
  hipStream_t stream;
  int device;
  int cus;
  uint64_t clock_hz;
  int64_t N;
  void* ws;
  size_t ws_bytes;
};

struct kiops_server;

namespace kiops {

// Barrier words and control block before a launch (one workgroup).
__global__ void kiops_reset_kernel(Barrier* b, Ctrl* c, unsigned* arrive, int nwg, uint64_t* arrive_t,
                                   uint64_t* tctx) {
  for (int i = threadIdx.x; i < nwg; i += blockDim.x) arrive[i] = 0u;
  for (int i = threadIdx.x; i < kCtxWords; i += blockDim.x) tctx[i] = 0u;
  for (int i = threadIdx.x; i < 3 * nwg; i += blockDim.x) arrive_t[i] = 0u;
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    b->gen = 0;
    b->abort = 0;
    c->phase = kPhaseDone;
    c->status = KIOPS_OK;
    c->t_work = c->t_wait = c->t_epi = 0;
    c->t_expm = c->t_arrive_max = c->t_arrive_mean = c->n_barriers = 0;
    c->t_red = c->t_pub = c->t_ser = 0;
    c->t_release_max = c->t_release_mean = 0;
  }
}

}  // namespace kiops

namespace {

constexpr size_t kAlign = 256;
constexpr int kGridExpmFrom = 96;   // padded basis size from which the exponential is spread over the grid
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t params, ctrl, bar, arrive, arrive_t, tctx, H, G, Y, sinv, coefc, fullc, partials, dpart, expm, trace, cgsave,
      slots, ubuf, bcopy, coef, total;
  int nwg, ndot_stride, q;
};

int elem_size(const kiops_operator* op) { return op->d.precision == KIOPS_MIXED ? 4 : 8; }

// Weights per cell of the general stencil form: 5 in 2-D, 7 in 3-D.
int weight_count(const kiops_operator* op) { return op->d.kind == KIOPS_OP_STENCIL2D_5PT ? 5 : 7; }

// Per-element coefficient streams a pass reads (algorithmic bytes, in units of
// one basis element): r and kappa for stencils; for CSR the matrix (values and
// column indices), the row pointers, and U_{k-1} read, U_k written and R_k read
// again by the product.
double coef_streams(const kiops_operator* op) {
  if (op->d.weights) return (double)weight_count(op) + 3.0;   // the weights, and U and R_k as for CSR
  if (op->d.kind == KIOPS_OP_CSR) {
    const double s = (double)elem_size(op);
    return (double)op->d.nnz / (double)op->N * (s + 4.0) / s + 4.0 / s + 3.0;
  }
  int c = 0;
  if (op->d.reaction) ++c;
  if (op->d.kappa) ++c;
  return c;
}

// Elements of T in the mixed-precision coefficient copies.
size_t coef_copy_elems(const kiops_operator* op) {
  if (op->d.weights) return (size_t)weight_count(op) * (size_t)op->N;
  if (op->d.kind == KIOPS_OP_CSR) return (size_t)op->d.nnz;
  return (size_t)((op->d.reaction ? 1 : 0) + (op->d.kappa ? 1 : 0)) * (size_t)op->N;
}

// Compile-time bound on p used by the stencil passes.
int p_bucket(int p) { return p == 0 ? 0 : (p <= 2 ? 2 : (p <= 4 ? 4 : 8)); }

// The 7-point marching pass serves 3-D operators and 2-D ones with a
// diffusivity field (nz = 1); the 5-point tile pass serves constant-diffusivity 2-D.
bool uses_3d(const kiops_operator* op) {
  if (op->d.weights) return false;   // the general form has a pass of its own
  return op->d.kind == KIOPS_OP_STENCIL3D_7PT || (op->d.kind == KIOPS_OP_STENCIL2D_5PT && op->d.kappa);
}

// z planes per work item of the marching pass (nominal; sizes the grid).
// FP64, whose chunks alternate their march direction: 16 (256^3: 7.65 solves/s
// against 7.48 with 24, 7.27 with 32, 6.97 with 12); the mixed form, marching
// in one direction: 24 (1.5% faster than 16 and 2% faster than 32, measured
// in FP64 before the alternation).
int zchunk(const kiops_operator* op) {
  return (int)std::min<int64_t>(op->d.precision == KIOPS_MIXED ? 24 : 16, op->d.nz);
}

// Number of z chunks for a grid of nwg workgroups: about nz / zchunk, raised (by at
// most half) so that the item count is a multiple of the grid when that is
// reachable, which gives every workgroup the same number of items.
int zchunks(const kiops_operator* op, int nwg) {
  using S = Stencil3D<double, 2>;
  const int64_t txy = ((op->d.nx + S::TX - 1) / S::TX) * ((op->d.ny + S::TY - 1) / S::TY);
  const int64_t nz = op->d.nz;
  const int64_t base = (nz + zchunk(op) - 1) / zchunk(op);
  for (int64_t c = base; c <= std::min<int64_t>(nz, base + base / 2); ++c)
    if ((txy * c) % nwg == 0) return (int)c;
  return (int)base;
}

// The row-marching 5-point pass (op_stencil2d_march.h) serves the one-solve
// kernel of large constant-diffusivity 2-D grids with windows of one or two
// vectors: strips of 256 columns, chunks of about 32 rows, enough items to
// give every CU work.  KIOPS_MARCH=0 selects the tile pass instead, and
// KIOPS_MARCH=2 the marching pass whenever the window allows it (tests).
int march_chunks(const kiops_operator* op) {   // chunks of at most kChunkRows rows (the march unrolls them)
  const int64_t c = Stencil2DMarch<double, 2>::kChunkRows;
  return (int)std::max<int64_t>(1, (op->d.ny + c - 1) / c);
}
int64_t march_items(const kiops_operator* op) {
  const int64_t W = Stencil2DMarch<double, 2>::W;
  return (op->d.nx + W - 1) / W * march_chunks(op);
}
bool use_march(const kiops_operator* op, int q) {
  if (op->d.kind != KIOPS_OP_STENCIL2D_5PT || op->d.kappa || (q != 1 && q != 2)) return false;
  const char* e = std::getenv("KIOPS_MARCH");   // experiment / test override
  const int mode = e ? std::atoi(e) : 1;
  if (mode == 0) return false;
  if (mode >= 2) return true;
  return op->d.nx >= Stencil2DMarch<double, 2>::W && march_items(op) >= op->cus;
}

// The pass a one-solve kernel runs for this operator and window (KIOPS_PASS_*).
int pass_kind(const kiops_operator* op, int q) {
  if (op->d.weights) return KIOPS_PASS_WEIGHTS;
  if (uses_3d(op)) return KIOPS_PASS_7PT;
  if (op->d.kind == KIOPS_OP_CSR) return KIOPS_PASS_CSR;
  if (use_march(op, q)) return KIOPS_PASS_MARCH2D;
  return (q == 3 || q == 4) ? KIOPS_PASS_WIDE2D : KIOPS_PASS_TILE2D;
}

// Kernel of an operator for p-bucket pb: the one-solve kernel or the group
// kernel; wide: the 5-point one-solve kernel for IOP windows of 3 and 4;
// march: the row-marching 5-point one-solve kernel; narrow: the 7-point
// one-solve kernel for IOP windows of 1 and 2.
const void* kernel_for_bucket(const kiops_operator* op, int pb, bool group, bool wide = false, bool march = false,
                              bool narrow = false, int tile_rows = 16) {
  const bool mixed = op->d.precision == KIOPS_MIXED;
  if (op->d.weights) return kernels_weights(mixed, pb, group);
  if (uses_3d(op)) return kernels_stencil3d(mixed, pb, group, narrow);
  if (op->d.kind == KIOPS_OP_STENCIL2D_5PT) {
    if (march && !group) return kernels_stencil2d_march(mixed, pb);
    return kernels_stencil2d(mixed, pb, group, wide, tile_rows);
  }
  if (op->d.kind == KIOPS_OP_CSR) return kernels_csr(mixed, pb, group);
  return nullptr;
}

// The one-solve kernel instantiation that serves an operator, p and the IOP window q.
const void* kernel_for(const kiops_operator* op, int p, int q) {
  return kernel_for_bucket(op, p_bucket(p), false, q == 3 || q == 4, use_march(op, q), q == 1 || q == 2);
}

// Work items of the pass: tiles (2-D tile pass, 64 x tile_rows), columns x z
// chunks (7-point pass), strips x row chunks (2-D marching pass), row blocks (CSR).
int64_t work_tiles(const kiops_operator* op, bool march = false, int tile_rows = 16) {
  if (march) return march_items(op);
  if (op->d.weights) return (op->N + kThreads - 1) / kThreads;   // row blocks
  if (uses_3d(op)) {
    using S = Stencil3D<double, 2>;
    const int64_t tx = (op->d.nx + S::TX - 1) / S::TX;
    const int64_t ty = (op->d.ny + S::TY - 1) / S::TY;
    const int64_t zc = zchunk(op);
    return tx * ty * ((op->d.nz + zc - 1) / zc);
  }
  if (op->d.kind == KIOPS_OP_STENCIL2D_5PT) {
    const int64_t tx = (op->d.nx + Stencil2D<double, 2>::TX - 1) / Stencil2D<double, 2>::TX;
    const int64_t ty = (op->d.ny + tile_rows - 1) / tile_rows;
    return tx * ty;
  }
  if (op->d.kind == KIOPS_OP_CSR) return (op->N + kThreads - 1) / kThreads;   // row blocks
  return 1;
}

// Persistent grid: all workgroups co-resident, no more than the tiles of work.
kiops_status grid_size(const kiops_operator* op, int p, int q, int* nwg) {
  const void* fn = kernel_for(op, p, q);
  if (!fn) return KIOPS_ERR_UNSUPPORTED;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads, 0) != hipSuccess || per_cu < 1)
    return KIOPS_ERR_DEVICE;
  // The 5-point tile pass runs best with two workgroups per CU (measured at
  // 2048^2: 110 us per Krylov step against 120 us with three); the marching
  // 7-point pass with all that fit.
  const char* pc = std::getenv("KIOPS_PER_CU");   // experiment override of the 2-D choice
  if (!uses_3d(op)) per_cu = std::min(per_cu, pc && std::atoi(pc) > 0 ? std::atoi(pc) : 2);
  int64_t g = (int64_t)per_cu * op->cus;
  const char* ov = std::getenv("KIOPS_GRID");   // experiment override, capped by co-residency
  if (ov && std::atoi(ov) > 0) g = std::min<int64_t>(g, std::atoi(ov));
  else g = std::min<int64_t>(g, std::max<int64_t>(1, work_tiles(op, use_march(op, q))));
  *nwg = (int)g;
  return KIOPS_OK;
}

// The error estimate an options block asks for (KIOPS_ESTIMATE_*), or -1 if invalid.
int resolve_estimate(const kiops_options* o) {
  const int e = o ? o->estimate : KIOPS_ESTIMATE_ONE_TERM;
  return (e >= KIOPS_ESTIMATE_ONE_TERM && e <= KIOPS_ESTIMATE_CORRECTED) ? e : -1;
}

// Default m_max: 128 (Section 3.6.2); 32 for the mixed form, whose FP32 basis
// loses accuracy over long recurrences (measured relative errors at m_max 128 /
// 64 / 32: 2.6e-4 / 6.7e-6 / 1.6e-6 on the 256^3 constant-coefficient box,
// 1.8e-4 / 1.8e-4 / 9.9e-7 and 3.2e-5 / 3.2e-5 / 5.6e-6 on small 3-D boxes
// with tau ||A||_1 of 306 and 101).
void resolve_options(const kiops_operator* op, const kiops_options* o, int* m_min, int* m_max,
                     int* max_sub) {
  const int m_default = op->d.precision == KIOPS_MIXED ? 32 : 128;
  *m_min = (o && o->m_min > 0) ? o->m_min : 10;
  *m_max = (o && o->m_max > 0) ? o->m_max : m_default;
  *max_sub = (o && o->max_substeps > 0) ? o->max_substeps : 100000;
}

Layout make_layout(const kiops_operator* op, int p, int q, int m_max, int nwg) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t at = off; off = align_up(off + bytes); return at; };
  L.nwg = nwg;
  L.q = q;
  L.ndot_stride = std::max(kPM, kDotSlots);
  L.params = take(4096);   // KParams followed by the operator struct
  L.ctrl = take(sizeof(Ctrl));
  L.bar = take(sizeof(Barrier));
  L.arrive = take(sizeof(unsigned) * (size_t)nwg);
  L.arrive_t = take(sizeof(uint64_t) * 3 * (size_t)nwg);
  L.tctx = take(sizeof(uint64_t) * kCtxWords);   // release words: zero before a launch, like the barrier words
  L.H = take(sizeof(double) * kLdh * kLdh);
  L.G = take(sizeof(double) * kLdh * kLdh);
  L.Y = take(sizeof(double) * kLdh * kPM);
  L.sinv = take(sizeof(double) * kLdh);
  L.coefc = take(sizeof(double) * kLdh);
  L.fullc = take(sizeof(double) * 2 * kLdh);
  L.partials = take(sizeof(double) * (size_t)nwg * L.ndot_stride);
  L.dpart = take(q == 0 ? sizeof(double) * (size_t)nwg * kDotFullStride : 0);
  L.expm = take(sizeof(double) * (size_t)kExpmSlots * kExpmSlot);
  L.trace = take(sizeof(double) * (size_t)kTraceMax * kTraceStride);
  L.cgsave = take(sizeof(double) * kLdh);
  const size_t es = (size_t)elem_size(op);
  L.slots = take(es * (size_t)(m_max + 1) * (size_t)op->N);
  L.ubuf = take((q == 0 || op->d.kind == KIOPS_OP_CSR || op->d.weights) ? es * (size_t)op->N : 0);
  L.bcopy = take(op->d.precision == KIOPS_MIXED ? es * (size_t)p * op->N : 0);
  L.coef = take(op->d.precision == KIOPS_MIXED ? es * coef_copy_elems(op) : 0);
  L.total = off;
  return L;
}

// A failed HIP call; with KIOPS_DEBUG=1 in the environment it is reported on stderr.
bool hip_ok(hipError_t e) {
  if (e == hipSuccess) return true;
  static const bool debug = [] {
    const char* v = std::getenv("KIOPS_DEBUG");
    return v && std::atoi(v) > 0;
  }();
  if (debug) std::fprintf(stderr, "kiops: HIP error %d: %s\n", (int)e, hipGetErrorString(e));
  return false;
}

template <typename T, int PB, int kTY = 16>
Stencil2DT<T, PB, false, kTY> make_stencil2d(const kiops_operator* op, int p, const double* const* V, char* ws,
                                             const Layout& L) {
  using S2 = Stencil2DT<T, PB, false, kTY>;
  const auto& d = op->d;
  S2 s{};
  s.N = op->N;
  s.nx = (int)d.nx;
  s.ny = (int)d.ny;
  s.tiles_x = (int)((d.nx + S2::TX - 1) / S2::TX);
  const int tiles_y = (int)((d.ny + S2::TY - 1) / S2::TY);
  s.ntiles = s.tiles_x * tiles_y;
  const double cD = d.diff / (d.h * d.h);
  const double cx = d.adv[0] / (2.0 * d.h);
  const double cy = d.adv[1] / (2.0 * d.h);
  s.wE = (T)(cD - cx);
  s.wW = (T)(cD + cx);
  s.wN = (T)(cD - cy);
  s.wS = (T)(cD + cy);
  s.wC = (T)(-4.0 * cD);
  s.p = p;
  s.ubuf = L.q == 0 ? reinterpret_cast<T*>(ws + L.ubuf) : nullptr;
  const bool mixed = d.precision == KIOPS_MIXED;
  for (int c = 0; c < kPM; ++c) s.B[c] = nullptr;
  if (mixed) {
    T* bc = reinterpret_cast<T*>(ws + L.bcopy);
    for (int c = 0; c < p; ++c) s.B[c] = bc + (size_t)c * op->N;
    s.r_src = d.reaction;
    s.r_dst = d.reaction ? reinterpret_cast<T*>(ws + L.coef) : nullptr;
    s.r = s.r_dst;
  } else {
    for (int c = 0; c < p; ++c) s.B[c] = reinterpret_cast<const T*>(V[p - c]);
    s.r = reinterpret_cast<const T*>(d.reaction);
    s.r_src = nullptr;
    s.r_dst = nullptr;
  }
  return s;
}

template <typename T, int PB>
Stencil2DRows8<T, PB> make_stencil2d_rows8(const kiops_operator* op, int p, const double* const* V, char* ws,
                                           const Layout& L) {
  return make_stencil2d<T, PB, 8>(op, p, V, ws, L);
}
template <typename T, int PB>
Stencil2DRows4<T, PB> make_stencil2d_rows4(const kiops_operator* op, int p, const double* const* V, char* ws,
                                           const Layout& L) {
  return make_stencil2d<T, PB, 4>(op, p, V, ws, L);
}

template <typename T, int PB>
Stencil2DMarch<T, PB> make_stencil2d_march(const kiops_operator* op, int p, const double* const* V, char* ws,
                                           const Layout& L) {
  const Stencil2D<T, PB> t = make_stencil2d<T, PB>(op, p, V, ws, L);   // coefficients and arrays
  Stencil2DMarch<T, PB> s{};
  s.N = t.N;
  s.nx = t.nx;
  s.ny = t.ny;
  s.nstrips = (int)((op->d.nx + Stencil2DMarch<T, PB>::W - 1) / Stencil2DMarch<T, PB>::W);
  s.nchunks = march_chunks(op);
  s.nitems = s.nstrips * s.nchunks;
  s.wE = t.wE; s.wW = t.wW; s.wN = t.wN; s.wS = t.wS; s.wC = t.wC;
  s.r = t.r;
  for (int c = 0; c < kPM; ++c) s.B[c] = t.B[c];
  s.p = t.p;
  s.r_src = t.r_src;
  s.r_dst = t.r_dst;
  s.ubuf = nullptr;
  return s;
}

template <typename T, int PB>
Stencil3D<T, PB> make_stencil3d(const kiops_operator* op, int p, const double* const* V, char* ws,
                                const Layout& L) {
  const auto& d = op->d;
  Stencil3D<T, PB> s{};
  s.N = op->N;
  s.nx = (int)d.nx;
  s.ny = (int)d.ny;
  s.nz = (int)d.nz;
  s.tiles_x = (int)((d.nx + Stencil3D<T, PB>::TX - 1) / Stencil3D<T, PB>::TX);
  s.tiles_y = (int)((d.ny + Stencil3D<T, PB>::TY - 1) / Stencil3D<T, PB>::TY);
  s.nchunks = zchunks(op, L.nwg);
  s.nitems = s.tiles_x * s.tiles_y * s.nchunks;
  s.h2inv = (T)(1.0 / (d.h * d.h));
  s.half_h2inv = (T)(0.5 / (d.h * d.h));
  s.cx = (T)(d.adv[0] / (2.0 * d.h));
  s.cy = (T)(d.adv[1] / (2.0 * d.h));
  s.cz = (T)(d.adv[2] / (2.0 * d.h));
  s.diff = (T)d.diff;
  s.p = p;
  s.ubuf = L.q == 0 ? reinterpret_cast<T*>(ws + L.ubuf) : nullptr;
  const bool mixed = d.precision == KIOPS_MIXED;
  for (int c = 0; c < kPM; ++c) s.B[c] = nullptr;
  if (mixed) {
    T* bc = reinterpret_cast<T*>(ws + L.bcopy);
    for (int c = 0; c < p; ++c) s.B[c] = bc + (size_t)c * op->N;
    T* coef = reinterpret_cast<T*>(ws + L.coef);
    s.r_src = d.reaction;
    s.r_dst = d.reaction ? coef : nullptr;
    s.r = s.r_dst;
    s.k_src = d.kappa;
    s.k_dst = d.kappa ? coef + (d.reaction ? (size_t)op->N : 0) : nullptr;
    s.kappa = s.k_dst;
  } else {
    for (int c = 0; c < p; ++c) s.B[c] = reinterpret_cast<const T*>(V[p - c]);
    s.r = reinterpret_cast<const T*>(d.reaction);
    s.kappa = reinterpret_cast<const T*>(d.kappa);
    s.r_src = s.k_src = nullptr;
    s.r_dst = s.k_dst = nullptr;
  }
  return s;
}

template <typename T, int PB>
CsrOp<T, PB> make_csr(const kiops_operator* op, int p, const double* const* V, char* ws, const Layout& L) {
  const auto& d = op->d;
  CsrOp<T, PB> s{};
  s.N = op->N;
  s.nnz = d.nnz;
  s.rowptr = d.rowptr;
  s.col = d.col;
  s.p = p;
  s.ubuf = reinterpret_cast<T*>(ws + L.ubuf);
  for (int c = 0; c < kPM; ++c) s.B[c] = nullptr;
  if (d.precision == KIOPS_MIXED) {
    T* bc = reinterpret_cast<T*>(ws + L.bcopy);
    for (int c = 0; c < p; ++c) s.B[c] = bc + (size_t)c * op->N;
    s.v_src = d.val;
    s.v_dst = reinterpret_cast<T*>(ws + L.coef);
    s.val = s.v_dst;
  } else {
    for (int c = 0; c < p; ++c) s.B[c] = reinterpret_cast<const T*>(V[p - c]);
    s.val = reinterpret_cast<const T*>(d.val);
    s.v_src = nullptr;
    s.v_dst = nullptr;
  }
  return s;
}

template <typename T, int PB>
WeightsOp<T, PB> make_weights(const kiops_operator* op, int p, const double* const* V, char* ws,
                              const Layout& L) {
  const auto& d = op->d;
  WeightsOp<T, PB> s{};
  s.N = op->N;
  s.nx = (int)d.nx;
  s.ny = (int)d.ny;
  s.nz = (int)d.nz;
  s.nw = weight_count(op);
  s.p = p;
  s.ubuf = reinterpret_cast<T*>(ws + L.ubuf);
  for (int c = 0; c < kPM; ++c) s.B[c] = nullptr;
  if (d.precision == KIOPS_MIXED) {
    T* bc = reinterpret_cast<T*>(ws + L.bcopy);
    for (int c = 0; c < p; ++c) s.B[c] = bc + (size_t)c * op->N;
    s.w_src = d.weights;
    s.w_dst = reinterpret_cast<T*>(ws + L.coef);
    s.W = s.w_dst;
  } else {
    for (int c = 0; c < p; ++c) s.B[c] = reinterpret_cast<const T*>(V[p - c]);
    s.W = reinterpret_cast<const T*>(d.weights);
    s.w_src = nullptr;
    s.w_dst = nullptr;
  }
  return s;
}

KParams make_params(const kiops_operator* op, const Layout& L, char* ws, double tau, int p,
                    const double* const* V, double tol, int m_init, int q, int m_min, int m_max,
                    int max_sub, int mode, double* w) {
  KParams P{};
  P.N = op->N;
  P.p = p;
  P.q = q;
  P.m_min = m_min;
  P.m_max = m_max;
  P.m_init = m_init;
  P.max_substeps = max_sub;
  P.mode = mode;
  P.mixed = op->d.precision == KIOPS_MIXED;
  P.nwg = L.nwg;
  P.ndot_stride = L.ndot_stride;
  P.T_end = tau;
  P.tol = tol;
  P.elem_bytes = (double)elem_size(op);
  P.coef_streams = coef_streams(op);
  P.spin_limit = op->clock_hz * 60ull;   // a minute without progress aborts the solve
  for (int k = 0; k <= kPM; ++k) P.b[k] = (k <= p) ? V[k] : nullptr;
  P.w = w;
  P.slots = ws + L.slots;
  P.bcopy = ws + L.bcopy;
  P.ctrl = reinterpret_cast<Ctrl*>(ws + L.ctrl);
  P.bar = reinterpret_cast<Barrier*>(ws + L.bar);
  P.arrive = reinterpret_cast<unsigned*>(ws + L.arrive);
  P.arrive_t = reinterpret_cast<uint64_t*>(ws + L.arrive_t);
  P.tctx = reinterpret_cast<uint64_t*>(ws + L.tctx);
  const char* ps = std::getenv("KIOPS_POLL_SLEEP");   // experiment override
  P.poll_sleep = ps ? std::max(0, std::min(64, std::atoi(ps))) : 1;
  P.ranks = 1;
  // the attempt's small exponential runs on the whole grid from this padded
  // size on (one workgroup below it, where a product is cheaper than a barrier)
  const char* ge = std::getenv("KIOPS_GRID_EXPM");   // experiment override (0: never)
  P.expm_grid = ge ? std::max(0, std::atoi(ge)) : kGridExpmFrom;
  const char* prof = std::getenv("KIOPS_PROFILE");
  P.profile = (prof && std::atoi(prof) > 0) ? 1 : 0;
  P.H = reinterpret_cast<double*>(ws + L.H);
  P.G = reinterpret_cast<double*>(ws + L.G);
  P.Y = reinterpret_cast<double*>(ws + L.Y);
  P.sinv = reinterpret_cast<double*>(ws + L.sinv);
  P.coefc = reinterpret_cast<double*>(ws + L.coefc);
  P.fullc = reinterpret_cast<double*>(ws + L.fullc);
  P.dpart = reinterpret_cast<double*>(ws + L.dpart);
  P.ubuf = (q == 0 || op->d.kind == KIOPS_OP_CSR || op->d.weights) ? ws + L.ubuf : nullptr;
  P.partials = reinterpret_cast<double*>(ws + L.partials);
  P.expm = reinterpret_cast<double*>(ws + L.expm);
  P.trace = reinterpret_cast<double*>(ws + L.trace);
  P.cgsave = reinterpret_cast<double*>(ws + L.cgsave);
  P.ntimes = 1;           // one output, at T_end (Task II)
  P.task1 = 0;
  P.times[0] = tau;
  P.wout[0] = w;
  return P;
}

template <class OpT>
void stage_op(unsigned char* host_block, const OpT& o) {
  static_assert(sizeof(OpT) <= 2048, "operator block");
  std::memcpy(host_block + 2048, &o, sizeof(OpT));
}

// Write the operator struct of the kernel instantiation for p-bucket pb
// (pb >= p) into blk + 2048.
kiops_status stage_op_block(const kiops_operator* op, int p, int pb, const double* const* V, char* ws,
                            const Layout& L, unsigned char* blk, bool march = false, int tile_rows = 16) {
  const bool mixed = op->d.precision == KIOPS_MIXED;
#define KIOPS_STAGE(MAKE)                                                                          \
  switch (pb) {                                                                                    \
    case 0: mixed ? stage_op(blk, MAKE<float, 0>(op, p, V, ws, L)) : stage_op(blk, MAKE<double, 0>(op, p, V, ws, L)); break; \
    case 2: mixed ? stage_op(blk, MAKE<float, 2>(op, p, V, ws, L)) : stage_op(blk, MAKE<double, 2>(op, p, V, ws, L)); break; \
    case 4: mixed ? stage_op(blk, MAKE<float, 4>(op, p, V, ws, L)) : stage_op(blk, MAKE<double, 4>(op, p, V, ws, L)); break; \
    default: mixed ? stage_op(blk, MAKE<float, 8>(op, p, V, ws, L)) : stage_op(blk, MAKE<double, 8>(op, p, V, ws, L)); break; \
  }
  if (op->d.weights) {
    KIOPS_STAGE(make_weights)
  } else if (uses_3d(op)) {
    KIOPS_STAGE(make_stencil3d)
  } else if (op->d.kind == KIOPS_OP_CSR) {
    KIOPS_STAGE(make_csr)
  } else if (op->d.kind == KIOPS_OP_STENCIL2D_5PT && march) {
    KIOPS_STAGE(make_stencil2d_march)
  } else if (op->d.kind == KIOPS_OP_STENCIL2D_5PT && tile_rows == 8) {
    KIOPS_STAGE(make_stencil2d_rows8)
  } else if (op->d.kind == KIOPS_OP_STENCIL2D_5PT && tile_rows == 4) {
    KIOPS_STAGE(make_stencil2d_rows4)
  } else if (op->d.kind == KIOPS_OP_STENCIL2D_5PT) {
    KIOPS_STAGE(make_stencil2d)
  } else {
    return KIOPS_ERR_UNSUPPORTED;
  }
#undef KIOPS_STAGE
  return KIOPS_OK;
}

// Group-kernel instantiation (batched and served forms) for p-bucket pb and,
// for the 2-D tile pass, tiles of tile_rows rows.
const void* group_kernel_for(const kiops_operator* op, int pb, int tile_rows = 16) {
  return kernel_for_bucket(op, pb, true, false, false, false, tile_rows);
}

// kiops_options.tile_rows of the batched form: 16 (0), 8 or 4; -1 if invalid.
int resolve_tile_rows(const kiops_options* o) {
  const int r = o ? o->tile_rows : 0;
  if (r == 0) return 16;
  return (r == 16 || r == 8 || r == 4) ? r : -1;
}

// Kernel family of an operator: instances of one batch must share it.
int op_family(const kiops_operator* op) {
  const int k = op->d.weights ? 3 : (uses_3d(op) ? 1 : (op->d.kind == KIOPS_OP_CSR ? 2 : 0));
  return k * 2 + (op->d.precision == KIOPS_MIXED ? 1 : 0);
}

// Launch one persistent solve and wait for its control block.
kiops_status run_solve(kiops_operator* op, char* ws, const Layout& L, KParams& P, int p, const double* const* V,
                       Ctrl* host_ctrl, unsigned* host_abort) {
  hipLaunchKernelGGL(kiops_reset_kernel, dim3(1), dim3(256), 0, op->stream, P.bar, P.ctrl, P.arrive, L.nwg,
                     P.arrive_t, P.tctx);
  if (!hip_ok(hipGetLastError())) return KIOPS_ERR_DEVICE;
  hipError_t e = hipSuccess;
  // parameter block: KParams at +0, operator struct at +2048 (host staging buffer)
  static_assert(sizeof(KParams) <= 2048, "params block");
  // workgroups per CU when the grid fills every CU evenly (the 7-point pass
  // deals more items to the workgroups placed first on a CU)
  P.ranks = (uses_3d(op) && L.nwg % op->cus == 0 && L.nwg / op->cus <= 4) ? L.nwg / op->cus : 1;
  // the marching 5-point pass balances the two workgroups of a CU by wave priority
  if (use_march(op, P.q) && L.nwg == 2 * op->cus) P.ranks = 2;
  const char* rk = std::getenv("KIOPS_RANKS");   // experiment override
  if (rk) P.ranks = std::max(1, std::min(4, std::atoi(rk)));
  alignas(256) unsigned char host_block[4096];
  std::memset(host_block, 0, sizeof(host_block));
  std::memcpy(host_block, &P, sizeof(KParams));
  KParams* dP = reinterpret_cast<KParams*>(ws + L.params);
  void* dOp = ws + L.params + 2048;
  const void* fn = kernel_for(op, p, P.q);
  if (!fn) return KIOPS_ERR_UNSUPPORTED;
  kiops_status st = stage_op_block(op, p, p_bucket(p), V, ws, L, host_block, use_march(op, P.q));
  if (st != KIOPS_OK) return st;
  if (!hip_ok(hipMemcpyAsync(dP, host_block, sizeof(host_block), hipMemcpyHostToDevice, op->stream)))
    return KIOPS_ERR_DEVICE;
  {
    void* args[] = {&dP, &dOp};
    const char* pad = std::getenv("KIOPS_PAD_LDS");   // experiment: unused dynamic LDS per workgroup
    const unsigned dyn = pad ? (unsigned)std::max(0, std::min(65536, std::atoi(pad))) : 0u;
    e = hipLaunchCooperativeKernel(fn, dim3(L.nwg), dim3(kThreads), args, dyn, op->stream);
  }
  if (!hip_ok(e)) return KIOPS_ERR_DEVICE;
  Barrier hb{};
  if (!hip_ok(hipMemcpyAsync(host_ctrl, P.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, op->stream)))
    return KIOPS_ERR_DEVICE;
  if (!hip_ok(hipMemcpyAsync(&hb, P.bar, sizeof(Barrier), hipMemcpyDeviceToHost, op->stream)))
    return KIOPS_ERR_DEVICE;
  if (!hip_ok(hipStreamSynchronize(op->stream))) return KIOPS_ERR_DEVICE;
  *host_abort = hb.abort;
  return KIOPS_OK;
}

void fill_stats(const Ctrl& c, int nwg, double clock_hz, kiops_stats* st) {
  if (!st) return;
  st->time_work_s = (double)c.t_work / clock_hz;
  st->time_wait_s = (double)c.t_wait / clock_hz;
  st->time_epilogue_s = (double)c.t_epi / clock_hz;
  st->time_expm_s = (double)c.t_expm / clock_hz;
  st->arrive_max_s = (double)c.t_arrive_max / clock_hz;
  st->arrive_mean_s = (double)c.t_arrive_mean / clock_hz;
  st->release_max_s = (double)c.t_release_max / clock_hz;
  st->release_mean_s = (double)c.t_release_mean / clock_hz;
  st->barriers = (int64_t)c.n_barriers;
  st->m_last = c.m;
  st->substeps = c.substeps;
  st->rejections = c.rejections;
  st->expms = c.expms;
  st->breakdowns = c.breakdowns;
  st->grid_blocks = nwg;
  st->matvecs = c.matvecs;
  st->last_omega = c.last_omega;
  st->t_reached = c.T_now;
  st->alg_bytes = c.alg_bytes;
  st->beta_last = c.beta;
  st->status = c.status;
  st->m_max = c.m_max;
  st->time_reduce_s = (double)c.t_red / clock_hz;
  st->time_publish_s = (double)c.t_pub / clock_hz;
  st->time_serial_s = (double)c.t_ser / clock_hz;
  st->clock_start_s = (double)c.t_begin / clock_hz;
  st->clock_end_s = (double)c.t_end / clock_hz;
}

kiops_status check_vectors(const kiops_operator* op, int p, const double* const* V, const double* w) {
  if (!V || !w || p < 0 || p > KIOPS_P_MAX) return KIOPS_ERR_INVALID_ARG;
  const size_t bytes = sizeof(double) * (size_t)op->N;
  for (int k = 0; k <= p; ++k) {
    if (!V[k]) return KIOPS_ERR_INVALID_ARG;
    if (k > 0) {
      const char* a = reinterpret_cast<const char*>(V[k]);
      const char* b = reinterpret_cast<const char*>(w);
      if (a < b + bytes && b < a + bytes) return KIOPS_ERR_INVALID_ARG;   // w overlaps b_k, k >= 1
    }
  }
  return KIOPS_OK;
}

__global__ void export_basis_kernel(const void* slots, const double* w, int mixed, int64_t N, int p,
                                    int nvec, const double* sinv, const double* Y, double* out) {
  const int64_t stride = N + p;
  const int64_t total = (int64_t)nvec * stride;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / stride) + 1;       // basis index, 1-based
    const int64_t n = e % stride;
    double v;
    if (n < N) {
      if (i == 1 && !mixed) v = w[n];
      else if (mixed) v = (double)reinterpret_cast<const float*>(slots)[(int64_t)(i - 1) * N + n];
      else v = reinterpret_cast<const double*>(slots)[(int64_t)(i - 1) * N + n];
    } else {
      v = Y[i * kPM + (n - N)];
    }
    out[e] = v * sinv[i];
  }
}

__global__ void export_h_kernel(const double* H, int m, double* out) {
  for (int e = threadIdx.x; e < (m + 1) * m; e += blockDim.x) {
    const int r = e / m, c = e % m;
    out[e] = H[(r + 1) * kLdh + (c + 1)];
  }
}

__global__ void small_expm_kernel(const double* Hs, int n, double tau, double* F, double* scratch) {
  __shared__ double lds[kLdsDoubles];
  const int n16 = pad16(n);
  double colmax = 0.0;
  for (int c = threadIdx.x; c < n16; c += kThreads) {
    double cs = 0.0;
    for (int r = 0; r < n16; ++r) {
      const double v = (r < n && c < n) ? tau * Hs[r * n + c] : 0.0;
      scratch[r * kExpmLd + c] = v;
      cs += fabs(v);
    }
    colmax = cs > colmax ? cs : colmax;
  }
  const double eta = wg_max(colmax, lds);
  const int slot = wg_expm(scratch, n, eta, lds);
  const double* R = scratch + (size_t)slot * kExpmSlot;
  for (int e = threadIdx.x; e < n * n; e += kThreads) F[e] = R[(e / n) * kExpmLd + (e % n)];
}

// ---------------------------------------------------------------- batches

struct BatchPlan {
  int gs = 0, ng = 0, pb = 0, m_min = 0, m_max = 0, max_sub = 0;
  int tile_rows = 16;                   // 2-D tile pass: rows per tile
  int nwg = 0;                          // workgroups of the launch
  const void* fn = nullptr;
  std::vector<int> gsize, wg0;          // per group: workgroups and the first of them
  std::vector<int> group_of;            // problem -> group
  std::vector<std::vector<int>> members;
  std::vector<size_t> group_off;        // group workspace offsets
  size_t ctrl_off = 0, block_off = 0, queue_off = 0, map_off = 0, total = 0;
};

size_t ctrl_stride() { return align_up(sizeof(Ctrl)); }

// Work estimate of a problem for the assignment: N times (1 + tau ||A||_1),
// ||A||_1 bounded from the operator description.
double work_estimate(const kiops_problem& pr) {
  const kiops_operator_desc& d = pr.op->d;
  double a = 1.0;
  if (d.kind != KIOPS_OP_CSR) {
    const int dims = d.nz > 1 ? 3 : 2;
    const double kap = d.kappa ? 1.0 : std::fabs(d.diff);
    a += 4.0 * dims * kap / (d.h * d.h) + (std::fabs(d.adv[0]) + std::fabs(d.adv[1]) + std::fabs(d.adv[2])) / d.h;
  } else {
    a += 10.0 * (double)d.nnz / (double)std::max<int64_t>(1, d.nrows);
  }
  return (double)pr.op->N * (1.0 + pr.tau * a);
}

kiops_status plan_batch(int count, const kiops_problem* probs, const kiops_options* opts, int group_size,
                        BatchPlan& B) {
  if (count < 1 || !probs) return KIOPS_ERR_INVALID_ARG;
  int pmax = 0;
  for (int i = 0; i < count; ++i) {
    const kiops_problem& pr = probs[i];
    if (!pr.op || !(pr.tau >= 0.0) || !std::isfinite(pr.tau) || !(pr.tol > 0.0) || !std::isfinite(pr.tol) ||
        pr.m_init < 1 || pr.q < 0 || pr.q > 8)
      return KIOPS_ERR_INVALID_ARG;
    kiops_status s = check_vectors(pr.op, pr.p, pr.V, pr.w);
    if (s != KIOPS_OK) return s;
    if (pr.q > kWinMax) return KIOPS_ERR_UNSUPPORTED;
    if (op_family(pr.op) != op_family(probs[0].op)) return KIOPS_ERR_UNSUPPORTED;
    pmax = std::max(pmax, pr.p);
  }
  resolve_options(probs[0].op, opts, &B.m_min, &B.m_max, &B.max_sub);
  if (B.m_max > KIOPS_M_MAX_LIMIT || B.m_min > B.m_max || B.m_min < 1) return KIOPS_ERR_INVALID_ARG;
  if (resolve_estimate(opts) != KIOPS_ESTIMATE_ONE_TERM) return KIOPS_ERR_UNSUPPORTED;
  B.tile_rows = resolve_tile_rows(opts);
  if (B.tile_rows < 0) return KIOPS_ERR_INVALID_ARG;
  B.pb = p_bucket(pmax);
  B.fn = group_kernel_for(probs[0].op, B.pb, B.tile_rows);
  if (!B.fn) return KIOPS_ERR_UNSUPPORTED;
  int per_cu = 0;
  if (!hip_ok(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, B.fn, kThreads, 0)) || per_cu < 1)
    return KIOPS_ERR_DEVICE;
  const int total = per_cu * probs[0].op->cus;
  int gs = group_size;
  if (gs <= 0) {
    // about a quarter of the median problem's work tiles, a power of two in [8, 64]
    std::vector<int64_t> tiles(count);
    for (int i = 0; i < count; ++i) tiles[i] = work_tiles(probs[i].op, false, B.tile_rows);
    std::nth_element(tiles.begin(), tiles.begin() + count / 2, tiles.end());
    const int64_t want = std::max<int64_t>(1, tiles[count / 2] / 4);
    gs = 8;
    while (gs < 64 && gs < want) gs *= 2;
  }
  if (gs > total) return KIOPS_ERR_INVALID_ARG;
  B.gs = gs;
  std::vector<double> est(count);
  double tot = 0.0;
  for (int i = 0; i < count; ++i) tot += (est[i] = work_estimate(probs[i]));
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return est[a] > est[b]; });
  // Groups: a problem whose share of the estimated work exceeds what one
  // group of gs workgroups gives it gets a group of its own, sized to its
  // share (gs times a power of two, within its work tiles); dedicated groups
  // take at most half of the workgroups.  The rest is split into groups of
  // gs that share the other problems.  (One group size for all would leave
  // the largest problem, in the batched workload a fifth of the work, on gs
  // workgroups and set the batch's time.)
  auto pow2_floor = [](int64_t v) { int64_t r = 1; while (2 * r <= v) r *= 2; return (int)r; };
  std::vector<int> dedicated;           // problem of each dedicated group
  int used = 0;
  const int budget = total / 2;
  if (std::getenv("KIOPS_BATCH_UNIFORM") == nullptr) {   // experiment override: groups of gs only
    for (int i : order) {
      if ((int)dedicated.size() + 1 >= count) break;   // keep one problem for the shared groups
      int want = gs;   // the power of two nearest (in ratio) to its share of the workgroups
      while (want < budget && 1.5 * (double)want < (double)total * est[i] / tot) want *= 2;
      want = std::min(want, std::max(gs, pow2_floor(std::max<int64_t>(1, work_tiles(probs[i].op, false, B.tile_rows)))));
      while (want > gs && used + want > budget) want /= 2;
      if (want <= gs) break;             // sorted: every later problem wants less
      dedicated.push_back(i);
      B.gsize.push_back(want);
      used += want;
    }
  }
  const int nshared = std::max(1, std::min((total - used) / gs, count - (int)dedicated.size()));
  for (int k = 0; k < nshared; ++k) B.gsize.push_back(gs);
  B.ng = (int)B.gsize.size();
  B.wg0.assign(B.ng, 0);
  for (int g = 1; g < B.ng; ++g) B.wg0[g] = B.wg0[g - 1] + B.gsize[g - 1];
  B.nwg = B.wg0[B.ng - 1] + B.gsize[B.ng - 1];
  if (B.nwg > total) return KIOPS_ERR_INVALID_ARG;
  // dedicated problems first, then longest estimated work first, each to the
  // shared group that would finish it first
  std::vector<double> load(B.ng, 0.0);
  B.group_of.assign(count, -1);
  B.members.assign(B.ng, {});
  for (size_t k = 0; k < dedicated.size(); ++k) {
    B.group_of[dedicated[k]] = (int)k;
    B.members[k].push_back(dedicated[k]);
    load[k] = est[dedicated[k]];
  }
  const int first_shared = (int)dedicated.size();
  for (int i : order) {
    if (B.group_of[i] >= 0) continue;
    int g = first_shared;
    for (int h = first_shared + 1; h < B.ng; ++h)
      if (load[h] < load[g] || (load[h] == load[g] && B.members[h].size() < B.members[g].size())) g = h;
    if ((int)B.members[g].size() >= kGroupQueueLen) return KIOPS_ERR_UNSUPPORTED;
    B.group_of[i] = g;
    B.members[g].push_back(i);
    load[g] += est[i];
  }
  // workspace: one region per group (the largest layout among its problems;
  // the barrier words sit at the same offsets in every layout of the group),
  // then per-problem control blocks, parameter blocks and the group queues
  size_t off = 0;
  B.group_off.assign(B.ng, 0);
  for (int g = 0; g < B.ng; ++g) {
    size_t need = 0;
    for (int i : B.members[g]) {
      const Layout L = make_layout(probs[i].op, probs[i].p, probs[i].q, B.m_max, B.gsize[g]);
      need = std::max(need, L.total);
    }
    B.group_off[g] = off;
    off = align_up(off + need);
  }
  B.ctrl_off = off;
  off = align_up(off + ctrl_stride() * count);
  B.block_off = off;
  off = align_up(off + (size_t)4096 * count);
  B.queue_off = off;
  off = align_up(off + sizeof(GroupQueue) * B.ng);
  B.map_off = off;
  off = align_up(off + sizeof(int) * (size_t)B.nwg);
  B.total = off;
  return KIOPS_OK;
}

kiops_status run_batch(int count, const kiops_problem* probs, const BatchPlan& B, char* ws, hipStream_t stream,
                       kiops_stats* stats, double* ms_out) {
  std::vector<unsigned char> blocks((size_t)4096 * count, 0);
  std::vector<unsigned char> ctrls(ctrl_stride() * count, 0);
  for (int i = 0; i < count; ++i) {
    Ctrl c{};
    c.phase = kPhaseDone;
    c.status = KIOPS_ERR_DEVICE;   // until the solve publishes its own
    std::memcpy(ctrls.data() + ctrl_stride() * i, &c, sizeof(Ctrl));
  }
  std::vector<GroupQueue> queues(B.ng);
  const uint64_t clock_hz = probs[0].op->clock_hz;
  for (int g = 0; g < B.ng; ++g) {
    GroupQueue& Q = queues[g];
    std::memset(&Q, 0, sizeof(GroupQueue));
    Q.wg0 = B.wg0[g];
    Q.gsize = B.gsize[g];
    Q.tail = (unsigned)B.members[g].size();
    Q.closed = 1;
    Q.idle_limit = clock_hz * 60ull;
    char* base = ws + B.group_off[g];
    for (size_t e = 0; e < B.members[g].size(); ++e) {
      const int i = B.members[g][e];
      const kiops_problem& pr = probs[i];
      const Layout L = make_layout(pr.op, pr.p, pr.q, B.m_max, B.gsize[g]);
      KParams P = make_params(pr.op, L, base, pr.tau, pr.p, pr.V, pr.tol, pr.m_init, pr.q, B.m_min, B.m_max,
                              B.max_sub, kModeSolve, pr.w);
      P.ctrl = reinterpret_cast<Ctrl*>(ws + B.ctrl_off + ctrl_stride() * i);
      unsigned char* blk = blocks.data() + (size_t)4096 * i;
      std::memcpy(blk, &P, sizeof(KParams));
      kiops_status s = stage_op_block(pr.op, pr.p, B.pb, pr.V, base, L, blk, false, B.tile_rows);
      if (s != KIOPS_OK) return s;
      Q.blocks[e] = reinterpret_cast<const unsigned char*>(ws + B.block_off + (size_t)4096 * i);
    }
    // the group's barrier words: zero (same offsets for every layout of the group)
    const Layout L0 = make_layout(probs[B.members[g][0]].op, probs[B.members[g][0]].p,
                                  probs[B.members[g][0]].q, B.m_max, B.gsize[g]);
    if (!hip_ok(hipMemsetAsync(base + L0.bar, 0, L0.H - L0.bar, stream))) return KIOPS_ERR_DEVICE;
  }
  std::vector<int> wg_group(B.nwg);
  for (int g = 0; g < B.ng; ++g)
    for (int k = 0; k < B.gsize[g]; ++k) wg_group[B.wg0[g] + k] = g;
  if (!hip_ok(hipMemcpyAsync(ws + B.ctrl_off, ctrls.data(), ctrls.size(), hipMemcpyHostToDevice, stream)) ||
      !hip_ok(hipMemcpyAsync(ws + B.block_off, blocks.data(), blocks.size(), hipMemcpyHostToDevice, stream)) ||
      !hip_ok(hipMemcpyAsync(ws + B.queue_off, queues.data(), sizeof(GroupQueue) * B.ng, hipMemcpyHostToDevice,
                             stream)) ||
      !hip_ok(hipMemcpyAsync(ws + B.map_off, wg_group.data(), sizeof(int) * wg_group.size(),
                             hipMemcpyHostToDevice, stream)))
    return KIOPS_ERR_DEVICE;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ms_out) {
    if (!hip_ok(hipEventCreate(&e0)) || !hip_ok(hipEventCreate(&e1))) return KIOPS_ERR_DEVICE;
    hipEventRecord(e0, stream);
  }
  GroupQueue* dq = reinterpret_cast<GroupQueue*>(ws + B.queue_off);
  const int* dmap = reinterpret_cast<const int*>(ws + B.map_off);
  void* args[] = {&dq, &dmap};
  if (!hip_ok(hipLaunchCooperativeKernel(B.fn, dim3(B.nwg), dim3(kThreads), args, 0, stream)))
    return KIOPS_ERR_DEVICE;
  if (ms_out) hipEventRecord(e1, stream);
  if (!hip_ok(hipMemcpyAsync(ctrls.data(), ws + B.ctrl_off, ctrls.size(), hipMemcpyDeviceToHost, stream)))
    return KIOPS_ERR_DEVICE;
  std::vector<unsigned> aborts(B.ng, 0);
  for (int g = 0; g < B.ng; ++g) {
    const Layout L0 = make_layout(probs[B.members[g][0]].op, probs[B.members[g][0]].p,
                                  probs[B.members[g][0]].q, B.m_max, B.gsize[g]);
    const Barrier* bar = reinterpret_cast<const Barrier*>(ws + B.group_off[g] + L0.bar);
    if (!hip_ok(hipMemcpyAsync(&aborts[g], &bar->abort, sizeof(unsigned), hipMemcpyDeviceToHost, stream)))
      return KIOPS_ERR_DEVICE;
  }
  if (!hip_ok(hipStreamSynchronize(stream))) return KIOPS_ERR_DEVICE;
  if (ms_out) {
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    *ms_out = ms;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
  }
  kiops_status first = KIOPS_OK;
  for (int i = 0; i < count; ++i) {
    Ctrl c;
    std::memcpy(&c, ctrls.data() + ctrl_stride() * i, sizeof(Ctrl));
    if (aborts[B.group_of[i]] && c.status == KIOPS_OK) c.status = KIOPS_ERR_DEVICE;
    if (stats) fill_stats(c, B.gsize[B.group_of[i]], (double)clock_hz, &stats[i]);
    if (first == KIOPS_OK && c.status != KIOPS_OK) first = (kiops_status)c.status;
  }
  return first;
}

// ---------------------------------------------------------------- server

constexpr int kServePB = 4;   // p-bucket of the served kernel (p <= 4)
constexpr bool kServedEnabled = true;   // compile-time switch of kiops_server_create

int serve_family(const kiops_operator* op) {
  const bool mixed = op->d.precision == KIOPS_MIXED;
  if (op->d.kind == KIOPS_OP_CSR) return -1;
  if (uses_3d(op)) return mixed ? kFamily3DMixed : kFamily3D;
  return mixed ? kFamily2DMixed : kFamily2D;
}

constexpr int64_t kGangPointsDefault = 8192;   // grid points per workgroup when sizing a gang

// Groups of group_size workgroups over `per_cu` workgroups per CU: one fewer
// than fit on a CU (at most two, at least one), so that a CU keeps room for a
// workgroup of other work beside the launch.
kiops_status serve_geometry(int group_size, int* gs_out, int* ng_out) {
  int dev = 0, cus = 0, fit = 0;
  if (!hip_ok(hipGetDevice(&dev)) ||
      !hip_ok(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) ||
      !hip_ok(hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, kernels_serve(), kThreads, 0)) || fit < 1)
    return KIOPS_ERR_DEVICE;
  const int per_cu = fit >= 3 ? 2 : 1;
  const int gs = group_size > 0 ? group_size : 16;
  if (gs > cus * per_cu || gs % 8 != 0) return KIOPS_ERR_INVALID_ARG;   // groups keep the XCD order of blocks
  *gs_out = gs;
  *ng_out = cus * per_cu / gs;
  return KIOPS_OK;
}

// Fixed part of a server workspace, in this order: one Barrier and one
// control block per group (a gang uses its first group's), the per-workgroup
// arrival slots, arrival clocks (3 per workgroup) and finish words.  The
// group queues and parameter blocks are not in the workspace (see Mailbox).
struct ServeLayout {
  size_t bar, ctrl, arrive, arrive_t, fin, pool;
};
ServeLayout serve_layout(int gs, int ng) {
  ServeLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t at = off; off = align_up(off + bytes); return at; };
  const size_t nwg = (size_t)gs * ng;
  L.bar = take(sizeof(Barrier) * ng);
  L.ctrl = take(ctrl_stride() * ng);
  L.arrive = take(sizeof(unsigned) * nwg);
  L.arrive_t = take(sizeof(uint64_t) * 3 * nwg);
  L.fin = take(sizeof(unsigned) * nwg);
  L.pool = off;
  return L;
}

// Mailbox of a server: its group queues, then one 4096-byte parameter block
// per group.  The host writes both while the served launch runs.  Memory
// from hipMalloc (the workspace) is coarse-grained: HIP makes host writes to
// it visible to kernels only at kernel boundaries, so a running kernel could
// see a queue tail before the block pointer and parameter block it
// publishes.  The mailbox is fine-grained device memory instead, coherent
// while kernels run; the served kernel reads the tails with system-scope
// acquires and writes its done words with system-scope releases.  Mailboxes
// are taken from a per-process list and given back by kiops_server_destroy,
// never freed.
constexpr size_t kMailboxBlock = 4096;
size_t mailbox_queue_bytes(int ng) { return align_up(sizeof(GroupQueue) * (size_t)ng); }
size_t mailbox_bytes(int ng) { return mailbox_queue_bytes(ng) + kMailboxBlock * (size_t)ng; }

struct Mailbox {
  int dev;
  size_t bytes;
  char* p;
};
std::mutex g_mailbox_mu;
std::vector<Mailbox> g_mailbox_free;

// A mailbox of at least `bytes` on device dev (current), its size in *got.
char* mailbox_take(int dev, size_t bytes, size_t* got) {
  {
    std::lock_guard<std::mutex> lk(g_mailbox_mu);
    for (size_t i = 0; i < g_mailbox_free.size(); ++i) {
      if (g_mailbox_free[i].dev == dev && g_mailbox_free[i].bytes >= bytes) {
        char* p = g_mailbox_free[i].p;
        *got = g_mailbox_free[i].bytes;
        g_mailbox_free.erase(g_mailbox_free.begin() + i);
        return p;
      }
    }
  }
  void* p = nullptr;
  if (!hip_ok(hipExtMallocWithFlags(&p, bytes, hipDeviceMallocFinegrained))) return nullptr;
  *got = bytes;
  return static_cast<char*>(p);
}

void mailbox_give(int dev, size_t bytes, char* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_mailbox_mu);
  g_mailbox_free.push_back(Mailbox{dev, bytes, p});
}

}  // namespace

struct kiops_server {
  struct Req {
    kiops_problem pr;
    std::vector<const double*> V;
    int g0 = -1, k = 0;                  // gang: groups [g0, g0 + k)
    size_t pool_off = 0, pool_bytes = 0;
    int done = 0;
    Ctrl ctrl{};
  };
  hipStream_t run = nullptr, io = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int dev = 0;
  char* mail = nullptr;                 // group queues, then parameter blocks (fine-grained)
  size_t mail_bytes = 0;
  int gs = 0, ng = 0, max_gang = 1;
  int64_t gang_points = kGangPointsDefault;
  uint64_t clock_hz = 0;
  ServeLayout L{};
  size_t pool_bytes = 0;
  std::map<size_t, size_t> free_list;   // pool offset -> bytes
  std::deque<int64_t> waiting;
  std::unordered_map<int64_t, Req> reqs;
  std::vector<int64_t> group_req;       // running ticket per group, -1 if free
  std::vector<unsigned> pushed;         // entries pushed per group
  std::vector<unsigned> last_epoch;     // barrier epoch each group's workgroups have reached
  int64_t next_ticket = 1;
  bool dead = false;
};

namespace {

bool pool_alloc(kiops_server* s, size_t bytes, size_t* off) {
  for (auto it = s->free_list.begin(); it != s->free_list.end(); ++it) {
    if (it->second >= bytes) {
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t at = it->first + bytes;
      s->free_list.erase(it);
      if (rest > 0) s->free_list[at] = rest;
      return true;
    }
  }
  return false;
}

void pool_free(kiops_server* s, size_t off, size_t bytes) {
  auto it = s->free_list.emplace(off, bytes).first;
  auto nx = std::next(it);
  if (nx != s->free_list.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    s->free_list.erase(nx);
  }
  if (it != s->free_list.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      s->free_list.erase(it);
    }
  }
}

// Groups a request runs on: the smallest power of two whose workgroups get at
// most gang_points grid points each, capped at the largest power of two that
// fits the launch and kept within the operator's work items (more workgroups
// than tiles, or z chunks thinner than the march needs, only add overhead).
int gang_groups(const kiops_server* s, const kiops_operator* op) {
  const int64_t items = std::max<int64_t>(1, work_tiles(op));
  const int64_t want = std::min<int64_t>((op->N + s->gang_points - 1) / s->gang_points, items);
  int k = 1;
  while ((int64_t)k * s->gs < want && 2 * k <= s->max_gang) k *= 2;
  if (k > 1 && (int64_t)k * s->gs > items) k /= 2;
  return k;
}

size_t request_bytes(const kiops_server* s, const kiops_problem& pr, int k) {
  int m_min, m_max, max_sub;
  resolve_options(pr.op, nullptr, &m_min, &m_max, &max_sub);
  return align_up(make_layout(pr.op, pr.p, pr.q, m_max, k * s->gs).total);
}

// Admit request t on the free gang [g0, g0 + k) with pool block off.
kiops_status admit(kiops_server* s, int64_t t, int g0, int k, size_t off, size_t bytes) {
  kiops_server::Req& R = s->reqs[t];
  const kiops_problem& pr = R.pr;
  int m_min, m_max, max_sub;
  resolve_options(pr.op, nullptr, &m_min, &m_max, &max_sub);
  char* base = s->ws + s->L.pool + off;
  const int nwg = k * s->gs;
  const int wg0 = g0 * s->gs;
  const Layout L = make_layout(pr.op, pr.p, pr.q, m_max, nwg);
  KParams P = make_params(pr.op, L, base, pr.tau, pr.p, R.V.data(), pr.tol, pr.m_init, pr.q, m_min, m_max,
                          max_sub, kModeSolve, pr.w);
  P.bar = reinterpret_cast<Barrier*>(s->ws + s->L.bar) + g0;
  P.ctrl = reinterpret_cast<Ctrl*>(s->ws + s->L.ctrl + ctrl_stride() * g0);
  P.arrive = reinterpret_cast<unsigned*>(s->ws + s->L.arrive) + wg0;
  P.arrive_t = reinterpret_cast<uint64_t*>(s->ws + s->L.arrive_t) + 3 * (size_t)wg0;
  P.family = serve_family(pr.op);
  P.wg0 = wg0;
  // Epochs start above every epoch any finished request has reached, on any
  // group: the release words and barrier words a finished request left in
  // the pool block or the barrier (which this request may reuse) then never
  // match an epoch of this one, and nothing has to be cleared first.
  unsigned e0 = 0;
  for (int g = 0; g < s->ng; ++g) e0 = std::max(e0, s->last_epoch[g]);
  P.epoch0 = e0;
  alignas(256) unsigned char blk[4096];
  std::memset(blk, 0, sizeof(blk));
  std::memcpy(blk, &P, sizeof(KParams));
  kiops_status st = stage_op_block(pr.op, pr.p, kServePB, R.V.data(), base, L, blk);
  if (st != KIOPS_OK) return st;
  Ctrl c{};
  c.phase = kPhaseDone;
  c.status = KIOPS_ERR_DEVICE;
  if (!hip_ok(hipMemcpyAsync(P.ctrl, &c, sizeof(Ctrl), hipMemcpyHostToDevice, s->io)))
    return KIOPS_ERR_DEVICE;
  GroupQueue* dq = reinterpret_cast<GroupQueue*>(s->mail);
  std::vector<const unsigned char*> ptrs(k);
  std::vector<unsigned> tails(k);
  for (int i = 0; i < k; ++i) {
    const int g = g0 + i;
    unsigned char* dblk =
        reinterpret_cast<unsigned char*>(s->mail + mailbox_queue_bytes(s->ng) + kMailboxBlock * g);
    ptrs[i] = dblk;
    tails[i] = s->pushed[g] + 1;
    if (!hip_ok(hipMemcpyAsync(dblk, blk, sizeof(blk), hipMemcpyHostToDevice, s->io)) ||
        !hip_ok(hipMemcpyAsync(&dq[g].blocks[s->pushed[g] % kGroupQueueLen], &ptrs[i], sizeof(ptrs[i]),
                               hipMemcpyHostToDevice, s->io)))
      return KIOPS_ERR_DEVICE;
  }
  // publish after every block of the gang is in place
  for (int i = 0; i < k; ++i)
    if (!hip_ok(hipMemcpyAsync(&dq[g0 + i].tail, &tails[i], sizeof(unsigned), hipMemcpyHostToDevice, s->io)))
      return KIOPS_ERR_DEVICE;
  if (!hip_ok(hipStreamSynchronize(s->io))) return KIOPS_ERR_DEVICE;
  for (int i = 0; i < k; ++i) {
    s->pushed[g0 + i] = tails[i];
    s->group_req[g0 + i] = t;
  }
  R.g0 = g0;
  R.k = k;
  R.pool_off = off;
  R.pool_bytes = bytes;
  return KIOPS_OK;
}

// First aligned free run of k groups outside [rlo, rhi), or -1.
int free_gang(const kiops_server* s, int k, int rlo, int rhi) {
  for (int g0 = 0; g0 + k <= s->ng; g0 += k) {
    if (g0 < rhi && rlo < g0 + k) continue;
    bool ok = true;
    for (int g = g0; g < g0 + k && ok; ++g) ok = s->group_req[g] < 0;
    if (ok) return g0;
  }
  return -1;
}

// Aligned run of k groups with the fewest busy groups (reserved for the
// request at the head of the queue so that smaller ones cannot starve it).
int reserve_gang(const kiops_server* s, int k) {
  int best = 0, best_busy = k + 1;
  for (int g0 = 0; g0 + k <= s->ng; g0 += k) {
    int busy = 0;
    for (int g = g0; g < g0 + k; ++g) busy += s->group_req[g] >= 0;
    if (busy < best_busy) { best = g0; best_busy = busy; }
  }
  return best;
}

}  // namespace

// ---------------------------------------------------------------- no-allocation scratch

// Device memory of kiops_phi_combination_noalloc: a fixed array in the code
// object, one copy per GPU the library runs on, held until the process ends.
// In host code `scratch` names a host-side stand-in, never the device array:
// its device address is taken once per device with hipGetSymbolAddress and
// only that address is used.
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kScratchDevices = 64;
std::mutex scratch_mutex;
char* scratch_ptr[kScratchDevices] = {};

// Device address of `scratch` on device dev (taken with dev current, once).
kiops_status scratch_of_device(int dev, char** out) {
  if (dev < 0 || dev >= kScratchDevices) return KIOPS_ERR_DEVICE;
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_ptr[dev]) {
    int cur = -1;
    if (!hip_ok(hipGetDevice(&cur))) return KIOPS_ERR_DEVICE;
    if (cur != dev && !hip_ok(hipSetDevice(dev))) return KIOPS_ERR_DEVICE;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) hipSetDevice(cur);
    if (!hip_ok(e) || !ptr || reinterpret_cast<uintptr_t>(ptr) % kAlign != 0) return KIOPS_ERR_DEVICE;
    scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = scratch_ptr[dev];
  return KIOPS_OK;
}

// One solve with the operator's workspace (ws == nullptr) or with the given
// device memory of ws_bytes (the no-allocation scratch).
kiops_status phi_combination_in(kiops_operator* op, char* ws, size_t ws_bytes, double tau, int p,
                                const double* const* V, double tol, int m_init, int q,
                                const kiops_options* opts, double* w, kiops_stats* stats) {
  if (!op) return KIOPS_ERR_INVALID_ARG;
  if (!(tau >= 0.0) || !std::isfinite(tau) || !(tol > 0.0) || !std::isfinite(tol) || m_init < 1 ||
      q < 0 || q > 8)
    return KIOPS_ERR_INVALID_ARG;
  kiops_status s = check_vectors(op, p, V, w);
  if (s != KIOPS_OK) return s;
  int m_min, m_max, max_sub;
  resolve_options(op, opts, &m_min, &m_max, &max_sub);
  if (m_max > KIOPS_M_MAX_LIMIT || m_min > m_max || m_min < 1) return KIOPS_ERR_INVALID_ARG;
  const int estimate = resolve_estimate(opts);
  if (estimate < 0) return KIOPS_ERR_INVALID_ARG;
  if (q > kWinMax) return KIOPS_ERR_UNSUPPORTED;
  if (!kernel_for(op, p, q)) return KIOPS_ERR_UNSUPPORTED;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (tau == 0.0) {
    if (w != V[0] &&
        !hip_ok(hipMemcpyAsync(w, V[0], sizeof(double) * op->N, hipMemcpyDeviceToDevice, op->stream)))
      return KIOPS_ERR_DEVICE;
    if (!hip_ok(hipStreamSynchronize(op->stream))) return KIOPS_ERR_DEVICE;
    return KIOPS_OK;
  }
  int nwg = 0;
  s = grid_size(op, p, q, &nwg);
  if (s != KIOPS_OK) return s;
  const Layout L = make_layout(op, p, q, m_max, nwg);
  if (!ws) {
    ws = reinterpret_cast<char*>(op->ws);
    ws_bytes = op->ws_bytes;
  }
  if (!ws || ws_bytes < L.total) return KIOPS_ERR_OUT_OF_MEMORY;
  KParams P = make_params(op, L, ws, tau, p, V, tol, m_init, q, m_min, m_max, max_sub, kModeSolve, w);
  P.estimate = estimate;
  Ctrl hc{};
  unsigned abort_flag = 0;
  s = run_solve(op, ws, L, P, p, V, &hc, &abort_flag);
  if (s != KIOPS_OK) return s;
  fill_stats(hc, nwg, (double)op->clock_hz, stats);
  if (stats) stats->pass_kind = pass_kind(op, q);
  if (abort_flag) return KIOPS_ERR_DEVICE;
  return (kiops_status)hc.status;
}

}  // namespace

extern "C" {

const char* kiops_status_string(kiops_status s) {
  switch (s) {
    case KIOPS_OK: return "ok";
    case KIOPS_ERR_INVALID_ARG: return "invalid argument";
    case KIOPS_ERR_OUT_OF_MEMORY: return "workspace missing or too small";
    case KIOPS_ERR_DEVICE: return "device error";
    case KIOPS_ERR_NONFINITE: return "non-finite value";
    case KIOPS_ERR_NOT_CONVERGED: return "substep limit reached";
    case KIOPS_ERR_BUDGET: return "over memory budget";
    case KIOPS_ERR_UNSUPPORTED: return "unsupported request";
  }
  return "unknown status";
}

kiops_status kiops_create_operator(const kiops_operator_desc* desc, void* hip_stream, kiops_operator** out) {
  if (!desc || !out) return KIOPS_ERR_INVALID_ARG;
  const kiops_operator_desc& d = *desc;
  int64_t N = 0;
  if (d.precision != KIOPS_FP64 && d.precision != KIOPS_MIXED) return KIOPS_ERR_INVALID_ARG;
  if (d.kind == KIOPS_OP_STENCIL2D_5PT || d.kind == KIOPS_OP_STENCIL3D_7PT) {
    if (d.nx < 1 || d.ny < 1 || d.nz < 1 || !(d.h > 0.0) || !std::isfinite(d.h)) return KIOPS_ERR_INVALID_ARG;
    if (d.kind == KIOPS_OP_STENCIL2D_5PT && d.nz != 1) return KIOPS_ERR_INVALID_ARG;
    if (d.nx > (1 << 30) || d.ny > (1 << 30) || d.nz > (1 << 30)) return KIOPS_ERR_INVALID_ARG;
    int64_t nxy = 0;
    if (__builtin_mul_overflow(d.nx, d.ny, &nxy) || __builtin_mul_overflow(nxy, d.nz, &N))
      return KIOPS_ERR_INVALID_ARG;
    // the passes address every array with 32-bit byte offsets
    if (N * (int64_t)sizeof(double) >= ((int64_t)1 << 32)) return KIOPS_ERR_INVALID_ARG;
    if (!std::isfinite(d.diff) || !std::isfinite(d.adv[0]) || !std::isfinite(d.adv[1]) ||
        !std::isfinite(d.adv[2]))
      return KIOPS_ERR_INVALID_ARG;
    // the general form takes the operator from its weights alone
    if (d.weights && (d.kappa || d.reaction || d.diff != 0.0 || d.adv[0] != 0.0 || d.adv[1] != 0.0 ||
                      d.adv[2] != 0.0))
      return KIOPS_ERR_INVALID_ARG;
  } else if (d.kind == KIOPS_OP_CSR) {
    if (d.weights) return KIOPS_ERR_INVALID_ARG;
    if (d.nrows < 1 || d.nnz < 0 || !d.rowptr || !d.col || (!d.val && d.nnz > 0)) return KIOPS_ERR_INVALID_ARG;
    // 32-bit byte offsets into val and the basis vectors
    if (d.nnz * (int64_t)sizeof(double) >= ((int64_t)1 << 32) || d.nrows >= ((int64_t)1 << 29))
      return KIOPS_ERR_INVALID_ARG;
    N = d.nrows;
  } else {
    return KIOPS_ERR_INVALID_ARG;
  }
  if (N > ((int64_t)1 << 34)) return KIOPS_ERR_INVALID_ARG;
  kiops_operator* op = new (std::nothrow) kiops_operator();
  if (!op) return KIOPS_ERR_OUT_OF_MEMORY;
  op->d = d;
  op->stream = reinterpret_cast<hipStream_t>(hip_stream);
  op->N = N;
  op->ws = nullptr;
  op->ws_bytes = 0;
  if (!hip_ok(hipGetDevice(&op->device))) { delete op; return KIOPS_ERR_DEVICE; }
  if (!hip_ok(hipDeviceGetAttribute(&op->cus, hipDeviceAttributeMultiprocessorCount, op->device))) {
    delete op;
    return KIOPS_ERR_DEVICE;
  }
  int khz = 0;
  if (!hip_ok(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, op->device)) || khz <= 0)
    khz = 100000;
  op->clock_hz = (uint64_t)khz * 1000ull;
  *out = op;
  return KIOPS_OK;
}

kiops_status kiops_destroy_operator(kiops_operator* op) {
  if (!op) return KIOPS_ERR_INVALID_ARG;
  delete op;
  return KIOPS_OK;
}

kiops_status kiops_device_info(const kiops_operator* op, int* compute_units, int* grid_blocks) {
  if (!op) return KIOPS_ERR_INVALID_ARG;
  if (compute_units) *compute_units = op->cus;
  if (grid_blocks) {
    int g = 0;
    kiops_status s = grid_size(op, 2, 2, &g);
    if (s != KIOPS_OK) return s;
    *grid_blocks = g;
  }
  return KIOPS_OK;
}

kiops_status kiops_apply(kiops_operator* op, const double* x, double* y) {
  if (!op || !x || !y) return KIOPS_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 7) return KIOPS_ERR_INVALID_ARG;
  const uintptr_t xa = reinterpret_cast<uintptr_t>(x), ya = reinterpret_cast<uintptr_t>(y);
  const uintptr_t nb = (uintptr_t)op->N * sizeof(double);
  if (xa < ya + nb && ya < xa + nb) return KIOPS_ERR_INVALID_ARG;   // overlapping vectors
  return hip_ok(kiops::launch_apply(op->d, op->N, x, y, op->stream)) ? KIOPS_OK : KIOPS_ERR_DEVICE;
}

kiops_status kiops_workspace_bytes(const kiops_operator* op, int p, int q, const kiops_options* opts,
                                   size_t* bytes) {
  if (!op || !bytes || p < 0 || p > KIOPS_P_MAX || q < 0 || q > 8) return KIOPS_ERR_INVALID_ARG;
  int m_min, m_max, max_sub;
  resolve_options(op, opts, &m_min, &m_max, &max_sub);
  if (m_max > KIOPS_M_MAX_LIMIT || m_min > m_max) return KIOPS_ERR_INVALID_ARG;
  int nwg = 0;
  kiops_status s = grid_size(op, p, q, &nwg);
  if (s != KIOPS_OK) return s;
  *bytes = make_layout(op, p, q, m_max, nwg).total;
  return KIOPS_OK;
}

kiops_status kiops_set_workspace(kiops_operator* op, void* dev_ptr, size_t bytes) {
  if (!op || (!dev_ptr && bytes > 0)) return KIOPS_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(dev_ptr) % kAlign != 0) return KIOPS_ERR_INVALID_ARG;
  op->ws = dev_ptr;
  op->ws_bytes = bytes;
  return KIOPS_OK;
}

kiops_status kiops_phi_combination(kiops_operator* op, double tau, int p, const double* const* V,
                                   double tol, int m_init, int q, const kiops_options* opts,
                                   double* w, kiops_stats* stats) {
  return phi_combination_in(op, nullptr, 0, tau, p, V, tol, m_init, q, opts, w, stats);
}

kiops_status kiops_phi_combination_noalloc(kiops_operator* op, double tau, int p, const double* const* V,
                                           double tol, int m_init, int q, const kiops_options* opts,
                                           double* w, kiops_stats* stats) {
  if (!op) return KIOPS_ERR_INVALID_ARG;
  char* ws = nullptr;
  const kiops_status s = scratch_of_device(op->device, &ws);
  if (s != KIOPS_OK) return s;
  return phi_combination_in(op, ws, kScratchBytes, tau, p, V, tol, m_init, q, opts, w, stats);
}

kiops_status kiops_phi_combination_times(kiops_operator* op, int n, const double* times, int task, int p,
                                         const double* const* V, double tol, int m_init, int q,
                                         const kiops_options* opts, double* const* W, kiops_stats* stats) {
  if (!op || !times || !W || n < 1 || n > KIOPS_MAX_TIMES || (task != 1 && task != 2)) return KIOPS_ERR_INVALID_ARG;
  if (!(tol > 0.0) || !std::isfinite(tol) || m_init < 1 || q < 0 || q > 8) return KIOPS_ERR_INVALID_ARG;
  for (int k = 0; k < n; ++k) {
    if (!(times[k] > 0.0) || !std::isfinite(times[k]) || (k > 0 && !(times[k] > times[k - 1])) || !W[k])
      return KIOPS_ERR_INVALID_ARG;
    for (int l = 0; l < k; ++l)
      if (W[l] == W[k]) return KIOPS_ERR_INVALID_ARG;
  }
  double* w = W[n - 1];
  kiops_status s = check_vectors(op, p, V, w);
  if (s != KIOPS_OK) return s;
  for (int k = 0; k + 1 < n; ++k)
    for (int i = 0; i <= p; ++i)
      if (W[k] == V[i]) return KIOPS_ERR_INVALID_ARG;
  int m_min, m_max, max_sub;
  resolve_options(op, opts, &m_min, &m_max, &max_sub);
  if (m_max > KIOPS_M_MAX_LIMIT || m_min > m_max || m_min < 1) return KIOPS_ERR_INVALID_ARG;
  const int estimate = resolve_estimate(opts);
  if (estimate < 0 || (estimate == KIOPS_ESTIMATE_CORRECTED && n > 1)) return KIOPS_ERR_INVALID_ARG;
  if (q > kWinMax) return KIOPS_ERR_UNSUPPORTED;
  if (!kernel_for(op, p, q)) return KIOPS_ERR_UNSUPPORTED;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  int nwg = 0;
  s = grid_size(op, p, q, &nwg);
  if (s != KIOPS_OK) return s;
  const double T_end = times[n - 1];
  const Layout L = make_layout(op, p, q, m_max, nwg);
  if (!op->ws || op->ws_bytes < L.total) return KIOPS_ERR_OUT_OF_MEMORY;
  KParams P = make_params(op, L, reinterpret_cast<char*>(op->ws), T_end, p, V, tol, m_init, q, m_min, m_max,
                          max_sub, kModeSolve, w);
  P.ntimes = n;
  P.task1 = task == 1 ? 1 : 0;
  P.estimate = estimate;
  for (int k = 0; k < n; ++k) {
    P.times[k] = times[k];
    P.wout[k] = W[k];
  }
  Ctrl hc{};
  unsigned abort_flag = 0;
  s = run_solve(op, reinterpret_cast<char*>(op->ws), L, P, p, V, &hc, &abort_flag);
  if (s != KIOPS_OK) return s;
  fill_stats(hc, nwg, (double)op->clock_hz, stats);
  if (stats) stats->pass_kind = pass_kind(op, q);
  if (abort_flag) return KIOPS_ERR_DEVICE;
  return (kiops_status)hc.status;
}

kiops_status kiops_iop_basis(kiops_operator* op, int p, const double* const* V, int m, int q,
                             double* basis, double* H, int* j_done, double* beta, double* nu_out) {
  if (!op || !basis || !H || m < 1 || m > KIOPS_M_MAX_LIMIT || q < 0 || q > kWinMax)
    return KIOPS_ERR_INVALID_ARG;
  if (!V || p < 0 || p > KIOPS_P_MAX) return KIOPS_ERR_INVALID_ARG;
  for (int k = 0; k <= p; ++k)
    if (!V[k]) return KIOPS_ERR_INVALID_ARG;
  if (!kernel_for(op, p, q)) return KIOPS_ERR_UNSUPPORTED;
  int nwg = 0;
  kiops_status s = grid_size(op, p, q, &nwg);
  if (s != KIOPS_OK) return s;
  const Layout L = make_layout(op, p, q, m, nwg);
  // w holds b_0 during the run: place it in the last slot row of the workspace tail
  const size_t need = L.total + align_up(sizeof(double) * (size_t)op->N);
  if (!op->ws || op->ws_bytes < need) return KIOPS_ERR_OUT_OF_MEMORY;
  char* ws = reinterpret_cast<char*>(op->ws);
  double* wtmp = reinterpret_cast<double*>(ws + L.total);
  KParams P = make_params(op, L, ws, 1.0, p, V, 1.0, m, q, 1, m, 1, kModeBasis, wtmp);
  Ctrl hc{};
  unsigned abort_flag = 0;
  s = run_solve(op, reinterpret_cast<char*>(op->ws), L, P, p, V, &hc, &abort_flag);
  if (s != KIOPS_OK) return s;
  if (abort_flag) return KIOPS_ERR_DEVICE;
  if (hc.status != KIOPS_OK) return (kiops_status)hc.status;
  const int jd = hc.breakdown ? (hc.kp - 1) : m;
  const int nvec = hc.breakdown ? jd : jd + 1;
  hipLaunchKernelGGL(export_basis_kernel, dim3(1024), dim3(256), 0, op->stream, P.slots, wtmp, P.mixed,
                     op->N, p, nvec, P.sinv, P.Y, basis);
  hipLaunchKernelGGL(export_h_kernel, dim3(1), dim3(256), 0, op->stream, P.H, m, H);
  if (!hip_ok(hipGetLastError()) || !hip_ok(hipStreamSynchronize(op->stream))) return KIOPS_ERR_DEVICE;
  if (j_done) *j_done = jd;
  if (beta) *beta = hc.beta;
  if (nu_out) *nu_out = hc.nu;
  return KIOPS_OK;
}

kiops_status kiops_small_expm(int n, const double* Hs, double tau, double* F, double* scratch,
                              void* hip_stream) {
  if (n < 1 || n > kExpmMaxN || !Hs || !F || !scratch || !std::isfinite(tau)) return KIOPS_ERR_INVALID_ARG;
  static_assert(KIOPS_EXPM_SCRATCH_DOUBLES == kExpmSlots * kExpmSlot, "expm scratch size");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  hipLaunchKernelGGL(small_expm_kernel, dim3(1), dim3(kThreads), 0, st, Hs, n, tau, F, scratch);
  if (!hip_ok(hipGetLastError()) || !hip_ok(hipStreamSynchronize(st))) return KIOPS_ERR_DEVICE;
  return KIOPS_OK;
}

kiops_status kiops_batch_plan(int count, const kiops_problem* probs, const kiops_options* opts, int group_size,
                              size_t* workspace_bytes, int* groups, int* group_size_used) {
  BatchPlan B;
  kiops_status s = plan_batch(count, probs, opts, group_size, B);
  if (s != KIOPS_OK) return s;
  if (workspace_bytes) *workspace_bytes = B.total;
  if (groups) *groups = B.ng;
  if (group_size_used) *group_size_used = B.gs;
  return KIOPS_OK;
}

kiops_status kiops_phi_batch(int count, const kiops_problem* probs, const kiops_options* opts, int group_size,
                             void* workspace, size_t workspace_bytes, void* hip_stream, kiops_stats* stats) {
  BatchPlan B;
  kiops_status s = plan_batch(count, probs, opts, group_size, B);
  if (s != KIOPS_OK) return s;
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % kAlign != 0) return KIOPS_ERR_INVALID_ARG;
  if (workspace_bytes < B.total) return KIOPS_ERR_OUT_OF_MEMORY;
  if (stats) std::memset(stats, 0, sizeof(kiops_stats) * count);
  return run_batch(count, probs, B, reinterpret_cast<char*>(workspace), reinterpret_cast<hipStream_t>(hip_stream),
                   stats, nullptr);
}

namespace {
// One autotuner measurement: the better of two runs of the plan (the first
// launch of a kernel instantiation also pays for loading its code).
kiops_status tune_run(int count, const kiops_problem* probs, const BatchPlan& B, void* workspace, void* hip_stream,
                      double* ms) {
  double best = 0.0;
  for (int r = 0; r < 2; ++r) {
    double t = 0.0;
    kiops_status s = run_batch(count, probs, B, reinterpret_cast<char*>(workspace),
                               reinterpret_cast<hipStream_t>(hip_stream), nullptr, &t);
    if (s != KIOPS_OK) return s;
    best = (r == 0 || t < best) ? t : best;
  }
  *ms = best;
  return KIOPS_OK;
}
}  // namespace

kiops_status kiops_batch_tune(int count, const kiops_problem* probs, const kiops_options* opts,
                              const int* candidates, int n, void* workspace, size_t workspace_bytes,
                              void* hip_stream, int* best, double* best_ms) {
  if (!candidates || n < 1 || !best) return KIOPS_ERR_INVALID_ARG;
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % kAlign != 0) return KIOPS_ERR_INVALID_ARG;
  double bms = 0.0;
  int bgs = 0;
  for (int c = 0; c < n; ++c) {
    BatchPlan B;
    kiops_status s = plan_batch(count, probs, opts, candidates[c], B);
    if (s != KIOPS_OK) return s;
    if (workspace_bytes < B.total) return KIOPS_ERR_OUT_OF_MEMORY;
    double ms = 0.0;
    s = tune_run(count, probs, B, workspace, hip_stream, &ms);
    if (s != KIOPS_OK) return s;
    if (bgs == 0 || ms < bms) { bms = ms; bgs = B.gs; }
  }
  *best = bgs;
  if (best_ms) *best_ms = bms;
  return KIOPS_OK;
}

kiops_status kiops_batch_tune_shape(int count, const kiops_problem* probs, const kiops_options* opts,
                                    const int* group_sizes, int ng, const int* tile_rows, int nt,
                                    void* workspace, size_t workspace_bytes, void* hip_stream,
                                    int* best_group_size, int* best_tile_rows, double* best_ms) {
  if (!group_sizes || ng < 1 || !tile_rows || nt < 1 || !best_group_size || !best_tile_rows)
    return KIOPS_ERR_INVALID_ARG;
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % kAlign != 0) return KIOPS_ERR_INVALID_ARG;
  if (count < 1 || !probs || !probs[0].op) return KIOPS_ERR_INVALID_ARG;
  kiops_options o = opts ? *opts : kiops_options{};
  for (int j = 0; j < nt; ++j) {
    o.tile_rows = tile_rows[j];
    if (resolve_tile_rows(&o) < 0) return KIOPS_ERR_INVALID_ARG;
  }
  // one tile shape for the other operator kinds
  const bool shaped = probs[0].op->d.kind == KIOPS_OP_STENCIL2D_5PT && !probs[0].op->d.weights;
  double bms = 0.0;
  int bgs = 0, brows = 0;
  for (int j = 0; j < (shaped ? nt : 1); ++j) {
    o.tile_rows = shaped ? tile_rows[j] : 0;
    for (int i = 0; i < ng; ++i) {
      BatchPlan B;
      kiops_status s = plan_batch(count, probs, &o, group_sizes[i], B);
      if (s != KIOPS_OK) return s;
      if (workspace_bytes < B.total) return KIOPS_ERR_OUT_OF_MEMORY;
      double ms = 0.0;
      s = tune_run(count, probs, B, workspace, hip_stream, &ms);
      if (s != KIOPS_OK) return s;
      if (bgs == 0 || ms < bms) { bms = ms; bgs = B.gs; brows = B.tile_rows; }
    }
  }
  *best_group_size = bgs;
  *best_tile_rows = brows;
  if (best_ms) *best_ms = bms;
  return KIOPS_OK;
}

kiops_status kiops_server_fixed_bytes(int group_size, size_t* bytes, int* groups) {
  int gs = 0, ng = 0;
  kiops_status st = serve_geometry(group_size, &gs, &ng);
  if (st != KIOPS_OK) return st;
  if (bytes) *bytes = serve_layout(gs, ng).pool;
  if (groups) *groups = ng;
  return KIOPS_OK;
}

kiops_status kiops_server_create(int group_size, int64_t points_per_workgroup, void* workspace,
                                 size_t workspace_bytes, void* run_stream, void* io_stream, kiops_server** out) {
  if (!out || !workspace || reinterpret_cast<uintptr_t>(workspace) % kAlign != 0) return KIOPS_ERR_INVALID_ARG;
  if (run_stream == io_stream || points_per_workgroup < 0) return KIOPS_ERR_INVALID_ARG;
  int gs = 0, ng = 0;
  kiops_status st = serve_geometry(group_size, &gs, &ng);
  if (st != KIOPS_OK) return st;
  const ServeLayout SL = serve_layout(gs, ng);
  if (workspace_bytes <= SL.pool) return KIOPS_ERR_OUT_OF_MEMORY;
  if (!kServedEnabled) return KIOPS_ERR_UNSUPPORTED;
  kiops_server* s = new (std::nothrow) kiops_server();
  if (!s) return KIOPS_ERR_OUT_OF_MEMORY;
  s->run = reinterpret_cast<hipStream_t>(run_stream);
  s->io = reinterpret_cast<hipStream_t>(io_stream);
  s->ws = reinterpret_cast<char*>(workspace);
  s->ws_bytes = workspace_bytes;
  s->gs = gs;
  s->ng = ng;
  while (2 * s->max_gang <= ng) s->max_gang *= 2;
  if (points_per_workgroup > 0) s->gang_points = points_per_workgroup;
  int dev = 0, khz = 0;
  hipGetDevice(&dev);
  s->dev = dev;
  s->mail = mailbox_take(dev, mailbox_bytes(ng), &s->mail_bytes);
  if (!s->mail) {
    delete s;
    return KIOPS_ERR_OUT_OF_MEMORY;
  }
  if (!hip_ok(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev)) || khz <= 0) khz = 100000;
  s->clock_hz = (uint64_t)khz * 1000ull;
  s->L = SL;
  s->pool_bytes = (workspace_bytes - SL.pool) / kAlign * kAlign;
  s->free_list[0] = s->pool_bytes;
  s->group_req.assign(ng, -1);
  s->pushed.assign(ng, 0);
  s->last_epoch.assign(ng, 0);
  std::vector<GroupQueue> q(ng);
  for (auto& Q : q) {
    std::memset(&Q, 0, sizeof(GroupQueue));
    Q.idle_limit = s->clock_hz * 600ull;   // a launch nobody feeds ends after ten minutes
    // an idle group polls its queue every few microseconds, not continuously:
    // hundreds of polling workgroups slow the memory accesses of busy ones
    const char* is = std::getenv("KIOPS_IDLE_SLEEP");   // experiment override
    Q.idle_sleep = is ? (unsigned)std::max(0, std::min(64, std::atoi(is))) : 4u;
  }
  // the whole workspace starts at zero: release words that requests leave in
  // the pool carry epochs of this server only (see admit)
  if (!hip_ok(hipMemsetAsync(s->ws, 0, SL.pool + s->pool_bytes, s->io)) ||
      !hip_ok(hipMemsetAsync(s->mail, 0, s->mail_bytes, s->io)) ||
      !hip_ok(hipMemcpyAsync(s->mail, q.data(), sizeof(GroupQueue) * ng, hipMemcpyHostToDevice, s->io)) ||
      !hip_ok(hipStreamSynchronize(s->io))) {
    mailbox_give(s->dev, s->mail_bytes, s->mail);
    delete s;
    return KIOPS_ERR_DEVICE;
  }
  GroupQueue* dq = reinterpret_cast<GroupQueue*>(s->mail);
  unsigned* fin = reinterpret_cast<unsigned*>(s->ws + SL.fin);
  uint64_t fin_limit = s->clock_hz * 60ull;
  void* args[] = {&dq, &fin, &s->gs, &fin_limit};
  if (!hip_ok(hipLaunchCooperativeKernel(kernels_serve(), dim3(ng * gs), dim3(kThreads), args, 0, s->run))) {
    mailbox_give(s->dev, s->mail_bytes, s->mail);
    delete s;
    return KIOPS_ERR_DEVICE;
  }
  *out = s;
  return KIOPS_OK;
}

kiops_status kiops_server_submit(kiops_server* s, const kiops_problem* pr, int64_t* ticket) {
  if (!s || !pr || !ticket) return KIOPS_ERR_INVALID_ARG;
  if (s->dead) return KIOPS_ERR_DEVICE;
  if (!pr->op || !(pr->tau >= 0.0) || !std::isfinite(pr->tau) || !(pr->tol > 0.0) || !std::isfinite(pr->tol) ||
      pr->m_init < 1 || pr->q < 1 || pr->q > kWinMax || pr->p < 0 || pr->p > kServePB)
    return pr->q == 0 ? KIOPS_ERR_UNSUPPORTED : KIOPS_ERR_INVALID_ARG;
  kiops_status st = check_vectors(pr->op, pr->p, pr->V, pr->w);
  if (st != KIOPS_OK) return st;
  if (serve_family(pr->op) < 0) return KIOPS_ERR_UNSUPPORTED;
  if (request_bytes(s, *pr, gang_groups(s, pr->op)) > s->pool_bytes) return KIOPS_ERR_BUDGET;
  kiops_server::Req R;
  R.pr = *pr;
  R.V.assign(pr->V, pr->V + pr->p + 1);
  R.pr.V = nullptr;
  const int64_t t = s->next_ticket++;
  s->reqs.emplace(t, std::move(R));
  s->waiting.push_back(t);
  *ticket = t;
  return kiops_server_progress(s, nullptr, nullptr);
}

kiops_status kiops_server_progress(kiops_server* s, int* running, int* waiting) {
  if (!s) return KIOPS_ERR_INVALID_ARG;
  if (s->dead) return KIOPS_ERR_DEVICE;
  // the done and exited words of every group queue
  std::vector<unsigned> words(2 * s->ng, 0);
  const GroupQueue* dq = reinterpret_cast<const GroupQueue*>(s->mail);
  if (!hip_ok(hipMemcpy2DAsync(words.data(), 2 * sizeof(unsigned), &dq->done, sizeof(GroupQueue),
                               2 * sizeof(unsigned), s->ng, hipMemcpyDeviceToHost, s->io)) ||
      !hip_ok(hipStreamSynchronize(s->io)))
    return KIOPS_ERR_DEVICE;
  for (int g = 0; g < s->ng; ++g) {
    if (words[2 * g + 1]) {   // a group has left: its launch is over
      if (std::getenv("KIOPS_DEBUG")) std::fprintf(stderr, "kiops: server group %d has exited\n", g);
      s->dead = true;
      return KIOPS_ERR_DEVICE;
    }
  }
  // a request is finished when every group of its gang has reported it
  for (int g0 = 0; g0 < s->ng; ++g0) {
    const int64_t t = s->group_req[g0];
    if (t < 0) continue;
    kiops_server::Req& R = s->reqs[t];
    if (R.g0 != g0) continue;
    bool fin = true;
    for (int g = g0; g < g0 + R.k && fin; ++g) fin = words[2 * g] >= s->pushed[g];
    if (!fin) continue;
    unsigned abort_word = 0;
    const Barrier* bar = reinterpret_cast<const Barrier*>(s->ws + s->L.bar) + g0;
    if (!hip_ok(hipMemcpyAsync(&R.ctrl, s->ws + s->L.ctrl + ctrl_stride() * g0, sizeof(Ctrl),
                               hipMemcpyDeviceToHost, s->io)) ||
        !hip_ok(hipMemcpyAsync(&abort_word, &bar->abort, sizeof(unsigned), hipMemcpyDeviceToHost, s->io)) ||
        !hip_ok(hipStreamSynchronize(s->io)))
      return KIOPS_ERR_DEVICE;
    if (abort_word) {   // a bounded wait expired: epochs and queues can no longer be trusted
      R.ctrl.status = KIOPS_ERR_DEVICE;
      s->dead = true;
    }
    R.done = 1;
    pool_free(s, R.pool_off, R.pool_bytes);
    for (int g = g0; g < g0 + R.k; ++g) {
      s->group_req[g] = -1;
      s->last_epoch[g] = R.ctrl.epoch_end;
    }
  }
  if (s->dead) return KIOPS_ERR_DEVICE;
  // admit waiting requests in arrival order; when the head of the queue finds
  // no free gang, its gang is reserved and at most eight later requests may go
  // first elsewhere
  int rlo = 0, rhi = 0;
  for (size_t i = 0; i < s->waiting.size() && i < 9;) {
    const int64_t t = s->waiting[i];
    const kiops_problem& pr = s->reqs[t].pr;
    const int k = gang_groups(s, pr.op);
    const int g0 = free_gang(s, k, rlo, rhi);
    const size_t bytes = request_bytes(s, pr, k);
    size_t off = 0;
    if (g0 >= 0 && pool_alloc(s, bytes, &off)) {
      kiops_status st = admit(s, t, g0, k, off, bytes);
      if (st != KIOPS_OK) return st;
      s->waiting.erase(s->waiting.begin() + i);
      continue;
    }
    if (i == 0 && g0 < 0) {
      rlo = reserve_gang(s, k);
      rhi = rlo + k;
    }
    ++i;
  }
  if (running) {
    int r = 0;
    for (int g = 0; g < s->ng; ++g) {
      const int64_t t = s->group_req[g];
      r += t >= 0 && s->reqs[t].g0 == g;
    }
    *running = r;
  }
  if (waiting) *waiting = (int)s->waiting.size();
  return KIOPS_OK;
}

kiops_status kiops_server_result(kiops_server* s, int64_t ticket, int* done, kiops_stats* stats) {
  if (!s || !done) return KIOPS_ERR_INVALID_ARG;
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return KIOPS_ERR_INVALID_ARG;
  *done = it->second.done;
  if (it->second.done) {
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      fill_stats(it->second.ctrl, it->second.k * s->gs, (double)s->clock_hz, stats);
    }
    s->reqs.erase(it);
  }
  return KIOPS_OK;
}

kiops_status kiops_server_destroy(kiops_server* s) {
  if (!s) return KIOPS_ERR_INVALID_ARG;
  const unsigned one = 1;
  GroupQueue* dq = reinterpret_cast<GroupQueue*>(s->mail);
  kiops_status st = KIOPS_OK;
  for (int g = 0; g < s->ng; ++g)
    if (!hip_ok(hipMemcpyAsync(&dq[g].closed, &one, sizeof(one), hipMemcpyHostToDevice, s->io))) st = KIOPS_ERR_DEVICE;
  if (!hip_ok(hipStreamSynchronize(s->io)) || !hip_ok(hipStreamSynchronize(s->run))) st = KIOPS_ERR_DEVICE;
  // the launch has ended (or the device is lost): the mailbox can serve
  // another server, unless the launch may still be running
  if (st == KIOPS_OK) mailbox_give(s->dev, s->mail_bytes, s->mail);
  delete s;
  return st;
}

kiops_status kiops_controller_decide(const kiops_ctrl_in* in, int j, double eps, int breakdown,
                                     kiops_ctrl_out* out) {
  if (!in || !out) return KIOPS_ERR_INVALID_ARG;
  CtrlIn ci;
  static_assert(sizeof(CtrlIn) == sizeof(kiops_ctrl_in), "controller input layout");
  static_assert(sizeof(CtrlOut) == sizeof(kiops_ctrl_out), "controller output layout");
  std::memcpy(&ci, in, sizeof(ci));
  const CtrlOut o = ctrl_decide(ci, j, eps, breakdown != 0);
  std::memcpy(out, &o, sizeof(o));
  return KIOPS_OK;
}

}  // extern "C"
