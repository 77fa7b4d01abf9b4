// Periodic 5-point stencil (2-D), constant diffusivity and advection,
// per-cell reaction (the operator of op_stencil2d.h), by row marching for
// large grids.
//
// A work item is a strip of W = 256 columns (one column per thread) over a
// chunk of rows; the workgroup marches through the chunk row by row, so each
// row of R_{kp-1}, r, B and the older window vector is loaded once, and the
// loads of the next kDepth - 1 row steps are in flight while a row is
// processed.  LDS holds a ring of three rows of R_{kp-1} (x-halo 2) and of
// R_kp (x-halo 1).
//
// The x-halo columns of the strip (two of R_{kp-1} and one of r, the older
// vector and B on each side) are fetched for every row of the chunk at the
// start of the item, one load per array (a lane per halo entry), and kept in
// LDS: a row step then issues only the loads of its own 256 columns.
// (Loading the halo columns row by row doubled the load instructions of a
// step, most of them with no lane active, and cost 13 of 58 us per pass at
// 2048^2, measured on the pass alone.)
//
// Row step j (formation row f = y_j + s, s = +-1 the march direction):
//   write R_{kp-1}(f + s) into the ring; form R_kp(f) on the x-halo-1 range
//   from U_{kp-1}(f) = A~ R_{kp-1}(f) (rows f - s, f, f + s); then, for the
//   output row y_j, U_kp = A~ R_kp (rows y_j - s, y_j, y_j + s), store R_kp(y_j)
//   and accumulate the inner products.  Two barriers per row.
//
// Chunks of a strip alternate direction (even chunks downwards, odd ones
// upwards), so two neighbouring chunks read their shared halo rows at the
// same time (both at the start of their march or both at the end), on the
// same XCD: the re-read is served by that XCD's L2.
//
// The arithmetic of a point is that of the tile pass (same operations in the
// same order), and windows of at most two vectors (IOP q = 1, 2) are served.
#pragma once

#include "buffer.h"
#include "pass_common.h"

namespace kiops {

template <typename T, int PB>
struct Stencil2DMarch {
  static constexpr int W = kThreads;          // strip width: one column per thread
  static constexpr int kRowR = W + 4;         // R_{kp-1} row with an x-halo of two
  static constexpr int kRowX = W + 2;         // R_kp row with an x-halo of one
  static constexpr int kDepth = 4;            // row steps whose loads are issued before the first is used
  static constexpr int kChunkRows = 32;       // most rows of a work item (the loop over them is unrolled)
  static constexpr int kMaxRows = kChunkRows;
  static constexpr int kPB = PB > 0 ? PB : 1;
  static constexpr int kHF = 2 + kPB;         // halo arrays of the formation: r, older vector, B
  static constexpr int kHRows = kMaxRows + 4; // relative rows -2 .. nrows + 1
  static constexpr int kLdsT = 3 * kRowR + 3 * kRowX + 4 * kHRows + 2 * kHF * kHRows;
  static constexpr int kLdsDoubles = (int)((kLdsT * sizeof(T) + 7) / 8);
  static constexpr bool kTwoPhase = false;    // one fused pass per Krylov step
  static constexpr int kWavesPerEU = 2;       // 256-VGPR budget: two workgroups per CU
  static_assert(4 * kHRows <= kThreads && 2 * kHRows <= kThreads, "one lane per halo entry");

  // loads of one row step at the thread's column
  struct RowLoads {
    T vr;               // R_{kp-1} at the row ahead
    T rv, ov, bv[kPB];  // r, the older vector (or w), B at the formation row
  };

  int64_t N;
  int nx, ny, nstrips, nchunks, nitems;   // item = strip * nchunks + chunk
  T wE, wW, wN, wS, wC;
  const T* r;
  const T* B[kPM];   // B[c] = b_{p-c} (Theorem 1 column order)
  int p;
  const double* r_src;   // mixed precision: float copy r <- r_src made at setup
  T* r_dst;
  T* ubuf;               // unused: windows of at most two vectors

  // y mod n for y in [-2n, 3n), without a branch (wave-uniform rows)
  __device__ static int wrap_row(int y, int n) {
    y = y < 0 ? y + n : y;
    y = y < 0 ? y + n : y;
    y = y >= n ? y - n : y;
    y = y >= n ? y - n : y;
    return y;
  }

  __device__ void setup_coefficients(const KParams& P, int64_t gt, int64_t gs) const {
    if (r_dst && r_src)
      for (int64_t n = gt; n < P.N; n += gs) r_dst[n] = (T)r_src[n];
  }

  __device__ void pass(const PassCtx<T>& c, const BasisPtrs<T>& bp, const double* w, T* Rout,
                       DotAcc& acc, T* lds) const {
    T* sR = lds;                    // 3 rows of kRowR: R_{kp-1} at column lx, index lx + 2
    T* sX = sR + 3 * kRowR;         // 3 rows of kRowX: R_kp at column lx, index lx + 1
    T* hR = sX + 3 * kRowX;         // R_{kp-1} halo: [m + 2][4] at columns -2, -1, wid, wid + 1
    T* hF = hR + 4 * kHRows;        // formation halo: [array][m + 1][2] at columns -1, wid
    const int t = threadIdx.x;
    const bool first = c.first != 0;
    const uint64_t nb = (uint64_t)N * sizeof(T);
    const bool has_old = !first && c.flo < c.src;   // R_{kp-2} in the window
    const bool win = c.ngd > 0;                     // inner products with R_{kp-1}
    const __amdgpu_buffer_rsrc_t rsR = make_rsrc(first ? nullptr : bp.get(c.src), nb);
    const __amdgpu_buffer_rsrc_t rsO = make_rsrc(has_old ? bp.get(c.src - 1) : nullptr, nb);
    const __amdgpu_buffer_rsrc_t rsW = make_rsrc(first ? w : nullptr, (uint64_t)N * 8);
    // FP64: the formation's second vector is w in the first pass, else R_{kp-2}
    const __amdgpu_buffer_rsrc_t rsOW =
        make_rsrc(first ? (const void*)w : (has_old ? (const void*)bp.get(c.src - 1) : nullptr), nb);
    const __amdgpu_buffer_rsrc_t rsr = make_rsrc(r, nb);
    const __amdgpu_buffer_rsrc_t rsOut = make_rsrc(c.write_out ? Rout : nullptr, nb);
    __amdgpu_buffer_rsrc_t rsB[kPB];
#pragma unroll
    for (int k = 0; k < kPB; ++k) rsB[k] = make_rsrc(k < PB && k < c.p ? B[k] : nullptr, nb);
    const T a = c.a, bsrc = c.bw[c.src], bold = has_old ? c.bw[c.src - 1] : T(0);

    // XCD-aware order (as in the tile pass): one contiguous band of the item
    // sequence per XCD, swept together by the band's workgroups; items of a
    // strip are consecutive, so neighbouring chunks run on one XCD
    const int nband = vgrid() < kXcds ? vgrid() : kXcds;
    const int band = vblock() % nband;
    const int nloc = (vgrid() - band + nband - 1) / nband;
    const int i_lo = (int)((int64_t)nitems * band / nband);
    const int i_hi = (int)((int64_t)nitems * (band + 1) / nband);
    // Two workgroups per CU (c.ranks == 2): the second half of the grid is
    // dispatched second onto every CU, and the SIMD arbitration favours the
    // older waves, so with equal priority the second workgroup of a CU fell
    // far behind the first (measured at 2048^2: 52 against 67 us per pass).
    // The later workgroup runs at a raised wave priority for the first third
    // of its rows, the earlier one for the other two thirds: both then arrive
    // together (55 and 55 us, the latest arrival 59 instead of 75 us).
    const bool two_per_cu = c.ranks == 2;
    const bool late = two_per_cu && vblock() >= vgrid() / 2;
    if (late) __builtin_amdgcn_s_setprio(1);
    for (int item = i_lo + vblock() / nband; item < i_hi; item += nloc) {
      const int strip = item / nchunks;
      const int chunk = item - strip * nchunks;
      const int x0 = strip * W;
      const int wid = (nx - x0) < W ? (nx - x0) : W;
      const int ylo = (int)((int64_t)ny * chunk / nchunks);
      const int yhi = (int)((int64_t)ny * (chunk + 1) / nchunks);
      const int nrows = yhi - ylo;
      const int s = (chunk & 1) ? -1 : 1;          // march direction
      const int ystart = s > 0 ? ylo : yhi - 1;
      const bool col = t < wid;                     // the thread's column is inside the strip
      const int gx = col ? x0 + t : 0;
      // row of relative index m (m in [-2, nrows + 1], so ystart + m s lies in
      // [-ny - 1, 2 ny + 1))
      auto row_of = [&](int m) { return wrap_row(ystart + m * s, ny); };
      auto slot = [](int m) { return (m + 6) % 3; };                         // ring slot of index m >= -2

      // ---- the halo columns of every row of the item, one load per array:
      // lane e < 4 (nrows + 4) takes R_{kp-1} at relative row e / 4 - 2 and
      // column {-2, -1, wid, wid + 1}[e % 4]; lane e < 2 (nrows + 2) the
      // formation arrays at row e / 2 - 1 and column {-1, wid}[e % 2].  They
      // are written to LDS after the first row loads have been issued.
      const bool inr = t < 4 * (nrows + 4), inf = t < 2 * (nrows + 2);
      T hv_r, hv_rr, hv_o, hv_b[kPB];
      {
        const int er = t & 3, ef = t & 1;
        const int hx = er == 0 ? -2 : (er == 1 ? -1 : (er == 2 ? wid : wid + 1));
        const int fx = ef == 0 ? -1 : wid;
        const uint32_t ir = (uint32_t)row_of((t >> 2) - 2) * (uint32_t)nx + (uint32_t)wrap_index(x0 + hx, nx);
        const uint32_t jf = (uint32_t)row_of((t >> 1) - 1) * (uint32_t)nx + (uint32_t)wrap_index(x0 + fx, nx);
        const uint32_t offf = inf ? jf * (uint32_t)sizeof(T) : kNoOffset;
        hv_r = buf_ld(rsR, inr ? ir * (uint32_t)sizeof(T) : kNoOffset, T(0));
        hv_rr = buf_ld(rsr, offf, T(0));
        if constexpr (sizeof(T) == 8) {
          hv_o = buf_ld(rsOW, offf, T(0));
        } else {
          const double w0 = buf_ld(rsW, inf ? jf * 8u : kNoOffset, 0.0);
          const T o0 = buf_ld(rsO, offf, T(0));
          hv_o = first ? (T)w0 : o0;
        }
#pragma unroll
        for (int k = 0; k < kPB; ++k) hv_b[k] = buf_ld(rsB[k], offf, T(0));
      }

      // every global load of row step j: R_{kp-1} at relative row j + 2, and
      // r, the older vector (or w) and B at relative row j + 1.  The steps
      // past the chunk load the last step's rows again (unused, served by the
      // caches), so every row step issues the same loads in the same order,
      // with no branch: the waits for a step's loads then count exactly the
      // later steps' loads.
      const int jlast = nrows - 1;
      auto issue = [&](int j, RowLoads& L) {
        const int jj = j < jlast ? j : jlast;
        const uint32_t ra = (uint32_t)row_of(jj + 2) * (uint32_t)nx;
        const uint32_t rf = (uint32_t)row_of(jj + 1) * (uint32_t)nx;
        L.vr = buf_ld(rsR, col ? (ra + gx) * (uint32_t)sizeof(T) : kNoOffset, T(0));
        const uint32_t fo = col ? (rf + gx) * (uint32_t)sizeof(T) : kNoOffset;
        L.rv = buf_ld(rsr, fo, T(0));
        if constexpr (sizeof(T) == 8) {
          // w (first pass) and the older vector are both FP64: one load
          L.ov = buf_ld(rsOW, fo, T(0));
        } else {
          // mixed: w is FP64, R_{kp-2} FP32; both loads are issued (one of the
          // two resources is empty) so that no branch separates them
          const double w0 = buf_ld(rsW, col ? (rf + gx) * 8u : kNoOffset, 0.0);
          const T o0 = buf_ld(rsO, fo, T(0));
          L.ov = first ? (T)w0 : o0;
        }
#pragma unroll
        for (int k = 0; k < kPB; ++k) L.bv[k] = buf_ld(rsB[k], fo, T(0));
      };
      // U_{kp-1} at column lx of the formation row (ring rows behind, centre,
      // ahead), then R_kp there
      auto form = [&](const T* Rb, const T* Rc, const T* Ra, int lx, T rv, T ov, T bprev) {
        if (first) return ov;
        const int o = lx + 2;
        const T ctr = Rc[o];
        const T vN = s > 0 ? Ra[o] : Rb[o];   // row y + 1
        const T vS = s > 0 ? Rb[o] : Ra[o];   // row y - 1
        T U = wE * Rc[o + 1];
        U = fma(wW, Rc[o - 1], U);
        U = fma(wN, vN, U);
        U = fma(wS, vS, U);
        U = fma(wC + rv, ctr, U);
        U += bprev;
        T X = a * U;
        X = fma(bsrc, ctr, X);
        if (has_old) X = fma(bold, ov, X);
        return X;
      };

      // prologue: R_{kp-1} at relative rows -2 and -1 of the strip's columns,
      // the loads of the first kDepth - 1 row steps, then the LDS writes of
      // the halo buffers and of the two rows
      const uint32_t r0 = (uint32_t)row_of(-2) * (uint32_t)nx, r1 = (uint32_t)row_of(-1) * (uint32_t)nx;
      const T a0 = buf_ld(rsR, col ? (r0 + gx) * (uint32_t)sizeof(T) : kNoOffset, T(0));
      const T a1 = buf_ld(rsR, col ? (r1 + gx) * (uint32_t)sizeof(T) : kNoOffset, T(0));
      RowLoads Ls[kDepth];
#pragma unroll
      for (int u = 0; u < kDepth - 1; ++u) issue(u - 2, Ls[u]);
      if (inr) hR[t] = hv_r;
      if (inf) {
        hF[0 * 2 * kHRows + t] = hv_rr;
        hF[1 * 2 * kHRows + t] = hv_o;
#pragma unroll
        for (int k = 0; k < kPB; ++k) hF[(2 + k) * 2 * kHRows + t] = hv_b[k];
      }
      if (col) {
        sR[slot(-2) * kRowR + t + 2] = a0;
        sR[slot(-1) * kRowR + t + 2] = a1;
      }
      __syncthreads();   // hR and hF written
      // halo lanes: the R_{kp-1} halo copy on lanes 0..3 of wave 0, the
      // formation halo on lanes 0 and 1 of wave 1 (spreading the extra work)
      const int hxl = t == 0 ? -2 : (t == 1 ? -1 : (t == 2 ? wid : wid + 1));
      const int tf = t - 64;
      const int fxl = tf == 0 ? -1 : wid;
      if (t < 4) {
        sR[slot(-2) * kRowR + hxl + 2] = hR[0 * 4 + t];
        sR[slot(-1) * kRowR + hxl + 2] = hR[1 * 4 + t];
      }
      // R_{kp-1} of the thread's column at relative rows j and j + 1 (the
      // window inner products), r and B y_cur at the output row
      T hist0 = T(0), hist1 = T(0), r_out = T(0), bc_out = T(0);
      auto process = [&](int j, const RowLoads& L) {
        const int m = j + 1;   // formation row
        if (two_per_cu && j == nrows / 3) {
          if (late) __builtin_amdgcn_s_setprio(0);
          else __builtin_amdgcn_s_setprio(1);
        }
        T* Rb = sR + slot(m - 1) * kRowR;
        T* Rc = sR + slot(m) * kRowR;
        T* Ra = sR + slot(m + 1) * kRowR;
        if (col) Ra[t + 2] = L.vr;
        if (t < 4) Ra[hxl + 2] = hR[(m + 1 + 2) * 4 + t];
        __syncthreads();
        // ---- R_kp on the formation row, columns -1 .. wid
        T bprev = T(0), bcur = T(0);
#pragma unroll
        for (int k = 0; k < kPB; ++k) {
          if (k < PB) {
            bprev = fma(L.bv[k], c.ybp[k], bprev);
            bcur = fma(L.bv[k], c.ybc[k], bcur);
          }
        }
        T* Xf = sX + slot(m) * kRowX;
        if (col) Xf[t + 1] = form(Rb, Rc, Ra, t, L.rv, L.ov, bprev);
        if (tf >= 0 && tf < 2) {
          const int e = (m + 1) * 2 + tf;
          T bpx = T(0);
#pragma unroll
          for (int k = 0; k < kPB; ++k)
            if (k < PB) bpx = fma(hF[(2 + k) * 2 * kHRows + e], c.ybp[k], bpx);
          Xf[fxl + 1] = form(Rb, Rc, Ra, fxl, hF[e], hF[2 * kHRows + e], bpx);
        }
        __syncthreads();
        // ---- U_kp on the output row j, output and inner products
        if (j >= 0) {
          const T* Xb = sX + slot(j - 1) * kRowX;
          const T* Xc = sX + slot(j) * kRowX;
          const T* Xa = sX + slot(j + 1) * kRowX;
          const int o = t + 1;
          const T X = Xc[o];
          const T vN = s > 0 ? Xa[o] : Xb[o];
          const T vS = s > 0 ? Xb[o] : Xa[o];
          T U = wE * Xc[o + 1];
          U = fma(wW, Xc[o - 1], U);
          U = fma(wN, vN, U);
          U = fma(wS, vS, U);
          U = fma(wC + r_out, X, U);
          U += bc_out;
          const uint32_t oo = col ? ((uint32_t)row_of(j) * (uint32_t)nx + gx) * (uint32_t)sizeof(T) : kNoOffset;
          buf_st(rsOut, oo, X);
          const double Xd = col ? (double)X : 0.0, Ud = col ? (double)U : 0.0;
          acc.RR = fma(Xd, Xd, acc.RR);
          acc.UU = fma(Ud, Ud, acc.UU);
          acc.Ck = fma(Xd, Ud, acc.Ck);
          if (win) {
            const double Rv = (double)hist0;
            acc.G[0] = fma(Rv, Xd, acc.G[0]);
            acc.C[0] = fma(Rv, Ud, acc.C[0]);
          }
        }
        hist0 = hist1;
        hist1 = L.vr;
        r_out = L.rv;
        bc_out = bcur;
      };
      // steps j = -2 .. jlast, at most kMaxRows + 2: the loop is unrolled
      // completely, so no register set is carried around a loop edge (the
      // compiler would copy the sets there and wait for every load first);
      // loads run kDepth - 1 steps ahead and are issued unconditionally (past
      // the chunk they repeat its last rows), so each wait counts exactly the
      // later steps' loads
#pragma unroll
      for (int u = 0; u < kMaxRows + 2; ++u) {
        issue(u - 2 + kDepth - 1, Ls[(u + kDepth - 1) % kDepth]);
        if (u - 2 <= jlast) process(u - 2, Ls[u % kDepth]);
      }
      __syncthreads();   // the rings and halo buffers are reused by the next item
    }
    if (two_per_cu) __builtin_amdgcn_s_setprio(0);
  }
};

}  // namespace kiops
