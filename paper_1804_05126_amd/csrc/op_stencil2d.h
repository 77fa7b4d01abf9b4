// Periodic 5-point stencil (2-D), constant diffusivity and advection,
// per-cell reaction:
//
//   (A u)_P = wE u_E + wW u_W + wN u_N + wS u_S + (wC + r_P) u_P,
//   wE = D/h^2 - ax/(2h), wW = D/h^2 + ax/(2h), wN = D/h^2 - ay/(2h),
//   wS = D/h^2 + ay/(2h), wC = -4 D/h^2   (E/W = x+-1, N/S = y+-1).
//
// Tiling: a workgroup of 256 threads owns a 64 x 16 tile of outputs.  R_{kp-1}
// is staged in LDS over the tile plus a halo of two; U_{kp-1} and then R_kp
// are formed on the tile plus a halo of one (a second LDS buffer); the
// stencil of R_kp gives U_kp on the tile.  Each thread owns one column of four
// consecutive rows of the tile (plus at most one position of the halo ring),
// so a wave's loads and stores cover 64 consecutive elements of a row.
//
// Every global load of a tile (the halo-2 region of R_{kp-1} and, at the
// thread's five positions, r, the p columns of B and the older window vector)
// is issued before the first use, so a tile costs one memory round trip.
// PB bounds p at compile time so that these loads land in registers.  All
// arrays are addressed as uniform base + 32-bit byte offset (one offset per
// position serves every array), so an array is limited to 4 GiB.
#pragma once

#include "buffer.h"
#include "pass_common.h"

namespace kiops {

// kWide: the instantiation for windows of 3 or 4 vectors (IOP q = 3, 4), which
// loads the one or two vectors older than R_{kp-2} with the tile, like the
// other arrays, and reuses them and R_{kp-2} for the window's inner products;
// a separate kernel, so that the common window of 2 keeps its own register
// allocation (the same code in one kernel cost q = 2 2%, measured).
// kTY: rows of a tile (16, 8 or 4; the batched form takes the height its
// autotuner picks: shorter tiles give small grids more work items, taller ones
// re-read fewer halo rows).  Each wave covers kTY / 4 rows of 64 columns.
template <typename T, int PB, bool kWide, int kTY = 16>
struct Stencil2DT {
  static constexpr int TX = 64, TY = kTY;
  static_assert(kTY == 4 || kTY == 8 || kTY == 16, "tile rows");
  static constexpr int kRW = kTY / 4;              // tile rows per wave (positions per thread)
  static constexpr int RX = TX + 4, RY = TY + 4;   // halo-2 region (R_{kp-1})
  static constexpr int SX = TX + 2, SY = TY + 2;   // halo-1 region (R_kp)
  static constexpr int kRingPos = SX * SY - TX * TY;  // halo-1 positions outside the tile
  static constexpr int kRegion = RX * RY;
  static constexpr int kRegionLoads = (kRegion + kThreads - 1) / kThreads;
  static constexpr int kPos = kRW + 1;             // kRW tile positions + 1 ring position
  static constexpr int kLdsT = RX * RY + SX * SY;  // elements of T
  static constexpr int kLdsDoubles = (int)((kLdsT * sizeof(T) + 7) / 8);
  static constexpr bool kTwoPhase = false;   // one fused pass per Krylov step
  // register budget of 256 VGPRs (two waves per SIMD, the two workgroups per
  // CU the grid uses): a tile's loads are held in registers, and at 168 or 128
  // the pass spills to scratch in its loop (measured: 3-4% slower per step at
  // 168, more after unrelated code changes shift the allocation)
  static constexpr int kWavesPerEU = 2;

  int64_t N;
  int nx, ny, tiles_x, ntiles;
  T wE, wW, wN, wS, wC;
  const T* r;
  const T* B[kPM];   // B[c] = b_{p-c} (Theorem 1 column order)
  int p;
  const double* r_src;   // mixed precision: float copy r <- r_src made at setup
  T* r_dst;
  T* ubuf;               // full window: U_kp output

  __device__ void setup_coefficients(const KParams& P, int64_t gt, int64_t gs) const {
    if (r_dst && r_src)
      for (int64_t n = gt; n < P.N; n += gs) r_dst[n] = (T)r_src[n];
  }

  __device__ static void ring_pos(int e, int& rx, int& ry) {
    // e in [0, kRingPos): top row, bottom row, left column, right column of the halo-1 ring
    if (e < SX) { rx = e - 1; ry = -1; return; }
    e -= SX;
    if (e < SX) { rx = e - 1; ry = TY; return; }
    e -= SX;
    if (e < TY) { rx = -1; ry = e; return; }
    e -= TY;
    rx = TX; ry = e;
  }

  __device__ void pass(const PassCtx<T>& c, const BasisPtrs<T>& bp, const double* w, T* Rout,
                       DotAcc& acc, T* lds) const {
    T* sR = lds;
    T* sX = lds + RX * RY;
    const int t = threadIdx.x;
    const int cx = t & (TX - 1);
    const int rg = (t >> 6) * kRW;
    const bool first = c.first != 0;
    const uint64_t nb = (uint64_t)N * sizeof(T);
    const bool has_old = !first && c.flo < c.src;          // R_{kp-2} in the window
    const bool more_old = !first && c.flo < c.src - 1;     // windows wider than 2
    const int n_extra = more_old ? c.src - 1 - c.flo : 0;   // vectors older than R_{kp-2}
    const bool near_old = kWide && n_extra > 0 && n_extra <= 2;
    const __amdgpu_buffer_rsrc_t rsE1 = make_rsrc(near_old ? bp.get(c.flo) : nullptr, nb);
    const __amdgpu_buffer_rsrc_t rsE2 = make_rsrc(near_old && n_extra == 2 ? bp.get(c.flo + 1) : nullptr, nb);
    const __amdgpu_buffer_rsrc_t rsR = make_rsrc(first ? nullptr : bp.get(c.src), nb);
    const __amdgpu_buffer_rsrc_t rsO = make_rsrc(has_old ? bp.get(c.src - 1) : nullptr, nb);
    const __amdgpu_buffer_rsrc_t rsW = make_rsrc(first ? w : nullptr, (uint64_t)N * 8);
    const __amdgpu_buffer_rsrc_t rsr = make_rsrc(r, nb);
    const __amdgpu_buffer_rsrc_t rsOut = make_rsrc(c.write_out ? Rout : nullptr, nb);
    const bool store_u = uniform(c.store_u) != 0;   // full window only: no store otherwise
    const __amdgpu_buffer_rsrc_t rsU = make_rsrc(store_u ? ubuf : nullptr, nb);
    __amdgpu_buffer_rsrc_t rsB[PB > 0 ? PB : 1];
#pragma unroll
    for (int k = 0; k < PB; ++k) rsB[k] = make_rsrc(k < c.p ? B[k] : nullptr, nb);
    int prx[kPos], pry[kPos];
#pragma unroll
    for (int i = 0; i < kRW; ++i) { prx[i] = cx; pry[i] = rg + i; }
    const bool ring = t < kRingPos;
    ring_pos(ring ? t : 0, prx[kRW], pry[kRW]);

    // XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs, so
    // workgroup b runs on XCD b % 8.  Each XCD takes one contiguous band of the
    // row-major tile sequence, and its workgroups sweep the band together, so
    // the tiles in flight on an XCD are horizontal and vertical neighbours and
    // their halos and rings are served by that XCD's L2.  (Grids smaller than
    // 8 use as many bands as workgroups.)
    const int nband = vgrid() < kXcds ? vgrid() : kXcds;
    const int band = vblock() % nband;
    const int nloc = (vgrid() - band + nband - 1) / nband;   // workgroups of this band
    const int t_lo = (int)((int64_t)ntiles * band / nband);
    const int t_hi = (int)((int64_t)ntiles * (band + 1) / nband);
    for (int tile = t_lo + vblock() / nband; tile < t_hi; tile += nloc) {
      const int x0 = (tile % tiles_x) * TX;
      const int y0 = (tile / tiles_x) * TY;
      // ---- issue every load of the tile
      T reg[kRegionLoads];
#pragma unroll
      for (int i = 0; i < kRegionLoads; ++i) {
        const int e = t + i * kThreads;
        const int ry2 = e / RX, rx2 = e - ry2 * RX;
        const int gx = wrap_index(x0 - 2 + rx2, nx);
        const int gy = wrap_index(y0 - 2 + ry2, ny);
        const uint32_t off = (e < kRegion) ? (uint32_t)(gy * nx + gx) * (uint32_t)sizeof(T) : kNoOffset;
        reg[i] = buf_ld(rsR, off, T(0));
      }
      uint32_t goff[kPos];
      T rv[kPos], ov[kPos], bv[kPos][PB > 0 ? PB : 1];
      T e1[kWide ? kPos : 1], e2[kWide ? kPos : 1];
#pragma unroll
      for (int q = 0; q < kPos; ++q) {
        const int gx = wrap_index(x0 + prx[q], nx);
        const int gy = wrap_index(y0 + pry[q], ny);
        const uint32_t idx = (uint32_t)(gy * nx + gx);
        goff[q] = (q < kRW || ring) ? idx * (uint32_t)sizeof(T) : kNoOffset;
        rv[q] = buf_ld(rsr, goff[q], T(0));
        if (first) ov[q] = (T)buf_ld(rsW, (q < kRW || ring) ? idx * 8u : kNoOffset, 0.0);
        else ov[q] = buf_ld(rsO, goff[q], T(0));
#pragma unroll
        for (int k = 0; k < PB; ++k) bv[q][k] = buf_ld(rsB[k], goff[q], T(0));
        if constexpr (kWide) {
          e1[q] = T(0);
          e2[q] = T(0);
          if (near_old) {
            e1[q] = buf_ld(rsE1, goff[q], T(0));
            if (n_extra == 2) e2[q] = buf_ld(rsE2, goff[q], T(0));
          }
        }
      }
      // ---- R_{kp-1} region into LDS
      if (!first) {
#pragma unroll
        for (int i = 0; i < kRegionLoads; ++i) {
          const int e = t + i * kThreads;
          if (e < kRegion) sR[e] = reg[i];
        }
      }
      __syncthreads();
      // ---- form R_kp on the halo-1 region
      T bcur[kRW];
#pragma unroll
      for (int q = 0; q < kPos; ++q) {
        if (q < kRW || ring) {
          T bprev = T(0), bc = T(0);
#pragma unroll
          for (int k = 0; k < PB; ++k) {
            bprev = fma(bv[q][k], c.ybp[k], bprev);
            bc = fma(bv[q][k], c.ybc[k], bc);
          }
          if (q < kRW) bcur[q] = bc;
          T X;
          if (first) {
            X = ov[q];
          } else {
            const int o = (pry[q] + 2) * RX + (prx[q] + 2);
            const T ctr = sR[o];
            T U = wE * sR[o + 1];
            U = fma(wW, sR[o - 1], U);
            U = fma(wN, sR[o + RX], U);
            U = fma(wS, sR[o - RX], U);
            U = fma(wC + rv[q], ctr, U);
            U += bprev;
            X = c.a * U;
            X = fma(c.bw[c.src], ctr, X);
            if (has_old) X = fma(c.bw[c.src - 1], ov[q], X);
            if (near_old) {
              if constexpr (kWide) {
                X = fma(c.bw[c.flo], e1[q], X);
                if (n_extra == 2) X = fma(c.bw[c.flo + 1], e2[q], X);
              }
            } else if (more_old) {
              // older window vectors (a full window streams every earlier
              // vector: eight loads in flight at a time)
              int i = c.flo;
              for (; i + 8 <= c.src - 1; i += 8) {
                T v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = buf_ld(make_rsrc(bp.get(i + u), nb), goff[q], T(0));
#pragma unroll
                for (int u = 0; u < 8; ++u) X = fma(c.bw[i + u], v[u], X);
              }
              for (; i < c.src - 1; ++i) X = fma(c.bw[i], buf_ld(make_rsrc(bp.get(i), nb), goff[q], T(0)), X);
            }
          }
          sX[(pry[q] + 1) * SX + (prx[q] + 1)] = X;
        }
      }
      __syncthreads();
      // ---- U_kp on the tile, output and inner products
#pragma unroll
      for (int i = 0; i < kRW; ++i) {
        const int ry = rg + i;
        const bool valid = (x0 + cx < nx) && (y0 + ry < ny);
        const int o = (ry + 1) * SX + (cx + 1);
        const T X = sX[o];
        T U = wE * sX[o + 1];
        U = fma(wW, sX[o - 1], U);
        U = fma(wN, sX[o + SX], U);
        U = fma(wS, sX[o - SX], U);
        U = fma(wC + rv[i], X, U);
        U += bcur[i];
        buf_st(rsOut, valid ? goff[i] : kNoOffset, X);
        if (store_u) buf_st(rsU, valid ? goff[i] : kNoOffset, U);
        const double Xd = valid ? (double)X : 0.0, Ud = valid ? (double)U : 0.0;
        acc.RR = fma(Xd, Xd, acc.RR);
        acc.UU = fma(Ud, Ud, acc.UU);
        acc.Ck = fma(Xd, Ud, acc.Ck);
#pragma unroll
        for (int d = 0; d < kWinMax - 1; ++d) {
          if (d < c.ngd) {
            const int idx = c.dlo + d;
            double Rv;
            if constexpr (kWide) {
              if (idx == c.src) Rv = (double)sR[(ry + 2) * RX + (cx + 2)];
              else if (idx == c.src - 1 && has_old) Rv = (double)ov[i];
              else if (near_old && idx == c.flo) Rv = (double)e1[i];
              else if (near_old && n_extra == 2 && idx == c.flo + 1) Rv = (double)e2[i];
              else Rv = (double)buf_ld(make_rsrc(bp.get(idx), nb), goff[i], T(0));
            } else {
              Rv = (idx == c.src) ? (double)sR[(ry + 2) * RX + (cx + 2)]
                                  : (double)buf_ld(make_rsrc(bp.get(idx), nb), goff[i], T(0));
            }
            acc.G[d] = fma(Rv, Xd, acc.G[d]);
            acc.C[d] = fma(Rv, Ud, acc.C[d]);
          }
        }
      }
      __syncthreads();
    }
  }
};

template <typename T, int PB>
using Stencil2D = Stencil2DT<T, PB, false>;
template <typename T, int PB>
using Stencil2DWide = Stencil2DT<T, PB, true>;
template <typename T, int PB>
using Stencil2DRows8 = Stencil2DT<T, PB, false, 8>;   // batched form: 64 x 8 tiles
template <typename T, int PB>
using Stencil2DRows4 = Stencil2DT<T, PB, false, 4>;   // batched form: 64 x 4 tiles

}  // namespace kiops
