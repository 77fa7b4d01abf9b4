// Periodic 7-point stencil in 3-D with per-cell diffusivity (the 5-point
// variable-coefficient 2-D operator is the case nz = 1):
//
//   (A u)_P = sum_d [ kf+_d (u_{P+e_d} - u_P) - kf-_d (u_P - u_{P-e_d}) ] / h^2
//             - a_d (u_{P+e_d} - u_{P-e_d}) / (2 h) + r_P u_P,
//   kf+-_d = (kappa_P + kappa_{P+-e_d}) / 2   (or the constant diff),
//
// flat index x + nx (y + ny z).  Along an axis of length 1 both differences
// vanish, which is what the wrapped neighbour (the cell itself) gives.
//
// Tiling (2.5-D): a workgroup owns a 32 x 8 column of the xy plane over a chunk
// of z planes and marches through it in z (32 x 8 rather than 64 x 4: the
// halo-2 planes of R_{kp-1} and kappa are 36 x 12 = 1.69 tile areas instead of
// 68 x 8 = 2.13, and a plane takes two region loads per thread instead of
// three).  LDS holds rolling windows
// of planes: R_{kp-1} (3 planes) and kappa (4 planes) over the tile plus an xy
// halo of two, and R_kp (3 planes) over the tile plus an xy halo of one.  For
// each plane z the workgroup loads plane z+1 of R_{kp-1} and kappa, forms R_kp
// on the halo-1 region of plane z from U_{kp-1} = A~ R_{kp-1} recomputed
// there, and then applies the stencil to R_kp on the tile of plane z-1 (U_kp),
// writes R_kp there and accumulates the inner products.  Each thread owns one
// xy position of the tile and at most one of the halo-1 ring.  Neighbouring
// chunks recompute two halo planes each.
#pragma once

#include "buffer.h"
#include "pass_common.h"

namespace kiops {

// kNarrow: the one-solve instantiation for IOP windows of one or two vectors
// (q = 1, 2), whose formation reads no vector older than R_{kp-2} and whose
// inner products take R_{kp-1} alone (from LDS); a separate kernel, since the
// branches that load older vectors, present in the same code, cost the common
// window 4% at 256^3 (measured).
template <typename T, int PB, bool kNarrow>
struct Stencil3DT {
  static constexpr int TX = 32, TY = 8;
  static_assert(TX * TY == kThreads && (TX & (TX - 1)) == 0, "one tile position per thread");
  static constexpr int RX = TX + 4, RY = TY + 4, RP = RX * RY;   // halo-2 plane (R_{kp-1}, kappa)
  static constexpr int SX = TX + 2, SY = TY + 2, SP = SX * SY;   // halo-1 plane (R_kp)
  static constexpr int kRingPos = SP - TX * TY;                   // halo-1 positions outside the tile
  static constexpr int kRegionLoads = (RP + kThreads - 1) / kThreads;
  static constexpr int kLdsT = 3 * RP + 4 * RP + 3 * SP;         // elements of T
  static constexpr int kLdsDoubles = (int)((kLdsT * sizeof(T) + 7) / 8);
  static constexpr bool kTwoPhase = false;   // one fused pass per Krylov step
  static constexpr int kWavesPerEU = sizeof(T) == 4 ? 3 : 3;
  static constexpr int kDepth = 3;   // FP32: plane steps whose loads are in flight at a time
  static constexpr int kSlabRows = 4;   // tile rows of a slab in the item order

  struct PlaneLoads {
    T vr[kRegionLoads], vk[kRegionLoads];   // halo-2 plane of R_{kp-1} and kappa
    uint32_t goff[2];
    T rv[2], ov[2], bv[2][PB > 0 ? PB : 1];  // r, older vector (or w), B at the two positions
  };

  int64_t N;
  int nx, ny, nz;
  int tiles_x, tiles_y, nchunks, nitems;   // z chunk c covers [nz c / nchunks, nz (c+1) / nchunks)
  T h2inv;            // 1 / h^2
  T half_h2inv;       // 1 / (2 h^2): face diffusivity (kappa_P + kappa_nb) / 2 folded in
  T cx, cy, cz;       // a_d / (2 h)
  T diff;             // face diffusivity when kappa is absent
  const T* kappa;     // per-cell diffusivity or null
  const T* r;         // per-cell reaction or null
  const T* B[kPM];    // B[c] = b_{p-c} (Theorem 1 column order)
  int p;
  const double* r_src;   // mixed precision: float copies made at setup
  T* r_dst;
  const double* k_src;
  T* k_dst;
  T* ubuf;               // full window: U_kp output

  __device__ void setup_coefficients(const KParams& P, int64_t gt, int64_t gs) const {
    if (r_dst && r_src)
      for (int64_t n = gt; n < P.N; n += gs) r_dst[n] = (T)r_src[n];
    if (k_dst && k_src)
      for (int64_t n = gt; n < P.N; n += gs) k_dst[n] = (T)k_src[n];
  }

  __device__ static void ring_pos(int e, int& rx, int& ry) {
    // e in [0, kRingPos): rows y = -1 and y = TY, then columns x = -1 and x = TX
    if (e < SX) { rx = e - 1; ry = -1; return; }
    e -= SX;
    if (e < SX) { rx = e - 1; ry = TY; return; }
    e -= SX;
    if (e < TY) { rx = -1; ry = e; return; }
    e -= TY;
    rx = TX; ry = e;
  }

  // z mod n for z in [-2n, 3n), without a branch (wave-uniform planes)
  __device__ static int wrap_plane(int z, int n) {
    z = z < 0 ? z + n : z;
    z = z < 0 ? z + n : z;
    z = z >= n ? z - n : z;
    z = z >= n ? z - n : z;
    return z;
  }

  // stencil of field u at the centre c, diffusivities at the centre and the six
  // neighbours, face diffusivity written as (kc + kn) * half_h2inv
  __device__ T apply(T c, T xp, T xm, T yp, T ym, T zp, T zm, T kc, T kxp, T kxm, T kyp, T kym,
                     T kzp, T kzm, T rc) const {
    T U = rc * c;
    U = fma((kc + kxp) * half_h2inv, xp - c, U);
    U = fma(-(kc + kxm) * half_h2inv, c - xm, U);
    U = fma((kc + kyp) * half_h2inv, yp - c, U);
    U = fma(-(kc + kym) * half_h2inv, c - ym, U);
    U = fma((kc + kzp) * half_h2inv, zp - c, U);
    U = fma(-(kc + kzm) * half_h2inv, c - zm, U);
    U = fma(-cx, xp - xm, U);
    U = fma(-cy, yp - ym, U);
    U = fma(-cz, zp - zm, U);
    return U;
  }

  __device__ void pass(const PassCtx<T>& c, const BasisPtrs<T>& bp, const double* w, T* Rout,
                       DotAcc& acc, T* lds) const {
    T* sR = lds;                 // 3 planes of RP
    T* sK = lds + 3 * RP;        // 4 planes of RP
    T* sX = lds + 7 * RP;        // 3 planes of SP
    const int t = threadIdx.x;
    const int tcx = t & (TX - 1);
    const int tcy = t / TX;
    const bool first = c.first != 0;
    const bool has_kappa = kappa != nullptr;
    const uint64_t nb = (uint64_t)N * sizeof(T);
    const bool has_old = !first && c.flo < c.src;
    const bool more_old = !first && c.flo < c.src - 1;
    const __amdgpu_buffer_rsrc_t rsR = make_rsrc(first ? nullptr : bp.get(c.src), nb);
    const __amdgpu_buffer_rsrc_t rsO = make_rsrc(has_old ? bp.get(c.src - 1) : nullptr, nb);
    const __amdgpu_buffer_rsrc_t rsW = make_rsrc(first ? w : nullptr, (uint64_t)N * 8);
    // FP64: the formation's second vector is w in the first pass, else R_{kp-2}
    const __amdgpu_buffer_rsrc_t rsOW =
        make_rsrc(first ? (const void*)w : (has_old ? (const void*)bp.get(c.src - 1) : nullptr), nb);
    const __amdgpu_buffer_rsrc_t rsr = make_rsrc(r, nb);
    const __amdgpu_buffer_rsrc_t rsK = make_rsrc(kappa, nb);
    const __amdgpu_buffer_rsrc_t rsOut = make_rsrc(c.write_out ? Rout : nullptr, nb);
    const bool store_u = uniform(c.store_u) != 0;   // full window only: no store otherwise
    const __amdgpu_buffer_rsrc_t rsU = make_rsrc(store_u ? ubuf : nullptr, nb);
    __amdgpu_buffer_rsrc_t rsB[PB > 0 ? PB : 1];
#pragma unroll
    for (int k = 0; k < PB; ++k) rsB[k] = make_rsrc(k < c.p ? B[k] : nullptr, nb);
    // the thread's halo-1 positions: 0 = its tile position, 1 = its ring position
    int prx[2], pry[2];
    prx[0] = tcx;
    pry[0] = tcy;
    const bool ring = t < kRingPos;
    ring_pos(ring ? t : 0, prx[1], pry[1]);
    const int plane = nx * ny;

    // XCD-aware order (as in the 2-D stencil): one contiguous band of the item
    // sequence per XCD, swept together by the band's workgroups
    const int nband = vgrid() < kXcds ? vgrid() : kXcds;
    const int band = vblock() % nband;
    const int nloc = (vgrid() - band + nband - 1) / nband;
    const int i_lo = (int)((int64_t)nitems * band / nband);
    const int i_hi = (int)((int64_t)nitems * (band + 1) / nband);
    // Items are dealt in rounds, one per workgroup of the band in position
    // order.  With R workgroups per CU the band's positions form R groups by
    // dispatch order (position p is on the CU's (p R / nloc)-th workgroup);
    // the first-dispatched workgroups are favoured by the SIMD arbitration and
    // finish their items sooner (measured at 256^3, three per CU: 330, 380 and
    // 427 us per pass), so the first group takes one item more and the last
    // one less.  cnt(p) is non-increasing in p, so the workgroups of round j
    // are the positions [0, size(j)) and position p takes item start(j) + p.
    const int pos = vblock() / nband;
    const int nbi = i_hi - i_lo;
    const int base = nbi / nloc;
    const int left = nbi - base * nloc;
    const int R = (c.ranks >= 2 && nloc % c.ranks == 0 && base >= 2) ? c.ranks : 1;
    const int gsz = nloc / R;
    auto cnt = [&](int q) {
      int v = base + (q < left ? 1 : 0);
      if (R >= 2) {
        const int g = q / gsz;
        v += (g == 0 ? 1 : 0) - (g == R - 1 ? 1 : 0);
      }
      return v;
    };
    auto round_size = [&](int j) {
      int lo = 0, hi = nloc;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cnt(mid) > j) lo = mid + 1;
        else hi = mid;
      }
      return lo;
    };
    const int mine = cnt(pos);
    int start = 0;
    for (int j = 0; j < mine; start += round_size(j), ++j) {
      const int item = i_lo + start + pos;
      // items run through slabs of kSlabRows tile rows: x fastest, then the
      // slab's rows, then z chunks (the last slab may have fewer rows)
      const int per_slab = tiles_x * kSlabRows * nchunks;
      const int nfull = tiles_y / kSlabRows;
      const int slab = item / per_slab < nfull ? item / per_slab : nfull;
      const int hs = slab < nfull ? kSlabRows : tiles_y - nfull * kSlabRows;
      const int rr = item - slab * per_slab;
      const int tx = rr % tiles_x;
      const int r2 = rr / tiles_x;
      const int x0 = tx * TX;
      const int y0 = (slab * kSlabRows + r2 % hs) * TY;
      const int zch = r2 / hs;
      const int z0 = (int)((int64_t)nz * zch / nchunks);
      const int z1 = (int)((int64_t)nz * (zch + 1) / nchunks);
      // FP64: chunks alternate their march direction (even chunks upwards in
      // z, odd ones downwards), so two neighbouring chunks reach their shared
      // boundary planes at the same time (both at the start of their march
      // or both at the end); measured at 256^3: FP64 7.22 -> 7.45 solves/s,
      // mixed 7.47 -> 7.41 (so the mixed form marches upwards only).
      // Plane steps run over the relative index l in [-1, nzc]; relative
      // plane l is z0 + l upwards and z1 - 1 - l downwards.
      const int sdir = (sizeof(T) == 8 && (zch & 1)) ? -1 : 1;
      const int nzc = z1 - z0;
      auto phys = [&](int l) { return sdir > 0 ? z0 + l : z1 - 1 - l; };

      // halo-2 region offsets of this thread (plane-independent part)
      uint32_t roff[kRegionLoads];
      bool rin[kRegionLoads];
#pragma unroll
      for (int i = 0; i < kRegionLoads; ++i) {
        const int e = t + i * kThreads;
        const int ry2 = e / RX, rx2 = e - ry2 * RX;
        rin[i] = e < RP;
        roff[i] = (uint32_t)(wrap_index(y0 - 2 + ry2, ny) * nx + wrap_index(x0 - 2 + rx2, nx));
      }
      uint32_t poff[2];
      bool pin[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        pin[q] = (q == 0) || ring;
        poff[q] = (uint32_t)(wrap_index(y0 + pry[q], ny) * nx + wrap_index(x0 + prx[q], nx));
      }
      auto region_load = [&](int zz, T* vr, T* vk) __attribute__((always_inline)) {
        const uint32_t zo = (uint32_t)(wrap_plane(zz, nz) * plane);
#pragma unroll
        for (int i = 0; i < kRegionLoads; ++i) {
          const uint32_t o = rin[i] ? (zo + roff[i]) * (uint32_t)sizeof(T) : kNoOffset;
          vr[i] = buf_ld(rsR, o, T(0));
          vk[i] = buf_ld(rsK, o, T(0));
        }
      };
      auto region_store = [&](int slot_r, int slot_k, const T* vr, const T* vk) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < kRegionLoads; ++i) {
          const int e = t + i * kThreads;
          if (e < RP) {
            if (!first) sR[slot_r * RP + e] = vr[i];
            sK[slot_k * RP + e] = has_kappa ? vk[i] : diff;
          }
        }
      };
      // prologue: relative planes -2 and -1 of R_{kp-1} and kappa (ring slots 0 and 1)
      {
        T vr0[kRegionLoads], vk0[kRegionLoads], vr1[kRegionLoads], vk1[kRegionLoads];
        region_load(phys(-2), vr0, vk0);
        region_load(phys(-1), vr1, vk1);
        region_store(0, 0, vr0, vk0);
        region_store(1, 1, vr1, vk1);
      }
      T rv_prev = T(0), bc_prev = T(0);
      // every global load of plane step l: relative plane l+1 of R_{kp-1} and
      // kappa, and r, the older window vector and B at the thread's positions
      // of relative plane l
      auto issue = [&](int l, PlaneLoads& L) __attribute__((always_inline)) {
        region_load(phys(l + 1), L.vr, L.vk);
        const uint32_t zo = (uint32_t)(wrap_plane(phys(l), nz) * plane);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          L.goff[q] = pin[q] ? (zo + poff[q]) * (uint32_t)sizeof(T) : kNoOffset;
          L.rv[q] = buf_ld(rsr, L.goff[q], T(0));
          if constexpr (sizeof(T) == 8) {
            L.ov[q] = buf_ld(rsOW, L.goff[q], T(0));   // w (first pass) or R_{kp-2}: one load, no branch
          } else {
            // mixed: w is FP64, R_{kp-2} FP32; both loads are issued (one of
            // the two resources is empty) so that no branch separates them
            const double w0 = buf_ld(rsW, pin[q] ? (zo + poff[q]) * 8u : kNoOffset, 0.0);
            const T o0 = buf_ld(rsO, L.goff[q], T(0));
            L.ov[q] = first ? (T)w0 : o0;
          }
#pragma unroll
          for (int k = 0; k < PB; ++k) L.bv[q][k] = buf_ld(rsB[k], L.goff[q], T(0));
        }
      };
      // relative planes: "ahead" is l + 1, "behind" l - 1; upwards ahead is
      // +z, downwards -z, which the stencil's z terms take into account
      const bool up = sdir > 0;
      auto process = [&](int l, const PlaneLoads& L) __attribute__((always_inline)) {
        const int lz = l + 2;                     // >= 1
        const int sr_m = (lz - 1) % 3, sr_c = lz % 3, sr_p = (lz + 1) % 3;
        const int sk_m2 = (lz + 2) % 4, sk_m = (lz + 3) % 4, sk_c = lz % 4, sk_p = (lz + 1) % 4;
        const int sx_c = (lz - 1) % 3, sx_m = (lz + 1) % 3, sx_m2 = lz % 3;   // X planes l, l-1, l-2
        region_store(sr_p, sk_p, L.vr, L.vk);
        __syncthreads();
        // ---- R_kp on the halo-1 region of relative plane l
        T bc_cur = T(0);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          if (pin[q]) {
            T bprev = T(0), bc = T(0);
#pragma unroll
            for (int k = 0; k < PB; ++k) {
              bprev = fma(L.bv[q][k], c.ybp[k], bprev);
              bc = fma(L.bv[q][k], c.ybc[k], bc);
            }
            if (q == 0) bc_cur = bc;
            T X;
            if (first) {
              X = L.ov[q];
            } else {
              const int o = (pry[q] + 2) * RX + (prx[q] + 2);
              const T* Rc = sR + sr_c * RP;
              const T* Kc = sK + sk_c * RP;
              const T ctr = Rc[o];
              const T ra = sR[sr_p * RP + o], rb = sR[sr_m * RP + o];
              const T ka = sK[sk_p * RP + o], kb = sK[sk_m * RP + o];
              T U = apply(ctr, Rc[o + 1], Rc[o - 1], Rc[o + RX], Rc[o - RX], up ? ra : rb, up ? rb : ra,
                          Kc[o], Kc[o + 1], Kc[o - 1], Kc[o + RX], Kc[o - RX], up ? ka : kb, up ? kb : ka,
                          L.rv[q]);
              U += bprev;
              X = c.a * U;
              X = fma(c.bw[c.src], ctr, X);
              if (has_old) X = fma(c.bw[c.src - 1], L.ov[q], X);
              if (!kNarrow && more_old) {
                // older window vectors (a full window streams every earlier
                // vector: eight loads in flight at a time)
                int i = c.flo;
                for (; i + 8 <= c.src - 1; i += 8) {
                  T v[8];
#pragma unroll
                  for (int u = 0; u < 8; ++u) v[u] = buf_ld(make_rsrc(bp.get(i + u), nb), L.goff[q], T(0));
#pragma unroll
                  for (int u = 0; u < 8; ++u) X = fma(c.bw[i + u], v[u], X);
                }
                for (; i < c.src - 1; ++i) X = fma(c.bw[i], buf_ld(make_rsrc(bp.get(i), nb), L.goff[q], T(0)), X);
              }
            }
            sX[sx_c * SP + (pry[q] + 1) * SX + (prx[q] + 1)] = X;
          }
        }
        __syncthreads();
        // ---- U_kp on the tile of relative plane l-1, output and inner products
        if (l - 1 >= 0) {
          const int o1 = (tcy + 1) * SX + (tcx + 1);
          const int o2 = (tcy + 2) * RX + (tcx + 2);
          const T* Xc = sX + sx_m * SP;
          const T* Kc = sK + sk_m * RP;
          const T X = Xc[o1];
          const T xa = sX[sx_c * SP + o1], xb = sX[sx_m2 * SP + o1];
          const T ka = sK[sk_c * RP + o2], kb = sK[sk_m2 * RP + o2];
          T U = apply(X, Xc[o1 + 1], Xc[o1 - 1], Xc[o1 + SX], Xc[o1 - SX], up ? xa : xb, up ? xb : xa,
                      Kc[o2], Kc[o2 + 1], Kc[o2 - 1], Kc[o2 + RX], Kc[o2 - RX], up ? ka : kb, up ? kb : ka,
                      rv_prev);
          U += bc_prev;
          const bool valid = (x0 + tcx < nx) && (y0 + tcy < ny);
          const uint32_t zo1 = (uint32_t)(wrap_plane(phys(l - 1), nz) * plane);
          const uint32_t off1 = (zo1 + poff[0]) * (uint32_t)sizeof(T);
          buf_st(rsOut, valid ? off1 : kNoOffset, X);
          if (store_u) buf_st(rsU, valid ? off1 : kNoOffset, U);
          const double Xd = valid ? (double)X : 0.0, Ud = valid ? (double)U : 0.0;
          acc.RR = fma(Xd, Xd, acc.RR);
          acc.UU = fma(Ud, Ud, acc.UU);
          acc.Ck = fma(Xd, Ud, acc.Ck);
          // inner products with the window [dlo, kp-1]: R_{kp-1} is in LDS,
          // older vectors (windows of three or more) are loaded here
          const double Rs = (double)sR[sr_m * RP + o2];
          if constexpr (kNarrow) {
            if (c.ngd > 0) {
              acc.G[0] = fma(Rs, Xd, acc.G[0]);
              acc.C[0] = fma(Rs, Ud, acc.C[0]);
            }
          } else {
#pragma unroll
            for (int d = 0; d < kWinMax - 1; ++d) {
              if (d < c.ngd) {
                const int idx = c.dlo + d;
                const double Rv = (idx == c.src) ? Rs : (double)buf_ld(make_rsrc(bp.get(idx), nb), off1, T(0));
                acc.G[d] = fma(Rv, Xd, acc.G[d]);
                acc.C[d] = fma(Rv, Ud, acc.C[d]);
              }
            }
          }
        }
        __syncthreads();
        rv_prev = L.rv[0];
        bc_prev = bc_cur;
      };
      // plane steps l = -1 .. nzc
      if constexpr (sizeof(T) == 4) {
        // three register sets rotate so that the loads of the next two plane
        // steps are in flight while the current one is processed; the issues
        // are unconditional (past the chunk they repeat its last plane,
        // served by the caches), so that no branch separates a load from the
        // wait that counts it and each wait leaves the later steps' loads in
        // flight
        PlaneLoads Ls[kDepth];
#pragma unroll
        for (int u = 0; u < kDepth - 1; ++u) issue(u - 1 < nzc ? u - 1 : nzc, Ls[u]);
        for (int lb = -1; lb <= nzc; lb += kDepth) {
#pragma unroll
          for (int u = 0; u < kDepth; ++u) {
            const int la = lb + u + kDepth - 1;
            issue(la < nzc ? la : nzc, Ls[(u + kDepth - 1) % kDepth]);
            if (lb + u <= nzc) process(lb + u, Ls[u]);
          }
        }
      } else {
        // two register sets alternate so that the loads of the next plane
        // step are in flight while the current one is processed (the FP64
        // sets leave no room for a third at three waves per SIMD; the
        // unconditional issue of the FP32 loop measured no faster here)
        PlaneLoads la, lb;
        issue(-1, la);
        for (int l = -1; l <= nzc; l += 2) {
          if (l + 1 <= nzc) issue(l + 1, lb);
          process(l, la);
          if (l + 1 > nzc) break;
          if (l + 2 <= nzc) issue(l + 2, la);
          process(l + 1, lb);
        }
      }
    }
  }
};

template <typename T, int PB>
using Stencil3D = Stencil3DT<T, PB, false>;
template <typename T, int PB>
using Stencil3DNarrow = Stencil3DT<T, PB, true>;

}  // namespace kiops
