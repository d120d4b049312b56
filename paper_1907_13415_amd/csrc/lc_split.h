// lc_split.h -- the step as two sweeps with LDS halo tiles.
//
//   split_lb : stress (Eq. 6) on the tile plus a one-site ring, kept in LDS;
//              body force, moments (Eq. 9), BGK collision with forcing and
//              push streaming for the tile; stores the force-corrected u.
//   split_q  : rate R(Q) and predictor Q^P on the tile plus ring (LDS),
//              then the corrector R(Q^P) and Q(n+1) for the tile
//              (Sec. 1.2.2, steps 1-5).
//
// A block owns a TX x TY column of sites and marches along z through a
// chunk of planes.  In-plane neighbours come from LDS planes staged with a
// two-site halo; z neighbours of computed quantities stay in registers of
// the owning thread (a three-plane window), so nothing is recomputed along
// z.  Every index is taken modulo the grid (periodic), so any grid size,
// including sizes smaller than the tile, is handled.  On two-dimensional
// lattices the block treats its single plane without the z pipeline.
// Both sweeps also take the isotropic stencils of lc_staged.h (template
// argument ST): the diagonal neighbours of Q and u are in the LDS regions,
// the rings of stress and predictor values gain the four corner sites, and
// in 3D the whole stress and the predictor are kept in three-plane LDS
// rings for the neighbours in the planes above and below.
#pragma once

#include "lc_staged.h"

namespace lc {

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2):
// hardware block b runs on XCD b % 8.  Remapping b to the logical tile
// (b % 8) * (nb / 8) + b / 8 gives every XCD one contiguous range of tiles,
// so neighbouring tiles (which share halo lines) meet in the same L2.
constexpr int NUM_XCD = 8;
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  if (nb % NUM_XCD != 0) return b;
  return (b % NUM_XCD) * (nb / NUM_XCD) + b / NUM_XCD;
}

__device__ __forceinline__ int wrapi(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}

template <int TX, int TY>
struct Tile {
  static constexpr int NT = TX * TY;
  static constexpr int W2 = TX + 4, H2 = TY + 4, R2 = W2 * H2;  // two-site halo
  static constexpr int W1 = TX + 2, H1 = TY + 2, R1 = W1 * H1;  // one-site halo
  static constexpr int RING = 2 * TX + 2 * TY;                  // one-site ring, no corners
  static_assert(RING <= NT, "tile too thin for its ring");
  // R1 coordinates of ring point k: top row, bottom row, left, right column.
  __device__ static __forceinline__ void ring(int k, int& i, int& j) {
    if (k < TX) {
      i = k + 1;
      j = 0;
    } else if (k < 2 * TX) {
      i = k - TX + 1;
      j = TY + 1;
    } else if (k < 2 * TX + TY) {
      i = 0;
      j = k - 2 * TX + 1;
    } else {
      i = TX + 1;
      j = k - 2 * TX - TY + 1;
    }
  }
  // R2 index of the R1 point (i, j).
  __device__ static __forceinline__ int r2(int i, int j) { return (i + 1) + W2 * (j + 1); }
};

// Stencil of a symmetric tensor from LDS planes: centre plane `m` indexed
// by the R2 index k, z neighbours in planes zp/zm at the same index.  With
// HALF unset the first differences are left undivided (twice d_g).
template <typename S, int DIM, int W2, int R2, bool HALF = true>
__device__ __forceinline__ void stencil_lds(const S (*m)[R2], const S (*zp)[R2], const S (*zm)[R2], int k,
                                            Sym<S>& c, Sym<S> (&d)[3], Sym<S>& L) {
  S v[5], lap[5], dx[5], dy[5], dz[5];
#pragma unroll
  for (int q = 0; q < 5; q++) {
    const S cc = m[q][k];
    const S xp = m[q][k + 1], xm = m[q][k - 1], yp = m[q][k + W2], ym = m[q][k - W2];
    v[q] = cc;
    dx[q] = HALF ? (xp - xm) * S(0.5) : xp - xm;
    dy[q] = HALF ? (yp - ym) * S(0.5) : yp - ym;
    S l = (xp + xm) + (yp + ym);
    if constexpr (DIM == 3) {
      const S zpv = zp[q][k], zmv = zm[q][k];
      dz[q] = HALF ? (zpv - zmv) * S(0.5) : zpv - zmv;
      l += zpv + zmv;
      lap[q] = l - S(6) * cc;
    } else {
      dz[q] = S(0);
      lap[q] = l - S(4) * cc;
    }
  }
  c = Sym<S>{v[0], v[1], v[2], v[3], v[4]};
  d[0] = Sym<S>{dx[0], dx[1], dx[2], dx[3], dx[4]};
  d[1] = Sym<S>{dy[0], dy[1], dy[2], dy[3], dy[4]};
  d[2] = Sym<S>{dz[0], dz[1], dz[2], dz[3], dz[4]};
  L = Sym<S>{lap[0], lap[1], lap[2], lap[3], lap[4]};
}

// Isotropic stencil (D2Q9) of a symmetric tensor from an LDS plane with row
// stride W: the centre value, the gradients (times two with HALF unset)
// and the Laplacian, each from the pairs of opposite velocities.  Per pair
// and component one difference and one sum: the gradient components take
// +-w_g (v+ - v-), the Laplacian 6 w_i (v+ + v-), and the centre's share,
// 6 sum_{i != 0} w_i v(x) = 6 (1 - w_0) v(x), is taken off once at the end.
template <typename S, int W, int RN, bool HALF = true>
__device__ __forceinline__ void stencil_lds_iso2(const S (*m)[RN], int k, Sym<S>& c, Sym<S> (&d)[3], Sym<S>& L) {
  using Lt = Lattice<0>;
  S v[5], lap[5], dx[5], dy[5];
#pragma unroll
  for (int q = 0; q < 5; q++) {
    const S cc = m[q][k];
    S gx = S(0), gy = S(0), l = S(0);
#pragma unroll
    for (int i = 1; i < Lt::q; i++) {
      if (Lt::opp(i) < i) continue;
      const int o = Lt::cx(i) + W * Lt::cy(i);
      const S vp = m[q][k + o], vm = m[q][k - o];
      const S wg = S((HALF ? 3.0 : 6.0) * Lt::w(i)), wl = S(6.0 * Lt::w(i));
      const S dif = vp - vm, sum = vp + vm;
      if (Lt::cx(i) != 0) gx += (Lt::cx(i) > 0 ? wg : -wg) * dif;
      if (Lt::cy(i) != 0) gy += (Lt::cy(i) > 0 ? wg : -wg) * dif;
      l += wl * sum;
    }
    v[q] = cc;
    dx[q] = gx;
    dy[q] = gy;
    lap[q] = l - S(6.0 * (1.0 - Lt::w(0))) * cc;
  }
  c = Sym<S>{v[0], v[1], v[2], v[3], v[4]};
  d[0] = Sym<S>{dx[0], dx[1], dx[2], dx[3], dx[4]};
  d[1] = Sym<S>{dy[0], dy[1], dy[2], dy[3], dy[4]};
  d[2] = sym_zero<S>();
  L = Sym<S>{lap[0], lap[1], lap[2], lap[3], lap[4]};
}

// Isotropic stencil (D3Q19) of a symmetric tensor from three LDS planes
// (centre m, above zp, below zm) with row stride W; the sums as in
// stencil_lds_iso2.
template <typename S, int W, int RN, bool HALF = true>
__device__ __forceinline__ void stencil_lds_iso3(const S (*m)[RN], const S (*zp)[RN], const S (*zm)[RN], int k,
                                                 Sym<S>& c, Sym<S> (&d)[3], Sym<S>& L) {
  using Lt = Lattice<1>;
  S v[5], lap[5], g[3][5];
#pragma unroll
  for (int q = 0; q < 5; q++) {
    const S cc = m[q][k];
    S gx = S(0), gy = S(0), gz = S(0), l = S(0);
#pragma unroll
    for (int i = 1; i < Lt::q; i++) {
      if (Lt::opp(i) < i) continue;
      const int o = Lt::cx(i) + W * Lt::cy(i);
      const S(*pp)[RN] = Lt::cz(i) > 0 ? zp : (Lt::cz(i) < 0 ? zm : m);
      const S(*pm)[RN] = Lt::cz(i) > 0 ? zm : (Lt::cz(i) < 0 ? zp : m);
      const S vp = pp[q][k + o], vm = pm[q][k - o];
      const S wg = S((HALF ? 3.0 : 6.0) * Lt::w(i)), wl = S(6.0 * Lt::w(i));
      const S dif = vp - vm, sum = vp + vm;
      if (Lt::cx(i) != 0) gx += (Lt::cx(i) > 0 ? wg : -wg) * dif;
      if (Lt::cy(i) != 0) gy += (Lt::cy(i) > 0 ? wg : -wg) * dif;
      if (Lt::cz(i) != 0) gz += (Lt::cz(i) > 0 ? wg : -wg) * dif;
      l += wl * sum;
    }
    v[q] = cc;
    g[0][q] = gx;
    g[1][q] = gy;
    g[2][q] = gz;
    lap[q] = l - S(6.0 * (1.0 - Lt::w(0))) * cc;
  }
  c = Sym<S>{v[0], v[1], v[2], v[3], v[4]};
#pragma unroll
  for (int a = 0; a < 3; a++) d[a] = Sym<S>{g[a][0], g[a][1], g[a][2], g[a][3], g[a][4]};
  L = Sym<S>{lap[0], lap[1], lap[2], lap[3], lap[4]};
}

// R1 coordinates of ring point k of a TX x TY tile: the one-site ring of
// Tile::ring for k < RING, then its four corners.
template <int TX, int TY>
__device__ __forceinline__ void ring_point(int k, int& i, int& j) {
  if (k < Tile<TX, TY>::RING) {
    Tile<TX, TY>::ring(k, i, j);
  } else {
    const int cn = k - Tile<TX, TY>::RING;
    i = (cn & 1) ? TX + 1 : 0;
    j = (cn & 2) ? TY + 1 : 0;
  }
}

// The NC component arrays of an LDS region: the first NA of type A, the
// rest of type B, read as A (the velocity of the mixed-precision form is
// stored in single precision next to a double-precision Q).
template <typename A, typename B, int NC, int NA>
struct RegionSrc {
  const A* a[NA];
  const B* b[NC > NA ? NC - NA : 1];
  __device__ __forceinline__ A operator()(int q, uint32_t s) const { return q < NA ? a[q][s] : A(b[q - NA][s]); }
};

// Load plane gz of NC component arrays (component stride N) into an LDS
// plane over the R2 region of the block, with periodic wrap.
// dst points at an LDS plane laid out [NC][R2].
template <typename S, int TX, int TY, int NC, typename SRC>
__device__ __forceinline__ void load_region(S* dst, const SRC& src, int x0, int y0, int gz, const GridDims& g,
                                            int tid) {
  constexpr int W2 = TX + 4, R2 = (TX + 4) * (TY + 4), NT = TX * TY;
  const uint32_t plane = uint32_t(g.nx) * uint32_t(g.ny) * uint32_t(gz);
  for (int k = tid; k < R2; k += NT) {
    const int i = k % W2, j = k / W2;
    const int gx = wrapi(x0 - 2 + i, g.nx), gy = wrapi(y0 - 2 + j, g.ny);
    const uint32_t s = plane + uint32_t(gx) + uint32_t(g.nx) * uint32_t(gy);
#pragma unroll
    for (int q = 0; q < NC; q++) dst[q * R2 + k] = src(q, s);
  }
}

// Register-staged form of load_region for software pipelining: fetch_region
// issues the global loads of a plane into registers (one iteration ahead),
// store_region later writes them to an LDS plane.
template <typename S, int TX, int TY, int NC>
struct RegionRegs {
  static constexpr int R2 = (TX + 4) * (TY + 4), NT = TX * TY;
  static constexpr int P = (R2 + NT - 1) / NT;  // points per thread
  S v[P][NC];
};

template <typename S, int TX, int TY, int NC, typename SRC>
__device__ __forceinline__ void fetch_region(RegionRegs<S, TX, TY, NC>& r, const SRC& src, int x0, int y0, int gz,
                                             const GridDims& g, int tid) {
  using RR = RegionRegs<S, TX, TY, NC>;
  constexpr int W2 = TX + 4;
  const uint32_t plane = uint32_t(g.nx) * uint32_t(g.ny) * uint32_t(gz);
#pragma unroll
  for (int p = 0; p < RR::P; p++) {
    const int k = tid + p * RR::NT;
    if (p < RR::P - 1 || k < RR::R2) {
      const int i = k % W2, j = k / W2;
      const int gx = wrapi(x0 - 2 + i, g.nx), gy = wrapi(y0 - 2 + j, g.ny);
      const uint32_t s = plane + uint32_t(gx) + uint32_t(g.nx) * uint32_t(gy);
#pragma unroll
      for (int q = 0; q < NC; q++) r.v[p][q] = src(q, s);
    }
  }
}

template <typename S, int TX, int TY, int NC>
__device__ __forceinline__ void store_region(const RegionRegs<S, TX, TY, NC>& r, S* dst, int tid) {
  using RR = RegionRegs<S, TX, TY, NC>;
#pragma unroll
  for (int p = 0; p < RR::P; p++) {
    const int k = tid + p * RR::NT;
    if (p < RR::P - 1 || k < RR::R2) {
#pragma unroll
      for (int q = 0; q < NC; q++) dst[q * RR::R2 + k] = r.v[p][q];
    }
  }
}

// Store of Q(n+1) = Q + (R(Q) + R(Q^P))/2 (Sec. 1.2.2, step 5) at site s;
// with SR the float sums are rounded stochastically, one uniform number per
// site (from the site index and the step's key) serving its five
// components (each rounding stays unbiased).
template <typename S, bool SR>
__device__ __forceinline__ void store_q_update(S* __restrict__ Qout, int64_t N, int64_t s, const Sym<S>& q,
                                               const Sym<S>& r, const Sym<S>& rp, uint32_t srkey) {
  if constexpr (SR) {
    const float u = site_uniform(uint32_t(s), srkey);
    __builtin_nontemporal_store(add_stochastic(q.xx, S(0.5) * (r.xx + rp.xx), u), &Qout[s]);
    __builtin_nontemporal_store(add_stochastic(q.xy, S(0.5) * (r.xy + rp.xy), u), &Qout[N + s]);
    __builtin_nontemporal_store(add_stochastic(q.xz, S(0.5) * (r.xz + rp.xz), u), &Qout[2 * N + s]);
    __builtin_nontemporal_store(add_stochastic(q.yy, S(0.5) * (r.yy + rp.yy), u), &Qout[3 * N + s]);
    __builtin_nontemporal_store(add_stochastic(q.yz, S(0.5) * (r.yz + rp.yz), u), &Qout[4 * N + s]);
  } else {
    __builtin_nontemporal_store(q.xx + S(0.5) * (r.xx + rp.xx), &Qout[s]);
    __builtin_nontemporal_store(q.xy + S(0.5) * (r.xy + rp.xy), &Qout[N + s]);
    __builtin_nontemporal_store(q.xz + S(0.5) * (r.xz + rp.xz), &Qout[2 * N + s]);
    __builtin_nontemporal_store(q.yy + S(0.5) * (r.yy + rp.yy), &Qout[3 * N + s]);
    __builtin_nontemporal_store(q.yz + S(0.5) * (r.yz + rp.yz), &Qout[4 * N + s]);
  }
}

// ---------------------------------------------------------------------------
// Sweep 1: stress in LDS, body force, moments, collision, streaming.
// Store of a sweep's output (f or Q of the next step), which no block reads
// again during the sweep: the nontemporal hint keeps it from displacing
// lines that are still to be reused (halo rows, the populations pulled from
// neighbouring tiles).  Measured: 3-5% on the stress/LB sweep, 256^3 and
// the 64-grid batch alike.
template <typename S>
__device__ __forceinline__ void store_out(S* p, S v) {
  __builtin_nontemporal_store(v, p);
}

// STREAM_F: read the populations with nontemporal loads (each is pulled by
// one site only; measured to help where many grids share the caches, and to
// hurt a single small grid that stays resident in them).  QT: the type of Q
// and of the molecular field, stress and body force (S, or double in the
// mixed-precision form, whose populations and collision stay in S), and of
// the velocity handed to sweep 2; cq holds the constants in that type.
template <int LAT, typename S, bool DEV, int TX, int TY, bool MRT = false, bool STREAM_F = false, typename QT = S,
          int ST = STENCIL_COMPACT>
__device__ __forceinline__ void split_lb_body(const QT* __restrict__ Qin, const S* __restrict__ fin,
                                              S* __restrict__ fout, QT* __restrict__ uout, const GridDims& g,
                                              const Coef<S>& c, const Coef<QT>& cq, int zc, int bx, int by, int bz,
                                              S* __restrict__ rec = nullptr) {
  using L = Lattice<LAT>;
  using T = Tile<TX, TY>;
  constexpr int DIM = L::dim;
  constexpr int NQP = DIM == 3 ? 3 : 1;  // Q planes held
  constexpr int NTP = DIM == 3 ? 2 : 1;  // stress planes held
  // tau_{a x} is needed at x +- 1 (rows 1..TY of the R1 region, all
  // columns) and tau_{a y} at y +- 1 (columns 1..TX, all rows)
  constexpr int NXA = T::W1 * TY, NYA = TX * T::H1;
  // isotropic stencils: the body force needs the stress at every lattice
  // neighbour, so the whole stress of the tile, its ring and the ring's
  // corners goes to LDS (sTi[plane slot][a][b][R1 index]; in 3D a ring of
  // the three planes p-1, p, p+1)
  constexpr bool ISO = ST == STENCIL_ISO;
  static_assert(!ISO || T::RING + 4 <= T::NT, "tile too thin for its ring and corners");
  constexpr int NI = ISO ? DIM : 1, RI = ISO ? T::R1 : 1, NPI = (ISO && DIM == 3) ? 3 : 1;
  __shared__ QT sQ[NQP][5][T::R2];
  __shared__ QT sTx[NTP][DIM][ISO ? 1 : NXA];
  __shared__ QT sTy[NTP][DIM][ISO ? 1 : NYA];
  __shared__ QT sTi[NPI][NI][NI][RI];

  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + TX * ty;
  const int x0 = bx * TX, y0 = by * TY;
  const int x = x0 + tx, y = y0 + ty;
  const bool own = x < g.nx && y < g.ny;
  const int64_t N = g.N;
  const RegionSrc<QT, QT, 5, 5> qsrc{{Qin, Qin + N, Qin + 2 * N, Qin + 3 * N, Qin + 4 * N}, {nullptr}};

  // stress at the R1 point (i, j) of plane slot m with z neighbours zp/zm
  auto tau_point = [&](int m, int zp, int zm, int i, int j, QT (&t)[3][3]) {
    Sym<QT> q, Lq, d[3];
    if constexpr (ISO && DIM == 2)
      stencil_lds_iso2<QT, T::W2, T::R2>(sQ[m], T::r2(i, j), q, d, Lq);
    else if constexpr (ISO)
      stencil_lds_iso3<QT, T::W2, T::R2>(sQ[m], sQ[zp], sQ[zm], T::r2(i, j), q, d, Lq);
    else
      stencil_lds<QT, DIM, T::W2, T::R2>(sQ[m], sQ[zp], sQ[zm], T::r2(i, j), q, d, Lq);
    const Sym<QT> H = molecular_field(q, Lq, cq);
    stress(q, H, d, cq, t);
  };
  // column b of the stress at the R1 point (i, j)
  auto tau_col = [&](int m, int zp, int zm, int i, int j, int b, QT (&col)[3]) {
    Sym<QT> q, Lq, d[3];
    stencil_lds<QT, DIM, T::W2, T::R2>(sQ[m], sQ[zp], sQ[zm], T::r2(i, j), q, d, Lq);
    const Sym<QT> H = molecular_field(q, Lq, cq);
    stress_col(q, H, d, cq, b, col);
  };
  // Ring sites in the rows above and below the tile need only tau_{a y},
  // those in the columns beside it only tau_{a x}.  With rows of 32 or 64
  // sites the two kinds fall in different waves and each wave computes just
  // its column; otherwise every ring site computes the whole stress.  All
  // entries round alike either way.
  constexpr bool COLS = TX % 32 == 0 && (TX * TY) % 64 == 0 && (2 * TX) % 64 == 0;
  // stress of the whole region of plane slot m into sT[ts]; returns the
  // owner's tau_{a z}
  auto tau_plane = [&](int m, int zp, int zm, int ts, QT (&tz)[3]) {
    if constexpr (ISO) {  // every site of the R1 region, corners included, into plane slot m
      auto put = [&](int i, int j) {
        QT t[3][3];
        tau_point(m, zp, zm, i, j, t);
        const int k = i + T::W1 * j;
#pragma unroll
        for (int a = 0; a < DIM; a++)
#pragma unroll
          for (int b = 0; b < DIM; b++) sTi[NPI == 3 ? m : 0][a][b][k] = t[a][b];
      };
      put(tx + 1, ty + 1);
      if (tid < T::RING + 4) {
        int i, j;
        ring_point<TX, TY>(tid, i, j);
        put(i, j);
      }
#pragma unroll
      for (int a = 0; a < 3; a++) tz[a] = QT(0);
    } else {
      {  // the owner's site
        QT t[3][3];
        tau_point(m, zp, zm, tx + 1, ty + 1, t);
        const int kx = (tx + 1) + T::W1 * ty, ky = tx + TX * (ty + 1);
#pragma unroll
        for (int a = 0; a < DIM; a++) {
          sTx[ts][a][kx] = t[a][0];
          sTy[ts][a][ky] = t[a][1];
        }
#pragma unroll
        for (int a = 0; a < 3; a++) tz[a] = t[a][2];
      }
      if (tid < T::RING) {  // a ring site
        int i, j;
        T::ring(tid, i, j);
        const bool row_ring = j == 0 || j == TY + 1;
        if constexpr (COLS) {
          QT col[3];
          tau_col(m, zp, zm, i, j, row_ring ? 1 : 0, col);
          if (row_ring) {
            const int ky = (i - 1) + TX * j;
#pragma unroll
            for (int a = 0; a < DIM; a++) sTy[ts][a][ky] = col[a];
          } else {
            const int kx = i + T::W1 * (j - 1);
#pragma unroll
            for (int a = 0; a < DIM; a++) sTx[ts][a][kx] = col[a];
          }
        } else {
          QT t[3][3];
          tau_point(m, zp, zm, i, j, t);
          if (row_ring) {
            const int ky = (i - 1) + TX * j;
#pragma unroll
            for (int a = 0; a < DIM; a++) sTy[ts][a][ky] = t[a][1];
          } else {
            const int kx = i + T::W1 * (j - 1);
#pragma unroll
            for (int a = 0; a < DIM; a++) sTx[ts][a][kx] = t[a][0];
          }
        }
      }
  }
  };

  // periodic neighbour offsets of the owner's site in plane z (unsigned
  // arithmetic modulo 2^32 on in-range indices)
  struct Off {
    uint32_t s, xp, xm, yp, ym, zp, zm;
  };
  auto offsets = [&](int z) {
    Off o;
    const uint32_t sy = uint32_t(g.nx), sz = uint32_t(g.nx) * uint32_t(g.ny);
    o.s = uint32_t(x) + sy * uint32_t(y) + sz * uint32_t(z);
    o.xp = (x + 1 == g.nx) ? 0u - uint32_t(g.nx - 1) : 1u;
    o.xm = (x == 0) ? uint32_t(g.nx - 1) : 0u - 1u;
    o.yp = (y + 1 == g.ny) ? 0u - uint32_t(g.ny - 1) * sy : sy;
    o.ym = (y == 0) ? uint32_t(g.ny - 1) * sy : 0u - sy;
    o.zp = (z + 1 == g.nz) ? 0u - uint32_t(g.nz - 1) * sz : sz;
    o.zm = (z == 0) ? uint32_t(g.nz - 1) * sz : 0u - sz;
    return o;
  };
  // gather the owner's populations of plane z: f_i(x) = buf_i(x - c_i)
  // (issued one plane ahead and consumed by lb_site)
  auto fetch_f = [&](int z, S (&f)[L::q]) {
    if (!own) return;
    const Off o = offsets(z);
#pragma unroll
    for (int i = 0; i < L::q; i++) {
      uint32_t d = o.s;
      if (L::cx(i) == 1) d += o.xm;
      if (L::cx(i) == -1) d += o.xp;
      if (L::cy(i) == 1) d += o.ym;
      if (L::cy(i) == -1) d += o.yp;
      if (L::cz(i) == 1) d += o.zm;
      if (L::cz(i) == -1) d += o.zp;
      const S* a = &(fin + size_t(i) * size_t(N))[d];
      if constexpr (STREAM_F)
        f[i] = __builtin_nontemporal_load(a);
      else
        f[i] = *a;
    }
  };
  // lattice-Boltzmann update of the owner's site in plane z; writes the
  // post-collision populations at the site (pull form)
  auto lb_site = [&](int z, int ts, const QT (&tzp)[3], const QT (&tzm)[3], S (&f)[L::q]) {
    if (!own) return;
    const int kx = (tx + 1) + T::W1 * ty, ky = tx + TX * (ty + 1);
    S F[3] = {S(0), S(0), S(0)};
    if constexpr (ISO) {  // F_a = 3 sum_i w_i sum_b c_ib tau_ab(x + c_i), over pairs
      using Lt = Lattice<LAT>;
      const int k1 = (tx + 1) + T::W1 * (ty + 1);
      // plane slots of z, z+1 and z-1 (3D): the stress of planes z-1..z+1
      const int sc = NPI == 3 ? (z + 3) % 3 : 0, sp = NPI == 3 ? (z + 4) % 3 : 0, sm = NPI == 3 ? (z + 2) % 3 : 0;
#pragma unroll
      for (int a = 0; a < DIM; a++) {
        QT acc = QT(0);
#pragma unroll
        for (int i = 1; i < Lt::q; i++) {
          if (Lt::opp(i) < i) continue;
          const int o = Lt::cx(i) + T::W1 * Lt::cy(i);
          const int pp = Lt::cz(i) > 0 ? sp : (Lt::cz(i) < 0 ? sm : sc);
          const int pm = Lt::cz(i) > 0 ? sm : (Lt::cz(i) < 0 ? sp : sc);
          QT dsum = QT(0);
#pragma unroll
          for (int b = 0; b < DIM; b++) {
            const int cb = b == 0 ? Lt::cx(i) : (b == 1 ? Lt::cy(i) : Lt::cz(i));
            if (cb == 0) continue;
            const QT dt = sTi[pp][a][b][k1 + o] - sTi[pm][a][b][k1 - o];
            dsum += cb > 0 ? dt : -dt;
          }
          acc += QT(3.0 * Lt::w(i)) * dsum;
        }
        F[a] = S(acc);
      }
    } else {
#pragma unroll
      for (int a = 0; a < DIM; a++) {
        QT acc = (sTx[ts][a][kx + 1] - sTx[ts][a][kx - 1]) + (sTy[ts][a][ky + TX] - sTy[ts][a][ky - TX]);
        if constexpr (DIM == 3) acc += tzp[a] - tzm[a];
        F[a] = S(QT(0.5) * acc);
      }
    }
    const uint32_t s = uint32_t(x) + uint32_t(g.nx) * (uint32_t(y) + uint32_t(g.ny) * uint32_t(z));
    S rho, mass, u[3];
    moments<LAT, S, DEV>(f, F, rho, u, mass);
#pragma unroll
    for (int a = 0; a < DIM; a++) (uout + size_t(a) * size_t(N))[s] = QT(u[a]);
    if (rec) {  // record rho and F of this step (reverse-mode replay)
      rec[s] = rho;
#pragma unroll
      for (int a = 0; a < DIM; a++) (rec + size_t(a + 1) * size_t(N))[s] = F[a];
    }
    if constexpr (MRT)
      collide_mrt<LAT, S, DEV>(f, rho, mass, u, F, c);
    else
      collide_pairs<LAT, S, DEV>(f, rho, mass, u, F, c);
#pragma unroll
    for (int i = 0; i < L::q; i++) store_out(&(fout + size_t(i) * size_t(N))[s], f[i]);
  };

  if constexpr (DIM == 2) {
    load_region<QT, TX, TY, 5>(&sQ[0][0][0], qsrc, x0, y0, 0, g, tid);
    __syncthreads();
    QT tz[3];
    S f[L::q];
    fetch_f(0, f);
    tau_plane(0, 0, 0, 0, tz);
    __syncthreads();
    lb_site(0, 0, tz, tz, f);
  } else {
    const int zb = bz * zc;
    const int ze = min(zb + zc, g.nz);
    auto slot = [](int p) { return (p + 3) % 3; };  // p >= -3
    // software pipeline: the halo region of plane p+2 and the populations of
    // plane p are in flight while plane p's stress and plane p-1's update run
    RegionRegs<QT, TX, TY, 5> rq;
    load_region<QT, TX, TY, 5>(&sQ[slot(zb - 2)][0][0], qsrc, x0, y0, wrapi(zb - 2, g.nz), g, tid);
    load_region<QT, TX, TY, 5>(&sQ[slot(zb - 1)][0][0], qsrc, x0, y0, wrapi(zb - 1, g.nz), g, tid);
    fetch_region<QT, TX, TY, 5>(rq, qsrc, x0, y0, wrapi(zb, g.nz), g, tid);
    QT tzA[3] = {QT(0), QT(0), QT(0)}, tzB[3] = {QT(0), QT(0), QT(0)}, tzC[3];
    S f[L::q];
    for (int p = zb - 1; p <= ze; p++) {
      store_region<QT, TX, TY, 5>(rq, &sQ[slot(p + 1)][0][0], tid);
      if (p + 2 <= ze + 1) fetch_region<QT, TX, TY, 5>(rq, qsrc, x0, y0, wrapi(p + 2, g.nz), g, tid);
      __syncthreads();
      tau_plane(slot(p), slot(p + 1), slot(p - 1), p & 1, tzC);
      __syncthreads();
      if (p - 1 >= zb) lb_site(p - 1, (p - 1) & 1, tzC, tzA, f);
      if (p >= zb && p < ze) fetch_f(p, f);
#pragma unroll
      for (int a = 0; a < 3; a++) {
        tzA[a] = tzB[a];
        tzB[a] = tzC[a];
      }
    }
  }
}

template <int LAT, typename S, bool DEV, int TX, int TY, int WPE, bool MRT = false, typename QT = S,
          int ST = STENCIL_COMPACT>
__global__ void __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(WPE)))
    split_lb(const QT* __restrict__ Qin, const S* __restrict__ fin, S* __restrict__ fout, QT* __restrict__ uout,
             GridDims g, Coef<S> c, Coef<QT> cq, int zc, S* __restrict__ rec) {
  const int nb = gridDim.x * gridDim.y * gridDim.z;
  const int t = xcd_remap(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), nb);
  split_lb_body<LAT, S, DEV, TX, TY, MRT, false, QT, ST>(Qin, fin, fout, uout, g, c, cq, zc, t % gridDim.x,
                                                     (t / gridDim.x) % gridDim.y, t / (gridDim.x * gridDim.y), rec);
}

// ---------------------------------------------------------------------------
// Sweep 2: predictor on tile + ring (LDS), corrector on the tile.  S is the
// type of Q, of the velocity and of the arithmetic.
// SR: the float form with stochastic rounding (molecular field summed in
// double, Q(n+1) rounded stochastically with the per-step key srkey).
template <int LAT, typename S, int TX, int TY, bool SR = false, int ST = STENCIL_COMPACT>
__device__ __forceinline__ void split_q_body(const S* __restrict__ Qin, const S* __restrict__ uin,
                                             S* __restrict__ Qout, const GridDims& g, const Coef<S>& c, int zc,
                                             int bx, int by, int bz, S* __restrict__ rec = nullptr,
                                             uint32_t srkey = 0) {
  using L = Lattice<LAT>;
  using T = Tile<TX, TY>;
  constexpr int DIM = L::dim;
  // Three LDS planes of Q and u (z-1, z, z+1 of the predictor).  Q^P on
  // the tile and its ring: in single precision one LDS plane for the
  // corrector's in-plane neighbours, its centre and z neighbours being the
  // owner's own predictor values kept in registers; in double precision
  // (one wave per SIMD, where registers are the scarcer resource) three LDS
  // planes, z-1, z and z+1 of the corrector.
  // isotropic stencils: the predictor also runs at the ring's corners, and
  // in 3D the corrector reads the predictor's diagonal neighbours in the
  // planes above and below, so three LDS planes of it are kept
  constexpr bool ISO = ST == STENCIL_ISO;
  constexpr bool ZREG = DIM == 3 && sizeof(S) == 4 && !ISO;
  constexpr int NP = DIM == 3 ? 3 : 1;
  constexpr int NPS = (DIM == 3 && !ZREG) ? 3 : 1;
  constexpr int NC = 5 + DIM;  // Q components then u components
  constexpr int NRING = ISO ? T::RING + 4 : T::RING;
  static_assert(NRING <= T::NT, "tile too thin for its ring");
  __shared__ S sQ[NP][NC][T::R2];
  __shared__ S sP[NPS][5][T::R1];

  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + TX * ty;
  const int x0 = bx * TX, y0 = by * TY;
  const int x = x0 + tx, y = y0 + ty;
  const bool own = x < g.nx && y < g.ny;
  const int64_t N = g.N;
  RegionSrc<S, S, NC, 5> csrc;
#pragma unroll
  for (int q = 0; q < 5; q++) csrc.a[q] = Qin + q * N;
#pragma unroll
  for (int a = 0; a < DIM; a++) csrc.b[a] = uin + a * N;

  // What the owner keeps from its predictor for its corrector: Q, R(Q) and
  // the flow terms (from u/2 and the undivided velocity differences; RAW
  // form).  Q^P = Q + R(Q) is formed from them again where needed (the same
  // expression, so the same rounding as the value shared through LDS).
  struct Stash {
    Sym<S> r;
    Flow<S> fl;
    Sym<S> q;
  };
  auto qp_of = [](const Stash& st) {
    return Sym<S>{st.q.xx + st.r.xx, st.q.xy + st.r.xy, st.q.xz + st.r.xz, st.q.yy + st.r.yy, st.q.yz + st.r.yz};
  };

  // rate and predictor at R1 point (i, j) of plane slot m; returns Q^P
  auto pred_point = [&](int m, int zp, int zm, int i, int j, Stash& st) {
    const int k = T::r2(i, j);
    Sym<S> q, Lq, d[3];
    if constexpr (ISO && DIM == 2)
      stencil_lds_iso2<S, T::W2, T::R2, false>(sQ[m], k, q, d, Lq);
    else if constexpr (ISO)
      stencil_lds_iso3<S, T::W2, T::R2, false>(sQ[m], sQ[zp], sQ[zm], k, q, d, Lq);
    else
      stencil_lds<S, DIM, T::W2, T::R2, false>(sQ[m], sQ[zp], sQ[zm], k, q, d, Lq);
    const Sym<S> H = SR ? molecular_field_exact(q, Lq, c) : molecular_field(q, Lq, c);
    S u[3], G[3][3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
      u[a] = a < DIM ? sQ[m][5 + a][k] * S(0.5) : S(0);
      if constexpr (ISO) {  // undivided: 6 sum_i w_i c_ib u_a(x + c_i), over pairs
        using Lt = Lattice<LAT>;
        S g0 = S(0), g1 = S(0), g2 = S(0);
        if (a < DIM) {
#pragma unroll
          for (int n = 1; n < Lt::q; n++) {
            if (Lt::opp(n) < n) continue;
            const int o = Lt::cx(n) + T::W2 * Lt::cy(n);
            const int pp = Lt::cz(n) > 0 ? zp : (Lt::cz(n) < 0 ? zm : m);
            const int pm = Lt::cz(n) > 0 ? zm : (Lt::cz(n) < 0 ? zp : m);
            const S dif = sQ[pp][5 + a][k + o] - sQ[pm][5 + a][k - o];
            const S w6 = S(6.0 * Lt::w(n));
            if (Lt::cx(n) != 0) g0 += (Lt::cx(n) > 0 ? w6 : -w6) * dif;
            if (Lt::cy(n) != 0) g1 += (Lt::cy(n) > 0 ? w6 : -w6) * dif;
            if (Lt::cz(n) != 0) g2 += (Lt::cz(n) > 0 ? w6 : -w6) * dif;
          }
        }
        G[a][0] = g0;
        G[a][1] = g1;
        G[a][2] = g2;
        continue;
      }
      G[a][0] = a < DIM ? sQ[m][5 + a][k + 1] - sQ[m][5 + a][k - 1] : S(0);
      G[a][1] = a < DIM ? sQ[m][5 + a][k + T::W2] - sQ[m][5 + a][k - T::W2] : S(0);
      if constexpr (DIM == 3)
        G[a][2] = sQ[zp][5 + a][k] - sQ[zm][5 + a][k];
      else
        G[a][2] = S(0);
    }
    st.fl = flow_terms<S, true>(u, G, c);
    st.r = be_rate_flow<S, true>(q, H, d, st.fl, c);
    st.q = q;
    return qp_of(st);
  };
  auto store_pred = [&](int b, int i, int j, const Sym<S>& qp) {
    const int k1 = i + T::W1 * j;
    sP[b][0][k1] = qp.xx;
    sP[b][1][k1] = qp.xy;
    sP[b][2][k1] = qp.xz;
    sP[b][3][k1] = qp.yy;
    sP[b][4][k1] = qp.yz;
  };
  const int k1 = (tx + 1) + T::W1 * (ty + 1);
  auto pred_at = [&](int b) { return Sym<S>{sP[b][0][k1], sP[b][1][k1], sP[b][2][k1], sP[b][3][k1], sP[b][4][k1]}; };
  // corrector at the owner's site of plane z: in-plane neighbours of Q^P
  // from sP[b], the centre pc and the z neighbours pzp / pzm (3D)
  // (bzp, bzm: the predictor planes above and below, read by the isotropic
  // stencil in 3D)
  auto corr_site = [&](int z, int b, const Stash& st, const Sym<S>& pc, const Sym<S>& pzp, const Sym<S>& pzm,
                       int bzp = 0, int bzm = 0) {
    if (!own) return;
    if constexpr (ISO) {
      Sym<S> pcc, Lp, d[3];
      if constexpr (DIM == 2)
        stencil_lds_iso2<S, T::W1, T::R1, false>(sP[b], k1, pcc, d, Lp);
      else
        stencil_lds_iso3<S, T::W1, T::R1, false>(sP[b], sP[bzp], sP[bzm], k1, pcc, d, Lp);
      const Sym<S> H = SR ? molecular_field_exact(pcc, Lp, c) : molecular_field(pcc, Lp, c);
      const Sym<S> Rp = be_rate_flow<S, true>(pcc, H, d, st.fl, c);
      const int64_t s = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
      if (rec) store_sym(rec, N, s, pcc);
      store_q_update<S, SR>(Qout, N, s, st.q, st.r, Rp, srkey);
      return;
    }
    const S vc[5] = {pc.xx, pc.xy, pc.xz, pc.yy, pc.yz};
    const S vzp[5] = {pzp.xx, pzp.xy, pzp.xz, pzp.yy, pzp.yz};
    const S vzm[5] = {pzm.xx, pzm.xy, pzm.xz, pzm.yy, pzm.yz};
    S lap[5], dx[5], dy[5], dz[5];
#pragma unroll
    for (int q = 0; q < 5; q++) {
      const S cc = vc[q];
      const S xp = sP[b][q][k1 + 1], xm = sP[b][q][k1 - 1];
      const S yp = sP[b][q][k1 + T::W1], ym = sP[b][q][k1 - T::W1];
      dx[q] = xp - xm;
      dy[q] = yp - ym;
      S l = (xp + xm) + (yp + ym);
      if constexpr (DIM == 3) {
        dz[q] = vzp[q] - vzm[q];
        l += vzp[q] + vzm[q];
        lap[q] = l - S(6) * cc;
      } else {
        dz[q] = S(0);
        lap[q] = l - S(4) * cc;
      }
    }
    const Sym<S> d[3] = {Sym<S>{dx[0], dx[1], dx[2], dx[3], dx[4]}, Sym<S>{dy[0], dy[1], dy[2], dy[3], dy[4]},
                         Sym<S>{dz[0], dz[1], dz[2], dz[3], dz[4]}};
    const Sym<S> Lp{lap[0], lap[1], lap[2], lap[3], lap[4]};
    const Sym<S> H = SR ? molecular_field_exact(pc, Lp, c) : molecular_field(pc, Lp, c);
    const Sym<S> Rp = be_rate_flow<S, true>(pc, H, d, st.fl, c);
    const int64_t s = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
    if (rec) store_sym(rec, N, s, pc);  // record the predictor (reverse-mode replay)
    store_q_update<S, SR>(Qout, N, s, st.q, st.r, Rp, srkey);
  };

  if constexpr (DIM == 2) {
    load_region<S, TX, TY, NC>(&sQ[0][0][0], csrc, x0, y0, 0, g, tid);
    __syncthreads();
    Stash st;
    const Sym<S> pc = pred_point(0, 0, 0, tx + 1, ty + 1, st);
    store_pred(0, tx + 1, ty + 1, pc);
    if (tid < NRING) {
      int i, j;
      ring_point<TX, TY>(tid, i, j);
      Stash tmp;
      store_pred(0, i, j, pred_point(0, 0, 0, i, j, tmp));
    }
    __syncthreads();
    corr_site(0, 0, st, pc, pc, pc);
  } else {
    const int zb = bz * zc;
    const int ze = min(zb + zc, g.nz);
    auto slot = [](int p) { return (p + 3) % 3; };  // p >= -3
    RegionRegs<S, TX, TY, NC> rq;
    load_region<S, TX, TY, NC>(&sQ[slot(zb - 2)][0][0], csrc, x0, y0, wrapi(zb - 2, g.nz), g, tid);
    load_region<S, TX, TY, NC>(&sQ[slot(zb - 1)][0][0], csrc, x0, y0, wrapi(zb - 1, g.nz), g, tid);
    fetch_region<S, TX, TY, NC>(rq, csrc, x0, y0, wrapi(zb, g.nz), g, tid);
    auto pslot = [](int p) { return (p + 3) % 3; };  // p >= -3
    Sym<S> pm = sym_zero<S>();  // Q^P of plane p-2 at the owner's site (ZREG)
    // one plane of the pipeline: predictor of plane p, corrector of p-1;
    // `prev` holds the stash of plane p-1, `cur` receives that of plane p
    auto iteration = [&](int p, const Stash& prev, Stash& cur) {
      // slot(p+1) = slot(p-2) was last read by the predictor of iteration
      // p-1, before that iteration's second barrier
      store_region<S, TX, TY, NC>(rq, &sQ[slot(p + 1)][0][0], tid);
      if (p + 2 <= ze + 1) fetch_region<S, TX, TY, NC>(rq, csrc, x0, y0, wrapi(p + 2, g.nz), g, tid);
      // plane p+1 of Q and u, and the Q^P written in iteration p-1, are
      // visible after this barrier
      __syncthreads();
      // without ZREG, sP[pslot(p)] was last read by the corrector of
      // iteration p-1, and the predictor values go there at once
      const Sym<S> own_p = pred_point(slot(p), slot(p + 1), slot(p - 1), tx + 1, ty + 1, cur);
      if constexpr (!ZREG) store_pred(pslot(p), tx + 1, ty + 1, own_p);
      const bool ring = tid < NRING;
      int ri = 0, rj = 0;
      Sym<S> ring_p = sym_zero<S>();
      if (ring) {
        ring_point<TX, TY>(tid, ri, rj);
        Stash tmp;
        ring_p = pred_point(slot(p), slot(p + 1), slot(p - 1), ri, rj, tmp);
        if constexpr (!ZREG) store_pred(pslot(p), ri, rj, ring_p);
      }
      if constexpr (ZREG) {
        const Sym<S> pc = qp_of(prev);  // Q^P of plane p-1
        if (p - 1 >= zb) corr_site(p - 1, 0, prev, pc, own_p, pm);
        // every corrector has read plane p-1 of Q^P, every predictor plane
        // p-1 of Q and u: both may be overwritten
        __syncthreads();
        store_pred(0, tx + 1, ty + 1, own_p);
        if (ring) store_pred(0, ri, rj, ring_p);
        pm = pc;
      } else {
        // Q^P of plane p visible; every predictor has read plane p-1 of Q
        // and u, which may be overwritten
        __syncthreads();
        if (p - 1 >= zb)
          corr_site(p - 1, pslot(p - 1), prev, pred_at(pslot(p - 1)), pred_at(pslot(p)), pred_at(pslot(p - 2)),
                    pslot(p), pslot(p - 2));
      }
    };
    // two planes per trip, so the two stashes swap roles without copies
    Stash stA{}, stB{};
    int p = zb - 1;
    for (; p + 1 <= ze; p += 2) {
      iteration(p, stA, stB);
      iteration(p + 1, stB, stA);
    }
    if (p <= ze) iteration(p, stA, stB);
  }
}

template <int LAT, typename S, int TX, int TY, int WPE, bool SR = false, int ST = STENCIL_COMPACT>
__global__ void __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(WPE)))
    split_q(const S* __restrict__ Qin, const S* __restrict__ uin, S* __restrict__ Qout, GridDims g, Coef<S> c,
            int zc, S* __restrict__ rec, uint32_t srkey) {
  const int nb = gridDim.x * gridDim.y * gridDim.z;
  const int t = xcd_remap(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), nb);
  split_q_body<LAT, S, TX, TY, SR, ST>(Qin, uin, Qout, g, c, zc, t % gridDim.x, (t / gridDim.x) % gridDim.y,
                                   t / (gridDim.x * gridDim.y), rec, srkey);
}

// Tile shapes of the two-sweep kernels (measured on 256^3; LDS per block at
// most 77 KB, so at least two blocks fit a CU).  S: the type of Q, which
// sets the LDS footprint of the tiles; SF: that of the populations (float
// in the mixed-precision form).
template <int LAT, typename S, typename SF = S>
struct SplitCfg {
  static constexpr bool d3 = Lattice<LAT>::dim == 3;
  static constexpr bool f64 = sizeof(S) == 8;
  static constexpr int LB_TX = (d3 && !f64) ? 64 : 32, LB_TY = 8;
  static constexpr int Q_TX = (d3 && f64) ? 16 : 32, Q_TY = 8;
  // planes per block along z in each sweep (16; 32 in the mixed form, which
  // measured 2% faster with it, where FP32 measured 0.8% faster with 16)
  static constexpr int ZC_LB = (sizeof(S) == 8 && sizeof(SF) == 4) ? 32 : 16, ZC_Q = 128;
  // waves per SIMD the register allocation is held to (the single-precision
  // 3D stress sweep runs two blocks of eight waves per CU)
  static constexpr int LB_WPE = (d3 && !f64) ? 4 : 1;
  static constexpr int Q_WPE = 1;
};

}  // namespace lc
