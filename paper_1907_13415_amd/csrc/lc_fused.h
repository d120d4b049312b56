// lc_fused.h -- the step as one pass over the grid: every block reads the
// populations and Q of its sites once (plus halos, mostly from cache) and
// writes the populations and Q of the next step once; nothing goes through
// HBM in between.
//
// One step maps (f, Q)(n) to (f, Q)(n+1) (Sec. 1.2; Sec. 1.2.2 steps 1-5;
// Eq. 7).  The new Q at a site depends on Q^P at distance 1, which depends
// on u and Q at distance 2; u depends on the body force there, which
// depends on the stress at distance 3, which depends on Q at distance 4.  A
// block owns a TX x TY column of sites and marches along z.  In the plane
// directions each stage is computed on a rectangle that shrinks by one site
// per stage (stress on radius 3, moments on radius 2, predictor on radius
// 1, corrector on the tile), so the block needs no data of its neighbours'
// stages; along z the stages run on different planes of the march (the
// stress one plane behind the newest Q plane, the moments two, the
// predictor three, the corrector four), and each keeps the planes its
// successor needs in LDS rings.  Blocks march through chunks of planes and
// recompute the stages of the few planes around a chunk's ends.
//
// Per iteration p (Q plane p newest), in this order, separated by barriers:
//   (a) load Q(p) on the radius-4 rectangle;
//   (b) stress of plane p-1 on the radius-3 rectangle (corners excepted);
//   (c) body force, moments and velocity of plane p-2 on the radius-2
//       rectangle; at the tile's own sites also the collision and the
//       store of the post-collision populations (pull form);
//   (d) predictor of plane p-3 on the radius-1 rectangle;
//   (e) corrector of plane p-4 at the tile's sites, store of Q(n+1).
// Region loops visit the tile's own sites first, in thread order, so the
// thread that computes a site's predictor also computes its corrector from
// values it keeps in registers, and the tile's collisions store whole rows.
#pragma once

#include "lc_split.h"

namespace lc {

// Rectangle of radius r around a TX x TY tile.
template <int TX, int TY, int r>
struct Rect {
  static constexpr int W = TX + 2 * r, H = TY + 2 * r, N = W * H;
};

// Rectangle coordinates (i, j) of entry k when the tile's own sites come
// first (row-major, k < TX*TY), then the rows above and below the tile,
// then the columns left and right of it.
template <int TX, int TY, int r>
__device__ __forceinline__ void tile_first(int k, int& i, int& j) {
  constexpr int NT = TX * TY, W = TX + 2 * r, BAND = W * r;
  if (k < NT) {
    i = r + k % TX;
    j = r + k / TX;
    return;
  }
  int m = k - NT;
  if (m < BAND) {
    i = m % W;
    j = m / W;
    return;
  }
  m -= BAND;
  if (m < BAND) {
    i = m % W;
    j = r + TY + m / W;
    return;
  }
  m -= BAND;
  const int row = m / (2 * r), c = m % (2 * r);
  j = r + row;
  i = c < r ? c : TX + c;
}

// Tile shapes of the single pass (LDS per block: FP32 D3Q19 about 132 KB,
// FP64 D3Q19 about 152 KB, so one block per CU in 3D) and threads per block
// (more threads than tile sites share the ring work and hide latency).
// On two-dimensional grids the runtime picks one of the FUSED2D_* shapes
// from the number of tiles.
template <int LAT, typename QT>
struct FusedCfg {
  static constexpr bool d3 = Lattice<LAT>::dim == 3;
  static constexpr bool f64 = sizeof(QT) == 8;
  static constexpr int TX = (d3 && f64) ? 16 : 32, TY = 8;
  static constexpr int NTHR = d3 ? (f64 ? 256 : 512) : TX * TY;
  static constexpr int ZC = 64;  // planes per block along z
};

// Two-dimensional shapes (TX, TY, threads).  A grid of at most one tile per
// CU is latency bound (one wave per SIMD with one thread per site): there a
// block of 1024 threads shares each stage's ring points among four threads
// per tile site, which shortens every wave's instruction stream and puts
// four waves on each SIMD; 16x8 tiles where the grid has few enough of
// them, else 32x8.  Up to four tiles per CU, two threads per site; larger
// grids keep one thread per site.  Measured on 65536 sites (256^2): 8.3 ->
// 6.1 us per step in FP32, 9.2 -> 7.3 us in FP64; on 16384 sites (128^2)
// 16x8 tiles 5.3 us (FP32) against 5.7 for 32x8 at 1024 threads; on 384^2
// two threads per site 9.5 against 10.8 us (FP32), 14.6 against 18.2 us
// (FP64).
constexpr int FUSED2D_SMALL_TX = 16, FUSED2D_SMALL_TY = 8, FUSED2D_SMALL_NTHR = 1024;
constexpr int FUSED2D_MID_TX = 32, FUSED2D_MID_TY = 8, FUSED2D_MID_NTHR = 1024;
constexpr int FUSED2D_HALF_TX = 32, FUSED2D_HALF_TY = 8, FUSED2D_HALF_NTHR = 512;
constexpr int FUSED2D_WIDE_TX = 32, FUSED2D_WIDE_TY = 8, FUSED2D_WIDE_NTHR = 256;
constexpr int FUSED2D_CUS = 256;  // compute units of the chip

// ST: the difference stencils (lc_staged.h); the isotropic ones on
// two-dimensional grids only, with the arithmetic of the two sweeps (the
// whole stress of the radius-3 rectangle, corners included, in LDS for the
// body force; the stencils of Q, u and Q^P from the pairs of opposite
// velocities).
template <int LAT, typename S, bool DEV, int TX, int TY, int NTHR, bool MRT, typename QT, bool SR,
          int ST = STENCIL_COMPACT>
__device__ __forceinline__ void fused_body(const QT* __restrict__ Qin, const S* __restrict__ fin,
                                           S* __restrict__ fout, QT* __restrict__ Qout, const GridDims& g,
                                           const Coef<S>& c, const Coef<QT>& cq, int zc, int bx, int by, int bz,
                                           uint32_t srkey) {
  using L = Lattice<LAT>;
  constexpr int DIM = L::dim;
  constexpr int NT = TX * TY;
  using R4 = Rect<TX, TY, 4>;
  using R3 = Rect<TX, TY, 3>;
  using R2 = Rect<TX, TY, 2>;
  using R1 = Rect<TX, TY, 1>;
  // stress columns kept: tau_{a x} at x-range of radius 3 and y-range of
  // radius 2 (for d_x at the radius-2 sites), tau_{a y} the other way round
  constexpr int WX = R3::W, NXA = R3::W * R2::H;
  constexpr int WY = R2::W, NYA = R2::W * R3::H;
  constexpr int NQS = DIM == 3 ? 5 : 1;  // Q planes p-4 .. p
  constexpr int NTS = DIM == 3 ? 2 : 1;  // in-plane stress planes
  constexpr int NZS = DIM == 3 ? 3 : 1;  // tau_{a z} planes
  constexpr int NUS = DIM == 3 ? 3 : 1;  // velocity planes
  constexpr int NPS = DIM == 3 ? 2 : 1;  // predictor planes
  constexpr bool ISO = ST == STENCIL_ISO;
  static_assert(!ISO || DIM == 2, "isotropic stencils in the single pass: two-dimensional grids");
  __shared__ QT sQ[NQS][5][R4::N];
  __shared__ QT sTx[NTS][DIM][ISO ? 1 : NXA];
  __shared__ QT sTy[NTS][DIM][ISO ? 1 : NYA];
  __shared__ QT sTi[ISO ? 2 : 1][ISO ? 2 : 1][ISO ? R3::N : 1];  // isotropic: tau_ab on the radius-3 rectangle
  __shared__ QT sTz[NZS][DIM == 3 ? 3 : 1][DIM == 3 ? R2::N : 1];
  __shared__ QT sU[NUS][DIM][R2::N];
  __shared__ QT sP[NPS][5][R1::N];

  static_assert(NTHR >= NT, "one thread per tile site at least");
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = (tid / TX) % TY;
  const int x0 = bx * TX, y0 = by * TY;
  const int64_t N = g.N;
  // threads tid < NT own the tile's sites; the others take ring sites only
  const bool own = tid < NT && x0 + tx < g.nx && y0 + ty < g.ny;

  // In-plane site indices (periodic) of the thread's points of the
  // radius-4 rectangle (Q loads) and of the radius-2 rectangle with their
  // neighbour offsets (population pulls); the same in every plane.
  constexpr int P4 = (R4::N + NTHR - 1) / NTHR, P2 = (R2::N + NTHR - 1) / NTHR;
  const uint32_t sy = uint32_t(g.nx), sz = uint32_t(g.nx) * uint32_t(g.ny);
  uint32_t q_off[P4];
#pragma unroll
  for (int n = 0; n < P4; n++) {
    const int k = tid + n * NTHR;
    const int i = k % R4::W, j = k / R4::W;
    q_off[n] = k < R4::N ? uint32_t(wrapi(x0 - 4 + i, g.nx)) + sy * uint32_t(wrapi(y0 - 4 + j, g.ny)) : 0u;
  }
  struct InPlane {
    uint32_t s, xp, xm, yp, ym;
  };
  InPlane ip[P2];
#pragma unroll
  for (int n = 0; n < P2; n++) {
    const int k = tid + n * NTHR;
    int i2 = 0, j2 = 0;
    if (k < R2::N) tile_first<TX, TY, 2>(k, i2, j2);
    const int gx = wrapi(x0 - 2 + i2, g.nx), gy = wrapi(y0 - 2 + j2, g.ny);
    ip[n].s = uint32_t(gx) + sy * uint32_t(gy);
    ip[n].xp = (gx + 1 == g.nx) ? 0u - uint32_t(g.nx - 1) : 1u;
    ip[n].xm = (gx == 0) ? uint32_t(g.nx - 1) : 0u - 1u;
    ip[n].yp = (gy + 1 == g.ny) ? 0u - uint32_t(g.ny - 1) * sy : sy;
    ip[n].ym = (gy == 0) ? uint32_t(g.ny - 1) * sy : 0u - sy;
  }

  // Register staging of the next plane's global loads (float forms in 3D,
  // where registers allow): the Q rectangle of plane p+1 and the populations
  // of the next moment plane are in flight while the stages of plane p run.
  constexpr bool PF = DIM == 3 && sizeof(QT) == 4;
  struct QRegs {
    QT v[PF ? P4 : 1][5];
  };
  struct FRegs {
    S v[PF ? P2 : 1][L::q];
  };
  auto fetch_q = [&](int gz, QRegs& r) {
    if constexpr (PF) {
      const uint32_t plane = sz * uint32_t(gz);
#pragma unroll
      for (int n = 0; n < P4; n++) {
        const int k = tid + n * NTHR;
        if (n == P4 - 1 && k >= R4::N) break;
        const uint32_t s = plane + q_off[n];
#pragma unroll
        for (int q = 0; q < 5; q++) r.v[n][q] = Qin[size_t(q) * size_t(N) + s];
      }
    }
  };
  auto store_q = [&](int m, const QRegs& r) {
    if constexpr (PF) {
#pragma unroll
      for (int n = 0; n < P4; n++) {
        const int k = tid + n * NTHR;
        if (n == P4 - 1 && k >= R4::N) break;
#pragma unroll
        for (int q = 0; q < 5; q++) sQ[m][q][k] = r.v[n][q];
      }
    }
  };

  // (a) Q of plane gz on the radius-4 rectangle into slot m
  auto load_q = [&](int m, int gz) {
    const uint32_t plane = sz * uint32_t(gz);
#pragma unroll
    for (int n = 0; n < P4; n++) {
      const int k = tid + n * NTHR;
      if (n == P4 - 1 && k >= R4::N) break;
      const uint32_t s = plane + q_off[n];
#pragma unroll
      for (int q = 0; q < 5; q++) sQ[m][q][k] = Qin[size_t(q) * size_t(N) + s];
    }
  };

  // (b) stress of the plane in slot m (z neighbours in zp, zm) on the
  // radius-3 rectangle without its corners
  auto stress_plane = [&](int m, int zp, int zm, int ts, int zs) {
    if constexpr (ISO) {  // every point of the rectangle: the body force reads the diagonal neighbours
      for (int k = tid; k < R3::N; k += NTHR) {
        const int i3 = k % R3::W, j3 = k / R3::W;
        Sym<QT> q, Lq, d[3];
        stencil_lds_iso2<QT, R4::W, R4::N>(sQ[m], (i3 + 1) + R4::W * (j3 + 1), q, d, Lq);
        const Sym<QT> H = molecular_field(q, Lq, cq);
        QT t[3][3];
        stress(q, H, d, cq, t);
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
          for (int b = 0; b < 2; b++) sTi[a][b][k] = t[a][b];
      }
      return;
    }
    for (int k = tid; k < R3::N; k += NTHR) {
      const int i3 = k % R3::W, j3 = k / R3::W;
      const bool xin = i3 >= 1 && i3 < R3::W - 1, yin = j3 >= 1 && j3 < R3::H - 1;
      if (!xin && !yin) continue;  // a corner: neither d_x nor d_y needs it
      Sym<QT> q, Lq, d[3];
      stencil_lds<QT, DIM, R4::W, R4::N>(sQ[m], sQ[zp], sQ[zm], (i3 + 1) + R4::W * (j3 + 1), q, d, Lq);
      const Sym<QT> H = molecular_field(q, Lq, cq);
      QT t[3][3];
      stress(q, H, d, cq, t);
      if (yin) {
        const int kx = i3 + WX * (j3 - 1);
#pragma unroll
        for (int a = 0; a < DIM; a++) sTx[ts][a][kx] = t[a][0];
      }
      if (xin) {
        const int ky = (i3 - 1) + WY * j3;
#pragma unroll
        for (int a = 0; a < DIM; a++) sTy[ts][a][ky] = t[a][1];
      }
      if constexpr (DIM == 3) {
        if (xin && yin) {
          const int k2 = (i3 - 1) + R2::W * (j3 - 1);
#pragma unroll
          for (int a = 0; a < 3; a++) sTz[zs][a][k2] = t[a][2];
        }
      }
    }
  };

  // (c) body force, moments and velocity of plane z on the radius-2
  // rectangle; the tile's own sites also collide and store (write: plane in
  // the block's chunk)
  // pull the populations of plane z at the thread's radius-2 points
  // f_i(x) = buf_i(x - c_i)
  auto pull = [&](int n, uint32_t plane, uint32_t zpo, uint32_t zmo, S (&f)[L::q]) {
    const uint32_t site = plane + ip[n].s;
#pragma unroll
    for (int i = 0; i < L::q; i++) {
      uint32_t d = site;
      if (L::cx(i) == 1) d += ip[n].xm;
      if (L::cx(i) == -1) d += ip[n].xp;
      if (L::cy(i) == 1) d += ip[n].ym;
      if (L::cy(i) == -1) d += ip[n].yp;
      if (L::cz(i) == 1) d += zmo;
      if (L::cz(i) == -1) d += zpo;
      f[i] = fin[size_t(i) * size_t(N) + d];
    }
  };
  auto zoffsets = [&](int gz, uint32_t& zpo, uint32_t& zmo) {
    zpo = (gz + 1 == g.nz) ? 0u - uint32_t(g.nz - 1) * sz : sz;
    zmo = (gz == 0) ? uint32_t(g.nz - 1) * sz : 0u - sz;
  };
  auto fetch_f = [&](int z, FRegs& r) {
    if constexpr (PF) {
      const int gz = wrapi(z, g.nz);
      uint32_t zpo, zmo;
      zoffsets(gz, zpo, zmo);
#pragma unroll
      for (int n = 0; n < P2; n++) {
        const int k = tid + n * NTHR;
        if (n == P2 - 1 && k >= R2::N) break;
        pull(n, sz * uint32_t(gz), zpo, zmo, r.v[n]);
      }
    }
  };

  auto lb_plane = [&](int z, int ts, int zsp, int zsm, int us, bool write, const FRegs* pre) {
    const int gz = wrapi(z, g.nz);
    const uint32_t plane = sz * uint32_t(gz);
    uint32_t zpo, zmo;
    zoffsets(gz, zpo, zmo);
#pragma unroll
    for (int n = 0; n < P2; n++) {
      const int k = tid + n * NTHR;
      if (n == P2 - 1 && k >= R2::N) break;
      int i2, j2;
      tile_first<TX, TY, 2>(k, i2, j2);
      const int k2 = i2 + R2::W * j2;
      S F[3] = {S(0), S(0), S(0)};
      if constexpr (ISO) {  // F_a = 3 sum_i w_i sum_b c_ib tau_ab(x + c_i), over pairs
        const int k3 = (i2 + 1) + R3::W * (j2 + 1);
#pragma unroll
        for (int a = 0; a < DIM; a++) {
          QT acc = QT(0);
#pragma unroll
          for (int i = 1; i < L::q; i++) {
            if (L::opp(i) < i) continue;
            const int o = L::cx(i) + R3::W * L::cy(i);
            QT dsum = QT(0);
#pragma unroll
            for (int b = 0; b < DIM; b++) {
              const int cb = b == 0 ? L::cx(i) : L::cy(i);
              if (cb == 0) continue;
              const QT dt = sTi[a][b][k3 + o] - sTi[a][b][k3 - o];
              dsum += cb > 0 ? dt : -dt;
            }
            acc += QT(3.0 * L::w(i)) * dsum;
          }
          F[a] = S(acc);
        }
      } else {
#pragma unroll
        for (int a = 0; a < DIM; a++) {
          const int kx = (i2 + 1) + WX * j2, ky = i2 + WY * (j2 + 1);
          QT acc = (sTx[ts][a][kx + 1] - sTx[ts][a][kx - 1]) + (sTy[ts][a][ky + WY] - sTy[ts][a][ky - WY]);
          if constexpr (DIM == 3) acc += sTz[zsp][a][k2] - sTz[zsm][a][k2];
          F[a] = S(QT(0.5) * acc);
        }
      }
      const uint32_t site = plane + ip[n].s;
      S f[L::q];
      if (PF && pre) {
#pragma unroll
        for (int i = 0; i < L::q; i++) f[i] = pre->v[PF ? n : 0][i];
      } else {
        pull(n, plane, zpo, zmo, f);
      }
      S rho, mass, u[3];
      moments<LAT, S, DEV>(f, F, rho, u, mass);
#pragma unroll
      for (int a = 0; a < DIM; a++) sU[us][a][k2] = QT(u[a]);
      if (write && k < NT && own) {
        if constexpr (MRT)
          collide_mrt<LAT, S, DEV>(f, rho, mass, u, F, c);
        else
          collide_pairs<LAT, S, DEV>(f, rho, mass, u, F, c);
#pragma unroll
        for (int i = 0; i < L::q; i++) store_out(&(fout + size_t(i) * size_t(N))[site], f[i]);
      }
    }
  };

  // What a tile site keeps from its predictor for its corrector (the same
  // quantities the two-sweep Q update keeps).
  struct Stash {
    Sym<QT> r;
    Flow<QT> fl;
    Sym<QT> q;
  };
  auto qp_of = [](const Stash& st) {
    return Sym<QT>{st.q.xx + st.r.xx, st.q.xy + st.r.xy, st.q.xz + st.r.xz, st.q.yy + st.r.yy, st.q.yz + st.r.yz};
  };
  // rate and predictor at radius-1 point (i1, j1): Q from slots m (centre
  // plane), zp, zm; velocity from slots um, uzp, uzm
  auto pred_point = [&](int m, int zp, int zm, int um, int uzp, int uzm, int i1, int j1, Stash& st) {
    const int k4 = (i1 + 3) + R4::W * (j1 + 3);
    const int k2 = (i1 + 1) + R2::W * (j1 + 1);
    Sym<QT> q, Lq, d[3];
    if constexpr (ISO)
      stencil_lds_iso2<QT, R4::W, R4::N, false>(sQ[m], k4, q, d, Lq);
    else
      stencil_lds<QT, DIM, R4::W, R4::N, false>(sQ[m], sQ[zp], sQ[zm], k4, q, d, Lq);
    const Sym<QT> H = SR ? molecular_field_exact(q, Lq, cq) : molecular_field(q, Lq, cq);
    QT u[3], G[3][3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
      u[a] = a < DIM ? sU[um][a][k2] * QT(0.5) : QT(0);
      if constexpr (ISO) {  // undivided: 6 sum_i w_i c_ib u_a(x + c_i), over pairs
        QT g0 = QT(0), g1 = QT(0), g2 = QT(0);
        if (a < DIM) {
#pragma unroll
          for (int i = 1; i < L::q; i++) {
            if (L::opp(i) < i) continue;
            const int o = L::cx(i) + R2::W * L::cy(i);
            const QT dif = sU[um][a][k2 + o] - sU[um][a][k2 - o];
            const QT w6 = QT(6.0 * L::w(i));
            if (L::cx(i) != 0) g0 += (L::cx(i) > 0 ? w6 : -w6) * dif;
            if (L::cy(i) != 0) g1 += (L::cy(i) > 0 ? w6 : -w6) * dif;
          }
        }
        G[a][0] = g0;
        G[a][1] = g1;
        G[a][2] = g2;
        continue;
      }
      G[a][0] = a < DIM ? sU[um][a][k2 + 1] - sU[um][a][k2 - 1] : QT(0);
      G[a][1] = a < DIM ? sU[um][a][k2 + R2::W] - sU[um][a][k2 - R2::W] : QT(0);
      if constexpr (DIM == 3)
        G[a][2] = sU[uzp][a][k2] - sU[uzm][a][k2];
      else
        G[a][2] = QT(0);
    }
    st.fl = flow_terms<QT, true>(u, G, cq);
    st.r = be_rate_flow<QT, true>(q, H, d, st.fl, cq);
    st.q = q;
    return qp_of(st);
  };
  // (d) predictor on the radius-1 rectangle into sP[ps]; the tile site's
  // stash into `own_st`
  auto pred_plane = [&](int m, int zp, int zm, int um, int uzp, int uzm, int ps, Stash& own_st) {
    for (int k = tid; k < R1::N; k += NTHR) {
      int i1, j1;
      tile_first<TX, TY, 1>(k, i1, j1);
      Stash tmp;
      Stash& st = k < NT ? own_st : tmp;
      const Sym<QT> qp = pred_point(m, zp, zm, um, uzp, uzm, i1, j1, st);
      const int k1 = i1 + R1::W * j1;
      sP[ps][0][k1] = qp.xx;
      sP[ps][1][k1] = qp.xy;
      sP[ps][2][k1] = qp.xz;
      sP[ps][3][k1] = qp.yy;
      sP[ps][4][k1] = qp.yz;
    }
  };
  // (e) corrector of the tile site in plane z: in-plane neighbours of Q^P
  // from sP[ps], the centre pc and the z neighbours pzp / pzm from registers
  const int k1 = (tx + 1) + R1::W * (ty + 1);
  auto corr_site = [&](int z, int ps, const Stash& st, const Sym<QT>& pc, const Sym<QT>& pzp, const Sym<QT>& pzm) {
    if (!own) return;
    if constexpr (ISO) {
      Sym<QT> pcc, Lp, d[3];
      stencil_lds_iso2<QT, R1::W, R1::N, false>(sP[ps], k1, pcc, d, Lp);
      const Sym<QT> H = SR ? molecular_field_exact(pcc, Lp, cq) : molecular_field(pcc, Lp, cq);
      const Sym<QT> Rp = be_rate_flow<QT, true>(pcc, H, d, st.fl, cq);
      const uint32_t s = uint32_t(x0 + tx) + uint32_t(g.nx) * (uint32_t(y0 + ty) + uint32_t(g.ny) * uint32_t(z));
      store_q_update<QT, SR>(Qout, N, int64_t(s), st.q, st.r, Rp, srkey);
      return;
    }
    const QT vc[5] = {pc.xx, pc.xy, pc.xz, pc.yy, pc.yz};
    const QT vzp[5] = {pzp.xx, pzp.xy, pzp.xz, pzp.yy, pzp.yz};
    const QT vzm[5] = {pzm.xx, pzm.xy, pzm.xz, pzm.yy, pzm.yz};
    QT lap[5], dx[5], dy[5], dz[5];
#pragma unroll
    for (int q = 0; q < 5; q++) {
      const QT cc = vc[q];
      const QT xp = sP[ps][q][k1 + 1], xm = sP[ps][q][k1 - 1];
      const QT yp = sP[ps][q][k1 + R1::W], ym = sP[ps][q][k1 - R1::W];
      dx[q] = xp - xm;
      dy[q] = yp - ym;
      QT l = (xp + xm) + (yp + ym);
      if constexpr (DIM == 3) {
        dz[q] = vzp[q] - vzm[q];
        l += vzp[q] + vzm[q];
        lap[q] = l - QT(6) * cc;
      } else {
        dz[q] = QT(0);
        lap[q] = l - QT(4) * cc;
      }
    }
    const Sym<QT> d[3] = {Sym<QT>{dx[0], dx[1], dx[2], dx[3], dx[4]}, Sym<QT>{dy[0], dy[1], dy[2], dy[3], dy[4]},
                          Sym<QT>{dz[0], dz[1], dz[2], dz[3], dz[4]}};
    const Sym<QT> Lp{lap[0], lap[1], lap[2], lap[3], lap[4]};
    const Sym<QT> H = SR ? molecular_field_exact(pc, Lp, cq) : molecular_field(pc, Lp, cq);
    const Sym<QT> Rp = be_rate_flow<QT, true>(pc, H, d, st.fl, cq);
    const uint32_t s = uint32_t(x0 + tx) + uint32_t(g.nx) * (uint32_t(y0 + ty) + uint32_t(g.ny) * uint32_t(z));
    store_q_update<QT, SR>(Qout, N, int64_t(s), st.q, st.r, Rp, srkey);
  };

  if constexpr (DIM == 2) {
    load_q(0, 0);
    __syncthreads();
    stress_plane(0, 0, 0, 0, 0);
    __syncthreads();
    lb_plane(0, 0, 0, 0, 0, true, nullptr);
    __syncthreads();
    Stash st;
    pred_plane(0, 0, 0, 0, 0, 0, 0, st);
    __syncthreads();
    const Sym<QT> pc = qp_of(st);
    corr_site(0, 0, st, pc, pc, pc);
  } else {
    const int zb = bz * zc;
    const int ze = min(zb + zc, g.nz);
    // ring slots of plane p (p >= zb - 8 > -2^30)
    auto s5 = [](int p) { return (p + (1 << 30)) % 5; };
    auto s3 = [](int p) { return (p + (1 << 30)) % 3; };
    auto s2 = [](int p) { return (p + (1 << 30)) & 1; };
    Sym<QT> pm = sym_zero<QT>();  // Q^P of plane p-5 at the tile site
    QRegs qr;
    FRegs fr;
    fetch_q(wrapi(zb - 4, g.nz), qr);
    // one iteration of the march (Q plane p newest); `prev` holds the stash
    // of plane p-4, `cur` receives that of plane p-3
    auto iteration = [&](int p, Stash& prev, Stash& cur) {
      // slot s5(p) = s5(p-5) was last read by the predictor of iteration p-1
      __syncthreads();
      if constexpr (PF) {
        store_q(s5(p), qr);
        if (p + 1 <= ze + 3) fetch_q(wrapi(p + 1, g.nz), qr);
      } else {
        load_q(s5(p), wrapi(p, g.nz));
      }
      __syncthreads();
      if (p - 1 >= zb - 3) stress_plane(s5(p - 1), s5(p), s5(p - 2), s2(p - 1), s3(p - 1));
      __syncthreads();
      if (p - 2 >= zb - 2)
        lb_plane(p - 2, s2(p - 2), s3(p - 1), s3(p - 3), s3(p - 2), p - 2 >= zb && p - 2 < ze, PF ? &fr : nullptr);
      // populations of the next moment plane, p - 1
      if (PF && p - 1 >= zb - 2 && p - 1 <= ze + 1) fetch_f(p - 1, fr);
      __syncthreads();
      if (p - 3 >= zb - 1)
        pred_plane(s5(p - 3), s5(p - 2), s5(p - 4), s3(p - 3), s3(p - 2), s3(p - 4), s2(p - 3), cur);
      const Sym<QT> pc = qp_of(prev);  // Q^P of plane p-4
      if (p - 4 >= zb) corr_site(wrapi(p - 4, g.nz), s2(p - 4), prev, pc, qp_of(cur), pm);
      pm = pc;
    };
    // two planes per trip, so the two stashes swap roles without copies
    Stash stA{}, stB{};
    int p = zb - 4;
    for (; p + 1 <= ze + 3; p += 2) {
      iteration(p, stA, stB);
      iteration(p + 1, stB, stA);
    }
    if (p <= ze + 3) iteration(p, stA, stB);
  }
}

template <int LAT, typename S, bool DEV, int TX, int TY, int NTHR, bool MRT, typename QT, bool SR,
          int ST = STENCIL_COMPACT>
__global__ void __launch_bounds__(NTHR)
    fused_step(const QT* __restrict__ Qin, const S* __restrict__ fin, S* __restrict__ fout, QT* __restrict__ Qout,
               GridDims g, Coef<S> c, Coef<QT> cq, int zc, uint32_t srkey) {
  const int nb = gridDim.x * gridDim.y * gridDim.z;
  const int t = xcd_remap(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), nb);
  fused_body<LAT, S, DEV, TX, TY, NTHR, MRT, QT, SR, ST>(Qin, fin, fout, Qout, g, c, cq, zc, t % gridDim.x,
                                               (t / gridDim.x) % gridDim.y, t / (gridDim.x * gridDim.y), srkey);
}

}  // namespace lc
