// lc_batch.h -- many independent two-dimensional grids in one launch.
//
// Each grid has its own size and parameters (for a temperature sweep each
// grid carries its own gamma).  The grids' fields are packed into shared
// arenas; a descriptor table gives every grid's size, arena offsets and
// coefficients, and a tile table maps each block of a launch to its grid.
// One launch of each sweep covers the tiles of all grids, so a time step of
// the whole batch is two launches, and a run of steps is captured once in a
// HIP graph and replayed.
#pragma once

#include "lc_split.h"

namespace lc {

// Key of the uniform numbers of the stochastic rounding at step `step` (the
// hash of the step counter; sites hash their index xor this key).  The
// single-grid step and the batched Q sweep take their keys from here, so a
// grid of a batch rounds as the same grid stepped alone.
LC_HD uint32_t step_key(int64_t step) { return pcg_hash(uint32_t(step) * 0x9E3779B9u + 0x7F4A7C15u); }

// S: type of the populations; QT: type of Q, the velocity and the
// molecular field, stress and body force (S, or double in the
// mixed-precision form).
template <typename S, typename QT = S>
struct BatchDesc {
  int nx, ny;
  int64_t N;
  int64_t f_off, q_off, u_off;  // element offsets into the arenas (f in S, Q and u in QT)
  int tile0[2], tiles_x[2];     // per sweep (0: LB, 1: Q): first block of this grid, tiles along x
  Coef<S> c;                    // constants in the population type
  Coef<QT> cq;                  // the same in the order-tensor type
};

// MRT: the multiple-relaxation-time collision (rates in the descriptors'
// constants); ST: the difference stencils (STENCIL_*).
template <int LAT, typename S, bool DEV, int TX, int TY, typename QT = S, bool MRT = false,
          int ST = STENCIL_COMPACT>
__global__ void __launch_bounds__(TX* TY)
    batch_lb(const BatchDesc<S, QT>* __restrict__ desc, const int* __restrict__ tile_grid,
             const QT* __restrict__ Qa, const S* __restrict__ fa, S* __restrict__ fb, QT* __restrict__ ua) {
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int k = tile_grid[b];
  const BatchDesc<S, QT> d = desc[k];
  const int t = b - d.tile0[0];
  const GridDims g{d.nx, d.ny, 1, d.N};
  // many grids stream through the caches together: populations read with
  // nontemporal loads
  split_lb_body<LAT, S, DEV, TX, TY, MRT, true, QT, ST>(Qa + d.q_off, fa + d.f_off, fb + d.f_off, ua + d.u_off, g,
                                                      d.c, d.cq, 1, t % d.tiles_x[0], t / d.tiles_x[0], 0);
}

// SR: the float form with stochastic rounding.  Its step key comes from
// the step count *step_base + step_off (modulo 2^32, as the key uses the
// count's low 32 bits): the host writes step_base before each run of
// launches (a captured graph of several steps, or one step), and each
// launch of the run carries its offset, so replays of a graph draw the keys
// of the steps they advance.
// The Q sweep runs in the order-tensor type QT; S is the population type
// of the descriptors.
template <int LAT, typename S, typename QT, int TX, int TY, bool SR = false, int ST = STENCIL_COMPACT>
__global__ void __launch_bounds__(TX* TY)
    batch_q(const BatchDesc<S, QT>* __restrict__ desc, const int* __restrict__ tile_grid,
            const QT* __restrict__ Qa, const QT* __restrict__ ua, QT* __restrict__ Qb,
            const uint32_t* __restrict__ step_base, int step_off) {
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int k = tile_grid[b];
  const BatchDesc<S, QT> d = desc[k];
  const int t = b - d.tile0[1];
  const GridDims g{d.nx, d.ny, 1, d.N};
  const uint32_t key = SR ? step_key(int64_t(*step_base) + step_off) : 0u;
  split_q_body<LAT, QT, TX, TY, SR, ST>(Qa + d.q_off, ua + d.u_off, Qb + d.q_off, g, d.cq, 1, t % d.tiles_x[1],
                                    t / d.tiles_x[1], 0, nullptr, key);
}

// Tile shapes the batch can run with, chosen per sweep by lc_batch_autotune
// (the stress sweep favours wide tiles, which share HBM lines; the Q sweep
// tiles with the smaller ring).
constexpr int BATCH_NV = 7;  // 32x8, 64x4, 16x16, 32x16, 64x8, 64x16, 128x8
__host__ __device__ constexpr int batch_tx(int v) {
  return v == 0 || v == 3 ? 32 : (v == 1 || v == 4 || v == 5 ? 64 : (v == 2 ? 16 : 128));
}
__host__ __device__ constexpr int batch_ty(int v) {
  return v == 0 || v == 4 || v == 6 ? 8 : (v == 1 ? 4 : 16);
}

}  // namespace lc
