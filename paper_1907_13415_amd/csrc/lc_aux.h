// lc_aux.h -- state conversion, field export and the observable reductions.
#pragma once

#include "lc_staged.h"

namespace lc {

// Every kernel here takes the population type S (with DEV for the deviation
// form) and the order-tensor type QT (S, or double in the mixed form).

// Logical double state -> storage form.  f_dev == nullptr: fluid at rest.
// The population buffer is in pull form: buf_i(y) = f_i(y + c_i).
template <int LAT, typename S, bool DEV, typename QT = S>
__global__ void __launch_bounds__(256) load_state(const double* __restrict__ f_dev,
                                                  const double* __restrict__ q_dev, S* __restrict__ f,
                                                  QT* __restrict__ Q, GridDims g) {
  using L = Lattice<LAT>;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t N = g.N;
  const int64_t s = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
  const Nbr nb = neighbours(x, y, z, g.nx, g.ny, g.nz);
#pragma unroll
  for (int i = 0; i < L::q; i++) {
    int64_t d = s;
    if (L::cx(i) == 1) d += nb.xp;
    if (L::cx(i) == -1) d += nb.xm;
    if (L::cy(i) == 1) d += nb.yp;
    if (L::cy(i) == -1) d += nb.ym;
    if (L::cz(i) == 1) d += nb.zp;
    if (L::cz(i) == -1) d += nb.zm;
    const double w = L::w(i);
    const double v = f_dev ? f_dev[i * N + d] : w;
    f[i * N + s] = DEV ? S(v - w) : S(v);
  }
#pragma unroll
  for (int k = 0; k < 5; k++) Q[k * N + s] = QT(q_dev[k * N + s]);
}

template <int LAT, typename S, bool DEV, typename QT = S>
__global__ void __launch_bounds__(256) export_fq(const S* __restrict__ fb, const QT* __restrict__ Q,
                                                 double* __restrict__ fo, double* __restrict__ qo, GridDims g) {
  using L = Lattice<LAT>;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t N = g.N;
  const int64_t s = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
  if (fo) {
    const Nbr nb = neighbours(x, y, z, g.nx, g.ny, g.nz);
    S f[L::q];
    gather_f<LAT, S>(fb, N, s, nb, f);
#pragma unroll
    for (int i = 0; i < L::q; i++) fo[i * N + s] = DEV ? L::w(i) + double(f[i]) : double(f[i]);
  }
  if (qo) {
#pragma unroll
    for (int k = 0; k < 5; k++) qo[k * N + s] = double(Q[k * N + s]);
  }
}

// Derived fields: 0 rho, 1 u (3), 2 force (3), 3 S.  Needs tau (QT) in
// scratch; ST: the difference stencil of the body force.
template <int LAT, typename S, bool DEV, typename QT = S, int ST = STENCIL_COMPACT>
__global__ void __launch_bounds__(256) export_derived(const S* __restrict__ fin, const QT* __restrict__ Q,
                                                      const QT* __restrict__ tau, double* __restrict__ out,
                                                      int which, GridDims g) {
  using L = Lattice<LAT>;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t N = g.N;
  const int64_t s = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
  if (which == 3) {
    const Sym<QT> q = load_sym(Q, N, s);
    out[s] = sqrt(1.5 * double(ddot(q, q)));
    return;
  }
  const Nbr nb = neighbours(x, y, z, g.nx, g.ny, g.nz);
  QT FQ[3];
  body_force<LAT, QT, ST>(tau, N, s, nb, FQ);
  const S F[3] = {S(FQ[0]), S(FQ[1]), S(FQ[2])};
  S f[L::q];
  gather_f<LAT, S>(fin, N, s, nb, f);
  S rho, mass, u[3];
  moments<LAT, S, DEV>(f, F, rho, u, mass);
  if (which == 0) {
    out[s] = DEV ? 1.0 + double(mass) : double(rho);
  } else if (which == 1) {
#pragma unroll
    for (int a = 0; a < 3; a++) out[a * N + s] = double(u[a]);
  } else {
#pragma unroll
    for (int a = 0; a < 3; a++) out[a * N + s] = double(FQ[a]);
  }
}

// ---------------------------------------------------------------------------
// Observables.  Each block writes OBS_W doubles of partial results; a single
// block then combines them in a fixed order (deterministic for a fixed
// launch shape).
constexpr int OBS_W = 8;  // mass, mom x3, umax, ssum, shalf, nonfinite

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  return v;
}

// Block-wide reduction of OBS_W values (blockDim.x * blockDim.y <= 1024,
// multiple of 64).  Entry 4 (umax) and 7 (nonfinite) take the max.
__device__ __forceinline__ void block_reduce_obs(double (&v)[OBS_W], double* __restrict__ dst) {
  __shared__ double part[16][OBS_W];
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int nw = (blockDim.x * blockDim.y + 63) >> 6;
#pragma unroll
  for (int k = 0; k < OBS_W; k++) v[k] = (k == 4 || k == 7) ? wave_max(v[k]) : wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < OBS_W; k++) part[wid][k] = v[k];
  }
  __syncthreads();
  if (tid < OBS_W) {
    double acc = part[0][tid];
    for (int w = 1; w < nw; w++) acc = (tid == 4 || tid == 7) ? fmax(acc, part[w][tid]) : acc + part[w][tid];
    dst[tid] = acc;
  }
}

template <int LAT, typename S, bool DEV, typename QT = S, int ST = STENCIL_COMPACT>
__global__ void __launch_bounds__(256) observe_partial(const S* __restrict__ fin, const QT* __restrict__ Q,
                                                       const QT* __restrict__ tau, double* __restrict__ partial,
                                                       GridDims g, int half_axis, int want_u) {
  using L = Lattice<LAT>;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  double v[OBS_W] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (x < g.nx && y < g.ny) {
    const int64_t N = g.N;
    const int64_t s = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
    S f[L::q];
    bool bad = false;
    double m = 0, jx = 0, jy = 0, jz = 0;
    const Nbr nb = neighbours(x, y, z, g.nx, g.ny, g.nz);
    gather_f<LAT, S>(fin, N, s, nb, f);
#pragma unroll
    for (int i = 0; i < L::q; i++) {
      const double fi = double(f[i]);
      bad |= !isfinite(fi);
      m += fi;
      jx += L::cx(i) * fi;
      jy += L::cy(i) * fi;
      jz += L::cz(i) * fi;
    }
    v[0] = DEV ? 1.0 + m : m;
    v[1] = jx;
    v[2] = jy;
    v[3] = jz;
    if (want_u) {
      QT FQ[3];
      body_force<LAT, QT, ST>(tau, N, s, nb, FQ);
      const S F[3] = {S(FQ[0]), S(FQ[1]), S(FQ[2])};
      S rho, u[3];
      moments<LAT, S, DEV>(f, F, rho, u);
      const double uu = double(u[0]) * u[0] + double(u[1]) * u[1] + double(u[2]) * u[2];
      v[4] = sqrt(uu);
    }
    const Sym<QT> q = load_sym(Q, N, s);
    const double qq = double(q.xx) * q.xx + double(q.yy) * q.yy + (double(q.xx) + q.yy) * (double(q.xx) + q.yy) +
                      2.0 * (double(q.xy) * q.xy + double(q.xz) * q.xz + double(q.yz) * q.yz);
    bad |= !isfinite(qq);
    const double Sv = sqrt(1.5 * qq);
    v[5] = Sv;
    const int n_ax = half_axis == 0 ? g.nx : (half_axis == 1 ? g.ny : g.nz);
    const int k = half_axis == 0 ? x : (half_axis == 1 ? y : z);
    const int c0 = n_ax / 2, c1 = n_ax / 2 + n_ax / 2;
    if (k == c0 || k == c1 % n_ax)
      v[6] = 0.5 * Sv;
    else if (k > c0 && k < c1)
      v[6] = Sv;
    v[7] = bad ? 1.0 : 0.0;
    if (bad) v[4] = 0.0;
  }
  const int64_t b = blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
  block_reduce_obs(v, partial + b * OBS_W);
}

__global__ void __launch_bounds__(256) observe_final(const double* __restrict__ partial, int64_t nblocks,
                                                     double* __restrict__ out) {
  double v[OBS_W] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t b = threadIdx.x; b < nblocks; b += blockDim.x) {
#pragma unroll
    for (int k = 0; k < OBS_W; k++)
      v[k] = (k == 4 || k == 7) ? fmax(v[k], partial[b * OBS_W + k]) : v[k] + partial[b * OBS_W + k];
  }
  block_reduce_obs(v, out);
}

}  // namespace lc
