// lc_runtime.hip -- the C ABI of include/lc.h: validation, context, scratch
// layout, kernel dispatch over (lattice, precision, variant).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/lc.h"
#include "lc_aux.h"
#include "lc_split.h"
#include "lc_fused.h"
#include "lc_batch.h"
#include "lc_vjp.h"
#include "lc_runtime.h"

namespace lc {

static thread_local std::string g_err;

lc_status fail(lc_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

lc_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return LC_OK;
  return fail(LC_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { g_err.clear(); }

int lattice_q(int lattice) { return lattice == LC_D2Q9 ? 9 : 19; }

lc_status check_grid(const lc_grid* g) {
  if (!g) return fail(LC_EINVAL, "grid is NULL");
  if (g->lattice != LC_D2Q9 && g->lattice != LC_D3Q19) return fail(LC_EINVAL, "unknown lattice %d", g->lattice);
  if (g->precision != LC_FP64 && g->precision != LC_FP32_DEV && g->precision != LC_MIXED &&
      g->precision != LC_FP32_SR)
    return fail(LC_EINVAL, "unknown precision %d", g->precision);
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return fail(LC_EINVAL, "grid dimensions must be >= 1");
  if (g->lattice == LC_D2Q9 && g->nz != 1) return fail(LC_EINVAL, "D2Q9 requires nz == 1");
  // site indices are 32-bit unsigned inside the sweeps; ny and nz index
  // launch grid dimensions, which are limited to 65535 blocks; launch
  // sizes round nx up to whole tiles in 32-bit arithmetic
  const double n = double(g->nx) * g->ny * g->nz;
  if (n > 4.0e9) return fail(LC_ENOMEM, "grid too large (%.3g sites; at most 4e9)", n);
  if (g->ny > 65535 || g->nz > 65535) return fail(LC_EINVAL, "ny and nz must not exceed 65535");
  if (g->nx > (1 << 30)) return fail(LC_EINVAL, "nx must not exceed 2^30");
  return LC_OK;
}

lc_status check_params(const lc_params* p) {
  if (!p) return fail(LC_EINVAL, "params is NULL");
  const double v[7] = {p->A0, p->gamma, p->K, p->Gamma, p->xi, p->eta, p->tau};
  for (double x : v)
    if (!std::isfinite(x)) return fail(LC_EINVAL, "parameters must be finite");
  if (!(p->tau > 0.5)) return fail(LC_EINVAL, "tau must exceed 1/2 (got %g)", p->tau);
  if (!(p->K >= 0)) return fail(LC_EINVAL, "K must be >= 0");
  if (!(p->Gamma > 0)) return fail(LC_EINVAL, "Gamma must be > 0");
  if (!(p->A0 > 0)) return fail(LC_EINVAL, "A0 must be > 0");
  const double eta = (p->tau - 0.5) / 3.0;
  if (std::fabs(p->eta - eta) > 1e-12 * std::fmax(1.0, std::fabs(eta)))
    return fail(LC_EINVAL, "eta (%g) inconsistent with tau: lattice viscosity is (tau-1/2)/3 = %g", p->eta, eta);
  return LC_OK;
}

template <typename S>
Coef<S> make_coef(const lc_params& p) {
  Coef<S> c;
  c.lin = S(-p.A0 * (1.0 - p.gamma / 3.0));
  c.quad = S(p.A0 * p.gamma);
  c.K = S(p.K);
  c.Gam = S(p.Gamma);
  c.xi = S(p.xi);
  c.xi_p = S((p.xi + 1.0) / 2.0);
  c.xi_m = S((p.xi - 1.0) / 2.0);
  c.omega = S(1.0 / p.tau);
  c.src = S(1.0 - 1.0 / (2.0 * p.tau));
  c.A0 = S(p.A0);
  for (int g = 0; g < 5; g++) c.mrt[g] = S(0);
  c.lin_d = -p.A0 * (1.0 - p.gamma / 3.0);
  c.quad_d = p.A0 * p.gamma;
  return c;
}

Layout layout_of(const lc_grid& g) {
  Layout L;
  const int64_t N = int64_t(g.nx) * g.ny * g.nz;
  const size_t es = g.precision == LC_FP64 ? 8 : 4;
  const size_t es_q = (g.precision == LC_FP32_DEV || g.precision == LC_FP32_SR) ? 4 : 8;
  const int dim = g.lattice == LC_D2Q9 ? 2 : 3;
  const int ntau = dim == 2 ? 4 : 9;
  auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
  L.N = N;
  L.q = lattice_q(g.lattice);
  L.es = es;
  L.es_q = es_q;
  L.f_bytes = size_t(L.q) * N * es;
  L.q_bytes = size_t(5) * N * es_q;
  size_t off = 0;
  L.off_tau = off;
  off = up(off + size_t(ntau) * N * es_q);
  L.off_u = off;
  off = up(off + size_t(dim) * N * es_q);
  L.off_qp = off;
  off = up(off + size_t(5) * N * es_q);
  L.off_r = off;
  off = up(off + size_t(5) * N * es_q);
  const dim3 grid = site_grid(g);
  L.nblocks = int64_t(grid.x) * grid.y * grid.z;
  L.off_partial = off;
  off = up(off + size_t(L.nblocks) * OBS_W * 8);
  L.off_obs = off;
  off = up(off + OBS_W * 8);
  L.off_vjp = off;
  if (g.lattice == LC_D2Q9 && g.precision == LC_FP64) {
    off = up(off + size_t(VJP_COMPS) * N * 8);
    off = up(off + size_t(3) * L.nblocks * 3 * 8);
  }
  L.scratch_bytes = off;
  return L;
}

dim3 site_block() { return dim3(SITE_TX, SITE_TY, 1); }

dim3 site_grid(const lc_grid& g) {
  const dim3 b = site_block();
  return dim3((g.nx + b.x - 1) / b.x, (g.ny + b.y - 1) / b.y, g.nz);
}

}  // namespace lc

using namespace lc;

struct lc_ctx {
  lc_grid g;
  lc_params p;
  lc_buffers b;
  hipStream_t stream;
  Layout L;
  int parity;
  int64_t step;
  bool loaded;
  int variant;     // LC_VARIANT_* as requested (AUTO resolved at each step)
  int stencil = LC_STENCIL_COMPACT;  // LC_STENCIL_*
  int zchunk;  // 0: default
  int coll;        // LC_COLL_*
  double mrt[5];   // MRT rates of the ghost groups
  // optional per-launch timing of the step kernels: events recorded on the
  // stream before and after each launch (kind 0: the stress/LB sweep or the
  // single pass, kind 1: the Q sweep), folded into the sums below whenever
  // the record reaches its cap, so a long timed run holds a bounded number
  // of events
  bool timing;
  struct Timed {
    hipEvent_t a, b;
    int kind;
  };
  std::vector<Timed> ev;
  std::vector<hipEvent_t> pool;   // idle events for reuse
  double acc_ms[2] = {0.0, 0.0};
  int64_t acc_n[2] = {0, 0};
  // second stream and ordering events of the overlapped reverse sweep
  // (created on first use)
  hipStream_t aux = nullptr;
  hipEvent_t vev[5] = {};
};

namespace lc {
static hipEvent_t ctx_event(lc_ctx* c) {
  hipEvent_t e = nullptr;
  if (!c->pool.empty()) {
    e = c->pool.back();
    c->pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    e = nullptr;
  }
  return e;
}
// Kernel constants of the context: parameters plus, for MRT, each ghost
// group's rate minus 1/tau.
template <typename S>
static Coef<S> ctx_coef(const lc_ctx* c) {
  Coef<S> k = make_coef<S>(c->p);
  if (c->coll == LC_COLL_MRT)
    for (int g = 0; g < 5; g++) k.mrt[g] = S(c->mrt[g] - 1.0 / c->p.tau);
  return k;
}

// Launches whose events the context holds before folding them.
constexpr size_t TIMED_CAP = 1024;

// Add the elapsed times of every recorded launch to the sums and return the
// events to the pool (waits for the last recorded event).
static lc_status ctx_fold(lc_ctx* c) {
  if (c->ev.empty()) return LC_OK;
  lc_status st = hip_check(hipEventSynchronize(c->ev.back().b), "timing sync");
  if (st) return st;
  for (const auto& t : c->ev) {
    float ms = 0;
    (void)hipEventElapsedTime(&ms, t.a, t.b);
    c->acc_ms[t.kind] += ms;
    c->acc_n[t.kind]++;
    c->pool.push_back(t.a);
    c->pool.push_back(t.b);
  }
  c->ev.clear();
  return LC_OK;
}

// Event before a timed launch (nullptr when timing is off or no event).
static hipEvent_t ctx_begin(lc_ctx* c, hipStream_t st) {
  if (!c->timing) return nullptr;
  if (c->ev.size() >= TIMED_CAP) (void)ctx_fold(c);
  hipEvent_t e = ctx_event(c);
  if (e) (void)hipEventRecord(e, st);
  return e;
}

static void ctx_end(lc_ctx* c, hipStream_t st, hipEvent_t a, int kind) {
  if (!a) return;
  hipEvent_t b = ctx_event(c);
  if (!b) {
    c->pool.push_back(a);
    return;
  }
  (void)hipEventRecord(b, st);
  c->ev.push_back(lc_ctx::Timed{a, b, kind});
}
}  // namespace lc

// ---------------------------------------------------------------------------
// Dispatch helpers.  Each is instantiated for (lattice, S = population and
// collision type, DEV = deviation storage, QT = order-tensor type).
template <int LAT, typename S, bool DEV, int ST>
static lc_status run_steps_staged_st(lc_ctx* c, int64_t n) {
  const GridDims gd{c->g.nx, c->g.ny, c->g.nz, c->L.N};
  const Coef<S> k = ctx_coef<S>(c);
  char* scr = static_cast<char*>(c->b.scratch);
  S* tau = reinterpret_cast<S*>(scr + c->L.off_tau);
  S* u = reinterpret_cast<S*>(scr + c->L.off_u);
  S* qp = reinterpret_cast<S*>(scr + c->L.off_qp);
  S* rq = reinterpret_cast<S*>(scr + c->L.off_r);
  const dim3 grid = site_grid(c->g), block = site_block();
  for (int64_t it = 0; it < n; it++) {
    const S* f0 = static_cast<const S*>(c->b.f[c->parity]);
    S* f1 = static_cast<S*>(c->b.f[c->parity ^ 1]);
    const S* q0 = static_cast<const S*>(c->b.Q[c->parity]);
    S* q1 = static_cast<S*>(c->b.Q[c->parity ^ 1]);
    hipLaunchKernelGGL((stage_tau<LAT, S, ST>), grid, block, 0, c->stream, q0, tau, gd, k);
    if (c->coll == LC_COLL_MRT)
      hipLaunchKernelGGL((stage_lb<LAT, S, DEV, true, ST>), grid, block, 0, c->stream, f0, tau, f1, u, gd, k);
    else
      hipLaunchKernelGGL((stage_lb<LAT, S, DEV, false, ST>), grid, block, 0, c->stream, f0, tau, f1, u, gd, k);
    hipLaunchKernelGGL((stage_pred<LAT, S, ST>), grid, block, 0, c->stream, q0, u, qp, rq, gd, k);
    hipLaunchKernelGGL((stage_corr<LAT, S, ST>), grid, block, 0, c->stream, q0, qp, rq, u, q1, gd, k);
    c->parity ^= 1;
    c->step++;
  }
  return hip_check(hipGetLastError(), "step launch");
}

template <int LAT, typename S, bool DEV, typename QT = S>
static lc_status run_steps_staged(lc_ctx* c, int64_t n) {
  if constexpr (!std::is_same<S, QT>::value) {
    return fail(LC_EUNSUPPORTED, "the staged variant has no mixed-precision form");
  } else {
    if (c->g.precision == LC_FP32_SR)
      return fail(LC_EUNSUPPORTED, "the staged variant has no stochastic-rounding form");
    if (c->stencil == LC_STENCIL_ISOTROPIC) return run_steps_staged_st<LAT, S, DEV, STENCIL_ISO>(c, n);
    return run_steps_staged_st<LAT, S, DEV, STENCIL_COMPACT>(c, n);
  }
}


// One step of the split sweeps between explicit buffers (pull-form
// populations) on stream st; u receives the force-corrected velocity.
// rec_lb / rec_q, when not null, record rho and F / the predictor for
// reverse-mode replay.  With mark, timing events bracket the two sweeps.
template <int LAT, typename S, bool DEV, typename QT = S>
static void step_split_ptrs(lc_ctx* c, hipStream_t st, bool mark, const S* f0, const QT* q0, S* f1, QT* q1, QT* u,
                            S* rec_lb, QT* rec_q) {
  // tile shapes of the order-tensor type, whose LDS regions dominate
  using C = SplitCfg<LAT, QT, S>;
  const GridDims gd{c->g.nx, c->g.ny, c->g.nz, c->L.N};
  const Coef<S> k = ctx_coef<S>(c);
  const Coef<QT> kq = ctx_coef<QT>(c);
  // MRT and the isotropic stencils march 32-plane chunks in the float
  // stress/LB sweep (1% and 3% faster there than 16)
  const bool wide = sizeof(S) == 4 && (c->coll == LC_COLL_MRT || c->stencil == LC_STENCIL_ISOTROPIC);
  // chunks longer than the grid are the whole depth (the block index
  // arithmetic stays within int)
  const int zc1 = C::d3 ? std::min(c->zchunk > 0 ? c->zchunk : (wide ? 32 : C::ZC_LB), c->g.nz) : 1;
  const int zc2 = C::d3 ? std::min(c->zchunk > 0 ? c->zchunk : C::ZC_Q, c->g.nz) : 1;
  const dim3 g1((c->g.nx + C::LB_TX - 1) / C::LB_TX, (c->g.ny + C::LB_TY - 1) / C::LB_TY,
                unsigned((c->g.nz + zc1 - 1) / zc1));
  const dim3 g2((c->g.nx + C::Q_TX - 1) / C::Q_TX, (c->g.ny + C::Q_TY - 1) / C::Q_TY,
                unsigned((c->g.nz + zc2 - 1) / zc2));
  hipEvent_t e = mark ? ctx_begin(c, st) : nullptr;
  if constexpr (std::is_same<S, QT>::value) {
    if (c->stencil == LC_STENCIL_ISOTROPIC) {  // the sweeps with the isotropic stencils
      // stress/LB tiles whose stress ring of three planes (3D) leaves room
      // for two blocks per CU: 32x8 (float), 16x8 (double in 3D)
      constexpr int ITX = (C::d3 && sizeof(S) == 8) ? 16 : 32, ITY = 8;
      const dim3 gi((c->g.nx + ITX - 1) / ITX, (c->g.ny + ITY - 1) / ITY, unsigned((c->g.nz + zc1 - 1) / zc1));
      if (c->coll == LC_COLL_MRT)
        hipLaunchKernelGGL((split_lb<LAT, S, DEV, ITX, ITY, 1, true, QT, STENCIL_ISO>), gi, dim3(ITX, ITY), 0, st, q0,
                           f0, f1, u, gd, k, kq, zc1, rec_lb);
      else
        hipLaunchKernelGGL((split_lb<LAT, S, DEV, ITX, ITY, 1, false, QT, STENCIL_ISO>), gi, dim3(ITX, ITY), 0, st,
                           q0, f0, f1, u, gd, k, kq, zc1, rec_lb);
      ctx_end(c, st, e, 0);
      e = mark ? ctx_begin(c, st) : nullptr;
      // the 3D float Q sweep with these stencils is held to two waves per
      // SIMD (some registers spill; measured 12% faster than one wave)
      constexpr int IQW = (C::d3 && sizeof(QT) == 4) ? 2 : C::Q_WPE;
      hipLaunchKernelGGL((split_q<LAT, QT, C::Q_TX, C::Q_TY, IQW, false, STENCIL_ISO>), g2,
                         dim3(C::Q_TX, C::Q_TY), 0, st, q0, u, q1, gd, kq, zc2, rec_q, 0u);
      ctx_end(c, st, e, 1);
      return;
    }
  }
  if (c->coll == LC_COLL_MRT)
    hipLaunchKernelGGL((split_lb<LAT, S, DEV, C::LB_TX, C::LB_TY, C::LB_WPE, true, QT>), g1,
                       dim3(C::LB_TX, C::LB_TY), 0, st, q0, f0, f1, u, gd, k, kq, zc1, rec_lb);
  else
    hipLaunchKernelGGL((split_lb<LAT, S, DEV, C::LB_TX, C::LB_TY, C::LB_WPE, false, QT>), g1,
                       dim3(C::LB_TX, C::LB_TY), 0, st, q0, f0, f1, u, gd, k, kq, zc1, rec_lb);
  ctx_end(c, st, e, 0);
  e = mark ? ctx_begin(c, st) : nullptr;
  if (std::is_same<QT, float>::value && c->g.precision == LC_FP32_SR)
    hipLaunchKernelGGL((split_q<LAT, QT, C::Q_TX, C::Q_TY, C::Q_WPE, std::is_same<QT, float>::value>), g2,
                       dim3(C::Q_TX, C::Q_TY), 0, st, q0, u, q1, gd, kq, zc2, rec_q, step_key(c->step));
  else
    hipLaunchKernelGGL((split_q<LAT, QT, C::Q_TX, C::Q_TY, C::Q_WPE>), g2, dim3(C::Q_TX, C::Q_TY), 0, st, q0, u, q1,
                       gd, kq, zc2, rec_q, 0u);
  ctx_end(c, st, e, 1);
}

// One launch of the single pass with tile TX x TY and NTHR threads.
template <int LAT, typename S, bool DEV, typename QT, int TX, int TY, int NTHR>
static void launch_fused(lc_ctx* c, hipStream_t st, int zc, const S* f0, const QT* q0, S* f1, QT* q1) {
  const GridDims gd{c->g.nx, c->g.ny, c->g.nz, c->L.N};
  const Coef<S> k = ctx_coef<S>(c);
  const Coef<QT> kq = ctx_coef<QT>(c);
  const dim3 grid((c->g.nx + TX - 1) / TX, (c->g.ny + TY - 1) / TY, unsigned((c->g.nz + zc - 1) / zc));
  constexpr bool F32 = std::is_same<QT, float>::value;
  const bool sr = F32 && c->g.precision == LC_FP32_SR;
  const uint32_t key = step_key(c->step);
  // the isotropic stencils: two-dimensional grids, FP64 and the FP32
  // deviation form (lc_set_stencil), BGK or MRT
  if constexpr (Lattice<LAT>::dim == 2 && std::is_same<S, QT>::value) {
    if (c->stencil == LC_STENCIL_ISOTROPIC) {
      if (c->coll == LC_COLL_MRT)
        hipLaunchKernelGGL((fused_step<LAT, S, DEV, TX, TY, NTHR, true, QT, false, STENCIL_ISO>), grid, dim3(NTHR), 0,
                           st, q0, f0, f1, q1, gd, k, kq, zc, key);
      else
        hipLaunchKernelGGL((fused_step<LAT, S, DEV, TX, TY, NTHR, false, QT, false, STENCIL_ISO>), grid, dim3(NTHR),
                           0, st, q0, f0, f1, q1, gd, k, kq, zc, key);
      return;
    }
  }
  if (c->coll == LC_COLL_MRT) {
    if (sr)
      hipLaunchKernelGGL((fused_step<LAT, S, DEV, TX, TY, NTHR, true, QT, F32>), grid, dim3(NTHR), 0, st, q0, f0, f1,
                         q1, gd, k, kq, zc, key);
    else
      hipLaunchKernelGGL((fused_step<LAT, S, DEV, TX, TY, NTHR, true, QT, false>), grid, dim3(NTHR), 0, st, q0, f0,
                         f1, q1, gd, k, kq, zc, key);
  } else {
    if (sr)
      hipLaunchKernelGGL((fused_step<LAT, S, DEV, TX, TY, NTHR, false, QT, F32>), grid, dim3(NTHR), 0, st, q0, f0,
                         f1, q1, gd, k, kq, zc, key);
    else
      hipLaunchKernelGGL((fused_step<LAT, S, DEV, TX, TY, NTHR, false, QT, false>), grid, dim3(NTHR), 0, st, q0, f0,
                         f1, q1, gd, k, kq, zc, key);
  }
}

// One step of the single pass between explicit buffers on stream st.  On a
// two-dimensional grid the tile shape and threads per tile follow from the
// number of tiles (FUSED2D_* in lc_fused.h).
template <int LAT, typename S, bool DEV, typename QT = S>
static void step_fused_ptrs(lc_ctx* c, hipStream_t st, bool mark, const S* f0, const QT* q0, S* f1, QT* q1) {
  using C = FusedCfg<LAT, QT>;
  hipEvent_t e = mark ? ctx_begin(c, st) : nullptr;
  if constexpr (C::d3) {
    const int zc = std::min(c->zchunk > 0 ? c->zchunk : C::ZC, c->g.nz);
    launch_fused<LAT, S, DEV, QT, C::TX, C::TY, C::NTHR>(c, st, zc, f0, q0, f1, q1);
  } else {
    auto tiles = [&](int tx, int ty) { return int64_t((c->g.nx + tx - 1) / tx) * ((c->g.ny + ty - 1) / ty); };
    if (tiles(FUSED2D_SMALL_TX, FUSED2D_SMALL_TY) <= FUSED2D_CUS)
      launch_fused<LAT, S, DEV, QT, FUSED2D_SMALL_TX, FUSED2D_SMALL_TY, FUSED2D_SMALL_NTHR>(c, st, 1, f0, q0, f1, q1);
    else if (tiles(FUSED2D_MID_TX, FUSED2D_MID_TY) <= FUSED2D_CUS)
      launch_fused<LAT, S, DEV, QT, FUSED2D_MID_TX, FUSED2D_MID_TY, FUSED2D_MID_NTHR>(c, st, 1, f0, q0, f1, q1);
    else if (tiles(FUSED2D_HALF_TX, FUSED2D_HALF_TY) <= 4 * FUSED2D_CUS)
      launch_fused<LAT, S, DEV, QT, FUSED2D_HALF_TX, FUSED2D_HALF_TY, FUSED2D_HALF_NTHR>(c, st, 1, f0, q0, f1, q1);
    else
      launch_fused<LAT, S, DEV, QT, FUSED2D_WIDE_TX, FUSED2D_WIDE_TY, FUSED2D_WIDE_NTHR>(c, st, 1, f0, q0, f1, q1);
  }
  ctx_end(c, st, e, 0);
}

template <int LAT, typename S, bool DEV, typename QT = S>
static lc_status run_steps_fused(lc_ctx* c, int64_t n) {
  for (int64_t it = 0; it < n; it++) {
    step_fused_ptrs<LAT, S, DEV, QT>(c, c->stream, true, static_cast<const S*>(c->b.f[c->parity]),
                                     static_cast<const QT*>(c->b.Q[c->parity]),
                                     static_cast<S*>(c->b.f[c->parity ^ 1]), static_cast<QT*>(c->b.Q[c->parity ^ 1]));
    c->parity ^= 1;
    c->step++;
  }
  return hip_check(hipGetLastError(), "step launch");
}

template <int LAT, typename S, bool DEV, typename QT = S>
static lc_status run_steps_split(lc_ctx* c, int64_t n) {
  QT* u = reinterpret_cast<QT*>(static_cast<char*>(c->b.scratch) + c->L.off_u);
  for (int64_t it = 0; it < n; it++) {
    step_split_ptrs<LAT, S, DEV, QT>(c, c->stream, true, static_cast<const S*>(c->b.f[c->parity]),
                                     static_cast<const QT*>(c->b.Q[c->parity]),
                                     static_cast<S*>(c->b.f[c->parity ^ 1]), static_cast<QT*>(c->b.Q[c->parity ^ 1]),
                                     u, nullptr, nullptr);
    c->parity ^= 1;
    c->step++;
  }
  return hip_check(hipGetLastError(), "step launch");
}

// The variant a step runs.  AUTO is the two-sweep variant, except the
// single pass (with the compact stencils) on two-dimensional grids of at
// most 384^2 sites, whose launches are latency bound and where one launch
// per step with several threads per tile site measured faster than the two
// sweeps in every precision (bit-identical results; 256^2: 6.1 against 8.8
// us in FP32, 7.3 against 9.5 us in FP64; 384^2: 9.3 against 11.1 and 14.5
// against 14.7 us; from 448^2 the mixed form, from 512^2 FP64 and FP32 with
// stochastic rounding are faster in two sweeps).
constexpr int64_t AUTO_FUSED_MAX_SITES = 384 * 384;
// With the isotropic stencils the single pass measured faster up to 256^2
// (128^2: 6.1 against 9.3 us in FP32, 7.1 against 10.6 in FP64; 256^2: 7.0
// against 9.8 and 8.7 against 11.1 us; at 320^2 FP64 is faster in two
// sweeps).
constexpr int64_t AUTO_FUSED_MAX_SITES_ISO = 256 * 256;
static int resolved_variant(const lc_ctx* c) {
  if (c->variant != LC_VARIANT_AUTO) return c->variant;
  if (c->stencil == LC_STENCIL_ISOTROPIC)
    return c->g.lattice == LC_D2Q9 && c->L.N <= AUTO_FUSED_MAX_SITES_ISO ? LC_VARIANT_FUSED : LC_VARIANT_SPLIT;
  if (c->g.lattice == LC_D2Q9 && c->L.N <= AUTO_FUSED_MAX_SITES) return LC_VARIANT_FUSED;
  return LC_VARIANT_SPLIT;
}

template <int LAT, typename S, bool DEV, typename QT = S>
static lc_status run_steps(lc_ctx* c, int64_t n) {
  const int v = resolved_variant(c);
  if (c->stencil == LC_STENCIL_ISOTROPIC && v == LC_VARIANT_FUSED && c->g.lattice != LC_D2Q9)
    return fail(LC_EUNSUPPORTED, "the single pass takes the isotropic stencils on D2Q9 grids only");
  if (v == LC_VARIANT_SPLIT) return run_steps_split<LAT, S, DEV, QT>(c, n);
  if (v == LC_VARIANT_FUSED) return run_steps_fused<LAT, S, DEV, QT>(c, n);
  return run_steps_staged<LAT, S, DEV, QT>(c, n);
}

template <int LAT, typename S, bool DEV, typename QT = S>
static lc_status compute_tau(lc_ctx* c) {
  const GridDims gd{c->g.nx, c->g.ny, c->g.nz, c->L.N};
  const Coef<QT> k = make_coef<QT>(c->p);
  QT* tau = reinterpret_cast<QT*>(static_cast<char*>(c->b.scratch) + c->L.off_tau);
  const QT* q = static_cast<const QT*>(c->b.Q[c->parity]);
  if (c->stencil == LC_STENCIL_ISOTROPIC)
    hipLaunchKernelGGL((stage_tau<LAT, QT, STENCIL_ISO>), site_grid(c->g), site_block(), 0, c->stream, q, tau, gd, k);
  else
    hipLaunchKernelGGL((stage_tau<LAT, QT>), site_grid(c->g), site_block(), 0, c->stream, q, tau, gd, k);
  return hip_check(hipGetLastError(), "stress launch");
}

template <int LAT, typename S, bool DEV, typename QT = S>
static lc_status do_load(lc_ctx* c, const double* f, const double* q) {
  const GridDims gd{c->g.nx, c->g.ny, c->g.nz, c->L.N};
  hipLaunchKernelGGL((load_state<LAT, S, DEV, QT>), site_grid(c->g), site_block(), 0, c->stream, f, q,
                     static_cast<S*>(c->b.f[0]), static_cast<QT*>(c->b.Q[0]), gd);
  return hip_check(hipGetLastError(), "load launch");
}

template <int LAT, typename S, bool DEV, typename QT = S>
static lc_status do_export(lc_ctx* c, int field, double* dst) {
  const int64_t N = c->L.N;
  const S* f = static_cast<const S*>(c->b.f[c->parity]);
  const QT* q = static_cast<const QT*>(c->b.Q[c->parity]);
  if (field == LC_FIELD_F || field == LC_FIELD_Q) {
    const GridDims gd{c->g.nx, c->g.ny, c->g.nz, N};
    hipLaunchKernelGGL((export_fq<LAT, S, DEV, QT>), site_grid(c->g), site_block(), 0, c->stream, f, q,
                       field == LC_FIELD_F ? dst : nullptr, field == LC_FIELD_Q ? dst : nullptr, gd);
    return hip_check(hipGetLastError(), "export launch");
  }
  int which = field == LC_FIELD_RHO ? 0 : field == LC_FIELD_U ? 1 : field == LC_FIELD_FORCE ? 2 : 3;
  if (which != 3) {
    lc_status st = compute_tau<LAT, S, DEV, QT>(c);
    if (st) return st;
  }
  const GridDims gd{c->g.nx, c->g.ny, c->g.nz, N};
  const QT* tau = reinterpret_cast<const QT*>(static_cast<char*>(c->b.scratch) + c->L.off_tau);
  if (c->stencil == LC_STENCIL_ISOTROPIC)
    hipLaunchKernelGGL((export_derived<LAT, S, DEV, QT, STENCIL_ISO>), site_grid(c->g), site_block(), 0, c->stream, f,
                       q, tau, dst, which, gd);
  else
    hipLaunchKernelGGL((export_derived<LAT, S, DEV, QT>), site_grid(c->g), site_block(), 0, c->stream, f, q, tau,
                       dst, which, gd);
  return hip_check(hipGetLastError(), "export launch");
}

// Reductions of the current state into OBS_W doubles at res (device),
// enqueued on the context stream.
template <int LAT, typename S, bool DEV, typename QT = S>
static lc_status do_observe_async(lc_ctx* c, uint32_t mask, int half_axis, double* res) {
  const int want_u = (mask & LC_OBS_UMAX) ? 1 : 0;
  if (want_u) {
    lc_status st = compute_tau<LAT, S, DEV, QT>(c);
    if (st) return st;
  }
  const GridDims gd{c->g.nx, c->g.ny, c->g.nz, c->L.N};
  char* scr = static_cast<char*>(c->b.scratch);
  const QT* tau = reinterpret_cast<const QT*>(scr + c->L.off_tau);
  double* partial = reinterpret_cast<double*>(scr + c->L.off_partial);
  const S* f = static_cast<const S*>(c->b.f[c->parity]);
  const QT* q = static_cast<const QT*>(c->b.Q[c->parity]);
  if (c->stencil == LC_STENCIL_ISOTROPIC)
    hipLaunchKernelGGL((observe_partial<LAT, S, DEV, QT, STENCIL_ISO>), site_grid(c->g), site_block(), 0, c->stream,
                       f, q, tau, partial, gd, half_axis, want_u);
  else
    hipLaunchKernelGGL((observe_partial<LAT, S, DEV, QT>), site_grid(c->g), site_block(), 0, c->stream, f, q, tau,
                       partial, gd, half_axis, want_u);
  hipLaunchKernelGGL(observe_final, dim3(1), dim3(256), 0, c->stream, partial, c->L.nblocks, res);
  return hip_check(hipGetLastError(), "observe launch");
}

template <int LAT, typename S, bool DEV, typename QT = S>
static lc_status do_observe(lc_ctx* c, uint32_t mask, int half_axis, double* host8) {
  double* res = reinterpret_cast<double*>(static_cast<char*>(c->b.scratch) + c->L.off_obs);
  lc_status st = do_observe_async<LAT, S, DEV, QT>(c, mask, half_axis, res);
  if (st) return st;
  st = hip_check(hipMemcpyAsync(host8, res, OBS_W * sizeof(double), hipMemcpyDeviceToHost, c->stream),
                 "observe copy");
  if (st) return st;
  return hip_check(hipStreamSynchronize(c->stream), "observe sync");
}

static void fill_observables(const double* h, uint32_t mask, int half_axis, int64_t step, lc_observables* out) {
  std::memset(out, 0, sizeof *out);
  if (mask & LC_OBS_MASS) out->mass = h[0];
  if (mask & LC_OBS_MOM) {
    out->mom[0] = h[1];
    out->mom[1] = h[2];
    out->mom[2] = h[3];
  }
  if (mask & LC_OBS_UMAX) out->umax = h[4];
  if (mask & LC_OBS_S) {
    out->ssum = h[5];
    out->ssum_half = h[6];
  }
  out->step = step;
  out->half_axis = half_axis;
  out->nonfinite = h[7] != 0.0 ? 1 : 0;
}

// LC_FP32_DEV and LC_FP32_SR share their storage and every kernel but the
// Q update, which the step dispatch picks from the precision.
#define LC_DISPATCH_LAT(ctx, LAT, FN, ...)                                              \
  ((ctx)->g.precision == LC_FP64    ? FN<LAT, double, false, double>(ctx, ##__VA_ARGS__) \
   : (ctx)->g.precision == LC_MIXED ? FN<LAT, float, true, double>(ctx, ##__VA_ARGS__)   \
                                    : FN<LAT, float, true, float>(ctx, ##__VA_ARGS__))
#define LC_DISPATCH(ctx, FN, ...)                                                 \
  ((ctx)->g.lattice == LC_D2Q9 ? LC_DISPATCH_LAT(ctx, 0, FN, ##__VA_ARGS__)       \
                               : LC_DISPATCH_LAT(ctx, 1, FN, ##__VA_ARGS__))

// ---------------------------------------------------------------------------
extern "C" {

const char* lc_last_error(void) { return g_err.c_str(); }

lc_status lc_lattice_info(int32_t lattice, int32_t* q, int32_t* c, double* w) {
  clear_error();
  if (!q) return fail(LC_EINVAL, "q is NULL");
  if (lattice == LC_D2Q9) {
    *q = 9;
    for (int i = 0; i < 9; i++) {
      if (c) {
        c[3 * i] = Lattice<0>::cx(i);
        c[3 * i + 1] = Lattice<0>::cy(i);
        c[3 * i + 2] = Lattice<0>::cz(i);
      }
      if (w) w[i] = Lattice<0>::w(i);
    }
    return LC_OK;
  }
  if (lattice == LC_D3Q19) {
    *q = 19;
    for (int i = 0; i < 19; i++) {
      if (c) {
        c[3 * i] = Lattice<1>::cx(i);
        c[3 * i + 1] = Lattice<1>::cy(i);
        c[3 * i + 2] = Lattice<1>::cz(i);
      }
      if (w) w[i] = Lattice<1>::w(i);
    }
    return LC_OK;
  }
  return fail(LC_EINVAL, "unknown lattice %d", lattice);
}

lc_status lc_buffer_bytes(const lc_grid* grid, size_t* f_bytes, size_t* q_bytes, size_t* scratch_bytes) {
  clear_error();
  lc_status st = check_grid(grid);
  if (st) return st;
  const Layout L = layout_of(*grid);
  if (f_bytes) *f_bytes = L.f_bytes;
  if (q_bytes) *q_bytes = L.q_bytes;
  if (scratch_bytes) *scratch_bytes = L.scratch_bytes;
  return LC_OK;
}

lc_status lc_init(const lc_grid* grid, const lc_params* params, const lc_buffers* bufs, void* stream,
                  lc_ctx** out) {
  clear_error();
  if (!out) return fail(LC_EINVAL, "out is NULL");
  *out = nullptr;
  lc_status st = check_grid(grid);
  if (st) return st;
  st = check_params(params);
  if (st) return st;
  if (!bufs) return fail(LC_EINVAL, "buffers is NULL");
  const void* ptrs[5] = {bufs->f[0], bufs->f[1], bufs->Q[0], bufs->Q[1], bufs->scratch};
  for (const void* p : ptrs) {
    if (!p) return fail(LC_EINVAL, "a buffer pointer is NULL");
    if (reinterpret_cast<uintptr_t>(p) & 255) return fail(LC_EINVAL, "buffers must be 256-byte aligned");
  }
  lc_ctx* c = new (std::nothrow) lc_ctx;
  if (!c) return fail(LC_ENOMEM, "context allocation failed");
  c->g = *grid;
  c->p = *params;
  c->b = *bufs;
  c->stream = static_cast<hipStream_t>(stream);
  c->L = layout_of(*grid);
  c->parity = 0;
  c->step = 0;
  c->loaded = false;
  c->variant = LC_VARIANT_AUTO;
  c->stencil = LC_STENCIL_COMPACT;
  c->coll = LC_COLL_BGK;
  for (double& r : c->mrt) r = 0.0;
  c->zchunk = 0;
  c->timing = false;
  *out = c;
  return LC_OK;
}

lc_status lc_set_params(lc_ctx* c, const lc_params* params) {
  clear_error();
  if (!c) return fail(LC_EINVAL, "ctx is NULL");
  lc_status st = check_params(params);
  if (st) return st;
  c->p = *params;
  return LC_OK;
}

lc_status lc_set_variant(lc_ctx* c, int32_t variant) {
  clear_error();
  if (!c) return fail(LC_EINVAL, "ctx is NULL");
  if (variant == LC_VARIANT_AUTO || variant == LC_VARIANT_SPLIT) {
    c->variant = variant;
    return LC_OK;
  }
  if (variant == LC_VARIANT_STAGED) {
    if (c->g.precision == LC_MIXED) return fail(LC_EUNSUPPORTED, "the staged variant has no mixed-precision form");
    if (c->g.precision == LC_FP32_SR)
      return fail(LC_EUNSUPPORTED, "the staged variant has no stochastic-rounding form");
    c->variant = LC_VARIANT_STAGED;
    return LC_OK;
  }
  if (variant == LC_VARIANT_FUSED) {
    c->variant = LC_VARIANT_FUSED;
    return LC_OK;
  }
  return fail(LC_EINVAL, "unknown variant %d", variant);
}

lc_status lc_set_collision(lc_ctx* c, int32_t kind, const double* rates, int32_t nrates) {
  clear_error();
  if (!c) return fail(LC_EINVAL, "ctx is NULL");
  if (kind == LC_COLL_BGK) {
    c->coll = LC_COLL_BGK;
    return LC_OK;
  }
  if (kind != LC_COLL_MRT) return fail(LC_EINVAL, "unknown collision %d", kind);
  const int ng = c->g.lattice == LC_D2Q9 ? Ghosts<0>::ngroups : Ghosts<1>::ngroups;
  if (!rates) return fail(LC_EINVAL, "rates is NULL");
  if (nrates != ng) return fail(LC_EINVAL, "this lattice takes %d MRT rates (got %d)", ng, nrates);
  for (int g = 0; g < ng; g++)
    if (!(rates[g] > 0.0 && rates[g] < 2.0)) return fail(LC_EINVAL, "MRT rate %d = %g outside (0, 2)", g, rates[g]);
  for (int g = 0; g < 5; g++) c->mrt[g] = g < ng ? rates[g] : 0.0;
  c->coll = LC_COLL_MRT;
  return LC_OK;
}

lc_status lc_set_stencil(lc_ctx* c, int32_t stencil) {
  clear_error();
  if (!c) return fail(LC_EINVAL, "ctx is NULL");
  if (stencil == LC_STENCIL_COMPACT) {
    c->stencil = stencil;
    return LC_OK;
  }
  if (stencil != LC_STENCIL_ISOTROPIC) return fail(LC_EINVAL, "unknown stencil %d", stencil);
  if (c->g.precision != LC_FP64 && c->g.precision != LC_FP32_DEV)
    return fail(LC_EUNSUPPORTED, "the isotropic stencils are provided in LC_FP64 and LC_FP32_DEV");
  c->stencil = stencil;
  return LC_OK;
}

lc_status lc_set_chunk(lc_ctx* c, int32_t planes) {
  clear_error();
  if (!c) return fail(LC_EINVAL, "ctx is NULL");
  if (planes < 0) return fail(LC_EINVAL, "planes must be >= 0");
  c->zchunk = planes;
  return LC_OK;
}

lc_status lc_load_state(lc_ctx* c, const double* f_dev, const double* q_dev) {
  clear_error();
  if (!c) return fail(LC_EINVAL, "ctx is NULL");
  if (!q_dev) return fail(LC_EINVAL, "Q_dev is NULL");
  c->parity = 0;
  c->step = 0;
  lc_status st = LC_DISPATCH(c, do_load, f_dev, q_dev);
  if (st == LC_OK) c->loaded = true;
  return st;
}

lc_status lc_step(lc_ctx* c, int64_t n) {
  clear_error();
  if (!c) return fail(LC_EINVAL, "ctx is NULL");
  if (n < 0) return fail(LC_EINVAL, "n must be >= 0");
  if (!c->loaded) return fail(LC_ESTATE, "lc_step before lc_load_state");
  if (n == 0) return LC_OK;
  return LC_DISPATCH(c, run_steps, n);
}

lc_status lc_observe(lc_ctx* c, uint32_t mask, int32_t half_axis, lc_observables* out) {
  clear_error();
  if (!c || !out) return fail(LC_EINVAL, "NULL argument");
  if (!c->loaded) return fail(LC_ESTATE, "lc_observe before lc_load_state");
  if (half_axis < 0 || half_axis > 2) return fail(LC_EINVAL, "half_axis must be 0, 1 or 2");
  double h[OBS_W];
  lc_status st = LC_DISPATCH(c, do_observe, mask, half_axis, h);
  if (st) return st;
  fill_observables(h, mask, half_axis, c->step, out);
  if (out->nonfinite) return fail(LC_ENONFINITE, "state holds NaN or Inf at step %lld", (long long)c->step);
  return LC_OK;
}

lc_status lc_export(lc_ctx* c, int32_t field, double* dst) {
  clear_error();
  if (!c || !dst) return fail(LC_EINVAL, "NULL argument");
  if (!c->loaded) return fail(LC_ESTATE, "lc_export before lc_load_state");
  if (field < LC_FIELD_F || field > LC_FIELD_S) return fail(LC_EINVAL, "unknown field %d", field);
  return LC_DISPATCH(c, do_export, field, dst);
}

}  // extern "C"

namespace lc {

static VjpFields vjp_fields(lc_ctx* c) {
  const int64_t N = c->L.N;
  double* base = reinterpret_cast<double*>(static_cast<char*>(c->b.scratch) + c->L.off_vjp);
  VjpFields v;
  double* p = base;
  auto take = [&](int comps) {
    double* r = p;
    p += size_t(comps) * N;
    return r;
  };
  v.tau = take(4);
  v.rho = take(1);
  v.u = take(2);
  v.F = take(2);
  v.qp = take(5);
  v.r = take(5);
  v.fbar = take(9);
  v.qpb = take(5);
  v.lpb = take(5);
  v.dqpb = take(10);
  v.ub = take(2);
  v.gb = take(4);
  v.rhob = take(1);
  v.fb = take(2);
  v.qb = take(5);
  v.hb = take(5);
  v.dqb = take(10);
  v.lb = take(5);
  v.nblocks = c->L.nblocks;
  // the partials follow at the next 256-byte boundary, as laid out
  v.part = reinterpret_cast<double*>((reinterpret_cast<uintptr_t>(base + size_t(VJP_COMPS) * N) + 255) &
                                     ~uintptr_t(255));
  return v;
}

// The reverse kernels of one step, given the forward quantities of that
// step in v (rho, u, F, predictor); parameter partials accumulate.  With
// fold, adj_q is assembled inside vjp_r1 from the previous reverse step's
// gathers; with finish, the gathers are applied to adj_q at the end (the
// last step of a call).
static void vjp_reverse(lc_ctx* c, const VjpFields& v, const double* q_n, double* adj_f, double* adj_q, bool fold,
                        bool finish) {
  const GridDims gd{c->g.nx, c->g.ny, 1, c->L.N};
  const Coef<double> k = make_coef<double>(c->p);
  const dim3 grid = site_grid(c->g), block = site_block();
  // two threads per site (two halves of each block along z), same tiles
  static_assert(REV_TX == SITE_TX && REV_TY == SITE_TY, "reverse tiles are the site tiles");
  const dim3 block2(REV_TX, REV_TY, 2);
  hipLaunchKernelGGL(vjp_r1, grid, block2, 0, c->stream, adj_f, adj_q, fold ? 1 : 0, v, gd, k);
  hipLaunchKernelGGL(vjp_r2, grid, block2, 0, c->stream, q_n, adj_q, v, gd, k);
  hipLaunchKernelGGL(vjp_r34, grid, block2, 0, c->stream, adj_f, q_n, v, gd, k);
  if (finish) hipLaunchKernelGGL(vjp_r5, grid, block, 0, c->stream, adj_q, v, gd);
}

static void vjp_begin(lc_ctx* c, const VjpFields& v) {
  hipLaunchKernelGGL(vjp_zero, dim3(8), dim3(256), 0, c->stream, v.part, 3 * v.nblocks * 3);
}

static void vjp_end(lc_ctx* c, const VjpFields& v, double* dparams) {
  hipLaunchKernelGGL(vjp_params, dim3(1), dim3(256), 0, c->stream, v.part, v.nblocks, dparams);
}

// One reverse step from a logical state: recompute the forward quantities,
// then reverse.
static void vjp_launch(lc_ctx* c, const double* f_n, const double* q_n, double* adj_f, double* adj_q,
                       double* dparams) {
  const GridDims gd{c->g.nx, c->g.ny, 1, c->L.N};
  const Coef<double> k = make_coef<double>(c->p);
  VjpFields v = vjp_fields(c);
  const dim3 grid = site_grid(c->g), block = site_block();
  vjp_begin(c, v);
  hipLaunchKernelGGL((stage_tau<0, double>), grid, block, 0, c->stream, q_n, v.tau, gd, k);
  hipLaunchKernelGGL(vjp_fwd_moments, grid, block, 0, c->stream, f_n, 0, v.tau, v, gd);
  hipLaunchKernelGGL((stage_pred<0, double>), grid, block, 0, c->stream, q_n, v.u, v.qp, v.r, gd, k);
  vjp_reverse(c, v, q_n, adj_f, adj_q, false, true);
  vjp_end(c, v, dparams);
}

static lc_status vjp_check(lc_ctx* c) {
  if (c->g.lattice != LC_D2Q9 || c->g.precision != LC_FP64)
    return fail(LC_EUNSUPPORTED, "the reverse step is provided for D2Q9 in double precision");
  if (c->coll != LC_COLL_BGK) return fail(LC_EUNSUPPORTED, "the reverse step is provided for the BGK collision");
  if (c->stencil != LC_STENCIL_COMPACT)
    return fail(LC_EUNSUPPORTED, "the reverse step is provided for the compact stencils");
  return LC_OK;
}

}  // namespace lc

extern "C" {

lc_status lc_vjp_step(lc_ctx* c, const double* f_n, const double* q_n, double* adj_f, double* adj_q,
                      double* dparams) {
  clear_error();
  if (!c || !f_n || !q_n || !adj_f || !adj_q || !dparams) return fail(LC_EINVAL, "NULL argument");
  lc_status st = vjp_check(c);
  if (st) return st;
  vjp_launch(c, f_n, q_n, adj_f, adj_q, dparams);
  return hip_check(hipGetLastError(), "reverse step launch");
}

size_t lc_vjp_history_bytes(const lc_grid* grid, int32_t n) {
  if (!grid || n < 1 || check_grid(grid) != LC_OK) return 0;
  const size_t N = size_t(grid->nx) * grid->ny * grid->nz;
  const size_t q = size_t(lattice_q(grid->lattice));
  const size_t es = grid->precision == LC_FP64 ? 8 : 4;
  // per step: populations, Q, and the recorded u, rho, F and predictor
  return size_t(n + 1) * (q + 5 + 10) * N * es;
}

}  // extern "C"

namespace lc {
// History of one segment: slot j holds f (9N, pull form), Q (5N), u (2N),
// rho and F (3N) and Q^P (5N) of step j.
struct VjpHist {
  double* h;
  int64_t N;
  double* slot(int j) const { return h + size_t(j) * 24 * N; }
  double* f(int j) const { return slot(j); }
  double* q(int j) const { return slot(j) + 9 * size_t(N); }
  double* u(int j) const { return slot(j) + 14 * size_t(N); }
  double* r(int j) const { return slot(j) + 16 * size_t(N); }
  double* p(int j) const { return slot(j) + 19 * size_t(N); }
};

// Replay n steps from a checkpoint on stream st, recording every step.
static void vjp_replay(lc_ctx* c, hipStream_t st, const double* f_ck, const double* q_ck, int n, const VjpHist& H) {
  const GridDims gd{c->g.nx, c->g.ny, 1, c->L.N};
  hipLaunchKernelGGL((load_state<0, double, false>), site_grid(c->g), site_block(), 0, st, f_ck, q_ck, H.f(0),
                     H.q(0), gd);
  for (int j = 0; j < n; j++)
    step_split_ptrs<0, double, false>(c, st, false, H.f(j), H.q(j), H.f(j + 1), H.q(j + 1), H.u(j), H.r(j), H.p(j));
}

// The reverse steps n-1 .. 0 of a recorded segment on the context stream.
static void vjp_walk(lc_ctx* c, VjpFields& v, int n, const VjpHist& H, double* adj_f, double* adj_q) {
  for (int j = n - 1; j >= 0; j--) {
    v.u = H.u(j);
    v.rho = H.r(j);
    v.F = H.r(j) + H.N;
    v.qp = H.p(j);
    vjp_reverse(c, v, H.q(j), adj_f, adj_q, j < n - 1, j == 0);
  }
}

static size_t up256(size_t v) { return (v + 255) & ~size_t(255); }
}  // namespace lc

extern "C" {

lc_status lc_vjp_segment(lc_ctx* c, const double* f_ck, const double* q_ck, int32_t n, void* hist, double* adj_f,
                         double* adj_q, double* dparams) {
  clear_error();
  if (!c || !f_ck || !q_ck || !hist || !adj_f || !adj_q || !dparams) return fail(LC_EINVAL, "NULL argument");
  if (n < 1) return fail(LC_EINVAL, "n must be >= 1");
  lc_status st = vjp_check(c);
  if (st) return st;
  if (reinterpret_cast<uintptr_t>(hist) & 255) return fail(LC_EINVAL, "history must be 256-byte aligned");
  const VjpHist H{static_cast<double*>(hist), c->L.N};
  vjp_replay(c, c->stream, f_ck, q_ck, n, H);
  VjpFields v = vjp_fields(c);
  vjp_begin(c, v);
  vjp_walk(c, v, n, H, adj_f, adj_q);
  vjp_end(c, v, dparams);
  // the context's own state is untouched
  return hip_check(hipGetLastError(), "reverse segment launch");
}

size_t lc_vjp_backward_bytes(const lc_grid* grid, int32_t n) {
  const size_t h = lc_vjp_history_bytes(grid, n);
  return h ? 2 * up256(h) : 0;
}

lc_status lc_vjp_backward(lc_ctx* c, int32_t nseg, const double* const* f_cks, const double* const* q_cks,
                          const int32_t* ns, void* hist, double* adj_f, double* adj_q, double* dparams) {
  clear_error();
  if (!c || !f_cks || !q_cks || !ns || !hist || !adj_f || !adj_q || !dparams) return fail(LC_EINVAL, "NULL argument");
  if (nseg < 1) return fail(LC_EINVAL, "nseg must be >= 1");
  lc_status st = vjp_check(c);
  if (st) return st;
  if (reinterpret_cast<uintptr_t>(hist) & 255) return fail(LC_EINVAL, "history must be 256-byte aligned");
  int32_t nmax = 0;
  for (int32_t k = 0; k < nseg; k++) {
    if (!f_cks[k] || !q_cks[k]) return fail(LC_EINVAL, "checkpoint %d is NULL", k);
    if (ns[k] < 1) return fail(LC_EINVAL, "segment %d has %d steps", k, ns[k]);
    nmax = ns[k] > nmax ? ns[k] : nmax;
  }
  if (!c->aux) {
    // events first, then the stream: the context keeps them only once all
    // exist, so a failed call leaves nothing half made
    hipEvent_t ev[5] = {};
    hipStream_t aux = nullptr;
    bool ok = true;
    for (hipEvent_t& e : ev) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&aux, hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
      for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
      if (aux) (void)hipStreamDestroy(aux);
      return fail(LC_EDEVICE, "cannot create the replay stream and its events");
    }
    for (int i = 0; i < 5; i++) c->vev[i] = ev[i];
    c->aux = aux;
  }
  const size_t half = up256(lc_vjp_history_bytes(&c->g, nmax));
  const VjpHist H[2] = {{static_cast<double*>(hist), c->L.N},
                        {reinterpret_cast<double*>(static_cast<char*>(hist) + half), c->L.N}};
  // Segment k is replayed into half k & 1 on the replay stream while the
  // context stream walks segment k + 1 back: events vev[0..1] mark a replay
  // done, vev[2..3] a walk done (per half), vev[4] the caller's prior work.
  hipEvent_t* rep = c->vev;
  hipEvent_t* walk = c->vev + 2;
  hipEvent_t entry = c->vev[4];
  auto chk = [](hipError_t e) { return e == hipSuccess; };
  bool ok = chk(hipEventRecord(entry, c->stream)) && chk(hipStreamWaitEvent(c->aux, entry, 0));
  VjpFields v = vjp_fields(c);
  vjp_begin(c, v);
  for (int32_t k = nseg - 1; ok && k >= -1; k--) {
    if (k >= 0) {
      // replay segment k once the walk that last used its half is done
      if (k + 2 < nseg) ok = ok && chk(hipStreamWaitEvent(c->aux, walk[k & 1], 0));
      vjp_replay(c, c->aux, f_cks[k], q_cks[k], ns[k], H[k & 1]);
      ok = ok && chk(hipEventRecord(rep[k & 1], c->aux));
    }
    const int32_t w = k + 1;  // the segment walked in this pass
    if (w < nseg) {
      ok = ok && chk(hipStreamWaitEvent(c->stream, rep[w & 1], 0));
      vjp_walk(c, v, ns[w], H[w & 1], adj_f, adj_q);
      ok = ok && chk(hipEventRecord(walk[w & 1], c->stream));
    }
  }
  vjp_end(c, v, dparams);
  if (!ok) return fail(LC_EDEVICE, "stream ordering of the reverse sweep failed");
  return hip_check(hipGetLastError(), "reverse sweep launch");
}

lc_status lc_sync(lc_ctx* c) {
  clear_error();
  if (!c) return fail(LC_EINVAL, "ctx is NULL");
  return hip_check(hipStreamSynchronize(c->stream), "sync");
}

int64_t lc_step_count(const lc_ctx* c) { return c ? c->step : -1; }

lc_status lc_set_timing(lc_ctx* c, int32_t enable) {
  clear_error();
  if (!c) return fail(LC_EINVAL, "ctx is NULL");
  c->timing = enable != 0;
  return LC_OK;
}

lc_status lc_get_timing(lc_ctx* c, double* ms, int64_t* launches) {
  clear_error();
  if (!c || !ms || !launches) return fail(LC_EINVAL, "NULL argument");
  ms[0] = ms[1] = 0.0;
  launches[0] = launches[1] = 0;
  lc_status st = hip_check(hipStreamSynchronize(c->stream), "timing sync");
  if (st) return st;
  st = ctx_fold(c);
  if (st) return st;
  for (int k = 0; k < 2; k++) {
    ms[k] = c->acc_ms[k];
    launches[k] = c->acc_n[k];
    c->acc_ms[k] = 0.0;
    c->acc_n[k] = 0;
  }
  return LC_OK;
}

lc_status lc_free(lc_ctx* c) {
  clear_error();
  if (!c) return LC_OK;
  for (const auto& t : c->ev) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->vev)
    if (e) (void)hipEventDestroy(e);
  if (c->aux) (void)hipStreamDestroy(c->aux);
  delete c;
  return LC_OK;
}

}  // extern "C"

// ===========================================================================
// Steps without allocation: the velocity between the two sweeps lives in a
// fixed device array of the library instead of a caller-provided scratch.
// ===========================================================================
namespace lc {

// One copy per GPU, held from the library's load until the process ends.
static __device__ __align__(256) unsigned char scratch[LC_STATIC_SCRATCH_BYTES];

constexpr int STATIC_MAX_DEVICES = 64;
static std::mutex g_static_mu;
static void* g_static_ptr[STATIC_MAX_DEVICES];

// Device address of the current GPU's copy of `scratch`, looked up once per
// device with that device current.  The array's name is a host-side
// stand-in and never reaches a kernel; only this address does.
static lc_status static_scratch_ptr(void** out) {
  int dev = -1;
  lc_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (st) return st;
  if (dev < 0 || dev >= STATIC_MAX_DEVICES) return fail(LC_EDEVICE, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    st = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (st) return st;
    if (!p) return fail(LC_EDEVICE, "static scratch has no device address");
    g_static_ptr[dev] = p;
  }
  *out = g_static_ptr[dev];
  return LC_OK;
}

// Bytes of the velocity the split sweeps hand from the first to the second.
static size_t static_velocity_bytes(const lc_grid& g) {
  const size_t N = size_t(g.nx) * g.ny * g.nz;
  const size_t dim = g.lattice == LC_D2Q9 ? 2 : 3;
  return dim * N * (g.precision == LC_FP64 || g.precision == LC_MIXED ? 8 : 4);
}

template <int LAT, typename S, bool DEV, typename QT = S>
static lc_status run_static(lc_ctx* c, void* u_dev, int64_t n) {
  QT* u = static_cast<QT*>(u_dev);
  for (int64_t it = 0; it < n; it++) {
    step_split_ptrs<LAT, S, DEV, QT>(c, c->stream, false, static_cast<const S*>(c->b.f[c->parity]),
                                     static_cast<const QT*>(c->b.Q[c->parity]),
                                     static_cast<S*>(c->b.f[c->parity ^ 1]), static_cast<QT*>(c->b.Q[c->parity ^ 1]),
                                     u, nullptr, nullptr);
    c->parity ^= 1;
  }
  return hip_check(hipGetLastError(), "step launch");
}

}  // namespace lc

extern "C" {

lc_status lc_step_static(const lc_grid* grid, const lc_params* params, void* const* f, void* const* Q,
                         int32_t parity, int64_t n, void* stream) {
  clear_error();
  lc_status st = check_grid(grid);
  if (st) return st;
  st = check_params(params);
  if (st) return st;
  if (!f || !Q) return fail(LC_EINVAL, "buffer array is NULL");
  if (parity != 0 && parity != 1) return fail(LC_EINVAL, "parity must be 0 or 1");
  if (n < 0) return fail(LC_EINVAL, "n must be >= 0");
  const void* ptrs[4] = {f[0], f[1], Q[0], Q[1]};
  for (const void* p : ptrs) {
    if (!p) return fail(LC_EINVAL, "a buffer pointer is NULL");
    if (reinterpret_cast<uintptr_t>(p) & 255) return fail(LC_EINVAL, "buffers must be 256-byte aligned");
  }
  if (grid->precision == LC_FP32_SR)
    return fail(LC_EUNSUPPORTED, "the stochastic-rounding form needs the step counter of a context");
  const size_t need = static_velocity_bytes(*grid);
  if (need > LC_STATIC_SCRATCH_BYTES)
    return fail(LC_ENOMEM, "grid needs %zu bytes of velocity scratch; the static buffer holds %zu", need,
                size_t(LC_STATIC_SCRATCH_BYTES));
  void* u = nullptr;
  st = static_scratch_ptr(&u);
  if (st) return st;
  if (n == 0) return LC_OK;
  // a context on the stack (no allocation): the split sweeps with BGK and
  // the default chunks, over the caller's buffers
  lc_ctx c;
  c.g = *grid;
  c.p = *params;
  c.b.f[0] = f[0];
  c.b.f[1] = f[1];
  c.b.Q[0] = Q[0];
  c.b.Q[1] = Q[1];
  c.b.scratch = nullptr;
  c.stream = static_cast<hipStream_t>(stream);
  c.L = layout_of(*grid);
  c.parity = parity;
  c.step = 0;
  c.loaded = true;
  c.variant = LC_VARIANT_SPLIT;
  c.zchunk = 0;
  c.coll = LC_COLL_BGK;
  for (double& r : c.mrt) r = 0.0;
  c.timing = false;
  return LC_DISPATCH((&c), run_static, u, n);
}

}  // extern "C"

// ===========================================================================
// Batched form.
// ===========================================================================
namespace lc {

struct BatchLayout {
  std::vector<size_t> f_off, q_off, u_off;  // byte offsets into the arenas / scratch u region
  size_t f_bytes = 0, q_bytes = 0;
  size_t off_desc = 0, off_map[BATCH_NV] = {}, off_u = 0, off_view = 0, off_res = 0;
  size_t off_step = 0;  // step count of the next run of launches (stochastic rounding keys)
  size_t scratch_bytes = 0;
  int tiles[BATCH_NV] = {};
  std::vector<int> tile0[BATCH_NV], tiles_x[BATCH_NV];
};

static lc_status batch_layout_of(int32_t n, const lc_grid* grids, BatchLayout& B) {
  if (n < 1 || !grids) return fail(LC_EINVAL, "need at least one grid");
  for (int k = 0; k < n; k++) {
    lc_status st = check_grid(&grids[k]);
    if (st) return st;
    if (grids[k].lattice != LC_D2Q9) return fail(LC_EUNSUPPORTED, "the batched form runs D2Q9 grids");
    if (grids[k].precision != grids[0].precision) return fail(LC_EINVAL, "all grids must share one precision");
  }
  auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
  // element sizes of f and of Q and u (double Q and u in the mixed form)
  const size_t es = grids[0].precision == LC_FP64 ? 8 : 4;
  const size_t es_q = grids[0].precision == LC_FP64 || grids[0].precision == LC_MIXED ? 8 : 4;
  B.f_off.resize(n);
  B.q_off.resize(n);
  B.u_off.resize(n);
  size_t fo = 0, qo = 0, uo = 0, view = 0;
  for (int v = 0; v < BATCH_NV; v++) {
    B.tile0[v].resize(n);
    B.tiles_x[v].resize(n);
    B.tiles[v] = 0;
  }
  for (int k = 0; k < n; k++) {
    const size_t N = size_t(grids[k].nx) * grids[k].ny;
    B.f_off[k] = fo;
    fo = up(fo + 9 * N * es);
    B.q_off[k] = qo;
    qo = up(qo + 5 * N * es_q);
    B.u_off[k] = uo;
    uo = up(uo + 2 * N * es_q);
    view = std::max(view, layout_of(grids[k]).scratch_bytes);
    for (int v = 0; v < BATCH_NV; v++) {
      const int tx = batch_tx(v), ty = batch_ty(v);
      const int ntx = (grids[k].nx + tx - 1) / tx, nty = (grids[k].ny + ty - 1) / ty;
      B.tile0[v][k] = B.tiles[v];
      B.tiles_x[v][k] = ntx;
      B.tiles[v] += ntx * nty;
    }
  }
  B.f_bytes = fo;
  B.q_bytes = qo;
  size_t off = 0;
  B.off_desc = off;
  off = up(off + size_t(n) * std::max(sizeof(BatchDesc<double>), sizeof(BatchDesc<float, double>)));
  for (int v = 0; v < BATCH_NV; v++) {
    B.off_map[v] = off;
    off = up(off + size_t(B.tiles[v]) * sizeof(int));
  }
  B.off_res = off;
  off = up(off + size_t(n) * OBS_W * sizeof(double));
  B.off_step = off;
  off = up(off + sizeof(uint32_t));
  B.off_u = off;
  off = up(off + uo);
  B.off_view = off;
  off = up(off + view);
  B.scratch_bytes = off;
  return LC_OK;
}

}  // namespace lc

struct lc_batch {
  int n;
  std::vector<lc_grid> grids;
  std::vector<lc_params> params;
  lc_buffers arena;
  hipStream_t stream;
  hipStream_t cap;  // private stream used only to capture graphs
  BatchLayout B;
  std::vector<lc_ctx> views;  // single-grid contexts over the arenas
  std::vector<char> host_desc;
  std::vector<int> host_map[BATCH_NV];
  int vt[2];  // tile shape of each sweep (0: LB, 1: Q)
  int coll = LC_COLL_BGK;  // LC_COLL_*, for every grid
  double mrt[5] = {};      // MRT rates of the ghost groups
  int stencil = LC_STENCIL_COMPACT;  // LC_STENCIL_*, for every grid
  int parity;
  int64_t step;
  bool loaded;
  static constexpr int G = 64;  // steps per captured graph (even)
  hipGraphExec_t exec[2];
  hipGraph_t graph[2];
};

namespace lc {

template <typename S, typename QT>
static void batch_fill_desc(lc_batch* b) {
  using D = BatchDesc<S, QT>;
  b->host_desc.assign(size_t(b->n) * sizeof(D), 0);
  D* d = reinterpret_cast<D*>(b->host_desc.data());
  for (int k = 0; k < b->n; k++) {
    d[k].nx = b->grids[k].nx;
    d[k].ny = b->grids[k].ny;
    d[k].N = int64_t(b->grids[k].nx) * b->grids[k].ny;
    d[k].f_off = int64_t(b->B.f_off[k] / sizeof(S));
    d[k].q_off = int64_t(b->B.q_off[k] / sizeof(QT));
    d[k].u_off = int64_t(b->B.u_off[k] / sizeof(QT));
    for (int w = 0; w < 2; w++) {
      d[k].tile0[w] = b->B.tile0[b->vt[w]][k];
      d[k].tiles_x[w] = b->B.tiles_x[b->vt[w]][k];
    }
    d[k].c = make_coef<S>(b->params[k]);
    d[k].cq = make_coef<QT>(b->params[k]);
    if (b->coll == LC_COLL_MRT)  // each group's rate minus this grid's 1/tau
      for (int g = 0; g < 5; g++) d[k].c.mrt[g] = S(b->mrt[g] - 1.0 / b->params[k].tau);
  }
}

// Upload the descriptor table for the current variant (asynchronous; the
// host copy lives in the batch object).
static lc_status batch_upload(lc_batch* b) {
  if (b->grids[0].precision == LC_FP64)
    batch_fill_desc<double, double>(b);
  else if (b->grids[0].precision == LC_MIXED)
    batch_fill_desc<float, double>(b);
  else
    batch_fill_desc<float, float>(b);
  char* scr = static_cast<char*>(b->arena.scratch);
  return hip_check(hipMemcpyAsync(scr + b->B.off_desc, b->host_desc.data(), b->host_desc.size(),
                                  hipMemcpyHostToDevice, b->stream),
                   "batch descriptor upload");
}

template <typename S, bool DEV, typename QT, bool MRT, int ST, int V>
static void batch_launch_lb(lc_batch* b, hipStream_t st, int parity) {
  constexpr int TX = batch_tx(V), TY = batch_ty(V);
  char* scr = static_cast<char*>(b->arena.scratch);
  const BatchDesc<S, QT>* desc = reinterpret_cast<const BatchDesc<S, QT>*>(scr + b->B.off_desc);
  const int* map = reinterpret_cast<const int*>(scr + b->B.off_map[V]);
  QT* u = reinterpret_cast<QT*>(scr + b->B.off_u);
  const S* f0 = static_cast<const S*>(b->arena.f[parity]);
  S* f1 = static_cast<S*>(b->arena.f[parity ^ 1]);
  const QT* q0 = static_cast<const QT*>(b->arena.Q[parity]);
  hipLaunchKernelGGL((batch_lb<0, S, DEV, TX, TY, QT, MRT, ST>), dim3(unsigned(b->B.tiles[V])), dim3(TX, TY), 0,
                     st, desc, map, q0, f0, f1, u);
}

template <typename S, typename QT, bool SR, int ST, int V>
static void batch_launch_q(lc_batch* b, hipStream_t st, int parity, int step_off) {
  constexpr int TX = batch_tx(V), TY = batch_ty(V);
  char* scr = static_cast<char*>(b->arena.scratch);
  const BatchDesc<S, QT>* desc = reinterpret_cast<const BatchDesc<S, QT>*>(scr + b->B.off_desc);
  const int* map = reinterpret_cast<const int*>(scr + b->B.off_map[V]);
  const QT* u = reinterpret_cast<const QT*>(scr + b->B.off_u);
  const uint32_t* step_base = reinterpret_cast<const uint32_t*>(scr + b->B.off_step);
  const QT* q0 = static_cast<const QT*>(b->arena.Q[parity]);
  QT* q1 = static_cast<QT*>(b->arena.Q[parity ^ 1]);
  hipLaunchKernelGGL((batch_q<0, S, QT, TX, TY, SR, ST>), dim3(unsigned(b->B.tiles[V])), dim3(TX, TY), 0, st, desc,
                     map, q0, u, q1, step_base, step_off);
}

template <typename S, bool DEV, typename QT, bool SR, bool MRT, int ST>
static void batch_launch(lc_batch* b, hipStream_t st, int parity, int step_off) {
  static_assert(BATCH_NV == 7, "one launch branch per tile shape");
  switch (b->vt[0]) {
    case 0: batch_launch_lb<S, DEV, QT, MRT, ST, 0>(b, st, parity); break;
    case 1: batch_launch_lb<S, DEV, QT, MRT, ST, 1>(b, st, parity); break;
    case 2: batch_launch_lb<S, DEV, QT, MRT, ST, 2>(b, st, parity); break;
    case 3: batch_launch_lb<S, DEV, QT, MRT, ST, 3>(b, st, parity); break;
    case 4: batch_launch_lb<S, DEV, QT, MRT, ST, 4>(b, st, parity); break;
    case 5: batch_launch_lb<S, DEV, QT, MRT, ST, 5>(b, st, parity); break;
    default: batch_launch_lb<S, DEV, QT, MRT, ST, 6>(b, st, parity); break;
  }
  switch (b->vt[1]) {
    case 0: batch_launch_q<S, QT, SR, ST, 0>(b, st, parity, step_off); break;
    case 1: batch_launch_q<S, QT, SR, ST, 1>(b, st, parity, step_off); break;
    case 2: batch_launch_q<S, QT, SR, ST, 2>(b, st, parity, step_off); break;
    case 3: batch_launch_q<S, QT, SR, ST, 3>(b, st, parity, step_off); break;
    case 4: batch_launch_q<S, QT, SR, ST, 4>(b, st, parity, step_off); break;
    case 5: batch_launch_q<S, QT, SR, ST, 5>(b, st, parity, step_off); break;
    default: batch_launch_q<S, QT, SR, ST, 6>(b, st, parity, step_off); break;
  }
}

// One step of every grid; step_off: the step's offset from the step count
// last written to the batch's step slot (stochastic rounding only).
template <bool MRT>
static void batch_launch_step_coll(lc_batch* b, hipStream_t st, int parity, int step_off) {
  // the isotropic stencils: LC_FP64 and LC_FP32_DEV (lc_batch_set_stencil)
  const bool iso = b->stencil == LC_STENCIL_ISOTROPIC;
  if (b->grids[0].precision == LC_FP64) {
    if (iso)
      batch_launch<double, false, double, false, MRT, STENCIL_ISO>(b, st, parity, step_off);
    else
      batch_launch<double, false, double, false, MRT, STENCIL_COMPACT>(b, st, parity, step_off);
  } else if (b->grids[0].precision == LC_MIXED) {
    batch_launch<float, true, double, false, MRT, STENCIL_COMPACT>(b, st, parity, step_off);
  } else if (b->grids[0].precision == LC_FP32_SR) {
    batch_launch<float, true, float, true, MRT, STENCIL_COMPACT>(b, st, parity, step_off);
  } else {
    if (iso)
      batch_launch<float, true, float, false, MRT, STENCIL_ISO>(b, st, parity, step_off);
    else
      batch_launch<float, true, float, false, MRT, STENCIL_COMPACT>(b, st, parity, step_off);
  }
}

static void batch_launch_step(lc_batch* b, hipStream_t st, int parity, int step_off) {
  if (b->coll == LC_COLL_MRT)
    batch_launch_step_coll<true>(b, st, parity, step_off);
  else
    batch_launch_step_coll<false>(b, st, parity, step_off);
}

// Write the step count of the next run of launches to the batch's step slot
// (read by the stochastic-rounding Q sweep; on the stream, never captured).
static lc_status batch_set_step(lc_batch* b) {
  if (b->grids[0].precision != LC_FP32_SR) return LC_OK;
  void* p = static_cast<char*>(b->arena.scratch) + b->B.off_step;
  return hip_check(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(p), int(uint32_t(b->step)), 1, b->stream),
                   "batch step count");
}

static void batch_drop_graphs(lc_batch* b) {
  for (int p = 0; p < 2; p++) {
    if (b->exec[p]) (void)hipGraphExecDestroy(b->exec[p]);
    if (b->graph[p]) (void)hipGraphDestroy(b->graph[p]);
    b->exec[p] = nullptr;
    b->graph[p] = nullptr;
  }
}

// Capture G steps starting from `parity` on the private stream.
static lc_status batch_build_graph(lc_batch* b, int parity) {
  lc_status st = hip_check(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal), "graph capture begin");
  if (st) return st;
  int p = parity;
  for (int i = 0; i < lc_batch::G; i++) {
    batch_launch_step(b, b->cap, p, i);
    p ^= 1;
  }
  hipGraph_t g = nullptr;
  st = hip_check(hipStreamEndCapture(b->cap, &g), "graph capture end");
  if (st) return st;
  hipGraphExec_t e = nullptr;
  st = hip_check(hipGraphInstantiate(&e, g, nullptr, nullptr, 0), "graph instantiate");
  if (st) {
    (void)hipGraphDestroy(g);
    return st;
  }
  b->graph[parity] = g;
  b->exec[parity] = e;
  return LC_OK;
}

static void batch_sync_views(lc_batch* b) {
  for (auto& v : b->views) {
    v.parity = b->parity;
    v.step = b->step;
  }
}

}  // namespace lc

extern "C" {

lc_status lc_batch_layout(int32_t ngrids, const lc_grid* grids, size_t* f_bytes, size_t* q_bytes,
                          size_t* scratch_bytes, size_t* f_offsets, size_t* q_offsets) {
  clear_error();
  BatchLayout B;
  lc_status st = batch_layout_of(ngrids, grids, B);
  if (st) return st;
  if (f_bytes) *f_bytes = B.f_bytes;
  if (q_bytes) *q_bytes = B.q_bytes;
  if (scratch_bytes) *scratch_bytes = B.scratch_bytes;
  for (int k = 0; k < ngrids; k++) {
    if (f_offsets) f_offsets[k] = B.f_off[k];
    if (q_offsets) q_offsets[k] = B.q_off[k];
  }
  return LC_OK;
}

lc_status lc_batch_init(int32_t ngrids, const lc_grid* grids, const lc_params* params, const lc_buffers* arena,
                        void* stream, lc_batch** out) {
  clear_error();
  if (!out) return fail(LC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!params || !arena) return fail(LC_EINVAL, "NULL argument");
  BatchLayout B;
  lc_status st = batch_layout_of(ngrids, grids, B);
  if (st) return st;
  for (int k = 0; k < ngrids; k++) {
    st = check_params(&params[k]);
    if (st) return st;
  }
  const void* ptrs[5] = {arena->f[0], arena->f[1], arena->Q[0], arena->Q[1], arena->scratch};
  for (const void* p : ptrs) {
    if (!p) return fail(LC_EINVAL, "an arena pointer is NULL");
    if (reinterpret_cast<uintptr_t>(p) & 255) return fail(LC_EINVAL, "arenas must be 256-byte aligned");
  }
  lc_batch* b = new (std::nothrow) lc_batch;
  if (!b) return fail(LC_ENOMEM, "batch allocation failed");
  b->n = ngrids;
  b->grids.assign(grids, grids + ngrids);
  b->params.assign(params, params + ngrids);
  b->arena = *arena;
  b->stream = static_cast<hipStream_t>(stream);
  b->B = B;
  b->vt[0] = b->vt[1] = 0;
  b->parity = 0;
  b->step = 0;
  b->loaded = false;
  for (int p = 0; p < 2; p++) {
    b->exec[p] = nullptr;
    b->graph[p] = nullptr;
  }
  st = hip_check(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking), "capture stream");
  if (st) {
    delete b;
    return st;
  }
  char* scr = static_cast<char*>(arena->scratch);
  b->views.resize(ngrids);
  for (int k = 0; k < ngrids; k++) {
    lc_ctx& v = b->views[k];
    v.g = grids[k];
    v.p = params[k];
    v.b.f[0] = static_cast<char*>(arena->f[0]) + B.f_off[k];
    v.b.f[1] = static_cast<char*>(arena->f[1]) + B.f_off[k];
    v.b.Q[0] = static_cast<char*>(arena->Q[0]) + B.q_off[k];
    v.b.Q[1] = static_cast<char*>(arena->Q[1]) + B.q_off[k];
    v.b.scratch = scr + B.off_view;
    v.stream = b->stream;
    v.L = layout_of(grids[k]);
    v.parity = 0;
    v.step = 0;
    v.loaded = false;
    v.variant = LC_VARIANT_SPLIT;
    v.zchunk = 0;
    v.coll = LC_COLL_BGK;
    for (double& r : v.mrt) r = 0.0;
    v.timing = false;
  }
  // tile -> grid maps for every tile shape
  for (int vv = 0; vv < BATCH_NV; vv++) {
    b->host_map[vv].resize(B.tiles[vv]);
    for (int k = 0; k < ngrids; k++) {
      const int t0 = B.tile0[vv][k];
      const int t1 = k + 1 < ngrids ? B.tile0[vv][k + 1] : B.tiles[vv];
      for (int t = t0; t < t1; t++) b->host_map[vv][t] = k;
    }
    st = hip_check(hipMemcpyAsync(scr + B.off_map[vv], b->host_map[vv].data(), b->host_map[vv].size() * sizeof(int),
                                  hipMemcpyHostToDevice, b->stream),
                   "tile map upload");
    if (st) {
      (void)hipStreamDestroy(b->cap);
      delete b;
      return st;
    }
  }
  st = batch_upload(b);
  if (st) {
    (void)hipStreamDestroy(b->cap);
    delete b;
    return st;
  }
  // the host tables must stay valid until the uploads have run
  st = hip_check(hipStreamSynchronize(b->stream), "batch init sync");
  if (st) {
    (void)hipStreamDestroy(b->cap);
    delete b;
    return st;
  }
  *out = b;
  return LC_OK;
}

lc_status lc_batch_load_state(lc_batch* b, int32_t k, const double* f_dev, const double* q_dev) {
  clear_error();
  if (!b) return fail(LC_EINVAL, "batch is NULL");
  if (k < 0 || k >= b->n) return fail(LC_EINVAL, "grid index out of range");
  if (!q_dev) return fail(LC_EINVAL, "Q_dev is NULL");
  // every grid of the batch shares one parity and step counter
  if (b->parity != 0 || b->step != 0) {
    for (auto& v : b->views) v.loaded = false;
    b->loaded = false;
  }
  b->parity = 0;
  b->step = 0;
  lc_ctx* c = &b->views[k];
  c->parity = 0;
  c->step = 0;
  lc_status st = LC_DISPATCH(c, do_load, f_dev, q_dev);
  if (st) return st;
  c->loaded = true;
  bool all = true;
  for (auto& v : b->views) all = all && v.loaded;
  b->loaded = all;
  return LC_OK;
}

lc_status lc_batch_step(lc_batch* b, int64_t n) {
  clear_error();
  if (!b) return fail(LC_EINVAL, "batch is NULL");
  if (n < 0) return fail(LC_EINVAL, "n must be >= 0");
  if (!b->loaded) return fail(LC_ESTATE, "load every grid of the batch before stepping");
  while (n >= lc_batch::G) {
    if (!b->exec[b->parity]) {
      lc_status st = batch_build_graph(b, b->parity);
      if (st) return st;
    }
    lc_status st = batch_set_step(b);
    if (st) return st;
    st = hip_check(hipGraphLaunch(b->exec[b->parity], b->stream), "graph launch");
    if (st) return st;
    n -= lc_batch::G;
    b->step += lc_batch::G;
  }
  for (int64_t i = 0; i < n; i++) {
    lc_status st = batch_set_step(b);
    if (st) return st;
    batch_launch_step(b, b->stream, b->parity, 0);
    b->parity ^= 1;
    b->step++;
  }
  batch_sync_views(b);
  return hip_check(hipGetLastError(), "batch step launch");
}

lc_status lc_batch_set_tiles(lc_batch* b, int32_t v_lb, int32_t v_q) {
  clear_error();
  if (!b) return fail(LC_EINVAL, "batch is NULL");
  if (v_lb < 0 || v_lb >= BATCH_NV || v_q < 0 || v_q >= BATCH_NV) return fail(LC_EINVAL, "tile variant out of range");
  if (v_lb == b->vt[0] && v_q == b->vt[1]) return LC_OK;
  b->vt[0] = v_lb;
  b->vt[1] = v_q;
  batch_drop_graphs(b);
  lc_status st = batch_upload(b);
  if (st) return st;
  return hip_check(hipStreamSynchronize(b->stream), "descriptor upload sync");
}

lc_status lc_batch_set_tile(lc_batch* b, int32_t variant) { return lc_batch_set_tiles(b, variant, variant); }

lc_status lc_batch_set_stencil(lc_batch* b, int32_t stencil) {
  clear_error();
  if (!b) return fail(LC_EINVAL, "batch is NULL");
  if (stencil != LC_STENCIL_COMPACT && stencil != LC_STENCIL_ISOTROPIC)
    return fail(LC_EINVAL, "unknown stencil %d", stencil);
  if (stencil == LC_STENCIL_ISOTROPIC && b->grids[0].precision != LC_FP64 && b->grids[0].precision != LC_FP32_DEV)
    return fail(LC_EUNSUPPORTED, "the isotropic stencils are provided in LC_FP64 and LC_FP32_DEV");
  b->stencil = stencil;
  // exports and observables of the grids differentiate with the same stencils
  for (auto& v : b->views) v.stencil = stencil;
  batch_drop_graphs(b);
  return LC_OK;
}

lc_status lc_batch_set_collision(lc_batch* b, int32_t kind, const double* rates, int32_t nrates) {
  clear_error();
  if (!b) return fail(LC_EINVAL, "batch is NULL");
  double r[5] = {0, 0, 0, 0, 0};
  if (kind == LC_COLL_MRT) {
    const int ng = Ghosts<0>::ngroups;
    if (!rates) return fail(LC_EINVAL, "rates is NULL");
    if (nrates != ng) return fail(LC_EINVAL, "D2Q9 takes %d MRT rates (got %d)", ng, nrates);
    for (int g = 0; g < ng; g++) {
      if (!(rates[g] > 0.0 && rates[g] < 2.0)) return fail(LC_EINVAL, "MRT rate %d = %g outside (0, 2)", g, rates[g]);
      r[g] = rates[g];
    }
  } else if (kind != LC_COLL_BGK) {
    return fail(LC_EINVAL, "unknown collision %d", kind);
  }
  b->coll = kind;
  for (int g = 0; g < 5; g++) b->mrt[g] = r[g];
  // the descriptors carry the rates, and captured graphs the kernels
  batch_drop_graphs(b);
  lc_status st = batch_upload(b);
  if (st) return st;
  return hip_check(hipStreamSynchronize(b->stream), "descriptor upload sync");
}

lc_status lc_batch_autotune(lc_batch* b, int32_t trial_steps, int32_t* chosen, double* ms_per_step) {
  clear_error();
  if (!b) return fail(LC_EINVAL, "batch is NULL");
  if (trial_steps < 1) return fail(LC_EINVAL, "trial_steps must be >= 1");
  if (!b->loaded) return fail(LC_ESTATE, "load every grid of the batch before tuning");
  hipEvent_t e0, e1;
  lc_status st = hip_check(hipEventCreate(&e0), "event");
  if (st) return st;
  st = hip_check(hipEventCreate(&e1), "event");
  if (st) {
    (void)hipEventDestroy(e0);
    return st;
  }
  // every pair of tile shapes (stress sweep, Q sweep)
  int best = 0;
  float best_ms = 1e30f;
  for (int v = 0; v < BATCH_NV * BATCH_NV && st == LC_OK; v++) {
    st = lc_batch_set_tiles(b, v % BATCH_NV, v / BATCH_NV);
    if (st) break;
    // one untimed step, then the timed trial
    st = lc_batch_step(b, 1);
    if (st) break;
    (void)hipEventRecord(e0, b->stream);
    st = lc_batch_step(b, trial_steps);
    if (st) break;
    (void)hipEventRecord(e1, b->stream);
    st = hip_check(hipEventSynchronize(e1), "event sync");
    if (st) break;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best_ms) {
      best_ms = ms;
      best = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  if (chosen) *chosen = best;
  if (ms_per_step) *ms_per_step = double(best_ms) / trial_steps;
  return lc_batch_set_tiles(b, best % BATCH_NV, best / BATCH_NV);
}

lc_status lc_batch_observe(lc_batch* b, uint32_t mask, int32_t half_axis, lc_observables* out) {
  clear_error();
  if (!b || !out) return fail(LC_EINVAL, "NULL argument");
  if (!b->loaded) return fail(LC_ESTATE, "batch not loaded");
  if (half_axis < 0 || half_axis > 2) return fail(LC_EINVAL, "half_axis must be 0, 1 or 2");
  batch_sync_views(b);
  double* res = reinterpret_cast<double*>(static_cast<char*>(b->arena.scratch) + b->B.off_res);
  for (int k = 0; k < b->n; k++) {
    lc_ctx* c = &b->views[k];
    lc_status st = LC_DISPATCH(c, do_observe_async, mask, half_axis, res + size_t(k) * OBS_W);
    if (st) return st;
  }
  std::vector<double> h(size_t(b->n) * OBS_W);
  lc_status st = hip_check(hipMemcpyAsync(h.data(), res, h.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream),
                           "batch observe copy");
  if (st) return st;
  st = hip_check(hipStreamSynchronize(b->stream), "batch observe sync");
  if (st) return st;
  bool bad = false;
  for (int k = 0; k < b->n; k++) {
    fill_observables(&h[size_t(k) * OBS_W], mask, half_axis, b->step, &out[k]);
    bad = bad || out[k].nonfinite;
  }
  if (bad) return fail(LC_ENONFINITE, "a grid of the batch holds NaN or Inf");
  return LC_OK;
}

lc_status lc_batch_export(lc_batch* b, int32_t k, int32_t field, double* dst) {
  clear_error();
  if (!b || !dst) return fail(LC_EINVAL, "NULL argument");
  if (k < 0 || k >= b->n) return fail(LC_EINVAL, "grid index out of range");
  if (field < LC_FIELD_F || field > LC_FIELD_S) return fail(LC_EINVAL, "unknown field %d", field);
  batch_sync_views(b);
  lc_ctx* c = &b->views[k];
  if (!c->loaded) return fail(LC_ESTATE, "grid not loaded");
  return LC_DISPATCH(c, do_export, field, dst);
}

lc_status lc_batch_free(lc_batch* b) {
  clear_error();
  if (!b) return LC_OK;
  batch_drop_graphs(b);
  (void)hipStreamDestroy(b->cap);
  delete b;
  return LC_OK;
}

}  // extern "C"
