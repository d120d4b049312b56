// lc_runtime.hip -- the C ABI of include/lc.h: validation, context, scratch
// layout, kernel dispatch over (lattice, precision, variant).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/lc.h"
#include "lc_aux.h"
#include "lc_split.h"
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
  if (g->precision != LC_FP64 && g->precision != LC_FP32_DEV)
    return fail(LC_EINVAL, "unknown precision %d", g->precision);
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return fail(LC_EINVAL, "grid dimensions must be >= 1");
  if (g->lattice == LC_D2Q9 && g->nz != 1) return fail(LC_EINVAL, "D2Q9 requires nz == 1");
  const double n = double(g->nx) * g->ny * g->nz;
  if (n > 4.0e9) return fail(LC_EINVAL, "grid too large (%.3g sites)", n);
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
  return c;
}

Layout layout_of(const lc_grid& g) {
  Layout L;
  const int64_t N = int64_t(g.nx) * g.ny * g.nz;
  const size_t es = g.precision == LC_FP64 ? 8 : 4;
  const int dim = g.lattice == LC_D2Q9 ? 2 : 3;
  const int ntau = dim == 2 ? 4 : 9;
  auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
  L.N = N;
  L.q = lattice_q(g.lattice);
  L.es = es;
  L.f_bytes = size_t(L.q) * N * es;
  L.q_bytes = size_t(5) * N * es;
  size_t off = 0;
  L.off_tau = off;
  off = up(off + size_t(ntau) * N * es);
  L.off_u = off;
  off = up(off + size_t(dim) * N * es);
  L.off_qp = off;
  off = up(off + size_t(5) * N * es);
  L.off_r = off;
  off = up(off + size_t(5) * N * es);
  const dim3 grid = site_grid(g);
  L.nblocks = int64_t(grid.x) * grid.y * grid.z;
  L.off_partial = off;
  off = up(off + size_t(L.nblocks) * OBS_W * 8);
  L.off_obs = off;
  off = up(off + OBS_W * 8);
  L.scratch_bytes = off;
  return L;
}

dim3 site_block() { return dim3(64, 4, 1); }

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
  int variant;
  int zchunk;  // 0: default
};

// ---------------------------------------------------------------------------
// Dispatch helpers.
template <int LAT, typename S, bool DEV>
static lc_status run_steps_staged(lc_ctx* c, int64_t n) {
  const GridDims gd{c->g.nx, c->g.ny, c->g.nz, c->L.N};
  const Coef<S> k = make_coef<S>(c->p);
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
    hipLaunchKernelGGL((stage_tau<LAT, S>), grid, block, 0, c->stream, q0, tau, gd, k);
    hipLaunchKernelGGL((stage_lb<LAT, S, DEV>), grid, block, 0, c->stream, f0, tau, f1, u, gd, k);
    hipLaunchKernelGGL((stage_pred<LAT, S>), grid, block, 0, c->stream, q0, u, qp, rq, gd, k);
    hipLaunchKernelGGL((stage_corr<LAT, S>), grid, block, 0, c->stream, q0, qp, rq, u, q1, gd, k);
    c->parity ^= 1;
    c->step++;
  }
  return hip_check(hipGetLastError(), "step launch");
}

// Tile shapes of the two-sweep kernels (LDS per block stays below 64 KB).
template <int LAT, typename S>
struct SplitCfg {
  static constexpr bool d3 = Lattice<LAT>::dim == 3;
  static constexpr bool f64 = sizeof(S) == 8;
  static constexpr int LB_TX = 32, LB_TY = (d3 && f64) ? 4 : 8;
  static constexpr int Q_TX = (d3 && f64) ? 16 : 32, Q_TY = 8;
  static constexpr int ZC = f64 ? 32 : 128;  // measured best on 256^3
  // waves per SIMD the register allocation is held to (LDS allows 4 blocks
  // of the single-precision 3D stress sweep per CU)
  static constexpr int LB_WPE = (d3 && !f64) ? 4 : 1;
  static constexpr int Q_WPE = 1;
};

template <int LAT, typename S, bool DEV>
static lc_status run_steps_split(lc_ctx* c, int64_t n) {
  using C = SplitCfg<LAT, S>;
  const GridDims gd{c->g.nx, c->g.ny, c->g.nz, c->L.N};
  const Coef<S> k = make_coef<S>(c->p);
  S* u = reinterpret_cast<S*>(static_cast<char*>(c->b.scratch) + c->L.off_u);
  const int zc = C::d3 ? (c->zchunk > 0 ? c->zchunk : C::ZC) : 1;
  const unsigned gz = unsigned((c->g.nz + zc - 1) / zc);
  const dim3 g1((c->g.nx + C::LB_TX - 1) / C::LB_TX, (c->g.ny + C::LB_TY - 1) / C::LB_TY, gz);
  const dim3 g2((c->g.nx + C::Q_TX - 1) / C::Q_TX, (c->g.ny + C::Q_TY - 1) / C::Q_TY, gz);
  for (int64_t it = 0; it < n; it++) {
    const S* f0 = static_cast<const S*>(c->b.f[c->parity]);
    S* f1 = static_cast<S*>(c->b.f[c->parity ^ 1]);
    const S* q0 = static_cast<const S*>(c->b.Q[c->parity]);
    S* q1 = static_cast<S*>(c->b.Q[c->parity ^ 1]);
    hipLaunchKernelGGL((split_lb<LAT, S, DEV, C::LB_TX, C::LB_TY, C::LB_WPE>), g1, dim3(C::LB_TX, C::LB_TY), 0, c->stream, q0,
                       f0, f1, u, gd, k, zc);
    hipLaunchKernelGGL((split_q<LAT, S, C::Q_TX, C::Q_TY, C::Q_WPE>), g2, dim3(C::Q_TX, C::Q_TY), 0, c->stream, q0, u, q1, gd,
                       k, zc);
    c->parity ^= 1;
    c->step++;
  }
  return hip_check(hipGetLastError(), "step launch");
}

template <int LAT, typename S, bool DEV>
static lc_status run_steps(lc_ctx* c, int64_t n) {
  if (c->variant == LC_VARIANT_SPLIT) return run_steps_split<LAT, S, DEV>(c, n);
  return run_steps_staged<LAT, S, DEV>(c, n);
}

template <int LAT, typename S, bool DEV>
static lc_status compute_tau(lc_ctx* c) {
  const GridDims gd{c->g.nx, c->g.ny, c->g.nz, c->L.N};
  const Coef<S> k = make_coef<S>(c->p);
  S* tau = reinterpret_cast<S*>(static_cast<char*>(c->b.scratch) + c->L.off_tau);
  hipLaunchKernelGGL((stage_tau<LAT, S>), site_grid(c->g), site_block(), 0, c->stream,
                     static_cast<const S*>(c->b.Q[c->parity]), tau, gd, k);
  return hip_check(hipGetLastError(), "stress launch");
}

template <int LAT, typename S, bool DEV>
static lc_status do_load(lc_ctx* c, const double* f, const double* q) {
  const GridDims gd{c->g.nx, c->g.ny, c->g.nz, c->L.N};
  hipLaunchKernelGGL((load_state<LAT, S, DEV>), site_grid(c->g), site_block(), 0, c->stream, f, q,
                     static_cast<S*>(c->b.f[0]), static_cast<S*>(c->b.Q[0]), gd);
  return hip_check(hipGetLastError(), "load launch");
}

template <int LAT, typename S, bool DEV>
static lc_status do_export(lc_ctx* c, int field, double* dst) {
  const int64_t N = c->L.N;
  const S* f = static_cast<const S*>(c->b.f[c->parity]);
  const S* q = static_cast<const S*>(c->b.Q[c->parity]);
  if (field == LC_FIELD_F || field == LC_FIELD_Q) {
    const GridDims gd{c->g.nx, c->g.ny, c->g.nz, N};
    hipLaunchKernelGGL((export_fq<LAT, S, DEV>), site_grid(c->g), site_block(), 0, c->stream, f, q,
                       field == LC_FIELD_F ? dst : nullptr, field == LC_FIELD_Q ? dst : nullptr, gd);
    return hip_check(hipGetLastError(), "export launch");
  }
  int which = field == LC_FIELD_RHO ? 0 : field == LC_FIELD_U ? 1 : field == LC_FIELD_FORCE ? 2 : 3;
  if (which != 3) {
    lc_status st = compute_tau<LAT, S, DEV>(c);
    if (st) return st;
  }
  const GridDims gd{c->g.nx, c->g.ny, c->g.nz, N};
  const S* tau = reinterpret_cast<const S*>(static_cast<char*>(c->b.scratch) + c->L.off_tau);
  hipLaunchKernelGGL((export_derived<LAT, S, DEV>), site_grid(c->g), site_block(), 0, c->stream, f, q, tau, dst,
                     which, gd);
  return hip_check(hipGetLastError(), "export launch");
}

template <int LAT, typename S, bool DEV>
static lc_status do_observe(lc_ctx* c, uint32_t mask, int half_axis, double* host8) {
  const int want_u = (mask & LC_OBS_UMAX) ? 1 : 0;
  if (want_u) {
    lc_status st = compute_tau<LAT, S, DEV>(c);
    if (st) return st;
  }
  const GridDims gd{c->g.nx, c->g.ny, c->g.nz, c->L.N};
  char* scr = static_cast<char*>(c->b.scratch);
  const S* tau = reinterpret_cast<const S*>(scr + c->L.off_tau);
  double* partial = reinterpret_cast<double*>(scr + c->L.off_partial);
  double* res = reinterpret_cast<double*>(scr + c->L.off_obs);
  hipLaunchKernelGGL((observe_partial<LAT, S, DEV>), site_grid(c->g), site_block(), 0, c->stream,
                     static_cast<const S*>(c->b.f[c->parity]), static_cast<const S*>(c->b.Q[c->parity]), tau,
                     partial, gd, half_axis, want_u);
  hipLaunchKernelGGL(observe_final, dim3(1), dim3(256), 0, c->stream, partial, c->L.nblocks, res);
  lc_status st = hip_check(hipGetLastError(), "observe launch");
  if (st) return st;
  st = hip_check(hipMemcpyAsync(host8, res, OBS_W * sizeof(double), hipMemcpyDeviceToHost, c->stream),
                 "observe copy");
  if (st) return st;
  return hip_check(hipStreamSynchronize(c->stream), "observe sync");
}

#define LC_DISPATCH(ctx, FN, ...)                                                   \
  ((ctx)->g.lattice == LC_D2Q9                                                      \
       ? ((ctx)->g.precision == LC_FP64 ? FN<0, double, false>(ctx, ##__VA_ARGS__)  \
                                        : FN<0, float, true>(ctx, ##__VA_ARGS__))   \
       : ((ctx)->g.precision == LC_FP64 ? FN<1, double, false>(ctx, ##__VA_ARGS__)  \
                                        : FN<1, float, true>(ctx, ##__VA_ARGS__)))

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
  c->variant = LC_VARIANT_SPLIT;
  c->zchunk = 0;
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
    c->variant = LC_VARIANT_SPLIT;
    return LC_OK;
  }
  if (variant == LC_VARIANT_STAGED) {
    c->variant = LC_VARIANT_STAGED;
    return LC_OK;
  }
  if (variant == LC_VARIANT_FUSED) return fail(LC_EUNSUPPORTED, "variant %d not available", variant);
  return fail(LC_EINVAL, "unknown variant %d", variant);
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
  out->step = c->step;
  out->half_axis = half_axis;
  out->nonfinite = h[7] != 0.0 ? 1 : 0;
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

lc_status lc_sync(lc_ctx* c) {
  clear_error();
  if (!c) return fail(LC_EINVAL, "ctx is NULL");
  return hip_check(hipStreamSynchronize(c->stream), "sync");
}

int64_t lc_step_count(const lc_ctx* c) { return c ? c->step : -1; }

lc_status lc_free(lc_ctx* c) {
  clear_error();
  delete c;
  return LC_OK;
}

}  // extern "C"
