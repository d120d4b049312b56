/*
 * lc.h -- C ABI of the MI355X hybrid lattice-Boltzmann / finite-difference
 * library for nematic liquid crystals.
 *
 * The method is that of Coelho, Araujo and Telo da Gama, "Lattice-Boltzmann
 * simulation of free nematic-isotropic interfaces" (arXiv:1907.13415):
 * the Beris-Edwards equation for the Landau-de Gennes order tensor Q
 * (Sec. 1.1, Eqs. 1-4) integrated by a predictor-corrector finite-difference
 * scheme (Sec. 1.2.2), coupled through the stress of Eq. (6) and its
 * divergence to a forced lattice-Boltzmann Navier-Stokes solver (Sec. 1.2.1,
 * Eqs. 7-9), on one grid with one time step (dx = dt = 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Grids are periodic in every direction.  The site index is
 *    s = x + nx*(y + ny*z), x fastest.  Two-dimensional grids use D2Q9 and
 *    nz = 1; D3Q19 accepts any nz >= 1.
 *  - Fields are structure-of-arrays, component-major: populations
 *    f[i*N + s] (i over the lattice velocities, see lc_lattice_info), order
 *    tensor Q[c*N + s] with c = (xx, xy, xz, yy, yz) and Qzz = -Qxx - Qyy.
 *  - Velocity order.  D2Q9: 0 (0,0); 1 (1,0); 2 (0,1); 3 (-1,0); 4 (0,-1);
 *    5 (1,1); 6 (-1,1); 7 (-1,-1); 8 (1,-1).  D3Q19: 0 rest; 1..6 = +x, -x,
 *    +y, -y, +z, -z; 7..18 = (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1)
 *    (-1,0,-1) (1,0,-1) (-1,0,1) (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1).
 *  - Storage precision.  LC_FP64 stores f and Q as double.  LC_FP32_DEV
 *    stores the deviation f_i - w_i*rho0 (rho0 = 1) and Q as float and does
 *    all per-site arithmetic in float; reductions accumulate in double.
 *    LC_MIXED stores f as LC_FP32_DEV does (float deviations, float moments
 *    and collision) and Q as double, with the molecular field, stress, body
 *    force and Q update in double: the float rounding
 *    of the Q right-hand side, which moves slow interfaces in LC_FP32_DEV,
 *    is gone, at 2(q*4 + 5*8) bytes per site update.  LC_MIXED runs the
 *    split and fused variants and the batched form (LC_VARIANT_STAGED:
 *    LC_EUNSUPPORTED).
 *    LC_FP32_SR stores f and Q as LC_FP32_DEV does and computes as it does,
 *    except in the Q update: the molecular field of Eq. (4) is summed in
 *    double from the float Q and Laplacian (its bulk terms nearly cancel),
 *    and Q(n+1) of Sec. 1.2.2 step 5 is rounded to float stochastically
 *    (round up or down with probabilities given by the distances, from a
 *    counter-based hash of the site index and the step count), so that
 *    increments below half a unit in the last place are not lost at every
 *    step; results depend on the step count since the last load, and are
 *    reproducible.  Split and fused variants and the batched form; no
 *    lc_step_static.
 *    Every load/export entry point speaks double "logical" values (full f)
 *    whatever the storage precision.
 *  - Memory ownership.  The caller allocates and owns every device buffer
 *    (for example as torch tensors); the library never allocates device
 *    memory.  It keeps only a small host-side context, for the batched
 *    form a captured HIP graph, and one fixed device array per GPU that
 *    serves lc_step_static.  All work is enqueued on the HIP stream
 *    given at init; only calls documented as synchronising wait for it.
 *  - Errors.  Every call returns an lc_status; on failure lc_last_error()
 *    gives a message (thread-local).  Asynchronous device errors surface at
 *    the next synchronising call.  No C++ exception crosses this ABI.
 */
#ifndef LC_H
#define LC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lc_status;
#define LC_OK 0
#define LC_EINVAL (-1)       /* bad argument: sizes, parameters, pointers */
#define LC_ENOMEM (-2)       /* buffer too small / host allocation failed */
#define LC_EDEVICE (-3)      /* HIP runtime error (message has the details) */
#define LC_ENONFINITE (-4)   /* NaN or Inf found in the state by lc_observe */
#define LC_ESTATE (-5)       /* call out of order (e.g. step before load) */
#define LC_EUNSUPPORTED (-6) /* valid request the library does not provide */

#define LC_D2Q9 0
#define LC_D3Q19 1

#define LC_FP64 0
#define LC_FP32_DEV 1
#define LC_MIXED 2
#define LC_FP32_SR 3

/* Collision operators for lc_set_collision. */
#define LC_COLL_BGK 0 /* single relaxation time (default) */
#define LC_COLL_MRT 1 /* multiple relaxation times, standard orthogonal moment bases */

/* Difference stencils for lc_set_stencil. */
#define LC_STENCIL_COMPACT 0   /* central differences, (2d+1)-point Laplacian (default) */
#define LC_STENCIL_ISOTROPIC 1 /* from the lattice velocities and weights */

/* Kernel variants for lc_set_variant. */
#define LC_VARIANT_AUTO 0
#define LC_VARIANT_STAGED 1 /* one kernel per stage, intermediates in scratch */
#define LC_VARIANT_SPLIT 2  /* two sweeps: LB update + velocity, then Q update */
#define LC_VARIANT_FUSED 3  /* one pass: reads f and Q once, writes them once */

/* A periodic grid of nx * ny * nz sites (nz == 1 for D2Q9; Sec. 2 runs
 * periodic boxes).  Every dimension >= 1, nx <= 2^30 and ny, nz <= 65535,
 * else LC_EINVAL; more than 4e9 sites (beyond the sweeps' 32-bit site
 * indices) is LC_ENOMEM. */
typedef struct {
  int32_t lattice;   /* LC_D2Q9 or LC_D3Q19 */
  int32_t precision; /* LC_FP64, LC_FP32_DEV, LC_MIXED or LC_FP32_SR */
  int32_t nx, ny, nz;
} lc_grid;

/* Model parameters in lattice units (Sec. 2 lists the paper's set).
 *   A0, gamma : bulk Landau-de Gennes coefficients of Eq. (3);
 *   K         : one-constant elasticity of Eq. (3);
 *   Gamma     : rotational diffusion constant of Eq. (1);
 *   xi        : flow-alignment parameter of Eq. (2);
 *   eta, tau  : viscosity of Eq. (5) and the BGK relaxation time; the
 *               lattice-Boltzmann viscosity is eta = rho0 (tau - 1/2)/3 with
 *               rho0 = 1, so eta must match tau to 1e-12 (relative).
 * Requirements: all finite, tau > 1/2, K >= 0, Gamma > 0, A0 > 0. */
typedef struct {
  double A0, gamma, K, Gamma, xi, eta, tau;
} lc_params;

/* Caller-owned device buffers.  f[0], f[1]: q*N values each; Q[0], Q[1]:
 * 5*N values each (element size 8 for LC_FP64, 4 for LC_FP32_DEV; for
 * LC_MIXED 4 for f and 8 for Q);
 * scratch: the scratch_bytes reported by lc_buffer_bytes.  All 256-byte aligned, disjoint, and
 * valid for the lifetime of the context. */
typedef struct {
  void *f[2];
  void *Q[2];
  void *scratch;
} lc_buffers;

/* Observables (all accumulated in double).
 *   mass      : sum of f over sites and velocities;
 *   mom[3]    : lattice momentum sum c_i f_i (conserved by the scheme);
 *   umax      : max over sites of |u|, u the force-corrected velocity of
 *               Eq. (9), which is the one Sec. 1.2.2 feeds to Eq. (1);
 *   ssum      : sum over sites of S = sqrt(1.5 Q:Q) (exact for uniaxial Q);
 *   ssum_half : sum of S over c <= k <= c + n/2 along half_axis (end planes
 *               weighted 1/2; c = n/2), which locates the right-hand
 *               interface of a slab centred at n/2 (Sec. 2.1);
 *   step      : steps taken since the last load;
 *   nonfinite : 1 if any NaN or Inf was found in f or Q. */
typedef struct {
  double mass;
  double mom[3];
  double umax;
  double ssum;
  double ssum_half;
  int64_t step;
  int32_t nonfinite;
  int32_t half_axis;
} lc_observables;

#define LC_OBS_MASS 1u
#define LC_OBS_MOM 2u
#define LC_OBS_UMAX 4u
#define LC_OBS_S 8u
#define LC_OBS_ALL 15u

/* Fields for lc_export (double, component-major, N sites each). */
#define LC_FIELD_F 0     /* q components: populations f_i */
#define LC_FIELD_Q 1     /* 5 components (xx, xy, xz, yy, yz) */
#define LC_FIELD_RHO 2   /* 1 component: density sum f_i */
#define LC_FIELD_U 3     /* 3 components: force-corrected velocity, Eq. (9) */
#define LC_FIELD_FORCE 4 /* 3 components: F_a = d_b Pi_ab + d_a P0 (Sec. 1.2.1) */
#define LC_FIELD_S 5     /* 1 component: sqrt(1.5 Q:Q) */

typedef struct lc_ctx lc_ctx;
typedef struct lc_batch lc_batch;

/* Message of the last failing call on this thread ("" if none).  Library
 * plumbing: implements no passage of the paper. */
const char *lc_last_error(void);

/* Velocity set of a lattice: *q, c[i*3 + a] (q*3 ints) and w[i] (q doubles).
 * c and w may be NULL to query q only.  The D2Q9 and D3Q19 velocity sets and
 * weights of Sec. 1.2.1 (Eq. 8 uses the weights, c_s^2 = 1/3), in the order
 * of the preamble.  LC_EINVAL for an unknown lattice or NULL q. */
lc_status lc_lattice_info(int32_t lattice, int32_t *q, int32_t *c, double *w);

/* Bytes of one f buffer, one Q buffer and the scratch buffer for a grid
 * (any output pointer may be NULL): f holds the q populations of Eq. (7) per
 * site, Q the five independent components of the traceless symmetric order
 * tensor of Sec. 1.1, in the storage precision of the grid.  LC_EINVAL for
 * a bad grid. */
lc_status lc_buffer_bytes(const lc_grid *grid, size_t *f_bytes, size_t *q_bytes,
                          size_t *scratch_bytes);

/* Create a context over caller-owned buffers for the time step of Sec. 1.2
 * (Eqs. 1-9) on `grid` with the parameters of Eqs. (1)-(5).  `stream` is a
 * hipStream_t (NULL = default stream).  Validates the grid, the parameters
 * and the buffers (LC_EINVAL); host allocation failure is LC_ENOMEM.  The
 * state is undefined until lc_load_state.  Defaults: variant AUTO, BGK
 * collision, compact stencils. */
lc_status lc_init(const lc_grid *grid, const lc_params *params, const lc_buffers *bufs,
                  void *stream, lc_ctx **out);

/* Replace the parameters of Eqs. (1)-(5) (same validation as lc_init); for
 * the temperature sweeps of Sec. 2.1.  Applies to the steps enqueued after
 * the call. */
lc_status lc_set_params(lc_ctx *ctx, const lc_params *params);

/* Choose the kernel variant (LC_VARIANT_*) of the step of Sec. 1.2 (the
 * same arithmetic in each; SPLIT and FUSED agree bit for bit).  AUTO (the
 * default) picks the fastest the library provides for the context's stencil
 * and grid: the two-sweep variant, except FUSED on D2Q9 grids of at most
 * 147456 (384^2) sites with the compact stencils and 65536 (256^2) with the
 * isotropic ones, where launches are latency bound and the single pass
 * measured faster in every precision.  FUSED runs every
 * stage of a step in one pass over the grid: a block recomputes the
 * stress, moments and predictor on shrinking rings around its tile instead
 * of reading them back from HBM.  LC_EUNSUPPORTED for the staged variant in
 * LC_MIXED. */
lc_status lc_set_variant(lc_ctx *ctx, int32_t variant);

/* Collision operator of the lattice-Boltzmann update.  LC_COLL_BGK (the
 * default): relaxation at 1/tau with the forcing term of Sec. 1.2.1.
 * LC_COLL_MRT: the multiple-relaxation-time operator the paper ran
 * (Sec. 1.2.1 names it but leaves its matrix and rates to another paper),
 * on the standard orthogonal moment bases (Lallemand and Luo 2000 for D2Q9,
 * d'Humieres et al. 2002 for D3Q19) with the same forcing in moment space:
 * m* = m - S (m - m_eq) + (I - S/2) M G.  Density, momentum and the
 * traceless stress relax at 1/tau (so the viscosity stays (tau - 1/2)/3);
 * rates[nrates] (host array) gives the rate of each other moment group:
 * D2Q9 (s_e, s_eps, s_q), D3Q19 (s_e, s_eps, s_q, s_pi, s_m), each in
 * (0, 2).  With every rate 1/tau, MRT equals BGK up to rounding.  Applies to
 * the steps enqueued after the call.  LC_EINVAL for an unknown kind, a
 * wrong count or a rate outside (0, 2).  The reverse step supports BGK
 * only (LC_EUNSUPPORTED otherwise). */
lc_status lc_set_collision(lc_ctx *ctx, int32_t kind, const double *rates, int32_t nrates);

/* Difference stencil of every derivative in the step: grad Q and lap Q
 * (Eqs. 2, 4, 6), the divergence of the stress (the body force of Sec.
 * 1.2.1) and grad u (Eq. 2).  LC_STENCIL_COMPACT (the default): the
 * second-order central differences and compact Laplacian of Sec. 1.2.2.
 * LC_STENCIL_ISOTROPIC: the option the closing remarks of Sec. 2.2 point to
 * for reducing spurious currents, derivatives from the lattice's own
 * velocities c_i and weights w_i (c_s^2 = 1/3):
 *   d_g V = 3 sum_i w_i c_ig V(x + c_i),  lap V = 6 sum_i w_i [V(x + c_i) - V(x)],
 * second order as well, with leading errors independent of direction.
 * Applies to the steps, exports and observables after the call.  The
 * isotropic stencils run in the two-sweep and staged variants, and in the
 * single pass on D2Q9 grids (lc_step returns LC_EUNSUPPORTED for
 * LC_VARIANT_FUSED on D3Q19), in LC_FP64 and LC_FP32_DEV (LC_EUNSUPPORTED
 * otherwise), with either collision; the batched form takes them through
 * lc_batch_set_stencil, and the reverse step uses the compact stencils only.
 * LC_EINVAL for an unknown stencil. */
lc_status lc_set_stencil(lc_ctx *ctx, int32_t stencil);

/* Planes each block marches through along z in the two-sweep and fused
 * kernels (>= 1; larger chunks recompute fewer boundary planes, smaller
 * chunks give more blocks; a chunk longer than nz is the whole depth).  0
 * restores the built-in default.  Ignored by 2D grids.  A launch-shape setting: implements no passage of the paper and
 * does not change results.  LC_EINVAL for planes < 0. */
lc_status lc_set_chunk(lc_ctx *ctx, int32_t planes);

/* Load the state from device arrays of double logical values: f_dev (q*N)
 * and Q_dev (5*N), the populations of Eq. (7) and the order tensor of
 * Sec. 1.1 (layout of the preamble).  f_dev == NULL loads the fluid at rest
 * with rho = 1, f_i = w_i (the initial condition of Sec. 2).  Resets the
 * step counter.  Asynchronous on the context stream.  LC_EINVAL for a NULL
 * context or Q_dev. */
lc_status lc_load_state(lc_ctx *ctx, const double *f_dev, const double *Q_dev);

/* Enqueue n >= 0 time steps of Sec. 1.2 (asynchronous on the context
 * stream): the molecular field (Eq. 4), stress (Eq. 6) and its divergence
 * as the body force (Sec. 1.2.1), density and force-corrected velocity
 * (Eq. 9), the predictor-corrector update of Q by Eqs. (1)-(2) (Sec. 1.2.2
 * steps 1-5), and the forced collision (Eq. 8 and the forcing term of
 * Sec. 1.2.1) with periodic streaming (Eq. 7).  LC_EINVAL for n < 0,
 * LC_ESTATE before lc_load_state, LC_EUNSUPPORTED for a variant, precision
 * and stencil that do not go together. */
lc_status lc_step(lc_ctx *ctx, int64_t n);

/* Reduce the current state to observables (mask of LC_OBS_*; fields not
 * requested are 0) with half-domain axis half_axis (0, 1, 2): mass and
 * momentum of Eq. (9), the force-corrected velocity of Eq. (9), the scalar
 * order S of Sec. 1.1 and the half-domain sum that locates the interface
 * of Sec. 2.1.  Synchronises the stream.  Returns LC_ENONFINITE (with *out
 * filled) if the state holds a NaN or Inf; LC_EINVAL for a bad axis or
 * NULL argument; LC_ESTATE before lc_load_state. */
lc_status lc_observe(lc_ctx *ctx, uint32_t mask, int32_t half_axis, lc_observables *out);

/* Write a field of the current state as double to dst_dev (device memory,
 * size given by the field, N = nx*ny*nz, component-major): the populations
 * of Eq. (7), the order tensor of Sec. 1.1, the density and force-corrected
 * velocity of Eq. (9), the body force of Sec. 1.2.1 or S.  Asynchronous.
 * LC_EINVAL for an unknown field or NULL argument; LC_ESTATE before
 * lc_load_state. */
lc_status lc_export(lc_ctx *ctx, int32_t field, double *dst_dev);

/* Reverse-mode step (adjoint) for gradients of a loss of the final state
 * with respect to the initial state and to gamma, K and Gamma.  Provided
 * for D2Q9 in LC_FP64 (LC_EUNSUPPORTED otherwise).
 *   f_n, Q_n : the state at step n, device arrays of double logical values
 *              (as lc_export writes them: q*N and 5*N), read only;
 *   adj_f, adj_Q : on entry the adjoint dL/d(state at n+1), on return
 *              dL/d(state at n) (device, q*N and 5*N doubles, overwritten);
 *   dparams  : device doubles [3]; dL/dgamma, dL/dK, dL/dGamma of this step
 *              are ADDED to them.
 * The step is differentiated exactly as the forward step computes it
 * (Eqs. 1-9 with the readings of lc_step).  Asynchronous; uses the reverse
 * fields of the scratch buffer, so reverse steps on one context must not
 * overlap. */
lc_status lc_vjp_step(lc_ctx *ctx, const double *f_n, const double *Q_n, double *adj_f, double *adj_Q,
                      double *dparams);

/* Bytes of the state history lc_vjp_segment needs for n steps (0 on bad
 * arguments). */
size_t lc_vjp_history_bytes(const lc_grid *grid, int32_t n);

/* Reverse sweep over one checkpoint segment (D2Q9, LC_FP64): starting from
 * the checkpoint state (f_ck, Q_ck: device arrays of double logical values),
 * replay the n steps, recording every state and the step's density, body
 * force, velocity and predictor in `hist` (caller-owned device buffer of
 * lc_vjp_history_bytes(grid, n) bytes, 256-byte aligned), then apply the n
 * reverse steps n-1 .. 0 to (adj_f, adj_Q) in place, adding the parameter
 * derivatives to dparams[3] as lc_vjp_step does.  The context's own state is
 * not modified.  Asynchronous on the context stream.  (Checkpoint-and-
 * recompute of the reverse mode; the paper has no adjoint.) */
lc_status lc_vjp_segment(lc_ctx *ctx, const double *f_ck, const double *Q_ck, int32_t n, void *hist,
                         double *adj_f, double *adj_Q, double *dparams);

/* Bytes of the history lc_vjp_backward needs when no segment is longer than
 * n steps: two segment histories (0 on bad arguments). */
size_t lc_vjp_backward_bytes(const lc_grid *grid, int32_t n);

/* The whole reverse sweep over nseg checkpoint segments (D2Q9, LC_FP64).
 * f_cks[k], Q_cks[k] (host arrays of nseg device pointers, double logical
 * values) are the checkpoints in forward order, ns[k] (host array) the steps
 * of segment k.  Segments are walked back from nseg-1 to 0 as
 * lc_vjp_segment does, but the replay of segment k-1 runs on a second stream
 * of the library while segment k is walked back on the context stream; the
 * two alternate between the halves of `hist` (lc_vjp_backward_bytes(grid,
 * max ns) bytes, 256-byte aligned).  adj_f, adj_Q are updated in place and
 * the parameter derivatives added to dparams[3].  Work the caller queued on
 * the context stream before the call is complete before any replay starts,
 * and all of the call's work is complete once the context stream reaches
 * the point after it.  The context's own state is not modified.
 * Asynchronous.  LC_EINVAL on NULL pointers, nseg < 1, a segment with fewer
 * than one step or a misaligned hist; LC_EDEVICE if the second stream or
 * its events cannot be created. */
lc_status lc_vjp_backward(lc_ctx *ctx, int32_t nseg, const double *const *f_cks, const double *const *Q_cks,
                          const int32_t *ns, void *hist, double *adj_f, double *adj_Q, double *dparams);

/* Wait for the context stream and report any pending device error
 * (LC_EDEVICE).  Library plumbing: implements no passage of the paper. */
lc_status lc_sync(lc_ctx *ctx);

/* Per-launch timing of the step kernels.  While enabled, lc_step records
 * HIP events on the context stream around each launch of the split and
 * fused variants (every 1024 launches the context waits for the recorded
 * ones and folds them into running sums, so the number of events it holds
 * stays bounded).  lc_get_timing synchronises, returns the summed
 * durations in milliseconds and the number of launches of kind 0 (the
 * stress/LB sweep, or the single pass of the fused variant) and kind 1 (the
 * Q sweep) since the last call, and resets the record.  Measurement plumbing:
 * implements no passage of the paper.  LC_EINVAL for a NULL context. */
lc_status lc_set_timing(lc_ctx *ctx, int32_t enable);
lc_status lc_get_timing(lc_ctx *ctx, double *ms /*[2]*/, int64_t *launches /*[2]*/);

/* Steps taken since the last load (-1 for a NULL context).  Library
 * plumbing. */
int64_t lc_step_count(const lc_ctx *ctx);

/* Destroy the context (device buffers stay with the caller).  Library
 * plumbing. */
lc_status lc_free(lc_ctx *ctx);

/* Size of the library's own device scratch used by lc_step_static. */
#define LC_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): lc_step
 * without a context or a scratch buffer.  Advances n >= 0 steps of the
 * split sweeps with BGK collision (exactly what lc_step computes on a
 * context with the default variant, collision and chunk) of the state held
 * in storage form in f[parity], Q[parity] (as a context over the same four
 * buffers holds it after lc_load_state or lc_step; f[0], f[1], Q[0], Q[1]
 * device pointers, 256-byte aligned, sized by lc_buffer_bytes), alternating
 * between the two buffers of each pair: the result is in f[parity ^ (n & 1)],
 * Q[parity ^ (n & 1)].  The velocity between the sweeps goes to a fixed
 * device array of LC_STATIC_SCRATCH_BYTES that the library holds on every
 * GPU it runs on until the process ends; grids whose velocity field (2 or
 * 3 components of N values, 4 bytes each in LC_FP32_DEV, else 8) exceeds
 * it are rejected with LC_ENOMEM.  The call allocates nothing, host or
 * device.  All calls on one GPU share that array: calls that overlap on one
 * GPU (other streams, other threads) race and must be ordered by the
 * caller.  Asynchronous on `stream` (a hipStream_t, NULL = default).
 * LC_EINVAL for a bad grid, parameters, parity, n or buffer. */
lc_status lc_step_static(const lc_grid *grid, const lc_params *params, void *const *f, void *const *Q,
                         int32_t parity, int64_t n, void *stream);

/* ---------------------------------------------------------------------------
 * Batched form: many independent two-dimensional D2Q9 grids of their own
 * sizes and parameters (for example a temperature sweep in gamma around the
 * coexistence value of Sec. 2.1) advanced together.  All grids share one
 * storage precision (any of the four; LC_EINVAL otherwise).  With
 * LC_FP32_SR every grid rounds its Q update with the uniform numbers of its
 * step count, so each grid of a batch equals the same grid stepped alone by
 * lc_step bit for bit.  The grids' fields live in
 * caller-owned arenas: grid k
 * occupies f_offsets[k] bytes into each f arena (9*N_k values) and
 * q_offsets[k] bytes into each Q arena (5*N_k values, double in the mixed
 * form), in the single-grid layout.  A step of the batch is two kernel launches covering the tiles of
 * every grid; runs of steps are captured once in a HIP graph (64 steps per
 * graph) and replayed on the batch stream.
 * ------------------------------------------------------------------------- */

/* Arena sizes and per-grid byte offsets (f_offsets, q_offsets: ngrids
 * entries each, may be NULL) for the many grids of a temperature sweep
 * (Sec. 2.1).  LC_EINVAL for a bad grid or mixed precisions,
 * LC_EUNSUPPORTED for D3Q19 grids. */
lc_status lc_batch_layout(int32_t ngrids, const lc_grid *grids, size_t *f_bytes, size_t *q_bytes,
                          size_t *scratch_bytes, size_t *f_offsets, size_t *q_offsets);

/* Create a batch over caller-owned arenas (arena->f[0..1], arena->Q[0..1],
 * arena->scratch sized by lc_batch_layout, 256-byte aligned).  params has
 * ngrids entries, each validated as in lc_init.  Synchronises the stream
 * once (descriptor upload). */
lc_status lc_batch_init(int32_t ngrids, const lc_grid *grids, const lc_params *params,
                        const lc_buffers *arena, void *stream, lc_batch **out);

/* Load grid k (same conventions as lc_load_state: Eq. (7) populations,
 * Sec. 1.1 order tensor).  Every grid must be
 * loaded before the batch steps; loading after steps were taken resets the
 * batch, and every grid must then be loaded again. */
lc_status lc_batch_load_state(lc_batch *b, int32_t k, const double *f_dev, const double *Q_dev);

/* Enqueue n >= 0 steps of Sec. 1.2 on every grid, each with its own
 * parameters (asynchronous; graph replays for whole runs of 64 steps,
 * direct launches for the rest).  LC_ESTATE until every grid is loaded. */
lc_status lc_batch_step(lc_batch *b, int64_t n);

/* Select the tile shape of each sweep: v_lb for the stress / LB sweep, v_q
 * for the Q sweep (0: 32x8, 1: 64x4, 2: 16x16, 3: 32x16, 4: 64x8, 5: 64x16,
 * 6: 128x8 sites per block).  Results do not depend on the tile shapes (a
 * launch shape: implements no passage of the paper).  LC_EINVAL outside
 * 0..6. */
lc_status lc_batch_set_tiles(lc_batch *b, int32_t v_lb, int32_t v_q);

/* lc_batch_set_tiles(b, variant, variant).  A launch shape: implements no
 * passage of the paper and does not change results. */
lc_status lc_batch_set_tile(lc_batch *b, int32_t variant);

/* Difference stencils of every grid of the batch, as lc_set_stencil (the
 * compact ones of Sec. 1.2.2, or the isotropic ones of the closing remarks
 * of Sec. 2.2 in LC_FP64 and LC_FP32_DEV, LC_EUNSUPPORTED otherwise); for
 * the steps, exports and observables after the call.  LC_EINVAL for an
 * unknown stencil. */
lc_status lc_batch_set_stencil(lc_batch *b, int32_t stencil);

/* Collision operator of every grid of the batch, as lc_set_collision
 * (Sec. 1.2.1; BGK by default, or MRT with the D2Q9 group rates
 * (s_e, s_eps, s_q), each grid's density, momentum and stress relaxing at
 * its own 1/tau).  Applies to the steps enqueued after the call and
 * synchronises the stream once (descriptor upload).  LC_EINVAL for an
 * unknown kind, a wrong count or a rate outside (0, 2). */
lc_status lc_batch_set_collision(lc_batch *b, int32_t kind, const double *rates, int32_t nrates);

/* Time every pair of tile shapes for trial_steps steps (after one untimed
 * step) with HIP events and keep the fastest; *chosen = v_lb + 7 * v_q.
 * The state advances by 49 * (trial_steps + 1) steps: tune before loading
 * the real state, or load it again afterwards.  Synchronises the stream.
 * Measurement plumbing: implements no passage of the paper. */
lc_status lc_batch_autotune(lc_batch *b, int32_t trial_steps, int32_t *chosen, double *ms_per_step);

/* Observables of every grid, as lc_observe (Eq. 9, Sec. 1.1, Sec. 2.1):
 * out has ngrids entries.  Synchronises. */
lc_status lc_batch_observe(lc_batch *b, uint32_t mask, int32_t half_axis, lc_observables *out);

/* Export a field of grid k (as lc_export: Eq. 7, Sec. 1.1, Eq. 9,
 * Sec. 1.2.1). */
lc_status lc_batch_export(lc_batch *b, int32_t k, int32_t field, double *dst_dev);

/* Destroy the batch (graphs and its capture stream; arenas stay with the
 * caller).  Library plumbing. */
lc_status lc_batch_free(lc_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* LC_H */
