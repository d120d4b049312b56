// lc_runtime.h -- host-side helpers shared by the runtime translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <cstdarg>

#include "../../include/lc.h"

namespace lc {

// Byte offsets of the pieces of the caller's scratch buffer.
struct Layout {
  int64_t N;
  int q;
  size_t es;    // element size of f
  size_t es_q;  // element size of Q, u and the stress scratch
  size_t f_bytes, q_bytes;
  size_t off_tau, off_u, off_qp, off_r;
  size_t off_partial, off_obs;
  size_t off_vjp;  // reverse-step fields (D2Q9 double only; 0 bytes otherwise)
  int64_t nblocks;
  size_t scratch_bytes;
};

lc_status fail(lc_status code, const char* fmt, ...);
lc_status hip_check(hipError_t e, const char* what);
void clear_error();
int lattice_q(int lattice);
lc_status check_grid(const lc_grid* g);
lc_status check_params(const lc_params* p);
Layout layout_of(const lc_grid& g);
// one site per thread: blocks of SITE_TX x SITE_TY sites, one z plane each
constexpr int SITE_TX = 64, SITE_TY = 4;
dim3 site_block();
dim3 site_grid(const lc_grid& g);

}  // namespace lc
