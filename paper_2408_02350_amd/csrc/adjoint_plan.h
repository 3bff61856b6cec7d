// Launch plan of the reverse transport (host and device code of the
// reverse step include this; the forward kernels do not).
#ifndef BGK_ADJOINT_PLAN_H
#define BGK_ADJOINT_PLAN_H

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bgk.h"

namespace bgk {

struct Ctx;

// A forward step's state that the reverse step reads (f-tilde's interior
// rows, f^{n+1}, and the moments of n+1), when the caller kept it from the
// forward pass instead of having the reverse step recompute it.
struct AdjState {
  const void* ft;
  const void* f1;
  const double* rho1;
  const double* U1;
  const double* T1;
};
hipError_t launch_adjoint_step_kept(const Ctx& c, const void* f_n, const double* U_n,
                                    const AdjState& s, const void* lam_f1, const double* lam_U1,
                                    const double* lam_rho1, const double* lam_T1, void* lam_f,
                                    double* lam_U, double* dJ_dlid);

// R velocities per lane for the interior patches, stepping along z in 3D
// and x in 2D (4 when 4 divides nv, else 2; FP32 storage in 3D: 5 when 5 divides nv,
// with 4 velocities' set-up cost spread over 5), Rw for the per-particle
// wall kernel (4 when 4 divides nv, else 2: at 5 its register footprint
// halves its waves), interior patches of P = 2 particles, and the 64-lane
// tiles of R (Rw) velocities the grid needs: one wavefront per (patch or
// wall particle, tile), each tile holding its part of lam_U per particle.
// Blocks of several wavefronts sharing one derivation of the edge records
// were slower in both precisions (the waves of a block then wait on the
// derivation together).
struct AdjPlan {
  int R, Rw, P, tiles, tiles_w;
};
inline AdjPlan adj_plan(const bgk_config& cfg) {
  int64_t nvel = 1;
  for (int a = 0; a < cfg.dim; ++a) nvel *= cfg.nv;
  AdjPlan p{};
  p.Rw = (cfg.nv % 4 == 0) ? 4 : 2;
  p.R = (cfg.dim == 3 && cfg.precision == BGK_FP32 && cfg.nv % 5 == 0) ? 5 : p.Rw;
  p.P = 2;
  p.tiles = static_cast<int>((nvel / p.R + 63) / 64);
  p.tiles_w = static_cast<int>((nvel / p.Rw + 63) / 64);
  return p;
}

}  // namespace bgk

#endif  // BGK_ADJOINT_PLAN_H
