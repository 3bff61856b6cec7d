// S5-S8 and the moment / Maxwellian helpers.
//
// One block of 256 threads owns one particle's row of f (all velocities,
// all components).  Each thread always handles the same velocities
// q = tid, tid + 256, ..., so every value it reads back in a later pass was
// written by itself (no cross-thread hazards inside a block).  Moment sums
// are FP64 in every precision mode, reduced in a fixed order (wavefront
// butterflies, then the four waves in order), so results are deterministic.
#include <algorithm>

#include "device_common.h"

namespace bgk {

// rho, U, T of one particle's row (Sec. 2 eqs. moments, internal_energy;
// Chu eq. macroeq; time-discrete fullmoment1a / moment1a, moment1b):
// rho = omega sum f1, U = sum v f1 / sum f1, then 3 rho T from the centred
// second moment (Chu: plus sum g2).  Returns the FP64 sums through refs.
template <int D, int NC, typename Real>
__device__ __forceinline__ void row_moments(const Real* row, size_t cs, int NV, int nv, double vmax,
                                            double omega, double* sh, double& rho, double* U,
                                            double& T) {
  double s[D + 1];
#pragma unroll
  for (int k = 0; k <= D; ++k) s[k] = 0.0;
  for (int q = threadIdx.x; q < NV; q += kThreads) {
    double v[3];
    velocity_of<D>(q, nv, vmax, v);
    const double f1 = static_cast<double>(row[q]);
    s[0] = s[0] + f1;
#pragma unroll
    for (int k = 0; k < D; ++k) s[1 + k] = s[1 + k] + v[k] * f1;
  }
  block_sum<D + 1>(s, sh);
  const double s0 = s[0];
  rho = omega * s0;
#pragma unroll
  for (int k = 0; k < D; ++k) U[k] = s[1 + k] / s0;
  double e[1] = {0.0};
  for (int q = threadIdx.x; q < NV; q += kThreads) {
    double v[3];
    velocity_of<D>(q, nv, vmax, v);
    double w2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double wk = v[k] - U[k];
      w2 = w2 + wk * wk;
    }
    e[0] = e[0] + w2 * static_cast<double>(row[q]);
    if (NC == 2) e[0] = e[0] + static_cast<double>(row[cs + q]);
  }
  block_sum<1>(e, sh);
  T = e[0] / (3.0 * s0);
}

struct CollideArgs {
  int N, NV, nv, count;
  double vmax, omega, kn, dt;
  const int32_t* plist;
  const void* ft;
  void* fo;
  double* rho;
  double* U;
  double* T;
  int32_t* err;
};

// S5-S6: moments of ft, tau at the new state, f = (tau ft + dt M)/(tau + dt).
template <int D, int NC, typename Real>
__global__ __launch_bounds__(kThreads) void k_collide(const CollideArgs a) {
  __shared__ double sh[4 * (D + 1)];
  const int i = a.plist[blockIdx.x];
  const size_t NVs = a.NV, cs = static_cast<size_t>(a.N) * NVs;
  const Real* ft = static_cast<const Real*>(a.ft) + static_cast<size_t>(i) * NVs;
  Real* fo = static_cast<Real*>(a.fo) + static_cast<size_t>(i) * NVs;
  double rho, U[3] = {0.0, 0.0, 0.0}, T;
  row_moments<D, NC, Real>(ft, cs, a.NV, a.nv, a.vmax, a.omega, sh, rho, U, T);
  if (threadIdx.x == 0) {
    a.rho[i] = rho;
    a.T[i] = T;
#pragma unroll
    for (int k = 0; k < D; ++k) a.U[static_cast<size_t>(k) * a.N + i] = U[k];
    if (!(rho > 0.0) || !(T > 0.0)) raise_error(a.err, BGK_ENONPHYS);
  }
  const double tau = a.kn * sqrt(2.0 / kPi) / (rho * sqrt(T));
  const double den = tau + a.dt;
  for (int q = threadIdx.x; q < a.NV; q += kThreads) {
    double v[3];
    velocity_of<D>(q, a.nv, a.vmax, v);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double M = maxwell<D>(c, rho, U, T, v);
      const double x = static_cast<double>(ft[c * cs + q]);
      fo[c * cs + q] = static_cast<Real>((tau * x + a.dt * M) / den);
    }
  }
}

template <typename Real, int D, int NC>
static void collide_t(const Ctx& c, const CollideArgs& a) {
  hipLaunchKernelGGL((k_collide<D, NC, Real>), dim3(a.count), dim3(kThreads), 0, c.stream, a);
}

static double omega_of(const bgk_config& cfg) {
  const double dv = 2.0 * cfg.vmax / static_cast<double>(cfg.nv - 1);
  double w = 1.0;
  for (int a = 0; a < cfg.dim; ++a) w = w * dv;
  return w;
}

hipError_t launch_collide(const Ctx& c, const void* ft, void* fout, double* rho, double* U,
                          double* T) {
  if (c.Ni == 0) return hipSuccess;
  CollideArgs a{c.N,       c.NV,  c.cfg.nv,  c.Ni,      c.cfg.vmax, omega_of(c.cfg), c.cfg.kn,
                c.cfg.dt,  c.d.cperm, ft, fout, rho, U, T, c.d.err};
  const bool f64 = c.cfg.precision == BGK_FP64;
  if (c.D == 2) {
    if (f64) collide_t<double, 2, 2>(c, a); else collide_t<float, 2, 2>(c, a);
  } else {
    if (f64) collide_t<double, 3, 1>(c, a); else collide_t<float, 3, 1>(c, a);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------ S7 walls
struct WallBcArgs {
  int N, NV, nv, cap, Nw, D;
  double vmax, omega, lid, wall_T;
  const int32_t* wall_list;
  const int32_t* wall_id;
  const int32_t* wcnt;
  const int32_t* widx;
  const double* wc0;
  void* f;
  double* rho;
  double* U;
  double* T;
  int32_t* err;
};

// Sum K doubles over a block of nw wavefronts in a fixed order (wavefront
// butterflies, then the waves in order); every thread receives the totals.
// sh must hold 16*K doubles.
template <int K>
__device__ __forceinline__ void block_sum_n(double (&v)[K], double* sh, int nw) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) sh[wid * K + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s = s + sh[w * K + k];
    v[k] = s;
  }
  __syncthreads();
}

// R consecutive elements of a row with the widest aligned vector access
// (p is aligned to R elements).
template <typename Real, int R>
__device__ __forceinline__ void load_vec(const Real* __restrict__ p, Real (&o)[R]) {
  constexpr int W = (R * sizeof(Real)) % 16 == 0 ? 16 / static_cast<int>(sizeof(Real)) : R;
  typedef Real V __attribute__((ext_vector_type(W)));
  const V* pv = reinterpret_cast<const V*>(__builtin_assume_aligned(p, W * sizeof(Real)));
#pragma unroll
  for (int i = 0; i < R / W; ++i) {
    const V x = pv[i];
#pragma unroll
    for (int w = 0; w < W; ++w) o[i * W + w] = x[w];
  }
}

// Diffuse reflection on wall particle b (one block of up to 256 threads, so
// that every wall particle's block is resident at once): arriving
// velocities (v.n <= 0, n the inward normal) take the interpolated interior
// value sum_e c0_e f_j; emitted ones take rho_w M[1, U_w, T_w] (Chu: G1 and
// T_w G1 scaled by rho_w) with rho_w from zero net mass flux; then the
// particle's moments in two passes (U first, then the centred second
// moment).  A thread handles R consecutive velocities (one vector load per
// stencil row and component, rows taken two at a time) and re-reads only
// the velocities it wrote itself.
template <int D, int NC, typename Real, int R>
__global__ __launch_bounds__(kThreads) void k_wall_bc(const WallBcArgs a) {
  __shared__ double sh[16 * (D + 1)];
  const int k = xcd_logical_block(blockIdx.x, gridDim.x);  // neighbouring walls share an L2
  const int nw = blockDim.x >> 6;
  const int b = a.wall_list[k];
  const int w = a.wall_id[b];
  const int axis = (w - 1) / 2;
  const double sgn = ((w - 1) % 2 == 0) ? 1.0 : -1.0;
  const bool is_lid = (w == 2 * D);
  double Uw[3] = {is_lid ? a.lid : 0.0, 0.0, 0.0};
  const int m = a.wcnt[k];
  const int32_t* row = a.widx + static_cast<size_t>(k) * a.cap;
  const double* c0 = a.wc0 + static_cast<size_t>(k) * a.cap;
  const size_t NVs = a.NV, cs = static_cast<size_t>(a.N) * NVs;
  Real* f = static_cast<Real*>(a.f);
  Real* fb = f + static_cast<size_t>(b) * NVs;
  const int step = R * static_cast<int>(blockDim.x);
  double flux[2] = {0.0, 0.0};
  for (int q0 = R * static_cast<int>(threadIdx.x); q0 < a.NV; q0 += step) {
    double s[NC][R];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int r = 0; r < R; ++r) s[c][r] = 0.0;
    // only arriving velocities are interpolated: skip the gather when all R
    // of this thread are emitted (whole waves on the faces normal to y, z)
    bool arriving = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      double v[3];
      velocity_of<D>(q0 + r, a.nv, a.vmax, v);
      arriving = arriving || sgn * v[axis] <= 0.0;
    }
    int e = arriving ? 0 : m;
    for (; e + 1 < m; e += 2) {
      Real x0[NC][R], x1[NC][R];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        load_vec<Real, R>(f + c * cs + static_cast<size_t>(row[e]) * NVs + q0, x0[c]);
        load_vec<Real, R>(f + c * cs + static_cast<size_t>(row[e + 1]) * NVs + q0, x1[c]);
      }
      const double w0 = c0[e], w1 = c0[e + 1];
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          s[c][r] = s[c][r] + w0 * static_cast<double>(x0[c][r]);
          s[c][r] = s[c][r] + w1 * static_cast<double>(x1[c][r]);
        }
    }
    if (e < m) {
      Real x0[NC][R];
#pragma unroll
      for (int c = 0; c < NC; ++c)
        load_vec<Real, R>(f + c * cs + static_cast<size_t>(row[e]) * NVs + q0, x0[c]);
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int r = 0; r < R; ++r) s[c][r] = s[c][r] + c0[e] * static_cast<double>(x0[c][r]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      double v[3];
      velocity_of<D>(q0 + r, a.nv, a.vmax, v);
      const double vn = sgn * v[axis];
      if (vn <= 0.0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const Real sr = static_cast<Real>(s[c][r]);
          fb[c * cs + q0 + r] = sr;
          if (c == 0) flux[0] = flux[0] + (-vn) * static_cast<double>(sr);
        }
      } else {
        flux[1] = flux[1] + vn * maxwell<D>(0, 1.0, Uw, a.wall_T, v);
      }
    }
  }
  block_sum_n<2>(flux, sh, nw);
  const double rho_w = flux[0] / flux[1];
  double sm[D + 1];
#pragma unroll
  for (int kk = 0; kk < D + 1; ++kk) sm[kk] = 0.0;
  for (int q0 = R * static_cast<int>(threadIdx.x); q0 < a.NV; q0 += step) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = q0 + r;
      double v[3];
      velocity_of<D>(q, a.nv, a.vmax, v);
      const double vn = sgn * v[axis];
      double x0;
      if (vn > 0.0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const Real y = static_cast<Real>(maxwell<D>(c, rho_w, Uw, a.wall_T, v));
          fb[c * cs + q] = y;
          if (c == 0) x0 = static_cast<double>(y);
        }
      } else {
        x0 = static_cast<double>(fb[q]);
      }
      sm[0] = sm[0] + x0;
#pragma unroll
      for (int kk = 0; kk < D; ++kk) sm[1 + kk] = sm[1 + kk] + v[kk] * x0;
    }
  }
  block_sum_n<D + 1>(sm, sh, nw);
  const double s0 = sm[0];
  double U[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < D; ++kk) U[kk] = sm[1 + kk] / s0;
  double e2[1] = {0.0};
  for (int q0 = R * static_cast<int>(threadIdx.x); q0 < a.NV; q0 += step) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = q0 + r;
      double v[3];
      velocity_of<D>(q, a.nv, a.vmax, v);
      double w2 = 0.0;
#pragma unroll
      for (int kk = 0; kk < D; ++kk) {
        const double wk = v[kk] - U[kk];
        w2 = w2 + wk * wk;
      }
      e2[0] = e2[0] + w2 * static_cast<double>(fb[q]);
      if (NC == 2) e2[0] = e2[0] + static_cast<double>(fb[cs + q]);
    }
  }
  block_sum_n<1>(e2, sh, nw);
  if (threadIdx.x == 0) {
    const double rho = a.omega * s0;
    const double T = e2[0] / (3.0 * s0);
    a.rho[b] = rho;
    a.T[b] = T;
#pragma unroll
    for (int kk = 0; kk < D; ++kk) a.U[static_cast<size_t>(kk) * a.N + b] = U[kk];
    if (!(rho > 0.0) || !(T > 0.0) || m == 0) raise_error(a.err, BGK_ENONPHYS);
  }
}

template <int D, int NC, typename Real>
static void wall_bc_t(const Ctx& c, const WallBcArgs& a) {
  const int R = (c.cfg.nv % 4 == 0) ? 4 : 2;  // nv is even
  const int lanes = c.NV / R;
  dim3 g(c.Nw), t(std::min(kThreads, (lanes + 63) / 64 * 64));
  if (R == 4) hipLaunchKernelGGL((k_wall_bc<D, NC, Real, 4>), g, t, 0, c.stream, a);
  else hipLaunchKernelGGL((k_wall_bc<D, NC, Real, 2>), g, t, 0, c.stream, a);
}

hipError_t launch_wall_bc(const Ctx& c, void* f, double* rho, double* U, double* T) {
  if (c.Nw == 0) return hipSuccess;
  WallBcArgs a{c.N,          c.NV,      c.cfg.nv,      c.cap,  c.Nw,   c.D,    c.cfg.vmax,
               omega_of(c.cfg), c.lid,  c.cfg.wall_T,  c.d.wall_list, c.d.wall_id, c.d.wcnt,
               c.d.widx,     c.d.wc0,   f,             rho,    U,      T,      c.d.err};
  const bool f64 = c.cfg.precision == BGK_FP64;
  if (c.D == 2) {
    if (f64) wall_bc_t<2, 2, double>(c, a); else wall_bc_t<2, 2, float>(c, a);
  } else {
    if (f64) wall_bc_t<3, 1, double>(c, a); else wall_bc_t<3, 1, float>(c, a);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------ S8 motion
__global__ void k_move(int N, int D, int Ni, double dt, double lo, double hi,
                       const int32_t* __restrict__ plist, const double* __restrict__ U,
                       double* __restrict__ x, int32_t* __restrict__ err) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= Ni) return;
  const int i = plist[k];
  int clamped = 0;
  for (int a = 0; a < D; ++a) {
    double y = x[static_cast<size_t>(a) * N + i] + dt * U[static_cast<size_t>(a) * N + i];
    if (y < lo) {
      y = lo;
      ++clamped;
    }
    if (y > hi) {
      y = hi;
      ++clamped;
    }
    x[static_cast<size_t>(a) * N + i] = y;
  }
  if (clamped) atomicAdd(&err[1], clamped);
}

hipError_t launch_move(const Ctx& c, double* x, const double* U) {
  if (c.Ni == 0) return hipSuccess;
  const double lo = 0.1 * c.cfg.dx, hi = 1.0 - 0.1 * c.cfg.dx;
  hipLaunchKernelGGL(k_move, dim3((c.Ni + 255) / 256), dim3(256), 0, c.stream, c.N, c.D, c.Ni,
                     c.cfg.dt, lo, hi, c.d.cperm, U, x, c.d.err);
  return hipGetLastError();
}

// ------------------------------------------------------------ moments, M
template <int D, int NC, typename Real>
__global__ __launch_bounds__(kThreads) void k_moments(int N, int NV, int nv, double vmax,
                                                       double omega, const void* fv, double* rho,
                                                       double* U, double* T) {
  __shared__ double sh[4 * (D + 1)];
  const int i = blockIdx.x;
  const size_t NVs = NV, cs = static_cast<size_t>(N) * NVs;
  const Real* row = static_cast<const Real*>(fv) + static_cast<size_t>(i) * NVs;
  double r, u[3] = {0.0, 0.0, 0.0}, t;
  row_moments<D, NC, Real>(row, cs, NV, nv, vmax, omega, sh, r, u, t);
  if (threadIdx.x == 0) {
    rho[i] = r;
    T[i] = t;
#pragma unroll
    for (int k = 0; k < D; ++k) U[static_cast<size_t>(k) * N + i] = u[k];
  }
}

hipError_t launch_moments(const Ctx& c, const void* f, double* rho, double* U, double* T) {
  const bool f64 = c.cfg.precision == BGK_FP64;
  const double om = omega_of(c.cfg);
  dim3 g(c.N), t(kThreads);
  if (c.D == 2) {
    if (f64) hipLaunchKernelGGL((k_moments<2, 2, double>), g, t, 0, c.stream, c.N, c.NV, c.cfg.nv, c.cfg.vmax, om, f, rho, U, T);
    else hipLaunchKernelGGL((k_moments<2, 2, float>), g, t, 0, c.stream, c.N, c.NV, c.cfg.nv, c.cfg.vmax, om, f, rho, U, T);
  } else {
    if (f64) hipLaunchKernelGGL((k_moments<3, 1, double>), g, t, 0, c.stream, c.N, c.NV, c.cfg.nv, c.cfg.vmax, om, f, rho, U, T);
    else hipLaunchKernelGGL((k_moments<3, 1, float>), g, t, 0, c.stream, c.N, c.NV, c.cfg.nv, c.cfg.vmax, om, f, rho, U, T);
  }
  return hipGetLastError();
}

template <int D, int NC, typename Real>
__global__ __launch_bounds__(kThreads) void k_maxwellian(int N, int NV, int nv, double vmax,
                                                          const double* __restrict__ rho,
                                                          const double* __restrict__ U,
                                                          const double* __restrict__ T, void* fv) {
  const int i = blockIdx.x;
  const size_t NVs = NV, cs = static_cast<size_t>(N) * NVs;
  Real* row = static_cast<Real*>(fv) + static_cast<size_t>(i) * NVs;
  double u[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < D; ++k) u[k] = U[static_cast<size_t>(k) * N + i];
  const double r = rho[i], t = T[i];
  for (int q = threadIdx.x; q < NV; q += kThreads) {
    double v[3];
    velocity_of<D>(q, nv, vmax, v);
#pragma unroll
    for (int c = 0; c < NC; ++c) row[c * cs + q] = static_cast<Real>(maxwell<D>(c, r, u, t, v));
  }
}

hipError_t launch_maxwellian(const Ctx& c, const double* rho, const double* U, const double* T,
                             void* f) {
  const bool f64 = c.cfg.precision == BGK_FP64;
  dim3 g(c.N), t(kThreads);
  if (c.D == 2) {
    if (f64) hipLaunchKernelGGL((k_maxwellian<2, 2, double>), g, t, 0, c.stream, c.N, c.NV, c.cfg.nv, c.cfg.vmax, rho, U, T, f);
    else hipLaunchKernelGGL((k_maxwellian<2, 2, float>), g, t, 0, c.stream, c.N, c.NV, c.cfg.nv, c.cfg.vmax, rho, U, T, f);
  } else {
    if (f64) hipLaunchKernelGGL((k_maxwellian<3, 1, double>), g, t, 0, c.stream, c.N, c.NV, c.cfg.nv, c.cfg.vmax, rho, U, T, f);
    else hipLaunchKernelGGL((k_maxwellian<3, 1, float>), g, t, 0, c.stream, c.N, c.NV, c.cfg.nv, c.cfg.vmax, rho, U, T, f);
  }
  return hipGetLastError();
}

}  // namespace bgk
