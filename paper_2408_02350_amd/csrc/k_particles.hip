// Particle management (Sec. 3.5.2, adding and removing points): two
// interior particles that come too close are replaced by one at their
// midpoint, particles are added where holes open, and f at every new
// particle is filled by least squares from the old cloud.
//
// Selection (the paper gives no thresholds or rule; this is the reading the
// library documents):
//  - merge: interior particles i < j that are each other's nearest interior
//    neighbour within h (ties to the lower index) and closer than the merge
//    radius become one interior particle at 0.5 (x_i + x_j);
//  - hole: an interior node k dx (0 < k < n-1 on every axis, n - 1 = 1/dx)
//    of the initial lattice with no particle of the merged cloud within the
//    hole radius gets a new interior particle;
//  - f at a new particle is the value row of the old cloud at its position
//    (the rule of the wall rows) applied to every velocity and component;
//    its rho, U, T are the moments of that f; the other particles keep f,
//    rho, U, T;
//  - the new cloud lists the untouched particles in their old order, then
//    the midpoints by the lower index of their pair, then the hole particles
//    by node index.
// Every decision is an FP64 comparison of a squared distance summed
// component by component, so the plan is exact and deterministic.
#include <climits>

#include "cloud_common.h"

namespace bgk {

CloudView cloud_view(const Ctx& c, const double* x);

namespace {

// Nearest interior neighbour of each interior particle within h (one wave
// per particle; -1 for wall particles and for none).
template <int D>
__global__ __launch_bounds__(64) void k_pm_nearest(int N, int nca, int ncell, double h2,
                                                   const double* __restrict__ x,
                                                   const double* __restrict__ xs,
                                                   const int32_t* __restrict__ wall_id,
                                                   const int32_t* __restrict__ cstart,
                                                   const int32_t* __restrict__ cperm,
                                                   int32_t* __restrict__ nn) {
  constexpr int NR = (D == 2 ? 9 : 27);
  __shared__ int32_t rb[NR], rpre[NR + 1];
  const int i = blockIdx.x, lane = threadIdx.x;
  if (wall_id[i] != 0) {
    if (lane == 0) nn[i] = -1;
    return;
  }
  double xi[D];
  int ci[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    xi[a] = x[static_cast<int64_t>(a) * N + i];
    ci[a] = cell_coord(xi[a], nca);
  }
  const int nr = cell_ranges<D, 1>(ci, nca, ncell, false, cstart, rb, rpre);
  const int total = rpre[nr];
  double best = 0.0;
  int bj = INT_MAX;
  for (int c = lane; c < total; c += kWave) {
    const int p = cand_slot(c, nr, rb, rpre);
    const int j = cperm[p];
    if (j == i) continue;
    double r2 = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double dl = xs[static_cast<int64_t>(a) * N + p] - xi[a];
      r2 = r2 + dl * dl;
    }
    if (r2 <= h2 && (bj == INT_MAX || r2 < best || (r2 == best && j < bj))) {
      best = r2;
      bj = j;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o, 64);
    const int oj = __shfl_xor(bj, o, 64);
    if (oj != INT_MAX && (bj == INT_MAX || ob < best || (ob == best && oj < bj))) {
      best = ob;
      bj = oj;
    }
  }
  if (lane == 0) nn[i] = bj == INT_MAX ? -1 : bj;
}

// Mutual nearest pairs closer than the merge radius (partner[] starts at -1;
// the lower index writes both entries, and a particle is in at most one
// mutual pair).
__global__ void k_pm_pairs(int N, int D, double rm2, const double* __restrict__ x,
                           const int32_t* __restrict__ nn, int32_t* __restrict__ partner) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int j = nn[i];
  if (j <= i || nn[j] != i) return;
  double r2 = 0.0;
  for (int a = 0; a < D; ++a) {
    const double dl = x[static_cast<int64_t>(a) * N + j] - x[static_cast<int64_t>(a) * N + i];
    r2 = r2 + dl * dl;
  }
  if (r2 < rm2) {
    partner[i] = j;
    partner[j] = i;
  }
}

// Flags for the scans: kept (not in a pair) and lower member of a pair.
__global__ void k_pm_flags(int N, const int32_t* __restrict__ partner, int32_t* __restrict__ keep,
                           int32_t* __restrict__ mid) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int p = partner[i];
  keep[i] = p < 0 ? 1 : 0;
  mid[i] = p > i ? 1 : 0;
}

template <int D>
__device__ __forceinline__ bool node_of(int64_t k, int nl, double dx, double* y) {
  bool inner = true;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const int ka = static_cast<int>(k % nl);
    k /= nl;
    inner = inner && ka > 0 && ka < nl - 1;
    y[a] = static_cast<double>(ka) * dx;
  }
  return inner;
}

// Hole flag of each lattice node (one wave per node): no particle of the
// merged cloud within the hole radius.  A pair is seen through its lower
// member, at the midpoint; with hole radius + merge radius <= h that member
// lies in the 3^d cells around the node whenever the midpoint is in range.
template <int D>
__global__ __launch_bounds__(64) void k_pm_holes(int N, int nca, int ncell, int nl, double dx,
                                                 double rh2, const double* __restrict__ x,
                                                 const double* __restrict__ xs,
                                                 const int32_t* __restrict__ cstart,
                                                 const int32_t* __restrict__ cperm,
                                                 const int32_t* __restrict__ partner,
                                                 int32_t* __restrict__ hole) {
  constexpr int NR = (D == 2 ? 9 : 27) * 2;
  __shared__ int32_t rb[NR], rpre[NR + 1];
  const int64_t k = blockIdx.x;
  const int lane = threadIdx.x;
  double y[D];
  if (!node_of<D>(k, nl, dx, y)) {
    if (lane == 0) hole[k] = 0;
    return;
  }
  int cy[D];
#pragma unroll
  for (int a = 0; a < D; ++a) cy[a] = cell_coord(y[a], nca);
  const int nr = cell_ranges<D, 1>(cy, nca, ncell, true, cstart, rb, rpre);
  const int total = rpre[nr];
  bool covered = false;
  for (int c = lane; c < total; c += kWave) {
    const int p = cand_slot(c, nr, rb, rpre);
    const int j = cperm[p];
    const int pj = partner[j];
    if (pj >= 0 && pj < j) continue;
    double r2 = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double q = pj > j ? 0.5 * (x[static_cast<int64_t>(a) * N + j] +
                                       x[static_cast<int64_t>(a) * N + pj])
                              : xs[static_cast<int64_t>(a) * N + p];
      const double dl = q - y[a];
      r2 = r2 + dl * dl;
    }
    covered = covered || r2 <= rh2;
  }
  const bool any = __ballot(covered) != 0;
  if (lane == 0) hole[k] = any ? 0 : 1;
}

struct PlaceArgs {
  int N, Nn, D;
  const double* x;
  const int32_t* wall_id;
  const double* rho;
  const double* U;
  const double* T;
  const int32_t* partner;
  const int32_t* keep;  // exclusive scans, [N] holds the totals
  const int32_t* mid;
  double* x_new;
  int32_t* wall_id_new;
  double* rho_new;
  double* U_new;
  double* T_new;
};

// Positions, owners and carried state of the kept particles and midpoints.
__global__ void k_pm_place(const PlaceArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  const int p = a.partner[i];
  if (p < 0) {
    const int q = a.keep[i];
    for (int d = 0; d < a.D; ++d) {
      a.x_new[static_cast<int64_t>(d) * a.Nn + q] = a.x[static_cast<int64_t>(d) * a.N + i];
      a.U_new[static_cast<int64_t>(d) * a.Nn + q] = a.U[static_cast<int64_t>(d) * a.N + i];
    }
    a.wall_id_new[q] = a.wall_id[i];
    a.rho_new[q] = a.rho[i];
    a.T_new[q] = a.T[i];
  } else if (p > i) {
    const int q = a.keep[a.N] + a.mid[i];
    for (int d = 0; d < a.D; ++d)
      a.x_new[static_cast<int64_t>(d) * a.Nn + q] =
          0.5 * (a.x[static_cast<int64_t>(d) * a.N + i] + a.x[static_cast<int64_t>(d) * a.N + p]);
    a.wall_id_new[q] = 0;
  }
}

template <int D>
__global__ void k_pm_place_holes(int64_t nodes, int nl, double dx, int N, int Nn,
                                 const int32_t* __restrict__ keep, const int32_t* __restrict__ mid,
                                 const int32_t* __restrict__ hole, double* __restrict__ x_new,
                                 int32_t* __restrict__ wall_id_new) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= nodes || hole[k + 1] == hole[k]) return;
  const int q = keep[N] + mid[N] + hole[k];
  double y[D];
  node_of<D>(k, nl, dx, y);
#pragma unroll
  for (int a = 0; a < D; ++a) x_new[static_cast<int64_t>(a) * Nn + q] = y[a];
  wall_id_new[q] = 0;
}

// f rows of the kept particles (one block per old particle).
template <typename Real>
__global__ void k_pm_copy_rows(int N, int Nn, int NC, int NV, const int32_t* __restrict__ partner,
                               const int32_t* __restrict__ keep, const Real* __restrict__ f,
                               Real* __restrict__ f_new) {
  const int i = blockIdx.x;
  if (partner[i] >= 0) return;
  const int q = keep[i];
  for (int c = 0; c < NC; ++c) {
    const Real* src = f + (static_cast<int64_t>(c) * N + i) * NV;
    Real* dst = f_new + (static_cast<int64_t>(c) * Nn + q) * NV;
    for (int v = threadIdx.x; v < NV; v += blockDim.x) dst[v] = src[v];
  }
}

struct NewRowArgs {
  CloudView cv;  // the old cloud
  int Nn, first, NV, nv;
  double vmax, omega;
  const void* f;
  const double* x_new;
  void* f_new;
  double* rho_new;
  double* U_new;
  double* T_new;
  int32_t* err;
};

// One wave per new particle q = first + block: its value row in the old
// cloud, the interpolated row of every component, then its moments (two
// passes, FP64; each lane re-reads only the velocities it wrote).
template <int D, int NC, typename Real>
__global__ __launch_bounds__(64) void k_pm_new_rows(const NewRowArgs a) {
  __shared__ ValueRowSm<D> sm;
  __shared__ double cw[256];
  const int q = a.first + blockIdx.x, lane = threadIdx.x;
  double xq[D];
#pragma unroll
  for (int d = 0; d < D; ++d) xq[d] = a.x_new[static_cast<int64_t>(d) * a.Nn + q];
  double hb = 0.0;
  const int m = value_row<D>(a.cv, xq, sm, hb);
  if (m < 0) {
    if (lane == 0) raise_error(a.err, m == -2 ? BGK_ENBR_OVERFLOW : BGK_ESINGULAR);
    return;
  }
  for (int e = lane; e < m; e += kWave) cw[e] = value_weight<D>(sm, e);
  __syncthreads();
  const Real* f = static_cast<const Real*>(a.f);
  Real* fo = static_cast<Real*>(a.f_new);
  const int64_t N = a.cv.N;
  double s0 = 0.0, s1[D];
#pragma unroll
  for (int d = 0; d < D; ++d) s1[d] = 0.0;
  for (int v = lane; v < a.NV; v += kWave) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double s = 0.0;
      for (int e = 0; e < m; ++e)
        s = s + cw[e] * static_cast<double>(f[(c * N + sm.srt[e]) * a.NV + v]);
      const Real y = static_cast<Real>(s);
      fo[(static_cast<int64_t>(c) * a.Nn + q) * a.NV + v] = y;
      if (c == 0) {
        double vel[3];
        velocity_of<D>(v, a.nv, a.vmax, vel);
        const double f1 = static_cast<double>(y);
        s0 = s0 + f1;
#pragma unroll
        for (int d = 0; d < D; ++d) s1[d] = s1[d] + vel[d] * f1;
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    s0 += __shfl_xor(s0, o, 64);
#pragma unroll
    for (int d = 0; d < D; ++d) s1[d] += __shfl_xor(s1[d], o, 64);
  }
  double U[D];
#pragma unroll
  for (int d = 0; d < D; ++d) U[d] = s1[d] / s0;
  double e2 = 0.0;
  for (int v = lane; v < a.NV; v += kWave) {
    double vel[3];
    velocity_of<D>(v, a.nv, a.vmax, vel);
    double w2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const double w = vel[d] - U[d];
      w2 = w2 + w * w;
    }
    e2 = e2 + w2 * static_cast<double>(fo[static_cast<int64_t>(q) * a.NV + v]);
    if (NC == 2) e2 = e2 + static_cast<double>(fo[(static_cast<int64_t>(a.Nn) + q) * a.NV + v]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) e2 += __shfl_xor(e2, o, 64);
  if (lane == 0) {
    const double rho = a.omega * s0, T = e2 / (3.0 * s0);
    a.rho_new[q] = rho;
    a.T_new[q] = T;
#pragma unroll
    for (int d = 0; d < D; ++d) a.U_new[static_cast<int64_t>(d) * a.Nn + q] = U[d];
    if (!(rho > 0.0) || !(T > 0.0)) raise_error(a.err, BGK_ENONPHYS);
  }
}

inline unsigned grid_for(int64_t n, int t) { return static_cast<unsigned>((n + t - 1) / t); }

}  // namespace

hipError_t launch_pm_plan(Ctx& c, const double* x, double rm, double rh) {
  const Pm& p = c.pm;
  hipError_t e = launch_cells(c, x);
  if (e != hipSuccess) return e;
  const double h2 = c.cfg.h * c.cfg.h;
  if (c.D == 2)
    hipLaunchKernelGGL(k_pm_nearest<2>, dim3(c.N), dim3(kWave), 0, c.stream, c.N, c.nca, c.ncell,
                       h2, x, c.d.xs, c.d.wall_id, c.d.cstart, c.d.cperm, p.nn);
  else
    hipLaunchKernelGGL(k_pm_nearest<3>, dim3(c.N), dim3(kWave), 0, c.stream, c.N, c.nca, c.ncell,
                       h2, x, c.d.xs, c.d.wall_id, c.d.cstart, c.d.cperm, p.nn);
  e = launch_fill_i32(c.stream, p.partner, c.N, -1);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pm_pairs, dim3(grid_for(c.N, 256)), dim3(256), 0, c.stream, c.N, c.D,
                     rm * rm, x, p.nn, p.partner);
  hipLaunchKernelGGL(k_pm_flags, dim3(grid_for(c.N, 256)), dim3(256), 0, c.stream, c.N, p.partner,
                     p.keep, p.mid);
  if (c.D == 2)
    hipLaunchKernelGGL(k_pm_holes<2>, dim3(static_cast<unsigned>(c.nodes)), dim3(kWave), 0,
                       c.stream, c.N, c.nca, c.ncell, c.nl, c.cfg.dx, rh * rh, x, c.d.xs,
                       c.d.cstart, c.d.cperm, p.partner, p.hole);
  else
    hipLaunchKernelGGL(k_pm_holes<3>, dim3(static_cast<unsigned>(c.nodes)), dim3(kWave), 0,
                       c.stream, c.N, c.nca, c.ncell, c.nl, c.cfg.dx, rh * rh, x, c.d.xs,
                       c.d.cstart, c.d.cperm, p.partner, p.hole);
  e = hipGetLastError();
  if (e == hipSuccess) e = launch_scan(c.stream, p.keep, c.N);
  if (e == hipSuccess) e = launch_scan(c.stream, p.mid, c.N);
  if (e == hipSuccess) e = launch_scan(c.stream, p.hole, static_cast<int>(c.nodes));
  return e;
}

hipError_t launch_pm_apply(const Ctx& c, const double* x, const void* f, const double* rho,
                           const double* U, const double* T, int Nn, int n_keep, int n_new,
                           double* x_new, int32_t* wall_id_new, void* f_new, double* rho_new,
                           double* U_new, double* T_new) {
  const Pm& p = c.pm;
  PlaceArgs pa{c.N, Nn, c.D, x, c.d.wall_id, rho, U, T, p.partner, p.keep, p.mid,
               x_new, wall_id_new, rho_new, U_new, T_new};
  hipLaunchKernelGGL(k_pm_place, dim3(grid_for(c.N, 256)), dim3(256), 0, c.stream, pa);
  if (c.D == 2)
    hipLaunchKernelGGL(k_pm_place_holes<2>, dim3(grid_for(c.nodes, 256)), dim3(256), 0, c.stream,
                       c.nodes, c.nl, c.cfg.dx, c.N, Nn, p.keep, p.mid, p.hole, x_new,
                       wall_id_new);
  else
    hipLaunchKernelGGL(k_pm_place_holes<3>, dim3(grid_for(c.nodes, 256)), dim3(256), 0, c.stream,
                       c.nodes, c.nl, c.cfg.dx, c.N, Nn, p.keep, p.mid, p.hole, x_new,
                       wall_id_new);
  const bool f64 = c.cfg.precision == BGK_FP64;
  if (f64)
    hipLaunchKernelGGL(k_pm_copy_rows<double>, dim3(c.N), dim3(256), 0, c.stream, c.N, Nn, c.NC,
                       c.NV, p.partner, p.keep, static_cast<const double*>(f),
                       static_cast<double*>(f_new));
  else
    hipLaunchKernelGGL(k_pm_copy_rows<float>, dim3(c.N), dim3(256), 0, c.stream, c.N, Nn, c.NC,
                       c.NV, p.partner, p.keep, static_cast<const float*>(f),
                       static_cast<float*>(f_new));
  if (n_new > 0) {
    NewRowArgs na{cloud_view(c, x), Nn, n_keep, c.NV, c.cfg.nv, c.cfg.vmax, omega_of(c.cfg), f,
                  x_new, f_new, rho_new, U_new, T_new, c.d.err};
    const dim3 g(n_new), b(kWave);
    if (c.D == 2) {
      if (f64) hipLaunchKernelGGL((k_pm_new_rows<2, 2, double>), g, b, 0, c.stream, na);
      else hipLaunchKernelGGL((k_pm_new_rows<2, 2, float>), g, b, 0, c.stream, na);
    } else {
      if (f64) hipLaunchKernelGGL((k_pm_new_rows<3, 1, double>), g, b, 0, c.stream, na);
      else hipLaunchKernelGGL((k_pm_new_rows<3, 1, float>), g, b, 0, c.stream, na);
    }
  }
  return hipGetLastError();
}

}  // namespace bgk
