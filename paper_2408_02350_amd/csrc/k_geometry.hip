// Geometry of one step: cell list, neighbour search (S1), weighted
// least-squares operators and edge frames (S2-S3), boundary interpolation
// rows (S7 part 1) and the patch unions the transport kernel walks.
//
// These kernels are cheap next to the transport (O(N m B^2) against
// O(N N_v m)); they are written for exactness first: FP64 throughout, the
// squared-distance predicate and the normal equations in the plain operation
// order (no contraction), deterministic outputs (sorted lists, no atomics on
// values).
#include <climits>

#include "device_common.h"

namespace bgk {

// ------------------------------------------------------------------ utils
__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_f64(double* p, int64_t n, double v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_copy_i32(const int32_t* __restrict__ s, int32_t* __restrict__ d, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}

static inline unsigned blocks_for(int64_t n, int t) { return static_cast<unsigned>((n + t - 1) / t); }

hipError_t launch_fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_f64(hipStream_t s, double* p, int64_t n, double v) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_copy_i32(hipStream_t s, const int32_t* src, int32_t* dst, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_i32, dim3(blocks_for(n, 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

// ------------------------------------------------------------ cell list
// Key of a particle: its cell (cells of size 1/nca >= h, x fastest), plus
// ncell for wall particles, so that the sorted permutation holds all interior
// particles first (in cell order) and the wall particles after them.
template <int D>
__global__ void k_cell_count(int N, int nca, int ncell, const double* __restrict__ x,
                             const int32_t* __restrict__ wall_id, int32_t* __restrict__ key,
                             int32_t* __restrict__ count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int c = 0, mul = 1;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    c += cell_coord(x[static_cast<int64_t>(a) * N + i], nca) * mul;
    mul *= nca;
  }
  const int k = c + (wall_id[i] != 0 ? ncell : 0);
  key[i] = k;
  atomicAdd(&count[k], 1);
}

// Exclusive scan of n int32 in place (one block of 1024 threads walking the
// array in chunks); a[n] receives the total.
__global__ __launch_bounds__(1024) void k_scan_inplace(int32_t* a, int n) {
  constexpr int PER = 8;
  __shared__ int32_t wsum[16];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  int carry = 0;
  for (int base = 0; base < n; base += 1024 * PER) {
    int v[PER];
    int s = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = base + tid * PER + k;
      v[k] = idx < n ? a[idx] : 0;
      s += v[k];
    }
    int incl = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o, 64);
      if (lane >= o) incl += t;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    if (wid == 0) {
      int w = lane < 16 ? wsum[lane] : 0;
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        const int t = __shfl_up(w, o, 64);
        if (lane >= o) w += t;
      }
      if (lane < 16) wsum[lane] = w;
    }
    __syncthreads();
    int run = carry + (incl - s) + (wid > 0 ? wsum[wid - 1] : 0);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = base + tid * PER + k;
      if (idx < n) a[idx] = run;
      run += v[k];
    }
    carry += wsum[15];
    __syncthreads();
  }
  if (tid == 0) a[n] = carry;
}

__global__ void k_cell_scatter(int N, const int32_t* __restrict__ key, int32_t* __restrict__ cursor,
                               int32_t* __restrict__ perm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int pos = atomicAdd(&cursor[key[i]], 1);
  perm[pos] = i;
}

// Sort each cell range ascending so that the permutation is deterministic.
__global__ void k_cell_sort(int nkeys, const int32_t* __restrict__ start, int32_t* __restrict__ perm) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nkeys) return;
  const int b = start[k], e = start[k + 1];
  for (int p = b + 1; p < e; ++p) {
    const int v = perm[p];
    int s = p;
    while (s > b && perm[s - 1] > v) {
      perm[s] = perm[s - 1];
      --s;
    }
    perm[s] = v;
  }
}

hipError_t launch_cells(const Ctx& c, const double* x) {
  const Dev& d = c.d;
  const int nkeys = 2 * c.ncell;
  hipError_t e = launch_fill_i32(c.stream, d.cstart, nkeys + 1, 0);
  if (e != hipSuccess) return e;
  if (c.D == 2)
    hipLaunchKernelGGL(k_cell_count<2>, dim3(blocks_for(c.N, 256)), dim3(256), 0, c.stream, c.N,
                       c.nca, c.ncell, x, d.wall_id, d.key, d.cstart);
  else
    hipLaunchKernelGGL(k_cell_count<3>, dim3(blocks_for(c.N, 256)), dim3(256), 0, c.stream, c.N,
                       c.nca, c.ncell, x, d.wall_id, d.key, d.cstart);
  hipLaunchKernelGGL(k_scan_inplace, dim3(1), dim3(1024), 0, c.stream, d.cstart, nkeys);
  e = launch_copy_i32(c.stream, d.cstart, d.ccursor, nkeys);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cell_scatter, dim3(blocks_for(c.N, 256)), dim3(256), 0, c.stream, c.N,
                     d.key, d.ccursor, d.cperm);
  hipLaunchKernelGGL(k_cell_sort, dim3(blocks_for(nkeys, 256)), dim3(256), 0, c.stream, nkeys,
                     d.cstart, d.cperm);
  return hipGetLastError();
}

// ------------------------------------------------------------ S1 neighbours
// One thread per particle scans the 3^D cells around its own (both the
// interior and the wall range of each) and inserts every j with
// |x_j - x_i|^2 <= h^2 into its row in ascending order.
template <int D>
__global__ void k_neighbors(int N, int nca, int ncell, double h2, int cap,
                            const double* __restrict__ x, const int32_t* __restrict__ cstart,
                            const int32_t* __restrict__ cperm, int32_t* __restrict__ cnt,
                            int32_t* __restrict__ idx, int32_t* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double xi[D];
  int ci[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    xi[a] = x[static_cast<int64_t>(a) * N + i];
    ci[a] = cell_coord(xi[a], nca);
  }
  int32_t* row = idx + static_cast<int64_t>(i) * cap;
  int m = 0;
  const int zlo = (D == 3) ? -1 : 0, zhi = (D == 3) ? 1 : 0;
  for (int dz = zlo; dz <= zhi; ++dz) {
    const int cz = (D == 3) ? ci[D - 1] + dz : 0;
    if (D == 3 && (cz < 0 || cz >= nca)) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      const int cy = ci[1] + dy;
      if (cy < 0 || cy >= nca) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        const int cx = ci[0] + dx;
        if (cx < 0 || cx >= nca) continue;
        const int cell = cx + nca * (cy + nca * cz);
        for (int part = 0; part < 2; ++part) {
          const int k = cell + part * ncell;
          const int pe = cstart[k + 1];
          for (int p = cstart[k]; p < pe; ++p) {
            const int j = cperm[p];
            double r2 = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) {
              const double dl = x[static_cast<int64_t>(a) * N + j] - xi[a];
              r2 = r2 + dl * dl;
            }
            if (r2 <= h2) {
              if (m < cap) {
                int s = m;
                while (s > 0 && row[s - 1] > j) {
                  row[s] = row[s - 1];
                  --s;
                }
                row[s] = j;
              }
              ++m;
            }
          }
        }
      }
    }
  }
  cnt[i] = m;
  atomicMax(&err[2], m);
  if (m > cap) raise_error(err, BGK_ENBR_OVERFLOW);
}

hipError_t launch_neighbors(const Ctx& c, const double* x, int32_t* cnt, int32_t* idx) {
  const double h2 = c.cfg.h * c.cfg.h;
  if (c.D == 2)
    hipLaunchKernelGGL(k_neighbors<2>, dim3(blocks_for(c.N, 128)), dim3(128), 0, c.stream, c.N,
                       c.nca, c.ncell, h2, c.cap, x, c.d.cstart, c.d.cperm, cnt, idx, c.d.err);
  else
    hipLaunchKernelGGL(k_neighbors<3>, dim3(blocks_for(c.N, 128)), dim3(128), 0, c.stream, c.N,
                       c.nca, c.ncell, h2, c.cap, x, c.d.cstart, c.d.cperm, cnt, idx, c.d.err);
  return hipGetLastError();
}

// ------------------------------------------------------------ S2-S3 WLS
template <int D, int DEG>
struct Basis {
  static constexpr int B = (DEG == 1) ? D + 1 : (D == 2 ? 6 : 10);
  static constexpr int NT = B * (B + 1) / 2;  // packed lower triangle
  __device__ static __forceinline__ void eval(const double* y, double* p) {
    p[0] = 1.0;
#pragma unroll
    for (int a = 0; a < D; ++a) p[1 + a] = y[a];
    if (DEG == 2) {
      int k = D + 1;
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a; b < D; ++b) p[k++] = y[a] * y[b];
    }
  }
};

__device__ __forceinline__ constexpr int tri(int r, int s) { return r * (r + 1) / 2 + s; }

// In-place Cholesky of a packed lower triangle; false on a non-positive pivot.
template <int B>
__device__ __forceinline__ bool cholesky_packed(double* A) {
#pragma unroll
  for (int j = 0; j < B; ++j) {
    double s = A[tri(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) s = s - A[tri(j, k)] * A[tri(j, k)];
    if (!(s > 0.0)) return false;
    const double ljj = sqrt(s);
    A[tri(j, j)] = ljj;
#pragma unroll
    for (int i = j + 1; i < B; ++i) {
      double t = A[tri(i, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) t = t - A[tri(i, k)] * A[tri(j, k)];
      A[tri(i, j)] = t / ljj;
    }
  }
  return true;
}

// Solve L L^T z = e_col with L packed.
template <int B>
__device__ __forceinline__ void chol_solve_unit(const double* L, int col, double* z) {
  double y[B];
#pragma unroll
  for (int i = 0; i < B; ++i) {
    double s = (i == col) ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < i; ++k) s = s - L[tri(i, k)] * y[k];
    y[i] = s / L[tri(i, i)];
  }
#pragma unroll
  for (int i = B - 1; i >= 0; --i) {
    double s = y[i];
#pragma unroll
    for (int k = i + 1; k < B; ++k) s = s - L[tri(k, i)] * z[k];
    z[i] = s / L[tri(i, i)];
  }
}

// Edge frame of x_j - x_i (Sec. 3.4.2) without trigonometric calls: in 2D
// n = dl/|dl|, t = n turned by +90 degrees; in 3D n = dl/r, t = (cos th cos
// phi, cos th sin phi, -sin th), b = (-sin phi, cos phi, 0) with sin th =
// r_xy/r, cos th = dz/r, cos phi = dx/r_xy, sin phi = dy/r_xy (phi = 0 on the
// z axis, as atan2(0, 0) = 0).
template <int D>
__device__ __forceinline__ void edge_frame(const double* dl, double* n, double* t, double* b) {
  if (D == 2) {
    const double r = sqrt(dl[0] * dl[0] + dl[1] * dl[1]);
    n[0] = dl[0] / r;
    n[1] = dl[1] / r;
    t[0] = -n[1];
    t[1] = n[0];
  } else {
    const double rxy = sqrt(dl[0] * dl[0] + dl[1] * dl[1]);
    const double r = sqrt(dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2]);
    const double st = rxy / r, ct = dl[2] / r;
    double cp = 1.0, sp = 0.0;
    if (rxy > 0.0) {
      cp = dl[0] / rxy;
      sp = dl[1] / rxy;
    }
    n[0] = st * cp;
    n[1] = st * sp;
    n[2] = ct;
    t[0] = ct * cp;
    t[1] = ct * sp;
    t[2] = -st;
    b[0] = -sp;
    b[1] = cp;
    b[2] = 0.0;
  }
}

struct WlsArgs {
  int N, cap, Ni, deg_cfg;
  double h, alpha;
  const double* x;
  const int32_t* plist;  // interior particles
  const int32_t* cnt;
  const int32_t* idx;
  double* grad;          // may be null
  double* ops;           // may be null
  float* ops32;          // may be null
  int32_t* degree;       // may be null
  int32_t* err;
};

template <int D, int DEG>
__device__ __forceinline__ bool wls_particle(const WlsArgs& a, int i, int m) {
  using Bs = Basis<D, DEG>;
  constexpr int B = Bs::B, DD = D * D;
  const int64_t row = static_cast<int64_t>(i) * a.cap;
  double xi[D];
#pragma unroll
  for (int k = 0; k < D; ++k) xi[k] = a.x[static_cast<int64_t>(k) * a.N + i];
  double A[Bs::NT];
#pragma unroll
  for (int k = 0; k < Bs::NT; ++k) A[k] = 0.0;
  for (int e = 0; e < m; ++e) {
    const int j = a.idx[row + e];
    double y[D], r2 = 0.0, p[B];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      y[k] = (a.x[static_cast<int64_t>(k) * a.N + j] - xi[k]) / a.h;
      r2 = r2 + y[k] * y[k];
    }
    const double w = exp(-a.alpha * r2);
    Bs::eval(y, p);
#pragma unroll
    for (int r = 0; r < B; ++r) {
      const double wp = w * p[r];
#pragma unroll
      for (int s = 0; s <= r; ++s) A[tri(r, s)] = A[tri(r, s)] + wp * p[s];
    }
  }
  if (!cholesky_packed<B>(A)) return false;
  double z[D][B];
#pragma unroll
  for (int k = 0; k < D; ++k) chol_solve_unit<B>(A, 1 + k, z[k]);
  for (int e = 0; e < m; ++e) {
    const int j = a.idx[row + e];
    double y[D], dl[D], r2 = 0.0, p[B];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      dl[k] = a.x[static_cast<int64_t>(k) * a.N + j] - xi[k];
      y[k] = dl[k] / a.h;
      r2 = r2 + y[k] * y[k];
    }
    const double w = exp(-a.alpha * r2);
    Bs::eval(y, p);
    double g[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      double s = 0.0;
#pragma unroll
      for (int r = 0; r < B; ++r) s = s + z[k][r] * p[r];
      g[k] = w * s / a.h;
    }
    if (a.grad) {
#pragma unroll
      for (int k = 0; k < D; ++k) a.grad[(row + e) * D + k] = g[k];
    }
    double o[DD];
    if (j == i) {
#pragma unroll
      for (int k = 0; k < DD; ++k) o[k] = 0.0;
    } else {
      double n[3], t[3], b[3];
      edge_frame<D>(dl, n, t, b);
      double ab = 0.0, bb = 0.0, gb = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        ab = ab + g[k] * n[k];
        bb = bb + g[k] * t[k];
        if (D == 3) gb = gb + g[k] * b[k];
      }
#pragma unroll
      for (int k = 0; k < D; ++k) {
        o[k] = ab * n[k];
        o[D + k] = bb * t[k];
        if (D == 3) o[2 * D + k] = gb * b[k];
      }
    }
    if (a.ops) {
#pragma unroll
      for (int k = 0; k < DD; ++k) a.ops[(row + e) * DD + k] = o[k];
    }
    if (a.ops32) {
#pragma unroll
      for (int k = 0; k < DD; ++k) a.ops32[(row + e) * DD + k] = static_cast<float>(o[k]);
    }
  }
  return true;
}

// One thread per interior particle.  Degree: the configured one if the
// stencil holds at least twice as many points as degree-2 basis functions,
// else 1 if it holds d+2 points, else BGK_ESINGULAR.
template <int D>
__global__ __launch_bounds__(128) void k_wls(const WlsArgs a) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.Ni) return;
  const int i = a.plist[k];
  const int m = min(a.cnt[i], a.cap);
  int deg = a.deg_cfg;
  if (deg == 2 && m < 2 * Basis<D, 2>::B) deg = 1;
  bool ok = m >= D + 2;
  if (ok) ok = (deg == 2) ? wls_particle<D, 2>(a, i, m) : wls_particle<D, 1>(a, i, m);
  if (!ok) {
    raise_error(a.err, BGK_ESINGULAR);
    deg = 0;
  }
  if (a.degree) a.degree[i] = deg;
}

hipError_t launch_wls(const Ctx& c, const double* x, const int32_t* cnt, const int32_t* idx,
                      double* grad, double* ops, float* ops32, int32_t* degree) {
  WlsArgs a{c.N, c.cap, c.Ni, c.cfg.wls_degree, c.cfg.h, c.cfg.alpha, x, c.d.cperm, cnt, idx,
            grad, ops, ops32, degree, c.d.err};
  if (c.Ni == 0) return hipSuccess;
  if (c.D == 2)
    hipLaunchKernelGGL(k_wls<2>, dim3(blocks_for(c.Ni, 128)), dim3(128), 0, c.stream, a);
  else
    hipLaunchKernelGGL(k_wls<3>, dim3(blocks_for(c.Ni, 128)), dim3(128), 0, c.stream, a);
  return hipGetLastError();
}

// ------------------------------------------------------------ wall rows
// One thread per wall particle b: interior particles within hb (first of h,
// 1.5h, 2h giving d+2 of them), ascending, and the degree-1 least-squares
// value weights at x_b (weights exp(-alpha r^2/hb^2)).
struct WallArgs {
  int N, cap, Nw, nca, ncell;
  double h, alpha;
  const double* x;
  const int32_t* wall_list;
  const int32_t* cstart;
  const int32_t* cperm;
  int32_t* wcnt;
  int32_t* widx;
  double* wc0;
  double* whb;
  int32_t* err;
};

template <int D>
__global__ __launch_bounds__(128) void k_wall_stencil(const WallArgs a) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.Nw) return;
  const int b = a.wall_list[k];
  double xb[D];
  int cb[D];
#pragma unroll
  for (int q = 0; q < D; ++q) {
    xb[q] = a.x[static_cast<int64_t>(q) * a.N + b];
    cb[q] = cell_coord(xb[q], a.nca);
  }
  const double mults[3] = {1.0, 1.5, 2.0};
  double hb = 0.0, hb2 = 0.0;
  int m = 0;
  const int zlo = (D == 3) ? -2 : 0, zhi = (D == 3) ? 2 : 0;
  for (int t = 0; t < 3; ++t) {
    hb = mults[t] * a.h;
    hb2 = hb * hb;
    m = 0;
    for (int dz = zlo; dz <= zhi; ++dz) {
      const int cz = (D == 3) ? cb[D - 1] + dz : 0;
      if (D == 3 && (cz < 0 || cz >= a.nca)) continue;
      for (int dy = -2; dy <= 2; ++dy) {
        const int cy = cb[1] + dy;
        if (cy < 0 || cy >= a.nca) continue;
        for (int dx = -2; dx <= 2; ++dx) {
          const int cx = cb[0] + dx;
          if (cx < 0 || cx >= a.nca) continue;
          const int cell = cx + a.nca * (cy + a.nca * cz);
          for (int p = a.cstart[cell]; p < a.cstart[cell + 1]; ++p) {
            const int j = a.cperm[p];
            double r2 = 0.0;
#pragma unroll
            for (int q = 0; q < D; ++q) {
              const double dl = a.x[static_cast<int64_t>(q) * a.N + j] - xb[q];
              r2 = r2 + dl * dl;
            }
            if (r2 <= hb2) {
              if (m < a.cap) {
                int32_t* row = a.widx + static_cast<int64_t>(k) * a.cap;
                int s = m;
                while (s > 0 && row[s - 1] > j) {
                  row[s] = row[s - 1];
                  --s;
                }
                row[s] = j;
              }
              ++m;
            }
          }
        }
      }
    }
    if (m >= D + 2) break;
  }
  a.whb[k] = hb;
  if (m < D + 2) {
    raise_error(a.err, BGK_ESINGULAR);
    a.wcnt[k] = 0;
    return;
  }
  if (m > a.cap) {
    raise_error(a.err, BGK_ENBR_OVERFLOW);
    a.wcnt[k] = 0;
    return;
  }
  using Bs = Basis<D, 1>;
  constexpr int B = Bs::B;
  const int32_t* row = a.widx + static_cast<int64_t>(k) * a.cap;
  double A[Bs::NT];
#pragma unroll
  for (int q = 0; q < Bs::NT; ++q) A[q] = 0.0;
  for (int e = 0; e < m; ++e) {
    const int j = row[e];
    double y[D], r2 = 0.0, p[B];
#pragma unroll
    for (int q = 0; q < D; ++q) {
      y[q] = (a.x[static_cast<int64_t>(q) * a.N + j] - xb[q]) / hb;
      r2 = r2 + y[q] * y[q];
    }
    const double w = exp(-a.alpha * r2);
    Bs::eval(y, p);
#pragma unroll
    for (int r = 0; r < B; ++r) {
      const double wp = w * p[r];
#pragma unroll
      for (int s = 0; s <= r; ++s) A[tri(r, s)] = A[tri(r, s)] + wp * p[s];
    }
  }
  if (!cholesky_packed<B>(A)) {
    raise_error(a.err, BGK_ESINGULAR);
    a.wcnt[k] = 0;
    return;
  }
  double z[B];
  chol_solve_unit<B>(A, 0, z);
  for (int e = 0; e < m; ++e) {
    const int j = row[e];
    double y[D], r2 = 0.0, p[B];
#pragma unroll
    for (int q = 0; q < D; ++q) {
      y[q] = (a.x[static_cast<int64_t>(q) * a.N + j] - xb[q]) / hb;
      r2 = r2 + y[q] * y[q];
    }
    const double w = exp(-a.alpha * r2);
    Bs::eval(y, p);
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < B; ++r) s = s + z[r] * p[r];
    a.wc0[static_cast<int64_t>(k) * a.cap + e] = w * s;
  }
  a.wcnt[k] = m;
}

hipError_t launch_wall_stencil(const Ctx& c, const double* x) {
  if (c.Nw == 0) return hipSuccess;
  WallArgs a{c.N, c.cap, c.Nw, c.nca, c.ncell, c.cfg.h, c.cfg.alpha, x, c.d.wall_list,
             c.d.cstart, c.d.cperm, c.d.wcnt, c.d.widx, c.d.wc0, c.d.whb, c.d.err};
  if (c.D == 2)
    hipLaunchKernelGGL(k_wall_stencil<2>, dim3(blocks_for(c.Nw, 128)), dim3(128), 0, c.stream, a);
  else
    hipLaunchKernelGGL(k_wall_stencil<3>, dim3(blocks_for(c.Nw, 128)), dim3(128), 0, c.stream, a);
  return hipGetLastError();
}

// Expand the compact wall rows to per-particle output arrays.
__global__ void k_scatter_wall_rows(int Nw, int cap, const int32_t* __restrict__ wall_list,
                                    const int32_t* __restrict__ wcnt,
                                    const int32_t* __restrict__ widx,
                                    const double* __restrict__ wc0,
                                    const double* __restrict__ whb, int32_t* cnt_out,
                                    int32_t* idx_out, double* c0_out, double* hb_out) {
  const int k = blockIdx.x;
  if (k >= Nw) return;
  const int b = wall_list[k];
  const int m = wcnt[k];
  if (threadIdx.x == 0) {
    cnt_out[b] = m;
    if (hb_out) hb_out[b] = whb[k];
  }
  for (int e = threadIdx.x; e < m; e += blockDim.x) {
    idx_out[static_cast<int64_t>(b) * cap + e] = widx[static_cast<int64_t>(k) * cap + e];
    c0_out[static_cast<int64_t>(b) * cap + e] = wc0[static_cast<int64_t>(k) * cap + e];
  }
}

hipError_t launch_scatter_wall_rows(const Ctx& c, int32_t* cnt_out, int32_t* idx_out,
                                    double* c0_out, double* hb_out) {
  if (c.Nw == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_wall_rows, dim3(c.Nw), dim3(64), 0, c.stream, c.Nw, c.cap,
                     c.d.wall_list, c.d.wcnt, c.d.widx, c.d.wc0, c.d.whb, cnt_out, idx_out,
                     c0_out, hb_out);
  return hipGetLastError();
}

// ------------------------------------------------------------ patch unions
// Interior particles, taken kPatch at a time in cell order, form a patch.
// The transport kernel walks the sorted union of the patch's neighbour
// lists (self excluded) once, loading each f_j row once for all of them.
// ue[u] holds, per patch slot t, the position of j in slot t's neighbour
// row in byte t (0xFF: j is not a neighbour of slot t).
__global__ void k_patches(int Ni, int cap, int ucap, const int32_t* __restrict__ plist,
                          const int32_t* __restrict__ cnt, const int32_t* __restrict__ idx,
                          int32_t* __restrict__ ucount, int32_t* __restrict__ uj,
                          uint32_t* __restrict__ ue, int32_t* __restrict__ err) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p * kPatch >= Ni) return;
  int pt[kPatch], head[kPatch], m[kPatch];
#pragma unroll
  for (int t = 0; t < kPatch; ++t) {
    const int g = p * kPatch + t;
    pt[t] = g < Ni ? plist[g] : -1;
    head[t] = 0;
    m[t] = pt[t] >= 0 ? min(cnt[pt[t]], cap) : 0;
  }
  int u = 0;
  for (;;) {
    int jmin = INT_MAX;
#pragma unroll
    for (int t = 0; t < kPatch; ++t) {
      const int32_t* row = idx + static_cast<int64_t>(max(pt[t], 0)) * cap;
      if (head[t] < m[t] && row[head[t]] == pt[t]) ++head[t];
      if (head[t] < m[t]) jmin = min(jmin, static_cast<int>(row[head[t]]));
    }
    if (jmin == INT_MAX) break;
    uint32_t pe = 0xFFFFFFFFu;
#pragma unroll
    for (int t = 0; t < kPatch; ++t) {
      const int32_t* row = idx + static_cast<int64_t>(max(pt[t], 0)) * cap;
      if (head[t] < m[t] && row[head[t]] == jmin) {
        pe = (pe & ~(0xFFu << (8 * t))) | (static_cast<uint32_t>(head[t]) << (8 * t));
        ++head[t];
      }
    }
    if (u < ucap) {
      uj[static_cast<int64_t>(p) * ucap + u] = jmin;
      ue[static_cast<int64_t>(p) * ucap + u] = pe;
    }
    ++u;
  }
  ucount[p] = min(u, ucap);
  atomicMax(&err[3], u);
}

hipError_t launch_patches(const Ctx& c) {
  if (c.npatch == 0) return hipSuccess;
  hipLaunchKernelGGL(k_patches, dim3(blocks_for(c.npatch, 128)), dim3(128), 0, c.stream, c.Ni,
                     c.cap, c.ucap, c.d.cperm, c.d.ncnt, c.d.nidx, c.d.ucount, c.d.uj, c.d.ue,
                     c.d.err);
  return hipGetLastError();
}

}  // namespace bgk
