// Geometry of one step: cell list, neighbour search (S1), weighted
// least-squares operators and edge frames (S2-S3), boundary interpolation
// rows (S7 part 1) and the patch unions the transport kernel walks.
//
// These kernels are cheap next to the transport (O(N m B^2) against
// O(N N_v m)); they are written for exactness first: FP64 throughout, the
// squared-distance predicate and the normal equations in the plain operation
// order (no contraction), deterministic outputs (sorted lists, no atomics on
// values).
#include <algorithm>
#include <climits>

#include "cloud_common.h"

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

// Largest of n int32 into *out (one atomic per block).
__global__ void k_max_i32(const int32_t* __restrict__ a, int n, int32_t* __restrict__ out) {
  int v = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    v = max(v, a[i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  __shared__ int wmax[4];
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(out, max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3])));
}

hipError_t launch_max_i32(hipStream_t s, const int32_t* a, int n, int32_t* out) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_max_i32, dim3(std::min(64u, blocks_for(n, 256))), dim3(256), 0, s, a, n,
                     out);
  return hipGetLastError();
}

// ------------------------------------------------------------ cell list
// Key of a particle: its cell (cells of size 1/nca >= h) in the order
// above, plus ncell for wall particles, so that the sorted permutation
// holds all interior particles first (in cell order) and the wall particles
// after them.
template <int D>
__global__ void k_cell_count(int N, int nca, int ncell, const double* __restrict__ x,
                             const int32_t* __restrict__ wall_id, int32_t* __restrict__ key,
                             int32_t* __restrict__ count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int cc[D];
#pragma unroll
  for (int a = 0; a < D; ++a) cc[a] = cell_coord(x[static_cast<int64_t>(a) * N + i], nca);
  const int c = cell_key<D>(cc, nca);
  const int k = c + (wall_id[i] != 0 ? ncell : 0);
  key[i] = k;
  atomicAdd(&count[k], 1);
}

// Exclusive scan of n int32 in place (one block of 1024 threads walking the
// array in chunks of 1024*PER); a[n] receives the total.  copy (may be null)
// receives the same n values.  Each chunk is read and written coalesced
// through LDS (padded one word in 32 against bank conflicts); each thread
// scans PER consecutive entries.
constexpr int kScanPer = 8;
__device__ __forceinline__ int scan_pad(int i) { return i + (i >> 5); }

__global__ __launch_bounds__(1024) void k_scan_inplace(int32_t* a, int n, int32_t* copy) {
  constexpr int PER = kScanPer, CH = 1024 * PER;
  __shared__ int32_t buf[CH + CH / 32];
  __shared__ int32_t wsum[16];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  int carry = 0;
  for (int base = 0; base < n; base += CH) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int i = k * 1024 + tid, g = base + i;
      buf[scan_pad(i)] = g < n ? a[g] : 0;
    }
    __syncthreads();
    int v[PER];
    int s = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      v[k] = buf[scan_pad(tid * PER + k)];
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
      buf[scan_pad(tid * PER + k)] = run;
      run += v[k];
    }
    carry += wsum[15];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int i = k * 1024 + tid, g = base + i;
      if (g < n) {
        const int x = buf[scan_pad(i)];
        a[g] = x;
        if (copy) copy[g] = x;
      }
    }
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

// Final position of each particle: its cell range, ascending particle index
// inside the range (so the permutation is deterministic).  Thread per slot p
// of the unsorted permutation: the rank of its particle among the range's
// entries.  The positions are copied into cell order (xs[a][q] = x[a][perm[q]])
// so that candidate positions are contiguous loads in the searches below.
__global__ void k_cell_rank(int N, int D, const int32_t* __restrict__ key,
                            const int32_t* __restrict__ start, const int32_t* __restrict__ perm2,
                            int32_t* __restrict__ perm, const double* __restrict__ x,
                            double* __restrict__ xs) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const int i = perm2[p];
  const int k = key[i];
  const int b = start[k], e = start[k + 1];
  int rank = 0;
  for (int q = b; q < e; ++q) rank += perm2[q] < i;
  const int dst = b + rank;
  perm[dst] = i;
  for (int a = 0; a < D; ++a) xs[static_cast<int64_t>(a) * N + dst] = x[static_cast<int64_t>(a) * N + i];
}

hipError_t launch_scan(hipStream_t s, int32_t* a, int n) {
  hipLaunchKernelGGL(k_scan_inplace, dim3(1), dim3(1024), 0, s, a, n, nullptr);
  return hipGetLastError();
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
  hipLaunchKernelGGL(k_scan_inplace, dim3(1), dim3(1024), 0, c.stream, d.cstart, nkeys,
                     d.ccursor);
  hipLaunchKernelGGL(k_cell_scatter, dim3(blocks_for(c.N, 256)), dim3(256), 0, c.stream, c.N,
                     d.key, d.ccursor, d.cperm2);
  hipLaunchKernelGGL(k_cell_rank, dim3(blocks_for(c.N, 256)), dim3(256), 0, c.stream, c.N, c.D,
                     d.key, d.cstart, d.cperm2, d.cperm, x, d.xs);
  return hipGetLastError();
}

// ------------------------------------------------------------ S1 neighbours
// One wave per particle: the lanes test the candidates of the 3^D cells
// around the particle's own (interior and wall ranges) against
// |x_j - x_i|^2 <= h^2, compact the hits, and store them ascending.
constexpr int kHitCap = 1024;  // hits kept in LDS (more are only counted)

template <int D>
__global__ __launch_bounds__(64) void k_neighbors(int N, int nca, int ncell, double h2, int cap,
                                                  const double* __restrict__ x,
                                                  const double* __restrict__ xs,
                                                  const int32_t* __restrict__ cstart,
                                                  const int32_t* __restrict__ cperm,
                                                  int32_t* __restrict__ cnt,
                                                  int32_t* __restrict__ idx,
                                                  int32_t* __restrict__ err) {
  constexpr int NR = (D == 2 ? 9 : 27) * 2;
  __shared__ int32_t rb[NR], rpre[NR + 1];
  __shared__ int32_t hits[kHitCap];
  const int i = blockIdx.x, lane = threadIdx.x;
  double xi[D];
  int ci[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    xi[a] = x[static_cast<int64_t>(a) * N + i];
    ci[a] = cell_coord(xi[a], nca);
  }
  const int nr = cell_ranges<D, 1>(ci, nca, ncell, true, cstart, rb, rpre);
  const int total = rpre[nr];
  int m = 0;
  for (int c0 = 0; c0 < total; c0 += kWave) {
    const int cidx = c0 + lane;
    bool hit = false;
    int j = 0;
    if (cidx < total) {
      const int p = cand_slot(cidx, nr, rb, rpre);
      j = cperm[p];
      double r2 = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const double dl = xs[static_cast<int64_t>(a) * N + p] - xi[a];
        r2 = r2 + dl * dl;
      }
      hit = r2 <= h2;
    }
    const uint64_t mask = __ballot(hit);
    const int pos = m + lanes_below(mask);
    if (hit && pos < kHitCap) hits[pos] = j;
    m += __popcll(mask);
  }
  __syncthreads();
  rank_sorted_store(hits, min(m, kHitCap), cap, idx + static_cast<int64_t>(i) * cap);
  if (lane == 0) {
    cnt[i] = m;
    if (m > cap) raise_error(err, BGK_ENBR_OVERFLOW);
  }
}

hipError_t launch_neighbors(const Ctx& c, const double* x, int32_t* cnt, int32_t* idx) {
  const double h2 = c.cfg.h * c.cfg.h;
  if (c.D == 2)
    hipLaunchKernelGGL(k_neighbors<2>, dim3(c.N), dim3(kWave), 0, c.stream, c.N, c.nca, c.ncell,
                       h2, c.cap, x, c.d.xs, c.d.cstart, c.d.cperm, cnt, idx, c.d.err);
  else
    hipLaunchKernelGGL(k_neighbors<3>, dim3(c.N), dim3(kWave), 0, c.stream, c.N, c.nca, c.ncell,
                       h2, c.cap, x, c.d.xs, c.d.cstart, c.d.cperm, cnt, idx, c.d.err);
  return hipGetLastError();
}

// ------------------------------------------------------------ S2-S3 WLS
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

// Sum of v over the 16 lanes of a DPP row, left in every lane of the row.
// Each step adds a lane's value to that of its partner (xor 1, xor 2, the
// mirrored quad, the mirrored half); IEEE addition is commutative, so every
// lane of the row ends with the same bits.
template <int CTRL>
__device__ __forceinline__ double row_dpp(double v) {
  const unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(v));
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(u & 0xffffffffu), CTRL, 0xF,
                                             0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(u >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(static_cast<long long>(
      (static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) |
      static_cast<unsigned>(lo)));
}

__device__ __forceinline__ double row_sum16(double v) {
  v = v + row_dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v = v + row_dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v = v + row_dpp<0x141>(v);  // row_half_mirror
  v = v + row_dpp<0x140>(v);  // row_mirror
  return v;
}

// Basis values of one scaled offset y for the fitted degree, zero beyond
// the degree's B functions: degree 2 and 1 as Basis::eval, degree 0 the
// offsets alone (first derivatives only, no constant).
template <int D>
__device__ __forceinline__ void wls_basis(int deg, const double* y, double* p) {
  constexpr int B2 = Basis<D, 2>::B;
  if (deg == 2) {
    Basis<D, 2>::eval(y, p);
  } else if (deg == 1) {
    Basis<D, 1>::eval(y, p);
#pragma unroll
    for (int r = D + 1; r < B2; ++r) p[r] = 0.0;
  } else {
#pragma unroll
    for (int r = 0; r < B2; ++r) p[r] = r < D ? y[r] : 0.0;
  }
}

// kWlsGroup interior particles per wavefront, one 16-lane DPP row each
// (row g handles particle blockIdx.x * kWlsGroup + g).  Per particle:
// each lane takes the neighbours e = lane, lane + 16, ... , forms the
// scaled offset y = (x_j - x_i)/h, the weight and the basis values, and
// adds W_e p(y_e) p(y_e)^T to its own copy of the packed normal matrix;
// the row's 16 partial matrices are summed with DPP moves, so that every
// lane holds all of A.  Every lane then factors A = L L^T and solves
// L L^T z = e_col for the gradient columns in registers (the same
// arithmetic in every lane of the row), and forms, for its own
// neighbours, the gradient row W_e z.p(y_e)/h, the edge frame of x_j - x_i
// and (P, Q[, R]).  The offsets, weights and indices of a lane's own
// neighbours wait in LDS between the two passes (no lane reads another's,
// so there is no barrier).  Degree: the configured one if the stencil holds
// at least twice as many points as degree-2 basis functions, else 1 if it
// holds d+2 points, else BGK_ESINGULAR (also on a non-positive pivot).
// Degree 0 is the fit as printed in Sec. 3.4.1: first derivatives only, the
// basis is the scaled offsets y (no constant; the particle itself has
// y = 0 and drops out), derivative k in column k.  A lower degree runs on
// the degree-2 sizes with the unused basis values zero and a unit diagonal
// in their rows of A, which leaves the fitted block and its solution as
// they are and zeros the rest.
constexpr int kWlsGroup = 4;
constexpr int kWlsRow = kWave / kWlsGroup;

template <int D>
__global__ __launch_bounds__(64) void k_wls(const WlsArgs a) {
  extern __shared__ double wls_sm[];
  constexpr int B2 = Basis<D, 2>::B, NT2 = Basis<D, 2>::NT, DD = D * D;
  constexpr int L = kWlsRow;
  const int lane = threadIdx.x, g = lane / L, gl = lane % L;
  const int pidx = blockIdx.x * kWlsGroup + g;
  const bool valid = pidx < a.Ni;
  const int i = valid ? a.plist[pidx] : 0;
  const int m = valid ? min(a.cnt[i], a.cap) : 0;
  int deg = a.deg_cfg;
  if (deg == 2 && m < 2 * B2) deg = 1;
  const int Bg = (deg == 2) ? B2 : (deg == 1 ? D + 1 : D);
  const bool enough = m >= D + 2;
  // per lane and local neighbour q: dl[D], W (doubles), j (int), stored
  // [q][field][lane] so that a wave's accesses are consecutive
  const int qmax = (a.cap + L - 1) / L;
  double* DL = wls_sm;                    // [qmax][D][64]
  double* WS = DL + qmax * D * kWave;     // [qmax][64]
  int32_t* JS = reinterpret_cast<int32_t*>(WS + qmax * kWave);  // [qmax][64]
  const int64_t row = static_cast<int64_t>(i) * a.cap;
  double xi[D];
#pragma unroll
  for (int k = 0; k < D; ++k) xi[k] = a.x[static_cast<int64_t>(k) * a.N + i];
  double A[NT2];
#pragma unroll
  for (int t = 0; t < NT2; ++t) A[t] = 0.0;
  for (int q = 0, e = gl; e < m; ++q, e += L) {
    const int j = a.idx[row + e];
    double y[D], r2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double dl = a.x[static_cast<int64_t>(k) * a.N + j] - xi[k];
      DL[(q * D + k) * kWave + lane] = dl;
      y[k] = dl / a.h;
      r2 = r2 + y[k] * y[k];
    }
    const double w = exp(-a.alpha * r2);
    WS[q * kWave + lane] = w;
    JS[q * kWave + lane] = j;
    double p[B2];
    wls_basis<D>(deg, y, p);
#pragma unroll
    for (int r = 0; r < B2; ++r) {
      const double wp = w * p[r];
#pragma unroll
      for (int s = 0; s <= r; ++s) A[tri(r, s)] = A[tri(r, s)] + wp * p[s];
    }
  }
#pragma unroll
  for (int t = 0; t < NT2; ++t) A[t] = row_sum16(A[t]);
#pragma unroll
  for (int r = 0; r < B2; ++r)
    if (r >= Bg) A[tri(r, r)] = 1.0;
  // A = L L^T in place, with the reciprocals of the diagonal kept
  bool bad = false;
  double inv[B2];
#pragma unroll
  for (int jc = 0; jc < B2; ++jc) {
    double s = A[tri(jc, jc)];
#pragma unroll
    for (int k = 0; k < jc; ++k) s = s - A[tri(jc, k)] * A[tri(jc, k)];
    bad = bad || !(s > 0.0);
    const double l = sqrt(s);
    A[tri(jc, jc)] = l;
    inv[jc] = 1.0 / l;
#pragma unroll
    for (int r = jc + 1; r < B2; ++r) {
      double t = A[tri(r, jc)];
#pragma unroll
      for (int k = 0; k < jc; ++k) t = t - A[tri(r, k)] * A[tri(jc, k)];
      A[tri(r, jc)] = t * inv[jc];
    }
  }
  const bool ok = valid && enough && !bad;
  // z_k = A^{-1} e_col(k): derivative k is column 1 + k (degree 1 and 2) or
  // k (degree 0)
  double z[D][B2];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const int col = deg == 0 ? k : 1 + k;
    double yv[B2];
#pragma unroll
    for (int r = 0; r < B2; ++r) {
      double s = (r == col) ? 1.0 : 0.0;
#pragma unroll
      for (int c = 0; c < r; ++c) s = s - A[tri(r, c)] * yv[c];
      yv[r] = s * inv[r];
    }
#pragma unroll
    for (int r = B2 - 1; r >= 0; --r) {
      double s = yv[r];
#pragma unroll
      for (int c = r + 1; c < B2; ++c) s = s - A[tri(c, r)] * z[k][c];
      z[k][r] = s * inv[r];
    }
  }
  if (ok) {
    for (int q = 0, e = gl; e < m; ++q, e += L) {
      const int j = JS[q * kWave + lane];
      const double w = WS[q * kWave + lane];
      double dl[D], y[D];
#pragma unroll
      for (int k = 0; k < D; ++k) {
        dl[k] = DL[(q * D + k) * kWave + lane];
        y[k] = dl[k] / a.h;
      }
      double p[B2];
      wls_basis<D>(deg, y, p);
      double gk[D];
#pragma unroll
      for (int k = 0; k < D; ++k) {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < B2; ++r) s = s + z[k][r] * p[r];
        gk[k] = w * s / a.h;
      }
      if (a.grad) {
#pragma unroll
        for (int k = 0; k < D; ++k) a.grad[(row + e) * D + k] = gk[k];
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
          ab = ab + gk[k] * n[k];
          bb = bb + gk[k] * t[k];
          if (D == 3) gb = gb + gk[k] * b[k];
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
  }
  if (valid && gl == 0) {
    if (!ok) raise_error(a.err, BGK_ESINGULAR);
    if (a.degree) a.degree[i] = ok ? deg : 0;
  }
}

static size_t wls_smem(int D, int cap) {
  const size_t qmax = static_cast<size_t>((cap + kWlsRow - 1) / kWlsRow);
  return qmax * kWave * ((D + 1) * sizeof(double) + sizeof(int32_t));
}

hipError_t launch_wls(const Ctx& c, const double* x, const int32_t* cnt, const int32_t* idx,
                      double* grad, double* ops, float* ops32, int32_t* degree) {
  WlsArgs a{c.N, c.cap, c.Ni, c.cfg.wls_degree, c.cfg.h, c.cfg.alpha, x, c.d.cperm, cnt, idx,
            grad, ops, ops32, degree, c.d.err};
  if (c.Ni == 0) return hipSuccess;
  const size_t sm = wls_smem(c.D, c.cap);
  const dim3 grid((c.Ni + kWlsGroup - 1) / kWlsGroup);
  if (c.D == 2)
    hipLaunchKernelGGL(k_wls<2>, grid, dim3(kWave), sm, c.stream, a);
  else
    hipLaunchKernelGGL(k_wls<3>, grid, dim3(kWave), sm, c.stream, a);
  return hipGetLastError();
}

// ------------------------------------------------------------ wall rows
// One wave per wall particle b: its value row at x_b (interior particles
// within hb, ascending, with their degree-1 least-squares value weights;
// value_row).
struct WallArgs {
  CloudView cv;
  const int32_t* wall_list;
  int32_t* wcnt;
  int32_t* widx;
  double* wc0;
  double* whb;
  int32_t* err;
};

template <int D>
__global__ __launch_bounds__(64) void k_wall_stencil(const WallArgs a) {
  __shared__ ValueRowSm<D> sm;
  const int k = blockIdx.x, lane = threadIdx.x;
  const int b = a.wall_list[k];
  double xb[D];
#pragma unroll
  for (int q = 0; q < D; ++q) xb[q] = a.cv.x[static_cast<int64_t>(q) * a.cv.N + b];
  double hb = 0.0;
  const int m = value_row<D>(a.cv, xb, sm, hb);
  if (lane == 0) a.whb[k] = hb;
  if (m < 0) {
    if (lane == 0) {
      raise_error(a.err, m == -2 ? BGK_ENBR_OVERFLOW : BGK_ESINGULAR);
      a.wcnt[k] = 0;
    }
    return;
  }
  const int64_t row = static_cast<int64_t>(k) * a.cv.cap;
  for (int e = lane; e < m; e += kWave) {
    a.widx[row + e] = sm.srt[e];
    a.wc0[row + e] = value_weight<D>(sm, e);
  }
  if (lane == 0) a.wcnt[k] = m;
}

CloudView cloud_view(const Ctx& c, const double* x) {
  return CloudView{c.N, c.cap, c.nca, c.ncell, c.cfg.h, c.cfg.alpha, x, c.d.xs, c.d.cstart,
                   c.d.cperm};
}

hipError_t launch_wall_stencil(const Ctx& c, const double* x) {
  if (c.Nw == 0) return hipSuccess;
  WallArgs a{cloud_view(c, x), c.d.wall_list, c.d.wcnt, c.d.widx, c.d.wc0, c.d.whb, c.d.err};
  if (c.D == 2)
    hipLaunchKernelGGL(k_wall_stencil<2>, dim3(c.Nw), dim3(kWave), 0, c.stream, a);
  else
    hipLaunchKernelGGL(k_wall_stencil<3>, dim3(c.Nw), dim3(kWave), 0, c.stream, a);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? launch_wall_unions(c) : e;
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
// Interior particles, taken tp at a time in cell order, form a patch.
// The transport walks the sorted union of the patch's neighbour lists (self
// excluded) once, loading each f_j row once for all of them.  ue[u] holds,
// per patch slot t, the position of j in slot t's neighbour row in byte t
// (0xFF: j is not a neighbour of slot t).
// One wave per patch: the slot rows are merged by rank (position of each
// entry = entries smaller than it in every row, ties ordered by slot),
// equal indices are grouped, and each group becomes one union entry.  The
// same kernel merges the interpolation rows of wall patches (rows indexed
// by wall-list slot, no self entry to drop: drop_self = 0).
__device__ __forceinline__ int lower_bound_i(const int32_t* v, int n, int x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (v[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(64) void k_patches(int Ni, int P, int cap, int ucap, int drop_self,
                                                const int32_t* __restrict__ plist,
                                                const int32_t* __restrict__ cnt,
                                                const int32_t* __restrict__ idx,
                                                int32_t* __restrict__ ucount,
                                                int32_t* __restrict__ uj, uint32_t* __restrict__ ue,
                                                int32_t* __restrict__ err) {
  extern __shared__ int32_t psm[];
  int32_t* rj = psm;                        // [P][cap] neighbour j (self removed)
  int32_t* re = rj + P * cap;          // [P][cap] its slot in the full row
  int32_t* mj = re + P * cap;          // [P*cap] merged j
  int32_t* mt = mj + P * cap;          // merged (slot t << 8 | e)
  __shared__ int32_t rn[kPatchMax], spt[kPatchMax], sm_[kPatchMax], sself[kPatchMax], spre[kPatchMax + 1];
  const int p = blockIdx.x, lane = threadIdx.x;
  if (lane < P) {
    const int g = p * P + lane;
    const int pt = g < Ni ? plist[g] : -1;
    spt[lane] = pt;
    sm_[lane] = pt >= 0 ? min(cnt[pt], cap) : 0;
    sself[lane] = 0;
  }
  __syncthreads();
  // self is in its row exactly once (at most once if the row overflowed):
  // find it in all rows at once, then copy the rows without it
  for (int w = lane; w < P * cap; w += kWave) {
    const int t = w / cap, e = w - t * cap;
    if (drop_self && e < sm_[t] && idx[static_cast<int64_t>(spt[t]) * cap + e] == spt[t])
      sself[t] = e + 1;
  }
  __syncthreads();
  for (int w = lane; w < P * cap; w += kWave) {
    const int t = w / cap, e = w - t * cap;
    if (e >= sm_[t]) continue;
    const int sp = sself[t] - 1;
    if (e == sp) continue;
    const int o = (sp >= 0 && e > sp) ? e - 1 : e;
    rj[t * cap + o] = idx[static_cast<int64_t>(spt[t]) * cap + e];
    re[t * cap + o] = e;
  }
  if (lane < P) rn[lane] = sself[lane] ? sm_[lane] - 1 : sm_[lane];
  __syncthreads();
  if (lane == 0) {
    spre[0] = 0;
    for (int t = 0; t < P; ++t) spre[t + 1] = spre[t] + rn[t];
  }
  __syncthreads();
  const int total = spre[P];
  // merged position of every (t, q): q plus, in each other row, the entries
  // before it (equal j in a lower slot t first)
  for (int w = lane; w < total; w += kWave) {
    int t = 0;
    while (w >= spre[t + 1]) ++t;
    const int q = w - spre[t];
    const int j = rj[t * cap + q];
    int pos = q;
    for (int s2 = 0; s2 < P; ++s2) {
      if (s2 == t) continue;
      const int* v = rj + s2 * cap;
      pos += (s2 < t) ? lower_bound_i(v, rn[s2], j + 1) : lower_bound_i(v, rn[s2], j);
    }
    mj[pos] = j;
    mt[pos] = (t << 8) | re[t * cap + q];
  }
  __syncthreads();
  int nu = 0;
  for (int c0 = 0; c0 < total; c0 += kWave) {
    const int q = c0 + lane;
    const bool head = q < total && (q == 0 || mj[q] != mj[q - 1]);
    const uint64_t mask = __ballot(head);
    const int u = nu + lanes_below(mask);
    if (head) {
      uint32_t pe = 0xFFFFFFFFu;
      for (int r = q; r < total && mj[r] == mj[q]; ++r) {
        const int t = mt[r] >> 8, e = mt[r] & 0xFF;
        pe = (pe & ~(0xFFu << (8 * t))) | (static_cast<uint32_t>(e) << (8 * t));
      }
      if (u < ucap) {
        uj[static_cast<int64_t>(p) * ucap + u] = mj[q];
        ue[static_cast<int64_t>(p) * ucap + u] = pe;
      }
    }
    nu += __popcll(mask);
  }
  if (lane == 0) ucount[p] = min(nu, ucap);
}

hipError_t launch_unions(const Ctx& c, int P, int n, const int32_t* plist, const int32_t* cnt,
                         const int32_t* idx, int drop_self, int ucap, int32_t* ucount,
                         int32_t* uj, uint32_t* ue) {
  if (n == 0) return hipSuccess;
  if (P < 1 || P > kPatchMax || ucap < P * c.cap) return hipErrorInvalidValue;
  const size_t sm = static_cast<size_t>(4) * P * c.cap * sizeof(int32_t);
  hipLaunchKernelGGL(k_patches, dim3((n + P - 1) / P), dim3(kWave), sm, c.stream, n, P, c.cap,
                     ucap, drop_self, plist, cnt, idx, ucount, uj, ue, c.d.err);
  return hipGetLastError();
}

hipError_t launch_patches(const Ctx& c) {
  return launch_unions(c, c.tp, c.Ni, c.d.cperm, c.d.ncnt, c.d.nidx, 1, c.ucap, c.d.ucount,
                       c.d.uj, c.d.ue);
}

hipError_t launch_wall_unions(const Ctx& c) {
  return launch_unions(c, kWallPatch, c.npw * kWallPatch, c.d.wpl, c.d.wcnt, c.d.widx, 0,
                       c.wucap, c.d.wucount, c.d.wuj, c.d.wue);
}

}  // namespace bgk
