// Reverse mode of one step with the MOVING cloud: the part of the adjoint
// that flows through the positions.  The frozen-cloud reverse step
// (k_adjoint.hip) treats the operators as constants; with the cloud moving,
// a step is (f^n, U^n, x^n, lid) -> (f^{n+1}, U^{n+1}, x^{n+1}, rho, T) and
// x^n enters through
//   S2-S3  the least-squares gradient rows g_ij(x) (Sec. 3.4.1) and the
//          edge frames (n, t[, b]) of x_j - x_i (Sec. 3.4.2), i.e. the upwind
//          vectors a_k = (g.e_k) e_k of every edge,
//   S7     the wall value rows c0_bj(x) (degree-1 fit at the wall particle),
//   S8     x^{n+1} = x^n + dt U^{n+1} (Sec. 3.2.1), clamped.
// Neighbour sets, stencil radii and fitted degrees are fixed by the
// positions' values (the map is piecewise smooth; the derivative is the one
// of the piece the state is on).  Given the adjoints of the outputs:
//   S8:    lam_U^{n+1} += dt lam_x^{n+1} and lam_x^n = lam_x^{n+1} on
//          coordinates the clamp left alone (zero where it clamped);
//   S4:    lam_a_k(i, e) = -2 dt sum_v [a_k.w < 0] w sum_c lam_ft_i (f_j - f_i)
//          (c_ij = 2 sum_k min(0, a_k.w), w = v - U_i^n);
//   S7:    lam_c0(b, e) = sum_{v, c} lam_arr_b(v) f^{n+1}_j(v) (the adjoint
//          reaching the interpolated half);
//   S2-S3: per particle, the reverse of a_k = (g.e_k) e_k through the frame
//          and of g_e = (W_e/h) Z^T p_e with Z = A^-1 E, A = sum W p p^T:
//          lam_A = -K Z^T with K = A^-1 lam_Z, so that
//          lam_W_e = (1/h) lam_g.Z^T p_e - sum_a (K_a.p_e)(z_a.p_e),
//          lam_p_e = (W_e/h) Z lam_g - W_e sum_a [K_a (z_a.p_e) + z_a (K_a.p_e)],
//          then y_e = (x_j - x_i)/h and W_e = exp(-alpha |y_e|^2);
//          the wall rows alike with z = A^-1 e_0 at the wall particle.
// Each edge's contribution to x_j is stored per (row, slot) and gathered by
// j over the transposed neighbour and wall-stencil indices: no atomics, a
// fixed summation order, bitwise repeatable results.
#include <type_traits>

#include "device_common.h"

namespace bgk {

struct MoveAdjArgs {
  int N, NV, nv, cap, Ni, Nw, deg_cfg;
  double vmax, h, alpha, dt, lo, hi;
  const int32_t* wall_id;
  const int32_t* wall_list;
  const int32_t* wpos;     // [N] wall-list index of a wall particle (-1: interior)
  const int32_t* plist;    // interior particles first
  const int32_t* ncnt;
  const int32_t* nidx;
  const int32_t* tidx;
  const int32_t* wcnt;
  const int32_t* widx;
  const double* whb;
  const int32_t* wtstart;
  const int32_t* wt;
  const double* x;         // x^n
  const double* U1;        // recomputed U^{n+1}
  const double* lam_U1;    // nullable
  const double* lam_x1;    // nullable
  double* lamU_eff;        // [D][N] lam_U1 + dt lam_x1 (unclamped interior coordinates)
  double* xpass;           // [D][N] lam_x1 where the position update passes it on
  double* lam_a;           // [N][cap][D*D]
  double* lc0;             // [Nw][cap]
  double* xc;              // [N][cap][D] contribution of row i's slot e to x_j
  double* xs;              // [N][D]      contribution of row i to x_i
  double* wxc;             // [Nw][cap][D]
  double* wxs;             // [Nw][D]
  double* lam_x;           // out [D][N]
};

// ------------------------------------------------------------ S8 reverse
__global__ void k_adjm_move_prep(const MoveAdjArgs a, int D) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.N) return;
  const bool inner = a.wall_id[j] == 0;
  for (int q = 0; q < D; ++q) {
    const size_t o = static_cast<size_t>(q) * a.N + j;
    const double lx = a.lam_x1 ? a.lam_x1[o] : 0.0;
    const double lu = a.lam_U1 ? a.lam_U1[o] : 0.0;
    bool pass = true;
    if (inner) {
      // the position update of k_move, operation for operation
      const double y = a.x[o] + a.dt * a.U1[o];
      pass = !(y < a.lo) && !(y > a.hi);
    }
    a.lamU_eff[o] = (inner && pass) ? lu + a.dt * lx : lu;
    a.xpass[o] = pass ? lx : 0.0;
  }
}

// ------------------------------------------------------------ S4: lam_a
// One block per interior particle; for each of its edges the block sums
// [p_k < 0] sdf(v) w(v) over all velocities (each thread a strided share of
// the grid, then a fixed-order block sum).
template <int D, int NC, typename Real>
__global__ __launch_bounds__(kThreads) void k_adjm_ops(const MoveAdjArgs a, const Real* ops,
                                                       const Real* f, const double* U,
                                                       const Real* lam_ft) {
  constexpr int DD = D * D;
  __shared__ double sh[4 * DD];
  const int i = a.plist[blockIdx.x];
  const size_t NVs = a.NV, cs = static_cast<size_t>(a.N) * NVs;
  const int m = min(a.ncnt[i], a.cap);
  const int64_t row = static_cast<int64_t>(i) * a.cap;
  double Ui[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < D; ++q) Ui[q] = U[static_cast<size_t>(q) * a.N + i];
  for (int e = 0; e < m; ++e) {
    const int j = a.nidx[row + e];
    double acc[DD];
#pragma unroll
    for (int k = 0; k < DD; ++k) acc[k] = 0.0;
    if (j != i) {
      double ak[DD];
#pragma unroll
      for (int k = 0; k < DD; ++k) ak[k] = static_cast<double>(ops[(row + e) * DD + k]);
      for (int q = threadIdx.x; q < a.NV; q += kThreads) {
        double v[3], w[D];
        velocity_of<D>(q, a.nv, a.vmax, v);
#pragma unroll
        for (int c = 0; c < D; ++c) w[c] = v[c] - Ui[c];
        double sdf = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const size_t oi = c * cs + static_cast<size_t>(i) * NVs + q;
          const size_t oj = c * cs + static_cast<size_t>(j) * NVs + q;
          sdf = sdf + static_cast<double>(lam_ft[oi]) *
                          (static_cast<double>(f[oj]) - static_cast<double>(f[oi]));
        }
#pragma unroll
        for (int k = 0; k < D; ++k) {
          double p = 0.0;
#pragma unroll
          for (int c = 0; c < D; ++c) p = p + ak[k * D + c] * w[c];
          if (p < 0.0) {
#pragma unroll
            for (int c = 0; c < D; ++c) acc[k * D + c] = acc[k * D + c] + sdf * w[c];
          }
        }
      }
    }
    block_sum<DD>(acc, sh);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < DD; ++k) a.lam_a[(row + e) * DD + k] = -2.0 * a.dt * acc[k];
    }
  }
}

// ------------------------------------------------------------ S7: lam_c0
// One block per wall particle (wall-list order): for every stencil entry
// the dot product of the adjoint reaching the interpolated half with the
// interior row f^{n+1}_j it interpolates (zero on the emitted half).
template <int NC, typename Real>
__global__ __launch_bounds__(kThreads) void k_adjm_wallrow(const MoveAdjArgs a, const Real* larr,
                                                           const Real* f1) {
  __shared__ double sh[4];
  const int k = blockIdx.x;
  const size_t NVs = a.NV, cs = static_cast<size_t>(a.N) * NVs;
  const int m = a.wcnt[k];
  for (int e = 0; e < m; ++e) {
    const int j = a.widx[static_cast<size_t>(k) * a.cap + e];
    double s[1] = {0.0};
    for (int q = threadIdx.x; q < a.NV; q += kThreads) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
        s[0] = s[0] + static_cast<double>(larr[(static_cast<size_t>(k) * NC + c) * NVs + q]) *
                          static_cast<double>(f1[c * cs + static_cast<size_t>(j) * NVs + q]);
    }
    block_sum<1>(s, sh);
    if (threadIdx.x == 0) a.lc0[static_cast<size_t>(k) * a.cap + e] = s[0];
  }
}

// ------------------------------------------------------------ S2-S3 reverse
__device__ __forceinline__ constexpr int tri_m(int r, int s) { return r * (r + 1) / 2 + s; }

// Basis of the forward fit (degree 2 or 1 with the constant, degree 0 the
// offsets alone), padded with zeros to the degree-2 size B2; and the
// transpose of its Jacobian applied to lp: ly_c += sum_r lp_r dp_r/dy_c.
template <int D>
__device__ __forceinline__ void basis_m(int deg, const double* y, double* p) {
  constexpr int B2 = D == 2 ? 6 : 10;
#pragma unroll
  for (int r = 0; r < B2; ++r) p[r] = 0.0;
  if (deg == 0) {
#pragma unroll
    for (int c = 0; c < D; ++c) p[c] = y[c];
    return;
  }
  p[0] = 1.0;
#pragma unroll
  for (int c = 0; c < D; ++c) p[1 + c] = y[c];
  if (deg == 2) {
    int r = D + 1;
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int b = c; b < D; ++b) p[r++] = y[c] * y[b];
  }
}
template <int D>
__device__ __forceinline__ void basis_m_rev(int deg, const double* y, const double* lp,
                                            double* ly) {
  if (deg == 0) {
#pragma unroll
    for (int c = 0; c < D; ++c) ly[c] = ly[c] + lp[c];
    return;
  }
#pragma unroll
  for (int c = 0; c < D; ++c) ly[c] = ly[c] + lp[1 + c];
  if (deg == 2) {
    int r = D + 1;
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int b = c; b < D; ++b) {
        // p_r = y_c y_b
        ly[c] = ly[c] + lp[r] * y[b];
        ly[b] = ly[b] + lp[r] * y[c];
        ++r;
      }
  }
}

// Cholesky factor of a packed symmetric B x B matrix in place, with the
// reciprocals of the diagonal; false on a non-positive pivot.
template <int B>
__device__ __forceinline__ bool chol_m(double* A, double* inv) {
  bool ok = true;
#pragma unroll
  for (int jc = 0; jc < B; ++jc) {
    double s = A[tri_m(jc, jc)];
#pragma unroll
    for (int k = 0; k < jc; ++k) s = s - A[tri_m(jc, k)] * A[tri_m(jc, k)];
    ok = ok && (s > 0.0);
    const double l = sqrt(s);
    A[tri_m(jc, jc)] = l;
    inv[jc] = 1.0 / l;
#pragma unroll
    for (int r = jc + 1; r < B; ++r) {
      double t = A[tri_m(r, jc)];
#pragma unroll
      for (int k = 0; k < jc; ++k) t = t - A[tri_m(r, k)] * A[tri_m(jc, k)];
      A[tri_m(r, jc)] = t * inv[jc];
    }
  }
  return ok;
}
// z = (L L^T)^-1 rhs
template <int B>
__device__ __forceinline__ void chol_solve_m(const double* L, const double* inv, const double* rhs,
                                             double* z) {
  double yv[B];
#pragma unroll
  for (int r = 0; r < B; ++r) {
    double s = rhs[r];
#pragma unroll
    for (int c = 0; c < r; ++c) s = s - L[tri_m(r, c)] * yv[c];
    yv[r] = s * inv[r];
  }
#pragma unroll
  for (int r = B - 1; r >= 0; --r) {
    double s = yv[r];
#pragma unroll
    for (int c = r + 1; c < B; ++c) s = s - L[tri_m(c, r)] * z[c];
    z[r] = s * inv[r];
  }
}

// Edge frame of the forward (trig-free): 2D n = dl/r, t = n turned by +90
// degrees; 3D n = dl/r, b = (-dl_y, dl_x, 0)/r_xy (b = (0, 1, 0) on the z
// axis), t = b x n.
template <int D>
__device__ __forceinline__ void frame_m(const double* dl, double* n, double* t, double* b,
                                        double& r, double& rxy) {
  if (D == 2) {
    r = sqrt(dl[0] * dl[0] + dl[1] * dl[1]);
    rxy = r;
    n[0] = dl[0] / r;
    n[1] = dl[1] / r;
    t[0] = -n[1];
    t[1] = n[0];
    n[2] = t[2] = b[0] = b[1] = b[2] = 0.0;
  } else {
    rxy = sqrt(dl[0] * dl[0] + dl[1] * dl[1]);
    r = sqrt(dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2]);
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
// Reverse of the frame: the adjoint of dl from those of n, t (, b).
template <int D>
__device__ __forceinline__ void frame_m_rev(const double* n, const double* t, const double* b,
                                            double r, double rxy, const double* ln,
                                            const double* lt, const double* lb, double* ld) {
  if (D == 2) {
    // t = (-n1, n0)
    const double m0 = ln[0] + lt[1], m1 = ln[1] - lt[0];
    const double nm = n[0] * m0 + n[1] * m1;
    ld[0] = (m0 - n[0] * nm) / r;
    ld[1] = (m1 - n[1] * nm) / r;
  } else {
    // t = b x n: lb += n x lt, ln += lt x b
    double mb[3], mn[3];
    mb[0] = lb[0] + (n[1] * lt[2] - n[2] * lt[1]);
    mb[1] = lb[1] + (n[2] * lt[0] - n[0] * lt[2]);
    mb[2] = lb[2] + (n[0] * lt[1] - n[1] * lt[0]);
    mn[0] = ln[0] + (lt[1] * b[2] - lt[2] * b[1]);
    mn[1] = ln[1] + (lt[2] * b[0] - lt[0] * b[2]);
    mn[2] = ln[2] + (lt[0] * b[1] - lt[1] * b[0]);
    // n = dl / r
    const double nm = n[0] * mn[0] + n[1] * mn[1] + n[2] * mn[2];
#pragma unroll
    for (int c = 0; c < 3; ++c) ld[c] = (mn[c] - n[c] * nm) / r;
    // b = (-dl_y, dl_x, 0) / r_xy
    if (rxy > 0.0) {
      const double bm = b[0] * mb[0] + b[1] * mb[1] + b[2] * mb[2];
      const double lu0 = (mb[0] - b[0] * bm) / rxy, lu1 = (mb[1] - b[1] * bm) / rxy;
      ld[0] = ld[0] + lu1;
      ld[1] = ld[1] - lu0;
    }
  }
}

// One thread per interior particle: the forward least squares and frames
// recomputed, then the reverse described at the top of the file.  Writes
// xc[i][e] (to x_j) for every slot (zero on the self slot) and xs[i].
template <int D>
__global__ __launch_bounds__(64) void k_adjm_geom(const MoveAdjArgs a) {
  constexpr int B2 = D == 2 ? 6 : 10, NT2 = B2 * (B2 + 1) / 2, DD = D * D;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.Ni) return;
  const int i = a.plist[k];
  const int m = min(a.ncnt[i], a.cap);
  const int64_t row = static_cast<int64_t>(i) * a.cap;
  int deg = a.deg_cfg;
  if (deg == 2 && m < 2 * B2) deg = 1;
  const int Bg = (deg == 2) ? B2 : (deg == 1 ? D + 1 : D);
  double xi[D];
#pragma unroll
  for (int c = 0; c < D; ++c) xi[c] = a.x[static_cast<size_t>(c) * a.N + i];
  double A[NT2], inv[B2];
#pragma unroll
  for (int t = 0; t < NT2; ++t) A[t] = 0.0;
  auto edge_geom = [&](int e, int& j, double (&dl)[D], double (&y)[D], double& w,
                       double (&p)[B2]) {
    j = a.nidx[row + e];
    double r2 = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      dl[c] = a.x[static_cast<size_t>(c) * a.N + j] - xi[c];
      y[c] = dl[c] / a.h;
      r2 = r2 + y[c] * y[c];
    }
    w = exp(-a.alpha * r2);
    basis_m<D>(deg, y, p);
  };
  for (int e = 0; e < m; ++e) {
    int j;
    double dl[D], y[D], w, p[B2];
    edge_geom(e, j, dl, y, w, p);
#pragma unroll
    for (int r = 0; r < B2; ++r) {
      const double wp = w * p[r];
#pragma unroll
      for (int s = 0; s <= r; ++s) A[tri_m(r, s)] = A[tri_m(r, s)] + wp * p[s];
    }
  }
#pragma unroll
  for (int r = 0; r < B2; ++r)
    if (r >= Bg) A[tri_m(r, r)] = 1.0;
  const bool ok = m >= D + 2 && chol_m<B2>(A, inv);
  double z[D][B2];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    double rhs[B2];
#pragma unroll
    for (int r = 0; r < B2; ++r) rhs[r] = (r == (deg == 0 ? c : 1 + c)) ? 1.0 : 0.0;
    chol_solve_m<B2>(A, inv, rhs, z[c]);
  }
  // per edge: g, the frame, and the adjoints of g and of the frame vectors
  auto edge_rev = [&](int e, int& j, double (&dl)[D], double (&y)[D], double& w, double (&p)[B2],
                      double (&zp)[D], double (&lg)[D], double (&ld)[D]) {
    edge_geom(e, j, dl, y, w, p);
    double g[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < D; ++c) {
      double s = 0.0;
#pragma unroll
      for (int r = 0; r < B2; ++r) s = s + z[c][r] * p[r];
      zp[c] = s;
      g[c] = w * s / a.h;
    }
    double dl3[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < D; ++c) dl3[c] = dl[c];
    double n[3], t[3], b[3], r, rxy;
    frame_m<D>(dl3, n, t, b, r, rxy);
    const double* la = a.lam_a + (row + e) * DD;
    double lP[3] = {0.0, 0.0, 0.0}, lQ[3] = {0.0, 0.0, 0.0}, lR[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < D; ++c) {
      lP[c] = la[c];
      lQ[c] = la[D + c];
      if (D == 3) lR[c] = la[2 * D + c];
    }
    double al = 0.0, be = 0.0, ga = 0.0, lal = 0.0, lbe = 0.0, lga = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      al = al + g[c] * n[c];
      be = be + g[c] * t[c];
      ga = ga + g[c] * b[c];
      lal = lal + lP[c] * n[c];
      lbe = lbe + lQ[c] * t[c];
      lga = lga + lR[c] * b[c];
    }
    double ln[3], lt[3], lb[3], ld3[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      ln[c] = al * lP[c] + lal * g[c];
      lt[c] = be * lQ[c] + lbe * g[c];
      lb[c] = ga * lR[c] + lga * g[c];
    }
    frame_m_rev<D>(n, t, b, r, rxy, ln, lt, lb, ld3);
#pragma unroll
    for (int c = 0; c < D; ++c) {
      lg[c] = lal * n[c] + lbe * t[c] + lga * b[c];
      ld[c] = ld3[c];
    }
  };
  // pass 1: lam_Z (column c: sum_e (W_e/h) lam_g_e[c] p_e)
  double LZ[D][B2];
#pragma unroll
  for (int c = 0; c < D; ++c)
#pragma unroll
    for (int r = 0; r < B2; ++r) LZ[c][r] = 0.0;
  if (ok) {
    for (int e = 0; e < m; ++e) {
      if (a.nidx[row + e] == i) continue;
      int j;
      double dl[D], y[D], w, p[B2], zp[D], lg[D], ld[D];
      edge_rev(e, j, dl, y, w, p, zp, lg, ld);
#pragma unroll
      for (int c = 0; c < D; ++c)
#pragma unroll
        for (int r = 0; r < B2; ++r) LZ[c][r] = LZ[c][r] + (w / a.h) * lg[c] * p[r];
    }
  }
  double K[D][B2];
#pragma unroll
  for (int c = 0; c < D; ++c) chol_solve_m<B2>(A, inv, LZ[c], K[c]);
  // pass 2: every edge's contribution to x_j (and, negated, to x_i)
  double own[D];
#pragma unroll
  for (int c = 0; c < D; ++c) own[c] = 0.0;
  for (int e = 0; e < m; ++e) {
    double out[D];
#pragma unroll
    for (int c = 0; c < D; ++c) out[c] = 0.0;
    if (ok && a.nidx[row + e] != i) {
      int j;
      double dl[D], y[D], w, p[B2], zp[D], lg[D], ld[D];
      edge_rev(e, j, dl, y, w, p, zp, lg, ld);
      double Kp[D];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < B2; ++r) s = s + K[c][r] * p[r];
        Kp[c] = s;
      }
      double lW = 0.0;
#pragma unroll
      for (int c = 0; c < D; ++c) lW = lW + lg[c] * zp[c] / a.h - Kp[c] * zp[c];
      double lp[B2];
#pragma unroll
      for (int r = 0; r < B2; ++r) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c)
          s = s + (w / a.h) * lg[c] * z[c][r] - w * (K[c][r] * zp[c] + z[c][r] * Kp[c]);
        lp[r] = s;
      }
      double ly[D];
#pragma unroll
      for (int c = 0; c < D; ++c) ly[c] = lW * w * (-2.0 * a.alpha * y[c]);
      basis_m_rev<D>(deg, y, lp, ly);
#pragma unroll
      for (int c = 0; c < D; ++c) {
        out[c] = ly[c] / a.h + ld[c];
        own[c] = own[c] - out[c];
      }
    }
#pragma unroll
    for (int c = 0; c < D; ++c) a.xc[(row + e) * D + c] = out[c];
  }
#pragma unroll
  for (int c = 0; c < D; ++c) a.xs[static_cast<size_t>(i) * D + c] = own[c];
}

// One thread per wall particle: the reverse of its degree-1 value row
// c0_e = W_e z.p_e, z = A^-1 e_0, y_e = (x_j - x_b)/hb.
template <int D>
__global__ __launch_bounds__(64) void k_adjm_wallgeom(const MoveAdjArgs a) {
  constexpr int B = D + 1, NT = B * (B + 1) / 2;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.Nw) return;
  const int bq = a.wall_list[k];
  const int m = a.wcnt[k];
  const double hb = a.whb[k];
  const size_t row = static_cast<size_t>(k) * a.cap;
  double xb[D];
#pragma unroll
  for (int c = 0; c < D; ++c) xb[c] = a.x[static_cast<size_t>(c) * a.N + bq];
  auto ent = [&](int e, double (&y)[D], double& w, double (&p)[B]) {
    const int j = a.widx[row + e];
    double r2 = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      y[c] = (a.x[static_cast<size_t>(c) * a.N + j] - xb[c]) / hb;
      r2 = r2 + y[c] * y[c];
    }
    w = exp(-a.alpha * r2);
    p[0] = 1.0;
#pragma unroll
    for (int c = 0; c < D; ++c) p[1 + c] = y[c];
  };
  double A[NT], inv[B];
#pragma unroll
  for (int t = 0; t < NT; ++t) A[t] = 0.0;
  for (int e = 0; e < m; ++e) {
    double y[D], w, p[B];
    ent(e, y, w, p);
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int s = 0; s <= r; ++s) A[tri_m(r, s)] = A[tri_m(r, s)] + w * p[r] * p[s];
  }
  const bool ok = m >= D + 2 && chol_m<B>(A, inv);
  double z[B], rhs[B], LZ[B], K[B];
#pragma unroll
  for (int r = 0; r < B; ++r) {
    rhs[r] = r == 0 ? 1.0 : 0.0;
    LZ[r] = 0.0;
  }
  chol_solve_m<B>(A, inv, rhs, z);
  const double* lc = a.lc0 + row;
  if (ok) {
    for (int e = 0; e < m; ++e) {
      double y[D], w, p[B];
      ent(e, y, w, p);
#pragma unroll
      for (int r = 0; r < B; ++r) LZ[r] = LZ[r] + lc[e] * w * p[r];
    }
  }
  chol_solve_m<B>(A, inv, LZ, K);
  double own[D];
#pragma unroll
  for (int c = 0; c < D; ++c) own[c] = 0.0;
  for (int e = 0; e < m; ++e) {
    double out[D];
#pragma unroll
    for (int c = 0; c < D; ++c) out[c] = 0.0;
    if (ok) {
      double y[D], w, p[B];
      ent(e, y, w, p);
      double zp = 0.0, Kp = 0.0;
#pragma unroll
      for (int r = 0; r < B; ++r) {
        zp = zp + z[r] * p[r];
        Kp = Kp + K[r] * p[r];
      }
      const double lW = lc[e] * zp - Kp * zp;
      double ly[D];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        // dp/dy_c = e_{1+c}
        const double lp = lc[e] * w * z[1 + c] - w * (K[1 + c] * zp + z[1 + c] * Kp);
        ly[c] = lW * w * (-2.0 * a.alpha * y[c]) + lp;
        out[c] = ly[c] / hb;
        own[c] = own[c] - out[c];
      }
    }
#pragma unroll
    for (int c = 0; c < D; ++c) a.wxc[(row + e) * D + c] = out[c];
  }
#pragma unroll
  for (int c = 0; c < D; ++c) a.wxs[static_cast<size_t>(k) * D + c] = own[c];
}

// ------------------------------------------------------------ gather
// lam_x_j = (S8 part) + j's own row + every row i that holds j (transposed
// slots, in j's row order) + every wall row that interpolates j (in
// wall-list order) + j's own wall row.
__global__ void k_adjm_xgather(const MoveAdjArgs a, int D) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.N) return;
  const bool inner = a.wall_id[j] == 0;
  const int m = min(a.ncnt[j], a.cap);
  const int64_t row = static_cast<int64_t>(j) * a.cap;
  for (int c = 0; c < D; ++c) {
    double s = a.xpass[static_cast<size_t>(c) * a.N + j];
    if (inner) s = s + a.xs[static_cast<size_t>(j) * D + c];
    for (int e = 0; e < m; ++e) {
      const int te = a.tidx[row + e];
      if (te < 0) continue;
      const int i = a.nidx[row + e];
      s = s + a.xc[(static_cast<int64_t>(i) * a.cap + te) * D + c];
    }
    for (int p = a.wtstart[j]; p < a.wtstart[j + 1]; ++p) {
      const int kk = a.wt[p] >> 8, e = a.wt[p] & 0xFF;
      s = s + a.wxc[(static_cast<size_t>(kk) * a.cap + e) * D + c];
    }
    if (!inner) s = s + a.wxs[static_cast<size_t>(a.wpos[j]) * D + c];
    a.lam_x[static_cast<size_t>(c) * a.N + j] = s;
  }
}

// ------------------------------------------------------------ launchers
static MoveAdjArgs move_args(const Ctx& c, const double* x, const double* lam_U1,
                             const double* lam_x1, double* lam_x) {
  const Adj& j = c.adj;
  const MoveAdj& v = c.madj;
  return MoveAdjArgs{c.N,        c.NV,       c.cfg.nv,   c.cap,      c.Ni,
                     c.Nw,       c.cfg.wls_degree, c.cfg.vmax, c.cfg.h, c.cfg.alpha,
                     c.cfg.dt,   0.1 * c.cfg.dx, 1.0 - 0.1 * c.cfg.dx,
                     c.d.wall_id, c.d.wall_list, v.wpos,  c.d.cperm,  c.d.ncnt,
                     c.d.nidx,   j.tidx,     c.d.wcnt,   c.d.widx,   c.d.whb,
                     j.wtstart,  j.wt,       x,          j.U1,       lam_U1,
                     lam_x1,     v.lamU_eff, v.xpass,    v.lam_a,    v.lc0,
                     v.xc,       v.xs,       v.wxc,      v.wxs,      lam_x};
}

hipError_t launch_adjoint_move_prep(const Ctx& c, const double* x, const double* lam_U1,
                                    const double* lam_x1) {
  const MoveAdjArgs a = move_args(c, x, lam_U1, lam_x1, nullptr);
  hipLaunchKernelGGL(k_adjm_move_prep, dim3((c.N + 255) / 256), dim3(256), 0, c.stream, a, c.D);
  return hipGetLastError();
}

hipError_t launch_adjoint_wallrow(const Ctx& c) {
  if (c.Nw == 0) return hipSuccess;
  const MoveAdjArgs a = move_args(c, nullptr, nullptr, nullptr, nullptr);
  if (c.cfg.precision == BGK_FP64) {
    const double* larr = static_cast<const double*>(c.adj.larr);
    const double* f1 = static_cast<const double*>(c.adj.f1);
    if (c.D == 2)
      hipLaunchKernelGGL((k_adjm_wallrow<2, double>), dim3(c.Nw), dim3(kThreads), 0, c.stream, a,
                         larr, f1);
    else
      hipLaunchKernelGGL((k_adjm_wallrow<1, double>), dim3(c.Nw), dim3(kThreads), 0, c.stream, a,
                         larr, f1);
  } else {
    const float* larr = static_cast<const float*>(c.adj.larr);
    const float* f1 = static_cast<const float*>(c.adj.f1);
    if (c.D == 2)
      hipLaunchKernelGGL((k_adjm_wallrow<2, float>), dim3(c.Nw), dim3(kThreads), 0, c.stream, a,
                         larr, f1);
    else
      hipLaunchKernelGGL((k_adjm_wallrow<1, float>), dim3(c.Nw), dim3(kThreads), 0, c.stream, a,
                         larr, f1);
  }
  return hipGetLastError();
}

template <typename Real>
static void launch_ops_t(const Ctx& c, const MoveAdjArgs& a, const void* f_n, const double* U_n) {
  const Real* ops = std::is_same<Real, double>::value
                        ? reinterpret_cast<const Real*>(c.d.ops64)
                        : reinterpret_cast<const Real*>(c.d.ops32);
  const Real* f = static_cast<const Real*>(f_n);
  const Real* lft = static_cast<const Real*>(c.adj.lam_ft);
  if (c.D == 2)
    hipLaunchKernelGGL((k_adjm_ops<2, 2, Real>), dim3(c.Ni), dim3(kThreads), 0, c.stream, a, ops,
                       f, U_n, lft);
  else
    hipLaunchKernelGGL((k_adjm_ops<3, 1, Real>), dim3(c.Ni), dim3(kThreads), 0, c.stream, a, ops,
                       f, U_n, lft);
}

hipError_t launch_adjoint_move_geometry(const Ctx& c, const void* f_n, const double* U_n,
                                        const double* x, double* lam_x) {
  const MoveAdjArgs a = move_args(c, x, nullptr, nullptr, lam_x);
  if (c.Ni) {
    if (c.cfg.precision == BGK_FP64)
      launch_ops_t<double>(c, a, f_n, U_n);
    else
      launch_ops_t<float>(c, a, f_n, U_n);
    const dim3 g((c.Ni + 63) / 64), b(64);
    if (c.D == 2)
      hipLaunchKernelGGL(k_adjm_geom<2>, g, b, 0, c.stream, a);
    else
      hipLaunchKernelGGL(k_adjm_geom<3>, g, b, 0, c.stream, a);
  }
  if (c.Nw) {
    const dim3 g((c.Nw + 63) / 64), b(64);
    if (c.D == 2)
      hipLaunchKernelGGL(k_adjm_wallgeom<2>, g, b, 0, c.stream, a);
    else
      hipLaunchKernelGGL(k_adjm_wallgeom<3>, g, b, 0, c.stream, a);
  }
  hipLaunchKernelGGL(k_adjm_xgather, dim3((c.N + 255) / 256), dim3(256), 0, c.stream, a, c.D);
  return hipGetLastError();
}

}  // namespace bgk
