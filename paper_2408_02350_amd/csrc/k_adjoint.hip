// Hand-written adjoint of one frozen-cloud step (S4-S7) and of the
// objective.  The step map is (f^n, U^n) -> (f^{n+1}, U^{n+1}, rho^{n+1},
// T^{n+1}); the operators are constants (the cloud does not move).  Given the
// adjoints of the outputs, the reverse pass runs:
//
//   walls      f_b = interp(f'_int) on arriving velocities, rho_w from the
//              zero-mass-flux balance, emitted rho_w M[1, U_w(lid), T_w],
//              then (rho, U, T)_b = moments(f_b)
//   relaxation f' = a(tau) ft + b(tau) M(rho', U', T'), (rho', U', T') =
//              moments(ft), tau = tau(rho', T')
//   transport  ft_i = f_i - dt sum_j c_ij(v; U_i) (f_j - f_i)
//
// Every scatter of the forward map becomes a gather over a transposed
// index (neighbour rows are symmetric: j in N_i <=> i in N_j; wall stencil
// rows are transposed by a sorted counting pass), so there are no atomics
// on the adjoint fields and the result is deterministic.  Reductions are
// FP64 in a fixed order.  Derivatives of |.| at 0 follow the + branch
// (c_ij = 2 sum_k min(0, p_k): d/dp = 1 only for p < 0).
#include <algorithm>
#include <climits>
#include <type_traits>

#include "device_common.h"
#include "adjoint_plan.h"

namespace bgk {

// ------------------------------------------------------------ transposes
// tidx[j][e'] = position of j in the row of i = nidx[j][e'] when i is an
// interior particle other than j, else -1.
__global__ void k_transpose_nbr(int N, int cap, const int32_t* __restrict__ wall_id,
                                const int32_t* __restrict__ cnt, const int32_t* __restrict__ idx,
                                int32_t* __restrict__ tidx) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const int m = min(cnt[j], cap);
  for (int e = 0; e < m; ++e) {
    const int i = idx[static_cast<int64_t>(j) * cap + e];
    int pos = -1;
    if (i != j && wall_id[i] == 0) {
      const int32_t* row = idx + static_cast<int64_t>(i) * cap;
      int lo = 0, hi = min(cnt[i], cap);
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (row[mid] < j) lo = mid + 1; else hi = mid;
      }
      if (lo < min(cnt[i], cap) && row[lo] == j) pos = lo;
    }
    tidx[static_cast<int64_t>(j) * cap + e] = pos;
  }
}

// Wall stencil transpose: for every particle j, the (wall list index k,
// slot e) with widx[k][e] = j, sorted by k.  Count, scan, scatter, sort.
__global__ void k_wt_count(int Nw, int cap, const int32_t* __restrict__ wcnt,
                           const int32_t* __restrict__ widx, int32_t* __restrict__ count) {
  const int k = blockIdx.x;
  if (k >= Nw) return;
  for (int e = threadIdx.x; e < wcnt[k]; e += blockDim.x)
    atomicAdd(&count[widx[static_cast<int64_t>(k) * cap + e]], 1);
}
__global__ void k_wt_scatter(int Nw, int cap, const int32_t* __restrict__ wcnt,
                             const int32_t* __restrict__ widx, int32_t* __restrict__ cursor,
                             int32_t* __restrict__ wt) {
  const int k = blockIdx.x;
  if (k >= Nw) return;
  for (int e = threadIdx.x; e < wcnt[k]; e += blockDim.x) {
    const int pos = atomicAdd(&cursor[widx[static_cast<int64_t>(k) * cap + e]], 1);
    wt[pos] = k * 256 + e;  // k-major key, e < 256
  }
}
__global__ void k_wt_sort(int N, const int32_t* __restrict__ start, int32_t* __restrict__ wt) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const int b = start[j], e = start[j + 1];
  for (int p = b + 1; p < e; ++p) {
    const int v = wt[p];
    int s = p;
    while (s > b && wt[s - 1] > v) {
      wt[s] = wt[s - 1];
      --s;
    }
    wt[s] = v;
  }
}

// ------------------------------------------------------------ moments adjoint
// Adjoint of (rho, U, T) = moments(f) at one velocity: the change of f_c(v)
// that the output adjoints (lr, lU, lT) ask for (S5 formulas; the centred
// second moment is stationary in U, so T has no U path).
template <int D, int NC>
__device__ __forceinline__ double mom_adj(int c, const double* v, double omega, double s0,
                                          const double* U, double T, double lr, const double* lU,
                                          double lT) {
  if (c == 1) return lT / (3.0 * s0);
  double w2 = 0.0, g = lr * omega;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const double wa = v[a] - U[a];
    w2 = w2 + wa * wa;
    g = g + lU[a] * wa / s0;
  }
  return g + lT * (w2 / (3.0 * s0) - T / s0);
}

template <typename Real>
struct AdjArgs {  // Real: storage of f-sized arrays and operators (FP64 or FP32)
  int N, NV, nv, cap, Nw, Ni, D;
  double vmax, omega, kn, dt, lid, wall_T;
  const int32_t* wall_id;
  const int32_t* wall_list;
  const int32_t* plist;
  const int32_t* ncnt;
  const int32_t* nidx;
  const int32_t* tidx;
  const Real* ops;
  const int32_t* wcnt;
  const int32_t* widx;
  const double* wc0;
  const int32_t* wtstart;
  const int32_t* wt;
  const Real* f_n;       // state n
  const double* U_n;
  const Real* ft;        // recomputed f-tilde (interior rows)
  const Real* f1;        // recomputed f^{n+1} (all rows)
  const double* rho1;      // recomputed outputs
  const double* U1;
  const double* T1;
  const Real* lam_f1;    // adjoint of f^{n+1}
  const double* lam_U1;    // adjoint of U^{n+1} (nullable)
  const double* lam_rho1;  // (nullable)
  const double* lam_T1;    // (nullable)
  Real* larr;            // [Nw][NC][NV] adjoint reaching the interpolated (arriving) half
  Real* lam_ft;          // [NC][N][NV]
  Real* lam_f;           // out: adjoint of f^n
  double* lam_U;           // out: adjoint of U^n
  double* lidpart;         // [Nw] dJ/dlid contributions
  double* gpart;           // [tiles][D][N] per-tile parts of lam_U
  int tiles;
  // reverse transport over the forward's patch unions (interior particles);
  // the wall kernel runs over jlist (the wall particles)
  const int32_t* jlist;    // [Nw] particles of the wall kernel
  const int32_t* ucount;   // [npatch]
  const int32_t* uj;       // [npatch][ucap]
  const uint32_t* ue;      // [npatch][ucap]
  int ucap;
};

// ------------------------------------------------------------ S7 adjoint
// The velocity nodes and the per-axis factors exp(-(v_k - U_w,a)^2 / (2 T_w))
// of the wall Maxwellian are tabulated in LDS (dynamic, (D+1)*nv doubles),
// and a thread's velocity digits are advanced by those of the block stride.
template <int D, int NC, typename Real>
__global__ __launch_bounds__(kThreads) void k_adj_wall(const AdjArgs<Real> a) {
  __shared__ double sh[4 * 4];
  extern __shared__ double vt[];  // nodes [nv], then factors [D][nv]
  const int k = blockIdx.x;
  const int b = a.wall_list[k];
  const int w = a.wall_id[b];
  const int axis = (w - 1) / 2;
  const double sgn = ((w - 1) % 2 == 0) ? 1.0 : -1.0;
  const bool is_lid = (w == 2 * D);
  double Uw[3] = {is_lid ? a.lid : 0.0, 0.0, 0.0};
  const size_t NVs = a.NV, cs = static_cast<size_t>(a.N) * NVs;
  const Real* fb = a.f1 + static_cast<size_t>(b) * NVs;
  const Real* lb = a.lam_f1 + static_cast<size_t>(b) * NVs;
  const double rho = a.rho1[b], T = a.T1[b];
  double U[3] = {0.0, 0.0, 0.0}, lU[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < D; ++q) {
    U[q] = a.U1[static_cast<size_t>(q) * a.N + b];
    if (a.lam_U1) lU[q] = a.lam_U1[static_cast<size_t>(q) * a.N + b];
  }
  const double lr = a.lam_rho1 ? a.lam_rho1[b] : 0.0;
  const double lT = a.lam_T1 ? a.lam_T1[b] : 0.0;
  const double s0 = rho / a.omega;
  const int nv = a.nv;
  double* et = vt + nv;
  for (int kk = threadIdx.x; kk < nv; kk += blockDim.x) vt[kk] = vnode(kk, nv, a.vmax);
  __syncthreads();
  for (int t = threadIdx.x; t < D * nv; t += blockDim.x) {
    const int ax = t / nv, kk = t - ax * nv;
    const double d = vt[kk] - Uw[ax];
    et[t] = exp(-(d * d) / (2.0 * a.wall_T));
  }
  __syncthreads();
  const double tpw = 2.0 * kPi * a.wall_T;
  const double normw = D == 3 ? 1.0 / (tpw * sqrt(tpw)) : 1.0 / tpw;  // M[1, U_w, T_w]
  // pass 1: fluxes and the adjoint reaching rho_w and the lid
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // F_in, F_out, g_rhow, dF_out/dlid
  double glid = 0.0;
  VelDigits<D> vd;
  vd.init(threadIdx.x, kThreads, nv);
  for (int q = threadIdx.x; q < a.NV; q += kThreads, vd.advance(nv)) {
    double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int ax = 0; ax < D; ++ax) v[ax] = vt[vd.k[ax]];
    const double vn = sgn * v[axis];
    if (vn <= 0.0) {
      acc[0] = acc[0] + (-vn) * fb[q];
    } else {
      double M0 = normw;
#pragma unroll
      for (int ax = 0; ax < D; ++ax) M0 = M0 * et[ax * nv + vd.k[ax]];
      acc[1] = acc[1] + vn * M0;
      const double dM = (v[0] - Uw[0]) / a.wall_T;  // dM/dlid / M (lid walls)
      if (is_lid) acc[3] = acc[3] + vn * M0 * dM;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double l = lb[c * cs + q] + mom_adj<D, NC>(c, v, a.omega, s0, U, T, lr, lU, lT);
        const double Mc = (c == 1) ? a.wall_T * M0 : M0;
        acc[2] = acc[2] + l * Mc;
        if (is_lid) glid = glid + l * Mc * dM;
      }
    }
  }
  block_sum<4>(acc, sh);
  double gl[1] = {glid};
  block_sum<1>(gl, sh);
  const double Fin = acc[0], Fout = acc[1], grw = acc[2];
  const double rho_w = Fin / Fout;
  // pass 2: adjoint on the arriving (interpolated) half
  Real* lo = a.larr + static_cast<size_t>(k) * NC * NVs;
  vd.init(threadIdx.x, kThreads, nv);
  for (int q = threadIdx.x; q < a.NV; q += kThreads, vd.advance(nv)) {
    double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int ax = 0; ax < D; ++ax) v[ax] = vt[vd.k[ax]];
    const double vn = sgn * v[axis];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double l = 0.0;
      if (vn <= 0.0) {
        l = lb[c * cs + q] + mom_adj<D, NC>(c, v, a.omega, s0, U, T, lr, lU, lT);
        if (c == 0) l = l + grw * (-vn) / Fout;
      }
      lo[c * NVs + q] = static_cast<Real>(l);
    }
  }
  if (threadIdx.x == 0)
    a.lidpart[k] = is_lid ? (rho_w * gl[0] + grw * (-rho_w / Fout) * acc[3]) : 0.0;
}

// ------------------------------------------------------------ S5-S6 adjoint
// Row loads and stores of R consecutive values as 16-byte (or 8-byte)
// vectors; the row offsets the callers pass are multiples of R.
template <typename Real, int R>
__device__ __forceinline__ void load_rs(const Real* __restrict__ p, Real (&o)[R]) {
  constexpr int B = R * static_cast<int>(sizeof(Real));
  constexpr int W = B % 16 == 0 ? 16 / static_cast<int>(sizeof(Real))
                                : (B % 8 == 0 ? 8 / static_cast<int>(sizeof(Real)) : 1);
  typedef Real V __attribute__((ext_vector_type(W)));
  const V* pv = reinterpret_cast<const V*>(__builtin_assume_aligned(p, W * sizeof(Real)));
#pragma unroll
  for (int i = 0; i < R / W; ++i) {
    const V x = pv[i];
#pragma unroll
    for (int w = 0; w < W; ++w) o[i * W + w] = x[w];
  }
}

template <typename Real, int R>
__device__ __forceinline__ void store_rs(Real* __restrict__ p, const Real (&o)[R]) {
  constexpr int B = R * static_cast<int>(sizeof(Real));
  constexpr int W = B % 16 == 0 ? 16 / static_cast<int>(sizeof(Real))
                                : (B % 8 == 0 ? 8 / static_cast<int>(sizeof(Real)) : 1);
  typedef Real V __attribute__((ext_vector_type(W)));
  V* pv = reinterpret_cast<V*>(__builtin_assume_aligned(p, W * sizeof(Real)));
#pragma unroll
  for (int i = 0; i < R / W; ++i) {
    V x;
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = o[i * W + w];
    pv[i] = x;
  }
}

// Digits of a group of R consecutive nodes along the fastest velocity axis:
// k[0] counts groups (nv/R per row of that axis), k[1..] are node indices.
// Advanced by the digits of a fixed stride, with no division per group.
template <int D>
struct GroupDigits {
  int k[D], st[D];
  __device__ void init(int g, int stride, int ng0, int nv) {
    k[0] = g % ng0;
    g /= ng0;
    st[0] = stride % ng0;
    stride /= ng0;
#pragma unroll
    for (int a = 1; a < D; ++a) {
      k[a] = g % nv;
      g /= nv;
      st[a] = stride % nv;
      stride /= nv;
    }
  }
  __device__ void advance(int ng0, int nv) {  // (the carry out of the last
    int x = k[0] + st[0];                      //  digit is past the grid)
    int carry = x >= ng0;
    k[0] = carry ? x - ng0 : x;
#pragma unroll
    for (int a = 1; a < D; ++a) {
      x = k[a] + st[a] + carry;
      carry = x >= nv;
      k[a] = carry ? x - nv : x;
    }
  }
};

// One block per interior particle.  A thread takes groups of R consecutive
// nodes along the fastest velocity axis (group g = tid + m kThreads), so the
// rows move as 16-byte vectors and the factors of the slower axes are formed
// once per group.  The velocity nodes and the per-axis factors
// exp(-(v_k - U_a)^2 / (2T)) of the particle's Maxwellian are tabulated in
// LDS (dynamic, (D+1)*nv doubles): M = norm * prod_a e_a[k_a], Chu G2 = T G1.
// Pass 1 gathers the adjoint of f' (lam_f1 plus what the wall rows that
// interpolate from the particle send back) and reduces the D+3 sums of the
// relaxation's and the moments' adjoint; pass 2 writes lam_ft.  The first
// KEEP groups of a thread keep the adjoint of f' in registers between the
// passes, in the storage precision (the whole row at the configured grids);
// later groups are gathered again, or, near a wall, read back from the
// particle's own lam_ft row, where pass 1 left them (same thread, same
// velocities; nothing else reads the row).
template <int D, int NC, typename Real, int R, int KEEP>
__global__ __launch_bounds__(kThreads) void k_adj_collide(const AdjArgs<Real> a) {
  __shared__ double sh[4 * (D + 4)];
  extern __shared__ double vt[];  // nodes [nv], then factors [D][nv]
  const int i = a.plist[blockIdx.x];
  const size_t NVs = a.NV, cs = static_cast<size_t>(a.N) * NVs;
  const double rho = a.rho1[i], T = a.T1[i];
  double U[3] = {0.0, 0.0, 0.0}, lU[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < D; ++q) {
    U[q] = a.U1[static_cast<size_t>(q) * a.N + i];
    if (a.lam_U1) lU[q] = a.lam_U1[static_cast<size_t>(q) * a.N + i];
  }
  const double lr = a.lam_rho1 ? a.lam_rho1[i] : 0.0;
  const double lT = a.lam_T1 ? a.lam_T1[i] : 0.0;
  const double s0 = rho / a.omega;
  const double tau = a.kn * sqrt(2.0 / kPi) / (rho * sqrt(T));
  const double den = tau + a.dt;
  const double ca = tau / den, cb = a.dt / den, dtau = a.dt / (den * den);  // d f'/d tau = (ft-M) dtau
  const double kap0 = (D == 3) ? 1.5 : 1.0;
  // d M / d T = M (-kap/T + |v-U|^2 / (2 T^2)), kap = d/2 (Chu G2: kap = 0)
  const double iT = 1.0 / T, h2 = 0.5 * iT * iT, kT = -kap0 * iT;
  const int ws = a.wtstart[i], we = a.wtstart[i + 1];
  const int nv = a.nv, ng0 = nv / R, ng = a.NV / R;
  double* et = vt + nv;
  for (int k = threadIdx.x; k < nv; k += blockDim.x) vt[k] = vnode(k, nv, a.vmax);
  __syncthreads();
  for (int t = threadIdx.x; t < D * nv; t += blockDim.x) {
    const int ax = t / nv, k = t - ax * nv;
    const double d = vt[k] - U[ax];
    et[t] = exp(-(d * d) / (2.0 * T));
  }
  __syncthreads();
  const double tp = 2.0 * kPi * T;
  const double norm = D == 3 ? rho / (tp * sqrt(tp)) : rho / tp;
  const Real* __restrict__ l1 = a.lam_f1 + static_cast<size_t>(i) * NVs;
  const Real* __restrict__ xr = a.ft + static_cast<size_t>(i) * NVs;
  Real* __restrict__ lrow = a.lam_ft + static_cast<size_t>(i) * NVs;
  const bool near = we > ws;
  // the slower axes of a group: their offsets w_a, sum w_a^2, prod e_a
  auto slow = [&](const int (&kd)[D], double (&w)[3], double& w2s, double& Ms) {
    w[0] = w[1] = w[2] = 0.0;
    w2s = 0.0;
    Ms = norm;
#pragma unroll
    for (int k = 1; k < D; ++k) {
      w[k] = vt[kd[k]] - U[k];
      w2s = w2s + w[k] * w[k];
      Ms = Ms * et[k * nv + kd[k]];
    }
  };
  // adjoint of f' at a group's R nodes (component c), rounded to storage
  auto gather = [&](int c, size_t q, Real (&o)[R]) {
    load_rs<Real, R>(l1 + c * cs + q, o);
    if (!near) return;
    double l[R];
#pragma unroll
    for (int r = 0; r < R; ++r) l[r] = static_cast<double>(o[r]);
    for (int p = ws; p < we; ++p) {
      const int kk = a.wt[p] >> 8, e = a.wt[p] & 0xFF;
      const double wgt = a.wc0[static_cast<size_t>(kk) * a.cap + e];
      Real y[R];
      load_rs<Real, R>(a.larr + (static_cast<size_t>(kk) * NC + c) * NVs + q, y);
#pragma unroll
      for (int r = 0; r < R; ++r) l[r] = l[r] + wgt * static_cast<double>(y[r]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) o[r] = static_cast<Real>(l[r]);
  };
  double s[D + 3];  // A1 = sum l M, A2 = sum l (ft - M), AU[d], AT
#pragma unroll
  for (int k = 0; k < D + 3; ++k) s[k] = 0.0;
  auto accum = [&](size_t q, const int (&kd)[D], const Real (&lq)[NC][R]) {
    double w[3], w2s, Ms;
    slow(kd, w, w2s, Ms);
    Real xq[NC][R];
#pragma unroll
    for (int c = 0; c < NC; ++c) load_rs<Real, R>(xr + c * cs + q, xq[c]);
    const int k0 = kd[0] * R;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double w0 = vt[k0 + r] - U[0];
      const double w2 = fma(w0, w0, w2s);
      const double M1 = Ms * et[k0 + r];
      const double dlog = fma(w2, h2, kT);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double M = c == 0 ? M1 : T * M1;
        const double l = static_cast<double>(lq[c][r]);
        const double lM = l * M;
        s[0] = s[0] + lM;
        s[1] = fma(l, static_cast<double>(xq[c][r]) - M, s[1]);
        s[2] = fma(lM, w0, s[2]);
#pragma unroll
        for (int k = 1; k < D; ++k) s[2 + k] = fma(lM, w[k], s[2 + k]);
        s[2 + D] = fma(lM, (c == 1) ? w2 * h2 : dlog, s[2 + D]);
      }
    }
  };
  Real lk[KEEP][NC][R];
  {
    GroupDigits<D> gd;
    gd.init(threadIdx.x, kThreads, ng0, nv);
    int g = threadIdx.x;
#pragma unroll
    for (int m = 0; m < KEEP; ++m, g += kThreads) {
      if (g < ng) {
        const size_t q = static_cast<size_t>(g) * R;
#pragma unroll
        for (int c = 0; c < NC; ++c) gather(c, q, lk[m][c]);
        accum(q, gd.k, lk[m]);
      }
      gd.advance(ng0, nv);
    }
    for (; g < ng; g += kThreads) {
      const size_t q = static_cast<size_t>(g) * R;
      Real lq[NC][R];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        gather(c, q, lq[c]);
        if (near) store_rs<Real, R>(lrow + c * cs + q, lq[c]);
      }
      accum(q, gd.k, lq);
      gd.advance(ng0, nv);
    }
  }
  block_sum<D + 3>(s, sh);
  const double g_rho = lr + cb * s[0] / rho + s[1] * dtau * (-tau / rho);
  double gU[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < D; ++k) gU[k] = lU[k] + cb * s[2 + k] / T;
  const double g_T = lT + cb * s[2 + D] + s[1] * dtau * (-tau / (2.0 * T));
  // the moments' adjoint at one velocity (S5: rho = omega sum f, U = sum v f
  // / s0, 3 s0 T = sum |v-U|^2 f (+ sum G2 in the Chu model)) as
  //   m0 + sum_a mU_a w_a + mT |w|^2  (first component),  mT  (second)
  const double is0 = 1.0 / s0, mT = g_T * is0 / 3.0, m0 = g_rho * a.omega - g_T * T * is0;
  double mU[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < D; ++k) mU[k] = gU[k] * is0;
  auto write = [&](size_t q, const int (&kd)[D], const Real (&lq)[NC][R]) {
    double w[3], w2s, Ms;
    slow(kd, w, w2s, Ms);
    double gs = fma(mT, w2s, m0);
#pragma unroll
    for (int k = 1; k < D; ++k) gs = fma(mU[k], w[k], gs);
    Real o[NC][R];
    const int k0 = kd[0] * R;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double w0 = vt[k0 + r] - U[0];
      const double g0 = fma(mU[0], w0, fma(mT, w0 * w0, gs));
#pragma unroll
      for (int c = 0; c < NC; ++c)
        o[c][r] = static_cast<Real>(fma(ca, static_cast<double>(lq[c][r]), c == 1 ? mT : g0));
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) store_rs<Real, R>(lrow + c * cs + q, o[c]);
  };
  {
    GroupDigits<D> gd;
    gd.init(threadIdx.x, kThreads, ng0, nv);
    int g = threadIdx.x;
#pragma unroll
    for (int m = 0; m < KEEP; ++m, g += kThreads) {
      if (g < ng) write(static_cast<size_t>(g) * R, gd.k, lk[m]);
      gd.advance(ng0, nv);
    }
    for (; g < ng; g += kThreads) {
      const size_t q = static_cast<size_t>(g) * R;
      Real lq[NC][R];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if (near) load_rs<Real, R>(lrow + c * cs + q, lq[c]);
        else load_rs<Real, R>(l1 + c * cs + q, lq[c]);
      }
      write(q, gd.k, lq);
      gd.advance(ng0, nv);
    }
  }
}

// ------------------------------------------------------------ S4 adjoint
// Wall particles: not transported themselves, so their adjoint of f^n is
// only the transposed term,
//   lam_f_j = - dt sum_{i in N_j interior, i != j} c_ij lam_ft_i,
// with c_ij = 2 sum_k min(0, a_k.(v - U_i)) from i's operator at the slot
// where j sits in i's row (transposed index), and they take no part in
// lam_U (the sum over tiles zeroes their rows).  One wavefront per (wall
// particle, tile of 64 lanes x R velocities along the fastest axis): the
// records (a_k, a_k.U_i) of a chunk of 32 neighbours are staged in LDS, c
// is formed as g.w - sum_k |a_k.w| with the projections advanced by their
// per-velocity increments, and each neighbour's lam_ft row is loaded one
// neighbour ahead.  Arithmetic in the storage precision.
constexpr int kAdjChunk = 32;

template <int D, int NC, typename Real, int R>
__global__ __launch_bounds__(64) void k_adj_transport_wall(const AdjArgs<Real> a) {
  using A = Real;
  constexpr int DD = D * D, REC = DD + D;  // a_k (d*d), a_k.U_i (d)
  __shared__ A rtr[kAdjChunk][REC];
  __shared__ int32_t ri[kAdjChunk], rfl[kAdjChunk];
  // tile-major logical order, each XCD on one contiguous range of particles
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x), nj = gridDim.x / a.tiles;
  const int tile = lb / nj, jb = lb - tile * nj;
  const int j = a.jlist[jb];
  const int tid = threadIdx.x;
  const size_t NVs = a.NV, cs = static_cast<size_t>(a.N) * NVs;
  const int m = min(a.ncnt[j], a.cap);
  const int64_t row = static_cast<int64_t>(j) * a.cap;
  const A dva = static_cast<A>(2.0 * a.vmax / static_cast<double>(a.nv - 1));
  const int ngroups = a.NV / R;
  const int g = tile * 64 + tid;
  const bool on = g < ngroups;
  const int q0 = on ? g * R : 0;
  A v0[D];
  {
    int q = q0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      v0[k] = static_cast<A>(vnode(q % a.nv, a.nv, a.vmax));
      q /= a.nv;
    }
  }
  A lf[R][NC];  // sum_i c_ij lam_ft_i (dt applied at the end)
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < NC; ++c) lf[r][c] = A(0);

  for (int c0 = 0; c0 < m; c0 += kAdjChunk) {
    const int cn = min(kAdjChunk, m - c0);
    __syncthreads();  // the previous chunk is consumed
    for (int w = tid; w < cn; w += 64) {
      const int e = c0 + w;
      const int i = a.nidx[row + e];
      const int te = a.tidx[row + e];
      const bool tr = te >= 0 && i != j;
      ri[w] = i;
      rfl[w] = tr ? 1 : 0;
      if (tr) {
        const Real* o = a.ops + (static_cast<int64_t>(i) * a.cap + te) * DD;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          double b = 0.0;
#pragma unroll
          for (int mm = 0; mm < D; ++mm) {
            const double x = static_cast<double>(o[k * D + mm]);
            rtr[w][k * D + mm] = static_cast<A>(x);
            b = b + x * a.U_n[static_cast<size_t>(mm) * a.N + i];
          }
          rtr[w][DD + k] = static_cast<A>(b);
        }
      }
    }
    __syncthreads();
    A la[R][NC], lb2[R][NC];
    auto load_edge = [&](int w, A (&li)[R][NC]) {
      const int i = ri[w];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        A t[R];
        load_rs<Real, R>(a.lam_ft + c * cs + static_cast<size_t>(i) * NVs + q0, t);
#pragma unroll
        for (int r = 0; r < R; ++r) li[r][c] = t[r];
      }
      asm volatile("" ::: "memory");
    };
    auto edge = [&](int w, const A (&li)[R][NC]) {
      if (!rfl[w]) return;
      const A* rc = rtr[w];
      A p[D], ik[D];
#pragma unroll
      for (int k = 0; k < D; ++k) {
        A s1 = -rc[DD + k];
#pragma unroll
        for (int mm = 0; mm < D; ++mm) s1 = fma(rc[k * D + mm], v0[mm], s1);
        p[k] = s1;
        ik[k] = rc[k * D] * dva;
      }
      A gw = p[0], dgw = ik[0];
#pragma unroll
      for (int k = 1; k < D; ++k) {
        gw = gw + p[k];
        dgw = dgw + ik[k];
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (r > 0) {
#pragma unroll
          for (int k = 0; k < D; ++k) p[k] = p[k] + ik[k];
          gw = gw + dgw;
        }
        A cm = gw;  // 2 sum_k min(0, p_k)
#pragma unroll
        for (int k = 0; k < D; ++k) cm = cm - fabs(p[k]);
#pragma unroll
        for (int c = 0; c < NC; ++c) lf[r][c] = fma(cm, li[r][c], lf[r][c]);
      }
    };
    load_edge(0, la);
    for (int w = 0; w < cn; w += 2) {
      if (w + 1 < cn) load_edge(w + 1, lb2);
      edge(w, la);
      if (w + 1 < cn) {
        if (w + 2 < cn) load_edge(w + 2, la);
        edge(w + 1, lb2);
      }
    }
  }
  if (on) {
    const A dt = static_cast<A>(a.dt);
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int r = 0; r < R; ++r)
        a.lam_f[c * cs + static_cast<size_t>(j) * NVs + q0 + r] = static_cast<Real>(-dt * lf[r][c]);
  }
}

// The same reverse transport for the interior particles, taken P at a time
// in cell order (the unions are merged once per frozen cloud): one
// wavefront per (patch, tile of 64 lanes x R velocities) walks the sorted
// union of the patch's neighbour lists once.  The own and transposed edge
// records of a chunk of union entries are derived into LDS (with the
// per-velocity increments and their sum, so the walk adds instead of
// multiplying) and read with wave-uniform addresses; each lane loads the
// two rows an entry needs (f^n_i for the U-derivative, lam_ft_i for the
// transposed term) one entry ahead, once for all P particles.  The
// per-velocity arithmetic is in the storage precision (FP32 storage: FP32
// arithmetic, half the registers of FP64 and within that storage's
// rounding); each lane's lam_U sums are folded per edge and reduced over the
// wave in FP64 in a fixed order.  The flux coefficient is formed as
// g.w - sum_k |a_k.w| (2 sum_k min(0, a_k.w) up to rounding) and the
// U-derivative sums from the signs of the projections (the derivative of
// the + branch at 0, except at a projection of exactly -0).
constexpr int kAdjUChunk = 32;


template <int D, int NC, typename Real, int R, int P>
__global__ __launch_bounds__(64) void k_adj_transport_patch(const AdjArgs<Real> a) {
  using A = Real;  // arithmetic of the per-velocity work
  // record: a_k (d*d), a_k.U (d)[, a_k[FA] dv (d), sum_k a_k[FA] dv].
  // FP64 keeps a_k and a_k.U only and forms the increments per edge (fewer
  // wave-uniform LDS reads at 2-4 velocities per lane)
  constexpr bool LEAN = std::is_same<Real, double>::value;
  // A lane's R velocities step along axis FA: x in 2D (consecutive nodes);
  // z in 3D (stride nv^2), along which R.w is constant (R has no z
  // component), so only the first KV projections advance, |R.w| is formed
  // once per edge, and its U-derivative sum is sign(R.w) times the group's.
  constexpr int FA = (D == 3) ? D - 1 : 0;
  constexpr int KV = (D == 3) ? D - 1 : D;
  constexpr int DD = D * D, REC = LEAN ? DD + D : DD + 2 * D + 1, CH = kAdjUChunk;
  __shared__ A rown[CH][P][REC], rtr[CH][P][REC];
  __shared__ int32_t ri[CH], rfl[CH][P];
  // tile-major logical order, each XCD on one contiguous range of patches
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x), np = gridDim.x / a.tiles;
  const int tile = lb / np, pb = lb - tile * np;
  const int tid = threadIdx.x, lane = tid;
  const size_t NVs = a.NV, cs = static_cast<size_t>(a.N) * NVs;
  const double dv = 2.0 * a.vmax / static_cast<double>(a.nv - 1);
  int jt[P];
#pragma unroll
  for (int t = 0; t < P; ++t) {
    const int gp = pb * P + t;
    jt[t] = gp < a.Ni ? a.plist[gp] : -1;
  }
  const int nu = a.ucount[pb];
  const size_t ub = static_cast<size_t>(pb) * a.ucap;
  A gU[P][D];
#pragma unroll
  for (int t = 0; t < P; ++t)
#pragma unroll
    for (int k = 0; k < D; ++k) gU[t][k] = A(0);
  const int ngroups = a.NV / R;
  const int g = tile * 64 + lane;
  const bool on = g < ngroups;
  // groups of one z plane first (3D), so consecutive lanes read consecutive
  // nodes of each plane
  const int zs = FA == 0 ? 1 : a.nv * a.nv;
  const uint32_t zsb = static_cast<uint32_t>(zs) * sizeof(Real);
  const int q0 = on ? (FA == 0 ? g * R : g % zs + (g / zs) * zs * R) : 0;
  const uint32_t qoff = static_cast<uint32_t>(q0) * sizeof(Real);
  // R values of this lane from / into the row that starts at p
  auto ldg = [&](const Real* p, A (&o)[R]) {
    if constexpr (FA == 0) load_rs<Real, R>(p + q0, o);
    else load_rz<Real, R>(p, qoff, zsb, o);
  };
  A v0[D];
  {
    int q = q0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      v0[k] = static_cast<A>(vnode(q % a.nv, a.nv, a.vmax));
      q /= a.nv;
    }
  }
  // lf = sum_i c_ij lam_ft_i (transposed term, dt applied at the end);
  // lj, fj: the particle's own lam_ft and f^n; csum = sum_i c_ji
  A lf[P][R][NC], lj[P][R][NC], fj[P][R][NC], csum[P][R];
#pragma unroll
  for (int t = 0; t < P; ++t) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      A t1[R], t2[R];
      if (jt[t] >= 0) {
        ldg(a.lam_ft + c * cs + static_cast<size_t>(jt[t]) * NVs, t1);
        ldg(a.f_n + c * cs + static_cast<size_t>(jt[t]) * NVs, t2);
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) t1[r] = t2[r] = A(0);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        lf[t][r][c] = A(0);
        lj[t][r][c] = t1[r];
        fj[t][r][c] = t2[r];
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) csum[t][r] = A(0);
  }

  // one record from the operator row o of particle k (U of particle k)
  auto make_rec = [&](const Real* o, int k, A* rec) {
    double ig = 0.0;
#pragma unroll
    for (int m = 0; m < D; ++m) {
      double b = 0.0;
#pragma unroll
      for (int mm = 0; mm < D; ++mm) {
        const double xo = static_cast<double>(o[m * D + mm]);
        rec[m * D + mm] = static_cast<A>(xo);
        b = b + xo * a.U_n[static_cast<size_t>(mm) * a.N + k];
      }
      const double inc = static_cast<double>(o[m * D + FA]) * dv;
      rec[DD + m] = static_cast<A>(b);
      if constexpr (!LEAN) {
        rec[DD + D + m] = static_cast<A>(inc);
        ig = ig + static_cast<double>(static_cast<A>(inc));
      }
    }
    if constexpr (!LEAN) rec[DD + 2 * D] = static_cast<A>(ig);
  };
  const A dva = static_cast<A>(dv);
  // the per-velocity increments of a record and their sum
  auto incs = [&](const A* rc, A (&ik)[D], A& dgw) {
    if constexpr (LEAN) {
#pragma unroll
      for (int k = 0; k < D; ++k) ik[k] = rc[k * D + FA] * dva;
      dgw = ik[0];
#pragma unroll
      for (int k = 1; k < D; ++k) dgw = dgw + ik[k];
    } else {
#pragma unroll
      for (int k = 0; k < D; ++k) ik[k] = rc[DD + D + k];
      dgw = rc[DD + 2 * D];
    }
  };

  for (int c0 = 0; c0 < nu; c0 += CH) {
    const int cn = min(CH, nu - c0);
    __syncthreads();  // the previous chunk is consumed
    for (int x = tid; x < cn * P; x += 64) {
      const int w = x / P, t = x - w * P;
      const size_t u = ub + c0 + w;
      const int i = a.uj[u];
      const int e = (a.ue[u] >> (8 * t)) & 0xFF;
      if (t == 0) ri[w] = i;
      int fl = 0;
      if (e != 0xFF) {
        // slot t's particle; the union holds no self entry
        const int j = a.plist[pb * P + t];
        const int64_t rj = static_cast<int64_t>(j) * a.cap + e;
        const int te = a.tidx[rj];
        fl = 1 | (te >= 0 ? 2 : 0);
        make_rec(a.ops + rj * DD, j, rown[w][t]);
        if (te >= 0) make_rec(a.ops + (static_cast<int64_t>(i) * a.cap + te) * DD, i, rtr[w][t]);
      }
      rfl[w][t] = fl;
    }
    __syncthreads();
    // rows of union entry w: f^n_i and lam_ft_i
    A fa[R][NC], la[R][NC], fb[R][NC], lb2[R][NC];
    auto load_entry = [&](int w, A (&fi)[R][NC], A (&li)[R][NC]) {
      const int i = ri[w];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        A t1[R], t2[R];
        ldg(a.f_n + c * cs + static_cast<size_t>(i) * NVs, t1);
        ldg(a.lam_ft + c * cs + static_cast<size_t>(i) * NVs, t2);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          fi[r][c] = t1[r];
          li[r][c] = t2[r];
        }
      }
      asm volatile("" ::: "memory");
    };
    // projections p_k = a_k.(v0 - U) of a record and g.w = sum_k p_k
    auto proj = [&](const A* rc, A (&p)[D], A& gw) {
#pragma unroll
      for (int k = 0; k < D; ++k) {
        A s1 = -rc[DD + k];
#pragma unroll
        for (int mm = 0; mm < D; ++mm) s1 = fma(rc[k * D + mm], v0[mm], s1);
        p[k] = s1;
      }
      gw = p[0];
#pragma unroll
      for (int k = 1; k < D; ++k) gw = gw + p[k];
      // the constant projections' |.| once
#pragma unroll
      for (int k = KV; k < D; ++k) gw = gw - fabs(p[k]);
    };
    auto entry = [&](int w, const A (&fi)[R][NC], const A (&li)[R][NC]) {
#pragma unroll
      for (int t = 0; t < P; ++t) {
        const int fl = rfl[w][t];
        if (fl & 1) {
          const A* rc = rown[w][t];
          A p[D], S[D], ik[D], gw;
          proj(rc, p, gw);
#pragma unroll
          for (int k = 0; k < D; ++k) S[k] = A(0);
          A dgw;
          incs(rc, ik, dgw);
          A sd = A(0);
#pragma unroll
          for (int r = 0; r < R; ++r) {
            if (r > 0) {
#pragma unroll
              for (int k = 0; k < KV; ++k) p[k] = p[k] + ik[k];
              gw = gw + dgw;
            }
            A cm = gw;  // 2 sum_k min(0, p_k)
#pragma unroll
            for (int k = 0; k < KV; ++k) cm = cm - fabs(p[k]);
            csum[t][r] = csum[t][r] + cm;
            A sdf = A(0);
#pragma unroll
            for (int c = 0; c < NC; ++c) sdf = fma(lj[t][r][c], fi[r][c] - fj[t][r][c], sdf);
            // sum over the group of [p_k < 0] sdf as (sum sdf - sum sign(p_k) sdf) / 2
            sd = sd + sdf;
#pragma unroll
            for (int k = 0; k < KV; ++k) S[k] = fma(copysign(A(1), p[k]), sdf, S[k]);
          }
          // a constant projection's sum: sign times the group's (exact)
#pragma unroll
          for (int k = KV; k < D; ++k) S[k] = copysign(A(1), p[k]) * sd;
          if (on) {
#pragma unroll
            for (int k = 0; k < D; ++k) S[k] = sd - S[k];  // 2 x the sums of [p_k < 0] sdf
#pragma unroll
            for (int mm = 0; mm < D; ++mm) {
              A tt = A(0);
#pragma unroll
              for (int k = 0; k < D; ++k) tt = fma(rc[k * D + mm], S[k], tt);
              gU[t][mm] = gU[t][mm] - tt;
            }
          }
        }
        if (fl & 2) {
          const A* rc = rtr[w][t];
          A p[D], ik[D], gw;
          proj(rc, p, gw);
          A dgw;
          incs(rc, ik, dgw);
#pragma unroll
          for (int r = 0; r < R; ++r) {
            if (r > 0) {
#pragma unroll
              for (int k = 0; k < KV; ++k) p[k] = p[k] + ik[k];
              gw = gw + dgw;
            }
            A cm = gw;
#pragma unroll
            for (int k = 0; k < KV; ++k) cm = cm - fabs(p[k]);
#pragma unroll
            for (int c = 0; c < NC; ++c) lf[t][r][c] = fma(cm, li[r][c], lf[t][r][c]);
          }
        }
      }
    };
    load_entry(0, fa, la);
    for (int w = 0; w < cn; w += 2) {
      if (w + 1 < cn) load_entry(w + 1, fb, lb2);
      entry(w, fa, la);
      if (w + 1 < cn) {
        if (w + 2 < cn) load_entry(w + 2, fa, la);
        entry(w + 1, fb, lb2);
      }
    }
  }
  const A dt = static_cast<A>(a.dt);
#pragma unroll
  for (int t = 0; t < P; ++t) {
    if (jt[t] < 0) continue;
    if (on) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        Real out[R];
#pragma unroll
        for (int r = 0; r < R; ++r)
          out[r] = fma(lj[t][r][c], fma(dt, csum[t][r], A(1)), -dt * lf[t][r][c]);
        Real* row = a.lam_f + c * cs + static_cast<size_t>(jt[t]) * NVs;
        if constexpr (FA == 0) {
#pragma unroll
          for (int r = 0; r < R; ++r) row[q0 + r] = out[r];
        } else {
          store_rz<Real, R>(row, qoff, zsb, out);
        }
      }
    }
#pragma unroll
    for (int mm = 0; mm < D; ++mm) {
      double s = static_cast<double>(gU[t][mm]);
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
      if (lane == 0) a.gpart[(static_cast<size_t>(tile) * D + mm) * a.N + jt[t]] = s;
    }
  }
}

// lam_U_j = -dt * (sum over the tiles of j, in tile order)  (interior j)
__global__ void k_adj_sum_tiles(int N, int D, int tiles, double dt,
                                const int32_t* __restrict__ wall_id,
                                const double* __restrict__ gpart, double* __restrict__ lam_U) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= static_cast<int64_t>(N) * D) return;
  const int mm = static_cast<int>(k / N), j = static_cast<int>(k - static_cast<int64_t>(mm) * N);
  double s = 0.0;
  for (int t = 0; t < tiles; ++t) s = s + gpart[(static_cast<size_t>(t) * D + mm) * N + j];
  lam_U[static_cast<size_t>(mm) * N + j] = wall_id[j] == 0 ? -dt * s : 0.0;
}

// ------------------------------------------------------------ objective
// J = dx^(d-1) sum_{lid b} q_n(b) + (ke/N) sum_i rho_i |U_i|^2 / 2,
// q_n = omega/2 sum_v (v_n - U_n)(|v-U|^2 f1 [+ f2]), n = last axis.
// Block per particle: its term of J into part[i] and its gradient rows.
template <int D, int NC, typename Real>
__global__ __launch_bounds__(kThreads) void k_objective(int N, int NV, int nv, double vmax,
                                                         double hw, double ke,
                                                         const int32_t* __restrict__ wall_id,
                                                         const Real* __restrict__ f,
                                                         const double* __restrict__ rho,
                                                         const double* __restrict__ U,
                                                         double* __restrict__ part,
                                                         Real* __restrict__ dJ_df,
                                                         double* __restrict__ dJ_drho,
                                                         double* __restrict__ dJ_dU) {
  __shared__ double sh[4 * (D + 1)];
  const int i = blockIdx.x;
  const size_t NVs = NV, cs = static_cast<size_t>(N) * NVs;
  const int an = D - 1;
  double Ui[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < D; ++a) Ui[a] = U[static_cast<size_t>(a) * N + i];
  const bool on_lid = wall_id[i] == 2 * D;  // block-uniform
  double s[D + 1];
#pragma unroll
  for (int k = 0; k <= D; ++k) s[k] = 0.0;
  for (int q = threadIdx.x; q < NV; q += kThreads) {
    double g0 = 0.0, g1 = 0.0;
    if (on_lid) {
      double v[3];
      velocity_of<D>(q, nv, vmax, v);
      double w2 = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a) w2 = w2 + (v[a] - Ui[a]) * (v[a] - Ui[a]);
      const double wn = v[an] - Ui[an];
      const double f1 = static_cast<double>(f[static_cast<size_t>(i) * NVs + q]);
      double e = w2 * f1;
      if (NC == 2) e = e + static_cast<double>(f[cs + static_cast<size_t>(i) * NVs + q]);
      s[0] = s[0] + wn * e;
#pragma unroll
      for (int a = 0; a < D; ++a) s[1 + a] = s[1 + a] - 2.0 * wn * (v[a] - Ui[a]) * f1;
      s[1 + an] = s[1 + an] - e;
      g0 = hw * wn * w2;
      g1 = hw * wn;
    }
    if (dJ_df) {
      dJ_df[static_cast<size_t>(i) * NVs + q] = static_cast<Real>(g0);
      if (NC == 2) dJ_df[cs + static_cast<size_t>(i) * NVs + q] = static_cast<Real>(g1);
    }
  }
  if (on_lid) block_sum<D + 1>(s, sh);
  if (threadIdx.x == 0) {
    double u2 = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) u2 = u2 + Ui[a] * Ui[a];
    part[i] = (on_lid ? hw * s[0] : 0.0) + (ke / N) * (0.5 * rho[i] * u2);
    if (dJ_drho) dJ_drho[i] = (ke / N) * 0.5 * u2;
    if (dJ_dU) {
#pragma unroll
      for (int a = 0; a < D; ++a)
        dJ_dU[static_cast<size_t>(a) * N + i] =
            (ke / N) * rho[i] * Ui[a] + (on_lid ? hw * s[1 + a] : 0.0);
    }
  }
}

// out = sum of part[0..n) in a fixed order (one block).
__global__ __launch_bounds__(kThreads) void k_sum_fixed(int n, const double* __restrict__ part,
                                                         double* __restrict__ out, int accumulate) {
  __shared__ double sh[4];
  double s[1] = {0.0};
  for (int k = threadIdx.x; k < n; k += kThreads) s[0] = s[0] + part[k];
  block_sum<1>(s, sh);
  if (threadIdx.x == 0) *out = accumulate ? *out + s[0] : s[0];
}

// lam_f += moments^T(lam_rho, lam_U, lam_T) for every particle.
template <int D, int NC, typename Real>
__global__ __launch_bounds__(kThreads) void k_moments_adj(int N, int NV, int nv, double vmax,
                                                           double omega,
                                                           const double* __restrict__ rho,
                                                           const double* __restrict__ U,
                                                           const double* __restrict__ T,
                                                           const double* __restrict__ lr,
                                                           const double* __restrict__ lU,
                                                           const double* __restrict__ lT,
                                                           Real* __restrict__ lam_f) {
  const int i = blockIdx.x;
  const size_t NVs = NV, cs = static_cast<size_t>(N) * NVs;
  double Ui[3] = {0.0, 0.0, 0.0}, lUi[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < D; ++a) {
    Ui[a] = U[static_cast<size_t>(a) * N + i];
    if (lU) lUi[a] = lU[static_cast<size_t>(a) * N + i];
  }
  const double s0 = rho[i] / omega, lri = lr ? lr[i] : 0.0, lTi = lT ? lT[i] : 0.0;
  for (int q = threadIdx.x; q < NV; q += kThreads) {
    double v[3];
    velocity_of<D>(q, nv, vmax, v);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      Real& o = lam_f[c * cs + static_cast<size_t>(i) * NVs + q];
      o = static_cast<Real>(static_cast<double>(o) +
                            mom_adj<D, NC>(c, v, omega, s0, Ui, T[i], lri, lUi, lTi));
    }
  }
}

// ------------------------------------------------------------ launchers
static double omega_adj(const bgk_config& cfg) {
  const double dv = 2.0 * cfg.vmax / static_cast<double>(cfg.nv - 1);
  double w = 1.0;
  for (int k = 0; k < cfg.dim; ++k) w = w * dv;
  return w;
}

hipError_t launch_adjoint_transposes(const Ctx& c) {
  const Adj& j = c.adj;
  hipLaunchKernelGGL(k_transpose_nbr, dim3((c.N + 127) / 128), dim3(128), 0, c.stream, c.N, c.cap,
                     c.d.wall_id, c.d.ncnt, c.d.nidx, j.tidx);
  hipError_t e = launch_fill_i32(c.stream, j.wtstart, c.N + 1, 0);
  if (e != hipSuccess) return e;
  if (c.Nw > 0)
    hipLaunchKernelGGL(k_wt_count, dim3(c.Nw), dim3(64), 0, c.stream, c.Nw, c.cap, c.d.wcnt,
                       c.d.widx, j.wtstart);
  e = launch_scan(c.stream, j.wtstart, c.N);
  if (e != hipSuccess) return e;
  e = launch_copy_i32(c.stream, j.wtstart, j.wtcursor, c.N);
  if (e != hipSuccess) return e;
  if (c.Nw > 0)
    hipLaunchKernelGGL(k_wt_scatter, dim3(c.Nw), dim3(64), 0, c.stream, c.Nw, c.cap, c.d.wcnt,
                       c.d.widx, j.wtcursor, j.wt);
  hipLaunchKernelGGL(k_wt_sort, dim3((c.N + 127) / 128), dim3(128), 0, c.stream, c.N, j.wtstart,
                     j.wt);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int P = adj_plan(c.cfg).P;
  return launch_unions(c, P, c.Ni, c.d.cperm, c.d.ncnt, c.d.nidx, 1, P * c.cap, j.ucount, j.uj,
                       j.ue);
}

// The patch kernel's instantiation for the plan: one wavefront per (patch,
// 64-lane tile).
template <int D, int NC, typename Real, int R>
static hipError_t launch_adj_patch(const Ctx& c, const AdjArgs<Real>& a, const AdjPlan& ap,
                                   int npa) {
  constexpr int P = 2;
  if (ap.P != P) return hipErrorInvalidValue;
  const int64_t nb = static_cast<int64_t>(npa) * ap.tiles;
  if (nb > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_adj_transport_patch<D, NC, Real, R, P>), dim3(static_cast<unsigned>(nb)),
                     dim3(64), 0, c.stream, a);
  return hipGetLastError();
}

// S5-S6 adjoint: 16-byte row pieces (R = 2 doubles, or 4 floats when 4
// divides nv), and 32 registers of the adjoint of f' kept per thread.
template <int D, int NC, typename Real>
static void launch_adj_collide(const Ctx& c, const AdjArgs<Real>& a, dim3 t, size_t lds) {
  constexpr int W = static_cast<int>(sizeof(Real)) / 4;
  if constexpr (W == 1) {
    if (c.cfg.nv % 4 == 0) {
      constexpr int R = 4, KEEP = 32 / (R * NC);
      hipLaunchKernelGGL((k_adj_collide<D, NC, Real, R, KEEP>), dim3(c.Ni), t, lds, c.stream, a);
      return;
    }
  }
  constexpr int R = 2, KEEP = 32 / (R * NC * W);
  hipLaunchKernelGGL((k_adj_collide<D, NC, Real, R, KEEP>), dim3(c.Ni), t, lds, c.stream, a);
}

template <typename Real>
static hipError_t adjoint_step_t(const Ctx& c, const Real* f_n, const double* U_n,
                                 const Real* lam_f1, const double* lam_U1, const double* lam_rho1,
                                 const double* lam_T1, Real* lam_f, double* lam_U,
                                 double* dJ_dlid, bool wall_rows, const AdjState* kept = nullptr) {
  const Adj& j = c.adj;
  // the recomputed step (the adjoint workspace), or the one the caller kept
  const AdjState st = kept ? *kept : AdjState{j.ft, j.f1, j.rho1, j.U1, j.T1};
  const Real* ops = std::is_same<Real, double>::value
                        ? reinterpret_cast<const Real*>(c.d.ops64)
                        : reinterpret_cast<const Real*>(c.d.ops32);
  AdjArgs<Real> a{c.N,        c.NV,       c.cfg.nv,   c.cap,       c.Nw,     c.Ni,     c.D,
                  c.cfg.vmax, omega_adj(c.cfg), c.cfg.kn, c.cfg.dt,  c.lid,    c.cfg.wall_T,
                  c.d.wall_id, c.d.wall_list, c.d.cperm, c.d.ncnt, c.d.nidx, j.tidx, ops,
                  c.d.wcnt,   c.d.widx,   c.d.wc0,    j.wtstart,   j.wt,     f_n,      U_n,
                  static_cast<const Real*>(st.ft), static_cast<const Real*>(st.f1), st.rho1, st.U1,
                  st.T1,      lam_f1,     lam_U1,     lam_rho1,    lam_T1,
                  static_cast<Real*>(j.larr), static_cast<Real*>(j.lam_ft), lam_f, lam_U,
                  j.lidpart, j.gpart, 0,
                  nullptr,    j.ucount,   j.uj,       j.ue,        0};
  const AdjPlan ap = adj_plan(c.cfg);
  a.ucap = ap.P * c.cap;
  dim3 t(kThreads);
  const size_t lds = static_cast<size_t>(c.D + 1) * c.cfg.nv * sizeof(double);
  // reverse transport: one wavefront per (patch of interior particles or
  // wall particle, 64-lane tile), then the tile parts of lam_U summed in
  // tile order
  const int R = ap.R;
  a.tiles = ap.tiles;
  const int npa = (c.Ni + ap.P - 1) / ap.P;
  const int64_t nbw = static_cast<int64_t>(c.Nw) * ap.tiles_w;
  if (nbw > INT32_MAX) return hipErrorInvalidValue;
  const dim3 tw(static_cast<unsigned>(nbw)), tt(64);
  AdjArgs<Real> aw = a;
  aw.jlist = c.d.wall_list;
  aw.tiles = ap.tiles_w;  // (wall rows of gpart: never summed into lam_U)
  hipError_t e = hipSuccess;
  if (c.D == 2) {
    if (c.Nw) hipLaunchKernelGGL((k_adj_wall<2, 2, Real>), dim3(c.Nw), t, lds, c.stream, a);
    if (wall_rows) {
      e = launch_adjoint_wallrow(c);
      if (e != hipSuccess) return e;
    }
    if (c.Ni) launch_adj_collide<2, 2, Real>(c, a, t, lds);
    if (R == 4) {
      if (npa) e = launch_adj_patch<2, 2, Real, 4>(c, a, ap, npa);
      if (e != hipSuccess) return e;
      if (c.Nw) hipLaunchKernelGGL((k_adj_transport_wall<2, 2, Real, 4>), tw, tt, 0, c.stream, aw);
    } else {
      if (npa) e = launch_adj_patch<2, 2, Real, 2>(c, a, ap, npa);
      if (e != hipSuccess) return e;
      if (c.Nw) hipLaunchKernelGGL((k_adj_transport_wall<2, 2, Real, 2>), tw, tt, 0, c.stream, aw);
    }
  } else {
    if (c.Nw) hipLaunchKernelGGL((k_adj_wall<3, 1, Real>), dim3(c.Nw), t, lds, c.stream, a);
    if (wall_rows) {
      e = launch_adjoint_wallrow(c);
      if (e != hipSuccess) return e;
    }
    if (c.Ni) launch_adj_collide<3, 1, Real>(c, a, t, lds);
    if (npa) {
      if constexpr (std::is_same<Real, float>::value) {
        if (R == 5) e = launch_adj_patch<3, 1, Real, 5>(c, a, ap, npa);
      } else {
        if (R == 5) return hipErrorInvalidValue;  // (the plan takes 5 for FP32 storage only)
      }
      if (R == 4) e = launch_adj_patch<3, 1, Real, 4>(c, a, ap, npa);
      if (R == 2) e = launch_adj_patch<3, 1, Real, 2>(c, a, ap, npa);
    }
    if (e != hipSuccess) return e;
    if (c.Nw) {
      if (ap.Rw == 4) hipLaunchKernelGGL((k_adj_transport_wall<3, 1, Real, 4>), tw, tt, 0, c.stream, aw);
      else hipLaunchKernelGGL((k_adj_transport_wall<3, 1, Real, 2>), tw, tt, 0, c.stream, aw);
    }
  }
  const int64_t nu = static_cast<int64_t>(c.N) * c.D;
  hipLaunchKernelGGL(k_adj_sum_tiles, dim3(static_cast<unsigned>((nu + 255) / 256)), dim3(256), 0,
                     c.stream, c.N, c.D, a.tiles, c.cfg.dt, c.d.wall_id, j.gpart, lam_U);
  if (c.Nw && dJ_dlid)
    hipLaunchKernelGGL(k_sum_fixed, dim3(1), t, 0, c.stream, c.Nw, j.lidpart, dJ_dlid, 1);
  return hipGetLastError();
}

hipError_t launch_adjoint_step(const Ctx& c, const void* f_n, const double* U_n,
                               const void* lam_f1, const double* lam_U1, const double* lam_rho1,
                               const double* lam_T1, void* lam_f, double* lam_U,
                               double* dJ_dlid, bool wall_rows) {
  if (c.cfg.precision == BGK_FP64)
    return adjoint_step_t<double>(c, static_cast<const double*>(f_n), U_n,
                                  static_cast<const double*>(lam_f1), lam_U1, lam_rho1, lam_T1,
                                  static_cast<double*>(lam_f), lam_U, dJ_dlid, wall_rows);
  return adjoint_step_t<float>(c, static_cast<const float*>(f_n), U_n,
                               static_cast<const float*>(lam_f1), lam_U1, lam_rho1, lam_T1,
                               static_cast<float*>(lam_f), lam_U, dJ_dlid, wall_rows);
}

hipError_t launch_adjoint_step_kept(const Ctx& c, const void* f_n, const double* U_n,
                                    const AdjState& s, const void* lam_f1, const double* lam_U1,
                                    const double* lam_rho1, const double* lam_T1, void* lam_f,
                                    double* lam_U, double* dJ_dlid) {
  if (c.cfg.precision == BGK_FP64)
    return adjoint_step_t<double>(c, static_cast<const double*>(f_n), U_n,
                                  static_cast<const double*>(lam_f1), lam_U1, lam_rho1, lam_T1,
                                  static_cast<double*>(lam_f), lam_U, dJ_dlid, false, &s);
  return adjoint_step_t<float>(c, static_cast<const float*>(f_n), U_n,
                               static_cast<const float*>(lam_f1), lam_U1, lam_rho1, lam_T1,
                               static_cast<float*>(lam_f), lam_U, dJ_dlid, false, &s);
}

template <typename Real>
static void objective_t(const Ctx& c, const Real* f, const double* rho, const double* U,
                        double hw, double ke, double* dJ_drho, double* dJ_dU, Real* dJ_df,
                        double* part) {
  if (c.D == 2)
    hipLaunchKernelGGL((k_objective<2, 2, Real>), dim3(c.N), dim3(kThreads), 0, c.stream, c.N,
                       c.NV, c.cfg.nv, c.cfg.vmax, hw, ke, c.d.wall_id, f, rho, U, part,
                       dJ_df, dJ_drho, dJ_dU);
  else
    hipLaunchKernelGGL((k_objective<3, 1, Real>), dim3(c.N), dim3(kThreads), 0, c.stream, c.N,
                       c.NV, c.cfg.nv, c.cfg.vmax, hw, ke, c.d.wall_id, f, rho, U, part,
                       dJ_df, dJ_drho, dJ_dU);
}

hipError_t launch_objective(const Ctx& c, const void* f, const double* rho, const double* U,
                            double ke, double* J, void* dJ_df, double* dJ_drho, double* dJ_dU,
                            double* part) {
  double area = 1.0;
  for (int k = 0; k < c.D - 1; ++k) area = area * c.cfg.dx;
  const double hw = 0.5 * omega_adj(c.cfg) * area;
  if (c.cfg.precision == BGK_FP64)
    objective_t<double>(c, static_cast<const double*>(f), rho, U, hw, ke, dJ_drho, dJ_dU,
                        static_cast<double*>(dJ_df), part);
  else
    objective_t<float>(c, static_cast<const float*>(f), rho, U, hw, ke, dJ_drho, dJ_dU,
                       static_cast<float*>(dJ_df), part);
  hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(kThreads), 0, c.stream, c.N, part, J, 0);
  return hipGetLastError();
}

template <typename Real>
static void moments_adjoint_t(const Ctx& c, const double* rho, const double* U, const double* T,
                              const double* lr, const double* lU, const double* lT, Real* lam_f) {
  const double om = omega_adj(c.cfg);
  if (c.D == 2)
    hipLaunchKernelGGL((k_moments_adj<2, 2, Real>), dim3(c.N), dim3(kThreads), 0, c.stream, c.N,
                       c.NV, c.cfg.nv, c.cfg.vmax, om, rho, U, T, lr, lU, lT, lam_f);
  else
    hipLaunchKernelGGL((k_moments_adj<3, 1, Real>), dim3(c.N), dim3(kThreads), 0, c.stream, c.N,
                       c.NV, c.cfg.nv, c.cfg.vmax, om, rho, U, T, lr, lU, lT, lam_f);
}

hipError_t launch_moments_adjoint(const Ctx& c, const double* rho, const double* U,
                                  const double* T, const double* lr, const double* lU,
                                  const double* lT, void* lam_f) {
  if (c.cfg.precision == BGK_FP64)
    moments_adjoint_t<double>(c, rho, U, T, lr, lU, lT, static_cast<double*>(lam_f));
  else
    moments_adjoint_t<float>(c, rho, U, T, lr, lU, lT, static_cast<float*>(lam_f));
  return hipGetLastError();
}

}  // namespace bgk
