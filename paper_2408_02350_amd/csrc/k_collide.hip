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

// Tables of one block in LDS (dynamic, (D+1)*nv doubles): the velocity
// nodes v_k, then per axis a the factor exp(-(v_k - U_a)^2 / (2T)) of one
// particle's Maxwellian, so that M = norm * prod_a e_a[k_a] (d*nv
// exponentials per particle instead of N_v).
__device__ __forceinline__ void fill_vtab(double* vt, int nv, double vmax) {
  for (int k = threadIdx.x; k < nv; k += blockDim.x) vt[k] = vnode(k, nv, vmax);
}

template <int D>
__device__ __forceinline__ void fill_etab(double* et, const double* vt, int nv, const double* U,
                                          double T) {
  for (int i = threadIdx.x; i < D * nv; i += blockDim.x) {
    const int a = i / nv, k = i - a * nv;
    const double d = vt[k] - U[a];
    et[i] = exp(-(d * d) / (2.0 * T));
  }
}


// Normalisation of the Maxwellian (Sec. 2 eq. maxwellian; Chu G1 in 2D).
template <int D>
__device__ __forceinline__ double maxwell_norm(double rho, double T) {
  const double tp = 2.0 * kPi * T;
  return D == 3 ? rho / (tp * sqrt(tp)) : rho / tp;
}

template <int D>
static inline size_t row_tab_bytes(int nv) {
  return static_cast<size_t>(D + 1) * nv * sizeof(double);
}

// rho, U, T of one particle's row (Sec. 2 eqs. moments, internal_energy;
// Chu eq. macroeq; time-discrete fullmoment1a / moment1a, moment1b):
// rho = omega sum f1, U = sum v f1 / sum f1, then 3 rho T from the centred
// second moment (Chu: plus sum g2).  vt: the velocity nodes in LDS.
template <int D, int NC, typename Real>
__device__ __forceinline__ void row_moments(const Real* row, size_t cs, int NV, int nv,
                                            const double* vt, double omega, double* sh,
                                            double& rho, double* U, double& T) {
  double s[D + 1];
#pragma unroll
  for (int k = 0; k <= D; ++k) s[k] = 0.0;
  VelDigits<D> vd;
  vd.init(threadIdx.x, kThreads, nv);
  for (int q = threadIdx.x; q < NV; q += kThreads, vd.advance(nv)) {
    const int* kq = vd.k;
    const double f1 = static_cast<double>(row[q]);
    s[0] = s[0] + f1;
#pragma unroll
    for (int k = 0; k < D; ++k) s[1 + k] = s[1 + k] + vt[kq[k]] * f1;
  }
  block_sum<D + 1>(s, sh);
  const double s0 = s[0];
  rho = omega * s0;
#pragma unroll
  for (int k = 0; k < D; ++k) U[k] = s[1 + k] / s0;
  double e[1] = {0.0};
  vd.init(threadIdx.x, kThreads, nv);
  for (int q = threadIdx.x; q < NV; q += kThreads, vd.advance(nv)) {
    const int* kq = vd.k;
    double w2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double wk = vt[kq[k]] - U[k];
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
  extern __shared__ double vt[];  // nodes, then per-axis Maxwellian factors
  const int i = a.plist[blockIdx.x];
  fill_vtab(vt, a.nv, a.vmax);
  __syncthreads();
  const size_t NVs = a.NV, cs = static_cast<size_t>(a.N) * NVs;
  const Real* ft = static_cast<const Real*>(a.ft) + static_cast<size_t>(i) * NVs;
  Real* fo = static_cast<Real*>(a.fo) + static_cast<size_t>(i) * NVs;
  double rho, U[3] = {0.0, 0.0, 0.0}, T;
  row_moments<D, NC, Real>(ft, cs, a.NV, a.nv, vt, a.omega, sh, rho, U, T);
  if (threadIdx.x == 0) {
    a.rho[i] = rho;
    a.T[i] = T;
#pragma unroll
    for (int k = 0; k < D; ++k) a.U[static_cast<size_t>(k) * a.N + i] = U[k];
    if (!(rho > 0.0) || !(T > 0.0)) raise_error(a.err, BGK_ENONPHYS);
  }
  const double tau = a.kn * sqrt(2.0 / kPi) / (rho * sqrt(T));
  const double den = tau + a.dt;
  double* et = vt + a.nv;
  fill_etab<D>(et, vt, a.nv, U, T);
  __syncthreads();
  const double norm = maxwell_norm<D>(rho, T);
  VelDigits<D> vd;
  vd.init(threadIdx.x, kThreads, a.nv);
  for (int q = threadIdx.x; q < a.NV; q += kThreads, vd.advance(a.nv)) {
    const int* kq = vd.k;
    double M = norm;
#pragma unroll
    for (int k = 0; k < D; ++k) M = M * et[k * a.nv + kq[k]];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double Mc = c == 0 ? M : T * M;  // Chu: G2 = T G1
      const double x = static_cast<double>(ft[c * cs + q]);
      fo[c * cs + q] = static_cast<Real>((tau * x + a.dt * Mc) / den);
    }
  }
}

template <typename Real, int D, int NC>
static void collide_t(const Ctx& c, const CollideArgs& a) {
  hipLaunchKernelGGL((k_collide<D, NC, Real>), dim3(a.count), dim3(kThreads),
                     row_tab_bytes<D>(c.cfg.nv), c.stream, a);
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
  // wall patches (kernel instances with P > 1): slots of each patch, and the
  // union of their interpolation rows
  const int32_t* wpl;
  const int32_t* wucount;
  const int32_t* wuj;
  const uint32_t* wue;
  int wucap;
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

// R consecutive elements of a row written with the widest aligned vector
// store (p is aligned to R elements).
template <typename Real, int R>
__device__ __forceinline__ void store_vec(Real* __restrict__ p, const Real (&x)[R]) {
  constexpr int W = (R * sizeof(Real)) % 16 == 0 ? 16 / static_cast<int>(sizeof(Real)) : R;
  typedef Real V __attribute__((ext_vector_type(W)));
  V* pv = reinterpret_cast<V*>(__builtin_assume_aligned(p, W * sizeof(Real)));
#pragma unroll
  for (int i = 0; i < R / W; ++i) {
    V y;
#pragma unroll
    for (int w = 0; w < W; ++w) y[w] = x[i * W + w];
    pv[i] = y;
  }
}

// Diffuse reflection on wall particles (S7; one block of up to 256 threads
// per wall particle, P = 1, or per wall patch of P wall particles of one
// face, P > 1).  With the owner wall's inward normal s e_a, the arriving
// velocities (s v_a <= 0) are exactly the half k_a < nv/2 (s > 0) or
// k_a >= nv/2 (s < 0) of axis a (v_k is odd about the grid centre and nv is
// even), and the emitted ones the other half.  Both halves are walked as
// groups of R consecutive velocities along the fastest axis (R divides
// nv/2), so every lane of a gather has work:
//   arriving: f_b(v) = sum_e c0_e f_j(v) (rows four at a time), and the
//     inflow sum_arriving (-v.n) f_b1;
//   emitted:  f_b = rho_w M[1, U_w, T_w] (Chu: G1 and T_w G1 scaled by rho_w),
//     rho_w = inflow / sum_emitted (v.n) M[1, U_w, T_w].
// A wall patch walks the ascending union of its particles' rows once, each
// row feeding every particle with its weight (0 where the row is not the
// particle's): each particle's sum takes its own terms in its own row order
// (adding exact zeros in between), so the result is the per-particle one
// bit for bit, with each f_j row read once per patch.
// The Maxwellian is a product of per-axis exponentials held in LDS, and the
// emitted outflow sum factorises into per-axis sums.  The particle's moments
// are summed as its values are written: sum f, sum v f and the second moment
// about the wall velocity, shifted exactly to the centred one once U is
// known, so no row is read back.
template <int D, int NC, typename Real, int R, int P>
__global__ __launch_bounds__(kThreads) void k_wall_bc(const WallBcArgs a) {
  // v_k [nv], exp(-(v_k - Uw_a)^2 / (2 T_w)) [D][nv]; wall patches then
  // hold the union's weights [wucap][P] and rows [wucap]
  extern __shared__ double wtab[];
  constexpr int SM = D + 2;  // per particle: sum f, sum v f (d), sum |v - U_w|^2 f (+ sum g2)
  __shared__ double sh[16 * P * SM];
  __shared__ double axsum[D];
  const int nv = a.nv, hv = nv / 2;
  double* vtab = wtab;
  double* etab = wtab + nv;
  double* uw = etab + D * nv;
  int32_t* ur = reinterpret_cast<int32_t*>(uw + (P > 1 ? a.wucap * P : 0));
  const int k = xcd_logical_block(blockIdx.x, gridDim.x);  // neighbouring walls share an L2
  const int nw = blockDim.x >> 6;
  int kt[P], bt[P];  // wall-list slot and particle of each patch entry (-1: empty)
#pragma unroll
  for (int t = 0; t < P; ++t) {
    kt[t] = P == 1 ? k : a.wpl[static_cast<size_t>(k) * P + t];
    bt[t] = kt[t] >= 0 ? a.wall_list[kt[t]] : -1;
  }
  const int w = a.wall_id[bt[0]];  // entry 0 always holds a particle
  const int axis = (w - 1) / 2;
  const double sgn = ((w - 1) % 2 == 0) ? 1.0 : -1.0;
  const bool is_lid = (w == 2 * D);
  const double Uw[3] = {is_lid ? a.lid : 0.0, 0.0, 0.0};
  const double Tw = a.wall_T;
  for (int i = threadIdx.x; i < D * nv; i += blockDim.x) {
    const int ax = i / nv, kk = i - ax * nv;
    const double v = vnode(kk, nv, a.vmax);
    if (ax == 0) vtab[kk] = v;
    const double dv = v - Uw[ax];
    etab[i] = exp(-(dv * dv) / (2.0 * Tw));
  }
  int nu = 0;
  if (P > 1) {
    nu = a.wucount[k];
    const size_t ub = static_cast<size_t>(k) * a.wucap;
    for (int u = threadIdx.x; u < nu; u += blockDim.x) {
      const uint32_t pe = a.wue[ub + u];
      ur[u] = a.wuj[ub + u];
#pragma unroll
      for (int t = 0; t < P; ++t) {
        const int e = (pe >> (8 * t)) & 0xFF;
        uw[u * P + t] = (kt[t] >= 0 && e != 0xFF)
                            ? a.wc0[static_cast<size_t>(kt[t]) * a.cap + e] : 0.0;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < D) {
    const int ax = threadIdx.x;
    double t = 0.0;
    for (int kk = 0; kk < nv; ++kk) {
      const double e = etab[ax * nv + kk];
      if (ax != axis) {
        t = t + e;
      } else {
        const double vn = sgn * vtab[kk];
        if (vn > 0.0) t = t + vn * e;
      }
    }
    axsum[ax] = t;
  }
  // normalisation of M[1, U_w, T_w] (Sec. 2; Chu G1 in 2D)
  const double tp = 2.0 * kPi * Tw;
  const double norm = D == 3 ? 1.0 / (tp * sqrt(tp)) : 1.0 / tp;

  int m[P];
#pragma unroll
  for (int t = 0; t < P; ++t) m[t] = kt[t] >= 0 ? a.wcnt[kt[t]] : 0;
  const int32_t* row = a.widx + static_cast<size_t>(k) * a.cap;
  const double* c0 = a.wc0 + static_cast<size_t>(k) * a.cap;
  const size_t NVs = a.NV, cs = static_cast<size_t>(a.N) * NVs;
  Real* f = static_cast<Real*>(a.f);
  const int G = a.NV / (2 * R);  // groups per half
  const int off_in = sgn > 0.0 ? 0 : hv, off_out = hv - off_in;
  // group g of the half whose axis-a indices start at offa: first velocity
  // index and its per-axis indices
  auto group_q = [&](int g, int offa, int (&kq)[3]) {
    int rest = g, q = 0, stride = 1;
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
      const int ext = (ax == axis ? hv : nv) / (ax == 0 ? R : 1);
      int kk = rest % ext;
      rest /= ext;
      if (ax == 0) kk *= R;
      if (ax == axis) kk += offa;
      kq[ax] = kk;
      q += kk * stride;
      stride *= nv;
    }
    return q;
  };

  double inflow[P];
  double sm[P * SM];
#pragma unroll
  for (int t = 0; t < P; ++t) inflow[t] = 0.0;
#pragma unroll
  for (int kk = 0; kk < P * SM; ++kk) sm[kk] = 0.0;
  for (int g = threadIdx.x; g < G; g += blockDim.x) {
    int kq[3] = {0, 0, 0};
    const int q0 = group_q(g, off_in, kq);
    double s[P][NC][R];
#pragma unroll
    for (int t = 0; t < P; ++t)
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int r = 0; r < R; ++r) s[t][c][r] = 0.0;
    const int n = P == 1 ? m[0] : nu;
    int e = 0;
    for (; e + 4 <= n; e += 4) {
      Real x[4][NC][R];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = P == 1 ? row[e + u] : ur[e + u];
#pragma unroll
        for (int c = 0; c < NC; ++c)
          load_vec<Real, R>(f + c * cs + static_cast<size_t>(j) * NVs + q0, x[u][c]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int t = 0; t < P; ++t) {
          const double wu = P == 1 ? c0[e + u] : uw[(e + u) * P + t];
#pragma unroll
          for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int r = 0; r < R; ++r)
              s[t][c][r] = s[t][c][r] + wu * static_cast<double>(x[u][c][r]);
        }
      }
    }
    for (; e < n; ++e) {
      Real x[NC][R];
      const int j = P == 1 ? row[e] : ur[e];
#pragma unroll
      for (int c = 0; c < NC; ++c)
        load_vec<Real, R>(f + c * cs + static_cast<size_t>(j) * NVs + q0, x[c]);
#pragma unroll
      for (int t = 0; t < P; ++t) {
        const double wu = P == 1 ? c0[e] : uw[e * P + t];
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int r = 0; r < R; ++r) s[t][c][r] = s[t][c][r] + wu * static_cast<double>(x[c][r]);
      }
    }
    double v[3] = {0.0, 0.0, 0.0}, wfix = 0.0;
#pragma unroll
    for (int ax = 1; ax < D; ++ax) {
      v[ax] = vtab[kq[ax]];
      wfix = wfix + v[ax] * v[ax];  // (U_w has no component off axis 0)
    }
#pragma unroll
    for (int t = 0; t < P; ++t) {
      if (bt[t] < 0) continue;
      Real* fb = f + static_cast<size_t>(bt[t]) * NVs;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        Real y[R];
#pragma unroll
        for (int r = 0; r < R; ++r) y[r] = static_cast<Real>(s[t][c][r]);
        store_vec<Real, R>(fb + c * cs + q0, y);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double x0 = static_cast<double>(y[r]);
          if (c == 0) {
            v[0] = vtab[kq[0] + r];
            const double w0 = v[0] - Uw[0];
            inflow[t] = inflow[t] + (-sgn * v[axis]) * x0;
            sm[t * SM] = sm[t * SM] + x0;
#pragma unroll
            for (int ax = 0; ax < D; ++ax) sm[t * SM + 1 + ax] = sm[t * SM + 1 + ax] + v[ax] * x0;
            sm[t * SM + 1 + D] = sm[t * SM + 1 + D] + (w0 * w0 + wfix) * x0;
          } else {
            sm[t * SM + 1 + D] = sm[t * SM + 1 + D] + x0;
          }
        }
      }
    }
  }
  block_sum_n<P>(inflow, sh, nw);  // its barriers also publish axsum
  double outflow = norm;
#pragma unroll
  for (int ax = 0; ax < D; ++ax) outflow = outflow * axsum[ax];
  double cw[P];
#pragma unroll
  for (int t = 0; t < P; ++t) {
    const double rho_w = inflow[t] / outflow;
    cw[t] = rho_w * norm;
  }
  for (int g = threadIdx.x; g < G; g += blockDim.x) {
    int kq[3] = {0, 0, 0};
    const int q0 = group_q(g, off_out, kq);
    double v[3] = {0.0, 0.0, 0.0}, wfix = 0.0;
#pragma unroll
    for (int ax = 1; ax < D; ++ax) {
      v[ax] = vtab[kq[ax]];
      wfix = wfix + v[ax] * v[ax];
    }
#pragma unroll
    for (int t = 0; t < P; ++t) {
      if (bt[t] < 0) continue;
      double efix = cw[t];
#pragma unroll
      for (int ax = 1; ax < D; ++ax) efix = efix * etab[ax * nv + kq[ax]];
      Real y[NC][R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double g1 = efix * etab[kq[0] + r];
        y[0][r] = static_cast<Real>(g1);
        if (NC == 2) y[NC - 1][r] = static_cast<Real>(Tw * g1);
        v[0] = vtab[kq[0] + r];
        const double w0 = v[0] - Uw[0];
        const double x0 = static_cast<double>(y[0][r]);
        sm[t * SM] = sm[t * SM] + x0;
#pragma unroll
        for (int ax = 0; ax < D; ++ax) sm[t * SM + 1 + ax] = sm[t * SM + 1 + ax] + v[ax] * x0;
        sm[t * SM + 1 + D] = sm[t * SM + 1 + D] + (w0 * w0 + wfix) * x0;
        if (NC == 2) sm[t * SM + 1 + D] = sm[t * SM + 1 + D] + static_cast<double>(y[NC - 1][r]);
      }
      Real* fb = f + static_cast<size_t>(bt[t]) * NVs;
#pragma unroll
      for (int c = 0; c < NC; ++c) store_vec<Real, R>(fb + c * cs + q0, y[c]);
    }
  }
  block_sum_n<P * SM>(sm, sh, nw);
  // the centred second moment from the sums about U_w: sum |v - U|^2 f =
  // sum |v - U_w|^2 f - s0 |U - U_w|^2 (exact; |U - U_w| is small, so
  // nothing cancels), without reading the row a third time
  double U[P][3], e2[P];
#pragma unroll
  for (int t = 0; t < P; ++t) {
    U[t][0] = U[t][1] = U[t][2] = 0.0;
    double du = 0.0;
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
      U[t][ax] = sm[t * SM + 1 + ax] / sm[t * SM];
      const double d = U[t][ax] - Uw[ax];
      du = du + d * d;
    }
    e2[t] = sm[t * SM + 1 + D] - sm[t * SM] * du;
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int t = 0; t < P; ++t) {
      if (bt[t] < 0) continue;
      const int b = bt[t];
      const double s0 = sm[t * SM];
      const double rho = a.omega * s0;
      const double T = e2[t] / (3.0 * s0);
      a.rho[b] = rho;
      a.T[b] = T;
#pragma unroll
      for (int ax = 0; ax < D; ++ax) a.U[static_cast<size_t>(ax) * a.N + b] = U[t][ax];
      if (!(rho > 0.0) || !(T > 0.0) || m[t] == 0) raise_error(a.err, BGK_ENONPHYS);
    }
  }
}

template <int D, int NC, typename Real, int R>
static void wall_bc_r(const Ctx& c, const WallBcArgs& a, dim3 t, size_t lds) {
  if constexpr (D == 3) {  // wall patches are formed in 3D only
    if (c.npw > 0) {
      const size_t ul = static_cast<size_t>(c.wucap) * (kWallPatch * sizeof(double) + sizeof(int32_t));
      hipLaunchKernelGGL((k_wall_bc<D, NC, Real, R, kWallPatch>), dim3(c.npw), t, lds + ul,
                         c.stream, a);
      return;
    }
  }
  hipLaunchKernelGGL((k_wall_bc<D, NC, Real, R, 1>), dim3(c.Nw), t, lds, c.stream, a);
}

template <int D, int NC, typename Real>
static void wall_bc_t(const Ctx& c, const WallBcArgs& a) {
  const int hv = c.cfg.nv / 2;  // nv is even
  const int R = hv % 4 == 0 ? 4 : (hv % 2 == 0 ? 2 : 1);
  const int groups = c.NV / (2 * R);
  const dim3 t(std::min(kThreads, (groups + 63) / 64 * 64));
  const size_t lds = static_cast<size_t>(D + 1) * c.cfg.nv * sizeof(double);
  if (R == 4) wall_bc_r<D, NC, Real, 4>(c, a, t, lds);
  else if (R == 2) wall_bc_r<D, NC, Real, 2>(c, a, t, lds);
  else wall_bc_r<D, NC, Real, 1>(c, a, t, lds);
}

hipError_t launch_wall_bc(const Ctx& c, void* f, double* rho, double* U, double* T) {
  if (c.Nw == 0) return hipSuccess;
  WallBcArgs a{c.N,          c.NV,      c.cfg.nv,      c.cap,  c.Nw,   c.D,    c.cfg.vmax,
               omega_of(c.cfg), c.lid,  c.cfg.wall_T,  c.d.wall_list, c.d.wall_id, c.d.wcnt,
               c.d.widx,     c.d.wc0,   f,             rho,    U,      T,      c.d.err,
               c.d.wpl,      c.d.wucount, c.d.wuj,     c.d.wue, c.wucap};
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
  extern __shared__ double vt[];
  const int i = blockIdx.x;
  const size_t NVs = NV, cs = static_cast<size_t>(N) * NVs;
  const Real* row = static_cast<const Real*>(fv) + static_cast<size_t>(i) * NVs;
  fill_vtab(vt, nv, vmax);
  __syncthreads();
  double r, u[3] = {0.0, 0.0, 0.0}, t;
  row_moments<D, NC, Real>(row, cs, NV, nv, vt, omega, sh, r, u, t);
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
  const size_t lds = static_cast<size_t>(c.D + 1) * c.cfg.nv * sizeof(double);
  if (c.D == 2) {
    if (f64) hipLaunchKernelGGL((k_moments<2, 2, double>), g, t, lds, c.stream, c.N, c.NV, c.cfg.nv, c.cfg.vmax, om, f, rho, U, T);
    else hipLaunchKernelGGL((k_moments<2, 2, float>), g, t, lds, c.stream, c.N, c.NV, c.cfg.nv, c.cfg.vmax, om, f, rho, U, T);
  } else {
    if (f64) hipLaunchKernelGGL((k_moments<3, 1, double>), g, t, lds, c.stream, c.N, c.NV, c.cfg.nv, c.cfg.vmax, om, f, rho, U, T);
    else hipLaunchKernelGGL((k_moments<3, 1, float>), g, t, lds, c.stream, c.N, c.NV, c.cfg.nv, c.cfg.vmax, om, f, rho, U, T);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- state check
// The health of a state (f, rho, U, T), typically f^{n+1} with the moments
// a step reported: per particle, its row's moments recomputed as bgk_moments
// does, against the given rho, U, T (after a step the difference is the
// relaxation's conservation defect: the discrete Maxwellian's moments differ
// from their parameters by the quadrature error), the smallest value and the
// counts of negative and of non-finite values over the row, and the
// particle's mass rho, momentum rho U and energy rho (|U|^2 + 3T)/2 (three
// degrees of freedom in both models: the Chu g2 carries the third).  Slots:
//   0 min f, 1 negatives, 2 non-finite, 3 |rho(f) - rho| / rho,
//   4 max_k |U_k(f) - U_k|, 5 |T(f) - T| / T, 6 rho, 7.. rho U (d), 7+d energy.
template <int D, int NC, typename Real>
__global__ __launch_bounds__(kThreads) void k_state_terms(int N, int NV, int nv, double vmax,
                                                           double omega, const void* fv,
                                                           const double* __restrict__ rho,
                                                           const double* __restrict__ U,
                                                           const double* __restrict__ T,
                                                           double* __restrict__ part) {
  __shared__ double sh[4 * (D + 1)];
  __shared__ double smin[4];
  extern __shared__ double vt[];
  const int i = blockIdx.x;
  const size_t NVs = NV, cs = static_cast<size_t>(N) * NVs;
  const Real* row = static_cast<const Real*>(fv) + static_cast<size_t>(i) * NVs;
  fill_vtab(vt, nv, vmax);
  __syncthreads();
  double r, u[3] = {0.0, 0.0, 0.0}, t;
  row_moments<D, NC, Real>(row, cs, NV, nv, vt, omega, sh, r, u, t);
  double mn = INFINITY, cnt[2] = {0.0, 0.0};
  for (int q = threadIdx.x; q < NV; q += kThreads) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double x = static_cast<double>(row[c * cs + q]);
      if (isfinite(x)) {
        mn = fmin(mn, x);
        if (x < 0.0) cnt[0] = cnt[0] + 1.0;
      } else {
        cnt[1] = cnt[1] + 1.0;
      }
    }
  }
  block_sum<2>(cnt, sh);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mn = fmin(mn, __shfl_xor(mn, o, 64));
  if ((threadIdx.x & 63) == 0) smin[threadIdx.x >> 6] = mn;
  __syncthreads();
  if (threadIdx.x == 0) {
    double* p = part + static_cast<size_t>(i) * kCheckTerms;
    const double ri = rho[i], Ti = T[i];
    double du = 0.0, u2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double Uk = U[static_cast<size_t>(k) * N + i];
      const double dk = fabs(u[k] - Uk);
      du = (dk > du || dk != dk) ? dk : du;
      u2 = u2 + Uk * Uk;
      p[7 + k] = ri * Uk;
    }
    p[0] = fmin(fmin(smin[0], smin[1]), fmin(smin[2], smin[3]));
    p[1] = cnt[0];
    p[2] = cnt[1];
    p[3] = fabs(r - ri) / ri;
    p[4] = du;
    p[5] = fabs(t - Ti) / Ti;
    p[6] = ri;
    p[7 + D] = 0.5 * ri * (u2 + 3.0 * Ti);
  }
}

// One block: slot 0 the minimum, slots 1, 2, 6.. the sums, slots 3-5 the
// maxima over the particles (NaN residuals propagate), each in a fixed order.
template <int D>
__global__ __launch_bounds__(kThreads) void k_state_reduce(int N, const double* __restrict__ part,
                                                            double* __restrict__ out) {
  constexpr int NS = 3 + D + 2;  // summed slots: 1, 2, 6 .. 7 + D
  __shared__ double sh[4 * NS];
  __shared__ double sx[4][4];
  double s[NS], mx[4] = {INFINITY, 0.0, 0.0, 0.0};  // min f, three maxima
#pragma unroll
  for (int k = 0; k < NS; ++k) s[k] = 0.0;
  for (int i = threadIdx.x; i < N; i += kThreads) {
    const double* p = part + static_cast<size_t>(i) * kCheckTerms;
    mx[0] = fmin(mx[0], p[0]);
    s[0] = s[0] + p[1];
    s[1] = s[1] + p[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) mx[1 + k] = (p[3 + k] > mx[1 + k] || p[3 + k] != p[3 + k]) ? p[3 + k] : mx[1 + k];
#pragma unroll
    for (int k = 0; k < D + 2; ++k) s[2 + k] = s[2 + k] + p[6 + k];
  }
  block_sum<NS>(s, sh);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mx[0] = fmin(mx[0], __shfl_xor(mx[0], o, 64));
#pragma unroll
    for (int k = 1; k < 4; ++k) {
      const double y = __shfl_xor(mx[k], o, 64);
      mx[k] = (y > mx[k] || y != y) ? y : mx[k];
    }
  }
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < 4; ++k) sx[threadIdx.x >> 6][k] = mx[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    double m[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) m[k] = sx[0][k];
    for (int w = 1; w < 4; ++w) {
      m[0] = fmin(m[0], sx[w][0]);
#pragma unroll
      for (int k = 1; k < 4; ++k) m[k] = (sx[w][k] > m[k] || sx[w][k] != sx[w][k]) ? sx[w][k] : m[k];
    }
    out[0] = m[0];
    out[1] = s[0];
    out[2] = s[1];
    out[3] = m[1];
    out[4] = m[2];
    out[5] = m[3];
#pragma unroll
    for (int k = 0; k < D + 2; ++k) out[6 + k] = s[2 + k];
    for (int k = 8 + D; k < kCheckTerms; ++k) out[k] = 0.0;
  }
}

hipError_t launch_state_check(const Ctx& c, const void* f, const double* rho, const double* U,
                              const double* T, double* out_dev) {
  const bool f64 = c.cfg.precision == BGK_FP64;
  const double om = omega_of(c.cfg);
  dim3 g(c.N), t(kThreads);
  const size_t lds = static_cast<size_t>(c.D + 1) * c.cfg.nv * sizeof(double);
  double* part = c.d.scheck;
  if (c.D == 2) {
    if (f64) hipLaunchKernelGGL((k_state_terms<2, 2, double>), g, t, lds, c.stream, c.N, c.NV, c.cfg.nv, c.cfg.vmax, om, f, rho, U, T, part);
    else hipLaunchKernelGGL((k_state_terms<2, 2, float>), g, t, lds, c.stream, c.N, c.NV, c.cfg.nv, c.cfg.vmax, om, f, rho, U, T, part);
    hipLaunchKernelGGL(k_state_reduce<2>, dim3(1), t, 0, c.stream, c.N, part, out_dev);
  } else {
    if (f64) hipLaunchKernelGGL((k_state_terms<3, 1, double>), g, t, lds, c.stream, c.N, c.NV, c.cfg.nv, c.cfg.vmax, om, f, rho, U, T, part);
    else hipLaunchKernelGGL((k_state_terms<3, 1, float>), g, t, lds, c.stream, c.N, c.NV, c.cfg.nv, c.cfg.vmax, om, f, rho, U, T, part);
    hipLaunchKernelGGL(k_state_reduce<3>, dim3(1), t, 0, c.stream, c.N, part, out_dev);
  }
  return hipGetLastError();
}

template <int D, int NC, typename Real>
__global__ __launch_bounds__(kThreads) void k_maxwellian(int N, int NV, int nv, double vmax,
                                                          const double* __restrict__ rho,
                                                          const double* __restrict__ U,
                                                          const double* __restrict__ T, void* fv) {
  extern __shared__ double vt[];
  const int i = blockIdx.x;
  const size_t NVs = NV, cs = static_cast<size_t>(N) * NVs;
  Real* row = static_cast<Real*>(fv) + static_cast<size_t>(i) * NVs;
  double u[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < D; ++k) u[k] = U[static_cast<size_t>(k) * N + i];
  const double r = rho[i], t = T[i];
  fill_vtab(vt, nv, vmax);
  __syncthreads();
  double* et = vt + nv;
  fill_etab<D>(et, vt, nv, u, t);
  __syncthreads();
  const double norm = maxwell_norm<D>(r, t);
  VelDigits<D> vd;
  vd.init(threadIdx.x, kThreads, nv);
  for (int q = threadIdx.x; q < NV; q += kThreads, vd.advance(nv)) {
    const int* kq = vd.k;
    double M = norm;
#pragma unroll
    for (int k = 0; k < D; ++k) M = M * et[k * nv + kq[k]];
#pragma unroll
    for (int c = 0; c < NC; ++c) row[c * cs + q] = static_cast<Real>(c == 0 ? M : t * M);
  }
}

hipError_t launch_maxwellian(const Ctx& c, const double* rho, const double* U, const double* T,
                             void* f) {
  const bool f64 = c.cfg.precision == BGK_FP64;
  dim3 g(c.N), t(kThreads);
  const size_t lds = static_cast<size_t>(c.D + 1) * c.cfg.nv * sizeof(double);
  if (c.D == 2) {
    if (f64) hipLaunchKernelGGL((k_maxwellian<2, 2, double>), g, t, lds, c.stream, c.N, c.NV, c.cfg.nv, c.cfg.vmax, rho, U, T, f);
    else hipLaunchKernelGGL((k_maxwellian<2, 2, float>), g, t, lds, c.stream, c.N, c.NV, c.cfg.nv, c.cfg.vmax, rho, U, T, f);
  } else {
    if (f64) hipLaunchKernelGGL((k_maxwellian<3, 1, double>), g, t, lds, c.stream, c.N, c.NV, c.cfg.nv, c.cfg.vmax, rho, U, T, f);
    else hipLaunchKernelGGL((k_maxwellian<3, 1, float>), g, t, lds, c.stream, c.N, c.NV, c.cfg.nv, c.cfg.vmax, rho, U, T, f);
  }
  return hipGetLastError();
}

}  // namespace bgk
