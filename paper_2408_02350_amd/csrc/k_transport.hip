// S4: explicit transport with the positive upwind flux (Sec. 3.2.1 eq.
// explicit; Sec. 3.4.2 eq. flux and its 3D form):
//
//   ft_i(v) = f_i(v) - dt sum_{j != i} c_ij(v) (f_j(v) - f_i(v)),
//   c_ij(v) = g.w - |P.w| - |Q.w| - |R.w| = 2 sum_k min(0, a_k.w),
//   w = v - U_i,  a_k in {P, Q, R}  (g = P + Q + R).
//
// Work decomposition: lanes run over velocities (f is [n_c][N][N_v] with the
// velocity contiguous, so every f_j load of a wavefront is one coalesced
// segment).  A block owns a patch of tp interior particles that are
// neighbours in the cell order and a tile of 256*R velocities; it walks the
// sorted union of the patch's neighbour lists once, so each f_j row segment
// is loaded once and applied to every patch particle that has j as a
// neighbour.  The per-edge vectors (P, Q, R) are wave-uniform and come in
// through the scalar cache.  Accumulation order per particle is its
// neighbour list order (ascending j), independent of the patch layout.
#include "device_common.h"

namespace bgk {

template <int MODE>
struct PrecT;
template <>
struct PrecT<BGK_FP64> {
  using real = double;
};
template <>
struct PrecT<BGK_FP32> {
  using real = float;
};
template <>
struct PrecT<BGK_BF16> {
  using real = float;
};

struct TransportArgs {
  int N, NV, nv, cap, Ni, npatch, ucap;
  double vmax, dt;
  const void* f;
  void* ft;
  const double* U;
  const void* ops;  // [N][cap][D*D] in the transport precision
  const int32_t* plist;
  const int32_t* ucount;
  const int32_t* uj;
  const uint32_t* ue;
};

__device__ __forceinline__ double fma_r(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fma_r(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double min0(double a) { return fmin(a, 0.0); }
__device__ __forceinline__ float min0(float a) { return fminf(a, 0.0f); }

// Round an FP32 value to BF16 (nearest even) and back.
__device__ __forceinline__ float bf16_round(float x) {
  return static_cast<float>(static_cast<__bf16>(x));
}

template <int D, int NC, int MODE, int R, int TP>
__global__ __launch_bounds__(kThreads) void k_transport(const TransportArgs a) {
  using Real = typename PrecT<MODE>::real;
  constexpr int DD = D * D;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const int patch = lb % a.npatch, tile = lb / a.npatch;
  const Real* __restrict__ f = static_cast<const Real*>(a.f);
  Real* __restrict__ ft = static_cast<Real*>(a.ft);
  const Real* __restrict__ ops = static_cast<const Real*>(a.ops);
  const size_t NVs = static_cast<size_t>(a.NV);
  const size_t cstride = static_cast<size_t>(a.N) * NVs;

  int pt[TP];
#pragma unroll
  for (int t = 0; t < TP; ++t) {
    const int g = patch * TP + t;
    pt[t] = g < a.Ni ? a.plist[g] : -1;
  }

  int q[R];
  bool ok[R];
  Real v[R][D];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    q[r] = tile * (kThreads * R) + r * kThreads + static_cast<int>(threadIdx.x);
    ok[r] = q[r] < a.NV;
    double vv[3];
    velocity_of<D>(ok[r] ? q[r] : 0, a.nv, a.vmax, vv);
#pragma unroll
    for (int k = 0; k < D; ++k) v[r][k] = static_cast<Real>(vv[k]);
  }

  Real fi[TP][R][NC], acc[TP][R][NC];
#pragma unroll
  for (int t = 0; t < TP; ++t)
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        fi[t][r][c] = (pt[t] >= 0 && ok[r])
                          ? f[c * cstride + static_cast<size_t>(pt[t]) * NVs + q[r]]
                          : Real(0);
        acc[t][r][c] = Real(0);
      }

  Real Ut[TP][D];
#pragma unroll
  for (int t = 0; t < TP; ++t)
#pragma unroll
    for (int k = 0; k < D; ++k)
      Ut[t][k] = pt[t] >= 0 ? static_cast<Real>(a.U[static_cast<size_t>(k) * a.N + pt[t]])
                            : Real(0);

  const int nu = a.ucount[patch];
  const int32_t* __restrict__ ujp = a.uj + static_cast<size_t>(patch) * a.ucap;
  const uint32_t* __restrict__ uep = a.ue + static_cast<size_t>(patch) * a.ucap;
  for (int u = 0; u < nu; ++u) {
    const int j = ujp[u];
    const uint32_t pe = uep[u];
    Real fj[R][NC];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < NC; ++c)
        fj[r][c] = ok[r] ? f[c * cstride + static_cast<size_t>(j) * NVs + q[r]] : Real(0);
#pragma unroll
    for (int t = 0; t < TP; ++t) {
      const uint32_t e = (pe >> (8 * t)) & 0xFFu;
      if (e != 0xFFu) {
        const Real* o = ops + (static_cast<size_t>(pt[t]) * a.cap + e) * DD;
        Real av[DD];
#pragma unroll
        for (int k = 0; k < DD; ++k) av[k] = o[k];
        Real bk[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
          Real s = av[k * D] * Ut[t][0];
#pragma unroll
          for (int m = 1; m < D; ++m) s = fma_r(av[k * D + m], Ut[t][m], s);
          bk[k] = s;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          Real cm = Real(0);
#pragma unroll
          for (int k = 0; k < D; ++k) {
            Real pk = -bk[k];
#pragma unroll
            for (int m = 0; m < D; ++m) pk = fma_r(av[k * D + m], v[r][m], pk);
            cm = cm + min0(pk);
          }
          const Real cval = cm + cm;
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const Real df = fj[r][c] - fi[t][r][c];
            if constexpr (MODE == BGK_BF16)
              acc[t][r][c] = fma_r(bf16_round(cval), bf16_round(df), acc[t][r][c]);
            else
              acc[t][r][c] = fma_r(cval, df, acc[t][r][c]);
          }
        }
      }
    }
  }

  const Real dt = static_cast<Real>(a.dt);
#pragma unroll
  for (int t = 0; t < TP; ++t)
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (pt[t] >= 0 && ok[r])
          ft[c * cstride + static_cast<size_t>(pt[t]) * NVs + q[r]] =
              fi[t][r][c] - dt * acc[t][r][c];
}

template <int D, int NC, int MODE, int TP>
static hipError_t launch_transport_t(const Ctx& c, const TransportArgs& a) {
  const int R = (c.NV >= 2 * kThreads) ? 2 : 1;
  const int ntile = (c.NV + kThreads * R - 1) / (kThreads * R);
  const int64_t nblocks = static_cast<int64_t>(c.npatch) * ntile;
  if (nblocks == 0) return hipSuccess;
  if (nblocks > INT32_MAX) return hipErrorInvalidValue;
  if (R == 2)
    hipLaunchKernelGGL((k_transport<D, NC, MODE, 2, TP>), dim3(static_cast<unsigned>(nblocks)),
                       dim3(kThreads), 0, c.stream, a);
  else
    hipLaunchKernelGGL((k_transport<D, NC, MODE, 1, TP>), dim3(static_cast<unsigned>(nblocks)),
                       dim3(kThreads), 0, c.stream, a);
  return hipGetLastError();
}

hipError_t launch_transport(const Ctx& c, const void* f_in, void* f_out, const double* U) {
  const int mode = c.cfg.precision;
  TransportArgs a{c.N,      c.NV,  c.cfg.nv, c.cap,   c.Ni,     c.npatch,  c.ucap,
                  c.cfg.vmax, c.cfg.dt, f_in,  f_out, U,
                  mode == BGK_FP64 ? static_cast<const void*>(c.d.ops64)
                                   : static_cast<const void*>(c.d.ops32),
                  c.d.cperm, c.d.ucount, c.d.uj, c.d.ue};
  if (c.D == 2) {
    if (mode == BGK_FP64)
      return c.tp == 2 ? launch_transport_t<2, 2, BGK_FP64, 2>(c, a)
                       : launch_transport_t<2, 2, BGK_FP64, 4>(c, a);
    if (mode == BGK_FP32) return launch_transport_t<2, 2, BGK_FP32, 4>(c, a);
    return launch_transport_t<2, 2, BGK_BF16, 4>(c, a);
  }
  if (mode == BGK_FP64) return launch_transport_t<3, 1, BGK_FP64, 4>(c, a);
  if (mode == BGK_FP32) return launch_transport_t<3, 1, BGK_FP32, 4>(c, a);
  return launch_transport_t<3, 1, BGK_BF16, 4>(c, a);
}

// Wall rows of the transported field are copies of the input (the staged
// transport call only; the full step overwrites them in S7).
template <typename Real>
__global__ void k_copy_wall_rows(int N, int NV, int NC, const int32_t* __restrict__ wall_list,
                                 const Real* __restrict__ src, Real* __restrict__ dst) {
  const int b = wall_list[blockIdx.x];
  const size_t cs = static_cast<size_t>(N) * NV;
  for (int c = 0; c < NC; ++c)
    for (int q = threadIdx.x; q < NV; q += blockDim.x)
      dst[c * cs + static_cast<size_t>(b) * NV + q] = src[c * cs + static_cast<size_t>(b) * NV + q];
}

hipError_t launch_copy_wall_rows(const Ctx& c, const void* f_in, void* f_out) {
  if (c.Nw == 0) return hipSuccess;
  if (c.cfg.precision == BGK_FP64)
    hipLaunchKernelGGL(k_copy_wall_rows<double>, dim3(c.Nw), dim3(kThreads), 0, c.stream, c.N,
                       c.NV, c.NC, c.d.wall_list, static_cast<const double*>(f_in),
                       static_cast<double*>(f_out));
  else
    hipLaunchKernelGGL(k_copy_wall_rows<float>, dim3(c.Nw), dim3(kThreads), 0, c.stream, c.N,
                       c.NV, c.NC, c.d.wall_list, static_cast<const float*>(f_in),
                       static_cast<float*>(f_out));
  return hipGetLastError();
}

}  // namespace bgk
