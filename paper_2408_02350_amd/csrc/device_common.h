// Device helpers shared by the libbgk kernels (gfx950, wave64).
// The library is compiled with -ffp-contract=off: every fused multiply-add
// in these kernels is written out explicitly with fma(), so that the
// geometry predicates and the least-squares arithmetic follow the plain
// operation order of the method.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bgk_internal.h"

namespace bgk {

constexpr double kPi = 3.14159265358979323846;

// Velocity node k of an axis with nv points on [-vmax, vmax], both ends
// included (Sec. 3.3): v_k = vmax (2k - (nv-1)) / (nv-1).
__device__ __forceinline__ double vnode(int k, int nv, double vmax) {
  return vmax * static_cast<double>(2 * k - (nv - 1)) / static_cast<double>(nv - 1);
}

template <int D>
__device__ __forceinline__ void velocity_of(int q, int nv, double vmax, double v[3]) {
  v[0] = v[1] = v[2] = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    v[a] = vnode(q % nv, nv, vmax);
    q /= nv;
  }
}

// Maxwellian of Sec. 2 (eq. maxwellian, exponent -|v-U|^2/(2T), R = 1) for
// D = 3; for D = 2 the Chu-reduced G1 = rho/(2 pi T) exp(-|v-U|^2/(2T)) and
// G2 = T G1 (Sec. 2.1).  comp selects G1 (0) or G2 (1).
template <int D>
__device__ __forceinline__ double maxwell(int comp, double rho, const double* U, double T,
                                          const double* v) {
  double s2 = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const double wa = v[a] - U[a];
    s2 = s2 + wa * wa;
  }
  const double two_pi = 2.0 * kPi;
  double norm;
  if (D == 3) {
    const double tp = two_pi * T;
    norm = rho / (tp * sqrt(tp));
  } else {
    norm = rho / (two_pi * T);
  }
  double g = norm * exp(-s2 / (2.0 * T));
  if (comp == 1) g = T * g;
  return g;
}

// Base-nv digits of a velocity index (fastest axis first), advanced by a
// fixed stride without integer division: a thread walking q = q0 + m stride
// takes the stride's digits once and adds them with carries.
template <int D>
struct VelDigits {
  int k[D], st[D];
  __device__ void init(int q, int stride, int nv) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      k[a] = q % nv;
      q /= nv;
      st[a] = stride % nv;
      stride /= nv;
    }
  }
  __device__ void advance(int nv) {  // (the carry out of the last digit is
    int carry = 0;                   //  past N_v: the loops end there)
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int x = k[a] + st[a] + carry;
      carry = x >= nv;
      k[a] = carry ? x - nv : x;
    }
  }
};

// Sum K doubles over a block of kThreads (= 4 waves of 64) in a fixed order;
// every thread receives the totals.  sh must hold 4*K doubles.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* sh) {
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
  for (int k = 0; k < K; ++k) v[k] = ((sh[k] + sh[K + k]) + sh[2 * K + k]) + sh[3 * K + k];
  __syncthreads();
}

// R elements of a row at a stride of zsb bytes (the lane's byte offset of the
// first in lane_off; the element offsets in scalar registers).  Lanes with
// consecutive offsets read one contiguous piece per element.
template <typename Real, int R>
__device__ __forceinline__ void load_rz(const Real* row, uint32_t lane_off, uint32_t zsb,
                                        Real (&o)[R]) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<Real*>(row), 0, 0x7fffffff, 0x00020000);
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if constexpr (sizeof(Real) == 8)
      o[r] = __builtin_bit_cast(Real, __builtin_amdgcn_raw_buffer_load_b64(rs, lane_off, r * zsb, 0));
    else
      o[r] = __builtin_bit_cast(Real, __builtin_amdgcn_raw_buffer_load_b32(rs, lane_off, r * zsb, 0));
  }
}

template <typename Real, int R>
__device__ __forceinline__ void store_rz(Real* row, uint32_t lane_off, uint32_t zsb,
                                         const Real (&o)[R]) {
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(row, 0, 0x7fffffff, 0x00020000);
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if constexpr (sizeof(Real) == 8)
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, o[r]), rs, lane_off, r * zsb, 0);
    else
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, o[r]), rs, lane_off,
                                            r * zsb, 0);
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Map the hardware block id to a logical id so that each XCD works on
// one contiguous range of logical blocks (neighbouring patches share f rows).
__device__ __forceinline__ int xcd_logical_block(int b, int n) {
  const int x = b & 7, local = b >> 3;
  const int q = n >> 3, r = n & 7;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + local;
}

__device__ __forceinline__ void raise_error(int32_t* err, int code) {
  atomicOr(&err[0], err_bit(code));
}

// Cell coordinate of a position component in [0, 1] with nca cells per axis
// (NaN and values outside the box land in the boundary cells).
__device__ __forceinline__ int cell_coord(double xa, int nca) {
  const double s = xa * static_cast<double>(nca);
  return (s >= 0.0) ? (s < static_cast<double>(nca) ? static_cast<int>(s) : nca - 1) : 0;
}

}  // namespace bgk
