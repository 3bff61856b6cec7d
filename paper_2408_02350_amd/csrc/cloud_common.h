// Device helpers shared by the geometry kernels and the particle
// management: the cell list order, candidate ranges of the cells around a
// point, wave-wide compaction and rank sort, the least-squares solve on one
// wave, and the degree-1 value row at a point (boundary interpolation rows
// and new particles).
#pragma once

#include "device_common.h"

namespace bgk {

// Order of the cells.  The first d-1 axes are cut into tiles of
// kCellTile<D> cells (strips in 2D, columns in 3D) and each tile is swept
// along the last axis, x fastest inside the tile.  Interior particles are
// processed in this order in patches of tp, and each XCD takes one
// contiguous range of patches; sweeping a narrow tile brings a neighbour row
// back within a few patches, while it is still in the XCD's L2 (a plain
// row-major order returns to it only one full row of cells later).
template <int D>
struct CellTile;
template <>
struct CellTile<2> {
  static constexpr int S = 12;
};
template <>
struct CellTile<3> {
  static constexpr int S = 4;
};

// Key of cell (cc[0], .., cc[D-1]), 0 <= cc < nca: a bijection onto
// [0, nca^D) that lists the tiles in order (last tile of an axis narrower
// when S does not divide nca).
template <int D>
__device__ __forceinline__ int cell_key(const int* cc, int nca) {
  constexpr int S = CellTile<D>::S;
  const int x0 = (cc[0] / S) * S, wx = min(S, nca - x0);
  if constexpr (D == 2) {
    return x0 * nca + cc[1] * wx + (cc[0] - x0);
  } else {
    const int y0 = (cc[1] / S) * S, wy = min(S, nca - y0);
    return nca * (y0 * nca + x0 * wy) + cc[2] * (wx * wy) + (cc[1] - y0) * wx + (cc[0] - x0);
  }
}

// ------------------------------------------------------------ wave helpers
// The kernels below run one wavefront (a block of 64 threads) per particle,
// patch or wall particle; lanes work on candidates / neighbours in parallel.
constexpr int kWave = 64;

__device__ __forceinline__ int lanes_below(uint64_t mask) {
  const int lane = threadIdx.x & 63;
  return __popcll(mask & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
}

// Ranges of the cells within +-S cells of cell coordinate ci (only the
// interior part when walls == false).  Writes range starts rb[] and the
// exclusive prefix of their lengths rpre[] (rpre[nr] = total) to LDS and
// returns nr.  Must be called by all 64 lanes.
template <int D, int S>
__device__ int cell_ranges(const int* ci, int nca, int ncell, bool walls,
                           const int32_t* __restrict__ cstart, int32_t* rb, int32_t* rpre) {
  constexpr int W = 2 * S + 1;
  constexpr int NC = (D == 2) ? W * W : W * W * W;
  const int parts = walls ? 2 : 1;
  const int nr = NC * parts;
  const int lane = threadIdx.x;
  int carry = 0;
  for (int r0 = 0; r0 < nr; r0 += kWave) {
    const int r = r0 + lane;
    int len = 0, b = 0;
    if (r < nr) {
      const int part = r % parts, co = r / parts;
      int cc[D], rem = co;
      bool ok = true;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        cc[a] = ci[a] + (rem % W) - S;
        rem /= W;
        ok = ok && cc[a] >= 0 && cc[a] < nca;
      }
      if (ok) {
        const int k = cell_key<D>(cc, nca) + part * ncell;
        b = cstart[k];
        len = cstart[k + 1] - b;
      }
    }
    int incl = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o, 64);
      if (lane >= o) incl += t;
    }
    if (r < nr) {
      rb[r] = b;
      rpre[r] = carry + incl - len;
    }
    carry += __shfl(incl, 63, 64);
  }
  if (lane == 0) rpre[nr] = carry;
  __syncthreads();
  return nr;
}

// Candidate c (0 <= c < rpre[nr]) -> its slot in the cell-ordered arrays.
__device__ __forceinline__ int cand_slot(int c, int nr, const int32_t* rb, const int32_t* rpre) {
  int lo = 0, hi = nr;  // rpre[lo] <= c < rpre[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (rpre[mid] <= c) lo = mid; else hi = mid;
  }
  return rb[lo] + (c - rpre[lo]);
}

// Write the n values of list[] to row[] in ascending order (rank sort; the
// values are distinct particle indices); only ranks < cap are written.
__device__ __forceinline__ void rank_sorted_store(const int32_t* list, int n, int cap,
                                                  int32_t* __restrict__ row) {
  for (int s = threadIdx.x; s < n; s += kWave) {
    const int v = list[s];
    int rank = 0;
    for (int q = 0; q < n; ++q) rank += (list[q] < v);
    if (rank < cap) row[rank] = v;
  }
}

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

// Weighted least squares on one wave, for the stencil already staged in LDS
// as P[e][B] (basis values) and W[e] (weights), e < m.  Builds
// A = sum_e W_e p_e p_e^T (each entry summed over e in order), factors it
// A = L L^T (Cholesky, column by column, the rows of a column in parallel),
// and solves L L^T z = e_col for the NCOL columns col0 .. col0+NCOL-1 into
// Z[k][B].  Returns false on a non-positive pivot.  All 64 lanes call it.
template <int B, int NCOL>
__device__ bool wave_lsq(int m, const double* P, const double* W, double* A, double* Z, int col0,
                         int* flag) {
  constexpr int NT = B * (B + 1) / 2;
  const int lane = threadIdx.x;
  for (int l = lane; l < NT; l += kWave) {
    int r = 0;
    while (tri(r + 1, 0) <= l) ++r;
    const int s = l - tri(r, 0);
    double acc = 0.0;
    for (int e = 0; e < m; ++e) acc = acc + (W[e] * P[e * B + r]) * P[e * B + s];
    A[l] = acc;
  }
  if (lane == 0) *flag = 0;
  __syncthreads();
  for (int j = 0; j < B; ++j) {
    if (lane == 0) {
      double s = A[tri(j, j)];
      for (int k = 0; k < j; ++k) s = s - A[tri(j, k)] * A[tri(j, k)];
      if (!(s > 0.0)) *flag = 1;
      A[tri(j, j)] = sqrt(s);
    }
    __syncthreads();
    if (*flag) return false;
    if (lane > j && lane < B) {
      double t = A[tri(lane, j)];
      for (int k = 0; k < j; ++k) t = t - A[tri(lane, k)] * A[tri(j, k)];
      A[tri(lane, j)] = t / A[tri(j, j)];
    }
    __syncthreads();
  }
  if (lane < NCOL) {
    const int col = col0 + lane;
    double y[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
      double s = (i == col) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < i; ++k) s = s - A[tri(i, k)] * y[k];
      y[i] = s / A[tri(i, i)];
    }
    double* z = Z + lane * B;
#pragma unroll
    for (int i = B - 1; i >= 0; --i) {
      double s = y[i];
#pragma unroll
      for (int k = i + 1; k < B; ++k) s = s - A[tri(k, i)] * z[k];
      z[i] = s / A[tri(i, i)];
    }
  }
  __syncthreads();
  return true;
}

// ------------------------------------------------------------ value rows
// The particle cloud as the geometry kernels see it: positions (and their
// cell-ordered copy xs), the cell list (cells of size 1/nca >= h, interior
// keys first, then wall keys), the support radius and the weight exponent.
struct CloudView {
  int N, cap, nca, ncell;
  double h, alpha;
  const double* x;
  const double* xs;
  const int32_t* cstart;
  const int32_t* cperm;
};

template <int D>
struct ValueRowSm {
  static constexpr int NR = (D == 2 ? 25 : 125), B = D + 1;
  int32_t rb[NR], rpre[NR + 1];
  int32_t sel[256], srt[256];  // cap <= 255
  double P[256 * B], W[256], A[B * (B + 1) / 2], Z[B];
  int flag;
};

// Value row at the point xq (one wave, all 64 lanes): the interior
// particles within hb, ascending in sm.srt[0..m), and their degree-1
// least-squares value weights at xq (weights exp(-alpha r^2/hb^2)),
// value_weight(sm, e).  hb is the first of h, 1.5h, 2h whose set holds at
// least d+2 particles, gives a positive-definite fit and keeps the
// extrapolation's amplification sum_e |c0_e| at most kValueRowAmp; the 2h
// row is taken without the bound.  (The bound is above the amplification of
// every row of the jittered initial lattices, 3.7 in 2D and 6.6 in 3D: it
// acts only where a moving cloud has left a near-degenerate stencil, whose
// extrapolation would otherwise amplify ~100-fold and drive the step
// non-physical.)  Candidates are the interior ranges of the cells within
// +-1 cell for h and within +-2 cells for the wider radii.  Returns m, or
// -1 (fewer than d+2 points or a non-positive pivot at 2h: BGK_ESINGULAR)
// or -2 (more than cap points: BGK_ENBR_OVERFLOW).
constexpr double kValueRowAmp = 8.0;

template <int D>
__device__ __forceinline__ double value_weight(const ValueRowSm<D>& sm, int e);

template <int D>
__device__ int value_row(const CloudView& a, const double* xq, ValueRowSm<D>& sm, double& hb) {
  constexpr int B = D + 1;
  const int lane = threadIdx.x;
  int cb[D];
#pragma unroll
  for (int q = 0; q < D; ++q) cb[q] = cell_coord(xq[q], a.nca);
  // cells are at least h wide: the first radius needs the 3^D cells around
  // xq, the wider ones the 5^D
  int nr = cell_ranges<D, 1>(cb, a.nca, a.ncell, false, a.cstart, sm.rb, sm.rpre);
  int total = sm.rpre[nr];
  const double mults[3] = {1.0, 1.5, 2.0};
  for (int t = 0; t < 3; ++t) {
    const bool last = t == 2;
    if (t == 1) {
      __syncthreads();
      nr = cell_ranges<D, 2>(cb, a.nca, a.ncell, false, a.cstart, sm.rb, sm.rpre);
      total = sm.rpre[nr];
    }
    hb = mults[t] * a.h;
    const double hb2 = hb * hb;
    int m = 0;
    for (int c0 = 0; c0 < total; c0 += kWave) {
      const int cidx = c0 + lane;
      bool in = false;
      int j = 0;
      if (cidx < total) {
        const int p = cand_slot(cidx, nr, sm.rb, sm.rpre);
        j = a.cperm[p];
        double r2 = 0.0;
#pragma unroll
        for (int q = 0; q < D; ++q) {
          const double dl = a.xs[static_cast<int64_t>(q) * a.N + p] - xq[q];
          r2 = r2 + dl * dl;
        }
        in = r2 <= hb2;
      }
      const uint64_t mask = __ballot(in);
      const int pos = m + lanes_below(mask);
      if (in && pos < 256) sm.sel[pos] = j;
      m += __popcll(mask);
    }
    __syncthreads();
    if (m < D + 2) {
      if (last) return -1;
      continue;
    }
    if (m > a.cap) return -2;
    rank_sorted_store(sm.sel, m, a.cap, sm.srt);
    __syncthreads();
    for (int e = lane; e < m; e += kWave) {
      const int j = sm.srt[e];
      double y[D], r2 = 0.0;
#pragma unroll
      for (int q = 0; q < D; ++q) {
        y[q] = (a.x[static_cast<int64_t>(q) * a.N + j] - xq[q]) / hb;
        r2 = r2 + y[q] * y[q];
      }
      sm.W[e] = exp(-a.alpha * r2);
      Basis<D, 1>::eval(y, sm.P + e * B);
    }
    __syncthreads();
    if (!wave_lsq<B, 1>(m, sm.P, sm.W, sm.A, sm.Z, 0, &sm.flag)) {
      if (last) return -1;
      __syncthreads();
      continue;
    }
    if (last) return m;
    // amplification of the row: every lane ends with the same sum
    double amp = 0.0;
    for (int e = lane; e < m; e += kWave) amp = amp + fabs(value_weight(sm, e));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) amp = amp + __shfl_xor(amp, o, kWave);
    if (amp <= kValueRowAmp) return m;
    __syncthreads();   // the next radius reuses the staging arrays
  }
  return -1;
}

template <int D>
__device__ __forceinline__ double value_weight(const ValueRowSm<D>& sm, int e) {
  constexpr int B = D + 1;
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < B; ++r) s = s + sm.Z[r] * sm.P[e * B + r];
  return sm.W[e] * s;
}

}  // namespace bgk
