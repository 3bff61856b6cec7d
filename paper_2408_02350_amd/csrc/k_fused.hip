// S4 + S5 + S6 fused: transport, moments and implicit relaxation of a patch
// of tp interior particles over ALL velocities in one block.
//
//   ft_i(v) = f_i(v) - dt sum_{j != i} c_ij(v) (f_j(v) - f_i(v)),
//   c_ij(v) = 2 sum_k min(0, a_k.(v - U_i)),  a_k in {P, Q[, R]}     (S4)
//   rho, U, T of ft in FP64                                           (S5)
//   f_i^{n+1} = (tau ft_i + dt M[rho, U, T]) / (tau + dt)             (S6)
//
// Layout of the work: a block owns one patch; thread tid handles R
// velocities q = q0 + r zs (r < R, R divides nv) that differ only in one
// velocity component, the stepping axis: each projection a_k.(v - U) is
// formed once and then advanced by a constant per r (one add).  In 2D the
// stepping axis is the fastest one, x (zs = 1: every row access of a thread
// is one contiguous R-element vector load or store).  In 3D it is z (zs =
// nv^2): the third frame vector has no z component, so its projection is
// the same for all R velocities and is formed once per edge; a row access
// is then R loads, each contiguous across the lanes of a wave.
// The block walks the sorted union of its particles' neighbour lists in
// chunks of one wave width: every wave holds the chunk's row indices and
// slot masks one per lane (read back with readlane, no LDS round trip on
// the row-load path), the per-edge data (a_k, a_k.U_i and the per-r
// increments) is staged in LDS and read back with wave-uniform addresses,
// and the f_j rows are loaded three union entries ahead (two for FP64 in
// 3D).
//
// The walk accumulates A = sum_j c_ij f_j (per component) and C = sum_j c_ij
// (shared by the components), so f_i is not needed until the end:
// ft = f_i (1 + dt C) - dt A.  (In the BF16-operand mode the products are
// taken of the differences f_j - f_i instead, which keeps the BF16 rounding
// proportional to the differences.)  After the walk ft stays in registers:
// the moments are summed in two passes (U first, then the centred second
// moment), each reduced in a fixed order (a wavefront reduce-scatter, then
// the waves in order), the Maxwellian is the product of
// per-axis exponentials (d*nv exp per particle instead of N_v), and f^{n+1}
// is written once.
//
// When N_v does not fit one block at the register budget of the precision
// (large 3D grids in FP64) the velocity range is split into tiles over
// several blocks; the kernel then writes f-tilde and the separate
// relaxation kernel finishes the step.
#include "device_common.h"

namespace bgk {

template <int MODE>
struct FPrec;
template <>
struct FPrec<BGK_FP64> {
  using real = double;
};
template <>
struct FPrec<BGK_FP32> {
  using real = float;
};
template <>
struct FPrec<BGK_BF16> {
  using real = float;
};

constexpr int kChunk = 64;   // union entries staged per LDS chunk
constexpr int kMaxNv = 64;   // velocity points per axis supported by the fused path

struct FusedArgs {
  int N, NV, nv, cap, Ni, npatch, ucap, bte;  // bte: velocity lanes per block
  double vmax, dt, kn, omega, dvs;  // dvs: velocity step between r and r+1 (stepping axis)
  const void* f;
  void* fo;          // f-tilde (unfused) or f^{n+1} (fused)
  const double* U;   // U^n
  const void* ops;   // [N][cap][D*D] in the transport precision
  const int32_t* plist;
  const int32_t* ucount;
  const int32_t* uj;
  const uint32_t* ue;
  double* rho;       // fused: new moments of the patch particles
  double* Unew;
  double* T;
  int32_t* err;
  void* fto;         // fused: f-tilde's interior rows as well (may be null)
  int ntl;           // velocity tiles walked in turn by one block (INLDS)
};

__device__ __forceinline__ double fma_t(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double min_t(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float min_t(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double abs_t(double a) { return fabs(a); }
__device__ __forceinline__ float abs_t(float a) { return fabsf(a); }
__device__ __forceinline__ float bf16r(float x) { return static_cast<float>(static_cast<__bf16>(x)); }
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
// (x, y) rounded to a BF16 pair (round to nearest even, one instruction)
__device__ __forceinline__ bf16x2 bf16_pair(float x, float y) {
  return bf16x2{static_cast<__bf16>(x), static_cast<__bf16>(y)};
}

// R consecutive elements from / to p with the widest aligned vector
// accesses R * sizeof(Real) allows (p is aligned to that vector: R*tid
// offsets into rows whose length is a multiple of 4 elements).
template <typename Real, int R>
__device__ __forceinline__ void load_r(const Real* __restrict__ p, Real (&o)[R]) {
  constexpr int B = R * static_cast<int>(sizeof(Real));
  constexpr int W = (B % 16 == 0) ? 16 / static_cast<int>(sizeof(Real))
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
// R consecutive elements of a row through a buffer resource: the row base
// is wave-uniform (scalar registers), the lane's byte offset a 32-bit
// vector register, so no per-load 64-bit address arithmetic.  Needs
// R * sizeof(Real) to be a multiple of 16 bytes.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <typename Real, int R>
__device__ __forceinline__ void load_rb(const Real* row, uint32_t lane_off, Real (&o)[R]) {
  constexpr int B = R * static_cast<int>(sizeof(Real));
  static_assert(B % 16 == 0, "buffer row loads take 16-byte pieces");
  constexpr int W = 16 / static_cast<int>(sizeof(Real));
  typedef Real V __attribute__((ext_vector_type(W)));
  // raw buffer of the row: stride 0, byte count beyond any row, and the
  // descriptor format word of the gfx9 family
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<Real*>(row), 0, 0x7fffffff, 0x00020000);
#pragma unroll
  for (int i = 0; i < B / 16; ++i) {
    const V x = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(rs, lane_off + 16 * i, 0, 0));
#pragma unroll
    for (int w = 0; w < W; ++w) o[i * W + w] = x[w];
  }
}

template <typename Real, int R>
__device__ __forceinline__ void store_r(Real* __restrict__ p, const Real (&o)[R]) {
  constexpr int B = R * static_cast<int>(sizeof(Real));
  constexpr int W = (B % 16 == 0) ? 16 / static_cast<int>(sizeof(Real))
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

// Sum K per-lane values (K a power of two, K <= 64) over the wavefront by
// recursive halving: after the step with offset o every lane keeps half of
// its values (the half selected by lane bit o) plus its partner's copy of
// that half.  On return the lane holds the total of value
// k = (lane / (64 / K)) % K.  The summation order is fixed.
template <int K, int N, int O>
__device__ __forceinline__ void halve_step(double (&v)[K], int lane) {
  if constexpr (N > 1) {
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
      const double send = up ? v[i] : v[i + N / 2];
      const double keep = up ? v[i + N / 2] : v[i];
      v[i] = keep + __shfl_xor(send, O, 64);
    }
    halve_step<K, N / 2, O / 2>(v, lane);
  }
}

template <int K>
__device__ __forceinline__ double wave_reduce_scatter(double (&v)[K]) {
  const int lane = threadIdx.x & 63;
  halve_step<K, K, 32>(v, lane);
  double x = v[0];
#pragma unroll
  for (int o = 32 / K; o > 0; o >>= 1) x = x + __shfl_xor(x, o, 64);
  return x;
}

constexpr int pow2_at_least(int n) { return n <= 1 ? 1 : 2 * pow2_at_least((n + 1) / 2); }

// INLDS: the block walks all ntl velocity tiles of its patch in turn; the
// f-tilde of every tile but the last waits in LDS (thread-private slots, no
// barrier), so the moments and the relaxation run in the same block and
// f-tilde never goes to HBM.
template <int D, int NC, int MODE, int R, bool FUSE, int TP, bool INLDS>
__global__ __launch_bounds__(1024) void k_fused(const FusedArgs a) {
  using Real = typename FPrec<MODE>::real;
  constexpr int DD = D * D;
  constexpr bool BF = (MODE == BGK_BF16);
  // products of differences c (f_j - f_i), so that the BF16 rounding scales
  // with the differences
  constexpr bool DIFF = BF;
  // 3D (not BF16): c = g.w - sum_k |a_k.w| with g.w = sum_k a_k.w advanced
  // by its own increment (|x| is a free source modifier: 3 adds per velocity
  // instead of 3 mins and 2 adds); 2D keeps 2 sum_k min(0, a_k.w) (equal cost)
  constexpr bool GW = (D == 3 && !BF);
  // record: a_k (d*d), a_k.U (d), a_k[FA]*dvs (d)[, their sum].  FP64
  // keeps only a_k and a_k.U (3D: 12 doubles, 6 instead of 8 wave-uniform
  // 16-byte LDS reads per edge; 2D: 6 instead of 8 doubles): every wave
  // reads each record of its edges once per 2-4 velocities, and those
  // broadcast reads occupy the LDS return path.  Its column FA (the
  // stepping axis, below) is held in units of the velocity step, a_k[FA]
  // dvs, which is then the per-step increment itself, and the lane's
  // velocity on that axis enters as v_FA / dvs = k_FA - (nv - 1) / 2 (exact).
  constexpr bool LEAN = (MODE == BGK_FP64);
  constexpr int REC = LEAN ? DD + D : DD + 2 * D + (GW ? 1 : 0);
  // In 3D the third frame vector b has no z component, so neither has R =
  // gamma b: the walk skips that product (the same sums, bit for bit), and
  // the lean record stores the increment of g.w, sum_k a_k[FA] dvs, in
  // its slot.
  constexpr bool RZ0 = (D == 3);
  // The R velocities of a lane step along axis FA: in 3D the z axis (memory
  // stride nv^2), along which R.w is constant (R has no z component), so only
  // the first KV projections advance and |R.w| is formed once per edge and
  // lane; in 2D the fastest axis, x (stride 1).
  constexpr int FA = (D == 3) ? D - 1 : 0;
  constexpr int KV = (D == 3) ? D - 1 : D;
  // Record layout.  Lean: the rows a_k (d*d), then a_k.U (d).  Full: for
  // each k the row a_k followed by a_k.U (in 3D one 16-byte piece of FP32),
  // then the increments a_k[FA] dvs (d)[, their sum].
  constexpr int RW = LEAN ? D : D + 1;                       // stride of the rows
  constexpr int IG = LEAN ? DD - 1 : D * RW + D;             // increment of g.w (3D)
  auto ia = [](int k, int m) constexpr { return k * RW + m; };                // a_k[m]
  auto ib = [](int k) constexpr { return LEAN ? DD + k : k * RW + D; };       // a_k.U
  auto ii = [](int k) constexpr { return LEAN ? k * D + FA : D * RW + k; };   // increment of p_k
  constexpr int KM = TP * (D + 1);              // first-pass moment sums per thread
  constexpr int KP = pow2_at_least(KM);
  constexpr int KP2 = pow2_at_least(TP);         // second pass: one sum per particle
  // the per-edge records are read only during the walk, the reduction
  // slots and exponential tables only after it: they share LDS
  struct Post {
    double red[16][KP > KP2 ? KP : KP2];
    double etab[TP][D][kMaxNv];
  };
  union Shared {
    Real lrec[kChunk][TP][REC];
    Post post;
  };
  __shared__ __align__(16) Shared sh;
  __shared__ double vtab[kMaxNv];
  __shared__ double pstat[TP][D + 5];           // rho, U[d], T, norm, a, b
  extern __shared__ __align__(16) unsigned char fts_raw[];  // INLDS tiles
  auto& lrec = sh.lrec;
  auto& red = sh.post.red;
  auto& etab = sh.post.etab;

  const int tid = threadIdx.x;
  const int nthreads = blockDim.x;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const int patch = lb % a.npatch;
  const int tile0 = INLDS ? 0 : lb / a.npatch;
  const int ntl = INLDS ? a.ntl : 1;
  // slot of (stored tile tl, particle t, velocity r, component c) of this thread
  Real* fts = reinterpret_cast<Real*>(fts_raw);
  auto fts_at = [&](int tl, int t, int r, int c) -> Real& {
    return fts[(((static_cast<size_t>(tl) * TP + t) * R + r) * NC + c) * a.bte + tid];
  };
  const Real* __restrict__ f = static_cast<const Real*>(a.f);
  Real* __restrict__ fo = static_cast<Real*>(a.fo);
  const Real* __restrict__ ops = static_cast<const Real*>(a.ops);
  const size_t NVs = static_cast<size_t>(a.NV);
  const size_t cs = static_cast<size_t>(a.N) * NVs;
  // elements between a lane's consecutive velocities
  const int zs = FA == 0 ? 1 : a.nv * a.nv;
  const uint32_t zsb = static_cast<uint32_t>(zs) * sizeof(Real);
  // R velocities of this thread at row offsets q0 + r zs, from a row's base
  auto store_v = [&](Real* base, int qq0, const Real (&o)[R]) {
    if constexpr (FA == 0) {
      store_r<Real, R>(base + qq0, o);
    } else {
      store_rz<Real, R>(base, static_cast<uint32_t>(qq0) * sizeof(Real), zsb, o);
    }
  };

  int pt[TP];
#pragma unroll
  for (int t = 0; t < TP; ++t) {
    const int g = patch * TP + t;
    pt[t] = g < a.Ni ? a.plist[g] : -1;
  }
  if (tid < a.nv) vtab[tid] = vnode(tid, a.nv, a.vmax);
  __syncthreads();

  // velocities of this thread in tile tile0 + tl: q = q0 + r zs; component
  // FA is kq[FA] + r, the others are fixed.  Lane L of the patch takes the
  // L-th group of R velocities, the groups of one z plane first (3D), so
  // that consecutive lanes hold consecutive velocities of each plane.
  auto tile_vel = [&](int tl, bool& on, int& qq0, int (&kk)[D]) {
    const int L = (tile0 + tl) * a.bte + tid;
    const int qs = FA == 0 ? R * L : L % zs + (L / zs) * zs * R;
    on = tid < a.bte && R * L < a.NV;
    qq0 = on ? qs : 0;
    int q = qq0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      kk[k] = q % a.nv;
      q /= a.nv;
    }
  };
  const int nu = a.ucount[patch];
  const int32_t* __restrict__ ujp = a.uj + static_cast<size_t>(patch) * a.ucap;
  const uint32_t* __restrict__ uep = a.ue + static_cast<size_t>(patch) * a.ucap;
  const Real dvs = static_cast<Real>(a.dvs);
  // ft = f - dt sum c (f_j - f_i) (DIFF), or = f (1 + dt sum c) - dt sum c f_j;
  // the factor 2 of c is folded into dt (except where BF16 rounds 2 cm, and
  // in the 3D form, whose g.w - sum |a_k.w| already is c)
  const Real dtf = static_cast<Real>((BF || GW) ? a.dt : 2.0 * a.dt);
  bool lane_on;
  int q0, kq[D];
  Real ft[TP][R][NC];

  for (int tl = 0; tl < ntl; ++tl) {
  tile_vel(tl, lane_on, q0, kq);
  Real v0[D];
#pragma unroll
  for (int k = 0; k < D; ++k) v0[k] = static_cast<Real>(vtab[kq[k]]);
  if constexpr (LEAN) v0[FA] = static_cast<Real>(kq[FA]) - static_cast<Real>(0.5 * (a.nv - 1));

  auto load_self = [&](int t, int c, Real (&o)[R]) {
    Real tmp[R];
    const Real* src = f + c * cs + static_cast<size_t>(max(pt[t], 0)) * NVs + q0;
    if constexpr (FA == 0)
      load_r<Real, R>(src, tmp);
    else
      load_rz<Real, R>(src - q0, static_cast<uint32_t>(q0) * sizeof(Real), zsb, tmp);
#pragma unroll
    for (int r = 0; r < R; ++r) o[r] = (pt[t] >= 0 && lane_on) ? tmp[r] : Real(0);
  };

  // DIFF: fi = f_i, acc = sum c (f_j - f_i).  Otherwise acc = sum c f_j and
  // csum = sum c.
  Real acc[TP][R][NC];
  Real fi[DIFF ? TP : 1][R][NC];
  Real csum[DIFF ? 1 : TP][R];
#pragma unroll
  for (int t = 0; t < TP; ++t)
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[t][r][c] = Real(0);
      if constexpr (!DIFF) csum[t][r] = Real(0);
    }
  if constexpr (DIFF) {
#pragma unroll
    for (int t = 0; t < TP; ++t)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        Real tmp[R];
        load_self(t, c, tmp);
#pragma unroll
        for (int r = 0; r < R; ++r) fi[t][r][c] = tmp[r];
      }
  }

  for (int c0 = 0; c0 < nu; c0 += kChunk) {
    const int cn = min(kChunk, nu - c0);
    // the chunk's union entries, one per lane of every wave (kChunk is the
    // wave width), read back with readlane: row index j << 4 | the mask of
    // the patch slots that have it (N < 2^27 under the size limits)
    uint32_t vju = 0;
    {
      const int l = tid & 63;
      if (l < cn) {
        const uint32_t pe = uep[c0 + l];
        uint32_t m = 0;
#pragma unroll
        for (int s2 = 0; s2 < TP; ++s2)
          if (((pe >> (8 * s2)) & 0xFFu) != 0xFFu) m |= 1u << s2;
        vju = (static_cast<uint32_t>(ujp[c0 + l]) << 4) | m;
      }
    }
    __syncthreads();  // the previous chunk is consumed
    // stage: one (u, t) record per thread
    for (int w = tid; w < cn * TP; w += nthreads) {
      const int u = w / TP, t = w - u * TP;
      const uint32_t pe = uep[c0 + u];
      const uint32_t e = (pe >> (8 * t)) & 0xFFu;
      Real* rec = lrec[u][t];
      if (e != 0xFFu) {
        const int i = a.plist[patch * TP + t];  // present slots are real particles
        const Real* o = ops + (static_cast<size_t>(i) * a.cap + e) * DD;
        Real av[DD];
#pragma unroll
        for (int k = 0; k < DD; ++k) av[k] = o[k];
#pragma unroll
        for (int k = 0; k < D; ++k) {
          Real b = Real(0);
#pragma unroll
          for (int m = 0; m < D; ++m)
            b = fma_t(av[k * D + m], static_cast<Real>(a.U[static_cast<size_t>(m) * a.N + i]), b);
          rec[ib(k)] = b;
          if constexpr (!LEAN) rec[ii(k)] = av[k * D + FA] * dvs;
        }
        if constexpr (GW && !LEAN) {
          Real gi = rec[ii(0)];
#pragma unroll
          for (int k = 1; k < D; ++k) gi = gi + rec[ii(k)];
          rec[IG] = gi;
        }
#pragma unroll
        for (int k = 0; k < D; ++k)
#pragma unroll
          for (int m = 0; m < D; ++m)
            rec[ia(k, m)] = (LEAN && m == FA) ? av[k * D + m] * dvs : av[k * D + m];
        if constexpr (LEAN && GW) {
          Real gi = rec[ii(0)];
#pragma unroll
          for (int k = 1; k < D; ++k) gi = gi + rec[ii(k)];
          rec[IG] = gi;
        }
      }
    }
    __syncthreads();

    // Neighbour rows are loaded three union entries ahead into a ring of
    // three register buffers (the loop is unrolled by three so the buffers
    // never move).  Loads are unconditional (clamped entry, lane-clamped
    // address), so the waits before each use are exact partial counts.
    Real ra[R][NC], rb[R][NC], rc[R][NC];
    const uint32_t lane_off = static_cast<uint32_t>(q0) * sizeof(Real);
    auto load_row = [&](int uu, Real (&buf)[R][NC]) {
      const int j = static_cast<int>(static_cast<uint32_t>(__builtin_amdgcn_readlane(vju, uu)) >> 4);
      const Real* src = f + static_cast<size_t>(j) * NVs;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        Real tmp[R];
        if constexpr (FA != 0)
          load_rz<Real, R>(src + c * cs, lane_off, zsb, tmp);
        else if constexpr ((R * sizeof(Real)) % 16 == 0)
          load_rb<Real, R>(src + c * cs, lane_off, tmp);
        else
          load_r<Real, R>(src + c * cs + q0, tmp);
#pragma unroll
        for (int r = 0; r < R; ++r) buf[r][c] = tmp[r];
      }
      // keep the prefetch where it is issued (the compiler would otherwise
      // sink it down to its first use, one entry later instead of three)
      asm volatile("" ::: "memory");
    };
    auto process = [&](int u, const Real (&fj)[R][NC]) {
      // Consume the row once in straight-line code, so that the wait for
      // its load is placed here (exact: the two newer rows stay in flight)
      // rather than inside the per-particle branches below.
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c) asm volatile("" ::"v"(fj[r][c]));
      const uint32_t mask = static_cast<uint32_t>(__builtin_amdgcn_readlane(vju, u)) & 15u;
#pragma unroll
      for (int t = 0; t < TP; ++t) {
        if (mask & (1u << t)) {
          const Real* rec = lrec[u][t];
          Real ik[D], p[D];
          // up to 4 velocities per thread: the whole record in registers,
          // read as 16-byte pieces where it is a whole number of them (one
          // broadcast read per 16 bytes instead of one per 8)
          constexpr bool V16 = R < 8 && (REC * sizeof(Real)) % 16 == 0;
          Real rv[V16 ? REC : 1];
          auto rc = [&](int k) -> Real {
            if constexpr (V16) return rv[k];
            return rec[k];
          };
          if constexpr (R >= 8) {
            // many velocities per thread: read the per-edge rows one at a
            // time, so that their registers are not all live at once
#pragma unroll
            for (int k = 0; k < D; ++k) {
              Real s1 = -rec[ib(k)];
#pragma unroll
              for (int m = 0; m < D; ++m)
                if (!(RZ0 && k == D - 1 && m == D - 1)) s1 = fma_t(rec[ia(k, m)], v0[m], s1);
              p[k] = s1;
              asm volatile("" ::: "memory");
            }
          } else {
            if constexpr (V16) {
              constexpr int W = 16 / static_cast<int>(sizeof(Real));
              typedef Real V __attribute__((ext_vector_type(W)));
              const V* rp = reinterpret_cast<const V*>(__builtin_assume_aligned(rec, 16));
#pragma unroll
              for (int i = 0; i < REC / W; ++i) {
                const V x = rp[i];
#pragma unroll
                for (int w = 0; w < W; ++w) rv[i * W + w] = x[w];
              }
            }
            Real av[DD], bk[D];
#pragma unroll
            for (int k = 0; k < D; ++k)
#pragma unroll
              for (int m = 0; m < D; ++m)
                av[k * D + m] = (RZ0 && k == D - 1 && m == D - 1) ? Real(0) : rc(ia(k, m));
#pragma unroll
            for (int k = 0; k < D; ++k) bk[k] = rc(ib(k));
#pragma unroll
            for (int k = 0; k < D; ++k) {
              Real s1 = -bk[k];
#pragma unroll
              for (int m = 0; m < D; ++m)
                if (!(RZ0 && k == D - 1 && m == D - 1)) s1 = fma_t(av[k * D + m], v0[m], s1);
              p[k] = s1;
            }
          }
#pragma unroll
          for (int k = 0; k < KV; ++k) ik[k] = rc(ii(k));
          // the projections past KV are constant along the lane's velocities:
          // their terms are formed once (GW: folded into g.w)
          Real gw = Real(0), ig = Real(0), cfix = Real(0);
          if constexpr (GW) {
            gw = p[0];
#pragma unroll
            for (int k = 1; k < D; ++k) gw = gw + p[k];
#pragma unroll
            for (int k = KV; k < D; ++k) gw = gw - abs_t(p[k]);
            ig = rc(IG);
          } else if constexpr (KV < D) {
            cfix = min_t(p[KV], Real(0));
#pragma unroll
            for (int k = KV + 1; k < D; ++k) cfix = cfix + min_t(p[k], Real(0));
          }
#pragma unroll
          for (int r = 0; r < R; ++r) {
            if (r > 0) {
#pragma unroll
              for (int k = 0; k < KV; ++k) p[k] = p[k] + ik[k];
              if constexpr (GW) gw = gw + ig;
            }
            Real cm;
            if constexpr (GW) {
              cm = gw;  // = 2 sum_k min(0, p_k)
#pragma unroll
              for (int k = 0; k < KV; ++k) cm = cm - abs_t(p[k]);
            } else {
              cm = min_t(p[0], Real(0));
#pragma unroll
              for (int k = 1; k < KV; ++k) cm = cm + min_t(p[k], Real(0));
              if constexpr (KV < D) cm = cm + cfix;
            }
            if constexpr (BF) {
#pragma unroll
              for (int c = 0; c < NC; ++c)
                acc[t][r][c] = fma_t(bf16r(cm + cm), bf16r(fj[r][c] - fi[t][r][c]), acc[t][r][c]);
            } else {
              csum[t][r] = csum[t][r] + cm;
#pragma unroll
              for (int c = 0; c < NC; ++c) acc[t][r][c] = fma_t(cm, fj[r][c], acc[t][r][c]);
            }
          }
        }
      }
    };
    const int last = cn - 1;
    if constexpr (BF && D == 2 && R <= 4) {
      // BF16 operands in 2D: the union is walked two rows at a time, and the
      // two products of a (slot, velocity, component) go through one packed
      // BF16 dot product with FP32 accumulation.  A slot that lacks one of
      // the two rows gets zero projections there, hence c = 0.  (Up to 4
      // velocities per lane: the four-row ring fits the registers.  In 3D,
      // with one component, the doubled per-edge set-up costs more than the
      // packed products save.)
      auto setup = [&](int uu, int t, bool on, Real (&p)[D], Real (&ik)[D]) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
          p[k] = Real(0);
          ik[k] = Real(0);
        }
        if (!on) return;
        const Real* rec = lrec[uu][t];
#pragma unroll
        for (int k = 0; k < D; ++k) {
          Real s1 = -rec[ib(k)];
#pragma unroll
          for (int m = 0; m < D; ++m) s1 = fma_t(rec[ia(k, m)], v0[m], s1);
          p[k] = s1;
          ik[k] = rec[ii(k)];
        }
      };
      auto process2 = [&](int u, const Real (&fa)[R][NC], const Real (&fb)[R][NC]) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            asm volatile("" ::"v"(fa[r][c]));
            asm volatile("" ::"v"(fb[r][c]));
          }
        const bool has_b = u + 1 < cn;
        const uint32_t ma = static_cast<uint32_t>(__builtin_amdgcn_readlane(vju, u)) & 15u;
        const uint32_t mb =
            has_b ? static_cast<uint32_t>(__builtin_amdgcn_readlane(vju, u + 1)) & 15u : 0u;
#pragma unroll
        for (int t = 0; t < TP; ++t) {
          const bool ta = (ma >> t) & 1u, tb = (mb >> t) & 1u;
          if (!(ta || tb)) continue;
          Real pa[D], ia[D], pb[D], ib[D];
          setup(u, t, ta, pa, ia);
          setup(u + 1, t, tb, pb, ib);
#pragma unroll
          for (int r = 0; r < R; ++r) {
            if (r > 0) {
#pragma unroll
              for (int k = 0; k < D; ++k) {
                pa[k] = pa[k] + ia[k];
                pb[k] = pb[k] + ib[k];
              }
            }
            Real ca = min_t(pa[0], Real(0)), cb = min_t(pb[0], Real(0));
#pragma unroll
            for (int k = 1; k < D; ++k) {
              ca = ca + min_t(pa[k], Real(0));
              cb = cb + min_t(pb[k], Real(0));
            }
            const bf16x2 cp = bf16_pair(ca + ca, cb + cb);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
              const bf16x2 dp = bf16_pair(fa[r][c] - fi[t][r][c], fb[r][c] - fi[t][r][c]);
              acc[t][r][c] = __builtin_amdgcn_fdot2_f32_bf16(cp, dp, acc[t][r][c], false);
            }
          }
        }
      };
      Real rd[R][NC];
      load_row(0, ra);
      load_row(min(1, last), rb);
      load_row(min(2, last), rc);
      load_row(min(3, last), rd);
      for (int u = 0; u < cn; u += 4) {
        process2(u, ra, rb);
        load_row(min(u + 4, last), ra);
        load_row(min(u + 5, last), rb);
        if (u + 2 < cn) process2(u + 2, rc, rd);
        load_row(min(u + 6, last), rc);
        load_row(min(u + 7, last), rd);
      }
    } else if constexpr (D == 3 && MODE == BGK_FP64 && R >= 4) {
      // FP64 in 3D at 4 velocities per lane fills the 128 registers of a
      // 1024-lane block: a two-row ring keeps it from spilling
      load_row(0, ra);
      load_row(min(1, last), rb);
      for (int u = 0; u < cn; u += 2) {
        process(u, ra);
        load_row(min(u + 2, last), ra);
        if (u + 1 < cn) process(u + 1, rb);
        load_row(min(u + 3, last), rb);
      }
    } else {
      load_row(0, ra);
      load_row(min(1, last), rb);
      load_row(min(2, last), rc);
      for (int u = 0; u < cn; u += 3) {
        process(u, ra);
        load_row(min(u + 3, last), ra);
        if (u + 1 < cn) process(u + 1, rb);
        load_row(min(u + 4, last), rb);
        if (u + 2 < cn) process(u + 2, rc);
        load_row(min(u + 5, last), rc);
      }
    }
  }

#pragma unroll
  for (int t = 0; t < TP; ++t) {
    if constexpr (DIFF) {
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c) ft[t][r][c] = fi[t][r][c] - dtf * acc[t][r][c];
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        Real self[R];
        load_self(t, c, self);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const Real g = fma_t(dtf, csum[t][r], Real(1));
          ft[t][r][c] = fma_t(self[r], g, -(dtf * acc[t][r][c]));
        }
      }
    }
  }
  if (FUSE && a.fto != nullptr) {
    Real* __restrict__ fto = static_cast<Real*>(a.fto);
#pragma unroll
    for (int t = 0; t < TP; ++t)
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (pt[t] >= 0 && lane_on) {
          Real tmp[R];
#pragma unroll
          for (int r = 0; r < R; ++r) tmp[r] = ft[t][r][c];
          store_v(fto + c * cs + static_cast<size_t>(pt[t]) * NVs, q0, tmp);
        }
  }
  if constexpr (INLDS) {
    // (lanes past bte have no slot: slot s of lane l is s * bte + l)
    if (tl + 1 < ntl && tid < a.bte) {
#pragma unroll
      for (int t = 0; t < TP; ++t)
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int c = 0; c < NC; ++c) fts_at(tl, t, r, c) = ft[t][r][c];
    }
  }
  }  // tiles

  if constexpr (!FUSE) {
#pragma unroll
    for (int t = 0; t < TP; ++t)
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (pt[t] >= 0 && lane_on) {
          Real tmp[R];
#pragma unroll
          for (int r = 0; r < R; ++r) tmp[r] = ft[t][r][c];
          store_v(fo + c * cs + static_cast<size_t>(pt[t]) * NVs, q0, tmp);
        }
    return;
  } else {
    // the records are consumed by every wave before red / etab reuse them
    __syncthreads();
    const int lane = tid & 63, wid = tid >> 6, nw = nthreads >> 6;
    // f-tilde of (tile tl, particle t, velocity r, component c) of this
    // thread: the stored tiles from LDS, the last one from registers
    // velocities of tile tl of this thread (the last tile's are at hand)
    auto epi_vel = [&](int tl, bool& on, int& qq0, int (&kk)[D]) {
      if constexpr (INLDS) {
        if (tl + 1 < ntl) {
          tile_vel(tl, on, qq0, kk);
          return;
        }
      }
      on = lane_on;
      qq0 = q0;
#pragma unroll
      for (int k = 0; k < D; ++k) kk[k] = kq[k];
    };
    auto ftv = [&](int tl, int t, int r, int c) -> double {
      if constexpr (INLDS) {
        if (tl + 1 < ntl) return static_cast<double>(fts_at(tl, t, r, c));
      }
      return static_cast<double>(ft[t][r][c]);
    };
    // ---- S5 pass 1 (FP64): s0 = sum f1, s1 = sum v f1
    double sm[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) sm[k] = 0.0;
    for (int tl = 0; tl < ntl; ++tl) {
      bool on;
      int qq0, kk[D];
      epi_vel(tl, on, qq0, kk);
      if (!on) continue;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double v[D];
#pragma unroll
        for (int k = 0; k < D; ++k) v[k] = vtab[k == FA ? kk[FA] + r : kk[k]];
#pragma unroll
        for (int t = 0; t < TP; ++t) {
          const double x = ftv(tl, t, r, 0);
          double* st = sm + t * (D + 1);
          st[0] = st[0] + x;
#pragma unroll
          for (int k = 0; k < D; ++k) st[1 + k] = st[1 + k] + v[k] * x;
        }
      }
    }
    {
      const double part = wave_reduce_scatter<KP>(sm);
      constexpr int G = 64 / KP;
      if (lane % G == 0) red[wid][(lane / G) % KP] = part;
    }
    __syncthreads();
    if (tid < KM) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s = s + red[w][tid];
      red[0][tid] = s;  // only wave 0's slot is overwritten after all reads
    }
    __syncthreads();
    if (tid < TP) {  // s0 and U of each particle (red is reused below)
      const double s0 = red[0][tid * (D + 1)];
      pstat[tid][0] = s0;
#pragma unroll
      for (int k = 0; k < D; ++k) pstat[tid][1 + k] = red[0][tid * (D + 1) + 1 + k] / s0;
    }
    __syncthreads();
    // ---- S5 pass 2: 3 rho T = sum |v-U|^2 f1 (+ sum f2), U from pass 1
    double se[KP2];
#pragma unroll
    for (int t = 0; t < KP2; ++t) se[t] = 0.0;
    for (int tl = 0; tl < ntl; ++tl) {
      bool on;
      int qq0, kk[D];
      epi_vel(tl, on, qq0, kk);
      if (!on) continue;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double v[D];
#pragma unroll
        for (int k = 0; k < D; ++k) v[k] = vtab[k == FA ? kk[FA] + r : kk[k]];
#pragma unroll
        for (int t = 0; t < TP; ++t) {
          double w2 = 0.0;
#pragma unroll
          for (int k = 0; k < D; ++k) {
            const double wk = v[k] - pstat[t][1 + k];
            w2 = w2 + wk * wk;
          }
          se[t] = se[t] + w2 * ftv(tl, t, r, 0);
          if (NC == 2) se[t] = se[t] + ftv(tl, t, r, NC - 1);
        }
      }
    }
    {
      const double part = wave_reduce_scatter<KP2>(se);
      constexpr int G = 64 / KP2;
      if (lane % G == 0) red[wid][(lane / G) % KP2] = part;
    }
    __syncthreads();
    if (tid < TP) {
      const int t = tid;
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s = s + red[w][t];
      const double s0 = pstat[t][0];
      const double rho = a.omega * s0;
      const double T = s / (3.0 * s0);
      const double tau = a.kn * sqrt(2.0 / kPi) / (rho * sqrt(T));
      const double rden = 1.0 / (tau + a.dt);
      double norm;
      if (D == 3) {
        const double tp = 2.0 * kPi * T;
        norm = rho / (tp * sqrt(tp));
      } else {
        norm = rho / (2.0 * kPi * T);
      }
      pstat[t][0] = rho;
      pstat[t][D + 1] = T;
      pstat[t][D + 2] = norm;
      pstat[t][D + 3] = tau * rden;   // f^{n+1} = a ft + b M, a = tau/(tau+dt)
      pstat[t][D + 4] = a.dt * rden;  //                       b = dt/(tau+dt)
      const int g = patch * TP + t;
      const int i = g < a.Ni ? a.plist[g] : -1;
      if (i >= 0) {
        a.rho[i] = rho;
        a.T[i] = T;
#pragma unroll
        for (int k = 0; k < D; ++k) a.Unew[static_cast<size_t>(k) * a.N + i] = pstat[t][1 + k];
        if (!(rho > 0.0) || !(T > 0.0)) raise_error(a.err, BGK_ENONPHYS);
      }
    }
    __syncthreads();
    // ---- per-axis exponential factors exp(-(v_k - U_a)^2 / (2T))
    for (int w = tid; w < TP * D * a.nv; w += nthreads) {
      const int t = w / (D * a.nv), rem = w - t * (D * a.nv);
      const int k = rem / a.nv, m = rem - k * a.nv;
      const double dv = vtab[m] - pstat[t][1 + k];
      etab[t][k][m] = exp(-(dv * dv) / (2.0 * pstat[t][D + 1]));
    }
    __syncthreads();
    // ---- S6: f^{n+1} = (tau ft + dt M)/(tau + dt) = a ft + b M
    for (int tl = 0; tl < ntl; ++tl) {
      bool on;
      int qq0, kk[D];
      epi_vel(tl, on, qq0, kk);
#pragma unroll
      for (int t = 0; t < TP; ++t) {
        if (pt[t] < 0 || !on) continue;
        const double T = pstat[t][D + 1], norm = pstat[t][D + 2];
        const double ca = pstat[t][D + 3], cb = pstat[t][D + 4];
        double efix = norm;
#pragma unroll
        for (int k = 0; k < D; ++k)
          if (k != FA) efix = efix * etab[t][k][kk[k]];
        Real out[NC][R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double M1 = efix * etab[t][FA][kk[FA] + r];
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const double M = (c == 1) ? T * M1 : M1;
            out[c][r] = static_cast<Real>(fma(cb, M, ca * ftv(tl, t, r, c)));
          }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c)
          store_v(fo + c * cs + static_cast<size_t>(pt[t]) * NVs, qq0, out[c]);
      }
    }
  }
}

// Launch plan: R velocities per thread along the stepping axis (R divides
// nv, so a thread's R velocities share every other component), at most
// Rmax for the precision and model (the per-thread accumulators are
// tp * R * (n_c + 1) values), and the fewest velocity tiles of at most
// 1024 threads (2D: fewer, see lanes_max).  One tile runs the fused
// relaxation.  Several FP64 tiles whose f-tilde (all but the last tile)
// fits the LDS next to the kernel's own tables are walked in turn by one
// block per patch (inlds), which then relaxes them; otherwise each tile is
// a block that writes f-tilde, and the separate relaxation kernel finishes.
struct FusedPlan {
  int R = 0, tiles = 0, bte = 0;
  bool inlds = false;
  size_t lds = 0;   // dynamic LDS bytes of the inlds variant
};

// LDS of one gfx950 workgroup, and what the fused kernel declares
// statically (upper bound over the instantiations that take inlds: 3D FP64
// and 2D FP64 with 2- or 4-particle patches)
constexpr size_t kLdsBytes = 160 * 1024;
constexpr size_t kFusedStaticLds = 34 * 1024;

// Instantiated (patch size, R) pairs per model and precision, within the
// register budget.
template <int D, int MODE, int TP, int R>
constexpr bool fused_instance() {
  if (MODE == BGK_FP64) return (R == 1 || R == 2 || R == 4) && !(D == 2 && TP == 4 && R == 4);
  if (D == 2) return TP == 4 && (R == 1 || R == 2 || R == 4 || R == 5);
  return TP == 4 && (R == 1 || R == 2 || R == 4 || R == 5 || R == 8 || R == 10);
}

static FusedPlan plan_fused(const Ctx& c) {
  const int D = c.D, nv = c.cfg.nv, NV = c.NV;
  const bool f64 = c.cfg.precision == BGK_FP64;
  // instantiated R, ascending
  static const int r64[] = {1, 2, 4};
  static const int r2d[] = {1, 2, 4, 5};
  static const int r3d[] = {1, 2, 4, 5, 8, 10};
  const bool wide = D == 2 && f64 && c.tp == 4;  // FP64 2D with 4-particle patches
  const int rmax = D == 2 ? (wide ? 2 : 4) : (f64 ? 4 : 10);
  const int* cand = f64 ? r64 : (D == 2 ? r2d : r3d);
  const int ncand = f64 ? 3 : (D == 2 ? 4 : 6);
  // 2D: at most 256 lanes, i.e. 4 velocities per lane at 32^2 (fewer,
  // wider row loads and one projection set-up per 4 velocities), or 512
  // lanes of 2 velocities for FP64 with 4-particle patches
  const int lanes_max = D == 2 ? (wide ? 512 : 256) : 1024;
  FusedPlan p;
  // one tile: the smallest admissible R that fits
  for (int i = 0; i < ncand; ++i) {
    const int R = cand[i];
    if (R > rmax || nv % R || NV / R > lanes_max) continue;
    p.R = R;
    p.tiles = 1;
    p.bte = NV / R;
    return p;
  }
  // several tiles: the largest admissible R
  for (int i = ncand - 1; i >= 0; --i) {
    const int R = cand[i];
    if (R > rmax || nv % R) continue;
    const int lanes = NV / R;
    p.R = R;
    p.tiles = (lanes + 1023) / 1024;
    p.bte = (lanes + p.tiles - 1) / p.tiles;
    if (f64) {
      const size_t nc = D == 2 ? 2 : 1;
      p.lds = static_cast<size_t>(p.tiles - 1) * c.tp * R * nc * p.bte * sizeof(double);
      p.inlds = p.lds + kFusedStaticLds <= kLdsBytes;
    }
    return p;
  }
  return p;
}

bool fused_supported(const Ctx& c) { return c.cfg.nv <= kMaxNv && plan_fused(c).R > 0; }

template <int D, int NC, int MODE, bool FUSE, int TP>
static hipError_t launch_fused_t(const Ctx& c, FusedArgs a, const FusedPlan& p) {
  a.bte = p.bte;
  a.dvs = 2.0 * c.cfg.vmax / (c.cfg.nv - 1);
  const bool inlds = FUSE && MODE == BGK_FP64 && p.tiles > 1 && p.inlds;
  a.ntl = inlds ? p.tiles : 1;
  const int bt = (a.bte + 63) / 64 * 64;
  dim3 g(c.npatch * (inlds ? 1 : p.tiles)), b(bt);
  const size_t lds = inlds ? p.lds : 0;
  // (the dynamic LDS size is set on the kernel before the launch: gfx950
  // gives one workgroup up to 160 KB)
#define BGK_LAUNCH_FUSED(RR, IL)                                                          \
  do {                                                                                    \
    auto kf = k_fused<D, NC, MODE, RR, FUSE, TP, IL>;                                     \
    if (lds) {                                                                            \
      const hipError_t ea = hipFuncSetAttribute(reinterpret_cast<const void*>(kf),        \
          hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));             \
      if (ea != hipSuccess) return ea;                                                    \
    }                                                                                     \
    hipLaunchKernelGGL(kf, g, b, lds, c.stream, a);                                       \
  } while (0)
  switch (p.R) {
#define BGK_R_CASE(RR)                                                                    \
  case RR:                                                                                \
    if constexpr (fused_instance<D, MODE, TP, RR>()) {                                    \
      if constexpr (FUSE && MODE == BGK_FP64) {                                           \
        if (inlds) BGK_LAUNCH_FUSED(RR, true);                                            \
        else BGK_LAUNCH_FUSED(RR, false);                                                 \
      } else {                                                                            \
        BGK_LAUNCH_FUSED(RR, false);                                                      \
      }                                                                                   \
    } else {                                                                              \
      return hipErrorInvalidValue;                                                        \
    }                                                                                     \
    break;
    BGK_R_CASE(1)
    BGK_R_CASE(2)
    BGK_R_CASE(4)
    BGK_R_CASE(5)
    BGK_R_CASE(8)
    BGK_R_CASE(10)
#undef BGK_R_CASE
#undef BGK_LAUNCH_FUSED
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <bool FUSE>
static hipError_t launch_fused_any(const Ctx& c, const FusedArgs& a, const FusedPlan& p) {
  const int mode = c.cfg.precision;
  if (c.D == 2) {
    if (mode == BGK_FP64)
      return c.tp == 2 ? launch_fused_t<2, 2, BGK_FP64, FUSE, 2>(c, a, p)
                       : launch_fused_t<2, 2, BGK_FP64, FUSE, 4>(c, a, p);
    if (mode == BGK_FP32) return launch_fused_t<2, 2, BGK_FP32, FUSE, 4>(c, a, p);
    return launch_fused_t<2, 2, BGK_BF16, FUSE, 4>(c, a, p);
  }
  if (mode == BGK_FP64) return launch_fused_t<3, 1, BGK_FP64, FUSE, 4>(c, a, p);
  if (mode == BGK_FP32) return launch_fused_t<3, 1, BGK_FP32, FUSE, 4>(c, a, p);
  return launch_fused_t<3, 1, BGK_BF16, FUSE, 4>(c, a, p);
}

static double omega_fused(const bgk_config& cfg) {
  const double dv = 2.0 * cfg.vmax / static_cast<double>(cfg.nv - 1);
  double w = 1.0;
  for (int k = 0; k < cfg.dim; ++k) w = w * dv;
  return w;
}

hipError_t launch_fused(const Ctx& c, const void* f_in, void* f_out, const double* U_in,
                        double* rho, double* U_out, double* T, bool fuse, void* f_tilde) {
  if (c.npatch == 0) return hipSuccess;
  const FusedPlan p = plan_fused(c);
  if (p.R == 0) return hipErrorInvalidValue;
  FusedArgs a{c.N, c.NV, c.cfg.nv, c.cap, c.Ni, c.npatch, c.ucap, 0,
              c.cfg.vmax, c.cfg.dt, c.cfg.kn, omega_fused(c.cfg), 0.0,
              f_in, f_out, U_in,
              c.cfg.precision == BGK_FP64 ? static_cast<const void*>(c.d.ops64)
                                          : static_cast<const void*>(c.d.ops32),
              c.d.cperm, c.d.ucount, c.d.uj, c.d.ue, rho, U_out, T, c.d.err,
              fuse ? f_tilde : nullptr, 1};
  if (fuse && (p.tiles == 1 || (p.inlds && c.cfg.precision == BGK_FP64)))
    return launch_fused_any<true>(c, a, p);
  // several velocity tiles: f-tilde first (into f_tilde if given, else
  // f_out), then relaxed into f_out
  void* ft = (fuse && f_tilde) ? f_tilde : f_out;
  a.fo = ft;
  a.fto = nullptr;
  hipError_t e = launch_fused_any<false>(c, a, p);
  if (e == hipSuccess && fuse) e = launch_collide(c, ft, f_out, rho, U_out, T);
  return e;
}

}  // namespace bgk
