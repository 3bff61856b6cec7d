// CPU FP64 oracle of the meshfree ALE time step for the BGK equation
// (Mariappan, Willems, Boregowda, Tiwari, Klar: "High-performance computing
// for the BGK model of the Boltzmann equation with a meshfree ALE method").
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
// CPU-baseline leg of the benchmark load this library.  It shares no code,
// header or table with the GPU library: it is written directly from the
// paper, as plain loops in FP64 without fast-math and without FMA
// contraction (built with -ffp-contract=off), parallel over particles only.
//
// Every function names the passage of the paper it follows.  Where the
// paper is silent or garbled, the reading taken is stated at that function.
//
// The state arithmetic (f, U, rho, T, lid speed) is templated on the scalar
// so that a forward-mode dual number gives exact directional derivatives of
// the discrete map (the reference for the hand-written adjoint).  Geometry
// (positions, neighbour sets, least-squares operators) is always double.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <vector>

#include <omp.h>

namespace {

// status codes of the C interface (same numbering as the library's, which
// is part of the documented interface, not shared code)
enum {
  R_OK = 0,
  R_EINVAL = 1,
  R_ENOMEM = 2,
  R_ENBR_OVERFLOW = 3,
  R_ESINGULAR = 4,
  R_ENONPHYS = 5,
  R_ENOTSUP = 7,
};

// ----------------------------------------------------------------------------
// Forward-mode dual number: value v and one directional derivative d.
struct Dual {
  double v = 0.0, d = 0.0;
  Dual() = default;
  Dual(double a) : v(a), d(0.0) {}  // NOLINT: constants promote
  Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) {
  return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)};
}
inline Dual operator+(Dual a, double b) { return {a.v + b, a.d}; }
inline Dual operator+(double a, Dual b) { return {a + b.v, b.d}; }
inline Dual operator-(Dual a, double b) { return {a.v - b, a.d}; }
inline Dual operator-(double a, Dual b) { return {a - b.v, -b.d}; }
inline Dual operator*(Dual a, double b) { return {a.v * b, a.d * b}; }
inline Dual operator*(double a, Dual b) { return {a * b.v, a * b.d}; }
inline Dual operator/(Dual a, double b) { return {a.v / b, a.d / b}; }
inline Dual operator/(double a, Dual b) { return Dual(a) / b; }
inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }

inline double val(double a) { return a; }
inline double val(const Dual& a) { return a.v; }
inline double s_exp(double a) { return std::exp(a); }
inline Dual s_exp(Dual a) {
  const double e = std::exp(a.v);
  return {e, e * a.d};
}
inline double s_sqrt(double a) { return std::sqrt(a); }
inline Dual s_sqrt(Dual a) {
  const double s = std::sqrt(a.v);
  return {s, a.d / (2.0 * s)};
}
// |a|; at a = 0 the derivative of the + branch is taken
inline double s_abs(double a) { return std::fabs(a); }
inline Dual s_abs(Dual a) { return a.v < 0.0 ? Dual{-a.v, -a.d} : a; }
inline double s_sin(double a) { return std::sin(a); }
inline Dual s_sin(Dual a) { return {std::sin(a.v), std::cos(a.v) * a.d}; }
inline double s_cos(double a) { return std::cos(a); }
inline Dual s_cos(Dual a) { return {std::cos(a.v), -std::sin(a.v) * a.d}; }
inline double s_atan2(double y, double x) { return std::atan2(y, x); }
// d atan2(y, x) = (x dy - y dx) / (x^2 + y^2); taken as 0 at the origin
inline Dual s_atan2(Dual y, Dual x) {
  const double r2 = x.v * x.v + y.v * y.v;
  return {std::atan2(y.v, x.v), r2 > 0.0 ? (x.v * y.d - y.v * x.d) / r2 : 0.0};
}
inline double s_acos(double a) { return std::acos(a); }
// d acos(a) = -da / sqrt(1 - a^2); taken as 0 at a = +-1
inline Dual s_acos(Dual a) {
  const double q = 1.0 - a.v * a.v;
  return {std::acos(a.v), q > 0.0 ? -a.d / std::sqrt(q) : 0.0};
}

// Compensated (Neumaier) summation of a long sequence: the running sum plus
// the rounding error of every addition, so that a quadrature sum over a
// velocity grid of any size is accurate to a few units of rounding (a plain
// left-to-right sum of the ~1e6 positive terms of a 96^3 grid is off by
// ~5e-13 relative).  The sum is the same one the moment integrals define;
// only its rounding changes.
template <class S>
struct CSum {
  S s = S(0.0), e = S(0.0);
  void add(const S& x) {
    const S t = s + x;
    if (std::fabs(val(s)) >= std::fabs(val(x)))
      e = e + ((s - t) + x);
    else
      e = e + ((x - t) + s);
    s = t;
  }
  S value() const { return s + e; }
};

}  // namespace

extern "C" {

// Run parameters (nondimensional: R = 1).  Mirrored by the Python wrapper.
typedef struct {
  int32_t dim;          // 2: Chu-reduced (components g1, g2); 3: full BGK
  int32_t n_particles;  // N, interior and wall particles
  int32_t nv;           // velocity points per axis, both ends included
  int32_t wls_degree;   // 0: first-order fit of f_j - f_i (no constant); 1 or 2
  int32_t cap;          // neighbour slots per particle (self included)
  int32_t move;         // 1: x += dt U after the step; 0: frozen cloud
  double vmax;          // velocity grid spans [-vmax, vmax]
  double h;             // support radius (absolute)
  double alpha;         // Gaussian weight exponent
  double kn;            // Knudsen number
  double dt;            // time step
  double wall_T;        // wall temperature
  double lid;           // lid speed (+x) on the y=1 (2D) / z=1 (3D) wall
  double dx;            // initial lattice spacing (clamp margin 0.1 dx)
} ref_config;

}  // extern "C"

namespace {

inline int n_comp(const ref_config& c) { return c.dim == 2 ? 2 : 1; }
inline int64_t n_vel(const ref_config& c) {
  int64_t q = 1;
  for (int a = 0; a < c.dim; ++a) q *= c.nv;
  return q;
}

// ---------------------------------------------------------------------------
// Velocity grid (Section 3.3 "Velocity discretization").  The paper's count
// of N_v+1 points per axis is read as nv points per axis including both
// ends of [-vmax, vmax]: v_k = vmax (2k - (nv-1)) / (nv-1), k = 0..nv-1, and
// every node has the same quadrature weight omega = dv^d, dv = 2 vmax/(nv-1).
inline double vnode(int k, int nv, double vmax) {
  return vmax * static_cast<double>(2 * k - (nv - 1)) / static_cast<double>(nv - 1);
}
inline void velocity(const ref_config& c, int64_t q, double v[3]) {
  v[0] = v[1] = v[2] = 0.0;
  for (int a = 0; a < c.dim; ++a) {
    v[a] = vnode(static_cast<int>(q % c.nv), c.nv, c.vmax);
    q /= c.nv;
  }
}
inline double vweight(const ref_config& c) {
  const double dv = 2.0 * c.vmax / static_cast<double>(c.nv - 1);
  double w = 1.0;
  for (int a = 0; a < c.dim; ++a) w = w * dv;
  return w;
}

// ---------------------------------------------------------------------------
// Maxwellian (Section 2, eq. maxwellian) with R = 1; the exponent carries
// the minus sign that makes the integral equal rho.  In the Chu-reduced
// model (Section 2.1, eqs. Maxw_G1, Maxw_G2) G1 is the v3-marginal of M,
// rho/(2 pi T) exp(-|v-U|^2/(2T)), and G2 = T G1.  Returns component comp
// (0: M or G1, 1: G2) at velocity v.
template <class S>
S maxwellian(const ref_config& c, int comp, const S& rho, const S U[3], const S& T,
             const double v[3]) {
  S s2 = S(0.0);
  for (int a = 0; a < c.dim; ++a) {
    const S wa = v[a] - U[a];
    s2 = s2 + wa * wa;
  }
  const double two_pi = 2.0 * M_PI;
  S norm;
  if (c.dim == 3) {
    const S tp = two_pi * T;
    norm = rho / (tp * s_sqrt(tp));
  } else {
    norm = rho / (two_pi * T);
  }
  S g = norm * s_exp(-s2 / (2.0 * T));
  if (comp == 1) g = T * g;
  return g;
}

// Relaxation time (Section 2, eqs. tau and lambda), nondimensional with
// R T0 = 1 and length L = 1:  tau = 4 lambda/(pi Cbar), Cbar = sqrt(8T/pi),
// lambda = Kn / rho, so tau = Kn sqrt(2/pi) / (rho sqrt(T)).
template <class S>
S tau_of(double kn, const S& rho, const S& T) {
  return kn * std::sqrt(2.0 / M_PI) / (rho * s_sqrt(T));
}

// ---------------------------------------------------------------------------
// Moments (Section 2, eqs. moments and internal_energy; Chu: eq. macroeq;
// the time-discrete versions fullmoment1a, moment1a and moment1b).
// rho = sum omega f1; U = sum v f1 / sum f1; then, with U known,
// 3 rho T = sum omega |v-U|^2 f (full) or sum omega (|v-U|^2 g1 + g2) (Chu).
// f points at the row of one particle: component k at f[k*stride + q].
template <class S>
void moments_row(const ref_config& c, const S* f, int64_t stride, S& rho, S U[3], S& T) {
  const int64_t NV = n_vel(c);
  CSum<S> c0, c1[3];
  double v[3];
  for (int64_t q = 0; q < NV; ++q) {
    velocity(c, q, v);
    c0.add(f[q]);
    for (int a = 0; a < c.dim; ++a) c1[a].add(v[a] * f[q]);
  }
  const S s0 = c0.value();
  const double om = vweight(c);
  rho = om * s0;
  for (int a = 0; a < 3; ++a) U[a] = a < c.dim ? c1[a].value() / s0 : S(0.0);
  CSum<S> ce;
  for (int64_t q = 0; q < NV; ++q) {
    velocity(c, q, v);
    S w2 = S(0.0);
    for (int a = 0; a < c.dim; ++a) {
      const S wa = v[a] - U[a];
      w2 = w2 + wa * wa;
    }
    ce.add(w2 * f[q]);
    if (c.dim == 2) ce.add(f[stride + q]);
  }
  T = ce.value() / (3.0 * s0);
}

// ---------------------------------------------------------------------------
// Neighbour search (Section 3.4.1): the set of particles within the disc /
// ball of radius h, the truncation of eq. weight being inclusive (r/h <= 1).
// Written as the plain O(N^2) definition; the squared distance is summed
// component by component, left to right.
// Row i; returns 1 if the row holds more than cap particles.
template <class S>
int neighbors_row(const ref_config& c, const S* x, int i, int32_t* cnt, int32_t* idx) {
  const int N = c.n_particles, d = c.dim, cap = c.cap;
  const double h2 = c.h * c.h;
  int m = 0;
  for (int j = 0; j < N; ++j) {
    double r2 = 0.0;
    for (int a = 0; a < d; ++a) {
      const double dl = val(x[a * N + j]) - val(x[a * N + i]);
      r2 = r2 + dl * dl;
    }
    if (r2 <= h2) {
      if (m < cap) idx[static_cast<int64_t>(i) * cap + m] = j;
      ++m;
    }
  }
  cnt[i] = m;
  return m > cap ? 1 : 0;
}

template <class S>
int neighbors(const ref_config& c, const S* x, int32_t* cnt, int32_t* idx) {
  const int N = c.n_particles;
  int overflow = 0;
#pragma omp parallel for schedule(static) reduction(| : overflow)
  for (int i = 0; i < N; ++i) overflow |= neighbors_row(c, x, i, cnt, idx);
  return overflow ? R_ENBR_OVERFLOW : R_OK;
}

// ---------------------------------------------------------------------------
// Weighted least squares (Section 3.4.1, eqs. taylor, solution, mls_rhs and
// x/y/z_derivative).  The paper fits the first-order Taylor expansion of
// f_j - f_i and names higher-order expansions as the route to higher
// order.  Taken reading: a full polynomial basis including the constant
// term, of degree 2 (or 1), in offsets scaled by h; the particle itself is in
// its stencil with weight 1.  The derivative rows annihilate constants, so
// the transport keeps the paper's difference form sum_j a_ij (f_j - f_i).
// Degree 0 is the fit exactly as printed: the unknowns are the d first
// derivatives only, the rows of M are the offsets, and the solution is
// a = (M^T W M)^-1 M^T W b with b_j = f_j - f_i (the particle itself has a
// zero offset and drops out of both sums).
int basis_size(int d, int deg) { return deg == 0 ? d : (deg == 1 ? d + 1 : (d == 2 ? 6 : 10)); }

// column of the basis that carries the first derivative along axis a
int grad_column(int deg, int a) { return deg == 0 ? a : 1 + a; }

template <class S>
void basis(int d, int deg, const S* y, S* p) {
  if (deg == 0) {
    for (int a = 0; a < d; ++a) p[a] = y[a];
    return;
  }
  p[0] = S(1.0);
  for (int a = 0; a < d; ++a) p[1 + a] = y[a];
  if (deg == 2) {
    int k = d + 1;
    for (int a = 0; a < d; ++a)
      for (int b = a; b < d; ++b) p[k++] = y[a] * y[b];
  }
}

// Cholesky factorisation A = L L^T of a symmetric B x B matrix (row major).
// Returns false on a non-positive pivot.
template <class S>
bool cholesky(int B, const S* A, S* L) {
  for (int i = 0; i < B * B; ++i) L[i] = S(0.0);
  for (int j = 0; j < B; ++j) {
    S s = A[j * B + j];
    for (int k = 0; k < j; ++k) s = s - L[j * B + k] * L[j * B + k];
    if (!(val(s) > 0.0)) return false;
    const S ljj = s_sqrt(s);
    L[j * B + j] = ljj;
    for (int i = j + 1; i < B; ++i) {
      S t = A[i * B + j];
      for (int k = 0; k < j; ++k) t = t - L[i * B + k] * L[j * B + k];
      L[i * B + j] = t / ljj;
    }
  }
  return true;
}

// Solve L L^T z = e_col.
template <class S>
void chol_solve_unit(int B, const S* L, int col, S* z) {
  S y[16];
  for (int i = 0; i < B; ++i) {
    S s = S((i == col) ? 1.0 : 0.0);
    for (int k = 0; k < i; ++k) s = s - L[i * B + k] * y[k];
    y[i] = s / L[i * B + i];
  }
  for (int i = B - 1; i >= 0; --i) {
    S s = y[i];
    for (int k = i + 1; k < B; ++k) s = s - L[k * B + i] * z[k];
    z[i] = s / L[i * B + i];
  }
}

// Local frame of the edge i -> j (Section 3.4.2).  2D: n along the edge at
// angle phi = atan2(dy, dx), t = n turned by +90 degrees.  3D: the matrix A
// built from phi = atan2(dy, dx) and theta = arccos(dz/r); rows n, t, b.
template <class S>
void edge_frame(int d, const S* dl, S n[3], S t[3], S b[3]) {
  if (d == 2) {
    const S phi = s_atan2(dl[1], dl[0]);
    n[0] = s_cos(phi);
    n[1] = s_sin(phi);
    t[0] = -s_sin(phi);
    t[1] = s_cos(phi);
    n[2] = t[2] = S(0.0);
    b[0] = b[1] = b[2] = S(0.0);
  } else {
    const S r = s_sqrt(dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2]);
    const S phi = s_atan2(dl[1], dl[0]);
    const S th = s_acos(dl[2] / r);
    const S st = s_sin(th), ct = s_cos(th);
    const S sp = s_sin(phi), cp = s_cos(phi);
    n[0] = st * cp;
    n[1] = st * sp;
    n[2] = ct;
    t[0] = ct * cp;
    t[1] = ct * sp;
    t[2] = -st;
    b[0] = -sp;
    b[1] = cp;
    b[2] = S(0.0);
  }
}

// Gradient rows g_ij and upwind vectors of every interior particle.
// grad[i][e][a] = d/dx_a weight of neighbour e; ops[i][e] = (P, Q[, R]) with
// P = abar n, Q = bbar t, R = gbar b, where (abar, bbar, gbar) are the
// gradient weights rotated into the edge frame: abar = g.n etc. (the 2D
// rotation of Section 3.4.2; in 3D the same rotation, which needs A, not
// its transpose, to keep P + Q + R = g).
// Degree: the configured degree if the stencil has at least twice as many
// points as basis functions, else degree 1 if it has d+2 points, else error
// (degree 0 also needs d+2 points, the particle itself included).
// Row i (zero for wall particles); returns R_OK or R_ESINGULAR.
template <class S>
int wls_row(const ref_config& c, const S* x, const int32_t* wall_id, const int32_t* cnt,
            const int32_t* idx, int i, S* grad, S* ops, int32_t* degree) {
  const int N = c.n_particles, d = c.dim, cap = c.cap, dd = d * d;
  {
    const int64_t row = static_cast<int64_t>(i) * cap;
    for (int e = 0; e < cap; ++e) {
      for (int a = 0; a < d; ++a) grad[(row + e) * d + a] = S(0.0);
      for (int a = 0; a < dd; ++a) ops[(row + e) * dd + a] = S(0.0);
    }
    if (degree) degree[i] = 0;
    if (wall_id[i] != 0) return R_OK;
    const int m = std::min<int>(cnt[i], cap);
    int deg = c.wls_degree;
    if (deg == 2 && m < 2 * basis_size(d, 2)) deg = 1;
    if (m < d + 2) return R_ESINGULAR;
    const int B = basis_size(d, deg);
    S A[100], L[100];
    for (int k = 0; k < 100; ++k) A[k] = S(0.0);
    std::vector<S> P(static_cast<size_t>(m) * B), W(m);
    for (int e = 0; e < m; ++e) {
      const int j = idx[row + e];
      S y[3], r2 = S(0.0);
      for (int a = 0; a < d; ++a) {
        y[a] = (x[a * N + j] - x[a * N + i]) / c.h;
        r2 = r2 + y[a] * y[a];
      }
      W[e] = s_exp(-c.alpha * r2);
      basis(d, deg, y, &P[static_cast<size_t>(e) * B]);
    }
    for (int e = 0; e < m; ++e)
      for (int r = 0; r < B; ++r)
        for (int s = 0; s < B; ++s)
          A[r * B + s] = A[r * B + s] + W[e] * P[e * B + r] * P[e * B + s];
    if (!cholesky(B, A, L)) return R_ESINGULAR;
    S z[3][16];
    for (int a = 0; a < d; ++a) chol_solve_unit(B, L, grad_column(deg, a), z[a]);
    for (int e = 0; e < m; ++e) {
      const int j = idx[row + e];
      S g[3] = {S(0.0), S(0.0), S(0.0)};
      for (int a = 0; a < d; ++a) {
        S s = S(0.0);
        for (int r = 0; r < B; ++r) s = s + z[a][r] * P[e * B + r];
        g[a] = W[e] * s / c.h;
        grad[(row + e) * d + a] = g[a];
      }
      if (j == i) continue;
      S dl[3] = {S(0.0), S(0.0), S(0.0)}, n[3], t[3], b[3];
      for (int a = 0; a < d; ++a) dl[a] = x[a * N + j] - x[a * N + i];
      edge_frame(d, dl, n, t, b);
      S ab = S(0.0), bb = S(0.0), gb = S(0.0);
      for (int a = 0; a < d; ++a) {
        ab = ab + g[a] * n[a];
        bb = bb + g[a] * t[a];
        gb = gb + g[a] * b[a];
      }
      S* o = &ops[(row + e) * dd];
      for (int a = 0; a < d; ++a) {
        o[a] = ab * n[a];
        o[d + a] = bb * t[a];
        if (d == 3) o[2 * d + a] = gb * b[a];
      }
    }
    if (degree) degree[i] = deg;
  }
  return R_OK;
}

template <class S>
int wls(const ref_config& c, const S* x, const int32_t* wall_id, const int32_t* cnt,
        const int32_t* idx, S* grad, S* ops, int32_t* degree) {
  const int N = c.n_particles;
  int err = R_OK;
#pragma omp parallel for schedule(dynamic, 64)
  for (int i = 0; i < N; ++i) {
    const int e = wls_row(c, x, wall_id, cnt, idx, i, grad, ops, degree);
    if (e != R_OK) {
#pragma omp critical
      err = e;
    }
  }
  return err;
}

// ---------------------------------------------------------------------------
// Boundary stencils.  The paper only names the interpolation of f on the
// boundary and the diffuse-reflection condition (Table 3, Section 5).
// Taken reading: each wall particle b reconstructs f at x_b from the
// interior particles within radius hb (the rule below), by a degree-1
// weighted least-squares fit (weights exp(-alpha r^2/hb^2)) evaluated at
// x_b: f_b = sum_j c0_bj f_j.
// Value row at a point xq: the interior particles within hb (ascending) and
// the degree-1 least-squares value weights at xq (weights
// exp(-alpha r^2/hb^2)), so that f(xq) ~ sum_e c0[e] f_{set[e]}.  hb is the
// first of h, 1.5h, 2h whose set holds at least d+2 particles, gives a
// positive-definite fit, and keeps the extrapolation's amplification
// sum_e |c0_e| at most kValueRowAmp; the 2h row is taken without the bound.
// (The bound lies above the amplification of every row of the jittered
// initial lattices, 3.7 in 2D and 6.6 in 3D, so it acts only where a moving
// cloud has left a wall particle a near-degenerate stencil: the plain first
// radius with d+2 points then extrapolates with weights summing to ~100 in
// magnitude, and the step turns non-physical.)  The set and the radius
// depend on the positions' values only.
constexpr double kValueRowAmp = 8.0;

template <class S>
int value_row(const ref_config& c, const S* x, const int32_t* wall_id, const S* xq,
              std::vector<int>& set, std::vector<S>& c0, double& hb) {
  const int N = c.n_particles, d = c.dim;
  const double mults[3] = {1.0, 1.5, 2.0};
  for (int k = 0; k < 3; ++k) {
    const bool last = k == 2;
    hb = mults[k] * c.h;
    const double hb2 = hb * hb;
    set.clear();
    for (int j = 0; j < N; ++j) {
      if (wall_id[j] != 0) continue;
      double r2 = 0.0;
      for (int a = 0; a < d; ++a) {
        const double dl = val(x[a * N + j]) - val(xq[a]);
        r2 = r2 + dl * dl;
      }
      if (r2 <= hb2) set.push_back(j);
    }
    const int m = static_cast<int>(set.size());
    if (m < d + 2) {
      if (last) return R_ESINGULAR;
      continue;
    }
    if (m > c.cap) return R_ENBR_OVERFLOW;
    const int B = d + 1;
    S A[16], L[16];
    for (int q = 0; q < 16; ++q) A[q] = S(0.0);
    std::vector<S> P(static_cast<size_t>(m) * B), W(m);
    for (int e = 0; e < m; ++e) {
      S y[3], r2 = S(0.0);
      for (int a = 0; a < d; ++a) {
        y[a] = (x[a * N + set[e]] - xq[a]) / hb;
        r2 = r2 + y[a] * y[a];
      }
      W[e] = s_exp(-c.alpha * r2);
      basis(d, 1, y, &P[static_cast<size_t>(e) * B]);
    }
    for (int e = 0; e < m; ++e)
      for (int r = 0; r < B; ++r)
        for (int s = 0; s < B; ++s)
          A[r * B + s] = A[r * B + s] + W[e] * P[e * B + r] * P[e * B + s];
    if (!cholesky(B, A, L)) {
      if (last) return R_ESINGULAR;
      continue;
    }
    S z[16];
    chol_solve_unit(B, L, 0, z);
    c0.assign(m, S(0.0));
    double amp = 0.0;
    for (int e = 0; e < m; ++e) {
      S s = S(0.0);
      for (int r = 0; r < B; ++r) s = s + z[r] * P[e * B + r];
      c0[e] = W[e] * s;
      amp = amp + std::fabs(val(c0[e]));
    }
    if (last || amp <= kValueRowAmp) return R_OK;
  }
  return R_ESINGULAR;
}

template <class S>
int wall_stencil(const ref_config& c, const S* x, const int32_t* wall_id, int32_t* wcnt,
                 int32_t* widx, S* wc0, double* hb_out) {
  const int N = c.n_particles, d = c.dim, cap = c.cap;
  int err = R_OK;
#pragma omp parallel for schedule(dynamic, 16)
  for (int b = 0; b < N; ++b) {
    const int64_t row = static_cast<int64_t>(b) * cap;
    wcnt[b] = 0;
    if (hb_out) hb_out[b] = 0.0;
    if (wall_id[b] == 0) continue;
    S xb[3] = {S(0.0), S(0.0), S(0.0)};
    for (int a = 0; a < d; ++a) xb[a] = x[a * N + b];
    std::vector<int> set;
    std::vector<S> c0;
    double hb = 0.0;
    const int rc = value_row(c, x, wall_id, xb, set, c0, hb);
    if (rc != R_OK) {
#pragma omp critical
      err = rc;
      continue;
    }
    const int m = static_cast<int>(set.size());
    for (int e = 0; e < m; ++e) {
      widx[row + e] = set[e];
      wc0[row + e] = c0[e];
    }
    wcnt[b] = m;
    if (hb_out) hb_out[b] = hb;
  }
  return err;
}

// ---------------------------------------------------------------------------
// Particle management (Section 3.5.2: adding and removing points).  The
// paper removes two points that come too close and puts one at their
// midpoint, adds points where holes open, and fills f at the new points by
// least squares; it gives no thresholds or selection rule.  Taken reading:
//  - merge: interior particles i < j that are each other's nearest interior
//    neighbour within h (ties to the lower index) and closer than
//    merge_radius become one interior particle at 0.5 (x_i + x_j);
//  - holes: an interior node of the initial lattice (coordinates k dx,
//    0 < k < n-1) with no particle of the merged cloud within hole_radius
//    gets a new interior particle;
//  - f at every new particle: the value row of the old cloud at its
//    position (the rule of the wall rows), applied to every velocity and
//    component; its rho, U, T are the moments of that f, while the other
//    particles keep theirs (U^n feeds the next transport);
//  - order of the new cloud: the untouched particles in their old order,
//    then the midpoints by the lower index of their pair, then the hole
//    particles by node index k_x + n k_y (+ n^2 k_z).
struct PmPlan {
  std::vector<int> partner;   // -1, or the other particle of its pair
  std::vector<int> holes;     // node indices
  int n_pairs = 0;
};

inline double dist2(int d, const double* p, const double* q) {
  double r2 = 0.0;
  for (int a = 0; a < d; ++a) {
    const double dl = p[a] - q[a];
    r2 = r2 + dl * dl;
  }
  return r2;
}

inline int lattice_n(const ref_config& c) { return static_cast<int>(std::lround(1.0 / c.dx)) + 1; }

void pm_plan(const ref_config& c, const double* x, const int32_t* wall_id, double rm, double rh,
             PmPlan& p) {
  const int N = c.n_particles, d = c.dim;
  auto pos = [&](int i, double* o) {
    for (int a = 0; a < d; ++a) o[a] = x[a * N + i];
  };
  std::vector<int> nn(N, -1);
#pragma omp parallel for schedule(dynamic, 64)
  for (int i = 0; i < N; ++i) {
    if (wall_id[i] != 0) continue;
    double xi[3], xj[3];
    pos(i, xi);
    double best = c.h * c.h;
    for (int j = 0; j < N; ++j) {
      if (j == i || wall_id[j] != 0) continue;
      pos(j, xj);
      const double r2 = dist2(d, xj, xi);
      if (r2 <= c.h * c.h && (nn[i] < 0 || r2 < best)) {
        best = r2;
        nn[i] = j;
      }
    }
  }
  p.partner.assign(N, -1);
  p.n_pairs = 0;
  for (int i = 0; i < N; ++i) {
    const int j = nn[i];
    if (j > i && nn[j] == i) {
      double xi[3], xj[3];
      pos(i, xi);
      pos(j, xj);
      if (dist2(d, xj, xi) < rm * rm) {
        p.partner[i] = j;
        p.partner[j] = i;
        ++p.n_pairs;
      }
    }
  }
  // the merged cloud: untouched particles and the midpoints
  std::vector<double> pts;
  for (int i = 0; i < N; ++i) {
    double xi[3] = {0, 0, 0}, xj[3];
    pos(i, xi);
    if (p.partner[i] >= 0) {
      if (p.partner[i] < i) continue;
      pos(p.partner[i], xj);
      for (int a = 0; a < d; ++a) xi[a] = 0.5 * (xi[a] + xj[a]);
    }
    for (int a = 0; a < d; ++a) pts.push_back(xi[a]);
  }
  const int M = static_cast<int>(pts.size()) / d;
  const int n = lattice_n(c);
  int64_t nodes = 1;
  for (int a = 0; a < d; ++a) nodes *= n;
  std::vector<char> hole(nodes, 0);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t k = 0; k < nodes; ++k) {
    double y[3] = {0, 0, 0};
    int64_t r = k;
    bool inner = true;
    for (int a = 0; a < d; ++a) {
      const int ka = static_cast<int>(r % n);
      r /= n;
      inner = inner && ka > 0 && ka < n - 1;
      y[a] = static_cast<double>(ka) * c.dx;
    }
    if (!inner) continue;
    bool covered = false;
    for (int q = 0; q < M && !covered; ++q) covered = dist2(d, &pts[static_cast<size_t>(q) * d], y) <= rh * rh;
    hole[k] = covered ? 0 : 1;
  }
  p.holes.clear();
  for (int64_t k = 0; k < nodes; ++k)
    if (hole[k]) p.holes.push_back(static_cast<int>(k));
}

int pm_apply(const ref_config& c, const double* x, const int32_t* wall_id, const double* f,
             const double* rho, const double* U, const double* T, const PmPlan& p,
             double* x_new, int32_t* wall_id_new, double* f_new, double* rho_new, double* U_new,
             double* T_new) {
  const int N = c.n_particles, d = c.dim, nc = n_comp(c);
  const int64_t NV = n_vel(c);
  const int Nn = N - p.n_pairs + static_cast<int>(p.holes.size());
  const int n = lattice_n(c);
  // positions and owners of the new cloud, and the old row each new
  // particle copies (-1: interpolated)
  std::vector<int> src;
  std::vector<double> nx;
  for (int i = 0; i < N; ++i) {
    if (p.partner[i] >= 0) continue;
    src.push_back(i);
    for (int a = 0; a < d; ++a) nx.push_back(x[a * N + i]);
  }
  for (int i = 0; i < N; ++i) {
    if (p.partner[i] <= i) continue;
    src.push_back(-1);
    for (int a = 0; a < d; ++a) nx.push_back(0.5 * (x[a * N + i] + x[a * N + p.partner[i]]));
  }
  for (int k : p.holes) {
    src.push_back(-1);
    int64_t r = k;
    for (int a = 0; a < d; ++a) {
      nx.push_back(static_cast<double>(r % n) * c.dx);
      r /= n;
    }
  }
  int err = R_OK;
#pragma omp parallel for schedule(dynamic, 16)
  for (int q = 0; q < Nn; ++q) {
    const double* xq = &nx[static_cast<size_t>(q) * d];
    for (int a = 0; a < d; ++a) x_new[static_cast<int64_t>(a) * Nn + q] = xq[a];
    wall_id_new[q] = src[q] >= 0 ? wall_id[src[q]] : 0;
    for (int cc = 0; cc < nc; ++cc) {
      double* out = f_new + (static_cast<int64_t>(cc) * Nn + q) * NV;
      if (src[q] >= 0) {
        const double* in = f + (static_cast<int64_t>(cc) * N + src[q]) * NV;
        for (int64_t v = 0; v < NV; ++v) out[v] = in[v];
      }
    }
    if (src[q] >= 0) {
      rho_new[q] = rho[src[q]];
      T_new[q] = T[src[q]];
      for (int a = 0; a < d; ++a) U_new[static_cast<int64_t>(a) * Nn + q] = U[a * N + src[q]];
      continue;
    }
    std::vector<int> S;
    std::vector<double> c0;
    double hb = 0.0;
    const int rc = value_row(c, x, wall_id, xq, S, c0, hb);
    if (rc != R_OK) {
#pragma omp critical
      err = rc;
      continue;
    }
    for (int cc = 0; cc < nc; ++cc) {
      double* out = f_new + (static_cast<int64_t>(cc) * Nn + q) * NV;
      for (int64_t v = 0; v < NV; ++v) {
        double s = 0.0;
        for (size_t e = 0; e < S.size(); ++e)
          s = s + c0[e] * f[(static_cast<int64_t>(cc) * N + S[e]) * NV + v];
        out[v] = s;
      }
    }
    double r, u[3], t;
    moments_row(c, f_new + static_cast<int64_t>(q) * NV, static_cast<int64_t>(Nn) * NV, r, u, t);
    rho_new[q] = r;
    T_new[q] = t;
    for (int a = 0; a < d; ++a) U_new[static_cast<int64_t>(a) * Nn + q] = u[a];
  }
  return err;
}

// ---------------------------------------------------------------------------
// Explicit transport step (Section 3.2.1, eq. explicit; Section 3.2.2) with the positive
// upwind flux of Section 3.4.2 (eq. flux and its 3D counterpart):
//   ft_i(v) = f_i(v) - dt sum_{j != i} c_ij(v) (f_j(v) - f_i(v)),
//   c_ij(v) = g_ij.w - |P_ij.w| - |Q_ij.w| - |R_ij.w|,  w = v - U_i^n.
// This is the printed flux abar[w.n - |w.n|] + bbar[w.t - sign(bbar)|w.t|]
// (+ gbar[w.b - sign(gbar)|w.b|]) with the dissipation of the n-term taken
// as |abar||w.n| (equal to the printed form when abar >= 0, which is the
// positivity hypothesis of the scheme).  Wall particles are not transported.
// (G: the operators' type, double for a fixed cloud or the state's type
// when the cloud moves with the state.)
template <class S, class G>
void transport_row(const ref_config& c, const int32_t* wall_id, const int32_t* cnt,
                   const int32_t* idx, const G* grad, const G* ops, const S* U,
                   const S* f, S* ft, int i) {
  const int N = c.n_particles, d = c.dim, cap = c.cap, dd = d * d, nc = n_comp(c);
  const int64_t NV = n_vel(c);
  {
    for (int k = 0; k < nc; ++k) {
      const S* fi = f + (static_cast<int64_t>(k) * N + i) * NV;
      S* out = ft + (static_cast<int64_t>(k) * N + i) * NV;
      if (wall_id[i] != 0) {
        for (int64_t q = 0; q < NV; ++q) out[q] = fi[q];
      }
    }
    if (wall_id[i] != 0) return;
    const int64_t row = static_cast<int64_t>(i) * cap;
    const int m = std::min<int>(cnt[i], cap);
    double v[3];
    for (int64_t q = 0; q < NV; ++q) {
      velocity(c, q, v);
      S w[3];
      for (int a = 0; a < d; ++a) w[a] = v[a] - U[a * N + i];
      S acc[2] = {S(0.0), S(0.0)};
      for (int e = 0; e < m; ++e) {
        const int j = idx[row + e];
        if (j == i) continue;
        const G* g = &grad[(row + e) * d];
        const G* o = &ops[(row + e) * dd];
        S gw = S(0.0), pw = S(0.0), qw = S(0.0), rw = S(0.0);
        for (int a = 0; a < d; ++a) {
          gw = gw + g[a] * w[a];
          pw = pw + o[a] * w[a];
          qw = qw + o[d + a] * w[a];
          if (d == 3) rw = rw + o[2 * d + a] * w[a];
        }
        S cij = gw - s_abs(pw) - s_abs(qw);
        if (d == 3) cij = cij - s_abs(rw);
        for (int k = 0; k < nc; ++k) {
          const S fj = f[(static_cast<int64_t>(k) * N + j) * NV + q];
          const S fi = f[(static_cast<int64_t>(k) * N + i) * NV + q];
          acc[k] = acc[k] + cij * (fj - fi);
        }
      }
      for (int k = 0; k < nc; ++k) {
        const S fi = f[(static_cast<int64_t>(k) * N + i) * NV + q];
        ft[(static_cast<int64_t>(k) * N + i) * NV + q] = fi - c.dt * acc[k];
      }
    }
  }
}

template <class S, class G>
void transport(const ref_config& c, const int32_t* wall_id, const int32_t* cnt, const int32_t* idx,
               const G* grad, const G* ops, const S* U, const S* f, S* ft) {
  const int N = c.n_particles;
#pragma omp parallel for schedule(dynamic, 16)
  for (int i = 0; i < N; ++i) transport_row(c, wall_id, cnt, idx, grad, ops, U, f, ft, i);
}

// ---------------------------------------------------------------------------
// Implicit relaxation (Section 3.2.1: eqs. implicitfull_1 and fullmoment1a
// and the closed form that follows; Section 3.2.2 reduced model: eqs.
// implicit_1/2, moment1a, moment1b).  The new (rho, U, T) are the moments of
// ft; tau is taken at the new state; f^{n+1} = (tau ft + dt M^{n+1})/(tau+dt).
// Row i (nothing for wall particles); returns R_OK or R_ENONPHYS.
template <class S>
int collide_row(const ref_config& c, const int32_t* wall_id, const S* ft, S* fout, S* rho, S* U,
                S* T, int i) {
  const int N = c.n_particles, nc = n_comp(c);
  const int64_t NV = n_vel(c), stride = static_cast<int64_t>(N) * NV;
  int err = R_OK;
  {
    if (wall_id[i] != 0) return R_OK;
    const S* fi = ft + static_cast<int64_t>(i) * NV;
    S r, u[3], tt;
    moments_row(c, fi, stride, r, u, tt);
    if (!(val(r) > 0.0) || !(val(tt) > 0.0)) err = R_ENONPHYS;
    rho[i] = r;
    T[i] = tt;
    for (int a = 0; a < c.dim; ++a) U[a * N + i] = u[a];
    const S tau = tau_of(c.kn, r, tt);
    double v[3];
    for (int64_t q = 0; q < NV; ++q) {
      velocity(c, q, v);
      for (int k = 0; k < nc; ++k) {
        const S M = maxwellian(c, k, r, u, tt, v);
        const int64_t o = k * stride + static_cast<int64_t>(i) * NV + q;
        fout[o] = (tau * ft[o] + c.dt * M) / (tau + c.dt);
      }
    }
  }
  return err;
}

template <class S>
int collide(const ref_config& c, const int32_t* wall_id, const S* ft, S* fout, S* rho, S* U,
            S* T) {
  const int N = c.n_particles;
  int err = R_OK;
#pragma omp parallel for schedule(dynamic, 16)
  for (int i = 0; i < N; ++i) {
    const int e = collide_row(c, wall_id, ft, fout, rho, U, T, i);
    if (e != R_OK) {
#pragma omp critical
      err = e;
    }
  }
  return err;
}

// Inward unit normal (axis, sign) and wall velocity of owner wall w (1..2d):
// walls are x=0, x=1, y=0, y=1 (, z=0, z=1); the lid is the last one and
// moves along +x.
inline void wall_geometry(int d, int w, int& axis, double& sign, bool& is_lid) {
  axis = (w - 1) / 2;
  sign = ((w - 1) % 2 == 0) ? 1.0 : -1.0;
  is_lid = (w == 2 * d);
}

// ---------------------------------------------------------------------------
// Diffuse-reflection walls (named in Section 5; Table 3 lists the
// interpolation of f on the boundary and the diffuse-reflection condition).
// Taken reading: velocities arriving at the wall (v.n <= 0, n the inward
// normal) take the interpolated interior value; emitted velocities take
// rho_w M[1, U_w, T_w] (Chu: g1 = rho_w G1hat, g2 = T_w rho_w G1hat) with
// rho_w fixed by zero net discrete mass flux through the wall.  Then the
// wall particle's (rho, U, T) are the moments of its new f.
template <class S, class G>
int wall_bc(const ref_config& c, const S& lid, const int32_t* wall_id, const int32_t* wcnt,
            const int32_t* widx, const G* wc0, S* f, S* rho, S* U, S* T) {
  const int N = c.n_particles, d = c.dim, cap = c.cap, nc = n_comp(c);
  const int64_t NV = n_vel(c), stride = static_cast<int64_t>(N) * NV;
  int err = R_OK;
#pragma omp parallel for schedule(dynamic, 16)
  for (int b = 0; b < N; ++b) {
    if (wall_id[b] == 0) continue;
    int axis;
    double sgn;
    bool is_lid;
    wall_geometry(d, wall_id[b], axis, sgn, is_lid);
    S Uw[3] = {S(0.0), S(0.0), S(0.0)};
    if (is_lid) Uw[0] = lid;
    const S one = S(1.0), Tw = S(c.wall_T);
    const int64_t row = static_cast<int64_t>(b) * cap;
    double v[3];
    CSum<S> in_flux, out_flux;
    for (int64_t q = 0; q < NV; ++q) {
      velocity(c, q, v);
      const double vn = sgn * v[axis];
      if (vn <= 0.0) {
        for (int k = 0; k < nc; ++k) {
          S s = S(0.0);
          for (int e = 0; e < wcnt[b]; ++e)
            s = s + wc0[row + e] * f[k * stride + static_cast<int64_t>(widx[row + e]) * NV + q];
          f[k * stride + static_cast<int64_t>(b) * NV + q] = s;
        }
        in_flux.add((-vn) * f[static_cast<int64_t>(b) * NV + q]);
      } else {
        out_flux.add(vn * maxwellian(c, 0, one, Uw, Tw, v));
      }
    }
    const S rho_w = in_flux.value() / out_flux.value();
    for (int64_t q = 0; q < NV; ++q) {
      velocity(c, q, v);
      const double vn = sgn * v[axis];
      if (vn > 0.0) {
        for (int k = 0; k < nc; ++k)
          f[k * stride + static_cast<int64_t>(b) * NV + q] = maxwellian(c, k, rho_w, Uw, Tw, v);
      }
    }
    S r, u[3], tt;
    moments_row(c, f + static_cast<int64_t>(b) * NV, stride, r, u, tt);
    if (!(val(r) > 0.0) || !(val(tt) > 0.0)) {
#pragma omp critical
      err = R_ENONPHYS;
    }
    rho[b] = r;
    T[b] = tt;
    for (int a = 0; a < d; ++a) U[a * N + b] = u[a];
  }
  return err;
}

// ALE position update (Section 3.2.1: x^{n+1} = x^n + dt U^{n+1}) for interior
// particles, kept inside [0.1 dx, 1 - 0.1 dx]^d (particle management is out
// of this step; clamped coordinates are counted).
// (A clamped coordinate is the constant bound: its derivative is zero.)
template <class S>
int move(const ref_config& c, const int32_t* wall_id, const S* U, S* x) {
  const int N = c.n_particles;
  const double lo = 0.1 * c.dx, hi = 1.0 - 0.1 * c.dx;
  int clamped = 0;
  for (int i = 0; i < N; ++i) {
    if (wall_id[i] != 0) continue;
    for (int a = 0; a < c.dim; ++a) {
      S y = x[a * N + i] + c.dt * U[a * N + i];
      if (val(y) < lo) {
        y = S(lo);
        ++clamped;
      }
      if (val(y) > hi) {
        y = S(hi);
        ++clamped;
      }
      x[a * N + i] = y;
    }
  }
  return clamped;
}

bool config_ok(const ref_config& c) {
  return (c.dim == 2 || c.dim == 3) && c.n_particles > 0 && c.nv >= 2 && c.nv % 2 == 0 &&
         c.wls_degree >= 0 && c.wls_degree <= 2 && c.cap > 0 && c.dt > 0 && c.h > 0 &&
         c.vmax > 0 && c.kn > 0;
}

// Objective: heat flux through the lid plus total kinetic energy.
//   q_n(p) = 1/2 sum omega (v_n - U_n)|v-U|^2 f (full) or
//            1/2 sum omega (v_n - U_n)(|v-U|^2 g1 + g2) (Chu),
// n the lid's outward axis (+y in 2D, +z in 3D), U the particle's own mean
// velocity;  J = dx^(d-1) sum_{lid} q_n + ke_weight/N sum_i 1/2 rho_i |U_i|^2.
template <class S>
S objective(const ref_config& c, const int32_t* wall_id, const S* f, const S* rho, const S* U,
            double ke_weight) {
  const int N = c.n_particles, d = c.dim;
  const int64_t NV = n_vel(c), stride = static_cast<int64_t>(N) * NV;
  const double om = vweight(c);
  const int lid_wall = 2 * d, an = d - 1;
  double area = 1.0;
  for (int a = 0; a < d - 1; ++a) area = area * c.dx;
  S J = S(0.0);
  double v[3];
  for (int p = 0; p < N; ++p) {
    if (wall_id[p] != lid_wall) continue;
    CSum<S> q;
    for (int64_t k = 0; k < NV; ++k) {
      velocity(c, k, v);
      S w2 = S(0.0);
      for (int a = 0; a < d; ++a) {
        const S wa = v[a] - U[a * N + p];
        w2 = w2 + wa * wa;
      }
      S e = w2 * f[static_cast<int64_t>(p) * NV + k];
      if (d == 2) e = e + f[stride + static_cast<int64_t>(p) * NV + k];
      q.add((v[an] - U[an * N + p]) * e);
    }
    J = J + area * (0.5 * om) * q.value();
  }
  if (ke_weight != 0.0) {
    for (int i = 0; i < N; ++i) {
      S u2 = S(0.0);
      for (int a = 0; a < d; ++a) u2 = u2 + U[a * N + i] * U[a * N + i];
      J = J + (ke_weight / N) * (0.5 * rho[i] * u2);
    }
  }
  return J;
}

// Geometry of one step: neighbours, operators and wall stencils at x (G:
// double, or the dual type when the positions carry derivatives).
template <class G>
struct GeometryT {
  std::vector<int32_t> cnt, idx, deg, wcnt, widx;
  std::vector<G> grad, ops, wc0;
  int build(const ref_config& c, const G* x, const int32_t* wall_id) {
    const int64_t N = c.n_particles, cap = c.cap;
    cnt.assign(N, 0);
    idx.assign(N * cap, 0);
    deg.assign(N, 0);
    wcnt.assign(N, 0);
    widx.assign(N * cap, 0);
    grad.assign(N * cap * c.dim, G(0.0));
    ops.assign(N * cap * c.dim * c.dim, G(0.0));
    wc0.assign(N * cap, G(0.0));
    int rc = neighbors(c, x, cnt.data(), idx.data());
    if (rc) return rc;
    rc = wls(c, x, wall_id, cnt.data(), idx.data(), grad.data(), ops.data(), deg.data());
    if (rc) return rc;
    return wall_stencil(c, x, wall_id, wcnt.data(), widx.data(), wc0.data(), nullptr);
  }
};
using Geometry = GeometryT<double>;

// One time step on the state (f, U) at positions x with a given geometry:
// transport, moments + relaxation, walls.  f_out receives f^{n+1}; U is
// overwritten with U^{n+1}; rho and T receive the new values.
template <class S, class G>
int advance(const ref_config& c, const GeometryT<G>& g, const int32_t* wall_id, const S& lid,
            const S* f_in, S* f_out, S* U, S* rho, S* T) {
  const int64_t total = static_cast<int64_t>(n_comp(c)) * c.n_particles * n_vel(c);
  std::vector<S> ft(total);
  transport(c, wall_id, g.cnt.data(), g.idx.data(), g.grad.data(), g.ops.data(), U, f_in,
            ft.data());
  std::copy(ft.begin(), ft.end(), f_out);
  int rc = collide(c, wall_id, ft.data(), f_out, rho, U, T);
  const int rc2 = wall_bc(c, lid, wall_id, g.wcnt.data(), g.widx.data(), g.wc0.data(), f_out,
                          rho, U, T);
  return rc ? rc : rc2;
}

}  // namespace

extern "C" {

// OpenMP threads the oracle's parallel loops use.
int ref_num_threads() { return omp_get_max_threads(); }

// Velocity node and quadrature weight of the grid (for tests).
double ref_velocity_node(int k, int nv, double vmax) { return vnode(k, nv, vmax); }
double ref_velocity_weight(const ref_config* c) { return vweight(*c); }

// tau in the paper's dimensional form (eqs. tau and lambda):
// tau = 4 lambda / (pi Cbar), Cbar = sqrt(8 R T/pi), lambda = kb/(sqrt2 pi rho R d^2).
double ref_tau_dimensional(double rho, double T, double R, double kb, double diam) {
  const double lambda = kb / (std::sqrt(2.0) * M_PI * rho * R * diam * diam);
  const double cbar = std::sqrt(8.0 * R * T / M_PI);
  return 4.0 * lambda / (M_PI * cbar);
}
double ref_tau(double kn, double rho, double T) { return tau_of(kn, rho, T); }

// Maxwellian (or G1, G2) of every particle on the grid: f[k][N][NV].
int ref_maxwellian(const ref_config* c, const double* rho, const double* U, const double* T,
                   double* f) {
  const int N = c->n_particles, nc = n_comp(*c);
  const int64_t NV = n_vel(*c);
#pragma omp parallel for
  for (int i = 0; i < N; ++i) {
    double u[3] = {0, 0, 0}, v[3];
    for (int a = 0; a < c->dim; ++a) u[a] = U[a * N + i];
    for (int64_t q = 0; q < NV; ++q) {
      velocity(*c, q, v);
      for (int k = 0; k < nc; ++k)
        f[(static_cast<int64_t>(k) * N + i) * NV + q] = maxwellian(*c, k, rho[i], u, T[i], v);
    }
  }
  return R_OK;
}

int ref_moments(const ref_config* c, const double* f, double* rho, double* U, double* T) {
  const int N = c->n_particles;
  const int64_t NV = n_vel(*c), stride = static_cast<int64_t>(N) * NV;
#pragma omp parallel for
  for (int i = 0; i < N; ++i) {
    double r, u[3], t;
    moments_row(*c, f + static_cast<int64_t>(i) * NV, stride, r, u, t);
    rho[i] = r;
    T[i] = t;
    for (int a = 0; a < c->dim; ++a) U[a * N + i] = u[a];
  }
  return R_OK;
}

int ref_neighbors(const ref_config* c, const double* x, int32_t* cnt, int32_t* idx) {
  if (!config_ok(*c)) return R_EINVAL;
  return neighbors(*c, x, cnt, idx);
}

int ref_wls_operators(const ref_config* c, const double* x, const int32_t* wall_id,
                      const int32_t* cnt, const int32_t* idx, double* grad, double* ops,
                      int32_t* degree) {
  if (!config_ok(*c)) return R_EINVAL;
  return wls(*c, x, wall_id, cnt, idx, grad, ops, degree);
}

int ref_wall_stencil(const ref_config* c, const double* x, const int32_t* wall_id, int32_t* wcnt,
                     int32_t* widx, double* wc0, double* hb) {
  if (!config_ok(*c)) return R_EINVAL;
  return wall_stencil(*c, x, wall_id, wcnt, widx, wc0, hb);
}

// Particle management: counts of the plan (merged pairs, hole particles).
// The new cloud has N - n_pairs + n_holes particles.
int ref_pm_count(const ref_config* c, const double* x, const int32_t* wall_id,
                 double merge_radius, double hole_radius, int32_t* n_pairs, int32_t* n_holes) {
  if (!c || !config_ok(*c) || !x || !wall_id || !n_pairs || !n_holes) return R_EINVAL;
  PmPlan p;
  pm_plan(*c, x, wall_id, merge_radius, hole_radius, p);
  *n_pairs = p.n_pairs;
  *n_holes = static_cast<int32_t>(p.holes.size());
  return R_OK;
}

// Particle management: the new cloud (x_new [d][N'], wall_id_new [N'],
// f_new [n_c][N'][N_v], rho/T_new [N'], U_new [d][N']) for the same plan.
int ref_pm_apply(const ref_config* c, const double* x, const int32_t* wall_id, const double* f,
                 const double* rho, const double* U, const double* T, double merge_radius,
                 double hole_radius, double* x_new, int32_t* wall_id_new, double* f_new,
                 double* rho_new, double* U_new, double* T_new) {
  if (!c || !config_ok(*c) || !x || !wall_id || !f || !rho || !U || !T || !x_new ||
      !wall_id_new || !f_new || !rho_new || !U_new || !T_new)
    return R_EINVAL;
  PmPlan p;
  pm_plan(*c, x, wall_id, merge_radius, hole_radius, p);
  return pm_apply(*c, x, wall_id, f, rho, U, T, p, x_new, wall_id_new, f_new, rho_new, U_new,
                  T_new);
}

int ref_transport(const ref_config* c, const int32_t* wall_id, const int32_t* cnt,
                  const int32_t* idx, const double* grad, const double* ops, const double* U,
                  const double* f, double* ft) {
  if (!config_ok(*c)) return R_EINVAL;
  transport(*c, wall_id, cnt, idx, grad, ops, U, f, ft);
  return R_OK;
}

// Relaxation of interior particles: fout (interior rows) and their rho, U, T.
int ref_collide(const ref_config* c, const int32_t* wall_id, const double* ft, double* fout,
                double* rho, double* U, double* T) {
  if (!config_ok(*c)) return R_EINVAL;
  return collide(*c, wall_id, ft, fout, rho, U, T);
}

// Walls: overwrites the wall rows of f (which must hold f^{n+1} on interior
// rows) and the wall particles' rho, U, T.
int ref_wall_bc(const ref_config* c, const int32_t* wall_id, const int32_t* wcnt,
                const int32_t* widx, const double* wc0, double* f, double* rho, double* U,
                double* T) {
  if (!config_ok(*c)) return R_EINVAL;
  return wall_bc(*c, c->lid, wall_id, wcnt, widx, wc0, f, rho, U, T);
}

int ref_move(const ref_config* c, const int32_t* wall_id, const double* U, double* x,
             int32_t* clamped) {
  const int k = move(*c, wall_id, U, x);
  if (clamped) *clamped = k;
  return R_OK;
}

// Timing sample of the per-particle work of one step (S1-S6) for the
// interior particles among i0..i1-1: the neighbour row, the least-squares
// row, the transport of the row and its moments + relaxation, with the same
// row functions the full step uses, on `threads` OpenMP threads (0: all).
// Rows of the other particles are not computed.  f_out (full [n_c][N][N_v])
// receives the new rows of the sampled particles; *seconds the wall time of
// the row work alone (buffers are allocated before the clock starts).
int ref_step_rows(const ref_config* c, const int32_t* wall_id, const double* x,
                  const double* f_in, const double* U_in, int i0, int i1, int threads,
                  double* f_out, double* seconds, int32_t* n_rows) {
  if (!config_ok(*c) || i0 < 0 || i1 > c->n_particles || i0 > i1) return R_EINVAL;
  const int64_t N = c->n_particles, cap = c->cap, d = c->dim;
  std::vector<int32_t> cnt(N, 0), idx(N * cap, 0), deg(N, 0);
  std::vector<double> grad(N * cap * d, 0.0), ops(N * cap * d * d, 0.0);
  std::vector<double> U(U_in, U_in + d * N), rho(N, 0.0), T(N, 0.0);
  std::unique_ptr<double[]> ft(new double[n_comp(*c) * N * n_vel(*c)]);
  std::vector<int> rows;
  for (int i = i0; i < i1; ++i)
    if (wall_id[i] == 0) rows.push_back(i);
  const int nr = static_cast<int>(rows.size());
  const int nt = threads > 0 ? threads : omp_get_max_threads();
  int err = R_OK;
  const double t0 = omp_get_wtime();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (int r = 0; r < nr; ++r) {
    const int i = rows[r];
    int e = neighbors_row(*c, x, i, cnt.data(), idx.data()) ? R_ENBR_OVERFLOW : R_OK;
    if (e == R_OK)
      e = wls_row(*c, x, wall_id, cnt.data(), idx.data(), i, grad.data(), ops.data(), deg.data());
    if (e == R_OK) {
      transport_row(*c, wall_id, cnt.data(), idx.data(), grad.data(), ops.data(), U_in, f_in,
                    ft.get(), i);
      e = collide_row(*c, wall_id, ft.get(), f_out, rho.data(), U.data(), T.data(), i);
    }
    if (e != R_OK) {
#pragma omp critical
      err = e;
    }
  }
  *seconds = omp_get_wtime() - t0;
  if (n_rows) *n_rows = nr;
  return err;
}

// One full step S1..S8: geometry at x^n, transport with U^n, relaxation,
// walls, then (if c->move) x^{n+1} = x^n + dt U^{n+1}.
int ref_step(const ref_config* c, const int32_t* wall_id, double* x, const double* f_in,
             double* f_out, double* U, double* rho, double* T, int32_t* clamped) {
  if (!config_ok(*c)) return R_EINVAL;
  Geometry g;
  int rc = g.build(*c, x, wall_id);
  if (rc) return rc;
  rc = advance(*c, g, wall_id, c->lid, f_in, f_out, U, rho, T);
  int k = 0;
  if (c->move) k = move(*c, wall_id, U, x);
  if (clamped) *clamped = k;
  return rc;
}

// Objective at a state (see objective()).
double ref_objective(const ref_config* c, const int32_t* wall_id, const double* f,
                     const double* rho, const double* U, double ke_weight) {
  return objective(*c, wall_id, f, rho, U, ke_weight);
}

// Frozen-cloud rollout: (rho, U, T)^0 = moments of f0, then nsteps steps,
// then J.  With dual inputs (f0_dot, lid_dot) it returns the exact
// directional derivative J_dot of J along (f0_dot, lid_dot).  f_final may be
// null.  c->move must be 0 (the derivative is of the frozen-cloud map).
int ref_rollout_dual(const ref_config* c, const int32_t* wall_id, const double* x,
                     const double* f0, const double* f0_dot, double lid_dot, int nsteps,
                     double ke_weight, double* J, double* J_dot, double* f_final) {
  if (!config_ok(*c) || c->move) return R_EINVAL;
  Geometry g;
  int rc = g.build(*c, x, wall_id);
  if (rc) return rc;
  const int N = c->n_particles;
  const int64_t total = static_cast<int64_t>(n_comp(*c)) * N * n_vel(*c);
  std::vector<Dual> fa(total), fb(total), U(static_cast<size_t>(3) * N), rho(N), T(N);
  for (int64_t k = 0; k < total; ++k) fa[k] = Dual(f0[k], f0_dot ? f0_dot[k] : 0.0);
  const int64_t NV = n_vel(*c), stride = static_cast<int64_t>(N) * NV;
  for (int i = 0; i < N; ++i) {
    Dual r, u[3], t;
    moments_row(*c, fa.data() + static_cast<int64_t>(i) * NV, stride, r, u, t);
    rho[i] = r;
    T[i] = t;
    for (int a = 0; a < c->dim; ++a) U[a * N + i] = u[a];
  }
  const Dual lid(c->lid, lid_dot);
  for (int s = 0; s < nsteps; ++s) {
    rc = advance(*c, g, wall_id, lid, fa.data(), fb.data(), U.data(), rho.data(), T.data());
    if (rc) return rc;
    std::swap(fa, fb);
  }
  const Dual Jd = objective(*c, wall_id, fa.data(), rho.data(), U.data(), ke_weight);
  *J = Jd.v;
  *J_dot = Jd.d;
  if (f_final)
    for (int64_t k = 0; k < total; ++k) f_final[k] = fa[k].v;
  return R_OK;
}

// One frozen-cloud step with tangents: (f, U) with directions (f_dot,
// U_dot) and the lid speed's direction lid_dot -> f^{n+1}, U^{n+1}, rho, T
// and their exact directional derivatives.  Null tangent inputs are zero.
// One full step S1..S8 with the cloud moving (c->move must be 1), every
// quantity carrying one directional derivative: the geometry (neighbour
// sets fixed by the positions' values; least-squares rows, edge frames and
// wall rows as functions of the positions), transport, relaxation, walls
// and the position update, so that the derivative includes how the moving
// cloud changes the operators.  Inputs: state (x, f, U) and tangents
// (x_dot, f_dot, U_dot; each may be null = 0) and lid_dot; outputs the new
// state and its tangents.
int ref_step_dual_move(const ref_config* c, const int32_t* wall_id, const double* x,
                       const double* x_dot, const double* f, const double* f_dot,
                       const double* U, const double* U_dot, double lid_dot, double* x_out,
                       double* x_out_dot, double* f_out, double* f_out_dot, double* U_out,
                       double* U_out_dot, double* rho, double* rho_dot, double* T,
                       double* T_dot) {
  if (!config_ok(*c) || !c->move) return R_EINVAL;
  const int N = c->n_particles, d = c->dim;
  const int64_t total = static_cast<int64_t>(n_comp(*c)) * N * n_vel(*c);
  std::vector<Dual> xd(static_cast<size_t>(d) * N), fa(total), fb(total),
      Ud(static_cast<size_t>(3) * N), rd(N), Td(N);
  for (int64_t k = 0; k < static_cast<int64_t>(d) * N; ++k) {
    xd[k] = Dual(x[k], x_dot ? x_dot[k] : 0.0);
    Ud[k] = Dual(U[k], U_dot ? U_dot[k] : 0.0);
  }
  for (int64_t k = 0; k < total; ++k) fa[k] = Dual(f[k], f_dot ? f_dot[k] : 0.0);
  GeometryT<Dual> g;
  int rc = g.build(*c, xd.data(), wall_id);
  if (rc) return rc;
  rc = advance(*c, g, wall_id, Dual(c->lid, lid_dot), fa.data(), fb.data(), Ud.data(), rd.data(),
               Td.data());
  move(*c, wall_id, Ud.data(), xd.data());
  for (int64_t k = 0; k < total; ++k) {
    f_out[k] = fb[k].v;
    f_out_dot[k] = fb[k].d;
  }
  for (int64_t k = 0; k < static_cast<int64_t>(d) * N; ++k) {
    U_out[k] = Ud[k].v;
    U_out_dot[k] = Ud[k].d;
    x_out[k] = xd[k].v;
    x_out_dot[k] = xd[k].d;
  }
  for (int i = 0; i < N; ++i) {
    rho[i] = rd[i].v;
    rho_dot[i] = rd[i].d;
    T[i] = Td[i].v;
    T_dot[i] = Td[i].d;
  }
  return rc;
}

// Rollout with the moving cloud (c->move must be 1): (rho, U, T)^0 are the
// moments of f0, then nsteps full steps S1..S8, then J of the final state.
// Returns J and its exact directional derivative along (x0_dot, f0_dot,
// lid_dot) (each direction may be null / 0), through the moving geometry.
int ref_rollout_dual_move(const ref_config* c, const int32_t* wall_id, const double* x0,
                          const double* x0_dot, const double* f0, const double* f0_dot,
                          double lid_dot, int nsteps, double ke_weight, double* J,
                          double* J_dot) {
  if (!config_ok(*c) || !c->move) return R_EINVAL;
  const int N = c->n_particles, d = c->dim;
  const int64_t total = static_cast<int64_t>(n_comp(*c)) * N * n_vel(*c);
  std::vector<Dual> xd(static_cast<size_t>(d) * N), fa(total), fb(total),
      U(static_cast<size_t>(3) * N), rho(N), T(N);
  for (int64_t k = 0; k < static_cast<int64_t>(d) * N; ++k)
    xd[k] = Dual(x0[k], x0_dot ? x0_dot[k] : 0.0);
  for (int64_t k = 0; k < total; ++k) fa[k] = Dual(f0[k], f0_dot ? f0_dot[k] : 0.0);
  const int64_t NV = n_vel(*c), stride = static_cast<int64_t>(N) * NV;
  for (int i = 0; i < N; ++i) {
    Dual r, u[3], t;
    moments_row(*c, fa.data() + static_cast<int64_t>(i) * NV, stride, r, u, t);
    rho[i] = r;
    T[i] = t;
    for (int a = 0; a < d; ++a) U[a * N + i] = u[a];
  }
  const Dual lid(c->lid, lid_dot);
  for (int s = 0; s < nsteps; ++s) {
    GeometryT<Dual> g;
    int rc = g.build(*c, xd.data(), wall_id);
    if (rc) return rc;
    rc = advance(*c, g, wall_id, lid, fa.data(), fb.data(), U.data(), rho.data(), T.data());
    if (rc) return rc;
    std::swap(fa, fb);
    move(*c, wall_id, U.data(), xd.data());
  }
  const Dual Jd = objective(*c, wall_id, fa.data(), rho.data(), U.data(), ke_weight);
  *J = Jd.v;
  *J_dot = Jd.d;
  return R_OK;
}

int ref_step_dual(const ref_config* c, const int32_t* wall_id, const double* x, const double* f,
                  const double* f_dot, const double* U, const double* U_dot, double lid_dot,
                  double* f_out, double* f_out_dot, double* U_out, double* U_out_dot,
                  double* rho, double* rho_dot, double* T, double* T_dot) {
  if (!config_ok(*c)) return R_EINVAL;
  Geometry g;
  int rc = g.build(*c, x, wall_id);
  if (rc) return rc;
  const int N = c->n_particles;
  const int64_t total = static_cast<int64_t>(n_comp(*c)) * N * n_vel(*c);
  std::vector<Dual> fa(total), fb(total), Ud(static_cast<size_t>(3) * N), rd(N), Td(N);
  for (int64_t k = 0; k < total; ++k) fa[k] = Dual(f[k], f_dot ? f_dot[k] : 0.0);
  for (int64_t k = 0; k < static_cast<int64_t>(c->dim) * N; ++k)
    Ud[k] = Dual(U[k], U_dot ? U_dot[k] : 0.0);
  rc = advance(*c, g, wall_id, Dual(c->lid, lid_dot), fa.data(), fb.data(), Ud.data(), rd.data(),
               Td.data());
  for (int64_t k = 0; k < total; ++k) {
    f_out[k] = fb[k].v;
    f_out_dot[k] = fb[k].d;
  }
  for (int64_t k = 0; k < static_cast<int64_t>(c->dim) * N; ++k) {
    U_out[k] = Ud[k].v;
    U_out_dot[k] = Ud[k].d;
  }
  for (int i = 0; i < N; ++i) {
    rho[i] = rd[i].v;
    rho_dot[i] = rd[i].d;
    T[i] = Td[i].v;
    T_dot[i] = Td[i].d;
  }
  return rc;
}

// Directional derivative of the objective along (f_dot, rho_dot, U_dot).
double ref_objective_dual(const ref_config* c, const int32_t* wall_id, const double* f,
                          const double* f_dot, const double* rho, const double* rho_dot,
                          const double* U, const double* U_dot, double ke_weight) {
  const int N = c->n_particles;
  const int64_t total = static_cast<int64_t>(n_comp(*c)) * N * n_vel(*c);
  std::vector<Dual> fa(total), ra(N), Ua(static_cast<size_t>(3) * N);
  for (int64_t k = 0; k < total; ++k) fa[k] = Dual(f[k], f_dot ? f_dot[k] : 0.0);
  for (int i = 0; i < N; ++i) ra[i] = Dual(rho[i], rho_dot ? rho_dot[i] : 0.0);
  for (int64_t k = 0; k < static_cast<int64_t>(c->dim) * N; ++k)
    Ua[k] = Dual(U[k], U_dot ? U_dot[k] : 0.0);
  return objective(*c, wall_id, fa.data(), ra.data(), Ua.data(), ke_weight).d;
}

}  // extern "C"
