// Memory and undefined-behaviour check of the CPU oracle (test
// infrastructure): compiled together with the oracle's source under
// AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_oracle_sanitizers.py, it calls every entry point of the oracle
// on small jittered 2D and 3D cavities (a deterministic jitter of its own;
// the values do not matter here, only that every access stays in bounds and
// no operation is undefined).  Exit status 0 and "sanitizer driver ok" on
// success; the sanitizers abort on the first finding.
#include "../oracle/bgk_oracle.cpp"

#include <cstdio>
#include <vector>

namespace {

struct Cloud {
  std::vector<double> x;
  std::vector<int32_t> wid;
};

// lattice of n^d nodes on [0,1]^d with a small deterministic jitter away
// from the walls; owner walls in the order x=0, x=1, y=0, y=1 (, z=0, z=1)
Cloud cloud(int d, int n) {
  const int N = d == 2 ? n * n : n * n * n;
  const double dx = 1.0 / (n - 1);
  Cloud c;
  c.x.assign(static_cast<size_t>(d) * N, 0.0);
  c.wid.assign(N, 0);
  uint64_t s = 12345;
  for (int p = 0; p < N; ++p) {
    int k[3] = {p % n, (p / n) % n, d == 3 ? p / (n * n) : 0};
    int owner = 0;
    for (int a = 0; a < d; ++a) {
      s = s * 6364136223846793005ull + 1442695040888963407ull;
      const double u = static_cast<double>(s >> 11) * (1.0 / 9007199254740992.0) - 0.5;
      const bool wall = k[a] == 0 || k[a] == n - 1;
      c.x[static_cast<size_t>(a) * N + p] = k[a] * dx + (wall ? 0.0 : 0.2 * dx * u);
      if (wall && owner == 0) owner = 2 * a + (k[a] == 0 ? 1 : 2);
    }
    c.wid[p] = owner;
  }
  return c;
}

int check(int rc, const char* what) {
  if (rc != R_OK) {
    std::printf("%s returned %d\n", what, rc);
    return 1;
  }
  return 0;
}

int run(int d, int n, int nv) {
  ref_config c{};
  c.dim = d;
  c.n_particles = d == 2 ? n * n : n * n * n;
  c.nv = nv;
  c.wls_degree = 2;
  c.cap = d == 2 ? 64 : 96;
  c.move = 1;
  c.vmax = 4.0;
  c.dx = 1.0 / (n - 1);
  c.h = (d == 2 ? 2.5 : 2.2) * c.dx;
  c.alpha = 6.0;
  c.kn = 0.8;
  c.dt = 0.5 * c.dx / (std::sqrt(static_cast<double>(d)) * c.vmax);
  c.wall_T = 1.1;
  c.lid = 0.2;
  Cloud cl = cloud(d, n);
  const int N = c.n_particles, nc = d == 2 ? 2 : 1;
  int64_t NV = 1;
  for (int a = 0; a < d; ++a) NV *= nv;
  const size_t F = static_cast<size_t>(nc) * N * NV;
  std::vector<double> rho(N, 1.0), U(static_cast<size_t>(d) * N, 0.0), T(N, 1.0), f(F), f1(F),
      f2(F), fd(F, 0.0), x = cl.x;
  for (int i = 0; i < N; ++i) {
    U[i] = 0.05 * std::sin(7.0 * i);
    T[i] = 1.0 + 0.05 * std::cos(3.0 * i);
  }
  int bad = 0;
  bad += check(ref_maxwellian(&c, rho.data(), U.data(), T.data(), f.data()), "maxwellian");
  for (size_t k = 0; k < F; ++k) fd[k] = 0.01 * f[k] * std::sin(0.37 * k);
  bad += check(ref_moments(&c, f.data(), rho.data(), U.data(), T.data()), "moments");
  std::vector<int32_t> cnt(N), idx(static_cast<size_t>(N) * c.cap), deg(N), wcnt(N),
      widx(static_cast<size_t>(N) * c.cap);
  std::vector<double> grad(static_cast<size_t>(N) * c.cap * d),
      ops(static_cast<size_t>(N) * c.cap * d * d), wc0(static_cast<size_t>(N) * c.cap), hb(N);
  bad += check(ref_neighbors(&c, x.data(), cnt.data(), idx.data()), "neighbors");
  bad += check(ref_wls_operators(&c, x.data(), cl.wid.data(), cnt.data(), idx.data(), grad.data(),
                                 ops.data(), deg.data()), "wls");
  bad += check(ref_wall_stencil(&c, x.data(), cl.wid.data(), wcnt.data(), widx.data(),
                                wc0.data(), hb.data()), "wall_stencil");
  bad += check(ref_transport(&c, cl.wid.data(), cnt.data(), idx.data(), grad.data(), ops.data(),
                             U.data(), f.data(), f1.data()), "transport");
  std::vector<double> r2(rho), U2(U), T2(T);
  bad += check(ref_collide(&c, cl.wid.data(), f1.data(), f2.data(), r2.data(), U2.data(),
                           T2.data()), "collide");
  bad += check(ref_wall_bc(&c, cl.wid.data(), wcnt.data(), widx.data(), wc0.data(), f2.data(),
                           r2.data(), U2.data(), T2.data()), "wall_bc");
  int32_t k = 0;
  std::vector<double> xm(x);
  bad += check(ref_move(&c, cl.wid.data(), U2.data(), xm.data(), &k), "move");
  double sec = 0.0;
  int32_t rows = 0;
  bad += check(ref_step_rows(&c, cl.wid.data(), x.data(), f.data(), U.data(), 0, N, 2, f1.data(),
                             &sec, &rows), "step_rows");
  std::vector<double> xs(x), Us(U), rs(N), Ts(N);
  bad += check(ref_step(&c, cl.wid.data(), xs.data(), f.data(), f1.data(), Us.data(), rs.data(),
                        Ts.data(), &k), "step");
  (void)ref_objective(&c, cl.wid.data(), f1.data(), rs.data(), Us.data(), 1.0);
  std::vector<double> xd(static_cast<size_t>(d) * N, 0.0), x1(xd), x1d(xd), U1(xd), U1d(xd),
      Ud(xd), r1(N), r1d(N), T1(N), T1d(N);
  for (size_t q = 0; q < xd.size(); ++q) xd[q] = (cl.wid[q % N] == 0) ? 1e-3 * std::cos(1.3 * q) : 0;
  bad += check(ref_step_dual_move(&c, cl.wid.data(), x.data(), xd.data(), f.data(), fd.data(),
                                  U.data(), Ud.data(), 0.5, x1.data(), x1d.data(), f1.data(),
                                  f2.data(), U1.data(), U1d.data(), r1.data(), r1d.data(),
                                  T1.data(), T1d.data()), "step_dual_move");
  double J = 0, Jd = 0;
  bad += check(ref_rollout_dual_move(&c, cl.wid.data(), x.data(), xd.data(), f.data(), fd.data(),
                                     1.0, 2, 1.0, &J, &Jd), "rollout_dual_move");
  c.move = 0;
  bad += check(ref_step_dual(&c, cl.wid.data(), x.data(), f.data(), fd.data(), U.data(), nullptr,
                             1.0, f1.data(), f2.data(), U1.data(), U1d.data(), r1.data(),
                             r1d.data(), T1.data(), T1d.data()), "step_dual");
  bad += check(ref_rollout_dual(&c, cl.wid.data(), x.data(), f.data(), fd.data(), 1.0, 2, 1.0, &J,
                                &Jd, f1.data()), "rollout_dual");
  (void)ref_objective_dual(&c, cl.wid.data(), f.data(), fd.data(), rho.data(), nullptr, U.data(),
                           nullptr, 1.0);
  // particle management on a disturbed copy of the cloud
  std::vector<double> xp(x);
  for (int i = 0; i < N; ++i)
    if (cl.wid[i] == 0) xp[i] += (i % 3 == 0 ? 0.4 : -0.3) * c.dx;
  int32_t np = 0, nh = 0;
  bad += check(ref_pm_count(&c, xp.data(), cl.wid.data(), 0.25 * c.dx, 0.45 * c.h, &np, &nh),
               "pm_count");
  const int Nn = N - np + nh;
  std::vector<double> xn(static_cast<size_t>(d) * Nn), fn(static_cast<size_t>(nc) * Nn * NV),
      rn(Nn), Un(static_cast<size_t>(d) * Nn), Tn(Nn);
  std::vector<int32_t> wn(Nn);
  bad += check(ref_pm_apply(&c, xp.data(), cl.wid.data(), f.data(), rho.data(), U.data(),
                            T.data(), 0.25 * c.dx, 0.45 * c.h, xn.data(), wn.data(), fn.data(),
                            rn.data(), Un.data(), Tn.data()), "pm_apply");
  return bad;
}

}  // namespace

int main() {
  int bad = run(2, 9, 6) + run(3, 6, 4);
  if (bad) return 1;
  std::printf("sanitizer driver ok\n");
  return 0;
}
