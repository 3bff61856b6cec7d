"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a value the
paper prints, a closed form, an independent library routine (scipy's KD-tree,
numpy's dense least squares), a textbook special case (first-order upwind on a
lattice), an invariant (positivity, conservation, symmetry), or finite
differences.  Together they are chosen so that a dropped term, a wrong sign or
index, or a transposed operand anywhere in the oracle fails at least one.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
from paper_2408_02350_amd.inputs import make_cloud, make_lattice

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def cfg(dim, n, nv, vmax, **kw):
    dx = 1.0 / (n - 1)
    base = dict(dim=dim, n_particles=n ** dim, nv=nv, wls_degree=2,
                cap=64 if dim == 2 else 96, move=1, vmax=vmax,
                h=(2.5 if dim == 2 else 2.2) * dx, alpha=6.0, kn=1.0,
                dt=0.5 * dx / (math.sqrt(dim) * vmax), wall_T=1.0, lid=0.1, dx=dx)
    base.update(kw)
    return oracle.config(**base)


def nodes(c):
    return np.array([oracle.velocity_node(k, c.nv, c.vmax) for k in range(c.nv)])


def grid_velocities(c):
    v = nodes(c)
    q = np.arange(c.NV)
    return np.stack([v[(q // c.nv ** a) % c.nv] for a in range(c.dim)], axis=1)


def geometry(c, x, wid):
    cnt, idx = oracle.neighbors(c, x)
    grad, ops, deg = oracle.wls_operators(c, x, wid, cnt, idx)
    return cnt, idx, grad, ops, deg


# ---------------------------------------------------------------- velocity grid
@pytest.mark.parametrize("nv,vmax", [(16, 4.0), (32, 5.0), (24, 4.0), (20, 4.0)])
def test_velocity_grid_nodes(nv, vmax):
    v = np.array([oracle.velocity_node(k, nv, vmax) for k in range(nv)])
    assert v[0] == -vmax and v[-1] == vmax
    assert np.array_equal(v, -v[::-1])           # exactly antisymmetric
    assert np.allclose(np.diff(v), 2 * vmax / (nv - 1), rtol=1e-14, atol=0)
    assert np.all(v != 0.0)                      # even nv: no zero node, no v.n = 0 ties


# ------------------------------------------------------- Maxwellian: closed forms
@pytest.mark.parametrize("dim,nv", [(2, 64), (3, 48)])
def test_maxwellian_discrete_moments_match_parameters(dim, nv):
    """Closed form: rho, U, T of M[rho, U, T] (Chu: of G1, G2) on a wide grid."""
    N = 4
    c = cfg(dim, 3, nv, 10.0, n_particles=N)
    rng = np.random.default_rng(1)
    rho = rng.uniform(0.5, 2.0, N)
    U = rng.uniform(-0.3, 0.3, (dim, N))
    T = rng.uniform(0.8, 1.2, N)
    f = oracle.maxwellian(c, rho, U, T)
    r2, U2, T2 = oracle.moments(c, f)
    assert np.max(np.abs(r2 - rho) / rho) < 1e-12
    assert np.max(np.abs(U2 - U)) < 1e-12
    assert np.max(np.abs(T2 - T) / T) < 1e-12
    assert f.min() >= 0.0


def test_chu_reduced_maxwellians_are_v3_marginals():
    """G1 = int M dv3 and G2 = int v3^2 M dv3 (Section 2.1), by summing the
    oracle's own 3D Maxwellian over v3 on a wide grid."""
    nv, vmax = 48, 10.0
    c3 = cfg(3, 3, nv, vmax, n_particles=1)
    c2 = cfg(2, 3, nv, vmax, n_particles=1)
    rho, T = 1.3, 0.9
    M3 = oracle.maxwellian(c3, [rho], np.array([[0.2], [-0.1], [0.0]]), [T])[0, 0]
    M3 = M3.reshape(nv, nv, nv)                  # [k3][k2][k1]
    G = oracle.maxwellian(c2, [rho], np.array([[0.2], [-0.1]]), [T])
    v = nodes(c3)
    dv = v[1] - v[0]
    G1 = (M3.sum(axis=0) * dv)
    G2 = ((M3 * (v ** 2)[:, None, None]).sum(axis=0) * dv)
    assert np.max(np.abs(G[0, 0].reshape(nv, nv) - G1)) < 1e-13 * G1.max()
    assert np.max(np.abs(G[1, 0].reshape(nv, nv) - G2)) < 1e-13 * G2.max()
    # and the energy identity (eq. id3) at equilibrium: 3 rho T from g1, g2
    r, U, TT = oracle.moments(c2, G)
    assert abs(TT[0] - T) < 1e-12 and abs(r[0] - rho) < 1e-12


# --------------------------------------------------------------- tau: printed
def test_tau_reproduces_printed_values():
    g = json.load(open(os.path.join(GOLDEN, "tau_argon.json")))
    C = g["constants"]
    for case in g["cases"]:
        tau = oracle.tau_dimensional(case["rho"], C["T0"], C["R"], C["kB"], C["diameter"])
        p = case["tau_printed"]
        half_unit = 0.5 * 10 ** (math.floor(math.log10(p)) - (case["printed_digits"] - 1))
        assert abs(tau - p) <= half_unit, (tau, p)


def test_tau_nondimensional_form_matches_dimensional():
    """tau = Kn sqrt(2/pi)/(rho sqrt(T)) in units L, sqrt(R T0) is the same law
    as eqs. tau/lambda, with Kn = lambda(rho0)/L.  The implied Knudsen numbers
    are the paper's printed 0.11 and 1.1 (for rho0 = 1 and 0.1)."""
    g = json.load(open(os.path.join(GOLDEN, "tau_argon.json")))
    C = g["constants"]
    t0 = C["L"] / math.sqrt(C["R"] * C["T0"])
    tau_dim_1 = oracle.tau_dimensional(1.0, C["T0"], C["R"], C["kB"], C["diameter"])
    kn = (tau_dim_1 / t0) / oracle.tau(1.0, 1.0, 1.0)
    assert round(kn, 2) == 0.11
    for rho, Tfac in [(0.1, 1.0), (0.7, 2.0), (2.0, 0.5)]:
        a = oracle.tau(kn, rho, Tfac) * t0
        b = oracle.tau_dimensional(rho, Tfac * C["T0"], C["R"], C["kB"], C["diameter"])
        assert abs(a - b) < 1e-13 * b
    kn01 = (oracle.tau_dimensional(0.1, C["T0"], C["R"], C["kB"], C["diameter"]) / t0) \
        / oracle.tau(1.0, 1.0, 1.0)
    assert round(kn01, 1) == 1.1


# --------------------------------------------------------------- neighbours
@pytest.mark.parametrize("dim,n,seed", [(2, 40, 0), (2, 40, 1), (3, 12, 0), (3, 12, 2)])
def test_neighbors_match_kdtree(dim, n, seed):
    x, wid = make_cloud(dim, n, seed)
    c = cfg(dim, n, 4, 4.0)
    cnt, idx = oracle.neighbors(c, x)
    tree = cKDTree(x.T)
    for i in range(c.n_particles):
        ref = sorted(tree.query_ball_point(x[:, i], r=c.h))
        assert list(idx[i, :cnt[i]]) == ref


def test_neighbor_overflow_is_reported():
    x, wid = make_cloud(2, 20, 0)
    c = cfg(2, 20, 4, 4.0, cap=8)
    with pytest.raises(oracle.OracleError) as e:
        oracle.neighbors(c, x)
    assert e.value.code == 3


# --------------------------------------------------------------- WLS operators
def _quadratic(dim, rng):
    a0 = rng.normal()
    b = rng.normal(size=dim)
    Cm = rng.normal(size=(dim, dim))
    fun = lambda X: a0 + b @ X + np.einsum("in,ij,jn->n", X, Cm, X)
    grad = lambda xi: b + (Cm + Cm.T) @ xi
    return fun, grad


@pytest.mark.parametrize("dim,n", [(2, 40), (3, 12)])
def test_wls_gradient_reproduces_quadratics(dim, n):
    x, wid = make_cloud(dim, n, 0)
    c = cfg(dim, n, 4, 4.0)
    cnt, idx, grad, ops, deg = geometry(c, x, wid)
    rng = np.random.default_rng(7)
    fun, dfun = _quadratic(dim, rng)
    p = fun(x)
    interior = np.nonzero(wid == 0)[0]
    assert np.all(deg[interior] == 2)
    worst = 0.0
    for i in interior:
        e = np.arange(cnt[i])
        js = idx[i, e]
        est = (grad[i, e, :] * (p[js] - p[i])[:, None]).sum(axis=0)
        worst = max(worst, np.max(np.abs(est - dfun(x[:, i]))))
        assert np.max(np.abs(grad[i, e, :].sum(axis=0))) < 1e-9     # annihilates constants
    assert worst < 1e-9


def _poly_basis(Y, deg):
    d = Y.shape[1]
    cols = [np.ones(len(Y))] + [Y[:, a] for a in range(d)]
    if deg == 2:
        cols += [Y[:, a] * Y[:, b] for a in range(d) for b in range(a, d)]
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("dim,n", [(2, 6), (3, 5)])
def test_wls_matches_dense_weighted_lstsq(dim, n):
    """Brute force: numpy lstsq on sqrt(W) P with the Gaussian weights of eq.
    weight gives the same derivative estimate at every interior particle."""
    x, wid = make_cloud(dim, n, 4)
    c = cfg(dim, n, 4, 4.0)
    cnt, idx, grad, ops, deg = geometry(c, x, wid)
    rng = np.random.default_rng(3)
    fvals = rng.normal(size=c.n_particles)
    for i in np.nonzero(wid == 0)[0]:
        js = idx[i, :cnt[i]]
        Y = (x[:, js] - x[:, i:i + 1]).T / c.h
        w = np.exp(-6.0 * (Y ** 2).sum(axis=1))
        P = _poly_basis(Y, deg[i])
        sw = np.sqrt(w)
        a, *_ = np.linalg.lstsq(sw[:, None] * P, sw * fvals[js], rcond=None)
        ref = a[1:1 + dim] / c.h
        est = (grad[i, :cnt[i], :] * fvals[js][:, None]).sum(axis=0)
        assert np.allclose(est, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


# Degree 0: the least-squares fit as printed in Sec. 3.4.1 (eqs. taylor,
# solution, x/y/z_derivative): unknowns are the first derivatives only, the
# rows of M are the offsets x_j - x_i, b_j = f_j - f_i, no constant column.
@pytest.mark.parametrize("dim,n", [(2, 30), (3, 10)])
def test_first_order_fit_reproduces_linear_functions(dim, n):
    x, wid = make_cloud(dim, n, 2)
    c = cfg(dim, n, 4, 4.0, wls_degree=0, h=3.1 / (n - 1), cap=200)
    cnt, idx, grad, ops, deg = geometry(c, x, wid)
    interior = np.nonzero(wid == 0)[0]
    assert np.all(deg[interior] == 0) and np.all(deg[wid != 0] == 0)
    b = np.random.default_rng(11).normal(size=dim)
    p = b @ x + 0.7
    for i in interior:
        e = np.arange(cnt[i])
        est = (grad[i, e, :] * (p[idx[i, e]] - p[i])[:, None]).sum(axis=0)
        assert np.max(np.abs(est - b)) <= 1e-12 * np.abs(b).max(), i
        # the particle itself has a zero offset: its row is exactly zero
        self_e = e[idx[i, e] == i]
        assert np.all(grad[i, self_e, :] == 0.0)


@pytest.mark.parametrize("dim,n", [(2, 7), (3, 5)])
def test_first_order_fit_matches_dense_weighted_lstsq(dim, n):
    """Brute force on the printed system: minimise sum_j w_j (b_j - M_j a)^2
    with M_j = x_j - x_i (unscaled), b_j = f_j - f_i and the truncated
    Gaussian weight exp(-alpha r^2 / h^2), by numpy lstsq."""
    x, wid = make_cloud(dim, n, 4)
    h = 3.1 / (n - 1)
    c = cfg(dim, n, 4, 4.0, wls_degree=0, h=h, cap=200)
    cnt, idx, grad, ops, deg = geometry(c, x, wid)
    fv = np.random.default_rng(5).normal(size=c.n_particles)
    for i in np.nonzero(wid == 0)[0]:
        js = idx[i, :cnt[i]]
        js = js[js != i]
        M = (x[:, js] - x[:, i:i + 1]).T
        w = np.exp(-6.0 * (M ** 2).sum(axis=1) / h ** 2)
        sw = np.sqrt(w)
        a, *_ = np.linalg.lstsq(sw[:, None] * M, sw * (fv[js] - fv[i]), rcond=None)
        est = (grad[i, :cnt[i], :] * (fv[idx[i, :cnt[i]]] - fv[i])[:, None]).sum(axis=0)
        assert np.allclose(est, a, rtol=1e-10, atol=1e-10 * np.abs(a).max()), i


@pytest.mark.parametrize("dim,n", [(2, 16), (3, 9)])
def test_first_order_fit_equals_linear_fit_on_symmetric_stencils(dim, n):
    """On an unjittered lattice, a stencil that does not reach a wall is
    point-symmetric, so sum_j w_j (x_j - x_i) = 0 and the fitted constant of
    the degree-1 basis decouples: both fits give the same gradient rows."""
    x, wid = make_lattice(dim, n)
    h = 3.1 / (n - 1)
    c0 = cfg(dim, n, 4, 4.0, wls_degree=0, h=h, cap=200)
    c1 = cfg(dim, n, 4, 4.0, wls_degree=1, h=h, cap=200)
    cnt, idx, g0, _, _ = geometry(c0, x, wid)
    _, _, g1, _, deg1 = geometry(c1, x, wid)
    assert np.all(deg1[wid == 0] == 1)
    lo, hi = h + 1e-12, 1.0 - h - 1e-12
    inner = [i for i in np.nonzero(wid == 0)[0] if np.all((x[:, i] > lo) & (x[:, i] < hi))]
    assert len(inner) > 0
    for i in inner:
        m = cnt[i]
        scale = np.abs(g1[i, :m]).max()
        assert np.max(np.abs(g0[i, :m] - g1[i, :m])) <= 1e-12 * scale, i
    # near a wall the stencil is one-sided and the two fits differ
    edge = [i for i in np.nonzero(wid == 0)[0] if np.any(x[:, i] < lo)]
    assert max(np.max(np.abs(g0[i, :cnt[i]] - g1[i, :cnt[i]])) for i in edge) > 1e-3


@pytest.mark.parametrize("dim,n", [(2, 20), (3, 9)])
def test_upwind_vectors_split_gradient_in_edge_frame(dim, n):
    """P + Q (+ R) = g; P is along the edge and carries g.n; Q, R are normal to
    the edge and to each other; in 3D R lies along z x (x_j - x_i)."""
    x, wid = make_cloud(dim, n, 5)
    c = cfg(dim, n, 4, 4.0)
    cnt, idx, grad, ops, deg = geometry(c, x, wid)
    for i in np.nonzero(wid == 0)[0][::3]:
        for e in range(cnt[i]):
            j = idx[i, e]
            if j == i:
                assert np.all(ops[i, e] == 0)
                continue
            g = grad[i, e]
            P, Q = ops[i, e, :dim], ops[i, e, dim:2 * dim]
            R = ops[i, e, 2 * dim:] if dim == 3 else np.zeros(dim)
            dl = x[:, j] - x[:, i]
            nrm = dl / np.linalg.norm(dl)
            s = np.abs(g).max()
            tol = 1e-12 * s   # acos near the poles limits the frame to ~1e-13
            assert np.allclose(P + Q + R, g, atol=tol)
            assert abs(P @ nrm - g @ nrm) < tol
            assert np.linalg.norm(P - (P @ nrm) * nrm) < tol
            assert abs(Q @ nrm) < tol and abs(R @ nrm) < tol
            if dim == 2:
                assert abs(Q @ np.array([-nrm[1], nrm[0]]) - g @ np.array([-nrm[1], nrm[0]])) < tol
            else:
                assert R[2] == 0.0
                zx = np.array([-dl[1], dl[0], 0.0])
                assert np.linalg.norm(np.cross(R, zx)) < tol * np.linalg.norm(zx)
                assert abs(Q @ R) < tol * s


# --------------------------------------------------------------- transport
def _rand_state(c, seed, lo=0.2, hi=1.0, umax=0.3):
    rng = np.random.default_rng(seed)
    f = rng.uniform(lo, hi, (c.nc, c.n_particles, c.NV))
    U = rng.uniform(-umax, umax, (c.dim, c.n_particles))
    return f, U


@pytest.mark.parametrize("dim", [2, 3])
def test_transport_is_first_order_upwind_on_a_lattice(dim):
    """On a lattice with only the 2d axis neighbours in reach (h = 1.2 dx) and
    a linear fit, the positive scheme is the textbook first-order upwind
    scheme, axis by axis."""
    n = 3
    x, wid = make_lattice(dim, n)
    dx = 0.5
    c = cfg(dim, n, 8, 2.0, h=1.2 * dx, wls_degree=1, dt=0.01)
    cnt, idx, grad, ops, deg = geometry(c, x, wid)
    ctr = sum(n ** a for a in range(dim))
    assert wid[ctr] == 0 and cnt[ctr] == 2 * dim + 1 and deg[ctr] == 1
    f, U = _rand_state(c, 11)
    ft = oracle.transport(c, wid, cnt, idx, grad, ops, U, f)
    w = grid_velocities(c) - U[:, ctr][None, :]
    for k in range(c.nc):
        fc = f[k, ctr]
        expect = fc.copy()
        for a in range(dim):
            lo, hi = f[k, ctr - n ** a], f[k, ctr + n ** a]
            expect -= (c.dt / dx) * (np.maximum(w[:, a], 0) * (fc - lo)
                                     + np.minimum(w[:, a], 0) * (hi - fc))
        assert np.allclose(ft[k, ctr], expect, rtol=1e-13, atol=1e-15)


def test_transport_keeps_a_uniform_field_bitwise():
    x, wid = make_cloud(2, 40, 0)
    c = cfg(2, 40, 16, 4.0)
    cnt, idx, grad, ops, deg = geometry(c, x, wid)
    rng = np.random.default_rng(2)
    row = rng.uniform(0.1, 1.0, (c.nc, 1, c.NV))
    f = np.repeat(row, c.n_particles, axis=1)
    _, U = _rand_state(c, 3)
    ft = oracle.transport(c, wid, cnt, idx, grad, ops, U, f)
    assert np.array_equal(ft, f)


@pytest.mark.parametrize("dim,n,nv", [(2, 40, 16), (3, 10, 8)])
def test_transport_is_positive_at_the_configured_dt(dim, n, nv):
    """Every c_ij(v) <= 0 and dt sum |c| <= 1 keep f >= 0 for rough data; a
    dt well above the bound does not."""
    x, wid = make_cloud(dim, n, 1)
    c = cfg(dim, n, nv, 4.0)
    cnt, idx, grad, ops, deg = geometry(c, x, wid)
    f, U = _rand_state(c, 5, lo=0.0, hi=1.0, umax=0.1)
    ft = oracle.transport(c, wid, cnt, idx, grad, ops, U, f)
    assert ft.min() >= 0.0
    c_big = cfg(dim, n, nv, 4.0, dt=4 * c.dt)
    ft_big = oracle.transport(c_big, wid, cnt, idx, grad, ops, U, f)
    assert ft_big.min() < 0.0


@pytest.mark.parametrize("dim,n,nv", [(2, 16, 8), (3, 8, 6)])
def test_transport_is_covariant_under_quarter_turns(dim, n, nv):
    """Rotating the cloud and the velocity grid by 90 degrees about z rotates
    the transported field (the 3D frame keeps b horizontal, which a turn about
    z preserves)."""
    x, wid = make_cloud(dim, n, 3)
    c = cfg(dim, n, nv, 4.0)
    f, U = _rand_state(c, 9)
    xr = x.copy()
    xr[0], xr[1] = 1.0 - x[1], x[0]
    Ur = U.copy()
    Ur[0], Ur[1] = -U[1], U[0]
    q = np.arange(c.NV)
    k = [(q // nv ** a) % nv for a in range(dim)]
    kr = [nv - 1 - k[1], k[0]] + k[2:]
    qr = sum(kr[a] * nv ** a for a in range(dim))
    fr = np.empty_like(f)
    fr[:, :, qr] = f
    g0 = geometry(c, x, wid)
    g1 = geometry(c, xr, wid)
    assert np.array_equal(g0[0], g1[0]) and np.array_equal(g0[1], g1[1])
    ft = oracle.transport(c, wid, *g0[:4], U, f)
    ftr = oracle.transport(c, wid, *g1[:4], Ur, fr)
    assert np.allclose(ftr[:, :, qr], ft, rtol=1e-12, atol=1e-14)


# --------------------------------------------------------------- collision
def _two_maxwellians(c, seed):
    rng = np.random.default_rng(seed)
    N = c.n_particles
    f = 0
    for _ in range(2):
        rho = rng.uniform(0.3, 1.0, N)
        U = rng.uniform(-0.5, 0.5, (c.dim, N))
        T = rng.uniform(0.8, 1.3, N)
        f = f + oracle.maxwellian(c, rho, U, T)
    return f


@pytest.mark.parametrize("dim,nv", [(2, 48), (3, 32)])
def test_collision_conserves_mass_momentum_energy(dim, nv):
    """On a grid wide enough that quadrature is exact to roundoff, the implicit
    relaxation keeps rho, rho U and the energy of a non-equilibrium f."""
    N = 6
    c = cfg(dim, 3, nv, 10.0, n_particles=N, kn=0.3, dt=0.05)
    wid = np.zeros(N, np.int32)
    ft = _two_maxwellians(c, 4)
    fout, rho, U, T = oracle.collide(c, wid, ft)
    r0, U0, T0 = oracle.moments(c, ft)
    r1, U1, T1 = oracle.moments(c, fout)
    assert np.allclose(rho, r0, rtol=1e-14) and np.allclose(T, T0, rtol=1e-14)
    assert np.max(np.abs(r1 - r0) / r0) < 1e-12
    assert np.max(np.abs(U1 - U0)) < 1e-12
    assert np.max(np.abs(T1 - T0) / T0) < 1e-12
    assert np.max(np.abs(fout - ft)) > 1e-3 * np.max(ft)      # it did relax


def test_collision_defect_bounded_by_quadrature_on_config_grid():
    """On the 16^2 / [-4,4] grid the conservation defect equals
    dt/(tau+dt) times the Maxwellian's quadrature defect (exactly)."""
    N = 5
    c = cfg(2, 3, 16, 4.0, n_particles=N, kn=1.0, dt=0.01)
    wid = np.zeros(N, np.int32)
    ft = _two_maxwellians(c, 6)
    fout, rho, U, T = oracle.collide(c, wid, ft)
    r1, U1, T1 = oracle.moments(c, fout)
    M = oracle.maxwellian(c, rho, U, T)
    rM, UM, TM = oracle.moments(c, M)
    tau = np.array([oracle.tau(c.kn, rho[i], T[i]) for i in range(N)])
    fac = c.dt / (tau + c.dt)
    assert np.allclose(r1 - rho, fac * (rM - rho), rtol=1e-8, atol=1e-15)
    assert np.allclose(r1 * U1 - rho * U, fac * (rM * UM - rho * U), rtol=1e-7, atol=1e-15)
    assert np.max(np.abs(rM - rho)) > 1e-7       # the grid's defect is visible here


# --------------------------------------------------------------- walls
def _wall_normal(dim, w):
    axis = (w - 1) // 2
    sign = 1.0 if (w - 1) % 2 == 0 else -1.0
    return axis, sign


def test_wall_bc_zero_net_mass_flux_and_rest_density():
    n = 16
    x, wid = make_cloud(2, n, 2)
    c = cfg(2, n, 16, 4.0)
    wcnt, widx, wc0, hb = oracle.wall_stencil(c, x, wid)
    assert np.all(wcnt[wid != 0] >= 4) and np.all(wcnt[wid == 0] == 0)
    f, _ = _rand_state(c, 8, lo=0.1, hi=1.0)
    N = c.n_particles
    fb, rho, U, T = oracle.wall_bc(c, wid, wcnt, widx, wc0, f, np.ones(N), np.zeros((2, N)),
                                   np.ones(N))
    V = grid_velocities(c)
    for b in np.nonzero(wid)[0]:
        axis, sgn = _wall_normal(2, wid[b])
        vn = sgn * V[:, axis]
        flux = vn * fb[0, b]
        assert abs(flux.sum()) < 1e-13 * np.abs(flux).sum()
        # arriving half is the interpolated interior value
        arr = vn <= 0
        interp = (wc0[b, :wcnt[b], None] * f[0, widx[b, :wcnt[b]]]).sum(axis=0)
        assert np.allclose(fb[0, b, arr], interp[arr], rtol=1e-13)
    # interior at the resting wall Maxwellian: walls reproduce it, rho_w = 1
    f0 = oracle.maxwellian(c, np.ones(N), np.zeros((2, N)), np.ones(N))
    c0 = cfg(2, n, 16, 4.0, lid=0.0)
    fb0, rho0, U0, T0 = oracle.wall_bc(c0, wid, wcnt, widx, wc0, f0, np.ones(N),
                                       np.zeros((2, N)), np.ones(N))
    assert np.allclose(fb0, f0, rtol=1e-12, atol=1e-16)


@pytest.mark.parametrize("dim,n,nv", [(2, 12, 16), (3, 6, 8)])
def test_walls_reproduce_a_rest_maxwellian_at_the_wall_temperature(dim, n, nv):
    """Resting lid, wall temperature T_w = 1.3, interior at M[1, 0, T_w]: the
    arriving half interpolates rows that all hold the same values, the
    zero-mass-flux density of the emitted half is 1 on the symmetric grid,
    and the emitted half is M[1, 0, T_w] (Chu: g2 = T_w g1).  A wall
    Maxwellian taken at T = 1, or a Chu g2 without its factor T_w, fails."""
    Tw = 1.3
    x, wid = make_cloud(dim, n, 3)
    c = cfg(dim, n, nv, 4.0, lid=0.0, wall_T=Tw)
    N = c.n_particles
    walls = wid != 0
    wcnt, widx, wc0, hb = oracle.wall_stencil(c, x, wid)
    fM = oracle.maxwellian(c, np.ones(N), np.zeros((dim, N)), np.full(N, Tw))
    f = fM.copy()
    f[:, walls] = 0.0
    fb, rho, U, T = oracle.wall_bc(c, wid, wcnt, widx, wc0, f, np.ones(N), np.zeros((dim, N)),
                                   np.ones(N))
    assert np.max(np.abs(fb - fM)) <= 1e-13 * fM.max()
    if dim == 2:
        assert np.allclose(fb[1, walls], Tw * fb[0, walls], rtol=1e-13, atol=0)
    rM, UM, TM = oracle.moments(c, fM)
    assert np.allclose(rho[walls], rM[walls], rtol=1e-12, atol=0)
    assert np.allclose(T[walls], TM[walls], rtol=1e-12, atol=0)
    assert np.max(np.abs(U[:, walls])) < 1e-13
    # the discrete moments sit within the quadrature defect of (1, 0, T_w)
    assert np.max(np.abs(T[walls] - Tw)) < 5e-3 and np.max(np.abs(rho[walls] - 1)) < 5e-3
    # the same walls at T_w = 1 give a different emitted half
    c1 = cfg(dim, n, nv, 4.0, lid=0.0, wall_T=1.0)
    fb1, *_ = oracle.wall_bc(c1, wid, wcnt, widx, wc0, f, np.ones(N), np.zeros((dim, N)),
                             np.ones(N))
    assert np.max(np.abs(fb1 - fM)) > 1e-3 * fM.max()


@pytest.mark.parametrize("dim", [2, 3])
def test_motion_clamps_interior_particles_and_never_moves_walls(dim):
    """S8: an interior particle pushed past 1 - 0.1 dx (or below 0.1 dx) ends
    exactly on the bound and is counted once per clamped coordinate; every
    other interior coordinate moves by exactly dt U; wall particles do not
    move whatever their U."""
    n = 8
    x, wid = make_cloud(dim, n, 4)
    c = cfg(dim, n, 4, 4.0)
    N = c.n_particles
    lo, hi = 0.1 * c.dx, 1.0 - 0.1 * c.dx
    rng = np.random.default_rng(5)
    U = rng.uniform(-0.2, 0.2, (dim, N))
    inner = np.nonzero(wid == 0)[0]
    up, down, both = inner[0], inner[-1], inner[len(inner) // 2]
    U[0, up] = (hi + 0.5 * c.dx - x[0, up]) / c.dt
    U[dim - 1, down] = (lo - 0.5 * c.dx - x[dim - 1, down]) / c.dt
    U[0, both] = (lo - 2.0 * c.dx - x[0, both]) / c.dt
    U[1, both] = (hi + 2.0 * c.dx - x[1, both]) / c.dt
    U[:, wid != 0] = 1e3
    x1, k = oracle.move(c, wid, U, x)
    assert k == 4
    assert x1[0, up] == hi and x1[dim - 1, down] == lo
    assert x1[0, both] == lo and x1[1, both] == hi
    assert np.array_equal(x1[:, wid != 0], x[:, wid != 0])
    free = np.zeros((dim, N), bool)
    free[:, inner] = True
    free[0, up] = free[dim - 1, down] = free[0, both] = free[1, both] = False
    assert np.array_equal(x1[free], (x + c.dt * U)[free])
    assert np.all(x1[:, inner] >= lo) and np.all(x1[:, inner] <= hi)


def _value_row_lstsq(x, wid, b, hb, dim):
    """Degree-1 weighted least-squares value row at x_b over the interior
    particles within hb, by numpy's lstsq (None below d+2 points)."""
    js = np.nonzero((wid == 0) & (((x - x[:, b:b + 1]) ** 2).sum(axis=0) <= hb * hb))[0]
    if len(js) < dim + 2:
        return js, None
    Y = (x[:, js] - x[:, b:b + 1]).T / hb
    w = np.sqrt(np.exp(-6.0 * (Y ** 2).sum(axis=1)))
    P = _poly_basis(Y, 1)
    # the value row is the first row of the weighted pseudo-inverse, times w
    pinv = np.linalg.pinv(w[:, None] * P)
    return js, pinv[0] * w


def _radius_by_rule(x, wid, b, h, dim):
    for m in (1.0, 1.5, 2.0):
        js, c0 = _value_row_lstsq(x, wid, b, m * h, dim)
        if c0 is not None and (m == 2.0 or np.abs(c0).sum() <= 8.0):
            return m * h
    return None


@pytest.mark.parametrize("dim", [2, 3])
def test_wall_row_widens_a_degenerate_stencil(dim):
    """A wall particle whose interior particles within h lie almost on one
    line (2D) or plane (3D) parallel to its wall: the linear extrapolation
    to the wall from that stencil amplifies by far more than 8, so the row
    is taken at 1.5h, where it is well conditioned; the row is the lstsq
    value row there."""
    n = 12 if dim == 2 else 8
    x, wid = make_cloud(dim, n, 1)
    c = cfg(dim, n, 4, 4.0)
    x = x.copy()
    b = (n // 2) if dim == 2 else (n // 2 + n * (n // 2))   # inside the low face of the last axis
    assert wid[b] != 0 and x[dim - 1, b] == 0.0
    near = (wid == 0) & (((x - x[:, b:b + 1]) ** 2).sum(axis=0) <= c.h ** 2)
    rng = np.random.default_rng(3)
    # flatten the interior stencil at h onto the first interior layer
    x[dim - 1, near] = c.dx * (1.0 + 1e-4 * rng.uniform(-1, 1, near.sum()))
    js, c0h = _value_row_lstsq(x, wid, b, c.h, dim)
    assert c0h is not None and np.abs(c0h).sum() > 100.0
    wcnt, widx, wc0, hb = oracle.wall_stencil(c, x, wid)
    assert hb[b] == 1.5 * c.h
    js, c0 = _value_row_lstsq(x, wid, b, 1.5 * c.h, dim)
    assert np.array_equal(widx[b, :wcnt[b]], js)
    assert np.allclose(wc0[b, :wcnt[b]], c0, rtol=1e-9, atol=1e-12)
    assert np.abs(wc0[b, :wcnt[b]]).sum() <= 8.0


@pytest.mark.parametrize("dim,n", [(2, 16), (3, 8)])
def test_wall_interpolation_rows_are_linear_lstsq_values(dim, n):
    x, wid = make_cloud(dim, n, 6)
    c = cfg(dim, n, 4, 4.0)
    wcnt, widx, wc0, hb = oracle.wall_stencil(c, x, wid)
    rng = np.random.default_rng(1)
    fv = rng.normal(size=c.n_particles)
    for b in np.nonzero(wid)[0]:
        js = widx[b, :wcnt[b]]
        assert np.all(wid[js] == 0) and np.all(np.diff(js) > 0)
        cb = wc0[b, :wcnt[b]]
        assert abs(cb.sum() - 1) < 1e-12
        assert np.allclose(cb @ x[:, js].T, x[:, b], atol=1e-12)
        Y = (x[:, js] - x[:, b:b + 1]).T / hb[b]
        w = np.exp(-6.0 * (Y ** 2).sum(axis=1))
        P = _poly_basis(Y, 1)
        a, *_ = np.linalg.lstsq(np.sqrt(w)[:, None] * P, np.sqrt(w) * fv[js], rcond=None)
        assert abs(cb @ fv[js] - a[0]) < 1e-11 * max(1, abs(a[0]))
        # radius rule: the first of h, 1.5h, 2h holding d+2 interior points
        # whose row amplifies by at most 8 (the 2h row without the bound)
        assert hb[b] == _radius_by_rule(x, wid, b, c.h, dim)


# --------------------------------------------------------------- full steps
@pytest.mark.parametrize("dim,n,nv,vmax,steps", [(2, 12, 48, 10.0, 8), (3, 6, 24, 9.0, 2)])
def test_rest_state_with_resting_walls_stays_fixed(dim, n, nv, vmax, steps):
    x, wid = make_cloud(dim, n, 0)
    c = cfg(dim, n, nv, vmax, lid=0.0)
    f0, rho, U, T = oracle.initial_state(c)
    x1, f1, U1, rho1, T1, k = oracle.run(c, wid, x, f0, U, steps)
    assert np.max(np.abs(f1 - f0)) < 1e-12 * f0.max()
    assert np.max(np.abs(U1)) < 1e-13
    assert np.max(np.abs(x1 - x)) < 1e-14


@pytest.mark.parametrize("dim,n,nv", [(2, 10, 8), (3, 6, 6)])
def test_mirror_symmetry_of_full_steps(dim, n, nv):
    """Reflecting x -> 1 - x, v1 -> -v1 and the lid speed maps the discrete
    cavity onto itself (the edge frames are reflection-covariant up to the
    sign of t or b, which the dissipation does not see)."""
    x, wid = make_lattice(dim, n)
    c = cfg(dim, n, nv, 4.0)
    cm = cfg(dim, n, nv, 4.0, lid=-c.lid)
    N = c.n_particles
    p = np.arange(N)
    ix = p % n
    perm = p - ix + (n - 1 - ix)                  # mirror partner of each particle
    xm = np.empty_like(x)
    xm[:, perm] = x
    xm[0, perm] = 1.0 - x[0]
    widm = np.empty_like(wid)
    swap = {0: 0, 1: 2, 2: 1}
    widm[perm] = [swap.get(w, w) for w in wid]
    assert np.array_equal(widm, wid)
    q = np.arange(c.NV)
    k1 = q % nv
    qm = q - k1 + (nv - 1 - k1)
    f0, rho, U, T = oracle.initial_state(c)
    f0m = np.empty_like(f0)
    f0m[:, perm[:, None], qm[None, :]] = f0
    Um = np.empty_like(U)
    Um[:, perm] = U
    Um[0, perm] = -U[0]
    steps = 3
    xa, fa, Ua, *_ = oracle.run(c, wid, x, f0, U, steps)
    xb, fb, Ub, *_ = oracle.run(cm, wid, xm, f0m, Um, steps)
    assert np.allclose(fb[:, perm[:, None], qm[None, :]], fa, rtol=1e-11, atol=1e-15)
    assert np.allclose(Ub[0, perm], -Ua[0], atol=1e-13)
    assert np.allclose(xb[0, perm], 1.0 - xa[0], atol=1e-13)
    assert np.max(np.abs(Ua[0])) > 1e-4          # the lid did drive a flow


def test_lid_drives_flow_and_config_dt_keeps_f_positive():
    from paper_2408_02350_amd.inputs import CONFIGS, cloud_for
    cf = CONFIGS["c1"]
    c = oracle.config(cf)
    x, wid = cloud_for(cf)
    f0, rho, U, T = oracle.initial_state(c)
    x1, f1, U1, rho1, T1, k = oracle.run(c, wid, x, f0, U, 3)
    assert f1.min() > 0
    lid = wid == 4
    assert np.all(U1[0, lid] > 0.02)
    assert k == 0
    # particles in the row below the lid are carried along +x by the gas
    below = (wid == 0) & (np.arange(c.n_particles) // cf.n == cf.n - 2)
    assert np.all(U1[0, below] > 0) and np.all(x1[0, below] > x[0, below])
    assert np.all(x1[:, wid != 0] == x[:, wid != 0])


@pytest.mark.parametrize("dim,n,nv", [(2, 12, 8), (3, 7, 6)])
def test_row_sample_equals_the_full_step_rows(dim, n, nv):
    """The timing sample (neighbour, least-squares, transport and relaxation
    rows of a window of particles) computes the sampled interior rows of
    f^{n+1} exactly as the full step does, on one thread and on several."""
    x, wid = make_cloud(dim, n, 2)
    c = cfg(dim, n, nv, 4.0)
    f0, *_ = oracle.initial_state(c)
    rng = np.random.default_rng(4)
    f = f0 * rng.uniform(0.8, 1.2, f0.shape)
    rho, U, T = oracle.moments(c, f)
    _, f1, *_ = oracle.step(c, wid, x, f, U)
    i0, i1 = n + 3, c.n_particles - n - 5
    rows = [i for i in range(i0, i1) if wid[i] == 0]
    for threads in (1, 3):
        fs, sec, nr = oracle.step_rows(c, wid, x, f, U, i0, i1, threads)
        assert nr == len(rows) and sec > 0
        assert np.array_equal(fs[:, rows], f1[:, rows])


# --------------------------------------------------------------- dual numbers
def test_dual_directional_derivative_matches_central_differences():
    n = 8
    x, wid = make_cloud(2, n, 0)
    c = cfg(2, n, 8, 4.0, move=0, kn=0.5)
    f0, *_ = oracle.initial_state(c)
    rng = np.random.default_rng(12)
    df = rng.normal(size=f0.shape) * f0 * 0.1
    steps = 3
    J, Jd, _ = oracle.rollout_dual(c, wid, x, f0, steps, f0_dot=df)
    eps = 1e-6
    Jp, *_ = oracle.rollout_dual(c, wid, x, f0 + eps * df, steps)
    Jm, *_ = oracle.rollout_dual(c, wid, x, f0 - eps * df, steps)
    fd = (Jp - Jm) / (2 * eps)
    assert abs(Jd - fd) < 1e-6 * abs(fd) + 1e-12
    _, Jl, _ = oracle.rollout_dual(c, wid, x, f0, steps, lid_dot=1.0)
    cp = cfg(2, n, 8, 4.0, move=0, kn=0.5, lid=c.lid + eps)
    cm = cfg(2, n, 8, 4.0, move=0, kn=0.5, lid=c.lid - eps)
    fdl = (oracle.rollout_dual(cp, wid, x, f0, steps)[0]
           - oracle.rollout_dual(cm, wid, x, f0, steps)[0]) / (2 * eps)
    assert abs(Jl - fdl) < 1e-6 * abs(fdl)
    assert abs(Jl) > 1e-6


# --------------------------------------------------------------- objective
def _heat_flux_state(c, a, U=None):
    """f = M[1, 0, 1] (1 + a w_n (|w|^2 - 5)) in 3D, w = v, n the last axis;
    in 2D its Chu reduction g1 = int f dv3 = M2 (1 + a w_n (|w|^2 - 4)),
    g2 = int v3^2 f dv3 = M2 (1 + a w_n (|w|^2 - 2)).  The perturbation has
    zero density, momentum and energy, and the exact heat flux along n is
    q_n = 1/2 E[w_n^2 |w|^2 (|w|^2 - 5)] a = (35 - 25) a / 2 = 5 a."""
    N = c.n_particles
    rho = np.ones(N)
    U = np.zeros((c.dim, N)) if U is None else U
    M = oracle.maxwellian(c, rho, U, np.ones(N))
    v = oracle.velocities(c)
    w2 = np.sum(v ** 2, axis=1)
    wn = v[:, c.dim - 1]
    if c.dim == 3:
        return M * (1 + a * wn * (w2 - 5))[None, None, :]
    f = M.copy()
    f[0] *= (1 + a * wn * (w2 - 4))[None, :]
    f[1] *= (1 + a * wn * (w2 - 2))[None, :]
    return f


@pytest.mark.parametrize("dim,nv,vmax", [(2, 48, 7.0), (3, 32, 7.0)])
def test_objective_heat_flux_of_a_hermite_perturbation(dim, nv, vmax):
    # closed form: every lid particle carries q_n = 5a, weighted by dx^(d-1)
    n = 4
    c = cfg(dim, n, nv, vmax)
    _, wid = make_cloud(dim, n, 0)
    a = 0.01
    f = _heat_flux_state(c, a)
    rho, U, T = oracle.moments(c, f)
    assert np.max(np.abs(U)) < 1e-9 and np.max(np.abs(rho - 1)) < 1e-9
    J = oracle.objective(c, wid, f, rho, U, ke_weight=0.0)
    n_lid = int(np.sum(wid == 2 * dim))
    exact = c.dx ** (dim - 1) * n_lid * 5 * a
    assert abs(J - exact) < 1e-6 * exact  # quadrature (grid truncation at vmax)
    # at U = 0 the flux is odd in a: the state with -a gives -J
    Z = np.zeros_like(U)
    Jp = oracle.objective(c, wid, f, rho, Z, ke_weight=0.0)
    Jm = oracle.objective(c, wid, _heat_flux_state(c, -a), rho, Z, ke_weight=0.0)
    assert abs(Jp + Jm) < 1e-12 * exact


@pytest.mark.parametrize("dim", [2, 3])
def test_objective_is_frame_invariant_and_counts_kinetic_energy(dim):
    # a drifting Maxwellian has no heat flux in its own frame; J is then the
    # kinetic-energy term alone: ke/N sum rho |U|^2 / 2
    n = 4
    c = cfg(dim, n, 24 if dim == 2 else 16, 7.0)
    _, wid = make_cloud(dim, n, 0)
    N = c.n_particles
    rng = np.random.default_rng(3)
    U0 = rng.uniform(-0.3, 0.3, (dim, N))
    r0 = rng.uniform(0.5, 1.5, N)
    f = oracle.maxwellian(c, r0, U0, np.ones(N))
    rho, U, T = oracle.moments(c, f)
    # (quadrature error only; a lab-frame flux would be O(rho |U| T))
    assert abs(oracle.objective(c, wid, f, rho, U, ke_weight=0.0)) < 1e-7 * c.dx ** (dim - 1)
    ke = 0.7
    J = oracle.objective(c, wid, f, rho, U, ke_weight=ke)
    J0 = oracle.objective(c, wid, f, rho, U, ke_weight=0.0)
    expect = ke / N * np.sum(0.5 * rho * np.sum(U ** 2, axis=0))
    assert abs((J - J0) - expect) < 1e-12 * expect


def test_step_and_objective_tangents_match_central_differences():
    n = 8
    x, wid = make_cloud(2, n, 1)
    c = cfg(2, n, 8, 4.0, move=0, kn=0.5)
    f0, rho0, U0, T0 = oracle.initial_state(c)
    rng = np.random.default_rng(5)
    f = f0 * (1 + 0.05 * rng.uniform(-1, 1, f0.shape))
    U = 0.05 * rng.uniform(-1, 1, U0.shape)
    df = f0 * rng.normal(size=f0.shape)
    dU = rng.normal(size=U0.shape) * 0.1
    dl = 0.7
    out = oracle.step_dual(c, wid, x, f, U, df, dU, dl)
    eps = 1e-6

    def run(s):
        cs = cfg(2, n, 8, 4.0, move=0, kn=0.5, lid=c.lid + s * dl)
        return oracle.step_dual(cs, wid, x, f + s * df, U + s * dU)

    p, m = run(eps), run(-eps)
    for k in (0, 2, 4, 6):  # f1, U1, rho, T
        fd = (p[k] - m[k]) / (2 * eps)
        assert np.max(np.abs(out[k + 1] - fd)) < 1e-7 * np.max(np.abs(fd)), k
    # the tangent of the lid alone is non-trivial
    assert np.max(np.abs(oracle.step_dual(c, wid, x, f, U, lid_dot=1.0)[1])) > 1e-6
    f1, _, U1, _, r1, _, T1, _ = out
    dr = rng.normal(size=r1.shape)
    d1 = oracle.objective_dual(c, wid, f1, r1, U1, df, dr, dU, ke_weight=0.5)
    fd = (oracle.objective(c, wid, f1 + eps * df, r1 + eps * dr, U1 + eps * dU, 0.5)
          - oracle.objective(c, wid, f1 - eps * df, r1 - eps * dr, U1 - eps * dU, 0.5)) / (2 * eps)
    assert abs(d1 - fd) < 1e-7 * abs(fd)
