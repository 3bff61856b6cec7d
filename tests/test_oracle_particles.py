"""Pins of the oracle's particle management (Sec. 3.5.2, adding and removing
points): planted clusters and holes with known outcomes, the merge rule on a
three-point cluster, and exact reproduction of linear fields at new points
(the degree-1 least-squares value fit reproduces them)."""
import math

import numpy as np
import pytest

import oracle
from paper_2408_02350_amd.inputs import make_cloud, make_lattice


def cfg(dim, n, nv=4, h_factor=None, **kw):
    dx = 1.0 / (n - 1)
    hf = h_factor or (2.5 if dim == 2 else 2.2)
    base = dict(dim=dim, n_particles=n ** dim, nv=nv, wls_degree=2, cap=64 if dim == 2 else 96,
                move=1, vmax=4.0, h=hf * dx, alpha=6.0, kn=1.0,
                dt=0.5 * dx / (math.sqrt(dim) * 4.0), wall_T=1.0, lid=0.1, dx=dx)
    base.update(kw)
    return oracle.config(**base)


def linear_field(c, x, seed):
    """f_c(x, v) = a_cv + b_cv . x for every component and velocity."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(1.0, 2.0, (c.nc, 1, c.NV))
    b = rng.uniform(-1.0, 1.0, (c.nc, c.dim, c.NV))
    return lambda X: a + np.einsum("cav,an->cnv", b, X)


def node_index(ijk, n):
    return sum(int(k) * n ** a for a, k in enumerate(ijk))


def lattice_pos(ijk, dx):
    return np.array([k * dx for k in ijk])


def drop(x, wid, keep):
    return np.ascontiguousarray(x[:, keep]), np.ascontiguousarray(wid[keep])


@pytest.mark.parametrize("dim,n", [(2, 16), (3, 8)])
def test_undisturbed_cloud_is_unchanged(dim, n):
    x, wid = make_cloud(dim, n, 1)
    c = cfg(dim, n)
    f = np.random.default_rng(2).uniform(0.1, 1.0, (c.nc, c.n_particles, c.NV))
    rm, rh = 0.25 * c.dx, 0.45 * c.h
    assert oracle.pm_count(c, x, wid, rm, rh) == (0, 0)
    xn, wn, fn, *_ = oracle.pm_apply(c, x, wid, f, rm, rh)
    assert np.array_equal(xn, x) and np.array_equal(wn, wid) and np.array_equal(fn, f)


@pytest.mark.parametrize("dim,n", [(2, 14), (3, 8)])
def test_planted_close_pair_merges_to_midpoint(dim, n):
    x, wid = make_lattice(dim, n)
    x = x.copy()
    c = cfg(dim, n)
    N = c.n_particles
    mid = [n // 2] * dim
    i = node_index(mid, n)
    j = i + 1                                  # the +x lattice neighbour
    assert wid[i] == 0 and wid[j] == 0
    x[:, j] = x[:, i]
    x[0, j] += 0.1 * c.dx                      # 0.1 dx from i
    rm, rh = 0.25 * c.dx, 0.45 * c.h
    assert oracle.pm_count(c, x, wid, rm, rh) == (1, 0)
    field = linear_field(c, x, 3)
    f = field(x)
    xn, wn, fn, *_ = oracle.pm_apply(c, x, wid, f, rm, rh)
    keep = [p for p in range(N) if p not in (i, j)]
    assert xn.shape == (dim, N - 1)
    assert np.array_equal(xn[:, :-1], x[:, keep]) and np.array_equal(wn[:-1], wid[keep])
    assert np.array_equal(fn[:, :-1], f[:, keep])
    xm = 0.5 * (x[:, i] + x[:, j])
    assert np.array_equal(xn[:, -1], xm) and wn[-1] == 0
    ref = field(xm[:, None])[:, 0]
    assert np.max(np.abs(fn[:, -1] - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("dim,n,rh_dx", [(2, 14, None), (3, 10, 1.5)])
def test_planted_hole_gets_a_particle_at_its_node(dim, n, rh_dx):
    """Remove the 3^d block of lattice particles around a node: only the
    block's centre node is farther than hole_radius from every particle
    left (2 dx against 1 dx for the others)."""
    x, wid = make_lattice(dim, n)
    c0 = cfg(dim, n)
    centre = [n // 2] * dim
    block = set()
    for off in np.ndindex(*([3] * dim)):
        block.add(node_index([k + o - 1 for k, o in zip(centre, off)], n))
    keep = [p for p in range(c0.n_particles) if p not in block]
    xk, wk = drop(x, wid, keep)
    c = cfg(dim, n, n_particles=len(keep))
    rh = 0.45 * c.h if rh_dx is None else rh_dx * c.dx
    assert rh > c.dx
    assert oracle.pm_count(c, xk, wk, 0.25 * c.dx, rh) == (0, 1)
    field = linear_field(c, xk, 4)
    f = field(xk)
    xn, wn, fn, *_ = oracle.pm_apply(c, xk, wk, f, 0.25 * c.dx, rh)
    assert xn.shape == (dim, len(keep) + 1)
    assert np.array_equal(xn[:, :-1], xk) and np.array_equal(fn[:, :-1], f)
    y = lattice_pos(centre, c.dx)
    assert np.array_equal(xn[:, -1], y) and wn[-1] == 0
    ref = field(y[:, None])[:, 0]
    assert np.max(np.abs(fn[:, -1] - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_three_point_cluster_merges_only_the_mutual_nearest_pair():
    """i, j, k on a line 0.10 dx and 0.15 dx apart: j is i's nearest and i is
    j's, k's nearest is j: exactly (i, j) merge; k stays."""
    n, dim = 14, 2
    x, wid = make_lattice(dim, n)
    x = x.copy()
    c = cfg(dim, n)
    i = node_index([6, 6], n)
    j, k = i + 1, i + 2
    x[:, j] = x[:, i] + np.array([0.10 * c.dx, 0.0])
    x[:, k] = x[:, j] + np.array([0.15 * c.dx, 0.0])
    rm, rh = 0.25 * c.dx, 0.45 * c.h
    assert oracle.pm_count(c, x, wid, rm, rh) == (1, 0)
    xn, *_ = oracle.pm_apply(c, x, wid, np.ones((c.nc, c.n_particles, c.NV)), rm, rh)
    assert np.array_equal(xn[:, -1], 0.5 * (x[:, i] + x[:, j]))
    assert any(np.array_equal(xn[:, q], x[:, k]) for q in range(xn.shape[1] - 1))
    # with k moved to 0.05 dx beyond j, j's nearest is k and k's is j: now
    # (j, k) is the mutual pair and i stays, although it is within the
    # merge radius of j
    x[:, k] = x[:, j] + np.array([0.05 * c.dx, 0.0])
    assert oracle.pm_count(c, x, wid, rm, rh) == (1, 0)
    xn, *_ = oracle.pm_apply(c, x, wid, np.ones((c.nc, c.n_particles, c.NV)), rm, rh)
    assert np.array_equal(xn[:, -1], 0.5 * (x[:, j] + x[:, k]))


def test_wall_particles_are_never_merged():
    n, dim = 12, 2
    x, wid = make_lattice(dim, n)
    x = x.copy()
    c = cfg(dim, n)
    b = node_index([5, 0], n)                  # bottom wall
    i = node_index([5, 1], n)
    assert wid[b] != 0 and wid[i] == 0
    x[:, i] = x[:, b] + np.array([0.0, 0.05 * c.dx])
    assert oracle.pm_count(c, x, wid, 0.25 * c.dx, 0.45 * c.h) == (0, 0)


@pytest.mark.parametrize("dim,n", [(2, 14), (3, 8)])
def test_state_of_kept_and_new_particles(dim, n):
    """Kept particles carry the rho, U, T given to them (U^n feeds the next
    transport); a new particle in a uniform Maxwellian field gets exactly
    that Maxwellian (the fit reproduces constants) and so its moments."""
    x, wid = make_lattice(dim, n)
    x = x.copy()
    c = cfg(dim, n)
    N = c.n_particles
    i = node_index([n // 2] * dim, n)
    x[:, i + 1] = x[:, i] + np.eye(dim)[0] * 0.1 * c.dx
    rho0 = np.full(N, 0.9)
    U0 = np.zeros((dim, N))
    U0[0] = 0.05
    T0 = np.full(N, 1.1)
    f = oracle.maxwellian(c, rho0, U0, T0)
    mr, mU, mT = oracle.moments(c, f)
    rng = np.random.default_rng(9)
    rho_in, U_in, T_in = rng.uniform(0.5, 1.5, N), rng.uniform(-0.1, 0.1, (dim, N)), \
        rng.uniform(0.5, 1.5, N)
    rm, rh = 0.25 * c.dx, 0.45 * c.h
    xn, wn, fn, rn, Un, Tn = oracle.pm_apply(c, x, wid, f, rm, rh, rho_in, U_in, T_in)
    keep = [p for p in range(N) if p not in (i, i + 1)]
    assert np.array_equal(rn[:-1], rho_in[keep]) and np.array_equal(Tn[:-1], T_in[keep])
    assert np.array_equal(Un[:, :-1], U_in[:, keep])
    assert np.max(np.abs(fn[:, -1] - f[:, i])) <= 1e-12 * np.max(np.abs(f))
    assert abs(rn[-1] - mr[i]) <= 1e-12 and abs(Tn[-1] - mT[i]) <= 1e-12
    assert np.max(np.abs(Un[:, -1] - mU[:, i])) <= 1e-12
