"""Pins of the oracle's derivatives through the moving cloud (the reference
for the geometric reverse mode): one full step S1-S8 with the positions,
the least-squares rows, the edge frames, the wall rows and the position
update all carrying a directional derivative (dual numbers), against
central differences of the oracle's plain FP64 step; and the moving-cloud
rollout objective against central differences of plain rollouts.  The
neighbour sets are fixed by the positions' values (a perturbation of 1e-6
moves no particle across h on these clouds, which the agreement itself
confirms).  Sec. 3.2.1 (position update), Sec. 3.4.1 (least squares),
Sec. 3.4.2 (edge frames)."""
import math

import numpy as np
import pytest

import oracle
from paper_2408_02350_amd.inputs import make_cloud


def cfg(dim, n, nv, vmax, **kw):
    dx = 1.0 / (n - 1)
    base = dict(dim=dim, n_particles=n ** dim, nv=nv, wls_degree=2,
                cap=64 if dim == 2 else 96, move=1, vmax=vmax,
                h=(2.5 if dim == 2 else 2.2) * dx, alpha=6.0, kn=0.7,
                dt=0.5 * dx / (math.sqrt(dim) * vmax), wall_T=1.0, lid=0.2, dx=dx)
    base.update(kw)
    return oracle.config(**base)


def with_(c, **kw):
    """A copy of the oracle configuration c with some fields replaced."""
    vals = {name: getattr(c, name) for name, _ in c._fields_}
    vals.update(kw)
    return oracle.config(**vals)


def state(c, x, seed):
    """A positive f near a Maxwellian with a smooth non-zero mean velocity,
    and U its moments."""
    rng = np.random.default_rng(seed)
    N = c.n_particles
    U0 = np.stack([0.3 * np.sin(np.pi * x[1]) * np.sin(np.pi * x[0])] +
                  [0.2 * np.cos(np.pi * x[a]) for a in range(1, c.dim)])
    f = oracle.maxwellian(c, 1.0 + 0.1 * x[0], U0, 1.0 + 0.05 * x[c.dim - 1])
    f = f * rng.uniform(0.95, 1.05, f.shape)
    rho, U, T = oracle.moments(c, f)
    return f, U


def fd_step(c, wid, x, f, U, dx_, df, dU, dlid, eps):
    def at(s):
        ce = with_(c, lid=c.lid + s * eps * dlid)
        x1, f1, U1, r1, T1, _ = oracle.step(ce, wid, x + s * eps * dx_, f + s * eps * df,
                                            U + s * eps * dU)
        return x1, f1, U1, r1, T1
    p, m = at(1), at(-1)
    return [(a - b) / (2 * eps) for a, b in zip(p, m)]


@pytest.mark.parametrize("dim,n,nv,seed", [(2, 9, 6, 0), (3, 6, 4, 1)])
def test_step_tangents_through_the_moving_cloud_match_central_differences(dim, n, nv, seed):
    x, wid = make_cloud(dim, n, seed)
    c = cfg(dim, n, nv, 4.0)
    f, U = state(c, x, seed)
    rng = np.random.default_rng(10 + seed)
    inner = wid == 0
    dxs = rng.normal(size=x.shape) * inner * c.dx      # interior positions only
    dfs = rng.normal(size=f.shape) * f * 0.1
    dUs = rng.normal(size=U.shape) * 0.1
    for name, d_x, d_f, d_U, d_l in (("x", dxs, None, None, 0.0), ("f", None, dfs, None, 0.0),
                                     ("U", None, None, dUs, 0.0), ("lid", None, None, None, 1.0),
                                     ("all", dxs, dfs, dUs, 0.5)):
        x1, x1d, f1, f1d, U1, U1d, r, rd, T, Td = oracle.step_dual_move(
            c, wid, x, f, U, x_dot=d_x, f_dot=d_f, U_dot=d_U, lid_dot=d_l)
        z = lambda a, like: np.zeros_like(like) if a is None else a
        fd = fd_step(c, wid, x, f, U, z(d_x, x), z(d_f, f), z(d_U, U), d_l, 1e-6)
        # central differences carry O(eps^2) truncation and a rounding
        # floor of ~u |value| / eps
        for got, ref, val, what in ((x1d, fd[0], x1, "x"), (f1d, fd[1], f1, "f"),
                                    (U1d, fd[2], U1, "U"), (rd, fd[3], r, "rho"),
                                    (Td, fd[4], T, "T")):
            scale = np.max(np.abs(ref))
            bound = 2e-6 * scale + 4e-16 * np.max(np.abs(val)) / 1e-6
            err = np.max(np.abs(got - ref))
            assert err <= bound, (name, what, err, scale)
        # the positions' own direction moves the operators: the f tangent
        # differs from the frozen-geometry one when x moves
        if name == "x":
            assert np.max(np.abs(f1d)) > 1e-3 * np.max(np.abs(f1))


@pytest.mark.parametrize("dim,n,nv", [(2, 8, 6), (3, 6, 4)])
def test_moving_step_with_still_positions_equals_the_frozen_tangent(dim, n, nv):
    """With no position direction, the f, U, rho, T tangents of the moving
    step equal those of the frozen-cloud dual step bit for bit (the dual
    geometry then carries zero derivatives)."""
    x, wid = make_cloud(dim, n, 3)
    c = cfg(dim, n, nv, 4.0)
    f, U = state(c, x, 3)
    rng = np.random.default_rng(4)
    df = rng.normal(size=f.shape) * f
    dU = rng.normal(size=U.shape) * 0.1
    mv = oracle.step_dual_move(c, wid, x, f, U, f_dot=df, U_dot=dU, lid_dot=0.3)
    fr = oracle.step_dual(with_(c, move=0), wid, x, f, U, f_dot=df, U_dot=dU,
                          lid_dot=0.3)
    for a, b in zip((mv[2], mv[3], mv[4], mv[5], mv[6], mv[7], mv[8], mv[9]), fr):
        assert np.array_equal(a, b)
    # and the new positions are x + dt U^{n+1} with tangent dt U1_dot
    inner = wid == 0
    assert np.array_equal(mv[0][:, inner], x[:, inner] + c.dt * mv[4][:, inner])
    assert np.array_equal(mv[1][:, inner], c.dt * mv[5][:, inner])
    assert np.all(mv[1][:, ~inner] == 0) and np.array_equal(mv[0][:, ~inner], x[:, ~inner])


@pytest.mark.parametrize("dim,n,nv,steps", [(2, 8, 6, 3), (3, 6, 4, 2)])
def test_moving_rollout_derivative_matches_central_differences(dim, n, nv, steps):
    x, wid = make_cloud(dim, n, 5)
    c = cfg(dim, n, nv, 4.0)
    f0, _ = state(c, x, 5)
    rng = np.random.default_rng(6)
    df = rng.normal(size=f0.shape) * f0 * 0.1

    def J_of(cc, f):
        rho, U, T = oracle.moments(cc, f)
        xs, fs, Us, rs, Ts, _ = oracle.run(cc, wid, x, f, U, steps)
        return oracle.objective(cc, wid, fs, rs, Us, 1.0)

    eps = 1e-6
    J, Jl = oracle.rollout_dual_move(c, wid, x, f0, steps, lid_dot=1.0)
    assert abs(J - J_of(c, f0)) <= 1e-13 * abs(J)
    fdl = (J_of(with_(c, lid=c.lid + eps), f0)
           - J_of(with_(c, lid=c.lid - eps), f0)) / (2 * eps)
    assert abs(Jl - fdl) <= 1e-6 * abs(fdl) and abs(fdl) > 1e-6
    _, Jf = oracle.rollout_dual_move(c, wid, x, f0, steps, f0_dot=df)
    fdf = (J_of(c, f0 + eps * df) - J_of(c, f0 - eps * df)) / (2 * eps)
    assert abs(Jf - fdf) <= 1e-6 * abs(fdf)
    # initial positions (interior): the derivative through every step's
    # geometry; eps 1e-7 keeps the perturbed runs on the same neighbour sets
    dxs = rng.normal(size=x.shape) * (wid == 0) * c.dx
    _, Jx = oracle.rollout_dual_move(c, wid, x, f0, steps, x0_dot=dxs)

    def J_at(xx):
        rho, U, T = oracle.moments(c, f0)
        xs, fs, Us, rs, Ts, _ = oracle.run(c, wid, xx, f0, U, steps)
        return oracle.objective(c, wid, fs, rs, Us, 1.0)

    ex = 1e-7
    fdx = (J_at(x + ex * dxs) - J_at(x - ex * dxs)) / (2 * ex)
    assert abs(Jx - fdx) <= 1e-5 * abs(fdx) and abs(fdx) > 1e-8
    # the moving cloud's derivative differs from the frozen cloud's
    _, Jl_frozen, _ = oracle.rollout_dual(with_(c, move=0), wid, x, f0, steps,
                                          lid_dot=1.0)
    assert abs(Jl - Jl_frozen) > 1e-8 * abs(Jl)
