"""CPU FP64 oracle of the meshfree ALE BGK step -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import this package.  It wraps ``liboracle.so``
(built from ``bgk_oracle.cpp`` by ``oracle/build.py``) with ctypes and takes
plain numpy arrays; it imports nothing from the GPU package.

Layouts (same as the library's public interface):
  x, U       float64 [d][N]
  f          float64 [n_c][N][N_v], velocity index k1 + nv*k2 (+ nv^2*k3)
  nbr idx    int32   [N][cap] (first cnt[i] entries used, ascending)
  grad       float64 [N][cap][d]
  ops        float64 [N][cap][d*d]  (P, Q[, R]) per edge
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB, build_oracle

_lib = None

STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "ENBR_OVERFLOW", 4: "ESINGULAR",
          5: "ENONPHYS", 7: "ENOTSUP"}


class OracleError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"oracle {where}: {STATUS.get(code, code)}")
        self.code = code


class RefConfig(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("n_particles", ctypes.c_int32), ("nv", ctypes.c_int32),
        ("wls_degree", ctypes.c_int32), ("cap", ctypes.c_int32), ("move", ctypes.c_int32),
        ("vmax", ctypes.c_double), ("h", ctypes.c_double), ("alpha", ctypes.c_double),
        ("kn", ctypes.c_double), ("dt", ctypes.c_double), ("wall_T", ctypes.c_double),
        ("lid", ctypes.c_double), ("dx", ctypes.c_double),
    ]

    @property
    def nc(self) -> int:
        return 2 if self.dim == 2 else 1

    @property
    def NV(self) -> int:
        return self.nv ** self.dim


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_oracle(force=True)
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        cp = ctypes.POINTER(RefConfig)
        L.ref_num_threads.restype = ctypes.c_int
        L.ref_velocity_node.restype = ctypes.c_double
        L.ref_velocity_node.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double]
        L.ref_velocity_weight.restype = ctypes.c_double
        L.ref_velocity_weight.argtypes = [cp]
        L.ref_tau.restype = ctypes.c_double
        L.ref_tau.argtypes = [ctypes.c_double] * 3
        L.ref_tau_dimensional.restype = ctypes.c_double
        L.ref_tau_dimensional.argtypes = [ctypes.c_double] * 5
        L.ref_maxwellian.argtypes = [cp, dp, dp, dp, dp]
        L.ref_moments.argtypes = [cp, dp, dp, dp, dp]
        L.ref_neighbors.argtypes = [cp, dp, ip, ip]
        L.ref_wls_operators.argtypes = [cp, dp, ip, ip, ip, dp, dp, ip]
        L.ref_wall_stencil.argtypes = [cp, dp, ip, ip, ip, dp, dp]
        L.ref_transport.argtypes = [cp, ip, ip, ip, dp, dp, dp, dp, dp]
        L.ref_collide.argtypes = [cp, ip, dp, dp, dp, dp, dp]
        L.ref_wall_bc.argtypes = [cp, ip, ip, ip, dp, dp, dp, dp, dp]
        L.ref_move.argtypes = [cp, ip, dp, dp, ip]
        L.ref_step.argtypes = [cp, ip, dp, dp, dp, dp, dp, dp, ip]
        L.ref_step_rows.argtypes = [cp, ip, dp, dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    dp, dp, ip]
        L.ref_objective.restype = ctypes.c_double
        L.ref_objective.argtypes = [cp, ip, dp, dp, dp, ctypes.c_double]
        L.ref_rollout_dual.argtypes = [cp, ip, dp, dp, dp, ctypes.c_double, ctypes.c_int,
                                       ctypes.c_double, dp, dp, dp]
        L.ref_step_dual.argtypes = [cp, ip, dp, dp, dp, dp, dp, ctypes.c_double,
                                    dp, dp, dp, dp, dp, dp, dp, dp]
        L.ref_step_dual_move.argtypes = [cp, ip, dp, dp, dp, dp, dp, dp, ctypes.c_double,
                                         dp, dp, dp, dp, dp, dp, dp, dp, dp, dp]
        L.ref_rollout_dual_move.argtypes = [cp, ip, dp, dp, dp, dp, ctypes.c_double, ctypes.c_int,
                                            ctypes.c_double, dp, dp]
        L.ref_objective_dual.restype = ctypes.c_double
        L.ref_objective_dual.argtypes = [cp, ip, dp, dp, dp, dp, dp, dp, ctypes.c_double]
        L.ref_pm_count.argtypes = [cp, dp, ip, ctypes.c_double, ctypes.c_double, ip, ip]
        L.ref_pm_apply.argtypes = [cp, dp, ip, dp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                   dp, ip, dp, dp, dp, dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _check(rc: int, where: str):
    if rc != 0:
        raise OracleError(rc, where)


def config(cfg=None, **kw) -> RefConfig:
    """Build a RefConfig from an object with the cavity attributes
    (dim, n_particles, nv, wls_degree, capacity, move, vmax, h, alpha, kn,
    dt, wall_T, lid, dx) and/or keyword overrides."""
    vals = {}
    if cfg is not None:
        vals = dict(dim=cfg.dim, n_particles=cfg.n_particles, nv=cfg.nv,
                    wls_degree=cfg.wls_degree, cap=cfg.capacity, move=cfg.move,
                    vmax=cfg.vmax, h=cfg.h, alpha=cfg.alpha, kn=cfg.kn, dt=cfg.dt,
                    wall_T=cfg.wall_T, lid=cfg.lid, dx=cfg.dx)
    vals.update(kw)
    c = RefConfig()
    for k, v in vals.items():
        setattr(c, k, v)
    return c


def num_threads() -> int:
    return lib().ref_num_threads()


def velocity_node(k, nv, vmax):
    return lib().ref_velocity_node(k, nv, vmax)


def velocity_weight(c):
    return lib().ref_velocity_weight(ctypes.byref(c))


def velocities(c) -> np.ndarray:
    """[NV][d] velocity vectors in grid order (via the oracle's node rule)."""
    nodes = np.array([velocity_node(k, c.nv, c.vmax) for k in range(c.nv)])
    q = np.arange(c.NV)
    return np.stack([nodes[(q // c.nv ** a) % c.nv] for a in range(c.dim)], axis=1)


def tau(kn, rho, T):
    return lib().ref_tau(kn, rho, T)


def tau_dimensional(rho, T, R, kb, diam):
    return lib().ref_tau_dimensional(rho, T, R, kb, diam)


def maxwellian(c, rho, U, T):
    N = c.n_particles
    f = np.empty((c.nc, N, c.NV))
    rho, U, T = _f64(rho), _f64(U), _f64(T)
    _check(lib().ref_maxwellian(ctypes.byref(c), _d(rho), _d(U), _d(T), _d(f)), "maxwellian")
    return f


def moments(c, f):
    N = c.n_particles
    f = _f64(f)
    rho, U, T = np.empty(N), np.zeros((c.dim, N)), np.empty(N)
    _check(lib().ref_moments(ctypes.byref(c), _d(f), _d(rho), _d(U), _d(T)), "moments")
    return rho, U, T


def initial_state(c):
    """f0 = M[1, 0, 1] (Chu: G1, G2) at every particle; (rho, U, T)0 = its moments."""
    N = c.n_particles
    f0 = maxwellian(c, np.ones(N), np.zeros((c.dim, N)), np.full(N, c.wall_T))
    rho, U, T = moments(c, f0)
    return f0, rho, U, T


def neighbors(c, x):
    N = c.n_particles
    x = _f64(x)
    cnt = np.zeros(N, np.int32)
    idx = np.zeros((N, c.cap), np.int32)
    _check(lib().ref_neighbors(ctypes.byref(c), _d(x), _i(cnt), _i(idx)), "neighbors")
    return cnt, idx


def wls_operators(c, x, wall_id, cnt, idx):
    N = c.n_particles
    x, wall_id, cnt, idx = _f64(x), _i32(wall_id), _i32(cnt), _i32(idx)
    grad = np.zeros((N, c.cap, c.dim))
    ops = np.zeros((N, c.cap, c.dim * c.dim))
    deg = np.zeros(N, np.int32)
    _check(lib().ref_wls_operators(ctypes.byref(c), _d(x), _i(wall_id), _i(cnt), _i(idx),
                                   _d(grad), _d(ops), _i(deg)), "wls_operators")
    return grad, ops, deg


def wall_stencil(c, x, wall_id):
    N = c.n_particles
    x, wall_id = _f64(x), _i32(wall_id)
    wcnt = np.zeros(N, np.int32)
    widx = np.zeros((N, c.cap), np.int32)
    wc0 = np.zeros((N, c.cap))
    hb = np.zeros(N)
    _check(lib().ref_wall_stencil(ctypes.byref(c), _d(x), _i(wall_id), _i(wcnt), _i(widx),
                                  _d(wc0), _d(hb)), "wall_stencil")
    return wcnt, widx, wc0, hb


def pm_count(c, x, wall_id, merge_radius, hole_radius):
    """Particle management plan: (merged pairs, hole particles)."""
    x, wall_id = _f64(x), _i32(wall_id)
    n_pairs = np.zeros(1, np.int32)
    n_holes = np.zeros(1, np.int32)
    _check(lib().ref_pm_count(ctypes.byref(c), _d(x), _i(wall_id), float(merge_radius),
                              float(hole_radius), _i(n_pairs), _i(n_holes)), "pm_count")
    return int(n_pairs[0]), int(n_holes[0])


def pm_apply(c, x, wall_id, f, merge_radius, hole_radius, rho=None, U=None, T=None):
    """The managed cloud: (x_new [d][N'], wall_id_new [N'], f_new [n_c][N'][N_v],
    rho_new, U_new [d][N'], T_new).  rho, U, T of the old cloud default to
    its moments."""
    pairs, holes = pm_count(c, x, wall_id, merge_radius, hole_radius)
    Nn = c.n_particles - pairs + holes
    x, wall_id, f = _f64(x), _i32(wall_id), _f64(f)
    if rho is None:
        rho, U, T = moments(c, f)
    rho, U, T = _f64(rho), _f64(U), _f64(T)
    xn = np.zeros((c.dim, Nn))
    wn = np.zeros(Nn, np.int32)
    fn = np.zeros((c.nc, Nn, c.NV))
    rn, Un, Tn = np.zeros(Nn), np.zeros((c.dim, Nn)), np.zeros(Nn)
    _check(lib().ref_pm_apply(ctypes.byref(c), _d(x), _i(wall_id), _d(f), _d(rho), _d(U), _d(T),
                              float(merge_radius), float(hole_radius), _d(xn), _i(wn), _d(fn),
                              _d(rn), _d(Un), _d(Tn)), "pm_apply")
    return xn, wn, fn, rn, Un, Tn


def transport(c, wall_id, cnt, idx, grad, ops, U, f):
    wall_id, cnt, idx = _i32(wall_id), _i32(cnt), _i32(idx)
    grad, ops, U, f = _f64(grad), _f64(ops), _f64(U), _f64(f)
    ft = np.empty_like(f)
    _check(lib().ref_transport(ctypes.byref(c), _i(wall_id), _i(cnt), _i(idx), _d(grad),
                               _d(ops), _d(U), _d(f), _d(ft)), "transport")
    return ft


def collide(c, wall_id, ft, rho=None, U=None, T=None):
    """Relax interior rows of ft; wall rows (and their rho, U, T) are copied."""
    N = c.n_particles
    wall_id, ft = _i32(wall_id), _f64(ft)
    fout = ft.copy()
    rho = np.zeros(N) if rho is None else _f64(rho).copy()
    U = np.zeros((c.dim, N)) if U is None else _f64(U).copy()
    T = np.zeros(N) if T is None else _f64(T).copy()
    _check(lib().ref_collide(ctypes.byref(c), _i(wall_id), _d(ft), _d(fout), _d(rho), _d(U),
                             _d(T)), "collide")
    return fout, rho, U, T


def wall_bc(c, wall_id, wcnt, widx, wc0, f, rho, U, T):
    wall_id, wcnt, widx, wc0 = _i32(wall_id), _i32(wcnt), _i32(widx), _f64(wc0)
    f, rho, U, T = _f64(f).copy(), _f64(rho).copy(), _f64(U).copy(), _f64(T).copy()
    _check(lib().ref_wall_bc(ctypes.byref(c), _i(wall_id), _i(wcnt), _i(widx), _d(wc0), _d(f),
                             _d(rho), _d(U), _d(T)), "wall_bc")
    return f, rho, U, T


def move(c, wall_id, U, x):
    x = _f64(x).copy()
    k = ctypes.c_int32(0)
    _check(lib().ref_move(ctypes.byref(c), _i(_i32(wall_id)), _d(_f64(U)), _d(x),
                          ctypes.byref(k)), "move")
    return x, k.value


def step(c, wall_id, x, f, U):
    """One step S1..S8. Returns (x_new, f_new, U_new, rho, T, clamped)."""
    N = c.n_particles
    wall_id = _i32(wall_id)
    x, U = _f64(x).copy(), _f64(U).copy()
    f = _f64(f)
    fout = np.empty_like(f)
    rho, T = np.zeros(N), np.zeros(N)
    k = ctypes.c_int32(0)
    _check(lib().ref_step(ctypes.byref(c), _i(wall_id), _d(x), _d(f), _d(fout), _d(U), _d(rho),
                          _d(T), ctypes.byref(k)), "step")
    return x, fout, U, rho, T, k.value


def step_rows(c, wall_id, x, f, U, i0, i1, threads=0):
    """Timing sample of one step's per-particle work (S1-S6) for the interior
    particles among i0..i1-1 on `threads` threads (0: all).  Returns
    (f_out, seconds, rows): f_out [n_c][N][N_v] holds f^{n+1} on the sampled
    rows only (other rows are left uninitialised)."""
    f, U, x = _f64(f), _f64(U), _f64(x)
    fout = np.empty_like(f)
    sec = ctypes.c_double(0.0)
    nr = ctypes.c_int32(0)
    _check(lib().ref_step_rows(ctypes.byref(c), _i(_i32(wall_id)), _d(x), _d(f), _d(U),
                               int(i0), int(i1), int(threads), _d(fout), ctypes.byref(sec),
                               ctypes.byref(nr)), "step_rows")
    return fout, sec.value, nr.value


def run(c, wall_id, x, f, U, nsteps):
    rho = T = None
    clamped = 0
    for _ in range(nsteps):
        x, f, U, rho, T, k = step(c, wall_id, x, f, U)
        clamped += k
    return x, f, U, rho, T, clamped


def objective(c, wall_id, f, rho, U, ke_weight=1.0):
    return lib().ref_objective(ctypes.byref(c), _i(_i32(wall_id)), _d(_f64(f)), _d(_f64(rho)),
                               _d(_f64(U)), ke_weight)


def rollout_dual(c, wall_id, x, f0, nsteps, f0_dot=None, lid_dot=0.0, ke_weight=1.0,
                 want_final=False):
    """Frozen-cloud rollout; returns (J, dJ along (f0_dot, lid_dot), f_final|None)."""
    f0 = _f64(f0)
    fd = _f64(f0_dot) if f0_dot is not None else None
    J, Jd = ctypes.c_double(0), ctypes.c_double(0)
    ff = np.empty_like(f0) if want_final else None
    _check(lib().ref_rollout_dual(ctypes.byref(c), _i(_i32(wall_id)), _d(_f64(x)), _d(f0),
                                  _d(fd) if fd is not None else None, lid_dot, nsteps, ke_weight,
                                  ctypes.byref(J), ctypes.byref(Jd),
                                  _d(ff) if ff is not None else None), "rollout_dual")
    return J.value, Jd.value, ff


def step_dual(c, wall_id, x, f, U, f_dot=None, U_dot=None, lid_dot=0.0):
    """One frozen-cloud step with tangents. Returns (f1, f1_dot, U1, U1_dot,
    rho, rho_dot, T, T_dot)."""
    N = c.n_particles
    f, U = _f64(f), _f64(U)
    fd = _f64(f_dot) if f_dot is not None else None
    Ud = _f64(U_dot) if U_dot is not None else None
    f1, f1d = np.empty_like(f), np.empty_like(f)
    U1, U1d = np.zeros((c.dim, N)), np.zeros((c.dim, N))
    r, rd, T, Td = np.zeros(N), np.zeros(N), np.zeros(N), np.zeros(N)
    _check(lib().ref_step_dual(ctypes.byref(c), _i(_i32(wall_id)), _d(_f64(x)), _d(f),
                               _d(fd) if fd is not None else None, _d(U),
                               _d(Ud) if Ud is not None else None, lid_dot, _d(f1), _d(f1d),
                               _d(U1), _d(U1d), _d(r), _d(rd), _d(T), _d(Td)), "step_dual")
    return f1, f1d, U1, U1d, r, rd, T, Td


def step_dual_move(c, wall_id, x, f, U, x_dot=None, f_dot=None, U_dot=None, lid_dot=0.0):
    """One step S1..S8 of the moving cloud (c.move = 1) with tangents through
    the geometry.  Returns (x1, x1_dot, f1, f1_dot, U1, U1_dot, rho, rho_dot,
    T, T_dot)."""
    N = c.n_particles
    x, f, U = _f64(x), _f64(f), _f64(U)
    keep = [_f64(v) if v is not None else None for v in (x_dot, f_dot, U_dot)]
    a = lambda v: _d(v) if v is not None else None
    x_dot, f_dot, U_dot = keep
    x1, x1d = np.zeros((c.dim, N)), np.zeros((c.dim, N))
    f1, f1d = np.empty_like(f), np.empty_like(f)
    U1, U1d = np.zeros((c.dim, N)), np.zeros((c.dim, N))
    r, rd, T, Td = np.zeros(N), np.zeros(N), np.zeros(N), np.zeros(N)
    wall_id = _i32(wall_id)
    _check(lib().ref_step_dual_move(ctypes.byref(c), _i(wall_id), _d(x), a(x_dot), _d(f),
                                    a(f_dot), _d(U), a(U_dot), float(lid_dot), _d(x1), _d(x1d),
                                    _d(f1), _d(f1d), _d(U1), _d(U1d), _d(r), _d(rd), _d(T),
                                    _d(Td)), "step_dual_move")
    return x1, x1d, f1, f1d, U1, U1d, r, rd, T, Td


def rollout_dual_move(c, wall_id, x0, f0, nsteps, f0_dot=None, lid_dot=0.0, ke_weight=1.0,
                      x0_dot=None):
    """Moving-cloud rollout (c.move = 1); returns (J, dJ along (x0_dot,
    f0_dot, lid_dot))."""
    J, Jd = ctypes.c_double(0), ctypes.c_double(0)
    x0, f0, wall_id = _f64(x0), _f64(f0), _i32(wall_id)
    fd = _f64(f0_dot) if f0_dot is not None else None
    xd = _f64(x0_dot) if x0_dot is not None else None
    _check(lib().ref_rollout_dual_move(ctypes.byref(c), _i(wall_id), _d(x0),
                                       _d(xd) if xd is not None else None,
                                       _d(f0), _d(fd) if fd is not None else None,
                                       float(lid_dot), int(nsteps),
                                       float(ke_weight), ctypes.byref(J), ctypes.byref(Jd)),
           "rollout_dual_move")
    return J.value, Jd.value


def objective_dual(c, wall_id, f, rho, U, f_dot=None, rho_dot=None, U_dot=None, ke_weight=1.0):
    """Directional derivative of objective() along (f_dot, rho_dot, U_dot)."""
    a = lambda v: _d(_f64(v)) if v is not None else None
    return lib().ref_objective_dual(ctypes.byref(c), _i(_i32(wall_id)), _d(_f64(f)), a(f_dot),
                                    _d(_f64(rho)), a(rho_dot), _d(_f64(U)), a(U_dot), ke_weight)
