"""Seeded synthetic inputs for the meshfree ALE BGK cavity step.

This module builds the point clouds and the run parameters of the cavity
problems (Section 5: a regular lattice of grid points in the unit square or
cube, at rest, with diffuse walls and a lid moving along +x).  It holds none
of the method's arithmetic: no velocity grid, no Maxwellian, no operators.
Both the GPU path and the CPU oracle take their inputs from here.

Units are nondimensional: length L = 1, velocity sqrt(R T0), so R = 1 and the
wall temperature is 1.

Cloud recipe
------------
* lattice x_k = k * dx, dx = 1/(n-1), particle index p = ix + n*iy (+ n^2*iz);
* jitter drawn as ``numpy.random.default_rng(seed).uniform(-0.1*dx, 0.1*dx,
  size=(N, d))`` in particle order;
* on a node lying on one or more walls, the jitter component normal to each
  of those walls is zeroed, so wall nodes stay on the wall;
* the owner wall of a boundary node is the first of x=0, x=1, y=0, y=1
  (, z=0, z=1) that contains it, numbered 1..2d; interior nodes get 0.  The
  lid is the y=1 wall (2D, id 4) or the z=1 wall (3D, id 6), so it owns only
  the nodes strictly inside its face.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Wall ids, 1-based: 2*axis + (0 for the low face, 1 for the high face) + 1.
LID_WALL = {2: 4, 3: 6}


@dataclasses.dataclass(frozen=True)
class CavityConfig:
    """Run parameters of one cavity workload (all nondimensional)."""

    name: str
    dim: int            # 2 = Chu-reduced BGK (g1, g2), 3 = full BGK
    n: int              # lattice points per axis; N = n**dim particles
    nv: int             # velocity points per axis (both ends included)
    vmax: float         # velocity grid spans [-vmax, vmax] per axis
    h_factor: float     # support radius h = h_factor * dx
    kn: float           # Knudsen number in tau = kn*sqrt(2/pi)/(rho*sqrt(T))
    lid: float          # lid speed along +x
    steps: int          # time steps of the workload
    move: int           # 1 = particles move with the gas, 0 = frozen cloud
    precision: str = "fp64"   # "fp64", "fp32" or "bf16"
    alpha: float = 6.0        # Gaussian weight exponent
    wls_degree: int = 2       # 1 = linear, 2 = quadratic full basis, 0 = first-derivative fit
    wall_T: float = 1.0
    seed: int = 0

    @property
    def n_particles(self) -> int:
        return self.n ** self.dim

    @property
    def n_velocities(self) -> int:
        return self.nv ** self.dim

    @property
    def n_comp(self) -> int:
        return 2 if self.dim == 2 else 1

    @property
    def dx(self) -> float:
        return 1.0 / (self.n - 1)

    @property
    def h(self) -> float:
        return self.h_factor * self.dx

    @property
    def dt(self) -> float:
        # CFL-type choice dt = 0.5 dx / (sqrt(d) vmax); the paper fixes one dt
        # for all resolutions without stating vmax, so it gives no other rule.
        return 0.5 * self.dx / (math.sqrt(self.dim) * self.vmax)

    @property
    def capacity(self) -> int:
        # neighbour-list slots per particle, self included: 64 (2D) / 96 (3D),
        # or for wider supports 1.25x the volume of the h-ball grown by the
        # jitter, in lattice cells, rounded up to 8 (3D at h = 3.1 dx: 208)
        base = 64 if self.dim == 2 else 96
        r = self.h_factor + 0.3
        vol = math.pi * r * r if self.dim == 2 else 4.0 / 3.0 * math.pi * r ** 3
        return min(255, max(base, int(math.ceil(1.25 * vol / 8.0)) * 8))

    def replace(self, **kw) -> "CavityConfig":
        return dataclasses.replace(self, **kw)


# The five cavity workloads: the Chu 2D cavity at CPU-finishable size, the
# 2D cavity at 200^2 x 32^2, the 3D cavity at 32^3 x 16^3 (precision path),
# the 2D differentiation case, and the 3D cavity at 48^3 x 20^3.
CONFIGS = {
    "c1": CavityConfig("c1_2d_chu_40x40_v16", 2, 40, 16, 4.0, 2.5, 1.0, 0.1, 10, 1),
    "c2": CavityConfig("c2_2d_chu_200x200_v32", 2, 200, 32, 5.0, 2.5, 1.0, 0.1, 200, 1),
    "c3": CavityConfig("c3_3d_32cube_v16", 3, 32, 16, 4.0, 2.2, 1.0, 0.1, 100, 1),
    "c4": CavityConfig("c4_2d_chu_100x100_v24_adjoint", 2, 100, 24, 4.0, 2.5, 0.5, 0.1, 50, 0),
    "c5": CavityConfig("c5_3d_48cube_v20", 3, 48, 20, 4.0, 2.2, 1.0, 0.1, 200, 1,
                       precision="fp32"),
}


# The paper's own cavity scales (Sec. 5, Tables 1 and 2): 20 velocity points
# per axis, 200^2..500^2 particles in 2D and 20^3..40^3 in 3D, support
# h = 3.1 dx and the first-derivative least-squares fit as printed
# (Sec. 3.4.1).  v_max is not given there; 4 is taken as for the other
# 20-point grid.  The paper reports whole runs in minutes without the step
# count, so these are timed per step only.
PAPER_SCALES = {
    **{f"p2_{n}": CavityConfig(f"paper_2d_chu_{n}x{n}_v20", 2, n, 20, 4.0, 3.1, 1.0, 0.1, 1, 1,
                               wls_degree=0) for n in (200, 300, 400, 500)},
    **{f"p3_{n}": CavityConfig(f"paper_3d_{n}cube_v20", 3, n, 20, 4.0, 3.1, 1.0, 0.1, 1, 1,
                               wls_degree=0) for n in (20, 30, 40)},
}


def lattice_indices(dim: int, n: int) -> np.ndarray:
    """Integer lattice coordinates [N][dim]; particle p = ix + n*iy (+ n^2*iz)."""
    return _lattice_ix_fastest(dim, n)


def _lattice_ix_fastest(dim: int, n: int) -> np.ndarray:
    p = np.arange(n ** dim, dtype=np.int64)
    out = np.empty((p.size, dim), dtype=np.int64)
    for a in range(dim):
        out[:, a] = (p // (n ** a)) % n
    return out


def make_cloud(dim: int, n: int, seed: int = 0, jitter: float = 0.1):
    """Jittered lattice in the unit box.

    Returns ``(x, wall_id)``: x is float64 [dim][N] (component-major),
    wall_id is int32 [N] (0 interior, 1..2*dim owner wall).
    """
    ijk = _lattice_ix_fastest(dim, n)
    N = ijk.shape[0]
    dx = 1.0 / (n - 1)
    rng = np.random.default_rng(seed)
    jit = rng.uniform(-jitter * dx, jitter * dx, size=(N, dim))
    on_low = ijk == 0
    on_high = ijk == n - 1
    jit[on_low | on_high] = 0.0
    x = ijk.astype(np.float64) * dx + jit
    # wall nodes: exact face coordinates
    x[on_low] = 0.0
    x[on_high] = 1.0
    wall_id = np.zeros(N, dtype=np.int32)
    for p_axis in range(dim):
        for side, mask in ((0, on_low[:, p_axis]), (1, on_high[:, p_axis])):
            wid = 2 * p_axis + side + 1
            take = mask & (wall_id == 0)
            wall_id[take] = wid
    return np.ascontiguousarray(x.T), wall_id


def make_lattice(dim: int, n: int):
    """Unjittered lattice (same layout as make_cloud)."""
    return make_cloud(dim, n, seed=0, jitter=0.0)


def disturbed_cloud(dim: int, n: int, seed: int = 0, amp: float = 0.45, drop: float = 0.2):
    """A cloud as particle management meets it after the particles have
    moved: the jittered lattice with every interior particle displaced by up
    to amp * dx more (uniform per component, kept inside [0.1 dx, 1 - 0.1 dx])
    and a fraction drop of the interior particles removed.  Returns
    (x, wall_id) like make_cloud."""
    x, wid = make_cloud(dim, n, seed)
    x = x.copy()
    dx = 1.0 / (n - 1)
    rng = np.random.default_rng(100 + seed)
    inner = wid == 0
    x[:, inner] += rng.uniform(-amp * dx, amp * dx, (dim, int(inner.sum())))
    np.clip(x, 0.1 * dx, 1 - 0.1 * dx, out=x, where=np.broadcast_to(inner, x.shape))
    keep = ~inner | (rng.uniform(size=wid.size) >= drop)
    return np.ascontiguousarray(x[:, keep]), np.ascontiguousarray(wid[keep])


def cloud_for(cfg: CavityConfig, seed: int | None = None):
    return make_cloud(cfg.dim, cfg.n, cfg.seed if seed is None else seed)


def random_state(shape, seed: int, lo: float = 0.5, hi: float = 1.5) -> np.ndarray:
    """Seeded positive random field, e.g. a perturbation of f for tests."""
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)
