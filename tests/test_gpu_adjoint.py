"""Reverse mode of the frozen-cloud step and of the rollout objective,
through the C interface, against the oracle's exact forward-mode derivatives
(dual numbers) and against central finite differences of the GPU forward.

Per step: for random output adjoints lam and input directions delta,
<lam, J delta> (J delta from the oracle's dual step) must equal
<J^T lam, delta> (J^T lam from bgk_adjoint_step).  The identity is checked
separately for the f, U and lid directions.  For the rollout, the
gradients of rollout_objective must match the oracle's dual rollout and
central differences (eps 1e-6) of the GPU forward.  Checkpoint spacing must
not change a single bit of the gradient.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2408_02350_amd.bgk as bgk
from paper_2408_02350_amd.adjoint import FrozenCavity, rollout_objective
from paper_2408_02350_amd.inputs import CONFIGS, CavityConfig, cloud_for, make_cloud

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)


def cavity(dim, n, nv, vmax=4.0, kn=1.0, lid=0.1):
    return CavityConfig(f"a{dim}d_n{n}_v{nv}", dim, n, nv, vmax, 2.5 if dim == 2 else 2.2, kn,
                        lid, 1, 0)


def t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def smooth_state(c, x, seed):
    """Positive f near a Maxwellian whose (rho, U, T) vary smoothly in x,
    with 5% noise; U^n small and unrelated to f (it is an independent input
    of the step)."""
    rng = np.random.default_rng(seed)
    N = c.n_particles
    ph = rng.uniform(0, 2 * np.pi, 3)
    s = np.sin(2 * np.pi * x[0] + ph[0]) * np.cos(2 * np.pi * x[1] + ph[1])
    rho = 1.0 + 0.2 * s
    T = 1.0 + 0.1 * np.cos(2 * np.pi * x[-1] + ph[2])
    U = 0.08 * np.stack([np.roll(s, k) for k in range(c.dim)])
    f = oracle.maxwellian(c, rho, U, T) * (1 + 0.05 * rng.uniform(-1, 1, (c.nc, N, c.NV)))
    Un = 0.05 * rng.uniform(-1, 1, (c.dim, N))
    return f, Un


class AdjCase:
    def __init__(self, cav, seed=0, precision="fp64", flags=0):
        self.cav = cav
        self.c = oracle.config(cav)
        self.x, self.wid = make_cloud(cav.dim, cav.n, seed)
        cfg = bgk.config_from(cav, precision, flags=bgk.BGK_FLAG_ADJOINT | flags)
        self.fdt = bgk.f_dtype(cfg)
        say(f"adjoint case {cav.name} seed={seed} N={cav.n_particles} NV={cav.n_velocities}")
        self.ctx = bgk.bgk_init(cfg, t(self.wid))
        self.x_t = t(self.x)


def dot(a, b):
    return float(np.sum(np.asarray(a, dtype=np.float64) * np.asarray(b, dtype=np.float64)))


CASES = [(2, 8, 8, 1.0, 0), (2, 11, 6, 0.1, 1), (3, 6, 4, 1.0, 0), (3, 7, 6, 0.5, 2)]
# a velocity grid larger than the reverse relaxation keeps in registers
# (2D FP64: 2 x 2 x 4 values per thread, 2048 velocities per block)
LARGE_NV = [(2, 8, 48, 1.0, 4)]


@pytest.mark.parametrize("dim,n,nv,kn,seed", CASES + LARGE_NV)
def test_adjoint_step_is_the_transpose_of_the_dual_step(dim, n, nv, kn, seed):
    k = AdjCase(cavity(dim, n, nv, kn=kn), seed)
    c = k.c
    f, U = smooth_state(c, k.x, seed)
    rng = np.random.default_rng(100 + seed)
    N = c.n_particles
    lf = rng.normal(size=f.shape)
    lU = rng.normal(size=(c.dim, N))
    lr = rng.normal(size=N)
    lT = rng.normal(size=N)
    dl = t(np.zeros(1))
    lam_f, lam_U = bgk.bgk_adjoint_step(k.ctx, t(f), t(U), k.x_t, t(lf), t(lU), t(lr), t(lT),
                                        dJ_dlid=dl)
    bgk.bgk_check(k.ctx)
    lam_f, lam_U, dlid = lam_f.cpu().numpy(), lam_U.cpu().numpy(), float(dl.item())

    def lhs(out):
        _, f1d, _, U1d, _, rd, _, Td = out
        terms = [lf * f1d, lU * U1d, lr * rd, lT * Td]
        return sum(float(np.sum(v)) for v in terms), sum(float(np.sum(np.abs(v))) for v in terms)

    df = f * rng.normal(size=f.shape)
    dU = 0.1 * rng.normal(size=U.shape)
    for name, kw, rhs in [("f", dict(f_dot=df), dot(lam_f, df)),
                          ("U", dict(U_dot=dU), dot(lam_U, dU)),
                          ("lid", dict(lid_dot=1.0), dlid)]:
        val, scale = lhs(oracle.step_dual(c, k.wid, k.x, f, U, **kw))
        say(f"  {name}: <lam, J d> = {val:.15e}  <J^T lam, d> = {rhs:.15e}")
        assert abs(val - rhs) <= 1e-11 * scale, name
    # wall particles do not move their own U^n into the step
    assert np.all(lam_U[:, k.wid != 0] == 0)


@pytest.mark.parametrize("dim,n,nv,kn,seed", [CASES[0], CASES[2], (3, 6, 10, 1.0, 3),
                                               (2, 8, 68, 1.0, 5), (3, 5, 24, 1.0, 6),
                                               (3, 5, 22, 1.0, 7)])
def test_adjoint_step_fp32_storage_against_the_dual_step(dim, n, nv, kn, seed):
    """FP32 storage of f and of the adjoints (FP32 arithmetic in the reverse
    transport's per-velocity work, FP64 in its lam_U reductions and in the
    other reverse kernels): the transpose identity holds to the FP32
    rounding.  The 10^3 velocity grid takes 5 velocities per lane in the
    interior patches and 2 in the wall kernel (different tile counts).  The
    68^2, 24^3 and 22^3 grids are larger than what the reverse relaxation
    keeps in registers between its passes (4096 velocities per block in 2D,
    8192 in 3D at 4 per group, 8192 at 2 per group), so part of each row is
    gathered a second time."""
    k = AdjCase(cavity(dim, n, nv, kn=kn), seed, precision="fp32")
    c = k.c
    f, U = smooth_state(c, k.x, seed)
    f = f.astype(np.float32).astype(np.float64)     # the state the GPU holds
    rng = np.random.default_rng(200 + seed)
    lf = rng.normal(size=f.shape).astype(np.float32).astype(np.float64)
    lU = rng.normal(size=(c.dim, c.n_particles))
    dl = t(np.zeros(1))
    lam_f, lam_U = bgk.bgk_adjoint_step(k.ctx, t(f).float(), t(U), k.x_t, t(lf).float(), t(lU),
                                        dJ_dlid=dl)
    bgk.bgk_check(k.ctx)
    lam_f, lam_U = lam_f.double().cpu().numpy(), lam_U.cpu().numpy()
    df = f * rng.normal(size=f.shape)
    dU = 0.1 * rng.normal(size=U.shape)
    for name, kw, rhs in [("f", dict(f_dot=df), dot(lam_f, df)),
                          ("U", dict(U_dot=dU), dot(lam_U, dU)),
                          ("lid", dict(lid_dot=1.0), float(dl.item()))]:
        out = oracle.step_dual(c, k.wid, k.x, f, U, **kw)
        terms = [lf * out[1], lU * out[3]]
        val = sum(float(np.sum(v)) for v in terms)
        scale = sum(float(np.sum(np.abs(v))) for v in terms)
        say(f"  fp32 {name}: <lam, J d> = {val:.9e}  <J^T lam, d> = {rhs:.9e}")
        assert abs(val - rhs) <= 1e-5 * scale, name


def test_adjoint_step_in_place_and_deterministic():
    k = AdjCase(cavity(2, 10, 8), 3)
    c = k.c
    f, U = smooth_state(c, k.x, 3)
    rng = np.random.default_rng(7)
    lf, lU = t(rng.normal(size=f.shape)), t(rng.normal(size=U.shape))
    a_f, a_U = bgk.bgk_adjoint_step(k.ctx, t(f), t(U), k.x_t, lf, lU)
    b_f, b_U = bgk.bgk_adjoint_step(k.ctx, t(f), t(U), k.x_t, lf, lU)
    assert torch.equal(a_f, b_f) and torch.equal(a_U, b_U)
    bgk.bgk_adjoint_step(k.ctx, t(f), t(U), k.x_t, lf, lU, lam_f=lf, lam_U=lU)
    bgk.bgk_check(k.ctx)
    assert torch.equal(lf, a_f) and torch.equal(lU, a_U)
    ft = t(f)
    with pytest.raises(bgk.BgkError) as e:   # output over an input
        bgk.bgk_adjoint_step(k.ctx, ft, t(U), k.x_t, lf, lU, lam_f=ft)
    assert e.value.code == bgk.BGK_EINVAL


@pytest.mark.parametrize("dim,n,nv,precision,flags", [
    (2, 10, 8, "fp64", 0), (3, 6, 6, "fp64", 0), (3, 6, 10, "fp32", 0), (2, 9, 8, "fp32", 0),
    (2, 10, 8, "fp64", bgk.BGK_FLAG_GENERIC), (3, 6, 6, "fp64", bgk.BGK_FLAG_GENERIC)])
def test_adjoint_step_kept_is_adjoint_step(dim, n, nv, precision, flags):
    """The reverse step on the state bgk_step_keep kept equals the reverse
    step that recomputes it, bit for bit; the forward step with the kept
    field equals bgk_step, bit for bit (fused and generic transport)."""
    k = AdjCase(cavity(dim, n, nv), 5, precision=precision, flags=flags)
    c = k.c
    f, U = smooth_state(c, k.x, 5)
    dt = torch.float64 if precision == "fp64" else torch.float32
    fn, Un = t(f).to(dt), t(U)
    f1, ft = torch.empty_like(fn), torch.empty_like(fn)
    U1 = Un.clone()
    rho1 = torch.empty(c.n_particles, dtype=torch.float64, device=DEV)
    T1 = torch.empty_like(rho1)
    bgk.bgk_step_keep(k.ctx, fn, f1, k.x_t, U1, rho1, T1, ft)
    g1, gU = torch.empty_like(fn), Un.clone()
    grho, gT = torch.empty_like(rho1), torch.empty_like(rho1)
    bgk.bgk_step(k.ctx, fn, g1, k.x_t, gU, grho, gT)
    bgk.bgk_check(k.ctx)
    assert torch.equal(f1, g1) and torch.equal(U1, gU) and torch.equal(rho1, grho)
    assert torch.equal(T1, gT)
    rng = np.random.default_rng(11)
    lf = t(rng.normal(size=f.shape)).to(dt)
    lU, lr, lT = (t(rng.normal(size=U.shape)), t(rng.normal(size=c.n_particles)),
                  t(rng.normal(size=c.n_particles)))
    d1, d2 = t(np.zeros(1)), t(np.zeros(1))
    a_f, a_U = bgk.bgk_adjoint_step(k.ctx, fn, Un, k.x_t, lf, lU, lr, lT, dJ_dlid=d1)
    b_f, b_U = bgk.bgk_adjoint_step_kept(k.ctx, fn, Un, k.x_t, (ft, f1, rho1, U1, T1), lf, lU,
                                         lr, lT, dJ_dlid=d2)
    bgk.bgk_check(k.ctx)
    assert torch.equal(a_f, b_f) and torch.equal(a_U, b_U) and torch.equal(d1, d2)
    with pytest.raises(bgk.BgkError) as e:   # the kept field over an input of the step
        bgk.bgk_step_keep(k.ctx, fn, f1, k.x_t, U1, rho1, T1, fn)
    assert e.value.code == bgk.BGK_EINVAL
    with pytest.raises(bgk.BgkError) as e:   # an output over a kept input
        bgk.bgk_adjoint_step_kept(k.ctx, fn, Un, k.x_t, (ft, f1, rho1, U1, T1), lf, lU,
                                  lam_f=ft)
    assert e.value.code == bgk.BGK_EINVAL


@pytest.mark.parametrize("dim,n,nv,precision", [(2, 9, 8, "fp64"), (3, 6, 6, "fp32")])
def test_kept_states_give_the_same_gradients(dim, n, nv, precision):
    """The rollout's backward pass with the kept forward states (one forward
    evaluation per step) and with recomputing reverse steps (two): the same
    J and gradients, bit for bit."""
    cav = cavity(dim, n, nv, kn=0.5)
    out = []
    for keep in (True, False):
        prob = FrozenCavity(cav, DEV, seed=1, precision=precision, keep_states=keep)
        f0 = prob.rest_state().requires_grad_(True)
        lid = torch.tensor(0.1, dtype=torch.float64, device=DEV, requires_grad=True)
        J = rollout_objective(prob, f0, lid, 7, 3)
        J.backward()
        out.append((J.item(), f0.grad.clone(), lid.grad.item()))
        del prob
    assert out[0][0] == out[1][0] and out[0][2] == out[1][2]
    assert torch.equal(out[0][1], out[1][1])


def test_adjoint_step_needs_the_adjoint_workspace():
    cav = cavity(2, 8, 4)
    x, wid = make_cloud(2, 8, 0)
    ctx = bgk.bgk_init(bgk.config_from(cav, "fp64"), t(wid))
    f = torch.ones((2, cav.n_particles, cav.n_velocities), dtype=torch.float64, device=DEV)
    U = torch.zeros((2, cav.n_particles), dtype=torch.float64, device=DEV)
    with pytest.raises(bgk.BgkError) as e:
        bgk.bgk_adjoint_step(ctx, f, U, t(x), f.clone())
    assert e.value.code == bgk.BGK_ENOTSUP
    # the flag needs FP64 or FP32 storage
    with pytest.raises(bgk.BgkError):
        bgk.bgk_init(bgk.config_from(cav, "bf16", flags=bgk.BGK_FLAG_ADJOINT), t(wid))


@pytest.mark.parametrize("dim,n,nv", [(2, 9, 8), (3, 5, 6)])
def test_objective_and_its_gradient_match_oracle(dim, n, nv):
    k = AdjCase(cavity(dim, n, nv), 0)
    c = k.c
    f, U = smooth_state(c, k.x, 1)
    rho, U, T = oracle.moments(c, f)
    (J, (gf, gr, gU)) = bgk.bgk_objective(k.ctx, t(f), t(rho), t(U), 0.6)
    bgk.bgk_check(k.ctx)
    Jr = oracle.objective(c, k.wid, f, rho, U, 0.6)
    assert abs(J.item() - Jr) <= 1e-12 * abs(Jr)
    rng = np.random.default_rng(2)
    df, dr, dU = f * rng.normal(size=f.shape), rng.normal(size=rho.shape), rng.normal(size=U.shape)
    for kw, val in [(dict(f_dot=df), dot(gf.cpu(), df)), (dict(rho_dot=dr), dot(gr.cpu(), dr)),
                    (dict(U_dot=dU), dot(gU.cpu(), dU))]:
        ref = oracle.objective_dual(c, k.wid, f, rho, U, ke_weight=0.6, **kw)
        assert abs(val - ref) <= 1e-11 * max(abs(ref), 1e-3 * abs(Jr)), kw.keys()
    # repeated calls give identical bits
    assert bgk.bgk_objective(k.ctx, t(f), t(rho), t(U), 0.6, want_grad=False).item() == J.item()


@pytest.mark.parametrize("dim,n,nv,steps,every", [(2, 10, 8, 5, 2), (3, 6, 6, 3, 2)])
def test_rollout_gradients_match_oracle_dual(dim, n, nv, steps, every):
    cav = cavity(dim, n, nv, kn=0.5)
    prob = FrozenCavity(cav, DEV, seed=0)
    c = oracle.config(cav)
    x, wid = make_cloud(dim, n, 0)
    say(f"rollout {cav.name} steps={steps} every={every}")
    f0 = prob.rest_state()
    rng = np.random.default_rng(4)
    f0n = f0.cpu().numpy() * (1 + 0.05 * rng.uniform(-1, 1, f0.shape))
    f0 = t(f0n).requires_grad_(True)
    lid = torch.tensor(cav.lid, dtype=torch.float64, device=DEV, requires_grad=True)
    J = rollout_objective(prob, f0, lid, steps, every, ke_weight=1.0)
    J.backward()
    delta = f0n * rng.normal(size=f0n.shape)
    Jr, Jd, _ = oracle.rollout_dual(c, wid, x, f0n, steps, f0_dot=delta)
    _, Jl, _ = oracle.rollout_dual(c, wid, x, f0n, steps, lid_dot=1.0)
    say(f"  J {J.item():.15e} vs {Jr:.15e}; dJ/dlid {lid.grad.item():.15e} vs {Jl:.15e}")
    assert abs(J.item() - Jr) <= 1e-12 * abs(Jr)
    assert abs(lid.grad.item() - Jl) <= 1e-10 * abs(Jl)
    g = dot(f0.grad.cpu(), delta)
    assert abs(g - Jd) <= 1e-10 * abs(Jd)


def test_checkpoint_spacing_does_not_change_the_gradient():
    cav = cavity(2, 9, 8, kn=0.5)
    prob = FrozenCavity(cav, DEV, seed=1)
    base = prob.rest_state()
    out = []
    for every in (1, 3, 7, 100):
        f0 = base.clone().requires_grad_(True)
        lid = torch.tensor(0.1, dtype=torch.float64, device=DEV, requires_grad=True)
        J = rollout_objective(prob, f0, lid, 7, every)
        J.backward()
        out.append((J.item(), f0.grad.clone(), lid.grad.item()))
    for J, gf, gl in out[1:]:
        assert J == out[0][0] and gl == out[0][2] and torch.equal(gf, out[0][1])


def test_fp32_storage_rollout_gradients_follow_fp64():
    cav = cavity(2, 16, 12, kn=0.5)
    g = {}
    rng = np.random.default_rng(11)
    delta = None
    for p in ("fp64", "fp32"):
        prob = FrozenCavity(cav, DEV, precision=p)
        f0 = prob.rest_state().requires_grad_(True)
        if delta is None:
            delta = rng.normal(size=tuple(f0.shape))
        lid = torch.tensor(cav.lid, dtype=torch.float64, device=DEV, requires_grad=True)
        J = rollout_objective(prob, f0, lid, 12, 4)
        J.backward()
        g[p] = (J.item(), lid.grad.item(),
                float(np.sum(f0.grad.double().cpu().numpy() * delta)))
    say(f"  fp64 {g['fp64']}\n  fp32 {g['fp32']}")
    for a, b in zip(g["fp32"], g["fp64"]):
        assert abs(a - b) <= 1e-4 * abs(b)


def test_zero_steps_is_the_objective_of_the_initial_moments():
    cav = cavity(2, 8, 8)
    prob = FrozenCavity(cav, DEV)
    c = oracle.config(cav)
    x, wid = make_cloud(2, 8, 0)
    rng = np.random.default_rng(9)
    f0n = prob.rest_state().cpu().numpy() * (1 + 0.1 * rng.uniform(-1, 1, (2, cav.n_particles,
                                                                            cav.n_velocities)))
    f0 = t(f0n).requires_grad_(True)
    J = rollout_objective(prob, f0, 0.1, 0, 1)
    J.backward()
    delta = rng.normal(size=f0n.shape) * f0n
    Jr, Jd, _ = oracle.rollout_dual(c, wid, x, f0n, 0, f0_dot=delta)
    assert abs(J.item() - Jr) <= 1e-12 * abs(Jr)
    assert abs(dot(f0.grad.cpu(), delta) - Jd) <= 1e-10 * abs(Jd)


def test_differentiation_workload_gradients_match_central_differences():
    # the 2D differentiation workload at full size: 100^2 particles, 24^2
    # velocities, Kn 0.5, 50 frozen-cloud steps, checkpoints every 10
    cav = CONFIGS["c4"]
    assert cav.move == 0
    prob = FrozenCavity(cav, DEV)
    say(f"c4 N={cav.n_particles} NV={cav.n_velocities} steps={cav.steps}")
    base = prob.rest_state()
    f0 = base.clone().requires_grad_(True)
    lid = torch.tensor(cav.lid, dtype=torch.float64, device=DEV, requires_grad=True)
    J = rollout_objective(prob, f0, lid, cav.steps, 10)
    J.backward()
    eps = 1e-6
    Jp = prob.objective(base, cav.lid + eps, cav.steps)
    Jm = prob.objective(base, cav.lid - eps, cav.steps)
    fd = (Jp - Jm) / (2 * eps)
    say(f"  dJ/dlid adjoint {lid.grad.item():.12e} central difference {fd:.12e}")
    assert abs(lid.grad.item() - fd) <= 1e-6 * abs(fd)
    rng = np.random.default_rng(0)
    delta = base * t(rng.normal(size=tuple(base.shape)))
    fdf = (prob.objective(base + eps * delta, cav.lid, cav.steps)
           - prob.objective(base - eps * delta, cav.lid, cav.steps)) / (2 * eps)
    g = float(torch.sum(f0.grad * delta).item())
    say(f"  <grad_f0 J, delta> adjoint {g:.12e} central difference {fdf:.12e}")
    assert abs(g - fdf) <= 1e-6 * abs(fdf)


def test_3d_window_after_the_moving_cloud_run():
    """The 48^3 x 20^3 cavity as configured: 200 forward steps with the
    moving cloud (FP32 storage), then the 20-step frozen-cloud window on the
    cloud and state the run reached, with checkpoints every 5 steps, for
    d(lid heat flux)/d(lid speed).  The FP64 window (started from the same
    state) is checked against central differences of its forward (eps
    1e-6), the FP32-storage window against the FP64 one to 1e-4."""
    torch.cuda.empty_cache()
    cav = CONFIGS["c5"]
    say(f"c5 forward N={cav.n_particles} NV={cav.n_velocities} steps={cav.steps} fp32, moving")
    sim = bgk.Simulation(cav, precision="fp32", device=DEV)
    sim.step(cav.steps)
    bgk.bgk_check(sim.ctx)
    x1 = sim.x.clone()
    f1 = sim.f.clone()
    moved = float((x1 - torch.from_numpy(cloud_for(cav)[0]).to(DEV)).abs().max().item())
    say(f"  largest displacement {moved:.3e}, clamped {bgk.bgk_diagnostics(sim.ctx)['clamped']}")
    assert moved > 0
    del sim
    torch.cuda.empty_cache()
    steps = 20
    frozen = cav.replace(move=0)
    prob = FrozenCavity(frozen, DEV, precision="fp64", x=x1)
    base = f1.double()
    f0 = base.clone().requires_grad_(True)
    lid = torch.tensor(cav.lid, dtype=torch.float64, device=DEV, requires_grad=True)
    J = rollout_objective(prob, f0, lid, steps, 5, ke_weight=0.0)
    J.backward()
    g = lid.grad.item()
    del f0, J
    torch.cuda.empty_cache()
    eps = 1e-6
    fd = (prob.objective(base, cav.lid + eps, steps, ke_weight=0.0)
          - prob.objective(base, cav.lid - eps, steps, ke_weight=0.0)) / (2 * eps)
    say(f"  dJ/dlid adjoint {g:.12e} central difference {fd:.12e}")
    assert abs(g - fd) <= 1e-6 * abs(fd)
    del prob, base
    torch.cuda.empty_cache()
    prob = FrozenCavity(frozen, DEV, precision="fp32", x=x1)
    f0 = f1.clone().requires_grad_(True)
    lid = torch.tensor(cav.lid, dtype=torch.float64, device=DEV, requires_grad=True)
    J = rollout_objective(prob, f0, lid, steps, 5, ke_weight=0.0)
    J.backward()
    g32 = lid.grad.item()
    say(f"  dJ/dlid with FP32 storage {g32:.9e}")
    assert abs(g32 - g) <= 1e-4 * abs(g)
    del prob, f0, J, f1
    torch.cuda.empty_cache()


def test_3d_window_lid_gradient_matches_central_differences():
    # the 3D cavity at scale: 48^3 particles, 20^3 velocities, a 20-step
    # frozen-cloud window with checkpoints every 5 steps (FP64 storage)
    torch.cuda.empty_cache()
    cav = CONFIGS["c5"].replace(precision="fp64", move=0)
    prob = FrozenCavity(cav, DEV)
    steps = 20
    say(f"c5 window N={cav.n_particles} NV={cav.n_velocities} steps={steps}")
    base = prob.rest_state()
    f0 = base.clone().requires_grad_(True)
    lid = torch.tensor(cav.lid, dtype=torch.float64, device=DEV, requires_grad=True)
    J = rollout_objective(prob, f0, lid, steps, 5)
    J.backward()
    g = lid.grad.item()
    del f0, J
    torch.cuda.empty_cache()
    eps = 1e-6
    fd = (prob.objective(base, cav.lid + eps, steps)
          - prob.objective(base, cav.lid - eps, steps)) / (2 * eps)
    say(f"  dJ/dlid adjoint {g:.12e} central difference {fd:.12e}")
    assert abs(g - fd) <= 1e-6 * abs(fd)
    del prob, base
    torch.cuda.empty_cache()
    # the same window with FP32 storage of f and of the adjoints
    prob = FrozenCavity(cav, DEV, precision="fp32")
    f0 = prob.rest_state().requires_grad_(True)
    lid = torch.tensor(cav.lid, dtype=torch.float64, device=DEV, requires_grad=True)
    J = rollout_objective(prob, f0, lid, steps, 5)
    J.backward()
    g32 = lid.grad.item()
    say(f"  dJ/dlid with FP32 storage {g32:.9e}")
    assert abs(g32 - g) <= 1e-4 * abs(g)
    del prob, f0, J
    torch.cuda.empty_cache()
