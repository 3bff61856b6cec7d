"""Gradients of a cavity rollout by the hand-written reverse step.

The rollout is the frozen-cloud map (S4-S7 of every step with the operators
of the fixed cloud, Sec. 3.2 and Sec. 5): (rho, U, T)^0 are the moments of
f^0, then ``nsteps`` steps, then the objective J(f, rho, U) of the final
state (lid heat flux plus weighted kinetic energy, see ``bgk_objective``).

``rollout_objective`` wraps it in a ``torch.autograd.Function``: the forward
pass keeps (f, U) every ``checkpoint_every`` steps; the backward pass walks
the segments in reverse, recomputes each segment's steps with
``bgk_step_keep``, which also keeps what the reverse step reads (f-tilde,
f^{n+1} and the new moments; about two f-sized arrays per step of the
segment), and runs ``bgk_adjoint_step_kept`` over them, accumulating dJ/dlid
on the device.  With ``keep_states=False`` the segment keeps only its
states and every ``bgk_adjoint_step`` recomputes its step (one f-sized
array per step, twice the forward work; the same gradients bit for bit).
All arithmetic runs in libbgk; torch only holds the buffers.
"""
from __future__ import annotations

import torch

from . import bgk as B
from .inputs import cloud_for


def segments(nsteps: int, every: int):
    """Checkpoint segments [(s0, s1), ...] covering steps 0..nsteps-1, in
    forward order; the state at s0 of each segment is stored."""
    if nsteps < 0 or every < 1:
        raise ValueError("nsteps >= 0 and checkpoint_every >= 1 are required")
    return [(s0, min(s0 + every, nsteps)) for s0 in range(0, nsteps, every)]


class FrozenCavity:
    """A cavity on one GPU with a frozen cloud, set up for forward and reverse
    passes (BGK_FLAG_ADJOINT).  precision: "fp64", or "fp32" for FP32
    storage of f and of its adjoint (reductions stay FP64).  x: positions
    [d][N] of the frozen cloud (a torch tensor or numpy array; default the
    workload's initial cloud), e.g. where a moving-cloud run left it."""

    def __init__(self, cav, device="cuda", seed=None, stream=None, precision="fp64", x=None,
                 keep_states=True, **overrides):
        if precision not in ("fp64", "fp32"):
            raise ValueError("the reverse mode runs in fp64 or fp32 storage")
        self.cav = cav
        self.keep_states = bool(keep_states)
        overrides = dict(overrides)
        overrides.update(move=0, flags=overrides.get("flags", 0) | B.BGK_FLAG_ADJOINT)
        self.cfg = B.config_from(cav, precision, **overrides)
        x0, wid = cloud_for(cav, seed)
        dev = torch.device(device)
        self.wall_id = torch.from_numpy(wid).to(dev)
        if x is None:
            self.x = torch.from_numpy(x0).to(dev)
        else:
            self.x = torch.as_tensor(x, dtype=torch.float64).to(dev).contiguous().clone()
            if tuple(self.x.shape) != tuple(x0.shape):
                raise ValueError(f"x must have shape {tuple(x0.shape)}")
        self.ctx = B.bgk_init(self.cfg, self.wall_id, stream)
        B.bgk_geometry(self.ctx, self.x)
        self.N, self.d, self.nc, self.NV = self.ctx.N, self.ctx.d, self.ctx.nc, self.ctx.NV

    def rest_state(self):
        """f^0 = M[1, 0, wall_T] at every particle (Chu: G1, G2)."""
        c = self.ctx
        rho = torch.ones(c.N, dtype=torch.float64, device=c.device)
        U = torch.zeros((c.d, c.N), dtype=torch.float64, device=c.device)
        T = torch.full((c.N,), float(self.cfg.wall_T), dtype=torch.float64, device=c.device)
        return B.bgk_maxwellian(c, rho, U, T)

    def forward(self, f0, lid, nsteps, every=None):
        """Run nsteps from f0 at lid speed ``lid``.  Returns the final state
        (f, rho, U, T) and the (f, U) stored at each segment start."""
        c = self.ctx
        B.bgk_set_lid_velocity(c, float(lid))
        f = f0.detach().clone()
        rho, U, T = B.bgk_moments(c, f)
        fn = torch.empty_like(f)
        starts = {s0 for s0, _ in segments(nsteps, every)} if every else set()
        saved = {}
        for s in range(nsteps):
            if s in starts:
                saved[s] = (f.clone(), U.clone())
            B.bgk_step(c, f, fn, self.x, U, rho, T)
            f, fn = fn, f
        return (f, rho, U, T), saved

    def objective(self, f0, lid, nsteps, ke_weight=1.0):
        """J after nsteps (forward only; a float)."""
        (f, rho, U, _), _ = self.forward(f0, lid, nsteps)
        J = B.bgk_objective(self.ctx, f, rho, U, ke_weight, want_grad=False)
        return float(J.item())


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(actx, f0, lid, problem, nsteps, every, ke_weight):
        (f, rho, U, _), saved = problem.forward(f0, lid, nsteps, every)
        J = B.bgk_objective(problem.ctx, f, rho, U, ke_weight, want_grad=False)
        actx.problem, actx.nsteps, actx.every, actx.ke = problem, nsteps, every, ke_weight
        actx.final = (f, rho, U)
        actx.saved = saved
        actx.lid = float(lid)
        actx.save_for_backward(f0)
        return J

    @staticmethod
    def backward(actx, gJ):
        (f0,) = actx.saved_tensors
        p, c = actx.problem, actx.problem.ctx
        B.bgk_set_lid_velocity(c, actx.lid)
        f, rho, U = actx.final
        _, (gf, grho, gU) = B.bgk_objective(c, f, rho, U, actx.ke, want_grad=True)
        g = gJ.to(torch.float64)
        lam_f, lam_U, lam_rho = gf.mul_(g), gU.mul_(g), grho.mul_(g)
        dlid = torch.zeros(1, dtype=torch.float64, device=c.device)
        first = True  # only the last step's rho, T feed the objective
        for s0, s1 in reversed(segments(actx.nsteps, actx.every)):
            fs, Us = actx.saved[s0]
            if p.keep_states:
                steps = []
                fa, Ua = fs, Us
                for _ in range(s0, s1):
                    fb, ft = torch.empty_like(fa), torch.empty_like(fa)
                    Ub = Ua.clone()  # U^n in, U^{n+1} out
                    rho_t, T_t = torch.empty_like(rho), torch.empty_like(rho)
                    B.bgk_step_keep(c, fa, fb, p.x, Ub, rho_t, T_t, ft)
                    steps.append((fa, Ua, (ft, fb, rho_t, Ub, T_t)))
                    fa, Ua = fb, Ub
                for fn, Un, kept in reversed(steps):
                    B.bgk_adjoint_step_kept(c, fn, Un, p.x, kept, lam_f, lam_U,
                                            lam_rho if first else None, None, lam_f, lam_U, dlid)
                    first = False
                del steps
                continue
            states = [(fs, Us)]
            fa, Ua = fs, Us.clone()
            rho_t = torch.empty_like(rho)
            T_t = torch.empty_like(rho)
            for _ in range(s0, s1 - 1):
                fb = torch.empty_like(fa)
                B.bgk_step(c, fa, fb, p.x, Ua, rho_t, T_t)
                fa = fb
                states.append((fa, Ua.clone()))
            for fn, Un in reversed(states):
                B.bgk_adjoint_step(c, fn, Un, p.x, lam_f, lam_U, lam_rho if first else None,
                                   None, lam_f, lam_U, dlid)
                first = False
            del states
        # (rho, U, T)^0 are the moments of f^0: U^0 enters the first step, and
        # with no steps rho^0 and U^0 enter J itself
        r0, U0, T0 = B.bgk_moments(c, f0)
        B.bgk_moments_adjoint(c, r0, U0, T0, lam_f, lam_rho if actx.nsteps == 0 else None,
                              lam_U, None)
        return lam_f, dlid.reshape(()), None, None, None, None


def rollout_objective(problem: FrozenCavity, f0: torch.Tensor, lid: torch.Tensor, nsteps: int,
                      checkpoint_every: int = 10, ke_weight: float = 1.0) -> torch.Tensor:
    """J of the frozen-cloud rollout from f0 at lid speed ``lid`` (0-d float64
    tensor); differentiable in f0 and lid."""
    if not isinstance(lid, torch.Tensor):
        lid = torch.tensor(float(lid), dtype=torch.float64, device=f0.device)
    return _Rollout.apply(f0, lid, problem, int(nsteps), int(checkpoint_every), float(ke_weight))


class MovingCavity:
    """A cavity on one GPU whose cloud moves with the gas (S8), set up for
    forward and reverse passes through the positions (BGK_FLAG_ADJOINT,
    move = 1).  precision: "fp64" or "fp32" storage of f and its adjoint."""

    def __init__(self, cav, device="cuda", seed=None, stream=None, precision="fp64",
                 **overrides):
        if precision not in ("fp64", "fp32"):
            raise ValueError("the reverse mode runs in fp64 or fp32 storage")
        self.cav = cav
        overrides = dict(overrides)
        overrides.update(move=1, flags=overrides.get("flags", 0) | B.BGK_FLAG_ADJOINT)
        self.cfg = B.config_from(cav, precision, **overrides)
        x, wid = cloud_for(cav, seed)
        dev = torch.device(device)
        self.wall_id = torch.from_numpy(wid).to(dev)
        self.x0 = torch.from_numpy(x).to(dev)
        self.ctx = B.bgk_init(self.cfg, self.wall_id, stream)
        self.N, self.d, self.nc, self.NV = self.ctx.N, self.ctx.d, self.ctx.nc, self.ctx.NV

    def rest_state(self):
        """f^0 = M[1, 0, wall_T] at every particle (Chu: G1, G2)."""
        c = self.ctx
        rho = torch.ones(c.N, dtype=torch.float64, device=c.device)
        U = torch.zeros((c.d, c.N), dtype=torch.float64, device=c.device)
        T = torch.full((c.N,), float(self.cfg.wall_T), dtype=torch.float64, device=c.device)
        return B.bgk_maxwellian(c, rho, U, T)

    def forward(self, f0, lid, nsteps, every=None, x0=None):
        """Run nsteps from (f0, x0) at lid speed ``lid``.  Returns the final
        state (f, rho, U, T, x) and the (f, U, x) stored at each segment
        start."""
        c = self.ctx
        B.bgk_set_lid_velocity(c, float(lid))
        f = f0.detach().clone()
        x = (self.x0 if x0 is None else x0).detach().clone()
        rho, U, T = B.bgk_moments(c, f)
        fn = torch.empty_like(f)
        starts = {s0 for s0, _ in segments(nsteps, every)} if every else set()
        saved = {}
        for s in range(nsteps):
            if s in starts:
                saved[s] = (f.clone(), U.clone(), x.clone())
            B.bgk_step(c, f, fn, x, U, rho, T)
            f, fn = fn, f
        return (f, rho, U, T, x), saved

    def objective(self, f0, lid, nsteps, ke_weight=1.0, x0=None):
        """J after nsteps (forward only; a float)."""
        (f, rho, U, _, _), _ = self.forward(f0, lid, nsteps, x0=x0)
        J = B.bgk_objective(self.ctx, f, rho, U, ke_weight, want_grad=False)
        return float(J.item())


class _RolloutMove(torch.autograd.Function):
    @staticmethod
    def forward(actx, f0, lid, x0, problem, nsteps, every, ke_weight):
        (f, rho, U, _, _), saved = problem.forward(f0, lid, nsteps, every, x0)
        J = B.bgk_objective(problem.ctx, f, rho, U, ke_weight, want_grad=False)
        actx.problem, actx.nsteps, actx.every, actx.ke = problem, nsteps, every, ke_weight
        actx.final = (f, rho, U)
        actx.saved = saved
        actx.lid = float(lid)
        actx.save_for_backward(f0)
        return J

    @staticmethod
    def backward(actx, gJ):
        (f0,) = actx.saved_tensors
        p, c = actx.problem, actx.problem.ctx
        B.bgk_set_lid_velocity(c, actx.lid)
        f, rho, U = actx.final
        _, (gf, grho, gU) = B.bgk_objective(c, f, rho, U, actx.ke, want_grad=True)
        g = gJ.to(torch.float64)
        lam_f, lam_U, lam_rho = gf.mul_(g), gU.mul_(g), grho.mul_(g)
        lam_x = torch.zeros_like(U)          # the objective does not read x
        dlid = torch.zeros(1, dtype=torch.float64, device=c.device)
        first = True  # only the last step's rho feeds the objective
        for s0, s1 in reversed(segments(actx.nsteps, actx.every)):
            fs, Us, xs = actx.saved[s0]
            states = [(fs, Us, xs)]
            fa, Ua, xa = fs, Us.clone(), xs.clone()
            rho_t = torch.empty_like(rho)
            T_t = torch.empty_like(rho)
            for _ in range(s0, s1 - 1):
                fb = torch.empty_like(fa)
                B.bgk_step(c, fa, fb, xa, Ua, rho_t, T_t)
                fa = fb
                states.append((fa, Ua.clone(), xa.clone()))
            for fn, Un, xn in reversed(states):
                B.bgk_adjoint_step_move(c, fn, Un, xn, lam_f, lam_U, lam_x,
                                        lam_rho if first else None, None, lam_f, lam_U, lam_x,
                                        dlid)
                first = False
            del states
        r0, U0, T0 = B.bgk_moments(c, f0)
        B.bgk_moments_adjoint(c, r0, U0, T0, lam_f, lam_rho if actx.nsteps == 0 else None,
                              lam_U, None)
        return lam_f, dlid.reshape(()), lam_x, None, None, None, None


def rollout_objective_move(problem: MovingCavity, f0: torch.Tensor, lid: torch.Tensor,
                           nsteps: int, checkpoint_every: int = 10, ke_weight: float = 1.0,
                           x0: torch.Tensor | None = None) -> torch.Tensor:
    """J of the rollout with the moving cloud from (f0, x0) at lid speed
    ``lid``; differentiable in f0, lid and x0 (the initial positions, default
    the workload's cloud).  Checkpoints hold (f, U, x) every
    checkpoint_every steps; the backward pass recomputes each segment and
    runs bgk_adjoint_step_move over it in reverse."""
    if not isinstance(lid, torch.Tensor):
        lid = torch.tensor(float(lid), dtype=torch.float64, device=f0.device)
    if x0 is None:
        x0 = problem.x0
    return _RolloutMove.apply(f0, lid, x0, problem, int(nsteps), int(checkpoint_every),
                              float(ke_weight))
