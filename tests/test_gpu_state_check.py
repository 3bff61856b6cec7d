"""bgk_state_check (the per-step health of a state) through the C interface:
the smallest value of f, the counts of negative and non-finite values, the
residuals of f's own moments against the step's rho, U, T, and the totals
of mass, momentum and energy, against the same quantities formed on the host
from the oracle's moments and numpy (sums in another order: 1e-12
relative)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2408_02350_amd.bgk as bgk
from paper_2408_02350_amd.inputs import CONFIGS, CavityConfig, make_cloud

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def host_check(c, f, rho, U, T):
    r, u, t = oracle.moments(c, f)
    fin = f[np.isfinite(f)]
    return {"min_f": float(fin.min()), "negatives": int((fin < 0).sum()),
            "nonfinite": int((~np.isfinite(f)).sum()),
            "rho_residual": float(np.max(np.abs(r - rho) / rho)),
            "U_residual": float(np.max(np.abs(u - U))),
            "T_residual": float(np.max(np.abs(t - T) / T)),
            "mass": float(rho.sum()), "momentum": list((rho * U).sum(axis=1)),
            "energy": float((0.5 * rho * ((U * U).sum(axis=0) + 3.0 * T)).sum())}


def compare(g, h, rtol):
    assert g["negatives"] == h["negatives"] and g["nonfinite"] == h["nonfinite"]
    assert g["min_f"] == pytest.approx(h["min_f"], rel=rtol, abs=0)
    for k in ("rho_residual", "U_residual", "T_residual"):
        assert abs(g[k] - h[k]) <= 1e-12 + rtol * abs(h[k]), k
    for k in ("mass", "energy"):
        assert g[k] == pytest.approx(h[k], rel=1e-12), k
    for a, b in zip(g["momentum"], h["momentum"]):
        assert abs(a - b) <= 1e-12 * h["mass"]


@pytest.mark.parametrize("name,precision,steps", [("c1", "fp64", 5), ("c3s", "fp32", 3)])
def test_state_check_after_steps(name, precision, steps):
    """After steps of a moving cavity: no negative or non-finite value, the
    moments of f^{n+1} differ from the step's moments (those of f-tilde) only
    by the relaxation's quadrature defect (small but not zero on the
    interior, zero to rounding on the wall rows, whose moments are taken
    from f^{n+1} itself), and every figure matches the host's."""
    cav = CONFIGS["c1"] if name == "c1" else CavityConfig("t3d_n8_v8", 3, 8, 8, 4.0, 2.2, 1.0,
                                                          0.1, 1, 1)
    sim = bgk.Simulation(cav.replace(precision=precision), precision=precision, device=DEV)
    sim.step(steps)
    g = bgk.bgk_state_check(sim.ctx, sim.f, sim.rho, sim.U, sim.T)
    c = oracle.config(cav)
    f = sim.f.double().cpu().numpy()
    h = host_check(c, f, sim.rho.cpu().numpy(), sim.U.cpu().numpy(), sim.T.cpu().numpy())
    print(f"  {name} {precision}: {g}", flush=True)
    compare(g, h, 1e-12 if precision == "fp64" else 1e-6)
    assert g["negatives"] == 0 and g["nonfinite"] == 0 and g["min_f"] > 0
    assert 0 < g["rho_residual"] < 1e-3


def test_state_check_flags_negative_and_nonfinite_values():
    """A state with planted negative values and a NaN and an Inf: the counts
    are exact, the minimum is over the finite values, and a non-finite row
    makes the residuals NaN."""
    cav = CONFIGS["c1"]
    c = oracle.config(cav)
    x, wid = make_cloud(cav.dim, cav.n, 0)
    ctx = bgk.bgk_init(bgk.config_from(cav, "fp64"), torch.from_numpy(wid).to(DEV))
    f, rho, U, T = oracle.initial_state(c)
    rng = np.random.default_rng(4)
    f = f * rng.uniform(0.9, 1.1, f.shape)
    idx = rng.choice(f.size, 7, replace=False)
    f.reshape(-1)[idx[:5]] = -rng.uniform(1e-6, 1e-3, 5)
    f.reshape(-1)[idx[5]] = np.nan
    f.reshape(-1)[idx[6]] = np.inf
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    g = bgk.bgk_state_check(ctx, t(f), t(rho), t(U), t(T))
    assert g["negatives"] == 5 and g["nonfinite"] == 2
    fin = f[np.isfinite(f)]
    assert g["min_f"] == fin.min()
    assert np.isnan(g["rho_residual"]) or np.isnan(g["T_residual"]) or np.isinf(g["rho_residual"])
    # the same state with the non-finite values removed: everything finite
    f2 = np.where(np.isfinite(f), f, 0.5)
    g2 = bgk.bgk_state_check(ctx, t(f2), t(rho), t(U), t(T))
    compare(g2, host_check(c, f2, rho, U, T), 1e-12)
