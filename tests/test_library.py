"""CPU checks of the C interface: the library loads, exports every symbol the
header declares, and validates configurations on the host (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bgk.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bgk_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2408_02350_amd.bgk as b
    if not os.path.exists(b.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return b


def test_header_symbols_are_exported(lib):
    L = lib.load_library()
    syms = declared_symbols()
    assert len(syms) >= 18
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(lib.EXPORTS) == syms


def test_hot_path_entry_points_present(lib):
    syms = declared_symbols()
    for s in ("bgk_init", "bgk_build_neighbors", "bgk_wls_operators", "bgk_step", "bgk_moments",
              "bgk_adjoint_step"):
        assert s in syms


def test_no_gpu_fallback_module():
    """The binding calls only the library: no numpy/torch arithmetic paths."""
    pkg = os.path.join(ROOT, "paper_2408_02350_amd")
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            s = open(os.path.join(pkg, f)).read()
            assert not re.search(r"^\s*(import|from)\s+oracle", s, flags=re.M), f
            assert "liboracle" not in s, f


def _cfg(lib, **kw):
    from paper_2408_02350_amd.inputs import CONFIGS
    return lib.config_from(CONFIGS["c1"], **kw)


def test_workspace_sizing_and_validation(lib):
    n = lib.bgk_workspace_bytes(_cfg(lib))
    assert n > 0
    bigger = lib.bgk_workspace_bytes(_cfg(lib, n_particles=3200))
    assert bigger > n
    # the largest velocity grid per axis (exponential tables of the wall
    # condition live in LDS)
    assert lib.bgk_workspace_bytes(_cfg(lib, nv=1024)) > 0
    # the reverse step's workspace, larger again with the moving cloud's
    frozen = lib.bgk_workspace_bytes(_cfg(lib, flags=2, move=0))
    assert frozen > n
    assert lib.bgk_workspace_bytes(_cfg(lib, flags=2, move=1)) > frozen
    for bad in (dict(nv=15), dict(nv=1026), dict(dim=4), dict(n_particles=0), dict(dt=-1.0),
                dict(wls_degree=3), dict(max_neighbors=300), dict(precision=5),
                dict(flags=2, precision=2), dict(flags=8), dict(h=0.0)):
        with pytest.raises(lib.BgkError) as e:
            lib.bgk_workspace_bytes(_cfg(lib, **bad))
        assert e.value.code == lib.BGK_EINVAL, bad


def test_null_arguments_rejected(lib):
    L = lib.load_library()
    out = ctypes.c_void_p()
    assert L.bgk_init(None, None, None, 0, None, ctypes.byref(out)) == lib.BGK_EINVAL
    assert L.bgk_step(None, None, None, None, None, None, None) == lib.BGK_EINVAL
    assert L.bgk_check(None) == lib.BGK_EINVAL
    assert L.bgk_last_error(None) == b"null context"


def test_checkpoint_segments_cover_every_step_once():
    from paper_2408_02350_amd.adjoint import segments
    for nsteps in (0, 1, 5, 10, 50, 53):
        for every in (1, 3, 10, 100):
            seg = segments(nsteps, every)
            steps = [s for s0, s1 in seg for s in range(s0, s1)]
            assert steps == list(range(nsteps))
            assert all(0 < s1 - s0 <= every for s0, s1 in seg)
    with pytest.raises(ValueError):
        segments(5, 0)


def test_adjoint_flag_rules(lib):
    bgk = lib
    L = bgk.load_library()
    from paper_2408_02350_amd.inputs import CONFIGS
    n = ctypes.c_size_t(0)
    plain = bgk.config_from(CONFIGS["c4"], "fp64")
    L.bgk_workspace_bytes(ctypes.byref(plain), ctypes.byref(n))
    base = n.value
    adj = bgk.config_from(CONFIGS["c4"], "fp64", flags=bgk.BGK_FLAG_ADJOINT)
    assert L.bgk_workspace_bytes(ctypes.byref(adj), ctypes.byref(n)) == bgk.BGK_OK
    cav = CONFIGS["c4"]
    f_bytes = 8 * 2 * cav.n_particles * cav.n_velocities
    assert n.value >= base + 3 * f_bytes      # f-tilde, lam_ft, wall adjoints
    c = bgk.config_from(CONFIGS["c4"], "fp64", flags=bgk.BGK_FLAG_ADJOINT)
    c.precision = bgk.BGK_BF16
    assert L.bgk_workspace_bytes(ctypes.byref(c), ctypes.byref(n)) == bgk.BGK_EINVAL
    # the moving cloud's reverse step (move = 1) reserves more
    frozen = n.value
    mv = bgk.config_from(CONFIGS["c4"], "fp64", flags=bgk.BGK_FLAG_ADJOINT, move=1)
    assert L.bgk_workspace_bytes(ctypes.byref(adj), ctypes.byref(n)) == bgk.BGK_OK
    frozen = n.value
    assert L.bgk_workspace_bytes(ctypes.byref(mv), ctypes.byref(n)) == bgk.BGK_OK
    assert n.value > frozen
