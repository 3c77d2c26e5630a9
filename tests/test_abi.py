"""CPU checks of the C-ABI library: it loads, exports every function that
include/dg.h declares, and its host-only calls validate configurations
(no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def dg():
    from paper_1904_11147_amd import dg as D
    if not os.path.exists(D.LIB_PATH):
        from paper_1904_11147_amd import build
        build.build()
    D.lib()
    return D


def test_exports_every_declared_symbol(dg):
    names = _declared()
    assert "dg_step" in names and "dg_limit" in names and "dg_init" in names
    L = dg.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(dg.EXPORTS)


def test_strerror(dg):
    assert dg.strerror(0) == "ok"
    assert "non-physical" in dg.strerror(-5)
    assert dg.strerror(12345) == "unknown error"


def test_workspace_bytes_and_validation(dg):
    c = dg.make_config(dim=2, equation=dg.EULER, order=2, nx=2048, ny=2048, bc=(1, 1, 1, 1))
    n = dg.workspace_bytes(c)
    state = 2048 * 2048 * 9 * 4 * 8
    assert n >= 2 * state and n < 2 * state + 2048 * 2048 * 16
    bad = [dict(dim=3), dict(order=4), dict(order=0), dict(nx=0), dict(dim=1, ny=5),
           dict(bc=(0, 1, 0, 0)), dict(limiter=7), dict(indicator=9), dict(negw_mode=5),
           dict(x0=1.0, x1=0.0), dict(weno_eps=0.0), dict(cfl=-1.0), dict(equation=3)]
    for kw in bad:
        base = dict(dim=1, equation=0, order=2, nx=16)
        base.update(kw)
        if base["dim"] == 1 and "ny" in kw:
            c = dg.make_config(**base)
            c.ny = kw["ny"]
        else:
            c = dg.make_config(**base)
        with pytest.raises(dg.DGError):
            dg.workspace_bytes(c)
    c = dg.make_config()
    c.abi_version = 99
    with pytest.raises(dg.DGError):
        dg.workspace_bytes(c)


def test_init_rejects_small_workspace_without_touching_device(dg):
    c = dg.make_config(dim=1, nx=8)
    h = ctypes.c_void_p()
    rc = dg.lib().dg_init(ctypes.byref(c), None, 0, None, ctypes.byref(h))
    assert rc == dg.DG_ERR_WORKSPACE
    rc = dg.lib().dg_init(ctypes.byref(c), ctypes.c_void_p(4096 + 8), 1 << 30, None, ctypes.byref(h))
    assert rc == dg.DG_ERR_WORKSPACE  # misaligned


def test_batch_workspace_and_validation(dg):
    """Batch sizes and rules are checked on the host before any device work."""
    def arr(*cfgs):
        return (dg.Config * len(cfgs))(*[dg.make_config(**c) for c in cfgs])

    def nbytes(*cfgs):
        n = ctypes.c_size_t()
        rc = dg.lib().dg_batch_workspace_bytes(arr(*cfgs), len(cfgs), ctypes.byref(n))
        return rc, n.value

    e2 = dict(dim=2, equation=dg.EULER, bc=(1, 1, 1, 1))
    rc, n = nbytes(dict(e2, order=1, nx=64, ny=64), dict(e2, order=3, nx=100, ny=80))
    states = 64 * 64 * 4 * 4 * 8 + 100 * 80 * 16 * 4 * 8
    assert rc == 0 and 2 * states <= n < 2 * states + 4 * 50000 * 4 + 8 * 20000 + 4 * 4096
    assert nbytes(dict(dim=1, equation=dg.EULER, order=2, nx=16))[0] == dg.DG_ERR_UNSUPPORTED
    assert nbytes(dict(e2, order=2, nx=8, ny=8, equation=dg.BURGERS))[0] == dg.DG_ERR_UNSUPPORTED
    assert nbytes(dict(e2, order=2, nx=8, ny=8), dict(e2, order=2, nx=8, ny=8, limiter=dg.LIM_NONE))[0] == \
        dg.DG_ERR_INVALID_ARG
    assert nbytes(dict(e2, order=2, nx=8, ny=8), dict(e2, order=1, nx=8, ny=8, indicator=dg.IND_ALL))[0] == \
        dg.DG_ERR_INVALID_ARG
    assert nbytes(dict(e2, order=2, nx=50000, ny=50000))[0] == dg.DG_ERR_UNSUPPORTED
    # per instance at most 2^27 / (N+1)^2 cells (32-bit byte offsets in the batched stage kernel)
    assert nbytes(dict(e2, order=2, nx=4096, ny=3640))[0] == 0  # 14.91e6 cells: 32 * 9 * n <= 2^32
    assert nbytes(dict(e2, order=2, nx=4096, ny=3641))[0] == dg.DG_ERR_UNSUPPORTED
    assert nbytes(dict(e2, order=3, nx=4096, ny=2048))[0] == 0
    assert nbytes(dict(e2, order=3, nx=4096, ny=2049))[0] == dg.DG_ERR_UNSUPPORTED
    n = ctypes.c_size_t()
    assert dg.lib().dg_batch_workspace_bytes(arr(dict(e2, order=2, nx=8, ny=8)), 0, ctypes.byref(n)) == \
        dg.DG_ERR_INVALID_ARG
    h = ctypes.c_void_p()
    one = arr(dict(e2, order=2, nx=8, ny=8))
    assert dg.lib().dg_batch_init(one, 1, None, 0, None, ctypes.byref(h)) == dg.DG_ERR_WORKSPACE


def test_boundary_and_positivity_validation(dg):
    """Wall, inflow and switching sides and the positivity flag are checked on
    the host: a wall or positivity needs the Euler equations, west/east sides
    never switch, inflow states must be admissible."""
    from paper_1904_11147_amd import workloads as W
    wl = W.double_mach(64)
    ok = dg.make_config(**{k: v for k, v in wl.config().items()})
    assert dg.workspace_bytes(ok) > 0
    bad = []
    bad.append(dict(wl.config(), bc_beyond=(2, -1, 2, 3)))           # a west side that switches
    bad.append(dict(wl.config(), bc_beyond=(-1, -1, 0, 3)))          # periodic beyond a switch
    st = np.array(wl.bc_extra["bc_state"])
    st[0, 0, 0] = -1.0
    bad.append(dict(wl.config(), bc_state=st))                        # negative inflow density
    st = np.array(wl.bc_extra["bc_state"])
    st[3, 1, 3] = 0.0
    bad.append(dict(wl.config(), bc_state=st))                        # zero pressure beyond the switch
    bad.append(dict(dim=1, equation=dg.BURGERS, order=1, nx=8, bc=(dg.REFLECTIVE, 1, 0, 0)))
    bad.append(dict(dim=1, equation=dg.BURGERS, order=1, nx=8, bc=(1, 1, 0, 0), positivity=1))
    bad.append(dict(dim=1, equation=dg.EULER, order=1, nx=8, bc=(1, 1, 0, 0), positivity=2))
    for kw in bad:
        with pytest.raises(dg.DGError):
            dg.workspace_bytes(dg.make_config(**kw))
    c = dg.make_config(**wl.config())
    c.pad = 1
    with pytest.raises(dg.DGError):
        dg.workspace_bytes(c)
    # batches take periodic and transmissive sides on uniform meshes, with
    # the scaling on for all instances or for none
    n = ctypes.c_size_t()
    e2 = dict(dim=2, equation=dg.EULER, order=2, nx=8, ny=8)
    cf = (dg.Config * 1)(dg.make_config(**dict(e2, bc=(dg.REFLECTIVE, 1, dg.REFLECTIVE, 1))))
    assert dg.lib().dg_batch_workspace_bytes(cf, 1, ctypes.byref(n)) == dg.DG_ERR_UNSUPPORTED
    cf = (dg.Config * 1)(dg.make_config(**dict(e2, bc=(1, 1, 1, 1), xn=np.linspace(0, 1, 9), yn=np.linspace(0, 1, 9))))
    assert dg.lib().dg_batch_workspace_bytes(cf, 1, ctypes.byref(n)) == dg.DG_ERR_UNSUPPORTED
    cf = (dg.Config * 1)(dg.make_config(**dict(e2, bc=(1, 1, 1, 1), positivity=1)))
    assert dg.lib().dg_batch_workspace_bytes(cf, 1, ctypes.byref(n)) == 0
    cf = (dg.Config * 2)(dg.make_config(**dict(e2, bc=(1, 1, 1, 1), positivity=1)),
                         dg.make_config(**dict(e2, bc=(1, 1, 1, 1))))
    assert dg.lib().dg_batch_workspace_bytes(cf, 2, ctypes.byref(n)) == dg.DG_ERR_INVALID_ARG


def test_learned_indicator_takes_periodic_and_transmissive_sides_only(dg):
    """The network's features see ghost cells by periodic wrap or even
    reflection (the sides it was trained on); walls, inflow and switching
    sides are rejected on the host."""
    from paper_1904_11147_amd import workloads as W
    e2 = dict(dim=2, equation=dg.EULER, order=2, nx=8, ny=8, indicator=dg.IND_LEARNED)
    assert dg.workspace_bytes(dg.make_config(**dict(e2, bc=(1, 1, 1, 1)))) > 0
    assert dg.workspace_bytes(dg.make_config(**dict(e2, bc=(0, 0, 1, 1)))) > 0
    for bc in ((dg.REFLECTIVE, 1, 1, 1), (1, 1, dg.REFLECTIVE, 1)):
        with pytest.raises(dg.DGError) as e:
            dg.workspace_bytes(dg.make_config(**dict(e2, bc=bc)))
        assert e.value.code == dg.DG_ERR_UNSUPPORTED
    wl = W.double_mach(64)  # inflow and wall sides, a switching north side
    with pytest.raises(dg.DGError) as e:
        dg.workspace_bytes(dg.make_config(**dict(wl.config(), indicator=dg.IND_LEARNED)))
    assert e.value.code == dg.DG_ERR_UNSUPPORTED
    st = np.zeros((4, 2, 4))
    st[:, :, 0], st[:, :, 3] = 1.0, 2.5  # an admissible inflow state
    with pytest.raises(dg.DGError) as e:
        dg.workspace_bytes(dg.make_config(**dict(e2, bc=(1, 1, 1, dg.INFLOW), bc_state=st)))
    assert e.value.code == dg.DG_ERR_UNSUPPORTED
    assert dg.workspace_bytes(dg.make_config(**dict(e2, indicator=dg.IND_TVB, bc=(1, 1, 1, dg.INFLOW),
                                                    bc_state=st))) > 0
