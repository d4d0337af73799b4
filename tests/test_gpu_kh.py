"""Kelvin-Helmholtz shear layers with dynamic refinement driven by the
density-jump indicator: the device indicator and the cycle-plus-regrid loop
against the oracle (the oracle's flags shared by both sides), then a long
GPU-only run whose regrids follow the device indicator, checked by the
conservation of every total across the regrids and by the growth of the
instability. Runs on an MI355X."""
import numpy as np
import pytest

from _helpers import print_case, rel_err, scales
from oracle.oracle import OracleMesh
from paper_2202_12309_amd import inputs

pytestmark = pytest.mark.gpu
G = 5.0 / 3.0
REFINE, DEREFINE = 0.02, 0.005
N8, NRB = (8, 8, 8), (4, 4, 4)


def _flags(eta):
    return np.where(eta > REFINE, 1, np.where(eta < DEREFINE, -1, 0)).astype(np.int8)


def _adapted_pair(**kh):
    """Root 32^3 in 8^3 blocks, max_level 2, refined twice from the initial
    state's density jumps (the generator evaluated on each new mesh)."""
    from paper_2202_12309_amd.binding import Mesh
    lv = inputs.uniform_leaves(NRB)
    om = OracleMesh(N8, NRB, lv, max_level=2)
    for _ in range(2):
        om.set_state(inputs.kelvin_helmholtz(om.leaves(), N8, NRB, **kh))
        om.regrid(_flags(om.density_jump()))
    gm = Mesh((32, 32, 32), N8, om.leaves(), max_level=2)
    assert np.array_equal(gm.leaves(), om.leaves())
    U0 = inputs.kelvin_helmholtz(gm.leaves(), N8, NRB, **kh)
    gm.upload(U0)
    om.set_state(U0)
    return gm, om


def _long_run(t_end, **kh):
    """Advance to t_end with a regrid every 10 cycles from the device's own
    density flags; returns (max |vy| at start and end, distinct leaf counts,
    |change of the totals|, their scale, final state)."""
    gm, om = _adapted_pair(**kh)
    del om
    T0 = gm.totals()
    U = gm.download()
    scale = scales(U, G)  # per variable; rho c for the momenta (the box has unit volume)
    vy0 = np.abs(U[:, 2] / U[:, 0]).max()
    meshes = set()
    t = 0.0
    while t < t_end:
        gm.step(10)
        gm.flag_density_jump(REFINE, DEREFINE)
        gm.regrid()
        meshes.add(gm.nleaves)
        t = gm.time()[0]
    U = gm.download()
    vy = np.abs(U[:, 2] / U[:, 0]).max()
    dT = np.abs(gm.totals() - T0)
    gm.close()
    return vy0, vy, meshes, dT, np.maximum(np.abs(T0), scale), U


def test_kh_density_indicator_and_regrid_parity():
    print_case("KH, 32^3 root in 8^3 blocks, 3 levels, 20 cycles, regrid every 5 by density jumps")
    gm, om = _adapted_pair()
    counts = np.bincount(gm.leaves()[:, 0], minlength=3)
    print("leaves per level", counts, flush=True)
    assert counts[2] > 0 and counts[1] > 0
    To0, Ao = om.totals()
    for s in range(4):
        gm.step(5)
        om.step(5)
        c = 5 * (s + 1)
        err = rel_err(gm.download(), om.state(), G)
        print(f"cycle {c}: leaves {gm.nleaves}, rel err {err}", flush=True)
        assert np.all(err <= 1e-11 * c), (c, err)
        eo = om.density_jump()
        fg, eg = gm.flag_density_jump(REFINE, DEREFINE)
        assert np.all(np.abs(eg - eo) <= 1e-10 * np.maximum(eo, 1e-4)), np.abs(eg - eo).max()
        near = (np.abs(eo - REFINE) <= 1e-9) | (np.abs(eo - DEREFINE) <= 1e-9)
        fo = _flags(eo)
        assert np.array_equal(fg[~near], fo[~near])
        gm.regrid(fo)
        om.regrid(fo)
        assert np.array_equal(gm.leaves(), om.leaves())
    # periodic box: every total survives cycles and regrids to round-off
    assert np.all(np.abs(gm.totals() - To0) <= 1e-13 * np.maximum(Ao, 1.0))


def test_kh_long_run_device_driven_regrids():
    """About 1600 cycles (t to 1.5, seed amplitude 0.1) with a regrid every
    10 cycles from the device's own flags: the totals stay at their initial
    values across every regrid, the mesh follows the deforming layers, and
    the y-velocity seed grows, while the same layers without shear (u0 = 0)
    do not amplify it."""
    print_case("KH long run, 32^3 root in 8^3 blocks, 3 levels, to t = 1.5, device flags every 10 cycles")
    vy0, vy, meshes, dT, scale, U = _long_run(1.5, amp=0.1)
    print(f"shear: distinct leaf counts {sorted(meshes)}, max|vy| {vy0:.4f} -> {vy:.4f}, dT {dT}", flush=True)
    assert np.all(dT <= 1e-12 * scale), dT
    assert len(meshes) >= 3
    assert vy > 2.0 * vy0
    assert np.all(U[:, 0] > 0.0)
    cvy0, cvy, _, cdT, cscale, _ = _long_run(1.5, amp=0.1, u0=0.0)
    print(f"no shear: max|vy| {cvy0:.4f} -> {cvy:.4f}", flush=True)
    assert np.all(cdT <= 1e-12 * cscale), cdT
    assert cvy < 1.2 * cvy0
