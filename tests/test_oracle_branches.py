"""Pins of the oracle's frozen-timestep cycles and of its branch signature
(the tools of the finite-difference checks of the reverse mode on
multilevel meshes). CPU only.

* Cycles with the recorded timesteps reproduce the CFL-timestep cycles bit
  for bit, on one and two levels.
* The case codes name the branch the limiter, minmod and HLLE wave-speed
  functions take: each code's formula equals the returned value.
* The signature is a function of the branches alone: equal for repeated
  runs and for perturbations too small to move any branch, different when a
  perturbation moves limiter or prolongation-slope cases."""
import numpy as np
import pytest

from oracle import oracle as orc
from oracle.oracle import OracleMesh
from paper_2202_12309_amd import inputs

G = 5.0 / 3.0


def _codes_lib():
    return orc.lib()


def test_mc_code_names_the_value():
    L = _codes_lib()
    rng = np.random.default_rng(1)
    seen = set()
    for _ in range(20000):
        dl, dr = rng.normal(size=2) * 10.0 ** rng.uniform(-3, 3, size=2)
        if rng.random() < 0.1:
            dr = 3.0 * dl  # a tie between the 2|dr| ... |dl+dr|/2 cases is avoided below
        v = L.orc_mc(dl, dr)
        k = L.orc_mc_code(dl, dr)
        seen.add(k)
        cand = {0: 0.0, 1: 2 * abs(dl), 2: 2 * abs(dr), 3: 0.5 * abs(dl + dr)}
        assert abs(v) == cand[k], (dl, dr, v, k)
    assert seen == {0, 1, 2, 3}
    assert L.orc_mc_code(1.0, -1.0) == 0 and L.orc_mc_code(0.0, 3.0) == 0
    assert L.orc_mc_code(1.0, 0.2) == 2 and L.orc_mc_code(1.0, 1.0) == 3 and L.orc_mc_code(0.2, 1.0) == 1


def test_minmod_code_names_the_value():
    L = _codes_lib()
    rng = np.random.default_rng(2)
    for _ in range(5000):
        a, b = rng.normal(size=2)
        v = L.orc_minmod(a, b)
        k = L.orc_minmod_code(a, b)
        assert v == {0: 0.0, 1: a, 2: b}[k], (a, b, v, k)


def test_hlle_code_names_the_bounds():
    """A supersonic flow to the right takes b- = 0 (case 2): the flux is the
    left state's flux; subsonic flow takes the Roe bound or the signal speed
    (cases 0 or 1) on each side."""
    L = _codes_lib()
    D = orc._dp
    wl = np.array([1.0, 3.0, 0.1, -0.2, 1.0])
    wr = np.array([0.8, 2.9, 0.0, 0.1, 0.9])
    k = L.orc_hlle_code(D(wl), D(wr), 0, G)
    assert k // 3 == 2, k
    f = np.zeros(5)
    L.orc_hlle(D(wl), D(wr), 0, G, D(f))
    E = wl[4] / (G - 1) + 0.5 * wl[0] * (wl[1:4] ** 2).sum()
    fl = np.array([wl[0] * wl[1], wl[0] * wl[1] ** 2 + wl[4], wl[0] * wl[1] * wl[2], wl[0] * wl[1] * wl[3],
                   (E + wl[4]) * wl[1]])
    assert np.allclose(f, fl, rtol=1e-14, atol=0)
    wl2 = np.array([1.0, 0.1, 0.0, 0.0, 1.0])
    wr2 = np.array([1.0, 0.1, 0.0, 0.0, 1.0])
    k2 = L.orc_hlle_code(D(wl2), D(wr2), 0, G)
    assert k2 % 3 in (0, 1) and k2 // 3 in (0, 1)


@pytest.mark.parametrize("two_level", [False, True])
def test_frozen_timestep_cycles_equal_cfl_cycles(two_level):
    nrb, n = (4, 4, 4), (8, 8, 8)
    lv = inputs.sphere_refined_leaves(nrb, radius=0.3) if two_level else inputs.uniform_leaves(nrb)
    om = OracleMesh(n, nrb, lv, max_level=1)
    U0 = inputs.blast(om.leaves(), n, nrb) if two_level else inputs.turbulent_box(om.leaves(), n, nrb, seed=3)
    om.set_state(U0)
    dts = []
    for _ in range(3):
        om.step(1)
        dts.append(om.time()[1])
    U3, t3 = om.state(), om.time()[0]
    om.set_state(U0)
    om.set_time(0.0, 0)
    om.step_dts(dts)
    assert np.array_equal(om.state(), U3)
    assert om.time()[0] == t3 and om.time()[2] == 3


def _smooth_mesh(two_level):
    """A smooth flow without symmetries (no exact ties between neighbouring
    differences) on 4^3 root blocks of 8^3; two_level: the root blocks
    meeting a ball of radius 0.2 about the centre refined."""
    nrb, n = (4, 4, 4), (8, 8, 8)
    lv = inputs.sphere_refined_leaves(nrb, radius=0.2) if two_level else inputs.uniform_leaves(nrb)
    om = OracleMesh(n, nrb, lv, max_level=1)
    return om, inputs.generic_flow(om.leaves(), n, nrb)


def _signature(om, U, cycles=1):
    om.set_state(U)
    om.set_time(0.0, 0)
    om.track_branches(True)
    om.step_dts([1e-3] * cycles)
    s = om.branch_signature()
    om.track_branches(False)
    return s


def test_signature_follows_the_limiter_branch():
    om, U = _smooth_mesh(False)
    s0 = _signature(om, U)
    assert s0 == _signature(om, U) and s0 != 0
    # a perturbation far below every branch margin keeps them all
    V = np.zeros_like(U)
    V[21, 0, 3, 3, 3] = 1.0
    assert _signature(om, U + 1e-13 * V) == _signature(om, U - 1e-13 * V) == s0
    # a density bump of +-0.2 makes the cell an extremum (or deepens one):
    # the limiter cases of its neighbours change
    sp, sm = _signature(om, U + 0.2 * V), _signature(om, U - 0.2 * V)
    assert sp != s0 and sm != s0 and sp != sm


def test_signature_follows_the_prolongation_slope_branch():
    """On two levels: a bump in the coarse cell next to the refined region
    makes it an extremum of the coarse field (the minmod cases of the
    prolonged ghost cells beside it and the limiter cases of its own faces
    change) and moves the signature; far smaller perturbations keep every
    case, including every prolongation slope's."""
    om, U = _smooth_mesh(True)
    s0 = _signature(om, U)
    assert s0 == _signature(om, U)
    lv = om.leaves()
    # a coarse leaf whose +x neighbour is refined: bump its last x cell
    q = next(i for i, l in enumerate(lv) if l[0] == 0 and tuple(l[1:]) == (0, 1, 1))
    assert any(l[0] == 1 and l[1] == 2 and l[2] in (2, 3) and l[3] in (2, 3) for l in lv)
    V = np.zeros_like(U)
    V[q, 0, 3, 3, 7] = 1.0
    assert _signature(om, U + 1e-13 * V) == _signature(om, U - 1e-13 * V) == s0
    assert _signature(om, U + 0.2 * V) != _signature(om, U - 0.2 * V)


@pytest.mark.parametrize("bc", [(1, 1, 0, 0, 0, 0), (2, 2, 0, 0, 0, 0)])
def test_signature_stable_at_walls(bc):
    """Outflow walls make the face states at the wall identical (the ghost
    copies the cell), so both HLLE bounds coincide up to rounding there; the
    flux and its derivative do not depend on the bound taken, and the
    signature records no case for such faces: a dense perturbation of 1e-12
    keeps it. Reflecting walls likewise."""
    om = OracleMesh((16, 16, 16), (2, 2, 2), inputs.uniform_leaves((2, 2, 2)), bc=bc)
    U = inputs.generic_flow(om.leaves(), (16, 16, 16), (2, 2, 2))
    V = np.random.default_rng(1).normal(size=U.shape)
    s0 = _signature(om, U, cycles=2)
    assert _signature(om, U + 1e-12 * V, cycles=2) == s0
    assert _signature(om, U - 1e-12 * V, cycles=2) == s0
