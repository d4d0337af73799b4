"""Pins of the oracle's domain boundaries (outflow, reflecting): ghost images,
agreement with the grid formulation, mirror symmetry against a doubled
periodic domain on one and two levels, conservation in a reflecting box,
and the tree logic across non-periodic faces. CPU only."""
import numpy as np
import pytest
import torch

from _helpers import rel_err
from oracle import torch_ref
from oracle.oracle import BC_OUTFLOW as OUT
from oracle.oracle import BC_PERIODIC as PER
from oracle.oracle import BC_REFLECT as REF
from oracle.oracle import OracleError, OracleMesh
from paper_2202_12309_amd import inputs

G = 5.0 / 3.0
N8 = (8, 8, 8)


def _conserved(rho, vx, vy, vz, p):
    return np.stack([rho, rho * vx, rho * vy, rho * vz,
                     p / (G - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz)])


def _flow(m):
    return inputs.smooth_flow(m.leaves(), m.n, m.nrb, xmin=m.xmin, xmax=m.xmax)


def test_extended_formulation_equals_roll_when_periodic():
    """The boundary-extended grid formulation with every face periodic is the
    torch.roll formulation, bitwise (same face states, same flux order)."""
    lv = inputs.uniform_leaves((2, 2, 2))
    U = inputs.turbulent_box(lv, N8, (2, 2, 2), seed=3)
    Gt = torch.tensor(torch_ref.blocks_to_global(U, lv, N8, (2, 2, 2)))
    a, _ = torch_ref.run(Gt, 3)
    b, _ = torch_ref.run(Gt, 3, bc=(PER,) * 6)
    assert torch.equal(a, b)


def test_ghost_images_at_walls():
    """Ghost cells beyond a reflecting face hold the mirror image (cell -1-m
    takes cell m) with the normal momentum negated; beyond an outflow face
    the nearest cell inside; an edge beyond both faces combines the two maps
    and flips only the reflected component."""
    nrb = (2, 2, 2)
    m = OracleMesh(N8, nrb, inputs.uniform_leaves(nrb), bc=(REF, OUT, OUT, REF, PER, PER))
    rng = np.random.default_rng(7)
    U = np.stack([_conserved(1.0 + 0.1 * rng.random((8, 8, 8)), *(0.3 * rng.normal(size=(3, 8, 8, 8))),
                             1.0 + 0.1 * rng.random((8, 8, 8))) for _ in range(m.nleaves)])
    m.set_state(U)
    lv = m.leaves()
    b0 = int(np.flatnonzero((lv[:, 1:] == [0, 0, 0]).all(axis=1))[0])  # touches x-, y-, z- (periodic)
    b1 = int(np.flatnonzero((lv[:, 1:] == [1, 1, 0]).all(axis=1))[0])  # touches x+, y+
    P0, P1 = m.padded(b0), m.padded(b1)
    a = slice(2, 10)
    u0, u1 = U[b0], U[b1]
    # x- reflecting: ghost i = -1 - m holds cell m, Mx negated
    for mm in (0, 1):
        g = P0[:, a, a, 1 - mm]
        want = u0[:, :, :, mm].copy()
        want[1] *= -1.0
        assert np.array_equal(g, want)
    # y- outflow: both ghost rows hold row 0, nothing negated
    for s in (0, 1):
        assert np.array_equal(P0[:, a, s, a], u0[:, :, 0, :])
    # x+ outflow: both ghost columns hold column n-1
    for s in (10, 11):
        assert np.array_equal(P1[:, a, a, s], u1[:, :, :, 7])
    # y+ reflecting: ghost row n + m holds row n-1-m, My negated
    for mm in (0, 1):
        want = u1[:, :, 7 - mm, :].copy()
        want[2] *= -1.0
        assert np.array_equal(P1[:, a, 10 + mm, a], want)
    # the (x-, y-) edge of b0: mirrored in x, clamped in y, only Mx negated
    for mm in (0, 1):
        want = u0[:, :, 0, mm].copy()
        want[1] *= -1.0
        assert np.array_equal(P0[:, a, 0, 1 - mm], want)


@pytest.mark.parametrize("bc", [(REF, REF, OUT, OUT, PER, PER), (OUT, REF, PER, PER, REF, OUT)])
@pytest.mark.parametrize("recon1", [0, 1])
def test_oracle_matches_grid_formulation_with_walls(bc, recon1):
    nrb = (2, 2, 2)
    lv = inputs.uniform_leaves(nrb)
    m = OracleMesh(N8, nrb, lv, bc=bc, stage1_recon=recon1)
    U0 = _flow(m)
    m.set_state(U0)
    m.step(3)
    Gt = torch.tensor(torch_ref.blocks_to_global(U0, m.leaves(), N8, nrb))
    Gn, _ = torch_ref.run(Gt, 3, stage1_recon=recon1, bc=bc)
    ref = torch_ref.global_to_blocks(Gn.numpy(), m.leaves(), N8)
    err = rel_err(m.state(), ref, G)
    assert np.all(err <= 1e-14), err


def _mirror_leaf(lf, nrb_doubled_x):
    L, lx, ly, lz = (int(v) for v in lf)
    return (L, (nrb_doubled_x << L) - 1 - lx, ly, lz)


def _doubled(half, half_leaves, max_level):
    """The periodic domain [0,2) x [0,1)^2 holding the half-domain state and
    its mirror image about x = 1 (and so about x = 0)."""
    nrb2 = (2 * half.nrb[0], half.nrb[1], half.nrb[2])
    lv2 = [tuple(int(v) for v in lf) for lf in half_leaves] + \
          [_mirror_leaf(lf, nrb2[0]) for lf in half_leaves]
    m2 = OracleMesh(N8, nrb2, lv2, xmax=(2.0, 1.0, 1.0), max_level=max_level)
    return m2


def _mirror_state(half, m2, Uh):
    idx = {tuple(int(v) for v in lf): b for b, lf in enumerate(half.leaves())}
    U2 = np.empty(m2.shape())
    for b, lf in enumerate(m2.leaves()):
        key = tuple(int(v) for v in lf)
        if key in idx:
            U2[b] = Uh[idx[key]]
        else:
            u = Uh[idx[_mirror_leaf(key, m2.nrb[0])]][:, :, :, ::-1].copy()
            u[1] *= -1.0
            U2[b] = u
    return U2


@pytest.mark.parametrize("levels", [1, 2])
def test_reflecting_walls_equal_mirrored_periodic_domain(levels):
    """A box with reflecting x faces evolves exactly like the left half of a
    periodic box twice as long holding the state and its mirror image (the
    HLLE flux through the symmetry plane equals the one the mirror ghosts
    give). On two levels the refined blocks touch both walls, so the
    prolongation stencils reach past the wall at the coarse level. Rounding
    alone separates the two (the doubled domain is symmetric only up to the
    order of the Roe-average sums)."""
    nrb = (2, 2, 2)
    if levels == 1:
        lv, ml = inputs.uniform_leaves(nrb), 0
    else:
        lv = [[0, x, y, z] for z in range(2) for y in range(2) for x in range(2)
              if (x, y, z) not in ((0, 0, 0), (1, 1, 1))]
        for (x, y, z) in ((0, 0, 0), (1, 1, 1)):
            lv += [[1, 2 * x + (c & 1), 2 * y + ((c >> 1) & 1), 2 * z + ((c >> 2) & 1)] for c in range(8)]
        ml = 1
    half = OracleMesh(N8, nrb, lv, max_level=ml, bc=(REF, REF, PER, PER, PER, PER))
    Uh = _flow(half)
    half.set_state(Uh)
    m2 = _doubled(half, half.leaves(), ml)
    m2.set_state(_mirror_state(half, m2, Uh))
    assert half.dt() == pytest.approx(m2.dt(), rel=1e-15)
    half.step(4)
    m2.step(4)
    idx2 = {tuple(int(v) for v in lf): b for b, lf in enumerate(m2.leaves())}
    U2 = m2.state()
    got = np.stack([U2[idx2[tuple(int(v) for v in lf)]] for lf in half.leaves()])
    err = rel_err(half.state(), got, G)
    assert np.all(err <= 1e-13), err
    # and the state is far from the initial one: the walls mattered
    assert rel_err(half.state(), Uh, G).max() > 1e-3


@pytest.mark.parametrize("levels", [1, 2])
def test_reflecting_box_conserves_mass_and_energy(levels):
    """No mass or energy crosses a reflecting face: the mirror states make
    the HLLE mass and energy fluxes there exactly zero, so the totals stay
    at their initial values up to summation rounding (a wrong image index
    leaves a mass flux through the wall)."""
    nrb = (4, 4, 4)
    lv = inputs.uniform_leaves(nrb) if levels == 1 else inputs.sphere_refined_leaves(nrb, radius=0.2)
    m = OracleMesh(N8, nrb, lv, max_level=levels - 1, bc=(REF,) * 6)
    m.set_state(_flow(m))
    T0, A0 = m.totals()
    m.step(5)
    T, _ = m.totals()
    assert abs(T[0] - T0[0]) <= 1e-13 * A0[0]
    assert abs(T[4] - T0[4]) <= 1e-13 * A0[4]
    # momentum is not conserved: the walls push back
    assert abs(T[1] - T0[1]) > 1e-6 * A0[1]


def test_outflow_keeps_a_uniform_flow_bitwise_on_two_levels():
    nrb = (4, 4, 4)
    m = OracleMesh(N8, nrb, inputs.sphere_refined_leaves(nrb, radius=0.2), max_level=1, bc=(OUT,) * 6)
    U0 = inputs.uniform_state(m.leaves(), N8, rho=1.2, v=(0.4, -0.3, 0.2), p=0.9)
    m.set_state(U0)
    m.step(3)
    assert np.array_equal(m.state(), U0)


def test_balance_across_the_domain_boundary():
    """Root block 0 of two along x refined to level 2 next to x = 0 (level-1
    leaves elsewhere in it): across a periodic x boundary those level-2
    leaves touch the level-0 root 1, two levels apart (rejected); with
    walls in x they have no neighbour there (accepted)."""
    nrb = (2, 1, 1)
    lv = [[0, 1, 0, 0]]
    for c in range(8):
        cx, cy, cz = c & 1, (c >> 1) & 1, (c >> 2) & 1
        if cx == 0:
            lv += [[2, 2 * cx + (g & 1), 2 * cy + ((g >> 1) & 1), 2 * cz + ((g >> 2) & 1)] for g in range(8)]
        else:
            lv.append([1, cx, cy, cz])
    with pytest.raises(OracleError):
        OracleMesh(N8, nrb, lv, max_level=2)
    OracleMesh(N8, nrb, lv, max_level=2, bc=(OUT, OUT, PER, PER, PER, PER))
    with pytest.raises(OracleError):  # periodic on one face only
        OracleMesh(N8, nrb, lv, max_level=2, bc=(PER, OUT, PER, PER, PER, PER))
