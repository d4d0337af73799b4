"""Pins of the oracle's multilevel pieces: tiling and 2:1 validation, ghost
values by copy / restriction / prolongation, flux correction, regridding.
CPU only."""
import math

import numpy as np
import pytest

from oracle.oracle import OracleError, OracleMesh
from paper_2202_12309_amd import inputs

N8 = (8, 8, 8)
NRB4 = (4, 4, 4)


def _amr_mesh(max_level=1, **kw):
    leaves = inputs.sphere_refined_leaves(NRB4, radius=0.2)
    return OracleMesh(N8, NRB4, leaves, max_level=max_level, **kw)


def test_sphere_refinement_counts():
    # 8^3 root blocks, the central 4^3 refined: 960 leaves of which 512 fine
    lv = inputs.sphere_refined_leaves((8, 8, 8))
    assert len(lv) == 960 and (lv[:, 0] == 1).sum() == 512
    m = _amr_mesh()
    assert m.nleaves == 56 + 64


def test_invalid_tilings_rejected():
    nrb = (2, 2, 2)
    lv = inputs.uniform_leaves(nrb).tolist()
    with pytest.raises(OracleError):  # gap
        OracleMesh(N8, nrb, lv[:-1])
    with pytest.raises(OracleError):  # overlap: a block and its child
        OracleMesh(N8, nrb, lv + [[1, 0, 0, 0]], max_level=1)
    # root block (0,0,0) refined once and its child at the high corner once
    # more: those level-2 blocks touch the level-0 roots across x = 1/2
    lv2 = [l for l in lv if l != [0, 0, 0, 0]]
    for c in range(8):
        ch = [1, c & 1, (c >> 1) & 1, (c >> 2) & 1]
        if ch == [1, 1, 1, 1]:
            for g in range(8):
                lv2.append([2, 2 + (g & 1), 2 + ((g >> 1) & 1), 2 + ((g >> 2) & 1)])
        else:
            lv2.append(ch)
    with pytest.raises(OracleError):
        OracleMesh(N8, nrb, lv2, max_level=2)
    # the same two-level refinement is valid once every root is refined once
    lv3 = [[1, x, y, z] for z in range(4) for y in range(4) for x in range(4) if (x, y, z) != (1, 1, 1)]
    lv3 += [[2, 2 + (g & 1), 2 + ((g >> 1) & 1), 2 + ((g >> 2) & 1)] for g in range(8)]
    OracleMesh(N8, nrb, lv3, max_level=2)


def test_uniform_preserved_bitwise_on_two_levels():
    m = _amr_mesh()
    U0 = inputs.uniform_state(m.leaves(), N8, rho=1.37, v=(0.31, -0.52, 0.11), p=0.83)
    m.set_state(U0)
    m.step(3)
    assert np.array_equal(m.state(), U0)


def test_ghosts_reproduce_linear_field():
    """A field linear in x, sampled at cell centres on every level, restricts
    to the coarse centres and prolongates to the fine centres exactly (up to
    rounding): every ghost away from the periodic wrap equals the field at
    its centre, whichever of copy / restriction / prolongation filled it."""
    m = _amr_mesh()
    lv = m.leaves()
    a, b = 2.0, 0.75
    U = np.empty(m.shape())
    for k, lf in enumerate(lv):
        x, _, _ = inputs.cell_centers(lf, N8, NRB4)
        U[k] = (a + b * x)[None] * np.array([1.0, 0.3, -0.2, 0.1, 5.0])[:, None, None, None]
    m.set_state(U)
    checked = 0
    kinds = set()
    for k, lf in enumerate(lv):
        P = m.padded(k)
        lev = lf[0]
        h = 1.0 / (NRB4[0] * N8[0] * (1 << lev))
        xs = (lf[1] * N8[0] + np.arange(-2, N8[0] + 2) + 0.5) * h
        want = (a + b * xs)[None, None, None, :] * np.array([1.0, 0.3, -0.2, 0.1, 5.0])[:, None, None, None]
        ok = (xs > 0) & (xs < 1)
        err = np.abs(P[..., ok] - np.broadcast_to(want, P.shape)[..., ok]).max()
        assert err <= 1e-13, (k, lf, err)
        checked += 1
        kinds.add(int(lev))
    assert checked == len(lv) and kinds == {0, 1}


def test_prolongation_and_restriction_not_trivial():
    """On non-linear data the coarse ghosts of a fine block differ from plain
    injection (slopes are used) and the fine ghosts of a coarse block are the
    8-cell means."""
    m = _amr_mesh()
    lv = m.leaves()
    U = np.empty(m.shape())
    for k, lf in enumerate(lv):
        x, y, z = inputs.cell_centers(lf, N8, NRB4)
        f = 1.0 + 0.1 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) + 0.05 * z * z
        U[k] = f[None]
    m.set_state(U)
    # a coarse block face-adjacent to the refined region (which spans blocks 1..2)
    kc = [k for k, lf in enumerate(lv) if tuple(lf) == (0, 0, 1, 1)][0]
    P = m.padded(kc)
    # its x-high ghosts lie in fine blocks (level 1, lx = 2)
    fine = {tuple(lf): k for k, lf in enumerate(lv)}
    for jj in range(8):
        for kk in range(8):
            for gi in range(2):
                gx, gy, gz = 8 + gi, jj, kk  # ghost cell in coarse block coords
                X = 0 * 8 + gx  # coarse global cell index (block lx = 0)
                Y, Z = 8 + gy, 8 + gz
                fx, fy, fz = 2 * X, 2 * Y, 2 * Z
                kf = fine[(1, fx // 8, fy // 8, fz // 8)]
                blk = U[kf, 0, fz % 8:fz % 8 + 2, fy % 8:fy % 8 + 2, fx % 8:fx % 8 + 2]
                assert abs(P[0, gz + 2, gy + 2, gx + 2] - blk.mean()) <= 1e-15
    # a fine block's coarse-side ghost is not the injected coarse value
    kf = [k for k, lf in enumerate(lv) if tuple(lf) == (1, 2, 3, 3)][0]
    P = m.padded(kf)
    kcoarse = [k for k, lf in enumerate(lv) if tuple(lf) == (0, 0, 1, 1)][0]
    inj = U[kcoarse, 0, 7, 7, 7]
    assert abs(P[0, 2 + 7, 2 + 7, 1] - inj) > 1e-6


@pytest.mark.parametrize("ic", ["turbulent", "blast"])
def test_amr_conservation(ic):
    m = _amr_mesh()
    lv = m.leaves()
    if ic == "blast":
        U0 = inputs.blast(lv, N8, NRB4)
    else:
        U0 = np.empty(m.shape())
        for k, lf in enumerate(lv):
            x, y, z = inputs.cell_centers(lf, N8, NRB4)
            rho = 1.0 + 0.3 * np.sin(2 * np.pi * x) * np.sin(4 * np.pi * y + 0.3) * np.cos(2 * np.pi * z)
            vx = 0.4 * np.cos(2 * np.pi * y)
            vy = -0.3 * np.sin(2 * np.pi * z)
            vz = 0.2 * np.sin(2 * np.pi * x)
            p = 1.0 + 0.2 * np.cos(2 * np.pi * (x + y))
            U0[k] = [rho, rho * vx, rho * vy, rho * vz, p / (2 / 3) + 0.5 * rho * (vx * vx + vy * vy + vz * vz)]
    m.set_state(U0)
    T0, A0 = m.totals()
    m.step(10)
    T1, A1 = m.totals()
    A = np.maximum(A0, A1)  # momentum of the blast starts at exactly zero
    assert np.all(np.abs(T1 - T0) <= 1e-14 * A * 10), np.abs(T1 - T0) / A


def test_amr_wave_error_bracketed():
    """A sound wave through a two-level mesh: its error after a quarter
    period lies between the all-fine error and the all-coarse error at the
    same timestep (all levels share the fine level's dt, which makes the
    coarse cells run at half the Courant number)."""
    T = 0.25

    def run(leaves, max_level, cfl=0.3):
        m = OracleMesh(N8, NRB4, leaves, max_level=max_level, cfl=cfl)
        U0 = inputs.sound_wave(m.leaves(), N8, NRB4, amp=1e-6, noise=0.0)
        m.set_state(U0)
        while m.time()[0] < T:
            m.step(1, T)
        U = m.state()
        err, vol = 0.0, 0.0
        for k, lf in enumerate(m.leaves()):
            x, _, _ = inputs.cell_centers(lf, N8, NRB4)
            dV = (1.0 / (32 << int(lf[0]))) ** 3
            exact = 1.0 + 1e-6 * np.sin(2 * np.pi * (x - T))
            err += np.abs(U[k, 0] - exact).sum() * dV
            vol += x.size * dV
        assert abs(vol - 1.0) < 1e-12
        return err
    e_c = run(inputs.uniform_leaves(NRB4), 0, cfl=0.15)
    e_f = run([(1, x, y, z) for z in range(8) for y in range(8) for x in range(8)], 1)
    e_m = run(inputs.sphere_refined_leaves(NRB4, radius=0.2), 1)
    assert e_f < e_m < e_c, (e_f, e_m, e_c)


def test_regrid_round_trip_is_identity():
    nrb = (2, 2, 2)
    m = OracleMesh(N8, nrb, inputs.uniform_leaves(nrb), max_level=1)
    U0 = inputs.turbulent_box(m.leaves(), N8, nrb, seed=9)
    m.set_state(U0)
    T0, A0 = m.totals()
    m.regrid(np.ones(m.nleaves, dtype=np.int8))
    assert m.nleaves == 64 and set(m.leaves()[:, 0]) == {1}
    T1, _ = m.totals()
    assert np.all(np.abs(T1 - T0) <= 1e-15 * A0)
    m.regrid(-np.ones(m.nleaves, dtype=np.int8))
    assert m.nleaves == 8
    np.testing.assert_array_equal(m.leaves(), OracleMesh(N8, nrb, inputs.uniform_leaves(nrb)).leaves())
    U1 = m.state()
    assert np.abs(U1 - U0).max() <= 4 * np.finfo(float).eps * np.abs(U0).max()
    # the other order is not an identity on non-linear data
    m.regrid(np.ones(m.nleaves, dtype=np.int8))
    Uf = m.state().copy()
    m.regrid(-np.ones(m.nleaves, dtype=np.int8))
    m.regrid(np.ones(m.nleaves, dtype=np.int8))
    assert np.allclose(m.state(), Uf, rtol=1e-12)  # R(P(.)) = id on the coarse data
    m2 = OracleMesh(N8, nrb, [(1, x, y, z) for z in range(4) for y in range(4) for x in range(4)],
                    max_level=1)
    # leaves at level 1 of a 2-block root grid = a 4-block level-0 grid
    as_root = [(0, x, y, z) for _, x, y, z in m2.leaves()]
    Ufine = inputs.turbulent_box(as_root, N8, (4, 4, 4), seed=9)
    m2.set_state(Ufine)
    m2.regrid(-np.ones(m2.nleaves, dtype=np.int8))
    m2.regrid(np.ones(m2.nleaves, dtype=np.int8))
    assert np.abs(m2.state() - Ufine).max() > 1e-3  # P(R(f)) != f


def test_regrid_enforces_balance():
    """Refining a fine block at the edge of the refined region to level 2
    forces its coarse neighbours to level 1."""
    m = _amr_mesh(max_level=2)
    lv = m.leaves()
    flags = np.zeros(len(lv), dtype=np.int8)
    target = [k for k, lf in enumerate(lv) if tuple(lf) == (1, 2, 2, 2)][0]
    flags[target] = 1
    m.regrid(flags)
    new = {tuple(l) for l in m.leaves()}
    assert (2, 4, 4, 4) in new
    # the level-0 block (0, 0, 0, 0) touches the corner of (1, 2, 2, 2) and must now be refined
    assert (0, 0, 0, 0) not in new and (1, 1, 1, 1) in new
    assert all(l[0] <= 2 for l in new)
    # the mesh after regrid is a valid balanced tiling (re-creating it validates)
    OracleMesh(N8, NRB4, m.leaves(), max_level=2)


def test_derefine_rejected_when_unbalanced():
    m = _amr_mesh(max_level=2)
    lv = m.leaves()
    flags = np.zeros(len(lv), dtype=np.int8)
    # refine one fine block to level 2, derefine all fine blocks: the
    # sibling group containing the refined block cannot merge, nor can any
    # group touching the new level-2 blocks
    target = [k for k, lf in enumerate(lv) if tuple(lf) == (1, 2, 2, 2)][0]
    flags[lv[:, 0] == 1] = -1
    flags[target] = 1
    m.regrid(flags)
    new = m.leaves()
    assert (new[:, 0] == 2).sum() == 8
    assert (new[:, 0] == 1).sum() > 0
    OracleMesh(N8, NRB4, new, max_level=2)


def test_regrid_conserves_totals():
    m = _amr_mesh()
    m.set_state(inputs.blast(m.leaves(), N8, NRB4))
    m.step(3)
    T0, A0 = m.totals()
    lv = m.leaves()
    flags = np.where(lv[:, 0] == 1, -1, 1).astype(np.int8)
    m.regrid(flags)
    T1, _ = m.totals()
    assert np.all(np.abs(T1 - T0) <= 1e-14 * A0)


# ---------------------------------------------------------------------------
# Pressure-jump refinement indicator (the criterion the tests and the bench use)
# ---------------------------------------------------------------------------

def _pressure_state(m, pfun):
    """rho = 1 at rest with pressure pfun(x, y, z) at the cell centres."""
    U = np.zeros(m.shape())
    g1 = m.gamma - 1.0
    for b in range(m.nleaves):
        x, y, z = m.cell_centers(b)
        U[b, 0] = 1.0
        U[b, 4] = pfun(x, y, z) / g1
    return U


def test_pressure_jump_uniform_is_zero():
    m = _amr_mesh()
    m.set_state(_pressure_state(m, lambda x, y, z: 0.7 + 0 * x))
    assert np.all(m.pressure_jump() == 0.0)


def test_pressure_jump_linear_field_closed_form():
    # P = a + s x: |P(x+dx) - P(x-dx)| / (P(x+dx) + P(x-dx)) = s dx / (a + s x),
    # largest at the lowest cell centre of the leaf; exact ghosts of a linear
    # field (copy, restriction, prolongation) make this hold on both levels
    # away from the periodic seam in x
    a, s = 2.0, 0.75
    m = _amr_mesh()
    m.set_state(_pressure_state(m, lambda x, y, z: a + s * x))
    eta = m.pressure_jump()
    lv = m.leaves()
    checked = 0
    for b, (lev, lx, ly, lz) in enumerate(lv):
        nx = NRB4[0] << lev
        if lx == 0 or lx == nx - 1:
            continue
        dx = 1.0 / (NRB4[0] * N8[0] * (1 << lev))
        xlo = (lx * N8[0] + 0.5) * dx
        want = s * dx / (a + s * xlo)
        assert abs(eta[b] - want) <= 1e-13 * want, (b, eta[b], want)
        checked += 1
    assert checked > 40


def test_pressure_jump_step_and_flags():
    # a pressure step across x = 1/2 (a level-0 face): the leaves on both
    # sides of it see exactly |P2 - P1| / (P2 + P1)
    p1, p2 = 0.1, 100.0
    nrb = (4, 2, 2)
    m = OracleMesh(N8, nrb, inputs.uniform_leaves(nrb), xmax=(2.0, 1.0, 1.0))
    m.set_state(_pressure_state(m, lambda x, y, z: np.where(x < 1.0, p1, p2)))
    eta = m.pressure_jump()
    want = (p2 - p1) / (p2 + p1)
    lv = m.leaves()
    for b, (lev, lx, ly, lz) in enumerate(lv):
        assert eta[b] == want  # every leaf touches x = 1 or the periodic seam
    flags = np.where(eta > 0.1, 1, np.where(eta < 0.02, -1, 0))
    assert np.all(flags == 1)


def _density_state(m, rfun, p=1.3):
    """Uniform pressure at rest with density rfun(x, y, z) at the cell centres."""
    U = np.zeros(m.shape())
    for b in range(m.nleaves):
        x, y, z = m.cell_centers(b)
        U[b, 0] = rfun(x, y, z)
        U[b, 4] = p / (m.gamma - 1.0)
    return U


def test_density_jump_pins():
    """The density indicator: zero on a uniform density (pressure jumps do
    not enter), s dy / (a + s y) at the lowest cell of each leaf on a linear
    density a + s y (two levels, away from the periodic seam), and exactly
    |r2 - r1| / (r2 + r1) at a density step across a level-0 face."""
    m = _amr_mesh()
    U = _density_state(m, lambda x, y, z: 0.8 + 0 * x)
    U[:, 4] *= np.where(np.arange(m.nleaves) % 2 == 0, 1.0, 3.0)[:, None, None, None]
    m.set_state(U)
    assert np.all(m.density_jump() == 0.0)
    assert m.pressure_jump().max() > 0.1
    a, s = 1.5, 0.6
    m.set_state(_density_state(m, lambda x, y, z: a + s * y))
    eta = m.density_jump()
    checked = 0
    for b, (lev, lx, ly, lz) in enumerate(m.leaves()):
        ny = NRB4[1] << lev
        if ly == 0 or ly == ny - 1:
            continue
        dy = 1.0 / (NRB4[1] * N8[1] * (1 << lev))
        want = s * dy / (a + s * (ly * N8[1] + 0.5) * dy)
        assert abs(eta[b] - want) <= 1e-13 * want, (b, eta[b], want)
        checked += 1
    assert checked > 40
    r1, r2 = 1.0, 2.0
    nrb = (2, 4, 2)
    m = OracleMesh(N8, nrb, inputs.uniform_leaves(nrb), xmax=(1.0, 2.0, 1.0))
    m.set_state(_density_state(m, lambda x, y, z: np.where(y < 1.0, r1, r2)))
    assert np.all(m.density_jump() == (r2 - r1) / (r2 + r1))


def test_paper_multilevel_mesh_block_counts():
    """The leaf generator reproduces the paper's multilevel mesh (the cube
    centred in the box, 2:1 balance over face, edge and corner neighbours)."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "multilevel_mesh_blocks.json")))
    nrb = (g["root_cells"] // g["block"],) * 3
    half = g["cube_side"] / 2
    lv = inputs.cube_refined_leaves(nrb, 0.5 - half, 0.5 + half, g["max_level"])
    counts = [int((lv[:, 0] == L).sum()) for L in range(g["max_level"] + 1)]
    assert counts == g["blocks_per_level"]
    # a valid, 2:1-balanced tiling the oracle accepts (with blocks of 8^3)
    m = OracleMesh((8, 8, 8), nrb, lv, max_level=g["max_level"])
    assert m.nleaves == len(lv)


# ---------------------------------------------------------------------------
# Regrid: the data of new children (prolongation of the composite field at
# the parent's level) pinned by closed forms.
# ---------------------------------------------------------------------------

_COEF = np.array([[2.0, 0.7, -0.4, 0.3],   # per variable: a + b x + c y + d z
                  [0.3, -0.2, 0.5, 0.1],
                  [-0.1, 0.4, 0.2, -0.6],
                  [0.2, 0.1, -0.3, 0.45],
                  [5.0, 1.1, 0.9, -0.8]])


def _linear_state(m, lv, nrb):
    U = np.empty(m.shape())
    for k, lf in enumerate(lv):
        x, y, z = inputs.cell_centers(lf, N8, nrb)
        for v in range(5):
            a, b, c, d = _COEF[v]
            U[k, v] = a + b * x + c * y + d * z
    return U


def _away_from_seam(lf, nrb):
    """Mask [n3][n2][n1] of the cells of a new child whose parent cell and
    the parent's two neighbours along every axis lie inside the periodic
    domain without wrapping (the linear field has its seam at 0 = 1)."""
    lev = int(lf[0])
    masks = []
    for d in range(3):
        Nc = nrb[d] * N8[d] << (lev - 1)
        J = int(lf[1 + d]) * N8[d] + np.arange(N8[d])
        I = J >> 1
        masks.append((I >= 1) & (I <= Nc - 2))
    mz, my, mx = np.meshgrid(masks[2], masks[1], masks[0], indexing="ij")
    return mz & my & mx


def _check_children(m, new_leaves, nrb, want_fn):
    U = m.state()
    lv = m.leaves()
    idx = {tuple(int(v) for v in l): k for k, l in enumerate(lv)}
    checked = 0
    for lf in new_leaves:
        k = idx[tuple(lf)]
        ok = _away_from_seam(lf, nrb)
        want = want_fn(lf)
        err = np.abs(U[k][:, ok] - want[:, ok]).max()
        assert err <= 1e-13 * np.abs(want).max(), (lf, err)
        checked += int(ok.sum())
    return checked


def test_regrid_children_reproduce_linear_field():
    """Refining every leaf of a field linear in x, y and z: each child cell
    takes the field's value at its own centre (the minmod slopes of a linear
    field are its differences, and a fine centre sits a quarter coarse cell
    from its parent's centre along each axis). A flipped slope sign, a slope
    along the wrong axis or a half-cell offset all fail this."""
    nrb = (4, 4, 4)
    m = OracleMesh(N8, nrb, inputs.uniform_leaves(nrb), max_level=1)
    m.set_state(_linear_state(m, m.leaves(), nrb))
    m.regrid(np.ones(m.nleaves, dtype=np.int8))
    assert m.nleaves == 512
    new = [tuple(int(v) for v in l) for l in m.leaves()]

    def want(lf):
        x, y, z = inputs.cell_centers(lf, N8, nrb)
        return np.stack([a + b * x + c * y + d * z for a, b, c, d in _COEF])
    assert _check_children(m, new, nrb, want) > 100000


def test_regrid_children_next_to_other_levels():
    """Two-level mesh, linear field sampled at every leaf's cell centres. A
    coarse leaf beside the refined region is split (the slope stencils of
    its outer parent cells reach into finer leaves: composite value =
    restriction) and a fine leaf inside the refined region is split to level
    2 (stencils in other level-1 leaves): every child cell equals the field
    at its centre."""
    m = _amr_mesh(max_level=2)
    lv = m.leaves()
    m.set_state(_linear_state(m, lv, NRB4))
    flags = np.zeros(len(lv), dtype=np.int8)
    tgt = {(0, 0, 1, 1): None, (1, 3, 3, 3): None}
    for k, l in enumerate(lv):
        if tuple(int(v) for v in l) in tgt:
            flags[k] = 1
    assert flags.sum() == 2
    m.regrid(flags)
    new = [(1, 2 * 0 + (c & 1), 2 * 1 + ((c >> 1) & 1), 2 * 1 + ((c >> 2) & 1)) for c in range(8)]
    new += [(2, 6 + (c & 1), 6 + ((c >> 1) & 1), 6 + ((c >> 2) & 1)) for c in range(8)]
    have = {tuple(int(v) for v in l) for l in m.leaves()}
    assert set(new) <= have and m.nleaves == len(lv) + 14

    def want(lf):
        x, y, z = inputs.cell_centers(lf, N8, NRB4)
        return np.stack([a + b * x + c * y + d * z for a, b, c, d in _COEF])
    # the children of (0,0,1,1) at its +x face take slopes from the composite
    # value in the refined root block (1,1,1): they are among those checked
    assert _check_children(m, new, NRB4, want) > 3000


def test_regrid_children_minmod_slopes():
    """The slopes are minmod-limited one-sided differences of the parent
    level. On f = 1 + x^2 (refine all, coarse width h, parent centre xc > h)
    minmod takes the smaller difference 2 xc h - h^2, so a child is
    c0 + s (2 xc h - h^2) / 4 with s = -1 / +1 for the lower / upper child
    (a central slope would give s xc h / 2). At an asymmetric kink
    f = 1 + 2 (x - xk) for x > xk, 1 + (xk - x) below, with xk a parent
    centre, the one-sided differences have opposite signs: both children of
    that parent keep its value."""
    nrb = (4, 1, 1)
    h = 1.0 / (nrb[0] * N8[0])

    def run(fx):
        m = OracleMesh(N8, nrb, inputs.uniform_leaves(nrb), max_level=1)
        U = np.zeros(m.shape())
        for k, lf in enumerate(m.leaves()):
            x, _, _ = inputs.cell_centers(lf, N8, nrb)
            U[k] = fx(x)[None]
        m.set_state(U)
        m.regrid(np.ones(m.nleaves, dtype=np.int8))
        xs, vals = [], []
        for k, lf in enumerate(m.leaves()):
            if lf[2] or lf[3]:
                continue  # one row of leaves along x
            x, _, _ = inputs.cell_centers(lf, N8, nrb)
            xs.append(x[0, 0])
            vals.append(m.state()[k, :, 0, 0])
        x = np.concatenate(xs)
        v = np.concatenate(vals, axis=1)
        o = np.argsort(x)
        return x[o], v[:, o]

    x, v = run(lambda x: 1.0 + x * x)
    I = np.floor(x / h).astype(int)
    xc = (I + 0.5) * h
    s = np.where(x > xc, 1.0, -1.0)
    sel = (I >= 1) & (I <= nrb[0] * N8[0] - 2)
    want = 1.0 + xc * xc + s * (2 * xc * h - h * h) / 4
    assert np.abs(v[:, sel] - want[sel]).max() <= 1e-14
    xk = 13.5 * h

    def kink(x):
        return 1.0 + np.where(x > xk, 2.0 * (x - xk), xk - x)
    x, v = run(kink)
    I = np.floor(x / h).astype(int)
    at = I == 13
    assert at.sum() == 2 and np.all(v[:, at] == 1.0)
    near = (I >= 1) & (I <= nrb[0] * N8[0] - 2) & ~at & (np.abs(I - 13) > 0)
    assert np.abs(v[:, near] - kink(x[near])).max() <= 1e-14
