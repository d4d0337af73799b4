"""Outflow and reflecting domain boundaries on the HIP path against the
oracle: one and two levels, regridding next to walls, the indicator at a
wall, and what the library accepts or refuses. Runs on an MI355X."""
import numpy as np
import pytest

from _helpers import print_case, rel_err
from oracle.oracle import BC_OUTFLOW as OUT
from oracle.oracle import BC_PERIODIC as PER
from oracle.oracle import BC_REFLECT as REF
from oracle.oracle import OracleMesh
from paper_2202_12309_amd import inputs

pytestmark = pytest.mark.gpu
G = 5.0 / 3.0
REFINE, DEREFINE = 0.1, 0.02


def _pair(nrb, n, leaves, bc, max_level=0, **kw):
    from paper_2202_12309_amd.binding import Mesh
    gm = Mesh(tuple(nrb[d] * n[d] for d in range(3)), n, leaves, max_level=max_level, bc=bc, **kw)
    om = OracleMesh(n, nrb, leaves, max_level=max_level, bc=bc)
    assert np.array_equal(gm.leaves(), om.leaves())
    return gm, om


def _compare(gm, om, cycles, per_cycle=1e-12):
    for c in range(1, cycles + 1):
        gm.step(1)
        om.step(1)
        if c in (1, 2, 5) or c == cycles:
            err = rel_err(gm.download(), om.state(), G)
            print(f"cycle {c}: rel err {err}", flush=True)
            assert np.all(err <= per_cycle * c), (c, err)
    To, Ao = om.totals()
    assert np.all(np.abs(gm.totals() - To) <= 1e-13 * np.maximum(Ao, 1.0))


@pytest.mark.parametrize("bc", [(REF, REF, OUT, OUT, PER, PER), (OUT, REF, PER, PER, REF, OUT),
                                (REF,) * 6, (OUT,) * 6])
def test_walls_single_level_parity(bc):
    print_case(f"walls {bc}, 64^3 as 8 blocks of 32^3, smooth flow, 10 cycles")
    n, nrb = (32, 32, 32), (2, 2, 2)
    gm, om = _pair(nrb, n, inputs.uniform_leaves(nrb), bc)
    U0 = inputs.smooth_flow(gm.leaves(), n, nrb)
    gm.upload(U0)
    om.set_state(U0)
    _compare(gm, om, 10)


@pytest.mark.parametrize("blk", [8, 16, 64])
def test_walls_block_sizes(blk):
    print_case(f"reflect x / outflow y, blocks of {blk}^3, 3 cycles")
    n = (blk,) * 3
    nrb = (2, 2, 2) if blk < 64 else (1, 1, 2)
    bc = (REF, REF, OUT, OUT, PER, PER)
    gm, om = _pair(nrb, n, inputs.uniform_leaves(nrb), bc)
    U0 = inputs.smooth_flow(gm.leaves(), n, nrb)
    gm.upload(U0)
    om.set_state(U0)
    _compare(gm, om, 3)


def test_walls_stage1_plm_variant():
    print_case("walls, stage-1 PLM variant, 32^3 as 8 blocks of 16^3, 5 cycles")
    n, nrb = (16, 16, 16), (2, 2, 2)
    bc = (OUT, OUT, REF, REF, REF, OUT)
    from paper_2202_12309_amd.binding import Mesh
    lv = inputs.uniform_leaves(nrb)
    gm = Mesh((32, 32, 32), n, lv, bc=bc, stage1_recon=1)
    om = OracleMesh(n, nrb, lv, bc=bc, stage1_recon=1)
    U0 = inputs.smooth_flow(gm.leaves(), n, nrb)
    gm.upload(U0)
    om.set_state(U0)
    _compare(gm, om, 5)


def _wall_refined_leaves():
    """Root blocks (2,2,2) of 16^3; the two diagonal roots touching the
    x- and x+ walls refined once."""
    lv = [[0, x, y, z] for z in range(2) for y in range(2) for x in range(2)
          if (x, y, z) not in ((0, 0, 0), (1, 1, 1))]
    for (x, y, z) in ((0, 0, 0), (1, 1, 1)):
        lv += [[1, 2 * x + (c & 1), 2 * y + ((c >> 1) & 1), 2 * z + ((c >> 2) & 1)] for c in range(8)]
    return lv


@pytest.mark.parametrize("bc", [(REF, REF, PER, PER, PER, PER), (OUT, REF, REF, OUT, OUT, REF)])
def test_walls_two_levels_parity(bc):
    """Refined blocks touch walls: prolongation stencils reach past the wall
    at the coarse level and fine-coarse faces end at the wall."""
    print_case(f"walls {bc}, two levels touching the walls, 16^3 blocks, 10 cycles")
    n, nrb = (16, 16, 16), (2, 2, 2)
    gm, om = _pair(nrb, n, _wall_refined_leaves(), bc, max_level=1)
    U0 = inputs.smooth_flow(gm.leaves(), n, nrb)
    gm.upload(U0)
    om.set_state(U0)
    _compare(gm, om, 10)


def test_walls_regrid_parity():
    """A blast next to a reflecting corner, regridded every 5 cycles with the
    oracle's flags on both sides: the tree logic and the data moves stop at
    walls the same way on both."""
    print_case("blast at a reflecting corner, 64^3 root in 16^3 blocks, regrid every 5, 20 cycles")
    n, nrb = (16, 16, 16), (4, 4, 4)
    bc = (REF, OUT, REF, OUT, PER, PER)
    lv = inputs.sphere_refined_leaves(nrb, center=(0.1, 0.1, 0.5), radius=0.2)
    gm, om = _pair(nrb, n, lv, bc, max_level=1)
    U0 = inputs.blast(gm.leaves(), n, nrb, center=(0.1, 0.1, 0.5))
    gm.upload(U0)
    om.set_state(U0)
    sizes = []
    for s in range(4):
        gm.step(5)
        om.step(5)
        c = 5 * (s + 1)
        err = rel_err(gm.download(), om.state(), G)
        print(f"cycle {c}: leaves {gm.nleaves}, rel err {err}", flush=True)
        assert np.all(err <= 1e-11 * c), (c, err)
        eo = om.pressure_jump()
        fg, eg = gm.flag_pressure_jump(REFINE, DEREFINE)
        assert np.all(np.abs(eg - eo) <= 1e-10 * np.maximum(eo, 1e-3))
        flags = np.where(eo > REFINE, 1, np.where(eo < DEREFINE, -1, 0)).astype(np.int8)
        gm.regrid(flags)
        om.regrid(flags)
        assert np.array_equal(gm.leaves(), om.leaves())
        sizes.append(gm.nleaves)
    assert len(set(sizes)) > 1 or sizes[0] != len(lv)


def test_outflow_uniform_flow_bitwise_two_levels():
    print_case("outflow walls, uniform flow, two levels, 5 cycles")
    n, nrb = (16, 16, 16), (2, 2, 2)
    from paper_2202_12309_amd.binding import Mesh
    lv = _wall_refined_leaves()
    gm = Mesh((32, 32, 32), n, lv, max_level=1, bc=(OUT,) * 6)
    U0 = inputs.uniform_state(gm.leaves(), n, rho=1.2, v=(0.4, -0.3, 0.2), p=0.9)
    gm.upload(U0)
    gm.step(5)
    assert np.array_equal(gm.download(), U0)


def test_wall_meshes_accepted_and_refused():
    from paper_2202_12309_amd.binding import Batch, Mesh, PkhError
    n, nrb = (8, 8, 8), (2, 1, 1)
    # level-2 leaves next to x = 0 and a level-0 root at x = 1/2: two levels
    # apart across the periodic x boundary, no neighbours across walls
    lv = [[0, 1, 0, 0]]
    for c in range(8):
        cx, cy, cz = c & 1, (c >> 1) & 1, (c >> 2) & 1
        if cx == 0:
            lv += [[2, 2 * cx + (g & 1), 2 * cy + ((g >> 1) & 1), 2 * cz + ((g >> 2) & 1)] for g in range(8)]
        else:
            lv.append([1, cx, cy, cz])
    with pytest.raises(PkhError):
        Mesh((16, 8, 8), n, lv, max_level=2)
    Mesh((16, 8, 8), n, lv, max_level=2, bc=(OUT, OUT, PER, PER, PER, PER)).close()
    with pytest.raises(PkhError):
        Mesh((16, 8, 8), n, lv, max_level=2, bc=(PER, OUT, PER, PER, PER, PER))
    with pytest.raises(PkhError):
        Mesh((16, 8, 8), n, lv, max_level=2, bc=(3, 3, PER, PER, PER, PER))
    # reverse mode and batches take walled meshes (the face-wise reverse);
    # the pencil/row reverse is refused there
    wm = Mesh((16, 16, 16), n, inputs.uniform_leaves((2, 2, 2)), bc=(REF,) * 6)
    tp = wm.tape(2)
    with pytest.raises(PkhError):
        tp.set_facewise(False)
    tp.close()
    Batch([wm]).close()
    wm.close()
