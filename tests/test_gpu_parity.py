"""Parity of the HIP path against the CPU oracle, element by element, on
seeded inputs; invariants that hold at any size. Runs on an MI355X."""
import math

import numpy as np
import pytest

from _helpers import print_case, rel_err, rel_err_per_variable
from oracle.oracle import OracleMesh
from paper_2202_12309_amd import inputs

pytestmark = pytest.mark.gpu
G = 5.0 / 3.0


def _pair(nroot, n, leaves, max_level=0, **kw):
    from paper_2202_12309_amd.binding import Mesh
    nrb = tuple(nroot[d] // n[d] for d in range(3))
    gm = Mesh(nroot, n, leaves, max_level=max_level, **kw)
    kw.pop("graph", None)
    om = OracleMesh(n, nrb, leaves, max_level=max_level, **kw)
    assert np.array_equal(gm.leaves(), om.leaves())  # same Morton storage order
    return gm, om, nrb


def _run_both(gm, om, U0, cycles, t_end=math.inf):
    gm.upload(U0)
    om.set_state(U0)
    gm.step(cycles, t_end)
    om.step(cycles, t_end)
    return gm.download(), om.state()


def test_upload_download_round_trip_bitwise():
    print_case("round trip 32^3 8x16^3")
    n = (16, 16, 16)
    gm, om, nrb = _pair((32, 32, 32), n, inputs.uniform_leaves((2, 2, 2)))
    U0 = inputs.turbulent_box(gm.leaves(), n, nrb, seed=3)
    gm.upload(U0)
    assert np.array_equal(gm.download(), U0)


@pytest.mark.parametrize("blk", [8, 16, 32, 64])
def test_uniform_state_preserved_bitwise(blk):
    print_case(f"uniform preservation blk={blk}")
    N = 64
    n = (blk, blk, blk)
    nrb = (N // blk,) * 3
    gm, om, _ = _pair((N, N, N), n, inputs.uniform_leaves(nrb))
    U0 = inputs.uniform_state(gm.leaves(), n, rho=1.37, v=(0.31, -0.52, 0.11), p=0.83)
    gm.upload(U0)
    gm.step(3)
    assert np.array_equal(gm.download(), U0)


@pytest.mark.parametrize("cycles,tol", [(1, 1e-12), (10, 1e-12)])
def test_sound_wave_64cube_8_blocks(cycles, tol):
    """64^3 periodic as 8 blocks of 32^3: sound wave amplitude 1e-6 plus
    white noise 1e-8, gamma 5/3, CFL 0.3."""
    print_case(f"sound wave 64^3 cycles={cycles}")
    n = (32, 32, 32)
    gm, om, nrb = _pair((64, 64, 64), n, inputs.uniform_leaves((2, 2, 2)))
    U0 = inputs.sound_wave(gm.leaves(), n, nrb, seed=1)
    Ug, Uo = _run_both(gm, om, U0, cycles)
    err = rel_err(Ug, Uo, G)
    # the same difference against each variable's own largest value: the
    # wave's momentum along x is ~1e-6 and the transverse momenta are the
    # 1e-8 noise alone, while the rounding of the momentum update is set by
    # the pressure term of the momentum flux (~rho c, six to eight orders of
    # magnitude larger); measured 6e-10 / 1.5e-8 after 1 cycle and 1.5e-9 /
    # 9e-8 after 10 for M_x / the transverse momenta
    err_own = rel_err_per_variable(Ug, Uo)
    print("rel err (momentum scale max(|M|, rho c))", err)
    print("rel err (per-variable scale max |b|)", err_own)
    assert np.all(err <= tol), err
    assert err_own[0] <= tol and err_own[4] <= tol, err_own
    assert err_own[1] <= 1e-8 and np.all(err_own[2:4] <= 1e-6), err_own
    tg, dtg, cg = gm.time()
    to, _, co = om.time()
    assert cg == co == cycles
    assert abs(tg - to) <= 1e-14 * to
    assert abs(dtg - om.dt()) <= 1e-14 * dtg
    Tg = gm.totals()
    To, Ao = om.totals()
    assert np.all(np.abs(Tg - To) <= 1e-13 * Ao + 1e-300), (Tg - To) / Ao


@pytest.mark.parametrize("blk", [8, 16, 32, 64])
def test_turbulent_box_block_sizes(blk):
    """Log-normal density, rms Mach 0.5: one recipe, four block sizes."""
    print_case(f"turbulent box 64^3 blk={blk}")
    N = 64
    n = (blk, blk, blk)
    nrb = (N // blk,) * 3
    gm, om, _ = _pair((N, N, N), n, inputs.uniform_leaves(nrb))
    U0 = inputs.turbulent_box(gm.leaves(), n, nrb, seed=2)
    Ug, Uo = _run_both(gm, om, U0, 3)
    err = rel_err(Ug, Uo, G)
    print("rel err", err)
    assert np.all(err <= 1e-12), err


def test_turbulent_box_100_cycles():
    print_case("turbulent box 32^3 8x16^3 100 cycles")
    n = (16, 16, 16)
    gm, om, nrb = _pair((32, 32, 32), n, inputs.uniform_leaves((2, 2, 2)))
    U0 = inputs.turbulent_box(gm.leaves(), n, nrb, seed=2)
    Ug, Uo = _run_both(gm, om, U0, 100)
    err = rel_err(Ug, Uo, G)
    print("rel err", err)
    assert np.all(err <= 1e-9), err
    assert abs(gm.time()[0] - om.time()[0]) <= 1e-12 * om.time()[0]


def test_rk2_variant_plm_predictor():
    print_case("stage-1 PLM variant")
    n = (16, 16, 16)
    gm, om, nrb = _pair((32, 32, 32), n, inputs.uniform_leaves((2, 2, 2)), stage1_recon=1)
    U0 = inputs.turbulent_box(gm.leaves(), n, nrb, seed=4)
    Ug, Uo = _run_both(gm, om, U0, 3)
    assert np.all(rel_err(Ug, Uo, G) <= 1e-12)


def test_t_end_clamp():
    print_case("t_end clamp")
    n = (16, 16, 16)
    gm, om, nrb = _pair((32, 32, 32), n, inputs.uniform_leaves((2, 2, 2)))
    U0 = inputs.sound_wave(gm.leaves(), n, nrb)
    Ug, Uo = _run_both(gm, om, U0, 6, t_end=0.02)
    assert gm.time()[0] == pytest.approx(0.02, rel=1e-15)
    assert np.all(rel_err(Ug, Uo, G) <= 1e-12)


def test_graph_replay_equals_eager():
    print_case("graph replay vs eager")
    from paper_2202_12309_amd.binding import Mesh
    n = (16, 16, 16)
    lv = inputs.uniform_leaves((2, 2, 2))
    U0 = inputs.turbulent_box(lv, n, (2, 2, 2), seed=6)
    a = Mesh((32, 32, 32), n, lv)
    b = Mesh((32, 32, 32), n, lv, graph=True)
    a.upload(U0)
    b.upload(U0)
    for rep in range(3):  # several replays with host work in between
        a.step(4)
        b.step(4)
        assert np.array_equal(a.download(), b.download()), rep
        assert a.time() == b.time()


def test_graph_replay_equals_eager_two_levels_with_regrid():
    """Multilevel cycle (flux correction and level-jump face fill in the
    captured graph), replayed several times, then a regrid (the graph is
    rebuilt for the new mesh) and more replays: bitwise equal to eager."""
    print_case("graph replay vs eager, two levels, regrid")
    from paper_2202_12309_amd.binding import Mesh
    nrb, n = (4, 4, 4), (8, 8, 8)
    lv = inputs.sphere_refined_leaves(nrb, radius=0.3)
    a = Mesh((32, 32, 32), n, lv, max_level=1)
    b = Mesh((32, 32, 32), n, lv, max_level=1, graph=True)
    U0 = inputs.blast(a.leaves(), n, nrb)
    a.upload(U0)
    b.upload(U0)
    for rep in range(3):
        a.step(3)
        b.step(3)
        assert np.array_equal(a.download(), b.download()), rep
        assert a.time() == b.time()
    fa, _ = a.flag_pressure_jump(0.1, 0.02)
    fb, _ = b.flag_pressure_jump(0.1, 0.02)
    assert np.array_equal(fa, fb)
    a.regrid()
    b.regrid()
    assert np.array_equal(a.leaves(), b.leaves())
    for rep in range(2):
        a.step(3)
        b.step(3)
        assert np.array_equal(a.download(), b.download()), rep


def test_deterministic_repeat():
    print_case("determinism")
    from paper_2202_12309_amd.binding import Mesh
    n = (32, 32, 32)
    lv = inputs.uniform_leaves((2, 2, 2))
    U0 = inputs.turbulent_box(lv, n, (2, 2, 2), seed=8)
    outs = []
    for _ in range(2):
        m = Mesh((64, 64, 64), n, lv)
        m.upload(U0)
        m.step(5)
        outs.append((m.download(), m.totals(), m.time()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]


def test_unphysical_state_latched():
    print_case("EPHYS latch")
    from paper_2202_12309_amd.binding import Mesh, PkhError
    n = (16, 16, 16)
    lv = inputs.uniform_leaves((1, 1, 1))
    m = Mesh((16, 16, 16), n, lv)
    U = inputs.uniform_state(lv, n)
    U[0, 4, 3, 3, 3] = -1.0
    m.upload(U)
    m.step(1)
    with pytest.raises(PkhError) as e:
        m.sync()
    assert e.value.name == "PKH_EPHYS"
    m.upload(inputs.uniform_state(lv, n))  # the latch clears on upload
    m.step(1)
    m.sync()


def test_invalid_meshes_rejected():
    print_case("invalid meshes")
    from paper_2202_12309_amd.binding import Mesh, PkhError
    n = (8, 8, 8)
    lv = inputs.uniform_leaves((2, 2, 2)).tolist()
    with pytest.raises(PkhError) as e:
        Mesh((16, 16, 16), n, lv[:-1])
    assert e.value.name == "PKH_ETILING"
    with pytest.raises(PkhError) as e:
        Mesh((16, 16, 16), (12, 8, 8), lv)
    assert e.value.name == "PKH_EINVAL"


# ---------------------------------------------------------------------------
# Multilevel meshes
# ---------------------------------------------------------------------------

def _amr_pair(nrb=(4, 4, 4), n=(16, 16, 16), radius=0.2, max_level=1):
    leaves = inputs.sphere_refined_leaves(nrb, radius=radius)
    nroot = tuple(nrb[d] * n[d] for d in range(3))
    return _pair(nroot, n, leaves, max_level=max_level)


@pytest.mark.parametrize("cycles", [1, 10])
def test_amr_blast_parity(cycles):
    print_case(f"AMR blast cycles={cycles}")
    gm, om, nrb = _amr_pair()
    U0 = inputs.blast(gm.leaves(), gm.n, nrb)
    Ug, Uo = _run_both(gm, om, U0, cycles)
    err = rel_err(Ug, Uo, G)
    print("rel err", err)
    assert np.all(err <= 1e-12), err
    To, Ao = om.totals()
    Tg = gm.totals()
    assert np.all(np.abs(Tg - To) <= 1e-13 * np.maximum(Ao, 1.0))


def test_amr_uniform_preserved_and_conservative():
    print_case("AMR uniform + conservation")
    gm, om, nrb = _amr_pair(n=(8, 8, 8))
    U0 = inputs.uniform_state(gm.leaves(), gm.n, rho=1.37, v=(0.31, -0.52, 0.11), p=0.83)
    gm.upload(U0)
    gm.step(3)
    assert np.array_equal(gm.download(), U0)
    U1 = inputs.sound_wave(gm.leaves(), gm.n, nrb, amp=1e-2, noise=1e-3)
    gm.upload(U1)
    om.set_state(U1)
    T0, A0 = om.totals()
    gm.step(10)
    T1 = gm.totals()
    assert np.all(np.abs(T1 - T0) <= 1e-14 * 10 * A0)


def test_amr_regrid_parity():
    print_case("AMR regrid")
    gm, om, nrb = _amr_pair(n=(8, 8, 8), max_level=2)
    U0 = inputs.blast(gm.leaves(), gm.n, nrb)
    Ug, Uo = _run_both(gm, om, U0, 2)
    lv = om.leaves()
    flags = np.zeros(len(lv), dtype=np.int8)
    flags[lv[:, 0] == 1] = -1
    flags[[k for k, l in enumerate(lv) if tuple(l) == (1, 3, 3, 3)]] = 1
    flags[[k for k, l in enumerate(lv) if tuple(l) == (0, 0, 0, 0)]] = 1
    gm.regrid(flags)
    om.regrid(flags)
    assert np.array_equal(gm.leaves(), om.leaves())
    Ug, Uo = gm.download(), om.state()
    assert np.all(rel_err(Ug, Uo, G) <= 1e-12)
    gm.step(3)
    om.step(3)
    assert np.all(rel_err(gm.download(), om.state(), G) <= 1e-12)


def test_packs_do_not_change_results():
    """One stage launch per pack of contiguous leaves (the paper's
    MeshBlockPacks) gives bitwise the result of one launch over every leaf,
    on a two-level mesh with flux correction and level-jump fills, and
    packs beyond the leaf count are clamped to one leaf per pack."""
    print_case("packs 1 / 3 / 7 / leaf count, two-level blast 64^3 root in 16^3 blocks, 5 cycles")
    from paper_2202_12309_amd.binding import Mesh, PkhError
    n, nrb = (16, 16, 16), (4, 4, 4)
    lv = inputs.sphere_refined_leaves(nrb, radius=0.3)
    outs = []
    for P in (1, 3, 7, 100000):
        gm = Mesh((64, 64, 64), n, lv, max_level=1)
        gm.set_tuning(0, P)
        assert gm.tuning()["packs"] == P
        gm.upload(inputs.blast(gm.leaves(), n, nrb))
        gm.step(5)
        outs.append(gm.download())
        gm.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    # and the packed runs equal the oracle's run of the same mesh
    om = OracleMesh(n, nrb, lv, max_level=1)
    om.set_state(inputs.blast(om.leaves(), n, nrb))
    om.step(5)
    err = rel_err(outs[1], om.state(), G)
    print("3 packs vs oracle, rel err", err, flush=True)
    assert np.all(err <= 5e-11), err
    gm = Mesh((64, 64, 64), n, lv, max_level=1)
    with pytest.raises(PkhError):
        gm.set_tuning(0, -1)
    gm.close()


@pytest.mark.parametrize("case", ["uniform32", "two_level16", "fp32_16"])
def test_tile_rows_do_not_change_results(case):
    """Every compiled tile shape gives bitwise the same state: a face shared
    by two tiles (or two blocks) is solved by the lower-face job of one and
    the upper-face job of the other, and both must round identically. Covers
    32^3 blocks (turbulent box), a two-level blast in 16^3 blocks (fine-coarse
    face fluxes written from both jobs, flux correction) and FP32 storage."""
    print_case(f"tile rows 4 / 8 / 16, {case}, 6 cycles")
    from paper_2202_12309_amd.binding import Mesh
    if case == "uniform32":
        n, nrb, N, lv, ml = (32, 32, 32), (2, 2, 2), 64, inputs.uniform_leaves((2, 2, 2)), 0
    elif case == "two_level16":
        n, nrb, N, ml = (16, 16, 16), (4, 4, 4), 64, 1
        lv = inputs.sphere_refined_leaves(nrb, radius=0.3)
    else:
        n, nrb, N, lv, ml = (16, 16, 16), (2, 2, 2), 32, inputs.uniform_leaves((2, 2, 2)), 0
    fp32 = case == "fp32_16"
    outs = []
    for tj in ((8, 16) if fp32 else (4, 8, 16)):
        gm = Mesh((N, N, N), n, lv, max_level=ml, fp32_state=fp32)
        gm.set_tuning(tj)
        assert gm.tuning()["tile_rows"] == tj
        if case == "two_level16":
            gm.upload(inputs.blast(gm.leaves(), n, nrb))
        else:
            gm.upload(inputs.turbulent_box(gm.leaves(), n, nrb, seed=2))
        gm.step(6)
        outs.append((gm.download(), gm.time()))
        gm.close()
    for U, t in outs[1:]:
        assert np.array_equal(U, outs[0][0])
        assert t == outs[0][1]


def test_full_size_bench_configuration_parity():
    """The bench workload itself: 256^3 in 512 blocks of 32^3, the default
    launch tiles (8 rows for the corrector, 16 for the predictor), against the oracle
    element by element after 1, 10 and 100 cycles (about a minute of oracle
    time on 16 threads); clock and totals too."""
    print_case("256^3 turbulent box, 512 blocks of 32^3, bench launch configuration, 100 cycles")
    n, N = (32, 32, 32), 256
    gm, om, nrb = _pair((N, N, N), n, inputs.uniform_leaves((8, 8, 8)))
    assert gm.tuning()["tile_rows"] == 8  # the corrector's default on 32-cell rows
    U0 = inputs.turbulent_box(gm.leaves(), n, nrb, seed=2)
    gm.upload(U0)
    om.set_state(U0)
    done = 0
    for upto, tol in ((1, 1e-12), (10, 1e-11), (100, 1e-9)):
        gm.step(upto - done)
        om.step(upto - done)
        done = upto
        err = rel_err(gm.download(), om.state(), G)
        print(f"cycle {upto}: rel err {err}", flush=True)
        assert np.all(err <= tol), (upto, err)
    assert abs(gm.time()[0] - om.time()[0]) <= 1e-12 * om.time()[0]
    To, Ao = om.totals()
    assert np.all(np.abs(gm.totals() - To) <= 1e-13 * np.maximum(Ao, 1.0))


@pytest.mark.parametrize("n,nrb,ml", [((32, 16, 8), (4, 2, 2), 0), ((16, 8, 8), (2, 4, 1), 0),
                                      ((64, 8, 4), (1, 2, 3), 0), ((16, 16, 8), (2, 1, 2), 1)])
def test_ragged_blocks_and_domains(n, nrb, ml):
    """Blocks that are not cubes in domains that are not cubes (edges 4 to
    64 cells, a single block along a direction, an odd number of blocks),
    and a two-level mesh of flat blocks: against the oracle after 3 cycles."""
    print_case(f"ragged blocks {n} x {nrb}, max level {ml}, 3 cycles")
    nroot = tuple(n[d] * nrb[d] for d in range(3))
    xmax = tuple(float(nroot[d]) / nroot[0] for d in range(3))  # cubic cells
    lv = inputs.uniform_leaves(nrb)
    if ml:
        lv = [l for l in lv.tolist() if l != [0, 0, 0, 0]]
        lv += [[1, c & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)]
    gm, om, _ = _pair(nroot, n, lv, max_level=ml, xmax=xmax)
    U0 = inputs.turbulent_box(gm.leaves(), n, nrb, seed=5) if not ml else \
        inputs.blast(gm.leaves(), n, nrb, center=(0.3, 0.2, 0.4), r=0.15, xmax=xmax)
    Ug, Uo = _run_both(gm, om, U0, 3)
    err = rel_err(Ug, Uo, G)
    print("rel err", err, flush=True)
    assert np.all(err <= 1e-12), err


def test_zero_cycles_is_a_no_op():
    print_case("step(0)")
    n = (16, 16, 16)
    gm, om, nrb = _pair((32, 32, 32), n, inputs.uniform_leaves((2, 2, 2)))
    U0 = inputs.turbulent_box(gm.leaves(), n, nrb, seed=7)
    gm.upload(U0)
    gm.step(0)
    assert np.array_equal(gm.download(), U0)
    t, _, cyc = gm.time()
    assert t == 0.0 and cyc == 0
