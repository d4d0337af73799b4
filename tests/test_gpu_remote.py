"""The multi-GPU data path forced on one GPU: a virtual partition whose
same-level faces between parts go through pack, one transfer per (sender,
receiver) message and unpack, against the oracle element by element and
against the direct reads of an unpartitioned mesh (bitwise) on one and two
levels, with walls, through regrids and graph replays. Runs on an MI355X."""
import numpy as np
import pytest

from _helpers import print_case, rel_err
from oracle.oracle import OracleMesh
from oracle.oracle import BC_OUTFLOW as OUT
from oracle.oracle import BC_PERIODIC as PER
from oracle.oracle import BC_REFLECT as REF
from paper_2202_12309_amd import inputs

pytestmark = pytest.mark.gpu
G = 5.0 / 3.0


def _mesh(lv, nrb, n, nparts=1, **kw):
    from paper_2202_12309_amd.binding import Mesh
    m = Mesh(tuple(nrb[d] * n[d] for d in range(3)), n, lv, **kw)
    if nparts > 1:
        m.set_partition(nparts)
    return m


@pytest.mark.parametrize("nparts", [2, 5, 64])
def test_partition_bitwise_uniform(nparts):
    print_case(f"partition {nparts}, 64^3 as 64 blocks of 16^3, turbulent box, 5 cycles")
    n, nrb = (16, 16, 16), (4, 4, 4)
    lv = inputs.uniform_leaves(nrb)
    ref = _mesh(lv, nrb, n)
    U0 = inputs.turbulent_box(ref.leaves(), n, nrb, seed=3)
    ref.upload(U0)
    ref.step(5)
    m = _mesh(lv, nrb, n, nparts)
    info = m.partition()
    assert info["nparts"] == nparts and info["remote_faces"] > 0
    if nparts == 64:  # every face of every block is remote
        assert info["remote_faces"] == 64 * 6
    m.upload(U0)
    m.kernel_timing(m.KT_REMOTE)
    m.step(5)
    assert m.kernel_times()["remote"][1] == 10  # one exchange per stage
    assert np.array_equal(m.download(), ref.download())
    assert np.array_equal(m.flag_pressure_jump(0.1, 0.02)[1], ref.flag_pressure_jump(0.1, 0.02)[1])


def test_partition_matches_oracle_uniform():
    """5 parts of 64 blocks of 16^3 (turbulent box): within 1e-12 of the
    oracle after 1 cycle and 1e-11 after 5."""
    print_case("partition 5 vs oracle, 64^3 as 64 blocks of 16^3, 1 + 4 cycles")
    n, nrb = (16, 16, 16), (4, 4, 4)
    lv = inputs.uniform_leaves(nrb)
    m = _mesh(lv, nrb, n, 5)
    om = OracleMesh(n, nrb, m.leaves())
    U0 = inputs.turbulent_box(m.leaves(), n, nrb, seed=3)
    m.upload(U0)
    om.set_state(U0)
    for cyc, tol in ((1, 1e-12), (4, 1e-11)):
        m.step(cyc)
        om.step(cyc)
        err = rel_err(m.download(), om.state(), G)
        print("rel err", err, flush=True)
        assert np.all(err <= tol), err


def test_partition_matches_oracle_two_levels_with_regrid():
    """3 parts of a two-level blast (64^3 root in 16^3 blocks), 5 cycles, a
    regrid with the oracle's pressure-jump flags applied to both sides (the
    partition is recut over the new leaves), 5 more cycles: within 1e-11 per
    cycle of the oracle, identical leaves, totals to 1e-13."""
    print_case("partition 3 vs oracle, two-level blast 64^3 root in 16^3 blocks, regrid")
    n, nrb = (16, 16, 16), (4, 4, 4)
    lv = inputs.sphere_refined_leaves(nrb, radius=0.3)
    m = _mesh(lv, nrb, n, 3, max_level=1)
    om = OracleMesh(n, nrb, m.leaves(), max_level=1)
    U0 = inputs.blast(m.leaves(), n, nrb)
    m.upload(U0)
    om.set_state(U0)
    for seg in range(2):
        m.step(5)
        om.step(5)
        c = 5 * (seg + 1)
        err = rel_err(m.download(), om.state(), G)
        print(f"cycle {c}: leaves {m.nleaves}, rel err {err}", flush=True)
        assert np.all(err <= 1e-11 * c), err
        To, Ao = om.totals()
        assert np.all(np.abs(m.totals() - To) <= 1e-13 * np.maximum(Ao, 1.0))
        if seg == 0:
            eta = om.pressure_jump()
            flags = np.where(eta > 0.1, 1, np.where(eta < 0.02, -1, 0)).astype(np.int8)
            m.regrid(flags)
            om.regrid(flags)
            assert np.array_equal(m.leaves(), om.leaves())
            assert m.partition()["nparts"] == 3


def test_partition_bitwise_two_levels_with_regrid_and_graph():
    print_case("partition 3, two-level blast 64^3 root in 16^3 blocks, regrid, graph replay")
    n, nrb = (16, 16, 16), (4, 4, 4)
    lv = inputs.sphere_refined_leaves(nrb, radius=0.3)
    outs = []
    for nparts, graph in ((1, False), (3, False), (3, True)):
        m = _mesh(lv, nrb, n, nparts, max_level=1, graph=graph)
        m.upload(inputs.blast(m.leaves(), n, nrb))
        m.step(5)
        flags, _ = m.flag_pressure_jump(0.1, 0.02)
        m.regrid(flags)
        assert m.partition()["nparts"] == nparts
        m.step(5)
        outs.append((m.leaves(), m.download()))
        m.close()
    for lv_o, u in outs[1:]:
        assert np.array_equal(lv_o, outs[0][0])
        assert np.array_equal(u, outs[0][1])


def test_partition_bitwise_with_walls_and_midrun_switch():
    """Walls and a partition set between steps (the ghost layers of faces
    that become remote are filled at the switch)."""
    print_case("partition 4 set mid-run, walls, 64^3 as 8 blocks of 32^3, 6 cycles")
    n, nrb = (32, 32, 32), (2, 2, 2)
    bc = (REF, OUT, PER, PER, OUT, REF)
    lv = inputs.uniform_leaves(nrb)
    ref = _mesh(lv, nrb, n, bc=bc)
    U0 = inputs.smooth_flow(ref.leaves(), n, nrb)
    ref.upload(U0)
    ref.step(6)
    m = _mesh(lv, nrb, n, bc=bc)
    m.upload(U0)
    m.step(3)
    m.set_partition(4)
    m.step(3)
    assert np.array_equal(m.download(), ref.download())
    m.set_partition(1)
    assert m.partition()["remote_faces"] == 0


def test_partition_refusals():
    from paper_2202_12309_amd.binding import Batch, PkhError
    n, nrb = (16, 16, 16), (2, 2, 2)
    m = _mesh(inputs.uniform_leaves(nrb), nrb, n)
    with pytest.raises(PkhError):
        m.set_partition(0)
    with pytest.raises(PkhError):
        m.set_partition(9)
    m.set_partition(2)
    with pytest.raises(PkhError):
        m.tape(2)
    with pytest.raises(PkhError):
        Batch([m])
    m.close()


def test_layout_changes_refused_while_tape_or_batch_attached():
    """A tape or a batch keeps pointers into the mesh's leaf layout: regrid
    and repartition return PKH_ESTATE while one exists and work again once
    it is destroyed; the state is untouched by the refused calls."""
    print_case("regrid / partition refused while a tape or batch holds the mesh")
    from paper_2202_12309_amd.binding import Batch, PkhError
    n, nrb = (16, 16, 16), (2, 2, 2)
    m = _mesh(inputs.uniform_leaves(nrb), nrb, n, max_level=1)
    m.upload(inputs.turbulent_box(m.leaves(), n, nrb, seed=3))
    m.step(1)
    before = m.download()
    flags = np.ones(m.nleaves, dtype=np.int8)
    for make in (lambda: m.tape(2), lambda: Batch([m])):
        h = make()
        for call in (lambda: m.regrid(flags), lambda: m.set_partition(2)):
            with pytest.raises(PkhError) as e:
                call()
            assert e.value.name == "PKH_ESTATE", e.value
        assert np.array_equal(m.download(), before) and m.nleaves == 8
        h.close()
    m.set_partition(2)
    m.set_partition(1)
    m.regrid(flags)
    assert m.nleaves == 64
    m.close()
