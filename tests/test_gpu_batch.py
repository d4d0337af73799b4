"""Batched instances: every instance of the plain per-mesh path, the grouped
(fused) launches and the captured-graph replays against the oracle element
by element; the three modes bitwise identical; autotuning leaves states and
clocks untouched. Runs on an MI355X."""
import numpy as np
import pytest

from _helpers import print_case, rel_err
from oracle.oracle import OracleMesh
from paper_2202_12309_amd import inputs

pytestmark = pytest.mark.gpu
G = 5.0 / 3.0


def _make(specs, stream):
    from paper_2202_12309_amd.binding import Mesh
    meshes = []
    for sp in specs:
        n = (sp["blk"],) * 3
        nrb = (sp["N"] // sp["blk"],) * 3
        m = Mesh((sp["N"],) * 3, n, inputs.uniform_leaves(nrb), stream=stream)
        m.upload(inputs.batch_state(sp, m.leaves()))
        meshes.append(m)
    return meshes


@pytest.mark.parametrize("mode", ["plain", "fused", "graph"])
def test_batch_instances_match_oracle(mode):
    """Six instances of the seeded mix (edges 32-64, blocks of 16^3 and 32^3,
    sound waves and blasts, each with its own timestep): after 1 cycle each
    instance is within 1e-12 of the oracle run of the same instance, after 7
    (a 6-cycle graph segment in graph mode) within 1e-11, with equal clocks
    to 1e-14 and totals to 1e-13."""
    print_case(f"batch of 6 vs oracle, mode {mode}, 1 + 6 cycles")
    import torch
    from paper_2202_12309_amd.binding import Batch
    specs = inputs.batch_mix(n=6, seed=11, sizes=(32, 48, 64))
    specs[0]["blk"] = 16
    stream = torch.cuda.Stream()
    meshes = _make(specs, stream)
    oms = []
    for sp, m in zip(specs, meshes):
        n = (sp["blk"],) * 3
        nrb = (sp["N"] // sp["blk"],) * 3
        om = OracleMesh(n, nrb, m.leaves())
        om.set_state(inputs.batch_state(sp, m.leaves()))
        oms.append(om)
    b = Batch(meshes)
    for cyc, tol in ((1, 1e-12), (6, 1e-11)):
        b.step(cyc, mode)
        for q, (m, om) in enumerate(zip(meshes, oms)):
            om.step(cyc)
            err = rel_err(m.download(), om.state(), G)
            print(f"instance {q} {specs[q]}: rel err {err}", flush=True)
            assert np.all(err <= tol), (q, err)
            tg, to = m.time(), om.time()
            assert tg[2] == to[2] and abs(tg[0] - to[0]) <= 1e-14 * abs(to[0]), (tg, to)
            To, Ao = om.totals()
            assert np.all(np.abs(m.totals() - To) <= 1e-13 * np.maximum(Ao, 1.0))
    b.close()


def test_fused_and_graph_equal_plain_bitwise():
    print_case("batch plain vs fused vs graph")
    import torch
    from paper_2202_12309_amd.binding import Batch
    specs = inputs.batch_mix(n=6, seed=11, sizes=(32, 48, 64))
    specs[0]["blk"] = 16
    results = {}
    for mode in ("plain", "fused", "graph"):
        stream = torch.cuda.Stream()
        meshes = _make(specs, stream)
        b = Batch(meshes)
        b.step(3, mode)
        b.step(4, mode)
        results[mode] = [(m.download(), m.time()) for m in meshes]
        b.close()
    for mode in ("fused", "graph"):
        for (Ua, ta), (Ub, tb) in zip(results["plain"], results[mode]):
            assert np.array_equal(Ua, Ub), mode
            assert ta == tb, mode


def test_graph_segments_and_remainder():
    print_case("batch graph 50-cycle segment + remainder")
    import torch
    from paper_2202_12309_amd.binding import Batch
    specs = inputs.batch_mix(n=3, seed=12, sizes=(32,))
    out = []
    for mode in ("fused", "graph"):
        stream = torch.cuda.Stream()
        meshes = _make(specs, stream)
        b = Batch(meshes)
        b.step(53, mode)  # one 50-cycle replay and 3 eager cycles
        out.append([m.download() for m in meshes])
        b.close()
    for Ua, Ub in zip(*out):
        assert np.array_equal(Ua, Ub)


def test_autotune_keeps_state():
    print_case("batch autotune")
    import torch
    from paper_2202_12309_amd.binding import Batch
    specs = inputs.batch_mix(n=4, seed=13, sizes=(32, 64))
    stream = torch.cuda.Stream()
    meshes = _make(specs, stream)
    b = Batch(meshes)
    b.step(2)
    before = [(m.download(), m.time()) for m in meshes]
    tiles = b.autotune(2)
    assert all(t in (2, 4, 8, 16) for t in tiles)
    for m, (U, t) in zip(meshes, before):
        assert np.array_equal(m.download(), U)
        assert m.time() == t
    # the tuned batch still matches a plain run
    stream2 = torch.cuda.Stream()
    ref = _make(specs, stream2)
    rb = Batch(ref)
    rb.step(2, "plain")
    b.step(3)
    rb.step(3, "plain")
    for m, r in zip(meshes, ref):
        assert np.array_equal(m.download(), r.download())


def test_single_mesh_autotune():
    print_case("mesh autotune")
    from paper_2202_12309_amd.binding import Mesh
    n, nrb = (32, 32, 32), (2, 2, 2)
    m = Mesh((64,) * 3, n, inputs.uniform_leaves(nrb))
    U0 = inputs.turbulent_box(m.leaves(), n, nrb, seed=3)
    m.upload(U0)
    t = m.autotune(2)
    assert t["tile_rows"] in (4, 8, 16)
    assert np.array_equal(m.download(), U0)
