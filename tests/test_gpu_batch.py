"""Batched instances: every instance of the plain per-mesh path, the grouped
(fused) launches, the captured-graph replays and the persistent launch
against the oracle element by element, on single-level mixes and on a mix
with multilevel and walled members; the four modes bitwise identical; the
persistent launch's bounded waits report an error instead of hanging;
autotuning leaves states and clocks untouched. Runs on an MI355X."""
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


@pytest.mark.parametrize("mode", ["plain", "fused", "graph", "persistent"])
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


def test_fused_graph_persistent_equal_plain_bitwise():
    print_case("batch plain vs fused vs graph vs persistent")
    import torch
    from paper_2202_12309_amd.binding import Batch
    specs = inputs.batch_mix(n=6, seed=11, sizes=(32, 48, 64))
    specs[0]["blk"] = 16
    results = {}
    for mode in ("plain", "fused", "graph", "persistent"):
        stream = torch.cuda.Stream()
        meshes = _make(specs, stream)
        b = Batch(meshes)
        b.step(3, mode)
        b.step(4, mode)
        results[mode] = [(m.download(), m.time()) for m in meshes]
        b.close()
    for mode in ("fused", "graph", "persistent"):
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
    assert b.tuning()["waves_per_simd"] in (2, 3)
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


def _mixed_members(stream):
    """A two-level blast (64^3 root in 16^3 blocks), a uniform sound wave in
    one 32^3 block, and a smooth flow between outflow and reflecting walls
    (32^3 in 16^3 blocks) -- with their oracle twins."""
    from oracle.oracle import BC_OUTFLOW as OUT, BC_PERIODIC as PER, BC_REFLECT as REF
    from paper_2202_12309_amd.binding import Mesh
    out = []
    nrb, n = (4, 4, 4), (16, 16, 16)
    lv = inputs.sphere_refined_leaves(nrb, radius=0.3)
    gm = Mesh((64,) * 3, n, lv, max_level=1, stream=stream)
    om = OracleMesh(n, nrb, gm.leaves(), max_level=1)
    out.append((gm, om, inputs.blast(gm.leaves(), n, nrb)))
    nrb, n = (1, 1, 1), (32, 32, 32)
    gm = Mesh((32,) * 3, n, inputs.uniform_leaves(nrb), stream=stream)
    om = OracleMesh(n, nrb, gm.leaves())
    out.append((gm, om, inputs.sound_wave(gm.leaves(), n, nrb, amp=1e-3, noise=1e-5)))
    nrb, n = (2, 2, 2), (16, 16, 16)
    bc = (REF, OUT, PER, PER, OUT, REF)
    gm = Mesh((32,) * 3, n, inputs.uniform_leaves(nrb), stream=stream, bc=bc)
    om = OracleMesh(n, nrb, gm.leaves(), bc=bc)
    out.append((gm, om, inputs.smooth_flow(gm.leaves(), n, nrb)))
    for gm, om, U0 in out:
        gm.upload(U0)
        om.set_state(U0)
    return out


@pytest.mark.parametrize("mode", ["plain", "fused", "graph", "persistent"])
def test_multilevel_and_walled_members_match_oracle(mode):
    """A batch holding a two-level mesh (flux correction and level-jump
    fills between the stages), a one-block mesh and a walled mesh: every
    member within 1e-12 of the oracle after 1 cycle and 1e-11 after 6, and
    bitwise equal to the plain path."""
    print_case(f"batch with multilevel and walled members vs oracle, mode {mode}")
    import torch
    from paper_2202_12309_amd.binding import Batch
    stream = torch.cuda.Stream()
    mem = _mixed_members(stream)
    b = Batch([m for m, _, _ in mem])
    for cyc, tol in ((1, 1e-12), (5, 1e-11)):
        b.step(cyc, mode)
        for q, (gm, om, _) in enumerate(mem):
            om.step(cyc)
            err = rel_err(gm.download(), om.state(), G)
            print(f"member {q}: rel err {err}", flush=True)
            assert np.all(err <= tol), (q, err)
            To, Ao = om.totals()
            assert np.all(np.abs(gm.totals() - To) <= 1e-13 * np.maximum(Ao, 1.0))
    b.close()
    # bitwise equal to the members' own launches
    stream2 = torch.cuda.Stream()
    ref = _mixed_members(stream2)
    for gm, _, _ in ref:
        gm.step(6)
    for (gm, _, _), (rm, _, _) in zip(mem, ref):
        assert np.array_equal(gm.download(), rm.download())
        assert gm.time() == rm.time()


def test_persistent_wait_bound_reports_instead_of_hanging():
    """With the wait bound set to zero every wait not met at once gives up:
    the launch drains and ends, and the members' next synchronising call
    reports PKH_ESTATE; a fresh upload clears the latch and the default
    bound runs normally again (equal to the plain path)."""
    print_case("persistent batch: zero wait bound -> PKH_ESTATE, then recovery")
    import torch
    from paper_2202_12309_amd.binding import Batch, PkhError
    specs = inputs.batch_mix(n=4, seed=14, sizes=(64,))
    stream = torch.cuda.Stream()
    meshes = _make(specs, stream)
    b = Batch(meshes)
    b.set_tuning(2, 0.0)
    assert b.tuning() == {"waves_per_simd": 2, "wait_limit_s": 0.0}
    b.step(3, "persistent")
    with pytest.raises(PkhError) as e:
        meshes[0].sync()
    assert e.value.name == "PKH_ESTATE"
    b.set_tuning(3, 2.0)
    for sp, m in zip(specs, meshes):
        m.upload(inputs.batch_state(sp, m.leaves()))
    b.step(3, "persistent")
    ref = _make(specs, torch.cuda.Stream())
    for m, r in zip(meshes, ref):
        r.step(3)
        assert np.array_equal(m.download(), r.download())
    with pytest.raises(PkhError):
        b.set_tuning(4, 1.0)


def test_persistent_needs_16_or_32_cell_rows():
    print_case("persistent batch refuses blocks of 8 cells per row")
    from paper_2202_12309_amd.binding import Batch, Mesh, PkhError
    m = Mesh((16,) * 3, (8, 8, 8), inputs.uniform_leaves((2, 2, 2)))
    m.upload(inputs.sound_wave(m.leaves(), (8, 8, 8), (2, 2, 2), amp=1e-3, noise=0.0))
    b = Batch([m])
    b.step(1, "fused")
    with pytest.raises(PkhError) as e:
        b.step(1, "persistent")
    assert e.value.name == "PKH_EINVAL"


@pytest.mark.parametrize("mode", ["fused", "persistent"])
def test_bench_mix_full_size_matches_oracle(mode):
    """The bench's batch workload itself: the 64-instance mix (seed 4, edges
    32-128, 49.7 million cells) in the launch configuration the bench times,
    two cycles, every instance against the oracle run of the same instance
    (one instance at a time on the oracle side): within 1e-12, equal clocks,
    totals to 1e-13."""
    print_case(f"bench batch mix, 64 instances, mode {mode}, 2 cycles")
    import torch
    from paper_2202_12309_amd.binding import Batch
    specs = inputs.batch_mix(n=64, seed=4)
    stream = torch.cuda.Stream()
    meshes = _make(specs, stream)
    b = Batch(meshes)
    b.step(2, mode)
    worst = 0.0
    for q, (sp, m) in enumerate(zip(specs, meshes)):
        n = (sp["blk"],) * 3
        nrb = (sp["N"] // sp["blk"],) * 3
        om = OracleMesh(n, nrb, m.leaves())
        om.set_state(inputs.batch_state(sp, m.leaves()))
        om.step(2)
        err = rel_err(m.download(), om.state(), G)
        worst = max(worst, float(err.max()))
        assert np.all(err <= 1e-12), (q, sp, err)
        tg, to = m.time(), om.time()
        assert tg[2] == to[2] and abs(tg[0] - to[0]) <= 1e-14 * abs(to[0]), (q, tg, to)
        To, Ao = om.totals()
        assert np.all(np.abs(m.totals() - To) <= 1e-13 * np.maximum(Ao, 1.0)), q
        del om
    print(f"64 instances: worst rel err {worst:.3g}", flush=True)
    b.close()
