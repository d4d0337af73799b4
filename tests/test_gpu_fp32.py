"""FP32 storage of the state on the HIP path (FP64 arithmetic, output
rounded once per stage) against the oracle's FP32-storage mode, its distance
from the FP64 path, and the meshes it refuses. Runs on an MI355X."""
import numpy as np
import pytest

from _helpers import print_case, rel_err
from oracle.oracle import OracleMesh
from paper_2202_12309_amd import inputs

pytestmark = pytest.mark.gpu
G = 5.0 / 3.0
ULP = 2.0 ** -24  # half the spacing of binary32 numbers, relative


def test_fp32_storage_parity_with_oracle():
    """Both sides compute each stage in FP64 and round once; their FP64
    values differ by rounding order only (~1e-16), so the stored floats are
    equal except where a value sits within that of a rounding boundary,
    one float ulp apart: at most a few ulps per cycle."""
    print_case("FP32 storage, 64^3 as 8 blocks of 32^3, turbulent box, 1 and 10 cycles")
    from paper_2202_12309_amd.binding import Mesh
    n, nrb = (32, 32, 32), (2, 2, 2)
    lv = inputs.uniform_leaves(nrb)
    gm = Mesh((64, 64, 64), n, lv, fp32_state=True)
    om = OracleMesh(n, nrb, lv, fp32_state=True)
    U0 = inputs.turbulent_box(gm.leaves(), n, nrb, seed=2)
    gm.upload(U0)
    om.set_state(U0)
    assert np.array_equal(gm.download(), om.state())  # upload rounds to nearest
    for c in range(1, 11):
        gm.step(1)
        om.step(1)
        if c in (1, 10):
            Ug, Uo = gm.download(), om.state()
            assert np.array_equal(Ug, Ug.astype(np.float32).astype(np.float64))
            err = rel_err(Ug, Uo, G)
            neq = int((Ug != Uo).sum())
            print(f"cycle {c}: rel err {err}, values differing {neq} of {Ug.size}", flush=True)
            assert np.all(err <= 8 * ULP * c), (c, err)
    To, Ao = om.totals()
    assert np.all(np.abs(gm.totals() - To) <= 1e-13 * np.maximum(Ao, 1.0))


def test_fp32_storage_against_fp64_path_at_full_size():
    """256^3 in 512 blocks of 32^3, 100 cycles (the bench configuration):
    the FP32-stored run stays within the accumulated float rounding of the
    FP64 run (measured here, bounded by 1e-5 relative)."""
    print_case("FP32 vs FP64 storage, 256^3 turbulent box, 100 cycles")
    from paper_2202_12309_amd.binding import Mesh
    n, nrb = (32, 32, 32), (8, 8, 8)
    lv = inputs.uniform_leaves(nrb)
    U0 = inputs.turbulent_box(lv, n, nrb, seed=2)
    out = []
    for fp32 in (False, True):
        gm = Mesh((256,) * 3, n, lv, fp32_state=fp32)
        gm.upload(U0 if fp32 else U0.astype(np.float32).astype(np.float64))
        gm.step(100)
        out.append(gm.download())
        gm.close()
    err = rel_err(out[1], out[0], G)
    print(f"FP32 vs FP64 storage after 100 cycles: rel err {err}", flush=True)
    assert np.all(err <= 1e-5), err
    assert err.max() > 0.0


def test_fp32_storage_refusals():
    from paper_2202_12309_amd.binding import Batch, Mesh, PkhError
    n = (16, 16, 16)
    with pytest.raises(PkhError):  # multilevel
        Mesh((32, 32, 32), n, inputs.uniform_leaves((2, 2, 2)), max_level=1, fp32_state=True)
    with pytest.raises(PkhError):  # walls
        Mesh((32, 32, 32), n, inputs.uniform_leaves((2, 2, 2)), bc=(1,) * 6, fp32_state=True)
    with pytest.raises(PkhError):  # rows of 8
        Mesh((16, 16, 16), (8, 8, 8), inputs.uniform_leaves((2, 2, 2)), fp32_state=True)
    m = Mesh((32, 32, 32), n, inputs.uniform_leaves((2, 2, 2)), fp32_state=True)
    with pytest.raises(PkhError):
        m.tape(2)
    with pytest.raises(PkhError):
        Batch([m])
    with pytest.raises(PkhError):
        m.set_partition(2)
    with pytest.raises(PkhError):
        m.flag_pressure_jump(0.1, 0.02)
    with pytest.raises(PkhError):
        m.set_tuning(4)
    m.close()
