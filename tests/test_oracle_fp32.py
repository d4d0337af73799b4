"""Pins of the oracle's FP32-storage mode (every stage computes in FP64 from
the stored values and rounds its output once to binary32). CPU only."""
import numpy as np

from _helpers import rel_err
from oracle.oracle import OracleMesh
from paper_2202_12309_amd import inputs

G = 5.0 / 3.0
N8, NRB = (8, 8, 8), (2, 2, 2)


def _f32(U):
    return U.astype(np.float32).astype(np.float64)


def _box():
    lv = inputs.uniform_leaves(NRB)
    return lv, _f32(inputs.turbulent_box(lv, N8, NRB, seed=3))


def test_one_stage_is_the_fp64_stage_rounded_once():
    """From a float-representable state, one FP32-storage stage equals the
    FP64 stage rounded to binary32, value by value: the rounding sits at the
    output only (not on fluxes, primitives or the update terms)."""
    lv, U0 = _box()
    for recon in (0, 1):
        m64 = OracleMesh(N8, NRB, lv)
        m32 = OracleMesh(N8, NRB, lv, fp32_state=True)
        m64.set_state(U0)
        m32.set_state(U0)
        coef = 0.4 * m64.dt()
        m64.stage_inplace(recon, coef)
        m32.stage_inplace(recon, coef)
        assert np.array_equal(m32.state(), _f32(m64.state()))
        assert not np.array_equal(m64.state(), m32.state())


def test_states_stay_float_and_close_to_fp64():
    """Through 10 cycles every stored value is a binary32 number, and the
    FP32-storage solution stays within the accumulated rounding of the FP64
    one (a few float ulps per cycle) while differing from it."""
    lv, U0 = _box()
    m64 = OracleMesh(N8, NRB, lv)
    m32 = OracleMesh(N8, NRB, lv, fp32_state=True)
    m64.set_state(U0)
    m32.set_state(U0)
    m64.step(10)
    m32.step(10)
    U32 = m32.state()
    assert np.array_equal(U32, _f32(U32))
    err = rel_err(U32, m64.state(), G)
    assert np.all(err <= 10 * 4 * 2.0 ** -24), err
    assert err.max() > 0.0


def test_fp32_uniform_state_preserved_and_input_rounded():
    lv = inputs.uniform_leaves(NRB)
    U0 = inputs.uniform_state(lv, N8, rho=1.1, v=(0.3, -0.2, 0.1), p=0.7)
    m = OracleMesh(N8, NRB, lv, fp32_state=True)
    m.set_state(U0)
    S0 = m.state()
    assert np.array_equal(S0, _f32(U0))
    m.step(3)
    assert np.array_equal(m.state(), S0)
