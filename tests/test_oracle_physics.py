"""Pins of the oracle's whole update on uniform meshes: invariants, closed
forms, an exact Riemann solution, decomposition independence, symmetry and an
independent re-derivation. CPU only."""
import json
import math
import os

import numpy as np
import pytest
import torch

from oracle import exact_riemann, torch_ref
from oracle.oracle import OracleMesh, OracleError
from paper_2202_12309_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")
G53 = 5.0 / 3.0


def _mesh(n, nrb, **kw):
    return OracleMesh(n, nrb, inputs.uniform_leaves(nrb), **kw)


@pytest.mark.parametrize("recon1", [0, 1])
def test_uniform_state_preserved_bitwise(recon1):
    m = _mesh((8, 8, 8), (2, 2, 2), stage1_recon=recon1)
    U0 = inputs.uniform_state(m.leaves(), m.n, rho=1.37, v=(0.31, -0.52, 0.11), p=0.83)
    m.set_state(U0)
    m.step(4)
    assert np.array_equal(m.state(), U0)


def test_dt_closed_form():
    # rho = 1, P = 0.6, gamma = 5/3 -> c = 1; v = (0.5, 0, 0); dx = 1/16
    m = _mesh((8, 8, 8), (2, 2, 2))
    m.set_state(inputs.uniform_state(m.leaves(), m.n, rho=1.0, v=(0.5, 0.0, 0.0), p=0.6))
    assert m.dt() == pytest.approx(0.3 * (1.0 / 16.0) / 1.5, rel=1e-15)
    # anisotropic cells: the smallest dx_d / (|v_d| + c) wins
    m2 = _mesh((8, 8, 8), (2, 2, 2), xmax=(1.0, 0.5, 2.0))
    m2.set_state(inputs.uniform_state(m2.leaves(), m2.n, rho=1.0, v=(0.0, 0.0, 3.0), p=0.6))
    want = 0.3 * min((1 / 16) / 1.0, (0.5 / 16) / 1.0, (2 / 16) / 4.0)
    assert m2.dt() == pytest.approx(want, rel=1e-15)


def test_totals_uniform_exact():
    m = _mesh((8, 8, 8), (2, 2, 2))
    m.set_state(inputs.uniform_state(m.leaves(), m.n, rho=1.25, v=(0.5, 0.25, -0.75), p=0.75))
    T, _ = m.totals()
    assert T[0] == 1.25
    assert T[1] == 1.25 * 0.5 and T[2] == 1.25 * 0.25 and T[3] == -1.25 * 0.75


def test_periodic_conservation():
    n, nrb = (16, 16, 16), (2, 2, 2)
    m = _mesh(n, nrb)
    m.set_state(inputs.turbulent_box(m.leaves(), n, nrb, seed=7))
    T0, A0 = m.totals()
    m.step(30)
    T1, _ = m.totals()
    assert np.all(np.abs(T1 - T0) <= 1e-14 * A0 * 30)


def _wave_error(N, axis=0, t_end=1.0):
    """L1 density error of a sound wave along `axis` after one period on an
    N x 4 x 4 (permuted) grid of cubic cells."""
    nb = [4, 4, 4]
    nrb = [1, 1, 1]
    blk = 16 if N >= 16 else N
    nb[axis] = blk
    nrb[axis] = N // blk
    xmax = [4.0 / N] * 3
    xmax[axis] = 1.0
    kvec = [0, 0, 0]
    kvec[axis] = 1
    m = OracleMesh(tuple(nb), tuple(nrb), inputs.uniform_leaves(nrb), xmax=tuple(xmax))
    U0 = inputs.sound_wave(m.leaves(), nb, nrb, amp=1e-6, noise=0.0, kvec=kvec, xmax=xmax)
    m.set_state(U0)
    for _ in range(100000):
        t, _, _ = m.time()
        if t >= t_end:
            break
        m.step(1, t_end)
    U = m.state()
    return np.abs(U[:, 0] - U0[:, 0]).mean(), m


def test_linear_wave_second_order():
    # MC clipping at the wave's extrema costs accuracy on the coarsest grids;
    # from N = 32 on the observed L1 order is above 2.
    errs = [_wave_error(N)[0] for N in (32, 64, 128)]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) >= 1.9, (errs, orders)
    assert errs[-1] < 1e-9  # amplitude 1e-6: below 0.1 per cent at N = 128


@pytest.mark.parametrize("axis", [1, 2])
def test_linear_wave_other_axes_match_x(axis):
    ex, mx = _wave_error(32, 0)
    ea, ma = _wave_error(32, axis)
    assert abs(ea - ex) <= 1e-12 * ex + 1e-22
    assert mx.time()[0] == ma.time()[0]


def _sod(N):
    g = 1.4
    n = (16, 4, 4)
    nrb = (N // 16, 1, 1)
    xmax = (2.0, 8.0 / N, 8.0 / N)  # cubic cells of width 2/N
    m = OracleMesh(n, nrb, inputs.uniform_leaves(nrb), gamma=g, xmax=xmax)
    U = np.empty(m.shape())
    for b, lf in enumerate(m.leaves()):
        x, _, _ = inputs.cell_centers(lf, n, nrb, xmax=xmax)
        hi = (x >= 0.5) & (x < 1.5)
        rho = np.where(hi, 1.0, 0.125)
        p = np.where(hi, 1.0, 0.1)
        U[b] = 0.0
        U[b, 0] = rho
        U[b, 4] = p / (g - 1)
    m.set_state(U)
    while m.time()[0] < 0.2:
        m.step(1, 0.2)
    U = m.state()
    xs = np.concatenate([inputs.cell_centers(lf, n, nrb, xmax=xmax)[0][0, 0] for lf in m.leaves()])
    rho = np.concatenate([U[b, 0, 0, 0] for b in range(len(U))])
    mom = np.concatenate([U[b, 1, 0, 0] for b in range(len(U))])
    ene = np.concatenate([U[b, 4, 0, 0] for b in range(len(U))])
    # y, z extent stays uniform bitwise
    for b in range(len(U)):
        for v in range(5):
            assert np.all(U[b, v] == U[b, v, :1, :1, :])
    return xs, rho, mom / rho, (g - 1) * (ene - 0.5 * mom * mom / rho)


def _sod_exact(xs):
    ref = json.load(open(os.path.join(GOLD, "sod_star_state.json")))
    g = ref["gamma"]
    (rl, ul, pl), (rr, ur, pr) = ref["left"], ref["right"]
    t = 0.2
    right = xs >= 1.0
    r1, u1, p1 = exact_riemann.sample((xs - 1.5) / t, rl, ul, pl, rr, ur, pr, g)
    r2, u2, p2 = exact_riemann.sample((0.5 - xs) / t, rl, ul, pl, rr, ur, pr, g)
    return (np.where(right, r1, r2), np.where(right, u1, -u2), np.where(right, p1, p2), ref)


@pytest.mark.slow
def test_sod_against_exact_riemann():
    errs = []
    for N in (128, 256, 512):
        xs, rho, u, p = _sod(N)
        re, ue, pe, ref = _sod_exact(xs)
        errs.append(np.abs(rho - re).mean())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) >= 0.6, (errs, orders)
    # star-region plateau between contact and shock at N = 512
    xm = 1.5 + 0.2 * 0.5 * (ref["u_star"] + ref["shock_speed"])
    k = np.argmin(np.abs(xs - xm))
    assert abs(p[k] - ref["p_star"]) <= 0.01 * ref["p_star"]
    assert abs(u[k] - ref["u_star"]) <= 0.01 * ref["u_star"]
    assert abs(rho[k] - ref["rho_star_right"]) <= 0.01 * ref["rho_star_right"]
    # the mirrored problem on the left half is the mirror image
    km = np.argmin(np.abs(xs - (2.0 - xm)))
    assert abs(p[km] - p[k]) <= 1e-12 * p[k]


def test_one_block_vs_many_bitwise():
    N = 32
    res = []
    for blk in (32, 16, 8):
        n = (blk, blk, blk)
        nrb = (N // blk,) * 3
        m = _mesh(n, nrb)
        U0 = inputs.turbulent_box(m.leaves(), n, nrb, seed=11)
        m.set_state(U0)
        m.step(3)
        G = torch_ref.blocks_to_global(m.state(), m.leaves(), n, nrb)
        res.append((G, m.time()))
    for G, tm in res[1:]:
        assert np.array_equal(G, res[0][0])
        assert tm == res[0][1]


def test_axis_permutation():
    n, nrb = (8, 8, 8), (2, 2, 2)
    m = _mesh(n, nrb)
    U0 = inputs.turbulent_box(m.leaves(), n, nrb, seed=3)
    G0 = torch_ref.blocks_to_global(U0, m.leaves(), n, nrb)
    m.set_state(U0)
    m.step(3)
    G1 = torch_ref.blocks_to_global(m.state(), m.leaves(), n, nrb)
    # rotate x -> y -> z: new(z, y, x) fields; velocity components cycle too
    def rot(G):
        R = np.transpose(G, (0, 2, 3, 1)).copy()  # new axes: (z'=y, y'=x, x'=z)
        out = R.copy()
        out[1], out[2], out[3] = R[3], R[1], R[2]
        return out
    m2 = _mesh(n, nrb)
    m2.set_state(torch_ref.global_to_blocks(rot(G0), m2.leaves(), n))
    m2.step(3)
    G2 = torch_ref.blocks_to_global(m2.state(), m2.leaves(), n, nrb)
    np.testing.assert_allclose(G2, rot(G1), rtol=0, atol=1e-14 * np.abs(G1).max())


@pytest.mark.parametrize("recon1", [0, 1])
def test_cross_check_against_grid_formulation(recon1):
    """The C oracle (blocks + ghost exchange) against the independent
    global-array formulation in torch_ref (neighbours by roll)."""
    n, nrb = (8, 8, 8), (2, 2, 2)
    m = _mesh(n, nrb, stage1_recon=recon1)
    U0 = inputs.turbulent_box(m.leaves(), n, nrb, seed=5)
    U0 += inputs.sound_wave(m.leaves(), n, nrb, amp=1e-2, noise=1e-3) - inputs.sound_wave(
        m.leaves(), n, nrb, amp=0.0, noise=0.0)
    m.set_state(U0)
    m.step(3)
    G0 = torch.tensor(torch_ref.blocks_to_global(U0, m.leaves(), n, nrb))
    G, dts = torch_ref.run(G0, 3, stage1_recon=recon1)
    Gc = torch_ref.blocks_to_global(m.state(), m.leaves(), n, nrb)
    scale = np.abs(Gc).reshape(5, -1).max(1)
    err = np.abs(G.numpy() - Gc).reshape(5, -1).max(1) / scale
    assert np.all(err <= 1e-14), err
    assert abs(sum(dts) - m.time()[0]) <= 1e-15


def test_unphysical_state_is_reported():
    m = _mesh((8, 8, 8), (1, 1, 1))
    U = inputs.uniform_state(m.leaves(), m.n)
    U[0, 4, 3, 3, 3] = -1.0  # negative energy -> negative pressure
    m.set_state(U)
    with pytest.raises(OracleError):
        m.step(1)
