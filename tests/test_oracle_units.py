"""Pins of the oracle's pointwise pieces: equation of state, MC limiter,
HLLE flux, exact Riemann solver. CPU only."""
import json
import math
import os

import numpy as np
import pytest

from oracle import exact_riemann
from oracle import oracle as orc

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# --- equation of state --------------------------------------------------

def test_prim_round_trip():
    g = 5.0 / 3.0
    rng = np.random.default_rng(0)
    for _ in range(50):
        rho, p = rng.uniform(0.1, 3.0), rng.uniform(0.1, 3.0)
        v = rng.normal(size=3)
        u = np.array([rho, rho * v[0], rho * v[1], rho * v[2], p / (g - 1) + 0.5 * rho * v @ v])
        w = orc.prim(u, g)
        np.testing.assert_allclose(w, [rho, *v, p], rtol=1e-13, atol=1e-14)


# --- MC limiter (van Leer 1977), hand cases -----------------------------

@pytest.mark.parametrize("dl,dr,want", [
    (1.0, 1.0, 1.0),      # smooth: central difference
    (1.0, 3.0, 2.0),      # 2|dl| binds
    (1.0, 0.2, 0.4),      # 2|dr| binds
    (1.0, -1.0, 0.0),     # extremum
    (0.0, 5.0, 0.0),      # flat side
    (-1.0, -3.0, -2.0),   # sign carried
    (-3.0, -1.0, -2.0),
])
def test_mc_cases(dl, dr, want):
    assert orc.mc(dl, dr) == want


def test_minmod_cases():
    assert orc.minmod(1.0, 3.0) == 1.0
    assert orc.minmod(-2.0, -0.5) == -0.5
    assert orc.minmod(1.0, -1.0) == 0.0
    assert orc.minmod(0.0, 1.0) == 0.0


# --- HLLE ---------------------------------------------------------------

def _phys_flux(w, d, g):
    rho, p = w[0], w[4]
    v = np.array(w[1:4])
    e = p / (g - 1) + 0.5 * rho * v @ v
    f = np.zeros(5)
    f[0] = rho * v[d]
    f[1:4] = rho * v[d] * v
    f[1 + d] += p
    f[4] = (e + p) * v[d]
    return f


def _cons(w, g):
    rho, p = w[0], w[4]
    v = np.array(w[1:4])
    return np.array([rho, *(rho * v), p / (g - 1) + 0.5 * rho * v @ v])


@pytest.mark.parametrize("d", [0, 1, 2])
def test_hlle_consistency(d):
    """F(U, U) equals the physical flux."""
    g = 5.0 / 3.0
    rng = np.random.default_rng(d)
    for _ in range(20):
        w = [rng.uniform(0.2, 2), *rng.normal(size=3), rng.uniform(0.2, 2)]
        np.testing.assert_allclose(orc.hlle(w, w, d, g), _phys_flux(w, d, g), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_hlle_supersonic_upwind(d):
    """All waves moving right: the flux is the left physical flux."""
    g = 1.4
    wl = [1.0, 0.0, 0.0, 0.0, 1.0]
    wr = [0.8, 0.0, 0.0, 0.0, 0.7]
    wl[1 + d] = 4.0
    wr[1 + d] = 3.9
    np.testing.assert_allclose(orc.hlle(wl, wr, d, g), _phys_flux(wl, d, g), rtol=1e-14)
    # mirrored: all waves moving left gives the right flux
    wl[1 + d], wr[1 + d] = -3.9, -4.0
    np.testing.assert_allclose(orc.hlle(wl, wr, d, g), _phys_flux(wr, d, g), rtol=1e-14)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_hlle_mirror_symmetry(d):
    """Reflecting the problem (swap sides, negate the normal velocity) negates
    the mass, transverse-momentum and energy fluxes and keeps the normal
    momentum flux."""
    g = 5.0 / 3.0
    rng = np.random.default_rng(10 + d)
    for _ in range(20):
        wl = np.array([rng.uniform(0.2, 2), *rng.normal(size=3), rng.uniform(0.2, 2)])
        wr = np.array([rng.uniform(0.2, 2), *rng.normal(size=3), rng.uniform(0.2, 2)])
        M = np.ones(5)
        M[1 + d] = -1.0
        f = orc.hlle(wl, wr, d, g)
        fm = orc.hlle(M * wr, M * wl, d, g)
        np.testing.assert_allclose(fm, -M * f, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("mach,u0", [(1.5, 0.0), (3.0, 0.2), (10.0, -0.3), (1.2, 2.0)])
def test_hlle_resolves_isolated_shock(d, mach, u0):
    """For a single Rankine-Hugoniot shock, the Roe-averaged speed u+a equals
    the shock speed S (Roe's property), so with Einfeldt's wave speeds the
    HLLE flux is exactly F_L = F_R - S (U_R - U_L). This fixes the Roe
    averages, the choice of the wave-speed bounds and the sign of the
    dissipation term together."""
    g = 5.0 / 3.0
    rr, pr = 1.3, 0.8
    cr = math.sqrt(g * pr / rr)
    S = u0 + mach * cr
    rl = rr * (g + 1) * mach ** 2 / ((g - 1) * mach ** 2 + 2)
    pl = pr * (2 * g * mach ** 2 - (g - 1)) / (g + 1)
    ul = S + (u0 - S) * rr / rl
    vt = (0.37, -0.21)
    wl = np.zeros(5)
    wr = np.zeros(5)
    wl[0], wl[4], wr[0], wr[4] = rl, pl, rr, pr
    wl[1 + d], wr[1 + d] = ul, u0
    t = [c for c in range(3) if c != d]
    wl[1 + t[0]] = wr[1 + t[0]] = vt[0]
    wl[1 + t[1]] = wr[1 + t[1]] = vt[1]
    # the pair really is a shock of speed S
    fl, fr = _phys_flux(wl, d, g), _phys_flux(wr, d, g)
    np.testing.assert_allclose(fr - fl, S * (_cons(wr, g) - _cons(wl, g)), rtol=1e-12, atol=1e-12)
    f = orc.hlle(wl, wr, d, g)
    scale = np.abs(fl).max()
    assert np.abs(f - fl).max() <= 1e-13 * scale


# --- exact Riemann solver against the published Sod star state ----------

def test_exact_riemann_sod_star():
    ref = json.load(open(os.path.join(GOLD, "sod_star_state.json")))
    g = ref["gamma"]
    (rl, ul, pl), (rr, ur, pr) = ref["left"], ref["right"]
    ps, us = exact_riemann.star_state(rl, ul, pl, rr, ur, pr, g)
    tol = ref["rel_tol"]
    assert abs(ps - ref["p_star"]) <= tol * ref["p_star"] + 5e-6
    assert abs(us - ref["u_star"]) <= tol * ref["u_star"] + 5e-6
    rho, u, p = exact_riemann.sample(np.array([us - 1e-9, us + 1e-9]), rl, ul, pl, rr, ur, pr, g)
    assert abs(rho[0] - ref["rho_star_left"]) <= 5e-6 + tol * ref["rho_star_left"]
    assert abs(rho[1] - ref["rho_star_right"]) <= 5e-6 + tol * ref["rho_star_right"]
    # wave positions: shock and rarefaction head
    s = ref["shock_speed"]
    rho, _, _ = exact_riemann.sample(np.array([s - 1e-4, s + 1e-4]), rl, ul, pl, rr, ur, pr, g)
    assert abs(rho[0] - ref["rho_star_right"]) < 1e-4 and rho[1] == rr
    h = ref["rarefaction_head"]
    rho, _, _ = exact_riemann.sample(np.array([h - 1e-4, h + 1e-3]), rl, ul, pl, rr, ur, pr, g)
    assert rho[0] == rl and rho[1] < rl
