"""The hand-written reverse-mode derivatives of the pointwise physics (EOS,
HLLE with Einfeldt speeds, PLM-MC face states) against central finite
differences of the same functions, compiled for the host from the GPU
sources. CPU only."""
import ctypes as C

import numpy as np
import pytest

from _helpers import host_check_lib

D = C.POINTER(C.c_double)


@pytest.fixture(scope="module")
def L():
    lib = host_check_lib()
    lib.pkhc_hlle.argtypes = [D, D, C.c_int, C.c_double, D]
    lib.pkhc_hlle_rev.argtypes = [D, D, C.c_int, C.c_double, D, D, D]
    lib.pkhc_face_plm.argtypes = [D, C.c_int, C.c_double, D]
    lib.pkhc_face_plm_rev.argtypes = [D, C.c_int, C.c_double, D, D]
    lib.pkhc_prim.argtypes = [D, C.c_double, D]
    lib.pkhc_prim_rev.argtypes = [D, C.c_double, D, D]
    lib.pkhc_mc.argtypes = [C.c_double, C.c_double]
    lib.pkhc_mc.restype = C.c_double
    lib.pkhc_mc_half.argtypes = [C.c_double, C.c_double]
    lib.pkhc_mc_half.restype = C.c_double
    return lib


def p(a):
    return a.ctypes.data_as(D)


def _state(rng, mach=0.6):
    return np.array([rng.uniform(0.5, 2.0), *rng.normal(scale=mach, size=3), rng.uniform(0.5, 2.0)])


def _fd(fun, x, h):
    cols = []
    for k in range(len(x)):
        e = np.zeros_like(x)
        e[k] = h * max(1.0, abs(x[k]))
        cols.append((fun(x + e) - fun(x - e)) / (2 * e[k]))
    return np.array(cols).T  # J[out, in]


@pytest.mark.parametrize("d", [0, 1, 2])
def test_hlle_adjoint_matches_fd(L, d):
    g = 5.0 / 3.0
    rng = np.random.default_rng(100 + d)
    for trial in range(40):
        wl, wr = _state(rng, 0.8), _state(rng, 0.8)
        if trial % 4 == 0:  # supersonic cases exercise the zero wave-speed branches
            wl[1 + d] += 3.0
            wr[1 + d] += 3.0

        def f(x):
            out = np.zeros(5)
            L.pkhc_hlle(p(np.ascontiguousarray(x[:5])), p(np.ascontiguousarray(x[5:])), d, g, p(out))
            return out
        x = np.concatenate([wl, wr])
        J = _fd(f, x, 1e-6)
        mu = rng.normal(size=5)
        gl, gr = np.zeros(5), np.zeros(5)
        L.pkhc_hlle_rev(p(wl), p(wr), d, g, p(mu), p(gl), p(gr))
        want = J.T @ mu
        got = np.concatenate([gl, gr])
        assert np.allclose(got, want, rtol=1e-6, atol=1e-7 * np.abs(want).max()), (trial, got, want)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_plm_face_adjoint_matches_fd(L, d):
    g = 5.0 / 3.0
    rng = np.random.default_rng(200 + d)
    checked = 0
    for trial in range(60):
        q = np.array([_state(rng, 0.5) for _ in range(4)])
        if trial % 3 == 0:  # smooth data: MC takes the central / 2|d| branches
            base = _state(rng, 0.5)
            q = base[None] + np.outer(np.arange(4) + 0.1 * rng.normal(size=4), rng.normal(size=5) * 0.05)
            q[:, 0] = np.abs(q[:, 0]) + 0.5
            q[:, 4] = np.abs(q[:, 4]) + 0.5

        def f(x):
            out = np.zeros(5)
            L.pkhc_face_plm(p(np.ascontiguousarray(x)), d, g, p(out))
            return out
        x = q.reshape(-1).copy()
        h = 1e-7
        J = _fd(f, x, h)
        # skip points where a limiter branch flips inside the difference stencil
        J2 = _fd(f, x, h / 4)
        if not np.allclose(J, J2, rtol=1e-4, atol=1e-6):
            continue
        mu = rng.normal(size=5)
        gq = np.zeros(20)
        L.pkhc_face_plm_rev(p(x), d, g, p(mu), p(gq))
        want = J.T @ mu
        assert np.allclose(gq, want, rtol=1e-5, atol=1e-6 * np.abs(want).max()), (trial, gq, want)
        checked += 1
    assert checked >= 40


def test_prim_adjoint_matches_fd(L):
    g = 1.4
    rng = np.random.default_rng(7)
    for _ in range(20):
        w = _state(rng, 1.0)
        u = np.array([w[0], *(w[0] * w[1:4]), w[4] / (g - 1) + 0.5 * w[0] * (w[1:4] @ w[1:4])])

        def f(x):
            out = np.zeros(5)
            L.pkhc_prim(p(np.ascontiguousarray(x)), g, p(out))
            return out
        J = _fd(f, u, 1e-7)
        gw = rng.normal(size=5)
        gu = np.zeros(5)
        L.pkhc_prim_rev(p(u), g, p(gw), p(gu))
        assert np.allclose(gu, J.T @ gw, rtol=1e-6, atol=1e-8)


def test_half_mc_slope_is_half_the_mc_slope(L):
    """The stage kernels offset face values by the half slope mc_half; it
    must equal 0.5 * MC bit for bit (scaling by powers of two is exact) on
    the limiter's hand cases, both signs, extrema, ties between the three
    candidates and random pairs over many magnitudes."""
    hand = [((1.0, 1.0), 0.5), ((1.0, 3.0), 1.0), ((1.0, 0.2), 0.2), ((1.0, -1.0), 0.0),
            ((0.0, 2.0), 0.0), ((-1.0, -3.0), -1.0), ((2.0, 0.0), 0.0)]
    for (dl, dr), want in hand:
        assert L.pkhc_mc_half(dl, dr) == want, (dl, dr)
    rng = np.random.default_rng(7)
    dl = rng.standard_normal(20000) * 10.0 ** rng.integers(-12, 6, 20000)
    dr = rng.standard_normal(20000) * 10.0 ** rng.integers(-12, 6, 20000)
    ties = [(1.0, 1.0 / 3.0), (3.0, 1.0), (1.0, 7.0 / 3.0), (-2.0, -2.0 / 3.0)]
    for a, b in list(zip(dl, dr)) + ties:
        h, f = L.pkhc_mc_half(a, b), L.pkhc_mc(a, b)
        assert np.float64(h).tobytes() == np.float64(0.5 * f).tobytes() or (h == 0.0 and f == 0.0), (a, b)
