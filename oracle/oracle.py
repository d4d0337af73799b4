"""ctypes wrapper of the C oracle (TEST INFRASTRUCTURE).

State arrays use the layout ``[nleaves][5][n3][n2][n1]`` (conserved variables
rho, Mx, My, Mz, E; x fastest), leaves in the oracle's storage order (Morton
order of their deepest-level corner), as returned by :meth:`OracleMesh.leaves`.
"""
import ctypes as C
import math
import os

import numpy as np

from . import build as _build

_lib = None

_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        _lib = load(path)
    return _lib


def use(path):
    """Make the oracle build at `path` the one every OracleMesh of this
    process uses (the timing build; call before any other use)."""
    global _lib
    _lib = load(path)
    return _lib


def load(path):
    """Load a build of the oracle and declare its entry points."""
    L = C.CDLL(path)
    L.orc_create.argtypes = [_I32, _I32, C.c_int32, _D, _D, C.c_double, C.c_double,
                             C.c_int32, _I32, _I32, C.c_int64, C.POINTER(C.c_void_p)]
    L.orc_create.restype = C.c_int
    L.orc_destroy.argtypes = [C.c_void_p]
    L.orc_nleaves.argtypes = [C.c_void_p]
    L.orc_nleaves.restype = C.c_int64
    L.orc_leaves.argtypes = [C.c_void_p, _I32]
    L.orc_set_state.argtypes = [C.c_void_p, _D]
    L.orc_set_fp32.argtypes = [C.c_void_p, C.c_int32]
    L.orc_get_state.argtypes = [C.c_void_p, _D]
    L.orc_set_time.argtypes = [C.c_void_p, C.c_double, C.c_int64]
    L.orc_error.argtypes = [C.c_void_p]
    L.orc_padded.argtypes = [C.c_void_p, C.c_int64, _D]
    L.orc_dt.argtypes = [C.c_void_p]
    L.orc_dt.restype = C.c_double
    L.orc_stage_inplace.argtypes = [C.c_void_p, C.c_int32, C.c_double]
    L.orc_step.argtypes = [C.c_void_p, C.c_int32, C.c_double]
    L.orc_time.argtypes = [C.c_void_p, _D, _D, C.POINTER(C.c_int64)]
    L.orc_totals.argtypes = [C.c_void_p, _D, _D]
    L.orc_regrid.argtypes = [C.c_void_p, C.POINTER(C.c_int8), C.c_int64]
    L.orc_mc.argtypes = [C.c_double, C.c_double]
    L.orc_mc.restype = C.c_double
    L.orc_minmod.argtypes = [C.c_double, C.c_double]
    L.orc_minmod.restype = C.c_double
    L.orc_hlle.argtypes = [_D, _D, C.c_int, C.c_double, _D]
    L.orc_prim.argtypes = [_D, C.c_double, _D]
    L.orc_threads.restype = C.c_int
    L.orc_step_dts.argtypes = [C.c_void_p, C.c_int32, _D]
    L.orc_track_branches.argtypes = [C.c_void_p, C.c_int32]
    L.orc_branch_signature.argtypes = [C.c_void_p]
    L.orc_branch_signature.restype = C.c_uint64
    L.orc_mc_code.argtypes = [C.c_double, C.c_double]
    L.orc_minmod_code.argtypes = [C.c_double, C.c_double]
    L.orc_hlle_code.argtypes = [_D, _D, C.c_int, C.c_double]
    return L


def _dp(a):
    return a.ctypes.data_as(_D)


class OracleError(RuntimeError):
    pass


# Boundary kinds per face (x-, x+, y-, y+, z-, z+).
BC_PERIODIC, BC_OUTFLOW, BC_REFLECT = 0, 1, 2


def threads():
    """OpenMP threads the oracle uses."""
    return int(lib().orc_threads())


def mc(dl, dr):
    return lib().orc_mc(float(dl), float(dr))


def minmod(a, b):
    return lib().orc_minmod(float(a), float(b))


def hlle(wl, wr, d, gamma):
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    f = np.zeros(5)
    lib().orc_hlle(_dp(wl), _dp(wr), int(d), float(gamma), _dp(f))
    return f


def prim(u, gamma):
    u = np.ascontiguousarray(u, dtype=np.float64)
    w = np.zeros(5)
    lib().orc_prim(_dp(u), float(gamma), _dp(w))
    return w


class OracleMesh:
    """Block mesh held by the C oracle.

    nblock: cells per block (n1, n2, n3); nroot_blocks: level-0 blocks per
    dimension; leaves: iterable of (level, lx, ly, lz); bc: boundary kind
    per face (x-, x+, y-, y+, z-, z+), BC_* values.
    """

    def __init__(self, nblock, nroot_blocks, leaves, gamma=5.0 / 3.0, cfl=0.3,
                 xmin=(0.0, 0.0, 0.0), xmax=(1.0, 1.0, 1.0), max_level=0, stage1_recon=0,
                 bc=(BC_PERIODIC,) * 6, fp32_state=False):
        n = np.array(nblock, dtype=np.int32)
        nrb = np.array(nroot_blocks, dtype=np.int32)
        locs = np.ascontiguousarray(np.array(leaves, dtype=np.int32).reshape(-1, 4))
        xmn = np.array(xmin, dtype=np.float64)
        xmx = np.array(xmax, dtype=np.float64)
        bca = np.array(bc, dtype=np.int32)
        assert bca.shape == (6,)
        h = C.c_void_p()
        rc = lib().orc_create(n.ctypes.data_as(_I32), nrb.ctypes.data_as(_I32), int(max_level),
                              _dp(xmn), _dp(xmx), float(gamma), float(cfl), int(stage1_recon),
                              bca.ctypes.data_as(_I32), locs.ctypes.data_as(_I32), len(locs), C.byref(h))
        if rc != 0:
            raise OracleError(f"orc_create failed with {rc}")
        self._h = h
        self.n = tuple(int(x) for x in n)
        self.nrb = tuple(int(x) for x in nrb)
        self.gamma = gamma
        self.cfl = cfl
        self.xmin = tuple(xmn)
        self.xmax = tuple(xmx)
        self.max_level = max_level
        self.bc = tuple(int(x) for x in bca)
        if fp32_state:
            lib().orc_set_fp32(h, 1)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().orc_destroy(h)
            self._h = None

    @property
    def nleaves(self):
        return int(lib().orc_nleaves(self._h))

    def leaves(self):
        out = np.zeros((self.nleaves, 4), dtype=np.int32)
        lib().orc_leaves(self._h, out.ctypes.data_as(_I32))
        return out

    def shape(self):
        n1, n2, n3 = self.n
        return (self.nleaves, 5, n3, n2, n1)

    def set_state(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == self.shape(), (U.shape, self.shape())
        lib().orc_set_state(self._h, _dp(U))

    def state(self):
        U = np.zeros(self.shape())
        lib().orc_get_state(self._h, _dp(U))
        return U

    def set_time(self, t, cycle=0):
        lib().orc_set_time(self._h, float(t), int(cycle))

    def padded(self, b):
        n1, n2, n3 = self.n
        out = np.zeros((5, n3 + 4, n2 + 4, n1 + 4))
        rc = lib().orc_padded(self._h, int(b), _dp(out))
        if rc != 0:
            raise OracleError(f"orc_padded failed with {rc}")
        return out

    def dt(self):
        return float(lib().orc_dt(self._h))

    def stage_inplace(self, recon, coef):
        rc = lib().orc_stage_inplace(self._h, int(recon), float(coef))
        if rc != 0:
            raise OracleError(f"orc_stage_inplace failed with {rc}")

    def step(self, ncycles, t_end=math.inf):
        rc = lib().orc_step(self._h, int(ncycles), float(t_end))
        if rc != 0:
            raise OracleError(f"orc_step failed with {rc}")

    def step_dts(self, dts):
        """Cycles with the given timesteps (one per cycle) instead of the CFL
        timestep: the map a frozen-timestep reverse mode differentiates."""
        d = np.ascontiguousarray(np.asarray(dts, dtype=np.float64))
        rc = lib().orc_step_dts(self._h, len(d), _dp(d))
        if rc != 0:
            raise OracleError(f"orc_step_dts failed with {rc}")

    def track_branches(self, on=True):
        """Start (signature reset) or stop recording the branch signature."""
        lib().orc_track_branches(self._h, 1 if on else 0)

    def branch_signature(self):
        """Order-free hash of every limiter, wave-speed and prolongation-slope
        branch taken by the stages since track_branches(True)."""
        return int(lib().orc_branch_signature(self._h))

    def time(self):
        t = C.c_double()
        dt = C.c_double()
        cyc = C.c_int64()
        lib().orc_time(self._h, C.byref(t), C.byref(dt), C.byref(cyc))
        return t.value, dt.value, cyc.value

    def totals(self):
        out = np.zeros(5)
        ab = np.zeros(5)
        lib().orc_totals(self._h, _dp(out), _dp(ab))
        return out, ab

    def regrid(self, flags):
        f = np.ascontiguousarray(np.asarray(flags, dtype=np.int8))
        rc = lib().orc_regrid(self._h, f.ctypes.data_as(C.POINTER(C.c_int8)), len(f))
        if rc != 0:
            raise OracleError(f"orc_regrid failed with {rc}")

    def _jump(self, quantity):
        n1, n2, n3 = self.n
        g1 = self.gamma - 1.0
        eta = np.zeros(self.nleaves)
        for b in range(self.nleaves):
            u = self.padded(b)
            if quantity == "pressure":
                ke = 0.5 * ((u[1] * u[1] + u[2] * u[2]) + u[3] * u[3]) / u[0]
                q = g1 * (u[4] - ke)
            else:
                q = u[0]
            a = slice(2, -2)
            jumps = []
            for lo, hi in (((a, a, slice(1, n1 + 1)), (a, a, slice(3, n1 + 3))),
                           ((a, slice(1, n2 + 1), a), (a, slice(3, n2 + 3), a)),
                           ((slice(1, n3 + 1), a, a), (slice(3, n3 + 3), a, a))):
                qm, qp = q[lo], q[hi]
                jumps.append((np.abs(qp - qm) / (qp + qm)).max())
            eta[b] = max(jumps)
        return eta

    def pressure_jump(self):
        """Refinement indicator per leaf (the paper leaves the criterion to
        the application): the largest |P(i+e_d) - P(i-e_d)| / (P(i+e_d) +
        P(i-e_d)) over active cells i and directions d, on the ghost-filled
        block. Plain numpy, no FMA, IEEE division."""
        return self._jump("pressure")

    def density_jump(self):
        """The same indicator on the density (contact and shear layers)."""
        return self._jump("density")

    def cell_centers(self, b):
        """Cell-centre coordinates (x, y, z) of leaf b, each [n3][n2][n1]."""
        lev, lx, ly, lz = (int(v) for v in self.leaves()[b])
        out = []
        for d, l in enumerate((lx, ly, lz)):
            nd = self.n[d]
            N = self.nrb[d] * nd * (1 << lev)
            dx = (self.xmax[d] - self.xmin[d]) / N
            out.append(self.xmin[d] + (l * nd + np.arange(nd) + 0.5) * dx)
        z, y, x = np.meshgrid(out[2], out[1], out[0], indexing="ij")
        return x, y, z
