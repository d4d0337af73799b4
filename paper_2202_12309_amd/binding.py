"""Thin ctypes binding of ``libpkhydro.so`` (the C-ABI of include/pkhydro.h).

Argument marshalling only: every step of the cycle runs in the HIP library.
PyTorch provides device memory (its caching allocator, through the
library's allocation callbacks) and the HIP stream. If the library is not
built the first call raises; there is no fallback path.
"""
import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpkhydro.so")

PKH_OK = 0
_CODES = {-1: "PKH_EINVAL", -2: "PKH_ETILING", -3: "PKH_EBALANCE", -4: "PKH_ENOMEM",
          -5: "PKH_EHIP", -6: "PKH_EPHYS", -7: "PKH_ESTATE"}
PKH_FLAG_GRAPH = 1
PKH_FLAG_FP32_STATE = 2


class PkhError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code
        self.name = _CODES.get(code, str(code))


class Config(C.Structure):
    _fields_ = [("nroot", C.c_int32 * 3), ("nblock", C.c_int32 * 3), ("nghost", C.c_int32),
                ("max_level", C.c_int32), ("xmin", C.c_double * 3), ("xmax", C.c_double * 3),
                ("gamma", C.c_double), ("cfl", C.c_double), ("bc", C.c_int32 * 6),
                ("stage1_recon", C.c_int32), ("limiter", C.c_int32), ("regrid_every", C.c_int32),
                ("flags", C.c_uint32)]


class Tuning(C.Structure):
    _fields_ = [("tile_rows", C.c_int32), ("packs", C.c_int32), ("reserved", C.c_int32 * 2)]


class BatchTuning(C.Structure):
    _fields_ = [("waves_per_simd", C.c_int32), ("reserved", C.c_int32), ("wait_limit_s", C.c_double)]


class Loc(C.Structure):
    _fields_ = [("level", C.c_int32), ("lx1", C.c_int32), ("lx2", C.c_int32), ("lx3", C.c_int32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)

_lib = None

# symbol -> (restype, argtypes)
_SIGS = {
    "pkh_mesh_create": (C.c_int, [C.POINTER(Config), C.POINTER(Loc), C.c_int64, C.c_void_p, ALLOC_FN,
                                  FREE_FN, C.c_void_p, C.POINTER(C.c_void_p)]),
    "pkh_mesh_destroy": (C.c_int, [C.c_void_p]),
    "pkh_mesh_blocks": (C.c_int, [C.c_void_p, C.POINTER(Loc), C.c_int64, C.POINTER(C.c_int64)]),
    "pkh_state_upload": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32]),
    "pkh_state_download": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32]),
    "pkh_exchange_boundaries": (C.c_int, [C.c_void_p]),
    "pkh_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_double]),
    "pkh_get_time": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                               C.POINTER(C.c_int64)]),
    "pkh_set_time": (C.c_int, [C.c_void_p, C.c_double, C.c_int64]),
    "pkh_set_refinement_flags": (C.c_int, [C.c_void_p, C.POINTER(C.c_int8), C.c_int64]),
    "pkh_regrid": (C.c_int, [C.c_void_p]),
    "pkh_flag_pressure_jump": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.POINTER(C.c_int8),
                                         C.POINTER(C.c_double)]),
    "pkh_flag_jump": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.POINTER(C.c_int8),
                                C.POINTER(C.c_double)]),
    "pkh_conserved_totals": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "pkh_conserved_totals_noalloc": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "pkh_sync": (C.c_int, [C.c_void_p]),
    "pkh_kernel_timing": (C.c_int, [C.c_void_p, C.c_uint32]),
    "pkh_set_tuning": (C.c_int, [C.c_void_p, C.POINTER(Tuning)]),
    "pkh_get_tuning": (C.c_int, [C.c_void_p, C.POINTER(Tuning)]),
    "pkh_kernel_times": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "pkh_set_partition": (C.c_int, [C.c_void_p, C.c_int32]),
    "pkh_get_partition": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32)]),
    "pkh_last_error": (C.c_char_p, []),
    "pkh_tape_create": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)]),
    "pkh_tape_destroy": (C.c_int, [C.c_void_p]),
    "pkh_tape_set_facewise": (C.c_int, [C.c_void_p, C.c_int32]),
    "pkh_forward_taped": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32]),
    "pkh_adjoint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pkh_tape_replay": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pkh_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]),
    "pkh_batch_set_tuning": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pkh_batch_get_tuning": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pkh_batch_destroy": (C.c_int, [C.c_void_p]),
    "pkh_batch_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_uint32]),
    "pkh_batch_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]),
    "pkh_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
}


def lib():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(the hydro path has no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != PKH_OK:
        raise PkhError(rc, lib().pkh_last_error().decode())


class _TorchAllocator:
    """Device memory from torch's caching allocator, handed to the library
    through its allocation callbacks."""

    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = device
        self.alloc_cb = ALLOC_FN(self._alloc)
        self.free_cb = FREE_FN(self._free)

    def _alloc(self, nbytes, stream, ctx):
        try:
            return self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device, stream or 0)
        except Exception:  # allocation failure is reported by the library
            return None

    def _free(self, ptr, stream, ctx):
        torch = self.torch
        if torch is None or getattr(torch, "cuda", None) is None:
            return  # interpreter shutdown: the process frees everything
        try:
            torch.cuda.caching_allocator_delete(ptr)
        except Exception:
            pass


def _as_locs(leaves):
    arr = np.ascontiguousarray(np.asarray(leaves, dtype=np.int32).reshape(-1, 4))
    locs = (Loc * len(arr))()
    C.memmove(locs, arr.ctypes.data, arr.nbytes)
    return locs, len(arr)


# Boundary kinds per face (pkh_config.bc: x-, x+, y-, y+, z-, z+).
BC_PERIODIC, BC_OUTFLOW, BC_REFLECT = 0, 1, 2
# Quantities of the jump refinement indicator.
JUMP_PRESSURE, JUMP_DENSITY = 0, 1


class Mesh:
    """A block mesh resident on the GPU.

    nroot: level-0 cells per dimension; nblock: cells per block; leaves:
    (level, lx, ly, lz) rows; bc: boundary kind per face (BC_*). The
    library stores leaves in Morton order: :meth:`leaves` returns that
    storage order, which every state array uses (``[nleaves][5][n3][n2][n1]``).
    """

    def __init__(self, nroot, nblock, leaves, gamma=5.0 / 3.0, cfl=0.3, xmin=(0.0, 0.0, 0.0),
                 xmax=(1.0, 1.0, 1.0), max_level=0, stage1_recon=0, graph=False, device=0,
                 stream=None, torch_alloc=True, bc=(0,) * 6, fp32_state=False):
        import torch
        self.torch = torch
        self.device = device
        if stream is None:
            # a dedicated stream at default priority (graph capture needs a
            # non-null stream)
            stream = torch.cuda.Stream(device=device)
        self.stream = stream
        cfg = Config()
        for d in range(3):
            cfg.nroot[d] = int(nroot[d])
            cfg.nblock[d] = int(nblock[d])
            cfg.xmin[d] = float(xmin[d])
            cfg.xmax[d] = float(xmax[d])
        cfg.nghost = 2
        cfg.max_level = int(max_level)
        cfg.gamma = float(gamma)
        cfg.cfl = float(cfl)
        for f in range(6):
            cfg.bc[f] = int(bc[f])
        cfg.stage1_recon = int(stage1_recon)
        cfg.limiter = 0
        cfg.regrid_every = 0
        cfg.flags = (PKH_FLAG_GRAPH if graph else 0) | (PKH_FLAG_FP32_STATE if fp32_state else 0)
        self.cfg = cfg
        self.n = tuple(int(x) for x in nblock)
        self._alloc = _TorchAllocator(device) if torch_alloc else None
        locs, nl = _as_locs(leaves)
        h = C.c_void_p()
        with torch.cuda.device(device):
            _check(lib().pkh_mesh_create(
                C.byref(cfg), locs, nl, C.c_void_p(stream.cuda_stream),
                self._alloc.alloc_cb if self._alloc else ALLOC_FN(),
                self._alloc.free_cb if self._alloc else FREE_FN(), None, C.byref(h)))
        self._h = h

    # -- bookkeeping ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pkh_mesh_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def nleaves(self):
        n = C.c_int64()
        _check(lib().pkh_mesh_blocks(self._h, None, 0, C.byref(n)))
        return n.value

    def leaves(self):
        n = self.nleaves
        locs = (Loc * n)()
        cnt = C.c_int64()
        _check(lib().pkh_mesh_blocks(self._h, locs, n, C.byref(cnt)))
        return np.frombuffer(bytes(locs), dtype=np.int32).reshape(n, 4).copy()

    def shape(self):
        n1, n2, n3 = self.n
        return (self.nleaves, 5, n3, n2, n1)

    # -- state -----------------------------------------------------------------
    def upload(self, U):
        """U: numpy array (host) or torch tensor on the mesh's device,
        float64, shape [nleaves][5][n3][n2][n1]."""
        torch = self.torch
        if isinstance(U, torch.Tensor) and U.is_cuda:
            assert U.dtype == torch.float64 and tuple(U.shape) == self.shape()
            U = U.contiguous()
            # order the caller's producer stream before the mesh stream
            self.stream.wait_stream(torch.cuda.current_stream(U.device))
            _check(lib().pkh_state_upload(self._h, C.c_void_p(U.data_ptr()), 1))
            U.record_stream(self.stream)
        else:
            a = np.ascontiguousarray(U, dtype=np.float64)
            assert a.shape == self.shape(), (a.shape, self.shape())
            _check(lib().pkh_state_upload(self._h, C.c_void_p(a.ctypes.data), 0))

    def download(self, device=False):
        torch = self.torch
        if device:
            out = torch.empty(self.shape(), dtype=torch.float64, device=f"cuda:{self.device}")
            _check(lib().pkh_state_download(self._h, C.c_void_p(out.data_ptr()), 1))
            return out
        out = np.empty(self.shape())
        _check(lib().pkh_state_download(self._h, C.c_void_p(out.ctypes.data), 0))
        return out

    # -- evolution -------------------------------------------------------------
    def exchange(self):
        _check(lib().pkh_exchange_boundaries(self._h))

    def step(self, n_cycles, t_end=math.inf):
        _check(lib().pkh_step(self._h, int(n_cycles), float(t_end)))

    def sync(self):
        _check(lib().pkh_sync(self._h))

    def time(self):
        t, dt, cyc = C.c_double(), C.c_double(), C.c_int64()
        _check(lib().pkh_get_time(self._h, C.byref(t), C.byref(dt), C.byref(cyc)))
        return t.value, dt.value, cyc.value

    def set_time(self, t, cycle=0):
        _check(lib().pkh_set_time(self._h, float(t), int(cycle)))

    def totals(self):
        out = (C.c_double * 5)()
        _check(lib().pkh_conserved_totals(self._h, out))
        return np.array(out[:])

    def totals_noalloc(self):
        """totals() through the entry point that allocates nothing (static
        device scratch shared by every call on the GPU)."""
        out = (C.c_double * 5)()
        _check(lib().pkh_conserved_totals_noalloc(self._h, out))
        return np.array(out[:])

    def set_tuning(self, tile_rows=0, packs=1):
        t = Tuning()
        t.tile_rows = int(tile_rows)
        t.packs = int(packs)
        _check(lib().pkh_set_tuning(self._h, C.byref(t)))

    def autotune(self, trial_cycles=3):
        """Time every compiled tile-rows choice and keep the fastest (state
        and clock restored afterwards)."""
        t = Tuning()
        _check(lib().pkh_autotune(self._h, int(trial_cycles), C.byref(t)))
        return {"tile_rows": t.tile_rows}

    def tuning(self):
        t = Tuning()
        _check(lib().pkh_get_tuning(self._h, C.byref(t)))
        return {"tile_rows": t.tile_rows, "packs": t.packs}

    KT_PREDICTOR, KT_CORRECTOR, KT_FILL, KT_FLUXCORR, KT_ADJOINT, KT_REMOTE = 1, 2, 4, 8, 16, 32

    def kernel_timing(self, kinds):
        _check(lib().pkh_kernel_timing(self._h, int(kinds)))

    def kernel_times(self):
        """{kind: (total ms, launches)} for predictor, corrector, fill,
        fluxcorr and adjoint (one reverse stage)."""
        ms = (C.c_double * 6)()
        cnt = (C.c_int64 * 6)()
        _check(lib().pkh_kernel_times(self._h, ms, cnt))
        names = ("predictor", "corrector", "fill", "fluxcorr", "adjoint", "remote")
        return {names[k]: (ms[k], cnt[k]) for k in range(6)}

    def set_partition(self, nparts):
        """Cut the leaves into nparts contiguous ranges whose shared
        same-level faces go through pack / transfer / unpack."""
        _check(lib().pkh_set_partition(self._h, int(nparts)))

    def partition(self):
        p, r, g = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().pkh_get_partition(self._h, C.byref(p), C.byref(r), C.byref(g)))
        return {"nparts": p.value, "remote_faces": r.value, "messages": g.value}

    # -- reverse mode ------------------------------------------------------------
    def tape(self, ckpt_every):
        return Tape(self, ckpt_every)

    def set_flags(self, flags):
        f = np.ascontiguousarray(np.asarray(flags, dtype=np.int8))
        _check(lib().pkh_set_refinement_flags(self._h, f.ctypes.data_as(C.POINTER(C.c_int8)), len(f)))

    def flag_jump(self, quantity, refine_above, derefine_below):
        """Set the flags from the device jump indicator of quantity
        (JUMP_PRESSURE or JUMP_DENSITY); returns (flags int8[nleaves], eta
        float64[nleaves]) in storage order."""
        n = self.nleaves
        f = np.zeros(n, dtype=np.int8)
        eta = np.zeros(n, dtype=np.float64)
        _check(lib().pkh_flag_jump(self._h, int(quantity), float(refine_above), float(derefine_below),
                                   f.ctypes.data_as(C.POINTER(C.c_int8)),
                                   eta.ctypes.data_as(C.POINTER(C.c_double))))
        return f, eta

    def flag_pressure_jump(self, refine_above, derefine_below):
        return self.flag_jump(JUMP_PRESSURE, refine_above, derefine_below)

    def flag_density_jump(self, refine_above, derefine_below):
        return self.flag_jump(JUMP_DENSITY, refine_above, derefine_below)

    def regrid(self, flags=None):
        if flags is not None:
            self.set_flags(flags)
        _check(lib().pkh_regrid(self._h))


class Tape:
    """Recording of taped cycles for the reverse mode."""

    def __init__(self, mesh, ckpt_every):
        self.mesh = mesh
        h = C.c_void_p()
        _check(lib().pkh_tape_create(mesh._h, int(ckpt_every), C.byref(h)))
        self._h = h

    def forward(self, n_cycles):
        _check(lib().pkh_forward_taped(self.mesh._h, self._h, int(n_cycles)))

    def replay(self):
        """Advance the mesh's current state with the recorded timesteps."""
        _check(lib().pkh_tape_replay(self.mesh._h, self._h))

    def set_facewise(self, on=True):
        """Use the face-wise reverse (needed with level jumps or walls)."""
        _check(lib().pkh_tape_set_facewise(self._h, 1 if on else 0))

    def adjoint(self, lam_final):
        """lam_final: float64 CUDA tensor in the upload layout; returns dL/dU0."""
        torch = self.mesh.torch
        lam = lam_final.contiguous()
        assert lam.dtype == torch.float64 and lam.is_cuda and tuple(lam.shape) == self.mesh.shape()
        self.mesh.stream.wait_stream(torch.cuda.current_stream(lam.device))
        out = torch.empty_like(lam)
        _check(lib().pkh_adjoint(self.mesh._h, self._h, C.c_void_p(lam.data_ptr()),
                                 C.c_void_p(out.data_ptr())))
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pkh_tape_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _euler_vl2_function():
    import torch

    class EulerVL2(torch.autograd.Function):
        """U_N = n_cycles of the VL2 cycle applied to U_0 on the GPU mesh;
        backward runs the hand-written adjoint with checkpointing (timesteps
        frozen at the forward's values)."""

        @staticmethod
        def forward(ctx, U0, mesh, n_cycles, ckpt_every):
            mesh.upload(U0)
            tape = mesh.tape(ckpt_every)
            tape.forward(n_cycles)
            UN = mesh.download(device=True)
            ctx.tape = tape
            return UN

        @staticmethod
        def backward(ctx, gUN):
            g0 = ctx.tape.adjoint(gUN.to(torch.float64))
            return g0, None, None, None

    return EulerVL2


_EULER_FN = None


def euler_vl2(U0, mesh, n_cycles, ckpt_every=10):
    """Differentiable n-cycle update of a state tensor [nleaves][5][n3][n2][n1]
    (float64, on the mesh's GPU) -- see EulerVL2."""
    global _EULER_FN
    if _EULER_FN is None:
        _EULER_FN = _euler_vl2_function()
    return _EULER_FN.apply(U0, mesh, int(n_cycles), int(ckpt_every))


BATCH_MODES = {"plain": 0, "fused": 1, "graph": 2, "persistent": 3}


class Batch:
    """Independent meshes advanced together (they must share a stream; they
    may be multilevel). Modes: 'plain' (each mesh's own launches), 'fused'
    (grouped launches over every mesh's tiles), 'graph' (fused, replayed
    from captured 50-cycle hipGraphs), 'persistent' (one persistent launch
    per segment of up to 50 cycles); bitwise identical results. tile_rows:
    tile rows of the grouped launches for every member (0: each mesh's own)."""

    def __init__(self, meshes, tile_rows=0):
        self.meshes = list(meshes)
        arr = (C.c_void_p * len(self.meshes))(*[m._h.value for m in self.meshes])
        h = C.c_void_p()
        tun = Tuning()
        tun.tile_rows = int(tile_rows)
        _check(lib().pkh_batch_create(arr, len(self.meshes), C.byref(tun), C.byref(h)))
        self._h = h

    def step(self, n_cycles, mode="fused"):
        _check(lib().pkh_batch_step(self._h, int(n_cycles), BATCH_MODES[mode]))

    def autotune(self, trial_cycles=3):
        out = (C.c_int32 * len(self.meshes))()
        _check(lib().pkh_batch_autotune(self._h, int(trial_cycles), out))
        return list(out)

    def set_tuning(self, waves_per_simd=0, wait_limit_s=2.0):
        """Persistent-mode knobs: kernel variant (2 or 3 waves per SIMD) and
        the bound of its waits in seconds."""
        t = BatchTuning()
        t.waves_per_simd = int(waves_per_simd)
        t.wait_limit_s = float(wait_limit_s)
        _check(lib().pkh_batch_set_tuning(self._h, C.byref(t)))

    def tuning(self):
        t = BatchTuning()
        _check(lib().pkh_batch_get_tuning(self._h, C.byref(t)))
        return {"waves_per_simd": t.waves_per_simd, "wait_limit_s": t.wait_limit_s}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pkh_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
