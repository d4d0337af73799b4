"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
import ctypes
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


CSRC = os.path.join(ROOT, "paper_2202_12309_amd", "csrc")
HOSTCHECK_LIB = os.path.join(ROOT, "paper_2202_12309_amd", "libpkhcheck.so")


def host_check_lib():
    """The library's host build of its pointwise physics and tile-shape
    choice (pkh_hostcheck.cpp), compiled with g++ when stale."""
    src = os.path.join(CSRC, "pkh_hostcheck.cpp")
    deps = [src] + [os.path.join(CSRC, h) for h in ("pkh_physics.h", "pkh_tiles.h")]
    if (not os.path.exists(HOSTCHECK_LIB)
            or os.path.getmtime(HOSTCHECK_LIB) < max(os.path.getmtime(d) for d in deps)):
        tmp = HOSTCHECK_LIB + f".tmp{os.getpid()}"
        subprocess.run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-I", CSRC, src, "-o", tmp],
                       check=True)
        os.replace(tmp, HOSTCHECK_LIB)
    return ctypes.CDLL(HOSTCHECK_LIB)


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def scales(U, gamma):
    """Per-variable error scales of a state [nb][5][...]: max |rho|, max |E|,
    and for each momentum component max over cells of max(|M|, rho c) --
    the size of the momentum-flux terms whose rounding enters M (a fluid
    near rest has |M| << rho c, so |M| alone is no scale)."""
    rho = U[:, 0]
    kin = 0.5 * (U[:, 1] ** 2 + U[:, 2] ** 2 + U[:, 3] ** 2) / rho
    p = (gamma - 1.0) * (U[:, 4] - kin)
    rc = np.sqrt(gamma * np.abs(p) * np.abs(rho))
    mmag = np.sqrt(U[:, 1] ** 2 + U[:, 2] ** 2 + U[:, 3] ** 2)
    sm = max(np.abs(mmag).max(), rc.max())
    return np.array([np.abs(rho).max(), sm, sm, sm, np.abs(U[:, 4]).max()])


def rel_err(a, b, gamma):
    """Per-variable max |a - b| over cells divided by the scale of b."""
    d = np.abs(a - b).reshape(a.shape[0], 5, -1).max(axis=(0, 2))
    return d / scales(b, gamma)


def rel_err_per_variable(a, b):
    """The plain per-variable reading: max |a - b| over cells divided by max
    |b| of the same variable (for a fluid near rest the momentum scale is
    then the flow's own tiny momentum, not the momentum-flux scale)."""
    d = np.abs(a - b).reshape(a.shape[0], 5, -1).max(axis=(0, 2))
    return d / np.abs(b).reshape(b.shape[0], 5, -1).max(axis=(0, 2))


def print_case(msg):
    print(f"[case] {msg}", flush=True)


def bump_directions(N, count, seed):
    """Seeded perturbation directions on an N^3 periodic grid, [5][N][N][N]:
    a Gaussian bump (unit variance in cells, cut at radius 3) with an N(0,1)
    weight per conserved variable. The first is centred on the corner shared
    by the eight blocks of a 2x2x2 decomposition; the others at random cells."""
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    out = []
    for t in range(count):
        c = np.full(3, N / 2 - 0.5) if t == 0 else rng.integers(0, N, 3).astype(float)
        d = [np.minimum(np.abs(a - ca), N - np.abs(a - ca)) for a, ca in zip((x, y, z), c)]
        r2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2
        bump = np.exp(-0.5 * r2) * (r2 <= 9.0)
        out.append(np.stack([bump * rng.normal() for _ in range(5)]))
    return out


def same_branches(log_a, log_b):
    """True when two branch logs of the reference formulation agree entry by
    entry (the two runs sit on the same smooth piece of the map)."""
    return len(log_a) == len(log_b) and all(bool((a == b).all()) for a, b in zip(log_a, log_b))
