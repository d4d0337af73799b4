"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


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


def print_case(msg):
    print(f"[case] {msg}", flush=True)
