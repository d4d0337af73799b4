"""Host-side behaviour that needs no GPU: the bench's one-GPU contract, the
binding failing loudly without the library, the byte model, and the seeded
inputs (deterministic, independent of the block decomposition)."""
import os
import subprocess
import sys

import numpy as np
import pytest

from _helpers import ROOT
from paper_2202_12309_amd import inputs


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_binding_raises_without_library(monkeypatch):
    from paper_2202_12309_amd import binding
    monkeypatch.setattr(binding, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libpkhydro.so"))
    monkeypatch.setattr(binding, "_lib", None, raising=False)
    with pytest.raises(RuntimeError):
        binding.lib()


def test_byte_model():
    sys.path.insert(0, ROOT)
    import bench
    corr, cycle = bench.algorithmic_bytes(32)
    assert corr == pytest.approx(135.0) and cycle == pytest.approx(222.5)
    assert bench.stage_floor_bytes() == (120.0, 200.0)
    assert bench.ghost_materialised_bytes(32) == pytest.approx(240 * 36 ** 3 / 32 ** 3 - 40)


def test_inputs_deterministic_and_decomposition_independent():
    # the same global field whether the mesh is one block or 8 blocks
    n1, nrb1 = (16, 16, 16), (1, 1, 1)
    n8, nrb8 = (8, 8, 8), (2, 2, 2)
    lv1, lv8 = inputs.uniform_leaves(nrb1), inputs.uniform_leaves(nrb8)
    for make in (lambda lv, n, nrb: inputs.turbulent_box(lv, n, nrb, seed=3),
                 lambda lv, n, nrb: inputs.sound_wave(lv, n, nrb, seed=3),
                 lambda lv, n, nrb: inputs.smooth_density(lv, n, nrb, seed=3)):
        a = make(lv1, n1, nrb1)
        b = make(lv8, n8, nrb8)
        assert np.array_equal(a, make(lv1, n1, nrb1))  # deterministic
        G = np.zeros((5, 16, 16, 16))
        for q, (lev, lx, ly, lz) in enumerate(lv8):
            G[:, lz * 8:(lz + 1) * 8, ly * 8:(ly + 1) * 8, lx * 8:(lx + 1) * 8] = b[q]
        assert np.array_equal(a[0], G)
