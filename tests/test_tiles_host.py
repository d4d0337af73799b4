"""The tile-shape choice of the stage kernels (host build of the library's
own function): every default or accepted request is a compiled variant that
divides the block's rows, for every block shape the mesh accepts. CPU only."""
import ctypes as C

import pytest

from _helpers import host_check_lib

COMPILED = {8: (8,), 16: (8, 16, 4), 32: (8, 4, 16), 64: (4, 2)}


@pytest.fixture(scope="module")
def rows():
    lib = host_check_lib()
    lib.pkhc_tile_rows.argtypes = [C.c_int, C.c_int, C.c_int, C.c_longlong, C.c_int]
    lib.pkhc_tile_rows.restype = C.c_int
    return lambda n1, n2, tj, nb, recon=1: lib.pkhc_tile_rows(n1, n2, tj, nb, recon)


def test_default_always_fits(rows):
    # the mesh accepts nblock[1] in multiples of 8 (n1 <= 32) or 4 (n1 = 64)
    for n1, step in ((8, 8), (16, 8), (32, 8), (64, 4)):
        for n2 in range(step, 9 * step, step):
            for nb in (0, 1, 8, 64, 512, 1024, 4096, 65536):
                for recon in (0, 1):
                    t = rows(n1, n2, 0, nb, recon)
                    assert t in COMPILED[n1] and n2 % t == 0, (n1, n2, nb, recon, t)


def test_default_choices(rows):
    # piecewise-linear stage on 32-cell rows: 8 rows (its three-wave variant)
    assert rows(32, 32, 0, 512) == 8 and rows(32, 32, 0, 0) == 8
    # donor-cell stage on 32-cell rows: 8 rows as well, whatever the launch
    assert rows(32, 32, 0, 512, 0) == 8   # 256^3 in 32^3 blocks: 8192 waves
    assert rows(32, 32, 0, 8, 0) == 8     # small launch
    assert rows(32, 32, 0, 0, 0) == 8     # launch size unknown
    for recon in (0, 1):
        assert rows(16, 16, 0, 960, recon) == 16    # two-level blast
        assert rows(16, 16, 0, 8, recon) == 8
        assert rows(64, 64, 0, 64, recon) == 4
    # 16 rows preferred but not a divisor: the next compiled choice below
    assert rows(32, 24, 0, 4096, 0) == 8
    assert rows(32, 8, 0, 4096, 0) == 8
    assert rows(16, 24, 0, 1024) == 8
    assert rows(16, 8, 0, 2048) == 8


def test_explicit_requests(rows):
    assert rows(32, 32, 4, 512) == 4
    assert rows(32, 24, 16, 0) == -1     # does not divide the rows
    assert rows(32, 32, 2, 0) == -1      # not compiled for this width
    assert rows(64, 8, 2, 0) == 2
    assert rows(12, 16, 0, 0) == -1      # no kernel for this width
