"""The totals entry point that allocates nothing (its partial sums live in a
static device array of the library) against pkh_conserved_totals on the same
meshes: bitwise equal, on two calls in a row with the second mesh smaller
than the first, and a mesh beyond the array's capacity is refused. Runs on
an MI355X, through the C-ABI."""
import ctypes as C

import numpy as np
import pytest

from _helpers import print_case
from paper_2202_12309_amd import inputs

pytestmark = pytest.mark.gpu


def _mesh(nrb, blk, make):
    from paper_2202_12309_amd.binding import Mesh
    n = (blk,) * 3
    m = Mesh(tuple(nrb[d] * blk for d in range(3)), n, inputs.uniform_leaves(nrb))
    m.upload(make(m.leaves(), n, nrb))
    m.step(2)
    return m


def _both(m):
    from paper_2202_12309_amd.binding import lib
    ref = (C.c_double * 5)()
    new = (C.c_double * 5)()
    assert lib().pkh_conserved_totals(m._h, ref) == 0
    assert lib().pkh_conserved_totals_noalloc(m._h, new) == 0, lib().pkh_last_error()
    return np.array(ref[:]), np.array(new[:])


def test_noalloc_totals_equal_allocating_totals():
    print_case("no-allocation totals vs pkh_conserved_totals: 512 then 27 leaves, then 512 again")
    big = _mesh((8, 8, 8), 16, lambda lv, n, nrb: inputs.turbulent_box(lv, n, nrb, seed=3))
    small = _mesh((3, 3, 3), 8, lambda lv, n, nrb: inputs.blast(lv, n, nrb))
    for m in (big, small, big):
        ref, new = _both(m)
        print("totals", ref, flush=True)
        assert np.array_equal(ref, new), (ref, new)
    # the binding's wrapper reads the same entry point
    assert np.array_equal(small.totals_noalloc(), small.totals())
    big.close()
    small.close()


def test_noalloc_totals_refuse_beyond_capacity():
    print_case("no-allocation totals refuse 67240 leaves (capacity 65536)")
    from paper_2202_12309_amd.binding import Mesh, PkhError
    nrb = (41, 41, 40)
    m = Mesh(tuple(8 * x for x in nrb), (8, 8, 8), inputs.uniform_leaves(nrb))
    with pytest.raises(PkhError) as e:
        m.totals_noalloc()
    assert e.value.name == "PKH_EINVAL"
    assert np.all(np.isfinite(m.totals()))  # the allocating entry point still works
    m.close()
