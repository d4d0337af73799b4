"""The operation-counting mirror of the oracle's pointwise formulas computes
the same values as the C oracle, and its counts match counts taken by hand
from the formulas. CPU only."""
import numpy as np

from oracle import flops, oracle as orc

G = 5.0 / 3.0


def _rand_prim(rng):
    return np.array([rng.uniform(0.5, 2.0), *rng.normal(0, 0.5, 3), rng.uniform(0.5, 2.0)])


def test_mirror_matches_the_c_oracle_value_for_value():
    rng = np.random.default_rng(11)
    for _ in range(200):
        w = _rand_prim(rng)
        u = np.array([w[0], w[0] * w[1], w[0] * w[2], w[0] * w[3],
                      w[4] / (G - 1.0) + 0.5 * w[0] * (w[1] ** 2 + w[2] ** 2 + w[3] ** 2)])
        got = [x.v for x in flops.prim([flops.F(x) for x in u], G)]
        assert np.array_equal(got, orc.prim(u, G))
        dl, dr = rng.normal(size=2)
        assert flops.mc(flops.F(dl), flops.F(dr)).v == orc.mc(dl, dr)
        wl, wr = _rand_prim(rng), _rand_prim(rng)
        for d in range(3):
            got = [x.v for x in flops.hlle([flops.F(x) for x in wl], [flops.F(x) for x in wr], d, G)]
            assert np.array_equal(got, orc.hlle(wl, wr, d, G))


def test_counts_by_hand():
    # MC on its slope branch: dl*dr (mul), 2|dl|, 2|dr| (2 mul), |dl+dr|/2
    # (add, mul); 4 comparisons (the sign test, two minima, the sign)
    flops.COUNTS.clear()
    flops.mc(flops.F(0.3), flops.F(0.5))
    assert dict(flops.COUNTS) == {"mul": 4, "add": 1, "cmp": 4}
    # primitive recovery: 3 velocities and the kinetic term over rho (4 div),
    # |M|^2 (3 mul, 2 add), 0.5 * ... (1 mul), E - ke (1 add), (gamma-1) * ... (1 mul)
    flops.COUNTS.clear()
    flops.prim([flops.F(1.0), flops.F(0.1), flops.F(0.2), flops.F(0.3), flops.F(2.0)], G)
    assert dict(flops.COUNTS) == {"div": 4, "mul": 5, "add": 3}
    c = flops.per_zone_cycle()
    # the corrector differs from the predictor by 3 faces x 5 variables x
    # (2 MC slopes + 4 differences + 2 half-slope terms)
    extra = {k: c["corrector"].get(k, 0) - c["predictor"].get(k, 0) for k in ("add", "mul", "cmp")}
    assert extra == {"add": 3 * 5 * (2 * 1 + 4 + 2), "mul": 3 * 5 * (2 * 4 + 2), "cmp": 3 * 5 * 2 * 4}
    assert c["cycle_flops"] == sum(c["flops"].values())


def test_bench_uses_the_counted_flops():
    import bench
    c = flops.per_zone_cycle()
    assert bench.ALG_FLOPS == c["flops"]
