"""Operation count of the method per zone-cycle (TEST INFRASTRUCTURE).

The oracle's pointwise formulas (primitive recovery, the MC limiter, HLLE with
Einfeldt wave speeds, the flux-divergence update and the CFL signal speed)
written once more over a counting number type, so that every FP64 operation
they perform is tallied by kind. The formulas follow the C oracle operation
for operation (no contraction: a*b + c is a multiply and an add); the tests
check them against the C functions value for value.

Per zone and cycle the method needs (Sec. 4.1, VL2):
  predictor: one primitive recovery per cell, one donor-cell HLLE face per
             cell and direction (three faces per zone), the update;
  corrector: one primitive recovery per cell, per face and direction the
             PLM-MC reconstruction of both face states (two MC slopes and two
             face values per variable) and HLLE, the update;
  the CFL signal speed of the updated cell.
Ghost-cell recomputations of an implementation are not counted.
"""
import math
from collections import Counter

COUNTS = Counter()


class F:
    """A float that counts the arithmetic done on it."""
    __slots__ = ("v",)

    def __init__(self, v):
        self.v = float(v)

    @staticmethod
    def _v(o):
        return o.v if isinstance(o, F) else float(o)

    def __add__(self, o):
        COUNTS["add"] += 1
        return F(self.v + F._v(o))

    __radd__ = __add__

    def __sub__(self, o):
        COUNTS["add"] += 1
        return F(self.v - F._v(o))

    def __rsub__(self, o):
        COUNTS["add"] += 1
        return F(F._v(o) - self.v)

    def __mul__(self, o):
        COUNTS["mul"] += 1
        return F(self.v * F._v(o))

    __rmul__ = __mul__

    def __truediv__(self, o):
        COUNTS["div"] += 1
        return F(self.v / F._v(o))

    def __rtruediv__(self, o):
        COUNTS["div"] += 1
        return F(F._v(o) / self.v)

    def __neg__(self):
        return F(-self.v)  # a sign flip, not an operation

    def __lt__(self, o):
        COUNTS["cmp"] += 1
        return self.v < F._v(o)

    def __gt__(self, o):
        COUNTS["cmp"] += 1
        return self.v > F._v(o)

    def __le__(self, o):
        COUNTS["cmp"] += 1
        return self.v <= F._v(o)


def fsqrt(x):
    COUNTS["sqrt"] += 1
    return F(math.sqrt(x.v))


def fabs(x):
    return F(abs(x.v))  # a sign clear, not an operation


# --- the oracle's formulas ---------------------------------------------------

def prim(u, gamma):
    """orc_prim: (rho, M, E) -> (rho, v, P)."""
    r = u[0]
    w = [r, u[1] / r, u[2] / r, u[3] / r]
    w.append((gamma - 1.0) * (u[4] - 0.5 * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / r))
    return w


def mc(dl, dr):
    """orc_mc: monotonised-central slope."""
    if dl * dr <= 0.0:
        return F(0.0)
    a, b, c = 2.0 * fabs(dl), 2.0 * fabs(dr), 0.5 * fabs(dl + dr)
    m = a
    if b < m:
        m = b
    if c < m:
        m = c
    return m if dl > 0.0 else -m


def hlle(wl, wr, d, gamma):
    """orc_hlle: HLLE flux normal to d from primitive face states."""
    gm1 = gamma - 1.0
    rl, pl, rr, pr = wl[0], wl[4], wr[0], wr[4]
    ul, ur = wl[1 + d], wr[1 + d]
    v2l = wl[1] * wl[1] + wl[2] * wl[2] + wl[3] * wl[3]
    v2r = wr[1] * wr[1] + wr[2] * wr[2] + wr[3] * wr[3]
    el = pl / gm1 + 0.5 * rl * v2l
    er = pr / gm1 + 0.5 * rr * v2r
    hl, hr = (el + pl) / rl, (er + pr) / rr
    cl, cr = fsqrt(gamma * pl / rl), fsqrt(gamma * pr / rr)
    sl, sr = fsqrt(rl), fsqrt(rr)
    r = sl / (sl + sr)
    vb = [r * wl[1 + c] + (1.0 - r) * wr[1 + c] for c in range(3)]
    hb = r * hl + (1.0 - r) * hr
    vb2 = vb[0] * vb[0] + vb[1] * vb[1] + vb[2] * vb[2]
    ab = fsqrt(gm1 * (hb - 0.5 * vb2))
    bp = vb[d] + ab
    if ur + cr > bp:
        bp = ur + cr
    if F(0.0) > bp:
        bp = F(0.0)
    bm = vb[d] - ab
    if ul - cl < bm:
        bm = ul - cl
    if F(0.0) < bm:
        bm = F(0.0)
    uL = [rl] + [rl * wl[1 + c] for c in range(3)] + [el]
    uR = [rr] + [rr * wr[1 + c] for c in range(3)] + [er]
    fl = [rl * ul] + [rl * ul * wl[1 + c] for c in range(3)] + [(el + pl) * ul]
    fr = [rr * ur] + [rr * ur * wr[1 + c] for c in range(3)] + [(er + pr) * ur]
    fl[1 + d] = fl[1 + d] + pl
    fr[1 + d] = fr[1 + d] + pr
    return [(bp * fl[v] - bm * fr[v] + bp * bm * (uR[v] - uL[v])) / (bp - bm) for v in range(5)]


def plm_faces(qm2, qm1, q0, qp1):
    """Both face states of the face between cells m1 and 0, per variable."""
    wl = [qm1[v] + 0.5 * mc(qm1[v] - qm2[v], q0[v] - qm1[v]) for v in range(5)]
    wr = [q0[v] - 0.5 * mc(q0[v] - qm1[v], qp1[v] - q0[v]) for v in range(5)]
    return wl, wr


def update(ubase, fx, fy, fz, dx, coef):
    """Ubase - coef * sum_d (F_d(+1/2) - F_d(-1/2)) / dx_d, per variable
    (fx etc.: pairs of lower and upper face fluxes)."""
    out = []
    for v in range(5):
        div = (fx[1][v] - fx[0][v]) / dx[0] + (fy[1][v] - fy[0][v]) / dx[1]
        div = div + (fz[1][v] - fz[0][v]) / dx[2]
        out.append(ubase[v] - coef * div)
    return out


def signal(u, gamma, dx):
    """CFL: the cell's smallest dx_d / (|v_d| + c) (as cfl_dt evaluates it)."""
    w = prim(u, gamma)
    cs = fsqrt(gamma * w[4] / w[0])
    best = None
    for d in range(3):
        q = dx[d] / (fabs(w[1 + d]) + cs)
        if best is None or q < best:
            best = q
    return best


def _tally(fn):
    COUNTS.clear()
    fn()
    return Counter(COUNTS)


def per_zone_cycle(gamma=5.0 / 3.0):
    """Operation counts per zone and cycle by kind (add, mul, div, sqrt and
    cmp), for the predictor, the corrector and the CFL signal speed, from one
    representative evaluation of each formula (a subsonic state in which
    every limiter takes its slope branch)."""
    def cell(k):
        # a smooth, subsonic profile: rho, M, E of cell k along a direction
        r = 1.0 + 0.1 * k
        vx, vy, vz, p = 0.2 + 0.01 * k, -0.1 + 0.02 * k, 0.05 + 0.03 * k, 1.0 + 0.05 * k
        return [F(r), F(r * vx), F(r * vy), F(r * vz), F(p / (gamma - 1.0) + 0.5 * r * (vx * vx + vy * vy + vz * vz))]
    cells = [cell(k) for k in range(4)]
    dx = (F(1.0), F(1.0), F(1.0))
    coef = F(0.001)

    c_prim = _tally(lambda: prim(cells[1], gamma))
    ws = [prim(c, gamma) for c in cells]
    c_dc = _tally(lambda: hlle(ws[1], ws[2], 0, gamma))
    c_rec = _tally(lambda: plm_faces(ws[0], ws[1], ws[2], ws[3]))
    f = [F(0.1 * v) for v in range(5)]
    c_upd = _tally(lambda: update(cells[1], (f, f), (f, f), (f, f), dx, coef))
    c_sig = _tally(lambda: signal(cells[1], gamma, dx))

    pred = c_prim + c_upd
    corr = c_prim + c_upd
    for _ in range(3):
        pred += c_dc
        corr += c_rec + c_dc
    flops = {k: sum(c[x] for x in ("add", "mul", "div", "sqrt")) for k, c in
             (("predictor", pred), ("corrector", corr), ("cfl", c_sig))}
    return {"predictor": dict(pred), "corrector": dict(corr), "cfl": dict(c_sig),
            "flops": flops, "cycle_flops": flops["predictor"] + flops["corrector"] + flops["cfl"]}


if __name__ == "__main__":
    import json
    print(json.dumps(per_zone_cycle(), indent=1))
