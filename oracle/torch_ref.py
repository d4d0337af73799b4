"""Uniform grid formulation in plain PyTorch CPU FP64 ops.

TEST INFRASTRUCTURE. An independent re-derivation of the same update as the
C oracle, written on one global array ``[5][N3][N2][N1]`` with neighbours
taken by ``torch.roll`` (no blocks, no ghost zones, no tables), so it
cross-checks the C oracle's block decomposition and ghost exchange. Through
autograd it is also the reference gradient of the adjoint: the timestep of
each cycle is detached (frozen), every other operation is differentiated.

Domain boundaries other than periodic (``bc`` per face x-, x+, y-, y+, z-,
z+: 0 periodic, 1 outflow, 2 reflecting) extend the array by two cells
beyond each face along the direction being differenced: the nearest cell
(outflow, zero gradient) or the mirror image with the normal velocity
negated (reflecting); fluxes are then taken on all N+1 faces.

Method (Parthenon paper Sec. 4.1; readings of the Athena++ lineage):
  * primitive variables w = (rho, v, P), P = (gamma-1)(E - |M|^2/(2 rho));
  * donor-cell or PLM reconstruction with the monotonised-central limiter;
  * HLLE with Einfeldt wave speeds from Roe averages;
  * VL2: U* = U - dt/2 D_DC(U), U' = U - dt D_PLM(U*);
  * dt = cfl * min_cells,d dx_d / (|v_d| + c).
"""
import torch

# tensor dim holding each spatial direction of a [5][N3][N2][N1] array
_DIM = {0: 3, 1: 2, 2: 1}


def to_prim(U, gamma):
    rho = U[0]
    vx, vy, vz = U[1] / rho, U[2] / rho, U[3] / rho
    kin = 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) / rho
    p = (gamma - 1.0) * (U[4] - kin)
    return torch.stack([rho, vx, vy, vz, p])


def mc_slope(dl, dr, log=None):
    a, b, c = 2.0 * dl.abs(), 2.0 * dr.abs(), 0.5 * (dl + dr).abs()
    mag = torch.minimum(torch.minimum(a, b), c)
    pos = dl * dr > 0.0
    if log is not None:
        # branch taken: 0 no slope, else 1 + which bound is the smallest
        # (first in the order 2|dl|, 2|dr|, |dl+dr|/2 on ties)
        which = torch.where(a <= torch.minimum(b, c), 1, torch.where(b <= c, 2, 3))
        log.append(torch.where(pos, which, 0).to(torch.int8))
    return torch.where(pos, torch.sign(dl) * mag, torch.zeros_like(dl))


def hlle_flux(wl, wr, d, gamma, log=None):
    """Conserved flux through faces normal to d from primitive states
    wl, wr shaped [5][...]. With ``log`` a list, appends the branches the
    wave-speed bounds take (which argument attains the max / min)."""
    g1 = gamma - 1.0
    rl, pl, rr, pr = wl[0], wl[4], wr[0], wr[4]
    vl, vr = wl[1:4], wr[1:4]
    ul, ur = vl[d], vr[d]
    el = pl / g1 + 0.5 * rl * (vl * vl).sum(0)
    er = pr / g1 + 0.5 * rr * (vr * vr).sum(0)
    hl, hr = (el + pl) / rl, (er + pr) / rr
    cl, cr = torch.sqrt(gamma * pl / rl), torch.sqrt(gamma * pr / rr)
    sl, sr = torch.sqrt(rl), torch.sqrt(rr)
    wgt = sl / (sl + sr)
    vbar = wgt * vl + (1.0 - wgt) * vr
    hbar = wgt * hl + (1.0 - wgt) * hr
    abar = torch.sqrt(g1 * (hbar - 0.5 * (vbar * vbar).sum(0)))
    zero = torch.zeros_like(ul)
    bp = torch.maximum(torch.maximum(vbar[d] + abar, ur + cr), zero)
    bm = torch.minimum(torch.minimum(vbar[d] - abar, ul - cl), zero)
    if log is not None:
        p1, p2 = vbar[d] + abar, ur + cr
        m1, m2 = vbar[d] - abar, ul - cl
        log.append(torch.where(p1 >= torch.maximum(p2, zero), 0, torch.where(p2 >= zero, 1, 2)).to(torch.int8))
        log.append(torch.where(m1 <= torch.minimum(m2, zero), 0, torch.where(m2 <= zero, 1, 2)).to(torch.int8))

    def phys(r, v, p, e):
        u = v[d]
        mom = [r * u * v[c] + (p if c == d else 0.0) for c in range(3)]
        return torch.stack([r * u] + mom + [(e + p) * u])

    def cons(r, v, e):
        return torch.stack([r, r * v[0], r * v[1], r * v[2], e])

    fl, fr = phys(rl, vl, pl, el), phys(rr, vr, pr, er)
    ul_c, ur_c = cons(rl, vl, el), cons(rr, vr, er)
    return (bp * fl - bm * fr + bp * bm * (ur_c - ul_c)) / (bp - bm)


def face_flux(W, d, recon, gamma, log=None):
    """Flux at the lower face (i - 1/2 along d) of every cell (periodic)."""
    ax = _DIM[d]
    q0 = W
    qm1 = torch.roll(W, 1, ax)
    if recon == 0:
        return hlle_flux(qm1, q0, d, gamma, log)
    qm2 = torch.roll(W, 2, ax)
    qp1 = torch.roll(W, -1, ax)
    wl = qm1 + 0.5 * mc_slope(qm1 - qm2, q0 - qm1, log)
    wr = q0 - 0.5 * mc_slope(q0 - qm1, qp1 - q0, log)
    return hlle_flux(wl, wr, d, gamma, log)


def extend(W, d, bc):
    """Primitive array W with two cells added beyond each face along d, per
    the boundary kind of that face: wrapped, the nearest cell (outflow), or
    the mirror image with velocity component d negated (reflecting)."""
    ax = _DIM[d]
    n = W.shape[ax]
    sign = torch.ones(5, dtype=W.dtype)
    sign[1 + d] = -1.0
    sign = sign.view(5, *([1] * (W.dim() - 1)))
    sides = []
    for side in (0, 1):
        kind = bc[2 * d + side]
        edge = W.narrow(ax, 0, 2) if side == 0 else W.narrow(ax, n - 2, 2)
        if kind == 0:
            g = W.narrow(ax, n - 2, 2) if side == 0 else W.narrow(ax, 0, 2)
        elif kind == 1:
            one = W.narrow(ax, 0, 1) if side == 0 else W.narrow(ax, n - 1, 1)
            g = torch.cat([one, one], ax)
        elif kind == 2:
            g = torch.flip(edge, (ax,)) * sign
        else:
            raise ValueError(f"unknown boundary kind {kind}")
        sides.append(g)
    return torch.cat([sides[0], W, sides[1]], ax)


def face_flux_bc(W, d, recon, gamma, bc, log=None):
    """Fluxes on the N+1 faces along d (face f between cells f-1 and f)."""
    ax = _DIM[d]
    n = W.shape[ax]
    Wp = extend(W, d, bc)
    qm2, qm1, q0, qp1 = (Wp.narrow(ax, o, n + 1) for o in range(4))
    if recon == 0:
        return hlle_flux(qm1, q0, d, gamma, log)
    wl = qm1 + 0.5 * mc_slope(qm1 - qm2, q0 - qm1, log)
    wr = q0 - 0.5 * mc_slope(q0 - qm1, qp1 - q0, log)
    return hlle_flux(wl, wr, d, gamma, log)


def divergence(U, recon, gamma, dx, log=None, bc=None):
    W = to_prim(U, gamma)
    D = None
    for d in range(3):
        ax = _DIM[d]
        if bc is None:
            F = face_flux(W, d, recon, gamma, log)
            term = (torch.roll(F, -1, ax) - F) / dx[d]
        else:
            F = face_flux_bc(W, d, recon, gamma, bc, log)
            n = W.shape[ax]
            term = (F.narrow(ax, 1, n) - F.narrow(ax, 0, n)) / dx[d]
        D = term if D is None else D + term
    return D


def cfl_dt(U, gamma, cfl, dx):
    W = to_prim(U, gamma)
    c = torch.sqrt(gamma * W[4] / W[0])
    best = None
    for d in range(3):
        q = (dx[d] / (W[1 + d].abs() + c)).min()
        best = q if best is None else torch.minimum(best, q)
    return cfl * best


def cycle(U, dt, gamma, dx, stage1_recon=0, log=None, bc=None):
    Us = U - 0.5 * dt * divergence(U, stage1_recon, gamma, dx, log, bc)
    return U - dt * divergence(Us, 1, gamma, dx, log, bc)


def run(U, ncycles, gamma=5.0 / 3.0, cfl=0.3, dx=None, stage1_recon=0, dts=None, log=None, bc=None):
    """Advance ncycles; the timestep is evaluated from the detached state
    (or taken from ``dts``). Returns (U, list of dt). With ``log`` a list,
    every limiter and wave-speed branch taken is appended to it (int8
    tensors), so two runs are on the same smooth piece of the map exactly
    when their logs are equal. ``bc``: boundary kind per face (None:
    periodic through ``torch.roll``)."""
    if dx is None:
        dx = tuple(1.0 / U.shape[3 - d] for d in range(3))
    used = []
    for c in range(ncycles):
        dt = cfl_dt(U.detach(), gamma, cfl, dx) if dts is None else torch.as_tensor(dts[c], dtype=U.dtype)
        used.append(float(dt))
        U = cycle(U, dt, gamma, dx, stage1_recon, log, bc)
    return U, used


def blocks_to_global(U, leaves, n, nrb):
    """[nleaves][5][n3][n2][n1] (level-0 leaves) -> [5][N3][N2][N1]."""
    import numpy as np
    G = np.zeros((5, nrb[2] * n[2], nrb[1] * n[1], nrb[0] * n[0]))
    for b, (lev, lx, ly, lz) in enumerate(leaves):
        G[:, lz * n[2]:(lz + 1) * n[2], ly * n[1]:(ly + 1) * n[1], lx * n[0]:(lx + 1) * n[0]] = U[b]
    return G


def global_to_blocks(G, leaves, n):
    import numpy as np
    U = np.zeros((len(leaves), 5, n[2], n[1], n[0]))
    for b, (lev, lx, ly, lz) in enumerate(leaves):
        U[b] = G[:, lz * n[2]:(lz + 1) * n[2], ly * n[1]:(ly + 1) * n[1], lx * n[0]:(lx + 1) * n[0]]
    return U
