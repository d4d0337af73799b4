"""Uniform periodic grid formulation in plain PyTorch CPU FP64 ops.

TEST INFRASTRUCTURE. An independent re-derivation of the same update as the
C oracle, written on one global array ``[5][N3][N2][N1]`` with neighbours
taken by ``torch.roll`` (no blocks, no ghost zones, no tables), so it
cross-checks the C oracle's block decomposition and ghost exchange. Through
autograd it is also the reference gradient of the adjoint: the timestep of
each cycle is detached (frozen), every other operation is differentiated.

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


def mc_slope(dl, dr):
    mag = torch.minimum(torch.minimum(2.0 * dl.abs(), 2.0 * dr.abs()), 0.5 * (dl + dr).abs())
    return torch.where(dl * dr > 0.0, torch.sign(dl) * mag, torch.zeros_like(dl))


def hlle_flux(wl, wr, d, gamma):
    """Conserved flux through faces normal to d from primitive states
    wl, wr shaped [5][...]."""
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

    def phys(r, v, p, e):
        u = v[d]
        mom = [r * u * v[c] + (p if c == d else 0.0) for c in range(3)]
        return torch.stack([r * u] + mom + [(e + p) * u])

    def cons(r, v, e):
        return torch.stack([r, r * v[0], r * v[1], r * v[2], e])

    fl, fr = phys(rl, vl, pl, el), phys(rr, vr, pr, er)
    ul_c, ur_c = cons(rl, vl, el), cons(rr, vr, er)
    return (bp * fl - bm * fr + bp * bm * (ur_c - ul_c)) / (bp - bm)


def face_flux(W, d, recon, gamma):
    """Flux at the lower face (i - 1/2 along d) of every cell."""
    ax = _DIM[d]
    q0 = W
    qm1 = torch.roll(W, 1, ax)
    if recon == 0:
        return hlle_flux(qm1, q0, d, gamma)
    qm2 = torch.roll(W, 2, ax)
    qp1 = torch.roll(W, -1, ax)
    wl = qm1 + 0.5 * mc_slope(qm1 - qm2, q0 - qm1)
    wr = q0 - 0.5 * mc_slope(q0 - qm1, qp1 - q0)
    return hlle_flux(wl, wr, d, gamma)


def divergence(U, recon, gamma, dx):
    W = to_prim(U, gamma)
    D = None
    for d in range(3):
        F = face_flux(W, d, recon, gamma)
        term = (torch.roll(F, -1, _DIM[d]) - F) / dx[d]
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


def cycle(U, dt, gamma, dx, stage1_recon=0):
    Us = U - 0.5 * dt * divergence(U, stage1_recon, gamma, dx)
    return U - dt * divergence(Us, 1, gamma, dx)


def run(U, ncycles, gamma=5.0 / 3.0, cfl=0.3, dx=None, stage1_recon=0, dts=None):
    """Advance ncycles; the timestep is evaluated from the detached state
    (or taken from ``dts``). Returns (U, list of dt)."""
    if dx is None:
        dx = tuple(1.0 / U.shape[3 - d] for d in range(3))
    used = []
    for c in range(ncycles):
        dt = cfl_dt(U.detach(), gamma, cfl, dx) if dts is None else torch.as_tensor(dts[c], dtype=U.dtype)
        used.append(float(dt))
        U = cycle(U, dt, gamma, dx, stage1_recon)
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
