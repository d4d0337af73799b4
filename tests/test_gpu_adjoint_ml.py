"""Reverse mode on meshes with level jumps and walls (the face-wise reverse:
transposed flux correction, restriction, prolongation with the forward's
minmod cases, wall images) against central differences of the oracle's
frozen-timestep cycles, on directions along which the oracle takes the same
branches at +h and -h; and the face-wise reverse against the pencil/row
reverse on a single-level mesh. Runs on an MI355X."""
import numpy as np
import pytest
import torch

from _helpers import print_case
from oracle.oracle import BC_OUTFLOW as OUT
from oracle.oracle import BC_PERIODIC as PER
from oracle.oracle import BC_REFLECT as REF
from oracle.oracle import OracleMesh
from paper_2202_12309_amd import inputs

pytestmark = pytest.mark.gpu


def _dv(leaves, nroot):
    """Cell volume of every leaf, [nleaves] (unit cube)."""
    return np.array([1.0 / float(np.prod(nroot)) / 8.0 ** int(l[0]) for l in leaves])


def _gradient(gm, U0, tgt, dV, cycles, ckpt, facewise=None):
    """dL/dU0 on the GPU for L = 1/2 sum (rho_N - rho_T)^2 dV, and the
    timesteps of the recorded cycles (from the GPU's own clock)."""
    tape = gm.tape(ckpt)
    if facewise is not None:
        tape.set_facewise(facewise)
    gm.upload(U0)
    dts = []
    tape.forward(cycles)
    UN = gm.download()
    lam = np.zeros_like(UN)
    lam[:, 0] = (UN[:, 0] - tgt) * dV[:, None, None, None]
    g = tape.adjoint(torch.tensor(lam, device="cuda")).cpu().numpy()
    tape.close()
    return g, UN, dts


def _oracle_dts(om, U0, cycles):
    om.set_state(U0)
    om.set_time(0.0, 0)
    dts = []
    for _ in range(cycles):
        om.step(1)
        dts.append(om.time()[1])
    return dts


def _fd_directions(om, U0, tgt, dV, dts, g, dirs, rtol):
    """For each direction the largest h of a sweep with equal oracle branch
    signatures at +h and -h; central difference of the loss against g.v.
    Returns the relative errors of the accepted directions."""
    def loss_rho(U, sign_h):
        om.set_state(U)
        om.set_time(0.0, 0)
        om.track_branches(True)
        om.step_dts(dts)
        sig = om.branch_signature()
        om.track_branches(False)
        return om.state()[:, 0] - tgt, sig

    accepted = []
    for v in dirs:
        dirder = float((g * v).sum())
        for h in (1e-5, 3e-6, 1e-6, 3e-7):
            ap, sp = loss_rho(U0 + h * v, 1)
            am, sm = loss_rho(U0 - h * v, -1)
            if sp != sm:
                print(f"h {h}: branches differ, next h", flush=True)
                continue
            fd = float((0.5 * (ap - am) * (ap + am) * dV[:, None, None, None]).sum() / (2 * h))
            rel = abs(fd - dirder) / abs(dirder)
            print(f"h {h}: dirder {dirder:.12e} fd {fd:.12e} rel {rel:.2e}", flush=True)
            accepted.append(rel)
            break
    return accepted


def _bumps(om, U0, count, seed, near_level_jump):
    """Localized directions (Gaussian bumps of 1.5 cells, an N(0,1) weight per
    conserved variable); the first ones centred on cells of leaves beside a
    level jump when asked."""
    rng = np.random.default_rng(seed)
    lv = om.leaves()
    out = []
    levels = lv[:, 0]
    for t in range(count):
        if near_level_jump and t < count - 1:
            # a coarse leaf cell next to a fine leaf, or a fine leaf cell next to a coarse leaf
            cand = np.where(levels == (t % 2))[0]
            q = int(rng.choice(cand))
        else:
            q = int(rng.integers(0, len(lv)))
        xc, yc, zc = (a.mean() for a in om.cell_centers(q))
        v = np.zeros_like(U0)
        for b in range(len(lv)):
            x, y, z = om.cell_centers(b)
            r2 = ((x - xc) ** 2 + (y - yc) ** 2 + (z - zc) ** 2) / (1.5 / 32) ** 2
            bump = np.exp(-0.5 * r2) * (r2 <= 9.0)
            for var in range(5):
                v[b, var] = bump
        v *= rng.normal(size=(1, 5, 1, 1, 1))
        out.append(v)
    return out


def _case(lv, nrb, n, max_level, bc=(PER,) * 6):
    from paper_2202_12309_amd.binding import Mesh
    nroot = tuple(nrb[d] * n[d] for d in range(3))
    gm = Mesh(nroot, n, lv, max_level=max_level, bc=bc)
    om = OracleMesh(n, nrb, lv, max_level=max_level, bc=bc)
    assert np.array_equal(gm.leaves(), om.leaves())
    U0 = inputs.generic_flow(gm.leaves(), n, nrb)
    tgt = 0.9 * U0[:, 0] + 0.1
    return gm, om, U0, tgt, _dv(gm.leaves(), nroot)


@pytest.mark.parametrize("recon1", [0, 1])
def test_two_level_gradient_matches_oracle_differences(recon1):
    """A two-level periodic mesh (32^3 root in 8^3 blocks, the 8 central root
    blocks refined: 120 leaves), a smooth flow without symmetries (so no
    branch sits at an exact tie), 2 cycles with a checkpoint
    every cycle: the GPU gradient along localized directions placed beside
    the level jumps meets the oracle's central differences to 1e-8."""
    print_case(f"two-level adjoint vs oracle FD, stage-1 recon {recon1}")
    from paper_2202_12309_amd.binding import Mesh
    nrb, n = (4, 4, 4), (8, 8, 8)
    lv = inputs.sphere_refined_leaves(nrb, radius=0.2)
    gm = Mesh((32,) * 3, n, lv, max_level=1, stage1_recon=recon1)
    om = OracleMesh(n, nrb, lv, max_level=1, stage1_recon=recon1)
    assert np.array_equal(gm.leaves(), om.leaves()) and gm.nleaves == 120
    U0 = inputs.generic_flow(gm.leaves(), n, nrb)
    tgt = 0.9 * U0[:, 0] + 0.1
    dV = _dv(gm.leaves(), (32, 32, 32))
    cycles = 2
    g, UN, _ = _gradient(gm, U0, tgt, dV, cycles, 1)
    dts = _oracle_dts(om, U0, cycles)
    assert np.abs(UN - om.state()).max() <= 1e-12 * np.abs(om.state()).max()
    acc = _fd_directions(om, U0, tgt, dV, dts, g, _bumps(om, U0, 6, seed=7, near_level_jump=True), 1e-8)
    assert len(acc) >= 4, acc
    assert max(acc) <= 1e-8, acc


@pytest.mark.parametrize("bc", [(REF, OUT, PER, PER, OUT, REF), (OUT, OUT, REF, REF, PER, PER)])
def test_walled_gradient_matches_oracle_differences(bc):
    """Outflow and reflecting walls (the transposed image rule), 32^3 in 8
    blocks of 16^3, 2 cycles: GPU gradient against the oracle's central
    differences to 1e-8 on branch-consistent directions, two of them at
    walls."""
    print_case(f"walled adjoint vs oracle FD, bc {bc}")
    nrb, n = (2, 2, 2), (16, 16, 16)
    gm, om, U0, tgt, dV = _case(inputs.uniform_leaves(nrb), nrb, n, 0, bc)
    cycles = 2
    g, UN, _ = _gradient(gm, U0, tgt, dV, cycles, 2)
    dts = _oracle_dts(om, U0, cycles)
    dirs = _bumps(om, U0, 4, seed=11, near_level_jump=False)
    # two bumps centred on wall cells
    for t, (q, cell) in enumerate(((0, (0, 0, 0)), (7, (15, 15, 15)))):
        x, y, z = (a[cell[2], cell[1], cell[0]] for a in om.cell_centers(q))
        v = np.zeros_like(U0)
        for b in range(om.nleaves):
            X, Y, Z = om.cell_centers(b)
            r2 = ((X - x) ** 2 + (Y - y) ** 2 + (Z - z) ** 2) / (1.5 / 32) ** 2
            v[b] = (np.exp(-0.5 * r2) * (r2 <= 9.0))[None]
        dirs.append(v * np.random.default_rng(20 + t).normal(size=(1, 5, 1, 1, 1)))
    acc = _fd_directions(om, U0, tgt, dV, dts, g, dirs, 1e-8)
    assert len(acc) >= 4, acc
    assert max(acc) <= 1e-8, acc


def test_two_level_walled_regrid_free_gradient():
    """Two levels and walls together (refinement touching a reflecting
    face): GPU gradient against the oracle's central differences."""
    print_case("two-level walled adjoint vs oracle FD")
    nrb, n = (4, 4, 4), (8, 8, 8)
    lv = inputs.sphere_refined_leaves(nrb, center=(0.1, 0.5, 0.5), radius=0.2)
    bc = (REF, OUT, PER, PER, PER, PER)
    gm, om, U0, tgt, dV = _case(lv, nrb, n, 1, bc)
    assert (gm.leaves()[:, 0] == 1).sum() > 0
    cycles = 2
    g, _, _ = _gradient(gm, U0, tgt, dV, cycles, 1)
    dts = _oracle_dts(om, U0, cycles)
    acc = _fd_directions(om, U0, tgt, dV, dts, g, _bumps(om, U0, 5, seed=13, near_level_jump=True), 1e-8)
    assert len(acc) >= 3, acc
    assert max(acc) <= 1e-8, acc


def test_facewise_reverse_equals_pencil_row_reverse():
    """On a single-level periodic mesh both reverse implementations apply:
    the face-wise one (atomic accumulation) equals the pencil/row one to
    1e-13 of the gradient's scale."""
    print_case("face-wise vs pencil/row reverse, 32^3 as 8 blocks of 16^3, 3 cycles")
    nrb, n = (2, 2, 2), (16, 16, 16)
    gm, om, U0, tgt, dV = _case(inputs.uniform_leaves(nrb), nrb, n, 0)
    g_rows, _, _ = _gradient(gm, U0, tgt, dV, 3, 2, facewise=False)
    g_face, _, _ = _gradient(gm, U0, tgt, dV, 3, 2, facewise=True)
    scale = np.abs(g_rows).max()
    err = np.abs(g_face - g_rows).max() / scale
    print("max rel diff", err, flush=True)
    assert err <= 1e-13, err
