"""Seeded synthetic inputs: leaf lists and initial states.

This module holds no arithmetic of the hydro method: it only builds block
lists and initial conditions, which the GPU path and the CPU oracle then
receive identically. It imports nothing from the rest of the package.

Random numbers come from a counter-based generator: SplitMix64 (Steele,
Lea & Flood 2014) keyed by (seed, field, global cell index), mapped to
uniforms in (0, 1) and to normals by Box-Muller. The initial state is
therefore independent of how the domain is cut into blocks.

State layout: ``[nleaves][5][n3][n2][n1]`` conserved variables
(rho, Mx, My, Mz, E), x fastest, leaves in the order given.
"""
import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _splitmix64(x):
    x = (x + np.uint64(0x9E3779B97F4A7C15)) & _M64
    z = x
    z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & _M64
    z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & _M64
    return z ^ (z >> np.uint64(31))


def uniforms(seed, field, index):
    """Uniform deviates in (0, 1) for integer cell indices (any shape)."""
    with np.errstate(over="ignore"):
        k = _splitmix64(np.uint64(seed))
        k = _splitmix64(k ^ np.uint64(field))
        x = _splitmix64(np.asarray(index, dtype=np.uint64) ^ k)
    return ((x >> np.uint64(11)).astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


def normals(seed, field, index):
    """Standard normal deviates by Box-Muller from two keyed streams."""
    index = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        u1 = uniforms(seed, 2 * field, index)
        u2 = uniforms(seed, 2 * field + 1, index)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


# ---------------------------------------------------------------------------
# Leaf lists
# ---------------------------------------------------------------------------

def uniform_leaves(nrb):
    """All level-0 blocks of a root grid of nrb = (bx, by, bz) blocks."""
    bx, by, bz = nrb
    return np.array([(0, x, y, z) for z in range(bz) for y in range(by) for x in range(bx)],
                    dtype=np.int32)


def sphere_refined_leaves(nrb, center=(0.5, 0.5, 0.5), radius=0.25, xmin=(0, 0, 0),
                          xmax=(1, 1, 1)):
    """Level-0 blocks, with every block whose open interior meets the open
    ball |x - center| < radius replaced by its 8 level-1 children."""
    out = []
    for z in range(nrb[2]):
        for y in range(nrb[1]):
            for x in range(nrb[0]):
                lo = [xmin[d] + (v) * (xmax[d] - xmin[d]) / nrb[d] for d, v in enumerate((x, y, z))]
                hi = [xmin[d] + (v + 1) * (xmax[d] - xmin[d]) / nrb[d] for d, v in enumerate((x, y, z))]
                near = [min(max(center[d], lo[d]), hi[d]) for d in range(3)]
                dist2 = sum((near[d] - center[d]) ** 2 for d in range(3))
                if dist2 < radius * radius:
                    for c in range(8):
                        out.append((1, 2 * x + (c & 1), 2 * y + ((c >> 1) & 1), 2 * z + ((c >> 2) & 1)))
                else:
                    out.append((0, x, y, z))
    return np.array(out, dtype=np.int32)


def cube_refined_leaves(nrb, lo=0.3, hi=0.7, max_level=3):
    """Leaves of a mesh on the unit cube with nrb level-0 blocks whose
    cubic region (lo, hi)^3 is refined to max_level: level by level, every
    leaf whose open extent meets the open cube is split into 8 children,
    then leaves are refined until every leaf's face, edge and corner
    neighbours are at most one level coarser (periodic). With 8^3 root
    blocks, the 0.4-side cube centred in the box and three levels this
    gives the paper's multilevel mesh (296, 1216, 1352, 21952 blocks on
    levels 0-3). Returns [n][4] (level, lx, ly, lz), unordered."""
    leaves = {(0, x, y, z) for z in range(nrb[2]) for y in range(nrb[1]) for x in range(nrb[0])}

    def nbl(L, d):
        return nrb[d] << L

    def cover(L, x, y, z):
        for Lc in range(L, -1, -1):
            sh = L - Lc
            key = (Lc, x >> sh, y >> sh, z >> sh)
            if key in leaves:
                return key
        return None

    def split(leaf):
        L, x, y, z = leaf
        leaves.discard(leaf)
        for c in range(8):
            leaves.add((L + 1, 2 * x + (c & 1), 2 * y + ((c >> 1) & 1), 2 * z + ((c >> 2) & 1)))

    def meets(leaf):
        L, x, y, z = leaf
        for d, c in enumerate((x, y, z)):
            w = 1.0 / nbl(L, d)
            if not (c * w < hi and (c + 1) * w > lo):
                return False
        return True

    def balance():
        changed = True
        while changed:
            changed = False
            for leaf in sorted(leaves, reverse=True):
                if leaf not in leaves or leaf[0] < 2:
                    continue
                L, x, y, z = leaf
                for dz in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            if not (dx or dy or dz):
                                continue
                            q = (L, (x + dx) % nbl(L, 0), (y + dy) % nbl(L, 1), (z + dz) % nbl(L, 2))
                            c = cover(*q)
                            if c is not None and c[0] < L - 1:
                                split(c)
                                changed = True

    for L in range(max_level):
        for leaf in [lf for lf in leaves if lf[0] == L and meets(lf)]:
            split(leaf)
        balance()
    return np.array(sorted(leaves), dtype=np.int32)


def cell_centers(leaf, n, nrb, xmin=(0.0, 0.0, 0.0), xmax=(1.0, 1.0, 1.0)):
    """Cell-centre coordinates (x, y, z), each shaped [n3][n2][n1]."""
    lev, lx, ly, lz = (int(v) for v in leaf)
    axes = []
    for d, l in enumerate((lx, ly, lz)):
        N = nrb[d] * n[d] * (1 << lev)
        dx = (xmax[d] - xmin[d]) / N
        axes.append(xmin[d] + (l * n[d] + np.arange(n[d]) + 0.5) * dx)
    z, y, x = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return x, y, z


def global_index(leaf, n, nrb):
    """Global cell index (k*N2 + j)*N1 + i at the leaf's level, [n3][n2][n1]."""
    lev, lx, ly, lz = (int(v) for v in leaf)
    N1 = nrb[0] * n[0] << lev
    N2 = nrb[1] * n[1] << lev
    i = lx * n[0] + np.arange(n[0], dtype=np.int64)
    j = ly * n[1] + np.arange(n[1], dtype=np.int64)
    k = lz * n[2] + np.arange(n[2], dtype=np.int64)
    K, J, I = np.meshgrid(k, j, i, indexing="ij")
    return ((K * N2 + J) * N1 + I).astype(np.uint64)


def _to_conserved(rho, vx, vy, vz, p, gamma):
    out = np.empty((5,) + np.shape(rho))
    out[0] = rho
    out[1] = rho * vx
    out[2] = rho * vy
    out[3] = rho * vz
    out[4] = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz)
    return out


# ---------------------------------------------------------------------------
# Initial conditions
# ---------------------------------------------------------------------------

def sound_wave(leaves, n, nrb, amp=1e-6, noise=1e-8, seed=1, gamma=5.0 / 3.0, rho0=1.0,
               p0=0.6, kvec=(1, 0, 0), xmin=(0, 0, 0), xmax=(1, 1, 1)):
    """Right-going linear sound wave on a uniform background plus keyed
    white noise on each conserved field.

    With rho0 = 1, p0 = 0.6, gamma = 5/3 the sound speed is 1 and the
    eigenvector is (1, 1, 0, 0, 1.5) along kvec = (1, 0, 0)."""
    cs = np.sqrt(gamma * p0 / rho0)
    kv = np.asarray(kvec, dtype=np.float64)
    khat = kv / np.linalg.norm(kv)
    h0 = (p0 / (gamma - 1.0) + p0) / rho0
    eig = np.array([1.0, cs * khat[0], cs * khat[1], cs * khat[2], h0])
    U = np.empty((len(leaves), 5, n[2], n[1], n[0]))
    for b, lf in enumerate(leaves):
        x, y, z = cell_centers(lf, n, nrb, xmin, xmax)
        phase = 2.0 * np.pi * (kv[0] * x + kv[1] * y + kv[2] * z)
        bg = _to_conserved(np.full_like(x, rho0), 0 * x, 0 * x, 0 * x, np.full_like(x, p0), gamma)
        s = np.sin(phase)
        U[b] = bg + amp * eig[:, None, None, None] * s[None]
        if noise:
            gi = global_index(lf, n, nrb)
            for v in range(5):
                U[b, v] += noise * normals(seed, v, gi)
    return U


def uniform_state(leaves, n, rho=1.0, v=(0.0, 0.0, 0.0), p=1.0, gamma=5.0 / 3.0):
    U = np.empty((len(leaves), 5, n[2], n[1], n[0]))
    one = np.ones((n[2], n[1], n[0]))
    U[:] = _to_conserved(rho * one, v[0] * one, v[1] * one, v[2] * one, p * one, gamma)[None]
    return U


def smooth_flow(leaves, n, nrb, gamma=5.0 / 3.0, xmin=(0, 0, 0), xmax=(1, 1, 1)):
    """A smooth flow with no symmetry, from the cell-centre coordinates (any
    levels): density 1 +- 0.4, pressure 1 +- 0.25, speeds up to about 0.6,
    not periodic across the domain (a test flow for walls)."""
    U = np.empty((len(leaves), 5, n[2], n[1], n[0]))
    tp = 2.0 * np.pi
    for b, lf in enumerate(leaves):
        x, y, z = cell_centers(lf, n, nrb, xmin, xmax)
        rho = 1.0 + 0.3 * np.sin(tp * (x + 0.13)) * np.cos(tp * (y - 0.2)) + 0.1 * np.cos(tp * z)
        vx = 0.2 + 0.3 * np.cos(tp * (x + y))
        vy = 0.3 * np.sin(tp * (x - z))
        vz = 0.25 * np.cos(tp * (y + 0.3 * x))
        p = 1.0 + 0.25 * np.sin(tp * (y + z + 0.1 * x))
        U[b] = _to_conserved(rho, vx, vy, vz, p, gamma)
    return U


def kelvin_helmholtz(leaves, n, nrb, seed=8, gamma=5.0 / 3.0, drho=1.0, u0=0.5, width=0.05,
                     amp=0.01, sigma=0.2, noise=1e-3, p0=2.5):
    """Two smoothed shear layers at y = 1/4 and 3/4 in a periodic unit box:
    density 1 outside and 1 + drho between them, x velocity -u0 outside and
    +u0 between them (tanh profiles of the given width), a single-mode y
    velocity seed amp sin(2 pi x) localised on the layers (Gaussian of width
    sigma), uniform pressure p0, and keyed white noise of size noise on the
    z velocity so the flow leaves the plane."""
    U = np.empty((len(leaves), 5, n[2], n[1], n[0]))
    tp = 2.0 * np.pi
    for b, lf in enumerate(leaves):
        x, y, z = cell_centers(lf, n, nrb)
        prof = np.tanh((y - 0.25) / width) - np.tanh((y - 0.75) / width)
        rho = 1.0 + 0.5 * drho * prof
        vx = u0 * (prof - 1.0)
        vy = amp * np.sin(tp * x) * (np.exp(-((y - 0.25) / sigma) ** 2) + np.exp(-((y - 0.75) / sigma) ** 2))
        vz = noise * normals(seed, 3, global_index(lf, n, nrb)) if noise else 0.0 * x
        U[b] = _to_conserved(rho, vx, vy, vz, np.full_like(x, p0), gamma)
    return U


def _smoothed_field(N, seed, field, sigma=4.0, trunc=12):
    """Unit-variance, zero-mean periodic field: keyed white noise convolved
    with a separable Gaussian (sigma cells, truncated at +-trunc cells)."""
    N1, N2, N3 = N
    idx = np.arange(N1 * N2 * N3, dtype=np.uint64).reshape(N3, N2, N1)
    w = normals(seed, field, idx)
    spec = np.fft.rfftn(w)
    kern = []
    for Nd in (N3, N2, N1):
        k = np.zeros(Nd)
        offs = np.arange(-trunc, trunc + 1)
        wts = np.exp(-0.5 * (offs / sigma) ** 2)
        wts /= wts.sum()
        np.add.at(k, offs % Nd, wts)
        kern.append(np.fft.fft(k))
    K3 = kern[0][:, None, None] * kern[1][None, :, None] * kern[2][None, None, : N1 // 2 + 1]
    g = np.fft.irfftn(spec * K3, s=(N3, N2, N1), axes=(0, 1, 2))
    g -= g.mean()
    g /= g.std()
    return g


def _scatter(fields, leaves, n):
    U = np.empty((len(leaves), 5, n[2], n[1], n[0]))
    for b, (lev, lx, ly, lz) in enumerate(leaves):
        assert lev == 0
        U[b] = fields[:, lz * n[2]:(lz + 1) * n[2], ly * n[1]:(ly + 1) * n[1], lx * n[0]:(lx + 1) * n[0]]
    return U


def generic_flow(leaves, n, nrb, seed=3, gamma=5.0 / 3.0, xmin=(0, 0, 0), xmax=(1, 1, 1)):
    """A smooth flow without symmetries, on leaves of any level: each of rho,
    v_x, v_y, v_z, P is a sum of 4 plane waves with seeded integer wave
    vectors (components in -2..2) and phases, so no field is constant along
    any direction and no two neighbouring differences are equal by
    construction (no exact ties in the limiter or wave-speed choices).
    rho = 1 + 0.3 f_0, v = 0.3 f_1..3, P = 1 + 0.2 f_4 with |f| <= 1."""
    rng = np.random.default_rng(seed)
    modes = [(rng.integers(-2, 3, size=(4, 3)), rng.uniform(0.0, 2.0 * np.pi, size=4)) for _ in range(5)]
    U = np.empty((len(leaves), 5, n[2], n[1], n[0]))
    for b, lf in enumerate(leaves):
        x, y, z = cell_centers(lf, n, nrb, xmin, xmax)
        f = []
        for ks, ph in modes:
            acc = np.zeros_like(x)
            for k, p in zip(ks, ph):
                acc += np.sin(2.0 * np.pi * (k[0] * x + k[1] * y + k[2] * z) + p)
            f.append(acc / 4.0)
        U[b] = _to_conserved(1.0 + 0.3 * f[0], 0.3 * f[1], 0.3 * f[2], 0.3 * f[3], 1.0 + 0.2 * f[4], gamma)
    return U


def turbulent_box(leaves, n, nrb, seed=2, gamma=5.0 / 3.0, sigma_ln=0.5, mach=0.5, p0=1.0):
    """Log-normal density rho = exp(sigma g - sigma^2/2) from a smoothed
    unit-variance field g, uniform pressure p0, and a velocity of three
    independent smoothed fields scaled to rms |v| = mach * sqrt(gamma p0)."""
    N = (nrb[0] * n[0], nrb[1] * n[1], nrb[2] * n[2])
    return scatter_global(turbulent_box_global(N, seed, gamma, sigma_ln, mach, p0), leaves, n)


def scatter_global(fields, leaves, n):
    """Level-0 leaves' blocks [nleaves][5][n3][n2][n1] cut from global
    conserved fields [5][N3][N2][N1]."""
    return _scatter(fields, leaves, n)


def turbulent_box_global(N, seed=2, gamma=5.0 / 3.0, sigma_ln=0.5, mach=0.5, p0=1.0):
    """The turbulent_box fields on the whole N[0] x N[1] x N[2] grid,
    [5][N3][N2][N1] (independent of any block decomposition)."""
    g = _smoothed_field(N, seed, 0)
    rho = np.exp(sigma_ln * g - 0.5 * sigma_ln * sigma_ln)
    del g
    scale = mach * np.sqrt(gamma * p0) / np.sqrt(3.0)
    vel = [scale * _smoothed_field(N, seed, 1 + d) for d in range(3)]
    fields = _to_conserved(rho, vel[0], vel[1], vel[2], p0 * np.ones_like(rho), gamma)
    del vel, rho
    return fields


def blast(leaves, n, nrb, p_in=100.0, p_out=0.1, r=0.1, rho0=1.0, center=(0.5, 0.5, 0.5),
          gamma=5.0 / 3.0, xmin=(0, 0, 0), xmax=(1, 1, 1)):
    """Spherical blast: uniform density at rest, pressure p_in where the cell
    centre lies within r of the centre, else p_out."""
    U = np.empty((len(leaves), 5, n[2], n[1], n[0]))
    # the outer state everywhere (as _to_conserved gives it), then the leaves
    # that can hold a cell centre inside the ball cell by cell
    U[:, 0] = rho0
    U[:, 1:4] = 0.0
    U[:, 4] = p_out / (gamma - 1.0) + 0.5 * rho0 * 0.0
    for b, lf in enumerate(leaves):
        lev = int(lf[0])
        d2 = 0.0
        for d in range(3):
            w = (xmax[d] - xmin[d]) / (nrb[d] << lev)
            lo = xmin[d] + int(lf[1 + d]) * w
            near = min(max(center[d], lo), lo + w)
            d2 += (near - center[d]) ** 2
        if d2 >= r * r:
            continue
        x, y, z = cell_centers(lf, n, nrb, xmin, xmax)
        d2 = (x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2
        p = np.where(d2 < r * r, p_in, p_out)
        U[b] = _to_conserved(rho0 + 0 * x, 0 * x, 0 * x, 0 * x, p, gamma)
    return U


def smooth_density(leaves, n, nrb, seed=5, amp=1e-3, kmax=4, rho0=1.0, p0=0.6,
                   gamma=5.0 / 3.0):
    """rho = rho0 + delta, delta a sum of Fourier modes 1 <= |k|_inf <= kmax
    with N(0,1) cosine and sine coefficients (keyed by mode index), rescaled
    to max |delta| = amp on the cells given; gas at rest, pressure p0."""
    ks = [(kx, ky, kz) for kz in range(-kmax, kmax + 1) for ky in range(-kmax, kmax + 1)
          for kx in range(-kmax, kmax + 1) if 1 <= max(abs(kx), abs(ky), abs(kz))]
    coef = normals(seed, 0, np.arange(2 * len(ks), dtype=np.uint64)).reshape(len(ks), 2)
    deltas = []
    for lf in leaves:
        x, y, z = cell_centers(lf, n, nrb)
        dl = np.zeros_like(x)
        for (kx, ky, kz), (a, bcoef) in zip(ks, coef):
            ph = 2.0 * np.pi * (kx * x + ky * y + kz * z)
            dl += a * np.cos(ph) + bcoef * np.sin(ph)
        deltas.append(dl)
    mx = max(np.abs(d).max() for d in deltas)
    U = np.empty((len(leaves), 5, n[2], n[1], n[0]))
    for b, dl in enumerate(deltas):
        rho = rho0 + amp * dl / mx
        U[b] = _to_conserved(rho, 0 * rho, 0 * rho, 0 * rho, p0 + 0 * rho, gamma)
    return U


def batch_mix(n=64, seed=4, sizes=(32, 48, 64, 80, 96, 112, 128)):
    """Seeded mix of independent periodic unit-cube instances: edge N drawn
    uniformly from `sizes`, block edge 32 when 32 divides N and a coin flip
    says so (else 16), initial condition a sound wave or a spherical blast
    (coin flip). Returns a list of dicts (N, blk, kind)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        N = int(rng.choice(sizes))
        blk = 32 if (N % 32 == 0 and rng.random() < 0.5) else 16
        kind = "blast" if rng.random() < 0.5 else "wave"
        out.append({"N": N, "blk": blk, "kind": kind})
    return out


def batch_state(spec, leaves):
    """Initial state of one batch instance (see batch_mix)."""
    n = (spec["blk"],) * 3
    nrb = (spec["N"] // spec["blk"],) * 3
    if spec["kind"] == "blast":
        return blast(leaves, n, nrb)
    return sound_wave(leaves, n, nrb, amp=1e-3, noise=0.0)
