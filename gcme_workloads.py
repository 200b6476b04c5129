"""Seeded synthetic inputs for the GCMe nonbonded path.

This module only draws inputs (positions, species, charges, parameters,
initial velocities); it contains none of the method's arithmetic.  Both the
FP64 oracle (tests) and the HIP library (tests, bench) are fed from here.

Workload recipe (reduced units, kT = 1, lengths in the bead diameter d):
  * number density 2.5 d^-3, the coarse-graining level the paper settles on
    (Parametrization section), so L = (N / 2.5)^(1/3) for cubic boxes;
  * positions uniform in [0, L)^3 (numpy PCG64 ``default_rng(seed)``), drawn
    on the 2^-32 L lattice of each edge (the engine's fixed-point grid) unless
    on_lattice=False;
  * charged beads chosen by permutation, exactly half +1 and half -1 (neutral);
  * species assigned by permutation in equal shares;
  * the mass radius sigma_t is tied to the charge radius a_t (one radius per
    species, as in the paper's water mapping d = 2 sigma);
  * A = 25 kT d^3 is what the parametrization formula gives for a four-to-one
    mapping at rho = 2.5.

The paper's own systems are MD snapshots of liquids; uniform random positions
give the same pair count as a liquid at this density (g(r) = 1 on average)
but more close contacts.  No dataset is involved.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

DENSITY = 2.5


@dataclass
class Workload:
    name: str
    pos: np.ndarray          # float64 [N, 3]
    type: np.ndarray         # int32 [N]
    z: np.ndarray            # int32 [N]
    vel: np.ndarray          # float64 [N, 3]
    box: tuple
    rc: float
    beta: float
    lB: float
    A: np.ndarray            # [nt, nt]
    sigma: np.ndarray        # [nt]
    a: np.ndarray            # [nt]
    grid: tuple
    order: int
    dt: float
    gamma: float
    kT: float
    mass: np.ndarray         # [nt]
    seed: int
    kmax: float = 0.0        # exact reciprocal sum cutoff (|k| <= kmax), 0 = unused
    extra: dict = field(default_factory=dict)

    @property
    def N(self):
        return len(self.pos)

    @property
    def nt(self):
        return len(self.sigma)


def smooth_size(x: float) -> int:
    """Smallest 2^a 3^b >= x."""
    best = None
    p2 = 1
    while p2 < 4 * x + 8:
        p3 = p2
        while p3 < 4 * x + 8:
            if p3 >= x and (best is None or p3 < best):
                best = p3
            p3 *= 3
        p2 *= 2
    return int(best)


def _charges(rng, N, frac):
    """round(frac/2 N) beads at +1 and as many at -1."""
    n_charged = 2 * int(round(0.5 * frac * N))
    z = np.zeros(N, dtype=np.int32)
    idx = rng.permutation(N)[:n_charged]
    z[idx[: n_charged // 2]] = 1
    z[idx[n_charged // 2:]] = -1
    return z


def _species(rng, N, nt):
    t = np.arange(N, dtype=np.int32) % nt
    return rng.permutation(t).astype(np.int32)


def _velocities(rng, N, mass_per_bead, kT):
    v = rng.standard_normal((N, 3)) * np.sqrt(kT / mass_per_bead)[:, None]
    v -= (v * mass_per_bead[:, None]).sum(0) / mass_per_bead.sum()
    return v


def _sym_uniform(rng, nt, lo, hi):
    m = rng.uniform(lo, hi, size=(nt, nt))
    return np.triu(m) + np.triu(m, 1).T


def lattice_positions(frac, box):
    """Positions x = (u / 2^32) L for integer u = floor(frac 2^32): the
    2^-32 L lattice on which the engine stores coordinates, so an input drawn
    here reaches both the oracle and the engine without rounding."""
    u = np.floor(np.asarray(frac, dtype=np.float64) * 4294967296.0)
    u = np.minimum(u, 4294967295.0)
    return u / 4294967296.0 * np.asarray(box, dtype=np.float64)


def bulk(name, N, seed, charged_frac, a_types, A, rc, beta, grid, order=5, lB=1.0,
         dt=0.02, gamma=1.0, kT=1.0, kmax=0.0, box=None, on_lattice=True):
    rng = np.random.default_rng(seed)
    L = (N / DENSITY) ** (1.0 / 3.0) if box is None else None
    box = (L, L, L) if box is None else tuple(float(b) for b in box)
    frac = rng.uniform(0.0, 1.0, size=(N, 3))
    pos = lattice_positions(frac, box) if on_lattice else frac * np.asarray(box)
    nt = len(a_types)
    typ = _species(rng, N, nt)
    z = _charges(rng, N, charged_frac)
    a = np.asarray(a_types, dtype=np.float64)
    mass = np.ones(nt)
    vel = _velocities(rng, N, mass[typ], kT)
    return Workload(name, pos, typ, z, vel, box, rc, beta, lB, np.asarray(A, dtype=np.float64),
                    a.copy(), a.copy(), tuple(grid), order, dt, gamma, kT, mass, seed, kmax)


def config1(on_lattice=True):
    """Plain method, FP64: N = 1536 at rho = 2.5, 10% +1 / 10% -1, a = 0.5,
    A = 25, lB = 1, rc = 3, beta = 1.0, exact k-sum |k| <= 8 (wavevector),
    SPME 32^3 order 5 on the GPU, velocity Verlet at dt = 0.02."""
    return bulk("bulk_N1536_fp64", 1536, 1, 0.2, [0.5], [[25.0]], 3.0, 1.0, (32, 32, 32),
                gamma=0.0, kmax=8.0, on_lattice=on_lattice)


def config2(on_lattice=True):
    """Bulk electrolyte: N = 32768, 20% charged, species a = 0.4 / 0.6 with
    A = {20, 25, 30}, rc = 3, beta = 1.1, SPME 64^3 order 5, BAOAB kT = 1,
    gamma = 1, dt = 0.02."""
    A = [[20.0, 25.0], [25.0, 30.0]]
    return bulk("bulk_N32768_mixed", 32768, 2, 0.2, [0.4, 0.6], A, 3.0, 1.1, (64, 64, 64),
                on_lattice=on_lattice)


def config3():
    """The polyelectrolyte-slab workload's composition and mesh as a periodic
    bulk box (the slab systems themselves, with bonds, electrodes and image
    charges, are slab_system and paper_slab): N = 200,000 in 40 x 40 x 50 (rho = 2.5),
    50,000 beads at +1 (the charged chain monomers) and 50,000 at -1 (the
    counterions), the rest neutral; one species a = sigma = 0.5, A = 25,
    rc = 3, beta = 1.1, SPME 96 x 96 x 128 order 5."""
    return bulk("bulk_N200000_slab_shape", 200000, 3, 0.5, [0.5], [[25.0]], 3.0, 1.1, (96, 96, 128),
                box=(40.0, 40.0, 50.0))


def slab_system(nx=16, ny=18, h=8.0, chain_len=20, x_p=0.1, seed=21, rc=2.5, beta=1.2, grid=(24, 24, 64),
                order=5, gap_factor=3.0, lB=1.0, A=25.0, dt=0.02, gamma=1.0, kT=1.0, name=None, metal=False,
                on_lattice=True):
    """The nonmetal-electrode slab of the polyelectrolyte adsorption study,
    at a chosen size.  Electrodes: two planes of fixed beads (type 1, half
    the electrolyte radius, infinite mass, neutral) on a triangular lattice
    of spacing 0.5 (nx sites per row, ny rows: Lx = 0.5 nx, Ly = 0.5 ny
    sqrt(3)/2; the paper's 25 x 25.11 is nx = 50, ny = 58), at z = 0.5 and
    z = h + 0.5.  Electrolyte (type 0, a = sigma = 0.5) at rho = 2.5 between
    them: polyanion chains of chain_len monomers at -1 and as many +1
    counterions (each an ion fraction x_p), the rest neutral solvent; chains
    are random walks of step 0.8 kept inside the slab.  The box is
    gap_factor h long in z (tripled for the slab correction).  Bonds k = 100,
    b = 0.8 join consecutive monomers (extra["bonds"], concatenated indices).

    metal=True: the perfectly conducting electrodes of the same study,
    by the method of image charges: electrode planes at z = 0 and z = H =
    h + 1, the electrolyte between them, the box 2 H long in z, and after
    the real beads one image bead per charged bead (type 2: infinite mass,
    no excluded volume, the opposite charge) at the reflection (x, y, -z)
    on the fixed-point lattice (extra["images"]: (image, source) pairs).

    on_lattice=False leaves the positions where they were drawn (the images
    then at the exact reflections of their sources)."""
    rng = np.random.default_rng(seed)
    sp = 0.5
    Lx, Ly = sp * nx, sp * ny * math.sqrt(3.0) / 2.0
    H = h + 1.0
    Lz = 2.0 * H if metal else gap_factor * H
    box = (Lx, Ly, Lz)
    z_el = (0.0, H) if metal else (0.5, h + 0.5)
    # electrode lattices
    ex, ey = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    ex = (ex + 0.5 * (ey % 2)) * sp
    ey = ey * sp * math.sqrt(3.0) / 2.0
    plane = np.c_[ex.ravel(), ey.ravel()]
    elec = np.vstack([np.c_[plane, np.full(len(plane), z_el[0])], np.c_[plane, np.full(len(plane), z_el[1])]])
    # electrolyte
    zlo, zhi = z_el[0] + 0.3, z_el[1] - 0.3
    n_e = int(round(DENSITY * Lx * Ly * h))
    n_chain = max(1, int(round(x_p * n_e / chain_len)))
    n_mono = n_chain * chain_len
    n_ci = n_mono
    n_sol = n_e - n_mono - n_ci
    assert n_sol >= 0, "ion fraction too high for this slab"
    mono = np.empty((n_mono, 3))
    for c in range(n_chain):
        x = np.array([rng.uniform(0, Lx), rng.uniform(0, Ly), rng.uniform(zlo, zhi)])
        for m in range(chain_len):
            if m:
                d = rng.standard_normal(3)
                x = x + 0.8 * d / np.linalg.norm(d)
                if x[2] < zlo:
                    x[2] = 2 * zlo - x[2]
                if x[2] > zhi:
                    x[2] = 2 * zhi - x[2]
            mono[c * chain_len + m] = x
    free = np.c_[rng.uniform(0, Lx, n_ci + n_sol), rng.uniform(0, Ly, n_ci + n_sol),
                 rng.uniform(zlo, zhi, n_ci + n_sol)]
    pos = np.vstack([mono, free, elec])
    pos[:, 0] %= Lx
    pos[:, 1] %= Ly
    if on_lattice:
        pos = lattice_positions(pos / np.asarray(box), box)
    N = len(pos)
    typ = np.zeros(N, dtype=np.int32)
    typ[n_mono + n_ci + n_sol:] = 1
    z = np.zeros(N, dtype=np.int32)
    z[:n_mono] = -1
    z[n_mono:n_mono + n_ci] = 1
    mass = np.array([1.0, np.inf])
    a = np.array([0.5, 0.25])
    Am = np.full((2, 2), float(A))
    images = np.zeros((0, 2), dtype=np.int32)
    if metal:
        src = np.nonzero(z)[0]
        if on_lattice:
            u = np.round(pos[src] / np.asarray(box) * 4294967296.0)
            u[:, 2] = np.mod(4294967296.0 - u[:, 2], 4294967296.0)
            ipos = u / 4294967296.0 * np.asarray(box)
        else:
            ipos = pos[src].copy()
            ipos[:, 2] = np.mod(-ipos[:, 2], box[2])
        images = np.c_[np.arange(N, N + len(src)), src].astype(np.int32)
        pos = np.vstack([pos, ipos])
        typ = np.r_[typ, np.full(len(src), 2)].astype(np.int32)
        z = np.r_[z, -z[src]].astype(np.int32)
        N = len(pos)
        mass = np.array([1.0, np.inf, np.inf])
        a = np.array([0.5, 0.25, 0.5])
        Am = np.zeros((3, 3))
        Am[:2, :2] = float(A)
    vel = np.zeros((N, 3))
    mob = typ == 0
    vel[mob] = _velocities(rng, int(mob.sum()), np.ones(int(mob.sum())), kT)
    bonds = np.array([[c * chain_len + m, c * chain_len + m + 1] for c in range(n_chain) for m in range(chain_len - 1)],
                     dtype=np.int32).reshape(-1, 2)
    kind = "metal" if metal else "slab"
    return Workload(name or f"{kind}_N{N}", pos, typ, z, vel, box, rc, beta, lB, Am, a.copy(), a.copy(),
                    tuple(grid), order, dt, gamma, kT, mass, seed,
                    extra=dict(bonds=bonds, bond_k=100.0, bond_b=0.8, slab=not metal, fixed_type=1,
                               images=images))


def paper_slab(metal=False, x_p=0.05, seed=6):
    """The adsorption study's system at its size: 96,000 electrolyte beads
    in a 25 x 25.11 x 61.16 slab between electrode lattices of 50 x 58 sites,
    chains of 60 monomers at ion fraction x_p; the box tripled along z for
    the slab correction (nonmetal) or doubled with image charges (metal).
    rc = 3, beta = 1.1 as for the bulk electrolyte; mesh spacing about 0.4
    (64 x 64 x 432, or 64 x 64 x 288 for the doubled box)."""
    return slab_system(nx=50, ny=58, h=61.16, chain_len=60, x_p=x_p, seed=seed, rc=3.0, beta=1.1,
                       grid=(64, 64, 288) if metal else (64, 64, 432), metal=metal,
                       name="slab_metal_images" if metal else "slab_nonmetal_corrected")


def polyelectrolyte_slab(metal=False, n_chains=2000, chain_len=50, n_counter=50000, n_solvent=50000, nx=80, ny=92,
                         seed=3, rc=3.0, beta=1.1, grid_xy=96, order=5, on_lattice=True):
    """The polyelectrolyte slab of the adsorption study at the size of the
    200,000-bead configuration: n_chains linear chains of chain_len beads in
    which every other bead (the first, third, ...) carries +1, joined by
    harmonic bonds (k = 100, b = 0.8); n_counter counterions at -1 and
    n_solvent neutral beads; all electrolyte beads a = sigma = 0.5 with
    A = 25 (one species, as in the study).  The electrolyte fills
    Lx x Ly x h at rho = 2.5 between two electrode lattices of fixed beads
    (type 1, a = sigma = 0.25, neutral, triangular lattice of spacing 0.5:
    nx sites per row, ny rows, Lx = 0.5 nx = 40, Ly = 0.5 ny sqrt(3)/2 =
    39.84), h = N_e / (2.5 Lx Ly).  Chains are random walks of step 0.8
    inside the slab.  Nonmetal electrodes: planes at z = 0.5 and h + 0.5,
    box tripled along z (H = h + 1, Lz = 3H) for the slab correction, mesh
    grid_xy^2 x 384 (spacing about 0.4).  Metal electrodes: planes at z = 0
    and H, box 2H long with one image bead (type 2: infinite mass, no
    excluded volume, opposite charge) per charged bead at its reflection
    (x, y, -z), mesh grid_xy^2 x 256.  rc = 3, beta = 1.1, order 5."""
    rng = np.random.default_rng(seed)
    sp = 0.5
    Lx, Ly = sp * nx, sp * ny * math.sqrt(3.0) / 2.0
    n_mono = n_chains * chain_len
    n_e = n_mono + n_counter + n_solvent
    h = n_e / (DENSITY * Lx * Ly)
    H = h + 1.0
    Lz = 2.0 * H if metal else 3.0 * H
    box = (Lx, Ly, Lz)
    z_el = (0.0, H) if metal else (0.5, h + 0.5)
    ex, ey = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    ex = (ex + 0.5 * (ey % 2)) * sp
    ey = ey * sp * math.sqrt(3.0) / 2.0
    plane = np.c_[ex.ravel(), ey.ravel()]
    elec = np.vstack([np.c_[plane, np.full(len(plane), z_el[0])], np.c_[plane, np.full(len(plane), z_el[1])]])
    zlo, zhi = z_el[0] + 0.3, z_el[1] - 0.3
    # chains: random walks of step 0.8 reflected at the slab faces
    start = np.c_[rng.uniform(0, Lx, n_chains), rng.uniform(0, Ly, n_chains), rng.uniform(zlo, zhi, n_chains)]
    steps = rng.standard_normal((n_chains, chain_len - 1, 3))
    steps *= 0.8 / np.linalg.norm(steps, axis=2, keepdims=True)
    mono = np.empty((n_chains, chain_len, 3))
    mono[:, 0] = start
    for m in range(1, chain_len):
        x = mono[:, m - 1] + steps[:, m - 1]
        zz = x[:, 2]
        zz = np.where(zz < zlo, 2 * zlo - zz, zz)
        zz = np.where(zz > zhi, 2 * zhi - zz, zz)
        x[:, 2] = zz
        mono[:, m] = x
    mono = mono.reshape(-1, 3)
    free = np.c_[rng.uniform(0, Lx, n_counter + n_solvent), rng.uniform(0, Ly, n_counter + n_solvent),
                 rng.uniform(zlo, zhi, n_counter + n_solvent)]
    pos = np.vstack([mono, free, elec])
    pos[:, 0] %= Lx
    pos[:, 1] %= Ly
    if on_lattice:
        pos = lattice_positions(pos / np.asarray(box), box)
    N = len(pos)
    typ = np.zeros(N, dtype=np.int32)
    typ[n_e:] = 1
    z = np.zeros(N, dtype=np.int32)
    z[:n_mono][np.arange(n_mono) % chain_len % 2 == 0] = 1
    z[n_mono:n_mono + n_counter] = -1
    assert z.sum() == 0, "chain charges and counterions must balance"
    mass = np.array([1.0, np.inf])
    a = np.array([0.5, 0.25])
    Am = np.full((2, 2), 25.0)
    images = np.zeros((0, 2), dtype=np.int32)
    if metal:
        src = np.nonzero(z)[0]
        if on_lattice:
            u = np.round(pos[src] / np.asarray(box) * 4294967296.0)
            u[:, 2] = np.mod(4294967296.0 - u[:, 2], 4294967296.0)
            ipos = u / 4294967296.0 * np.asarray(box)
        else:
            ipos = pos[src].copy()
            ipos[:, 2] = np.mod(-ipos[:, 2], box[2])
        images = np.c_[np.arange(N, N + len(src)), src].astype(np.int32)
        pos = np.vstack([pos, ipos])
        typ = np.r_[typ, np.full(len(src), 2)].astype(np.int32)
        z = np.r_[z, -z[src]].astype(np.int32)
        N = len(pos)
        mass = np.array([1.0, np.inf, np.inf])
        a = np.array([0.5, 0.25, 0.5])
        Am = np.zeros((3, 3))
        Am[:2, :2] = 25.0
    vel = np.zeros((N, 3))
    mob = typ == 0
    vel[mob] = _velocities(rng, int(mob.sum()), np.ones(int(mob.sum())), 1.0)
    c = np.arange(n_chains)[:, None] * chain_len + np.arange(chain_len - 1)[None, :]
    bonds = np.c_[c.ravel(), c.ravel() + 1].astype(np.int32)
    grid = (grid_xy, grid_xy, 256 if metal else 384)
    return Workload("polyelectrolyte_slab_metal" if metal else "polyelectrolyte_slab_nonmetal", pos, typ, z, vel, box,
                    rc, beta, 1.0, Am, a.copy(), a.copy(), grid, order, 0.02, 1.0, 1.0, mass, seed,
                    extra=dict(bonds=bonds, bond_k=100.0, bond_b=0.8, slab=not metal, fixed_type=1, images=images,
                               n_electrolyte=n_e))


def config4(on_lattice=True):
    """Large bulk: N = 2^21, three species a = 0.3/0.5/0.7, A ~ U(15, 35)
    symmetric (seeded), 15% charged, rc = 2.5, beta = 1.2, SPME 256^3."""
    rng = np.random.default_rng(1004)
    A = _sym_uniform(rng, 3, 15.0, 35.0)
    return bulk("bulk_N2097152", 2097152, 4, 0.15, [0.3, 0.5, 0.7], A, 2.5, 1.2, (256, 256, 256),
                on_lattice=on_lattice)


def config5(n_replicas=256, seed=5, on_lattice=True):
    """Batched replicas: N_r log-uniform in [500, 8000], 2 species with
    a ~ U(0.3, 0.7), A ~ U(15, 35) symmetric, charged fraction U(0.1, 0.3),
    rc = 2.5, beta = 1.2, grid = smallest 2^a 3^b >= L/0.37, order 5."""
    rng = np.random.default_rng(seed)
    reps = []
    for r in range(n_replicas):
        n = int(round(math.exp(rng.uniform(math.log(500), math.log(8000)))))
        a = rng.uniform(0.3, 0.7, size=2)
        A = _sym_uniform(rng, 2, 15.0, 35.0)
        f = rng.uniform(0.1, 0.3)
        L = (n / DENSITY) ** (1.0 / 3.0)
        K = smooth_size(L / 0.37)
        reps.append(bulk(f"replica{r}", n, seed * 100003 + r, f, a, A, 2.5, 1.2, (K, K, K),
                         on_lattice=on_lattice))
    return reps


def small_bulk(N=300, seed=11, charged_frac=0.3, a_types=(0.4, 0.6), rc=2.0, beta=1.1,
               grid=(16, 16, 16), A=None, box=None, order=5, on_lattice=True):
    """A few-hundred-bead box for fast parity cases (several tiles, ragged)."""
    nt = len(a_types)
    if A is None:
        A = _sym_uniform(np.random.default_rng(seed + 7), nt, 15.0, 35.0)
    return bulk(f"small_N{N}", N, seed, charged_frac, list(a_types), A, rc, beta, grid, order=order,
                box=box, on_lattice=on_lattice)


def rock_salt(n_cells: int, r0: float = 1.0):
    """NaCl lattice: n_cells^3 conventional cubes of side 2 r0, 8 ions each,
    alternating +1/-1 on a simple cubic lattice of spacing r0."""
    n = 2 * n_cells
    g = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1).reshape(-1, 3)
    z = np.where(g.sum(1) % 2 == 0, 1, -1).astype(np.int32)
    return g.astype(np.float64) * r0, z, (n * r0,) * 3


def cesium_chloride(n_cells: int, a0: float = 1.0):
    """CsCl lattice: n_cells^3 cubes of side a0, +1 at corners, -1 at centres."""
    g = np.stack(np.meshgrid(np.arange(n_cells), np.arange(n_cells), np.arange(n_cells), indexing="ij"),
                 -1).reshape(-1, 3).astype(np.float64) * a0
    pos = np.concatenate([g, g + 0.5 * a0])
    z = np.concatenate([np.ones(len(g), np.int32), -np.ones(len(g), np.int32)])
    return pos, z, (n_cells * a0,) * 3
