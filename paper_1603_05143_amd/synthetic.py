"""Seeded synthetic atomic configurations.

This module only builds inputs: lattices, grains, noise, species and
orientations.  It holds none of the classification arithmetic, so both the
FP64 reference implementation (``oracle/``) and the HIP path can be fed from
it without sharing any of the method's code.

Every generator takes an explicit ``seed`` and uses numpy's PCG64, so a
configuration is a pure function of its arguments.  Positions are float64,
shape ``(n, 3)``, wrapped into ``[0, L)`` for periodic boxes.  Species are
int8 (0 = majority "A" atom, 1 = minority "B" atom).

The workloads stand in for the paper's benchmark systems (a quenched
Cu-precipitate-in-Fe sample and a 2.8 M-atom Cu3Pt polycrystal, Sec. 5),
which are not available: a ~0.92 M-atom periodic polycrystal of FCC, BCC
and HCP grains, a ~4 M-atom box of ordered-alloy slabs with species, a
stream of polycrystal frames of uneven size, and small perfect or noisy
crystals and clusters for tests.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 160305143

# ----------------------------------------------------------------------------
# lattice motifs (fractional coordinates within the conventional cell)
# ----------------------------------------------------------------------------
FCC_MOTIF = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
BCC_MOTIF = np.array([[0, 0, 0], [0.5, 0.5, 0.5]])
SC_MOTIF = np.array([[0.0, 0.0, 0.0]])


@dataclass
class Frame:
    """One synthetic frame: positions, optional species and box lengths."""
    positions: np.ndarray            # (n, 3) float64
    box: np.ndarray                  # (3,) float64; 0 = open along that axis
    species: np.ndarray | None = None  # (n,) int8
    labels: dict = field(default_factory=dict)  # generator-side truth (grain id, phase, ...)

    @property
    def n(self) -> int:
        return int(self.positions.shape[0])


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_rotations(rng: np.random.Generator, m: int) -> np.ndarray:
    """m rotation matrices uniform on SO(3) (Shoemake's subgroup algorithm)."""
    u1, u2, u3 = rng.random(m), rng.random(m), rng.random(m)
    a, b = np.sqrt(1 - u1), np.sqrt(u1)
    q = np.stack([a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2),
                  b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)], axis=1)
    return quat_to_matrix(q)


def quat_to_matrix(q: np.ndarray) -> np.ndarray:
    """Rotation matrices of unit quaternions (w, x, y, z); shape (..., 3, 3)."""
    q = np.asarray(q, dtype=np.float64)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    r = np.empty(q.shape[:-1] + (3, 3))
    r[..., 0, 0] = 1 - 2 * (y * y + z * z)
    r[..., 0, 1] = 2 * (x * y - w * z)
    r[..., 0, 2] = 2 * (x * z + w * y)
    r[..., 1, 0] = 2 * (x * y + w * z)
    r[..., 1, 1] = 1 - 2 * (x * x + z * z)
    r[..., 1, 2] = 2 * (y * z - w * x)
    r[..., 2, 0] = 2 * (x * z - w * y)
    r[..., 2, 1] = 2 * (y * z + w * x)
    r[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def lattice_block(motif: np.ndarray, cell: np.ndarray, reps) -> np.ndarray:
    """Sites of a block of ``reps`` conventional cells (cell = 3x3 rows)."""
    nx, ny, nz = reps
    ijk = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz),
                               indexing="ij"), axis=-1).reshape(-1, 1, 3)
    frac = (ijk + motif[None, :, :]).reshape(-1, 3)
    return frac @ cell


def hcp_cell(a: float, c_over_a: float):
    """Orthohexagonal HCP cell (4 atoms) with c along z."""
    c = a * c_over_a
    cell = np.array([[a, 0, 0], [0, a * math.sqrt(3), 0], [0, 0, c]])
    motif = np.array([[0, 0, 0], [0.5, 0.5, 0],
                      [0.5, 1.0 / 6.0, 0.5], [0.0, 2.0 / 3.0, 0.5]])
    return motif, cell


def wrap(pos: np.ndarray, box: np.ndarray) -> np.ndarray:
    out = pos.copy()
    for d in range(3):
        if box[d] > 0:
            out[:, d] = np.mod(out[:, d], box[d])
            out[:, d][out[:, d] >= box[d]] = 0.0
    return out


# ----------------------------------------------------------------------------
# perfect crystals (test inputs)
# ----------------------------------------------------------------------------
def perfect_crystal(kind: str, reps=(4, 4, 4), a: float = 3.615,
                    c_over_a: float = math.sqrt(8.0 / 3.0)) -> Frame:
    """Perfect periodic crystal: 'fcc', 'bcc', 'sc', 'hcp', 'L12', 'L10', 'B2'."""
    kind_l = kind.lower()
    species = None
    if kind_l in ("fcc", "l12", "l10", "a1"):
        cell = np.eye(3) * a
        pos = lattice_block(FCC_MOTIF, cell, reps)
        if kind_l == "l12":
            species = np.tile(np.array([1, 0, 0, 0], np.int8), int(np.prod(reps)))
        elif kind_l == "l10":
            species = np.tile(np.array([0, 0, 1, 1], np.int8), int(np.prod(reps)))
        elif kind_l == "a1":
            species = np.zeros(len(pos), np.int8)
        box = np.array(reps, dtype=np.float64) * a
    elif kind_l in ("bcc", "b2", "a2"):
        cell = np.eye(3) * a
        pos = lattice_block(BCC_MOTIF, cell, reps)
        if kind_l == "b2":
            species = np.tile(np.array([0, 1], np.int8), int(np.prod(reps)))
        elif kind_l == "a2":
            species = np.zeros(len(pos), np.int8)
        box = np.array(reps, dtype=np.float64) * a
    elif kind_l == "sc":
        cell = np.eye(3) * a
        pos = lattice_block(SC_MOTIF, cell, reps)
        box = np.array(reps, dtype=np.float64) * a
    elif kind_l == "hcp":
        motif, cell = hcp_cell(a, c_over_a)
        pos = lattice_block(motif, cell, reps)
        box = np.array([reps[0] * cell[0, 0], reps[1] * cell[1, 1], reps[2] * cell[2, 2]])
    else:
        raise ValueError(kind)
    return Frame(positions=wrap(pos, box), box=box, species=species,
                 labels={"kind": kind_l})


def mackay_icosahedron(shells: int, nn: float = 2.55) -> np.ndarray:
    """Atoms of a Mackay icosahedron with ``shells`` shells around a centre.

    shells=1 gives 13 atoms, 2 gives 55, 3 gives 147.  ``nn`` is the radial
    distance from the centre to the first shell.
    """
    phi = (1 + math.sqrt(5)) / 2
    v = []
    for s1 in (1, -1):
        for s2 in (phi, -phi):
            v += [(0, s1, s2), (s1, s2, 0), (s2, 0, s1)]
    verts = np.array(v, dtype=np.float64)
    verts /= np.linalg.norm(verts[0])
    # edges and faces of the icosahedron
    d = np.linalg.norm(verts[:, None] - verts[None], axis=-1)
    emin = d[d > 1e-9].min()
    adj = np.abs(d - emin) < 1e-6
    faces = [(i, j, k) for i in range(12) for j in range(i + 1, 12) for k in range(j + 1, 12)
             if adj[i, j] and adj[j, k] and adj[i, k]]
    edges = [(i, j) for i in range(12) for j in range(i + 1, 12) if adj[i, j]]
    pts = [np.zeros(3)]
    for s in range(1, shells + 1):
        vs = verts * s
        pts += list(vs)
        for i, j in edges:
            for t in range(1, s):
                pts.append(vs[i] + (vs[j] - vs[i]) * t / s)
        for i, j, k in faces:
            for a_ in range(1, s):
                for b_ in range(1, s - a_):
                    c_ = s - a_ - b_
                    pts.append((vs[i] * a_ + vs[j] * b_ + vs[k] * c_) / s)
    return np.array(pts) * nn


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------
def config0(seed: int | None = None) -> Frame:
    """Periodic 4x4x4 FCC supercell, a = 3.615 A, Gaussian noise 0.05 A (256 atoms)."""
    seed = BASE_SEED + 0 if seed is None else seed
    rng = rng_for(seed)
    f = perfect_crystal("fcc", (4, 4, 4), a=3.615)
    pos = f.positions + rng.normal(0.0, 0.05, size=f.positions.shape)
    return Frame(positions=wrap(pos, f.box), box=f.box, labels={"config": 0})


# phase -> (motif, lattice constant, c/a, species of the motif sites or None
# for a pure element, fraction of B atoms drawn at random or None)
_PHASES = {
    "fcc": (FCC_MOTIF, 3.615, None, None, None),
    "bcc": (BCC_MOTIF, 2.87, None, None, None),
    "hcp": (None, 2.51, 1.633, None, None),
    # ordered alloys of the alloy-slab workload (species 1 = B)
    "l12": (FCC_MOTIF, 3.57, None, np.array([1, 0, 0, 0], np.int8), None),
    "l10": (FCC_MOTIF, 3.85, 0.97, np.array([0, 0, 1, 1], np.int8), None),
    "b2": (BCC_MOTIF, 2.88, None, np.array([0, 1], np.int8), None),
    "a1": (FCC_MOTIF, 3.57, None, None, 0.25),
}


def _phase_cell(phase: str):
    motif, a, coa, _, _ = _PHASES[phase]
    if phase == "hcp":
        return hcp_cell(a, coa)
    cell = np.eye(3) * a
    if coa is not None:
        cell[2, 2] = a * coa
    return motif, cell


def _min_image(d: np.ndarray, box: np.ndarray) -> np.ndarray:
    out = d.copy()
    for k in range(3):
        if box[k] > 0:
            out[..., k] -= box[k] * np.round(out[..., k] / box[k])
    return out


def polycrystal(L: float = 220.0, n_grains: int = 16, sigma: float = 0.10,
                seed: int | None = None, phases=("fcc", "bcc", "hcp"),
                min_dist: float = 1.2) -> Frame:
    """Periodic Voronoi polycrystal (the ~1 M-atom workload at L = 220 A).

    Grain centres are uniform in the cubic box, orientations uniform on SO(3)
    and each grain's lattice is drawn uniformly from ``phases``.  A site
    belongs to the grain whose centre is nearest under the minimum image.
    Of each cross-grain pair closer than ``min_dist`` the atom with the
    higher (grain, index) is deleted.  Gaussian noise ``sigma`` is added last.
    If any phase is an alloy (``l12``, ``l10``, ``b2``, ``a1``) the frame
    carries species (0 on the sites of pure phases).
    """
    from scipy.spatial import cKDTree

    seed = BASE_SEED + 1 if seed is None else seed
    rng = rng_for(seed)
    box = np.array([L, L, L], dtype=np.float64)
    centres = rng.random((n_grains, 3)) * L
    rots = random_rotations(rng, n_grains)
    phase_idx = rng.integers(0, len(phases), size=n_grains)
    ctree = cKDTree(centres, boxsize=L)

    # radius that covers each Voronoi cell, from a coarse grid sample
    g = max(8, int(L / 4.0))
    grid = (np.stack(np.meshgrid(*[np.arange(g)] * 3, indexing="ij"), -1).reshape(-1, 3) + 0.5) * (L / g)
    dist, owner = ctree.query(grid)
    cover = np.zeros(n_grains)
    np.maximum.at(cover, owner, dist)
    cover += math.sqrt(3) * L / g + 4.0

    with_species = any(_PHASES[ph][3] is not None or _PHASES[ph][4] is not None for ph in phases)
    all_pos, all_grain, all_spc = [], [], []
    for gi in range(n_grains):
        motif, cell = _phase_cell(phases[phase_idx[gi]])
        r = cover[gi]
        # integer range of cells whose sites can reach within r of the centre
        reach = np.ceil(r / np.min(np.abs(np.diag(cell)))) + 1
        rng_cells = np.arange(-reach, reach + 1)
        ijk = np.stack(np.meshgrid(rng_cells, rng_cells, rng_cells, indexing="ij"), -1).reshape(-1, 3)
        sites = ((ijk[:, None, :] + motif[None]) .reshape(-1, 3)) @ cell
        inside = np.einsum("ij,ij->i", sites, sites) <= r * r
        sites = sites[inside]
        d = sites @ rots[gi].T
        p = wrap(d + centres[gi], box)
        _, own = ctree.query(p)
        # each point of space once: the site's offset from the centre must be
        # its own minimum image (matters when a grain spans most of the box)
        keep = (own == gi) & np.all(np.abs(d) < 0.5 * L, axis=1)
        all_pos.append(p[keep])
        all_grain.append(np.full(int(keep.sum()), gi, dtype=np.int32))
        if with_species:
            _, _, _, smotif, bfrac = _PHASES[phases[phase_idx[gi]]]
            if smotif is not None:
                spc = np.tile(smotif, len(ijk))[inside][keep]
            elif bfrac is not None:
                spc = (rng.random(int(keep.sum())) < bfrac).astype(np.int8)
            else:
                spc = np.zeros(int(keep.sum()), np.int8)
            all_spc.append(spc)
    pos = np.concatenate(all_pos)
    grain = np.concatenate(all_grain)
    species = np.concatenate(all_spc) if with_species else None

    # delete the higher (grain, index) atom of each too-close pair: pairs
    # across grain boundaries, and across the periodic seam of a grain that
    # meets its own image (lattice neighbours are never this close)
    tree = cKDTree(pos, boxsize=L)
    pairs = tree.query_pairs(min_dist, output_type="ndarray")
    if len(pairs):
        a_, b_ = pairs[:, 0], pairs[:, 1]
        key_a = grain[a_].astype(np.int64) * (1 << 32) + a_
        key_b = grain[b_].astype(np.int64) * (1 << 32) + b_
        victim = np.where(key_a > key_b, a_, b_)
        alive = np.ones(len(pos), bool)
        alive[victim] = False
        pos, grain = pos[alive], grain[alive]
        if species is not None:
            species = species[alive]

    pos = pos + rng.normal(0.0, sigma, size=pos.shape)
    return Frame(positions=wrap(pos, box), box=box, species=species,
                 labels={"grain": grain, "phases": [phases[i] for i in phase_idx],
                         "rotations": rots, "centres": centres})


def alloy_slabs(n_cells: int = 102, a_l12: float = 3.57, a_l10: float = 3.85,
                coa_l10: float = 0.97, a_b2: float = 2.88, antisite: float = 0.02,
                vacancy: float = 0.01, sigma: float = 0.25, seed: int | None = None) -> Frame:
    """Four x-slabs: L1_2 A3B, L1_0 AB (c along z), B2 AB and random FCC A3B.

    The box is cubic with L = n_cells * a_l12 (364.1 A at the default, ~4 M
    atoms).  Each slab's lattice constants are rescaled (<1 %) so that its
    cell counts are commensurate with L along y and z; along x the slabs meet
    at planar interfaces.  ``antisite`` of the atoms of each slab swap species
    with a random partner of the other species in the same slab,
    ``vacancy`` of the sites are removed and Gaussian noise ``sigma`` is added.
    """
    seed = BASE_SEED + 2 if seed is None else seed
    rng = rng_for(seed)
    L = n_cells * a_l12
    box = np.array([L, L, L])
    w = L / 4.0
    chunks_p, chunks_s, chunks_slab = [], [], []

    def fill(slab, motif, species_motif, ax, ay, az):
        nx = max(1, int(round(w / ax)))
        ny = max(1, int(round(L / ay)))
        nz = max(1, int(round(L / az)))
        cell = np.diag([w / nx, L / ny, L / nz])
        p = lattice_block(motif, cell, (nx, ny, nz)) + np.array([slab * w, 0, 0])
        s = np.tile(species_motif, nx * ny * nz).astype(np.int8)
        return p, s

    # slab 0: L1_2 A3B -- B on the cube corners
    p, s = fill(0, FCC_MOTIF, np.array([1, 0, 0, 0]), a_l12, a_l12, a_l12)
    chunks_p.append(p); chunks_s.append(s); chunks_slab.append(np.full(len(p), 0, np.int8))
    # slab 1: L1_0 AB -- alternating (001) planes, c along z
    p, s = fill(1, FCC_MOTIF, np.array([0, 0, 1, 1]), a_l10, a_l10, a_l10 * coa_l10)
    chunks_p.append(p); chunks_s.append(s); chunks_slab.append(np.full(len(p), 1, np.int8))
    # slab 2: B2 AB
    p, s = fill(2, BCC_MOTIF, np.array([0, 1]), a_b2, a_b2, a_b2)
    chunks_p.append(p); chunks_s.append(s); chunks_slab.append(np.full(len(p), 2, np.int8))
    # slab 3: disordered FCC, 25 % B
    p, _ = fill(3, FCC_MOTIF, np.array([0, 0, 0, 0]), a_l12, a_l12, a_l12)
    s = (rng.random(len(p)) < 0.25).astype(np.int8)
    chunks_p.append(p); chunks_s.append(s); chunks_slab.append(np.full(len(p), 3, np.int8))

    pos = np.concatenate(chunks_p)
    spc = np.concatenate(chunks_s)
    slab = np.concatenate(chunks_slab)
    # antisite swaps within each slab
    for sl in range(4):
        idx = np.nonzero(slab == sl)[0]
        m = int(antisite * len(idx) / 2)
        a_idx = idx[spc[idx] == 0]
        b_idx = idx[spc[idx] == 1]
        m = min(m, len(a_idx), len(b_idx))
        if m > 0:
            pa = rng.choice(a_idx, m, replace=False)
            pb = rng.choice(b_idx, m, replace=False)
            spc[pa], spc[pb] = 1, 0
    keep = rng.random(len(pos)) >= vacancy
    pos, spc, slab = pos[keep], spc[keep], slab[keep]
    pos = pos + rng.normal(0.0, sigma, size=pos.shape)
    return Frame(positions=wrap(pos, box), box=box, species=spc, labels={"slab": slab})


SERVING_PHASES = ("fcc", "bcc", "hcp", "l12", "l10", "b2", "a1")


def serving_frame(n: int, seed: int, sigma: float | None = None) -> Frame:
    """One frame of the serving stream: a small periodic polycrystal of ~n atoms.

    Grain lattices are drawn from the phases of the polycrystal and of the
    alloy-slab workloads (FCC, BCC, HCP, L1_2, L1_0, B2, random FCC), so
    frames carry species; the grain count is max(1, n / 60000) and the cubic
    box is sized for ~n atoms at the mean density of the phases (at least
    22 A).  ``sigma`` defaults to U[0.02, 0.3].
    """
    rng = rng_for(seed)
    if sigma is None:
        sigma = float(rng.uniform(0.02, 0.3))
    rho = 0.0862
    L = max(22.0, (n / rho) ** (1.0 / 3.0))
    n_grains = max(1, int(n // 60000))
    f = polycrystal(L=L, n_grains=n_grains, sigma=sigma, seed=int(rng.integers(1 << 31)),
                    phases=SERVING_PHASES)
    f.labels["sigma"] = sigma
    return f


def serving_stream(n_frames: int = 2000, lo: float = 1e3, hi: float = 2e6,
                   seed: int | None = None):
    """Frame sizes (log-uniform in [lo, hi]) and per-frame seeds of the stream."""
    seed = BASE_SEED + 3 if seed is None else seed
    rng = rng_for(seed)
    sizes = np.exp(rng.uniform(math.log(lo), math.log(hi), n_frames)).astype(np.int64)
    seeds = rng.integers(0, 1 << 31, n_frames)
    return sizes, seeds


def subsample_box(frame: Frame, frac: float, seed: int = 0) -> Frame:
    """Periodic sub-cube of a frame (used to make small versions of big configs)."""
    L = frame.box
    cut = L * frac ** (1.0 / 3.0)
    m = np.all(frame.positions < cut, axis=1)
    return Frame(positions=frame.positions[m].copy(), box=np.zeros(3),
                 species=None if frame.species is None else frame.species[m].copy())


def _rsa_tile(dims, dmin: float, rng: np.random.Generator,
              rounds=(0.15, 0.3, 0.6, 1.0, 2.0, 3.0, 5.0)) -> np.ndarray:
    """Random sequential adsorption in a periodic box: points arrive as
    Poisson batches of the given densities (per A^3); a point is kept iff it
    lies at least ``dmin`` from every point kept before it (arrival order is
    a uniform random priority within each batch)."""
    from scipy.spatial import cKDTree

    dims = np.asarray(dims, dtype=np.float64)
    vol = float(np.prod(dims))
    pts = np.zeros((0, 3))
    for rho in rounds:
        p = rng.random((int(rng.poisson(rho * vol)), 3)) * dims
        if len(pts):
            d, _ = cKDTree(pts, boxsize=dims).query(p, distance_upper_bound=dmin)
            p = p[~np.isfinite(d)]
        if not len(p):
            continue
        pairs = cKDTree(p, boxsize=dims).query_pairs(dmin, output_type="ndarray")
        prio = rng.random(len(p))
        alive = np.ones(len(p), bool)
        keep = np.zeros(len(p), bool)
        a_, b_ = (pairs[:, 0], pairs[:, 1]) if len(pairs) else (np.zeros(0, int), np.zeros(0, int))
        # the points kept by sequential arrival in priority order: repeatedly
        # keep every live point that arrives before all its live neighbours
        while alive.any():
            live = alive[a_] & alive[b_]
            aa, bb = a_[live], b_[live]
            first = alive.copy()
            first[np.where(prio[aa] < prio[bb], bb, aa)] = False
            keep |= first
            alive &= ~first
            alive[np.concatenate([bb[first[aa]], aa[first[bb]]])] = False
        pts = np.concatenate([pts, p[keep]])
    return pts


def mixed_frame(n_cells: int = 256, a_bcc: float = 2.87, vacancy: float = 0.01, n_ico: int = 200,
                ico_nn: float = 2.55, n_sc: int = 10, a_sc: float = 2.6, sc_edge: float = 40.0,
                clearance: float = 1.2, slab_frac: float = 0.15, rsa_dmin: float = 2.2,
                sigma: float = 0.15, seed: int | None = None) -> Frame:
    """The ~32 M-atom mixed frame: a periodic BCC matrix (a = 2.87 A, L =
    n_cells a, ``vacancy`` of the sites removed) holding ``n_ico`` Mackay
    icosahedra (half of 55 atoms, half of 147; first-shell radius ``ico_nn``;
    random orientations), ``n_sc`` simple-cubic cubes (a = 2.6 A, edge ~40 A,
    random orientations) and a slab of ``slab_frac`` of the volume (all y, z)
    filled by random sequential adsorption with minimum distance ``rsa_dmin``
    (liquid-like; jammed near 0.06 per A^3).  Inclusions replace the matrix
    inside their outer radius (cubes: their extent) plus ``clearance``; of
    each pair closer than ``clearance`` across a slab face the slab atom is
    removed.  The slab is tiled from one periodic adsorption block of 1/288
    of its volume.  Gaussian noise ``sigma`` is added last.  labels["kind"]:
    0 matrix, 1 icosahedron, 2 simple cubic, 3 slab.
    """
    from scipy.spatial import cKDTree

    seed = BASE_SEED + 4 if seed is None else seed
    rng = rng_for(seed)
    n, a = n_cells, a_bcc
    L = n * a
    box = np.array([L, L, L])
    w = slab_frac * L  # slab: x in [0, w)
    # inclusions: centres outside the slab, no two closer than their radii + 2 clearances
    ico_shells = np.array([2] * (n_ico // 2) + [3] * (n_ico - n_ico // 2))
    m_side = int(round(sc_edge / a_sc))  # cells per cube edge (m_side + 1 points)
    half = 0.5 * m_side * a_sc
    radii = np.concatenate([ico_shells * ico_nn, np.full(n_sc, half * math.sqrt(3.0))])
    kinds = np.concatenate([np.ones(n_ico, int), np.full(n_sc, 2)])
    order = np.argsort(-radii, kind="stable")
    centres = np.zeros((len(radii), 3))
    placed = []
    for idx in order:
        r = radii[idx] + clearance
        for _ in range(10000):
            c = np.array([w + r + rng.random() * (L - w - 2 * r), rng.random() * L, rng.random() * L])
            ok = True
            for j in placed:
                d = _min_image(c - centres[j], box)
                if np.linalg.norm(d) < r + radii[j] + 3 * clearance:
                    ok = False
                    break
            if ok:
                break
        centres[idx] = c
        placed.append(idx)
    rots = random_rotations(rng, len(radii))

    # matrix: BCC site (s, i, j, k) at a (i, j, k) + a s (1/2, 1/2, 1/2)
    keep = rng.random(2 * n * n * n) >= vacancy
    keep = keep.reshape(2, n, n, n)
    lo_cell = int(math.ceil(w / a))  # cells with x >= w: sublattice 0 from i = lo_cell
    keep[0, :lo_cell] = False
    keep[1, :int(math.ceil(w / a - 0.5))] = False
    inc_pos, inc_kind = [], []
    for idx in range(len(radii)):
        c, R = centres[idx], rots[idx]
        if kinds[idx] == 1:
            pts = mackay_icosahedron(int(ico_shells[idx]), ico_nn) @ R.T
            rad = ico_shells[idx] * ico_nn + clearance
        else:
            g = np.arange(m_side + 1) * a_sc - half
            pts = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3) @ R.T
            rad = half * math.sqrt(3.0) + clearance
        inc_pos.append(pts + c)
        inc_kind.append(np.full(len(pts), kinds[idx], np.int8))
        # matrix sites near the centre (periodic index window)
        for s in (0, 1):
            lo = np.floor((c - rad) / a - 0.5 * s).astype(int)
            hi = np.ceil((c + rad) / a - 0.5 * s).astype(int)
            ii = [np.arange(lo[d], hi[d] + 1) for d in range(3)]
            I, J, K = np.meshgrid(*ii, indexing="ij")
            sp = (np.stack([I, J, K], -1) + 0.5 * s) * a - c
            sp = _min_image(sp, box)
            if kinds[idx] == 1:
                inside = np.einsum("...d,...d->...", sp, sp) <= rad * rad
            else:
                loc = sp @ R  # cube frame
                inside = np.all(np.abs(loc) <= half + clearance, axis=-1)
            keep[s, I[inside] % n, J[inside] % n, K[inside] % n] = False
    s_idx, i_idx, j_idx, k_idx = np.nonzero(keep)
    del keep
    mat = (np.stack([i_idx, j_idx, k_idx], -1).astype(np.float64) + 0.5 * s_idx[:, None]) * a
    del s_idx, i_idx, j_idx, k_idx

    # slab: one periodic adsorption block tiled 2 x 12 x 12
    tiles = (2, 12, 12)
    tdims = np.array([w / tiles[0], L / tiles[1], L / tiles[2]])
    tile = _rsa_tile(tdims, rsa_dmin, rng)
    off = np.stack(np.meshgrid(*[np.arange(t) for t in tiles], indexing="ij"), -1).reshape(-1, 1, 3) * tdims
    slab = (tile[None] + off).reshape(-1, 3)
    # slab atoms too close to the matrix across the two slab faces
    near_m = mat[(mat[:, 0] < w + 2 * clearance) | (mat[:, 0] > L - 2 * clearance)]
    near_s = (slab[:, 0] < 2 * clearance) | (slab[:, 0] > w - 2 * clearance)
    if len(near_m) and near_s.any():
        d, _ = cKDTree(near_m, boxsize=L).query(wrap(slab[near_s], box), distance_upper_bound=clearance)
        drop = np.zeros(len(slab), bool)
        drop[np.nonzero(near_s)[0][np.isfinite(d)]] = True
        slab = slab[~drop]

    pos = np.concatenate([mat, np.concatenate(inc_pos), slab])
    kind = np.concatenate([np.zeros(len(mat), np.int8), np.concatenate(inc_kind),
                           np.full(len(slab), 3, np.int8)])
    del mat
    pos += rng.normal(0.0, sigma, size=pos.shape)
    return Frame(positions=wrap(pos, box), box=box,
                 labels={"kind": kind, "centres": centres, "inclusion_kind": kinds,
                         "slab_density": len(slab) / (w * L * L)})
