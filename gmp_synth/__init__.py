"""Seeded synthetic inputs for the GMP feature path.

This module only draws numbers: atomic structures (positions, species,
lattice, periodicity), per-element Gaussian density primitives (B, beta) and
probe sets (orders, widths, overlap threshold).  It holds none of the
method's arithmetic, so both the HIP path and the CPU oracle may use it.

The paper ships its density primitives in pseudopotential files and its
structures in a pickled example set; neither is available, so every input
here is synthetic, shaped like the workloads the method targets (periodic
crystals of several elements, isolated clusters, batches of many small
structures, one large periodic system).

All generators take a ``numpy.random.Generator`` or a seed and are
deterministic for a given seed.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Probes", "Batch", "density_tables", "rsa_periodic", "rsa_cluster",
    "triclinic_cell", "make_batch", "config", "CONFIG_NAMES", "small_periodic",
    "small_cluster", "upstream_gradient", "disorder",
]


@dataclasses.dataclass
class Probes:
    """Probe set plus per-element density primitives.

    orders:        angular orders l (each in 0..4, or -1 for the local
                   density, which takes no sigma), output order as given
    sigmas:        Gaussian probe widths in Angstrom, output order as given
    prim_offsets:  int32 [n_elements+1]; element e owns primitives
                   prim_offsets[e] .. prim_offsets[e+1]-1
    B, beta:       float64 [n_prims]; primitive B*exp(-beta*r^2)
    tau:           overlap threshold (sets the cutoff per sigma)
    screening:     per-primitive screening (each primitive only inside its
                   own threshold radius), a variant of the cutoff rule
    radial_intervals: 0, or the interval count of tabulated radial factors
                   (a speed variant of the HIP path's forward)
    """
    orders: np.ndarray
    sigmas: np.ndarray
    prim_offsets: np.ndarray
    B: np.ndarray
    beta: np.ndarray
    tau: float
    screening: bool = False
    radial_intervals: int = 0

    @property
    def n_elements(self) -> int:
        return int(len(self.prim_offsets) - 1)

    @property
    def n_features(self) -> int:
        return int(sum(1 if int(l) == -1 else len(self.sigmas) for l in self.orders))


@dataclasses.dataclass
class Batch:
    """Packed batch of structures (CSR over atoms).

    atom_offsets: int64 [n_structs+1]
    pos:          float64 [n_atoms, 3] Cartesian, Angstrom
    species:      int32 [n_atoms]
    cell:         float64 [n_structs, 3, 3]; row m is lattice vector a_m
    pbc:          uint8 [n_structs]; bit k set = periodic along a_k
    occupancy:    float64 [n_atoms] fractional site occupancies, or None (all 1)
    """
    atom_offsets: np.ndarray
    pos: np.ndarray
    species: np.ndarray
    cell: np.ndarray
    pbc: np.ndarray
    occupancy: Optional[np.ndarray] = None

    @property
    def n_structs(self) -> int:
        return int(len(self.atom_offsets) - 1)

    @property
    def n_atoms(self) -> int:
        return int(self.atom_offsets[-1])

    def structure(self, s: int):
        a, b = int(self.atom_offsets[s]), int(self.atom_offsets[s + 1])
        return (self.pos[a:b], self.species[a:b], self.cell[s], int(self.pbc[s]))


def _rng(seed_or_rng) -> np.random.Generator:
    if isinstance(seed_or_rng, np.random.Generator):
        return seed_or_rng
    return np.random.default_rng(seed_or_rng)


def _log_uniform(rng, lo, hi, size=None):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))


def density_tables(rng, n_elements: int, n_prims, B_range=(0.01, 10.0),
                   beta_range=(0.1, 30.0)):
    """Per-element primitives: B log-uniform in B_range, beta log-uniform in
    beta_range (1/Angstrom^2).  ``n_prims`` is an int or an inclusive
    (lo, hi) range drawn per element."""
    rng = _rng(rng)
    counts = []
    for _ in range(n_elements):
        if isinstance(n_prims, (tuple, list)):
            counts.append(int(rng.integers(n_prims[0], n_prims[1] + 1)))
        else:
            counts.append(int(n_prims))
    offs = np.zeros(n_elements + 1, dtype=np.int32)
    offs[1:] = np.cumsum(counts)
    n = int(offs[-1])
    B = _log_uniform(rng, B_range[0], B_range[1], n)
    beta = _log_uniform(rng, beta_range[0], beta_range[1], n)
    return offs, B.astype(np.float64), beta.astype(np.float64)


def _image_shifts(cell, reach):
    """Integer lattice shifts n with |n_k| <= ceil(1/2 + reach/h_k): every
    image within ``reach`` of a point whose fractional offset was rounded
    into [-1/2, 1/2] (cell rows are lattice vectors, h_k the heights)."""
    inv = np.linalg.inv(cell)
    heights = 1.0 / np.linalg.norm(inv, axis=0)
    nmax = [int(math.ceil(0.5 + reach / h)) for h in heights]
    rng_ = [np.arange(-m, m + 1) for m in nmax]
    g = np.stack(np.meshgrid(*rng_, indexing="ij"), axis=-1).reshape(-1, 3)
    return g.astype(np.float64)


def rsa_periodic(rng, cell, n_atoms: int, dmin: float, max_tries=2_000_000):
    """Random sequential addition of ``n_atoms`` points in a periodic cell,
    rejecting any candidate closer than ``dmin`` to an accepted point or any
    of its periodic images.  Uses a fractional-coordinate grid for large
    cells and an all-pairs image check for small ones."""
    rng = _rng(rng)
    cell = np.asarray(cell, dtype=np.float64)
    inv = np.linalg.inv(cell)
    heights = 1.0 / np.linalg.norm(inv, axis=0)
    ng = np.maximum(1, np.floor(heights / dmin).astype(int))
    if np.all(ng >= 3) and n_atoms > 512:
        return _rsa_grid(rng, cell, inv, ng, n_atoms, dmin, max_tries)
    shifts = _image_shifts(cell, dmin) @ cell  # Cartesian image offsets
    pts = np.empty((n_atoms, 3))
    k = 0
    tries = 0
    d2 = dmin * dmin

    def min_d2(r, others):
        fr = (others - r) @ inv
        fr -= np.round(fr)
        dd = (fr @ cell)[:, None, :] + shifts[None, :, :]
        return np.min(np.einsum("kid,kid->ki", dd, dd))

    while k < n_atoms:
        # Candidates are drawn in blocks and accepted in draw order, each one
        # tested against every point accepted before it: the same sequence as
        # one-by-one random sequential addition with these draws.
        block = rng.random((64, 3)) @ cell
        tries += len(block)
        if tries > max_tries:
            raise RuntimeError("random sequential addition did not converge")
        if k:
            fr = (block[:, None, :] - pts[None, :k, :]) @ inv
            fr -= np.round(fr)
            dd = (fr @ cell)[:, :, None, :] + shifts[None, None, :, :]
            ok = np.min(np.einsum("bkid,bkid->bki", dd, dd), axis=(1, 2)) >= d2
        else:
            ok = np.ones(len(block), bool)
        k_block = k
        for bi in np.flatnonzero(ok):
            r = block[bi]
            if k > k_block and min_d2(r, pts[k_block:k]) < d2:
                continue
            pts[k] = r
            k += 1
            if k == n_atoms:
                break
    return pts


def _rsa_grid(rng, cell, inv, ng, n_atoms, dmin, max_tries):
    cells = {}
    pts = np.empty((n_atoms, 3))
    fpts = np.empty((n_atoms, 3))
    d2 = dmin * dmin
    k = 0
    tries = 0
    offs = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    while k < n_atoms:
        # draw candidates in blocks to amortise the Python overhead
        block = rng.random((256, 3))
        for f in block:
            tries += 1
            if tries > max_tries:
                raise RuntimeError("random sequential addition did not converge")
            g = (f * ng).astype(int) % ng
            ok = True
            cand = []
            for o in offs:
                key = ((g[0] + o[0]) % ng[0], (g[1] + o[1]) % ng[1], (g[2] + o[2]) % ng[2])
                lst = cells.get(key)
                if lst:
                    cand.extend(lst)
            if cand:
                df = fpts[cand] - f
                df -= np.round(df)
                dc = df @ cell
                if np.min(np.einsum("ij,ij->i", dc, dc)) < d2:
                    ok = False
            if not ok:
                continue
            pts[k] = f @ cell
            fpts[k] = f
            cells.setdefault((int(g[0]), int(g[1]), int(g[2])), []).append(k)
            k += 1
            if k == n_atoms:
                break
    return pts


def rsa_cluster(rng, n_atoms: int, radius: float, dmin: float, max_tries=2_000_000):
    """Random sequential addition inside a sphere of ``radius`` (no images).
    Candidates are drawn in blocks and accepted in draw order."""
    rng = _rng(rng)
    pts = np.empty((n_atoms, 3))
    k = 0
    tries = 0
    d2 = dmin * dmin
    while k < n_atoms:
        block = rng.uniform(-radius, radius, (64, 3))
        tries += len(block)
        if tries > max_tries:
            raise RuntimeError("random sequential addition did not converge")
        inside = np.einsum("bd,bd->b", block, block) <= radius * radius
        if k:
            diff = block[:, None, :] - pts[None, :k, :]
            ok = inside & (np.min(np.einsum("bkd,bkd->bk", diff, diff), axis=1) >= d2)
        else:
            ok = inside
        k_block = k
        for bi in np.flatnonzero(ok):
            r = block[bi]
            if k > k_block:
                dv = pts[k_block:k] - r
                if np.min(np.einsum("kd,kd->k", dv, dv)) < d2:
                    continue
            pts[k] = r
            k += 1
            if k == n_atoms:
                break
    return pts


def triclinic_cell(rng, volume: float, angle_range=(70.0, 110.0),
                   aspect_range=(0.8, 1.25), min_vol_ratio=0.5):
    """A random triclinic cell of the given volume.  Angles are uniform in
    ``angle_range`` (degrees), edge-length ratios b/a and c/a log-uniform in
    ``aspect_range``; draws are rejected unless V/(abc) >= min_vol_ratio."""
    rng = _rng(rng)
    while True:
        al, be, ga = np.radians(rng.uniform(angle_range[0], angle_range[1], 3))
        ca, cb, cg = math.cos(al), math.cos(be), math.cos(ga)
        disc = 1.0 - ca * ca - cb * cb - cg * cg + 2.0 * ca * cb * cg
        if disc <= 0.0 or math.sqrt(disc) < min_vol_ratio:
            continue
        rb = _log_uniform(rng, *aspect_range)
        rc = _log_uniform(rng, *aspect_range)
        a = (volume / (rb * rc * math.sqrt(disc))) ** (1.0 / 3.0)
        b, c = rb * a, rc * a
        sg = math.sin(ga)
        a1 = np.array([a, 0.0, 0.0])
        a2 = np.array([b * cg, b * sg, 0.0])
        cx = c * cb
        cy = c * (ca - cb * cg) / sg
        cz = math.sqrt(max(c * c - cx * cx - cy * cy, 0.0))
        a3 = np.array([cx, cy, cz])
        return np.stack([a1, a2, a3])


def _species_uniform(rng, n, n_elements):
    return rng.integers(0, n_elements, size=n).astype(np.int32)


def make_batch(structs: Sequence, occupancy=None) -> Batch:
    """Pack a list of (pos, species, cell, pbc) into a CSR batch; occupancy
    (optional) is one array per structure."""
    offs = np.zeros(len(structs) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(s[0]) for s in structs])
    pos = np.concatenate([np.asarray(s[0], dtype=np.float64).reshape(-1, 3) for s in structs], axis=0)
    spec = np.concatenate([np.asarray(s[1], dtype=np.int32) for s in structs])
    cell = np.stack([np.asarray(s[2], dtype=np.float64).reshape(3, 3) for s in structs])
    pbc = np.array([int(s[3]) for s in structs], dtype=np.uint8)
    occ = None
    if occupancy is not None:
        occ = np.concatenate([np.asarray(o, dtype=np.float64).reshape(-1) for o in occupancy])
        assert len(occ) == len(spec)
    return Batch(offs, np.ascontiguousarray(pos), spec, cell, pbc, occ)


def disorder(rng, struct, n_elements: int, mixed: float = 0.3, vacant: float = 0.2):
    """A disordered version of (pos, species, cell, pbc): a fraction `mixed`
    of the sites become shared by two species (one entry per species at the
    same position, occupancies w and 1 - w), a fraction `vacant` keep one
    species with occupancy in (0.3, 1); returns (struct, occupancy)."""
    rng = _rng(rng)
    pos, spec, cell, pbc = struct
    pos_out, spec_out, occ_out = [], [], []
    for r, e in zip(np.asarray(pos), np.asarray(spec)):
        u = rng.random()
        if u < mixed and n_elements > 1:
            w = rng.uniform(0.1, 0.9)
            e2 = (int(e) + 1 + int(rng.integers(n_elements - 1))) % n_elements
            pos_out += [r, r]; spec_out += [int(e), e2]; occ_out += [w, 1.0 - w]
        elif u < mixed + vacant:
            pos_out.append(r); spec_out.append(int(e)); occ_out.append(rng.uniform(0.3, 1.0))
        else:
            pos_out.append(r); spec_out.append(int(e)); occ_out.append(1.0)
    return ((np.asarray(pos_out, np.float64).reshape(-1, 3), np.asarray(spec_out, np.int32), cell, pbc),
            np.asarray(occ_out, np.float64))


def scatter_images(rng, pos, cell, reach=1):
    """Move every atom by a random lattice vector with integer components in
    [-reach, reach]; the structure is unchanged, the stored coordinates are
    not inside the home cell any more."""
    rng = _rng(rng)
    n = rng.integers(-reach, reach + 1, size=(len(pos), 3)).astype(np.float64)
    return pos + n @ np.asarray(cell)


# --------------------------------------------------------------------------
# Workloads.  Seeds 1..5 are the defaults of the five named configurations.
# --------------------------------------------------------------------------

CONFIG_NAMES = ("C1", "C2", "C3", "C4", "C5")

CONFIG_TEXT = {
    "C1": "periodic cubic 10 A cell, 64 atoms (2 elements x 32), dmin 1.8 A, "
          "4 primitives/element B~logU[0.01,10] beta~logU[0.1,20]; l=0..2 x "
          "sigma {0.25,0.5,0.75,1.0}; tau 1e-11",
    "C2": "periodic 40x40x40 A cell, 4096 atoms, 5 elements (Dirichlet "
          "proportions), dmin 1.6 A, 5 primitives/element B~logU[0.01,10] "
          "beta~logU[0.1,30]; l=0..4 x 8 sigma geomspace(0.1,1.6); tau 1e-11",
    "C3": "2048 structures, N~round(exp(U(ln8,ln256))); even index periodic "
          "triclinic (angles 70-110 deg, 0.08 atoms/A^3), odd index isolated "
          "cluster (sphere at 0.08 atoms/A^3); dmin 1.6 A; 10 elements with "
          "3-6 primitives; l=0..4 x 8 sigma geomspace(0.1,1.6); tau 1e-11",
    "C4": "512 periodic triclinic structures, N~U{32..200}, 0.08 atoms/A^3, "
          "dmin 1.6 A, 4 elements x 4 primitives B~logU[0.01,10] "
          "beta~logU[0.1,30]; l=0..3 x 6 sigma geomspace(0.15,1.2); tau 1e-11",
    "C5": "periodic cubic cell (1e5/0.092)^(1/3)=102.8 A, 100000 atoms, "
          "6 elements x 6 primitives, dmin 1.5 A; l=0..4 x 10 sigma "
          "geomspace(0.1,2.0); tau 1e-11",
}


def config(name: str, seed: Optional[int] = None, n_structs: Optional[int] = None,
           n_atoms: Optional[int] = None):
    """Build one of the five workloads.  Returns (Batch, Probes).

    ``n_structs`` shrinks the batched workloads (C3, C4) and ``n_atoms`` the
    single-structure ones (C2, C5) for quick tests; by default the full sizes
    are generated.
    """
    name = name.upper()
    if seed is None:
        seed = CONFIG_NAMES.index(name) + 1
    rng = np.random.default_rng(seed)
    if name == "C1":
        offs, B, beta = density_tables(rng, 2, 4, (0.01, 10.0), (0.1, 20.0))
        cell = np.eye(3) * 10.0
        pos = rsa_periodic(rng, cell, 64, 1.8)
        spec = np.repeat(np.arange(2, dtype=np.int32), 32)
        rng.shuffle(spec)
        probes = Probes(np.array([0, 1, 2], np.int32), np.array([0.25, 0.5, 0.75, 1.0]),
                        offs, B, beta, 1e-11)
        return make_batch([(pos, spec, cell, 7)]), probes
    if name in ("C2", "C5"):
        if name == "C2":
            n = 4096 if n_atoms is None else int(n_atoms)
            E, K, dmin = 5, 5, 1.6
            edge = 40.0 if n_atoms is None else 40.0 * (n / 4096.0) ** (1.0 / 3.0)
            sig = np.geomspace(0.1, 1.6, 8)
        else:
            n = 100_000 if n_atoms is None else int(n_atoms)
            E, K, dmin = 6, 6, 1.5
            edge = (n / 0.092) ** (1.0 / 3.0)
            sig = np.geomspace(0.1, 2.0, 10)
        offs, B, beta = density_tables(rng, E, K, (0.01, 10.0), (0.1, 30.0))
        cell = np.eye(3) * edge
        pos = rsa_periodic(rng, cell, n, dmin)
        if name == "C2":
            prop = rng.dirichlet(np.ones(E))
            cnt = np.floor(prop * n).astype(int)
            while cnt.sum() < n:
                cnt[int(np.argmax(prop * n - cnt))] += 1
            spec = np.repeat(np.arange(E, dtype=np.int32), cnt)
            rng.shuffle(spec)
        else:
            spec = _species_uniform(rng, n, E)
        probes = Probes(np.arange(5, dtype=np.int32), sig, offs, B, beta, 1e-11)
        return make_batch([(pos, spec, cell, 7)]), probes
    if name == "C3":
        ns = 2048 if n_structs is None else int(n_structs)
        offs, B, beta = density_tables(rng, 10, (3, 6), (0.01, 10.0), (0.1, 30.0))
        structs = []
        for s in range(ns):
            N = int(round(math.exp(rng.uniform(math.log(8), math.log(256)))))
            if s % 2 == 0:
                cell = triclinic_cell(rng, N / 0.08)
                pos = rsa_periodic(rng, cell, N, 1.6)
                pbc = 7
            else:
                radius = (3.0 * N / (4.0 * math.pi * 0.08)) ** (1.0 / 3.0)
                pos = rsa_cluster(rng, N, radius, 1.6)
                cell = np.zeros((3, 3))
                pbc = 0
            structs.append((pos, _species_uniform(rng, N, 10), cell, pbc))
        probes = Probes(np.arange(5, dtype=np.int32), np.geomspace(0.1, 1.6, 8),
                        offs, B, beta, 1e-11)
        return make_batch(structs), probes
    if name == "C4":
        ns = 512 if n_structs is None else int(n_structs)
        offs, B, beta = density_tables(rng, 4, 4, (0.01, 10.0), (0.1, 30.0))
        structs = []
        for s in range(ns):
            N = int(rng.integers(32, 201))
            cell = triclinic_cell(rng, N / 0.08)
            pos = rsa_periodic(rng, cell, N, 1.6)
            structs.append((pos, _species_uniform(rng, N, 4), cell, 7))
        probes = Probes(np.arange(4, dtype=np.int32), np.geomspace(0.15, 1.2, 6),
                        offs, B, beta, 1e-11)
        return make_batch(structs), probes
    raise ValueError(f"unknown workload {name!r}")


def upstream_gradient(rng, n_atoms: int, n_features: int):
    """Seeded N(0,1) upstream gradient over the features."""
    rng = _rng(rng)
    return rng.standard_normal((n_atoms, n_features))


# --------------------------------------------------------------------------
# Small structures for tests.
# --------------------------------------------------------------------------

def small_periodic(rng, n_atoms=12, n_elements=2, density=0.05, dmin=1.4,
                   cell=None, scatter=True, pbc=7):
    """A small periodic triclinic structure (coordinates optionally scattered
    over neighbouring images)."""
    rng = _rng(rng)
    if cell is None:
        cell = triclinic_cell(rng, n_atoms / density)
    pos = rsa_periodic(rng, cell, n_atoms, dmin)
    if scatter:
        pos = scatter_images(rng, pos, cell)
    return (pos, _species_uniform(rng, n_atoms, n_elements), np.asarray(cell, float), pbc)


def small_cluster(rng, n_atoms=8, n_elements=2, radius=3.0, dmin=1.2):
    rng = _rng(rng)
    pos = rsa_cluster(rng, n_atoms, radius, dmin)
    return (pos, _species_uniform(rng, n_atoms, n_elements), np.zeros((3, 3)), 0)


def small_probes(rng, orders=(0, 1, 2, 3, 4), n_sigmas=3, n_elements=2, n_prims=(1, 3),
                 tau=1e-8, sig_range=(0.3, 1.2), beta_range=(0.3, 6.0), B_range=(0.05, 5.0)):
    """A light probe set with short cutoffs, for tiny oracle-checked cases."""
    rng = _rng(rng)
    offs, B, beta = density_tables(rng, n_elements, n_prims, B_range, beta_range)
    sig = np.sort(_log_uniform(rng, sig_range[0], sig_range[1], n_sigmas))
    return Probes(np.asarray(orders, np.int32), sig, offs, B, beta, float(tau))
