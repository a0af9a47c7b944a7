"""Invariances the GMP features must have, checked on the FP64 oracle:
rotation and reflection, translation, moving an atom by a lattice vector,
supercell replication, permutation of atoms, and the zeros that cubic
symmetry forces on orders 1..3."""
import numpy as np
import pytest

import gmp_synth as gs
import oracle


def _probes(seed, orders=(0, 1, 2, 3, 4)):
    return gs.small_probes(np.random.default_rng(seed), orders=orders, n_sigmas=3,
                           n_elements=2, n_prims=(1, 3), tau=1e-8)


def _struct(seed, n=10):
    return gs.small_periodic(np.random.default_rng(seed), n_atoms=n, n_elements=2,
                             density=0.05, dmin=1.4)


def _close(a, b, rel=1e-10):
    """Per-feature comparison scaled by the column magnitude (a feature that
    vanishes by symmetry is compared on the scale of its column)."""
    scale = np.maximum(np.abs(b).max(axis=0, keepdims=True), 1e-300)
    return np.all(np.abs(a - b) <= rel * scale + 1e-14 * np.abs(b))


def _random_orthogonal(rng, reflect):
    Q, R = np.linalg.qr(rng.normal(size=(3, 3)))
    Q = Q * np.sign(np.diag(R))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    if reflect:
        Q = Q @ np.diag([1.0, 1.0, -1.0])
    return Q


@pytest.mark.parametrize("reflect", [False, True])
def test_rotation_invariance(reflect):
    probes = _probes(1)
    pos, spec, cell, pbc = _struct(2)
    F0 = oracle.features((pos, spec, cell, pbc), probes)
    Q = _random_orthogonal(np.random.default_rng(3), reflect)
    F1 = oracle.features((pos @ Q.T, spec, cell @ Q.T, pbc), probes)
    assert _close(F1, F0)


def test_rotation_invariance_cluster():
    probes = _probes(4)
    pos, spec, cell, pbc = gs.small_cluster(np.random.default_rng(5), n_atoms=9, radius=3.0)
    F0 = oracle.features((pos, spec, cell, pbc), probes)
    Q = _random_orthogonal(np.random.default_rng(6), True)
    F1 = oracle.features((pos @ Q.T + 3.3, spec, cell, pbc), probes)
    assert _close(F1, F0)


def test_translation_invariance():
    probes = _probes(7)
    pos, spec, cell, pbc = _struct(8)
    F0 = oracle.features((pos, spec, cell, pbc), probes)
    F1 = oracle.features((pos + np.array([0.37, -1.9, 5.1]), spec, cell, pbc), probes)
    assert _close(F1, F0)


def test_lattice_shift_invariance():
    probes = _probes(9)
    pos, spec, cell, pbc = _struct(10)
    F0 = oracle.features((pos, spec, cell, pbc), probes)
    rng = np.random.default_rng(11)
    shift = rng.integers(-3, 4, size=(len(pos), 3)) @ cell
    F1 = oracle.features((pos + shift, spec, cell, pbc), probes)
    assert _close(F1, F0)


def test_supercell_replication():
    probes = _probes(12)
    pos, spec, cell, pbc = _struct(13, n=6)
    F0 = oracle.features((pos, spec, cell, pbc), probes)
    reps = []
    for a in range(2):
        for b in range(2):
            for c in range(2):
                reps.append(pos + np.array([a, b, c]) @ cell)
    big = np.concatenate(reps)
    F1 = oracle.features((big, np.tile(spec, 8), 2 * cell, pbc), probes)
    for r in range(8):
        assert _close(F1[r * len(pos):(r + 1) * len(pos)], F0)


def test_permutation_equivariance():
    probes = _probes(14)
    pos, spec, cell, pbc = _struct(15)
    F0 = oracle.features((pos, spec, cell, pbc), probes)
    perm = np.random.default_rng(16).permutation(len(pos))
    F1 = oracle.features((pos[perm], spec[perm], cell, pbc), probes)
    assert _close(F1, F0[perm])


def test_same_element_swap_leaves_features():
    """Exchanging the positions of two atoms of the same element permutes
    their feature rows and leaves every other row unchanged."""
    probes = _probes(17)
    pos, spec, cell, pbc = _struct(18, n=12)
    same = np.flatnonzero(spec == spec[0])
    assert len(same) >= 2
    a, b = same[0], same[1]
    p2 = pos.copy(); p2[[a, b]] = pos[[b, a]]
    F0 = oracle.features((pos, spec, cell, pbc), probes)
    F1 = oracle.features((p2, spec, cell, pbc), probes)
    idx = np.arange(len(pos)); idx[[a, b]] = [b, a]
    assert _close(F1, F0[idx])


@pytest.mark.parametrize("lattice", ["sc", "fcc"])
def test_cubic_symmetry_zeros(lattice):
    """A site with cubic point symmetry has no l=1,2,3 multipole; l=4 survives."""
    probes = _probes(19)
    a = 3.1
    if lattice == "sc":
        pos = np.zeros((1, 3)); cell = np.eye(3) * a
    else:
        cell = np.eye(3) * (a * 1.6)
        pos = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]]) @ cell
    spec = np.zeros(len(pos), np.int32)
    F = oracle.features((pos, spec, cell, 7), probes)
    S = len(probes.sigmas)
    F0 = F[:, 0:S]
    for o, l in enumerate(probes.orders):
        blk = F[:, o * S:(o + 1) * S]
        if l in (1, 2, 3):
            assert np.all(blk <= 1e-11 * F0.max())
        if l == 4:
            assert np.all(blk > 1e-6 * F0.max())
