"""The oracle's analytic gradient of L = sum G*F against central finite
differences of L over a frozen pair set (h = 1e-5 A), plus the identities
that translation and rotation invariance force on it."""
import numpy as np
import pytest

import gmp_synth as gs
import oracle


def _probes(seed, orders=(0, 1, 2, 3, 4)):
    return gs.small_probes(np.random.default_rng(seed), orders=orders, n_sigmas=2,
                           n_elements=2, n_prims=(1, 2), tau=1e-7)


def _fd_check(struct, probes, G, idx_pos, cell_entries, h=1e-5, rel=1e-6):
    pos, spec, cell, pbc = struct
    gpos, gcell, F = oracle.grad(struct, probes, G)
    pairs = oracle.frozen_pairs(struct, probes)
    L0 = oracle.loss_frozen(struct, probes, G, pairs)
    assert L0 == pytest.approx(float(np.sum(G * F)), rel=1e-12)
    scale = max(np.abs(gpos).max(), np.abs(gcell).max())
    for (i, k) in idx_pos:
        p1 = pos.copy(); p1[i, k] += h
        p2 = pos.copy(); p2[i, k] -= h
        fd = (oracle.loss_frozen((p1, spec, cell, pbc), probes, G, pairs)
              - oracle.loss_frozen((p2, spec, cell, pbc), probes, G, pairs)) / (2 * h)
        assert abs(fd - gpos[i, k]) <= rel * scale, (i, k, fd, gpos[i, k])
    for (a, k) in cell_entries:
        c1 = cell.copy(); c1[a, k] += h
        c2 = cell.copy(); c2[a, k] -= h
        fd = (oracle.loss_frozen((pos, spec, c1, pbc), probes, G, pairs)
              - oracle.loss_frozen((pos, spec, c2, pbc), probes, G, pairs)) / (2 * h)
        assert abs(fd - gcell[a, k]) <= rel * scale, (a, k, fd, gcell[a, k])
    return gpos, gcell


def test_grad_fd_periodic():
    rng = np.random.default_rng(1)
    struct = gs.small_periodic(rng, n_atoms=6, density=0.05, dmin=1.4)
    probes = _probes(2)
    G = rng.standard_normal((6, probes.n_features))
    idx = [(i, k) for i in range(6) for k in range(3)]
    cells = [(a, k) for a in range(3) for k in range(3)]
    _fd_check(struct, probes, G, idx, cells)


def test_grad_fd_cluster():
    rng = np.random.default_rng(3)
    struct = gs.small_cluster(rng, n_atoms=6, radius=2.5)
    probes = _probes(4)
    G = rng.standard_normal((6, probes.n_features))
    _fd_check(struct, probes, G, [(i, k) for i in range(6) for k in range(3)], [])


def test_grad_identities_periodic():
    """sum_i g_i = 0 (translation) and sum_i g_i (x) R_i + sum_m G_m (x) a_m
    symmetric (rotation)."""
    rng = np.random.default_rng(5)
    struct = gs.small_periodic(rng, n_atoms=8, density=0.05, dmin=1.4)
    probes = _probes(6)
    G = rng.standard_normal((8, probes.n_features))
    gpos, gcell, _ = oracle.grad(struct, probes, G)
    scale = np.abs(gpos).max()
    assert np.abs(gpos.sum(axis=0)).max() <= 1e-11 * scale * len(gpos)
    pos, cell = struct[0], struct[2]
    vir = gpos.T @ pos + gcell.T @ cell
    assert np.abs(vir - vir.T).max() <= 1e-10 * np.abs(vir).max()


def test_grad_identities_cluster():
    rng = np.random.default_rng(7)
    struct = gs.small_cluster(rng, n_atoms=8, radius=3.0)
    probes = _probes(8)
    G = rng.standard_normal((8, probes.n_features))
    gpos, gcell, _ = oracle.grad(struct, probes, G)
    scale = np.abs(gpos).max()
    assert np.abs(gpos.sum(axis=0)).max() <= 1e-11 * scale * len(gpos)
    torque = np.cross(struct[0], gpos).sum(axis=0)
    assert np.abs(torque).max() <= 1e-10 * scale * np.abs(struct[0]).max() * len(gpos)
    assert np.all(gcell == 0.0)


def test_grad_isolated_atom_is_zero():
    probes = _probes(9)
    G = np.ones((1, probes.n_features))
    gpos, gcell, _ = oracle.grad((np.zeros((1, 3)), np.zeros(1, np.int32), np.zeros((3, 3)), 0), probes, G)
    assert np.all(gpos == 0.0)


def test_grad_restricted_to_listed_centres():
    """The gradient restricted to listed centres (used where the full oracle
    gradient of a large system is too slow): with every centre listed it is
    oracle grad() bit for bit; with a subset it equals grad() with G zero on
    the other centres, and central differences of the frozen-pair loss with
    that G (an independent check of the restriction)."""
    rng = np.random.default_rng(11)
    struct = gs.small_periodic(rng, n_atoms=7, density=0.05, dmin=1.4)
    probes = _probes(12)
    G = rng.standard_normal((7, probes.n_features))
    gp_all, gc_all, _ = oracle.grad(struct, probes, G)
    gp, gc = oracle.grad_centres(struct, probes, np.arange(7), G)
    assert np.array_equal(gp, gp_all) and np.array_equal(gc, gc_all)
    sub = np.array([5, 1, 3])
    Gz = np.zeros_like(G)
    Gz[sub] = G[sub]
    gp_z, gc_z, _ = oracle.grad(struct, probes, Gz)
    gp_s, gc_s = oracle.grad_centres(struct, probes, sub, G[sub])
    scale = max(np.abs(gp_z).max(), np.abs(gc_z).max())
    assert np.abs(gp_s - gp_z).max() <= 1e-14 * scale and np.abs(gc_s - gc_z).max() <= 1e-14 * scale
    gp_fd, gc_fd = _fd_check(struct, probes, Gz, [(i, k) for i in range(7) for k in range(3)],
                             [(a, k) for a in range(3) for k in range(3)])
    assert np.abs(gp_s - gp_fd).max() <= 1e-14 * scale


def test_neighbors_many_equal_single_lists():
    """Lists of many centres computed together are the single-centre lists."""
    rng = np.random.default_rng(13)
    struct = gs.small_periodic(rng, n_atoms=9, density=0.06, dmin=1.3)
    probes = _probes(14)
    rc2 = oracle.cutoffs(probes)
    cs = [4, 0, 8, 2]
    r = oracle.neighbors_many(struct, rc2, cs)
    for t, c in enumerate(cs):
        one = oracle.neighbors(struct, rc2, c)
        lo, hi = r["offs"][t], r["offs"][t + 1]
        for key in ("j", "n", "q", "shell", "e"):
            assert np.array_equal(r[key][lo:hi], one[key]), key
