"""Pins of the oracle's per-pair feature Jacobian (the paper's feature
derivatives with respect to atom positions) against finite differences of
the feature values over a frozen pair set: for weights R (random, and unit
vectors of single features), d/dR_{a,k} sum R F equals the Jacobian
assembled per atom, and d/dcell likewise; order -1 and occupancies
included."""
import numpy as np
import pytest

import gmp_synth as gs
import oracle


def _check(struct, probes, R, occupancy=None, h=1e-5):
    pos, spec, cell, pbc = struct
    n = len(pos)
    jac, offs = oracle.jacobian(struct, probes, occupancy=occupancy)
    rc2 = oracle.cutoffs(probes)
    _, m = oracle.wrap(pos, cell, pbc)
    gpos = np.zeros((n, 3))
    gcell = np.zeros((3, 3))
    for i in range(n):
        nb = oracle.neighbors(struct, rc2, i)
        v = np.einsum("f,pfk->pk", R[i], jac[offs[i]:offs[i + 1]])
        np.add.at(gpos, nb["j"], v)
        gpos[i] -= v.sum(axis=0)
        nt = nb["n"] - m[nb["j"]] + m[i]
        gcell += nt.T @ v
    pairs = oracle.frozen_pairs(struct, probes)
    scale = max(np.abs(gpos).max(), np.abs(gcell).max())

    def L(ps, c):
        return oracle.loss_frozen((ps, spec, c, pbc), probes, R, pairs, occupancy=occupancy)
    for a in range(n):
        for k in range(3):
            p1 = pos.copy(); p1[a, k] += h
            p2 = pos.copy(); p2[a, k] -= h
            assert abs((L(p1, cell) - L(p2, cell)) / (2 * h) - gpos[a, k]) <= 1e-6 * scale, (a, k)
    if pbc:
        for a in range(3):
            for k in range(3):
                c1 = cell.copy(); c1[a, k] += h
                c2 = cell.copy(); c2[a, k] -= h
                assert abs((L(pos, c1) - L(pos, c2)) / (2 * h) - gcell[a, k]) <= 1e-6 * scale, (a, k)
    # the analytic gradient is the same contraction
    rp, rc, _ = oracle.grad(struct, probes, R, occupancy=occupancy)
    assert np.allclose(rp, gpos, rtol=0, atol=1e-12 * scale) and np.allclose(rc, gcell, rtol=0, atol=1e-12 * scale)


def _probes(seed, orders):
    return gs.small_probes(np.random.default_rng(seed), orders=orders, n_sigmas=2, n_elements=2, n_prims=(1, 3),
                           tau=1e-7)


def test_jacobian_fd_periodic_random_weights():
    rng = np.random.default_rng(1)
    st = gs.small_periodic(rng, n_atoms=5, density=0.05, dmin=1.4)
    p = _probes(2, (-1, 0, 1, 2))
    _check(st, p, rng.standard_normal((5, p.n_features)))


@pytest.mark.parametrize("f", [0, 1, 2, 3, 4])
def test_jacobian_fd_single_feature(f):
    """Unit weights on one feature of every centre pin that feature's own
    Jacobian columns."""
    rng = np.random.default_rng(3)
    st = gs.small_cluster(rng, n_atoms=6, radius=2.5)
    p = _probes(4, (3, -1, 1))
    R = np.zeros((6, p.n_features))
    R[:, f] = 1.0
    _check(st, p, R)


def test_jacobian_fd_with_occupancy():
    rng = np.random.default_rng(5)
    st, occ = gs.disorder(rng, gs.small_periodic(rng, n_atoms=4, density=0.05, dmin=1.4), n_elements=2)
    p = _probes(6, (0, 2, 4))
    _check(st, p, rng.standard_normal((len(st[0]), p.n_features)), occupancy=occ)


def test_jacobian_isolated_atom_is_zero():
    p = _probes(7, (-1, 0, 1, 2))
    jac, offs = oracle.jacobian((np.zeros((1, 3)), np.zeros(1, np.int32), np.zeros((3, 3)), 0), p)
    assert offs.tolist() == [0, 1] and np.all(jac == 0.0)
