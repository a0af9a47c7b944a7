"""Pins of the oracle's disordered-structure mode (per-atom fractional
occupancy scaling the atom's density; paper, section "Overview": disordered
structures are supported) against routes that do not use the occupancy code:

* an occupancy w on every atom of species e equals species e with its
  primitive weights B scaled by w (the probe-table route);
* a site split into two co-located entries of the same species with
  occupancies w and 1 - w equals the ordered site, for every other centre;
* the isolated-atom closed form w sum_k B (alpha/lambda)^(3/2);
* occupancy 1 reproduces the ordered structure bit for bit;
* the analytic gradient against finite differences of the value.
"""
import numpy as np
import pytest

import gmp_synth as gs
import oracle


def _probes(seed, orders=(-1, 0, 1, 2, 3), tau=1e-9):
    return gs.small_probes(np.random.default_rng(seed), orders=orders, n_sigmas=3, n_elements=2,
                           n_prims=(1, 3), tau=tau)


def test_unit_occupancy_is_ordered_structure():
    st = gs.small_periodic(np.random.default_rng(1), n_atoms=8, density=0.05, dmin=1.4)
    p = _probes(2)
    assert oracle.features(st, p, occupancy=np.ones(8)).tobytes() == oracle.features(st, p).tobytes()


def test_species_occupancy_equals_scaled_weights():
    rng = np.random.default_rng(3)
    pos, spec, cell, pbc = gs.small_periodic(rng, n_atoms=10, density=0.05, dmin=1.4)
    p = _probes(4)
    w = 0.37
    occ = np.where(spec == 1, w, 1.0)
    F_occ = oracle.features((pos, spec, cell, pbc), p, occupancy=occ)
    B = p.B.copy()
    B[p.prim_offsets[1]:p.prim_offsets[2]] *= w
    # the cutoffs must stay those of the unscaled table: pin that they do not move
    q = gs.Probes(p.orders, p.sigmas, p.prim_offsets, B, p.beta, p.tau)
    assert np.array_equal(oracle.cutoffs(q), oracle.cutoffs(p))
    F_tab = oracle.features((pos, spec, cell, pbc), q)
    assert np.allclose(F_occ, F_tab, rtol=1e-13, atol=1e-300)


def test_split_site_equals_ordered_site():
    rng = np.random.default_rng(5)
    pos, spec, cell, pbc = gs.small_periodic(rng, n_atoms=9, density=0.05, dmin=1.4)
    p = _probes(6)
    F0 = oracle.features((pos, spec, cell, pbc), p)
    k = 4
    pos2 = np.concatenate([pos, pos[k:k + 1]])
    spec2 = np.concatenate([spec, spec[k:k + 1]])
    occ = np.ones(10)
    occ[k], occ[9] = 0.25, 0.75
    F2 = oracle.features((pos2, spec2, cell, pbc), p, occupancy=occ)
    assert np.allclose(F2[:9][np.arange(9) != k], F0[np.arange(9) != k], rtol=1e-12, atol=1e-300)
    # both halves of the split site see the same environment (themselves included)
    assert np.allclose(F2[k], F2[9], rtol=1e-12) and np.allclose(F2[k], F0[k], rtol=1e-12)


def test_isolated_atom_occupancy():
    p = _probes(7, orders=(0, 2))
    w = 0.6
    F = oracle.features((np.zeros((1, 3)), np.array([1], np.int32), np.zeros((3, 3)), 0), p,
                        occupancy=np.array([w]))
    sl = slice(p.prim_offsets[1], p.prim_offsets[2])
    for s, sg in enumerate(p.sigmas):
        a = 1.0 / (2 * sg * sg)
        want = w * np.sum(p.B[sl] * (a / (a + p.beta[sl])) ** 1.5)
        assert F[0, s] == pytest.approx(abs(want), rel=1e-13)
    assert np.all(F[0, 3:] == 0.0)


def test_occupancy_grad_fd():
    rng = np.random.default_rng(8)
    st, occ = gs.disorder(rng, gs.small_periodic(rng, n_atoms=5, density=0.05, dmin=1.4), n_elements=2,
                          mixed=0.4, vacant=0.4)
    pos, spec, cell, pbc = st
    n = len(pos)
    p = _probes(9, tau=1e-7)
    G = rng.standard_normal((n, p.n_features))
    gpos, gcell, F = oracle.grad(st, p, G, occupancy=occ)
    pairs = oracle.frozen_pairs(st, p)
    L0 = oracle.loss_frozen(st, p, G, pairs, occupancy=occ)
    assert L0 == pytest.approx(float(np.sum(G * F)), rel=1e-12)
    scale = max(np.abs(gpos).max(), np.abs(gcell).max())
    h = 1e-5
    for i in range(n):
        for k in range(3):
            p1 = pos.copy(); p1[i, k] += h
            p2 = pos.copy(); p2[i, k] -= h
            fd = (oracle.loss_frozen((p1, spec, cell, pbc), p, G, pairs, occupancy=occ)
                  - oracle.loss_frozen((p2, spec, cell, pbc), p, G, pairs, occupancy=occ)) / (2 * h)
            assert abs(fd - gpos[i, k]) <= 1e-6 * scale, (i, k)
    for a in range(3):
        for k in range(3):
            c1 = cell.copy(); c1[a, k] += h
            c2 = cell.copy(); c2[a, k] -= h
            fd = (oracle.loss_frozen((pos, spec, c1, pbc), p, G, pairs, occupancy=occ)
                  - oracle.loss_frozen((pos, spec, c2, pbc), p, G, pairs, occupancy=occ)) / (2 * h)
            assert abs(fd - gcell[a, k]) <= 1e-6 * scale, (a, k)
