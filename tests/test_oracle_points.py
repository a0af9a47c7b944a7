"""Pins of the oracle's reference-point mode (features at arbitrary positions
instead of the atoms; paper, section "Overview"):

* a point placed on an atom reproduces that atom's features bit for bit
  (same wrap, same images, same canonical list);
* one atom in vacuum seen from a point at distance r: the dimer closed form
  F_l = sqrt((2l-1)!! l!) |c_l(r^2)| r^l and the density sum_k B e^{-beta r^2};
* a point farther than every cutoff sees nothing;
* invariance under lattice translations of a point, rotations of the whole
  system, and a common translation (sum of all gradients = 0);
* the analytic gradient (atoms, points, cell) against finite differences.
"""
import math

import numpy as np
import pytest

import gmp_synth as gs
import oracle


def _probes(seed, orders=(-1, 0, 1, 2, 3, 4), tau=1e-9, n_sigmas=3):
    return gs.small_probes(np.random.default_rng(seed), orders=orders, n_sigmas=n_sigmas, n_elements=2,
                           n_prims=(1, 3), tau=tau)


def _dfact(n):
    return 1 if n <= 0 else n * _dfact(n - 2)


def test_point_on_atom_is_that_atoms_features():
    st = gs.small_periodic(np.random.default_rng(1), n_atoms=9, density=0.05, dmin=1.4)
    p = _probes(2)
    F = oracle.features(st, p)
    for i in (0, 4, 8):
        Fp = oracle.point_features(st, p, st[0][i:i + 1])
        assert Fp.tobytes() == F[i:i + 1].tobytes()


def test_point_near_isolated_atom_closed_form():
    p = _probes(3, tau=1e-12)
    e = 1
    sl = slice(p.prim_offsets[e], p.prim_offsets[e + 1])
    atom = np.array([[0.4, -1.0, 2.0]])
    d = np.array([0.6, 0.8, -0.3])
    r2 = float(d @ d)
    F = oracle.point_features((atom, np.array([e], np.int32), np.zeros((3, 3)), 0), p, atom - d)[0]
    f = 0
    for l in p.orders:
        if l == -1:
            assert F[f] == pytest.approx(np.sum(p.B[sl] * np.exp(-p.beta[sl] * r2)), rel=1e-13)
            f += 1
            continue
        for sg in p.sigmas:
            a = 1.0 / (2 * sg * sg)
            lam = a + p.beta[sl]
            c = np.sum(p.B[sl] * (a / lam) ** 1.5 * (p.beta[sl] / lam) ** l * np.exp(-a * p.beta[sl] / lam * r2))
            want = math.sqrt(_dfact(2 * l - 1) * math.factorial(l)) * abs(c) * r2 ** (l / 2)
            assert F[f] == pytest.approx(want, rel=1e-12), (l, sg)
            f += 1


def test_far_point_sees_nothing():
    p = _probes(4, tau=1e-4)
    st = gs.small_cluster(np.random.default_rng(5), n_atoms=5, radius=2.0)
    rc = math.sqrt(oracle.cutoffs(p).max())
    far = np.array([[rc + 10.0, 0.0, 0.0]])
    assert np.all(oracle.point_features(st, p, far) == 0.0)
    gpos, gpts, gcell, _ = oracle.point_grad(st, p, far, np.ones((1, p.n_features)))
    assert np.all(gpos == 0.0) and np.all(gpts == 0.0)


def test_point_invariances():
    rng = np.random.default_rng(6)
    pos, spec, cell, pbc = gs.small_periodic(rng, n_atoms=8, density=0.05, dmin=1.4)
    p = _probes(7)
    pts = rng.uniform(0, 1, (5, 3)) @ cell
    F0 = oracle.point_features((pos, spec, cell, pbc), p, pts)
    moved = pts + np.array([1, -2, 0]) @ cell
    assert np.allclose(oracle.point_features((pos, spec, cell, pbc), p, moved), F0, rtol=1e-12, atol=0)
    Q, R = np.linalg.qr(rng.normal(size=(3, 3)))
    Q = Q * np.sign(np.diag(R))
    F1 = oracle.point_features((pos @ Q.T, spec, cell @ Q.T, pbc), p, pts @ Q.T)
    scale = np.abs(F0).max(axis=0, keepdims=True)
    assert np.all(np.abs(F1 - F0) <= 1e-10 * scale + 1e-14 * np.abs(F0))


def _fd_points(struct, p, pts, G, occupancy=None, h=1e-5):
    pos, spec, cell, pbc = struct
    gpos, gpts, gcell, F = oracle.point_grad(struct, p, pts, G, occupancy=occupancy)
    pairs = oracle.point_frozen_pairs(struct, p, pts)
    L0 = oracle.point_loss_frozen(struct, p, pts, G, pairs, occupancy=occupancy)
    assert L0 == pytest.approx(float(np.sum(G * F)), rel=1e-12)
    scale = max(np.abs(gpos).max(), np.abs(gpts).max(), np.abs(gcell).max())

    def L(ps, pt, c):
        return oracle.point_loss_frozen((ps, spec, c, pbc), p, pt, G, pairs, occupancy=occupancy)
    for i in range(len(pos)):
        for k in range(3):
            p1 = pos.copy(); p1[i, k] += h
            p2 = pos.copy(); p2[i, k] -= h
            assert abs((L(p1, pts, cell) - L(p2, pts, cell)) / (2 * h) - gpos[i, k]) <= 1e-6 * scale
    for r in range(len(pts)):
        for k in range(3):
            q1 = pts.copy(); q1[r, k] += h
            q2 = pts.copy(); q2[r, k] -= h
            assert abs((L(pos, q1, cell) - L(pos, q2, cell)) / (2 * h) - gpts[r, k]) <= 1e-6 * scale
    if pbc:
        for a in range(3):
            for k in range(3):
                c1 = cell.copy(); c1[a, k] += h
                c2 = cell.copy(); c2[a, k] -= h
                assert abs((L(pos, pts, c1) - L(pos, pts, c2)) / (2 * h) - gcell[a, k]) <= 1e-6 * scale
    # a common translation of atoms and points changes nothing
    tot = gpos.sum(axis=0) + gpts.sum(axis=0)
    assert np.abs(tot).max() <= 1e-11 * scale * (len(pos) + len(pts))


def test_point_grad_fd_periodic():
    rng = np.random.default_rng(8)
    st = gs.small_periodic(rng, n_atoms=5, density=0.05, dmin=1.4)
    p = _probes(9, tau=1e-7, n_sigmas=2)
    pts = rng.uniform(0, 1, (3, 3)) @ st[2] + np.array([0.0, 0.0, -4.0])  # one outside the home cell
    _fd_points(st, p, pts, rng.standard_normal((3, p.n_features)))


def test_point_grad_fd_cluster_with_occupancy():
    rng = np.random.default_rng(10)
    st, occ = gs.disorder(rng, gs.small_cluster(rng, n_atoms=5, radius=2.5), n_elements=2)
    p = _probes(11, tau=1e-7, n_sigmas=2)
    pts = rng.normal(size=(3, 3)) * 1.5
    _fd_points(st, p, pts, rng.standard_normal((3, p.n_features)), occupancy=occ)
