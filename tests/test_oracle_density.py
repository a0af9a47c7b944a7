"""Pins of the oracle's order -1 feature (the local density at the centre,
one feature without a width; paper, section "Examples") against things
other than its own formula:

* the cutoff: every primitive's density at rc_{-1} is <= tau, with equality
  for the defining primitive, and rc_{-1} is the sigma -> 0 limit of the
  per-sigma cutoff rule;
* closed forms: an isolated atom (the self term only) and a dimer;
* the sigma -> 0 limit of the order-0 feature (the probe Gaussian tends to a
  delta function), which is itself pinned by quadrature;
* rotation, translation and supercell invariance;
* the analytic gradient against finite differences of the value.
"""
import numpy as np
import pytest

import gmp_synth as gs
import oracle


def _probes(seed, orders=(-1, 0, 2), n_sigmas=2, tau=1e-8):
    return gs.small_probes(np.random.default_rng(seed), orders=orders, n_sigmas=n_sigmas,
                           n_elements=2, n_prims=(1, 3), tau=tau)


def test_layout_counts():
    p = _probes(0, orders=(0, -1, 3), n_sigmas=3)
    assert oracle.n_features(p.orders, 3) == 7 == p.n_features
    assert oracle.n_components(p.orders, 3) == 3 * 1 + 1 + 3 * 10
    assert oracle.n_slots(p) == 4
    rc2 = oracle.cutoffs(p)
    assert rc2.shape == (4,)
    assert rc2[:3].tobytes() == oracle.sigma_cutoffs(p).tobytes()
    assert rc2[3] == oracle.density_cutoff(p)


def test_density_cutoff_is_threshold_crossing():
    p = _probes(1, tau=1e-9)
    rc2 = oracle.density_cutoff(p)
    vals = np.abs(p.B) * np.exp(-p.beta * rc2)
    assert np.all(vals <= p.tau * (1 + 1e-12))
    assert vals.max() == pytest.approx(p.tau, rel=1e-12)


def test_density_cutoff_is_small_sigma_limit():
    """rc(sigma)^2 -> rc_{-1}^2 as sigma -> 0 (A0 -> |B|, gamma -> beta)."""
    p = _probes(2, tau=1e-10)
    lim = oracle.density_cutoff(p)
    prev = None
    for sg in (1e-2, 1e-3, 1e-4):
        q = gs.Probes(np.array([0], np.int32), np.array([sg]), p.prim_offsets, p.B, p.beta, p.tau)
        err = abs(oracle.sigma_cutoffs(q)[0] - lim) / lim
        if prev is not None:
            assert err < prev * 0.02  # converges like sigma^2
        prev = err
    assert prev < 1e-7


def test_isolated_atom_density_is_sum_of_weights():
    p = _probes(3)
    for e in range(p.n_elements):
        struct = (np.array([[0.3, -0.2, 1.1]]), np.array([e], np.int32), np.zeros((3, 3)), 0)
        F = oracle.features(struct, p)
        lo, hi = p.prim_offsets[e], p.prim_offsets[e + 1]
        assert F[0, 0] == pytest.approx(abs(p.B[lo:hi].sum()), rel=1e-14)


@pytest.mark.parametrize("r", [0.9, 2.0, 3.5])
def test_dimer_density_closed_form(r):
    p = _probes(4, tau=1e-12)
    rc2 = oracle.density_cutoff(p)
    assert r * r <= rc2
    d = np.array([0.36, -0.48, 0.8]) * r
    struct = (np.array([[0.0, 0.0, 0.0], d]), np.array([0, 1], np.int32), np.zeros((3, 3)), 0)
    F = oracle.features(struct, p)
    for i, (ei, ej) in enumerate([(0, 1), (1, 0)]):
        si = slice(p.prim_offsets[ei], p.prim_offsets[ei + 1])
        sj = slice(p.prim_offsets[ej], p.prim_offsets[ej + 1])
        want = p.B[si].sum() + np.sum(p.B[sj] * np.exp(-p.beta[sj] * r * r))
        assert F[i, 0] == pytest.approx(want, rel=1e-13)


def test_dimer_beyond_density_cutoff_sees_only_itself():
    p = _probes(5, tau=1e-3)
    rc2 = oracle.density_cutoff(p)
    r = np.sqrt(rc2) * 1.01
    struct = (np.array([[0.0, 0.0, 0.0], [0.0, r, 0.0]]), np.array([0, 0], np.int32), np.zeros((3, 3)), 0)
    F = oracle.features(struct, gs.Probes(np.array([-1], np.int32), p.sigmas, p.prim_offsets, p.B, p.beta, p.tau))
    s0 = slice(p.prim_offsets[0], p.prim_offsets[1])
    assert F[0, 0] == pytest.approx(p.B[s0].sum(), rel=1e-14)


def test_density_is_order0_small_sigma_limit():
    """The order-0 probe with a normalised Gaussian of width sigma tends to
    the density at the centre as sigma -> 0; the error falls like sigma^2."""
    rng = np.random.default_rng(6)
    struct = gs.small_cluster(rng, n_atoms=7, radius=2.5)
    p = _probes(7, tau=1e-11)
    dens = oracle.features(struct, gs.Probes(np.array([-1], np.int32), p.sigmas, p.prim_offsets, p.B,
                                             p.beta, p.tau))[:, 0]
    errs = []
    for sg in (1e-2, 1e-3):
        q = gs.Probes(np.array([0], np.int32), np.array([sg]), p.prim_offsets, p.B, p.beta, p.tau)
        F0 = oracle.features(struct, q)[:, 0]
        errs.append(np.max(np.abs(F0 - dens) / dens))
    assert errs[1] < errs[0] * 0.02
    assert errs[1] < 1e-5


def _rot(seed):
    Q, R = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    return Q * np.sign(np.diag(R))


def test_density_invariances():
    p = _probes(8, orders=(-1,))
    pos, spec, cell, pbc = gs.small_periodic(np.random.default_rng(9), n_atoms=8, density=0.05, dmin=1.4)
    F0 = oracle.features((pos, spec, cell, pbc), p)
    Q = _rot(10)
    assert np.allclose(oracle.features((pos @ Q.T, spec, cell @ Q.T, pbc), p), F0, rtol=1e-12, atol=0)
    assert np.allclose(oracle.features((pos + np.array([1.7, -0.3, 4.0]), spec, cell, pbc), p), F0,
                       rtol=1e-12, atol=0)
    moved = pos.copy()
    moved[3] += cell[0] - 2 * cell[2]
    assert np.allclose(oracle.features((moved, spec, cell, pbc), p), F0, rtol=1e-12, atol=0)
    # 2x1x1 supercell: both copies of every atom see the primitive cell's density
    sup = np.concatenate([pos, pos + cell[0]])
    scell = cell.copy()
    scell[0] *= 2
    Fs = oracle.features((sup, np.concatenate([spec, spec]), scell, pbc), p)
    assert np.allclose(Fs, np.concatenate([F0, F0]), rtol=1e-12, atol=0)


def _fd(struct, probes, G, h=1e-5):
    pos, spec, cell, pbc = struct
    gpos, gcell, F = oracle.grad(struct, probes, G)
    pairs = oracle.frozen_pairs(struct, probes)
    assert oracle.loss_frozen(struct, probes, G, pairs) == pytest.approx(float(np.sum(G * F)), rel=1e-12)
    scale = max(np.abs(gpos).max(), np.abs(gcell).max())
    for i in range(len(pos)):
        for k in range(3):
            p1 = pos.copy(); p1[i, k] += h
            p2 = pos.copy(); p2[i, k] -= h
            fd = (oracle.loss_frozen((p1, spec, cell, pbc), probes, G, pairs)
                  - oracle.loss_frozen((p2, spec, cell, pbc), probes, G, pairs)) / (2 * h)
            assert abs(fd - gpos[i, k]) <= 1e-6 * scale, (i, k, fd, gpos[i, k])
    if pbc:
        for a in range(3):
            for k in range(3):
                c1 = cell.copy(); c1[a, k] += h
                c2 = cell.copy(); c2[a, k] -= h
                fd = (oracle.loss_frozen((pos, spec, c1, pbc), probes, G, pairs)
                      - oracle.loss_frozen((pos, spec, c2, pbc), probes, G, pairs)) / (2 * h)
                assert abs(fd - gcell[a, k]) <= 1e-6 * scale, (a, k, fd, gcell[a, k])


def test_density_grad_fd_periodic():
    rng = np.random.default_rng(11)
    struct = gs.small_periodic(rng, n_atoms=5, density=0.05, dmin=1.4)
    p = _probes(12, orders=(1, -1, 0), tau=1e-7)
    _fd(struct, p, rng.standard_normal((5, p.n_features)))


def test_density_only_grad_fd_cluster():
    rng = np.random.default_rng(13)
    struct = gs.small_cluster(rng, n_atoms=6, radius=2.5)
    p = _probes(14, orders=(-1,), tau=1e-7)
    _fd(struct, p, rng.standard_normal((6, p.n_features)))


def test_density_dimer_gradient_closed_form():
    """d rho_0 / d R_1 = sum_k B_k (-2 beta_k) e^{-beta_k r^2} (R_1 - R_0)."""
    p = _probes(15, orders=(-1,), tau=1e-12)
    d = np.array([0.5, 1.2, -0.7])
    struct = (np.array([[0.0, 0.0, 0.0], d]), np.array([0, 1], np.int32), np.zeros((3, 3)), 0)
    G = np.array([[1.0], [0.0]])
    gpos, _, _ = oracle.grad(struct, p, G)
    s1 = slice(p.prim_offsets[1], p.prim_offsets[2])
    r2 = d @ d
    want = np.sum(p.B[s1] * (-2 * p.beta[s1]) * np.exp(-p.beta[s1] * r2)) * d
    assert np.allclose(gpos[1], want, rtol=1e-13, atol=0)
    assert np.allclose(gpos[0], -want, rtol=1e-13, atol=0)
