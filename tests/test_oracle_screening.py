"""Pins of the oracle's per-primitive screening mode (a primitive contributes
to a slot only where its own l=0 overlap reaches the threshold tau; the
speed variant of the cutoff rule):

* the error bound against the unscreened function: every skipped term of a
  radial factor is below tau, so |mu_screened - mu| <= tau sum |P_c(d)| over
  the skipped (pair, primitive) terms, and the weighted norm inherits it;
* with one element of one primitive the screening radius is the slot
  cutoff, so nothing changes;
* the dimer closed form with the rule applied per primitive;
* the analytic gradient against finite differences.
"""
import math

import numpy as np
import pytest

import gmp_synth as gs
import oracle


def _screened(p, on=True):
    return gs.Probes(p.orders, p.sigmas, p.prim_offsets, p.B, p.beta, p.tau, screening=on)


def _radius2(A0, gam, tau):
    return np.where(A0 > tau, np.log(np.maximum(A0, 1e-300) / tau) / gam, -1.0)


def test_screening_error_bound():
    rng = np.random.default_rng(1)
    st = gs.small_periodic(rng, n_atoms=8, n_elements=2, density=0.06, dmin=1.2)
    p = gs.small_probes(rng, orders=(-1, 0, 1, 2, 3, 4), n_sigmas=3, n_elements=2, n_prims=(3, 5), tau=1e-4,
                        beta_range=(0.2, 20.0))
    F0 = oracle.features(st, p)
    F1 = oracle.features(st, _screened(p))
    assert not np.array_equal(F0, F1)  # the screening skips something here
    pos, spec, cell, pbc = st
    rw, m = oracle.wrap(pos, cell, pbc)
    rc2 = oracle.cutoffs(p)
    S = len(p.sigmas)
    for i in range(len(pos)):
        nb = oracle.neighbors(st, rc2, i)
        d = rw[nb["j"]] - rw[i] + nb["n"] @ cell
        f = 0
        for l in p.orders:
            if l == -1:
                skipped = 0
                for q, e in zip(nb["q"], nb["e"]):
                    if q > rc2[S]:
                        continue
                    sl = slice(p.prim_offsets[e], p.prim_offsets[e + 1])
                    thr = _radius2(np.abs(p.B[sl]), p.beta[sl], p.tau)
                    skipped += int(np.sum(np.float32(q) > thr.astype(np.float32)))
                assert abs(F1[i, f] - F0[i, f]) <= p.tau * skipped * (1 + 1e-9) + 1e-15
                f += 1
                continue
            comps = oracle.components(l)
            w = np.array([math.factorial(l) / (math.factorial(a) * math.factorial(b) * math.factorial(c))
                          for a, b, c in comps])
            Pabs = np.abs(np.stack([oracle.solid_harmonic(*abc, d)[0] for abc in comps], 1))  # [pairs, comps]
            for s, sg in enumerate(p.sigmas):
                alpha = 1.0 / (2 * sg * sg)
                dmu = np.zeros(len(comps))
                for t, (q, e) in enumerate(zip(nb["q"], nb["e"])):
                    if q > rc2[s]:
                        continue
                    sl = slice(p.prim_offsets[e], p.prim_offsets[e + 1])
                    lam = alpha + p.beta[sl]
                    thr = _radius2(np.abs(p.B[sl]) * (alpha / lam) ** 1.5, alpha * p.beta[sl] / lam, p.tau)
                    nskip = int(np.sum(np.float32(q) > thr.astype(np.float32)))
                    dmu += p.tau * nskip * Pabs[t]
                bound = math.sqrt(float(np.sum(w * dmu * dmu)))
                assert abs(F1[i, f] - F0[i, f]) <= bound * (1 + 1e-9) + 1e-15, (i, l, s)
                f += 1


def test_one_primitive_is_unchanged():
    rng = np.random.default_rng(2)
    st = gs.small_periodic(rng, n_atoms=7, n_elements=1, density=0.05, dmin=1.3)
    p = gs.small_probes(rng, orders=(-1, 0, 2, 4), n_sigmas=3, n_elements=1, n_prims=(1, 1), tau=1e-8)
    assert np.allclose(oracle.features(st, _screened(p)), oracle.features(st, p), rtol=1e-15, atol=0)


def test_dimer_screened_closed_form():
    p = gs.Probes(np.array([0, -1], np.int32), np.array([0.3, 0.8]), np.array([0, 3], np.int32),
                  np.array([2.0, 0.7, 0.05]), np.array([25.0, 2.0, 0.3]), 1e-4, screening=True)
    r2 = 4.0 ** 2
    st = (np.array([[0.0, 0.0, 0.0], [4.0, 0.0, 0.0]]), np.zeros(2, np.int32), np.zeros((3, 3)), 0)
    F = oracle.features(st, p)
    skipped = []
    for s, sg in enumerate(p.sigmas):
        a = 1.0 / (2 * sg * sg)
        lam = a + p.beta
        A0 = p.B * (a / lam) ** 1.5
        gam = a * p.beta / lam
        thr = _radius2(np.abs(A0), gam, p.tau).astype(np.float32)
        self_t = np.sum(np.where(np.float32(0.0) <= thr, A0, 0.0))
        other = np.sum(np.where(np.float32(r2) <= thr, A0 * np.exp(-gam * r2), 0.0))
        assert F[0, s] == pytest.approx(abs(self_t + other), rel=1e-13)
        skipped.append(np.float32(r2) > thr)
    skipped = np.array(skipped)
    assert skipped.any() and not skipped.all()  # the rule takes some primitives and not others
    thr = _radius2(np.abs(p.B), p.beta, p.tau).astype(np.float32)
    dens = np.sum(np.where(np.float32(0.0) <= thr, p.B, 0.0)) + \
        np.sum(np.where(np.float32(r2) <= thr, p.B * np.exp(-p.beta * r2), 0.0))
    assert F[0, 2] == pytest.approx(dens, rel=1e-13)


def test_screened_grad_fd():
    rng = np.random.default_rng(3)
    st = gs.small_periodic(rng, n_atoms=5, n_elements=2, density=0.06, dmin=1.2)
    p = _screened(gs.small_probes(rng, orders=(-1, 0, 1, 2), n_sigmas=2, n_elements=2, n_prims=(3, 4),
                                  tau=1e-5, beta_range=(0.2, 20.0)))
    pos, spec, cell, pbc = st
    G = rng.standard_normal((5, p.n_features))
    gpos, gcell, F = oracle.grad(st, p, G)
    pairs = oracle.frozen_pairs(st, p)
    assert oracle.loss_frozen(st, p, G, pairs) == pytest.approx(float(np.sum(G * F)), rel=1e-12)
    scale = max(np.abs(gpos).max(), np.abs(gcell).max())
    h = 1e-5
    for i in range(5):
        for k in range(3):
            p1 = pos.copy(); p1[i, k] += h
            p2 = pos.copy(); p2[i, k] -= h
            fd = (oracle.loss_frozen((p1, spec, cell, pbc), p, G, pairs)
                  - oracle.loss_frozen((p2, spec, cell, pbc), p, G, pairs)) / (2 * h)
            assert abs(fd - gpos[i, k]) <= 1e-6 * scale
