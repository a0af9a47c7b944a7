"""Pins of the oracle's conditioning reference F_abs (the feature built from
the absolute values of the pair terms; kappa = F_abs / F attributes an FP32
error to cancellation): it equals F where no term can cancel, bounds F from
above everywhere, and stays positive where symmetry makes F vanish."""
import numpy as np

import gmp_synth as gs
import oracle


def _probes(seed, orders=(0, 1, 2, 3)):
    p = gs.small_probes(np.random.default_rng(seed), orders=orders, n_sigmas=2, n_elements=2, n_prims=(1, 3),
                        tau=1e-8)
    return gs.Probes(p.orders, p.sigmas, p.prim_offsets, np.abs(p.B), p.beta, p.tau)


def test_order_zero_with_positive_weights_has_no_cancellation():
    rng = np.random.default_rng(1)
    struct = gs.small_periodic(rng, n_atoms=6, density=0.05, dmin=1.4)
    p = _probes(2)
    F = oracle.features(struct, p)
    Fa = oracle.features_abs(struct, p)
    S = len(p.sigmas)
    # order 0 comes first: every term B (a/l)^1.5 e^{-gq} is positive
    assert np.array_equal(Fa[:, :S], F[:, :S])
    assert np.all(Fa >= F * (1 - 1e-15))


def test_isolated_atom_and_symmetric_site():
    p = _probes(3)
    one = (np.zeros((1, 3)), np.zeros(1, np.int32), np.zeros((3, 3)), 0)
    assert np.array_equal(oracle.features_abs(one, p), oracle.features(one, p))
    # simple cubic, one atom per cell: F_1 vanishes by symmetry, F_abs does not
    a = 3.0
    sc = (np.zeros((1, 3)), np.zeros(1, np.int32), np.eye(3) * a, 7)
    F = oracle.features(sc, p)
    Fa = oracle.features_abs(sc, p)
    S = len(p.sigmas)
    assert np.all(F[:, S:2 * S] <= 1e-13 * F[:, :S])
    assert np.all(Fa[:, S:2 * S] > 1e-3 * Fa[:, :S])


def test_restricted_centres_match_full():
    rng = np.random.default_rng(4)
    struct = gs.small_cluster(rng, n_atoms=7, radius=3.0)
    p = _probes(5)
    full = oracle.features_abs(struct, p)
    cs = [6, 2, 3]
    assert np.array_equal(oracle.features_abs(struct, p, centres=cs), full[cs])
