"""The interpolation bound of the tabulated radial factors (CPU).

A tabulated plan replaces c_{l,s,e}(q) = sum_k A_k exp(-gamma_k q) with a
cubic Hermite interpolant in r = sqrt(q) on equal intervals of width h
(values and r-derivatives at both ends).  The interpolation error of a
cubic Hermite interpolant is at most h^4/384 max|f''''|, and the fourth
r-derivative of exp(-gamma r^2), gamma^2 (16 u^2 - 48 u + 12) e^{-u} with
u = gamma r^2, is at most 12 gamma^2 in magnitude (its value at r = 0), so
|c - p| <= h^4/32 sum_k gamma_k^2 |A_k|; on the interval [r_lo, r_lo + h] the
fourth derivative is also at most gamma^2 envelope(gamma r_lo^2) (the
function is decreasing beyond u = 4.2), a much smaller local bound for the
far pairs of diffuse slots.  These tests check both bounds by
dense sampling of the interpolant built the same way, for the probe shapes
of the workloads, and the validation of the plan field."""
import ctypes

import numpy as np
import pytest

import gmp_synth as gs
import oracle


def hermite_table(f, df, rc, n):
    """Coefficients (in t = (r - r_k)/h) of the cubic Hermite interpolant of f
    on n equal intervals of [0, rc]."""
    h = rc / n
    r = np.arange(n + 1) * h
    f0, f1, d0, d1 = f(r[:-1]), f(r[1:]), df(r[:-1]), df(r[1:])
    return h, np.stack([f0, h * d0, 3 * (f1 - f0) - h * (2 * d0 + d1), 2 * (f0 - f1) + h * (d0 + d1)], 1)


def evaluate(h, coef, r):
    k = np.minimum((r / h).astype(int), len(coef) - 1)
    t = r / h - k
    a = coef[k]
    return ((a[:, 3] * t + a[:, 2]) * t + a[:, 1]) * t + a[:, 0]


def envelope(u_lo):
    """max over u >= u_lo of |16 u^2 - 48 u + 12| e^{-u}: 12 (its value at 0)
    up to u = 4.2, beyond which the function is positive and decreasing."""
    u_lo = np.asarray(u_lo, float)
    return np.where(u_lo < 4.2, 12.0, (16 * u_lo ** 2 - 48 * u_lo + 12) * np.exp(-u_lo))


def test_envelope_of_the_fourth_derivative():
    u = np.linspace(0, 60, 600001)
    g4 = np.abs(16 * u ** 2 - 48 * u + 12) * np.exp(-u)
    tail_max = np.maximum.accumulate(g4[::-1])[::-1]  # max over u' >= u
    assert np.all(tail_max <= envelope(u) * (1 + 1e-12))
    assert tail_max[0] == pytest.approx(12.0)


def test_fourth_derivative_bound_of_a_gaussian():
    # max over r of |d^4/dr^4 exp(-g r^2)| = 12 g^2, at r = 0
    for g in (0.05, 1.0, 19.0):
        u = np.linspace(0, 40, 400001)
        d4 = g ** 2 * (16 * u ** 2 - 48 * u + 12) * np.exp(-u)
        assert np.abs(d4).max() == pytest.approx(12 * g ** 2, rel=1e-12)


@pytest.mark.parametrize("name", ["C1", "C2", "C5"])
def test_interpolation_error_within_bound(name):
    b, p = gs.config(name, n_atoms=64) if name in ("C2", "C5") else gs.config(name)
    rc = np.sqrt(oracle.cutoffs(p))
    rng = np.random.default_rng(3)
    for s in range(len(p.sigmas)):
        alpha = 1.0 / (2 * p.sigmas[s] ** 2)
        for e in range(p.n_elements):
            Bk = p.B[p.prim_offsets[e]:p.prim_offsets[e + 1]]
            bk = p.beta[p.prim_offsets[e]:p.prim_offsets[e + 1]]
            lam = alpha + bk
            gam = alpha * bk / lam
            for l in (0, 2, 4):
                A = Bk * (alpha / lam) ** 1.5 * (bk / lam) ** l
                f = lambda r: np.exp(-np.outer(r * r, gam)) @ A
                df = lambda r: (np.exp(-np.outer(r * r, gam)) * (-2 * np.outer(r, gam))) @ A
                for n in (256, 2048):
                    h, coef = hermite_table(f, df, rc[s], n)
                    r = np.sort(rng.uniform(0, rc[s], 20000))
                    err = np.abs(evaluate(h, coef, r) - f(r)).max()
                    bound = h ** 4 / 32 * np.sum(gam ** 2 * np.abs(A))
                    assert err <= bound * (1 + 1e-9) + 1e-15 * np.abs(A).sum(), (name, s, e, l, n, err, bound)
                    # the interval-local bound: h^4/384 sum_k gamma_k^2 |A_k| envelope(gamma_k r_lo^2)
                    r_lo = np.floor(r / h) * h
                    local = h ** 4 / 384 * (np.abs(A) * gam ** 2 * envelope(np.outer(r_lo ** 2, gam))).sum(1)
                    ev = np.abs(evaluate(h, coef, r) - f(r))
                    assert np.all(ev <= local * (1 + 1e-9) + 1e-15 * np.abs(A).sum())
                    # the values at the radial factor's own reference points
                    assert np.allclose(evaluate(h, coef, np.array([0.0, rc[s]])), f(np.array([0.0, rc[s]])),
                                       rtol=1e-12, atol=0)


def test_radial_intervals_validation():
    from paper_2303_12980_amd import _lib
    L = _lib.load()
    p = gs.small_probes(np.random.default_rng(1), n_sigmas=2)
    keep = [np.ascontiguousarray(p.orders, np.int32), np.ascontiguousarray(p.sigmas, np.float64),
            np.ascontiguousarray(p.prim_offsets, np.int32), np.ascontiguousarray(p.B), np.ascontiguousarray(p.beta)]
    d = _lib.ProbeDesc(len(keep[0]), keep[0].ctypes.data_as(_lib.P_i32), len(keep[1]),
                       keep[1].ctypes.data_as(_lib.P_dbl), len(keep[2]) - 1, keep[2].ctypes.data_as(_lib.P_i32),
                       keep[3].ctypes.data_as(_lib.P_dbl), keep[4].ctypes.data_as(_lib.P_dbl), p.tau, 0, 0)
    rc2 = np.zeros(4)
    call = lambda: L.gmp_probe_cutoffs(ctypes.byref(d), rc2.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    for n, code in ((0, 0), (16, 0), (65536, 0), (8, 1), (-1, 1), (65537, 1)):
        d.radial_intervals = n
        assert call() == code, n
    d.radial_intervals, d.screening = 64, 1
    assert call() == _lib.GMP_E_UNSUPPORTED
