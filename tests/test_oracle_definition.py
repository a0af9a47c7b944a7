"""Pins of the FP64 oracle against things other than itself.

* the solid harmonics against their derivative definition (sympy) and
  against harmonicity (numerical Laplacian);
* the closed-form overlap against brute-force 3-D quadrature of the
  defining integral (probe Gaussian x angular probe x density primitives);
* the isolated-atom and dimer closed forms;
* the Legendre addition-theorem form of the rotation-invariant norm;
* the cutoff rule (every primitive's l=0 overlap at rc is <= tau, with
  equality for the defining primitive).
"""
import math

import numpy as np
import pytest
import sympy as sp
from scipy.special import eval_legendre

import gmp_synth as gs
import oracle


def _sym_harmonic(a, b, c):
    """(-1)^l |u|^(2l+1) d^a_x d^b_y d^c_z (1/|u|) as a sympy polynomial."""
    x, y, z = sp.symbols("x y z", real=True)
    r = sp.sqrt(x * x + y * y + z * z)
    l = a + b + c
    expr = 1 / r
    if a:
        expr = sp.diff(expr, x, a)
    if b:
        expr = sp.diff(expr, y, b)
    if c:
        expr = sp.diff(expr, z, c)
    poly = sp.simplify(sp.expand(sp.simplify((-1) ** l * r ** (2 * l + 1) * expr)))
    return (x, y, z), sp.expand(poly)


ALL_ABC = [abc for l in range(5) for abc in oracle.components(l)]


@pytest.fixture(scope="module")
def sym_polys():
    return {abc: _sym_harmonic(*abc) for abc in ALL_ABC}


@pytest.mark.parametrize("abc", ALL_ABC)
def test_solid_harmonic_matches_derivative_definition(abc, sym_polys):
    (x, y, z), poly = sym_polys[abc]
    assert poly.is_polynomial(x, y, z)
    f = sp.lambdify((x, y, z), poly, "numpy")
    grads = [sp.lambdify((x, y, z), sp.diff(poly, v), "numpy") for v in (x, y, z)]
    rng = np.random.default_rng(sum(abc) * 7 + abc[0])
    pts = rng.normal(size=(40, 3)) * 2.0
    v, g = oracle.solid_harmonic(*abc, pts)
    ref = np.broadcast_to(np.asarray(f(pts[:, 0], pts[:, 1], pts[:, 2]), float), (len(pts),))
    scale = np.linalg.norm(pts, axis=1) ** sum(abc)
    assert np.allclose(v, ref, rtol=1e-12, atol=1e-12 * scale.max())
    for k in range(3):
        gr = np.broadcast_to(np.asarray(grads[k](pts[:, 0], pts[:, 1], pts[:, 2]), float), (len(pts),))
        assert np.allclose(g[:, k], gr, rtol=1e-11, atol=1e-11 * scale.max())


@pytest.mark.parametrize("abc", ALL_ABC)
def test_solid_harmonic_is_harmonic(abc):
    """Laplacian by a 4th-order central stencil vanishes; degree-l homogeneity."""
    rng = np.random.default_rng(11)
    pts = rng.normal(size=(10, 3))
    h = 1e-2
    lap = np.zeros(len(pts))
    for k in range(3):
        e = np.zeros(3); e[k] = h
        vals = [oracle.solid_harmonic(*abc, pts + s * e)[0] for s in (-2, -1, 0, 1, 2)]
        lap += (-vals[0] + 16 * vals[1] - 30 * vals[2] + 16 * vals[3] - vals[4]) / (12 * h * h)
    v0 = oracle.solid_harmonic(*abc, pts)[0]
    l = sum(abc)
    assert np.all(np.abs(lap) < 1e-6 * max(1.0, np.abs(v0).max()) * 10 ** l)
    # homogeneity P(t u) = t^l P(u)
    v2 = oracle.solid_harmonic(*abc, 1.7 * pts)[0]
    assert np.allclose(v2, 1.7 ** l * v0, rtol=1e-12, atol=1e-13)


def _quadrature_mu(centre, others, sigmas, B, beta, sym_polys, half=5.5, h=0.08):
    """Trapezoid quadrature of int rho(r) P_abc(r-Ri) G_sigma(r-Ri) d^3r on a
    uniform grid centred on the centre atom; rho sums every listed atom's
    primitives (the centre included).  The integrand is a sum of Gaussians
    times polynomials, for which the uniform trapezoid rule converges
    spectrally.  Returns {(l, sigma index): components of order l}."""
    ax = np.arange(-half, half + h / 2, h)
    X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
    rr = X * X + Y * Y + Z * Z
    rho = np.zeros_like(X)
    for (R, Bk, bk) in [(np.zeros(3), B[0], beta[0])] + [(o - centre, B[i + 1], beta[i + 1]) for i, o in enumerate(others)]:
        d2 = (X - R[0]) ** 2 + (Y - R[1]) ** 2 + (Z - R[2]) ** 2
        for b_, be_ in zip(Bk, bk):
            rho += b_ * np.exp(-be_ * d2)
    ws = [(2 * math.pi * sg * sg) ** -1.5 * np.exp(-rr / (2 * sg * sg)) * rho * h ** 3 for sg in sigmas]
    out = {}
    for l in range(5):
        for s in range(len(sigmas)):
            out[(l, s)] = []
        for abc in oracle.components(l):
            (x, y, z), poly = sym_polys[abc]
            f = sp.lambdify((x, y, z), poly, "numpy")
            P = np.broadcast_to(np.asarray(f(X, Y, Z), float), X.shape)
            for s in range(len(sigmas)):
                out[(l, s)].append(float(np.sum(ws[s] * P)))
    return {k: np.array(v) for k, v in out.items()}


def test_closed_form_matches_quadrature(sym_polys):
    """Three isolated atoms, two elements; every component of l <= 4 at two
    widths, against direct quadrature of the defining integral."""
    pos = np.array([[0.0, 0.0, 0.0], [0.7, -0.4, 1.1], [-0.9, 0.5, 0.3]])
    spec = np.array([0, 1, 0], np.int32)
    offs = np.array([0, 2, 3], np.int32)
    B = np.array([1.7, -0.4, 0.9])
    beta = np.array([0.9, 2.5, 1.6])
    sigmas = np.array([0.45, 0.6])
    probes = gs.Probes(np.arange(5, dtype=np.int32), sigmas, offs, B, beta, 1e-30)
    F, mu = oracle.features((pos, spec, np.zeros((3, 3)), 0), probes, centres=[0], with_mu=True)
    per_atom_B = [B[offs[e]:offs[e + 1]] for e in spec]
    per_atom_beta = [beta[offs[e]:offs[e + 1]] for e in spec]
    quad = _quadrature_mu(pos[0], pos[1:], sigmas, per_atom_B, per_atom_beta, sym_polys)
    off = 0
    for l in range(5):
        nc = len(oracle.components(l))
        for s, sg in enumerate(sigmas):
            ref = quad[(l, s)]
            got = mu[0, off + s * nc: off + (s + 1) * nc]
            scale = np.abs(ref).max()
            assert np.allclose(got, ref, rtol=1e-9, atol=1e-10 * scale), (l, sg, got, ref)
        off += len(sigmas) * nc


def test_isolated_atom():
    """One atom in vacuum: F_0 = sum_k B (alpha/(alpha+beta))^(3/2) (Gaussian
    product at zero separation), F_{l>=1} = 0."""
    rng = np.random.default_rng(3)
    probes = gs.small_probes(rng, n_elements=1, n_prims=4, tau=1e-12)
    F = oracle.features((np.zeros((1, 3)), np.zeros(1, np.int32), np.zeros((3, 3)), 0), probes)
    S = len(probes.sigmas)
    for s, sg in enumerate(probes.sigmas):
        a = 1 / (2 * sg * sg)
        ref = abs(np.sum(probes.B * (a / (a + probes.beta)) ** 1.5))
        assert F[0, s] == pytest.approx(ref, rel=1e-13)
    assert np.all(F[0, S:] == 0.0)


def test_dimer_closed_form():
    """Two atoms in vacuum at distance r: F_l = sqrt((2l-1)!! l!) |c_l(r^2)| r^l
    for l >= 1 (the centre's own term has no l >= 1 part)."""
    rng = np.random.default_rng(5)
    probes = gs.small_probes(rng, n_elements=2, n_prims=3, tau=1e-14)
    u = rng.normal(size=3); u /= np.linalg.norm(u)
    r = 1.9
    pos = np.stack([np.zeros(3), r * u])
    spec = np.array([0, 1], np.int32)
    F = oracle.features((pos, spec, np.zeros((3, 3)), 0), probes)
    S = len(probes.sigmas)
    Bj = probes.B[probes.prim_offsets[1]:probes.prim_offsets[2]]
    bj = probes.beta[probes.prim_offsets[1]:probes.prim_offsets[2]]
    for o, l in enumerate(probes.orders):
        if l == 0:
            continue
        dfact = float(np.prod(np.arange(2 * l - 1, 0, -2)))
        for s, sg in enumerate(probes.sigmas):
            c = oracle.radial(l, sg, Bj, bj, [r * r])[0]
            ref = math.sqrt(dfact * math.factorial(l)) * abs(c) * r ** l
            assert F[0, o * S + s] == pytest.approx(ref, rel=1e-12)


def test_addition_theorem_form():
    """F_l^2 = (2l-1)!! l! sum_{j,j'} g_j g_j' P_l(cos theta_jj'), g_j = c_l(r_j^2) r_j^l:
    an O(n^2) component-free second algorithm for the same norm."""
    rng = np.random.default_rng(9)
    probes = gs.small_probes(rng, n_elements=2, n_prims=(2, 3), tau=1e-14)
    struct = gs.small_cluster(rng, n_atoms=7, radius=2.6, dmin=1.1)
    pos, spec = struct[0], struct[1]
    F = oracle.features(struct, probes)
    S = len(probes.sigmas)
    for i in range(len(pos)):
        d = np.delete(pos, i, axis=0) - pos[i]
        e = np.delete(spec, i)
        r = np.linalg.norm(d, axis=1)
        cos = np.clip((d @ d.T) / np.outer(r, r), -1, 1)
        for o, l in enumerate(probes.orders):
            if l == 0:
                continue
            dfact = float(np.prod(np.arange(2 * l - 1, 0, -2)))
            for s, sg in enumerate(probes.sigmas):
                g = np.array([oracle.radial(l, sg, probes.B[probes.prim_offsets[ee]:probes.prim_offsets[ee + 1]],
                                            probes.beta[probes.prim_offsets[ee]:probes.prim_offsets[ee + 1]],
                                            [rr * rr])[0] * rr ** l for ee, rr in zip(e, r)])
                ref2 = dfact * math.factorial(l) * g @ eval_legendre(l, cos) @ g
                assert F[i, o * S + s] ** 2 == pytest.approx(ref2, rel=1e-11, abs=1e-24)


def test_cutoff_rule():
    """At rc(sigma) every primitive's l=0 overlap is <= tau and the defining
    one equals tau; beyond the rc of all sigmas nothing is a neighbour."""
    rng = np.random.default_rng(21)
    b, probes = gs.config("C2", n_atoms=64)
    rc2 = oracle.cutoffs(probes)
    for s, sg in enumerate(probes.sigmas):
        vals = []
        for k in range(len(probes.B)):
            vals.append(abs(oracle.radial(0, sg, probes.B[k:k + 1], probes.beta[k:k + 1], [rc2[s]])[0]))
        vals = np.array(vals)
        assert np.all(vals <= probes.tau * (1 + 1e-9))
        assert vals.max() == pytest.approx(probes.tau, rel=1e-9)
