"""Tabulated radial factors on the HIP path, against the exact oracle.

A tabulated plan reads c_{l,s,e} from cubic Hermite tables in r = sqrt(q)
whose error on the interval [r_lo, r_lo + h] is at most
eps = h^4/384 sum_k gamma_k^2 |A_{l,s,e,k}| envelope(gamma_k r_lo^2)
(pinned in test_tabulated_bound.py).  A component then moves by at most
sum_j eps |P_abc(d_j)| w_j and, by the addition theorem
(sum_abc l!/(a!b!c!) P_abc(d)^2 = (2l-1)!! l! r^{2l}), a feature by at most
sum_j eps_{s,e_j,l} sqrt((2l-1)!! l!) r_j^l w_j over the pairs of its slot.
Every feature must stay within that bound plus the FP32 bar (1e-5 relative
above the threshold, the threshold itself below it) of the exact oracle;
the gradient (exact radial factors over the tabulated forward's components)
within 1e-5 of the oracle's."""
import numpy as np
import pytest

import gmp_synth as gs
import oracle
from gpu_helpers import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_12980_amd as g
    g.load()
    return g


def _envelope(u_lo):
    # max over u >= u_lo of |16 u^2 - 48 u + 12| e^{-u} (pinned in test_tabulated_bound.py)
    return np.where(u_lo < 4.2, 12.0, (16 * u_lo ** 2 - 48 * u_lo + 12) * np.exp(-u_lo))


def _eps(p, n, s, e, l, q):
    """Interpolation bound of c_{l,s,e} at squared distances q with n
    intervals (slot s; the density slot after the sigmas), on the interval
    that holds each q: h^4/384 sum_k gamma_k^2 |A_k| envelope(gamma_k r_lo^2)."""
    rc = np.sqrt(oracle.cutoffs(p))
    h = rc[s] / n
    Bk = p.B[p.prim_offsets[e]:p.prim_offsets[e + 1]]
    bk = p.beta[p.prim_offsets[e]:p.prim_offsets[e + 1]]
    if s >= len(p.sigmas):  # density: B exp(-beta q)
        if l != 0:
            return np.zeros_like(q)
        gam, A = bk, Bk
    else:
        alpha = 1.0 / (2 * p.sigmas[s] ** 2)
        lam = alpha + bk
        gam = alpha * bk / lam
        A = Bk * (alpha / lam) ** 1.5 * (bk / lam) ** l
    r_lo = np.floor(np.sqrt(q) / h) * h
    return h ** 4 / 384 * (np.abs(A) * gam ** 2 * _envelope(np.outer(r_lo ** 2, gam))).sum(1)


def feature_bounds(struct, p, n, centres, occupancy=None):
    """[len(centres), nf] bound of |F_tab - F_exact| from the oracle's lists."""
    rc2 = oracle.cutoffs(p)
    nb = oracle.neighbors_many(struct, rc2, centres)
    S = len(p.sigmas)
    occ = np.ones(len(struct[0])) if occupancy is None else np.asarray(occupancy)
    out = np.zeros((len(centres), p.n_features))
    owner = np.repeat(np.arange(len(centres)), np.diff(nb["offs"]))
    q, e, w = nb["q"], nb["e"], occ[nb["j"]]
    f = 0
    for l in p.orders:
        l = int(l)
        ll = max(l, 0)
        scale = np.sqrt(np.prod(np.arange(2 * ll - 1, 0, -2)) * np.prod(np.arange(1, ll + 1)))
        for s in ([S] if l == -1 else range(S)):
            eps = np.zeros_like(q)
            for ee in range(p.n_elements):
                sel = e == ee
                eps[sel] = _eps(p, n, s, ee, ll, q[sel])
            term = np.where(q <= rc2[s], eps * scale * q ** (ll / 2) * w, 0.0)
            out[:, f] = np.bincount(owner, weights=term, minlength=len(centres))
            f += 1
    return out


def _check(F, Fref, bound, tau):
    err = np.abs(F - Fref)
    allow = bound + np.where(Fref > tau, 1e-5 * Fref, tau)
    assert np.all(err <= allow), float((err / allow).max())
    return float((err / np.maximum(bound + 1e-300, 1e-300)).max()), float(bound.max())


@pytest.mark.parametrize("prec,n", [("fp32c", 512), ("fp32w", 512), ("fp32c", 4096)])
def test_tabulated_small_batch(g, prec, n):
    rng = np.random.default_rng(81)
    structs = [gs.small_periodic(rng, n_atoms=20, n_elements=3, density=0.06, dmin=1.3),
               gs.small_cluster(rng, n_atoms=9, n_elements=3, radius=3.0),
               gs.small_periodic(rng, n_atoms=4, n_elements=3, density=0.08, dmin=1.0)]
    occ = [rng.uniform(0.5, 1.0, len(st[0])) for st in structs]
    b = gs.make_batch(structs, occupancy=occ)
    p0 = gs.small_probes(rng, orders=(-1, 0, 1, 2, 3, 4), n_sigmas=3, n_elements=3, n_prims=(2, 6), tau=1e-9)
    p = gs.Probes(p0.orders, p0.sigmas, p0.prim_offsets, p0.B, p0.beta, p0.tau, radial_intervals=n)
    plan = g.GMPPlan.from_probes(p, prec)
    db = g.DeviceBatch.from_batch(b)
    ws = g.Workspace()
    nb = g.build_neighbors(plan, db, ws)
    F, mu = g.features(plan, db, nb, ws)
    G = torch.as_tensor(rng.standard_normal((b.n_atoms, p.n_features)), device="cuda")
    gp, gc = g.features_backward(plan, db, nb, ws, mu, F, G)
    F, gp, gc = F.double().cpu().numpy(), gp.cpu().numpy(), gc.cpu().numpy()
    worst = 0.0
    for s in range(b.n_structs):
        a0, a1 = int(b.atom_offsets[s]), int(b.atom_offsets[s + 1])
        st = b.structure(s)
        rp, rcell, Fref = oracle.grad(st, p0, G.cpu().numpy()[a0:a1], occupancy=occ[s])
        bound = feature_bounds(st, p0, n, np.arange(a1 - a0), occupancy=occ[s])
        r, bmax = _check(F[a0:a1], Fref, bound, p.tau)
        scale = max(np.abs(rp).max(), np.abs(rcell).max())
        e = max(np.abs(gp[a0:a1] - rp).max(), np.abs(gc[s] - rcell).max()) / scale
        say(f"[tabulated {prec} n={n}] structure {s}: max bound {bmax:.2e}, gradient error {e:.2e}")
        assert e <= 1e-5
        worst = max(worst, bmax)


def test_tabulated_full_size_sampled(g):
    b, p0 = gs.config("C2")
    n = 2048
    p = gs.Probes(p0.orders, p0.sigmas, p0.prim_offsets, p0.B, p0.beta, p0.tau, radial_intervals=n)
    cs = np.sort(np.random.default_rng(83).choice(b.n_atoms, 24, replace=False)).astype(np.int32)
    Fref = oracle.features(b.structure(0), p0, centres=cs)
    bound = feature_bounds(b.structure(0), p0, n, cs)
    for prec in ("fp32c", "fp32w"):
        plan = g.GMPPlan.from_probes(p, prec)
        db = g.DeviceBatch.from_batch(b)
        ws = g.Workspace()
        nb = g.build_neighbors(plan, db, ws, reverse=False)
        F, _ = g.features(plan, db, nb, ws)
        Fn = F.double().cpu().numpy()[cs]
        _check(Fn, Fref, bound, p.tau)
        big = Fref > p.tau
        rel = float(np.max(np.abs(Fn[big] - Fref[big]) / Fref[big]))
        say(f"[tabulated C2 {prec}] max rel {rel:.2e}, max bound / F {float(np.max(bound[big] / Fref[big])):.2e}")
        del nb, F
        torch.cuda.empty_cache()
