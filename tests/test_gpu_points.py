"""Features at reference points (centres that are not atoms) on the HIP
path vs the FP64 oracle, through the C ABI: lists bit-exact, features to
the usual bars, a point on an atom bitwise equal to that atom's features,
gradients with respect to atoms, points and cell, bitwise-repeatable
backward."""
import numpy as np
import pytest

import gmp_synth as gs
import oracle
from gpu_helpers import say, assert_features

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {"fp64": 1e-11, "fp32c": 1e-5, "fp32w": 1e-5}
GTOL = {"fp64": 1e-11, "fp32c": 1e-5, "fp32w": 1e-5}


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_12980_amd as g
    g.load()
    return g


@pytest.fixture(scope="module")
def ws(g):
    return g.Workspace()


def _case(seed, orders=(-1, 0, 1, 2, 3, 4), occupancy=False):
    """Mixed batch and its reference points: inside and outside the home
    cell, on atoms, far from a cluster, and a structure without points."""
    rng = np.random.default_rng(seed)
    structs = [gs.small_periodic(rng, n_atoms=12, n_elements=3, density=0.06, dmin=1.3),
               gs.small_cluster(rng, n_atoms=8, n_elements=3, radius=3.0),
               gs.small_periodic(rng, n_atoms=9, n_elements=3, density=0.04, dmin=1.3, pbc=3),
               gs.small_periodic(rng, n_atoms=3, n_elements=3, density=0.08, dmin=1.0),
               gs.small_cluster(rng, n_atoms=4, n_elements=3, radius=2.0)]
    occs = None
    if occupancy:
        dis = [gs.disorder(rng, st, n_elements=3) for st in structs]
        structs, occs = [d[0] for d in dis], [d[1] for d in dis]
    b = gs.make_batch(structs, occupancy=occs)
    pts = []
    for s, (pos, spec, cell, pbc) in enumerate(structs):
        if s == 4:
            pts.append(np.zeros((0, 3)))
            continue
        if pbc:
            p = rng.uniform(-0.3, 1.3, (5, 3)) @ cell
        else:
            p = rng.normal(size=(5, 3)) * 2.0
        p = np.concatenate([p, pos[:2]])  # two points on atoms
        if s == 1:
            p = np.concatenate([p, [[60.0, 0.0, 0.0]]])  # beyond every cutoff
        pts.append(p)
    po = np.zeros(len(structs) + 1, np.int64)
    po[1:] = np.cumsum([len(p) for p in pts])
    probes = gs.small_probes(rng, orders=orders, n_sigmas=3, n_elements=3, n_prims=(1, 4), tau=1e-9)
    return b, np.concatenate(pts), po, probes


def _run(g, ws, b, pts, po, p, precision):
    plan = g.GMPPlan.from_probes(p, precision)
    db = g.DeviceBatch.from_batch(b).with_points(pts, po)
    nb = g.build_neighbors(plan, db, ws)
    F, mu = g.features(plan, db, nb, ws)
    torch.cuda.synchronize()
    return plan, db, nb, F, mu


def _check_point_lists(nb, b, pts, po, p):
    rc2 = oracle.cutoffs(p)
    E, S = p.n_elements, oracle.n_slots(p)
    offs = nb.offsets.cpu().numpy()
    assert int(offs[-1]) == nb.n_pairs
    NT = b.n_atoms + len(pts)
    wrap = nb.wrap.view(NT, 3).cpu().numpy()
    rw = nb.rw.view(3, NT).t().cpu().numpy()
    for s in range(b.n_structs):
        st = b.structure(s)
        a0 = int(b.atom_offsets[s])
        for c in range(int(po[s]), int(po[s + 1])):
            prw, pm = oracle.wrap(pts[c:c + 1], st[2], st[3])
            assert np.array_equal(wrap[b.n_atoms + c], pm[0])
            assert rw[b.n_atoms + c].tobytes() == prw[0].tobytes()
            ref = oracle.point_neighbors(st, rc2, pts[c])
            lo, hi = int(offs[c]), int(offs[c + 1])
            assert hi - lo == len(ref["j"]), (s, c)
            J = nb.j[lo:hi].cpu().numpy()
            w = nb.shift[lo:hi].cpu().numpy().view(np.uint8).reshape(-1, 4)
            assert np.array_equal(J, ref["j"] + a0)
            assert np.array_equal(w[:, :3].view(np.int8).astype(np.int32), ref["n"])
            assert np.array_equal(w[:, 3].astype(np.int32), ref["e"])
            bs = nb.bucket_start[c * (S * E + 1):(c + 1) * (S * E + 1)].cpu().numpy()
            se = nb.sigma_end[c * S:(c + 1) * S].cpu().numpy()
            bucket = ref["shell"] * E + ref["e"]
            assert np.array_equal(bs, np.searchsorted(np.sort(bucket), np.arange(S * E + 1), side="left"))
            assert np.array_equal(se, np.array([int(np.sum(ref["q"] <= rc2[t])) for t in range(S)]))


@pytest.mark.parametrize("precision", ["fp64", "fp32c", "fp32w"])
def test_point_lists_and_features(g, ws, precision):
    b, pts, po, p = _case(51)
    say(f"[reference points {precision}: {len(pts)} points, {b.n_atoms} atoms]")
    plan, db, nb, F, mu = _run(g, ws, b, pts, po, p, precision)
    assert F.shape == (len(pts), p.n_features)
    _check_point_lists(nb, b, pts, po, p)
    Fref, muref = oracle.point_features_batch(b, p, po, pts, with_mu=True)
    r, a = assert_features(F.cpu().numpy(), Fref, p.tau, TOL[precision])
    if precision == "fp64":
        scale = np.abs(muref).max(axis=0, keepdims=True)
        assert np.all(np.abs(mu.cpu().numpy() - muref) <= 1e-11 * scale + 1e-300)
    far = int(po[1]) + 7  # the point beyond every cutoff
    assert torch.all(F[far] == 0)
    say(f"  max rel {r:.2e}")


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_point_on_atom_bitwise_equals_atom(g, ws, precision):
    b, pts, po, p = _case(53)
    say(f"[point on atom {precision}]")
    _, _, _, Fp, _ = _run(g, ws, b, pts, po, p, precision)
    plan = g.GMPPlan.from_probes(p, precision)
    db = g.DeviceBatch.from_batch(b)
    nb = g.build_neighbors(plan, db, ws)
    Fa, _ = g.features(plan, db, nb, ws)
    for s in range(4):
        a0 = int(b.atom_offsets[s])
        c = int(po[s]) + 5  # the first of the two points placed on atoms 0, 1 of structure s
        assert torch.equal(Fp[c], Fa[a0]) and torch.equal(Fp[c + 1], Fa[a0 + 1])


@pytest.mark.parametrize("precision", ["fp64", "fp32c", "fp32w"])
@pytest.mark.parametrize("occupancy", [False, True])
def test_point_backward_vs_oracle(g, ws, precision, occupancy):
    b, pts, po, p = _case(55, orders=(-1, 0, 2, 3), occupancy=occupancy)
    say(f"[reference points backward {precision} occupancy={occupancy}]")
    plan, db, nb, F, mu = _run(g, ws, b, pts, po, p, precision)
    G = np.random.default_rng(56).standard_normal((len(pts), p.n_features))
    gp, gc = g.features_backward(plan, db, nb, ws, mu, F, torch.as_tensor(G, device="cuda"))
    gp2, gc2 = g.features_backward(plan, db, nb, ws, mu, F, torch.as_tensor(G, device="cuda"))
    assert torch.equal(gp, gp2) and torch.equal(gc, gc2)
    gp, gc = gp.cpu().numpy(), gc.cpu().numpy()
    N = b.n_atoms
    for s in range(b.n_structs):
        a0, a1 = int(b.atom_offsets[s]), int(b.atom_offsets[s + 1])
        c0, c1 = int(po[s]), int(po[s + 1])
        occ = None if b.occupancy is None else b.occupancy[a0:a1]
        rpos, rpts, rcell, _ = oracle.point_grad(b.structure(s), p, pts[c0:c1], G[c0:c1], occupancy=occ)
        scale = max(np.abs(rpos).max(initial=0), np.abs(rpts).max(initial=0), np.abs(rcell).max(initial=0))
        if scale == 0.0:
            assert np.all(gp[a0:a1] == 0) and np.all(gp[N + c0:N + c1] == 0) and np.all(gc[s] == 0)
            continue
        e1 = np.abs(gp[a0:a1] - rpos).max()
        e2 = np.abs(gp[N + c0:N + c1] - rpts).max(initial=0)
        e3 = np.abs(gc[s] - rcell).max()
        say(f"  struct {s}: atoms {e1 / scale:.2e} points {e2 / scale:.2e} cell {e3 / scale:.2e}")
        assert max(e1, e2, e3) <= GTOL[precision] * scale


def test_points_without_atoms(g, ws):
    """A structure with points but no atoms: empty lists, zero features."""
    rng = np.random.default_rng(57)
    cell = np.eye(3) * 8.0
    st = gs.small_periodic(rng, n_atoms=5, n_elements=2, density=0.05, dmin=1.3)
    b = gs.make_batch([(np.zeros((0, 3)), np.zeros(0, np.int32), cell, 7), st])
    pts = np.concatenate([rng.uniform(0, 8, (3, 3)), st[0][:1]])
    po = np.array([0, 3, 4], np.int64)
    p = gs.small_probes(rng, orders=(0, 1, 2), n_sigmas=2, n_elements=2, n_prims=(1, 2), tau=1e-8)
    plan, db, nb, F, mu = _run(g, ws, b, pts, po, p, "fp64")
    assert torch.all(F[:3] == 0)
    assert_features(F[3:].cpu().numpy(), oracle.point_features(st, p, pts[3:]), p.tau, TOL["fp64"])


def test_points_in_large_cell_multipass_sort(g, ws):
    """4096 atoms (the by-neighbour sort of the backward takes two radix
    passes) and a 4x4x4 grid of points: features and all gradients vs the
    oracle."""
    b, p = gs.config("C2")
    p = gs.Probes(np.array([-1, 0, 1, 2], np.int32), p.sigmas[:4], p.prim_offsets, p.B, p.beta, p.tau)
    cell = b.cell[0]
    f = (np.stack(np.meshgrid(*[np.arange(4)] * 3, indexing="ij"), -1).reshape(-1, 3) + 0.5) / 4.0
    pts = f @ cell
    po = np.array([0, len(pts)], np.int64)
    say(f"[points in the 4096-atom cell: {len(pts)} points]")
    for precision in ("fp64", "fp32c"):
        plan, db, nb, F, mu = _run(g, ws, b, pts, po, p, precision)
        Fref = oracle.point_features(b.structure(0), p, pts)
        assert_features(F.cpu().numpy(), Fref, p.tau, TOL[precision])
        G = np.random.default_rng(59).standard_normal((len(pts), p.n_features))
        gp, gc = g.features_backward(plan, db, nb, ws, mu, F, torch.as_tensor(G, device="cuda"))
        rpos, rpts, rcell, _ = oracle.point_grad(b.structure(0), p, pts, G)
        gp, gc = gp.cpu().numpy(), gc.cpu().numpy()
        scale = max(np.abs(rpos).max(), np.abs(rpts).max(), np.abs(rcell).max())
        e = max(np.abs(gp[:b.n_atoms] - rpos).max(), np.abs(gp[b.n_atoms:] - rpts).max(), np.abs(gc[0] - rcell).max())
        say(f"  {precision}: {nb.n_pairs} pairs, max grad err {e / scale:.2e}")
        assert e <= GTOL[precision] * scale
