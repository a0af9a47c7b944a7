"""Disordered structures (per-atom fractional occupancy) on the HIP path vs
the FP64 oracle, through the C ABI: features and gradients to the usual
bars, unit occupancy bitwise equal to no occupancy, lists independent of
the occupancies, a non-finite occupancy reported by the build."""
import numpy as np
import pytest

import gmp_synth as gs
import oracle
from gpu_helpers import say, run_path, check_neighbors, assert_features

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


def _disordered_batch(seed, orders=(-1, 0, 1, 2, 3, 4), n_sigmas=3):
    rng = np.random.default_rng(seed)
    base = [gs.small_periodic(rng, n_atoms=12, n_elements=3, density=0.06, dmin=1.3),
            gs.small_cluster(rng, n_atoms=8, n_elements=3, radius=3.0),
            gs.small_periodic(rng, n_atoms=9, n_elements=3, density=0.04, dmin=1.3, pbc=3),
            gs.small_periodic(rng, n_atoms=3, n_elements=3, density=0.08, dmin=1.0)]
    structs, occs = [], []
    for st in base:
        d, o = gs.disorder(rng, st, n_elements=3, mixed=0.3, vacant=0.3)
        structs.append(d)
        occs.append(o)
    p = gs.small_probes(rng, orders=orders, n_sigmas=n_sigmas, n_elements=3, n_prims=(1, 4), tau=1e-9)
    return gs.make_batch(structs, occupancy=occs), p


@pytest.mark.parametrize("precision", ["fp64", "fp32c", "fp32w"])
def test_disordered_features(g, ws, precision):
    b, p = _disordered_batch(41)
    say(f"[disordered features {precision}: {b.n_atoms} entries]")
    plan, db, nb, F, mu = run_path(g, b, p, precision, ws)
    check_neighbors(nb, b, p)
    Fref = oracle.features_batch(b, p)
    r, a = assert_features(F.cpu().numpy(), Fref, p.tau, TOL[precision])
    say(f"  max rel {r:.2e}")


@pytest.mark.parametrize("precision", ["fp64", "fp32c", "fp32w"])
def test_disordered_backward(g, ws, precision):
    b, p = _disordered_batch(43, orders=(-1, 0, 2, 3))
    say(f"[disordered backward {precision}]")
    plan, db, nb, F, mu = run_path(g, b, p, precision, ws)
    rng = np.random.default_rng(44)
    G = rng.standard_normal((b.n_atoms, p.n_features))
    gp, gc = g.features_backward(plan, db, nb, ws, mu, F, torch.as_tensor(G, device="cuda"))
    gp, gc = gp.cpu().numpy(), gc.cpu().numpy()
    for s in range(b.n_structs):
        a0, a1 = b.atom_offsets[s], b.atom_offsets[s + 1]
        rp, rc, _ = oracle.grad(b.structure(s), p, G[a0:a1], occupancy=b.occupancy[a0:a1])
        scale = max(np.abs(rp).max(), np.abs(rc).max())
        ep, ec = np.abs(gp[a0:a1] - rp).max(), np.abs(gc[s] - rc).max()
        say(f"  struct {s}: pos err {ep / scale:.2e} cell err {ec / scale:.2e}")
        assert ep <= GTOL[precision] * scale and ec <= GTOL[precision] * scale


@pytest.mark.parametrize("precision", ["fp64", "fp32c", "fp32w"])
def test_unit_occupancy_bitwise(g, ws, precision):
    b, p = _disordered_batch(45)
    ones = gs.Batch(b.atom_offsets, b.pos, b.species, b.cell, b.pbc, np.ones(b.n_atoms))
    none = gs.Batch(b.atom_offsets, b.pos, b.species, b.cell, b.pbc, None)
    say(f"[unit occupancy {precision}]")
    _, _, nb1, F1, mu1 = run_path(g, ones, p, precision, ws)
    _, _, nb0, F0, mu0 = run_path(g, none, p, precision, ws)
    assert torch.equal(F1, F0) and torch.equal(mu1, mu0)
    assert torch.equal(nb1.j[:nb1.n_pairs], nb0.j[:nb0.n_pairs])


def test_occupancy_update_between_graph_replays(g, ws):
    """The occupancies are read at feature time: changing them in place and
    replaying a captured step gives the features of the new occupancies."""
    b, p = _disordered_batch(47)
    plan = g.GMPPlan.from_probes(p, "fp64")
    db = g.DeviceBatch.from_batch(b)
    nb = g.build_neighbors(plan, db, ws)
    step = g.CapturedStep(plan, db, ws, nb, backward=False)
    step.replay()
    torch.cuda.synchronize()
    assert_features(step.F.cpu().numpy(), oracle.features_batch(b, p), p.tau, TOL["fp64"])
    occ2 = np.clip(b.occupancy * 0.5 + 0.2, 0.0, 1.0)
    db.occupancy.copy_(torch.as_tensor(occ2, device="cuda"))
    step.replay()
    torch.cuda.synchronize()
    b2 = gs.Batch(b.atom_offsets, b.pos, b.species, b.cell, b.pbc, occ2)
    assert_features(step.F.cpu().numpy(), oracle.features_batch(b2, p), p.tau, TOL["fp64"])


def test_nonfinite_occupancy_reported(g, ws):
    b, p = _disordered_batch(49)
    occ = b.occupancy.copy()
    occ[3] = np.nan
    bad = gs.Batch(b.atom_offsets, b.pos, b.species, b.cell, b.pbc, occ)
    plan = g.GMPPlan.from_probes(p, "fp32c")
    db = g.DeviceBatch.from_batch(bad)
    with pytest.raises(g.GMPError):
        g.build_neighbors(plan, db, ws)
