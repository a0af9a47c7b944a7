"""Order -1 (the local density at the centre, one feature without a width)
on the HIP path vs the FP64 oracle, through the C ABI.

Same bars as the other parity tests: neighbour lists (now with the density
cutoff slot) bit-exact; features within 1e-11 (FP64) or 1e-5 (FP32 modes)
relative above the threshold, tau absolute below; gradients norm-wise per
structure within 1e-11 (FP64) or 1e-5 (FP32 modes).
"""
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


def _with_orders(p, orders):
    return gs.Probes(np.asarray(orders, np.int32), p.sigmas, p.prim_offsets, p.B, p.beta, p.tau)


@pytest.fixture(scope="module")
def c1_dens():
    """The 64-atom periodic cell with the paper's example order list
    (-1, 0, 1, 2) and four sigmas."""
    b, p = gs.config("C1")
    p = _with_orders(p, (-1, 0, 1, 2))
    return b, p, oracle.features_batch(b, p, with_mu=True)


def _mixed_batch(seed, orders):
    rng = np.random.default_rng(seed)
    structs = [
        gs.small_periodic(rng, n_atoms=14, n_elements=3, density=0.06, dmin=1.3),
        gs.small_periodic(rng, n_atoms=3, n_elements=3, density=0.08, dmin=1.0),
        gs.small_cluster(rng, n_atoms=9, n_elements=3, radius=3.2),
        gs.small_periodic(rng, n_atoms=10, n_elements=3, density=0.04, dmin=1.3, pbc=3),
        gs.small_cluster(rng, n_atoms=1, n_elements=3),
    ]
    probes = gs.small_probes(rng, orders=orders, n_sigmas=3, n_elements=3, n_prims=(1, 4), tau=1e-9)
    return gs.make_batch(structs), probes


@pytest.mark.parametrize("precision", ["fp64", "fp32c", "fp32w"])
def test_c1_density_lists_and_features(g, ws, c1_dens, precision):
    b, p, (Fref, muref) = c1_dens
    say(f"[c1 orders -1,0,1,2 {precision}]")
    plan, db, nb, F, mu = run_path(g, b, p, precision, ws)
    assert plan.n_slots == len(p.sigmas) + 1 and plan.n_features == 1 + 3 * len(p.sigmas)
    assert np.array_equal(plan.rc2, oracle.cutoffs(p))
    assert check_neighbors(nb, b, p, centres={0: [0, 9, 31, 63]}) == 4
    r, a = assert_features(F.cpu().numpy(), Fref, p.tau, TOL[precision])
    if precision == "fp64":
        scale = np.abs(muref).max(axis=0, keepdims=True)
        assert np.all(np.abs(mu.cpu().numpy() - muref) <= 1e-11 * scale + 1e-300)
    say(f"  max rel {r:.2e}")


@pytest.mark.parametrize("orders", [(-1,), (2, -1, 4), (0, 1, -1)])
@pytest.mark.parametrize("precision", ["fp64", "fp32c", "fp32w"])
def test_density_position_and_mixed_structures(g, ws, orders, precision):
    b, p = _mixed_batch(21, orders)
    say(f"[mixed batch orders {orders} {precision}]")
    plan, db, nb, F, mu = run_path(g, b, p, precision, ws)
    check_neighbors(nb, b, p)
    Fref = oracle.features_batch(b, p)
    r, a = assert_features(F.cpu().numpy(), Fref, p.tau, TOL[precision])
    say(f"  max rel {r:.2e}")


def test_density_slot_not_the_smallest_cutoff(g, ws):
    """A wide probe with a loose threshold has a shorter cutoff than the
    density: the density slot then sits in the middle of the shell order."""
    rng = np.random.default_rng(23)
    b = gs.make_batch([gs.small_periodic(rng, n_atoms=12, n_elements=2, density=0.06, dmin=1.3),
                       gs.small_cluster(rng, n_atoms=7, n_elements=2, radius=3.0)])
    p = gs.Probes(np.array([0, -1, 1], np.int32), np.array([0.4, 4.0, 6.0]), np.array([0, 2, 3], np.int32),
                  np.array([1.0, 0.5, 2.0]), np.array([1.0, 0.4, 2.5]), 5e-3)
    rc2 = oracle.cutoffs(p)  # the widest probe's cutoff is 0 (only the self term)
    assert rc2[2] == 0.0 < rc2[3] < rc2[0] < rc2[1], rc2
    say(f"[density slot between sigmas, rc2 {rc2}]")
    for precision in ("fp64", "fp32c"):
        plan, db, nb, F, mu = run_path(g, b, p, precision, ws)
        check_neighbors(nb, b, p)
        assert_features(F.cpu().numpy(), oracle.features_batch(b, p), p.tau, TOL[precision])


@pytest.mark.parametrize("precision", ["fp64", "fp32c", "fp32w"])
@pytest.mark.parametrize("orders", [(-1, 0, 1, 2), (3, -1)])
def test_density_backward_vs_oracle(g, ws, precision, orders):
    rng = np.random.default_rng(29)
    structs = [gs.small_periodic(rng, n_atoms=12, n_elements=2, density=0.06, dmin=1.3),
               gs.small_cluster(rng, n_atoms=8, n_elements=2, radius=3.0),
               gs.small_periodic(rng, n_atoms=3, n_elements=2, density=0.08, dmin=1.0)]
    b = gs.make_batch(structs)
    p = gs.small_probes(rng, orders=orders, n_sigmas=3, n_elements=2, n_prims=(1, 3), tau=1e-9)
    say(f"[density backward {orders} {precision}]")
    plan, db, nb, F, mu = run_path(g, b, p, precision, ws)
    G = rng.standard_normal((b.n_atoms, p.n_features))
    gp, gc = g.features_backward(plan, db, nb, ws, mu, F, torch.as_tensor(G, device="cuda"))
    gp, gc = gp.cpu().numpy(), gc.cpu().numpy()
    for s in range(b.n_structs):
        a0, a1 = b.atom_offsets[s], b.atom_offsets[s + 1]
        rp, rc, _ = oracle.grad(b.structure(s), p, G[a0:a1])
        scale = max(np.abs(rp).max(), np.abs(rc).max())
        ep = np.abs(gp[a0:a1] - rp).max()
        ec = np.abs(gc[s] - rc).max()
        say(f"  struct {s}: pos err {ep / scale:.2e} cell err {ec / scale:.2e}")
        assert ep <= GTOL[precision] * scale and ec <= GTOL[precision] * scale


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_density_batch_invariant(g, ws, precision):
    b, p = _mixed_batch(31, (-1, 0, 2))
    say(f"[density batch invariance {precision}]")
    plan, db, nb, F1, mu1 = run_path(g, b, p, precision, ws)
    for s in range(b.n_structs):
        _, _, _, Fs, _ = run_path(g, gs.make_batch([b.structure(s)]), p, precision, ws)
        a0, a1 = b.atom_offsets[s], b.atom_offsets[s + 1]
        assert torch.equal(Fs, F1[a0:a1])
