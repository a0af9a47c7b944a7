"""Per-primitive screening (the speed variant of the truncation) on the HIP
path vs the oracle's screened mode, through the C ABI: lists unchanged and
bit-exact, features, gradients and the per-pair Jacobian to the usual bars;
screened features stay within the oracle's own screened-vs-exact distance."""
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


def _case(seed, orders=(-1, 0, 1, 2, 3, 4)):
    rng = np.random.default_rng(seed)
    structs = [gs.small_periodic(rng, n_atoms=14, n_elements=3, density=0.06, dmin=1.2),
               gs.small_cluster(rng, n_atoms=9, n_elements=3, radius=3.0),
               gs.small_periodic(rng, n_atoms=3, n_elements=3, density=0.08, dmin=1.0)]
    p = gs.small_probes(rng, orders=orders, n_sigmas=3, n_elements=3, n_prims=(3, 6), tau=1e-6,
                        beta_range=(0.2, 25.0))
    p.screening = True
    return gs.make_batch(structs), p


@pytest.mark.parametrize("precision", ["fp64", "fp32c", "fp32w"])
def test_screened_features(g, ws, precision):
    b, p = _case(71)
    say(f"[screened features {precision}]")
    plan, db, nb, F, mu = run_path(g, b, p, precision, ws)
    check_neighbors(nb, b, p)
    Fref = oracle.features_batch(b, p)
    exact = gs.Probes(p.orders, p.sigmas, p.prim_offsets, p.B, p.beta, p.tau)
    Fex = oracle.features_batch(b, exact)
    assert not np.array_equal(Fref, Fex)  # the case skips primitives
    r, a = assert_features(F.cpu().numpy(), Fref, p.tau, TOL[precision])
    say(f"  max rel vs screened oracle {r:.2e}; screened vs exact (oracle) {np.abs(Fref - Fex).max():.2e}")


@pytest.mark.parametrize("precision", ["fp64", "fp32c", "fp32w"])
def test_screened_backward_and_jacobian(g, ws, precision):
    b, p = _case(73, orders=(-1, 0, 2, 3))
    say(f"[screened backward / jacobian {precision}]")
    plan, db, nb, F, mu = run_path(g, b, p, precision, ws)
    G = np.random.default_rng(74).standard_normal((b.n_atoms, p.n_features))
    gp, gc = g.features_backward(plan, db, nb, ws, mu, F, torch.as_tensor(G, device="cuda"))
    gp, gc = gp.cpu().numpy(), gc.cpu().numpy()
    J = g.feature_jacobian(plan, db, nb, ws, mu).double()
    for s in range(b.n_structs):
        a0, a1 = int(b.atom_offsets[s]), int(b.atom_offsets[s + 1])
        rp, rc, _ = oracle.grad(b.structure(s), p, G[a0:a1])
        scale = max(np.abs(rp).max(), np.abs(rc).max())
        assert np.abs(gp[a0:a1] - rp).max() <= GTOL[precision] * scale
        assert np.abs(gc[s] - rc).max() <= GTOL[precision] * scale
        Jr, _ = oracle.jacobian(b.structure(s), p)
        Js = J[g.pairs_by_centre(nb, np.arange(a0, a1))].cpu().numpy()  # lists in atom order
        assert np.abs(Js - Jr).max() <= GTOL[precision] * np.abs(Jr).max()
