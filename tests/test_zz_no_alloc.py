"""gmp_features_noalloc (the forward without a workspace, its scratch in a
fixed device array) against gmp_features, through the C ABI: two calls in a
row, the second on a smaller batch, each bitwise equal to the workspace
entry point's output; a batch beyond the array is rejected with
GMP_E_NOMEM and a message that names both sizes."""
import ctypes

import numpy as np
import pytest

import gmp_synth as gs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_12980_amd as g
    g.load()
    return g


def _noalloc(g, plan, db, nb, F, mu):
    from paper_2303_12980_amd import _lib
    L = _lib.load()
    bd, nd = db.desc(), nb.desc()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return L.gmp_features_noalloc(plan.handle, ctypes.byref(bd), ctypes.byref(nd), ctypes.c_void_p(F.data_ptr()),
                                  ctypes.c_void_p(mu.data_ptr()), stream)


def _case(g, b, p, prec):
    plan = g.GMPPlan.from_probes(p, prec)
    db = g.DeviceBatch.from_batch(b)
    ws = g.Workspace()
    nb = g.build_neighbors(plan, db, ws, reverse=False)
    Fw, muw = g.features(plan, db, nb, ws)
    F = torch.full_like(Fw, float("nan"))
    mu = torch.full_like(muw, float("nan"))
    return plan, db, nb, Fw, muw, F, mu


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_noalloc_matches_workspace_entry_point(g, prec):
    # first call: the 4096-atom cell (l <= 4, 8 sigmas), then a smaller batch
    # (64-atom cell and a mixed small batch) on the same GPU's scratch
    rng = np.random.default_rng(71)
    small = gs.make_batch([gs.small_periodic(rng, n_atoms=20, n_elements=2, density=0.06, dmin=1.3),
                           gs.small_cluster(rng, n_atoms=7, n_elements=2, radius=3.0)])
    ps = gs.small_probes(rng, orders=(-1, 0, 1, 2, 3, 4), n_sigmas=3, n_elements=2, n_prims=(1, 3), tau=1e-9)
    for name, (b, p) in (("C2", gs.config("C2")), ("small", (small, ps))):
        plan, db, nb, Fw, muw, F, mu = _case(g, b, p, prec)
        assert _noalloc(g, plan, db, nb, F, mu) == 0
        torch.cuda.synchronize()
        print(f"[noalloc {prec} {name}] {b.n_atoms} atoms, {nb.n_pairs} pairs", flush=True)
        assert torch.equal(F, Fw), name
        assert torch.equal(mu, muw), name


def test_noalloc_rejects_a_batch_beyond_its_scratch(g):
    from paper_2303_12980_amd import _lib
    b, p = gs.config("C2")
    plan = g.GMPPlan.from_probes(p, "fp32c")
    plan.set_tuning(chunk_pairs=64)  # one work item per 64 pairs: ~86,000 items need ~190 MB
    db = g.DeviceBatch.from_batch(b)
    ws = g.Workspace()
    nb = g.build_neighbors(plan, db, ws, reverse=False)
    F = torch.zeros((b.n_atoms, p.n_features), dtype=torch.float32, device="cuda")
    mu = torch.zeros((b.n_atoms, plan.n_components), dtype=torch.float64, device="cuda")
    st = _noalloc(g, plan, db, nb, F, mu)
    assert st == _lib.GMP_E_NOMEM
    msg = _lib.load().gmp_last_error().decode()
    assert "scratch" in msg and str(64 << 20) in msg
    torch.cuda.synchronize()
    assert bool((F == 0).all())  # nothing was launched
