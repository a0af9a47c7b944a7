"""HIP path vs the FP64 oracle, through the C ABI, on seeded inputs.

Neighbour lists: bit-exact (order, image shifts, segment and sigma-prefix
boundaries, wrap indices, wrapped coordinates).
Features: the overlap-threshold rule -- relative error <= 1e-11 (FP64 path)
or <= 1e-5 (FP32 compensated path) where the oracle feature exceeds the
threshold tau, absolute error <= tau elsewhere.
Gradients: max |g - g_ref| <= tol * max |g_ref| per structure, tol 1e-11
(FP64) / 1e-5 (FP32 compensated).
"""
import numpy as np
import pytest

import gmp_synth as gs
import oracle
from gpu_helpers import say, run_path, check_neighbors, assert_features, feature_errors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


@pytest.fixture(scope="module")
def c1():
    b, p = gs.config("C1")
    return b, p, oracle.features_batch(b, p, with_mu=True)


def _small_batch(seed):
    rng = np.random.default_rng(seed)
    structs = [
        gs.small_periodic(rng, n_atoms=14, n_elements=3, density=0.06, dmin=1.3),
        gs.small_periodic(rng, n_atoms=3, n_elements=3, density=0.08, dmin=1.0),  # cutoff >> cell
        gs.small_cluster(rng, n_atoms=9, n_elements=3, radius=3.2),
        gs.small_periodic(rng, n_atoms=10, n_elements=3, density=0.04, dmin=1.3, pbc=3),  # slab
        gs.small_cluster(rng, n_atoms=1, n_elements=3),  # single isolated atom
        gs.small_periodic(rng, n_atoms=1, n_elements=3, density=0.1),  # one atom, periodic
    ]
    probes = gs.small_probes(rng, orders=(0, 1, 2, 3, 4), n_sigmas=4, n_elements=3, n_prims=(1, 4), tau=1e-9)
    return gs.make_batch(structs), probes


@pytest.mark.parametrize("precision", ["fp64", "fp32c", "fp32w"])
def test_c1_neighbors_bit_exact(g, ws, c1, precision):
    b, p, _ = c1
    say(f"[c1 neighbours {precision}]")
    plan, db, nb, F, mu = run_path(g, b, p, precision, ws)
    assert np.array_equal(plan.rc2, oracle.cutoffs(p))
    assert check_neighbors(nb, b, p) == 64


def test_c1_features_fp64(g, ws, c1):
    b, p, (Fref, muref) = c1
    say("[c1 features fp64]")
    plan, db, nb, F, mu = run_path(g, b, p, "fp64", ws)
    r, a = assert_features(F.cpu().numpy(), Fref, p.tau, 1e-11)
    scale = np.abs(muref).max(axis=0, keepdims=True)
    assert np.all(np.abs(mu.cpu().numpy() - muref) <= 1e-11 * scale + 1e-300)
    say(f"  max rel {r:.2e}")


@pytest.mark.parametrize("precision", ["fp32c", "fp32w"])
def test_c1_features_fp32(g, ws, c1, precision):
    b, p, (Fref, muref) = c1
    say(f"[c1 features {precision}]")
    plan, db, nb, F, mu = run_path(g, b, p, precision, ws)
    r, a = assert_features(F.cpu().numpy(), Fref, p.tau, 1e-5)
    say(f"  max rel {r:.2e}")


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32c", 1e-5), ("fp32w", 1e-5)])
def test_small_batch_mixed_structures(g, ws, precision, tol):
    b, p = _small_batch(3)
    say(f"[small batch {precision}]")
    plan, db, nb, F, mu = run_path(g, b, p, precision, ws)
    check_neighbors(nb, b, p)
    Fref = oracle.features_batch(b, p)
    r, a = assert_features(F.cpu().numpy(), Fref, p.tau, tol)
    say(f"  max rel {r:.2e}")


@pytest.mark.parametrize("chunk", [0, 64, 100, 1000])
def test_chunked_overlap_matches(g, ws, c1, chunk):
    """Splitting centres into chunks changes only the summation order."""
    b, p, (Fref, _) = c1
    say(f"[c1 chunk {chunk}]")
    plan, db, nb, F, mu = run_path(g, b, p, "fp64", ws, tuning=dict(chunk_pairs=chunk))
    assert_features(F.cpu().numpy(), Fref, p.tau, 1e-11)


@pytest.mark.parametrize("precision", ["fp64", "fp32c", "fp32w"])
@pytest.mark.parametrize("bin_divisor,blocks", [(1, 0), (3, 1), (4, 0)])
def test_tunings_do_not_change_lists_or_features(g, ws, c1, bin_divisor, blocks, precision):
    """Cell-list bin size and the persistent grid size change only the work
    decomposition: lists stay bit-exact, features within the tolerance."""
    b, p, (Fref, _) = c1
    say(f"[c1 bin_divisor {bin_divisor} blocks/CU {blocks} {precision}]")
    plan, db, nb, F, mu = run_path(g, b, p, precision, ws,
                                   tuning=dict(bin_divisor=bin_divisor, blocks_per_cu=blocks))
    assert check_neighbors(nb, b, p, centres={0: [0, 17, 63]}) == 3
    assert_features(F.cpu().numpy(), Fref, p.tau, 1e-11 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32c", 1e-5), ("fp32w", 1e-5)])
def test_backward_vs_oracle(g, ws, precision, tol):
    rng = np.random.default_rng(17)
    structs = [gs.small_periodic(rng, n_atoms=12, n_elements=2, density=0.06, dmin=1.3),
               gs.small_cluster(rng, n_atoms=8, n_elements=2, radius=3.0),
               gs.small_periodic(rng, n_atoms=3, n_elements=2, density=0.08, dmin=1.0)]
    b = gs.make_batch(structs)
    p = gs.small_probes(rng, orders=(0, 1, 2, 3, 4), n_sigmas=3, n_elements=2, n_prims=(1, 3), tau=1e-9)
    say(f"[backward {precision}]")
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
        assert ep <= tol * scale and ec <= tol * scale


@pytest.mark.parametrize("precision", ["fp64", "fp32c", "fp32w"])
def test_deterministic_and_batch_invariant(g, ws, precision):
    b, p = _small_batch(5)
    say(f"[determinism {precision}]")
    plan, db, nb, F1, mu1 = run_path(g, b, p, precision, ws)
    _, _, _, F2, mu2 = run_path(g, b, p, precision, ws)
    assert torch.equal(F1, F2) and torch.equal(mu1, mu2)
    for s in range(b.n_structs):
        one = gs.make_batch([b.structure(s)])
        _, _, _, Fs, _ = run_path(g, one, p, precision, ws)
        a0, a1 = b.atom_offsets[s], b.atom_offsets[s + 1]
        assert torch.equal(Fs, F1[a0:a1])
