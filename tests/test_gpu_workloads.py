"""The HIP path on the full-size workloads, against the FP64 oracle on
sampled outputs the oracle computes one by one (same tolerance rule as the
small-case parity tests), through the C ABI in the launch configuration the
benchmark uses.  Every list, every gradient of the differentiation batch and
the large system's backward are checked in test_gpu_fullsize.py."""
import numpy as np
import pytest

import gmp_synth as gs
import oracle
from gpu_helpers import say, run_path, check_neighbors, assert_features

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {"fp64": 1e-11, "fp32c": 1e-5, "fp32w": 1e-5}


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


def test_c2_full_size_sampled(g, ws):
    b, p = gs.config("C2")
    cs = np.sort(np.random.default_rng(0).choice(b.n_atoms, 48, replace=False)).astype(np.int32)
    say("[C2] oracle on 48 sampled centres")
    Fref, muref = oracle.features(b.structure(0), p, centres=cs, with_mu=True)
    for prec in ["fp64", "fp32c", "fp32w"]:
        plan, db, nb, F, mu = run_path(g, b, p, prec, ws)
        if prec == "fp64":
            say(f"[C2] neighbours: {nb.n_pairs} pairs")
            assert check_neighbors(nb, b, p, centres={0: list(cs[:12])}) == 12
        r, a = assert_features(F.cpu().numpy()[cs], Fref, p.tau, TOL[prec])
        say(f"[C2 {prec}] max rel {r:.2e}")
        torch.cuda.empty_cache()


def test_c2_graph_step_as_benchmarked(g, ws):
    """The benchmarked step itself: build + forward + adjoint recorded into
    one HIP graph (FP32 compensated) on the 4096-atom cell; replays equal the
    eager launches bit for bit and the features meet the bar on sampled
    centres."""
    b, p = gs.config("C2")
    cs = np.sort(np.random.default_rng(2).choice(b.n_atoms, 24, replace=False)).astype(np.int32)
    Fref = oracle.features(b.structure(0), p, centres=cs)
    plan = g.GMPPlan.from_probes(p, "fp32c")
    db = g.DeviceBatch.from_batch(b)
    w = g.Workspace()
    G = torch.as_tensor(np.random.default_rng(7).standard_normal((b.n_atoms, p.n_features)), device="cuda")
    nb = g.build_neighbors(plan, db, w)
    F0, mu0 = g.features(plan, db, nb, w)
    gp0, gc0 = g.features_backward(plan, db, nb, w, mu0, F0, G)
    F0, gp0, gc0 = F0.clone(), gp0.clone(), gc0.clone()
    step = g.CapturedStep(plan, db, w, nb, backward=True, G=G)
    for r in range(2):
        step.replay()
        torch.cuda.synchronize()
        assert torch.equal(step.F, F0), f"replay {r}: features differ from eager"
        assert torch.equal(step.gpos.view(3, -1).t(), gp0), f"replay {r}: gradient differs from eager"
        assert torch.equal(step.gcell.view(-1, 3, 3), gc0), f"replay {r}: cell gradient differs from eager"
    g.check_status(w)
    r, a = assert_features(step.F.cpu().numpy()[cs], Fref, p.tau, TOL["fp32c"])
    say(f"[C2 graph step] max rel {r:.2e}")
    del step
    torch.cuda.empty_cache()


def _c3_sample(b):
    n = np.diff(b.atom_offsets)
    per = np.flatnonzero(b.pbc != 0)
    clu = np.flatnonzero(b.pbc == 0)
    pick = {int(per[np.argmax(n[per])]), int(clu[np.argmax(n[clu])]), int(per[np.argmin(n[per])]),
            int(clu[np.argmin(n[clu])])}
    pick |= set(int(x) for x in np.random.default_rng(1).choice(b.n_structs, 8, replace=False))
    return sorted(pick)


def test_c3_batched_sampled_and_batch_invariant(g, ws):
    say("[C3] generating 2048 structures")
    b, p = gs.config("C3")
    sample = _c3_sample(b)
    for prec in ["fp32c", "fp64"]:
        plan, db, nb, F, mu = run_path(g, b, p, prec, ws)
        say(f"[C3 {prec}] {b.n_atoms} atoms, {nb.n_pairs} pairs")
        Fn = F.cpu().numpy()
        if prec == "fp64":
            check_neighbors(nb, b, p, centres={s: list(range(min(4, int(b.atom_offsets[s + 1] - b.atom_offsets[s]))))
                                               for s in sample})
        worst = 0.0
        for s in sample:
            a0, a1 = int(b.atom_offsets[s]), int(b.atom_offsets[s + 1])
            r, _ = assert_features(Fn[a0:a1], oracle.features(b.structure(s), p), p.tau, TOL[prec])
            worst = max(worst, r)
        say(f"[C3 {prec}] max rel over {len(sample)} structures {worst:.2e}")
        if prec == "fp32c":
            for s in sample[:6]:
                a0, a1 = int(b.atom_offsets[s]), int(b.atom_offsets[s + 1])
                _, _, _, Fs, _ = run_path(g, gs.make_batch([b.structure(s)]), p, prec, ws)
                assert torch.equal(Fs, F[a0:a1]), f"structure {s} differs alone vs batched"
        torch.cuda.empty_cache()
