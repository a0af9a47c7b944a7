"""Full-size parity of the HIP path against the FP64 oracle, in the launch
configuration the benchmark uses (one plan per precision, default tuning):

* neighbour lists bit-exact for every centre of the 4096-atom cell and of
  all 512 differentiation structures, and for 1,200 sampled centres of the
  100,000-atom cell;
* the adjoint of all 512 differentiation structures against the oracle's
  analytic gradient (positions and cell; 1e-5 in the FP32 modes, 1e-11 in
  FP64, norm-wise per structure), and central finite differences
  (h = 1e-5 A) of the GPU's own FP64 forward over every position and cell
  entry of 8 seeded structures;
* the adjoint of the 100,000-atom cell with an upstream gradient that is
  non-zero on 24 sampled centres only, against the oracle's gradient
  restricted to those centres, for every atom and the cell.

The oracle runs on the host's cores (its C code releases the GIL; the
structures of a batch are computed in parallel threads)."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import gmp_synth as gs
import oracle
from gpu_helpers import say, run_path, check_lists_many, check_reverse, assert_features

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GTOL = {"fp64": 1e-11, "fp32c": 1e-5, "fp32w": 1e-5}
WORKERS = max(1, min(16, len(os.sched_getaffinity(0))))


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_12980_amd as g
    g.load()
    return g


@pytest.fixture(scope="module")
def c4():
    say("[C4] generating 512 structures")
    b, p = gs.config("C4")
    G = gs.upstream_gradient(4, b.n_atoms, p.n_features)
    return b, p, G


@pytest.fixture(scope="module")
def c4_oracle(c4):
    """Oracle features and analytic gradients of all 512 structures."""
    b, p, G = c4

    def one(s):
        a0, a1 = int(b.atom_offsets[s]), int(b.atom_offsets[s + 1])
        return oracle.grad(b.structure(s), p, G[a0:a1])

    say(f"[C4] oracle gradients of {b.n_structs} structures on {WORKERS} threads")
    with ThreadPoolExecutor(WORKERS) as ex:
        return list(ex.map(one, range(b.n_structs)))


def test_c2_lists_every_centre(g):
    b, p = gs.config("C2")
    plan = g.GMPPlan.from_probes(p, "fp32c")
    db = g.DeviceBatch.from_batch(b)
    ws = g.Workspace()
    nb = g.build_neighbors(plan, db, ws)
    torch.cuda.synchronize()
    say(f"[C2] {nb.n_pairs} pairs: every list against the oracle")
    assert check_lists_many(nb, b, p, 0) == b.n_atoms
    check_reverse(nb)
    del nb
    torch.cuda.empty_cache()


def test_c4_lists_every_centre(g, c4):
    b, p, _ = c4
    plan = g.GMPPlan.from_probes(p, "fp32c")
    db = g.DeviceBatch.from_batch(b)
    ws = g.Workspace()
    nb = g.build_neighbors(plan, db, ws)
    torch.cuda.synchronize()
    say(f"[C4] {nb.n_pairs} pairs: every list of {b.n_structs} structures against the oracle")
    with ThreadPoolExecutor(WORKERS) as ex:
        checked = sum(ex.map(lambda s: check_lists_many(nb, b, p, s), range(b.n_structs)))
    assert checked == b.n_atoms
    check_reverse(nb)
    del nb
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["fp32c", "fp32w", "fp64"])
def test_c4_gradients_every_structure(g, c4, c4_oracle, prec):
    b, p, G = c4
    ws = g.Workspace()
    plan, db, nb, F, mu = run_path(g, b, p, prec, ws)
    Gt = torch.as_tensor(G, device="cuda")
    gp, gc = g.features_backward(plan, db, nb, ws, mu, F, Gt)
    gp, gc, Fn = gp.cpu().numpy(), gc.cpu().numpy(), F.double().cpu().numpy()
    worst, worst_f = 0.0, 0.0
    for s in range(b.n_structs):
        a0, a1 = int(b.atom_offsets[s]), int(b.atom_offsets[s + 1])
        rp, rc, Fr = c4_oracle[s]
        scale = max(np.abs(rp).max(), np.abs(rc).max())
        e = max(np.abs(gp[a0:a1] - rp).max(), np.abs(gc[s] - rc).max()) / scale
        assert e <= GTOL[prec], f"structure {s}: gradient error {e:.3e}"
        worst = max(worst, e)
        r, _ = assert_features(Fn[a0:a1], Fr, p.tau, 1e-11 if prec == "fp64" else 1e-5)
        worst_f = max(worst_f, r)
    say(f"[C4 {prec}] 512 structures: max gradient error {worst:.2e}, max feature rel error {worst_f:.2e}")
    del nb, F, mu
    torch.cuda.empty_cache()


def test_c4_finite_differences_8_structures(g, c4):
    """Central differences (h = 1e-5 A) of L_s = sum G F over structure s,
    over the frozen pair set, on the FP64 GPU forward, for every position and
    cell entry of 8 seeded structures; the perturbation of one entry is
    applied to all 8 structures at once (they are independent)."""
    b, p, G = c4
    sel = sorted(np.random.default_rng(44).choice(b.n_structs, 8, replace=False).tolist())
    sub = gs.make_batch([b.structure(s) for s in sel])
    Gs = np.concatenate([G[int(b.atom_offsets[s]):int(b.atom_offsets[s + 1])] for s in sel])
    ws = g.Workspace()
    plan, db, nb, F, mu = run_path(g, sub, p, "fp64", ws)
    Gt = torch.as_tensor(Gs, device="cuda")
    gp, gc = g.features_backward(plan, db, nb, ws, mu, F, Gt)
    gp, gc = gp.cpu().numpy(), gc.cpu().numpy()
    offs = sub.atom_offsets.astype(np.int64)
    owner = torch.as_tensor(np.repeat(np.arange(len(sel)), np.diff(offs)), device="cuda")
    xyz0, cell0 = db.xyz.clone(), db.cell.clone()

    def losses(xyz, cell):
        Fh, _ = g.features(plan, db, nb, ws, with_components=False, xyz=xyz, cell=cell)
        per_atom = (Fh * Gt).sum(dim=1)
        return torch.zeros(len(sel), dtype=torch.float64, device="cuda").index_add_(0, owner, per_atom)

    h = 1e-5
    n = np.diff(offs)
    scale = np.array([max(np.abs(gp[offs[t]:offs[t + 1]]).max(), np.abs(gc[t]).max()) for t in range(len(sel))])
    worst = 0.0
    for a in range(int(n.max())):
        live = np.flatnonzero(n > a)
        idx = torch.as_tensor(offs[live] + a, device="cuda")
        for k in range(3):
            xp, xm = xyz0.clone(), xyz0.clone()
            xp[k, idx] += h
            xm[k, idx] -= h
            fd = ((losses(xp, cell0) - losses(xm, cell0)) / (2 * h)).cpu().numpy()
            err = np.abs(fd[live] - gp[offs[live] + a, k]) / scale[live]
            worst = max(worst, float(err.max()))
            assert err.max() <= 1e-6, (a, k, err.max())
    for ent in range(9):
        cp, cm = cell0.clone(), cell0.clone()
        cp[:, ent] += h
        cm[:, ent] -= h
        fd = ((losses(xyz0, cp) - losses(xyz0, cm)) / (2 * h)).cpu().numpy()
        err = np.abs(fd - gc.reshape(-1, 9)[:, ent]) / scale
        worst = max(worst, float(err.max()))
        assert err.max() <= 1e-6, (ent, err.max())
    say(f"[C4 fd] structures {sel}: {int(n.sum()) * 3 + 9 * len(sel)} entries, max |fd - adjoint| / max|g| "
        f"{worst:.2e}")


@pytest.fixture(scope="module")
def c5():
    say("[C5] generating 100000 atoms")
    b, p = gs.config("C5")
    return b, p


def test_c5_lists_sampled(g, c5):
    b, p = c5
    plan = g.GMPPlan.from_probes(p, "fp32c")
    db = g.DeviceBatch.from_batch(b)
    ws = g.Workspace()
    nb = g.build_neighbors(plan, db, ws)
    torch.cuda.synchronize()
    cs = np.sort(np.random.default_rng(55).choice(b.n_atoms, 1200, replace=False))
    say(f"[C5] {nb.n_pairs} pairs: 1200 sampled lists against the oracle")
    assert check_lists_many(nb, b, p, 0, cs) == 1200
    check_reverse(nb)
    del nb
    torch.cuda.empty_cache()


def test_c5_backward_on_sampled_centres(g, c5):
    """G non-zero on 24 sampled centres only: every atom's gradient and the
    cell gradient against the oracle's gradient restricted to them."""
    b, p = c5
    rng = np.random.default_rng(57)
    cs = np.sort(rng.choice(b.n_atoms, 24, replace=False)).astype(np.int32)
    Gc = rng.standard_normal((len(cs), p.n_features))
    say("[C5] oracle gradient restricted to 24 centres")
    rp, rc = oracle.grad_centres(b.structure(0), p, cs, Gc)
    Fref = oracle.features(b.structure(0), p, centres=cs)
    scale = max(np.abs(rp).max(), np.abs(rc).max())
    Gfull = np.zeros((b.n_atoms, p.n_features))
    Gfull[cs] = Gc
    ws = g.Workspace()
    for prec in ["fp32c", "fp32w", "fp64"]:
        plan, db, nb, F, mu = run_path(g, b, p, prec, ws)
        gp, gc = g.features_backward(plan, db, nb, ws, mu, F, torch.as_tensor(Gfull, device="cuda"))
        torch.cuda.synchronize()
        e_pos = np.abs(gp.cpu().numpy() - rp).max() / scale
        e_cell = np.abs(gc.cpu().numpy()[0] - rc).max() / scale
        r, _ = assert_features(F.double().cpu().numpy()[cs], Fref, p.tau, 1e-11 if prec == "fp64" else 1e-5)
        say(f"[C5 {prec}] gradient error: atoms {e_pos:.2e}, cell {e_cell:.2e}; features {r:.2e}")
        assert e_pos <= GTOL[prec] and e_cell <= GTOL[prec]
        del nb, F, mu, gp, gc
        torch.cuda.empty_cache()
