"""The torch.autograd.Function wrapper and the library's output layout.

* GMPFunction: torch.autograd.grad through it equals gmp_features_backward
  bit for bit (it only marshals arguments), and the oracle's analytic
  gradient within the parity bar.
* Layout: the library's feature vector of an isolated dimer, position by
  position, equals the closed forms listed in the paper's feature
  enumeration order (tests/golden/feature_enumeration.json), in every
  precision."""
import os
import sys

import numpy as np
import pytest

import gmp_synth as gs
import oracle
from gpu_helpers import say, assert_features

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import layout_dimer as ld  # noqa: E402


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_12980_amd as g
    g.load()
    return g


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32c", 1e-5), ("fp32w", 1e-5)])
def test_gmpfunction_autograd(g, prec, tol):
    rng = np.random.default_rng(61)
    structs = [gs.small_periodic(rng, n_atoms=14, n_elements=2, density=0.06, dmin=1.3),
               gs.small_cluster(rng, n_atoms=9, n_elements=2, radius=3.0)]
    b = gs.make_batch(structs)
    p = gs.small_probes(rng, orders=(-1, 0, 1, 2, 3), n_sigmas=3, n_elements=2, n_prims=(1, 3), tau=1e-9)
    plan = g.GMPPlan.from_probes(p, prec)
    db = g.DeviceBatch.from_batch(b)
    ws = g.Workspace()
    nb = g.build_neighbors(plan, db, ws)
    G = torch.as_tensor(rng.standard_normal((b.n_atoms, p.n_features)), device="cuda").to(plan.dtype)
    xyz = db.xyz.clone().requires_grad_(True)
    cell = db.cell.clone().requires_grad_(True)
    F = g.GMPFunction.apply(xyz, cell, plan, db, nb, ws)
    loss = (F * G).sum()
    gx, gcell = torch.autograd.grad(loss, (xyz, cell))
    F2, mu2 = g.features(plan, db, nb, ws)
    gp, gc = g.features_backward(plan, db, nb, ws, mu2, F2, G)
    torch.cuda.synchronize()
    assert torch.equal(F, F2)
    assert torch.equal(gx, gp.t()) and torch.equal(gcell, gc.reshape(-1, 9))
    gx, gcell = gx.t().cpu().numpy(), gcell.cpu().numpy()
    Gn = G.double().cpu().numpy()
    for s in range(b.n_structs):
        a0, a1 = int(b.atom_offsets[s]), int(b.atom_offsets[s + 1])
        rp, rc, Fr = oracle.grad(b.structure(s), p, Gn[a0:a1])
        scale = max(np.abs(rp).max(), np.abs(rc).max())
        e = max(np.abs(gx[a0:a1] - rp).max(), np.abs(gcell[s].reshape(3, 3) - rc).max()) / scale
        say(f"[GMPFunction {prec}] structure {s}: gradient error {e:.2e}")
        assert e <= tol
        assert_features(F.detach().double().cpu().numpy()[a0:a1], Fr, p.tau, tol)


@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32w"])
def test_library_output_layout_is_the_golden_enumeration(g, prec):
    fx = ld.golden()
    p = gs.Probes(np.array(fx["orders"], np.int32), np.array(fx["sigmas"]), np.array([0, 2], np.int32),
                  ld.B, ld.BETA, 1e-12)
    plan = g.GMPPlan.from_probes(p, prec)
    labels = plan.labels()
    assert [(l, 0 if l == -1 else s) for l, s in labels] == [(l, 0 if l == -1 else s) for l, s in fx["features"]]
    b = gs.make_batch([ld.dimer_structure()])
    db = g.DeviceBatch.from_batch(b)
    ws = g.Workspace()
    nb = g.build_neighbors(plan, db, ws)
    F, _ = g.features(plan, db, nb, ws)
    got = F.double().cpu().numpy()[0]
    want = ld.expected_vector()
    rel = np.abs(got - want) / want
    say(f"[layout {prec}] max rel {rel.max():.2e}")
    assert rel.max() <= (1e-12 if prec == "fp64" else 1e-6)
