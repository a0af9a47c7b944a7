"""Full per-pair feature Jacobian on the HIP path vs the FP64 oracle, through
the C ABI: per structure max |J - J_ref| <= tol * max |J_ref| (1e-11 FP64,
1e-5 FP32 modes), pairs in the same canonical order; its contraction with
an upstream gradient, assembled per atom on the GPU, reproduces the adjoint
(atoms and reference points)."""
import numpy as np
import pytest

import gmp_synth as gs
import oracle
from gpu_helpers import say, run_path

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

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


def _batch(seed, orders, occupancy=False):
    rng = np.random.default_rng(seed)
    structs = [gs.small_periodic(rng, n_atoms=10, n_elements=2, density=0.06, dmin=1.3),
               gs.small_cluster(rng, n_atoms=7, n_elements=2, radius=2.8),
               gs.small_periodic(rng, n_atoms=3, n_elements=2, density=0.08, dmin=1.0)]
    occs = None
    if occupancy:
        dis = [gs.disorder(rng, st, n_elements=2) for st in structs]
        structs, occs = [d[0] for d in dis], [d[1] for d in dis]
    p = gs.small_probes(rng, orders=orders, n_sigmas=3, n_elements=2, n_prims=(1, 3), tau=1e-9)
    return gs.make_batch(structs, occupancy=occs), p


@pytest.mark.parametrize("precision", ["fp64", "fp32c", "fp32w"])
@pytest.mark.parametrize("orders,occupancy", [((0, 1, 2, 3, 4), False), ((-1, 0, 2), True)])
def test_jacobian_vs_oracle(g, ws, precision, orders, occupancy):
    b, p = _batch(61, orders, occupancy)
    say(f"[jacobian {precision} orders {orders} occupancy={occupancy}]")
    plan, db, nb, F, mu = run_path(g, b, p, precision, ws)
    J = g.feature_jacobian(plan, db, nb, ws, mu).double()
    cnt = (nb.offsets[1:] - nb.offsets[:-1])[nb.slot.long()].cpu().numpy()  # list length per centre
    for s in range(b.n_structs):
        a0, a1 = int(b.atom_offsets[s]), int(b.atom_offsets[s + 1])
        occ = None if b.occupancy is None else b.occupancy[a0:a1]
        Jr, ro = oracle.jacobian(b.structure(s), p, occupancy=occ)
        Jg = J[g.pairs_by_centre(nb, np.arange(a0, a1))].cpu().numpy()  # lists in atom order
        assert Jg.shape == Jr.shape
        assert np.array_equal(cnt[a0:a1], np.diff(ro))
        scale = np.abs(Jr).max()
        err = np.abs(Jg - Jr).max()
        say(f"  struct {s}: {len(Jr)} pairs, max err {err / scale:.2e}")
        assert err <= GTOL[precision] * scale


def _assemble(g, nb, J, G, n_total, wrap, n_structs, centre_struct, centre_index):
    """dL/dpos (atoms then centres that are points) and dL/dcell of
    L = sum G F from the per-pair Jacobian, on the GPU."""
    ic = g.pair_centres(nb)
    v = torch.einsum("pf,pfk->pk", G[ic].double(), J.double())
    gp = torch.zeros((n_total, 3), dtype=torch.float64, device=v.device)
    gp.index_add_(0, nb.j[:nb.n_pairs].long(), v)
    gp.index_add_(0, centre_index[ic], -v)
    w = nb.shift[:nb.n_pairs]
    n = torch.stack([((w >> (8 * k)) & 0xff).to(torch.int8).long() for k in range(3)], 1)
    nt = (n - wrap[nb.j[:nb.n_pairs].long()] + wrap[centre_index[ic]]).double()
    gc = torch.zeros((n_structs, 3, 3), dtype=torch.float64, device=v.device)
    gc.index_add_(0, centre_struct[ic], nt[:, :, None] * v[:, None, :])
    return gp, gc


@pytest.mark.parametrize("points", [False, True])
def test_jacobian_contraction_is_the_adjoint(g, ws, points):
    b, p = _batch(63, (-1, 0, 1, 2))
    plan = g.GMPPlan.from_probes(p, "fp64")
    db = g.DeviceBatch.from_batch(b)
    rng = np.random.default_rng(64)
    if points:
        pts, po = [], [0]
        for s in range(b.n_structs):
            pos, _, cell, pbc = b.structure(s)
            q = rng.uniform(0, 1, (4, 3)) @ cell if pbc else rng.normal(size=(4, 3)) * 2.0
            pts.append(q)
            po.append(po[-1] + 4)
        db = db.with_points(np.concatenate(pts), po)
        cstruct = torch.as_tensor(np.repeat(np.arange(b.n_structs), 4), device="cuda")
    else:
        cstruct = torch.as_tensor(np.repeat(np.arange(b.n_structs), np.diff(b.atom_offsets)), device="cuda")
    say(f"[jacobian contraction, points={points}]")
    nb = g.build_neighbors(plan, db, ws)
    F, mu = g.features(plan, db, nb, ws)
    J = g.feature_jacobian(plan, db, nb, ws, mu)
    G = torch.as_tensor(rng.standard_normal((db.n_centres, p.n_features)), device="cuda")
    gp_ref, gc_ref = g.features_backward(plan, db, nb, ws, mu, F, G)
    cidx = torch.arange(db.n_centres, device="cuda") + (db.n_atoms if points else 0)
    wrap = nb.wrap.view(db.n_total, 3).long()
    gp, gc = _assemble(g, nb, J, G, db.n_total, wrap, b.n_structs, cstruct, cidx)
    scale = max(gp_ref.abs().max().item(), gc_ref.abs().max().item())
    assert (gp - gp_ref).abs().max().item() <= 1e-12 * scale
    assert (gc - gc_ref).abs().max().item() <= 1e-12 * scale
