"""Edge cases of the HIP path through the C ABI: empty batches and empty
structures, capacity overflow in the no-sync build, invalid inputs that the
library must reject with a status code, and neighbour lists longer than the
in-LDS sort."""
import numpy as np
import pytest

import gmp_synth as gs
import oracle
from gpu_helpers import say, assert_features

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_12980_amd as g
    g.load()
    return g


def _probes(seed=3, **kw):
    return gs.small_probes(np.random.default_rng(seed), orders=(0, 1, 2, 3, 4), n_sigmas=3, n_elements=2,
                           n_prims=(1, 3), tau=1e-9, **kw)


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_batch_without_atoms(g, precision):
    say(f"[empty batch {precision}]")
    p = _probes()
    empty = gs.Batch(np.zeros(3, np.int64), np.zeros((0, 3)), np.zeros(0, np.int32),
                     np.stack([np.eye(3) * 5.0, np.eye(3) * 6.0]), np.array([7, 0], np.uint8))
    plan = g.GMPPlan.from_probes(p, precision)
    db = g.DeviceBatch.from_batch(empty)
    ws = g.Workspace()
    nb = g.build_neighbors(plan, db, ws)
    assert nb.n_pairs == 0
    F, mu = g.features(plan, db, nb, ws)
    assert tuple(F.shape) == (0, p.n_features)
    gp, gc = g.features_backward(plan, db, nb, ws, mu, F, torch.zeros((0, p.n_features), device="cuda"))
    torch.cuda.synchronize()
    assert tuple(gp.shape) == (0, 3)
    assert torch.equal(gc.cpu(), torch.zeros((2, 3, 3), dtype=torch.float64))


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_empty_structures_inside_a_batch(g, precision):
    say(f"[empty structures inside a batch {precision}]")
    rng = np.random.default_rng(8)
    s1 = gs.small_periodic(rng, n_atoms=9, n_elements=2, density=0.06, dmin=1.3)
    s2 = gs.small_cluster(rng, n_atoms=6, n_elements=2, radius=3.0)
    none = (np.zeros((0, 3)), np.zeros(0, np.int32), np.eye(3) * 7.0, 7)
    b = gs.make_batch([none, s1, none, s2, none])
    p = _probes()
    plan = g.GMPPlan.from_probes(p, precision)
    db = g.DeviceBatch.from_batch(b)
    ws = g.Workspace()
    nb = g.build_neighbors(plan, db, ws)
    F, mu = g.features(plan, db, nb, ws)
    Fref = oracle.features_batch(b, p)
    assert_features(F.cpu().numpy(), Fref, p.tau, 1e-11 if precision == "fp64" else 1e-5)
    G = torch.as_tensor(rng.standard_normal((b.n_atoms, p.n_features)), device="cuda")
    gp, gc = g.features_backward(plan, db, nb, ws, mu, F, G)
    gc = gc.cpu().numpy()
    for s in (0, 2, 4):
        assert np.all(gc[s] == 0.0)


def test_nosync_overflow_is_reported(g):
    say("[no-sync capacity overflow]")
    b, p = gs.config("C1")
    plan = g.GMPPlan.from_probes(p, "fp32c")
    db = g.DeviceBatch.from_batch(b)
    ws = g.Workspace()
    nb = g.build_neighbors(plan, db, ws)
    small = g.Neighbors(plan, db, nb.n_pairs // 2)
    small.max_list = nb.max_list
    g.rebuild_neighbors_nosync(plan, db, ws, small)
    # the forward and the adjoint still run on the overflowed lists: centres
    # whose list fits are exact, the others read nothing and give zeros
    small.n_pairs = small.capacity
    F, mu = g.features(plan, db, small, ws)
    gp, gc = g.features_backward(plan, db, small, ws, mu, F, torch.ones_like(F))
    torch.cuda.synchronize()
    with pytest.raises(g.GMPError, match="CAPACITY"):
        g.check_status(ws)
    # the workspace status is cleared by the check: a fitting rebuild is clean again
    g.rebuild_neighbors_nosync(plan, db, ws, nb)
    g.check_status(ws)
    Fref, _ = g.features(plan, db, nb, ws)
    offs = small.offsets.cpu().numpy()
    fits = (offs[1:] <= small.capacity)[small.slot.cpu().numpy()]  # per list slot -> per centre
    assert fits.any() and not fits.all()
    Fh, Fr = F.cpu().numpy(), Fref.cpu().numpy()
    assert np.array_equal(Fh[fits], Fr[fits])
    assert np.all(Fh[~fits] == 0.0)
    assert torch.isfinite(gp).all() and torch.isfinite(gc).all()


def test_nosync_overflow_with_points(g):
    """Reference points whose lists overflow a no-sync rebuild: reported by
    the status word; points whose list fits are exact, the others zero, and
    the backward (by-neighbour sort included) stays finite."""
    say("[no-sync capacity overflow, reference points]")
    b, p = gs.config("C1")
    cell = b.cell[0]
    pts = np.random.default_rng(5).uniform(0, 1, (40, 3)) @ cell
    plan = g.GMPPlan.from_probes(p, "fp32c")
    db = g.DeviceBatch.from_batch(b).with_points(pts, [0, len(pts)])
    ws = g.Workspace()
    nb = g.build_neighbors(plan, db, ws)
    small = g.Neighbors(plan, db, nb.n_pairs // 2)
    small.max_list = nb.max_list
    g.rebuild_neighbors_nosync(plan, db, ws, small)
    small.n_pairs = small.capacity
    F, mu = g.features(plan, db, small, ws)
    gp, gc = g.features_backward(plan, db, small, ws, mu, F, torch.ones_like(F))
    J = g.feature_jacobian(plan, db, small, ws, mu)
    torch.cuda.synchronize()
    with pytest.raises(g.GMPError, match="CAPACITY"):
        g.check_status(ws)
    Fref, _ = g.features(plan, db, nb, ws)
    offs = small.offsets.cpu().numpy()
    fits = (offs[1:] <= small.capacity)[small.slot.cpu().numpy()]  # per list slot -> per centre
    assert fits.any() and not fits.all()
    Fh, Fr = F.cpu().numpy(), Fref.cpu().numpy()
    assert np.array_equal(Fh[fits], Fr[fits])
    assert np.all(Fh[~fits] == 0.0)
    assert torch.isfinite(gp).all() and torch.isfinite(gc).all() and J.shape[0] == small.capacity


def test_two_call_capacity_pattern(g):
    say("[two-call capacity]")
    b, p = gs.config("C1")
    plan = g.GMPPlan.from_probes(p, "fp64")
    db = g.DeviceBatch.from_batch(b)
    ws = g.Workspace()
    nb = g.build_neighbors(plan, db, ws, capacity=16)
    ref = g.build_neighbors(plan, db, ws)
    assert nb.capacity >= nb.n_pairs == ref.n_pairs
    assert torch.equal(nb.j[:nb.n_pairs], ref.j[:ref.n_pairs])


def test_species_out_of_range_is_rejected(g):
    say("[species out of range]")
    rng = np.random.default_rng(4)
    pos, spec, cell, pbc = gs.small_periodic(rng, n_atoms=6, n_elements=2, density=0.06, dmin=1.3)
    spec = spec.copy()
    spec[2] = 5
    b = gs.make_batch([(pos, spec, cell, pbc)])
    plan = g.GMPPlan.from_probes(_probes(), "fp32c")
    with pytest.raises(g.GMPError, match="INVALID"):
        g.build_neighbors(plan, g.DeviceBatch.from_batch(b), g.Workspace())


def test_nonfinite_position_is_rejected(g):
    say("[non-finite position]")
    rng = np.random.default_rng(5)
    pos, spec, cell, pbc = gs.small_periodic(rng, n_atoms=6, n_elements=2, density=0.06, dmin=1.3)
    pos = pos.copy()
    pos[3, 1] = np.nan
    b = gs.make_batch([(pos, spec, cell, pbc)])
    plan = g.GMPPlan.from_probes(_probes(), "fp32c")
    with pytest.raises(g.GMPError, match="NONFINITE"):
        g.build_neighbors(plan, g.DeviceBatch.from_batch(b), g.Workspace())


def test_singular_cell_is_rejected(g):
    say("[singular cell]")
    rng = np.random.default_rng(6)
    pos, spec, cell, pbc = gs.small_periodic(rng, n_atoms=4, n_elements=2, density=0.06, dmin=1.3)
    cell = np.array(cell, float).copy()
    cell[2] = cell[0] + cell[1]
    b = gs.make_batch([(pos, spec, cell, 7)])
    plan = g.GMPPlan.from_probes(_probes(), "fp32c")
    with pytest.raises(g.GMPError, match="CELL"):
        g.build_neighbors(plan, g.DeviceBatch.from_batch(b), g.Workspace())


def _lattice_probes(tau, n_elements=1):
    return gs.Probes(np.array([0, 1, 2], np.int32), np.array([3.0]), np.arange(n_elements + 1, dtype=np.int32),
                     np.full(n_elements, 5.0), np.full(n_elements, 0.3), tau)


@pytest.mark.parametrize("n_atoms,tau", [(1, 1e-14), (2, 1e-17)])
def test_lists_longer_than_8192(g, n_atoms, tau):
    """Atoms in a 1.8 A cubic cell with 26-29 A cutoffs: one atom (one
    bucket of ~12,600 images, sorted in the enlarged LDS sort) and two atoms
    of two species (~33,000 neighbours per centre in two buckets of ~16,500,
    more than the sort holds: filled one bucket range at a time).  Lists
    bit-exact against the oracle, features within 1e-11 (FP64) where they
    are not the cancelled remainder of symmetric images."""
    p = _lattice_probes(tau, n_atoms)
    pos = np.array([[0.0, 0.0, 0.0], [0.9, 0.8, 0.7]])[:n_atoms]
    b = gs.make_batch([(pos, np.arange(n_atoms, dtype=np.int32), np.eye(3) * 1.8, 7)])
    plan = g.GMPPlan.from_probes(p, "fp64")
    db = g.DeviceBatch.from_batch(b)
    ws = g.Workspace()
    nb = g.build_neighbors(plan, db, ws)
    F, _ = g.features(plan, db, nb, ws)
    torch.cuda.synchronize()
    sizes = np.diff(nb.offsets.cpu().numpy())
    say(f"[long lists] {n_atoms} atoms: list lengths {sizes.tolist()}")
    assert sizes.min() > 12000
    from gpu_helpers import check_lists_many
    assert check_lists_many(nb, b, p, 0) == n_atoms
    # features that vanish by the lattice's symmetry are rounding residuals
    # of ~1e4 cancelling images on both sides (kappa = F_abs / F ~ 1e13): the
    # bar there is the FP64 rounding of the terms, 64 * 2^-53 * F_abs
    Fref = oracle.features_batch(b, p)
    Fabs = oracle.features_abs(b.structure(0), p)
    err = np.abs(F.cpu().numpy() - Fref)
    ok = (err <= 1e-11 * Fref) | (err <= 64 * 2.0 ** -53 * Fabs) | ((Fref <= p.tau) & (err <= p.tau))
    assert ok.all(), float(err.max())
    good = Fref > 1e-8 * Fabs
    assert good.any() and np.all(err[good] <= 1e-11 * Fref[good])


def test_bucket_longer_than_the_sort_is_unsupported(g):
    """One atom in the 1.8 A cell with a ~35 A cutoff: a single bucket of
    ~30,000 images, more than the 160 KB LDS sort holds."""
    p = _lattice_probes(1e-25)
    rc = float(np.sqrt(oracle.cutoffs(p).max()))
    assert 33.0 < rc < 37.0
    b = gs.make_batch([(np.zeros((1, 3)), np.zeros(1, np.int32), np.eye(3) * 1.8, 7)])
    plan = g.GMPPlan.from_probes(p, "fp64")
    with pytest.raises(g.GMPError, match="UNSUPPORTED"):
        g.build_neighbors(plan, g.DeviceBatch.from_batch(b), g.Workspace())


def test_nosync_bucket_longer_than_the_long_sort_is_stale(g):
    """One atom in the 1.8 A cell with a ~27 A cutoff: one bucket of ~12,600
    images, which the long-list sort holds.  Shrunk by 20% in place, the
    no-sync rebuild of a captured step meets a bucket of ~24,000 images,
    more than the 160 KB LDS sort holds: the captured step's status word
    reports GMP_E_STALE, and a synchronous build GMP_E_UNSUPPORTED."""
    p = _lattice_probes(1e-14)
    b = gs.make_batch([(np.zeros((1, 3)), np.zeros(1, np.int32), np.eye(3) * 1.8, 7)])
    plan = g.GMPPlan.from_probes(p, "fp64")
    db = g.DeviceBatch.from_batch(b)
    ws = g.Workspace()
    nb0 = g.build_neighbors(plan, db, ws)
    assert 12000 < nb0.n_pairs < 14000
    nbc = g.build_neighbors(plan, db, ws, capacity=3 * nb0.n_pairs)
    step = g.CapturedStep(plan, db, ws, nbc, backward=False)
    step.replay()
    step.check_status()
    db.xyz.mul_(0.8)
    db.cell.mul_(0.8)
    step.replay()
    with pytest.raises(g.GMPError) as ei:
        step.check_status()
    assert ei.value.status == 8  # GMP_E_STALE
    with pytest.raises(g.GMPError, match="UNSUPPORTED"):
        g.build_neighbors(plan, db, g.Workspace())
