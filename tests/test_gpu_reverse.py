"""Reverse-pair index on buckets of every size: one species and one cutoff
slot put a centre's whole list in one bucket, and the overlap threshold
sweeps the list length across multiples of 16 (the reverse search first
bisects every 16th key of the partner's bucket, then a 16-key window).
Lists bit-exact against the oracle, every pair's reverse entry its mirror."""
import numpy as np
import pytest

import gmp_synth as gs
import oracle
from gpu_helpers import say, run_path, check_neighbors

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


@pytest.mark.parametrize("tau", [1e-5, 3e-6, 1e-7, 1e-10, 1e-14, 1e-20])
def test_reverse_index_across_bucket_sizes(g, ws, tau):
    rng = np.random.default_rng(91)
    structs = [gs.small_periodic(rng, n_atoms=n, n_elements=1, density=0.05, dmin=1.1) for n in (3, 8, 13)]
    structs.append(gs.small_cluster(rng, n_atoms=21, n_elements=1, radius=4.0))
    b = gs.make_batch(structs)
    p = gs.Probes(np.array([0], np.int32), np.array([0.5]), np.array([0, 1], np.int32),
                  np.array([1.0]), np.array([1.0]), tau)
    say(f"[reverse index, tau={tau:g}: rc={np.sqrt(oracle.cutoffs(p)[0]):.2f} A]")
    plan, db, nb, F, mu = run_path(g, b, p, "fp32c", ws)
    sizes = np.diff(nb.offsets.cpu().numpy())
    say(f"  list lengths {sizes.min()}..{sizes.max()}, {int(nb.n_pairs)} pairs")
    check_neighbors(nb, b, p)
