"""Neighbour set of the oracle against an independent vectorised brute force
(numpy, a much larger image box, the same floating-point operation order),
bit for bit; the symmetry of the relation; and membership semantics checked
against a plain distance computation away from the cutoff."""
import numpy as np
import pytest

import gmp_synth as gs
import oracle


def _cross(a, b):
    return np.array([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]])


def _np_wrap(pos, cell, pbc):
    if not pbc:
        return pos.copy(), np.zeros((len(pos), 3), np.int64)
    a1, a2, a3 = cell
    c23, c31, c12 = _cross(a2, a3), _cross(a3, a1), _cross(a1, a2)
    V = (a1[0] * c23[0] + a1[1] * c23[1]) + a1[2] * c23[2]
    b = np.stack([c23 / V, c31 / V, c12 / V])
    f = (pos[:, 0:1] * b[:, 0] + pos[:, 1:2] * b[:, 1]) + pos[:, 2:3] * b[:, 2]
    m = np.where([(pbc >> k) & 1 for k in range(3)], np.floor(f), 0.0)
    t = m[:, 0:1] * a1 + m[:, 1:2] * a2
    t = t + m[:, 2:3] * a3
    return pos - t, m.astype(np.int64)


def _np_neighbors(struct, rc2, centre, box=None):
    pos, spec, cell, pbc = struct
    rw, m = _np_wrap(np.asarray(pos, float), np.asarray(cell, float), pbc)
    rcmax2 = rc2.max()
    if box is None:
        box = 6
    rngs = [np.arange(-box, box + 1) if (pbc >> k) & 1 else np.array([0]) for k in range(3)]
    out = []
    for n1 in rngs[0]:
        for n2 in rngs[1]:
            for n3 in rngs[2]:
                if pbc:
                    sh = (float(n1) * cell[0] + float(n2) * cell[1]) + float(n3) * cell[2]
                else:
                    sh = np.zeros(3)
                d = (rw - rw[centre]) + sh
                q = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
                for j in np.flatnonzero(q <= rcmax2):
                    shell = int(np.sum(rc2 < q[j]))
                    out.append((shell, int(spec[j]), int(j), int(n1), int(n2), int(n3), q[j]))
    out.sort(key=lambda t: t[:6])
    return out


CASES = {
    "triclinic": lambda r: gs.small_periodic(r, n_atoms=10, density=0.06, dmin=1.3),
    "tiny_cell_many_images": lambda r: gs.small_periodic(r, n_atoms=3, density=0.08, dmin=1.0),
    "cluster": lambda r: gs.small_cluster(r, n_atoms=9, radius=3.5),
    "slab_pbc_xy": lambda r: gs.small_periodic(r, n_atoms=8, density=0.04, dmin=1.3, pbc=3),
}


@pytest.mark.parametrize("case", list(CASES))
def test_neighbors_bit_exact_vs_numpy(case):
    rng = np.random.default_rng(abs(hash(case)) % 1000)
    struct = CASES[case](rng)
    probes = gs.small_probes(rng, n_sigmas=3, tau=1e-6)
    rc2 = oracle.cutoffs(probes)
    for i in range(len(struct[0])):
        ref = _np_neighbors(struct, rc2, i)
        got = oracle.neighbors(struct, rc2, i)
        assert len(got["j"]) == len(ref)
        for k, t in enumerate(ref):
            assert (int(got["shell"][k]), int(got["e"][k]), int(got["j"][k]), *map(int, got["n"][k])) == t[:6]
            assert got["q"][k].tobytes() == np.float64(t[6]).tobytes()


@pytest.mark.parametrize("case", list(CASES))
def test_relation_is_symmetric(case):
    rng = np.random.default_rng(7 + len(case))
    struct = CASES[case](rng)
    probes = gs.small_probes(rng, n_sigmas=2, tau=1e-6)
    rc2 = oracle.cutoffs(probes)
    lists = [oracle.neighbors(struct, rc2, i) for i in range(len(struct[0]))]
    table = {}
    for i, nb in enumerate(lists):
        for j, n, q in zip(nb["j"], nb["n"], nb["q"]):
            table[(i, int(j), tuple(int(x) for x in n))] = q.tobytes()
    for (i, j, n), qb in table.items():
        assert table[(j, i, tuple(-x for x in n))] == qb


def test_membership_matches_plain_distance():
    """Away from the cutoff surface, (j, n) is a neighbour exactly when the
    Cartesian image distance is below rc_max (no wrapping in the reference)."""
    rng = np.random.default_rng(31)
    pos, spec, cell, pbc = gs.small_periodic(rng, n_atoms=7, density=0.05, dmin=1.3)
    probes = gs.small_probes(rng, n_sigmas=2, tau=1e-6)
    rc2 = oracle.cutoffs(probes)
    rc = np.sqrt(rc2.max())
    _, m = oracle.wrap(pos, cell, pbc)
    for i in range(len(pos)):
        nb = oracle.neighbors((pos, spec, cell, pbc), rc2, i)
        got = {(int(j), *(int(x) for x in (n - m[j] + m[i]))) for j, n in zip(nb["j"], nb["n"])}
        ref = set()
        for n1 in range(-8, 9):
            for n2 in range(-8, 9):
                for n3 in range(-8, 9):
                    d = pos - pos[i] + np.array([n1, n2, n3]) @ cell
                    r = np.linalg.norm(d, axis=1)
                    for j in np.flatnonzero(r < rc - 1e-9):
                        ref.add((int(j), n1, n2, n3))
                    for j in np.flatnonzero(np.abs(r - rc) <= 1e-9):
                        pytest.skip("pair on the cutoff surface")
        assert got == ref


def test_every_sigma_uses_a_prefix():
    """In canonical order the pairs a sigma uses (q <= rc(sigma)^2) come first."""
    rng = np.random.default_rng(51)
    struct = gs.small_periodic(rng, n_atoms=9, n_elements=3, density=0.06, dmin=1.3)
    probes = gs.small_probes(rng, n_sigmas=4, n_elements=3, tau=1e-7)
    rc2 = oracle.cutoffs(probes)
    for i in range(len(struct[0])):
        nb = oracle.neighbors(struct, rc2, i)
        for s in range(len(rc2)):
            used = nb["q"] <= rc2[s]
            k = int(used.sum())
            assert used[:k].all() and not used[k:].any()


def test_self_images_present_when_cutoff_exceeds_cell():
    rng = np.random.default_rng(41)
    pos, spec, cell, pbc = np.zeros((1, 3)), np.zeros(1, np.int32), np.eye(3) * 3.0, 7
    probes = gs.small_probes(rng, n_elements=1, n_sigmas=1, tau=1e-6)
    rc2 = oracle.cutoffs(probes)
    nb = oracle.neighbors((pos, spec, cell, pbc), rc2, 0)
    n = nb["n"]
    # every lattice point within rc, including the centre itself
    exp_count = sum(1 for a in range(-10, 11) for b in range(-10, 11) for c in range(-10, 11)
                    if 9.0 * (a * a + b * b + c * c) <= rc2.max())
    assert len(n) == exp_count
    assert (0, 0, 0) in {tuple(x) for x in n}
