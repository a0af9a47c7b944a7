"""Shared helpers of the GPU parity tests: run the HIP path through the
C ABI and compare with the FP64 oracle."""
import sys

import numpy as np

import oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_path(g, batch_np, probes, precision, ws, reverse=True, tuning=None):
    import torch
    plan = g.GMPPlan.from_probes(probes, precision)
    if tuning:
        plan.set_tuning(**tuning)
    db = g.DeviceBatch.from_batch(batch_np)
    nb = g.build_neighbors(plan, db, ws, reverse=reverse)
    F, mu = g.features(plan, db, nb, ws)
    torch.cuda.synchronize()
    return plan, db, nb, F, mu


def check_neighbors(nb, batch_np, probes, centres=None):
    """Bit-exact comparison of the canonical lists (j, shift, species byte),
    the species-segment starts and the sigma-prefix ends with the oracle."""
    rc2 = oracle.cutoffs(probes)
    offs = nb.offsets.cpu().numpy()
    P = int(offs[-1])
    assert P == nb.n_pairs
    J = nb.j[:P].cpu().numpy()
    n, e = nb.shifts_numpy()
    E, S = probes.n_elements, len(probes.sigmas)
    bs = nb.bucket_start.cpu().numpy().reshape(-1, S * E + 1)
    se = nb.sigma_end.cpu().numpy().reshape(-1, S)
    wrap = nb.wrap.cpu().numpy().reshape(-1, 3)
    rw = nb.rw.cpu().numpy().reshape(3, -1).T
    if nb.reverse is not None:
        # every pair's reverse entry is its mirror (j, i, -n)
        rev = nb.reverse[:P].cpu().numpy().astype(np.int64)
        assert np.all(rev >= 0)
        centre = np.repeat(np.arange(len(offs) - 1), np.diff(offs))
        tgt = offs[J] + rev
        assert np.all(rev < np.diff(offs)[J])
        assert np.array_equal(J[tgt], centre)
        assert np.array_equal(n[tgt], -n)
    checked = 0
    for s in range(batch_np.n_structs):
        a0, a1 = int(batch_np.atom_offsets[s]), int(batch_np.atom_offsets[s + 1])
        struct = batch_np.structure(s)
        orw, om = oracle.wrap(struct[0], struct[2], struct[3])
        assert np.array_equal(wrap[a0:a1], om)
        assert rw[a0:a1].tobytes() == orw.tobytes()
        loc = range(a1 - a0) if centres is None else [c for c in centres.get(s, [])]
        for li in loc:
            gi = a0 + li
            ref = oracle.neighbors(struct, rc2, li)
            lo, hi = int(offs[gi]), int(offs[gi + 1])
            assert hi - lo == len(ref["j"]), (s, li, hi - lo, len(ref["j"]))
            assert np.array_equal(J[lo:hi], ref["j"] + a0)
            assert np.array_equal(n[lo:hi], ref["n"])
            assert np.array_equal(e[lo:hi], ref["e"])
            # bucket starts (shell-major, species-minor) and sigma prefixes
            bucket = ref["shell"] * E + ref["e"]
            for b in range(S * E + 1):
                assert bs[gi, b] == int(np.sum(bucket < b))
            for ss in range(S):
                assert se[gi, ss] == int(np.sum(ref["q"] <= rc2[ss]))
            checked += 1
    return checked


def feature_errors(F, Fref, tau):
    """Per-feature errors under the tolerance rule: relative error where the
    oracle feature exceeds the overlap threshold, absolute error elsewhere."""
    F = np.asarray(F, np.float64)
    big = Fref > tau
    rel = np.zeros_like(Fref)
    rel[big] = np.abs(F[big] - Fref[big]) / Fref[big]
    ab = np.where(big, 0.0, np.abs(F - Fref))
    return float(rel.max(initial=0.0)), float(ab.max(initial=0.0))


def assert_features(F, Fref, tau, rel_tol):
    r, a = feature_errors(F, Fref, tau)
    assert r <= rel_tol, f"max relative error {r:.3e} > {rel_tol:.1e}"
    assert a <= tau, f"max absolute error below threshold {a:.3e} > {tau:.1e}"
    return r, a
