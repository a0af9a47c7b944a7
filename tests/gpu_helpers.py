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


def check_reverse(nb):
    """Every pair's reverse entry is its mirror (j, i, -n) -- checked on the GPU."""
    import torch
    P = nb.n_pairs
    offs = nb.offsets
    cnt = offs[1:] - offs[:-1]
    centre = torch.repeat_interleave(torch.arange(len(cnt), device=offs.device, dtype=torch.int64), cnt)
    J = nb.j[:P].long()
    rev = nb.reverse[:P].long()
    assert bool((rev >= 0).all()) and bool((rev < cnt[J]).all())
    tgt = offs[J] + rev
    assert bool((J[tgt] == centre).all())
    w = nb.shift[:P]
    nk = [((w >> (8 * k)) & 0xff).to(torch.int8) for k in range(3)]
    for k in range(3):
        assert bool((nk[k][tgt].int() == -nk[k].int()).all())


def check_neighbors(nb, batch_np, probes, centres=None):
    """Bit-exact comparison of the canonical lists (j, shift, species byte),
    the bucket starts and the sigma-prefix ends with the oracle, for all
    centres or the sampled ones ({structure: [local centres]}), plus the
    reverse index of every pair."""
    rc2 = oracle.cutoffs(probes)
    offs = nb.offsets.cpu().numpy()
    P = int(offs[-1])
    assert P == nb.n_pairs
    E, S = probes.n_elements, oracle.n_slots(probes)
    if nb.reverse is not None:
        check_reverse(nb)
    wrap_all = nb.wrap.view(-1, 3)
    rw_all = nb.rw.view(3, -1)
    checked = 0
    for s in range(batch_np.n_structs):
        loc = None if centres is None else centres.get(s, [])
        if loc is not None and len(loc) == 0:
            continue
        a0, a1 = int(batch_np.atom_offsets[s]), int(batch_np.atom_offsets[s + 1])
        struct = batch_np.structure(s)
        orw, om = oracle.wrap(struct[0], struct[2], struct[3])
        assert np.array_equal(wrap_all[a0:a1].cpu().numpy(), om)
        assert rw_all[:, a0:a1].t().contiguous().cpu().numpy().tobytes() == orw.tobytes()
        if loc is None:
            loc = range(a1 - a0)
        for li in loc:
            gi = a0 + li
            ref = oracle.neighbors(struct, rc2, li)
            lo, hi = int(offs[gi]), int(offs[gi + 1])
            assert hi - lo == len(ref["j"]), (s, li, hi - lo, len(ref["j"]))
            J = nb.j[lo:hi].cpu().numpy()
            w = nb.shift[lo:hi].cpu().numpy().view(np.uint8).reshape(-1, 4)
            n = w[:, :3].view(np.int8).astype(np.int32)
            e = w[:, 3].astype(np.int32)
            assert np.array_equal(J, ref["j"] + a0)
            assert np.array_equal(n, ref["n"])
            assert np.array_equal(e, ref["e"])
            bs = nb.bucket_start[gi * (S * E + 1):(gi + 1) * (S * E + 1)].cpu().numpy()
            se = nb.sigma_end[gi * S:(gi + 1) * S].cpu().numpy()
            bucket = ref["shell"] * E + ref["e"]
            assert np.array_equal(bs, np.searchsorted(np.sort(bucket), np.arange(S * E + 1), side="left"))
            assert np.array_equal(se, np.array([int(np.sum(ref["q"] <= rc2[t])) for t in range(S)]))
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
