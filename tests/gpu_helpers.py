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
    """Every pair's reverse entry is its mirror (j, i, -n) -- checked on the GPU.
    Lists are stored per list slot: slot k holds the list of centre order[k]."""
    import torch
    P = nb.n_pairs
    offs = nb.offsets
    cnt = offs[1:] - offs[:-1]
    N = len(cnt)
    order, slot = nb.order[:N].long(), nb.slot[:N].long()
    assert torch.equal(order[slot], torch.arange(N, device=offs.device)), "order and slot are not inverse"
    centre = order[torch.repeat_interleave(torch.arange(N, device=offs.device, dtype=torch.int64), cnt)]
    J = nb.j[:P].long()
    tgt = nb.reverse[:P].long()  # pair index of the mirror
    kj = slot[J]
    assert bool((tgt >= offs[kj]).all()) and bool((tgt < offs[kj + 1]).all()), "mirror outside j's list"
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
    slot = nb.slot.cpu().numpy()
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
            ki = int(slot[gi])  # list slot of atom gi
            lo, hi = int(offs[ki]), int(offs[ki + 1])
            assert hi - lo == len(ref["j"]), (s, li, hi - lo, len(ref["j"]))
            J = nb.j[lo:hi].cpu().numpy()
            w = nb.shift[lo:hi].cpu().numpy().view(np.uint8).reshape(-1, 4)
            n = w[:, :3].view(np.int8).astype(np.int32)
            e = w[:, 3].astype(np.int32)
            assert np.array_equal(J, ref["j"] + a0)
            assert np.array_equal(n, ref["n"])
            assert np.array_equal(e, ref["e"])
            bs = nb.bucket_start[ki * (S * E + 1):(ki + 1) * (S * E + 1)].cpu().numpy()
            se = nb.sigma_end[ki * S:(ki + 1) * S].cpu().numpy()
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


def check_lists_many(nb, batch_np, probes, s, local=None):
    """Bit-exact comparison, vectorized over many centres, of structure s's
    lists (j, shifts, species byte, bucket starts, sigma-prefix ends, wrap
    indices and wrapped positions) with the oracle's lists of the same
    centres (local indices; None = every atom of the structure).  Returns
    the number of centres checked."""
    rc2 = oracle.cutoffs(probes)
    E, S = probes.n_elements, oracle.n_slots(probes)
    a0, a1 = int(batch_np.atom_offsets[s]), int(batch_np.atom_offsets[s + 1])
    struct = batch_np.structure(s)
    loc = np.arange(a1 - a0, dtype=np.int32) if local is None else np.asarray(local, np.int32)
    orw, om = oracle.wrap(struct[0], struct[2], struct[3])
    assert np.array_equal(nb.wrap.view(-1, 3)[a0:a1].cpu().numpy(), om)
    assert nb.rw.view(3, -1)[:, a0:a1].t().contiguous().cpu().numpy().tobytes() == orw.tobytes()
    ref = oracle.neighbors_many(struct, rc2, loc)
    offs = nb.offsets.cpu().numpy()
    gi = nb.slot.cpu().numpy()[a0 + loc.astype(np.int64)].astype(np.int64)  # list slots of the centres
    lo, hi = offs[gi], offs[gi + 1]
    cnt = hi - lo
    assert np.array_equal(cnt, np.diff(ref["offs"])), "list lengths differ"
    idx = np.repeat(lo - ref["offs"][:-1], cnt) + np.arange(int(cnt.sum()))
    import torch
    it = torch.as_tensor(idx, device=nb.j.device)
    J = nb.j[it].cpu().numpy()
    w = nb.shift[it].cpu().numpy().view(np.uint8).reshape(-1, 4)
    assert np.array_equal(J, ref["j"] + a0), "neighbour indices differ"
    assert np.array_equal(w[:, :3].view(np.int8).astype(np.int32), ref["n"]), "image shifts differ"
    assert np.array_equal(w[:, 3].astype(np.int32), ref["e"]), "species bytes differ"
    k = len(loc)
    owner = np.repeat(np.arange(k), cnt)
    bucket = ref["shell"] * E + ref["e"]
    per = np.bincount(owner * (S * E) + bucket, minlength=k * S * E).reshape(k, S * E)
    bs_ref = np.concatenate([np.zeros((k, 1), np.int64), np.cumsum(per, axis=1)], axis=1)
    bs = nb.bucket_start.view(-1, S * E + 1)[torch.as_tensor(gi, device=nb.j.device)].cpu().numpy()
    assert np.array_equal(bs, bs_ref), "bucket starts differ"
    se_ref = np.stack([np.bincount(owner, weights=(ref["q"] <= rc2[t]), minlength=k) for t in range(S)], 1)
    se = nb.sigma_end.view(-1, S)[torch.as_tensor(gi, device=nb.j.device)].cpu().numpy()
    assert np.array_equal(se, se_ref.astype(np.int64)), "sigma-prefix ends differ"
    return k


def conditioning(Fabs, Fref, tau):
    """kappa = F_abs / F_ref per feature above the threshold (inf elsewhere):
    F_abs is the feature of the absolute values of the pair terms, so a large
    kappa says a feature is the small remainder of cancelling terms, whose
    FP32 error is bounded by about 2^-24 F_abs rather than 2^-24 F_ref."""
    Fabs = np.asarray(Fabs, np.float64)
    out = np.full(Fref.shape, np.inf)
    big = Fref > tau
    out[big] = Fabs[big] / Fref[big]
    return out
