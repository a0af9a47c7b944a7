"""Throughput of the GMP feature path on one MI355X.

Workload: the single-structure "plain method at scale" case -- a periodic
40 x 40 x 40 A cell with 4096 atoms of 5 elements (Dirichlet proportions,
minimum pair distance 1.6 A), 5 Gaussian primitives per element
(B log-uniform [0.01, 10], beta log-uniform [0.1, 30] 1/A^2), probes
l = 0..4 x 8 sigmas log-spaced 0.1..1.6 A (40 features per atom),
overlap threshold 1e-11; synthetic, seeded.

One step = the whole hot path on that batch: lattice wrap + cell list +
neighbour lists (with reverse index), forward features (overlap + norm),
and the adjoint with a seeded N(0,1) upstream gradient (dL/dR, dL/dcell),
recorded once into a HIP graph and replayed once per step (the neighbour
build runs in its no-sync mode with the capacity of a first, synchronous
build).  The reported value is atoms*features/s of that step in the FP32
compensated path; the FP32-wide and FP64 paths, forward-only rates and
eager (one host call per stage) timings are reported beside it.
Per-kernel durations come from HIP events recorded by the library around
each launch on the launch stream (torch's current stream) in separate
eager steps.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# autotuner choices of this run (a fresh box searches; the file is a scratch cache)
TUNE_CACHE = os.path.join(ROOT, "gpurun_out", "tune_cache.json")
PEAK_FP32_TFLOPS = 157.3     # MI355X vector FP32 (packed issue)
# non-packed FP32 FMA: 256 CU x 4 SIMD x 16 lanes x 2 flops x 2.4 GHz (this build issues no packed FP32)
PEAK_FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
PEAK_FP64_TFLOPS = 78.6      # MI355X vector FP64
PEAK_HBM_GBS = 8000.0
# v_exp_f32 is a quarter-rate transcendental: 256 CU x 4 SIMD x 16 lanes / 4 x 2.4 GHz
PEAK_EXP_PER_S = 256 * 4 * 16 / 4 * 2.4e9
# one wavefront VALU instruction per CU per cycle (4 SIMD x 16 lanes, 64-wide waves)
VALU_WAVE_INSTS_PER_S = 256 * 2.4e9


def counter_record(kernel):
    """Counter figures committed under profiles/ for this kernel, or None
    when the kernel's sources changed since they were taken."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "counters_C2.json")) as f:
            rec = json.load(f)["kernels"][kernel]
    except (OSError, KeyError, ValueError):
        return None
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    return rec if h.hexdigest() == rec["sources_sha256"] else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="C2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--sample-centres", type=int, default=48)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-per-structure comparison")
    ap.add_argument("--no-split", action="store_true",
                    help="skip the eager steps whose reverse search runs on a second stream (kernel traces "
                         "then hold no launches slowed by a concurrent kernel)")
    ap.add_argument("--no-others", action="store_true", help="skip the other workloads (512 structures, 1e5 atoms)")
    ap.add_argument("--no-density", action="store_true",
                    help="skip the order -1 (local density), occupancy (disordered), reference-point, Jacobian and "
                         "screening variants")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 256 MiB device copy three times (counter calibration)")
    return ap.parse_args()


def _median_ms(fn, reps, torch):
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t) * 1e3)
    return float(np.median(ts))


def other_workloads(g, gs, torch, steps=5, warmup=2):
    from paper_2303_12980_amd import autotune
    """Graph-replayed fwd+bwd step (FP32 compensated, neighbour build
    included) on the differentiation workload (512 periodic triclinic
    structures of 32-200 atoms, l=0..3 x 6 sigma) and on the large single
    system (100,000 atoms in a 102.8 A cubic cell, l=0..4 x 10 sigma)."""
    out = {}
    for name, label in (("C4", "512 periodic triclinic structures, 32-200 atoms, 4 elements, l=0..3 x 6 sigma"),
                        ("C5", "periodic 102.8 A cubic cell, 100000 atoms, 6 elements, l=0..4 x 10 sigma")):
        t0 = time.time()
        batch, probes = gs.config(name)
        gen_s = time.time() - t0
        db = g.DeviceBatch.from_batch(batch)
        plan = g.GMPPlan.from_probes(probes, "fp32c")
        ws = g.Workspace()
        tune = autotune.autotune(plan, db, ws, candidates=autotune.STEP_CANDIDATES, backward=True, reps=2,
                                 cache_path=TUNE_CACHE)
        nb = g.build_neighbors(plan, db, ws)
        G = torch.as_tensor(np.random.default_rng(7).standard_normal((batch.n_atoms, probes.n_features)),
                            device="cuda")
        split = bool(tune.get("concurrent_reverse", False))
        fb = g.CapturedStep(plan, db, ws, nb, backward=True, G=G, concurrent_reverse=split)
        nbf = g.build_neighbors(plan, db, ws, reverse=False)
        fo = g.CapturedStep(plan, db, ws, nbf, backward=False)
        for _ in range(warmup):
            fb.replay()
            fo.replay()
        t_fb = _median_ms(fb.replay, steps, torch)
        t_fo = _median_ms(fo.replay, steps, torch)
        g.check_status(ws)
        af = batch.n_atoms * probes.n_features
        out[name] = {"workload": label, "atoms": batch.n_atoms, "features_per_atom": probes.n_features,
                     "pairs": int(nb.n_pairs),
                     "tuning": dict(tune["tuning"], searched=not tune["cached"], concurrent_reverse=split),
                     "fwd_bwd_ms": t_fb, "fwd_ms": t_fo,
                     "atoms_features_per_s_fwd_bwd": af / (t_fb * 1e-3), "atoms_features_per_s_fwd": af / (t_fo * 1e-3)}
        print(f"[bench] {name}: {batch.n_atoms} atoms, {nb.n_pairs} pairs (generated in {gen_s:.1f}s), tuning "
              f"{tune['tuning']}, reverse search on a second stream: {split}: fwd+bwd {t_fb:.2f} ms, "
              f"fwd {t_fo:.2f} ms", file=sys.stderr, flush=True)
        del fb, fo, nb, nbf, ws, db, G
        torch.cuda.empty_cache()
    return out


def density_variant(g, gs, torch, batch, probes, db, steps=10, warmup=3):
    """The same 4096-atom cell with order -1 (the local density, one feature
    without a width) added in front of the orders: graph-replayed fwd+bwd
    and fwd steps in FP32 compensated mode, and the FP64 oracle on sampled
    centres for the accuracy of the density feature."""
    import oracle
    pd = gs.Probes(np.concatenate([[-1], probes.orders]).astype(np.int32), probes.sigmas, probes.prim_offsets,
                   probes.B, probes.beta, probes.tau)
    N, nf = batch.n_atoms, pd.n_features
    plan = g.GMPPlan.from_probes(pd, "fp32c")
    ws = g.Workspace()
    nb = g.build_neighbors(plan, db, ws)
    nbf = g.build_neighbors(plan, db, ws, reverse=False)
    G = torch.as_tensor(np.random.default_rng(7).standard_normal((N, nf)), device="cuda")
    fb = g.CapturedStep(plan, db, ws, nb, backward=True, G=G)
    fo = g.CapturedStep(plan, db, ws, nbf, backward=False)
    for _ in range(warmup):
        fb.replay()
        fo.replay()
    t_fb = _median_ms(fb.replay, steps, torch)
    t_fo = _median_ms(fo.replay, steps, torch)
    g.check_status(ws)
    cs = np.sort(np.random.default_rng(13).choice(N, size=min(24, N), replace=False))
    Fref = oracle.features(batch.structure(0), pd, centres=cs)
    Fg = fb.F.double().cpu().numpy()[cs]
    big = Fref > pd.tau
    out = {"orders": [int(x) for x in pd.orders], "features_per_atom": nf, "n_slots": plan.n_slots,
           "density_rc2": float(plan.rc2[-1]), "pairs": int(nb.n_pairs), "fwd_bwd_ms": t_fb, "fwd_ms": t_fo,
           "atoms_features_per_s_fwd_bwd": N * nf / (t_fb * 1e-3), "atoms_features_per_s_fwd": N * nf / (t_fo * 1e-3),
           "density_max_rel_err": float(np.max(np.abs(Fg[:, 0] - Fref[:, 0]) / Fref[:, 0])),
           "all_max_rel_err": float(np.max(np.abs(Fg[big] - Fref[big]) / Fref[big])), "sampled_centres": len(cs)}
    print(f"[bench] order -1 added: fwd+bwd {t_fb:.3f} ms, fwd {t_fo:.3f} ms, density max rel err "
          f"{out['density_max_rel_err']:.2e}", file=sys.stderr, flush=True)
    del fb, fo, nb, nbf, ws, G
    torch.cuda.empty_cache()
    return out


def occupancy_variant(g, gs, torch, batch, probes, steps=10, warmup=3):
    """The same 4096-atom cell as a disordered structure: every atom given a
    fractional occupancy in [0.5, 1] (same pair set): graph-replayed fwd+bwd
    and fwd steps in FP32 compensated mode, and the FP64 oracle on sampled
    centres."""
    import oracle
    occ = np.random.default_rng(17).uniform(0.5, 1.0, batch.n_atoms)
    bo = gs.Batch(batch.atom_offsets, batch.pos, batch.species, batch.cell, batch.pbc, occ)
    N, nf = batch.n_atoms, probes.n_features
    db = g.DeviceBatch.from_batch(bo)
    plan = g.GMPPlan.from_probes(probes, "fp32c")
    ws = g.Workspace()
    nb = g.build_neighbors(plan, db, ws)
    nbf = g.build_neighbors(plan, db, ws, reverse=False)
    G = torch.as_tensor(np.random.default_rng(7).standard_normal((N, nf)), device="cuda")
    fb = g.CapturedStep(plan, db, ws, nb, backward=True, G=G)
    fo = g.CapturedStep(plan, db, ws, nbf, backward=False)
    for _ in range(warmup):
        fb.replay()
        fo.replay()
    t_fb = _median_ms(fb.replay, steps, torch)
    t_fo = _median_ms(fo.replay, steps, torch)
    g.check_status(ws)
    cs = np.sort(np.random.default_rng(19).choice(N, size=min(24, N), replace=False))
    Fref = oracle.features(batch.structure(0), probes, centres=cs, occupancy=occ)
    Fg = fb.F.double().cpu().numpy()[cs]
    big = Fref > probes.tau
    out = {"occupancy": "uniform [0.5, 1] on every atom", "pairs": int(nb.n_pairs), "fwd_bwd_ms": t_fb,
           "fwd_ms": t_fo, "atoms_features_per_s_fwd_bwd": N * nf / (t_fb * 1e-3),
           "max_rel_err": float(np.max(np.abs(Fg[big] - Fref[big]) / Fref[big])), "sampled_centres": len(cs)}
    print(f"[bench] occupancies: fwd+bwd {t_fb:.3f} ms, fwd {t_fo:.3f} ms, max rel err {out['max_rel_err']:.2e}",
          file=sys.stderr, flush=True)
    del fb, fo, nb, nbf, ws, G, db
    torch.cuda.empty_cache()
    return out


def points_variant(g, gs, torch, batch, probes, steps=10, warmup=3):
    """Features at reference points of the 4096-atom cell: a 16x16x16 grid
    of points (cell centres of a regular fractional grid) as the centres;
    graph-replayed fwd+bwd (gradients with respect to atoms, points and
    cell) and fwd steps in FP32 compensated mode, and the FP64 oracle on
    sampled points."""
    import oracle
    cell = batch.cell[0]
    f = (np.stack(np.meshgrid(*[np.arange(16)] * 3, indexing="ij"), -1).reshape(-1, 3) + 0.5) / 16.0
    pts = f @ cell
    M, nf = len(pts), probes.n_features
    db = g.DeviceBatch.from_batch(batch).with_points(pts, [0, M])
    plan = g.GMPPlan.from_probes(probes, "fp32c")
    ws = g.Workspace()
    nb = g.build_neighbors(plan, db, ws)
    G = torch.as_tensor(np.random.default_rng(7).standard_normal((M, nf)), device="cuda")
    fb = g.CapturedStep(plan, db, ws, nb, backward=True, G=G)
    fo = g.CapturedStep(plan, db, ws, nb, backward=False)
    for _ in range(warmup):
        fb.replay()
        fo.replay()
    t_fb = _median_ms(fb.replay, steps, torch)
    t_fo = _median_ms(fo.replay, steps, torch)
    g.check_status(ws)
    cs = np.sort(np.random.default_rng(23).choice(M, size=24, replace=False))
    Fref = oracle.point_features(batch.structure(0), probes, pts[cs])
    Fg = fb.F.double().cpu().numpy()[cs]
    big = Fref > probes.tau
    out = {"points": "16x16x16 grid in the 40 A cell", "n_points": M, "pairs": int(nb.n_pairs),
           "fwd_bwd_ms": t_fb, "fwd_ms": t_fo, "points_features_per_s_fwd_bwd": M * nf / (t_fb * 1e-3),
           "points_features_per_s_fwd": M * nf / (t_fo * 1e-3),
           "max_rel_err": float(np.max(np.abs(Fg[big] - Fref[big]) / Fref[big])), "sampled_points": len(cs)}
    print(f"[bench] reference points: fwd+bwd {t_fb:.3f} ms, fwd {t_fo:.3f} ms, max rel err {out['max_rel_err']:.2e}",
          file=sys.stderr, flush=True)
    del fb, fo, nb, ws, G, db
    torch.cuda.empty_cache()
    return out


def jacobian_variant(g, gs, torch, batch, probes, db, steps=5, warmup=2):
    """Full per-pair feature Jacobian (no contraction) of the 4096-atom cell,
    FP32 compensated plan: time of one gmp_feature_jacobian call (adjoint
    coefficients + pair kernel) and the rate at which it writes the
    P x n_features x 3 output."""
    plan = g.GMPPlan.from_probes(probes, "fp32c")
    ws = g.Workspace()
    nb = g.build_neighbors(plan, db, ws, reverse=False)
    F, mu = g.features(plan, db, nb, ws)
    out = torch.empty((plan.n_features, 3, nb.n_pairs), dtype=torch.float32, device="cuda")

    def run():
        g.feature_jacobian(plan, db, nb, ws, mu, out=out)
    for _ in range(warmup):
        run()
    t = _median_ms(run, steps, torch)
    with g.profile() as pr:
        run()
        torch.cuda.synchronize()
    kern = {k: v[1] / v[0] for k, v in pr.result.items()}
    nbytes = out.numel() * 4
    res = {"pairs": int(nb.n_pairs), "features_per_atom": plan.n_features, "output_bytes": nbytes,
           "call_ms": t, "pair_kernel_ms": kern.get("jacobian"),
           "output_GB_per_s_pair_kernel": nbytes / (kern["jacobian"] * 1e-3) / 1e9 if "jacobian" in kern else None}
    print(f"[bench] jacobian: {nbytes / 1e9:.2f} GB in {t:.3f} ms per call", file=sys.stderr, flush=True)
    del out, nb, ws, F, mu
    torch.cuda.empty_cache()
    return res


def screening_variant(g, gs, torch, batch, probes, db, steps=10, warmup=3):
    """The same 4096-atom cell with per-primitive screening (each primitive
    only inside its own threshold radius): graph-replayed fwd+bwd and fwd in
    FP32 compensated mode, its deviation from the screened FP64 oracle and
    the screened oracle's own distance from the unscreened one on sampled
    centres."""
    import oracle
    ps = gs.Probes(probes.orders, probes.sigmas, probes.prim_offsets, probes.B, probes.beta, probes.tau,
                   screening=True)
    N, nf = batch.n_atoms, ps.n_features
    plan = g.GMPPlan.from_probes(ps, "fp32c")
    ws = g.Workspace()
    nb = g.build_neighbors(plan, db, ws)
    nbf = g.build_neighbors(plan, db, ws, reverse=False)
    G = torch.as_tensor(np.random.default_rng(7).standard_normal((N, nf)), device="cuda")
    fb = g.CapturedStep(plan, db, ws, nb, backward=True, G=G)
    fo = g.CapturedStep(plan, db, ws, nbf, backward=False)
    for _ in range(warmup):
        fb.replay()
        fo.replay()
    t_fb = _median_ms(fb.replay, steps, torch)
    t_fo = _median_ms(fo.replay, steps, torch)
    g.check_status(ws)
    with g.profile() as pr:
        g.features(plan, db, nbf, ws)
        torch.cuda.synchronize()
    cs = np.sort(np.random.default_rng(29).choice(N, size=24, replace=False))
    Fs = oracle.features(batch.structure(0), ps, centres=cs)
    Fe = oracle.features(batch.structure(0), probes, centres=cs)
    Fg = fb.F.double().cpu().numpy()[cs]
    big = Fs > probes.tau
    out = {"fwd_bwd_ms": t_fb, "fwd_ms": t_fo, "atoms_features_per_s_fwd_bwd": N * nf / (t_fb * 1e-3),
           "overlap_kernel_ms": pr.result["overlap"][1] / pr.result["overlap"][0],
           "max_rel_err_vs_screened_oracle": float(np.max(np.abs(Fg[big] - Fs[big]) / Fs[big])),
           "screened_vs_unscreened_oracle_max_rel": float(np.max(np.abs(Fs[big] - Fe[big]) / Fe[big])),
           "sampled_centres": len(cs)}
    print(f"[bench] screening: fwd+bwd {t_fb:.3f} ms, fwd {t_fo:.3f} ms, overlap {out['overlap_kernel_ms']:.3f} ms",
          file=sys.stderr, flush=True)
    del fb, fo, nb, nbf, ws, G
    torch.cuda.empty_cache()
    return out


def tabulated_variant(g, gs, torch, batch, probes, db, steps=10, warmup=3, intervals=2048):
    """Tabulated radial factors (cubic Hermite tables in r = sqrt(q),
    `intervals` per slot and element) on the 4096-atom cell: graph-replayed
    fwd+bwd and fwd steps in FP32 compensated mode, the overlap kernel beside
    the exact one, the FP64 oracle on sampled centres; and the overlap of both
    on the same cell with 16 primitives per element (where the table's fixed
    cost per pair meets the exponentials' cost per primitive)."""
    import oracle
    pt = gs.Probes(probes.orders, probes.sigmas, probes.prim_offsets, probes.B, probes.beta, probes.tau,
                   radial_intervals=intervals)
    N, nf = batch.n_atoms, pt.n_features
    plan = g.GMPPlan.from_probes(pt, "fp32c")
    ws = g.Workspace()
    nb = g.build_neighbors(plan, db, ws)
    nbf = g.build_neighbors(plan, db, ws, reverse=False)
    G = torch.as_tensor(np.random.default_rng(7).standard_normal((N, nf)), device="cuda")
    fb = g.CapturedStep(plan, db, ws, nb, backward=True, G=G)
    fo = g.CapturedStep(plan, db, ws, nbf, backward=False)
    for _ in range(warmup):
        fb.replay()
        fo.replay()
    t_fb = _median_ms(fb.replay, steps, torch)
    t_fo = _median_ms(fo.replay, steps, torch)
    fb.check_status()
    cs = np.sort(np.random.default_rng(37).choice(N, size=24, replace=False))
    Fref = oracle.features(batch.structure(0), probes, centres=cs)
    Fg = fb.F.double().cpu().numpy()[cs]
    big = Fref > probes.tau

    def overlap_ms(p, prec):
        pl = g.GMPPlan.from_probes(p, prec)
        w = g.Workspace()
        n2 = g.build_neighbors(pl, db, w, reverse=False)
        g.features(pl, db, n2, w)
        torch.cuda.synchronize()
        with g.profile() as pr:
            for _ in range(5):
                g.features(pl, db, n2, w)
            torch.cuda.synchronize()
        return pr.result["overlap"][1] / pr.result["overlap"][0]
    rng = np.random.default_rng(5)
    o16, B16, b16 = gs.density_tables(rng, probes.n_elements, 16, (0.01, 10.0), (0.1, 30.0))
    kern = {}
    for label, (po, B, be) in (("5_primitives", (probes.prim_offsets, probes.B, probes.beta)),
                               ("16_primitives", (o16, B16, b16))):
        for nint in (0, intervals):
            pp = gs.Probes(probes.orders, probes.sigmas, po, B, be, probes.tau, radial_intervals=nint)
            kern[f"{label}_{'tabulated' if nint else 'exact'}_ms"] = {
                prec: round(overlap_ms(pp, prec), 4) for prec in ("fp32c", "fp32w")}
    out = {"intervals_per_slot_and_element": intervals, "fwd_bwd_ms": t_fb, "fwd_ms": t_fo,
           "atoms_features_per_s_fwd_bwd": N * nf / (t_fb * 1e-3),
           "max_rel_err_vs_exact_oracle": float(np.max(np.abs(Fg[big] - Fref[big]) / Fref[big])),
           "sampled_centres": len(cs), "overlap_kernel": kern}
    print(f"[bench] tabulated radial: fwd+bwd {t_fb:.3f} ms, overlap {kern}", file=sys.stderr, flush=True)
    del fb, fo, nb, nbf, ws, G
    torch.cuda.empty_cache()
    return out


def batched_vs_per_structure(g, gs, torch):
    """2048 structures of 8-256 atoms (half periodic triclinic, half
    clusters), FP32 compensated forward (neighbour build + overlap + norm):
    one batched launch sequence replayed from a HIP graph, against the same
    work issued structure by structure through the C ABI with pre-sized
    capacity and no graph.  Outputs of the two must be bitwise equal."""
    import ctypes
    from paper_2303_12980_amd import _lib, autotune
    t0 = time.time()
    batch, probes = gs.config("C3")
    print(f"[bench] batched workload: {batch.n_structs} structures, {batch.n_atoms} atoms "
          f"({time.time() - t0:.1f}s to generate)", file=sys.stderr, flush=True)
    db = g.DeviceBatch.from_batch(batch)
    plan = g.GMPPlan.from_probes(probes, "fp32c")
    ws = g.Workspace()
    tune = autotune.autotune(plan, db, ws, backward=False, reps=2, candidates=[
        dict(chunk_pairs=c, bin_divisor=b, blocks_per_cu=0) for c in (1024, 2048, 4096) for b in (2, 3)],
        cache_path=TUNE_CACHE)
    print(f"[bench] autotuned {tune['tuning']} ({'cached' if tune['cached'] else 'searched'})",
          file=sys.stderr, flush=True)
    nb = g.build_neighbors(plan, db, ws, reverse=False)
    step = g.CapturedStep(plan, db, ws, nb, backward=False)
    for _ in range(3):
        step.replay()
    graph_ms = _median_ms(step.replay, 20, torch)
    g.check_status(ws)

    def eager():
        g.rebuild_neighbors_nosync(plan, db, ws, nb)
        g.features(plan, db, nb, ws, True, out=step.F, comp_out=step.mu)
    eager_ms = _median_ms(eager, 5, torch)
    Fb, mub = step.F.clone(), step.mu.clone()

    # per-structure launches: pre-built descriptors, one shared workspace
    L = _lib.load()
    offs_h = batch.atom_offsets
    poffs = nb.offsets.cpu().numpy()
    Fp = torch.empty_like(Fb)
    mup = torch.empty_like(mub)
    calls = []
    need = 0
    for s in range(batch.n_structs):
        a0, a1 = int(offs_h[s]), int(offs_h[s + 1])
        v = db.structure(s, a0, a1)
        nbs = g.Neighbors(plan, v, int(poffs[a1] - poffs[a0]), reverse=False)
        nbs.n_pairs = nbs.capacity
        nbs.max_list = int(np.diff(poffs[a0:a1 + 1]).max())
        need = max(need, plan.workspace_bytes(1, a1 - a0, nbs.capacity))
        calls.append((v, nbs, v.desc(), nbs.desc(), Fp[a0:a1], mup[a0:a1]))
    wbuf = ws.get(need)
    wptr, wn = wbuf.data_ptr(), wbuf.numel()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def per_structure():
        for v, nbs, bd, nd, F, mu in calls:
            st = L.gmp_build_neighbors(plan.handle, ctypes.byref(bd), ctypes.byref(nd), None, ctypes.c_void_p(wptr),
                                       ctypes.c_size_t(wn), stream)
            st = st or L.gmp_features(plan.handle, ctypes.byref(bd), ctypes.byref(nd), ctypes.c_void_p(F.data_ptr()),
                                      ctypes.c_void_p(mu.data_ptr()), ctypes.c_void_p(wptr), ctypes.c_size_t(wn),
                                      stream)
            if st:
                _lib.check(st)
    per_structure()
    per_ms = _median_ms(per_structure, 3, torch)
    g.check_status(ws)
    # HIP events around single replays (after two warm-up replays): median of 10
    for _ in range(2):
        step.replay()
    ev_ms = []
    for _ in range(10):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        step.replay()
        ev[1].record()
        torch.cuda.synchronize()
        ev_ms.append(ev[0].elapsed_time(ev[1]))
    graph_event_ms = float(np.median(ev_ms))
    bitwise = bool(torch.equal(Fp, Fb)) and bool(torch.equal(mup, mub))
    N, nf = batch.n_atoms, probes.n_features
    return {
        "workload": f"{batch.n_structs} structures, {N} atoms (8-256 each, half periodic triclinic at "
                    f"0.08/A^3, half clusters), 10 elements, 3-6 primitives, l=0..4 x 8 sigma, fp32c forward",
        "atoms": N, "pairs": int(nb.n_pairs), "tuning": tune["tuning"],
        "graph_replay_ms": graph_ms, "graph_replay_event_ms": graph_event_ms, "batched_eager_ms": eager_ms,
        "per_structure_ms": per_ms,
        "speedup_graph_vs_per_structure": per_ms / graph_ms,
        "atoms_features_per_s_graph": N * nf / (graph_ms * 1e-3),
        "bitwise_equal_to_per_structure": bitwise,
    }


# monomial terms of the solid harmonics of each order with r^2 expanded
# (1, 3, 12, 28, 63 for l = 0..4): the per-pair polynomial work of the cost model
POLY_TERMS = {0: 1, 1: 3, 2: 12, 3: 28, 4: 63}


def algorithmic_counts(nb, probes, rc2):
    """Per-launch algorithmic work of the overlap kernel, from the lists, as
    the cost model counts it: per pair, q (5 flops) and the polynomials
    (2 flops per monomial term of every requested order, r^2 expanded); per
    (pair, active sigma) and primitive, one multiply for the exponent and a
    multiply-add per order for the radial factors (the exponential itself is
    counted separately against the transcendental rate); per (pair, active
    sigma), a multiply-add per requested component for the accumulation.
    `executed_alg` is the smaller count of the operations the recursion
    actually needs (q, one multiply per monomial of degree >= 2)."""
    E, S = probes.n_elements, len(probes.sigmas)
    offs = nb.offsets.cpu().numpy()
    bs = nb.bucket_start.cpu().numpy().reshape(-1, S * E + 1).astype(np.int64)
    sizes = np.diff(bs, axis=1).reshape(-1, S, E)          # [N, shell, species]
    rank = np.array([int(np.sum(rc2 < rc2[s])) for s in range(S)])
    active = np.cumsum(sizes, axis=1)[:, rank, :]          # [N, sigma, species] pairs each sigma uses
    K = np.diff(probes.prim_offsets).astype(np.int64)      # primitives per element
    L = [int(l) for l in probes.orders]
    lmax = max(L)
    ncomp = int(sum((l + 1) * (l + 2) // 2 for l in L))
    terms = int(sum(POLY_TERMS[l] for l in L))
    nmono_hi = (lmax + 1) * (lmax + 2) * (lmax + 3) // 6 - 4 if lmax >= 2 else 0
    pairs = int(offs[-1])
    pair_sigma = int(active.sum())
    exps = int((active.sum(axis=(0, 1)) * K).sum())
    flops = pairs * (5 + 2 * terms) + exps * (1 + 2 * len(L)) + pair_sigma * 2 * ncomp
    executed_alg = pairs * (5 + nmono_hi) + exps * (2 + 2 * len(L)) + pair_sigma * 2 * ncomp
    return dict(pairs=pairs, pair_sigma=pair_sigma, exps=exps, flops=flops, executed_alg=executed_alg,
                per_pair=5 + 2 * terms, per_exp=1 + 2 * len(L), per_pair_sigma=2 * ncomp)


def list_bytes(nb, n_centres, n_slots, n_elements):
    """Algorithmic bytes the neighbour build writes: per pair the neighbour
    index, the packed shift and the reverse index (12 B); per centre the list
    offset (8 B), the bucket starts (4 (S E + 1) B) and the prefix ends (4 S B)."""
    return int(nb.n_pairs) * 12 + n_centres * (8 + 4 * (n_slots * n_elements + 1) + 4 * n_slots)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(oracle, batch, probes, n_features):
    """The oracle's forward (brute-force neighbours + closed-form overlaps,
    OpenMP over centres), median of 3 runs: on every available core over all
    centres of the workload, and on one core over a 256-centre sample."""
    avail = len(os.sched_getaffinity(0))
    threads = min(int(os.environ.get("OMP_NUM_THREADS", "0")) or avail, avail)
    N = batch.n_atoms
    struct = batch.structure(0)
    prev = oracle.set_threads(threads)

    def med(fn):
        ts = []
        for _ in range(3):
            t = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts))
    t_all = med(lambda: oracle.features(struct, probes))
    oracle.set_threads(1)
    sample = np.sort(np.random.default_rng(31).choice(N, size=min(256, N), replace=False))
    t_one = med(lambda: oracle.features(struct, probes, centres=sample))
    oracle.set_threads(prev)
    return {"value": N * n_features / t_all, "unit": "atoms*features/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle forward (brute-force neighbours + closed-form overlaps) over all {N} centres "
                      f"of the workload on {threads} OpenMP threads, median of 3 runs ({t_all:.2f} s); forward "
                      f"only",
            "single_core": {"value": len(sample) * n_features / t_one, "unit": "atoms*features/s", "cores": 1,
                            "sample": f"{len(sample)} sampled centres of the same workload, median of 3 runs "
                                      f"({t_one:.2f} s)"},
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "affinity_cpus": avail}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: sharding (structures of a batch across "
                                   "GPUs with no exchange; a large system by centres with one reduction of the "
                                   "position gradients) is not executed", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import gmp_synth as gs
    import paper_2303_12980_amd as g

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        a = torch.ones(256 << 18, dtype=torch.float32, device=dev)
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        del a, c
    t0 = time.time()
    batch, probes = gs.config(args.workload)
    N, nf = batch.n_atoms, probes.n_features
    print(f"[bench] workload {args.workload}: {N} atoms, {nf} features, generated in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    db = g.DeviceBatch.from_batch(batch, dev)
    G = torch.as_tensor(np.random.default_rng(7).standard_normal((N, nf)), device=dev)

    from paper_2303_12980_amd import autotune
    tunings = {}

    def make(prec):
        plan = g.GMPPlan.from_probes(probes, prec)
        w = g.Workspace(dev)
        tune = autotune.autotune(plan, db, w, candidates=autotune.STEP_CANDIDATES, backward=True, reps=3,
                                 cache_path=TUNE_CACHE)
        tunings[prec] = dict(tune["tuning"], step_ms=tune["ms"],
                             concurrent_reverse=bool(tune.get("concurrent_reverse", False)))
        for k in ("graph_ms_one_stream", "graph_ms_two_streams"):
            if k in tune:
                tunings[prec][k] = tune[k]
        how = "cached" if tune["cached"] else ("search off: defaults" if tune["ms"] is None else "searched")
        tunings[prec]["how"] = how
        print(f"[bench] {prec} autotuned {tune['tuning']}, reverse search on a second stream: "
              f"{tunings[prec]['concurrent_reverse']} ({how})", file=sys.stderr, flush=True)
        nb = g.build_neighbors(plan, db, w)
        return plan, w, nb

    rev_stream = torch.cuda.Stream()
    ev_built, ev_rev = torch.cuda.Event(), torch.cuda.Event()

    def eager_step(plan, w, nb, backward=True, split=False):
        # a forward-only step builds its lists without the reverse index; with
        # split the reverse-pair search runs on a second stream beside the forward
        nb2 = g.build_neighbors(plan, db, w, reverse=backward, out=nb, defer_reverse=split)
        if split:
            ev_built.record()
            rev_stream.wait_event(ev_built)
            with torch.cuda.stream(rev_stream):
                g.build_reverse(plan, db, w, nb2)
            ev_rev.record(rev_stream)
        F, mu = g.features(plan, db, nb2, w)
        if backward:
            if split:
                torch.cuda.current_stream().wait_event(ev_rev)
            g.features_backward(plan, db, nb2, w, mu, F, G)
        return F

    def wall_ms(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps * 1e3

    results, graphs = {}, {}
    for prec in (["fp32c", "fp32w"] + ([] if args.no_fp64 else ["fp64"])):
        plan, w, nb = make(prec)
        nbf = g.build_neighbors(plan, db, w, reverse=False)
        r = {}
        r["eager_fwd_bwd_ms"] = wall_ms(lambda: eager_step(plan, w, nb, True), args.steps, args.warmup)
        r["eager_fwd_ms"] = wall_ms(lambda: eager_step(plan, w, nbf, False), args.steps, args.warmup)
        if not args.no_split:
            r["eager_split_fwd_bwd_ms"] = wall_ms(lambda: eager_step(plan, w, nb, True, True), args.steps, args.warmup)
        fb = g.CapturedStep(plan, db, w, nb, backward=True, G=G,
                            concurrent_reverse=tunings[prec]["concurrent_reverse"])
        r["graph_fwd_bwd_ms"] = wall_ms(fb.replay, args.steps, args.warmup)
        fo = g.CapturedStep(plan, db, w, nbf, backward=False)
        r["graph_fwd_ms"] = wall_ms(fo.replay, args.steps, args.warmup)
        g.check_status(w)
        results[prec] = r
        graphs[prec] = (plan, w, nb, fb, nbf)
        print(f"[bench] {prec}: graph fwd+bwd {r['graph_fwd_bwd_ms']:.3f} ms, fwd {r['graph_fwd_ms']:.3f} ms; "
              f"eager fwd+bwd {r['eager_fwd_bwd_ms']:.3f} ms (reverse on a second stream: "
              f"{r.get('eager_split_fwd_bwd_ms', float('nan')):.3f} ms)", file=sys.stderr, flush=True)

    def kernel_profile(prec, backward, steps=5):
        plan, w, nb, _, nbf = graphs[prec]
        nb = nb if backward else nbf
        eager_step(plan, w, nb, backward)
        torch.cuda.synchronize()
        with g.profile() as pr:
            for _ in range(steps):
                eager_step(plan, w, nb, backward)
            torch.cuda.synchronize()
        return {k: dict(launches=v[0], avg_ms=v[1] / v[0], ms_per_step=v[1] / steps) for k, v in pr.result.items()}

    plan32, _, nb32, step32, _ = graphs["fp32c"]
    dt_fb = results["fp32c"]["graph_fwd_bwd_ms"] * 1e-3
    dt_f = results["fp32c"]["graph_fwd_ms"] * 1e-3
    # per-kernel averages (library HIP events around each launch, eager steps)
    kern = kernel_profile("fp32c", True)
    kern_f = kernel_profile("fp32c", False)
    dom = max(kern, key=lambda k: kern[k]["ms_per_step"])
    counts = algorithmic_counts(nb32, probes, plan32.rc2)
    ov = kern["overlap"]
    achieved = counts["flops"] / (ov["avg_ms"] * 1e-3) / 1e12
    rec = counter_record("overlap")
    h3_ms = sum(kern[k]["avg_ms"] for k in ("nbr_count", "nbr_fill_sort", "nbr_reverse") if k in kern)
    h3_bytes = list_bytes(nb32, N, plan32.n_slots, probes.n_elements)
    roofline = {"kernel": "overlap", "bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "flop_count": {"per_pair": counts["per_pair"], "per_primitive_exp": counts["per_exp"],
                               "per_pair_sigma": counts["per_pair_sigma"], "pairs": counts["pairs"],
                               "primitive_exps": counts["exps"], "pair_sigmas": counts["pair_sigma"]},
                "executed_alg": {"flops_per_launch": counts["executed_alg"],
                                 "tflops": round(counts["executed_alg"] / (ov["avg_ms"] * 1e-3) / 1e12, 3)},
                "peak_nonpacked_fp32": round(PEAK_FP32_NONPACKED_TFLOPS, 1),
                "frac_nonpacked": round(achieved / PEAK_FP32_NONPACKED_TFLOPS, 4),
                "traffic": rec["hbm_bytes_per_launch"] if rec else None,
                # counts and durations of the same profiled runs (the profiler adds a few % per launch)
                "executed": ({"fp32_tflops": 64 * rec["valu_flops_fp32_per_wave"] / (rec["avg_us_trace"] * 1e-6) / 1e12,
                              "valu_issue_frac": rec["valu_insts"] / (rec["avg_us_trace"] * 1e-6) / VALU_WAVE_INSTS_PER_S,
                              "avg_us_profiled": rec["avg_us_trace"],
                              "source": "profiles/counters_C2.json"} if rec and rec.get("avg_us_trace") else None),
                "exp_rate_per_s": counts["exps"] / (ov["avg_ms"] * 1e-3),
                "exp_frac": counts["exps"] / (ov["avg_ms"] * 1e-3) / PEAK_EXP_PER_S,
                "algorithmic_flops_per_launch": counts["flops"], "avg_launch_ms": ov["avg_ms"],
                "dominant_kernel_of_step": dom,
                "h3": {"kernels": "nbr_count + nbr_fill_sort + nbr_reverse", "ms": round(h3_ms, 5),
                       "algorithmic_bytes": h3_bytes, "GBps": round(h3_bytes / (h3_ms * 1e-3) / 1e9, 1),
                       "frac_hbm": round(h3_bytes / (h3_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}}

    # accuracy on sampled centres vs the FP64 oracle (outputs of the last graph replays)
    import oracle
    rng = np.random.default_rng(11)
    cs = np.sort(rng.choice(N, size=min(args.sample_centres, N), replace=False))
    Fref = oracle.features(batch.structure(0), probes, centres=cs)
    big = Fref > probes.tau
    Fabs = oracle.features_abs(batch.structure(0), probes, centres=cs)
    kappa = Fabs[big] / Fref[big]
    acc = {"sampled_centres": int(len(cs)), "rule": "max |F-F_ref|/F_ref over F_ref > tau",
           "kappa": {"definition": "F_abs / F_ref, F_abs the feature of the absolute pair terms",
                     "max": float(kappa.max()), "median": float(np.median(kappa))}}
    for prec, (_, _, _, st, _) in graphs.items():
        Fg = st.F.double().cpu().numpy()[cs]
        acc[f"{prec}_max_rel_err"] = float(np.max(np.abs(Fg[big] - Fref[big]) / Fref[big]))
        acc[f"{prec}_max_err_over_2^-24_Fabs"] = float(np.max(np.abs(Fg - Fref) / (2.0 ** -24 * Fabs)))

    # CPU baseline: the oracle, forward (all cores over every centre; one core on a sample)
    cpu = None if args.no_cpu_baseline else cpu_baseline(oracle, batch, probes, nf)

    atoms_feat = N * nf
    value = atoms_feat / dt_fb
    out = {
        "metric": "atoms*features/s (fwd+bwd, FP32 compensated, incl. neighbour build; one graph replay per step)",
        "value": value, "unit": "atoms*features/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt_fb * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"{args.workload}: periodic 40x40x40 A cell, {N} atoms, 5 elements, "
                                f"5 primitives/element, l=0..4 x 8 sigma (0.1-1.6 A), tau 1e-11"
                                if args.workload.upper() == "C2" else
                                f"{args.workload}: {gs.CONFIG_TEXT[args.workload.upper()]}"),
                   "atoms": N, "features_per_atom": nf, "pairs": counts["pairs"], "precision": "fp32c"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "rates": {
            **{f"{prec}_{mode}": atoms_feat / (r[f"{kind}_{mode}_ms"] * 1e-3)
               for prec, r in results.items() for kind in ("graph", "eager") for mode in ("fwd_bwd", "fwd")
               if kind == "graph"},
            **{f"{prec}_{mode}_eager": atoms_feat / (r[f"eager_{mode}_ms"] * 1e-3)
               for prec, r in results.items() for mode in ("fwd_bwd", "fwd")},
            "fp32c_fwd_kernels_only": atoms_feat / (1e-3 * (kern_f["overlap"]["avg_ms"] + kern_f["norm"]["avg_ms"])),
        },
        "timings_ms": results,
        "tuning": tunings,
        "accuracy": acc,
        "kernels_fp32c_ms_per_step": {k: round(v["ms_per_step"], 5) for k, v in kern.items()},
    }
    if not args.no_fp64:
        out["kernels_fp64_ms_per_step"] = {k: round(v["ms_per_step"], 5) for k, v in kernel_profile("fp64", True).items()}
    out["kernels_fp32w_ms_per_step"] = {k: round(v["ms_per_step"], 5) for k, v in kernel_profile("fp32w", True).items()}
    if not args.no_density:
        out["density_variant"] = density_variant(g, gs, torch, batch, probes, db)
        out["occupancy_variant"] = occupancy_variant(g, gs, torch, batch, probes)
        out["points_variant"] = points_variant(g, gs, torch, batch, probes)
        out["jacobian"] = jacobian_variant(g, gs, torch, batch, probes, db)
        out["screening_variant"] = screening_variant(g, gs, torch, batch, probes, db)
        out["tabulated_variant"] = tabulated_variant(g, gs, torch, batch, probes, db)
    if not args.no_batched:
        del graphs, plan32, nb32, step32
        torch.cuda.empty_cache()
        out["batched"] = batched_vs_per_structure(g, gs, torch)
    if not args.no_others:
        out["other_workloads"] = other_workloads(g, gs, torch)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
