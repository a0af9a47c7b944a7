"""FP64 CPU oracle for GMP features (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It wraps ``gmp_oracle.c`` (plain C,
built with gcc, no FMA contraction, no fast-math) through ctypes and shares
nothing with the HIP library.

Every function here follows the definitions written at the top of
``gmp_oracle.c``: the closed-form Gaussian-product overlap of a solid
Maxwell-Cartesian harmonic probe with Gaussian density primitives, the
per-width cutoff inferred from the overlap threshold, the brute-force
neighbour set over periodic images, and the weighted root-sum-square
feature (GMP-Featurizer, arXiv 2303.12980, section "Examples").
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gmp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

CFLAGS = ["-O3", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (x86-64 baseline ISA, portable across hosts)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            L = ctypes.CDLL(_LIB)
            dp = ctypes.POINTER(ctypes.c_double)
            ip = ctypes.POINTER(ctypes.c_int32)
            lp = ctypes.POINTER(ctypes.c_int64)
            c_int, c_dbl, c_i64 = ctypes.c_int, ctypes.c_double, ctypes.c_int64
            L.oracle_cutoffs.argtypes = [c_int, dp, c_int, ip, dp, dp, c_dbl, dp]
            L.oracle_cutoffs.restype = c_int
            L.oracle_density_cutoff.argtypes = [c_int, ip, dp, dp, c_dbl, dp]
            L.oracle_density_cutoff.restype = c_int
            L.oracle_wrap.argtypes = [c_int, dp, dp, c_int, dp, ip]
            L.oracle_wrap.restype = c_int
            L.oracle_neighbors.argtypes = [c_int, dp, ip, dp, c_int, c_int, dp, c_int, c_i64,
                                           ip, ip, dp, ip, ip]
            L.oracle_neighbors.restype = c_i64
            probe_args = [c_int, ip, c_int, dp, c_int, ip, dp, dp, c_dbl, c_int]
            L.oracle_slot_cutoffs.argtypes = [*probe_args, dp]
            L.oracle_slot_cutoffs.restype = c_int
            L.oracle_features.argtypes = [c_int, dp, ip, dp, c_int, *probe_args, c_int, ip, dp, dp, dp]
            L.oracle_features.restype = c_int
            L.oracle_grad.argtypes = [c_int, dp, ip, dp, c_int, *probe_args, dp, dp, dp, dp, dp]
            L.oracle_grad.restype = c_int
            L.oracle_set_threads.argtypes = [c_int]
            L.oracle_set_threads.restype = c_int
            L.oracle_features_abs.argtypes = [c_int, dp, ip, dp, c_int, *probe_args, c_int, ip, dp, dp]
            L.oracle_features_abs.restype = c_int
            L.oracle_grad_centres.argtypes = [c_int, dp, ip, dp, c_int, *probe_args, c_int, ip, dp, dp, dp, dp]
            L.oracle_grad_centres.restype = c_int
            L.oracle_neighbors_many.argtypes = [c_int, dp, ip, dp, c_int, c_int, dp, c_int, ip, lp, c_i64,
                                                ip, ip, dp, ip, ip]
            L.oracle_neighbors_many.restype = c_i64
            L.oracle_loss_frozen.argtypes = [c_int, dp, ip, dp, *probe_args, lp, ip, ip, dp, dp, dp, dp]
            L.oracle_loss_frozen.restype = c_int
            L.oracle_point_neighbors.argtypes = [c_int, dp, ip, dp, c_int, c_int, dp, dp, c_i64,
                                                 ip, ip, dp, ip, ip]
            L.oracle_point_neighbors.restype = c_i64
            L.oracle_point_features.argtypes = [c_int, dp, ip, dp, c_int, *probe_args, c_int, dp, dp, dp, dp]
            L.oracle_point_features.restype = c_int
            L.oracle_point_grad.argtypes = [c_int, dp, ip, dp, c_int, *probe_args, c_int, dp, dp, dp, dp, dp,
                                            dp, dp]
            L.oracle_point_grad.restype = c_int
            L.oracle_point_loss_frozen.argtypes = [c_int, dp, ip, dp, *probe_args, c_int, dp, lp, ip, ip, dp,
                                                   dp, dp, dp]
            L.oracle_point_loss_frozen.restype = c_int
            L.oracle_jacobian.argtypes = [c_int, dp, ip, dp, c_int, *probe_args, c_i64, dp, dp, ip]
            L.oracle_jacobian.restype = c_i64
            L.oracle_solid_harmonic.argtypes = [c_int, c_int, c_int, c_int, dp, dp, dp]
            L.oracle_solid_harmonic.restype = None
            L.oracle_radial.argtypes = [c_int, c_dbl, c_int, dp, dp, c_int, dp, dp]
            L.oracle_radial.restype = None
            _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _l(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _check(st):
    if st != 0:
        raise OracleError(f"oracle status {st}")


def _probe_args(probes):
    keep = []
    o, op = _i(probes.orders); keep.append(o)
    s, sp = _d(probes.sigmas); keep.append(s)
    po, pop = _i(probes.prim_offsets); keep.append(po)
    B, Bp = _d(probes.B); keep.append(B)
    be, bep = _d(probes.beta); keep.append(be)
    args = [len(o), op, len(s), sp, len(po) - 1, pop, Bp, bep, float(probes.tau),
            int(bool(getattr(probes, "screening", False)))]
    return keep, args


def n_components(orders: Sequence[int], n_sigmas: int) -> int:
    """Components of one centre: n_sigmas * ncomp(l) per order, 1 for order -1."""
    return int(sum(1 if l == -1 else n_sigmas * (l + 1) * (l + 2) // 2 for l in orders))


def n_features(orders: Sequence[int], n_sigmas: int) -> int:
    """Features of one centre: n_sigmas per order, 1 for order -1."""
    return int(sum(1 if l == -1 else n_sigmas for l in orders))


def n_slots(probes) -> int:
    """Cutoff slots: the sigmas, plus the density when order -1 is requested."""
    return len(probes.sigmas) + (1 if -1 in [int(l) for l in probes.orders] else 0)


def sigma_cutoffs(probes) -> np.ndarray:
    """rc(sigma)^2 for every sigma."""
    keep, a = _probe_args(probes)
    rc2 = np.zeros(len(probes.sigmas))
    _check(lib().oracle_cutoffs(a[2], a[3], a[4], a[5], a[6], a[7], a[8],
                                rc2.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return rc2


def density_cutoff(probes) -> float:
    """rc_{-1}^2 of the local density (order -1)."""
    keep, a = _probe_args(probes)
    out = ctypes.c_double(0.0)
    _check(lib().oracle_density_cutoff(a[4], a[5], a[6], a[7], a[8], ctypes.byref(out)))
    return out.value


def cutoffs(probes) -> np.ndarray:
    """rc^2 of every cutoff slot: the sigmas in order, then the density when
    order -1 is requested."""
    keep, a = _probe_args(probes)
    rc2 = np.zeros(n_slots(probes))
    _check(lib().oracle_slot_cutoffs(*a, rc2.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return rc2


def wrap(pos, cell, pbc):
    pos, pp = _d(pos)
    cell, cp = _d(np.asarray(cell).reshape(9))
    n = len(pos)
    rw = np.zeros((n, 3))
    m = np.zeros((n, 3), dtype=np.int32)
    _check(lib().oracle_wrap(n, pp, cp, int(pbc), rw.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             m.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return rw, m


def neighbors(struct, rc2, centre: int):
    """Canonical neighbour list of one centre: dict with j, n [k,3], q, shell."""
    pos, spec, cell, pbc = struct
    pos, pp = _d(pos)
    spec, sp = _i(spec)
    cell, cp = _d(np.asarray(cell).reshape(9))
    rc2, rp = _d(rc2)
    st = ctypes.c_int32(0)
    cap = 1024
    while True:
        j = np.zeros(cap, np.int32); n = np.zeros((cap, 3), np.int32)
        q = np.zeros(cap); sh = np.zeros(cap, np.int32)
        cnt = lib().oracle_neighbors(len(pos), pp, sp, cp, int(pbc), len(rc2), rp, int(centre), cap,
                                     j.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                     n.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                     q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     sh.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                     ctypes.byref(st))
        _check(st.value)
        if cnt <= cap:
            return dict(j=j[:cnt], n=n[:cnt], q=q[:cnt], shell=sh[:cnt],
                        e=np.asarray(spec)[j[:cnt]])
        cap = int(cnt)


def set_threads(n: int) -> int:
    """OpenMP threads of the oracle's loops over centres; returns the previous count."""
    return int(lib().oracle_set_threads(int(n)))


def neighbors_many(struct, rc2, centres):
    """Canonical lists of many centres (the same lists as neighbors(), in
    parallel over centres): dict with offs [k+1], j, n [P,3], q, shell, e."""
    pos, spec, cell, pbc = struct
    pos, pp = _d(pos)
    spec, sp = _i(spec)
    cell, cp = _d(np.asarray(cell).reshape(9))
    rc2, rp = _d(rc2)
    cl, clp = _i(np.asarray(centres))
    offs = np.zeros(len(cl) + 1, np.int64)
    st = ctypes.c_int32(0)
    L = lib()
    ip = ctypes.POINTER(ctypes.c_int32)
    total = L.oracle_neighbors_many(len(pos), pp, sp, cp, int(pbc), len(rc2), rp, len(cl), clp,
                                    offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 0, None, None, None,
                                    None, ctypes.byref(st))
    _check(st.value)
    j = np.zeros(max(total, 1), np.int32); n = np.zeros((max(total, 1), 3), np.int32)
    q = np.zeros(max(total, 1)); sh = np.zeros(max(total, 1), np.int32)
    t2 = L.oracle_neighbors_many(len(pos), pp, sp, cp, int(pbc), len(rc2), rp, len(cl), clp,
                                 offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), total,
                                 j.ctypes.data_as(ip), n.ctypes.data_as(ip), _dp(q), sh.ctypes.data_as(ip),
                                 ctypes.byref(st))
    _check(st.value)
    assert t2 == total
    j, n, q, sh = j[:total], n[:total], q[:total], sh[:total]
    return dict(offs=offs, j=j, n=n, q=q, shell=sh, e=np.asarray(spec)[j])


def _occ(occupancy, n):
    """(keep-alive array, pointer) of the per-atom occupancies, or (None, None)."""
    if occupancy is None:
        return None, None
    o = np.ascontiguousarray(occupancy, dtype=np.float64)
    assert o.shape == (n,)
    return o, o.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def features(struct, probes, centres: Optional[Sequence[int]] = None, with_mu: bool = False,
             occupancy=None):
    """F [n_centres, nf] (order-major, sigma-minor; one feature for order -1)
    and optionally mu [n_centres, nc] laid out (order, sigma, component).
    occupancy: per-atom fractional occupancies (None: all 1)."""
    pos, spec, cell, pbc = struct
    pos, pp = _d(pos)
    spec, sp = _i(spec)
    cell, cp = _d(np.asarray(cell).reshape(9))
    keep, a = _probe_args(probes)
    if centres is None:
        nc, cptr, carr = -1, None, None
        ncent = len(pos)
    else:
        carr, cptr = _i(np.asarray(centres))
        nc = ncent = len(carr)
    nf = n_features(probes.orders, len(probes.sigmas))
    F = np.zeros((ncent, nf))
    ncomp = n_components(probes.orders, len(probes.sigmas))
    mu = np.zeros((ncent, ncomp)) if with_mu else None
    occ, op = _occ(occupancy, len(pos))
    _check(lib().oracle_features(len(pos), pp, sp, cp, int(pbc), *a, nc, cptr,
                                 F.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 mu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if with_mu else None, op))
    return (F, mu) if with_mu else F


def features_abs(struct, probes, centres: Optional[Sequence[int]] = None, occupancy=None):
    """F_abs [n_centres, nf]: the features of the absolute values of the pair
    terms (the conditioning reference kappa = F_abs / F of a feature)."""
    pos, spec, cell, pbc = struct
    pos, pp = _d(pos)
    spec, sp = _i(spec)
    cell, cp = _d(np.asarray(cell).reshape(9))
    keep, a = _probe_args(probes)
    if centres is None:
        nc, cptr, carr, ncent = -1, None, None, len(pos)
    else:
        carr, cptr = _i(np.asarray(centres))
        nc = ncent = len(carr)
    F = np.zeros((ncent, n_features(probes.orders, len(probes.sigmas))))
    occ, op = _occ(occupancy, len(pos))
    _check(lib().oracle_features_abs(len(pos), pp, sp, cp, int(pbc), *a, nc, cptr,
                                     F.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), op))
    return F


def features_batch(batch, probes, with_mu=False):
    Fs, mus = [], []
    occ = getattr(batch, "occupancy", None)
    for s in range(batch.n_structs):
        a0, a1 = int(batch.atom_offsets[s]), int(batch.atom_offsets[s + 1])
        r = features(batch.structure(s), probes, with_mu=with_mu,
                     occupancy=None if occ is None else occ[a0:a1])
        if with_mu:
            Fs.append(r[0]); mus.append(r[1])
        else:
            Fs.append(r)
    F = np.concatenate(Fs, axis=0)
    return (F, np.concatenate(mus, axis=0)) if with_mu else F


def grad(struct, probes, G, occupancy=None):
    """Analytic dL/dR [n,3] and dL/dcell [3,3] of L = sum G*F, plus F."""
    pos, spec, cell, pbc = struct
    pos, pp = _d(pos)
    spec, sp = _i(spec)
    cell, cp = _d(np.asarray(cell).reshape(9))
    keep, a = _probe_args(probes)
    G, gp = _d(G)
    n = len(pos)
    gpos = np.zeros((n, 3)); gcell = np.zeros((3, 3))
    F = np.zeros((n, n_features(probes.orders, len(probes.sigmas))))
    occ, op = _occ(occupancy, n)
    _check(lib().oracle_grad(n, pp, sp, cp, int(pbc), *a, gp,
                             gpos.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             gcell.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             F.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), op))
    return gpos, gcell, F


def grad_centres(struct, probes, centres, G, occupancy=None):
    """Analytic dL/dR [n,3] and dL/dcell [3,3] of L = sum_t G[t] . F[centres[t]]:
    the gradient of oracle grad() with the upstream gradient zero on every
    centre not listed (centres distinct; G [len(centres), nf])."""
    pos, spec, cell, pbc = struct
    pos, pp = _d(pos)
    spec, sp = _i(spec)
    cell, cp = _d(np.asarray(cell).reshape(9))
    keep, a = _probe_args(probes)
    cl, clp = _i(np.asarray(centres))
    G, gp = _d(np.asarray(G).reshape(len(cl), -1))
    n = len(pos)
    gpos = np.zeros((n, 3)); gcell = np.zeros((3, 3))
    occ, op = _occ(occupancy, n)
    _check(lib().oracle_grad_centres(n, pp, sp, cp, int(pbc), *a, len(cl), clp, gp,
                                     gpos.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     gcell.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), op))
    return gpos, gcell


def frozen_pairs(struct, probes):
    """Pair list of the current configuration in raw-position form (j, n~, q),
    for finite differences with the pair set held fixed."""
    pos, spec, cell, pbc = struct
    rc2 = cutoffs(probes)
    _, m = wrap(pos, cell, pbc)
    po = [0]; pj = []; pn = []; pq = []
    for i in range(len(pos)):
        nb = neighbors(struct, rc2, i)
        pj.append(nb["j"])
        pn.append(nb["n"] - m[nb["j"]] + m[i])
        pq.append(nb["q"])
        po.append(po[-1] + len(nb["j"]))
    return (np.asarray(po, np.int64), np.concatenate(pj).astype(np.int32),
            np.concatenate(pn).astype(np.int32), np.concatenate(pq))


def loss_frozen(struct, probes, G, pairs, occupancy=None):
    pos, spec, cell, pbc = struct
    pos, pp = _d(pos)
    spec, sp = _i(spec)
    cell, cp = _d(np.asarray(cell).reshape(9))
    keep, a = _probe_args(probes)
    po, pop = _l(pairs[0]); pj, pjp = _i(pairs[1]); pn, pnp = _i(pairs[2]); pq, pqp = _d(pairs[3])
    G, gp = _d(G)
    out = ctypes.c_double(0.0)
    occ, op = _occ(occupancy, len(pos))
    _check(lib().oracle_loss_frozen(len(pos), pp, sp, cp, *a, pop, pjp, pnp, pqp, gp, ctypes.byref(out), op))
    return out.value


def solid_harmonic(a: int, b: int, c: int, pts):
    pts, p = _d(np.asarray(pts).reshape(-1, 3))
    v = np.zeros(len(pts)); g = np.zeros((len(pts), 3))
    lib().oracle_solid_harmonic(a, b, c, len(pts), p, v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return v, g


def radial(l: int, sigma: float, B, beta, q):
    B, Bp = _d(B); beta, bp = _d(beta); q, qp = _d(np.atleast_1d(q))
    out = np.zeros(len(q))
    lib().oracle_radial(int(l), float(sigma), len(B), Bp, bp, len(q), qp,
                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def components(l: int):
    """(a, b, c) of order l in the oracle's component order."""
    out = []
    for a in range(l, -1, -1):
        for b in range(l - a, -1, -1):
            out.append((a, b, l - a - b))
    return out


# ---------------------------------------------------------------- reference points
def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def point_neighbors(struct, rc2, point):
    """Canonical neighbour list of one reference point (same dict as neighbors())."""
    pos, spec, cell, pbc = struct
    pos, pp = _d(pos)
    spec, sp = _i(spec)
    cell, cp = _d(np.asarray(cell).reshape(9))
    rc2, rp = _d(rc2)
    pt, ptp = _d(np.asarray(point).reshape(3))
    st = ctypes.c_int32(0)
    cap = 1024
    while True:
        j = np.zeros(cap, np.int32); n = np.zeros((cap, 3), np.int32)
        q = np.zeros(cap); sh = np.zeros(cap, np.int32)
        cnt = lib().oracle_point_neighbors(len(pos), pp, sp, cp, int(pbc), len(rc2), rp, ptp, cap,
                                           j.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                           n.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(q),
                                           sh.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(st))
        _check(st.value)
        if cnt <= cap:
            return dict(j=j[:cnt], n=n[:cnt], q=q[:cnt], shell=sh[:cnt], e=np.asarray(spec)[j[:cnt]])
        cap = int(cnt)


def point_features(struct, probes, points, with_mu: bool = False, occupancy=None):
    """F [n_points, nf] (and mu [n_points, nc]) at reference points [n_points, 3]."""
    pos, spec, cell, pbc = struct
    pos, pp = _d(pos)
    spec, sp = _i(spec)
    cell, cp = _d(np.asarray(cell).reshape(9))
    pts, ptp = _d(np.asarray(points, np.float64).reshape(-1, 3))
    keep, a = _probe_args(probes)
    nf = n_features(probes.orders, len(probes.sigmas))
    F = np.zeros((len(pts), nf))
    mu = np.zeros((len(pts), n_components(probes.orders, len(probes.sigmas)))) if with_mu else None
    occ, op = _occ(occupancy, len(pos))
    _check(lib().oracle_point_features(len(pos), pp, sp, cp, int(pbc), *a, len(pts), ptp, _dp(F),
                                       _dp(mu) if with_mu else None, op))
    return (F, mu) if with_mu else F


def point_features_batch(batch, probes, point_offsets, points, with_mu=False):
    """Features at the reference points of every structure of a batch
    (points of structure s: points[point_offsets[s]:point_offsets[s+1]])."""
    Fs, mus = [], []
    occ = getattr(batch, "occupancy", None)
    for s in range(batch.n_structs):
        a0, a1 = int(batch.atom_offsets[s]), int(batch.atom_offsets[s + 1])
        r = point_features(batch.structure(s), probes, points[point_offsets[s]:point_offsets[s + 1]],
                           with_mu=with_mu, occupancy=None if occ is None else occ[a0:a1])
        if with_mu:
            Fs.append(r[0]); mus.append(r[1])
        else:
            Fs.append(r)
    F = np.concatenate(Fs, axis=0)
    return (F, np.concatenate(mus, axis=0)) if with_mu else F


def point_grad(struct, probes, points, G, occupancy=None):
    """dL/dR [n,3], dL/dP [n_points,3], dL/dcell [3,3] of L = sum G*F(points), plus F."""
    pos, spec, cell, pbc = struct
    pos, pp = _d(pos)
    spec, sp = _i(spec)
    cell, cp = _d(np.asarray(cell).reshape(9))
    pts, ptp = _d(np.asarray(points, np.float64).reshape(-1, 3))
    keep, a = _probe_args(probes)
    G, gp = _d(G)
    gpos = np.zeros((len(pos), 3)); gpts = np.zeros((len(pts), 3)); gcell = np.zeros((3, 3))
    F = np.zeros((len(pts), n_features(probes.orders, len(probes.sigmas))))
    occ, op = _occ(occupancy, len(pos))
    _check(lib().oracle_point_grad(len(pos), pp, sp, cp, int(pbc), *a, len(pts), ptp, gp, _dp(gpos), _dp(gpts),
                                   _dp(gcell), _dp(F), op))
    return gpos, gpts, gcell, F


def point_frozen_pairs(struct, probes, points):
    """Pair lists of the reference points in raw-position form (j, n~, q)."""
    pos, spec, cell, pbc = struct
    rc2 = cutoffs(probes)
    _, m = wrap(pos, cell, pbc)
    pts = np.asarray(points, np.float64).reshape(-1, 3)
    _, pm = wrap(pts, cell, pbc)
    po = [0]; pj = []; pn = []; pq = []
    for r in range(len(pts)):
        nb = point_neighbors(struct, rc2, pts[r])
        pj.append(nb["j"])
        pn.append(nb["n"] - m[nb["j"]] + pm[r])
        pq.append(nb["q"])
        po.append(po[-1] + len(nb["j"]))
    return (np.asarray(po, np.int64), np.concatenate(pj).astype(np.int32),
            np.concatenate(pn).reshape(-1, 3).astype(np.int32), np.concatenate(pq))


def point_loss_frozen(struct, probes, points, G, pairs, occupancy=None):
    pos, spec, cell, pbc = struct
    pos, pp = _d(pos)
    spec, sp = _i(spec)
    cell, cp = _d(np.asarray(cell).reshape(9))
    pts, ptp = _d(np.asarray(points, np.float64).reshape(-1, 3))
    keep, a = _probe_args(probes)
    po, pop = _l(pairs[0]); pj, pjp = _i(pairs[1]); pn, pnp = _i(pairs[2]); pq, pqp = _d(pairs[3])
    G, gp = _d(G)
    out = ctypes.c_double(0.0)
    occ, op = _occ(occupancy, len(pos))
    _check(lib().oracle_point_loss_frozen(len(pos), pp, sp, cp, *a, len(pts), ptp, pop, pjp, pnp, pqp, gp,
                                          ctypes.byref(out), op))
    return out.value


def jacobian(struct, probes, occupancy=None):
    """Per-pair feature Jacobian J [P, nf, 3] (dF_{i,f}/dd_p, pairs of every
    centre in canonical order, centres in index order) and the list offsets
    [n_atoms+1]."""
    pos, spec, cell, pbc = struct
    pos, pp = _d(pos)
    spec, sp = _i(spec)
    cell, cp = _d(np.asarray(cell).reshape(9))
    keep, a = _probe_args(probes)
    nf = n_features(probes.orders, len(probes.sigmas))
    occ, op = _occ(occupancy, len(pos))
    st = ctypes.c_int32(0)
    rc2 = cutoffs(probes)
    counts = [len(neighbors(struct, rc2, i)["j"]) for i in range(len(pos))]
    total = int(sum(counts))
    jac = np.zeros((max(total, 1), nf, 3))
    n = lib().oracle_jacobian(len(pos), pp, sp, cp, int(pbc), *a, total, _dp(jac), op, ctypes.byref(st))
    _check(st.value)
    assert n == total
    offs = np.zeros(len(pos) + 1, np.int64)
    offs[1:] = np.cumsum(counts)
    return jac[:total], offs
