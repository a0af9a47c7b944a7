"""Python front end of the gfx950 GMP feature library.

Thin marshalling over the C ABI (include/gmp.h): PyTorch provides device
memory and the current stream; every step of the path (wrap, cell list,
neighbour lists, overlaps, norms, adjoint) runs in libgmp.so.

Feature layout follows the featurizer's enumeration (paper, "Examples"):
the probe set is the Cartesian product orders x sigmas, order-major and
sigma-minor; order -1 (the local density) takes no sigma and contributes a
single feature where it stands in the orders.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import GMPError, check

__all__ = ["GMPPlan", "DeviceBatch", "Neighbors", "Workspace", "build_neighbors", "rebuild_neighbors_nosync",
           "build_reverse",
           "check_status", "features", "features_backward", "feature_jacobian", "pair_centres", "pairs_by_centre",
           "GMPFunction",
           "CapturedStep", "feature_labels",
           "profile", "GMPError"]


def _stream_ptr(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def feature_labels(orders: Sequence[int], sigmas: Sequence[float]):
    """(order, sigma) of every feature in output order.  Order -1 (the local
    density) carries no sigma and contributes one feature, listed first where
    it appears in the orders."""
    out = []
    for l in orders:
        if l == -1:
            out.append((-1, 0))
            continue
        for s in sigmas:
            out.append((int(l), float(s)))
    return out


class GMPPlan:
    """Probe set + density primitives + precision (wraps gmp_plan)."""

    def __init__(self, orders, sigmas, prim_offsets, B, beta, overlap_threshold, precision="fp32c",
                 screening=False, radial_intervals=0):
        """radial_intervals > 0 (FP32 precisions): the forward reads the radial
        factors from per-(slot, element, order) cubic tables in r = sqrt(q)
        with that many intervals (see gmp_probe_desc.radial_intervals)."""
        L = _lib.load()
        self._orders = np.ascontiguousarray(orders, dtype=np.int32)
        self._sigmas = np.ascontiguousarray(sigmas, dtype=np.float64)
        self._poff = np.ascontiguousarray(prim_offsets, dtype=np.int32)
        self._B = np.ascontiguousarray(B, dtype=np.float64)
        self._beta = np.ascontiguousarray(beta, dtype=np.float64)
        self.tau = float(overlap_threshold)
        prec = {"fp64": _lib.GMP_FP64, "fp32c": _lib.GMP_FP32_COMPENSATED, "fp32w": _lib.GMP_FP32_WIDE}[precision]
        self.precision = precision
        d = _lib.ProbeDesc(len(self._orders), self._orders.ctypes.data_as(_lib.P_i32),
                           len(self._sigmas), self._sigmas.ctypes.data_as(_lib.P_dbl),
                           len(self._poff) - 1, self._poff.ctypes.data_as(_lib.P_i32),
                           self._B.ctypes.data_as(_lib.P_dbl), self._beta.ctypes.data_as(_lib.P_dbl),
                           self.tau, 1 if screening else 0, int(radial_intervals))
        self.screening = bool(screening)
        self.radial_intervals = int(radial_intervals)
        h = ctypes.c_void_p(0)
        check(L.gmp_plan_create(ctypes.byref(d), prec, ctypes.byref(h)))
        self._h = h
        nf, nc, ns = _lib.c_i32(0), _lib.c_i32(0), _lib.c_i32(0)
        check(L.gmp_plan_info(h, ctypes.byref(nf), ctypes.byref(nc), ctypes.byref(ns), None))
        rc2 = np.zeros(ns.value)
        check(L.gmp_plan_info(h, None, None, None, rc2.ctypes.data_as(_lib.P_dbl)))
        # cutoff slots: the sigmas, then the local density when order -1 is requested
        self.n_features, self.n_components, self.n_slots, self.rc2 = nf.value, nc.value, ns.value, rc2
        self.n_elements = len(self._poff) - 1
        self.dtype = torch.float64 if precision == "fp64" else torch.float32

    @classmethod
    def from_probes(cls, probes, precision="fp32c"):
        return cls(probes.orders, probes.sigmas, probes.prim_offsets, probes.B, probes.beta, probes.tau,
                   precision, getattr(probes, "screening", False), getattr(probes, "radial_intervals", 0))

    @property
    def orders(self):
        return self._orders.copy()

    @property
    def sigmas(self):
        return self._sigmas.copy()

    @property
    def handle(self):
        return self._h

    def labels(self):
        return feature_labels(self._orders, self._sigmas)

    def get_tuning(self) -> dict:
        t = _lib.Tuning()
        check(_lib.load().gmp_plan_get_tuning(self._h, ctypes.byref(t)))
        return dict(chunk_pairs=t.chunk_pairs, bin_divisor=t.bin_divisor, blocks_per_cu=t.blocks_per_cu,
                    adj_items=t.adj_items, sigma_groups=t.sigma_groups)

    def set_tuning(self, **kw):
        cur = self.get_tuning()
        cur.update(kw)
        t = _lib.Tuning(cur["chunk_pairs"], cur["bin_divisor"], cur["blocks_per_cu"], cur["adj_items"],
                        cur["sigma_groups"])
        check(_lib.load().gmp_plan_set_tuning(self._h, ctypes.byref(t)))

    def workspace_bytes(self, n_structs, n_atoms, capacity, n_points=0) -> int:
        b = ctypes.c_size_t(0)
        check(_lib.load().gmp_workspace_size(self._h, int(n_structs), int(n_atoms), int(n_points), int(capacity),
                                             ctypes.byref(b)))
        return int(b.value)

    def batch_workspace_bytes(self, batch: "DeviceBatch", capacity) -> int:
        return self.workspace_bytes(batch.n_structs, batch.n_atoms, capacity, batch.n_points)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib._lib is not None:
            _lib._lib.gmp_plan_destroy(h)
            self._h = None


class DeviceBatch:
    """Packed CSR batch resident on the GPU (wraps gmp_batch)."""

    def __init__(self, atom_offsets, pos, species, cell, pbc, device="cuda", occupancy=None, points=None,
                 point_offsets=None):
        """occupancy: per-atom fractional site occupancies (disordered
        structures), or None for all 1.  points [M, 3] with point_offsets
        [n_structs+1]: reference points, which then are the centres (features
        at those positions instead of at the atoms)."""
        self.atom_offsets = torch.as_tensor(np.asarray(atom_offsets, np.int64), device=device)
        pos = torch.as_tensor(np.asarray(pos, np.float64), device=device)
        self.xyz = pos.t().contiguous()  # [3, N] SoA
        self.species = torch.as_tensor(np.asarray(species, np.int32), device=device)
        self.cell = torch.as_tensor(np.asarray(cell, np.float64).reshape(-1, 9), device=device).contiguous()
        self.pbc = torch.as_tensor(np.asarray(pbc, np.uint8), device=device)
        self.n_structs = int(self.atom_offsets.numel() - 1)
        self.n_atoms = int(self.species.numel())
        self.occupancy = None
        if occupancy is not None:
            self.occupancy = torch.as_tensor(np.asarray(occupancy, np.float64), device=device).contiguous()
            if self.occupancy.shape != (self.n_atoms,):
                raise ValueError("occupancy must have one entry per atom")
        self.point_offsets, self.pxyz, self.n_points = None, None, 0
        if point_offsets is not None:
            po = np.asarray(point_offsets, np.int64)
            pts = np.asarray(points, np.float64).reshape(-1, 3)
            if len(po) != self.n_structs + 1 or po[0] != 0 or po[-1] != len(pts) or np.any(np.diff(po) < 0):
                raise ValueError("point_offsets must be a CSR over the structures' points")
            self.point_offsets = torch.as_tensor(po, device=device)
            self.pxyz = torch.as_tensor(pts, device=device).t().contiguous()  # [3, M] SoA
            self.n_points = len(pts)

    @property
    def n_centres(self) -> int:
        """Atoms, or the reference points when they are given."""
        return self.n_points if self.point_offsets is not None else self.n_atoms

    @property
    def n_total(self) -> int:
        return self.n_atoms + self.n_points

    @classmethod
    def from_batch(cls, b, device="cuda"):
        return cls(b.atom_offsets, b.pos, b.species, b.cell, b.pbc, device, getattr(b, "occupancy", None))

    def with_points(self, points, point_offsets) -> "DeviceBatch":
        """The same atoms (sharing memory) with reference points as the centres."""
        v = DeviceBatch.__new__(DeviceBatch)
        v.__dict__.update(self.__dict__)
        dev = self.species.device
        po = np.asarray(point_offsets, np.int64)
        pts = np.asarray(points, np.float64).reshape(-1, 3)
        if len(po) != self.n_structs + 1 or po[0] != 0 or po[-1] != len(pts) or np.any(np.diff(po) < 0):
            raise ValueError("point_offsets must be a CSR over the structures' points")
        v.point_offsets = torch.as_tensor(po, device=dev)
        v.pxyz = torch.as_tensor(pts, device=dev).t().contiguous()
        v.n_points = len(pts)
        return v

    def structure(self, s: int, a0: int, a1: int) -> "DeviceBatch":
        """One-structure batch viewing this batch's memory (atoms a0:a1 of
        structure s); host offsets are passed in to avoid a device read."""
        v = DeviceBatch.__new__(DeviceBatch)
        dev = self.species.device
        v.atom_offsets = torch.tensor([0, a1 - a0], dtype=torch.int64, device=dev)
        v.xyz = self.xyz[:, a0:a1]
        v.species = self.species[a0:a1]
        v.cell = self.cell[s:s + 1]
        v.pbc = self.pbc[s:s + 1]
        v.occupancy = None if self.occupancy is None else self.occupancy[a0:a1]
        v.point_offsets, v.pxyz, v.n_points = None, None, 0
        v.n_structs, v.n_atoms = 1, a1 - a0
        return v

    def desc(self, xyz: Optional[torch.Tensor] = None, cell: Optional[torch.Tensor] = None):
        xyz = self.xyz if xyz is None else xyz
        cell = self.cell if cell is None else cell
        return _lib.BatchDesc(self.n_structs, self.n_atoms, self.atom_offsets.data_ptr(), xyz[0].data_ptr(),
                              xyz[1].data_ptr(), xyz[2].data_ptr(), self.species.data_ptr(), cell.data_ptr(),
                              self.pbc.data_ptr(),
                              self.occupancy.data_ptr() if self.occupancy is not None else 0,
                              self.n_points, self.point_offsets.data_ptr() if self.point_offsets is not None else 0,
                              *((self.pxyz[k].data_ptr() for k in range(3)) if self.n_points > 0 else (0, 0, 0)))


class Workspace:
    """Grow-only device scratch buffer."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = torch.empty(0, dtype=torch.uint8, device=device)

    def get(self, nbytes: int) -> torch.Tensor:
        if self.buf.numel() < nbytes:
            self.buf = torch.empty(int(nbytes * 1.1) + 4096, dtype=torch.uint8, device=self.device)
        return self.buf


class Neighbors:
    """Canonical neighbour lists (wraps gmp_neighbors)."""

    def __init__(self, plan: GMPPlan, batch: DeviceBatch, capacity: int, reverse: bool = True):
        dev = batch.species.device
        N, NT = batch.n_centres, batch.n_total  # lists per centre; wrap / rw per atom and point
        E, S = plan.n_elements, plan.n_slots
        self.capacity = int(capacity)
        self.n_pairs = 0   # pairs of the last synchronous build (host views of the lists)
        self.synced = False  # False after a no-sync rebuild: the pair count is known on the device only
        self.max_list = 0  # longest list of the last synchronous build (sizes no-sync rebuilds)
        self.offsets = torch.zeros(N + 1, dtype=torch.int64, device=dev)
        self.j = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=dev)
        self.shift = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=dev)
        self.bucket_start = torch.empty(N * (S * E + 1), dtype=torch.int32, device=dev)
        self.sigma_end = torch.empty(N * S, dtype=torch.int32, device=dev)
        self.wrap = torch.empty(NT * 3, dtype=torch.int32, device=dev)
        self.rw = torch.empty(3 * NT, dtype=torch.float64, device=dev)
        # list slots: slot k holds the list of centre order[k]; slot[i] is the slot of centre i
        self.order = torch.empty(max(N, 1), dtype=torch.int32, device=dev)
        self.slot = torch.empty(max(N, 1), dtype=torch.int32, device=dev)
        # reference points need no reverse index (the backward orders pairs by neighbour itself)
        reverse = reverse and batch.point_offsets is None
        self.reverse = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=dev) if reverse else None

    def desc(self):
        # after a no-sync rebuild the count of the earlier synchronous build is
        # stale: pass 0 (unknown), so the library bounds pair ranges by the
        # capacity and the list ends it reads on the device
        return _lib.NbrDesc(self.capacity, self.n_pairs if self.synced else 0, self.offsets.data_ptr(), self.j.data_ptr(),
                            self.shift.data_ptr(), self.bucket_start.data_ptr(), self.sigma_end.data_ptr(),
                            self.wrap.data_ptr(), self.rw.data_ptr(),
                            self.reverse.data_ptr() if self.reverse is not None else 0, self.max_list,
                            self.order.data_ptr(), self.slot.data_ptr())

    def list_range(self, i):
        """[lo, hi) of centre i's list in j / shift (host read)."""
        k = int(self.slot[i])
        return int(self.offsets[k]), int(self.offsets[k + 1])

    # host-side views for tests
    def shifts_numpy(self):
        w = self.shift[: self.n_pairs].cpu().numpy().view(np.uint8).reshape(-1, 4)
        return w[:, :3].view(np.int8).astype(np.int32), w[:, 3].astype(np.int32)


def build_neighbors(plan: GMPPlan, batch: DeviceBatch, ws: Workspace, capacity: Optional[int] = None,
                    reverse: bool = True, stream=None, out: Optional[Neighbors] = None,
                    defer_reverse: bool = False) -> Neighbors:
    """Neighbour lists with the two-call capacity pattern.  ``out`` reuses
    the buffers of an earlier result for the same batch shape when its
    capacity suffices.  With ``defer_reverse`` the reverse-pair search is
    left to build_reverse (which may run on another stream while the
    forward runs)."""
    L = _lib.load()
    call = L.gmp_build_lists if defer_reverse else L.gmp_build_neighbors
    if capacity is None:
        capacity = out.capacity if out is not None else max(1024, batch.n_centres * 64)
    for _ in range(2):
        if out is not None and out.capacity >= capacity and (out.reverse is not None) == (
                reverse and batch.point_offsets is None):
            nb = out
        else:
            nb = Neighbors(plan, batch, capacity, reverse)
        nbytes = plan.batch_workspace_bytes(batch, nb.capacity)
        buf = ws.get(nbytes)
        bd, nd = batch.desc(), nb.desc()
        npairs = ctypes.c_int64(0)
        st = call(plan.handle, ctypes.byref(bd), ctypes.byref(nd), ctypes.byref(npairs), _ptr(buf), buf.numel(),
                  _stream_ptr(stream))
        if st == _lib.GMP_E_CAPACITY:
            capacity = int(npairs.value)
            continue
        check(st)
        nb.n_pairs = int(npairs.value)
        nb.synced = True
        nb.max_list = int(nd.max_list)
        return nb
    raise GMPError(_lib.GMP_E_CAPACITY, "capacity retry failed")


def rebuild_neighbors_nosync(plan: GMPPlan, batch: DeviceBatch, ws: Workspace, nb: Neighbors, stream=None,
                             defer_reverse: bool = False):
    """Rebuild the lists into nb without any host synchronization (usable
    under stream capture).  nb.capacity must suffice; an overflow or a
    device-side error is reported later by check_status()."""
    L = _lib.load()
    call = L.gmp_build_lists if defer_reverse else L.gmp_build_neighbors
    nbytes = plan.batch_workspace_bytes(batch, nb.capacity)
    buf = ws.get(nbytes)
    bd, nd = batch.desc(), nb.desc()
    check(call(plan.handle, ctypes.byref(bd), ctypes.byref(nd), None, _ptr(buf), buf.numel(), _stream_ptr(stream)))
    nb.synced = False
    return nb


def build_reverse(plan: GMPPlan, batch: DeviceBatch, ws: Workspace, nb: Neighbors, stream=None):
    """Reverse-pair index of lists built with defer_reverse into ``ws``."""
    bd, nd = batch.desc(), nb.desc()
    check(_lib.load().gmp_build_reverse(plan.handle, ctypes.byref(bd), ctypes.byref(nd), _ptr(ws.buf),
                                        ws.buf.numel(), _stream_ptr(stream)))
    return nb


def check_status(ws: Workspace, stream=None):
    """Synchronize and raise on a device-side condition recorded in ws."""
    check(_lib.load().gmp_check_status(_ptr(ws.buf), ws.buf.numel(), _stream_ptr(stream)))


def features(plan: GMPPlan, batch: DeviceBatch, nb: Neighbors, ws: Workspace, with_components=True,
             xyz=None, cell=None, out=None, comp_out=None, stream=None):
    L = _lib.load()
    N = batch.n_centres
    dev = batch.species.device
    F = out if out is not None else torch.empty((N, plan.n_features), dtype=plan.dtype, device=dev)
    mu = None
    if with_components:
        mu = comp_out if comp_out is not None else torch.empty((N, plan.n_components), dtype=torch.float64,
                                                               device=dev)
    nbytes = plan.batch_workspace_bytes(batch, nb.capacity)
    buf = ws.get(nbytes)
    bd, nd = batch.desc(xyz, cell), nb.desc()
    check(L.gmp_features(plan.handle, ctypes.byref(bd), ctypes.byref(nd), _ptr(F), _ptr(mu), _ptr(buf),
                         buf.numel(), _stream_ptr(stream)))
    return F, mu


def features_backward(plan: GMPPlan, batch: DeviceBatch, nb: Neighbors, ws: Workspace, mu, F, G,
                      want_cell=True, xyz=None, cell=None, stream=None):
    """dL/dpositions [n_total, 3] (atoms, then reference points) and
    dL/dcell [n_structs, 3, 3] for L = sum G*F."""
    L = _lib.load()
    N = batch.n_total
    dev = batch.species.device
    G = G.to(dtype=plan.dtype).contiguous()
    gpos = torch.empty(3 * N, dtype=torch.float64, device=dev)
    gcell = torch.empty(batch.n_structs * 9, dtype=torch.float64, device=dev) if want_cell else None
    nbytes = plan.batch_workspace_bytes(batch, nb.capacity)
    buf = ws.get(nbytes)
    bd, nd = batch.desc(xyz, cell), nb.desc()
    check(L.gmp_features_backward(plan.handle, ctypes.byref(bd), ctypes.byref(nd), _ptr(mu), _ptr(F), _ptr(G),
                                  _ptr(gpos), _ptr(gcell), _ptr(buf), buf.numel(), _stream_ptr(stream)))
    gp = gpos.view(3, N).t()
    return gp, (gcell.view(-1, 3, 3) if want_cell else None)


def feature_jacobian(plan: GMPPlan, batch: DeviceBatch, nb: Neighbors, ws: Workspace, mu, xyz=None, cell=None,
                     out=None, stream=None):
    """Per-pair feature Jacobian (no contraction): returns J [P, n_features, 3]
    with J[p, f] = dF_{i,f}/dd_p for pair p = (i; j, n) of the lists (a view
    of the [n_features, 3, ld] buffer the library writes; P = nb.n_pairs).
    Centres of the pairs: pair_centres(nb); neighbours: nb.j."""
    L = _lib.load()
    ld = nb.n_pairs if nb.synced and nb.n_pairs > 0 else nb.capacity
    dev = batch.species.device
    buf = out if out is not None else torch.empty((plan.n_features, 3, max(ld, 1)), dtype=plan.dtype, device=dev)
    ld = buf.shape[2]
    wsb = ws.get(plan.batch_workspace_bytes(batch, nb.capacity))
    bd, nd = batch.desc(xyz, cell), nb.desc()
    check(L.gmp_feature_jacobian(plan.handle, ctypes.byref(bd), ctypes.byref(nd), _ptr(mu), _ptr(buf), ld,
                                 _ptr(wsb), wsb.numel(), _stream_ptr(stream)))
    return buf[:, :, :nb.n_pairs].permute(2, 0, 1)


def pair_centres(nb: Neighbors):
    """Centre index of every pair of the lists (int64 [n_pairs]; the lists
    are stored per list slot, slot k holding centre order[k]'s)."""
    offs = nb.offsets
    cnt = offs[1:] - offs[:-1]
    slots = torch.repeat_interleave(torch.arange(len(cnt), device=offs.device, dtype=torch.int64), cnt)
    return nb.order[: len(cnt)].long()[slots]


def pairs_by_centre(nb: Neighbors, centres=None):
    """Pair indices of the given centres' lists (default: all), centre after
    centre in the given order, each list in its own order (int64, device)."""
    offs = nb.offsets
    N = offs.numel() - 1
    c = torch.arange(N, device=offs.device) if centres is None else torch.as_tensor(centres, device=offs.device)
    k = nb.slot[:N].long()[c.long()]
    lo, cnt = offs[k], offs[k + 1] - offs[k]
    start = torch.repeat_interleave(lo - (torch.cumsum(cnt, 0) - cnt), cnt)
    return start + torch.arange(int(cnt.sum()), device=offs.device)


class GMPFunction(torch.autograd.Function):
    """features = GMPFunction.apply(xyz [3,N] fp64, cell [n_s,9] fp64, plan, batch, nbrs, ws).

    The neighbour lists (pair set) are held fixed: the gradient is that of
    the features over the given pairs, dL/dxyz and dL/dcell with Cartesian
    positions held fixed when the cell moves."""

    @staticmethod
    def forward(ctx, xyz, cell, plan, batch, nb, ws):
        F, mu = features(plan, batch, nb, ws, True, xyz=xyz.contiguous(), cell=cell.contiguous())
        ctx.save_for_backward(xyz, cell, F, mu)
        ctx.plan, ctx.batch, ctx.nb, ctx.ws = plan, batch, nb, ws
        return F

    @staticmethod
    def backward(ctx, gF):
        xyz, cell, F, mu = ctx.saved_tensors
        gp, gc = features_backward(ctx.plan, ctx.batch, ctx.nb, ctx.ws, mu, F, gF.contiguous(), True,
                                   xyz=xyz.contiguous(), cell=cell.contiguous())
        return gp[:ctx.batch.n_atoms].t().contiguous(), gc.reshape(-1, 9), None, None, None, None


class CapturedStep:
    """Neighbour rebuild (no-sync mode) + forward (+ adjoint) recorded once
    into a HIP graph through torch.cuda.graph and replayed: one host call
    launches the whole batch.  Outputs live in fixed buffers (F, mu, and
    grad_pos / grad_cell when backward=True); inputs are read from the
    batch's tensors, so updating batch.xyz / batch.cell in place and
    replaying featurizes the new geometry.  `nb` (from a sync build) fixes
    the capacity; call check_status(ws) to see overflows.  With backward
    and concurrent_reverse, the reverse-pair search is recorded on a second
    stream beside the forward and the adjoint waits for it: slower than one
    stream where the search is short (4096 atoms: 1.08 -> 1.12 ms), faster
    where it is long and bound by memory latency (100,000 atoms: 56.2 ->
    52.9 ms); off by default, autotune.autotune times both for a step."""

    def __init__(self, plan: GMPPlan, batch: DeviceBatch, ws: Workspace, nb: Neighbors, backward=False, G=None,
                 concurrent_reverse=False):
        self.plan, self.batch, self.ws, self.nb = plan, batch, ws, nb
        dev = batch.species.device
        N = batch.n_centres
        ws.get(plan.batch_workspace_bytes(batch, nb.capacity))  # grow before capture
        self.F = torch.empty((N, plan.n_features), dtype=plan.dtype, device=dev)
        self.mu = torch.empty((N, plan.n_components), dtype=torch.float64, device=dev)
        self.backward = backward
        self.split = backward and concurrent_reverse and nb.reverse is not None
        if self.split:
            self.rev_stream = torch.cuda.Stream()
            self.ev_built = torch.cuda.Event()
            self.ev_rev = torch.cuda.Event()
        if backward:
            self.G = torch.zeros((N, plan.n_features), dtype=plan.dtype, device=dev)
            if G is not None:
                self.G.copy_(G)
            self.gpos = torch.empty(3 * batch.n_total, dtype=torch.float64, device=dev)
            self.gcell = torch.empty(batch.n_structs * 9, dtype=torch.float64, device=dev)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self._run()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._run()
        # the graph holds raw addresses: keep every buffer it touches alive;
        # the workspace buffer is the one captured (ws.buf may be replaced
        # later by a larger eager call on the same Workspace)
        self.ws_buf = ws.buf
        self._held = (ws.buf, nb.offsets, nb.j, nb.shift, nb.bucket_start, nb.sigma_end, nb.wrap, nb.rw,
                      nb.reverse, nb.order, nb.slot, batch.xyz, batch.cell, batch.species, batch.atom_offsets, batch.pbc,
                      batch.occupancy, batch.point_offsets, batch.pxyz)

    def _run(self):
        L = _lib.load()
        main = torch.cuda.current_stream()
        rebuild_neighbors_nosync(self.plan, self.batch, self.ws, self.nb, defer_reverse=self.split)
        if self.split:
            self.ev_built.record(main)
            self.rev_stream.wait_event(self.ev_built)
            with torch.cuda.stream(self.rev_stream):
                build_reverse(self.plan, self.batch, self.ws, self.nb)
            self.ev_rev.record(self.rev_stream)
        features(self.plan, self.batch, self.nb, self.ws, True, out=self.F, comp_out=self.mu)
        if self.backward:
            if self.split:
                main.wait_event(self.ev_rev)
            buf = self.ws.buf
            bd, nd = self.batch.desc(), self.nb.desc()
            check(L.gmp_features_backward(self.plan.handle, ctypes.byref(bd), ctypes.byref(nd), _ptr(self.mu),
                                          _ptr(self.F), _ptr(self.G), _ptr(self.gpos), _ptr(self.gcell), _ptr(buf),
                                          buf.numel(), _stream_ptr(None)))

    def replay(self):
        self.graph.replay()

    def check_status(self, stream=None):
        """Synchronize and raise on a device-side condition (list overflow,
        a list that outgrew the sort, non-finite input) that replays recorded
        in the captured workspace."""
        check(_lib.load().gmp_check_status(_ptr(self.ws_buf), self.ws_buf.numel(), _stream_ptr(stream)))


class profile:
    """Context manager: per-kernel HIP-event timings of library launches."""

    def __enter__(self):
        check(_lib.load().gmp_profile_begin())
        self.result = {}
        return self

    def __exit__(self, *exc):
        n = _lib.c_i32(0)
        names = ctypes.create_string_buffer(64 * 64)
        launches = (_lib.c_i32 * 64)()
        ms = (_lib.c_dbl * 64)()
        check(_lib.load().gmp_profile_end(64, ctypes.byref(n), names, launches, ms))
        for k in range(n.value):
            nm = names.raw[64 * k: 64 * k + 64].split(b"\0", 1)[0].decode()
            self.result[nm] = (int(launches[k]), float(ms[k]))
        return False
