"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every symbol include/gmp.h declares; probe validation returns the
documented status codes; the library's cutoffs equal the oracle's bit for
bit; the feature enumeration matches the paper's printed example."""
import ctypes
import json
import os
import re
import sys

import numpy as np
import pytest

import gmp_synth as gs
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    import paper_2303_12980_amd as g
    return g.load()


def _header_symbols():
    src = open(os.path.join(ROOT, "include", "gmp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gmp_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(lib):
    import paper_2303_12980_amd as g
    syms = _header_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(g.EXPORTS) == syms


def _desc(probes):
    import paper_2303_12980_amd._lib as L
    keep = [np.ascontiguousarray(probes.orders, np.int32), np.ascontiguousarray(probes.sigmas, np.float64),
            np.ascontiguousarray(probes.prim_offsets, np.int32), np.ascontiguousarray(probes.B, np.float64),
            np.ascontiguousarray(probes.beta, np.float64)]
    d = L.ProbeDesc(len(keep[0]), keep[0].ctypes.data_as(L.P_i32), len(keep[1]), keep[1].ctypes.data_as(L.P_dbl),
                    len(keep[2]) - 1, keep[2].ctypes.data_as(L.P_i32), keep[3].ctypes.data_as(L.P_dbl),
                    keep[4].ctypes.data_as(L.P_dbl), float(probes.tau))
    return d, keep


@pytest.mark.parametrize("name", ["C1", "C2", "C4"])
@pytest.mark.parametrize("density", [False, True])
def test_cutoffs_bit_exact_vs_oracle(lib, name, density):
    kw = dict(n_atoms=64) if name == "C2" else (dict(n_structs=2) if name == "C4" else {})
    _, probes = gs.config(name, **kw)
    if density:  # order -1 adds the density cutoff slot after the sigmas
        probes.orders = np.concatenate([[-1], probes.orders]).astype(np.int32)
    d, keep = _desc(probes)
    rc2 = np.zeros(oracle.n_slots(probes))
    assert lib.gmp_probe_cutoffs(ctypes.byref(d), rc2.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == 0
    assert rc2.tobytes() == oracle.cutoffs(probes).tobytes()
    assert len(rc2) == len(probes.sigmas) + int(density)


def _status(lib, probes):
    d, keep = _desc(probes)
    rc2 = np.zeros(max(1, len(probes.sigmas)) + 1)
    return lib.gmp_probe_cutoffs(ctypes.byref(d), rc2.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))


def _probes(**kw):
    base = dict(orders=np.array([0, 1, 2], np.int32), sigmas=np.array([0.5, 1.0]),
                prim_offsets=np.array([0, 2], np.int32), B=np.array([1.0, 2.0]), beta=np.array([0.5, 3.0]),
                tau=1e-8)
    base.update(kw)
    return gs.Probes(**base)


@pytest.mark.parametrize("bad,code", [
    (dict(orders=np.array([0, 5], np.int32)), 1),
    (dict(orders=np.array([1, 1], np.int32)), 1),
    (dict(orders=np.array([-1, 0], np.int32)), 0),
    (dict(orders=np.array([-1], np.int32)), 0),
    (dict(orders=np.array([0, -1, -1], np.int32)), 1),
    (dict(orders=np.array([-2, 0], np.int32)), 1),
    (dict(orders=np.array([-1, 0], np.int32), sigmas=np.linspace(0.2, 1.0, 16)), 1),
    (dict(orders=np.array([0], np.int32), sigmas=np.linspace(0.2, 1.0, 16)), 0),
    (dict(sigmas=np.array([0.5, 0.0])), 1),
    (dict(sigmas=np.array([np.nan])), 1),
    (dict(beta=np.array([0.5, -1.0])), 1),
    (dict(B=np.array([np.inf, 1.0])), 1),
    (dict(tau=0.0), 1),
    (dict(prim_offsets=np.array([0, 3, 2], np.int32), B=np.ones(3), beta=np.ones(3)), 1),
])
def test_probe_validation_codes(lib, bad, code):
    assert _status(lib, _probes(**bad)) == code


def test_valid_probes_ok(lib):
    assert _status(lib, _probes()) == 0
    assert lib.gmp_last_error() is not None


def test_paper_feature_enumeration():
    """The feature set is the Cartesian product of orders and sigmas,
    order-major; order -1 contributes a single feature."""
    from paper_2303_12980_amd.gmp import feature_labels
    fx = json.load(open(os.path.join(ROOT, "tests", "golden", "feature_enumeration.json")))
    got = feature_labels(fx["orders"], fx["sigmas"])
    want = [tuple(x) for x in fx["features"]]
    assert [(a, (0 if a == -1 else b)) for a, b in got] == [(a, (0 if a == -1 else b)) for a, b in want]


def test_screening_flag_validation(lib):
    d, keep = _desc(_probes())
    rc2 = np.zeros(4)
    for flag, code in ((0, 0), (1, 0), (2, 1), (-1, 1)):
        d.screening = flag
        assert lib.gmp_probe_cutoffs(ctypes.byref(d), rc2.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == code


def test_density_cutoff_slot_bit_exact(lib):
    """With order -1 the library's last cutoff slot is the density radius,
    bit-equal to the oracle's."""
    p = _probes(orders=np.array([2, -1, 0], np.int32))
    d, keep = _desc(p)
    rc2 = np.zeros(3)
    assert lib.gmp_probe_cutoffs(ctypes.byref(d), rc2.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == 0
    assert rc2.tobytes() == oracle.cutoffs(p).tobytes()
    assert rc2[2] == oracle.density_cutoff(p)


def test_oracle_output_layout_is_the_golden_enumeration():
    """The oracle's feature vector of an isolated dimer, position by
    position, equals the closed forms listed in the golden enumeration's
    order (every (order, sigma) has its own value)."""
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import layout_dimer as ld
    fx = ld.golden()
    p = gs.Probes(np.array(fx["orders"], np.int32), np.array(fx["sigmas"]), np.array([0, 2], np.int32),
                  ld.B, ld.BETA, 1e-12)
    want = ld.expected_vector()
    assert len(np.unique(np.round(want, 12))) == len(want)
    F = oracle.features(ld.dimer_structure(), p)[0]
    assert np.allclose(F, want, rtol=1e-13, atol=0)
