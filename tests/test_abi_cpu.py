"""Host-side tests of the C ABI: the library loads, exports what include/pcls.h
declares, and the host planner validates input with the documented codes.
No compute call is made (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2606_06656_amd import pcls, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "pcls.h")).read()
    return sorted(set(re.findall(r"\b(pcls_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = pcls.load_library()
    declared = header_functions()
    assert len(declared) >= 11
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(pcls.EXPORTS) == declared


def plan_status(n, row_ptr, lit, types, params=None, weights=None):
    L = pcls.load_library()
    rp = np.ascontiguousarray(row_ptr, np.int32)
    li = np.ascontiguousarray(lit, np.int32)
    ty = np.ascontiguousarray(types, np.int8)
    pa = None if params is None else np.ascontiguousarray(params, np.int32)
    we = None if weights is None else np.ascontiguousarray(weights, np.float32)
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    st = L.pcls_plan(n, len(rp) - 1, rp.ctypes.data, li.ctypes.data if len(li) else None, ty.ctypes.data,
                     None if pa is None else pa.ctypes.data, None if we is None else we.ctypes.data,
                     ctypes.byref(h), ctypes.byref(ws))
    msg = L.pcls_last_error().decode()
    if st == 0:
        L.pcls_destroy(h)
    return st, msg, ws.value


def test_plan_accepts_valid():
    st, msg, ws = plan_status(4, [0, 3, 5], [1, -2, 3, 4, -1], [0, 1], [0, 1])
    assert st == pcls.PCLS_OK, msg
    assert ws > 0 and ws % 256 == 0


@pytest.mark.parametrize("case,code", [
    (dict(n=3, row_ptr=[1, 3], lit=[1, 2, 3], types=[0]), pcls.PCLS_E_INVALID),          # row_ptr[0] != 0
    (dict(n=3, row_ptr=[0, 2, 1], lit=[1, 2], types=[0, 0]), pcls.PCLS_E_INVALID),       # decreasing
    (dict(n=3, row_ptr=[0, 0], lit=[], types=[0]), pcls.PCLS_E_INVALID),                 # empty constraint
    (dict(n=3, row_ptr=[0, 2], lit=[1, 0], types=[0]), pcls.PCLS_E_INVALID),             # literal 0
    (dict(n=3, row_ptr=[0, 2], lit=[1, 4], types=[0]), pcls.PCLS_E_INVALID),             # out of range
    (dict(n=3, row_ptr=[0, 2], lit=[1, -4], types=[0]), pcls.PCLS_E_INVALID),
    (dict(n=3, row_ptr=[0, 2], lit=[2, -2], types=[0]), pcls.PCLS_E_DUPVAR),             # repeated variable
    (dict(n=3, row_ptr=[0, 2], lit=[1, 2], types=[9]), pcls.PCLS_E_INVALID),             # bad type
    (dict(n=3, row_ptr=[0, 2], lit=[1, 2], types=[1], params=[2]), pcls.PCLS_E_INVALID),  # XOR parity
    (dict(n=3, row_ptr=[0, 2], lit=[1, 2], types=[2], params=[3]), pcls.PCLS_E_INVALID),  # kappa > k
    (dict(n=3, row_ptr=[0, 2], lit=[1, 2], types=[2], params=[-1]), pcls.PCLS_E_INVALID),
    (dict(n=3, row_ptr=[0, 2], lit=[1, 2], types=[0], weights=[np.inf]), pcls.PCLS_E_INVALID),
    (dict(n=0, row_ptr=[0], lit=[], types=[]), pcls.PCLS_E_INVALID),                     # no variables
])
def test_plan_rejects(case, code):
    st, msg, _ = plan_status(case["n"], case["row_ptr"], case["lit"], case["types"], case.get("params"),
                             case.get("weights"))
    assert st == code, msg
    assert msg


def test_plan_rejects_long_constraint():
    n = 300
    st, msg, _ = plan_status(n, [0, 257], list(range(1, 258)), [0])
    assert st == pcls.PCLS_E_UNSUPPORTED, msg
    st, msg, _ = plan_status(n, [0, 256], list(range(1, 257)), [0])
    assert st == pcls.PCLS_OK, msg


def test_plan_null_pointers():
    L = pcls.load_library()
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    assert L.pcls_plan(3, 1, None, None, None, None, None, ctypes.byref(h), ctypes.byref(ws)) == pcls.PCLS_E_INVALID
    rp = np.array([0, 2], np.int32)
    assert L.pcls_plan(3, 1, rp.ctypes.data, None, None, None, None, ctypes.byref(h),
                       ctypes.byref(ws)) == pcls.PCLS_E_INVALID
    assert L.pcls_plan(3, 1, rp.ctypes.data, None, None, None, None, None, None) == pcls.PCLS_E_INVALID


def test_unbound_problem_calls_fail_cleanly():
    inst = synth.c1_3sat(0)
    p = pcls.Plan.from_instance(inst)
    L = pcls.load_library()
    assert L.pcls_evaluate(p.handle, 4, None, None, None, None) == pcls.PCLS_E_WORKSPACE
    assert L.pcls_step(p.handle, 4, None, 0.1, 1, None, None) == pcls.PCLS_E_WORKSPACE
    assert L.pcls_extract(p.handle, 4, None, None, None, None, None) == pcls.PCLS_E_WORKSPACE
    assert L.pcls_upload(p.handle, None, 1 << 20, None) == pcls.PCLS_E_WORKSPACE
    assert L.pcls_upload(p.handle, ctypes.c_void_p(256), 16, None) == pcls.PCLS_E_WORKSPACE  # too small
    assert L.pcls_upload(None, None, 0, None) == pcls.PCLS_E_INVALID


def test_info_and_launch_settings():
    inst = synth.c2_mixed()
    p = pcls.Plan.from_instance(inst)
    info = p.info()
    assert (info.n_vars, info.n_cons, info.n_lits, info.max_len) == (2000, 6800, 22600, 8)
    assert info.n_segments == 3  # OR-3 products, XOR-5 products, CARD>=3 of 8 through the count window
    assert dict(zip(pcls.KIND_NAMES, info.cons_by_kind)) == {"prod1": 6600, "prod2": 0, "dft": 0, "pmf": 200,
                                                             "const": 0}
    assert info.lds_bytes_per_restart == 2000 * 8
    p.set_launch(4, 1024)
    assert (p.info().tile_restarts, p.info().block_threads) == (4, 1024)
    with pytest.raises(pcls.PclsError):
        p.set_launch(3, 0)
    with pytest.raises(pcls.PclsError):
        p.set_launch(0, 300)
    with pytest.raises(pcls.PclsError):
        p.set_launch(64, 0)  # 2000 x 64 restarts do not fit in LDS
    g = pcls.Plan.from_instance(inst, force_generic=True)
    assert g.info().n_segments == 3
    assert list(g.info().cons_by_kind) == [0, 0, 6800, 0, 0]


def test_plan_segments_by_kind():
    inst = synth.mixed_small(n=64, seed=3, kmax=40, count=200)
    p = pcls.Plan.from_instance(inst)
    info = p.info()
    assert info.n_cons == inst.m and info.n_lits == inst.L
    assert 1 <= info.n_segments <= 4 * 18


def _expected_kind(sp):
    """Evaluation path the planner should pick for a spectrum (sp_t = -1 when the
    constraint holds with t true literals): a product form when one exists, the
    count window when the spectrum is constant past w counts at one end with
    w <= 4 for k <= 8, or w <= half the length bucket (12, 16, 24, 32, 48)
    for 8 < k <= 48, else the DFT."""
    k = len(sp) - 1
    if all(v == sp[0] for v in sp):
        return "const"
    if all(v == sp[1] for v in sp[1:]) or all(v == sp[0] for v in sp[:k]):
        return "prod1"
    if all(sp[t] == (sp[0] if t % 2 == 0 else -sp[0]) for t in range(k + 1)):
        return "prod1"
    if k >= 3 and all(v == sp[1] for v in sp[1:k]):
        return "prod2"
    wt = max([t + 1 for t in range(k + 1) if sp[t] != sp[k]], default=0)
    wf = max([f + 1 for f in range(k + 1) if sp[k - f] != sp[0]], default=0)
    if k <= 8 and min(wt, wf) <= 4:
        return "pmf"
    bucket = next(b for b in (12, 16, 24, 32, 48, 10 ** 9) if k <= b)
    if 8 < k <= 48 and 2 * min(wt, wf) <= bucket:
        return "pmf"
    return "dft"


@pytest.mark.parametrize("k", list(range(1, 18)) + [23, 24, 25, 31, 32, 33, 47, 48, 49, 63, 64, 65])
def test_plan_picks_evaluation_path(k):
    from oracle import coeffs as C
    for ctype in (C.OR, C.XOR, C.CARD_GE, C.NAE, C.EO, C.AMO, C.EK):
        params = range(k + 1) if ctype in (C.CARD_GE, C.EK) else ([0, 1] if ctype == C.XOR else [0])
        for prm in params:
            inst = synth.Instance(n=k, row_ptr=np.array([0, k], np.int32), lit=np.arange(1, k + 1, dtype=np.int32),
                                  ctype=np.array([ctype], np.int8), param=np.array([prm], np.int32))
            counts = dict(zip(pcls.KIND_NAMES, pcls.Plan.from_instance(inst).info().cons_by_kind))
            want = _expected_kind(list(C.spectrum(ctype, k, prm)))
            assert counts[want] == 1, (C.TYPE_NAMES[ctype], k, prm, counts, want)


def test_bucket_tables():
    """Table 1 pads lengths above 8 to powers of two only: fewer or equal
    segments, the same evaluation kinds for the short constraints; the table is
    reported and an unknown table is refused."""
    inst = synth.mixed_small(n=120, seed=4, kmax=40, count=300)
    p0 = pcls.Plan.from_instance(inst)
    p1 = pcls.Plan.from_instance(inst, bucket_table=1)
    assert p0.info().bucket_table == 0 and p1.info().bucket_table == 1
    assert p1.info().n_segments <= p0.info().n_segments
    assert p0.info().n_cons == p1.info().n_cons == inst.m
    with pytest.raises(pcls.PclsError) as e:
        pcls.Plan.from_instance(inst, bucket_table=2)
    assert e.value.status == pcls.PCLS_E_INVALID
    # a 12-literal threshold: count window of 6 fits the 12 bucket (table 0) and the 16 bucket (table 1)
    k = 12
    one = synth.Instance(n=k, row_ptr=np.array([0, k], np.int32), lit=np.arange(1, k + 1, dtype=np.int32),
                         ctype=np.array([synth.CARD_GE], np.int8), param=np.array([6], np.int32))
    for t in (0, 1):
        counts = dict(zip(pcls.KIND_NAMES, pcls.Plan.from_instance(one, bucket_table=t).info().cons_by_kind))
        assert counts["pmf"] == 1
