"""C ABI: the library loads, exports every declared symbol, and rejects bad
descriptors during validation (before any device call) - CPU only."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2008_03237_amd", "libdlpno.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libdlpno.so not built")


def declared():
    src = open(os.path.join(ROOT, "include", "dlpno.h")).read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)      # declarations only, not the comments
    return sorted(set(re.findall(r"\b(dlpno_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    L = C.CDLL(LIB)
    names = declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def _problem(**kw):
    from paper_2008_03237_amd.lib import Problem, Pair, Inputs, Options, PAIR_DTYPE, CPL_DTYPE
    from workload import build_problem
    prob = build_problem("tiny")
    pairs = np.zeros(prob.n_pairs, dtype=PAIR_DTYPE)
    for f, v in (("i", prob.pi), ("j", prob.pj), ("npno", prob.npno), ("naux", prob.naux), ("blocks", prob.blocks),
                 ("off_B", prob.off_B), ("off_T", prob.off_T), ("off_K", prob.off_K), ("off_eps", prob.off_eps)):
        pairs[f] = v
    cpl = np.zeros(prob.n_couplings, dtype=CPL_DTYPE)
    cpl["src_pair"], cpl["k"], cpl["side"], cpl["off_S"] = prob.cpl_src, prob.cpl_k, prob.cpl_side, prob.cpl_off_S
    somo = prob.is_somo.copy()
    rowptr = prob.cpl_rowptr.copy()
    for k, fn in kw.items():
        fn(pairs, cpl, somo, rowptr)
    keep = [pairs, cpl, somo, rowptr, prob.f_a, prob.f_b]
    P = Problem(prob.n_occ, prob.n_pairs, prob.n_couplings, somo.ctypes.data, pairs.ctypes.data, rowptr.ctypes.data,
                cpl.ctypes.data, prob.f_a.ctypes.data, prob.f_b.ctypes.data, prob.n_B, prob.n_T, prob.n_K,
                len(prob.eps_a), prob.n_S, 0, None, None)
    # fake (never dereferenced) device pointers: validation fails before any device access
    I = Inputs(16, 16, 16, 16, 16)
    return P, I, keep


def _create(P, I, opts=None):
    from paper_2008_03237_amd.lib import lib, Options
    L = lib()
    h = C.c_void_p()
    st = L.dlpno_plan_create(C.byref(P), C.byref(I), C.byref(opts) if opts else None, None, C.byref(h))
    return st, L.dlpno_last_error().decode()


@pytest.mark.parametrize("mut,status", [
    ({"npno": lambda pa, c, s, r: pa.__setitem__("npno", np.where(np.arange(len(pa)) == 3, 65, pa["npno"]))}, -2),
    ({"naux": lambda pa, c, s, r: pa.__setitem__("naux", np.where(np.arange(len(pa)) == 3, 0, pa["naux"]))}, -2),
    ({"mask": lambda pa, c, s, r: pa.__setitem__("blocks", np.where(np.arange(len(pa)) == 5, pa["blocks"] ^ 1, pa["blocks"]))}, -1),
    ({"offB": lambda pa, c, s, r: pa.__setitem__("off_B", pa["off_B"] + 10 ** 9)}, -3),
    ({"ij": lambda pa, c, s, r: pa.__setitem__("i", np.where(np.arange(len(pa)) == 2, 99, pa["i"]))}, -2),
    ({"csr": lambda pa, c, s, r: r.__setitem__(3, r[4] + 1)}, -1),
    ({"side": lambda pa, c, s, r: c.__setitem__("side", np.where(np.arange(len(c)) == 7, 2, c["side"]))}, -2),
    ({"src": lambda pa, c, s, r: c.__setitem__("src_pair", np.where(np.arange(len(c)) == 7, (c["src_pair"] + 1) % len(pa), c["src_pair"]))}, -1),
    ({"offS": lambda pa, c, s, r: c.__setitem__("off_S", c["off_S"] + 10 ** 9)}, -3),
    ({"somo": lambda pa, c, s, r: s.__setitem__(0, 2)}, -1),
])
def test_validation_errors(mut, status):
    P, I, keep = _problem(**mut)
    st, msg = _create(P, I)
    assert st == status, (st, msg)
    assert msg


def test_bad_options():
    from paper_2008_03237_amd.lib import Options
    P, I, keep = _problem()
    st, _ = _create(P, I, Options(7, 8, 3, 0, 0, 0))
    assert st == -1
    st, _ = _create(P, I, Options(0, 9, 3, 0, 0, 0))
    assert st == -1


def test_status_strings():
    from paper_2008_03237_amd.lib import lib
    L = lib()
    for s in range(-8, 1):
        assert L.dlpno_status_string(s)


def test_f12_energy_rejects_a_null_plan():
    from paper_2008_03237_amd.lib import lib
    L = lib()
    st = L.dlpno_f12_energy(None, None, None, None, None, None, None)
    assert st != 0 and "NULL" in L.dlpno_last_error().decode()


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_pno_plan_validation_on_host():
    """dlpno_pno_plan_create rejects bad descriptors before touching the GPU."""
    import ctypes as C
    from paper_2008_03237_amd.lib import lib
    from workload.pno import build_pno_problem, PNO_PAIR_DTYPE
    prob = build_pno_problem("tiny")
    L = lib()
    for field, value, code in (("dim", 0, -2), ("dim", 65, -2), ("blocks", 16, -1), ("first", -1, -2),
                               ("off_C", prob.n_C, -3), ("diagonal", 2, -1)):
        bad = prob.pairs.copy()
        bad[3][field] = value
        h = C.c_void_p()
        st = L.dlpno_pno_plan_create(bad.ctypes.data_as(C.c_void_p), len(bad), prob.n_X, prob.n_F, prob.n_C,
                                     prob.n_v, C.byref(h))
        assert st == code, (field, st)
        assert h.value is None
    assert PNO_PAIR_DTYPE.itemsize == 48


def _ring_problem(precision=0, **mut):
    """The tiny workload with ring couplings (descriptors only; fake device
    pointers that validation never dereferences)."""
    from paper_2008_03237_amd.lib import Problem, Inputs, Options, PAIR_DTYPE, CPL_DTYPE, RING_DTYPE
    from workload import build_problem
    prob = build_problem("tiny", ring=0.05)
    pairs = np.zeros(prob.n_pairs, dtype=PAIR_DTYPE)
    for f, v in (("i", prob.pi), ("j", prob.pj), ("npno", prob.npno), ("naux", prob.naux), ("blocks", prob.blocks),
                 ("off_B", prob.off_B), ("off_T", prob.off_T), ("off_K", prob.off_K), ("off_eps", prob.off_eps)):
        pairs[f] = v
    cpl = np.zeros(prob.n_couplings, dtype=CPL_DTYPE)
    cpl["src_pair"], cpl["k"], cpl["side"], cpl["off_S"] = prob.cpl_src, prob.cpl_k, prob.cpl_side, prob.cpl_off_S
    ring = np.zeros(prob.n_ring, dtype=RING_DTYPE)
    ring["src_pair"], ring["m"], ring["role"] = prob.ring_src, prob.ring_m, prob.ring_role
    ring["off_S"], ring["off_X"], ring["off_J"] = prob.ring_off_S, prob.ring_off_X, prob.ring_off_J
    rrow = prob.ring_rowptr.copy()
    for fn in mut.values():
        fn(prob, ring, rrow)
    keep = [pairs, cpl, ring, rrow, prob]
    P = Problem(prob.n_occ, prob.n_pairs, prob.n_couplings, prob.is_somo.ctypes.data, pairs.ctypes.data,
                prob.cpl_rowptr.ctypes.data, cpl.ctypes.data, prob.f_a.ctypes.data, prob.f_b.ctypes.data, prob.n_B,
                prob.n_T, prob.n_K, len(prob.eps_a), prob.n_S, 0, None, None, len(ring), rrow.ctypes.data,
                ring.ctypes.data, prob.n_Rg)
    I = Inputs(16, 16, 16, 16, 16, 16)
    return P, I, Options(precision, 8, 3, 0, 0, 0), keep


def _diag_ring(prob):
    """Index of a ring coupling whose target is a diagonal pair."""
    for p in range(prob.n_pairs):
        if prob.pi[p] == prob.pj[p] and prob.ring_rowptr[p + 1] > prob.ring_rowptr[p]:
            return int(prob.ring_rowptr[p])
    raise AssertionError("no diagonal target")


@pytest.mark.parametrize("mut,status", [
    ({"role": lambda pr, r, rr: r.__setitem__("role", np.where(np.arange(len(r)) == 4, 2, r["role"]))}, -2),
    ({"diag": lambda pr, r, rr: r["role"].__setitem__(_diag_ring(pr), 1)}, -1),
    ({"m": lambda pr, r, rr: r.__setitem__("m", np.where(np.arange(len(r)) == 4, (r["m"] + 1) % pr.n_occ, r["m"]))}, -1),
    ({"offX": lambda pr, r, rr: r["off_X"].__setitem__(9, pr.n_Rg)}, -3),
    ({"offJ": lambda pr, r, rr: r["off_J"].__setitem__(9, -1)}, -3),
    ({"offS": lambda pr, r, rr: r["off_S"].__setitem__(9, pr.n_S)}, -3),
    ({"csr": lambda pr, r, rr: rr.__setitem__(3, rr[4] + 1)}, -1),
])
def test_ring_validation_errors(mut, status):
    P, I, opts, keep = _ring_problem(**mut)
    st, msg = _create(P, I, opts)
    assert st == status, (st, msg)
    assert msg


def test_ring_needs_its_integrals():
    from paper_2008_03237_amd.lib import Inputs
    P, I, opts, keep = _ring_problem()
    st, msg = _create(P, Inputs(16, 16, 16, 16, 16, None), opts)
    assert st == -1, (st, msg)


def test_unknown_option_flag():
    from paper_2008_03237_amd.lib import Options
    P, I, keep = _problem()
    st, _ = _create(P, I, Options(0, 8, 3, 0, 0, 8))
    assert st == -1                      # no such flag
