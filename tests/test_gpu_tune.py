"""The autotuner's persistent cache (dlpno_autotune_cached) through the C ABI:
a miss tunes and writes the entry, a later plan reads it without timing and
keeps the residual at parity; entries are kept per (architecture, precision)."""
import json

import numpy as np
import pytest

import oracle
from oracle.model import unpack_T
from tests.gpu_helpers import compare_blocks, device_problem, oracle_inputs
from workload import build_problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_autotune_cache_miss_then_hit(tmp_path):
    path = str(tmp_path / "tune.json")
    prob = build_problem("chain", n_occ=24, band=6, somos=(7, 16))
    plan, dev = device_problem(prob)
    assert plan.autotune_cached(dev["T"], path) is False
    entries = json.load(open(path))["entries"]
    assert len(entries) == 1 and entries[0]["precision"] == 0
    sched = [l for l in plan.info().splitlines() if l.startswith("ladder variants")]
    plan.close()
    plan2, dev2 = device_problem(prob)
    assert plan2.autotune_cached(dev2["T"], path) is True
    info = plan2.info()
    assert "read from" in info
    assert [l for l in info.splitlines() if l.startswith("ladder variants")] == sched
    R = plan2.residual(dev2["T"])
    torch.cuda.synchronize()
    inp = oracle_inputs(prob)
    compare_blocks(prob, R.cpu().numpy(), oracle.residual_os(inp, unpack_T(prob, prob.materialize("T"))), rel=1e-12)
    plan2.close()
    # another precision: a miss that adds its own entry and keeps the first
    p3, dev3 = device_problem(prob, precision="bf16x2")
    assert p3.autotune_cached(dev3["T"], path) is False
    entries = json.load(open(path))["entries"]
    assert sorted(e["precision"] for e in entries) == [0, 2]
    p3.close()
