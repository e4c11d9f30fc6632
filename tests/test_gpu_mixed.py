"""Split precision (BF16x2 / FP16x2 on MFMA) and FP64 iterative refinement."""
import numpy as np
import pytest

import oracle
from oracle.model import unpack_T
from tests.gpu_helpers import device_problem, oracle_inputs
from workload import build_problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CODE = {"AA": 0, "BB": 1, "AB": 2, "BA": 3}


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("precision,rel", [("bf16x2", 2e-4), ("fp16x2", 2e-5), ("fp32", 2e-5)])
def test_split_residual_accuracy(precision, rel):
    prob = build_problem("chain", n_occ=24, band=6, somos=(7, 16))
    plan, dev = device_problem(prob, precision=precision)
    R = plan.residual(dev["T"])
    torch.cuda.synchronize()
    inp = oracle_inputs(prob)
    T = unpack_T(prob, prob.materialize("T"))
    Ro = oracle.residual_os(inp, T)
    # error of the contracted (ladder + projection) part, relative to it
    Rl = oracle.residual_os(inp, T, terms=("ladder", "projection"))
    Rg = unpack_T(prob, R.cpu().numpy())
    num = np.sqrt(sum(np.sum((Rg[k] - Ro[k]) ** 2) for k in Ro))
    den = np.sqrt(sum(np.sum(Rl[k] ** 2) for k in Rl))
    print(precision, "relative error of the contractions %.3e" % (num / den))
    assert num <= rel * den
    plan.close()


def _converged_oracle(prob, n_iter=40):
    inp = oracle_inputs(prob)
    zero = unpack_T(prob, np.zeros(prob.n_T))
    T, hist = oracle.solve(inp, zero, n_iter, use_diis=True, tol_r=1e-11, tol_e=1e-13)
    R = oracle.residual_os(inp, T)
    Tn = oracle.jacobi(inp, T, R)
    return oracle.pair_energies(inp, Tn), hist


@pytest.mark.parametrize("precision", ["bf16x2", "fp16x2"])
def test_mixed_refinement_matches_converged_oracle(precision):
    prob = build_problem("chain", n_occ=20, band=5, somos=(6, 13))
    e_ref, hist = _converged_oracle(prob)
    plan, dev = device_problem(prob, precision=precision, T_random=False)
    T = dev["T"]
    R, e_pair, e_tot, rmax = plan.solve_mixed(3, 12, T)
    ep = e_pair.cpu().numpy().reshape(-1, 4)
    worst = max(abs(ep[p, CODE[n]] - v) for (p, n), v in e_ref.items())
    tot_err = abs(float(e_tot.cpu()[0]) - sum(e_ref.values()))
    E, Rm = plan.history()
    print(precision, "outer history E", E, "max|R|", Rm, "worst pair %.2e total %.2e" % (worst, tot_err))
    assert worst <= 1e-7
    assert tot_err <= 1e-6
    plan.close()


def test_mixed_c160_vs_fp64():
    """Precision study at the C160H322-shaped size: BF16x2 inner iterations with
    3 FP64 refinements against the converged FP64 GPU solution."""
    prob = build_problem("c160")
    plan, dev = device_problem(prob, precision="fp64", T_random=False)
    T64 = dev["T"]
    plan.iterate(25, T64)
    _, e64, et64, r64 = plan.iterate(1, T64)
    E64, R64 = plan.history()
    print("fp64 history", E64[-5:], R64[-5:])
    e64 = e64.cpu().numpy()
    et64 = float(et64.cpu()[0])
    plan.close()
    from paper_2008_03237_amd import Plan
    mp = Plan(prob, dev["B"], dev["S"], dev["K"], plan._dev[3], plan._dev[4], precision="bf16x2")
    Tm = torch.zeros_like(T64)
    _, em, etm, rm = mp.solve_mixed(3, 12, Tm)
    em = em.cpu().numpy()
    d_pair = np.max(np.abs(em.reshape(-1, 4).sum(1) - e64.reshape(-1, 4).sum(1)))
    d_tot = abs(float(etm.cpu()[0]) - et64)
    print("E fp64 %.10f mixed %.10f  max pair err %.3e total err %.3e" % (et64, float(etm.cpu()[0]), d_pair, d_tot))
    assert d_pair <= 1e-7
    assert d_tot <= 1e-6
    mp.close()
