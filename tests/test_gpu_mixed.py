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


def _per_block_contraction_error(prob, Rg_flat, Tflat):
    """Worst per-block error of the residual relative to that block's contracted
    part (ladder + projection): Frobenius and max-abs."""
    inp = oracle_inputs(prob)
    T = unpack_T(prob, Tflat)
    Ro = oracle.residual_os(inp, T)
    C = oracle.residual_os(inp, T, terms=("ladder", "projection"))
    Rg = unpack_T(prob, Rg_flat)
    worst_f = worst_m = 0.0
    where = None
    for k in Ro:
        d = Rg[k] - Ro[k]
        ef = float(np.linalg.norm(d)) / float(np.linalg.norm(C[k]))
        em = float(np.max(np.abs(d))) / float(np.max(np.abs(C[k])))
        if ef > worst_f:
            worst_f, where = ef, k
        worst_m = max(worst_m, em)
    return worst_f, worst_m, where


# per block, about 5x the worst errors measured on the device (Frobenius,
# max-abs): BF16x2 7.0e-6, 1.0e-5; FP16x2 6.6e-7, 1.2e-6; FP32 7.2e-7, 1.5e-6
TOL = {"bf16x2": (3.5e-5, 5e-5), "fp16x2": (3.5e-6, 6e-6), "fp32": (3.5e-6, 7.5e-6)}


@pytest.mark.parametrize("precision", ["bf16x2", "fp16x2", "fp32"])
def test_split_residual_accuracy_per_block(precision):
    """Every block of the mini chain (all four tile classes, every spin-block
    class) within tol of the oracle, relative to the block's own ladder +
    projection part: an error confined to one tile class or spin block is not
    averaged away."""
    prob = build_problem("chain", n_occ=24, band=6, somos=(7, 16))
    plan, dev = device_problem(prob, precision=precision)
    R = plan.residual(dev["T"])
    torch.cuda.synchronize()
    ef, em, where = _per_block_contraction_error(prob, R.cpu().numpy(), prob.materialize("T"))
    print(precision, "worst block: Frobenius %.3e (block %s), max-abs %.3e" % (ef, where, em))
    assert ef <= TOL[precision][0] and em <= TOL[precision][1]
    plan.close()


@pytest.mark.parametrize("precision", ["bf16x2", "fp16x2"])
def test_split_accuracy_with_block_magnitudes_over_six_decades(precision):
    """Amplitude blocks scaled by 1, 1e-2, 1e-4 and 1e-6 pair by pair: the FP16
    power-of-two scales of neighbouring blocks then differ by up to 2^20, which
    the projection's stage-1 products must absorb without overflow or loss of
    their low halves.  Per-block errors as in the test above."""
    prob = build_problem("chain", n_occ=24, band=6, somos=(7, 16))
    plan, dev = device_problem(prob, precision=precision)
    Th = prob.materialize("T")
    for p in range(prob.n_pairs):
        o = int(prob.off_T[p])
        size = int(prob.n_blocks()[p]) * int(prob.npno[p]) ** 2
        Th[o:o + size] *= 10.0 ** (-2 * (p % 4))
    R = plan.residual(torch.from_numpy(Th).cuda())
    torch.cuda.synchronize()
    assert torch.isfinite(R).all()
    ef, em, where = _per_block_contraction_error(prob, R.cpu().numpy(), Th)
    print(precision, "six decades, worst block: Frobenius %.3e (block %s), max-abs %.3e" % (ef, where, em))
    assert ef <= TOL[precision][0] and em <= TOL[precision][1]
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


def test_mixed_and_fp32_c160_vs_fp64():
    """Precision study at the C160H322-shaped size (18,901 pairs): BF16x2 and
    FP16x2 inner iterations with 3 FP64 refinements, each within 1e-7 Eh per
    pair and 1e-6 Eh in total of the converged FP64 GPU solution; and the plain
    FP32 path iterated until max|R| stalls, whose error is reported."""
    prob = build_problem("c160")
    plan, dev = device_problem(prob, precision="fp64", T_random=False)
    T64 = dev["T"]
    _, _, _, _, n64 = plan.solve(40, T64, tol_r=1e-11, tol_e=1e-12)
    _, e64, et64, r64 = plan.iterate(1, T64)
    print("fp64 converged in", n64, "iterations, max|R| %.2e" % float(r64.cpu()[0]), flush=True)
    e64 = e64.cpu().numpy().reshape(-1, 4).sum(1)
    et64 = float(et64.cpu()[0])
    eps_a, eps_b = plan._dev[3], plan._dev[4]
    plan.close()
    from paper_2008_03237_amd import Plan
    for precision in ("bf16x2", "fp16x2"):
        mp = Plan(prob, dev["B"], dev["S"], dev["K"], eps_a, eps_b, precision=precision)
        Tm = torch.zeros_like(T64)
        _, em, etm, rm = mp.solve_mixed(3, 4, Tm)
        d_pair = np.max(np.abs(em.cpu().numpy().reshape(-1, 4).sum(1) - e64))
        d_tot = abs(float(etm.cpu()[0]) - et64)
        print("%s: E fp64 %.10f mixed %.10f  max pair err %.3e total err %.3e max|R| %.2e" % (
            precision, et64, float(etm.cpu()[0]), d_pair, d_tot, float(rm.cpu()[0])), flush=True)
        assert d_pair <= 1e-7
        assert d_tot <= 1e-6
        mp.close()
        del Tm
    p32 = Plan(prob, dev["B"], dev["S"], dev["K"], eps_a, eps_b, precision="fp32")
    T32 = torch.zeros_like(T64)
    best = None
    for _ in range(20):
        _, e32, et32, r32 = p32.iterate(2, T32)
        r = float(r32.cpu()[0])
        if best is not None and r >= 0.5 * best:
            break
        best = r if best is None else min(best, r)
    d_pair = np.max(np.abs(e32.cpu().numpy().reshape(-1, 4).sum(1) - e64))
    d_tot = abs(float(et32.cpu()[0]) - et64)
    print("fp32: stalls at max|R| %.2e; max pair err %.3e total err %.3e" % (r, d_pair, d_tot), flush=True)
    # FP32 contractions (24-bit operands) without refinement: the same energy gate
    assert d_pair <= 1e-7 and d_tot <= 1e-6
    p32.close()
