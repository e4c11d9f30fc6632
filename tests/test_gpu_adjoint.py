"""Adjoint kernels and the autograd Function vs the FP64 oracle and finite differences."""
import numpy as np
import pytest

import oracle
from oracle.model import unpack_T
from tests.gpu_helpers import antisymmetrize_same_spin, compare_blocks, device_problem, oracle_inputs
from workload import build_problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _flatB(prob, dB):
    out = np.zeros(prob.n_B)
    for p, v in dB.items():
        o = int(prob.off_B[p])
        out[o:o + v.size] = v.ravel()
    return out


@pytest.mark.parametrize("precision,rel", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_vjp_matches_oracle(precision, rel):
    prob = build_problem("chain", n_occ=20, band=5, somos=(6, 13))
    plan, dev = device_problem(prob, precision=precision)
    rng = np.random.default_rng(5)
    G = torch.from_numpy(rng.standard_normal(prob.n_T)).cuda()
    dT, dB = plan.vjp(dev["T"], G)
    torch.cuda.synchronize()
    inp = oracle_inputs(prob)
    T = unpack_T(prob, prob.materialize("T"))
    Gd = unpack_T(prob, G.cpu().numpy())
    dTo, dBo = oracle.vjp(inp, T, Gd)
    compare_blocks(prob, dT.cpu().numpy(), dTo, rel=rel)
    got = dB.cpu().numpy()
    want = _flatB(prob, dBo)
    for p in range(prob.n_pairs):
        o, sz = int(prob.off_B[p]), int(prob.naux[p] * prob.npno[p] ** 2)
        d = np.linalg.norm(got[o:o + sz] - want[o:o + sz])
        assert d <= rel * max(np.linalg.norm(want[o:o + sz]), 1e-300) + 1e-300, (p, d)
    plan.close()


def test_fp32_residual_close_to_fp64_oracle():
    prob = build_problem("chain", n_occ=24, band=6, somos=(7, 16))
    plan, dev = device_problem(prob, precision="fp32")
    R = plan.residual(dev["T"])
    torch.cuda.synchronize()
    inp = oracle_inputs(prob)
    Ro = oracle.residual_os(inp, unpack_T(prob, prob.materialize("T")))
    compare_blocks(prob, R.cpu().numpy(), Ro, rel=2e-5)
    plan.close()


@pytest.mark.parametrize("general", [False, True])
def test_dot_product_identity_on_device(general):
    # <G, J dT> = <J^T G, dT> with J the residual's linear part (FP64, mini
    # chain).  Default plans take antisymmetric same-spin blocks (dT in that
    # space, G general); general_T plans take any dT.
    from paper_2008_03237_amd import Plan
    prob = build_problem("chain", n_occ=24, band=6, somos=(7, 16))
    plan0, dev = device_problem(prob)
    plan = Plan(prob, dev["B"], dev["S"], dev["K"], plan0._dev[3], plan0._dev[4], general_T=general)
    plan0.close()
    rng = np.random.default_rng(8)
    G = torch.from_numpy(rng.standard_normal(prob.n_T)).cuda()
    X = torch.from_numpy(rng.standard_normal(prob.n_T)).cuda()
    if not general:
        X = antisymmetrize_same_spin(prob, X)
    zero = torch.zeros_like(X)
    # only elements of stored blocks: the alignment gaps between pairs are never written
    mask = torch.zeros(prob.n_T, dtype=torch.float64, device="cuda")
    for p in range(prob.n_pairs):
        o = int(prob.off_T[p])
        mask[o:o + int(prob.n_blocks()[p]) * int(prob.npno[p]) ** 2] = 1.0
    G, X = G * mask, X * mask
    JX = (plan.residual(X) - plan.residual(zero)) * mask
    JtG, _ = plan.vjp(X, G, want_dB=False)
    a = float(torch.dot(G, JX))
    b = float(torch.dot(JtG * mask, X))
    assert abs(a - b) <= 1e-11 * abs(a)
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_autograd_lagrangian_central_differences_50_pairs(precision):
    """Config of the differentiation study: chain sizes; directional central
    differences (h = 1e-5, FP64 residuals) on 50 random pairs for T and B."""
    from paper_2008_03237_amd import Plan
    from paper_2008_03237_amd.autograd import residual
    prob = build_problem("chain")
    plan, dev = device_problem(prob, precision=precision)
    rng = np.random.default_rng(2024)
    pick = rng.choice(prob.n_pairs, 50, replace=False)
    Lam = torch.from_numpy(rng.standard_normal(prob.n_T) * 1e-2).cuda()
    T = dev["T"].clone().requires_grad_(True)
    B = dev["B"]
    B.requires_grad_(True)
    # L = E(T) + <Lambda, R(T, B)> with the pair energy functional of the
    # amplitudes E(T) = sum_blocks w <K^{ss'}, T> (w = 1/2 same spin, 1
    # opposite spin), evaluated here with torch from the driver integrals
    Kflat = prob.materialize("K")
    Kw = np.zeros(prob.n_T)
    for p in range(prob.n_pairs):
        n, o = int(prob.npno[p]), int(prob.off_T[p])
        Kp = Kflat[int(prob.off_K[p]):int(prob.off_K[p]) + n * n].reshape(n, n)
        for name in prob.block_list(p):
            Kw[o:o + n * n] = (0.5 * (Kp - Kp.T) if name in ("AA", "BB") else Kp).ravel()
            o += n * n
    Kw = torch.from_numpy(Kw).cuda()
    R = residual(T, B, plan)
    L = torch.dot(Kw, T) + torch.dot(Lam, R)
    L.backward()
    gT, gB = T.grad.detach(), B.grad.detach()
    B.requires_grad_(False)
    # directions supported on the picked pairs
    dTdir = torch.zeros(prob.n_T, dtype=torch.float64, device="cuda")
    dBdir = torch.zeros_like(dev["B"])
    nblk = prob.n_blocks()
    for p in pick:
        o, nb = int(prob.off_T[p]), int(nblk[p])
        sz = nb * int(prob.npno[p]) ** 2
        dTdir[o:o + sz] = torch.from_numpy(rng.standard_normal(sz)).cuda()
    antisymmetrize_same_spin(prob, dTdir)            # a direction in the amplitude space
    for p in pick:
        m, n = int(prob.naux[p]), int(prob.npno[p])
        o, sz = int(prob.off_B[p]), m * n * n
        d = rng.standard_normal((m, n, n))
        d = (d + d.transpose(0, 2, 1)) / 2          # B^Q stays symmetric, as the library requires
        dBdir[o:o + sz] = torch.from_numpy(d.ravel()).cuda()
    h = 1e-5
    fp = Plan(prob, dev["B"], dev["S"], dev["K"], plan._dev[3], plan._dev[4])   # FP64 residuals for the differences

    def Lof(Tx):
        return float(torch.dot(Kw, Tx)) + float(torch.dot(Lam, fp.residual(Tx)))
    with torch.no_grad():
        fd_T = (Lof(dev["T"] + h * dTdir) - Lof(dev["T"] - h * dTdir)) / (2 * h)
        an_T = float(torch.dot(gT, dTdir))
        Bp = dev["B"] + h * dBdir
        Bm = dev["B"] - h * dBdir
        pp = Plan(prob, Bp, dev["S"], dev["K"], plan._dev[3], plan._dev[4])
        pm = Plan(prob, Bm, dev["S"], dev["K"], plan._dev[3], plan._dev[4])
        fd_B = (float(torch.dot(Lam, pp.residual(dev["T"]))) - float(torch.dot(Lam, pm.residual(dev["T"])))) / (2 * h)
        an_B = float(torch.dot(gB, dBdir))
    tol = 1e-7 if precision == "fp64" else 1e-4
    print(precision, "dT: fd %.12e an %.12e   dB: fd %.12e an %.12e" % (fd_T, an_T, fd_B, an_B))
    assert abs(fd_T - an_T) <= tol * abs(an_T)
    assert abs(fd_B - an_B) <= tol * abs(an_B)
    for x in (pp, pm, fp, plan):
        x.close()


def test_vjp_refuses_data_without_the_adjoint_symmetries():
    """The VJP evaluates the transposed residual with the forward kernels, which
    needs symmetric occupied Fock matrices and transposed overlap blocks on
    reverse couplings.  Data without them: the forward residual still runs,
    the product is refused (DLPNO_ERR_UNSUPPORTED) instead of being silently
    wrong; the same data made consistent again is accepted."""
    from paper_2008_03237_amd import DlpnoError, Plan
    prob = build_problem("chain", n_occ=12, band=3, somos=(4, 8), npno=("fixed", 10), naux=("fixed", 30))
    plan, dev = device_problem(prob)
    G = torch.ones_like(dev["T"])
    plan.vjp(dev["T"], G)                                  # consistent data: accepted
    plan.close()
    # a non-symmetric beta Fock matrix
    fb = prob.f_b.copy()
    fb[2, 3] += 1e-3
    prob_f = build_problem("chain", n_occ=12, band=3, somos=(4, 8), npno=("fixed", 10), naux=("fixed", 30))
    prob_f.f_b = fb
    eps_a, eps_b = torch.from_numpy(prob.eps_a).cuda(), torch.from_numpy(prob.eps_b).cuda()
    pf = Plan(prob_f, dev["B"], dev["S"], dev["K"], eps_a, eps_b)
    pf.residual(dev["T"])
    with pytest.raises(DlpnoError) as ei:
        pf.vjp(dev["T"], G)
    assert ei.value.status == -8 and "symmetric" in str(ei.value)
    pf.close()
    # one overlap block that is no longer the transpose of its reverse
    e = int(prob.cpl_rowptr[7])
    S2 = dev["S"].clone()
    S2[int(prob.cpl_off_S[e]) + 3] += 1e-6
    ps = Plan(prob, dev["B"], S2, dev["K"], eps_a, eps_b)
    ps.residual(dev["T"])
    with pytest.raises(DlpnoError) as ei:
        ps.vjp(dev["T"], G)
    assert ei.value.status == -8 and "transpose" in str(ei.value)
    with pytest.raises(DlpnoError):                       # the verdict is kept
        ps.vjp(dev["T"], G)
    ps.close()
