"""PNO construction on the GPU (dlpno_pno_build through the C ABI) against
the FP64 oracle (oracle.pno) on the same seeded inputs.

Tolerances (both sides are backward-stable FP64 eigensolvers, u = 2^-53):
  occupations   |d lambda| <= 64 u ||D||                     (Weyl)
  PNO subspace  sin(angle) <= 64 u ||D|| / g, g = lambda_n - lambda_{n+1}
  eps           |d eps| <= 64 u ||F|| (1 + ||D|| / g)
  C             |d C| <= 64 u (||D|| / g + ||F|| / h) + 1e-14, h = the
                smallest gap between kept orbital energies
The number kept must be identical; every workload asserts that no
occupation lies within a relative 1e-9 of T_CutPNO, so that rounding cannot
decide it."""
import numpy as np
import pytest

from oracle.pno import build_pnos, pair_density
from workload.pno import build_pno_problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
U = 2.0 ** -53


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def run_gpu(prob, t_cut=None):
    from paper_2008_03237_amd import PnoPlan
    from workload.gpu import device_pno_fields
    dev = device_pno_fields(prob)
    plan = PnoPlan(prob.pairs, prob.n_X, prob.n_F, prob.n_C, prob.n_v)
    occ, eps, C, nk, sw = plan.build(dev["X"], dev["F"], prob.t_cut if t_cut is None else t_cut, want_sweeps=True)
    torch.cuda.synchronize()
    plan.close()
    return occ.cpu().numpy(), eps.cpu().numpy(), C.cpu().numpy(), nk.cpu().numpy(), sw.cpu().numpy()


def oracle_pair(prob, p, t_cut):
    blocks, F = prob.pair_inputs(p)
    N = int(prob.pairs[p]["dim"])
    D = pair_density(blocks, bool(prob.pairs[p]["diagonal"])) if blocks else np.zeros((N, N))
    occ, n, C, eps = build_pnos(D, F, t_cut)
    return D, F, occ, n, C, eps


def check_pair(prob, p, got, t_cut, guard=True):
    occ_g, eps_g, C_g, nk_g, _ = got
    d = prob.pairs[p]
    N, ov, oc = int(d["dim"]), int(d["off_v"]), int(d["off_C"])
    D, F, occ, n, C, eps = oracle_pair(prob, p, t_cut)
    nD, nF = max(np.abs(occ).max(), 1e-300), np.linalg.norm(F, 2)
    if guard and t_cut > 0:
        assert np.all(np.abs(occ / t_cut - 1.0) > 1e-9), (p, "occupation at the threshold")
    assert nk_g[p] == n, (p, nk_g[p], n)
    np.testing.assert_allclose(occ_g[ov:ov + N], occ, rtol=0, atol=64 * U * nD, err_msg="occ pair %d" % p)
    Cg = C_g[oc:oc + N * N].reshape(N, N)
    assert np.all(Cg[:, n:] == 0.0) and np.all(eps_g[ov + n:ov + N] == 0.0)
    if n == 0:
        return
    g = occ[n - 1] - (occ[n] if n < N else 0.0)
    h = np.min(np.diff(eps)) if n > 1 else 1.0
    tol_e = 64 * U * nF * (1.0 + nD / g)
    np.testing.assert_allclose(eps_g[ov:ov + n], eps, rtol=0, atol=tol_e, err_msg="eps pair %d" % p)
    tol_c = 64 * U * (nD / g + nF / h) + 1e-14
    Ck = Cg[:, :n]
    for k in range(n):
        a = np.sort(np.abs(C[:, k]))[::-1]
        if N > 1 and a[0] - a[1] <= 2 * tol_c:   # near tie: either sign is the convention
            assert min(np.abs(Ck[:, k] - C[:, k]).max(), np.abs(Ck[:, k] + C[:, k]).max()) <= tol_c, (p, k)
        else:
            assert np.abs(Ck[:, k] - C[:, k]).max() <= tol_c, (p, k, np.abs(Ck[:, k] - C[:, k]).max(), tol_c)
    np.testing.assert_allclose(Ck.T @ Ck, np.eye(n), atol=1e-13)
    np.testing.assert_allclose(Ck.T @ F @ Ck, np.diag(eps_g[ov:ov + n]), atol=1e-12 * nF)


def test_pno_generator_bitwise_on_device():
    from workload.gpu import device_pno_fields
    prob = build_pno_problem("tiny")
    dev = device_pno_fields(prob)
    for f in ("X", "F"):
        host = prob.materialize(f)
        assert np.array_equal(dev[f].cpu().numpy()[:host.size], host), f


@pytest.mark.parametrize("name", ["tiny", "chain"])
def test_pno_parity_every_pair(name):
    prob = build_pno_problem(name)
    print("case pno", name, prob.n_pairs, "pairs", flush=True)
    got = run_gpu(prob)
    sw = got[4].reshape(-1, 2)
    assert np.all(got[3] >= 0) and np.all((sw[:, 0] >= 1) & (sw[:, 0] <= 40))
    print("density sweeps max %d mean %.2f; kept mean %.1f" % (sw[:, 0].max(), sw[:, 0].mean(), got[3].mean()))
    for p in range(prob.n_pairs):
        check_pair(prob, p, got, prob.t_cut)


def test_pno_full_size_sampled():
    prob = build_pno_problem("c160")
    print("case pno c160", prob.n_pairs, "pairs", flush=True)
    got = run_gpu(prob)
    assert np.all(got[3] >= 0)
    rng = np.random.default_rng(5)
    sample = np.unique(np.concatenate([[0, prob.n_pairs - 1], rng.choice(prob.n_pairs, 200, replace=False),
                                       np.nonzero(prob.pairs["dim"] == 64)[0][:20]]))
    for p in sample:
        check_pair(prob, int(p), got, prob.t_cut)


@pytest.mark.parametrize("dom", [("fixed", 1), ("fixed", 2), ("fixed", 63), ("fixed", 64)])
def test_pno_domain_edges(dom):
    prob = build_pno_problem("tiny", dom=dom)
    got = run_gpu(prob)
    for p in range(prob.n_pairs):
        check_pair(prob, p, got, prob.t_cut)


def test_pno_keep_all_and_keep_none():
    prob = build_pno_problem("tiny")
    got = run_gpu(prob, t_cut=-1.0)           # every occupation kept: n = N
    assert np.array_equal(got[3], prob.pairs["dim"])
    for p in range(0, prob.n_pairs, 3):
        check_pair(prob, p, got, -1.0, guard=False)
    got = run_gpu(prob, t_cut=1.0)            # none kept: every pair's C block is zero
    assert np.all(got[3] == 0)
    for d in prob.pairs:                      # (the alignment gaps between blocks are never written)
        assert np.all(got[2][d["off_C"]:d["off_C"] + d["dim"] ** 2] == 0.0)
    for p in range(0, prob.n_pairs, 5):
        check_pair(prob, p, got, 1.0)


def test_pno_pairs_without_amplitudes():
    # a SOMO's diagonal pair stores no spin block: its density is zero
    prob = build_pno_problem("tiny")
    empty = np.nonzero(prob.pairs["blocks"] == 0)[0]
    assert len(empty) == 2
    got = run_gpu(prob)
    for p in empty:
        d = prob.pairs[p]
        assert got[3][p] == 0
        assert np.all(got[0][d["off_v"]:d["off_v"] + d["dim"]] == 0.0)


def test_pno_nonfinite_input_reported():
    from paper_2008_03237_amd import PnoPlan
    from workload.gpu import device_pno_fields
    prob = build_pno_problem("tiny")
    dev = device_pno_fields(prob)
    p = int(np.nonzero(prob.pairs["blocks"] != 0)[0][7])
    dev["X"][int(prob.pairs[p]["off_X"])] = float("nan")
    plan = PnoPlan(prob.pairs, prob.n_X, prob.n_F, prob.n_C, prob.n_v)
    _, _, _, nk, _ = plan.build(dev["X"], dev["F"], prob.t_cut)
    nk = nk.cpu().numpy()
    assert nk[p] == -3 and np.all(np.delete(nk, p) >= 0)
    plan.close()


def oracle_overlaps(prob_pno, res):
    """S of every coupling of the residual workload `res` from the oracle's
    own PNOs; also returns the per-pair coefficient tolerances."""
    from oracle.pno import pno_overlap
    Cs, tol = [], []
    for p in range(prob_pno.n_pairs):
        D, F, occ, n, C, eps = oracle_pair(prob_pno, p, prob_pno.t_cut)
        N = C.shape[0]
        if n == 0:
            C = np.zeros((N, 1))
            tol.append(0.0)
        else:
            g = occ[n - 1] - (occ[n] if n < N else 0.0)
            h = np.min(np.diff(eps)) if n > 1 else 1.0
            tol.append(64 * U * (max(occ[0], 1e-300) / g + np.linalg.norm(F, 2) / h) + 1e-14)
        Cs.append(C)
    S = np.zeros(res.n_S)
    first = prob_pno.pairs["first"]
    for p in range(res.n_pairs):
        for e in range(res.cpl_rowptr[p], res.cpl_rowptr[p + 1]):
            q = int(res.cpl_src[e])
            blk = pno_overlap(Cs[p], int(first[p]), Cs[q], int(first[q]))
            S[res.cpl_off_S[e]:res.cpl_off_S[e] + blk.size] = blk.ravel()
    return S, np.array(tol)


def gpu_pipeline(name):
    """PNOs on the GPU, then the residual workload with n_p = the PNO counts
    and the S blocks of its coupling list from dlpno_pno_overlap."""
    from paper_2008_03237_amd import PnoPlan
    from workload import build_problem
    from workload.gpu import device_pno_fields
    pp = build_pno_problem(name)
    dev = device_pno_fields(pp)
    plan = PnoPlan(pp.pairs, pp.n_X, pp.n_F, pp.n_C, pp.n_v)
    occ, eps, C, nk, _ = plan.build(dev["X"], dev["F"], pp.t_cut)
    nk_h = nk.cpu().numpy()
    res = build_problem(name, npno=("given", np.maximum(nk_h, 1)))
    plan.overlap_prepare(nk_h, res.cpl_rowptr, res.cpl_src, res.cpl_off_S, res.n_S)
    S = plan.overlap(C)
    torch.cuda.synchronize()
    plan.close()
    return pp, res, nk_h, S


@pytest.mark.parametrize("name", ["tiny", "chain"])
def test_pno_overlap_parity(name):
    pp, res, nk, S = gpu_pipeline(name)
    print("case pno overlap", name, int(res.cpl_rowptr[-1]), "couplings", flush=True)
    S_o, tol = oracle_overlaps(pp, res)
    S_g = S.cpu().numpy()[:res.n_S]
    for p in range(res.n_pairs):
        for e in range(res.cpl_rowptr[p], res.cpl_rowptr[p + 1]):
            q = int(res.cpl_src[e])
            o, size = int(res.cpl_off_S[e]), int(res.npno[p] * res.npno[q])
            d = np.abs(S_g[o:o + size] - S_o[o:o + size]).max()
            assert d <= 8.0 * (tol[p] + tol[q]) + 1e-13, (p, q, d)


def test_residual_on_pno_built_inputs():
    """The hot path on inputs produced by the PNO stage: n_p and S from the GPU
    PNO build, against the oracle residual with n_p and S from the oracle's PNO
    build.  S inherits the PNOs' subspace error (1e-10 at worst here), hence the
    looser 1e-8 bound on R."""
    import oracle
    from oracle.model import unpack_T
    from paper_2008_03237_amd import Plan
    from tests.gpu_helpers import compare_blocks
    from workload.gpu import device_fields
    pp, res, nk, S = gpu_pipeline("tiny")
    res.S_host, _ = oracle_overlaps(pp, res)
    dev = device_fields(res, fields=("B", "K", "T"))
    plan = Plan(res, dev["B"], S, dev["K"], torch.from_numpy(res.eps_a).cuda(), torch.from_numpy(res.eps_b).cuda())
    R = plan.residual(dev["T"])
    torch.cuda.synchronize()
    inp = oracle.Inputs.from_problem(res, B=res.materialize("B"), K=res.materialize("K"), S=res.materialize("S"))
    Ro = oracle.residual_os(inp, unpack_T(res, res.materialize("T")))
    compare_blocks(res, R.cpu().numpy(), Ro, rel=1e-8)
    plan.close()
