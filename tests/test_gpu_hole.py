"""Hole-hole ladder (first slice of the remaining CCSD terms) on the GPU against
the FP64 oracle, through the C ABI: the term
    sum_{k in occ_s, l in occ_s'} (k i | l j) S_{ij,kl} T^{ss'}_{(k,l)} S_{kl,ij}
runs as extra couplings of the projection launches."""
import numpy as np
import pytest

import oracle
from oracle.model import unpack_T
from tests.gpu_helpers import compare_blocks, device_problem, oracle_inputs
from workload import build_problem
from workload.problem import segment_values

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CODE = {"AA": 0, "BB": 1, "AB": 2, "BA": 3}


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _mini(**kw):
    return build_problem("chain", n_occ=24, band=6, somos=(7, 16), hole_ladder=0.02, **kw)


@pytest.mark.parametrize("cfg", ["tiny", "mini", "mini_spin"])
def test_residual_update_energy_parity_with_hole_ladder(cfg):
    if cfg == "tiny":
        prob = build_problem("tiny", hole_ladder=0.02)
    else:
        prob = _mini(fock_spin=0.3 if cfg == "mini_spin" else 0.0)
    print("case", cfg, prob.n_pairs, "pairs", prob.n_couplings, "Fock couplings", prob.n_hh, "hole-hole", flush=True)
    assert prob.n_hh > 0
    plan, dev = device_problem(prob)
    R = plan.residual(dev["T"])
    Tn, e_pair, e_tot = plan.update(dev["T"], R)
    torch.cuda.synchronize()
    inp = oracle_inputs(prob)
    T = unpack_T(prob, prob.materialize("T"))
    Ro = oracle.residual_os(inp, T)
    # the hole-hole part is not negligible against the tolerance
    Rh = oracle.residual_os(inp, T, terms=("hole",))
    assert max(float(np.max(np.abs(v))) for v in Rh.values()) > 1e-6 * max(float(np.max(np.abs(v))) for v in Ro.values())
    Tno = oracle.jacobi(inp, T, Ro)
    eo = oracle.pair_energies(inp, Tno)
    compare_blocks(prob, R.cpu().numpy(), Ro, rel=1e-12)
    compare_blocks(prob, Tn.cpu().numpy(), Tno, rel=1e-12)
    ep = e_pair.cpu().numpy().reshape(-1, 4)
    for (p, name), v in eo.items():
        assert abs(ep[p, CODE[name]] - v) <= 1e-10, (p, name)
    assert abs(float(e_tot.cpu()[0]) - sum(eo.values())) <= 1e-10
    plan.close()


def test_flop_count_includes_hole_hole_terms():
    prob = _mini()
    plan, dev = device_problem(prob)
    inp = oracle_inputs(prob)
    T = unpack_T(prob, prob.materialize("T"))
    proj = 0.0
    for p in range(prob.n_pairs):
        n = int(prob.npno[p])
        for name in inp.blocks(p):
            for (w, q, S, src) in oracle.model.projection_terms(inp, T, p, name) + oracle.hole_terms(inp, T, p, name):
                nq = int(prob.npno[q])
                proj += 2.0 * n * nq * (n + nq)
    assert plan.flop_count()[1] == proj
    plan.close()


def test_iterations_with_hole_ladder_match_oracle():
    prob = build_problem("chain", n_occ=20, band=5, somos=(6, 13), hole_ladder=0.02)
    plan, dev = device_problem(prob, T_random=False)
    n_it = 10
    plan.iterate(n_it, dev["T"])
    E_gpu, _ = plan.history()
    inp = oracle_inputs(prob)
    zero = unpack_T(prob, np.zeros(prob.n_T))
    To, hist = oracle.solve(inp, zero, n_it, use_diis=True)
    for k in range(n_it):
        assert abs(E_gpu[k] - hist[k][0]) <= 1e-10, (k, E_gpu[k], hist[k][0])
    compare_blocks(prob, dev["T"].cpu().numpy(), To, rel=1e-9)
    plan.close()


@pytest.mark.parametrize("precision,rel", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_vjp_with_hole_ladder_matches_oracle(precision, rel):
    """The hole-hole operator is self-adjoint for real integrals, (k i | l j) =
    (i k | j l), so the VJP's gather over reverse couplings covers it."""
    prob = build_problem("chain", n_occ=16, band=4, somos=(5, 11), hole_ladder=0.02)
    plan, dev = device_problem(prob, precision=precision)
    rng = np.random.default_rng(8)
    G = torch.from_numpy(rng.standard_normal(prob.n_T)).cuda()
    dT, _ = plan.vjp(dev["T"], G, want_dB=False)
    torch.cuda.synchronize()
    inp = oracle_inputs(prob)
    T = unpack_T(prob, prob.materialize("T"))
    dTo, _ = oracle.vjp(inp, T, unpack_T(prob, G.cpu().numpy()))
    compare_blocks(prob, dT.cpu().numpy(), dTo, rel=rel)
    plan.close()


@pytest.mark.parametrize("precision,tol", [("bf16x2", (3.5e-5, 5e-5)), ("fp16x2", (3.5e-6, 6e-6))])
def test_split_precision_with_hole_ladder_per_block(precision, tol):
    prob = _mini()
    plan, dev = device_problem(prob, precision=precision)
    R = plan.residual(dev["T"])
    torch.cuda.synchronize()
    inp = oracle_inputs(prob)
    T = unpack_T(prob, prob.materialize("T"))
    Ro = oracle.residual_os(inp, T)
    C = oracle.residual_os(inp, T, terms=("ladder", "projection", "hole"))
    Rg = unpack_T(prob, R.cpu().numpy())
    ef = max(float(np.linalg.norm(Rg[k] - Ro[k]) / np.linalg.norm(C[k])) for k in Ro)
    em = max(float(np.max(np.abs(Rg[k] - Ro[k])) / np.max(np.abs(C[k]))) for k in Ro)
    print(precision, "with hole-hole ladder: worst block Frobenius %.3e, max-abs %.3e" % (ef, em))
    assert ef <= tol[0] and em <= tol[1]
    plan.close()


def test_full_chain_sampled_with_hole_ladder():
    prob = build_problem("chain", hole_ladder=0.02)
    print("case chain with hole-hole ladder:", prob.n_pairs, "pairs", prob.n_hh, "hole-hole couplings", flush=True)
    plan, dev = device_problem(prob)
    R = plan.residual(dev["T"])
    torch.cuda.synchronize()
    rng = np.random.default_rng(77)
    n = prob.npno
    pick = sorted(set(rng.choice(prob.n_pairs, 10, replace=False).tolist()))
    inp = oracle_inputs(prob, full=False)
    need = set(pick)
    for p in pick:
        need.update(prob.cpl_src[prob.cpl_rowptr[p]:prob.cpl_rowptr[p + 1]].tolist())
        need.update(prob.hh_src[prob.hh_rowptr[p]:prob.hh_rowptr[p + 1]].tolist())
    T = {}
    for p in need:
        o = int(prob.off_T[p])
        for name in oracle.stored_blocks(int(prob.pi[p]), int(prob.pj[p]), prob.is_somo.astype(bool)):
            seg = prob.segs["T"][np.searchsorted(prob.segs["T"]["off"], o)]
            T[(p, name)] = segment_values(prob.seed, seg).reshape(n[p], n[p])
            o += int(n[p]) ** 2
    Ro = oracle.residual_os(inp, T, pairs=pick)
    Rg = R.cpu().numpy()
    for (p, name), ref in Ro.items():
        i = oracle.stored_blocks(int(prob.pi[p]), int(prob.pj[p]), prob.is_somo.astype(bool)).index(name)
        o = int(prob.off_T[p]) + i * int(n[p]) ** 2
        got = Rg[o:o + int(n[p]) ** 2].reshape(n[p], n[p])
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref), (p, name)
    plan.close()
