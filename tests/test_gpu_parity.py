"""FP64 GPU path vs the FP64 CPU oracle (through the C ABI)."""
import numpy as np
import pytest

import oracle
from oracle.model import unpack_T, pack_T
from tests.gpu_helpers import device_problem, oracle_inputs, compare_blocks
from workload import build_problem
from workload.problem import segment_values

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _oracle_step(prob, inp, Tflat):
    T = unpack_T(prob, Tflat)
    R = oracle.residual_os(inp, T)
    Tn = oracle.jacobi(inp, T, R)
    e = oracle.pair_energies(inp, Tn)
    return T, R, Tn, e


def test_generator_bitwise_on_device():
    from workload.gpu import device_fields
    prob = build_problem("chain", n_occ=16, band=4, somos=(5, 11))
    dev = device_fields(prob)
    for f in ("B", "K", "T", "S"):
        host = prob.materialize(f)
        got = dev[f][:host.size].cpu().numpy()
        assert np.array_equal(got.view(np.uint64), host.view(np.uint64)), f


@pytest.mark.parametrize("cfg,fock_spin", [("tiny", 0.0), ("mini", 0.0), ("tiny", 0.3), ("mini", 0.3)])
def test_residual_update_energy_parity(cfg, fock_spin):
    """fock_spin > 0: the beta off-diagonal occupied Fock differs from the
    alpha one, so every projection term must take the Fock matrix of the
    replaced electron's spin (a swap changes the residual by ~1e-5 relative)."""
    if cfg == "tiny":
        prob = build_problem("tiny", fock_spin=fock_spin)
    else:
        prob = build_problem("chain", n_occ=24, band=6, somos=(7, 16), fock_spin=fock_spin)
    print("case", cfg, "fock_spin", fock_spin, prob.n_pairs, "pairs", flush=True)
    plan, dev = device_problem(prob)
    R = plan.residual(dev["T"])
    Tn, e_pair, e_tot = plan.update(dev["T"], R)
    torch.cuda.synchronize()
    inp = oracle_inputs(prob)
    T, Ro, Tno, eo = _oracle_step(prob, inp, prob.materialize("T"))
    compare_blocks(prob, R.cpu().numpy(), Ro, rel=1e-12)
    compare_blocks(prob, Tn.cpu().numpy(), Tno, rel=1e-12)
    ep = e_pair.cpu().numpy().reshape(-1, 4)
    code = {"AA": 0, "BB": 1, "AB": 2, "BA": 3}
    for (p, name), v in eo.items():
        assert abs(ep[p, code[name]] - v) <= 1e-10, (p, name)
    assert abs(float(e_tot.cpu()[0]) - sum(eo.values())) <= 1e-10
    plan.close()


@pytest.mark.parametrize("general", [False, True])
def test_general_amplitudes_flag(general):
    """Same-spin blocks are taken antisymmetric by default (only the lower
    tiles of their contributions are computed, the upper ones mirrored);
    with general_T every tile is computed.  Residuals of a random T whose
    same-spin blocks are antisymmetric (default) or not (general_T) vs the
    oracle's plain formula."""
    from paper_2008_03237_amd import Plan
    prob = build_problem("chain", n_occ=24, band=6, somos=(7, 16))
    plan0, dev = device_problem(prob)
    plan = Plan(prob, dev["B"], dev["S"], dev["K"], plan0._dev[3], plan0._dev[4], general_T=general)
    plan0.close()
    rng = np.random.default_rng(31)
    Th = rng.standard_normal(prob.n_T) * 1e-2
    if not general:
        somo = prob.is_somo.astype(bool)
        for p in range(prob.n_pairs):
            n, o = int(prob.npno[p]), int(prob.off_T[p])
            for name in oracle.stored_blocks(int(prob.pi[p]), int(prob.pj[p]), somo):
                if name in ("AA", "BB"):
                    blk = Th[o:o + n * n].reshape(n, n)
                    Th[o:o + n * n] = ((blk - blk.T) / 2).ravel()
                o += n * n
    R = plan.residual(torch.from_numpy(Th).cuda())
    torch.cuda.synchronize()
    inp = oracle_inputs(prob)
    Ro = oracle.residual_os(inp, unpack_T(prob, Th))
    compare_blocks(prob, R.cpu().numpy(), Ro, rel=1e-12)
    plan.close()


def test_tile_classes_all_present_in_mini():
    prob = build_problem("chain", n_occ=24, band=6, somos=(7, 16))
    nt = set(((prob.npno + 15) // 16).tolist())
    assert nt == {1, 2, 3, 4}


def test_determinism_bitwise():
    prob = build_problem("chain", n_occ=24, band=6, somos=(7, 16))
    plan, dev = device_problem(prob)
    # zero-filled outputs: the alignment padding between pairs is never written
    R1 = plan.residual(dev["T"], torch.zeros_like(dev["T"]))
    R2 = plan.residual(dev["T"], torch.zeros_like(dev["T"]))
    torch.cuda.synchronize()
    assert torch.equal(R1.view(torch.int64), R2.view(torch.int64))
    plan.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("bf16x2", 1e-5)])
def test_worker_counts_and_queues(precision, tol):
    # The persistent launches keep one work queue per XCD and start each
    # workgroup on the queue blockIdx % 8; with fewer than eight workgroups, or
    # a count that is not a multiple of eight, some queues are drained only by
    # waves that move on from their own.  The worker count also sets the item
    # size (the Q ranges summed per partial slot), so results agree to rounding
    # only; a lost or repeated item would change them far beyond the tolerance.
    prob = build_problem("chain", n_occ=24, band=6, somos=(7, 16))
    ref = None
    for workers in (0, 1, 3, 13):
        print("case", precision, "workers", workers, flush=True)
        plan, dev = device_problem(prob, precision=precision, n_workers=workers)
        # zero-filled output: the alignment padding between pairs is never written
        R = plan.residual(dev["T"], torch.zeros_like(dev["T"]))
        R2 = plan.residual(dev["T"], torch.zeros_like(dev["T"]))
        torch.cuda.synchronize()
        plan.close()
        assert torch.equal(R.view(torch.int64), R2.view(torch.int64)), workers
        if ref is None:
            ref = R
        else:
            d = float((R - ref).abs().max())
            assert d <= tol * float(ref.abs().max()), (workers, d)


def test_iterations_match_oracle_with_diis():
    prob = build_problem("chain", n_occ=20, band=5, somos=(6, 13))
    plan, dev = device_problem(prob, T_random=False)
    T = dev["T"]
    n_it = 8
    plan.iterate(n_it, T)
    E_gpu, rmax_gpu = plan.history()
    inp = oracle_inputs(prob)
    zero = {k: np.zeros_like(v) for k, v in unpack_T(prob, np.zeros(prob.n_T)).items()}
    To, hist = oracle.solve(inp, zero, n_it, use_diis=True)
    assert len(E_gpu) == n_it
    for k in range(n_it):
        assert abs(E_gpu[k] - hist[k][0]) <= 1e-10, (k, E_gpu[k], hist[k][0])
        assert abs(rmax_gpu[k] - hist[k][1]) <= 1e-12 * max(1.0, hist[k][1]) + 1e-14
    compare_blocks(prob, T.cpu().numpy(), To, rel=1e-10)
    plan.close()


def test_diis_drop_and_coefficients_match_oracle():
    """DIIS in lockstep with the oracle on the 20-orbital chain: stored vector
    counts, drops and extrapolation coefficients after every iteration up to
    the first drop (iteration 7, where the normalised bordered matrix of the
    eight errors has condition number ~2.5e15, 25x over the 1e14 threshold,
    so rounding cannot flip the decision), energies and amplitudes after 12
    iterations (later drop decisions lie within 1% of the threshold and are
    not compared)."""
    prob = build_problem("chain", n_occ=20, band=5, somos=(6, 13))
    plan, dev = device_problem(prob, T_random=False)
    inp = oracle_inputs(prob)
    zero = unpack_T(prob, np.zeros(prob.n_T))
    n_it, n_lock = 12, 8
    trace = []
    To, hist = oracle.solve(inp, zero, n_it, use_diis=True, trace=trace)
    T = dev["T"]
    for k in range(n_it):
        plan.iterate(1, T)
        cnt, drops, coef = plan.diis_state()
        ocnt, odrops, oc = trace[k]
        print("iteration", k, "gpu", cnt, drops, "oracle", ocnt, odrops, flush=True)
        if k < n_lock:
            assert (cnt, drops) == (ocnt, odrops), (k, cnt, drops, ocnt, odrops)
            if oc is not None:
                np.testing.assert_allclose(coef, oc, rtol=0, atol=1e-9)
    assert trace[n_lock - 1][1] == 1                 # the drop happened ...
    E_gpu, _ = plan.history()
    for k in range(n_it):                            # ... and the solve still matches
        assert abs(E_gpu[k] - hist[k][0]) <= 1e-10, (k, E_gpu[k], hist[k][0])
    compare_blocks(prob, T.cpu().numpy(), To, rel=1e-9)
    plan.close()


def test_plain_jacobi_iterations_match_oracle():
    prob = build_problem("chain", n_occ=16, band=4, somos=(5, 11))
    plan, dev = device_problem(prob, diis_max=0, T_random=False)
    plan.iterate(5, dev["T"])
    E_gpu, _ = plan.history()
    inp = oracle_inputs(prob)
    zero = unpack_T(prob, np.zeros(prob.n_T))
    To, hist = oracle.solve(inp, zero, 5, use_diis=False)
    for k in range(5):
        assert abs(E_gpu[k] - hist[k][0]) <= 1e-10
    compare_blocks(prob, dev["T"].cpu().numpy(), To, rel=1e-11)
    plan.close()


def test_nonfinite_detected():
    from paper_2008_03237_amd import DlpnoError
    prob = build_problem("tiny")
    plan, dev = device_problem(prob)
    dev["T"][int(prob.off_T[40]) + 3] = float("nan")
    with pytest.raises(DlpnoError) as ei:
        plan.iterate(1, dev["T"])
    assert ei.value.status == -5
    plan.close()


@pytest.mark.parametrize("cfg,nsample,fock_spin", [("chain", 12, 0.0), ("c160", 6, 0.0), ("chain", 12, 0.3)])
def test_full_size_sampled_residual(cfg, nsample, fock_spin):
    """Full workload in the benchmark's launch configuration; a seeded sample of
    target pairs recomputed by the oracle one by one (inputs regenerated).
    fock_spin > 0: spin-dependent off-diagonal occupied Fock."""
    prob = build_problem(cfg, fock_spin=fock_spin)
    print("case", cfg, "fock_spin", fock_spin, "pairs", prob.n_pairs, flush=True)
    plan, dev = device_problem(prob)
    R = plan.residual(dev["T"])
    Tn, e_pair, _ = plan.update(dev["T"], R)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1234)
    n = prob.npno
    nb = prob.n_blocks()
    # always include the largest pair, a SOMO pair and a pair with one block
    pick = set(rng.choice(prob.n_pairs, nsample, replace=False).tolist())
    pick.add(int(np.argmax(n.astype(np.int64) ** 3 * prob.naux)))
    pick.add(int(np.where(nb == 1)[0][0]))
    pick.add(int(np.where(nb == 2)[0][0]))
    inp = oracle_inputs(prob, full=False)
    # amplitudes of the sampled pairs and of every source they read
    need = set(pick)
    for p in pick:
        need.update(prob.cpl_src[prob.cpl_rowptr[p]:prob.cpl_rowptr[p + 1]].tolist())
    T = {}
    for p in need:
        o = int(prob.off_T[p])
        for name in oracle.stored_blocks(int(prob.pi[p]), int(prob.pj[p]), prob.is_somo.astype(bool)):
            seg = prob.segs["T"][np.searchsorted(prob.segs["T"]["off"], o)]
            T[(p, name)] = segment_values(prob.seed, seg).reshape(n[p], n[p])
            o += int(n[p]) ** 2
    Ro = oracle.residual_os(inp, T, pairs=sorted(pick))
    # Jacobi update and pair-block energies of the sampled pairs
    Tno = oracle.jacobi(inp, {k: T[k] for k in Ro}, Ro)
    eo = oracle.pair_energies(inp, Tno)
    Rg = R.cpu().numpy()
    Tg = Tn.cpu().numpy()
    ep = e_pair.cpu().numpy().reshape(-1, 4)
    code = {"AA": 0, "BB": 1, "AB": 2, "BA": 3}
    for (p, name), ref in Ro.items():
        i = oracle.stored_blocks(int(prob.pi[p]), int(prob.pj[p]), prob.is_somo.astype(bool)).index(name)
        o = int(prob.off_T[p]) + i * int(n[p]) ** 2
        got = Rg[o:o + int(n[p]) ** 2].reshape(n[p], n[p])
        d = np.linalg.norm(got - ref)
        assert d <= 1e-12 * np.linalg.norm(ref), (p, name, d, np.linalg.norm(ref))
        assert float(np.max(np.abs(got - ref))) <= 1e-12 * float(np.max(np.abs(ref))), (p, name)
        tg = Tg[o:o + int(n[p]) ** 2].reshape(n[p], n[p])
        assert np.linalg.norm(tg - Tno[(p, name)]) <= 1e-12 * np.linalg.norm(Tno[(p, name)]), (p, name)
        assert abs(ep[p, code[name]] - eo[(p, name)]) <= 1e-10, (p, name, ep[p, code[name]], eo[(p, name)])
    plan.close()


def test_graph_replay_matches_eager():
    """hipGraph replays (several, with host work between them) equal eager launches."""
    prob = build_problem("chain", n_occ=20, band=5, somos=(6, 13))
    plan, dev = device_problem(prob, T_random=False)
    T1 = dev["T"].clone()
    T2 = dev["T"].clone()
    plan.iterate(3, T1)              # captured graph, 3 replays
    _ = T1.sum().item()
    plan.iterate(2, T1)              # 2 more replays after eager torch work
    E_graph, _ = plan.history()
    plan.reset()
    plan.set_profiling(True)         # profiling bypasses the graph
    plan.iterate(5, T2)
    plan.set_profiling(False)
    E_eager, _ = plan.history()
    assert np.array_equal(E_graph, E_eager)
    assert torch.equal(T1.view(torch.int64), T2.view(torch.int64))
    plan.close()


@pytest.mark.parametrize("n", [1, 4, 5, 8, 16, 17, 22, 24, 26, 33, 39, 43, 48, 49, 55, 59, 64])
def test_every_tile_remainder_against_oracle(n):
    """Fixed PNO count n per pair: one, two, three and four tiles of 16 with
    every remainder R of k-steps in the last tile (row strips for R < 4, and
    column strips of the last a-tile for R <= 2; full tiles for R = 4) in the
    two-wave and the cooperative ladder launches,
    same-spin mirroring, and SOMO-SOMO pairs with one block next to diagonal
    SOMO pairs with none (SOMOs 3 and 5 within the band: pairs with none, one,
    two or four stored blocks)."""
    prob = build_problem("chain", n_occ=10, band=3, somos=(3, 5), npno=("fixed", n), naux=("uniform", 40, 90))
    print("case n =", n, prob.n_pairs, "pairs", prob.n_couplings, "couplings", flush=True)
    assert (prob.n_blocks() == 0).any() and (prob.n_blocks() == 1).any()
    plan, dev = device_problem(prob)
    R = plan.residual(dev["T"])
    torch.cuda.synchronize()
    inp = oracle_inputs(prob)
    Ro = oracle.residual_os(inp, unpack_T(prob, prob.materialize("T")))
    compare_blocks(prob, R.cpu().numpy(), Ro, rel=1e-12)
    plan.close()


def test_diagonal_pairs_only_no_couplings():
    """Band 0: only diagonal pairs, no projection terms (an empty projection
    queue), one block per DOMO pair and none per SOMO pair."""
    prob = build_problem("chain", n_occ=8, band=0, somos=(2, 5), naux=("uniform", 40, 90))
    assert prob.n_couplings == 0
    plan, dev = device_problem(prob)
    R = plan.residual(dev["T"])
    Tn, e_pair, e_tot = plan.update(dev["T"], R)
    torch.cuda.synchronize()
    inp = oracle_inputs(prob)
    T, Ro, Tno, eo = _oracle_step(prob, inp, prob.materialize("T"))
    compare_blocks(prob, R.cpu().numpy(), Ro, rel=1e-12)
    compare_blocks(prob, Tn.cpu().numpy(), Tno, rel=1e-12)
    assert abs(float(e_tot.cpu()[0]) - sum(eo.values())) <= 1e-10
    plan.close()


def test_flop_count_profiling_and_autotune():
    """dlpno_flop_count against the formula over the oracle's own term list;
    phase timers count one launch per kind; the autotuner's schedule keeps
    the residual at parity."""
    prob = build_problem("chain", n_occ=24, band=6, somos=(7, 16))
    plan, dev = device_problem(prob)
    inp = oracle_inputs(prob)
    T = unpack_T(prob, prob.materialize("T"))
    somo = prob.is_somo.astype(bool)
    lad = proj = 0.0
    for p in range(prob.n_pairs):
        n, m = int(prob.npno[p]), int(prob.naux[p])
        for name in oracle.stored_blocks(int(prob.pi[p]), int(prob.pj[p]), somo):
            lad += 4.0 * m * n ** 3
            for (w, q, S, src) in oracle.model.projection_terms(inp, T, p, name):
                nq = int(prob.npno[q])
                proj += 2.0 * n * nq * (n + nq)
    fl_l, fl_p = plan.flop_count()
    assert (fl_l, fl_p) == (lad, proj)
    plan.set_profiling(True)
    plan.residual(dev["T"])
    ms, cnt = plan.phase_times()
    plan.set_profiling(False)
    # the mini chain has pairs of 1..4 tiles: the two-wave and cooperative
    # ladder launches and both projection launches run (the one-wave ladder
    # launch only for leftovers)
    assert cnt[6] == 1 and cnt[7] == 1 and cnt[5] == 1 and cnt[8] == 1 and cnt[1] == 1 and cnt[0] <= 1
    assert ms[5] > 0 and ms[6] > 0 and ms[7] > 0 and ms[8] > 0
    plan.autotune(dev["T"])
    assert "autotune best" in plan.info()
    R = plan.residual(dev["T"])
    torch.cuda.synchronize()
    compare_blocks(prob, R.cpu().numpy(), oracle.residual_os(inp, T), rel=1e-12)
    plan.close()
