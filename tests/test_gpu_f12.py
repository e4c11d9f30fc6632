"""F12 correction on the GPU (through the C ABI) against the FP64 oracle."""
import numpy as np
import pytest

from oracle import f12
from tests.gpu_helpers import device_problem
from workload import build_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("cfg", ["tiny", "mini", "chain"])
def test_f12_energy_matches_oracle(cfg):
    prob = {"tiny": lambda: build_problem("tiny"),
            "mini": lambda: build_problem("chain", n_occ=24, band=6, somos=(7, 16)),
            "chain": lambda: build_problem("chain", n_occ=40, band=8, somos=(13, 27))}[cfg]()
    print("case", cfg, prob.n_pairs, "pairs", flush=True)
    from workload.gpu import device_fields
    plan, dev = device_problem(prob)
    W = device_fields(prob, fields=("W",))["W"]
    scal_h = prob.f12_scalars()
    scal = torch.from_numpy(scal_h).cuda()
    e_pair, e_tot = plan.f12_energy(dev["T"], W, scal)
    torch.cuda.synchronize()
    _, ep_o, tot_o = f12.f12_energy(prob, prob.materialize("T"), prob.materialize("W"), scal_h)
    ep = e_pair.cpu().numpy().reshape(-1, 4)
    scale = np.abs(ep_o).max()
    assert np.abs(ep - ep_o).max() <= 1e-13 * scale, np.abs(ep - ep_o).max()
    assert abs(float(e_tot.cpu()[0]) - tot_o) <= 1e-12 * abs(tot_o)
    # repeated call: bitwise equal (fixed-order sums)
    e_pair2, e_tot2 = plan.f12_energy(dev["T"], W, scal)
    torch.cuda.synchronize()
    assert torch.equal(e_pair.view(torch.int64), e_pair2.view(torch.int64))
    assert torch.equal(e_tot.view(torch.int64), e_tot2.view(torch.int64))
    plan.close()


def test_f12_energy_zero_amplitudes_gives_the_scalar_terms():
    prob = build_problem("tiny")
    from workload.gpu import device_fields
    plan, dev = device_problem(prob, T_random=False)
    W = device_fields(prob, fields=("W",))["W"]
    scal_h = prob.f12_scalars()
    _, e_tot = plan.f12_energy(dev["T"], W, torch.from_numpy(scal_h).cuda())
    torch.cuda.synchronize()
    _, _, tot_o = f12.f12_energy(prob, np.zeros(prob.n_T), prob.materialize("W"), scal_h)
    assert abs(float(e_tot.cpu()[0]) - tot_o) <= 1e-13 * abs(tot_o)
    plan.close()


def test_f12_full_size_sampled():
    """c160 workload in the benchmark's configuration; the F12 energies of a
    seeded sample of pairs recomputed by the oracle block by block from
    regenerated inputs, and the total against the sum of the GPU's pair
    energies."""
    from oracle.model import stored_blocks
    from workload.gpu import device_fields
    from workload.problem import segment_values
    prob = build_problem("c160")
    print("case c160 pairs", prob.n_pairs, flush=True)
    plan, dev = device_problem(prob)
    W = device_fields(prob, fields=("W",))["W"]
    scal_h = prob.f12_scalars()
    e_pair, e_tot = plan.f12_energy(dev["T"], W, torch.from_numpy(scal_h).cuda())
    torch.cuda.synchronize()
    ep = e_pair.cpu().numpy().reshape(-1, 4)
    rng = np.random.default_rng(99)
    nb = prob.n_blocks()
    blk0 = np.concatenate([[0], np.cumsum(nb)[:-1]])
    pick = set(rng.choice(prob.n_pairs, 40, replace=False).tolist())
    pick.add(int(np.argmax(prob.npno)))
    pick.add(int(np.where(nb == 1)[0][0]))
    pick.add(int(np.where(nb == 2)[0][0]))
    somo = prob.is_somo.astype(bool)
    for p in sorted(pick):
        n = int(prob.npno[p])
        for k, name in enumerate(stored_blocks(int(prob.pi[p]), int(prob.pj[p]), somo)):
            o = int(prob.off_T[p]) + k * n * n
            i = np.searchsorted(prob.segs["T"]["off"], o)
            Tb = segment_values(prob.seed, prob.segs["T"][i]).reshape(n, n)
            Wb = segment_values(prob.seed, prob.segs["W"][i]).reshape(n, n)
            ref = f12.block_energy(name, Wb, Tb, scal_h[blk0[p] + k])
            got = ep[p, ("AA", "BB", "AB", "BA").index(name)]
            assert abs(got - ref) <= 1e-13 * max(abs(ref), 1e-3), (p, name, got, ref)
    assert abs(float(e_tot.cpu()[0]) - ep.sum()) <= 1e-12 * abs(ep.sum())
    plan.close()
