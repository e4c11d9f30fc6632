"""Shared set-up for the GPU tests: device inputs, plans, oracle comparisons."""
import numpy as np

import oracle
from oracle.model import unpack_T


def device_problem(prob, precision="fp64", diis_max=8, diis_start=3, T_random=True, **plan_options):
    import torch
    from paper_2008_03237_amd import Plan
    from workload.gpu import device_fields
    ring = getattr(prob, "n_ring", 0) > 0
    dev = device_fields(prob, fields=("B", "S", "K", "T", "Rg") if ring else ("B", "S", "K", "T"))
    eps_a = torch.from_numpy(prob.eps_a).cuda()
    eps_b = torch.from_numpy(prob.eps_b).cuda()
    if ring:
        plan_options.setdefault("ring_ints", dev["Rg"])
    plan = Plan(prob, dev["B"], dev["S"], dev["K"], eps_a, eps_b, precision=precision, diis_max=diis_max,
                diis_start=diis_start, **plan_options)
    if not T_random:
        dev["T"].zero_()
    return plan, dev


def antisymmetrize_same_spin(prob, flat):
    """Replace every same-spin (AA, BB) block of a flat amplitude-shaped device
    vector by its antisymmetric part (the physical amplitude space)."""
    somo = prob.is_somo.astype(bool)
    for p in range(prob.n_pairs):
        n = int(prob.npno[p])
        o = int(prob.off_T[p])
        for name in oracle.stored_blocks(int(prob.pi[p]), int(prob.pj[p]), somo):
            if name in ("AA", "BB"):
                blk = flat[o:o + n * n].view(n, n)
                blk.copy_((blk - blk.t()) / 2)
            o += n * n
    return flat


def oracle_inputs(prob, full=True):
    if full:
        return oracle.Inputs.from_problem(prob, B=prob.materialize("B"), K=prob.materialize("K"),
                                          S=prob.materialize("S"))
    return oracle.Inputs.from_problem(prob)


def compare_blocks(prob, flat_gpu, ref_blocks, rel=1e-12, pairs=None):
    """Per block: ||d||_F <= rel ||ref||_F + tiny, and max|d| <= rel * max|ref| over all."""
    got = unpack_T(prob, flat_gpu)
    gmax = max(float(np.max(np.abs(v))) for v in ref_blocks.values())
    worst = 0.0
    for k, ref in ref_blocks.items():
        d = got[k] - ref
        nr = float(np.linalg.norm(ref))
        nd = float(np.linalg.norm(d))
        assert nd <= rel * nr + rel * gmax * 1e-3, (k, nd, nr)
        assert float(np.max(np.abs(d))) <= rel * gmax, (k, float(np.max(np.abs(d))), gmax)
        worst = max(worst, nd / max(nr, 1e-300))
    return worst
