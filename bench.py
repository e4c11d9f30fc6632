"""Benchmark: open-shell DLPNO doubles-residual iterations on one MI355X.

One step = one full iteration of the hot path on the whole workload:
ladder + projection contractions (persistent grouped kernel), Fock dressing,
Jacobi update, pair/total energies and DIIS.  The timed steps are launched
with HIP events around every phase; the same steps replayed as one hipGraph
are timed afterwards for comparison.

Prints ONE JSON line with the pair-residual GFLOP/s (algorithmic ladder +
projection FLOPs per iteration / wall time per iteration), CCSD iterations
per second, the roofline of the dominant kernel (the grouped kernel, timed with
HIP events on its own stream) and the FP64 CPU oracle timed on a bounded
sample of the same workload on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}


def cpu_baseline(prob, n_pairs=400, seed=99, repeats=3):
    """Time the FP64 oracle on a contiguous window of pairs of the workload
    (inputs regenerated from the seeded counters beforehand, not timed);
    median of `repeats` runs.  The flop count is the algorithmic one of the
    terms the oracle applies (ladder 4 m n^3 per block, projection
    2 n_p n_q (n_p + n_q) per applied term)."""
    import concurrent.futures as cf

    import numpy as np

    import oracle
    from oracle.model import projection_terms
    from workload.problem import segment_values

    blas, threads = "unknown", os.cpu_count() or 1
    try:
        from threadpoolctl import threadpool_info
        info = [d for d in threadpool_info() if d.get("user_api") == "blas"]
        if info:
            blas = "%s %s" % (info[0].get("internal_api", "?"), info[0].get("version", ""))
            threads = max(d.get("num_threads", 1) for d in info)
    except Exception:
        pass
    P = prob.n_pairs
    rng = np.random.default_rng(seed)
    start = int(rng.integers(0, max(1, P - n_pairs)))
    pick = list(range(start, min(P, start + n_pairs)))
    inp = oracle.Inputs.from_problem(prob)
    n = prob.npno
    need = set(pick)
    for p in pick:
        need.update(prob.cpl_src[prob.cpl_rowptr[p]:prob.cpl_rowptr[p + 1]].tolist())
    somo = prob.is_somo.astype(bool)

    def gen_T(p):
        out = {}
        o = int(prob.off_T[p])
        for name in oracle.stored_blocks(int(prob.pi[p]), int(prob.pj[p]), somo):
            seg = prob.segs["T"][np.searchsorted(prob.segs["T"]["off"], o)]
            out[(p, name)] = segment_values(prob.seed, seg).reshape(n[p], n[p])
            o += int(n[p]) ** 2
        return out

    def gen_pair(p):
        inp.B(p)
        for e in range(prob.cpl_rowptr[p], prob.cpl_rowptr[p + 1]):
            inp.S(p, int(prob.cpl_src[e]))

    T = {}
    with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 4)) as ex:
        for d in ex.map(gen_T, sorted(need)):
            T.update(d)
        list(ex.map(gen_pair, pick))
    flops = 0.0
    for p in pick:
        for name in inp.blocks(p):
            flops += 4.0 * float(prob.naux[p]) * float(n[p]) ** 3
            for (_, q, _, _) in projection_terms(inp, T, p, name):
                flops += 2.0 * float(n[p]) * float(n[q]) * float(n[p] + n[q])
    times = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        R = oracle.residual_os(inp, T, pairs=pick)
        Tn = oracle.jacobi(inp, {k: T[k] for k in R}, R)
        oracle.pair_energies(inp, Tn)
        times.append(time.perf_counter() - t0)
    dt = sorted(times)[len(times) // 2]
    return {"value": round(flops / dt / 1e9, 3), "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": "%d contiguous pairs (of %d) of the same workload: residual + Jacobi + pair energies, "
                      "median of %d runs, %.1f s each (%s)" % (len(pick), P, repeats, dt,
                                                              ", ".join("%.1f" % t for t in times)),
            "blas": blas, "host_cpus": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c160")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-pairs", type=int, default=400)
    ap.add_argument("--no-mixed", action="store_true", help="skip the split-precision / refinement leg")
    ap.add_argument("--no-f12", action="store_true", help="skip the F12-correction leg")
    ap.add_argument("--mixed-precisions", default="bf16x2,fp16x2",
                    help="comma-separated split precisions of the mixed leg (bf16x2, fp16x2, fp32)")
    ap.add_argument("--mixed-outer", type=int, default=2, help="FP64 refinement steps")
    ap.add_argument("--mixed-inner", type=int, default=4, help="low-precision iterations per refinement step")
    ap.add_argument("--mixed-also", default="3x3",
                    help="further refinement schedules OUTERxINNER timed for every split precision ('' = none)")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-path leg")
    ap.add_argument("--no-hole", action="store_true", help="skip the hole-hole ladder leg")
    ap.add_argument("--no-ring", action="store_true", help="skip the ring/exchange-term leg")
    ap.add_argument("--no-occ", action="store_true",
                    help="skip the leg with the quadratic part of the occupied Fock intermediate")
    ap.add_argument("--ring-scale", type=float, default=0.05,
                    help="scale of the synthetic integral blocks of the ring/exchange-term leg")
    ap.add_argument("--no-pno", action="store_true", help="skip the PNO-construction leg")
    ap.add_argument("--no-somo-virt", action="store_true", help="skip the SOMO-augmented virtual space leg")
    ap.add_argument("--hole-scale", type=float, default=0.02,
                    help="scale of the synthetic occupied integrals of the hole-hole ladder leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device copy first (reference for HBM byte counters)")
    ap.add_argument("--profile-residuals", type=int, default=0,
                    help="profiling run: only N residual evaluations per precision of --profile-precisions "
                         "(default schedule), one JSON line of their kernel times, nothing else")
    ap.add_argument("--profile-precisions", default="fp64,bf16x2,fp16x2")
    ap.add_argument("--profile-pno", type=int, default=0,
                    help="profiling run: only N PNO builds and N overlap launches of the workload, one JSON line")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: runs on one GPU only (sharding the pairs across GPUs is not implemented); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2008_03237_amd import Plan
    from workload import build_problem
    from workload.gpu import device_fields

    def log(msg):
        print("[bench %.1fs] %s" % (time.perf_counter() - t_setup, msg), file=sys.stderr, flush=True)

    t_setup = time.perf_counter()
    if args.copy_calibration:
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    if args.profile_pno > 0:
        print(json.dumps(profile_pno(args, log)), flush=True)
        return
    prob = build_problem(args.workload)
    log("workload %s: %d pairs, %d couplings" % (args.workload, prob.n_pairs, prob.n_couplings))
    dev = device_fields(prob)
    log("inputs generated on the device")
    eps_a = torch.from_numpy(prob.eps_a).cuda()
    eps_b = torch.from_numpy(prob.eps_b).cuda()
    if args.profile_residuals > 0:
        print(json.dumps(profile_residuals(prob, dev, eps_a, eps_b, args, log)), flush=True)
        return
    plan = Plan(prob, dev["B"], dev["S"], dev["K"], eps_a, eps_b, precision=args.precision)
    T = dev["T"]                 # seeded amplitudes: the autotuner times the grouped kernel on them
    log("plan created")
    if not args.no_autotune:
        plan.autotune(T)
        log("autotuned:\n" + plan.info())
    T.zero_()                    # iterations start from T = 0
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    fl_ladder, fl_proj = plan.flop_count()
    flops = fl_ladder + fl_proj

    # warmup (graph replay), then K timed iterations.  The timed iterations are
    # launched eagerly with HIP events around each phase on the plan's stream,
    # so the grouped kernel's duration comes from the timed region itself.
    plan.iterate(args.warmup, T)
    torch.cuda.synchronize()
    plan.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, e_tot, rmax = plan.iterate(args.steps, T)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms, cnt = plan.phase_times()
    plan.set_profiling(False)
    ms_step = dt / max(args.steps, 1) * 1e3
    E_hist, R_hist = plan.history()
    log("timed %d iterations: %.3f ms/iteration, E = %s" % (args.steps, ms_step, E_hist[-1:]))
    # the same iterations replayed as one hipGraph (context: launch overhead)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.iterate(args.steps, T)
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - t0) / max(args.steps, 1) * 1e3

    # dominant kernel: the grouped kernel over the ladder items, in up to three
    # launches per residual (phase 6: pairs of at most three PNO tiles at two
    # waves per SIMD; phase 7: four-tile pairs, one workgroup per item, two
    # waves per SIMD; phase 0: anything else, one wave per SIMD); its
    # projection launch (phase 5) is reported beside it
    lad1_ms = ms[0] / max(cnt[0], 1)
    lad2_ms = ms[6] / max(cnt[6], 1)
    lad4_ms = ms[7] / max(cnt[7], 1)
    kern_ms = lad1_ms + lad2_ms + lad4_ms
    # projection: phase 8 (two waves per SIMD) and phase 5 (one)
    proj1_ms = ms[5] / max(cnt[5], 1)
    proj2_ms = ms[8] / max(cnt[8], 1)
    proj_ms = proj1_ms + proj2_ms
    achieved = fl_ladder / (kern_ms / 1e3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    # counter record of the ladder launches (rocprofv3, profiles/): HBM bytes
    # and issued MFMA flops per residual, used only while it describes this
    # kernel source and schedule
    traffic, issued = None, None
    schedule = schedule_line(plan)
    cfile = os.path.join(ROOT, "profiles", "grouped_%s_%s_counters.json" % (args.workload, args.precision))
    if os.path.exists(cfile):
        with open(cfile) as f:
            tr = json.load(f)
        if tr.get("kernel_source_sha") == kernel_source_sha() and tr.get("schedule") == schedule:
            traffic = tr.get("bytes_per_residual")
            issued = tr.get("issued_flops_per_residual")

    out = {
        "metric": "pair-residual GFLOP/s (ladder + projection, algorithmic) per CCSD iteration",
        "value": round(flops / (ms_step / 1e3) / 1e9, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "iter_per_s": round(1e3 / ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic (seeded Philox counters; alkane-chain-shaped pair list)",
        "config": {"workload": args.workload, "pairs": prob.n_pairs, "pair_blocks": int(prob.n_blocks().sum()),
                   "couplings": int(prob.n_couplings), "n_occ": prob.n_occ, "somos": int(prob.is_somo.sum()),
                   "flops_ladder": fl_ladder, "flops_projection": fl_proj, "B_GB": round(prob.n_B * 8 / 1e9, 2),
                   "S_GB": round(prob.n_S * 8 / 1e9, 2), "hipgraph": True, "autotuned": not args.no_autotune},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 4), "traffic": traffic,
                     "frac_issued": round(issued / (kern_ms / 1e3) / 1e12 / peak, 4) if issued else None,
                     "issued_flops_per_residual": issued,
                     "kernel": "grouped_kernel<%s, ladder items>" % ("double" if args.precision == "fp64" else "float"),
                     "kernel_ms": round(kern_ms, 3), "residuals": int(max(cnt[0], cnt[6], cnt[7])),
                     "launch_ms": {"two_waves_per_simd": round(lad2_ms, 3), "cooperative": round(lad4_ms, 3),
                                   "one_wave_per_simd": round(lad1_ms, 3)},
                     "flops_per_residual": fl_ladder, "schedule": schedule},
        "projection_kernel": {"kernel": "grouped_kernel<%s, projection items>" % (
                                  "double" if args.precision == "fp64" else "float"),
                              "kernel_ms": round(proj_ms, 3), "flops_per_residual": fl_proj,
                              "launch_ms": {"two_waves_per_simd": round(proj2_ms, 3),
                                            "one_wave_per_simd": round(proj1_ms, 3)},
                              "achieved": round(fl_proj / (proj_ms / 1e3) / 1e12, 3) if proj_ms > 0 else None,
                              "frac": round(fl_proj / (proj_ms / 1e3) / 1e12 / peak, 4) if proj_ms > 0 else None},
        "ms_per_step_graph": round(ms_graph, 3),
        "energy_last": float(E_hist[-1]) if len(E_hist) else None,
        "setup_s": round(setup_s, 1),
    }
    log("grouped kernel: ladder %.3f ms (two-wave launch %.3f, cooperative %.3f, one-wave %.3f), projection %.3f ms "
        "(two-wave %.3f, one-wave %.3f) per residual" % (kern_ms, lad2_ms, lad4_ms, lad1_ms, proj_ms, proj2_ms, proj1_ms))
    if not args.no_f12:
        out["f12"] = f12_leg(prob, plan, T, log)
    if not (args.no_mixed and args.no_fp32) and args.precision == "fp64":
        ref = fp64_reference(prob, plan, log)
        if not args.no_mixed:
            out["mixed"] = mixed_leg(prob, dev, eps_a, eps_b, args, flops, ref, log)
        if not args.no_fp32:
            out["fp32"] = fp32_leg(prob, dev, eps_a, eps_b, args, fl_ladder, fl_proj, ref, log)
    if not args.no_hole and args.precision == "fp64":
        out["hole_ladder"] = hole_leg(args, dev, eps_a, eps_b, fl_proj, log)
    if not args.no_ring and args.precision == "fp64":
        out["ring"] = ring_leg(args, dev, eps_a, eps_b, log)
    if not args.no_occ and args.precision == "fp64":
        out["quadratic_occ"] = occ_leg(args, prob, dev, eps_a, eps_b, log)
    if not args.no_pno:
        out["pno"] = pno_leg(args, log)
    plan.close()
    if not args.no_somo_virt and args.precision == "fp64":
        # the main leg's inputs make room for the larger augmented ones
        del plan, dev, T, eps_a, eps_b
        torch.cuda.empty_cache()
        out["somo_virt"] = somo_virt_leg(args, flops, log)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, n_pairs=args.cpu_pairs)
    print(json.dumps(out), flush=True)


def f12_leg(prob, plan, T, log):
    """The F12 correction (V-tilde contraction and spin-adapted pair energies)
    with the amplitudes the timed iterations left, on synthetic W = V + C and
    F12 scalars: HIP-event time of dlpno_f12_energy (block kernel and the
    pair/total reduction) and its algorithmic HBM bytes, T and W once."""
    import torch
    from workload.gpu import device_fields
    W = device_fields(prob, fields=("W",))["W"]
    scal = torch.from_numpy(prob.f12_scalars()).cuda()
    e_pair, e_tot = plan.f12_energy(T, W, scal)
    torch.cuda.synchronize()
    reps = 20
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        plan.f12_energy(T, W, scal, e_pair, e_tot)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    nblk = int(prob.n_blocks().sum())
    nbytes = 2 * 8 * prob.n_T + 8 * 6 * nblk + 8 * (nblk + 4 * prob.n_pairs + 1)
    res = {"kernels": "f12_kernel + reduce_parts_kernel + reduce_final_kernel", "ms": round(ms, 4), "algorithmic_bytes": nbytes,
           "achieved_GBps": round(nbytes / (ms / 1e3) / 1e9, 1),
           "hbm_frac": round(nbytes / (ms / 1e3) / 1e9 / 8000.0, 4),
           "energy_f12": float(e_tot.cpu()[0]), "amplitudes": "after the timed iterations"}
    log("f12 leg: %s" % res)
    del W
    return res


def profile_residuals(prob, dev, eps_a, eps_b, args, log):
    """Profiling run (rocprofv3 kernel traces and counters): for each precision,
    a plan with the default schedule and args.profile_residuals residual
    evaluations of the seeded amplitudes; their per-launch kernel times."""
    import torch

    from paper_2008_03237_amd import Plan
    out = {"workload": args.workload, "residuals": args.profile_residuals, "launch_ms": {}}
    names = ["ladder one-wave", "finish", "reduce", "diis", "convert", "projection one-wave", "ladder two-wave",
             "ladder cooperative", "projection two-wave"]
    for prec in args.profile_precisions.split(","):
        plan = Plan(prob, dev["B"], dev["S"], dev["K"], eps_a, eps_b, precision=prec)
        R = torch.empty_like(dev["T"])
        plan.set_profiling(True)
        for k in range(args.profile_residuals):
            plan.residual(dev["T"], R)
            log("%s residual %d done" % (prec, k))
        torch.cuda.synchronize()
        ms, cnt = plan.phase_times()
        plan.set_profiling(False)
        out["launch_ms"][prec] = {names[k]: round(ms[k] / cnt[k], 3) for k in range(len(names)) if cnt[k] > 0}
        out.setdefault("schedule", {})[prec] = schedule_line(plan)
        fl, fp = plan.flop_count()
        out.setdefault("flops_per_residual", {"ladder": fl, "projection": fp})
        plan.close()
        del R
    return out


# LDS bandwidth of the chip: 256 CUs x 128 bytes per clock x 2.4 GHz
LDS_PEAK_TBPS = 256 * 128 * 2.4e9 / 1e12


def pno_leg(args, log):
    """PNO construction for every pair of the workload's pair list (domains
    of 40..64 functions, T_CutPNO = 1e-7): HIP-event time of dlpno_pno_build
    (one launch).  Its bound is the LDS traffic of the Jacobi rotations: per
    round of a sweep over an m x m matrix (m = N rounded up to even), the
    matrix and the eigenvector matrix are each read and written once,
    4 m^2 doubles; rounds = sweeps x (m - 1), from the launch's own sweep
    counts, for the density and the PNO Fock matrix (m = n_p rounded up)."""
    import numpy as np
    import torch

    from paper_2008_03237_amd import PnoPlan
    from workload.gpu import device_pno_fields
    from workload.pno import build_pno_problem
    prob = build_pno_problem(args.workload)
    dev = device_pno_fields(prob)
    plan = PnoPlan(prob.pairs, prob.n_X, prob.n_F, prob.n_C, prob.n_v)
    out = plan.build(dev["X"], dev["F"], prob.t_cut, want_sweeps=True)
    torch.cuda.synchronize()
    reps = 5
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        plan.build(dev["X"], dev["F"], prob.t_cut, *out[:4], sweeps=out[4])
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    nk = out[3].cpu().numpy().astype(np.int64)
    sw = out[4].cpu().numpy().reshape(-1, 2).astype(np.int64)
    if np.any(nk < 0):
        raise RuntimeError("PNO construction failed for %d pairs" % int((nk < 0).sum()))
    m1 = prob.pairs["dim"].astype(np.int64)
    m1 += m1 & 1
    m2 = nk + (nk & 1)
    lds_bytes = int((32 * m1 * m1 * sw[:, 0] * np.maximum(m1 - 1, 0)).sum()
                    + (32 * m2 * m2 * sw[:, 1] * np.maximum(m2 - 1, 0)).sum())
    ach = lds_bytes / (ms / 1e3) / 1e12
    log("PNO construction: %d pairs in %.3f ms, %.1f PNOs kept per pair" % (prob.n_pairs, ms, nk.mean()))
    res = {"kernel": "pno_build_kernel", "workload": "%s pair list, domains %d..%d, T_CutPNO %.0e"
           % (args.workload, int(prob.pairs["dim"].min()), int(prob.pairs["dim"].max()), prob.t_cut),
           "pairs": prob.n_pairs, "ms": round(ms, 3), "pairs_per_s": round(prob.n_pairs / (ms / 1e3), 1),
           "kept_mean": round(float(nk.mean()), 2),
           "sweeps_mean": [round(float(sw[:, 0].mean()), 2), round(float(sw[nk > 0, 1].mean()), 2)],
           "roofline": {"bound": "lds", "achieved": round(ach, 3), "peak": round(LDS_PEAK_TBPS, 2), "unit": "TB/s",
                        "frac": round(ach / LDS_PEAK_TBPS, 4), "lds_bytes": lds_bytes}}
    # the S blocks of the residual's coupling list with these PNO counts; its
    # algorithmic HBM bytes: every S block written once, every C read once
    from workload import build_problem
    rp = build_problem(args.workload, npno=("given", np.maximum(nk, 1)))
    plan.overlap_prepare(nk, rp.cpl_rowptr, rp.cpl_src, rp.cpl_off_S, rp.n_S)
    S = plan.overlap(out[2])
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        plan.overlap(out[2], S)
    b.record()
    torch.cuda.synchronize()
    ms_o = a.elapsed_time(b) / reps
    nbytes = 8 * (rp.n_S + prob.n_C)
    log("PNO overlaps: %d couplings in %.3f ms" % (int(rp.cpl_rowptr[-1]), ms_o))
    # counter record (rocprofv3 FETCH_SIZE + WRITE_SIZE of one launch), used
    # only while it describes this source and workload
    traffic = None
    cfile = os.path.join(ROOT, "profiles", "pno_%s_counters.json" % args.workload)
    if os.path.exists(cfile):
        with open(cfile) as f:
            rec = json.load(f)
        if rec.get("pno_source_sha") == pno_source_sha():
            traffic = rec.get("overlap_bytes_per_launch")
    res["overlap"] = {"kernel": "pno_overlap_kernel", "couplings": int(rp.cpl_rowptr[-1]), "ms": round(ms_o, 3),
                      "S_GB": round(rp.n_S * 8 / 1e9, 2),
                      "roofline": {"bound": "hbm", "achieved": round(nbytes / (ms_o / 1e3) / 1e9, 1), "peak": 8000.0,
                                   "unit": "GB/s", "frac": round(nbytes / (ms_o / 1e3) / 8e12, 4),
                                   "algorithmic_bytes": nbytes, "traffic": traffic}}
    plan.close()
    del dev, S, out
    return res


def profile_pno(args, log):
    """args.profile_pno PNO builds and overlap launches of the workload (for
    rocprofv3), with their HIP-event times."""
    import numpy as np
    import torch

    from paper_2008_03237_amd import PnoPlan
    from workload import build_problem
    from workload.gpu import device_pno_fields
    from workload.pno import build_pno_problem
    prob = build_pno_problem(args.workload)
    dev = device_pno_fields(prob)
    plan = PnoPlan(prob.pairs, prob.n_X, prob.n_F, prob.n_C, prob.n_v)
    out = plan.build(dev["X"], dev["F"], prob.t_cut, want_sweeps=True)
    torch.cuda.synchronize()
    nk = out[3].cpu().numpy().astype(np.int64)
    rp = build_problem(args.workload, npno=("given", np.maximum(nk, 1)))
    plan.overlap_prepare(nk, rp.cpl_rowptr, rp.cpl_src, rp.cpl_off_S, rp.n_S)
    S = plan.overlap(out[2])
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {"workload": args.workload, "pairs": prob.n_pairs, "couplings": int(rp.cpl_rowptr[-1])}
    for name, fn in (("pno_build_kernel", lambda: plan.build(dev["X"], dev["F"], prob.t_cut, *out[:4], sweeps=out[4])),
                     ("pno_overlap_kernel", lambda: plan.overlap(out[2], S))):
        a.record()
        for _ in range(args.profile_pno):
            fn()
        b.record()
        torch.cuda.synchronize()
        res[name + "_ms"] = round(a.elapsed_time(b) / args.profile_pno, 3)
        log("%s: %.3f ms" % (name, res[name + "_ms"]))
    plan.close()
    return res


def somo_virt_leg(args, flops_base, log):
    """The same workload with every PNO set augmented by the SOMOs as beta-only
    virtual functions (n_p + 2 functions per pair, masks on the alpha
    indices): FP64 iterations from T = 0, timed like the main leg."""
    import torch

    from paper_2008_03237_amd import Plan
    from workload import build_problem
    from workload.gpu import device_fields
    prob = build_problem(args.workload, somo_virt=True)
    dev = device_fields(prob, fields=("B", "S", "K"))
    eps_a = torch.from_numpy(prob.eps_a).cuda()
    eps_b = torch.from_numpy(prob.eps_b).cuda()
    plan = Plan(prob, dev["B"], dev["S"], dev["K"], eps_a, eps_b)
    T = torch.zeros(max(prob.n_T, 1), dtype=torch.float64, device="cuda")
    plan.iterate(args.warmup, T)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, e_tot, rmax = plan.iterate(args.steps, T)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) / max(args.steps, 1) * 1e3
    fl, fp = plan.flop_count()
    row = {"pno_plus_somo_mean": round(float(prob.npno.mean()), 2), "ms_per_step": round(ms_step, 3),
           "value_gflops": round((fl + fp) / (ms_step / 1e3) / 1e9, 2), "flops": fl + fp,
           "flops_vs_main": round((fl + fp) / flops_base, 4), "energy_after": float(e_tot.cpu()[0]),
           "iterations": args.warmup + args.steps, "max_abs_R": float(rmax.cpu()[0]),
           "B_GB": round(prob.n_B * 8 / 1e9, 2)}
    log("SOMO-augmented leg: %s" % row)
    plan.close()
    del dev, T
    torch.cuda.empty_cache()
    return row


def hole_leg(args, dev, eps_a, eps_b, fl_proj_base, log):
    """The same workload with the hole-hole ladder added (the first of the
    CCSD terms beyond the hot path's model): synthetic occupied integrals
    (k i | l j) within two orbitals of (i, j), one extra coupling per ordered
    (k, l), run by the projection launches.  FP64 iterations from T = 0,
    timed like the main leg; then the same with the quadratic term on those
    couplings."""
    import torch

    from paper_2008_03237_amd import Plan
    from workload import build_problem
    from workload.gpu import device_fields
    prob = build_problem(args.workload, hole_ladder=args.hole_scale)
    S = device_fields(prob, fields=("S",))["S"]          # B, K and eps are those of the main leg
    plan = Plan(prob, dev["B"], S, dev["K"], eps_a, eps_b)
    T = torch.zeros(max(prob.n_T, 1), dtype=torch.float64, device="cuda")
    plan.iterate(args.warmup, T)
    torch.cuda.synchronize()
    plan.set_profiling(True)
    t0 = time.perf_counter()
    _, _, e_tot, rmax = plan.iterate(args.steps, T)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) / max(args.steps, 1) * 1e3
    ms, cnt = plan.phase_times()
    plan.set_profiling(False)
    fl, fp = plan.flop_count()
    proj_ms = ms[5] / max(cnt[5], 1) + ms[8] / max(cnt[8], 1)
    row = {"hole_hole_couplings": int(prob.n_hh), "ms_per_step": round(ms_step, 3),
           "value_gflops": round((fl + fp) / (ms_step / 1e3) / 1e9, 2),
           "flops_hole_hole": fp - fl_proj_base, "flops_projection_and_hole_hole": fp,
           "projection_ms": round(proj_ms, 3),
           "projection_tflops": round(fp / (proj_ms / 1e3) / 1e12, 3) if proj_ms > 0 else None,
           "energy_after": float(e_tot.cpu()[0]), "iterations": args.warmup + args.steps,
           "max_abs_R": float(rmax.cpu()[0]), "S_GB": round(prob.n_S * 8 / 1e9, 2)}
    log("hole-hole ladder leg: %s" % row)
    plan.close()
    # the same couplings carrying the quadratic term: per residual a kernel
    # computes their weights from T (phase 9), then the same launches run
    pq = Plan(prob, dev["B"], S, dev["K"], eps_a, eps_b, quadratic=True)
    T.zero_()
    pq.iterate(args.warmup, T)
    torch.cuda.synchronize()
    pq.set_profiling(True)
    t0 = time.perf_counter()
    _, _, e_q, r_q = pq.iterate(args.steps, T)
    torch.cuda.synchronize()
    ms_q = (time.perf_counter() - t0) / max(args.steps, 1) * 1e3
    msq, cntq = pq.phase_times()
    pq.set_profiling(False)
    fq = [l for l in pq.info().splitlines() if "quadratic-term weights" in l]
    fl_w = float(fq[0].split()[-1]) if fq else None
    w_ms = msq[9] / max(cntq[9], 1)
    row["quadratic"] = {"ms_per_step": round(ms_q, 3), "weights_kernel_ms": round(w_ms, 3),
                        "weights_flops": fl_w,
                        "weights_tflops": round(fl_w / (w_ms / 1e3) / 1e12, 3) if fl_w and w_ms > 0 else None,
                        "energy_after": float(e_q.cpu()[0]), "max_abs_R": float(r_q.cpu()[0])}
    log("quadratic term: %s" % row["quadratic"])
    pq.close()
    del S, T
    return row


def ring_leg(args, dev, eps_a, eps_b, log):
    """The same workload with the ring/exchange term added (linear in the
    doubles): synthetic integral blocks X = (m e|b y) and J = (m y|b e) for
    every replacing occupied m within two orbitals of the shared index, summed
    per target block by the ring kernel (FP64 MFMA).  FP64 iterations from
    T = 0, timed like the main leg; the ring kernel's time per residual and its
    rate against the FP64 MFMA peak."""
    import torch

    from paper_2008_03237_amd import Plan
    from workload import build_problem
    from workload.gpu import device_fields
    prob = build_problem(args.workload, ring=args.ring_scale)
    f = device_fields(prob, fields=("S", "Rg"))         # B, K and eps are those of the main leg
    plan = Plan(prob, dev["B"], f["S"], dev["K"], eps_a, eps_b, ring_ints=f["Rg"])
    T = torch.zeros(max(prob.n_T, 1), dtype=torch.float64, device="cuda")
    plan.iterate(args.warmup, T)
    torch.cuda.synchronize()
    plan.set_profiling(True)
    t0 = time.perf_counter()
    _, _, e_tot, rmax = plan.iterate(args.steps, T)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) / max(args.steps, 1) * 1e3
    ms, cnt = plan.phase_times()
    plan.set_profiling(False)
    fl_ring, n_contr = plan.ring_flop_count()
    ring_ms = ms[10] / max(cnt[10], 1)
    tf = fl_ring / (ring_ms / 1e3) / 1e12 if ring_ms > 0 else None
    row = {"ring_couplings": int(prob.n_ring), "contractions": int(n_contr), "ms_per_step": round(ms_step, 3),
           "ring_kernel": "ring_kernel (FP64 MFMA 16x16x4)", "ring_kernel_ms": round(ring_ms, 3),
           "ring_flops_per_residual": fl_ring, "ring_tflops": round(tf, 3) if tf else None,
           "ring_frac_fp64_peak": round(tf / 78.6, 4) if tf else None,
           "energy_after": float(e_tot.cpu()[0]), "iterations": args.warmup + args.steps,
           "max_abs_R": float(rmax.cpu()[0]), "ring_ints_GB": round(prob.n_Rg * 8 / 1e9, 2),
           "S_GB": round(prob.n_S * 8 / 1e9, 2)}
    log("ring/exchange leg: %s" % row)
    plan.close()
    del f, T
    torch.cuda.empty_cache()
    return row


def occ_leg(args, prob, dev, eps_a, eps_b, log):
    """The same workload with the quadratic part of the occupied Fock
    intermediate (DLPNO_FLAG_QUADRATIC_OCC): per residual F^s_mj is formed from
    T over every occupied-Fock coupling (factors S K S^T built once) and
    dresses the projection weights.  FP64 iterations from T = 0, timed like the
    main leg; the kernels forming F against HBM (they read the factors and the
    dotted amplitude blocks once)."""
    import torch

    from paper_2008_03237_amd import Plan
    from workload import build_problem
    pq = build_problem(args.workload, quadratic_occ=True)
    t0 = time.perf_counter()
    plan = Plan(pq, dev["B"], dev["S"], dev["K"], eps_a, eps_b, quadratic_occ=True)
    setup_s = time.perf_counter() - t0
    T = torch.zeros(max(pq.n_T, 1), dtype=torch.float64, device="cuda")
    plan.iterate(args.warmup, T)
    torch.cuda.synchronize()
    plan.set_profiling(True)
    t0 = time.perf_counter()
    _, _, e_tot, rmax = plan.iterate(args.steps, T)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) / max(args.steps, 1) * 1e3
    ms, cnt = plan.phase_times()
    plan.set_profiling(False)
    line = [l for l in plan.info().splitlines() if l.startswith("occupied-intermediate")]
    words = line[0].split() if line else []
    factors_gb = float(words[words.index("factors") + 1]) if "factors" in words else None
    flops = float(words[-4]) if line else None
    occ_ms = ms[9] / max(cnt[9], 1)
    # algorithmic bytes: the factors once per residual (the dotted amplitude
    # blocks, read by every contribution of their pair, are mostly L2 hits)
    gbps = factors_gb / (occ_ms / 1e3) if factors_gb and occ_ms > 0 else None
    row = {"ms_per_step": round(ms_step, 3), "occ_kernels_ms": round(occ_ms, 3), "flops_per_residual": flops,
           "factors_GB": factors_gb, "factor_read_GBps": round(gbps, 1) if gbps else None,
           "factor_read_hbm_frac": round(gbps / 8000.0, 4) if gbps else None, "setup_s": round(setup_s, 1),
           "energy_after": float(e_tot.cpu()[0]), "iterations": args.warmup + args.steps,
           "max_abs_R": float(rmax.cpu()[0])}
    log("occupied-intermediate leg: %s" % row)
    plan.close()
    del T
    torch.cuda.empty_cache()
    return row


def fp64_reference(prob, plan64, log):
    """The converged FP64 solve (DIIS, from T = 0 to max|R| < 1e-9), timed:
    the reference of the precision legs."""
    import torch
    plan64.reset()
    T64 = torch.zeros(max(prob.n_T, 1), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n64 = 0
    while n64 < 60:
        _, e64, et64, r64 = plan64.iterate(2, T64)
        n64 += 2
        if float(r64.cpu()[0]) < 1e-9:
            break
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    ref = {"seconds": t64, "iterations": n64, "e_pair": e64.cpu().numpy().reshape(-1, 4).sum(1),
           "energy": float(et64.cpu()[0]), "max_abs_R": float(r64.cpu()[0])}
    log("fp64 reference solve: %d iterations, %.3f s, E = %.12f" % (n64, t64, ref["energy"]))
    del T64
    return ref


def split_precision_row(prob, dev, eps_a, eps_b, precision, args, flops, ref, log):
    """One split precision: grouped kernel throughput, the refined mixed solve
    (args.mixed_outer FP64 refinements of args.mixed_inner low-precision
    iterations) and the inner-only iteration, against the FP64 reference."""
    import numpy as np
    import torch

    from paper_2008_03237_amd import Plan
    mp = Plan(prob, dev["B"], dev["S"], dev["K"], eps_a, eps_b, precision=precision)
    Tm = torch.zeros(max(prob.n_T, 1), dtype=torch.float64, device="cuda")
    mp.solve_mixed(1, 1, Tm)              # warm-up (split conversions, code objects)
    Tm.zero_()
    mp.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, em, etm, rm = mp.solve_mixed(args.mixed_outer, args.mixed_inner, Tm)
    torch.cuda.synchronize()
    tm = time.perf_counter() - t0
    emn = em.cpu().numpy().reshape(-1, 4).sum(1)
    # other schedules (e.g. three refinements), each from T = 0
    others = {}
    for sched in [x for x in args.mixed_also.split(",") if x]:
        no, ni = (int(v) for v in sched.split("x"))
        To = torch.zeros_like(Tm)
        mp.reset()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, eo, eto, ro = mp.solve_mixed(no, ni, To)
        torch.cuda.synchronize()
        eon = eo.cpu().numpy().reshape(-1, 4).sum(1)
        te = abs(float(eto.cpu()[0]) - ref["energy"])
        pe = float(np.max(np.abs(eon - ref["e_pair"])))
        others[sched] = {"mixed_solve_s": round(time.perf_counter() - t1, 3),
                         "vs_fp64_solve": round((time.perf_counter() - t1) / ref["seconds"], 3),
                         "total_energy_error": te, "max_pair_energy_error": pe,
                         "gate_1e-7_pair_1e-6_total": bool(pe <= 1e-7 and te <= 1e-6)}
        del To
    # split grouped kernel alone (HIP events inside the library)
    mp.set_profiling(True)
    for _ in range(3):
        mp.residual(Tm)
    ms, cnt = mp.phase_times()
    mp.set_profiling(False)
    k_lad = ms[0] / max(cnt[0], 1)
    k_proj = ms[5] / max(cnt[5], 1)
    k_ms = k_lad + k_proj
    conv_ms = ms[4] / max(cnt[4], 1)
    # inner only: the low-precision residuals iterated (FP64 update, energies
    # and DIIS) with no FP64 refinement, until max|R| stops falling
    Ti = torch.zeros_like(Tm)
    mp.reset()
    best, n_in, r_now = None, 0, None
    while n_in < 40:
        _, ei, eti, ri = mp.iterate(2, Ti)
        n_in += 2
        r_now = float(ri.cpu()[0])
        if best is not None and r_now >= 0.5 * best:
            break
        best = r_now if best is None else min(best, r_now)
    ein = ei.cpu().numpy().reshape(-1, 4).sum(1)
    # split B and S (hi and lo halves, rows padded to 16) read by one split launch
    n16 = 16 * ((prob.npno.astype(np.int64) + 15) // 16)
    split_B = float((prob.naux.astype(np.int64) * prob.npno * n16 * prob.n_blocks().clip(0, 1)).sum()) * 2 * 2
    tgt = np.repeat(np.arange(prob.n_pairs), np.diff(prob.cpl_rowptr))
    split_S = float((prob.npno[tgt].astype(np.int64) * n16[prob.cpl_src]).sum()) * 2 * 2
    row = {"refinements": args.mixed_outer, "inner_iterations": args.mixed_inner,
           "kernel_ms": round(k_ms, 3), "ladder_ms": round(k_lad, 3), "projection_ms": round(k_proj, 3),
           "split_T_ms": round(conv_ms, 3),
           "achieved_tflops": round(flops / (k_ms / 1e3) / 1e12, 3),
           "mixed_solve_s": round(tm, 3), "vs_fp64_solve": round(tm / ref["seconds"], 3),
           "energy_mixed": float(etm.cpu()[0]),
           "total_energy_error": abs(float(etm.cpu()[0]) - ref["energy"]),
           "max_pair_energy_error": float(np.max(np.abs(emn - ref["e_pair"]))),
           "max_abs_R_mixed": float(rm.cpu()[0]),
           "gate_1e-7_pair_1e-6_total": bool(float(np.max(np.abs(emn - ref["e_pair"]))) <= 1e-7 and
                                             abs(float(etm.cpu()[0]) - ref["energy"]) <= 1e-6),
           "inner_only": {"iterations": n_in, "max_abs_R": r_now,
                          "total_energy_error": abs(float(eti.cpu()[0]) - ref["energy"]),
                          "max_pair_energy_error": float(np.max(np.abs(ein - ref["e_pair"])))},
           "other_schedules": others,
           "split_bytes_per_launch": split_B + split_S,
           "hbm_frac": round((split_B + split_S) / (k_ms / 1e3) / 8e12, 4)}
    log("mixed leg %s: %s" % (precision, row))
    mp.close()
    del Tm, Ti
    return row


def mixed_leg(prob, dev, eps_a, eps_b, args, flops, ref, log):
    """Split precisions with FP64 refinement against the converged FP64 solve."""
    out = {"fp64_solve_s": round(ref["seconds"], 3), "fp64_iterations": ref["iterations"],
           "energy_fp64": ref["energy"], "precisions": {}}
    for prec in args.mixed_precisions.split(","):
        out["precisions"][prec] = split_precision_row(prob, dev, eps_a, eps_b, prec, args, flops, ref, log)
    return out


def fp32_leg(prob, dev, eps_a, eps_b, args, fl_ladder, fl_proj, ref, log):
    """The plain FP32 path (FP32 MFMA contractions, FP64 dressing, update,
    energies and DIIS): time per iteration, the ladder launch against the
    FP32 peak, and the energies of the FP32 iteration run until max|R| stops
    falling, against the converged FP64 solve."""
    import numpy as np
    import torch

    from paper_2008_03237_amd import Plan
    p32 = Plan(prob, dev["B"], dev["S"], dev["K"], eps_a, eps_b, precision="fp32")
    T = torch.zeros(max(prob.n_T, 1), dtype=torch.float64, device="cuda")
    p32.iterate(2, T)
    torch.cuda.synchronize()
    p32.set_profiling(True)
    t0 = time.perf_counter()
    p32.iterate(args.steps, T)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) / max(args.steps, 1) * 1e3
    ms, cnt = p32.phase_times()
    p32.set_profiling(False)
    lad = ms[0] / max(cnt[0], 1)
    proj = ms[5] / max(cnt[5], 1)
    T.zero_()
    p32.reset()
    best, n_it, r_now = None, 0, None
    while n_it < 40:
        _, e32, et32, r32 = p32.iterate(2, T)
        n_it += 2
        r_now = float(r32.cpu()[0])
        if best is not None and r_now >= 0.5 * best:
            break
        best = r_now if best is None else min(best, r_now)
    e32n = e32.cpu().numpy().reshape(-1, 4).sum(1)
    row = {"ms_per_step": round(ms_step, 3), "value_gflops": round((fl_ladder + fl_proj) / (ms_step / 1e3) / 1e9, 2),
           "ladder_ms": round(lad, 3), "projection_ms": round(proj, 3),
           "ladder_tflops": round(fl_ladder / (lad / 1e3) / 1e12, 3),
           "ladder_frac_fp32_peak": round(fl_ladder / (lad / 1e3) / 1e12 / PEAK_TFLOPS["fp32"], 4),
           "iterations_to_stall": n_it, "max_abs_R": r_now,
           "total_energy_error": abs(float(et32.cpu()[0]) - ref["energy"]),
           "max_pair_energy_error": float(np.max(np.abs(e32n - ref["e_pair"])))}
    log("fp32 leg: %s" % row)
    p32.close()
    del T
    return row


def schedule_line(plan):
    """The tile-variant choice of the grouped kernel's work items (plan summary)."""
    for line in plan.info().splitlines():
        if line.startswith("ladder variants by tiles"):
            return line.strip()
    return ""


def _code_only(text):
    """C++ source without comments and blank-line/indent differences."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.strip() for line in text.splitlines() if line.strip())


def kernel_source_sha():
    """Hash of the grouped kernel's sources and of its schedule builder,
    comments left out: the HBM traffic record is used only while it describes
    this code."""
    import hashlib
    h = hashlib.sha256()
    for f in ("grouped_impl.h", "grouped_f64.hip", "grouped_f32.hip", "internal.h", "plan.hip", "plan_internal.h"):
        with open(os.path.join(ROOT, "paper_2008_03237_amd", "csrc", f)) as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def pno_source_sha():
    """Hash of the PNO kernels' source, comments left out (the counter record
    of the PNO leg is used only while it describes this code)."""
    import hashlib
    with open(os.path.join(ROOT, "paper_2008_03237_amd", "csrc", "pno.hip")) as fh:
        return hashlib.sha256(_code_only(fh.read()).encode()).hexdigest()[:16]


if __name__ == "__main__":
    main()
