"""Benchmark of the GCMe nonbonded hot path on one MI355X.

A step is one pass of the whole path: integrator half-kick/drift/noise, cell
binning and deterministic sort, excluded-volume pair kernel, smeared-Coulomb
real-space kernel, B-spline spreading, 3D FFT, Green's-function convolution,
inverse FFT, force gather and the second half-kick, replayed from a captured
HIP graph.  Workload: bulk electrolyte, N = 32768 beads at rho = 2.5, 20%
charged, two species, rc = 3, SPME 64^3 order 5, BAOAB Langevin at dt = 0.02
(synthetic seeded inputs; see gcme_workloads.config2).

Prints ONE JSON line.  `value` = unordered pairs within the cutoff per step
x steps per second (pair interactions/s).  ns/day uses tau = 3.18 ps (the
paper's four-to-one mapping).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

TAU_PS = 3.18

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
# VALU issue: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 instruction per SIMD
# every 4 cycles (16 lanes per cycle)
PEAK_VALU_GINSTR = 256 * 4 * 2.4 / 4  # = 614.4

# Algorithmic FP operations per unordered pair within the cutoff (both
# forces by Newton's third law): separation 3, r^2 5, exponent 1, exp 1,
# prefactor 1, force scale 1, force vector 3, +f_i 3, -f_j 3, energy 1.
FLOP_PER_GCM_PAIR = 22
# Distance test a neighbour search needs for each in-range pair it keeps:
# separation 3, r^2 5.
FLOP_PER_DISTANCE_TEST = 8
# Charged pair, real-space bracket: separation 3, r^2 5, sqrt 1, 1/r 1, two
# erfc 2, difference and scale 2, two Gaussians (2 mul + 2 exp) 4, bracket
# 4, force vector 3, +f_i 3, -f_j 3, z_i z_j lB 2, energy 1.
FLOP_PER_ELEC_PAIR = 35


# Default tuning per workload (cells_per_cutoff, beads_per_cluster,
# charges_per_cluster, direct_pairs, stream_layout, then optionally
# mesh_tile_x, mesh_tile_y, gather_tile_x, gather_tile_y, half_pairs; the
# form --tuning takes): the fastest measured on MI355X for that workload
# (the library's autotuner's pick, bench.py --autotune, or, for the
# 2,097,152-bead system, interleaved step timings of the candidates, which
# beat it), fixed so that every run, and the kernel traces under profiles/,
# time the same kernels.
DEFAULT_TUNING = {
    "bulk_N32768": "3,8,4,3,2",
    "bulk_N2097152": "2,8,8,1,0,4,4,8,4",
    "batched_256": "2,8,4,1,3,16,8,16,8",
}

# workload name -> its DEFAULT_TUNING key
DEFAULT_KEYS = {"bulk_N32768_mixed": "bulk_N32768", "bulk_N2097152": "bulk_N2097152"}

# stages of more than one kernel launch
MULTI_KERNEL_STAGES = {"sort"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--workload", default="bulk_N32768",
                    choices=["bulk_N32768", "bulk_N2097152", "batched_256", "slab_nonmetal", "slab_metal",
                             "polyelectrolyte_slab_nonmetal", "polyelectrolyte_slab_metal"],
                    help="the slab systems (the adsorption study's size, and the 200,000-bead "
                         "polyelectrolyte slab) and the 256 batched replicas time the step loop only")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the tuning with the library's autotuner (after the warm-up) instead of the "
                         "workload's default tuning")
    ap.add_argument("--tuning", default="",
                    help="cells_per_cutoff,beads_per_cluster,charges_per_cluster[,direct_pairs[,stream_layout"
                         "[,mesh_tile_x,mesh_tile_y[,gather_tile_x,gather_tile_y[,half_pairs]]]]] in place of "
                         "the workload's default tuning")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--timing-steps", type=int, default=20,
                    help="steps of the stage-timing pass (HIP event nodes in the step graph)")
    ap.add_argument("--isolated-stages", action="store_true",
                    help="also time each stage alone (replays of that stage only)")
    ap.add_argument("--profile-reps", type=int, default=20)
    ap.add_argument("--steps-only", action="store_true",
                    help="only the timed step loop (for profiler runs)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the FP64, 2M-bead and batched-replica measurements")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one plain device copy of this size and exit (HBM counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU runs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    if args.copy_calib_mib:
        n = args.copy_calib_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes_each_way": n * 4}))
        return

    import gcme_workloads as W
    from paper_2403_08148_amd import GCMe, params_from_workload

    slab = args.workload.startswith("slab") or args.workload.startswith("polyelectrolyte")
    if args.workload == "batched_256":
        ws = W.config5()
        eng, _ = engine_for(ws, args.precision, tune=False)
        w = ws[0]
        slab = True  # the step loop only
    elif slab:
        metal = args.workload.endswith("_metal")
        w = W.paper_slab(metal=metal) if args.workload.startswith("slab") else W.polyelectrolyte_slab(metal=metal)
        eng, _ = engine_for([w], args.precision, tune=False)
    else:
        w = W.config2() if args.workload == "bulk_N32768" else W.config4()
        eng = GCMe([w.N], precision=args.precision, seed=12345)
        eng.set_params(params_from_workload(w))
        eng.set_state(w.pos, w.type, w.z, w.vel)
    tun_s = args.tuning or DEFAULT_TUNING.get(args.workload, "")
    if tun_s and not args.autotune:
        apply_tuning(eng, tun_s)

    # warm-up (also relaxes the random start a little); the first run of
    # steps captures every step graph a later run replays
    eng.step(args.warmup)
    eng.sync()
    if args.autotune:
        eng.autotune()
    # capture the step graphs if the autotuner's tuning dropped them, so that
    # no graph is built inside the timed region
    eng.step(0)
    eng.sync()
    tuning = eng.tuning()
    pairs0 = eng.count_pairs()
    torch.cuda.synchronize()
    stream = eng.stream  # the stream every kernel of the engine runs on
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    eng.step(args.steps)
    e1.record(stream)
    eng.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    pairs1 = eng.count_pairs()
    pairs = 0.5 * (pairs0 + pairs1)
    steps_per_s = 1000.0 / ms_step
    value = pairs * steps_per_s
    ns_day = steps_per_s * w.dt * TAU_PS * 86400.0 / 1000.0
    if args.steps_only or slab:
        print(json.dumps({"workload": args.workload if args.workload == "batched_256" else w.name,
                          "n_beads": eng.N, "ms_per_step": ms_step, "pairs": pairs,
                          "pair_interactions_per_s": value, "tuning": tuning}))
        return

    # per-stage device times inside real steps: each one-kernel stage's
    # execution span in the step graph, from the kernels' own wavefront
    # start/end stamps
    stages = eng.time_stages(args.timing_steps)
    eng.sync()
    isolated = None
    if args.isolated_stages:
        isolated = eng.profile_step(args.profile_reps)
        eng.sync()
    nq = int((w.z != 0).sum())
    obs = eng.step(1, observe=True)
    eng.sync()
    E = obs["energy"].cpu().numpy()[0]

    # charged pairs within the cutoff at the final positions (for the
    # charged-pair stages' algorithmic counts)
    cc_pairs = charged_pairs(eng, w)
    direct = tuning.get("direct_pairs", 0)
    stage_roof = stage_rooflines(w, stages, tuning, pairs, cc_pairs, nq, args.precision)
    # the dominant kernel: the longest stage that is one kernel launch (the
    # sort stage is four)
    dom = max((k for k in stage_roof if k not in MULTI_KERNEL_STAGES), key=lambda k: stages[k])
    roof = dict(stage_roof[dom])
    roof["launch_us"] = stages[dom] * 1e3
    roof["launch_us_source"] = (f"mean over {args.timing_steps} steps of the kernel's execution span in the step "
                                f"graph: first wavefront start to last wavefront end on the GPU's real-time counter "
                                f"(gcme_time_stages)")
    prof = profiled_launch_us(dom, tuning, args.workload)
    if prof is not None:
        roof["launch_us_rocprof"] = prof
    roof["traffic"] = measured_traffic(dom, tuning) if args.precision == "mixed" else None
    vi = measured_valu(dom, tuning) if args.precision == "mixed" else None
    if vi is not None:
        ach = vi / (stages[dom] * 1e-3) / 1e9
        roof["valu_issue"] = {"instr_per_launch": vi, "achieved": ach, "peak": PEAK_VALU_GINSTR,
                              "unit": "G wave-instr/s", "frac": ach / PEAK_VALU_GINSTR}
    # the excluded-volume pair kernel's own figure is always reported
    gcm_tflops = stage_roof["pair_gcm"]["achieved"]

    # mixed-precision forces against the plain FP64 GPU form at the same state
    # (the initial positions), then the other workloads
    extras = None
    if not args.no_extras:
        eng.close()
        extras = extra_workloads(w)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, pairs)

    out = {
        "metric": "pair interactions/s (N=32k bulk GCMe, rc=3, SPME 64^3) + ns/day",
        "value": value,
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n_beads": w.N, "density": 2.5, "charged_fraction": float(nq) / w.N,
                   "cutoff": w.rc, "beta": w.beta, "pme_grid": list(w.grid), "order": w.order, "dt": w.dt,
                   "integrator": "BAOAB Langevin", "precision": args.precision, "tuning": tuning},
        "ns_per_day": ns_day,
        "tau_per_day": steps_per_s * w.dt * 86400.0,  # simulated time in the paper's reduced unit tau
        "steps_per_s": steps_per_s,
        "pairs_within_cutoff": pairs,
        "wall_s_timed": wall,
        "stage_ms": stages,
        "stage_ms_isolated": isolated,
        "pair_gcm_tflops": gcm_tflops,
        "charged_pairs_within_cutoff": cc_pairs,
        "stage_roofline": stage_roof,
        "energy_terms_last_step": {k: float(v) for k, v in zip(
            ["ex", "real", "recip", "corr", "self", "pot", "kin"], E)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extras,
    }
    print(json.dumps(out), flush=True)
    if args.no_extras:
        eng.close()


def stage_rooflines(w, stages, tuning, pairs, cc_pairs, nq, precision):
    """Each one-kernel stage's achieved rate against its bound: algorithmic
    work per launch (FLOP for the pair kernels, bytes for the others; the
    kernels table of the design notes) over the stage's measured launch
    time."""
    K = w.grid
    nch = K[0] * K[1] * (K[2] // 2 + 1)
    cs = 16 if precision == "fp64" else 8
    peak_alu = PEAK_FP64_TFLOPS if precision == "fp64" else PEAK_FP32_TFLOPS
    # a list-free pair kernel does its neighbour search itself: its stage
    # carries the distance tests too (and the list stage is empty)
    direct = tuning.get("direct_pairs", 0)
    half = tuning.get("half_pairs", 0)
    search_g = (direct & 1) or (half & 3)
    search_q = (direct & 2) or (half >> 2) & 3
    gcm_flop = FLOP_PER_GCM_PAIR + (FLOP_PER_DISTANCE_TEST if search_g else 0)
    elec_flop = FLOP_PER_ELEC_PAIR + (FLOP_PER_DISTANCE_TEST if search_q else 0)
    alg = {
        "int_first": ("hbm", w.N * (12 + 24 + 24 + 12 + 24 + 24)),
        "sort": ("hbm", w.N * (12 + 4 + 4 + 12 + 24 + 4 + 4 + 12 + 24 + 4 + 4 + 16)),
        "list_gcm": ("alu", FLOP_PER_DISTANCE_TEST * pairs),
        "pair_gcm": ("alu", gcm_flop * pairs),
        "list_elec": ("alu", FLOP_PER_DISTANCE_TEST * cc_pairs),
        "pair_elec": ("alu", elec_flop * cc_pairs),
        "spread_z": ("hbm", nq * 16 + nch * cs),
        "fft_y": ("hbm", 2 * nch * cs),
        "fft_conv": ("hbm", 2 * nch * cs),
        "fft_y_inv": ("hbm", 2 * nch * cs),
        "z_gather": ("hbm", nch * cs + nq * (16 + 4 + 24)),
        "int_last": ("hbm", w.N * (12 + 24 + 24 + 12 + 24 + 4)),
    }

    def roof_of(name):
        bound, amount = alg[name]
        t = stages[name] * 1e-3
        if t <= 0:
            return None
        if bound == "alu":
            ach = amount / t / 1e12
            return {"bound": "alu", "kernel": name, "achieved": ach, "peak": peak_alu, "unit": "TFLOP/s",
                    "frac": ach / peak_alu, "launch_us": stages[name] * 1e3}
        ach = amount / t / 1e9
        return {"bound": "hbm", "kernel": name, "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": ach / PEAK_HBM_GBS, "launch_us": stages[name] * 1e3}

    # list stages of list-free pairs are empty; with column clusters the list
    # stage is the column pass (not an algorithmic step of its own)
    skip = {"list_gcm"} if search_g else set()
    skip |= {"list_elec"} if search_q else set()
    return {k: roof_of(k) for k in stages if k in alg and stages[k] > 0 and k not in skip}


def time_steps(eng, steps, warmup):
    """ms per graph-replayed step on the engine's stream (HIP events)."""
    import torch
    eng.step(warmup)
    eng.sync()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(eng.stream)
    eng.step(steps)
    e1.record(eng.stream)
    eng.sync()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def apply_tuning(eng, tun_s):
    """Set a tuning given in the form --tuning takes; returns the engine's
    tuning."""
    v = [int(x) for x in tun_s.split(",")]
    eng.set_tuning(cells_per_cutoff=v[0], beads_per_cluster=v[1], charges_per_cluster=v[2],
                   direct_pairs=v[3] if len(v) > 3 else -1, stream_layout=v[4] if len(v) > 4 else -1,
                   mesh_tile_x=v[5] if len(v) > 6 else -1, mesh_tile_y=v[6] if len(v) > 6 else -1,
                   gather_tile_x=v[7] if len(v) > 8 else -1, gather_tile_y=v[8] if len(v) > 8 else -1,
                   half_pairs=v[9] if len(v) > 9 else -1)
    return eng.tuning()


def engine_for(ws, precision, tune=True, kmax=0.0):
    """An engine over the workloads (kmax > 0: the exact reciprocal sum over
    |k| <= kmax in place of the mesh)."""
    from paper_2403_08148_amd import GCMe, params_from_workload
    from paper_2403_08148_amd import _binding as B
    import numpy as np
    eng = GCMe([x.N for x in ws], precision=precision, seed=12345)
    off, bonds, images = 0, [], []
    for r, x in enumerate(ws):
        ex = x.extra
        over = dict(kmax=kmax)
        if ex.get("slab"):
            over["flags"] = B.GCME_FLAG_SLAB_CORRECTION
        if "bonds" in ex:
            over.update(bond_k=ex["bond_k"], bond_b=ex["bond_b"])
            bonds.append(ex["bonds"] + off)
        if len(ex.get("images", ())):
            images.append(ex["images"] + off)
        eng.set_params(params_from_workload(x, **over), replica=r)
        off += x.N
    if bonds:
        eng.set_bonds(np.concatenate(bonds))
    if images:
        eng.set_images(np.concatenate(images))
    eng.set_state(np.concatenate([x.pos for x in ws]), np.concatenate([x.type for x in ws]),
                  np.concatenate([x.z for x in ws]), np.concatenate([x.vel for x in ws]))
    tuning = eng.autotune() if tune else eng.tuning()
    return eng, tuning


def extra_workloads(w):
    """The plain FP64 form of the same workload, the 2,097,152-bead bulk
    system (mixed and FP64), 256 batched replicas against one engine per
    replica called in sequence, the 200,000-bead system with the
    polyelectrolyte workload's composition and mesh (periodic), and the
    1,536-bead plain-method system with the exact reciprocal sum against its
    mesh form, and the adsorption study's slab systems (nonmetal and metal
    electrodes) at its size."""
    import numpy as np
    import gcme_workloads as W
    out = {}

    def forces(eng):
        f = eng.forces_energy(energy=False, virial=False)["force"]
        eng.sync()
        return f.double().cpu().numpy()

    # 1. same workload, plain FP64 GPU form (autotuned; mixed at the
    #    headline's default tuning); mixed force error against it
    res = {}
    fr = {}
    for prec in ("mixed", "fp64"):
        eng, tun = engine_for([w], prec, tune=prec != "mixed" or w.name not in DEFAULT_KEYS)
        if prec == "mixed" and w.name in DEFAULT_KEYS:
            tun = apply_tuning(eng, DEFAULT_TUNING[DEFAULT_KEYS[w.name]])
        fr[prec] = forces(eng)
        ms = time_steps(eng, 200, 20)
        res[prec] = {"ms_per_step": ms, "tuning": tun}
        eng.close()
    res["mixed_force_rel_rms_vs_fp64"] = float(np.linalg.norm(fr["mixed"] - fr["fp64"]) / np.linalg.norm(fr["fp64"]))
    out[w.name] = res

    # 2. N = 2,097,152 bulk, mixed (its default tuning, at which the
    #    committed profiles are taken) and FP64 (autotuned)
    w4 = W.config4()
    res = {}
    fr = {}
    for prec in ("mixed", "fp64"):
        eng, tun = engine_for([w4], prec, tune=prec != "mixed")
        if prec == "mixed":
            tun = apply_tuning(eng, DEFAULT_TUNING["bulk_N2097152"])
        fr[prec] = forces(eng)
        ms = time_steps(eng, 40, 5)
        pairs = eng.count_pairs()
        res[prec] = {"ms_per_step": ms, "pair_interactions_per_s": pairs * 1000.0 / ms,
                     "ns_per_day": 1000.0 / ms * w4.dt * TAU_PS * 86400.0 / 1000.0, "pairs_within_cutoff": pairs,
                     "tuning": tun}
        if prec == "mixed":
            # every kernel of the step against its bound (as for the headline)
            st = eng.time_stages(3)
            eng.sync()
            nq4 = int((w4.z != 0).sum())
            res[prec]["stage_ms"] = st
            res[prec]["stage_roofline"] = stage_rooflines(w4, st, tun, pairs, charged_pairs(eng, w4), nq4, prec)
            prof = profiled_launch_us("pair_gcm", tun, w4.name)
            if prof is not None and res[prec]["stage_roofline"].get("pair_gcm"):
                res[prec]["stage_roofline"]["pair_gcm"]["launch_us_rocprof"] = prof
        eng.close()
    res["mixed_force_rel_rms_vs_fp64"] = float(np.linalg.norm(fr["mixed"] - fr["fp64"]) / np.linalg.norm(fr["fp64"]))
    out[w4.name] = res

    # 3. 256 batched replicas (one engine, one graph per step) against the
    #    same replicas each in its own engine, stepped one after another
    ws = W.config5()
    eng, _ = engine_for(ws, "mixed", tune=False)
    tun = apply_tuning(eng, DEFAULT_TUNING["batched_256"])
    ms_b = time_steps(eng, 100, 10)
    pairs = eng.count_pairs()
    eng.close()
    ms_seq = 0.0
    for x in ws:
        e1, _ = engine_for([x], "mixed", tune=False)
        ms_seq += time_steps(e1, 20, 3)
        e1.close()
    out["batched_256_replicas"] = {"n_beads": int(sum(x.N for x in ws)), "ms_per_step": ms_b,
                                   "pair_interactions_per_s": pairs * 1000.0 / ms_b,
                                   "sequential_ms_per_step": ms_seq, "speedup_vs_sequential": ms_seq / ms_b,
                                   "tuning": tun}

    # 4. the polyelectrolyte workload's composition, box and mesh as a
    #    periodic bulk box (N = 200,000, 50% charged, SPME 96 x 96 x 128)
    w3 = W.config3()
    res = {}
    fr = {}
    for prec in ("mixed", "fp64"):
        eng, tun = engine_for([w3], prec)
        fr[prec] = forces(eng)
        ms = time_steps(eng, 50, 5)
        pairs = eng.count_pairs()
        res[prec] = {"ms_per_step": ms, "pair_interactions_per_s": pairs * 1000.0 / ms,
                     "ns_per_day": 1000.0 / ms * w3.dt * TAU_PS * 86400.0 / 1000.0, "pairs_within_cutoff": pairs,
                     "tuning": tun}
        eng.close()
    res["mixed_force_rel_rms_vs_fp64"] = float(np.linalg.norm(fr["mixed"] - fr["fp64"]) / np.linalg.norm(fr["fp64"]))
    out[w3.name] = res

    # 5. the plain-method configuration (N = 1536) with the reciprocal sum
    #    taken exactly over |k| <= 8, against the same system on its 32^3 mesh
    w1 = W.config1()
    res = {}
    fr = {}
    for prec in ("fp64", "mixed"):
        for mode, km in (("exact_k_sum", w1.kmax), ("spme_32", 0.0)):
            eng, tun = engine_for([w1], prec, kmax=km)
            fr[(prec, mode)] = forces(eng)
            res[f"{prec}_{mode}"] = {"ms_per_step": time_steps(eng, 200, 20), "tuning": tun}
            eng.close()
    fx = fr[("fp64", "exact_k_sum")]
    res["mixed_force_rel_rms_vs_fp64_exact"] = float(np.linalg.norm(fr[("mixed", "exact_k_sum")] - fx) /
                                                     np.linalg.norm(fx))
    res["spme_force_rel_rms_vs_exact_fp64"] = float(np.linalg.norm(fr[("fp64", "spme_32")] - fx) / np.linalg.norm(fx))
    res["kmax"] = w1.kmax
    out[w1.name] = res

    # 6. the adsorption study's slab systems at its size, and the
    #    200,000-bead polyelectrolyte slab (2,000 chains of 50, counterions,
    #    solvent): nonmetal electrodes (slab correction, box tripled) and
    #    metal electrodes (image charges, box doubled), with bonded chains
    #    and fixed electrode lattices
    for ws6 in (W.paper_slab(metal=False), W.paper_slab(metal=True), W.polyelectrolyte_slab(metal=False),
                W.polyelectrolyte_slab(metal=True)):
        res = {"n_beads": ws6.N, "n_mobile": int((ws6.type == 0).sum()), "box": list(ws6.box),
               "grid": list(ws6.grid), "bonds": int(len(ws6.extra["bonds"])),
               "images": int(len(ws6.extra["images"]))}
        for prec in ("mixed", "fp64"):
            eng, tun = engine_for([ws6], prec)
            ms = time_steps(eng, 50, 5)
            pairs = eng.count_pairs()
            res[prec] = {"ms_per_step": ms, "pair_interactions_per_s": pairs * 1000.0 / ms,
                         "ns_per_day": 1000.0 / ms * ws6.dt * TAU_PS * 86400.0 / 1000.0,
                         "pairs_within_cutoff": pairs, "tuning": tun}
            eng.close()
        out[ws6.name] = res
    return out


def charged_pairs(eng, w):
    """Unordered charged pairs with r < rc at the engine's current positions
    (scipy KD tree on the host)."""
    import numpy as np
    from scipy.spatial import cKDTree
    pos, _, _ = eng.get_state()
    eng.sync()
    p = pos.t().cpu().numpy()
    q = np.mod(p[w.z != 0], w.box)
    return int(len(cKDTree(q, boxsize=w.box).query_pairs(w.rc)))


def code_digest(text):
    """sha256 of source text without // comments, blank lines and repeated
    whitespace: changes when the code changes, not when a comment does."""
    import hashlib
    import re
    lines = []
    for line in text.split("\n"):
        line = re.sub(r"//.*", "", line).strip()
        if line:
            lines.append(" ".join(line.split()))
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()


def pair_gcm_key(tuning):
    """What selects the excluded-volume pair kernel: the cell size, the
    cluster size, the list choice and the column-cluster mode."""
    return (f"{tuning['cells_per_cutoff']},{tuning['beads_per_cluster']},{tuning.get('direct_pairs', 0) & 1},"
            f"{tuning.get('half_pairs', 0) & 3}")


def measured_traffic(stage, tuning):
    """HBM bytes per launch of a stage from committed rocprofv3 counter runs
    (profiles/traffic_<stage>.json: FETCH_SIZE and WRITE_SIZE in KiB per
    dispatch for the kernel under each measured tuning, each scaled by what the
    counter reads for a plain device copy of known size), or None when no run
    matches the tuning or the kernel source changed since the runs."""
    path = os.path.join(ROOT, "profiles", f"traffic_{stage}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    with open(os.path.join(ROOT, t["source"])) as f:
        if code_digest(f.read()) != t["source_code_sha256"]:
            return None
    key = pair_gcm_key(tuning)
    run = next((r for r in t["runs"] if r["key"] == key), None)
    if run is None:
        return None
    cb = float(t["copy_bytes"])
    fetch = run["fetch_kib"] * 1024.0 * cb / (t["copy_fetch_kib"] * 1024.0)
    write = run["write_kib"] * 1024.0 * cb / (t["copy_write_kib"] * 1024.0)
    return fetch + write


def profiled_launch_us(stage, tuning, workload):
    """The committed rocprofv3 kernel-trace mean duration (us) of the stage's
    kernel for this workload and tuning (profiles/launch_<stage>.json), or
    None when none matches or the kernel source changed since the trace."""
    path = os.path.join(ROOT, "profiles", f"launch_{stage}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    with open(os.path.join(ROOT, t["source"])) as f:
        if code_digest(f.read()) != t["source_code_sha256"]:
            return None
    key = ",".join(str(tuning[k]) for k in ("cells_per_cutoff", "beads_per_cluster", "charges_per_cluster",
                                            "direct_pairs", "stream_layout", "mesh_tile_x", "mesh_tile_y",
                                            "gather_tile_x", "gather_tile_y", "half_pairs"))
    run = next((r for r in t["runs"] if r["key"] == key and r["workload"] == workload), None)
    return None if run is None else float(run["mean_us"])


def measured_valu(stage, tuning):
    """VALU wavefront instructions per launch of a stage's kernel from the
    committed counter runs (profiles/valu_<stage>.json), or None when no run
    matches the tuning or the kernel source changed since the runs."""
    path = os.path.join(ROOT, "profiles", f"valu_{stage}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    with open(os.path.join(ROOT, t["source"])) as f:
        if code_digest(f.read()) != t["source_code_sha256"]:
            return None
    key = pair_gcm_key(tuning)
    run = next((r for r in t["runs"] if r["key"] == key), None)
    return None if run is None else float(run["valu_instr"])


def cpu_baseline(w, pairs, budget_s=15.0):
    """The FP64 oracle (cell-list real space + SPME on the same mesh, BAOAB
    steps) run on the host cores for a bounded number of MD steps of the same
    workload (~budget_s seconds), reported in the same unit."""
    from oracle import oracle as O
    O.build(force=False)
    p = O.Params(w.box, w.rc, w.beta, w.lB, w.A, w.sigma, w.a)
    t0 = time.perf_counter()
    O.forces(w.pos, w.type, w.z, p, recip_mode=O.RECIP_SPME, K=w.grid, order=w.order)
    t_eval = time.perf_counter() - t0
    n = int(max(3, min(200, budget_s / max(t_eval, 1e-3))))
    import numpy as np
    ids = np.arange(w.N, dtype=np.int32)
    t0 = time.perf_counter()
    O.md(w.pos, w.vel, w.type, w.z, ids, p, w.mass, w.dt, w.gamma, w.kT, 12345, 0, 0, n,
         recip_mode=O.RECIP_SPME, K=w.grid, order=w.order)
    dt = time.perf_counter() - t0
    # md() evaluates the forces once before its loop, so n + 1 evaluations
    sps = n / dt
    return {"value": pairs * sps, "unit": "pair interactions/s", "cores": O.num_threads(), "kind": "oracle",
            "steps_per_s": sps,
            "sample": f"{n} BAOAB steps (+1 initial force evaluation) of {w.name} ({w.N} beads) "
                      f"on the host, {dt:.1f} s"}


if __name__ == "__main__":
    main()
