#!/usr/bin/env python3
"""Throughput of the ring-polymer MD hot path on one MI355X.

Workload: 4,096 flexible 3-site waters (12,288 atoms) in a 49.7 A cube, rc 9 A, SPME 64^3
order 5, P = 32 beads, 300 K, dt 0.5 fs: one step = normal-mode BAOAB + centroid-list
check/rebuild + bonded + real-space pairs + SPME on all 32 beads. The headline `value` is
the bead-batched path with FP32 pair forces (ns/day); the plain path (one launch per bead,
all FP64) and the batched FP64 path are timed beside it on the same input. Inputs are
seeded and synthetic and resident on the GPU before the timed region starts.

    python bench.py [--gpus 1] [--steps 1000] [--warmup 20]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
FP64_VECTOR_PEAK_TFLOPS = 78.6

# Algorithmic work per launch of each kernel class (the unit counts behind the roofline).
#   pair   : FP32 flops; 30 per in-range pair-bead interaction (each pair once) and 8 per
#            centroid-list candidate pair-bead test
#   spread : bytes; bead positions read once + every grid value written once
#   fft    : bytes; the grid read once and written once for the whole forward transform,
#            influence-function product and inverse transform (the kernels make three
#            read + write passes, so the achieved figure is against that minimum)
#   gather : bytes; grid read once + positions read + gradient read and written
#   nm     : bytes; Q, P, grad V read, Q, P, x and the FP32 offsets written
FLOPS_PER_PAIR = 30.0
FLOPS_PER_CANDIDATE = 8.0


def measured_traffic(cls):
    """HBM bytes per launch of the class's kernel from the committed FETCH_SIZE / WRITE_SIZE
    counter record (profiles/traffic_<class>_water4096_P32.json), scaled by the copy
    calibration; None when there is no record or the kernel's sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{cls}_water4096_P32.json")
    if not os.path.exists(path):
        return None, None, None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec["source_sha256"]:
        return None, "kernel sources changed since the counters were taken", None
    b = (rec["fetch_size_kib_per_dispatch"] * 1024 * rec["fetch_scale"]
         + rec["write_size_kib_per_dispatch"] * 1024 * rec["write_scale"])
    return b, os.path.relpath(path, ROOT), rec.get("l2_hit_rate")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--plain-steps", type=int, default=None,
                    help="steps for the plain FP64 comparison (default: --steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip plain and batched FP64")
    ap.add_argument("--breakdown", action="store_true", help="print per-kernel-class times")
    ap.add_argument("--no-graph", action="store_true", help="launch kernels instead of graphs")
    ap.add_argument("--windows", action="store_true",
                    help="only the 16-window free-energy workload (one JSON line)")
    ap.add_argument("--adqtb", action="store_true",
                    help="only the 21,952-water adQTB workload (one JSON line)")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="for hardware counters: a 256 MiB device copy (calibration), then "
                         "--steps launched steps of the batched FP32-pair path; no JSON")
    return ap.parse_args()


def pair_counts(s):
    """In-range pair-bead interactions (each pair once) and candidate pair-bead tests of the
    initial configuration, from a periodic k-d tree on every bead."""
    import numpy as np
    from scipy.spatial import cKDTree
    L = float(s.box[0])
    mol = np.arange(s.n_atoms) // 3
    inrange = 0
    for b in range(s.n_beads):
        w = np.mod(s.pos[b], L)
        w[w >= L] = 0.0
        pr = cKDTree(w, boxsize=L).query_pairs(s.cutoff, output_type="ndarray")
        inrange += int(np.count_nonzero(mol[pr[:, 0]] != mol[pr[:, 1]]))
    c = s.pos.mean(axis=0)
    w = np.mod(c, L)
    w[w >= L] = 0.0
    pr = cKDTree(w, boxsize=L).query_pairs(s.cutoff + s.skin, output_type="ndarray")
    cand = int(np.count_nonzero(mol[pr[:, 0]] != mol[pr[:, 1]])) * s.n_beads
    return inrange, cand


def algorithmic_work(cls, s, counts):
    N, P = s.n_atoms, s.n_beads
    K = s.pme_grid
    grid = K[0] * K[1] * K[2] * P * 8           # bytes of all bead grids (FP64)
    xb = 3 * N * P * 8
    if cls == "pair":
        inr, cand = counts
        return "flops", FLOPS_PER_PAIR * inr + FLOPS_PER_CANDIDATE * cand
    if cls == "spread":
        return "bytes", xb + grid
    if cls == "fft":
        return "bytes", 2 * grid
    if cls == "gather":
        return "bytes", grid + xb + 2 * xb
    if cls == "nm":
        return "bytes", 6 * xb + N * P * 16
    raise ValueError(cls)


def phase_rooflines(s, per_class, counts, ms_step):
    """Each timed kernel class against its own roofline (algorithmic work per step / its
    measured time per step), and the step's roofline time: the sum over the classes of
    work / peak, against the measured step."""
    phases, t_roof = {}, 0.0
    for cl, ms in per_class.items():
        kind, work = algorithmic_work(cl, s, counts)
        sec = ms * 1e-3
        if kind == "bytes":
            ach, peak, unit, bound = work / sec / 1e9, HBM_PEAK_GBS, "GB/s", "hbm"
            t_roof += work / (HBM_PEAK_GBS * 1e9)
        else:
            ach, peak, unit, bound = (work / sec / 1e12, FP32_VECTOR_PEAK_TFLOPS, "TFLOP/s",
                                      "alu")
            t_roof += work / (FP32_VECTOR_PEAK_TFLOPS * 1e12)
        phases[cl] = {"bound": bound, "ms_per_step": ms, "work": work,
                      "work_unit": "bytes" if kind == "bytes" else "flops",
                      "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak}
    step = {"t_roof_ms": t_roof * 1e3, "t_measured_ms": ms_step, "frac": t_roof * 1e3 / ms_step,
            "note": "roofline time of the five kernel classes (list, bonded and set-up kernels "
                    "carry little algorithmic work) against the whole measured step"}
    return phases, step


def force_loss_timing(q, qa, n_configs=8):
    """Differentiation workload: 1,024-water P=16 configurations, loss = mean squared force
    error against the forces of perturbed parameters, gradient with respect to the charges
    and LJ parameters by the library's mixed derivatives (torch autograd, device tensors)."""
    import torch
    import synth
    boxes = [synth.diff_box(k) for k in range(n_configs)]
    s0 = boxes[0]
    qp, sp, ep = synth.perturbed_parameters(s0, 1)
    ref = q.Context.from_system(s0, charge=qp, lj_sigma=sp, lj_epsilon=ep, precision=q.FP32_PAIRS)
    c = q.Context.from_system(s0, precision=q.FP32_PAIRS)
    dev = torch.device("cuda")
    refs = [torch.tensor(ref.eval(b.pos)[1], device=dev) for b in boxes]
    ref.close()
    prm = [torch.tensor(v, dtype=torch.float64, device=dev, requires_grad=True)
           for v in (s0.charge, s0.lj_epsilon, s0.lj_sigma)]

    def one(b, Fr):
        pos = torch.tensor(b.pos, dtype=torch.float64, device=dev, requires_grad=True)
        F = qa.forces(c, pos, *prm)
        loss = ((F - Fr) ** 2).mean()
        return torch.autograd.grad(loss, prm)

    one(boxes[0], refs[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b, Fr in zip(boxes, refs):
        one(b, Fr)
    torch.cuda.synchronize()
    dt_cfg = (time.perf_counter() - t0) / n_configs
    c.close()
    return {"workload": "1,024 waters, 31.3 A, P=16, SPME 32^3 order 5; loss = mean squared "
                        "force error vs perturbed parameters (charges +-5%, sigma/epsilon +-3%)",
            "ms_per_configuration": dt_cfg * 1e3, "configurations_timed": n_configs,
            "projected_64_configurations_s": 64 * dt_cfg,
            "calls_per_configuration": "forces (eval), mixed parameter derivatives + H v (hvp), "
                                       "parameter gradients (param_grad)"}


def windows_timing(q, steps=20, warmup=3):
    """The batched free-energy workload: 16 alchemical windows lambda = i/15 of the 12-atom
    solute in 256-2,048 waters with P = 8/16/32 (780-6,156 atoms each), FP32 pairs, each
    window's launch shapes picked by qhp_autotune, stepped as one group (one captured
    graph per step of all windows, one branch per window). Also: the same windows stepped
    one after another (each its own graph per step), and the cost of one sample of the BAR
    inputs (every window's bead energies at its two neighbours' couplings)."""
    import torch
    import synth
    systems = [synth.alchemical_window(i) for i in range(16)]
    ctxs = [q.Context.from_system(s, precision=q.FP32_PAIRS) for s in systems]
    try:
        for c, s in zip(ctxs, systems):
            c.set_state(s.pos, s.vel, 0)
        tiles = [c.autotune(5) for c in ctxs]
        bead_atoms = sum(s.n_atoms * s.n_beads for s in systems)
        with q.Group(ctxs) as g:
            g.step(warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.step(steps)
            torch.cuda.synchronize()
            t_group = time.perf_counter() - t0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c in ctxs:
            c.step(steps)
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t0
        lam = [i / 15 for i in range(16)]
        pos = [c.get_state()[0] for c in ctxs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, c in enumerate(ctxs):
            for j in (i - 1, i + 1):
                if 0 <= j < 16:
                    c.eval_lambda(pos[i], max(0.0, 2 * lam[j] - 1), min(1.0, 2 * lam[j]),
                                  forces=False)
        t_bar = time.perf_counter() - t0
    finally:
        for c in ctxs:
            c.close()
    return {"windows": 16, "atoms": [s.n_atoms for s in systems],
            "beads": [s.n_beads for s in systems], "bead_atoms_total": bead_atoms,
            "autotuned": tiles,
            "autotuned_fields": ["spread_beads", "spread_z_tiles", "yz_plane_slots",
                                 "pair_atoms_per_block"],
            "group_ms_per_step": t_group / steps * 1e3,
            "group_bead_atom_steps_per_s": bead_atoms * steps / t_group,
            "sequential_ms_per_step": t_seq / steps * 1e3,
            "group_speedup_vs_sequential": t_seq / t_group,
            "bar_sample_ms": t_bar * 1e3, "steps": steps,
            "note": "FP32 pairs (rc 7.8 A so that 2 (rc + skin) stays below the 19.7 A "
                    "edge of the 256-water boxes); BAR sample = 30 evaluations at the "
                    "neighbouring couplings from host positions"}


def adqtb_timing(q, stream):
    """The adQTB workload: 21,952 waters (65,856 atoms), 87.3 A cube, P = 1, FP32 pairs,
    128^3 grid, gamma0 20 /ps, 1,024-step segments. Two full segments from step 0 (each
    ends with the spectra, the gamma adaptation and the next segment's coloured noise),
    then 500 steps inside a segment; the difference prices the segment-end work."""
    import torch
    import synth
    s = synth.adqtb_box()
    c = q.Context.from_system(s, precision=q.FP32_PAIRS, thermostat=q.ADQTB, stream=stream)
    try:
        c.set_state(s.pos, s.vel, 0)
        shapes = c.autotune(3)
        c.set_state(s.pos, s.vel, 0)
        nseg = s.qtb_nseg
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.step(2 * nseg)
        torch.cuda.synchronize()
        t_seg = time.perf_counter() - t0
        t0 = time.perf_counter()
        c.step(500)
        torch.cuda.synchronize()
        t_in = time.perf_counter() - t0
    finally:
        c.close()
    # the same box on a 112^3 grid (0.78 A spacing: grid edges that are not powers of two
    # take the plain transform path), 300 steps inside the first segment
    import dataclasses
    s112 = dataclasses.replace(s, pme_grid=(112, 112, 112))
    c = q.Context.from_system(s112, precision=q.FP32_PAIRS, thermostat=q.ADQTB, stream=stream)
    try:
        c.set_state(s112.pos, s112.vel, 0)
        c.autotune(3)
        c.set_state(s112.pos, s112.vel, 0)
        c.step(10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.step(300)
        torch.cuda.synchronize()
        ms_112 = (time.perf_counter() - t0) / 300 * 1e3
    finally:
        c.close()
    ms = t_seg / (2 * nseg) * 1e3
    ms_in = t_in / 500 * 1e3
    return {"workload": "water21952_adqtb: 21,952 waters, 87.3 A, P=1, rc 9 A, SPME 128^3 "
                        "order 5, gamma0 20 /ps, N_seg 1,024, FP32 pairs",
            "steps": 2 * nseg, "ms_per_step": ms,
            "ns_per_day": s.dt * 86400e-6 / (ms * 1e-3),
            "atom_steps_per_s": s.n_atoms / (ms * 1e-3),
            "ms_per_step_inside_a_segment": ms_in,
            "segment_end_ms": (ms - ms_in) * nseg,
            "autotuned": dict(zip(("spread_beads", "spread_z_tiles", "yz_plane_slots",
                                   "pair_atoms_per_block"), shapes)),
            "grid_112": {"ms_per_step_inside_a_segment": ms_112, "steps": 300,
                         "note": "SPME 112^3 (0.78 A spacing), the plain path for grid "
                                 "edges that are not powers of two"}}


def cpu_baseline(s, budget_s=20.0):
    """The oracle as it stands, on a bounded sample: the centroid pair list and the full
    per-bead potential of as many beads as fit in about `budget_s` seconds."""
    import resource
    from oracle import forces as ofo
    t0 = time.perf_counter()
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    pairs = ofo.pair_list(ofo.centroids_of(s.pos), s.box, s.cutoff + s.skin)
    t_list = time.perf_counter() - t0
    nb = 0
    t_beads = 0.0
    while nb < s.n_beads and (nb < 1 or t_list + t_beads < budget_s):
        t1 = time.perf_counter()
        ofo.bead_potential(s.pos[nb], s, pairs)
        t_beads += time.perf_counter() - t1
        nb += 1
    wall = time.perf_counter() - t0
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    step_s = t_list + t_beads / nb * s.n_beads          # one list build + all beads
    return {
        "value": s.n_atoms * s.n_beads / step_s,
        "unit": "bead*atom-steps/s",
        "cores": max(1, round(cpu / wall)),
        "kind": "oracle",
        "sample": (f"numpy FP64 oracle: centroid pair list + potential and forces of {nb} of "
                   f"{s.n_beads} beads of the 4,096-water box ({wall:.1f} s), scaled to one "
                   f"step of all beads ({step_s:.1f} s/step)"),
        "ns_per_day": 86400.0 / step_s * s.dt * 1e-6,
    }


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world}).", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    import paper_2212_03137_amd as q

    s = synth.large_rpmd()
    stream = torch.cuda.current_stream().cuda_stream
    dt = s.dt

    def make(prec, ex, graph=not args.no_graph, **kw):
        c = q.Context.from_system(s, precision=prec, exec_mode=ex, stream=stream,
                                  use_graph=graph, **kw)
        c.set_state(s.pos, s.vel, 0)
        return c

    def timed(c, steps, prof=None):
        if prof:
            c.profile(prof)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.step(steps)                 # one call: K steps, one host sync at the end
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        pr = c.profile_read() if prof else None
        if prof:
            c.profile("off")
        return t, pr

    if args.windows:
        print(json.dumps({"alchemical_windows": windows_timing(q, steps=max(1, args.steps),
                                                               warmup=args.warmup)}))
        return
    if args.adqtb:
        print(json.dumps({"adqtb_box": adqtb_timing(q, stream)}))
        return

    if args.pmc_probe:
        # a plain copy of known size (256 MiB read, 256 MiB written) to scale the
        # FETCH_SIZE / WRITE_SIZE counters, then launched steps of the timed path
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        c = make(q.FP32_PAIRS, q.BATCHED, graph=False)
        c.step(args.warmup)
        # one fixed launch shape that the autotuner picks for this box (its choice between
        # close candidates varies from run to run), so that every counter pass sees the
        # same kernels
        c.set_launch(16, 1, 1, 4)
        c.step(args.steps)
        c.close()
        torch.cuda.synchronize()
        print("pmc probe done", file=sys.stderr)
        return

    # --- which kernel class dominates the batched FP32-pair step (short untimed pass) ---
    main_ctx = make(q.FP32_PAIRS, q.BATCHED)
    main_ctx.step(args.warmup)
    spread_block = main_ctx.autotune(5)
    classes = ["pair", "spread", "fft", "gather", "nm"]
    per_class = {}
    for cl in classes:
        _, (ms, n) = timed(main_ctx, 20, cl)
        per_class[cl] = ms / 20.0
    dominant = max(per_class, key=per_class.get)
    if args.breakdown:
        print(json.dumps({"breakdown_ms_per_step": per_class}), file=sys.stderr)

    # --- timed region: exactly K steps (each step one graph replay) ---
    t, _ = timed(main_ctx, args.steps)
    ms_step = t / args.steps * 1e3
    steps_per_s = args.steps / t
    ns_day = steps_per_s * dt * 86400.0 * 1e-6
    bas = steps_per_s * s.n_atoms * s.n_beads
    # --- the same K steps launched kernel by kernel, HIP events around the dominant class
    #     on the context's stream (graph replays carry no per-kernel events) ---
    t_prof, (dom_ms, dom_n) = timed(main_ctx, args.steps, dominant)
    main_ctx.close()

    counts = pair_counts(s)
    kind, work = algorithmic_work(dominant, s, counts)
    # one event pair brackets one step's launch(es) of the class (the 5 FFT passes count
    # as one unit of work)
    avg_s = dom_ms / dom_n * 1e-3 if dom_n else float("nan")
    if kind == "bytes":
        achieved = work / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    else:
        achieved = work / avg_s / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"], roof["traffic_source"], roof["l2_hit_rate"] = measured_traffic(dominant)
    roof["traffic_unit"] = "HBM bytes per launch"
    roof["kernel"] = dominant
    roof["avg_launch_ms"] = dom_ms / dom_n if dom_n else None
    roof["launches"] = dom_n
    roof["profiled_region_ms_per_step"] = t_prof / args.steps * 1e3

    out = {
        "metric": "ns/day & bead·atom-steps/s, 4096-water RPMD P=32; batched vs plain",
        "value": ns_day,
        "unit": "ns/day",
        "bead_atom_steps_per_s": bas,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pairs + f64",
        "data": "synthetic (seeded jittered-lattice water, thermal ring polymers)",
        "config": {"workload": "water4096_P32: 4,096 flexible 3-site waters, 49.7 A cube, "
                               "rc 9 A, SPME 64^3 order 5, P=32, 300 K, dt 0.5 fs, "
                               "bead-batched FP32-pair path",
                   "n_atoms": s.n_atoms, "n_beads": s.n_beads, "parallelism": "single GPU",
                   "autotuned": {"spread_beads": spread_block[0],
                                 "spread_z_tiles": spread_block[1],
                                 "yz_plane_slots": spread_block[2],
                                 "pair_atoms_per_block": spread_block[3]}},
        "roofline": roof,
        "breakdown_ms_per_step": per_class,
    }
    out["phase_rooflines"], out["step_roofline"] = phase_rooflines(s, per_class, counts,
                                                                   ms_step)

    if not args.no_compare:
        comp = {}
        for name, prec, ex in (("batched_fp64", q.FP64, q.BATCHED), ("plain_fp64", q.FP64, q.PLAIN)):
            c = make(prec, ex)
            c.step(args.warmup)
            k = args.plain_steps or args.steps
            tt, _ = timed(c, k)
            c.close()
            sps = k / tt
            comp[name] = {"ns_per_day": sps * dt * 86400e-6, "ms_per_step": tt / k * 1e3,
                          "bead_atom_steps_per_s": sps * s.n_atoms * s.n_beads, "steps": k}
        # BAOAB-RESPA with ring-polymer contraction (Sec. "Multi-timestep Methods"): V_s on
        # 4 contracted beads once per outer step of 4 inner steps (2 fs), V_f every 0.5 fs
        P_c, nalt = 4, 4
        try:
            c = make(q.FP32_PAIRS, q.BATCHED, rpc_beads=P_c, respa_nalt=nalt)
            c.step(max(1, args.warmup // nalt))
            k = max(1, args.steps // nalt)
            tt, _ = timed(c, k)
            c.close()
            sps = k * nalt / tt                     # inner (0.5 fs) steps per second
            comp["rpc4_respa4_fp32"] = {
                "ns_per_day": sps * dt * 86400e-6, "ms_per_outer_step": tt / k * 1e3,
                "outer_steps": k, "rpc_beads": P_c, "respa_nalt": nalt,
                "note": "V_f (bonds, angles) on 32 beads every 0.5 fs; V_s on 4 contracted "
                        "beads every 2 fs"}
        except Exception as e:                      # reported, not fatal to the headline
            comp["rpc4_respa4_fp32"] = {"error": str(e)}
        # derivatives beyond the forces, on the same configuration (device tensors): a
        # Hessian-vector product of all 32 beads and the parameter gradients
        try:
            from paper_2212_03137_amd import autograd as qa
            c = make(q.FP32_PAIRS, q.BATCHED, graph=False)
            pos_d = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
            v_d = torch.randn_like(pos_d)
            qa._hvp(c, pos_d, v_d)
            qa._param_grad(c, pos_d)
            reps = 20
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                qa._hvp(c, pos_d, v_d)
            t_h = (time.perf_counter() - t0) / reps
            t0 = time.perf_counter()
            for _ in range(reps):
                qa._param_grad(c, pos_d)
            t_p = (time.perf_counter() - t0) / reps
            c.close()
            comp["derivatives"] = {"hvp_ms": t_h * 1e3, "param_grad_ms": t_p * 1e3,
                                   "note": "one call each on all 32 beads, FP32 pair terms "
                                           "(r, 1/r, erfc, exp) with FP64 products and sums, "
                                           "list rebuilt and forces evaluated inside"}
            comp["derivatives"]["force_loss"] = force_loss_timing(q, qa)
        except Exception as e:
            comp["derivatives"] = {"error": str(e)}
        try:
            comp["alchemical_windows"] = windows_timing(q)
        except Exception as e:
            comp["alchemical_windows"] = {"error": str(e)}
        try:
            comp["adqtb_box"] = adqtb_timing(q, stream)
        except Exception as e:
            comp["adqtb_box"] = {"error": str(e)}
        out["compare"] = comp
        out["speedup_vs_plain_fp64"] = ns_day / comp["plain_fp64"]["ns_per_day"]

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(s)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
