"""Throughput of the HEVI dynamical-core step on one MI355X.

Workload: gas-giant-like planet on the g6 icosahedral grid (40962 columns) x
32 levels, large step 300 s with 8 acoustic substeps (13 substeps per large
step), Newtonian relaxation (1e5 s) toward a day/night equilibrium
temperature, synthetic seeded initial state.  A "step" is one large step:
the per-step hyperdiffusion and [t] terms, three RK stages of slow tendencies
and all 13 acoustic substeps (explicit horizontal momentum, HEVI vertical
solve, divergence damping), then the physics.

Metric: cell-updates/s per acoustic substep,
    N_col * L * (1 + 3n/2) * K / T_wall,
with T_wall the time of K graph-launched large steps (inputs resident in
HBM).  Printed as one JSON line with the FP64 value, the mixed-precision
value beside it, the HBM roofline of the dominant kernel and the FP64 oracle
timed on the host cores.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E datasheet peak
BF16_PEAK_TFLOPS = 2500.0   # MI355X dense BF16 matrix peak


def vert_bytes_per_cell(L, mixed):
    """Algorithmic bytes of one acoustic phase-V launch per cell: distinct
    field words read and written once, plus the per-column stencil geometry
    (neighbour ids and 7 coefficient vectors) once per column."""
    h = 4 if mixed else 8
    reads = 3 * h + h + h + 8 + 8 + 8 + h + 8 + h + h + 8 + 8   # M, thL, Gam, rho, rth, W, p*, S_W, H_rho, H_rth, rho_t, p_t
    writes = 8 + 8 + 8 + h + h                                  # rho, rth, W, p*, D
    geom = 6 * 4 + 21 * h
    return reads + writes + geom / L


def hmom_bytes_per_cell(L, mixed):
    """Algorithmic bytes of one acoustic phase-M launch per cell: M, S_M, p*
    and D read, M written, plus per column the neighbour ids, the 7 gradient
    coefficient vectors, the radial unit vector and the two-ring damping
    stencil (18 ids and 18 weight vectors)."""
    h = 4 if mixed else 8
    fields = 11 * h              # M in (3), S_M (3), p* (1), D (1), M out (3)
    geom = 6 * 4 + 21 * h + 3 * h + 18 * 4 + 54 * h
    return fields + geom / L


def achieved_gbs(w, kt, mixed):
    """Algorithmic GB/s of the two acoustic kernels from their mean launch
    times (ms)."""
    out = {}
    for name, per_cell in (("vert", vert_bytes_per_cell), ("hmom", hmom_bytes_per_cell)):
        t = kt[name][0] * 1e-3
        out[name] = per_cell(w.n_lev, mixed) * w.cells / t / 1e9 if t > 0 else 0.0
    return out


def counter_traffic():
    """HBM bytes per phase-V launch from the committed FETCH_SIZE/WRITE_SIZE
    counter summary (scaled by the copy-kernel calibration), if it was taken
    on the kernels as they are now; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "vert_g6L32_counters.json")
    src = os.path.join(ROOT, "paper_1607_05535_amd", "csrc", "kernels.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    return rec["hbm_bytes_per_launch"] if rec.get("kernels_hip_sha256") == sha else None


def run_gpu(w, precision, steps, warmup):
    import torch
    from paper_1607_05535_amd import thor
    g = thor.Grid(w.glevel)
    st = thor.State(g, *thor.structs_from_workload(w, precision), device="cuda:0")
    n = w.n_acoustic
    tuned = thor.thor_autotune(st.handle, n)
    st.step(warmup, n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.step(steps, n)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    sc, rc = st.scalars()
    if rc != 0:
        raise RuntimeError("non-finite state after the timed steps")
    # kernel durations with HIP events on the state's stream
    thor.thor_set_timing(st.handle, 1)
    st.step(steps, n)
    kt = {k: thor.thor_kernel_time(st.handle, k) for k in ("vert", "hmom", "slow", "large")}
    thor.thor_set_timing(st.handle, 0)
    torch.cuda.synchronize()
    return T, kt, sc, tuned


def mixed_one_day():
    """FP64 and mixed precision on the g7 (163842 columns) x 48 level gas
    giant for one Earth day (288 steps of 300 s): per-field relative L2
    difference of the mixed form against FP64 on the same GPU, and the time
    of each."""
    import numpy as np
    import torch
    import workloads
    from paper_1607_05535_amd import thor
    w = workloads.gas_giant_c3()
    g = thor.Grid(w.glevel)
    out, fields, times = {}, {}, {}
    for prec in (0, 1):
        st = thor.State(g, *thor.structs_from_workload(w, prec), device="cuda:0")
        thor.thor_autotune(st.handle, w.n_acoustic)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st.step(w.n_large, w.n_acoustic)
        torch.cuda.synchronize()
        times[prec] = time.perf_counter() - t0
        fields[prec] = {k: st.field(k)[0] for k in ("T", "u", "v", "w", "p")}
        del st
        torch.cuda.empty_cache()
    a, b = fields[0], fields[1]
    speed = np.sqrt(a["u"] ** 2 + a["v"] ** 2 + a["w"] ** 2)
    for k in ("T", "u", "v", "w", "p"):
        den = np.linalg.norm(speed) if k in ("u", "v", "w") else np.linalg.norm(a[k])
        out[k] = float(np.linalg.norm(b[k] - a[k]) / den)
    return {"workload": "gas giant g7 (163842 columns) x 48 levels, 288 steps of 300 s (one day)",
            "rel_l2_vs_fp64": out, "max_speed_fp64": float(speed.max()),
            "seconds_fp64": times[0], "seconds_mixed": times[1], "speedup": times[0] / times[1]}


def run_physics_case(w, label, steps, warmup):
    """One of the paper's two benchmark setups at its own size, FP64 and
    mixed, autotuned: cell-updates/s and kernel times."""
    T, kt, sc, tuned = run_gpu(w, 0, steps, warmup)
    T32, _, _, _ = run_gpu(w, 1, steps, warmup)
    return {"workload": label, "value": w.cells * w.substeps_per_large * steps / T, "unit": "cell-updates/s",
            "ms_per_step": T / steps * 1e3, "max_speed": sc["max_speed"],
            "mixed": {"value": w.cells * w.substeps_per_large * steps / T32, "ms_per_step": T32 / steps * 1e3,
                      "speedup_vs_fp64": T / T32},
            "kernel_ms": {k: v[0] for k, v in kt.items()}}


def run_zonal(reps=20):
    """Post-processing of one snapshot of the g6 L32 benchmark state: u, v,
    T, theta interpolated to 20 pressure levels and reduced over 36 latitude
    bands (mean and eddy passes), FP64."""
    import numpy as np
    import torch
    import workloads
    from paper_1607_05535_amd import thor
    w = workloads.gas_giant_c2()
    g = thor.Grid(w.glevel)
    st = thor.State(g, *thor.structs_from_workload(w), device="cuda:0")
    st.step(2, w.n_acoustic)
    plev = np.geomspace(2e3, 2e7, 20)
    z = thor.Zonal(st, g, w.radius, w.gravity, 36, plev)
    z.accumulate()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        z.accumulate()
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / reps * 1e-3
    # state read (rho, rho theta, M) + interpolated values written once and read twice
    bytes_ = w.cells * 5 * 8.0 + w.n_col * len(plev) * 5 * 8.0 * 3
    return {"workload": "g6 L32 snapshot, 20 pressure levels, 36 bands", "ms_per_snapshot": t * 1e3,
            "GBs": bytes_ / t / 1e9}


def run_ensemble(steps, warmup):
    """The 64-planet ensemble advanced with one launch per phase, against the
    same planets advanced one after the other with the single-planet path."""
    import torch
    import workloads
    from paper_1607_05535_amd import thor
    ws = workloads.ensemble()
    grids = {}
    members = []
    for i, w in enumerate(ws):
        grids.setdefault(w.glevel, thor.Grid(w.glevel))
        pl, v, num, fo, ini = thor.structs_from_workload(w)
        ini.planet_index = i
        members.append((pl, v, num, fo, ini))
    updates = sum(w.cells * w.substeps_per_large for w in ws) * steps
    b = thor.Batch([grids[w.glevel] for w in ws], members)
    wpb = b.autotune(8)
    b.step(warmup, 8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps, 8)
    torch.cuda.synchronize()
    Tb = time.perf_counter() - t0
    del b
    torch.cuda.empty_cache()
    Ts = 0.0
    for i, w in enumerate(ws):
        st = thor.State(grids[w.glevel], *members[i])
        st.step(warmup, 8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st.step(steps, 8)
        torch.cuda.synchronize()
        Ts += time.perf_counter() - t0
        del st
    # the single-planet path on the ensemble's own level counts: the first g6
    # member of each level count alone (autotuned, graph-replayed), and the
    # rate the ensemble's cell mix would have if every planet ran at the rate
    # of the g6 planet with its level count
    rate_by_L = {}
    for L in sorted({w.n_lev for w in ws}):
        cand = [i for i, w in enumerate(ws) if w.n_lev == L and w.glevel == 6]
        if not cand:
            continue
        i = cand[0]
        st = thor.State(grids[6], *members[i])
        thor.thor_autotune(st.handle, 8)
        st.step(warmup, 8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st.step(steps, 8)
        torch.cuda.synchronize()
        rate_by_L[L] = ws[i].cells * ws[i].substeps_per_large * steps / (time.perf_counter() - t0)
        del st
    same_mix = None
    if all(w.n_lev in rate_by_L for w in ws):
        same_mix = updates / sum(w.cells * w.substeps_per_large * steps / rate_by_L[w.n_lev] for w in ws)
    return {"value": updates / Tb, "unit": "cell-updates/s", "planets": len(ws),
            "cells": sum(w.cells for w in ws), "ms_per_step": Tb / steps * 1e3,
            "one_by_one_value": updates / Ts, "speedup_vs_one_by_one": Ts / Tb,
            "single_g6_planet_value_by_levels": rate_by_L, "same_mix_single_planet_value": same_mix,
            "vs_same_mix_single_planet": (updates / Tb) / same_mix if same_mix else None,
            "autotuned_wavefronts_per_workgroup": wpb}


def run_corrector_mlp(reps=20):
    """The corrector network at the g5 L32 shape (inputs 7 columns x 5 fields
    x 32 levels, three hidden layers of 256, 160 outputs): one inference pass
    over all 10242 coarse columns (with the fused 4-layer kernel, and layer
    by layer for comparison) and one training step on 4096 columns, as
    matrix-core FLOP/s against the dense BF16 peak.  At this shape inference
    moves ~61 MB for 9.4 GFLOP (~150 flop/byte, under the ~310 flop/byte
    ridge of 2.5 PFLOP/s over 8 TB/s), so its bound is HBM: its GB/s is
    reported too.  Times are host-launched (HIP events around 20 calls)."""
    import torch
    from paper_1607_05535_amd import thor
    widths = [1120, 256, 256, 256, 160]
    n_inf, n_train = 10242, 4096
    net = thor.MLP(widths, n_inf, seed=1)
    g = torch.Generator(device="cuda:0").manual_seed(5)
    x = torch.randn(n_inf, widths[0], device="cuda:0", generator=g).to(torch.bfloat16)
    y = torch.empty(n_inf, widths[-1], device="cuda:0")
    t = torch.randn(n_train, widths[-1], device="cuda:0", generator=g)
    pairs = list(zip(widths[:-1], widths[1:]))
    f_fwd = sum(2.0 * i * o for i, o in pairs)                  # per row
    f_train = 2 * f_fwd + sum(2.0 * i * o for i, o in pairs[1:])  # forward, dW, dH (no dX)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    t_inf = timed(lambda: net.forward(x, y))          # fused 4-layer kernel (the default)
    net.set_fused(False)
    t_inf_layered = timed(lambda: net.forward(x, y))
    net.set_fused(True)
    t_tr = timed(lambda: net.train_step(x[:n_train], t, 1e-4))
    # inference traffic: inputs, weights, each hidden activation written and
    # read once (bf16), outputs written (fp32)
    b_inf = (2.0 * n_inf * widths[0] + sum(2.0 * i * o + 4.0 * o for i, o in pairs)
             + sum(4.0 * n_inf * o for o in widths[1:-1]) + 4.0 * n_inf * widths[-1])
    return {"widths": widths,
            "inference_rows": n_inf, "inference_ms": t_inf * 1e3, "inference_ms_layer_by_layer": t_inf_layered * 1e3,
            "inference_bytes": b_inf, "inference_GBs": b_inf / t_inf / 1e9,
            "inference_TFLOPs": f_fwd * n_inf / t_inf / 1e12,
            "train_rows": n_train, "train_step_ms": t_tr * 1e3,
            "train_TFLOPs": f_train * n_train / t_tr / 1e12,
            "peak_TFLOPs": BF16_PEAK_TFLOPS,
            "inference_frac": f_fwd * n_inf / t_inf / 1e12 / BF16_PEAK_TFLOPS}


def run_corrector_c5(seeds, pairs, steps):
    """The learned form at its own configuration: coarse g5 L32 corrected
    toward the g7 L32 run restricted to g5 (gas giant, coarse step 600 s,
    fine 150 s, one Earth day of fine spin-up per trajectory), trained on
    (seeds - 1) x pairs snapshot pairs and judged on the last seed's pairs:
    per-field RMS error of the plain and of the corrected coarse step against
    the restricted fine run, and the wall time of 600 s of simulated time,
    coarse step + corrector against four fine steps."""
    from paper_1607_05535_amd import train_corrector
    t0 = time.perf_counter()
    rep = train_corrector.run(7, 5, seeds=seeds, pairs=pairs, spinup=576, steps=steps, batch=4096, lr=1e-3)
    rep["workload"] = (f"g7 L32 fine -> g5 L32 coarse gas giant, {(seeds - 1) * pairs} training pairs, "
                       f"{pairs} held out, {steps} Adam steps of 4096 columns")
    rep["seconds_total"] = time.perf_counter() - t0
    return rep


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, n_steps=1):
    """The FP64 oracle on the host: n_steps whole large steps of the workload
    (per-step terms, three RK stages of slow terms, every acoustic substep,
    the physics), timed end to end after the grid and initial state are
    built, with every BLAS/OpenMP pool held to one thread."""
    from threadpoolctl import threadpool_limits
    from oracle import dynamics as odyn
    from oracle import grid as ogrid
    G = ogrid.Grid(w.glevel, k=100.0)
    model, st = odyn.model_from_workload(w, G)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        st = odyn.run(model, st, n_steps, w.n_acoustic)
        T = time.perf_counter() - t0
    value = w.cells * w.substeps_per_large * n_steps / T
    return dict(value=value, unit="cell-updates/s", cores=1, kind="oracle",
                sample=(f"{w.name}: {n_steps} whole large step(s) of the oracle ({T:.1f} s; "
                        f"{w.substeps_per_large} acoustic substeps each), not extrapolated"),
                seconds=T, steps=n_steps, cpu_model=cpu_model(), host_cpus=os.cpu_count())


def stream_GBs(n_src, n_dst, n, reps=20):
    """GB/s of the library's streaming kernel (thor_stream_mix) reading n_src
    and writing n_dst FP64 arrays of n words: what the memory system delivers
    for a kernel's traffic mix without its arithmetic or gathers."""
    import torch
    from paper_1607_05535_amd import thor
    src = [torch.full((n,), 1.0 + k, dtype=torch.float64, device="cuda:0") for k in range(n_src)]
    dst = [torch.empty(n, dtype=torch.float64, device="cuda:0") for _ in range(n_dst)]
    thor.stream_mix(src, dst)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        thor.stream_mix(src, dst)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / reps * 1e-3
    del src, dst
    torch.cuda.empty_cache()
    return 8.0 * n * (n_src + n_dst) / t / 1e9


def copy_GBs():
    """Read + write GB/s of a plain 1 GiB device copy (the streaming kernel
    with one source and one destination of 2^27 words)."""
    return stream_GBs(1, 1, 1 << 27, reps=10)


def copy_probe():
    """A plain device copy of known size (1 GiB read + 1 GiB written): the
    reference for scaling FETCH_SIZE / WRITE_SIZE counters and for the
    achievable streaming bandwidth."""
    import torch
    n = 1 << 27                       # doubles = 1 GiB
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    T = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n,
                      "ms": T * 1e3, "GBs_read_plus_write": 16 * n / T / 1e9}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-one-day", action="store_true")
    ap.add_argument("--no-corrector", action="store_true")
    ap.add_argument("--no-c5", action="store_true", help="skip the learned form's own-configuration leg")
    ap.add_argument("--c5-seeds", type=int, default=4, help="trajectories of the C5 leg (the last held out)")
    ap.add_argument("--c5-pairs", type=int, default=100, help="pairs per trajectory of the C5 leg")
    ap.add_argument("--c5-steps", type=int, default=1500, help="Adam steps of the C5 leg")
    ap.add_argument("--no-hot-jupiter", action="store_true")
    ap.add_argument("--no-zonal", action="store_true")
    ap.add_argument("--no-energy-fixer", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only time a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--cpu-baseline-only", action="store_true",
                    help="only the oracle on one host core: the g4 L20 Earth case (10 steps) "
                         "and the g6 L32 benchmark (3 steps)")
    ap.add_argument("--physics-only", action="store_true",
                    help="only the hot-Jupiter and Held-Suarez benchmark setups (g5 L37)")
    ap.add_argument("--corrector-mlp-only", action="store_true",
                    help="only the corrector network's inference and training rates (g5 shape)")
    args = ap.parse_args()
    if args.corrector_mlp_only:
        print(json.dumps({"corrector_mlp": run_corrector_mlp()}), flush=True)
        return
    if args.copy_probe:
        copy_probe()
        return
    if args.cpu_baseline_only:
        import workloads
        for wc, k in ((workloads.earth_c1(), 10), (workloads.gas_giant_c2(), 3)):
            print(json.dumps({"workload": wc.name, "cpu_baseline": cpu_baseline(wc, k)}), flush=True)
        return
    if args.physics_only:
        import workloads
        print(json.dumps({"hot_jupiter": run_physics_case(
                              workloads.hot_jupiter(glevel=5, n_lev=37), "hot-Jupiter benchmark g5 L37",
                              args.steps, args.warmup),
                          "held_suarez": run_physics_case(
                              workloads.held_suarez(glevel=5, n_lev=37), "Held-Suarez benchmark g5 L37",
                              args.steps, args.warmup)}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU (there is no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import workloads
    w = workloads.gas_giant_c2()
    subs = w.substeps_per_large
    updates = w.cells * subs * args.steps

    T64, kt64, sc64, tuned64 = run_gpu(w, 0, args.steps, args.warmup)
    copy_bw = copy_GBs()
    # phase V's own-column traffic: 14 FP64 arrays read (M, theta_L, rho,
    # rho theta, W, p*, p[t], rho[t], Gamma, the two hyperdiffusion
    # tendencies, the slow W forcing) and 5 written (rho, rho theta, W, p*, D)
    # over the padded cells
    ceiling = stream_GBs(14, 5, w.n_col * ((w.n_lev + 3) // 4 * 4))
    value = updates / T64
    vmean = kt64["vert"][0] * 1e-3
    vb = vert_bytes_per_cell(w.n_lev, False) * w.cells
    achieved = vb / vmean / 1e9 if vmean > 0 else 0.0
    out = {
        "metric": "cell-updates/s per acoustic substep, g6 L32, FP64 vs mixed; % HBM roofline",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T64 / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": ("gas giant g6 (40962 columns) x 32 levels, dt 300 s, "
                                "8 acoustic substeps (13 per large step), Newtonian relaxation, "
                                "divergence damping"),
                   "n_col": w.n_col, "n_lev": w.n_lev, "substeps_per_step": subs},
        "roofline": {"bound": "hbm", "kernel": "vert (acoustic phase V)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic(),
                     "bytes_per_launch": vb, "mean_launch_ms": kt64["vert"][0],
                     "copy_GBs": copy_bw, "frac_of_copy": achieved / copy_bw,
                     "mix_ceiling_GBs": ceiling, "frac_of_mix_ceiling": achieved / ceiling},
        # phase M + phase V kernel time per substep, as cell-updates/s
        "kernel_only_substep_value": w.cells / ((kt64["vert"][0] + kt64["hmom"][0]) * 1e-3),
        "kernel_ms": {k: v[0] for k, v in kt64.items()},
        "achieved_GBs": achieved_gbs(w, kt64, False),
        "autotuned_wavefronts_per_workgroup": tuned64,
    }
    if not args.no_mixed:
        T32, kt32, sc32, tuned32 = run_gpu(w, 1, args.steps, args.warmup)
        out["mixed"] = {"dtype": "f32 horizontal / f64 vertical", "value": updates / T32,
                        "ms_per_step": T32 / args.steps * 1e3,
                        "speedup_vs_fp64": T64 / T32,
                        "achieved_GBs": achieved_gbs(w, kt32, True),
                        "kernel_ms": {k: v[0] for k, v in kt32.items()}}
        if not args.no_one_day:
            out["mixed"]["one_day"] = mixed_one_day()
    if not args.no_energy_fixer:
        wf = workloads.gas_giant_c2()
        wf.energy_fixer = True
        Tf, ktf, scf, _ = run_gpu(wf, 0, args.steps, args.warmup)
        out["energy_fixer"] = {"workload": "the g6 L32 workload with the uniform internal-energy fixer",
                               "value": updates / Tf, "ms_per_step": Tf / args.steps * 1e3,
                               "overhead_vs_fp64": Tf / T64 - 1.0}
    if not args.no_variants:
        # the switchable approximations of the g6 L32 workload, FP64
        out["variants"] = {}
        for name, attr, val in (("hydrostatic", "hydrostatic", True), ("shallow", "shallow", True),
                                ("cubic_vertical_interpolation", "lagrange_order", 3),
                                ("anelastic", "anelastic", True)):
            wv = workloads.gas_giant_c2()
            setattr(wv, attr, val)
            kv = max(1, args.steps // 2)
            Tv, _, _, _ = run_gpu(wv, 0, kv, args.warmup)
            out["variants"][name] = {"value": wv.cells * subs * kv / Tv, "unit": "cell-updates/s",
                                     "ms_per_step": Tv / kv * 1e3}
    if not args.no_hot_jupiter:
        out["hot_jupiter"] = run_physics_case(
            workloads.hot_jupiter(glevel=5, n_lev=37),
            "hot-Jupiter benchmark g5 (10242 columns) x 37 levels to 4875 km, dt 600 s, n = 8",
            args.steps, args.warmup)
        out["held_suarez"] = run_physics_case(
            workloads.held_suarez(glevel=5, n_lev=37),
            "Held-Suarez benchmark g5 (10242 columns) x 37 levels to 32 km, dt 1000 s, n = 8",
            args.steps, args.warmup)
    if not args.no_zonal:
        out["zonal_postprocessing"] = run_zonal()
    if not args.no_ensemble:
        out["ensemble"] = run_ensemble(max(1, args.steps // 10), 2)
    if not args.no_corrector:
        out["corrector_mlp"] = run_corrector_mlp()
    if not args.no_c5:
        out["corrector_c5"] = run_corrector_c5(args.c5_seeds, args.c5_pairs, args.c5_steps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
