"""Benchmark of the colour-gradient LBM time step on one MI355X.

Workload: D3Q19 drainage in a synthetic rock, single precision, MRT: a 256^3
voxel box made from a seeded Gaussian random field (correlation length 8)
thresholded to porosity 0.22 in the rock region with the spanning pore cluster
kept, ten pure-fluid layers at each end and solid side walls, initially
wetting-saturated, non-wetting fluid injected at z = 0 by a Zou-He inlet with
rho_in - rho_out = 0.02, theta = 30 deg (Scheme-I), tau_r = 1.0, tau_b = 0.6,
sigma = 0.01, beta = 0.95.

One step = the whole step (phase field, both extrapolations, normals with
wetting, and the fused stream-collide-recolour kernel) over all fluid nodes.
Prints one JSON line: MLUPS counted over fluid nodes (value) and over all
voxels, the HBM roofline of the dominant kernel from HIP events in the timed
region, and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
B_ALG_F32_D3Q19 = 2 * 19 * 2 * 4  # two colours x Q x (read + write) x 4 bytes = 304


def workload(n=256):
    from paper_2407_10914_amd import inputs

    case = inputs.grf_rock(n=n, corr=8.0, porosity=0.22, seed=inputs.MASTER_SEED, buffer=10)
    kw = dict(dim=3, periodic=case.periodic, tau_r=1.0, tau_b=0.6, sigma=0.01, beta=0.95, scheme=1,
              theta_deg=30.0, bc=1, rho_in=1.02, rho_out=1.0, zeta_r=1.0, collision=1)
    return case, kw


# the sources that define the step kernels (k_main and the stages before it)
STEP_SOURCES = ("lattice.hpp", "step.hpp", "kernels.hpp", "kernels_f32.hip")


def kernel_source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2407_10914_amd", "csrc")
    for f in STEP_SOURCES:
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def read_profile(n_fluid, block):
    """The committed rocprofv3 PMC summary's figures (HBM bytes per k_main
    launch, measured bytes per fluid node over the whole step), or None when
    missing, taken from other kernel sources or at another block size."""
    path = os.path.join(ROOT, "profiles", "k_main_rock256_f32_pmc.md")
    if not os.path.exists(path):
        return None
    meta = {}
    for line in open(path):
        if line.startswith("<!--") and "traffic:" in line:
            body = line.strip()[4:-3].split("traffic:", 1)[1]
            meta = json.loads(body)
    if not meta or meta.get("kernel_hash") != kernel_source_hash() or meta.get("n_fluid") != n_fluid:
        return None
    if meta.get("block", 256) != block:
        return None
    return meta


def read_traffic(n_fluid, block):
    """HBM bytes per k_main launch from the committed profile (see read_profile)."""
    meta = read_profile(n_fluid, block)
    return None if meta is None else meta.get("bytes_per_launch")


def cpu_baseline(case, kw, budget_s=20.0, threads=None):
    """The CPU oracle on the same 256^3 rock: setup untimed, then whole steps
    until about budget_s seconds of stepping (at least one), with `threads`
    OpenMP threads (default: what the environment gives it)."""
    import oracle as O

    if threads is None:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    threads = O.set_threads(threads)
    o = O.OracleSim(case.solid, eps="f32", **kw)
    o.set_phase(case.phi0)
    n_fluid = int((case.solid == 0).sum())
    steps, t0 = 0, time.perf_counter()
    while True:
        o.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or el / steps * (steps + 1) > 1.5 * budget_s:
            break
    del o
    return dict(value=round(n_fluid * steps / el / 1e6, 3), unit="MLUPS", cores=threads, kind="oracle",
                sample=f"{steps} step(s) of the same 256^3 rock (FP64 oracle, {n_fluid} fluid nodes), "
                       f"{el:.1f} s, OpenMP threads={threads}",
                hours_for_10k_steps=round(el / steps * 1e4 / 3600, 2))


def fp64_leg(case, kw, steps=50, warmup=5, tune=True):
    """The same 256^3 step in double precision (the build that reproduces the
    oracle bit for bit): fluid-node MLUPS and k_main's algorithmic rate
    (608 B per node), block sizes from the run's tuner (256 threads per block
    with tune=False)."""
    import torch

    from paper_2407_10914_amd.sim import Sim

    sim = Sim(case.solid, precision="f64", **kw)
    sim.set_phase(case.phi0)
    n_fluid = sim.info()["fluid"]
    report = sim.tune(reps=2) if tune else "256 threads per block"
    sim.step(warmup)
    sim.sync()
    sim.set_timing(["k_main"])
    sim.reset_timing()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    sim.sync()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    cnt, kms = sim.kernel_times()["k_main"]
    sim.set_timing(None)
    del sim
    torch.cuda.empty_cache()
    main_us = kms / max(cnt, 1) * 1e3
    return {"mlups": round(n_fluid * steps / (ms / 1e3) / 1e6, 1), "ms_per_step": round(ms / steps, 4),
            "k_main_us": round(main_us, 2),
            "k_main_alg_gbs": round(2 * 19 * 2 * 8 * n_fluid / (main_us * 1e-6) / 1e9, 1), "steps": steps,
            "tuning": report}


def batched_leg(steps, warmup, count=64, ref_edge=256):
    """64 sessile-drop runs (edges drawn from {48, 64, 96, 128}, contact angles
    uniform in 15-165 deg, Scheme-I for even and Scheme-II for odd runs, FP32
    MRT) advanced by the batched persistent launches, against one large run of
    the same setup (edge 256, 90 deg)."""
    import torch

    from paper_2407_10914_amd import inputs
    from paper_2407_10914_amd.sim import Batch, Sim

    edges = inputs.sweep_edges(count)
    thetas = inputs.contact_angles(count)

    def make(edge, theta, scheme):
        c = inputs.sessile_3d(edge=edge)
        s = Sim(c.solid, dim=3, periodic=c.periodic, tau_r=1.0, tau_b=1.0, sigma=1.0 / 45.0, beta=0.95,
                scheme=scheme, theta_deg=theta, collision=1, precision="f32")
        s.set_phase(c.phi0)
        return s

    t0 = time.perf_counter()
    sims = [make(edges[k], thetas[k], 1 if k % 2 == 0 else 2) for k in range(count)]
    batch = Batch(sims)
    voxels = sum(e ** 3 for e in edges)
    report = batch.tune(reps=3)
    print(f"# batch setup+tune {time.perf_counter() - t0:.1f} s: {report}", file=sys.stderr, flush=True)
    batch.step(warmup)
    batch.sync()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    batch.step(steps)
    e1.record(stream)
    batch.sync()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    nodes = batch.info()["total_nodes"]
    batched = nodes * steps / (ms / 1e3) / 1e6
    del batch
    del sims
    torch.cuda.empty_cache()
    # the single large run of the same setup
    big = make(ref_edge, 90.0, 1)
    big.tune(reps=3)
    big.step(warmup)
    big.sync()
    torch.cuda.synchronize()
    e0.record(stream)
    big.step(steps)
    e1.record(stream)
    big.sync()
    torch.cuda.synchronize()
    ms1 = e0.elapsed_time(e1)
    single = big.info()["fluid"] * steps / (ms1 / 1e3) / 1e6
    del big
    torch.cuda.empty_cache()
    return {"runs": count, "voxels": int(voxels), "fluid_nodes": int(nodes), "steps": steps,
            "batched_mlups": round(batched, 1), "single_256_sessile_mlups": round(single, 1),
            "ratio": round(batched / single, 4), "tuning": report}


def adjoint_k_for_memory(info, n_steps, free_bytes, share=0.7):
    """The largest checkpoint interval K <= n_steps whose device memory fits in
    `share` of the free bytes: per state of the ring one state copy and its
    kept front fields (phase and normal grids per voxel, C and force per
    node; FP32 sizes), n_steps/K checkpoints, and the adjoint's own fields
    (about six state copies).  K >= n_steps keeps every state of the forward
    sweep, so the reverse sweep recomputes nothing."""
    V, Np = info["voxels"], (info["fluid"] + 255) // 256 * 256
    front = V * (4 + 12) + Np * (12 + 16)
    st = info["state_bytes"]
    budget = share * free_bytes - 6 * st
    for K in range(n_steps, 0, -1):
        need = K * (st + front) + (-(-n_steps // K) - 1 + 2) * st
        if need <= budget:
            return K
    return 1


def adjoint_leg(n_steps=2000, K=0, n=128, K_ref=100):
    """Adjoint through drainage: the 128^3 Gaussian-random-field rock (porosity
    0.22, z periodic, non-wetting fluid in the inlet buffer, body force 1e-5
    along z), a per-voxel contact-angle field of 40 deg on the solid, FP32
    MRT Scheme-I; objective = non-wetting mass saturation of the rock region
    after n_steps.  Checkpoints every K steps; K = 0 takes the largest K that
    the device's free memory holds (up to n_steps: then the forward sweep keeps
    every state and the reverse sweep recomputes nothing), and the same call
    is also timed with K_ref for comparison.  The forward step time is taken
    on the same run by plain stepping."""
    import torch

    from paper_2407_10914_amd import inputs
    from paper_2407_10914_amd.sim import Sim

    case, th = inputs.drainage_rock(n=n)
    nz = case.solid.shape[0]
    buf = case.meta["buffer"]
    kw = dict(dim=3, periodic=case.periodic, tau_r=1.0, tau_b=0.6, sigma=0.01, beta=0.95, scheme=1,
              theta_deg=40.0, collision=1, g=(0.0, 0.0, 1e-5))
    sim = Sim(case.solid, precision="f32", theta_field=th, **kw)
    n_fluid = sim.info()["fluid"]
    sim.set_phase(case.phi0)
    sim.tune(reps=3)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sim.set_phase(case.phi0)
    sim.step(20)
    sim.sync()
    sim.set_phase(case.phi0)
    torch.cuda.synchronize()
    e0.record(stream)
    sim.step(n_steps)
    e1.record(stream)
    sim.sync()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / n_steps
    sim.set_phase(case.phi0)
    sim.adjoint("saturation", n_steps=4, checkpoint_every=2, lo=buf, hi=nz - buf, field_grad=True)  # warm-up
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    if K <= 0:
        K = adjoint_k_for_memory(sim.info(), n_steps, free)

    def timed(k):
        sim.set_phase(case.phi0)
        t0 = time.perf_counter()
        r = sim.adjoint("saturation", n_steps=n_steps, checkpoint_every=k, lo=buf, hi=nz - buf, field_grad=True)
        return r, time.perf_counter() - t0

    try:
        r, wall = timed(K)
    except Exception as e:  # the memory estimate was too optimistic: the reference interval
        print(f"# adjoint with K = {K} failed ({e}); K = {K_ref}", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        K, K_ref = K_ref, 0
        r, wall = timed(K)
    gf = r["dJ_dtheta_field"]
    out = {"workload": f"{n}^3 drainage rock, FP32 MRT Scheme-I, theta(x) = 40 deg, g_z = 1e-5, "
                       f"objective S_nw (rock region) after {n_steps} steps, checkpoint every {K}",
           "fluid_nodes": int(n_fluid), "steps": n_steps, "K": K, "J": r["J"], "dJ_dtheta": r["dJ_dtheta"],
           "dJ_dgz": float(r["dJ_dg"][2]), "dJ_dtheta_field_l2": float(gf.norm()),
           "forward_ms_per_step": round(fwd_ms, 5), "adjoint_forward_sweep_ms": round(r["ms_forward"], 2),
           "adjoint_reverse_ms": round(r["ms_reverse"], 2),
           "ratio_reverse_to_forward": round(r["ms_reverse"] / (n_steps * fwd_ms), 4),
           "ratio_total_to_forward": round((r["ms_forward"] + r["ms_reverse"]) / (n_steps * fwd_ms), 4),
           "wall_s": round(wall, 3), "work_gb": round(r["work_bytes"] / 1e9, 3),
           "device_free_gb_before": round(free / 1e9, 1)}
    J0, d0 = r["J"], r["dJ_dtheta"]
    del gf, r
    torch.cuda.empty_cache()
    if K_ref and K_ref != K:
        r, wall = timed(K_ref)
        out["with_K_ref"] = {"K": K_ref, "adjoint_forward_sweep_ms": round(r["ms_forward"], 2),
                             "adjoint_reverse_ms": round(r["ms_reverse"], 2),
                             "ratio_reverse_to_forward": round(r["ms_reverse"] / (n_steps * fwd_ms), 4),
                             "ratio_total_to_forward": round((r["ms_forward"] + r["ms_reverse"]) / (n_steps * fwd_ms),
                                                             4),
                             "work_gb": round(r["work_bytes"] / 1e9, 3),
                             "same_J": r["J"] == J0, "same_dJ_dtheta": r["dJ_dtheta"] == d0}
        del r
        torch.cuda.empty_cache()
    del sim
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=40)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the double-precision step of the same workload")
    ap.add_argument("--curve-steps", type=int, default=10000,
                    help="after the timed region, continue the drainage to this step and record the saturation "
                         "every tenth of it (0: off)")
    ap.add_argument("--no-tune", action="store_true", help="keep 256 threads per block for every kernel")
    ap.add_argument("--adjoint-steps", type=int, default=2000)
    ap.add_argument("--adjoint-k", type=int, default=0,
                    help="checkpoint interval of the adjoint leg (0: the largest that free device memory holds)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run the library's plain 1 GiB copy kernel (reference for the HBM byte counters)")
    ap.add_argument("--windows", type=int, default=5, help="timed windows the --steps are split into (median)")
    ap.add_argument("--graph", action="store_true", help="replay the timed steps from captured HIP graphs")
    ap.add_argument("--no-ceiling", action="store_true",
                    help="skip the streaming-kernel sweep that measures the HBM ceiling")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the step runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2407_10914_amd.sim import Sim

    torch.cuda.set_device(0)
    t_setup = time.perf_counter()
    case, kw = workload(args.n)
    sim = Sim(case.solid, precision="f32", **kw)
    sim.set_phase(case.phi0)
    info = sim.info()
    n_fluid = info["fluid"]
    print(f"# setup {time.perf_counter() - t_setup:.1f} s, fluid nodes {n_fluid}, voxels {info['voxels']}",
          file=sys.stderr, flush=True)
    tuning = None
    if not args.no_tune:
        tuning = sim.tune(reps=5)
        print(f"# tuned: {tuning}", file=sys.stderr, flush=True)
    main_block = int(tuning.split("k_main: block ")[1].split()[0]) if tuning else 256

    if args.graph:
        sim.set_graph(True)  # the warm-up captures the two step graphs
    sim.step(args.warmup)
    sim.sync()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    # headline: exactly --steps steps, split into --windows windows bracketed
    # by HIP events on the run's stream (no per-launch events inside); the
    # value is the median window's rate
    nw = max(1, min(args.windows, args.steps))
    sizes = [args.steps // nw + (1 if k < args.steps % nw else 0) for k in range(nw)]
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(nw + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(stream)
    for k, m in enumerate(sizes):
        sim.step(m)
        evs[k + 1].record(stream)
    sim.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    win_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(nw)]
    gpu_ms = evs[0].elapsed_time(evs[nw])
    per_step = sorted(w / m for w, m in zip(win_ms, sizes))
    ms_per_step = per_step[nw // 2] if nw % 2 else 0.5 * (per_step[nw // 2 - 1] + per_step[nw // 2])
    mlups = n_fluid / (ms_per_step / 1e3) / 1e6
    vox_mlups = info["voxels"] / (ms_per_step / 1e3) / 1e6
    mlups_all = n_fluid * args.steps / (gpu_ms / 1e3) / 1e6
    # the dominant kernel's launches, timed in a window of their own
    sim.set_timing(["k_main"])
    sim.reset_timing()
    sim.step(args.steps)
    sim.sync()
    kt = sim.kernel_times()
    sim.set_timing(None)
    main_n, main_ms = kt["k_main"]
    obs = sim.observe(axis=2, plane=args.n // 2)
    main_avg_s = main_ms / max(main_n, 1) / 1e3
    achieved = B_ALG_F32_D3Q19 * n_fluid / main_avg_s / 1e9
    traffic = read_traffic(n_fluid, main_block)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": "k_main",
            "bytes_alg_per_launch": B_ALG_F32_D3Q19 * n_fluid, "avg_launch_us": round(main_avg_s * 1e6, 2),
            "block": main_block}
    step_frac = mlups * 1e6 * B_ALG_F32_D3Q19 / (HBM_PEAK_GBS * 1e9)
    roof["step_hbm_frac_alg"] = round(step_frac, 4)  # the whole step's algorithmic rate against the peak
    prof = read_profile(n_fluid, main_block)
    if prof and prof.get("step_bytes_per_node"):
        # measured HBM bytes of all step kernels per fluid-node update (counters) at this run's step rate
        roof["step_traffic_bytes_per_node"] = prof["step_bytes_per_node"]
        roof["step_traffic_gbs"] = round(prof["step_bytes_per_node"] * mlups * 1e6 / 1e9, 1)
    ceiling = None
    if not args.no_ceiling:
        from paper_2407_10914_amd import roofline

        best, _ = roofline.stream_ceiling(gib=4.0, reps=5)
        ceiling = {k: {kk: v[kk] for kk in ("gbs", "grid", "block", "nontemporal")} for k, v in best.items()}
        top = max(v["gbs"] for v in best.values())
        roof["frac_of_measured_ceiling"] = round(achieved / top, 4)
        roof["measured_ceiling_gbs"] = top
        print(f"# streaming ceiling (4 GiB per buffer): {ceiling}", file=sys.stderr, flush=True)
    curve = None
    if args.curve_steps > sim.time:
        # the drainage itself, untimed: nonwetting saturation (mass based, all
        # fluid nodes, buffers included) and the node-count wetting saturation
        curve = []
        every = max(1, args.curve_steps // 10)
        while sim.time < args.curve_steps:
            sim.step(min(every - sim.time % every, args.curve_steps - sim.time))
            o = sim.observe(check=False)
            curve.append([int(o["step"]), round(o["sat_nw_mass"], 6), round(o["sat_w"], 6)])
            if o["nan_count"] > 0:
                curve[-1].append("non-finite values in the state")
                break
        print(f"# saturation curve: {curve}", file=sys.stderr, flush=True)
    del sim
    torch.cuda.empty_cache()
    if args.copy_calib:
        # the library's own plain copy kernel (k_stream<2, false>) over 1 GiB:
        # the reference of known size for the HBM byte counters
        from paper_2407_10914_amd import roofline

        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        ms = roofline.probe("copy", x, y, 1 << 30, 8 * cus, 256, False, reps=3)
        torch.cuda.synchronize()
        print(f"# copy calibration: 1 GiB copy kernel, {ms:.3f} ms per launch (4 launches)", file=sys.stderr,
              flush=True)
        del x, y
    f64 = None
    if not args.no_fp64:
        f64 = fp64_leg(case, kw, tune=not args.no_tune)
        print(f"# fp64: {f64}", file=sys.stderr, flush=True)
    batched = None
    if not args.no_batch:
        batched = batched_leg(args.batch_steps, max(2, args.warmup // 4))
    adj = None
    if not args.no_adjoint:
        adj = adjoint_leg(args.adjoint_steps, args.adjoint_k)
        print(f"# adjoint: {adj}", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(case, kw)
        cpu["single_thread"] = cpu_baseline(case, kw, threads=1)
        print(f"# cpu oracle: {cpu}", file=sys.stderr, flush=True)
    line = {
        "metric": "MLUPS D3Q19 color-gradient 256^3; batched MLUPS; adjoint/forward time ratio",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"D3Q19 two-phase drainage, synthetic Gaussian-random-field rock {args.n}^3, "
                               "porosity 0.22, Zou-He drho=0.02, Scheme-I 30 deg, MRT, FP32",
                   "fluid_nodes": n_fluid, "voxels": info["voxels"], "voxel_mlups": round(vox_mlups, 1),
                   "step_hbm_frac_alg": round(step_frac, 4), "wall_s": round(wall, 3),
                   "timing": {"windows": nw, "steps_per_window": sizes, "window_ms": [round(w, 4) for w in win_ms],
                              "value_is": "median window", "mlups_all_windows": round(mlups_all, 1),
                              "launches": "hipGraph replay" if args.graph else "plain"},
                   "hbm_ceiling": ceiling,
                   "sat_nw_mass": obs["sat_nw_mass"], "tuning": tuning,
                   "saturation_curve": None if curve is None else {"columns": ["step", "S_nw_mass", "S_w"],
                                                                   "rows": curve},
                   "fp64": f64, "batched": batched, "adjoint": adj},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
