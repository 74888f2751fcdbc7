#!/usr/bin/env python3
"""Throughput of the fused D2Q9 volume-averaged LB sweep on one MI355X.

Workload (default): the 4096 x 4096 periodic porous box -- Gaussian-random-field
porosity (correlation length 16) in [0.3, 1.0], tau = 0.6, body force 1e-6 along
x, Ergun drag, FP32 populations stored as deviations from the local rest state.
A step is one time step of the method over the whole lattice (one sweep
launch).  Inputs are resident in HBM before timing starts.

Prints one JSON line with MLUPS, the HBM roofline of the sweep kernel, the
FP16-storage sweep on the 8192^2 box beside it, the gradient leg, the ensemble
leg (64 uneven channels, batched launches), the paper's Couette experiment
against eq. (velocity), and the CPU baseline: the FP64
oracle timed on the host cores on bounded samples of the workloads.  The
oracle runs only in that leg; its sample results also give the accuracy
figures (the GPU runs the same samples -- the 512^2 crops of the boxes, a small
channel for the gradient, the smallest ensemble member -- and the fields are
compared afterwards).  --no-cpu-baseline therefore also drops the accuracy.

  python bench.py [--steps K] [--warmup W] [--workload box4096_f32|box8192_f16|channel_f64]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0   # MI355X HBM3E peak
# VALU issue of MI355X without packed FP32: 256 compute units x 4 SIMDs, each SIMD
# retiring one 64-lane instruction every 4 cycles, at 2.4 GHz: 614.4e9 wave
# instructions per second (39.3e12 lane operations; packed FP32 doubles that to the
# 157.3 TFLOP/s FMA peak, and packed FP32 is not used here)
PEAK_VALU_WAVE_INSTS = 256 * 4 * 2.4e9 / 4
PROFILE_TRAFFIC = {"box4096_f32": os.path.join(ROOT, "profiles", "sweep_traffic_box4096_f32.md"),
                   "box8192_f16": os.path.join(ROOT, "profiles", "sweep_traffic_box8192_f16.md"),
                   "ensemble64_f32": os.path.join(ROOT, "profiles",
                                                  "batch_traffic_ensemble64_f32.md")}
PROFILE_VALU = {"box4096_f32": os.path.join(ROOT, "profiles", "sweep_valu_box4096_f32.md"),
                "box8192_f16": os.path.join(ROOT, "profiles", "sweep_valu_box8192_f16.md"),
                "ensemble64_f32": os.path.join(ROOT, "profiles", "batch_valu_ensemble64_f32.md")}
MULTI_KERNEL = {1: "k_sweep_vec", 2: "k_sweep_tb2", 3: "k_sweep_tb3", 4: "k_sweep_tb4"}
BATCH_KERNEL = {1: "k_batch_sweep", 2: "k_batch_tb2", 3: "k_batch_tb3", 4: "k_batch_tb4"}
KERNEL_SRC = os.path.join(ROOT, "paper_1406_6438_amd", "csrc", "lbm_vans.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes_per_node(storage: str) -> int:
    """Population loads + stores of one node plus its porosity load."""
    pop = {"f64": 8, "f32": 4, "f16": 2}[storage]
    eps = 8 if storage == "f64" else 4
    return 9 * pop + 9 * pop + eps


def kernel_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def summary_value(path, kernel: str, field: str):
    """A per-launch figure of `kernel` (field "<field>: <number>") from a committed
    rocprofv3 counter summary, if it was taken on the current kernel source; else None.
    A summary holds one block per kernel ("kernel: <name> ..." up to its source hash)."""
    if path is None or not os.path.exists(path):
        return None
    txt = open(path).read()
    for block in re.findall(r"kernel: (.*?kernel_source_sha256_16:\s*[0-9a-f]+)", txt, re.S):
        name = block.split()[0]
        if not (name == kernel or name.startswith(kernel + "<") or
                name.startswith("_ZN12_GLOBAL__N_1" + str(len(kernel)) + kernel)):
            continue
        m_hash = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", block)
        m_val = re.search(field + r":\s*([0-9.eE+]+)", block)
        if m_hash and m_val and m_hash.group(1) == kernel_hash():
            return float(m_val.group(1))
    return None


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the workload's committed counter summary
    (None unless taken on the current kernel source)."""
    return summary_value(PROFILE_TRAFFIC.get(workload), kernel, "hbm_bytes_per_launch")


def measured_valu(workload: str, kernel: str):
    """(VALU wave instructions, VALU-active quad-cycles summed over waves, VALU-busy
    fraction) per launch of `kernel` from the workload's committed SQ counter summary
    (None unless taken on the current kernel source)."""
    path = PROFILE_VALU.get(workload)
    vals = [summary_value(path, kernel, f) for f in
            ("valu_insts_per_launch", "valu_active_quad_cycles_per_launch", "valu_busy_frac")]
    return None if None in vals else tuple(vals)


def roofline(kernel: str, workload: str, bytes_per_node: float, nodes: int, launch_s: float,
             steps_per_launch: int, pass_rows: int):
    """Roofline of one launch of the dominant kernel.  achieved / frac: the pass's
    algorithmic bytes (one read of the state and the porosity, one write of the state:
    bytes_per_node per node however many steps the launch takes) over the measured
    launch time, against the HBM peak.  alu: the VALU instructions the counters count
    per launch at the chip's non-packed issue rate, a time floor of its own; frac_binding
    is the larger floor over the launch time."""
    ach = bytes_per_node * nodes / launch_s / 1e9
    traffic = measured_traffic(workload, kernel)
    valu = measured_valu(workload, kernel)
    out = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
           "frac": round(ach / PEAK_HBM_GBPS, 4), "traffic": traffic, "kernel": kernel,
           "steps_per_launch": steps_per_launch, "pass_rows": pass_rows,
           "bytes_per_node_per_launch": bytes_per_node,
           "bytes_per_node_step": round(bytes_per_node / steps_per_launch, 3),
           "launch_us": round(launch_s * 1e6, 2),
           "one_step_equivalent_GBps": round(ach * steps_per_launch, 1)}
    if traffic is not None:
        out["traffic_GBps"] = round(traffic / launch_s / 1e9, 1)
        out["traffic_frac"] = round(traffic / launch_s / 1e9 / PEAK_HBM_GBPS, 4)
    hbm_floor = bytes_per_node * nodes / (PEAK_HBM_GBPS * 1e9)
    if valu is not None:
        insts, quads, busy = valu
        # one quad-cycle of a SIMD per full-rate instruction (transcendental and FP64
        # instructions take more): the VALU-active quad-cycles over 1024 SIMDs at 2.4 GHz
        valu_floor = quads / PEAK_VALU_WAVE_INSTS
        out["alu"] = {"valu_wave_insts_per_launch": insts,
                      "valu_active_quad_cycles_per_launch": quads,
                      "peak_quad_cycles_per_s": PEAK_VALU_WAVE_INSTS,
                      "time_floor_us": round(valu_floor * 1e6, 2),
                      "frac": round(valu_floor / launch_s, 4),
                      "valu_busy_frac_counter": busy,
                      "valu_insts_per_node_step": round(insts * 64 / (nodes * steps_per_launch), 1)}
        out["frac_binding"] = round(max(hbm_floor, valu_floor) / launch_s, 4)
        out["binding"] = "alu" if valu_floor > hbm_floor else "hbm"
    return out


def copy_bandwidth_gbps(torch, nbytes=2 << 30, reps=10) -> float:
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / dt / 1e9


def make_workload(name: str):
    from paper_1406_6438_amd import workloads as W
    return {"box4096_f32": W.BOX_4096_F32, "box8192_f16": W.BOX_8192_F16,
            "channel_f64": W.CHANNEL_64x32}[name]


def lbm_params(w, lbm, Lx=None, Ly=None):
    return lbm.Params(Lx=Lx or w.Lx, Ly=Ly or w.Ly, tau=w.tau,
                      bc_y=lbm.BC_BOUNCEBACK if w.walls_y else lbm.BC_PERIODIC,
                      storage=lbm.STORAGE[w.storage], d_p=w.d_p, G=(w.Gx, w.Gy),
                      rho0=w.rho0, fp16_scale_log2=10)


def cast_eps(eps, storage):
    import numpy as np
    return eps if storage == "f64" else eps.astype(np.float32).astype(np.float64)

def oracle_params(spec: dict):
    """oracle.Params from a plain description: the GPU legs describe their accuracy
    samples as data, and only the CPU-baseline leg touches the oracle."""
    import oracle
    kw = dict(spec)
    for k in ("bc_x", "bc_y"):
        kw[k] = {"periodic": oracle.PERIODIC, "wall": oracle.WALL, "open": oracle.OPEN,
                 "inout": oracle.INOUT}[kw.get(k, "periodic")]
    return oracle.Params(**kw)


def cpu_baseline_leg(w, eps, budget_s: float, jobs: list):
    """The FP64 oracle on the host cores: (1) the full lattice of the main workload for as
    many whole steps as fit in the time budget (the reported rate); (2) the accuracy
    samples the GPU legs ran (each job: oracle parameters, porosity, steps and kind, "u"
    for the final velocity field or "grad" for the outlet-flux gradient), timed too.
    Returns (the cpu_baseline dict, the oracle result of every job)."""
    import oracle
    spec = {"Lx": w.Lx, "Ly": w.Ly, "tau": w.tau, "bc_y": "wall" if w.walls_y else "periodic",
            "d_p": w.d_p, "Gx": w.Gx, "Gy": w.Gy, "rho0": w.rho0}
    p = oracle_params(spec)
    threads = oracle.default_threads()
    e = cast_eps(eps, w.storage)
    f = oracle.init(p, e)
    t0 = time.perf_counter()
    f = oracle.steps(p, e, f, 1, threads)
    t1 = time.perf_counter() - t0
    k = max(1, min(int(budget_s / max(t1, 1e-9)), 100000))
    t0 = time.perf_counter()
    oracle.steps(p, e, f, k, threads)
    dt = time.perf_counter() - t0
    del f
    # the same on one thread, on a budget of its own (a few steps of the full lattice)
    f = oracle.init(p, e)
    t0 = time.perf_counter()
    f = oracle.steps(p, e, f, 1, 1)
    t1s = time.perf_counter() - t0
    k1 = max(1, min(int(budget_s / 3.0 / max(t1s, 1e-9)), 100000))
    t0 = time.perf_counter()
    oracle.steps(p, e, f, k1, 1)
    dt1 = time.perf_counter() - t0
    del f
    out = {"value": round(w.Lx * w.Ly * k / dt / 1e6, 3), "unit": "MLUPS", "cores": threads,
           "kind": "oracle",
           "sample": f"{w.Lx}x{w.Ly} lattice of the same workload, {k} FP64 steps after 1 "
                     f"untimed step ({dt:.1f} s), OpenMP over rows on {threads} threads (the "
                     f"host share: OMP_NUM_THREADS, else the CPU count capped at 16)",
           "host_cpu_count": os.cpu_count(),
           "one_thread": {"value": round(w.Lx * w.Ly * k1 / dt1 / 1e6, 3), "unit": "MLUPS",
                          "steps": k1, "seconds": round(dt1, 2)},
           "build": "gcc " + " ".join(oracle.CFLAGS),
           "accuracy_samples": []}
    log(f"[bench] cpu baseline {out['value']} MLUPS on {threads} threads")
    results = []
    for job in jobs:
        pj = oracle_params(job["params"])
        t0 = time.perf_counter()
        if job["kind"] == "grad":
            J, g = oracle.grad_outlet_flux(pj, job["eps"], job["steps"], threads)
            res = {"J": J, "grad": g}
        else:
            m = oracle.moments(pj, job["eps"], oracle.run(pj, job["eps"], job["steps"]))
            res = {"ux": m["ux"], "uy": m["uy"]}
        dtj = time.perf_counter() - t0
        results.append(res)
        nodes = job["params"]["Lx"] * job["params"]["Ly"]
        out["accuracy_samples"].append({"name": job["name"], "seconds": round(dtj, 2),
                                        "MLUPS": round(nodes * job["steps"] / dtj / 1e6, 2)})
        log(f"[bench] oracle sample {job['name']}: {dtj:.1f} s")
    return out, results


def rel_l2(a, b) -> float:
    import numpy as np
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def speed_error(gpu, res) -> float:
    """rel. L2 of |u| of a GPU run against the oracle's result of the same sample."""
    import numpy as np
    return rel_l2(np.hypot(*gpu), np.hypot(res["ux"], res["uy"]))


def crop_sample(w, lbm, steps: int, plan):
    """The GPU run of the top-left 512^2 crop of the workload's porosity, run periodic
    in the launch plan of the timed run (plan = steps per pass, rows per chunk of the
    multi-step pass), and the matching oracle job."""
    import dataclasses
    from paper_1406_6438_amd import workloads as W
    n = W.CROP
    eps = cast_eps(W.crop_porosity(w, n), w.storage)
    p = dataclasses.replace(lbm_params(w, lbm, n, n), steps_per_pass=plan[0],
                            pass_rows=plan[1])
    s = lbm.Solver(p, eps)
    s.step(steps)
    m = s.moments(want_diag=False)
    gpu = (m["ux"].double().cpu().numpy(), m["uy"].double().cpu().numpy())
    s.close()
    job = {"name": f"{w.name} crop {n}x{n}, {steps} steps", "kind": "u", "steps": steps,
           "eps": eps, "params": {"Lx": n, "Ly": n, "tau": w.tau, "d_p": w.d_p, "Gx": w.Gx,
                                  "Gy": w.Gy, "rho0": w.rho0}}
    return gpu, job


def time_sweep(w, lbm, torch, steps: int, warmup: int, single_steps: int = 0, reps: int = 5):
    """Times `steps` steps `reps` times in a row (after `warmup` untimed steps) with HIP
    events on the library's stream, one pair around the whole run and one around every
    launch (each lbm_vans_step call below takes exactly one launch).  Returns a dict:
    seconds of every repetition and their median, the mean duration of the launches
    that take the plan's full steps per pass (the dominant kernel), the final
    diagnostics record, the porosity, the seconds per step when every step is its own
    launch (k_sweep_vec; None without single_steps) and the launch plan (most steps per
    pass, rows per chunk of the multi-step pass)."""
    import statistics
    eps = w.porosity()
    s = lbm.Solver(lbm_params(w, lbm), cast_eps(eps, w.storage))
    plan = s.pass_plan
    spl = plan[0]
    log(f"[bench] {w.name}: warmup {warmup} steps; plan {plan}")
    s.step(warmup)
    torch.cuda.synchronize()
    Ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    rep_s, launch_s = [], []
    for _ in range(reps):
        e0, e1 = Ev(), Ev()
        marks = []
        torch.cuda.synchronize()
        e0.record(s.stream)
        k = 0
        while k < steps:
            m = min(spl, steps - k)
            a, b = Ev(), Ev()
            a.record(s.stream)
            s.step(m)
            b.record(s.stream)
            marks.append((m, a, b))
            k += m
        e1.record(s.stream)
        torch.cuda.synchronize()
        rep_s.append(e0.elapsed_time(e1) / 1e3)
        launch_s += [a.elapsed_time(b) / 1e3 for m, a, b in marks if m == spl]
    single = None
    if single_steps > 0:
        e0, e1 = Ev(), Ev()
        e0.record(s.stream)
        for _ in range(single_steps):
            s.step(1)
        e1.record(s.stream)
        torch.cuda.synchronize()
        single = e0.elapsed_time(e1) / 1e3 / single_steps
    diag = s.moments()["diag"]
    s.close()
    del s
    torch.cuda.empty_cache()
    med = statistics.median(rep_s)
    launch = sum(launch_s) / len(launch_s) if launch_s else med / steps * spl
    log(f"[bench] {w.name}: {steps} steps x {reps}: median {med * 1e3:.2f} ms "
        f"({', '.join(f'{t * 1e3:.2f}' for t in rep_s)}); {len(launch_s)} launches of {spl} "
        f"steps, {launch * 1e6:.2f} us each"
        + (f"; one step per launch: {single * 1e6:.1f} us/step" if single else ""))
    return {"median_s": med, "rep_s": rep_s, "launch_s": launch, "launches": len(launch_s),
            "diag": diag, "eps": eps, "single_s": single, "plan": plan}


def adjoint_params(lbm, w, Lx=None, Ly=None):
    from paper_1406_6438_amd import workloads as W
    U = W.ADJOINT_U_IN
    return lbm.Params(Lx=Lx or w.Lx, Ly=Ly or w.Ly, tau=w.tau, bc_x=lbm.BC_INOUT,
                      bc_y=lbm.BC_BOUNCEBACK, storage=lbm.STORAGE[w.storage], d_p=w.d_p,
                      rho0=w.rho0, u0=(U, 0.0), u_in=U, rho_out=W.ADJOINT_RHO_OUT)


def adjoint_leg(lbm, torch, no_accuracy: bool):
    """dJ/deps of the outlet mass flux on the 1024x512 channel (velocity inlet, pressure
    outlet) after 4000 steps
    (checkpoints every 200): wall time of the whole gradient (forward with checkpoints,
    per-segment recompute, reverse), and the plain FP32 forward on the same workload.
    Returns (leg dict, accuracy sample: GPU gradient, oracle job, description)."""
    from paper_1406_6438_amd import workloads as W
    import numpy as np
    w = W.ADJOINT_CHANNEL
    K = W.ADJOINT_CKPT
    eps = cast_eps(w.porosity(), w.storage)
    p = adjoint_params(lbm, w)
    s = lbm.Solver(p, eps)
    log(f"[bench] adjoint: {w.name}, {w.steps} steps, checkpoints every {K}")
    s.grad(50, K)                                   # warm-up (first launches)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, g = s.grad(w.steps, K)
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    # the plain forward of the same workload on the same GPU
    s2 = lbm.Solver(p, eps)
    s2.step(20)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s2.stream)
    s2.step(w.steps)
    e1.record(s2.stream)
    torch.cuda.synchronize()
    t_fwd = e0.elapsed_time(e1) / 1e3
    s2.close()
    s.close()
    del s, s2, g
    torch.cuda.empty_cache()
    cells = w.Lx * w.Ly
    m_grad = cells * w.steps / t_grad / 1e6
    m_fwd = cells * w.steps / t_fwd / 1e6
    # algorithmic bytes per node-step: forward with checkpoints (76) + recompute (76)
    # + the FP64 reverse step (gather of the FP32 state 36, FP32 porosity 4, FP32
    # adjoints in 36 and out 36, three FP64 accumulators read and written 48) + the
    # checkpoint copy (read and write of 36 B every K steps)
    bps = 76 + 76 + 36 + 4 + 36 + 36 + 48 + 72 / K
    out = {"workload": w.name, "steps": w.steps, "ckpt_every": K, "J": J,
           "value": round(m_grad, 2), "unit": "MLUPS (forward node-steps per second of the "
                                                  "whole gradient computation)",
           "seconds": round(t_grad, 4), "fwd_fp32_same_gpu_MLUPS": round(m_fwd, 2),
           "vs_fp32_forward_same_gpu": round(m_grad / m_fwd, 3),
           "bytes_per_node_step": round(bps, 2),
           "achieved_GBps": round(bps * cells * w.steps / t_grad / 1e9, 1)}
    log(f"[bench] adjoint: {t_grad:.3f} s, {m_grad:.0f} MLUPS-equivalent; forward {m_fwd:.0f} MLUPS")
    sample = None
    if not no_accuracy:
        n, L = 300, (96, 40)
        sp = lbm.Params(**{**p.__dict__, "Lx": L[0], "Ly": L[1], "d_p": 60.0})
        e = cast_eps(W.grf_porosity(L[0], L[1], seed=43, ell=6.0, lo=0.4, hi=1.0), "f32")
        sg = lbm.Solver(sp, e)
        Jg, gg = sg.grad(n, 50)
        gg = gg.cpu().numpy()
        sg.close()
        U = W.ADJOINT_U_IN
        job = {"name": f"gradient {L[0]}x{L[1]} channel, {n} steps", "kind": "grad",
               "steps": n, "eps": e,
               "params": {"Lx": L[0], "Ly": L[1], "tau": w.tau, "bc_x": "inout", "bc_y": "wall",
                          "d_p": 60.0, "rho0": w.rho0, "u0x": U, "u_in": U,
                          "rho_out": W.ADJOINT_RHO_OUT}}
        sample = (gg, job, f"{L[0]}x{L[1]} channel of the same kind (velocity inlet, pressure "
                           f"outlet), {n} steps, checkpoints every 50")
    return out, sample


def ensemble_leg(lbm, torch, no_accuracy: bool, steps: int, warmup: int, grad: bool):
    """The 64-member ensemble of uneven channels (velocity inlet, pressure outlet; FP32):
    launch shape picked by the
    library's autotuner (single-step launches of each width and grid, the two- and the
    three-step pass), then `steps` batched steps (replayed as 24-step graphs) timed with
    HIP events; the same steps as plain launches; the gradient of every member's outlet
    flux after 2000 steps (checkpoints every 45).
    Returns (leg dict, accuracy sample of the smallest member or None)."""
    import numpy as np
    from paper_1406_6438_amd import workloads as W
    U = W.ENSEMBLE_U
    members = W.ensemble()
    cells = sum(m.Lx * m.Ly for m in members)
    log(f"[bench] ensemble: {len(members)} members, {cells / 1e6:.2f}M nodes")

    def params(m):
        return lbm.Params(Lx=m.Lx, Ly=m.Ly, tau=m.tau, bc_x=lbm.BC_INOUT,
                          bc_y=lbm.BC_BOUNCEBACK, storage=lbm.F32_SHIFTED, d_p=m.d_p,
                          u0=(U, 0.0), u_in=U, rho_out=1.0)

    eps = [cast_eps(m.porosity(), "f32") for m in members]
    sv = [lbm.Solver(params(m), e) for m, e in zip(members, eps)]
    b = lbm.Batch(sv)
    best, trials = b.tune(reps=5)
    log(f"[bench] ensemble tuned: {best}")
    b.step(warmup)
    torch.cuda.synchronize()

    def timed(n):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(b.stream)
        b.step(n)
        e1.record(b.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    t_graph = timed(steps)
    b.configure(best["vec"], best["grid"], 0, best["steps_per_pass"], best["pass_rows"])
    t_plain = timed(steps)
    b.configure(best["vec"], best["grid"], best["graph_steps"], best["steps_per_pass"],
                best["pass_rows"])
    spl, rows = b.pass_plan
    bpn = algorithmic_bytes_per_node("f32")
    # the graphs replay launches of spl steps: the time of one is the time per step x spl
    roof = roofline(BATCH_KERNEL[spl], "ensemble64_f32" if len(members) == 64 else "-", bpn,
                    cells, t_graph / steps * spl, spl, rows)
    roof["launch_time"] = "time per step of the graph replays x steps per launch"
    out = {"workload": f"ensemble_{len(members)}_channels_f32", "members": len(members),
           "nodes": cells, "Lx_range": [min(m.Lx for m in members), max(m.Lx for m in members)],
           "steps": steps, "value": round(cells * steps / t_graph / 1e6, 2), "unit": "MLUPS",
           "ms_per_step": round(t_graph * 1e3 / steps, 5),
           "plain_launches_ms_per_step": round(t_plain * 1e3 / steps, 5),
           "tuned": best, "trials": trials, "roofline": roof}
    ach = roof["achieved"]
    log(f"[bench] ensemble: {out['value']:.0f} MLUPS, {ach:.0f} GB/s (graphs), "
        f"{cells * steps / t_plain / 1e6:.0f} MLUPS plain launches")
    if grad:
        # gradient of every member's outlet flux
        K = W.ENSEMBLE_CKPT
        nbytes = lbm.lbm_vans_batch_grad_work_bytes(b.b, lbm.OBJ_OUTLET_FLUX,
                                                    W.ENSEMBLE_STEPS, K)
        b.grad(20, 10)                                  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J, g = b.grad(W.ENSEMBLE_STEPS, K)
        torch.cuda.synchronize()
        t_grad = time.perf_counter() - t0
        del g
        m_grad = cells * W.ENSEMBLE_STEPS / t_grad / 1e6
        out["gradient"] = {"steps": W.ENSEMBLE_STEPS, "ckpt_every": K,
                           "seconds": round(t_grad, 3), "value": round(m_grad, 2),
                           "unit": "MLUPS (forward node-steps per second of the whole gradient)",
                           "vs_forward_same_gpu": round(m_grad / out["value"], 3),
                           "workspace_GB": round(nbytes / 1e9, 2),
                           "J_min_max": [min(J), max(J)]}
        log(f"[bench] ensemble gradient: {t_grad:.2f} s, {m_grad:.0f} MLUPS-equivalent, "
            f"workspace {nbytes / 1e9:.1f} GB")
    _close_all(sv, b)
    sample = None
    if not no_accuracy:
        k = int(np.argmin([m.Lx * m.Ly for m in members]))
        m = members[k]
        sg = lbm.Solver(params(m), eps[k])
        sg.step(W.ENSEMBLE_STEPS)
        mg = sg.moments(want_diag=False)
        gpu = (mg["ux"].double().cpu().numpy(), mg["uy"].double().cpu().numpy())
        sg.close()
        job = {"name": f"ensemble member {k} ({m.Lx}x{m.Ly}), {W.ENSEMBLE_STEPS} steps",
               "kind": "u", "steps": W.ENSEMBLE_STEPS, "eps": eps[k],
               "params": {"Lx": m.Lx, "Ly": m.Ly, "tau": m.tau, "bc_x": "inout", "bc_y": "wall",
                          "d_p": m.d_p, "u0x": U, "u_in": U, "rho_out": 1.0}}
        sample = (gpu, job, f"member {k} ({m.Lx}x{m.Ly}, the smallest), "
                            f"{W.ENSEMBLE_STEPS} steps")
    torch.cuda.empty_cache()
    return out, sample


def eq_velocity_profile(c, L: int, eps: float):
    """Solution of the paper's eq. (velocity) for a Couette case, read with d^2/dy^2 and
    |u| u: nu u'' - (eps nu / K) u - (eps^2 F_eps / sqrt(K)) |u| u = 0, u = 0 on the plate
    at y = -1/2, u = U on the plate at y = L - 1/2, at the node rows y + 1/2."""
    import math
    import numpy as np
    from scipy.integrate import solve_bvp
    a = eps * c.nu / c.K
    b = eps ** 2 * (1.75 / math.sqrt(150.0 * eps ** 3)) / math.sqrt(c.K)

    def rhs(_, Y):
        return np.vstack([Y[1], (a * Y[0] + b * np.abs(Y[0]) * Y[0]) / c.nu])

    s = np.linspace(0.0, float(L), 401)
    sol = solve_bvp(rhs, lambda ya, yb: np.array([ya[0], yb[0] - c.U]), s,
                    np.vstack([c.U * s / L, np.full_like(s, c.U / L)]), tol=1e-10,
                    max_nodes=200000)
    return sol.sol(np.arange(L) + 0.5)[0]


def couette_leg(lbm, torch):
    """The paper's Couette experiment on the GPU (FP64, 80 x 80, porosity 0.1, upper
    plate sliding, 160000 steps per case): the largest deviation of the profile at
    x = H/2 from the solution of eq. (velocity), relative to the plate velocity."""
    import numpy as np
    from paper_1406_6438_amd import workloads as W
    L, eps0, n = W.COUETTE_L, W.COUETTE_EPS, W.COUETTE_STEPS
    cases = []
    t0 = time.perf_counter()
    for Re, Da in W.COUETTE_CASES:
        c = W.couette_case(Re, Da)
        p = lbm.Params(Lx=L, Ly=L, tau=c.tau, bc_y=lbm.BC_BOUNCEBACK, storage=lbm.F64,
                       d_p=c.d_p, u_wall=(0.0, c.U))
        s = lbm.Solver(p, np.full((L, L), eps0))
        s.step(n)
        ux = s.moments(want_diag=False)["ux"].cpu().numpy()
        s.close()
        err = float(np.abs(ux[:, L // 2] - eq_velocity_profile(c, L, eps0)).max() / c.U)
        cases.append({"Re": Re, "Da": Da, "tau": c.tau, "U": c.U,
                      "max_err_vs_eq_velocity_over_U": err})
        log(f"[bench] couette Re {Re} Da {Da}: max |u - eq.(velocity)| / U = {err:.2e}")
    return {"lattice": f"{L}x{L}", "porosity": eps0, "steps": n, "storage": "f64",
            "seconds": round(time.perf_counter() - t0, 2), "cases": cases}


def _close_all(solvers, batch):
    batch.close()
    for s in solvers:
        s.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="box4096_f32",
                    choices=["box4096_f32", "box8192_f16", "channel_f64"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle on the host (and with it every accuracy figure)")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-fp16", action="store_true",
                    help="skip the FP16-storage leg (8192^2 box) reported beside the main line")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the gradient leg (1024x512 open channel) reported beside the main line")
    ap.add_argument("--no-ensemble", action="store_true",
                    help="skip the ensemble leg (64 uneven open channels) reported beside the main line")
    ap.add_argument("--no-couette", action="store_true",
                    help="skip the paper's Couette experiment reported beside the main line")
    ap.add_argument("--ensemble-steps", type=int, default=2000,
                    help="timed steps of the ensemble leg (--no-adjoint also skips its gradient)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (the "
              "domain decomposition is a design, not code); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    want_acc = not args.no_accuracy and not args.no_cpu_baseline

    import torch
    from paper_1406_6438_amd import lbm

    lbm.load()
    w = make_workload(args.workload)
    log(f"[bench] workload {w.name}: {w.Lx}x{w.Ly}, storage {w.storage}")
    ts = time_sweep(w, lbm, torch, args.steps, args.warmup, single_steps=200)
    gpu_s, diag, eps, single_s, plan = (ts["median_s"], ts["diag"], ts["eps"], ts["single_s"],
                                        ts["plan"])
    cells = w.Lx * w.Ly
    mlups = cells * args.steps / gpu_s / 1e6
    bpn = algorithmic_bytes_per_node(w.storage)
    spl = plan[0]                       # steps per launch of the timed run
    roof = roofline(MULTI_KERNEL[spl], args.workload, bpn, cells, ts["launch_s"], spl, plan[1])
    copy_bw = copy_bandwidth_gbps(torch)
    roof["device_copy_GBps"] = round(copy_bw, 1)
    log(f"[bench] {mlups:.1f} MLUPS; {roof['kernel']} {roof['launch_us']} us per launch, "
        f"{roof['achieved']} GB/s of pass bytes ({roof['frac']:.3f} of peak); device copy "
        f"{copy_bw:.1f} GB/s")

    # accuracy samples: (target dict, GPU result, oracle job, description)
    samples = []
    acc = None
    if want_acc and w.storage != "f64":
        gpu, job = crop_sample(w, lbm, w.steps, plan)
        acc = {"kernel": roof["kernel"], "steps_per_pass": plan[0], "pass_rows": plan[1]}
        samples.append((acc, gpu, job, f"top-left 512x512 crop of the porosity field, periodic, "
                                       f"{w.steps} steps in the timed run's launch plan"))

    fp16 = None
    if not args.no_fp16 and args.workload == "box4096_f32":
        w16 = make_workload("box8192_f16")
        steps16 = 300
        t16 = time_sweep(w16, lbm, torch, steps16, args.warmup, single_steps=100)
        g16, d16, s16, plan16 = t16["median_s"], t16["diag"], t16["single_s"], t16["plan"]
        cells16 = w16.Lx * w16.Ly
        m16 = cells16 * steps16 / g16 / 1e6
        b16 = algorithmic_bytes_per_node("f16")
        fp16 = {"workload": w16.name, "value": round(m16, 2), "unit": "MLUPS", "steps": steps16,
                "reps": len(t16["rep_s"]), "ms_per_step": round(g16 * 1e3 / steps16, 5),
                "roofline": roofline(MULTI_KERNEL[plan16[0]], "box8192_f16", b16, cells16,
                                     t16["launch_s"], plan16[0], plan16[1]),
                "single_step": {"kernel": "k_sweep_vec", "value": round(cells16 / s16 / 1e6, 2),
                                "unit": "MLUPS", "frac": round(b16 * cells16 / s16 / 1e9 /
                                                                PEAK_HBM_GBPS, 4)},
                "vs_fp32_same_gpu": round(m16 / mlups, 3),
                "nonfinite_nodes": d16[6], "accuracy": None}
        log(f"[bench] fp16: {m16:.1f} MLUPS, {fp16['roofline']['achieved']} GB/s of pass bytes")
        if want_acc:
            gpu, job = crop_sample(w16, lbm, w16.steps, plan16)
            fp16["accuracy"] = {"kernel": fp16["roofline"]["kernel"],
                                "steps_per_pass": plan16[0], "pass_rows": plan16[1]}
            samples.append((fp16["accuracy"], gpu, job, "top-left 512x512 crop of the 8192^2 "
                                                        f"porosity field, periodic, {w16.steps} "
                                                        "steps in the timed run's launch plan"))

    adj = None
    if not args.no_adjoint and args.workload == "box4096_f32":
        adj, smp = adjoint_leg(lbm, torch, not want_acc)
        if smp is not None:
            adj["accuracy"] = {}
            samples.append((adj["accuracy"], smp[0], smp[1], smp[2]))

    ens = None
    if not args.no_ensemble and args.workload == "box4096_f32":
        ens, smp = ensemble_leg(lbm, torch, not want_acc, args.ensemble_steps, args.warmup,
                                not args.no_adjoint)
        if smp is not None:
            ens["accuracy"] = {}
            samples.append((ens["accuracy"], smp[0], smp[1], smp[2]))

    couette = None
    if not args.no_couette and args.workload == "box4096_f32":
        couette = couette_leg(lbm, torch)

    cpu = None
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline (~{args.cpu_seconds:.0f} s) and {len(samples)} oracle samples")
        cpu, results = cpu_baseline_leg(w, eps, args.cpu_seconds, [s[2] for s in samples])
        for (target, gpu, job, desc), res in zip(samples, results):
            if job["kind"] == "grad":
                target["rel_l2_grad_vs_fp64_oracle_adjoint"] = rel_l2(gpu, res["grad"])
            else:
                target["rel_l2_u_vs_fp64_oracle"] = speed_error(gpu, res)
            target["sample"] = desc
            log(f"[bench] accuracy {job['name']}: {target}")

    out = {
        "metric": "MLUPS & % HBM roofline (D2Q9 FP32 fwd, FP16-store, adjoint) at fixed error",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(gpu_s * 1e3 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "f16": "f16-store/f32"}[w.storage],
        "data": "synthetic",
        "config": {"workload": w.name, "Lx": w.Lx, "Ly": w.Ly, "tau": w.tau,
                   "porosity": "GRF l=16 in [0.3,1.0]" if w.eps_kind == "grf" else f"uniform {w.eps_value}",
                   "d_p": round(w.d_p, 4), "G": [w.Gx, w.Gy], "storage": w.storage,
                   "boundaries": "periodic" if not w.walls_y else "periodic x, bounce-back y"},
        "roofline": roof,
        "timing": {"reps": len(ts["rep_s"]), "statistic": "median",
                   "rep_ms": [round(t * 1e3, 4) for t in ts["rep_s"]],
                   "launches_timed": ts["launches"]},
        "single_step": None if single_s is None else {
            "kernel": "k_sweep_vec", "value": round(cells / single_s / 1e6, 2), "unit": "MLUPS",
            "achieved": round(bpn * cells / single_s / 1e9, 1),
            "frac": round(bpn * cells / single_s / 1e9 / PEAK_HBM_GBPS, 4),
            "launch_us": round(single_s * 1e6, 2)},
        "accuracy": acc,
        "fp16_store": fp16,
        "adjoint": adj,
        "ensemble": ens,
        "couette": couette,
        "cpu_baseline": cpu,
        "mass_check": {"sum_eps_rho": diag[0], "nonfinite_nodes": diag[6]},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
