"""Benchmark of the Taylor--Couette time step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Workload (default tc-heated-n64): heated Taylor--Couette, eta = 0.71,
Re_i = 100, Re_o = 0, Ra = 1e4, Pr = 0.7, N_r = 64, 64 x 127 Fourier modes
(192 x 192 padded grid), seeded synthetic initial state, dynamic time step
(CFL 0.5).  One step = nonlinear term + predictor solve + nonlinear term +
corrector solve.  Prints one JSON line: mixed-precision steps/s (value), the
FP64 steps/s on the same grid, the mixed-vs-FP64 error per field, the
roofline figures of the dominant kernel (HIP events on the library stream)
and the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("time steps/s per grid, mixed vs FP64 at stated error; "
          "adjoint/forward cost ratio")
HBM_PEAK_GBS = 8000.0


def _field_bytes(w):
    return w["N_r"] * w["M_theta"] * w["M_z"] * 16


def kernel_bytes(name, w, prec):
    """Algorithmic HBM bytes of one launch of each kernel (compulsory reads and
    writes of its inputs and outputs, each array counted once)."""
    F = 4 if w["Ra"] != 0 else 3
    n_in = 9 if F == 4 else 6
    S = _field_bytes(w)
    esz = 8 if prec == "mixed" else 16
    K = (w["M_z"] - 1) // 2
    I = w["N_r"] * w["M_theta"] * 3 * (K + 1) * esz
    kp1 = K + 1
    fac_row = 9 * 8
    nops_v = (w["M_theta"] + 1) * kp1
    nops_m = w["M_theta"] * kp1
    if name == "zinv":
        return F * S + n_in * I
    if name == "theta":
        return (n_in + F) * I
    if name == "zfwd":
        return F * I + F * S + (S if F == 4 else 0)
    if name == "rhs":
        return 3 * F * S + F * S
    if name == "div":
        return 3 * S + S
    if name == "sweep_pt":
        b = 2 * S + nops_m * w["N_r"] * fac_row
        if F == 4:
            b += 2 * S + nops_m * w["N_r"] * fac_row
        return b
    nmodes = w["M_theta"] * w["M_z"]
    if name == "vel_rhs":
        # right sides f - grad p0 in place: read 3S + p0, write 3S
        return 3 * S + S + 3 * S
    if name == "sweep_vel":
        # three Helmholtz sweeps: read 3S, write 3S, velocity factors
        return 3 * S + 3 * S + nops_v * w["N_r"] * fac_row
    if name == "influence":
        return 3 * 18 * nmodes * 16 + nops_m * 32 + nmodes * 32
    if name == "finalize":
        # the step's variant: no pressure (read X, lambda, six response
        # columns; write the state)
        return F * S + nmodes * 32 + nops_m * 6 * w["N_r"] * 8 + F * S
    return 0


# device kernel behind each timed stage of the default workload (mixed
# precision, the reported value; 192-point transforms)
DEVICE_KERNEL_WORKLOAD = "tc-heated-n64"
DEVICE_KERNEL = {"zinv": "nsc::k_zinv<float, 192>", "theta": "nsc::k_theta<float, true, 192>",
                 "zfwd": "nsc::k_zfwd<float, 192>", "rhs": "nsc::k_rhs<4>", "div": "nsc::k_div2<2>",
                 "sweep_pt": "nsc::k_sweep<true, 0, 64>", "sweep_vel": "nsc::k_sweep<true, 1, 64>",
                 "vel_rhs": "nsc::k_vel_rhs<1>", "finalize": "nsc::k_finalize<false>",
                 "influence": "nsc::k_influence"}


def source_digest():
    """SHA-256 over the HIP/C++ sources of the library (sorted by name): the
    traffic counters of a committed profile apply only to the same kernels."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1908_00587_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def committed_traffic(wname, stage):
    """HBM bytes per launch of a stage's kernel from the committed counter
    summary profiles/hbm-traffic_<workload>.txt (FETCH_SIZE + WRITE_SIZE,
    each scaled by the calibration kernel's reading), or None when the file
    is missing or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"hbm-traffic_{wname}.txt")
    if wname != DEVICE_KERNEL_WORKLOAD or not os.path.exists(path) or stage not in DEVICE_KERNEL:
        return None
    digest, rows = None, {}
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) == 2 and parts[0] == "source_sha256":
                digest = parts[1]
            elif len(parts) >= 2 and parts[0] == "bytes_per_launch":
                rows[" ".join(parts[2:])] = float(parts[1])
    if digest != source_digest():
        return None
    return rows.get(DEVICE_KERNEL[stage])


def calibration_copy():
    """A plain streaming kernel of known size (dst = -src: 256 MiB read,
    256 MiB written) after a 1 GiB fill that evicts the caches, so that the
    FETCH_SIZE / WRITE_SIZE counters of a profiled run can be scaled to bytes."""
    import torch
    src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    evict = torch.empty(128 * 1024 * 1024, dtype=torch.float64, device="cuda")
    evict.fill_(2.0)
    torch.cuda.synchronize()
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst, evict


def run_gpu(args, wname):
    import torch

    import paper_1908_00587_amd as nsc
    from paper_1908_00587_amd.workloads import WORKLOADS, amplitudes, params

    w = WORKLOADS[wname]
    torch.cuda.set_device(0)
    ctx = nsc.Context(*params(wname))
    amps = amplitudes(wname).cuda()
    u0 = ctx.initial_state(amps)
    dt_max = w["dt"]
    if w["dynamic"]:
        _, c = ctx.nonlinear(u0, cfl=True)
        dt0 = min(dt_max, 0.5 * float(c.cpu()[0]))
    else:
        dt0 = w["dt"]

    def run(prec, steps, warmup, profile=False):
        ctx.set_precision(prec)
        ctx.set_timestep(dt=dt0, dynamic=w["dynamic"], cfl=0.5, dt_max=dt_max)
        u = u0.clone()
        dt = dt0
        for _ in range(warmup):
            dt = ctx.step(u, dt)
        torch.cuda.synchronize()
        if profile:
            ctx.timings()
            ctx.set_profiling(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            dt = ctx.step(u, dt)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        tim = None
        if profile:
            ctx.set_profiling(False)
            tim = ctx.timings()
        return el, u, dt, tim

    K, W = args.steps, args.warmup
    # untimed warm-up run of both precisions (first factorisation, code load)
    run("fp64", 2, 0)
    run("mixed", 2, 0)
    t64, u64, dt64, _ = run("fp64", K, W)
    tmx, umx, dtmx, _ = run("mixed", K, W)
    # per-kernel durations: same K steps again, each kernel between HIP events
    _, _, _, tim = run("mixed", min(K, 50), W, profile=True)

    def wnorm(x):
        return float(torch.linalg.vector_norm(x))

    err = {}
    names = ["u_r", "u_theta", "u_z", "T"][:ctx.F]
    for f, nm in enumerate(names):
        err[nm] = wnorm(umx[f] - u64[f]) / max(wnorm(u64[f]), 1e-300)

    # dominant kernel and its roofline
    best = None
    for kname, (ms, cnt) in tim.items():
        if cnt == 0 or kname in ("factor", "remap"):
            continue
        if best is None or ms > best[1]:
            best = (kname, ms, cnt)
    kname, ms, cnt = best
    avg_s = ms / cnt / 1e3
    byt = kernel_bytes(kname, w, "mixed")
    achieved = byt / avg_s / 1e9
    per_kernel = {k: {"ms_total": round(v[0], 4), "launches": v[1],
                      "avg_us": round(1e3 * v[0] / v[1], 3) if v[1] else None,
                      "GBps": round(kernel_bytes(k, w, "mixed") / (v[0] / v[1] / 1e3) / 1e9, 1)
                      if v[1] and kernel_bytes(k, w, "mixed") else None}
                  for k, v in tim.items()}
    ctx.close()
    calibration_copy()
    return dict(K=K, W=W, t64=t64, tmx=tmx, err=err, dt_end=(dt64, dtmx), dominant=kname,
                avg_us=avg_s * 1e6, bytes=byt, achieved=achieved, per_kernel=per_kernel)


def run_adjoint(steps, wname="tc-adjoint-n64", ckpt=20):
    """Adjoint/forward cost ratio on the adjoint workload (eta = 0.71,
    Re_i = 200, N_r = 64, 32 x 63 modes, dt = 5e-4): wall time of the
    gradient pass (checkpoint recompute + vector-Jacobian products) over the
    wall time of the plain forward rollout of the same steps, both after an
    untimed warm-up of each."""
    import torch

    import paper_1908_00587_amd as nsc
    from paper_1908_00587_amd.adjoint import rollout, rollout_energy
    from paper_1908_00587_amd.workloads import WORKLOADS, amplitudes, params

    w = WORKLOADS[wname]
    ctx = nsc.Context(*params(wname))
    u0 = ctx.initial_state(amplitudes(wname).cuda())
    dt = w["dt"]
    ctx.set_timestep(dt=dt)
    rollout(ctx, u0, 4, dt)  # warm-up (factorisation)
    # untimed gradient pass: first-call set-up (adjoint workspaces, code load)
    rollout_energy(ctx, u0.clone().requires_grad_(True), 4, dt, ckpt_every=ckpt).backward()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rollout(ctx, u0, steps, dt)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    y = u0.clone().requires_grad_(True)
    e = rollout_energy(ctx, y, steps, dt, ckpt_every=ckpt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e.backward()
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    ctx.close()
    return {"workload": wname, "steps": steps, "checkpoint_every": ckpt,
            "forward_ms": round(1e3 * t_fwd, 3), "gradient_ms": round(1e3 * t_bwd, 3),
            "ratio": round(t_bwd / t_fwd, 3)}


def run_cpu(wname, steps):
    import torch

    import oracle as O
    from paper_1908_00587_amd.workloads import WORKLOADS, amplitudes, params

    w = WORKLOADS[wname]
    p = O.Params(*params(wname))
    u = O.initial_state(p, amplitudes(wname))
    dt0 = min(w["dt"], 0.5 * O.cfl_dt(p, u)) if w["dynamic"] else w["dt"]
    t0 = time.perf_counter()
    O.run(p, u, steps, dt0=dt0, dynamic=w["dynamic"], cfl=0.5, dt_max=w["dt"])
    el = time.perf_counter() - t0
    return dict(value=steps / el, unit="steps/s", cores=torch.get_num_threads(), kind="oracle",
                sample=f"{steps} FP64 oracle steps of {wname} (dense LU, DFT matrices), "
                       f"{el:.1f} s")


RESTART_FROM = "tc-heated-n64"
RESTART_TO = (96, 96, 191)  # N_r, M_theta, M_z after the restart


def run_restart(reps=20, cpu=True):
    """Restart with a change of resolution (section 2.1): the heated
    workload's state carried to N_r = 96 and 96 x 191 modes by the remap
    kernel (device time from the library's stage timer, HIP events on its
    stream), the state file written and read back through the local disk,
    and the oracle's remap of the same state on the host."""
    import os
    import tempfile

    import torch

    import paper_1908_00587_amd as nsc
    from paper_1908_00587_amd.workloads import amplitudes, params

    args = params(RESTART_FROM)
    n1, mt1, mz1 = RESTART_TO
    src = nsc.Context(*args)
    u = src.initial_state(amplitudes(RESTART_FROM).cuda())
    ctx = nsc.Context(*args[:5], n1, mt1, mz1, args[8])
    out = ctx.empty()
    for _ in range(3):
        ctx.remap_state(u, out)
    ctx.timings()
    ctx.set_profiling(True)
    for _ in range(reps):
        ctx.remap_state(u, out)
    ctx.set_profiling(False)
    ms, cnt = ctx.timings()["remap"]
    avg_us = 1e3 * ms / cnt
    F, n0, mt0, mz0 = u.shape
    kept = min(mt0, mt1) * (2 * min((mz0 - 1) // 2, (mz1 - 1) // 2) + 1)
    alg = 16 * F * (n0 * kept + n1 * mt1 * mz1)  # source modes read once, target written once
    fd, path = tempfile.mkstemp(suffix=".nsc")
    os.close(fd)
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        src.save_state(u, path, time=0.0)
        t_save = time.perf_counter() - t0
        t0 = time.perf_counter()
        ctx.load_state(path, out)
        torch.cuda.synchronize()
        t_load = time.perf_counter() - t0
        fbytes = os.path.getsize(path)
    finally:
        os.remove(path)
    res = {
        "metric": "restart remap throughput",
        "value": round(alg / (avg_us * 1e-6) / 1e9, 1), "unit": "GB/s",
        "workload": f"{RESTART_FROM} -> N_r {n1}, {mt1} x {mz1} modes",
        "avg_launch_us": round(avg_us, 2), "launches": cnt, "bytes_per_launch": alg,
        "roofline": {"bound": "hbm", "achieved": round(alg / (avg_us * 1e-6) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(alg / (avg_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None},
        "file": {"bytes": fbytes, "save_s": round(t_save, 4), "load_with_remap_s": round(t_load, 4)},
        "cpu_baseline": None,
    }
    if cpu:
        import oracle as O
        p0 = O.Params(*args)
        p1 = O.Params(*args[:5], n1, mt1, mz1, args[8])
        uc = u.cpu()
        t0 = time.perf_counter()
        O.remap_state(p1, uc, n0)
        el = time.perf_counter() - t0
        res["cpu_baseline"] = dict(value=round(1.0 / el, 4), unit="remaps/s",
                                   cores=torch.get_num_threads(), kind="oracle",
                                   sample=f"one FP64 oracle remap of the same state, {el:.2f} s")
    return res


def _pmc_means(paths):
    """{kernel: {counter: mean over dispatches}} from rocprofv3 --pmc CSVs."""
    import csv
    import re
    from collections import defaultdict
    acc = defaultdict(lambda: defaultdict(list))
    for path in paths:
        with open(path, newline="") as fh:
            for row in csv.DictReader(fh):
                name = row["Kernel_Name"]
                short = name.replace("(anonymous namespace)::", "").split("(")[0]
                if short.startswith("void "):
                    short = short[5:]
                if not short.startswith("nsc::"):
                    # library kernels (copies, fills) are told apart by their
                    # functor and size
                    fun = re.findall(r"at::native::(?:\(anonymous namespace\)::)?(\w+)", name)
                    tag = fun[1] if len(fun) > 1 else short
                    short = tag[:30] + " grid=" + row["Grid_Size"]
                acc[short][row["Counter_Name"]].append(float(row["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in acc.items()}


def traffic_report(wname, fetch_csv, write_csv):
    """Text of profiles/hbm-traffic_<workload>.txt: per-launch HBM bytes of
    every library kernel, FETCH_SIZE and WRITE_SIZE (KiB per dispatch) each
    scaled by what the counter reads for the calibration kernel (256 MiB read
    and written)."""
    f = _pmc_means([fetch_csv])
    w = _pmc_means([write_csv])
    cal = max((k for k in f if not k.startswith("nsc::")), key=lambda k: f[k]["FETCH_SIZE"])
    kib = 256 * 1024
    ff = kib / f[cal]["FETCH_SIZE"]
    fw = kib / w[cal]["WRITE_SIZE"]
    out = [f"# HBM traffic per launch, workload {wname}",
           f"# calibration kernel {cal}: FETCH_SIZE {f[cal]['FETCH_SIZE']:.1f} KiB, "
           f"WRITE_SIZE {w[cal]['WRITE_SIZE']:.1f} KiB for {kib} KiB each "
           f"-> factors {ff:.4f} (fetch), {fw:.4f} (write)",
           f"source_sha256 {source_digest()}"]
    for k in sorted(f):
        if k.startswith("nsc::") and k in w:
            b = 1024 * (ff * f[k]["FETCH_SIZE"] + fw * w[k]["WRITE_SIZE"])
            out.append(f"fetch_write_kib {f[k]['FETCH_SIZE']:.1f} {w[k]['WRITE_SIZE']:.1f} {k}")
            out.append(f"bytes_per_launch {b:.0f} {k}")
    return "\n".join(out)


def trace_summary(stats_csv, trace_csv):
    """Text summary of a rocprofv3 --kernel-trace --stats run: the per-kernel
    statistics table, then the library kernels per launch configuration
    (grid and workgroup), which separates the workloads and stages that
    share a kernel."""
    import csv
    from collections import defaultdict
    out = ["kernel statistics (rocprofv3 --stats)",
           f"{'kernel':70s} {'calls':>7s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} "
           f"{'total_ms':>9s} {'pct':>6s}"]
    for r in csv.DictReader(open(stats_csv, newline="")):
        name = r["Name"].replace("(anonymous namespace)::", "").split("(")[0]
        name = name[5:] if name.startswith("void ") else name
        out.append(f"{name[:70]:70s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:9.2f} "
                   f"{float(r['MinNs']) / 1e3:9.2f} {float(r['MaxNs']) / 1e3:9.2f} "
                   f"{float(r['TotalDurationNs']) / 1e6:9.3f} {float(r['Percentage']):6.2f}")
    acc = defaultdict(list)
    for r in csv.DictReader(open(trace_csv, newline="")):
        name = r["Kernel_Name"].replace("(anonymous namespace)::", "").split("(")[0]
        name = name[5:] if name.startswith("void ") else name
        if not name.startswith("nsc::"):
            continue
        grid = "x".join(r[f"Grid_Size_{a}"] for a in "XYZ")
        wg = "x".join(r[f"Workgroup_Size_{a}"] for a in "XYZ")
        acc[(name, grid, wg)].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    out += ["", "library kernels per launch configuration (kernel trace)",
            f"{'kernel':40s} {'grid (threads)':>22s} {'workgroup':>12s} {'calls':>7s} {'avg_us':>9s}"]
    for (name, grid, wg), v in sorted(acc.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"{name[:40]:40s} {grid:>22s} {wg:>12s} {len(v):7d} {sum(v) / len(v) / 1e3:9.2f}")
    return "\n".join(out)


def pmc_summary(paths):
    """Per-kernel average of each hardware counter over the dispatches of
    rocprofv3 --pmc counter-collection CSV files (one line per kernel)."""
    acc = _pmc_means(paths)
    counters = sorted({c for k in acc.values() for c in k})
    width = [max(14, len(c) + 2) for c in counters]
    print("kernel".ljust(48) + "".join(c.rjust(wd) for c, wd in zip(counters, width)))
    for k in sorted(acc):
        cells = [f"{acc[k][c]:.6g}" if c in acc[k] else "-" for c in counters]
        print(k[:48].ljust(48) + "".join(x.rjust(wd) for x, wd in zip(cells, width)))


def main():
    if len(sys.argv) > 2 and sys.argv[1] == "--pmc-summary":
        pmc_summary(sys.argv[2:])
        return
    if len(sys.argv) == 4 and sys.argv[1] == "--trace-summary":
        print(trace_summary(sys.argv[2], sys.argv[3]))
        return
    if len(sys.argv) == 5 and sys.argv[1] == "--traffic-report":
        print(traffic_report(*sys.argv[2:]))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="tc-heated-n64")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=40)
    ap.add_argument("--restart", action="store_true",
                    help="measure the restart remap instead of the time step")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the multi-GPU sharding is a "
              "design, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.restart:
        print(json.dumps(run_restart(cpu=not args.no_cpu)), flush=True)
        return
    from paper_1908_00587_amd.workloads import WORKLOADS
    w = WORKLOADS[args.workload]
    g = run_gpu(args, args.workload)
    adj = run_adjoint(args.adjoint_steps) if args.adjoint_steps > 0 else None
    cpu = None if args.no_cpu else run_cpu(args.workload, args.cpu_steps)
    K = g["K"]
    mx_sps = K / g["tmx"]
    fp_sps = K / g["t64"]
    out = {
        "metric": METRIC,
        "value": round(mx_sps, 2),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": g["W"],
        "ms_per_step": round(1e3 * g["tmx"] / K, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "N_r": w["N_r"], "M_theta": w["M_theta"],
                   "M_z": w["M_z"], "N_theta": 3 * w["M_theta"],
                   "N_z": 3 * ((w["M_z"] - 1) // 2 + 1), "Re_i": w["Re_i"], "Ra": w["Ra"],
                   "dynamic_dt": w["dynamic"], "n_corr": 1, "precision": "mixed",
                   "parallelism": "single-gpu"},
        "fp64": {"value": round(fp_sps, 2), "unit": "steps/s",
                 "ms_per_step": round(1e3 * g["t64"] / K, 4)},
        "mixed_speedup_vs_fp64": round(mx_sps / fp_sps, 3),
        "mixed_vs_fp64_rel_err": {k: float(f"{v:.3e}") for k, v in g["err"].items()},
        "roofline": {"bound": "hbm", "kernel": g["dominant"],
                     "achieved": round(g["achieved"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(g["achieved"] / HBM_PEAK_GBS, 4),
                     "traffic": committed_traffic(args.workload, g["dominant"]),
                     "bytes_per_launch": g["bytes"], "avg_launch_us": round(g["avg_us"], 3)},
        "adjoint_forward_cost_ratio": adj,
        "kernels": g["per_kernel"],
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
