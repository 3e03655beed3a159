"""Benchmark of the Taylor--Couette time step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Main line (value): the heated workload tc-heated-n64 -- eta = 0.71,
Re_i = 100, Re_o = 0, Ra = 1e4, Pr = 0.7, N_r = 64, 64 x 127 Fourier modes
(192 x 192 padded grid), seeded synthetic initial state, dynamic time step
(CFL 0.5) -- in mixed precision (FP32 transforms and products, FP64
solves).  One step = nonlinear term + predictor solve + nonlinear term +
corrector solve.  The JSON line also carries the FP64 steps/s on the same
grid, the mixed-vs-FP64 error per field (relative to the field and to its
deviation from the basic state), the roofline of the dominant kernel (HIP
events on the library stream), every other workload's steps/s and kernel
rooflines (per_config: mixed and FP64, FP64 left out where its theta line
set does not fit the LDS), the adjoint/forward cost ratio on the adjoint
workload's schedule (200 steps, checkpoint every 20) and the FP64 CPU oracle
timed on a bounded sample of the main workload.
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


# device kernels behind each timed stage in mixed precision, by name prefix
# (template arguments depend on the grid and geometry: transform lengths,
# field counts, line-set shapes, the LDS or global-memory sweep)
STAGE_KERNELS = {"theta": ("nsc::k_theta<float,", "nsc::k_theta_fx<float,"),
                 "zinv": ("nsc::k_zinv<float,",), "zfwd": ("nsc::k_zfwd<float,",),
                 "rhs": ("nsc::k_rhs<",), "div": ("nsc::k_div2<",),
                 "sweep_pt": ("nsc::k_sweep<true, 0,", "nsc::k_sweep<false, 0,"),
                 "sweep_vel": ("nsc::k_sweep<true, 1,", "nsc::k_sweep<false, 1,"),
                 "vel_rhs": ("nsc::k_vel_rhs<",), "finalize": ("nsc::k_finalize<false>",),
                 "influence": ("nsc::k_influence<",)}


def source_digest():
    """SHA-256 over the library's HIP/C++ sources (sorted by name) with the
    comments and the layout taken out: the traffic counters of a committed
    profile apply only to the same code, and a change of wording in a
    comment does not make them stale."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_1908_00587_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(csrc, name)) as fh:
                text = fh.read()
            # one left-to-right pass, so that a "/*" inside a line comment
            # (or a "//" inside a block comment) is taken as comment text
            text = re.sub(r"//[^\n]*|/\*.*?\*/", " ", text, flags=re.S)
            h.update(name.encode() + b"\0" + " ".join(text.split()).encode())
    return h.hexdigest()


def committed_traffic(wname, stage):
    """(device kernel, HBM bytes per launch) of a stage from the committed
    counter summary profiles/hbm-traffic_<workload>.txt (FETCH_SIZE +
    WRITE_SIZE, each scaled by the calibration kernel's reading); bytes None
    when the file is missing, the library code changed since the counters
    were taken, or no single kernel of the file matches the stage."""
    path = os.path.join(ROOT, "profiles", f"hbm-traffic_{wname}.txt")
    prefixes = STAGE_KERNELS.get(stage, ())
    if not prefixes or not os.path.exists(path):
        return None, None
    digest, rows = None, {}
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) == 2 and parts[0] == "code_sha256":
                digest = parts[1]
            elif len(parts) >= 2 and parts[0] == "bytes_per_launch":
                rows[" ".join(parts[2:])] = float(parts[1])
    hits = [k for k in rows if k.startswith(prefixes)]
    if len(hits) != 1:
        return None, None
    return hits[0], (rows[hits[0]] if digest == source_digest() else None)


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


def measure(wname, steps, warmup, precisions=("fp64", "mixed"), profile_steps=50):
    """Steps/s of one workload per precision (HIP-synchronised wall time of
    `steps` steps after `warmup` untimed ones), the mixed-vs-FP64 error per
    field, and each kernel's device time from the library's stage timer
    (HIP events on its stream) over a separate run of min(steps,
    profile_steps) mixed steps."""
    import torch

    import paper_1908_00587_amd as nsc
    from paper_1908_00587_amd._lib import NSC_ERR_STATE, NscError
    from paper_1908_00587_amd.workloads import (WORKLOADS, amplitudes, is_pipe, params,
                                                pipe_params)

    w = WORKLOADS[wname]
    torch.cuda.set_device(0)
    ctx = nsc.Context.pipe(*pipe_params(wname)) if is_pipe(wname) else nsc.Context(*params(wname))
    amps = amplitudes(wname).cuda()
    u0 = ctx.initial_state(amps)
    base = ctx.initial_state(0 * amps)  # the basic state: Couette flow (and conduction)
    dt_max = w["dt"]
    if w["dynamic"]:
        ctx.set_precision("mixed")
        _, c = ctx.nonlinear(u0, cfl=True)
        dt0 = min(dt_max, 0.5 * float(c.cpu()[0]))
    else:
        dt0 = w["dt"]

    def run(prec, nsteps, nwarm, profile=False, dynamic=w["dynamic"]):
        ctx.set_precision(prec)
        ctx.set_timestep(dt=dt0, dynamic=dynamic, cfl=0.5, dt_max=dt_max)
        u = u0.clone()
        dt = dt0
        for _ in range(nwarm):
            dt = ctx.step(u, dt)
        torch.cuda.synchronize()
        if profile:
            ctx.timings()
            ctx.set_profiling(True)
        t0 = time.perf_counter()
        for _ in range(nsteps):
            dt = ctx.step(u, dt)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        tim = None
        if profile:
            ctx.set_profiling(False)
            tim = ctx.timings()
        return el, u, tim

    res = {"workload": wname, "steps": steps, "warmup": warmup}
    out = {}
    skipped = {}
    for prec in precisions:
        try:
            run(prec, 2, 0)  # untimed: first factorisation, code load
        except NscError as e:
            if e.code != NSC_ERR_STATE:
                raise
            skipped[prec] = ("the FP64 theta line set (all fields of one padded line "
                             "with the twiddles) exceeds one workgroup's LDS on this grid")
            continue
        el, _, _ = run(prec, steps, warmup)
        out[prec] = el
        res[prec] = {"steps_per_s": round(steps / el, 3), "ms_per_step": round(1e3 * el / steps, 4)}
    for prec, why in skipped.items():
        res[prec] = {"skipped": why}
    if "fp64" in out and "mixed" in out:
        # error of the mixed path: both precisions over the same fixed steps
        # (the dynamic control could pick different step sizes), from u0
        ncmp = min(steps, 20)
        res["error_steps"] = f"{ncmp} steps at the fixed dt {dt0:.4g} from the initial state"
        umx = run("mixed", ncmp, 0, dynamic=False)[1]
        u64 = run("fp64", ncmp, 0, dynamic=False)[1]
        names = ["u_r", "u_theta", "u_z", "T"][:ctx.F]
        nrm = lambda x: float(torch.linalg.vector_norm(x))  # noqa: E731
        res["mixed_vs_fp64_rel_err"] = {
            nm: float(f"{nrm(umx[f] - u64[f]) / max(nrm(u64[f]), 1e-300):.3e}")
            for f, nm in enumerate(names)}
        # relative to the field's deviation from the basic state (u_r has none)
        res["mixed_vs_fp64_pert_rel_err"] = {
            nm: float(f"{nrm(umx[f] - u64[f]) / max(nrm(u64[f] - base[f]), 1e-300):.3e}")
            for f, nm in enumerate(names)}
        res["mixed_speedup_vs_fp64"] = round(out["fp64"] / out["mixed"], 3)
        del umx, u64
    del out
    if "mixed" in precisions:
        _, _, tim = run("mixed", min(steps, profile_steps), warmup, profile=True)
        kern = {}
        for k, (ms, cnt) in tim.items():
            if cnt == 0 or k in ("remap",):
                continue
            byt = kernel_bytes(k, w, "mixed")
            avg_s = ms / cnt / 1e3
            e = {"avg_us": round(1e6 * avg_s, 3), "launches": cnt}
            if byt:
                gbs = byt / avg_s / 1e9
                e.update(bytes_per_launch=byt, GBps=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4))
            kern[k] = e
        best = max((k for k in kern if k not in ("factor",)),
                   key=lambda k: kern[k]["avg_us"] * kern[k]["launches"])
        kb = kern[best]
        dev, traffic = committed_traffic(wname, best)
        res["roofline"] = {"bound": "hbm", "kernel": best,
                           "device_kernel": dev or " or ".join(STAGE_KERNELS.get(best, ())),
                           "achieved": kb["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": kb["frac"], "traffic": traffic,
                           "bytes_per_launch": kb["bytes_per_launch"],
                           "avg_launch_us": kb["avg_us"]}
        res["kernels"] = kern
    ctx.close()
    del u0, base, amps, ctx
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res


def run_adjoint(steps=200, wname="tc-adjoint-n64", ckpt=20):
    """Adjoint/forward cost ratio on the adjoint workload's schedule (eta =
    0.71, Re_i = 200, N_r = 64, 32 x 63 modes, dt = 5e-4, 200 steps,
    checkpoint every 20): wall time of the gradient pass (checkpoint
    recompute + vector--Jacobian products) over the wall time of the plain
    forward rollout of the same steps, both after an untimed warm-up of
    each."""
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


def run_adjoint_largest():
    """The largest workload's adjoint schedule (N_r = 256, 512 x 1023 modes,
    mixed precision): 100 steps at a fixed CFL-sized dt = 2e-6, then the
    gradient of the final perturbation energy over the last 50 with a
    checkpoint every 10, checkpoints in pinned host memory and stage states
    recomputed per step (the backward pass's memory options, which this
    grid needs on one GPU).  Ratio = (energy + gradient pass) / forward
    rollout of the same 50 steps."""
    import torch

    import paper_1908_00587_amd as nsc
    from paper_1908_00587_amd.adjoint import rollout, rollout_energy
    from paper_1908_00587_amd.workloads import amplitudes, params

    wname = "tc-conv-n256"
    ctx = nsc.Context(*params(wname))
    ctx.set_precision("mixed")
    u = ctx.initial_state(amplitudes(wname).cuda())
    dt = 2e-6
    ctx.set_timestep(dt=dt)
    for _ in range(50):
        ctx.step(u, dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u50 = u.clone()
    u = rollout(ctx, u50, 50, dt)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    del u
    y = u50.clone().requires_grad_(True)
    t0 = time.perf_counter()
    e = rollout_energy(ctx, y, 50, dt, ckpt_every=10, offload=True, keep_stages=False)
    e.backward()
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    free, total = torch.cuda.mem_get_info()
    ctx.close()
    return {"workload": wname, "steps": 50, "checkpoint_every": 10, "precision": "mixed",
            "dt": dt, "options": "offload=True, keep_stages=False",
            "forward_ms": round(1e3 * t_fwd, 1), "gradient_ms": round(1e3 * t_all, 1),
            "ratio": round(t_all / t_fwd, 3),
            "device_GiB_in_use_at_end": round((total - free) / 2**30, 1)}


def host_cpu():
    """Model name of the host CPU and the CPUs this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


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
    model, ncpu = host_cpu()
    return dict(value=steps / el, unit="steps/s", cores=torch.get_num_threads(), kind="oracle",
                sample=f"{steps} FP64 oracle steps of {wname} (dense LU, DFT matrices), "
                       f"{el:.1f} s",
                cpu_model=model, affinity_cpus=ncpu)


def run_cpu_fast(wname, steps):
    """The same step on the host, evaluated the way a CPU code would
    (oracle.fast: FFTs over every host thread, radial systems inverted once
    per step size and batched over the modes), with the workload's time-step
    control; the inversions for the first step size are done before the
    clock starts, later ones (on a change of step size) are timed."""
    import torch

    import oracle as O
    from oracle.fast import Stepper
    from paper_1908_00587_amd.workloads import WORKLOADS, amplitudes, params

    w = WORKLOADS[wname]
    p = O.Params(*params(wname))
    u = O.initial_state(p, amplitudes(wname))
    s = Stepper(p)
    dt = w["dt"]
    if w["dynamic"]:
        dt = min(w["dt"], 0.5 * s.nonlinear(u)[1])
    s.set_dt(dt)
    changes = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        u, dtc = s.step(u, dt)
        if w["dynamic"]:
            nd = O.next_dt(dt, dtc, 0.5, w["dt"])
            changes += nd != dt
            dt = nd
    el = time.perf_counter() - t0
    model, ncpu = host_cpu()
    return dict(value=steps / el, unit="steps/s", cores=s.workers, kind="oracle-fast",
                torch_threads=torch.get_num_threads(),
                sample=f"{steps} FP64 steps of {wname} (FFTs, per-step-size inverses, "
                       f"{changes} step-size changes), {el:.1f} s",
                cpu_model=model, affinity_cpus=ncpu)


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
    cal = [k for k in f if "neg_kernel" in k and k in w]
    if len(cal) != 1:
        raise SystemExit(f"traffic report: expected one calibration kernel, found {cal}")
    cal = cal[0]
    kib = 256 * 1024
    ff = kib / f[cal]["FETCH_SIZE"]
    fw = kib / w[cal]["WRITE_SIZE"]
    out = [f"# HBM traffic per launch, workload {wname}",
           f"# calibration kernel {cal}: FETCH_SIZE {f[cal]['FETCH_SIZE']:.1f} KiB, "
           f"WRITE_SIZE {w[cal]['WRITE_SIZE']:.1f} KiB for {kib} KiB each "
           f"-> factors {ff:.4f} (fetch), {fw:.4f} (write)",
           f"code_sha256 {source_digest()}"]
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


# the other workloads of the per_config block: timed steps, warm-up steps
PER_CONFIG = {"tc-iso-n32": (100, 5), "tc-heated-n64": (200, 5), "tc-adjoint-n64": (200, 5),
              "tc-turb-n128": (20, 3), "tc-conv-n256": (5, 2), "pipe-n64": (100, 5)}


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
    ap.add_argument("--cpu-steps", type=int, default=6)
    ap.add_argument("--cpu-fast-steps", type=int, default=60)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-per-config", action="store_true",
                    help="time the main workload only")
    ap.add_argument("--adjoint-steps", type=int, default=200)
    ap.add_argument("--adjoint-ckpt", type=int, default=20)
    ap.add_argument("--adjoint-only", action="store_true",
                    help="print only the adjoint/forward ratio on the adjoint workload's schedule")
    ap.add_argument("--adjoint-largest", action="store_true",
                    help="print the adjoint/forward ratio on the largest workload's schedule "
                         "(about two minutes) instead of the time step")
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
    if args.adjoint_largest:
        print(json.dumps(run_adjoint_largest()), flush=True)
        return
    if args.adjoint_only:
        print(json.dumps(run_adjoint(args.adjoint_steps, ckpt=args.adjoint_ckpt)), flush=True)
        return
    from paper_1908_00587_amd.workloads import WORKLOADS
    w = WORKLOADS[args.workload]
    K, W = args.steps, args.warmup
    g = measure(args.workload, K, W)
    calibration_copy()  # the known-size kernel that scales counter readings in profiled runs
    per = {}
    if not args.no_per_config:
        for wname, (k, wu) in PER_CONFIG.items():
            if wname == args.workload:
                continue
            print(f"bench: per-config {wname}", file=sys.stderr, flush=True)
            per[wname] = measure(wname, k, wu)
    adj = (run_adjoint(args.adjoint_steps, ckpt=args.adjoint_ckpt)
           if args.adjoint_steps > 0 else None)
    cpu = None if args.no_cpu else run_cpu(args.workload, args.cpu_steps)
    cpu_fast = None if args.no_cpu else run_cpu_fast(args.workload, args.cpu_fast_steps)
    mx = g["mixed"]
    fp = g.get("fp64", {})
    out = {
        "metric": METRIC,
        "value": mx["steps_per_s"],
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": mx["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "geometry": w.get("geometry", "cylinders"),
                   "N_r": w["N_r"], "M_theta": w["M_theta"],
                   "M_z": w["M_z"], "N_theta": 3 * w["M_theta"],
                   "N_z": 3 * ((w["M_z"] - 1) // 2 + 1), "Re": w.get("Re", w.get("Re_i")),
                   "Ra": w["Ra"], "dynamic_dt": w["dynamic"], "n_corr": 1,
                   "precision": "mixed", "parallelism": "single-gpu"},
        "fp64": {"value": fp.get("steps_per_s"), "unit": "steps/s",
                 "ms_per_step": fp.get("ms_per_step")},
        "mixed_speedup_vs_fp64": g.get("mixed_speedup_vs_fp64"),
        "mixed_vs_fp64_rel_err": g.get("mixed_vs_fp64_rel_err"),
        "mixed_vs_fp64_pert_rel_err": g.get("mixed_vs_fp64_pert_rel_err"),
        "error_steps": g.get("error_steps"),
        "roofline": g["roofline"],
        "kernels": g["kernels"],
        "per_config": per,
        "adjoint_forward_cost_ratio": adj,
        "cpu_baseline": cpu,
        "cpu_fast": cpu_fast,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
