"""The paper's illustrative heated example (section 3) on this library: a hot
rotating inner cylinder (Re_i = 50) inside a cooled stationary outer one,
three runs at Ra = 2130, 2840 and 3550, the first started from the basic
state with a small single-harmonic disturbance and each later one from the
final state of the previous run, read back from a state file into a context
with the next Rayleigh number (the restart of section 2.1).  Recorded: the
Nusselt number at the inner cylinder and u_theta at a mid-gap probe.

The paper gives neither the radius ratio, the Prandtl number nor the axial
period of these runs; the defaults below are assumptions and are returned
with the result, so the outcome is a qualitative check of the behaviour the
paper describes (Nu_i = 1 while the flow is conductive), not a reproduction
of its figure.

    python -m paper_1908_00587_amd.scenario [--t-each 4.0] [--precision mixed]
"""
import argparse
import json
import math
import os
import tempfile
import time

import torch

from .api import Context

DEFAULTS = dict(eta=0.5, Re_i=50.0, Pr=0.7, L_z=2 * math.pi, N_r=33, M_theta=16, M_z=31,
                ras=(2130.0, 2840.0, 3550.0), t_each=4.0, dt=1e-3, every=20, amp=1e-3,
                mode=(1, 1), precision="mixed")


def rayleigh_ramp(**kw):
    """Run the three segments; returns the parameters, per-segment series of
    (t, Nu_i, Nu_o, u_theta at the probe) and the timing.  N_r odd puts the
    probe row exactly at mid-gap."""
    c = dict(DEFAULTS)
    c.update(kw)
    N_r, M_t, M_z = c["N_r"], c["M_theta"], c["M_z"]
    K = (M_z - 1) // 2
    mid = N_r // 2
    fd, path = tempfile.mkstemp(suffix=".nsc")
    os.close(fd)
    segments = []
    steps = 0
    t = 0.0
    u = None
    t_wall = time.perf_counter()
    try:
        for ra in c["ras"]:
            ctx = Context(c["eta"], c["Re_i"], 0.0, ra, c["Pr"], N_r, M_t, M_z, c["L_z"])
            ctx.set_precision(c["precision"])
            ctx.set_timestep(dt=c["dt"], dynamic=True, cfl=0.5, dt_max=c["dt"])
            if u is None:
                amps = torch.zeros(ctx.F, M_t, M_z, dtype=torch.complex128)
                m, k = c["mode"]
                amps[:, m, K + k] = c["amp"]
                u = ctx.initial_state(amps.cuda())
            else:
                u, t = ctx.load_state(path)
            rec = []
            dt = c["dt"]
            t_end = t + c["t_each"]

            def record():
                d = ctx.diagnostics(u)
                pr = ctx.probe(u, [mid], [0.0], [0.0])
                nu = d.cpu().tolist()
                rec.append((t, nu[0], nu[1], float(pr[0, 1].cpu())))

            record()
            while t < t_end - 1e-12:
                for _ in range(c["every"]):
                    dt_next = ctx.step(u, dt)
                    t += dt
                    dt = dt_next
                    steps += 1
                record()
            ctx.save_state(u, path, time=t)
            segments.append(dict(Ra=ra, series=rec))
            del ctx
    finally:
        os.remove(path)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    params = {k: v for k, v in c.items() if k != "ras"}
    params["ras"] = list(c["ras"])
    return dict(params=params, segments=segments, steps=steps, wall_s=wall,
                steps_per_s=steps / wall)


def summary(res):
    """Per segment: Nu_i at the start, its extremes and its value at the end,
    the time Nu_i first departs from 1 by 1 %, and the probe signal's range
    over the last quarter of the segment."""
    out = []
    for seg in res["segments"]:
        s = seg["series"]
        nu = [x[1] for x in s]
        t0 = s[0][0]
        left = next((x[0] - t0 for x in s if abs(x[1] - 1.0) > 0.01), None)
        tail = [x[3] for x in s if x[0] >= s[-1][0] - 0.25 * (s[-1][0] - t0)]
        out.append(dict(Ra=seg["Ra"], t_start=round(t0, 4), nu_start=round(nu[0], 6),
                        nu_min=round(min(nu), 6), nu_max=round(max(nu), 6),
                        nu_end=round(nu[-1], 6),
                        t_departs_1pct=None if left is None else round(left, 3),
                        probe_tail_range=[round(min(tail), 6), round(max(tail), 6)]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--t-each", type=float, default=DEFAULTS["t_each"])
    ap.add_argument("--precision", default=DEFAULTS["precision"])
    a = ap.parse_args()
    res = rayleigh_ramp(t_each=a.t_each, precision=a.precision)
    print(json.dumps(dict(params=res["params"], steps=res["steps"],
                          steps_per_s=round(res["steps_per_s"], 1),
                          segments=summary(res))), flush=True)


if __name__ == "__main__":
    main()
