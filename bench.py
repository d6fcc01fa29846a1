#!/usr/bin/env python3
"""Throughput of the FC(Gram)-based spectral ISPH projection step on one MI355X.

Headline workload: 2D 1024 x 1024 lattice on [0,1]^2 with walls on all four
sides (Dirichlet velocity, homogeneous Neumann pressure), FC(Gram) d = 5,
C = 25 (extended 1049 x 1049), Wendland C2 kernel h = 1.3 dx, nu = 1e-3,
rho = 1, first-order projection steps from a seeded manufactured
decaying-vortex flow with its exact forcing and wall data, FP64.  All inputs
are resident on the GPU before the timed region.  The manufactured trajectory
is restarted from its initial condition every 25 steps (an on-device copy
inside the timed region), so every timed step runs on a bounded state.

Variants (written to a JSON file, --full-out): the other operator
evaluations, the FP32-mixed form, the 3D 256^3 channel (walls on y only, 20
steps from a manufactured divergence-free field, FP64 and FP32-mixed, with the
FP32-vs-FP64 error after steps 1 and 20), the batched and served workloads and
the per-kernel tables.

stdout: one compact JSON line (metric, value in Mpts/s = physical points x
steps / s, roofline of the dominant kernel from live HIP-event timings on the
library's stream - one event pair per timed step, around that kernel only;
algorithmic bytes with the method's extended period n + C - and the CPU oracle
baseline on a bounded sample).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FC-spectral ISPH step Mpts/s + %HBM roofline; batched solves/s, p99 latency"
HBM_PEAK_GBS = 8000.0
CYCLE = 25
# RK3 restart cycle in whole steps: three projections per step, so the corner
# mode of the four-wall lattice grows three times as fast per step as in FOP
CYCLE_RK3 = 8
C_FC = 25


# ------------------------------------------------------------------ bytes
def algorithmic_bytes_2d(n: int, fp32: bool = False, L: int = 0, rk3: bool = False, fused_ppe: bool = True) -> dict:
    """Compulsory HBM bytes of one launch of each kernel kind of the 2D n x n
    step (every input read once, every output written once).  State arrays are
    FP64; spectra and derivative outputs are FP64 or FP32; L is the operator
    transform length of the walled axes (n + C, or the window length).  rk3:
    the u* epilogue also writes F (2 fields) and, in sub-steps 1 and 2, reads
    the previous F (2 fields): 10/3 fields more per launch on average.
    fused_ppe (the FFT routes): the PPE's forward row pass reads the
    divergence's x spectrum instead of the stored right-hand side, and its
    inverse row pass also writes phi's x spectrum (the separate C2R store and
    x forward pass are gone); the PPE passes are FP64 in both forms.
    Callers pass L = n + C, the extended period of the method: a longer
    transform that an evaluation route chooses (the smooth window length) is
    the route's own cost, not algorithmic work."""
    P = n * n
    H = (L or n + C_FC) // 2 + 1
    ce = 8 if fp32 else 16
    te = 4 if fp32 else 8
    S = n * H * ce                 # one x half-spectrum array (the form's precision)
    S64 = n * H * 16               # one FP64 x half-spectrum array
    R = P * 8                      # one real FP64 field
    Rt = P * te                    # one derivative / rhs field
    out = {
        "rows_fwd_pair": 2 * R + 2 * S,
        "cols_op_step_a": 2 * S + 6 * S,
        # the epilogue also writes the FP64 x spectra of (u*, v*) (the fused
        # first pass of the divergence; the separate rows forward goes away)
        "rows_inv_step_a": 6 * S + 4 * R + 2 * R + 2 * S64,
        # the divergence, the PPE and stage D run FP64 transforms in both forms
        "cols_div": 2 * S64 + S64,
        "rows_inv_store": S + Rt,
        "ppe_rows_fwd": (n * H * 16 if fused_ppe else Rt) + P * 8,
        "ppe_cols_solve": P * 16,
        "ppe_rows_inv": P * 8 + R + (n * H * 16 if fused_ppe else 0),
        "rows_fwd": R + S,
        "cols_op_step_d": S64 + 2 * S64,
        "rows_inv_step_d": 2 * S64 + 2 * R + 2 * R,
        "direct_step_a": 6 * R,
        "direct_div": 2 * R + Rt,
        "direct_step_d": 5 * R,
    }
    if rk3:
        out["rows_inv_step_a"] += 10 * R // 3
        out["direct_step_a"] += 10 * R // 3
    return out


def algorithmic_bytes_3d(n: int, fp32: bool = False, L: int = 0, force: bool = False) -> dict:
    """Same for the 3D n^3 channel (walls on y): x half spectra with n or
    L rows per z plane (L = the y transform length)."""
    P = n ** 3
    H = n // 2 + 1
    ce = 8 if fp32 else 16
    te = 4 if fp32 else 8
    Sx = n * n * H * ce
    Sy = (L or n + C_FC) * n * H * ce
    R = P * 8
    Rt = P * te
    out = {
        "rows_fwd_pair": 2 * R + 2 * Sx,
        "rows_fwd": R + Sx,
        "cols_z_op_step_a": 3 * Sy + 12 * Sy,
        "rows_inv_step_a3": 12 * Sx + 3 * R + (3 * R if force else 0) + 3 * R,
        "cols_z_div": 3 * Sy + Sy,
        "rows_inv_store": Sx + Rt,
        "ppe_rows_fwd": Rt + P * ce // 2,
        "ppe_cols_y_fwd": P * ce,
        "ppe_cols_z_solve": P * ce,
        "ppe_cols_y_inv": P * ce,
        "ppe_rows_inv": P * ce // 2 + R,
        "cols_z_op_step_d": Sy + 3 * Sy,
        "rows_inv_step_d3": 3 * Sx + 3 * R + 3 * R,
    }
    for k in (1, 2, 3):
        out[f"cols_y_fwd{k}"] = k * (Sx + Sy)
        out[f"cols_y_inv{k}"] = k * (Sy + Sx)
    return out


def sources_digest() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2606_06247_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()


def counter_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC
    summary of `workload` (FETCH_SIZE and WRITE_SIZE, each scaled by the
    factor a plain copy of known size gives), or None if there is none or the
    kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("sources_sha256") != sources_digest():
        return None
    k = rec.get("workloads", {}).get(workload, {}).get(kernel)
    if not k:
        return None
    return round(1024 * (k["fetch_kib"] * rec["fetch_factor"] + k["write_kib"] * rec["write_factor"]))


# ------------------------------------------------------------------ CPU baseline
def cpu_baseline(n: int, steps: int, budget_s: float) -> dict:
    """The oracle on the host cores, in its FFT operator mode (scipy.fft with
    workers = all cores; dense per-axis PPE transforms through the BLAS): the
    same math as its direct tap-sum mode, which the tests cross-check."""
    import numpy as np
    from oracle import fcgram, step
    from oracle.lattice import walled_box
    from paper_2606_06247_amd import synth
    threads = [os.cpu_count() or 1]
    try:
        from threadpoolctl import threadpool_info
        threads += [p.get("num_threads", 1) for p in threadpool_info()]
    except Exception:
        pass
    tabs = fcgram.load()
    lat = walled_box((n, n))
    nu = 1e-3
    dx = 1.0 / (n - 1)
    dt = min(0.2 * dx, 0.1 * dx * dx / nu)
    flow = synth.DecayingVortexFlow(n, nu)
    u0 = list(flow.velocity(0.0))
    A, B = flow.force_parts()
    u = u0
    done = 0
    el = 0.0
    while done < steps and el < budget_s:
        c = done % CYCLE
        if c == 0:
            u = [x.copy() for x in u0]
        th = (c + 0.5) * dt
        f = [math.exp(-th) * a + math.exp(-2 * th) * b for a, b in zip(A, B)]
        w = [math.exp(-(c + 1) * dt) * x for x in u0]
        t0 = time.perf_counter()
        u, _ = step.project_step(lat, tabs, u, force=f, wall=w, dt=dt, nu=nu, opmode="fft")
        el += time.perf_counter() - t0
        done += 1
    assert all(np.all(np.isfinite(x)) for x in u)
    return {"value": round(n * n * done / el / 1e6, 4), "unit": "Mpts/s", "cores": int(max(threads)),
            "kind": "oracle",
            "sample": f"{done} FOP steps of the same {n}x{n} workload (oracle fft mode: scipy.fft, "
                      f"workers = all cores; same restart cycle), {el:.1f} s of step time"}


# ------------------------------------------------------------------ timing
def timed(ctx, step, steps: int, warmup: int, reset=None, profile_steps: int = 10, known=None):
    """Runs warmup calls of step(k); then an untimed profiling pass of
    min(steps, profile_steps) calls with every kernel bracketed by HIP events
    (per-kernel breakdown, dominant kernel); then, after reset(), the timed
    region: `steps` calls with events around the dominant kernel only (one pair
    per step on the library's stream, so the other kernels run without event
    overhead).  Returns wall seconds and event ms of the timed region, the
    dominant kernel's live record and the profile (record, event ms, calls)."""
    import torch
    for k in range(warmup):
        step(k)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    nprof = max(1, min(steps, profile_steps))
    ctx.read_timing()
    ctx.set_timing(True)
    q0, q1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    q0.record(stream)
    for k in range(nprof):
        step(k)
    q1.record(stream)
    ctx.set_timing(False)
    prof = ctx.read_timing()
    prof_ms = q0.elapsed_time(q1)
    # the dominant kernel among those with a byte model (known), if any
    cand = {k: v for k, v in prof.items() if known is None or k in known} or prof
    dom = max(cand.items(), key=lambda kv: kv[1][1])[0]
    if reset is not None:
        reset()
    ctx.set_timing(True, only=dom)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for k in range(steps):
        step(k)
    e1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.set_timing(False)
    live = ctx.read_timing()
    return t1 - t0, e0.elapsed_time(e1), live, (prof, prof_ms, nprof)


def summarise(live: dict, profile, ab: dict, steps: int, ms_per_step: float, workload: str):
    """Roofline of the dominant kernel from its live timed-region record; the
    per-kernel breakdown (launches per call, average, share of the pass) from
    the profiling pass."""
    prof, prof_ms, nprof = profile
    per_kernel = {}
    for name, (cnt, tot) in sorted(prof.items(), key=lambda kv: -kv[1][1]):
        avg_ms = tot / cnt
        rec = {"launches_per_step": round(cnt / nprof, 2), "avg_us": round(1e3 * avg_ms, 2),
               "share": round(tot / max(prof_ms, 1e-9), 4)}
        if name in ab:
            rec["GBs"] = round(ab[name] / (avg_ms * 1e-3) / 1e9, 1)
        per_kernel[name] = rec
    dom = max(live.items(), key=lambda kv: kv[1][1])[0]
    dom_avg_s = live[dom][1] / live[dom][0] * 1e-3
    achieved = ab[dom] / dom_avg_s / 1e9
    step_bytes = sum(ab[k] * prof[k][0] for k in prof if k in ab) / nprof
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": counter_traffic(workload, dom),
                "bytes_per_launch": ab[dom], "avg_launch_us": round(dom_avg_s * 1e6, 2),
                "launches_timed": live[dom][0],
                "step_algorithmic_GB": round(step_bytes / 1e9, 4),
                "step_frac": round(step_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    return roofline, per_kernel


def rel_l2(a, b) -> float:
    import torch
    den = torch.linalg.vector_norm(b).item()
    return torch.linalg.vector_norm(a - b).item() / (den if den > 0 else 1.0)


# ------------------------------------------------------------------ 2D workload
def run_2d(op_eval: str, n: int, steps: int, warmup: int, precision: str = "fp64", schedule=None,
           scheme: str = "fop", fc: str = "gram") -> dict:
    """Time `steps` FOP steps (scheme "fop") or whole low-storage RK3 steps of
    three sub-steps (scheme "rk3") of the 2D n x n workload."""
    import torch

    from paper_2606_06247_amd import api, synth

    nu, rho = 1e-3, 1.0
    dx = 1.0 / (n - 1)
    dt = min(0.2 * dx, 0.1 * dx * dx / nu)
    dev = "cuda:0"
    flow = synth.DecayingVortexFlow(n, nu, rho)
    u0 = [torch.from_numpy(c).to(dev) for c in flow.velocity(0.0)]
    A, B = flow.force_parts()
    A = [torch.from_numpy(c).to(dev) for c in A]
    B = [torch.from_numpy(c).to(dev) for c in B]
    forces, walls = [], []
    cycle = CYCLE if scheme == "fop" else CYCLE_RK3
    if fc == "poly":
        # with the paper's FC the four-wall trajectory leaves the finite range
        # within a 25-step cycle: every step restarts from the initial state
        cycle = 1
    # sub-step boundaries within a step (one sub-step for FOP)
    cs = [0.0, 1.0] if scheme == "fop" else [0.0, 8 / 15, 10 / 15, 1.0]
    for c in range(cycle):
        for q in range(len(cs) - 1):
            th = (c + 0.5 * (cs[q] + cs[q + 1])) * dt
            forces.append([(math.exp(-th) * a + math.exp(-2 * th) * b).contiguous() for a, b in zip(A, B)])
            walls.append([(math.exp(-(c + cs[q + 1]) * dt) * v).contiguous() for v in u0])
    u = [c.clone() for c in u0]
    p = torch.empty_like(u0[0])
    F = [torch.zeros_like(u0[0]) for _ in range(2)]

    ctx = api.Context(0)
    prob = api.Problem(n=(n, n), walled=(True, True), dx=dx, vel_bc=(("D", "D"), ("D", "D")),
                       prs_bc=(("N", "N"), ("N", "N")), rho=rho, op_eval=op_eval, precision=precision)
    if schedule and op_eval == "fft_window":
        prob.window_len = (schedule["window_len"],) * 2
        prob.lines_per_group = schedule["lines_per_group"]
        prob.radix_order = schedule.get("radix_order", 0)
    if fc == "poly":
        # the paper's own FC: 10 fit points, degree 5, extension n / 4
        prob.fc_kind, prob.fc_d, prob.fc_p, prob.fc_C = "poly", 10, 5, n // 4
    plan = api.Plan(ctx, prob)

    def step(k):
        c = k % cycle
        if c == 0:
            u[0].copy_(u0[0])
            u[1].copy_(u0[1])
        if scheme == "fop":
            plan.project_step(u, dt, nu, p_out=p, force=forces[c], wall=walls[c])
        else:
            for q in range(3):
                plan.rk3_substep(q, u, F, dt, nu, p_out=p, force=forces[3 * c + q], wall=walls[3 * c + q])

    ab = algorithmic_bytes_2d(n, precision == "fp32", n + (n // 4 if fc == "poly" else C_FC), rk3=scheme == "rk3",
                              fused_ppe=op_eval != "direct")
    # the timed steps start at k = 0, which restarts the trajectory
    wall_s, gpu_ms, live, profile = timed(ctx, step, steps, warmup, known=ab)
    ms_per_step = 1e3 * wall_s / steps
    finite = bool(all(torch.isfinite(c).all().item() for c in u))
    # context: the state after the last timed step against the exact flow at
    # its time (the trajectory restarts every `cycle` steps)
    t_end = ((steps - 1) % cycle + 1) * dt
    exact = flow.velocity(t_end)
    err = [c.cpu().numpy() - e for c, e in zip(u, exact)]
    vs_exact = {"t": t_end, "steps_into_cycle": (steps - 1) % cycle + 1,
                "rms_error": float(f"{math.sqrt(sum(float((e * e).mean()) for e in err) / 2):.3e}"),
                "rel_l2": float(f"{math.sqrt(sum(float((e * e).sum()) for e in err) / sum(float((x * x).sum()) for x in exact)):.3e}")}
    wl = f"2d_{n}_{precision}_{op_eval}" + ("" if scheme == "fop" else "_rk3") + ("" if fc == "gram" else "_fcpoly")
    roofline, per_kernel = summarise(live, profile, ab, steps, ms_per_step, wl)
    if scheme == "fop":
        # the method's compulsory I/O per FOP step, fully fused: 16 FP64 words
        # per point (u, v, f_x, f_y in; u* out and read twice; b; phi; u, v out)
        comp = 16 * n * n * 8
        roofline["step_compulsory_GB"] = round(comp / 1e9, 4)
        roofline["step_compulsory_frac"] = round(comp / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return {"value": round(n * n * steps / wall_s / 1e6, 2), "ms_per_step": round(ms_per_step, 4),
            "gpu_event_ms": round(gpu_ms, 3), "state_finite": finite, "roofline": roofline,
            "kernels": per_kernel, "transform_lengths": plan.transform_lengths(), "vs_exact": vs_exact}


def run_calls(n: int = 64, reps: int = 200) -> dict:
    """The small lattice of every boundary call: n x n on the unit square,
    Dirichlet velocity and pressure on all four walls, manufactured fields
    (seeds 0, 1, 2); microseconds per call (device time between events around
    `reps` back-to-back calls, after warm-up) for each operator evaluation."""
    import torch

    from paper_2606_06247_amd import api, synth
    ctx = api.Context(0)
    dx = 1.0 / (n - 1)
    u, v, pr = (torch.from_numpy(synth.poly_trig_2d(n, k, dx=dx)).cuda() for k in range(3))
    out = {}
    for oe in ("fft_window", "fft", "direct"):
        prob = api.Problem(n=(n, n), walled=(True, True), dx=dx, vel_bc=(("D", "D"), ("D", "D")),
                           prs_bc=(("D", "D"), ("D", "D")), op_eval=oe)
        plan = api.Plan(ctx, prob)
        ext = plan.fc_extend(u)
        g = plan.spectral_grad(pr, api.PRESSURE)
        d = plan.spectral_div([u, v])
        lp = plan.spectral_lap(u)
        phi = plan.ppe_solve(d)
        us = [u.clone(), v.clone()]
        calls = {
            "fc_extend": lambda: plan.fc_extend(u, api.VELOCITY, out=ext),
            "spectral_grad": lambda: plan.spectral_grad(pr, api.PRESSURE, out=g),
            "spectral_div": lambda: plan.spectral_div([u, v], out=d),
            "spectral_lap": lambda: plan.spectral_lap(u, api.VELOCITY, out=lp),
            "ppe_solve": lambda: plan.ppe_solve(d, out=phi),
            "project_step": lambda: plan.project_step(us, 1e-4, 1e-3, p_out=phi),
        }
        rec = {}
        for name, fn in calls.items():
            for _ in range(20):
                fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            rec[name] = round(1e3 * e0.elapsed_time(e1) / reps, 2)
        out[oe] = rec
    return out


_INPUTS_2D = {}


def inputs_2d(n: int, nsteps: int):
    """Device-resident initial velocity, forcing and wall data of the first
    nsteps steps of the 2D workload (built once per size)."""
    import torch

    from paper_2606_06247_amd import synth
    key = (n, nsteps)
    if key not in _INPUTS_2D:
        nu = 1e-3
        dx = 1.0 / (n - 1)
        dt = min(0.2 * dx, 0.1 * dx * dx / nu)
        flow = synth.DecayingVortexFlow(n, nu)
        u0 = [torch.from_numpy(c).cuda() for c in flow.velocity(0.0)]
        A, B = flow.force_parts()
        A = [torch.from_numpy(c).cuda() for c in A]
        B = [torch.from_numpy(c).cuda() for c in B]
        f = [[math.exp(-(k + 0.5) * dt) * a + math.exp(-2 * (k + 0.5) * dt) * b for a, b in zip(A, B)]
             for k in range(nsteps)]
        w = [[math.exp(-(k + 1) * dt) * v for v in u0] for k in range(nsteps)]
        _INPUTS_2D[key] = (dt, nu, u0, f, w)
    return _INPUTS_2D[key]


def fp32_error_2d(n: int, op_eval: str, nsteps: int = 20) -> dict:
    """Relative L2 of the FP32-mixed form against the FP64 form after 1 and
    nsteps steps of the 2D workload (same inputs)."""
    import torch

    from paper_2606_06247_amd import api
    dt, nu, u0, forces, walls = inputs_2d(n, nsteps)
    dx = 1.0 / (n - 1)
    ctx = api.Context(0)
    res = {}
    states = {}
    for prec in ("fp64", "fp32"):
        prob = api.Problem(n=(n, n), walled=(True, True), dx=dx, vel_bc=(("D", "D"), ("D", "D")),
                           prs_bc=(("N", "N"), ("N", "N")), op_eval=op_eval, precision=prec)
        plan = api.Plan(ctx, prob)
        u = [c.clone() for c in u0]
        p = torch.empty_like(u[0])
        snaps = {}
        for k in range(nsteps):
            plan.project_step(u, dt, nu, p_out=p, force=forces[k], wall=walls[k])
            if k + 1 in (1, nsteps):
                snaps[k + 1] = [c.clone() for c in u] + [p.clone()]
        states[prec] = snaps
    for k in (1, nsteps):
        res[f"step{k}"] = {name: float(f"{rel_l2(a, b):.3e}") for name, a, b in
                           zip(("u", "v", "p"), states["fp32"][k], states["fp64"][k])}
    return res


# ------------------------------------------------------------------ 3D workload
_CHANNEL = {}


def run_3d(n: int, steps: int, warmup: int, precision: str, ref_states=None, op_eval: str = "fft") -> dict:
    """Time `steps` FOP steps of the n^3 channel (walls on y, no forcing) from
    the manufactured divergence-free field; the timed steps run from the
    initial state (the warm-up steps run on a copy)."""
    import torch

    from paper_2606_06247_amd import api, synth
    nu, rho = 1e-3, 1.0
    dx = 1.0 / (n - 1)
    dt = min(0.2 * dx, 0.1 * dx * dx / nu)
    if n not in _CHANNEL:
        _CHANNEL[n] = synth.ChannelFlow3D((n, n, n), 20, 21).u
    u0 = [torch.from_numpy(c).cuda() for c in _CHANNEL[n]]
    zero_wall = torch.zeros_like(u0[0])
    walls = [zero_wall, zero_wall, zero_wall]
    u = [c.clone() for c in u0]
    p = torch.empty_like(u0[0])
    ctx = api.Context(0)
    prob = api.Problem(n=(n, n, n), walled=(False, True, False), dx=dx,
                       vel_bc=(None, ("D", "D"), None), prs_bc=(None, ("N", "N"), None),
                       rho=rho, precision=precision, op_eval=op_eval)
    plan = api.Plan(ctx, prob)
    snaps = {}

    def step(k):
        plan.project_step(u, dt, nu, p_out=p, force=None, wall=walls)

    for k in range(warmup):
        step(k)
    for c, c0 in zip(u, u0):
        c.copy_(c0)

    def timed_step(k):
        step(k)
        if ref_states is not None and k + 1 in (1, steps):
            snaps[k + 1] = [c.clone() for c in u] + [p.clone()]

    def reset():
        for c, c0 in zip(u, u0):
            c.copy_(c0)

    ab = algorithmic_bytes_3d(n, precision == "fp32", n + C_FC)
    wall_s, gpu_ms, live, profile = timed(ctx, timed_step, steps, 0, reset=reset, known=ab)
    ms_per_step = 1e3 * wall_s / steps
    finite = bool(all(torch.isfinite(c).all().item() for c in u))
    roofline, per_kernel = summarise(live, profile, ab, steps, ms_per_step, f"3d_{n}_{precision}_{op_eval}")
    out = {"value": round(n ** 3 * steps / wall_s / 1e6, 2), "ms_per_step": round(ms_per_step, 4),
           "gpu_event_ms": round(gpu_ms, 3), "state_finite": finite, "roofline": roofline,
           "kernels": per_kernel, "steps": steps, "transform_lengths": plan.transform_lengths()}
    if ref_states is not None:
        ref_states.update(snaps)
    return out


# ------------------------------------------------------------------ batched workload
BATCH_SIZES = (64, 96, 128, 192, 256, 384, 512)
TUNE_BATCH = 8        # lattices per timed batch when tuning a size class for the batched form


def batch_instances(count: int, seed: int = 30) -> list:
    """(n, velocity walls) per instance: n ~ U{64..512}, then each of the four
    walls Dirichlet or Neumann, drawn in that order from one stream."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice(BATCH_SIZES))
        vel = tuple(tuple(str(rng.choice(["D", "N"])) for _ in range(2)) for _ in range(2))
        out.append((n, vel))
    return out


def _complement(v):
    return tuple(("N" if a == "D" else "D", "N" if b == "D" else "D") for a, b in v)


def run_batch(count: int, precision: str, reps: int, schedules: dict, ref_u=None) -> dict:
    """One FOP step of every instance per batch step: plain per-plan loop,
    grouped launch, and grouped launch replayed from a HIP graph."""
    import torch

    from paper_2606_06247_amd import api, synth
    dt, nu = 1e-4, 1e-3
    inst = batch_instances(count)
    ctx = api.Context(0)
    plans, states, walls, pts = [], [], [], 0
    for i, (n, vel) in enumerate(inst):
        sch = schedules.get(n, {})
        wl = sch.get("window_len", 0)
        prob = api.Problem(n=(n, n), walled=(True, True), dx=1.0 / (n - 1), vel_bc=vel,
                           prs_bc=_complement(vel), precision=precision, op_eval="fft_window",
                           window_len=(wl, wl) if wl else (), lines_per_group=sch.get("lines_per_group", 0),
                           radix_order=sch.get("radix_order", 0), batched=True)
        plans.append(api.Plan(ctx, prob))
        u = [synth.poly_trig_2d(n, 1000 + 2 * i), synth.poly_trig_2d(n, 1001 + 2 * i)]
        states.append([torch.from_numpy(c).cuda() for c in u])
        walls.append([c.clone() for c in states[-1]])
        pts += n * n
    init = [[c.clone() for c in st] for st in states]
    pbuf = [torch.empty_like(st[0]) for st in states]
    # equality of one batched step with one plain step (copies of the state)
    plain = [[c.clone() for c in st] for st in init]
    for i in range(count):
        plans[i].project_step(plain[i], dt, nu, p_out=pbuf[i], wall=walls[i])
    b = api.Batch(ctx, count)
    for i in range(count):
        b.add_step(plans[i], states[i], dt, nu, p_out=pbuf[i], wall=walls[i])
    b.launch()
    torch.cuda.synchronize()
    mism = [i for i in range(count) if not all(torch.equal(states[i][a], plain[i][a]) for a in range(2))]
    equal = not mism
    max_diff = max([float((states[i][a] - plain[i][a]).abs().max()) for i in mism for a in range(2)] + [0.0])
    fp32_err = None
    if ref_u is not None:
        errs = sorted(max(rel_l2(states[i][a], ref_u[i][a]) for a in range(2)) for i in range(count))
        fp32_err = {"max": float(f"{errs[-1]:.3e}"), "median": float(f"{errs[len(errs) // 2]:.3e}")}
    first_step = [[c.clone() for c in st] for st in states] if precision == "fp64" else None
    del plain

    def clock(fn):
        for st, st0 in zip(states, init):
            for c, c0 in zip(st, st0):
                c.copy_(c0)
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    def plain_loop():
        for i in range(count):
            plans[i].project_step(states[i], dt, nu, p_out=pbuf[i], wall=walls[i])

    t_plain = clock(plain_loop)
    t_batch = clock(b.launch)
    b.capture()
    t_graph = clock(b.replay)
    items, groups, launches = b.info()
    # algorithmic bytes of one batch step (sum of the per-instance step models)
    step_bytes = 0
    for (n, _), pl in zip(inst, plans):
        ab = algorithmic_bytes_2d(n, precision == "fp32", n + C_FC)
        step_bytes += sum(ab[k] for k in ("rows_fwd_pair", "cols_op_step_a", "rows_inv_step_a", "cols_div",
                                          "ppe_rows_fwd", "ppe_cols_solve", "ppe_rows_inv",
                                          "cols_op_step_d", "rows_inv_step_d"))
        step_bytes -= 2 * n * n * 8        # no forcing arrays read
    out = {"instances": count, "points": pts, "groups": groups, "grouped_launches": launches,
           "batched_equals_plain_bitwise": bool(equal),
           "instances_differing_from_plain": len(mism), "max_abs_diff_vs_plain": max_diff,
           "solves_per_s": {"plain_loop": round(count / t_plain, 1), "batched": round(count / t_batch, 1),
                            "batched_graph": round(count / t_graph, 1)},
           "ms_per_batch_step": {"plain_loop": round(1e3 * t_plain, 3), "batched": round(1e3 * t_batch, 3),
                                 "batched_graph": round(1e3 * t_graph, 3)},
           "Mpts_per_s_graph": round(pts / t_graph / 1e6, 1),
           "roofline": {"bound": "hbm", "achieved": round(step_bytes / t_graph / 1e9, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(step_bytes / t_graph / 1e9 / HBM_PEAK_GBS, 4),
                        "basis": "sum of the per-instance step byte models / graph-replay step time"}}
    if fp32_err is not None:
        out["fp32_vs_fp64_rel_l2_step1"] = fp32_err
    del b
    return out, first_step



# ------------------------------------------------------------------ serving workload
def run_serving(precision: str, lams, max_requests: int, window_s: float, plain_lams=()) -> dict:
    """Poisson request streams at each rate on one server (plans and input
    templates resident across rates): continuous batching, and the plain
    per-request path on the same resident plans."""
    from paper_2606_06247_amd import serve
    streams = {}
    for lam in lams:
        count = int(min(max_requests, max(50, lam * window_s)))
        streams[lam] = serve.make_requests(lam, count, seed=40)
    shapes = sorted({(r.dims, r.n) for rs in streams.values() for r in rs})
    srv = serve.Server(precision, hbm_budget=200e9, max_batch=16, lanes=4)
    srv.warm(shapes)
    warm = [serve.Request(i, 0.0, r.kind, r.dims, r.n, r.seed) for i, r in enumerate(streams[lams[0]][:32])]
    srv.run(warm, realtime=False)
    out = {"resident_plans_created": srv.stats["plans_created"], "shapes": len(shapes)}
    for lam in lams:
        st = srv.run(streams[lam], realtime=True)
        rec = {"served": st}
        if lam in plain_lams:
            reqs2 = serve.make_requests(lam, len(streams[lam]), seed=40)
            rec["plain_per_request"] = serve.run_plain(reqs2, srv)
        out[str(lam)] = rec
        log(f"  lambda {lam}: {st['solves_per_s']} solves/s p50 {st['p50_ms']} ms p99 {st['p99_ms']} ms"
            + (f"; plain p99 {rec['plain_per_request']['p99_ms']} ms" if lam in plain_lams else ""))
    del srv
    return out


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--n3", type=int, default=256, help="3D channel lattice n^3")
    ap.add_argument("--steps3", type=int, default=20)
    ap.add_argument("--batch", type=int, default=512, help="instances of the batched workload")
    ap.add_argument("--serve-requests", type=int, default=1200)
    ap.add_argument("--serve-window", type=float, default=3.0)
    ap.add_argument("--cpu-steps", type=int, default=30)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="library default schedules (no autotuning)")
    ap.add_argument("--op-eval", choices=["fft", "fft_window", "direct"], default="fft_window")
    ap.add_argument("--no-variants", action="store_true",
                    help="time only the headline workload")
    ap.add_argument("--full-out", default=os.path.join("gpurun_out", "bench_full.json"),
                    help="file for the variants and per-kernel tables ('' = none); stdout keeps one "
                         "compact JSON line")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    ap.add_argument("--only", choices=["fp32", "batch"], default=None,
                    help="only run one secondary workload (the FP32-mixed 2D step, or the FP64 batch of "
                         "--batch lattices) and print its record: a profiling entry point, not the bench line")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        src = torch.ones(args.copy_probe * (1 << 20) // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_MiB": args.copy_probe, "bytes": src.numel() * 8}))
        return 0
    if args.gpus != 1:
        print("bench.py: the library runs one lattice per GPU in one process; --gpus must be 1 (there is no multi-GPU path)", file=sys.stderr)
        return 2
    if args.only:
        from paper_2606_06247_amd import api as _api, tune
        tctx = _api.Context(0)
        if args.only == "fp32":
            sched = None if args.no_tune else tune.tune_2d(tctx, args.n, "fp32", lines=(1, 2, 4))
            v = run_2d(args.op_eval, args.n, args.steps, args.warmup, precision="fp32", schedule=sched)
            print(json.dumps({"workload": f"2d_{args.n}_fp32_{args.op_eval}", "value": v["value"], "unit": "Mpts/s",
                              "ms_per_step": v["ms_per_step"], "schedule": sched, "roofline": v["roofline"]}))
        else:
            sched = {} if args.no_tune else {nb: tune.tune_2d(tctx, nb, "fp64", lines=(1, 2), batch=TUNE_BATCH)
                                             for nb in BATCH_SIZES}
            rec, _ = run_batch(args.batch, "fp64", max(1, min(args.steps, 20)), sched)
            print(json.dumps({"workload": f"batch_{args.batch}_fp64", "solves_per_s": rec["solves_per_s"],
                              "ms_per_batch_step": rec["ms_per_batch_step"], "groups": rec["groups"],
                              "grouped_launches": rec["grouped_launches"],
                              "batched_equals_plain_bitwise": rec["batched_equals_plain_bitwise"]}))
        return 0
    n = args.n
    from paper_2606_06247_amd import api as _api, tune
    sched64 = sched32 = None
    if not args.no_tune:
        log(f"tuning {n} fp64 / fp32")
        sched64 = tune.tune_2d(_api.Context(0), n, "fp64", lines=(1, 2, 4))
        sched32 = tune.tune_2d(_api.Context(0), n, "fp32", lines=(1, 2, 4))
    log(f"headline 2d {n} fp64 {args.op_eval}")
    head = run_2d(args.op_eval, n, args.steps, args.warmup, schedule=sched64)
    log(f"  {head['value']} Mpts/s")
    L_used = head["transform_lengths"]
    out = {"metric": METRIC, "value": head["value"], "unit": "Mpts/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"2D {n}x{n} FC(Gram)-spectral ISPH first-order projection steps, "
                                  "walls on 4 sides (Dirichlet velocity, Neumann pressure), "
                                  f"FC(Gram) d=5 C=25 (extended period {n + 25}), Wendland C2 h=1.3dx, "
                                  "nu=1e-3, manufactured decaying-vortex flow; restarted workload: the "
                                  f"trajectory restarts from its initial state every {CYCLE} steps "
                                  "(on-device copy inside the timed region)",
                      "n": n, "precision": "fp64", "op_eval": args.op_eval,
                      "transform_length": L_used[0], "restart_every_steps": CYCLE,
                      "state_finite": head["state_finite"],
                      "schedule": sched64 if args.op_eval == "fft_window" else None},
           "roofline": head["roofline"]}
    full = dict(out, kernels=head["kernels"], gpu_event_ms=head["gpu_event_ms"], vs_exact=head["vs_exact"])
    if not args.no_variants:
        log("calls 2d 64 (us per call)")
        full["calls_64_us"] = run_calls(64)
        keep = ("value", "ms_per_step", "state_finite", "transform_lengths", "roofline", "kernels", "vs_exact")
        var = {}
        for oe in ("fft", "fft_window", "direct"):
            if oe != args.op_eval:
                log(f"variant 2d {n} fp64 {oe}")
                v = run_2d(oe, n, args.steps, args.warmup, schedule=sched64)
                var[f"2d_{n}_fp64_{oe}"] = {k: v[k] for k in keep if k in v}
        log(f"variant 2d {n} fp64 {args.op_eval} RK3")
        v = run_2d(args.op_eval, n, max(1, args.steps // 3), args.warmup, schedule=sched64, scheme="rk3")
        rec = {k: v[k] for k in keep if k in v}
        rec["workload"] = ("the same 1024^2 workload advanced by whole low-storage RK3 steps (three sub-steps, "
                           "forcing at sub-step midpoints, wall data at sub-step ends), restart every "
                           f"{CYCLE_RK3} steps; value = points x RK3 steps / s")
        var[f"2d_{n}_fp64_{args.op_eval}_rk3"] = rec
        for oe in ("fft_window", "fft"):
            log(f"variant 2d {n} fp64 {oe} paper FC")
            v = run_2d(oe, n, args.steps, args.warmup, schedule=sched64, fc="poly")
            rec = {k: v[k] for k in keep if k in v}
            rec["workload"] = (f"the same 1024^2 FOP workload with the paper's own FC (least-squares degree-5 fit "
                               f"to 10 points per wall, quintic blend, extension {n // 4} points, extended period "
                               f"{n + n // 4}); every step restarts from the initial state (on-device copy in the "
                               "timed region)")
            var[f"2d_{n}_fp64_{oe}_fcpoly"] = rec
        for oe in ("fft", "fft_window", "direct"):
            log(f"variant 2d {n} fp32 {oe}")
            v = run_2d(oe, n, args.steps, args.warmup, precision="fp32", schedule=sched32)
            rec = {k: v[k] for k in keep if k in v}
            rec["dtype"] = "f32 transforms, f64 FC/divide/state"
            rec["fp32_vs_fp64_rel_l2"] = fp32_error_2d(n, oe)
            var[f"2d_{n}_fp32_{oe}"] = rec
        n3 = args.n3
        for oe in ("fft", "fft_window"):
            ref64, ref32 = {}, {}
            for prec, ref in (("fp64", ref64), ("fp32", ref32)):
                log(f"variant 3d {n3} {prec} {oe}")
                v = run_3d(n3, args.steps3, 2, prec, ref, op_eval=oe)
                rec = {k: v[k] for k in keep if k in v}
                rec["steps"] = args.steps3
                rec["workload"] = (f"3D {n3}^3 channel, walls on y (Dirichlet velocity, Neumann pressure), "
                                   f"periodic x and z, extended {n3}x{n3 + 25}x{n3}, {args.steps3} steps "
                                   "from a manufactured divergence-free field, no forcing")
                var[f"3d_{n3}_{prec}_{oe}"] = rec
            var[f"3d_{n3}_fp32_{oe}"]["fp32_vs_fp64_rel_l2"] = {
                f"step{k}": {name: float(f"{rel_l2(a, b):.3e}") for name, a, b in
                             zip(("u", "v", "w", "p"), ref32[k], ref64[k])} for k in sorted(ref64)}
            del ref64, ref32
        # batched solves (512 independent 2D lattices), schedules from the
        # autotuner timing graph-replayed batches of each size class
        tctx = _api.Context(0)
        for prec in ("fp64", "fp32"):
            sched = {}
            for nb in BATCH_SIZES:
                if not args.no_tune:
                    log(f"tuning {nb} {prec} (batches of {TUNE_BATCH})")
                    sched[nb] = tune.tune_2d(tctx, nb, prec, lines=(1, 2), batch=TUNE_BATCH)
            log(f"batch {args.batch} {prec}")
            rec, first = run_batch(args.batch, prec, 5, sched, ref_u=ref_batch if prec == "fp32" else None)
            if prec == "fp64":
                ref_batch = first
            if sched:
                # the same batch on the library's default schedules
                dflt, _ = run_batch(args.batch, prec, 5, {})
                rec["solves_per_s_default_schedules"] = dflt["solves_per_s"]
            rec["schedules"] = {str(k): v for k, v in sched.items()}
            rec["workload"] = (f"{args.batch} independent 2D lattices, n ~ U{{64..512}} (seed 30), each wall "
                               "Dirichlet or Neumann velocity (complementary pressure), manufactured fields, "
                               "one FOP step per instance per batch step, windowed-FFT operators")
            var[f"batch_{args.batch}_{prec}"] = rec
        del ref_batch
        # served requests (Poisson streams, continuous batching)
        for prec in ("fp64", "fp32"):
            log(f"serving {prec}")
            var[f"serving_{prec}"] = {
                "workload": "Poisson arrivals; 50% projection steps / 50% PPE solves; 75% 2D n ~ logU(64, 1024), "
                            "25% 3D channel n ~ logU(64, 192), sizes in multiples of 16; HBM budget 200 GB; "
                            f"at most {args.serve_requests} requests or {args.serve_window} s of arrivals per rate; "
                            "4 lanes, batches of one class: up to 16 2D or 2 3D requests",
                "rates": run_serving(prec, (50, 100, 200, 500, 1000, 2000, 5000, 10000), args.serve_requests,
                                     args.serve_window, plain_lams=(50, 500, 2000, 5000, 10000))}
        full["variants"] = var
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = full["cpu_baseline"] = cpu_baseline(n, args.cpu_steps, args.cpu_seconds)
    if args.full_out:
        os.makedirs(os.path.dirname(os.path.abspath(args.full_out)), exist_ok=True)
        with open(args.full_out, "w") as fh:
            json.dump(full, fh, indent=1)
        log(f"variants and per-kernel tables written to {args.full_out}")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
