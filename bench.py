#!/usr/bin/env python3
"""Benchmark of the comoving PPM gas step on one MI355X.

Headline workload (box512_stress): the 512^3 stress box (density contrast up
to 10^4 with ln rho ~ N(., 2^2) clipped at +-ln 100, T/T_mean lognormal
sigma_ln 1.5, k^-2 velocities of sigma 0.5 clipped to Mach 30, g ~ N(0,
0.2^2)), a 0.10 -> 0.11 over 10 steps, one level dt.  The metric compares,
on the same GPU and inputs:
  * plain FP64 with the domain as one box (one launch per stage);
  * the chosen form: FP32-mixed + batched, the domain as an 8^3 grid of 64^3
    patches in one batched plan with the same-level ghost fill, with or
    without the learned Riemann flux (network trained, untimed, on about 2e7
    faces harvested from stress fields of other seeds).
`value` is the fastest FP32-mixed batched form whose density stays within
1e-3 relative L1 of plain FP64 after the timed steps (the FP64 run's dt
sequence drives every form); every form's rate, error and fallback rate is
in the line.  One timed step is [batched step -> patch-grid ghost fill].

`roofline` is that of the chosen form's dominant stage kernel: algorithmic
flops per launch (the oracle's operation counts per work unit,
profiles/opcounts_step.json, times the launch's units, with the measured
two-shock iterations) over the launch's mean duration from HIP events the
library records around its stage launches on the step's stream.
`hbm_step` is the whole step's algorithmic bytes (the padded state and
gravity read once, the valid state written once) over the step time.

Other legs (same JSON line):
  box256 (single 256^3 box of smooth flow, 20 steps): plain FP64 vs FP32-mixed;
  learned256 (a fresh-seed 256^3 box of the same type, 20 steps): FP32-mixed
    with and without the learned flux (all twelve solves, or stages 0-1);
  level4096 (4096 boxes, edges from {16, 24, 32, 48, 64}, per-box dt, a
    0.25 -> 0.255): batched plan, its HIP-graph replay and the learned form,
    against per-box plain FP64 launches, with density error against FP64;
  variants (PLM, linearised solver, gravity form 2, gamma 1.4), level
  ghost fill, two-level reflux/average-down, gravity input;
  cpu_baseline: the FP64 oracle on 64^3 patches of the headline fields, on
  all usable host cores (threads, at most 16) and on one.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "zone-updates/s (plain FP64 vs FP32+batched+learned flux) + % HBM roofline"
HBM_PEAK_GBS = 8000.0
ALU_PEAK_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz, FP64 and FP32
STAGES = ("prim", "flat", "trace", "riem0", "riem1", "riem2", "update")
MODE_NAMES = ("staged", "persistent", "fused")  # NYX_LAUNCH_* 0, 1, 2
RIEMANN = ("riem0", "riem1", "riem2")
OPCOUNTS = os.path.join(ROOT, "profiles", "opcounts_step.json")
OPCOUNT_KEYS = {"box256": "box256_smooth fields (64^3 box of the same distributions, seed 2)",
                "box512_stress": "box512_stress fields (64^3 box of the same distributions, seed 5)"}


def units(n):
    """Work units of each stage kernel's grid on one box n = (nx, ny, nz):
    padded cells, cells of [-1, n]^3, tracing cell-directions, the faces of
    each Riemann stage, valid cells."""
    nx, ny, nz = n
    P = (nx + 8) * (ny + 8) * (nz + 8)
    E = (nx + 2) * (ny + 2) * (nz + 2)
    ext = (nx, ny, nz)
    f0 = f1 = f2 = 0
    for d in range(3):
        e = [x + 2 for x in ext]
        e[d] = ext[d] + 1
        f0 += e[0] * e[1] * e[2]
        for t in range(3):
            if t != d:
                e1 = [x + 2 for x in ext]
                e1[d] = ext[d] + 1
                e1[t] = ext[t]
                f1 += e1[0] * e1[1] * e1[2]
        e2 = list(ext)
        e2[d] = ext[d] + 1
        f2 += e2[0] * e2[1] * e2[2]
    return {"prim": P, "flat": E, "trace": 3 * E, "riem0": f0, "riem1": f1, "riem2": f2,
            "update": nx * ny * nz}


def flop_table(key):
    """Per-unit flops of each stage counted by the oracle on `key`'s fields."""
    with open(OPCOUNTS) as fh:
        return json.load(fh)["workloads"][OPCOUNT_KEYS[key]]


def stage_flops(table, stage, shapes, iters_per_face):
    """Algorithmic flops of one launch of `stage` over boxes of `shapes`: the
    oracle's flops per unit times the units; for a Riemann stage the flops
    outside the Newton iterations per face plus the flops of one iteration
    times the measured iterations per face (the GPU's counter, the mean over
    the three Riemann stages)."""
    u = sum(units(n)[stage] for n in shapes)
    row = table[stage]
    if stage in RIEMANN:
        return u * (row["flops_per_face_outside_iterations"] +
                    row["flops_per_iteration"] * iters_per_face)
    return u * row["flops_per_unit"]


def bytes_per_launch(stage, n, rb):
    """Algorithmic HBM bytes of one stage launch on an n^3 box in this staged
    design: every distinct input value read once and every output written
    once (rb = bytes of a stage-array element: 8 in FP64, 4 in FP32-mixed)."""
    P, E, V = (n + 8) ** 3, (n + 2) ** 3, n ** 3
    return {
        "prim": 6 * 8 * P + 6 * rb * P,
        "flat": 4 * rb * P + rb * E,
        "trace": 6 * rb * P + 3 * rb * P + rb * E + 30 * rb * E,
        "riem0": 30 * rb * E + 15 * rb * E,
        "riem1": 30 * rb * E + 15 * rb * E + 30 * rb * E,
        "riem2": 30 * rb * E + 30 * rb * E + 15 * rb * E,
        "update": 15 * rb * E + (6 * 8 + 3 * rb) * V + 6 * 8 * V,
    }[stage]


def step_bytes(shapes, grav_bytes):
    """Algorithmic bytes of one whole step (one fused pass): the padded FP64
    state and the padded gravity read once, the valid FP64 state written
    once."""
    tot = 0
    for (nx, ny, nz) in shapes:
        P = (nx + 8) * (ny + 8) * (nz + 8)
        tot += (48 + 3 * grav_bytes) * P + 48 * nx * ny * nz
    return tot


def roofline_of(stage_ms, table, shapes, iters, step_ms, grav_bytes, form, workload,
                tune=None, persistent_ms=None, fused=False):
    """The dominant kernel's figures: algorithmic TFLOP/s against the vector
    ALU peak (the dominant stage kernel, the fused final-stage kernel, or the
    persistent step kernel, which runs every stage), and the whole step's
    algorithmic bytes against HBM."""
    if persistent_ms is not None:
        dom, ms = "step_persistent", persistent_ms
        fl = sum(stage_flops(table, st, shapes, iters) for st in STAGES)
    else:
        dom = max(kernel_stages(fused), key=lambda s: kernel_ms(stage_ms, s))
        ms = kernel_ms(stage_ms, dom)
        fl = kernel_flops(table, dom, shapes, iters)
    ach = fl / (ms * 1e-3) / 1e12
    t = None
    if tune is not None and persistent_ms is None and dom in STAGES:
        t = measured_traffic(dom, form, tune[STAGES.index(dom)], workload)
    roof = {"bound": "alu" if dom in RIEMANN + ("trace", "step_persistent", "front", "final")
            else "hbm",
            "kernel": dom, "ms_per_launch": round(ms, 4),
            "flops_per_launch": fl, "achieved": round(ach, 3), "peak": ALU_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(ach / ALU_PEAK_TFLOPS, 4), "traffic": t}
    if roof["bound"] == "hbm":
        b = sum(bytes_per_launch(dom, n[0], 4) for n in shapes)
        gbs = b / (ms * 1e-3) / 1e9
        roof.update({"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4)})
    sb = step_bytes(shapes, grav_bytes)
    gbs = sb / (step_ms * 1e-3) / 1e9
    hbm = {"bytes_per_step": sb, "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}
    return roof, hbm


# the fused launch mode's kernels: "front" = trace + riem0 (k_front),
# "final" = riem2 + update (k_final)
FUSED_STAGES = ("prim", "flat", "front", "riem1", "final")
FUSED_PARTS = {"front": ("trace", "riem0"), "final": ("riem2", "update")}


def kernel_stages(fused):
    return FUSED_STAGES if fused else STAGES


def kernel_ms(stage_ms, stage):
    """ms of a stage kernel; a fused kernel's time is what the library's
    events report for its first stage (the second stage's interval is
    empty), so the sum of both is the fused launch's."""
    return sum(stage_ms[s] for s in FUSED_PARTS.get(stage, (stage,)))


def kernel_flops(table, stage, shapes, iters):
    return sum(stage_flops(table, s, shapes, iters) for s in FUSED_PARTS.get(stage, (stage,)))


def stage_rates(stage_ms, table, shapes, iters, fused=False):
    """Per-kernel ms, algorithmic TFLOP/s (oracle op counts)."""
    out = {}
    for s in kernel_stages(fused):
        ms = kernel_ms(stage_ms, s)
        fl = kernel_flops(table, s, shapes, iters)
        out[s] = {"ms": round(ms, 4), "tflops": round(fl / max(ms, 1e-9) / 1e9, 3)}
    return out
KERNEL_SOURCES = ("paper_1301_4498_amd/csrc/nyx_step.hip", "paper_1301_4498_amd/csrc/nyx_internal.h",
                  "paper_1301_4498_amd/csrc/nyx_mlp_dev.h")


def _code_tokens(text):
    """C++ source with comments removed and whitespace collapsed (the hashed
    sources hold no string literal that contains a comment marker)."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash():
    """sha256 over the code of the stage kernels' sources (comments and
    whitespace do not enter) and the compiler flags of their two builds
    (other translation units of the library do not enter)."""
    import hashlib
    from paper_1301_4498_amd import build as B
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f)) as fh:
            h.update(_code_tokens(fh.read()).encode())
    flags = [B.COMMON] + [u for u in B.UNITS if u[0] == "nyx_step.hip"]
    h.update(repr(flags).encode())
    return h.hexdigest()


def measured_traffic(kernel, form, candidate, workload=None):
    """HBM bytes per launch of `kernel` under launch-order candidate
    `candidate` (the autotuner's choice for its stage) from the committed
    rocprofv3 counter record (profiles/traffic_*.json) of that workload, or
    None when no record was taken on the current kernel sources.  A record
    holds one value per candidate: the cell order changes how often
    neighbours are re-read from HBM, so the traffic of one order says
    nothing of another."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json"))):
        with open(path) as fh:
            rec = json.load(fh)
        if (rec.get("kernel") == kernel and rec.get("form") == form and
                (workload is None or rec.get("workload") == workload) and
                rec.get("sources_sha256") == kernel_source_hash()):
            return rec["bytes_per_launch_by_candidate"][candidate]
    return None


def aligned(torch, nbytes):
    raw = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    off = (-raw.data_ptr()) % 256
    return raw[off:off + nbytes]




def run_plan(nyx, torch, plan, A0, bufs, G, steps, warmup, dt_of, a_at, fill, dt_next_of=None):
    """`warmup` untimed steps of a batched plan from the initial state A0,
    with the device counters summed over them; then, from A0 again, `steps`
    timed steps (HIP events on torch's current stream, the library's stream)
    with the library's per-stage events.  dt_of(k) / dt_next_of(k): device dt
    tensors of step k; fill(state): the ghost fill after each step (a no-op
    where the plan reads ghost cells from their sources).  Returns ms per
    step, per-stage ms per step, the counters and the final state buffer."""
    st = torch.zeros(10, dtype=torch.int64, device="cuda")
    bufs[0].copy_(A0)
    for k in range(max(min(warmup, steps), 1)):
        plan.step(bufs[k % 2], G, dt_of(k), a_at(k), a_at(k + 1), bufs[(k + 1) % 2],
                  dt_next=dt_next_of(k) if dt_next_of else None, stats=st)
        fill(bufs[(k + 1) % 2])
    torch.cuda.synchronize()
    stats = nyx.stats_dict(st)
    bufs[0].copy_(A0)
    torch.cuda.synchronize()
    nyx._lib.profile_enable(True)
    nyx._lib.profile_read(reset=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    e0.record()
    for k in range(steps):
        ev[k][0].record()
        plan.step(bufs[k % 2], G, dt_of(k), a_at(k), a_at(k + 1), bufs[(k + 1) % 2],
                  dt_next=dt_next_of(k) if dt_next_of else None)
        ev[k][1].record()
        fill(bufs[(k + 1) % 2])
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    stage_ms, seq = nyx._lib.profile_read(reset=True)
    nyx._lib.profile_enable(False)
    stage_ms = {s: v / max(seq, 1) for s, v in stage_ms.items()}
    # the step call alone (every kernel it enqueues), per step
    stage_ms["step_call"] = sum(a.elapsed_time(b) for a, b in ev) / steps
    return ms, stage_ms, stats, bufs[steps % 2]


def iters_per_face(stats):
    return stats["riemann_iters"] / max(stats["riemann_calls"], 1)


def fallback_rate(stats):
    return stats["mlp_fallback"] / max(stats["mlp_used"] + stats["mlp_fallback"], 1)


def run_box(nyx, torch, w, prm, steps, warmup, table):
    """Time `steps` steps (after `warmup`) of one periodic box with a one-box
    batched plan and device-resident dt from the fused CFL of the previous
    step; returns rates, stage times and the final density."""
    n = w.n[0]
    box = nyx.make_box(w.n, 4, w.dx)
    gdt = torch.float64 if prm.precision == nyx.NYX_FP64 else torch.float32
    U = torch.from_numpy(w.state).cuda()
    Uo = U.clone()
    G = torch.from_numpy(w.grav).to(gdt).cuda()
    _, one = nyx.Batch.workspace_bytes(prm, [box])
    ws = aligned(torch, one)
    plan = nyx.Batch(prm, [box], ws)
    # the box is its own periodic domain: its ghost cells are read from their
    # periodic images inside the step, so no fill runs between steps
    plan.set_ghost_source(0)
    dts = torch.zeros(2, dtype=torch.float64, device="cuda")
    plan.estimate_dt(U, w.a0, 0.5, dts[0:1])
    # launch orders per stage from the library's autotuner (untimed); near-ties
    # go to the order with the least HBM traffic where a counter record of the
    # current kernels exists for this workload
    form = "mixed" if prm.precision != nyx.NYX_FP64 else "fp64"
    traffic = {}
    for i, stg in enumerate(STAGES):
        if prm.riemann == nyx.NYX_RIEMANN_LEARNED:
            break  # the records are of the plain kernels
        per = [measured_traffic(stg, form, c, "box256_smooth") for c in range(16)]
        if all(v is not None for v in per):
            traffic[i] = per
    tune, tune_ms = plan.autotune(U, G, dts[0:1], w.a_at(0), w.a_at(1), Uo, dt_next=dts[1:2],
                                  reps=3, traffic=traffic or None)
    # launch mode by time (the fused final stage where the form allows it)
    mode, mode_ms = plan.autotune_mode(U, G, dts[0:1], w.a_at(0), w.a_at(1), Uo, reps=3)
    persistent = mode == nyx.NYX_LAUNCH_PERSISTENT
    fused = mode == nyx.NYX_LAUNCH_FUSED and not (prm.learned_stages_mask & 4)
    st = torch.zeros(10, dtype=torch.int64, device="cuda")
    bufs = [U, Uo]
    k = 0

    def one_step(stats=None):
        nonlocal k
        src, dst = bufs[k % 2], bufs[(k + 1) % 2]
        plan.step(src, G, dts[k % 2:k % 2 + 1], w.a_at(k), w.a_at(k + 1), dst,
                  dt_next=dts[(k + 1) % 2:(k + 1) % 2 + 1], stats=stats)
        k += 1

    for i in range(max(warmup, 1)):
        one_step(st if i == 0 else None)  # counters of the first step
    torch.cuda.synchronize()
    stats = nyx.stats_dict(st)
    it = iters_per_face(stats)
    nyx._lib.profile_enable(True)
    nyx._lib.profile_read(reset=True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        one_step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    stage_ms, seq = nyx._lib.profile_read(reset=True)
    nyx._lib.profile_enable(False)
    stage_ms = {s: v / max(seq, 1) for s, v in stage_ms.items()}
    rho = bufs[k % 2].reshape(6, n + 8, n + 8, n + 8)[0, 4:-4, 4:-4, 4:-4].cpu().numpy()
    finite = bool(torch.isfinite(bufs[k % 2]).all().item())
    plan.close()
    del ws, U, Uo, G, bufs
    torch.cuda.empty_cache()
    mixed = prm.precision != nyx.NYX_FP64
    roof, hbm = roofline_of(stage_ms, table, [w.n], it, ms / steps, 4 if mixed else 8,
                            "fp64" if not mixed else "mixed", "box256_smooth", tune,
                            persistent_ms=ms / steps if persistent else None,  # the whole step
                            fused=fused)
    return {"zone_updates_per_s": n ** 3 * steps / (ms * 1e-3), "ms_per_step": ms / steps,
            "launch_mode": MODE_NAMES[mode], "mode_step_ms": dict(zip(MODE_NAMES, mode_ms)),
            "stage": None if persistent else stage_rates(stage_ms, table, [w.n], it, fused),
            "mean_riemann_iters": it,
            "stats_first_step": stats, "finite": finite, "rho": rho, "tuning": tune,
            "tuning_ms": tune_ms, "roofline": roof, "hbm_step": hbm}


def box256_leg(nyx, torch, synth, steps, warmup, log, n=256):
    """Single 256^3 box of smooth flow (seed 2): plain FP64 against
    FP32-mixed."""
    import numpy as np
    w = synth.config2(n=n)
    table = flop_table("box256")
    out = {"workload": "box256_smooth: one periodic %d^3 box + 4 ghosts, smooth-flow fields "
                       "(seed 2), a 0.25->0.26, CFL 0.5" % n, "steps": steps, "forms": {}}
    res = {}
    for f, prec in (("fp64", nyx.NYX_FP64), ("mixed", nyx.NYX_MIXED)):
        res[f] = run_box(nyx, torch, w, nyx.default_params(precision=prec), steps, warmup, table)
        log("box256 %s: %.3e zone-updates/s" % (f, res[f]["zone_updates_per_s"]))
    for f, v in res.items():
        v["rho_l1_vs_fp64"] = float(np.abs(v["rho"] - res["fp64"]["rho"]).sum() /
                                    np.abs(res["fp64"]["rho"]).sum())
        out["forms"][f] = {k: v[k] for k in ("zone_updates_per_s", "ms_per_step", "launch_mode",
                                             "mode_step_ms", "stage", "mean_riemann_iters",
                                             "finite", "rho_l1_vs_fp64", "tuning", "roofline",
                                             "hbm_step")}
    return out, w


def learned256_leg(nyx, torch, synth, learn, flux, steps, warmup, log, n=256):
    """A fresh-seed 256^3 box of the smooth-flow type (seed 7, not a training
    seed), 20 steps: FP32-mixed against the learned flux on all twelve
    solves per zone and on stages 0-1 only; density L1 against FP64 and
    against FP32-mixed, fallback rate."""
    import numpy as np
    w = synth.config2(n=n, seed=7)
    table = flop_table("box256")
    out = {"workload": "box256_smooth type, seed 7 (fresh), %d^3, a 0.25->0.26" % n,
           "steps": steps, "forms": {}}
    res = {}
    for f in ("fp64", "mixed", "learned", "learned01"):
        if f == "fp64":
            prm = nyx.default_params(precision=nyx.NYX_FP64)
        elif f == "mixed":
            prm = nyx.default_params(precision=nyx.NYX_MIXED)
        else:
            prm = learn.learned_params(flux, tol=1e-3, stages=7 if f == "learned" else 3)
        res[f] = run_box(nyx, torch, w, prm, steps, warmup, table)
        log("learned256 %s: %.3e zone-updates/s" % (f, res[f]["zone_updates_per_s"]))
    for f, v in res.items():
        r = {k: v[k] for k in ("zone_updates_per_s", "ms_per_step", "launch_mode", "stage",
                               "mean_riemann_iters", "finite")}
        for ref in ("fp64", "mixed"):
            r["rho_l1_vs_" + ref] = float(np.abs(v["rho"] - res[ref]["rho"]).sum() /
                                          np.abs(res[ref]["rho"]).sum())
        if f.startswith("learned"):
            r["fallback_rate"] = fallback_rate(v["stats_first_step"])
            r["gain_vs_mixed"] = v["zone_updates_per_s"] / res["mixed"]["zone_updates_per_s"]
        out["forms"][f] = r
    return out


def headline_leg(nyx, torch, synth, learn, steps, warmup, log, n=512, m=64, learned=True):
    """box512_stress: plain FP64 with the domain as one box, against
    FP32-mixed (and mixed + learned flux trained on stress faces) on an
    (n/m)^3 grid of m^3 patches in one batched plan with the same-level
    ghost fill and one level dt (the FP64 run's dt sequence).  Every plan is
    autotuned (untimed) first."""
    t0 = time.perf_counter()
    grid = (n // m,) * 3
    nb = grid[0] * grid[1] * grid[2]
    a0, a1 = 0.10, 0.11
    table = flop_table("box512_stress")

    def a_at(k):
        return a0 + (a1 - a0) * k / steps

    state, grav = synth.stress_fields_torch(n=n)
    log("stress fields ready in %.1f s" % (time.perf_counter() - t0))
    zones = n ** 3
    out = {"workload": "box512_stress: %d^3, density contrast <= 1e4, Mach <= 30, g ~ N(0, 0.2^2), "
                       "a 0.10->0.11, one level dt" % n, "steps": steps,
           "patches": "%d x %d^3" % (nb, m), "forms": {}}
    # plain FP64, one box, dt from its own fused CFL
    prm = nyx.default_params()
    box = nyx.make_box((n, n, n), 4, 1.0 / n)
    _, one = nyx.Batch.workspace_bytes(prm, [box])
    ws = aligned(torch, one)
    plan = nyx.Batch(prm, [box], ws)
    # the box is its own periodic domain: the primitive stage reads each ghost
    # cell's periodic image, so no separate ghost fill runs between steps
    plan.set_ghost_source(0)
    A0 = state
    bufs = [state.clone(), state.clone()]  # ghost cells stay the initial ones
    dts = torch.zeros(steps + 1, dtype=torch.float64, device="cuda")
    plan.estimate_dt(A0, a0, 0.5, dts[0:1])
    tune, _ = plan.autotune(A0, grav, dts[0:1], a_at(0), a_at(1), bufs[1], reps=2)
    # the plain step in its fastest launch mode too
    mode, mode_ms = plan.autotune_mode(A0, grav, dts[0:1], a_at(0), a_at(1), bufs[1], reps=2)
    persistent = mode == nyx.NYX_LAUNCH_PERSISTENT
    fused = mode == nyx.NYX_LAUNCH_FUSED
    ms, stage_ms, st, fin = run_plan(nyx, torch, plan, A0, bufs, grav, steps, warmup,
                                     lambda k: dts[k:k + 1], a_at, lambda s: None,
                                     dt_next_of=lambda k: dts[k + 1:k + 2])
    if persistent:
        assert not plan.persistent_aborted()
    rho64 = fin[0, 4:-4, 4:-4, 4:-4].contiguous()
    it = iters_per_face(st)
    roof, hbm = roofline_of(stage_ms, table, [(n, n, n)], it, ms, 8, "fp64", "box512_stress",
                            tune, persistent_ms=stage_ms["step_call"] if persistent else None,
                            fused=fused)
    out["forms"]["fp64_one_box"] = {
        "zone_updates_per_s": zones / (ms * 1e-3), "ms_per_step": ms,
        "launch_mode": MODE_NAMES[mode], "mode_step_ms": dict(zip(MODE_NAMES, mode_ms)),
        "stage": None if persistent else stage_rates(stage_ms, table, [(n, n, n)], it, fused),
        "mean_riemann_iters": it, "stats": st, "tuning": tune, "roofline": roof, "hbm_step": hbm,
        "finite": bool(torch.isfinite(fin).all().item())}
    log("stress fp64 one box: %.3e zone-updates/s" % (zones / (ms * 1e-3)))
    dt_host = dts.cpu().tolist()
    plan.close()
    del plan, ws, bufs, fin
    torch.cuda.empty_cache()
    # the same domain as patches (FP32 gravity), the FP64 run's level dt
    P = (m + 8) ** 3
    A0 = torch.cat([p.reshape(-1) for p in synth.split_patches(state, grid)])
    G32 = torch.cat([p.reshape(-1).float() for p in synth.split_patches(grav, grid)])
    sample = [(synth.split_patches(state, grid)[b].cpu().numpy(),
               synth.split_patches(grav, grid)[b].cpu().numpy()) for b in range(0, nb, nb // 64)]
    del state, grav
    torch.cuda.empty_cache()
    dtp = dts[:steps, None].expand(steps, nb).contiguous()
    boxes = [nyx.make_box((m, m, m), 4, 1.0 / n, state_off=6 * P * b, grav_off=3 * P * b)
             for b in range(nb)]
    shapes = [(m, m, m)] * nb
    # the mixed form as built (the star-state iteration stops at FP32
    # resolution), and with the FP64 form's stopping rule for comparison
    runs = [("mixed_patches", nyx.default_params(precision=nyx.NYX_MIXED)),
            ("mixed_patches_fp64_stop", nyx.default_params(precision=nyx.NYX_MIXED,
                                                           mixed_riemann_stop=1e-14))]
    if learned:
        sflux, out["learned_training"] = train_learned_stress(nyx, learn, synth, log)
        runs.append(("learned_patches", learn.learned_params(sflux, tol=1e-3, stages=7)))
    for name, prm in runs:
        _, one = nyx.Batch.workspace_bytes(prm, boxes)
        ws = aligned(torch, one)
        plan = nyx.Batch(prm, boxes, ws)
        # the same-level ghost exchange: the primitive stage reads each ghost
        # cell's source cell in the neighbouring patch (bitwise the result of
        # a ghost fill before the step), so no separate fill runs
        plan.set_ghost_source(1, grid)
        bufs = [A0.clone(), A0.clone()]  # ghost cells stay the initial ones
        # launch orders by time; near-ties go to the order with the least
        # HBM traffic where a counter record of the current kernels exists
        traffic = {}
        for i, stg in enumerate(STAGES):
            per = [measured_traffic(stg, "mixed", c, "box512_stress_patches") for c in range(16)]
            if all(v is not None for v in per):
                traffic[i] = per
        tune, _ = plan.autotune(A0, G32, dtp[0], a_at(0), a_at(1), bufs[1], reps=2,
                                traffic=(traffic or None) if name == "mixed_patches" else None)
        # staged, persistent or fused-final launch, whichever is fastest
        mode, mode_ms = plan.autotune_mode(A0, G32, dtp[0], a_at(0), a_at(1), bufs[1], reps=2)
        persistent = mode == nyx.NYX_LAUNCH_PERSISTENT
        fused = mode == nyx.NYX_LAUNCH_FUSED and not name.startswith("learned")

        ms, stage_ms, st, fin = run_plan(nyx, torch, plan, A0, bufs, G32, steps, warmup,
                                         lambda k: dtp[k], a_at, lambda s: None)
        if persistent:
            assert not plan.persistent_aborted()
        rho = synth.join_valid(fin, grid, (m, m, m))[0]
        l1 = float((rho - rho64).abs().sum() / rho64.abs().sum())
        it = iters_per_face(st)
        roof, hbm = roofline_of(stage_ms, table, shapes, it, ms, 4, "mixed",
                                "box512_stress_patches", tune,
                                persistent_ms=stage_ms["step_call"] if persistent else None,
                                fused=fused)
        r = {"zone_updates_per_s": zones / (ms * 1e-3), "ms_per_step": ms,
             "rho_l1_vs_fp64": l1, "finite": bool(torch.isfinite(fin).all().item()),
             "launch_mode": MODE_NAMES[mode],
             "mode_step_ms": dict(zip(MODE_NAMES, mode_ms)),
             "stage": None if persistent else stage_rates(stage_ms, table, shapes, it, fused),
             "step_call_ms": stage_ms["step_call"], "mean_riemann_iters": it,
             "stats": st, "tuning": tune, "roofline": roof, "hbm_step": hbm}
        if name.startswith("learned"):
            r["fallback_rate"] = fallback_rate(st)
        out["forms"][name] = r
        log("stress %s: %.3e zone-updates/s, rho L1 vs FP64 %.2e" % (name, r["zone_updates_per_s"], l1))
        plan.close()
        del plan, ws, bufs, fin
        torch.cuda.empty_cache()
    if "learned_patches" in out["forms"]:
        out["forms"]["learned_patches"]["gain_vs_mixed_patches"] = (
            out["forms"]["learned_patches"]["zone_updates_per_s"] /
            out["forms"]["mixed_patches"]["zone_updates_per_s"])
    out["dt_first"] = dt_host[0]
    return out, sample, (a_at(0), a_at(1)), 1.0 / n
def train_learned(nyx, learn, synth, log):
    """Harvest about 2e7 final-stage faces of plain FP64 steps on ten 64^3
    boxes of the same field type (seeds 100-109) and train the network
    (untimed)."""
    t0 = time.perf_counter()
    ws = [synth.config2(n=64, seed=100 + s) for s in range(10)]
    rec = learn.harvest(ws, steps=8, keep_fraction=0.31, capacity=21_000_000, seed=100)
    f = learn.LearnedFlux(seed=1)
    epochs = 4
    hist = f.train(rec, epochs=epochs, batch=16384)
    f.pack()
    info = {"records": int(rec.shape[0]), "boxes": "10 x 64^3, seeds 100-109, 8 steps",
            "epochs": epochs, "loss_first_epoch": hist[0],
            "loss_last_epoch": hist[-1], "seconds": round(time.perf_counter() - t0, 1)}
    log("learned flux trained: %s" % info)
    return f, info


def train_learned_stress(nyx, learn, synth, log):
    """A second network for the stress workload: about 2e7 final-stage faces
    of plain FP64 steps on ten 64^3 boxes of the stress fields (seeds
    500-509), trained like the first (untimed)."""
    t0 = time.perf_counter()
    ws = [synth.config5(n=64, seed=500 + s) for s in range(10)]
    rec = learn.harvest(ws, steps=8, keep_fraction=0.31, capacity=21_000_000, seed=500)
    f = learn.LearnedFlux(seed=2)
    epochs = 4
    hist = f.train(rec, epochs=epochs, batch=16384)
    f.pack()
    info = {"records": int(rec.shape[0]), "boxes": "10 x 64^3 stress fields, seeds 500-509, 8 steps",
            "epochs": epochs, "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1],
            "seconds": round(time.perf_counter() - t0, 1)}
    log("stress network trained: %s" % info)
    return f, info




def level_leg(nyx, torch, synth, learn, flux, steps, warmup, log):
    """4096 uneven boxes (each axis from {16, 24, 32, 48, 64}), smooth-flow
    fields per box, self-periodic ghosts, a 0.25 -> 0.255 over the steps.
    Plain FP64 batched first, with per-box dt from its fused CFL; its dt
    sequence then drives FP32-mixed batched (also replayed as a captured HIP
    graph) and mixed + learned flux, whose densities are compared with the
    FP64 run's over every box's valid cells; per-box FP64 launches (one
    nyx_hydro_step per box) are the baseline of the batching gain."""
    shapes = synth.config3_shapes()
    t0 = time.perf_counter()
    V = int(sum(a * b * c for a, b, c in shapes))
    out = {"boxes": len(shapes), "valid_cells": V, "steps": steps, "a": [0.25, 0.255]}
    a0, a1 = 0.25, 0.255

    def a_at(k):
        return a0 + (a1 - a0) * k / steps

    table = flop_table("box256")
    res = {}
    rho64 = None
    dt_seq = None
    forms = [("fp64", nyx.default_params(precision=nyx.NYX_FP64)),
             ("mixed", nyx.default_params(precision=nyx.NYX_MIXED))]
    if flux is not None:
        forms.append(("learned", learn.learned_params(flux, tol=1e-3, stages=7)))
    gdt_of = {"fp64": torch.float64, "mixed": torch.float32, "learned": torch.float32}
    for form, prm in forms:
        state, grav, offs = synth.level_fields_torch(shapes, grav_dtype=gdt_of[form])
        log("level fields (%s) ready in %.1f s" % (form, time.perf_counter() - t0))
        boxes = [nyx.make_box(n, 4, 1.0 / 256, state_off=so, grav_off=go)
                 for n, (so, go) in zip(shapes, offs)]
        _, one = nyx.Batch.workspace_bytes(prm, boxes)
        free = torch.cuda.mem_get_info()[0]
        wsb = min(one, int(free - 3 * state.numel() * 8 - (8 << 30)))
        ws = aligned(torch, wsb)
        plan = nyx.Batch(prm, boxes, ws)
        # every box is its own periodic domain: ghosts read from their images
        # inside the step
        plan.set_ghost_source(0)
        bufs = [state.clone(), state.clone()]  # ghost cells stay the initial ones
        if dt_seq is None:
            dt_seq = torch.zeros((steps + 1, len(boxes)), dtype=torch.float64, device="cuda")
            plan.estimate_dt(state, a0, 0.5, dt_seq[0])
            dt_next_of = lambda k: dt_seq[k + 1]  # noqa: E731
        else:
            dt_next_of = None
        tune, _ = plan.autotune(state, grav, dt_seq[0], a_at(0), a_at(1), bufs[1], reps=2)
        mode_ms = None
        if form != "fp64":
            mode, mode_ms = plan.autotune_mode(state, grav, dt_seq[0], a_at(0), a_at(1), bufs[1],
                                               reps=2)
        persistent = plan.launch_mode == nyx.NYX_LAUNCH_PERSISTENT
        fused = plan.launch_mode == nyx.NYX_LAUNCH_FUSED and form != "learned"
        ms, stage_ms, st, fin = run_plan(nyx, torch, plan, state, bufs, grav, steps, warmup,
                                         lambda k: dt_seq[k], a_at, lambda s: None,
                                         dt_next_of=dt_next_of)
        if persistent:
            assert not plan.persistent_aborted()
        it = iters_per_face(st)
        finite = bool(torch.isfinite(fin).all().item())
        # density of every box's valid cells
        num = torch.zeros((), dtype=torch.float64, device="cuda")
        den = torch.zeros((), dtype=torch.float64, device="cuda")
        rho_boxes = []
        for n, (so, _go) in zip(shapes, offs):
            nx, ny, nz = n
            P = (nx + 8) * (ny + 8) * (nz + 8)
            r = fin[so:so + P].view(nz + 8, ny + 8, nx + 8)[4:-4, 4:-4, 4:-4]
            if rho64 is None:
                rho_boxes.append(r.clone())
            else:
                ref = rho64[len(rho_boxes)]
                rho_boxes.append(None)
                num += (r - ref).abs().sum()
                den += ref.abs().sum()
        if rho64 is None:
            rho64 = rho_boxes
        roof, hbm = roofline_of(stage_ms, table, shapes, it, ms, 8 if form == "fp64" else 4,
                                form, "level4096", tune,
                                persistent_ms=stage_ms["step_call"] if persistent else None,
                                fused=fused)
        r = {"batched_zone_updates_per_s": V / (ms * 1e-3), "batched_ms_per_step": ms,
             "groups": plan.num_groups, "tuning": tune, "finite": finite,
             "launch_mode": MODE_NAMES[plan.launch_mode],
             "mode_step_ms": dict(zip(MODE_NAMES, mode_ms)) if mode_ms else None,
             "stage": None if persistent else stage_rates(stage_ms, table, shapes, it, fused),
             "mean_riemann_iters": it, "roofline": roof, "hbm_step": hbm}
        if form != "fp64":
            r["rho_l1_vs_fp64"] = float(num / den)
        if form == "learned":
            r["fallback_rate"] = fallback_rate(st)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        if form == "mixed":
            # two steps captured once, replayed
            def step(k):
                plan.step(bufs[k % 2], grav, dt_seq[k], a_at(k), a_at(k + 1), bufs[(k + 1) % 2])

            g = torch.cuda.CUDAGraph()
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                with torch.cuda.graph(g, stream=s):
                    step(0)
                    step(1)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            e0.record()
            for _ in range(steps // 2):
                g.replay()
            e1.record()
            torch.cuda.synchronize()
            gms = e0.elapsed_time(e1) / (2 * (steps // 2))
            r["graph_zone_updates_per_s"] = V / (gms * 1e-3)
            r["graph_ms_per_step"] = gms
            del g
        if form == "fp64":
            # per-box launches: one nyx_hydro_step per box (workspace of the largest box)
            big = max(nyx.workspace_bytes(prm, b) for b in boxes)
            wsb1 = aligned(torch, big)
            dth = dt_seq[0].cpu().tolist()
            torch.cuda.synchronize()
            e0.record()
            for b, bx in enumerate(boxes):
                nyx.hydro_step(prm, bx, state, grav, dth[b], a_at(0), a_at(1), bufs[1],
                               workspace=wsb1)
            e1.record()
            torch.cuda.synchronize()
            pms = e0.elapsed_time(e1)
            r["per_box_zone_updates_per_s"] = V / (pms * 1e-3)
            r["per_box_ms_per_step"] = pms
            del wsb1
        res[form] = r
        log("level %s: %s" % (form, {k: (float("%.4g" % v) if isinstance(v, float) else v)
                                     for k, v in r.items() if k not in ("stage", "tuning")}))
        plan.close()
        del plan, ws, state, grav, bufs, fin  # the plan object holds its workspace
        torch.cuda.empty_cache()
    del rho64
    torch.cuda.empty_cache()
    out["forms"] = res
    out["gain_batched_graph_vs_per_box_plain_fp64"] = (
        res["mixed"]["graph_zone_updates_per_s"] / res["fp64"]["per_box_zone_updates_per_s"])
    return out
def variants_leg(nyx, torch, w, steps, warmup, log):
    """The scheme variants of Sec. 3.2 on the benchmark box (FP32-mixed, each
    against its own plain FP64 run): PLM reconstruction, the linearised
    Riemann solver, the second form of the energy gravity term, and gamma =
    1.4, where the expansion term of the energy equations is applied."""
    import numpy as np
    out = {}
    for name, kw in (("plm", dict(recon=nyx.NYX_RECON_PLM)),
                     ("linearized_riemann", dict(riemann=nyx.NYX_RIEMANN_LINEARIZED)),
                     ("gravity_energy_form2", dict(grav_energy_form=2)),
                     ("gamma14_expansion", dict(gamma=1.4))):
        m = run_box(nyx, torch, w, nyx.default_params(precision=nyx.NYX_MIXED, **kw), steps, warmup,
                    flop_table("box256"))
        f = run_box(nyx, torch, w, nyx.default_params(precision=nyx.NYX_FP64, **kw), steps, warmup,
                    flop_table("box256"))
        l1 = float(np.abs(m["rho"] - f["rho"]).sum() / np.abs(f["rho"]).sum())
        out[name] = {"mixed_zone_updates_per_s": m["zone_updates_per_s"],
                     "fp64_zone_updates_per_s": f["zone_updates_per_s"],
                     "mixed_rho_l1_vs_fp64": l1, "finite": m["finite"] and f["finite"],
                     "mean_riemann_iters": m["mean_riemann_iters"]}
        log("variant %s: mixed %.3e, fp64 %.3e zone-updates/s, rho L1 %.2e"
            % (name, m["zone_updates_per_s"], f["zone_updates_per_s"], l1))
    return out


def level_fill_leg(nyx, torch, log, reps=5):
    """Ghost fill of AMR levels (Sec. 4.1): (a) 512 patches of 64^3 tiling
    a periodic 512^3 domain, every ghost cell a copy; (b) a fine level of 8
    boxes of 64^3 over the central 128^3 of a 512^3 domain above a coarse
    level of 64 boxes of 64^3 (ratio 2): copies between the fine boxes and
    limited linear interpolation from the coarse level on the outer faces.
    Algorithmic bytes: a copied cell reads and writes 6 FP64 components; an
    interpolated cell writes 6 and reads the coarse cell's 6 once per 8
    children."""
    m, ng = 64, 4
    P = (m + 2 * ng) ** 3
    out = {}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def grid_boxes(g, dx, lo0=(0, 0, 0)):
        boxes, lo = [], []
        for b in range(g[0] * g[1] * g[2]):
            boxes.append(nyx.make_box((m, m, m), ng, dx, state_off=6 * P * b))
            ijk = (b % g[0], (b // g[0]) % g[1], b // (g[0] * g[1]))
            lo.append(tuple(lo0[d] + m * ijk[d] for d in range(3)))
        return boxes, lo

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    # (a) copies only
    boxes, lo = grid_boxes((8, 8, 8), 1.0 / 512)
    state = torch.rand(512 * 6 * P, dtype=torch.float64, device="cuda")
    plan = nyx.FillPlan(boxes, lo, (512, 512, 512))
    nc, ni = plan.counts()
    ms = timed(lambda: plan.fill(state))
    gbs = nc * 96 / (ms * 1e-3) / 1e9
    out["patch_grid_512"] = {"copied_cells": nc, "ms": ms, "gbs": gbs,
                             "hbm_frac": gbs / HBM_PEAK_GBS}
    log("level fill, 512 x 64^3 patches: %.3f ms, %.0f GB/s" % (ms, gbs))
    plan.close()
    del state, plan
    torch.cuda.empty_cache()
    # (b) two levels
    cboxes, clo = grid_boxes((4, 4, 4), 1.0 / 256)
    cstate = torch.rand(64 * 6 * P, dtype=torch.float64, device="cuda")
    cplan = nyx.FillPlan(cboxes, clo, (256, 256, 256))
    cplan.fill(cstate)
    fboxes, flo = grid_boxes((2, 2, 2), 1.0 / 512, lo0=(192, 192, 192))
    fstate = torch.rand(8 * 6 * P, dtype=torch.float64, device="cuda")
    fplan = nyx.FillPlan(fboxes, flo, (512, 512, 512), coarse=(cboxes, clo))
    nc, ni = fplan.counts()
    ms = timed(lambda: fplan.fill(fstate, cstate))
    gbs = (nc * 96 + ni * (48 + 6)) / (ms * 1e-3) / 1e9
    out["two_level"] = {"copied_cells": nc, "interpolated_cells": ni, "ms": ms, "gbs": gbs,
                        "hbm_frac": gbs / HBM_PEAK_GBS}
    log("level fill, 8 fine boxes over 64 coarse boxes: %d copied, %d interpolated, %.3f ms, "
        "%.0f GB/s" % (nc, ni, ms, gbs))
    cplan.close()
    fplan.close()
    return out


def two_level_leg(nyx, torch, synth, w, log, steps=4):
    """One coarse step and two fine substeps with reflux and average-down
    (Sec. 4.3, Steps 2 and 8), FP32-mixed: the benchmark fields on a coarse
    level of 64 boxes of 64^3 (periodic 256^3), and a fine level of 8 boxes
    of 64^3 over the central 128^3 of the 512^3 fine domain (the coarse data
    injected).  Per two-level step: coarse ghost fill, coarse step feeding
    the flux register, coarse ghost fill of the new state, fine ghost fills
    from the coarse level interpolated in time to each substep's start, two
    fine substeps feeding the register, reflux, average-down.  Reports
    composite zone-updates/s (coarse cells + 2 x fine cells per step), the
    time of the sync kernels, and the composite mass change."""
    import numpy as np
    m, ng = 64, 4
    P = (m + 2 * ng) ** 3
    prm = nyx.default_params(precision=nyx.NYX_MIXED)
    cpad = synth.split_patches(w.state, (4, 4, 4))
    gpad = synth.split_patches(w.grav, (4, 4, 4))

    def boxes_of(g, dx, lo0=(0, 0, 0)):
        bx, lo = [], []
        for b in range(g[0] * g[1] * g[2]):
            bx.append(nyx.make_box((m, m, m), ng, dx, state_off=6 * P * b, grav_off=3 * P * b))
            ijk = (b % g[0], (b // g[0]) % g[1], b // (g[0] * g[1]))
            lo.append(tuple(lo0[d] + m * ijk[d] for d in range(3)))
        return bx, lo

    cb, clo = boxes_of((4, 4, 4), 1.0 / 256)
    fb, flo = boxes_of((2, 2, 2), 1.0 / 512, lo0=(192, 192, 192))
    c = torch.from_numpy(np.concatenate([np.ascontiguousarray(x).ravel() for x in cpad])).cuda()
    cg = torch.from_numpy(np.concatenate([np.ascontiguousarray(x).ravel() for x in gpad])).to(
        torch.float32).cuda()
    # fine data: the coarse cells under each fine box, injected (children = parent)
    fs, fgs = [], []
    for lo in flo:
        C0 = [x // 2 for x in lo]
        sl = (slice(None),) + tuple(slice(C0[2 - a] + ng - ng // 2, C0[2 - a] + ng + m // 2 + ng // 2)
                                    for a in range(3))
        for src, dst in ((w.state, fs), (w.grav, fgs)):
            blk = src[sl]
            dst.append(np.ascontiguousarray(blk.repeat(2, 1).repeat(2, 2).repeat(2, 3)).ravel())
    f = torch.from_numpy(np.concatenate(fs)).cuda()
    fg = torch.from_numpy(np.concatenate(fgs)).to(torch.float32).cuda()
    c2, f2 = c.clone(), f.clone()
    cfill = nyx.FillPlan(cb, clo, (256, 256, 256))
    ffill = nyx.FillPlan(fb, flo, (512, 512, 512), coarse=(cb, clo))
    sync = nyx.SyncPlan((fb, flo), (cb, clo), (512, 512, 512))
    nfaces, ncells, ncov = sync.counts()
    reg = sync.register()
    cbat = nyx.Batch(prm, cb, aligned(torch, nyx.Batch.workspace_bytes(prm, cb)[1]))
    fbat = nyx.Batch(prm, fb, aligned(torch, nyx.Batch.workspace_bytes(prm, fb)[1]))
    dtc = torch.zeros(64, dtype=torch.float64, device="cuda")
    cfill.fill(c)
    cbat.estimate_dt(c, w.a0, 0.5, dtc)
    cbat.min_dt(dtc)
    dt_c = float(dtc[0])
    dtf = torch.full((8,), 0.5 * dt_c, dtype=torch.float64, device="cuda")
    ffill.fill(f, c)
    a = [w.a0 + (w.a1 - w.a0) * k / (2 * steps + 2) for k in range(2 * steps + 3)]
    cbat.autotune(c, cg, dtc, a[0], a[2], c2, reps=2)
    fbat.autotune(f, fg, dtf, a[0], a[1], f2, reps=2)
    cbat.set_flux_register(sync, 0, reg)
    fbat.set_flux_register(sync, 1, reg)

    def composite_mass(cs, fst):
        cv = synth.join_valid(cs.view(-1), (4, 4, 4), (m, m, m))[0].cpu().numpy()
        fv = synth.join_valid(fst.view(-1), (2, 2, 2), (m, m, m))[0].cpu().numpy()
        return 8.0 * (cv.sum() - cv[96:160, 96:160, 96:160].sum()) + fv.sum()

    def two_level_step(k, src, dst):
        """coarse src -> dst (synchronised in dst); the fine level returns to f"""
        reg.zero_()
        cfill.fill(src)
        cbat.step(src, cg, dtc, a[2 * k], a[2 * k + 2], dst)
        cfill.fill(dst)
        ffill.fill(f, src)
        fbat.step(f, fg, dtf, a[2 * k], a[2 * k + 1], f2)
        ffill.fill(f2, src, coarse_new=dst, theta=0.5)
        fbat.step(f2, fg, dtf, a[2 * k + 1], a[2 * k + 2], f)
        sync.reflux(dst, reg)
        sync.average_down(dst, f)

    bufs = [c, c2]
    two_level_step(0, c, c2)
    torch.cuda.synchronize()
    mass0 = composite_mass(c2, f)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(1, steps + 1):
        two_level_step(k, bufs[k % 2], bufs[(k + 1) % 2])
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    mass1 = composite_mass(bufs[(steps + 1) % 2], f)
    # the same two-level steps replayed as one captured HIP graph (two steps,
    # the coarse state ping-ponging between the buffers)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            two_level_step(1, c, c2)
            two_level_step(2, c2, c)
    graph.replay()
    torch.cuda.synchronize()
    reps_g = max(steps // 2, 1)
    e0.record()
    for _ in range(reps_g):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1) / (2 * reps_g)
    del graph
    cells = 64 * m ** 3 + 2 * 8 * m ** 3
    # the sync kernels alone
    reps = 10
    e0.record()
    for _ in range(reps):
        sync.reflux(c2, reg)
        sync.average_down(c2, f)
    e1.record()
    torch.cuda.synchronize()
    sync_ms = e0.elapsed_time(e1) / reps
    out = {"coarse": "64 x 64^3 (256^3 periodic)", "fine": "8 x 64^3 over the central 128^3",
           "interface_faces": nfaces, "reflux_cells": ncells, "covered_cells": ncov,
           "ms_per_two_level_step": ms, "zone_updates_per_s": cells / (ms * 1e-3),
           "graph_ms_per_two_level_step": graph_ms,
           "graph_zone_updates_per_s": cells / (graph_ms * 1e-3),
           "sync_ms": sync_ms, "sync_frac": sync_ms / ms,
           "composite_mass_rel_change": abs(mass1 - mass0) / abs(mass0)}
    log("two-level step: %.3f ms, %.3e zone-updates/s (graph replay %.3f ms), reflux + "
        "average-down %.4f ms, composite mass change %.1e"
        % (ms, out["zone_updates_per_s"], graph_ms, sync_ms, out["composite_mass_rel_change"]))
    fbat.set_flux_register(None, 1, None)
    cbat.set_flux_register(None, 0, None)
    for x in (cfill, ffill, cbat, fbat, sync):
        x.close()
    return out


def gravity_leg(nyx, torch, synth, w, log, reps=3):
    """The gravity input of the step on the benchmark box (Sec. 2.4, 3.4):
    256^3 dark-matter particles (one per cell, displaced from the cell
    centres by N(0, 0.3 dx) per axis, equal masses of the mean gas density)
    deposited by cloud-in-cell, the periodic Poisson solve of the total
    density (deposit + the state's gas density) to a relative residual of
    1e-10 from zero and from the previous solution, and g = -grad(phi) into
    the FP32 padded gravity array of the step.  Algorithmic bytes: deposit
    32 B per particle read + 8 x 8 B of atomic adds; a red-black sweep of the
    finest level reads phi and f and writes phi, 24 B per cell; the gradient
    reads phi (8 B per cell) and writes 3 FP32 per padded cell."""
    import numpy as np
    n = w.n[0]
    dx = w.dx
    dom = (n, n, n)
    rng = np.random.default_rng(21)
    c = (np.arange(n) + 0.5) * dx
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    pos = np.stack([xx.ravel(), yy.ravel(), zz.ravel()])
    pos += rng.normal(0.0, 0.3 * dx, pos.shape)
    npart = pos.shape[1]
    mass = np.full(npart, float(w.state[0].mean()) * dx ** 3)
    pos_d = torch.from_numpy(pos).cuda()
    mass_d = torch.from_numpy(mass).cuda()
    del pos, zz, yy, xx
    box = nyx.make_box(w.n, 4, dx)
    state = torch.from_numpy(w.state).cuda()
    rho = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
    phi = torch.zeros_like(rho)
    grav = torch.zeros((3,) + w.state.shape[1:], dtype=torch.float32, device="cuda")
    solver = nyx.PoissonSolver(dom)
    coef = 4 * np.pi * 1.0 / w.a0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, k=reps):
        e0.record()
        for _ in range(k):
            out = fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k, out

    def deposit():
        rho.zero_()
        nyx.cic_deposit(pos_d, mass_d, dom, dx, rho)

    deposit()
    torch.cuda.synchronize()
    dep_ms, _ = timed(deposit)

    def cold():
        phi.zero_()
        return solver.solve(rho, phi, dx, coef, tol=1e-10, max_vcycles=40, state=state, box=box)

    cold()
    cold_ms, (cyc, rel) = timed(cold)
    # a warm start: the previous solution for a slightly moved density
    pos_d.add_(0.05 * dx)
    deposit()
    warm_ms, (wcyc, wrel) = timed(lambda: solver.solve(rho, phi, dx, coef, tol=1e-10,
                                                       max_vcycles=40, state=state, box=box), 1)
    grad_ms, _ = timed(lambda: nyx.gravity_from_phi(phi, dom, dx, box, grav, nyx.NYX_MIXED))
    # fixed-cycle form: kernels only, the V-cycle rate
    vc_ms, _ = timed(lambda: solver.enqueue(rho, phi, dx, coef, cyc, state=state, box=box))
    P = (n + 8) ** 3
    out = {"particles": npart, "deposit_ms": dep_ms,
           "deposit_gbs": npart * (32 + 64) / (dep_ms * 1e-3) / 1e9,
           "solve_cold_ms": cold_ms, "vcycles_cold": cyc, "rel_resid_cold": rel,
           "solve_warm_ms": warm_ms, "vcycles_warm": wcyc, "rel_resid_warm": wrel,
           "ms_per_vcycle_no_sync": vc_ms / cyc, "gradient_ms": grad_ms,
           "gradient_gbs": (n ** 3 * 8 + P * 12) / (grad_ms * 1e-3) / 1e9}
    log("gravity: deposit %d particles %.3f ms; solve %d V-cycles %.2f ms (rel resid %.1e), warm "
        "%d V-cycles %.2f ms; %.3f ms per V-cycle; gradient %.3f ms"
        % (npart, dep_ms, cyc, cold_ms, rel, wcyc, warm_ms, vc_ms / cyc, grad_ms))
    return out




def launch_modes_leg(nyx, torch, synth, log):
    """Staged, persistent and fused-final launches of FP32-mixed batched
    plans on small workloads, where launch overhead weighs most: the 32^3
    box of the smallest configuration, and a level of 512 boxes of 16^3
    (smooth-flow fields).  Every mode from nyx_batch_autotune_mode (best of 5
    steps after one untimed, launch orders autotuned first)."""
    out = {}
    cases = {"box32_plain (one 32^3 box)": [(32, 32, 32)], "level of 512 boxes of 16^3": [(16, 16, 16)] * 512}
    for name, shapes in cases.items():
        if len(shapes) == 1:
            w = synth.config1()
            state = torch.from_numpy(w.state).cuda()
            grav = torch.from_numpy(w.grav).float().cuda()
            boxes = [nyx.make_box(w.n, 4, w.dx)]
            a0 = w.a0
        else:
            state, grav, offs = synth.level_fields_torch(shapes, grav_dtype=torch.float32)
            boxes = [nyx.make_box(n, 4, 1.0 / 256, state_off=so, grav_off=go)
                     for n, (so, go) in zip(shapes, offs)]
            a0 = 0.25
        prm = nyx.default_params(precision=nyx.NYX_MIXED)
        _, one = nyx.Batch.workspace_bytes(prm, boxes)
        ws = aligned(torch, one)
        plan = nyx.Batch(prm, boxes, ws)
        dt = torch.zeros(len(boxes), dtype=torch.float64, device="cuda")
        plan.estimate_dt(state, a0, 0.5, dt)
        other = torch.empty_like(state)
        plan.autotune(state, grav, dt, a0, a0 * 1.001, other, reps=2)
        mode, ms = plan.autotune_mode(state, grav, dt, a0, a0 * 1.001, other, reps=5)
        V = sum(a * b * c for a, b, c in shapes)
        out[name] = {"%s_ms" % m: v for m, v in zip(MODE_NAMES, ms)}
        out[name].update({"%s_zone_updates_per_s" % m: V / (v * 1e-3) if v > 0 else None
                          for m, v in zip(MODE_NAMES, ms)})
        out[name]["kept"] = MODE_NAMES[mode]
        log("launch modes, %s: staged %.4f ms, persistent %.4f ms, fused %.4f ms"
            % (name, ms[0], ms[1], ms[2]))
        plan.close()
        del plan, ws, state, grav, other
        torch.cuda.empty_cache()
    return out


def cpu_baseline(sample, a_pair, dx, dt, budget_s=12.0):
    """The FP64 oracle on 64^3 patches (+4 ghosts, cut from the headline's
    fields): one step per patch, on all usable host cores (one thread per
    core, at most 16; the oracle's C step releases the GIL) for about
    `budget_s` seconds, then one patch on one thread."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    m = sample[0][0].shape[-1] - 8
    threads = max(1, min(16, len(os.sched_getaffinity(0))))

    def one(i):
        U, g = sample[i % len(sample)]
        oracle.hydro_step(U, g, 4, dt, dx, a_pair[0], a_pair[1])
        return 1

    done = 0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        i = 0
        while time.perf_counter() - t0 < budget_s:
            done += sum(ex.map(one, range(i, i + threads)))
            i += threads
    el = time.perf_counter() - t0
    t1 = time.perf_counter()
    one(0)
    el1 = time.perf_counter() - t1
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")),
                         "")
    except OSError:
        pass
    return {"value": m ** 3 * done / el, "unit": "zone-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d one-step runs of %d^3 patches (+4 ghosts) of the headline's stress "
                      "fields (%d distinct patches), %d threads" % (done, m, len(sample), threads),
            "single_thread": {"value": m ** 3 / el1, "unit": "zone-updates/s", "cores": 1},
            "host": {"cpu_model": model, "nproc": os.cpu_count(),
                     "usable_cpus": len(os.sched_getaffinity(0))}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="steps of the headline (box512_stress)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=512, help="edge of the headline domain")
    ap.add_argument("--steps256", type=int, default=20, help="steps of the 256^3 legs")
    ap.add_argument("--no-learned", action="store_true", help="skip every learned-flux form")
    ap.add_argument("--no-box256", action="store_true", help="skip the 256^3 legs")
    ap.add_argument("--no-level", action="store_true", help="skip the 4096-box batched leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the PLM / linearised-solver / gravity-form-2 leg")
    ap.add_argument("--no-fill", action="store_true", help="skip the level ghost-fill leg")
    ap.add_argument("--no-two-level", action="store_true",
                    help="skip the two-level step (reflux, average-down) leg")
    ap.add_argument("--no-gravity", action="store_true",
                    help="skip the gravity input leg (deposit, Poisson solve, gradient)")
    ap.add_argument("--only-headline", action="store_true", help="the headline leg alone")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB (3 times), to scale HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the path would shard by boxes with a "
              "halo exchange; multi-GPU runs are not part of it)", file=sys.stderr)
        sys.exit(2)
    import torch

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if args.copy_calibration:
        nbytes = 1 << 30
        a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        b.copy_(a)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(3):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes,
                          "ms_per_copy": ms, "gbs_read_plus_write": 2 * nbytes / ms / 1e6}))
        return
    if args.only_headline:
        args.no_box256 = args.no_level = args.no_variants = args.no_fill = True
        args.no_two_level = args.no_gravity = True
    import paper_1301_4498_amd as nyx
    from paper_1301_4498_amd import learn, synth
    nyx.lib()
    H, sample, a_pair, dxh = headline_leg(nyx, torch, synth, learn, args.steps, args.warmup, log,
                                          n=args.n, learned=not args.no_learned)
    F = H["forms"]
    base = F["fp64_one_box"]
    ok = [f for f in F if f not in ("fp64_one_box", "mixed_patches_fp64_stop") and F[f]["finite"]
          and F[f]["rho_l1_vs_fp64"] <= 1e-3]
    chosen = max(ok, key=lambda f: F[f]["zone_updates_per_s"]) if ok else "fp64_one_box"
    R = F[chosen]
    learned_used = chosen.startswith("learned")
    out = {
        "metric": METRIC,
        "value": R["zone_updates_per_s"],
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": R["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64+bf16" if learned_used else ("f64" if chosen == "fp64_one_box" else "f32+f64"),
        "data": "synthetic",
        "config": {"workload": "box512_stress: one %d^3 periodic domain (density contrast <= 1e4, "
                               "Mach <= 30, strong gravity, a 0.10->0.11, one level dt); chosen "
                               "form %s on %s patches; plain FP64 as one box alongside"
                               % (args.n, chosen, H["patches"]),
                   "form": chosen, "parallelism": "none",
                   "ghost_exchange": "inside the step: the primitive stage reads each ghost "
                                     "cell's source cell (the neighbouring patch's, the one "
                                     "box's periodic image), bitwise a ghost fill before it"},
        "plain_fp64_zone_updates_per_s": base["zone_updates_per_s"],
        "gain_vs_plain_fp64": R["zone_updates_per_s"] / base["zone_updates_per_s"],
        "rho_l1_vs_fp64": R.get("rho_l1_vs_fp64"),
        "roofline": R["roofline"],
        "hbm_step": R["hbm_step"],
        "box512_stress": H,
    }
    log("headline: %s %.3e zone-updates/s (plain FP64 one box %.3e, x%.2f); roofline %s %s %.3f"
        % (chosen, R["zone_updates_per_s"], base["zone_updates_per_s"],
           out["gain_vs_plain_fp64"], R["roofline"]["kernel"], R["roofline"]["bound"],
           R["roofline"]["frac"]))
    flux = None
    w = None
    if not args.no_box256:
        out["box256"], w = box256_leg(nyx, torch, synth, args.steps256, args.warmup, log)
        if not args.no_learned:
            flux, out["learned_training"] = train_learned(nyx, learn, synth, log)
            out["learned256"] = learned256_leg(nyx, torch, synth, learn, flux, args.steps256,
                                               args.warmup, log)
    if not args.no_level:
        out["level4096"] = level_leg(nyx, torch, synth, learn, flux, 10, args.warmup, log)
        out["launch_modes"] = launch_modes_leg(nyx, torch, synth, log)
    if w is None and not (args.no_variants and args.no_two_level and args.no_gravity):
        w = synth.config2(n=256)
    if not args.no_variants:
        out["variants"] = variants_leg(nyx, torch, w, 10, args.warmup, log)
    if not args.no_fill:
        out["level_fill"] = level_fill_leg(nyx, torch, log)
    if not args.no_two_level:
        out["two_level"] = two_level_leg(nyx, torch, synth, w, log)
    if not args.no_gravity:
        out["gravity"] = gravity_leg(nyx, torch, synth, w, log)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sample, a_pair, dxh, H["dt_first"])
        log("cpu baseline: %.3e zone-updates/s on %d threads (one thread %.3e)"
            % (out["cpu_baseline"]["value"], out["cpu_baseline"]["cores"],
               out["cpu_baseline"]["single_thread"]["value"]))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
