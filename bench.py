#!/usr/bin/env python3
"""Throughput of the RK4 hot path on one MI355X.

A "step" is one classic RK4 step over the whole grid of the workload (four
stage launches, or two fused stage-pair launches); the metric is
cell-velocity-stage updates per second (nz * nv * 4 per step) plus the HBM
bandwidth those updates imply.  The default (headline) workload is the
largest single-GPU configuration: WENO7 on 2^20 x 512 cells (L = 1e5,
omega = 1e-3, lambda = 10, ELN-crossing Gaussian family), in the
FP32-with-FP64-accumulation form, with its FP64 twin beside it.  The same line
carries, as secondary entries, WENO7 on 65536 x 256 and FD + KO on
16384 x 128 (autotuned over single stages, fused stage pairs and the whole
step in one launch) in both forms and the batch of 64 uneven instances, each
with its roofline, and a copy-bandwidth ceiling measured in the same run.

Output: one JSON line on stdout.  Inputs are resident in HBM before the
timed region starts.  --gpus N with N > 1 exits: the library runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell·v·stage updates/s + HBM GB/s, FP32 vs FP64 at stated error vs oracle"
PEAK_HBM_GBPS = 8000.0
WORKLOADS = {
    "fd_ko_16384x128": lambda prec: __import__("paper_2203_12866_amd.workloads", fromlist=["x"]).fd_16384x128(2, prec),
    "fv_weno7_65536x256": lambda prec: __import__("paper_2203_12866_amd.workloads", fromlist=["x"]).fv_65536x256(3, prec),
    "fv_weno7_1048576x512": lambda prec: __import__("paper_2203_12866_amd.workloads", fromlist=["x"]).fv_1m_x512(5, prec),
    "fd_ko_512x32": lambda prec: dict(__import__("paper_2203_12866_amd.workloads", fromlist=["x"]).small_fd(1), precision=prec),
}
FORMS = {"fp32acc": 1, "fp64": 0}
DEFAULT_WORKLOAD = "fv_weno7_1048576x512"
# grids above this many cells are compared between forms on slabs (cosenu_get_rows)
# instead of whole states copied to the host
SLAB_CELLS = 1 << 26
SLAB_ROWS = 2048
KERNEL_SOURCES = ("paper_2203_12866_amd/csrc/stage_kernels.hip",)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# VALU issue capacity of the chip: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64
# instruction per 4 cycles per SIMD (16 lanes per cycle for FP64 and for
# unpacked FP32), in billions of wave instructions per second
PEAK_VALU_GINST = 256 * 4 * 2.4 / 4.0
SIMDS, CLOCK_HZ = 256 * 4, 2.4e9


def profile_entry(workload: str, form: str):
    """The committed rocprofv3 summary of one launch of this workload and form
    (HBM bytes, VALU instructions), or None if it is missing or was taken on
    different kernel sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_hash():
        return None
    return t.get("entries", {}).get(f"{workload}/{form}")


def measured_traffic(workload: str, form: str):
    """HBM bytes per launch from the committed counter summary, or None."""
    e = profile_entry(workload, form)
    return None if e is None else e.get("bytes_per_launch")


def alu_roofline(workload: str, form: str, launch_s: float):
    """VALU issue rate of the launches: the profiled VALU wave instructions per
    launch over the launch duration measured in this run, against the chip's
    issue capacity; None without a matching profile."""
    e = profile_entry(workload, form)
    if e is None or not e.get("valu_insts_per_launch"):
        return None
    g = e["valu_insts_per_launch"] / launch_s / 1e9
    out = {"achieved": g, "peak": PEAK_VALU_GINST, "unit": "G VALU wave64 instructions/s",
           "frac": g / PEAK_VALU_GINST, "valu_insts_per_launch": e["valu_insts_per_launch"]}
    if e.get("valu_issue_cycles_per_launch"):
        # the same instructions priced per class (FP64 and transcendental instructions take more
        # issue cycles than FP32 ones): the share of the chip's issue cycles the launch needs
        out["priced_frac"] = e["valu_issue_cycles_per_launch"] / (SIMDS * CLOCK_HZ * launch_s)
    return out


def tracked(w, c0, c1):
    """The quantities the configuration tracks, from the diagnostics at the
    start and the end of a run: the survival probabilities and the drift of
    every quantity the discrete scheme conserves at this omega and lambda
    (N_nu, N_nubar and the trace of M0 always; all of M0 at omega = lambda = 0;
    M0_z at omega = 0; B.M0 at lambda = 0), relative to N_nu + N_nubar."""
    scale = abs(c0["N_nu"]) + abs(c0["N_nubar"])
    d = {"N_nu": c1["N_nu"] - c0["N_nu"], "N_nubar": c1["N_nubar"] - c0["N_nubar"],
         "M0_trace": c1["M0"][0] - c0["M0"][0]}
    if w["omega"] == 0.0:
        d["M0_z"] = c1["M0"][3] - c0["M0"][3]
    if w["lam"] == 0.0:
        d["B_dot_M0"] = c1["B_dot_M0"] - c0["B_dot_M0"]
    if w["omega"] == 0.0 and w["lam"] == 0.0:
        d["M0_x"] = c1["M0"][1] - c0["M0"][1]
        d["M0_y"] = c1["M0"][2] - c0["M0"][2]
    return {"t": c1["t"], "steps": c1["step"], "Pee_nu": c1["Pee_nu"], "Pee_nubar": c1["Pee_nubar"],
            "dP_max": c1["dP_max"], "max_rel_drift": max(abs(v) for v in d.values()) / scale,
            "rel_drift": {k: v / scale for k, v in d.items()}}


def _slab_starts(w):
    """Three slab positions: the perturbation at the domain centre, the periodic
    seam, and a seeded random place."""
    import numpy as np
    nz = w["nz"]
    rng = np.random.default_rng(12345)
    return [nz // 2 - SLAB_ROWS // 2, nz - SLAB_ROWS // 2, int(rng.integers(0, nz))]


def run_form(cosenu, torch, w, steps, warmup, seg, stage_steps, fused=True):
    sim = cosenu.Sim(w)
    c0 = sim.conserved()
    sim.bind_torch_stream()
    sim.set_fusion(fused)
    chosen = sim.autotune() if seg is None else seg
    if seg is not None:
        sim.set_seg_rows(seg)
    sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev_ms = sim.time_steps(steps)           # HIP events around the K steps, then waits
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms = sim.time_stages(stage_steps)  # one event pair around every stage launch
    info = sim.info()
    if w["nz"] * w["nv"] > SLAB_CELLS:
        state = {z0: sim.get_rows(z0, SLAB_ROWS) for z0 in _slab_starts(w)}
    else:
        state = sim.get_state()
    track = tracked(w, c0, sim.conserved())
    sim.close()
    cells = w["nz"] * w["nv"]
    # average launch duration over the timed region: HIP events on the sim's
    # stream around the K graph launches (4 single stages or 2 fused stage
    # pairs per step)
    nl = info["launches_per_step"]
    launch_s = ev_ms / (nl * steps) / 1e3
    return dict(seg=chosen, wall=wall, ev_ms=ev_ms, stage_ms=stage_ms, info=info, state=state, tracked=track,
                updates=cells * 4.0 * steps / wall, launches=nl,
                gbps_model=info["bytes_per_step"] * steps / wall / 1e9,
                launch_s=launch_s,
                stage_us=[m * 1e3 / stage_steps for m in stage_ms[:nl]],
                achieved_gbps=info["bytes_per_step"] / nl / launch_s / 1e9)


def form_difference(a, b):
    """FP32-form minus FP64-form state: max-abs over everything, and the
    off-diagonal planes relative to their largest magnitude (whole states, or
    the same slabs of both)."""
    import numpy as np
    if isinstance(a, dict):
        a = np.concatenate([a[k] for k in sorted(a)], axis=1)
        b = np.concatenate([b[k] for k in sorted(b)], axis=1)
    off = [2, 3, 6, 7]
    return {"max_abs": float(np.abs(a - b).max()),
            "max_rel_offdiag": float(np.abs(a[off] - b[off]).max() / max(np.abs(b[off]).max(), 1e-300))}


def copy_ceiling(torch, gib=2, reps=10):
    """Device-to-device copy bandwidth (bytes read + written per second) of a
    torch copy of `gib` GiB, timed with events on torch's stream: the practical
    streaming ceiling of this GPU, measured in the same run."""
    n = (gib << 30) // 4
    a = torch.ones(n, device="cuda", dtype=torch.float32)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    gbps = 2.0 * a.numel() * a.element_size() * reps / (ms * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return {"gbps": gbps, "what": f"torch device copy of {gib} GiB, {reps} repetitions (read + write bytes)"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_sample(o, w, rows, steps):
    """Time the oracle over `steps` whole RK4 steps of a periodic slab of `rows`
    z rows (the full grid when rows = nz), with the workload's dz and dt."""
    nz = w["nz"]
    ws = w if rows >= nz else dict(w, nz=rows, L=rows * (w["L"] / nz))
    p = o.problem_from_workload(ws)
    y0 = o.initial_state_for(ws)
    t0 = time.perf_counter()
    y = o.rk4(p, y0, steps)
    dt = time.perf_counter() - t0
    return rows * w["nv"] * 4.0 * steps / dt, dt, y


def cpu_baseline(cosenu, w, budget_s):
    """The FP64 oracle (as it stands: O(nv) self-interaction sum per cell,
    OpenMP over z) on a bounded sample of the workload, on all host threads and
    on one; where the full grid fits the budget, also the GPU forms' error
    against it after the same steps."""
    import numpy as np
    from oracle import oracle as o
    nz, nv = w["nz"], w["nv"]
    threads = o.num_threads()
    probe_rows = min(nz, 64)
    rate, _, _ = _oracle_sample(o, w, probe_rows, 1)
    full_step_s = nz * nv * 4.0 / rate
    errs = None
    if full_step_s <= budget_s:
        n = max(1, min(20, int(budget_s / full_step_s)))
        rate, total, y = _oracle_sample(o, w, nz, n)
        sample = f"{n} RK4 step(s) of the full {nz}x{nv} grid from the initial state, {total:.1f} s"
        errs = {"steps": n, "vs_oracle": {}}
        for form, prec in FORMS.items():
            with cosenu.Sim(dict(w, precision=prec)) as s:
                s.step(n)
                g = s.get_state()
            e = {"max_abs": float(np.abs(g - y).max())}
            if prec != 0:
                e["max_rel_offdiag"] = float(np.abs(g[2:4] - y[2:4]).max() / np.abs(y[2:4]).max())
            errs["vs_oracle"][form] = e
    else:
        rows = max(probe_rows, min(nz, int(budget_s * rate / (nv * 4.0)) // 64 * 64))
        rate, total, _ = _oracle_sample(o, w, rows, 1)
        sample = f"1 RK4 step of a periodic {rows}x{nv} z-slab (same dz, dt) of the {nz}x{nv} grid, {total:.1f} s"
    # one thread, on a slab sized to about a third of the budget
    o.set_num_threads(1)
    try:
        r1, _, _ = _oracle_sample(o, w, min(nz, 16), 1)
        rows1 = max(16, min(nz, int(budget_s / 3.0 * r1 / (nv * 4.0)) // 16 * 16))
        r1, t1, _ = _oracle_sample(o, w, rows1, 1)
    finally:
        o.set_num_threads(threads)
    cb = {"value": rate, "unit": "cell·v·stage updates/s", "cores": threads, "kind": "oracle",
          "cpu_model": cpu_model(), "host_threads": os.cpu_count(),
          "sample": f"FP64 oracle, {threads} threads: {sample}",
          "one_core": {"value": r1, "cores": 1,
                       "sample": f"1 RK4 step of a periodic {rows1}x{nv} z-slab, 1 thread, {t1:.1f} s"}}
    return cb, errs


def cpu_baseline_per_config(budget_each: float):
    """The FP64 oracle (all host threads) on a bounded sample of every
    configuration, as cell-velocity-stage updates/s: the 512 x 32 case whole,
    periodic z-slabs (same dz and dt) of the others, and slabs of the first
    four instances of the 64-instance batch (their nv and schemes differ)."""
    from oracle import oracle as o
    from paper_2203_12866_amd import workloads as wl
    out = {}

    def slab_rate(w, budget):
        r, _, _ = _oracle_sample(o, w, min(w["nz"], 16), 1)
        rows = max(16, min(w["nz"], int(budget * r / (w["nv"] * 4.0)) // 16 * 16))
        return _oracle_sample(o, w, rows, 1)[:2] + (rows,)

    w1 = wl.small_fd(1)
    r1, t1, _ = _oracle_sample(o, w1, w1["nz"], 2)
    out["fd_ko_512x32"] = {"value": r1, "sample": f"2 RK4 steps of the whole 512x32 grid, {t1:.1f} s"}
    for name, w in (("fd_ko_16384x128", wl.fd_16384x128(2, 0)), ("fv_weno7_65536x256", wl.fv_65536x256(3, 0)),
                    ("fv_weno7_1048576x512", wl.fv_1m_x512(5, 0))):
        r, t, rows = slab_rate(w, budget_each)
        out[name] = {"value": r, "sample": f"1 RK4 step of a periodic {rows}x{w['nv']} z-slab, {t:.1f} s"}
    upd = secs = 0.0
    parts = []
    for w in wl.batch_64(4)[:4]:
        w = dict(w, precision=0)
        r, t, rows = slab_rate(w, budget_each / 4.0)
        upd += r * t
        secs += t
        parts.append(f"{rows}x{w['nv']} {'FD' if w['scheme'] == 0 else 'WENO7'}")
    out["batch_64"] = {"value": upd / secs, "sample": "1 RK4 step of periodic z-slabs of instances 0-3 ("
                       + ", ".join(parts) + f"), {secs:.1f} s"}
    for v in out.values():
        v["unit"] = "cell·v·stage updates/s"
    return out


# kernel variants of a batch, in the order cosenu_batch_autotune reports them
BATCH_VARIANTS = ["fd_nv<=32", "fd_nv>32", "weno7_nv<=32", "weno7_nv>32", "fd_ko3_nv<=32", "fd_ko3_nv>32",
                  "fd_pairs_w2", "fd_pairs_w4", "fd_pairs_w6", "fd_pairs_w8",
                  "fd_whole_w2", "fd_whole_w4", "fd_whole_w6", "fd_whole_w8"]


def run_batch(cosenu, torch, insts, steps, warmup):
    """The batched workload: every instance advanced by one step graph per
    step, segment lengths chosen in place by the batch autotuner (one per
    kernel variant)."""
    b = cosenu.Batch(insts)
    t0 = time.perf_counter()
    segs = b.autotune()
    tune_s = time.perf_counter() - t0
    b.step(warmup)
    b.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev_ms = b.time_steps(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    infos = [b.info(i) for i in range(len(insts))]
    bad = sum(1 for i in range(len(insts)) if b.conserved(i)["nonfinite"])
    b.close()
    cells = sum(w["nz"] * w["nv"] for w in insts)
    bytes_step = sum(inf["bytes_per_step"] for inf in infos)
    launch_s = ev_ms / (4.0 * steps) / 1e3
    fused = sum(1 for inf in infos if inf["launches_per_step"] == 2)
    whole = sum(1 for inf in infos if inf["launches_per_step"] == 1)
    return dict(wall=wall, ev_ms=ev_ms, cells=cells, updates=cells * 4.0 * steps / wall, fused=fused, whole=whole,
                gbps_model=bytes_step * steps / wall / 1e9, bytes_step=bytes_step,
                achieved_gbps=bytes_step / 4.0 / launch_s / 1e9, launch_s=launch_s,
                segs=segs, tune_s=tune_s, nonfinite=bad)


def batch_summary(r, insts, steps):
    n_fd = sum(1 for w in insts if w["scheme"] == 0)
    return {
        "value": r["updates"], "unit": "cell·v·stage updates/s", "steps": steps,
        "ms_per_step": r["wall"] * 1e3 / steps,
        "config": {"workload": "batch_64", "instances": len(insts), "fd_ko": n_fd, "fv_weno7": len(insts) - n_fd,
                   "cells": r["cells"], "nz_range": [min(w["nz"] for w in insts), max(w["nz"] for w in insts)],
                   "nv_set": sorted({w["nv"] for w in insts}), "form": "FP32 stencils, FP64 moments/commutator/RK4",
                   "seg_rows_per_variant": {k: v for k, v in zip(BATCH_VARIANTS, r["segs"]) if v},
                   "fused_pair_instances": r["fused"], "whole_step_instances": r["whole"]},
        "modelled_gbps": r["gbps_model"],
        "bytes_per_update": r["bytes_step"] / (r["cells"] * 4.0),
        # the variants' launch chains overlap, so there is no single launch
        # duration: the whole step's algorithmic bytes over its graph time
        "roofline": {"bound": "hbm", "achieved": r["achieved_gbps"], "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": r["achieved_gbps"] / PEAK_HBM_GBPS,
                     "traffic": measured_traffic("batch_64", "fp32acc"),
                     "kernel": "batch_quad_kernel / batch_pair_kernel (FD whole steps or fused pairs) and "
                               "batch_stage_kernel (WENO7, FD nv<=32), one launch chain per variant, concurrent "
                               "graph branches",
                     "step_us": r["ev_ms"] * 1e3 / steps},
        "nonfinite_instances": r["nonfinite"],
        "autotune_s": r["tune_s"],
    }


def batch_main(args, cosenu, torch):
    from paper_2203_12866_amd import workloads as wl
    insts = wl.batch_64(4)
    r = run_batch(cosenu, torch, insts, args.steps, args.warmup)
    print(f"[bench] batch_64 fp32acc: {r['updates']:.4e} upd/s, {r['gbps_model']:.0f} GB/s modelled, "
          f"segments per variant {r['segs']} tuned in {r['tune_s']:.1f} s", file=sys.stderr, flush=True)
    b = batch_summary(r, insts, args.steps)
    out = {"metric": METRIC, "value": b["value"], "unit": b["unit"], "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": b["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32+f64acc", "data": "synthetic"}
    out.update({k: v for k, v in b.items() if k not in out})
    print(json.dumps(out), flush=True)


def kernel_name(w, launches, form):
    f = "FP32acc" if form == "fp32acc" else "FP64"
    if launches == 1:
        return f"quad_kernel<FD,{f}> (the whole RK4 step in one launch)"
    if launches == 2:
        return f"pair_kernel<FD,{f}> (stages 1+2 and 3+4 fused)"
    return f"stage_kernel<FD,{f}>" if w["scheme"] == 0 else f"stage_kernel<WENO7,{f}>"


PATHS = {1: "whole step", 2: "fused stage pairs", 4: "single stages"}


def run_workload(cosenu, torch, name, steps, warmup, seg, stage_steps, fused):
    """Both forms of one workload: per-form throughput, the roofline of its
    dominant kernel, the FP32-form / FP64-form difference and the tracked
    quantities."""
    mk = WORKLOADS[name]
    res = {}
    for form, prec in FORMS.items():
        res[form] = run_form(cosenu, torch, mk(prec), steps, warmup, seg, stage_steps, fused=fused)
        print(f"[bench] {name} {form}: {res[form]['updates']:.4e} upd/s, "
              f"{res[form]['gbps_model']:.0f} GB/s modelled, seg {res[form]['seg']}, "
              f"{res[form]['launches']} launches/step", file=sys.stderr, flush=True)
    w = mk(1)
    cells = w["nz"] * w["nv"]
    forms = {}
    for form, r in res.items():
        nl = r["launches"]
        suffix = {1: "/whole", 2: "/pairs", 4: ""}[nl]
        traffic = measured_traffic(name, form + suffix)
        hbm = {"bound": "hbm", "achieved": r["achieved_gbps"], "peak": PEAK_HBM_GBPS, "unit": "GB/s",
               "frac": r["achieved_gbps"] / PEAK_HBM_GBPS, "traffic": traffic}
        if traffic:
            # counter bytes per launch over this run's launch duration, and over the algorithmic bytes
            hbm["traffic_gbps"] = traffic / r["launch_s"] / 1e9
            hbm["traffic_over_algorithmic"] = traffic / (r["info"]["bytes_per_step"] / nl)
        alu = alu_roofline(name, form + suffix, r["launch_s"])
        if nl == 1 and alu is not None:
            # the whole step moves 32 B per update: VALU issue is its bound
            roof = dict(bound="alu", **{k: v for k, v in alu.items()}, hbm=hbm)
        else:
            roof = dict(hbm, alu=alu)
        roof.update({"kernel": kernel_name(w, nl, form), "launches_per_step": nl, "path": PATHS[nl],
                     "avg_launch_us": r["launch_s"] * 1e6, "launch_us_eager": r["stage_us"]})
        forms[form] = {
            "value": r["updates"], "ms_per_step": r["wall"] * 1e3 / steps, "modelled_gbps": r["gbps_model"],
            "bytes_per_update": r["info"]["bytes_per_step"] / (cells * 4.0),
            "roofline": roof,
            "seg_rows": r["seg"],
            "waves_per_workgroup": r["info"]["waves_per_workgroup"],
        }
    return {
        "config": {"workload": name, "nz": w["nz"], "nv": w["nv"], "L": w["L"], "cfl": w["cfl"],
                   "scheme": "FD+KO" if w["scheme"] == 0 else "FV+WENO7", "alpha": w["alpha"],
                   "omega": w["omega"], "lambda": w["lam"], "steps": steps},
        "forms": forms,
        "fp32_speedup_over_fp64": res["fp32acc"]["updates"] / res["fp64"]["updates"],
        "fp32_vs_fp64_after_run": dict(form_difference(res["fp32acc"]["state"], res["fp64"]["state"]),
                                       compared="whole state" if cells <= SLAB_CELLS else
                                       f"3 slabs of {SLAB_ROWS} rows (centre, periodic seam, random)"),
        "tracked": {"fp32acc": res["fp32acc"]["tracked"], "fp64": res["fp64"]["tracked"],
                    "drift_ratio_fp32_over_fp64": res["fp32acc"]["tracked"]["max_rel_drift"] /
                    max(res["fp64"]["tracked"]["max_rel_drift"], 1e-300)},
        "_res": res,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS) + ["batch_64"])
    ap.add_argument("--seg-rows", type=int, default=None, help="fixed launch shape (default: autotune)")
    ap.add_argument("--stage-steps", type=int, default=3, help="steps timed launch by launch (eager, per-stage breakdown)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the secondary workloads (WENO7 65536x256 and the 64-instance batch)")
    ap.add_argument("--secondary-steps", type=int, default=200, help="timed steps of the secondary workloads")
    ap.add_argument("--no-fusion", action="store_true", help="four single-stage launches per step")
    ap.add_argument("--fusion", type=int, default=1, choices=(0, 1, 2),
                    help="0 single stages, 1 fused (the autotuner picks the path), 2 the whole step in one launch "
                         "where supported (with --seg-rows, which skips the autotuner)")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for the CPU baseline")
    ap.add_argument("--cpu-budget-per-config", type=float, default=3.0,
                    help="seconds of oracle work per configuration for cpu_baseline.per_config (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB between device buffers six times (the reference for the HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU only; multi-GPU (z-sharded) execution is not implemented",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2203_12866_amd import cosenu

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        a = torch.ones(1 << 28, device="cuda")
        b = torch.empty_like(a)
        for _ in range(6):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"copied {a.numel() * a.element_size()} bytes x 6", file=sys.stderr)
        return
    if args.workload == "batch_64":
        return batch_main(args, cosenu, torch)
    ceiling = copy_ceiling(torch)
    print(f"[bench] copy ceiling {ceiling['gbps']:.0f} GB/s", file=sys.stderr, flush=True)
    fusion = 0 if args.no_fusion else args.fusion
    main_run = run_workload(cosenu, torch, args.workload, args.steps, args.warmup, args.seg_rows, args.stage_steps,
                            fusion)
    res = main_run.pop("_res")
    head = res["fp32acc"]
    hf = main_run["forms"]["fp32acc"]
    w = WORKLOADS[args.workload](1)
    roof = dict(hf["roofline"])
    roof["stream_ceiling"] = ceiling["gbps"]
    roof["frac_of_stream_ceiling"] = roof["achieved"] / ceiling["gbps"]
    out = {
        "metric": METRIC,
        "value": head["updates"],
        "unit": "cell·v·stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["wall"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64acc",
        "data": "synthetic",
        "config": dict(main_run["config"], form="FP32 stencils, FP64 moments/commutator/RK4", seg_rows=head["seg"],
                       waves_per_workgroup=hf["waves_per_workgroup"]),
        "modelled_gbps": hf["modelled_gbps"],
        "bytes_per_update": hf["bytes_per_update"],
        "roofline": roof,
        "copy_ceiling": ceiling,
        "fp64_form": main_run["forms"]["fp64"],
        "fp32_speedup_over_fp64": main_run["fp32_speedup_over_fp64"],
        "fp32_vs_fp64_after_run": main_run["fp32_vs_fp64_after_run"],
        "tracked": main_run["tracked"],
    }
    if res["fp32acc"]["launches"] < 4:  # the same form on four single-stage launches, for comparison
        single = run_form(cosenu, torch, WORKLOADS[args.workload](1), args.steps, args.warmup, args.seg_rows,
                          args.stage_steps, fused=False)
        print(f"[bench] {args.workload} fp32acc single stages: {single['updates']:.4e} upd/s", file=sys.stderr,
              flush=True)
        out["fp32acc_single_stages"] = {
            "value": single["updates"], "ms_per_step": single["wall"] * 1e3 / args.steps,
            "bytes_per_update": single["info"]["bytes_per_step"] / (w["nz"] * w["nv"] * 4.0),
            "roofline_achieved_gbps": single["achieved_gbps"], "seg_rows": single["seg"],
            "bitwise_equal_to_fused": bool(np.array_equal(single["state"], head["state"])),
        }
    del res, head
    if not args.no_secondary and args.workload == DEFAULT_WORKLOAD:
        sec = {}
        for name in ("fv_weno7_65536x256", "fd_ko_16384x128"):
            r3 = run_workload(cosenu, torch, name, args.secondary_steps, args.warmup, None, args.stage_steps, True)
            r3.pop("_res")
            sec[name] = r3
        from paper_2203_12866_amd import workloads as wl
        insts = wl.batch_64(4)
        rb = run_batch(cosenu, torch, insts, args.secondary_steps, args.warmup)
        print(f"[bench] batch_64 fp32acc: {rb['updates']:.4e} upd/s", file=sys.stderr, flush=True)
        sec["batch_64"] = batch_summary(rb, insts, args.secondary_steps)
        out["secondary"] = sec
    if not args.no_cpu_baseline:
        cb, errs = cpu_baseline(cosenu, WORKLOADS[args.workload](0), args.cpu_budget)
        if args.cpu_budget_per_config > 0 and args.workload == DEFAULT_WORKLOAD:
            cb["per_config"] = cpu_baseline_per_config(args.cpu_budget_per_config)
        out["cpu_baseline"] = cb
        if errs is not None:
            out["error_vs_oracle"] = errs
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
