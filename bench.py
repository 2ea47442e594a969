"""Benchmark of the M1 radiation step on one MI355X.

Headline: cell updates/s of one step (m1_step_explicit + m1_step_implicit)
on the spherical 192x96x192 workload with FP32 transport, the FP64
implicit solve and the GPU-trained MLP opacity surrogate; the plain FP64
form and the other forms are timed beside it.  Inputs are synthetic and
resident in device memory before timing starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--only | --form NAME]

Prints one JSON line.  --only times the headline form alone, --form NAME
one of the other forms alone (both used under rocprofv3).  --gpus N > 1 is
refused: the implementation runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Vector-ALU issue peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes per clock at
# 2.4 GHz, one FP32 or FP64 lane operation each (the published 157.3 TFLOP/s
# FP32 figure counts packed FMAs, 78.6 TFLOP/s FP64 counts FMAs: both are this
# rate times 4 and 2).  Transcendental instructions issue at half this rate.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def algorithmic_valu_ops(kernel, opacity_kind, geom="spherical"):
    """Vector-ALU lane operations per cell the method needs in the FP32
    transport / FP64 implicit / bfloat16-MFMA network form (hand count of the
    formulation; a transcendental counts 2 because it issues at half rate).

    transport, per cell: 3 faces x 164 (two face states 8, two f-fixes 40,
      two closures 84, limited speeds + HLL 32) + 3 directions x 4 fields x 11
      (van Leer slopes) + update 72 (divergence 24, spherical sources with the
      centre closure 41, fix-ups 7) = 696.
    implicit with the network: 128 tanh x 6 (exp2, reciprocal, add, fma) +
      64 second-layer bias + 128 output-layer FMAs + 192 (bfloat16 hi/lo split
      of the 64 first-layer activations) + 18 (network inputs and outputs) +
      80 (FP64 solve: temperature, four divisions, Cramer, damping, gas
      update) = 1250.  The 64x64 layer and the first layer run on the matrix
      cores and are not counted here."""
    if kernel == "transport":
        return 3 * 164 + 12 * 11 + (72 if geom != "cartesian" else 31)
    if opacity_kind == "mlp":
        return 128 * 6 + 64 + 128 + 192 + 18 + 80
    return 80


def algorithmic_bytes(kernel, precision, opacity_kind):
    """Bytes each kernel must move per cell: every field read once and
    written once (ghost re-reads excluded), gas in FP64, radiation and the
    opacity cache in the form's precision."""
    s = 4 if precision == "f32" else 8
    if kernel == "transport":
        return 4 * s + s + 4 * s                 # E,F in; tau in; E*,F* out
    cache = 0 if opacity_kind == "const" else 4 * s   # rho kP, tau in and out
    return 4 * s + 40 + 4 * s + 32 + cache      # E*,F* in; rho,m,Eg in; E,F out; m,Eg out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    # the GPU clock ramps up over the first 100-150 steps of sustained
    # stepping (ms/step falls by 10-30 %); the default warm-up covers it
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--only", action="store_true", help="time the headline form only")
    ap.add_argument("--form", default=None, help="time one named form alone and print its figures")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--train-steps", type=int, default=None, help="override the Adam step count")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def train_surrogate(m1, I, torch, solver, steps):
    ntr, nev = 1_000_000, 100_000
    import numpy as np
    smp = np.concatenate([I.mlp_samples(ntr, 4), I.mlp_samples(nev, 5)])
    dsmp = torch.from_numpy(smp).to("cuda")
    cfg = dict(I.MLP_TRAIN)
    if steps:
        cfg["steps"] = steps
    rep = m1.m1_mlp_train(solver.ctx, dsmp, ntr, nev, I.mlp_init(7), **cfg)
    return rep


def time_form(m1, torch, prob, precision, K, W, mlp_train_steps=0, I=None, rk2=False):
    """Returns dict with cells/s and per-kernel average durations (rk2: the
    second-order step, timed as a whole; its per-kernel fields are those of
    the split step on the same state)."""
    mlp = None
    if prob.opacity["kind"] == 3:
        # construct with the table, then train the surrogate in place
        tab_prob = prob
        tab_prob.opacity = dict(prob.opacity, kind=2)
        s = m1.Solver(tab_prob, precision=precision)
        rep = train_surrogate(m1, I, torch, s, mlp_train_steps)
        tab_prob.opacity["kind"] = 3
        log(f"  surrogate trained: {rep}")
        mlp = rep
    else:
        s = m1.Solver(prob, precision=precision, second_order=rk2)
    dt = prob.dt
    stream = s.stream
    for _ in range(W):
        s.step(dt, rk2=rk2)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t0 = time.perf_counter()
    for _ in range(K):
        if rk2:
            m1.m1_step_rk2(s.ctx, dt)
        else:
            m1.m1_step_explicit(s.ctx, dt)
            m1.m1_step_implicit(s.ctx, dt)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    # per-kernel durations: events around each launch on the launch stream
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
    for k in range(K):
        ev[k][0].record(stream)
        m1.m1_step_explicit(s.ctx, dt)
        ev[k][1].record(stream)
        m1.m1_step_implicit(s.ctx, dt)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    t_tr = sum(ev[k][0].elapsed_time(ev[k][1]) for k in range(K)) / K
    t_im = sum(ev[k][1].elapsed_time(ev[k][2]) for k in range(K)) / K
    d = s.diagnostics()
    s.close()
    n = prob.ncells
    return dict(cells_per_s=n * K / (ms * 1e-3), ms_per_step=ms / K, wall_s=wall,
                transport_ms=t_tr, implicit_ms=t_im, counters=d["counters"], mlp=mlp)


def fp32_deviation(m1, torch, prob, steps=100):
    """Per-field deviation of the FP32 form from the FP64 form after the
    same number of steps from the same input (field_errors)."""
    st = {}
    for prec in ("p64", "f32"):
        s = m1.Solver(prob, precision=prec)
        s.step(prob.dt, steps)
        s.sync()
        st[prec] = {k: v.detach().to(torch.float64).clone() for k, v in s.t.items() if k != "rho"}
        s.close()
    return field_errors(st["f32"], st["p64"])


def field_errors(a, b):
    """Per field of state a against state b: [sum |a - b| / sum |b|,
    max |a - b| / max |b|] (fields of b that are zero everywhere: absolute)."""
    out = {}
    for k, ref in b.items():
        d = (a[k] - ref).abs()
        l1, mx = float(ref.abs().sum()), float(ref.abs().max())
        out[k] = [float(d.sum()) / (l1 if l1 > 0 else 1.0), float(d.max()) / (mx if mx > 0 else 1.0)]
    return out


def copy_bandwidth(torch, n=1 << 28, reps=10):
    """Device-to-device copy rate (bytes read + written per second, GB/s) of
    a 1 GiB FP32 array on this GPU, timed with events."""
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 8.0 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def source_hash(kernel):
    """sha256 of the translation unit a kernel is built from (and its headers)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2606_26268_amd", "csrc")
    files = {"transport": ["transport.hip", "m1_device.h"],
             "implicit": ["implicit.hip", "opacity_device.h", "mlp_device.h"]}[kernel]
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed counter runs (profiles/
    traffic.json), or None if absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(f"{kernel}:{workload}")
    if not rec or rec.get("source") != source_hash(kernel):
        return None
    return rec["bytes_per_launch"]


def copy_calibration():
    import torch
    n = 1 << 28                       # 2^28 float32 = 1 GiB read + 1 GiB written
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))


def oracle_baseline(I, seconds_target=15.0, threads=None, shape=(96, 48, 96)):
    """The FP64 oracle on a bounded sample of the headline workload: the
    same spherical recipe with the MLP surrogate on a reduced grid, with all
    host threads (threads=None) or the given number."""
    import numpy as np
    from oracle import oracle as orc
    if threads is not None:
        orc.set_threads(threads)
    p = I.make_c4(nr=shape[0], nth=shape[1], nph=shape[2])
    tab = p.opacity
    a = tab["log10_kP"].astype(np.float64)
    b = tab["log10_kR"].astype(np.float64)
    norm = np.array([a.mean(), a.std(), b.mean(), b.std()])
    o = orc.Oracle(p, dict(theta=I.mlp_init(7).astype(np.float64), norm=norm, bf16=True))
    st = p.fields
    steps, t = 0, 0.0
    while t < seconds_target and steps < 20:
        t0 = time.perf_counter()
        st, _ = o.run(st, p.dt, 1)
        t += time.perf_counter() - t0
        steps += 1
    cores = orc.max_threads()
    shp = "x".join(str(v) for v in shape)
    return dict(value=p.ncells * steps / t, unit="cell updates/s", cores=cores, kind="oracle",
                sample=f"spherical recipe with MLP opacity on {shp} cells, {steps} steps, {t:.1f} s")


def form_table(I):
    """The forms timed beside the headline: name -> (problem maker,
    precision, second-order step)."""
    def mg8():
        return I.make_multigroup(8, (128, 128, 128))

    def general():
        # the general transport kernel: Lax-Friedrichs flux with the simple
        # clip, reflective walls in x and irradiation heating
        pg = I.make_c1()
        pg.recon, pg.riemann = 2, 1
        pg.bc = [[I.REFLECT, I.REFLECT], [I.PERIODIC, I.PERIODIC], [I.PERIODIC, I.PERIODIC]]
        pg.irr = pg.fields["rho"] * 0.1
        return pg

    return {"c3_f32_table": (I.make_c3, "f32", False), "c3_p64_table": (I.make_c3, "p64", False),
            "c1_p64_const": (I.make_c1, "p64", False), "c1_f32_const": (I.make_c1, "f32", False),
            "c2_p64_const": (I.make_c2, "p64", False), "c2_f32_const": (I.make_c2, "f32", False),
            "c1_mg8_f32": (mg8, "f32", False), "c1_mg8_p64": (mg8, "p64", False),
            # the second-order step (two split steps and the average)
            "c3_f32_table_rk2": (I.make_c3, "f32", True), "c1_mg8_f32_rk2": (mg8, "f32", True),
            "c1_f32_general": (general, "f32", False),
            # the optically thin pulse the scheme's performance section times
            # (256^3, scattering only, second-order steps)
            "p0_pulse_f32_rk2": (I.make_pulse3d, "f32", True), "p0_pulse_p64_rk2": (I.make_pulse3d, "p64", True)}


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_2606_26268_amd import inputs as I
    from paper_2606_26268_amd import m1
    K, W = args.steps, args.warmup

    table = form_table(I)
    if args.form:
        # one named form alone (for profiling); prints its own figures
        if args.form not in table:
            print(json.dumps({"error": f"unknown form {args.form}", "forms": sorted(table)}))
            sys.exit(2)
        mk, prec, rk2 = table[args.form]
        r = time_form(m1, torch, mk(), prec, K, W, rk2=rk2)
        print(json.dumps({"form": args.form, "cells_per_s": r["cells_per_s"], "ms_per_step": r["ms_per_step"],
                          "transport_ms": r["transport_ms"], "implicit_ms": r["implicit_ms"]}))
        return

    log("headline: spherical 192x96x192, f32 transport + f64 implicit + MLP opacity")
    head = time_form(m1, torch, I.make_c4(), "f32", K, W, args.train_steps, I)
    forms = {"c4_f32_mlp": head}
    if not args.only:
        for name, (mk, prec, rk2) in table.items():
            log(f"form {name}")
            forms[name] = time_form(m1, torch, mk(), prec, K, W, rk2=rk2)
        # accuracy of the FP32 forms: 100 steps against the FP64 form
        for name in ("c3_f32_table", "c1_f32_const", "c2_f32_const", "c1_mg8_f32"):
            log(f"fp32 deviation {name}")
            forms[name]["vs_p64"] = fp32_deviation(m1, torch, table[name][0]())

    ncell = 192 * 96 * 192
    # HBM fractions are also given against what a plain copy reaches here
    copy_gbs = copy_bandwidth(torch)
    # both kernels of the headline form are bound by vector-ALU issue (the
    # counter runs under profiles/ show it); the roofline is that of the
    # longer one, with its HBM figures alongside
    kern = "transport" if head["transport_ms"] >= head["implicit_ms"] else "implicit"
    per_kernel = {}
    for kn in ("transport", "implicit"):
        kms = head["transport_ms"] if kn == "transport" else head["implicit_ms"]
        ops = algorithmic_valu_ops(kn, "mlp") * ncell
        byts = algorithmic_bytes(kn, "f32", "mlp") * ncell
        per_kernel[kn] = dict(ms_per_launch=kms, algorithmic_ops_per_launch=ops,
                              tops=ops / (kms * 1e-3) / 1e12, algorithmic_bytes_per_launch=byts,
                              hbm_gbs=byts / (kms * 1e-3) / 1e9, traffic=measured_traffic(kn, "c4_f32_mlp"))
    k = per_kernel[kern]
    roofline = dict(bound="alu", achieved=round(k["tops"], 2), peak=round(VALU_PEAK_TOPS, 2), unit="TOP/s",
                    frac=round(k["tops"] / VALU_PEAK_TOPS, 4), traffic=k["traffic"], kernel=kern,
                    ms_per_launch=k["ms_per_launch"], algorithmic_ops_per_launch=k["algorithmic_ops_per_launch"],
                    hbm_achieved_gbs=round(k["hbm_gbs"], 1), hbm_frac=round(k["hbm_gbs"] / HBM_PEAK_GBS, 4),
                    hbm_copy_gbs=round(copy_gbs, 1), hbm_frac_of_copy=round(k["hbm_gbs"] / copy_gbs, 4),
                    kernels=per_kernel)

    out_forms = {}
    for name, r in forms.items():
        prec = "f32" if "f32" in name else "p64"
        kind = "const" if ("const" in name or "mg" in name or "general" in name) else "table"
        bps = algorithmic_bytes("transport", prec, kind) + algorithmic_bytes("implicit", prec, kind)
        if "general" in name:
            bps += 8                      # the irradiation heating array
        if "_mg8_" in name:
            # per group: transport (E, F, tau in; E*, F* out) and E*, F* in / E, F out; gas once
            s = 4 if prec == "f32" else 8
            bps = 8 * (9 * s + 8 * s) + 72
        if name.endswith("_rk2"):
            bps *= 2                      # two split steps per second-order step
        out_forms[name] = dict(cells_per_s=r["cells_per_s"], ms_per_step=r["ms_per_step"],
                               transport_ms=r["transport_ms"], implicit_ms=r["implicit_ms"],
                               bytes_per_cell_step=bps,
                               hbm_frac=r["cells_per_s"] * bps / (HBM_PEAK_GBS * 1e9),
                               hbm_frac_of_copy=r["cells_per_s"] * bps / (copy_gbs * 1e9),
                               fixups=r["counters"][:3])
        if "vs_p64" in r:
            out_forms[name]["vs_p64"] = {k: [float("%.3g" % v[0]), float("%.3g" % v[1])] for k, v in r["vs_p64"].items()}
    cpu = None
    if not args.no_cpu:
        cpu = oracle_baseline(I)
        if not args.only:
            one = oracle_baseline(I, seconds_target=8.0, threads=1, shape=(48, 24, 48))
            cpu["one_thread"] = dict(value=one["value"], sample=one["sample"])
    line = {
        "metric": "M1 cell updates/s (explicit+implicit), FP32/MLP form vs FP64 plain, 1 MI355X",
        "value": head["cells_per_s"],
        "unit": "cell updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 transport / f64 implicit / bf16-mfma mlp",
        "data": "synthetic",
        "config": {"workload": "spherical 192x96x192 log-r grid, perturbed r^-2 density, r^-1/2 T, "
                               "FP32 transport + FP64 implicit + MLP opacity (100-step run)",
                   "cells": ncell},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": out_forms,
        "mlp_training": head["mlp"],
        "context": {"paper_rmhd_cell_updates_per_s_per_mi250x_node": 7.6e8},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
