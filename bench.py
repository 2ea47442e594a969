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
    ap.add_argument("--oracle-configs", action="store_true",
                    help="only time the CPU oracle on bounded samples of the FP64 workloads (no GPU)")
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


# timed repetitions of the K steps; the median is reported and every
# repetition listed.  After an idle GPU the clock ramps up over the first
# ~100 steps of this workload (20-step repetitions after a 5-step warm-up
# measured 0.310, 0.282, 0.270, 0.264, 0.256 ms/step), so with short
# warm-ups the median of eleven repetitions is the sustained rate
REPS = 11


def time_form(m1, torch, prob, precision, K, W, mlp_train_steps=0, I=None, rk2=False, reps=REPS):
    """Returns dict with cells/s and per-kernel average durations.  The K
    timed steps are repeated `reps` times (HIP events on the launch stream
    around each repetition) and the median repetition is reported (rk2: the
    second-order step, timed as a whole; its per-kernel fields are those of
    the split step on the same state)."""
    mlp = mlp_weights = None
    if prob.opacity["kind"] == 3:
        # construct with the table, then train the surrogate in place
        tab_prob = prob
        tab_prob.opacity = dict(prob.opacity, kind=2)
        s = m1.Solver(tab_prob, precision=precision)
        rep = train_surrogate(m1, I, torch, s, mlp_train_steps)
        tab_prob.opacity["kind"] = 3
        log(f"  surrogate trained: {rep}")
        mlp = rep
        theta, norm = m1.m1_mlp_get(s.ctx)
        mlp_weights = dict(theta=theta, norm=norm)
    else:
        s = m1.Solver(prob, precision=precision, second_order=rk2)
    dt = prob.dt
    stream = s.stream
    for _ in range(W):
        s.step(dt, rk2=rk2)
    torch.cuda.synchronize()
    rep_ms, walls = [], []
    for _ in range(reps):
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
        walls.append(time.perf_counter() - t0)
        rep_ms.append(e0.elapsed_time(e1))
    ms = sorted(rep_ms)[len(rep_ms) // 2]
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
    return dict(cells_per_s=n * K / (ms * 1e-3), ms_per_step=ms / K, wall_s=sum(walls),
                rep_ms_per_step=[round(v / K, 5) for v in rep_ms],
                transport_ms=t_tr, implicit_ms=t_im, counters=d["counters"], mlp=mlp,
                mlp_weights=mlp_weights)


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


def measured_valu(kernel, workload, ms):
    """Vector-issue figures of a kernel from the committed instruction
    counter run (profiles/valu.json: SQ_INSTS_VALU, SQ_INSTS_VALU_TRANS_F32,
    SQ_WAVES per dispatch), or None if absent or taken on a different kernel
    source.  issue_frac: the issue cycles those instructions need (4 per
    wavefront instruction on a 16-lane SIMD, 8 for a transcendental) spread
    over the 1024 SIMDs, against the launch time at the 2.4 GHz peak clock."""
    path = os.path.join(ROOT, "profiles", "valu.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(f"{kernel}:{workload}")
    if not rec or rec.get("source") != source_hash(kernel):
        return None
    per_wave = rec["valu_per_wave"]
    trans = rec["trans_per_wave"]
    cycles = 4.0 * (per_wave + trans) * rec["waves"] / 1024.0
    return dict(valu_per_wave=per_wave, trans_per_wave=trans, waves=rec["waves"],
                issue_frac=round(cycles / (2.4e9 * ms * 1e-3), 4))


def copy_calibration():
    import torch
    n = 1 << 28                       # 2^28 float32 = 1 GiB read + 1 GiB written
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))


def cpu_model():
    """Host CPU model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_baseline(I, weights=None, seconds_target=15.0, threads=None, shape=(96, 48, 96)):
    """The FP64 oracle on a bounded sample of the headline workload: the
    same spherical recipe with the MLP surrogate (the GPU-trained weights
    when given) on a reduced grid, with all host threads (threads=None) or
    the given number."""
    import numpy as np
    from oracle import oracle as orc
    if threads is not None:
        orc.set_threads(threads)
    p = I.make_c4(nr=shape[0], nth=shape[1], nph=shape[2])
    if weights is None:
        tab = p.opacity
        a = tab["log10_kP"].astype(np.float64)
        b = tab["log10_kR"].astype(np.float64)
        weights = dict(theta=I.mlp_init(7), norm=np.array([a.mean(), a.std(), b.mean(), b.std()]))
    o = orc.Oracle(p, dict(theta=np.asarray(weights["theta"], dtype=np.float64), norm=weights["norm"], bf16=True))
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
                cpu_model=cpu_model(),
                sample=f"spherical recipe with the MLP opacity on {shp} cells, {steps} steps, {t:.1f} s")


def oracle_configs(I, seconds_target=8.0):
    """The FP64 oracle on the host cores, on the FP64 workloads at full grid
    size: whole steps, one at a time, until seconds_target has passed or
    the workload's own step count is reached; with all host threads, and
    the 128^3 box also with one thread.  Prints one JSON line."""
    from oracle import oracle as orc
    runs = [("c1 128^3 turbulent box, constant opacity", I.make_c1, None),
            ("c1 128^3 turbulent box, constant opacity", I.make_c1, 1),
            ("c3 spherical 192x96x192, bilinear table", I.make_c3, None),
            ("c2 256^3 turbulent box, constant opacity", I.make_c2, None)]
    allt = orc.max_threads()
    out = {"cpu_model": cpu_model(), "runs": []}
    for label, mk, threads in runs:
        p = mk()
        orc.set_threads(threads if threads else allt)
        o = orc.Oracle(p)
        st, steps, t = p.fields, 0, 0.0
        while t < seconds_target and steps < p.steps:
            t0 = time.perf_counter()
            st, _ = o.run(st, p.dt, 1)
            t += time.perf_counter() - t0
            steps += 1
        out["runs"].append(dict(workload=label, cores=orc.max_threads(), steps=steps, seconds=round(t, 2),
                                cell_updates_per_s=p.ncells * steps / t))
        log(f"  {label}, {orc.max_threads()} threads: {p.ncells * steps / t:.3e} cell updates/s")
    orc.set_threads(allt)
    print(json.dumps(out))


def _log10_opacity(m1, torch, ctx, rho, T):
    """log10 kappa_P, log10 kappa_R of a context's opacity source at host
    (rho, T) points, evaluated on the device."""
    import numpy as np
    r = torch.from_numpy(np.ascontiguousarray(rho, dtype=np.float64)).to("cuda")
    t = torch.from_numpy(np.ascontiguousarray(T, dtype=np.float64)).to("cuda")
    kP, kR = torch.empty_like(r), torch.empty_like(r)
    m1.m1_opacity_eval(ctx, r.numel(), r, t, kP, kR)
    m1.m1_sync(ctx)
    return np.log10(kP.cpu().numpy()), np.log10(kR.cpu().numpy())


def mlp_gain(m1, torch, I, weights, table_sizes=(128, 512, 2048, 4096), K=20, W=20):
    """What the trained network changes against the bilinear table it
    replaces, measured on the device (the table lookup is the reference):

    * model bytes: network parameters (FP32 master), its packed inference
      buffer, and the two 128 x 128 FP32 tables;
    * max |kappa_net / kappa_table - 1| over the held-out samples and over
      the cells of the spherical workload;
    * error of each against the smooth function the table samples;
    * smoothness: the jump of d log10 kappa / d log10 T across the table's
      node lines and, for comparison, across the mid-cell lines (one-sided
      slopes over h/16 next to each line): the bilinear table has a kink at
      every node and none between, the network the same small jump (its
      curvature over the stencil, plus rounding) everywhere;
    * the implicit kernel's time with the table at several node counts (the
      same function sampled finer; the cache footprint grows as nodes^2)."""
    import numpy as np
    tab = I.make_table()
    lr_off, lt_off = tab["lr_off"], tab["lt_off"]
    p = I.make_uniform(I.CARTESIAN, (64, 1, 1), 1)
    p.opacity = tab
    # FP64 contexts: the table is interpolated in FP64 (the network computes
    # in FP32 in any form)
    st = m1.Solver(p, "p64")
    sm = m1.Solver(p, "p64")
    m1.m1_set_opacity_mlp(sm.ctx, weights["theta"], weights["norm"])
    out = {"model_bytes": {"network_parameters_fp32": 4 * m1.M1_MLP_NPARAM,
                           "network_packed_inference_buffer": 4 * 9860,
                           "table_two_128x128_fp32": 2 * 4 * tab["nr"] * tab["nt"]}}

    def compare(rho, T, lr, lt):
        tP, tR = _log10_opacity(m1, torch, st.ctx, rho, T)
        nP, nR = _log10_opacity(m1, torch, sm.ctx, rho, T)
        rec = {"max_rel_err_P": float(np.abs(10.0 ** (nP - tP) - 1).max()),
               "max_rel_err_R": float(np.abs(10.0 ** (nR - tR) - 1).max())}
        if lr is not None:
            gP, gR = I.table_log10_kappa(lr, lt)
            rec["table_vs_function_max_dex"] = [float(np.abs(tP - gP).max()), float(np.abs(tR - gR).max())]
            rec["network_vs_function_max_dex"] = [float(np.abs(nP - gP).max()), float(np.abs(nR - gR).max())]
        return rec

    held = I.mlp_samples(100_000, 5).astype(np.float64)
    lr, lt = held[:, 0], held[:, 1]
    out["held_out"] = compare(10.0 ** (lr - lr_off), 10.0 ** (lt - lt_off), lr, lt)
    c = I.make_c3()
    rho = c.fields["rho"].ravel()
    T = c.fields["Eg"].ravel() * (c.gamma - 1.0) / rho
    out["spherical_cells"] = compare(rho, T, None, None)
    # slopes in log10 T on both sides of every interior node line, and of
    # every mid-cell line for comparison, at five densities (one-sided
    # differences over h/16 at h/16..h/8 from the line)
    h = (tab["lt1"] - tab["lt0"]) / (tab["nt"] - 1)
    dens = np.linspace(tab["lr0"] + 1.0, tab["lr1"] - 1.0, 5)
    d = h / 16.0
    offs = np.array([-2.0, -1.0, 1.0, 2.0]) * d
    jumps = {}
    for name, ctx in (("table", st.ctx), ("network", sm.ctx)):
        rec = {}
        for where, lines in (("nodes", tab["lt0"] + h * np.arange(1, tab["nt"] - 1)),
                             ("mid_cells", tab["lt0"] + h * (np.arange(1, tab["nt"] - 2) + 0.5))):
            LRn, LTn = np.meshgrid(dens, lines, indexing="ij")
            pts_lt = (LTn.ravel()[:, None] + offs[None, :]).ravel()
            pts_lr = np.repeat(LRn.ravel(), 4)
            vals = _log10_opacity(m1, torch, ctx, 10.0 ** (pts_lr - lr_off), 10.0 ** (pts_lt - lt_off))
            for kname, v in zip(("P", "R"), vals):
                v = v.reshape(-1, 4)
                jump = np.abs((v[:, 3] - v[:, 2]) - (v[:, 1] - v[:, 0])) / d
                rec[f"{kname}_{where}_max"] = float(jump.max())
        jumps[name] = rec
    out["slope_jump_across_nodes_dex_per_dex"] = jumps
    st.close()
    sm.close()
    scan = {}
    for n in table_sizes:
        prob = I.make_c3()
        prob.opacity = I.make_table(n, n)
        r = time_form(m1, torch, prob, "f32", K, W, reps=1)
        scan[str(n)] = {"implicit_ms": r["implicit_ms"], "cells_per_s": r["cells_per_s"],
                        "table_bytes": 2 * 4 * n * n}
        log(f"  table {n}x{n}: implicit {r['implicit_ms']:.4f} ms")
    out["table_size_scan"] = scan
    return out


def form_table(I):
    """The forms timed beside the headline: name -> (problem maker,
    precision, second-order step)."""
    def mg8():
        return I.make_multigroup(8, (128, 128, 128))

    def limo3():
        # LimO3 reconstruction (the general kernel's third-order limiter)
        p3 = I.make_c3()
        p3.limiter = 1
        return p3

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
            "c3_f32_limo3": (limo3, "f32", False), "c3_p64_limo3": (limo3, "p64", False),
            # the optically thin pulse the scheme's performance section times
            # (256^3, scattering only, second-order steps)
            "p0_pulse_f32_rk2": (I.make_pulse3d, "f32", True), "p0_pulse_p64_rk2": (I.make_pulse3d, "p64", True)}


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.oracle_configs:
        from paper_2606_26268_amd import inputs as I
        oracle_configs(I)
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
    # roofline of the dominant (longer) kernel of the headline form on the
    # algorithmic-bytes basis: bytes per cell x cells / average launch time,
    # against the 8 TB/s HBM peak; the counter-measured traffic and the
    # vector-issue figures (instruction counters) are given beside it
    kern = "transport" if head["transport_ms"] >= head["implicit_ms"] else "implicit"
    per_kernel = {}
    for kn in ("transport", "implicit"):
        kms = head["transport_ms"] if kn == "transport" else head["implicit_ms"]
        byts = algorithmic_bytes(kn, "f32", "mlp") * ncell
        per_kernel[kn] = dict(ms_per_launch=kms, algorithmic_bytes_per_launch=byts,
                              hbm_gbs=byts / (kms * 1e-3) / 1e9, traffic=measured_traffic(kn, "c4_f32_mlp"),
                              valu=measured_valu(kn, "c4_f32_mlp", kms))
    k = per_kernel[kern]
    roofline = dict(bound="hbm", achieved=round(k["hbm_gbs"], 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(k["hbm_gbs"] / HBM_PEAK_GBS, 4), traffic=k["traffic"], kernel=kern,
                    ms_per_launch=k["ms_per_launch"], algorithmic_bytes_per_launch=k["algorithmic_bytes_per_launch"],
                    bytes_per_cell=algorithmic_bytes(kern, "f32", "mlp"), cells_per_launch=ncell,
                    hbm_copy_gbs=round(copy_gbs, 1), frac_of_copy=round(k["hbm_gbs"] / copy_gbs, 4),
                    valu=k["valu"], kernels=per_kernel)

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
    gain = None
    if not args.only:
        log("network vs table")
        gain = mlp_gain(m1, torch, I, head["mlp_weights"])
        gain["cells_per_s"] = {"network_c4": forms["c4_f32_mlp"]["cells_per_s"],
                               "table_c3": forms["c3_f32_table"]["cells_per_s"]}
        gain["implicit_ms"] = {"network_c4": forms["c4_f32_mlp"]["implicit_ms"],
                               "table_c3": forms["c3_f32_table"]["implicit_ms"]}
    cpu = None
    if not args.no_cpu:
        cpu = oracle_baseline(I, head["mlp_weights"])
        if not args.only:
            one = oracle_baseline(I, head["mlp_weights"], seconds_target=8.0, threads=1, shape=(48, 24, 48))
            cpu["one_thread"] = dict(value=one["value"], sample=one["sample"])
    line = {
        "metric": "M1 cell updates/s (explicit+implicit), FP32/MLP form vs FP64 plain, 1 MI355X",
        "value": head["cells_per_s"],
        "unit": "cell updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": head["ms_per_step"],
        "ms_per_step_repetitions": head["rep_ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 transport / f64 implicit / bf16-mfma mlp",
        "data": "synthetic",
        "config": {"workload": "spherical 192x96x192 log-r grid, perturbed r^-2 density, r^-1/2 T, "
                               "FP32 transport + FP64 implicit + MLP opacity; "
                               f"{K} timed steps after {W} warm-up steps, median of {REPS} repetitions",
                   "cells": ncell, "repetitions": REPS},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": out_forms,
        "mlp_training": head["mlp"],
        "mlp_gain": gain,
        "context": {"paper_rmhd_cell_updates_per_s_per_mi250x_node": 7.6e8},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
