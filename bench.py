#!/usr/bin/env python3
"""Throughput of the Abelian-Higgs leapfrog on one MI355X.

Workload: a 512^3 periodic lattice in the matter era (a ~ tau^2), s = 0,
lambda0 = 2, e0 = 1, sigma = 1, dx = 0.5, dt = 0.1, seeded random-phase
initial state, string length and <v^2> measured every 20 steps (the
configuration the paper times at 512^3, Sec. 3 and Table 2).  A bench step is
one leapfrog step of the whole lattice (Eqs. (4)-(7)), with the diagnostics
of Eqs. (9)-(11) on the steps the cadence selects.

Prints ONE JSON line: FP32 storage and arithmetic (FP64 bookkeeping and
reductions) is the headline ``value``, in the 20-plane layout where unmeasured
steps go in pairs through the two-steps-per-pass kernel (``--layout 15``: one
step per pass).  The other layout, the FP64 kernels and the plain FP64 kernel
are reported beside it.  A plain device-to-device copy runs first: its rate is the
reference bandwidth of the line, and its half second of work brings the GPU to its working
clock before any form is timed.  ``roofline`` is for the dominant kernel (the step
kernel): its mean launch time is taken inside the timed region, from HIP events
on the library's stream around the passes that measured nothing (one launch of
it each, after a few-microsecond bookkeeping kernel); ``cpu_baseline`` times the
FP64 CPU oracle on a bounded sample of the same workload on this host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E peak, GB/s
N = 512
MEASURE_EVERY = 20
BYTES_PER_SITE = {"f32": 80, "f64": 160}   # read + write of the 10-field state once


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=N, help="lattice extent (default 512)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-secondary", action="store_true", help="FP32 headline only")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched ensemble")
    ap.add_argument("--kernel", default="auto", choices=["auto", "plain", "tiled", "tiled2"])
    ap.add_argument("--layout", type=int, default=20, choices=[15, 20],
                    help="field planes: 20 lets unmeasured steps go two per pass (default)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy (reference for the "
                         "HBM byte counters of a profiler run)")
    return ap.parse_args()


def run_form(AH, torch, n, prec, kernel, steps, warmup, layout=15, s=0.0):
    """Time `steps` steps with the measurement cadence after `warmup` steps (one more,
    untimed, when that leaves an odd step index and passes go in pairs), then the same
    number of steps without diagnostics.  Both timed regions are
    one library call per pass (one step, or a pair with the two-step kernel),
    each bracketed by events on the library's stream, so the dominant kernel's
    duration is read inside the timed region from the calls that measured
    nothing (each one launch of it after a few-microsecond bookkeeping kernel).
    Returns a dict."""
    # tau_end = n dx / 2, half a light-crossing time (Sec. 2), with a(tau_end) = 1
    p = AH.Params(n, n, n, precision=prec, dx=0.5, dt=0.1, tau0=0.0, tau_ref=n * 0.5 / 2.0,
                  era_p=2.0, s=s, seed=2024,
                  layout=AH.AH_LAYOUT_20 if layout == 20 else AH.AH_LAYOUT_15)
    # the library's choice: pairs through the two-step kernel in the 20-plane layout
    two = layout == 20 and kernel in (AH.AH_KERNEL_TILED2, AH.AH_KERNEL_AUTO)
    per = 2 if two else 1
    planes = AH.alloc_planes(p)
    ctx = AH.Context([p], [planes])
    if kernel != AH.AH_KERNEL_AUTO:
        ctx.set_kernel(kernel)
    stream = ctx.stream
    # the warmup steps take the measurement cadence too, so that every path the timed
    # region takes (the measuring kernels, the observations' return) has run once
    ctx.step(warmup, measure_every=MEASURE_EVERY)
    # with pairs, the timed region starts on an even step (one more untimed step when
    # the warmup count is odd), so that it takes the same passes as the steady state
    # of a long run: pairs, and at each measured state the read-only pass
    extra = ctx.current_step() % per
    if extra:
        ctx.step(extra)
    torch.cuda.synchronize()

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def timed_passes(measure):
        calls, obs = [], []
        t0, t1 = ev(), ev()
        torch.cuda.synchronize()
        t0.record(stream)
        done = 0
        while done < steps:
            # pairs from even step counts, so the calls follow the schedule one
            # call of all the steps would take
            k = min(per - ctx.current_step() % per, steps - done)
            a, b = ev(), ev()
            a.record(stream)
            o = ctx.step(k, measure_every=MEASURE_EVERY) if measure else ctx.step(k)
            b.record(stream)
            calls.append((a, b, k == per and not o))
            obs += o or []
            done += k
        t1.record(stream)
        torch.cuda.synchronize()
        plain = sorted(a.elapsed_time(b) for a, b, one in calls if one)
        if not plain:
            raise SystemExit("bench.py: no unmeasured %d-step call to time the kernel by; "
                             "give more --steps" % per)
        return t0.elapsed_time(t1), plain, obs

    # whole-job throughput with the measurement cadence (the reported value)
    ms, kt, obs = timed_passes(True)
    # and without diagnostics (from a step index of the same parity)
    ms_nd, _, _ = timed_passes(False)
    last = obs[-1][0] if obs else None
    ctx.close()
    del planes
    torch.cuda.empty_cache()
    return {"rate": n ** 3 * steps / (ms * 1e-3), "ms_per_step": ms / steps,
            "warmup_steps": warmup + extra,
            "rate_no_diag": n ** 3 * steps / (ms_nd * 1e-3), "kernel_ms": sum(kt) / len(kt),
            "kernel_ms_median": kt[len(kt) // 2], "launches_timed": len(kt), "per": per,
            "last": last}


def run_slab(AH, torch, passes=30, nxy=1024, nz=128):
    """One GPU's share of a z-decomposed 1024^3 lattice over 8 GPUs: an nxy x nxy x nz
    FP32 slab with two halo planes a side (20-plane layout, two steps per pass).  The
    halo of the current copy is refilled before every pass from the slab's own opposite
    faces by device copies, standing in for the exchange with the z neighbours."""
    H = 2
    p = AH.Params(nxy, nxy, nz, precision=AH.AH_FP32, dx=0.5, dt=0.1, tau0=1.0,
                  tau_ref=nxy * 0.25, era_p=2.0, s=0.0, init=AH.AH_INIT_VACUUM,
                  layout=AH.AH_LAYOUT_20, z_halo=H)
    planes = AH.alloc_planes(p)
    ctx = AH.Context([p], [planes])
    stream = torch.cuda.current_stream()

    def refill():
        c0 = ctx.current_planes(0)[0]         # the ten fields of a copy are contiguous
        cur = planes[c0:c0 + 10]
        cur[:, :H] = cur[:, nz:nz + H]
        cur[:, H + nz:] = cur[:, H:2 * H]

    # a non-trivial state: random phases on the slab
    g = torch.Generator(device="cuda").manual_seed(7)
    th = torch.rand((nz, nxy, nxy), generator=g, device="cuda") * (2 * math.pi) - math.pi
    planes[0, H:H + nz] = torch.cos(th)
    planes[1, H:H + nz] = torch.sin(th)
    del th
    refill()
    for _ in range(3):
        ctx.step(2)
        refill()
    torch.cuda.synchronize()
    # one pass and one refill at a time, each bracketed by events, inside the timed region
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    marks = []
    ev[0].record(stream)
    for _ in range(passes):
        a, b, c = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        a.record(stream)
        ctx.step(2)
        b.record(stream)
        refill()
        c.record(stream)
        marks.append((a, b, c))
    ev[1].record(stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1])
    kt = [a.elapsed_time(b) for a, b, _ in marks]
    ct = [b.elapsed_time(c) for _, b, c in marks]
    ctx.close()
    del planes
    torch.cuda.empty_cache()
    sites = nxy * nxy * nz
    plane_bytes = nxy * nxy * 4
    # per pass and face: phi, A on two planes, Pi, E on one (15 plane-values)
    face_bytes = 15 * plane_bytes
    return {"workload": f"{nxy}x{nxy}x{nz} FP32 z-slab (one GPU's share of a {nxy}^3 lattice "
                        f"over {nxy // nz} GPUs), {H} halo planes a side refilled by device "
                        "copies from its own faces before every two-step pass",
            "value": sites * 2 * passes / (ms * 1e-3), "unit": "site-updates/s",
            "ms_per_pass": ms / passes, "kernel_ms": sum(kt) / len(kt),
            "halo_refill_ms": sum(ct) / len(ct),
            "kernel_frac_algorithmic": BYTES_PER_SITE["f32"] * sites * 2
            / (sum(kt) / len(kt) * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "exchange_bytes_per_face_per_pass": face_bytes,
            "exchange_ms_at_153GBs_per_link": face_bytes / 153e9 * 1e3}


# HBM bytes per launch of the dominant kernel from the profiler's byte counters
# (FETCH_SIZE x 2 + WRITE_SIZE x 1, factors from a 1 GiB device copy measured
# in the same runs), for the kernel as it was profiled; the summaries and
# commands are in profiles/.  Keyed by (dtype, layout, kernel option, lattice);
# each figure carries a digest of the kernel's sources and build options when
# the counters were taken, and is reported only while they are unchanged.
PROFILED_TRAFFIC_BYTES = {
    # k_step_tiled2<float, 9, true>, profiles/step_tiled2_512cubed.md:
    # (3311112 KiB x 2 + 5242880 KiB) per launch
    ("f32", 20, "auto", 512): (12.150e9, "facda5f1456b18e4"),
}
# sources of the FP32 two-step kernel's translation unit; its compile options are
# hashed with them
KERNEL_UNIT = "k_step_tiled2_f32.hip"
KERNEL_SOURCES = ("paper_1809_00995_amd/csrc/k_step_tiled2_f32.hip",
                  "paper_1809_00995_amd/csrc/k_step_tiled2.hpp",
                  "paper_1809_00995_amd/csrc/k_step_tiled2_api.hpp",
                  "paper_1809_00995_amd/csrc/k_step_tiled.hpp",
                  "paper_1809_00995_amd/csrc/ah_device.hpp",
                  "include/ah.h")


def _code_only(text):
    """C/C++ source without its comments and with whitespace collapsed, so that the
    digest follows the code, not its prose (the sources hold no string literal with
    comment delimiters in it)."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_digest():
    import hashlib
    from paper_1809_00995_amd import build
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    h.update(" ".join(build.unit_options(KERNEL_UNIT)).encode())
    return h.hexdigest()[:16]


def profiled_traffic(dt, layout, kernel, n):
    """(bytes per launch, note): None when no counters were taken for this form or
    the kernel's sources changed since."""
    v = PROFILED_TRAFFIC_BYTES.get((dt, layout, kernel, n))
    if v is None:
        return None, "no counter run for this form"
    nbytes, digest = v
    if digest != kernel_digest():
        return None, "kernel sources changed since the counters were taken"
    return nbytes, "profiles/step_tiled2_512cubed.md"


def ensemble_params(AH, layout=20):
    """48 x 128^3 + 16 x 64^3 + 4 x 256^3, FP32; realization r: radiation s=1 if r is even,
    matter s=0 if odd; seed 1000 + r; each runs to its own tau_end = N dx / 2 (n_end)."""
    lay = AH.AH_LAYOUT_20 if layout == 20 else AH.AH_LAYOUT_15
    ps = []
    for n, count in ((256, 4), (128, 48), (64, 16)):
        for _ in range(count):
            r = len(ps)
            rad = r % 2 == 0
            tau_end = n * 0.5 / 2.0
            ps.append(AH.Params(n, n, n, precision=AH.AH_FP32, dx=0.5, dt=0.1, tau0=0.0,
                                tau_ref=tau_end, era_p=1.0 if rad else 2.0, s=1.0 if rad else 0.0,
                                seed=1000 + r, n_end=int(round(tau_end / 0.1)), layout=lay))
    return ps


def run_ensemble(AH, torch, batched, graph_steps, tune, layout=20):
    """The whole ensemble to completion (640 steps), diagnostics every 20 steps.
    Returns (total site-updates/s, seconds, tuning)."""
    ps = ensemble_params(AH, layout)
    planes = [AH.alloc_planes(p) for p in ps]
    ctx = AH.Context(ps, planes)
    tuning = None
    ctx.set_launch(batched, graph_steps)
    if tune:
        tuning = ctx.autotune()               # for the launch form just set
    # one measured stretch outside the timing: first launches, the batched form's work
    # lists and its step graphs are made on first use
    ctx.step(MEASURE_EVERY, measure_every=MEASURE_EVERY)
    torch.cuda.synchronize()
    total = sum(p.sites * (p.n_end - MEASURE_EVERY) for p in ps)
    stream = torch.cuda.current_stream()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    # the observations are decoded into Python objects after the timed region
    rec = ctx.step(max(p.n_end for p in ps) - MEASURE_EVERY, measure_every=MEASURE_EVERY,
                   decode=False)
    t1.record(stream)
    torch.cuda.synchronize()
    sec = t0.elapsed_time(t1) * 1e-3
    assert len(rec.decode()) == len(rec) > 0
    assert all(ctx.current_step(r) == p.n_end for r, p in enumerate(ps))
    ctx.close()
    del planes
    torch.cuda.empty_cache()
    return total / sec, sec, tuning


def secondary(line, name, fn):
    """line[name] = fn(); a form that fails records its error instead, so that the
    headline line is printed whatever happens to the forms after it."""
    try:
        line[name] = fn()
    except (Exception, SystemExit) as e:      # run_form exits on too few steps
        line[name] = {"error": f"{type(e).__name__}: {e}"}
    v = line[name].get("value")
    print(f"# {name}: " + (f"{v:.4g} site-updates/s" if v is not None else line[name]["error"]),
          file=sys.stderr, flush=True)


def gpu_warmup(AH, torch, n, layout, seconds=0.5):
    """About `seconds` of the workload (steps with the measurement cadence) on a scratch
    n^3 FP32 lattice, untimed, before the first timed form.  Measured on one GPU: after
    the device-copy warm-up alone the first form timed in a process ran 4-7 % below the
    same form timed again (its passes 2-4 % slower); after this warm-up the two agree
    within 0.5 %.  A warm-up of passes alone, without the measurements, left 2 %."""
    p = AH.Params(n, n, n, precision=AH.AH_FP32, tau0=0.0, tau_ref=n * 0.25, era_p=2.0, s=0.0,
                  seed=1, layout=AH.AH_LAYOUT_20 if layout == 20 else AH.AH_LAYOUT_15)
    planes = AH.alloc_planes(p)
    with AH.Context([p], [planes]) as ctx:
        t = time.perf_counter()
        while time.perf_counter() - t < seconds:
            ctx.step(MEASURE_EVERY, measure_every=MEASURE_EVERY)
            torch.cuda.synchronize()
    del planes
    torch.cuda.empty_cache()


def device_copy_rate(torch, reps=200, timed=20):
    """GB/s (read + write) of a plain 1 GiB device-to-device copy on this GPU, the mean of
    the last `timed` of `reps` copies.  Run before the first timed form, the copies also
    bring the GPU to its working clock (about half a second of full-bandwidth work)."""
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps - timed):
        dst.copy_(src)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(timed):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    rate = timed * 2 * src.numel() * 4 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return rate


def oracle_rate(n, k):
    """Site-updates/s of the FP64 oracle (test infrastructure) over k steps of an n^3
    matter-era lattice, and the seconds it took."""
    import oracle as O
    p = O.Params(n, n, n, tau0=1.0, tau_ref=n * 0.5 / 2, era_p=2.0, s=0.0, seed=2024)
    st = O.init_random_phase(p)
    st = O.step(p, 10, st)                     # warm the pages
    t = time.perf_counter()
    for i in range(k):
        st = O.step(p, 11 + i, st)
    dt = time.perf_counter() - t
    return n ** 3 * k / dt, dt


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline():
    """The FP64 oracle on a bounded sample of the benchmark's workload on this host: the
    512^3 lattice for 6 steps (about 13 s) on all the threads OpenMP gives it, and
    128^3 x 6 steps on one thread (a child process with OMP_NUM_THREADS=1, which
    touches no GPU)."""
    import subprocess
    import oracle as O
    n, k = 512, 6
    rate, dt = oracle_rate(n, k)
    out = {"value": rate, "unit": "site-updates/s", "cores": O.threads(), "kind": "oracle",
           "sample": f"FP64 CPU oracle, {n}^3 matter era s=0, {k} steps ({dt:.1f} s)",
           "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    code = ("import json, sys; sys.path.insert(0, %r); import bench; r, dt = bench.oracle_rate(128, 6); "
            "print(json.dumps([r, dt]))" % ROOT)
    try:
        res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                             timeout=120, env={**os.environ, "OMP_NUM_THREADS": "1"})
        r1, dt1 = json.loads(res.stdout.strip().splitlines()[-1])
        out["single_thread"] = {"value": r1, "sample": f"128^3, 6 steps ({dt1:.1f} s)"}
    except (subprocess.SubprocessError, ValueError, IndexError) as e:
        out["single_thread"] = {"value": None, "error": str(e)[:200]}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the exchange between "
              "z-slabs on several GPUs is not built (its 'slab' form times one GPU's share)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1809_00995_amd as AH
    kern = {"auto": AH.AH_KERNEL_AUTO, "plain": AH.AH_KERNEL_PLAIN,
            "tiled": AH.AH_KERNEL_TILED, "tiled2": AH.AH_KERNEL_TILED2}[args.kernel]
    n, K, W = args.n, args.steps, args.warmup
    other = 15 if args.layout == 20 else 20

    copy_gbs = device_copy_rate(torch)
    gpu_warmup(AH, torch, n, args.layout)
    f32 = run_form(AH, torch, n, AH.AH_FP32, kern, K, W, args.layout)
    rate32, ms32, kms32, per32, last32 = (f32["rate"], f32["ms_per_step"], f32["kernel_ms"],
                                          f32["per"], f32["last"])
    print(f"# fp32 {args.kernel} layout {args.layout}: {rate32:.4g} site-updates/s, "
          f"{ms32:.3f} ms/step, step kernel {kms32:.3f} ms per {per32}-step launch",
          file=sys.stderr, flush=True)
    achieved = BYTES_PER_SITE["f32"] * n ** 3 * per32 / (kms32 * 1e-3) / 1e9
    kname = "two-steps-per-pass kernel" if per32 == 2 else "step kernel"
    traffic, traffic_note = profiled_traffic("f32", args.layout, args.kernel, n)
    # the floor of the kernel's own design: one read and one write of the state
    # per launch, whatever the number of steps it advances
    floor_bps = BYTES_PER_SITE["f32"] // per32
    line = {
        "metric": "lattice site-updates/s and % HBM roofline, FP32 vs FP64 kernel, 512^3",
        "value": rate32, "unit": "site-updates/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": ms32, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "warmup_steps_run": f32["warmup_steps"],
        "config": {"workload": f"{n}^3 periodic lattice, matter era a~tau^2, s=0, lambda0=2, "
                               f"e0=1, sigma=1, dx=0.5, dt=0.1, random-phase init, string "
                               f"length and <v^2> every {MEASURE_EVERY} steps",
                   "lattice": [n, n, n], "measure_every": MEASURE_EVERY, "kernel": args.kernel,
                   "layout": args.layout,
                   "precision": "FP32 fields and stencil, FP64 bookkeeping and reductions"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "frac_basis": "algorithmic: 80 B per site-update (the 40 B/site state read "
                                   "and written once per step) x site-updates per launch / "
                                   "launch time; traffic_frac is the measured-bytes fraction, "
                                   "design_floor the kernel's own 40 B floor",
                     "traffic": traffic, "traffic_source": traffic_note,
                     "kernel": kname, "steps_per_launch": per32,
                     "bytes_per_site_update": BYTES_PER_SITE["f32"],
                     "algorithmic_bytes_per_launch": BYTES_PER_SITE["f32"] * n ** 3 * per32,
                     "kernel_ms": kms32,
                     "kernel_ms_median": f32["kernel_ms_median"],
                     "launches_timed": f32["launches_timed"],
                     "design_floor": {
                         "bytes_per_site_update": floor_bps,
                         "note": "one read and one write of the 40 B/site FP32 state per launch "
                                 "of %d step(s); frac above 1 on the per-step roofline means "
                                 "fewer bytes than one pass per step" % per32,
                         "achieved": floor_bps * n ** 3 * per32 / (kms32 * 1e-3) / 1e9,
                         "frac": floor_bps * n ** 3 * per32 / (kms32 * 1e-3) / 1e9
                         / HBM_PEAK_GBS}},
        "without_diagnostics": {"value": f32["rate_no_diag"], "steps": K},
    }
    # the paper's own evolution rate, for context only (another GPU, and its
    # figure excludes the diagnostics): 7.75e-10 GPU-seconds per site-update
    # for the three evolution kernels at 512^3 (Sec. 3, performance comparison)
    line["paper_context"] = {
        "value": 1.0 / 7.75e-10, "unit": "site-updates/s",
        "hardware": "NVIDIA Quadro P5000 (the paper's GPU, Sec. 3), FP32",
        "workload": "512^3, evolution kernels only (no diagnostics)",
        "ratio_of_value_without_diagnostics": f32["rate_no_diag"] * 7.75e-10}
    if traffic is not None:
        # measured HBM bytes per launch (profiler counters) at this run's kernel time
        line["roofline"]["traffic_GBs"] = traffic / (kms32 * 1e-3) / 1e9
        line["roofline"]["traffic_frac"] = line["roofline"]["traffic_GBs"] / HBM_PEAK_GBS
    if last32 is not None:
        line["last_obs"] = {"step": last32.step, "n_wind": last32.n_wind,
                            "xi_w": last32.xi_w, "v2_L": last32.v2[0]}
    def form_entry(prec, kk, lay, dt, s=0.0):
        f = run_form(AH, torch, n, prec, kk, K, W, lay, s=s)
        ach = BYTES_PER_SITE[dt] * n ** 3 * f["per"] / (f["kernel_ms"] * 1e-3) / 1e9
        e = {"value": f["rate"], "ms_per_step": f["ms_per_step"],
             "value_without_diagnostics": f["rate_no_diag"], "kernel_ms": f["kernel_ms"],
             "steps_per_launch": f["per"], "layout": lay, "achieved_algorithmic_GBs": ach,
             "frac_algorithmic": ach / HBM_PEAK_GBS}
        if s:
            e["s"] = s
        return e

    def plain_entry():
        kp = max(10, K // 4)
        fp = run_form(AH, torch, n, AH.AH_FP64, AH.AH_KERNEL_PLAIN, kp, 2)
        return {"value": fp["rate"], "ms_per_step": fp["ms_per_step"],
                "kernel_ms": fp["kernel_ms"], "steps": kp}

    def ensemble_entry():
        rb, sb, tuning = run_ensemble(AH, torch, True, 10, True)
        rs, ss, _ = run_ensemble(AH, torch, False, 0, False)
        r15, s15, _ = run_ensemble(AH, torch, True, 10, True, layout=15)
        return {
            "workload": "48 x 128^3 + 16 x 64^3 + 4 x 256^3 FP32, radiation s=1 / matter s=0 "
                        "alternating, each to tau_end = N dx / 2 (320 / 160 / 640 steps), "
                        f"diagnostics every {MEASURE_EVERY} steps",
            "value": rb, "unit": "site-updates/s", "seconds": sb,
            # the whole-job rate (diagnostics included) in 80 B site-updates
            "value_frac_algorithmic": rb * BYTES_PER_SITE["f32"] / 1e9 / HBM_PEAK_GBS,
            "launch": "20-plane layout, one persistent launch per pass (unmeasured steps two "
                      "per pass), 10-step hipGraphs, autotuned tiles",
            "tile_y": tuning[0] if tuning else None,
            "per_realization_launches": {"value": rs, "seconds": ss},
            "speedup_vs_per_realization": rb / rs,
            "one_step_per_pass": {"value": r15, "seconds": s15, "layout": 15}}

    if not args.no_secondary:
        for name, prec, lay, dt in (("fp32_layout%d" % other, AH.AH_FP32, other, "f32"),
                                    ("fp64", AH.AH_FP64, args.layout, "f64"),
                                    ("fp64_layout%d" % other, AH.AH_FP64, other, "f64")):
            secondary(line, name, lambda: form_entry(prec, kern, lay, dt))
        # the second leg of the 512^3 matter-era workload: s = 1 (true equations of motion)
        secondary(line, "fp32_s1", lambda: form_entry(AH.AH_FP32, kern, args.layout, "f32", s=1.0))
        secondary(line, "plain_fp64", plain_entry)
        if "value" in line["plain_fp64"]:
            line["speedup_fp32_vs_plain_fp64"] = rate32 / line["plain_fp64"]["value"]
            if "value" in line["fp64"]:
                line["speedup_fp64_vs_plain_fp64"] = (line["fp64"]["value"]
                                                      / line["plain_fp64"]["value"])
        secondary(line, "slab", lambda: run_slab(AH, torch))
    if not args.no_secondary and not args.no_ensemble:
        secondary(line, "ensemble", ensemble_entry)
    line["roofline"]["copy_GBs"] = copy_gbs
    if traffic is not None:
        line["roofline"]["traffic_frac_of_copy"] = line["roofline"]["traffic_GBs"] / copy_gbs
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = {"read": src.numel() * 4, "written": dst.numel() * 4}
        del src, dst
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
