"""Benchmark of the hot path on one MI355X.

Headline workload: the largest configuration, the thin anisotropic
RF-dressed shell in a 2048 x 2048 x 1024 bounding box (h = 0.0306, kappa =
12.9, mask V < 61 -> 59,748,872 active sites, g = 1e4, dt = 5e-5).  One bench
step is one RK4 step of the whole shell in complex128 (FP64 throughout);
`value` counts site updates per second over exactly --steps timed steps,
inputs resident in HBM.  The same steps in complex64 (FP32 stencil, FP64
reductions) and the difference between the two states are reported beside
it, as in the precision study.

Also reported: the RF bubble (1024 x 1024 x 512, 16,028,656 active sites)
in both precisions, one bench step there being one imaginary-time step plus
two RK4 steps (the 5k : 10k ratio of its job), with the job end to end; the
adjoint gradient rate on the 256^3 hollowing ramp (grads/s vs plain FP64
forward runs); the 64-instance batched sweep (hipGraph; forward, and forward
plus adjoint in complex64 against complex128); the integrators, the
real-state imaginary time, the staged ramp, the 19/27-point stencils, the
tiny shell; the full 20,000-step precision study on the downscaled shell
against the oracle's stored run; per-kernel timing (HIP events on the launch
stream) with the roofline of the dominant kernel; and the FP64 CPU oracle
timed on bounded samples of the workloads.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# The CPU baseline is the oracle on one core: BLAS/OpenMP pools are pinned to
# one thread before NumPy/SciPy load (the GPU legs do not use them).
for _v in ("OMP_NUM_THREADS", "MKL_NUM_THREADS", "OPENBLAS_NUM_THREADS", "BLIS_NUM_THREADS",
           "NUMEXPR_NUM_THREADS", "VECLIB_MAXIMUM_THREADS"):
    os.environ[_v] = "1"

import numpy as np  # noqa: E402

METRIC = "active-site GPE updates/s + % HBM roofline; adjoint grads/s vs plain FP64"
HBM_PEAK_GBPS = 8000.0

# algorithmic bytes per active site per launch (each input read once from HBM,
# each output written once), by kernel family; R = bytes of a real, C = 2R
def algo_bytes(fam: str, R: int, scheme: int = 0) -> int:
    C = 2 * R
    if scheme == 1 and fam == "rk_stage2":
        return 2 * C + R + 2 * C         # y2, y0, U -> y3, A
    if scheme == 1 and fam == "rk_stage4":
        return 2 * C + R + C             # y4, A, U -> y0
    table = {
        "itp_pass1": C + R + C,          # psi, P -> tmp
        "itp_pass2": C + R + C,          # tmp, P -> psi
        "rk_stage1": C + R + C,          # y0, U -> y2
        "rk_stage2": 2 * C + R + C,      # y2, y0, U -> y3
        "rk_stage3": 2 * C + R + C,      # y3, y0, U -> y4
        "rk_stage4": 4 * C + R + C,      # y4, y0, y2, y3, U -> y0
        "observe": C + R,
        "adj_stage4": C + C + R + 2 * C,            # lam, Y4, U -> u3, lacc
        "adj_stage3": C + C + R + C + C + 2 * C,    # u3, Y3, U, lam, lacc -> u2, lacc
        "adj_stage2": C + C + R + C + C + 2 * C,
        "adj_stage1": C + C + R + C + C,            # u1, Y1, U, lacc -> lam
    }
    return table.get(fam, 0)


# stored stage states each stage of the memory-optimised forms (App. A)
# reads at the site besides its stencil input: the non-zero entries of the
# a* rows (and of b* for the last stage) other than the input's own
RK_HIST = {"rkhe3": [0, 1, 2], "rkck": [0, 1, 2, 3, 4, 5]}


def rk_generic_bytes(integrator: str, R: int) -> int:
    """Algorithmic HBM bytes per site per step: every stage reads its input
    state, the stored states it combines and the field, and writes one state."""
    C = 2 * R
    return sum((1 + h) * C + R + C for h in RK_HIST[integrator])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def batch_ramp(w):
    """(omega, knot_t, knot_values, kind) of a ramped workload for Batch calls."""
    from paper_2603_05447_amd import GPE_POT_RF_RAMP, GPE_POT_SHELL_RAMP
    return (w.omega, w.knot_t, w.knot_delta, GPE_POT_SHELL_RAMP if w.kind == "shell" else GPE_POT_RF_RAMP)


_WORKLOADS = {}


def workload(name: str, *args):
    """Seeded workload, built once per run (the 60M-site shell takes a while)."""
    key = (name,) + args
    if key not in _WORKLOADS:
        from workloads import configs
        t = time.time()
        _WORKLOADS[key] = getattr(configs, name)(*args)
        log(f"[bench] {name}{args}: {_WORKLOADS[key].n_active} sites ({time.time() - t:.1f}s)")
    return _WORKLOADS[key]


# Algorithmic bytes per active site per time step of the whole step (each
# stencil input read once per stage, each stored state written once), the
# figures the roofline targets are stated in: imaginary time 2 passes, RK4
# the four memory-optimised stages in the App. A storage scheme.
STEP_BYTES = {"itp": {"c128": 80, "c64": 40}, "rk4": {"c128": 240, "c64": 120}}


def step_roofline(n: int, ms_per_step: float, phase: str, dtype: str) -> dict:
    b = STEP_BYTES[phase][dtype]
    gbps = b * n / (ms_per_step * 1e-3) / 1e9
    return {"bytes_per_site_step": b, "ms_per_step": ms_per_step, "site_updates_per_s": n / (ms_per_step * 1e-3),
            "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS}


def profiled_traffic(family: str, workload: str = "c2_c128", variant: int = 0):
    """Calibrated HBM bytes per launch of `family` on `workload` under launch
    variant `variant` from the committed rocprofv3 summaries (profiles/*.txt,
    FETCH_SIZE + WRITE_SIZE scaled by a copy kernel of known size), or None
    when no summary was taken on the current kernel source."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2603_05447_amd", "csrc", "kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt"))):
        for line in open(f):
            if not line.startswith("TRAFFIC "):
                continue
            kv = dict(item.split("=", 1) for item in line.split()[1:])
            if (kv.get("family") == family and kv.get("sha256") == sha and kv.get("workload", "c2_c128") == workload
                    and kv.get("variant", "0") == str(variant)):
                return int(kv["fetch_bytes"]) + int(kv["write_bytes"]), os.path.basename(f)
    return None, None


def cpu_model() -> str:
    """The host CPU as /proc/cpuinfo names it: model name, family/model/stepping,
    clock and the number of logical CPUs the kernel reports."""
    info = {}
    n = 0
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" not in line:
                    continue
                k, v = (x.strip() for x in line.split(":", 1))
                if k == "processor":
                    n += 1
                if k in ("model name", "cpu family", "model", "stepping", "cpu MHz", "cache size") and k not in info:
                    info[k] = v
    except OSError:
        pass
    if not info:
        return platform.processor() or "unknown"
    return (f"{info.get('model name', '?')} (family {info.get('cpu family', '?')}, model {info.get('model', '?')}, "
            f"stepping {info.get('stepping', '?')}, {info.get('cpu MHz', '?')} MHz, cache {info.get('cache size', '?')}, "
            f"{n} logical CPUs in /proc/cpuinfo)")


def cpu_threads() -> dict:
    """Threads the oracle's numeric libraries may use (all pinned to one)."""
    out = {v: os.environ.get(v) for v in ("OMP_NUM_THREADS", "MKL_NUM_THREADS", "OPENBLAS_NUM_THREADS")}
    try:
        from threadpoolctl import threadpool_info
        out["threadpools"] = [{"api": d.get("internal_api"), "num_threads": d.get("num_threads")}
                              for d in threadpool_info()]
    except Exception as e:   # threadpoolctl is optional
        out["threadpools"] = f"unavailable: {e}"
    return out


# ---------------------------------------------------------------------------
def setup_c2(dev, dtype):
    import torch
    from paper_2603_05447_amd import Grid, Potential
    from workloads import configs
    t = time.time()
    w = configs.c2()
    log(f"[bench] C2 inputs: {w.n_active} sites, {w.runs.shape[0]} runs ({time.time() - t:.1f}s)")
    cdt = torch.complex128 if dtype == "c128" else torch.complex64
    rdt = torch.float64 if dtype == "c128" else torch.float32
    g = Grid.from_box(w.box, runs=w.runs, device=0)
    U = torch.tensor(w.field, dtype=rdt, device=dev)
    psi = torch.tensor(w.psi0, dtype=cdt, device=dev)
    d_itp, d_rt = w.extra["delta_itp"], w.extra["delta_rt"]
    pot_itp = Potential.rf(U, w.omega, [0.0], [d_itp])
    pot_rt = Potential.rf(U, w.omega, [0.0], [d_rt])
    return w, g, U, psi, pot_itp, pot_rt


def run_phase_timed(g, psi, pot_itp, pot_rt, w, k_itp, k_rt, configs=None):
    """k_itp imaginary-time then k_rt RK4 steps; configs = (variant for
    imaginary time, variant for real time) or None for the grid's own."""
    import torch
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record(s)
    if k_itp:
        if configs:
            g.set_config(configs[0])
        g.imag_time(psi, pot_itp, w.g, w.dt, k_itp, observe=False)
    e1.record(s)
    if k_rt:
        if configs:
            g.set_config(configs[1])
        g.real_time(psi, pot_rt, w.g, w.dt, k_rt, observe=False)
    e2.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), e1.elapsed_time(e2)


def achievable_copy_gbps(dev, mib: int = 1024, reps: int = 10) -> float:
    """Bandwidth of the library's plain streaming copy (1 GiB read + 1 GiB
    written), HIP events on the launch stream: the achievable ceiling the
    passes are read against beside the 8 TB/s vendor peak."""
    import torch
    from paper_2603_05447_amd import stream_copy
    src = torch.ones(mib << 20, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        stream_copy(src, dst)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        stream_copy(src, dst)
    e1.record(s)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    ok = bool(torch.equal(src, dst))
    del src, dst
    torch.cuda.empty_cache()
    if not ok:
        raise RuntimeError("stream copy produced wrong bytes")
    return 2.0 * (mib << 20) / (us * 1e-6) / 1e9


def kernel_table(kern: dict, R: int, scheme: int, n: int) -> dict:
    """Per kernel family: launches, average duration (HIP events on the launch
    stream) and algorithmic GB/s."""
    kernels = {}
    for fam, v in kern.items():
        if v["launches"] == 0:
            continue
        avg_us = 1e3 * v["total_ms"] / v["launches"]
        b = algo_bytes(fam, R, scheme) * n
        kernels[fam] = {"launches": v["launches"], "avg_us": avg_us, "total_ms": v["total_ms"],
                        "algo_bytes_per_launch": b, "GBps": (b / (avg_us * 1e-6) / 1e9) if b else None}
    return kernels


def dominant_roofline(kern: dict, workload: str, copy_gbps=None, variant=0) -> dict:
    """Roofline of the kernel family that takes the most time."""
    dom = max((f for f in kern if kern[f]["GBps"] is not None), key=lambda f: kern[f]["total_ms"])
    k = kern[dom]
    traffic, tsrc = profiled_traffic(dom, workload, variant) if isinstance(variant, int) else (None, None)
    r = {"bound": "hbm", "kernel": dom, "achieved": k["GBps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
         "frac": k["GBps"] / HBM_PEAK_GBPS, "traffic": traffic, "traffic_unit": "bytes/launch",
         "traffic_source": tsrc, "algo_bytes_per_launch": k["algo_bytes_per_launch"],
         "avg_launch_us": k["avg_us"], "launches": k["launches"]}
    if copy_gbps:
        r["achievable_copy_GBps"] = copy_gbps
        r["frac_of_copy"] = k["GBps"] / copy_gbps
    return r


def bench_c2(args, dev, dtype, report):
    import torch
    from paper_2603_05447_amd import KernelTimer
    from paper_2603_05447_amd import config_describe
    w, g, U, psi, pot_itp, pot_rt = setup_c2(dev, dtype)
    n = w.n_active
    R = 8 if dtype == "c128" else 4
    if args.config is not None:
        g.set_config(args.config)
    tune = None
    phase_cfg = None
    if args.autotune or dtype == "c64":
        # complex64 runs each phase with the variant the tuner picks for it on
        # this grid (variant 0, the default, is the complex128 choice)
        scratch = psi.clone()
        b_itp, t_itp = g.autotune(scratch, pot_itp, w.g, w.dt, reps=5, phase="itp")
        b_rt, t_rt = g.autotune(scratch, pot_rt, w.g, w.dt, reps=5)
        del scratch
        phase_cfg = (b_itp, b_rt)
        tune = {"itp": {"best": b_itp, "ms_per_step": {str(k): t for k, t in enumerate(t_itp)}},
                "rk4": {"best": b_rt, "ms_per_step": {str(k): t for k, t in enumerate(t_rt)}},
                "variants": {str(k): config_describe(k) for k in range(len(t_rt))}}
        log(f"[bench] autotune {dtype}: imaginary time variant {b_itp}, RK4 variant {b_rt}")
    # warmup (also builds the chunk tables)
    run_phase_timed(g, psi, pot_itp, pot_rt, w, max(args.warmup, 1), 2 * max(args.warmup, 1), phase_cfg)
    scheme = config_describe(g.get_config())["rk_scheme"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_itp, ms_rt = run_phase_timed(g, psi, pot_itp, pot_rt, w, args.steps, 2 * args.steps, phase_cfg)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # kernel durations: the same K steps again with a HIP event pair around
    # every launch on the launch stream (kept out of the timed region above:
    # the event pairs serialise the launches and add about 5 % to a step)
    with KernelTimer() as kt:
        ms_itp_k, ms_rt_k = run_phase_timed(g, psi, pot_itp, pot_rt, w, args.steps, 2 * args.steps, phase_cfg)
        kern = kt.read()
    total_ms = ms_itp + ms_rt
    # untimed check: the state is still normalised / finite
    obs = g.observe(psi, pot_rt, 0.0, w.g)
    res = {
        "n_active": n,
        "ms_per_step": total_ms / args.steps,
        "wall_s": wall,
        "site_updates_per_s": n * 3 * args.steps / (total_ms * 1e-3),
        "itp": {"ms_per_step": ms_itp / args.steps, "site_updates_per_s": n * args.steps / (ms_itp * 1e-3),
                "eff_GBps": 2 * algo_bytes("itp_pass1", R) * n * args.steps / (ms_itp * 1e-3) / 1e9},
        "rt_rk4": {"ms_per_step": ms_rt / (2 * args.steps),
                   "site_updates_per_s": n * 2 * args.steps / (ms_rt * 1e-3),
                   "eff_GBps": sum(algo_bytes(f"rk_stage{i}", R, scheme) for i in range(1, 5)) * n * 2 * args.steps
                   / (ms_rt * 1e-3) / 1e9,
                   "algo_bytes_per_site_step": sum(algo_bytes(f"rk_stage{i}", R, scheme) for i in range(1, 5)),
                   "rk_scheme": scheme},
        "final_norm": obs["norm"],
        "config": g.get_config() if phase_cfg is None else {"itp": phase_cfg[0], "rk4": phase_cfg[1]},
        "autotune": tune,
        "step_roofline": {"itp": step_roofline(n, ms_itp / args.steps, "itp", dtype),
                          "rk4": step_roofline(n, ms_rt / (2 * args.steps), "rk4", dtype)},
        "kernel_timing": {"note": "per-launch durations from a second pass of the same steps with an event "
                                  "pair around every launch; that pass's step times:",
                          "itp_ms_per_step": ms_itp_k / args.steps, "rk4_ms_per_step": ms_rt_k / (2 * args.steps)},
    }
    res["kernels"] = kernel_table(kern, R, scheme, n)
    report[dtype] = res
    del psi, U, g
    torch.cuda.empty_cache()
    return w


def bench_integrators(args, dev, report):
    """Real time on the RF bubble with each explicit integrator (Sec.
    II.A): ms per step and effective bandwidth of the memory-optimised forms."""
    import torch
    from paper_2603_05447_amd import config_describe
    w, g, U, psi, pot_itp, pot_rt = setup_c2(dev, "c128")
    n, R = w.n_active, 8
    steps = max(args.int_steps, 1)
    out = {"workload": "rf-bubble 1024x1024x512, 16,028,656 active sites, complex128", "steps": steps}
    scheme = config_describe(g.get_config())["rk_scheme"]
    for integ in ("rk4", "rkhe3", "rkck"):
        g.real_time(psi, pot_rt, w.g, w.dt, 2, observe=False, integrator=integ)     # warm-up
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        g.real_time(psi, pot_rt, w.g, w.dt, steps, observe=False, integrator=integ)
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        b = (sum(algo_bytes(f"rk_stage{i}", R, scheme) for i in range(1, 5)) if integ == "rk4"
             else rk_generic_bytes(integ, R))
        out[integ] = {"ms_per_step": ms, "site_updates_per_s": n / (ms * 1e-3),
                      "algo_bytes_per_site_step": b, "eff_GBps": b * n / (ms * 1e-3) / 1e9,
                      "stages": {"rk4": 4, "rkhe3": 3, "rkck": 6}[integ]}
        log(f"[bench] {integ}: {ms:.3f} ms/step, {b} B/site/step, {out[integ]['eff_GBps']:.0f} GB/s")
    obs = g.observe(psi, pot_rt, 0.0, w.g)
    out["final_norm"] = obs["norm"]
    report["integrators_c2"] = out
    del psi, U, g
    torch.cuda.empty_cache()


def bench_itp_real(args, dev, report):
    """Imaginary time on the RF bubble on a real state (Sec. II.A: a
    real start stays real) against the complex form of the same step."""
    import torch
    w, g, U, psi, pot_itp, pot_rt = setup_c2(dev, "c128")
    n = w.n_active
    steps = max(args.int_steps, 1)
    real = psi.real.abs().contiguous()
    out = {"workload": "rf-bubble 1024x1024x512, 16,028,656 active sites, float64 state vs complex128",
           "steps": steps}
    for name, x, b in (("complex128", psi, 2 * algo_bytes("itp_pass1", 8)), ("float64", real, 2 * 3 * 8)):
        variant, times = 0, None
        if name == "float64":
            # the real state runs in the variant the tuner picks for it (the
            # complex one in variant 0, its own choice on this grid)
            scratch = x.clone()
            variant, times = g.autotune(scratch, pot_itp, w.g, w.dt, reps=5, phase="itp")
            del scratch
        g.imag_time(x, pot_itp, w.g, w.dt, 2, observe=False)      # warm-up
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        g.imag_time(x, pot_itp, w.g, w.dt, steps, observe=False)
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out[name] = {"ms_per_step": ms, "site_updates_per_s": n / (ms * 1e-3), "algo_bytes_per_site_step": b,
                     "eff_GBps": b * n / (ms * 1e-3) / 1e9, "launch_config": variant}
        if times is not None:
            out[name]["autotune_ms_per_step"] = {str(k): v for k, v in enumerate(times)}
        log(f"[bench] ITP {name} (variant {variant}): {ms:.3f} ms/step, {b} B/site/step, "
            f"{out[name]['eff_GBps']:.0f} GB/s")
    out["speedup_real_over_complex"] = out["complex128"]["ms_per_step"] / out["float64"]["ms_per_step"]
    report["itp_real_c2"] = out
    del psi, real, U, g
    torch.cuda.empty_cache()


def bench_restage(args, dev, report):
    """One stage of a staged ramp on the RF bubble (Sec. V): post-selection
    on the device from two box potentials, the carry-over of psi to the new
    grid, and real time with the potential interpolated between the stage
    arrays (two field reads per stage instead of one)."""
    import torch
    from paper_2603_05447_amd import Grid, Potential
    w, g, U_c, psi, pot_itp, pot_rt = setup_c2(dev, "c128")
    box = w.box
    ax = [torch.tensor(box.axis(d), dtype=torch.float64, device=dev) for d in range(3)]
    U = 0.5 * (ax[0][:, None, None] ** 2 + ax[1][None, :, None] ** 2 + 4.0 * ax[2][None, None, :] ** 2)
    Va = torch.sqrt((U - 60.0) ** 2 + 4.0).contiguous()
    Vb = torch.sqrt((U - 62.0) ** 2 + 4.0).contiguous()
    del U
    torch.cuda.synchronize()
    t = time.perf_counter()
    g2 = Grid.from_threshold(box.n, box.h, box.x0, Va, Vb, 27.0, device=0)
    t_sel = time.perf_counter() - t
    t = time.perf_counter()
    psi2 = g2.remap_from(g, psi)
    torch.cuda.synchronize()
    t_remap = time.perf_counter() - t
    fa, fb = g2.pack(Va), g2.pack(Vb)
    del Va, Vb
    steps = max(args.int_steps, 1)
    pot = Potential.lerp(fa, fb, 0.0, steps * w.dt)
    g2.real_time(psi2, pot, w.g, w.dt, 2, observe=False)       # warm-up
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    g2.real_time(psi2, pot, w.g, w.dt, steps, observe=False)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    b = 224 + 4 * 8
    report["restage_c2"] = {
        "workload": "stage Delta 60 -> 62 of the rf-bubble 1024x1024x512 box, cutoff 27 on min(V_a, V_b)",
        "n_active_before": w.n_active, "n_active_after": g2.n_active, "post_selection_s": t_sel,
        "remap_ms": 1e3 * t_remap, "lerp_rk4_ms_per_step": ms, "algo_bytes_per_site_step": b,
        "eff_GBps": b * g2.n_active / (ms * 1e-3) / 1e9}
    log(f"[bench] restage: select {t_sel:.2f}s, remap {1e3 * t_remap:.1f} ms, LERP RK4 {ms:.3f} ms/step "
        f"({g2.n_active} sites)")
    del psi, psi2, fa, fb, g, g2
    torch.cuda.empty_cache()


def bench_hoc(args, dev, report):
    """The 19-point HOC stencil (App. B eq. (B2)) and the cubic 27-point one
    on the RF bubble: the same passes as the 7-point path with 16 / 24
    lateral taps per site."""
    import torch
    w, g, U, psi, pot_itp, pot_rt = setup_c2(dev, "c128")
    n = w.n_active
    steps = max(args.int_steps, 1)
    out = {"workload": "rf-bubble 1024x1024x512, 16,028,656 active sites, complex128", "steps": steps}
    for pts in (7, 19, 27):
        g.set_stencil(pts)
        res = {}
        for name, fn, b in (("itp", lambda k: g.imag_time(psi, pot_itp, w.g, w.dt, k, observe=False), 80),
                            ("rk4", lambda k: g.real_time(psi, pot_rt, w.g, w.dt, k, observe=False), 224)):
            fn(2)
            torch.cuda.synchronize()
            s = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            fn(steps)
            e1.record(s)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            res[name] = {"ms_per_step": ms, "site_updates_per_s": n / (ms * 1e-3),
                         "eff_GBps": b * n / (ms * 1e-3) / 1e9}
        if pts != 7:
            res["segments"] = int(g.hoc_segments(pts).shape[0])
        out[f"{pts}pt"] = res
        log(f"[bench] {pts}-point: ITP {res['itp']['ms_per_step']:.3f} ms, RK4 {res['rk4']['ms_per_step']:.3f} ms")
    g.set_stencil(7)
    report["hoc19_c2"] = out
    del psi, U, g
    torch.cuda.empty_cache()


def bench_c1(args, dev, report):
    """C1, the tiny shell (40,600 sites, 500 imaginary-time steps, complex128):
    it fits in L2 / Infinity Cache, so only the update rate is reported, beside
    the FP64 oracle running the same 500 steps on one host core."""
    import torch
    from paper_2603_05447_amd import Grid, Potential
    from workloads import configs
    w = configs.c1()
    g = Grid.from_box(w.box, runs=w.runs, device=0)
    V = torch.tensor(w.field, dtype=torch.float64, device=dev)
    psi = torch.tensor(w.psi0, dtype=torch.complex128, device=dev)
    pot = Potential.static(V)
    g.imag_time(psi.clone(), pot, w.g, w.dt, 5, observe=False)      # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    obs = g.imag_time(psi, pot, w.g, w.dt, w.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    out = {"workload": w.name, "n_active": w.n_active, "steps": w.steps, "s": el,
           "site_updates_per_s": w.n_active * w.steps / el, "energy": obs["energy"]}
    if not args.no_cpu:
        from oracle import itp, operator as op
        from workloads import site_linear_index
        T = op.kinetic_direct(w.box.n, w.box.h, site_linear_index(w.box, w.runs))
        t = time.perf_counter()
        itp.imaginary_time(T, w.psi0, w.field, w.g, w.dt, w.box.dV, w.steps)
        ct = time.perf_counter() - t
        out["oracle_1core_site_updates_per_s"] = w.n_active * w.steps / ct
    report["c1"] = out
    log(f"[bench] C1: {out['site_updates_per_s']:.3g} site-updates/s on the GPU")


def cpu_baseline(args):
    """The FP64 oracle, single-threaded, on a slab of the headline workload:
    the active sites of x-planes [960, 1088) of the 2048 x 2048 x 1024 shell
    (the same shell, Dirichlet at the slab faces), one RK4 step per repeat."""
    from oracle import operator as op, realtime as rt
    from oracle.potential import RFRamp
    from workloads import site_linear_index
    w = workload("c5")
    runs, idx = _slab(w, 960, 1088)
    t = time.perf_counter()
    T = op.kinetic_direct(w.box.n, w.box.h, site_linear_index(w.box, runs))
    t_build = time.perf_counter() - t
    ramp = RFRamp(w.field[idx], w.omega, w.knot_t, w.knot_delta)
    psi = w.psi0[idx]
    reps, times = 0, []
    t_all = time.perf_counter()
    while True:
        t = time.perf_counter()
        psi = rt.rk4_step(T, psi, reps * w.dt, w.dt, ramp, w.g)
        times.append(time.perf_counter() - t)
        reps += 1
        if reps >= 3 and (time.perf_counter() - t_all > args.cpu_seconds or reps >= 60):
            break
    med = float(np.median(times))
    return {"value": idx.size / med, "unit": "site-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"FP64 NumPy/SciPy oracle, single thread, on x-planes [960,1088) of the headline shell "
                      f"({idx.size} active sites); median of {reps} repeats of 1 RK4 step "
                      f"(operator build {t_build:.1f}s not counted)",
            "host_cpu": cpu_model(), "host_threads_available": os.cpu_count(), "threads": cpu_threads()}


def cpu_c2_slab(args):
    """The FP64 oracle, single-threaded, on x-planes [448, 576) of the RF
    bubble (1024 x 1024 x 512): one imaginary-time step plus two RK4 steps
    per repeat."""
    from oracle import operator as op, itp, realtime as rt
    from oracle.potential import RFRamp
    from workloads import configs, site_linear_index
    w = configs.c2()
    runs, idx = _slab(w, 448, 576)
    U = w.field[idx]
    psi = w.psi0[idx]
    lin = site_linear_index(w.box, runs)
    t = time.perf_counter()
    T = op.kinetic_direct(w.box.n, w.box.h, lin)
    t_build = time.perf_counter() - t
    V = np.sqrt((U - w.extra["delta_itp"]) ** 2 + w.omega ** 2)
    P = itp.propagator(V, w.dt)
    ramp = RFRamp(U, w.omega, [0.0], [w.extra["delta_rt"]])
    reps, times = 0, []
    t_all = time.perf_counter()
    while True:
        t = time.perf_counter()
        psi, _ = itp.itp_step(T, psi, P, w.g, w.dt, w.box.dV)
        psi = rt.rk4_step(T, psi, 0.0, w.dt, ramp, w.g)
        psi = rt.rk4_step(T, psi, w.dt, w.dt, ramp, w.g)
        times.append(time.perf_counter() - t)
        reps += 1
        if reps >= 3 and (time.perf_counter() - t_all > args.cpu_seconds / 2 or reps >= 50):
            break
    med = float(np.median(times))
    return {"sample": f"x-planes [448,576) of the RF bubble ({idx.size} active sites); median of {reps} repeats "
                      f"of 1 imaginary-time + 2 RK4 steps (operator build {t_build:.1f}s not counted)",
            "site_updates_per_s": idx.size * 3 / med}


def _slab(w, i_lo, i_hi):
    """Active sites of x-planes [i_lo, i_hi) of a workload: (runs, compact indices)."""
    sel = (w.runs[:, 0] >= i_lo) & (w.runs[:, 0] < i_hi)
    runs = w.runs[sel]
    lens = runs[:, 3] - runs[:, 2]
    starts = np.concatenate([[0], np.cumsum(w.runs[:, 3] - w.runs[:, 2])[:-1]])[sel]
    return runs, np.concatenate([np.arange(s, s + l) for s, l in zip(starts, lens)])


def cpu_per_config(args, report):
    """The FP64 oracle (one thread) on the other workloads, each on a bounded
    sample, beside the GPU rate of the same work where the report has it:
    the RF bubble on x-planes [448, 576), C3 loss + gradient over a 4-step
    prefix of the ramp on the whole grid, C4 10 RK4 steps of four sampled
    instances, and a 20-step prefix of the downscaled shell."""
    from oracle import operator as op, realtime as rt, adjoint as adj
    from oracle.potential import RFRamp
    from workloads import configs, site_linear_index
    out = {}
    c2 = cpu_c2_slab(args)
    if "c128" in report:
        c2["gpu_site_updates_per_s_c128"] = report["c128"]["site_updates_per_s"]
    out["c2_slab"] = c2
    # C3: forward + adjoint, 10 steps, whole grid
    w = configs.c3()
    T = op.kinetic_direct(w.box.n, w.box.h, site_linear_index(w.box, w.runs))
    ramp = RFRamp(w.field, w.omega, w.knot_t, w.knot_delta)
    rng = np.random.default_rng(7)
    tgt = w.psi0 * np.exp(1j * rng.uniform(0.0, 0.3, w.n_active))
    tgt /= np.sqrt(np.sum(np.abs(tgt) ** 2) * w.box.dV)
    k = 4
    t = time.perf_counter()
    adj.fidelity_grad(T, ramp, w.g, w.dt, 0.0, k, w.psi0, tgt, w.box.dV)
    el = time.perf_counter() - t
    c3 = {"sample": f"loss + 8-knot gradient over the first {k} of {w.steps} steps, {w.n_active} sites",
          "s_per_step": el / k}
    if "adjoint_c3" in report:
        gpu = report["adjoint_c3"]["s_per_grad"] / report["adjoint_c3"]["steps"]
        c3["gpu_s_per_step"] = gpu
        c3["gpu_speedup"] = (el / k) / gpu
    out["c3_forward_adjoint"] = c3
    del T, ramp, tgt, w
    # C4: four sampled instances, complex128, 10 RK4 steps each
    sites, el = 0, 0.0
    from oracle.potential import ShellRamp
    for i in (0, 21, 42, 63):
        w = configs.c4_instance(i)
        T = op.kinetic_direct(w.box.n, w.box.h, site_linear_index(w.box, w.runs))
        ramp = ShellRamp(w.field, w.omega, w.knot_t, w.knot_delta)
        t = time.perf_counter()
        rt.real_time(T, w.psi0, ramp, w.g, w.dt, 0.0, 10)
        el += time.perf_counter() - t
        sites += w.n_active
    c4 = {"sample": f"instances 0, 21, 42, 63 ({sites} sites), 10 RK4 steps each", "site_updates_per_s": sites * 10 / el}
    if "batched_c4" in report:
        c4["gpu_site_updates_per_s_c64_batched"] = report["batched_c4"]["graph"]["site_updates_per_s"]
    out["c4_sampled"] = c4
    # C5 subdomain (the shell shrunk 8x per axis, same thickness in grid
    # units): a 20-step prefix of the 20,000-step study
    w = workload("c5_subdomain", 8)
    T = op.kinetic_direct(w.box.n, w.box.h, site_linear_index(w.box, w.runs))
    ramp = RFRamp(w.field, w.omega, w.knot_t, w.knot_delta)
    t = time.perf_counter()
    rt.real_time(T, w.psi0, ramp, w.g, w.dt, 0.0, 20)
    el = time.perf_counter() - t
    sub = {"sample": f"{w.name} ({w.n_active} sites), the first 20 of 20,000 RK4 steps",
           "site_updates_per_s": w.n_active * 20 / el}
    if "c5_subdomain" in report:
        sub["gpu_site_updates_per_s_c128"] = report["c5_subdomain"]["c128"]["site_updates_per_s"]
    out["c5_subdomain_prefix"] = sub
    out["cores"] = 1
    out["threads"] = cpu_threads()
    return out


def bench_adjoint(args, dev, report):
    """256^3 hollowing ramp: loss + 8-knot gradient by the adjoint, vs plain
    FP64 forward runs of the same 2000 steps."""
    import torch
    from paper_2603_05447_amd import Grid, Potential
    from workloads import configs
    w = configs.c3(steps=args.adj_steps)
    g = Grid.from_box(w.box, runs=w.runs, device=0)
    U = torch.tensor(w.field, dtype=torch.float64, device=dev)
    # psi0 / target: ground states at the first and last detuning (imaginary time on the GPU)
    psi0 = torch.tensor(w.psi0, dtype=torch.complex128, device=dev)
    g.imag_time(psi0, Potential.rf(U, w.omega, [0.0], [w.knot_delta[0]]), w.g, 1e-3, 300, observe=False)
    tgt = psi0.clone()
    g.imag_time(tgt, Potential.rf(U, w.omega, [0.0], [w.knot_delta[-1]]), w.g, 1e-3, 300, observe=False)
    pot = Potential.rf(U, w.omega, w.knot_t, w.knot_delta)
    # the ramp lasts 2 time units whatever the step count: refuse a dt above RK4's bound
    g.real_time(psi0.clone(), pot, w.g, w.dt, 1, observe=False, check_stability=True)
    g.fidelity_grad(psi0, tgt, pot, w.g, w.dt, 20)   # warmup
    torch.cuda.synchronize()
    t = time.perf_counter()
    loss, grad = g.fidelity_grad(psi0, tgt, pot, w.g, w.dt, w.steps)
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t
    p = psi0.clone()
    g.real_time(p, pot, w.g, w.dt, 20, observe=False)
    torch.cuda.synchronize()
    t = time.perf_counter()
    g.real_time(p, pot, w.g, w.dt, w.steps, observe=False)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t
    report["adjoint_c3"] = {"workload": w.name, "n_active": w.n_active, "steps": w.steps,
                            "grads_per_s": 1.0 / t_grad, "s_per_grad": t_grad,
                            "forward_fp64_runs_per_s": 1.0 / t_fwd, "grad_over_forward_time": t_grad / t_fwd,
                            "loss": loss, "grad": [float(x) for x in grad]}
    del g, U, psi0, tgt, p
    torch.cuda.empty_cache()


def bench_batched(args, dev, report):
    """64 instances (96^3..192^3 boxes; harmonic shells whose radius is
    ramped over 8 knots), complex64 storage with FP64 reductions, one
    hipGraph-captured step replayed per step."""
    import torch
    from paper_2603_05447_amd import Grid, Batch, GPE_C64, GPE_MODE_RT
    from workloads import configs
    t = time.time()
    ws = [configs.c4_instance(i, steps=args.batch_steps) for i in range(args.batch_n)]
    log(f"[bench] C4 inputs: {sum(w.n_active for w in ws)} sites in {len(ws)} instances ({time.time() - t:.1f}s)")
    grids = [Grid.from_box(w.box, runs=w.runs, device=0) for w in ws]
    b = Batch(grids, device=0)
    psi = torch.tensor(np.concatenate([w.psi0 for w in ws]), dtype=torch.complex64, device=dev)
    field = torch.tensor(np.concatenate([w.field for w in ws]), dtype=torch.float32, device=dev)
    ramps = [batch_ramp(w) for w in ws]
    gs, dts = [w.g for w in ws], [w.dt for w in ws]
    work = torch.empty(b.work_bytes(GPE_C64, GPE_MODE_RT, 1), dtype=torch.uint8, device=dev)
    from paper_2603_05447_amd import config_describe
    # the batch's own launch variant: timed over every variant on replayed steps of this batch
    scratch = psi.clone()
    t = time.perf_counter()
    best, times = b.autotune(scratch, field, ramps, gs, dts, reps=3, use_graph=True)
    t_tune = time.perf_counter() - t
    del scratch
    log(f"[bench] C4 batch autotune: variant {best} ({config_describe(best)}), "
        f"{times[best]:.3f} ms/step vs variant 0 {times[0]:.3f} ms/step ({t_tune:.1f} s)")
    scheme = config_describe(best)["rk_scheme"]
    out = {"autotune": {"best": best, "ms_per_step": {str(k): v for k, v in enumerate(times)},
                        "variant": config_describe(best), "tune_s": t_tune}}
    for use_graph in (False, True):
        b.real_time(psi, field, ramps, gs, dts, 5, use_graph=use_graph, work=work, observe=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        obs = b.real_time(psi, field, ramps, gs, dts, args.batch_steps, use_graph=use_graph, work=work)
        el = time.perf_counter() - t
        out["graph" if use_graph else "eager"] = {
            "s": el, "site_updates_per_s": b.total * args.batch_steps / el,
            "eff_GBps": sum(algo_bytes(f"rk_stage{i}", 4, scheme) for i in range(1, 5)) * b.total * args.batch_steps
            / el / 1e9,
            "step_roofline": step_roofline(b.total, 1e3 * el / args.batch_steps, "rk4", "c64"),
            "norm_min": min(o["norm"] for o in obs), "norm_max": max(o["norm"] for o in obs)}
    # forward + adjoint of every instance in one batched call (sqrt(N) checkpoints), complex64 storage
    # against complex128 throughout: loss and 8 knot gradients per instance
    rng = np.random.default_rng(4242)
    tg = []
    for w in ws:
        t_ = w.psi0 * np.exp(1j * rng.uniform(0.0, 0.3, w.n_active))
        tg.append(t_ / np.sqrt(np.sum(np.abs(t_) ** 2) * w.box.dV))
    tg = np.concatenate(tg)
    psi0 = np.concatenate([w.psi0 for w in ws])
    adj = {}
    for name, cdt, rdt in (("c64", torch.complex64, torch.float32), ("c128", torch.complex128, torch.float64)):
        p0 = torch.tensor(psi0, dtype=cdt, device=dev)
        tt = torch.tensor(tg, dtype=cdt, device=dev)
        fd = torch.tensor(np.concatenate([w.field for w in ws]), dtype=rdt, device=dev)
        b.fidelity_grad(p0, tt, fd, ramps, gs, dts, 10, use_graph=True)      # warmup
        torch.cuda.synchronize()
        t = time.perf_counter()
        loss, grads = b.fidelity_grad(p0, tt, fd, ramps, gs, dts, args.batch_steps, use_graph=True)
        el = time.perf_counter() - t
        pf = p0.clone()
        b.real_time(pf, fd, ramps, gs, dts, 5, use_graph=True, observe=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        b.real_time(pf, fd, ramps, gs, dts, args.batch_steps, use_graph=True, observe=False)
        torch.cuda.synchronize()
        el_f = time.perf_counter() - t
        adj[name] = {"s": el, "instance_grads_per_s": len(ws) / el, "forward_s": el_f,
                     "grad_over_forward_time": el / el_f, "loss": np.asarray(loss), "grads": np.stack(grads)}
        del p0, tt, fd, pf
    g64, g128 = adj["c64"].pop("grads"), adj["c128"].pop("grads")
    l64, l128 = adj["c64"].pop("loss"), adj["c128"].pop("loss")
    adj["c64_vs_c128"] = {
        "grad_rel_err_max": float(np.max(np.abs(g64 - g128).max(axis=1) / np.abs(g128).max(axis=1))),
        "grad_rel_err_median": float(np.median(np.abs(g64 - g128).max(axis=1) / np.abs(g128).max(axis=1))),
        "loss_abs_err_max": float(np.max(np.abs(l64 - l128)))}
    out["forward_adjoint"] = adj
    report["batched_c4"] = {"instances": len(ws), "total_sites": b.total, "steps": args.batch_steps, **out}
    del b, grids, psi, field, work
    torch.cuda.empty_cache()


def bench_c5(args, dev, report):
    """The headline workload, the largest configuration: the thin RF-dressed
    shell in a 2048 x 2048 x 1024 box (59,748,872 active sites).  In each
    precision (complex128, FP64 throughout; complex64, FP32 stencil with FP64
    reductions) from the same seeded start: the grid tuner picks the launch
    variant, W warm-up steps run on a copy, the timed region is exactly K RK4
    steps of the state, and a second pass of K steps with an event pair around
    every launch gives the per-kernel durations.  Then the complex64 state is
    compared with the complex128 one after the same K steps."""
    import torch
    from paper_2603_05447_amd import Grid, Potential, KernelTimer, config_describe
    w = workload("c5")
    g = Grid.from_box(w.box, runs=w.runs, device=0)
    K = args.c5 if args.c5 else args.steps
    out = {"workload": w.name, "n_active": w.n_active, "steps": K, "warmup": args.warmup}
    n0 = float(np.sum(np.abs(w.psi0) ** 2)) * w.box.dV
    res = {}
    for dtype, cdt, rdt in (("c128", torch.complex128, torch.float64), ("c64", torch.complex64, torch.float32)):
        R = 8 if dtype == "c128" else 4
        U = torch.tensor(w.field, dtype=rdt, device=dev)
        psi = torch.tensor(w.psi0, dtype=cdt, device=dev)
        pot = Potential.rf(U, w.omega, w.knot_t, w.knot_delta)
        # the launch variant the tuner picks for this precision on this grid
        # (or the one --c5-config names)
        scratch = psi.clone()
        if args.c5_config is None:
            best, times = g.autotune(scratch, pot, w.g, w.dt, reps=5)
            log(f"[bench] C5 {dtype} autotune: variant {best} ({config_describe(best)})")
        else:
            best, times = args.c5_config, []
            g.set_config(best)
        scheme = config_describe(best)["rk_scheme"]
        g.real_time(scratch, pot, w.g, w.dt, max(args.warmup, 1), observe=False)
        del scratch
        e0 = g.observe(psi, pot, 0.0, w.g)["energy"]
        # timed region: exactly K steps
        torch.cuda.synchronize()
        s_ = torch.cuda.current_stream()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t = time.perf_counter()
        ev0.record(s_)
        g.real_time(psi, pot, w.g, w.dt, K, observe=False)
        ev1.record(s_)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        ms_step = ev0.elapsed_time(ev1) / K
        obs = g.observe(psi, pot, K * w.dt, w.g)
        res[dtype] = psi.to(torch.complex128).cpu().numpy()
        # per-kernel durations: K more steps with an event pair around every launch
        with KernelTimer() as kt:
            g.real_time(psi, pot, w.g, w.dt, K, t0=K * w.dt, observe=False, check_stability=False)
            kern = kernel_table(kt.read(), R, scheme, w.n_active)
        out[dtype] = {"ms_per_step": ms_step, "wall_s": wall, "site_updates_per_s": w.n_active / (ms_step * 1e-3),
                      "eff_GBps": sum(algo_bytes(f"rk_stage{i}", R, scheme) for i in range(1, 5))
                      * w.n_active / (ms_step * 1e-3) / 1e9,
                      "step_roofline": step_roofline(w.n_active, ms_step, "rk4", dtype),
                      "kernels": kern,
                      "launch_variant": best,
                      "autotune_ms_per_step": {str(k): v for k, v in enumerate(times)},
                      "roofline": dominant_roofline(kern, f"c5_{dtype}", variant=g.get_config()),
                      "norm_drift": obs["norm"] - n0, "energy_start": e0, "energy": obs["energy"]}
        log(f"[bench] C5 {dtype}: {out[dtype]['site_updates_per_s']:.4g} site-updates/s over {K} RK4 steps")
        del U, psi
        g.release_work()
        torch.cuda.empty_cache()
    a, b = res["c64"], res["c128"]
    out["c64_vs_c128_rel_l2"] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    ov = np.vdot(b, a)
    out["c64_vs_c128_phase_aligned"] = float(1.0 - abs(ov) / (np.linalg.norm(a) * np.linalg.norm(b)))
    report["precision_c5"] = out


def bench_c5_subdomain(args, dev, report):
    """The precision study over its full horizon on the downscaled shell
    (2048 x 2048 x 1024 shrunk 8x per axis, 931,864 sites, the same thickness
    in grid units): 20,000 RK4 steps in complex128 and complex64 against the
    FP64 oracle's stored run (sampled sites after 20 / 200 / 2,000 / 20,000
    steps, norm and energy), when the stored run is present."""
    import torch
    from paper_2603_05447_amd import Grid, Potential
    w = workload("c5_subdomain", 8)
    ref = None
    path = os.path.join(ROOT, "tests", "golden", "c5_subdomain_s8.npz")
    if os.path.exists(path):
        ref = np.load(path)
    g = Grid.from_box(w.box, runs=w.runs, device=0)
    out = {"workload": w.name, "n_active": w.n_active, "steps": w.steps, "oracle_reference": ref is not None}
    n0 = float(np.sum(np.abs(w.psi0) ** 2)) * w.box.dV
    for dtype, cdt, rdt in (("c128", torch.complex128, torch.float64), ("c64", torch.complex64, torch.float32)):
        U = torch.tensor(w.field, dtype=rdt, device=dev)
        psi = torch.tensor(w.psi0, dtype=cdt, device=dev)
        pot = Potential.rf(U, w.omega, w.knot_t, w.knot_delta)
        res = {"errors_vs_oracle": {}}
        done, t_run = 0, 0.0
        for stop in (20, 200, 2000, w.steps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            obs = g.real_time(psi, pot, w.g, w.dt, stop - done, t0=done * w.dt)
            t_run += time.perf_counter() - t
            done = stop
            if ref is not None:
                k = list(ref["sample_steps"]).index(stop)
                idx = torch.as_tensor(ref["sample_index"], device=dev)
                got = psi[idx].to(torch.complex128).cpu().numpy()
                want = ref["samples"][k]
                ov = np.vdot(want, got)
                res["errors_vs_oracle"][str(stop)] = {
                    "rel_l2": float(np.linalg.norm(got - want) / np.linalg.norm(want)),
                    "phase_aligned": float(1.0 - abs(ov) / (np.linalg.norm(got) * np.linalg.norm(want))),
                    "max_abs_over_max": float(np.max(np.abs(got - want)) / np.max(np.abs(want)))}
        res["s"] = t_run
        res["site_updates_per_s"] = w.n_active * w.steps / t_run
        res["norm_drift"] = obs["norm"] - n0
        res["energy"] = obs["energy"]
        if ref is not None:
            ro = ref["obs"][list(ref["obs_steps"]).index(w.steps)]
            res["oracle_norm"], res["oracle_energy"] = float(ro[0]), float(ro[1])
            res["norm_rel_err"] = abs(obs["norm"] - ro[0]) / ro[0]
            res["energy_rel_err"] = abs(obs["energy"] - ro[1]) / abs(ro[1])
        out[dtype] = res
        log(f"[bench] C5 subdomain {dtype}: {w.steps} steps in {t_run:.2f} s; "
            f"{res['errors_vs_oracle'].get(str(w.steps), {})}")
        del U, psi
    g.release_work()
    torch.cuda.empty_cache()
    report["c5_subdomain"] = out


def bench_c2_job(args, dev, report):
    """The RF bubble job end to end, in complex128 and complex64: the ground
    state by imaginary time at Delta = 60, then RK4 real time after the
    quench to Delta = 62 (dt = 2e-4 for both), with observables at the phase
    boundaries and the complex64 final state against the complex128 one."""
    import torch
    out, finals = {}, {}
    for dtype in ("c128", "c64"):
        w, g, U, psi, pot_itp, pot_rt = setup_c2(dev, dtype)
        torch.cuda.synchronize()
        t = time.perf_counter()
        o_itp = g.imag_time(psi, pot_itp, w.g, w.dt, args.job_itp)
        t_itp = time.perf_counter() - t
        o0 = g.observe(psi, pot_rt, 0.0, w.g)
        torch.cuda.synchronize()
        t = time.perf_counter()
        o_rt = g.real_time(psi, pot_rt, w.g, w.dt, args.job_rt)
        t_rt = time.perf_counter() - t
        finals[dtype] = psi.to(torch.complex128).cpu().numpy()
        out[dtype] = {"imag_time_s": t_itp, "real_time_s": t_rt, "total_s": t_itp + t_rt,
                      "site_updates_per_s": w.n_active * (args.job_itp + args.job_rt) / (t_itp + t_rt),
                      "ground_state": {"norm": o_itp["norm"], "energy": o_itp["energy"], "mu": o_itp["mu"]},
                      "real_time": {"energy_start": o0["energy"], "energy_end": o_rt["energy"],
                                    "norm_end": o_rt["norm"]}}
        log(f"[bench] job {dtype}: imaginary time {t_itp:.2f} s, real time {t_rt:.2f} s")
        del g, U, psi
        torch.cuda.empty_cache()
    a, b = finals["c64"], finals["c128"]
    out["c64_vs_c128_rel_l2"] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    out["c64_vs_c128_phase_aligned"] = float(1.0 - abs(np.vdot(b, a)) / (np.linalg.norm(a) * np.linalg.norm(b)))
    report["job_c2"] = {"workload": "rf-bubble 1024x1024x512, 16,028,656 active sites, g=2000, dt=2e-4",
                        "imag_time_steps": args.job_itp, "real_time_steps": args.job_rt, **out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", type=int, default=None, help="launch variant index (default: library default)")
    ap.add_argument("--autotune", action="store_true", help="time every launch variant and use the fastest")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-cpu-all", action="store_true",
                    help="skip the oracle on samples of the 256^3 ramp, the batch and the 60M-site shell")
    ap.add_argument("--no-extras", action="store_true", help="skip complex64, adjoint and batched legs")
    ap.add_argument("--adj-steps", type=int, default=2000,
                    help="steps of the 2-time-unit adjoint ramp (dt = 2/steps; RK4 needs steps >= 1100)")
    ap.add_argument("--batch-n", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=1000)
    ap.add_argument("--int-steps", type=int, default=100, help="steps per integrator in the RKHE3/RK4/RKCK leg")
    ap.add_argument("--c5-config", type=int, default=None,
                    help="launch variant for the large shell (default: the grid tuner picks one per precision)")
    ap.add_argument("--c5", type=int, default=0,
                    help="timed RK4 steps on the large shell, the headline workload (default: --steps; the "
                         "full precision study is 20000)")
    ap.add_argument("--job", action=argparse.BooleanOptionalAction, default=None,
                    help="run the RF bubble job end to end (imaginary then real time) in both precisions "
                         "(default: on, off with --no-extras)")
    ap.add_argument("--job-itp", type=int, default=5000)
    ap.add_argument("--job-rt", type=int, default=10000)
    ap.add_argument("--legs", default="all",
                    help="comma list of legs to run (for profiling one workload): c5, c2, c64, adjoint, "
                         "batched, integrators, itp_real, restage, hoc, c1, c5_subdomain, job; 'all' runs every "
                         "leg. Without c5 (the headline workload) no headline line is printed, only the legs' "
                         "report")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run a plain elementwise copy of this many MiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.job is None:
        args.job = not args.no_extras
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2603_05447_amd as p
    p.load_library()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    report = {}
    t_start = time.time()
    if args.calib_copy_mb > 0:
        x = torch.ones(args.calib_copy_mb * 2 ** 20 // 8, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1.0, out=y)      # reads and writes calib_copy_mb MiB each
        torch.cuda.synchronize()
        del x, y
        torch.cuda.empty_cache()
    legs = None if args.legs == "all" else set(args.legs.split(","))

    def leg(name: str) -> bool:
        return legs is None or name in legs

    copy_gbps = None
    if leg("c5"):
        bench_c5(args, dev, report)
        copy_gbps = achievable_copy_gbps(dev)
        log(f"[bench] streaming copy: {copy_gbps:.0f} GB/s")
    if leg("c2"):
        bench_c2(args, dev, "c128", report)
        log(f"[bench] RF bubble c128 done: {report['c128']['site_updates_per_s']:.4g} site-updates/s")
    if not args.no_extras:
        if leg("c64"):
            bench_c2(args, dev, "c64", report)
            log(f"[bench] RF bubble c64 done: {report['c64']['site_updates_per_s']:.4g} site-updates/s")
        if leg("adjoint"):
            bench_adjoint(args, dev, report)
            log(f"[bench] adjoint done: {report['adjoint_c3']['grads_per_s']:.3g} grads/s")
        if leg("batched"):
            bench_batched(args, dev, report)
            log("[bench] batched done")
        if leg("integrators"):
            bench_integrators(args, dev, report)
            log("[bench] integrators done")
        if leg("itp_real"):
            bench_itp_real(args, dev, report)
            log("[bench] real imaginary time done")
        if leg("restage"):
            bench_restage(args, dev, report)
            log("[bench] restage done")
        if leg("hoc"):
            bench_hoc(args, dev, report)
            log("[bench] 19-point stencil done")
        if leg("c1"):
            bench_c1(args, dev, report)
        if leg("c5_subdomain"):
            bench_c5_subdomain(args, dev, report)
    if args.job and leg("job"):
        bench_c2_job(args, dev, report)
        log("[bench] RF bubble job done")
    if not leg("c5"):
        print(json.dumps({"legs": sorted(legs), "report": report}, default=float), flush=True)
        return
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args)
        log(f"[bench] cpu baseline: {cpu['value']:.4g} site-updates/s")
    if not args.no_cpu and not args.no_cpu_all and not args.no_extras:
        report["cpu_oracle_per_config"] = cpu_per_config(args, report)
        log("[bench] oracle on the other workloads done")

    c5 = report["precision_c5"]
    main_res = c5["c128"]
    kern = main_res["kernels"]
    roofline = dominant_roofline(kern, "c5_c128", copy_gbps, variant=main_res["launch_variant"])
    roofline_steps = {f"c5_rk4_{dt}": c5[dt]["step_roofline"] for dt in ("c128", "c64")}
    roofline_steps.update({f"c2_{ph}_{dt}": report[dt]["step_roofline"][ph]
                           for dt in ("c128", "c64") if dt in report for ph in ("itp", "rk4")})
    line = {
        "metric": METRIC,
        "value": main_res["site_updates_per_s"],
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": c5["steps"],
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "large thin shell: 2048x2048x1024 box, h=0.0306, anisotropic RF-dressed shell "
                               "(kappa=12.9), mask V<61, 59,748,872 active sites (1.39 %), g=1e4, dt=5e-5, "
                               "complex128 (FP64 throughout); one step = 1 RK4 step; the complex64 run of the "
                               "same steps is in precision_c5",
                   "n_active": c5["n_active"], "launch_config": main_res["launch_variant"]},
        "roofline": roofline,
        "roofline_steps": roofline_steps,
        "cpu_baseline": cpu,
        "precision_c5": c5,
        "wall_s": time.time() - t_start,
    }
    if "c128" in report:
        line["phases_c2"] = {"c128": {k2: v for k2, v in report["c128"].items() if k2 != "kernels"}}
        line["kernels_c2_c128"] = report["c128"]["kernels"]
        line["roofline_c2"] = dominant_roofline(report["c128"]["kernels"], "c2_c128", copy_gbps,
                                                variant=report["c128"]["config"])
    if "c64" in report:
        line.setdefault("phases_c2", {})["c64"] = {k2: v for k2, v in report["c64"].items() if k2 != "kernels"}
        line["kernels_c2_c64"] = report["c64"]["kernels"]
    for key in ("adjoint_c3", "batched_c4", "integrators_c2", "itp_real_c2", "restage_c2", "hoc19_c2", "c1",
                "c5_subdomain", "job_c2", "cpu_oracle_per_config"):
        if key in report:
            line[key] = report[key]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
