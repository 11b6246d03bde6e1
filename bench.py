"""Throughput of the single-copy, two-step-merged D3Q19 BGK update on one MI355X.

    python bench.py [--gpus 1] [--steps 500] [--warmup 20] [--scheme swap2] [--storage f32]

Workload: 512^3 periodic lattice, FP32 (offset) storage and arithmetic,
tau = 0.6, 3D Taylor-Green vortex (u0 = 0.02, k = 2 pi / 512) plus seeded
uniform noise of amplitude 1e-3 per velocity component.  A "step" is one
lattice time step; the merged scheme advances two per launch.  The fields are
made on the host and copied in before timing; the timed region only runs
lbm_step on device-resident data.

Prints one JSON line: MLUPS over the timed region (HIP events on the stream the
kernels run on), a roofline entry for the dominant kernel (the marching kernel,
timed per launch by the library's event hook) against the 8 TB/s HBM peak, and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}
METRIC = "D3Q19 MLUPS and % HBM roofline, 1 GPU; adjoint/forward step-time ratio"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--scheme", default="swap2", choices=["swap2", "swap1", "two_array", "swap3"])
    ap.add_argument("--storage", default="f32", choices=["f32", "f64", "f16", "bf16"])
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--workload", default="tgv", choices=["tgv", "cavity", "large", "channel"],
                    help="tgv: the periodic Taylor-Green + noise workload (tau 0.6); cavity: lid-driven cavity "
                         "(tau 0.52, five walls, +y lid at 0.05 along x, rest state); large: periodic random-phase "
                         "Taylor-Green (tau 0.55, seed 4) built on the device, for 1024^3; channel: the adjoint's "
                         "channel (periodic x, walls in y and z, tau 0.8, per-cell force N(0, 1e-12) seed 1, rest "
                         "state)")
    ap.add_argument("--shape", default=None, metavar="NXxNYxNZ", help="a lattice of this shape instead of --size cubed")
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--velocities", type=int, default=19, choices=[15, 19, 27],
                    help="velocity set (D3Q15 and D3Q27: FP64/FP32 storage, planes of one round)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=24.0, help="target length of the oracle sample (the estimate from a short timing runs long, so the sample lands near 10-20 s)")
    ap.add_argument("--copy-probe", type=int, default=1 << 31, metavar="BYTES",
                    help="device-to-device copy of BYTES bytes (a multiple of 16; 0 skips the probes): achievable "
                         "read+write rate, counter calibration; also runs the access-pattern probe on the lattice")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward ratio")
    ap.add_argument("--no-storage-sweep", action="store_true", help="skip the FP16/BF16 storage runs")
    ap.add_argument("--no-large", action="store_true", help="skip the 1024^3 single-copy run")
    ap.add_argument("--no-cpu-context", action="store_true",
                    help="skip the paper's sequential CPU algorithms (Fuse Swap, two-step, prism) on the host")
    return ap.parse_args()


def traffic_entry(kernel_key):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except Exception:
        return None
    ent = data.get(kernel_key)
    if not ent:
        return None
    from paper_2208_05429_amd.build import source_digest
    if ent.get("source_digest") != source_digest():
        return None
    return ent.get("bytes_per_launch")


def cpu_baseline(target_s):
    """The FP64 oracle (as it stands) on a bounded sample of the workload: a
    64^3 crop-sized periodic lattice with the same tau and initial-field
    recipe, run for as many steps as fit in about target_s seconds."""
    import oracle
    from paper_2208_05429_amd import workloads as wl
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    threads = max(1, min(threads, os.cpu_count() or 1))
    oracle.set_threads(threads)
    shape = (64, 64, 64)
    rho0, u0 = wl.taylor_green_3d(shape, 0.02)
    u0 += wl.uniform_noise(shape, 1e-3, 20805429)
    o = oracle.Oracle(shape, 0.6)
    f = o.init(rho0, u0)
    f = o.run(f, 2)  # first touch of the arrays and threads, untimed
    t0 = time.perf_counter()
    f = o.run(f, 8)
    dt = (time.perf_counter() - t0) / 8
    steps = max(2, int(target_s / max(dt, 1e-6)))
    t0 = time.perf_counter()
    o.run(f, steps)
    el = time.perf_counter() - t0
    n = int(np.prod(shape))
    # the same oracle on one thread, over a quarter of the time
    oracle.set_threads(1)
    t0 = time.perf_counter()
    o.run(f, 2)
    dt1 = (time.perf_counter() - t0) / 2
    steps1 = max(2, int(target_s / 4 / max(dt1, 1e-6)))
    t0 = time.perf_counter()
    o.run(f, steps1)
    el1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    return {"value": round(n * steps / el / 1e6, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"64^3 periodic Taylor-Green+noise, tau=0.6, {steps} steps, FP64 two-array, {el:.1f} s",
            "value_1_thread": round(n * steps1 / el1 / 1e6, 3), "sample_1_thread": f"{steps1} steps, {el1:.1f} s",
            "cpu": _cpu_model()}


def cpu_context(size=256, steps=2):
    """The paper's own sequential CPU algorithms (liblbm_cpu.so, one thread,
    FP64, the lid-driven cavity of Sec. 5.1 at size^3): Fuse Swap (Alg. 1),
    the two-step sweep (Alg. 2) in lexicographic order and with the prism
    traversal.  Context for the paper's relative CPU speedups (Sec. 5.2), not a
    target: MLUPS of each and the two-step variants' ratio to Fuse Swap."""
    from paper_2208_05429_amd import capi, host
    shape = (size,) * 3
    cfg = capi.make_config(shape, 0.52, faces=(1, 1, 1, 2, 1, 1), wall_u=(0.05, 0.0, 0.0))
    g = host.lbm_cpu_init(cfg)
    host.lbm_cpu_fuse_swap(cfg, g, 1)  # first touch
    runs = {"fuse_swap": lambda: host.lbm_cpu_fuse_swap(cfg, g, steps),
            "two_step": lambda: host.lbm_cpu_two_step(cfg, g, steps, 0),
            "two_step_prism16": lambda: host.lbm_cpu_two_step(cfg, g, steps, 16),
            "two_step_prism64": lambda: host.lbm_cpu_two_step(cfg, g, steps, 64)}
    out = {}
    for name, fn in runs.items():
        t0 = time.perf_counter()
        fn()
        out[name] = round(size ** 3 * steps / (time.perf_counter() - t0) / 1e6, 2)
    return {"MLUPS": out, "vs_fuse_swap": {k: round(v / out["fuse_swap"], 3) for k, v in out.items() if k != "fuse_swap"},
            "workload": f"{size}^3 lid-driven cavity, tau 0.52, FP64, {steps} steps each, one thread",
            "paper_two_step_prism_vs_fuse_prism_sequential": {"Haswell": 1.188, "Skylake": 1.155, "KNL": 1.0115}}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def adjoint_ratio(shape, steps, checkpoint, reps=3, scheme="swap2", merged=True, variant=0):
    """Backward (recompute + merged adjoint) time per step over merged forward
    time per step, for L = sum |u_T - u*|^2 on a channel (periodic x, walls in
    y and z, tau 0.8) under a per-cell force N(0, 1e-12) (seed 1); u* from a
    forward run under a hidden force (seed 2).  Also: the checkpointing
    forward of the autograd function per step, and the merged adjoint kernel
    alone against one merged forward pass."""
    import torch
    from paper_2208_05429_amd import workloads as wl
    from paper_2208_05429_amd.adjoint import ForceAdjoint
    from paper_2208_05429_amd.lattice import Lattice
    faces = ("periodic", "periodic", "wall", "wall", "wall", "wall")
    F = torch.from_numpy(wl.normal_field(shape, 1e-6, 1)).float().cuda()
    hidden = torch.from_numpy(wl.normal_field(shape, 1e-6, 2)).float().cuda()
    lat = Lattice(shape, 0.8, "f32", "swap2", faces, force=hidden)
    f0 = lat.f.clone()
    lat.step(steps)
    _, ut, _, _ = lat.macroscopic(want=("u",))
    lat.close()
    lat = Lattice(shape, 0.8, "f32", scheme, faces, force=F, f=f0.clone(), variant=variant)
    spec = dict(shape=shape, tau=0.8, storage="f32", faces=faces, steps=steps, checkpoint=checkpoint, merged=merged,
                scheme=scheme, variant=variant)
    fwd, bwd, ckf = [], [], []
    for r in range(reps + 1):
        lat.f.copy_(f0)
        torch.cuda.synchronize()
        e0, e1 = _events()
        e0.record()
        lat.step(steps)
        e1.record()
        torch.cuda.synchronize()
        Fp = F.clone().requires_grad_(True)
        c0, c1 = _events()
        c0.record()
        u = ForceAdjoint.apply(Fp, f0, spec)
        c1.record()
        L = ((u - ut.float()) ** 2).sum()
        torch.cuda.synchronize()
        b0, b1 = _events()
        b0.record()
        L.backward()
        b1.record()
        torch.cuda.synchronize()
        if r:  # the first round warms up
            fwd.append(e0.elapsed_time(e1))
            bwd.append(b0.elapsed_time(b1))
            ckf.append(c0.elapsed_time(c1))
    # the adjoint kernel alone (one reverse call of the configuration's steps)
    # against the forward kernel over the same steps (out of place)
    kk = 2 if merged else 1
    lam = torch.randn((19,) + tuple(shape), device="cuda")
    lout = torch.empty_like(lam)
    gF = torch.zeros((3,) + tuple(shape), device="cuda")
    from paper_2208_05429_amd import capi
    n = 20
    a0, a1 = _events()
    a0.record()
    for _ in range(n):
        capi.lbm_step_adjoint(lat.ctx, lat.f.data_ptr(), lam.data_ptr(), lout.data_ptr(), gF.data_ptr(), kk)
    a1.record()
    f1 = torch.empty_like(lat.f)
    m0, m1 = _events()
    m0.record()
    for _ in range(n):
        lat.step_into(lat.f, f1, kk)
    m1.record()
    torch.cuda.synchronize()
    lat.close()
    fw, bw, cf = float(np.median(fwd)) / steps, float(np.median(bwd)) / steps, float(np.median(ckf)) / steps
    ka, kf = a0.elapsed_time(a1) / (kk * n), m0.elapsed_time(m1) / (kk * n)
    return {"shape": list(shape), "steps": steps, "checkpoint": checkpoint, "scheme": scheme, "variant": variant,
            "reverse_steps_per_call": 2 if merged else 1, "forward_ms_per_step": round(fw, 5),
            "backward_ms_per_step": round(bw, 5), "ratio": round(bw / fw, 3),
            "checkpointing_forward_ms_per_step": round(cf, 5),
            "adjoint_kernel_ms_per_step": round(ka, 5), "forward_kernel_ms_per_step": round(kf, 5),
            "kernel_ratio": round(ka / kf, 3)}


def storage_sweep(size, steps):
    """MLUPS of the merged kernel with FP16 / BF16 offset storage on the bench workload."""
    import torch
    from paper_2208_05429_amd import workloads as wl
    from paper_2208_05429_amd.lattice import Lattice
    shape = (size,) * 3
    _, u0 = wl.tgv_512_fields(shape)
    u0 = torch.from_numpy(u0).cuda()
    out = {}
    for st in ("f16", "bf16"):
        lat = Lattice(shape, wl.TGV_512["tau"], st, "swap2", u0=u0)
        lat.step(4)
        torch.cuda.synchronize()
        e0, e1 = _events()
        e0.record()
        lat.step(steps)
        e1.record()
        torch.cuda.synchronize()
        out[st] = round(np.prod(shape) * steps / (e0.elapsed_time(e1) * 1e-3) / 1e6, 1)
        lat.close()
        del lat
        torch.cuda.empty_cache()
    return out


def large_run(size, steps, storage="f32"):
    """The large single-copy run: size^3 (FP32; FP64 where only one copy fits),
    periodic, tau 0.55, random-phase Taylor-Green field (seed 4), merged passes
    in rounds over bands of tile rows when the plane has more tiles than
    co-resident workgroups."""
    import torch
    from paper_2208_05429_amd import workloads as wl
    from paper_2208_05429_amd.lattice import Lattice
    cfg = wl.TGV_1024
    shape = (size,) * 3
    u0 = wl.taylor_green_3d_device(shape, cfg["u0"], wl.random_phases(cfg["phase_seed"]), "cuda")
    lat = Lattice(shape, cfg["tau"], storage, "swap2", u0=u0)
    del u0
    torch.cuda.empty_cache()
    lat.step(2)
    torch.cuda.synchronize()
    lat.set_kernel_timing(True)
    e0, e1 = _events()
    e0.record()
    lat.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kms, kn = lat.kernel_time()
    s = lat.sums()
    lat.close()
    del lat
    torch.cuda.empty_cache()
    N = size ** 3
    kper = kms[1] / max(kn[1], 1)
    b = 8 if storage == "f64" else 4
    return {"shape": list(shape), "storage": storage, "steps": steps,
            "MLUPS": round(N * steps / (ms * 1e-3) / 1e6, 1),
            "ms_per_step": round(ms / steps, 4), "march_ms_per_pass": round(kper, 4),
            "achieved_GBs": round(2 * 19 * b * N / (kper * 1e-3) / 1e9, 1),
            "distributions_GB": round(19 * b * N / 1e9, 1), "mass_finite": bool(np.isfinite(s).all())}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    if a.steps < 1 or a.warmup < 0:
        print("--steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2208_05429_amd import capi
    from paper_2208_05429_amd import workloads as wl
    from paper_2208_05429_amd.lattice import Lattice

    shape = (a.size,) * 3 if a.shape is None else tuple(int(v) for v in a.shape.lower().split("x"))
    if len(shape) != 3 or min(shape) < 1:
        print(f"--shape must be NXxNYxNZ (got {a.shape})", file=sys.stderr)
        sys.exit(2)
    sname = f"{a.size}^3" if a.shape is None else "x".join(str(v) for v in shape)
    N = int(np.prod(shape))
    print(f"[bench] building {shape} {a.storage} {a.scheme} {a.workload}", file=sys.stderr, flush=True)
    if a.workload == "cavity":
        tau = wl.CAVITY_256["tau"]
        lat = Lattice(shape, tau, a.storage, a.scheme, ("wall", "wall", "wall", "moving", "wall", "wall"),
                      (wl.CAVITY_256["lid_u"], 0.0, 0.0), variant=a.variant, velocities=a.velocities)
        wdesc = (f"{sname} lid-driven cavity D3Q{a.velocities} BGK tau={tau}, halfway bounce-back on 5 walls, +y lid "
                 f"u=({wl.CAVITY_256['lid_u']},0,0), rest state, {a.storage} storage")
    elif a.workload == "large":
        cfg = wl.TGV_1024
        tau = cfg["tau"]
        u0_dev = wl.taylor_green_3d_device(shape, cfg["u0"], wl.random_phases(cfg["phase_seed"]), "cuda")
        lat = Lattice(shape, tau, a.storage, a.scheme, u0=u0_dev, variant=a.variant, velocities=a.velocities)
        del u0_dev
        wdesc = (f"{sname} periodic D3Q{a.velocities} BGK tau={tau}, random-phase Taylor-Green u0={cfg['u0']} (seed "
                 f"{cfg['phase_seed']}), {a.storage} storage")
    elif a.workload == "channel":
        tau = 0.8
        F = torch.from_numpy(wl.normal_field(shape, 1e-6, 1)).to(torch.float64 if a.storage == "f64" else torch.float32)
        lat = Lattice(shape, tau, a.storage, a.scheme, ("periodic", "periodic", "wall", "wall", "wall", "wall"),
                      force=F.cuda(), variant=a.variant, velocities=a.velocities)
        del F
        wdesc = (f"{sname} channel D3Q{a.velocities} BGK tau={tau}, periodic x, bounce-back walls in y and z, per-cell body "
                 f"force N(0, 1e-12) (seed 1), rest state, {a.storage} storage")
    else:
        tau = wl.TGV_512["tau"]
        _, u0 = wl.tgv_512_fields(shape)
        u0_dev = torch.from_numpy(u0).to("cuda")
        del u0
        lat = Lattice(shape, tau, a.storage, a.scheme, u0=u0_dev, variant=a.variant, velocities=a.velocities)
        del u0_dev
        wdesc = (f"{sname} periodic D3Q{a.velocities} BGK tau={tau}, Taylor-Green u0=0.02 + U(+-1e-3) noise "
                 f"(seed 20805429), {a.storage} storage")
    torch.cuda.empty_cache()
    print(f"[bench] warmup {a.warmup} steps", file=sys.stderr, flush=True)
    lat.step(a.warmup)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    lat.set_kernel_timing(True)
    torch.cuda.synchronize()
    e0.record(stream)
    lat.step(a.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kms, kn = lat.kernel_time()
    lat.set_kernel_timing(False)
    print(f"[bench] timed {a.steps} steps in {ms:.2f} ms", file=sys.stderr, flush=True)
    sums = lat.sums()
    if not np.all(np.isfinite(sums)):
        print("[bench] non-finite state after the timed run", file=sys.stderr)
        sys.exit(3)

    mlups = N * a.steps / (ms * 1e-3) / 1e6
    # A merged scheme runs steps // M launches of M steps and, for a remainder,
    # one shorter launch; the roofline is that of the M-step launches (the
    # dominant kernel), the remainder's launch is reported beside.
    Mmax = {"swap2": 2, "swap3": 3}.get(a.scheme, 1)
    M = next((m for m in range(Mmax, 0, -1) if kn[m - 1] > 0), 1)
    k = M - 1
    avg_kernel_ms = kms[k] / max(kn[k], 1)
    s = BYTES[a.storage]
    Qv = a.velocities
    alg_bytes = 2 * Qv * s * N  # one read and one write of the single copy per launch
    achieved = alg_bytes / (avg_kernel_ms * 1e-3) / 1e9
    kernel_key = (f"march_M{M}_{a.storage}_{a.size}" if a.scheme != "two_array" else f"two_array_{a.storage}_{a.size}")
    if a.variant:
        kernel_key += f"_v{a.variant}"
    if a.shape is not None:
        kernel_key += "_" + sname
    if a.workload != "tgv":
        kernel_key += "_" + a.workload
    if Qv != 19:
        kernel_key += f"_q{Qv}"
    traffic = traffic_entry(kernel_key)
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms / a.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": a.storage,
        "data": "synthetic",
        "config": {"workload": wdesc,
                   "scheme": a.scheme, "steps_per_launch": M, "variant": a.variant,
                   "bytes_per_lattice_update": 2 * Qv * s / M},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "k_march" if a.scheme != "two_array" else "k_two_array",
                     "avg_kernel_ms": round(avg_kernel_ms, 4), "launches": kn[k],
                     "steps_per_launch": M, "algorithmic_bytes_per_launch": alg_bytes},
        "conservation": {"mass": sums[0], "momentum": list(sums[1:])},
    }
    if traffic:
        # measured HBM bytes (rocprofv3, calibrated) over the same launch time
        out["roofline"]["measured_gbs"] = round(traffic / (avg_kernel_ms * 1e-3) / 1e9, 1)
    for m in range(1, M):
        if kn[m - 1] > 0:
            # the launch of the remaining steps (fewer than M)
            msr = kms[m - 1] / kn[m - 1]
            out["roofline"][f"remainder_launch_{m}_steps"] = {
                "launches": kn[m - 1], "avg_kernel_ms": round(msr, 4),
                "achieved": round(2 * Qv * s * N / (msr * 1e-3) / 1e9, 1)}
    if a.copy_probe and a.scheme != "two_array" and a.storage != "f64" and shape[2] % 2 == 0 and Qv == 19:
        # the kernel's access pattern without its compute (the library's
        # pattern probe: same work items and pair accesses, no halo, no LDS,
        # no hazard checks; it stores back what it loaded)
        try:
            t = []
            for _ in range(4):
                c0, c1 = _events()
                c0.record(stream)
                capi.lbm_probe_pattern(lat.cfg, lat.f.data_ptr(), M, stream.cuda_stream)
                c1.record(stream)
                torch.cuda.synchronize()
                t.append(c0.elapsed_time(c1))
            pms = float(np.median(t[1:]))
            pgbs = alg_bytes / (pms * 1e-3) / 1e9
            out["pattern_probe"] = {"ms_per_pass": round(pms, 4), "gbs": round(pgbs, 1),
                                    "frac_of_peak": round(pgbs / HBM_PEAK_GBS, 4),
                                    "kernel_frac_of_pattern": round(achieved / pgbs, 4)}
        except capi.LbmError as ex:
            out["pattern_probe"] = {"unsupported": str(ex)}
    lat.close()
    del lat
    torch.cuda.empty_cache()
    if a.copy_probe:
        # achievable rate of the 1:1 read/write mix of an in-place pass: the
        # library's 16-byte streaming copy (on the marching kernel's grid of
        # 256 workgroups, and on larger grids), and torch's device copy
        src = torch.empty(a.copy_probe // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)

        def best_of(fn, reps=4):
            fn()
            torch.cuda.synchronize()
            best = 1e30
            for _ in range(reps):
                c0, c1 = _events()
                c0.record(stream)
                fn()
                c1.record(stream)
                torch.cuda.synchronize()
                best = min(best, c0.elapsed_time(c1))
            return 2 * a.copy_probe / (best * 1e-3) / 1e9

        hip = {b: round(best_of(lambda: capi.lbm_probe_copy(src.data_ptr(), dst.data_ptr(), a.copy_probe, b,
                                                             stream.cuda_stream)), 1)
               for b in (256, 1024, 4096)}
        torch_gbs = best_of(lambda: dst.copy_(src))
        copy_gbs = round(max(max(hip.values()), torch_gbs), 1)  # the best copy measured
        out["roofline"]["copy_gbs"] = copy_gbs
        out["roofline"]["frac_of_copy"] = round(achieved / copy_gbs, 4)
        out["copy_probe"] = {"bytes": a.copy_probe, "hip_copy16_gbs_by_grid": hip,
                             "torch_copy_gbs": round(torch_gbs, 1)}
        if "pattern_probe" in out and "gbs" in out["pattern_probe"]:
            out["pattern_probe"]["frac_of_copy"] = round(out["pattern_probe"]["gbs"] / copy_gbs, 4)
        del src, dst
        torch.cuda.empty_cache()
    headline = (a.storage == "f32" and a.scheme == "swap2" and a.workload == "tgv" and a.shape is None
                and Qv == 19)
    if headline and not a.no_storage_sweep:
        print("[bench] FP16/BF16 storage runs", file=sys.stderr, flush=True)
        sw = storage_sweep(a.size, 40)
        out["reduced_precision"] = {"MLUPS": sw, "speedup_vs_f32": {k: round(v / mlups, 3) for k, v in sw.items()}}
    if headline and not a.no_large:
        print("[bench] 1024^3 single-copy run", file=sys.stderr, flush=True)
        out["large_1024"] = large_run(1024, 50)
        print("[bench] 1024^3 FP64 single-copy run (two copies would not fit in HBM)", file=sys.stderr, flush=True)
        out["large_1024_f64"] = large_run(1024, 10, "f64")
    if not a.no_adjoint:
        print("[bench] adjoint/forward ratio", file=sys.stderr, flush=True)
        wk = adjoint_ratio((128, 64, 64), 200, 20)
        # on this small lattice the marching passes are bound by the latency
        # of each plane: the plain two-array scheme (forward and recompute)
        # with single reverse steps is the faster configuration
        wk2 = adjoint_ratio((128, 64, 64), 200, 20, scheme="two_array", merged=False)
        # the merged scheme on the 16 x 16 tiles of kernel variant 5 (more,
        # shorter plane iterations for a lattice this small)
        wk3 = adjoint_ratio((128, 64, 64), 200, 20, variant=5)
        best_fw = min(wk["forward_ms_per_step"], wk2["forward_ms_per_step"], wk3["forward_ms_per_step"])
        best_bw = min(wk["backward_ms_per_step"], wk2["backward_ms_per_step"], wk3["backward_ms_per_step"])
        out["adjoint"] = {"workload": wk, "workload_two_array_single_reverse_steps": wk2,
                          "workload_merged_16x16_tiles": wk3,
                          "workload_best_backward_over_best_forward": round(best_bw / best_fw, 3),
                          "bandwidth_bound": adjoint_ratio((256, 256, 256), 40, 20, reps=2),
                          # every other state kept (20 x 1.3 GB): no recompute in the backward
                          "bandwidth_bound_every_other_state": adjoint_ratio((256, 256, 256), 40, 2, reps=2)}
    if not a.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(a.cpu_seconds)
    else:
        out["cpu_baseline"] = None
    if not a.no_cpu_context:
        print("[bench] the paper's CPU algorithms on the host", file=sys.stderr, flush=True)
        out["cpu_context"] = cpu_context()
    print(json.dumps(out), flush=True)
    # every library context is released before the interpreter exits (those
    # the autograd graphs held go with the graphs)
    import gc
    gc.collect()
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
