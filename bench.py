#!/usr/bin/env python3
"""Throughput of the RAAR hot path on one MI355X.

A step is one RAAR iteration over every frame of the large-frame scan
(2048 x 2048 object, 2025 frames of 256 x 256, Fresnel-defocused aperture
probe, jittered raster step 40, Poisson noise at 1e8 photons per frame,
beta = 0.75, known probe): gather, batched 2-D FFT, Fourier-modulus
projection, inverse FFT, RAAR update and overlap merge.  The scan is
synthetic and seeded; its intensities come from the library's own forward
model on the GPU, then Poisson noise.  Inputs are resident in HBM before the
timed region.

Prints ONE JSON line.  `value` is frames/s per RAAR iteration.  `roofline`
reports the dominant kernel's algorithmic HBM bytes per launch over its mean
launch time (HIP events on the library's stream during the timed region).
`cpu_baseline` times the FP64 oracle on a bounded sub-scan on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "frames/s per RAAR iteration + achieved HBM GB/s (% peak), plain vs batched/grad"


def algorithmic_bytes(K: int, m: int, n: int, form: int = 1) -> dict:
    """Bytes the method itself must move per iteration, attributed to the
    kernel that moves them (intermediates an implementation adds are not
    counted).  Per frame pixel: carry read 8, amplitudes 4, carry write 8,
    merge input write 8, merge input read 8 (36 B).  Per object pixel:
    gathered object read 8, D^-1 read 4, object write 8 (20 B)."""
    fp = K * m * m
    op = n * n
    out = {"iteration": 36 * fp + 20 * op}
    if m == 256 and form == 2:   # Fourier-domain carry: gather + rows, columns with the carry, strip merge
        out.update({"frame": 8 * op, "cols": 28 * fp, "merge": 8 * fp + 12 * op})
    elif m == 256:               # three passes: row (carry + gather), column (amplitudes), output row (writes)
        out.update({"frame": 8 * fp + 8 * op, "cols": 4 * fp, "frame_out": 16 * fp, "merge": 8 * fp + 12 * op})
    else:                        # one fused frame kernel
        out.update({"frame": 28 * fp + 8 * op, "merge": 8 * fp + 12 * op})
    return out


def kernel_names(m: int, form: int) -> dict:
    if m == 256 and form == 2:
        return {"frame": "mp_row_fwd<256, GATHER>", "cols": "col_carry_kernel", "merge": "strip_merge_kernel"}
    if m == 256:
        return {"frame": "mp_row_fwd<256, RAAR>", "cols": "mp_col<256, RAAR>", "frame_out": "mp_row_inv<256, RAAR>",
                "merge": "merge_kernel<T, MK_V>"}
    return {"frame": f"fg_kernel<{m}, RAAR>", "merge": "merge_kernel<T, MK_V>"}


def gpu_workload(steps: int, warmup: int, timing: bool, fft_block: int = 0):
    import numpy as np
    import torch

    from paper_1602_01448_amd import Plan
    from sharp_data import gen

    dev = torch.device("cuda", 0)
    s = gen.config_scan(3)
    plan = Plan.tuned(s.n, s.n, s.m, s.positions, device=dev, **({"fft_block": fft_block} if fft_block else {}))
    obj = torch.from_numpy(s.obj.astype(np.complex64)).to(dev)
    probe = torch.from_numpy(s.probe.astype(np.complex64)).to(dev)
    I = plan.simulate(obj, probe)
    c = s.photons / (I.double().sum().item() / s.K)
    gcuda = torch.Generator(device=dev)
    gcuda.manual_seed(16023)
    I = torch.poisson(I * c, generator=gcuda).float()
    plan.set_data(I)
    plan.set_probe((probe * float(np.sqrt(c))).contiguous())
    plan.set_object(torch.from_numpy(s.psi0.astype(np.complex64)).to(dev))
    del obj, I
    plan.raar(warmup, s.beta)
    torch.cuda.synchronize(dev)
    if timing:
        plan.timing(True)
        plan.timing_read()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(dev)
    t0.record()
    for _ in range(steps):
        plan.raar(1, s.beta)
    t1.record()
    torch.cuda.synchronize(dev)
    ms = t0.elapsed_time(t1)
    kt = plan.timing_read() if timing else {}
    plan.timing(False)
    eps = plan.metrics()
    return s, plan, ms, kt, eps


def grad_form(reps: int = 10) -> dict:
    """Amplitude-loss gradient on the gradient workload (512^2 object, 1024
    frames of 128^2): frames/s = K / (time of one sharp_grad call)."""
    import numpy as np
    import torch

    from paper_1602_01448_amd import Plan
    from sharp_data import gen

    dev = torch.device("cuda", 0)
    s = gen.config_scan(4)
    psi, w = gen.gradient_point(s)
    plan = Plan.tuned(s.n, s.n, s.m, s.positions, kind="grad", device=dev)
    I = plan.simulate(torch.from_numpy(s.obj.astype(np.complex64)).to(dev),
                      torch.from_numpy(s.probe.astype(np.complex64)).to(dev))
    plan.set_data(I)
    tpsi = torch.from_numpy(psi.astype(np.complex64)).to(dev)
    tw = torch.from_numpy(w.astype(np.complex64)).to(dev)
    for _ in range(3):
        plan.grad(tpsi, tw)
    torch.cuda.synchronize(dev)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        plan.grad(tpsi, tw)
    t1.record()
    torch.cuda.synchronize(dev)
    ms = t0.elapsed_time(t1) / reps
    fp = s.K * s.m * s.m
    alg = 20 * fp + 16 * s.n * s.n
    return {"workload": "gradient: object 512x512, 1024 frames 128x128", "frames_per_s": round(s.K / (ms / 1e3), 1),
            "ms_per_call": round(ms, 4), "achieved_alg_GBps": round(alg / (ms / 1e3) / 1e9, 1)}


def probe_form(iters: int = 20) -> dict:
    """Probe refinement every iteration on the probe-retrieval workload (512^2
    object, 841 frames of 64^2, Poisson 1e6 photons/frame, probe from the
    data): ms per iteration without constraints and with the Fourier mask plus
    the centre-of-mass correction of the probe update."""
    import numpy as np
    import torch

    from paper_1602_01448_amd import Plan
    from sharp_data import gen

    dev = torch.device("cuda", 0)
    s = gen.config_scan(2)
    obj = torch.from_numpy(s.obj.astype(np.complex64)).to(dev)
    w = torch.from_numpy(s.probe.astype(np.complex64)).to(dev)
    f = np.fft.fftfreq(s.m) * s.m
    mask = torch.from_numpy((np.hypot(f[:, None], f[None, :]) < s.m / 4).astype(np.float32)).to(dev)
    out = {"workload": f"probe refinement every iteration: object {s.n}x{s.n}, {s.K} frames {s.m}x{s.m}"}
    for name, center in (("plain", False), ("mask_and_center", True)):
        plan = Plan(s.n, s.n, s.m, s.positions, probe_every=1, probe_center=center, device=dev)
        I = plan.simulate(obj, w)
        plan.set_data(I).init_probe()
        if center:
            plan.set_probe_constraint(mask=mask)
        plan.set_object(torch.from_numpy(s.psi0.astype(np.complex64)).to(dev)).raar(2, s.beta)
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize(dev)
        t0.record()
        plan.raar(iters, s.beta)
        t1.record()
        torch.cuda.synchronize(dev)
        out[f"{name}_ms_per_iteration"] = round(t0.elapsed_time(t1) / iters, 4)
        del plan
    return out


def batched_form(iters: int = 20) -> dict:
    """32 independent uneven scans (n 256..1024, m in {64,128,256}, 100..1500
    frames), 20 RAAR iterations: batched (one graph launch) vs the same plans
    iterated one after another."""
    import numpy as np
    import torch

    from paper_1602_01448_amd import Batch, Plan
    from sharp_data import gen

    dev = torch.device("cuda", 0)
    scans = gen.batch_scans()
    plans = []
    for s in scans:
        p = Plan(s.n, s.n, s.m, s.positions, device=dev)
        w = torch.from_numpy(s.probe.astype(np.complex64)).to(dev)
        I = p.simulate(torch.from_numpy(s.obj.astype(np.complex64)).to(dev), w)
        p.set_data(I).set_probe(w).set_object(torch.from_numpy(s.psi0.astype(np.complex64)).to(dev))
        plans.append(p)
    frames = sum(s.K for s in scans)
    b = Batch(plans)
    b.raar(iters, 0.75)          # warm-up and graph capture
    for p in plans:
        p.raar(1, 0.75)
    torch.cuda.synchronize(dev)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    b.raar(iters, 0.75)
    t1.record()
    torch.cuda.synchronize(dev)
    ms_b = t0.elapsed_time(t1)
    t0.record()
    for p in plans:
        p.raar(iters, 0.75)
    t1.record()
    torch.cuda.synchronize(dev)
    ms_p = t0.elapsed_time(t1)
    return {"workload": f"{len(scans)} uneven scans, {frames} frames, {iters} iterations",
            "batched_frames_per_s": round(frames * iters / (ms_b / 1e3), 1),
            "plain_sequential_frames_per_s": round(frames * iters / (ms_p / 1e3), 1),
            "speedup": round(ms_p / ms_b, 3)}


# HBM bytes per iteration of the large-frame kernels from rocprofv3 counters
# (FETCH_SIZE x 2.0 and WRITE_SIZE x 1.0: the ratios the same counters give
# for a 1 GiB device copy), summed over the kernel's launches in one
# iteration, taken on the kernels as they stand; the summary with its
# commands is profiles/raar_carry_form_2048obj_2025x256_kernels.txt.  To be
# emptied whenever these kernels change until the counters are taken again.
MEASURED_TRAFFIC = {("cols", 2): 4_778_800_000, ("merge", 2): 2_218_700_000}


def traffic_for(kernel: str, form: int, launches_per_iteration: float):
    v = MEASURED_TRAFFIC.get((kernel, form))
    return None if v is None else round(v / launches_per_iteration)


def copy_calibration(nbytes: int = 1 << 30) -> None:
    """A plain device copy of known size, so that the memory counters of the
    profiled kernels can be scaled (run under rocprofv3 --pmc)."""
    import torch

    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"copy calibration: {nbytes} bytes read, {nbytes} bytes written", file=sys.stderr, flush=True)


def fig3_form(max_iters: int = 1000, check_every: int = 5, target: float = 5e-4) -> dict:
    """The shape of the paper's only published benchmark: 10,000 frames of 128^2
    from a 1000^2 image, periodic boundaries, known probe; RAAR (beta 0.75) from
    a U[0,1) start until eps_0 < 5e-4 (Eq. (solutionmetric): Q*-weighted error
    against the known object, minimised over a global phase).  eps_0 is
    evaluated every `check_every` iterations outside the timed iterations."""
    import numpy as np
    import torch

    from paper_1602_01448_amd import Plan
    from sharp_data import gen

    dev = torch.device("cuda", 0)
    s = gen.fig3_scan()
    plan = Plan.tuned(s.n, s.n, s.m, s.positions, periodic=True, device=dev)
    obj = torch.from_numpy(s.obj.astype(np.complex64)).to(dev)
    w = torch.from_numpy(s.probe.astype(np.complex64)).to(dev)
    plan.set_data(plan.simulate(obj, w)).set_probe(w)
    D = plan.apply("QSTAR", plan.apply("Q", torch.ones_like(obj))).real.double()
    B = (D * obj.to(torch.complex128))
    nb2 = (B.abs() ** 2).sum().item()
    plan.set_object(torch.from_numpy(s.psi0.astype(np.complex64)).to(dev))

    def eps0():
        A = D * plan.object().to(torch.complex128)
        na2 = (A.abs() ** 2).sum().item()
        cross = torch.vdot(A.flatten(), B.flatten()).abs().item()
        return float(np.sqrt(max(na2 + nb2 - 2 * cross, 0.0) / nb2))

    torch.cuda.synchronize(dev)
    spent, it, e = 0.0, 0, eps0()
    while it < max_iters and e >= target:
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        plan.raar(check_every, 0.75)
        t1.record()
        torch.cuda.synchronize(dev)
        spent += t0.elapsed_time(t1) / 1e3
        it += check_every
        e = eps0()
    return {"workload": "10,000 frames 128x128, 1000x1000 object, periodic, known probe (paper's benchmark shape)",
            "iterations": it, "eps0": e, "reached": bool(e < target), "seconds": round(spent, 4),
            "ms_per_iteration": round(1e3 * spent / max(it, 1), 4),
            "paper": "< 2 s to eps0 < 5e-4 on 16 GTX Titan GPUs in 4 nodes (context, other hardware)"}


def cpu_baseline(budget_rows: int = 5, iters: int = 2) -> dict:
    """The FP64 oracle on the frames of the first raster rows of the same
    scan (an object strip that holds them), timed over `iters` iterations."""
    import numpy as np

    import oracle as O
    from sharp_data import gen

    from threadpoolctl import threadpool_limits

    s = gen.config_scan(3)
    sel = np.where(s.positions[:, 0] < budget_rows * 40 - 2)[0]
    pos = s.positions[sel]
    ny = int(pos[:, 0].max()) + s.m
    with threadpool_limits(limits=1):          # NumPy's FFT is single-threaded; keep BLAS there too
        I = O.forward_intensity(s.obj[:ny], s.probe, pos)
        t = time.perf_counter()
        O.raar(I, pos, (ny, s.n), s.m, iters, s.beta, psi0=s.psi0[:ny], w0=s.probe)
        dt = time.perf_counter() - t
    return {"value": round(len(sel) * iters / dt, 3), "unit": "frames/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(sel)} frames of 256x256 (first {budget_rows} raster rows, {ny}x{s.n} object strip), "
                      f"{iters} RAAR iterations incl. set-up, NumPy FP64, one thread"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="do not bracket kernels with HIP events")
    ap.add_argument("--no-forms", action="store_true", help="skip the gradient and batched comparisons")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (reference for memory counters)")
    ap.add_argument("--fft-block", type=int, default=0, choices=(0, 128, 256, 512),
                    help="m=256 pass workgroup threads (0: tuned or library default)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on exactly one GPU (asked for {args.gpus}); "
              "multi-GPU sharding is a design note only", file=sys.stderr)
        return 2

    import torch

    if args.copy_calibration:
        copy_calibration()
    s, plan, ms, kt, eps = gpu_workload(args.steps, args.warmup, not args.no_timing, args.fft_block)
    plan.sync()
    ms_step = ms / args.steps
    fps = s.K / (ms_step / 1e3)
    form = plan.info()["frame_launch"]
    B = algorithmic_bytes(s.K, s.m, s.n, form)
    out = {
        "metric": METRIC,
        "value": round(fps, 1),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded scan, intensities from the library's forward model + Poisson noise)",
        "config": {"workload": "large-frame RAAR: object 2048x2048, 2025 frames 256x256, step 40 jitter 2, "
                               "1e8 photons/frame, beta 0.75, known probe",
                   "object": s.n, "frame": s.m, "frames": s.K, "beta": s.beta,
                   "frame_launch": form, "strip_rows": plan.info()["strip_rows"],
                   "fft_block": plan.info()["fft_block"], "merge_tile": plan.info()["tile"],
                   "merge_split": plan.info()["merge_split"]},
        "achieved_alg_GBps": round(B["iteration"] / (ms_step / 1e3) / 1e9, 1),
        "alg_frac_of_hbm_peak": round(B["iteration"] / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
        "eps_a_last": float(eps[-1]) if len(eps) else None,
    }
    if kt:
        per = {k: {"ms_mean": round(v[0] / v[1], 4), "launches": v[1]} for k, v in kt.items()}
        out["kernels"] = per
        # dominant kernel: the longest mean launch among those with algorithmic bytes
        dom = max((k for k in per if k in B), key=lambda k: per[k]["ms_mean"])
        # bytes per launch (a kernel may be launched more than once per step)
        lpi = per[dom]["launches"] / args.steps
        per_launch = B[dom] / lpi
        ach = per_launch / (per[dom]["ms_mean"] / 1e3) / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                           "frac": round(ach / HBM_PEAK_GBPS, 4), "traffic": traffic_for(dom, form, lpi),
                           "kernel": kernel_names(s.m, form).get(dom, dom), "alg_bytes_per_launch": round(per_launch),
                           "launch_ms": per[dom]["ms_mean"]}
    del plan
    if not args.no_forms:
        out["forms"] = {"grad": grad_form(), "batched": batched_form(), "paper_fig3": fig3_form(),
                        "probe_constraints": probe_form()}
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
