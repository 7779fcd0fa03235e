"""Autotuner for the launch shapes of a scan geometry.

Times candidate launch configurations of the library on the GPU and keeps the
fastest per geometry:

* the form of the iteration for 128 x 128 and 256 x 256 frames (carry in
  the Fourier domain or in frame space; at 256 x 256 also whether the column
  pass forms its own row transform), for the 256 x 256 Fourier-carry forms
  the strip height of the fused merge (1 or 2 object rows), and for the
  256 x 256 frame-space form the pass workgroup size (128, 256 or 512
  threads, i.e. 8, 16 or 32 rows / columns of a frame per workgroup);
* merge tile side (16, 32, 64) and frame-chunk split of the overlap merge,
  for every form that uses the tile merge;
* the workgroup count of the gradient frame kernel;
* for a batch of scans, one set of per-scan options for the whole batch:
  library defaults, each scan's own tuned options, or one merge tile side
  for every scan (the batched launches group scans by frame size and tile
  side, so uniform choices mean fewer, fuller launches) -- timed as a whole.

Candidates are timed with HIP events over a few RAAR iterations (or gradient
calls) on synthetic data of the geometry's shape; every candidate computes
the same iterates (the tests check this), so only time decides.  Results go
to a JSON cache keyed by GPU architecture and geometry; ``Plan.tuned`` and
the benchmark read it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import time

import numpy as np
import torch

from .plan import Plan

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "gfx950.json")


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "gfx950"


def geometry_key(kind: str, nx: int, ny: int, m: int, positions, periodic: bool) -> str:
    pos = np.ascontiguousarray(positions, dtype=np.int32)
    digest = hashlib.sha1(pos.tobytes()).hexdigest()[:12]
    return f"{_arch()}:{kind}:{nx}x{ny}:m{m}:K{len(pos)}:p{int(periodic)}:{digest}"


def load_cache(path: str = CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: str = CACHE) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(kind: str, nx: int, ny: int, m: int, positions, periodic: bool = False, path: str = CACHE) -> dict:
    return load_cache(path).get(geometry_key(kind, nx, ny, m, positions, periodic), {}).get("options", {})


def _merge_candidates(n: int):
    out = []
    for tile in (16, 32, 64):
        tiles = ((n + tile - 1) // tile) ** 2
        splits = {1}
        s = 1
        while tiles * s < 2048 and s < 16:
            s *= 2
            splits.add(s)
        out += [{"tile": tile, "merge_split": sp} for sp in sorted(splits)]
    return out


def _frame_candidates(m: int):
    if m == 256:
        return ([{"frame_launch": f, "strip_rows": r} for f in (3, 2) for r in (1, 2)]
                + [{"frame_launch": 1, "fft_block": b} for b in (128, 256, 512)])
    if m == 128:
        return [{"frame_launch": 2}, {"frame_launch": 1}]
    return [{}]


def _uses_tile_merge(m: int, frame_opts: dict) -> bool:
    """Every form except the 256 x 256 Fourier-carry forms (whose merge is
    fused into their strip pass) ends with the tile merge."""
    return not (m == 256 and frame_opts.get("frame_launch") in (2, 3))


def _synthetic(plan: Plan, seed: int):
    g = torch.Generator(device=plan.device)
    g.manual_seed(seed)
    dev = plan.device
    obj = torch.polar(0.5 + 0.5 * torch.rand(plan.ny, plan.nx, generator=g, device=dev),
                      torch.rand(plan.ny, plan.nx, generator=g, device=dev) * 3.0 - 1.5)
    yy = torch.arange(plan.m, device=dev, dtype=torch.float32) - plan.m // 2
    probe = torch.exp(-(yy[:, None] ** 2 + yy[None, :] ** 2) / (2 * (plan.m / 5.0) ** 2)).to(torch.complex64)
    return obj.to(torch.complex64).contiguous(), probe.contiguous()


def _settle(run, warm_ms: float = 50.0) -> None:
    """Run `run()` (one step) for about `warm_ms` of GPU time (5 to 200 steps)
    before anything is timed: the clocks take some tens of milliseconds of
    steady work to settle."""
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    run()
    t1.record()
    torch.cuda.synchronize()
    n = int(min(200, max(5, warm_ms / max(t0.elapsed_time(t1), 1e-3))))
    for _ in range(n):
        run()


def _time_raar(plan: Plan, iters: int, reps: int) -> float:
    obj, probe = _synthetic(plan, 1602)
    I = plan.simulate(obj, probe)
    plan.set_data(I).set_probe(probe).set_object(torch.ones_like(obj))
    _settle(lambda: plan.raar(1, 0.75))
    best = float("inf")
    for _ in range(reps):
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize(plan.device)
        t0.record()
        plan.raar(iters, 0.75)
        t1.record()
        torch.cuda.synchronize(plan.device)
        best = min(best, t0.elapsed_time(t1) / iters)
    plan.sync()
    return best


def _time_grad(plan: Plan, reps: int, calls: int = 20) -> float:
    """Best over `reps` of the mean time of `calls` back-to-back calls, after
    the clocks have settled."""
    obj, probe = _synthetic(plan, 1603)
    plan.set_data(plan.simulate(obj, probe))
    psi = torch.ones_like(obj)
    _settle(lambda: plan.grad(psi, probe))
    best = float("inf")
    for _ in range(reps):
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize(plan.device)
        t0.record()
        for _ in range(calls):
            plan.grad(psi, probe)
        t1.record()
        torch.cuda.synchronize(plan.device)
        best = min(best, t0.elapsed_time(t1) / calls)
    return best


def tune_raar(nx: int, ny: int, m: int, positions, periodic: bool = False, iters: int = 3, reps: int = 3,
              path: str = CACHE, verbose: bool = False) -> dict:
    """Fastest launch options for RAAR on this geometry: every form of the
    iteration, and for the forms that end with the tile merge every merge
    candidate; cached."""
    key = geometry_key("raar", nx, ny, m, positions, periodic)
    results = []
    best, best_t = {}, float("inf")
    for fc in _frame_candidates(m):
        merges = _merge_candidates(max(nx, ny)) if _uses_tile_merge(m, fc) else [{}]
        for mc in merges:
            opts = {**fc, **mc}
            p = Plan(nx, ny, m, positions, periodic=periodic, **opts)
            t = _time_raar(p, iters, reps)
            results.append((opts, t))
            if verbose:
                print(f"  {opts}: {t:.4f} ms/iteration", flush=True)
            if t < best_t:
                best, best_t = opts, t
            del p
    cache = load_cache(path)
    cache[key] = {"options": best, "ms_per_iteration": round(best_t, 5), "tried": len(results),
                  "when": time.strftime("%Y-%m-%d %H:%M:%S")}
    save_cache(cache, path)
    return best


def tune_grad(nx: int, ny: int, m: int, positions, periodic: bool = False, reps: int = 5, path: str = CACHE,
              verbose: bool = False) -> dict:
    """Fastest gradient grid, merge tile and merge frame-chunk split on this
    geometry; cached."""
    key = geometry_key("grad", nx, ny, m, positions, periodic)
    best, best_t = {}, float("inf")
    for gg in (64, 128, 256, 512, 1024):
        for tile in (16, 32, 64):
            for split in (1, 2, 4, 8):
                opts = {"grad_groups": gg, "tile": tile, "merge_split": split}
                p = Plan(nx, ny, m, positions, periodic=periodic, **opts)
                t = _time_grad(p, reps)
                if verbose:
                    print(f"  {opts}: {t:.4f} ms/call", flush=True)
                if t < best_t:
                    best, best_t = opts, t
                del p
    cache = load_cache(path)
    cache[key] = {"options": best, "ms_per_call": round(best_t, 5), "when": time.strftime("%Y-%m-%d %H:%M:%S")}
    save_cache(cache, path)
    return best


def batch_key(scans) -> str:
    h = hashlib.sha1()
    for sc in scans:
        h.update(np.asarray([sc.n, sc.n, sc.m], np.int64).tobytes())
        h.update(np.ascontiguousarray(sc.positions, dtype=np.int32).tobytes())
    return f"{_arch()}:batch:{len(scans)}:{h.hexdigest()[:12]}"


def batch_options(scans, path: str = CACHE) -> list:
    """Per-scan options the batch tuner stored for this list of scans (each
    scan: object n x n, frame m, positions), else library defaults."""
    got = load_cache(path).get(batch_key(scans), {}).get("options")
    if got is None or len(got) != len(scans):
        return [{} for _ in scans]
    return [dict(o) for o in got]


def _time_batch(scans, opts, iters: int, reps: int) -> float:
    from .batch import Batch
    plans = []
    for sc, o in zip(scans, opts):
        p = Plan(sc.n, sc.n, sc.m, sc.positions, **o)
        obj, probe = _synthetic(p, 1604)
        p.set_data(p.simulate(obj, probe)).set_probe(probe).set_object(torch.ones_like(obj))
        plans.append(p)
    b = Batch(plans)
    b.raar(iters, 0.75)          # graph capture
    _settle(lambda: b.raar(iters, 0.75))
    best = float("inf")
    for _ in range(reps):
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record()
        b.raar(iters, 0.75)
        t1.record()
        torch.cuda.synchronize()
        best = min(best, t0.elapsed_time(t1) / iters)
    del b, plans
    return best


def tune_batch(scans, iters: int = 3, reps: int = 3, path: str = CACHE, verbose: bool = False) -> list:
    """Fastest per-scan option set for batched RAAR over `scans`, timed as a
    whole batch; cached under the batch's geometry key."""
    cands = {"defaults": [{} for _ in scans],
             "per_scan_tuned": [lookup("raar", sc.n, sc.n, sc.m, sc.positions, False, path) for sc in scans]}
    for tile in (16, 32):
        cands[f"tile{tile}"] = [{} if (sc.m == 256) else {"tile": tile} for sc in scans]
    best, best_t, tried = None, float("inf"), {}
    for name, opts in cands.items():
        t = _time_batch(scans, opts, iters, reps)
        tried[name] = round(t, 5)
        if verbose:
            print(f"  {name}: {t:.4f} ms/iteration", flush=True)
        if t < best_t:
            best, best_t = (name, opts), t
    cache = load_cache(path)
    cache[batch_key(scans)] = {"options": best[1], "choice": best[0], "ms_per_iteration": round(best_t, 5),
                               "tried": tried, "when": time.strftime("%Y-%m-%d %H:%M:%S")}
    save_cache(cache, path)
    return best[1]


def main() -> None:
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from sharp_data import gen

    ap = argparse.ArgumentParser(description="tune launch shapes of the benchmark workloads")
    ap.add_argument("--workloads", default="1,2,3,4,fig3")
    ap.add_argument("--path", default=CACHE)
    args = ap.parse_args()
    for w in args.workloads.split(","):
        if w == "batch":
            scans = gen.batch_scans()
            for s in scans:
                print(f"tuning raar {s.name}", flush=True)
                tune_raar(s.n, s.n, s.m, s.positions, path=args.path, reps=2, iters=2)
            print("tuning the batch as a whole", flush=True)
            tune_batch(scans, path=args.path, verbose=True)
            continue
        if w == "fig3":
            s = gen.fig3_scan()
            print(f"tuning raar {s.name}", flush=True)
            print(tune_raar(s.n, s.n, s.m, s.positions, periodic=True, path=args.path, verbose=True), flush=True)
            continue
        s = gen.config_scan(int(w))
        if int(w) == 4:
            print(f"tuning grad {s.name}", flush=True)
            print(tune_grad(s.n, s.n, s.m, s.positions, path=args.path, verbose=True), flush=True)
        else:
            print(f"tuning raar {s.name}", flush=True)
            print(tune_raar(s.n, s.n, s.m, s.positions, path=args.path, verbose=True), flush=True)


if __name__ == "__main__":
    main()
