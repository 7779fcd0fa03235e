"""Batched execution of independent scans of uneven sizes: every scan of a
batch must reproduce its single-scan run bit for bit (same kernels, same
summation order), and one scan is checked against the FP64 oracle."""
import numpy as np
import pytest

import oracle as O
from helpers import c64, check_object, to_dev, to_host
from sharp_data import gen

pytestmark = pytest.mark.gpu


def _small_scans():
    """Uneven scans covering every frame-size class."""
    out = []
    for j, (n, m, g) in enumerate([(96, 16, 7), (150, 32, 9), (200, 64, 6), (300, 128, 5), (400, 256, 3),
                                   (260, 64, 11), (180, 32, 4)]):
        rng = np.random.default_rng(100 + j)
        pos = gen.raster_positions(g, (n - m) / max(g - 1, 1), n, m, jitter=2, rng=rng)
        out.append(gen.Scan(f"s{j}", n, m, pos, gen.random_object(rng, n, n), gen.gaussian_probe(m, 6.0 * m / 32),
                            rng.uniform(0, 1, (n, n)).astype(complex), None, 0.75, 5, 0, 1, False, None))
    return out


def _plan(s, I, **kw):
    from paper_1602_01448_amd import Plan
    p = Plan(s.n, s.n, s.m, s.positions, **kw)
    p.set_data(to_dev(I)).set_probe(to_dev(c64(s.probe))).set_object(to_dev(c64(s.psi0)))
    return p


def _data(s):
    return O.forward_intensity(s.obj, s.probe, s.positions).astype(np.float32)


def test_batch_equals_single_scans_bitwise():
    from paper_1602_01448_amd import Batch
    scans = _small_scans()
    data = [_data(s) for s in scans]
    single = [_plan(s, I) for s, I in zip(scans, data)]
    for p in single:
        p.raar(4, 0.75).raar(3, 0.9)
    batched = [_plan(s, I) for s, I in zip(scans, data)]
    b = Batch(batched)
    b.raar(4, 0.75).raar(3, 0.9)
    for s, p, q in zip(scans, single, batched):
        assert np.array_equal(to_host(p.object()), to_host(q.object())), s.name
        assert np.array_equal(p.metrics(), q.metrics()), s.name
    # graph replay: a second call with the same (n, beta) continues the runs
    for p in single:
        p.raar(4, 0.75)
    b.raar(4, 0.75)
    for s, p, q in zip(scans, single, batched):
        assert np.array_equal(to_host(p.object()), to_host(q.object())), s.name
        assert q.info()["iteration"] == 11


def test_batch_matches_oracle():
    from paper_1602_01448_amd import Batch
    scans = _small_scans()[:4]
    data = [_data(s) for s in scans]
    plans = [_plan(s, I) for s, I in zip(scans, data)]
    Batch(plans).raar(5, 0.75)
    for s, I, p in zip(scans, data, plans):
        ref = O.raar(I.astype(np.float64), s.positions, (s.n, s.n), s.m, 5, 0.75, psi0=c64(s.psi0),
                     w0=c64(s.probe))
        D = O.illumination_density(s.probe, s.positions, (s.n, s.n))
        check_object(to_host(p.object()), ref["psi"], D, 1e-4, where=s.name)


def test_batch_full_size_uneven_scans_bitwise():
    """The 32 uneven scans of the batching workload (n 256..1024, m in
    {64, 128, 256}, 100..1500 frames), two iterations: batched = single."""
    import torch

    from paper_1602_01448_amd import Batch, Plan
    scans = gen.batch_scans()
    single, batched = [], []
    for s in scans:
        obj = to_dev(c64(s.obj))
        w = to_dev(c64(s.probe))
        for lst in (single, batched):
            p = Plan(s.n, s.n, s.m, s.positions)
            I = p.simulate(obj, w)
            p.set_data(I).set_probe(w).set_object(to_dev(c64(s.psi0)))
            lst.append(p)
    for p in single:
        p.raar(2, 0.75)
    Batch(batched).raar(2, 0.75)
    torch.cuda.synchronize()
    for s, p, q in zip(scans, single, batched):
        assert np.array_equal(to_host(p.object()), to_host(q.object())), s.name


def test_batch_streaming_scan_bitwise():
    """A 128^2 scan whose frame arrays exceed the last-level cache (streaming
    accesses) next to a small one: batched = single, bit for bit."""
    import torch

    from paper_1602_01448_amd import Batch, Plan
    rng = np.random.default_rng(7)
    n, m = 128 + 45 * 10, 128
    big = gen.Scan("big", n, m, gen.raster_positions(46, 10, n, m, jitter=2, rng=rng), gen.random_object(rng, n, n),
                   gen.gaussian_probe(m, 24.0), rng.uniform(0, 1, (n, n)).astype(complex), None, 0.75, 3, 0, 1,
                   False, None)
    scans = [big, _small_scans()[3]]
    single, batched = [], []
    for s in scans:
        obj, w = to_dev(c64(s.obj)), to_dev(c64(s.probe))
        for lst in (single, batched):
            p = Plan(s.n, s.n, s.m, s.positions)
            p.set_data(p.simulate(obj, w)).set_probe(w).set_object(to_dev(c64(s.psi0)))
            lst.append(p)
    assert [p.info()["streaming"] for p in single] == [1, 0]
    for p in single:
        p.raar(3, 0.75)
    Batch(batched).raar(3, 0.75)
    torch.cuda.synchronize()
    for s, p, q in zip(scans, single, batched):
        assert np.array_equal(to_host(p.object()), to_host(q.object())), s.name
        assert np.array_equal(p.metrics(), q.metrics()), s.name


def test_batch_rejects_probe_refinement_and_unready_plans():
    from paper_1602_01448_amd import Batch, Plan, SharpError
    s = _small_scans()[1]
    p = Plan(s.n, s.n, s.m, s.positions, probe_every=1)
    p.set_data(to_dev(_data(s))).set_probe(to_dev(c64(s.probe))).set_object(to_dev(c64(s.psi0)))
    with pytest.raises(SharpError):
        Batch([p])

    q = Plan(s.n, s.n, s.m, s.positions)
    with pytest.raises(SharpError):
        Batch([q])


def test_batch_refuses_a_plan_moved_to_another_workspace():
    """A member plan given a new workspace after the batch took its pointers:
    the batch returns NOT_READY without launching, and runs again, equal to
    the single-scan run bit for bit, once its workspace is set again."""
    import ctypes

    import torch
    from paper_1602_01448_amd import Batch, SharpError
    from paper_1602_01448_amd._lib import check, lib
    scans = _small_scans()[:3]
    data = [_data(s) for s in scans]
    plans = [_plan(s, I) for s, I in zip(scans, data)]
    b = Batch(plans)
    b.raar(2, 0.75)
    p = plans[1]
    nbytes = lib.sharp_workspace_bytes(p.handle)
    p.workspace = torch.empty(nbytes, dtype=torch.uint8, device=p.device)
    check(lib.sharp_set_workspace(p.handle, ctypes.c_void_p(p.workspace.data_ptr()), nbytes), "ws")
    p.set_data(to_dev(data[1])).set_probe(to_dev(c64(scans[1].probe))).set_object(to_dev(c64(scans[1].psi0)))
    before = [to_host(q.object()) for q in plans]
    with pytest.raises(SharpError) as e:
        b.raar(1, 0.75)
    assert e.value.status == -4
    torch.cuda.synchronize()
    assert all(np.array_equal(to_host(q.object()), x) for q, x in zip(plans, before))
    check(lib.sharp_batch_set_workspace(b._h, ctypes.c_void_p(b.workspace.data_ptr()), b.workspace.numel()), "bws")
    b.raar(3, 0.75)
    single = _plan(scans[1], data[1]).raar(3, 0.75)
    assert np.array_equal(to_host(single.object()), to_host(p.object()))


def test_batch_large_frame_forms_bitwise():
    """m = 256 scans in both Fourier-carry forms (form 3: column pass with its
    own row transform) batched with smaller scans: batched = single, bit for
    bit, and the form-3 scan against the oracle."""
    from paper_1602_01448_amd import Batch
    scans = _small_scans()
    rng = np.random.default_rng(808)
    n, m = 448, 256
    big = gen.Scan("f3", n, m, gen.raster_positions(4, 64.0, n, m, jitter=2, rng=rng), gen.random_object(rng, n, n),
                   gen.gaussian_probe(m, 48.0), rng.uniform(0, 1, (n, n)).astype(complex), None, 0.75, 3, 0, 1,
                   False, None)
    cases = [(scans[4], 3), (big, 3), (big, 2), (scans[1], 0), (scans[3], 0)]
    data = [_data(s) for s, _ in cases]
    single = [_plan(s, I, frame_launch=f) for (s, f), I in zip(cases, data)]
    batched = [_plan(s, I, frame_launch=f) for (s, f), I in zip(cases, data)]
    assert [p.info()["frame_launch"] for p in single[:3]] == [3, 3, 2]
    for p in single:
        p.raar(3, 0.75)
    Batch(batched).raar(3, 0.75)
    for (s, f), p, q in zip(cases, single, batched):
        assert np.array_equal(to_host(p.object()), to_host(q.object())), (s.name, f)
        assert np.array_equal(p.metrics(), q.metrics()), (s.name, f)
    ref = O.raar(data[1].astype(np.float64), big.positions, (n, n), m, 3, 0.75, psi0=c64(big.psi0), w0=c64(big.probe))
    D = O.illumination_density(big.probe, big.positions, (n, n))
    check_object(to_host(batched[1].object()), ref["psi"], D, 1e-4)
