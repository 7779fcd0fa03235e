"""Edge cases of the RAAR path on the GPU against the FP64 oracle:
an all-zero frame in the data projector (sgn(0) := 1), negative intensities,
the illumination threshold eps_D,
rectangular objects (nx != ny) for every frame-kernel family and both carry
forms, a single frame, frames at the last valid position, periodic wrap on
rectangular objects, and probe refinement on a rectangular object."""
import numpy as np
import pytest

import oracle as O
from helpers import c64, check_close, check_object, to_dev, to_host
from sharp_data import gen

pytestmark = pytest.mark.gpu


def _run(ny, nx, m, pos, n_iter=3, periodic=False, probe_every=0, seed=0, **kw):
    from paper_1602_01448_amd import Plan
    rng = np.random.default_rng(seed)
    obj = (rng.uniform(0.5, 1.0, (ny, nx)) * np.exp(1j * rng.uniform(-1.5, 1.5, (ny, nx))))
    probe = gen.gaussian_probe(m, m / 5)
    psi0 = rng.uniform(0, 1, (ny, nx)).astype(complex)
    pos = np.asarray(pos, np.int32)
    I = O.forward_intensity(obj, probe, pos, periodic).astype(np.float32)
    p = Plan(nx, ny, m, pos, periodic=periodic, probe_every=probe_every, **kw)
    p.set_data(to_dev(I)).set_probe(to_dev(c64(probe))).set_object(to_dev(c64(psi0))).raar(n_iter, 0.75)
    ref = O.raar(I.astype(np.float64), pos, (ny, nx), m, n_iter, 0.75, psi0=psi0, w0=probe,
                 probe_every=probe_every, periodic=periodic)
    D = O.illumination_density(ref["w"], pos, (ny, nx), periodic)
    got = to_host(p.object())
    assert got.shape == (ny, nx)
    return p, got, ref, D


def _raster(ny, nx, m, gy, gx):
    ys = np.linspace(0, ny - m, gy).round().astype(int)
    xs = np.linspace(0, nx - m, gx).round().astype(int)
    return [(y, x) for y in ys for x in xs]


@pytest.mark.parametrize("m,ny,nx,form", [(32, 96, 160, 1), (64, 320, 192, 1), (128, 200, 352, 1), (128, 352, 200, 2),
                                          (256, 300, 700, 1), (256, 700, 300, 2), (256, 300, 700, 3),
                                          (256, 700, 300, 3)])
def test_rectangular_objects(m, ny, nx, form):
    pos = _raster(ny, nx, m, 4, 5)
    p, got, ref, D = _run(ny, nx, m, pos, frame_launch=form, seed=m + ny)
    assert p.info()["frame_launch"] == (form if m >= 128 else 1)
    check_object(got, ref["psi"], D, 1e-4)
    assert np.max(np.abs(p.metrics() - ref["eps_a"]) / ref["eps_a"]) < 1e-4


@pytest.mark.parametrize("m,n,form", [(16, 16, 0), (32, 48, 0), (128, 128, 0), (256, 256, 0), (256, 300, 0),
                                      (256, 256, 3), (256, 300, 3)])
def test_single_frame(m, n, form):
    """One frame; for n = m it covers the whole object."""
    p, got, ref, D = _run(n, n, m, [(n - m, n - m)], seed=m, frame_launch=form)
    check_object(got, ref["psi"], D, 1e-4)


@pytest.mark.parametrize("m,form", [(32, 0), (128, 0), (256, 0), (256, 3)])
def test_periodic_rectangular(m, form):
    ny, nx = 2 * m + 24, 3 * m + 40
    rng = np.random.default_rng(m)
    pos = np.stack([rng.integers(0, ny, 12), rng.integers(0, nx, 12)], 1)
    p, got, ref, D = _run(ny, nx, m, pos, periodic=True, seed=m + 1, frame_launch=form)
    check_object(got, ref["psi"], D, 1e-4)


@pytest.mark.parametrize("m,form", [(64, 0), (128, 0), (256, 0), (256, 3)])
def test_probe_refinement_rectangular(m, form):
    ny, nx = 2 * m + 16, 3 * m
    pos = _raster(ny, nx, m, 4, 6)
    p, got, ref, D = _run(ny, nx, m, pos, probe_every=1, seed=m + 2, frame_launch=form)
    check_close(to_host(p.probe()), ref["w"], 1e-4)
    check_object(got, ref["psi"], D, 1e-4)


def _frames_case(m, seed, negative=False):
    rng = np.random.default_rng(seed)
    n, K = 2 * m + 24, 4
    pos = rng.integers(0, n - m + 1, size=(K, 2)).astype(np.int32)
    obj = gen.random_object(rng, n, n)
    probe = gen.gaussian_probe(m, m / 5)
    I = O.forward_intensity(obj, probe, pos)
    if negative:
        # a background subtraction gone too far: about a fifth of the entries < 0
        I = I - np.quantile(I, 0.2)
    z = rng.standard_normal((K, m, m)) + 1j * rng.standard_normal((K, m, m))
    return rng, n, pos, c64(probe), I.astype(np.float32), c64(z), c64(obj)


@pytest.mark.parametrize("m", [16, 32, 64, 128, 256])
def test_data_projector_of_an_all_zero_frame(m):
    """P_a of a frame that is exactly zero: F z = 0 in every bin, sgn(0) := 1
    (reading R2), so P_a z = F* a for that frame (closed form), and the other
    frames are unaffected."""
    from paper_1602_01448_amd import Plan
    rng, n, pos, w, I, z, _ = _frames_case(m, 300 + m)
    z[1] = 0
    p = Plan(n, n, m, pos)
    p.set_data(to_dev(I)).set_probe(to_dev(w))
    y = to_host(p.apply("PA", to_dev(z)))
    a = np.sqrt(I.astype(np.float64))
    check_close(y, O.P_a(z, a), 1e-5, where=f"m={m}")
    check_close(y[1], O.idft(a[1]), 1e-5, where=f"m={m} zero frame")


@pytest.mark.parametrize("m,form", [(32, 0), (128, 0), (256, 0), (256, 3)])
def test_negative_intensities_are_clamped(m, form):
    """Intensities below zero enter as amplitude 0 (a = sqrt(max(I, 0)),
    Sec. "Forward model"): the data projector and the eps_a history (whose
    norm ||a|| uses the clamped values) match the oracle."""
    from paper_1602_01448_amd import Plan
    rng, n, pos, w, I, z, obj = _frames_case(m, 310 + m, negative=True)
    assert (I < 0).mean() > 0.1
    a = np.sqrt(np.maximum(I.astype(np.float64), 0.0))
    p = Plan(n, n, m, pos, frame_launch=form)
    p.set_data(to_dev(I)).set_probe(to_dev(w))
    check_close(to_host(p.apply("PA", to_dev(z))), O.P_a(z, a), 1e-5, where=f"m={m}")
    psi0 = c64(rng.uniform(0, 1, (n, n)))
    p.set_object(to_dev(psi0)).raar(3, 0.75)
    ref = O.raar(I.astype(np.float64), pos, (n, n), m, 3, 0.75, psi0=psi0, w0=w)
    assert np.max(np.abs(p.metrics() - ref["eps_a"]) / ref["eps_a"]) < 1e-4
    D = O.illumination_density(w, pos, (n, n))
    check_object(to_host(p.object()), ref["psi"], D, 1e-4, where=f"m={m}")


def _threshold_between(D, q=0.3):
    """A float32 threshold strictly between two illumination values near the
    q-quantile of the covered pixels, at least 1e-4 (relative) from every D,
    so that FP32 (GPU) and FP64 (oracle) sort every pixel the same way."""
    v = np.unique(D[D > 0])
    k = int(q * len(v))
    for j in range(k, len(v) - 1):
        if v[j + 1] > v[j] * (1 + 1e-3):
            eps = float(np.float32(np.sqrt(v[j] * v[j + 1])))
            assert np.min(np.abs(D - eps)) > 1e-4 * eps
            return eps
    raise AssertionError("no gap found")


@pytest.mark.parametrize("m,form", [(32, 0), (128, 0), (256, 0), (256, 3)])
def test_density_threshold(m, form):
    """Option eps_D > 0: (Q*Q)^{-1} is 1/D only where D > eps_D (reading R3);
    the object update and a RAAR run match the oracle with the same
    threshold, and the pixels at or below it stay exactly 0."""
    from paper_1602_01448_amd import Plan
    rng, n, pos, w, I, z, obj = _frames_case(m, 320 + m)
    D = O.illumination_density(w, pos, (n, n))
    eps = _threshold_between(D)
    assert 0.1 < np.mean(D[D > 0] <= eps) < 0.6
    p = Plan(n, n, m, pos, eps_D=eps, frame_launch=form)
    p.set_data(to_dev(I)).set_probe(to_dev(w))
    got = to_host(p.apply("OBJECT", to_dev(z)))
    check_close(got, O.object_update(z, w, pos, (n, n), eps_D=eps), 1e-5, where=f"m={m}")
    assert np.all(got[D <= eps] == 0)
    check_close(to_host(p.apply("PQ", to_dev(z))), O.P_Q(z, w, pos, (n, n), eps_D=eps), 1e-5, where=f"m={m}")
    psi0 = c64(rng.uniform(0, 1, (n, n)))
    p.set_object(to_dev(psi0)).raar(4, 0.75)
    ref = O.raar(I.astype(np.float64), pos, (n, n), m, 4, 0.75, psi0=psi0, w0=w, eps_D=eps)
    Dw = np.where(D > eps, D, 0.0)
    check_object(to_host(p.object()), ref["psi"], Dw, 1e-4, where=f"m={m}")
    assert np.max(np.abs(p.metrics() - ref["eps_a"]) / ref["eps_a"]) < 1e-4
