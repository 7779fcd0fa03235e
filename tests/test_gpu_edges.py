"""Edge cases of the RAAR path on the GPU against the FP64 oracle:
rectangular objects (nx != ny) for every frame-kernel family and both carry
forms, a single frame, frames at the last valid position, periodic wrap on
rectangular objects, and probe refinement on a rectangular object."""
import numpy as np
import pytest

import oracle as O
from helpers import c64, dweighted, rel, to_dev, to_host
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
                                          (256, 300, 700, 1), (256, 700, 300, 2)])
def test_rectangular_objects(m, ny, nx, form):
    pos = _raster(ny, nx, m, 4, 5)
    p, got, ref, D = _run(ny, nx, m, pos, frame_launch=form, seed=m + ny)
    assert p.info()["frame_launch"] == (form if m >= 128 else 1)
    assert dweighted(got, ref["psi"], D) < 1e-4
    assert np.max(np.abs(p.metrics() - ref["eps_a"]) / ref["eps_a"]) < 1e-4


@pytest.mark.parametrize("m,n", [(16, 16), (32, 48), (128, 128), (256, 256), (256, 300)])
def test_single_frame(m, n):
    """One frame; for n = m it covers the whole object."""
    p, got, ref, D = _run(n, n, m, [(n - m, n - m)], seed=m)
    assert dweighted(got, ref["psi"], D) < 1e-4


@pytest.mark.parametrize("m", [32, 128, 256])
def test_periodic_rectangular(m):
    ny, nx = 2 * m + 24, 3 * m + 40
    rng = np.random.default_rng(m)
    pos = np.stack([rng.integers(0, ny, 12), rng.integers(0, nx, 12)], 1)
    p, got, ref, D = _run(ny, nx, m, pos, periodic=True, seed=m + 1)
    assert dweighted(got, ref["psi"], D) < 1e-4


@pytest.mark.parametrize("m", [64, 128, 256])
def test_probe_refinement_rectangular(m):
    ny, nx = 2 * m + 16, 3 * m
    pos = _raster(ny, nx, m, 4, 6)
    p, got, ref, D = _run(ny, nx, m, pos, probe_every=1, seed=m + 2)
    assert rel(to_host(p.probe()), ref["w"]) < 1e-4
    assert dweighted(got, ref["psi"], D) < 1e-4
