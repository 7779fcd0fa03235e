"""Probe constraints of the probe update (algorithm box, step 7): Fourier
mask, Fourier amplitudes and the centre-of-mass correction, on the GPU
against the FP64 oracle, for every frame-kernel family (m = 64 frame-space
kernel, m = 128 register-resident kernel, m = 256 column/strip passes)."""
import numpy as np
import pytest

import oracle as O
from helpers import c64, check_close, check_object, to_dev, to_host
from sharp_data import gen

pytestmark = pytest.mark.gpu

GEOM = {64: (192, 5, 32.0), 128: (320, 4, 64.0), 256: (512, 3, 128.0)}


def _offset_gaussian(m, c, sigma):
    y, x = np.mgrid[0:m, 0:m]
    return np.exp(-((y - c) ** 2 + (x - c) ** 2) / (2 * sigma ** 2)).astype(complex)


def _setup(m, seed, center_offset=None):
    n, g, step = GEOM[m]
    rng = np.random.default_rng(seed)
    pos = gen.raster_positions(g, step, n, m, jitter=2, rng=rng)
    obj = gen.random_object(rng, n, n)
    if center_offset is None:
        probe = gen.gaussian_probe(m, m / 5)
    else:
        probe = _offset_gaussian(m, m / 2 + center_offset, m / 5)
    I = O.forward_intensity(obj, probe, pos)
    psi0 = rng.uniform(0, 1, (n, n)).astype(complex)
    return n, pos, probe, I, psi0


def _lowpass(m):
    f = np.fft.fftfreq(m) * m
    return (np.hypot(f[:, None], f[None, :]) < m / 4).astype(np.float64)


def _run(m, n, pos, I, psi0, w0, n_iter, form=0, **kw):
    from paper_1602_01448_amd import Plan
    center = kw.pop("center", False)
    p = Plan(n, n, m, pos, probe_every=1, probe_center=center, frame_launch=form)
    p.set_data(to_dev(I.astype(np.float32))).set_probe(to_dev(c64(w0)))
    if "mask" in kw:
        p.set_probe_constraint(mask=to_dev(kw["mask"].astype(np.float32)))
    if "amplitudes" in kw:
        p.set_probe_constraint(amplitudes=to_dev(kw["amplitudes"].astype(np.float32)))
    p.set_object(to_dev(c64(psi0))).raar(n_iter, 0.75)
    return to_host(p.object()), to_host(p.probe())


@pytest.mark.parametrize("m,form", [(64, 0), (128, 0), (256, 0), (256, 3)])
@pytest.mark.parametrize("kind", ["mask", "amplitudes", "center"])
def test_probe_constraint_matches_oracle(m, form, kind):
    # centre-of-mass case: a probe centred a quarter pixel off the frame
    # centre, so that the corrected centroids stay clear of the half-pixel
    # ties at m/2 +- 1/2 (checked below)
    n, pos, probe, I, psi0 = _setup(m, 60 + m, 0.25 if kind == "center" else None)
    w0 = probe * 1.1
    kw, okw = {}, {}
    if kind == "mask":
        kw["mask"] = okw["probe_mask"] = _lowpass(m)
    elif kind == "amplitudes":
        kw["amplitudes"] = okw["probe_amplitudes"] = np.abs(O.dft(probe))
    else:
        w0 = np.roll(probe, (5, -6), axis=(0, 1))   # the first update moves it back
        kw["center"] = okw["probe_center_com"] = True
    I32 = I.astype(np.float32).astype(np.float64)
    trace = []
    ref = O.raar(I32, pos, (n, n), m, 3, 0.75, psi0=c64(psi0), w0=c64(w0), probe_every=1, trace=trace, **okw)
    if kind == "center":
        # the GPU decides the roll from single-precision sums: every centroid the
        # oracle corrects must sit well away from a half-pixel tie, so that both
        # sides take the same integer
        assert len(trace) == 3
        for c in trace:
            for v in c:
                f = (m // 2 - v + 0.5) % 1.0
                assert min(f, 1.0 - f) >= 0.05, (m, c)
    psi, w = _run(m, n, pos, I, psi0, w0, 3, form, **kw)
    D = O.illumination_density(ref["w"], pos, (n, n))
    check_close(w, ref["w"], 1e-4)
    check_object(psi, ref["psi"], D, 1e-4)
    if kind == "center":
        pw = np.abs(w) ** 2
        yy, xx = np.mgrid[0:m, 0:m]
        assert abs((pw * yy).sum() / pw.sum() - m // 2) <= 0.5 and abs((pw * xx).sum() / pw.sum() - m // 2) <= 0.5
