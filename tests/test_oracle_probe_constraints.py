"""Pins of the oracle's probe constraints and centre-of-mass correction
(algorithm box, step 7; readings R14, R15) against closed forms, a
brute-force DFT and invariances -- not against the oracle's own formulas."""
import numpy as np
import pytest

import oracle as O


def _brute_dft(w):
    """(F w)[k] = (1/m) sum_r exp(+2 pi i k.r / m) w[r], summed term by term."""
    m = w.shape[0]
    out = np.zeros((m, m), complex)
    for ky in range(m):
        for kx in range(m):
            s = 0j
            for y in range(m):
                for x in range(m):
                    s += np.exp(2j * np.pi * (ky * y + kx * x) / m) * w[y, x]
            out[ky, kx] = s / m
    return out


def _probe(m, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))


def test_all_ones_mask_is_identity():
    w = _probe(8)
    assert np.allclose(O.probe_fourier_constraint(w, mask=np.ones((8, 8))), w, atol=1e-13)


def test_dc_only_mask_gives_the_mean():
    """Keeping only the DC bin leaves the constant mean of w (closed form)."""
    w = _probe(8, 1)
    mask = np.zeros((8, 8))
    mask[0, 0] = 1.0
    out = O.probe_fourier_constraint(w, mask=mask)
    assert np.allclose(out, np.full((8, 8), w.mean()), atol=1e-13)


def test_mask_multiplies_the_spectrum():
    w = _probe(6, 2)
    mask = (np.random.default_rng(3).uniform(size=(6, 6)) > 0.4).astype(float)
    out = O.probe_fourier_constraint(w, mask=mask)
    assert np.allclose(_brute_dft(out), _brute_dft(w) * mask, atol=1e-12)


def test_amplitude_constraint_sets_magnitudes_keeps_phases():
    w = _probe(6, 4)
    amp = np.random.default_rng(5).uniform(0.5, 2.0, size=(6, 6))
    out = O.probe_fourier_constraint(w, amplitudes=amp)
    Fo, Fw = _brute_dft(out), _brute_dft(w)
    assert np.allclose(np.abs(Fo), amp, atol=1e-12)
    assert np.allclose(Fo / np.abs(Fo), Fw / np.abs(Fw), atol=1e-12)


def test_mask_takes_precedence_over_amplitudes():
    w = _probe(6, 6)
    mask = np.ones((6, 6))
    out = O.probe_fourier_constraint(w, mask=mask, amplitudes=np.full((6, 6), 3.0))
    assert np.allclose(out, w, atol=1e-13)


@pytest.mark.parametrize("p,q", [(0, 0), (3, 13), (15, 1), (8, 8)])
def test_center_moves_a_delta_to_the_frame_centre(p, q):
    m = 16
    w = np.zeros((m, m), complex)
    w[p, q] = 2.0 - 1.0j
    out = O.probe_center(w)
    expect = np.zeros((m, m), complex)
    expect[m // 2, m // 2] = 2.0 - 1.0j
    assert np.array_equal(out, expect)


def test_center_shift_of_an_offset_gaussian():
    m = 64
    y, x = np.mgrid[0:m, 0:m]
    g = np.exp(-((y - 35.0) ** 2 + (x - 27.0) ** 2) / (2 * 4.0 ** 2)) * np.exp(1j * 0.3 * x)
    assert O.probe_center_shift(g) == (-3, 5)
    out = O.probe_center(g)
    yy, xx = np.mgrid[0:m, 0:m]
    p = np.abs(out) ** 2
    assert abs((p * yy).sum() / p.sum() - 32) < 0.5 and abs((p * xx).sum() / p.sum() - 32) < 0.5


def test_center_rounds_half_up():
    """Centroid exactly half a pixel before the centre: shifted by +1."""
    m = 16
    w = np.zeros((m, m), complex)
    w[7, 8] = w[8, 8] = 1.0          # centroid y = 7.5
    assert O.probe_center_shift(w) == (1, 0)


def test_center_is_invariant_to_a_prior_roll():
    m = 32
    y, x = np.mgrid[0:m, 0:m]
    g = np.exp(-((y - 13.0) ** 2 + (x - 20.0) ** 2) / (2 * 3.0 ** 2)).astype(complex)
    assert np.array_equal(O.probe_center(g), O.probe_center(np.roll(g, (2, -3), axis=(0, 1))))


def _scan():
    from sharp_data import gen
    rng = np.random.default_rng(77)
    n, m = 64, 16
    pos = gen.raster_positions(7, 8.0, n, m, jitter=0, rng=rng)
    obj = gen.random_object(rng, n, n)
    probe = gen.gaussian_probe(m, 3.0)
    I = O.forward_intensity(obj, probe, pos)
    psi0 = rng.uniform(0, 1, (n, n)).astype(complex)
    return n, m, pos, probe, I, psi0


def test_raar_with_unit_mask_equals_unconstrained():
    n, m, pos, probe, I, psi0 = _scan()
    a = O.raar(I, pos, (n, n), m, 4, 0.75, psi0=psi0, probe_every=1)
    b = O.raar(I, pos, (n, n), m, 4, 0.75, psi0=psi0, probe_every=1, probe_mask=np.ones((m, m)))
    assert np.allclose(a["psi"], b["psi"], atol=1e-12) and np.allclose(a["w"], b["w"], atol=1e-12)


def test_raar_amplitude_constraint_holds_after_updates():
    n, m, pos, probe, I, psi0 = _scan()
    amp = np.abs(_brute_dft(probe))
    r = O.raar(I, pos, (n, n), m, 3, 0.75, psi0=psi0, probe_every=1, probe_amplitudes=amp)
    assert np.allclose(np.abs(_brute_dft(r["w"])), amp, atol=1e-10)


def test_raar_centering_keeps_the_probe_centred():
    n, m, pos, probe, I, psi0 = _scan()
    r = O.raar(I, pos, (n, n), m, 3, 0.75, psi0=psi0, probe_every=1, probe_center_com=True)
    p = np.abs(r["w"]) ** 2
    yy, xx = np.mgrid[0:m, 0:m]
    assert abs((p * yy).sum() / p.sum() - m // 2) <= 0.5 and abs((p * xx).sum() / p.sum() - m // 2) <= 0.5


@pytest.mark.parametrize("p,q", [(0, 0), (3, 13), (15, 1)])
def test_centroid_of_a_delta_is_its_pixel(p, q):
    w = np.zeros((16, 16), complex)
    w[p, q] = 0.5j
    assert O.probe_centroid(w) == (float(p), float(q))
    assert O.probe_centroid(np.zeros((16, 16), complex)) is None


@pytest.mark.parametrize("delta,shift", [(1e-9, 1), (-1e-9, 0)])
def test_center_decides_a_near_tie_in_double_precision(delta, shift):
    """|w|^2 = 1 + delta at row 7 and 1 at row 8: the centroid is
    7.5 - delta / (2 (2 + delta)), so the roll is 1 for delta > 0 and 0 for
    delta < 0.  A single-precision sum (1 + 1e-9 rounds to 1) would see the
    exact tie and take 1 both times."""
    m = 16
    w = np.zeros((m, m), complex)
    w[7, 8] = np.sqrt(1.0 + delta)
    w[8, 8] = 1.0
    assert O.probe_center_shift(w) == (shift, 0)


def test_raar_records_the_centroids_it_corrects():
    n, m, pos, probe, I, psi0 = _scan()
    trace = []
    O.raar(I, pos, (n, n), m, 3, 0.75, psi0=psi0, probe_every=1, probe_center_com=True, trace=trace)
    assert len(trace) == 3 and all(len(c) == 2 for c in trace)
