"""Pins of the oracle's RAAR iteration (algorithm box, step 5, with the
relaxed-averaged-alternating-reflections sign) and of the full reconstruction
sequence."""
import numpy as np

import oracle as O
from sharp_data import gen


def _crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _setup(rng, n=40, m=16, step=8, periodic=False):
    pos = (np.array([(step * j, step * k) for j in range(n // step) for k in range(n // step)], np.int32)
           if periodic else gen.raster_positions((n - m) // step + 1, step, n, m))
    w = gen.gaussian_probe(m, m / 5.0)
    psi = gen.random_object(rng, n, n)
    return pos, w, psi


def test_identity_data_projector_closed_form(rng):
    """With P_a replaced by I the map is (1 - beta) I + beta P_Q: the range(Q)
    part of z is kept and the rest shrinks by (1 - beta) per step.  The
    printed sign beta(P_Q - I) would instead grow it by |1 - 3 beta|."""
    pos, w, _ = _setup(rng)
    n = 40
    z0 = _crandn(rng, len(pos), 16, 16)
    PQ = lambda v: O.P_Q(v, w, pos, (n, n))  # noqa: E731
    beta, L = 0.75, 12
    z = z0
    for _ in range(L):
        z = O.raar_step(z, beta, lambda v: v, PQ)
    p = PQ(z0)
    ref = p + (1 - beta) ** L * (z0 - p)
    assert np.linalg.norm(z - ref) < 1e-12 * np.linalg.norm(z0)
    assert np.linalg.norm(z0 - p) > 0.1 * np.linalg.norm(z0)


def test_beta_one_is_douglas_rachford(rng):
    pos, w, psi = _setup(rng)
    n = 40
    a = np.sqrt(O.forward_intensity(psi, w, pos))
    z = _crandn(rng, len(pos), 16, 16)
    Pa = lambda v: O.P_a(v, a)  # noqa: E731
    PQ = lambda v: O.P_Q(v, w, pos, (n, n))  # noqa: E731
    Ra = 2 * Pa(z) - z
    dr = 0.5 * ((2 * PQ(Ra) - Ra) + z)
    assert np.linalg.norm(O.raar_step(z, 1.0, Pa, PQ) - dr) < 1e-12 * np.linalg.norm(z)


def test_truth_is_a_fixed_point(rng):
    pos, w, psi = _setup(rng)
    n = 40
    a = np.sqrt(O.forward_intensity(psi, w, pos))
    z = O.Q(psi, w, pos)
    z1 = O.raar_step(z, 0.75, lambda v: O.P_a(v, a), lambda v: O.P_Q(v, w, pos, (n, n)))
    assert np.linalg.norm(z1 - z) < 1e-13 * np.linalg.norm(z)


def test_converges_to_zero_fourier_error_periodic(rng):
    """Noiseless consistent data, periodic boundaries, known probe, random
    start: the Fourier error goes to zero and the object is recovered up to
    a global phase."""
    n, m, s = 32, 16, 4
    pos = np.array([(s * j, s * k) for j in range(n // s) for k in range(n // s)], np.int32)
    w = gen.gaussian_probe(m, m / 5.0)
    psi = gen.random_object(np.random.default_rng(0), n, n)
    I = O.forward_intensity(psi, w, pos, periodic=True)
    start = np.random.default_rng(1).uniform(0, 1, (n, n)).astype(complex)
    out = O.raar(I, pos, (n, n), m, 400, 0.75, psi0=start, w0=w, periodic=True)
    e = out["eps_a"]
    assert e[0] > 0.3
    assert e[-1] < 2e-4
    z0 = O.Q(psi, w, pos, periodic=True)
    assert O.eps_0(out["z"], z0, w, pos, (n, n), periodic=True) < 1e-3


def test_near_truth_start_decreases(rng):
    pos, w, psi = _setup(rng)
    n = 40
    I = O.forward_intensity(psi, w, pos)
    start = psi * (1 + 0.1 * _crandn(np.random.default_rng(3), n, n))
    out = O.raar(I, pos, (n, n), 16, 60, 0.75, psi0=start, w0=w, record_extra=True)
    e = out["eps_a"]
    assert e[-1] < 0.2 * e[0]
    assert np.all(out["eps_Q"] >= 0) and np.all(out["eps_Delta"] >= 0)


def test_probe_refinement_keeps_consistent_truth(rng):
    """Start at the true object and probe with noiseless data: the object
    update returns psi and the probe update returns w every iteration."""
    pos, w, psi = _setup(rng)
    n = 40
    w = w * np.exp(1j * 0.2 * np.arange(16)[None, :])
    I = O.forward_intensity(psi, w, pos)
    out = O.raar(I, pos, (n, n), 16, 4, 0.75, psi0=psi, w0=w, probe_every=1)
    assert np.max(np.abs(out["w"] - w)) < 1e-11
    D = O.illumination_density(w, pos, (n, n))
    assert np.max(np.abs(out["psi"] - psi)[D > 0]) < 1e-11


def test_printed_sign_diverges(rng):
    """Reading R1 evidence: the operator as printed grows the component off
    range(Q) by |1 - 3 beta| per step when P_a = I."""
    pos, w, _ = _setup(rng)
    n = 40
    z0 = _crandn(rng, len(pos), 16, 16)
    PQ = lambda v: O.P_Q(v, w, pos, (n, n))  # noqa: E731
    z = z0
    beta = 0.75
    for _ in range(20):
        z = 2 * beta * PQ(z) + (1 - 2 * beta) * z + beta * (PQ(z) - z)
    assert np.linalg.norm(z) > 50 * np.linalg.norm(z0)
