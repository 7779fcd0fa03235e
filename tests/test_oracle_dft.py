"""Pins of the oracle's 2-D DFT against the definition in Sec. "Forward model":
(F f)(q) = (1/m) sum_r e^{2 pi i q.r} f(r), q.r = (mu mu' + nu nu')/m."""
import numpy as np
import pytest

import oracle as O


def _crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 8])
def test_dft_brute_force_four_index_sum(rng, m):
    f = _crandn(rng, m, m)
    ref = np.zeros((m, m), dtype=complex)
    for qy in range(m):
        for qx in range(m):
            acc = 0j
            for ry in range(m):
                for rx in range(m):
                    acc += np.exp(2j * np.pi * (qy * ry + qx * rx) / m) * f[ry, rx]
            ref[qy, qx] = acc / m
    assert np.max(np.abs(O.dft(f) - ref)) < 1e-13 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("m", [16, 32, 64])
def test_dft_matrix_form_agrees(rng, m):
    f = _crandn(rng, 3, m, m)
    assert np.linalg.norm(O.dft(f) - O.dft_by_matrix(f)) < 1e-13 * np.linalg.norm(f)


@pytest.mark.parametrize("m,r0", [(8, (0, 1)), (16, (3, 5)), (32, (31, 0))])
def test_dft_of_shifted_delta_closed_form(m, r0):
    """A unit impulse at r0 maps to the plane wave e^{+2 pi i q.r0/m}/m; this
    fixes both the sign of the exponent and the 1/m scale."""
    f = np.zeros((m, m), dtype=complex)
    f[r0] = 1.0
    q = np.arange(m)
    ref = np.exp(2j * np.pi * (q[:, None] * r0[0] + q[None, :] * r0[1]) / m) / m
    assert np.max(np.abs(O.dft(f) - ref)) < 1e-15


def test_dft_of_constant_is_scaled_delta():
    m = 16
    F = O.dft(np.full((m, m), 2.0 + 1.0j))
    ref = np.zeros((m, m), dtype=complex)
    ref[0, 0] = m * (2.0 + 1.0j)
    assert np.max(np.abs(F - ref)) < 1e-13


@pytest.mark.parametrize("m", [16, 64, 256])
def test_parseval_and_unitarity(rng, m):
    f = _crandn(rng, 2, m, m)
    F = O.dft(f)
    assert abs(np.linalg.norm(F) - np.linalg.norm(f)) < 1e-12 * np.linalg.norm(f)
    assert np.linalg.norm(O.idft(F) - f) < 1e-13 * np.linalg.norm(f)


def test_conjugate_twin():
    """|F conj(z)| is |F z| index-reflected: the sign of F matters for data."""
    rng = np.random.default_rng(1)
    z = _crandn(rng, 8, 8)
    A = np.abs(O.dft(z))
    B = np.abs(O.dft(np.conj(z)))
    refl = np.roll(A[::-1, ::-1], 1, axis=(0, 1))
    assert np.max(np.abs(B - refl)) < 1e-13
