"""GPU parity of the individual operators against the FP64 oracle: F, F*, Q,
Q*, P_a, P_Q, the object update, the forward model and the initial probe.
Inputs are complex64; the oracle upcasts the same values.  Tolerances: 1e-5
normwise per projection (relative), 2e-6 for the transforms alone."""
import numpy as np
import pytest

import oracle as O
from helpers import c64, check_close, to_dev, to_host
from sharp_data import gen

pytestmark = pytest.mark.gpu

# (m, K, n): K leaves ragged frame groups (16 frames per group at m = 16, 4 at m = 32)
SIZES = [(16, 19, 40), (32, 7, 64), (64, 3, 100), (128, 2, 160), (256, 2, 280)]


def _crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _plan(n, m, pos, **kw):
    from paper_1602_01448_amd import Plan
    return Plan(n, n, m, pos, **kw)


def _scan(m, K, n, seed=0, periodic=False):
    rng = np.random.default_rng(seed + m)
    if periodic:
        pos = rng.integers(0, n, size=(K, 2)).astype(np.int32)
    else:
        pos = rng.integers(0, n - m + 1, size=(K, 2)).astype(np.int32)
    psi = c64(gen.random_object(rng, n, n))
    w = c64(gen.gaussian_probe(m, m / 5.0) * np.exp(1j * rng.uniform(-1, 1, (m, m))))
    return rng, pos, psi, w


@pytest.mark.parametrize("m,K,n", SIZES)
def test_dft_and_inverse(m, K, n):
    rng, pos, psi, w = _scan(m, K, n)
    p = _plan(n, m, pos)
    z = c64(_crandn(rng, K, m, m))
    F = to_host(p.apply("F", to_dev(z)))
    Fi = to_host(p.apply("FINV", to_dev(z)))
    check_close(F, O.dft(z), 2e-6)
    check_close(Fi, O.idft(z), 2e-6)


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("m,K,n", SIZES)
def test_Q_and_Qstar(m, K, n, periodic):
    rng, pos, psi, w = _scan(m, K, n, periodic=periodic)
    p = _plan(n, m, pos, periodic=periodic)
    p.set_probe(to_dev(w))
    zq = to_host(p.apply("Q", to_dev(psi)))
    check_close(zq, O.Q(psi, w, pos, periodic), 1e-6)
    z = c64(_crandn(rng, K, m, m))
    qs = to_host(p.apply("QSTAR", to_dev(z)))
    check_close(qs, O.Qstar(z, w, pos, (n, n), periodic), 1e-6)


@pytest.mark.parametrize("m,K,n", SIZES)
def test_data_projector(m, K, n):
    rng, pos, psi, w = _scan(m, K, n)
    p = _plan(n, m, pos)
    I = O.forward_intensity(psi, w, pos).astype(np.float32)
    p.set_data(to_dev(I))
    p.set_probe(to_dev(w))
    z = c64(_crandn(rng, K, m, m))
    y = to_host(p.apply("PA", to_dev(z)))
    ref = O.P_a(z, np.sqrt(I.astype(np.float64)))
    check_close(y, ref, 1e-5)


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("m,K,n", SIZES)
def test_overlap_projector_and_object_update(m, K, n, periodic):
    rng, pos, psi, w = _scan(m, K, n, periodic=periodic)
    p = _plan(n, m, pos, periodic=periodic)
    p.set_probe(to_dev(w))
    z = c64(_crandn(rng, K, m, m))
    y = to_host(p.apply("PQ", to_dev(z)))
    check_close(y, O.P_Q(z, w, pos, (n, n), periodic), 1e-5)
    obj = to_host(p.apply("OBJECT", to_dev(z)))
    ref = O.object_update(z, w, pos, (n, n), periodic)
    check_close(obj, ref, 1e-5)
    D = O.illumination_density(w, pos, (n, n), periodic)
    assert np.all(obj[D == 0] == 0)


@pytest.mark.parametrize("tile,split", [(16, 1), (16, 3), (32, 2), (64, 1), (64, 5)])
def test_merge_tilings_agree(tile, split):
    """Every tile size and frame split gives the oracle's P_Q within tolerance."""
    m, K, n = 32, 30, 100
    rng, pos, psi, w = _scan(m, K, n, seed=5)
    p = _plan(n, m, pos, tile=tile, merge_split=split)
    p.set_probe(to_dev(w))
    z = c64(_crandn(rng, K, m, m))
    check_close(to_host(p.apply("PQ", to_dev(z))), O.P_Q(z, w, pos, (n, n)), 1e-5)


@pytest.mark.parametrize("m,K,n", SIZES)
def test_forward_model(m, K, n):
    rng, pos, psi, w = _scan(m, K, n)
    p = _plan(n, m, pos)
    I = to_host(p.simulate(to_dev(psi), to_dev(w)))
    ref = O.forward_intensity(psi, w, pos)
    assert np.linalg.norm(I - ref) / np.linalg.norm(ref) < 1e-5


@pytest.mark.parametrize("m,K,n", SIZES)
def test_initial_probe(m, K, n):
    rng, pos, psi, w = _scan(m, K, n)
    p = _plan(n, m, pos)
    I = O.forward_intensity(psi, w, pos).astype(np.float32)
    p.set_data(to_dev(I))
    p.init_probe()
    got = to_host(p.probe())
    check_close(got, O.init_probe(I.astype(np.float64)), 1e-5)


def test_read_reference_runs():
    """The device read-rate reference (a measurement utility) reads a buffer
    with a ragged tail and leaves one finite float per workgroup."""
    import ctypes

    import torch

    from paper_1602_01448_amd._lib import check, lib
    n = (1 << 20) + 3 * 4   # floats: 4 MiB + 48 bytes, a multiple of 16 bytes
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    sink = torch.full((2048,), float("nan"), dtype=torch.float32, device="cuda")
    check(lib.sharp_read_reference(ctypes.c_void_p(x.data_ptr()), n * 4, ctypes.c_void_p(sink.data_ptr()), None),
          "sharp_read_reference")
    torch.cuda.synchronize()
    s = sink.cpu()
    assert torch.isfinite(s).all()
    assert float(s.sum()) > 0
