"""Pins of the oracle's amplitude-loss gradient: central finite differences
(h = 1e-3), PyTorch float64 autograd on an independent formulation, the
zero at the noiseless truth and the error-reduction identity."""
import numpy as np
import pytest

import oracle as O
from sharp_data import gen


@pytest.fixture(scope="module")
def sub():
    s = gen.config_scan("4s")
    a = np.sqrt(O.forward_intensity(s.obj, s.probe, s.positions))
    psi, w = gen.gradient_point(s)
    return s, a, psi, w


def test_central_finite_differences(sub):
    s, a, psi, w = sub
    L, gpsi, gw = O.amplitude_grad(psi, w, s.positions, a)
    h = 1e-3
    rng = np.random.default_rng(7)
    errs = []
    for which, arr, g in (("psi", psi, gpsi), ("w", w, gw)):
        for _ in range(6):
            idx = tuple(int(rng.integers(0, d)) for d in arr.shape)
            for unit in (1.0, 1.0j):
                def f(t):
                    p, q = psi.copy(), w.copy()
                    (p if which == "psi" else q)[idx] += t * unit
                    return O.amplitude_loss(p, q, s.positions, a)
                fd = (f(h) - f(-h)) / (2 * h)
                an = (g[idx] * np.conj(unit)).real   # directional derivative along `unit`
                errs.append(abs(fd - an) / max(abs(an), 1e-3 * np.max(np.abs(g))))
    assert max(errs) < 1e-4, errs


def test_matches_torch_autograd(sub):
    torch = pytest.importorskip("torch")
    s, a, psi, w = sub
    L, gpsi, gw = O.amplitude_grad(psi, w, s.positions, a)
    tp = torch.tensor(psi, dtype=torch.complex128, requires_grad=True)
    tw = torch.tensor(w, dtype=torch.complex128, requires_grad=True)
    m = w.shape[0]
    frames = torch.stack([tp[y:y + m, x:x + m] for y, x in s.positions.tolist()])
    Z = torch.fft.ifft2(tw[None] * frames, norm="ortho")
    loss = ((Z.abs() - torch.tensor(a)) ** 2).sum()
    loss.backward()
    assert abs(loss.item() - L) < 1e-10 * L
    assert np.linalg.norm(tp.grad.numpy() - gpsi) < 1e-10 * np.linalg.norm(gpsi)
    assert np.linalg.norm(tw.grad.numpy() - gw) < 1e-10 * np.linalg.norm(gw)


def test_zero_at_noiseless_truth(sub):
    s, a, _, _ = sub
    L, gpsi, gw = O.amplitude_grad(s.obj, s.probe, s.positions, a)
    assert L < 1e-24
    assert np.max(np.abs(gpsi)) < 1e-12 and np.max(np.abs(gw)) < 1e-12


def test_error_reduction_identity(sub):
    """g_psi = 2 (D psi - Q* P_a Q psi), so psi - g_psi/(2D) = Q* P_a Q psi / D."""
    s, a, psi, w = sub
    _, gpsi, _ = O.amplitude_grad(psi, w, s.positions, a)
    shape = psi.shape
    D = O.illumination_density(w, s.positions, shape)
    z = O.Q(psi, w, s.positions)
    ref = 2 * (D * psi - O.Qstar(O.P_a(z, a), w, s.positions, shape))
    assert np.linalg.norm(gpsi - ref) < 1e-12 * np.linalg.norm(ref)
