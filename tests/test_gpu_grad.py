"""GPU amplitude-loss gradient (hand-written adjoint) against the FP64 oracle
gradient and, through the torch.autograd.Function, against torch's own
conventions.  Tolerance 1e-5 normwise."""
import numpy as np
import pytest

import oracle as O
from helpers import c64, check_close, to_dev, to_host
from sharp_data import gen

pytestmark = pytest.mark.gpu


def _setup(cfg, **opts):
    from paper_1602_01448_amd import Plan
    s = gen.config_scan(cfg)
    I = O.forward_intensity(s.obj, s.probe, s.positions).astype(np.float32)
    psi, w = gen.gradient_point(s)
    psi, w = c64(psi), c64(w)
    p = Plan(s.n, s.n, s.m, s.positions, **opts)
    p.set_data(to_dev(I))
    return s, p, np.sqrt(I.astype(np.float64)), psi, w


# the last case is the benchmark's tuned launch: 16^2 merge tiles whose frame
# lists are split into four chunks, summed by the second merge pass
@pytest.mark.parametrize("cfg,opts", [("4s", {}), (4, {}), (4, {"grad_groups": 256, "tile": 16, "merge_split": 4})])
def test_gradient_matches_oracle(cfg, opts):
    s, p, a, psi, w = _setup(cfg, **opts)
    loss, gpsi, gw = p.grad(to_dev(psi), to_dev(w))
    L, rpsi, rw = O.amplitude_grad(psi, w, s.positions, a)
    assert abs(loss.item() - L) / L < 1e-5
    check_close(to_host(gpsi), rpsi, 1e-5)
    check_close(to_host(gw), rw, 1e-5)


@pytest.mark.parametrize("groups", [1, 3, 64])
def test_gradient_independent_of_partial_count(groups):
    from paper_1602_01448_amd import Plan
    s = gen.config_scan("4s")
    I = O.forward_intensity(s.obj, s.probe, s.positions).astype(np.float32)
    psi, w = map(c64, gen.gradient_point(s))
    p = Plan(s.n, s.n, s.m, s.positions, grad_groups=groups)
    p.set_data(to_dev(I))
    _, gpsi, gw = p.grad(to_dev(psi), to_dev(w))
    _, rpsi, rw = O.amplitude_grad(psi, w, s.positions, np.sqrt(I.astype(np.float64)))
    check_close(to_host(gw), rw, 1e-5)
    check_close(to_host(gpsi), rpsi, 1e-5)


@pytest.mark.parametrize("m,K,n", [(32, 9, 80), (64, 12, 160), (256, 3, 300)])
def test_gradient_other_sizes(m, K, n):
    from paper_1602_01448_amd import Plan
    rng = np.random.default_rng(m)
    pos = rng.integers(0, n - m + 1, size=(K, 2)).astype(np.int32)
    obj = gen.random_object(rng, n, n)
    probe = gen.gaussian_probe(m, m / 5)
    I = O.forward_intensity(obj, probe, pos).astype(np.float32)
    psi = c64(obj * (1 + 0.2 * rng.standard_normal((n, n))))
    w = c64(probe * (1 + 0.1 * rng.standard_normal((m, m))))
    p = Plan(n, n, m, pos)
    p.set_data(to_dev(I))
    loss, gpsi, gw = p.grad(to_dev(psi), to_dev(w))
    L, rpsi, rw = O.amplitude_grad(psi, w, pos, np.sqrt(I.astype(np.float64)))
    assert abs(loss.item() - L) / L < 1e-5
    check_close(to_host(gpsi), rpsi, 1e-5)
    check_close(to_host(gw), rw, 1e-5)


@pytest.mark.parametrize("form,groups,periodic", [(1, 0, False), (2, 0, False), (2, 1, False), (2, 7, False),
                                                 (2, 0, True)])
def test_gradient_frame128_forms(form, groups, periodic):
    """m = 128: frame-space kernel and the register-resident kernel (with its
    per-workgroup probe-gradient slots, any workgroup count), against the
    oracle; periodic wrap on an object side that is not a multiple of 128."""
    from paper_1602_01448_amd import Plan
    rng = np.random.default_rng(128 + groups)
    n, m, K = (330, 128, 23)
    hi = n if periodic else n - m + 1
    pos = rng.integers(0, hi, size=(K, 2)).astype(np.int32)
    obj = gen.random_object(rng, n, n)
    probe = gen.gaussian_probe(m, 24.0)
    I = O.forward_intensity(obj, probe, pos, periodic).astype(np.float32)
    psi = c64(obj * (1 + 0.2 * rng.standard_normal((n, n))))
    w = c64(probe * (1 + 0.1 * rng.standard_normal((m, m))))
    p = Plan(n, n, m, pos, periodic=periodic, frame_launch=form, grad_groups=groups)
    p.set_data(to_dev(I))
    assert p.info()["frame_launch"] == form
    loss, gpsi, gw = p.grad(to_dev(psi), to_dev(w))
    L, rpsi, rw = O.amplitude_grad(psi, w, pos, np.sqrt(I.astype(np.float64)), periodic)
    assert abs(loss.item() - L) / L < 1e-5
    check_close(to_host(gpsi), rpsi, 1e-5)
    check_close(to_host(gw), rw, 1e-5)


def test_autograd_function():
    import torch
    from paper_1602_01448_amd import AmplitudeLoss
    s, p, a, psi, w = _setup("4s")
    tpsi = to_dev(psi).requires_grad_(True)
    tw = to_dev(w).requires_grad_(True)
    loss = AmplitudeLoss.apply(tpsi, tw, p)
    (3.0 * loss).backward()
    L, rpsi, rw = O.amplitude_grad(psi, w, s.positions, a)
    check_close(to_host(tpsi.grad), 3.0 * rpsi, 1e-5)
    check_close(to_host(tw.grad), 3.0 * rw, 1e-5)
    # directional derivative of the GPU loss along a random direction
    rng = np.random.default_rng(0)
    d = c64(rng.standard_normal(psi.shape) + 1j * rng.standard_normal(psi.shape))
    d /= np.linalg.norm(d)
    h = 1e-2
    with torch.no_grad():
        lp = AmplitudeLoss.apply(to_dev(c64(psi + h * d)), tw.detach(), p).item()
        lm = AmplitudeLoss.apply(to_dev(c64(psi - h * d)), tw.detach(), p).item()
    fd = (lp - lm) / (2 * h)
    an = np.real(np.vdot(rpsi, d))
    assert abs(fd - an) < 1e-2 * max(1.0, abs(an))
