"""Pins of the oracle's Q, Q*, D, P_a, P_Q, the object and probe updates,
the initial probe and the metrics (Sec. "Forward model", Sec. "Phase
retrieval", Eqs. (overlap), (Pa), (Pq), (standardobject), (standardprobe),
(solutionmetric))."""
import numpy as np
import pytest

import oracle as O
from sharp_data import gen


def _crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _dense_Q(w, positions, n, periodic):
    """Q as an explicit (K m^2) x (n^2) matrix, built entry by entry from
    z_i(r) = w(r) psi(r + x_i)."""
    m = w.shape[0]
    K = len(positions)
    M = np.zeros((K * m * m, n * n), dtype=complex)
    for i, (py, px) in enumerate(positions):
        for ry in range(m):
            for rx in range(m):
                y, x = py + ry, px + rx
                if periodic:
                    y, x = y % n, x % n
                M[i * m * m + ry * m + rx, y * n + x] += w[ry, rx]
    return M


CASES = [
    # n, m, positions, periodic
    (7, 3, [(0, 0), (0, 2), (2, 1), (4, 4), (3, 0)], False),
    (6, 4, [(0, 0), (1, 3), (4, 5), (5, 1)], True),
]


@pytest.mark.parametrize("n,m,positions,periodic", CASES)
def test_Q_and_Qstar_against_dense_matrix(rng, n, m, positions, periodic):
    pos = np.array(positions, dtype=np.int32)
    w = _crandn(rng, m, m)
    psi = _crandn(rng, n, n)
    z = _crandn(rng, len(pos), m, m)
    M = _dense_Q(w, pos, n, periodic)
    assert np.max(np.abs(O.Q(psi, w, pos, periodic).ravel() - M @ psi.ravel())) < 1e-13
    assert np.max(np.abs(O.Qstar(z, w, pos, (n, n), periodic).ravel()
                         - M.conj().T @ z.ravel())) < 1e-13
    # Q*Q = diag(D)
    D = O.illumination_density(w, pos, (n, n), periodic)
    QhQ = M.conj().T @ M
    assert np.max(np.abs(QhQ - np.diag(D.ravel()))) < 1e-13


@pytest.mark.parametrize("n,m,positions,periodic", CASES)
def test_P_Q_equals_Q_pinv_Q(rng, n, m, positions, periodic):
    pos = np.array(positions, dtype=np.int32)
    w = _crandn(rng, m, m)
    z = _crandn(rng, len(pos), m, m)
    M = _dense_Q(w, pos, n, periodic)
    ref = M @ np.linalg.pinv(M) @ z.ravel()
    got = O.P_Q(z, w, pos, (n, n), periodic).ravel()
    assert np.linalg.norm(got - ref) < 1e-12 * np.linalg.norm(ref)


def test_P_Q_idempotent_selfadjoint_and_keeps_range(rng):
    n, m = 40, 16
    pos = gen.raster_positions(4, 8, n, m)
    w = gen.gaussian_probe(m, 4.0) * np.exp(1j * rng.uniform(-1, 1, (m, m)))
    z1 = _crandn(rng, len(pos), m, m)
    z2 = _crandn(rng, len(pos), m, m)
    P = lambda v: O.P_Q(v, w, pos, (n, n))  # noqa: E731
    p1 = P(z1)
    assert np.linalg.norm(P(p1) - p1) < 1e-12 * np.linalg.norm(p1)
    assert abs(np.vdot(P(z1), z2) - np.vdot(z1, P(z2))) < 1e-11 * np.linalg.norm(z1) * np.linalg.norm(z2)
    psi = _crandn(rng, n, n)
    Qpsi = O.Q(psi, w, pos)
    assert np.linalg.norm(P(Qpsi) - Qpsi) < 1e-12 * np.linalg.norm(Qpsi)


def test_adjoint_identity(rng):
    n, m = 50, 16
    pos = gen.raster_positions(5, 8, n, m, jitter=2, rng=rng)
    w = _crandn(rng, m, m)
    psi = _crandn(rng, n, n)
    z = _crandn(rng, len(pos), m, m)
    lhs = np.vdot(O.Q(psi, w, pos), z)
    rhs = np.vdot(psi, O.Qstar(z, w, pos, (n, n)))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_density_closed_forms():
    # periodic raster with step s dividing m and n, flat probe: D = (m/s)^2 |w|^2
    n, m, s = 32, 8, 2
    pos = np.array([(s * j, s * k) for j in range(n // s) for k in range(n // s)], np.int32)
    D = O.illumination_density(np.full((m, m), 0.5 + 0.5j), pos, (n, n), periodic=True)
    assert np.max(np.abs(D - (m / s) ** 2 * 0.5)) < 1e-12
    # non-periodic: the corner pixel is covered by the first frame only
    n, m = 40, 16
    pos = gen.raster_positions(4, 8, n, m)
    w = gen.gaussian_probe(m, 4.0)
    D = O.illumination_density(w, pos, (n, n))
    assert abs(D[0, 0] - abs(w[0, 0]) ** 2) < 1e-15
    assert abs(D[n - 1, n - 1] - abs(w[m - 1, m - 1]) ** 2) < 1e-15
    # uncovered pixels have D = 0 and dplus = 0 there
    pos = np.array([(0, 0), (20, 20)], np.int32)
    D = O.illumination_density(w, pos, (n, n))
    assert D[18, 2] == 0.0 and O.dplus(D)[18, 2] == 0.0


def test_P_a_scalar_frames_are_circle_projection(rng):
    """With 1x1 frames F is the identity, so P_a z = a z/|z| (and a at z = 0)."""
    z = _crandn(rng, 10, 1, 1)
    z[3] = 0.0
    a = rng.uniform(0.1, 2.0, (10, 1, 1))
    ref = a * z / np.where(np.abs(z) == 0, 1.0, np.abs(z))
    ref[3] = a[3]
    assert np.max(np.abs(O.P_a(z, a) - ref)) < 1e-15


def test_P_a_properties(rng):
    m, K = 16, 5
    z = _crandn(rng, K, m, m)
    a = np.abs(O.dft(_crandn(rng, K, m, m)))
    y = O.P_a(z, a)
    assert np.max(np.abs(np.abs(O.dft(y)) - a)) < 1e-13
    assert np.linalg.norm(O.P_a(y, a) - y) < 1e-13 * np.linalg.norm(y)
    # residual identity: ||(P_a - I) z|| = || |Fz| - a ||
    lhs = np.linalg.norm(y - z)
    rhs = np.linalg.norm(np.abs(O.dft(z)) - a)
    assert abs(lhs - rhs) < 1e-12 * rhs
    # nearest point among random points with the same Fourier modulus
    for _ in range(20):
        x = O.idft(a * np.exp(2j * np.pi * rng.uniform(size=a.shape)))
        assert np.linalg.norm(y - z) <= np.linalg.norm(x - z) + 1e-12


def test_P_a_zero_spectrum_takes_phase_zero():
    m = 4
    z = np.zeros((1, m, m), complex)
    a = np.full((1, m, m), 3.0)
    y = O.P_a(z, a)
    assert np.max(np.abs(O.dft(y) - 3.0)) < 1e-14


def test_object_update_recovers_object_where_covered(rng):
    n, m = 48, 16
    pos = np.array([(0, 0), (0, 12), (12, 0), (12, 12), (30, 30)], np.int32)
    w = gen.gaussian_probe(m, 4.0) * np.exp(0.3j)
    psi = _crandn(rng, n, n)
    D = O.illumination_density(w, pos, (n, n))
    got = O.object_update(O.Q(psi, w, pos), w, pos, (n, n))
    cov = D > 0
    assert np.max(np.abs(got[cov] - psi[cov])) < 1e-12
    assert np.all(got[~cov] == 0)
    assert np.any(~cov)


def test_probe_update_recovers_probe(rng):
    n, m = 48, 16
    pos = gen.raster_positions(4, 10, n, m)
    psi = gen.random_object(rng, n, n)
    w = _crandn(rng, m, m)
    got = O.probe_update(O.Q(psi, w, pos), psi, pos)
    assert np.max(np.abs(got - w)) < 1e-12


def test_probe_update_zero_denominator():
    n, m = 16, 4
    pos = np.array([(0, 0), (4, 4)], np.int32)
    psi = np.ones((n, n), complex)
    psi[0:4, 0:4] = 0
    psi[4:8, 4:8] = 0
    z = np.ones((2, m, m), complex)
    assert np.all(O.probe_update(z, psi, pos) == 0)


def test_init_probe_closed_form():
    """Flat object, probe whose spectrum g is real, positive and even: the
    data are |g|^2 in every frame, so F^{-1} sqrt(mean I) returns the probe
    itself, shifted to the frame centre."""
    m, n = 16, 40
    q = np.fft.fftfreq(m)
    g = np.exp(-(q[:, None] ** 2 + q[None, :] ** 2) / 0.02) + 0.1
    w = O.idft(g)
    pos = gen.raster_positions(4, 8, n, m)
    I = O.forward_intensity(np.ones((n, n), complex), w, pos)
    ref = np.roll(w, (m // 2, m // 2), axis=(0, 1))
    assert np.max(np.abs(O.init_probe(I) - ref)) < 1e-13


def test_eps_0_closed_form_matches_phase_search(rng):
    n, m = 32, 8
    pos = gen.raster_positions(4, 8, n, m)
    w = gen.gaussian_probe(m, 3.0)
    psi0 = gen.random_object(rng, n, n)
    z0 = O.Q(psi0, w, pos)
    z = np.exp(0.7j) * z0 + 0.05 * _crandn(rng, *z0.shape)
    A = O.Qstar(z, w, pos, (n, n))
    B = O.Qstar(z0, w, pos, (n, n))
    phis = np.linspace(0, 2 * np.pi, 3600, endpoint=False)
    grid = min(np.linalg.norm(np.exp(1j * p) * A - B) for p in phis) / np.linalg.norm(B)
    val = O.eps_0(z, z0, w, pos, (n, n))
    assert val <= grid + 1e-12
    assert grid - val < 1e-5            # the grid resolves the optimum to O(dphi^2)
    assert abs(O.eps_0(np.exp(2.1j) * z, z0, w, pos, (n, n)) - val) < 1e-12
    assert O.eps_0(z0 * np.exp(-1.3j), z0, w, pos, (n, n)) < 1e-7


def test_eps_a_residual_identity(rng):
    m = 16
    z = _crandn(rng, 3, m, m)
    a = rng.uniform(0, 1, (3, m, m))
    ref = np.linalg.norm(np.abs(np.fft.ifft2(z, norm="ortho")) - a) / np.linalg.norm(a)
    assert abs(O.eps_a(z, a) - ref) < 1e-13


# ----------------------------------------------------------------------------
# eps_Q and eps_Delta (Eqs. (overlapmetric), (stagnationmetric))
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("n,m,positions,periodic", CASES)
def test_eps_Q_against_dense_projector(rng, n, m, positions, periodic):
    """||(P_Q - I) z|| / ||a|| with P_Q = M pinv(M) for the entry-by-entry
    matrix M of Q (a textbook projector, not the oracle's P_Q); the
    normaliser is ||a|| (not ||z||) and the sign is P_Q - I (P_Q + I gives a
    different value)."""
    pos = np.array(positions, dtype=np.int32)
    w = _crandn(rng, m, m)
    z = _crandn(rng, len(pos), m, m)
    a = rng.uniform(0.5, 2.0, (len(pos), m, m))
    M = _dense_Q(w, pos, n, periodic)
    resid = M @ (np.linalg.pinv(M) @ z.ravel()) - z.ravel()
    ref = np.sqrt(np.sum(np.abs(resid) ** 2)) / np.sqrt(np.sum(a ** 2))
    got = O.eps_Q(z, w, pos, (n, n), a, periodic)
    assert abs(got - ref) < 1e-12 * ref
    plus = M @ (np.linalg.pinv(M) @ z.ravel()) + z.ravel()
    assert abs(got - np.linalg.norm(plus) / np.linalg.norm(a)) > 0.1 * ref
    assert abs(O.eps_Q(z, w, pos, (n, n), 2.0 * a, periodic) - ref / 2) < 1e-12 * ref


def test_eps_Q_vanishes_on_the_range_of_Q(rng):
    n, m = 40, 16
    pos = gen.raster_positions(4, 8, n, m)
    w = gen.gaussian_probe(m, 4.0)
    z = O.Q(_crandn(rng, n, n), w, pos)
    a = np.abs(O.dft(z))
    assert O.eps_Q(z, w, pos, (n, n), a) < 1e-14


def test_eps_Delta_closed_forms(rng):
    """z_new = z_old + c e_j (one element changed by c) with a = 2 everywhere:
    eps_Delta = |c| / (2 sqrt(K m^2)); unchanged frames give 0."""
    K, m = 5, 4
    z_old = _crandn(rng, K, m, m)
    a = np.full((K, m, m), 2.0)
    z_new = z_old.copy()
    z_new[3, 1, 2] += 3.0 - 4.0j
    assert abs(O.eps_Delta(z_new, z_old, a) - 5.0 / (2.0 * np.sqrt(K * m * m))) < 1e-15
    assert O.eps_Delta(z_old, z_old, a) == 0.0
    assert abs(O.eps_Delta(z_new, z_old, 4.0 * a) - 5.0 / (8.0 * np.sqrt(K * m * m))) < 1e-15


def test_recorded_extra_metrics_follow_the_iterates(rng):
    """raar(record_extra) records, after iteration l, ||(P_Q - I) z^(l)|| and
    ||z^(l) - z^(l-1)|| over ||a||, with z^(0) = Q psi0 (reading R5); checked
    with the dense projector and the iterates of shorter runs."""
    n, m, positions, periodic = CASES[0]
    pos = np.array(positions, dtype=np.int32)
    w = _crandn(rng, m, m)
    psi = _crandn(rng, n, n)
    psi0 = _crandn(rng, n, n)
    I = O.forward_intensity(psi, w, pos)
    a = np.sqrt(I)
    M = _dense_Q(w, pos, n, periodic)
    P = M @ np.linalg.pinv(M)
    L = 4
    out = O.raar(I, pos, (n, n), m, L, 0.75, psi0=psi0, w0=w, record_extra=True)
    z_prev = (M @ psi0.ravel()).reshape(len(pos), m, m)
    na = np.sqrt(np.sum(a ** 2))
    for l in range(1, L + 1):
        z_l = O.raar(I, pos, (n, n), m, l, 0.75, psi0=psi0, w0=w)["z"]
        eq = np.linalg.norm(P @ z_l.ravel() - z_l.ravel()) / na
        ed = np.linalg.norm(z_l - z_prev) / na
        assert abs(out["eps_Q"][l - 1] - eq) < 1e-10 * max(eq, 1e-300) + 1e-15
        assert abs(out["eps_Delta"][l - 1] - ed) < 1e-12 * ed
        z_prev = z_l
    assert out["eps_Delta"][0] > 1e-3


@pytest.mark.parametrize("n,m,positions,periodic", CASES)
def test_P_Q_with_density_threshold_is_the_restricted_projector(rng, n, m, positions, periodic):
    """With the threshold eps_D the object update leaves the pixels with
    D <= eps_D at 0, and P_Q is the orthogonal projector onto Q of objects
    supported on D > eps_D: M_S pinv(M_S), M_S the columns of the dense Q
    matrix for those pixels (reading R3)."""
    pos = np.array(positions, dtype=np.int32)
    w = _crandn(rng, m, m)
    z = _crandn(rng, len(pos), m, m)
    D = O.illumination_density(w, pos, (n, n), periodic)
    eps = np.quantile(D[D > 0], 0.3)
    S = (D > eps).ravel()
    assert 0 < S.sum() < np.count_nonzero(D)
    M = _dense_Q(w, pos, n, periodic)[:, S]
    ref = M @ np.linalg.pinv(M) @ z.ravel()
    got = O.P_Q(z, w, pos, (n, n), periodic, eps_D=eps).ravel()
    assert np.linalg.norm(got - ref) < 1e-12 * np.linalg.norm(ref)
    obj = O.object_update(z, w, pos, (n, n), periodic, eps_D=eps)
    assert np.all(obj.ravel()[~S] == 0)
    assert np.linalg.norm(obj.ravel()[S] - np.linalg.pinv(M) @ z.ravel()) < 1e-12 * np.linalg.norm(obj)


def test_extract_is_the_window_and_wraps_periodically(rng):
    """T_i psi is the m x m window at the frame's top-left corner (Sec.
    "Forward model"); with periodic boundaries the window wraps modulo the
    object size: written out index by index."""
    n, m = 9, 4
    psi = _crandn(rng, n, n)
    pos = np.array([(0, 0), (5, 2), (7, 8)], dtype=np.int32)
    got = O.extract(psi, pos[:2], m)
    assert np.array_equal(got[0], psi[0:4, 0:4]) and np.array_equal(got[1], psi[5:9, 2:6])
    got = O.extract(psi, pos, m, periodic=True)
    for i, (py, px) in enumerate(pos):
        for ry in range(m):
            for rx in range(m):
                assert got[i, ry, rx] == psi[(py + ry) % n, (px + rx) % n]


def test_sgn_unit_modulus_and_zero_convention(rng):
    """sgn(u) = u / |u| with sgn(0) := 1 (Eq. (Pa), reading R2): unit modulus,
    sgn(u) |u| = u, and exactly 1 at an exact zero (also -0)."""
    u = _crandn(rng, 50)
    s = O.sgn(u)
    assert np.allclose(np.abs(s), 1.0, atol=1e-15) and np.allclose(s * np.abs(u), u, atol=1e-14)
    z = O.sgn(np.array([0.0 + 0.0j, -0.0 + 0.0j, complex(0.0, -0.0)]))
    assert np.array_equal(z, np.ones(3, dtype=complex))
    tiny = O.sgn(np.array([1e-300 + 0j, -1e-300j]))   # nonzero however small: u / |u|, not the zero rule
    assert np.allclose(tiny, [1.0, -1j], atol=1e-15)


@pytest.mark.parametrize("m", [2, 5, 8])
def test_dft_matrix_entries_and_unitarity(m):
    """W_jk = e^{+2 pi i jk/m} / sqrt(m), the unitary matrix of the paper's
    transform (Sec. "Forward model"): its entries written out, and W W* = I."""
    W = O.dft_matrix(m)
    j, k = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    assert np.allclose(W, np.exp(2j * np.pi * j * k / m) / np.sqrt(m), atol=1e-15)
    assert np.allclose(W @ W.conj().T, np.eye(m), atol=1e-14)
