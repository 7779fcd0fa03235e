"""FP64 reference implementation of the SHARP RAAR hot path.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously correct
CPU statement of what the GPU library computes.  Only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path never does.  It shares no code with the HIP library.

Everything follows the paper (Marchesini et al., "SHARP: a distributed,
GPU-based ptychographic solver", arXiv:1602.01448):

  * frames, the illumination operator Q and the stacked forms:
    Sec. "Forward model", Eqs. (data0), (forwardproblem1), (data), (overlap),
    (standardprobe0);
  * the 2-D DFT F, unitary with the e^{+2 pi i q.r} sign: Sec. "Forward model";
  * the data projector P_a: Eq. (Pa); the overlap projector P_Q: Eq. (Pq);
  * object and probe updates: Eqs. (standardobject), (standardprobe);
  * the reconstruction sequence (algorithm box in Sec. "Phase retrieval");
  * metrics eps_a, eps_Q, eps_Delta, eps_0: Eqs. (amplitudemetric),
    (overlapmetric), (stagnationmetric), (solutionmetric).

Readings taken where the paper is silent, ambiguous or garbled (the GPU path
takes the same ones):

  R1  The printed RAAR update in the algorithm box carries beta(P_Q - I); that
      operator has eigenvalue 1 - 3 beta on the orthogonal complement of
      range(Q) and diverges for beta > 2/3.  The relaxed averaged alternating
      reflections map it cites (Luke) has beta(I - P_Q); that form is used:
      z <- [2 beta P_Q P_a + (1 - 2 beta) P_a + beta (I - P_Q)] z.
  R2  sgn(u) = u/|u| with sgn(0) := 1 (exact-zero test) inside P_a.
  R3  (Q*Q)^{-1} is applied as D^+ with D^+ = 1/D where D > 0 and 0 where
      D = 0 (pixels no frame covers get psi = 0).  An optional threshold
      eps_D >= 0 (a user option, 0 by default) widens the zero set to
      D <= eps_D: P_Q then projects onto the frames of objects supported on
      the pixels with D > eps_D.
  R4  Probe update: w = 0 where the denominator S* T |psi|^2 is 0.
  R5  z^(0) = Q psi^(0) (algorithm step 4); the "z^(0) = 0" next to the
      metrics is read as part of the eps_Delta definition only.
  R6  Positions are integer top-left corners (y, x) with 0 <= x_i <= n - m;
      with ``periodic`` the frame wraps modulo the object size.
  R7  Initial probe: w0 = roll(F^{-1} sqrt(mean_i I_i), (m//2, m//2)) (the
      paper does not say where the probe is centred; the frame centre is
      used).
  R8  Probe refinement: psi^(l) is formed with the probe used in iteration l,
      then w is updated from (psi^(l), z^(l)) and D is rebuilt.
  R9  Frames are summed in ascending frame index everywhere.
  R10 Gradient of L = sum_i sum_q (|F(w T_i psi)|_q - a_iq)^2 in the complex
      convention g = dL/dRe + i dL/dIm (no 1/2 in L).
  R14 Probe constraints (algorithm step 7): F is the frame transform of the
      data (unitary, DC at [0][0]); the Fourier mask m_w multiplies F w; the
      Fourier amplitudes a_w replace |F w| with sgn(0) := 1; when both are
      given the mask is used (the box tests for the mask first).
  R15 Centre-of-mass correction (algorithm step 7): the centroid c of |w|^2
      over pixel indices (y, x) in 0..m-1 (no wrap), formed in FP64 (the paper
      states no precision); w is rolled circularly by the integer
      s = floor(m/2 - c + 1/2) per axis, which puts the centroid within half a
      pixel of the frame centre (m/2, m/2) without interpolation.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "dft", "idft", "dft_matrix", "dft_by_matrix",
    "extract", "Q", "Qstar", "illumination_density", "dplus",
    "forward_intensity", "sgn", "P_a", "P_Q",
    "raar_step", "raar", "object_update", "probe_update", "init_probe",
    "probe_fourier_constraint", "probe_centroid", "probe_center_shift", "probe_center",
    "eps_a", "eps_Q", "eps_Delta", "eps_0", "amplitude_loss", "amplitude_grad",
]


# ----------------------------------------------------------------------------
# 2-D DFT  (Sec. "Forward model": (F f)(q) = (1/m) sum_r e^{2 pi i q.r} f(r))
# ----------------------------------------------------------------------------
def dft(z):
    """F over the last two axes: unitary, e^{+2 pi i} sign.  numpy's inverse
    FFT with orthonormal scaling is exactly this sum (library primitive)."""
    return np.fft.ifft2(np.asarray(z, dtype=np.complex128), norm="ortho")


def idft(Z):
    """F* = F^{-1} over the last two axes (e^{-2 pi i} sign, 1/m scale)."""
    return np.fft.fft2(np.asarray(Z, dtype=np.complex128), norm="ortho")


def dft_matrix(m: int) -> np.ndarray:
    """W_{jk} = e^{2 pi i (j k mod m)/m} / sqrt(m); the 2-D F is W Z W^T."""
    j = np.arange(m)
    return np.exp(2j * np.pi * (np.outer(j, j) % m) / m) / np.sqrt(m)


def dft_by_matrix(z):
    """F written as the DFT-matrix product W Z W^T (slow cross-check of dft)."""
    z = np.asarray(z, dtype=np.complex128)
    W = dft_matrix(z.shape[-1])
    return W @ z @ W.T


# ----------------------------------------------------------------------------
# Frame extraction T_i, illumination operator Q and its adjoint
# (Sec. "Forward model", Eqs. (overlap), (standardprobe0))
# ----------------------------------------------------------------------------
def _rows_cols(p, m, shape, periodic):
    ny, nx = shape
    y, x = int(p[0]), int(p[1])
    if periodic:
        return (np.arange(y, y + m) % ny), (np.arange(x, x + m) % nx)
    if not (0 <= y <= ny - m and 0 <= x <= nx - m):
        raise ValueError(f"frame at {(y, x)} leaves the {ny}x{nx} object")
    return np.arange(y, y + m), np.arange(x, x + m)


def extract(psi, positions, m, periodic=False):
    """T psi: the K frames psi(r + x_i), shape (K, m, m)."""
    psi = np.asarray(psi, dtype=np.complex128)
    out = np.empty((len(positions), m, m), dtype=np.complex128)
    for i, p in enumerate(positions):
        r, c = _rows_cols(p, m, psi.shape, periodic)
        out[i] = psi[np.ix_(r, c)]
    return out


def Q(psi, w, positions, periodic=False):
    """z_i(r) = w(r) psi(r + x_i)."""
    w = np.asarray(w, dtype=np.complex128)
    return w[None] * extract(psi, positions, w.shape[0], periodic)


def _scatter_add(frames, positions, shape, periodic):
    out = np.zeros(shape, dtype=frames.dtype)
    m = frames.shape[-1]
    for i, p in enumerate(positions):          # ascending frame order (R9)
        r, c = _rows_cols(p, m, shape, periodic)
        out[np.ix_(r, c)] += frames[i]
    return out


def Qstar(z, w, positions, shape, periodic=False):
    """Q* z = sum_i T_i^T (conj(w) z_i)."""
    w = np.asarray(w, dtype=np.complex128)
    return _scatter_add(np.conj(w)[None] * np.asarray(z, dtype=np.complex128),
                        positions, shape, periodic)


def illumination_density(w, positions, shape, periodic=False):
    """D = diag(Q*Q) = sum_i T_i^T |w|^2 (Eq. (Pq) and (standardobject))."""
    w = np.asarray(w, dtype=np.complex128)
    aw2 = np.broadcast_to(np.abs(w) ** 2, (len(positions),) + w.shape)
    return _scatter_add(np.ascontiguousarray(aw2), positions, shape, periodic).real


def dplus(D, eps_D=0.0):
    """(Q*Q)^{-1} as used here: 1/D where D > eps_D, 0 elsewhere (R3)."""
    D = np.asarray(D, dtype=np.float64)
    out = np.zeros_like(D)
    nz = D > eps_D
    out[nz] = 1.0 / D[nz]
    return out


def forward_intensity(psi, w, positions, periodic=False):
    """I_i = |F Q_i psi|^2 (Eq. (data0) squared)."""
    return np.abs(dft(Q(psi, w, positions, periodic))) ** 2


# ----------------------------------------------------------------------------
# Projectors (Eqs. (Pa), (Pq))
# ----------------------------------------------------------------------------
def sgn(u):
    """u/|u| with sgn(0) = 1 (R2)."""
    u = np.asarray(u, dtype=np.complex128)
    mag = np.abs(u)
    out = np.ones_like(u)
    nz = mag != 0
    out[nz] = u[nz] / mag[nz]
    return out


def P_a(z, a):
    """P_a z = F* (F z / |F z|) a."""
    return idft(sgn(dft(z)) * np.asarray(a, dtype=np.float64))


def P_Q(z, w, positions, shape, periodic=False, D=None, eps_D=0.0):
    """P_Q z = Q (Q*Q)^{-1} Q* z."""
    if D is None:
        D = illumination_density(w, positions, shape, periodic)
    return Q(dplus(D, eps_D) * Qstar(z, w, positions, shape, periodic), w, positions, periodic)


# ----------------------------------------------------------------------------
# Updates (Eqs. (standardobject), (standardprobe))
# ----------------------------------------------------------------------------
def object_update(z, w, positions, shape, periodic=False, D=None, eps_D=0.0):
    """psi = Q* z / Q*Q  (0 where D = 0, or D <= eps_D, R3)."""
    if D is None:
        D = illumination_density(w, positions, shape, periodic)
    return dplus(D, eps_D) * Qstar(z, w, positions, shape, periodic)


def probe_update(z, psi, positions, periodic=False):
    """w = S* diag(T conj(psi)) z / S* T |psi|^2  (0 where the denominator is 0, R4).
    S* sums the frame stack over i."""
    T = extract(psi, positions, z.shape[-1], periodic)
    num = np.sum(np.conj(T) * z, axis=0)
    den = np.sum(np.abs(T) ** 2, axis=0)
    out = np.zeros_like(num)
    nz = den > 0
    out[nz] = num[nz] / den[nz]
    return out


def probe_fourier_constraint(w, mask=None, amplitudes=None):
    """Algorithm step 7: w := F^{-1}{(F w) m_w} if a mask is given, else
    w := F^{-1}{sgn(F w) a_w} if Fourier amplitudes are given, else w (R14)."""
    w = np.asarray(w, dtype=np.complex128)
    if mask is not None:
        return idft(dft(w) * np.asarray(mask, dtype=np.float64))
    if amplitudes is not None:
        return idft(sgn(dft(w)) * np.asarray(amplitudes, dtype=np.float64))
    return w


def probe_centroid(w):
    """Centroid (cy, cx) of |w|^2 over the pixel indices 0..m-1 (R15), in
    FP64; None when w is zero."""
    p = np.abs(np.asarray(w, dtype=np.complex128)) ** 2
    tot = p.sum()
    if tot <= 0:
        return None
    idx = np.arange(p.shape[0], dtype=np.float64)
    return float((p.sum(axis=1) * idx).sum() / tot), float((p.sum(axis=0) * idx).sum() / tot)


def probe_center_shift(w):
    """Integer roll (sy, sx) that brings the |w|^2 centroid to the frame
    centre: s = floor(m/2 - c + 1/2) per axis (R15)."""
    c = probe_centroid(w)
    if c is None:
        return 0, 0
    half = w.shape[-1] // 2
    return int(np.floor(half - c[0] + 0.5)), int(np.floor(half - c[1] + 0.5))


def probe_center(w):
    """Centre-of-mass drift correction of algorithm step 7: roll w by
    probe_center_shift(w)."""
    sy, sx = probe_center_shift(w)
    return np.roll(np.asarray(w, dtype=np.complex128), (sy, sx), axis=(0, 1))


def init_probe(I):
    """w0 = F^{-1} sqrt(mean_i I_i), centred on the frame (algorithm step 2, R7)."""
    I = np.asarray(I, dtype=np.float64)
    w0 = idft(np.sqrt(np.maximum(np.mean(I, axis=0), 0.0)))
    m = I.shape[-1]
    return np.roll(w0, (m // 2, m // 2), axis=(0, 1))


# ----------------------------------------------------------------------------
# Metrics (Eqs. (amplitudemetric) ... (solutionmetric))
# ----------------------------------------------------------------------------
def eps_a(z, a):
    """||(P_a - I) z|| / ||a||."""
    return np.linalg.norm(P_a(z, a) - z) / np.linalg.norm(a)


def eps_Q(z, w, positions, shape, a, periodic=False):
    """||(P_Q - I) z|| / ||a||."""
    return np.linalg.norm(P_Q(z, w, positions, shape, periodic) - z) / np.linalg.norm(a)


def eps_Delta(z_new, z_old, a):
    """||z^(l) - z^(l-1)|| / ||a||."""
    return np.linalg.norm(np.asarray(z_new) - np.asarray(z_old)) / np.linalg.norm(a)


def eps_0(z, z0, w, positions, shape, periodic=False):
    """min_phi ||Q*(e^{i phi} z - z0)|| / ||Q* z0||.  With A = Q*z, B = Q*z0
    the minimum over the global phase is attained at phi = -arg<A, B>, where
    ||e^{i phi} A - B||^2 = ||A||^2 + ||B||^2 - 2 |<A, B>|."""
    A = Qstar(z, w, positions, shape, periodic)
    B = Qstar(z0, w, positions, shape, periodic)
    nA2 = np.vdot(A, A).real
    nB2 = np.vdot(B, B).real
    val = max(nA2 + nB2 - 2.0 * abs(np.vdot(A, B)), 0.0)
    return np.sqrt(val) / np.sqrt(nB2)


# ----------------------------------------------------------------------------
# RAAR (algorithm box, step 5, with reading R1)
# ----------------------------------------------------------------------------
def raar_step(z, beta, proj_a, proj_Q):
    """One RAAR map z -> 2b P_Q P_a z + (1-2b) P_a z + b (z - P_Q z).
    Written with the reflection-free rearrangement
    beta z + (1 - 2 beta) y + beta P_Q(2 y - z), y = P_a z,
    which is the same linear combination because P_Q is linear."""
    y = proj_a(z)
    return beta * z + (1.0 - 2.0 * beta) * y + beta * proj_Q(2.0 * y - z)


def raar(I, positions, shape, m, n_iter, beta=0.75, psi0=None, w0=None,
         probe_every=0, probe_start=1, periodic=False, record_extra=False, eps_D=0.0,
         rng_init=None, probe_mask=None, probe_amplitudes=None, probe_center_com=False,
         trace=None):
    """The reconstruction sequence of the algorithm box.

    Returns a dict with the object psi (step 6 of the last iteration), the
    probe w, the frames z, the per-iteration eps_a (measured on the z that
    enters the iteration) and, with ``record_extra``, eps_Q and eps_Delta.
    ``trace``, a list, receives the |w|^2 centroid each centre-of-mass
    correction starts from (a record only; the iteration does not read it).
    """
    I = np.asarray(I, dtype=np.float64)
    a = np.sqrt(np.maximum(I, 0.0))                       # variance-stabilised amplitudes
    w = init_probe(I) if w0 is None else np.asarray(w0, dtype=np.complex128)
    if psi0 is None:                                      # step 3
        psi0 = rng_init.uniform(0.0, 1.0, size=shape).astype(np.complex128)
    D = illumination_density(w, positions, shape, periodic)   # step 4
    z = Q(psi0, w, positions, periodic)
    hist = {"eps_a": [], "eps_Q": [], "eps_Delta": []}
    psi = object_update(z, w, positions, shape, periodic, D, eps_D)
    for it in range(1, n_iter + 1):
        hist["eps_a"].append(eps_a(z, a))
        z_old = z
        z = raar_step(z, beta, lambda v: P_a(v, a),
                      lambda v: P_Q(v, w, positions, shape, periodic, D, eps_D))  # step 5
        psi = object_update(z, w, positions, shape, periodic, D, eps_D)          # step 6
        if record_extra:
            hist["eps_Q"].append(eps_Q(z, w, positions, shape, a, periodic))
            hist["eps_Delta"].append(eps_Delta(z, z_old, a))
        if probe_every and it >= probe_start and (it - probe_start) % probe_every == 0:
            w = probe_update(z, psi, positions, periodic)                  # step 7
            w = probe_fourier_constraint(w, probe_mask, probe_amplitudes)
            if probe_center_com:
                if trace is not None:
                    trace.append(probe_centroid(w))
                w = probe_center(w)
            D = illumination_density(w, positions, shape, periodic)
    return {"psi": psi, "w": w, "z": z, **{k: np.array(v) for k, v in hist.items()}}


# ----------------------------------------------------------------------------
# Amplitude loss and its gradient (R10)
# ----------------------------------------------------------------------------
def amplitude_loss(psi, w, positions, a, periodic=False):
    """L = sum_i sum_q (|F(w T_i psi)|_q - a_iq)^2."""
    Z = dft(Q(psi, w, positions, periodic))
    return float(np.sum((np.abs(Z) - np.asarray(a, dtype=np.float64)) ** 2))


def amplitude_grad(psi, w, positions, a, periodic=False):
    """(L, g_psi, g_w) with g = dL/dRe + i dL/dIm:
    r = 2 (z - P_a z), g_psi = Q* r, g_w = sum_i conj(T_i psi) r_i, z = Q_w psi.
    (L = ||z - P_a z||^2 because F is unitary; the squared distance to a set
    has real gradient 2 (z - P(z)).)"""
    psi = np.asarray(psi, dtype=np.complex128)
    w = np.asarray(w, dtype=np.complex128)
    z = Q(psi, w, positions, periodic)
    r = 2.0 * (z - P_a(z, a))
    g_psi = Qstar(r, w, positions, psi.shape, periodic)
    g_w = np.sum(np.conj(extract(psi, positions, w.shape[0], periodic)) * r, axis=0)
    return amplitude_loss(psi, w, positions, a, periodic), g_psi, g_w
