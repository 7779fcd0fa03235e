"""Synthetic scan recipes.

Geometry follows the paper's discrete far-field model (Sec. "Forward model"):
an n_y x n_x object psi, an m x m probe w, and K integer frame positions x_i
(top-left corner, (y, x) order) with 0 <= x_i <= n - m.  The workloads are
the five benchmark shapes this project measures on:

  1  plain RAAR   object 128^2, Gaussian probe 32^2 (sigma 6), 13x13 raster step 8
  2  RAAR + probe refinement: object 512^2 smooth phase, aperture probe 64^2
     (radius 20, quadratic phase), 29x29 raster step 16 jitter +-2, 1e6 photons
  3  large frames: object 2048^2, Fresnel-propagated aperture 256^2 (radius
     60, Fresnel number 10), 45x45 raster step 40 jitter +-2, 1e8 photons
  4  gradient: object 512^2, Gaussian probe 128^2 (sigma 24), 32x32 raster
     step 12 jitter +-2; subcase "4s": 64^2 object, 16^2 probe, 5x5 step 12
  5  batching: 32 independent scans of uneven sizes (see ``batch_scans``)

Seeds: ``SeedSequence(16020 + cfg)`` spawned into five PCG64 streams
(object, probe, positions, noise, init).  Every draw is documented where it
is made so that the recipe can be reproduced bit for bit.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

STREAMS = ("object", "probe", "positions", "noise", "init")


def streams_for(seed) -> dict:
    """Five independent PCG64 generators spawned from one seed sequence."""
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
    return {name: np.random.default_rng(s) for name, s in zip(STREAMS, ss.spawn(5))}


# ----------------------------------------------------------------------------
# objects
# ----------------------------------------------------------------------------
def random_object(rng, ny: int, nx: int) -> np.ndarray:
    """i.i.d. amplitude U[0.5, 1] and phase U[-pi/2, pi/2] (amplitude drawn first)."""
    amp = rng.uniform(0.5, 1.0, size=(ny, nx))
    ph = rng.uniform(-np.pi / 2, np.pi / 2, size=(ny, nx))
    return amp * np.exp(1j * ph)


def smooth_phase_object(rng, ny: int, nx: int, sigma: float = 4.0) -> np.ndarray:
    """Unit amplitude; phase = (pi/2) f / max|f| with f white N(0,1) noise
    filtered by a periodic Gaussian of standard deviation ``sigma`` pixels."""
    f = rng.standard_normal((ny, nx))
    ky = np.fft.fftfreq(ny)[:, None]
    kx = np.fft.fftfreq(nx)[None, :]
    g = np.exp(-2.0 * np.pi ** 2 * sigma ** 2 * (ky ** 2 + kx ** 2))
    f = np.real(np.fft.ifft2(np.fft.fft2(f) * g))
    ph = (np.pi / 2) * f / np.max(np.abs(f))
    return np.exp(1j * ph)


# ----------------------------------------------------------------------------
# probes (centre c = m // 2, grid r = (y, x) in {0..m-1}^2)
# ----------------------------------------------------------------------------
def _radius2(m: int) -> np.ndarray:
    c = m // 2
    y, x = np.mgrid[0:m, 0:m]
    return (y - c) ** 2 + (x - c) ** 2


def gaussian_probe(m: int, sigma: float) -> np.ndarray:
    """exp(-|r - c|^2 / (2 sigma^2)) with flat phase (sigma is on the amplitude)."""
    return np.exp(-_radius2(m) / (2.0 * sigma ** 2)).astype(np.complex128)


def aperture_probe(m: int, radius: float) -> np.ndarray:
    """circ(|r - c| <= radius) * exp(i alpha |r - c|^2), alpha = 2 pi / radius^2
    (one wave of defocus phase at the rim)."""
    r2 = _radius2(m)
    alpha = 2.0 * np.pi / radius ** 2
    return np.where(r2 <= radius ** 2, np.exp(1j * alpha * r2), 0.0)


def fresnel_aperture_probe(m: int, radius: float, fresnel_number: float) -> np.ndarray:
    """A circular aperture propagated in the Fresnel approximation:
    w = ifft2(fft2(circ) * exp(-i pi lz (fx^2 + fy^2))) with f in cycles/pixel
    and lz = radius^2 / fresnel_number (numpy's non-unitary fft pair)."""
    circ = (_radius2(m) <= radius ** 2).astype(np.complex128)
    lz = radius ** 2 / fresnel_number
    f = np.fft.fftfreq(m)
    kern = np.exp(-1j * np.pi * lz * (f[:, None] ** 2 + f[None, :] ** 2))
    return np.fft.ifft2(np.fft.fft2(circ) * kern)


# ----------------------------------------------------------------------------
# scan positions
# ----------------------------------------------------------------------------
def raster_positions(g: int, step: float, n: int, m: int, K: int | None = None,
                     jitter: int = 0, rng=None) -> np.ndarray:
    """Row-major g x g raster (round(step*j), round(step*k)), the first K of
    them, plus integer jitter U{-jitter..jitter} per axis (drawn as one
    (K, 2) integer array), clamped to [0, n - m].  Returns int32 (K, 2) (y, x)."""
    pos = np.array([(int(round(step * j)), int(round(step * k)))
                    for j in range(g) for k in range(g)], dtype=np.int64)
    if K is not None:
        pos = pos[:K]
    if jitter:
        pos = pos + rng.integers(-jitter, jitter + 1, size=pos.shape)
    return np.clip(pos, 0, n - m).astype(np.int32)


# ----------------------------------------------------------------------------
# photon noise
# ----------------------------------------------------------------------------
def apply_poisson(I: np.ndarray, photons_per_frame: float, rng):
    """Global photon scaling c = N / mean_i sum_q I_i(q), then Poisson(c I).
    Returns (float32 counts, c).  A probe used as 'known' with these counts
    must be scaled by sqrt(c)."""
    K = I.shape[0]
    c = photons_per_frame / (np.sum(I, dtype=np.float64) / K)
    return rng.poisson(c * np.asarray(I, dtype=np.float64)).astype(np.float32), float(c)


# ----------------------------------------------------------------------------
# scan descriptions
# ----------------------------------------------------------------------------
@dataclass
class Scan:
    """One synthetic scan: the truth, the geometry and the run settings."""
    name: str
    n: int                      # object side (square objects)
    m: int                      # frame side
    positions: np.ndarray       # int32 (K, 2), (y, x) top-left
    obj: np.ndarray             # complex128 (n, n) true object
    probe: np.ndarray           # complex128 (m, m) true probe
    psi0: np.ndarray            # complex128 (n, n) start object (real U[0,1))
    photons: float | None = None    # Poisson photons per frame (None = noiseless)
    beta: float = 0.75
    n_iter: int = 10
    probe_every: int = 0        # 0 = known probe
    probe_start: int = 1
    periodic: bool = False
    streams: dict = field(default=None, repr=False)

    @property
    def K(self) -> int:
        return int(self.positions.shape[0])


def _start_object(rng, n):
    """Start image filled with U[0,1) real values (paper, algorithm step 3)."""
    return rng.uniform(0.0, 1.0, size=(n, n)).astype(np.complex128)


def config_scan(cfg) -> Scan:
    """Scan recipe for workload ``cfg`` in {1, 2, 3, 4, '4s'}."""
    key = {1: 1, 2: 2, 3: 3, 4: 4, "4s": 4}[cfg]
    st = streams_for(1602 * 10 + key)
    if cfg == 1:
        n, m = 128, 32
        obj = random_object(st["object"], n, n)
        probe = gaussian_probe(m, 6.0)
        pos = raster_positions(13, 8, n, m)
        return Scan("plain-128-32x169", n, m, pos, obj, probe, _start_object(st["init"], n),
                    None, 0.75, 10, 0, 1, False, st)
    if cfg == 2:
        n, m = 512, 64
        obj = smooth_phase_object(st["object"], n, n, 4.0)
        probe = aperture_probe(m, 20.0)
        pos = raster_positions(29, 16, n, m, jitter=2, rng=st["positions"])
        return Scan("probe-512-64x841", n, m, pos, obj, probe, _start_object(st["init"], n),
                    1e6, 0.75, 100, 1, 1, False, st)
    if cfg == 3:
        n, m = 2048, 256
        obj = random_object(st["object"], n, n)
        probe = fresnel_aperture_probe(m, 60.0, 10.0)
        pos = raster_positions(45, 40, n, m, jitter=2, rng=st["positions"])
        return Scan("large-2048-256x2025", n, m, pos, obj, probe, _start_object(st["init"], n),
                    1e8, 0.75, 50, 0, 1, False, st)
    if cfg == 4:
        n, m = 512, 128
        obj = random_object(st["object"], n, n)
        probe = gaussian_probe(m, 24.0)
        pos = raster_positions(32, 12, n, m, jitter=2, rng=st["positions"])
        return Scan("grad-512-128x1024", n, m, pos, obj, probe, _start_object(st["init"], n),
                    None, 0.75, 1, 0, 1, False, st)
    if cfg == "4s":
        n, m = 64, 16
        obj = random_object(st["object"], n, n)
        probe = gaussian_probe(m, 3.0)
        pos = raster_positions(5, 12, n, m)
        return Scan("grad-64-16x25", n, m, pos, obj, probe, _start_object(st["init"], n),
                    None, 0.75, 1, 0, 1, False, st)
    raise ValueError(f"unknown workload {cfg!r}")


def fig3_scan() -> Scan:
    """Shape of the paper's benchmark (Fig. "timing" caption): 10,000 frames of
    128 x 128 from a 1000 x 1000 image with periodic boundaries and a known
    probe.  The paper's object and zone-plate probe are not available; the
    stand-ins are the i.i.d. object of workload 1 and a Fresnel-propagated
    aperture (radius 30 px, Fresnel number 10).  Raster step 10 px, 100 x 100
    positions, noiseless, start image U[0,1)."""
    st = streams_for(1602 * 10 + 6)
    n, m, step = 1000, 128, 10
    pos = np.array([(step * j, step * k) for j in range(n // step) for k in range(n // step)], dtype=np.int32)
    return Scan("fig3-1000-128x10000-periodic", n, m, pos, random_object(st["object"], n, n),
                fresnel_aperture_probe(m, 30.0, 10.0), _start_object(st["init"], n), None, 0.75, 2000, 0, 1,
                True, st)


def gradient_point(scan: Scan):
    """Evaluation point of the gradient workloads: psi = U[0,1) real (the start
    object), w = w_true (1 + 0.1 xi) with xi ~ N(0,1) real from the init stream
    (drawn after the start object)."""
    xi = scan.streams["init"].standard_normal(scan.probe.shape)
    return scan.psi0.copy(), scan.probe * (1.0 + 0.1 * xi)


def batch_scans(count: int = 32, n_range=(256, 1024), m_choices=(64, 128, 256),
                K_range=(100, 1500)) -> list:
    """Uneven independent scans.  Scan j uses SeedSequence([16025, j]); from its
    positions stream: n ~ U{n_range}, then m ~ U{m_choices} redrawn until
    m <= n/2, then K ~ U{K_range}; raster g = ceil(sqrt K), step (n-m)/(g-1)
    rounded per position, first K positions, jitter +-2.  Object as workload
    1, Gaussian probe sigma = 6 m / 32, noiseless, 20 iterations."""
    scans = []
    for j in range(count):
        st = streams_for(np.random.SeedSequence([16025, j]))
        pr = st["positions"]
        n = int(pr.integers(n_range[0], n_range[1] + 1))
        while True:
            m = int(pr.choice(np.asarray(m_choices)))
            if m <= n // 2:
                break
        K = int(pr.integers(K_range[0], K_range[1] + 1))
        g = int(math.ceil(math.sqrt(K)))
        step = (n - m) / (g - 1)
        pos = raster_positions(g, step, n, m, K=K, jitter=2, rng=pr)
        obj = random_object(st["object"], n, n)
        probe = gaussian_probe(m, 6.0 * m / 32.0)
        scans.append(Scan(f"batch{j:02d}-{n}-{m}x{K}", n, m, pos, obj, probe,
                          _start_object(st["init"], n), None, 0.75, 20, 0, 1, False, st))
    return scans


def shard_share(scan: Scan, g: int, G: int) -> dict:
    """One GPU's share of `scan` under a split into G horizontal strips: the
    range of top-left rows [0, n - m] is cut into G equal parts and GPU g takes
    the frames whose top-left row lies in part g (equal cuts of the object
    itself would leave the last GPU without frames, since no frame starts
    below n - m).  Returns those frames with positions relative to the part's
    first row, the object rows they read (the strip plus a halo of m - 1 rows)
    as (ny, nx), and the true and start objects cut to them."""
    n, m = scan.n, scan.m
    span = n - m + 1
    y0, y1 = g * span // G, (g + 1) * span // G
    sel = np.where((scan.positions[:, 0] >= y0) & (scan.positions[:, 0] < y1))[0]
    pos = scan.positions[sel].copy()
    pos[:, 0] -= y0
    ny = min(n - y0, int(pos[:, 0].max()) + m) if len(sel) else 0
    return {"ny": ny, "nx": n, "m": m, "positions": np.ascontiguousarray(pos, dtype=np.int32), "frames": sel,
            "obj": scan.obj[y0:y0 + ny].copy(), "psi0": scan.psi0[y0:y0 + ny].copy(), "probe": scan.probe,
            "row0": y0}


def small_batch_scans(count: int = 64) -> list:
    """Many small independent scans for the batched form: each has the shape
    of workload 1 (object 128 x 128, 169 frames of 32 x 32 on a 13 x 13
    raster with step 8, Gaussian probe sigma 6, noiseless, start U[0,1)).
    Scan j uses SeedSequence([16027, j])."""
    scans = []
    for j in range(count):
        st = streams_for(np.random.SeedSequence([16027, j]))
        n, m = 128, 32
        scans.append(Scan(f"small{j:02d}-128-32x169", n, m, raster_positions(13, 8, n, m),
                          random_object(st["object"], n, n), gaussian_probe(m, 6.0), _start_object(st["init"], n),
                          None, 0.75, 20, 0, 1, False, st))
    return scans
