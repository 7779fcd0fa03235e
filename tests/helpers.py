"""Shared helpers of the GPU tests: tensor conversion and the parity
measures.

Object parity (`check_object`) applies four measures:
  * D-weighted normwise ||D (psi - ref)|| / ||D ref|| with D = diag(Q*Q), the
    weighting of the solution metric, Eq. (solutionmetric): <= tol;
  * D-weighted per element max|D (psi - ref)| / max|D ref|, so that a few
    wrong pixels cannot hide in the norm: <= tol;
  * unweighted normwise and per-element errors over the well-lit pixels
    D >= 1e-3 max D: <= tol sqrt(1e3) (~31.6 tol).  The FP32 rounding of
    the frame transforms is spread evenly over a frame, so after the object
    update psi = Q* z / D its contribution at a pixel scales like
    sum |w| / D ~ D^(-1/2) relative to the brightest pixels: down to
    D = 1e-3 max D that amplification is at most sqrt(1e3).  A value that
    is wrong (an index or sign mistake) is off by O(1) and still fails;
  * exact zeros where no frame covers a pixel (D = 0: the object update sets
    them to 0, reading R3).
Frame-space quantities, probes and gradients (`check_close`) are held to a
normwise and a per-element bound, max|x - ref| <= tol max|ref|."""
import numpy as np

LIT = 1e-3                 # well-lit pixels: D >= LIT * max D
LIT_FACTOR = LIT ** -0.5   # rounding amplification allowed down to LIT * max D


def rel(a, b):
    """Normwise relative error ||a - b|| / ||b||."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def elem(a, b):
    """Per-element error relative to the largest reference entry,
    max|a - b| / max|b|."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def dweighted(psi, ref, D):
    """D-weighted object error ||D (psi - ref)|| / ||D ref||."""
    return float(np.linalg.norm(D * (psi - ref)) / np.linalg.norm(D * ref))


def object_errors(psi, ref, D):
    psi = np.asarray(psi, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    D = np.asarray(D, dtype=np.float64)
    lit = D >= LIT * D.max()
    return {"dweighted": dweighted(psi, ref, D), "dweighted_elem": elem(D * psi, D * ref),
            "lit": rel(psi[lit], ref[lit]), "lit_elem": elem(psi[lit], ref[lit]),
            "uncovered_nonzero": int(np.count_nonzero(psi[D == 0]))}


def check_object(psi, ref, D, tol=1e-4, where=""):
    """Assert object parity under all four measures (module docstring).
    Returns the measures."""
    tol_lit = tol * LIT_FACTOR
    e = object_errors(psi, ref, D)
    msg = f"{where} {e}"
    assert e["dweighted"] < tol, msg
    assert e["dweighted_elem"] < tol, msg
    assert e["lit"] < tol_lit, msg
    assert e["lit_elem"] < tol_lit, msg
    assert e["uncovered_nonzero"] == 0, msg
    return e


def check_close(x, ref, tol, where=""):
    """Assert normwise and per-element parity of a frame stack, probe or
    gradient.  Returns (normwise, per-element)."""
    r, m = rel(x, ref), elem(x, ref)
    assert r < tol and m < tol, f"{where} normwise {r:.3e} per-element {m:.3e} (tol {tol})"
    return r, m


def c64(x):
    return np.ascontiguousarray(np.asarray(x), dtype=np.complex64)


def to_dev(x, dtype=None):
    import torch
    arr = np.ascontiguousarray(x if dtype is None else np.asarray(x, dtype=dtype))
    return torch.from_numpy(arr).to("cuda")


def to_host(t):
    return t.detach().cpu().numpy()
