"""Python face of a SHARP plan: torch tensors in, torch tensors out; all work
runs in libsharp's HIP kernels on the caller's current stream."""
from __future__ import annotations

from ctypes import POINTER, byref, c_float, c_int, c_int32, c_void_p

import numpy as np
import torch

from ._lib import OPS, SharpOptions, SharpPlanInfo, check, lib


def _ptr(t: torch.Tensor) -> c_void_p:
    return c_void_p(t.data_ptr())


def _need(t: torch.Tensor, dtype, shape, device, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected {dtype} {tuple(shape)}, got {t.dtype} {tuple(t.shape)}")
    if t.device != device:
        raise ValueError(f"{name}: expected device {device}, got {t.device}")
    return t.contiguous()


class Plan:
    """One scan: object ny x nx, K frames of m x m at integer positions (y, x).

    Parameters follow the paper's inputs (algorithm box, step 1) and user
    options (Sec. "Computational Methodology")."""

    def __init__(self, nx: int, ny: int, m: int, positions, periodic: bool = False, probe_every: int = 0,
                 probe_start: int = 1, eps_D: float = 0.0, tile: int = 0, merge_split: int = 0,
                 grad_groups: int = 0, frame_launch: int = 0, fft_block: int = 0, strip_rows: int = 0,
                 probe_center: bool = False, device="cuda"):
        pos = np.ascontiguousarray(np.asarray(positions), dtype=np.int32)
        if pos.ndim != 2 or pos.shape[1] != 2:
            raise ValueError("positions must be (K, 2) (y, x)")
        self.nx, self.ny, self.m, self.K = int(nx), int(ny), int(m), int(pos.shape[0])
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        opts = SharpOptions(int(periodic), int(probe_every), int(probe_start), float(eps_D), int(tile),
                            int(merge_split), int(grad_groups), int(frame_launch), int(fft_block), int(strip_rows),
                            int(bool(probe_center)))
        h = c_void_p()
        check(lib.sharp_plan_create(byref(h), self.nx, self.ny, self.m, self.K,
                                    pos.ctypes.data_as(POINTER(c_int32)), byref(opts)), "sharp_plan_create")
        self._h = h
        self._destroy = lib.sharp_plan_destroy   # bound now: usable while the interpreter shuts down
        self.positions = pos
        nbytes = lib.sharp_workspace_bytes(h)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._stream()
        check(lib.sharp_set_workspace(h, _ptr(self.workspace), nbytes), "sharp_set_workspace")

    @classmethod
    def tuned(cls, nx: int, ny: int, m: int, positions, kind: str = "raar", periodic: bool = False, **kw):
        """A plan with the launch options the autotuner stored for this geometry
        (library defaults when the geometry has not been tuned)."""
        from .autotune import lookup
        opts = dict(lookup(kind, nx, ny, m, positions, periodic))
        opts.update(kw)
        return cls(nx, ny, m, positions, periodic=periodic, **opts)

    # -- plumbing ---------------------------------------------------------
    @property
    def handle(self) -> c_void_p:
        return self._h

    def _stream(self):
        s = torch.cuda.current_stream(self.device)
        check(lib.sharp_set_stream(self._h, c_void_p(s.cuda_stream)), "sharp_set_stream")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                torch.cuda.synchronize(self.device)
            except Exception:
                pass
            self._destroy(h)
            self._h = c_void_p()

    def info(self) -> dict:
        i = SharpPlanInfo()
        check(lib.sharp_get_plan_info(self._h, byref(i)), "sharp_get_plan_info")
        return {k: getattr(i, k) for k, _ in SharpPlanInfo._fields_}

    # -- inputs -----------------------------------------------------------
    def set_data(self, I: torch.Tensor):
        I = _need(I, torch.float32, (self.K, self.m, self.m), self.device, "I")
        self._stream()
        check(lib.sharp_set_data(self._h, _ptr(I)), "sharp_set_data")
        self._keep = I
        return self

    def set_probe(self, w: torch.Tensor):
        w = _need(w, torch.complex64, (self.m, self.m), self.device, "w")
        self._stream()
        check(lib.sharp_set_probe(self._h, _ptr(w)), "sharp_set_probe")
        self._keep_w = w
        return self

    def init_probe(self):
        self._stream()
        check(lib.sharp_init_probe(self._h), "sharp_init_probe")
        return self

    def set_probe_constraint(self, mask: torch.Tensor | None = None, amplitudes: torch.Tensor | None = None):
        """Fourier mask m_w (takes precedence) or Fourier amplitudes a_w applied
        after every probe update (algorithm box, step 7); neither = no constraint."""
        vals = mask if mask is not None else amplitudes
        kind = 1 if mask is not None else 2 if amplitudes is not None else 0
        ptr = None
        if vals is not None:
            vals = _need(vals, torch.float32, (self.m, self.m), self.device, "mask" if kind == 1 else "amplitudes")
            ptr = _ptr(vals)
        self._stream()
        check(lib.sharp_set_probe_constraint(self._h, kind, ptr), "sharp_set_probe_constraint")
        return self

    def set_object(self, psi: torch.Tensor):
        psi = _need(psi, torch.complex64, (self.ny, self.nx), self.device, "psi")
        self._stream()
        check(lib.sharp_set_object(self._h, _ptr(psi)), "sharp_set_object")
        self._keep_psi = psi
        return self

    # -- iterate / outputs --------------------------------------------------
    def raar(self, n: int, beta: float = 0.75):
        self._stream()
        check(lib.sharp_raar_iterate(self._h, int(n), c_float(beta)), "sharp_raar_iterate")
        return self

    def object(self) -> torch.Tensor:
        out = torch.empty((self.ny, self.nx), dtype=torch.complex64, device=self.device)
        self._stream()
        check(lib.sharp_get_object(self._h, _ptr(out)), "sharp_get_object")
        return out

    def probe(self) -> torch.Tensor:
        out = torch.empty((self.m, self.m), dtype=torch.complex64, device=self.device)
        self._stream()
        check(lib.sharp_get_probe(self._h, _ptr(out)), "sharp_get_probe")
        return out

    def metrics(self, max_n: int = 4096) -> np.ndarray:
        buf = (c_float * max_n)()
        n = c_int()
        self._stream()
        check(lib.sharp_get_metrics(self._h, buf, max_n, byref(n)), "sharp_get_metrics")
        return np.array(buf[: n.value], dtype=np.float32)

    def sync(self):
        self._stream()
        check(lib.sharp_sync(self._h), "sharp_sync")

    # -- gradient / forward model / operators ---------------------------------
    def grad(self, psi: torch.Tensor, w: torch.Tensor, want_psi: bool = True, want_w: bool = True):
        psi = _need(psi, torch.complex64, (self.ny, self.nx), self.device, "psi")
        w = _need(w, torch.complex64, (self.m, self.m), self.device, "w")
        loss = torch.empty((), dtype=torch.float32, device=self.device)
        gpsi = torch.empty_like(psi) if want_psi else None
        gw = torch.empty_like(w) if want_w else None
        self._stream()
        check(lib.sharp_grad(self._h, _ptr(psi), _ptr(w), _ptr(loss),
                             _ptr(gpsi) if gpsi is not None else None,
                             _ptr(gw) if gw is not None else None), "sharp_grad")
        return loss, gpsi, gw

    def simulate(self, psi: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
        psi = _need(psi, torch.complex64, (self.ny, self.nx), self.device, "psi")
        w = _need(w, torch.complex64, (self.m, self.m), self.device, "w")
        out = torch.empty((self.K, self.m, self.m), dtype=torch.float32, device=self.device)
        self._stream()
        check(lib.sharp_simulate(self._h, _ptr(psi), _ptr(w), _ptr(out)), "sharp_simulate")
        return out

    def apply(self, op: str, x: torch.Tensor) -> torch.Tensor:
        frames = (self.K, self.m, self.m)
        obj = (self.ny, self.nx)
        in_shape, out_shape = {
            "F": (frames, frames), "FINV": (frames, frames), "Q": (obj, frames), "QSTAR": (frames, obj),
            "PA": (frames, frames), "PQ": (frames, frames), "OBJECT": (frames, obj)}[op]
        x = _need(x, torch.complex64, in_shape, self.device, "x")
        out = torch.empty(out_shape, dtype=torch.complex64, device=self.device)
        self._stream()
        check(lib.sharp_apply(self._h, OPS[op], _ptr(x), _ptr(out)), f"sharp_apply({op})")
        return out

    # -- kernel timing -------------------------------------------------------
    TIMER_NAMES = ("frame", "cols", "frame_out", "merge", "reduce", "probe", "copy", "spare")

    def timing(self, on: bool = True):
        check(lib.sharp_timing_enable(self._h, int(on)), "sharp_timing_enable")
        return self

    def timing_read(self) -> dict:
        import ctypes
        ms = (ctypes.c_double * 8)()
        n = (ctypes.c_longlong * 8)()
        self._stream()
        check(lib.sharp_timing_read(self._h, ms, n), "sharp_timing_read")
        return {name: (ms[i], n[i]) for i, name in enumerate(self.TIMER_NAMES) if n[i]}

    # -- checkpoint ----------------------------------------------------------
    def state(self) -> torch.Tensor:
        buf = torch.empty(lib.sharp_state_bytes(self._h), dtype=torch.uint8, device=self.device)
        self._stream()
        check(lib.sharp_get_state(self._h, _ptr(buf)), "sharp_get_state")
        return buf

    def load_state(self, buf: torch.Tensor):
        buf = _need(buf, torch.uint8, (lib.sharp_state_bytes(self._h),), self.device, "state")
        self._stream()
        check(lib.sharp_set_state(self._h, _ptr(buf)), "sharp_set_state")
        return self

    def state_parts(self, buf: torch.Tensor) -> dict:
        """Views of the documented state segments (see sharp_get_state)."""
        def up(v):
            return (v + 255) // 256 * 256
        sizes = [("u", self.K * self.m * self.m, torch.complex64), ("psi_v", self.nx * self.ny, torch.complex64),
                 ("psi_l", self.nx * self.ny, torch.complex64), ("w", self.m * self.m, torch.complex64),
                 ("w_g", self.m * self.m, torch.complex64), ("hist", 4096, torch.float32)]
        out, off = {}, 0
        for name, n, dt in sizes:
            nbytes = n * (8 if dt == torch.complex64 else 4)
            out[name] = buf[off:off + nbytes].view(dt)
            off = up(off + nbytes)
        out["u"] = out["u"].view(self.K, self.m, self.m)
        out["psi_v"] = out["psi_v"].view(self.ny, self.nx)
        out["psi_l"] = out["psi_l"].view(self.ny, self.nx)
        out["w"] = out["w"].view(self.m, self.m)
        out["w_g"] = out["w_g"].view(self.m, self.m)
        return out

    def csr(self):
        info = self.info()
        ptr = np.zeros(info["tiles_x"] * info["tiles_y"] + 1, np.int32)
        fr = np.zeros(max(info["csr_nnz"], 1), np.int32)
        P = POINTER(c_int32)
        check(lib.sharp_get_plan_csr(self._h, ptr.ctypes.data_as(P), fr.ctypes.data_as(P)), "sharp_get_plan_csr")
        return ptr, fr[: info["csr_nnz"]]
