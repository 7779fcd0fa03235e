"""Many independent scans iterated together: one launch sequence per
iteration for all scans, captured once into a hipGraph and replayed."""
from __future__ import annotations

from ctypes import byref, c_float, c_void_p

import torch

from ._lib import check, lib


class Batch:
    """``Batch([plan, ...]).raar(n, beta)`` runs n RAAR iterations of every
    plan.  Each plan must have data, probe and object set and no probe
    refinement; plans keep their own state (read them with plan.object()).
    The plans must outlive the batch."""

    def __init__(self, plans, device=None):
        self.plans = list(plans)
        if not self.plans:
            raise ValueError("empty batch")
        self.device = device or self.plans[0].device
        arr = (c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        h = c_void_p()
        check(lib.sharp_batch_create(byref(h), len(self.plans), arr), "sharp_batch_create")
        self._h = h
        self._destroy = lib.sharp_batch_destroy   # bound now: usable while the interpreter shuts down
        nbytes = max(int(lib.sharp_batch_workspace_bytes(h)), 256)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._stream()
        check(lib.sharp_batch_set_workspace(h, c_void_p(self.workspace.data_ptr()), nbytes),
              "sharp_batch_set_workspace")

    def _stream(self):
        s = torch.cuda.current_stream(self.device)
        check(lib.sharp_batch_set_stream(self._h, c_void_p(s.cuda_stream)), "sharp_batch_set_stream")

    def raar(self, n: int, beta: float = 0.75):
        self._stream()
        check(lib.sharp_batch_raar_iterate(self._h, int(n), c_float(beta)), "sharp_batch_raar_iterate")
        return self

    @property
    def frames(self) -> int:
        return sum(p.K for p in self.plans)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                torch.cuda.synchronize(self.device)
            except Exception:
                pass
            self._destroy(h)
            self._h = c_void_p()
