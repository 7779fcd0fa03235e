"""MI355X-native RAAR ptychography hot path (SHARP, arXiv:1602.01448).

`Plan` wraps one scan; `AmplitudeLoss` exposes the hand-written adjoint as a
torch.autograd.Function; `Batch` runs many independent scans together.  All
computation happens in libsharp.so (HIP, gfx950); this package only moves
pointers and sizes across the C ABI.
"""
from ._lib import OPS, SharpError, load  # noqa: F401
from .plan import Plan  # noqa: F401
from .autograd import AmplitudeLoss  # noqa: F401
from .batch import Batch  # noqa: F401
