"""MI355X-native spacetime-multigrid (STFAS) keyframe smoke control.

The solver is the HIP library libstfas.so (csrc/), reached through its C
interface (include/stfas.h, include/stfas_ops.h); `stfas` is the Python
binding with the same names, `autograd` wraps one simulation step as a
torch.autograd.Function, and `serving` is the continuous-batching request
loop.
"""
from . import _lib  # noqa: F401

__all__ = ["stfas", "autograd", "serving", "build"]
