"""MI355X-native hot path of F-Hash (arXiv 2507.03836).

The compute path is libfhash.so (hand-written HIP for gfx950) behind the C ABI
in include/fhash.h; `_lib` is its thin ctypes binding and `model` wires the
calls into a training step, an autograd function and inference.
"""
from . import _lib  # noqa: F401

__all__ = ["_lib"]
