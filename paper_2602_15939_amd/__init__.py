"""MI355X (gfx950) particle hot path of the extended particle-in-cell methods of
Bacchini et al. (arXiv 2602.15939): shearing box with orbital advection, expanding box
and leaky box, behind the C ABI of include/pic.h.

The compute runs in the HIP library ``libpic.so`` (built by ``build.py``); this package
only marshals arguments (``_lib``), wraps a box (``box.Box``) and generates seeded
synthetic inputs (``synth``).
"""
from . import _lib  # noqa: F401

__all__ = ["_lib", "box", "synth", "build"]
