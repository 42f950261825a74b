"""MI355X (gfx950) implementation of the CDNA wavefront-centric execution-time
model: batched prediction, adjoint, device calibration and tile selection.

The HIP library is loaded on first use of the binding; the seeded input
generators (`synth`) import without it.
"""
import importlib

__all__ = ["synth", "wavemodel"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
