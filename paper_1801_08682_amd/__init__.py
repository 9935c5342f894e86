"""MI355X-native ADER-DG time step (arXiv:1801.08682, Charrier & Weinzierl).

Hot path: hand-written HIP kernels for gfx950 behind the C ABI of
include/adg.h (libadg.so).  This package adds only the ctypes binding
(``_lib``), a torch-buffer stepper (``stepper``), seeded inputs (``inputs``),
the reverse-mode rollout (``rollout``) and the build script (``build``).
Nothing here computes a step on the CPU.
"""

__all__ = ["inputs", "Stepper"]


def __getattr__(name):
    if name == "Stepper":
        from .stepper import Stepper
        return Stepper
    raise AttributeError(name)
