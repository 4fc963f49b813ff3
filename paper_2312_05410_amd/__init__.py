"""MI355X-native explicit PVD phase-field stepper (arXiv 2312.05410's DNS step).

The compute path is libpf.so (hand-written HIP for gfx950, C ABI in
include/pf.h); `Simulator` is a thin ctypes binding over it that takes device
memory and streams from PyTorch.
"""
from .inputs import PFParams, initial_state, random_state, realisation_draws  # noqa: F401


def __getattr__(name):
    # the binding imports torch; keep `import paper_2312_05410_amd.inputs` light
    if name in ("Simulator", "load", "dt_limit", "workspace_bytes", "PFError"):
        from . import _lib

        return getattr(_lib, name)
    raise AttributeError(name)
