"""MI355X (gfx950) block-step Hermite N-body hot path.

``abi``  -- ctypes binding of libnbody.so (the C-ABI of include/nbody.h);
``sim``  -- Simulation, a thin PyTorch-memory front end over it;
``build_lib`` -- compiles the HIP sources in-tree.
"""
from . import abi  # noqa: F401

__all__ = ["abi", "Simulation"]


def __getattr__(name):
    if name == "Simulation":
        from .sim import Simulation
        return Simulation
    raise AttributeError(name)
