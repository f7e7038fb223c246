"""MI355X (gfx950) block-step Hermite N-body hot path.

``abi``  -- ctypes binding of libnbody.so (the C-ABI of include/nbody.h);
``sim``  -- Simulation and Batch, thin PyTorch-memory front ends over it;
``build_lib`` -- compiles the HIP sources in-tree.
"""
from . import abi  # noqa: F401

__all__ = ["abi", "Simulation", "Batch"]


def __getattr__(name):
    if name in ("Simulation", "Batch"):
        from . import sim
        return getattr(sim, name)
    raise AttributeError(name)
