"""MI355X-native short-range Lennard-Jones MD hot path (gfx950 HIP behind a C ABI).

Submodules: ops (one wrapper per C entry point), md (timestep loop),
autograd (differentiable forces), trajectory (checkpointed backprop through
short trajectories).  Importing the package loads nothing; the HIP library
is loaded on first use and its absence is an error.
"""
__all__ = ["ops", "md", "autograd", "trajectory", "build"]
