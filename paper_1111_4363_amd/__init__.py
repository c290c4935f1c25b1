"""Least-action TDSE relaxation on MI355X: HIP library liblam.so plus binding.

The library implements one propagation step of the least-action method of
Walters ("An efficient parallel method for relaxing to the minimum action
wavefunction"): subvolume relaxation inside a multigrid V-cycle, its adjoint,
and the gradients of a loss with respect to the potential and pulse
amplitudes.  ``lam`` is the ctypes binding; importing this package does not
load the library (``lam.load_library()`` does, and fails loudly if the
library is not built).
"""
from . import lam  # noqa: F401

__all__ = ["lam"]
