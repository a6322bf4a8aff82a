"""MI355X (gfx950) implementation of the projection method's hot path:
the diagonally preconditioned Krylov solve of the lifted Fourier-Galerkin
system of a quasiperiodic elliptic problem, its correctors and the
homogenized coefficient.

* ``qp``        -- ctypes binding of libqp.so (C ABI in include/qp.h)
* ``workloads`` -- seeded synthetic inputs (no method arithmetic)
* ``build``     -- hipcc build of libqp.so
"""
from . import workloads  # noqa: F401

__all__ = ["workloads"]
