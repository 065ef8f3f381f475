"""MI355X-native DROT: Douglas-Rachford splitting for discrete optimal
transport, with the dense per-iteration sweep in hand-written HIP kernels for
gfx950 behind the C ABI of include/drot.h (libdrot.so).

    from paper_2110_11738_amd import drot
    X, result, mu, nu = drot.solve(C, p, q, rho, tol)
"""
from . import drot  # noqa: F401

__all__ = ["drot"]
