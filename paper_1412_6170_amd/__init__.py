"""mknn -- repeated k-NN queries over massive moving 2D objects on MI355X.

The compute path is the HIP library ``libmknn.so`` (built from ``csrc/``)
behind the C ABI declared in ``include/mknn.h``; ``binding`` marshals
arguments to it.  The library is loaded on first use and a missing build
raises immediately: there is no CPU fallback.
"""
__all__ = ["binding", "workloads"]
