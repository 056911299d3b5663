"""qvpu: batched state-vector circuits, Pauli-sum expectations and adjoint gradients on one MI355X.

Importing the package loads nothing native; the HIP library is loaded on first use through
``paper_2406_03466_amd.qvpu`` (ctypes binding of the C interface declared in include/qvpu.h).
"""
__all__ = ["workloads"]
