"""Polynomial-preconditioned GMRES(m) on MI355X (gfx950).

The compute path is the HIP library ``libpp`` built from ``csrc/``; this
package holds its thin Python binding (``binding``), a torch autograd wrapper
(``autograd``) and the seeded workload generators (``workloads``).  The
binding is imported lazily so that ``workloads`` can be used without the
shared library.
"""
__all__ = ["workloads"]
