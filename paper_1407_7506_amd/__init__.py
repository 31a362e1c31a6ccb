"""libppcg: MI355X-native hot path of the PPCG eigensolver
(Vecharynski, Yang, Pask, "A Projected Preconditioned Conjugate Gradient
Algorithm for Computing Many Extreme Eigenpairs of a Hermitian Matrix").

Importing the package loads nothing native.  The ctypes binding in
``paper_1407_7506_amd.binding`` loads ``libppcg.so`` on first use and raises
if it is missing; there is no CPU fallback.
"""

__all__ = ["inputs", "binding"]
