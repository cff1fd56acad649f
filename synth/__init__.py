"""Seeded synthetic inputs shaped like the semiconductor/insulator cells of the
all-electron periodic G0W0 study (Ren et al., arXiv:2011.01400).

This package only draws random numbers and packs them into the arrays the
method takes as inputs (eigenvalues, eigenvectors, real-space LRI triple
coefficients, Coulomb matrices, momentum matrix elements).  It holds none of
the method's arithmetic: no Fourier transform, no product-basis transform, no
response function, no screening, no frequency grid.  Both the FP64 oracle and
the HIP path read the same generated arrays.
"""
from .systems import CellSpec, System, CONFIGS, make_system, make_config  # noqa: F401
