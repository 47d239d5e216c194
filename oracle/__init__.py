"""CPU oracle of the entropy-stable SBP-SAT residual (Rojas et al., arXiv 1911.10966).

TEST INFRASTRUCTURE ONLY. Nothing on the product path may import, call or execute
this package: only the test suite, the smoke check and the benchmark's CPU-baseline
leg use it. It shares no code with the HIP library.

It is a plain, slow, NumPy implementation written from the paper: every function
cites the section or equation it follows, and works for any NumPy scalar type
(float64 for parity, complex128 for complex-step derivatives, longdouble for the
rounding floor). Arrays use the axes (component, element, i3, i2, i1); direction
xi_l (l = 0, 1, 2) is the element-array axis ``3 - l``.

Parity status: every function is pinned by a test in ``tests/test_oracle_*.py``
against the SBP definition, closed forms, textbook special cases, the entropy and
conservation identities the method is built to satisfy, an independent literal
dense-matrix form, symbolic derivatives of the continuous equations, and the
paper's stationary isentropic vortex.
"""
from . import operators, geometry, gas, residual, dense, jvp  # noqa: F401
