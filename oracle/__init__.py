"""CPU oracle for the ISCI sigma step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call or link anything in this package.  The HIP
library never routes through it and shares no code with it.

Contents
--------
isci_oracle.c   plain C: string enumeration, determinant addressing,
                Slater-Condon matrix elements as sums of screened integral
                units with signs from explicit operator manipulation, the
                sigma product, the diagonal, per-bucket term counts, the
                dense Hamiltonian of tiny spaces and the screening bound.
oracle.py       ctypes binding plus numpy pieces: closed-form space
                dimension, dense diagonalisation, a textbook Davidson
                eigensolver on top of the oracle sigma, the closed-form
                reference energy.

Parity status of every function is recorded in its docstring; each one is
pinned by a ``-m "not gpu"`` test against something other than itself.
"""
from .oracle import *  # noqa: F401,F403
