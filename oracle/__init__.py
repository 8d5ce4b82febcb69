"""FP64 CPU oracle for the XTRG beta-doubling step -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct NumPy implementation of what the HIP library
computes, written from the paper (Chen, Chen, Chen, Li, Weichselbaum,
"Exponential thermal tensor network approach for quantum lattice models").
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or run anything in this package.  The product path
(``paper_1801_00142_amd``) never imports it, and this package imports nothing
from the product path: the two share only the input descriptions in
``workloads.py``.

Modules
  ed           exact diagonalisation: dense H as a sum of Kronecker products
  mpo          automaton Hamiltonian MPO (App. B.1) and plain MPO algebra
  xtrg         initial state (Sec. II.C, Eq. RhoTau; App. C.2), variational product
               compression (App. D.1, Eq. LSEProd, Fig. VMPO), doubling
               (Eqs. rhoinit, rho:scale2), observables (Eq. ThermalQuan),
               MPO entanglement (Eq. purif)
  closed_forms XY-chain partition function (App. F), high-T series,
               closed forms of Tr and Frobenius norm of I - tau H

Every function states the passage it follows.  Pins (tests/test_oracle_*.py)
tie each part to something other than the oracle itself: exact
diagonalisation, closed forms, brute force on tiny inputs, invariants.
"""
