"""FP64 CPU oracle for the deterministic neural-backflow NQS hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_2601_21310_amd``) never imports it, and the two share no code; the only
module both use is ``synth`` (seeded input generation, none of the method's
arithmetic).

Modules
-------
hamiltonian  Slater-Condon elements, H_SS, excitations, operator-algebra dense H,
             PT2 external sum (plain C in ``sc_oracle.c`` via ctypes)
ansatz       neural backflow amplitude psi(x) = det A(x), Eqs. 2-4 (torch, float64)
energy       variational energy and gradient, Eqs. 11-12 (torch autograd, float64)
pt2          Epstein-Nesbet correction, Eq. 13
fci          exact diagonalisation of a dense H (numpy eigh)
"""
