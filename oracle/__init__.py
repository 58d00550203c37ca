"""Plain FP64 CPU oracle for the energy-stable phase-field-crystal (PFC) scheme.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
anything in this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library; the only module both sides use is ``pfc_inputs`` (seeded initial
conditions, which hold none of the method's arithmetic).

Modules
-------
``scheme``   grid operators, discrete energy, the discrete variational derivative
             and the semi-implicit residual (Sec. 3, Eqs. (7)-(12)), the exact
             Jacobian (Sec. 4, Eq. (19)), Newton with an exact sparse direct solve
             (Sec. 4, Eqs. (17)-(20)) and adaptive time stepping (Sec. 3, Eq. (16)).
``schwarz``  reference routines for the solver pieces that are approximations
             rather than definitions: the overlapping decomposition, the Schwarz
             preconditioners (Sec. 4, Eqs. (22)-(26)), textbook ILU(0),
             right-preconditioned (F)GMRES (Sec. 4, Eq. (21)) and the inexact
             Newton-Krylov-Schwarz time step they make up (Eqs. (17)-(24)).
``cnn``      FP64 reference of the small convolutional network used as a learned
             Newton initial guess (forward, hand-written backward, Adam).

Parity status: every function is pinned by ``tests/test_oracle_*.py`` against
closed forms, exact identities of the paper, brute force or library routines,
except the ones whose header says "parity unpinned".
"""
