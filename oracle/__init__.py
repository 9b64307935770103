"""FP64 CPU oracle for the Laplace-domain elastodynamic BEM solve and the
frequency-domain drivers on top of it (FSM inversion, vector fitting, AFS) and
the warm-start network.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library ``paper_1511_04355_amd`` and neither imports the
other; the two meet only in the seeded inputs of ``synth``.

Modules:
  bem  -- fundamental solutions, element integrals, collocation assembly,
          dense LU and GMRES solves (paper Section 2.1, Eq. 1-2)
  fsm  -- Fourier-series inversion by direct summation (Section 2.2, Eq. 3-4)
  vf   -- vector fitting (Section 2.3, Eq. 5-6)
  afs  -- adaptive frequency sampling (Section 3, Eq. 7-14 and the Algorithm)
  mlp  -- plain FP64 multilayer perceptron, forward/backward/Adam
"""
from . import bem, fsm, vf, afs, mlp  # noqa: F401
