"""Plain, slow FP64 CPU oracle for the high-order immersed-interface Poisson solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
this package: only the test-suite, the smoke entry point and the benchmark's
cpu_baseline leg use it.  It shares no code with the HIP library; the only module
both sides import is the seeded input description in ``workloads.py``, which
holds none of the method's arithmetic.

What it computes, each piece following the paper (Gabbard, Paris & van Rees,
"A high order multigrid-preconditioned immersed interface solver for the
Poisson equation with boundary and interface conditions", JCP 2025):

  geometry.py  analytic level sets, node labels, control points (Sec. 2.1)
  fd.py        central second-derivative stencils and sigma(k) (Sec. 2.5, Table 1)
  lsq.py       least-squares ghost stencils per control point (Sec. 2.1-2.2)
  iim.py       the assembled system L_Omega u + L_Gamma u_Gamma = f (Sec. 2.3)
  sw.py        Shortley-Weller discretizations with intersection shifting (Sec. 3.1)
  mg.py        geometric multigrid V-cycle on the SW operator (Sec. 3.3)
  krylov.py    right-preconditioned FGMRES(m) (Sec. 4.1)
  singular.py  the bordered system of pure-Neumann problems (Sec. 2.3)

Every function is written for a reader checking it against the paper by eye:
no blocking, fusion or reordering beyond what the definitions state.
Parity status of each function is recorded in its docstring; functions without
an independent pin say "parity unpinned".
"""

INACTIVE, PLUS, MINUS, BOX = 0, 1, 2, 3
