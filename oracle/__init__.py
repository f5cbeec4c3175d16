"""CPU oracle for adaptive black-hole ray tracing (Gelles et al. 2021).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call, link or execute anything
in this package.  The product library never routes through it; it shares no
code with the HIP path (the two implement the written method independently).

Modules
  ray.py      ctypes binding of ray_oracle.c (per-ray geodesic + transfer, FP64)
  refine.py   the paper's level-by-level refinement (Sec. 3.2, Eqs. 5-6, App. A)
  metrics.py  interpolation fraction, flux error, normalised MSE (Sec. 4.1,
              Eqs. 7-9)
  build.py    compiles ray_oracle.c with gcc
"""
