"""Independent CPU oracle for the variable-coefficient Stokes solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import, call, link or execute
anything in this package.  It shares no code with the HIP library under
``paper_1901_07892_amd/`` and never imports it; the only module both use is
``workloads`` (seeded input generation, none of the solver's arithmetic).

Contents
  assemble.py      O1  the discrete system as one sparse matrix (definition)
  direct.py        O5  dense / SuperLU solves of that matrix, zero-mean pressure
  stokes_oracle.c  O2  independent stencil apply
                   O3  FGMRES with modified Gram-Schmidt
                   O4  projection preconditioner, lexicographic Gauss-Seidel
                       multigrid for both subsolves
  native.py        ctypes loader for liboracle.so (built with gcc + OpenMP)
  coefficients.py  the coefficient step: smoothed Heaviside, two-step property
                   law, face densities from level sets averaged onto faces
  unet.py          the learned stage's network (forward pass)
  rigid.py         rigid-body constraint projection after the solve: four-point
                   kernel interpolation and spreading with wall mirrors,
                   prescribed or free-body (momentum-redistributed) motion

Parity of the GPU solve is measured on the solution of the linear system,
never on iterates.  The multigrid inside O4 has no parity of its own
("parity unpinned"): it only decides how fast O3 gets to the solution, which
is pinned by the direct solves.
"""
