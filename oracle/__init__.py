"""Plain, slow FP64 CPU oracle for the PPCG eigensolver.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import anything here.  It shares
no code with the HIP path (``paper_1407_7506_amd``); the only common module is
the seeded input generator ``paper_1407_7506_amd.inputs``, which holds none
of the method's arithmetic.

Modules
  stencil   matrix-free H = -1/2 Lap_h + diag(V) by np.roll, dense assembly
  dense     small dense steps: Cholesky-QR, block pencils, Rayleigh-Ritz
  ppcg_ref  the PPCG iteration (paper, Algorithm 3 with sections 5.1-5.7)
  brute     dense brute-force eigendecomposition for tiny grids
  grad      dL/dV by projected Sternheimer solves and by the dense formula
  rng       the start block from Philox-4x32-10 and Box-Muller

Every function is pinned by a ``-m "not gpu"`` test against something other
than itself (closed forms, brute force, library routines, invariants); see
the module docstrings for what pins each one.
"""
