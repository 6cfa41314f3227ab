"""Plain FP64 CPU oracle of the Sakurai-Sugiura shifted-CG eigensolver.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute anything under this package; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it. It shares no code with the HIP library:
the only common module is `synth`, which draws the random inputs.

Contents (each function cites the passage of the paper it follows):
  wilson      explicit sparse Hermitian Wilson matrix A = gamma5 (I - kappa D)
              (Sec. 4) and the free-field spectrum used to pin it.
  quadrature  nodes, normalised nodes and weights on the two horizontal lines
              (Sec. 3) and on the circle (Sec. 2.1, after eq. 2); filter eq. (3).
  solvers     per-shift direct solves of eq. (4) and the shifted CG method
              (Sec. 2.2, eq. 5 and the Hermitian-seed argument).
  ss          moments eq. (2), Rayleigh-Ritz and Hankel extraction (Sec. 2.1),
              acceptance rule (Sec. 3).
"""
