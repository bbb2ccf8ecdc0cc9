"""FP64 CPU oracle for the randomized high-order t-SVT (test infrastructure only).

This package is the plain, slow, obviously-correct reference that the HIP path is
checked against.  It is test infrastructure: only the test suite, the smoke entry
point and the CPU-baseline leg of the benchmark may import it.  The product path
(the C-ABI library and its Python binding) never calls into it.

It shares no code with the HIP path.  The only thing both sides agree on is the
definition of the counter-based Gaussian generator that draws the sketch matrices
(Philox4x32-10 + Box-Muller), which each side implements on its own from the
published definition.

Modules
-------
philox      Philox4x32-10 and the Gaussian test matrices Omega.
transforms  transform matrices, mode-k products, the invertible transform L and
            its inverse, face slices, t-product and T-SVD (Sec. II).
prox        scalar proximity operators of the nonconvex penalties (Sec. IV-B).
tsvt        deterministic GNHTSVT (Def. 4.3, Alg. 4 deterministic branch) and the
            per-slice randomized t-SVT (sketch, power iterations, small SVD).
solver      pure low-rank-prior ADMM for completion and robust completion (Sec. V).
mlp         FP64 reference of the rank-predictor MLP (forward/backward/Adam).

Parity status of every function is listed in its docstring; functions without an
independent pin say "parity unpinned".
"""
