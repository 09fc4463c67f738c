"""Plain FP64 CPU oracle for the randomized LU decomposition (Shabat et al.,
arXiv 1310.7202, Section 4: Algorithm 4.1 in ``rlu``, Algorithm 4.4 in
``fast``).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.
The product path (the HIP library and its Python binding) never calls it and
shares no code with it: no kernels, no helpers, no constants.

Every function is written to be read against the paper: no blocking, no
fusion, no reordering beyond what the algorithm states.  Floating point is
IEEE binary64 throughout (NumPy / LAPACK via NumPy and SciPy).

Pinned by (see ``tests/test_oracle_*.py``):
  * ``rlu.randomized_lu``      -- exact rank-k reconstruction, Eckart-Young
    lower bound, Theorem 4.1 upper bound, the projection identity of the
    proof of Theorem 4.1, oversampling invariance under partial pivoting,
    LAPACK getrf special cases, SciPy/NumPy least squares, full-rank
    reconstruction, and exact-rational Schur-complement brute force.
  * ``rlu.lu_partial_pivot``   -- LAPACK getrf (SciPy) and the closed-form
    block elimination, in exact rational arithmetic on tiny inputs.
  * ``rlu.lu_col_pivot``       -- LAPACK getrf of the transpose (pivots) and
    the closed-form Schur complement.
  * ``rlu.power_sketch_plain`` -- Section 5.2, (A A^T)^q A G for small q:
    the closed form U S^(2q+1) V^T G of a matrix built from its SVD.
  * ``rlu.power_sketch_normalized`` -- Section 5.2's normalized scheme (a
    reading): the same pivots and factors as the plain product (the
    normalization is a right triangular factor); q = 0 is Step 2; exact
    rank-k reconstruction; the error falls with q on the paper's slowly
    decaying spectrum.
  * ``rlu.power_sketch``       -- plain up to PLAIN_POWER_MAX_Q, normalized
    above (both pinned above).
  * ``rlu.lu_normalize``       -- LAPACK getrf: P L from scipy.linalg.lu.
  * ``rlu.lstsq_rank_deficient`` -- Algorithm 4.3: consistent rank-k systems
    solved with at most k nonzeros; the residual equals LAPACK's least-squares
    minimum (numpy.linalg.lstsq); A^{-1} b in the full-rank square case.
  * ``rlu.upper_solve``        -- SciPy solve_triangular; a zero row gives 0.
  * ``rlu.spectral_norm_estimate``, ``rlu.residual(exact=False)``,
    ``rlu._power_norm`` -- exact SVD values (to 1e-6 relative) with a clear
    top gap, a clustered top and the paper's slow decay; the lower-bound
    property; the residual operator against the formed difference.
  * ``rlu.pivot_gate``         -- constructed diagnostics on either side of
    each threshold; exact ties and rank deficiency; LAPACK's pivots on the
    gated prefix.
  * ``rlu.kappa``              -- closed forms (diagonal, orthogonal, SVD
    construction) and the Gram-route accuracy it predicts.
  * ``rlu.column_pivoted_qr``, ``rlu.rrlu`` -- the rank-revealing Step 3:
    LAPACK geqp3's column order, each pivot the largest remaining column,
    the inequalities of Theorem 3.1, exact rank, the projection identity,
    the mean error below partial pivoting's when l > k.
  * ``fast.*`` (Algorithm 4.4) -- the SRFT draws (balanced signs, uniform
    distinct selection), the Hartley transform against NumPy's FFT, the
    ID's defining properties and the inequality of its lemma's proof,
    exact rank, Eckart-Young, Step 6 against NumPy least squares.
  * ``philox.srft_signs``, ``philox.srft_selection`` -- with the pins above.
  * ``bounds.xi``              -- Table 4.1 of the paper, 9 of 9 rows.
  * ``philox.philox4x32_10``   -- Random123 known-answer vectors.
  * ``philox.gaussian_matrix`` -- Box-Muller closed form on fixed uniforms and
    moment / Kolmogorov-Smirnov checks.
Parity unpinned: nothing in this package (every function has a pin above).
"""
