"""FP64 CPU oracle of Algorithm 4.1 (randomized LU) of Shabat et al.,
arXiv 1310.7202, Section 4.

TEST INFRASTRUCTURE ONLY: see the package docstring for who may call this.

Conventions (the paper uses permutation matrices, Section 3.1, Eq. 3.1; this
oracle uses 0-based index vectors with the same meaning):
  * ``p`` (length m):  (P A)(i, :) = A(p[i], :)
  * ``q`` (length n):  (A Q)(:, j) = A(:, q[j])
  * ``ipiv[j]`` / ``qpiv[j]``: LAPACK-style swap sequence -- at step j the
    row (column) at position j was exchanged with the one at position
    ipiv[j] (qpiv[j]).

Readings of the paper taken here (where the paper is silent or leaves a choice):
  * Step 3 uses LU with partial pivoting (the Remark after Algorithm 4.1
    allows it in place of RRLU), factoring all l columns of Y; Step 4 then
    keeps the first k columns of L_y.
  * Ties in a pivot search go to the lowest current position (LAPACK i?amax).
  * A zero pivot (whole active column zero) is recorded in ``info`` as the
    1-based step, and that step's scaling and update are skipped, as in
    LAPACK getf2; the factorization continues.
  * Step 5's pseudo-inverse is applied as a least-squares solve through a
    Householder QR of L_y.  The paper's Remark forms (L_y^T L_y)^{-1} L_y^T;
    the two agree in exact arithmetic and the QR route is the more accurate
    reference.
  * Step 6 is row-by-row elimination with column pivoting; L_b is unit lower
    triangular and U_b carries the pivots.  If a pivot is zero, column j of
    L_b below the diagonal is left zero.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def sketch(A: np.ndarray, G: np.ndarray) -> np.ndarray:
    """Step 2 of Algorithm 4.1: Y = A G (a plain matrix product)."""
    return A @ G


def lu_partial_pivot(Y: np.ndarray):
    """Step 3 of Algorithm 4.1 with partial pivoting (Remark after Alg. 4.1).

    Unblocked right-looking Gaussian elimination on the m x w matrix Y
    (m >= w): at step j the pivot is the entry of largest magnitude in the
    active part of column j (lowest position on ties); the two full rows are
    exchanged; the multipliers are the active column divided by the pivot;
    the trailing block receives the rank-one update.

    Returns (LU, ipiv, p, info, diag) where LU packs the unit-lower factor
    below the diagonal and U on and above it (positions, i.e. rows of P Y),
    and ``diag`` holds per-step pivot diagnostics used to gate pivot
    comparisons: |pivot|, the relative gap to the runner-up, and max |Y|.
    """
    LU = np.array(Y, dtype=np.float64, copy=True)
    m, w = LU.shape
    if w > m:
        raise ValueError("lu_partial_pivot expects a tall matrix (m >= w)")
    ipiv = np.zeros(w, dtype=np.int64)
    p = np.arange(m, dtype=np.int64)
    info = 0
    piv_abs = np.zeros(w)
    gap = np.zeros(w)
    ymax = float(np.max(np.abs(LU))) if LU.size else 0.0
    for j in range(w):
        col = np.abs(LU[j:, j])
        r = j + int(np.argmax(col))
        piv_abs[j] = col[r - j]
        if col.size > 1:
            second = np.partition(col, col.size - 2)[col.size - 2]
            gap[j] = (piv_abs[j] - second) / piv_abs[j] if piv_abs[j] > 0 else 0.0
        else:
            gap[j] = 1.0
        ipiv[j] = r
        if r != j:
            LU[[j, r], :] = LU[[r, j], :]
            p[[j, r]] = p[[r, j]]
        pivot = LU[j, j]
        if pivot != 0.0:
            LU[j + 1:, j] = LU[j + 1:, j] / pivot
            LU[j + 1:, j + 1:] -= np.outer(LU[j + 1:, j], LU[j, j + 1:])
        elif info == 0:
            info = j + 1
    return LU, ipiv, p, info, {"piv_abs": piv_abs, "gap": gap, "max_abs": ymax}


def column_pivoted_qr(Y: np.ndarray, order=None):
    """Householder QR with column pivoting (Businger and Golub), the column
    choice of the rank-revealing Step 3 (Algorithm 4.1 as listed, with the
    RRLU of Section 3.1, Theorem 3.1).

    At step j the remaining column whose part on rows j.. has the largest
    2-norm (lowest current position on ties; norms recomputed at every
    step) is exchanged into position j, and a Householder reflection zeroes
    it below the diagonal and is applied to the columns on its right.

    Returns (R, qy, diag): R (w x w upper triangular) with Y[:, qy] = Q R,
    the column order qy, and per-step diagnostics (largest remaining norm,
    relative gap to the runner-up, and the largest column norm of Y).

    With ``order`` (a column order computed elsewhere) the same steps are
    taken with that order's column at each step instead of the largest, and
    diag["ratio"][j] records its remaining norm over the largest: an order
    is a valid column-pivoted order where every ratio is 1 up to rounding."""
    W = np.array(Y, dtype=np.float64, copy=True)
    m, w = W.shape
    if w > m:
        raise ValueError("column_pivoted_qr expects a tall matrix (m >= w)")
    qy = np.arange(w, dtype=np.int64)
    top = np.zeros(w)
    gap = np.zeros(w)
    ratio = np.ones(w)
    ymax = float(np.max(np.linalg.norm(W, axis=0))) if W.size else 0.0
    for j in range(w):
        norms = np.linalg.norm(W[j:, j:], axis=0)
        c = j + int(np.argmax(norms))
        if order is not None:
            best = norms[c - j]
            c = j + int(np.nonzero(qy[j:] == order[j])[0][0])
            ratio[j] = norms[c - j] / best if best > 0 else 1.0
        top[j] = norms[c - j]
        if norms.size > 1:
            second = np.partition(norms, norms.size - 2)[norms.size - 2]
            gap[j] = (top[j] - second) / top[j] if top[j] > 0 else 0.0
        else:
            gap[j] = 1.0
        if c != j:
            W[:, [j, c]] = W[:, [c, j]]
            qy[[j, c]] = qy[[c, j]]
        x = W[j:, j]
        nx = np.linalg.norm(x)
        if nx == 0.0:
            continue
        alpha = -nx if x[0] >= 0 else nx
        v = x.copy()
        v[0] -= alpha
        v /= np.linalg.norm(v)
        W[j:, j:] -= 2.0 * np.outer(v, v @ W[j:, j:])
    R = np.triu(W[:w, :w])
    return R, qy, {"piv_abs": top, "gap": gap, "max_abs": ymax, "ratio": ratio}


def rrlu(Y: np.ndarray, order=None):
    """The rank-revealing Step 3 of Algorithm 4.1 as listed: P Y Q_y =
    L_y U_y with the column permutation Q_y of ``column_pivoted_qr`` and
    the partial-pivot LU (``lu_partial_pivot``) of Y Q_y, all columns
    factored.  Returns (LU, ipiv, p, info, diag, qy, qdiag) with LU the
    packed factors of Y[:, qy].  ``order`` as in ``column_pivoted_qr``."""
    _, qy, qdiag = column_pivoted_qr(Y, order)
    LU, ipiv, p, info, diag = lu_partial_pivot(np.asarray(Y)[:, qy])
    return LU, ipiv, p, info, diag, qy, qdiag


def unit_lower(LU: np.ndarray, k: int) -> np.ndarray:
    """Step 4 of Algorithm 4.1: L_y <- L_y(:, 1:k), the unit-lower part of
    the first k columns of the packed factor."""
    m = LU.shape[0]
    L = np.tril(LU[:, :k], -1)
    L[np.arange(k), np.arange(k)] = 1.0
    return L[:m, :k]


def pinv_apply(Ly: np.ndarray, PA: np.ndarray) -> np.ndarray:
    """Step 5 of Algorithm 4.1: B = L_y^dagger (P A).

    L_y has full column rank (unit diagonal), so its pseudo-inverse is the
    least-squares solution operator; it is applied through the reduced
    Householder QR  L_y = Q R:  B = R^{-1} Q^T (P A).
    """
    Q, R = np.linalg.qr(Ly, mode="reduced")
    return scipy.linalg.solve_triangular(R, Q.T @ PA, lower=False)


def lu_col_pivot(B: np.ndarray):
    """Step 6 of Algorithm 4.1: LU of the k x n matrix B with column
    pivoting, B Q = L_b U_b (k <= n).

    Row-by-row elimination: at step j the pivot is the entry of largest
    magnitude in the active part of row j (lowest position on ties); the two
    full columns are exchanged; the entries of column j below the pivot are
    divided by it to give column j of L_b, and the trailing rows receive the
    rank-one update.  U_b is the upper-trapezoidal part of the result.

    Returns (Lb, Ub, qpiv, q, info, diag).
    """
    W = np.array(B, dtype=np.float64, copy=True)
    k, n = W.shape
    if k > n:
        raise ValueError("lu_col_pivot expects a wide matrix (k <= n)")
    Lb = np.eye(k)
    qpiv = np.zeros(k, dtype=np.int64)
    q = np.arange(n, dtype=np.int64)
    info = 0
    piv_abs = np.zeros(k)
    gap = np.zeros(k)
    bmax = float(np.max(np.abs(W))) if W.size else 0.0
    for j in range(k):
        row = np.abs(W[j, j:])
        c = j + int(np.argmax(row))
        piv_abs[j] = row[c - j]
        if row.size > 1:
            second = np.partition(row, row.size - 2)[row.size - 2]
            gap[j] = (piv_abs[j] - second) / piv_abs[j] if piv_abs[j] > 0 else 0.0
        else:
            gap[j] = 1.0
        qpiv[j] = c
        if c != j:
            W[:, [j, c]] = W[:, [c, j]]
            q[[j, c]] = q[[c, j]]
        pivot = W[j, j]
        if pivot != 0.0:
            Lb[j + 1:, j] = W[j + 1:, j] / pivot
            W[j + 1:, j:] -= np.outer(Lb[j + 1:, j], W[j, j:])
        elif info == 0:
            info = j + 1
    Ub = np.triu(W)
    return Lb, Ub, qpiv, q, info, {"piv_abs": piv_abs, "gap": gap, "max_abs": bmax}


def lu_normalize(X: np.ndarray) -> np.ndarray:
    """The normalization of the power scheme (Section 5.2): X (tall, w
    columns) is replaced by the unit-lower factor of its partial-pivot LU
    (the factorization of Step 3), put back in X's own row order, i.e.
    P^T L where P X = L U.  When U is nonsingular this equals X U^{-1}: the
    same column space, with every entry bounded by 1 in magnitude."""
    LU, _, p, _, _ = lu_partial_pivot(X)
    L = unit_lower(LU, X.shape[1])
    out = np.empty_like(L)
    out[p, :] = L
    return out


# Section 5.2 replaces Step 2 by Y = (A A^*)^q A G for a small integer q and
# asks for a normalized scheme for larger q.  Up to this q the oracle forms
# the plain product; above it, the normalized scheme.
PLAIN_POWER_MAX_Q = 2


def power_sketch_plain(A: np.ndarray, G: np.ndarray, q: int) -> np.ndarray:
    """Y = (A A^T)^q A G by plain products, no normalization (Section 5.2
    for small q)."""
    if q < 0:
        raise ValueError("q must be >= 0")
    Y = sketch(A, G)
    for _ in range(q):
        Y = A @ (A.T @ Y)
    return Y


def power_sketch_normalized(A: np.ndarray, G: np.ndarray, q: int) -> np.ndarray:
    """The normalized power scheme (Section 5.2, for larger q): A G is
    followed by q rounds of one product with A^T and one with A, and every
    product except the last is replaced by ``lu_normalize`` of it.  Each
    normalization multiplies the block on the right by an upper-triangular
    matrix, which changes neither the pivots nor the unit-lower factor of
    Step 3, so Steps 3-8 agree with the plain product in exact arithmetic
    (a reading of the paper; pinned against ``power_sketch_plain``)."""
    if q < 0:
        raise ValueError("q must be >= 0")
    Y = sketch(A, G)
    for _ in range(q):
        Y = lu_normalize(Y)
        Z = lu_normalize(A.T @ Y)
        Y = A @ Z
    return Y


def power_sketch(A: np.ndarray, G: np.ndarray, q: int) -> np.ndarray:
    """Step 2 with q power iterations (Section 5.2): Y = (A A^*)^q A G,
    formed plainly for q <= PLAIN_POWER_MAX_Q and by the normalized scheme
    above that."""
    if q <= PLAIN_POWER_MAX_Q:
        return power_sketch_plain(A, G, q)
    return power_sketch_normalized(A, G, q)


def randomized_lu(A: np.ndarray, k: int, l: int, G: np.ndarray, q: int = 0,
                  scheme: str = "auto", step3: str = "partial", order=None) -> dict:
    """Algorithm 4.1 of the paper, Steps 2-8, for a given Gaussian G (Step 1).

    Inputs: A (m x n), k (target rank), l (number of sketch columns,
    k <= l <= min(m, n)), G (n x l) and the number q of power iterations
    of Section 5.2 (0: the plain Step 2).  ``scheme`` picks how the power
    sketch is formed: "plain", "normalized", or "auto" (plain up to
    PLAIN_POWER_MAX_Q, normalized above).  ``step3`` is "partial" (the LU
    with partial pivoting the Remark after Algorithm 4.1 allows) or "rrlu"
    (the rank-revealing LU of the listing, ``rrlu``; ``order`` fixes its
    column order, see ``column_pivoted_qr``).  Returns a dict with the outputs
    L (m x k unit lower trapezoidal), U (k x n upper trapezoidal), p, q and
    the intermediates (Y, packed LU of Y, ipiv, L_y, B, L_b, qpiv, info words
    and pivot diagnostics).
    """
    A = np.asarray(A, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    m, n = A.shape
    if not (1 <= k <= l <= min(m, n)):
        raise ValueError("need 1 <= k <= l <= min(m, n)")
    if G.shape != (n, l):
        raise ValueError("G must be n x l")
    make = {"auto": power_sketch, "plain": power_sketch_plain,
            "normalized": power_sketch_normalized}[scheme]
    Y = make(A, G, q)                                  # Step 2 (Section 5.2)
    return randomized_lu_from_sketch(A, k, Y, step3, order)


def randomized_lu_from_sketch(A: np.ndarray, k: int, Y: np.ndarray,
                              step3: str = "partial", order=None) -> dict:
    """Steps 3-8 of Algorithm 4.1 for a given sketch Y (m x l); ``step3`` as
    in ``randomized_lu``."""
    A = np.asarray(A, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    m, n = A.shape
    if Y.shape[0] != m or not (1 <= k <= Y.shape[1] <= min(m, n)):
        raise ValueError("need an m x l sketch with 1 <= k <= l <= min(m, n)")
    qy, qdiag = None, None
    if step3 == "rrlu":
        LUy, ipiv, p, info_y, diag_y, qy, qdiag = rrlu(Y, order)  # Step 3, P Y Q_y = L_y U_y
    elif step3 == "partial":
        LUy, ipiv, p, info_y, diag_y = lu_partial_pivot(Y)     # Step 3 (Remark)
    else:
        raise ValueError("step3 must be 'partial' or 'rrlu'")
    Ly = unit_lower(LUy, k)                            # Step 4
    B = pinv_apply(Ly, A[p, :])                        # Step 5
    Lb, Ub, qpiv, q, info_b, diag_b = lu_col_pivot(B)  # Step 6
    L = Ly @ Lb                                        # Step 7
    U = Ub                                             # Step 8
    return {
        "L": L, "U": U, "p": p, "q": q,
        "Y": Y, "LUy": LUy, "ipiv": ipiv, "Ly": Ly, "B": B,
        "Lb": Lb, "Ub": Ub, "qpiv": qpiv,
        "info": (info_y, info_b),
        "diag_y": diag_y, "diag_b": diag_b,
        "qy": qy, "diag_qy": qdiag,
    }


def upper_solve(U1: np.ndarray, y: np.ndarray) -> np.ndarray:
    """z_1 = U_1^{-1} y for the k x k upper-triangular U_1 (Step 3 of
    Algorithm 4.3), by back substitution, one right-hand side per column of
    y.  A zero diagonal entry (a zero pivot of Step 6, whose row of U is
    zero) makes z_1[j] a free variable; it is set to 0, as the paper sets
    z_2."""
    k = U1.shape[0]
    y = np.array(y, dtype=np.float64, copy=True).reshape(k, -1)
    z = np.zeros_like(y)
    for j in range(k - 1, -1, -1):
        rhs = y[j] - U1[j, j + 1:] @ z[j + 1:]
        z[j] = rhs / U1[j, j] if U1[j, j] != 0.0 else 0.0
    return z


def lstsq_rank_deficient(out: dict, b: np.ndarray) -> np.ndarray:
    """Algorithm 4.3, Steps 2-5, on the factors of Algorithm 4.1
    (P A Q ~ L U): y = L^dagger P b, z_1 = U_1^{-1} y, z = (z_1; 0),
    x = Q z.  b is m x r (or a vector); returns x (n x r, or a vector).

    L^dagger is applied as a least-squares solve through the QR of L (as in
    Step 5).  With the index-vector conventions of this module,
    (P b)[i] = b[p[i]] and (Q z)[q[j]] = z[j].
    """
    L, U, p, q = out["L"], out["U"], out["p"], out["q"]
    k = L.shape[1]
    n = U.shape[1]
    b = np.asarray(b, dtype=np.float64)
    vec = b.ndim == 1
    B = b.reshape(b.shape[0], -1)
    c = B[p, :]                                      # P b
    y = pinv_apply(L, c)                             # Step 2
    z1 = upper_solve(U[:, :k], y)                    # Step 3
    z = np.zeros((n, B.shape[1]))                    # Step 4: z_2 = 0
    z[:k] = z1
    x = np.empty_like(z)                             # Step 5: x = Q z
    x[q, :] = z
    return x[:, 0] if vec else x


def permuted(A: np.ndarray, p: np.ndarray, q: np.ndarray) -> np.ndarray:
    """P A Q with the index-vector conventions of this module."""
    return np.asarray(A)[np.ix_(p, q)]


def spectral_norm(X: np.ndarray) -> float:
    """Largest singular value (Section 3 notation), by a full SVD."""
    if X.size == 0:
        return 0.0
    return float(np.linalg.svd(X, compute_uv=False)[0])


def residual_operator(A: np.ndarray, out: dict):
    """The residual E = L U - P A Q of Theorem 4.1 as a pair of products
    (X -> E X, Y -> E^T Y), never forming E: (P A Q) X is A applied to X
    with its rows put in the order q^{-1}, then rows picked by p."""
    L, U, p, q = out["L"], out["U"], out["p"], out["q"]
    qinv = np.empty_like(q)
    qinv[q] = np.arange(q.size)
    pinv = np.empty_like(p)
    pinv[p] = np.arange(p.size)

    def mv(X):
        return L @ (U @ X) - (A @ X[qinv])[p]

    def rmv(Y):
        return U.T @ (L.T @ Y) - (A.T @ Y[pinv])[q]

    return mv, rmv, U.shape[1]


def spectral_norm_estimate(mv, rmv, n: int, iters: int = 60, block: int = 8,
                           seed: int = 0) -> float:
    """Largest singular value of an operator given by its products, by
    subspace iteration on E^T E with a block of ``block`` Gaussian start
    vectors (orthonormalized after every step), then the largest singular
    value of E X on the final orthonormal block X.  Always a lower bound
    (||E X||_2 <= ||E||_2 for orthonormal X); the error in sigma_1 decays
    like (sigma_{block+1} / sigma_1)^(2 iters), so a cluster of up to
    ``block`` near-equal leading values does not slow it down."""
    b = max(1, min(block, n))
    X = np.random.default_rng(seed).standard_normal((n, b))
    X, _ = np.linalg.qr(X)
    for _ in range(iters):
        Z = rmv(mv(X))
        if not np.any(Z):
            return 0.0
        X, _ = np.linalg.qr(Z)
    return float(np.linalg.svd(mv(X), compute_uv=False)[0])


def residual(A: np.ndarray, out: dict, exact: bool = True, iters: int = 60,
             seed: int = 0) -> float:
    """||L U - P A Q||_2 (the quantity bounded by Theorem 4.1).

    ``exact`` uses a full SVD of the difference; otherwise
    ``spectral_norm_estimate`` on ``residual_operator`` (the difference is
    never formed, for large inputs)."""
    if exact:
        L, U, p, q = out["L"], out["U"], out["p"], out["q"]
        return spectral_norm(L @ U - permuted(A, p, q))
    mv, rmv, n = residual_operator(np.asarray(A), out)
    return spectral_norm_estimate(mv, rmv, n, iters=iters, seed=seed)


def relative_residual(A: np.ndarray, out: dict, exact: bool = True) -> float:
    """Relative error of Section 5.1: ||L U - P A Q||_2 / ||A||_2."""
    den = spectral_norm(A) if exact else _power_norm(A)
    return residual(A, out, exact=exact) / den


def _power_norm(A: np.ndarray, iters: int = 60, seed: int = 1) -> float:
    """||A||_2 by ``spectral_norm_estimate`` (A is never factored)."""
    A = np.asarray(A)
    return spectral_norm_estimate(lambda X: A @ X, lambda Y: A.T @ Y, A.shape[1],
                                  iters=iters, seed=seed)


def pivot_gate(diag: dict, u: float = 2.0 ** -53, gap_min: float = 1e-8,
               mag_factor: float = 1e3) -> int:
    """Number of leading pivot steps whose choice is numerically decided:
    every step up to it has a relative gap to the runner-up >= gap_min and a
    pivot magnitude >= mag_factor * u * max|input|.  Pivot sequences of two
    correct implementations must agree on this prefix."""
    thr = mag_factor * u * diag["max_abs"]
    n = 0
    for g, a in zip(diag["gap"], diag["piv_abs"]):
        if g < gap_min or a < thr:
            break
        n += 1
    return n


def kappa(X: np.ndarray) -> float:
    """2-norm condition number (diagnostic for the Gram route of Step 5)."""
    s = np.linalg.svd(X, compute_uv=False)
    return float(s[0] / s[-1]) if s[-1] > 0 else float("inf")
