"""FP64 CPU oracle of Algorithm 4.4 (fast randomized LU) of Shabat et al.,
arXiv 1310.7202, Section 4.5, with the SRFT of Section 3.3 and the
interpolative decomposition (ID) of Section 3.4.

TEST INFRASTRUCTURE ONLY: see the package docstring for who may call this.

Readings taken here (each listed with its reason in the design notes):
  * R = D F S with a REAL fast transform: F is the orthonormal discrete
    Hartley transform, F_jk = (cos(2 pi jk/n) + sin(2 pi jk/n)) / sqrt(n),
    and D = diag(+1 / -1), the real points of the unit circle.  The paper's
    complex DFT would make every factor of a real A complex; the Hartley
    transform is real, orthogonal and has an O(n log n) algorithm (it is
    Re(FFT) - Im(FFT)), so R keeps orthonormal columns as in Section 3.3.
  * S selects l distinct columns, drawn without replacement in a random
    order (a repeated column would make Y rank deficient and its full-rank
    ID undefined).  The draws come from ``philox.srft_signs`` and
    ``philox.srft_selection``.
  * Step 3 is the partial-pivot LU (the Remark after Algorithm 4.1), or the
    rank-revealing form of ``rlu.rrlu``.
  * Step 5's full-rank ID of Y is taken from the LU of Step 3, as Section
    3.4 allows: J = the l rows the pivots chose, X = Y Y(J, :)^{-1}, so that
    Y = X Y(J, :) and X(J, :) = I.
"""
from __future__ import annotations

import numpy as np

from oracle import philox, rlu


def hartley_matrix(n: int) -> np.ndarray:
    """The orthonormal n x n discrete Hartley transform (symmetric)."""
    jk = np.outer(np.arange(n), np.arange(n)) % n
    ang = 2.0 * np.pi * jk / n
    return (np.cos(ang) + np.sin(ang)) / np.sqrt(n)


def srft_matrix(n: int, d: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Step 1 of Algorithm 4.4: R = D F S (n x l), formed explicitly."""
    F = hartley_matrix(n)
    return np.asarray(d, dtype=np.float64)[:, None] * F[:, np.asarray(s)]


def row_id_from_lu(Y: np.ndarray, p: np.ndarray):
    """Step 5 of Algorithm 4.4: the full-rank ID Y = X Y(J, :) with J the
    first l rows of the row order p of Step 3's pivoted LU and X =
    Y Y(J, :)^{-1} (an l x l solve)."""
    l = Y.shape[1]
    J = np.asarray(p)[:l]
    X = np.linalg.solve(Y[J, :].T, Y.T).T
    return X, J


def fast_randomized_lu(A: np.ndarray, k: int, l: int, d: np.ndarray, s: np.ndarray,
                       step3: str = "partial") -> dict:
    """Algorithm 4.4 for the SRFT draws d (n signs) and s (l columns).

    Returns L (m x k unit lower trapezoidal), U (k x n upper trapezoidal),
    p, q and the intermediates (R, Y, the ID's X and J, B, ...)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if not (1 <= k <= l <= min(m, n)):
        raise ValueError("need 1 <= k <= l <= min(m, n)")
    R = srft_matrix(n, d, s)                               # Step 1
    Y = A @ R                                              # Step 2
    qy = None
    if step3 == "rrlu":                                    # Step 3
        LUy, ipiv, p, info_y, diag_y, qy, _ = rlu.rrlu(Y)
    else:
        LUy, ipiv, p, info_y, diag_y = rlu.lu_partial_pivot(Y)
    Ly = rlu.unit_lower(LUy, k)                            # Step 4
    X, J = row_id_from_lu(Y, p)                            # Step 5
    XA = X @ A[J, :]
    B = rlu.pinv_apply(Ly, XA[p, :])                       # Step 6: L_y^+ P X A(J, :)
    Lb, Ub, qpiv, q, info_b, diag_b = rlu.lu_col_pivot(B)  # Step 7
    L = Ly @ Lb                                            # Step 8
    U = Ub                                                 # Step 9
    return {"L": L, "U": U, "p": p, "q": q, "R": R, "Y": Y, "LUy": LUy, "ipiv": ipiv,
            "Ly": Ly, "X": X, "J": J, "B": B, "Lb": Lb, "Ub": Ub, "qpiv": qpiv, "qy": qy,
            "info": (info_y, info_b), "diag_y": diag_y, "diag_b": diag_b}


def fast_randomized_lu_seeded(A: np.ndarray, k: int, l: int, seed: int,
                              step3: str = "partial") -> dict:
    """Algorithm 4.4 with the SRFT drawn from ``seed``."""
    n = np.asarray(A).shape[1]
    return fast_randomized_lu(A, k, l, philox.srft_signs(n, seed),
                              philox.srft_selection(n, l, seed), step3)
