"""The three-matrix Douglas-Rachford iteration for OT, written out literally.

Test infrastructure only.  For tiny sizes this is the independent reading of
Section 3 that pins the one-matrix Algorithm 1:

* eq. (dr:def) / (drot:general:form): X_{k+1} = [Y_k - rho C]_+,
  Z_{k+1} = P_X(2 X_{k+1} - Y_k), Y_{k+1} = Y_k + Z_{k+1} - X_{k+1};
* Lemma 2 (projection onto {X : X e = p, X^T f = q}):
  P(X) = X - (1/n)((Xe - p) e^T - gamma f e^T) - (1/m)(f (X^T f - q)^T - gamma f e^T),
  gamma = f^T (Xe - p) / (m+n).

`project_lstsq` computes the same projection a second, generic way (the
minimum-norm correction through the explicit constraint matrix), which pins
the closed form of Lemma 2.
"""
from __future__ import annotations

import numpy as np


def project_lemma2(W: np.ndarray, p: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Closed-form projection of Lemma 2."""
    m, n = W.shape
    e = np.ones(n)
    f = np.ones(m)
    r = W @ e - p
    s = W.T @ f - q
    gamma = f @ r / (m + n)
    ffe = np.outer(f, e)
    return W - (np.outer(r, e) - gamma * ffe) / n - (np.outer(f, s) - gamma * ffe) / m


def constraint_matrix(m: int, n: int) -> np.ndarray:
    """The (m+n) x (m n) matrix of the linear map A(X) = (X e, X^T f), acting
    on X flattened row-major."""
    A = np.zeros((m + n, m * n))
    for i in range(m):
        for j in range(n):
            A[i, i * n + j] = 1.0
            A[m + j, i * n + j] = 1.0
    return A


def project_lstsq(W: np.ndarray, p: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Euclidean projection onto {A x = b} as w - A^+ (A w - b), with the
    Moore-Penrose pseudo-inverse (A has rank m+n-1; b lies in its range when
    the two masses agree, so this is the exact projection)."""
    m, n = W.shape
    A = constraint_matrix(m, n)
    w = W.reshape(-1)
    resid = A @ w - np.concatenate([p, q])
    y = np.linalg.pinv(A) @ resid
    return (w - y).reshape(m, n)


def dr3_iterate(C: np.ndarray, p: np.ndarray, q: np.ndarray, rho: float, iters: int,
                Y0: np.ndarray | None = None):
    """Run the literal three-matrix DR for `iters` steps from Y_0 (default p q^T).

    Returns lists X[1..K], Z[1..K], Y[0..K] (Y has K+1 entries).
    """
    Y = np.outer(p, q) if Y0 is None else np.array(Y0, dtype=np.float64)
    Xs, Zs, Ys = [], [], [Y.copy()]
    for _ in range(iters):
        X = np.maximum(Y - rho * C, 0.0)
        Z = project_lemma2(2.0 * X - Y, p, q)
        Y = Y + Z - X
        Xs.append(X)
        Zs.append(Z)
        Ys.append(Y.copy())
    return Xs, Zs, Ys
