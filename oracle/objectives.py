"""Relaxed objectives and their gradients in float64 (the truth).

Sec. 3 defines, for the adjacency matrix A (notation paragraph of Sec. 2):
  * MIS, Eq. (3):           h(x)   = 1^T x - (gamma/2) x^T A x,  gamma > 1,
                            grad h = 1 - gamma A x          (proof of Prop. 3.1)
  * MaxCut Laplacian, Eq. (4): f_L(x) = (1/4) x^T L x, L = D - A; on {-1,1}^n
                            it is the cut value.
  * MaxCut perturbed Laplacian, Eq. (5): f_P(x) = x^T (L + lambda I) x.
  * MaxCut adjacency, Eq. (6): f_A(x) = -x^T A x.
  * MaxCut perturbed bias, Eq. (7): f_B(x) = -lambda 1^T x - x^T A x,
                            grad f_B = -2 A x - lambda 1    (proof of Thm. 3.6)
Weighted MaxCut (the +-1 torus) uses A_uv = w_uv.

Columns of X are independent iterates (the batch of Alg. 3 / Alg. 4).
Test infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

MIS = "mis"
MAXCUT = "maxcut"        # perturbed bias f_B, Eq. (7): the formulation the algorithms use
MAXCUT_L = "maxcut_fl"   # Laplacian f_L, Eq. (4)
MAXCUT_P = "maxcut_fp"   # perturbed Laplacian f_P, Eq. (5)
MAXCUT_A = "maxcut_fa"   # adjacency f_A, Eq. (6)
CUT_KINDS = (MAXCUT, MAXCUT_L, MAXCUT_P, MAXCUT_A)


def adjacency(graph, dtype=np.float64) -> sp.csr_matrix:
    """A as a scipy CSR matrix (weights if present, else ones)."""
    data = np.ones(graph.nnz, dtype=dtype) if graph.weight is None else graph.weight.astype(dtype)
    return sp.csr_matrix((data, graph.col_idx.astype(np.int64), graph.row_ptr.astype(np.int64)),
                         shape=(graph.n, graph.n))


def h(X, A, gamma):
    """Eq. (3) per column: 1^T x - (gamma/2) x^T A x."""
    X = np.asarray(X, dtype=np.float64)
    return X.sum(axis=0) - 0.5 * gamma * np.einsum("vb,vb->b", X, A @ X)


def grad_h(X, A, gamma):
    """1 - gamma A x (derivative in the proof of Prop. 3.1)."""
    return 1.0 - gamma * (A @ np.asarray(X, dtype=np.float64))


def f_B(X, A, lam):
    """Eq. (7) per column: -lambda 1^T x - x^T A x."""
    X = np.asarray(X, dtype=np.float64)
    return -lam * X.sum(axis=0) - np.einsum("vb,vb->b", X, A @ X)


def grad_f_B(X, A, lam):
    """-2 A x - lambda 1 (proof of Thm. 3.6 (i))."""
    return -2.0 * (A @ np.asarray(X, dtype=np.float64)) - lam


def f_A(X, A):
    """Eq. (6): -x^T A x."""
    X = np.asarray(X, dtype=np.float64)
    return -np.einsum("vb,vb->b", X, A @ X)


def laplacian(A):
    d = np.asarray(A.sum(axis=1)).ravel()
    return sp.diags(d) - A


def f_L(X, A):
    """Eq. (4): (1/4) x^T L x."""
    X = np.asarray(X, dtype=np.float64)
    return 0.25 * np.einsum("vb,vb->b", X, laplacian(A) @ X)


def f_P(X, A, lam):
    """Eq. (5): x^T (L + lambda I) x."""
    X = np.asarray(X, dtype=np.float64)
    return np.einsum("vb,vb->b", X, laplacian(A) @ X) + lam * np.einsum("vb,vb->b", X, X)


def grad_f_L(X, A):
    """Gradient of Eq. (4): (1/2) L x.  (The text's proof of Prop. 3.2 writes
    L x; differentiating (1/4) x^T L x with L symmetric gives L x / 2.)"""
    X = np.asarray(X, dtype=np.float64)
    return 0.5 * (laplacian(A) @ X)


def grad_f_P(X, A, lam):
    """Gradient of Eq. (5): 2 (L + lambda I) x.  (The proof of Thm. 3.3 steps
    by alpha/2 (L + lambda I) x, which changes alpha only; both fix every
    binary point.)"""
    X = np.asarray(X, dtype=np.float64)
    return 2.0 * (laplacian(A) @ X + lam * X)


def grad_f_A(X, A):
    """Gradient of Eq. (6): -2 A x."""
    return -2.0 * (A @ np.asarray(X, dtype=np.float64))


def objective(kind, X, A, param):
    """The objective the path ascends: h for MIS, f_B (or the formulation
    named by ``kind``) for MaxCut."""
    if kind == MIS:
        return h(X, A, param)
    if kind == MAXCUT_L:
        return f_L(X, A)
    if kind == MAXCUT_P:
        return f_P(X, A, param)
    if kind == MAXCUT_A:
        return f_A(X, A)
    return f_B(X, A, param)


def gradient(kind, X, A, param):
    if kind == MIS:
        return grad_h(X, A, param)
    if kind == MAXCUT_L:
        return grad_f_L(X, A)
    if kind == MAXCUT_P:
        return grad_f_P(X, A, param)
    if kind == MAXCUT_A:
        return grad_f_A(X, A)
    return grad_f_B(X, A, param)


def hessian_vec(kind, A, param, M):
    """H m for the (quadratic) objective of ``kind``: its gradient is
    grad(0) + H x."""
    M = np.asarray(M, dtype=np.float64)
    if kind == MIS:
        return -param * (A @ M)
    if kind == MAXCUT_L:
        return 0.5 * (laplacian(A) @ M)
    if kind == MAXCUT_P:
        return 2.0 * (laplacian(A) @ M + param * M)
    return -2.0 * (A @ M)


def box(kind):
    """Projection box of the PGA update (Sec. 3): [0,1] for MIS, [-1,1] for MaxCut."""
    return (0.0, 1.0) if kind == MIS else (-1.0, 1.0)


def linear_and_hessian(kind, param):
    """Objective written as c^T x + (1/2) x^T H x with H = eta A:
    MIS c = 1, eta = -gamma; MaxCut c = -lambda, eta = -2."""
    return (1.0, -param) if kind == MIS else (-param, -2.0)
