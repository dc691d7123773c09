"""Projected gradient ascent on the relaxed objectives.

Sec. 3 gives the update x <- Pi(x + alpha G) with Pi the projection onto
the box ([0,1]^n for MIS, [-1,1]^n for MaxCut) and G the gradient; Sec. 5
uses momentum ascent (MGA), whose form the paper does not print: the
reading used here is the heavy ball v <- mu v + G, x <- Pi(x + alpha v).

Two precisions:
  * ``step64``  float64 truth, A x by a sparse product;
  * ``step32``  float32 replay.  Rounding at 0.5 / 0 (Sec. 3) turns the
    iterate into integers, so the solver must reach those decisions in the
    precision the GPU computes in.  The replay fixes one order of
    operations: per row, acc starts at 0 and adds w_vu * x_u for the
    neighbours u in ascending CSR order (unit weights: acc + x_u); then
    g = 1 - gamma*acc (MIS) or g = (-lambda) - 2*acc (MaxCut); with
    momentum v = mu*v + g; y = x + alpha*d; x' = min(max(y, lo), hi).
    Every operation is one IEEE float32 rounding (no fused multiply-add).

Also here: the initialisations (uniform, and the degree-based one of
Alg. 1 / Alg. 2) and the adjoint of K unrolled steps.
Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

from . import objectives as obj
from . import philox

F32 = np.float32


def step64(X, A, kind, alpha, param, mu=0.0, V=None):
    """One float64 PGA / MGA step on every column.  Returns (X', V')."""
    X = np.asarray(X, dtype=np.float64)
    g = obj.gradient(kind, X, A, param)
    if mu:
        V = mu * (np.zeros_like(X) if V is None else np.asarray(V, dtype=np.float64)) + g
        d = V
    else:
        d = g
    lo, hi = obj.box(kind)
    return np.clip(X + alpha * d, lo, hi), V


def neighbour_sum32(graph, X):
    """float32 sum over neighbours in ascending CSR order, one rounding per add.

    Unweighted or +-1 weights: scipy's CSR product in float32, which starts
    every row at 0 and adds its terms into a float32 accumulator in stored
    order; the products by +-1 are exact, so a fused multiply-add in the
    library could not change a rounding.  (Pinned bit for bit against the
    position-by-position loop, ``neighbour_sum32_positions``, which serves
    every other weight.)"""
    X = np.asarray(X, dtype=F32)
    if graph.weight is not None and not np.all(np.abs(graph.weight) == 1):
        return neighbour_sum32_positions(graph, X)
    A = _csr32(graph)
    return np.asarray(A @ X, dtype=F32).reshape(X.shape)


def _csr32(graph):
    """The graph's float32 CSR matrix, built once per graph object."""
    import scipy.sparse as sp
    cached = getattr(graph, "_oracle_csr32", None)
    if cached is not None and cached[0] is graph.row_ptr and cached[1] is graph.col_idx:
        return cached[2]
    data = np.ones(graph.nnz, dtype=F32) if graph.weight is None else graph.weight.astype(F32)
    A = sp.csr_matrix((data, graph.col_idx, graph.row_ptr), shape=(graph.n, graph.n))
    graph._oracle_csr32 = (graph.row_ptr, graph.col_idx, A)
    return A


def neighbour_sum32_positions(graph, X):
    """The definition, vectorised over rows: the k-th stored neighbour of
    every row of degree > k is added for k = 0, 1, ... (float32, one
    rounding per add, each row in ascending CSR order)."""
    X = np.asarray(X, dtype=F32)
    acc = np.zeros_like(X)
    deg = np.diff(graph.row_ptr).astype(np.int64)
    rp = graph.row_ptr.astype(np.int64)
    for k in range(int(deg.max()) if len(deg) else 0):
        rows = np.flatnonzero(deg > k)
        j = rp[rows] + k
        u = graph.col_idx[j]
        if graph.weight is None:
            acc[rows] = acc[rows] + X[u]
        else:
            acc[rows] = acc[rows] + graph.weight[j].astype(F32)[:, None] * X[u]
    return acc


def weighted_degree32(graph):
    """W_v = sum of the row's weights (the degree when unweighted), exact in float32."""
    deg = np.diff(graph.row_ptr.astype(np.int64))
    if graph.weight is None:
        return deg.astype(F32)
    rows = np.repeat(np.arange(graph.n), deg)
    return np.bincount(rows, weights=graph.weight.astype(np.float64), minlength=graph.n).astype(F32)


def gradient32(graph, X, kind, param):
    """float32 gradient, one rounding per operation in the order written:
    MIS 1 - gamma acc; f_B -lambda - 2 acc; f_L 0.5 (W x - acc);
    f_P 2 ((W x - acc) + lambda x); f_A -2 acc (acc = A x summed in CSR order)."""
    X = np.asarray(X, dtype=F32)
    acc = neighbour_sum32(graph, X)
    if kind == obj.MIS:
        return F32(1.0) - F32(param) * acc
    if kind in (obj.MAXCUT_L, obj.MAXCUT_P):
        W = weighted_degree32(graph)[:, None]
        t = W * X - acc
        if kind == obj.MAXCUT_L:
            return F32(0.5) * t
        return F32(2.0) * (t + F32(param) * X)
    if kind == obj.MAXCUT_A:
        return F32(-2.0) * acc
    return F32(-F32(param)) - F32(2.0) * acc


def step32(graph, X, kind, alpha, param, mu=0.0, V=None):
    """One float32 replay step (order of operations in the module doc)."""
    X = np.asarray(X, dtype=F32)
    g = gradient32(graph, X, kind, param)
    if mu:
        V = F32(mu) * (np.zeros_like(X) if V is None else np.asarray(V, dtype=F32)) + g
        d = V
    else:
        d = g
    lo, hi = obj.box(kind)
    y = X + F32(alpha) * d
    return np.minimum(np.maximum(y, F32(lo)), F32(hi)), V


# --------------------------------------------------------------------------
# initialisation
# --------------------------------------------------------------------------

def init_uniform(kind, n, traj, seed, start=0, rows=None):
    """x0 ~ U[0,1)^n for MIS; for MaxCut the same draw mapped by 2u - 1 onto
    the box [-1,1]^n (the affine map of the MaxCut degree initialisation,
    Alg. 2).  ``traj`` is the array of trajectory ids (one per column);
    ``start`` numbers the fresh starts of the outer loop (the round field
    of the Philox counter); ``rows`` (optional) selects the vertices
    returned."""
    traj = np.asarray(traj, dtype=np.uint64)
    v = np.arange(n, dtype=np.uint64) if rows is None else np.asarray(rows, dtype=np.uint64)
    u = philox.u32_to_unit_f32(philox.vertex_u32(seed, philox.PURPOSE_INIT, traj[None, :], start, v[:, None]))
    if kind == obj.MIS:
        return u
    return F32(2.0) * u - F32(1.0)


def degree_base(kind, deg):
    """d_base of Alg. 1 (MIS: 1 - d(v)/Delta) and Alg. 2 (MaxCut:
    2(1 - d(v)/Delta) - 1); an edgeless graph (Delta = 0) takes 1."""
    deg = np.asarray(deg, dtype=np.float64)
    dmax = deg.max() if len(deg) else 0.0
    base = np.ones_like(deg) if dmax == 0 else 1.0 - deg / dmax
    return base if kind == obj.MIS else 2.0 * base - 1.0


def init_degree(kind, deg, traj, seed, sigma, start=0):
    """Pi(d_base + eps), eps ~ N(0, sigma^2 I) (Alg. 1 / Alg. 2 initialisation).
    The Gaussian comes from the Box-Muller transform of two uniforms
    u1 in (0,1], u2 in [0,1) drawn with purpose NOISE (round field =
    ``start``)."""
    n = len(deg)
    traj = np.asarray(traj, dtype=np.uint64)
    a, b = philox.vertex_pair_u32(seed, philox.PURPOSE_NOISE, traj[None, :], start,
                                  np.arange(n, dtype=np.uint64)[:, None])
    u1 = ((a >> np.uint32(8)).astype(np.float64) + 1.0) * 2.0**-24
    u2 = (b >> np.uint32(8)).astype(np.float64) * 2.0**-24
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    lo, hi = obj.box(kind)
    return np.clip(degree_base(kind, deg)[:, None] + sigma * z, lo, hi)


# --------------------------------------------------------------------------
# differentiation through the objective and through unrolled steps
# --------------------------------------------------------------------------

def objective_and_grad(graph, kind, param, X, scale=None):
    """f per column (float64) and scale_b * grad f (float64) at X."""
    A = obj.adjacency(graph)
    f = obj.objective(kind, X, A, param)
    g = obj.gradient(kind, X, A, param)
    if scale is not None:
        g = g * np.asarray(scale, dtype=np.float64)[None, :]
    return f, g


def unrolled_forward(graph, kind, param, alpha, K, X0, precision="fp64"):
    """x_{k+1} = Pi(x_k + alpha g(x_k)), k = 0..K-1; returns [x_0, ..., x_K]."""
    xs = [np.asarray(X0, dtype=np.float64 if precision == "fp64" else F32)]
    A = obj.adjacency(graph)
    for _ in range(K):
        if precision == "fp64":
            xs.append(step64(xs[-1], A, kind, alpha, param)[0])
        else:
            xs.append(step32(graph, xs[-1], kind, alpha, param)[0])
    return xs


def unrolled_backward(graph, kind, param, alpha, K, X0, dL_dXK, precision="fp64"):
    """Adjoint of the K-step map (float64 arithmetic).

    With z_k = x_k + alpha g(x_k), x_{k+1} = Pi(z_k), mask_k = [lo <= z_k <= hi]
    and g(x) = g(0) + H x (every objective here is quadratic):
        mu_k   = mask_k * lam_{k+1}
        dL/dalpha += <mu_k, g(x_k)>
        lam_k  = mu_k + alpha * H mu_k
    starting from lam_K = dL/dx_K.  ``precision`` selects the forward pass
    that decides the masks (the float32 replay when comparing with a
    float32 forward).  Returns (dL/dX0, dL/dalpha per column)."""
    xs = unrolled_forward(graph, kind, param, alpha, K, X0, precision)
    A = obj.adjacency(graph)
    lo, hi = obj.box(kind)
    lam = np.asarray(dL_dXK, dtype=np.float64)
    dalpha = np.zeros(lam.shape[1])
    for k in range(K - 1, -1, -1):
        xk = xs[k]
        if precision == "fp64":
            g = obj.gradient(kind, xk, A, param)
            z = xk + alpha * g
        else:
            g32 = gradient32(graph, xk, kind, param)
            z = (xk + F32(alpha) * g32).astype(np.float64)
            g = obj.gradient(kind, xk.astype(np.float64), A, param)
        mask = (z >= lo) & (z <= hi)
        mu = np.where(mask, lam, 0.0)
        dalpha += np.einsum("vb,vb->b", mu, g)
        lam = mu + alpha * obj.hessian_vec(kind, A, param, mu)
    return lam, dalpha
