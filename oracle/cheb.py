"""Chebyshev nodes and Lagrange polynomials (oracle; test infrastructure only).

Paper: Sec. 2.2 "Polynomial Interpolation of kappa" (nodes of the first kind,
ascending, and the Lagrange product formula); App. "PTTK Method" (parametric
vectors v_k(theta_k), entries l_i on [alpha_k^theta, beta_k^theta]).

Reading: the paper names first-kind Chebyshev nodes and orders them ascending
but prints no formula; the standard one is used,
    eta_i = (a+b)/2 - (b-a)/2 * cos((2i-1) pi / (2p)),  i = 1..p.
"""

import numpy as np


def chebyshev_nodes(a, b, p):
    """First-kind Chebyshev nodes on [a, b], ascending (Sec. 2.2)."""
    i = np.arange(1, p + 1, dtype=np.float64)
    return (a + b) / 2.0 - (b - a) / 2.0 * np.cos((2.0 * i - 1.0) * np.pi / (2.0 * p))


def lagrange(nodes, x):
    """Lagrange basis by the product formula of Sec. 2.2.

    Returns an array of shape x.shape + (p,) whose [..., k] entry is
    l_k(x) = prod_{i != k} (x - eta_i) / (eta_k - eta_i).
    At a node the value is exactly 1 or 0 (each factor is exactly 1 or a 0
    factor appears).
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    p = nodes.shape[0]
    out = np.ones(x.shape + (p,), dtype=np.float64)
    for k in range(p):
        for i in range(p):
            if i != k:
                out[..., k] *= (x - nodes[i]) / (nodes[k] - nodes[i])
    return out


def lagrange_deriv(nodes, x):
    """Derivative of the Lagrange basis: the product rule applied to Sec. 2.2.

    l_k'(x) = sum_{m != k} 1/(eta_k - eta_m) * prod_{i != k, m} (x - eta_i)/(eta_k - eta_i).
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    p = nodes.shape[0]
    out = np.zeros(x.shape + (p,), dtype=np.float64)
    for k in range(p):
        for m in range(p):
            if m == k:
                continue
            term = np.full(x.shape, 1.0 / (nodes[k] - nodes[m]))
            for i in range(p):
                if i != k and i != m:
                    term = term * (x - nodes[i]) / (nodes[k] - nodes[i])
            out[..., k] += term
    return out


def parametric_vectors(theta, theta_lo, theta_hi, p_theta, deriv_dim=None):
    """Parametric vectors v_i(theta_i), i = 1..d_theta (App. PTTK review).

    [v_k(theta_k)]_i = l_i^{[alpha_k, beta_k]}(theta_k).  With ``deriv_dim = i``
    the i-th vector is replaced by its derivative v_i'(theta_i), which gives
    the partial derivative of the multilinear parametric approximation in
    theta_i (the approximation is linear in each v_i separately).
    """
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    vs = []
    for k in range(theta.shape[0]):
        nodes = chebyshev_nodes(theta_lo[k], theta_hi[k], p_theta)
        if deriv_dim is not None and k == deriv_dim:
            vs.append(lagrange_deriv(nodes, theta[k]))
        else:
            vs.append(lagrange(nodes, theta[k]))
    return vs


def tensor_nodes(lo, hi, p):
    """Multidimensional Chebyshev nodes of a box (Sec. 2.2).

    Returns an array (p**d, d) whose row with flat index
    i_1 + i_2 p + ... (little-endian, Sec. 2.1 "Reshape Command", axis 1 fastest)
    is (eta_{i_1}^{(B_1)}, ..., eta_{i_d}^{(B_d)}).
    """
    lo = np.atleast_1d(np.asarray(lo, dtype=np.float64))
    hi = np.atleast_1d(np.asarray(hi, dtype=np.float64))
    d = lo.shape[0]
    per_axis = [chebyshev_nodes(lo[k], hi[k], p) for k in range(d)]
    P = p ** d
    out = np.empty((P, d), dtype=np.float64)
    for flat in range(P):
        rem = flat
        for k in range(d):
            out[flat, k] = per_axis[k][rem % p]
            rem //= p
    return out


def tensor_lagrange(lo, hi, p, X):
    """Multidimensional Lagrange basis Lambda_i(x) = prod_k l_{i_k}(x_k) (Sec. 2.2).

    Returns (m, p**d) with columns in the little-endian flat order of
    ``tensor_nodes``.  This equals the face-splitting product
    U_d (face) ... (face) U_1 of Sec. 3.2 (cluster basis).
    """
    lo = np.atleast_1d(np.asarray(lo, dtype=np.float64))
    hi = np.atleast_1d(np.asarray(hi, dtype=np.float64))
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    d = lo.shape[0]
    facs = [lagrange(chebyshev_nodes(lo[k], hi[k], p), X[:, k]) for k in range(d)]
    out = facs[0]
    for k in range(1, d):
        # row-wise Kronecker: new column index = old + p^k * j_k  (axis 1 fastest)
        out = (facs[k][:, :, None] * out[:, None, :]).reshape(X.shape[0], -1)
    return out
