"""Parametric kernels kappa(x, y; theta) (oracle; test infrastructure only).

The workloads use closed-form kernels (the paper's Table "kernel functions"
lists E = exp(-r/lambda), which is Matern-1/2; the Gaussian and Matern-3/2 are
the standard closed forms with length scale l, and the anisotropic Gaussian has
one length scale per axis), and the table's Matern kernel with free smoothness nu
(two parameters, lambda and nu).  All are stationary and symmetric, which is what the
translation-invariance argument of Sec. 5.2 needs.

Each kernel takes broadcastable arrays x (..., d), y (..., d), theta (..., d_theta)
and returns kappa with the broadcast leading shape.
"""

import numpy as np


def _r2(x, y):
    diff = np.asarray(x, dtype=np.float64) - np.asarray(y, dtype=np.float64)
    return np.sum(diff * diff, axis=-1)


def gaussian(x, y, theta):
    """exp(-r^2 / (2 l^2)), theta = (l,)."""
    l = np.asarray(theta, dtype=np.float64)[..., 0]
    return np.exp(-_r2(x, y) / (2.0 * l * l))


def matern32(x, y, theta):
    """(1 + sqrt(3) r / l) exp(-sqrt(3) r / l), theta = (l,)."""
    l = np.asarray(theta, dtype=np.float64)[..., 0]
    s = np.sqrt(3.0) * np.sqrt(_r2(x, y)) / l
    return (1.0 + s) * np.exp(-s)


def matern12(x, y, theta):
    """exp(-r / l) (the paper's exponential kernel E), theta = (l,)."""
    l = np.asarray(theta, dtype=np.float64)[..., 0]
    return np.exp(-np.sqrt(_r2(x, y)) / l)


def aniso_gaussian(x, y, theta):
    """exp(-sum_k (x_k - y_k)^2 / (2 l_k^2)), theta = (l_1, ..., l_d), d_theta = d."""
    diff = np.asarray(x, dtype=np.float64) - np.asarray(y, dtype=np.float64)
    l = np.asarray(theta, dtype=np.float64)
    return np.exp(-np.sum(diff * diff / (2.0 * l * l), axis=-1))


def matern(x, y, theta):
    """Matern kernel with free smoothness (Table "Kernel functions", MN), theta = (lambda, nu):
    2^(1 - nu) / Gamma(nu) z^nu K_nu(z), z = sqrt(2 nu) r / lambda, K_nu the modified Bessel
    function of the second kind (scipy.special.kv), and the limit 1 at r = 0.  The table
    prints Gamma(lambda) in the prefactor; the normalising constant of the Matern family is
    Gamma(nu), which is what makes the value 1 at r = 0."""
    from scipy.special import gammaln, kv
    th = np.asarray(theta, dtype=np.float64)
    lam, nu = th[..., 0], th[..., 1]
    r = np.sqrt(_r2(x, y))
    z = np.sqrt(2.0 * nu) * r / lam
    z, nu = np.broadcast_arrays(z, nu)
    out = np.ones(z.shape)
    pos = z > 0
    zp, nup = z[pos], nu[pos]
    with np.errstate(under="ignore"):
        out[pos] = np.exp((1.0 - nup) * np.log(2.0) - gammaln(nup) + nup * np.log(zp)) * kv(nup, zp)
    return out


def poly_test(x, y, theta):
    """Test-only polynomial kernel theta^2 |x - y|^2 + theta, theta = (t,).

    Degree 2 in every coordinate of x and y and in theta: Chebyshev interpolation
    with p_s >= 3 and p_theta >= 3 reproduces it exactly (up to rounding), so the
    whole pipeline must equal the textbook dense product K(theta) x.
    """
    t = np.asarray(theta, dtype=np.float64)[..., 0]
    return t * t * _r2(x, y) + t


def poly2_test(x, y, theta):
    """Test-only polynomial kernel with two parameters: t1 |x - y|^2 + t2^2, d_theta = 2."""
    t = np.asarray(theta, dtype=np.float64)
    return t[..., 0] * _r2(x, y) + t[..., 1] * t[..., 1]


def theta_free_test(x, y, theta):
    """Test-only kernel that ignores theta: exp(-|x - y|^2).  K~(theta) must then be constant."""
    r2 = _r2(x, y)
    t = np.asarray(theta, dtype=np.float64)[..., 0]
    return np.exp(-r2) * np.ones_like(t)


KERNELS = {
    "gaussian": (gaussian, 1),
    "matern32": (matern32, 1),
    "matern12": (matern12, 1),
    "aniso_gaussian": (aniso_gaussian, None),  # d_theta = d
    "matern": (matern, 2),
    "poly_test": (poly_test, 1),
    "poly2_test": (poly2_test, 2),
    "theta_free_test": (theta_free_test, 1),
}
