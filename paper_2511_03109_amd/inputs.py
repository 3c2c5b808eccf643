"""Seeded synthetic inputs and workload definitions.

This module holds no arithmetic of the method: it only draws the point clouds,
parameter samples and right-hand sides, and names the workloads.  Both the HIP
path (through the binding) and the CPU oracle are fed from it, so the two read
identical bytes.

Generators are ``numpy.random.default_rng([workload_id, stream])`` with streams
0 points, 1 theta samples, 2 right-hand sides X, 3 the vector u of a bilinear
form, 4 mixture parameters, 5 the right-hand side y of a linear solve.

The paper draws its points uniformly from [0, 1]^d (Sec. 6, "Other Problem
Settings"); the mixture workload draws an 8-component Gaussian mixture in the
unit square to obtain uneven cluster sizes.
"""

import numpy as np

STREAM_POINTS, STREAM_THETA, STREAM_X, STREAM_U, STREAM_MIX, STREAM_Y = range(6)


def rng(workload_id, stream):
    return np.random.default_rng([int(workload_id), int(stream)])


def uniform_points(n, d, workload_id):
    """n points uniform in [0, 1]^d, row-major (n, d) float64."""
    return rng(workload_id, STREAM_POINTS).random((n, d))


def mixture_points(n, workload_id, components=8):
    """n points in [0, 1]^2 from a Gaussian mixture, rejection-resampled into the square.

    Means ~ U[0.15, 0.85]^2, isotropic std ~ U[0.015, 0.08], weights ~ U[0.25, 1]
    normalised.
    """
    g = rng(workload_id, STREAM_MIX)
    means = g.uniform(0.15, 0.85, size=(components, 2))
    stds = g.uniform(0.015, 0.08, size=components)
    w = g.uniform(0.25, 1.0, size=components)
    w = w / w.sum()
    gp = rng(workload_id, STREAM_POINTS)
    out = np.empty((0, 2))
    while out.shape[0] < n:
        m = 2 * (n - out.shape[0]) + 16
        comp = gp.choice(components, size=m, p=w)
        pts = means[comp] + stds[comp, None] * gp.standard_normal((m, 2))
        ok = np.all((pts >= 0.0) & (pts <= 1.0), axis=1)
        out = np.concatenate([out, pts[ok]], axis=0)
    return np.ascontiguousarray(out[:n])


def theta_samples(T, lo, hi, workload_id):
    """T parameter values uniform in the box [lo, hi] (one row per sample)."""
    lo = np.atleast_1d(np.asarray(lo, dtype=np.float64))
    hi = np.atleast_1d(np.asarray(hi, dtype=np.float64))
    u = rng(workload_id, STREAM_THETA).random((T, lo.shape[0]))
    return lo + (hi - lo) * u


def normal_vectors(n, R, workload_id, stream=STREAM_X):
    """An (n, R) array of N(0, 1) entries (column j is right-hand side j)."""
    return rng(workload_id, stream).standard_normal((n, R))


# Workload definitions.  eta2 = (num, den) is the admissibility parameter
# squared as a rational; leaf is the target leaf size from which the uniform
# tree depth is derived.
WORKLOADS = {
    1: dict(name="gauss2d_n2048", n=2048, d=2, points="uniform", kernel="gaussian",
            theta_lo=[0.1], theta_hi=[0.5], p_s=6, p_theta=9, leaf=64, eta2=(1, 1),
            tol=1e-8, theta=[0.25], R=1),
    2: dict(name="matern32_3d_n65536", n=65536, d=3, points="uniform", kernel="matern32",
            theta_lo=[0.05], theta_hi=[0.5], p_s=5, p_theta=11, leaf=128, eta2=(3, 1),
            tol=1e-8, T=8, R=16),
    3: dict(name="aniso_mixture2d_n32768", n=32768, d=2, points="mixture",
            kernel="aniso_gaussian", theta_lo=[0.05, 0.05], theta_hi=[0.5, 0.5], p_s=6,
            p_theta=7, leaf=64, eta2=(2, 1), tol=1e-8, T=64, R=32),
    4: dict(name="gauss2d_n131072_grad", n=131072, d=2, points="uniform", kernel="gaussian",
            theta_lo=[0.05], theta_hi=[0.5], p_s=6, p_theta=9, leaf=64, eta2=(2, 1),
            tol=1e-8, theta=[0.2], R=1),
    5: dict(name="matern12_2d_n262144_cg", n=262144, d=2, points="uniform", kernel="matern12",
            theta_lo=[0.05], theta_hi=[0.5], p_s=6, p_theta=9, leaf=64, eta2=(2, 1),
            tol=1e-8, theta=[0.1], nugget=1e-2, R=1),
    6: dict(name="matern_nu_3d_n4096", n=4096, d=3, points="uniform", kernel="matern",
            theta_lo=[0.1, 0.5], theta_hi=[1.0, 3.0], p_s=5, p_theta=7, leaf=64, eta2=(3, 1),
            tol=1e-8, T=8, R=16),
    7: dict(name="exp_3d_n32768", n=32768, d=3, points="uniform", kernel="matern12",
            theta_lo=[0.25], theta_hi=[1.0], p_s=5, p_theta=9, leaf=64, eta2=(3, 1),
            tol=1e-8, T=8, R=16),
}


def points_for(workload_id, n=None):
    """Points of a workload (optionally with a different n, same recipe and seed)."""
    w = WORKLOADS[workload_id]
    n = w["n"] if n is None else n
    if w["points"] == "mixture":
        return mixture_points(n, workload_id)
    return uniform_points(n, w["d"], workload_id)
