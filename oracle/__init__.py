"""Slow, plain FP64 CPU oracle for the online stage of parametric H^2-matrices.

TEST INFRASTRUCTURE ONLY.  This package is the independent reference that the
HIP implementation is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import or call anything in it.
The product path (the C-ABI library and its Python binding) never imports it,
and it never imports the product path: the two share no code.  Inputs are
passed in as arrays by the caller.

Every function cites the passage of arxiv 2511.03109 ("Parametric Hierarchical
Matrix Approximations to Kernel Matrices") that it follows.  Where the paper is
silent or garbled the reading taken is stated at the function.

Modules
-------
cheb     Chebyshev nodes of the first kind, Lagrange basis and its derivative
         (Sec. 2.2; parametric vectors, App. PTTK review).
kernels  The parametric kernels of the workloads (closed forms) plus test-only
         kernels used as pins (a polynomial kernel, a parameter-free kernel).
tree     Cluster tree (Alg. ConstructClusterTree), block cluster tree
         (Alg. ConstructBlockClusterTree, admissibility eq. in Sec. 3.3 with
         the distance/diameter of App. "Additional definitions"), and
         translation classes (Sec. 5.2).
tucker   Truncated higher-order SVD (the default compression).
tt       TT-cross with partially pivoted ACA, TT-rounding, the conversion of the
         cores into spatial factors and a parameter core, and the core-by-core
         coupling of Alg. "Modified H^2-Matrix MVM" (Sec. 2.1, App. PTTK review).
hmat     Offline stage (Alg. "Offline Stage: Parametric H^2"), online stage
         (Alg. "Online Stage"; PTTK online), H^2 MVM (Alg. "H^2-matrix MVM"
         with FastForward / FastBackward), derivative, dense assembly, the
         plain interpolant definition, and the sampled-row error estimator
         (Sec. 6, "Error Calculation").

Parity status: every function is pinned by a ``-m "not gpu"`` test under
``tests/test_oracle_*.py`` (closed forms, brute force, library routines,
polynomial exactness, node reproduction, the paper's printed NF ratios).
"""

from . import cheb, kernels, tree, tucker, tt, hmat  # noqa: F401
