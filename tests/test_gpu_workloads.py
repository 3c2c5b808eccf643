"""GPU parity at the workloads' own sizes, through the C ABI, against the CPU oracle on
sampled rows (the oracle computes a row of K~(theta) x from the blocks on that row's
leaf-to-root path), with the same tolerances as tests/test_gpu_parity.py.

  - n = 65536 3-D Matern-3/2, 8 slots x 16 RHS (the benchmark step, factored near field):
    every slot on the rows of 62 leaves, all 632 couplings of every slot, the near blocks of
    the sampled rows;
  - n = 32768 8-component mixture, anisotropic Gaussian, 64 slots x 32 RHS: through the
    autotuned configuration and a recorded graph replayed with new theta;
  - n = 131072 2-D Gaussian: forward and backward of y = K~(l) x through the autograd
    Function (dL/dx rows, dK~/dl x rows, dL/dl against a central difference);
  - n = 262144 2-D Matern-1/2 + nugget 1e-2: the operator on rows, and an FP64 CG solve to
    relative residual 1e-6 checked on the oracle's rows.
"""

from fractions import Fraction

import numpy as np
import pytest

from oracle import hmat, kernels, tree as otree
from paper_2511_03109_amd import inputs

from test_gpu_parity import TOL64, _close, _close_scalar, _torch

pytestmark = pytest.mark.gpu


def _compress(fn, items):
    """Oracle compressions, one after another (NumPy's LAPACK parallelises each one; calling
    it from several Python threads at once is not relied on)."""
    for it in items:
        fn(it)


def _sample_leaves(t, n_even, n_big, big_size, big_max=10 ** 9):
    """n_even leaves spread over the tree order plus up to n_big leaves of big_size + 1 ..
    big_max points (several row chunks in the near-field kernels); their points' original
    indices."""
    leaves = list(t.leaves)
    even = [leaves[i] for i in np.linspace(0, len(leaves) - 1, n_even).astype(int)]
    big = [s for s in leaves if big_size < t.end[s] - t.begin[s] <= big_max]
    if big:
        big = [big[i] for i in np.linspace(0, len(big) - 1, min(n_big, len(big))).astype(int)]
    sel = sorted(set(even) | set(big))
    return sel, np.concatenate([t.perm[t.begin[s]:t.end[s]] for s in sel])


def _workload(wid, n=None):
    from paper_2511_03109_amd import api
    w = inputs.WORKLOADS[wid]
    X = inputs.points_for(wid) if n is None else inputs.points_for(wid, n)
    l_max = otree.default_l_max(X.shape[0], w["d"], w["leaf"])
    lt = api.Tree(X, l_max=l_max, eta2=w["eta2"])
    lm = api.Model(lt, w["kernel"], w["theta_lo"], w["theta_hi"], p_s=w["p_s"], p_theta=w["p_theta"],
                   tol=w["tol"])
    om = hmat.PH2(X, l_max=l_max, eta2=Fraction(*w["eta2"]), kernel=kernels.KERNELS[w["kernel"]][0],
                  theta_lo=w["theta_lo"], theta_hi=w["theta_hi"], p_s=w["p_s"], p_theta=w["p_theta"],
                  tol=w["tol"])
    sizes = [om.tree.end[s] - om.tree.begin[s] for s in om.tree.leaves]
    return w, X, lt, lm, om, max(sizes) ** 2


def test_benchmark_workload_full_size():
    torch = _torch()
    from paper_2511_03109_amd import api
    w, X, lt, lm, om, ne = _workload(2)
    T, R = w["T"], w["R"]
    thetas = inputs.theta_samples(T, w["theta_lo"], w["theta_hi"], 2)
    inst = api.Instance(lm, thetas)
    assert inst.factored
    x = inputs.normal_vectors(w["n"], T * R, 2).T.reshape(T, R, w["n"])
    y = inst.matvec(torch.tensor(np.ascontiguousarray(x), device="cuda")).cpu().numpy()
    sel, rows = _sample_leaves(om.tree, 32, 32, 128)
    near, _, _, _ = om.blocks_for_rows(rows)
    _compress(om.far_factors, range(len(om.classes)))
    _compress(om.near_factors, near)
    for t in range(T):
        oi = om.instantiate(thetas[t], near_blocks=near if t in (0, T - 1) else [])
        Cg = np.stack([inst.coupling(c, t) for c in range(len(om.classes))])
        Co = np.stack([oi["C"][c] for c in range(len(om.classes))])
        _close(Cg, Co, what=f"all {len(om.classes)} couplings, slot {t}")
        if t in (0, T - 1):
            Dg = np.concatenate([inst.near_block(b, t).ravel() for b in near])
            Do = np.concatenate([oi["D"][b].ravel() for b in near])
            _close(Dg, Do, what=f"{len(near)} near blocks of the sampled rows, slot {t}", max_entries=ne)
        ref = om.matvec_rows_inst(om.instantiate(thetas[t], near_blocks=near), x[t].T, rows)
        _close(y[t][:, rows].T, ref, what=f"rows of {len(sel)} leaves, slot {t}", max_entries=ne)


@pytest.mark.parametrize("near", ["factored", "blocks"])
def test_mixture_sweep_full_size_tuned_graph(near):
    torch = _torch()
    from paper_2511_03109_amd import api
    w, X, lt, lm, om, ne = _workload(3)
    T, R, n = w["T"], w["R"], w["n"]
    thetas = inputs.theta_samples(T, w["theta_lo"], w["theta_hi"], 3)
    inst = api.Instance(lm, thetas, near=near)
    x = torch.tensor(np.ascontiguousarray(inputs.normal_vectors(n, T * R, 3).T.reshape(T, R, n)), device="cuda")
    y = torch.empty_like(x)
    cfg = inst.autotune(x, y)
    print(f"[parity] mixture ({near}) autotune: {cfg}", flush=True)
    s = torch.cuda.Stream()
    g = inst.record(x, y, stream=s)
    th2 = inputs.theta_samples(T, w["theta_lo"], w["theta_hi"], 33)
    g.launch(th2)
    s.synchronize()
    got = y.cpu().numpy()
    ref_eager = torch.empty_like(x)
    inst.reinstantiate(th2)
    inst.matvec(x, ref_eager)
    torch.cuda.synchronize()
    assert torch.equal(torch.tensor(got, device="cuda"), ref_eager)
    del g
    sel, rows = _sample_leaves(om.tree, 12, 2, 128, 260)
    near, _, _, _ = om.blocks_for_rows(rows)
    _compress(om.far_factors, range(len(om.classes)))
    _compress(om.near_factors, near)
    xs = x.cpu().numpy()
    for t in (0, 21, 42, 63):
        ref = om.matvec_rows_inst(om.instantiate(th2[t], near_blocks=near), xs[t].T, rows)
        _close(got[t][:, rows].T, ref, what=f"graph replay, rows of {len(sel)} leaves, slot {t}", max_entries=ne)


def test_gradient_workload_full_size():
    torch = _torch()
    from paper_2511_03109_amd import api
    w, X, lt, lm, om, ne = _workload(4)
    n, l0 = w["n"], w["theta"][0]
    u = inputs.normal_vectors(n, 1, 4, inputs.STREAM_U)[:, 0]
    x = inputs.normal_vectors(n, 1, 4)[:, 0]
    theta = torch.tensor([l0], dtype=torch.float64, requires_grad=True)
    xd = torch.tensor(x, device="cuda", requires_grad=True)
    ud = torch.tensor(u, device="cuda")
    yv = api.k_theta_matvec(lm, theta, xd)
    (yv * ud).sum().backward()
    gth = float(theta.grad[0])
    gx = xd.grad.cpu().numpy()
    dKx = api.Instance(lm, [l0], grad_dim=0).matvec(xd.detach()).cpu().numpy()
    sel, rows = _sample_leaves(om.tree, 48, 0, 10 ** 9)
    near, _, _, _ = om.blocks_for_rows(rows)
    _compress(om.far_factors, range(len(om.classes)))
    _compress(om.near_factors, near)
    _close(yv.detach().cpu().numpy()[rows], om.matvec_rows(l0, x, rows), what="forward rows")
    _close(gx[rows], om.matvec_rows(l0, u, rows), what="dL/dx rows (K~ u)")
    _close(dKx[rows], om.matvec_rows(l0, x, rows, deriv_dim=0), what="dK~/dl x rows")
    # dL/dl = u . dK~/dl x: the library's full-size value against a central difference of its
    # own forward (h = 1e-5): truncation h^2 |L'''| / 6 plus 1e-14 ||u|| ||y|| / h of rounding
    h = 1e-5
    Lp = float((api.Instance(lm, [l0 + h]).matvec(xd.detach()) * ud).sum())
    Lm = float((api.Instance(lm, [l0 - h]).matvec(xd.detach()) * ud).sum())
    fd = (Lp - Lm) / (2 * h)
    bound = 1e-7 * abs(fd) + 1e-14 * float(ud.norm() * yv.detach().norm()) / h
    print(f"[parity] dL/dl {gth:.12e} vs central difference {fd:.12e}: {abs(gth - fd):.3e} (bound {bound:.3e})",
          flush=True)
    assert abs(gth - fd) <= bound
    assert abs(gth - float(np.dot(u, dKx))) <= TOL64 * np.linalg.norm(u) * np.linalg.norm(dKx)


def test_cg_workload_full_size():
    torch = _torch()
    from paper_2511_03109_amd import api
    w, X, lt, lm, om, ne = _workload(5)
    n, th, nug = w["n"], w["theta"][0], w["nugget"]
    y = inputs.normal_vectors(n, 1, 5, inputs.STREAM_Y)[:, 0]
    hi = api.Instance(lm, [th])
    a, st = api.cg_solve(hi, torch.tensor(y, device="cuda"), nugget=nug, tol=1e-6, max_iter=20000)
    print(f"[parity] cg at n = {n}: {st}", flush=True)
    assert st["converged"] == 1 and st["rel_residual"] <= 1e-6
    sel, rows = _sample_leaves(om.tree, 48, 0, 10 ** 9)
    near, _, _, _ = om.blocks_for_rows(rows)
    _compress(om.far_factors, range(len(om.classes)))
    _compress(om.near_factors, near)
    Ka_lib = hi.matvec(a, nugget=nug).cpu().numpy()
    an = a.cpu().numpy()
    Ka_or = om.matvec_rows(th, an, rows, nugget=nug)
    # a solves an ill-conditioned system, so (K~ + nugget I) a cancels: the rounding of each row
    # sum is relative to sum_j |K~_ij| |a_j|, not to the result.  The kernel is positive, so
    # (K~ + nugget I) |a| is that magnitude, and the MVM bound is taken relative to it.
    Kabs_or = om.matvec_rows(th, np.abs(an), rows, nugget=nug)
    err = np.linalg.norm(Ka_lib[rows] - Ka_or)
    print(f"[parity] (K~ + nugget I) a on the rows: {err / np.linalg.norm(Ka_or):.3e} of the result, "
          f"{err / np.linalg.norm(Kabs_or):.3e} of (K~ + nugget I) |a| (cancellation "
          f"{np.linalg.norm(Kabs_or) / np.linalg.norm(Ka_or):.1f}x)", flush=True)
    assert err <= TOL64 * np.linalg.norm(Kabs_or)
    # the residual on the oracle's rows, against the size the reported relative residual
    # implies per row (a loose check: the residual need not be spread evenly over the rows)
    r = y[rows] - Ka_or
    rms_rows = np.linalg.norm(r) / np.sqrt(len(rows))
    rms_all = st["rel_residual"] * np.linalg.norm(y) / np.sqrt(n)
    print(f"[parity] residual rms on {len(rows)} oracle rows {rms_rows:.3e}, over all rows (library) {rms_all:.3e}",
          flush=True)
    assert rms_rows <= 10 * rms_all + TOL64 * np.linalg.norm(Ka_or) / np.sqrt(len(rows))
