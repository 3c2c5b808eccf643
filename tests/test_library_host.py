"""CPU tests of the native library's host logic: symbol exports and the cluster tree,
block lists and translation classes, compared bit for bit with the oracle."""

import os
import re

import numpy as np
import pytest

from oracle import tree as otree
from paper_2511_03109_amd import _lib, api, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "ph.h")).read()
    declared = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(ph_\w+)\s*\(", header, re.M))
    assert len(declared) >= 20
    lib = _lib.lib()
    for name in declared:
        assert hasattr(lib, name), name
    assert set(_lib.SIGNATURES) == declared
    assert lib.ph_version().startswith(b"ph-mi355x")


def _compare(X, l_max, eta2, lo=0.0, hi=1.0):
    n, d = X.shape
    lt = api.Tree(X, lo=lo, hi=hi, l_max=l_max, eta2=eta2)
    ot = otree.build_cluster_tree(X, lo, hi, l_max)
    near_o, far_o = otree.build_block_tree(ot, eta2[0] if eta2[1] == 1 else
                                           __import__("fractions").Fraction(*eta2))
    cls_o, bc_o = otree.translation_classes(ot, far_o)
    assert np.array_equal(lt.perm(), ot.perm)
    nd = lt.nodes()
    assert nd["level"].tolist() == ot.level
    assert [tuple(c) for c in nd["coords"].tolist()] == [tuple(c) for c in ot.coords]
    assert nd["begin"].tolist() == ot.begin and nd["end"].tolist() == ot.end
    assert nd["parent"].tolist() == ot.parent
    near, far, fcls = lt.blocks()
    assert [tuple(b) for b in near.tolist()] == near_o
    assert [tuple(b) for b in far.tolist()] == far_o
    assert fcls.tolist() == bc_o
    lev, off = lt.classes()
    assert [(int(l), tuple(o)) for l, o in zip(lev.tolist(), off.tolist())] == cls_o
    assert lt.info["near_entries"] == sum(len(ot.idx[s]) * len(ot.idx[u]) for s, u in near_o)
    return lt


@pytest.mark.parametrize("wid", [1, 2])
def test_tree_bit_exact_workload_geometry(wid):
    w = inputs.WORKLOADS[wid]
    n = w["n"] if wid == 1 else 8192
    X = inputs.points_for(wid, n)
    l_max = otree.default_l_max(n, w["d"], w["leaf"])
    _compare(X, l_max, w["eta2"])


def test_tree_bit_exact_mixture_uneven():
    X = inputs.points_for(3, 4096)
    _compare(X, 4, (2, 1))


@pytest.mark.parametrize("d,n,l,eta2", [(1, 333, 5, (1, 1)), (2, 100, 4, (2, 1)), (3, 700, 2, (3, 1)),
                                         (2, 50, 0, (2, 1)), (2, 1, 3, (2, 1)), (3, 500, 3, (1, 2))])
def test_tree_bit_exact_small_and_degenerate(d, n, l, eta2):
    X = np.random.default_rng([d, n]).random((n, d))
    _compare(X, l, eta2)


def test_tree_ties_on_split_planes():
    # points on dyadic grid lines: every tie must go to the lower half, as in the oracle
    g = np.arange(0, 9) / 8.0
    X = np.array([(a, b) for a in g for b in g])
    _compare(X, 3, (2, 1))


def test_leaf_size_derivation():
    X = inputs.points_for(1)
    t = api.Tree(X, leaf_size=64, l_max=-1, eta2=(1, 1))
    assert t.info["l_max"] == otree.default_l_max(2048, 2, 64) == 3
    assert t.info["n_near"] == 1012


@pytest.mark.parametrize("bad", ["nan", "outside", "d4", "eta"])
def test_tree_rejects_bad_input(bad):
    X = np.random.default_rng(0).random((10, 2))
    kw = dict(l_max=2)
    if bad == "nan":
        X[3, 1] = np.nan
    elif bad == "outside":
        X[0, 0] = 1.5
    elif bad == "d4":
        X = np.random.default_rng(0).random((10, 4))
    else:
        kw["eta2"] = (0, 1)
    with pytest.raises(_lib.PHError) as e:
        api.Tree(X, **kw)
    assert e.value.code == _lib.PH_EINVAL


def test_entry_points_reject_null_handles():
    """Every entry point that takes a handle returns PH_EINVAL with a message for a NULL one
    (checked before any HIP call, so this runs without a GPU)."""
    import ctypes as C
    lib = _lib.lib()
    d = C.c_double(0.0)
    out = C.c_void_p()
    calls = {
        "ph_tree_info_get": lambda: lib.ph_tree_info_get(None, None),
        "ph_offline_compress": lambda: lib.ph_offline_compress(None, None, None, C.byref(out)),
        "ph_model_info_get": lambda: lib.ph_model_info_get(None, None),
        "ph_instantiate": lambda: lib.ph_instantiate(None, C.byref(d), 1, 0, None, C.byref(out)),
        "ph_instantiate_grad": lambda: lib.ph_instantiate_grad(None, C.byref(d), 1, -1, 0, None,
                                                              C.byref(out)),
        "ph_matvec": lambda: lib.ph_matvec(None, None, None, 1, 1.0, 0.0, 0.0, None),
        "ph_bilinear": lambda: lib.ph_bilinear(None, None, None, 1, None, None),
        "ph_cg_solve": lambda: lib.ph_cg_solve(None, None, None, None, 0.0, 1e-6, 10, 1, 1e-6,
                                               None, None),
        "ph_autotune": lambda: lib.ph_autotune(None, None, None, 1, None, None),
        "ph_graph_create": lambda: lib.ph_graph_create(None, None, None, 1, 0.0, None, C.byref(out)),
        "ph_graph_launch": lambda: lib.ph_graph_launch(None, None, None),
        "ph_inst_near_block": lambda: lib.ph_inst_near_block(None, 0, 0, None),
        "ph_inst_coupling": lambda: lib.ph_inst_coupling(None, 0, 0, None),
    }
    for name, call in calls.items():
        assert call() == _lib.PH_EINVAL, name
        assert lib.ph_last_error(), name
    assert not out.value
    for free in ("ph_tree_free", "ph_model_free", "ph_inst_free", "ph_graph_free"):
        getattr(lib, free)(None)          # freeing NULL is a no-op


@pytest.mark.parametrize("bad,code", [("p_s", _lib.PH_EINVAL), ("p_theta", _lib.PH_EINVAL),
                                      ("tol", _lib.PH_EINVAL), ("box", _lib.PH_EINVAL),
                                      ("d_theta", _lib.PH_EUNSUPPORTED), ("P", _lib.PH_EUNSUPPORTED),
                                      ("aniso3d", _lib.PH_EUNSUPPORTED), ("matern_nu0", _lib.PH_EINVAL)])
def test_offline_rejects_bad_options(bad, code):
    """The offline stage validates its options on the host before any work or upload."""
    d = 3 if bad in ("P", "aniso3d") else 2
    t = api.Tree(np.random.default_rng(1).random((50, d)), l_max=1)
    kernel, lo, hi = "matern12", [0.1], [0.5]
    kw = dict(p_s=4, p_theta=5, tol=1e-8)
    if bad == "p_s":
        kw["p_s"] = 0
    elif bad == "p_theta":
        kw["p_theta"] = 17
    elif bad == "tol":
        kw["tol"] = float("nan")
    elif bad == "box":
        lo, hi = [0.5], [0.5]
    elif bad == "d_theta":
        lo, hi = [0.1, 0.1], [0.5, 0.5]
    elif bad == "P":
        kw["p_s"] = 6                     # 6^3 = 216 > 128
    elif bad == "matern_nu0":
        kernel, lo, hi = "matern", [0.1, 0.0], [0.5, 2.0]   # nu must stay positive on Theta
    else:
        kernel, lo, hi = "aniso_gaussian", [0.1] * 2, [0.5] * 2
    import ctypes as C
    opts = _lib.OfflineOpts()
    opts.kernel = _lib.KERNELS[kernel]
    opts.d_theta = len(lo)
    for k in range(len(lo)):
        opts.theta_lo[k], opts.theta_hi[k] = lo[k], hi[k]
    opts.p_s, opts.p_theta, opts.tol, opts.num_threads = kw["p_s"], kw["p_theta"], kw["tol"], 1
    out = C.c_void_p()
    lib = _lib.lib()
    # NULL stream: the call must fail in the option checks, before anything is uploaded
    assert lib.ph_offline_compress(t._h, C.byref(opts), None, C.byref(out)) == code
    assert lib.ph_last_error() and not out.value
    # the TT-compressed offline stage validates the same options the same way
    assert lib.ph_offline_compress_tt(t._h, C.byref(opts), 1, None, C.byref(out)) == code
    assert not out.value


def test_offline_tt_rejects_bad_coupling():
    import ctypes as C
    t = api.Tree(np.random.default_rng(1).random((50, 2)), l_max=1)
    opts = _lib.OfflineOpts()
    opts.kernel = _lib.KERNELS["gaussian"]
    opts.d_theta = 1
    opts.theta_lo[0], opts.theta_hi[0] = 0.1, 0.5
    opts.p_s, opts.p_theta, opts.tol, opts.num_threads = 4, 5, 1e-8, 1
    out = C.c_void_p()
    assert _lib.lib().ph_offline_compress_tt(t._h, C.byref(opts), 2, None, C.byref(out)) == _lib.PH_EINVAL
    assert not out.value


@pytest.mark.parametrize("d", [1, 2, 3])
def test_kernel_eval_matches_oracle(d):
    """ph_kernel_eval (the library's host kernel values, the ones its offline stage uses)
    against the oracle's kernels.  Closed forms: 8 ulp of 1 (same formulas, different
    rounding order).  Matern with free nu (Bessel K_nu of the library's own routine against
    scipy's): relative 1e-12 over nu in [0.5, 3] and z = sqrt(2 nu) r / lambda from 0 to 40
    (scipy's K_nu is itself accurate to about 1e-13 there); the value 1 at r = 0."""
    from oracle import kernels
    g = np.random.default_rng(40 + d)
    X = g.random((400, d))
    Y = np.concatenate([g.random((399, d)), X[-1:]])     # the last pair at r = 0
    atol = 8 * np.finfo(float).eps
    for name, th in (("gaussian", [0.21]), ("matern32", [0.13]), ("matern12", [0.4])):
        np.testing.assert_allclose(api.kernel_eval(name, X, Y, th), kernels.KERNELS[name][0](X, Y, np.array(th)),
                                   rtol=0, atol=atol)
    if d <= 2:
        th = np.array([0.2, 0.35][:d])
        np.testing.assert_allclose(api.kernel_eval("aniso_gaussian", X, Y, th), kernels.aniso_gaussian(X, Y, th),
                                   rtol=0, atol=atol)
    for lam, nu in ((0.1, 0.5), (0.25, 0.77), (0.3, 1.0), (0.5, 1.5), (0.7, 2.03), (1.0, 2.5), (0.4, 3.0)):
        got = api.kernel_eval("matern", X, Y, [lam, nu])
        ref = kernels.matern(X, Y, np.array([lam, nu]))
        assert got[-1] == 1.0 and ref[-1] == 1.0
        big = ref > 1e-300
        assert np.max(np.abs(got[big] / ref[big] - 1)) <= 1e-12, (lam, nu)
        assert np.all(np.abs(got[~big]) <= 1e-290)


def test_kernel_eval_rejects_bad_input():
    import ctypes as C
    lib = _lib.lib()
    x = np.zeros((2, 2))
    out = np.zeros(2)
    dp = C.POINTER(C.c_double)
    th = np.array([0.5, 1.5])
    call = lambda k, d, thv, n=2: lib.ph_kernel_eval(k, d, x.ctypes.data_as(dp), x.ctypes.data_as(dp), n,
                                                     thv.ctypes.data_as(dp), out.ctypes.data_as(dp))
    assert call(_lib.KERNELS["matern"], 2, th) == _lib.PH_OK
    assert lib.ph_kernel_eval(6, 2, None, None, 2, None, None) == _lib.PH_EINVAL
    assert call(_lib.KERNELS["matern"], 4, th) == _lib.PH_EINVAL
    assert call(_lib.KERNELS["matern"], 2, th, n=-1) == _lib.PH_EINVAL
    assert call(99, 2, th) == _lib.PH_EUNSUPPORTED
    assert call(_lib.KERNELS["matern"], 2, np.array([0.5, 0.0])) == _lib.PH_EDOMAIN
    assert call(_lib.KERNELS["gaussian"], 2, np.array([-0.5])) == _lib.PH_EDOMAIN
    assert lib.ph_last_error()


def test_counter_records_key_on_each_kernel_definition():
    """The benchmark's counter records are keyed by the text of each hot kernel's own
    definition: the extraction finds every kernel, returns exactly one definition (template
    line to closing brace), and an edit outside that text leaves the key unchanged."""
    import bench
    csrc = os.path.join(ROOT, "paper_2511_03109_amd", "csrc")
    for k, files in bench.KERNEL_SOURCES.items():
        text = open(os.path.join(csrc, files[0])).read()
        body = bench.kernel_text(text, k)
        assert body.startswith("template <") and body.endswith("\n}\n")
        assert f" {k}(" in body.split("\n")[1]
        assert body.count("\n}\n") == 1
        h = bench.source_hash(k)
        edited = {f: open(os.path.join(csrc, f)).read() for f in files}
        edited[files[0]] = edited[files[0]] + "\n// trailing edit\n"
        assert bench.source_hash(k, read=lambda f: edited[f]) == h
        edited[files[0]] = edited[files[0]].replace(body, body.replace("{", "{ ", 1))
        assert bench.source_hash(k, read=lambda f: edited[f]) != h


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU; --gpus N > 1 exits with a message before touching a GPU."""
    import json
    import subprocess
    import sys
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode != 0
    msg = json.loads(res.stdout.strip().splitlines()[-1])["error"]
    assert "single GPU" in msg


@pytest.mark.parametrize("kernel,d,lo,hi,p_s,p_theta,tol", [
    ("gaussian", 2, [0.05], [0.5], 5, 7, 1e-8),
    ("matern32", 3, [0.1], [0.6], 4, 5, 1e-6),
    ("matern", 2, [0.25, 0.5], [1.0, 3.0], 4, 5, 1e-6),
])
def test_tt_far_ranks_match_oracle(kernel, d, lo, hi, p_s, p_theta, tol):
    """ph_tt_far_ranks (host only, no GPU): the TT ranks of every translation class's far tensor
    and the number of kernel values evaluated equal those of the oracle's TT-cross on the same
    tensors (same pivots; mirrored classes reversed)."""
    from fractions import Fraction
    from oracle import hmat, kernels
    n, l_max, eta2 = (900, 3, (2, 1)) if d == 2 else (1200, 2, (3, 1))
    X = np.random.default_rng([21, d]).random((n, d))
    t = api.Tree(X, l_max=l_max, eta2=eta2)
    ranks, ev = api.tt_far_ranks(t, kernel, lo, hi, p_s=p_s, p_theta=p_theta, tol=tol)
    om = hmat.PH2(X, l_max=l_max, eta2=Fraction(*eta2), kernel=kernels.KERNELS[kernel][0], theta_lo=lo,
                  theta_hi=hi, p_s=p_s, p_theta=p_theta, tol=tol, compress="tt")
    assert ranks.shape == (len(om.classes), 2 * d + len(lo) + 1)
    for key in range(len(om.classes)):
        mk = om._mirror_key(key)
        cores = om.far_tt_cores(mk if mk is not None else key)
        r = [c.shape[0] for c in cores] + [1]
        if mk is not None:
            r = r[::-1]
        assert list(ranks[key]) == r, f"class {key} {om.classes[key]}"
    assert ev == om.tt_evals
