"""Benchmark: online stage of the parametric H^2-matrix on one MI355X.

One step = instantiate K~(theta) at T = 8 parameter values (one ph_instantiate call:
parametric vectors, far couplings, near blocks) + the H^2 MVM of each instance with
R = 16 right-hand sides (one ph_matvec call), on n = 65536 points uniform in [0,1]^3
with the Matern-3/2 kernel, l in [0.05, 0.5], 5^3 spatial / 11 parameter Chebyshev
nodes, tolerance 1e-8.  Inputs are resident on the device before timing.

Prints one JSON line.  value = ms per theta (instantiate + MVM), lower is better.
"""

import argparse
import json
import os
import sys
import time
from fractions import Fraction

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ms per θ-instantiate + H-MVM and HBM GB/s at n=65536; batched/BF16 vs FP64"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_MFMA_PEAK_TFS = 78.6      # MI355X dense FP64 matrix
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
CSRC = os.path.join(ROOT, "paper_2511_03109_amd", "csrc")
# source files whose text determines each hot kernel's code: the kernel's own definition in
# the first file (template line to closing brace), the whole shared header
KERNEL_SOURCES = {
    "k_coupling": ["k_matvec.hip", "ph_device.hpp"],
    "k_near_mvm": ["k_matvec.hip", "ph_device.hpp"],
    "k_near_instantiate": ["k_instantiate.hip", "ph_device.hpp"],
    "k_near_fused": ["k_near_fused.hip", "ph_device.hpp"],
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_text(text, kernel):
    """The definition of `kernel` in a source text: from its template line to the first
    closing brace in column 0."""
    import re
    m = re.search(r"^template <[^>]*>\n__global__[^\n]*\b" + kernel + r"\(", text, re.M)
    if m is None:
        raise KeyError(kernel)
    end = text.index("\n}\n", m.start())
    return text[m.start():end + 3]


def source_hash(kernel, read=None):
    """Hash of the kernel's definition and the shared header; read(f) returns a source
    file's text (default: the working tree)."""
    import hashlib
    if read is None:
        def read(f):
            with open(os.path.join(CSRC, f)) as fh:
                return fh.read()
    files = KERNEL_SOURCES[kernel]
    h = hashlib.sha256()
    h.update(kernel_text(read(files[0]), kernel).encode())
    for f in files[1:]:
        h.update(read(f).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch from the committed counter record, or None when absent or
    taken on a different version of the kernel's source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh).get(kernel)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha") != source_hash(kernel):
        return None
    return rec["bytes_per_launch"]


def cpu_baseline(w, X, l_max, thetas, x_host, sample_leaves=160):
    """Time the CPU oracle on a bounded sample of the same workload.

    Sample: all rows of `sample_leaves` target leaves spread over the tree, for every
    theta of the step and the workload's R right-hand sides.  Timed per theta: the
    parametric vectors, near-field instantiation of those leaves' near blocks,
    instantiation of every far coupling, the full upward pass, and the coupling / near
    products / downward pass of those leaves' paths.  The per-leaf parts are scaled
    linearly to all leaves.  Compression (the offline stage) is not timed.
    """
    from threadpoolctl import threadpool_info

    from oracle import hmat, kernels
    t0 = time.time()
    om = hmat.PH2(X, l_max=l_max, eta2=Fraction(*w["eta2"]), kernel=kernels.KERNELS[w["kernel"]][0],
                  theta_lo=w["theta_lo"], theta_hi=w["theta_hi"], p_s=w["p_s"], p_theta=w["p_theta"],
                  tol=w["tol"])
    t = om.tree
    leaves = [t.leaves[i] for i in np.linspace(0, len(t.leaves) - 1, sample_leaves).astype(int)]
    rows = np.concatenate([t.perm[t.begin[s]:t.end[s]] for s in leaves])
    near, _, _, _ = om.blocks_for_rows(rows)
    all_keys = list(range(len(om.classes)))
    for k in all_keys:
        om.far_factors(k)
    for b in near:
        om.near_factors(b)
    log(f"[cpu_baseline] oracle setup + compression (untimed) {time.time() - t0:.1f} s")
    nleaf = len(t.leaves)
    scale = nleaf / sample_leaves
    est, measured = [], 0.0
    for ti, theta in enumerate(thetas):
        xs = x_host[ti].T                     # (n, R)
        ta = time.perf_counter()
        vs = om.theta_vectors(theta)
        D = {b: om.near_block(b, vs) for b in near}
        tb = time.perf_counter()
        C = {k: om.coupling(k, vs) for k in all_keys}
        tc = time.perf_counter()
        om._upward(xs[t.perm])
        td = time.perf_counter()
        om.matvec_rows_inst({"D": D, "C": C}, xs, rows)
        te = time.perf_counter()
        # matvec_rows_inst repeats the upward pass: subtract it from the per-leaf part
        per_leaf_mvm = max((te - td) - (td - tc), 0.0)
        est.append((tb - ta) * scale + (tc - tb) + (td - tc) + per_leaf_mvm * scale)
        measured += te - ta
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {
        "value": float(np.mean(est)) * 1e3, "unit": "ms per theta (instantiate + MVM, 16 RHS), extrapolated",
        "cores": int(threads), "kind": "oracle", "cpu_model": cpu_model,
        "host_cpus_visible": len(os.sched_getaffinity(0)),
        "sample": f"{sample_leaves} of {nleaf} target leaves ({len(rows)} rows, {len(near)} near blocks) for "
                  f"each of {len(thetas)} theta, all {len(all_keys)} far couplings, full upward pass; "
                  f"per-leaf work scaled by {scale:.0f}x; measured {measured:.1f} s of oracle work",
    }


# ---------------------------------------------------------------- secondary measurements
def _model(wid, n=None):
    from paper_2511_03109_amd import api, inputs
    w = inputs.WORKLOADS[wid]
    X = inputs.points_for(wid) if n is None else inputs.points_for(wid, n)
    t0 = time.time()
    tree = api.Tree(X, leaf_size=w["leaf"], l_max=-1, eta2=tuple(w["eta2"]))
    model = api.Model(tree, w["kernel"], w["theta_lo"], w["theta_hi"], p_s=w["p_s"], p_theta=w["p_theta"],
                      tol=w["tol"])
    log(f"[bench] {w['name']}: offline stage {time.time() - t0:.1f} s; tree {tree.info}; model {model.info}")
    return w, X, tree, model


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def step_legs(model, thetas, x_host, T, R, y64, args):
    """The same work in other forms, each timed like the headline (events around K steps
    after W warm-up steps): FP64 one theta at a time (T = 1 instances, near blocks in
    memory), FP64 batched with the near blocks in memory, FP64 batched after ph_autotune (which
    may run the near field concurrently with the far field), FP32 and BF16 batched.  Each
    low-precision result's relative error is taken against the FP64 headline output y64
    (which matches the oracle to 1e-12)."""
    import torch
    from paper_2511_03109_amd import api
    steps, warmup = max(3, min(args.steps, 10)), max(1, args.warmup)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    legs = {}
    x64 = torch.tensor(np.ascontiguousarray(x_host), device="cuda")
    # one theta at a time: T separate instances of one slot each
    singles = [api.Instance(model, thetas[t:t + 1]) for t in range(T)]
    ys = torch.empty_like(x64)

    def per_theta():
        for t in range(T):
            singles[t].reinstantiate(thetas[t:t + 1])
            singles[t].matvec(x64[t], ys[t])
    ms = timed(per_theta)
    legs["fp64_one_theta_at_a_time"] = {"ms_per_theta": ms / T, "near_field": "blocks in memory", "T": 1,
                                        "rel_error_vs_headline": float((ys - y64).norm() / y64.norm())}
    del singles
    ib = api.Instance(model, thetas, near="blocks")
    yb = torch.empty_like(x64)
    ms = timed(lambda: (ib.reinstantiate(thetas), ib.matvec(x64, yb)))
    legs["fp64_batched_blocks_in_memory"] = {"ms_per_theta": ms / T, "T": T,
                                             "rel_error_vs_headline": float((yb - y64).norm() / y64.norm())}
    del ib, yb
    torch.cuda.empty_cache()
    # the headline step after ph_autotune on the same instance shape: coupling chunks, prefetch
    # depth, near field on the instance's second stream or not, near-field launch shape
    ia = api.Instance(model, thetas)
    ya = torch.empty_like(x64)
    cfg = ia.autotune(x64, ya)
    ms = timed(lambda: (ia.reinstantiate(thetas), ia.matvec(x64, ya)))
    legs["fp64_autotuned"] = {"ms_per_theta": ms / T, "T": T, "config": cfg,
                              "rel_error_vs_headline": float((ya - y64).norm() / y64.norm())}
    del ia, ya
    torch.cuda.empty_cache()
    x32 = x64.float()
    for dt in ("f32", "bf16"):
        inst = api.Instance(model, thetas, dtype=dt)
        yl = torch.empty_like(x32)
        ms = timed(lambda: (inst.reinstantiate(thetas), inst.matvec(x32, yl)))
        legs[dt + "_batched"] = {"ms_per_theta": ms / T, "T": T, "factored": inst.factored,
                                 "rel_error_vs_fp64": float((yl.double() - y64).norm() / y64.norm())}
        del inst, yl
        torch.cuda.empty_cache()
    return legs


def mode_precision(args):
    """The benchmark step with FP64, FP32 and BF16 instances; error of each against the FP64
    instance (which matches the oracle to 1e-12) on the full output."""
    import torch
    from paper_2511_03109_amd import api, inputs
    w, X, tree, model = _model(2)
    n, T, R = w["n"], w["T"], w["R"]
    thetas = inputs.theta_samples(T, w["theta_lo"], w["theta_hi"], 2)
    xh = np.ascontiguousarray(inputs.normal_vectors(n, T * R, 2).T.reshape(T, R, n))
    res, y64 = {}, None
    for dt in ("f64", "f32", "bf16"):
        tdt = torch.float64 if dt == "f64" else torch.float32
        x = torch.tensor(xh, device="cuda", dtype=tdt)
        y = torch.empty_like(x)
        inst = api.Instance(model, thetas, dtype=dt)
        ms_inst = _timed(lambda: inst.reinstantiate(thetas), args.steps, args.warmup)
        ms_mvm = _timed(lambda: inst.matvec(x, y), args.steps, args.warmup)
        ms_step = _timed(lambda: (inst.reinstantiate(thetas), inst.matvec(x, y)), args.steps, args.warmup)
        yd = y.double()
        if y64 is None:
            y64 = yd.clone()
        err = float(torch.linalg.vector_norm(yd - y64) / torch.linalg.vector_norm(y64))
        res[dt] = {"ms_per_theta": ms_step / T, "ms_instantiate_per_theta": ms_inst / T,
                   "ms_matvec_per_theta": ms_mvm / T, "rel_error_vs_fp64": err}
        del inst
        torch.cuda.empty_cache()
    for dt in ("f32", "bf16"):
        res[dt]["speedup_vs_fp64"] = res["f64"]["ms_per_theta"] / res[dt]["ms_per_theta"]
    print(json.dumps({"metric": "ms per θ-instantiate + H-MVM by precision", "unit": "ms per theta",
                      "higher_is_better": False, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "config": {"workload": w["name"], "T": T, "R": R}, "data": "synthetic", "results": res}))


def mode_cg(args):
    """(K~(l) + 1e-2 I) a = y at n = 262144 (Matern-1/2, l = 0.1) to relative residual 1e-6
    in FP64: plain FP64 CG against FP64 refinement around FP32 and BF16 inner solves."""
    import torch
    from paper_2511_03109_amd import api, inputs
    w, X, tree, model = _model(5)
    n, nug, th = w["n"], w["nugget"], w["theta"][0]
    y = torch.tensor(inputs.normal_vectors(n, 1, 5, inputs.STREAM_Y)[:, 0], device="cuda")
    res = {}
    for lo_dt in (None, "f32", "bf16"):
        t0 = time.perf_counter()
        hi = api.Instance(model, [th])
        lo = api.Instance(model, [th], dtype=lo_dt) if lo_dt else None
        torch.cuda.synchronize()
        t_inst = time.perf_counter() - t0
        t0 = time.perf_counter()
        # inner tolerance: FP32 solves the correction almost to the target (one or two FP64
        # refinement steps); BF16 is asked for two digits per step
        a, st = api.cg_solve(hi, y, nugget=nug, tol=1e-6, lo=lo, max_iter=20000 if lo is None else 60,
                             inner_max=20000, inner_tol=1e-2 if lo_dt == "bf16" else 5e-7)
        torch.cuda.synchronize()
        t_solve = time.perf_counter() - t0
        mvm = _timed(lambda: (lo or hi).matvec(y if lo is None else y.float()), 5, 2)
        res[lo_dt or "f64"] = {"solve_s": t_solve, "instantiate_s": t_inst, "stats": st,
                               "ms_per_inner_matvec": mvm}
        del hi, lo, a
        torch.cuda.empty_cache()
    for k in ("f32", "bf16"):
        if res[k]["stats"]["converged"]:
            res[k]["speedup_vs_fp64_cg"] = res["f64"]["solve_s"] / res[k]["solve_s"]
    # the batched form: 16 right-hand sides solved together (ph_cg_solve_batch), every column to
    # the same 1e-6 FP64 residual; time per solve against the single-RHS FP64 CG
    RB = 16
    Yb = torch.tensor(np.ascontiguousarray(inputs.normal_vectors(n, RB, 5, inputs.STREAM_Y).T), device="cuda")
    for lo_dt in (None, "f32"):
        hi = api.Instance(model, [th])
        lo = api.Instance(model, [th], dtype=lo_dt) if lo_dt else None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a, st = api.cg_solve(hi, Yb, nugget=nug, tol=1e-6, lo=lo, max_iter=20000 if lo is None else 60,
                             inner_max=20000, inner_tol=5e-7)
        torch.cuda.synchronize()
        t_solve = time.perf_counter() - t0
        key = f"batched16_{lo_dt or 'f64'}"
        res[key] = {"solve_s": t_solve, "solve_s_per_rhs": t_solve / RB, "stats": st,
                    "speedup_per_rhs_vs_fp64_cg": res["f64"]["solve_s"] / (t_solve / RB) if st["converged"] else None}
        del hi, lo, a
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "solve time to relative residual 1e-6, FP64 CG vs FP64-refined FP32/BF16, single and 16 RHS",
                      "unit": "s", "higher_is_better": False, "n_gpus": 1,
                      "config": {"workload": w["name"], "n": n, "theta": th, "nugget": nug}, "data": "synthetic",
                      "results": res}))


def mode_grad(args):
    """Forward y = K~(l) x and backward of L = u . y (dL/dl, dL/dx) through the autograd
    Function at n = 131072; the gradient against a central difference with h = 1e-5."""
    import torch
    from paper_2511_03109_amd import api, inputs
    w, X, tree, model = _model(4)
    n, th = w["n"], w["theta"][0]
    u = torch.tensor(inputs.normal_vectors(n, 1, 4, inputs.STREAM_U)[:, 0], device="cuda")
    xv = torch.tensor(inputs.normal_vectors(n, 1, 4)[:, 0], device="cuda")

    def fwd_bwd():
        theta = torch.tensor([th], dtype=torch.float64, requires_grad=True)
        x = xv.clone().requires_grad_(True)
        L = (api.k_theta_matvec(model, theta, x) * u).sum()
        L.backward()
        return theta.grad, x.grad, L

    ms_fb = _timed(fwd_bwd, args.steps, args.warmup)

    def fwd():
        with torch.no_grad():
            return (api.k_theta_matvec(model, torch.tensor([th], dtype=torch.float64), xv) * u).sum()

    ms_f = _timed(fwd, args.steps, args.warmup)
    g, gx, L = fwd_bwd()
    h = 1e-5
    Lp = float((api.Instance(model, [th + h]).matvec(xv) * u).sum())
    Lm = float((api.Instance(model, [th - h]).matvec(xv) * u).sum())
    fd = (Lp - Lm) / (2 * h)
    print(json.dumps({"metric": "ms per forward + backward of y = K(l) x", "value": ms_fb, "unit": "ms",
                      "higher_is_better": False, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "config": {"workload": w["name"], "n": n, "theta": th}, "data": "synthetic",
                      "ms_forward": ms_f, "dL_dl": float(g[0]), "central_difference": fd,
                      "rel_diff_vs_fd": abs(float(g[0]) - fd) / abs(fd)}))


def mode_sweep(args):
    """64 (l1, l2) of the anisotropic Gaussian on the 8-component mixture, 32 RHS each: one
    instance of T = 64 slots, autotuned, instantiate + MVM recorded as one graph."""
    import torch
    from paper_2511_03109_amd import api, inputs
    w, X, tree, model = _model(3)
    n, T, R = w["n"], w["T"], w["R"]
    thetas = inputs.theta_samples(T, w["theta_lo"], w["theta_hi"], 3)
    x = torch.tensor(np.ascontiguousarray(inputs.normal_vectors(n, T * R, 3).T.reshape(T, R, n)), device="cuda")
    y = torch.empty_like(x)
    inst = api.Instance(model, thetas)
    ms_eager_default = _timed(lambda: (inst.reinstantiate(thetas), inst.matvec(x, y)), args.steps, args.warmup)
    cfg = inst.autotune(x, y)
    ms_eager = _timed(lambda: (inst.reinstantiate(thetas), inst.matvec(x, y)), args.steps, args.warmup)
    s = torch.cuda.Stream()
    g = inst.record(x, y, stream=s)
    rng = np.random.default_rng(3)
    batches = [rng.uniform(w["theta_lo"], w["theta_hi"], (T, 2)) for _ in range(4)]
    k = [0]

    def replay():
        g.launch(batches[k[0] % 4])
        k[0] += 1

    with torch.cuda.stream(s):
        ms_graph = _timed(replay, args.steps, args.warmup)
    print(json.dumps({"metric": "ms per θ-instantiate + H-MVM in a 64-θ sweep (recorded graph)",
                      "value": ms_graph / T, "unit": "ms per theta (32 RHS)", "higher_is_better": False,
                      "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "config": {"workload": w["name"], "n": n, "T": T, "R": R}, "data": "synthetic",
                      "autotuned": cfg, "ms_per_theta_eager_default": ms_eager_default / T,
                      "ms_per_theta_eager_tuned": ms_eager / T, "model": model.info}))


def mode_matern(args):
    """Matern kernel with free smoothness, theta = (lambda, nu) on [0.1, 1] x [0.5, 3], n = 8^4 in
    [0,1]^3 (the paper's larger-parameter-range setting): offline time, then 8 (lambda, nu)
    instantiated and applied to 16 RHS each, timed like the headline, with per-stage times."""
    import torch
    from paper_2511_03109_amd import _lib, api, inputs
    t0 = time.time()
    w, X, tree, model = _model(6)
    offline_s = time.time() - t0
    n, T, R = w["n"], w["T"], w["R"]
    thetas = inputs.theta_samples(T, w["theta_lo"], w["theta_hi"], 6)
    x = torch.tensor(np.ascontiguousarray(inputs.normal_vectors(n, T * R, 6).T.reshape(T, R, n)), device="cuda")
    y = torch.empty_like(x)
    inst = api.Instance(model, thetas)
    ms = _timed(lambda: (inst.reinstantiate(thetas), inst.matvec(x, y)), args.steps, args.warmup)
    lib = _lib.lib()
    stats = _lib.TraceStats()
    lib.ph_trace_read(stats, 1)
    lib.ph_trace_enable(1)
    for _ in range(5):
        inst.reinstantiate(thetas)
        inst.matvec(x, y)
    torch.cuda.synchronize()
    lib.ph_trace_enable(0)
    _lib.check(lib.ph_trace_read(stats, 1), "ph_trace_read")
    stages = {nm: stats.ms[i] / 5 for i, nm in enumerate(_lib.STAGES) if stats.count[i]}
    print(json.dumps({"metric": "ms per (lambda, nu)-instantiate + H-MVM, Matern with free nu",
                      "value": ms / T, "unit": "ms per theta (16 RHS)", "higher_is_better": False,
                      "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
                      "config": {"workload": w["name"], "n": n, "theta_box": [w["theta_lo"], w["theta_hi"]],
                                 "p_s": w["p_s"], "p_theta": w["p_theta"], "T": T, "R": R,
                                 "near_field": "factored" if inst.factored else "blocks"},
                      "data": "synthetic", "offline_s": offline_s, "stage_ms_per_step": stages,
                      "model": model.info}))


def mode_hmatrix(args):
    """The parametric H-matrix format against the H^2 format on the same workload (E kernel,
    lambda in [0.25, 1], n = 8^5 in [0,1]^3, the paper's parameter space): offline time of each,
    then 8 lambda instantiated and applied to 16 RHS each, timed like the headline, with
    per-stage times; relative difference of the two outputs."""
    import torch
    from paper_2511_03109_amd import _lib, api, inputs
    w = inputs.WORKLOADS[7]
    n, T, R = w["n"], w["T"], w["R"]
    X = inputs.points_for(7)
    tree = api.Tree(X, leaf_size=w["leaf"], l_max=-1, eta2=tuple(w["eta2"]))
    thetas = inputs.theta_samples(T, w["theta_lo"], w["theta_hi"], 7)
    x = torch.tensor(np.ascontiguousarray(inputs.normal_vectors(n, T * R, 7).T.reshape(T, R, n)), device="cuda")
    lib = _lib.lib()
    res, ys = {}, {}
    for fmt in ("h", "h2"):
        t0 = time.time()
        model = api.Model(tree, w["kernel"], w["theta_lo"], w["theta_hi"], p_s=w["p_s"], p_theta=w["p_theta"],
                          tol=w["tol"], format=fmt)
        torch.cuda.synchronize()
        offline_s = time.time() - t0
        y = torch.empty_like(x)
        inst = api.Instance(model, thetas)
        ms = _timed(lambda: (inst.reinstantiate(thetas), inst.matvec(x, y)), args.steps, args.warmup)
        stats = _lib.TraceStats()
        lib.ph_trace_read(stats, 1)
        lib.ph_trace_enable(1)
        for _ in range(3):
            inst.reinstantiate(thetas)
            inst.matvec(x, y)
        torch.cuda.synchronize()
        lib.ph_trace_enable(0)
        _lib.check(lib.ph_trace_read(stats, 1), "ph_trace_read")
        res[fmt] = {"ms_per_theta": ms / T, "offline_s": offline_s,
                    "stage_ms_per_step": {nm: stats.ms[i] / 3 for i, nm in enumerate(_lib.STAGES) if stats.count[i]},
                    "device_bytes": model.info["device_bytes"]}
        ys[fmt] = y.clone()
        del inst, model
        torch.cuda.empty_cache()
    diff = float(torch.linalg.vector_norm(ys["h"] - ys["h2"]) / torch.linalg.vector_norm(ys["h2"]))
    print(json.dumps({"metric": "ms per lambda-instantiate + MVM, parametric H-matrix vs H^2 format",
                      "value": res["h"]["ms_per_theta"], "unit": "ms per theta (16 RHS)", "higher_is_better": False,
                      "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "config": {"workload": w["name"], "n": n, "T": T, "R": R, "p_s": w["p_s"],
                                 "p_theta": w["p_theta"], "theta_box": [w["theta_lo"], w["theta_hi"]]},
                      "data": "synthetic", "results": res, "rel_diff_h_vs_h2": diff}))


def mode_offline(args):
    """The offline stage with the kernel tensors evaluated on the host against on the GPU (the
    compression runs on the host in both), for the benchmark workload and the Matern free-nu
    workload; seconds per offline stage and the relative difference of the two models' MVMs."""
    import torch
    from paper_2511_03109_amd import api, inputs
    out = {}
    for wid in (2, 6):
        w = inputs.WORKLOADS[wid]
        X = inputs.points_for(wid)
        tree = api.Tree(X, leaf_size=w["leaf"], l_max=-1, eta2=tuple(w["eta2"]))
        thetas = inputs.theta_samples(1, w["theta_lo"], w["theta_hi"], wid)
        x = torch.tensor(np.ascontiguousarray(inputs.normal_vectors(w["n"], 16, wid).T), device="cuda")
        res, ys = {}, {}
        for where in ("host", "gpu"):
            torch.cuda.synchronize()
            t0 = time.time()
            model = api.Model(tree, w["kernel"], w["theta_lo"], w["theta_hi"], p_s=w["p_s"],
                              p_theta=w["p_theta"], tol=w["tol"], offline=where)
            torch.cuda.synchronize()
            res[where + "_s"] = time.time() - t0
            ys[where] = api.Instance(model, thetas).matvec(x)
            res["kernel_evals"] = model.info["kernel_evals"]
            del model
        res["rel_diff_mvm"] = float(torch.linalg.vector_norm(ys["gpu"] - ys["host"]) /
                                    torch.linalg.vector_norm(ys["host"]))
        res["speedup"] = res["host_s"] / res["gpu_s"]
        out[w["name"]] = res
        log(f"[bench] offline {w['name']}: {res}")
    print(json.dumps({"metric": "offline stage seconds, kernel tensors on the host vs on the GPU",
                      "unit": "s", "higher_is_better": False, "n_gpus": 1, "data": "synthetic", "results": out}))


def mode_tt(args):
    """The paper's compression (TT-cross + TT-rounding) against the truncated HOSVD on the same
    workloads (the benchmark, Matern-3/2 n = 65536, and the E kernel at n = 8^5 with the paper's
    lambda box): host offline seconds, kernel evaluations, mean ranks and device bytes of each;
    then 8 theta instantiated and applied to 16 RHS each, timed like the headline, for the HOSVD
    model (couplings formed), the TT model with couplings formed and the TT model with the
    implicit coupling of Alg. "Modified H^2-Matrix MVM"; relative differences of the outputs."""
    import torch
    from paper_2511_03109_amd import _lib, api, inputs
    lib = _lib.lib()
    out = {}
    for wid in (7, 2):
        w = inputs.WORKLOADS[wid]
        n, T, R = w["n"], w["T"], w["R"]
        X = inputs.points_for(wid)
        tree = api.Tree(X, leaf_size=w["leaf"], l_max=-1, eta2=tuple(w["eta2"]))
        thetas = inputs.theta_samples(T, w["theta_lo"], w["theta_hi"], wid)
        x = torch.tensor(np.ascontiguousarray(inputs.normal_vectors(n, T * R, wid).T.reshape(T, R, n)), device="cuda")
        res, ys = {}, {}
        for name, kw in (("hosvd", {}), ("tt", {"compress": "tt"}),
                         ("tt_implicit", {"compress": "tt", "coupling": "implicit"})):
            torch.cuda.synchronize()
            t0 = time.time()
            model = api.Model(tree, w["kernel"], w["theta_lo"], w["theta_hi"], p_s=w["p_s"], p_theta=w["p_theta"],
                              tol=w["tol"], **kw)
            torch.cuda.synchronize()
            offline_s = time.time() - t0
            y = torch.empty_like(x)
            inst = api.Instance(model, thetas)
            ms = _timed(lambda: (inst.reinstantiate(thetas), inst.matvec(x, y)), args.steps, args.warmup)
            stats = _lib.TraceStats()
            lib.ph_trace_read(stats, 1)
            lib.ph_trace_enable(1)
            for _ in range(3):
                inst.reinstantiate(thetas)
                inst.matvec(x, y)
            torch.cuda.synchronize()
            lib.ph_trace_enable(0)
            _lib.check(lib.ph_trace_read(stats, 1), "ph_trace_read")
            info = model.info
            res[name] = {"offline_s": offline_s, "kernel_evals": info["kernel_evals"],
                         "far_rank_mean": info["far_rank_mean"], "near_rank_mean": info["near_rank_mean"],
                         "device_bytes": info["device_bytes"], "ms_per_theta": ms / T,
                         "stage_ms_per_step": {nm: stats.ms[i] / 3 for i, nm in enumerate(_lib.STAGES)
                                               if stats.count[i]}}
            ys[name] = y.clone()
            log(f"[bench] tt {w['name']} {name}: {res[name]}")
            del inst, model
            torch.cuda.empty_cache()
        for name in ("tt", "tt_implicit"):
            res[name]["rel_diff_vs_hosvd"] = float(torch.linalg.vector_norm(ys[name] - ys["hosvd"]) /
                                                   torch.linalg.vector_norm(ys["hosvd"]))
        res["rel_diff_implicit_vs_formed"] = float(torch.linalg.vector_norm(ys["tt_implicit"] - ys["tt"]) /
                                                   torch.linalg.vector_norm(ys["tt"]))
        out[w["name"]] = res
    print(json.dumps({"metric": "TT-cross vs HOSVD compression; formed vs implicit coupling",
                      "unit": "ms per theta (16 RHS) / s offline", "higher_is_better": False, "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "data": "synthetic", "results": out}))


def mode_ttrank(args):
    """The TT compression at the paper's parametric H^2 configuration (Matern (lambda, nu) in
    [0.25, 1] x [0.5, 3], n = 8^4 and 8^5 uniform in [0,1]^3, l_max 2 and 3, eta = sqrt(3),
    p_s = 8, p_theta = 27, tol 1e-5): the TT ranks of every translation class's far tensor
    (ph_tt_far_ranks, host only; P = 512 is beyond the online kernels, so no model is built),
    then the paper's Rank (mean over far blocks of max(r_d, r_{d+d_theta})) and Coupling Ratio
    (entries of the TT-stored couplings of all far blocks over n^2), next to the values the paper
    prints for its own TT-cross.  The printed Coupling Ratio formula lists the spatial cores
    1..3 and, on the source side, only the last two; the plain ratios count all 2 d spatial cores
    (p_s r_{i-1} r_i each) plus r_d r_{d+d_theta}, the `_as_printed` ones the printed terms.  The
    formula sums over far blocks, but the printed values match one coupling per translation
    class; both counts are reported."""
    from paper_2511_03109_amd import api
    paper = {4: 0.14734703302383423, 5: 0.004155942238867283}   # Table "ph_h2_induced", MN
    out = {}
    d, dth, ps = 3, 2, 8
    N = 2 * d + dth
    for e, l_max in ((4, 2), (5, 3)):
        n = 8 ** e
        X = np.random.default_rng([17, e]).random((n, d))
        tree = api.Tree(X, l_max=l_max, eta2=(3, 1))
        t0 = time.time()
        ranks, ev = api.tt_far_ranks(tree, "matern", [0.25, 0.5], [1.0, 3.0], p_s=ps, p_theta=27, tol=1e-5)
        secs = time.time() - t0
        _, _, fcls = tree.blocks()
        nb = np.bincount(fcls, minlength=ranks.shape[0]).astype(np.float64)
        r = ranks.astype(np.float64)
        rank = float(np.sum(nb * np.maximum(r[:, d], r[:, d + dth])) / np.sum(nb))
        spatial = sum(r[:, i - 1] * r[:, i] for i in range(1, d + 1)) + \
            sum(r[:, i - 1] * r[:, i] for i in range(d + dth + 1, N + 1))
        printed = sum(r[:, i - 1] * r[:, i] for i in range(1, d + 1)) + \
            sum(r[:, i] * r[:, i + 1] for i in range(d + dth + 1, N))
        mid = r[:, d] * r[:, d + dth]
        cr = float(np.sum(nb * (ps * spatial + mid)) / n ** 2)
        cr_p = float(np.sum(nb * (ps * printed + mid)) / n ** 2)
        # one stored coupling per translation class (Sec. 5.2): the paper's printed values match
        # this count, not one per far block
        cr_c = float(np.sum(ps * spatial + mid) / n ** 2)
        cr_cp = float(np.sum(ps * printed + mid) / n ** 2)
        out[f"n=8^{e}"] = {"classes": int(ranks.shape[0]), "far_blocks": int(nb.sum()), "rank": rank,
                           "coupling_ratio_per_class": cr_c, "coupling_ratio_per_class_as_printed": cr_cp,
                           "coupling_ratio_per_block": cr, "coupling_ratio_per_block_as_printed": cr_p,
                           "paper_coupling_ratio": paper[e], "tt_ranks_mean": [float(v) for v in r.mean(axis=0)],
                           "kernel_evals": int(ev), "seconds": secs}
        log(f"[bench] ttrank n=8^{e}: {out[f'n=8^{e}']}")
    print(json.dumps({"metric": "TT ranks and coupling ratio at the paper's parametric H^2 configuration (MN)",
                      "unit": "ratio", "data": "synthetic", "results": out}))


MODES = {"precision": mode_precision, "cg": mode_cg, "grad": mode_grad, "sweep": mode_sweep,
         "matern": mode_matern, "hmatrix": mode_hmatrix, "offline": mode_offline, "tt": mode_tt,
         "ttrank": mode_ttrank}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-leaves", type=int, default=160)
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the comparison legs (per-theta FP64, near blocks in memory, FP32, BF16)")
    ap.add_argument("--mode", default="step", choices=["step", "precision", "cg", "grad", "sweep", "matern", "hmatrix",
                                                    "offline", "tt", "ttrank"],
                    help="step (default): the benchmark step; precision: FP64 / FP32 / BF16 instances of "
                         "the same step; cg: (K + 1e-2 I) a = y at n = 262144 by FP64 CG and by FP64 "
                         "refinement around FP32 / BF16; grad: forward + backward of y = K(l) x at "
                         "n = 131072; sweep: 64 theta x 32 RHS on the mixture, one recorded graph")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes 5 times (to scale "
                         "profiler byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.empty(args.copy_calibration // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_calibration, "repeats": 5}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "--gpus must be 1: the library runs on a single GPU "
                                   "(sharding across GPUs is not implemented)"}))
        sys.exit(2)
    if args.mode != "step":
        MODES[args.mode](args)
        return

    import torch

    from paper_2511_03109_amd import _lib, api, inputs

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    torch.cuda.set_device(0)
    wid = 2
    w = inputs.WORKLOADS[wid]
    n, T, R = w["n"], w["T"], w["R"]
    X = inputs.points_for(wid)
    t0 = time.time()
    tree = api.Tree(X, leaf_size=w["leaf"], l_max=-1, eta2=tuple(w["eta2"]))
    model = api.Model(tree, w["kernel"], w["theta_lo"], w["theta_hi"], p_s=w["p_s"],
                      p_theta=w["p_theta"], tol=w["tol"])
    torch.cuda.synchronize()
    log(f"[bench] offline stage {time.time() - t0:.1f} s; tree {tree.info}; model {model.info}")
    thetas = inputs.theta_samples(T, w["theta_lo"], w["theta_hi"], wid)
    x_host = inputs.normal_vectors(n, T * R, wid).T.reshape(T, R, n)
    x = torch.tensor(np.ascontiguousarray(x_host), device="cuda")
    y = torch.empty_like(x)
    inst = api.Instance(model, thetas)
    factored = inst.factored
    stream = torch.cuda.current_stream()

    def step():
        inst.reinstantiate(thetas)
        inst.matvec(x, y)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    lib = _lib.lib()
    # the headline: K steps with tracing off, bracketed by events on the stream every launch
    # of the step uses (the library's default runs the whole step on the caller's stream)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    ms_step = total_ms / args.steps
    # per-kernel durations: a separate pass with an event pair around every launch
    stats = _lib.TraceStats()
    lib.ph_trace_read(stats, 1)
    lib.ph_trace_enable(1)
    trace_steps = max(3, min(args.steps, 10))
    for _ in range(trace_steps):
        step()
    torch.cuda.synchronize()
    lib.ph_trace_enable(0)
    _lib.check(lib.ph_trace_read(stats, 1), "ph_trace_read")
    per_stage = {name: {"ms_total": stats.ms[i], "launches": stats.count[i],
                        "ms_avg": stats.ms[i] / max(stats.count[i], 1)}
                 for i, name in enumerate(_lib.STAGES)}
    inst_ms = sum(per_stage[k]["ms_total"] for k in ("theta", "far_inst", "near_inst")) / trace_steps
    mvm_ms = sum(per_stage[k]["ms_total"] for k in _lib.STAGES[3:]) / trace_steps

    # Roofline of the hot kernels, from algorithmic work per launch (all T slots) and the
    # average launch time measured above with HIP events on the launching stream.
    mi = model.info
    P = mi["P"]
    ncls = tree.info["n_classes"]
    nfar = tree.info["n_far"]
    # near blocks are stored once per pair (s <= t): sum over s <= t of n_s n_t entries
    nd = tree.nodes()
    leaf_sizes = (nd["end"] - nd["begin"])[nd["level"] == tree.info["l_max"]]
    stored = (mi["near_entries"] + float(np.sum(leaf_sizes.astype(np.float64) ** 2))) / 2.0
    if factored:
        kernels = {
            # each stored factor entry P_b[k][e] read once per batch of 8 slots, x read and y
            # written once per slot
            "k_near_fused": ("near_mvm", "hbm", 8.0 * mi["near_factor_entries"] * ((T + 7) // 8)
                             + 8.0 * T * 2.0 * n * R),
            "k_coupling": ("coupling", "mfma", 2.0 * P * P * R * nfar * T),
        }
    else:
        kernels = {
            # each stored factor entry P_b[k][e] read once, each stored block entry written once per slot
            "k_near_instantiate": ("near_inst", "hbm", 8.0 * mi["near_factor_entries"] + 8.0 * T * stored),
            # each stored block entry read once per slot (it serves D_st and D_ts), x and y once
            "k_near_mvm": ("near_mvm", "hbm", 8.0 * T * (stored + 2.0 * n * R)),
            # y_hat_s += C x_hat_t for every far block: 2 P^2 R flops per block and slot
            "k_coupling": ("coupling", "mfma", 2.0 * P * P * R * nfar * T),
        }
    roof = {}
    for kname, (stage, bound, work) in kernels.items():
        ms = per_stage[stage]["ms_avg"]
        if bound == "hbm":
            ach, peak, unit = work / (ms * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s"
        else:
            ach, peak, unit = work / (ms * 1e-3) / 1e12, FP64_MFMA_PEAK_TFS, "TFLOP/s"
        roof[kname] = {"bound": bound, "kernel": kname, "achieved": ach, "peak": peak, "unit": unit,
                       "frac": ach / peak, "traffic": measured_traffic(kname),
                       "algorithmic_per_launch": work, "avg_launch_ms": ms,
                       "ms_per_step": per_stage[stage]["ms_total"] / trace_steps}
    dominant = max(roof, key=lambda k: roof[k]["ms_per_step"])
    # whole-step algorithmic bytes (near factors once per step, D write + read when the
    # blocks are materialised, couplings, vectors)
    step_bytes = (8.0 * mi["near_factor_entries"] + T * 8.0 * ((0 if factored else 2 * stored)
                  + 2 * ncls * P * P + 4 * n * R + 2 * tree.info["n_nodes"] * P * R))
    legs = {} if args.no_legs else step_legs(model, thetas, x_host, T, R, y, args)
    out = {
        "metric": METRIC,
        "value": ms_step / T,
        "unit": "ms per theta (instantiate + MVM with 16 RHS)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w["name"], "n": n, "d": w["d"], "kernel": w["kernel"],
                   "theta_box": [w["theta_lo"][0], w["theta_hi"][0]], "p_s": w["p_s"],
                   "p_theta": w["p_theta"], "leaf": w["leaf"], "eta2": list(w["eta2"]),
                   "tol": w["tol"], "T": T, "R": R, "l_max": tree.info["l_max"],
                   "near_field": "factored (blocks formed inside the MVM)" if factored else "blocks in memory"},
        "ms_instantiate_per_theta": inst_ms / T,
        "ms_matvec_per_theta": mvm_ms / T,
        "step_algorithmic_GBps": step_bytes / (ms_step * 1e-3) / 1e9,
        "stages": per_stage,
        "roofline": roof[dominant],
        "kernels": roof,
        "legs": legs,
        "model": {"near_entries": mi["near_entries"], "near_factor_entries": mi["near_factor_entries"],
                  "near_rank_mean": mi["near_rank_mean"], "far_rank_mean": mi["far_rank_mean"],
                  "classes": ncls, "far_blocks": tree.info["n_far"], "near_blocks": tree.info["n_near"],
                  "device_bytes": mi["device_bytes"]},
        "paper_context": ">100x online speedup vs H-ACA (56x-309x), Python on Intel Xeon w9-3575X; "
                         "CPU only, different kernels and sizes",
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, X, tree.info["l_max"], thetas, x_host,
                                           args.cpu_sample_leaves)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
