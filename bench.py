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
# source files whose text determines each hot kernel's code
KERNEL_SOURCES = {
    "k_coupling": ["k_matvec.hip", "ph_device.hpp"],
    "k_near_mvm": ["k_matvec.hip", "ph_device.hpp"],
    "k_near_instantiate": ["k_instantiate.hip", "ph_device.hpp"],
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(kernel):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
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
    return {
        "value": float(np.mean(est)) * 1e3, "unit": "ms per theta (instantiate + MVM, 16 RHS), extrapolated",
        "cores": int(threads), "kind": "oracle",
        "sample": f"{sample_leaves} of {nleaf} target leaves ({len(rows)} rows, {len(near)} near blocks) for "
                  f"each of {len(thetas)} theta, all {len(all_keys)} far couplings, full upward pass; "
                  f"per-leaf work scaled by {scale:.0f}x; measured {measured:.1f} s of oracle work",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-leaves", type=int, default=160)
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
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(multi-GPU sharding is described in the design notes, not built)"}))
        sys.exit(2)

    import torch

    from oracle import tree as otree  # noqa: F401  (only for l_max derivation parity)
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
    stream = torch.cuda.current_stream()

    def step():
        inst.reinstantiate(thetas)
        inst.matvec(x, y)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    lib = _lib.lib()
    stats = _lib.TraceStats()
    lib.ph_trace_read(stats, 1)
    lib.ph_trace_enable(1)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    lib.ph_trace_enable(0)
    _lib.check(lib.ph_trace_read(stats, 1), "ph_trace_read")
    total_ms = ev0.elapsed_time(ev1)
    ms_step = total_ms / args.steps
    per_stage = {name: {"ms_total": stats.ms[i], "launches": stats.count[i],
                        "ms_avg": stats.ms[i] / max(stats.count[i], 1)}
                 for i, name in enumerate(_lib.STAGES)}
    inst_ms = sum(per_stage[k]["ms_total"] for k in ("theta", "far_inst", "near_inst")) / args.steps
    mvm_ms = sum(per_stage[k]["ms_total"] for k in _lib.STAGES[3:]) / args.steps  # sum of kernel times (streams overlap)

    # Roofline of the hot kernels, from algorithmic work per launch (all T slots) and the
    # average launch time measured above with HIP events on the launching stream.
    mi = model.info
    P = mi["P"]
    ncls = tree.info["n_classes"]
    nfar = tree.info["n_far"]
    kernels = {
        # each stored factor entry P_b[k][e] read once, each near-block entry written once per slot
        "k_near_instantiate": ("near_inst", "hbm", 8.0 * mi["near_factor_entries"] + 8.0 * T * mi["near_entries"]),
        # D read once, x and y once per slot
        "k_near_mvm": ("near_mvm", "hbm", 8.0 * T * (mi["near_entries"] + 2.0 * n * R)),
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
                       "ms_per_step": per_stage[stage]["ms_total"] / args.steps}
    dominant = max(roof, key=lambda k: roof[k]["ms_per_step"])
    # whole-step algorithmic bytes per theta (near factors once per step, D write + read,
    # couplings, vectors)
    step_bytes = (8.0 * mi["near_factor_entries"] + T * 8.0 * (2 * mi["near_entries"]
                  + 2 * ncls * P * P + 4 * n * R + 2 * tree.info["n_nodes"] * P * R))
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
                   "tol": w["tol"], "T": T, "R": R, "l_max": tree.info["l_max"]},
        "ms_instantiate_per_theta": inst_ms / T,
        "ms_matvec_per_theta": mvm_ms / T,
        "step_algorithmic_GBps": step_bytes / (ms_step * 1e-3) / 1e9,
        "stages": per_stage,
        "roofline": roof[dominant],
        "kernels": roof,
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
