"""The allocation-free MVM entry point (ph_matvec_noalloc) against ph_matvec, through the
C ABI: two calls in a row on one GPU, the second with a smaller input, each bit-identical to
ph_matvec on the same instance (same kernels and launch configuration, scratch taken from
the library's fixed per-GPU array instead of the instance), and a request larger than that
array rejected with PH_EINVAL before anything is launched."""

import ctypes as C

import numpy as np
import pytest

from paper_2511_03109_amd import inputs

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _noalloc(inst, x, y, R, alpha=1.0, beta=0.0, nugget=0.0):
    from paper_2511_03109_amd import _lib
    return _lib.lib().ph_matvec_noalloc(inst._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), R, alpha,
                                        beta, nugget, None)


def test_noalloc_matches_matvec_then_smaller_call():
    torch = _torch()
    from paper_2511_03109_amd import _lib, api
    n = 3000
    X = inputs.points_for(2, n)
    tree = api.Tree(X, l_max=2, eta2=(3, 1))
    model = api.Model(tree, "matern32", [0.05], [0.5], p_s=5, p_theta=9, tol=1e-8)
    # first call: 4 slots (factored near field), 16 right-hand sides, alpha / beta / nugget
    th4 = inputs.theta_samples(4, [0.05], [0.5], 9)
    big = api.Instance(model, th4)
    x = torch.tensor(np.ascontiguousarray(inputs.normal_vectors(n, 4 * 16, 91).T.reshape(4, 16, n)), device="cuda")
    y0 = torch.tensor(np.ascontiguousarray(inputs.normal_vectors(n, 4 * 16, 92).T.reshape(4, 16, n)), device="cuda")
    ref = y0.clone()
    big.matvec(x, ref, alpha=0.5, beta=2.0, nugget=0.01)
    got = y0.clone()
    torch.cuda.synchronize()
    _lib.check(_noalloc(big, x, got, 16, 0.5, 2.0, 0.01), "ph_matvec_noalloc")
    torch.cuda.synchronize()
    print(f"[no-alloc] call 1: T = 4, R = 16, max |diff| {float((got - ref).abs().max()):.3e}", flush=True)
    assert torch.equal(got, ref)
    # second call: a smaller input on the same array (one slot, near blocks in memory, R = 3)
    small = api.Instance(model, [0.2])
    xs = torch.tensor(np.ascontiguousarray(inputs.normal_vectors(n, 3, 93).T), device="cuda")
    ref2 = small.matvec(xs)
    got2 = torch.full_like(xs, float("nan"))
    torch.cuda.synchronize()
    _lib.check(_noalloc(small, xs, got2, 3), "ph_matvec_noalloc")
    torch.cuda.synchronize()
    print(f"[no-alloc] call 2: T = 1, R = 3, max |diff| {float((got2 - ref2).abs().max()):.3e}", flush=True)
    assert torch.equal(got2, ref2)
    # the first instance again after the smaller call (the array keeps the last contents)
    got3 = y0.clone()
    _lib.check(_noalloc(big, x, got3, 16, 0.5, 2.0, 0.01), "ph_matvec_noalloc")
    torch.cuda.synchronize()
    assert torch.equal(got3, ref)


def test_noalloc_rejects_requests_beyond_its_scratch():
    torch = _torch()
    from paper_2511_03109_amd import _lib, api
    n = 3000
    X = inputs.points_for(2, n)
    tree = api.Tree(X, l_max=2, eta2=(3, 1))
    model = api.Model(tree, "matern32", [0.05], [0.5], p_s=5, p_theta=9, tol=1e-8)
    inst = api.Instance(model, [0.3])
    R = 1500   # x and y in tree order alone need 2 x 3000 x 1504 x 8 B = 72 MB
    x = torch.zeros(R, n, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    code = _noalloc(inst, x, y, R)
    msg = _lib.lib().ph_last_error().decode()
    print(f"[no-alloc] oversized request: status {code}: {msg}", flush=True)
    assert code == _lib.PH_EINVAL
    assert "scratch" in msg
