"""bsd_unroll_backward_noalloc (partial gradients in the library's own device
array, no allocation) against bsd_unroll_backward (caller's workspace),
through the C ABI: identical gradients on two calls in a row, the second
with fewer shots; sizes beyond the array are refused."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

import gpu_common as gc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KEY = "bb144_cc_p0.05"


@pytest.fixture(scope="module")
def bsd():
    import paper_2512_07057_amd as m
    m.load()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return m


def _p(t):
    return C.c_void_p(t.data_ptr())


def _forward(lib, code, syn, lam, alpha, K):
    shots, T = syn.shape[0], alpha.numel()
    ck_n, ws_n = C.c_int64(), C.c_int64()
    assert lib.bsd_unroll_sizes(code._h, T, K, shots, C.byref(ck_n), C.byref(ws_n)) == 0
    post = torch.empty((shots, code.n), dtype=lam.dtype, device="cuda")
    ck = torch.empty(max(ck_n.value, 1), dtype=lam.dtype, device="cuda")
    assert lib.bsd_unroll_forward(code._h, lam.element_size(), T, K, shots, _p(syn), _p(lam),
                                  _p(alpha), _p(post), _p(ck), None) == 0
    return post, ck, ws_n.value


def _both(lib, code, syn, lam, alpha, K, gpost):
    shots, T = syn.shape[0], alpha.numel()
    post, ck, ws_n = _forward(lib, code, syn, lam, alpha, K)
    ws = torch.empty(max(ws_n, 1), dtype=lam.dtype, device="cuda")
    gl_ref, ga_ref = torch.empty_like(lam), torch.empty_like(alpha)
    assert lib.bsd_unroll_backward(code._h, lam.element_size(), T, K, shots, _p(syn), _p(lam),
                                   _p(alpha), _p(ck), _p(gpost), _p(gl_ref), _p(ga_ref), _p(ws),
                                   None) == 0
    gl, ga = torch.full_like(lam, 7.0), torch.full_like(alpha, 7.0)
    rc = lib.bsd_unroll_backward_noalloc(code._h, lam.element_size(), T, K, shots, _p(syn),
                                         _p(lam), _p(alpha), _p(ck), _p(gpost), _p(gl), _p(ga),
                                         None)
    assert rc == 0, lib.bsd_last_error()
    torch.cuda.synchronize()
    return (gl_ref.cpu().numpy(), ga_ref.cpu().numpy()), (gl.cpu().numpy(), ga.cpu().numpy())


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_backward_equals_workspace_backward(bsd, dtype):
    lib = bsd.load()
    pr = gc.problem(KEY)
    code = bsd.Code.from_problem(pr)
    d = gc.samples("W1", 4000, seed=81)
    rng = np.random.default_rng(3)
    lam = torch.tensor(np.log((1 - pr.p) / pr.p) * rng.uniform(0.8, 1.2, pr.n), dtype=dtype,
                       device="cuda")
    alpha = torch.tensor(rng.uniform(0.5, 0.9, 25), dtype=dtype, device="cuda")
    syn_all = torch.from_numpy(np.ascontiguousarray(d["syndromes"])).cuda()
    # two calls in a row, the second smaller; the array keeps the first's contents
    for shots in (4000 if dtype == torch.float32 else 3000, 700):
        syn = syn_all[:shots].contiguous()
        gpost = torch.tensor(rng.standard_normal((shots, pr.n)), dtype=dtype, device="cuda")
        gc.log("no-alloc backward", dtype, shots)
        ref, got = _both(lib, code, syn, lam, alpha, 5, gpost)
        np.testing.assert_array_equal(got[0], ref[0])
        np.testing.assert_array_equal(got[1], ref[1])
        assert np.abs(ref[0]).max() > 0
    # beyond the array: refused with its limit
    big = 8 * 2 ** 20 // ((pr.n + 25) * lam.element_size()) + 1
    syn = syn_all[:1].expand(big, pr.m).contiguous()
    gl, ga = torch.empty_like(lam), torch.empty_like(alpha)
    rc = lib.bsd_unroll_backward_noalloc(code._h, lam.element_size(), 25, 5, big, _p(syn), _p(lam),
                                         _p(alpha), _p(syn), _p(syn), _p(gl), _p(ga), None)
    assert rc == bsd.BSD_EINVAL
    assert b"limit" in lib.bsd_last_error()
