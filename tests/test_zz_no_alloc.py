"""ibm_classify_noalloc through the C ABI (needs an MI355X).

The entry point that allocates no device memory must classify exactly like
ibm_classify (bit-exact flags, same counts) on consecutive calls that share
its fixed per-device scratch -- the second smaller than the first, then one
with both body kinds -- and must refuse an input whose scratch exceeds the
fixed size without touching the device.
"""
import numpy as np
import pytest

from paper_2605_04335_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_04335_amd as P
    return P


def _cases():
    mem = W.membrane_case(64, nc=40, ns=120)
    small = W.sphere_case(32)
    mixed = W.Problem("mixed_40", W.uniform_faces(40), W.uniform_faces(40), W.uniform_faces(40),
                      [W.sphere((0.3, 0.3, 0.5), 0.15), W.plate((0.7, 0.6, 0.5), 0.2, 0.5, 20, 50, 0.03, 0.4)])
    return [("membrane_64", mem), ("sphere_32", small), ("sphere_plate_40", mixed)]


def test_noalloc_classify_equals_classify(P):
    import torch
    prev = None
    for name, p in _cases():
        say("noalloc", name, p.shape)
        ref, cref = P.classify(p.xf, p.yf, p.zf, p.bodies)
        # the output buffer is poisoned: every cell must be written
        out = torch.full((p.npts,), 0xA5, dtype=torch.uint8, device="cuda")
        got, cgot, need = P.classify_noalloc(p.xf, p.yf, p.zf, p.bodies, out)
        torch.cuda.synchronize()
        assert 0 < need <= P.CLASSIFY_NOALLOC_MAX_BYTES
        assert torch.equal(got, ref), "cells differ: %d" % int((got != ref).sum())
        assert cgot == cref
        if prev is not None and name == "sphere_32":
            assert p.npts < prev  # the second call is the smaller input
        prev = p.npts


def test_noalloc_refuses_oversize_input(P):
    import torch
    p = W.membrane_case(640, rhs=False)  # 262M cells with a membrane: ~100 MB of scratch
    tiny = torch.zeros(16, dtype=torch.uint8, device="cuda")
    G = P._GridArgs(p.xf, p.yf, p.zf)
    B = P._BodyArgs(p.bodies)
    st = P._ClassStats()
    need = P.ctypes.c_size_t()
    rc = P.lib().ibm_classify_noalloc(P.ctypes.byref(G.g), B.arr, P.ctypes.c_int32(B.n), P._tptr(tiny),
                                      P.ctypes.byref(st), P.ctypes.byref(need), P._stream())
    assert rc == P.IBM_ENOMEM
    assert need.value > P.CLASSIFY_NOALLOC_MAX_BYTES
    assert b"scratch" in P.lib().ibm_last_error()
    torch.cuda.synchronize()
    assert int(tiny.sum()) == 0  # nothing was enqueued
    # the entry point still works after the refusal
    q = W.sphere_case(32)
    ref, _ = P.classify(q.xf, q.yf, q.zf, q.bodies)
    got, _, _ = P.classify_noalloc(q.xf, q.yf, q.zf, q.bodies)
    assert torch.equal(got, ref)
