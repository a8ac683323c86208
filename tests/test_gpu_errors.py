"""Error paths of the C ABI, called through ctypes on the GPU: every argument
check returns its status code (KMX_EINVAL = 1, KMX_EUNSUPPORTED = 4) with a
message, before any work is enqueued, and leaves the outputs untouched.  The
data checks (weights finite and >= 0, k at most the number of positive
weights, and the opt-in scan for values that are not finite) run kernels of
their own; no test here hands a kernel data it cannot take."""
import ctypes
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

EINVAL, EUNSUPPORTED = 1, 4


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_04265_amd import kmx
    rng = np.random.default_rng(0)
    X = torch.from_numpy(rng.normal(size=(500, 8)).astype(np.float32)).cuda()
    return kmx, kmx.Context(0), X


def _status(kmx, fn, *a, **kw):
    with pytest.raises(kmx.KmxError) as e:
        fn(*a, **kw)
    assert len(str(e.value)) > len("kmx status 1: ")
    return e.value.status, str(e.value)


def test_seed_weight_checks(env):
    import torch
    kmx, ctx, X = env
    w = torch.ones(500, device="cuda")
    w[:497] = 0.0                                  # three positive weights
    C, idx = ctx.seed(X, 3, w=w, rng_seed=1)       # all three are drawn
    assert sorted(idx.cpu().tolist()) == [497, 498, 499]
    st, msg = _status(kmx, ctx.seed, X, 4, w=w)
    assert st == EINVAL and "positive weight" in msg
    for bad in (-1.0, float("nan"), float("inf")):
        w2 = torch.ones(500, device="cuda")
        w2[123] = bad
        st, msg = _status(kmx, ctx.seed, X, 2, w=w2)
        assert st == EINVAL and "negative or not finite" in msg
    st, _ = _status(kmx, ctx.seed, X, 0)
    assert st == EINVAL
    st, _ = _status(kmx, ctx.seed, X, 501)
    assert st == EINVAL


def test_weight_checks_of_the_other_calls(env):
    import torch
    kmx, ctx, X = env
    C = X[:5].contiguous()
    w = torch.ones(500, device="cuda")
    w[7] = -0.5
    for fn, args in ((ctx.lloyd, (X, C, 2)), (ctx.cost, (X, C))):
        st, msg = _status(kmx, fn, *args, w=w)
        assert st == EINVAL and "negative or not finite" in msg
    st, msg = _status(kmx, ctx.lloyd, X, C, 2, w=w, graph=True)
    assert st == EINVAL
    st, msg = _status(kmx, ctx.lloyd_routed, X, C, 2, w=w)
    assert st == EINVAL
    st, msg = _status(kmx, ctx.lloyd_batched, [{"X": X, "C": C}, {"X": X, "C": C, "w": w}], 2)
    assert st == EINVAL and "problem 1" in msg
    # zero weights are valid for Lloyd (empty clusters keep their centers)
    w0 = torch.zeros(500, device="cuda")
    w0[:10] = 1.0
    C2, lab, hist, it = ctx.lloyd(X, C, 2, w=w0, prec="fp32")
    assert it == 2 and np.isfinite(hist).all()


def test_shape_and_argument_checks(env):
    import torch
    kmx, ctx, X = env
    L = kmx.lib()
    p = ctx._p
    C = X[:5].contiguous()
    lab = torch.full((500,), -3, dtype=torch.int32, device="cuda")
    vp = ctypes.c_void_p
    Xp, Cp, lp = vp(X.data_ptr()), vp(C.data_ptr()), vp(lab.data_ptr())

    def code(st, *needle):
        assert st != 0
        msg = L.kmx_last_error(p).decode()
        for s in needle:
            assert s in msg, msg
        return st

    assert code(L.kmx_assign(p, None, 500, 8, 8, Cp, 5, 0, lp, None, None, None), "X") == EINVAL
    assert code(L.kmx_assign(p, Xp, 0, 8, 8, Cp, 5, 0, lp, None, None, None), "n") == EINVAL
    assert code(L.kmx_assign(p, Xp, 500, 0, 8, Cp, 5, 0, lp, None, None, None), "d") == EINVAL
    assert code(L.kmx_assign(p, Xp, 500, 8, 7, Cp, 5, 0, lp, None, None, None), "ldx") == EINVAL
    assert code(L.kmx_assign(p, Xp, 500, 8, 8, Cp, 0, 0, lp, None, None, None), "k") == EINVAL
    assert code(L.kmx_assign(p, Xp, 500, 8, 8, Cp, 501, 0, lp, None, None, None), "k") == EINVAL
    assert code(L.kmx_assign(p, Xp, 500, 8, 8, Cp, 5, 7, lp, None, None, None),
                "precision") == EINVAL
    assert code(L.kmx_assign(p, Xp, 500, 8, 8, None, 5, 0, lp, None, None, None), "C") == EINVAL
    assert code(L.kmx_assign(p, Xp, 500, 8, 8, Cp, 5, 0, None, None, None, None),
                "label") == EINVAL
    hist = (ctypes.c_double * 4)()
    it = ctypes.c_int32(0)
    assert code(L.kmx_lloyd(p, Xp, 500, 8, 8, None, Cp, 5, -1, -1.0, 0, lp, hist,
                            ctypes.byref(it)), "max_iter") == EINVAL
    assert code(L.kmx_lloyd(p, Xp, 500, 8, 8, None, Cp, 5, 3, -1.0, 0, lp, None,
                            ctypes.byref(it)), "cost_hist") == EINVAL
    assert code(L.kmx_update(p, Xp, 500, 8, 8, None, None, 5, Cp, Cp, None, None),
                "label") == EINVAL
    cost = ctypes.c_double(0)
    assert code(L.kmx_cost(p, Xp, 500, 8, 8, None, Cp, 5, 0, None), "cost_out") == EINVAL
    # unsupported requests
    Y = torch.empty((500, 32), device="cuda")
    V = torch.empty((8, 20), device="cuda")
    assert code(L.kmx_project(p, Xp, 500, 8, 8, vp(V.data_ptr()), 20, vp(Y.data_ptr()), 32),
                "d_out") == EUNSUPPORTED
    arr = (kmx.Problem * 1)()
    arr[0] = kmx.Problem(X.data_ptr(), 500, 8, 8, None, C.data_ptr(), 5, None)
    h2 = (ctypes.c_double * 3)()
    assert code(L.kmx_lloyd_batched(p, arr, 1, 2, 0, h2), "BF16") == EUNSUPPORTED
    arr[0] = kmx.Problem(X.data_ptr(), 500, 8, 8, None, C.data_ptr(), 501, None)
    assert code(L.kmx_lloyd_batched(p, arr, 1, 2, 1, h2), "problem 0") == EINVAL
    assert code(L.kmx_lloyd_batched(p, arr, 0, 2, 1, h2), "no problems") == EINVAL
    torch.cuda.synchronize()
    assert (lab == -3).all()          # nothing was written by a refused call
    # the context still works after the refusals
    lab2, _, _, _ = ctx.assign(X, C, prec="fp32")
    assert int(lab2.min()) >= 0 and int(lab2.max()) < 5


def test_router_argument_checks(env):
    import torch
    kmx, ctx, X = env
    st, msg = _status(kmx, ctx.router, 8, 5000)
    assert st == EUNSUPPORTED
    r = ctx.router(8, 5)
    C = X[:6].contiguous()
    st, msg = _status(kmx, ctx.lloyd_routed, X, C, 2, router=r)
    assert st == EINVAL and "router shape" in msg


def test_validate_scan_rejects_non_finite_inputs(env):
    import torch
    kmx, _, X = env
    os.environ["KMX_VALIDATE"] = "1"
    try:
        vctx = kmx.Context(0)
    finally:
        del os.environ["KMX_VALIDATE"]
    Xb = X.clone()
    Xb[17, 3] = float("nan")
    Xb[400, 0] = float("-inf")
    C = X[:5].contiguous()
    for fn, args in ((vctx.assign, (Xb, C)), (vctx.cost, (Xb, C)), (vctx.lloyd, (Xb, C, 2)),
                     (vctx.seed, (Xb, 3))):
        st, msg = _status(kmx, fn, *args)
        assert st == EINVAL and "X holds 2 entries" in msg
    Cb = C.clone()
    Cb[2, 2] = float("inf")
    st, msg = _status(kmx, vctx.assign, X, Cb)
    assert st == EINVAL and "centers" in msg
    # finite inputs pass the scan and give the same labels as without it
    lab_v, _, _, _ = vctx.assign(X, C, prec="bf16")
    lab_p, _, _, _ = env[1].assign(X, C, prec="bf16")
    assert torch.equal(lab_v, lab_p)
    vctx.close()
