"""gcp_bound_noalloc (workspace in the library's static device array, no
allocation inside the call) against gcp_bound, through the C ABI.

Two calls in a row, the second with fewer rows, then the first size again:
bounds, verified flags and gradients must equal gcp_bound's (the same
kernels on the same inputs; tolerance of the fp32 path, 1e-5 relative,
and in fact bit for bit), device free memory must not change across the
calls, and a call whose workspace exceeds the array fails cleanly.
"""
import numpy as np
import pytest

from workloads import gen

pytestmark = pytest.mark.gpu


def _dev():
    import torch
    return torch.device("cuda:0")


def _inputs(prob, P, seed):
    import torch
    from oracle import gcp_oracle as O
    rng = np.random.default_rng(seed)
    prep = O.Prepared(prob)
    a = rng.random((P.M, prep.n_I)).astype(np.float32)
    b = np.asarray(prob.beta, np.float32).reshape(P.M, -1)
    c = (rng.random((P.M, P.N)) * 0.1).astype(np.float32)
    t = lambda x: torch.tensor(x, device=_dev())  # noqa: E731
    return t(a), t(b), t(c)


def _pair(prob, P, a, b, c, mode, grads):
    """(gcp_bound results, gcp_bound_noalloc results) as numpy arrays."""
    import torch
    from paper_2208_05740_amd import binding as B
    ref, ver_ref, g_ref = B.bound(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a, b, c, mode=mode, grads=grads,
                                  verified=True)
    out = torch.empty(P.M, dtype=torch.float64, device=_dev())
    ver = torch.empty(P.M, dtype=torch.uint8, device=_dev())
    g = (torch.empty_like(a), torch.empty_like(b), torch.empty_like(c)) if grads else None
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    B.bound_noalloc(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a, b, c, out, ver, g, mode=mode)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    n = lambda t: t.cpu().numpy()  # noqa: E731
    return ((n(ref), n(ver_ref), [n(x) for x in g_ref] if grads else None),
            (n(out), n(ver), [n(x) for x in g] if grads else None), free0, free1)


def _check(r, s, tol):
    assert np.all(np.abs(s[0] - r[0]) <= tol * np.abs(r[0]))
    assert np.array_equal(s[0], r[0])
    assert np.array_equal(s[1], r[1])
    if r[2] is not None:
        for x, y in zip(s[2], r[2]):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("name,mode", [("mlp784", 0), ("mlp784", 1), ("cnn", 0)])
def test_noalloc_equals_gcp_bound_on_two_calls(name, mode):
    from paper_2208_05740_amd import binding as B
    print(f"no-alloc vs gcp_bound: {name} mode={mode}", flush=True)
    big = gen.make_workload(name, 0, B=5)
    small = gen.make_workload(name, 0, B=3)
    Pb = B.Problem(big, device=_dev())
    Ps = B.Problem(small, device=_dev())
    ab, bb, cb = _inputs(big, Pb, 1)
    as_, bs, cs = _inputs(small, Ps, 2)
    # first use on the device (looks up the array), then the two calls of the test
    _pair(big, Pb, ab, bb, cb, mode, True)
    frees = []
    for prob, P, a, b, c, grads in ((big, Pb, ab, bb, cb, True), (small, Ps, as_, bs, cs, True),
                                    (small, Ps, as_, bs, cs, False)):
        r, s, f0, f1 = _pair(prob, P, a, b, c, mode, grads)
        _check(r, s, 1e-5)
        frees.append((f0, f1))
    for f0, f1 in frees:
        assert f0 == f1, frees


def test_noalloc_rejects_a_workspace_beyond_the_array():
    import torch
    from paper_2208_05740_amd import binding as B
    print("no-alloc size limit", flush=True)
    prob = gen.make_workload("mlp784", 0, B=1024)
    P = B.Problem(prob, device=_dev())
    a, b, c = _inputs(prob, P, 3)
    out = torch.empty(P.M, dtype=torch.float64, device=_dev())
    g = (torch.empty_like(a), torch.empty_like(b), torch.empty_like(c))
    with pytest.raises(B.GcpError) as ei:
        B.bound_noalloc(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a, b, c, out, None, g)
    assert ei.value.code == -4 and "static workspace" in str(ei.value)
    # the handles and the entry point still work afterwards
    small = gen.make_workload("mlp784", 0, B=2)
    Ps = B.Problem(small, device=_dev())
    r, s, _, _ = _pair(small, Ps, *_inputs(small, Ps, 4), 0, True)
    _check(r, s, 1e-5)
