"""gcp_prepare: after it, bound and optimisation calls of the prepared shapes
allocate no device memory and never wait for the device, so they can be
captured into a HIP graph (through torch's graph capture).  Checked through
the C ABI: device free memory is unchanged over repeated calls, and every
replay of a captured gcp_optimize equals the eager call bit for bit (the
parameters are reset by eager copies between the replays).
"""
import numpy as np
import pytest

from workloads import gen

pytestmark = pytest.mark.gpu


def _dev():
    import torch
    return torch.device("cuda:0")


def _setup(which, mode):
    import torch
    from oracle import gcp_oracle as O
    from paper_2208_05740_amd import binding as B
    prob = gen.make_workload("mlp784", 0, B=64) if which == "mlp784" else \
        gen.make_tiny("cnn16", 4, B=6, splits=(1, 3), n_cuts=5, input_terms=1)
    P = B.Problem(prob, device=_dev())
    M = P.M
    t = lambda x: torch.tensor(np.asarray(x, np.float32).reshape(M, -1), device=_dev())  # noqa: E731
    a0, b0, c0 = t(O.full_alpha(prob)), t(prob.beta), t(prob.gamma)
    B.prepare(P.net, P.S, P.splits, P.cuts, iters=prob.opt["iters"], mode=mode)
    return prob, P, a0, b0, c0


@pytest.mark.parametrize("which,mode", [("mlp784", 0), ("mlp784", 1), ("cnn", 0)])
def test_prepared_calls_allocate_nothing(which, mode):
    import torch
    from paper_2208_05740_amd import binding as B
    print(f"prepare, then calls: {which} mode={mode}", flush=True)
    prob, P, a0, b0, c0 = _setup(which, mode)
    o = prob.opt
    a, b, c = a0.clone(), b0.clone(), c0.clone()
    st = torch.zeros(B.adam_state_size(P.M, P.n_I, P.K, P.N), dtype=torch.float32, device=_dev())
    out = torch.empty(P.M, dtype=torch.float64, device=_dev())
    ver = torch.empty(P.M, dtype=torch.uint8, device=_dev())
    ga, gb, gc = torch.empty_like(a), torch.empty_like(b), torch.empty_like(c)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        a.copy_(a0); b.copy_(b0); c.copy_(c0); st.zero_()
        B.optimize(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a, b, c, st, iters=o["iters"], lr_alpha=o["lr_alpha"],
                   lr_mult=o["lr_mult"], decay=o["decay"], mode=mode, bound_out=out, verified_out=ver)
        B.lib().gcp_bound(P.net.h, B._ptr(P.x0), float(P.eps), B._ptr(P.C), P.S, P.splits.h,
                          P.cuts.h if P.cuts else None, B._ptr(a), B._ptr(b) if b.numel() else None,
                          B._ptr(c) if c.numel() else None, mode, B._ptr(out), B._ptr(ver), B._ptr(ga),
                          B._ptr(gb) if gb.numel() else None, B._ptr(gc) if gc.numel() else None, B._stream())
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0


@pytest.mark.parametrize("which,mode", [("mlp784", 0), ("mlp784", 1), ("cnn", 1)])
def test_prepared_optimize_replays_from_a_captured_graph(which, mode):
    import torch
    from paper_2208_05740_amd import binding as B
    print(f"prepare, capture, replay: {which} mode={mode}", flush=True)
    prob, P, a0, b0, c0 = _setup(which, mode)
    o = prob.opt
    a, b, c = a0.clone(), b0.clone(), c0.clone()
    st = torch.zeros(B.adam_state_size(P.M, P.n_I, P.K, P.N), dtype=torch.float32, device=_dev())
    out = torch.empty(P.M, dtype=torch.float64, device=_dev())
    ver = torch.empty(P.M, dtype=torch.uint8, device=_dev())

    def reset():
        a.copy_(a0); b.copy_(b0); c.copy_(c0); st.zero_()

    def call():
        B.optimize(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a, b, c, st, iters=o["iters"], lr_alpha=o["lr_alpha"],
                   lr_mult=o["lr_mult"], decay=o["decay"], mode=mode, bound_out=out, verified_out=ver)

    reset()
    call()
    torch.cuda.synchronize()
    ref = [x.cpu().numpy().copy() for x in (out, ver, a, b, c, st)]
    reset()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        call()
    for rep in range(3):
        reset()
        graph.replay()
        torch.cuda.synchronize()
        got = [x.cpu().numpy() for x in (out, ver, a, b, c, st)]
        for x, y in zip(got, ref):
            assert np.array_equal(x, y), rep
        # eager work between the replays
        reset()
        call()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref[0])
