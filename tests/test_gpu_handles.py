"""Handle lifetime and argument-set caching, through the C ABI.

* A captured optimisation iteration is cached per argument set; a split or
  cut handle re-created after the old one was destroyed (possibly at the
  same host address) must not replay a graph that points at the old one.
* The grouped-launch plan of gcp_optimize_batch must not be reused when the
  optimiser settings change.
* Cut coefficients that are not fp32 values: the library stores fp32
  coefficients and widens the cut's offset by |fp32(c) - c| times the
  largest magnitude the variable takes under the root bounds, so the cut it
  applies still holds (the offset enters the bound as -gamma.d, Theorem 3.1).
"""
import copy

import numpy as np
import pytest

from workloads import gen

pytestmark = pytest.mark.gpu


def _dev():
    import torch
    return torch.device("cuda:0")


def _start(prob, P):
    import torch
    from oracle import gcp_oracle as O
    t = lambda x: torch.tensor(np.asarray(x, np.float32).reshape(P.M, -1), device=_dev())  # noqa: E731
    return t(O.full_alpha(prob)), t(prob.beta), t(prob.gamma)


def _opt(P, prob, a0, b0, c0, graph, lr_alpha=None, mode=0):
    import torch
    from paper_2208_05740_amd import binding as B
    a, b, c = a0.clone(), b0.clone(), c0.clone()
    st = torch.zeros(B.adam_state_size(P.M, P.n_I, P.K, P.N), dtype=torch.float32, device=_dev())
    o = prob.opt
    out, _ = B.optimize(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a, b, c, st, iters=o["iters"],
                        lr_alpha=o["lr_alpha"] if lr_alpha is None else lr_alpha, lr_mult=o["lr_mult"],
                        decay=o["decay"], use_graph=graph, mode=mode)
    torch.cuda.synchronize()
    return out.cpu().numpy(), a.cpu().numpy(), c.cpu().numpy()


def test_graph_replay_after_recreating_splits_and_cuts():
    from paper_2208_05740_amd import binding as B
    print("graph replay after re-created handles", flush=True)
    p = gen.make_tiny("mlp", 2, B=6, splits=(1, 3), n_cuts=5)
    P = B.Problem(p, device=_dev())
    a0, b0, c0 = _start(p, P)
    _opt(P, p, a0, b0, c0, graph=True)          # captures a graph for the first handles
    for rep in range(3):
        # same B and K, other split sides and cut offsets: new handles,
        # created right after the old ones were destroyed
        p.splits.sign = np.where(p.splits.node >= 0, -p.splits.sign, p.splits.sign).astype(p.splits.sign.dtype)
        p.cuts.d = p.cuts.d + 0.25
        P.splits = None
        P.splits = B.Splits(P.net, p.splits)
        P.cuts = None
        P.cuts = B.Cuts(P.net, p.cuts)
        got = _opt(P, p, a0, b0, c0, graph=True)
        ref = _opt(P, p, a0, b0, c0, graph=False)
        for x, y in zip(got, ref):
            assert np.array_equal(x, y), rep


def test_batch_plan_follows_optimiser_settings():
    import torch
    from paper_2208_05740_amd import binding as B
    print("batch plan with changed optimiser settings", flush=True)
    probs = gen.make_batch(seed=5, n_inst=3, bmax=24)
    Ps = [B.Problem(p, device=_dev()) for p in probs]
    o = probs[0].opt
    for lr in (o["lr_alpha"], 0.03, o["lr_alpha"]):
        items, ref = [], []
        for p, P in zip(probs, Ps):
            a0, b0, c0 = _start(p, P)
            ref.append(_opt(P, p, a0, b0, c0, graph=False, lr_alpha=lr))
            items.append(dict(P=P, alpha=a0.clone(), beta=b0.clone(), gamma=c0.clone(),
                              state=torch.zeros(B.adam_state_size(P.M, P.n_I, P.K, P.N), dtype=torch.float32,
                                                device=_dev()),
                              bound=torch.empty(P.M, dtype=torch.float64, device=_dev()),
                              verified=torch.empty(P.M, dtype=torch.uint8, device=_dev())))
        B.optimize_batch(items, iters=o["iters"], lr_alpha=lr, lr_mult=o["lr_mult"], decay=o["decay"], use_graph=True)
        torch.cuda.synchronize()
        for it, (g, a, c) in zip(items, ref):
            assert np.array_equal(it["bound"].cpu().numpy(), g), lr
            assert np.array_equal(it["alpha"].cpu().numpy(), a), lr


def test_cut_coefficients_off_fp32_widen_the_offset():
    import torch
    from paper_2208_05740_amd import binding as B
    print("cut coefficients that are not fp32 values", flush=True)
    p = gen.make_tiny("mlp", 4, B=3, splits=(1, 2), n_cuts=6, input_terms=0)
    P = B.Problem(p, device=_dev())
    a, b, c = _start(p, P)
    c = torch.rand(c.shape, generator=torch.Generator(device=_dev()).manual_seed(3), device=_dev())
    ref, _, _ = B.bound(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a, b, c)
    q = copy.deepcopy(p)
    cu = q.cuts
    node_entry = cu.node >= 0
    assert node_entry.any()
    # a relative nudge far below half an fp32 ulp: fp32(coef') == coef
    cu.coef = np.where(node_entry, cu.coef * (1.0 + 2.0 ** -30), cu.coef)
    assert np.all(cu.coef.astype(np.float32).astype(np.float64) == p.cuts.coef)
    Cq = B.Cuts(P.net, cu)
    got, _, _ = B.bound(P.net, P.x0, P.eps, P.C, P.splits, Cq, a, b, c)
    torch.cuda.synchronize()
    # expected widening per cut: sum over its entries of |fp32(c) - c| times
    # max|x| = max(|l|, |u|) (H), max(u, 0) (G) or 1 (Q)
    slack = np.zeros(cu.n)
    for e in np.nonzero(node_entry)[0]:
        k, nd, j, kd = int(cu.cut[e]), int(cu.node[e]), int(cu.neuron[e]), int(cu.kind[e])
        l, u = p.lu[[i for i, n in enumerate(p.net.nodes) if n.relu].index(nd)]
        rng = max(abs(l[j]), abs(u[j])) if kd == 0 else (max(u[j], 0.0) if kd == 1 else 1.0)
        slack[k] += abs(cu.coef[e] - p.cuts.coef[e]) * rng
    assert slack.max() > 0
    shift = c.cpu().numpy().astype(np.float64) @ slack      # the bound moves down by gamma.(d' - d)
    assert shift.min() > 1e-10
    d = got.cpu().numpy() - (ref.cpu().numpy() - shift)
    # d' is rounded up by one ulp of d, and the two fp64 row sums round apart
    assert np.all(np.abs(d) <= 1e-12), (d, shift)
    # input-variable coefficients have no range before the call: rejected
    r = copy.deepcopy(p)
    r.cuts.node[0] = -1
    r.cuts.kind[0] = 1
    r.cuts.neuron[0] = 0
    r.cuts.coef[0] = 0.1
    with pytest.raises(B.GcpError) as ei:
        B.Cuts(P.net, r.cuts)
    assert ei.value.code == -1
