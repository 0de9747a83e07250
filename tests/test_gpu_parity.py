"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances:
  * FP32 path: |g_gpu - g_oracle| <= 1e-5 * max(|g|, T), T = the sum of the
    magnitudes of every term added into the bound (the oracle's
    error_scale); the fp32 GEMMs round each product with unit 6e-8 and the
    sums are fp64, so the error is a small multiple of that scale.
  * gradients: |d_gpu - d_oracle| <= 1e-4 * (max_row |d_oracle| + 1).
  * BF16 path: bf16 operands carry 8 mantissa bits (unit 4e-3); the bound
    error is checked at 2e-2 of T.
"""
import copy

import numpy as np
import pytest

from oracle import gcp_oracle as O
from oracle import lp
from workloads import gen

pytestmark = pytest.mark.gpu


def _dev():
    import torch
    return torch.device("cuda:0")


def upload(prob):
    from paper_2208_05740_amd import binding as B
    return B.Problem(prob, device=_dev())


def params(prob, P, alpha=None, beta=None, gamma=None):
    import torch
    a = O.full_alpha(prob) if alpha is None else alpha
    b = prob.beta if beta is None else beta
    c = prob.gamma if gamma is None else gamma
    t = lambda x: torch.tensor(np.asarray(x, np.float32).reshape(P.M, -1), device=_dev())  # noqa: E731
    return t(a), t(b), t(c), a, b, c


def rel_err(g_gpu, g_ref, scale):
    return np.abs(g_gpu - g_ref) / np.maximum(np.abs(g_ref), scale)


def check_bound(prob, mode=0, tol=1e-5, alpha=None, beta=None, gamma=None, grads=True, gtol=1e-4):
    from paper_2208_05740_amd import binding as B
    P = upload(prob)
    a, b, c, a64, b64, c64 = params(prob, P, alpha, beta, gamma)
    out, ver, g = B.bound(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a, b, c, mode=mode, grads=grads,
                          verified=True)
    import torch
    torch.cuda.synchronize()
    gb = out.cpu().numpy()
    a32 = a.cpu().numpy().astype(np.float64).reshape(prob.B, prob.S, -1)
    b32 = b.cpu().numpy().astype(np.float64).reshape(prob.B, prob.S, -1)
    c32 = c.cpu().numpy().astype(np.float64).reshape(prob.B, prob.S, -1)
    ref, ga, gbb, gc = O.bound_and_grad(prob, a32, b32, c32)
    ref = ref.reshape(-1)
    T = O.error_scale(prob, a32, b32, c32).reshape(-1)
    err = rel_err(gb, ref, T)
    assert err.max() <= tol, (err.max(), gb[:4], ref[:4])
    assert np.array_equal(ver.cpu().numpy(), (gb >= 0).astype(np.uint8))
    if grads:
        for got, want in zip(g, (ga, gbb, gc)):
            got = got.cpu().numpy().reshape(prob.B * prob.S, -1)
            want = want.reshape(prob.B * prob.S, -1)
            if want.size == 0:
                continue
            scale = np.abs(want).max(1, keepdims=True) + 1.0
            d = np.abs(got - want) / scale
            assert d.max() <= gtol, (d.max(), np.unravel_index(d.argmax(), d.shape))
    return gb, ref, T


def test_mlp8_fp32_bound_and_gradients_match_oracle():
    check_bound(gen.make_workload("mlp8", 0))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tiny_mlp_with_splits_and_cuts(seed):
    p = gen.make_tiny("mlp", seed, B=5, splits=(1, 3), n_cuts=6, input_terms=1)
    check_bound(p)


def test_mlp784_small_batch_fp32():
    # 784-256x6-10 with 200 cuts, 1-8 splits per domain: several column tiles
    # per layer and a ragged last row tile (M = 5 * 9 = 45).
    p = gen.make_workload("mlp784", 0, B=5)
    rng = np.random.default_rng(0)
    prep = O.Prepared(p)
    alpha = rng.random((p.B, p.S, prep.n_I)).astype(np.float32)
    gamma = (rng.random((p.B, p.S, p.cuts.n)) * 0.1).astype(np.float32)
    check_bound(p, alpha=alpha, gamma=gamma)


def test_mlp784_small_batch_bf16_close_to_oracle():
    p = gen.make_workload("mlp784", 0, B=3)
    check_bound(p, mode=1, tol=2e-2, grads=False)


def test_no_cuts_no_splits_edge_case():
    p = gen.make_tiny("mlp", 3, B=2, splits=(0, 0), n_cuts=0)
    check_bound(p)


def test_single_row():
    p = gen.make_tiny("mlp", 4, B=1, splits=(1, 1), n_cuts=2, S=1)
    check_bound(p)


@pytest.mark.parametrize("kind", ["cnn16", "res16"])
@pytest.mark.parametrize("B,S", [(1, 1), (1, 2), (5, 1)])
def test_conv_row_counts_off_the_four_row_groups(kind, B, S):
    # conv workgroups take four batch rows: 1, 2 and 5 rows leave 3, 2 and 3
    # of them empty
    p = gen.make_tiny(kind, 6, B=B, splits=(1, 2), n_cuts=4, S=S, input_terms=1)
    check_bound(p)


def test_invalid_inputs_raise():
    import torch
    from paper_2208_05740_amd import binding as B
    p = gen.make_tiny("mlp", 0, B=2, splits=(1, 2), n_cuts=3)
    P = upload(p)
    a, b, c, *_ = params(p, P)
    bad = a.clone()
    bad[0, 0] = 1.5
    with pytest.raises(B.GcpError) as ei:
        B.bound(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, bad, b, c, validate=True)
    assert ei.value.code == -2
    bad = c.clone()
    bad[0, 0] = float("nan")
    with pytest.raises(B.GcpError) as ei:
        B.bound(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a, b, bad, validate=True)
    assert ei.value.code == -3
    with pytest.raises(B.GcpError):
        B.bound(P.net, P.x0, -1.0, P.C, P.splits, P.cuts, a, b, c)
    # a split on a root-stable neuron is rejected at packing time
    prep = O.Prepared(p)
    q = prep.relu[0]
    stable = int(np.nonzero(prep.cls[q] != 2)[0][0])
    sp = gen.Splits(np.array([[q]], np.int32), np.array([[stable]], np.int32), np.array([[1]], np.int8))
    with pytest.raises(B.GcpError):
        B.Splits(P.net, sp)
    torch.cuda.synchronize()


def test_bad_splits_cuts_and_call_arguments_are_rejected_before_any_launch():
    """Host-side validation of the handles and call arguments (include/gcp.h):
    every case returns GCP_EINVAL and leaves nothing launched."""
    import torch
    from paper_2208_05740_amd import binding as B
    p = gen.make_tiny("mlp", 0, B=2, splits=(1, 2), n_cuts=3)
    P = upload(p)
    prep = O.Prepared(p)
    q = prep.relu[0]
    unst = [int(j) for j in np.nonzero(prep.cls[q] == 2)[0]]
    out_node = len(p.net.nodes) - 1

    def splits(node, neuron, sign):
        a = lambda x, t: np.asarray(x, t).reshape(len(x), -1)  # noqa: E731
        return gen.Splits(a(node, np.int32), a(neuron, np.int32), a(sign, np.int8))

    def rejected(make):
        with pytest.raises(B.GcpError) as ei:
            make()
        assert ei.value.code == -1, ei.value

    z = np.zeros((0, 1))
    rejected(lambda: B.Splits(P.net, gen.Splits(z.astype(np.int32), z.astype(np.int32), z.astype(np.int8))))
    rejected(lambda: B.Splits(P.net, splits([[-1] * 128], [[0] * 128], [[1] * 128])))        # K > 127
    rejected(lambda: B.Splits(P.net, splits([[q]], [[unst[0]]], [[0]])))                     # sign 0
    rejected(lambda: B.Splits(P.net, splits([[q, q]], [[unst[0], unst[0]]], [[1, -1]])))     # split twice
    rejected(lambda: B.Splits(P.net, splits([[out_node]], [[0]], [[1]])))                    # not a ReLU node
    rejected(lambda: B.Splits(P.net, splits([[q]], [[8]], [[1]])))                           # neuron out of range

    def cuts(cut, node, neuron, kind, n=1):
        e = len(cut)
        return gen.Cuts(n, np.asarray(cut, np.int32), np.asarray(node, np.int32), np.asarray(neuron, np.int32),
                        np.asarray(kind, np.int8), np.ones(e), np.zeros(n))
    rejected(lambda: B.Cuts(P.net, cuts([1], [q], [0], [0])))                   # cut index >= N
    rejected(lambda: B.Cuts(P.net, cuts([0], [q], [0], [3])))                   # unknown coefficient kind
    rejected(lambda: B.Cuts(P.net, cuts([0], [-1], [0], [0])))                  # input entry of kind H
    rejected(lambda: B.Cuts(P.net, cuts([0], [q], [8], [0])))                   # neuron out of range
    rejected(lambda: B.Cuts(P.net, cuts([0], [out_node], [0], [0])))            # output node

    a, b, c, *_ = params(p, P)
    rejected(lambda: B.bound(P.net, P.x0, P.eps, P.C[:0], P.splits, P.cuts, a, b, c))          # S = 0
    rejected(lambda: B.bound(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a, b, c, mode=7))      # unknown mode
    other = upload(gen.make_tiny("mlp", 0, B=2, splits=(1, 2), n_cuts=3))
    rejected(lambda: B.bound(P.net, P.x0, P.eps, P.C, other.splits, P.cuts, a, b, c))         # foreign splits
    rejected(lambda: B.bound(P.net, P.x0, P.eps, P.C, P.splits, other.cuts, a, b, c))         # foreign cuts
    torch.cuda.synchronize()
    # the handles still work after the rejected calls
    out, _, _ = B.bound(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a, b, c)
    ref = O.bound(p, O.full_alpha(p), p.beta, p.gamma).reshape(-1)
    assert np.allclose(out.cpu().numpy(), ref, rtol=1e-5, atol=1e-5)


def test_unsupported_net_structures_are_rejected_at_creation():
    """Structures the bound pass has no form for fail when the net is created
    (GCP_EUNSUPPORTED), not in a later call: the input feeding two edges, an
    identity edge from the input, a ReLU node nothing consumes."""
    from paper_2208_05740_amd import binding as B
    from workloads.gen import Edge, Net, Node
    r = np.random.default_rng(0)
    W = lambda o, i: gen._f32(r.normal(0.0, 0.4, (o, i)))  # noqa: E731
    b = lambda n: gen._f32(r.normal(0.0, 0.3, n))  # noqa: E731
    nets = [
        ("several consumers", Net((6,), [Node((8,), b(8), [Edge(-1, "dense", W(8, 6))]),
                                         Node((8,), b(8), [Edge(0, "dense", W(8, 8)), Edge(-1, "dense", W(8, 6))]),
                                         Node((3,), b(3), [Edge(1, "dense", W(3, 8))], relu=False)])),
        ("identity edge", Net((6,), [Node((6,), b(6), [Edge(-1, "identity")]),
                                     Node((3,), b(3), [Edge(0, "dense", W(3, 6))], relu=False)])),
        ("without consumers", Net((6,), [Node((8,), b(8), [Edge(-1, "dense", W(8, 6))]),
                                         Node((8,), b(8), [Edge(0, "dense", W(8, 8))]),
                                         Node((3,), b(3), [Edge(0, "dense", W(3, 8))], relu=False)])),
    ]
    x0 = r.random(6)
    for why, net in nets:
        lu = gen.ibp_bounds(net, x0, 0.1)
        with pytest.raises(B.GcpError) as ei:
            B.Net(net, lu)
        assert ei.value.code == -6 and why in str(ei.value), (why, str(ei.value))
    ok = Net((6,), [Node((8,), b(8), [Edge(-1, "dense", W(8, 6))]),
                    Node((3,), b(3), [Edge(0, "dense", W(3, 8))], relu=False)])
    B.Net(ok, gen.ibp_bounds(ok, x0, 0.1))      # the device is usable afterwards


def test_autograd_function_matches_adjoint():
    import torch
    from paper_2208_05740_amd import binding as B
    p = gen.make_tiny("mlp", 1, B=3, splits=(1, 2), n_cuts=4)
    P = upload(p)
    a, b, c, *_ = params(p, P)
    a.requires_grad_(True); b.requires_grad_(True); c.requires_grad_(True)
    w = torch.linspace(0.5, 1.5, P.M, device=a.device, dtype=torch.float64)
    out = B.gcp_bound_autograd(P, a, b, c)
    (out * w).sum().backward()
    _, _, g = B.bound(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a.detach(), b.detach(), c.detach(), grads=True)
    wf = w.float()[:, None]
    assert torch.allclose(a.grad, g[0] * wf) and torch.allclose(c.grad, g[2] * wf)
    assert torch.allclose(b.grad, g[1] * wf)


def _optimize(prob, P, mode, iters=20, a=None, b=None, c=None):
    import torch
    from paper_2208_05740_amd import binding as B
    a0, b0, c0, *_ = params(prob, P)
    a = a0.clone() if a is None else a
    b = b0.clone() if b is None else b
    c = c0.clone() if c is None else c
    st = torch.zeros(B.adam_state_size(P.M, P.n_I, P.K, P.N), dtype=torch.float32, device=_dev())
    o = prob.opt
    out, ver = B.optimize(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a, b, c, st, iters=iters,
                          lr_alpha=o["lr_alpha"], lr_mult=o["lr_mult"], decay=o["decay"], mode=mode)
    torch.cuda.synchronize()
    return out.cpu().numpy(), a, b, c


@pytest.mark.parametrize("kind,seed", [("mlp", 0), ("mlp", 2)])
def test_optimize_zero_iterations_is_the_certified_bound(kind, seed):
    p = gen.make_tiny(kind, seed, B=3, splits=(1, 2), n_cuts=4)
    P = upload(p)
    g, a, b, c = _optimize(p, P, 0, iters=0)
    ref = O.bound(p).reshape(-1)
    T = O.error_scale(p).reshape(-1)
    assert rel_err(g, ref, T).max() <= 1e-5


@pytest.mark.parametrize("which", ["tiny", "mlp784"])
def test_optimize_fp32_matches_oracle_optimisation(which):
    p = gen.make_tiny("mlp", 1, B=4, splits=(1, 2), n_cuts=6, gamma_dist="zero") if which == "tiny" \
        else gen.make_workload("mlp784", 0, B=2)
    P = upload(p)
    g, a, b, c = _optimize(p, P, 0)
    # certifying pass = the oracle's bound at the device's final parameters
    a64, b64, c64 = (x.cpu().numpy().astype(np.float64).reshape(p.B, p.S, -1) for x in (a, b, c))
    ref = O.bound(p, a64, b64, c64).reshape(-1)
    T = O.error_scale(p, a64, b64, c64).reshape(-1)
    assert rel_err(g, ref, T).max() <= 1e-5
    assert np.all(a64 >= 0) and np.all(a64 <= 1) and np.all(b64 >= 0) and np.all(c64 >= 0)
    # the same 20 Adam steps in fp64 end at (nearly) the same bound
    go, *_ = O.optimize(p)
    To = O.error_scale(p).reshape(-1)
    assert rel_err(g, go.reshape(-1), To).max() <= 1e-3, rel_err(g, go.reshape(-1), To).max()
    # and the optimisation improved on the starting point
    g0 = O.bound(p).reshape(-1)
    assert np.mean(g) > np.mean(g0)


def test_optimize_bf16_final_bound_close_to_fp32():
    p = gen.make_workload("mlp784", 0, B=4)
    P = upload(p)
    g32, *_ = _optimize(p, P, 0)
    g16, a, b, c = _optimize(p, P, 1)
    rel = np.abs(g16 - g32) / np.abs(g32)
    assert rel.max() <= 1e-3, (np.median(rel), rel.max())
    # the bf16-optimised parameters are certified exactly (fp32/fp64 pass)
    a64, b64, c64 = (x.cpu().numpy().astype(np.float64).reshape(p.B, p.S, -1) for x in (a, b, c))
    ref = O.bound(p, a64, b64, c64).reshape(-1)
    T = O.error_scale(p, a64, b64, c64).reshape(-1)
    assert rel_err(g16, ref, T).max() <= 1e-5


# ------------------------------------------------------------------ conv / residual nets

@pytest.mark.parametrize("kind,seed", [("cnn16", 0), ("cnn16", 3), ("res16", 1), ("res16", 2)])
def test_conv_and_residual_fp32_bound_and_gradients(kind, seed):
    p = gen.make_tiny(kind, seed, B=3, splits=(1, 3), n_cuts=6, input_terms=1)
    check_bound(p)


def test_conv_bf16_close_to_oracle():
    p = gen.make_tiny("cnn16", 5, B=4, splits=(1, 3), n_cuts=6)
    check_bound(p, mode=1, tol=2e-2, grads=False)


def test_cnn_small_batch_fp32():
    # Conv(3,16,4,s2,p1) - Conv(16,32,4,s2,p1) - 2048-100-10 with 500 cuts
    p = gen.make_workload("cnn", 0, B=2)
    rng = np.random.default_rng(1)
    prep = O.Prepared(p)
    alpha = rng.random((p.B, p.S, prep.n_I)).astype(np.float32)
    gamma = (rng.random((p.B, p.S, p.cuts.n)) * 0.05).astype(np.float32)
    check_bound(p, alpha=alpha, gamma=gamma)


def test_resnet_single_domain_fp32():
    p = gen.make_workload("resnet", 0, B=1)
    rng = np.random.default_rng(2)
    gamma = (rng.random((p.B, p.S, p.cuts.n)) * 0.05).astype(np.float32)
    check_bound(p, gamma=gamma)


def test_optimize_conv_matches_oracle():
    p = gen.make_tiny("res16", 3, B=2, splits=(1, 2), n_cuts=5, gamma_dist="zero")
    P = upload(p)
    g, a, b, c = _optimize(p, P, 0)
    a64, b64, c64 = (x.cpu().numpy().astype(np.float64).reshape(p.B, p.S, -1) for x in (a, b, c))
    ref = O.bound(p, a64, b64, c64).reshape(-1)
    T = O.error_scale(p, a64, b64, c64).reshape(-1)
    assert rel_err(g, ref, T).max() <= 1e-5
    go, *_ = O.optimize(p)
    To = O.error_scale(p).reshape(-1)
    assert rel_err(g, go.reshape(-1), To).max() <= 1e-3


GRAPH_CASES = [
    ("mlp784", dict(seed=1, B=3, roots="ibp"), 0),
    ("tiny", dict(kind="cnn", seed=2, B=3, splits=(1, 2), n_cuts=6, input_terms=1), 0),
    ("tiny", dict(kind="res16", seed=4, B=2, splits=(1, 2), n_cuts=5, input_terms=1), 1),
    ("cnn", dict(seed=0, B=2, roots="ibp"), 0),       # 3x32x32 stem: the direct transposed conv
    ("cnn", dict(seed=0, B=2, roots="ibp"), 1),
]


@pytest.mark.parametrize("case", range(len(GRAPH_CASES)))
def test_graph_replayed_optimisation_equals_eager(case):
    # One Adam iteration captured in a hipGraph and replayed must give the
    # same final parameters and bound as the eager loop, on every call, with
    # eager work in between: dense nets, conv nets (the input term through
    # the transposed conv) and a residual DAG, in both precisions.
    import torch
    from paper_2208_05740_amd import binding as B
    which, kw, mode = GRAPH_CASES[case]
    kw = dict(kw)
    print(f"graph replay: {which} {kw} mode={mode}", flush=True)
    if which == "tiny":
        p = gen.make_tiny(kw.pop("kind"), kw.pop("seed"), **kw)
    else:
        p = gen.make_workload(which, kw.pop("seed"), **kw)
    P = upload(p)
    a0, b0, c0, *_ = params(p, P)
    o = p.opt

    def run(graph):
        a, b, c = a0.clone(), b0.clone(), c0.clone()
        st = torch.zeros(B.adam_state_size(P.M, P.n_I, P.K, P.N), dtype=torch.float32, device=_dev())
        out, _ = B.optimize(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a, b, c, st, iters=o["iters"],
                            lr_alpha=o["lr_alpha"], lr_mult=o["lr_mult"], decay=o["decay"], mode=mode,
                            use_graph=graph)
        torch.cuda.synchronize()
        return out.cpu().numpy(), a.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()

    ref = run(False)
    for rep in range(3):
        got = run(True)
        for x, y in zip(got, ref):
            assert np.array_equal(x, y), rep
        eager = run(False)
        for x, y in zip(eager, ref):
            assert np.array_equal(x, y), rep


@pytest.mark.parametrize("kind", ["mlp", "cnn16", "res16"])
def test_first_call_on_a_side_stream_while_the_null_stream_is_busy(kind):
    # A fresh net's first gcp_optimize allocates and clears its workspace;
    # on a caller's stream that does not wait for the null stream, the
    # iterations must still see the cleared buffers and their own tables
    # (the null stream is kept busy, so a clear left queued there would land
    # after them).  The result must equal the same call on the default stream.
    import torch
    from paper_2208_05740_amd import binding as B
    if torch.cuda.default_stream().cuda_stream != 0:
        pytest.skip("the default stream is not the null stream")
    print(f"first call on a side stream: {kind}", flush=True)
    p = gen.make_tiny(kind, 2, B=6, splits=(1, 3), n_cuts=6, input_terms=1)
    g_ref, a_ref, b_ref, c_ref = _optimize(p, upload(p), 0)
    P = upload(p)                                       # fresh net: no workspace yet
    s = torch.cuda.Stream()
    x = torch.rand(4096, 4096, device=_dev())
    for _ in range(30):                                 # tens of ms of work on the null stream
        x = torch.tanh(x @ x)
    with torch.cuda.stream(s):
        g, a, b, c = _optimize(p, P, 0)
    torch.cuda.synchronize()
    assert np.isfinite(x.sum().item())
    assert np.array_equal(g, g_ref)
    for got, want in ((a, a_ref), (b, b_ref), (c, c_ref)):
        assert torch.equal(got, want)


# ------------------------------------------------------------------ batched instances

def _batch_items(probs, Ps):
    import torch
    from paper_2208_05740_amd import binding as B
    items = []
    for p, P in zip(probs, Ps):
        a, b, c, *_ = params(p, P)
        items.append(dict(P=P, alpha=a, beta=b, gamma=c,
                          state=torch.zeros(B.adam_state_size(P.M, P.n_I, P.K, P.N), dtype=torch.float32,
                                            device=_dev()),
                          bound=torch.empty(P.M, dtype=torch.float64, device=_dev()),
                          verified=torch.empty(P.M, dtype=torch.uint8, device=_dev())))
    return items


@pytest.mark.parametrize("mode", [0, 1])
def test_batched_optimisation_equals_per_instance(mode):
    # uneven instances (depth, width, input size, domains, cuts) optimised in
    # grouped launches must give exactly the per-instance results
    import torch
    from paper_2208_05740_amd import binding as B
    probs = gen.make_batch(seed=3, n_inst=5, bmax=24)
    Ps = [upload(p) for p in probs]
    o = probs[0].opt
    # an fp32 certifying pass first, so the buffers shared by both
    # precisions hold fp32 data in their padding when the bf16 passes run
    for p, P in zip(probs, Ps):
        _optimize(p, P, 0, iters=1)
    ref = []
    for p, P in zip(probs, Ps):
        g, a, b, c = _optimize(p, P, mode)
        ref.append((g, a.cpu().numpy(), c.cpu().numpy()))
    for graph in (False, True, True):
        items = _batch_items(probs, Ps)
        B.optimize_batch(items, iters=o["iters"], lr_alpha=o["lr_alpha"], lr_mult=o["lr_mult"], decay=o["decay"],
                         mode=mode, use_graph=graph)
        torch.cuda.synchronize()
        for it, (g, a, c) in zip(items, ref):
            assert np.array_equal(it["bound"].cpu().numpy(), g)
            assert np.array_equal(it["alpha"].cpu().numpy(), a)
            assert np.array_equal(it["gamma"].cpu().numpy(), c)


@pytest.mark.parametrize("kind,mode", [("mlp", 1), ("mlp", 0), ("cnn16", 1), ("res16", 1), ("res16", 0)])
def test_recomputed_ahat_equals_stored(kind, mode):
    # a_hat rebuilt in the adjoint from the consumer's Lambda (same GEMM, same
    # tiles) must give exactly the results of storing it in the bound pass
    import torch
    from paper_2208_05740_amd import binding as B
    p = gen.make_tiny(kind, 1, B=5, splits=(1, 3), n_cuts=6)
    P = upload(p)
    o = p.opt
    outs = []
    for flag in (B.GCP_FLAG_STORE_AHAT, B.GCP_FLAG_RECOMPUTE):
        a, b, c, *_ = params(p, P)
        st = torch.zeros(B.adam_state_size(P.M, P.n_I, P.K, P.N), dtype=torch.float32, device=_dev())
        g, _ = B.optimize(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a, b, c, st, iters=5,
                          lr_alpha=o["lr_alpha"], lr_mult=o["lr_mult"], decay=o["decay"], mode=mode | flag)
        a2, b2, c2, *_ = params(p, P)
        _, _, grads = B.bound(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a2, b2, c2, mode=mode | flag, grads=True)
        torch.cuda.synchronize()
        outs.append([g.cpu().numpy(), a.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()] +
                    [x.cpu().numpy() for x in grads])
    for x, y in zip(*outs):
        assert np.array_equal(x, y)


def test_batched_optimisation_mixed_alone_and_grouped(monkeypatch):
    # instances above the work threshold run their own launches, the rest are
    # grouped; either way the results equal per-instance gcp_optimize
    import torch
    from paper_2208_05740_amd import binding as B
    probs = gen.make_batch(seed=6, n_inst=6, bmax=48)
    work = sorted(p.B * p.S * max((n.size + 15) // 16 * 16 for n in p.net.nodes) for p in probs)
    thr = (work[2] + work[3]) // 2
    assert work[0] < thr <= work[-1]
    monkeypatch.setenv("GCP_BATCH_ALONE_WORK", str(thr))
    Ps = [upload(p) for p in probs]
    o = probs[0].opt
    ref = []
    for p, P in zip(probs, Ps):
        g, a, b, c = _optimize(p, P, 1)
        ref.append((g, a.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()))
    for graph in (False, True):
        items = _batch_items(probs, Ps)
        B.optimize_batch(items, iters=o["iters"], lr_alpha=o["lr_alpha"], lr_mult=o["lr_mult"], decay=o["decay"],
                         mode=1, use_graph=graph)
        torch.cuda.synchronize()
        for it, (g, a, b, c) in zip(items, ref):
            assert np.array_equal(it["bound"].cpu().numpy(), g)
            assert np.array_equal(it["alpha"].cpu().numpy(), a)
            assert np.array_equal(it["beta"].cpu().numpy(), b)
            assert np.array_equal(it["gamma"].cpu().numpy(), c)


@pytest.mark.parametrize("mode", [0, 1])
def test_batched_optimisation_conv_and_residual_instances(mode, monkeypatch):
    # conv and residual instances above the work threshold run alone (their
    # own gcp_optimize launches) beside grouped dense instances, with results
    # equal to per-instance gcp_optimize; below it they would be grouped, and
    # the call is rejected with EUNSUPPORTED before anything runs
    import torch
    from paper_2208_05740_amd import binding as B
    print(f"batch with conv and residual instances, mode={mode}", flush=True)
    probs = [gen.make_tiny("cnn", 2, B=4, splits=(1, 2), n_cuts=6, input_terms=1),
             gen.make_tiny("mlp", 3, B=5, splits=(1, 3), n_cuts=6),
             gen.make_tiny("res16", 4, B=3, splits=(1, 2), n_cuts=5),
             gen.make_tiny("mlp", 5, B=2, splits=(0, 0), n_cuts=0)]
    work = [p.B * p.S * max((n.size + 15) // 16 * 16 for n in p.net.nodes) for p in probs]
    dense = [1, 3]
    lo, hi = max(work[i] for i in dense), min(w for i, w in enumerate(work) if i not in dense)
    assert lo < hi
    Ps = [upload(p) for p in probs]
    o = probs[0].opt
    ref = []
    for p, P in zip(probs, Ps):
        g, a, b, c = _optimize(p, P, mode)
        ref.append((g, a.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()))
    monkeypatch.setenv("GCP_BATCH_ALONE_WORK", str((lo + hi) // 2))
    for graph in (False, True):
        items = _batch_items(probs, Ps)
        B.optimize_batch(items, iters=o["iters"], lr_alpha=o["lr_alpha"], lr_mult=o["lr_mult"], decay=o["decay"],
                         mode=mode, use_graph=graph)
        torch.cuda.synchronize()
        for it, (g, a, b, c) in zip(items, ref):
            assert np.array_equal(it["bound"].cpu().numpy(), g)
            assert np.array_equal(it["alpha"].cpu().numpy(), a)
            assert np.array_equal(it["beta"].cpu().numpy(), b)
            assert np.array_equal(it["gamma"].cpu().numpy(), c)
    monkeypatch.delenv("GCP_BATCH_ALONE_WORK")
    items = _batch_items(probs, Ps)
    for it in items:
        it["bound"].fill_(float("nan"))
    before = [{k: it[k].clone() for k in ("alpha", "beta", "gamma", "state")} for it in items]
    with pytest.raises(B.GcpError) as e:
        B.optimize_batch(items, iters=o["iters"], mode=mode)
    torch.cuda.synchronize()
    assert e.value.code == -6 and "conv" in str(e.value), str(e.value)
    for it, b0 in zip(items, before):
        assert torch.isnan(it["bound"]).all()
        for k, v in b0.items():
            assert torch.equal(it[k], v), k
    # an alone instance with another net's splits: EINVAL, again before anything runs
    monkeypatch.setenv("GCP_BATCH_ALONE_WORK", str((lo + hi) // 2))
    bad = copy.copy(Ps[2])
    bad.splits = Ps[0].splits
    items[2]["P"] = bad
    with pytest.raises(B.GcpError) as e:
        B.optimize_batch(items, iters=o["iters"], mode=mode)
    torch.cuda.synchronize()
    assert e.value.code == -1 and "another net" in str(e.value), str(e.value)
    for it, b0 in zip(items, before):
        assert torch.isnan(it["bound"]).all()
        for k, v in b0.items():
            assert torch.equal(it[k], v), k


def test_batched_optimisation_certified_bound_matches_oracle():
    import torch
    from paper_2208_05740_amd import binding as B
    probs = gen.make_batch(seed=5, n_inst=3, bmax=16)
    Ps = [upload(p) for p in probs]
    items = _batch_items(probs, Ps)
    B.optimize_batch(items, iters=5)
    torch.cuda.synchronize()
    for p, it in zip(probs, items):
        a64, b64, c64 = (it[k].cpu().numpy().astype(np.float64).reshape(p.B, p.S, -1) for k in ("alpha", "beta", "gamma"))
        ref = O.bound(p, a64, b64, c64).reshape(-1)
        T = O.error_scale(p, a64, b64, c64).reshape(-1)
        assert rel_err(it["bound"].cpu().numpy(), ref, T).max() <= 1e-5


# ------------------------------------------------------------ general output form
@pytest.mark.parametrize("kind,seed", [("mlp", 0), ("mlp", 3), ("cnn", 1)])
def test_materialised_output_lambda_matches_oracle(kind, seed, monkeypatch):
    # the output's Lambda = C pushed through the ordinary kernels (instead of
    # the C W shortcut) gives the same bounds and gradients
    monkeypatch.setenv("GCP_OUT_GENERAL", "1")
    p = gen.make_tiny(kind, seed, B=3, splits=(1, 2), n_cuts=5)
    check_bound(p, mode=0)


# ------------------------------------------------------------ intermediate bounds
@pytest.mark.parametrize("kind,seed", [("mlp", 0), ("cnn", 1), ("res", 2), ("cnn16", 3), ("res16", 4)])
def test_crown_intermediate_bounds_match_oracle(kind, seed):
    # layer by layer: node k's bounds from the device against the oracle's
    # CROWN on the same prefix, both given the device's bounds of nodes < k
    import torch
    from paper_2208_05740_amd import binding as B
    from oracle import crown
    p = gen.make_tiny(kind, seed, eps=0.1)
    x0 = torch.tensor(p.x0, dtype=torch.float64, device=_dev())
    got = B.crown_bounds(p.net, x0, p.eps)
    want = crown.crown_intermediate_bounds(p.net, p.x0, p.eps, lu_given=got)
    for (gl, gu), (wl, wu) in zip(got, want):
        scale = np.abs(wl) + np.abs(wu) + 1.0
        assert (np.abs(gl - wl) / scale).max() <= 1e-5
        assert (np.abs(gu - wu) / scale).max() <= 1e-5
    # sound: every sampled point's pre-activations lie inside
    rng = np.random.default_rng(seed)
    xs = p.x0[None, :] + p.eps * rng.uniform(-1, 1, size=(2000, p.x0.size))
    _, pre = lp.plain_forward(p.net, xs, return_pre=True)
    relu = [i for i, n in enumerate(p.net.nodes) if n.relu]
    for (l, u), i in zip(got, relu):
        assert (pre[i] >= l[None, :] - 1e-6).all() and (pre[i] <= u[None, :] + 1e-6).all()


@pytest.mark.parametrize("kind,seed", [("mlp", 5), ("cnn", 6), ("res", 7), ("res16", 8)])
def test_domain_intermediate_bounds_match_oracle(kind, seed):
    # one BaB domain (splits that a reference point satisfies): layer by layer
    # against the oracle given the device's earlier bounds, and sound on the
    # sampled points of the domain
    import torch
    from paper_2208_05740_amd import binding as B
    from oracle import crown
    p = gen.make_tiny(kind, seed, eps=0.1)
    rng = np.random.default_rng(seed)
    x_ref = p.x0 + p.eps * rng.uniform(-1, 1, size=p.x0.size)
    root = crown.crown_intermediate_bounds(p.net, p.x0, p.eps)
    _, pre_ref = lp.plain_forward(p.net, x_ref[None, :], return_pre=True)
    relu = [i for i, n in enumerate(p.net.nodes) if n.relu]
    cand = [(k, int(j)) for (l, u), k in zip(root, relu) for j in np.nonzero((l < 0) & (u > 0))[0]]
    pick = rng.choice(len(cand), size=min(5, len(cand)), replace=False)
    sp = [(k, j, 1 if pre_ref[k][0][j] >= 0 else -1) for k, j in (cand[t] for t in pick)]
    x0 = torch.tensor(p.x0, dtype=torch.float64, device=_dev())
    got = B.crown_bounds(p.net, x0, p.eps, splits=sp)
    want = crown.crown_intermediate_bounds(p.net, p.x0, p.eps, lu_given=got, splits=sp)
    for (gl, gu), (wl, wu) in zip(got, want):
        scale = np.abs(wl) + np.abs(wu) + 1.0
        assert (np.abs(gl - wl) / scale).max() <= 1e-5
        assert (np.abs(gu - wu) / scale).max() <= 1e-5
        assert (gl <= gu).all()
    xs = p.x0[None, :] + p.eps * rng.uniform(-1, 1, size=(20000, p.x0.size))
    xs[0] = x_ref
    _, pre = lp.plain_forward(p.net, xs, return_pre=True)
    keep = np.ones(xs.shape[0], bool)
    for k, j, sg in sp:
        keep &= sg * pre[k][:, j] >= 0
    for (l, u), i in zip(got, relu):
        assert (pre[i][keep] >= l[None, :] - 1e-6).all() and (pre[i][keep] <= u[None, :] + 1e-6).all()
    # the domain's bounds are valid root bounds of a net for that domain
    net = B.Net(p.net, got)
    del net


def test_crown_intermediate_bounds_as_root_bounds_mlp784():
    # CROWN bounds of a 784-256x3-10 MLP computed on the device: tighter than
    # interval bounds on the deeper layers, and usable as root bounds
    import torch
    from paper_2208_05740_amd import binding as B
    from oracle import crown
    net = gen.mlp_net(np.random.default_rng(11), [784, 256, 256, 256, 10])
    x0 = np.random.default_rng(12).uniform(0, 1, 784)
    eps = 0.015
    got = B.crown_bounds(net, torch.tensor(x0, dtype=torch.float64, device=_dev()), eps)
    ibp = gen.ibp_bounds(net, x0, eps)
    assert np.allclose(got[0][0], ibp[0][0], rtol=1e-5, atol=1e-5)
    for (l, u), (il, iu) in list(zip(got, ibp))[1:]:
        assert (u - l).mean() < (iu - il).mean()
    # node 1 against the oracle given the device's node-0 bounds
    want = crown.crown_intermediate_bounds(type(net)(net.in_shape, net.nodes[:2]), x0, eps, lu_given=got[:1])
    scale = np.abs(want[1][0]) + np.abs(want[1][1]) + 1.0
    assert (np.abs(got[1][0] - want[1][0]) / scale).max() <= 1e-5
    assert (np.abs(got[1][1] - want[1][1]) / scale).max() <= 1e-5


# ------------------------------------------------------------ branch and bound
# (seed, eps, spec row) of tiny MLPs whose root bound is negative after the 20
# Adam iterations but whose exact minimum (one LP per activation pattern) is
# positive: only branching can verify them
BAB_CASES = [(9, 0.1, 0), (21, 0.15, 0), (31, 0.1, 0), (7, 0.1, 1)]


def _tiny_plain(seed, eps, n_cuts=0):
    return gen.make_tiny("mlp", seed, B=1, splits=(0, 0), n_cuts=n_cuts, eps=eps, alpha_init="crown",
                         gamma_dist="zero", beta_dist="zero")


@pytest.mark.parametrize("seed,eps,row", BAB_CASES)
def test_bab_verifies_properties_that_need_branching(seed, eps, row):
    from paper_2208_05740_amd import binding as B
    p = _tiny_plain(seed, eps)
    exact = lp.mip_value_enum(p, 0, row)
    root = O.optimize(p)[0][row]
    assert exact > 0 and root < 0
    P = upload(p)
    r = B.bab(P.net, P.x0, P.eps, P.C[row].contiguous(), batch=8, max_depth=16)
    assert r["status"] == B.GCP_BAB_VERIFIED, r
    assert r["bounded"] > 1 and r["unresolved"] == 0 and r["open"] == 0
    assert 0.0 <= r["lower"] <= exact + 1e-6


def test_bab_with_cuts_verifies_and_never_verifies_a_false_property():
    # sound on every row of a few tiny nets (with valid cuts): verified only
    # when the exact minimum is positive, and the reported lower bound never
    # exceeds the exact minimum when not verified
    from paper_2208_05740_amd import binding as B
    n_false = n_true = 0
    for seed in range(6):
        p = _tiny_plain(seed, 0.15, n_cuts=4)
        if sum(int(((l < 0) & (u > 0)).sum()) for l, u in p.lu) > 12:
            continue
        P = upload(p)
        for row in range(p.S):
            exact = lp.mip_value_enum(p, 0, row)
            r = B.bab(P.net, P.x0, P.eps, P.C[row].contiguous(), P.cuts, batch=16, max_depth=16)
            if r["status"] == B.GCP_BAB_VERIFIED:
                assert exact > 0 and r["lower"] <= exact + 1e-6
                n_true += 1
            else:
                assert r["lower"] <= exact + 1e-6
                n_false += exact < 0
    assert n_true > 0 and n_false > 0


# ------------------------------------------------------------ full sizes, sampled rows
def _full_size_check(name, B, n_rows, seed=0):
    # the workload at the size the bench times: bf16-optimised, fp32/fp64
    # certified bounds of every row on the device; a random sample of rows
    # recomputed by the oracle at the device's final parameters (fp64)
    import torch
    from paper_2208_05740_amd import binding as B_
    prob = gen.make_workload(name, 0, B=B)
    P = upload(prob)
    M = P.M
    a = torch.tensor(gen.crown_alpha_init(prob.lu), dtype=torch.float32, device=_dev()).expand(M, -1).contiguous()
    b = torch.tensor(prob.beta.reshape(M, -1), dtype=torch.float32, device=_dev())
    c = torch.zeros(M, P.N, dtype=torch.float32, device=_dev())
    st = torch.zeros(B_.adam_state_size(M, P.n_I, P.K, P.N), dtype=torch.float32, device=_dev())
    o = prob.opt
    out, ver = B_.optimize(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a, b, c, st, iters=o["iters"],
                           lr_alpha=o["lr_alpha"], lr_mult=o["lr_mult"], decay=o["decay"], mode=B_.GCP_MODE_BF16)
    torch.cuda.synchronize()
    g = out.cpu().numpy()
    assert np.isfinite(g).all()
    assert np.array_equal(ver.cpu().numpy(), (g >= 0).astype(np.uint8))
    rows = np.sort(np.random.default_rng(seed).choice(M, size=n_rows, replace=False))
    f64 = lambda t: t.cpu().numpy().astype(np.float64)[rows]  # noqa: E731
    ref = O.bound(prob, alpha=f64(a), beta=f64(b), gamma=f64(c), rows=rows, flat=True)
    T = O.error_scale(prob, alpha=f64(a), beta=f64(b), gamma=f64(c), rows=rows, flat=True)
    assert rel_err(g[rows], ref, T).max() <= 1e-5


def test_mlp784_full_size_sampled_rows():
    _full_size_check("mlp784", 1024, 48)


def test_cnn_full_size_sampled_rows():
    _full_size_check("cnn", 2048, 12)


def test_resnet_full_size_sampled_rows():
    _full_size_check("resnet", 4096, 3)


@pytest.mark.parametrize("kind", ["mlp", "cnn16", "res16"])
def test_zero_radius_bound_is_the_network_output(kind):
    # eps = 0: every neuron is stable at x0 and the bound is c^T f(x0) itself
    import torch
    from paper_2208_05740_amd import binding as B
    p = gen.make_tiny(kind, 2, B=2, eps=0.0, n_cuts=0)
    P = upload(p)
    a, b, c, *_ = params(p, P)
    out, _, _ = B.bound(P.net, P.x0, 0.0, P.C, P.splits, P.cuts, a, b, c, mode=0)
    torch.cuda.synchronize()
    f = lp.plain_forward(p.net, p.x0[None, :])[0]
    want = np.tile(p.C @ f, p.B)
    assert np.allclose(out.cpu().numpy(), want, rtol=1e-5, atol=1e-5 * (1 + np.abs(f).max()))


# ------------------------------------------------------------ soundness and finite differences
@pytest.mark.parametrize("name", ["mlp8", "mlp784"])
def test_certified_bounds_never_exceed_sampled_minimum(name):
    # after the bf16-optimised ascent and the fp32/fp64 certifying pass, no
    # bound is above the minimum of c^T f over sampled points of its domain
    import torch
    from paper_2208_05740_amd import binding as B
    prob = gen.make_workload(name, 0, B=None if name == "mlp8" else 16)
    P = upload(prob)
    a, b, c, *_ = params(prob, P)
    st = torch.zeros(B.adam_state_size(P.M, P.n_I, P.K, P.N), dtype=torch.float32, device=_dev())
    out, _ = B.optimize(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a, b, c, st, iters=20, mode=B.GCP_MODE_BF16)
    torch.cuda.synchronize()
    g = out.cpu().numpy().reshape(prob.B, prob.S)
    for dom in range(prob.B):
        smin = lp.sampled_min(prob, b=dom, n=20000 if name == "mlp784" else 100000, seed=dom)
        assert (g[dom] <= smin + 1e-9).all(), (dom, g[dom], smin)


@pytest.mark.parametrize("name,seed,B_,n", [("cnn", 3, 4, 2000), ("resnet", 5, 2, 100)])
def test_conv_certified_bounds_never_exceed_points_of_their_domains(name, seed, B_, n):
    # CNN and ResNet workloads: every domain keeps its split neurons but takes
    # their signs from a reference point, so the reference point and the
    # sampled points around it that meet the splits are points of the domain;
    # the certified bound may not exceed c^T f at any of them
    import dataclasses

    import torch
    from paper_2208_05740_amd import binding as B
    prob = gen.make_workload(name, 0, B=B_)
    rng = np.random.default_rng(seed)
    x_ref = prob.x0 + prob.eps * rng.uniform(-1, 1, size=prob.x0.size)
    _, pre_ref = lp.plain_forward(prob.net, x_ref[None, :], return_pre=True)
    sp = prob.splits
    sign = sp.sign.copy()
    for b_ in range(sp.B):
        for s_ in range(sp.K):
            if sp.node[b_, s_] >= 0:
                sign[b_, s_] = 1 if pre_ref[int(sp.node[b_, s_])][0][int(sp.neuron[b_, s_])] >= 0 else -1
    prob = dataclasses.replace(prob, splits=gen.Splits(sp.node, sp.neuron, sign))
    P = upload(prob)
    a, b, c, *_ = params(prob, P)
    st = torch.zeros(B.adam_state_size(P.M, P.n_I, P.K, P.N), dtype=torch.float32, device=_dev())
    out, _ = B.optimize(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a, b, c, st, iters=20, mode=B.GCP_MODE_BF16)
    torch.cuda.synchronize()
    g = out.cpu().numpy().reshape(prob.B, prob.S)
    X = np.clip(x_ref[None, :] + 0.05 * prob.eps * rng.uniform(-1, 1, size=(n, x_ref.size)),
                prob.x0 - prob.eps, prob.x0 + prob.eps)
    X[0] = x_ref
    fx, pre = lp.plain_forward(prob.net, X, return_pre=True)
    for dom in range(prob.B):
        ok = np.ones(X.shape[0], bool)
        for s_ in range(sp.K):
            if sp.node[dom, s_] >= 0:
                v = pre[int(sp.node[dom, s_])][:, int(sp.neuron[dom, s_])]
                ok &= (v >= 0) if sign[dom, s_] > 0 else (v <= 0)
        assert ok[0]
        vmin = (fx[ok] @ prob.C.T).min(0)
        assert (g[dom] <= vmin + 1e-9).all(), (dom, g[dom], vmin)


@pytest.mark.parametrize("kind,B_", [("res16", 2), ("resnet", 1)])
def test_adjoint_gradient_matches_central_differences(kind, B_):
    # d bound / d alpha and d gamma from the device adjoint against central
    # differences of the device bound (fp32 GEMMs, fp64 sums); the bound is
    # piecewise linear in each coordinate, so coordinates whose one-sided
    # slopes disagree (a kink within the step) are skipped
    import torch
    from paper_2208_05740_amd import binding as B
    if kind == "resnet":
        prob = gen.make_workload("resnet", 0, B=B_)
    else:
        prob = gen.make_tiny(kind, 4, B=B_, splits=(1, 2), n_cuts=5)
    P = upload(prob)
    a, b, c, *_ = params(prob, P)
    a = a.clamp(0.05, 0.95)          # interior of the box, so +-h stays feasible
    _, _, (ga, gb, gc) = B.bound(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a, b, c, mode=0, grads=True)

    def total(a_, c_):
        out, _, _ = B.bound(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a_, b, c_, mode=0)
        return float(out.double().sum().cpu())

    # rounding noise of a central difference: fp32 unit roundoff times the
    # total magnitude of the terms summed into the bound, over the step
    a64 = a.cpu().numpy().astype(np.float64).reshape(prob.B, prob.S, -1)
    b64 = b.cpu().numpy().astype(np.float64).reshape(prob.B, prob.S, -1)
    c64 = c.cpu().numpy().astype(np.float64).reshape(prob.B, prob.S, -1)
    T = float(O.error_scale(prob, a64, b64, c64).sum())
    rng = np.random.default_rng(7)
    h = 1e-2
    noise = 4 * 2.0 ** -24 * T / h
    checked = 0
    for which, t, g in (("alpha", a, ga), ("gamma", c, gc)):
        if t.numel() == 0:
            continue
        flat = t.view(-1)
        for idx in rng.choice(flat.numel(), size=min(12, flat.numel()), replace=False):
            f0 = total(a, c)
            old = float(flat[idx])
            flat[idx] = old + h
            fp = total(a, c)
            flat[idx] = old - h
            fm = total(a, c)
            flat[idx] = old
            up, down = (fp - f0) / h, (f0 - fm) / h
            scale = max(abs(up), abs(down), 1.0)
            if abs(up - down) > 1e-3 * scale + 2 * noise:
                continue                     # kink within the step
            fd = (fp - fm) / (2 * h)
            got = float(g.view(-1)[idx])
            assert abs(got - fd) <= 1e-3 * max(abs(fd), abs(got)) + noise, (which, idx, got, fd, noise)
            checked += 1
    assert checked >= 6


def test_c_abi_example_program_matches_oracle(tmp_path):
    # the command-line example drives gcp_net_create / gcp_splits_create /
    # gcp_cuts_create / gcp_bound from C++ with the HIP runtime alone
    import os
    import subprocess
    exe = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2208_05740_amd",
                       "examples", "gcp_bound_mlp")
    assert os.path.exists(exe), "example not built"
    p = gen.make_tiny("mlp", 3, B=3, splits=(1, 2), n_cuts=5, input_terms=1)
    rng = np.random.default_rng(3)
    prep = O.Prepared(p)
    f32 = lambda x: np.asarray(x, np.float32).astype(np.float64)  # noqa: E731
    a = f32(rng.random((p.B, p.S, prep.n_I)))
    b = f32(rng.random((p.B, p.S, p.splits.K)) * 0.5 * (p.splits.node >= 0)[:, None, :])
    c = f32(rng.random((p.B, p.S, p.cuts.n)) * 0.5)
    net = p.net
    dims = [net.in_size] + [n.size for n in net.nodes]
    out = [f"{len(net.nodes)} " + " ".join(map(str, dims))]
    for n in net.nodes:
        out.append(" ".join(repr(float(v)) for v in np.asarray(n.edges[0].W, np.float32).ravel()))
        out.append(" ".join(repr(float(v)) for v in np.asarray(n.bias, np.float32)))
    for l, u in p.lu:
        out.append(" ".join(repr(float(v)) for v in l))
        out.append(" ".join(repr(float(v)) for v in u))
    out.append(" ".join(repr(float(v)) for v in p.x0) + f" {p.eps!r}")
    out.append(f"{p.S} " + " ".join(repr(float(v)) for v in p.C.ravel()))
    sp = p.splits
    out.append(f"{sp.B} {sp.K} " + " ".join(map(str, sp.node.ravel())) + " " + " ".join(map(str, sp.neuron.ravel()))
               + " " + " ".join(map(str, sp.sign.ravel())))
    cu = p.cuts
    ents = " ".join(f"{cu.cut[e]} {cu.node[e]} {cu.neuron[e]} {cu.kind[e]} {float(cu.coef[e])!r}"
                    for e in range(cu.cut.size))
    out.append(f"{cu.n} {cu.cut.size} {ents} " + " ".join(repr(float(v)) for v in cu.d))
    out.append(f"{prep.n_I} " + " ".join(repr(float(v)) for x in (a, b, c) for v in x.ravel()))
    path = tmp_path / "problem.txt"
    path.write_text("\n".join(out) + "\n")
    r = subprocess.run([exe, str(path), "fp32"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    got = np.array([float(t) for t in r.stdout.split()])
    ref = O.bound(p, a, b, c).reshape(-1)
    T = O.error_scale(p, a, b, c).reshape(-1)
    assert got.shape == ref.shape
    assert rel_err(got, ref, T).max() <= 1e-5, (got, ref)
