"""Networks whose nodes sum several inputs (Theorem 3.1 over a DAG: a node's
Lambda is the sum of what its consumers push back through their edges) against
the FP64 oracle, through the C ABI.

Two small dense DAGs exercise how the bound pass and the adjoint combine a
node's contributions: a node whose two in-edges are identity edges (its
adjoint runs elementwise after both have been accumulated), and a node fed
by an identity edge and a dense edge (the fused epilogue of the dense edge
takes the identity contribution as its accumulated input; in fp32 it reads
the identity source in place, in both passes).  Splits, cuts and input cuts
are live.  Tolerances as in the other parity tests: fp32 bound within 1e-5
of max(|g|, T), gradients within 1e-4 of the row's largest, bf16 bound
within 2e-2 of T.
"""
import math

import numpy as np
import pytest

from oracle import gcp_oracle as O
from workloads import gen
from workloads.gen import Edge, Net, Node

pytestmark = pytest.mark.gpu


def _dev():
    import torch
    return torch.device("cuda:0")


def _w(rng, o, i):
    return gen._f32(rng.normal(0.0, math.sqrt(2.0 / i), (o, i)))


def _dag(kind, seed):
    """input 6 -> n0 dense 8 -> n1 dense 8 -> n2 (8) -> n3 dense 5 -> out 3, with n2 = identity(n0) +
    identity(n1) ('two_identity') or identity(n0) + dense(n1) ('identity_dense')."""
    r_w, r_x, r_cut, r_split, r_par = gen._streams([seed, 97])
    b = lambda n: gen._f32(r_w.normal(0.0, math.sqrt(0.1), n))  # noqa: E731
    n0 = Node((8,), b(8), [Edge(-1, "dense", _w(r_w, 8, 6))])
    n1 = Node((8,), b(8), [Edge(0, "dense", _w(r_w, 8, 8))])
    if kind == "two_identity":
        n2 = Node((8,), b(8), [Edge(0, "identity"), Edge(1, "identity")])
    else:
        n2 = Node((8,), b(8), [Edge(0, "identity"), Edge(1, "dense", _w(r_w, 8, 8))])
    n3 = Node((5,), b(5), [Edge(2, "dense", _w(r_w, 5, 8))])
    out = Node((3,), b(3), [Edge(3, "dense", _w(r_w, 3, 5))], relu=False)
    net = Net((6,), [n0, n1, n2, n3, out])
    x0 = r_x.random(6)
    return gen.make_problem(f"dag-{kind}", net, x0, 0.1, None, 4, 1, 2, 6, 2, 4, (r_cut, r_split, r_par),
                            alpha_init="given", gamma_dist="uniform", input_terms=1)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("kind,seed", [("two_identity", 1), ("two_identity", 2), ("identity_dense", 3),
                                       ("identity_dense", 4)])
def test_dag_bound_and_gradients_match_oracle(kind, seed, mode):
    import torch
    from paper_2208_05740_amd import binding as B
    print(f"DAG {kind} seed={seed} mode={mode}", flush=True)
    prob = _dag(kind, seed)
    P = B.Problem(prob, device=_dev())
    t = lambda x: torch.tensor(np.asarray(x, np.float32).reshape(P.M, -1), device=_dev())  # noqa: E731
    a, b, c = t(O.full_alpha(prob)), t(prob.beta), t(prob.gamma)
    out, ver, g = B.bound(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a, b, c, mode=mode, grads=True,
                          verified=True)
    torch.cuda.synchronize()
    f = lambda x: x.cpu().numpy().astype(np.float64).reshape(prob.B, prob.S, -1)  # noqa: E731
    ref, ga, gb, gc = O.bound_and_grad(prob, f(a), f(b), f(c))
    ref = ref.reshape(-1)
    T = O.error_scale(prob, f(a), f(b), f(c)).reshape(-1)
    got = out.cpu().numpy()
    err = np.abs(got - ref) / np.maximum(np.abs(ref), T)
    print(f"  max rel err {err.max():.2e}", flush=True)
    assert err.max() <= (2e-2 if mode else 1e-5), err.max()
    assert np.array_equal(ver.cpu().numpy(), (got >= 0).astype(np.uint8))
    if mode == 0:
        for gg, want in zip(g, (ga, gb, gc)):
            want = want.reshape(prob.B * prob.S, -1)
            if want.size == 0:
                continue
            d = np.abs(gg.cpu().numpy().reshape(want.shape) - want) / (np.abs(want).max(1, keepdims=True) + 1.0)
            assert d.max() <= 1e-4, d.max()
