"""The fused dense-chain optimisation (every Adam iteration of an MLP in one
launch, Lambda and d a_hat kept in LDS) against the per-layer launches,
through the C ABI.

The fused kernel runs the per-layer kernels' own epilogue code, and each of
its GEMMs accumulates over K in the same order with the same MFMA
instructions, so the whole 20-iteration optimisation (Theorem 3.1's bound,
its adjoint, Appendix C.1's projected Adam) must give bit-identical final
parameters, Adam moments and certified bounds.  The per-layer launches
themselves are checked against the FP64 oracle elsewhere; the certified
bound of the fused run is checked against the oracle here too.
"""
import os

import numpy as np
import pytest

from oracle import gcp_oracle as O
from workloads import gen

pytestmark = pytest.mark.gpu


def _dev():
    import torch
    return torch.device("cuda:0")


def _run(prob, P, mode, fused, iters=None):
    import torch
    from paper_2208_05740_amd import binding as B
    os.environ["GCP_FUSED"] = "1" if fused else "0"
    try:
        M = P.M
        a = torch.tensor(np.asarray(O.full_alpha(prob), np.float32).reshape(M, -1), device=_dev())
        b = torch.tensor(np.asarray(prob.beta, np.float32).reshape(M, -1), device=_dev())
        c = torch.tensor(np.asarray(prob.gamma, np.float32).reshape(M, -1), device=_dev())
        st = torch.zeros(B.adam_state_size(M, P.n_I, P.K, P.N), dtype=torch.float32, device=_dev())
        o = prob.opt
        B.profile_enable(True)
        out, ver = B.optimize(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a, b, c, st,
                              iters=o["iters"] if iters is None else iters, lr_alpha=o["lr_alpha"],
                              lr_mult=o["lr_mult"], decay=o["decay"], mode=mode)
        torch.cuda.synchronize()
        B.profile_enable(False)
        ran = {k for k, v in B.profile_read().items() if v["launches"]}
    finally:
        os.environ.pop("GCP_FUSED", None)
    n = lambda t: t.cpu().numpy()  # noqa: E731
    return dict(bound=n(out), ver=n(ver), alpha=n(a), beta=n(b), gamma=n(c), state=n(st)), ran


CASES = [
    ("tiny", dict(kind="mlp", seed=1, B=5, splits=(1, 3), n_cuts=6, input_terms=1)),
    ("tiny", dict(kind="mlp", seed=7, B=3, splits=(0, 0), n_cuts=0)),
    ("mlp784", dict(B=5)),
    ("mlp784", dict(B=1024)),
]


def _problem(which, kw):
    if which == "tiny":
        kw = dict(kw)
        kind, seed = kw.pop("kind"), kw.pop("seed")
        return gen.make_tiny(kind, seed, **kw)
    return gen.make_workload(which, 0, **kw)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_fused_chain_equals_per_layer_launches(case, mode):
    from paper_2208_05740_amd import binding as B
    which, kw = CASES[case]
    print(f"fused chain vs per-layer: {which} {kw} mode={mode}", flush=True)
    prob = _problem(which, kw)
    P = B.Problem(prob, device=_dev())
    ref, ran_ref = _run(prob, P, mode, fused=False)
    got, ran = _run(prob, P, mode, fused=True)
    tag = "chain." + ("bf16" if mode else "fp32")
    assert tag in ran and tag not in ran_ref, (sorted(ran), sorted(ran_ref))
    for k in ref:
        same = np.array_equal(got[k], ref[k])
        if not same:
            d = np.abs(got[k].astype(np.float64) - ref[k].astype(np.float64))
            print(f"  {k}: max |diff| {d.max():.3e} at {np.unravel_index(d.argmax(), d.shape)}", flush=True)
        assert same, k


def test_fused_chain_certified_bound_matches_oracle():
    from paper_2208_05740_amd import binding as B
    print("fused chain certified bound vs oracle", flush=True)
    prob = gen.make_tiny("mlp", 2, B=6, splits=(1, 3), n_cuts=6, input_terms=1)
    P = B.Problem(prob, device=_dev())
    got, ran = _run(prob, P, 0, fused=True)
    assert "chain.fp32" in ran
    f = lambda x: x.astype(np.float64).reshape(prob.B, prob.S, -1)  # noqa: E731
    ref = O.bound(prob, f(got["alpha"]), f(got["beta"]), f(got["gamma"])).reshape(-1)
    T = O.error_scale(prob, f(got["alpha"]), f(got["beta"]), f(got["gamma"])).reshape(-1)
    err = np.abs(got["bound"] - ref) / np.maximum(np.abs(ref), T)
    assert err.max() <= 1e-5, err.max()
    go, *_ = O.optimize(prob)
    To = O.error_scale(prob).reshape(-1)
    assert (np.abs(got["bound"] - go.reshape(-1)) / np.maximum(np.abs(go.reshape(-1)), To)).max() <= 1e-3
