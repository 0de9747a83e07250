"""The persistent dataflow optimisation (GCP_FLAG_PERSIST: every Adam
iteration in one launch whose workgroups claim (iteration, step, row panel,
column tile) items and wait per panel for the steps before) against the
per-layer launches, through the C ABI.

Each (domain, spec row) of Theorem 3.1 is an independent problem, so the
dataflow order changes nothing in the arithmetic: every item runs the
per-layer kernels' epilogue code on accumulators that every tile shape sums
over K in the same order.  The final parameters, Adam moments and certified
bounds of the 20-iteration optimisation (Appendix C.1) must therefore be
bit-identical to the per-layer launches, on the first call of an argument
set (one eager iteration, then the launch) and on a repeated call (all
iterations in the launch), with either ordering protocol between
workgroups: the default one (one claim queue per XCD, so a producer's stores
need only reach the L2 its consumers share) and agent-scope fences.  The per-layer launches are checked against the FP64 oracle
elsewhere; the certified bound of a persistent run is checked against the
oracle here too.
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


class _Run:
    """Parameters on the device, reset to the same start before every call
    (the same pointers each time, so a repeated call finds its cached plan)."""

    def __init__(self, prob, P):
        import torch
        from paper_2208_05740_amd import binding as B
        M = P.M
        self.prob, self.P = prob, P
        self.a0 = torch.tensor(np.asarray(O.full_alpha(prob), np.float32).reshape(M, -1), device=_dev())
        self.b0 = torch.tensor(np.asarray(prob.beta, np.float32).reshape(M, -1), device=_dev())
        self.c0 = torch.tensor(np.asarray(prob.gamma, np.float32).reshape(M, -1), device=_dev())
        self.a, self.b, self.c = self.a0.clone(), self.b0.clone(), self.c0.clone()
        self.st = torch.zeros(B.adam_state_size(M, P.n_I, P.K, P.N), dtype=torch.float32, device=_dev())

    def __call__(self, mode, persist, sync="default"):
        import torch
        from paper_2208_05740_amd import binding as B
        P, o = self.P, self.prob.opt
        self.a.copy_(self.a0)
        self.b.copy_(self.b0)
        self.c.copy_(self.c0)
        self.st.zero_()
        if sync != "default":
            os.environ["GCP_PERSIST_SYNC"] = sync
        try:
            B.profile_enable(True)
            out, ver = B.optimize(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, self.a, self.b, self.c, self.st,
                                  iters=o["iters"], lr_alpha=o["lr_alpha"], lr_mult=o["lr_mult"], decay=o["decay"],
                                  mode=mode | (B.GCP_FLAG_PERSIST if persist else 0))
            torch.cuda.synchronize()
            B.profile_enable(False)
            ran = {k for k, v in B.profile_read().items() if v["launches"]}
        finally:
            os.environ.pop("GCP_PERSIST_SYNC", None)
        n = lambda t: t.cpu().numpy()  # noqa: E731
        return dict(bound=n(out), ver=n(ver), alpha=n(self.a), beta=n(self.b), gamma=n(self.c), state=n(self.st)), ran


CASES = [
    ("tiny", dict(kind="mlp", seed=1, B=5, splits=(1, 3), n_cuts=6, input_terms=1)),
    ("tiny", dict(kind="mlp", seed=7, B=3, splits=(0, 0), n_cuts=0)),
    ("mlp784", dict(B=5)),          # 45 rows: one full panel and a ragged one
    ("mlp784", dict(B=37)),         # 333 rows over 11 panels, fewer than the claim queues on some
    ("mlp784", dict(B=1024)),       # the benchmark's 9216 rows
]


def _problem(which, kw):
    if which == "tiny":
        kw = dict(kw)
        kind, seed = kw.pop("kind"), kw.pop("seed")
        return gen.make_tiny(kind, seed, **kw)
    return gen.make_workload(which, 0, **kw)


def _same(got, ref):
    for k in ref:
        same = np.array_equal(got[k], ref[k])
        if not same:
            d = np.abs(got[k].astype(np.float64) - ref[k].astype(np.float64))
            print(f"  {k}: max |diff| {d.max():.3e} at {np.unravel_index(d.argmax(), d.shape)}", flush=True)
        assert same, k


@pytest.mark.parametrize("sync", ["default", "agent"])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_persistent_launch_equals_per_layer_launches(case, mode, sync):
    from paper_2208_05740_amd import binding as B
    which, kw = CASES[case]
    print(f"persistent vs per-layer: {which} {kw} mode={mode} sync={sync}", flush=True)
    prob = _problem(which, kw)
    P = B.Problem(prob, device=_dev())
    run = _Run(prob, P)
    ref, ran_ref = run(mode, persist=False)
    tag = "persist." + ("bf16" if mode else "fp32")
    for call in ("first", "repeated"):
        got, ran = run(mode, persist=True, sync=sync)
        print(f"  {call} call", flush=True)
        assert tag in ran and tag not in ran_ref, (sorted(ran), sorted(ran_ref))
        _same(got, ref)


def test_persistent_certified_bound_matches_oracle():
    from paper_2208_05740_amd import binding as B
    print("persistent certified bound vs oracle", flush=True)
    prob = gen.make_tiny("mlp", 2, B=6, splits=(1, 3), n_cuts=6, input_terms=1)
    P = B.Problem(prob, device=_dev())
    got, ran = _Run(prob, P)(0, persist=True)
    assert "persist.fp32" in ran
    f = lambda x: x.astype(np.float64).reshape(prob.B, prob.S, -1)  # noqa: E731
    ref = O.bound(prob, f(got["alpha"]), f(got["beta"]), f(got["gamma"])).reshape(-1)
    T = O.error_scale(prob, f(got["alpha"]), f(got["beta"]), f(got["gamma"])).reshape(-1)
    err = np.abs(got["bound"] - ref) / np.maximum(np.abs(ref), T)
    assert err.max() <= 1e-5, err.max()


def test_persistent_flag_ignored_where_the_schedule_is_not_dense():
    """A CNN's conv edges are not in the persistent kernel's step kinds: the
    flag falls back to the per-layer launches with identical results."""
    from paper_2208_05740_amd import binding as B
    print("persistent flag on a CNN", flush=True)
    prob = gen.make_tiny("cnn", 3, B=2, splits=(1, 2), n_cuts=4)
    P = B.Problem(prob, device=_dev())
    run = _Run(prob, P)
    ref, _ = run(0, persist=False)
    got, ran = run(0, persist=True)
    assert "persist.fp32" not in ran
    _same(got, ref)


@pytest.mark.parametrize("mode", [0, 1])
def test_batch_in_one_persistent_launch_equals_per_instance(mode):
    """gcp_optimize_batch with GCP_FLAG_PERSIST: every instance of an uneven
    batch (depth, width, input size, domains, cuts differ) runs its
    iterations in one persistent launch, eagerly and as a replayed captured
    graph, on the first and on repeated calls; bounds, parameters and the
    multipliers must equal one gcp_optimize per instance bit for bit."""
    import torch
    from paper_2208_05740_amd import binding as B
    from test_gpu_parity import _batch_items, _optimize, upload
    print(f"batch in one persistent launch, mode={mode}", flush=True)
    probs = gen.make_batch(seed=3, n_inst=5, bmax=24)
    Ps = [upload(p) for p in probs]
    o = probs[0].opt
    for p, P in zip(probs, Ps):   # fp32 data in the padding shared by both precisions, as the batch tests do
        _optimize(p, P, 0, iters=1)
    ref = []
    for p, P in zip(probs, Ps):
        g, a, b, c = _optimize(p, P, mode)
        ref.append((g, a.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()))
    for graph in (False, True, True):
        items = _batch_items(probs, Ps)
        B.profile_enable(True)
        B.optimize_batch(items, iters=o["iters"], lr_alpha=o["lr_alpha"], lr_mult=o["lr_mult"], decay=o["decay"],
                         mode=mode | B.GCP_FLAG_PERSIST, use_graph=graph)
        torch.cuda.synchronize()
        B.profile_enable(False)
        ran = {k for k, v in B.profile_read().items() if v["launches"]}
        print(f"  graph={graph}", flush=True)
        if not graph:
            assert ("persist." + ("bf16" if mode else "fp32")) in ran, sorted(ran)
        for it, (g, a, b, c) in zip(items, ref):
            assert np.array_equal(it["bound"].cpu().numpy(), g)
            assert np.array_equal(it["alpha"].cpu().numpy(), a)
            assert np.array_equal(it["beta"].cpu().numpy(), b)
            assert np.array_equal(it["gamma"].cpu().numpy(), c)


def test_persistent_wait_limit_ends_the_launch_with_sound_bounds(monkeypatch):
    """The bounded wait's exit path, forced from the host: with a spin limit
    of one wall-clock tick every wait that is not met at once aborts the
    launch (every workgroup stops; nothing hangs), and the certifying pass's
    bounds are then replaced by -inf, a valid lower bound, with no row
    verified.  If no item had to wait, the results are the ordinary ones."""
    import torch
    from paper_2208_05740_amd import binding as B
    print("persistent launch abort path (spin limit 1 tick)", flush=True)
    prob = gen.make_workload("mlp784", 0, B=64)
    P = B.Problem(prob, device=_dev())
    run = _Run(prob, P)
    ref, _ = run(0, persist=False)
    run(0, persist=True)                      # builds the plan with the ordinary limit
    monkeypatch.setenv("GCP_PERSIST_SPIN_TICKS", "1")
    got, ran = run(0, persist=True)           # every iteration in the persistent launch
    torch.cuda.synchronize()
    assert "persist.fp32" in ran
    aborted = bool(np.all(np.isneginf(got["bound"])))
    print(f"  aborted: {aborted}", flush=True)
    if aborted:
        assert not got["ver"].any()
    else:
        _same(got, ref)
    monkeypatch.delenv("GCP_PERSIST_SPIN_TICKS")
    again, _ = run(0, persist=True)           # the next call starts from a clear latch
    _same(again, ref)


def test_full_size_batch_in_one_persistent_launch_equals_grouped_launches():
    """The 64 uneven MLP instances (42,144 domains) as the benchmark runs
    them: in one persistent launch (GCP_FLAG_PERSIST) the final bounds and
    parameters equal, bit for bit, those of the default launches (small
    instances grouped, large ones alone on side streams)."""
    import torch
    from paper_2208_05740_amd import binding as B
    print("full-size batch: persistent launch vs grouped launches", flush=True)
    probs = gen.make_batch(seed=0)
    Ps = [B.Problem(p, device=_dev()) for p in probs]
    o = probs[0].opt
    a0 = [torch.tensor(gen.crown_alpha_init(p.lu), dtype=torch.float32, device=_dev()).expand(P.M, -1).contiguous()
          for p, P in zip(probs, Ps)]
    items = [dict(P=P, alpha=torch.empty_like(a), beta=torch.empty(P.M, P.K, dtype=torch.float32, device=_dev()),
                  gamma=torch.empty(P.M, P.N, dtype=torch.float32, device=_dev()),
                  state=torch.empty(B.adam_state_size(P.M, P.n_I, P.K, P.N), dtype=torch.float32, device=_dev()),
                  bound=torch.empty(P.M, dtype=torch.float64, device=_dev()),
                  verified=torch.empty(P.M, dtype=torch.uint8, device=_dev())) for P, a in zip(Ps, a0)]

    def run(flags):
        for p, it, a in zip(probs, items, a0):
            it["alpha"].copy_(a)
            it["beta"].copy_(torch.tensor(p.beta.reshape(it["P"].M, -1), dtype=torch.float32))
            it["gamma"].zero_()
            it["state"].zero_()
        B.optimize_batch(items, iters=o["iters"], lr_alpha=o["lr_alpha"], lr_mult=o["lr_mult"], decay=o["decay"],
                         b1=o["adam_b1"], b2=o["adam_b2"], adam_eps=o["adam_eps"], mode=flags)
        torch.cuda.synchronize()
        return [{k: it[k].cpu().numpy() for k in ("bound", "alpha", "beta", "gamma")} for it in items]

    ref = run(B.GCP_MODE_FP32)
    got = run(B.GCP_MODE_FP32 | B.GCP_FLAG_PERSIST)
    for i, (g, r) in enumerate(zip(got, ref)):
        for k in r:
            assert np.array_equal(g[k], r[k]), (i, probs[i].name, k)
