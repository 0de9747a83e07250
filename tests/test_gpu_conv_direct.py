"""The direct transposed convolution of the concretisation over the input
(Theorem 3.1's input term through a conv edge: a_hat over the input is
Lambda of the first conv node times the conv's matrix, then the box is
concretised and the input cuts' G terms are added) against the FP64 oracle
and against the MFMA slab kernel, through the C ABI.

The direct kernel applies where the input has at most four channels and a
stride phase has 2x2 or 3x3 taps.  Both kernels are selected from the host:
with autotuning off and an empty tile cache the direct kernel is the default
launch where it applies; GCP_CONV_DIRECT=0 leaves it out.  The library's
event profiler names the launch that ran.

Cases: single-channel tiny networks (3x3 stride 2, 4x4 stride 2 and 3x3
stride 1 stems; input cuts, so the epilogue's cut terms and gamma-gradient
pieces are live), 2- and 4-channel tiny networks (every channel count the
kernel is built for; rows of whole and of partial staging vectors), the
3x32x32 CNN stem (4x4 stride 2, two row bands) and the ResNet stem (3x3
stride 1, three bands), with batch rows that leave a ragged last group of
four.  Tolerances are those of the other parity tests: FP32
bound within 1e-5 of max(|g|, T) of the oracle (T the sum of the magnitudes
of the terms added), gradients within 1e-4 of the row's largest, bf16
within 2e-2 of T.  Direct and slab results differ only in the order of the
fp32 sums of each a_hat element.
"""
import contextlib
import os

import numpy as np
import pytest

from oracle import gcp_oracle as O
from workloads import gen

pytestmark = pytest.mark.gpu


def _dev():
    import torch
    return torch.device("cuda:0")


@contextlib.contextmanager
def _conc_kernel(which, tmp_path):
    saved = {k: os.environ.get(k) for k in ("GCP_TILE_CACHE", "GCP_AUTOTUNE", "GCP_CONV_DIRECT")}
    cache = tmp_path / f"tiles_{which}.txt"
    cache.write_text("")
    os.environ["GCP_TILE_CACHE"] = str(cache)
    os.environ["GCP_AUTOTUNE"] = "0"
    if which == "slab":
        os.environ["GCP_CONV_DIRECT"] = "0"
    else:
        os.environ.pop("GCP_CONV_DIRECT", None)
    try:
        yield
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _bound(prob, mode, which, tmp_path):
    """gcp_bound with gradients on a fresh upload (so no plan is reused),
    with the chosen concretisation kernel; returns numpy results and the
    kernel classes that ran."""
    import torch
    from paper_2208_05740_amd import binding as B
    with _conc_kernel(which, tmp_path):
        P = B.Problem(prob, device=_dev())
        t = lambda x: torch.tensor(np.asarray(x, np.float32).reshape(P.M, -1), device=_dev())  # noqa: E731
        a, b, c = t(O.full_alpha(prob)), t(prob.beta), t(prob.gamma)
        B.profile_enable(True)
        out, ver, g = B.bound(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, a, b, c, mode=mode, grads=True,
                              verified=True)
        torch.cuda.synchronize()
        B.profile_enable(False)
        ran = {k for k, v in B.profile_read().items() if v["launches"]}
    n = lambda x: x.cpu().numpy()  # noqa: E731
    return dict(bound=n(out), ver=n(ver), grads=[n(x) for x in g], a=a, b=b, c=c), ran


def _multichannel(seed, in_shape, stem):
    """A small conv net on a multi-channel input: the stem conv (c_out, k,
    stride, pad), a 3x3 conv, dense 5, out 3; splits, cuts and input cuts."""
    r_w, r_x, r_cut, r_split, r_par = gen._streams([seed, 98])
    net = gen.cnn_net(r_w, in_shape, (stem, (3, 3, 1, 1)), (5, 3))
    x0 = r_x.random(net.in_size)
    return gen.make_problem(f"tiny-c{in_shape[0]}", net, x0, 0.1, None, 3, 1, 2, 5, 2, 4, (r_cut, r_split, r_par),
                            alpha_init="given", gamma_dist="uniform", input_terms=1)


CASES = [
    ("tiny", "cnn", 1, dict(B=5, splits=(1, 3), n_cuts=6, input_terms=1)),     # 1x6x6, 3x3 s2
    ("tiny", "cnn16", 2, dict(B=3, splits=(1, 2), n_cuts=6, input_terms=1)),   # 1x8x8, 4x4 s2
    ("tiny", "res", 3, dict(B=2, splits=(1, 2), n_cuts=5, input_terms=1)),     # 1x4x4, 3x3 s1
    ("tiny", "res16", 4, dict(B=3, splits=(0, 0), n_cuts=0)),                  # no cuts, no splits
    ("cnn", None, 0, dict(B=3)),       # 3x32x32, 4x4 s2: 27 rows, a ragged group of four
    ("resnet", None, 0, dict(B=1)),    # 3x32x32, 3x3 s1
    ("multi", (2, 7, 7), 5, (3, 4, 2, 1)),   # 2 channels, 4x4 s2, rows of 3 (element-wise staging)
    ("multi", (2, 8, 8), 6, (3, 4, 2, 1)),   # 2 channels, 4x4 s2, rows of 4
    ("multi", (4, 6, 6), 7, (2, 3, 1, 1)),   # 4 channels, 3x3 s1
]


def _problem(which, kind, seed, kw):
    if which == "tiny":
        return gen.make_tiny(kind, seed, **kw)
    if which == "multi":
        return _multichannel(seed, kind, kw)
    return gen.make_workload(which, seed, **kw)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_direct_conc_matches_oracle_and_slab(case, tmp_path):
    which, kind, seed, kw = CASES[case]
    print(f"direct transposed conv: {which} {kind} seed={seed} {kw}", flush=True)
    prob = _problem(which, kind, seed, kw)
    got, ran = _bound(prob, 0, "direct", tmp_path)
    assert "convT_conc.fp32.direct" in ran, sorted(ran)
    ref_s, ran_s = _bound(prob, 0, "slab", tmp_path)
    assert "convT_conc.fp32" in ran_s and "convT_conc.fp32.direct" not in ran_s, sorted(ran_s)

    f = lambda x: x.cpu().numpy().astype(np.float64).reshape(prob.B, prob.S, -1)  # noqa: E731
    a, b, c = f(got["a"]), f(got["b"]), f(got["c"])
    ref, ga, gb, gc = O.bound_and_grad(prob, a, b, c)
    ref = ref.reshape(-1)
    T = O.error_scale(prob, a, b, c).reshape(-1)
    for name, res in (("direct", got), ("slab", ref_s)):
        err = np.abs(res["bound"] - ref) / np.maximum(np.abs(ref), T)
        print(f"  {name}: max rel err {err.max():.2e}", flush=True)
        assert err.max() <= 1e-5, (name, err.max())
        assert np.array_equal(res["ver"], (res["bound"] >= 0).astype(np.uint8))
        for gg, want in zip(res["grads"], (ga, gb, gc)):
            want = want.reshape(prob.B * prob.S, -1)
            if want.size == 0:
                continue
            d = np.abs(gg.reshape(want.shape) - want) / (np.abs(want).max(1, keepdims=True) + 1.0)
            assert d.max() <= 1e-4, (name, d.max())
    # the two kernels against each other, at the same tolerance
    err = np.abs(got["bound"] - ref_s["bound"]) / np.maximum(np.abs(ref_s["bound"]), T)
    assert err.max() <= 1e-5, err.max()


@pytest.mark.parametrize("case", [0, 4, 7])
def test_direct_conc_bf16_close_to_oracle(case, tmp_path):
    which, kind, seed, kw = CASES[case]
    print(f"direct transposed conv, bf16: {which} {kind} seed={seed} {kw}", flush=True)
    prob = _problem(which, kind, seed, kw)
    got, ran = _bound(prob, 1, "direct", tmp_path)
    assert "convT_conc.bf16.direct" in ran, sorted(ran)
    f = lambda x: x.cpu().numpy().astype(np.float64).reshape(prob.B, prob.S, -1)  # noqa: E731
    a, b, c = f(got["a"]), f(got["b"]), f(got["c"])
    ref = O.bound(prob, a, b, c).reshape(-1)
    T = O.error_scale(prob, a, b, c).reshape(-1)
    err = np.abs(got["bound"] - ref) / np.maximum(np.abs(ref), T)
    print(f"  max rel err {err.max():.2e}", flush=True)
    assert err.max() <= 2e-2, err.max()
