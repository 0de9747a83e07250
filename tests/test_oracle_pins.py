"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names what it checks and why a plausible mistake in the oracle
would fail it:
  * Lemma A.1 by brute-force 1-D maximisation (wrong sign in pi*, wrong h
    case, swapped l/u);
  * the beta = gamma = 0 case equals textbook CROWN in primal form
    (Proposition 3.2; wrong slope, intercept, bias sign, concretisation);
  * weak duality g <= f*_LP-cut <= f*_MIP <= sampled minimum (Theorem 3.1
    soundness; any term with a wrong sign or a dropped cut term breaks it
    for some random multipliers);
  * optimised alpha reaches the Planet LP optimum (strong duality of the
    cut-free LP, so the whole recursion is tight, not merely sound);
  * splits passed as beta equal the same constraints passed as cut rows
    (the split special case of Sec. 3.1);
  * the oracle's gradient equals central finite differences;
  * the conv adjoint equals the explicit matrix transpose;
  * the Adam step equals torch.optim.Adam (maximize) plus projection.
"""
import numpy as np
import pytest
import torch

from oracle import crown, gcp_oracle as O, lp
from workloads import gen


# ---------------------------------------------------------------- Lemma A.1

def _brute_h(l, u, C, s, n=20001):
    # max over pi in [0, C] of  l pi - ReLU(u (C - pi) + l pi - s)
    pi = np.linspace(0.0, C, n)
    f = l * pi - np.maximum(u * (C - pi) + l * pi - s, 0.0)
    k = int(np.argmax(f))
    # refine: the function is concave piecewise linear; check the kink too
    cands = [pi[k]]
    if u - l != 0:
        cands.append(np.clip((u * C - s) / (u - l), 0.0, C))
    return max(l * p - max(u * (C - p) + l * p - s, 0.0) for p in cands)


def test_lemma_closed_form_matches_brute_force():
    rng = np.random.default_rng(1)
    for _ in range(3000):
        l = -rng.exponential(1.0)
        u = rng.exponential(1.0)
        C = rng.exponential(1.0) * (rng.random() < 0.9)
        s = rng.normal() * 2.0
        a_hat = torch.tensor([-C], dtype=torch.float64)
        pi, h = O.unstable_pi_h(a_hat, torch.tensor([s], dtype=torch.float64),
                                torch.tensor([l], dtype=torch.float64),
                                torch.tensor([u], dtype=torch.float64))
        hb = _brute_h(l, u, C, s)
        assert abs(h.item() - hb) <= 1e-9 * (1 + abs(hb)), (l, u, C, s, h.item(), hb)
        assert -1e-12 <= pi.item() <= C + 1e-12
        # the closed-form pi* attains h
        p = pi.item()
        assert abs(l * p - max(u * (C - p) + l * p - s, 0.0) - h.item()) < 1e-9


def test_lemma_printed_plus_sign_would_be_unsound():
    # The theorem as printed has +beta^T Q in pi*; with it the inner maximum
    # is overstated for some inputs, which the brute force exposes.  This
    # guards the sign reading the oracle uses.
    rng = np.random.default_rng(2)
    worst = 0.0
    for _ in range(2000):
        l, u, C, s = -rng.exponential(), rng.exponential(), rng.exponential(), rng.normal() * 2
        p = np.clip((u * C + s) / (u - l), 0.0, C)
        val = l * p - max(u * (C - p) + l * p - s, 0.0)
        worst = max(worst, val - _brute_h(l, u, C, s))
    assert worst <= 1e-9   # plugging any feasible pi is never above the max ...
    # ... but the printed case formula for h (l * pi with the '+' pi) is:
    bad = 0
    for _ in range(2000):
        l, u, C, s = -rng.exponential(), rng.exponential(), rng.exponential(), rng.normal() * 2
        if l * C <= s <= u * C:
            p = np.clip((u * C + s) / (u - l), 0.0, C)
            if l * p > _brute_h(l, u, C, s) + 1e-9:
                bad += 1
    assert bad > 0


# -------------------------------------------------- CROWN special case (T2)

@pytest.mark.parametrize("kind,seed", [("mlp", 0), ("mlp", 3), ("cnn", 1), ("res", 2)])
def test_zero_multipliers_equal_textbook_crown(kind, seed):
    p = gen.make_tiny(kind, seed, B=1, splits=(0, 0), n_cuts=3)
    prep = O.Prepared(p)
    a = O.full_alpha(p, prep)
    g = O.bound(p, a, p.beta, np.zeros_like(p.gamma), prep=prep)
    for s in range(p.S):
        apn = []
        for q in prep.relu:
            full = np.zeros(p.net.nodes[q].size)
            full[prep.unst_cols[q]] = a[0, s, prep.alpha_pos[q]]
            apn.append(full)
        ref = crown.crown_bound(p.net, p.lu, p.x0, p.eps, p.C[s], apn)
        assert abs(g[0, s] - ref) <= 1e-10 * (1 + abs(ref))


def test_mlp8_zero_gamma_equals_crown():
    p = gen.make_workload("mlp8", 0)
    prep = O.Prepared(p)
    a = O.full_alpha(p, prep)
    g = O.bound(p, a, p.beta, np.zeros_like(p.gamma), prep=prep)
    for s in range(p.S):
        apn = []
        for q in prep.relu:
            full = np.zeros(p.net.nodes[q].size)
            full[prep.unst_cols[q]] = a[0, s, prep.alpha_pos[q]]
            apn.append(full)
        assert abs(g[0, s] - crown.crown_bound(p.net, p.lu, p.x0, p.eps, p.C[s], apn)) < 1e-10


# ------------------------------------------------------ weak duality (T4)

def _random_params(p, rng, scale=1.0):
    prep = O.Prepared(p)
    a = rng.random((p.B, p.S, prep.n_I))
    b = rng.random((p.B, p.S, p.splits.K)) * scale * (p.splits.node >= 0)[:, None, :]
    c = rng.random((p.B, p.S, p.cuts.n)) * scale
    return a, b, c


@pytest.mark.parametrize("kind,seed", [("mlp", 0), ("mlp", 5), ("cnn", 1), ("res", 2)])
def test_bound_below_lp_mip_and_samples(kind, seed):
    p = gen.make_tiny(kind, seed, B=3, splits=(1, 2), n_cuts=5, input_terms=1)
    rng = np.random.default_rng(seed)
    lpv = np.array([[lp.lp_value(p, b, s) for s in range(p.S)] for b in range(p.B)])
    mip = np.array([[lp.mip_value(p, b, s) for s in range(p.S)] for b in range(p.B)])
    smp = np.array([lp.sampled_min(p, b, n=20000, seed=seed) for b in range(p.B)])
    assert np.all(lpv <= mip + 1e-7)
    assert np.all(mip <= smp + 1e-7)
    for trial in range(20):
        a, b, c = _random_params(p, rng, scale=[0.0, 0.1, 1.0, 5.0][trial % 4])
        g = O.bound(p, a, b, c)
        assert np.all(g <= lpv + 1e-8), (g, lpv)


def test_mlp8_tight_cuts_bound_below_lp_and_enumerated_mip():
    p = gen.make_workload("mlp8", 0)
    # tighten every cut to the MIP maximum of its left side (still valid)
    p.cuts.d[:] = [lp.cut_max(p, k) for k in range(p.cuts.n)]
    rng = np.random.default_rng(7)
    lpv = np.array([lp.lp_value(p, 0, s) for s in range(p.S)])
    enum = np.array([lp.mip_value_enum(p, 0, s) for s in range(p.S)])
    mip = np.array([lp.mip_value(p, 0, s) for s in range(p.S)])
    smp = lp.sampled_min(p, 0, n=100000)
    assert np.allclose(enum, mip, atol=1e-7)
    assert np.all(lpv <= enum + 1e-8) and np.all(enum <= smp + 1e-8)
    for trial in range(40):
        a, b, c = _random_params(p, rng, scale=[0.0, 0.3, 1.0, 3.0][trial % 4])
        assert np.all(O.bound(p, a, b, c) <= lpv + 1e-8)


# ------------------------------------------- tightness: Planet LP optimum (T5)

@pytest.mark.slow
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_optimised_alpha_reaches_planet_lp(seed):
    p = gen.make_tiny("mlp", seed, B=1, splits=(0, 0), n_cuts=0)
    lpv = np.array([lp.lp_value(p, 0, s) for s in range(p.S)])
    g, a, _, _ = O.optimize(p, iters=400, opt=dict(decay=0.995, lr_alpha=0.05))
    assert np.all(g <= lpv + 1e-9)
    assert np.all(lpv - g <= 1e-4 * (1 + np.abs(lpv))), (g, lpv)


# ------------------------------------------- splits as special cuts (T3)

@pytest.mark.parametrize("kind", ["mlp", "cnn"])
def test_splits_equal_cut_encoding(kind):
    p = gen.make_tiny(kind, 4, B=3, splits=(1, 3), n_cuts=3)
    rng = np.random.default_rng(0)
    a, b, c = _random_params(p, rng)
    g = O.bound(p, a, b, c)
    # same splits (class override) with zero beta, plus one cut row per
    # (domain, slot): x_j <= 0 -> H_jj = +1, x_j >= 0 -> H_jj = -1, d = 0,
    # whose multiplier is that domain's beta (zero for other domains).
    sp = p.splits
    extra = [(b_, k) for b_ in range(p.B) for k in range(sp.K) if sp.node[b_, k] >= 0]
    cu = p.cuts
    N0 = cu.n
    cut = list(cu.cut); node = list(cu.node); neu = list(cu.neuron)
    kind_ = list(cu.kind); coef = list(cu.coef)
    for i, (b_, k) in enumerate(extra):
        cut.append(N0 + i); node.append(sp.node[b_, k]); neu.append(sp.neuron[b_, k])
        kind_.append(gen.KIND_H); coef.append(-1.0 if sp.sign[b_, k] > 0 else 1.0)
    p2 = gen.Problem(p.name, p.net, p.lu, p.x0, p.eps, p.C, sp,
                     gen.Cuts(N0 + len(extra), np.array(cut, np.int32), np.array(node, np.int32),
                              np.array(neu, np.int32), np.array(kind_, np.int8), np.array(coef),
                              np.concatenate([cu.d, np.zeros(len(extra))])),
                     "given", a, np.zeros_like(b), None)
    c2 = np.concatenate([c, np.zeros((p.B, p.S, len(extra)))], axis=2)
    for i, (b_, k) in enumerate(extra):
        c2[b_, :, N0 + i] = b[b_, :, k]
    g2 = O.bound(p2, a, np.zeros_like(b), c2)
    assert np.allclose(g, g2, rtol=0, atol=1e-10)


def test_no_cuts_is_beta_crown():
    # With no cut rows the bound is the beta-CROWN bound: identical to the
    # same problem with every gamma at zero.
    p = gen.make_tiny("mlp", 2, B=2, splits=(1, 2), n_cuts=4)
    rng = np.random.default_rng(3)
    a, b, c = _random_params(p, rng)
    p0 = gen.Problem(p.name, p.net, p.lu, p.x0, p.eps, p.C, p.splits, gen.Cuts.empty(),
                     "given", a, b, np.zeros((p.B, p.S, 0)))
    assert np.allclose(O.bound(p0, a, b, np.zeros((p.B, p.S, 0))),
                       O.bound(p, a, b, np.zeros_like(c)), atol=1e-12)


# ------------------------------------------------- gradient vs FD (T6)

@pytest.mark.parametrize("kind,seed", [("mlp", 0), ("cnn", 1), ("res", 2)])
def test_gradient_matches_finite_differences(kind, seed):
    p = gen.make_tiny(kind, seed, B=2, splits=(1, 2), n_cuts=5, input_terms=1)
    rng = np.random.default_rng(seed)
    a, b, c = _random_params(p, rng, scale=0.5)
    g, ga, gb, gc = O.bound_and_grad(p, a, b, c)
    h = 1e-6
    checked = 0
    for arr, grad in ((a, ga), (b, gb), (c, gc)):
        flat = arr.reshape(-1)
        for idx in rng.choice(flat.size, size=min(flat.size, 25), replace=False) if flat.size else []:
            x = arr.copy().reshape(-1)
            x[idx] += h
            gp = O.bound(p, *[x.reshape(arr.shape) if y is arr else y for y in (a, b, c)])
            x[idx] -= 2 * h
            gm = O.bound(p, *[x.reshape(arr.shape) if y is arr else y for y in (a, b, c)])
            fd = (gp - gm).sum() / (2 * h)
            an = grad.reshape(-1)[idx]
            assert abs(fd - an) <= 1e-3 * max(1.0, abs(an)) + 1e-6, (idx, fd, an)
            checked += 1
    assert checked > 20


def test_gradient_finite_where_a_neuron_has_equal_bounds():
    """Lemma A.1's middle case needs l < u; a neuron with l = u (24 of them
    in the second node here) must add nothing undefined to the derivative:
    the gradient is finite and equals central finite differences."""
    p = gen.make_tiny("res16", 4, B=3, splits=(0, 0), n_cuts=0)
    assert any(np.any(l == u) for l, u in p.lu)
    a = np.asarray(O.full_alpha(p), np.float64)
    b, c = np.asarray(p.beta, np.float64), np.asarray(p.gamma, np.float64)
    _, ga, _, _ = O.bound_and_grad(p, a, b, c)
    assert np.all(np.isfinite(ga))
    rng = np.random.default_rng(4)
    h = 1e-6
    for idx in rng.choice(a.size, size=25, replace=False):
        x = a.copy().reshape(-1)
        x[idx] += h
        gp = O.bound(p, x.reshape(a.shape), b, c)
        x[idx] -= 2 * h
        gm = O.bound(p, x.reshape(a.shape), b, c)
        fd = (gp - gm).sum() / (2 * h)
        an = ga.reshape(-1)[idx]
        assert abs(fd - an) <= 1e-3 * max(1.0, abs(an)) + 1e-6, (idx, fd, an)


# ------------------------------------------------- conv adjoint pin

@pytest.mark.parametrize("shape", [((2, 5, 5), 3, 4, 2, 1), ((3, 6, 6), 2, 3, 1, 1),
                                   ((2, 4, 4), 3, 1, 2, 0), ((1, 8, 8), 2, 4, 2, 1)])
def test_conv_transpose_equals_explicit_matrix(shape):
    (ci, hi, wi), co, k, s, pd = shape
    rng = np.random.default_rng(0)
    e = gen.Edge(-1, "conv", rng.normal(size=(co, ci, k, k)), s, pd)
    ho = (hi + 2 * pd - k) // s + 1
    A = lp.edge_matrix(e, (co, ho, ho), (ci, hi, wi))
    lam = rng.normal(size=(3, co * ho * ho))
    got = O.edge_transpose(e, torch.from_numpy(lam), (co, ho, ho), (ci, hi, wi)).numpy()
    assert np.allclose(got, lam @ A, atol=1e-12)
    x = rng.normal(size=(3, ci * hi * wi))
    assert np.allclose(O.edge_forward(e, torch.from_numpy(x), (ci, hi, wi)).numpy(), x @ A.T, atol=1e-12)


# ------------------------------------------------- Adam step pin

def test_adam_step_equals_torch_adam_maximize():
    rng = np.random.default_rng(0)
    x0 = rng.random(50)
    grads = [rng.normal(size=50) for _ in range(5)]
    x = x0.copy(); m = np.zeros(50); v = np.zeros(50)
    t = torch.tensor(x0.copy(), requires_grad=True)
    lr0, dec = 0.1, 0.9
    opt = torch.optim.Adam([t], lr=lr0, betas=(0.9, 0.999), eps=1e-8, maximize=True)
    for it, gr in enumerate(grads):
        x, m, v = O.adam_step(x, gr, m, v, it + 1, lr0 * dec ** it, 0.9, 0.999, 1e-8, -np.inf, np.inf)
        for gparam in opt.param_groups:
            gparam["lr"] = lr0 * dec ** it
        t.grad = torch.tensor(gr)
        opt.step()
    assert np.allclose(x, t.detach().numpy(), atol=1e-12)


# ------------------------------------------------- generator validity

@pytest.mark.parametrize("kind", ["mlp", "cnn", "res"])
def test_ibp_bounds_and_cuts_hold_on_samples(kind):
    p = gen.make_tiny(kind, 3, B=1, n_cuts=6, input_terms=1)
    rng = np.random.default_rng(0)
    X = p.x0 + p.eps * (2 * rng.random((5000, p.net.in_size)) - 1)
    out, pre = lp.plain_forward(p.net, X, return_pre=True)
    relu = p.net.relu_nodes
    lhs = np.zeros((X.shape[0], p.cuts.n))
    for k, q in enumerate(relu):
        l, u = p.lu[k]
        assert np.all(pre[q] >= l - 1e-9) and np.all(pre[q] <= u + 1e-9)
    cu = p.cuts
    for e in range(cu.cut.size):
        nd, j, kd = int(cu.node[e]), int(cu.neuron[e]), int(cu.kind[e])
        if nd < 0:
            val = X[:, j]
        else:
            x = pre[nd][:, j]
            val = (x, np.maximum(x, 0), (x > 0).astype(float))[kd]
        lhs[:, cu.cut[e]] += cu.coef[e] * val
    assert np.all(lhs <= cu.d + 1e-9)


def test_workload_shapes():
    p = gen.make_workload("mlp784", 0, B=3)
    assert p.net.in_size == 784 and [n.size for n in p.net.nodes] == [256] * 6 + [10]
    assert p.S == 9 and p.cuts.n == 200 and p.splits.K == 8
    p3 = gen.make_workload("cnn", 0, B=2)
    assert [n.size for n in p3.net.nodes] == [4096, 2048, 100, 10]
    p5 = gen.make_workload("resnet", 0, B=1)
    assert sum(n.size for n in p5.net.nodes if n.relu) == 73728


@pytest.mark.parametrize("kind,seed", [("mlp", 0), ("mlp", 3), ("cnn", 1), ("res", 2)])
def test_error_scale_equals_textbook_crown_term_sum(kind, seed):
    # The scale T that every parity tolerance divides by, pinned from above
    # and below: with beta = gamma = 0 it must equal the sum of the term
    # magnitudes that the independent primal-form CROWN adds up (bias terms,
    # chord intercepts, input terms), so a term counted twice or dropped in
    # T fails here.
    p = gen.make_tiny(kind, seed, B=2, splits=(0, 0), n_cuts=3)
    prep = O.Prepared(p)
    a = np.random.default_rng(seed).random((p.B, p.S, prep.n_I))
    zb, zc = np.zeros_like(p.beta), np.zeros_like(p.gamma)
    T = O.error_scale(p, a, zb, zc, prep=prep).reshape(p.B, p.S)
    g = O.bound(p, a, zb, zc, prep=prep)
    for b in range(p.B):
        for s in range(p.S):
            apn = []
            for q in prep.relu:
                full = np.zeros(p.net.nodes[q].size)
                full[prep.unst_cols[q]] = a[b, s, prep.alpha_pos[q]]
                apn.append(full)
            val, scale = crown.crown_bound(p.net, p.lu, p.x0, p.eps, p.C[s], apn, with_scale=True)
            assert abs(g[b, s] - val) <= 1e-10 * (1 + abs(val))
            assert abs(T[b, s] - scale) <= 1e-10 * scale, (T[b, s], scale)


def test_error_scale_dominates_bound():
    p = gen.make_tiny("cnn", 0, B=2, splits=(1, 2), n_cuts=4)
    g = O.bound(p)
    T = O.error_scale(p)
    assert np.all(T.reshape(g.shape) >= np.abs(g) - 1e-12)


# ------------------------------- optimised bound: sound and near-tight (T4/T5)

@pytest.mark.parametrize("kind,seed", [("mlp", 0), ("mlp", 5), ("cnn", 1), ("res", 2)])
def test_optimised_gcp_is_sound_and_close_to_lp_with_tight_cuts(kind, seed):
    # Gradient ascent drives the multipliers towards any term the rule gets
    # wrong in the unsound direction, so the optimised bound must still sit
    # below f*_LP-cut; and since the cuts are tight (d = MIP max), the
    # closed-form rule should come close to the LP value (Appendix A notes
    # it need not reach it exactly).
    p = gen.make_tiny(kind, seed, B=2, splits=(1, 2), n_cuts=6, input_terms=1,
                      gamma_dist="zero", beta_dist="zero")
    p.cuts.d[:] = [lp.cut_max(p, k) for k in range(p.cuts.n)]
    lpv = np.array([[lp.lp_value(p, b, s) for s in range(p.S)] for b in range(p.B)])
    g, _, _, _ = O.optimize(p, iters=300, opt=dict(decay=0.99, lr_alpha=0.05, lr_mult=0.05))
    g = g.reshape(p.B, p.S)
    assert np.all(g <= lpv + 1e-7), (g, lpv)
    fin = np.isfinite(lpv)
    assert np.all(lpv[fin] - g[fin] <= 5e-3 * (1 + np.abs(lpv[fin]))), (g, lpv)


def _with_cuts(p, rows, d):
    """Copy of p whose cuts are the given (node, neuron, kind, coef) rows."""
    cut = np.array([r[0] for r in rows], np.int32)
    return gen.Problem(p.name, p.net, p.lu, p.x0, p.eps, p.C, p.splits,
                       gen.Cuts(len(d), cut, np.array([r[1] for r in rows], np.int32),
                                np.array([r[2] for r in rows], np.int32),
                                np.array([r[3] for r in rows], np.int8),
                                np.array([r[4] for r in rows], np.float64), np.array(d, np.float64)),
                       "given", p.alpha, p.beta, None)


def test_cut_on_fixed_z_of_active_neuron_is_a_constant_constraint():
    # A cut  Q z_j + 0 <= d  on a neuron that is active in the subdomain
    # (z_j fixed at 1) is the constant inequality Q <= d; its Lagrangian term
    # gamma (Q - d) must shift the bound by exactly that, for either sign of
    # Q.  On an inactive neuron (z_j = 0) the shift is -gamma d.
    p = gen.make_tiny("mlp", 4, B=1, splits=(2, 2), n_cuts=1, alpha_init="given")
    assert set(p.splits.sign[0].tolist()) == {1, -1}
    sp = p.splits
    a = p.alpha
    b = np.zeros_like(p.beta)
    base_p = _with_cuts(p, [], [])
    g0 = O.bound(base_p, a, b, np.zeros((1, p.S, 0)))
    for k in range(sp.K):
        nd, j, sg = int(sp.node[0, k]), int(sp.neuron[0, k]), int(sp.sign[0, k])
        for Q, d in ((0.7, 0.9), (-0.4, 0.1)):
            pc = _with_cuts(p, [(0, nd, j, gen.KIND_Q, Q)], [d])
            gam = 1.3
            g = O.bound(pc, a, b, np.full((1, p.S, 1), gam))
            zval = 1.0 if sg > 0 else 0.0
            assert np.allclose(g, g0 + gam * (Q * zval - d), atol=1e-12)


def test_cut_on_pre_activation_of_first_layer_neuron_has_lagrangian_slope():
    # A cut  H x_j <= d  on an unstable neuron j of the first ReLU layer adds
    # gamma (H x_j - d) to the Lagrangian, with x_j = W1_j . x + b_j.  For a
    # small gamma >= 0 (no sign of v = Lambda^(1) W^(1) flips, the neuron's
    # relaxation case is untouched) the bound therefore moves with slope
    #     H (W1_j . x0 - eps sign(v) . W1_j + b_j) - d.
    # v itself is recovered independently as dg/dx0 (g is affine in x0 for a
    # fixed sign pattern, with gradient v).
    p = gen.make_tiny("mlp", 0, B=1, splits=(0, 0), n_cuts=1)
    prep = O.Prepared(p)
    q = prep.relu[0]
    j = int(prep.unst_cols[q][0])
    H, d = 0.8, 0.3
    pc = _with_cuts(p, [(0, q, j, gen.KIND_H, H)], [d])
    a, b = p.alpha, p.beta
    step = 1e-7
    g0 = O.bound(pc, a, b, np.zeros((1, p.S, 1)))
    slope = (O.bound(pc, a, b, np.full((1, p.S, 1), step)) - g0) / step
    W1 = p.net.nodes[q].edges[0].W
    v = np.zeros((p.S, p.x0.size))
    for k in range(p.x0.size):
        pk = _with_cuts(p, [(0, q, j, gen.KIND_H, H)], [d])
        pk.x0 = p.x0.copy()
        pk.x0[k] += step
        v[:, k] = (O.bound(pk, a, b, np.zeros((1, p.S, 1)))[0] - g0[0]) / step
    for s_ in range(p.S):
        cj = W1[j] @ p.x0 - p.eps * np.sign(v[s_]) @ W1[j] + p.net.nodes[q].bias[j]
        assert abs(slope[0, s_] - (H * cj - d)) < 1e-5 * (1 + abs(cj)), (slope, cj)


def test_mlp8_golden_values():
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "mlp8_oracle.json")
    ref = json.load(open(path))
    p = gen.make_workload("mlp8", 0)
    g, ga, gb, gc = O.bound_and_grad(p)
    assert np.allclose(g, ref["bound"], rtol=1e-12, atol=1e-12)
    assert np.allclose(ga, ref["d_alpha"], rtol=1e-12, atol=1e-12)
    assert np.allclose(gc, ref["d_gamma"], rtol=1e-12, atol=1e-12)
    assert np.all(g[0] <= np.array(ref["lp_cut"]) + 1e-9)
    assert np.all(np.array(ref["lp_cut"]) <= np.array(ref["mip"]) + 1e-9)


# ------------------------------------------------------------ intermediate bounds
@pytest.mark.parametrize("kind", ["mlp", "cnn", "res"])
def test_crown_intermediate_bounds_exact_at_zero_radius(kind):
    # with eps = 0 every bound is the pre-activation at x0 itself
    p = gen.make_tiny(kind, 0)
    lu = crown.crown_intermediate_bounds(p.net, p.x0, 0.0)
    _, pre = lp.plain_forward(p.net, p.x0[None, :], return_pre=True)
    relu = [i for i, n in enumerate(p.net.nodes) if n.relu]
    for (l, u), i in zip(lu, relu):
        assert np.allclose(l, pre[i][0], atol=1e-9) and np.allclose(u, pre[i][0], atol=1e-9)


@pytest.mark.parametrize("kind", ["mlp", "cnn", "res"])
def test_crown_intermediate_bounds_first_layer_is_interval_arithmetic(kind):
    # node 0 is affine in the input: l, u = A x0 + b -/+ eps * |A| 1
    p = gen.make_tiny(kind, 1, eps=0.2)
    lu = crown.crown_intermediate_bounds(p.net, p.x0, p.eps)
    node = p.net.nodes[0]
    A = sum(lp.edge_matrix(e, node.shape, p.net.shape_of(e.src)) for e in node.edges)
    mid = A @ p.x0 + node.bias
    rad = p.eps * np.abs(A).sum(axis=1)
    assert np.allclose(lu[0][0], mid - rad, atol=1e-9) and np.allclose(lu[0][1], mid + rad, atol=1e-9)


@pytest.mark.parametrize("kind,seed", [("mlp", 2), ("cnn", 3), ("res", 4)])
def test_crown_intermediate_bounds_contain_sampled_preactivations(kind, seed):
    p = gen.make_tiny(kind, seed, eps=0.2)
    lu = crown.crown_intermediate_bounds(p.net, p.x0, p.eps)
    rng = np.random.default_rng(seed)
    xs = p.x0[None, :] + p.eps * rng.uniform(-1, 1, size=(4000, p.x0.size))
    xs[:64] = p.x0[None, :] + p.eps * np.sign(rng.uniform(-1, 1, size=(64, p.x0.size)))   # box vertices
    _, pre = lp.plain_forward(p.net, xs, return_pre=True)
    relu = [i for i, n in enumerate(p.net.nodes) if n.relu]
    for (l, u), i in zip(lu, relu):
        assert (pre[i] >= l[None, :] - 1e-9).all() and (pre[i] <= u[None, :] + 1e-9).all()


# ------------------------------- explicit pi (Appendix A, closing remark)

def test_explicit_pi_h_is_the_lemma_objective():
    # h(pi) of the free-pi form is the single-neuron objective of the proof:
    # never above Lemma A.1's optimum (brute force), equal to it at
    # pi = pi*, and its maximum over a fine rho grid reaches it.
    rng = np.random.default_rng(11)
    grid = torch.linspace(0.0, 1.0, 4001, dtype=torch.float64)
    for _ in range(400):
        l = -rng.exponential(1.0)
        u = rng.exponential(1.0)
        C = rng.exponential(1.0)
        s = rng.normal() * 2.0
        T = lambda x: torch.full_like(grid, x)
        _, h = O.explicit_pi_h(T(-C), T(s), T(l), T(u), grid)
        hb = _brute_h(l, u, C, s)
        assert h.max().item() <= hb + 1e-9 * (1 + abs(hb))
        assert hb - h.max().item() <= (u - l) * C / 4000 + 1e-12
        pi_star, h_star = O.unstable_pi_h(torch.tensor([-C], dtype=torch.float64),
                                          torch.tensor([s], dtype=torch.float64),
                                          torch.tensor([l], dtype=torch.float64),
                                          torch.tensor([u], dtype=torch.float64))
        t1 = lambda x: torch.tensor([x], dtype=torch.float64)
        _, h1 = O.explicit_pi_h(t1(-C), t1(s), t1(l), t1(u), t1(pi_star.item() / C))
        assert abs(h1.item() - h_star.item()) <= 1e-9 * (1 + abs(hb))


@pytest.mark.parametrize("kind,seed", [("mlp", 0), ("cnn", 1), ("res", 2)])
def test_explicit_pi_at_lemma_ratio_without_cut_terms_is_closed_form(kind, seed):
    # With gamma = 0 every s_j is 0 and Lemma A.1's pi* is n u/(u - l):
    # rho = u/(u - l) must reproduce the closed-form bound exactly.
    p = gen.make_tiny(kind, seed, B=2, splits=(1, 2), n_cuts=5, input_terms=1)
    rng = np.random.default_rng(seed)
    a, b, c = _random_params(p, rng, scale=0.5)
    c[:] = 0.0
    g0 = O.bound(p, a, b, c)
    g1 = O.bound_pi(p, a, b, c, O.full_rho(p))
    assert np.allclose(g0, g1, rtol=1e-12, atol=1e-10)
    # and a different rho gives a different (not larger) value somewhere
    r = rng.random(O.full_rho(p).shape)
    assert np.all(O.bound_pi(p, a, b, c, r) <= g0 + 1e-9)


@pytest.mark.parametrize("kind,seed", [("mlp", 0), ("mlp", 5), ("cnn", 1), ("res", 2)])
def test_explicit_pi_bound_below_lp(kind, seed):
    # any rho in [0, 1] is a feasible dual point: weak duality against the
    # LP-cut optimum, for random multipliers of every scale
    p = gen.make_tiny(kind, seed, B=3, splits=(1, 2), n_cuts=5, input_terms=1)
    rng = np.random.default_rng(seed + 100)
    lpv = np.array([[lp.lp_value(p, b, s) for s in range(p.S)] for b in range(p.B)])
    for trial in range(12):
        a, b, c = _random_params(p, rng, scale=[0.0, 0.1, 1.0, 5.0][trial % 4])
        r = rng.random(a.shape)
        g = O.bound_pi(p, a, b, c, r)
        assert np.all(g <= lpv + 1e-8), (g, lpv)


@pytest.mark.parametrize("kind,seed", [("mlp", 0), ("cnn", 1), ("res", 2)])
def test_explicit_pi_gradient_matches_finite_differences(kind, seed):
    p = gen.make_tiny(kind, seed, B=2, splits=(1, 2), n_cuts=5, input_terms=1)
    rng = np.random.default_rng(seed)
    a, b, c = _random_params(p, rng, scale=0.5)
    r = rng.random(a.shape)
    _, ga, gb, gc, gr = O.bound_and_grad_pi(p, a, b, c, r)
    h = 1e-6
    checked = 0
    args = [a, b, c, r]
    for k, grad in enumerate((ga, gb, gc, gr)):
        arr = args[k]
        flat = arr.reshape(-1)
        for idx in rng.choice(flat.size, size=min(flat.size, 20), replace=False) if flat.size else []:
            x = arr.copy().reshape(-1)
            x[idx] += h
            gp = O.bound_pi(p, *[x.reshape(arr.shape) if i == k else y for i, y in enumerate(args)])
            x[idx] -= 2 * h
            gm = O.bound_pi(p, *[x.reshape(arr.shape) if i == k else y for i, y in enumerate(args)])
            fd = (gp - gm).sum() / (2 * h)
            an = grad.reshape(-1)[idx]
            assert abs(fd - an) <= 1e-3 * max(1.0, abs(an)) + 1e-6, (k, idx, fd, an)
            checked += 1
    assert checked > 20


@pytest.mark.parametrize("kind,seed", [("mlp", 0), ("cnn", 1)])
def test_optimised_explicit_pi_is_sound_with_tight_cuts(kind, seed):
    p = gen.make_tiny(kind, seed, B=2, splits=(1, 2), n_cuts=6, input_terms=1,
                      gamma_dist="zero", beta_dist="zero")
    p.cuts.d[:] = [lp.cut_max(p, k) for k in range(p.cuts.n)]
    lpv = np.array([[lp.lp_value(p, b, s) for s in range(p.S)] for b in range(p.B)])
    g, *_ = O.optimize_pi(p, iters=150, opt=dict(decay=0.99, lr_alpha=0.05, lr_mult=0.05))
    assert np.all(g.reshape(p.B, p.S) <= lpv + 1e-7), (g, lpv)


# ------------------------------- intermediate bounds of one BaB domain

def _domain_splits(p, rng, n_split, x_ref):
    # split root-unstable neurons of the ReLU nodes with the signs their
    # pre-activations take at x_ref, so x_ref lies in the domain
    root = crown.crown_intermediate_bounds(p.net, p.x0, p.eps)
    _, pre = lp.plain_forward(p.net, x_ref[None, :], return_pre=True)
    relu = [i for i, n in enumerate(p.net.nodes) if n.relu]
    cand = [(k, j) for (l, u), k in zip(root, relu) for j in np.nonzero((l < 0) & (u > 0))[0]]
    pick = rng.choice(len(cand), size=min(n_split, len(cand)), replace=False)
    return [(k, int(j), 1 if pre[k][0][j] >= 0 else -1) for k, j in (cand[t] for t in pick)]


@pytest.mark.parametrize("kind,seed", [("mlp", 2), ("cnn", 3), ("res", 4)])
def test_domain_intermediate_bounds_contain_the_domain_samples(kind, seed):
    p = gen.make_tiny(kind, seed, eps=0.2)
    rng = np.random.default_rng(seed)
    x_ref = p.x0 + p.eps * rng.uniform(-1, 1, size=p.x0.size)
    sp = _domain_splits(p, rng, 4, x_ref)
    lu = crown.crown_intermediate_bounds(p.net, p.x0, p.eps, splits=sp)
    xs = p.x0[None, :] + p.eps * rng.uniform(-1, 1, size=(20000, p.x0.size))
    xs[0] = x_ref
    _, pre = lp.plain_forward(p.net, xs, return_pre=True)
    keep = np.ones(xs.shape[0], bool)
    for k, j, sg in sp:
        keep &= sg * pre[k][:, j] >= 0
    assert keep.sum() >= 1
    relu = [i for i, n in enumerate(p.net.nodes) if n.relu]
    for (l, u), i in zip(lu, relu):
        assert (pre[i][keep] >= l[None, :] - 1e-9).all() and (pre[i][keep] <= u[None, :] + 1e-9).all()
    for k, j, sg in sp:   # each split neuron's own bound is clamped at 0
        l, u = lu[relu.index(k)]
        assert (l[j] >= 0.0) if sg > 0 else (u[j] <= 0.0)


@pytest.mark.parametrize("kind", ["mlp", "cnn", "res"])
def test_domain_intermediate_bounds_exact_at_zero_radius(kind):
    # eps = 0 with splits that x0 satisfies: every neuron takes the piece it
    # takes at x0, so every bound is x0's pre-activation
    p = gen.make_tiny(kind, 0, eps=0.2)
    rng = np.random.default_rng(5)
    sp = _domain_splits(p, rng, 3, p.x0)
    lu = crown.crown_intermediate_bounds(p.net, p.x0, 0.0, splits=sp)
    _, pre = lp.plain_forward(p.net, p.x0[None, :], return_pre=True)
    relu = [i for i, n in enumerate(p.net.nodes) if n.relu]
    for (l, u), i in zip(lu, relu):
        assert np.allclose(l, pre[i][0], atol=1e-9) and np.allclose(u, pre[i][0], atol=1e-9)


def test_domain_intermediate_bounds_without_splits_are_the_root_bounds():
    p = gen.make_tiny("res", 1, eps=0.2)
    a = crown.crown_intermediate_bounds(p.net, p.x0, p.eps)
    b = crown.crown_intermediate_bounds(p.net, p.x0, p.eps, splits=[])
    for (l0, u0), (l1, u1) in zip(a, b):
        assert np.array_equal(l0, l1) and np.array_equal(u0, u1)


# ------------------------------- stored CROWN root bounds of the benchmark workloads

@pytest.mark.parametrize("kind,seed", [("mlp", 1), ("cnn", 2), ("res", 3)])
def test_root_bounds_equal_textbook_crown_layer_by_layer(kind, seed):
    # the batched root-bound computation (Theorem 3.1 at beta = gamma = 0 on
    # each prefix network, rows +e_j / -e_j) against the primal-form textbook
    # CROWN given the same earlier bounds, node by node; the stored values are
    # rounded outward to fp32, so within one fp32 ulp and on the outer side
    from oracle import root_bounds
    p = gen.make_tiny(kind, seed, eps=0.1)
    ours = root_bounds.crown_root_bounds(p.net, p.x0, p.eps, chunk=7)
    ref = crown.crown_intermediate_bounds(p.net, p.x0, p.eps, lu_given=ours)
    for (l, u), (lr, ur) in zip(ours, ref):
        assert np.all(l <= lr + 1e-12) and np.all(u >= ur - 1e-12)
        assert np.all(lr - l <= 2.0 ** -23 * np.abs(lr) + 1e-300)
        assert np.all(u - ur <= 2.0 ** -23 * np.abs(ur) + 1e-300)
        assert np.all(l.astype(np.float32).astype(np.float64) == l)


@pytest.mark.parametrize("name", ["mlp784", "cnn", "resnet"])
def test_stored_root_bounds_contain_sampled_preactivations(name):
    # the workloads' stored bounds are valid over the box: sampled points and
    # box vertices stay inside, and they are no looser than interval bounds
    net, x0, eps = gen.workload_net(name, 0)
    lu = gen.load_root_bounds(name, 0, net, x0, eps)
    ibp = gen.ibp_bounds(net, x0, eps)
    rng = np.random.default_rng(5)
    n = 64 if name == "resnet" else 512
    xs = x0[None, :] + eps * rng.uniform(-1, 1, size=(n, x0.size))
    xs[: n // 8] = x0[None, :] + eps * np.sign(rng.uniform(-1, 1, size=(n // 8, x0.size)))
    _, pre = lp.plain_forward(net, xs, return_pre=True)
    for (l, u), (li, ui), i in zip(lu, ibp, net.relu_nodes):
        assert (pre[i] >= l[None, :]).all() and (pre[i] <= u[None, :]).all()
        assert np.all(l >= li) and np.all(u <= ui)
