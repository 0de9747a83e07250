"""Plain FP64 reference of the GCP-CROWN bound (test infrastructure only).

Follows Theorem 3.1 (Sec. 3.1; restated with proof in Appendix A) in the
coefficient form Lambda := -nu, one (domain, spec row) at a time; rows are
independent scalar problems, so they are simply stacked along dim 0.

Readings of the paper adopted here (all listed in the design notes):
  * Dual objective: the input term is  v.x0 - eps*||v||_1  with
    v = Lambda^(1) W^(1): the minimum of a linear function over the box
    (Appendix A says the norm comes from minimising over x).
  * [.]_- in the unstable rule is the magnitude of the negative part,
    max(-x, 0), so that mu + tau = [nu_hat]_- >= 0.
  * pi* = clip((u [nu_hat]_+ - beta^T Q_{:,j}) / (u - l), 0, [nu_hat]_+):
    Lemma A.1 applied with q = -beta^T Q_{:,j} (the printed '+' does not
    follow from the lemma); h is taken per the theorem's three cases.
  * Bias term: + sum_i Lambda^(i).b^(i) (Lagrangian constraint x - Wx - b).
  * Class ties: active if l >= 0, else inactive if u <= 0, else unstable.
  * z of a neuron that is active in the subdomain (root-active or split
    x >= 0) is fixed at 1, of an inactive one at 0, so a cut's Q term on
    an active neuron adds Q.gamma to the constant.
  * Splits are the special cuts of Sec. 3.1 ('Connection to CROWN-like
    methods'): an x >= 0 split makes the neuron active and adds -beta to
    its Lambda; an x <= 0 split makes it inactive and adds +beta.
  * Residual (DAG) nets: the coefficient on a post-activation sums the
    contributions of all of its consumers.
Naming follows the library: beta multiplies split constraints, gamma
multiplies cut rows (the paper calls both beta).
"""
from __future__ import annotations

import numpy as np
import torch

ACTIVE, INACTIVE, UNSTABLE = 1, 0, 2


def root_classes(l, u):
    """Class of each neuron from its root bounds (Sec. 2 neuron classes)."""
    c = np.full(l.shape[0], UNSTABLE, np.int8)
    c[u <= 0] = INACTIVE
    c[l >= 0] = ACTIVE
    return c


def _t(a):
    return torch.as_tensor(np.asarray(a), dtype=torch.float64)


def edge_transpose(e, lam, dst_shape, src_shape):
    """Row vectors times the edge's matrix: returns lam @ A for the linear
    map A: x_hat_src -> x_dst (dense W, conv, identity)."""
    M = lam.shape[0]
    if e.kind == "identity":
        return lam
    if e.kind == "dense":
        return lam @ _t(e.W)
    if e.kind == "conv":
        co, ho, wo = dst_shape
        ci, hi, wi = src_shape
        kh = e.W.shape[2]
        oph = hi - ((ho - 1) * e.stride - 2 * e.pad + kh)
        opw = wi - ((wo - 1) * e.stride - 2 * e.pad + e.W.shape[3])
        y = torch.nn.functional.conv_transpose2d(
            lam.reshape(M, co, ho, wo), _t(e.W), stride=e.stride, padding=e.pad,
            output_padding=(oph, opw))
        return y.reshape(M, -1)
    raise ValueError(e.kind)


def edge_forward(e, x, src_shape):
    """The edge's linear map applied to rows of x."""
    M = x.shape[0]
    if e.kind == "identity":
        return x
    if e.kind == "dense":
        return x @ _t(e.W).T
    if e.kind == "conv":
        y = torch.nn.functional.conv2d(x.reshape((M,) + tuple(src_shape)), _t(e.W),
                                       stride=e.stride, padding=e.pad)
        return y.reshape(M, -1)
    raise ValueError(e.kind)


class Prepared:
    """Per-node index structures derived from a workloads.Problem."""

    def __init__(self, prob):
        self.prob = prob
        net = prob.net
        self.relu = [i for i, n in enumerate(net.nodes) if n.relu]
        self.rel_pos = {p: k for k, p in enumerate(self.relu)}
        self.out = len(net.nodes) - 1
        self.cls, self.unst_cols, self.alpha_pos = {}, {}, {}
        off = 0
        for k, p in enumerate(self.relu):
            l, u = prob.lu[k]
            c = root_classes(l, u)
            cols = np.nonzero(c == UNSTABLE)[0]
            self.cls[p] = c
            self.unst_cols[p] = cols
            self.alpha_pos[p] = off + np.arange(cols.size)
            off += cols.size
        self.n_I = off
        sp = prob.splits
        for b in range(sp.B):
            seen = set()
            for k in range(sp.K):
                if sp.node[b, k] >= 0:
                    key = (int(sp.node[b, k]), int(sp.neuron[b, k]))
                    assert key not in seen, "duplicate split in one domain"
                    seen.add(key)


def unstable_pi_h(a_hat, s, l, u):
    """pi* and h of an unstable neuron (Theorem 3.1, Lemma A.1).

    With n = [nu_hat]_+ = [-a_hat]_+ (the coefficient mass that the upper
    relaxation must carry) and q = -s, s = (gamma^T Q)_j, Lemma A.1 gives
      s >= u n           : pi* = 0,                      h = 0
      s <= l n           : pi* = n,                      h = s
      l n < s < u n      : pi* = (u n - s) / (u - l),    h = l pi*
    i.e. pi* = clip((u n - s)/(u - l), 0, n) and h = l pi* - [u(n - pi*) + l pi* - s]_+.
    The case is chosen on detached values so the derivative follows the
    selected branch.  The middle case needs l n < s < u n with n > 0, so
    u > l there; elsewhere the quotient is not used and its denominator is
    set to 1, so that a neuron with u = l adds no 0/0 to the derivative."""
    n = torch.relu(-a_hat)
    with torch.no_grad():
        case_zero = s >= u * n
        case_full = (~case_zero) & (s <= l * n)
        case_mid = (~case_zero) & (~case_full)
    pi_mid = (u * n - s) / torch.where(case_mid, u - l, torch.ones_like(u - l))
    pi = torch.where(case_mid, pi_mid, torch.where(case_full, n, torch.zeros_like(n)))
    h = torch.where(case_mid, l * pi_mid, torch.where(case_full, s, torch.zeros_like(s)))
    return pi, h


def explicit_pi_h(a_hat, s, l, u, rho):
    """pi and h of an unstable neuron when pi is a free variable instead of
    Lemma A.1's maximiser (the remark closing the proof of Theorem 3.1 in
    Appendix A: pi and the upper-relaxation multiplier can be optimised too).

    The single-neuron problem of the proof maximises
      h(pi) = l pi - [u (n - pi) + l pi - s]_+      over 0 <= pi <= n,
    n = [-a_hat]_+ (the upper multiplier being n - pi).  Every feasible pi is
    a valid dual point, so the bound stays sound; pi = rho * n with
    rho in [0, 1] is the parametrisation used here."""
    n = torch.relu(-a_hat)
    pi = rho * n
    h = l * pi - torch.relu(u * n - (u - l) * pi - s)
    return pi, h


def _cut_term(prob, gamma, node, kind, size):
    """(gamma^T X)_j for X in {H, G, Q} of one node: a sparse gather."""
    cu = prob.cuts
    sel = (cu.node == node) & (cu.kind == kind)
    out = torch.zeros(gamma.shape[0], size, dtype=torch.float64)
    if not sel.any():
        return out
    k = torch.as_tensor(cu.cut[sel].astype(np.int64))
    j = torch.as_tensor(cu.neuron[sel].astype(np.int64))
    c = _t(cu.coef[sel])
    return out.index_add(1, j, gamma[:, k] * c)


def bound_rows(prob, alpha, beta, gamma, prep=None, rows=None, with_scale=False, rho=None, lams=None):
    """Theorem 3.1 objective g for every (domain, spec row).

    alpha [M, n_I], beta [M, K], gamma [M, N] are float64 tensors over the
    M = B*S rows (row r belongs to domain r // S and spec row r % S) and
    may require grad.  ``rows`` optionally restricts to a subset of row ids
    (alpha/beta/gamma are then given for those rows only).
    Returns g [M]; with ``with_scale`` also the sum of the magnitudes of
    every term added into g (the natural scale of its rounding error):
    sum|v_k x0_k| + eps*||v||_1 + sum|Lambda_j b_j| + sum|h_j| +
    sum|s_j (active)| + sum|gamma_k d_k|.
    ``rho`` [M, n_I] (optional, layout of alpha) replaces Lemma A.1's pi* of
    every root-unstable neuron by pi = rho * [-a_hat]_+ (explicit_pi_h).
    ``lams`` (optional dict) receives Lambda [M, size] of every ReLU node,
    keyed by node index (read-only view of the recursion, for tests)."""
    prep = prep or Prepared(prob)
    net = prob.net
    S = prob.S
    if rows is None:
        rows = np.arange(prob.B * S)
    rows = np.asarray(rows)
    M = rows.size
    dom = rows // S
    srow = rows % S
    sp = prob.splits

    out_node = net.nodes[prep.out]
    lam_out = _t(prob.C)[torch.as_tensor(srow)]
    K = lam_out @ _t(out_node.bias)
    T = (lam_out * _t(out_node.bias)).abs().sum(1)
    acc = {}

    def push(i, lam):
        node = net.nodes[i]
        for e in node.edges:
            contrib = edge_transpose(e, lam, node.shape, net.shape_of(e.src))
            acc[e.src] = acc[e.src] + contrib if e.src in acc else contrib

    push(prep.out, lam_out)
    for p in reversed(prep.relu):
        node = net.nodes[p]
        d = node.size
        a_hat = acc.get(p, torch.zeros(M, d, dtype=torch.float64)) + _cut_term(prob, gamma, p, 1, d)
        t = _cut_term(prob, gamma, p, 0, d)
        s = _cut_term(prob, gamma, p, 2, d)
        l = _t(prob.lu[prep.rel_pos[p]][0]).expand(M, d)
        u = _t(prob.lu[prep.rel_pos[p]][1]).expand(M, d)
        cls = np.broadcast_to(prep.cls[p], (M, d)).copy()
        split_term = torch.zeros(M, d, dtype=torch.float64)
        for k in range(sp.K):
            hit = np.nonzero(sp.node[dom, k] == p)[0]
            if hit.size == 0:
                continue
            j = sp.neuron[dom[hit], k].astype(np.int64)
            sg = sp.sign[dom[hit], k].astype(np.int64)
            cls[hit, j] = np.where(sg > 0, ACTIVE, INACTIVE)
            vals = -_t(sg.astype(np.float64)) * beta[torch.as_tensor(hit), k]
            split_term = split_term.index_put((torch.as_tensor(hit), torch.as_tensor(j)), vals,
                                              accumulate=True)
        act = torch.as_tensor(cls == ACTIVE)
        ina = torch.as_tensor(cls == INACTIVE)
        uns = torch.as_tensor(cls == UNSTABLE)

        # alpha scattered onto the root-unstable columns of this node
        cols = torch.as_tensor(prep.unst_cols[p].astype(np.int64))
        a_full = torch.zeros(M, d, dtype=torch.float64)
        if cols.numel():
            a_full = a_full.index_copy(1, cols, alpha[:, torch.as_tensor(prep.alpha_pos[p])])

        if rho is None:
            pi, h = unstable_pi_h(a_hat, s, l, u)
        else:
            r_full = torch.zeros(M, d, dtype=torch.float64)
            if cols.numel():
                r_full = r_full.index_copy(1, cols, rho[:, torch.as_tensor(prep.alpha_pos[p])])
            pi, h = explicit_pi_h(a_hat, s, l, u, r_full)
        lam_uns = a_full * torch.relu(a_hat) - pi + t

        lam = torch.where(act, a_hat + t, torch.where(ina, t, lam_uns)) + split_term
        K = K + lam @ _t(node.bias) + (h * uns).sum(1) + (s * act).sum(1)
        if with_scale:
            T = T + (lam * _t(node.bias)).abs().sum(1) + (h * uns).abs().sum(1) + (s * act).abs().sum(1)
        if lams is not None:
            lams[p] = lam.detach().clone()
        push(p, lam)

    v = acc.get(-1, torch.zeros(M, net.in_size, dtype=torch.float64)) + \
        _cut_term(prob, gamma, -1, 1, net.in_size)
    x0 = _t(prob.x0)
    dvec = _t(prob.cuts.d)
    g = v @ x0 - prob.eps * v.abs().sum(1) + K - gamma @ dvec
    if with_scale:
        T = T + (v * x0).abs().sum(1) + prob.eps * v.abs().sum(1) + (gamma * dvec).abs().sum(1)
        return g, T
    return g


def full_alpha(prob, prep=None):
    """Alpha [B, S, n_I] as float64 (expanding the CROWN-adaptive start)."""
    prep = prep or Prepared(prob)
    if prob.alpha_init == "given":
        return np.asarray(prob.alpha, np.float64)
    a = []
    for k, p in enumerate(prep.relu):
        l, u = prob.lu[k]
        c = prep.unst_cols[p]
        a.append((u[c] >= -l[c]).astype(np.float64))
    vec = np.concatenate(a) if a else np.zeros(0)
    return np.broadcast_to(vec, (prob.B, prob.S, vec.size)).copy()


def bound(prob, alpha=None, beta=None, gamma=None, rows=None, prep=None, flat=False):
    """numpy wrapper: bounds [B, S] (or [len(rows)] for a row subset)."""
    prep = prep or Prepared(prob)
    a, b, c = _params(prob, alpha, beta, gamma, rows, prep, flat)
    with torch.no_grad():
        g = bound_rows(prob, a, b, c, prep, rows)
    g = g.numpy()
    return g if rows is not None else g.reshape(prob.B, prob.S)


def _params(prob, alpha, beta, gamma, rows, prep, flat=False):
    """Parameters as [M, .] float64 tensors.  ``flat`` means the caller's
    arrays are already restricted to ``rows``; otherwise they are full
    [B, S, .] arrays (or None for the problem's own starting values)."""
    M = prob.B * prob.S
    if flat:
        return _t(alpha), _t(beta), _t(gamma)
    alpha = full_alpha(prob, prep) if alpha is None else alpha
    beta = prob.beta if beta is None else beta
    gamma = prob.gamma if gamma is None else gamma
    a = _t(alpha).reshape(M, -1)
    b = _t(beta).reshape(M, -1)
    c = _t(gamma).reshape(M, -1)
    if rows is not None:
        r = torch.as_tensor(np.asarray(rows))
        a, b, c = a[r], b[r], c[r]
    return a, b, c


def bound_and_grad(prob, alpha=None, beta=None, gamma=None, rows=None, prep=None, flat=False):
    """Bounds and d(sum of bounds)/d(alpha, beta, gamma) by float64 reverse
    mode; each row only depends on its own parameters, so this is the
    per-row gradient.  Kinks: relu'(0) = 0, |.|'(0) = 0, and the case of
    the unstable rule is chosen by the same comparisons as the value."""
    prep = prep or Prepared(prob)
    a, b, c = _params(prob, alpha, beta, gamma, rows, prep, flat)
    a = a.clone().requires_grad_(True)
    b = b.clone().requires_grad_(True)
    c = c.clone().requires_grad_(True)
    g = bound_rows(prob, a, b, c, prep, rows)
    g.sum().backward()
    shp = (lambda x: x) if rows is not None else (lambda x: x.reshape(prob.B, prob.S, -1))
    gv = g.detach().numpy()
    return (gv if rows is not None else gv.reshape(prob.B, prob.S),
            shp(_grad(a)), shp(_grad(b)), shp(_grad(c)))


def _grad(x):
    return np.zeros(tuple(x.shape)) if x.grad is None else x.grad.numpy()


def adam_step(x, grad, m, v, t, lr, b1, b2, eps, lo, hi):
    """One projected Adam ascent step (step count t >= 1), numpy float64."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    x = x + lr * mh / (np.sqrt(vh) + eps)
    x = np.clip(x, lo, hi)
    return x, m, v


def optimize(prob, iters=None, alpha=None, beta=None, gamma=None, rows=None, opt=None, prep=None,
             history=False, flat=False):
    """Gradient ascent on alpha (lr 0.1), beta and gamma (lr 0.02) with Adam,
    learning rates decayed by 0.9 per iteration (Appendix C.1), projecting
    alpha into [0, 1] and the multipliers onto >= 0 after every step; the
    objective is the sum of the rows' bounds (rows are independent).
    Returns (bound at the final parameters [M], alpha, beta, gamma) as flat
    [M, .] arrays over ``rows`` (all rows when None).  With ``flat`` the
    starting parameters are given already restricted to ``rows``."""
    prep = prep or Prepared(prob)
    o = dict(prob.opt)
    o.update(opt or {})
    iters = o["iters"] if iters is None else iters
    rows = np.arange(prob.B * prob.S) if rows is None else np.asarray(rows)
    a, b, c = (x.numpy().copy() for x in _params(prob, alpha, beta, gamma, rows, prep, flat))
    ma, va = np.zeros_like(a), np.zeros_like(a)
    mb, vb = np.zeros_like(b), np.zeros_like(b)
    mc, vc = np.zeros_like(c), np.zeros_like(c)
    hist = []
    b1, b2, ae = o["adam_b1"], o["adam_b2"], o["adam_eps"]
    for it in range(iters):
        g, ga, gb, gc = bound_and_grad(prob, a, b, c, rows=rows, prep=prep, flat=True)
        hist.append(g)
        dec = o["decay"] ** it
        a, ma, va = adam_step(a, ga, ma, va, it + 1, o["lr_alpha"] * dec, b1, b2, ae, 0.0, 1.0)
        b, mb, vb = adam_step(b, gb, mb, vb, it + 1, o["lr_mult"] * dec, b1, b2, ae, 0.0, np.inf)
        c, mc, vc = adam_step(c, gc, mc, vc, it + 1, o["lr_mult"] * dec, b1, b2, ae, 0.0, np.inf)
    gfin = bound(prob, a, b, c, rows=rows, prep=prep, flat=True)
    out = (gfin, a, b, c)
    return out + (hist,) if history else out


def node_lambdas(prob, alpha=None, beta=None, gamma=None, rows=None, prep=None, flat=False):
    """Lambda [rows, size] of every ReLU node at the given parameters (the
    multipliers of the Theorem 3.1 recursion), keyed by node index."""
    prep = prep or Prepared(prob)
    a, b, c = _params(prob, alpha, beta, gamma, rows, prep, flat)
    lams = {}
    with torch.no_grad():
        bound_rows(prob, a, b, c, prep, rows, lams=lams)
    return {k: v.numpy() for k, v in lams.items()}


def error_scale(prob, alpha=None, beta=None, gamma=None, rows=None, prep=None, flat=False, rho=None):
    """Per-row sum of the magnitudes of all terms added into the bound (of
    the explicit-pi bound when ``rho`` is given)."""
    prep = prep or Prepared(prob)
    a, b, c = _params(prob, alpha, beta, gamma, rows, prep, flat)
    r = None if rho is None else _rho_param(prob, rho, rows, prep, flat)
    with torch.no_grad():
        _, T = bound_rows(prob, a, b, c, prep, rows, with_scale=True, rho=r)
    return T.numpy()


# ---------------------------------------------------------------- explicit pi
def full_rho(prob, prep=None):
    """Starting rho [B, S, n_I]: u / (u - l), which is Lemma A.1's pi* / n
    whenever the neuron's cut term s is 0 (no cut uses its z), so the first
    bound equals the closed form's on cut-free neurons."""
    prep = prep or Prepared(prob)
    r = []
    for k, p in enumerate(prep.relu):
        l, u = prob.lu[k]
        c = prep.unst_cols[p]
        r.append(u[c] / (u[c] - l[c]))
    vec = np.concatenate(r) if r else np.zeros(0)
    return np.broadcast_to(vec, (prob.B, prob.S, vec.size)).copy()


def _rho_param(prob, rho, rows, prep, flat):
    if flat:
        return _t(rho)
    rho = full_rho(prob, prep) if rho is None else rho
    r = _t(rho).reshape(prob.B * prob.S, -1)
    if rows is not None:
        r = r[torch.as_tensor(np.asarray(rows))]
    return r


def bound_pi(prob, alpha=None, beta=None, gamma=None, rho=None, rows=None, prep=None, flat=False):
    """Bounds with explicit pi = rho * [-a_hat]_+ (explicit_pi_h)."""
    prep = prep or Prepared(prob)
    a, b, c = _params(prob, alpha, beta, gamma, rows, prep, flat)
    r = _rho_param(prob, rho, rows, prep, flat)
    with torch.no_grad():
        g = bound_rows(prob, a, b, c, prep, rows, rho=r)
    g = g.numpy()
    return g if rows is not None else g.reshape(prob.B, prob.S)


def bound_and_grad_pi(prob, alpha=None, beta=None, gamma=None, rho=None, rows=None, prep=None, flat=False):
    """bound_pi and d(sum of bounds)/d(alpha, beta, gamma, rho) in float64
    reverse mode (same kink conventions as bound_and_grad)."""
    prep = prep or Prepared(prob)
    a, b, c = _params(prob, alpha, beta, gamma, rows, prep, flat)
    r = _rho_param(prob, rho, rows, prep, flat)
    a, b, c, r = (x.clone().requires_grad_(True) for x in (a, b, c, r))
    g = bound_rows(prob, a, b, c, prep, rows, rho=r)
    g.sum().backward()
    shp = (lambda x: x) if rows is not None else (lambda x: x.reshape(prob.B, prob.S, -1))
    gv = g.detach().numpy()
    return (gv if rows is not None else gv.reshape(prob.B, prob.S),
            shp(_grad(a)), shp(_grad(b)), shp(_grad(c)), shp(_grad(r)))


def optimize_pi(prob, iters=None, alpha=None, beta=None, gamma=None, rho=None, rows=None, opt=None, prep=None,
                flat=False):
    """optimize with rho as a fourth parameter: Adam ascent with alpha's
    learning rate, projected onto [0, 1] like alpha.  Returns (bound [M],
    alpha, beta, gamma, rho) over ``rows``."""
    prep = prep or Prepared(prob)
    o = dict(prob.opt)
    o.update(opt or {})
    iters = o["iters"] if iters is None else iters
    rows = np.arange(prob.B * prob.S) if rows is None else np.asarray(rows)
    a, b, c = (x.numpy().copy() for x in _params(prob, alpha, beta, gamma, rows, prep, flat))
    r = _rho_param(prob, rho, rows, prep, flat).numpy().copy()
    ma, va = np.zeros_like(a), np.zeros_like(a)
    mb, vb = np.zeros_like(b), np.zeros_like(b)
    mc, vc = np.zeros_like(c), np.zeros_like(c)
    mr, vr = np.zeros_like(r), np.zeros_like(r)
    b1, b2, ae = o["adam_b1"], o["adam_b2"], o["adam_eps"]
    for it in range(iters):
        _, ga, gb, gc, gr = bound_and_grad_pi(prob, a, b, c, r, rows=rows, prep=prep, flat=True)
        dec = o["decay"] ** it
        a, ma, va = adam_step(a, ga, ma, va, it + 1, o["lr_alpha"] * dec, b1, b2, ae, 0.0, 1.0)
        b, mb, vb = adam_step(b, gb, mb, vb, it + 1, o["lr_mult"] * dec, b1, b2, ae, 0.0, np.inf)
        c, mc, vc = adam_step(c, gc, mc, vc, it + 1, o["lr_mult"] * dec, b1, b2, ae, 0.0, np.inf)
        r, mr, vr = adam_step(r, gr, mr, vr, it + 1, o["lr_alpha"] * dec, b1, b2, ae, 0.0, 1.0)
    gfin = bound_pi(prob, a, b, c, r, rows=rows, prep=prep, flat=True)
    return gfin, a, b, c, r
