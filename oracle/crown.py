"""Textbook (alpha-)CROWN in primal form (test infrastructure only).

An independent derivation of the cut-free, split-free special case, used
to pin the GCP-CROWN oracle (Proposition 3.2 and the CROWN paragraph of
Sec. 3.1: with every multiplier at zero the rule is CROWN's).  Here the
ReLU of an unstable neuron is bounded by two lines chosen by the sign of
its coefficient lam_hat on the post-activation x_hat:
  lam_hat >= 0: x_hat >= alpha * x          (lower line, slope alpha)
  lam_hat <  0: x_hat <= u/(u-l) * (x - l)  (upper chord)
and the resulting linear function of the input is minimised over the box
in closed form: min_{|x-x0|<=eps} w.x = w.x0 - eps*||w||_1.
"""
from __future__ import annotations

import numpy as np

from .lp import edge_matrix


def crown_bound(net, lu, x0, eps, c, alpha_per_node, fixed=None, with_scale=False):
    """Lower bound of c^T f(x) over the box.  alpha_per_node[k] is the lower
    slope of every neuron of the k-th ReLU node (used where unstable).
    fixed[(node, neuron)] = +1 / -1 replaces the ReLU of that neuron by its
    active (x_hat = x) / inactive (x_hat = 0) piece: the network of a BaB
    domain with those splits, whose bound over the box also bounds it over
    the domain (Sec. 3.1, splits; no split multipliers here).

    with_scale: also return the sum of the magnitudes of the individual
    terms the bound adds up (each bias term lam_j b_j, each chord intercept,
    each input term w_k x0_k and eps |w_k|), counted term by term here in
    the primal form."""
    fixed = fixed or {}
    scale = 0.0
    relu = [i for i, n in enumerate(net.nodes) if n.relu]
    pos = {p: k for k, p in enumerate(relu)}
    coef = {}          # coefficient row on each post-activation
    out = net.nodes[-1]
    const = float(c @ out.bias)

    def spread(node, lam):
        for e in node.edges:
            A = edge_matrix(e, node.shape, net.shape_of(e.src))
            coef[e.src] = coef.get(e.src, 0.0) + lam @ A

    spread(out, np.asarray(c, np.float64))
    scale += float(np.abs(np.asarray(c, np.float64) * out.bias).sum())
    for p in reversed(relu):
        node = net.nodes[p]
        lam_hat = np.asarray(coef.get(p, np.zeros(node.size)), np.float64)
        l, u = lu[pos[p]]
        lam = np.zeros(node.size)
        for j in range(node.size):
            fx = fixed.get((p, j), 0)
            if fx > 0 or (fx == 0 and l[j] >= 0):
                lam[j] = lam_hat[j]
            elif fx < 0 or u[j] <= 0:
                lam[j] = 0.0
            elif lam_hat[j] >= 0:
                lam[j] = alpha_per_node[pos[p]][j] * lam_hat[j]
            else:
                slope = u[j] / (u[j] - l[j])
                lam[j] = lam_hat[j] * slope
                const += lam_hat[j] * (-slope * l[j])
                scale += abs(lam_hat[j] * slope * l[j])
        const += float(lam @ node.bias)
        scale += float(np.abs(lam * node.bias).sum())
        spread(node, lam)
    w = coef.get(-1, np.zeros(net.in_size))
    val = float(w @ x0 - eps * np.abs(w).sum() + const)
    if with_scale:
        return val, scale + float(np.abs(w * x0).sum() + eps * np.abs(w).sum())
    return val


def crown_intermediate_bounds(net, x0, eps, lu_given=None, splits=None):
    """Layer-by-layer CROWN bounds on every ReLU node's pre-activation
    (intermediate bounds of Sec. 2, computed as in CROWN: the bounds of node k
    are the CROWN bounds of the prefix network that ends at node k's
    pre-activation, for the spec rows +e_j and -e_j, with the bounds of the
    earlier nodes and CROWN-adaptive lower slopes alpha = 1 where u >= -l,
    else 0).  Returns [(l, u)] per ReLU node.

    With lu_given, node k uses lu_given[:k] for the earlier nodes instead of
    its own results (to compare one layer at a time with another
    implementation).

    splits: optional [(node, neuron, sign)] of one BaB domain (sign +1 for
    x >= 0, -1 for x <= 0): the bounds over that domain instead of the whole
    box.  A split neuron of an earlier node takes its linear piece (as in
    crown_bound's fixed), and its own bounds are clamped at 0 (l = max(l, 0)
    for x >= 0, u = min(u, 0) for x <= 0); a split that contradicts the
    bounds (the domain is empty, up to rounding) leaves the neuron at
    exactly 0."""
    import dataclasses

    relu = [i for i, n in enumerate(net.nodes) if n.relu]
    fixed_all = {(int(n), int(j)): int(sg) for n, j, sg in (splits or [])}
    lu = []
    for pos, k in enumerate(relu):
        node = net.nodes[k]
        prev = list(lu_given[:pos]) if lu_given is not None else list(lu)
        prefix = type(net)(net.in_shape, list(net.nodes[:k]) + [dataclasses.replace(node, relu=False)])
        apn = [np.where(u >= -l, 1.0, 0.0) for l, u in prev]
        fixed = {key: sg for key, sg in fixed_all.items() if key[0] < k}
        lo = np.empty(node.size)
        hi = np.empty(node.size)
        for j in range(node.size):
            e = np.zeros(node.size)
            e[j] = 1.0
            lo[j] = crown_bound(prefix, prev, x0, eps, e, apn, fixed)
            hi[j] = -crown_bound(prefix, prev, x0, eps, -e, apn, fixed)
        for (n, j), sg in fixed_all.items():
            if n != k:
                continue
            if sg > 0:
                lo[j] = max(lo[j], 0.0)
                hi[j] = max(hi[j], lo[j])
            else:
                hi[j] = min(hi[j], 0.0)
                lo[j] = min(lo[j], hi[j])
        lu.append((lo, hi))
    return lu
