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


def crown_bound(net, lu, x0, eps, c, alpha_per_node):
    """Lower bound of c^T f(x) over the box.  alpha_per_node[k] is the lower
    slope of every neuron of the k-th ReLU node (used where unstable)."""
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
    for p in reversed(relu):
        node = net.nodes[p]
        lam_hat = np.asarray(coef.get(p, np.zeros(node.size)), np.float64)
        l, u = lu[pos[p]]
        lam = np.zeros(node.size)
        for j in range(node.size):
            if l[j] >= 0:
                lam[j] = lam_hat[j]
            elif u[j] <= 0:
                lam[j] = 0.0
            elif lam_hat[j] >= 0:
                lam[j] = alpha_per_node[pos[p]][j] * lam_hat[j]
            else:
                slope = u[j] / (u[j] - l[j])
                lam[j] = lam_hat[j] * slope
                const += lam_hat[j] * (-slope * l[j])
        const += float(lam @ node.bias)
        spread(node, lam)
    w = coef.get(-1, np.zeros(net.in_size))
    return float(w @ x0 - eps * np.abs(w).sum() + const)
