"""Exact reference values that pin the bound oracle (test infrastructure only).

* ``lp_value``: the LP relaxation with cuts, eq. lp_with_cuts (Sec. 3.1),
  i.e. eqs. mip_layer, mip_output, mip_unstab1..4, mip_active,
  mip_inactive, 0 <= z <= 1 and the cut rows (eq. cuts), solved by HiGHS.
  Theorem 3.1 says the bound never exceeds this value (weak duality).
* ``mip_value``: the same with z binary for the unstable neurons
  (eqs. mip_output..mip_inactive), by HiGHS branch and bound, and
  ``mip_value_enum``: by enumerating every activation pattern of the
  unstable neurons with one LP each (tiny nets).
* ``sampled_min``: min of c^T f(x) over random points and vertices of the
  box, keeping only points that satisfy the domain's split constraints.

Splits enter as extra rows (x_j <= 0 or -x_j <= 0) and fix the neuron's
class; the z of a neuron that is active (inactive) in the subdomain is
fixed at 1 (0).  Conv edges are expanded to explicit matrices here by
plain loops over output positions.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sps
from scipy.optimize import Bounds, LinearConstraint, linprog, milp

from .gcp_oracle import ACTIVE, INACTIVE, UNSTABLE, root_classes


def edge_matrix(e, dst_shape, src_shape):
    """Explicit matrix of an edge's linear map x_hat_src -> x_dst."""
    dsrc = int(np.prod(src_shape))
    ddst = int(np.prod(dst_shape))
    if e.kind == "identity":
        return np.eye(ddst, dsrc)
    if e.kind == "dense":
        return np.asarray(e.W, np.float64)
    co, ho, wo = dst_shape
    ci, hi, wi = src_shape
    kh, kw = e.W.shape[2], e.W.shape[3]
    A = np.zeros((ddst, dsrc))
    for o in range(co):
        for y in range(ho):
            for x in range(wo):
                r = (o * ho + y) * wo + x
                for c in range(ci):
                    for ky in range(kh):
                        iy = y * e.stride - e.pad + ky
                        if iy < 0 or iy >= hi:
                            continue
                        for kx in range(kw):
                            ix = x * e.stride - e.pad + kx
                            if ix < 0 or ix >= wi:
                                continue
                            A[r, (c * hi + iy) * wi + ix] += e.W[o, c, ky, kx]
    return A


def plain_forward(net, x, return_pre=False):
    """Network evaluation with explicit matrices; x [n, d0]."""
    x = np.asarray(x, np.float64).reshape(-1, net.in_size)
    post = {-1: x}
    pre_all = {}
    out = None
    for i, node in enumerate(net.nodes):
        pre = np.tile(node.bias, (x.shape[0], 1))
        for e in node.edges:
            pre = pre + post[e.src] @ edge_matrix(e, node.shape, net.shape_of(e.src)).T
        pre_all[i] = pre
        if node.relu:
            post[i] = np.maximum(pre, 0.0)
        else:
            out = pre
    return (out, pre_all) if return_pre else out


class _Layout:
    def __init__(self, net):
        self.d0 = net.in_size
        self.relu = [i for i, n in enumerate(net.nodes) if n.relu]
        self.off = {}
        o = self.d0
        for p in self.relu:
            d = net.nodes[p].size
            self.off[p] = (o, o + d, o + 2 * d)   # x, x_hat, z
            o += 3 * d
        self.n = o

    def xhat(self, src):
        return (0, self.d0) if src < 0 else (self.off[src][1], None)


def _build(prob, b, s, integer=False, fixed_z=None):
    """Assemble the LP (or MIP) of domain b, spec row s."""
    net = prob.net
    L = _Layout(net)
    n = L.n
    lo = np.full(n, -np.inf)
    hi = np.full(n, np.inf)
    lo[:L.d0] = prob.x0 - prob.eps
    hi[:L.d0] = prob.x0 + prob.eps
    eq_rows, eq_rhs, in_rows, in_rhs = [], [], [], []
    integrality = np.zeros(n)
    sp = prob.splits
    split_of = {}
    for k in range(sp.K):
        if sp.node[b, k] >= 0:
            split_of[(int(sp.node[b, k]), int(sp.neuron[b, k]))] = int(sp.sign[b, k])
    mats = {}
    zpos = []

    def src_cols(src, size):
        if src < 0:
            return np.arange(L.d0)
        return L.off[src][1] + np.arange(size)

    for k, p in enumerate(L.relu):
        node = net.nodes[p]
        d = node.size
        ox, oh, oz = L.off[p]
        # x_p - sum_e A_e x_hat_src = b_p
        Arow = sps.lil_matrix((d, n))
        for j in range(d):
            Arow[j, ox + j] = 1.0
        for e in node.edges:
            A = edge_matrix(e, node.shape, net.shape_of(e.src))
            cols = src_cols(e.src, A.shape[1])
            Arow[:, cols] = Arow[:, cols] - A
        eq_rows.append(Arow.tocsr())
        eq_rhs.append(node.bias.copy())
        l, u = prob.lu[k]
        cls = root_classes(l, u)
        for j in range(d):
            c = cls[j]
            sg = split_of.get((p, j))
            if sg is not None:
                c = ACTIVE if sg > 0 else INACTIVE
                r = sps.lil_matrix((1, n))
                r[0, ox + j] = -1.0 if sg > 0 else 1.0   # -x <= 0  or  x <= 0
                in_rows.append(r.tocsr())
                in_rhs.append(0.0)
            if c == ACTIVE:
                r = sps.lil_matrix((1, n))
                r[0, oh + j] = 1.0
                r[0, ox + j] = -1.0
                eq_rows.append(r.tocsr())
                eq_rhs.append(np.zeros(1))
                lo[oz + j] = hi[oz + j] = 1.0
            elif c == INACTIVE:
                lo[oh + j] = hi[oh + j] = 0.0
                lo[oz + j] = hi[oz + j] = 0.0
            else:
                lo[oz + j], hi[oz + j] = 0.0, 1.0
                zpos.append(oz + j)
                if integer:
                    integrality[oz + j] = 1
                rows = [  # (x, xh, z) coefficients, rhs
                    ((0.0, -1.0, 0.0), 0.0),
                    ((1.0, -1.0, 0.0), 0.0),
                    ((0.0, 1.0, -u[j]), 0.0),
                    ((-1.0, 1.0, -l[j]), -l[j]),
                ]
                for (cx, ch, cz), rhs in rows:
                    r = sps.lil_matrix((1, n))
                    if cx:
                        r[0, ox + j] = cx
                    if ch:
                        r[0, oh + j] = ch
                    if cz:
                        r[0, oz + j] = cz
                    in_rows.append(r.tocsr())
                    in_rhs.append(rhs)
    if fixed_z is not None:
        for pos, val in zip(zpos, fixed_z):
            lo[pos] = hi[pos] = float(val)
    # cuts
    cu = prob.cuts
    if cu.n:
        Cm = sps.lil_matrix((cu.n, n))
        for e in range(cu.cut.size):
            nd, j, kd = int(cu.node[e]), int(cu.neuron[e]), int(cu.kind[e])
            if nd < 0:
                col = j
            else:
                ox, oh, oz = L.off[nd]
                col = (ox, oh, oz)[kd] + j
            Cm[int(cu.cut[e]), col] += cu.coef[e]
        in_rows.append(Cm.tocsr())
        in_rhs.append(cu.d.copy())
    # objective c^T (sum_e A_e x_hat_src + b_out)
    out = net.nodes[-1]
    cvec = prob.C[s]
    obj = np.zeros(n)
    const = float(cvec @ out.bias)
    for e in out.edges:
        A = edge_matrix(e, out.shape, net.shape_of(e.src))
        cols = src_cols(e.src, A.shape[1])
        obj[cols] += cvec @ A
    Aeq = sps.vstack(eq_rows).tocsr()
    beq = np.concatenate([np.atleast_1d(x) for x in eq_rhs])
    Aub = sps.vstack(in_rows).tocsr() if in_rows else None
    bub = np.concatenate([np.atleast_1d(x) for x in in_rhs]) if in_rhs else None
    return obj, const, Aeq, beq, Aub, bub, lo, hi, integrality, zpos


def lp_value(prob, b=0, s=0):
    """f*_LP-cut of one (domain, spec row); +inf if the LP is infeasible."""
    obj, const, Aeq, beq, Aub, bub, lo, hi, _, _ = _build(prob, b, s)
    res = linprog(obj, A_ub=Aub, b_ub=bub, A_eq=Aeq, b_eq=beq,
                  bounds=list(zip(lo, hi)), method="highs")
    if res.status == 2:
        return np.inf
    assert res.status == 0, res.message
    return res.fun + const


def mip_value(prob, b=0, s=0):
    """f*_MIP by HiGHS branch and bound; +inf if infeasible."""
    obj, const, Aeq, beq, Aub, bub, lo, hi, integ, _ = _build(prob, b, s, integer=True)
    cons = [LinearConstraint(Aeq, beq, beq)]
    if Aub is not None:
        cons.append(LinearConstraint(Aub, -np.inf, bub))
    res = milp(obj, constraints=cons, integrality=integ, bounds=Bounds(lo, hi),
               options=dict(mip_rel_gap=0.0))
    if res.status == 2:
        return np.inf
    assert res.status == 0, res.message
    return res.fun + const


def mip_value_enum(prob, b=0, s=0, max_unstable=12):
    """f*_MIP as the minimum over all z patterns of the unstable neurons,
    one LP per pattern."""
    obj, const, Aeq, beq, Aub, bub, lo, hi, _, zpos = _build(prob, b, s)
    assert len(zpos) <= max_unstable
    best = np.inf
    for pat in itertools.product((0.0, 1.0), repeat=len(zpos)):
        lo2, hi2 = lo.copy(), hi.copy()
        for pos, v in zip(zpos, pat):
            lo2[pos] = hi2[pos] = v
        res = linprog(obj, A_ub=Aub, b_ub=bub, A_eq=Aeq, b_eq=beq,
                      bounds=list(zip(lo2, hi2)), method="highs")
        if res.status == 0:
            best = min(best, res.fun + const)
    return best


def cut_max(prob, k, b=0):
    """max of cut k's left side over the MIP of domain b (to make tight cuts)."""
    obj, const, Aeq, beq, Aub, bub, lo, hi, integ, _ = _build(prob, b, 0, integer=True)
    cu = prob.cuts
    sel = cu.cut == k
    L = _Layout(prob.net)
    w = np.zeros(L.n)
    for e in np.nonzero(sel)[0]:
        nd, j, kd = int(cu.node[e]), int(cu.neuron[e]), int(cu.kind[e])
        col = j if nd < 0 else L.off[nd][kd] + j
        w[col] += cu.coef[e]
    cons = [LinearConstraint(Aeq, beq, beq)]
    res = milp(-w, constraints=cons + ([LinearConstraint(Aub, -np.inf, bub)] if Aub is not None else []),
               integrality=integ, bounds=Bounds(lo, hi), options=dict(mip_rel_gap=0.0))
    assert res.status == 0, res.message
    return -res.fun


def sampled_min(prob, b=0, n=100000, seed=0, vertices=True):
    """min over sampled box points (and all vertices when d0 <= 12) of
    c_s^T f(x) for every spec row s, over points meeting domain b's splits.
    Returns [S] (inf where no sample met the splits)."""
    rng = np.random.default_rng(seed)
    d0 = prob.net.in_size
    X = prob.x0 + prob.eps * (2.0 * rng.random((n, d0)) - 1.0)
    if vertices and d0 <= 12:
        V = np.array(list(itertools.product((-1.0, 1.0), repeat=d0)))
        X = np.vstack([X, prob.x0 + prob.eps * V])
    out, pre = plain_forward(prob.net, X, return_pre=True)
    ok = np.ones(X.shape[0], bool)
    sp = prob.splits
    for k in range(sp.K):
        if sp.node[b, k] >= 0:
            xv = pre[int(sp.node[b, k])][:, int(sp.neuron[b, k])]
            ok &= (xv >= 0) if sp.sign[b, k] > 0 else (xv <= 0)
    vals = out[ok] @ prob.C.T
    if vals.shape[0] == 0:
        return np.full(prob.S, np.inf)
    return vals.min(0)
