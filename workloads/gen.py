"""Seeded synthetic workloads shaped like the paper's verification problems.

Everything here is *input*: a ReLU network (Sec. 2, "The NN verification
problem"), an L-inf box around x0, margin specification rows e_y - e_j,
root pre-activation bounds l <= x <= u obtained by interval arithmetic
(IBP, one of the cheap methods the paper names for them in Sec. 2), BaB
split domains (Appendix B, Fig. 3) and valid cutting planes (eq. "cuts").

The cutting planes are nonnegative combinations of the LP-relaxation rows
of root-unstable neurons (eqs. mip_unstab1..mip_unstab4 plus 0 <= z <= 1),
so each is implied by the LP and therefore valid for the MIP.  Like the
cuts in the paper's case study (Appendix C.2) they span several layers and
every cut has an integer-variable (z) term.

Random streams: numpy.random.default_rng over SeedSequence(seed).spawn(5)
for (weights, x0, cuts, splits, parameters), so each part is reproducible
on its own.  Nothing in this module evaluates the GCP-CROWN bound.
"""
from __future__ import annotations

import hashlib
import math
import os
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

# ---------------------------------------------------------------------------
# Network description
# ---------------------------------------------------------------------------

KIND_H, KIND_G, KIND_Q = 0, 1, 2   # cut coefficient on x (pre), x_hat (post), z


@dataclass
class Edge:
    """One linear input of a node: x_node += op(x_hat_src).

    src = -1 is the network input.  kind is 'dense' (W is [out, in]),
    'conv' (W is [c_out, c_in, kh, kw], with stride and pad, no dilation)
    or 'identity'.
    """
    src: int
    kind: str
    W: Optional[np.ndarray] = None
    stride: int = 1
    pad: int = 0


@dataclass
class Node:
    """A layer x = sum_e op_e(x_hat_src(e)) + bias, followed by a ReLU
    unless it is the network output (the last node)."""
    shape: Tuple[int, ...]
    bias: np.ndarray
    edges: List[Edge]
    relu: bool = True

    @property
    def size(self) -> int:
        return int(np.prod(self.shape))


@dataclass
class Net:
    in_shape: Tuple[int, ...]
    nodes: List[Node]

    @property
    def in_size(self) -> int:
        return int(np.prod(self.in_shape))

    @property
    def relu_nodes(self) -> List[int]:
        return [i for i, n in enumerate(self.nodes) if n.relu]

    def shape_of(self, src: int) -> Tuple[int, ...]:
        return self.in_shape if src < 0 else self.nodes[src].shape


@dataclass
class Splits:
    """BaB split constraints, up to K per domain.

    node[b, k], neuron[b, k]: the split neuron (node = -1 marks an unused
    slot).  sign[b, k] = +1 for the split x >= 0, -1 for x <= 0."""
    node: np.ndarray    # int32 [B, K]
    neuron: np.ndarray  # int32 [B, K]
    sign: np.ndarray    # int8  [B, K]

    @property
    def B(self) -> int:
        return self.node.shape[0]

    @property
    def K(self) -> int:
        return self.node.shape[1]


@dataclass
class Cuts:
    """N cuts  sum_i H^(i) x^(i) + G^(i) x_hat^(i) + Q^(i) z^(i) <= d  in
    coordinate form: entry e adds coef[e] * var(kind[e]) of neuron
    neuron[e] of node node[e] to the left side of cut cut[e].  node = -1
    with kind G is a coefficient on the network input x."""
    n: int
    cut: np.ndarray     # int32 [nnz]
    node: np.ndarray    # int32 [nnz]
    neuron: np.ndarray  # int32 [nnz]
    kind: np.ndarray    # int8  [nnz]
    coef: np.ndarray    # float64 [nnz]
    d: np.ndarray       # float64 [N]

    @staticmethod
    def empty() -> "Cuts":
        z = np.zeros(0, np.int32)
        return Cuts(0, z, z.copy(), z.copy(), np.zeros(0, np.int8),
                    np.zeros(0), np.zeros(0))


@dataclass
class Problem:
    name: str
    net: Net
    lu: List[Tuple[np.ndarray, np.ndarray]]   # root bounds per ReLU node
    x0: np.ndarray
    eps: float
    C: np.ndarray                              # [S, d_out]
    splits: Splits
    cuts: Cuts
    alpha_init: str                            # 'crown' or 'given'
    alpha: Optional[np.ndarray]                # [B, S, n_I] when 'given'
    beta: np.ndarray                           # [B, S, K]
    gamma: np.ndarray                          # [B, S, N]
    opt: dict = field(default_factory=dict)

    @property
    def B(self) -> int:
        return self.splits.B

    @property
    def S(self) -> int:
        return self.C.shape[0]


# ---------------------------------------------------------------------------
# Plain network evaluation (used for the spec choice and for IBP)
# ---------------------------------------------------------------------------

def _apply_edge(e: Edge, xs: np.ndarray, src_shape, positive: Optional[bool] = None):
    """Apply op_e to a batch xs [n, prod(src_shape)] (float64)."""
    import torch
    W = e.W
    if e.kind == "identity":
        return xs
    if positive is True:
        W = np.maximum(W, 0.0)
    elif positive is False:
        W = np.minimum(W, 0.0)
    if e.kind == "dense":
        return xs @ W.T
    if e.kind == "conv":
        t = torch.from_numpy(np.ascontiguousarray(xs)).reshape((xs.shape[0],) + tuple(src_shape))
        y = torch.nn.functional.conv2d(t, torch.from_numpy(np.ascontiguousarray(W)),
                                       stride=e.stride, padding=e.pad)
        return y.reshape(xs.shape[0], -1).numpy()
    raise ValueError(e.kind)


def forward(net: Net, x: np.ndarray) -> np.ndarray:
    """Evaluate the network on a batch x [n, d0]; returns [n, d_out]."""
    x = np.asarray(x, np.float64).reshape(-1, net.in_size)
    post = {-1: x}
    out = None
    for i, node in enumerate(net.nodes):
        pre = np.broadcast_to(node.bias, (x.shape[0], node.size)).copy()
        for e in node.edges:
            pre += _apply_edge(e, post[e.src], net.shape_of(e.src))
        if node.relu:
            post[i] = np.maximum(pre, 0.0)
        else:
            out = pre
    return out


def ibp_bounds(net: Net, x0: np.ndarray, eps: float):
    """Interval bounds on every ReLU node's pre-activation over the box."""
    lo = {-1: (x0 - eps)[None, :]}
    hi = {-1: (x0 + eps)[None, :]}
    lu = []
    for i, node in enumerate(net.nodes):
        if not node.relu:
            continue
        l = np.broadcast_to(node.bias, (1, node.size)).copy()
        u = l.copy()
        for e in node.edges:
            sh = net.shape_of(e.src)
            if e.kind == "identity":
                l += lo[e.src]
                u += hi[e.src]
            else:
                l += _apply_edge(e, lo[e.src], sh, True) + _apply_edge(e, hi[e.src], sh, False)
                u += _apply_edge(e, hi[e.src], sh, True) + _apply_edge(e, lo[e.src], sh, False)
        l, u = _f32_down(l), _f32_up(u)
        lu.append((l[0].copy(), u[0].copy()))
        lo[i] = np.maximum(l, 0.0)
        hi[i] = np.maximum(u, 0.0)
    return lu


def unstable_index(lu):
    """Position of each root-unstable neuron (l < 0 < u) in the flat alpha
    vector, node-major and neuron-ascending; -1 elsewhere.  This is the
    layout convention of the alpha argument, not a bound computation."""
    idx, off = [], 0
    for l, u in lu:
        m = (l < 0) & (u > 0)
        a = np.full(l.shape[0], -1, np.int64)
        a[m] = off + np.arange(int(m.sum()))
        off += int(m.sum())
        idx.append(a)
    return idx, off


def num_relu_neurons(net: Net) -> int:
    return sum(n.size for n in net.nodes if n.relu)


# ---------------------------------------------------------------------------
# Network builders
# ---------------------------------------------------------------------------

def _f32(a):
    """Values exactly representable in fp32 (kept as float64), so a device
    copy in fp32 holds the very same numbers the fp64 oracle uses."""
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


def _f32_down(a):
    f = np.asarray(a, np.float64).astype(np.float32)
    f = np.where(f.astype(np.float64) > a, np.nextafter(f, np.float32(-np.inf)), f)
    return f.astype(np.float64)


def _f32_up(a):
    f = np.asarray(a, np.float64).astype(np.float32)
    f = np.where(f.astype(np.float64) < a, np.nextafter(f, np.float32(np.inf)), f)
    return f.astype(np.float64)


def _bias(rng, n, var=0.1):
    return _f32(rng.normal(0.0, math.sqrt(var), n))


def mlp_net(rng, dims, w_var_num=2.0, b_var=0.1) -> Net:
    """Dense ReLU chain dims[0] -> ... -> dims[-1]; W ~ N(0, w_var_num/fan_in)."""
    nodes = []
    for k in range(1, len(dims)):
        fan_in = dims[k - 1]
        W = _f32(rng.normal(0.0, math.sqrt(w_var_num / fan_in), (dims[k], fan_in)))
        nodes.append(Node((dims[k],), _bias(rng, dims[k], b_var),
                          [Edge(k - 2, "dense", W)], relu=(k < len(dims) - 1)))
    return Net((dims[0],), nodes)


def _conv_out(h, k, s, p):
    return (h + 2 * p - k) // s + 1


def _conv_w(rng, co, ci, k):
    return _f32(rng.normal(0.0, math.sqrt(2.0 / (ci * k * k)), (co, ci, k, k)))


def cnn_net(rng, in_shape=(3, 32, 32), convs=((16, 4, 2, 1), (32, 4, 2, 1)), fcs=(100, 10)) -> Net:
    """Conv layers (c_out, k, stride, pad) with ReLU, then dense layers; the
    last dense layer is the output."""
    nodes = []
    c, h = in_shape[0], in_shape[1]
    src = -1
    for co, k, s, p in convs:
        ho = _conv_out(h, k, s, p)
        nodes.append(Node((co, ho, ho), _bias(rng, co * ho * ho), [Edge(src, "conv", _conv_w(rng, co, c, k), s, p)]))
        src = len(nodes) - 1
        c, h = co, ho
    d = c * h * h
    for i, f in enumerate(fcs):
        nodes.append(Node((f,), _bias(rng, f), [Edge(src, "dense", _f32(rng.normal(0, math.sqrt(2.0 / d), (f, d))))],
                          relu=(i < len(fcs) - 1)))
        src = len(nodes) - 1
        d = f
    return Net(tuple(in_shape), nodes)


def cnn_wide_net(rng) -> Net:
    """Conv(3,16,4,s2,p1) - Conv(16,32,4,s2,p1) - Linear(2048,100) - Linear(100,10):
    the 'Wide' / CNN-A shape of Table 4 with padding 1 (2048 = 32*8*8)."""
    return cnn_net(rng)


def resnet_net(rng, stem=16, stages=(16, 32, 64), hw=32, in_ch=3) -> Net:
    """Stem Conv(3,stem,3) then one residual block per stage, stride 2
    between stages, then Linear(c*h*w, 10).  Block (an assumed reading of
    'ResBlock'): y = ReLU(conv2(ReLU(conv1 x)) + skip(x)), 3x3 convs with
    padding 1, skip = identity or a 1x1 stride-2 conv when the shape changes."""
    nodes = [Node((stem, hw, hw), _bias(rng, stem * hw * hw),
                  [Edge(-1, "conv", _conv_w(rng, stem, in_ch, 3), 1, 1)])]
    c, h, src = stem, hw, 0
    for si, co in enumerate(stages):
        s = 1 if si == 0 else 2
        ho = _conv_out(h, 3, s, 1)
        a = Node((co, ho, ho), _bias(rng, co * ho * ho), [Edge(src, "conv", _conv_w(rng, co, c, 3), s, 1)])
        nodes.append(a)
        ia = len(nodes) - 1
        edges = [Edge(ia, "conv", _conv_w(rng, co, co, 3), 1, 1)]
        if s == 1 and co == c:
            edges.append(Edge(src, "identity"))
        else:
            edges.append(Edge(src, "conv", _conv_w(rng, co, c, 1), s, 0))
        nodes.append(Node((co, ho, ho), _bias(rng, co * ho * ho), edges))
        src = len(nodes) - 1
        c, h = co, ho
    d = c * h * h
    nodes.append(Node((10,), _bias(rng, 10), [Edge(src, "dense", _f32(rng.normal(0, math.sqrt(2.0 / d), (10, d))))],
                      relu=False))
    return Net((in_ch, hw, hw), nodes)


# ---------------------------------------------------------------------------
# Specification, splits, cuts
# ---------------------------------------------------------------------------

def margin_spec(net: Net, x0: np.ndarray, S: Optional[int] = None) -> np.ndarray:
    """Rows e_y - e_j for the non-target classes j, y = argmax f(x0)."""
    f = forward(net, x0[None, :])[0]
    y = int(np.argmax(f))
    d = f.shape[0]
    rows = []
    for j in range(d):
        if j == y:
            continue
        r = np.zeros(d)
        r[y] = 1.0
        r[j] = -1.0
        rows.append(r)
    C = np.array(rows)
    return C if S is None else C[:S]


def _unstable_list(lu):
    out = []
    for p, (l, u) in enumerate(lu):
        for j in np.nonzero((l < 0) & (u > 0))[0]:
            out.append((p, int(j)))
    return out


def make_splits(rng, lu, relu_nodes, B, kmin, kmax) -> Splits:
    """Each domain splits kmin..kmax distinct root-unstable neurons, each
    with a random side (x >= 0 or x <= 0)."""
    cand = _unstable_list(lu)
    K = kmax
    node = np.full((B, K), -1, np.int32)
    neuron = np.zeros((B, K), np.int32)
    sign = np.zeros((B, K), np.int8)
    if K == 0 or not cand:
        return Splits(node, neuron, sign)
    for b in range(B):
        m = int(rng.integers(kmin, kmax + 1))
        m = min(m, len(cand))
        pick = rng.choice(len(cand), size=m, replace=False)
        for k, c in enumerate(pick):
            p, j = cand[c]
            node[b, k] = relu_nodes[p]
            neuron[b, k] = j
            sign[b, k] = 1 if rng.random() < 0.5 else -1
    return Splits(node, neuron, sign)


def make_cuts(rng, lu, relu_nodes, n_cuts, kmin, kmax, multi_layer=True,
              input_terms=0, x0=None, eps=None) -> Cuts:
    """n_cuts LP-implied cuts, each over kmin..kmax root-unstable neurons.

    For one unstable neuron (l < 0 < u) the LP rows (all '<=') are
      -x_hat <= 0;  x - x_hat <= 0;  x_hat - u z <= 0;
      x_hat - x - l z <= -l;  z <= 1;  -z <= 0.
    A cut adds each row with a weight in U[0,1] (a row is dropped with
    probability 1/3).  With input_terms > 0 a cut also adds that many
    input-box rows  +-x_k <= x0_k + eps  /  -x0_k + eps  (coefficients on
    the network input, node = -1)."""
    cand = _unstable_list(lu)
    by_node = {}
    for p, j in cand:
        by_node.setdefault(p, []).append(j)
    nodes_avail = sorted(by_node)
    acc = {}
    d = np.zeros(n_cuts)
    if not cand:
        return Cuts.empty()

    def add(k, node, j, kind, c):
        key = (k, node, j, kind)
        acc[key] = acc.get(key, 0.0) + c

    for k in range(n_cuts):
        m = int(rng.integers(kmin, kmax + 1))
        m = min(m, len(cand))
        chosen = set()
        if multi_layer and len(nodes_avail) >= 2:
            two = rng.choice(len(nodes_avail), size=2, replace=False)
            for t in two:
                p = nodes_avail[t]
                chosen.add((p, int(rng.choice(by_node[p]))))
        while len(chosen) < m:
            chosen.add(cand[int(rng.integers(len(cand)))])
        for p, j in sorted(chosen):
            l, u = lu[p][0][j], lu[p][1][j]
            w = rng.random(6)
            keep = rng.random(6) >= 1.0 / 3.0
            if not keep.any():
                keep[int(rng.integers(6))] = True
            w = w * keep
            nd = relu_nodes[p]
            # -x_hat <= 0
            add(k, nd, j, KIND_G, -w[0])
            # x - x_hat <= 0
            add(k, nd, j, KIND_H, w[1]); add(k, nd, j, KIND_G, -w[1])
            # x_hat - u z <= 0
            add(k, nd, j, KIND_G, w[2]); add(k, nd, j, KIND_Q, -w[2] * u)
            # x_hat - x - l z <= -l
            add(k, nd, j, KIND_G, w[3]); add(k, nd, j, KIND_H, -w[3]); add(k, nd, j, KIND_Q, -w[3] * l)
            d[k] += -w[3] * l
            # z <= 1 ; -z <= 0
            add(k, nd, j, KIND_Q, w[4] - w[5])
            d[k] += w[4]
        for _ in range(input_terms):
            q = int(rng.integers(x0.shape[0]))
            w = rng.random()
            if rng.random() < 0.5:
                add(k, -1, q, KIND_G, w); d[k] += w * (x0[q] + eps)
            else:
                add(k, -1, q, KIND_G, -w); d[k] += w * (-x0[q] + eps)
    # Coefficients are rounded to fp32 values (the device stores fp32) and each
    # cut's offset is widened by |rounded - exact| times the largest magnitude
    # the variable takes (|x| <= max(|l|, |u|), 0 <= x_hat <= max(u, 0),
    # 0 <= z <= 1, inputs within the box), so the rounded cut is still valid
    # and both sides of every comparison see the same numbers.
    pos = {nd: p for p, nd in enumerate(relu_nodes)}
    keys = sorted(k for k, v in acc.items() if np.float32(v) != 0.0)
    coef = np.array([acc[k] for k in keys], np.float64)
    c32 = _f32(coef)
    for (k, node, j, kind), c, c_r in zip(keys, coef, c32):
        if c == c_r:
            continue
        if node < 0:
            rng_ = max(abs(x0[j] - eps), abs(x0[j] + eps))
        else:
            l, u = lu[pos[node]][0][j], lu[pos[node]][1][j]
            rng_ = max(abs(l), abs(u)) if kind == KIND_H else (max(u, 0.0) if kind == KIND_G else 1.0)
        d[k] += abs(c_r - c) * rng_
    return Cuts(
        n_cuts,
        np.array([k[0] for k in keys], np.int32),
        np.array([k[1] for k in keys], np.int32),
        np.array([k[2] for k in keys], np.int32),
        np.array([k[3] for k in keys], np.int8),
        c32,
        d,
    )


# ---------------------------------------------------------------------------
# The workload configurations
# ---------------------------------------------------------------------------

OPT_DEFAULT = dict(iters=20, lr_alpha=0.1, lr_mult=0.02, decay=0.9,
                   adam_b1=0.9, adam_b2=0.999, adam_eps=1e-8)


def make_problem(name, net, x0, eps, S, B, kmin_split, kmax_split, n_cuts,
                 cut_kmin, cut_kmax, streams, alpha_init="crown",
                 beta_dist="uniform", gamma_dist="zero", input_terms=0, lu=None) -> Problem:
    """A problem on `net` around x0; root bounds `lu` as given, else by
    interval arithmetic."""
    r_cut, r_split, r_par = streams
    x0 = _f32(x0)
    if lu is None:
        lu = ibp_bounds(net, x0, eps)
    rel = net.relu_nodes
    C = margin_spec(net, x0, S)
    splits = make_splits(r_split, lu, rel, B, kmin_split, kmax_split)
    cuts = make_cuts(r_cut, lu, rel, n_cuts, cut_kmin, cut_kmax,
                     input_terms=input_terms, x0=x0, eps=eps)
    _, n_I = unstable_index(lu)
    S = C.shape[0]
    alpha = None
    if alpha_init == "given":
        alpha = _f32(r_par.random((B, S, n_I)))
    K = splits.K
    if beta_dist == "uniform":
        beta = _f32(r_par.random((B, S, K))) * (splits.node >= 0)[:, None, :]
    else:
        beta = np.zeros((B, S, K))
    if gamma_dist == "uniform":
        gamma = _f32(r_par.random((B, S, cuts.n)))
    else:
        gamma = np.zeros((B, S, cuts.n))
    return Problem(name, net, lu, x0, float(eps), C, splits, cuts, alpha_init,
                   alpha, beta, gamma, dict(OPT_DEFAULT))


def crown_alpha_init(lu):
    """The usual CROWN-adaptive lower slope per root-unstable neuron:
    1 where u >= -l, else 0 (a starting point for the optimiser only)."""
    out = []
    for l, u in lu:
        m = (l < 0) & (u > 0)
        out.append((u[m] >= -l[m]).astype(np.float64))
    return np.concatenate(out) if out else np.zeros(0)


def rho_init(lu):
    """Starting rho of the explicit-pi form per root-unstable neuron:
    u / (u - l), the upper relaxation's slope (a starting point only)."""
    out = []
    for l, u in lu:
        m = (l < 0) & (u > 0)
        out.append(u[m] / (u[m] - l[m]))
    return np.concatenate(out) if out else np.zeros(0)


def _streams(seed):
    ss = np.random.SeedSequence(seed).spawn(5)
    return [np.random.default_rng(s) for s in ss]


WORKLOAD_NAMES = ("mlp8", "mlp784", "cnn", "batch", "resnet")
DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


def workload_net(name: str, seed: int = 0):
    """The network, centre x0 (fp32 values) and radius of a named workload."""
    r_w, r_x = _streams(seed)[:2]
    if name == "mlp784":
        return mlp_net(r_w, [784] + [256] * 6 + [10]), _f32(r_x.random(784)), 0.015
    if name == "cnn":
        return cnn_wide_net(r_w), _f32(r_x.random(3 * 32 * 32)), 2.0 / 255.0
    if name == "resnet":
        return resnet_net(r_w), _f32(r_x.random(3 * 32 * 32)), 2.0 / 255.0
    raise ValueError(f"no stored root bounds for workload {name!r}")


def inputs_digest(net: Net, x0, eps) -> str:
    """Fingerprint of what root bounds depend on (weights, biases, x0, eps),
    stored beside them so a changed generator cannot pick up stale bounds."""
    h = hashlib.sha256()
    for n in net.nodes:
        h.update(np.ascontiguousarray(n.bias, np.float64).tobytes())
        for e in n.edges:
            h.update(f"{e.src}:{e.kind}:{e.stride}:{e.pad}".encode())
            if e.W is not None:
                h.update(np.ascontiguousarray(e.W, np.float64).tobytes())
    h.update(np.ascontiguousarray(x0, np.float64).tobytes())
    h.update(repr(float(eps)).encode())
    return h.hexdigest()


def root_bounds_path(name: str, seed: int = 0) -> str:
    return os.path.join(DATA, f"{name}_s{seed}_crown_roots.npz")


def load_root_bounds(name: str, seed: int, net: Net, x0, eps):
    """Stored CROWN root bounds of a workload (written by oracle/root_bounds.py
    from the float64 oracle; fp32 values rounded outward), checked against the
    network they were computed for."""
    path = root_bounds_path(name, seed)
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: run `python -m oracle.root_bounds {name}`")
    with np.load(path, allow_pickle=False) as z:
        if str(z["digest"]) != inputs_digest(net, x0, eps):
            raise ValueError(f"{path} was computed for another network or input")
        lu = []
        for i in range(len(net.relu_nodes)):
            lu.append((z[f"l{i}"].astype(np.float64), z[f"u{i}"].astype(np.float64)))
    return lu


def make_workload(name: str, seed: int = 0, B: Optional[int] = None, roots: str = "crown", **kw):
    """The named synthetic workloads (B overrides the number of domains):
      mlp8    MLP 8-16-16-3, one domain, S = 2, 8 cuts (small enough for exact
              LP / MIP checks);
      mlp784  MLP 784-256x6-10, 1024 domains, S = 9, 200 cuts;
      cnn     Conv(3,16,4,s2)-Conv(16,32,4,s2)-2048-100-10 on 3x32x32, 2048
              domains, 500 cuts;
      resnet  stem 16, residual blocks 16/32/64, linear 10 on 3x32x32, 4096
              domains, 1000 cuts;
      batch   64 uneven MLP instances (returns a list of Problems).
    roots: root bounds of mlp784, cnn and resnet -- "crown" (the stored
    float64 CROWN bounds, Sec. 2's intermediate bounds) or "ibp" (interval
    arithmetic); mlp8 and batch use interval arithmetic."""
    r_w, r_x, r_cut, r_split, r_par = _streams(seed)
    if name in ("mlp784", "cnn", "resnet") and roots == "crown":
        net, x0, eps = workload_net(name, seed)
        kw["lu"] = load_root_bounds(name, seed, net, x0, eps)
    elif roots not in ("crown", "ibp"):
        raise ValueError(f"roots must be 'crown' or 'ibp', not {roots!r}")
    if name == "mlp8":
        # W ~ N(0, 1/fan_in), b ~ N(0, 0.1); eps = 0.05; S = 2; one domain, no
        # splits; 8 cuts over 2-4 neurons; alpha, gamma ~ U[0,1]
        net = mlp_net(r_w, [8, 16, 16, 3], w_var_num=1.0)
        x0 = r_x.random(8)
        return make_problem("mlp8-16-16-3", net, x0, 0.05, 2, B or 1, 0, 0, 8, 2, 4,
                            (r_cut, r_split, r_par), alpha_init="given",
                            beta_dist="zero", gamma_dist="uniform", **kw)
    if name == "mlp784":
        net = mlp_net(r_w, [784] + [256] * 6 + [10])
        x0 = r_x.random(784)
        return make_problem("mlp784-256x6-10", net, x0, 0.015, 9, B or 1024, 1, 8, 200, 2, 6,
                            (r_cut, r_split, r_par), **kw)
    if name == "cnn":
        net = cnn_wide_net(r_w)
        x0 = r_x.random(3 * 32 * 32)
        return make_problem("cnn-3x32x32-c16-c32-2048-100-10", net, x0, 2.0 / 255.0, 9, B or 2048, 1, 8, 500,
                            2, 6, (r_cut, r_split, r_par), **kw)
    if name == "resnet":
        net = resnet_net(r_w)
        x0 = r_x.random(3 * 32 * 32)
        return make_problem("resnet-3x32x32-16-32-64", net, x0, 2.0 / 255.0, 9, B or 4096, 1, 8, 1000, 2, 6,
                            (r_cut, r_split, r_par), **kw)
    if name == "batch":
        return make_batch(seed, **kw)
    raise ValueError(f"unknown workload {name!r}; one of {WORKLOAD_NAMES}")


def make_batch(seed: int = 0, n_inst: int = 64, bmax: int = 4096,
                      bscale: float = 1.0) -> List[Problem]:
    """Uneven instances: MLP depth U{3..9} linear layers, hidden width
    U[64, 1024], input 784 (eps 0.015) or 3072 (eps 2/255), domains
    log-uniform in [16, bmax] (times bscale), cuts U{50..1000}, S = 9."""
    r = np.random.default_rng(np.random.SeedSequence([seed, 4]))
    out = []
    for i in range(n_inst):
        depth = int(r.integers(3, 10))
        width = int(r.integers(64, 1025))
        d0 = 784 if r.random() < 0.5 else 3072
        eps = 0.015 if d0 == 784 else 2.0 / 255.0
        B = int(round(math.exp(r.uniform(math.log(16), math.log(bmax)))))
        B = max(1, int(round(B * bscale)))
        n_cuts = int(r.integers(50, 1001))
        r_w, r_x, r_cut, r_split, r_par = _streams([seed, 4, i])
        net = mlp_net(r_w, [d0] + [width] * (depth - 1) + [10])
        x0 = r_x.random(d0)
        out.append(make_problem(f"batch-mlp-inst{i}", net, x0, eps, 9, B, 1, 8, n_cuts, 2, 6,
                                (r_cut, r_split, r_par)))
    return out


def make_tiny(kind: str, seed: int = 0, B: int = 1, splits=(0, 0), n_cuts: int = 4,
              cut_k=(2, 4), eps: float = 0.1, S: Optional[int] = None,
              alpha_init: str = "given", gamma_dist: str = "uniform",
              beta_dist: str = "uniform", input_terms: int = 0) -> Problem:
    """Small problems for exact (LP / MIP / enumeration) checks.
    kind: 'mlp' (6-8-8-3), 'cnn' (1x6x6, two convs, dense 5, out 3),
    'res' (1x4x4 stem, identity block, stride-2 block, out 3), or 'cnn16' /
    'res16' (the same structures on an 8x8 input, every spatial size a
    multiple of 16 positions)."""
    r_w, r_x, r_cut, r_split, r_par = _streams([seed, 99])
    if kind == "mlp":
        net = mlp_net(r_w, [6, 8, 8, 3], w_var_num=1.0)
    elif kind == "cnn":
        net = cnn_net(r_w, (1, 6, 6), ((2, 3, 2, 1), (3, 3, 1, 1)), (5, 3))
    elif kind == "cnn16":    # spatial sizes multiples of 16 positions
        net = cnn_net(r_w, (1, 8, 8), ((2, 4, 2, 1), (3, 3, 1, 1)), (5, 3))
    elif kind in ("res", "res16"):
        if kind == "res":
            net = resnet_net(r_w, stem=1, stages=(1, 2), hw=4, in_ch=1)
        else:
            net = resnet_net(r_w, stem=2, stages=(2, 3), hw=8, in_ch=1)
        last = net.nodes[-1]
        W = last.edges[0].W
        net.nodes[-1] = Node((3,), last.bias[:3], [Edge(last.edges[0].src, "dense", W[:3])], relu=False)
    else:
        raise ValueError(kind)
    x0 = r_x.random(net.in_size)
    return make_problem(f"tiny-{kind}", net, x0, eps, S, B, splits[0], splits[1], n_cuts,
                        cut_k[0], cut_k[1], (r_cut, r_split, r_par), alpha_init=alpha_init,
                        beta_dist=beta_dist, gamma_dist=gamma_dist, input_terms=input_terms)
