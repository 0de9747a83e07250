"""Root pre-activation bounds by layer-by-layer CROWN, float64 (test infrastructure only).

Sec. 2 takes the intermediate bounds l <= x^(i) <= u of every ReLU layer as
given, obtained from a cheaper bound method.  The benchmark workloads use
CROWN's, computed here node by node: the bounds of node k's pre-activation
are the Theorem 3.1 bound with beta = gamma = 0 and no splits (which is
CROWN, pinned against the independent primal form in ``crown.py``) of the
prefix network that ends at node k's pre-activation, for the spec rows +e_j
(lower bound) and -e_j (minus the upper bound), the earlier nodes carrying the
bounds already found and CROWN-adaptive lower slopes (1 where u >= -l,
else 0).  The results are rounded outward to fp32 values, so the device copy
and the float64 oracle see the very same numbers.

Run as a script it writes the stored root bounds of the benchmark workloads
(``workloads/data``), which the input generator reads:
    python -m oracle.root_bounds [mlp784 cnn resnet]
"""
from __future__ import annotations

import dataclasses
import os
import sys

import numpy as np
import torch

from . import gcp_oracle as O

DATA = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "workloads", "data")


def _down(a):
    f = np.asarray(a, np.float64).astype(np.float32)
    f = np.where(f.astype(np.float64) > a, np.nextafter(f, np.float32(-np.inf)), f)
    return f.astype(np.float64)


def _up(a):
    f = np.asarray(a, np.float64).astype(np.float32)
    f = np.where(f.astype(np.float64) < a, np.nextafter(f, np.float32(np.inf)), f)
    return f.astype(np.float64)


def crown_root_bounds(net, x0, eps, chunk=2048, log=None):
    """[(l, u)] for every ReLU node of ``net`` (a workloads.gen.Net) over the
    box |x - x0| <= eps, CROWN layer by layer, rounded outward to fp32."""
    from workloads import gen
    lu = []
    for pos, k in enumerate(net.relu_nodes):
        node = net.nodes[k]
        d = node.size
        prefix = gen.Net(net.in_shape, list(net.nodes[:k]) + [dataclasses.replace(node, relu=False)])
        lo, hi = np.empty(d), np.empty(d)
        for s0 in range(0, 2 * d, chunk):
            rows = np.arange(s0, min(2 * d, s0 + chunk))
            C = np.zeros((rows.size, d))
            C[np.arange(rows.size), rows % d] = np.where(rows < d, 1.0, -1.0)
            splits = gen.Splits(np.full((1, 0), -1, np.int32), np.zeros((1, 0), np.int32), np.zeros((1, 0), np.int8))
            prob = gen.Problem("prefix", prefix, list(lu), x0, float(eps), C, splits, gen.Cuts.empty(), "crown",
                               None, np.zeros((1, rows.size, 0)), np.zeros((1, rows.size, 0)))
            prep = O.Prepared(prob)
            a = torch.as_tensor(O.full_alpha(prob, prep).reshape(rows.size, -1))
            z = torch.zeros(rows.size, 0, dtype=torch.float64)
            with torch.no_grad():
                g = O.bound_rows(prob, a, z, z, prep).numpy()
            lo[rows[rows < d]] = g[rows < d]
            hi[rows[rows >= d] - d] = -g[rows >= d]
        bad = lo > hi   # an exactly determined pre-activation can come out a rounding error apart
        lo[bad], hi[bad] = hi[bad], lo[bad]
        lu.append((_down(lo), _up(hi)))
        if log:
            m = (lu[-1][0] < 0) & (lu[-1][1] > 0)
            log(f"  node {k}: {d} neurons, {int(m.sum())} unstable")
    return lu


def write(name, seed=0):
    from workloads import gen
    net, x0, eps = gen.workload_net(name, seed)
    print(f"{name} (seed {seed}): CROWN root bounds", flush=True)
    lu = crown_root_bounds(net, x0, eps, log=lambda m: print(m, flush=True))
    os.makedirs(DATA, exist_ok=True)
    arrs = {}
    for i, (l, u) in enumerate(lu):
        arrs[f"l{i}"] = l.astype(np.float32)
        arrs[f"u{i}"] = u.astype(np.float32)
    path = gen.root_bounds_path(name, seed)
    np.savez_compressed(path, digest=np.array(gen.inputs_digest(net, x0, eps)), **arrs)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    for nm in (sys.argv[1:] or ["mlp784", "cnn", "resnet"]):
        write(nm)
