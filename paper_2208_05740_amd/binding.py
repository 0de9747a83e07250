"""ctypes binding of libgcp.so (C ABI in include/gcp.h).

Argument marshalling only: every step of the bound pass, its adjoint and
the optimiser runs in the HIP library.  torch supplies device memory and the
current stream.  The library must be built (``python -m
paper_2208_05740_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgcp.so")

GCP_MODE_FP32 = 0
GCP_MODE_BF16 = 1
GCP_FLAG_VALIDATE = 0x100
GCP_FLAG_RECOMPUTE = 0x200     # recompute a_hat in the adjoint wherever possible
GCP_FLAG_STORE_AHAT = 0x400    # store a_hat of every layer
GCP_FLAG_OUTWARD = 0x800       # subtract the pass's rounding slack from every bound
GCP_FLAG_PERSIST = 0x1000      # iterations as one persistent dataflow launch (dense nets)
EDGE_KIND = {"dense": 0, "conv": 1, "identity": 2}
ERRORS = {-1: "EINVAL", -2: "ERANGE", -3: "ENONFINITE", -4: "ENOMEM", -5: "EDEVICE", -6: "EUNSUPPORTED"}


class GcpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class EdgeDesc(C.Structure):
    _fields_ = [("src", C.c_int32), ("kind", C.c_int32), ("W", C.POINTER(C.c_float)),
                ("kh", C.c_int32), ("kw", C.c_int32), ("stride", C.c_int32), ("pad", C.c_int32)]


class NodeDesc(C.Structure):
    _fields_ = [("c", C.c_int32), ("h", C.c_int32), ("w", C.c_int32),
                ("bias", C.POINTER(C.c_float)), ("lower", C.POINTER(C.c_double)),
                ("upper", C.POINTER(C.c_double)), ("n_edges", C.c_int32),
                ("edges", C.POINTER(EdgeDesc))]


class NetDesc(C.Structure):
    _fields_ = [("in_c", C.c_int32), ("in_h", C.c_int32), ("in_w", C.c_int32),
                ("n_nodes", C.c_int32), ("nodes", C.POINTER(NodeDesc))]


class NetInfo(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("in_size", C.c_int32), ("out_size", C.c_int32),
                ("n_relu", C.c_int64), ("n_unstable", C.c_int64)]


class OptDesc(C.Structure):
    _fields_ = [("iters", C.c_int32), ("lr_alpha", C.c_float), ("lr_mult", C.c_float),
                ("decay", C.c_float), ("adam_b1", C.c_float), ("adam_b2", C.c_float),
                ("adam_eps", C.c_float), ("use_graph", C.c_int32)]


class BatchItem(C.Structure):
    _fields_ = [("net", C.c_void_p), ("x0", C.c_void_p), ("eps", C.c_double), ("C", C.c_void_p), ("S", C.c_int32),
                ("splits", C.c_void_p), ("cuts", C.c_void_p), ("alpha", C.c_void_p), ("beta", C.c_void_p),
                ("gamma", C.c_void_p), ("adam_state", C.c_void_p), ("bound", C.c_void_p), ("verified", C.c_void_p)]


class BabOpt(C.Structure):
    _fields_ = [("batch", C.c_int32), ("max_depth", C.c_int32), ("max_domains", C.c_int64),
                ("max_pool", C.c_int64), ("retries", C.c_int32), ("opt", OptDesc), ("mode", C.c_int32)]


class BabResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("lower", C.c_double), ("bounded", C.c_int64), ("rounds", C.c_int64),
                ("max_open", C.c_int64), ("open", C.c_int64), ("unresolved", C.c_int64)]


GCP_BAB_VERIFIED = 1
GCP_BAB_UNKNOWN = 0

_LIB = None
EXPORTS = ["gcp_net_create", "gcp_net_destroy", "gcp_net_get_info", "gcp_cuts_create", "gcp_cuts_destroy",
           "gcp_splits_create", "gcp_splits_destroy", "gcp_bound", "gcp_optimize", "gcp_optimize_batch",
           "gcp_crown_bounds", "gcp_net_get_unstable", "gcp_cuts_info", "gcp_bab", "gcp_profile_enable",
           "gcp_profile_read", "gcp_last_error", "gcp_version"]


def lib():
    """Load libgcp.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2208_05740_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.gcp_net_create.argtypes = [C.POINTER(NetDesc), C.POINTER(vp)]
    L.gcp_net_destroy.argtypes = [vp]
    L.gcp_net_get_info.argtypes = [vp, C.POINTER(NetInfo)]
    L.gcp_cuts_create.argtypes = [vp, i32, i64, vp, vp, vp, vp, vp, vp, C.POINTER(vp)]
    L.gcp_cuts_destroy.argtypes = [vp]
    L.gcp_splits_create.argtypes = [vp, i32, i32, vp, vp, vp, C.POINTER(vp)]
    L.gcp_splits_destroy.argtypes = [vp]
    L.gcp_bound.argtypes = [vp, vp, dbl, vp, i32, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp]
    L.gcp_bound_noalloc.argtypes = L.gcp_bound.argtypes
    L.gcp_bound_noalloc.restype = C.c_int
    L.gcp_prepare.argtypes = [vp, i32, vp, vp, i32, i32, vp]
    L.gcp_prepare.restype = C.c_int
    L.gcp_optimize.argtypes = [vp, vp, dbl, vp, i32, vp, vp, vp, vp, vp, vp, C.POINTER(OptDesc), i32, vp, vp, vp]
    L.gcp_bound_pi.argtypes = [vp, vp, dbl, vp, i32, vp, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]
    L.gcp_optimize_pi.argtypes = [vp, vp, dbl, vp, i32, vp, vp, vp, vp, vp, vp, vp, C.POINTER(OptDesc), i32, vp, vp,
                                  vp]
    L.gcp_optimize_batch.argtypes = [i32, C.POINTER(BatchItem), C.POINTER(OptDesc), i32, vp]
    L.gcp_crown_bounds.argtypes = [C.POINTER(NetDesc), vp, dbl, C.POINTER(vp), C.POINTER(vp), i32, vp]
    L.gcp_crown_bounds_domain.argtypes = [C.POINTER(NetDesc), vp, dbl, i32, vp, vp, vp, C.POINTER(vp), C.POINTER(vp),
                                          i32, vp]
    L.gcp_net_get_unstable.argtypes = [vp, vp, vp, vp, vp]
    L.gcp_cuts_info.argtypes = [vp, C.POINTER(i32)]
    L.gcp_bab.argtypes = [vp, vp, dbl, vp, vp, C.POINTER(BabOpt), C.POINTER(BabResult), vp]
    L.gcp_profile_enable.argtypes = [i32]
    L.gcp_profile_read.argtypes = [i32, C.c_char_p, i32, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.gcp_last_error.restype = C.c_char_p
    L.gcp_version.restype = C.c_char_p
    for f in ("gcp_net_create", "gcp_net_destroy", "gcp_net_get_info", "gcp_cuts_create", "gcp_cuts_destroy",
              "gcp_splits_create", "gcp_splits_destroy", "gcp_bound", "gcp_optimize", "gcp_profile_enable",
              "gcp_profile_read", "gcp_optimize_batch", "gcp_crown_bounds", "gcp_net_get_unstable",
              "gcp_cuts_info", "gcp_bab"):
        getattr(L, f).restype = C.c_int
    _LIB = L
    return L


def _check(rc):
    if rc != 0:
        raise GcpError(rc, lib().gcp_last_error().decode())


def _ptr(a):
    """Data pointer of a numpy array or torch tensor (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def _net_desc(net, lu):
    """gcp_net_desc of a workloads.Net (root bounds from lu, or none); returns
    the descriptor and the host arrays it points into."""
    keep = []

    def f32(a):
        a = np.ascontiguousarray(a, np.float32)
        keep.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_float))

    def f64(a):
        a = np.ascontiguousarray(a, np.float64)
        keep.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_double))

    nodes = (NodeDesc * len(net.nodes))()
    relu_pos = 0
    edge_arrays = []
    for i, n in enumerate(net.nodes):
        shape = tuple(n.shape) if len(n.shape) == 3 else (n.size, 1, 1)
        edges = (EdgeDesc * len(n.edges))()
        for k, e in enumerate(n.edges):
            edges[k].src = e.src
            edges[k].kind = EDGE_KIND[e.kind]
            if e.W is not None:
                edges[k].W = f32(e.W)
            if e.kind == "conv":
                edges[k].kh, edges[k].kw = e.W.shape[2], e.W.shape[3]
            edges[k].stride, edges[k].pad = e.stride, e.pad
        edge_arrays.append(edges)
        nodes[i].c, nodes[i].h, nodes[i].w = shape
        nodes[i].bias = f32(n.bias)
        if n.relu and lu is not None:
            nodes[i].lower = f64(lu[relu_pos][0])
            nodes[i].upper = f64(lu[relu_pos][1])
            relu_pos += 1
        nodes[i].n_edges = len(n.edges)
        nodes[i].edges = edges
    ins = tuple(net.in_shape) if len(net.in_shape) == 3 else (net.in_size, 1, 1)
    keep += [nodes, edge_arrays]
    return NetDesc(ins[0], ins[1], ins[2], len(net.nodes), nodes), keep


class Net:
    """Device copy of a workloads.Net with its root bounds."""

    def __init__(self, net, lu):
        desc, keep = _net_desc(net, lu)
        h = C.c_void_p()
        _check(lib().gcp_net_create(C.byref(desc), C.byref(h)))
        self.h = h
        info = NetInfo()
        _check(lib().gcp_net_get_info(h, C.byref(info)))
        self.info = info
        self.n_I = int(info.n_unstable)

    def __del__(self):
        if getattr(self, "h", None) and _LIB is not None:
            _LIB.gcp_net_destroy(self.h)
            self.h = None


def crown_bounds(net, x0, eps: float, mode: int = GCP_MODE_FP32, splits=None):
    """gcp_crown_bounds: CROWN pre-activation bounds of every ReLU node of a
    workloads.Net over the box around x0 (a device fp64 tensor), computed on
    the device; returns [(l, u)] as host fp64 arrays, one pair per ReLU node.
    splits: optional [(node, neuron, sign)] of one BaB domain
    (gcp_crown_bounds_domain: the bounds over that domain)."""
    desc, keep = _net_desc(net, None)
    relu = [n for n in net.nodes if n.relu]
    lo = [np.empty(n.size, np.float64) for n in relu]
    hi = [np.empty(n.size, np.float64) for n in relu]
    lp = (C.c_void_p * len(relu))(*[a.ctypes.data for a in lo])
    up = (C.c_void_p * len(relu))(*[a.ctypes.data for a in hi])
    if splits:
        sn = np.ascontiguousarray([s[0] for s in splits], np.int32)
        sj = np.ascontiguousarray([s[1] for s in splits], np.int32)
        sg = np.ascontiguousarray([s[2] for s in splits], np.int8)
        _check(lib().gcp_crown_bounds_domain(C.byref(desc), _ptr(x0), float(eps), len(splits), sn.ctypes.data,
                                             sj.ctypes.data, sg.ctypes.data, lp, up, mode, _stream()))
    else:
        _check(lib().gcp_crown_bounds(C.byref(desc), _ptr(x0), float(eps), lp, up, mode, _stream()))
    return list(zip(lo, hi))


def bab(net: Net, x0, eps: float, c_row, cuts: Optional["Cuts"] = None, batch=64, max_depth=16,
        max_domains=100000, max_pool=100000, retries=4, iters=20, lr_alpha=0.1, lr_mult=0.02, decay=0.9, b1=0.9,
        b2=0.999, adam_eps=1e-8, mode: int = GCP_MODE_FP32):
    """gcp_bab on one spec row c_row (device fp64 [d_out]); returns a dict of
    the gcp_bab_result fields."""
    o = BabOpt(batch, max_depth, max_domains, max_pool, retries,
               OptDesc(iters, lr_alpha, lr_mult, decay, b1, b2, adam_eps, 0), mode)
    r = BabResult()
    _check(lib().gcp_bab(net.h, _ptr(x0), float(eps), _ptr(c_row), cuts.h if cuts else None, C.byref(o), C.byref(r),
                         _stream()))
    return {k: getattr(r, k) for k, _ in BabResult._fields_}


def net_unstable(net: Net):
    """(node, neuron, lower, upper) of the root-unstable neurons in alpha row order."""
    n = net.n_I
    node, neuron = np.empty(n, np.int32), np.empty(n, np.int32)
    lo, hi = np.empty(n, np.float64), np.empty(n, np.float64)
    _check(lib().gcp_net_get_unstable(net.h, _ptr(node), _ptr(neuron), _ptr(lo), _ptr(hi)))
    return node, neuron, lo, hi


class Cuts:
    def __init__(self, net: Net, cuts):
        self.N = int(cuts.n)
        a = [np.ascontiguousarray(x) for x in (cuts.cut.astype(np.int32), cuts.node.astype(np.int32),
                                               cuts.neuron.astype(np.int32), cuts.kind.astype(np.int8),
                                               cuts.coef.astype(np.float64), cuts.d.astype(np.float64))]
        h = C.c_void_p()
        _check(lib().gcp_cuts_create(net.h, self.N, a[0].size, *[x.ctypes.data for x in a], C.byref(h)))
        self.h = h
        self.net = net

    def __del__(self):
        if getattr(self, "h", None) and _LIB is not None:
            _LIB.gcp_cuts_destroy(self.h)
            self.h = None


class Splits:
    def __init__(self, net: Net, splits):
        self.B, self.K = splits.node.shape
        a = [np.ascontiguousarray(x) for x in (splits.node.astype(np.int32), splits.neuron.astype(np.int32),
                                               splits.sign.astype(np.int8))]
        h = C.c_void_p()
        _check(lib().gcp_splits_create(net.h, self.B, self.K, *[x.ctypes.data for x in a], C.byref(h)))
        self.h = h
        self.net = net

    def __del__(self):
        if getattr(self, "h", None) and _LIB is not None:
            _LIB.gcp_splits_destroy(self.h)
            self.h = None


def bound(net: Net, x0, eps: float, Cspec, splits: Splits, cuts: Optional[Cuts], alpha, beta, gamma,
          mode: int = GCP_MODE_FP32, grads: bool = False, verified: bool = False, validate: bool = False):
    """gcp_bound on torch device tensors; returns (bound[M] fp64, verified or
    None, (d_alpha, d_beta, d_gamma) or None)."""
    import torch
    dev = x0.device
    S = Cspec.shape[0]
    M = splits.B * S
    out = torch.empty(M, dtype=torch.float64, device=dev)
    ver = torch.empty(M, dtype=torch.uint8, device=dev) if verified else None
    g = None
    if grads:
        g = (torch.empty_like(alpha), torch.empty_like(beta), torch.empty_like(gamma))
    md = mode | (GCP_FLAG_VALIDATE if validate else 0)
    _check(lib().gcp_bound(net.h, _ptr(x0), float(eps), _ptr(Cspec), S, splits.h, cuts.h if cuts else None,
                           _ptr(alpha) if alpha.numel() else None, _ptr(beta) if beta.numel() else None,
                           _ptr(gamma) if gamma.numel() else None, md, _ptr(out), _ptr(ver),
                           *((_ptr(t) if t.numel() else None) for t in g) if g else (None, None, None),
                           _stream()))
    return out, ver, g


def prepare(net: Net, S: int, splits: Splits, cuts: Optional[Cuts], iters: int = 20, mode: int = GCP_MODE_FP32):
    """gcp_prepare: size the workspace and tune every tile shape for these
    shapes, so later bound / optimize calls of them allocate and wait for
    nothing."""
    _check(lib().gcp_prepare(net.h, S, splits.h, cuts.h if cuts else None, iters, mode, _stream()))


def bound_noalloc(net: Net, x0, eps: float, Cspec, splits: Splits, cuts: Optional[Cuts], alpha, beta, gamma,
                  out, verified=None, grads=None, mode: int = GCP_MODE_FP32):
    """gcp_bound_noalloc (no device allocation inside the call; workspace in
    the library's static array) into caller-allocated outputs: out [M] fp64,
    verified [M] uint8 or None, grads = (d_alpha, d_beta, d_gamma) or None."""
    S = Cspec.shape[0]
    _check(lib().gcp_bound_noalloc(net.h, _ptr(x0), float(eps), _ptr(Cspec), S, splits.h, cuts.h if cuts else None,
                                   _ptr(alpha) if alpha.numel() else None, _ptr(beta) if beta.numel() else None,
                                   _ptr(gamma) if gamma.numel() else None, mode, _ptr(out),
                                   _ptr(verified) if verified is not None else None,
                                   *((_ptr(t) if t.numel() else None) for t in grads) if grads else (None, None, None),
                                   _stream()))
    return out


def optimize(net: Net, x0, eps: float, Cspec, splits: Splits, cuts: Optional[Cuts], alpha, beta, gamma,
             adam_state, iters=20, lr_alpha=0.1, lr_mult=0.02, decay=0.9, b1=0.9, b2=0.999, adam_eps=1e-8,
             mode: int = GCP_MODE_FP32, use_graph: bool = False, bound_out=None, verified_out=None):
    """gcp_optimize (alpha, beta, gamma, adam_state updated in place);
    returns (bound[M] fp64 of the certifying pass, verified[M] uint8)."""
    import torch
    dev = x0.device
    S = Cspec.shape[0]
    M = splits.B * S
    out = bound_out if bound_out is not None else torch.empty(M, dtype=torch.float64, device=dev)
    ver = verified_out if verified_out is not None else torch.empty(M, dtype=torch.uint8, device=dev)
    o = OptDesc(iters, lr_alpha, lr_mult, decay, b1, b2, adam_eps, int(use_graph))
    _check(lib().gcp_optimize(net.h, _ptr(x0), float(eps), _ptr(Cspec), S, splits.h, cuts.h if cuts else None,
                              _ptr(alpha) if alpha.numel() else None, _ptr(beta) if beta.numel() else None,
                              _ptr(gamma) if gamma.numel() else None, _ptr(adam_state), C.byref(o), mode,
                              _ptr(out), _ptr(ver), _stream()))
    return out, ver


def bound_pi(net: Net, x0, eps: float, Cspec, splits: Splits, cuts: Optional[Cuts], alpha, beta, gamma, rho,
             mode: int = GCP_MODE_FP32, grads: bool = False, verified: bool = False, validate: bool = False):
    """gcp_bound_pi (explicit pi = rho * [-a_hat]_+); returns (bound[M],
    verified or None, (d_alpha, d_beta, d_gamma, d_rho) or None)."""
    import torch
    dev = x0.device
    S = Cspec.shape[0]
    M = splits.B * S
    out = torch.empty(M, dtype=torch.float64, device=dev)
    ver = torch.empty(M, dtype=torch.uint8, device=dev) if verified else None
    g = None
    if grads:
        g = (torch.empty_like(alpha), torch.empty_like(beta), torch.empty_like(gamma), torch.empty_like(rho))
    md = mode | (GCP_FLAG_VALIDATE if validate else 0)
    opt = lambda t: _ptr(t) if t.numel() else None
    _check(lib().gcp_bound_pi(net.h, _ptr(x0), float(eps), _ptr(Cspec), S, splits.h, cuts.h if cuts else None,
                              opt(alpha), opt(beta), opt(gamma), opt(rho), md, _ptr(out), _ptr(ver),
                              *(opt(t) for t in g) if g else (None, None, None, None), _stream()))
    return out, ver, g


def optimize_pi(net: Net, x0, eps: float, Cspec, splits: Splits, cuts: Optional[Cuts], alpha, beta, gamma, rho,
                adam_state, iters=20, lr_alpha=0.1, lr_mult=0.02, decay=0.9, b1=0.9, b2=0.999, adam_eps=1e-8,
                mode: int = GCP_MODE_FP32, use_graph: bool = False):
    """gcp_optimize_pi (alpha, beta, gamma, rho, adam_state updated in place;
    adam_state of adam_state_size(..., explicit_pi=True) floats); returns
    (bound[M] fp64 of the certifying pass, verified[M] uint8)."""
    import torch
    dev = x0.device
    S = Cspec.shape[0]
    M = splits.B * S
    out = torch.empty(M, dtype=torch.float64, device=dev)
    ver = torch.empty(M, dtype=torch.uint8, device=dev)
    o = OptDesc(iters, lr_alpha, lr_mult, decay, b1, b2, adam_eps, int(use_graph))
    opt = lambda t: _ptr(t) if t.numel() else None
    _check(lib().gcp_optimize_pi(net.h, _ptr(x0), float(eps), _ptr(Cspec), S, splits.h, cuts.h if cuts else None,
                                 opt(alpha), opt(beta), opt(gamma), opt(rho), _ptr(adam_state), C.byref(o), mode,
                                 _ptr(out), _ptr(ver), _stream()))
    return out, ver


def optimize_batch(items, iters=20, lr_alpha=0.1, lr_mult=0.02, decay=0.9, b1=0.9, b2=0.999, adam_eps=1e-8,
                   mode: int = GCP_MODE_FP32, use_graph: bool = False):
    """gcp_optimize_batch over a list of dicts with keys P (a Problem),
    alpha, beta, gamma, state, bound, verified (device tensors; updated /
    written in place)."""
    arr = (BatchItem * len(items))()
    for i, it in enumerate(items):
        P = it["P"]
        arr[i] = BatchItem(P.net.h.value, _ptr(P.x0), float(P.eps), _ptr(P.C), P.S, P.splits.h.value,
                           P.cuts.h.value if P.cuts else None,
                           _ptr(it["alpha"]) if it["alpha"].numel() else None,
                           _ptr(it["beta"]) if it["beta"].numel() else None,
                           _ptr(it["gamma"]) if it["gamma"].numel() else None,
                           _ptr(it["state"]), _ptr(it["bound"]), _ptr(it["verified"]))
    o = OptDesc(iters, lr_alpha, lr_mult, decay, b1, b2, adam_eps, int(use_graph))
    _check(lib().gcp_optimize_batch(len(items), arr, C.byref(o), mode, _stream()))


def adam_state_size(M, n_I, K, N, explicit_pi=False):
    return 2 * M * (n_I + K + N) + (2 * M * n_I if explicit_pi else 0)


class Problem:
    """A workloads.Problem uploaded to the current device."""

    def __init__(self, prob, device="cuda"):
        import torch
        self.prob = prob
        self.net = Net(prob.net, prob.lu)
        self.cuts = Cuts(self.net, prob.cuts) if prob.cuts.n > 0 else None
        self.splits = Splits(self.net, prob.splits)
        self.x0 = torch.tensor(prob.x0, dtype=torch.float64, device=device)
        self.C = torch.tensor(prob.C, dtype=torch.float64, device=device)
        self.eps = prob.eps
        self.S = prob.S
        self.B = prob.B
        self.M = prob.B * prob.S
        self.n_I = self.net.n_I
        self.K = prob.splits.K
        self.N = prob.cuts.n


def _bound_autograd():
    import torch

    class GCPBound(torch.autograd.Function):
        """bound = GCPBound.apply(problem, alpha, beta, gamma, mode): the
        forward runs gcp_bound with gradients requested; the backward scales
        the adjoint's per-row gradients by grad_output."""

        @staticmethod
        def forward(ctx, P, alpha, beta, gamma, mode=GCP_MODE_FP32):
            out, _, g = bound(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, alpha.detach(), beta.detach(),
                              gamma.detach(), mode=mode, grads=True)
            ctx.save_for_backward(*g)
            return out

        @staticmethod
        def backward(ctx, go):
            ga, gb, gc = ctx.saved_tensors
            w = go.to(torch.float32)[:, None]
            return None, ga * w, gb * w, gc * w, None

    return GCPBound


_GCPBound = None


def gcp_bound_autograd(P, alpha, beta, gamma, mode=GCP_MODE_FP32):
    global _GCPBound
    if _GCPBound is None:
        _GCPBound = _bound_autograd()
    return _GCPBound.apply(P, alpha, beta, gamma, mode)


def profile_enable(on: bool = True):
    """Start (reset) or stop the library's per-kernel event timing."""
    _check(lib().gcp_profile_enable(1 if on else 0))


def profile_read():
    """Per kernel class: {name: dict(launches, ms, bytes, alg_bytes, flops)} (bytes: every operand
    once; alg_bytes: optimiser-state traffic only)."""
    out = {}
    i = 0
    buf = C.create_string_buffer(256)
    while True:
        n, ms, by, al, fl = C.c_int64(), C.c_double(), C.c_double(), C.c_double(), C.c_double()
        rc = lib().gcp_profile_read(i, buf, 256, C.byref(n), C.byref(ms), C.byref(by), C.byref(al), C.byref(fl))
        if rc != 0:
            break
        if n.value:   # classes registered by earlier runs but not launched since the reset are left out
            out[buf.value.decode()] = dict(launches=n.value, ms=ms.value, bytes=by.value, alg_bytes=al.value,
                                           flops=fl.value)
        i += 1
    return out
