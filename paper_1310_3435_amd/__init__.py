"""MI355X library for stochastic-deterministic domain decomposition of the
linear Winslow mesh generator (Bihlo & Haynes, arXiv 1310.3435).

This module is the thin Python binding of ``libsdd.so``: it marshals
arguments into the C structures of ``include/sdd.h`` and calls the entry
points of the same names.  Device memory and streams come from PyTorch
(``torch.cuda`` tensors and the current stream); every step of the method
runs in the library's HIP kernels.  There is no CPU fallback: without the
built library or without a GPU the calls raise.
"""

from __future__ import annotations

import ctypes as C
import functools
import inspect
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsdd.so")

SDD_FP64, SDD_FP32 = 0, 1
PREC = {"fp64": SDD_FP64, "fp32": SDD_FP32}
SDD_EXIT_END_OF_STEP, SDD_EXIT_BRIDGE, SDD_EXIT_EXPONENTIAL = 0, 1, 2
EXIT_TEST = {"step": SDD_EXIT_END_OF_STEP, "bridge": SDD_EXIT_BRIDGE, "expo": SDD_EXIT_EXPONENTIAL}
TERM = {"gauss": 0, "ring": 1, "sech2": 2, "sin2": 3}
BMAP = {"identity": 0, "affine": 1, "annulus": 2, "table": 3}
PLACEMENT = {"uniform": 0, "equidistributed": 1}
INTERP = {"linear": 0, "pchip": 1}
MAX_TERMS = 4


class SddError(RuntimeError):
    pass


class SddCappedWarning(UserWarning):
    """Some paths stopped at the step cap (SDD_WARN_CAPPED)."""


class sdd_density_term(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad", C.c_int32), ("amp", C.c_double), ("coef", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("r0", C.c_double), ("nx", C.c_double),
                ("ny", C.c_double)]


class sdd_density(C.Structure):
    _fields_ = [("base", C.c_double), ("n_terms", C.c_int32), ("pad", C.c_int32),
                ("term", sdd_density_term * MAX_TERMS)]


class sdd_bmap(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_per_edge", C.c_int32), ("p", C.c_double * 8), ("table", C.c_void_p)]


class sdd_layout(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("sx", C.c_int32), ("sy", C.c_int32)]


class sdd_walk_stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("paths", C.c_int64), ("capped", C.c_int64), ("t_stoc_ms", C.c_double)]


class sdd_request(C.Structure):
    _fields_ = [("w", sdd_density), ("bmap", sdd_bmap), ("layout", sdd_layout), ("k", C.c_int32),
                ("placement", C.c_int32), ("interp", C.c_int32), ("exit_test", C.c_int32), ("dt", C.c_double),
                ("se_target", C.c_double), ("paths_per_node", C.c_int64), ("seed", C.c_uint64),
                ("t_max", C.c_double)]


class sdd_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("pad", C.c_int32), ("n_nodes", C.c_int64), ("paths_per_node", C.c_int64),
                ("steps", C.c_int64), ("capped", C.c_int64), ("max_se", C.c_double), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double), ("t_queue_ms", C.c_double),
                ("t_stoc_ms", C.c_double), ("t_fill_ms", C.c_double), ("t_sub_ms", C.c_double)]


SDD_OK, SDD_WARN_CAPPED = 0, 1
SDD_EINVAL, SDD_EAGAIN, SDD_ECANCELED, SDD_EUNSUPPORTED = -1, -4, -5, -6

PATH_RECORD = np.dtype([("exit_xi", "<f8"), ("exit_eta", "<f8"), ("steps", "<i8"), ("side", "<i4"),
                        ("capped", "<i4")])

_lib = None


def lib() -> C.CDLL:
    """Load libsdd.so (built by ``paper_1310_3435_amd/build.py``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise SddError(f"{LIB_PATH} is missing: run paper_1310_3435_amd/build.py (or __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, D, U64, SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint64, C.c_size_t
    L.sdd_status_string.restype = C.c_char_p
    L.sdd_status_string.argtypes = [C.c_int]
    L.sdd_version.restype = I32
    L.sdd_create.argtypes = [I32, C.POINTER(P)]
    L.sdd_create.restype = C.c_int
    L.sdd_destroy.argtypes = [P]
    L.sdd_destroy.restype = None
    L.sdd_workspace_bytes.argtypes = [I64, I64, I32]
    L.sdd_workspace_bytes.restype = SZ
    L.sdd_interface_estimate.argtypes = [P, C.POINTER(sdd_density), C.POINTER(sdd_bmap), P, I64, I64, I64, D, U64,
                                         I32, D, I32, P, P, P, P, P, P, SZ, P]
    L.sdd_interface_estimate.restype = C.c_int
    L.sdd_interface_estimate_noalloc.argtypes = [P, C.POINTER(sdd_density), C.POINTER(sdd_bmap), P, I64, I64, I64,
                                                 D, U64, I32, D, I32, P, P, P, P, P, P]
    L.sdd_interface_estimate_noalloc.restype = C.c_int
    L.sdd_noalloc_max_nodes.argtypes = []
    L.sdd_noalloc_max_nodes.restype = I64
    L.sdd_walk_status.argtypes = [C.POINTER(sdd_walk_stats)]
    L.sdd_walk_status.restype = C.c_int
    L.sdd_layout_node_count.argtypes = [C.POINTER(sdd_layout), I32]
    L.sdd_layout_node_count.restype = I64
    L.sdd_layout_nodes.argtypes = [P, C.POINTER(sdd_layout), I32, I32, C.POINTER(sdd_density), P, P]
    L.sdd_layout_nodes.restype = C.c_int
    L.sdd_bmap_edge1d_table.argtypes = [P, C.POINTER(sdd_density), I32, P, P]
    L.sdd_bmap_edge1d_table.restype = C.c_int
    L.sdd_fill_interfaces.argtypes = [P, C.POINTER(sdd_layout), I32, C.POINTER(sdd_bmap), P, P, I32, P, P, P]
    L.sdd_fill_interfaces.restype = C.c_int
    L.sdd_subdomain_workspace_bytes.argtypes = [C.POINTER(sdd_layout)]
    L.sdd_subdomain_workspace_bytes.restype = SZ
    L.sdd_subdomain_solve.argtypes = [P, C.POINTER(sdd_density), C.POINTER(sdd_bmap), C.POINTER(sdd_layout), P, P,
                                      D, I32, P, P, P, P, SZ, P]
    L.sdd_subdomain_solve.restype = C.c_int
    L.sdd_layout_nodes_extrema.argtypes = [P, C.POINTER(sdd_layout), C.POINTER(sdd_density), I32, P, P, P]
    L.sdd_layout_nodes_extrema.restype = C.c_int
    L.sdd_fill_interfaces_counts.argtypes = [P, C.POINTER(sdd_layout), I32, P, C.POINTER(sdd_bmap), P, P, I32, P, P,
                                             P]
    L.sdd_fill_interfaces_counts.restype = C.c_int
    L.sdd_grid_nodes.argtypes = [P, I32, I32, P, P]
    L.sdd_grid_nodes.restype = C.c_int
    L.sdd_assemble_mesh.argtypes = [P, I32, I32, C.POINTER(sdd_bmap), P, P, P]
    L.sdd_assemble_mesh.restype = C.c_int
    L.sdd_quality_workspace_bytes.argtypes = [I32, I32]
    L.sdd_quality_workspace_bytes.restype = SZ
    L.sdd_mesh_quality.argtypes = [P, I32, I32, P, P, P, P, SZ, P]
    L.sdd_mesh_quality.restype = C.c_int
    L.sdd_mesh_compare.argtypes = [P, I32, I32, C.POINTER(sdd_density), P, P, P, P, SZ, P]
    L.sdd_mesh_compare.restype = C.c_int
    L.sdd_smooth_workspace_bytes.argtypes = [C.POINTER(sdd_layout)]
    L.sdd_smooth_workspace_bytes.restype = SZ
    L.sdd_mesh_smooth.argtypes = [P, C.POINTER(sdd_layout), I32, D, D, I32, P, P, SZ, P]
    L.sdd_mesh_smooth.restype = C.c_int
    L.sdd_smooth_interfaces_workspace_bytes.argtypes = [C.POINTER(sdd_layout)]
    L.sdd_smooth_interfaces_workspace_bytes.restype = SZ
    L.sdd_smooth_interfaces.argtypes = [P, C.POINTER(sdd_layout), I32, P, P, P, SZ, P]
    L.sdd_smooth_interfaces.restype = C.c_int
    L.sdd_server_create.argtypes = [P, SZ, I32, I64, I64, I64, C.POINTER(P)]
    L.sdd_server_create.restype = C.c_int
    L.sdd_server_submit.argtypes = [P, C.POINTER(sdd_request), P, C.POINTER(C.c_uint64)]
    L.sdd_server_submit.restype = C.c_int
    L.sdd_server_poll.argtypes = [P, C.c_uint64, C.POINTER(sdd_result)]
    L.sdd_server_poll.restype = C.c_int
    L.sdd_server_wait.argtypes = [P, C.c_uint64, C.POINTER(sdd_result)]
    L.sdd_server_wait.restype = C.c_int
    L.sdd_server_cancel.argtypes = [P, C.c_uint64]
    L.sdd_server_cancel.restype = C.c_int
    L.sdd_server_clock.argtypes = [P]
    L.sdd_server_clock.restype = D
    L.sdd_server_destroy.argtypes = [P]
    L.sdd_server_destroy.restype = C.c_int
    _lib = L
    return L


EXPORTS = ["sdd_status_string", "sdd_version", "sdd_create", "sdd_destroy", "sdd_workspace_bytes",
           "sdd_interface_estimate", "sdd_walk_status", "sdd_interface_estimate_noalloc", "sdd_noalloc_max_nodes", "sdd_layout_node_count", "sdd_layout_nodes", "sdd_bmap_edge1d_table",
           "sdd_fill_interfaces", "sdd_subdomain_workspace_bytes", "sdd_subdomain_solve", "sdd_server_create",
           "sdd_server_submit", "sdd_server_poll", "sdd_server_wait", "sdd_server_cancel", "sdd_server_clock",
           "sdd_server_destroy", "sdd_quality_workspace_bytes", "sdd_mesh_quality", "sdd_mesh_compare",
           "sdd_smooth_workspace_bytes", "sdd_mesh_smooth", "sdd_smooth_interfaces_workspace_bytes",
           "sdd_smooth_interfaces", "sdd_grid_nodes", "sdd_assemble_mesh", "sdd_layout_nodes_extrema",
           "sdd_fill_interfaces_counts"]


def _check(rc: int, what: str):
    if rc != 0:
        raise SddError(f"{what}: {lib().sdd_status_string(rc).decode()} ({rc})")


# ------------------------------------------------------------ marshalling

def make_density(d: dict) -> sdd_density:
    D = sdd_density()
    D.base = float(d["base"])
    terms = d["terms"]
    if len(terms) > MAX_TERMS:
        raise SddError(f"at most {MAX_TERMS} density terms")
    D.n_terms = len(terms)
    for i, t in enumerate(terms):
        T = D.term[i]
        T.kind = TERM[t["kind"]]
        for f in ("amp", "coef", "cx", "cy", "r0", "nx", "ny"):
            setattr(T, f, float(t.get(f, 0.0)))
    return D


def make_layout(L: dict) -> sdd_layout:
    return sdd_layout(int(L["nx"]), int(L["ny"]), int(L["sx"]), int(L["sy"]))


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise SddError("no GPU visible: the library runs only on the device")
    return torch


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise SddError("expected a contiguous device tensor")
    return t.data_ptr()


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _on_stream(fn):
    """Run an entry point with its ``stream`` argument as torch's current
    stream, so that the outputs and workspaces it allocates belong to the
    stream its kernels run on: torch then reuses a freed workspace only in
    that stream's order."""
    sig = inspect.signature(fn)

    @functools.wraps(fn)
    def wrapped(*args, **kwargs):
        stream = sig.bind_partial(*args, **kwargs).arguments.get("stream")
        if stream is None:
            return fn(*args, **kwargs)
        with _torch().cuda.stream(stream):
            return fn(*args, **kwargs)
    return wrapped


class Bmap:
    """Boundary map descriptor; a table map keeps its device table alive."""

    def __init__(self, desc: dict, ctx: "Context" = None, density: Optional[dict] = None):
        self.desc = desc
        self.s = sdd_bmap()
        self.table = None
        kind = desc["kind"]
        for i, v in enumerate(desc.get("p", [])):
            self.s.p[i] = float(v)
        if kind == "edge1d":
            if ctx is None or density is None:
                raise SddError("an edge1d map needs the context and the density")
            self.table = sdd_bmap_edge1d_table(ctx, density, int(desc.get("n_per_edge", 4097)))
            self.s.kind = BMAP["table"]
        elif kind == "table":
            torch = _torch()
            self.table = torch.as_tensor(np.ascontiguousarray(desc["table"], dtype=np.float64)).cuda()
            self.s.kind = BMAP["table"]
        else:
            self.s.kind = BMAP[kind]
        if self.table is not None:
            self.s.n_per_edge = int(self.table.shape[1])
            self.s.table = self.table.data_ptr()


class Context:
    """Owns an ``sdd_ctx`` bound to one HIP device."""

    def __init__(self, device: int = 0):
        _torch()
        self.device = device
        h = C.c_void_p()
        _check(lib().sdd_create(device, C.byref(h)), "sdd_create")
        self.h = h
        self._ws = {}

    def workspace(self, nbytes: int):
        """A reusable device workspace of at least nbytes for the current
        stream.  Calls on one stream run in order and share it; each stream
        has its own, so calls on different streams do not overlap in it."""
        torch = _torch()
        key = torch.cuda.current_stream().cuda_stream
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=f"cuda:{self.device}")
            self._ws[key] = ws
        return ws

    def close(self):
        if self.h:
            lib().sdd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ entry points

def sdd_version() -> int:
    return int(lib().sdd_version())


def sdd_create(device: int = 0) -> Context:
    return Context(device)


def sdd_workspace_bytes(n_nodes: int, paths_per_node: int, prec: str = "fp64") -> int:
    return int(lib().sdd_workspace_bytes(int(n_nodes), int(paths_per_node), PREC[prec]))


@_on_stream
def sdd_interface_estimate(ctx: Context, density: dict, bmap, nodes, paths_per_node: int, dt: float, seed: int,
                           prec: str = "fp64", t_max: float = 8.0, path_begin: int = 0, want_se: bool = True,
                           want_sums: bool = False, want_stats: bool = True, per_path: bool = False,
                           stream=None, out: Optional[dict] = None, exit_test: str = "step") -> dict:
    """Monte Carlo estimate at every node (device tensors in, device tensors out).

    exit_test: "step" (end-of-step test), "bridge" (plus the Brownian-bridge
    test) or "expo" (exponential time stepping with mean step dt).
    nodes: device float64 [n, 2].  Returns dict with 'mean' [n,2], and as
    requested 'se' [n,2], 'sums' [n,4], 'stats' (int64 [4]: steps, paths,
    capped, and the walk time in ms as the bits of a float64; see
    walk_stats) and 'per_path' (uint8 [n, N, 32] records).  Results are
    valid after the stream synchronises.  Pass ``out`` (a previous result
    dict) to reuse its buffers: each is checked against this call's shape.
    """
    torch = _torch()
    B = bmap if isinstance(bmap, Bmap) else Bmap(bmap, ctx, density)
    D = make_density(density)
    n = int(nodes.shape[0])
    dev = nodes.device
    f64 = dict(dtype=torch.float64, device=dev)
    want = {"mean": ((n, 2), torch.float64, True), "se": ((n, 2), torch.float64, want_se),
            "sums": ((n, 4), torch.float64, want_sums), "stats": ((4,), torch.int64, want_stats),
            "per_path": ((n, int(paths_per_node), 32), torch.uint8, per_path)}
    o = out if out is not None else {}
    for key, (shape, dtype, on) in want.items():
        t = o.get(key)
        if not on:
            o.pop(key, None)
            continue
        if t is not None and (tuple(t.shape) != shape or t.dtype != dtype or t.device != dev
                              or not t.is_contiguous()):
            raise SddError(f"out['{key}'] has shape {tuple(t.shape)} {t.dtype} on {t.device}; "
                           f"this call needs {shape} {dtype} on {dev}")
        if t is None:
            o[key] = torch.empty(shape, dtype=dtype, device=dev)
    wsb = sdd_workspace_bytes(n, paths_per_node, prec)
    if wsb == 0:
        raise SddError("sdd_interface_estimate: invalid argument (node or path count)")
    ws = ctx.workspace(wsb)
    rc = lib().sdd_interface_estimate(
        ctx.h, C.byref(D), C.byref(B.s), _ptr(nodes), n, int(paths_per_node), int(path_begin), float(dt),
        C.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), PREC[prec], float(t_max), EXIT_TEST[exit_test],
        _ptr(o["mean"]), _ptr(o.get("se")), _ptr(o.get("sums")), _ptr(o.get("stats")), _ptr(o.get("per_path")),
        _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "sdd_interface_estimate")
    o["_bmap"] = B
    return o


def walk_stats(stats, warn: bool = True) -> dict:
    """Host view of a walk's device stats (int64 [4]): steps, paths, capped,
    t_stoc_ms.  Synchronises with the stats' producer (a device-to-host
    copy).  Warns (SddCappedWarning) when sdd_walk_status reports capped
    paths."""
    a = stats.cpu().numpy()
    s = sdd_walk_stats(int(a[0]), int(a[1]), int(a[2]), float(a[3:4].view(np.float64)[0]))
    if warn and lib().sdd_walk_status(C.byref(s)) == SDD_WARN_CAPPED:
        import warnings
        warnings.warn(f"{s.capped} of {s.paths} paths stopped at the step cap", SddCappedWarning, stacklevel=2)
    return {"steps": s.steps, "paths": s.paths, "capped": s.capped, "t_stoc_ms": s.t_stoc_ms}


def path_records(per_path) -> np.ndarray:
    """Per-path records (device uint8 [n, N, 32]) as a host structured array."""
    a = per_path.cpu().numpy()
    return a.view(PATH_RECORD).reshape(a.shape[0], a.shape[1])


def sdd_layout_node_count(layout: dict, k: int) -> int:
    L = make_layout(layout)
    v = int(lib().sdd_layout_node_count(C.byref(L), int(k)))
    if v < 0:
        raise SddError("invalid layout")
    return v


@_on_stream
def sdd_layout_nodes(ctx: Context, layout: dict, k: int, placement: str = "uniform",
                     density: Optional[dict] = None, stream=None):
    torch = _torch()
    L = make_layout(layout)
    n = sdd_layout_node_count(layout, k)
    nodes = torch.empty((max(n, 1), 2), dtype=torch.float64, device=f"cuda:{ctx.device}")
    D = make_density(density) if density is not None else None
    rc = lib().sdd_layout_nodes(ctx.h, C.byref(L), int(k), PLACEMENT[placement],
                                C.byref(D) if D is not None else None, _ptr(nodes), _stream(stream))
    _check(rc, "sdd_layout_nodes")
    return nodes[:n]


@_on_stream
def sdd_layout_nodes_extrema(ctx: Context, layout: dict, density: dict, cap: int, stream=None):
    """(nodes, counts): crosspoints, then `cap` slots per segment holding the
    extrema of w_s and w_ss along it (Sec. 3.6); unused slots are (-1, -1)."""
    torch = _torch()
    L = make_layout(layout)
    n = sdd_layout_node_count(layout, cap)
    nseg = (L.sx - 1) * L.sy + (L.sy - 1) * L.sx
    dev = f"cuda:{ctx.device}"
    nodes = torch.empty((max(n, 1), 2), dtype=torch.float64, device=dev)
    counts = torch.zeros(max(nseg, 1), dtype=torch.int32, device=dev)
    D = make_density(density)
    _check(lib().sdd_layout_nodes_extrema(ctx.h, C.byref(L), C.byref(D), int(cap), _ptr(nodes), _ptr(counts),
                                          _stream(stream)), "sdd_layout_nodes_extrema")
    return nodes[:n], counts[:nseg]


@_on_stream
def sdd_bmap_edge1d_table(ctx: Context, density: dict, n_per_edge: int = 4097, stream=None):
    torch = _torch()
    D = make_density(density)
    table = torch.empty((4, int(n_per_edge), 2), dtype=torch.float64, device=f"cuda:{ctx.device}")
    _check(lib().sdd_bmap_edge1d_table(ctx.h, C.byref(D), int(n_per_edge), _ptr(table), _stream(stream)),
           "sdd_bmap_edge1d_table")
    return table


@_on_stream
def sdd_fill_interfaces(ctx: Context, layout: dict, k: int, bmap, nodes, values, interp: str = "linear",
                        stream=None, density: Optional[dict] = None, counts=None) -> Tuple[object, object]:
    """Interface lines from the node estimates; with `counts` (device int32)
    the node list has k slots per segment (sdd_fill_interfaces_counts)."""
    torch = _torch()
    B = bmap if isinstance(bmap, Bmap) else Bmap(bmap, ctx, density)
    L = make_layout(layout)
    f64 = dict(dtype=torch.float64, device=f"cuda:{ctx.device}")
    vert = torch.empty((max(L.sx - 1, 0), L.ny, 2), **f64)
    horiz = torch.empty((max(L.sy - 1, 0), L.nx, 2), **f64)
    pv = _ptr(vert) if vert.numel() else None
    ph = _ptr(horiz) if horiz.numel() else None
    if counts is None:
        rc = lib().sdd_fill_interfaces(ctx.h, C.byref(L), int(k), C.byref(B.s), _ptr(nodes), _ptr(values),
                                       INTERP[interp], pv, ph, _stream(stream))
    else:
        rc = lib().sdd_fill_interfaces_counts(ctx.h, C.byref(L), int(k), _ptr(counts), C.byref(B.s), _ptr(nodes),
                                              _ptr(values), INTERP[interp], pv, ph, _stream(stream))
    _check(rc, "sdd_fill_interfaces")
    return vert, horiz


def sdd_subdomain_workspace_bytes(layout: dict) -> int:
    L = make_layout(layout)
    return int(lib().sdd_subdomain_workspace_bytes(C.byref(L)))


@_on_stream
def sdd_subdomain_solve(ctx: Context, density: dict, bmap, layout: dict, vert, horiz, tol: float = 1e-13,
                        max_sweeps: int = 100000, stream=None, mesh=None) -> dict:
    torch = _torch()
    B = bmap if isinstance(bmap, Bmap) else Bmap(bmap, ctx, density)
    D = make_density(density)
    L = make_layout(layout)
    dev = f"cuda:{ctx.device}"
    if mesh is None:
        mesh = torch.empty((L.ny, L.nx, 2), dtype=torch.float64, device=dev)
    nsub = L.sx * L.sy
    sweeps = torch.empty(nsub, dtype=torch.int32, device=dev)
    resid = torch.empty(nsub, dtype=torch.float64, device=dev)
    wsb = sdd_subdomain_workspace_bytes(layout)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    rc = lib().sdd_subdomain_solve(ctx.h, C.byref(D), C.byref(B.s), C.byref(L),
                                   _ptr(vert) if vert is not None and vert.numel() else None,
                                   _ptr(horiz) if horiz is not None and horiz.numel() else None,
                                   float(tol), int(max_sweeps), _ptr(mesh), _ptr(sweeps), _ptr(resid), _ptr(ws),
                                   ws.numel(), _stream(stream))
    _check(rc, "sdd_subdomain_solve")
    return {"mesh": mesh, "sweeps": sweeps, "resid": resid, "_ws": ws}


# ------------------------------------------------------ whole-grid mesh

@_on_stream
def sdd_grid_nodes(ctx: Context, nx: int, ny: int, stream=None):
    """Device float64 [(nx-2)(ny-2), 2]: every interior grid node, row by row."""
    torch = _torch()
    nodes = torch.empty(((nx - 2) * (ny - 2), 2), dtype=torch.float64, device=f"cuda:{ctx.device}")
    _check(lib().sdd_grid_nodes(ctx.h, int(nx), int(ny), _ptr(nodes), _stream(stream)), "sdd_grid_nodes")
    return nodes


@_on_stream
def sdd_assemble_mesh(ctx: Context, nx: int, ny: int, bmap: "Bmap", values, stream=None):
    """Device mesh [ny, nx, 2]: boundary map on the ring, values inside."""
    torch = _torch()
    mesh = torch.empty((ny, nx, 2), dtype=torch.float64, device=values.device)
    _check(lib().sdd_assemble_mesh(ctx.h, int(nx), int(ny), C.byref(bmap.s), _ptr(values), _ptr(mesh),
                                   _stream(stream)), "sdd_assemble_mesh")
    return mesh


@_on_stream
def run_probabilistic(ctx: Context, cfg: dict, stream=None) -> dict:
    """The whole mesh by Monte Carlo at every interior node (Sec. 3.3) [->
    Perona-Malik smoothing of the whole grid (Sec. 3.4)], all on the GPU."""
    dens = cfg["density"]
    B = Bmap(cfg["bmap"], ctx, dens)
    nx, ny = cfg["layout"]["nx"], cfg["layout"]["ny"]
    nodes = sdd_grid_nodes(ctx, nx, ny, stream=stream)
    est = sdd_interface_estimate(ctx, dens, B, nodes, cfg["paths"], cfg["dt"], cfg["seed"], cfg.get("prec", "fp64"),
                                 stream=stream, exit_test=cfg.get("exit_test", "step"))
    mesh = sdd_assemble_mesh(ctx, nx, ny, B, est["mean"], stream=stream)
    pm = cfg.get("pm")
    if pm:
        sdd_mesh_smooth(ctx, {"nx": nx, "ny": ny, "sx": 1, "sy": 1}, mesh, pm["dt"], pm["k"], pm["steps"], False,
                        stream=stream)
    return {"nodes": nodes, "est": est, "mesh": mesh, "_keep": B}


# ------------------------------------------------ quality and smoothing

@_on_stream
def sdd_mesh_quality(ctx: Context, mesh, want_cells: bool = False, stream=None) -> dict:
    """Q of every cell (eq. (11)) and {Q_max, Q_mean, folded} as device
    tensors: 'out' float64 [3], 'q' [ny-1, nx-1] if want_cells."""
    torch = _torch()
    ny, nx = int(mesh.shape[0]), int(mesh.shape[1])
    dev = mesh.device
    out = torch.empty(3, dtype=torch.float64, device=dev)
    q = torch.empty((ny - 1, nx - 1), dtype=torch.float64, device=dev) if want_cells else None
    ws = ctx.workspace(int(lib().sdd_quality_workspace_bytes(nx, ny)))
    _check(lib().sdd_mesh_quality(ctx.h, nx, ny, _ptr(mesh), _ptr(q), _ptr(out), _ptr(ws), ws.numel(),
                                  _stream(stream)), "sdd_mesh_quality")
    return {"out": out, "q": q}


@_on_stream
def sdd_mesh_compare(ctx: Context, density: dict, mesh, ref, stream=None):
    """Device float64 [2]: l_inf of the density at the nodes, largest node
    displacement."""
    torch = _torch()
    ny, nx = int(mesh.shape[0]), int(mesh.shape[1])
    out = torch.empty(2, dtype=torch.float64, device=mesh.device)
    D = make_density(density)
    ws = ctx.workspace(int(lib().sdd_quality_workspace_bytes(nx, ny)))
    _check(lib().sdd_mesh_compare(ctx.h, nx, ny, C.byref(D), _ptr(mesh), _ptr(ref), _ptr(out), _ptr(ws),
                                  ws.numel(), _stream(stream)), "sdd_mesh_compare")
    return out


@_on_stream
def sdd_mesh_smooth(ctx: Context, layout: dict, mesh, dt: float, k: float, steps: int, per_subdomain=True,
                    stream=None):
    """Perona-Malik FTCS smoothing of the device mesh [ny, nx, 2] in place (eq. (12)).
    per_subdomain: True (each subdomain alone), False (the whole grid) or
    "shifted" (subdomains moved by half their size, a second cycle)."""
    torch = _torch()
    L = make_layout(layout)
    mode = 2 if per_subdomain == "shifted" else (1 if per_subdomain else 0)
    ws = torch.empty(int(lib().sdd_smooth_workspace_bytes(C.byref(L))), dtype=torch.uint8, device=mesh.device)
    _check(lib().sdd_mesh_smooth(ctx.h, C.byref(L), mode, float(dt), float(k), int(steps),
                                 _ptr(mesh), _ptr(ws), ws.numel(), _stream(stream)), "sdd_mesh_smooth")
    return mesh


@_on_stream
def sdd_smooth_interfaces(ctx: Context, layout: dict, vert, horiz, span: int, stream=None):
    """Local quadratic regression of the device interface lines in place (Sec. 4)."""
    torch = _torch()
    L = make_layout(layout)
    ws = torch.empty(max(int(lib().sdd_smooth_interfaces_workspace_bytes(C.byref(L))), 256), dtype=torch.uint8,
                     device=f"cuda:{ctx.device}")
    _check(lib().sdd_smooth_interfaces(ctx.h, C.byref(L), int(span),
                                       _ptr(vert) if vert is not None and vert.numel() else None,
                                       _ptr(horiz) if horiz is not None and horiz.numel() else None,
                                       _ptr(ws), ws.numel(), _stream(stream)), "sdd_smooth_interfaces")
    return vert, horiz


# ------------------------------------------------------------ pipeline

@_on_stream
def run_pipeline(ctx: Context, cfg: dict, stream=None, per_path: bool = False) -> dict:
    """Nodes -> interface estimate -> fill [-> interface smoothing] ->
    subdomain solves [-> Perona-Malik smoothing], all on the GPU."""
    dens = cfg["density"]
    B = Bmap(cfg["bmap"], ctx, dens)
    L = cfg["layout"]
    counts = None
    if cfg.get("placement") == "extrema":
        nodes, counts = sdd_layout_nodes_extrema(ctx, L, dens, cfg["k"], stream=stream)
    else:
        nodes = sdd_layout_nodes(ctx, L, cfg["k"], cfg.get("placement", "uniform"), dens, stream=stream)
    est = sdd_interface_estimate(ctx, dens, B, nodes, cfg["paths"], cfg["dt"], cfg["seed"], cfg.get("prec", "fp64"),
                                 t_max=cfg.get("t_max", 8.0), per_path=per_path, stream=stream,
                                 exit_test=cfg.get("exit_test", "step"))
    vert, horiz = sdd_fill_interfaces(ctx, L, cfg["k"], B, nodes, est["mean"], cfg.get("interp", "linear"),
                                      stream=stream, counts=counts)
    if cfg.get("smooth_span", 0) > 0:
        sdd_smooth_interfaces(ctx, L, vert, horiz, int(cfg["smooth_span"]), stream=stream)
    sol = sdd_subdomain_solve(ctx, dens, B, L, vert, horiz, stream=stream)
    pm = cfg.get("pm")
    if pm:
        sdd_mesh_smooth(ctx, L, sol["mesh"], pm["dt"], pm["k"], pm["steps"], pm.get("per_subdomain", True),
                        stream=stream)
    return {"nodes": nodes, "counts": counts, "est": est, "vert": vert, "horiz": horiz, "mesh": sol["mesh"],
            "sweeps": sol["sweeps"],
            "resid": sol["resid"], "_keep": (B, sol)}


# ------------------------------------------------------------ serving

def make_request(req: dict) -> sdd_request:
    """sdd_request from a dict with the keys of workloads.serving_requests()."""
    R = sdd_request()
    R.w = make_density(req["density"])
    b = req["bmap"]
    R.bmap.kind = BMAP[b["kind"]]
    for i, v in enumerate(b.get("p", [])):
        R.bmap.p[i] = float(v)
    R.layout = make_layout(req["layout"])
    R.k = int(req["k"])
    R.placement = PLACEMENT[req.get("placement", "uniform")]
    R.interp = INTERP[req.get("interp", "linear")]
    R.exit_test = EXIT_TEST[req.get("exit_test", "step")]
    R.dt = float(req["dt"])
    R.se_target = float(req.get("se_target", 0.0))
    R.paths_per_node = int(req.get("paths", 0))
    R.seed = int(req["seed"]) & 0xFFFFFFFFFFFFFFFF
    R.t_max = float(req.get("t_max", 0.0))
    return R


class Server:
    """Request server of the C ABI (sdd_server_*): continuous batching of
    whole mesh requests on the device.  Meshes land in host numpy arrays."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int = 1 << 30, max_slots: int = 64,
                 max_nodes: int = 8192, max_points: int = 257 * 257, launch_paths: int = 0):
        self.ctx = ctx
        h = C.c_void_p()
        _check(lib().sdd_server_create(ctx.h, int(hbm_budget_bytes), int(max_slots), int(max_nodes),
                                       int(max_points), int(launch_paths), C.byref(h)), "sdd_server_create")
        self.h = h
        self.meshes = {}

    def submit(self, req: dict) -> int:
        R = make_request(req)
        L = req["layout"]
        mesh = np.zeros((L["ny"], L["nx"], 2))
        rid = C.c_uint64()
        _check(lib().sdd_server_submit(self.h, C.byref(R), mesh.ctypes.data_as(C.c_void_p), C.byref(rid)),
               "sdd_server_submit")
        self.meshes[rid.value] = mesh
        return rid.value

    def _result(self, rc, res, rid):
        """status 0 (SDD_OK) or 1 (SDD_WARN_CAPPED: done, some paths capped)
        means the mesh is there; negative values are errors."""
        out = {"status": rc, "n_nodes": res.n_nodes, "paths_per_node": res.paths_per_node, "steps": res.steps,
               "capped": res.capped, "max_se": res.max_se, "t_submit": res.t_submit, "t_admit": res.t_admit,
               "t_done": res.t_done, "t_queue_ms": res.t_queue_ms, "t_stoc_ms": res.t_stoc_ms,
               "t_fill_ms": res.t_fill_ms, "t_sub_ms": res.t_sub_ms, "mesh": self.meshes.pop(rid, None)}
        return out

    def poll(self, rid: int):
        res = sdd_result()
        rc = lib().sdd_server_poll(self.h, rid, C.byref(res))
        if rc == SDD_EAGAIN:
            return None
        if rc == SDD_EINVAL:
            raise SddError("unknown request id")
        return self._result(rc, res, rid)

    def wait(self, rid: int):
        res = sdd_result()
        rc = lib().sdd_server_wait(self.h, rid, C.byref(res))
        if rc == SDD_EINVAL:
            raise SddError("unknown request id")
        return self._result(rc, res, rid)

    def cancel(self, rid: int):
        _check(lib().sdd_server_cancel(self.h, rid), "sdd_server_cancel")

    def clock(self) -> float:
        return float(lib().sdd_server_clock(self.h))

    def close(self):
        if self.h:
            _check(lib().sdd_server_destroy(self.h), "sdd_server_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
