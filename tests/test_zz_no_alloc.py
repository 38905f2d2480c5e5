"""The allocation-free estimate (sdd_interface_estimate_noalloc) against
sdd_interface_estimate through the C ABI: two calls in a row, the second
smaller (fewer nodes, fewer paths, other precision and exit test), each
bitwise equal to the workspace call on the same inputs; then the node
limit is refused before anything runs."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _call(sdd, ctx, fn, d, nodes, N, dt, seed, prec, exit_test, per_path):
    import torch
    n = nodes.shape[0]
    D = sdd.make_density(d)
    B = sdd.Bmap({"kind": "annulus", "p": [1.0, 2.0, 0.0, 1.5]}, ctx)
    dev = "cuda"
    mean = torch.full((n, 2), np.nan, dtype=torch.float64, device=dev)
    se = torch.full((n, 2), np.nan, dtype=torch.float64, device=dev)
    sums = torch.full((n, 4), np.nan, dtype=torch.float64, device=dev)
    stats = torch.zeros(4, dtype=torch.int64, device=dev)
    rec = torch.zeros((n, N, 32), dtype=torch.uint8, device=dev) if per_path else None
    args = [ctx.h, C.byref(D), C.byref(B.s), nodes.data_ptr(), n, N, 0, dt, C.c_uint64(seed), sdd.PREC[prec], 8.0,
            sdd.EXIT_TEST[exit_test], mean.data_ptr(), se.data_ptr(), sums.data_ptr(), stats.data_ptr(),
            rec.data_ptr() if per_path else None]
    if fn == "noalloc":
        rc = sdd.lib().sdd_interface_estimate_noalloc(*args, None)
    else:
        wsb = sdd.sdd_workspace_bytes(n, N, prec)
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        rc = sdd.lib().sdd_interface_estimate(*args, ws.data_ptr(), wsb, None)
    assert rc == 0, rc
    torch.cuda.synchronize()
    out = {"mean": mean.cpu().numpy(), "se": se.cpu().numpy(), "sums": sums.cpu().numpy(),
           "stats": stats.cpu().numpy()[:3]}
    if per_path:
        out["per_path"] = rec.cpu().numpy()
    return out


def test_noalloc_matches_the_workspace_call_twice():
    import torch

    import paper_1310_3435_amd as sdd
    ctx = sdd.Context(0)
    assert sdd.lib().sdd_noalloc_max_nodes() == 65536
    cases = [  # the second call is smaller, so stale sums of the first would show
        (W.random_density(31, 3), W.random_nodes(900, 31), 3000, 1e-3, 101, "fp32", "step", False),
        (W.random_density(32, 2), W.random_nodes(70, 32), 500, 2e-3, 102, "fp64", "bridge", True),
    ]
    for d, nodes_h, N, dt, seed, prec, et, pp in cases:
        nodes = torch.as_tensor(nodes_h).cuda()
        say(f"noalloc: {nodes_h.shape[0]} nodes x {N} paths, {prec}, {et}")
        a = _call(sdd, ctx, "noalloc", d, nodes, N, dt, seed, prec, et, pp)
        b = _call(sdd, ctx, "workspace", d, nodes, N, dt, seed, prec, et, pp)
        for k in a:
            assert np.array_equal(a[k], b[k]), k
        assert np.all(np.isfinite(a["mean"])) and a["stats"][1] == nodes_h.shape[0] * N
    # more nodes than the static scratch holds: refused, nothing written
    n = 65537
    big = torch.as_tensor(W.random_nodes(n, 33)).cuda()
    D = sdd.make_density({"base": 1.0, "terms": []})
    B = sdd.Bmap({"kind": "identity"}, ctx)
    mean = torch.zeros((n, 2), dtype=torch.float64, device="cuda")
    rc = sdd.lib().sdd_interface_estimate_noalloc(ctx.h, C.byref(D), C.byref(B.s), big.data_ptr(), n, 16, 0, 1e-3,
                                                  C.c_uint64(1), 1, 8.0, 0, mean.data_ptr(), None, None, None, None,
                                                  None)
    assert rc == -2   # SDD_ENOSPC
    torch.cuda.synchronize()
    assert float(mean.abs().max()) == 0.0
