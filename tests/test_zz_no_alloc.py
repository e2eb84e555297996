"""The allocation-free entry point hcu_gram_noalloc (scratch in the
library's fixed device array, no context) against hcu_gram of a context
(workspace scratch) on the same blocks: two calls in a row, the second with
a smaller input, for real FP64 and complex FP32 blocks.  Same kernels and
summation order, so the FP64 results must agree to rounding (bar 1e-13
relative); FP32 products are accumulated identically, bar 1e-6 relative."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _contexts(kind):
    from paper_2507_23612_amd import hcu
    out = []
    for name, ns in (("c1", 200), ("tiny", 40)):          # second: smaller grid and fewer states
        cfg = workloads.make_config(name)
        cfg["ns"] = ns
        if kind == "c64":
            cfg["kpts"] = np.array([[0.18, -0.18, 0.28]])
        out.append((cfg, hcu.HcuContext(cfg, "fp64" if kind == "f64" else "mixed")))
    return out


@pytest.mark.parametrize("kind", ["f64", "c64"])
def test_gram_noalloc_matches_gram(kind):
    torch = _torch()
    from paper_2507_23612_amd import hcu
    for call, ((cfg, ctx), ncol) in enumerate(zip(_contexts(kind), (200, 33))):
        print(f"[gpu] gram_noalloc {kind} call {call}: grid {list(cfg['n'])} ncol {ncol}", flush=True)
        cp = kind == "c64"
        Y = torch.from_numpy(workloads.random_block(ctx.nd, ctx.ns, 61 + call, complex_=cp)).cuda().to(ctx.dtype)
        HY = torch.from_numpy(workloads.random_block(ctx.nd, ctx.ns, 71 + call, complex_=cp)).cuda().to(ctx.dtype)
        S_ref, H_ref = ctx.gram(Y, HY, ncol=ncol, ld=ctx.nd)
        w = 2 if cp else 1
        S_d = torch.full((ncol, ncol * w), 7.0, dtype=torch.float64, device="cuda")
        H_d = torch.full((ncol, ncol * w), 7.0, dtype=torch.float64, device="cuda")
        dv = float(np.prod(np.asarray(cfg["L"]) / np.asarray(cfg["n"])))
        st = hcu.gram_noalloc(Y, HY, ncol, ctx.nd, ctx.nd, "fp64" if kind == "f64" else "mixed", cp, dv,
                              S_d, H_d, torch.cuda.current_stream())
        assert st == hcu.HCU_OK
        torch.cuda.synchronize()
        S_n, H_n = S_d.cpu().numpy(), H_d.cpu().numpy()
        if cp:
            S_n = S_n[:, 0::2] + 1j * S_n[:, 1::2]
            H_n = H_n[:, 0::2] + 1j * H_n[:, 1::2]
        S_n, H_n = S_n.T, H_n.T                     # device matrices are column-major
        bar = 1e-13 if kind == "f64" else 1e-6
        for got, want in ((S_n, S_ref), (H_n, H_ref)):
            err = np.max(np.abs(got - want)) / np.max(np.abs(want))
            print(f"[gpu] gram_noalloc {kind} call {call}: rel diff {err:.2e}", flush=True)
            assert err <= bar
        ctx.close()


def test_gram_noalloc_rejects_beyond_scratch():
    torch = _torch()
    from paper_2507_23612_amd import hcu
    x = torch.zeros(16, dtype=torch.float64, device="cuda")
    # 4096 states need more partial sums than the fixed scratch holds;
    # refused before any device work (the small buffers are never read)
    assert hcu.gram_noalloc(x, x, 4096, 1000, 1000, "fp64", False, 1.0, x, x) == hcu.HCU_OOM
    assert hcu.gram_noalloc(x, x, 8, 1000, 999, "fp64", False, 1.0, x, x) == hcu.HCU_INVALID_ARG
