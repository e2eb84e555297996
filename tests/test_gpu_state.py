"""Save and resume of the SCF state through the C ABI: a context restored
from a snapshot continues the SCF exactly as the original does."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _ctx(cfg, precision=None):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_23612_amd import hcu
    ctx = hcu.HcuContext(cfg, precision)
    ctx.set_hubbard_occupation(hcu.initial_occupation(ctx, cfg))
    for s in range(ctx.nspin):
        for ik in range(ctx.nk):
            X0, v0 = hcu.start_inputs(ctx, cfg, s, ik)
            ctx.set_start(s, ik, X0, v0)
    return ctx


@pytest.mark.parametrize("name,kpts,precision", [("c1", False, "fp64"), ("tiny", True, "fp64"),
                                                 ("c1", False, "mixed")])
def test_resume_continues_identically(name, kpts, precision):
    cfg = workloads.make_config(name)
    if kpts:
        cfg = workloads.with_kpoints(cfg)
    a = _ctx(cfg, precision)
    a.scf_begin()
    for _ in range(5):
        a.scf_step()
    snap = a.save_state()
    ref = [a.scf_step() for _ in range(6)]
    b = _ctx(cfg, precision)
    b.load_state(snap)
    got = [b.scf_step() for _ in range(6)]
    for r, g in zip(ref, got):
        assert g["iteration"] == r["iteration"]
        assert g["F"] == r["F"] and g["residual"] == r["residual"]
    np.testing.assert_array_equal(b.get_eigenvalues(), a.get_eigenvalues())
    np.testing.assert_array_equal(b.get_hubbard_occupation(), a.get_hubbard_occupation())
    print(f"[gpu] resume {name} k={kpts} {precision}: F after resume {got[-1]['F']:.12f}", flush=True)


def test_load_rejects_foreign_state():
    from paper_2507_23612_amd import hcu
    a = _ctx(workloads.make_config("tiny"))
    a.scf_begin()
    a.scf_step()
    snap = a.save_state()
    b = _ctx(workloads.make_config("c1"))
    with pytest.raises(hcu.HcuError):
        b.load_state(snap)
    with pytest.raises(hcu.HcuError):
        a.load_state(snap[:100])
    bad = snap.copy()
    bad[:8] = 0
    with pytest.raises(hcu.HcuError):
        a.load_state(bad)
