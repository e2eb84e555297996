"""The library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer: the problem set-up (grid, atom supports, brick
tables, projection bricks and their destination rows), input validation and
the error paths of the C ABI, on the workloads of the tests and benchmarks,
with the sanitized build (python -m paper_2507_23612_amd.build --sanitize:
host pass instrumented, device code unchanged) loaded into a child process
with the sanitizer runtime preloaded.  No device call is made.

Any sanitizer report aborts the child (halt_on_error), which fails the test.
"""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB_SAN = os.path.join(ROOT, "paper_2507_23612_amd", "lib", "libhcu_san.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

CHILD = textwrap.dedent(r"""
    import ctypes, sys
    import numpy as np
    sys.path.insert(0, ROOT)
    import workloads
    from paper_2507_23612_amd import hcu
    lib = hcu.load_library(LIB_SAN)
    ptr = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    def create(cfg, want=hcu.HCU_OK):
        prob = hcu.Problem(cfg)
        h = ctypes.c_void_p()
        st = lib.hcu_create(ctypes.byref(prob.p), ctypes.byref(h))
        assert st == want, (st, lib.hcu_last_error(h))
        return h

    cfgs = {name: workloads.make_config(name) for name in ("tiny", "c1", "c5", "c2", "c3")}
    cfgs["tiny_kpoints"] = workloads.with_kpoints(cfgs["tiny"])
    hx = dict(cfgs["tiny"]); hx["hxc"] = True
    cfgs["tiny_hxc"] = hx
    for name, cfg in cfgs.items():
        h = create(cfg)
        n = ctypes.c_size_t()
        assert lib.hcu_workspace_size(h, ctypes.byref(n)) == hcu.HCU_OK and n.value > 0
        sz = hcu.hcu_sizes()
        assert lib.hcu_get_sizes(h, ctypes.byref(sz)) == hcu.HCU_OK
        nh = lib.hcu_num_hubbard_atoms(h)
        nspin = int(cfg["nspin"])
        D = np.zeros((nspin, max(nh, 1), 5, 5))
        D[:, :] = 0.2 * np.eye(5)
        if nh:
            bad = D.copy(); bad[0, 0, 1, 3] = np.nan
            assert lib.hcu_set_hubbard_occupation(h, ptr(bad)) == hcu.HCU_NAN
            bad = D.copy(); bad[0, nh - 1, 0, 4] = 0.05
            assert lib.hcu_set_hubbard_occupation(h, ptr(bad)) == hcu.HCU_INVALID_ARG
            assert lib.hcu_set_hubbard_occupation(h, ptr(D)) == hcu.HCU_NOT_BOUND
        assert lib.hcu_chfsi_pass(h, 0, 0) == hcu.HCU_NOT_BOUND
        assert lib.hcu_apply_h(h, 0, 0, None, None, 1, 10) == hcu.HCU_NOT_BOUND
        assert lib.hcu_get_potential(h, None, None) == hcu.HCU_NOT_BOUND
        lib.hcu_destroy(h)
        print("created and destroyed", name, "workspace", n.value, flush=True)

    tiny = cfgs["tiny"]
    for key, val in (("n0", 7), ("kT", 0.0), ("ns", 4)):
        bad = dict(tiny); bad[key] = val
        h = create(bad, hcu.HCU_INVALID_ARG)
        assert lib.hcu_last_error(h)
        lib.hcu_destroy(h)
    bad = workloads.with_kpoints(tiny); bad["hxc"] = True
    h = create(bad, hcu.HCU_INVALID_ARG)
    lib.hcu_destroy(h)

    b = ctypes.c_void_p()
    assert lib.hcu_batch_create(None, 0, ctypes.byref(b)) == hcu.HCU_INVALID_ARG
    m = ctypes.c_void_p()
    dims = (ctypes.c_int * 4)(64, 128, 128, 30)
    assert lib.hcu_mlp_create(dims, 3, 64, ctypes.byref(m)) == hcu.HCU_OK
    n = ctypes.c_int64()
    assert lib.hcu_mlp_param_count(m, ctypes.byref(n)) == hcu.HCU_OK
    assert lib.hcu_mlp_forward(m, None, 1, None, 0) == hcu.HCU_NOT_BOUND
    lib.hcu_mlp_destroy(m)
    bad = (ctypes.c_int * 4)(64, 0, 128, 30)
    assert lib.hcu_mlp_create(bad, 3, 16, ctypes.byref(m)) == hcu.HCU_INVALID_ARG
    lib.hcu_mlp_destroy(m)
    print("sanitized host checks passed", flush=True)
""")


def _runtime():
    r = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isfile(path) else None


@pytest.mark.skipif(not os.path.exists(LIB_SAN),
                    reason="sanitized library not built (python -m paper_2507_23612_amd.build --sanitize)")
def test_host_code_clean_under_asan_and_ubsan():
    rt = _runtime()
    if rt is None:
        pytest.skip("sanitizer runtime not found")
    env = dict(os.environ)
    # the runtime goes first (it must initialise before anything it
    # instruments); whatever the environment already preloads stays loaded
    env["LD_PRELOAD"] = rt + (":" + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    # the interpreter itself is not instrumented: its allocations are not
    # leak-checked; every other report stops the child
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0:exitcode=86"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=87"
    code = f"ROOT = {ROOT!r}\nLIB_SAN = {LIB_SAN!r}\n" + CHILD
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout[-2000:] + "\n" + r.stderr[-4000:])
    assert r.returncode == 0, tail
    assert "sanitized host checks passed" in r.stdout, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, tail
