"""The library's host code (argument checks, sizes, the host CSR pattern,
the batch work-list code) rebuilt with AddressSanitizer on the host side
only (the device code is the ordinary build) and driven through its
host-only entry points in a child process running under the ASan runtime:
valid and malformed descriptions, every NULL argument the header allows,
patterns for p = 1..5.  No GPU is touched (plan creation is refused on the
host before any device call for the malformed descriptions used here); a
heap overflow, use after free or similar in that code aborts the child with
an ASan report."""
import glob
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2207_00280_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

CHILD = textwrap.dedent(r'''
    import ctypes, sys
    import numpy as np
    sys.path.insert(0, sys.argv[2])
    import workloads as W
    from paper_2207_00280_amd import igafem as ig
    ig.LIB_PATH = sys.argv[1]
    L = ig.lib()
    assert "gfx950" in ig.version()
    # valid descriptions: sizes and the host pattern, every degree
    for p in range(1, 6):
        for K in ((1, 1, 1), (3, 2, 4), (7, 1, 2)):
            d = ig.make_desc(p, K, [W.open_uniform_knots(k, p) for k in K])
            assert L.igaf_desc_check(ctypes.byref(d)) == 0
            sz = ig.desc_sizes(d)
            rp, col = ig.csr_pattern_host(d)
            assert rp[-1] == sz["nnz"] and len(col) == sz["nnz"]
            for a in range(3):
                r0, r1 = ig.desc_shared_run(d, a)
                assert 0 <= r0 <= r1 <= K[a]
            i = ctypes.c_int32()
            assert L.igaf_desc_shared_run(ctypes.byref(d), 3, ctypes.byref(i), ctypes.byref(i)) == ig.EINVAL
            assert L.igaf_desc_shared_run(ctypes.byref(d), 0, None, ctypes.byref(i)) == ig.EINVAL
    # repeated interior knots (accepted) and malformed ones (refused)
    t = W.repeated_knots([0.5], [3], 3)
    d = ig.make_desc(3, (len(t) - 7, 2, 2), [t, W.open_uniform_knots(2, 3), W.open_uniform_knots(2, 3)])
    assert L.igaf_desc_check(ctypes.byref(d)) == 0
    bad = []
    t = W.open_uniform_knots(4, 2).copy(); t[4], t[5] = t[5], t[4]
    bad.append((2, (4, 2, 2), [t, W.open_uniform_knots(2, 2), W.open_uniform_knots(2, 2)]))
    t = W.open_uniform_knots(3, 2).copy(); t[1] = 0.1
    bad.append((2, (3, 2, 2), [t, W.open_uniform_knots(2, 2), W.open_uniform_knots(2, 2)]))
    t = W.repeated_knots([0.5], [4], 2)
    bad.append((2, (len(t) - 5, 1, 1), [t, W.open_uniform_knots(1, 2), W.open_uniform_knots(1, 2)]))
    t = W.open_uniform_knots(3, 1).copy(); t[2] = float("nan")
    bad.append((1, (3, 1, 1), [t, W.open_uniform_knots(1, 1), W.open_uniform_knots(1, 1)]))
    for p, K, knots in bad:
        d = ig.make_desc(p, K, knots)
        assert L.igaf_desc_check(ctypes.byref(d)) == ig.EINVAL
        h = ctypes.c_void_p()
        assert L.igaf_plan_create(ctypes.byref(d), ctypes.byref(h)) == ig.EINVAL and h.value is None
        assert len(L.igaf_last_error()) > 0
    # sizes refused before any knot is read (degree, element counts) ...
    for p, K0 in ((0, 2), (2, 0), (2, 1 << 21)):
        d = ig.make_desc(2, (2, 2, 2), [W.open_uniform_knots(2, 2)] * 3)
        d.degree, d.nelem[0] = p, K0
        assert L.igaf_desc_check(ctypes.byref(d)) == ig.EINVAL
    # ... and a global size beyond int32 column indices, with full knot vectors
    d = ig.make_desc(1, (2000, 2000, 2000), [W.open_uniform_knots(2000, 1)] * 3)
    assert L.igaf_desc_check(ctypes.byref(d)) == ig.EINVAL
    assert "int32" in L.igaf_last_error().decode()
    # NULL arguments
    assert L.igaf_desc_check(None) == ig.EINVAL
    assert L.igaf_plan_create(None, None) == ig.EINVAL
    assert L.igaf_plan_sizes(None, None, None, None, None, None) == ig.EINVAL
    assert L.igaf_csr_pattern_host(None, None, None) == ig.EINVAL
    assert L.igaf_desc_shared_run(None, 0, None, None) == ig.EINVAL
    assert L.igaf_element_matrices(None, 1, None, None, None, None) == ig.EINVAL
    assert L.igaf_integrate_assemble(None, 1, None, None, None, None, None, None) == ig.EINVAL
    assert L.igaf_kappa_grad(None, None, None, 1.0, 1.0, 1.0, None, None, None) == ig.EINVAL
    assert L.igaf_bilinear_form(None, None, None, None, 1.0, 1.0, None, None) == ig.EINVAL
    assert L.igaf_apply(None, None, None, 1.0, 1.0, None, None, None) == ig.EINVAL
    assert L.igaf_apply_static(None, None, None, 1.0, 1.0, None, None) == ig.EINVAL
    assert L.igaf_wq_prepare(None) == ig.EINVAL
    assert L.igaf_batch_create(None, 0, None) == ig.EINVAL
    assert L.igaf_batch_info(None, None, None, None) == ig.EINVAL
    assert L.igaf_batch_set_degree_config(None, 3, 0, 1, 16) == ig.EINVAL
    L.igaf_plan_destroy(None)
    L.igaf_batch_destroy(None)
    print("host checks ok")
''')


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_host_code_under_address_sanitizer(tmp_path):
    rt = _asan_runtime()
    if rt is None or not os.path.exists(HIPCC):
        pytest.skip("no hipcc / clang ASan runtime in this image")
    from paper_2207_00280_amd import build as b

    objs = []
    flags = [f for f in b.FLAGS if f != "-O3"] + ["-O1", "-g"]
    for src in b.SOURCES:
        obj = os.path.join(str(tmp_path), src + ".o")
        cmd = [HIPCC] + flags + ["-c", os.path.join(b.CSRC, src), "-o", obj]
        if src.endswith(".cpp"):   # the host-only sources: instrumented on the host side
            cmd = [HIPCC] + flags + ["-x", "hip", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                                     "-fno-omit-frame-pointer", "-c", os.path.join(b.CSRC, src), "-o", obj]
        else:
            prebuilt = os.path.join(b.OBJ, src + ".o")
            if os.path.exists(prebuilt) and os.path.getmtime(prebuilt) >= os.path.getmtime(os.path.join(b.CSRC, src)):
                objs.append(prebuilt)
                continue
        subprocess.run(cmd, check=True, capture_output=True)
        objs.append(obj)
    lib = os.path.join(str(tmp_path), "libigafem_asan.so")
    subprocess.run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-shared-libasan", "-o", lib] + objs, check=True, capture_output=True)
    # the ASan runtime must come first among the preloaded libraries; any
    # library the environment already preloads stays in the list after it
    pre = " ".join(x for x in (rt, os.environ.get("LD_PRELOAD", "")) if x)
    env = dict(os.environ, LD_PRELOAD=pre, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               HIP_VISIBLE_DEVICES="")
    r = subprocess.run([sys.executable, "-c", CHILD, lib, ROOT], env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0 and "host checks ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
    assert "AddressSanitizer" not in r.stderr
