"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only, no GPU calls).

The library's host code (argument validation, status and error strings of every entry point; the
device code is built as usual) and the oracle's reference tree (tree_ref.c, every list builder) are
compiled with -fsanitize=address,undefined for the host only and driven from a child process that
preloads the sanitizer runtime; any report aborts the child, which fails the test.
"""
import glob
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2507_21913_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/lib/llvm/bin/clang"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def _asan_runtime():
    libs = glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    return libs[0] if libs else None


pytestmark = pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG) and _asan_runtime()),
                                reason="ROCm clang and its sanitizer runtime are needed")


@pytest.fixture(scope="module")
def sanitized_libs(tmp_path_factory):
    d = tmp_path_factory.mktemp("asan")
    procs = []
    objs = []
    for f in ("api.hip", "tree.hip", "fmm.hip", "tune.hip"):
        o = str(d / (f + ".o"))
        objs.append(o)
        procs.append(subprocess.Popen([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
                                       "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + SAN +
                                      ["-c", os.path.join(CSRC, f), "-o", o],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out.decode(errors="replace")[-2000:]
    lib = str(d / "libfmmhp_asan.so")
    subprocess.check_call([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-shared-libasan"] + SAN +
                          ["-o", lib] + objs)
    tree = str(d / "libtree_ref_asan.so")
    subprocess.check_call([CLANG, "-O1", "-g", "-ffp-contract=off", "-fPIC", "-shared", "-shared-libasan",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           "-o", tree, os.path.join(ROOT, "oracle", "tree_ref.c"), "-lm"])
    return lib, tree


DRIVER = textwrap.dedent("""
    import ctypes, sys
    sys.path.insert(0, sys.argv[3])
    import numpy as np
    import paper_2507_21913_amd as F
    F.LIB_PATH = sys.argv[1]
    L = F.lib()
    assert sorted(F.header_functions()) == sorted(n for n in F.header_functions() if hasattr(L, n))
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    good = F.Opts(20, 40, 0, 0)
    st = []
    st.append(L.fmmhp_plan_create(10, fake, fake, None, None, 1.0, 0.0, ctypes.byref(good), None, None))
    st.append(L.fmmhp_plan_create(0, fake, fake, None, None, 1.0, 0.0, ctypes.byref(good), None, ctypes.byref(h)))
    st.append(L.fmmhp_plan_create(10, fake, fake, fake, None, 1.0, 0.0, ctypes.byref(good), None, ctypes.byref(h)))
    for re, im in ((0.0, 0.0), (-1.0, 0.5), (1.0, -0.1), (float("nan"), 0.0), (float("inf"), 0.0)):
        st.append(L.fmmhp_plan_create(10, fake, fake, None, None, re, im, ctypes.byref(good), None, ctypes.byref(h)))
        L.fmmhp_last_error_message()
    for o in (F.Opts(0, 40, 0, 0), F.Opts(41, 40, 0, 0), F.Opts(20, 0, 0, 0), F.Opts(20, 40, 31, 0),
              F.Opts(20, 40, 0, 64), F.Opts(20, 40, 0, 12), F.Opts(20, 40, 0, 0, 4, 0), F.Opts(20, 40, 0, 0, 0, 17)):
        st.append(L.fmmhp_plan_create(10, fake, fake, None, None, 1.0, 0.0, ctypes.byref(o), None, ctypes.byref(h)))
        L.fmmhp_last_error_message()
    st.append(L.fmmhp_plan_create_targets(0, fake, fake, 10, fake, fake, 1.0, 0.0, ctypes.byref(good), None,
                                          ctypes.byref(h)))
    off = (ctypes.c_int64 * 3)(0, 5, 3)
    lam = (ctypes.c_double * 4)(1.0, 0.0, 1.0, 0.0)
    st.append(L.fmmhp_batch_plan_create(2, ctypes.cast(off, ctypes.c_void_p), fake, fake,
                                        ctypes.cast(lam, ctypes.c_void_p), ctypes.byref(good), None, ctypes.byref(h)))
    for f in (L.fmmhp_eval, L.fmmhp_eval_complex, L.fmmhp_eval_noalloc):
        st.append(f(None, 1, None, None, None))
    st.append(L.fmmhp_backward(None, None, None, None, None, None, None, None))
    st.append(L.fmmhp_backward_device(None, None, None, None, None, None, None, None))
    assert L.fmmhp_plan_destroy(None) == 0  # destroying NULL is a no-op
    for k in range(8):
        L.fmmhp_status_string(k)
    assert h.value is None and all(s != 0 for s in st), st
    # the reference tree, every list, on random and clustered points with coincident ones
    import oracle.tree as T
    T._LIB = sys.argv[2]
    rng = np.random.default_rng(3)
    for n, leaf in ((300, 8), (2000, 16), (500, 1)):
        x = rng.uniform(0.0, 1.0, n)
        y = rng.uniform(1e-3, 1.0, n)
        x[: n // 10] = 0.25
        y[: n // 10] = 0.5
        t = T.build(x, y, leaf)
        assert t["nbox"] > 0 and sum(t["count"][t["leaf"] == 1]) == n
    print("SANITIZED_OK")
""")


def test_host_code_clean_under_sanitizers(sanitized_libs, tmp_path):
    lib, tree = sanitized_libs
    drv = tmp_path / "drive.py"
    drv.write_text(DRIVER)
    env = dict(os.environ, LD_PRELOAD=_asan_runtime(), ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, str(drv), lib, tree, ROOT], env=env, capture_output=True, text=True,
                       timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "SANITIZED_OK" in out, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
