"""Host code of the library under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only).

The host side of the library (contraction planner, workspace arena, tape,
checkpoint and SVD-record bookkeeping, configuration validation) runs in full
in the dry run behind ctm_workspace_size: every allocation, every tensor view
and every control-flow branch of a sweep, a move, the energy and the reverse
pass, with the device calls skipped.  This test compiles ctm.cpp and
engine.cpp again with the host pass instrumented (the device code of those
files and the kernel objects are the ordinary build), loads that library in a
child process with the sanitizer runtime preloaded, and sizes a set of
configurations that between them take every branch of the path: both
precisions of the contractions, chi_I < chi_E, p = 4, the App. B projector
flags alone and together, checkpoint blocks with a shorter last block, forward
only, and rejected configurations.  Any sanitizer report fails the test.
"""
import glob
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2502_10298_amd import build as bld  # noqa: E402

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _asan_runtime():
    for pat in ("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so",
                "/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"):
        hits = sorted(glob.glob(pat))
        if hits:
            return hits[-1]
    return None


CHILD = textwrap.dedent("""
    import sys
    sys.path.insert(0, {root!r})
    from paper_2502_10298_amd import binding as b
    b.LIB_PATH = {lib!r}
    cases = [
        # Lx, Ly, p, D, chi_E, chi_I, prec, grad, n, ckpt, alt_yr, half_teal
        (1, 1, 2, 2, 8, 8, "fp64", False, 0, 1, False, False),
        (1, 1, 2, 2, 8, 8, "fp64", True, 3, 2, False, False),
        (2, 2, 2, 8, 128, 128, "bf16x3", True, 4, 4, False, False),
        (2, 2, 2, 8, 128, 128, "bf16x3", True, 7, 5, True, True),
        (1, 2, 4, 4, 32, 16, "fp32", True, 3, 2, True, False),
        (1, 1, 2, 6, 72, 72, "bf16x6", True, 40, 5, False, True),
        (2, 1, 2, 3, 12, 7, "fp64", True, 5, 5, True, True),
        (1, 1, 4, 12, 170, 170, "bf16x3", False, 0, 1, False, False),
    ]
    for (Lx, Ly, p, D, ce, ci, prec, grad, n, ck, alt, half) in cases:
        cfg = b.make_config(Lx, Ly, p, D, ce, ci, prec=prec, alt_yr=alt, half_teal=half)
        need = b.workspace_size(cfg, grad, n, ck)
        assert need > 0
        assert b.lib().ctm_env_elems(b.ctypes.byref(cfg)) > 0
        assert b.lib().ctm_projectors_elems(b.ctypes.byref(cfg)) > 0
        print("sized", Lx, Ly, p, D, ce, ci, prec, grad, n, ck, alt, half, need, flush=True)
    # rejected configurations: chi_I below D with the identity boundary, a
    # rank-limited M beyond the Householder limit (teal half projectors at
    # chi_E D^2 > 8192)
    for (Lx, Ly, p, D, ce, ci, half) in [(1, 1, 2, 4, 8, 2, False), (1, 1, 2, 12, 128, 128, True)]:
        cfg = b.make_config(Lx, Ly, p, D, ce, ci, half_teal=half)
        try:
            b.workspace_size(cfg, False, 0, 1)
        except b.CtmError as e:
            assert e.status == b.CTM_EINVAL
            print("rejected", Lx, Ly, p, D, ce, ci, half, flush=True)
        else:
            raise AssertionError("configuration accepted")
    print("done", flush=True)
""")


def test_host_code_under_asan_and_ubsan(tmp_path):
    asan = _asan_runtime()
    if asan is None or not os.path.exists(HIPCC):
        pytest.skip("hipcc or the clang sanitizer runtime is not installed")
    # the kernel objects of the ordinary build (compiled here when absent)
    os.makedirs(bld.BUILD, exist_ok=True)
    kernel_objs = []
    for src in bld.SOURCES:
        if src.endswith(".hip"):
            obj = os.path.join(bld.BUILD, src + ".o")
            if not os.path.exists(obj):
                obj = bld._compile(src)
            kernel_objs.append(obj)
    # host pass of the two host sources instrumented; each sanitizer flag
    # applies to the host compilation only
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
    flags = [f for f in bld.FLAGS if f != "-O3"] + ["-O1", "-g"]
    procs, objs = [], []
    for src in ("ctm.cpp", "engine.cpp"):
        obj = str(tmp_path / (src + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([HIPCC, *flags, *san, "-x", "hip", "-c", os.path.join(bld.CSRC, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out[-3000:]
    lib = str(tmp_path / "libsplitctm_san.so")
    r = subprocess.run([HIPCC, f"--offload-arch={bld.ARCH}", "-shared", "-fPIC", *san[:4], "-o", lib, *objs,
                        *kernel_objs], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, lib=lib)], capture_output=True, text=True,
                       env=env, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert out.count("sized") == 8 and out.count("rejected") == 2 and "done" in out, out[-4000:]
