"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only, no GPU needed).

Every source of libfem is compiled with the sanitizers on the host side only
(device code is built as usual) and linked with tests/host/abi_host_check.cpp
into one executable, which runs the argument checks of the C ABI, the parsing
and writing of the batch tuner's cache file (malformed, truncated, oversized
and binary lines), the quadrature-rule builder and the parameter checks of the
function catalogue. A sanitizer report or a failed check fails the test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "hostcheck")
DRIVER = os.path.join(ROOT, "tests", "host", "abi_host_check.cpp")
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _stale(target, sources):
    if not os.path.exists(target):
        return True
    t = os.path.getmtime(target)
    return any(os.path.getmtime(s) > t for s in sources)


def build_host_check():
    import concurrent.futures as cf
    from paper_1409_4618_amd import build as b
    os.makedirs(OUT, exist_ok=True)
    headers = [os.path.join(b.CSRC, f) for f in os.listdir(b.CSRC) if f.endswith(".h")]
    headers.append(os.path.join(ROOT, "include", "fem.h"))
    jobs = [(os.path.join(b.CSRC, s), os.path.join(OUT, os.path.splitext(s)[0] + ".o"), b.SOURCE_FLAGS.get(s, []))
            for s in b.SOURCES]
    jobs.append((DRIVER, os.path.join(OUT, "abi_host_check.o"), ["-x", "hip"]))

    def compile_one(job):
        src, obj, extra = job
        if not _stale(obj, [src] + headers):
            return
        cmd = [b.HIPCC, *b.COMMON, *b.DEVICE_FLAGS, *SAN_HOST, *extra, "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        list(ex.map(compile_one, jobs))
    exe = os.path.join(OUT, "abi_host_check")
    objs = [j[1] for j in jobs]
    if _stale(exe, objs):
        cmd = [CLANG, "-fsanitize=address,undefined", *objs, "-L/opt/rocm/lib", "-lamdhip64",
               "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stderr}")
    return exe


@pytest.mark.skipif(not os.path.exists(CLANG) or shutil.which("hipcc") is None and
                    not os.path.exists("/opt/rocm/bin/hipcc"), reason="ROCm toolchain not installed")
def test_host_code_under_sanitizers(tmp_path):
    exe = build_host_check()
    env = dict(os.environ)
    # the HIP runtime keeps allocations until exit by design: no leak report
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["HIP_VISIBLE_DEVICES"] = ""
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "host checks passed" in r.stdout
