"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code, run on the CPU.

* The oracle (oracle.c, oracle3d.c) with gcc's sanitizers, driven by tests/sanitize/oracle_driver.c
  through every exported function on small lattices, refusals included.
* The library's host code (cgkmc.hip with the sanitizers on the host side only; the device code
  is compiled as usual but never launched), driven by tests/sanitize/host_driver.c through the
  arena planning of every kernel family and the argument checks every entry point makes before
  any HIP call.

Any sanitizer report aborts the driver (halt_on_error), so the test passes only on a clean run.
Leak detection is off for the library driver: the HIP runtime keeps process-lifetime
allocations."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-8000:]}"
    return r


def test_oracle_under_address_and_undefined_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_driver")
        _run(["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "oracle"), os.path.join(HERE, "oracle_driver.c"),
              os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "oracle", "oracle3d.c"), "-lm", "-o", exe])
        r = _run([exe], env=ENV)
        assert "oracle driver ok" in r.stdout


def test_library_host_code_under_address_and_undefined_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        lib = os.path.join(d, "libcgkmc_san.so")
        exe = os.path.join(d, "host_driver")
        san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-Xarch_host", "-fno-sanitize-recover=all"]
        _run([HIPCC, "--offload-arch=gfx950", "-std=c++17", "-O1", "-g", "-fPIC", "-shared",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *san,
              "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1407_5026_amd", "csrc"),
              "-o", lib, os.path.join(ROOT, "paper_1407_5026_amd", "csrc", "cgkmc.hip")])
        _run([HIPCC, "-x", "c++", "-O1", "-g", *san, "-I", os.path.join(ROOT, "include"),
              os.path.join(HERE, "host_driver.c"), "-o", exe, "-L", d, "-lcgkmc_san", f"-Wl,-rpath,{d}"])
        env = dict(ENV, ASAN_OPTIONS="detect_leaks=0", HIP_VISIBLE_DEVICES="")
        r = _run([exe], env=env)
        assert "host driver ok" in r.stdout
