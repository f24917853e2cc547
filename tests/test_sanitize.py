"""Host sanitizer builds (AddressSanitizer + UndefinedBehaviorSanitizer):
the oracle's C decomposition on random graphs, and the C ABI's host-side
argument and snapshot checks (the library's host code instrumented, its
device code as usual).  CPU only: nothing here launches a kernel."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1612_09368_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, **kw):
    out = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert out.returncode == 0, (cmd, out.stdout[-3000:], out.stderr[-3000:])
    return out


def test_oracle_bz_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc missing")
    exe = tmp_path / "bz_san"
    _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
          "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "bz.c"),
          os.path.join(HERE, "host", "bz_sanitize_main.c"), "-o", str(exe)])
    out = _run([str(exe)], env=ENV, timeout=300)
    assert "bz: ok" in out.stdout


def test_abi_host_paths_under_sanitizers(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc missing")
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include")]
    api = tmp_path / "cm_api_san.o"
    kern = tmp_path / "cm_kernels.o"
    jobs = [subprocess.Popen([HIPCC, *common, *SAN, "-c", os.path.join(CSRC, "cm_api.hip"), "-o", str(api)],
                             stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)]
    # the device code needs no instrumentation: reuse the library build's
    # object when it is newer than every source, else compile it
    built = os.path.join(ROOT, "paper_1612_09368_amd", "_build", "cm_kernels.o")
    newest = max(os.path.getmtime(os.path.join(CSRC, f)) for f in os.listdir(CSRC))
    if os.path.exists(built) and os.path.getmtime(built) > newest:
        kern = built
    else:
        jobs.append(subprocess.Popen([HIPCC, *common, "-c", os.path.join(CSRC, "cm_kernels.hip"), "-o", str(kern)],
                                     stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for j in jobs:
        out, _ = j.communicate()
        assert j.returncode == 0, out[-3000:]
    main = tmp_path / "abi_main.o"
    _run([HIPCC, *common, *SAN, "-c", os.path.join(HERE, "host", "abi_sanitize_main.cpp"), "-o", str(main)])
    exe = tmp_path / "abi_san"
    _run([HIPCC, "--offload-arch=gfx950", *SAN, str(main), str(api), str(kern), "-o", str(exe),
          "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"])
    out = _run([str(exe), str(tmp_path)], env=ENV, timeout=300)
    assert "abi: ok" in out.stdout
