"""The partition's iteration-stamped keys (cm_keys.h), checked on the host:
keys fall strictly with (iteration, round) over the whole stamp range a
handle uses before it restarts its stamps, and matched_before accepts
exactly the earlier rounds of the same iteration."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_key_arithmetic_across_the_stamp_range(tmp_path):
    exe = tmp_path / "keys_check"
    subprocess.check_call(["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                           os.path.join(HERE, "host", "keys_check.cpp"), "-o", str(exe)],
                          stderr=subprocess.DEVNULL)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout
    assert "keys: ok" in out.stdout
