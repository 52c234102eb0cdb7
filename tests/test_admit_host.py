"""CPU check of the serving loop's device-memory heap and admission policy
(bfc_heap.h, bfc_admit.h), built for the host with sanitizers and driven by a
fake device: blocks never overlap or leave the budget, allocation fails only
when no free range is long enough, no busy scene is evicted, one request per
scene runs at a time, a request that cannot start is passed by a bounded
number of later ones, every request completes or is rejected (only when its
scene and step exceed the whole budget, or its creation failed), and the
loop always makes progress."""
import os
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2510_10256_amd", "csrc")


@pytest.fixture(scope="module")
def exe():
    d = tempfile.mkdtemp(prefix="admit_host_")
    out = os.path.join(d, "admit_host")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-Wall", "-Wextra", "-Werror", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", CSRC, os.path.join(HERE, "host", "admit_host.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out


@pytest.mark.parametrize("seed", range(1, 7))
def test_heap_against_unit_map(exe, seed):
    r = subprocess.run([exe, str(seed), "0"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.startswith("heap ok")


@pytest.mark.parametrize("seed", range(1, 13))
def test_admission_with_fake_device(exe, seed):
    r = subprocess.run([exe, str(seed), "1"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    f = dict(kv.split("=") for kv in r.stdout.split()[2:])
    # eviction binds under the budget, and a scene above the budget is turned away
    assert int(f["evicted"]) > 0 and int(f["too_big"]) > 0
    assert int(f["peak"]) <= int(f["size"])
