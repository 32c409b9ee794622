"""The host side of the C-ABI library under AddressSanitizer, without a GPU.

The library is rebuilt with host-side ASan (device code untouched) and a
child process, with the ASan runtime preloaded, loads it in place of the
regular build and runs the host ABI checks (argument validation before any
device call, the tune-table parser) plus a seeded fuzz of the tune-file
reader.  Any invalid host memory access aborts the child with an ASan
report."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_2605_25974_amd import build as B  # noqa: E402

CHILD = r"""
import os, sys
import numpy as np
sys.path.insert(0, {root!r})
import paper_2605_25974_amd as pl
pl.LIB_PATH = {lib!r}
import pytest
rc = pytest.main(["-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                  os.path.join({root!r}, "tests", "test_abi_host.py")])
if rc != 0:
    sys.exit(int(rc))
assert os.path.samefile(pl.LIB_PATH, {lib!r})
rng = np.random.default_rng(7)
path = os.path.join({tmp!r}, "fuzz.txt")
for i in range(2000):
    if i % 2:
        data = bytes(rng.integers(0, 256, int(rng.integers(0, 200)), dtype=np.uint8))
    else:
        vals = rng.integers(-5, 5000, int(rng.integers(0, 12)))
        data = (" ".join(str(int(v)) for v in vals) + "\n").encode()
    with open(path, "wb") as f:
        f.write(data)
    try:
        pl.tune_load(path)
    except pl.PauliError:
        pass
pl.tune_save(os.path.join({tmp!r}, "out.txt"))
print("ASAN-CHILD-DONE", flush=True)
"""


@pytest.mark.skipif(not os.path.exists(B.HIPCC), reason="hipcc not installed")
def test_host_abi_under_asan(tmp_path):
    rt = B.asan_runtime()
    if rt is None:
        pytest.skip("the compiler ships no shared ASan runtime")
    lib = B.build_asan()
    env = dict(os.environ)
    env["LD_PRELOAD"] = rt
    # the interpreter itself is not instrumented: its allocations are not leaks of ours
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["HIP_VISIBLE_DEVICES"] = ""  # host paths only, even on a machine with a GPU
    code = CHILD.format(root=ROOT, lib=lib, tmp=str(tmp_path))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=900, cwd=str(tmp_path))
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert r.returncode == 0 and "ASAN-CHILD-DONE" in out, out[-4000:]
    shutil.rmtree(B.ASAN_DIR, ignore_errors=True)
