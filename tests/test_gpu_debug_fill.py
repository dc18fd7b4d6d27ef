"""No step kernel reads an LDS cell that no thread wrote for the plane in hand:
the debug build of the library (libsclbm_debug.so) overwrites every density
slot and exchange buffer with NaN before each plane, so such a read would turn
populations into NaN.  Every step kernel, tile shape and storage format on
ragged and whole-row boxes in both boundary modes gives the same bits with the
regular and the debug build (tests/debug_fill_cases.py, one process each)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2112_09972_amd")


def run_cases(lib):
    env = dict(os.environ, SCLBM_LIBRARY=lib)
    out = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "debug_fill_cases.py")], env=env, cwd=ROOT,
                         capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-3000:]
    return json.loads(out.stdout.strip().splitlines()[-1])


def test_debug_fill_build_gives_the_same_bits():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    debug = os.path.join(PKG, "libsclbm_debug.so")
    if not os.path.exists(debug):
        pytest.fail("libsclbm_debug.so is not built (build() builds it)")
    reg = run_cases(os.path.join(PKG, "libsclbm.so"))
    dbg = run_cases(debug)
    assert dbg["library"].endswith("libsclbm_debug.so")
    assert set(reg["cases"]) == set(dbg["cases"])
    for key in reg["cases"]:
        assert dbg["cases"][key]["finite"], key
        assert reg["cases"][key]["sha"] == dbg["cases"][key]["sha"], key
