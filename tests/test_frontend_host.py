"""The Python front end fails loudly instead of falling back: a missing HIP
library and host tensors are errors, not a CPU path (no GPU needed)."""
import importlib
import os
import subprocess
import sys

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_missing_library_is_an_error():
    # a fresh interpreter, so the loaded library of this process is untouched
    code = (
        "import paper_2508_19140_amd._lib as L\n"
        "L.LIB_PATH = '/nonexistent/libinpc_raster.so'\n"
        "L._lib = None\n"
        "try:\n"
        "    L.lib()\n"
        "except RuntimeError as e:\n"
        "    print('raised:', e)\n"
        "else:\n"
        "    print('loaded')\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    assert "raised:" in r.stdout and "no non-HIP fallback" in r.stdout


def test_rasterize_rejects_host_tensors():
    inpc = importlib.import_module("paper_2508_19140_amd")
    from scenes import make_camera
    pos = torch.zeros(4, 3)
    op = torch.zeros(4)
    feat = torch.zeros(4, 2)
    with pytest.raises(ValueError, match="GPU"):
        inpc.rasterize(pos, op, feat, make_camera(8, 8, 4.0))
