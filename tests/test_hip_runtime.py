"""The package and PyTorch share one HIP runtime, whichever is imported first (a test
module that loads the library at collection must not leave a second runtime behind for
the GPU tests)."""
import subprocess
import sys

import pytest


def test_single_hip_runtime_when_library_loads_first():
    pytest.importorskip("torch")
    code = (
        "import paper_1512_03318_amd\n"
        "import torch\n"
        "libs = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
        "print(len(libs))\n"
    )
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, check=True,
                         cwd=__import__("os").path.dirname(__import__("os").path.dirname(__file__)))
    assert out.stdout.strip().splitlines()[-1] == "1", out.stdout
