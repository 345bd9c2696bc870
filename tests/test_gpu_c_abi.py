"""The library from a plain C program (tests/c_abi/heff_driver.c): no Python and no
PyTorch in the process that runs the kernels, only include/mrdmrg.h, libmrdmrg.so and
the HIP runtime.  The test packs an oracle window problem, runs heff_driver as a child
process and compares its matvec and Lanczos energy with the FP64 oracle."""
import os
import struct
import subprocess
import sys

import numpy as np
import pytest

from oracle import blocksparse as bs
from oracle import lanczos as olz

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1512_03318_amd as pk  # noqa: E402
from gpu_helpers import WindowGPU, max_rel, problem  # noqa: E402

DRIVER = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "heff_driver")


def _bond(d):
    qs = sorted(d)
    return (struct.pack("<i", len(qs)) + b"".join(struct.pack("<ii", *q) for q in qs)
            + b"".join(struct.pack("<i", d[q]) for q in qs))


def _site(W, ql, qr, qs):
    W = np.ascontiguousarray(np.asarray(W, dtype=np.complex128))
    dl, _, _, dr = W.shape
    ch = lambda qq: b"".join(struct.pack("<ii", int(a), int(b)) for a, b in np.asarray(qq).reshape(-1, 2))
    return struct.pack("<ii", dl, dr) + ch(ql) + ch(qr) + ch(qs) + W.tobytes()


def _arr(x):
    x = np.ascontiguousarray(x, dtype=np.complex128)
    return struct.pack("<q", x.size) + x.tobytes()


@pytest.mark.parametrize("prec,tol", [(pk.DM_FP64, 1e-12), (pk.DM_BF16X3, 1e-4)])
def test_c_program_matvec_and_lanczos(prec, tol, tmp_path):
    assert os.path.exists(DRIVER), "build heff_driver with __graft_entry__.build()"
    wl, L, W1, W2, R, th, keys, mpo = problem("ly4_chi64")
    j, ly = wl.j, wl.ly
    g = WindowGPU(wl, L, R, mpo)
    blob = (struct.pack("<iii", ly, prec, 30) + _bond(wl.bonds[j]) + _bond(wl.bonds[j + 2])
            + _site(mpo.W[j], mpo.qbond[j], mpo.qbond[j + 1], mpo.qsite[j])
            + _site(mpo.W[j + 1], mpo.qbond[j + 1], mpo.qbond[j + 2], mpo.qsite[j + 1])
            + _arr(g.Lf) + _arr(g.Rf) + _arr(g.pack_theta(th)))
    src, dst = tmp_path / "in.bin", tmp_path / "out.bin"
    src.write_bytes(blob)
    print(f"C driver prec={prec}", flush=True)
    sys.stdout.flush()
    r = subprocess.run([DRIVER, str(src), str(dst)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    out = dst.read_bytes()
    n = struct.unpack_from("<q", out, 0)[0]
    y = np.frombuffer(out, dtype=np.complex128, count=n, offset=8)
    energy, iters = struct.unpack_from("<di", out, 8 + 16 * n)
    ref = bs.heff_apply(L, W1, W2, R, th)
    assert max_rel(g.unpack_theta(y), ref, keys) < tol
    mv = lambda v: bs.flatten(bs.heff_apply(L, W1, W2, R, bs.unflatten(v, keys)), keys)
    eo, _, ko, _, _ = olz.lanczos(mv, bs.flatten(th, keys), max_iter=30)
    assert iters == ko
    assert abs(energy - eo) <= (1e-10 if prec == pk.DM_FP64 else 1e-6) * abs(eo)
