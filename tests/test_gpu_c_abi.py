"""The library from a plain C program (tests/c_abi/heff_driver.c): no Python and no
PyTorch in the process that runs the kernels, only include/mrdmrg.h, libmrdmrg.so and
the HIP runtime.  The test packs an oracle window problem, runs heff_driver as a child
process and compares with the FP64 oracle: its matvec, its Lanczos energy, both
environment updates (output sizes from dm_layout) and a two-instance batched Lanczos."""
import os
import struct
import subprocess
import sys

import numpy as np
import pytest

import workloads
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
    rng = np.random.default_rng(77)
    A = workloads.left_isometry(rng, wl.bonds[j], wl.bonds[j + 1], wl.qsite[j], ly)
    B = workloads.right_isometry(rng, wl.bonds[j + 1], wl.bonds[j + 2], wl.qsite[j + 1], ly)
    a, b, c = (pk.Bond(wl.bonds[k]) for k in (j, j + 1, j + 2))
    qs1 = [tuple(map(int, q)) for q in mpo.qsite[j]]
    qs2 = [tuple(map(int, q)) for q in mpo.qsite[j + 1]]
    blob = (struct.pack("<iii", ly, prec, 30) + _bond(wl.bonds[j]) + _bond(wl.bonds[j + 2])
            + _site(mpo.W[j], mpo.qbond[j], mpo.qbond[j + 1], mpo.qsite[j])
            + _site(mpo.W[j + 1], mpo.qbond[j + 1], mpo.qbond[j + 2], mpo.qsite[j + 1])
            + _arr(g.Lf) + _arr(g.Rf) + _arr(g.pack_theta(th))
            + _bond(wl.bonds[j + 1])
            + _arr(pk.pack(A, pk.LAYOUT_SITE, ly, a, b, qs1=qs1))
            + _arr(pk.pack(B, pk.LAYOUT_SITE, ly, b, c, qs1=qs2)))
    src, dst = tmp_path / "in.bin", tmp_path / "out.bin"
    src.write_bytes(blob)
    print(f"C driver prec={prec}", flush=True)
    sys.stdout.flush()
    r = subprocess.run([DRIVER, str(src), str(dst)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    out = dst.read_bytes()
    n = struct.unpack_from("<q", out, 0)[0]
    y = np.frombuffer(out, dtype=np.complex128, count=n, offset=8)
    pos = 8 + 16 * n
    energy, iters = struct.unpack_from("<di", out, pos)
    pos += 12
    envs = []
    for _ in range(2):
        m = struct.unpack_from("<q", out, pos)[0]
        envs.append(np.frombuffer(out, dtype=np.complex128, count=m, offset=pos + 8))
        pos += 8 + 16 * m
    eb = struct.unpack_from("<2d", out, pos)
    kb = struct.unpack_from("<2i", out, pos + 16)
    ref = bs.heff_apply(L, W1, W2, R, th)
    assert max_rel(g.unpack_theta(y), ref, keys) < tol
    mv = lambda v: bs.flatten(bs.heff_apply(L, W1, W2, R, bs.unflatten(v, keys)), keys)
    eo, _, ko, _, _ = olz.lanczos(mv, bs.flatten(th, keys), max_iter=30)
    etol = (1e-10 if prec == pk.DM_FP64 else 1e-6) * abs(eo)
    assert iters == ko
    assert abs(energy - eo) <= etol
    assert list(kb) == [ko, ko]
    assert all(abs(e - eo) <= etol for e in eb)
    # environment updates against the oracle
    envl = pk.unpack(envs[0], pk.LAYOUT_ENV_L, ly, b, qw=mpo.qbond[j + 1])
    envr = pk.unpack(envs[1], pk.LAYOUT_ENV_R, ly, b, qw=mpo.qbond[j + 1])
    for got, refd in ((envl, bs.env_left_update(L, A, W1)), (envr, bs.env_right_update(R, B, W2))):
        assert set(refd) <= set(got)
        num = max(np.abs(got[k] - refd.get(k, 0)).max() for k in got)
        den = max(np.abs(v).max() for v in refd.values())
        assert num / den < tol
