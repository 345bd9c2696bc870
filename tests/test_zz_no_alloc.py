"""env_update_left_noalloc (the left environment update whose tables and intermediates
live in the library's fixed per-device region) against env_update_left, called through
the C ABI: equal results bit for bit, on two calls in a row whose second input is
smaller (the region keeps the first call's contents), in every precision, and against
the FP64 oracle; a window whose scratch does not fit is refused before any work."""
import sys

import numpy as np
import pytest

import workloads
from oracle import blocksparse as bs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1512_03318_amd as pk  # noqa: E402
from gpu_helpers import mpo_site, problem, to_dev  # noqa: E402

TOL = {pk.DM_FP64: 1e-12, pk.DM_FP32: 2e-5, pk.DM_BF16X3: 1e-4}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def left_case(name, seed):
    wl, L, W1, W2, R, th, keys, mpo = problem(name)
    j, ly = wl.j, wl.ly
    rng = np.random.default_rng(seed)
    A = workloads.left_isometry(rng, wl.bonds[j], wl.bonds[j + 1], wl.qsite[j], ly)
    a, b = pk.Bond(wl.bonds[j]), pk.Bond(wl.bonds[j + 1])
    W = mpo_site(mpo, j)
    Ld = to_dev(pk.pack(L, pk.LAYOUT_ENV_L, ly, a, qw=mpo.qbond[j]))
    Ad = to_dev(pk.pack(A, pk.LAYOUT_SITE, ly, a, b, qs1=[tuple(q) for q in mpo.qsite[j]]))
    _, n = pk.layout(pk.LAYOUT_ENV_L, ly, b, qw=mpo.qbond[j + 1])
    ref = bs.env_left_update(L, A, mpo.W[j])
    return ly, a, b, W, Ld, Ad, n, ref, mpo.qbond[j + 1]


@pytest.mark.parametrize("prec", [pk.DM_FP64, pk.DM_FP32, pk.DM_BF16X3])
def test_noalloc_equals_env_update_left(prec):
    # the larger window first, then a smaller one over the same region
    for name, seed in (("ly6_chi200", 3), ("ly4_chi64", 4)):
        say(f"env_update_left_noalloc {name} prec={prec}")
        ly, a, b, W, Ld, Ad, n, ref, qw = left_case(name, seed)
        want = torch.empty(n, dtype=torch.complex128, device="cuda")
        got = torch.full((n,), complex("nan"), dtype=torch.complex128, device="cuda")
        pk.env_update_left(ly, a, b, W, Ld, Ad, want, prec)
        pk.env_update_left_noalloc(ly, a, b, W, Ld, Ad, got, prec)
        torch.cuda.synchronize()
        assert torch.equal(got, want), name
        blocks = pk.unpack(got.cpu().numpy(), pk.LAYOUT_ENV_L, ly, b, qw=qw)
        num = max(np.abs(blocks[k] - ref.get(k, 0)).max() for k in blocks)
        den = max(np.abs(v).max() for v in ref.values())
        say(f"  bit-identical to env_update_left; relative error vs the oracle {num / den:.3e}")
        assert num / den < TOL[prec]


def test_noalloc_refuses_what_does_not_fit():
    # the Ly=8, chi=3200 window's left update needs several hundred MB of scratch
    wl = workloads.preset("ly8_chi3200")
    j, ly = wl.j, wl.ly
    m = pk.HofstadterMPO(wl.Ly, wl.Lx, wl.flux[0], wl.flux[1], wl.t, wl.V, wl.basis)
    W = m.site(j)
    a, b = pk.Bond(wl.bonds[j]), pk.Bond(wl.bonds[j + 1])
    _, nl = pk.layout(pk.LAYOUT_ENV_L, ly, a, qw=W.ql)
    _, ns = pk.layout(pk.LAYOUT_SITE, ly, a, b, qs1=W.qs)
    _, no = pk.layout(pk.LAYOUT_ENV_L, ly, b, qw=W.qr)
    L = torch.zeros(nl, dtype=torch.complex128, device="cuda")
    A = torch.zeros(ns, dtype=torch.complex128, device="cuda")
    out = torch.full((no,), 7.0, dtype=torch.complex128, device="cuda")
    with pytest.raises(pk.LibraryError) as e:
        pk.env_update_left_noalloc(ly, a, b, W, L, A, out, pk.DM_FP64)
    assert e.value.code == pk.DM_ERR_ALLOC
    assert "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())  # refused before any work was queued
