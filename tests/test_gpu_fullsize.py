"""Parity at full size: the benchmark's Ly=8, chi=3200 centre window (104 sectors, MPO
bond dimensions 28/26/28), in the tile shapes and K splits the benchmark runs, and the
Ly=10, chi=6000 centre window (150 sectors, flux 1/10) whose stated precision is FP32.

One matvec and both environment updates per precision against the FP64 oracle.
The environments have seeded Gaussian entries with the exact block structure of the
window (a contraction's result does not depend on the environments being physical), so
the oracle needs no sweep through the 256 sites; the MPO is the oracle's own."""
import sys

import numpy as np
import pytest

import workloads
from oracle import blocksparse as bs
from oracle import mpo as omp
from oracle import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1512_03318_amd as pk  # noqa: E402
from gpu_helpers import block_rel, max_rel, mpo_site, to_dev  # noqa: E402

TOL = {pk.DM_FP64: 1e-12, pk.DM_FP32: 2e-5, pk.DM_BF16X3: 1e-4}
CASES = [("ly8_chi3200", pk.DM_FP64), ("ly8_chi3200", pk.DM_FP32), ("ly8_chi3200", pk.DM_BF16X3),
         ("ly10_chi6000", pk.DM_FP64), ("ly10_chi6000", pk.DM_FP32)]
_cases = {}


def case(name):
    if name not in _cases:
        _case = _cases[name] = {}
        print(f"building the {name} window with the oracle ...", flush=True)
        sys.stdout.flush()
        wl = workloads.preset(name)
        m = omp.build(synth.cylinder_of(wl), wl.basis)
        j, ly = wl.j, wl.ly
        rng = np.random.default_rng(31)
        L = workloads.random_env(rng, wl.bonds[j], m.qbond[j], ly, "L")
        R = workloads.random_env(rng, wl.bonds[j + 2], m.qbond[j + 2], ly, "R")
        th = wl.theta()
        A = workloads.left_isometry(rng, wl.bonds[j], wl.bonds[j + 1], wl.qsite[j], ly)
        B = workloads.right_isometry(rng, wl.bonds[j + 1], wl.bonds[j + 2], wl.qsite[j + 1], ly)
        keys = bs.theta_keys(wl.bonds[j], wl.bonds[j + 2], wl.qsite[j], wl.qsite[j + 1], ly)
        _case.update(wl=wl, m=m, L=L, R=R, th=th, A=A, B=B, keys=keys,
                     heff=bs.heff_apply(L, m.W[j], m.W[j + 1], R, th),
                     envl=bs.env_left_update(L, A, m.W[j]),
                     envr=bs.env_right_update(R, B, m.W[j + 1]))
    return _cases[name]


@pytest.mark.parametrize("name,prec", CASES)
def test_fullsize_matvec(name, prec):
    c = case(name)
    tol = TOL[prec]
    wl, m = c["wl"], c["m"]
    j, ly = wl.j, wl.ly
    print(f"full-size matvec {name} prec={prec}", flush=True)
    a, cb = pk.Bond(wl.bonds[j]), pk.Bond(wl.bonds[j + 2])
    w1, w2 = mpo_site(m, j), mpo_site(m, j + 1)
    qs1 = [tuple(q) for q in m.qsite[j]]
    qs2 = [tuple(q) for q in m.qsite[j + 1]]
    Lf = to_dev(pk.pack(c["L"], pk.LAYOUT_ENV_L, ly, a, qw=m.qbond[j]))
    Rf = to_dev(pk.pack(c["R"], pk.LAYOUT_ENV_R, ly, cb, qw=m.qbond[j + 2]))
    plan = pk.HeffPlan(ly, a, cb, w1, w2, Lf, Rf, prec)
    x = to_dev(pk.pack(c["th"], pk.LAYOUT_THETA, ly, a, cb, qs1=qs1, qs2=qs2))
    y = torch.empty_like(x)
    pk.heff_apply(plan, x, y)
    torch.cuda.synchronize()
    got = pk.unpack(y.cpu().numpy(), pk.LAYOUT_THETA, ly, a, cb, qs1=qs1, qs2=qs2)
    err = max_rel(got, c["heff"], c["keys"])
    berr = block_rel(got, c["heff"], c["keys"])
    print(f"  max relative error {err:.3e}, worst block {berr:.3e}", flush=True)
    assert err < tol


@pytest.mark.parametrize("name,prec", CASES)
def test_fullsize_env_updates(name, prec):
    c = case(name)
    tol = TOL[prec]
    wl, m = c["wl"], c["m"]
    j, ly = wl.j, wl.ly
    print(f"full-size environment updates {name} prec={prec}", flush=True)
    a, b, cb = (pk.Bond(wl.bonds[k]) for k in (j, j + 1, j + 2))
    for left in (True, False):
        if left:
            W = mpo_site(m, j)
            env = to_dev(pk.pack(c["L"], pk.LAYOUT_ENV_L, ly, a, qw=m.qbond[j]))
            site = to_dev(pk.pack(c["A"], pk.LAYOUT_SITE, ly, a, b, qs1=[tuple(q) for q in m.qsite[j]]))
            _, n = pk.layout(pk.LAYOUT_ENV_L, ly, b, qw=m.qbond[j + 1])
            out = torch.empty(n, dtype=torch.complex128, device="cuda")
            pk.env_update_left(ly, a, b, W, env, site, out, prec)
            got = pk.unpack(out.cpu().numpy(), pk.LAYOUT_ENV_L, ly, b, qw=m.qbond[j + 1])
            ref = c["envl"]
        else:
            W = mpo_site(m, j + 1)
            env = to_dev(pk.pack(c["R"], pk.LAYOUT_ENV_R, ly, cb, qw=m.qbond[j + 2]))
            site = to_dev(pk.pack(c["B"], pk.LAYOUT_SITE, ly, b, cb, qs1=[tuple(q) for q in m.qsite[j + 1]]))
            _, n = pk.layout(pk.LAYOUT_ENV_R, ly, b, qw=m.qbond[j + 1])
            out = torch.empty(n, dtype=torch.complex128, device="cuda")
            pk.env_update_right(ly, b, cb, W, env, site, out, prec)
            got = pk.unpack(out.cpu().numpy(), pk.LAYOUT_ENV_R, ly, b, qw=m.qbond[j + 1])
            ref = c["envr"]
        assert set(ref) <= set(got)
        num = max(np.abs(got[k] - ref.get(k, 0)).max() for k in got)
        den = max(np.abs(v).max() for v in ref.values())
        print(f"  {'left' if left else 'right'}: max relative error {num / den:.3e}", flush=True)
        assert num / den < tol
