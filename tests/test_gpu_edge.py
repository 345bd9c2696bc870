"""Edge cases of the block structure on the GPU, against the FP64 oracle.

* Ragged blocks: every sector dimension of the window's three bonds is drawn from the
  sizes around the MFMA block (16), the K chunk (32) and the workgroup tiles (64, 128):
  1, 2, 15, 16, 17, 31, 32, 33, 63, 64, 65, 127, 128, 129 -- tile tails, single rows and
  columns, K shorter than one chunk, and exact multiples, in every precision, for the
  matvec, both environment updates (random, non-isometric site tensors: the update is a
  plain contraction) and the FP64 Lanczos solve.
* No charge-allowed theta block: an empty problem is planned, applied and updated as a
  no-op, and a Lanczos solve on it is refused with DM_ERR_LAYOUT.
* The largest benchmark window (Ly=10, chi=6000, 150 sectors): the BF16x3 matvec in the
  benchmark's tile shapes and K splits against the full oracle matvec."""
import sys

import numpy as np
import pytest

import workloads
from oracle import blocksparse as bs
from oracle import lanczos as olz
from oracle import mpo as omp
from oracle import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1512_03318_amd as pk  # noqa: E402
from gpu_helpers import max_rel, mpo_site, to_dev  # noqa: E402

EDGE = [1, 2, 15, 16, 17, 31, 32, 33, 63, 64, 65, 127, 128, 129]
PRECS = [(pk.DM_FP64, 1e-12), (pk.DM_FP32, 2e-5), (pk.DM_BF16X3, 1e-4)]
_cache = {}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ragged():
    """Window of the ly4_chi64 workload with its bonds' sector dimensions replaced by
    the edge sizes (cycled, shifted per bond), the oracle's MPO and seeded tensors."""
    if "ragged" not in _cache:
        wl = workloads.preset("ly4_chi64")
        m = omp.build(synth.cylinder_of(wl), wl.basis)
        j, ly = wl.j, wl.ly
        bonds = [{q: EDGE[(i + 3 * k) % len(EDGE)] for i, q in enumerate(sorted(wl.bonds[j + k]))}
                 for k in range(3)]
        rng = np.random.default_rng(7)
        L = workloads.random_env(rng, bonds[0], m.qbond[j], ly, "L")
        R = workloads.random_env(rng, bonds[2], m.qbond[j + 2], ly, "R")
        th = workloads.random_theta(rng, bonds[0], bonds[2], wl.qsite[j], wl.qsite[j + 1], ly)
        A = workloads.random_site(rng, bonds[0], bonds[1], wl.qsite[j], ly)
        B = workloads.random_site(rng, bonds[1], bonds[2], wl.qsite[j + 1], ly)
        keys = bs.theta_keys(bonds[0], bonds[2], wl.qsite[j], wl.qsite[j + 1], ly)
        _cache["ragged"] = dict(wl=wl, m=m, bonds=bonds, L=L, R=R, th=th, A=A, B=B, keys=keys)
    return _cache["ragged"]


def _plan(c, prec):
    wl, m, bonds = c["wl"], c["m"], c["bonds"]
    j, ly = wl.j, wl.ly
    a, cb = pk.Bond(bonds[0]), pk.Bond(bonds[2])
    Lf = to_dev(pk.pack(c["L"], pk.LAYOUT_ENV_L, ly, a, qw=m.qbond[j]))
    Rf = to_dev(pk.pack(c["R"], pk.LAYOUT_ENV_R, ly, cb, qw=m.qbond[j + 2]))
    return pk.HeffPlan(ly, a, cb, mpo_site(m, j), mpo_site(m, j + 1), Lf, Rf, prec)


def _theta_io(c):
    wl, m, bonds = c["wl"], c["m"], c["bonds"]
    j, ly = wl.j, wl.ly
    qs1 = [tuple(q) for q in m.qsite[j]]
    qs2 = [tuple(q) for q in m.qsite[j + 1]]
    a, cb = pk.Bond(bonds[0]), pk.Bond(bonds[2])
    pack = lambda t: pk.pack(t, pk.LAYOUT_THETA, ly, a, cb, qs1=qs1, qs2=qs2)
    unpack = lambda f: pk.unpack(f, pk.LAYOUT_THETA, ly, a, cb, qs1=qs1, qs2=qs2)
    return pack, unpack


def test_ragged_dims_cover_the_edge_sizes():
    c = ragged()
    for b in c["bonds"]:
        assert set(b.values()) == set(EDGE)


@pytest.mark.parametrize("prec,tol", PRECS)
def test_ragged_matvec(prec, tol):
    c = ragged()
    say(f"ragged matvec prec={prec} chi={[sum(b.values()) for b in c['bonds']]}")
    pack, unpack = _theta_io(c)
    plan = _plan(c, prec)
    x = to_dev(pack(c["th"]))
    y = torch.empty_like(x)
    pk.heff_apply(plan, x, y)
    torch.cuda.synchronize()
    m, j = c["m"], c["wl"].j
    ref = bs.heff_apply(c["L"], m.W[j], m.W[j + 1], c["R"], c["th"])
    assert max_rel(unpack(y.cpu().numpy()), ref, c["keys"]) < tol


@pytest.mark.parametrize("prec,tol", PRECS)
def test_ragged_env_updates(prec, tol):
    c = ragged()
    wl, m, bonds = c["wl"], c["m"], c["bonds"]
    j, ly = wl.j, wl.ly
    a, b, cb = (pk.Bond(x) for x in bonds)
    say(f"ragged environment updates prec={prec}")
    for left in (True, False):
        if left:
            env = to_dev(pk.pack(c["L"], pk.LAYOUT_ENV_L, ly, a, qw=m.qbond[j]))
            site = to_dev(pk.pack(c["A"], pk.LAYOUT_SITE, ly, a, b, qs1=[tuple(q) for q in m.qsite[j]]))
            _, n = pk.layout(pk.LAYOUT_ENV_L, ly, b, qw=m.qbond[j + 1])
            out = torch.empty(n, dtype=torch.complex128, device="cuda")
            pk.env_update_left(ly, a, b, mpo_site(m, j), env, site, out, prec)
            got = pk.unpack(out.cpu().numpy(), pk.LAYOUT_ENV_L, ly, b, qw=m.qbond[j + 1])
            ref = bs.env_left_update(c["L"], c["A"], m.W[j])
        else:
            env = to_dev(pk.pack(c["R"], pk.LAYOUT_ENV_R, ly, cb, qw=m.qbond[j + 2]))
            site = to_dev(pk.pack(c["B"], pk.LAYOUT_SITE, ly, b, cb, qs1=[tuple(q) for q in m.qsite[j + 1]]))
            _, n = pk.layout(pk.LAYOUT_ENV_R, ly, b, qw=m.qbond[j + 1])
            out = torch.empty(n, dtype=torch.complex128, device="cuda")
            pk.env_update_right(ly, b, cb, mpo_site(m, j + 1), env, site, out, prec)
            got = pk.unpack(out.cpu().numpy(), pk.LAYOUT_ENV_R, ly, b, qw=m.qbond[j + 1])
            ref = bs.env_right_update(c["R"], c["B"], m.W[j + 1])
        assert set(ref) <= set(got)
        num = max(np.abs(got[k] - ref.get(k, 0)).max() for k in got)
        den = max(np.abs(v).max() for v in ref.values())
        assert num / den < tol, (left, num / den)


def test_ragged_lanczos_fp64():
    c = ragged()
    say("ragged lanczos fp64")
    pack, unpack = _theta_io(c)
    plan = _plan(c, pk.DM_FP64)
    x = to_dev(pack(c["th"]))
    e, k = pk.lanczos_ground(plan, x, 30, 1e-14)
    m, j, keys = c["m"], c["wl"].j, c["keys"]
    mv = lambda v: bs.flatten(bs.heff_apply(c["L"], m.W[j], m.W[j + 1], c["R"], bs.unflatten(v, keys)), keys)
    eo, vo, ko, _, _ = olz.lanczos(mv, bs.flatten(c["th"], keys), max_iter=30)
    assert k == ko
    assert abs(e - eo) <= 1e-10 * abs(eo)
    v = bs.flatten(unpack(x.cpu().numpy()), keys)
    assert 1 - abs(np.vdot(vo, v)) < 1e-8


def test_misaligned_theta_is_refused():
    """Complex FP64 vectors are moved as 16-byte elements: a theta 8 bytes off is refused
    before any work is queued, and the aligned call still works afterwards."""
    c = ragged()
    say("misaligned theta")
    pack, _ = _theta_io(c)
    plan = _plan(c, pk.DM_FP64)
    x = to_dev(pack(c["th"]))
    n = x.numel()
    raw = torch.zeros(2 * n + 2, dtype=torch.float64, device="cuda")
    off = raw[1:1 + 2 * n]  # starts 8 bytes into the allocation
    assert off.data_ptr() % 16 == 8
    off.copy_(torch.view_as_real(x).reshape(-1))
    y = torch.empty_like(x)
    for call in (lambda: pk.heff_apply(plan, off, y), lambda: pk.heff_apply(plan, x, off),
                 lambda: pk.lanczos_ground(plan, off, 30, 1e-14)):
        with pytest.raises(pk.LibraryError) as ei:
            call()
        assert ei.value.code == pk.DM_ERR_ARG
    e, k = pk.lanczos_ground(plan, x, 30, 1e-14)
    assert np.isfinite(e) and k > 0


def test_profile_stride():
    """dm_heff_profile(k) records every k-th matvec; a negative stride is refused."""
    c = ragged()
    say("profile stride")
    pack, _ = _theta_io(c)
    plan = _plan(c, pk.DM_BF16X3)
    x = to_dev(pack(c["th"]))
    y = torch.empty_like(x)
    plan.profile(True, every=4)
    for _ in range(8):
        pk.heff_apply(plan, x, y)
    ms, n = plan.profile_read()
    assert n == 2 and all(t > 0 for t in ms[:3]), (n, ms)
    plan.profile(True, every=1)
    pk.heff_apply(plan, x, y)
    assert plan.profile_read()[1] == 1
    with pytest.raises(pk.LibraryError) as ei:
        plan.profile(True, every=-1)
    assert ei.value.code == pk.DM_ERR_ARG
    plan.profile(False)


def test_window_without_theta_blocks():
    """Bond charges two particles apart cannot be joined by two sites: the theta layout,
    the matvec tables and the middle-bond environments are empty."""
    wl = workloads.preset("ly3_chi16")
    m = omp.build(synth.cylinder_of(wl), wl.basis)
    j, ly = wl.j, wl.ly
    a = pk.Bond({(0, 0): 3, (0, 1): 2})
    cb = pk.Bond({(5, 0): 4})
    b = pk.Bond({(9, 0): 2})
    w1, w2 = mpo_site(m, j), mpo_site(m, j + 1)
    rng = np.random.default_rng(3)
    L = workloads.random_env(rng, {(0, 0): 3, (0, 1): 2}, m.qbond[j], ly, "L")
    R = workloads.random_env(rng, {(5, 0): 4}, m.qbond[j + 2], ly, "R")
    Lf = to_dev(pk.pack(L, pk.LAYOUT_ENV_L, ly, a, qw=m.qbond[j]))
    Rf = to_dev(pk.pack(R, pk.LAYOUT_ENV_R, ly, cb, qw=m.qbond[j + 2]))
    _, n = pk.layout(pk.LAYOUT_THETA, ly, a, cb, qs1=[tuple(q) for q in m.qsite[j]],
                     qs2=[tuple(q) for q in m.qsite[j + 1]])
    assert n == 0
    for prec, _ in PRECS:
        say(f"empty window prec={prec}")
        plan = pk.HeffPlan(ly, a, cb, w1, w2, Lf, Rf, prec)
        assert plan.n == 0 and sum(plan.flops) == 0
        x = torch.zeros(1, dtype=torch.complex128, device="cuda")
        y = torch.full((1,), 7.0, dtype=torch.complex128, device="cuda")
        pk.heff_apply(plan, x, y)
        torch.cuda.synchronize()
        assert complex(y.cpu()[0]) == 7.0  # nothing written
        with pytest.raises(pk.LibraryError) as ei:
            pk.lanczos_ground(plan, x, 30, 1e-14)
        assert ei.value.code == pk.DM_ERR_LAYOUT
        # left update onto a middle bond no site block reaches: empty output, no-op
        _, nA = pk.layout(pk.LAYOUT_SITE, ly, a, b, qs1=[tuple(q) for q in m.qsite[j]])
        _, nL = pk.layout(pk.LAYOUT_ENV_L, ly, b, qw=m.qbond[j + 1])
        assert nA == 0
        site = torch.zeros(1, dtype=torch.complex128, device="cuda")
        out = torch.full((max(nL, 1),), 7.0, dtype=torch.complex128, device="cuda")
        pk.env_update_left(ly, a, b, w1, Lf, site, out, prec)
        torch.cuda.synchronize()
        assert bool((out.cpu() == 0).all()) if nL else complex(out.cpu()[0]) == 7.0


def test_largest_window_bf16x3_matvec():
    """Ly=10, chi=6000: the BF16x3 matvec at the largest benchmark size against the
    oracle's full matvec (seeded Gaussian environments of the exact block structure)."""
    say("building the Ly=10 chi=6000 window with the oracle ...")
    wl = workloads.preset("ly10_chi6000")
    m = omp.build(synth.cylinder_of(wl), wl.basis)
    j, ly = wl.j, wl.ly
    rng = np.random.default_rng(41)
    L = workloads.random_env(rng, wl.bonds[j], m.qbond[j], ly, "L")
    R = workloads.random_env(rng, wl.bonds[j + 2], m.qbond[j + 2], ly, "R")
    th = wl.theta()
    keys = bs.theta_keys(wl.bonds[j], wl.bonds[j + 2], wl.qsite[j], wl.qsite[j + 1], ly)
    a, cb = pk.Bond(wl.bonds[j]), pk.Bond(wl.bonds[j + 2])
    qs1 = [tuple(q) for q in m.qsite[j]]
    qs2 = [tuple(q) for q in m.qsite[j + 1]]
    Lf = to_dev(pk.pack(L, pk.LAYOUT_ENV_L, ly, a, qw=m.qbond[j]))
    Rf = to_dev(pk.pack(R, pk.LAYOUT_ENV_R, ly, cb, qw=m.qbond[j + 2]))
    plan = pk.HeffPlan(ly, a, cb, mpo_site(m, j), mpo_site(m, j + 1), Lf, Rf, pk.DM_BF16X3)
    x = to_dev(pk.pack(th, pk.LAYOUT_THETA, ly, a, cb, qs1=qs1, qs2=qs2))
    y = torch.empty_like(x)
    pk.heff_apply(plan, x, y)
    torch.cuda.synchronize()
    say("oracle matvec ...")
    ref = bs.heff_apply(L, m.W[j], m.W[j + 1], R, th)
    got = pk.unpack(y.cpu().numpy(), pk.LAYOUT_THETA, ly, a, cb, qs1=qs1, qs2=qs2)
    err = max_rel(got, ref, keys)
    say(f"  max relative error {err:.3e}")
    assert err < 1e-4
