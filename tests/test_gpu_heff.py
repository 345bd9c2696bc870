"""GPU parity of the two-site matvec, the environment updates and Lanczos against the
FP64 oracle, on seeded synthetic cylinders (inputs built by the oracle, same on both
sides)."""
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
from gpu_helpers import WindowGPU, block_rel, max_rel, mpo_site, problem, to_dev  # noqa: E402
from helpers import heff_flops  # noqa: E402

CASES = ["ly3_chi16", "ly4_chi64", "ly6_chi200", "ly6_chi800"]
# FP32: 2^-24 per product; BF16x3: three bf16 products per real product, about 2^-17
PRECS = [(pk.DM_FP64, 1e-12), (pk.DM_FP32, 2e-5), (pk.DM_BF16X3, 1e-4)]
# per-block relative error (Frobenius norm of each theta' block): the same rounding,
# measured against each block's own size instead of the largest element
BLOCK_TOL = {pk.DM_FP64: 1e-11, pk.DM_FP32: 2e-4, pk.DM_BF16X3: 1e-3}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("prec,tol", PRECS)
def test_heff_apply_parity(name, prec, tol):
    wl, L, W1, W2, R, th, keys, mpo = problem(name)
    say(f"heff_apply {name} prec={prec} n={sum(m*n for _, (m, n) in keys)}")
    g = WindowGPU(wl, L, R, mpo)
    plan = g.plan(prec)
    x = to_dev(g.pack_theta(th))
    y = torch.empty_like(x)
    pk.heff_apply(plan, x, y)
    torch.cuda.synchronize()
    got = g.unpack_theta(y.cpu().numpy())
    ref = bs.heff_apply(L, W1, W2, R, th)
    err, berr = max_rel(got, ref, keys), block_rel(got, ref, keys)
    say(f"  max relative error {err:.3e}, worst block {berr:.3e}")
    assert err < tol
    assert berr < BLOCK_TOL[prec]


@pytest.mark.parametrize("name", CASES + ["ly8_chi3200"])
def test_plan_flops_equal_the_charge_count(name):
    """The flop counts a plan reports (the numerator of every GFLOP/s figure) equal a
    count written from charges and bond dimensions alone."""
    import workloads
    from oracle import mpo as omp
    from oracle import synth
    wl = workloads.preset(name)
    m = omp.build(synth.cylinder_of(wl), wl.basis)
    j, ly = wl.j, wl.ly
    a, c = pk.Bond(wl.bonds[j]), pk.Bond(wl.bonds[j + 2])
    w1, w2 = mpo_site(m, j), mpo_site(m, j + 1)
    _, nl = pk.layout(pk.LAYOUT_ENV_L, ly, a, qw=m.qbond[j])
    _, nr = pk.layout(pk.LAYOUT_ENV_R, ly, c, qw=m.qbond[j + 2])
    L = torch.zeros(nl, dtype=torch.complex128, device="cuda")
    R = torch.zeros(nr, dtype=torch.complex128, device="cuda")
    qs1 = [tuple(map(int, q)) for q in m.qsite[j]]
    qs2 = [tuple(map(int, q)) for q in m.qsite[j + 1]]
    ref = heff_flops(wl.bonds[j], wl.bonds[j + 2], m.W[j], m.W[j + 1], m.qbond[j], m.qbond[j + 2],
                     qs1, qs2, ly)
    for prec in (pk.DM_FP64, pk.DM_BF16X3):
        plan = pk.HeffPlan(ly, a, c, w1, w2, L, R, prec)
        say(f"plan flops {name} prec={prec}: {plan.flops} vs {ref}")
        assert tuple(plan.flops) == ref


@pytest.mark.parametrize("name", CASES)
def test_lanczos_parity_fp64(name):
    wl, L, W1, W2, R, th, keys, mpo = problem(name)
    say(f"lanczos {name}")
    g = WindowGPU(wl, L, R, mpo)
    plan = g.plan(pk.DM_FP64)
    x = to_dev(g.pack_theta(th))
    e, k = pk.lanczos_ground(plan, x, 30, 1e-14)
    mv = lambda v: bs.flatten(bs.heff_apply(L, W1, W2, R, bs.unflatten(v, keys)), keys)
    eo, vo, ko, _, _ = olz.lanczos(mv, bs.flatten(th, keys), max_iter=30)
    assert k == ko
    assert abs(e - eo) <= 1e-10 * abs(eo)
    v = bs.flatten(g.unpack_theta(x.cpu().numpy()), keys)
    assert 1 - abs(np.vdot(vo, v)) < 1e-8


@pytest.mark.parametrize("max_iter", [8, 17, 25, 48])
def test_lanczos_parity_basis_sizes(max_iter):
    """Krylov bases of every register width of the fused subtraction-projection pass
    (up to 8, 16, 24 and 32 vectors) and one beyond it (unfused passes)."""
    wl, L, W1, W2, R, th, keys, mpo = problem("ly4_chi64")
    say(f"lanczos ly4_chi64 max_iter={max_iter}")
    g = WindowGPU(wl, L, R, mpo)
    plan = g.plan(pk.DM_FP64)
    x = to_dev(g.pack_theta(th))
    e, k = pk.lanczos_ground(plan, x, max_iter, 1e-14)
    mv = lambda v: bs.flatten(bs.heff_apply(L, W1, W2, R, bs.unflatten(v, keys)), keys)
    eo, vo, ko, _, _ = olz.lanczos(mv, bs.flatten(th, keys), max_iter=max_iter)
    assert k == ko
    assert abs(e - eo) <= 1e-10 * abs(eo)
    v = bs.flatten(g.unpack_theta(x.cpu().numpy()), keys)
    assert 1 - abs(np.vdot(vo, v)) < 1e-8


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("prec,tol", PRECS)
def test_env_updates_parity(name, prec, tol):
    wl, L, W1, W2, R, th, keys, mpo = problem(name)
    j, ly = wl.j, wl.ly
    say(f"env updates {name} prec={prec}")
    # left: L at bond j -> bond j+1 with a fresh left isometry on site j
    rng = np.random.default_rng(99)
    A = workloads.left_isometry(rng, wl.bonds[j], wl.bonds[j + 1], wl.qsite[j], ly)
    a, b = pk.Bond(wl.bonds[j]), pk.Bond(wl.bonds[j + 1])
    W = mpo_site(mpo, j)
    Lf = to_dev(pk.pack(L, pk.LAYOUT_ENV_L, ly, a, qw=mpo.qbond[j]))
    Af = to_dev(pk.pack(A, pk.LAYOUT_SITE, ly, a, b, qs1=[tuple(q) for q in mpo.qsite[j]]))
    _, nout = pk.layout(pk.LAYOUT_ENV_L, ly, b, qw=mpo.qbond[j + 1])
    Lo = torch.empty(nout, dtype=torch.complex128, device="cuda")
    pk.env_update_left(ly, a, b, W, Lf, Af, Lo, prec)
    got = pk.unpack(Lo.cpu().numpy(), pk.LAYOUT_ENV_L, ly, b, qw=mpo.qbond[j + 1])
    ref = bs.env_left_update(L, A, mpo.W[j])
    num = max(np.abs(got[k] - ref.get(k, 0)).max() for k in got)
    den = max(np.abs(v).max() for v in ref.values())
    assert set(ref) <= set(got)
    assert num / den < tol
    # right: R at bond j+2 -> bond j+1 with a fresh right isometry on site j+1
    B = workloads.right_isometry(rng, wl.bonds[j + 1], wl.bonds[j + 2], wl.qsite[j + 1], ly)
    b, c = pk.Bond(wl.bonds[j + 1]), pk.Bond(wl.bonds[j + 2])
    W = mpo_site(mpo, j + 1)
    Rf = to_dev(pk.pack(R, pk.LAYOUT_ENV_R, ly, c, qw=mpo.qbond[j + 2]))
    Bf = to_dev(pk.pack(B, pk.LAYOUT_SITE, ly, b, c, qs1=[tuple(q) for q in mpo.qsite[j + 1]]))
    _, nout = pk.layout(pk.LAYOUT_ENV_R, ly, b, qw=mpo.qbond[j + 1])
    Ro = torch.empty(nout, dtype=torch.complex128, device="cuda")
    pk.env_update_right(ly, b, c, W, Rf, Bf, Ro, prec)
    got = pk.unpack(Ro.cpu().numpy(), pk.LAYOUT_ENV_R, ly, b, qw=mpo.qbond[j + 1])
    ref = bs.env_right_update(R, B, mpo.W[j + 1])
    num = max(np.abs(got[k] - ref.get(k, 0)).max() for k in got)
    den = max(np.abs(v).max() for v in ref.values())
    assert set(ref) <= set(got)
    assert num / den < tol


def test_lanczos_graph_replays_equal_eager():
    """Each Lanczos step is one HIP graph replay; replays (several calls, with eager work
    and synchronisation in between) must give exactly the eager result."""
    import os
    wl, L, W1, W2, R, th, keys, mpo = problem("ly6_chi200")
    say("lanczos graph vs eager")
    g = WindowGPU(wl, L, R, mpo)
    eager = g.plan(pk.DM_FP64)
    os.environ["MRDMRG_GRAPH"] = "1"
    try:
        graphed = g.plan(pk.DM_FP64)
    finally:
        os.environ.pop("MRDMRG_GRAPH")
    x0 = to_dev(g.pack_theta(th))
    xe = x0.clone()
    ee, ke = pk.lanczos_ground(eager, xe, 30, 1e-14)
    for rep in range(3):
        xg = x0.clone()
        eg, kg = pk.lanczos_ground(graphed, xg, 30, 1e-14)
        y = torch.empty_like(x0)
        pk.heff_apply(graphed, x0, y)          # eager work between replays
        torch.cuda.synchronize()
        assert kg == ke and eg == ee, (rep, eg, ee)
        assert torch.equal(xg, xe)


def test_lanczos_breakdown_on_exact_eigenvector():
    """A start vector in a one-dimensional invariant subspace stops after one step."""
    wl, L, W1, W2, R, th, keys, mpo = problem("ly3_chi16")
    g = WindowGPU(wl, L, R, mpo)
    plan = g.plan(pk.DM_FP64)
    mv = lambda v: bs.flatten(bs.heff_apply(L, W1, W2, R, bs.unflatten(v, keys)), keys)
    dim = sum(m * n for _, (m, n) in keys)
    H = np.array([mv(np.eye(dim)[i]) for i in range(dim)]).T
    lam, vec = np.linalg.eigh((H + H.conj().T) / 2)
    x = to_dev(g.pack_theta(bs.unflatten(vec[:, 0].copy(), keys)))
    e, k = pk.lanczos_ground(plan, x, 30, 1e-10)
    assert k == 1
    assert abs(e - lam[0]) < 1e-10 * max(1, abs(lam[0]))
