"""The real formulation of the mixed basis (eq. rot, Sec. IV D) on the GPU.

The MPO is the oracle's eq. rot form (real entries), the isometries and theta are real,
so the environments are real; the plans take DM_FP64 / DM_FP32 / DM_BF16X3 with DM_REAL and
float64 buffers in the usual block layouts.  Checked against the FP64 oracle:

* one matvec per precision, small to Ly=6 chi=800, and at the Ly=8 chi=3200 centre window
  (seeded real environments of the exact block structure), element and block errors;
* the flop counts are a quarter of the complex plan's (2 per real multiply-add);
* FP64 Lanczos against the oracle's Lanczos (same step count, energy, Ritz vector),
  including a theta of odd length (its last complex pair is half padding);
* the real plan and the complex plan on the same (real) data give the same solve;
* both environment updates in every precision;
* the P2 warm-start gate in FP32 and BF16x3 against the oracle's ground state (Ly=6
  chi=800).
"""
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
from gpu_helpers import WindowGPU, block_rel, max_rel, mpo_site, to_dev  # noqa: E402

TOL = {pk.DM_FP64: 1e-12, pk.DM_FP32: 2e-5, pk.DM_BF16X3: 1e-4}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


_probs = {}


def real_problem(name):
    """(wl, L, W1, W2, R, theta, keys, mpo) of a preset window in the real formulation."""
    if name not in _probs:
        wl = workloads.preset(name, real=True)
        _probs[name] = (wl,) + tuple(synth.window_problem(wl))
    return _probs[name]


def real_dev(flat):
    """A packed complex layout with zero imaginary parts -> float64 on the device."""
    assert np.abs(flat.imag).max() == 0
    return to_dev(np.ascontiguousarray(flat.real))


def cplx(t):
    return t.cpu().numpy().astype(np.complex128)


def real_plan(g, prec):
    return pk.HeffPlan(g.ly, g.a, g.c, g.w1, g.w2, real_dev(g.Lf), real_dev(g.Rf), prec | pk.DM_REAL)


@pytest.mark.parametrize("prec", [pk.DM_FP64, pk.DM_FP32, pk.DM_BF16X3])
@pytest.mark.parametrize("name", ["ly3_chi16", "ly4_chi64", "ly6_chi200", "ly6_chi800"])
def test_real_heff_apply_parity(name, prec):
    wl, L, W1, W2, R, th, keys, mpo = real_problem(name)
    g = WindowGPU(wl, L, R, mpo)
    plan = real_plan(g, prec)
    x = real_dev(g.pack_theta(th))
    y = torch.empty_like(x)
    say(f"real heff_apply {name} prec={prec} n={x.numel()}")
    pk.heff_apply(plan, x, y)
    got = g.unpack_theta(cplx(y))
    ref = bs.heff_apply(L, W1, W2, R, th)
    err, berr = max_rel(got, ref, keys), block_rel(got, ref, keys)
    say(f"  max relative error {err:.3e}, worst block {berr:.3e}")
    assert err <= TOL[prec]
    # a quarter of the complex plan's flops (2 per real multiply-add instead of 8)
    cp = g.plan(prec)
    assert all(abs(r * 4 - c) <= 1e-9 * c for r, c in zip(plan.flops, cp.flops))


@pytest.mark.parametrize("name", ["ly3_chi16", "ly4_chi64", "ly6_chi200"])
def test_real_lanczos_parity_fp64(name):
    wl, L, W1, W2, R, th, keys, mpo = real_problem(name)
    g = WindowGPU(wl, L, R, mpo)
    plan = real_plan(g, pk.DM_FP64)
    x = real_dev(g.pack_theta(th))
    say(f"real lanczos {name} n={x.numel()} (odd: {x.numel() % 2 == 1})")
    e, k = pk.lanczos_ground(plan, x, 30, 1e-14)
    mv = lambda v: bs.flatten(bs.heff_apply(L, W1, W2, R, bs.unflatten(v, keys)), keys)
    eo, vo, ko, _, _ = olz.lanczos(mv, bs.flatten(th, keys), max_iter=30)
    say(f"  steps {k} (oracle {ko}), energy {e:.14f} (oracle {eo:.14f})")
    assert k == ko
    assert abs(e - eo) <= 1e-10 * abs(eo)
    v = bs.flatten(g.unpack_theta(cplx(x)), keys)
    assert 1 - abs(np.vdot(vo, v)) < 1e-8


def test_real_and_complex_plans_agree():
    """The same real window through the real plan and through the complex plan (its data
    stored as complex with zero imaginary parts): the same solve up to rounding."""
    wl, L, W1, W2, R, th, keys, mpo = real_problem("ly6_chi200")
    g = WindowGPU(wl, L, R, mpo)
    xr = real_dev(g.pack_theta(th))
    xc = to_dev(g.pack_theta(th))
    er, kr = pk.lanczos_ground(real_plan(g, pk.DM_FP64), xr, 30, 1e-14)
    ec, kc = pk.lanczos_ground(g.plan(pk.DM_FP64), xc, 30, 1e-14)
    say(f"real {er:.14f} ({kr} steps), complex {ec:.14f} ({kc} steps)")
    assert kr == kc
    assert abs(er - ec) <= 1e-12 * abs(ec)
    vc = xc.cpu().numpy()
    assert np.abs(vc.imag).max() <= 1e-12
    assert np.abs(vc.real - xr.cpu().numpy()).max() <= 1e-9


@pytest.mark.parametrize("prec", [pk.DM_FP64, pk.DM_FP32, pk.DM_BF16X3])
def test_real_env_updates(prec):
    wl, L, W1, W2, R, th, keys, mpo = real_problem("ly6_chi200")
    j, ly = wl.j, wl.ly
    rng = np.random.default_rng(41)
    A = workloads.left_isometry(rng, wl.bonds[j], wl.bonds[j + 1], wl.qsite[j], ly, real=True)
    B = workloads.right_isometry(rng, wl.bonds[j + 1], wl.bonds[j + 2], wl.qsite[j + 1], ly, real=True)
    a, b, c = (pk.Bond(wl.bonds[i]) for i in (j, j + 1, j + 2))
    w1, w2 = mpo_site(mpo, j), mpo_site(mpo, j + 1)
    qs1, qs2 = [tuple(q) for q in mpo.qsite[j]], [tuple(q) for q in mpo.qsite[j + 1]]
    say(f"real environment updates prec={prec}")
    Lf = real_dev(pk.pack(L, pk.LAYOUT_ENV_L, ly, a, qw=mpo.qbond[j]))
    Af = real_dev(pk.pack(A, pk.LAYOUT_SITE, ly, a, b, qs1=qs1))
    _, nl = pk.layout(pk.LAYOUT_ENV_L, ly, b, qw=mpo.qbond[j + 1])
    Lo = torch.empty(nl, dtype=torch.float64, device="cuda")
    pk.env_update_left(ly, a, b, w1, Lf, Af, Lo, prec | pk.DM_REAL)
    ref = bs.env_left_update(L, A, W1)
    got = pk.unpack(cplx(Lo), pk.LAYOUT_ENV_L, ly, b, qw=mpo.qbond[j + 1])
    kl = [(k, None) for k in ref]
    errl = max_rel(got, ref, kl)
    Rf = real_dev(pk.pack(R, pk.LAYOUT_ENV_R, ly, c, qw=mpo.qbond[j + 2]))
    Bf = real_dev(pk.pack(B, pk.LAYOUT_SITE, ly, b, c, qs1=qs2))
    _, nr = pk.layout(pk.LAYOUT_ENV_R, ly, b, qw=mpo.qbond[j + 1])
    Ro = torch.empty(nr, dtype=torch.float64, device="cuda")
    pk.env_update_right(ly, b, c, w2, Rf, Bf, Ro, prec | pk.DM_REAL)
    refr = bs.env_right_update(R, B, W2)
    gotr = pk.unpack(cplx(Ro), pk.LAYOUT_ENV_R, ly, b, qw=mpo.qbond[j + 1])
    errr = max_rel(gotr, refr, [(k, None) for k in refr])
    say(f"  left {errl:.3e}, right {errr:.3e}")
    assert errl <= TOL[prec] and errr <= TOL[prec]


def test_real_plan_rejects_complex_mpo():
    cwl = workloads.preset("ly3_chi16")
    m = omp.build(synth.cylinder_of(cwl), "mixed")  # complex phases
    j = cwl.j
    a, c = pk.Bond(cwl.bonds[j]), pk.Bond(cwl.bonds[j + 2])
    _, nl = pk.layout(pk.LAYOUT_ENV_L, cwl.ly, a, qw=m.qbond[j])
    _, nr = pk.layout(pk.LAYOUT_ENV_R, cwl.ly, c, qw=m.qbond[j + 2])
    Lz = torch.zeros(nl, dtype=torch.float64, device="cuda")
    Rz = torch.zeros(nr, dtype=torch.float64, device="cuda")
    with pytest.raises(pk.LibraryError):
        pk.HeffPlan(cwl.ly, a, c, mpo_site(m, j), mpo_site(m, j + 1), Lz, Rz, pk.DM_FP64 | pk.DM_REAL)


def test_real_fullsize_matvec():
    """Ly=8 chi=3200 centre window in the real formulation: seeded real environments of
    the exact block structure, FP64 and FP32 matvecs against the oracle."""
    say("building the real Ly=8 chi=3200 window with the oracle ...")
    wl = workloads.preset("ly8_chi3200", real=True)
    m = omp.build(synth.cylinder_of(wl), "mixed", real=True)
    j, ly = wl.j, wl.ly
    rng = np.random.default_rng(37)
    L = workloads.random_env(rng, wl.bonds[j], m.qbond[j], ly, "L", real=True)
    R = workloads.random_env(rng, wl.bonds[j + 2], m.qbond[j + 2], ly, "R", real=True)
    th = wl.theta()
    keys = bs.theta_keys(wl.bonds[j], wl.bonds[j + 2], wl.qsite[j], wl.qsite[j + 1], ly)
    say("  oracle matvec ...")
    ref = bs.heff_apply(L, m.W[j], m.W[j + 1], R, th)
    say("  uploading the window ...")
    g = WindowGPU(wl, L, R, m)
    x = real_dev(g.pack_theta(th))
    for prec in (pk.DM_FP64, pk.DM_FP32, pk.DM_BF16X3):
        plan = real_plan(g, prec)
        y = torch.empty_like(x)
        pk.heff_apply(plan, x, y)
        got = g.unpack_theta(cplx(y))
        err, berr = max_rel(got, ref, keys), block_rel(got, ref, keys)
        say(f"  prec={prec}: max relative error {err:.3e}, worst block {berr:.3e}")
        assert err <= TOL[prec]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", [pk.DM_FP32, pk.DM_BF16X3])
def test_real_warm_start_gate(prec):
    """P2 gate in FP32 and BF16x3 on the real formulation: the oracle's ground state of
    the Ly=6 chi=800 window, start theta_gs + 1e-3 noise, 30 GPU steps; |dE/E| <= 1e-9
    and 1 - |<gs|theta>| <= 1e-6 (the energy is the FP64 Rayleigh quotient)."""
    wl, L, W1, W2, R, th, keys, mpo = real_problem("ly6_chi800")
    g = WindowGPU(wl, L, R, mpo)
    mv = lambda v: bs.flatten(bs.heff_apply(L, W1, W2, R, bs.unflatten(v, keys)), keys)
    if "gs" not in _probs:
        say("oracle ground state of the real Ly=6 chi=800 window ...")
        _probs["gs"] = olz.ground_state(mv, bs.flatten(th, keys), tol_res=1e-10)
    egs, vgs, *_ = _probs["gs"]
    vgs = vgs * np.exp(-1j * np.angle(vgs[np.argmax(np.abs(vgs))]))  # real up to rounding
    rng = np.random.default_rng(5)
    noise = rng.standard_normal(vgs.shape)
    x0 = vgs.real + 1e-3 * noise / np.linalg.norm(noise)  # relative noise 1e-3, as in the complex gate
    x0 /= np.linalg.norm(x0)
    x = real_dev(g.pack_theta(bs.unflatten(x0 + 0j, keys)))
    e, k = pk.lanczos_ground(real_plan(g, prec), x, 30, 1e-14)
    v = bs.flatten(g.unpack_theta(cplx(x)), keys)
    de, ov = abs(e - egs) / abs(egs), 1 - abs(np.vdot(vgs, v)) / np.linalg.norm(v)
    say(f"  prec={prec} steps={k} dE/E={de:.3e} 1-overlap={ov:.3e}")
    assert de <= 1e-9 and ov <= 1e-6
