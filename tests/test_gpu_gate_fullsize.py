"""The precision gate at the benchmark's window, against the FP64 CPU oracle.

Window: Ly=8, chi=3200 centre bond (orbitals 127/128 of an 8 x 32 cylinder, flux 1/8,
t = V = 1, 104 sectors).  The oracle contracts the environments from the workload's
seeded isometries with its own MPO (H_eff is then the Hamiltonian projected on the
window's basis, Hermitian) and converges the lowest eigenpair (E_gs, theta_gs) of H_eff
with restarted FP64 Lanczos to |H v - E v| <= 1e-10 |H|.  The library gets the same L,
W1, W2, R, and runs at most 30 Lanczos steps in each precision from theta_gs plus
seeded complex Gaussian noise of relative size 1e-3, normalised (the warm start a DMRG
sweep gives), with the Krylov basis, reorthogonalisation, tridiagonal problem and the
final Rayleigh quotient in FP64.  Gate:
    |E - E_gs| / |E_gs| <= 1e-9   and   1 - |<theta_gs|theta>| <= 1e-6,
with a 10x margin for the FP64 path.  The oracle part takes a few minutes of host time
(two environment sweeps over 127 sites each, then a few hundred oracle matvecs)."""
import sys
import time

import numpy as np
import pytest

import workloads
from oracle import blocksparse as bs
from oracle import lanczos as olz
from oracle import mpo as omp
from oracle import synth

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1800)]

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1512_03318_amd as pk  # noqa: E402
from gpu_helpers import WindowGPU, to_dev  # noqa: E402

NOISE = 1e-3
GATE_E, GATE_OV = 1e-9, 1e-6
_case = {}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def case():
    if _case:
        return _case
    t0 = time.perf_counter()
    wl = workloads.preset("ly8_chi3200")
    say("oracle: MPO of the 8 x 32 cylinder ...")
    m = omp.build(synth.cylinder_of(wl), wl.basis)
    j = wl.j
    L = bs.left_boundary()
    for i in range(j):
        L = bs.env_left_update(L, wl.site_tensor(i), m.W[i])
        if i % 16 == 15:
            say(f"oracle: left environment {i + 1}/{j} sites ({time.perf_counter() - t0:.0f} s)")
    R = bs.right_boundary((wl.N_tot, wl.K_tot))
    for q, i in enumerate(range(wl.n - 1, j + 1, -1)):
        R = bs.env_right_update(R, wl.site_tensor(i), m.W[i])
        if q % 16 == 15:
            say(f"oracle: right environment {q + 1}/{wl.n - j - 2} sites ({time.perf_counter() - t0:.0f} s)")
    keys = bs.theta_keys(wl.bonds[j], wl.bonds[j + 2], wl.qsite[j], wl.qsite[j + 1], wl.ly)
    nmv = [0]

    def mv(v):
        nmv[0] += 1
        if nmv[0] % 25 == 0:
            say(f"oracle: {nmv[0]} matvecs of the ground-state solve ({time.perf_counter() - t0:.0f} s)")
        return bs.flatten(bs.heff_apply(L, m.W[j], m.W[j + 1], R, bs.unflatten(v, keys)), keys)

    e_gs, v_gs, res, n = olz.ground_state(mv, bs.flatten(wl.theta(), keys), tol_res=1e-10)
    say(f"oracle: E_gs = {e_gs:.15f}, residual {res:.2e}, {n} matvecs, {time.perf_counter() - t0:.0f} s")
    _case.update(wl=wl, keys=keys, e_gs=e_gs, v_gs=v_gs, g=WindowGPU(wl, L, R, m))
    return _case


@pytest.mark.parametrize("prec", [pk.DM_FP64, pk.DM_FP32, pk.DM_BF16X3])
def test_fullsize_warm_start_gate_against_the_oracle(prec):
    c = case()
    say(f"P2 gate ly8_chi3200 prec={prec}")
    v_gs, e_gs, keys, g = c["v_gs"], c["e_gs"], c["keys"], c["g"]
    rng = np.random.default_rng(2024)
    noise = rng.standard_normal(v_gs.size) + 1j * rng.standard_normal(v_gs.size)
    th0 = v_gs + NOISE * noise / np.linalg.norm(noise)
    th0 /= np.linalg.norm(th0)
    plan = g.plan(prec)
    x = to_dev(g.pack_theta(bs.unflatten(th0, keys)))
    e, k = pk.lanczos_ground(plan, x, 30, 1e-14)
    v = bs.flatten(g.unpack_theta(x.cpu().numpy()), keys)
    v /= np.linalg.norm(v)
    de = abs(e - e_gs) / abs(e_gs)
    ov = 1 - abs(np.vdot(v_gs, v))
    say(f"  steps={k} E={e:.15f} dE/E={de:.3e} 1-overlap={ov:.3e}")
    margin = 10.0 if prec == pk.DM_FP64 else 1.0
    assert de <= GATE_E / margin
    assert ov <= GATE_OV / margin
