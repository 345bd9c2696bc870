"""Infinite-cylinder DMRG by unit-cell growth on the GPU (dm_idmrg) against the oracle.

* Ly=3, flux 1/3, V=1, three-ring cells (9 orbitals), three particles per cell: from the
  same seeded start (one-cell random blocks, two random right-canonical cells) the GPU's
  total energies E_j equal the oracle's iDMRG iteration by iteration, and the Schmidt
  values between the last two cells agree sector by sector.
  With one particle of momentum 1 added per cell (two cells carry k = 2), the growth
  moves every charge by (6, 2), which reorders sectors: the same comparison then checks
  the panel permutation of the moved site tensors and environment.
* The same cylinder in the real form of eq. rot (the rotated bulk cell, real isometries):
  the eigensolves run DM_REAL plans on the real parts, and the energies equal the oracle's
  iDMRG on the same real cell.
* The same cylinder at V=0: the energy added per iteration, per orbital, reaches the
  free-fermion Bloch-band value (closed form).
* The model of Fig. 3 (Ly=10, flux 1/3, V/t=0.1, the lowest band filled: ten particles
  per three-ring cell of 30 orbitals) in the mixed basis (complex and the real form of
  eq. rot) and in the real-space basis: time per growth iteration, energy per orbital and
  centre entropy (printed; asserted: every energy per orbital lies above the V=0 Bloch
  value, and the mixed basis converges).
"""
import time
import sys
from fractions import Fraction

import numpy as np
import pytest

import workloads
from oracle import free, idmrg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1512_03318_amd as pk  # noqa: E402
from gpu_helpers import to_dev  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_start(cell, gs):
    """The growth start on the device: the two cells as a library MPS, the cell's MPO
    sites and the two block environments (contracted by the oracle)."""
    ly, n = gs.ly, gs.n
    qs = [[tuple(map(int, q)) for q in cell.qsite[i % n]] for i in range(2 * n)]
    bonds = gs.bonds[n:3 * n + 1]
    B = [pk.Bond(b) for b in bonds]
    tens = [to_dev(pk.pack(gs.cells[i], pk.LAYOUT_SITE, ly, B[i], B[i + 1], qs1=qs[i])) for i in range(2 * n)]
    psi = pk.MPS(ly, bonds, qs, tens)
    sites = [pk.MpoSite(cell.W[i], cell.qbond[i], cell.qbond[i + 1], cell.qsite[i]) for i in range(n)]
    L0, R0 = idmrg.block_envs(cell, gs.left, gs.right, next(iter(gs.bonds[-1])))
    l0 = to_dev(pk.pack(L0, pk.LAYOUT_ENV_L, ly, B[0], qw=cell.qbond[0]))
    r0 = to_dev(pk.pack(R0, pk.LAYOUT_ENV_R, ly, B[-1], qw=cell.qbond[0]))
    return psi, sites, (L0, R0), (l0, r0)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("K_cell", [0, 1])
def test_gpu_idmrg_equals_the_oracle(K_cell):
    cell = idmrg.bulk_cell(3, Fraction(1, 3), 1.0, 1.0, 3)
    gs = workloads.growth_start(3, 3, 3, K_cell, 32, 17)
    n, chi, iters = gs.n, 32, 4
    say(f"iDMRG Ly=3 flux 1/3 V=1, {n}-orbital cell (D {cell.W[0].shape[0]}), two cells' charge {gs.d}, "
        f"chi={chi}, {iters} iterations")
    psi, sites, (L0, R0), (l0, r0) = gpu_start(cell, gs)
    e = pk.idmrg(psi, sites, gs.d, l0, r0, iters, chi)
    r = idmrg.run(cell, gs.cells, gs.bonds[n:3 * n + 1], iters, chi, L0, R0, gs.d)
    say(f"  GPU    {['%.12f' % x for x in e]}")
    say(f"  oracle {['%.12f' % x for x in r.energies]}")
    for j in range(iters):
        assert abs(e[j] - r.energies[j]) <= 1e-9 * abs(r.energies[j]), j
    bond = psi.bond(n)
    want = r.schmidt[-1]
    assert bond == {q: len(v) for q, v in sorted(want.items())}
    lam = psi.schmidt(n)
    pos = 0
    for q in sorted(bond):
        assert np.abs(lam[pos:pos + bond[q]] - want[q]).max() <= 1e-8, q
        pos += bond[q]
    ent, _ = pk.entanglement(lam)
    say(f"  centre bond: {len(bond)} sectors, {sum(bond.values())} states, entropy {ent:.10f}")


@pytest.mark.timeout(900)
def test_gpu_idmrg_real_form_equals_the_oracle():
    cell = idmrg.bulk_cell(3, Fraction(1, 3), 1.0, 1.0, 3, real=True)
    gs = workloads.growth_start(3, 3, 3, 0, 32, 19, real=True)
    n, chi, iters = gs.n, 32, 4
    say(f"iDMRG, eq. rot form: Ly=3 flux 1/3 V=1, chi={chi}, {iters} iterations, DM_REAL eigensolves")
    psi, sites, (L0, R0), (l0, r0) = gpu_start(cell, gs)
    e = pk.idmrg(psi, sites, gs.d, l0, r0, iters, chi, prec=pk.DM_FP64 | pk.DM_REAL)
    r = idmrg.run(cell, gs.cells, gs.bonds[n:3 * n + 1], iters, chi, L0, R0, gs.d)
    say(f"  GPU    {['%.12f' % x for x in e]}")
    say(f"  oracle {['%.12f' % x for x in r.energies]}")
    for j in range(iters):
        assert abs(e[j] - r.energies[j]) <= 1e-9 * abs(r.energies[j]), j
    lam = psi.schmidt(n)
    want = np.concatenate([r.schmidt[-1][q] for q in sorted(r.schmidt[-1])])
    assert np.abs(lam - want).max() <= 1e-8
    # the state stays real: the centre site tensor has zero imaginary parts
    assert torch.abs(psi.tensor(n).imag).max().item() == 0.0


@pytest.mark.timeout(900)
def test_gpu_idmrg_free_fermions_reach_the_bulk_energy():
    cell = idmrg.bulk_cell(3, Fraction(1, 3), 1.0, 0.0, 3)
    gs = workloads.growth_start(3, 3, 3, 0, 64, 7)
    psi, sites, _, (l0, r0) = gpu_start(cell, gs)
    e = pk.idmrg(psi, sites, gs.d, l0, r0, 6, 64)
    per = idmrg.energy_per_orbital(e, gs.n)
    exact = free.bulk_energy_per_orbital(3, 1, 3)
    say(f"iDMRG V=0: energy per orbital {['%.9f' % x for x in per]}, Bloch bands {exact:.9f}")
    assert abs(per[-1] - exact) < 5e-5


def gpu_block_envs(cell, gs, sites):
    """L0 and R0 contracted on the device (env_update_left / _right) from the boundary
    states R and F through the growth start's random one-cell blocks."""
    ly, n = gs.ly, gs.n
    B = [pk.Bond(b) for b in gs.bonds]
    qs = [[tuple(map(int, q)) for q in cell.qsite[i]] for i in range(n)]
    one = np.ones((1, 1), dtype=np.complex128)
    L = to_dev(pk.pack({((0, 0), cell.r, (0, 0)): one}, pk.LAYOUT_ENV_L, ly, B[0], qw=cell.qbond[0]))
    for i in range(n):
        A = to_dev(pk.pack(gs.left[i], pk.LAYOUT_SITE, ly, B[i], B[i + 1], qs1=qs[i]))
        out = torch.zeros(pk.layout(pk.LAYOUT_ENV_L, ly, B[i + 1], qw=cell.qbond[i + 1])[1],
                          dtype=torch.complex128, device="cuda")
        pk.env_update_left(ly, B[i], B[i + 1], sites[i], L, A, out)
        L = out
    q = next(iter(gs.bonds[-1]))
    R = to_dev(pk.pack({(q, cell.f, q): one}, pk.LAYOUT_ENV_R, ly, B[4 * n], qw=cell.qbond[0]))
    for i in range(n - 1, -1, -1):
        j = 3 * n + i
        Bt = to_dev(pk.pack(gs.right[i], pk.LAYOUT_SITE, ly, B[j], B[j + 1], qs1=qs[i]))
        out = torch.zeros(pk.layout(pk.LAYOUT_ENV_R, ly, B[j], qw=cell.qbond[i])[1],
                          dtype=torch.complex128, device="cuda")
        pk.env_update_right(ly, B[j], B[j + 1], sites[i], R, Bt, out)
        R = out
    return L, R


@pytest.mark.timeout(900)
def test_gpu_idmrg_fig3_model():
    """Fig. 3's cylinder: Ly=10, flux 1/3, V/t=0.1, 1/3 filling, three-ring cells."""
    Ly = 10
    runs = {"mixed": [(100, 8), (200, 8), (400, 8)], "mixed_eq_rot": [(100, 8), (200, 8), (400, 8)],
            "real": [(100, 3), (200, 3)]}
    e0 = free.bulk_energy_per_orbital(Ly, 1, 3)
    res = {}
    for name, plan in runs.items():
        basis, rot = ("mixed", True) if name == "mixed_eq_rot" else (name, False)
        t0 = time.perf_counter()
        cell = idmrg.bulk_cell(Ly, Fraction(1, 3), 1.0, 0.1, 3, basis=basis, real=rot)
        say(f"{name}: bulk cell of {cell.n_sites} orbitals, D {min(w.shape[0] for w in cell.W)}.."
            f"{max(w.shape[0] for w in cell.W)} ({time.perf_counter() - t0:.1f} s on the host)")
        for chi, iters in plan:
            gs = workloads.growth_start(Ly, 3, Ly, (Ly * (Ly - 1) // 2) % Ly, chi, 30 + chi, basis=basis,
                                        real=rot)
            n = gs.n
            qs = [[tuple(map(int, q)) for q in cell.qsite[i % n]] for i in range(2 * n)]
            bonds = gs.bonds[n:3 * n + 1]
            Bd = [pk.Bond(b) for b in bonds]
            tens = [to_dev(pk.pack(gs.cells[i], pk.LAYOUT_SITE, gs.ly, Bd[i], Bd[i + 1], qs1=qs[i]))
                    for i in range(2 * n)]
            psi = pk.MPS(gs.ly, bonds, qs, tens)
            sites = [pk.MpoSite(cell.W[i], cell.qbond[i], cell.qbond[i + 1], cell.qsite[i]) for i in range(n)]
            l0, r0 = gpu_block_envs(cell, gs, sites)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            e = pk.idmrg(psi, sites, gs.d, l0, r0, iters, chi, prec=pk.DM_FP64 | (pk.DM_REAL if rot else 0))
            dt = (time.perf_counter() - t1) / iters
            per = idmrg.energy_per_orbital(e, n)
            lam = psi.schmidt(n)
            ent, _ = pk.entanglement(lam[lam > 0])
            res[(name, chi)] = (per, dt)
            say(f"  chi={chi}: {dt:.2f} s per growth iteration ({iters}), energy per orbital "
                f"{['%.6f' % x for x in per]}, centre entropy {ent:.6f}, {len(psi.bond(n))} sectors")
            assert all(x > e0 for x in per)  # V n n >= 0: above the V=0 Bloch-band energy
    for chi in (100, 200):
        say(f"chi={chi}: real-space / mixed time per growth iteration "
            f"{res[('real', chi)][1] / res[('mixed', chi)][1]:.1f}x")
    for chi in (100, 200, 400):
        say(f"chi={chi}: mixed complex / eq. rot time per growth iteration "
            f"{res[('mixed', chi)][1] / res[('mixed_eq_rot', chi)][1]:.2f}x")
    per = res[("mixed", 400)][0]
    say(f"mixed chi=400: last two estimates {per[-2]:.6f}, {per[-1]:.6f} (V=0 Bloch value {e0:.6f})")
    assert abs(per[-1] - per[-2]) < 2e-3


_cells = {}


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name,chi,iters", [("mixed", 800, 4), ("mixed_eq_rot", 800, 4),
                                            ("mixed", 1600, 3), ("mixed_eq_rot", 1600, 3)])
def test_gpu_idmrg_fig3_large_chi(name, chi, iters):
    """The Fig. 3 cylinder's growth at chi = 800 and 1600 in the mixed basis, complex and in
    the real form of eq. rot: the centre bond reaches chi, its Schmidt values are
    normalised, and every energy per orbital lies above the V = 0 Bloch-band value."""
    Ly, rot = 10, name == "mixed_eq_rot"
    if rot not in _cells:
        _cells[rot] = idmrg.bulk_cell(Ly, Fraction(1, 3), 1.0, 0.1, 3, basis="mixed", real=rot)
    cell = _cells[rot]
    gs = workloads.growth_start(Ly, 3, Ly, (Ly * (Ly - 1) // 2) % Ly, chi, 30 + chi, real=rot)
    n = gs.n
    qs = [[tuple(map(int, q)) for q in cell.qsite[i % n]] for i in range(2 * n)]
    bonds = gs.bonds[n:3 * n + 1]
    Bd = [pk.Bond(b) for b in bonds]
    tens = [to_dev(pk.pack(gs.cells[i], pk.LAYOUT_SITE, gs.ly, Bd[i], Bd[i + 1], qs1=qs[i]))
            for i in range(2 * n)]
    psi = pk.MPS(gs.ly, bonds, qs, tens)
    sites = [pk.MpoSite(cell.W[i], cell.qbond[i], cell.qbond[i + 1], cell.qsite[i]) for i in range(n)]
    l0, r0 = gpu_block_envs(cell, gs, sites)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    e = pk.idmrg(psi, sites, gs.d, l0, r0, iters, chi, prec=pk.DM_FP64 | (pk.DM_REAL if rot else 0))
    dt = (time.perf_counter() - t1) / iters
    per = idmrg.energy_per_orbital(e, n)
    lam = psi.schmidt(n)
    ent, _ = pk.entanglement(lam[lam > 0])
    say(f"{name} chi={chi}: {dt:.2f} s per growth iteration ({iters}), energy per orbital "
        f"{['%.6f' % x for x in per]}, centre entropy {ent:.6f}, {len(psi.bond(n))} sectors")
    assert sum(psi.bond(n).values()) == chi
    assert abs(np.sum(lam ** 2) - 1) < 1e-10
    assert all(x > free.bulk_energy_per_orbital(Ly, 1, 3) for x in per)
