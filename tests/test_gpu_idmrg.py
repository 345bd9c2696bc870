"""Infinite-cylinder DMRG by unit-cell growth on the GPU (dm_idmrg) against the oracle.

* Ly=3, flux 1/3, V=1, three-ring cells (9 orbitals), three particles per cell: from the
  same seeded start (one-cell random blocks, two random right-canonical cells) the GPU's
  total energies E_j equal the oracle's iDMRG iteration by iteration, and the Schmidt
  values between the last two cells agree sector by sector.
* The same cylinder at V=0: the energy added per iteration, per orbital, reaches the
  free-fermion Bloch-band value (closed form).
"""
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
def test_gpu_idmrg_equals_the_oracle():
    cell = idmrg.bulk_cell(3, Fraction(1, 3), 1.0, 1.0, 3)
    gs = workloads.growth_start(3, 3, 3, 0, 32, 17)
    n, chi, iters = gs.n, 32, 4
    say(f"iDMRG Ly=3 flux 1/3 V=1, {n}-orbital cell (D {cell.W[0].shape[0]}), chi={chi}, {iters} iterations")
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
def test_gpu_idmrg_free_fermions_reach_the_bulk_energy():
    cell = idmrg.bulk_cell(3, Fraction(1, 3), 1.0, 0.0, 3)
    gs = workloads.growth_start(3, 3, 3, 0, 64, 7)
    psi, sites, _, (l0, r0) = gpu_start(cell, gs)
    e = pk.idmrg(psi, sites, gs.d, l0, r0, 6, 64)
    per = idmrg.energy_per_orbital(e, gs.n)
    exact = free.bulk_energy_per_orbital(3, 1, 3)
    say(f"iDMRG V=0: energy per orbital {['%.9f' % x for x in per]}, Bloch bands {exact:.9f}")
    assert abs(per[-1] - exact) < 5e-5
