"""Pins of the oracle's infinite-cylinder pieces (no GPU).

* The bulk MPO cell read off the finite-state machine (Sec. IV), mixed basis (complex and
  in the real form of eq. rot) and real-space basis: copies of it between the boundary vectors picking R and F contract to the
  Hamiltonian of the finite cylinder built from the term lists (eqs. H_kin, H_int;
  eq. H_real) by exact diagonalisation's operator algebra, which shares nothing with the
  machine.
* The free-fermion energy per orbital of the infinite cylinder (Bloch bands of eq. H_kin
  with the magnetic cell) against finite cylinders: the energy added by 2 x more rings of a
  gapped band insulator is the bulk energy up to exponentially small end effects.
* iDMRG by unit-cell growth at V = 0 (flux 1/3, lowest band filled) converges to that
  closed form in the mixed basis (complex and the real form of eq. rot) and in the
  real-space basis.
"""
from fractions import Fraction

import numpy as np
import pytest

import workloads
from oracle import ed, free, idmrg, model


@pytest.mark.parametrize("basis,rot", [("mixed", False), ("mixed", True), ("real", False)])
@pytest.mark.parametrize("Ly,flux,rings,copies", [(3, Fraction(1, 1), 1, 3), (3, Fraction(1, 3), 3, 1),
                                                  (4, Fraction(1, 2), 2, 1)])
def test_bulk_cell_chain_contracts_to_hamiltonian(Ly, flux, rings, copies, basis, rot):
    cell = idmrg.bulk_cell(Ly, flux, 1.0, 1.0, rings, basis=basis, real=rot)
    if rot:  # eq. rot: every entry real
        assert max(np.abs(w.imag).max() for w in cell.W) == 0
    n = rings * Ly
    assert cell.n_sites == n and cell.W[0].shape[0] == cell.W[-1].shape[3]
    assert np.array_equal(cell.qbond[0], cell.qbond[-1])
    cyl = model.Cylinder(Ly, rings * copies, flux, 1.0, 1.0)
    H = ed.hamiltonian(model.terms_for(cyl, basis), ed.sector_basis(cyl.n_orb)).toarray()
    got = idmrg.cell_chain_dense(cell, copies)
    assert np.abs(got - H).max() < 1e-12


@pytest.mark.parametrize("Ly,q", [(3, 3), (4, 4)])
def test_bulk_free_fermion_energy_against_finite_cylinders(Ly, q):
    e_bulk = free.bulk_energy_per_orbital(Ly, 1, q)
    e = {Lx: free.ground_energy(model.Cylinder(Ly, Lx, Fraction(1, q), 1.0, 0.0), Lx * Ly // q)
         for Lx in (16 * q, 32 * q)}
    assert abs((e[32 * q] - e[16 * q]) / (16 * q * Ly) - e_bulk) < 1e-12


@pytest.mark.parametrize("basis,rot,seed,n_iter,tol", [
    ("mixed", False, 7, 6, 5e-5),
    # the real form of eq. rot from real isometries: real arithmetic throughout
    ("mixed", True, 8, 10, 1e-4),
    ("real", False, 7, 10, 1e-4),
])
def test_idmrg_free_fermions_reach_the_bulk_energy(basis, rot, seed, n_iter, tol):
    """Ly=3, flux 1/3, V=0, three particles per three-ring cell (the lowest band), chi=64:
    the energy added per iteration, per orbital, reaches the Bloch-band value in the mixed
    basis, in its real form (eq. rot) and in the real-space basis.  The growth approaches it
    with a decaying oscillation whose size depends on the random start (about 4e-3 after
    three iterations from a real start, 1e-5 to 1e-4 after ten)."""
    cell = idmrg.bulk_cell(3, Fraction(1, 3), 1.0, 0.0, 3, basis=basis, real=rot)
    gs = workloads.growth_start(3, 3, 3, 0, 64, seed, basis=basis, real=rot)
    L0, R0 = idmrg.block_envs(cell, gs.left, gs.right, next(iter(gs.bonds[-1])))
    r = idmrg.run(cell, gs.cells, gs.bonds[gs.n:3 * gs.n + 1], n_iter, 64, L0, R0, gs.d)
    e = idmrg.energy_per_orbital(r.energies, cell.n_sites)
    exact = free.bulk_energy_per_orbital(3, 1, 3)
    print("energy per orbital", e, "exact", exact)
    assert abs(e[-1] - exact) < tol
    # the Schmidt values at the centre are normalised and every (N, k) sector is a charge
    # of the bond between two cells (N near the filling of the cells to its left)
    lam = np.concatenate(list(r.schmidt[-1].values()))
    assert abs(np.sum(lam ** 2) - 1) < 1e-12
    cells_left = len(r.energies) + 1          # the initial block, the absorbed cells, one cell
    assert all(abs(q[0] - 3 * cells_left) <= 4 for q in r.schmidt[-1])


@pytest.mark.parametrize("K_cell", [0, 1])
def test_growth_start_shapes(K_cell):
    """The seeded start of the growth: the left block's tensors are left isometries from
    the vacuum, the two cells' and the right block's are right isometries, and the two
    cells' last bond is their first with every charge moved by d."""
    gs = workloads.growth_start(3, 3, 3, K_cell, 32, 17)
    n, ly, d = gs.n, gs.ly, gs.d
    assert d == (6, (2 * K_cell) % 3)
    moved = {idmrg.shift_charge(q, d, ly): m for q, m in gs.bonds[n].items()}
    assert moved == gs.bonds[3 * n] and len(gs.bonds[n]) > 1
    assert gs.bonds[0] == {(0, 0): 1} and gs.bonds[4 * n] == {(12, (4 * K_cell) % 3): 1}
    for i, A in enumerate(gs.left):  # sum_{a,s} A^H A = 1 per sector of the right bond
        for qb, m in gs.bonds[i + 1].items():
            g = sum(blk.conj().T @ blk for (qa, s, qb2), blk in A.items() if qb2 == qb)
            assert np.abs(g - np.eye(m)).max() < 1e-12
    for off, tens in ((n, gs.cells), (3 * n, gs.right)):
        for i, B in enumerate(tens):  # sum_{s,c} B B^H = 1 per sector of the left bond
            for qb, m in gs.bonds[off + i].items():
                g = sum(blk @ blk.conj().T for (qb2, s, qc), blk in B.items() if qb2 == qb)
                assert np.abs(g - np.eye(m)).max() < 1e-12
