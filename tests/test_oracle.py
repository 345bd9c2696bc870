"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

* the two bases give the same spectrum (eq. H_real vs eqs. H_kin + H_int, exact);
* V = 0 energies equal the free-fermion closed form built from eq. H_kin's levels;
* the worked example of Fig. 7a (magnitude (V/L) 2 |cos 2a - cos 4a|, a = 2 pi / 8) and
  the 2 (1 - cos q) V / L density-density coefficient of Sec. IV D;
* the MPO contracted to a dense matrix equals the Hamiltonian assembled directly from
  the term lists; the real-space MPO has D = 3L + 2 in the bulk (Sec. IV C);
* <psi2|H|psi1> (H from exact diagonalisation) equals <theta2|H_eff theta1>;
* Lanczos reduces to the library eigensolver when run to the full dimension;
* DMRG at lossless bond dimension equals exact diagonalisation.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import workloads
from oracle import blocksparse as bs
from oracle import dmrg, ed, free, lanczos, model, mpo, synth

from helpers import mps_vector

GOLD = os.path.join(os.path.dirname(__file__), "golden")
SMALL = [(2, 4, Fraction(1, 4)), (2, 3, Fraction(1, 3)), (3, 3, Fraction(1, 3))]


@pytest.mark.parametrize("Lx,Ly,flux", SMALL)
@pytest.mark.parametrize("V", [0.0, 1.0])
def test_bases_have_equal_spectra(Lx, Ly, flux, V):
    cyl = model.Cylinder(Ly, Lx, flux, 1.0, V)
    basis = ed.sector_basis(cyl.n_orb)
    hm = ed.hamiltonian(model.mixed_terms(cyl), basis).toarray()
    hr = ed.hamiltonian(model.real_terms(cyl), basis).toarray()
    assert np.abs(hm - hm.conj().T).max() < 1e-14
    assert np.abs(np.linalg.eigvalsh(hm) - np.linalg.eigvalsh(hr)).max() < 1e-12


@pytest.mark.parametrize("Lx,Ly,flux", SMALL + [(3, 4, Fraction(1, 4))])
def test_free_fermion_closed_form(Lx, Ly, flux):
    cyl = model.Cylinder(Ly, Lx, flux, 1.0, 0.0)
    basis = ed.sector_basis(cyl.n_orb)
    h = ed.hamiltonian(model.mixed_terms(cyl), basis).toarray()
    assert abs(np.linalg.eigvalsh(h)[0] - free.fock_ground_energy(cyl)) < 1e-11
    mom = model.orbital_momenta(cyl, "mixed")
    for N in (1, 2, 3):
        es = [ed.lowest(ed.hamiltonian(model.mixed_terms(cyl),
                                       ed.sector_basis(cyl.n_orb, N, mom, K, Ly)))[0]
              for K in range(Ly) if len(ed.sector_basis(cyl.n_orb, N, mom, K, Ly))]
        assert abs(min(es) - free.ground_energy(cyl, N)) < 1e-11


def test_cfg1_free_energy_and_ed_regression():
    cyl0 = model.Cylinder(4, 8, Fraction(1, 4), 1.0, 0.0)
    # lowest four levels of the Ly=4, Lx=8, flux 1/4 cylinder at V = 0
    lev = free.levels(cyl0)[0]
    assert lev[3] < lev[4] - 1e-3            # no Fermi-level tie at N = 4
    cyl = model.Cylinder(4, 8, Fraction(1, 4), 1.0, 1.0)
    mom = model.orbital_momenta(cyl, "mixed")
    gold = json.load(open(os.path.join(GOLD, "ed_energies.json")))["ly4_lx8_flux1_4_V1_N4"]
    H = ed.hamiltonian(model.mixed_terms(cyl), ed.sector_basis(32, 4, mom, 2, 4))
    assert abs(ed.lowest(H)[0] - gold["2"][0]) < 1e-10
    # interaction raises the energy above the free value
    assert gold["2"][0] > free.ground_energy(cyl0, 4)


def _matrix_element(cyl, created, annihilated):
    """<created|H|annihilated> for two occupation sets on the chain."""
    basis = ed.sector_basis(cyl.n_orb, len(created))
    H = ed.hamiltonian(model.mixed_terms(cyl), basis)
    i = np.searchsorted(basis, sum(1 << c for c in created))
    j = np.searchsorted(basis, sum(1 << c for c in annihilated))
    return H[i, j]


def test_fig7a_worked_example():
    g = json.load(open(os.path.join(GOLD, "paper_values.json")))["fig7a_term"]
    V = 1.3
    cyl = model.Cylinder(g["L"], 1, Fraction(1, 8), 1.0, V)
    el = _matrix_element(cyl, g["orbitals_created"], g["orbitals_annihilated"])
    # c+_0 c_2 c_4 c+_6 |{2,4}> = -|{0,6}> with the Jordan-Wigner signs of eq. JW, so the
    # coefficient of the chain-ordered product is -<{0,6}|H|{2,4}>
    coef = -el
    alpha = 2 * np.pi / 8
    paper = (V / 8) * 2 * (np.cos(2 * alpha) - np.cos(4 * alpha))
    assert abs(abs(coef) - g["abs_coefficient_over_V"] * V) < 1e-14
    assert abs(abs(coef) - abs(paper)) < 1e-14
    # sign under these conventions (chain-ordered product, Fourier sign of eq. H_kin)
    assert abs(coef + paper) < 1e-14


@pytest.mark.parametrize("L", [5, 6])
def test_density_density_coefficient(L):
    V = 0.7
    cyl = model.Cylinder(L, 1, Fraction(1, L), 1.0, V)
    basis = ed.sector_basis(L)
    H = ed.hamiltonian([t for t in model.mixed_terms(cyl) if t.fam[0] == "intra"], basis)
    diag = lambda occ: H[np.searchsorted(basis, sum(1 << c for c in occ))] .toarray()[0][
        np.searchsorted(basis, sum(1 << c for c in occ))].real
    for k in range(L):
        for q in range(1, L):
            kq = (k + q) % L
            nn = diag([k, kq]) - diag([k]) - diag([kq]) + diag([])
            assert abs(nn - 2 * (1 - np.cos(2 * np.pi * q / L)) * V / L) < 1e-13


@pytest.mark.parametrize("Lx,Ly,flux", SMALL + [(2, 5, Fraction(1, 5))])
@pytest.mark.parametrize("basis", ["mixed", "real"])
def test_mpo_contracts_to_hamiltonian(Lx, Ly, flux, basis):
    cyl = model.Cylinder(Ly, Lx, flux, 1.0, 1.0)
    H = ed.hamiltonian(model.terms_for(cyl, basis), ed.sector_basis(cyl.n_orb)).toarray()
    raw = mpo.build(cyl, basis, merge=False)
    merged = mpo.build(cyl, basis, merge=True)
    for m in (raw, merged):
        mpo.check_charges(m)
        assert np.abs(mpo.to_dense(m) - H).max() < 1e-12
    assert max(merged.bond_dims()) <= max(raw.bond_dims())


@pytest.mark.parametrize("Lx,Ly,flux", SMALL + [(3, 4, Fraction(1, 4))])
def test_eq_rot_mpo_is_real_and_exact(Lx, Ly, flux):
    """Eq. rot: the mixed-basis MPO rewritten with real numbers only; it keeps the
    machine's bond dimension (Sec. IV D) and charges and still contracts to H."""
    cyl = model.Cylinder(Ly, Lx, flux, 1.0, 1.0)
    raw = mpo.build(cyl, "mixed", merge=False)
    rot = mpo.build(cyl, "mixed", merge=False, real=True)
    merged = mpo.build(cyl, "mixed", real=True)
    assert rot.bond_dims() == raw.bond_dims()
    assert any(np.abs(w.imag).max() > 0 for w in raw.W)      # the phases were complex
    H = ed.hamiltonian(model.mixed_terms(cyl), ed.sector_basis(cyl.n_orb)).toarray()
    for m in (rot, merged):
        assert all(np.abs(w.imag).max() == 0 for w in m.W)
        mpo.check_charges(m)
        if cyl.n_orb <= 12:
            assert np.abs(mpo.to_dense(m) - H).max() < 1e-12


def test_eq_rot_turns_a_phase_pair_into_a_rotation():
    """A transition between two branch pairs that carries (e^{i t}, e^{-i t}) on the
    diagonal becomes the real 2 x 2 rotation [[cos t, -sin t], [sin t, cos t]]: the
    similarity of eq. rot, read off the machine's own states."""
    cyl = model.Cylinder(4, 2, Fraction(1, 4), 1.0, 1.0)
    raw = mpo.build(cyl, "mixed", merge=False)
    rot = mpo.build(cyl, "mixed", merge=False, real=True)
    seen = 0
    for i, w in enumerate(raw.W):
        kin, kout = raw.keys[i], raw.keys[i + 1]
        jin = {k: j for j, k in enumerate(kin)}
        jout = {k: j for j, k in enumerate(kout)}
        for p, k in enumerate(kin):
            q = mpo._branch_partner(k)
            if q is None or k[2] != 1:
                continue
            m = jin[q]
            for pp, ko in enumerate(kout):
                qo = mpo._branch_partner(ko)
                if qo is None or ko[2] != 1:
                    continue
                mm = jout[qo]
                for sp_, s in ((1, 0), (0, 1), (1, 1), (0, 0)):
                    c = w[p, sp_, s, pp]
                    if abs(c) < 1e-12 or abs(c.imag) < 1e-9:
                        continue
                    # conjugate branch carries conj(c), no cross terms
                    assert abs(w[m, sp_, s, mm] - np.conj(c)) < 1e-13
                    assert abs(w[p, sp_, s, mm]) == 0 and abs(w[m, sp_, s, pp]) == 0
                    blk = rot.W[i][np.ix_([p, m], [sp_], [s], [pp, mm])][:, 0, 0, :]
                    want = np.array([[c.real, -c.imag], [c.imag, c.real]])
                    assert np.abs(blk - want).max() < 1e-13
                    seen += 1
    assert seen > 0


def test_real_window_heff_is_real_and_equals_ed():
    """A window of the real formulation (real MPO, real isometries and theta): every
    block of L, R and H_eff theta is real, and <theta2|H_eff theta1> equals
    <psi2|H|psi1> with H from exact diagonalisation."""
    wl = workloads.make_workload("pin", 3, 4, (1, 3), 16, 7, real=True)
    L, W1, W2, R, th1, keys, m = synth.window_problem(wl)
    assert all(np.abs(w.imag).max() == 0 for w in m.W)
    for env in (L, R):
        assert max(np.abs(b.imag).max() for b in env.values()) == 0
    rng = np.random.default_rng(1)
    th2 = {k: rng.standard_normal(v.shape) + 0j for k, v in th1.items()}
    h1 = bs.heff_apply(L, W1, W2, R, th1)
    assert max(np.abs(b.imag).max() for b in h1.values()) == 0
    cyl = synth.cylinder_of(wl)
    H = ed.hamiltonian(model.terms_for(cyl, "mixed"), ed.sector_basis(wl.n))
    p1, p2 = mps_vector(wl, th1), mps_vector(wl, th2)
    lhs = np.vdot(p2, H @ p1)
    rhs = np.vdot(bs.flatten(th2, keys), bs.flatten(h1, keys))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


@pytest.mark.parametrize("L", [3, 4, 5])
def test_real_space_bond_dimension(L):
    cyl = model.Cylinder(L, 4, Fraction(1, L), 1.0, 1.0)
    dims = mpo.build(cyl, "real").bond_dims()
    bulk = dims[L + 1: 3 * L]
    assert all(d == 3 * L + 2 for d in bulk), bulk


def test_mixed_mpo_sizes_report():
    """D is an output of the construction (values of Fig. 8a are not available): check
    the ring-boundary bonds of the mixed MPO equal the real-space 3L + 2 and the bound
    D <= 26 L + 9 of Sec. IV D holds everywhere."""
    L = 6
    cyl = model.Cylinder(L, 3, Fraction(1, L), 1.0, 1.0)
    dims = mpo.build(cyl, "mixed").bond_dims()
    assert dims[L] == dims[2 * L] == 3 * L + 2
    assert max(dims) <= 26 * L + 9


@pytest.mark.parametrize("basis", ["mixed", "real"])
def test_heff_bilinear_equals_ed(basis):
    wl = workloads.make_workload("pin", 3, 4, (1, 3), 16, 7, basis=basis)
    L, W1, W2, R, th1, keys, _ = synth.window_problem(wl)
    rng = np.random.default_rng(1)
    th2 = {k: rng.standard_normal(v.shape) + 1j * rng.standard_normal(v.shape) for k, v in th1.items()}
    cyl = synth.cylinder_of(wl)
    H = ed.hamiltonian(model.terms_for(cyl, basis), ed.sector_basis(wl.n))
    p1, p2 = mps_vector(wl, th1), mps_vector(wl, th2)
    lhs = np.vdot(p2, H @ p1)
    h1 = bs.flatten(bs.heff_apply(L, W1, W2, R, th1), keys)
    rhs = np.vdot(bs.flatten(th2, keys), h1)
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))
    # isometries: the MPS norm equals the norm of theta
    assert abs(np.vdot(p1, p1) - np.vdot(bs.flatten(th1, keys), bs.flatten(th1, keys))) < 1e-12
    # Hermitian
    h2 = bs.flatten(bs.heff_apply(L, W1, W2, R, th2), keys)
    assert abs(np.vdot(bs.flatten(th2, keys), h1) - np.conj(np.vdot(bs.flatten(th1, keys), h2))) < 1e-12


def test_isometries():
    wl = workloads.preset("ly4_chi64")
    for i in (3, wl.j - 1):
        A = wl.site_tensor(i)
        for qb in wl.bonds[i + 1]:
            blocks = [blk for (qa, s, q), blk in A.items() if q == qb]
            M = np.vstack(blocks)
            assert np.abs(M.conj().T @ M - np.eye(M.shape[1])).max() < 1e-13
    for i in (wl.j + 2, wl.n - 3):
        B = wl.site_tensor(i)
        for qb in wl.bonds[i]:
            M = np.hstack([blk for (q, s, qc), blk in sorted(B.items(), key=lambda kv: (kv[0][1], kv[0][2])) if q == qb])
            assert np.abs(M @ M.conj().T - np.eye(M.shape[0])).max() < 1e-13


def test_lanczos_full_dimension_matches_library():
    rng = np.random.default_rng(0)
    n = 24
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    h = (a + a.conj().T) / 2
    e, x, k, _, _ = lanczos.lanczos(lambda v: h @ v, rng.standard_normal(n) + 0j, max_iter=n)
    lam, vec = np.linalg.eigh(h)
    assert k == n
    assert abs(e - lam[0]) < 1e-12
    assert 1 - abs(np.vdot(vec[:, 0], x)) < 1e-12
    e5, _, _, al, be = lanczos.lanczos(lambda v: h @ v, rng.standard_normal(n) + 0j, max_iter=5)
    assert e5 >= lam[0] - 1e-12                               # Ritz value above lambda_min
    t = np.diag(al) + np.diag(be, 1) + np.diag(be, -1)
    assert np.linalg.eigvalsh(t)[-1] <= lam[-1] + 1e-12       # interlacing at the top


def test_restarted_lanczos_ground_state():
    """Restarted Lanczos converges to LAPACK's lowest eigenpair (n = 300 >> 30 steps),
    including the effective Hamiltonian of a small window against its dense matrix."""
    rng = np.random.default_rng(3)
    n = 300
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    h = (a + a.conj().T) / 2
    e, x, res, nmv = lanczos.ground_state(lambda v: h @ v, rng.standard_normal(n) + 0j, tol_res=1e-11)
    lam, vec = np.linalg.eigh(h)
    assert nmv > 30 and abs(e - lam[0]) < 1e-11 and 1 - abs(np.vdot(vec[:, 0], x)) < 1e-12
    assert np.linalg.norm(h @ x - e * x) == pytest.approx(res, rel=1e-6)
    wl = workloads.preset("ly3_chi16")
    L, W1, W2, R, th, keys, _ = synth.window_problem(wl)
    mv = lambda v: bs.flatten(bs.heff_apply(L, W1, W2, R, bs.unflatten(v, keys)), keys)
    dim = sum(m * n for _, (m, n) in keys)
    H = np.array([mv(np.eye(dim)[i]) for i in range(dim)]).T
    lam = np.linalg.eigvalsh((H + H.conj().T) / 2)
    e, x, res, _ = lanczos.ground_state(mv, bs.flatten(th, keys), tol_res=1e-12)
    assert abs(e - lam[0]) < 1e-10 * abs(lam[0])


def test_lanczos_breakdown_on_eigenvector():
    h = np.diag(np.arange(6, dtype=float)).astype(complex)
    v = np.zeros(6, complex)
    v[2] = 1
    e, x, k, _, _ = lanczos.lanczos(lambda u: h @ u, v, max_iter=30)
    assert k == 1 and abs(e - 2.0) < 1e-15


def test_dmrg_lossless_equals_ed():
    cyl = model.Cylinder(3, 4, Fraction(1, 3), 1.0, 1.0)
    m = mpo.build(cyl, "mixed")
    wl = workloads.make_workload("init", 3, 4, (1, 3), 64, 21, N_tot=2, K_tot=1)
    r = dmrg.run(m, wl.right_canonical_mps(), [64], 3, sweeps_per_chi=2)
    mom = model.orbital_momenta(cyl, "mixed")
    e_ed = ed.lowest(ed.hamiltonian(model.mixed_terms(cyl), ed.sector_basis(12, 2, mom, 1, 3)))[0]
    assert abs(r.energy - e_ed) < 1e-10


def test_dmrg_cfg1_chi64_variational():
    """Ly=4, Lx=8, flux 1/4, V=1, N=4 in its ground sector K=2, chi = 64."""
    gold = json.load(open(os.path.join(GOLD, "ed_energies.json")))["ly4_lx8_flux1_4_V1_N4"]
    e_ed = gold["2"][0]
    cyl = model.Cylinder(4, 8, Fraction(1, 4), 1.0, 1.0)
    m = mpo.build(cyl, "mixed")
    wl = workloads.make_workload("init", 4, 8, (1, 4), 64, 21, N_tot=4, K_tot=2)
    r = dmrg.run(m, wl.right_canonical_mps(), [64, 64], 4, sweeps_per_chi=1,
                 rng=np.random.default_rng(3), noise=1e-4)
    assert r.energy >= e_ed - 1e-10
    assert r.energy - e_ed < 1e-7
    # Schmidt values at the centre are labelled by (N, k) and normalised
    tot = sum(float(np.sum(s ** 2)) for s in r.schmidt.values())
    assert abs(tot - 1) < 1e-10
