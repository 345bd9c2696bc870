"""Two-site split (block SVD truncation) and finite two-site DMRG sweeps on the GPU,
against the oracle and exact diagonalisation.

* dm_theta_split against the oracle's split: the same new bond, the same Schmidt values
  per (N, k) sector, the same truncated two-site tensor (left . right, which does not
  depend on the singular-vector phases), canonical site tensors; with and without
  truncation, both sweep directions.
* Ly=4, Lx=8, flux 1/4, V=1, N=4, K=2 (the exact-diagonalisation check of the DMRG):
  sweeps at chi=160 keep every Schmidt value (the cut is lossless), so the energy equals
  exact diagonalisation (-10.812773825927, K=2) and the momentum-resolved entanglement
  spectrum at the centre equals the Schmidt values of the exact ground state, sector by
  sector; at chi=64 the sweep energies equal the oracle's sweep from the same start.
* The same cylinder's bond problems as the oracle's DMRG meets them: after the oracle
  converges at chi=64, one more right sweep hands out every two-site problem (L, R, theta
  and bonds of dimension 1 to 64); heff_apply matches the oracle's matvec on each of them
  in FP64, FP32 and BF16x3, and FP64 Lanczos matches the oracle's Lanczos on several.
"""
import json
import os
import sys
from fractions import Fraction

import numpy as np
import pytest

import workloads
from oracle import blocksparse as bs
from oracle import dmrg as odmrg
from oracle import ed
from oracle import model
from oracle import mpo as ompo

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1512_03318_amd as pk  # noqa: E402
from gpu_helpers import WindowGPU, block_rel, max_rel, problem, to_dev  # noqa: E402
from oracle import lanczos as olz  # noqa: E402

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dense_blocks(flat, kind, ly, x, y, **kw):
    return pk.unpack(flat.cpu().numpy(), kind, ly, x, y, **kw)


@pytest.mark.parametrize("chi", [10_000, 40])
@pytest.mark.parametrize("move_right", [True, False])
def test_theta_split_matches_the_oracle(chi, move_right):
    wl, L, W1, W2, R, th, keys, mpo = problem("ly4_chi64")
    j, ly = wl.j, wl.ly
    qs1 = [tuple(map(int, q)) for q in mpo.qsite[j]]
    qs2 = [tuple(map(int, q)) for q in mpo.qsite[j + 1]]
    a, c = pk.Bond(wl.bonds[j]), pk.Bond(wl.bonds[j + 2])
    say(f"theta split chi={chi} move_right={move_right}")
    x = to_dev(pk.pack(th, pk.LAYOUT_THETA, ly, a, c, qs1=qs1, qs2=qs2))
    sp = pk.Split(ly, a, c, qs1, qs2, x, chi, 1e-14, move_right)
    ol, orr, osch, odisc = odmrg.split_theta(th, chi, ly, qs1, "right" if move_right else "left")
    # the same bond and Schmidt values
    want = {qb: len(v) for qb, v in osch.items()}
    assert sp.bond == want
    ref = np.concatenate([osch[qb] for qb in sorted(osch)])
    assert np.abs(sp.schmidt - ref).max() <= 1e-12
    assert abs(sp.discarded - odisc) <= 1e-12
    # the same truncated theta
    b = pk.Bond(sp.bond)
    left = dense_blocks(sp.left, pk.LAYOUT_SITE, ly, a, b, qs1=qs1)
    right = dense_blocks(sp.right, pk.LAYOUT_SITE, ly, b, c, qs1=qs2)
    got = bs.contract_two_site(left, right, ly)
    refth = bs.contract_two_site(ol, orr, ly)
    num = max(np.abs(got.get(k, 0) - v).max() for k, v in refth.items())
    den = max(np.abs(v).max() for v in refth.values())
    say(f"  sectors {len(sp.bond)}, kept {len(sp.schmidt)}, theta error {num / den:.2e}")
    assert num / den <= 1e-12
    # canonical form of the unitary side
    if move_right:  # sum_{a, s} A^H A = 1 per bond sector b
        for qb, m in sp.bond.items():
            g = sum(blk.conj().T @ blk for (qa, s, qb2), blk in left.items() if qb2 == qb)
            assert np.abs(g - np.eye(m)).max() <= 1e-12
    else:  # sum_{s, c} B B^H = 1
        for qb, m in sp.bond.items():
            g = sum(blk @ blk.conj().T for (qb2, s, qc), blk in right.items() if qb2 == qb)
            assert np.abs(g - np.eye(m)).max() <= 1e-12


_cfg1 = {}


def cfg1():
    if not _cfg1:
        cyl = model.Cylinder(4, 8, Fraction(1, 4), 1.0, 1.0)
        m = ompo.build(cyl, "mixed")
        wl = workloads.make_workload("init", 4, 8, (1, 4), 64, 21, N_tot=4, K_tot=2)
        _cfg1.update(cyl=cyl, m=m, wl=wl)
    return _cfg1


def gpu_mps(wl, m):
    ly, n = wl.ly, wl.n
    init = wl.right_canonical_mps()
    qs = [[tuple(map(int, q)) for q in m.qsite[i]] for i in range(n)]
    bonds = [pk.Bond(b) for b in wl.bonds]
    tens = [to_dev(pk.pack(init[i], pk.LAYOUT_SITE, ly, bonds[i], bonds[i + 1], qs1=qs[i])) for i in range(n)]
    sites = [pk.MpoSite(m.W[i], m.qbond[i], m.qbond[i + 1], m.qsite[i]) for i in range(n)]
    return pk.MPS(ly, wl.bonds, qs, tens), sites, init


def ed_schmidt(cyl, n_left):
    """Schmidt values of the exact ground state (N=4, K=2) across the cut after
    n_left orbitals, per sector (N_left, K_left mod Ly)."""
    mom = model.orbital_momenta(cyl, "mixed")
    basis = ed.sector_basis(cyl.n_orb, 4, mom, 2, cyl.Ly)
    H = ed.hamiltonian(model.mixed_terms(cyl), basis)
    e0, psi = ed.ground_state(H)
    mask = (1 << n_left) - 1
    groups = {}
    for amp, st in zip(psi, basis.astype(np.int64)):
        lo, hi = int(st) & mask, int(st) >> n_left
        nl = bin(lo).count("1")
        kl = sum(int(mom[i]) for i in range(n_left) if (lo >> i) & 1) % cyl.Ly
        groups.setdefault((nl, kl), {}).setdefault(lo, {})[hi] = amp
    out = {}
    for q, rows in groups.items():
        cols = sorted({h for r in rows.values() for h in r})
        ci = {h: k for k, h in enumerate(cols)}
        M = np.zeros((len(rows), len(cols)), dtype=complex)
        for i, (lo, r) in enumerate(sorted(rows.items())):
            for h, v in r.items():
                M[i, ci[h]] = v
        s = np.linalg.svd(M, compute_uv=False)
        out[q] = s[s > 1e-12]
    return e0, out


@pytest.mark.timeout(900)
def test_gpu_sweeps_lossless_equal_exact_diagonalisation():
    c = cfg1()
    wl, m, cyl = c["wl"], c["m"], c["cyl"]
    say("GPU two-site DMRG, Ly=4 Lx=8, chi=160 (lossless)")
    psi, sites, _ = gpu_mps(wl, m)
    e = pk.dmrg_sweeps(psi, sites, 6, 160, 30, 1e-14, pk.DM_FP64)
    e_ed = json.load(open(os.path.join(GOLD, "ed_energies.json")))["ly4_lx8_flux1_4_V1_N4"]["2"][0]
    say(f"  sweep energies {['%.12f' % x for x in e]}  ED {e_ed:.12f}")
    assert abs(e[-1] - e_ed) <= 1e-10
    # momentum-resolved entanglement spectrum at the centre against the exact state
    n_left = wl.n // 2
    bond = psi.bond(n_left)
    lam = psi.schmidt(n_left)
    e0, exact = ed_schmidt(cyl, n_left)
    assert abs(e0 - e_ed) < 1e-10
    pos = 0
    got = {}
    for q in sorted(bond):
        got[q] = lam[pos:pos + bond[q]]
        pos += bond[q]
    for q, s in exact.items():
        g = got.get(q, np.zeros(0))
        g = g[g > 1e-12]
        assert len(g) == len(s), (q, len(g), len(s))
        assert np.abs(g - s).max() <= 1e-8, q
    ent, es = pk.entanglement(lam[lam > 1e-300])
    want = -sum(float(np.sum(s ** 2 * np.log(s ** 2))) for s in exact.values())
    say(f"  centre cut: {len(exact)} (N, k) sectors, entropy {ent:.10f} (exact {want:.10f}), "
        f"lowest entanglement energies {np.sort(es)[:4]}")
    assert abs(ent - want) <= 1e-8


@pytest.mark.timeout(900)
def test_gpu_sweeps_equal_the_oracle_sweeps_at_chi64():
    c = cfg1()
    wl, m = c["wl"], c["m"]
    say("GPU two-site DMRG, Ly=4 Lx=8, chi=64, against the oracle's sweeps")
    psi, sites, init = gpu_mps(wl, m)
    e = pk.dmrg_sweeps(psi, sites, 3, 64, 30, 1e-14, pk.DM_FP64)
    # the oracle with the same start, schedule and Lanczos length (no residual stop)
    r = odmrg.run(m, init, [64], wl.ly, sweeps_per_chi=1, tol_e=0.0, max_iter=30, tol_res=1e-300,
                  cutoff=1e-14)
    say(f"  GPU {['%.12f' % x for x in e]}")
    say(f"  oracle {['%.12f' % x for x in r.energies[:3]]}")
    for s in range(3):
        assert abs(e[s] - r.energies[s]) <= 1e-9 * abs(r.energies[s]), s


class _Captured(Exception):
    pass


_cfg1_bonds = []


def cfg1_bond_problems():
    """Every two-site problem of one right sweep of the oracle's DMRG on the cfg1 cylinder,
    taken after the oracle has converged at chi=64: (i, L, R, theta, keys, left bond,
    right bond) per bond."""
    if not _cfg1_bonds:
        c = cfg1()
        wl, m = c["wl"], c["m"]
        say("oracle DMRG on Ly=4 Lx=8 at chi=64 (to convergence), then one captured right sweep ...")
        r = odmrg.run(m, wl.right_canonical_mps(), [64], wl.ly, sweeps_per_chi=1)

        def grab(i, L, R, th, keys, da, dc):
            _cfg1_bonds.append((i, L, R, th, keys, da, dc))
            if len(_cfg1_bonds) == wl.n - 1:
                raise _Captured

        try:
            odmrg.run(m, r.tensors, [64], wl.ly, sweeps_per_chi=1, capture=grab)
        except _Captured:
            pass
        say(f"  {len(_cfg1_bonds)} bond problems, left bond dimensions "
            f"{[sum(b[5].values()) for b in _cfg1_bonds]}")
    return _cfg1_bonds


def _window(i, da, dc):
    c = cfg1()

    class W:  # the fields WindowGPU reads
        ly = c["wl"].ly
        j = i
        bonds = {i: da, i + 2: dc}
    return W


@pytest.mark.timeout(900)
def test_heff_apply_on_captured_cfg1_bond_problems():
    probs = cfg1_bond_problems()
    m = cfg1()["m"]
    tol = {pk.DM_FP64: 1e-12, pk.DM_FP32: 2e-5, pk.DM_BF16X3: 1e-4}
    worst = {p: 0.0 for p in tol}
    for i, L, R, th, keys, da, dc in probs:
        g = WindowGPU(_window(i, da, dc), L, R, m)
        x = to_dev(g.pack_theta(th))
        ref = bs.heff_apply(L, m.W[i], m.W[i + 1], R, th)
        for prec in tol:
            plan = g.plan(prec)
            y = torch.empty_like(x)
            pk.heff_apply(plan, x, y)
            got = g.unpack_theta(y.cpu().numpy())
            err, berr = max_rel(got, ref, keys), block_rel(got, ref, keys)
            worst[prec] = max(worst[prec], err)
            assert err <= tol[prec] and (prec != pk.DM_FP64 or berr <= 1e-12), (i, prec, err, berr)
    say(f"  worst relative error over {len(probs)} bonds: FP64 {worst[pk.DM_FP64]:.2e}, "
        f"FP32 {worst[pk.DM_FP32]:.2e}, BF16x3 {worst[pk.DM_BF16X3]:.2e}")


@pytest.mark.timeout(900)
def test_lanczos_on_captured_cfg1_bond_problems():
    probs = cfg1_bond_problems()
    m = cfg1()["m"]
    for i, L, R, th, keys, da, dc in [probs[k] for k in (0, 2, 6, len(probs) // 2, len(probs) - 3)]:
        g = WindowGPU(_window(i, da, dc), L, R, m)
        x = to_dev(g.pack_theta(th))
        e, k = pk.lanczos_ground(g.plan(pk.DM_FP64), x, 30, 1e-14)
        mv = lambda v, L=L, R=R, i=i, keys=keys: bs.flatten(
            bs.heff_apply(L, m.W[i], m.W[i + 1], R, bs.unflatten(v, keys)), keys)
        eo, vo, ko, _, _ = olz.lanczos(mv, bs.flatten(th, keys), max_iter=30)
        say(f"  bond {i} (n={x.numel()}): steps {k} (oracle {ko}), energy {e:.12f} (oracle {eo:.12f})")
        assert k == ko
        assert abs(e - eo) <= 1e-10 * abs(eo)
        v = bs.flatten(g.unpack_theta(x.cpu().numpy()), keys)
        assert 1 - abs(np.vdot(vo, v)) / np.linalg.norm(v) < 1e-8
