"""Seeded synthetic MPS workloads on a Hofstadter cylinder (sizes and random numbers only).

Recipe (each step is a workload choice, not part of the method):

* chain of n = Lx * Ly orbitals, orbital i = x * Ly + m, local states |0>, |1> with
  charges (0, 0) and (1, m) (mixed basis) or (1, 0) with modulus 1 (real-space basis);
* bond b (left of orbital b) carries the total charge of the orbitals left of it; the
  left end is (0, 0), the right end (N_tot, K_tot);
* sector dimensions on bond b: weight exp(-(N - Nbar_b)^2 / (2 sigma_N^2)) for
  |N - Nbar_b| <= ceil(3 sigma_N), uniform over k, Nbar_b = round(b * N_tot / n), chi
  apportioned by largest remainder, then clipped forward and backward until every
  left site tensor can be an isometry from (a, s) to b and every right site tensor an
  isometry from (s, c) to b;
* isometries: complex Gaussian entries (real and imaginary parts N(0, 1/2)), QR per
  charge block, columns rephased so that diag(R) > 0; one numpy generator per site from
  ``SeedSequence(seed).spawn(n + 1)``, the last one for the two-site wavefunction;
* ``real=True`` (mixed basis only): the same recipe with real N(0, 1) entries, for the
  real formulation of the mixed-basis Hamiltonian (eq. rot) whose MPO is real.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from math import ceil, sqrt

import numpy as np


def site_charges(Lx: int, Ly: int, basis: str = "mixed"):
    """[(0,0), (1,m)] per orbital (mixed) or [(0,0), (1,0)] (real space, modulus 1)."""
    out = []
    for x in range(Lx):
        for m in range(Ly):
            out.append(((0, 0), (1, m if basis == "mixed" else 0)))
    return out


def _add(a, b, ly):
    return (a[0] + b[0], (a[1] + b[1]) % ly)


def _sub(a, b, ly):
    return (a[0] - b[0], (a[1] - b[1]) % ly)


def _apportion(chi: int, weights: dict) -> dict:
    keys = sorted(weights)
    w = np.array([weights[k] for k in keys], dtype=np.float64)
    raw = chi * w / w.sum()
    base = np.floor(raw).astype(np.int64)
    rem = int(chi - base.sum())
    frac = raw - base
    order = sorted(range(len(keys)), key=lambda i: (-frac[i], i))
    for i in order[:rem]:
        base[i] += 1
    return {k: int(d) for k, d in zip(keys, base) if d > 0}


def bond_sectors(n: int, qsite, ly: int, chi: int, N_tot: int, K_tot: int,
                 sigma_N: float) -> list[dict]:
    """Sector dimensions {(N, k): dim} on bonds 0..n."""
    bonds = []
    width = int(ceil(3.0 * sigma_N))
    for b in range(n + 1):
        if b == 0:
            bonds.append({(0, 0): 1})
            continue
        if b == n:
            bonds.append({(N_tot, K_tot % ly): 1})
            continue
        nbar = int(round(b * N_tot / n))
        lo = max(0, N_tot - (n - b), nbar - width)
        hi = min(b, N_tot, nbar + width)
        weights = {(N, k): float(np.exp(-(N - nbar) ** 2 / (2.0 * sigma_N ** 2)))
                   for N in range(lo, hi + 1) for k in range(ly)}
        bonds.append(_apportion(chi, weights))
    _clip(bonds, qsite, ly)
    return [dict(sorted(bd.items())) for bd in bonds]


def _clip(bonds: list, qsite, ly: int) -> None:
    """Shrink sector dimensions in place until every left site tensor can be an isometry
    from (a, s) to b and every right site tensor one from (s, c) to b."""
    n = len(bonds) - 1
    changed = True
    while changed:
        changed = False
        for b in range(1, n + 1):
            prev = bonds[b - 1]
            for q in list(bonds[b]):
                cap = sum(prev.get(_sub(q, qsite[b - 1][s], ly), 0) for s in (0, 1))
                if bonds[b][q] > cap:
                    changed = True
                    if cap:
                        bonds[b][q] = cap
                    else:
                        del bonds[b][q]
        for b in range(n - 1, -1, -1):
            nxt = bonds[b + 1]
            for q in list(bonds[b]):
                cap = sum(nxt.get(_add(q, qsite[b][s], ly), 0) for s in (0, 1))
                if bonds[b][q] > cap:
                    changed = True
                    if cap:
                        bonds[b][q] = cap
                    else:
                        del bonds[b][q]


def _gauss(rng, shape, real=False):
    """Complex Gaussian (real and imaginary parts N(0, 1/2)), or with real=True real
    N(0, 1) entries (stored complex with zero imaginary parts)."""
    if real:
        return rng.standard_normal(shape).astype(np.complex128)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / sqrt(2.0)


def _isometry(rng, rows: int, cols: int, real=False) -> np.ndarray:
    if rows < cols:
        raise ValueError("isometry needs rows >= cols")
    q, r = np.linalg.qr(_gauss(rng, (rows, cols), real))
    d = np.diag(r)
    return q * (d / np.abs(d))[None, :]


def left_isometry(rng, bl: dict, br: dict, qs, ly: int, real=False) -> dict:
    """A[a, s, b] with sum_{a,s} conj(A[a,s,b]) A[a,s,b'] = delta_{bb'}; blocks keyed (qa, s, qb)."""
    out = {}
    for qb, mb in br.items():
        parts = [(s, _sub(qb, qs[s], ly)) for s in (0, 1)]
        parts = [(s, qa) for s, qa in parts if qa in bl]
        rows = sum(bl[qa] for _, qa in parts)
        q = _isometry(rng, rows, mb, real)
        r0 = 0
        for s, qa in parts:
            out[(qa, s, qb)] = q[r0:r0 + bl[qa]].copy()
            r0 += bl[qa]
    return out


def right_isometry(rng, bl: dict, br: dict, qs, ly: int, real=False) -> dict:
    """B[b, s, c] with sum_{s,c} B[b,s,c] conj(B[b',s,c]) = delta_{bb'}; blocks keyed (qb, s, qc)."""
    out = {}
    for qb, mb in bl.items():
        parts = [(s, _add(qb, qs[s], ly)) for s in (0, 1)]
        parts = [(s, qc) for s, qc in parts if qc in br]
        cols = sum(br[qc] for _, qc in parts)
        q = _isometry(rng, cols, mb, real).conj().T    # (mb, cols), orthonormal rows
        c0 = 0
        for s, qc in parts:
            out[(qb, s, qc)] = q[:, c0:c0 + br[qc]].copy()
            c0 += br[qc]
    return out


def random_site(rng, bl: dict, br: dict, qs, ly: int) -> dict:
    """Site tensor M[a, s, b] with Gaussian blocks (not an isometry), blocks keyed
    (qa, s, qb) for every charge-allowed q(a) + q(s) = q(b)."""
    out = {}
    for qb, mb in br.items():
        for s in (0, 1):
            qa = _sub(qb, qs[s], ly)
            if qa in bl:
                out[(qa, s, qb)] = _gauss(rng, (bl[qa], mb))
    return out


def random_theta(rng, ba: dict, bc: dict, qs1, qs2, ly: int, real=False) -> dict:
    """Two-site wavefunction theta[a, s1, s2, c], blocks keyed (qa, s1, s2, qc), unnormalised."""
    out = {}
    for qa, ma in ba.items():
        for s1 in (0, 1):
            for s2 in (0, 1):
                qc = _add(_add(qa, qs1[s1], ly), qs2[s2], ly)
                if qc in bc:
                    out[(qa, s1, s2, qc)] = _gauss(rng, (ma, bc[qc]), real)
    return out


def random_env(rng, bond: dict, qw, ly: int, side: str, real=False) -> dict:
    """Random environment blocks with the block structure of a left (side="L",
    q(a') = q(a) + q(w)) or right (side="R", same rule on (c', c)) environment on
    ``bond`` with MPO state charges ``qw`` (given by the caller).  Keys (q', w, q)."""
    out = {}
    for w, qwv in enumerate(qw):
        for q, m in bond.items():
            qp = _add(q, (int(qwv[0]), int(qwv[1])), ly)
            if qp in bond:
                out[(qp, w, q)] = _gauss(rng, (bond[qp], m), real)
    return out


@dataclass
class Workload:
    """A finite cylinder MPS with a two-site window at orbitals (j, j+1)."""

    name: str
    Ly: int
    Lx: int
    flux: tuple          # (p, q): phi = 2 pi p / q
    t: float
    V: float
    chi: int
    N_tot: int
    K_tot: int
    sigma_N: float
    seed: int
    basis: str = "mixed"
    j: int = -1
    real: bool = False   # real entries (the eq. rot formulation of the mixed basis)
    bonds: list = field(default_factory=list, repr=False)
    qsite: list = field(default_factory=list, repr=False)

    @property
    def n(self) -> int:
        return self.Lx * self.Ly

    @property
    def ly(self) -> int:
        return self.Ly if self.basis == "mixed" else 1

    def rng(self, i: int) -> np.random.Generator:
        """Generator of site i (0 <= i < n) or of theta (i = n)."""
        child = np.random.SeedSequence(self.seed).spawn(self.n + 1)[i]
        return np.random.default_rng(child)

    def site_tensor(self, i: int) -> dict:
        """Left isometry for i < j, right isometry for i > j + 1."""
        if i < self.j:
            return left_isometry(self.rng(i), self.bonds[i], self.bonds[i + 1], self.qsite[i], self.ly,
                                 self.real)
        if i > self.j + 1:
            return right_isometry(self.rng(i), self.bonds[i], self.bonds[i + 1], self.qsite[i], self.ly,
                                  self.real)
        raise ValueError("sites j and j+1 belong to the two-site window")

    def right_canonical_mps(self) -> list:
        """Right isometries on every site (a normalised random state with the target charge)."""
        return [right_isometry(self.rng(i), self.bonds[i], self.bonds[i + 1], self.qsite[i], self.ly,
                               self.real) for i in range(self.n)]

    def theta(self) -> dict:
        j = self.j
        return random_theta(self.rng(self.n), self.bonds[j], self.bonds[j + 2],
                            self.qsite[j], self.qsite[j + 1], self.ly, self.real)


def make_workload(name, Ly, Lx, flux, chi, seed, t=1.0, V=1.0, N_tot=None, K_tot=0,
                  sigma_N=None, basis="mixed", j=None, real=False) -> Workload:
    n = Lx * Ly
    if N_tot is None:
        N_tot = (Lx * Ly) // (2 * flux[1])        # half of the lowest band
    if sigma_N is None:
        sigma_N = sqrt(Ly / 2.0)
    if j is None:
        j = n // 2 - 1
    ly = Ly if basis == "mixed" else 1
    qsite = site_charges(Lx, Ly, basis)
    if real and basis != "mixed":
        raise ValueError("real entries are the eq. rot form of the mixed basis")
    wl = Workload(name, Ly, Lx, tuple(flux), t, V, chi, N_tot, K_tot % ly, sigma_N, seed, basis, j, real=real)
    wl.qsite = qsite
    wl.bonds = bond_sectors(n, qsite, ly, chi, N_tot, K_tot % ly, sigma_N)
    return wl


def centre_workload(name, Ly, chi, seed, basis="mixed", V=1.0, real=False) -> Workload:
    """Centre-bond problem at flux 1/Ly: Lx starts at 2 Ly and doubles until the clipped
    bond dimension at the window reaches 0.95 chi (a dilute cylinder clips the extreme
    particle-number sectors)."""
    Lx = 2 * Ly
    while True:
        wl = make_workload(name, Ly, Lx, (1, Ly), chi, seed, V=V, basis=basis, real=real)
        if sum(wl.bonds[wl.j].values()) >= 0.95 * chi or Lx >= 64 * Ly:
            return wl
        Lx *= 2


PRESETS = {
    # name: (Ly, chi, seed) -- centre-bond problems
    "ly6_chi800": (6, 800, 2),
    "ly8_chi3200": (8, 3200, 3),
    "ly10_chi6000": (10, 6000, 5),
    "ly4_chi200": (4, 200, 12),
    "ly6_chi200": (6, 200, 13),
    "ly8_chi400": (8, 400, 14),
    "ly4_chi64": (4, 64, 11),
    "ly3_chi16": (3, 16, 15),
    "ly8_chi2000": (8, 2000, 16),  # the largest window of the many-window batch
}


def preset(name: str, basis: str = "mixed", real: bool = False) -> Workload:
    """Named centre-bond workloads (see PRESETS); real=True: real entries (eq. rot)."""
    Ly, chi, seed = PRESETS[name]
    return centre_workload(name, Ly, chi, seed, basis=basis, real=real)


@dataclass
class GrowthStart:
    """Seeded start of the infinite-cylinder growth: a left block of one cell (left
    isometries from the vacuum), two cells (right isometries) and a right block of one
    cell (right isometries to the single last sector); the two cells' last bond is their
    first bond with every charge moved by the two cells' charge ``d``."""

    ly: int
    n: int                  # orbitals per cell
    qsite: list             # local charges of the 4 n orbitals
    bonds: list             # 4 n + 1 bonds
    left: list              # n tensors
    cells: list             # 2 n tensors
    right: list             # n tensors
    d: tuple


def growth_start(Ly: int, rings: int, N_cell: int, K_cell: int, chi: int, seed: int,
                 sigma_N: float | None = None, basis: str = "mixed", real: bool = False) -> GrowthStart:
    """Sizes from the bond recipe on a chain of four cells (Ly x 4 rings, charge
    4 (N_cell, K_cell)); bond n and bond 3 n are cut to the sectors they share under the
    move by two cells (the smaller dimension) and the chain is clipped again until both
    agree.  Tensors: one generator per orbital from ``SeedSequence(seed).spawn(4 n)``.
    basis="real": the real-space basis (charges (1, 0), modulus 1; K_cell ignored);
    real=True: real isometries (the real form of eq. rot of the mixed basis)."""
    n, ly = rings * Ly, (Ly if basis == "mixed" else 1)
    if sigma_N is None:
        sigma_N = sqrt(Ly / 2.0)
    qsite = site_charges(4 * rings, Ly, basis)
    d = (2 * N_cell, (2 * K_cell) % ly)
    bonds = bond_sectors(4 * n, qsite, ly, chi, 4 * N_cell, (4 * K_cell) % ly, sigma_N)
    bonds = [dict(b) for b in bonds]
    while True:
        a, b = bonds[n], bonds[3 * n]
        common = {q: min(m, b.get(_add(q, d, ly), 0)) for q, m in a.items()}
        common = {q: m for q, m in common.items() if m > 0}
        moved = {_add(q, d, ly): m for q, m in common.items()}
        moved = {(q[0], q[1]): m for q, m in moved.items()}
        bonds[n], bonds[3 * n] = dict(common), moved
        _clip(bonds, qsite, ly)
        if bonds[n] == common and bonds[3 * n] == moved:
            break
    if not bonds[n]:
        raise ValueError("no sector survives on the cell boundary")
    bonds = [dict(sorted(bd.items())) for bd in bonds]
    kids = np.random.SeedSequence(seed).spawn(4 * n)

    def g(i):
        return np.random.default_rng(kids[i])

    left = [left_isometry(g(i), bonds[i], bonds[i + 1], qsite[i], ly, real) for i in range(n)]
    cells = [right_isometry(g(i), bonds[i], bonds[i + 1], qsite[i], ly, real) for i in range(n, 3 * n)]
    right = [right_isometry(g(i), bonds[i], bonds[i + 1], qsite[i], ly, real) for i in range(3 * n, 4 * n)]
    return GrowthStart(ly, n, qsite, bonds, left, cells, right, d)
