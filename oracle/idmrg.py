"""Infinite-cylinder DMRG by unit-cell growth.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper's runs are (i)DMRG on infinite cylinders (Sec. I, Sec. III A, Fig. 3) on the
finite-state-machine MPO of Sec. IV; it does not restate the infinite algorithm.  This
module uses the infinite-system growth form of DMRG with a unit cell of ``c`` rings
(n = c * Ly orbitals, c a multiple of the magnetic period in x so that the MPO repeats):

* the bulk MPO cell is read off a long finite machine: the state keys of a cell, moved
  by c rings, are the keys of the next cell, and the MPO matrices agree under that
  relabelling (checked); the cell's boundary bond carries the ready state R and the
  final state F;
* the system is [left block] [two cells] [right block]; the blocks enter only through
  their environments, so the two cells are a finite two-site DMRG problem on 2n
  orbitals.  The growth starts from blocks of one cell each holding seeded random
  isometries (environments contracted from the boundary states R and F of eq. MPO),
  not from the bare boundaries: the bond where a block meets the two cells becomes,
  one iteration later, the bond between the new cells, and a single-sector boundary
  there would freeze its charge (a two-site update can only give the middle bond
  sectors that both outer bonds reach, and next to a one-sector bond they reach that
  sector alone);
* one iteration: bring the two cells to right-canonical form (a left pass of splits
  without eigensolves), then ``sweeps`` two-site sweeps; the last one stops at the bond
  between the cells, where theta is split twice (U | S V^H and U S | V^H of one SVD);
  its Lanczos energy is the total energy of the 2 (j + 1) cell cylinder;
* growth: the left cell (left-canonical) joins the left block, the right cell
  (right-canonical) the right block, and the next two cells start from the right
  cell (the Schmidt values at its left) followed by the left cell, moved by two cells;
  moving by two cells adds the two cells' charge to every bond charge (N exactly, k
  modulo Ly), which also moves the right block's environment;
* energy per orbital: (E_j - E_{j-1}) / (2 n).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction

import numpy as np

from . import blocksparse as bs
from .dmrg import split_theta
from .lanczos import lanczos
from .model import Cylinder
from .mpo import F_KEY, R_KEY, build


@dataclass
class MPOCell:
    """Bulk MPO cell: W[i] (D_i, 2, 2, D_{i+1}) for i < n with D_n = D_0 and the same
    state order at both ends; qbond[b] the state charges, qsite the local charges;
    r, f: indices of the ready and final states on the boundary bond."""

    W: list
    qbond: list
    qsite: np.ndarray
    ly: int
    r: int
    f: int

    @property
    def n_sites(self) -> int:
        return len(self.W)


def _moved(key, c: int):
    """The same machine state c rings further right (every family key holds its ring x
    at position 1)."""
    if key in (R_KEY, F_KEY):
        return key
    return (key[0], key[1] + c) + tuple(key[2:])


def bulk_cell(Ly: int, flux: Fraction, t: float, V: float, rings: int, basis: str = "mixed",
              real: bool = False) -> MPOCell:
    """The MPO of ``rings`` rings deep inside a long cylinder (Sec. IV), checked to
    repeat: cell 2 and cell 3 of a 6-cell machine agree under the key shift; real=True:
    the mixed basis in the real form of eq. rot (Sec. IV D)."""
    cyl = Cylinder(Ly, 6 * rings, Fraction(flux), t, V)
    m = build(cyl, basis, real=real)
    n = rings * Ly
    k0 = 2 * n                      # first site of cell 2

    def perm(b_from, b_to, shift):
        idx = {k: j for j, k in enumerate(m.keys[b_to])}
        out = []
        for k in m.keys[b_from]:
            mk = _moved(k, shift)
            if mk not in idx:
                raise AssertionError("MPO state has no counterpart one cell over")
            out.append(idx[mk])
        if len(out) != len(m.keys[b_to]):
            raise AssertionError("MPO bond dimension differs one cell over")
        return np.array(out)

    for i in range(n):               # cell 3 = cell 2 under the relabelling
        pl = perm(k0 + i, k0 + n + i, rings)
        pr = perm(k0 + i + 1, k0 + n + i + 1, rings)
        if not np.allclose(m.W[k0 + n + i][pl][..., pr], m.W[k0 + i], atol=1e-14, rtol=0):
            raise AssertionError(f"MPO does not repeat at cell site {i}")
    # the right boundary bond of cell 2 (= left bond of cell 3) in the order of its left bond
    back = perm(k0, k0 + n, rings)   # state j at bond k0 <-> state back[j] at bond k0 + n
    W = [m.W[k0 + i].copy() for i in range(n)]
    W[-1] = W[-1][..., back]
    qbond = [m.qbond[k0 + i].copy() for i in range(n)] + [m.qbond[k0].copy()]
    keys = m.keys[k0]
    return MPOCell(W, qbond, m.qsite[k0:k0 + n].copy(), m.ly, keys.index(R_KEY), keys.index(F_KEY))


def cell_chain_dense(cell: MPOCell, copies: int) -> np.ndarray:
    """``copies`` cells in a row between the boundary vectors picking R and F, contracted
    to a dense matrix (basis index sum_i s_i 2^i), for tests on tiny cells."""
    Ws = cell.W * copies
    T = Ws[0][cell.r]                 # (2, 2, D)
    dim = 2
    for w in Ws[1:]:
        T = np.einsum("abw,wcdv->cadbv", T, w).reshape(2 * dim, 2 * dim, -1)
        dim *= 2
    return T[:, :, cell.f]


def shift_charge(q, d, ly):
    return (int(q[0] + d[0]), int((q[1] + d[1]) % ly))


def shift_blocks(blocks: dict, d, ly) -> dict:
    """Relabel the bond charges of a site tensor {(qa, s, qb)} or an environment
    {(q', w, q)} by adding d to both."""
    return {(shift_charge(k[0], d, ly), k[1], shift_charge(k[2], d, ly)): v for k, v in blocks.items()}


@dataclass
class IDMRGResult:
    energies: list = field(default_factory=list)      # E_j, total energy of 2 (j + 1) cells
    schmidt: list = field(default_factory=list)       # per iteration: {q(centre): values}
    tensors: list = field(default_factory=list)       # last iteration's two cells
    bonds: list = field(default_factory=list)         # and their 2n + 1 bonds


def block_envs(cell: MPOCell, left: list, right: list, q_end) -> tuple:
    """Environments of a left block (left-canonical tensors from the vacuum, the ready
    state R) and a right block (right-canonical tensors up to the single sector q_end,
    the final state F), one cell each."""
    L = {((0, 0), cell.r, (0, 0)): np.ones((1, 1), dtype=np.complex128)}
    for i, A in enumerate(left):
        L = bs.env_left_update(L, A, cell.W[i])
    q = (int(q_end[0]), int(q_end[1]))
    R = {(q, cell.f, q): np.ones((1, 1), dtype=np.complex128)}
    for i in range(len(right) - 1, -1, -1):
        R = bs.env_right_update(R, right[i], cell.W[i])
    return L, R


def run(cell: MPOCell, init: list, bonds: list, n_iter: int, chi: int, L0: dict, R0: dict, d,
        sweeps: int = 1, max_iter: int = 30, tol_res: float | None = 1e-300,
        cutoff: float = 1e-14) -> IDMRGResult:
    """iDMRG by unit-cell growth from ``init``: 2n site tensors on ``bonds`` (2n + 1 dicts
    {(N, k): dim}) between the left block's environment L0 and the right block's R0
    (right-canonical form is not required); the last bond must be the first moved by
    the two cells' charge d.  The two-site space at a bond is every charge-allowed block
    of its two outer bonds' sectors (the bond lists, kept through every split; a sector
    whose blocks a truncation has emptied in one site tensor still spans the space)."""
    n, ly = cell.n_sites, cell.ly
    W = cell.W + cell.W
    qsite = [tuple(map(tuple, q)) for q in cell.qsite] * 2
    T = [dict(t) for t in init]
    B = [dict(b) for b in bonds]
    if len(B) != 2 * n + 1 or {shift_charge(q, d, ly): m for q, m in B[0].items()} != B[-1]:
        raise ValueError("the last bond of the two cells must be the first moved by d")
    L, R = L0, R0
    res = IDMRGResult()
    N2 = 2 * n
    for it in range(n_iter):
        Ls = [None] * (N2 + 1)
        Rs = [None] * (N2 + 1)
        Ls[0], Rs[N2] = L, R
        def split(i, th, move):
            left, right, sch, disc = split_theta(th, chi, ly, qsite[i], move, cutoff)
            B[i + 1] = {q: len(v) for q, v in sorted(sch.items())}
            return left, right, sch, disc

        # right-canonical form: splits moving left, no eigensolve
        for i in range(N2 - 2, -1, -1):
            th = bs.contract_two_site(T[i], T[i + 1], ly)
            T[i], T[i + 1], _, _ = split(i, th, "left")
            Rs[i + 1] = bs.env_right_update(Rs[i + 2], T[i + 1], W[i + 1])

        def solve(i):
            th = bs.contract_two_site(T[i], T[i + 1], ly)
            keys = bs.theta_keys(B[i], B[i + 2], qsite[i], qsite[i + 1], ly)
            Li, Ri, W1, W2 = Ls[i], Rs[i + 2], W[i], W[i + 1]

            def mv(v):
                return bs.flatten(bs.heff_apply(Li, W1, W2, Ri, bs.unflatten(v, keys)), keys)

            e, vec, _, _, _ = lanczos(mv, bs.flatten(th, keys), max_iter=max_iter, tol_res=tol_res)
            return e, bs.unflatten(vec, keys)

        e = np.inf
        for sweep in range(sweeps):
            for i in range(N2 - 1):
                e, th = solve(i)
                T[i], T[i + 1], _, _ = split(i, th, "right")
                Ls[i + 1] = bs.env_left_update(Ls[i], T[i], W[i])
            stop = n if sweep == sweeps - 1 else 0
            for i in range(N2 - 2, stop - 1, -1):
                e, th = solve(i)
                T[i], T[i + 1], _, _ = split(i, th, "left")
                Rs[i + 1] = bs.env_right_update(Rs[i + 2], T[i + 1], W[i + 1])
        # the bond between the two cells
        e, th = solve(n - 1)
        A, SV, sch, _ = split(n - 1, th, "right")
        _, Bn, _, _ = split_theta(th, chi, ly, qsite[n - 1], "left", cutoff)
        T[n - 1], T[n] = A, SV
        res.energies.append(float(e))
        res.schmidt.append(sch)
        if it + 1 == n_iter:
            break
        L = bs.env_left_update(Ls[n - 1], A, W[n - 1])
        R = shift_blocks(bs.env_right_update(Rs[n + 1], Bn, W[n]), d, ly)
        T = [SV] + T[n + 1:] + [shift_blocks(t, d, ly) for t in T[:n]]
        B = B[n:] + [{shift_charge(q, d, ly): m for q, m in b.items()} for b in B[1:n + 1]]
    res.tensors = T
    res.bonds = B
    return res


def energy_per_orbital(energies: list, n: int) -> list:
    """(E_j - E_{j-1}) / (2 n) for j >= 1."""
    return [(energies[j] - energies[j - 1]) / (2 * n) for j in range(1, len(energies))]
