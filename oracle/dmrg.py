"""Finite two-site DMRG with block-wise SVD truncation.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper runs (i)DMRG on the mixed-basis MPO (Sec. I, Sec. III A) and reads Schmidt
values off the decomposition at a cut (Sec. III C: |psi> = sum lambda_a |a>_L |a>_R,
entanglement energies -2 ln lambda_a, each Schmidt state labelled by (N, k)).  The
sweep schedule itself is not given; this module uses the textbook finite two-site
algorithm:

* start from a right-canonical MPS with the target (N, K) (a seeded random state: a
  product state cannot move a particle between orbitals of different momentum in a
  two-site update, since the kinetic term only couples equal momenta one ring apart);
* sweep left to right and back; at bond (i, i+1) form theta = M_i M_{i+1}, replace it
  by the lowest Lanczos eigenvector of H_eff, split it by an SVD per charge block of
  the middle bond, keep the globally largest chi singular values (ties broken by
  (sector, index)), drop values below ``cutoff``, renormalise, and update the
  environment on the side the sweep leaves behind;
* in all stages but the last, a small random admixture (weight ``noise``, drawn from
  a generator passed in by the caller) is added to theta before the split so that
  charge sectors emptied by an early truncation can be repopulated (the standard
  remedy for two-site DMRG with long-range couplings); the last stage has none;
* repeat sweeps until the energy changes by less than ``tol_e``.
"""
from __future__ import annotations

from collections import defaultdict
from dataclasses import dataclass, field

import numpy as np

from . import blocksparse as bs
from .lanczos import lanczos


def product_state(occ: list[int], qsite, ly: int):
    """MPS tensors {(qa, s, qb): [[1]]} and bonds of the product state with occupations occ."""
    tensors, bonds = [], [{(0, 0): 1}]
    q = (0, 0)
    for i, s in enumerate(occ):
        qn = bs.qadd(q, qsite[i][s], ly)
        tensors.append({(q, s, qn): np.ones((1, 1), dtype=np.complex128)})
        bonds.append({qn: 1})
        q = qn
    return tensors, bonds


def split_theta(theta: dict, chi: int, ly: int, qs1, move: str, cutoff: float = 1e-14):
    """SVD of theta[(a s1), (s2 c)] per middle charge q(b) = q(a) + q(s1).

    move='right': returns (A = U, M = S V^H); move='left': (M = U S, B = V^H).
    Also returns the kept Schmidt values per sector and the discarded weight."""
    rows, cols = defaultdict(dict), defaultdict(dict)
    for (qa, s1, s2, qc), blk in theta.items():
        qb = bs.qadd(qa, qs1[s1], ly)
        rows[qb][(qa, s1)] = blk.shape[0]
        cols[qb][(s2, qc)] = blk.shape[1]
    svd = {}
    cand = []
    for qb in sorted(rows):
        rk = sorted(rows[qb])
        ck = sorted(cols[qb])
        roff, r0 = {}, 0
        for k in rk:
            roff[k] = r0
            r0 += rows[qb][k]
        coff, c0 = {}, 0
        for k in ck:
            coff[k] = c0
            c0 += cols[qb][k]
        M = np.zeros((r0, c0), dtype=np.complex128)
        for (qa, s1, s2, qc), blk in theta.items():
            if bs.qadd(qa, qs1[s1], ly) != qb:
                continue
            i, j = roff[(qa, s1)], coff[(s2, qc)]
            M[i:i + blk.shape[0], j:j + blk.shape[1]] = blk
        u, s, vh = np.linalg.svd(M, full_matrices=False)
        svd[qb] = (u, s, vh, roff, coff, rows[qb], cols[qb])
        cand.extend((-float(v), qb, idx) for idx, v in enumerate(s))
    cand.sort()
    total = sum(c[0] ** 2 for c in cand)
    kept = [c for c in cand[:chi] if -c[0] > cutoff]
    keep_n = defaultdict(int)
    for _, qb, idx in kept:
        keep_n[qb] = max(keep_n[qb], idx + 1)
    norm = np.sqrt(sum(c[0] ** 2 for c in kept))
    discarded = max(0.0, 1.0 - sum(c[0] ** 2 for c in kept) / total)
    left, right, schmidt = {}, {}, {}
    for qb, k in keep_n.items():
        u, s, vh, roff, coff, rdim, cdim = svd[qb]
        u, s, vh = u[:, :k], s[:k] / norm, vh[:k]
        schmidt[qb] = s
        lu = u * s[None, :] if move == "left" else u
        rv = vh if move == "left" else s[:, None] * vh
        for (qa, s1), m in rdim.items():
            left[(qa, s1, qb)] = lu[roff[(qa, s1)]:roff[(qa, s1)] + m].copy()
        for (s2, qc), m in cdim.items():
            right[(qb, s2, qc)] = rv[:, coff[(s2, qc)]:coff[(s2, qc)] + m].copy()
    return left, right, schmidt, discarded


@dataclass
class DMRGResult:
    energy: float
    energies: list = field(default_factory=list)
    schmidt: dict = field(default_factory=dict)
    max_discarded: float = 0.0
    tensors: list = field(default_factory=list)


def run(mpo, init: list, chis: list[int], ly: int, sweeps_per_chi: int = 4,
        tol_e: float = 1e-10, max_iter: int = 30, tol_res: float = 1e-10,
        cutoff: float = 1e-14, noise: float = 1e-3, rng=None, capture=None) -> DMRGResult:
    """Two-site DMRG from a right-canonical initial MPS ``init`` (list of block dicts).
    ``chis`` is the bond-dimension schedule, one entry per stage; the last stage sweeps
    until convergence (at most 4 * sweeps_per_chi sweeps).  ``capture``, if given, is
    called before each two-site eigensolve with the bond problem
    (i, L, R, theta, keys, left bond dims, right bond dims); it does not change the run."""
    n = mpo.n_sites
    qsite = [tuple(map(tuple, q)) for q in mpo.qsite]
    M = [dict(t) for t in init]
    qtot = next(iter(M[-1]))[2]
    # bond lists: the two-site space at a bond is every charge-allowed block of its outer
    # bonds' sectors, kept through the splits (a sector a truncation has emptied in one
    # site tensor still spans the space)
    B = [_left_dims(M[0])] + [{**_right_dims(M[i]), **(_left_dims(M[i + 1]) if i + 1 < n else {})}
                              for i in range(n)]
    Ls = [None] * (n + 1)
    Rs = [None] * (n + 1)
    Ls[0] = bs.left_boundary()
    Rs[n] = bs.right_boundary(qtot)
    for i in range(n - 1, 1, -1):
        Rs[i] = bs.env_right_update(Rs[i + 1], M[i], mpo.W[i])
    res = DMRGResult(energy=np.inf)
    prev = np.inf
    sched = [(c, sweeps_per_chi, noise) for c in chis[:-1]] + [(chis[-1], 4 * sweeps_per_chi, 0.0)]
    if rng is None:
        sched = [(c, k, 0.0) for c, k, _ in sched]
    e = np.inf
    for stage, (chi, nsweeps, eps) in enumerate(sched):
        for sweep in range(nsweeps):
            for direction in ("right", "left"):
                bonds = range(n - 1) if direction == "right" else range(n - 2, -1, -1)
                for i in bonds:
                    theta = bs.contract_two_site(M[i], M[i + 1], ly)
                    keys = bs.theta_keys(B[i], B[i + 2], qsite[i], qsite[i + 1], ly)
                    L, R = Ls[i], Rs[i + 2]
                    W1, W2 = mpo.W[i], mpo.W[i + 1]

                    def mv(v, L=L, R=R, W1=W1, W2=W2, keys=keys):
                        return bs.flatten(bs.heff_apply(L, W1, W2, R, bs.unflatten(v, keys)), keys)

                    if capture is not None:
                        capture(i, L, R, theta, keys, dict(B[i]), dict(B[i + 2]))

                    e, vec, _, _, _ = lanczos(mv, bs.flatten(theta, keys), max_iter=max_iter,
                                              tol_res=tol_res)
                    if eps > 0:
                        g = rng.standard_normal(len(vec)) + 1j * rng.standard_normal(len(vec))
                        vec = vec + eps * g / np.linalg.norm(g)
                    theta = bs.unflatten(vec, keys)
                    move = "right" if direction == "right" else "left"
                    left, right, sch, disc = split_theta(theta, chi, ly, qsite[i], move, cutoff)
                    B[i + 1] = {q: len(v) for q, v in sorted(sch.items())}
                    res.max_discarded = max(res.max_discarded, disc)
                    M[i], M[i + 1] = left, right
                    if direction == "right":
                        Ls[i + 1] = bs.env_left_update(Ls[i], M[i], mpo.W[i])
                    else:
                        Rs[i + 1] = bs.env_right_update(Rs[i + 2], M[i + 1], mpo.W[i + 1])
                    if i == n // 2 - 1:
                        res.schmidt = sch
            res.energies.append(e)
            if abs(e - prev) < tol_e and stage == len(sched) - 1:
                res.energy = e
                res.tensors = M
                return res
            prev = e
    res.energy = e
    res.tensors = M
    return res


def _left_dims(A: dict) -> dict:
    return {k[0]: v.shape[0] for k, v in A.items()}


def _right_dims(B: dict) -> dict:
    return {k[2]: v.shape[1] for k, v in B.items()}
