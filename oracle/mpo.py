"""Matrix product operators from finite-state machines.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Follows Sec. IV A-B (finite-state machines and eq. MPO) and Sec. IV C-D (real-space and
mixed-basis Hofstadter MPOs):

* Every term of the Hamiltonian is one path of a finite-state machine from the "ready"
  state R to the "final" state F.  The transition taken at site i places the local
  operator on site i; R -> R and F -> F place the identity.  Rows and columns of the MPO
  matrix M^[i] are the machine's states at the bonds left and right of site i, and the
  boundary vectors pick R on the left end and F on the right end (eq. MPO).
* A state in the middle of a path is labelled by the term family, the set of the
  term's operators ("roles") already placed and the total charge they carry.  For the
  mixed-basis families the charge includes the momentum modulo Ly, which plays the
  part of the momentum labels of the states A_mu(k), C_mu(k) of Sec. IV D (Fig. 7a):
  the rest of a term only depends on that total, so terms share states.
* Fermion signs (eq. JW, occupation form c_i = prod_{j<i} (-1)^{n_j} a_i): operators
  are placed in chain order; placing role r at a site while an earlier role (in the
  term's written product order) is still unplaced is one exchange of two fermion
  operators and gives a factor -1.  The local operator is the product of the roles
  placed there (in written order) times Z = (-1)^n if an odd number of fermion
  operators of the term are still to come to the right; on a site where the term
  places nothing the machine passes Z or 1 by the same rule.
* States are created only along actual term paths, so every state is reachable from R
  and co-reachable to F (the trimming of Sec. IV D); an explicit reachability pass
  checks this anyway.
* ``deparallelise`` then merges states whose MPO columns (or rows) are proportional.
  This is an exact rewriting, not a truncation.  (The paper trims unreachable states
  only; merging parallel states is an addition here and only lowers D.)

Local basis of every orbital: |0> empty, |1> occupied.  W[w, s', s, w'] = <s'|op|s>.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .model import FERMIONIC, DELTA_N, Term

I2 = np.eye(2, dtype=np.complex128)
Z2 = np.diag([1.0, -1.0]).astype(np.complex128)
OPS = {
    "+": np.array([[0, 0], [1, 0]], dtype=np.complex128),   # c+ : |0> -> |1>
    "-": np.array([[0, 1], [0, 0]], dtype=np.complex128),   # c  : |1> -> |0>
    "n": np.array([[0, 0], [0, 1]], dtype=np.complex128),
}

R_KEY = ("R",)
F_KEY = ("F",)


@dataclass
class MPO:
    """Open-boundary MPO; W[i] has shape (D_i, 2, 2, D_{i+1}); bond 0 and bond n hold one
    state (R and F).  qbond[b][w] = (N, k) charge placed by the operator string left of
    bond b in state w; qsite[i] = [(0, 0), (1, m_i)] charges of the local states."""

    W: list
    qbond: list
    qsite: np.ndarray
    ly: int
    keys: list

    @property
    def n_sites(self) -> int:
        return len(self.W)

    def bond_dims(self) -> list[int]:
        return [w.shape[0] for w in self.W] + [self.W[-1].shape[3]]


def _state_key(term: Term, placed: frozenset, dN: int, dk: int):
    mask = sum(1 << r for r in placed)
    return term.fam + (mask, dN, dk % term.ly)


def _register(table: dict, kin, kid, kout, mat):
    if kid in table.get(kin, {}):
        old = table[kin][kid][1]
        if not np.allclose(old, mat, atol=1e-13, rtol=0):
            raise AssertionError(f"inconsistent transition {kin} -> {kout}")
        return
    table.setdefault(kin, {})[kid] = (kout, mat)


def fsm_mpo(n_sites: int, terms: list[Term], momenta, ly: int) -> MPO:
    """Build the MPO of sum(terms) by the finite-state machine of Sec. IV."""
    trans = [dict() for _ in range(n_sites)]   # per site: {kin: {kid: (kout, matrix)}}
    for term in terms:
        roles = range(len(term.ops))
        sites = [s for s, _ in term.ops]
        kinds = [k for _, k in term.ops]
        ferm = [FERMIONIC[k] for k in kinds]
        placed: frozenset = frozenset()
        dN = dk = 0
        key = R_KEY
        for i in range(min(sites), max(sites) + 1):
            here = [r for r in roles if sites[r] == i]
            if not here:
                unplaced = sum(ferm[r] for r in roles if r not in placed)
                _register(trans[i], key, key, key, Z2 if unplaced % 2 else I2)
                continue
            after = placed | frozenset(here)
            op = I2.copy()
            for r in here:
                op = op @ OPS[kinds[r]]
            if sum(ferm[r] for r in roles if r not in after) % 2:
                op = op @ Z2
            sign = 1.0
            for r in here:
                if ferm[r] and sum(ferm[rp] for rp in roles if rp < r and rp not in after) % 2:
                    sign = -sign
            coef = sign * (term.fam_coef if not placed else 1.0)
            for r in here:
                coef *= term.role_f[r]
                dN += term.charge[r][0]
                dk += term.charge[r][1]
            if len(after) == len(term.ops):
                if dN != 0 or dk % ly != 0:
                    raise ValueError(f"term {term.fam} does not conserve charge")
                _register(trans[i], key, ("F", term.fam), F_KEY, coef * op)
                key = F_KEY
            else:
                nkey = _state_key(term, after, dN, dk)
                _register(trans[i], key, nkey, nkey, coef * op)
                key = nkey
            placed = after
    for i in range(n_sites):
        _register(trans[i], R_KEY, R_KEY, R_KEY, I2)
        _register(trans[i], F_KEY, F_KEY, F_KEY, I2)

    # reachability from R (left end) and co-reachability to F (right end)
    fwd = [set() for _ in range(n_sites + 1)]
    fwd[0] = {R_KEY}
    for i in range(n_sites):
        for kin in fwd[i]:
            for kout, _ in trans[i].get(kin, {}).values():
                fwd[i + 1].add(kout)
    bwd = [set() for _ in range(n_sites + 1)]
    bwd[n_sites] = {F_KEY}
    for i in range(n_sites - 1, -1, -1):
        for kin, outs in trans[i].items():
            if any(kout in bwd[i + 1] for kout, _ in outs.values()):
                bwd[i].add(kin)
    live = [fwd[b] & bwd[b] for b in range(n_sites + 1)]

    def charge(key):
        if key in (R_KEY, F_KEY):
            return (0, 0)
        return (key[-2], key[-1])

    def order(key):
        rank = 0 if key == R_KEY else (2 if key == F_KEY else 1)
        return (rank, charge(key), repr(key))

    keys = [sorted(live[b], key=order) for b in range(n_sites + 1)]
    index = [{k: j for j, k in enumerate(keys[b])} for b in range(n_sites + 1)]
    W = []
    for i in range(n_sites):
        w = np.zeros((len(keys[i]), 2, 2, len(keys[i + 1])), dtype=np.complex128)
        for kin, outs in trans[i].items():
            if kin not in index[i]:
                continue
            for kout, mat in outs.values():
                if kout in index[i + 1]:
                    w[index[i][kin], :, :, index[i + 1][kout]] += mat
        W.append(w)
    qbond = [np.array([charge(k) for k in keys[b]], dtype=np.int64).reshape(-1, 2)
             for b in range(n_sites + 1)]
    qsite = np.array([[(0, 0), (1, int(momenta[i]) % ly)] for i in range(n_sites)], dtype=np.int64)
    return MPO(W, qbond, qsite, ly, keys)


def _parallel_groups(vecs: np.ndarray, charges: np.ndarray, protect: set):
    """For each vector j return (k, lam) with vecs[j] = lam * vecs[k] for the first such
    earlier k of equal charge, or None.  Zero vectors map to (-1, 0)."""
    out = []
    seen: dict = {}
    for j, v in enumerate(vecs):
        nz = np.flatnonzero(np.abs(v) > 1e-14)
        if len(nz) == 0:
            out.append((-1, 0.0))
            continue
        p = nz[0]
        u = v / v[p]
        sig = (tuple(charges[j]), tuple(nz), tuple(np.round(u[nz], 9)))
        hit = None
        if j not in protect:
            for k in seen.get(sig, []):
                lam = v[p] / vecs[k][p]
                if np.allclose(v, lam * vecs[k], atol=1e-13 * np.abs(v).max(), rtol=0):
                    hit = (k, lam)
                    break
        if hit is None:
            seen.setdefault(sig, []).append(j)
        out.append(hit)
    return out


def deparallelise(mpo: MPO, max_rounds: int = 50) -> MPO:
    """Merge proportional MPO states (exact).  Columns of W[i] proportional to an earlier
    column: w_j = lam w_k  =>  drop j and add lam * row j of W[i+1] to row k.  Rows of
    W[i] proportional to an earlier row are merged the mirrored way.  R and F are kept."""
    W = [w.copy() for w in mpo.W]
    q = [c.copy() for c in mpo.qbond]
    keys = [list(k) for k in mpo.keys]
    n = len(W)
    for _ in range(max_rounds):
        changed = False
        for i in range(n - 1):          # columns of W[i] = states at bond i+1
            A, B = W[i], W[i + 1]
            prot = {j for j, k in enumerate(keys[i + 1]) if k in (R_KEY, F_KEY)}
            groups = _parallel_groups(np.moveaxis(A, 3, 0).reshape(A.shape[3], -1), q[i + 1], prot)
            keep = []
            for j, g in enumerate(groups):
                if g is None:
                    keep.append(j)
                elif g[0] >= 0:
                    B[g[0]] += g[1] * B[j]
                    changed = True
                else:
                    changed = True
            W[i], W[i + 1] = A[..., keep], B[keep]
            q[i + 1] = q[i + 1][keep]
            keys[i + 1] = [keys[i + 1][j] for j in keep]
        for i in range(n - 1, 0, -1):   # rows of W[i] = states at bond i
            A, B = W[i - 1], W[i]
            prot = {j for j, k in enumerate(keys[i]) if k in (R_KEY, F_KEY)}
            groups = _parallel_groups(B.reshape(B.shape[0], -1), q[i], prot)
            keep = []
            for j, g in enumerate(groups):
                if g is None:
                    keep.append(j)
                elif g[0] >= 0:
                    A[..., g[0]] += g[1] * A[..., j]
                    changed = True
                else:
                    changed = True
            W[i - 1], W[i] = A[..., keep], B[keep]
            q[i] = q[i][keep]
            keys[i] = [keys[i][j] for j in keep]
        if not changed:
            break
    return MPO(W, q, mpo.qsite.copy(), mpo.ly, keys)


def _branch_partner(key):
    """The state of the other phase branch with the same roles and charge, or None.
    Only the intra-ring family carries a branch: key = ("intra", x, s, mask, dN, dk)."""
    if len(key) == 6 and key[0] == "intra":
        return ("intra", key[1], -key[2]) + key[3:]
    return None


def rotate_real(mpo: MPO) -> MPO:
    """Eq. rot: rewrite the complex phases of the mixed-basis MPO with real arithmetic.

    The two branches s = +-1 of the intra-ring term carry conjugate phases e^{+-i alpha}
    and are otherwise the same, so at every bond conj(W) = P W P, where P swaps each
    branch pair (p, m) and fixes every other state.  With the bond basis change T that
    maps a pair to ((e_p + e_m) / sqrt2, i (e_p - e_m) / sqrt2) (conj(T) = P T), the
    rotated W'[i] = T_i^{-1} W[i] T_{i+1} obeys conj(W') = W', i.e. it is real; this is
    the similarity of eq. rot written per pair (diag(e^{i a}, e^{-i a}) becomes the
    rotation by a).  The bond dimension and the states' charges are unchanged (a pair
    shares its charge).  Applied to the finite-state machine's MPO (with state keys)."""
    n = mpo.n_sites
    pairs = []  # per bond: (p, m) index pairs
    for b in range(n + 1):
        keys = mpo.keys[b]
        idx = {k: j for j, k in enumerate(keys)}
        pb = []
        for j, k in enumerate(keys):
            q = _branch_partner(k)
            if q is None or k[2] != 1:
                continue
            m = idx.get(q)
            if m is None:
                raise AssertionError(f"branch state {k} has no partner at bond {b}")
            pb.append((j, m))
        pairs.append(np.array(pb, dtype=np.int64).reshape(-1, 2))
    # T is the identity outside the pair blocks [[1, i], [1, -i]] / sqrt2 (columns: the
    # new states p', m' in the old basis); T^{-1} on a pair is [[1, 1], [-i, i]] / sqrt2
    r2 = 1 / np.sqrt(2)
    W = []
    for i in range(n):
        w = mpo.W[i].copy()
        p, m = pairs[i + 1][:, 0], pairs[i + 1][:, 1]   # columns: W T_{i+1}
        cp, cm = w[..., p].copy(), w[..., m].copy()
        w[..., p] = (cp + cm) * r2
        w[..., m] = 1j * (cp - cm) * r2
        p, m = pairs[i][:, 0], pairs[i][:, 1]           # rows: T_i^{-1} W
        rp, rm = w[p].copy(), w[m].copy()
        w[p] = (rp + rm) * r2
        w[m] = 1j * (rm - rp) * r2
        scale = max(np.abs(w).max(), 1.0)
        if np.abs(w.imag).max() > 1e-12 * scale:
            raise AssertionError(f"rotated MPO not real at site {i}")
        W.append(w.real.astype(np.complex128))
    return MPO(W, [q.copy() for q in mpo.qbond], mpo.qsite.copy(), mpo.ly, [list(k) for k in mpo.keys])


def build(cyl, basis: str, merge: bool = True, real: bool = False) -> MPO:
    """Hofstadter MPO of eq. H_real ("real") or eqs. H_kin + H_int ("mixed"); with real=True
    (mixed basis) the phases rewritten by eq. rot, so every entry is real."""
    from .model import terms_for, orbital_momenta
    ly = cyl.Ly if basis == "mixed" else 1
    m = fsm_mpo(cyl.n_orb, terms_for(cyl, basis), orbital_momenta(cyl, basis), ly)
    if real:
        if basis != "mixed":
            raise ValueError("eq. rot applies to the mixed basis")
        m = rotate_real(m)
    return deparallelise(m) if merge else m


def to_dense(mpo: MPO) -> np.ndarray:
    """Contract eq. MPO to a dense 2^n x 2^n matrix, basis index sum_i s_i 2^i."""
    T = mpo.W[0][0]                          # (2, 2, D1): bond 0 holds only R
    dim = 2
    for i in range(1, mpo.n_sites):
        T = np.einsum("abw,wcdv->cadbv", T, mpo.W[i]).reshape(2 * dim, 2 * dim, -1)
        dim *= 2
    return T[:, :, 0]                        # bond n holds only F


def check_charges(mpo: MPO) -> None:
    """Every nonzero W[w, s', s, w'] obeys q(w') = q(w) + q(s') - q(s) (N exact, k mod ly)."""
    for i, w in enumerate(mpo.W):
        for a, sp_, s, b in zip(*np.nonzero(np.abs(w) > 0)):
            lhs = mpo.qbond[i + 1][b]
            rhs = mpo.qbond[i][a] + mpo.qsite[i][sp_] - mpo.qsite[i][s]
            if lhs[0] != rhs[0] or (lhs[1] - rhs[1]) % mpo.ly:
                raise AssertionError(f"charge rule broken at site {i}")
