"""Host-side tests of the C ABI (no GPU calls): exports, layouts, validation errors,
and the library's Hofstadter MPO against exact diagonalisation."""
import os
import re
from fractions import Fraction

import numpy as np
import pytest

import paper_1512_03318_amd as pk
import workloads
from oracle import ed, model, mpo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "mrdmrg.h")).read()
    names = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(\w+)\s*\(", hdr, re.M))
    names |= set(re.findall(r"^\s*(?:int|void|const char\*)\s*\n?\s*(\w+)\(", hdr, re.M))
    assert {"heff_apply", "lanczos_ground", "env_update_left", "env_update_right",
            "lanczos_ground_batched", "dm_layout", "dm_heff_plan_create"} <= names
    for n in names:
        assert hasattr(pk.lib, n), n


def test_binding_error_codes_match_header():
    hdr = open(os.path.join(ROOT, "include", "mrdmrg.h")).read()
    codes = dict(re.findall(r"#define (DM_(?:OK|ERR_\w+)) \(?(-?\d+)\)?", hdr))
    assert len(codes) == 9
    for name, v in codes.items():
        assert getattr(pk, name) == int(v), name


def _bonds():
    wl = workloads.preset("ly4_chi64")
    return wl, pk.Bond(wl.bonds[wl.j]), pk.Bond(wl.bonds[wl.j + 2])


def test_theta_layout_covers_buffer_once():
    wl, a, c = _bonds()
    qs1 = [tuple(q) for q in wl.qsite[wl.j]]
    qs2 = [tuple(q) for q in wl.qsite[wl.j + 1]]
    blocks, n = pk.layout(pk.LAYOUT_THETA, wl.ly, a, c, qs1=qs1, qs2=qs2)
    seen = np.zeros(n, dtype=int)
    for idx, r, cc, off, ld in blocks:
        for i in range(r):
            seen[off + i * ld: off + i * ld + cc] += 1
    assert (seen == 1).all()
    th = wl.theta()
    flat = pk.pack(th, pk.LAYOUT_THETA, wl.ly, a, c, qs1=qs1, qs2=qs2)
    back = pk.unpack(flat, pk.LAYOUT_THETA, wl.ly, a, c, qs1=qs1, qs2=qs2)
    assert set(back) == set(th)
    assert all(np.array_equal(back[k], th[k]) for k in th)


def test_layouts_with_a_wide_charge_range():
    """Sector lookup over a wide range of N (a sector 10^6 particles away: the library's
    sorted-search path instead of its dense table) gives the same blocks for the original
    sectors; the far sector only adds its own blocks after them."""
    wl, a, c = _bonds()
    qs1 = [tuple(q) for q in wl.qsite[wl.j]]
    qs2 = [tuple(q) for q in wl.qsite[wl.j + 1]]
    far = (max(q[0] for q in wl.bonds[wl.j + 2]) + 10**6, 0)
    a_w = pk.Bond({**wl.bonds[wl.j], far: 2})
    c_w = pk.Bond({**wl.bonds[wl.j + 2], far: 3})
    m = mpo.build(model.Cylinder(wl.Ly, wl.Lx, Fraction(*wl.flux), 1.0, 1.0), "mixed")
    for kind, args, kw in ((pk.LAYOUT_THETA, (a, c), dict(qs1=qs1, qs2=qs2)),
                           (pk.LAYOUT_THETA, (a_w, c_w), dict(qs1=qs1, qs2=qs2)),
                           (pk.LAYOUT_ENV_L, (a,), dict(qw=m.qbond[wl.j])),
                           (pk.LAYOUT_ENV_L, (a_w,), dict(qw=m.qbond[wl.j]))):
        if args[0] is a:
            ref, nref = pk.layout(kind, wl.ly, *args, **kw)
            continue
        got, n = pk.layout(kind, wl.ly, *args, **kw)
        assert got[:len(ref)] == ref
        extra = got[len(ref):]
        assert extra and n > nref
        far_idx = len(wl.bonds[wl.j])  # the far sector sorts last in a_w (and in c_w)
        assert all(b[0][0] == far_idx for b in extra)


@pytest.mark.parametrize("kind", [pk.LAYOUT_ENV_L, pk.LAYOUT_ENV_R])
def test_env_layout_covers_buffer_once(kind):
    wl, a, c = _bonds()
    m = mpo.build(model.Cylinder(wl.Ly, wl.Lx, Fraction(*wl.flux), 1.0, 1.0), "mixed")
    qw = m.qbond[wl.j]
    blocks, n = pk.layout(kind, wl.ly, a, qw=qw)
    seen = np.zeros(n, dtype=int)
    for idx, r, cc, off, ld in blocks:
        qa = np.array(a.q[idx[0]]) if kind == pk.LAYOUT_ENV_L else np.array(a.q[idx[0]])
        for i in range(r):
            seen[off + i * ld: off + i * ld + cc] += 1
        # charge rule q(bra) = q(ket) + q(w)
        bra, ket = np.array(a.q[idx[0]]), np.array(a.q[idx[2]])
        if kind == pk.LAYOUT_ENV_R:
            bra, ket = np.array(a.q[idx[0]]), np.array(a.q[idx[2]])
        d = bra - ket - np.array(qw[idx[1]])
        assert d[0] == 0 and d[1] % wl.ly == 0
    assert (seen == 1).all()


def test_bad_inputs_return_error_codes():
    with pytest.raises(pk.LibraryError) as e:
        pk.Bond({(0, 5): 3})  # k outside [0, ly) is detected when used
        pk.layout(pk.LAYOUT_SITE, 4, pk.Bond({(0, 5): 3}), pk.Bond({(0, 0): 1}))
    assert e.value.code == -2
    with pytest.raises(pk.LibraryError) as e:
        pk.layout(pk.LAYOUT_SITE, 4, pk.Bond({(0, 0): 0}), pk.Bond({(0, 0): 1}))
    assert e.value.code == -3
    # MPO entry that breaks the charge rule
    W = np.zeros((1, 2, 2, 1), complex)
    W[0, 1, 0, 0] = 1.0          # |0> -> |1> but q(w') = q(w)
    bad = pk.MpoSite(W, [(0, 0)], [(0, 0)], [(0, 0), (1, 1)])
    b = pk.Bond({(0, 0): 1})
    with pytest.raises(pk.LibraryError) as e:
        pk.env_update_left(4, b, b, bad, None, None, None, stream=0)
    assert e.value.code == -2


def _dense(m):
    T = m.site(0).W[0]
    dim = 2
    for i in range(1, m.n_sites):
        T = np.einsum("abw,wcdv->cadbv", T, m.site(i).W).reshape(2 * dim, 2 * dim, -1)
        dim *= 2
    return T[:, :, 0]


@pytest.mark.parametrize("Lx,Ly", [(2, 4), (3, 3), (2, 5)])
@pytest.mark.parametrize("basis", ["mixed", "real"])
def test_library_mpo_equals_hamiltonian(Lx, Ly, basis):
    cyl = model.Cylinder(Ly, Lx, Fraction(1, Ly), 1.0, 1.0)
    H = ed.hamiltonian(model.terms_for(cyl, basis), ed.sector_basis(cyl.n_orb)).toarray()
    m = pk.HofstadterMPO(Ly, Lx, 1, Ly, 1.0, 1.0, basis)
    assert np.abs(_dense(m) - H).max() < 1e-12
    dims = [m.site(i).W.shape[0] for i in range(m.n_sites)] + [1]
    assert dims == mpo.build(cyl, basis).bond_dims()


def test_library_mpo_real_space_bond_dimension():
    for L in (3, 4, 6):
        m = pk.HofstadterMPO(L, 4, 1, L, 1.0, 1.0, "real")
        dims = [m.site(i).W.shape[0] for i in range(m.n_sites)]
        assert all(d == 3 * L + 2 for d in dims[L + 1: 3 * L])
