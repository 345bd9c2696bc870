"""ctypes marshalling for libmrdmrg.so (no arithmetic of the method lives here)."""
from __future__ import annotations

import ctypes as C
import os
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmrdmrg.so")

DM_FP64, DM_FP32, DM_BF16X3 = 0, 1, 2
DM_REAL = 16  # OR'ed into DM_FP64 / DM_FP32 / DM_BF16X3: real (float64) operands, the eq. rot form
LAYOUT_SITE, LAYOUT_THETA, LAYOUT_ENV_L, LAYOUT_ENV_R = 0, 1, 2, 3
# error codes of include/mrdmrg.h
DM_OK, DM_ERR_ARG, DM_ERR_CHARGE, DM_ERR_DIM, DM_ERR_LAYOUT = 0, -1, -2, -3, -4
DM_ERR_DTYPE, DM_ERR_ALLOC, DM_ERR_HIP, DM_ERR_NONFINITE = -5, -6, -7, -8


class LibraryError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mrdmrg error {code}: {msg}")
        self.code = code


if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is missing: build it with `python paper_1512_03318_amd/build.py`")
# One HIP runtime per process.  PyTorch ships its own copies of the HIP and HSA runtimes;
# loaded before PyTorch, the library would bind the system copies and PyTorch would then
# load a second pair beside them (two runtimes share neither device memory nor pinned
# allocations).  Importing PyTorch first makes the library bind the copies it loaded.
try:
    import torch  # noqa: F401
except ImportError:
    pass
lib = C.CDLL(_LIB_PATH)


class DmCharge(C.Structure):
    _fields_ = [("n", C.c_int32), ("k", C.c_int32)]


class DmBond(C.Structure):
    _fields_ = [("nsec", C.c_int32), ("q", C.POINTER(DmCharge)), ("dim", C.POINTER(C.c_int32))]


class DmMpoSite(C.Structure):
    _fields_ = [("dl", C.c_int32), ("dr", C.c_int32), ("ql", C.POINTER(DmCharge)),
                ("qr", C.POINTER(DmCharge)), ("qs", DmCharge * 2), ("w", C.POINTER(C.c_double))]


class DmLayoutDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("ly", C.c_int32), ("x", C.POINTER(DmBond)),
                ("y", C.POINTER(DmBond)), ("nw", C.c_int32), ("qw", C.POINTER(DmCharge)),
                ("qs1", DmCharge * 2), ("qs2", DmCharge * 2)]


class DmBlock(C.Structure):
    _fields_ = [("idx", C.c_int32 * 3), ("rows", C.c_int32), ("cols", C.c_int32),
                ("off", C.c_int64), ("ld", C.c_int64)]


_vp = C.c_void_p
_i32, _i64, _f64 = C.c_int32, C.c_int64, C.c_double
_sigs = {
    "dm_layout": (_i32, [C.POINTER(DmLayoutDesc), C.POINTER(_i64), C.POINTER(_i64), C.POINTER(DmBlock)]),
    "dm_heff_plan_create": (_i32, [_i32, C.POINTER(DmBond), C.POINTER(DmBond), C.POINTER(DmMpoSite),
                                   C.POINTER(DmMpoSite), _vp, _vp, _i32, _vp, C.POINTER(_vp)]),
    "dm_heff_plan_destroy": (None, [_vp]),
    "dm_heff_info": (_i32, [_vp, C.POINTER(_i64), C.POINTER(_f64)]),
    "dm_heff_sizes": (_i32, [_vp, C.POINTER(_i64)]),
    "heff_apply": (_i32, [_vp, _vp, _vp, _vp]),
    "lanczos_ground": (_i32, [_vp, _vp, _i32, _f64, C.POINTER(_f64), C.POINTER(_i32), _vp]),
    "env_update_left": (_i32, [_i32, C.POINTER(DmBond), C.POINTER(DmBond), C.POINTER(DmMpoSite),
                               _vp, _vp, _vp, _i32, _vp]),
    "env_update_right": (_i32, [_i32, C.POINTER(DmBond), C.POINTER(DmBond), C.POINTER(DmMpoSite),
                                _vp, _vp, _vp, _i32, _vp]),
    "env_update_left_noalloc": (_i32, [_i32, C.POINTER(DmBond), C.POINTER(DmBond), C.POINTER(DmMpoSite),
                                       _vp, _vp, _vp, _i32, _vp]),
    "dm_batch_create": (_i32, [_i32, C.POINTER(_vp), _vp, C.POINTER(_vp)]),
    "dm_batch_destroy": (None, [_vp]),
    "dm_batch_info": (_i64, [_vp, C.c_char_p, _i64]),
    "lanczos_ground_batched": (_i32, [_vp, C.POINTER(_vp), _i32, _f64, C.POINTER(_f64),
                                      C.POINTER(_i32), C.POINTER(_f64), _vp]),
    "dm_theta_split": (_i32, [_i32, C.POINTER(DmBond), C.POINTER(DmBond), C.POINTER(DmCharge),
                              C.POINTER(DmCharge), _vp, _i32, _f64, _i32, _vp, C.POINTER(_vp)]),
    "dm_split_bond": (_i32, [_vp, C.POINTER(_i32), C.POINTER(DmCharge), C.POINTER(_i32)]),
    "dm_split_tensors": (_i32, [_vp, C.POINTER(_vp), C.POINTER(_i64), C.POINTER(_vp), C.POINTER(_i64)]),
    "dm_split_schmidt": (_i32, [_vp, C.POINTER(_f64), C.POINTER(_f64)]),
    "dm_split_copy": (_i32, [_vp, _vp, _vp, _vp]),
    "dm_split_destroy": (None, [_vp]),
    "dm_mps_create": (_i32, [_i32, _i32, C.POINTER(DmBond), C.POINTER(DmCharge), C.POINTER(_vp), _vp,
                             C.POINTER(_vp)]),
    "dm_mps_destroy": (None, [_vp]),
    "dm_mps_bond": (_i32, [_vp, _i32, C.POINTER(_i32), C.POINTER(DmCharge), C.POINTER(_i32)]),
    "dm_mps_tensor": (_i32, [_vp, _i32, C.POINTER(_vp), C.POINTER(_i64)]),
    "dm_mps_copy": (_i32, [_vp, _i32, _vp, _vp]),
    "dm_mps_schmidt": (_i32, [_vp, _i32, C.POINTER(_f64), C.POINTER(_i64)]),
    "dm_dmrg_sweeps": (_i32, [_vp, C.POINTER(DmMpoSite), _i32, _i32, _i32, _f64, _i32, C.POINTER(_f64), _vp]),
    "dm_idmrg": (_i32, [_vp, C.POINTER(DmMpoSite), DmCharge, _vp, _vp, _i32, _i32, _i32, _i32, _f64, _i32,
                        C.POINTER(_f64), _vp]),
    "dm_entanglement": (_i32, [C.POINTER(_f64), _i64, C.POINTER(_f64), C.POINTER(_f64)]),
    "dm_mpo_hofstadter": (_i32, [_i32, _i32, _i32, _i32, _f64, _f64, _i32, C.POINTER(_vp)]),
    "dm_mpo_n_sites": (_i32, [_vp]),
    "dm_mpo_site_get": (_i32, [_vp, _i32, C.POINTER(DmMpoSite)]),
    "dm_mpo_destroy": (None, [_vp]),
    "dm_heff_profile": (_i32, [_vp, _i32]),
    "dm_heff_profile_read": (_i32, [_vp, C.POINTER(_f64), C.POINTER(_i64)]),
    "dm_env_flops": (_i32, [_i32, _i32, C.POINTER(DmBond), C.POINTER(DmBond), C.POINTER(DmMpoSite),
                            C.POINTER(_f64)]),
    "dm_last_error": (C.c_char_p, []),
}
for _name, (_res, _args) in _sigs.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def _check(code):
    if code != 0:
        raise LibraryError(code, lib.dm_last_error().decode())


def _stream(stream):
    if stream is None:
        import torch
        return _vp(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return _vp(stream)
    return _vp(stream.cuda_stream)


def _ptr(t):
    if t is None:
        return _vp(0)
    return _vp(t.data_ptr())


def _charges(q) -> "C.Array":
    q = np.asarray(q, dtype=np.int32).reshape(-1, 2)
    arr = (DmCharge * max(len(q), 1))()
    for i, (n, k) in enumerate(q):
        arr[i].n, arr[i].k = int(n), int(k)
    return arr


class Bond:
    """A virtual bond: sectors (N, k) in increasing order with dimensions."""

    def __init__(self, sectors: dict):
        items = sorted((tuple(map(int, q)), int(d)) for q, d in sectors.items())
        self.q = [q for q, _ in items]
        self.dim = [d for _, d in items]
        self.index = {q: i for i, q in enumerate(self.q)}
        self._q = _charges(self.q)
        self._dim = (C.c_int32 * max(len(self.dim), 1))(*self.dim)
        self.c = DmBond(len(self.q), self._q, self._dim)

    def __len__(self):
        return len(self.q)


class MpoSite:
    """Host MPO site tensor W[w, s', s, w'] with the charges of its legs."""

    def __init__(self, W, ql, qr, qs):
        self.W = np.ascontiguousarray(np.asarray(W, dtype=np.complex128))
        dl, _, _, dr = self.W.shape
        self._ql, self._qr = _charges(ql), _charges(qr)
        qs = np.asarray(qs, dtype=np.int32).reshape(2, 2)
        self.qs = [tuple(map(int, x)) for x in qs]
        self.ql = [tuple(map(int, x)) for x in np.asarray(ql).reshape(-1, 2)]
        self.qr = [tuple(map(int, x)) for x in np.asarray(qr).reshape(-1, 2)]
        self._w = self.W.view(np.float64).reshape(-1)
        self.c = DmMpoSite(dl, dr, self._ql, self._qr,
                           (DmCharge * 2)(DmCharge(*self.qs[0]), DmCharge(*self.qs[1])),
                           self._w.ctypes.data_as(C.POINTER(C.c_double)))


def layout(kind, ly, x: Bond, y: Bond | None = None, qw=None, qs1=((0, 0), (0, 0)),
           qs2=((0, 0), (0, 0))):
    """Block list of a canonical layout: (structured array of blocks, total elements)."""
    d = DmLayoutDesc()
    d.kind, d.ly = kind, ly
    d.x = C.pointer(x.c)
    d.y = C.pointer(y.c) if y is not None else C.POINTER(DmBond)()
    qwa = _charges(qw if qw is not None else [(0, 0)])
    d.nw = 0 if qw is None else len(qw)
    d.qw = qwa
    d.qs1 = (DmCharge * 2)(DmCharge(*qs1[0]), DmCharge(*qs1[1]))
    d.qs2 = (DmCharge * 2)(DmCharge(*qs2[0]), DmCharge(*qs2[1]))
    nb, ne = _i64(), _i64()
    _check(lib.dm_layout(C.byref(d), C.byref(nb), C.byref(ne), None))
    blocks = (DmBlock * max(nb.value, 1))()
    _check(lib.dm_layout(C.byref(d), C.byref(nb), C.byref(ne), blocks))
    out = [(tuple(b.idx), b.rows, b.cols, b.off, b.ld) for b in blocks[:nb.value]]
    return out, ne.value


def _key_fns(kind, x: Bond, y: Bond | None):
    """Map a block's index triple to the numpy block-dict key used by callers."""
    if kind == LAYOUT_SITE:
        return lambda i: (x.q[i[0]], i[1], y.q[i[2]])
    if kind == LAYOUT_THETA:
        return lambda i: (x.q[i[0]], i[1] >> 1, i[1] & 1, y.q[i[2]])
    return lambda i: (x.q[i[0]], i[1], x.q[i[2]])


def pack(blocks: dict, kind, ly, x: Bond, y: Bond | None = None, **kw) -> np.ndarray:
    """Flat complex128 array in the canonical layout from {key: block} (missing = 0)."""
    lay, n = layout(kind, ly, x, y, **kw)
    flat = np.zeros(n, dtype=np.complex128)
    key = _key_fns(kind, x, y)
    for idx, r, c, off, ld in lay:
        blk = blocks.get(key(idx))
        if blk is None:
            continue
        if blk.shape != (r, c):
            raise ValueError(f"block {key(idx)} has shape {blk.shape}, layout wants {(r, c)}")
        view = np.lib.stride_tricks.as_strided(flat[off:], shape=(r, c), strides=(16 * ld, 16))
        view[...] = blk
    return flat


def unpack(flat: np.ndarray, kind, ly, x: Bond, y: Bond | None = None, **kw) -> dict:
    lay, n = layout(kind, ly, x, y, **kw)
    flat = np.ascontiguousarray(flat)
    key = _key_fns(kind, x, y)
    out = {}
    for idx, r, c, off, ld in lay:
        out[key(idx)] = np.lib.stride_tricks.as_strided(flat[off:], shape=(r, c),
                                                        strides=(16 * ld, 16)).copy()
    return out


class HeffPlan:
    """dm_heff_plan: H_eff of one two-site window (L, W1, W2, R bound at creation)."""

    def __init__(self, ly, a: Bond, c: Bond, w1: MpoSite, w2: MpoSite, L, R, prec=DM_FP64,
                 stream=None):
        self.ly, self.a, self.c, self.w1, self.w2, self.prec = ly, a, c, w1, w2, prec
        h = _vp()
        _check(lib.dm_heff_plan_create(ly, C.byref(a.c), C.byref(c.c), C.byref(w1.c),
                                       C.byref(w2.c), _ptr(L), _ptr(R), prec, _stream(stream),
                                       C.byref(h)))
        self.h = h
        # the destructor keeps its own reference: at interpreter exit the module's
        # globals (``lib``) may already be cleared when this object is collected
        self._destroy = lib.dm_heff_plan_destroy
        n = _i64()
        fl = (_f64 * 3)()
        _check(lib.dm_heff_info(h, C.byref(n), fl))
        self.n = n.value
        self.flops = tuple(fl)
        sz = (_i64 * 5)()
        _check(lib.dm_heff_sizes(h, sz))
        self.sizes = dict(zip(("L", "R", "theta", "X", "Z"), (int(v) for v in sz)))

    def profile(self, enable=True, every=1):
        """Record the stage times of every `every`-th matvec (enable=False: stop)."""
        _check(lib.dm_heff_profile(self.h, int(every) if enable else 0))

    def profile_read(self):
        """(ms per kernel [L.theta GEMM, mixing, (.).R GEMM, K-split reduction] accumulated,
        matvecs recorded)."""
        ms = (_f64 * 4)()
        n = _i64()
        _check(lib.dm_heff_profile_read(self.h, ms, C.byref(n)))
        return list(ms), n.value

    def __del__(self):
        # at interpreter exit the process's device memory goes with it: no library call
        if getattr(self, "h", None) and not sys.is_finalizing():
            self._destroy(self.h)
            self.h = None


def env_flops(left: bool, ly, x: Bond, y: Bond, w: MpoSite) -> float:
    f = _f64()
    _check(lib.dm_env_flops(1 if left else 0, ly, C.byref(x.c), C.byref(y.c), C.byref(w.c), C.byref(f)))
    return f.value


def heff_apply(plan: HeffPlan, theta, theta_out, stream=None):
    _check(lib.heff_apply(plan.h, _ptr(theta), _ptr(theta_out), _stream(stream)))


def lanczos_ground(plan: HeffPlan, theta, max_iter=30, tol=1e-14, stream=None):
    e, k = _f64(), _i32()
    _check(lib.lanczos_ground(plan.h, _ptr(theta), max_iter, tol, C.byref(e), C.byref(k),
                              _stream(stream)))
    return e.value, k.value


def env_update_left(ly, a: Bond, b: Bond, w: MpoSite, L, A, L_out, prec=DM_FP64, stream=None):
    _check(lib.env_update_left(ly, C.byref(a.c), C.byref(b.c), C.byref(w.c), _ptr(L), _ptr(A),
                               _ptr(L_out), prec, _stream(stream)))


def env_update_left_noalloc(ly, a: Bond, b: Bond, w: MpoSite, L, A, L_out, prec=DM_FP64, stream=None):
    _check(lib.env_update_left_noalloc(ly, C.byref(a.c), C.byref(b.c), C.byref(w.c), _ptr(L), _ptr(A),
                                       _ptr(L_out), prec, _stream(stream)))


def env_update_right(ly, b: Bond, c: Bond, w: MpoSite, R, B, R_out, prec=DM_FP64, stream=None):
    _check(lib.env_update_right(ly, C.byref(b.c), C.byref(c.c), C.byref(w.c), _ptr(R), _ptr(B),
                                _ptr(R_out), prec, _stream(stream)))


class Batch:
    """dm_batch: merged task tables of several plans."""

    def __init__(self, plans, stream=None):
        self.plans = list(plans)
        arr = (_vp * len(self.plans))(*[p.h.value for p in self.plans])
        h = _vp()
        _check(lib.dm_batch_create(len(self.plans), arr, _stream(stream), C.byref(h)))
        self.h = h
        self._destroy = lib.dm_batch_destroy

    def info(self) -> str:
        """Tile shape chosen per problem bucket (after the first solve)."""
        n = lib.dm_batch_info(self.h, None, 0)
        buf = C.create_string_buffer(max(1, n))
        lib.dm_batch_info(self.h, buf, len(buf))
        return buf.value.decode()

    def __del__(self):
        # at interpreter exit the process's device memory goes with it: no library call
        if getattr(self, "h", None) and not sys.is_finalizing():
            self._destroy(self.h)
            self.h = None


def lanczos_ground_batched(batch: Batch, thetas, max_iter=30, tol=1e-14, stream=None):
    n = len(batch.plans)
    ptrs = (_vp * n)(*[t.data_ptr() for t in thetas])
    e = (_f64 * n)()
    k = (_i32 * n)()
    us = (_f64 * n)()
    _check(lib.lanczos_ground_batched(batch.h, ptrs, max_iter, tol, e, k, us, _stream(stream)))
    return list(e), list(k), list(us)


class HofstadterMPO:
    """dm_mpo_hofstadter: the library's own MPO of eq. H (basis 'mixed' or 'real'; with
    rot=True the mixed-basis MPO in the real form of eq. rot)."""

    def __init__(self, Ly, Lx, p, q, t=1.0, V=1.0, basis="mixed", rot=False):
        if rot and basis != "mixed":
            raise ValueError("eq. rot applies to the mixed basis")
        code = 2 if rot else (0 if basis == "mixed" else 1)
        h = _vp()
        _check(lib.dm_mpo_hofstadter(Ly, Lx, p, q, t, V, code, C.byref(h)))
        self.h = h
        self._destroy = lib.dm_mpo_destroy
        self.ly = Ly if basis == "mixed" else 1
        self.n_sites = lib.dm_mpo_n_sites(h)

    def site(self, i) -> MpoSite:
        s = DmMpoSite()
        _check(lib.dm_mpo_site_get(self.h, i, C.byref(s)))
        W = np.ctypeslib.as_array(s.w, shape=(s.dl * 4 * s.dr * 2,)).view(np.complex128)
        W = W.reshape(s.dl, 2, 2, s.dr).copy()
        ql = [(s.ql[i].n, s.ql[i].k) for i in range(s.dl)]
        qr = [(s.qr[i].n, s.qr[i].k) for i in range(s.dr)]
        qs = [(s.qs[0].n, s.qs[0].k), (s.qs[1].n, s.qs[1].k)]
        return MpoSite(W, ql, qr, qs)

    def __del__(self):
        # at interpreter exit the process's device memory goes with it: no library call
        if getattr(self, "h", None) and not sys.is_finalizing():
            self._destroy(self.h)
            self.h = None


def _bond_of(getter, *args) -> dict:
    n = _i32()
    _check(getter(*args, C.byref(n), None, None))
    q = (DmCharge * max(n.value, 1))()
    d = (_i32 * max(n.value, 1))()
    _check(getter(*args, C.byref(n), q, d))
    return {(q[i].n, q[i].k): d[i] for i in range(n.value)}


class Split:
    """dm_split: theta split at its middle bond by the block SVD truncation.
    .bond: {(N, k): dim} of the new bond; .left / .right: device complex128 tensors in
    the SITE layouts (copies); .schmidt: kept values; .discarded: discarded weight."""

    def __init__(self, ly, a: Bond, c: Bond, qs1, qs2, theta, chi, cutoff=1e-14, move_right=True,
                 stream=None):
        import torch
        h = _vp()
        q1 = (DmCharge * 2)(DmCharge(*qs1[0]), DmCharge(*qs1[1]))
        q2 = (DmCharge * 2)(DmCharge(*qs2[0]), DmCharge(*qs2[1]))
        _check(lib.dm_theta_split(ly, C.byref(a.c), C.byref(c.c), q1, q2, _ptr(theta), int(chi), float(cutoff),
                                  1 if move_right else 0, _stream(stream), C.byref(h)))
        try:
            self.bond = _bond_of(lib.dm_split_bond, h)
            nl, nr = _i64(), _i64()
            _check(lib.dm_split_tensors(h, None, C.byref(nl), None, C.byref(nr)))
            dev = theta.device
            self.left = torch.empty(nl.value, dtype=torch.complex128, device=dev)
            self.right = torch.empty(nr.value, dtype=torch.complex128, device=dev)
            _check(lib.dm_split_copy(h, _ptr(self.left), _ptr(self.right), _stream(stream)))
            torch.cuda.synchronize(dev)
            vals = (_f64 * max(1, sum(self.bond.values())))()
            disc = _f64()
            _check(lib.dm_split_schmidt(h, vals, C.byref(disc)))
            self.schmidt = np.array(vals[:sum(self.bond.values())])
            self.discarded = disc.value
        finally:
            lib.dm_split_destroy(h)


class MPS:
    """dm_mps: an MPS held by the library (site tensors on the device)."""

    def __init__(self, ly, bonds, qs, tensors, stream=None):
        self.ly, self.n = ly, len(tensors)
        self._bonds = [Bond(b) for b in bonds]
        arr = (DmBond * len(self._bonds))(*[b.c for b in self._bonds])
        q = _charges([x for pair in qs for x in pair])
        ptrs = (_vp * self.n)(*[t.data_ptr() for t in tensors])
        h = _vp()
        _check(lib.dm_mps_create(ly, self.n, arr, q, ptrs, _stream(stream), C.byref(h)))
        self.h = h
        self._destroy = lib.dm_mps_destroy

    def bond(self, i) -> dict:
        return _bond_of(lib.dm_mps_bond, self.h, i)

    def tensor(self, i, device="cuda"):
        import torch
        n = _i64()
        _check(lib.dm_mps_tensor(self.h, i, None, C.byref(n)))
        out = torch.empty(n.value, dtype=torch.complex128, device=device)
        _check(lib.dm_mps_copy(self.h, i, _ptr(out), _stream(None)))
        torch.cuda.synchronize()
        return out

    def schmidt(self, i) -> np.ndarray:
        n = _i64()
        _check(lib.dm_mps_schmidt(self.h, i, None, C.byref(n)))
        vals = (_f64 * max(1, n.value))()
        _check(lib.dm_mps_schmidt(self.h, i, vals, C.byref(n)))
        return np.array(vals[:n.value])

    def __del__(self):
        # at interpreter exit the process's device memory goes with it: no library call
        if getattr(self, "h", None) and not sys.is_finalizing():
            self._destroy(self.h)
            self.h = None


def dmrg_sweeps(psi: MPS, sites, nsweeps, chi, max_iter=30, cutoff=1e-14, prec=DM_FP64, stream=None):
    """Energies after each of nsweeps two-site sweeps (dm_dmrg_sweeps)."""
    arr = (DmMpoSite * len(sites))(*[s.c for s in sites])
    e = (_f64 * nsweeps)()
    _check(lib.dm_dmrg_sweeps(psi.h, arr, nsweeps, chi, max_iter, cutoff, prec, e, _stream(stream)))
    return list(e)


def idmrg(psi: MPS, cell, d, L0, R0, n_iter, chi, sweeps=1, max_iter=30, cutoff=1e-14, prec=DM_FP64,
          stream=None):
    """Energies E_j of n_iter growth iterations (dm_idmrg); psi holds 2 len(cell) orbitals,
    d = charge of the two cells, L0 / R0 device environments of the initial blocks."""
    arr = (DmMpoSite * len(cell))(*[s.c for s in cell])
    e = (_f64 * n_iter)()
    _check(lib.dm_idmrg(psi.h, arr, DmCharge(int(d[0]), int(d[1])), _ptr(L0), _ptr(R0), n_iter, sweeps, chi,
                        max_iter, cutoff, prec, e, _stream(stream)))
    return list(e)


def entanglement(values):
    """(entropy, entanglement energies -2 ln lambda) of one cut's Schmidt values."""
    v = np.ascontiguousarray(values, dtype=np.float64)
    ent = _f64()
    out = np.zeros(max(1, v.size))
    _check(lib.dm_entanglement(v.ctypes.data_as(C.POINTER(C.c_double)), v.size, C.byref(ent),
                               out.ctypes.data_as(C.POINTER(C.c_double))))
    return ent.value, out[:v.size]
