"""Batched Lanczos: many windows of different shape in one set of launches.

With the plans' own tile shapes (tuning off) each instance of a batch runs exactly the
arithmetic of its single-plan solve (same kernels per tile, same fixed-order
reductions): energies, step counts and Ritz vectors equal the single-plan results bit
for bit.  With the tuned shapes (default) the block GEMMs may sum in another order:
results agree to the precision's rounding.  Both match the FP64 oracle's Lanczos."""
import sys
import time

import numpy as np
import pytest

from oracle import blocksparse as bs
from oracle import lanczos as olz

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1512_03318_amd as pk  # noqa: E402
from gpu_helpers import WindowGPU, problem, to_dev  # noqa: E402

NAMES = ["ly3_chi16", "ly4_chi64", "ly6_chi200", "ly4_chi64", "ly3_chi16"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def starts(name, seed):
    wl, L, W1, W2, R, th, keys, mpo = problem(name)
    rng = np.random.default_rng(seed)
    v = bs.flatten(th, keys)
    return v + 0.3 * (rng.standard_normal(v.size) + 1j * rng.standard_normal(v.size))


# matvec tolerance of each precision (relative to the largest element)
TOL = {pk.DM_FP64: 1e-12, pk.DM_FP32: 2e-5, pk.DM_BF16X3: 1e-4}


@pytest.mark.parametrize("tuned", [False, True])
@pytest.mark.parametrize("prec", [pk.DM_FP64, pk.DM_FP32, pk.DM_BF16X3])
def test_batched_equals_single(prec, tuned, monkeypatch):
    say(f"batched vs single prec={prec} tuned={tuned}")
    monkeypatch.setenv("MRDMRG_TUNE", "1" if tuned else "0")
    gs, plans, x0 = [], [], []
    for i, name in enumerate(NAMES):
        wl, L, W1, W2, R, th, keys, mpo = problem(name)
        g = WindowGPU(wl, L, R, mpo)
        gs.append((g, keys))
        plans.append(g.plan(prec))
        x0.append(to_dev(g.pack_theta(bs.unflatten(starts(name, 10 + i), keys))))
    batch = pk.Batch(plans)
    for rep in range(2):
        xb = [x.clone() for x in x0]
        t0 = time.perf_counter()
        eb, kb, us = pk.lanczos_ground_batched(batch, xb, 30, 1e-14)
        wall_us = 1e6 * (time.perf_counter() - t0)
        for i, p in enumerate(plans):
            xs = x0[i].clone()
            es, ks = pk.lanczos_ground(p, xs, 30, 1e-14)
            assert kb[i] == ks, (rep, i)
            # untuned batches run the single plans' kernels and tiles, so FP64 and FP32
            # results are the same bit for bit; a BF16x3 plan's own matvec runs on
            # pre-split operands (stream-K order), the batch on FP32 operands
            if tuned or prec == pk.DM_BF16X3:
                assert abs(eb[i] - es) <= 100 * TOL[prec] * abs(es), (rep, i, eb[i], es)
                assert 1 - abs(complex(torch.vdot(xb[i], xs))) <= 100 * TOL[prec], (rep, i)
            else:
                assert eb[i] == es, (rep, i, eb[i], es)
                assert torch.equal(xb[i], xs)
            assert 0 < us[i] <= wall_us
    if tuned:
        say(batch.info())
        assert batch.info().count("bucket") >= 2
    if prec == pk.DM_FP64:
        for i, name in enumerate(NAMES):
            wl, L, W1, W2, R, th, keys, mpo = problem(name)
            mv = lambda v: bs.flatten(bs.heff_apply(L, W1, W2, R, bs.unflatten(v, keys)), keys)
            eo, vo, ko, _, _ = olz.lanczos(mv, starts(name, 10 + i), max_iter=30)
            assert kb[i] == ko and abs(eb[i] - eo) <= 1e-10 * abs(eo)


def test_batch_rejects_mixed_precision_and_repeats():
    wl, L, W1, W2, R, th, keys, mpo = problem("ly3_chi16")
    g = WindowGPU(wl, L, R, mpo)
    p64, p32 = g.plan(pk.DM_FP64), g.plan(pk.DM_FP32)
    with pytest.raises(pk.LibraryError):
        pk.Batch([p64, p32])
    with pytest.raises(pk.LibraryError):
        pk.Batch([p64, p64])


# The many-window workload spans Ly in {4, 6, 8} and chi in [200, 2000]: one batch with
# its largest window (Ly=8, chi=2000) beside small and mid-size ones, in the batched
# workload's precision (FP32) and in FP64, tuned tiles, against the oracle's 30-step
# Lanczos from the same start vectors.
SCALE_NAMES = ["ly8_chi2000", "ly4_chi200", "ly6_chi800", "ly3_chi16", "ly6_chi200"]
SCALE_TOL = {pk.DM_FP64: 1e-10, pk.DM_FP32: 1e-6}
_oracle_runs = {}


def oracle_run(name, seed):
    if (name, seed) not in _oracle_runs:
        wl, L, W1, W2, R, th, keys, mpo = problem(name)
        mv = lambda v: bs.flatten(bs.heff_apply(L, W1, W2, R, bs.unflatten(v, keys)), keys)
        t0 = time.perf_counter()
        eo, vo, ko, _, _ = olz.lanczos(mv, starts(name, seed), max_iter=30)
        say(f"  oracle Lanczos {name}: {ko} steps, {time.perf_counter() - t0:.1f} s")
        _oracle_runs[(name, seed)] = (eo, vo, ko)
    return _oracle_runs[(name, seed)]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", [pk.DM_FP32, pk.DM_FP64])
def test_batched_at_many_window_scale(prec, monkeypatch):
    monkeypatch.setenv("MRDMRG_TUNE", "1")
    say(f"batched at scale prec={prec}: building the windows with the oracle ...")
    gs, plans, x0 = [], [], []
    for i, name in enumerate(SCALE_NAMES):
        wl, L, W1, W2, R, th, keys, mpo = problem(name)
        say(f"  {name}: chi={sum(wl.bonds[wl.j].values())} n={sum(m * n for _, (m, n) in keys)}")
        g = WindowGPU(wl, L, R, mpo)
        gs.append((g, keys))
        plans.append(g.plan(prec))
        x0.append(to_dev(g.pack_theta(bs.unflatten(starts(name, 40 + i), keys))))
    batch = pk.Batch(plans)
    xb = [x.clone() for x in x0]
    eb, kb, us = pk.lanczos_ground_batched(batch, xb, 30, 1e-14)
    say(batch.info())
    for i, name in enumerate(SCALE_NAMES):
        eo, vo, ko = oracle_run(name, 40 + i)
        g, keys = gs[i]
        v = bs.flatten(g.unpack_theta(xb[i].cpu().numpy()), keys)
        de = abs(eb[i] - eo) / abs(eo)
        ov = 1 - abs(np.vdot(vo, v / np.linalg.norm(v)))
        say(f"  {name}: steps {kb[i]} (oracle {ko}) dE/E={de:.3e} 1-overlap={ov:.3e} done at {us[i]:.0f} us")
        assert kb[i] == ko
        assert de <= SCALE_TOL[prec]
