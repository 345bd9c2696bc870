#!/usr/bin/env python3
"""Benchmark of the mixed real/momentum-space cylinder DMRG hot path on one MI355X.

One step = one bond update of the sweep, every row of the hot path on one batch of
synthetic input (Ly=8, chi=3200 centre window, flux 1/8, t = V = 1):

  plan      charge matching of L, W1, W2, R, theta into block task tables (host) and
            precision staging of L and R (device);
  lanczos   30-step Lanczos ground state of H_eff (each step one matvec: L.theta block
            GEMMs, MPO mixing, (.).R block GEMMs), FP64 reorthogonalisation and
            tridiagonal solve, plus the FP64 Rayleigh quotient in low precision;
  env       env_update_left and env_update_right through the window.

Inputs are resident in HBM before the timed region: the library's own Hofstadter MPO,
environments contracted on the GPU from seeded isometries (workloads), and a seeded
random start vector.  value = algorithmic GFLOP of the step / step time, where the
flops are counted from the library's task tables (8 real flops per complex
multiply-add, no padding).  Matrix products run in --prec (default bf16x3: bf16 hi/lo
split products with FP32 accumulation); Lanczos is FP64 in every mode.  Afterwards the
three precisions are compared on the same window (matvec time, cold start, and the
warm-start gate against the converged FP64 ground state).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec bf16x3|fp32|fp64]
  python bench.py --workload ly10_chi6000 --compare-real   (real-space basis ratios)
  python bench.py --batched                                  (64 independent windows)
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H_eff matvec GFLOP/s & Lanczos time at Ly=8 χ=3200: FP32/BF16x3 vs FP64"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}   # dense MFMA, MI355X
VECTOR_TFLOPS = {"fp64": 78.6, "fp32": 157.3}                    # vector ALU, MI355X
HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_inputs(pk, torch, wl, stream):
    """Environments at the window from seeded isometries, contracted on the GPU.  A
    workload with real entries (wl.real) is built in the real formulation of eq. rot:
    the library's real MPO, float64 tensors, DM_REAL updates."""
    import workloads
    real = getattr(wl, "real", False)
    mpo = pk.HofstadterMPO(wl.Ly, wl.Lx, wl.flux[0], wl.flux[1], wl.t, wl.V, wl.basis, rot=real)
    ly, j, n = wl.ly, wl.j, wl.n
    dev = torch.device("cuda:0")
    bonds = [pk.Bond(b) for b in wl.bonds]
    sites = [mpo.site(i) for i in range(n)]
    dt = torch.float64 if real else torch.complex128
    flag = pk.DM_REAL if real else 0

    def dev_of(flat):
        return torch.from_numpy(flat.real.copy() if real else flat).to(dev)

    L = torch.ones(1, dtype=dt, device=dev)
    for i in range(j):
        A = dev_of(pk.pack(wl.site_tensor(i), pk.LAYOUT_SITE, ly, bonds[i], bonds[i + 1], qs1=sites[i].qs))
        _, nout = pk.layout(pk.LAYOUT_ENV_L, ly, bonds[i + 1], qw=sites[i].qr)
        Lo = torch.empty(nout, dtype=dt, device=dev)
        pk.env_update_left(ly, bonds[i], bonds[i + 1], sites[i], L, A, Lo, pk.DM_FP64 | flag, stream)
        L = Lo
        if i % 32 == 31:
            log(f"  left environment: {i + 1}/{j} sites")
    R = torch.ones(1, dtype=dt, device=dev)
    for i in range(n - 1, j + 1, -1):
        B = dev_of(pk.pack(wl.site_tensor(i), pk.LAYOUT_SITE, ly, bonds[i], bonds[i + 1], qs1=sites[i].qs))
        _, nout = pk.layout(pk.LAYOUT_ENV_R, ly, bonds[i], qw=sites[i].ql)
        Ro = torch.empty(nout, dtype=dt, device=dev)
        pk.env_update_right(ly, bonds[i], bonds[i + 1], sites[i], R, B, Ro, pk.DM_FP64 | flag, stream)
        R = Ro
        if i % 32 == 0:
            log(f"  right environment: {n - i}/{n - j - 2} sites")
    a, b, c = bonds[j], bonds[j + 1], bonds[j + 2]
    w1, w2 = sites[j], sites[j + 1]
    theta = dev_of(pk.pack(wl.theta(), pk.LAYOUT_THETA, ly, a, c, qs1=w1.qs, qs2=w2.qs))
    import numpy as np
    rng = np.random.default_rng(1234)
    Aj = dev_of(pk.pack(workloads.left_isometry(rng, wl.bonds[j], wl.bonds[j + 1], wl.qsite[j], ly, real),
                        pk.LAYOUT_SITE, ly, a, b, qs1=w1.qs))
    Bj = dev_of(pk.pack(workloads.right_isometry(rng, wl.bonds[j + 1], wl.bonds[j + 2], wl.qsite[j + 1], ly, real),
                        pk.LAYOUT_SITE, ly, b, c, qs1=w2.qs))
    _, nl = pk.layout(pk.LAYOUT_ENV_L, ly, b, qw=w1.qr)
    _, nr = pk.layout(pk.LAYOUT_ENV_R, ly, b, qw=w2.ql)
    out = dict(ly=ly, a=a, b=b, c=c, w1=w1, w2=w2, L=L, R=R, theta=theta, Aj=Aj, Bj=Bj,
               Lnext=torch.empty(nl, dtype=dt, device=dev),
               Rnext=torch.empty(nr, dtype=dt, device=dev),
               D=(w1.W.shape[0], w1.W.shape[3], w2.W.shape[3]), flag=flag)
    out["env_flops"] = (pk.env_flops(True, ly, a, b, w1), pk.env_flops(False, ly, b, c, w2))
    return out


PROFILE_EVERY = 4


def run_step(pk, inp, prec, iters, stream, profile=False):
    """One bond update; returns (energy, iterations, plan, host times)."""
    t0 = time.perf_counter()
    plan = pk.HeffPlan(inp["ly"], inp["a"], inp["c"], inp["w1"], inp["w2"], inp["L"], inp["R"],
                       prec, stream)
    if profile:
        # stage times from every PROFILE_EVERY-th matvec: each recorded HIP event costs
        # the stream a few microseconds, five per recorded matvec
        plan.profile(True, every=PROFILE_EVERY)
    th = inp["theta"].clone()
    t1 = time.perf_counter()
    e, k = pk.lanczos_ground(plan, th, iters, 1e-14, stream)
    t2 = time.perf_counter()
    pk.env_update_left(inp["ly"], inp["a"], inp["b"], inp["w1"], inp["L"], inp["Aj"], inp["Lnext"], prec, stream)
    pk.env_update_right(inp["ly"], inp["b"], inp["c"], inp["w2"], inp["R"], inp["Bj"], inp["Rnext"], prec, stream)
    t3 = time.perf_counter()
    return e, k, plan, (t1 - t0, t2 - t1, t3 - t2)


def step_flops(plan, k, prec, env_flops, pk):
    mv = sum(plan.flops)
    n_mv = k + (1 if prec != pk.DM_FP64 else 0)
    return n_mv * mv + sum(env_flops)


def matvec_time(pk, torch, inp, prec, stream, reps=20, plan=None):
    if plan is None:
        plan = pk.HeffPlan(inp["ly"], inp["a"], inp["c"], inp["w1"], inp["w2"], inp["L"], inp["R"], prec, stream)
    x = inp["theta"]
    y = torch.empty_like(x)
    for _ in range(3):
        pk.heff_apply(plan, x, y, stream)
    s = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(s)
    for _ in range(reps):
        pk.heff_apply(plan, x, y, stream)
    ev[1].record(s)
    torch.cuda.synchronize()
    return ev[0].elapsed_time(ev[1]) / reps, sum(plan.flops), plan.flops


def copy_calibration(nbytes=1 << 30, reps=5):
    """A plain streaming kernel of known traffic (read nbytes, write nbytes per launch):
    the reference against which the HBM byte counters of the other kernels are scaled."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_kernel": "elementwise neg (float32)", "read_bytes": nbytes,
                      "write_bytes": nbytes, "launches": reps}), flush=True)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "ly8_chi3200_bf16x3_hbm_traffic.md")
KERNEL_SOURCES = ["gemm_bf16x3.hip", "gemm_presplit.hip", "kernels.hip", "device.hpp", "internal.hpp"]


def measured_traffic(workload, pname):
    """Per-launch HBM bytes of the matvec kernels from the committed rocprofv3 counter
    summary, or {} when it does not apply: another workload or precision, or kernel
    sources that changed since the counters were taken (their hash is stored with them)."""
    import hashlib
    import re
    if workload != "ly8_chi3200" or pname != "bf16x3" or not os.path.exists(TRAFFIC_PROFILE):
        return {}
    m = re.search(r"```json\n(.*?)\n```", open(TRAFFIC_PROFILE).read(), re.S)
    if not m:
        return {}
    rec = json.loads(m.group(1))
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1512_03318_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return rec["kernels"] if h.hexdigest() == rec["sources_sha256"] else {}


def stage_rooflines(pk, plan, prec, pname, prof, nmv, workload):
    """Roofline of each matvec kernel from its in-run device time (HIP events on the
    launch stream, averaged over the sampled matvecs) and its algorithmic work.

    Algorithmic bytes are those of the matvec's own operands only: L, R and the MPO
    tensors W1, W2 read, theta read and theta' written, each once, in the precision it
    is stored in (the L.theta GEMM reads the FP32 copy of theta in the low-precision
    modes; BF16x3 writes theta' in FP64).  The intermediates X (L.theta) and Z (mixed)
    are not algorithmic bytes: their traffic is overhead, visible as the ratio of the
    counted HBM bytes (profiles/, when they match the kernel sources) to the algorithmic
    ones.  Per kernel: L.theta GEMM = 8 flop per complex MAC of its task table over
    L + theta bytes; (.).R GEMM over R + theta' bytes; MPO mixing over the W bytes (it
    runs on the vector ALUs).  A kernel's bound is the roof its algorithmic work reaches
    first (matrix cores for BF16x3: the bf16 dense peak over three bf16 products per real
    product; HBM at 8 TB/s); `frac` is its achieved fraction of that roof."""
    eb = 16 if prec == pk.DM_FP64 else 8
    avg = [p / max(nmv, 1) for p in prof]
    # BF16x3: the kernels that split FP32 operands while staging them, or with
    # MRDMRG_PRESPLIT=1 the kernels on pre-split operands (stream-K unless MRDMRG_SK=0)
    presplit = os.environ.get("MRDMRG_PRESPLIT", "0") == "1"
    streamk = os.environ.get("MRDMRG_SK", "1") != "0"
    if presplit and streamk:
        bf3 = ("mrd::gemm_sk_kernel<0>", "mrd::gemm_sk_kernel<1>", "mrd::mix_slab_kernel<float, __bf16, false>",
               "mrd::gemm_sk_reduce_kernel<1>")
    elif presplit:
        bf3 = ("mrd::gemm_ps_kernel<128, 64, 2, 2, false, 0>", "mrd::gemm_ps_kernel<128, 32, 4, 1, true, 1>",
               "mrd::mix_slab_kernel<float, __bf16, false>", "mrd::gemm_split_reduce_kernel<float, 144, mrd::PsProb, false>")
    else:
        bf3 = ("mrd::gemm_bf3_kernel<0, 128, 64, 2, 2, false, false>", "mrd::gemm_bf3_kernel<148, 128, 32, 4, 1, true, false>",
               "mrd::mix_slab_kernel<float, float, false>", "mrd::gemm_split_reduce_kernel<float, 148, mrd::GemmProb, false>")
    gemm = {pk.DM_FP64: ("mrd::gemm_kernel<double, 0, false, false>", "mrd::gemm_kernel<double, 20, true, false>"),
            pk.DM_FP32: ("mrd::gemm_kernel<float, 0, false, false>", "mrd::gemm_kernel<float, 20, true, false>"),
            pk.DM_BF16X3: bf3[:2]}[prec]
    mixk = {pk.DM_FP64: "mrd::mix_slab_kernel<double, double, false>",
            pk.DM_FP32: "mrd::mix_slab_kernel<float, float, false>",
            pk.DM_BF16X3: bf3[2]}[prec]
    redk = {pk.DM_FP64: "mrd::gemm_split_reduce_kernel<double, 20, mrd::GemmProb, false>",
            pk.DM_FP32: "mrd::gemm_split_reduce_kernel<float, 20, mrd::GemmProb, false>",
            pk.DM_BF16X3: bf3[3]}[prec]
    traffic = measured_traffic(workload, pname)
    hw = 3 if prec == pk.DM_BF16X3 else 1
    peak_alg = PEAK_TFLOPS[pname] / hw
    sz = plan.sizes
    w_bytes = 16 * (plan.w1.W.size + plan.w2.W.size)
    th_in = sz["theta"] * eb
    th_out = sz["theta"] * (16 if prec in (pk.DM_FP64, pk.DM_BF16X3) else 8)
    rows = [(gemm[0], "L.theta block GEMM", plan.flops[0], sz["L"] * eb + th_in, "matrix"),
            (mixk, "MPO mixing", plan.flops[1], w_bytes, "alu"),
            (gemm[1], "(.).R block GEMM", plan.flops[2], sz["R"] * eb + th_out, "matrix"),
            (redk, "(.).R K-split reduction", 0.0, 0, None)]
    stages = []
    for i, (kern, what, flops, nbytes, unit) in enumerate(rows):
        t = avg[i] * 1e-3
        tr = traffic.get(kern)
        counted = (tr["read_bytes"] + tr["write_bytes"]) if tr else None
        r = {"kernel": f"{kern} ({what}, {pname})", "avg_launch_ms": round(avg[i], 4),
             "algorithmic_flops": flops, "algorithmic_bytes": nbytes, "traffic": counted,
             "traffic_ratio": round(counted / nbytes, 2) if (counted and nbytes) else None}
        if tr:
            r["traffic_read_write"] = [tr["read_bytes"], tr["write_bytes"]]
        if unit == "matrix" and t > 0:
            t_mfma, t_hbm = flops / (peak_alg * 1e12), nbytes / (HBM_GBS * 1e9)
            tf = flops / t / 1e12
            r.update({"bound": "mfma" if t_mfma >= t_hbm else "hbm",
                      "mfma_floor_us": round(1e6 * t_mfma, 2), "hbm_floor_us": round(1e6 * t_hbm, 2),
                      "flop_per_byte": round(flops / nbytes, 1),
                      "ridge_flop_per_byte": round(peak_alg * 1e12 / (HBM_GBS * 1e9), 1)})
            if t_mfma >= t_hbm:
                r.update({"achieved": round(tf, 3), "peak": round(peak_alg, 1), "unit": "TFLOP/s",
                          "frac": round(tf / peak_alg, 4)})
            else:
                ach = nbytes / t / 1e9
                r.update({"achieved": round(ach, 1), "peak": HBM_GBS, "unit": "GB/s",
                          "frac": round(ach / HBM_GBS, 4)})
            r["mfma_frac"] = round(tf / peak_alg, 4)
            if hw > 1:
                r["matrix_peak_note"] = (f"{PEAK_TFLOPS[pname]} TFLOP/s bf16 dense / {hw} bf16 products "
                                         "per algorithmic real product")
        elif unit == "alu" and t > 0:
            peak_v = VECTOR_TFLOPS["fp64" if prec == pk.DM_FP64 else "fp32"]
            tf = flops / t / 1e12
            r.update({"bound": "alu", "achieved": round(tf, 3), "peak": peak_v, "unit": "TFLOP/s",
                      "frac": round(tf / peak_v, 4)})
        stages.append(r)
    dom = max(range(3), key=lambda i: avg[i])
    out = dict(stages[dom])
    out["stages"] = stages
    out["profiled_matvecs"] = nmv  # HIP-event samples (every PROFILE_EVERY-th matvec)
    return out


def matvec_roofline(pk, plan, prec, pname, mv_ms, stages):
    """The whole matvec against the matrix-core roof: all its algorithmic flops over
    L + R + W + theta + theta' bytes, and the counted HBM bytes of its kernels (when the
    counters match the sources) over those algorithmic bytes."""
    eb = 16 if prec == pk.DM_FP64 else 8
    sz = plan.sizes
    hw = 3 if prec == pk.DM_BF16X3 else 1
    peak_alg = PEAK_TFLOPS[pname] / hw
    nbytes = (sz["L"] + sz["R"] + sz["theta"]) * eb + 16 * (plan.w1.W.size + plan.w2.W.size) + \
        sz["theta"] * (16 if prec in (pk.DM_FP64, pk.DM_BF16X3) else 8)
    flops = sum(plan.flops)
    tf = flops / (mv_ms * 1e-3) / 1e12
    counted = [st["traffic"] for st in stages]
    total = sum(counted) if all(c is not None for c in counted) else None
    return {"algorithmic_flops": flops, "algorithmic_bytes": nbytes, "ms": round(mv_ms, 4),
            "achieved": round(tf, 3), "peak": round(peak_alg, 1), "unit": "TFLOP/s",
            "frac": round(tf / peak_alg, 4),
            "mfma_floor_us": round(1e6 * flops / (peak_alg * 1e12), 2),
            "hbm_floor_us": round(1e6 * nbytes / (HBM_GBS * 1e9), 2),
            "traffic": total, "traffic_ratio": round(total / nbytes, 2) if total else None}


def precision_report(pk, torch, inp, iters, stream, noise=1e-3, reps=3):
    """Per precision: matvec time, cold-start Lanczos energy (same seeded start vector as
    the timed steps), and the warm-start gate: the start vector is the FP64 ground state
    (restarted FP64 Lanczos until the energy is stationary to 1e-15) plus seeded noise of
    relative size `noise`; reported are |E - E_gs| / |E_gs|, 1 - |<theta_gs|theta>| and
    the median wall time of the solve (max `iters` steps)."""
    precs = {"fp64": pk.DM_FP64, "fp32": pk.DM_FP32, "bf16x3": pk.DM_BF16X3}
    mk = lambda q: pk.HeffPlan(inp["ly"], inp["a"], inp["c"], inp["w1"], inp["w2"], inp["L"], inp["R"],
                               q, stream)
    plan64 = mk(pk.DM_FP64)
    gs = inp["theta"].clone()
    e_gs, e_prev, restarts = 0.0, None, 0
    for restarts in range(1, 41):
        e_gs, _ = pk.lanczos_ground(plan64, gs, iters, 1e-14, stream)
        if e_prev is not None and abs(e_gs - e_prev) <= 1e-15 * abs(e_gs):
            break
        e_prev = e_gs
    gs = gs / torch.linalg.vector_norm(gs)
    hv = torch.empty_like(gs)
    pk.heff_apply(plan64, gs, hv, stream)
    resid = float(torch.linalg.vector_norm(hv - e_gs * gs))
    g = torch.Generator().manual_seed(2024)
    nz = torch.complex(torch.randn(gs.numel(), generator=g, dtype=torch.float64),
                       torch.randn(gs.numel(), generator=g, dtype=torch.float64)).to(gs.device)
    warm = gs + noise * nz / torch.linalg.vector_norm(nz)
    warm = warm / torch.linalg.vector_norm(warm)
    out = {"ground_state": {"energy": e_gs, "restarts": restarts, "residual": resid, "noise": noise,
                            "reference": "the library's FP64 path (restarted Lanczos on the GPU); the "
                                         "same gate against the FP64 CPU oracle's ground state of this "
                                         "window runs in tests/test_gpu_gate_fullsize.py"}}
    for name, q in precs.items():
        plan = mk(q)
        ms, _, _ = matvec_time(pk, torch, inp, q, stream, plan=plan)
        cold = inp["theta"].clone()
        e_cold, _ = pk.lanczos_ground(plan, cold, iters, 1e-14, stream)
        ts, e, k, x = [], 0.0, 0, None
        for _ in range(reps):
            x = warm.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e, k = pk.lanczos_ground(plan, x, iters, 1e-14, stream)
            ts.append(time.perf_counter() - t0)
        x = x / torch.linalg.vector_norm(x)
        ov = 1.0 - float(torch.abs(torch.vdot(gs, x)))
        out[name] = {"matvec_ms": round(ms, 4), "matvec_gflops": round(sum(plan.flops) / ms / 1e6, 2),
                     "lanczos_warm_ms": round(1e3 * statistics.median(ts), 3), "warm_steps": k,
                     "warm_rel_energy_err": abs(e - e_gs) / abs(e_gs), "warm_1_minus_overlap": ov,
                     "gate_passed": abs(e - e_gs) / abs(e_gs) <= 1e-9 and ov <= 1e-6,
                     "cold_energy": e_cold}
    for name in precs:
        out[name]["cold_rel_energy_diff_vs_fp64"] = abs(out[name]["cold_energy"] - out["fp64"]["cold_energy"]) / \
            abs(out["fp64"]["cold_energy"])
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(wl, iters=30):
    """The FP64 oracle on the host: a 30-step oracle Lanczos of the same window with
    random environments of the exact block structure (bounded sample)."""
    import numpy as np

    import workloads
    from oracle import blocksparse as bs
    from oracle import lanczos as olz
    from oracle import mpo as omp
    from oracle import synth
    m = omp.build(synth.cylinder_of(wl), wl.basis)
    j = wl.j
    rng = np.random.default_rng(7)
    L = workloads.random_env(rng, wl.bonds[j], m.qbond[j], wl.ly, "L")
    R = workloads.random_env(rng, wl.bonds[j + 2], m.qbond[j + 2], wl.ly, "R")
    keys = bs.theta_keys(wl.bonds[j], wl.bonds[j + 2], wl.qsite[j], wl.qsite[j + 1], wl.ly)
    th = bs.flatten(wl.theta(), keys)
    nmv = [0]

    def mv(v):
        nmv[0] += 1
        return bs.flatten(bs.heff_apply(L, m.W[j], m.W[j + 1], R, bs.unflatten(v, keys)), keys)

    # flops of one matvec from the oracle's own block structure (8 per complex MAC)
    flops = 0.0
    byl = {}
    for (qa, s1, s2, qc), blk in wl.theta().items():
        byl.setdefault(qa, []).append(blk.shape[1])
    for (qap, w, qa), lb in L.items():
        for nc in byl.get(qa, []):
            flops += 8.0 * lb.shape[0] * lb.shape[1] * nc
    t0 = time.perf_counter()
    olz.lanczos(mv, th, max_iter=iters)
    dt = time.perf_counter() - t0
    # the (.).R half has the same shape class; count it from R blocks and theta rows
    byr = {}
    for (qa, s1, s2, qc), blk in wl.theta().items():
        byr.setdefault(qc, []).append(blk.shape[0])
    for (qcp, w, qc), rb in R.items():
        for na in byr.get(qcp, []):
            flops += 8.0 * rb.shape[0] * rb.shape[1] * na
    cores = len(os.sched_getaffinity(0))
    return {"value": round(nmv[0] * flops / dt / 1e9, 3), "unit": "GFLOP/s", "cores": cores,
            "cpu_model": cpu_model(), "kind": "oracle",
            "sample": f"{iters}-step FP64 oracle Lanczos (numpy, per-block matmuls) of the same "
                      f"window, random environments of the exact block structure, {dt:.1f} s; "
                      f"block-GEMM flops only"}


def window_costs(pk, torch, ly, a, b, c, w1, w2, L, R, theta, A, B, prec, stream, reps=5):
    """Median device times (ms) of one matvec and of the two environment updates of a
    window, with their task-table flops and the stored elements of L, R and theta."""
    plan = pk.HeffPlan(ly, a, c, w1, w2, L, R, prec, stream)
    y = torch.empty_like(theta)
    _, nl = pk.layout(pk.LAYOUT_ENV_L, ly, b, qw=w1.qr)
    _, nr = pk.layout(pk.LAYOUT_ENV_R, ly, b, qw=w2.ql)
    Lo = torch.empty(nl, dtype=torch.complex128, device=theta.device)
    Ro = torch.empty(nr, dtype=torch.complex128, device=theta.device)
    s = torch.cuda.current_stream()

    def med(fn):
        fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            fn()
            e1.record(s)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return sorted(ts)[reps // 2]

    t_mv = med(lambda: pk.heff_apply(plan, theta, y, stream))
    t_l = med(lambda: pk.env_update_left(ly, a, b, w1, L, A, Lo, prec, stream))
    t_r = med(lambda: pk.env_update_right(ly, b, c, w2, R, B, Ro, prec, stream))
    return {"matvec_ms": round(t_mv, 4), "env_left_ms": round(t_l, 4), "env_right_ms": round(t_r, 4),
            "matvec_gflop": round(sum(plan.flops) / 1e9, 4),
            "env_gflop": round((pk.env_flops(True, ly, a, b, w1) + pk.env_flops(False, ly, b, c, w2)) / 1e9, 4),
            "elements_L_R_theta": int(L.numel() + R.numel() + theta.numel()),
            "sectors": len(a.q) if hasattr(a, "q") else None}


def compare_real(pk, torch, wl, inp, prec, stream):
    """The same window in the real-space basis (charge N only, real-space MPO of the same
    cylinder, same chi and sector rule): cost ratios real / mixed.  Environments of the
    exact block structure with seeded Gaussian entries (costs do not depend on values)."""
    import numpy as np

    import workloads
    mixed = window_costs(pk, torch, inp["ly"], inp["a"], inp["b"], inp["c"], inp["w1"], inp["w2"],
                         inp["L"], inp["R"], inp["theta"], inp["Aj"], inp["Bj"], prec, stream)
    wr = workloads.make_workload(wl.name + "_real", wl.Ly, wl.Lx, wl.flux, wl.chi, wl.seed, basis="real")
    mpo = pk.HofstadterMPO(wr.Ly, wr.Lx, wr.flux[0], wr.flux[1], wr.t, wr.V, "real")
    j = wr.j
    w1, w2 = mpo.site(j), mpo.site(j + 1)
    a, b, c = (pk.Bond(wr.bonds[k]) for k in (j, j + 1, j + 2))
    rng = np.random.default_rng(55)
    dev = inp["theta"].device

    def up(x):
        return torch.from_numpy(x).to(dev)

    L = up(pk.pack(workloads.random_env(rng, wr.bonds[j], w1.ql, 1, "L"), pk.LAYOUT_ENV_L, 1, a, qw=w1.ql))
    R = up(pk.pack(workloads.random_env(rng, wr.bonds[j + 2], w2.qr, 1, "R"), pk.LAYOUT_ENV_R, 1, c, qw=w2.qr))
    th = up(pk.pack(workloads.random_theta(rng, wr.bonds[j], wr.bonds[j + 2], w1.qs, w2.qs, 1),
                    pk.LAYOUT_THETA, 1, a, c, qs1=w1.qs, qs2=w2.qs))
    A = up(pk.pack(workloads.left_isometry(rng, wr.bonds[j], wr.bonds[j + 1], wr.qsite[j], 1),
                   pk.LAYOUT_SITE, 1, a, b, qs1=w1.qs))
    B = up(pk.pack(workloads.right_isometry(rng, wr.bonds[j + 1], wr.bonds[j + 2], wr.qsite[j + 1], 1),
                   pk.LAYOUT_SITE, 1, b, c, qs1=w2.qs))
    real = window_costs(pk, torch, 1, a, b, c, w1, w2, L, R, th, A, B, prec, stream)
    mixed["sectors"] = len(wl.bonds[wl.j])
    real["sectors"] = len(wr.bonds[j])
    mixed["mpo_D"] = list(inp["D"])
    real["mpo_D"] = [w1.W.shape[0], w1.W.shape[3], w2.W.shape[3]]
    ratio = {k: round(real[k] / mixed[k], 2) for k in
             ("matvec_gflop", "env_gflop", "elements_L_R_theta", "matvec_ms", "env_left_ms", "env_right_ms")}
    return {"mixed": mixed, "real": real, "real_over_mixed": ratio,
            "chi_real": int(sum(wr.bonds[j].values())), "chi_mixed": int(sum(wl.bonds[wl.j].values()))}


def eq_rot_report(pk, torch, wl, inp, iters, stream, reps=3):
    """The real formulation of eq. rot at the same window: the library's real MPO, real
    isometries and theta (float64), DM_REAL plans.  Matvec and cold-start Lanczos times
    in FP64, FP32 and BF16x3 next to the complex plans' (same sectors, same chi; the windows'
    random entries differ, so their energies are not compared here -- the GPU tests
    check one window both ways)."""
    import statistics

    import workloads
    wr = workloads.preset(wl.name, real=True)
    log("eq. rot (real formulation): building the window ...")
    rin = build_inputs(pk, torch, wr, stream)

    def solve_ms(plan, x0):
        ts = []
        e = k = None
        for _ in range(reps):
            x = x0.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e, k = pk.lanczos_ground(plan, x, iters, 1e-14, stream)
            ts.append(1e3 * (time.perf_counter() - t0))
        return statistics.median(ts), e, k

    out = {"mpo_D": list(rin["D"]), "workload": wr.name, "entries": "real (float64)"}
    for name, prec in (("fp64", pk.DM_FP64), ("fp32", pk.DM_FP32), ("bf16x3", pk.DM_BF16X3)):
        cplan = pk.HeffPlan(inp["ly"], inp["a"], inp["c"], inp["w1"], inp["w2"], inp["L"], inp["R"], prec, stream)
        rplan = pk.HeffPlan(rin["ly"], rin["a"], rin["c"], rin["w1"], rin["w2"], rin["L"], rin["R"],
                            prec | pk.DM_REAL, stream)
        cms, cfl, _ = matvec_time(pk, torch, inp, prec, stream, plan=cplan)
        rms, rfl, _ = matvec_time(pk, torch, rin, prec, stream, plan=rplan)
        clz, _, _ = solve_ms(cplan, inp["theta"])
        rlz, re_, rk = solve_ms(rplan, rin["theta"])
        out[name] = {"matvec_ms": round(rms, 4), "matvec_gflop": round(rfl / 1e9, 3),
                     "matvec_gflops": round(rfl / rms / 1e6, 1), "lanczos_ms": round(rlz, 3),
                     "lanczos_steps": rk, "energy": re_,
                     "complex_matvec_ms": round(cms, 4), "complex_lanczos_ms": round(clz, 3),
                     "matvec_speedup_over_complex": round(cms / rms, 2),
                     "lanczos_speedup_over_complex": round(clz / rlz, 2),
                     "flops_over_complex": round(rfl / cfl, 4)}
        log(f"  {name}: real matvec {rms:.4f} ms (complex {cms:.4f}), Lanczos {rlz:.2f} ms (complex {clz:.2f})")
        del cplan, rplan
    out["bytes_over_complex"] = round((rin["L"].numel() * 8 + rin["R"].numel() * 8 + rin["theta"].numel() * 8) /
                                      (inp["L"].numel() * 16 + inp["R"].numel() * 16 + inp["theta"].numel() * 16), 4)
    return out


# ---------------------------------------------------------------------------------
# The Fig. 3 workload's cost curves (Sec. III B): Ly=10, flux 1/3, V/t=0.1, lowest band
# filled (N = n/3), chi from 100 to 12800, in the mixed basis (complex, and the real form
# of eq. rot) and in the real-space basis.  Centre windows of a finite cylinder (Lx=6,
# two magnetic cells) with the sector rule of the synthetic workloads; the values of
# L, R, theta and the site tensors are seeded Gaussians drawn on the device at the
# layouts' sizes (costs do not depend on them).  The paper's curves come from converged
# iDMRG on an infinite cylinder; this re-measures time and memory per chi only.
# ---------------------------------------------------------------------------------
FIG3_CHI = (100, 200, 400, 800, 1600, 3200, 6400, 12800)


def fig3_window(pk, torch, basis, rot, chi, prec, stream, reps=3):
    import workloads
    Ly, Lx, flux, V = 10, 6, (1, 3), 0.1
    n = Ly * Lx
    wl = workloads.make_workload(f"fig3_{basis}{'_rot' if rot else ''}_chi{chi}", Ly, Lx, flux, chi, 3,
                                 V=V, N_tot=n // 3, basis=basis, real=rot)
    mpo = pk.HofstadterMPO(Ly, Lx, flux[0], flux[1], 1.0, V, basis, rot=rot)
    j, ly = wl.j, wl.ly
    a, b, c = (pk.Bond(wl.bonds[k]) for k in (j, j + 1, j + 2))
    w1, w2 = mpo.site(j), mpo.site(j + 1)
    dt = torch.float64 if rot else torch.complex128
    flag = pk.DM_REAL if rot else 0
    gen = torch.Generator(device="cuda").manual_seed(chi)

    def rnd(kind, *args, **kw):
        _, ne = pk.layout(kind, ly, *args, **kw)
        return torch.randn(max(ne, 1), dtype=dt, device="cuda", generator=gen)[:ne]

    L = rnd(pk.LAYOUT_ENV_L, a, qw=w1.ql)
    R = rnd(pk.LAYOUT_ENV_R, c, qw=w2.qr)
    th = rnd(pk.LAYOUT_THETA, a, c, qs1=w1.qs, qs2=w2.qs)
    A = rnd(pk.LAYOUT_SITE, a, b, qs1=w1.qs)
    B = rnd(pk.LAYOUT_SITE, b, c, qs1=w2.qs)
    _, nl = pk.layout(pk.LAYOUT_ENV_L, ly, b, qw=w1.qr)
    _, nr = pk.layout(pk.LAYOUT_ENV_R, ly, b, qw=w2.ql)
    Lo = torch.empty(nl, dtype=dt, device="cuda")
    Ro = torch.empty(nr, dtype=dt, device="cuda")
    plan = pk.HeffPlan(ly, a, c, w1, w2, L, R, prec | flag, stream)
    y = torch.empty_like(th)
    s = torch.cuda.current_stream()

    def med(fn):
        fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            fn()
            e1.record(s)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return sorted(ts)[reps // 2]

    t_mv = med(lambda: pk.heff_apply(plan, th, y, stream))
    t_l = med(lambda: pk.env_update_left(ly, a, b, w1, L, A, Lo, prec | flag, stream))
    t_r = med(lambda: pk.env_update_right(ly, b, c, w2, R, B, Ro, prec | flag, stream))
    sz = plan.sizes
    eb = (8 if rot else 16) // (2 if prec != pk.DM_FP64 else 1)
    res = {"chi": int(sum(wl.bonds[j].values())), "sectors": len(wl.bonds[j]),
           "mpo_D": [w1.W.shape[0], w1.W.shape[3], w2.W.shape[3]],
           "matvec_ms": round(t_mv, 4), "env_ms": round(t_l + t_r, 4),
           # one bond update of the benchmark's kind: 30 matvecs and both updates
           "bond_update_model_ms": round(30 * t_mv + t_l + t_r, 3),
           "matvec_gflop": round(sum(plan.flops) / 1e9, 4),
           "state_bytes": int((sz["L"] + sz["R"] + sz["theta"]) * eb),
           "matvec_bytes": int((sz["L"] + sz["R"] + sz["theta"] + sz["X"] + sz["Z"]) * eb)}
    del plan, L, R, th, A, B, Lo, Ro, y
    torch.cuda.empty_cache()
    return res


def fig3_main(args):
    import torch

    import paper_1512_03318_amd as pk
    stream = torch.cuda.current_stream()
    prec = {"fp64": pk.DM_FP64, "fp32": pk.DM_FP32}.get(args.prec, pk.DM_FP64)
    rows = []
    for chi in FIG3_CHI:
        row = {"chi_target": chi}
        for key, basis, rot in (("mixed", "mixed", False), ("mixed_eq_rot", "mixed", True), ("real_space", "real", False)):
            row[key] = fig3_window(pk, torch, basis, rot, chi, prec, stream)
            log(f"fig3 chi={chi} {key}: matvec {row[key]['matvec_ms']} ms, state {row[key]['state_bytes'] / 1e6:.1f} MB")
        m, r, q = row["mixed"], row["real_space"], row["mixed_eq_rot"]
        row["real_space_over_mixed"] = {"bond_update_time": round(r["bond_update_model_ms"] / m["bond_update_model_ms"], 2),
                                        "state_memory": round(r["state_bytes"] / m["state_bytes"], 2),
                                        "matvec_gflop": round(r["matvec_gflop"] / m["matvec_gflop"], 2)}
        row["real_space_over_eq_rot"] = {"bond_update_time": round(r["bond_update_model_ms"] / q["bond_update_model_ms"], 2),
                                         "state_memory": round(r["state_bytes"] / q["state_bytes"], 2)}
        rows.append(row)
    print(json.dumps({"workload": "fig3: Ly=10, flux 1/3, V/t=0.1, N = n/3, chi 100..12800",
                      "precision": args.prec if args.prec in ("fp64", "fp32") else "fp64",
                      "data": "synthetic (seeded Gaussian tensors of the exact block structure)",
                      "rows": rows}), flush=True)


# ---------------------------------------------------------------------------------
# Many independent windows in one batched Lanczos (64 windows, Ly in {4, 6, 8},
# chi in [200, 2000], seeds from SeedSequence(4).spawn(64)).
# ---------------------------------------------------------------------------------
def batched_specs(n=64, seed=4):
    import numpy as np
    out = []
    for i, ss in enumerate(np.random.SeedSequence(seed).spawn(n)):
        r = np.random.default_rng(ss)
        Ly = int(r.choice([4, 6, 8]))
        chi = int(r.integers(200, 2001))
        out.append((i, Ly, chi, int(ss.generate_state(1)[0])))
    return out


_MPO_CACHE = {}


def _mpo(pk, wl):
    key = (wl.Ly, wl.Lx)
    if key not in _MPO_CACHE:
        _MPO_CACHE[key] = pk.HofstadterMPO(wl.Ly, wl.Lx, wl.flux[0], wl.flux[1], wl.t, wl.V, wl.basis)
    return _MPO_CACHE[key]


def batched_instance_host(spec):
    """Host part of one window: seeded isometries of every site outside the window and
    the start vector, packed in the library's layouts (runs in a worker process)."""
    from threadpoolctl import threadpool_limits

    import paper_1512_03318_amd as pk
    import workloads
    with threadpool_limits(1):  # one BLAS thread per worker: the workers share the cores
        return _instance_host(pk, workloads, spec)


def _instance_host(pk, workloads, spec):
    i, Ly, chi, seed = spec
    wl = workloads.centre_workload(f"window{i}", Ly, chi, seed)
    mpo = _mpo(pk, wl)
    ly, j, n = wl.ly, wl.j, wl.n
    bonds = [pk.Bond(b) for b in wl.bonds]
    qs = [mpo.site(k).qs for k in range(n)]
    left = [pk.pack(wl.site_tensor(k), pk.LAYOUT_SITE, ly, bonds[k], bonds[k + 1], qs1=qs[k])
            for k in range(j)]
    right = [pk.pack(wl.site_tensor(k), pk.LAYOUT_SITE, ly, bonds[k], bonds[k + 1], qs1=qs[k])
             for k in range(n - 1, j + 1, -1)]
    theta = pk.pack(wl.theta(), pk.LAYOUT_THETA, ly, bonds[j], bonds[j + 2], qs1=qs[j], qs2=qs[j + 1])
    return spec, left, right, theta


def batched_main(args):
    import numpy as np
    from concurrent.futures import ProcessPoolExecutor
    specs = batched_specs()
    # workers are forked and given all their jobs before this process touches the GPU
    workers = max(1, min(8, len(os.sched_getaffinity(0))))
    pool = ProcessPoolExecutor(max_workers=workers)
    futs = [pool.submit(batched_instance_host, sp) for sp in specs]

    import torch

    import paper_1512_03318_amd as pk
    import workloads
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    prec = {"fp64": pk.DM_FP64, "fp32": pk.DM_FP32, "bf16x3": pk.DM_BF16X3}[args.prec]
    t0 = time.perf_counter()
    plans, x0, shapes = [], [], []
    while futs:
        (i, Ly, chi, seed), left, right, theta = futs.pop(0).result()  # drop each result once used
        wl = workloads.centre_workload(f"window{i}", Ly, chi, seed)
        mpo = _mpo(pk, wl)
        ly, j, n = wl.ly, wl.j, wl.n
        bonds = [pk.Bond(b) for b in wl.bonds]
        sites = [mpo.site(k) for k in range(n)]
        L = torch.ones(1, dtype=torch.complex128, device=dev)
        for k in range(j):
            _, nout = pk.layout(pk.LAYOUT_ENV_L, ly, bonds[k + 1], qw=sites[k].qr)
            Lo = torch.empty(nout, dtype=torch.complex128, device=dev)
            pk.env_update_left(ly, bonds[k], bonds[k + 1], sites[k], L, torch.from_numpy(left[k]).to(dev),
                               Lo, pk.DM_FP64, stream)
            L = Lo
        R = torch.ones(1, dtype=torch.complex128, device=dev)
        for q, k in enumerate(range(n - 1, j + 1, -1)):
            _, nout = pk.layout(pk.LAYOUT_ENV_R, ly, bonds[k], qw=sites[k].ql)
            Ro = torch.empty(nout, dtype=torch.complex128, device=dev)
            pk.env_update_right(ly, bonds[k], bonds[k + 1], sites[k], R, torch.from_numpy(right[q]).to(dev),
                                Ro, pk.DM_FP64, stream)
            R = Ro
        plans.append(pk.HeffPlan(ly, bonds[j], bonds[j + 2], sites[j], sites[j + 1], L, R, prec, stream))
        x0.append(torch.from_numpy(theta).to(dev))
        shapes.append({"Ly": Ly, "chi": int(sum(wl.bonds[j].values())), "Lx": wl.Lx,
                       "sectors": len(wl.bonds[j]), "n": int(theta.size)})
        if i % 8 == 7:
            log(f"  windows ready: {i + 1}/{len(specs)} ({time.perf_counter() - t0:.1f} s)")
    pool.shutdown()
    torch.cuda.synchronize()
    log(f"{len(plans)} windows ready in {time.perf_counter() - t0:.1f} s")

    batch = pk.Batch(plans, stream)
    iters = args.iters

    def solve_batched():
        xs = [x.clone() for x in x0]
        torch.cuda.synchronize()
        t = time.perf_counter()
        e, k, us = pk.lanczos_ground_batched(batch, xs, iters, 1e-14, stream)
        return time.perf_counter() - t, e, k, us

    for _ in range(args.warmup):
        solve_batched()
    runs = [solve_batched() for _ in range(args.steps)]
    wall = sorted(r[0] for r in runs)[len(runs) // 2]
    _, e_b, k_b, us = runs[-1]
    flops = sum(k * sum(p.flops) for k, p in zip(k_b, plans))
    if prec != pk.DM_FP64:
        flops += sum(sum(p.flops) for p in plans)
    # the same solves one plan at a time
    xs = [x.clone() for x in x0]
    torch.cuda.synchronize()
    t = time.perf_counter()
    e_s = [pk.lanczos_ground(p, x, iters, 1e-14, stream)[0] for p, x in zip(plans, xs)]
    seq = time.perf_counter() - t
    us_sorted = sorted(us)
    out = {"metric": "batched Lanczos ground states of 64 independent windows (Ly in {4,6,8}, "
                     "chi in [200,2000]) per second",
           "value": round(len(plans) / wall, 2), "unit": "solves/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * wall, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": {pk.DM_FP64: "fp64", pk.DM_FP32: "fp32", pk.DM_BF16X3: "bf16x3"}[prec],
           "data": "synthetic",
           "config": {"workload": "batch64_ly4-8_chi200-2000", "instances": len(plans),
                      "lanczos_iters": iters, "precision": args.prec},
           "gflops": round(flops / wall / 1e9, 1),
           "p50_done_ms": round(us_sorted[len(us) // 2] / 1e3, 3),
           "p99_done_ms": round(us_sorted[min(len(us) - 1, int(0.99 * len(us)))] / 1e3, 3),
           "sequential_ms": round(1e3 * seq, 3),
           "speedup_vs_sequential": round(seq / wall, 3),
           "max_rel_energy_diff_vs_sequential": max(abs(a - b) / abs(b) for a, b in zip(e_b, e_s)),
           "tile_tuning": batch.info().strip().splitlines(),
           "chi_range": [min(s["chi"] for s in shapes), max(s["chi"] for s in shapes)],
           "theta_elems_range": [min(s["n"] for s in shapes), max(s["n"] for s in shapes)]}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ly8_chi3200")
    ap.add_argument("--prec", default="bf16x3", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--iters", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--compare-real", action="store_true",
                    help="also time the same window in the real-space basis (cost ratios)")
    ap.add_argument("--no-eq-rot", action="store_true",
                    help="skip the real formulation (eq. rot) of the same window")
    ap.add_argument("--fig3", action="store_true",
                    help="only the Fig. 3 workload's cost curves (chi 100..12800, mixed / eq. rot / real space)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain elementwise copy of 1 GiB (HBM counter calibration)")
    ap.add_argument("--batched", action="store_true",
                    help="64 independent windows in one batched Lanczos instead of one bond update")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the library has no "
              f"multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.fig3:
        return fig3_main(args)
    if args.batched:
        batched_main(args)
        return
    if args.copy_calibration:
        copy_calibration()
        return

    import torch

    import paper_1512_03318_amd as pk
    import workloads
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    prec = {"fp64": pk.DM_FP64, "fp32": pk.DM_FP32, "bf16x3": pk.DM_BF16X3}[args.prec]

    wl = workloads.preset(args.workload)
    t0 = time.perf_counter()
    inp = build_inputs(pk, torch, wl, stream)
    torch.cuda.synchronize()
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s: {args.workload} Lx={wl.Lx} "
        f"chi={sum(wl.bonds[wl.j].values())} sectors={len(wl.bonds[wl.j])} D={inp['D']}")

    for i in range(args.warmup):
        e, k, _, ts = run_step(pk, inp, prec, args.iters, stream)
        log(f"warmup {i}: E={e:.12f} iters={k} plan/lanczos/env s = {ts}")
    torch.cuda.synchronize()
    host = []
    flops = 0.0
    prof = [0.0, 0.0, 0.0, 0.0]
    nmv = 0
    t0 = time.perf_counter()
    for i in range(args.steps):
        # per-kernel HIP events on the launch stream, recorded inside the timed steps
        e, k, plan, ts = run_step(pk, inp, prec, args.iters, stream, profile=True)
        ms, nm = plan.profile_read()
        prof = [p + q for p, q in zip(prof, ms)]
        nmv += nm
        flops += step_flops(plan, k, prec, inp["env_flops"], pk)
        host.append(ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = 1e3 * elapsed / args.steps
    value = flops / elapsed / 1e9
    lanczos_ms = 1e3 * statistics.median(t[1] for t in host)
    log(f"timed {args.steps} steps: {ms_step:.2f} ms/step, {value:.1f} GFLOP/s, lanczos {lanczos_ms:.2f} ms, E={e:.12f}")

    roofline = stage_rooflines(pk, plan, prec, args.prec, prof, nmv, args.workload)
    mv_ms, mv_flops, _ = matvec_time(pk, torch, inp, prec, stream)
    out = {"metric": METRIC, "value": round(value, 2), "unit": "GFLOP/s", "n_gpus": 1,
           "value_is": "algorithmic GFLOP of one bond update (host plan, 30-step Lanczos with one "
                       "matvec per step plus the FP64 Rayleigh-quotient matvec, both environment "
                       "updates) divided by its wall time; matvec_gflops is one heff_apply alone",
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": {pk.DM_FP64: "fp64", pk.DM_FP32: "fp32", pk.DM_BF16X3: "bf16x3"}[prec], "data": "synthetic",
           "config": {"workload": args.workload, "Ly": wl.Ly, "Lx": wl.Lx, "flux": f"{wl.flux[0]}/{wl.flux[1]}",
                      "chi": int(sum(wl.bonds[wl.j].values())), "sectors": len(wl.bonds[wl.j]),
                      "mpo_D": list(inp["D"]), "lanczos_iters": args.iters, "precision": args.prec,
                      "lanczos_fp64": True},
           "energy": e, "lanczos_steps": k,
           "lanczos_ms": round(lanczos_ms, 3),
           # host wall time per phase of a timed step (medians): plan creation, Lanczos
           # (synchronising), both environment updates (enqueued, not waited for)
           "phase_ms": {"plan": round(1e3 * statistics.median(t[0] for t in host), 3),
                        "lanczos": round(lanczos_ms, 3),
                        "env_updates": round(1e3 * statistics.median(t[2] for t in host), 3)},
           "matvec_ms": round(mv_ms, 4), "matvec_gflops": round(mv_flops / mv_ms / 1e6, 2),
           "matvec_gflop": round(mv_flops / 1e9, 4),
           "roofline": roofline,
           "matvec_roofline": matvec_roofline(pk, plan, prec, args.prec, mv_ms, roofline["stages"])}
    if not args.no_fp64_compare:
        log("precision comparison (cold and warm start) ...")
        out["precisions"] = precision_report(pk, torch, inp, args.iters, stream)
        p = out["precisions"]
        # Lanczos time of the solve alone (warm start, median of 3; the in-step figure
        # above also absorbs the previous step's queued environment updates)
        out["lanczos_warm_ms"] = p[args.prec]["lanczos_warm_ms"]
        out["speedup_vs_fp64"] = {
            q: {"matvec": round(p["fp64"]["matvec_ms"] / p[q]["matvec_ms"], 3),
                "lanczos": round(p["fp64"]["lanczos_warm_ms"] / p[q]["lanczos_warm_ms"], 3)}
            for q in ("fp32", "bf16x3")}
    if args.compare_real:
        log("real-space basis comparison ...")
        out["real_space"] = compare_real(pk, torch, wl, inp, prec, stream)
    if not args.no_eq_rot:
        out["eq_rot"] = eq_rot_report(pk, torch, wl, inp, args.iters, stream)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
