#!/usr/bin/env python3
"""Throughput of the interlaced PCS P(k) estimator on one MI355X.

Headline workload: 512^3 Zel'dovich-displaced particles (L = 2000 Mpc/h,
float32) -> PCS deposit on a 1024^3 grid and on the grid shifted by H/2 ->
3D FFT -> interlace + deconvolve -> P(k) in dk = k_f shells to Nyquist
(512 bins).  A step is one deposit -> transform -> power over the resident
particles.  Beside it (same JSON line): a batch of 64 uneven mocks on 128^3
grids replayed as one HIP graph, forward + backward of a P(k) loss for
128^3 particles on a 256^3 grid, the direct-summation engine, the
paper's own Zel'dovich shape (360^3 particles on a 480^3 mixed-radix grid),
the extensions (order 6, eight interlaced grids, masses) at 512^3, and
orders 1..4 with and without interlacing at the headline size.

Prints ONE JSON line on stdout; progress goes to stderr.
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

PEAK_HBM_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))

# HBM bytes per launch of a kernel group, from two rocprofv3 --pmc runs of
# this script (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), scaled by what
# the same counters read for a plain 1 GiB device copy (x2 for FETCH_SIZE,
# x1 for WRITE_SIZE).  They hold only for the kernel sources they were taken
# with: the SHA-256 prefix of those files is recorded, and a mismatch reports
# the traffic as unknown (null).
MEASURED_TRAFFIC = {
    "deposit": {
        "sources": ["paper_1512_07295_amd/csrc/deposit.hip",
                    "paper_1512_07295_amd/csrc/particles.hpp",
                    "paper_1512_07295_amd/csrc/fsest_internal.hpp"],
        "sha256_16": "ed4bfdfd521b6dbe",
        "workload": "pcs_il_n1024_za512",
        "read_bytes": 2 * 1835244 * 1024,
        "write_bytes": 8388618 * 1024,
    },
}


def measured_traffic(group, workload):
    """Counter-measured HBM bytes per launch, or None if stale/absent."""
    rec = MEASURED_TRAFFIC.get(group)
    if rec is None or rec["workload"] != workload:
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != rec["sha256_16"]:
        return None
    return rec["read_bytes"] + rec["write_bytes"]


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def algorithmic_bytes(label, n_particles, n, nz, n_grids, nkeys, sets=1):
    """Bytes a kernel group must move per launch (float32 positions, `sets`
    particle sets of n^3 cells each)."""
    cells = sets * n * n * nz
    return {
        # positions read twice (histogram, super-bucket pass); 16-byte
        # records written and read once in super-bucket order with their
        # 2-byte bucket index, and written once in bucket order
        # (12 + 12 + 18 + 18 + 16 B); bucket offsets and counts written
        "bucket_sort": 76 * n_particles + 8 * nkeys,
        # 16-byte records read once, every grid written once
        "deposit": 16 * n_particles + 4 * n_grids * sets * n * n * n,
        # complex grid read and written once per pass
        "fft_x": 16 * cells,
        "fft_y": 16 * cells,
        # complex grid read once (last-axis FFT, interlace, deconvolve, bin)
        "power_fused_z": 8 * cells,
        # adjoint: forward z FFT, gradient spectrum and inverse z FFT of the
        # grid read and written once; inverse y and x passes likewise
        "adjoint_fused_z": 16 * cells,
        "ifft_y": 16 * cells,
        "ifft_x": 16 * cells,
        # positions read, gradients written, every gradient grid read once
        "gather_grad": 24 * n_particles + 4 * n_grids * sets * n * n * n,
    }.get(label)


def stage_rooflines(prof, bytes_of, copy_gbs):
    """Per kernel group: ms per launch, fraction of the 8 TB/s HBM peak and
    of the measured copy bandwidth for its algorithmic bytes; and the
    dominant group's roofline entry."""
    stages, frac, frac_copy = {}, {}, {}
    dom = None
    for name, (ms, cnt) in prof.items():
        per = ms / cnt
        stages[name] = round(per, 4)
        b = bytes_of(name)
        if b:
            gbs = b / (per * 1e-3) / 1e9
            frac[name] = round(gbs / PEAK_HBM_GBS, 4)
            if copy_gbs:
                frac_copy[name] = round(gbs / copy_gbs, 4)
            if dom is None or per > dom[1]:
                dom = (name, per, b, gbs)
    roof = None
    if dom:
        name, per, b, gbs = dom
        roof = {"bound": "hbm", "kernel": name, "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
                "frac_of_measured_copy": round(gbs / copy_gbs, 4) if copy_gbs else None,
                "traffic": None, "algorithmic_bytes_per_launch": b, "ms_per_launch": round(per, 4)}
    return stages, frac, frac_copy, roof


def copy_bandwidth(torch, gib=2, reps=10):
    """Device-to-device copy of `gib` GiB (read + write counted), HIP events on
    the current stream, best of `reps`: the bandwidth a plain streaming
    kernel reaches on this GPU."""
    a = torch.ones(gib * 256 * 1024 * 1024, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    gbs = 2 * a.numel() * 4 / (best * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    log("device copy: %.1f GB/s (%d GiB, best of %d)" % (gbs, gib, reps))
    return gbs


PEAK_FP32_MATRIX_TFLOPS = 157.3


def closed_triangles(n_bins):
    """Every (b1, b2, b3) with b1 >= b2 >= b3 >= 1 and b1 <= b2 + b3."""
    out = []
    for b1 in range(1, n_bins + 1):
        for b2 in range(1, b1 + 1):
            for b3 in range(max(1, b1 - b2), b2 + 1):
                out.append((b1, b2, b3))
    return np.array(out, dtype=np.int32)


def bispectrum_mfma_work(tri, n_dk, n_bins):
    """(M, jobs) of the library's bispectrum for these triangles: the
    alias-free field grid (smallest 2^a 3^b 5^c above 3R, R the largest |m_a|
    of the shells) and the 16x16 MFMA tiles (fixed b1 - b2; 16 consecutive
    b2 by 16 consecutive b3) that cover the triangles."""
    r = ((2 * n_bins + 1) * n_dk - 1) // 2
    m = 3 * r + 1

    def smooth(v):
        for p in (2, 3, 5):
            while v % p == 0:
                v //= p
        return v == 1

    while not smooth(m):
        m += 1
    d = tri[:, 0] - tri[:, 1]
    bs = np.maximum(d, 1)
    keys = (d.astype(np.int64) * 64 + (tri[:, 1] - bs) // 16) * 64 + (tri[:, 2] - bs) // 16
    return m, len(np.unique(keys))


def bispectrum_leg(args, torch, F, est, n_dk=2, n_bins=128, copy_gbs=None):
    """FFT-shell bispectrum of the headline workload (the handle has just
    transformed it): 128 shells of 2 k_f up to k_N/2, every closed triangle.
    The first call also sums the counts (sum JJJ), later calls reuse them.
    Roofline: the MFMA triple sums (f32 16x16x4 tiles, flops the tiles
    execute) against the FP32 matrix peak."""
    tri = closed_triangles(n_bins)
    m, njobs = bispectrum_mfma_work(tri, n_dk, n_bins)
    nbytes = F.estimator_bispectrum_workspace_bytes(est.h, n_dk, n_bins, len(tri))
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    ptr = (buf.data_ptr() + 255) // 256 * 256
    bk = torch.empty(len(tri), dtype=torch.float64, device="cuda")
    nt = torch.empty_like(bk)
    times, profs = [], []
    for it in range(3):
        F.estimator_profile(est.h, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F.estimator_bispectrum(est.h, 0, n_dk, n_bins, tri, len(tri), ptr, nbytes, bk, nt)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        F.estimator_profile(est.h, 0)
        profs.append(F.profile_table(est.h))
        log("bispectrum call %d: %.3f s" % (it, times[-1]))
    del buf
    torch.cuda.empty_cache()
    cached = profs[-1]
    tri_ms = cached["bispec_triple"][0]
    passes = 1  # the cached calls sum the delta fields only
    mfma_flops = 2.0 * njobs * 256 * float(m) ** 3 * passes
    useful_flops = 2.0 * len(tri) * float(m) ** 3 * passes
    achieved = mfma_flops / (tri_ms * 1e-3) / 1e12
    return {"value": round(times[-1], 3), "unit": "s per call (count sums reused)",
            "first_call_s": round(times[0], 3), "calls_s": [round(t, 3) for t in times],
            "stage_ms_cached_call": {k: round(v[0], 2) for k, v in cached.items()},
            "stage_ms_first_call": {k: round(v[0], 2) for k, v in profs[0].items()},
            "field_grid": m, "mfma_tiles": njobs, "n_triangles": len(tri),
            "useful_gflops": round(useful_flops / times[-1] / 1e9, 1),
            "roofline": {"bound": "mfma", "kernel": "k_bs_triple (f32 16x16x4)",
                         "achieved": round(achieved, 2), "peak": PEAK_FP32_MATRIX_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_MATRIX_TFLOPS, 4),
                         "traffic": None,
                         "flops_per_call": mfma_flops, "ms_per_call": round(tri_ms, 2)},
            "config": {"workload": "FFT-shell bispectrum of the headline particles on the 1024^3 "
                                   "grid: 128 shells of 2 k_f (to k_N/2), all %d closed triangles; "
                                   "fields on the alias-free %d^3 grid" % (len(tri), m),
                       "n_dk": n_dk, "n_bins": n_bins}}


def headline(args, torch, F, est_mod, synth, copy_gbs=None):
    n_side, box, n = 512, 2000.0, 1024
    t0 = time.time()
    pos_h = synth.zeldovich(n_side, box, 3, dtype=np.float32)
    log("generated %d Zel'dovich particles in %.1f s" % (len(pos_h), time.time() - t0))
    pos = torch.as_tensor(pos_h, device="cuda")
    del pos_h
    npart = pos.shape[0]
    est = est_mod.Estimator(n, box, 4, True, 1, npart)
    n_bins = n // 2
    k = torch.empty((1, n_bins), dtype=torch.float64, device="cuda")
    pk = torch.empty_like(k)
    nm = torch.empty((1, n_bins), dtype=torch.int64, device="cuda")

    def step():
        F.estimator_deposit(est.h, pos, F.EST_F32, None, npart)
        F.estimator_transform(est.h)
        F.estimator_power(est.h, 1, n_bins, 0, k, pk, nm)

    t0 = time.time()
    if args.launch_choice is None:
        choice = est.autotune(pos, n_bins=n_bins, iters=2)
        log("autotuner picked launch shapes %d in %.1f s" % (choice, time.time() - t0))
    else:
        choice = args.launch_choice
        est.set_launch(choice)
        log("launch shapes %d (given)" % choice)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done (%d steps)" % args.warmup)
    F.estimator_profile(est.h, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    F.estimator_profile(est.h, 0)
    prof = F.profile_table(est.h)
    log("timed %d steps: %.3f ms/step" % (args.steps, 1e3 * dt / args.steps))
    for name, (ms, cnt) in sorted(prof.items(), key=lambda kv: -kv[1][0]):
        log("  %-16s %9.3f ms/launch  (%d launches)" % (name, ms / cnt, cnt))
    # dominant kernel group and its roofline
    nkeys = (n // 4) ** 3 + 1
    dom = max((kv for kv in prof.items() if algorithmic_bytes(kv[0], npart, n, n, 2, nkeys)),
              key=lambda kv: kv[1][0])
    name, (ms, cnt) = dom
    per_launch_ms = ms / cnt
    bytes_per = algorithmic_bytes(name, npart, n, n, 2, nkeys)
    achieved = bytes_per / (per_launch_ms * 1e-3) / 1e9
    stages = {kname: round(v[0] / v[1], 4) for kname, v in prof.items()}
    roof_all, roof_copy = {}, {}
    for kname, (kms, kcnt) in prof.items():
        b = algorithmic_bytes(kname, npart, n, n, 2, nkeys)
        if b:
            roof_all[kname] = round(b / (kms / kcnt * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
            if copy_gbs:
                roof_copy[kname] = round(b / (kms / kcnt * 1e-3) / 1e9 / copy_gbs, 4)
    result = {
        "value": npart * args.steps / dt / 1e6,
        "ms_per_step": 1e3 * dt / args.steps,
        "npart": npart,
        "roofline": {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": measured_traffic(name, "pcs_il_n1024_za512"),
                     "algorithmic_bytes_per_launch": bytes_per,
                     "ms_per_launch": round(per_launch_ms, 4),
                     "measured_copy_gbs": round(copy_gbs, 1) if copy_gbs else None,
                     "frac_of_measured_copy": round(achieved / copy_gbs, 4) if copy_gbs else None},
        "stage_ms": stages,
        "stage_hbm_frac": roof_all,
        "stage_copy_frac": roof_copy,
        "launch_choice": choice,
        "p_first_bins": [float(x) for x in pk[0, :4].cpu().numpy()],
    }
    if not args.no_bispectrum:
        result["bispectrum"] = bispectrum_leg(args, torch, F, est, copy_gbs=copy_gbs)
    est.close()
    del pos
    torch.cuda.empty_cache()
    return result


def batched(args, torch, F, est_mod, synth, copy_gbs=None):
    box, n, n_mocks = 500.0, 128, 64
    t0 = time.time()
    pos_h, offs_h = synth.mocks(n_mocks, box, 100)
    log("generated %d mocks (%d particles) in %.1f s" % (n_mocks, len(pos_h), time.time() - t0))
    pos = torch.as_tensor(pos_h, device="cuda")
    offs = torch.as_tensor(offs_h, device="cuda")
    npart = len(pos_h)
    est = est_mod.Estimator(n, box, 4, True, n_mocks, npart)
    choice = est.autotune(pos, offsets=offs, iters=2)
    log("autotuner picked candidate %d" % choice)
    est.capture(pos, offsets=offs)
    for _ in range(args.warmup):
        est.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        est.replay()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log("batched: %.3f ms per graph replay" % (1e3 * dt / args.steps))
    # stage breakdown: the same three calls made directly (events are not
    # recorded inside a captured graph)
    k = torch.empty((n_mocks, n // 2), dtype=torch.float64, device="cuda")
    pk = torch.empty_like(k)
    nm = torch.empty((n_mocks, n // 2), dtype=torch.int64, device="cuda")
    F.estimator_profile(est.h, 1)
    t1 = time.perf_counter()
    for _ in range(args.steps):
        F.estimator_deposit(est.h, pos, F.EST_F32, offs, npart)
        F.estimator_transform(est.h)
        F.estimator_power(est.h, 1, n // 2, 0, k, pk, nm)
    torch.cuda.synchronize()
    dt_direct = time.perf_counter() - t1
    F.estimator_profile(est.h, 0)
    prof = F.profile_table(est.h)
    nkeys = n_mocks * (n // 4) ** 3 + 1
    stages, frac, frac_copy, roof = stage_rooflines(
        prof, lambda name: algorithmic_bytes(name, npart, n, n, 2, nkeys, sets=n_mocks), copy_gbs)
    for name, ms in sorted(stages.items(), key=lambda kv: -kv[1]):
        log("  batched %-14s %8.3f ms" % (name, ms))
    est.close()
    return {"value": npart * args.steps / dt / 1e6, "unit": "Mparticles/s",
            "ms_per_step": 1e3 * dt / args.steps, "autotune_choice": choice,
            "ms_per_step_direct_calls": round(1e3 * dt_direct / args.steps, 4),
            "stage_ms": stages, "stage_hbm_frac": frac, "stage_copy_frac": frac_copy,
            "roofline": roof,
            "config": {"workload": "64 mocks, Poisson counts around log-uniform means in [1e5, 4e6] "
                                   "(even uniform, odd Zel'dovich), L=500, 128^3 grids, PCS + "
                                   "interlacing, one HIP graph replay per step",
                       "n_particles": npart}}


def fwd_bwd(args, torch, F, est_mod, synth, copy_gbs=None):
    box, n, n_bins = 1000.0, 256, 128
    pos = torch.as_tensor(synth.zeldovich(128, box, 5, dtype=np.float32), device="cuda")
    tgt = torch.as_tensor(synth.zeldovich(128, box, 6, dtype=np.float32), device="cuda")
    npart = pos.shape[0]
    est = est_mod.Estimator(n, box, 4, True, 1, npart)
    _, target, counts = est.power(tgt, n_bins=n_bins)
    sigma2 = 2 * target ** 2 / counts.double()

    def step():
        x = pos.detach().requires_grad_(True)
        p = est_mod.PowerSpectrumFn.apply(x, est, 1, n_bins, None)
        loss = ((p - target) ** 2 / sigma2).sum()
        loss.backward()
        return x.grad

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log("fwd+bwd: %.3f ms per step" % (1e3 * dt / args.steps))
    # stage breakdown (forward and adjoint kernel groups) over as many steps
    F.estimator_profile(est.h, 1)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    F.estimator_profile(est.h, 0)
    prof = F.profile_table(est.h)
    nkeys = (n // 4) ** 3 + 1
    # per launch (groups such as the sort and deposit run twice per step:
    # forward and the adjoint's recomputation)
    per_launch = {name: (ms / cnt, 1) for name, (ms, cnt) in prof.items()}
    _, frac, frac_copy, roof = stage_rooflines(
        per_launch, lambda name: algorithmic_bytes(name, npart, n, n, 2, nkeys), copy_gbs)
    stages = {name: round(ms / args.steps, 4) for name, (ms, cnt) in prof.items()}
    launches = {name: int(cnt) // args.steps for name, (ms, cnt) in prof.items()}
    for name, ms in sorted(stages.items(), key=lambda kv: -kv[1]):
        log("  fwd+bwd %-16s %8.3f ms per step (%d launches)" % (name, ms, launches[name]))
    est.close()
    return {"value": npart * args.steps / dt / 1e6, "unit": "Mparticles/s",
            "ms_per_step": 1e3 * dt / args.steps,
            "stage_ms_per_step": stages, "stage_launches_per_step": launches,
            "stage_hbm_frac": frac, "stage_copy_frac": frac_copy, "roofline": roof,
            "config": {"workload": "128^3 Zel'dovich particles, L=1000, 256^3 grid, PCS + interlacing, "
                                   "chi^2 loss of 128 P(k) bins vs a second seed, forward + adjoint",
                       "n_particles": npart}}


def orders_leg(args, torch, F, est_mod, synth):
    """The headline workload (512^3 Zel'dovich particles, 1024^3 grid) with
    every order p = 1..4, with and without interlacing (same step; launch
    shapes autotuned for each order and interlacing choice)."""
    n_side, box, n = 512, 2000.0, 1024
    pos = torch.as_tensor(synth.zeldovich(n_side, box, 3, dtype=np.float32), device="cuda")
    npart = pos.shape[0]
    n_bins = n // 2
    k = torch.empty((1, n_bins), dtype=torch.float64, device="cuda")
    pk = torch.empty_like(k)
    nm = torch.empty((1, n_bins), dtype=torch.int64, device="cuda")
    out = {}
    for order in (1, 2, 3, 4):
        for il in (0, 1):
            est = est_mod.Estimator(n, box, order, il, 1, npart)
            choice = est.autotune(pos, n_bins=n_bins, iters=2)

            def step():
                F.estimator_deposit(est.h, pos, F.EST_F32, None, npart)
                F.estimator_transform(est.h)
                F.estimator_power(est.h, 1, n_bins, 0, k, pk, nm)

            for _ in range(args.warmup):
                step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                step()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            est.close()
            torch.cuda.empty_cache()
            name = "p%d_%s" % (order, "interlaced" if il else "single")
            out[name] = {"value": round(npart * args.steps / dt / 1e6, 2), "unit": "Mparticles/s",
                         "ms_per_step": round(1e3 * dt / args.steps, 4), "launch_choice": choice}
            log("orders %s: %.3f ms per step" % (name, 1e3 * dt / args.steps))
    out["config"] = {"workload": "512^3 Zel'dovich particles, L=2000, 1024^3 grid, P(k) in k_f "
                                 "shells to Nyquist, launch shapes autotuned per order", "n_particles": npart}
    del pos
    torch.cuda.empty_cache()
    return out


def paper_za_leg(args, torch, F, est_mod, synth):
    """The paper's Zel'dovich measurement shape (Sec. 3.3): 360^3 particles,
    L = 2400 Mpc/h, N_G = 480 (2^5 3 5: mixed-radix FFT), PCS + interlacing,
    P(k) in k_f shells to Nyquist.  Same step as the headline."""
    n_side, box, n = 360, 2400.0, 480
    pos = torch.as_tensor(synth.zeldovich(n_side, box, 7, dtype=np.float32), device="cuda")
    npart = pos.shape[0]
    est = est_mod.Estimator(n, box, 4, True, 1, npart)
    n_bins = n // 2
    k = torch.empty((1, n_bins), dtype=torch.float64, device="cuda")
    pk = torch.empty_like(k)
    nm = torch.empty((1, n_bins), dtype=torch.int64, device="cuda")

    def step():
        F.estimator_deposit(est.h, pos, F.EST_F32, None, npart)
        F.estimator_transform(est.h)
        F.estimator_power(est.h, 1, n_bins, 0, k, pk, nm)

    choice = est.autotune(pos, n_bins=n_bins, iters=2)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    F.estimator_profile(est.h, 1)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    F.estimator_profile(est.h, 0)
    prof = F.profile_table(est.h)
    est.close()
    log("paper ZA 480^3: %.3f ms per step" % (1e3 * dt / args.steps))
    nkeys = (n // 4) ** 3 + 1
    frac = {}
    for kname, (kms, kcnt) in prof.items():
        b = algorithmic_bytes(kname, npart, n, n, 2, nkeys)
        if b:
            frac[kname] = round(b / (kms / kcnt * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
    return {"value": round(npart * args.steps / dt / 1e6, 2), "unit": "Mparticles/s",
            "ms_per_step": round(1e3 * dt / args.steps, 4), "launch_choice": choice,
            "stage_ms": {kname: round(v[0] / v[1], 4) for kname, v in prof.items()},
            "stage_hbm_frac": frac,
            "config": {"workload": "360^3 Zel'dovich particles, L=2400, 480^3 grid (mixed radix), "
                                   "PCS + interlacing, P(k) in k_f shells to Nyquist (240 bins)",
                       "n_particles": npart}}


def variants_leg(args, torch, F, est_mod, synth):
    """The headline step with the paper's extensions, on 256^3 Zel'dovich
    particles and a 512^3 grid (L = 1000): order 6, eight interlaced grids,
    per-particle masses; each against the plain PCS + pair at the same size."""
    n_side, box, n = 256, 1000.0, 512
    pos = torch.as_tensor(synth.zeldovich(n_side, box, 9, dtype=np.float32), device="cuda")
    npart = pos.shape[0]
    masses = torch.as_tensor(np.random.default_rng(1).exponential(1.0, npart).astype(np.float32),
                             device="cuda")
    out = {}
    for name, order, code, weighted in (("pcs_pair", 4, 1, False), ("order6_pair", 6, 1, False),
                                        ("pcs_eight_grids", 4, 3, False),
                                        ("pcs_pair_masses", 4, 1, True)):
        est = est_mod.Estimator(n, box, order, code, 1, npart, weighted=weighted)
        if weighted:
            est.set_weights(masses)
        n_bins = n // 2
        k = torch.empty((1, n_bins), dtype=torch.float64, device="cuda")
        pk = torch.empty_like(k)
        nm = torch.empty((1, n_bins), dtype=torch.int64, device="cuda")

        def step():
            F.estimator_deposit(est.h, pos, F.EST_F32, None, npart)
            F.estimator_transform(est.h)
            F.estimator_power(est.h, 1, n_bins, 0, k, pk, nm)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        F.estimator_profile(est.h, 1)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        F.estimator_profile(est.h, 0)
        prof = F.profile_table(est.h)
        est.close()
        out[name] = {"value": round(npart * args.steps / dt / 1e6, 2), "unit": "Mparticles/s",
                     "ms_per_step": round(1e3 * dt / args.steps, 4),
                     "stage_ms": {kname: round(v[0] / v[1], 4) for kname, v in prof.items()}}
        log("variant %s: %.3f ms per step" % (name, 1e3 * dt / args.steps))
    out["config"] = {"workload": "256^3 Zel'dovich particles, L=1000, 512^3 grid, P(k) in k_f shells "
                                 "to Nyquist; default launch shapes", "n_particles": npart}
    return out


PEAK_FP32_VECTOR_TFLOPS = 157.3


def direct_leg(args, torch, est_mod, synth):
    """Direct summation delta_DS (eq. deltaDS) of 64^3 Zel'dovich particles
    over every half-spectrum mode of a 64^3 grid; ALU-bound.  Algorithmic
    work per (particle, mode) term: one complex multiply and one complex add,
    8 flops, against the FP32 vector peak."""
    box, n, n_side = 500.0, 64, 64
    pos = torch.as_tensor(synth.zeldovich(n_side, box, 12, dtype=np.float32), device="cuda")
    npart = pos.shape[0]
    est = est_mod.Estimator(n, box, 4, True, 1, npart)
    terms = npart * n * n * (n // 2 + 1)
    for _ in range(max(1, args.warmup // 2)):
        est.direct_delta(pos)
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        est.direct_delta(pos)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    est.close()
    tflops = 8.0 * terms / dt / 1e12
    log("direct sum: %.2f ms per call, %.3g terms/s" % (1e3 * dt, terms / dt))
    return {"value": round(terms / dt / 1e9, 2), "unit": "Gterms/s", "ms_per_call": round(1e3 * dt, 3),
            "roofline": {"bound": "alu", "achieved": round(tflops, 2), "peak": PEAK_FP32_VECTOR_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(tflops / PEAK_FP32_VECTOR_TFLOPS, 4),
                         "traffic": None, "flops_per_term": 8},
            "config": {"workload": "delta_DS of 64^3 Zel'dovich particles (L=500) at every "
                                   "half-spectrum mode of a 64^3 grid",
                       "n_particles": npart, "terms": terms}}


def bias_experiment(torch, est_mod, synth, n_side=192, n=128, box=1000.0):
    """Sec. 3.2 on synthetic Zel'dovich particles: |P_G/P_DS - 1| and
    |P_{G-DS}/P_DS - 1| per shell for p = 1..4 with and without interlacing,
    P_DS from the GPU direct sum (one JSON line per configuration)."""
    pos = torch.as_tensor(synth.zeldovich(n_side, box, 50, dtype=np.float32), device="cuda")
    est = est_mod.Estimator(n, box, 4, True, 1, pos.shape[0])
    t0 = time.perf_counter()
    dds = est.direct_delta(pos)
    log("bias: direct sum of %d particles on %d^3 modes in %.1f s" % (pos.shape[0], n, time.perf_counter() - t0))
    k, p_ds, nm = est.spectrum_power(dds)
    p_ds = p_ds.cpu().numpy()
    k_n = np.pi * n / box
    for order in (1, 2, 3, 4):
        for il in (False, True):
            e = est_mod.Estimator(n, box, order, il, 1, pos.shape[0])
            e.deposit(pos)
            e.transform()
            dg = e.export_delta()
            _, p_g, _ = e.spectrum_power(dg)
            _, p_x, _ = e.spectrum_power(dg, dds)
            e.close()
            print(json.dumps({"order": order, "interlace": il,
                              "k_over_kN": [round(float(v) / k_n, 4) for v in k.cpu().numpy()],
                              "abs_PG_over_PDS_m1": [float("%.3g" % v) for v in np.abs(p_g.cpu().numpy() / p_ds - 1)],
                              "abs_PGDS_over_PDS_m1": [float("%.3g" % v) for v in np.abs(p_x.cpu().numpy() / p_ds - 1)]}),
                  flush=True)
    est.close()


def cpu_baseline():
    """The FP64 oracle on the 256^3 configuration: 256^3 Zel'dovich particles
    (L = 1000), 256^3 grid, PCS + interlacing, P(k) in k_f shells to Nyquist;
    one run (about 20-30 s of CPU work)."""
    import oracle
    import synth
    workers = len(os.sched_getaffinity(0))
    try:
        ram_gb = os.sysconf("SC_PAGE_SIZE") * os.sysconf("SC_PHYS_PAGES") / 1e9
    except (ValueError, OSError):
        ram_gb = None
    pos = synth.zeldovich(256, 1000.0, 2, dtype=np.float32)
    t0 = time.perf_counter()
    oracle.power(pos, 1000.0, 256, 4, True, 1, 128, workers=workers)
    dt = time.perf_counter() - t0
    log("cpu oracle, 256^3 particles on 256^3: %.1f s" % dt)
    return {"value": round(len(pos) / dt / 1e6, 4), "unit": "Mparticles/s", "cores": workers,
            "kind": "oracle", "host_ram_gb": round(ram_gb, 1) if ram_gb else None,
            "sample": "the 256^3 configuration: 256^3 Zel'dovich particles (L=1000) on a 256^3 "
                      "grid, PCS + interlacing, P(k) in k_f shells to Nyquist (1/8 of the "
                      "headline particles, 1/64 of its cells); FP64 numpy deposit on one core, "
                      "scipy FFT on %d threads; one run of %.1f s" % (workers, dt)}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-extra", action="store_true", help="skip the batched and fwd+bwd legs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bispectrum", action="store_true", help="skip the bispectrum leg")
    ap.add_argument("--launch-choice", type=int, default=None,
                    help="headline launch shapes (0..47) instead of autotuning them")
    ap.add_argument("--bias", action="store_true",
                    help="only run the aliasing comparison against direct summation (Sec. 3.2)")
    ap.add_argument("--leg", choices=["batched", "fwd_bwd", "direct_sum", "paper_za_480", "variants",
                                      "orders_1024"],
                    default=None, help="only run one of the extra legs (for profiling)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.calib_copy:
        a = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": a.numel() * 4, "copies": 3}), flush=True)
        return
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import paper_1512_07295_amd as F
    from paper_1512_07295_amd import estimator as est_mod
    import synth

    if args.bias:
        bias_experiment(torch, est_mod, synth)
        return
    if args.leg:
        legs = {"batched": lambda: batched(args, torch, F, est_mod, synth, copy_bandwidth(torch)),
                "fwd_bwd": lambda: fwd_bwd(args, torch, F, est_mod, synth, copy_bandwidth(torch)),
                "direct_sum": lambda: direct_leg(args, torch, est_mod, synth),
                "paper_za_480": lambda: paper_za_leg(args, torch, F, est_mod, synth),
                "variants": lambda: variants_leg(args, torch, F, est_mod, synth),
                "orders_1024": lambda: orders_leg(args, torch, F, est_mod, synth)}
        print(json.dumps({"leg": args.leg, "result": legs[args.leg]()}), flush=True)
        return

    copy_gbs = copy_bandwidth(torch)
    head = headline(args, torch, F, est_mod, synth, copy_gbs)
    extra = {}
    if "bispectrum" in head:
        extra["bispectrum"] = head.pop("bispectrum")
    if not args.no_extra:
        extra["batched"] = batched(args, torch, F, est_mod, synth, copy_gbs)
        extra["fwd_bwd"] = fwd_bwd(args, torch, F, est_mod, synth, copy_gbs)
        extra["direct_sum"] = direct_leg(args, torch, est_mod, synth)
        extra["paper_za_480"] = paper_za_leg(args, torch, F, est_mod, synth)
        extra["variants"] = variants_leg(args, torch, F, est_mod, synth)
        extra["orders_1024"] = orders_leg(args, torch, F, est_mod, synth)
    out = {
        "metric": "Mparticles/s end-to-end P(k), PCS+interlace 1024^3 grid; fwd+bwd & batched vs plain",
        "value": round(head["value"], 2),
        "unit": "Mparticles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "512^3 Zel'dovich particles (P(k) ~ k^-1.5, rms displacement 0.3 "
                               "lattice spacing, L=2000 Mpc/h, float32) -> 1024^3 grid, PCS (p=4) "
                               "+ interlacing, P(k) in k_f shells to Nyquist (512 bins)",
                   "n_particles": head["npart"], "n_grid": 1024, "order": 4, "interlace": True,
                   "parallelism": "single GPU"},
        "roofline": head["roofline"],
        "stage_ms": head["stage_ms"],
        "stage_hbm_frac": head["stage_hbm_frac"],
        "stage_copy_frac": head["stage_copy_frac"],
        "measured_copy_gbs": round(copy_gbs, 1),
        "launch_choice": head["launch_choice"],
    }
    out.update(extra)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
