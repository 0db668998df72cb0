"""Benchmark of the TaylorGrid SDF-fitting hot path on one MI355X.

Workload (the paper's 3D SDF fitting task, Sec. 3.2, at the 128^3 resolution of Table 1/2):
128^3 vertices on [-1,1]^3, order K=2 (10 FP32 coefficients per vertex), 2^20 queries per
step (half uniform in the box, half jittered points on a seeded union of 8 spheres and a
torus), L1 reconstruction + 0.1 * eikonal, Adam lr 1e-2.  One step = bucketing sort +
forward (f, grad f) with the loss in its epilogue + the coefficient adjoint with the Adam
update of every coefficient applied in the same pass.  The separate calls (forward, loss,
backward, Adam) are timed too; their forward + backward is the fwd+bwd figure.  Query
batches are generated on the host before timing and are resident in HBM.

Further sections (each can be switched off by a flag) time the precision forms, the full
SDF objective, the quality measures, the order scaling, the radiance-field form and serving;
the CPU baseline times the FP64 oracle on a bounded sample of the same steps.

Prints one JSON line.  --gpus must be 1: the path runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2402_14415_amd import synth  # noqa: E402  (input generators only)

METRIC = "queries/s fwd+bwd at 128^3 K=2 (and % HBM peak); served query p50/p99 latency"
HBM_PEAK_GBS = 8000.0
COPY_REF_BYTES = 256 << 20
FLUSH_BYTES = 512 << 20  # written before a cold repetition: twice the 256 MB Infinity Cache
# VALU issue peak: 1024 SIMDs each issuing one wave64 FP32 instruction every 4 cycles at 2.4 GHz
VALU_WAVE_INSTR_PEAK = 1024 * 2.4e9 / 4
# VALU wave instructions per wave of 64 served points of k_query (SQ_INSTS_VALU / SQ_WAVES =
# 9.335e6 / 2.057e4 per dispatch), from the SQ counter pass of the serving section
# (profiles/sq_counters_serving_kernel.md)
QUERY_VALU_PER_WAVE = 453.8
RES = 128
ORDER = 2
NQ = 1 << 20
EIK = 0.1
LR = 1e-2


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def unique_vertices(q, res, lo=-1.0, hi=1.0):
    h = (hi - lo) / (res - 1)
    c = np.minimum(np.floor((np.clip(q, lo, hi) - lo) / h).astype(np.int64), res - 2)
    ids = []
    for b in range(8):
        v = c + np.array([(b >> a) & 1 for a in range(3)])
        ids.append(v[:, 0] + res * (v[:, 1] + res * v[:, 2]))
    return int(np.unique(np.concatenate(ids)).size)


def algorithmic_bytes(nq, U, C, nvert):
    """Bytes each call must move (what the method needs, not what the kernels happen to
    move); U = distinct vertices the batch touches."""
    fwd = nq * (12 + 16) + U * C * 4          # read q, write f and grad f; read touched coefficients
    loss = nq * (4 + 12 + 4) + nq * (4 + 12)  # read f, grad f, d; write g_f, g_grad
    bwd = nq * (12 + 16) + U * C * 4          # read q, g_f, g_grad; write touched gradients
    adam = nvert * C * 4 * 7                  # read master, m, v, grad; write master, m, v
    fwd_loss = nq * (12 + 4 + 16) + U * C * 4  # read q, d; write g_f, g_grad; read touched coefficients
    # (the training step keeps d and the upstream gradients in bucket order; the bytes are the same)
    bwd_adam = nq * (12 + 16) + nvert * C * 4 * 6  # read q, g_f, g_grad; read and write master, m, v
    return {"sort": 0, "forward": fwd, "loss": loss, "backward": bwd, "adam": adam,
            "forward_loss": fwd_loss, "backward_adam": bwd_adam}


def unique_vertices_dev(q, res, lo=-1.0, hi=1.0):
    """Distinct vertices the queries q (a device tensor [n, 3]) touch, counted on the device
    with a bitmap (input analysis for the algorithmic byte counts, not the method)."""
    import torch

    h = (hi - lo) / (res - 1)
    c = torch.clamp(torch.floor((torch.clamp(q.double(), lo, hi) - lo) / h).long(), max=res - 2)
    seen = torch.zeros(res ** 3, dtype=torch.bool, device=q.device)
    for b in range(8):
        v = c + torch.tensor([(b >> a) & 1 for a in range(3)], device=q.device)
        seen[v[:, 0] + res * (v[:, 1] + res * v[:, 2])] = True
    return int(seen.sum())


def percentiles(xs):
    xs = np.asarray(xs, dtype=np.float64)
    return {"median": float(np.median(xs)), "p10": float(np.percentile(xs, 10)), "p90": float(np.percentile(xs, 90))}


def fwd_bwd_bench(grid, q, gf, gg, ws, f, g, reps=200, warmup=20, flush=None, packed=False):
    """The metric's forward + backward: tg_forward (f, grad f in query order) then
    tg_backward (dC from precomputed upstream gradients) on one stream, timed with HIP events
    per repetition, and the bucketing sort that both reuse.  With `packed`, f is the [n, 4]
    output of tg_forward_packed and gf the [n, 4] packed upstream (g, gg unused).  With `flush` (a 512 MiB device
    buffer) the Infinity Cache (MALL) is flushed before the sort and again between the sort
    and the forward, by rewriting the buffer outside the timed windows.  Returns per-repetition
    medians and p10 / p90 in microseconds (sort_fwd_bwd adds the sort's window to fwd_bwd's)."""
    import torch

    s = torch.cuda.current_stream(q.device)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(reps)]
    for e5 in evs:
        for e in e5:
            e.record(s)
    torch.cuda.synchronize()
    for i in range(warmup + reps):
        e = evs[i - warmup] if i >= warmup else None
        if flush is not None:
            flush.add_(1.0)
        e and e[0].record(s)
        grid.sort(q, ws)
        e and e[1].record(s)
        if flush is not None:
            flush.add_(1.0)
        e and e[2].record(s)
        if packed:
            grid.forward_packed(q, ws, out=f)
        else:
            grid.forward(q, ws, out=(f, g))
        e and e[3].record(s)
        if packed:
            grid.backward(q, ws, packed=gf)
        else:
            grid.backward(q, ws, gf, gg)
        e and e[4].record(s)
    torch.cuda.synchronize()
    us = lambda a, b: np.array([1e3 * e[a].elapsed_time(e[b]) for e in evs])
    return {"fwd_bwd": percentiles(us(2, 4)), "sort_fwd_bwd": percentiles(us(0, 1) + us(2, 4)),
            "sort": percentiles(us(0, 1)), "forward": percentiles(us(2, 3)), "backward": percentiles(us(3, 4))}


def strip_comments(src):
    """C/C++ source without its comments and with runs of whitespace collapsed, so that a
    change to comments alone leaves the kernel hash unchanged (string and character literals
    are kept as they are)."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_sha256():
    """Hash of the library's sources (comments excluded): the counter summaries record it, and
    their traffic figures are used only while it matches."""
    import glob
    import hashlib

    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(ROOT, "paper_2402_14415_amd", "csrc", "*"))):
        h.update(os.path.basename(path).encode())
        with open(path, encoding="utf-8") as fh:
            h.update(strip_comments(fh.read()).encode())
    return h.hexdigest()


def measured_traffic(call):
    """HBM bytes per launch of `call` from the committed counter summary, or None when the
    kernels have changed since the counters were taken (source hash mismatch)."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_sdf_fit_128_K2_fp32.md")
    if not os.path.exists(path):
        return None
    vals, sha = {}, None
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic_bytes_per_launch:"):
                for kv in line.split(":", 1)[1].split():
                    k, v = kv.split("=")
                    vals[k] = float(v)
            elif line.startswith("kernel_source_sha256:"):
                sha = line.split(":", 1)[1].strip()
    if sha != kernel_source_sha256():
        return None
    return vals.get(call)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _omp_threads(n):
    """Set the OpenMP thread count of this process (the oracle's loops)."""
    import ctypes

    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


def cpu_baseline(C64, batches, min_seconds=10.0, max_steps=64, single_queries=1 << 18):
    """The FP64 oracle on the same step (forward + loss + adjoint over a batch of 2^20
    queries, then Adam over every coefficient), on the host cores, repeated over the bench's
    batches until at least min_seconds of work have run; then on one thread, the same step
    over the first single_queries queries of a batch."""
    import oracle

    geom = oracle.Geometry(3, (RES,) * 3, ORDER, (-1.0,) * 3, (1.0,) * 3)
    flat = C64.reshape(-1).copy()
    m = np.zeros_like(flat)
    v = np.zeros_like(flat)

    def one_step(q, d, step):
        nonlocal flat, m, v
        f, g = oracle.forward(geom, flat.reshape(C64.shape), q)
        _, gf, gg = oracle.sdf_loss(f, g, d, EIK)
        dC, _ = oracle.backward(geom, flat.reshape(C64.shape), q, gf, gg)
        flat, m, v, _ = oracle.adam(flat, m, v, dC.reshape(-1), LR, step=step)

    threads = oracle.threads()
    _omp_threads(threads)
    steps, nq = 0, 0
    t0 = time.perf_counter()
    while steps < max_steps and (steps == 0 or time.perf_counter() - t0 < min_seconds):
        q, d = batches[steps % len(batches)]
        one_step(q, d, steps + 1)
        steps += 1
        nq += len(q)
    dt = time.perf_counter() - t0
    q, d = batches[0]
    _omp_threads(1)
    t1 = time.perf_counter()
    one_step(q[:single_queries], d[:single_queries], steps + 1)
    dt1 = time.perf_counter() - t1
    _omp_threads(threads)
    return {"value": nq / dt, "unit": "queries/s", "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{steps} full training steps of {len(batches[0][0])} scene queries each at {RES}^3 K={ORDER} "
                      f"(forward + loss + adjoint + Adam over {flat.size} coefficients), FP64, {dt:.1f} s",
            "single_thread": {"value": single_queries / dt1, "unit": "queries/s", "cores": 1,
                              "sample": f"one training step of {single_queries} scene queries (forward + loss + "
                                        f"adjoint, then Adam over every coefficient), FP64, {dt1:.1f} s"}}


def serving_bench(dev, batches_dev, n_req=400, fit_steps=20):
    """Serving form: 16 resident BF16 grids (resolution log-uniform in [64, 256], order 1 or
    2, each fitted to the scene for a few Adam steps), requests of log-uniform 1e3..4e6
    uniform points.  Saturated throughput first (all requests queued at once), then Poisson
    arrivals at 50% and 90% of the saturated request rate; latency = completion - arrival."""
    import torch

    from paper_2402_14415_amd.grid import TaylorGrid, sdf_loss
    from paper_2402_14415_amd.serving import Server, run_trace

    rng = np.random.default_rng(2)
    gen = torch.Generator(device=dev)
    gen.manual_seed(2)
    grids, desc = [], []
    for k in range(16):
        res = int(round(np.exp(rng.uniform(np.log(64), np.log(256)))))
        order = int(rng.integers(1, 3))
        C = (order + 1) * (order + 2) * (order + 3) // 6
        C0 = torch.randn((res, res, res, C), generator=gen, device=dev) * 0.05
        g = TaylorGrid(3, (res,) * 3, order, (-1.0,) * 3, (1.0,) * 3, storage="bf16", coeffs=C0, device=dev)
        del C0
        nq = batches_dev[0][0].shape[0]
        ws = g.workspace(nq)
        for it in range(fit_steps):
            q, d = batches_dev[it % len(batches_dev)]
            g.sort(q, ws)
            f, gr = g.forward(q, ws)
            _, gf, gg = sdf_loss(f, gr, d, EIK, ws)
            g.backward(q, ws, gf, gg)
            g.adam_step(ws, lr=LR)
        torch.cuda.synchronize()
        srv_g = TaylorGrid(3, (res,) * 3, order, (-1.0,) * 3, (1.0,) * 3, storage="bf16", coeffs=g.master,
                           device=dev, optimizer=False)
        del g, ws
        grids.append(srv_g)
        desc.append({"res": res, "order": order})
    torch.cuda.synchronize()
    torch.cuda.empty_cache()

    log(f"bench: serving grids fitted: {desc}")
    nmax = 4_000_000
    pool = torch.rand((2 * nmax, 3), generator=gen, device=dev) * 2.0 - 1.0

    # the serving kernel alone: one launch of 16 requests of 2^20 uniform points, one per grid
    from paper_2402_14415_amd.grid import query

    npk = 1 << 20
    kreqs, alg_bytes = [], 0
    for k in range(16):
        qk = pool[k * npk:(k + 1) * npk]
        kreqs.append((k, qk, torch.empty(npk, device=dev), torch.empty((npk, 3), device=dev)))
        Ck = (desc[k]["order"] + 1) * (desc[k]["order"] + 2) * (desc[k]["order"] + 3) // 6
        alg_bytes += npk * 28 + unique_vertices_dev(qk, desc[k]["res"]) * Ck * 2  # BF16 coefficients
    kev = [torch.cuda.Event(enable_timing=True) for _ in range(11)]
    for e in kev:
        e.record()
    query(grids, kreqs)
    torch.cuda.synchronize()
    kev[0].record()
    for r in range(10):
        query(grids, kreqs)
        kev[r + 1].record()
    torch.cuda.synchronize()
    k_us = float(np.median([kev[r].elapsed_time(kev[r + 1]) * 1e3 for r in range(10)]))
    kpts = 16 * npk
    kernel = {"points": kpts, "us": k_us, "points_per_s": kpts / (k_us * 1e-6),
              "hbm": {"algorithmic_bytes": alg_bytes, "achieved_GBs": alg_bytes / (k_us * 1e-6) / 1e9,
                      "peak": HBM_PEAK_GBS, "frac": alg_bytes / (k_us * 1e-6) / 1e9 / HBM_PEAK_GBS},
              "valu": None if QUERY_VALU_PER_WAVE is None else {
                  "wave_instructions_per_wave": QUERY_VALU_PER_WAVE,
                  "achieved_wave_instr_per_s": QUERY_VALU_PER_WAVE * kpts / 64 / (k_us * 1e-6),
                  "peak_wave_instr_per_s": VALU_WAVE_INSTR_PEAK,
                  "frac": QUERY_VALU_PER_WAVE * kpts / 64 / (k_us * 1e-6) / VALU_WAVE_INSTR_PEAK}}
    log(f"bench: serving kernel: {kernel}")
    del kreqs

    def make_requests(seed):
        r = np.random.default_rng(seed)
        out = []
        for _ in range(n_req):
            n = int(round(np.exp(r.uniform(np.log(1e3), np.log(4e6)))))
            off = int(r.integers(0, nmax))
            out.append((int(r.integers(0, 16)), pool[off:off + n]))
        return out

    res = {"grids": desc, "requests_per_phase": n_req, "budget_bytes": 1 << 30, "fit_steps": fit_steps,
           "kernel": kernel}
    srv = Server(grids, budget_bytes=1 << 30, streams=2, depth=4, chunk_points=1 << 20)
    # warm-up pass (allocator, kernels)
    run_trace(srv, [(0.0, g, q) for g, q in make_requests(9)[:40]])
    sat = run_trace(srv, [(0.0, g, q) for g, q in make_requests(10)])
    torch.cuda.synchronize()
    log(f"bench: serving saturated: {sat}")
    res["saturated"] = sat
    mean_n = sat["points"] / sat["requests"]
    sat_rate = sat["queries_per_s"] / mean_n
    for frac, seed in ((0.5, 11), (0.9, 12)):
        lam = frac * sat_rate
        r = np.random.default_rng(seed)
        reqs = make_requests(seed)
        arr = np.cumsum(r.exponential(1.0 / lam, size=len(reqs)))
        out = run_trace(srv, [(float(t), g, q) for t, (g, q) in zip(arr, reqs)])
        torch.cuda.synchronize()
        out["arrival_rate_per_s"] = lam
        res[f"poisson_{int(frac * 100)}pct"] = out
    return res


def precision_bench(dev, steps=10, warmup=3, n_batches=2):
    """Precision form at 256^3, K=2, 2^22 queries per step: the training step with FP32, BF16
    and FP16 coefficient storage (FP32 master and accumulation), every form starting from the
    same coefficients; the separate calls and the fused tg_train_step are both timed.  Then
    each trained grid's field on 2^16 held-out scene points (seed 1) against the FP64 oracle:
    the arithmetic error (oracle on the storage-rounded coefficients the kernels read) and the
    deployment error (oracle on the FP32 master), max and RMS of f_GPU - f_oracle."""
    import torch

    import oracle
    from paper_2402_14415_amd.grid import TaylorGrid, sdf_loss

    res, nq = 256, 1 << 22
    scene = synth.Scene(0)
    batches = []
    for b in range(n_batches):
        q, d = synth.scene_batch(scene, nq, seed=0, step=100 + b)
        batches.append((torch.tensor(q, dtype=torch.float32, device=dev), torch.tensor(d, dtype=torch.float32, device=dev)))
    qh64, _ = synth.scene_batch(scene, 1 << 16, seed=1, step=0)
    qh64 = qh64.astype(np.float32).astype(np.float64)
    qh = torch.tensor(qh64, dtype=torch.float32, device=dev)
    C0 = torch.from_numpy(synth.normal_coeffs((res, res, res, 10), std=0.05, seed=0)[0].astype(np.float32))
    geom = oracle.Geometry(3, (res,) * 3, 2, (-1.0,) * 3, (1.0,) * 3)
    out = {"workload": "sdf_fit_256^3_K2", "queries_per_step": nq, "steps": steps, "held_out_points": len(qh64),
           "forms": {}}
    for storage in ("f32", "bf16", "f16"):
        grid = TaylorGrid(3, (res,) * 3, 2, (-1.0,) * 3, (1.0,) * 3, storage=storage, coeffs=C0, device=dev)
        ws = grid.workspace(nq)
        f = torch.empty(nq, device=dev)
        g = torch.empty((nq, 3), device=dev)
        gf = torch.empty(nq, device=dev)
        gg = torch.empty((nq, 3), device=dev)
        loss = torch.empty(3, dtype=torch.float64, device=dev)
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(steps)]
        for it in range(warmup + steps):
            q, d = batches[it % len(batches)]
            e = evs[it - warmup] if it >= warmup else None
            e and e[0].record()
            grid.sort(q, ws)
            e and e[1].record()
            grid.forward(q, ws, out=(f, g))
            e and e[2].record()
            sdf_loss(f, g, d, EIK, ws, g_f=gf, g_grad=gg, loss=loss)
            e and e[3].record()
            grid.backward(q, ws, gf, gg)
            e and e[4].record()
            grid.adam_step(ws, lr=LR)
            e and e[5].record()
        torch.cuda.synchronize()
        names = ["sort", "forward", "loss", "backward", "adam"]
        us = {nm: 1e3 * float(np.mean([e[k].elapsed_time(e[k + 1]) for e in evs])) for k, nm in enumerate(names)}
        step_us = 1e3 * float(np.mean([e[0].elapsed_time(e[5]) for e in evs]))
        # the fused training step, continuing from the same state
        fev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
        for e4 in fev:
            for e in e4:
                e.record()
        torch.cuda.synchronize()
        for it in range(steps):
            q, d = batches[it % len(batches)]
            fev[it][0].record()
            grid.train_step(q, d, ws, eik_weight=EIK, lr=LR, loss=loss, stage_events=fev[it][1:])
        torch.cuda.synchronize()
        fused_us = 1e3 * float(np.mean([e[0].elapsed_time(e[3]) for e in fev]))
        fused_stage = {nm: 1e3 * float(np.mean([e[k].elapsed_time(e[k + 1]) for e in fev]))
                       for k, nm in enumerate(["sort", "forward_loss", "backward_adam"])}
        # the trained grid's field on the held-out points against the FP64 oracle
        wsh = grid.workspace(qh.shape[0])
        grid.sort(qh, wsh)
        fh, _ = grid.forward(qh, wsh, want_grad=False)
        torch.cuda.synchronize()
        fh64 = fh.double().cpu().numpy()
        master64 = grid.master.double().cpu().numpy()
        stored64 = master64 if storage == "f32" else grid.coeffs.double().cpu().numpy()
        errs = {}
        for name, C in (("arithmetic", stored64), ("deployment", master64)):
            e = fh64 - oracle.forward(geom, C, qh64, want_grad=False)
            errs[name] = {"max": float(np.max(np.abs(e))), "rms": float(np.sqrt(np.mean(e * e)))}
        del master64, stored64
        out["forms"][storage] = {
            "us_per_call": us, "step_us": step_us, "step_queries_per_s": nq / (step_us * 1e-6),
            "fwd_bwd_queries_per_s": nq / ((us["forward"] + us["backward"]) * 1e-6),
            "fused_step_us": fused_us, "fused_step_queries_per_s": nq / (fused_us * 1e-6),
            "fused_stage_us": fused_stage,
            "sdf_error_vs_fp64_oracle": errs, "final_loss": float(loss[0])}
        log(f"bench: precision {storage}: {out['forms'][storage]}")
        del grid, ws, wsh
        torch.cuda.empty_cache()
    return out


def radiance_bench(dev, steps=10, warmup=3, train_steps=2000, n_pool=64, n_heldout=8, n_rays=4096, n_samples=256,
                   res=160):
    """Radiance-field form: a 160^3 density grid (K=2, ReLU) and a three-channel K=1 colour grid,
    4096 rays x 256 stratified samples per step from cameras on a radius-4 sphere.  Targets
    are the ray colours of the seeded blob volume, rendered by the library's own compositing
    from the volume's density and colour at the samples.  One step evaluates the two grids
    (one shared sort, a forward each), composites with the photometric loss and its adjoint,
    and applies the fused adjoint + Adam to each grid.  The step is timed per stage, then the
    fit runs to train_steps steps over a pool of n_pool batches, and the PSNR of the rendered
    colours against the targets is measured on n_heldout batches of other rays (seed 1)
    before and after, as the paper reports PSNR of its radiance fields (Sec. 4.2)."""
    import torch

    from paper_2402_14415_amd.radiance import RadianceField, composite

    vol = synth.BlobVolume(0)
    rng = np.random.default_rng(0)
    field = RadianceField((res,) * 3, coeffs=(
        torch.from_numpy((0.5 + 0.05 * rng.standard_normal((res, res, res, 10))).astype(np.float32)),
        [torch.from_numpy((0.5 + 0.05 * rng.standard_normal((res, res, res, 4))).astype(np.float32))
         for _ in range(3)]), device=dev)

    def make_batch(seed, b):
        o, d = synth.camera_rays(n_rays, seed=seed, step=b)
        q64, delta64 = synth.stratified_samples(o, d, n_samples, seed=seed, step=b)
        q = torch.tensor(q64, dtype=torch.float32, device=dev)
        delta = torch.tensor(delta64, dtype=torch.float32, device=dev)
        dens, col = vol.density_and_colour_torch(q)
        rgb = composite(dens.float().contiguous(), col.t().float().contiguous(), delta, n_samples,
                        field.reduce_ws)[0]
        return q, delta, rgb

    batches = [make_batch(0, b) for b in range(n_pool)]
    heldout = [make_batch(1, b) for b in range(n_heldout)]
    n = n_rays * n_samples
    ws = field.workspace(n)

    def psnr():
        se, cnt = 0.0, 0
        for q, delta, target in heldout:
            rgb = field.render(q, delta, n_samples, ws)
            se += float(((rgb.double() - target.double()) ** 2).sum())
            cnt += target.numel()
        return -10.0 * math.log10(se / cnt)  # colours in [0, 1]: peak 1

    psnr0 = psnr()
    bufs = (torch.empty(n, device=dev), torch.empty((3, n), device=dev), torch.empty((n_rays, 3), device=dev),
            torch.empty(1, dtype=torch.float64, device=dev), torch.empty(n, device=dev),
            torch.empty((3, n), device=dev))
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps + warmup)]
    for e4 in ev:
        for e in e4:
            e.record()
    torch.cuda.synchronize()
    losses = []
    for i in range(steps + warmup):
        q, delta, target = batches[i % n_pool]
        ev[i][0].record()
        loss = field.train_step(q, delta, n_samples, target, ws, lr=1e-2, bufs=bufs, stage_events=ev[i][1:])
        if i == 0:
            losses.append(float(loss[0]))
    torch.cuda.synchronize()
    stage = lambda k: float(np.median([ev[i][k].elapsed_time(ev[i][k + 1]) * 1e3 for i in range(warmup, warmup + steps)]))
    step_us = float(np.median([ev[i][0].elapsed_time(ev[i][3]) * 1e3 for i in range(warmup, warmup + steps)]))
    comp_us = stage(1)
    t0 = time.perf_counter()
    for i in range(steps + warmup, train_steps):
        q, delta, target = batches[i % n_pool]
        loss = field.train_step(q, delta, n_samples, target, ws, lr=1e-2, bufs=bufs)
    torch.cuda.synchronize()
    fit_s = time.perf_counter() - t0
    losses.append(float(loss[0]))
    psnr1 = psnr()
    comp_bytes = n * 36 + n_rays * 24  # f, 3 colours, delta in; g_f, 3 g_c out; target in, colour out
    return {"workload": f"radiance_{res}^3_density_K2_relu_colour_K1x3ch", "rays_per_step": n_rays,
            "composite_kernel": {"us": comp_us, "algorithmic_bytes": comp_bytes,
                                 "GBs": comp_bytes / (comp_us * 1e-6) / 1e9,
                                 "frac": comp_bytes / (comp_us * 1e-6) / 1e9 / HBM_PEAK_GBS},
            "samples_per_ray": n_samples, "step_us": step_us, "rays_per_s": n_rays / (step_us * 1e-6),
            "samples_per_s": n / (step_us * 1e-6),
            "stage_us": {"sort_and_evaluate_2_grids": stage(0), "composite_loss_adjoint": stage(1),
                         "adjoint_adam_2_grids": stage(2)},
            "train_steps": train_steps, "training_pool_rays": n_pool * n_rays,
            "fit_seconds_after_timing": fit_s, "loss_first_last": losses,
            "heldout_rays": n_heldout * n_rays, "psnr_db_before": psnr0, "psnr_db_after": psnr1}


def objective_bench(dev, C32, dev_batches, U, steps=10, warmup=3):
    """The paper's full SDF objective at the headline size (128^3, K=2, 2^20 scene queries):
    L1 weighted by Eq. 7 (k = ln 3 / (2 h): half weight two cells from the surface) + 0.1
    eikonal + 2e-5 TV (Sec. 4.1's lambda_2), one tg_train_step per step; the TV kernel and the
    coarse-to-fine transfer (64^3 -> 128^3) timed on their own with HIP events."""
    import torch

    from paper_2402_14415_amd.grid import TaylorGrid

    h = 2.0 / (RES - 1)
    k = math.log(3.0) / (2.0 * h)
    grid = TaylorGrid(3, (RES,) * 3, ORDER, (-1.0,) * 3, (1.0,) * 3, coeffs=C32, device=dev)
    ws = grid.workspace(NQ)
    loss = torch.empty(4, dtype=torch.float64, device=dev)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps + warmup)]
    for e4 in ev:
        for e in e4:
            e.record()
    torch.cuda.synchronize()
    losses = []
    for i in range(steps + warmup):
        q, d = dev_batches[i % len(dev_batches)]
        ev[i][0].record()
        grid.train_step(q, d, ws, eik_weight=EIK, lr=LR, loss=loss, surface_k=k, tv_weight=2e-5,
                        stage_events=ev[i][1:])
        if i == 0 or i == steps + warmup - 1:
            losses.append([float(x) for x in loss.cpu()])
    torch.cuda.synchronize()
    med = lambda a, b: float(np.median([ev[i][a].elapsed_time(ev[i][b]) * 1e3 for i in range(warmup, warmup + steps)]))
    step_us = med(0, 3)
    # the TV kernel alone (reads and writes every coefficient once)
    red = torch.empty(grid.workspace_bytes(0), dtype=torch.uint8, device=dev)
    tv_ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    for e in tv_ev:
        e.record()
    torch.cuda.synchronize()
    tv_ev[0].record()
    for i in range(steps):
        grid.tv_loss(2e-5, red)
        tv_ev[i + 1].record()
    torch.cuda.synchronize()
    tv_us = float(np.median([tv_ev[i].elapsed_time(tv_ev[i + 1]) * 1e3 for i in range(steps)]))
    tv_bytes = RES ** 3 * 10 * 8
    # coarse-to-fine transfer 64^3 -> 128^3
    coarse = TaylorGrid(3, (64,) * 3, ORDER, (-1.0,) * 3, (1.0,) * 3,
                        coeffs=C32[::2, ::2, ::2].contiguous(), device=dev)
    up_ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    for e in up_ev:
        e.record()
    torch.cuda.synchronize()
    up_ev[0].record()
    for i in range(steps):
        grid.upsample_from(coarse)
        up_ev[i + 1].record()
    torch.cuda.synchronize()
    up_us = float(np.median([up_ev[i].elapsed_time(up_ev[i + 1]) * 1e3 for i in range(steps)]))
    up_bytes = RES ** 3 * 10 * 12 + 64 ** 3 * 10 * 4  # master + two moments written, coarse read once
    return {"workload": "sdf_fit_128^3_K2_fp32_full_objective",
            "objective": {"eik_weight": EIK, "surface_k": k, "tv_weight": 2e-5},
            "step_us": step_us, "queries_per_s": NQ / (step_us * 1e-6),
            "stage_us": {"sort": med(0, 1), "tv_and_forward_loss": med(1, 2), "backward_adam": med(2, 3)},
            "loss_first_last": losses,
            "tv_kernel": {"us": tv_us, "algorithmic_bytes": tv_bytes, "GBs": tv_bytes / (tv_us * 1e-6) / 1e9,
                          "frac": tv_bytes / (tv_us * 1e-6) / 1e9 / HBM_PEAK_GBS},
            "upsample_64_to_128": {"us": up_us, "algorithmic_bytes": up_bytes,
                                   "GBs": up_bytes / (up_us * 1e-6) / 1e9}}


def quality_bench(dev, dev_batches, scene, fit_steps=1000, n_points=100_000, n_surface=100_000, reps=5,
                  lattice=2):
    """Quality of 128^3 grids of order 0, 1 and 2 fitted to the scene (from zero coefficients,
    fit_steps training steps of the headline loss over the headline batches each: the 3D
    SDF-fitting workload's 1000 steps) against the analytic scene, as the paper evaluates its
    reconstructions (Sec. 4.1): IoU of the inside sets on uniform points, and the Chamfer-L1
    distance between the mesh that marching cubes extracts from the learned field (on the
    lattice `lattice` times finer than the grid) and points on the scene's surface; the
    Euclidean Chamfer distance beside it.  The evaluation kernels of the K = 2 grid are timed
    with HIP events."""
    import torch

    from paper_2402_14415_amd import quality
    from paper_2402_14415_amd.grid import TaylorGrid

    rng = np.random.default_rng(11)
    pts = torch.tensor(rng.uniform(-1, 1, size=(n_points, 3)), dtype=torch.float32, device=dev)
    d = torch.tensor(scene.sdf(pts.cpu().double().numpy()), dtype=torch.float32, device=dev)
    surf = torch.tensor(scene.surface_points(np.random.default_rng(12), n_surface), dtype=torch.float32, device=dev)

    def timed(fn):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        for e in ev:
            e.record()
        torch.cuda.synchronize()
        ev[0].record()
        for i in range(reps):
            r = fn()
            ev[i + 1].record()
        torch.cuda.synchronize()
        return r, float(np.median([ev[i].elapsed_time(ev[i + 1]) * 1e3 for i in range(reps)]))

    orders, kernels = {}, {}
    for order in (0, 1, 2):
        grid = TaylorGrid(3, (RES,) * 3, order, (-1.0,) * 3, (1.0,) * 3, device=dev)
        wfit = grid.workspace(NQ)
        loss = torch.empty(3, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(fit_steps):
            q, dd = dev_batches[i % len(dev_batches)]
            grid.train_step(q, dd, wfit, eik_weight=EIK, lr=LR, loss=loss)
        torch.cuda.synchronize()
        fit_s = time.perf_counter() - t0
        fit_loss = float(loss[0])
        del wfit
        ws = grid.workspace(n_points)
        red = torch.empty(grid.workspace_bytes(0), dtype=torch.uint8, device=dev)

        def evaluate():
            grid.sort(pts, ws)
            return grid.forward(pts, ws, want_grad=False)[0]

        f, fwd_us = timed(evaluate)
        counts = torch.empty(2, dtype=torch.int64, device=dev)
        _, iou_us = timed(lambda: quality.iou_counts(f, d, red, counts))
        iou, inter, union = quality.iou(f, d, red)
        vals, lat_us = timed(lambda: quality.field_lattice(grid, lattice))
        tri, total = quality.mesh(vals, (-1.0,) * 3, (1.0,) * 3)
        lat = quality.MeshLattice(vals.shape, (-1.0,) * 3, (1.0,) * 3, dev)
        tri2 = torch.empty_like(tri)
        _, mesh_us = timed(lambda: lat.run(vals, tri2, total))
        mv = tri.reshape(-1, 3).contiguous()
        out = torch.empty(3, dtype=torch.float64, device=dev)
        chws = quality.chamfer_workspace(mv.shape[0], surf.shape[0], dev)
        _, ch_us = timed(lambda: quality.chamfer_into(mv, surf, out, chws, norm=1))
        ch = [float(x) for x in out.cpu()]
        quality.chamfer_into(mv, surf, out, chws, norm=2)
        ch2 = [float(x) for x in out.cpu()]
        orders[f"K{order}"] = {"fit_seconds": fit_s, "fit_loss": fit_loss, "iou": iou, "triangles": total,
                               "chamfer_l1": ch[0], "chamfer_l1_mesh_to_surface": ch[1],
                               "chamfer_l1_surface_to_mesh": ch[2], "chamfer_euclidean": ch2[0]}
        log(f"bench: quality K={order}: " + json.dumps(orders[f"K{order}"]))
        if order == 2:
            n_lat = vals.numel()
            pairs = 2 * mv.shape[0] * surf.shape[0]
            mesh_bytes = 2 * n_lat * 4 + total * 36  # the lattice read by both passes, the triangles written
            kernels = {"us": {"sort_and_forward": fwd_us, "iou_counts": iou_us, "field_lattice": lat_us,
                              "mesh": mesh_us, "chamfer": ch_us},
                       "lattice_points": n_lat,
                       "mesh_kernel": {"algorithmic_bytes": mesh_bytes, "GBs": mesh_bytes / (mesh_us * 1e-6) / 1e9,
                                       "frac": mesh_bytes / (mesh_us * 1e-6) / 1e9 / HBM_PEAK_GBS},
                       # exact nearest points on bucket grids: the rate against comparing every pair
                       "chamfer_kernel": {"points": int(mv.shape[0] + surf.shape[0]),
                                          "points_per_s": (mv.shape[0] + surf.shape[0]) / (ch_us * 1e-6),
                                          "every_pair_equivalent": pairs}}
        del grid, ws, vals, tri, tri2, mv, chws, lat
    return {"workload": f"quality_of_sdf_fit_{RES}^3_by_order", "fit_steps": fit_steps, "iou_points": n_points,
            "surface_points": n_surface, "mesh": f"marching cubes of the field on the lattice {lattice}x finer",
            "orders": orders, "kernels_K2": kernels}


def order_scaling_bench(dev, dev_batches, steps=10, warmup=3):
    """Time and bytes against the Taylor order at the headline size (128^3, 2^20 scene queries
    per step, the headline step): K = 0, 1, 2 and order 2 with the full 3 x 3 Hessian stored
    (13 coefficients per vertex).  Ratios are to K = 0; the paper's Table 2 reports, for its
    Linear / 1st Taylor / Taylor grids at 128^3, training times 7.0 / 27.1 / 95.0 s and sizes
    9.2 / 32.7 / 106.0 MB (ratios 1 : 3.9 : 13.6 and 1 : 3.6 : 11.5)."""
    import torch

    from paper_2402_14415_amd.grid import TaylorGrid

    rows = {}
    for name, order, layout in (("K0", 0, "symmetric"), ("K1", 1, "symmetric"), ("K2", 2, "symmetric"),
                                ("K2_full_hessian", 2, "full")):
        g = TaylorGrid(3, (RES,) * 3, order, (-1.0,) * 3, (1.0,) * 3, device=dev, hessian=layout)
        gen = torch.Generator(device=dev)
        gen.manual_seed(0)
        g.master.copy_(torch.randn(g.shape, generator=gen, device=dev) * 0.05)
        ws = g.workspace(NQ)
        loss = torch.empty(3, dtype=torch.float64, device=dev)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        for e in ev:
            e.record()
        for i in range(warmup):
            q, d = dev_batches[i % len(dev_batches)]
            g.train_step(q, d, ws, eik_weight=EIK, lr=LR, loss=loss)
        torch.cuda.synchronize()
        ev[0].record()
        for i in range(steps):
            q, d = dev_batches[i % len(dev_batches)]
            g.train_step(q, d, ws, eik_weight=EIK, lr=LR, loss=loss)
            ev[i + 1].record()
        torch.cuda.synchronize()
        us = float(np.median([ev[i].elapsed_time(ev[i + 1]) * 1e3 for i in range(steps)]))
        rows[name] = {"coeffs_per_vertex": g.C, "coeff_MB": RES ** 3 * g.C * 4 / 1e6, "step_us": us}
        del g, ws
    t0, b0 = rows["K0"]["step_us"], rows["K0"]["coeff_MB"]
    for r in rows.values():
        r["time_ratio"] = r["step_us"] / t0
        r["size_ratio"] = r["coeff_MB"] / b0
    return {"workload": f"sdf_fit_{RES}^3_order_scaling", "rows": rows,
            "paper_table2_ratios": {"time": [1.0, 27.1 / 7.0, 95.0 / 7.0], "size": [1.0, 32.7 / 9.2, 106.0 / 9.2]}}


def nq_sweep(grid, dev_batches, exps=(20, 21, 22, 23, 24), reps=20, warmup=5):
    """Forward + backward (warm) at 2^20 .. 2^24 scene queries on the headline grid.  Batches
    beyond the four distinct 2^20 ones repeat them with N(0, 1e-3) jitter (the spatial mix is
    unchanged); upstream gradients are seeded normals scaled by 1/n."""
    import torch

    rows = {}
    base = torch.cat([q for q, _ in dev_batches])
    gen = torch.Generator(device=base.device)
    gen.manual_seed(3)
    for e in exps:
        n = 1 << e
        parts, have = [], 0
        while have < n:
            take = min(n - have, base.shape[0])
            blk = base[:take]
            if have >= base.shape[0]:
                blk = torch.clamp(blk + 1e-3 * torch.randn(blk.shape, generator=gen, device=blk.device), -1.0, 1.0)
            parts.append(blk)
            have += take
        q = torch.cat(parts).contiguous()
        gf = torch.randn(n, generator=gen, device=q.device) / n
        gg = torch.randn((n, 3), generator=gen, device=q.device) / n
        f = torch.empty(n, device=q.device)
        g = torch.empty((n, 3), device=q.device)
        ws = grid.workspace(n)
        U = unique_vertices_dev(q, RES)
        r = fwd_bwd_bench(grid, q, gf, gg, ws, f, g, reps=reps, warmup=warmup)
        b = algorithmic_bytes(n, U, 10, RES ** 3)
        fb_bytes = b["forward"] + b["backward"]
        t, ts = r["fwd_bwd"]["median"], r["sort_fwd_bwd"]["median"]
        rows[f"2^{e}"] = {"queries": n, "unique_vertices": U, "fwd_bwd_us": t, "sort_fwd_bwd_us": ts,
                          "queries_per_s": n / (t * 1e-6), "queries_per_s_with_sort": n / (ts * 1e-6),
                          "frac": fb_bytes / (t * 1e-6) / 1e9 / HBM_PEAK_GBS,
                          "frac_with_sort": fb_bytes / (ts * 1e-6) / 1e9 / HBM_PEAK_GBS}
        log(f"bench: sweep 2^{e}: " + json.dumps(rows[f"2^{e}"]))
        del q, gf, gg, f, g, ws
        torch.cuda.empty_cache()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--batches", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-breakdown", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-radiance", action="store_true")
    ap.add_argument("--no-objective", action="store_true")
    ap.add_argument("--no-quality", action="store_true")
    ap.add_argument("--no-order-scaling", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--fwd-bwd-reps", type=int, default=200,
                    help="repetitions of the warm and the cold fwd+bwd measurement (each after 20 warm-up)")
    ap.add_argument("--copy-reference", action="store_true",
                    help="end with device-to-device copies of 256 MiB (the reference kernel that scales the "
                         "FETCH_SIZE / WRITE_SIZE counters of a profiling run)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this path runs on one GPU only (no multi-GPU path is built); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2402_14415_amd.grid import TaylorGrid, sdf_loss

    dev = torch.device("cuda", 0)
    log("bench: generating inputs")
    C64, _ = synth.normal_coeffs((RES, RES, RES, 10), std=0.05, seed=0)
    scene = synth.Scene(0)
    batches = []
    for b in range(args.batches):
        q, d = synth.scene_batch(scene, NQ, seed=0, step=b)
        batches.append((q, d))
    U = unique_vertices(batches[0][0], RES)

    grid = TaylorGrid(3, (RES,) * 3, ORDER, (-1.0,) * 3, (1.0,) * 3,
                      coeffs=torch.from_numpy(C64.astype(np.float32)), device=dev)
    dev_batches = [(torch.tensor(q, dtype=torch.float32, device=dev), torch.tensor(d, dtype=torch.float32, device=dev))
                   for q, d in batches]
    ws = grid.workspace(NQ)
    f = torch.empty(NQ, device=dev)
    g = torch.empty((NQ, 3), device=dev)
    gf = torch.empty(NQ, device=dev)
    gg = torch.empty((NQ, 3), device=dev)
    loss = torch.empty(3, dtype=torch.float64, device=dev)
    gns = torch.empty(1, dtype=torch.float64, device=dev)

    def step(i, ev=None):
        """The training step as it runs in production: one call that sorts, evaluates the
        field with the loss in its epilogue and applies the adjoint with Adam in the same
        pass (the target and the upstream gradients stay in bucket order)."""
        q, d = dev_batches[i % len(dev_batches)]
        if ev is not None:
            ev[0].record(torch.cuda.current_stream(dev))
        grid.train_step(q, d, ws, eik_weight=EIK, lr=LR, loss=loss, grad_norm_sq=gns,
                        stage_events=ev[1:] if ev is not None else None)

    def step_unfused(i, ev):
        """The same step through the separate calls (forward, loss, backward, Adam)."""
        q, d = dev_batches[i % len(dev_batches)]
        s = torch.cuda.current_stream(dev)
        ev[0].record(s)
        grid.sort(q, ws)
        ev[1].record(s)
        grid.forward(q, ws, out=(f, g))
        ev[2].record(s)
        sdf_loss(f, g, d, EIK, ws, g_f=gf, g_grad=gg, loss=loss)
        ev[3].record(s)
        grid.backward(q, ws, gf, gg)
        ev[4].record(s)
        grid.adam_step(ws, lr=LR, grad_norm_sq=gns)
        ev[5].record(s)

    log("bench: warmup")
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    first_loss = float(loss[0])

    log("bench: timed region")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = NQ / (elapsed / args.steps)
    log(f"bench: {ms_per_step:.3f} ms/step, {value:.3e} queries/s, loss {first_loss:.4f} -> {float(loss[0]):.4f}")

    C = 10
    nvert = RES ** 3
    alg = algorithmic_bytes(NQ, U, C, nvert)
    per_call_us, unfused_us = {}, {}
    if not args.no_breakdown:
        # Per-call durations from HIP events recorded on the stream the kernels run on.
        reps = max(10, args.steps)
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(reps)]
        for e4 in evs:  # create the events before their handles are passed down
            for e in e4:
                e.record()
        torch.cuda.synchronize()
        for i in range(reps):
            step(i, evs[i])
        torch.cuda.synchronize()
        for k, nm in enumerate(["sort", "forward_loss", "backward_adam"]):
            per_call_us[nm] = 1e3 * float(np.mean([e[k].elapsed_time(e[k + 1]) for e in evs]))
        log("bench: per-call us " + json.dumps({k: round(v, 2) for k, v in per_call_us.items()}))
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(reps)]
        for i in range(reps):
            step_unfused(i, evs[i])
        torch.cuda.synchronize()
        for k, nm in enumerate(["sort", "forward", "loss", "backward", "adam"]):
            unfused_us[nm] = 1e3 * float(np.mean([e[k].elapsed_time(e[k + 1]) for e in evs]))
        log("bench: unfused per-call us " + json.dumps({k: round(v, 2) for k, v in unfused_us.items()}))

    step_alg = alg["forward_loss"] + alg["backward_adam"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sdf_fit_128^3_K2_fp32", "grid_vertices": f"{RES}^3", "order": ORDER,
                   "queries_per_step": NQ, "loss": "L1 + 0.1*eikonal", "optimizer": "Adam lr=1e-2",
                   "step": "tg_train_step: sort + forward with loss epilogue + adjoint with Adam in the same pass",
                   "unique_vertices": U},
        "step_hbm": {"algorithmic_bytes": step_alg,
                     "achieved_GBs": step_alg / (ms_per_step * 1e-3) / 1e9,
                     "frac": step_alg / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS},
    }
    if per_call_us:
        dom = max(per_call_us, key=lambda k: per_call_us[k])
        ach = alg[dom] / (per_call_us[dom] * 1e-6) / 1e9
        traffic = measured_traffic(dom)
        out["roofline"] = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
                           "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                           "algorithmic_bytes": alg[dom]}
        # the metric's forward + backward (query-order outputs, precomputed upstream gradients),
        # warm and with the Infinity Cache flushed before each repetition
        q0, d0 = dev_batches[0]
        grid.sort(q0, ws)
        grid.forward(q0, ws, out=(f, g))
        sdf_loss(f, g, d0, EIK, ws, g_f=gf, g_grad=gg, loss=loss)
        flush = torch.zeros(FLUSH_BYTES // 4, dtype=torch.float32, device=dev)
        fb_bytes = alg["forward"] + alg["backward"]
        fb = {"algorithmic_bytes": fb_bytes, "unique_vertices": U, "repetitions": args.fwd_bwd_reps,
              "flush_bytes": FLUSH_BYTES}
        # the same calls with (f, grad f) and (g_f, g_grad) packed in one 16-byte row per query
        fg4 = torch.empty((NQ, 4), device=dev)
        up4 = torch.cat([gf[:, None], gg], dim=1).contiguous()
        fb["packed"] = {"layout": "tg_forward_packed + tg_backward(TG_BWD_PACKED): [n][4] rows (f, grad f) "
                                  "and (g_f, g_grad)"}
        for lay, dst in (("separate", fb), ("packed", fb["packed"])):
            for mode, fl in (("warm", None), ("cold", flush)):
                if lay == "packed":
                    r = fwd_bwd_bench(grid, q0, up4, None, ws, fg4, None, reps=args.fwd_bwd_reps, flush=fl,
                                      packed=True)
                else:
                    r = fwd_bwd_bench(grid, q0, gf, gg, ws, f, g, reps=args.fwd_bwd_reps, flush=fl)
                t, ts = r["fwd_bwd"]["median"], r["sort_fwd_bwd"]["median"]
                r["queries_per_s"] = NQ / (t * 1e-6)
                r["frac"] = fb_bytes / (t * 1e-6) / 1e9 / HBM_PEAK_GBS
                r["queries_per_s_with_sort"] = NQ / (ts * 1e-6)
                r["frac_with_sort"] = fb_bytes / (ts * 1e-6) / 1e9 / HBM_PEAK_GBS
                dst[mode] = r
                log(f"bench: fwd+bwd {mode} ({lay}): {t:.1f} us ({r['frac']:.3f} of HBM peak), "
                    f"with the sort {ts:.1f} us")
        del flush, fg4, up4
        out["fwd_bwd"] = fb
        # the metric's forward + backward beside the dominant kernel: fractions of HBM peak,
        # warm and cold, without and with the sort both calls reuse, for both output layouts
        out["roofline"]["fwd_bwd_frac"] = {m: {"frac": fb[m]["frac"], "frac_with_sort": fb[m]["frac_with_sort"]}
                                           for m in ("warm", "cold")}
        out["roofline"]["fwd_bwd_frac"]["packed"] = {
            m: {"frac": fb["packed"][m]["frac"], "frac_with_sort": fb["packed"][m]["frac_with_sort"]}
            for m in ("warm", "cold")}
        # The same batch handed over in brick order (its points and upstream gradients permuted
        # together; the results are the same values, permuted): what the query-order scatter
        # of f, grad f and the gather of g_f, g_grad cost in the calls above.
        cell = torch.clamp(((q0 + 1.0) * ((RES - 1) / 2.0)).floor().long(), 0, RES - 2)
        bk = cell // 8
        nb = (RES + 7) // 8
        loc = cell % 8
        key = ((bk[:, 2] * nb + bk[:, 1]) * nb + bk[:, 0]) * 512 + loc[:, 0] + 8 * loc[:, 1] + 64 * loc[:, 2]
        order = torch.argsort(key)
        qc, gfc, ggc = q0[order].contiguous(), gf[order].contiguous(), gg[order].contiguous()
        rc = fwd_bwd_bench(grid, qc, gfc, ggc, ws, f, g, reps=args.fwd_bwd_reps)
        tc = rc["fwd_bwd"]["median"]
        fb["brick_ordered_batch"] = {"fwd_bwd": rc["fwd_bwd"], "forward": rc["forward"], "backward": rc["backward"],
                                     "queries_per_s": NQ / (tc * 1e-6), "frac": fb_bytes / (tc * 1e-6) / 1e9 / HBM_PEAK_GBS}
        log(f"bench: fwd+bwd warm, the batch in brick order: {tc:.1f} us ({fb['brick_ordered_batch']['frac']:.3f} of HBM peak)")
        if not args.no_sweep:
            out["nq_sweep"] = nq_sweep(grid, dev_batches)
        out["breakdown_us"] = per_call_us
        out["unfused_breakdown_us"] = unfused_us
        out["kernels"] = {nm: {"us": t, "algorithmic_bytes": alg[nm], "GBs": alg[nm] / (t * 1e-6) / 1e9}
                          for nm, t in list(per_call_us.items()) + list(unfused_us.items()) if alg.get(nm)}
    if not args.no_precision:
        log("bench: precision forms")
        out["precision"] = precision_bench(dev)
    if not args.no_order_scaling:
        log("bench: order scaling")
        out["order_scaling"] = order_scaling_bench(dev, dev_batches)
        log(f"bench: order scaling {json.dumps(out['order_scaling'])}")
    if not args.no_quality:
        log("bench: quality of the fitted grid")
        out["quality"] = quality_bench(dev, dev_batches, scene)
        log(f"bench: quality {json.dumps(out['quality'])}")
    if not args.no_objective:
        log("bench: full SDF objective")
        out["full_objective"] = objective_bench(dev, torch.from_numpy(C64.astype(np.float32)), dev_batches, U)
        log(f"bench: full objective {json.dumps(out['full_objective'])}")
    if not args.no_radiance:
        log("bench: radiance form")
        out["radiance"] = radiance_bench(dev)
        log(f"bench: radiance {json.dumps(out['radiance'])}")
    if not args.no_serving:
        log("bench: serving")
        out["serving"] = serving_bench(dev, dev_batches)
        sv = out["serving"]
        log("bench: serving saturated %.3e q/s; p50/p99 ms at 50%%: %.3f/%.3f, at 90%%: %.3f/%.3f" % (
            sv["saturated"]["queries_per_s"], sv["poisson_50pct"]["p50_ms"], sv["poisson_50pct"]["p99_ms"],
            sv["poisson_90pct"]["p50_ms"], sv["poisson_90pct"]["p99_ms"]))
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(C64.astype(np.float32).astype(np.float64), batches)
        log(f"bench: cpu baseline {out['cpu_baseline']['value']:.3e} queries/s ({out['cpu_baseline']['sample']})")
    if args.copy_reference:
        src = torch.empty(COPY_REF_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_reference_bytes"] = COPY_REF_BYTES
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
