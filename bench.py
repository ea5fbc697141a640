"""Benchmark: batched Alg. 1 search on the SIFT-shaped workload, one GPU.

Workload: base 1,000,000 x 128 (integers 0..255 stored as fp32), NSSG graph
R = 50 built by the CPU oracle, 10,000 unindexed queries, K = 100, pool L =
the smallest swept L whose oracle recall@10 is >= 0.95. One step = one
ssg_search call over all 10,000 queries (every step of the hot path: entry
selection, expansions, gathers, distances, merges, output). Inputs are
resident in HBM before timing starts.

Prints one JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
WORKLOAD = "c2"


def log(*a):
    print(f"[bench {time.strftime('%H:%M:%S')}]", *a, file=sys.stderr, flush=True)


def source_digest() -> str:
    """sha1 prefix of the search kernels' sources (the kernel file and its
    shared header)."""
    h = hashlib.sha1()
    for name in ("ssg_search.hip", "ssg_search_common.h"):
        with open(os.path.join(ROOT, "paper_1907_06146_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:12]


def recall_at(ids: np.ndarray, gt: np.ndarray, k: int) -> float:
    """Eq. 1: |R n G| / |G| with R, G the first k ids, averaged over queries."""
    a = ids[:, :k].astype(np.int64)
    b = gt[:, :k].astype(np.int64)
    hit = sum(len(np.intersect1d(x[x >= 0], y)) for x, y in zip(a, b))
    return hit / float(b.size)


def algorithmic_bytes(ndc, degsum, d, s, K, elem=4):
    """Bytes Alg. 1 itself must move per query: the query, the s entry
    vectors, the neighbour ids of every expanded node (4 bytes times the sum
    of their out-degrees), one vector per further distance computation, and
    the K (id, dist) outputs."""
    ndc = np.asarray(ndc, np.float64)
    degsum = np.asarray(degsum, np.float64)
    return 4 * d + s * d * elem + 4 * degsum + (ndc - s) * d * elem + 8 * K


def moved_bytes(ndc, hops, d, R, s, K, elem=4):
    """The same with every expansion reading its whole fixed-width row (R
    ids, what the n x R layout stores): the bytes the kernel moves."""
    ndc = np.asarray(ndc, np.float64)
    hops = np.asarray(hops, np.float64)
    return 4 * d + s * d * elem + hops * 4 * R + (ndc - s) * d * elem + 8 * K


def dist_error(base, q, ids, dd):
    """Relative error of returned distances against FP64 recomputation of
    the same (query, id) pairs (padding skipped): (max, mean)."""
    ids = np.asarray(ids)
    ok = ids >= 0
    x = base[np.where(ok, ids, 0).reshape(-1)].astype(np.float64).reshape(ids.shape + (base.shape[1],))
    ref = ((q.astype(np.float64)[:, None, :] - x) ** 2).sum(-1)
    rel = np.abs(np.asarray(dd, np.float64) - ref) / np.maximum(ref, 1e-30)
    rel = rel[ok]
    return (float(rel.max()), float(rel.mean())) if rel.size else (0.0, 0.0)


def host_cores():
    """Logical CPUs this process may run on, and the machine's count."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return avail, os.cpu_count() or avail


def traffic_from_profile(kernel_tag: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"{kernel_tag}_counters.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        c = json.load(f)
    if c.get("source_digest") != source_digest():
        return None
    return c.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--L", type=int, default=0, help="pool size (default: operating point)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sample", type=int, default=0, help="queries for the CPU baseline")
    ap.add_argument("--waves-per-block", type=int, default=0)
    ap.add_argument("--hash-log2", type=int, default=0)
    ap.add_argument("--variant", type=int, default=0, help="gather shape variant")
    ap.add_argument("--no-forms", action="store_true", help="skip the BF16 / FP8 forms")
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5", "build", "sharded", "alpha",
                                                        "scaling", "exact", "shapes"],
                    help="c2: the headline search; c3: storage precisions on 960-d data; "
                         "c4: mixed L/K batched form; c5: serving; build: GPU index build "
                         "(kNN graph and Alg. 3's pruning loops) on the 1M x 128 set; sharded: "
                         "partitioned search over random shards on the 1M x 128 set; alpha: "
                         "minimum-angle sweep; scaling: build and search cost against n; exact: "
                         "exact SSG (Alg. 2) degrees and greedy path lengths on 10,000 points; "
                         "shapes: launch-shape sweep of the headline search")
    ap.add_argument("--shards", type=int, default=4, help="sharded: number of shards")
    ap.add_argument("--offered-rps", type=float, default=4000.0, help="c5: request arrival rate")
    ap.add_argument("--requests", type=int, default=8000, help="c5: number of requests")
    ap.add_argument("--scaling-mode", default="prefix", choices=["prefix", "density"],
                    help="scaling: prefixes of the 1M set, or a fresh draw per n with n / 1,000 "
                         "components (the same points per component at every n)")
    ap.add_argument("--oversubscribe", type=float, default=6.0,
                    help="serving admission: LDS budget = this x the chip's LDS (6: about the "
                         "3 batch slots of 8,192 queries the count-based admission held)")
    ap.add_argument("--serve-data", default="c5", help="c5: index to serve (c5, or c4 for a smaller run)")
    ap.add_argument("--serve-mode", default="batch", choices=["batch", "request"],
                    help="c5: continuous batching of waiting requests, or one launch per request")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="for counter runs: 3 launches of the timed configuration, then a 1 GiB "
                         "element-wise copy whose bytes calibrate the counters; no output")
    ap.add_argument("--pmc-form", default="f32", choices=["f32", "bf16", "fp8"],
                    help="with --pmc-probe: the storage form searched (BF16 / FP8 with the FP32 "
                         "rerank of every returned entry)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {a.gpus}); the index and every query "
              "fit one MI355X, and no multi-GPU path is built", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1907_06146_amd import graph_io, quantize, search

    if a.workload == "exact":
        print(json.dumps(bench_exact(a)), flush=True)
        return
    if a.workload == "shapes":
        print(json.dumps(bench_shapes(a)), flush=True)
        return
    if a.workload in ("alpha", "scaling"):
        print(json.dumps(bench_alpha(a) if a.workload == "alpha" else bench_scaling(a)), flush=True)
        return
    if a.workload == "sharded":
        print(json.dumps(bench_sharded(a)), flush=True)
        return
    if a.workload == "build":
        print(json.dumps(bench_build(a)), flush=True)
        return
    if a.workload == "c3":
        print(json.dumps(bench_precision_c3(a)), flush=True)
        return
    if a.workload == "c4":
        print(json.dumps(bench_batched(a)), flush=True)
        return
    if a.workload == "c5":
        print(json.dumps(bench_serving(a)), flush=True)
        return
    cfg = synth.CONFIGS[WORKLOAD]
    t0 = time.time()
    gc = graph_io.load(WORKLOAD)
    meta = gc["meta"]
    base = synth.base_vectors(cfg)
    if synth.checksum(base) != meta["base_sha"]:
        raise SystemExit("regenerated base vectors do not match the graph cache")
    q = synth.queries(cfg, base)
    droot = os.path.join(graph_io.default_root(), WORKLOAD)
    with open(os.path.join(droot, "sweep.json")) as f:
        sweep = json.load(f)
    L = a.L or sweep["L_op"]
    K = cfg["K"]
    gt = np.load(os.path.join(droot, "gt_ids.npy"), allow_pickle=False)
    ondc = np.load(os.path.join(droot, f"oracle_L{L}_ndc.npy"), allow_pickle=False)
    ohops = np.load(os.path.join(droot, f"oracle_L{L}_hops.npy"), allow_pickle=False)
    odeg = np.load(os.path.join(droot, f"oracle_L{L}_degsum.npy"), allow_pickle=False)
    log(f"data ready in {time.time() - t0:.1f}s: n={base.shape[0]} d={base.shape[1]} nq={len(q)} "
        f"R={gc['graph'].shape[1]} L={L} K={K}")

    dev = torch.device("cuda:0")
    tb = torch.from_numpy(base).to(dev)
    tg = graph_io.to_device(gc["graph"], dev)
    te = graph_io.to_device(gc["entry_ids"], dev)
    tq = torch.from_numpy(q).to(dev)
    ids = torch.empty((len(q), K), dtype=torch.int32, device=dev)
    dd = torch.empty((len(q), K), dtype=torch.float32, device=dev)
    kw = dict(out=(ids, dd), waves_per_block=a.waves_per_block, hash_log2=a.hash_log2,
              gather_variant=a.variant)
    stream = torch.cuda.current_stream(dev)

    if a.pmc_probe:
        if a.pmc_form == "f32":
            codes, pkw = tb, kw
        else:
            codes, scale = quantize(tb, a.pmc_form)
            pkw = dict(kw, dim_scale=scale, base_f32=tb, rerank_k=K)
        for _ in range(3):
            search(codes, tg, te, tq, K, L, **pkw)
        torch.cuda.synchronize()
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)  # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        log("pmc probe done: 3 search launches, 1 GiB copy")
        return

    for _ in range(a.warmup):
        search(tb, tg, te, tq, K, L, **kw)
    torch.cuda.synchronize()
    gids = ids.cpu().numpy()
    r10 = recall_at(gids, gt, 10)
    _, _, gndc, ghops = search(tb, tg, te, tq, K, L, stats=True, waves_per_block=a.waves_per_block,
                               hash_log2=a.hash_log2, gather_variant=a.variant)
    gndc = gndc.cpu().numpy()
    log(f"warmup done; GPU recall@10 = {r10:.4f}; GPU NDC {gndc.mean():.1f} "
        f"(oracle {np.mean(ondc):.1f})")

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(a.steps):
        search(tb, tg, te, tq, K, L, **kw)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    gpu_ms = ev0.elapsed_time(ev1)
    launch_ms = gpu_ms / a.steps
    qps = len(q) * a.steps / (gpu_ms / 1e3)
    log(f"{a.steps} steps: {gpu_ms:.3f} ms GPU ({launch_ms:.4f} ms/launch), wall {wall * 1e3:.1f} ms")

    R = gc["graph"].shape[1]
    bq = algorithmic_bytes(ondc, odeg, base.shape[1], cfg["s"], K)
    bytes_launch = float(bq.sum())
    achieved = bytes_launch / (launch_ms / 1e3) / 1e9
    moved = float(moved_bytes(ondc, ohops, base.shape[1], R, cfg["s"], K).sum())
    traffic = traffic_from_profile("c2_search_f32")
    # steady state: 100,000 further distinct queries (their own oracle NDC and
    # expanded-row bytes), so the launch is not dominated by the latency of
    # its last-started queries
    steady = steady_state(tb, tg, te, K, L, cfg, droot, a, stream)
    log(f"steady state: {steady}")
    ceiling = gather_ceiling(tb, base.shape[1] * 4, int(np.sum(ondc)))
    log(f"random {base.shape[1] * 4}-byte row gather ceiling: {ceiling:.0f} GB/s")
    out = {
        "metric": "queries/sec at recall@10>=0.95 (1Mx128, 1 GPU); achieved HBM GB/s vs peak",
        "value": qps,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": launch_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sift-shaped synthetic, base 1,000,000 x 128 integers 0..255 "
                               "(fp32), NSSG R=50 alpha=60, 10,000 unindexed queries",
                   "K": K, "L": L, "metric": "l2", "nq": int(len(q)), "n": int(base.shape[0]),
                   "d": int(base.shape[1]), "R": int(gc["graph"].shape[1])},
        "recall10": r10,
        "oracle_recall10": next((r["recall10"] for r in sweep["rows"] if r["L"] == L), None),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_query": float(bq.mean()),
                     "moved_bytes_per_query": moved / len(q),
                     "moved_GBps": moved / (launch_ms / 1e3) / 1e9,
                     "oracle_expanded_degree_mean": float(np.sum(odeg) / np.sum(ohops)),
                     "oracle_ndc_mean": float(np.mean(ondc)), "oracle_hops_mean": float(np.mean(ohops)),
                     "gpu_ndc_mean": float(gndc.mean()),
                     "gather_ceiling_GBps": ceiling, "frac_of_gather_ceiling": achieved / ceiling},
        "steady_state_100k_queries": steady,
        "kernel_source": source_digest(),
    }
    if not a.no_forms:
        out["forms"] = precision_forms(tb, tg, te, tq, K, L, gt, sweep, cfg, a, launch_ms, base, q, droot)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(base, gc, q, K, L, cfg, a.cpu_sample)
    print(json.dumps(out), flush=True)


def steady_state(tb, tg, te, K, L, cfg, droot, a, stream):
    """The FP32 search over the 100,000 steady-state queries (distinct from
    the headline set and from each other): time per launch, throughput,
    algorithmic bytes from their own oracle counts, and agreement of the
    first 10 ids with the oracle's."""
    import torch

    import synth
    from paper_1907_06146_amd import search
    qs = synth.steady_queries(cfg)
    ondc = np.load(os.path.join(droot, f"steady_L{L}_ndc.npy"), allow_pickle=False)
    odeg = np.load(os.path.join(droot, f"steady_L{L}_degsum.npy"), allow_pickle=False)
    oids = np.load(os.path.join(droot, f"steady_L{L}_ids10.npy"), allow_pickle=False)
    gt = np.load(os.path.join(droot, "steady_gt_ids.npy"), allow_pickle=False)
    tq = torch.from_numpy(qs).to(tb.device)
    ids = torch.empty((len(qs), K), dtype=torch.int32, device=tb.device)
    dd = torch.empty((len(qs), K), dtype=torch.float32, device=tb.device)
    kw = dict(out=(ids, dd), waves_per_block=a.waves_per_block, hash_log2=a.hash_log2,
              gather_variant=a.variant)
    ms = _time(lambda: search(tb, tg, te, tq, K, L, **kw), 5, 1, stream)
    got = ids[:, :10].cpu().numpy().view(np.uint32)
    bq = algorithmic_bytes(ondc, odeg, qs.shape[1], cfg["s"], K)
    gbs = float(bq.sum()) / (ms / 1e3) / 1e9
    return {"queries": int(len(qs)), "ms_per_launch": ms, "qps": len(qs) / ms * 1e3,
            "achieved_GBps": gbs, "frac": gbs / PEAK_HBM_GBS,
            "first10_equal_oracle": float((got == oids).all(1).mean()),
            "recall10": recall_at(got, gt, 10), "distinct_queries": True}


def _time(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def gather_ceiling(base_t, row_bytes, m, seed=0, rows_per_wave=16):
    """Random-row gather rate of the device in the search's access shape
    (ssg_probe_gather): m uniformly random rows of row_bytes, GB/s."""
    import ctypes

    import torch

    from paper_1907_06146_amd import _lib
    dev = base_t.device
    n = base_t.shape[0]
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    ids = torch.randint(0, n, (m,), dtype=torch.int32, device=dev, generator=g)
    out = torch.empty((m + rows_per_wave - 1) // rows_per_wave, dtype=torch.int32, device=dev)
    st = torch.cuda.current_stream()

    def fn():
        _lib.check(_lib.lib().ssg_probe_gather(
            ctypes.c_void_p(base_t.data_ptr()), n, row_bytes, ctypes.c_void_p(ids.data_ptr()), m,
            rows_per_wave, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st.cuda_stream)))
    ms = _time(fn, 5, 2, st)
    return m * row_bytes / (ms / 1e3) / 1e9


def precision_forms(tb, tg, te, tq, K, L_fp32, gt, sweep, cfg, a, fp32_ms, base_np, q_np, droot):
    """BF16 and FP8-E4M3 storage (FP32 accumulation, then an FP32 rerank of
    every returned pool entry, the first min(K, L)) on the same workload: for each form the
    smallest swept L whose GPU recall@10 is >= 0.95, its time per launch of
    the 10,000 queries in the default launch shape and in the fastest shape
    of the autotuner, and the same on the 100,000 steady-state queries, where
    FP32 also runs in its fastest shape."""
    import torch

    import synth
    from paper_1907_06146_amd import quantize, search
    from paper_1907_06146_amd.autotune import tune_search

    stream = torch.cuda.current_stream()
    nq = tq.shape[0]
    d = tb.shape[1]
    rr = K  # every returned entry is re-scored in FP32
    qs = torch.from_numpy(synth.steady_queries(cfg)).to(tb.device)
    sgt = np.load(os.path.join(droot, "steady_gt_ids.npy"), allow_pickle=False)
    f32_shape, _, _ = tune_search(tb, tg, te, tq, K, L_fp32, reps=3)
    f32_steady_shape, _, _ = tune_search(tb, tg, te, qs, K, L_fp32, reps=2)
    # the chosen shape re-timed on its own (the tuner's figure is the best of
    # several noisy timings)
    f32_steady_ms = _time(lambda: search(tb, tg, te, qs, K, L_fp32, **f32_steady_shape), 5, 1, stream)
    f32_tuned_ms = _time(lambda: search(tb, tg, te, tq, K, L_fp32, **f32_shape), a.steps, 2, stream)
    forms = {"fp32": {"L": L_fp32, "ms_per_step": fp32_ms, "qps": nq / fp32_ms * 1e3,
                      "tuned_shape": f32_shape, "tuned_ms_per_step": f32_tuned_ms,
                      "steady_state": {"shape": f32_steady_shape, "ms_per_launch": f32_steady_ms,
                                       "qps": len(qs) / f32_steady_ms * 1e3}}}
    log(f"form fp32: {forms['fp32']}")
    Ls = sorted(set(sweep_Ls(sweep)) | {L_fp32})
    for fmt in ("bf16", "fp8"):
        codes, scale = quantize(tb, fmt)
        torch.cuda.synchronize()
        best = None
        for L in Ls:
            kw = dict(dim_scale=scale, base_f32=tb, rerank_k=rr)
            ids, _ = search(codes, tg, te, tq, K, L, **kw)
            torch.cuda.synchronize()
            r10 = recall_at(ids.cpu().numpy(), gt, 10)
            if r10 < 0.95:
                continue
            ms = _time(lambda: search(codes, tg, te, tq, K, L, **kw), a.steps, 2, stream)
            shape, _, _ = tune_search(codes, tg, te, tq, K, L, dim_scale=scale, base_f32=tb, rerank_k=rr)
            tuned = _time(lambda: search(codes, tg, te, tq, K, L, **kw, **shape), a.steps, 2, stream)
            s_shape, _, _ = tune_search(codes, tg, te, qs, K, L, dim_scale=scale, base_f32=tb,
                                        rerank_k=rr, reps=2)
            s_ms = _time(lambda: search(codes, tg, te, qs, K, L, **kw, **s_shape), 5, 1, stream)
            s_ids, _ = search(codes, tg, te, qs, K, L, **kw, **s_shape)
            torch.cuda.synchronize()
            s_r10 = recall_at(s_ids.cpu().numpy(), sgt, 10)
            _, _, ndc, hops = search(codes, tg, te, tq, K, L, stats=True, **kw)
            ndc = ndc.double().mean().item()
            hops = hops.double().mean().item()
            ids_h, dd_h = search(codes, tg, te, tq, K, L, **kw)
            torch.cuda.synchronize()
            emax, emean = dist_error(base_np, q_np, ids_h.cpu().numpy(), dd_h.cpu().numpy())
            # the search phase alone: its distances are those of the stored codes
            si, sd = search(codes, tg, te, tq, K, L, dim_scale=scale)
            torch.cuda.synchronize()
            smax, smean = dist_error(base_np, q_np, si.cpu().numpy(), sd.cpu().numpy())
            eb = 2 if fmt == "bf16" else 1
            bq = 4 * d + cfg["s"] * d * eb + hops * 4 * tg.shape[1] + (ndc - cfg["s"]) * d * eb \
                + min(L, rr) * d * 4 + 8 * K
            ceil = gather_ceiling(codes, d * eb, int(nq * ndc))
            best = {"L": L, "recall10": r10, "ms_per_step": ms, "qps": nq / ms * 1e3,
                    "speedup_vs_fp32": fp32_ms / ms,
                    "tuned_shape": shape, "tuned_ms_per_step": tuned,
                    "tuned_speedup_vs_tuned_fp32": f32_tuned_ms / tuned,
                    "steady_state": {"shape": s_shape, "ms_per_launch": s_ms, "qps": len(qs) / s_ms * 1e3,
                                     "recall10": s_r10,
                                     "speedup_vs_fp32_fastest_shape": f32_steady_ms / s_ms},
                    "gpu_ndc_mean": ndc, "moved_bytes_per_query": bq,
                    "moved_GBps": bq * nq / (ms / 1e3) / 1e9,
                    "gather_ceiling_GBps": ceil, "rerank": f"fp32, first {min(L, rr)} pool entries",
                    "dist_rel_err_vs_fp64": {"max": emax, "mean": emean},
                    "search_phase_dist_rel_err_vs_fp64": {"max": smax, "mean": smean}}
            break
        forms[fmt] = best
        log(f"form {fmt}: {best}")
    return forms


def sweep_Ls(sweep):
    return [r["L"] for r in sweep["rows"]]


def recall_mixed(ids, gt, K_arr):
    """Mean over queries of |R n G| / K_i with each query's own K_i (Eq. 1)."""
    hit = 0.0
    for r, k in enumerate(K_arr):
        x = ids[r, :k]
        hit += len(np.intersect1d(x[x >= 0], gt[r, :k])) / float(k)
    return hit / len(K_arr)


def _load(name):
    import synth
    from paper_1907_06146_amd import graph_io
    cfg = synth.CONFIGS[name]
    gc = graph_io.load(name)
    base = synth.base_vectors(cfg)
    if synth.checksum(base) != gc["meta"]["base_sha"]:
        raise SystemExit(f"regenerated {name} base vectors do not match the graph cache")
    q = synth.queries(cfg, base)
    droot = os.path.join(graph_io.default_root(), name)
    if os.path.exists(os.path.join(droot, "gt_ids.npy")):
        gt = np.load(os.path.join(droot, "gt_ids.npy"), allow_pickle=False)
    else:  # compact form: the first K_i ground-truth ids of each query, packed
        rg = gc["meta"]["ragged"]["gt_ids"]
        Kq = np.load(os.path.join(droot, "mixed_K.npy"), allow_pickle=False).astype(np.int64)
        vals = graph_io.unpack_bits(np.load(os.path.join(droot, "gt_ids_bits.npy"), allow_pickle=False),
                                    rg["bits"], int(Kq.sum()))
        gt = np.full((len(Kq), rg["width"]), 0xFFFFFFFF, np.uint32)
        gt[np.arange(rg["width"])[None, :] < Kq[:, None]] = vals
    return cfg, gc, base, q, gt


def bench_batched(a):
    """Deep-shaped 1M x 96 unit-norm workload, inner product, 100,000 queries
    with their own L in {16..512} and K in {1, 10, 100}: the plain FP32 search
    launched once per (L, K) group, against one graph-captured batched
    launch (FP32, and BF16 with an FP32 rerank of each query's K)."""
    import torch

    import synth
    from paper_1907_06146_amd import graph_io, quantize, search
    from paper_1907_06146_amd.autotune import tune
    from paper_1907_06146_amd.batched import BatchedSearch

    t0 = time.time()
    cfg, gc, base, q, gt = _load("c4")
    Lq, Kq = synth.query_params("c4")
    dev = torch.device("cuda:0")
    tb = torch.from_numpy(base).to(dev)
    tg = graph_io.to_device(gc["graph"], dev)
    te = graph_io.to_device(gc["entry_ids"], dev)
    tq = torch.from_numpy(q).to(dev)
    nq = len(q)
    kst = int(Kq.max())
    stream = torch.cuda.current_stream()
    log(f"c4 ready in {time.time() - t0:.1f}s: n={len(base)} nq={nq}")
    if a.pmc_probe:  # counter runs: one batched launch per form (default shapes), then a 1 GiB copy
        qb, _ = quantize(tb, "bf16")
        for bse, kw in ((tb, {}), (qb, dict(base_f32=tb, rerank=-2))):
            bs = BatchedSearch(bse, tg, te, tq, Lq, Kq, "ip", use_graph=False, **kw)
            bs.run()
            torch.cuda.synchronize()
            bs.close()
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log("pmc probe done: batched FP32 and BF16 + rerank launches, 1 GiB copy")
        return {"pmc_probe": True}
    # plain: one launch per (L, K) group
    groups = {}
    for i, key in enumerate(zip(Lq.tolist(), Kq.tolist())):
        groups.setdefault(key, []).append(i)
    plan = []
    for (L, K), rows in sorted(groups.items()):
        rows = np.asarray(rows)
        tr = torch.from_numpy(rows).to(dev)
        plan.append((L, K, rows, tq[tr].contiguous(),
                     torch.empty((len(rows), K), dtype=torch.int32, device=dev),
                     torch.empty((len(rows), K), dtype=torch.float32, device=dev)))

    def plain():
        for L, K, rows, qq, oi, od in plan:
            search(tb, tg, te, qq, K, L, "ip", out=(oi, od))
    ms_plain = _time(plain, max(3, a.steps // 4), 1, stream)
    ids_plain = np.full((nq, kst), -1, np.int32)
    for L, K, rows, qq, oi, od in plan:
        ids_plain[rows, :K] = oi.cpu().numpy()
    r_plain = recall_mixed(ids_plain, gt, Kq)
    log(f"plain fp32: {len(plan)} launches, {ms_plain:.3f} ms, recall {r_plain:.4f}")
    out = {"metric": "mixed-L/K batch queries/s at equal recall (1M x 96 unit-norm, IP, 1 GPU)",
           "unit": "queries/s", "workload": "deep-shaped synthetic 1,000,000 x 96, 100,000 "
           "queries, L in {16..512}, K in {1, 10, 100}", "n_gpus": 1,
           "plain_fp32": {"launches": len(plan), "ms": ms_plain, "qps": nq / ms_plain * 1e3,
                          "recall_at_Ki": r_plain}}
    qb, _ = quantize(tb, "bf16")
    tune_path = os.path.join(graph_io.default_root(), "autotune.json")
    for name, bse, kw in (("batched_fp32", tb, {}),
                          ("batched_bf16_rerank", qb, dict(base_f32=tb, rerank=-1)),
                          ("batched_bf16_rerank_2k", qb, dict(base_f32=tb, rerank=-2)),
                          ("batched_bf16_rerank_4k", qb, dict(base_f32=tb, rerank=-4))):
        t = time.time()
        shapes = tune(bse, tg, te, tq, Lq, Kq, "ip", sample=2048, reps=2, cache_path=tune_path, **kw)
        log(f"{name}: tuned in {time.time() - t:.1f}s: {shapes}")
        bs = BatchedSearch(bse, tg, te, tq, Lq, Kq, "ip", shapes=shapes, use_graph=True, **kw)
        ms = _time(bs.run, max(3, a.steps // 4), 1, stream)
        ids = bs.out_ids.cpu().numpy()
        r = recall_mixed(ids, gt, Kq)
        same = float(np.mean((ids == ids_plain).all(1)))
        out[name] = {"ms": ms, "qps": nq / ms * 1e3, "recall_at_Ki": r, "speedup_vs_plain": ms_plain / ms,
                     "rows_equal_to_plain": same, "shapes": {str(k): v for k, v in shapes.items()},
                     "rerank": {0: "none", -1: "first K_i", -2: "first 2 K_i", -4: "first 4 K_i"}[
                         kw.get("rerank", 0)]}
        if name != "batched_fp32":
            out[name]["speedup_vs_batched_fp32"] = out["batched_fp32"]["ms"] / ms
        log(f"{name}: {ms:.3f} ms, recall {r:.4f}, x{ms_plain / ms:.2f}")
        bs.close()
    out["value"] = out["batched_bf16_rerank"]["qps"]
    return out


def bench_exact(a):
    """Exact SSG study (the paper's table on SIFT10K, here on 10,000 points of
    the SIFT-shaped synthetic mixture): Alg. 2 graphs for 60 and 30 degrees
    built on the GPU, their average and maximum out-degree, and for graphs of
    at most 64 out-edges per node (the search kernel's row width: the graphs
    truncated at 40 and 64 edges) the greedy path length of Alg. 1 with L = 1
    from a random start: for 1,000 indexed queries (base points; success =
    the query itself is found) and 1,000 unindexed queries (success = the
    exact nearest neighbour is found)."""
    import torch

    import synth
    from paper_1907_06146_amd import search
    from paper_1907_06146_amd.binding import exact_ssg

    base = np.ascontiguousarray(synth.base_vectors("c2s")[:10_000])
    n = len(base)
    unq = synth.queries("c2s", synth.base_vectors("c2s"))[:1000]
    rng = np.random.default_rng(2024)
    idx_q = rng.choice(n, 1000, replace=False)
    qs = np.concatenate([base[idx_q], unq]).astype(np.float32)
    dev = torch.device("cuda:0")
    tb = torch.from_numpy(base).to(dev)
    tq = torch.from_numpy(qs).to(dev)
    # exact nearest neighbour of each unindexed query (FP64, ties by id)
    b64 = base.astype(np.float64)
    nn = np.array([int(np.lexsort((np.arange(n), ((b64 - u) ** 2).sum(1)))[0]) for u in unq.astype(np.float64)])
    starts = torch.from_numpy(rng.integers(0, n, (len(qs), 1)).astype(np.int32)).to(dev)
    rows = []
    for alpha in (60.0, 30.0):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        full, deg = exact_ssg(tb, alpha, cap=64)
        dt = time.perf_counter() - t0
        deg = deg.cpu().numpy()
        for cap in (40, 64):
            g = full[:, :cap].contiguous()
            ids, _, _, hops = search(tb, g, starts, tq, 1, 1, stats=True, entry_group_size=1)
            torch.cuda.synchronize()
            ids = ids.cpu().numpy()[:, 0]
            hops = hops.cpu().numpy().astype(np.float64)
            gk = (g >= 0).sum(1).cpu().numpy()
            rows.append({"alpha": alpha, "build_s": dt, "aod_full": float(deg.mean()),
                         "mod_full": int(deg.max()), "truncated_at": cap, "aod": float(gk.mean()),
                         "mod": int(gk.max()),
                         "path_indexed": float(hops[:1000].mean() - 1.0),
                         "found_indexed": float((ids[:1000] == idx_q).mean()),
                         "path_unindexed": float(hops[1000:].mean() - 1.0),
                         "found_unindexed": float((ids[1000:] == nn).mean())})
            log(f"exact SSG: {rows[-1]}")
    return {"metric": "exact SSG degrees and greedy (L = 1) path lengths, 10,000 x 128, 1 GPU",
            "workload": "10,000 points of the sift-shaped synthetic mixture; path length = moves "
                        "of Alg. 1 with L = 1 from a random start (expansions - 1)", "rows": rows,
            "data": "synthetic (seeded)"}


def _gpu_nssg(tb, knn, cfg, alpha):
    """Forward and reverse pruning on the GPU plus s random navigating nodes
    (no DFS spanning); returns (graph, entry ids, prune + reverse seconds)."""
    import torch

    from paper_1907_06146_amd.binding import nssg_prune, nssg_reverse
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = nssg_reverse(tb, nssg_prune(tb, knn, cfg["l"], cfg["R"], alpha), alpha)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    e = np.random.default_rng(cfg["seed"] + 41).choice(tb.shape[0], cfg["s"], replace=False)
    return g, torch.from_numpy(e.astype(np.int32)).to(tb.device), dt


def _first_L(fn, Ls, target):
    """Smallest L whose recall reaches target: returns (L, recall, extra) or the last row."""
    last = None
    for L in Ls:
        r, extra = fn(L)
        last = (L, r, extra)
        if r >= target:
            return last
    return last


def bench_alpha(a):
    """Minimum-angle sweep (the paper's angle experiment) on the SIFT-shaped
    1M x 128 set: one exact kNN graph, then an NSSG per angle built on the
    GPU; for each angle the average out-degree and the search cost at
    recall@10 = 0.95 (10,000 queries, K = 100): the distance count (NDC),
    expansions and pool size interpolated on the recall-NDC curve over
    L = 20..300, averaged over three draws of the navigating nodes, and the
    throughput at the first grid L reaching the target."""
    import torch

    from paper_1907_06146_amd import search
    from paper_1907_06146_amd.binding import knn_graph

    cfg, gc, base, q, gt = _load("c2")
    dev = torch.device("cuda:0")
    tb = torch.from_numpy(base).to(dev)
    tq = torch.from_numpy(q).to(dev)
    stream = torch.cuda.current_stream()
    knn, _, _ = knn_graph(tb, cfg["knn_k"])
    n = len(base)
    Ls = list(range(20, 101, 10)) + list(range(120, 301, 20))
    target = 0.95
    rows = []
    for alpha in (40.0, 45.0, 50.0, 55.0, 60.0, 65.0, 70.0):
        g, e, dt = _gpu_nssg(tb, knn, cfg, alpha)
        aod = float((g >= 0).sum().item()) / n
        entries = [e] + [torch.from_numpy(np.random.default_rng(cfg["seed"] + 41 + k).choice(
            n, cfg["s"], replace=False).astype(np.int32)).to(dev) for k in (1, 2)]
        curve = []
        for L in Ls:
            rs, nd, hp = [], [], []
            for ent in entries:
                ids, _, ndc, hops = search(tb, g, ent, tq, cfg["K"], L, stats=True)
                torch.cuda.synchronize()
                rs.append(recall_at(ids.cpu().numpy(), gt, 10))
                nd.append(ndc.double().mean().item())
                hp.append(hops.double().mean().item())
            curve.append((L, float(np.mean(rs)), float(np.mean(nd)), float(np.mean(hp))))
        hit = next((i for i, c in enumerate(curve) if c[1] >= target), None)
        row = {"alpha": alpha, "aod": aod, "prune_reverse_s": dt,
               "curve": [{"L": c[0], "recall10": c[1], "ndc": c[2], "hops": c[3]} for c in curve]}
        if hit is not None:
            if hit == 0:
                L_t, ndc_t, hops_t = curve[0][0], curve[0][2], curve[0][3]
            else:
                (L0, r0, n0, h0), (L1, r1, n1, h1) = curve[hit - 1], curve[hit]
                w = (target - r0) / max(r1 - r0, 1e-12)
                L_t, ndc_t, hops_t = L0 + w * (L1 - L0), n0 + w * (n1 - n0), h0 + w * (h1 - h0)
            Lg = curve[hit][0]
            ms = _time(lambda: search(tb, g, e, tq, cfg["K"], Lg), a.steps, a.warmup, stream)
            row.update(L_interp=L_t, ndc=ndc_t, hops=hops_t, L_grid=Lg, ms=ms, qps=len(q) / ms * 1e3)
        else:
            row.update(best_recall10=curve[-1][1])
        rows.append(row)
        log(f"alpha {alpha}: aod {aod:.1f} " + str({k: v for k, v in row.items() if k != "curve"}))
    return {"metric": "search cost per minimum angle at recall@10 = 0.95 (1M x 128, 1 GPU)",
            "workload": "sift-shaped synthetic 1,000,000 x 128, NSSG l = 100, R = 50 built on the GPU "
                        "(no DFS spanning), 10,000 queries, K = 100, 3 draws of the 10 navigating nodes",
            "rows": rows, "data": "synthetic (seeded)"}


def bench_scaling(a):
    """Build and search cost against n (the paper's complexity experiment):
    prefixes of the SIFT-shaped set (its order is random, so each prefix is a
    uniform sample) from 62,500 to 1,000,000 points, each indexed on the GPU
    (kNN graph, then forward and reverse pruning = edge selection) and
    searched with the 10,000 queries over a fine L grid, from three draws of
    the navigating nodes. Recall@10 is against each prefix's exact top 10
    (FP64 GPU matrix product; exact for these integer vectors). The search
    cost at a recall target is the distance count (NDC) interpolated on the
    recall-NDC curve averaged over the three draws, so a target falling
    between two grid points does not jump to the next L. The costs are then
    fitted against n^(1/d') log n (the paper's bound, d' the intrinsic
    dimension of the data, about 13 here)."""
    import torch

    from paper_1907_06146_amd import search
    from paper_1907_06146_amd.binding import knn_graph

    import synth
    cfg, gc, base, q, gt_full = _load("c2")
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    Ls = list(range(20, 101, 10)) + list(range(120, 301, 20))
    if a.scaling_mode == "density":
        # a fresh draw per n with n / 1,000 components: every size has the same
        # points per component (1,000) and the same local structure
        def data(n):
            c = dict(synth.CONFIGS["c2"], n=n, comps=n // 1000, nq_unindexed=10_000, nq_indexed=0,
                     seed=synth.CONFIGS["c2"]["seed"] + 97 + n // 62_500)
            b = synth.base_vectors(c)
            return b, synth.queries(c, b)
    else:
        def data(n):
            return base[:n], q
    targets = (0.95, 0.99)
    lid = 13.0
    rows = []
    for n in (62_500, 125_000, 250_000, 500_000, 1_000_000):
        bn, qq = data(n)
        tb = torch.from_numpy(np.ascontiguousarray(bn)).to(dev)
        tq = torch.from_numpy(qq).to(dev)
        qn = (tq.double() ** 2).sum(1, keepdim=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        knn, _, _ = knn_graph(tb, cfg["knn_k"])
        torch.cuda.synchronize()
        t_knn = time.perf_counter() - t0
        g, e, t_edge = _gpu_nssg(tb, knn, cfg, cfg["alpha"])
        # exact top 10 of each query over the prefix (integer data: every FP64
        # sum is exact), ties by id
        gt = np.empty((len(qq), 10), np.int64)
        tb64 = tb.double()
        xn = (tb64 ** 2).sum(1)
        for lo in range(0, len(qq), 1000):
            dd = qn[lo:lo + 1000] + xn[None, :] - 2.0 * (tq[lo:lo + 1000].double() @ tb64.t())
            key = dd * (n + 1) + torch.arange(n, device=dev, dtype=torch.float64)[None, :]
            gt[lo:lo + 1000] = torch.topk(key, 10, dim=1, largest=False).indices.cpu().numpy()
        entries = [e] + [torch.from_numpy(np.random.default_rng(cfg["seed"] + 41 + k).choice(
            n, cfg["s"], replace=False).astype(np.int32)).to(dev) for k in (1, 2)]
        curve = []
        for L in Ls:
            rs, nd, hp = [], [], []
            for ent in entries:
                ids, _, ndc, hops = search(tb, g, ent, tq, cfg["K"], L, stats=True)
                torch.cuda.synchronize()
                rs.append(recall_at(ids.cpu().numpy(), gt, 10))
                nd.append(ndc.double().mean().item())
                hp.append(hops.double().mean().item())
            curve.append((L, float(np.mean(rs)), float(np.mean(nd)), float(np.mean(hp)),
                          float(np.min(rs)), float(np.max(rs))))
        at = {}
        for t in targets:
            hit = next((i for i, c in enumerate(curve) if c[1] >= t), None)
            if hit is None:
                at[str(t)] = None
                continue
            if hit == 0:
                L_t, ndc_t, hops_t = curve[0][0], curve[0][2], curve[0][3]
            else:
                (L0, r0, n0, h0, _, _), (L1, r1, n1, h1, _, _) = curve[hit - 1], curve[hit]
                w = (t - r0) / max(r1 - r0, 1e-12)
                L_t, ndc_t, hops_t = L0 + w * (L1 - L0), n0 + w * (n1 - n0), h0 + w * (h1 - h0)
            ms = _time(lambda: search(tb, g, e, tq, cfg["K"], curve[hit][0]), a.steps, a.warmup, stream)
            at[str(t)] = {"L_interp": L_t, "ndc": ndc_t, "hops": hops_t, "L_grid": curve[hit][0],
                          "ms_at_L_grid": ms, "qps_at_L_grid": len(qq) / ms * 1e3}
        row = {"n": n, "knn_s": t_knn, "edge_selection_s": t_edge,
               "aod": float((g >= 0).sum().item()) / n, "at_recall": at,
               "curve": [{"L": c[0], "recall10": c[1], "ndc": c[2], "hops": c[3],
                          "recall10_min": c[4], "recall10_max": c[5]} for c in curve]}
        rows.append(row)
        log(f"n {n}: aod {row['aod']:.2f} at {at}")
        del tb, tb64, knn, g
    fits = {}
    for t in targets:
        pts = [(r["n"], r["at_recall"][str(t)]["ndc"]) for r in rows if r["at_recall"][str(t)]]
        if len(pts) >= 2:
            x = np.array([n ** (1.0 / lid) * np.log(n) for n, _ in pts])
            y = np.array([c for _, c in pts])
            c1 = float((x * y).sum() / (x * x).sum())  # least squares through the origin
            fits[str(t)] = {"model": "ndc = c * n^(1/13) * ln n", "c": c1,
                            "rel_residuals": [float(v) for v in (y - c1 * x) / y]}
    sets = ("prefixes of the sift-shaped synthetic 1,000,000 x 128 set" if a.scaling_mode == "prefix"
            else "a fresh draw of the sift-shaped mixture per n with n / 1,000 components")
    return {"metric": "index build and search cost against n at fixed recall@10 (1 GPU)",
            "workload": f"{sets}, NSSG l = 100, R = 50, 60 degrees built on the GPU, 10,000 queries, "
                        "K = 100, 3 draws of the 10 navigating nodes", "mode": a.scaling_mode,
            "rows": rows, "fits": fits, "data": "synthetic (seeded)"}


def bench_sharded(a):
    """Partitioned search (Sec. 6.5) on the SIFT-shaped 1M x 128 set: S random
    shards, each with an NSSG built on the GPU (exact kNN graph, forward and
    reverse pruning; no DFS spanning), the 10,000 queries searched in every
    shard (K = 100 per shard) and merged on the device; for each swept L the
    recall@10 and throughput, against the one-graph FP32 search at the
    oracle's operating point."""
    import torch

    import synth
    from paper_1907_06146_amd import graph_io, search
    from paper_1907_06146_amd.binding import knn_graph, nssg_prune, nssg_reverse
    from paper_1907_06146_amd.sharded import ShardedIndex, partition

    cfg, gc, base, q, gt = _load("c2")
    sweep = json.load(open(os.path.join(graph_io.default_root(), "c2", "sweep.json")))
    L1 = sweep["L_op"] or cfg["L"]
    dev = torch.device("cuda:0")
    tb = torch.from_numpy(base).to(dev)
    tq = torch.from_numpy(q).to(dev)
    stream = torch.cuda.current_stream()
    K = cfg["K"]
    nq = len(q)
    # one-graph baseline
    tg = graph_io.to_device(gc["graph"], dev)
    te = graph_io.to_device(gc["entry_ids"], dev)
    one_ms = _time(lambda: search(tb, tg, te, tq, K, L1), a.steps, a.warmup, stream)
    one_ids, _ = search(tb, tg, te, tq, K, L1)
    torch.cuda.synchronize()
    one = {"L": L1, "ms": one_ms, "qps": nq / one_ms * 1e3, "recall10": recall_at(one_ids.cpu().numpy(), gt, 10)}
    log(f"one graph: {one}")
    # shards, built on the GPU
    S = a.shards
    parts = partition(len(base), S, seed=cfg["seed"] + 21)
    bases, graphs, entries = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s_, gids in enumerate(parts):
        bs = tb.index_select(0, torch.from_numpy(gids).to(dev)).contiguous()
        knn, _, _ = knn_graph(bs, cfg["knn_k"])
        g2 = nssg_reverse(bs, nssg_prune(bs, knn, cfg["l"], cfg["R"], cfg["alpha"]), cfg["alpha"])
        e = np.random.default_rng(cfg["seed"] + 31 + s_).choice(len(gids), cfg["s"], replace=False)
        bases.append(bs)
        graphs.append(g2)
        entries.append(torch.from_numpy(e.astype(np.int32)).to(dev))
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    log(f"{S} shard graphs built on the GPU in {build_s:.2f}s")
    idx = ShardedIndex(bases, graphs, entries, parts)  # one launch over all shards
    per_shard = ShardedIndex(bases, graphs, entries, parts, combined=False)
    rows = []
    best = None
    for L in (20, 30, 40, 50, 60, 80, 100):
        ids, _ = idx.search(tq, K, L)
        ids2, _ = per_shard.search(tq, K, L)
        torch.cuda.synchronize()
        r10 = recall_at(ids.cpu().numpy(), gt, 10)
        same = bool(torch.equal(ids, ids2))
        ms = _time(lambda: idx.search(tq, K, L), a.steps, a.warmup, stream)
        ms2 = _time(lambda: per_shard.search(tq, K, L), max(2, a.steps // 2), 1, stream)
        row = {"L": L, "recall10": r10, "ms": ms, "qps": nq / ms * 1e3,
               "ms_launch_per_shard": ms2, "same_ids_both_modes": same}
        rows.append(row)
        log(f"sharded S={S}: {row}")
        if best is None and r10 >= 0.95:
            best = row
    return {"metric": "partitioned search queries/s at recall@10 >= 0.95 (1M x 128, 1 GPU)",
            "value": best["qps"] if best else None, "unit": "queries/s", "n_gpus": 1,
            "workload": f"sift-shaped synthetic 1,000,000 x 128, {S} random shards, 10,000 "
                        f"queries, K = 100 per shard, merged to 100", "shards": S,
            "shard_build_s": build_s, "rows": rows, "chosen": best, "one_graph": one,
            "vs_one_graph": (best["qps"] / one["qps"]) if best else None, "data": "synthetic (seeded)"}


def bench_build(a):
    """Index build on the SIFT-shaped 1M x 128 integer set: exact kNN graph
    (K = 100) on the matrix cores, then the forward and reverse pruning loops
    of Alg. 3 (l = 100, R = 50, 60 degrees). The kNN scan is priced against the
    dense BF16 matrix-core peak with the self-join's 2 n^2 d flops."""
    import torch

    import synth
    from paper_1907_06146_amd.binding import knn_graph, nssg_prune, nssg_reverse

    cfg = synth.CONFIGS["c2"]
    base = synth.base_vectors(cfg)
    n, d = base.shape
    tb = torch.from_numpy(base).cuda()
    times = {"knn": [], "prune": [], "reverse": []}
    for rep in range(1 + max(1, a.steps // 10)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ids, _, st = knn_graph(tb, cfg["knn_k"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g1 = nssg_prune(tb, ids, cfg["l"], cfg["R"], cfg["alpha"])
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        nssg_reverse(tb, g1, cfg["alpha"])
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        if rep == 0:
            continue  # warm-up
        times["knn"].append(t1 - t0)
        times["prune"].append(t2 - t1)
        times["reverse"].append(t3 - t2)
        log(f"build rep {rep}: knn {t1 - t0:.3f}s prune {t2 - t1:.3f}s reverse {t3 - t2:.3f}s {st}")
    med = {k: float(np.median(v)) for k, v in times.items()}
    flops = 2.0 * n * n * d
    out = {"metric": "index build seconds (kNN graph + Alg. 3 pruning loops), 1 GPU",
           "value": med["knn"] + med["prune"] + med["reverse"], "unit": "s", "higher_is_better": False,
           "n_gpus": 1, "workload": "sift-shaped synthetic 1,000,000 x 128 integers, kNN K = 100, "
           "l = 100, R = 50, alpha = 60 degrees", "stage_s": med, "exact_path": st["exact_path"],
           "roofline_knn": {"bound": "mfma", "achieved": flops / med["knn"] / 1e12, "peak": 2500.0,
                            "unit": "TFLOP/s", "frac": flops / med["knn"] / 1e12 / 2500.0,
                            "note": "whole kNN call (prep, scan, rerank); 2 n^2 d flops"},
           "data": "synthetic (seeded)"}
    if not a.no_cpu:
        from oracle import core
        rows = np.random.default_rng(0).choice(n, 64, replace=False)
        t0 = time.perf_counter()
        core.bruteforce(base, base[rows], cfg["knn_k"], "l2", skip=rows)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": dt / len(rows) * n, "unit": "s (kNN graph, extrapolated)",
                               "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
                               "kind": "oracle",
                               "sample": f"{len(rows)} rows of the exact kNN graph by the oracle's "
                                         f"FP64 full scan ({dt:.1f}s), scaled to {n} rows"}
    return out


def bench_precision_c3(a):
    """GIST-shaped 1M x 960 workload (values in [0, 1], squared L2), 1,000
    queries, K = 10: FP32, BF16 and FP8-E4M3 storage (FP32 accumulation),
    each without rerank, with an FP32 rerank of the returned K and of the
    whole pool, at every swept pool size: throughput, recall@10 and the error
    of the returned distances against FP64 recomputation. Then the 16,000
    steady-state queries (distinct, with their own exact top 10) at L = 200."""
    import torch

    from paper_1907_06146_amd import graph_io, quantize, search

    t0 = time.time()
    cfg, gc, base, q, gt = _load("c3")
    log(f"c3 data ready in {time.time() - t0:.1f}s")
    sweep = json.load(open(os.path.join(graph_io.default_root(), "c3", "sweep.json")))
    orc = {r["L"]: r for r in sweep["rows"]}
    dev = torch.device("cuda:0")
    tb = torch.from_numpy(base).to(dev)
    tg = graph_io.to_device(gc["graph"], dev)
    te = graph_io.to_device(gc["entry_ids"], dev)
    tq = torch.from_numpy(q).to(dev)
    K = cfg["K"]
    nq, d = q.shape
    stream = torch.cuda.current_stream()
    codes = {"fp32": (tb, None)}
    codes["bf16"] = quantize(tb, "bf16")
    codes["fp8"] = quantize(tb, "fp8")
    torch.cuda.synchronize()
    elem = {"fp32": 4, "bf16": 2, "fp8": 1}
    q64 = q.astype(np.float64)

    def dist_err(ids, dd):
        x = base[ids.reshape(-1)].astype(np.float64).reshape(nq, K, d)
        ref = ((q64[:, None, :] - x) ** 2).sum(-1)
        rel = np.abs(dd.astype(np.float64) - ref) / np.maximum(ref, 1e-30)
        return float(rel.max()), float(rel.mean())

    rows = []
    for L in sorted(orc):
        for fmt in ("fp32", "bf16", "fp8"):
            for rr in ((0,) if fmt == "fp32" else (0, K, L)):
                cb, sc = codes[fmt]
                kw = dict(dim_scale=sc)
                if rr:
                    kw.update(base_f32=tb, rerank_k=rr)
                ids, dd, ndc, hops = search(cb, tg, te, tq, K, L, stats=True, **kw)
                torch.cuda.synchronize()
                ids_h = ids.cpu().numpy()
                emax, emean = dist_err(ids_h, dd.cpu().numpy())
                ms = _time(lambda: search(cb, tg, te, tq, K, L, **kw), a.steps, a.warmup, stream)
                ndc_m = ndc.double().mean().item()
                hops_m = hops.double().mean().item()
                bq = moved_bytes(ndc_m, hops_m, d, tg.shape[1], cfg["s"], K, elem[fmt]) \
                    + min(rr, L) * d * 4
                row = {"L": L, "form": fmt + (f"+fp32 rerank of {min(rr, L)}" if rr else ""),
                       "recall10": recall_at(ids_h, gt, 10), "oracle_recall10": orc[L]["recall10"],
                       "ms": ms, "qps": nq / ms * 1e3, "ndc": ndc_m, "hops": hops_m,
                       "moved_bytes_per_query": bq, "moved_GBps": bq * nq / (ms / 1e3) / 1e9,
                       "dist_rel_err_max": emax, "dist_rel_err_mean": emean}
                rows.append(row)
                log(row)
    # steady state: 16,000 further distinct queries (one launch fills the device)
    import synth
    steady = {}
    tq16 = torch.from_numpy(synth.steady_queries(cfg)).to(dev)
    sgt = np.load(os.path.join(graph_io.default_root(), "c3", "steady_gt_ids.npy"), allow_pickle=False)
    Ls = 200
    for fmt, rr in (("fp32", 0), ("bf16", K), ("fp8", K), ("bf16", Ls), ("fp8", Ls)):
        cb, sc = codes[fmt]
        kw = dict(dim_scale=sc)
        if rr:
            kw.update(base_f32=tb, rerank_k=rr)
        ms = _time(lambda: search(cb, tg, te, tq16, K, Ls, **kw), max(3, a.steps // 2), 1, stream)
        ids, _ = search(cb, tg, te, tq16, K, Ls, **kw)
        torch.cuda.synchronize()
        name = fmt + (f"+fp32 rerank of {rr}" if rr else "")
        steady[name] = {"L": Ls, "queries": int(tq16.shape[0]), "ms": ms, "qps": tq16.shape[0] / ms * 1e3,
                        "recall10": recall_at(ids.cpu().numpy(), sgt, 10)}
        log(f"steady {name}: {steady[name]}")
    for name, v in steady.items():
        v["speedup_vs_fp32"] = steady["fp32"]["ms"] / v["ms"]
    return {"metric": "queries/s and recall@10 per storage precision (GIST-shaped 1M x 960, 1 GPU)",
            "unit": "queries/s", "n_gpus": 1, "workload": "gist-shaped synthetic 1,000,000 x 960 in "
            "[0, 1], 1,000 queries, K = 10, squared L2", "rows": rows, "steady_state_16k_distinct": steady,
            "data": "synthetic (seeded)"}


def synth_cfg(name):
    import synth
    return synth.CONFIGS[name]


def bench_serving(a):
    """Serving: 5M x 96 unit-norm base (BF16 search, FP32 rerank of K = 10)
    resident in HBM; Poisson arrivals of requests of 1..256 queries with one
    L in {32..256}. Default: continuous batching (every waiting request joins
    the next mixed batch, 3 batch slots); --serve-mode request launches each
    request on its own (8 slots)."""
    import torch

    from paper_1907_06146_amd import graph_io, quantize
    from paper_1907_06146_amd.serve import (BatchScheduler, GpuBatchDevice, GpuDevice, Scheduler,
                                            poisson_requests, run, summarize)

    t0 = time.time()
    cfg, gc, base, q, gt = _load(a.serve_data)
    scfg = synth_cfg("c5")
    dev = torch.device("cuda:0")
    tb = torch.from_numpy(base).to(dev)
    tg = graph_io.to_device(gc["graph"], dev)
    te = graph_io.to_device(gc["entry_ids"], dev)
    qb, _ = quantize(tb, "bf16")
    torch.cuda.synchronize()
    log(f"{a.serve_data} ready in {time.time() - t0:.1f}s: n={len(base)}")
    rng = np.random.default_rng(scfg["seed"] + 5)
    reqs, picks = poisson_requests(rng, a.requests, a.offered_rps, q, scfg["L_choices"], scfg["K"],
                                   max_batch=256)
    warm, _ = poisson_requests(np.random.default_rng(1), 50, 1e6, q, [64], scfg["K"], max_batch=64)
    if a.serve_mode == "batch":
        n_slots, max_batch = 3, 8192
        # --hash-log2 / --waves-per-block, when given, set every bucket's launch shape
        shapes = None
        if a.hash_log2 or a.waves_per_block:
            shapes = {cap: {"hash_log2": a.hash_log2, "waves_per_block": a.waves_per_block}
                      for cap in (64, 128, 256, 512)}
        gdev = GpuBatchDevice(qb, tg, te, n_slots=n_slots, max_batch=max_batch, max_K=scfg["K"],
                              metric="ip", base_f32=tb, rerank=True, shapes=shapes)
        run(warm, BatchScheduler(gdev, n_slots, max_batch))
        # admission by bytes: LDS of twice what the chip holds at once, plus
        # the slots' staging and output buffers
        budget = gdev.budget(oversubscribe=a.oversubscribe)
        sch = BatchScheduler(gdev, n_slots=n_slots, max_batch=max_batch, budget=budget)
    else:
        n_slots = 8
        gdev = GpuDevice(qb, tg, te, n_slots=n_slots, max_batch=256, max_K=scfg["K"], metric="ip",
                         base_f32=tb, rerank=True)
        run(warm, Scheduler(gdev, n_slots, 4096))
        sch = Scheduler(gdev, n_slots=n_slots, inflight_budget=6144)
    done = run(reqs, sch)
    s = summarize(done)
    hit = 0.0
    nqs = 0
    for r, p in zip(sorted(done, key=lambda r: r.rid), picks):
        for row, qi in zip(r.ids, p):
            hit += len(np.intersect1d(row[row >= 0], gt[qi, :10])) / 10.0
            nqs += 1
    s.update(recall10=hit / nqs, offered_rps=a.offered_rps,
             offered_qps=float(a.offered_rps * np.mean([len(r.queries) for r in reqs])),
             mode=a.serve_mode, slots=n_slots, max_running=sch.max_running_seen)
    if a.serve_mode == "batch":
        s.update(batches=sch.batches, max_batch_queries=sch.max_batch_seen,
                 budget={"lds_bytes": budget.lds_bytes, "hbm_bytes": budget.hbm_bytes,
                         "max_lds_in_flight": sch.max_inflight_seen[0],
                         "max_hbm_in_flight": sch.max_inflight_seen[1],
                         "waits_for_budget": sch.budget_waits})
    log(f"serving: {s}")
    return {"metric": "serving queries/s and p50/p99 latency (BF16 + FP32 rerank, 1 GPU)",
            "index": f"{a.serve_data}: {len(base)} x {base.shape[1]}", "value": s["qps"],
            "unit": "queries/s", "n_gpus": 1, **s}

def bench_shapes(a):
    """Launch-shape sweep of the headline search (1M x 128, L = 80, K = 100):
    gather variant x visited-cache size x waves per workgroup for FP32, BF16
    and FP8 storage (no rerank: the search's own shape), on the 10,000
    queries and on the 100,000 distinct steady-state queries. FP32 and BF16
    (lossless on these integers) rows are checked against the oracle's ids;
    FP8 rows report recall@10."""
    import torch
    import synth
    from paper_1907_06146_amd import graph_io, search, quantize
    cfg = synth.CONFIGS[WORKLOAD]
    gc = graph_io.load(WORKLOAD)
    base = synth.base_vectors(cfg)
    if synth.checksum(base) != gc["meta"]["base_sha"]:
        raise SystemExit("regenerated base vectors do not match the graph cache")
    q = synth.queries(cfg, base)
    droot = os.path.join(graph_io.default_root(), WORKLOAD)
    with open(os.path.join(droot, "sweep.json")) as f:
        L = a.L or json.load(f)["L_op"]
    K = cfg["K"]
    oi = np.load(os.path.join(droot, f"oracle_L{L}_ids.npy"), allow_pickle=False)
    gt = np.load(os.path.join(droot, "gt_ids.npy"), allow_pickle=False)
    dev = torch.device("cuda:0")
    tb = torch.from_numpy(base).to(dev)
    tg = graph_io.to_device(gc["graph"], dev)
    te = graph_io.to_device(gc["entry_ids"], dev)
    forms = {"f32": (tb, None), "bf16": quantize(tb, "bf16"), "fp8": quantize(tb, "fp8")}
    stream = torch.cuda.current_stream(dev)
    variants = {"f32": (0, 1, 2, 3, 4, 6), "bf16": (0, 2, 3, 4, 7, 8), "fp8": (0, 1, 2, 3)}
    plan = [(dt, v, hl, w) for dt in ("f32", "bf16", "fp8") for v in variants[dt]
            for hl in (11, 12) for w in (1, 2)]
    rows = []
    sets = (("headline", torch.from_numpy(q).to(dev)),
            ("steady", torch.from_numpy(synth.steady_queries(cfg)).to(dev)))
    for name, tq in sets:
        ids = torch.empty((len(tq), K), dtype=torch.int32, device=dev)
        dd = torch.empty((len(tq), K), dtype=torch.float32, device=dev)
        for dt, var, hl, wpb in plan:
            bse, sc = forms[dt]
            kw = dict(out=(ids, dd), gather_variant=var, hash_log2=hl, waves_per_block=wpb, dim_scale=sc)
            ms = _time(lambda: search(bse, tg, te, tq, K, L, **kw), 10 if name == "headline" else 3, 2, stream)
            r = dict(queries=len(tq), set=name, dtype=dt, variant=var, hash_log2=hl, waves_per_block=wpb,
                     ms=ms, qps=len(tq) / ms * 1e3)
            if name == "headline":
                got = ids.cpu().numpy()
                if dt == "fp8":
                    r["recall10"] = recall_at(got, gt, 10)
                else:
                    r["ids_equal_oracle"] = bool(np.array_equal(got.view(np.uint32), oi))
            log(f"shapes: {r}")
            rows.append(r)
    return {"metric": "launch-shape sweep of the 1M x 128 search (L = %d, K = %d)" % (L, K),
            "unit": "ms per launch", "rows": rows, "data": "synthetic (seeded)"}


def cpu_baseline(base, gc, q, K, L, cfg, sample):
    """The FP64 CPU oracle (Alg. 1, all host threads) on a bounded sample of
    the same queries, scaled to queries/s."""
    from oracle import core
    m = sample or len(q)
    qs = q[:m]
    t = time.perf_counter()
    core.search(base, gc["graph"], gc["entry_ids"], qs, K, L, cfg["metric"])
    one = time.perf_counter() - t
    reps = int(min(50, max(1, np.ceil(10.0 / max(one, 1e-3)))))  # about 10 s of CPU work
    t = time.perf_counter()
    for _ in range(reps):
        core.search(base, gc["graph"], gc["entry_ids"], qs, K, L, cfg["metric"])
    el = time.perf_counter() - t
    threads = core.threads()
    log(f"cpu oracle: {reps} x {m} queries in {el:.2f}s on {threads} threads")
    # one thread, as the paper times its searches: about 3 s of queries
    m1 = int(min(len(q), max(50, 3.0 * reps * m / el / max(threads, 1))))
    core.threads(1)
    try:
        t = time.perf_counter()
        core.search(base, gc["graph"], gc["entry_ids"], q[:m1], K, L, cfg["metric"])
        el1 = time.perf_counter() - t
    finally:
        core.threads(threads)
    log(f"cpu oracle: {m1} queries in {el1:.2f}s on 1 thread")
    avail, total = host_cores()
    return {"value": reps * m / el, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "threads": threads, "host_cpus_available": avail, "host_cpus_total": total,
            "sample": f"{reps} passes over {m} of the {len(q)} queries, same graph, L={L}, "
                      f"K={K}, FP64, {el:.1f} s",
            "single_thread": {"value": m1 / el1, "unit": "queries/s",
                              "sample": f"first {m1} queries, {el1:.1f} s"}}


if __name__ == "__main__":
    main()
