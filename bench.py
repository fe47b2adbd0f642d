#!/usr/bin/env python3
"""kNN-graph build benchmark on one MI355X.

Workload (default): n = 1,000,000 points, d = 50, FP32, a 50-component
Gaussian mixture with anisotropic covariances (eigenvalues log-uniform on
[0.1, 10]), k = 15.  One step = one blocking nndescent_build call on data
already resident in HBM (init, every iteration, final re-rank).  Steps use
algorithm seeds 0..steps-1 after `warmup` untimed calls.

Two forms are timed: plain FP32 NNDescent (random init, FP32 MFMA join) and
the BF16 form seeded by a trained encoder (BF16 MFMA join, FP32 re-rank of
the final lists); the headline line is the latter, both are in "forms".

Reported: points/s = n * steps / wall time of the timed steps (and the
spread of the per-step times), recall@15 of every timed step's graph on
10,000 sampled rows against the GPU exact path (knn_exact_query,
parity-tested against the CPU oracle; the graph's own distances are not
trusted: indices are checked and distances recomputed in FP64), the
minimum over steps being the headline recall, the roofline of the dominant kernel (the local
join: algorithmic bytes / its HIP-event time, both accumulated by the
library over the timed steps; counter-measured HBM bytes per launch from the
committed rocprofv3 summary while its kernel source is unchanged), an
attainable-bandwidth copy measurement, the BF16 form's join distance error
against FP64, the encoder's training cost (outside the timed region), and
the CPU oracle on a bounded sample of the workload (sequential NNDescent at
the FP32 form's settings with its recall, and the exact oracle's per-query
rate on all host cores), the fuzzy graph (UMAP weights) built from the
headline graph, and the exact path (knn_exact, both precisions) on the
70,000 x 784 pixel-like set.  Other configurations (--config pixel70k |
scale10m) print the same line.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# NNDescent settings of the two forms (K_b, rho, caps); delta is the paper's 0.015.
# The BF16 forms keep K_b = 2k = 30 entries, the FP32 re-rank's width; the
# FP32 form K_b = 31 (each the smallest list that keeps recall@15 above 0.98
# by about 0.002 over seeds 0-4).
# rev_slots = s (= K_b at rho = 1): the join reads the reverse-edge table
# directly; a larger table (the library default) joins more reverse edges per
# iteration but, on this workload, costs more time than it saves at equal recall.
FORMS = {
    "fp32": dict(precision="fp32", build_k=31, sample_rate=1.0, max_iters=30, delta=0.015,
                 join_cap=4, cand_slots=64, rev_slots=31),
    "bf16-learned": dict(precision="bf16", build_k=30, sample_rate=1.0, max_iters=30, delta=0.015,
                         join_cap=4, cand_slots=96, rev_slots=30, init_kind="encoder", proj_count=4, proj_window=8),
    # controls for the encoder's benefit (--form all): same BF16 form, random
    # init, and seeding through an untrained encoder of the same shape
    "bf16-random": dict(precision="bf16", build_k=30, sample_rate=1.0, max_iters=30, delta=0.015,
                        join_cap=4, cand_slots=96, rev_slots=30),
    "bf16-untrained": dict(precision="bf16", build_k=30, sample_rate=1.0, max_iters=30, delta=0.015,
                           join_cap=4, cand_slots=96, rev_slots=30, init_kind="encoder", proj_count=4, proj_window=8),
    # FP16 MFMA distances (exact operands for FP16-stored data), same settings
    "fp16-learned": dict(precision="fp16", build_k=30, sample_rate=1.0, max_iters=30, delta=0.015,
                         join_cap=4, cand_slots=96, rev_slots=30, init_kind="encoder", proj_count=4, proj_window=8),
    # E independent BF16 + learned runs joined through continuations seeded with
    # their union (--form ensemble): the 10M workload's route past the recall
    # one run reaches at the largest supported K_b
    "bf16-learned-e2": dict(precision="bf16", build_k=32, sample_rate=1.0, max_iters=30, delta=0.015,
                            join_cap=4, cand_slots=96, rev_slots=32, init_kind="encoder", proj_count=4,
                            proj_window=8, ensemble=2),
    "bf16-learned-e3": dict(precision="bf16", build_k=32, sample_rate=1.0, max_iters=30, delta=0.015,
                            join_cap=4, cand_slots=96, rev_slots=32, init_kind="encoder", proj_count=4,
                            proj_window=8, ensemble=3),
}
# encoder training (reported separately, not in the timed region)
TRAIN = dict(n=100_000, seed=100, k=15, steps=1000, batch=4096, lr=2e-3, precision="bf16")

CONFIGS = {
    "gmm1m": dict(n=1_000_000, d=50, desc="1,000,000 x 50 FP32, 50-component anisotropic GMM, k=15"),
    "pixel70k": dict(n=70_000, d=784, desc="70,000 x 784 FP32 pixel-like (10 clusters, 1/255 levels), k=15"),
    "scale10m": dict(n=10_000_000, d=50,
                     desc="10,000,000 x 50 FP16, 200-component anisotropic GMM, Zipf(1.1) weights, k=15"),
}


def make_data(config: str, seed: int = 0, n=None):
    import numpy as np
    from paper_2603_04035_amd import datagen
    c = CONFIGS[config]
    n = c["n"] if n is None else n
    if config == "gmm1m":
        return datagen.gmm_anisotropic(n=n, d=c["d"], comps=50, seed=seed)
    if config == "scale10m":
        return datagen.gmm_anisotropic(n=n, d=c["d"], comps=200, zipf=1.1, seed=seed, dtype=np.float16)
    return datagen.pixel_like(n=n, seed=seed)


def train_encoder(config: str):
    """Encoder trained on a fresh sample of the same distribution and its exact graph."""
    import torch
    import paper_2603_04035_amd as knn
    Xt = torch.from_numpy(make_data(config, seed=TRAIN["seed"], n=TRAIN["n"])).to("cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    idx, _ = knn.knn_exact(Xt, TRAIN["k"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    enc = knn.Encoder(Xt.shape[1], seed=1)
    log = enc.train(Xt, idx, steps=TRAIN["steps"], batch=TRAIN["batch"], lr=TRAIN["lr"], seed=3,
                    precision=TRAIN["precision"])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return enc, {"train_points": TRAIN["n"], "exact_graph_s": round(t1 - t0, 3),
                 "train_s": round(t2 - t1, 3), "steps": TRAIN["steps"], "batch": TRAIN["batch"],
                 "precision": TRAIN["precision"],
                 "loss_first": float(log[:20].mean()), "loss_last": float(log[-20:].mean())}


def exact_rows(X, rows, k):
    """The exact k-th neighbour distance of each sampled row (GPU exact path,
    parity-tested against the CPU oracle)."""
    import torch
    import paper_2603_04035_amd as knn
    rows_t = torch.as_tensor(rows, dtype=torch.int64, device=X.device)
    _, edist = knn.knn_exact_query(X[rows_t].contiguous(), X, k, q_self=rows_t.to(torch.int32))
    return rows_t, edist[:, k - 1].double()


def recall_gpu(X, G, D, rows, k, exact=None):
    """Tie-aware recall@k of the graph's sampled rows.  The returned
    distances are not trusted: an entry counts only if its index is in
    range, not the row itself and not repeated in the row, and its distance
    recomputed here in FP64 from X is within the exact k-th neighbour
    distance (relative slack 1e-5 for the exact path's FP32 rounding)."""
    import torch
    rows_t, kth = exact_rows(X, rows, k) if exact is None else exact
    n = X.shape[0]
    hits = 0
    for c0 in range(0, len(rows), 1000):
        r = rows_t[c0:c0 + 1000]
        g = G[r, :k].long()
        ok = (g >= 0) & (g < n) & (g != r[:, None])
        # a repeated index counts once: every copy after the first is dropped
        ok &= ~((g[:, :, None] == g[:, None, :]) & torch.ones(k, k, dtype=torch.bool, device=g.device).tril(-1)).any(2)
        gc = torch.where(ok, g, r[:, None])
        xr = X[r].double()
        true = ((X[gc].double() - xr[:, None, :]) ** 2).sum(-1).sqrt()
        good = ok & (true <= kth[c0:c0 + 1000, None] * (1.0 + 1e-5))
        hits += int(good.sum().item())
    return hits / (len(rows) * k)


def host_cpu():
    """Host cores visible to this process and the CPU model."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"os_cpu_count": os.cpu_count(), "omp_threads": int(os.environ.get("OMP_NUM_THREADS", "0")) or None,
            "model": model}


def cpu_baseline(Xnp, k, form, sample_n, exact_queries=1000):
    """The CPU oracle on a bounded sample of the workload.

    * Sequential NNDescent (one core) at the timed FP32 form's settings
      (K_b, rho, delta, iteration cap) on the first sample_n rows, with its
      recall@k on 500 of those rows against the oracle's exact lists of the
      same subset.  NNDescent's cost grows faster than n, so the rate on the
      subset overstates the full workload's.
    * The exact oracle (FP64 brute force, OpenMP over all host cores) on
      exact_queries rows of the full workload: queries/s.
    """
    import numpy as np
    import oracle
    from paper_2603_04035_amd import datagen
    sub = np.ascontiguousarray(Xnp[:sample_n])
    p = FORMS[form]
    t0 = time.perf_counter()
    idx, _, iters, _ = oracle.nndescent(sub, p["build_k"], max_iters=p["max_iters"], rho=p["sample_rate"],
                                        delta=p["delta"], seed=0)
    dt = time.perf_counter() - t0
    rows = datagen.sample_queries(sample_n, 500, seed=2)
    _, O2 = oracle.exact_knn(sub, k, rows=rows)
    rec = oracle.recall_at_k(sub, rows, idx[rows, :k], np.sqrt(O2[:, -1]), k)
    q = datagen.sample_queries(Xnp.shape[0], exact_queries, seed=3)
    t1 = time.perf_counter()
    oracle.exact_query(Xnp, Xnp[q], k, q_self=q)
    de = time.perf_counter() - t1
    return {"value": round(sample_n / dt, 1), "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": f"sequential NNDescent (K_b={p['build_k']}, rho={p['sample_rate']}, delta={p['delta']}, "
                      f"the FP32 form's settings) on the first {sample_n} of the {Xnp.shape[0]} rows, "
                      f"{dt:.1f} s, {iters} iterations"
                      + ("; rate on the subset overstates the full workload's" if sample_n < Xnp.shape[0] else ""),
            "recall_at_15": round(float(rec), 5), "host": host_cpu(),
            "exact_oracle": {"queries": exact_queries, "s": round(de, 2),
                             "queries_per_s": round(exact_queries / de, 1), "cores": host_cpu()["omp_threads"]
                             or os.cpu_count(),
                             "note": "FP64 brute force over all rows, OpenMP across queries"}}


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` (a CONFIGS key) from the
    committed rocprofv3 counter summaries (FETCH_SIZE and WRITE_SIZE scaled
    by a plain copy's readings), or None when no summary covers that kernel
    and workload or the kernel source changed since."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        text = open(path).read()
        for block in re.findall(r"```json\n(.*?)\n```", text, re.S):
            try:
                rec = json.loads(block)
            except ValueError:
                continue
            if rec.get("kernel") != kernel or rec.get("workload") != workload:
                continue
            src = os.path.join(ROOT, rec["source"])
            if not os.path.exists(src):
                continue
            h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
            if h == rec.get("source_sha256_16"):
                return int(rec["bytes_per_launch"]), os.path.relpath(path, ROOT)
    return None, None


def copy_bandwidth(mib: int = 1024, reps: int = 5):
    """Attainable HBM bandwidth of a plain device-to-device copy (read + write
    bytes / event time), the measured counterpart of the 8 TB/s peak."""
    import torch
    nbytes = mib << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    return round(2 * nbytes / (ms * 1e-3) / 1e9, 1)


def join_roofline(stats, n, d, p, kernel, workload):
    """Local-join roofline: algorithmic bytes per launch / HIP-event time per
    launch against the HBM peak (every form's join gathers rows and offers
    candidates at random; its Gram runs on MFMA, whose algorithmic rate, 2 d
    flops per joined pair, is reported beside it)."""
    import numpy as np
    K = stats[-1]["build_k"]
    s_ = int(np.ceil(p["sample_rate"] * K))
    rb = 4 if p["precision"] == "fp32" else 2
    launches = sum(st["iters"] for st in stats)
    gathered_rows = sum(st["bytes_gathered"] for st in stats) / (d * rb)
    emitted = sum(sum(st["emitted"]) for st in stats)
    list_bytes = launches * n * (4 * s_ + 4 * K + 2 * 8 * s_)   # new_f, old_f, 4-byte reverse slots read+reset
    alg_bytes = gathered_rows * (d * rb + 8) + list_bytes + 8 * emitted
    join_ms = sum(st["ms_join"] for st in stats)
    achieved = alg_bytes / (join_ms * 1e-3) / 1e9
    traffic, source = measured_traffic(kernel, workload)
    pairs = sum(st["pairs_joined"] for st in stats)
    gram_tflops = 2.0 * d * pairs / (join_ms * 1e-3) / 1e12
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "gram_tflops": round(gram_tflops, 2),
            "traffic": traffic, "traffic_source": source, "kernel": kernel, "launches": launches,
            "alg_bytes_per_launch": int(alg_bytes / max(launches, 1)),
            "alg_flops_per_launch": int(2 * d * pairs / max(launches, 1)),
            "ms_per_launch": round(join_ms / max(launches, 1), 4)}


def distance_error(X, Xnp, k, p, rows):
    """Relative error of the BF16 form's working-list squared distances (BF16
    MFMA join, norm expansion, FP32 accumulation) against FP64 distances of
    the input values, over every listed pair of the sampled rows."""
    import numpy as np
    import paper_2603_04035_amd as knn
    _, _, _, (si, sd, _) = knn.nndescent_build(X, k, seed=0, return_state=True, **p)
    si, sd = si.cpu().numpy()[rows], sd.cpu().numpy()[rows].astype(np.float64)
    ok = si >= 0
    a = np.repeat(rows, si.shape[1]).reshape(si.shape)[ok]
    b = si[ok]
    X64 = Xnp.astype(np.float64)
    true = ((X64[a] - X64[b]) ** 2).sum(axis=1)
    m = true > 0
    e = np.abs(sd[ok][m] - true[m]) / true[m]
    return {"pairs": int(m.sum()), "rel_max": float(e.max()), "rel_p50": float(np.percentile(e, 50)),
            "rel_p99": float(np.percentile(e, 99))}


def exact_path(X, k, reps=3):
    """knn_exact of X among itself in each precision: wall time per call and
    the GEMM's algorithmic rate 2 n^2 d / time against the MFMA peak of the
    precision (FP32 157.3 TFLOP/s, BF16 and FP16 2500 TFLOP/s dense)."""
    import torch
    import paper_2603_04035_amd as knn
    n, d = X.shape
    out = {}
    for prec, peak in (("fp32", 157.3), ("bf16", 2500.0), ("fp16", 2500.0)):
        knn.knn_exact(X, k, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            knn.knn_exact(X, k, precision=prec)
        torch.cuda.synchronize()
        ms = 1000.0 * (time.perf_counter() - t0) / reps
        tflops = 2.0 * n * n * d / (ms * 1e-3) / 1e12
        out[prec] = {"ms": round(ms, 3), "roofline": {"bound": "mfma", "achieved": round(tflops, 2), "peak": peak,
                                                      "unit": "TFLOP/s", "frac": round(tflops / peak, 4),
                                                      "traffic": None,
                                                      "note": "2 n^2 d flops / whole knn_exact call"}}
    return out


def chunk_knob(X, k, limits_mib=(0, 1024, 512, 384, 320, 288, 256), reps=2):
    """knn_exact_query_limited of X among itself (FP32) under decreasing
    scratch limits: ms per call, or the error when even one 128-query chunk
    does not fit beside the staged reference set."""
    import torch
    import paper_2603_04035_amd as knn
    n = X.shape[0]
    qs = torch.arange(n, dtype=torch.int32, device=X.device)
    out = []
    for mib in limits_mib:
        lim = int(mib) << 20
        try:
            knn.knn_exact_query(X, X, k, q_self=qs, workspace_limit=lim)
        except knn.KnnError as e:
            out.append({"limit_mib": mib, "error": str(e).split(":")[0]})
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            knn.knn_exact_query(X, X, k, q_self=qs, workspace_limit=lim)
        torch.cuda.synchronize()
        out.append({"limit_mib": mib or None, "ms": round(1000.0 * (time.perf_counter() - t0) / reps, 3)})
    return out


def pca_quality(X, p=50, k=10, reps=3):
    """PCA of X to p dimensions (FP64 Gram on MFMA, subspace iteration) and
    the quality metrics of the 2-D PCA embedding (exact ranks in both
    spaces): ms per call.  Rooflines: the Gram's n d (d + 1) FP64 flops per
    PCA call against the FP64 MFMA peak (78.6 TFLOP/s), and the rank pass's
    2 n^2 d FP32 flops per quality call against the FP32 MFMA peak."""
    import torch
    import paper_2603_04035_amd as knn
    n, d = X.shape
    knn.pca(X, p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        knn.pca(X, p)
    torch.cuda.synchronize()
    ms_pca = 1000.0 * (time.perf_counter() - t0) / reps
    Y = knn.pca(X, 2)[0]
    m = knn.quality(X, Y, k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        m = knn.quality(X, Y, k)
    torch.cuda.synchronize()
    ms_q = 1000.0 * (time.perf_counter() - t0) / reps
    gram_tf = n * d * (d + 1) / (ms_pca * 1e-3) / 1e12
    rank_tf = 2.0 * n * n * d / (ms_q * 1e-3) / 1e12
    return {"pca": {"ms": round(ms_pca, 3), "p": p,
                    "roofline": {"bound": "mfma", "achieved": round(gram_tf, 2), "peak": 78.6, "unit": "TFLOP/s",
                                 "frac": round(gram_tf / 78.6, 4), "traffic": None,
                                 "note": "n d (d+1) FP64 Gram flops / whole knn_pca call"}},
            "quality": {"ms": round(ms_q, 3), "k": k, "embedding": "2-D PCA",
                        "knn_preservation": round(m[0], 5), "trustworthiness": round(m[1], 5),
                        "continuity": round(m[2], 5),
                        "roofline": {"bound": "mfma", "achieved": round(rank_tf, 2), "peak": 157.3, "unit": "TFLOP/s",
                                     "frac": round(rank_tf / 157.3, 4), "traffic": None,
                                     "note": "2 n^2 d rank-pass flops / whole knn_quality call (the rank pass "
                                             "also yields the exact k-NN in X; the call also runs the 2-D "
                                             "exact k-NN and rank pass)"}}}


def fuzzy_measure(G, D, reps=3):
    """knn_fuzzy_graph on the built graph: ms per call and points/s."""
    import torch
    import paper_2603_04035_amd as knn
    knn.fuzzy_graph(G, D)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = knn.fuzzy_graph(G, D)
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / reps
    n, k = G.shape
    return {"ms": round(ms, 3), "points_per_s": round(n / (ms * 1e-3), 1), "nnz": int(out[4].numel()),
            "edges_in": int(n * k)}


def progress(msg):
    """One line per finished phase on stderr (the JSON result goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_form(X, k, form, steps, warmup, rows, config, encoder=None, Xnp=None):
    import torch
    import paper_2603_04035_amd as knn
    p = dict(FORMS[form])
    if form == "bf16-untrained":
        encoder = knn.Encoder(X.shape[1], seed=1)
    if p.get("init_kind") == "encoder":
        p["encoder"] = encoder
    for w in range(warmup):
        knn.nndescent_build(X, k, seed=1000 + w, **p)
    torch.cuda.synchronize()
    progress(f"{form}: {warmup} warmup build(s) done")
    stats, walls, graphs = [], [], []
    t0 = time.perf_counter()
    for s in range(steps):
        ts = time.perf_counter()
        G, D, st = knn.nndescent_build(X, k, seed=s, **p)   # blocking: returns after the build
        walls.append(time.perf_counter() - ts)
        stats.append(st)
        graphs.append(G)   # a reference: each call returns new tensors
        progress(f"{form}: step {s + 1}/{steps} {1000.0 * walls[-1]:.2f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n, d = X.shape
    # recall of every timed step's graph (one algorithm seed each), after the timing
    ex = exact_rows(X, rows, k)
    per_step = [recall_gpu(X, g, None, rows, k, exact=ex) for g in graphs]
    del graphs
    recall = min(per_step)
    kern = {"fp32": "nnd_join_mfma_kernel<0>", "bf16": "nnd_join_mfma_kernel<1>",
            "fp16": "nnd_join_mfma_kernel<2>"}[p["precision"]]
    last = stats[-1]
    cfg = {kk: vv for kk, vv in p.items() if kk != "encoder"}
    cfg["build_k"] = last["build_k"]
    err = None
    if p["precision"] != "fp32" and Xnp is not None:
        err = distance_error(X, Xnp, k, p, rows[:2000])
    progress(f"{form}: recall {recall:.5f}")
    import numpy as np
    return {"value": round(n * steps / wall, 1), "ms_per_step": round(1000.0 * wall / steps, 3),
            "ms_per_step_std": round(1000.0 * float(np.std(walls)), 3),
            "bf16_distance_error_vs_fp64": err,
            "recall_at_15": round(recall, 5), "recall_ok": recall >= 0.98,
            "recall_at_15_per_step": [round(x, 5) for x in per_step], "iters": last["iters"],
            "params": cfg,
            "ms_breakdown": {kk: round(last[kk], 3) for kk in
                             ("ms_init", "ms_sample", "ms_join", "ms_merge", "ms_final", "ms_total")},
            "per_iter": {"updates": last["updates"], "offers": last["emitted"],
                         "ms_join": [round(x, 3) for x in last["ms_join_iter"]]},
            "roofline": join_roofline(stats, n, d, p, kern, config),
            "_graph": (G, D)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="gmm1m", choices=sorted(CONFIGS))
    ap.add_argument("--form", default="both", choices=sorted(FORMS) + ["both", "all", "ensemble"],
                    help="both: fp32 and bf16-learned; all: also the bf16-random and bf16-untrained controls")
    ap.add_argument("--k", type=int, default=15)
    ap.add_argument("--recall-rows", type=int, default=10000)
    ap.add_argument("--cpu-sample", type=int, default=50_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-only", action="store_true",
                    help="only run the CPU oracle leg (no GPU) on the first --cpu-sample rows of --config; "
                         "--cpu-sample 1000000 times the full 1M workload")
    ap.add_argument("--no-exact", action="store_true", help="skip the exact-path timing of the default line")
    ap.add_argument("--exact", action="store_true",
                    help="only time the exact path (knn_exact of the workload in FP32, BF16 and FP16, and FP32 "
                         "under decreasing scratch limits)")
    ap.add_argument("--pca-quality", action="store_true",
                    help="only time knn_pca (p = 50) and knn_quality of the 2-D PCA embedding on --config")
    ap.add_argument("--fuzzy-only", action="store_true",
                    help="only build the FP32-form graph once and run the fuzzy graph on it 3 times (profiling)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (counter calibration)")
    args = ap.parse_args()

    if args.copy_probe:
        import torch
        nbytes = args.copy_probe << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nbytes, "copies": 3}), flush=True)
        return

    if args.cpu_only:
        Xnp = make_data(args.config)
        cpu = cpu_baseline(Xnp, args.k, "fp32", min(args.cpu_sample, Xnp.shape[0]))
        print(json.dumps({"cpu_baseline": cpu, "config": {"workload": CONFIGS[args.config]["desc"]}}), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the kNN graph build runs on a single device "
              "and has no multi-GPU path; run it with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_04035_amd import datagen

    k = args.k
    Xnp = make_data(args.config)
    n, d = Xnp.shape
    X = torch.from_numpy(Xnp).to("cuda")
    torch.cuda.synchronize()
    if args.exact:
        print(json.dumps({"exact_path": exact_path(X, k), "chunk_knob": chunk_knob(X, k),
                          "config": {"workload": CONFIGS[args.config]["desc"]}, "n": n, "d": d, "k": k}),
              flush=True)
        return
    if args.pca_quality:
        print(json.dumps({"pca_quality": pca_quality(X, k=min(k, 16)),
                          "config": {"workload": CONFIGS[args.config]["desc"]}}), flush=True)
        return
    if args.fuzzy_only:
        import paper_2603_04035_amd as knn
        G, D, _ = knn.nndescent_build(X, k, seed=0, **FORMS["fp32"])
        print(json.dumps({"fuzzy_graph": fuzzy_measure(G, D),
                          "config": {"workload": CONFIGS[args.config]["desc"]}}), flush=True)
        return
    rows = datagen.sample_queries(n, args.recall_rows, seed=2)
    forms = {"both": ["fp32", "bf16-learned"],
             "all": ["fp32", "bf16-learned", "bf16-random", "bf16-untrained", "fp16-learned"],
             "ensemble": ["bf16-learned", "bf16-learned-e2", "bf16-learned-e3"]}.get(args.form, [args.form])
    results, training = {}, None
    encoder = None
    if any(FORMS[f].get("init_kind") == "encoder" and f != "bf16-untrained" for f in forms):
        encoder, training = train_encoder(args.config)
        progress(f"encoder trained in {training['train_s']} s")
    for f in forms:
        results[f] = run_form(X, k, f, args.steps, args.warmup, rows, args.config, encoder, Xnp)
    head = "bf16-learned" if "bf16-learned" in results else forms[0]
    h = results[head]
    G, D = h["_graph"]
    fuzzy = fuzzy_measure(G, D)
    progress(f"fuzzy graph {fuzzy['ms']} ms")
    for r in results.values():
        r.pop("_graph", None)
    del G, D
    exact = pca_q = None
    if not args.no_exact and args.config == "gmm1m":
        Xp = torch.from_numpy(make_data("pixel70k")).to("cuda")
        exact = {"workload": CONFIGS["pixel70k"]["desc"], **exact_path(Xp, k)}
        progress(f"exact path fp32 {exact['fp32']['ms']} ms, bf16 {exact['bf16']['ms']} ms")
        pca_q = pca_quality(Xp)
        progress(f"pca {pca_q['pca']['ms']} ms, quality {pca_q['quality']['ms']} ms")
        del Xp

    copy_gbs = copy_bandwidth()
    for r in results.values():
        rl = r["roofline"]
        rl["frac_of_measured_copy"] = round(rl["achieved"] / copy_gbs, 4)
    cpu = None
    if not args.no_cpu_baseline and int(os.environ.get("RANK", "0")) == 0:
        cpu = cpu_baseline(Xnp, k, "fp32", min(args.cpu_sample, n))
        progress(f"cpu baseline {cpu['value']:.0f} points/s")

    out = {
        "metric": "kNN graph build points/sec at recall@15>=0.98 (NNDescent)",
        "value": h["value"], "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": h["ms_per_step"], "ms_per_step_std": h["ms_per_step_std"],
        "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16" if FORMS[head]["precision"] == "bf16" else "f32", "data": "synthetic",
        "config": {"workload": CONFIGS[args.config]["desc"], "form": head, "k": k},
        "recall_at_15": h["recall_at_15"], "recall_ok": h["recall_ok"],
        "roofline": h["roofline"], "hbm_copy_gbs": copy_gbs,
        "cpu_baseline": cpu,
        "forms": results,
        "encoder_training": training,
        "fuzzy_graph": fuzzy,
        "exact_path": exact,
        "pca_quality": pca_q,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
