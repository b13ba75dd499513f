#!/usr/bin/env python3
"""Benchmark: time to a k-embedding at 1e-6 relative eigenvalue error.

Workload: sparse biharmonic classical scaling of a radially deformed
icosphere (subdivision level 7, n = 163,842 vertices, 8 seeded spherical
harmonics of degree <= 6, amplitude 5%), l = 2,000 geodesic farthest-point
landmarks, P thresholded to p_row = 10 (p = 809, nnz = 1.62M), W = squared
Dijkstra landmark distances, k = 3.  Inputs are synthetic and
generated from fixed seeds (cached on disk after the first run).

A step is one sbmds_embed call on device-resident inputs: start block,
all iterations of the precision schedule up to the certified 1e-6 bound,
and the embedding Z (left on the device).  Four forms are timed on the same
GPU, each to the same certified bound and at each block width of --blocks
(16 and 8: the three wanted eigenvalues and the five negative ones of larger
magnitude than the rest fit in 8): plain fp32 iterations from a random
start, bf16 bulk iterations refined in fp32, and fp32 iterations from the
landmark-MDS start and from the learned start (a network trained first, on
the GPU, on 12 smaller meshes of the same family).  The fastest is the chosen
form and gives `value`; the plain fp32 time at block 16 is reported beside
it.  The batched workload runs at block 16.

Prints one JSON line.  Only one GPU is used; --gpus above 1 is refused.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_form(sb, torch, prob, prec, steps, warmup, k, block, flags=0, start=None, tune_cache=None,
              mlp_weights=None):
    import numpy as np
    geo = {}
    if start in (sb.START_LMDS, sb.START_LEARNED):
        geo = {"xyz": torch.from_numpy(prob["V"].astype(np.float32)).cuda(),
               "landmark_vertex": torch.from_numpy(prob["landmarks"].astype(np.int32)).cuda()}
    p = sb.Problem.from_arrays(*(torch.from_numpy(prob[x]).cuda() for x in ("rowptr", "col", "val", "W")), **geo)
    kw = {}
    if start is not None:
        kw["start"] = start
    if mlp_weights is not None:
        kw["mlp_weights"] = mlp_weights
    t0 = time.perf_counter()
    ctx = sb.Context([p], k=k, block=block, prec=prec, flags=flags, tune_cache=tune_cache, **kw)
    log(f"create (upload, transpose, copies{', autotune' if tune_cache else ''}) {1e3 * (time.perf_counter() - t0):.1f} ms")
    Z = torch.empty((prob["n"], k), dtype=torch.float32, device="cuda")
    for _ in range(warmup):
        ctx.embed(Z_out=Z)
    ctx.reset_kernel_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = None
    for _ in range(steps):
        _, eig, reps, rc = ctx.embed(Z_out=Z)
        if rc != 0:
            raise RuntimeError(f"solve did not certify (status {rc})")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    stats = ctx.kernel_stats()
    ctx.close()
    return ms, eig[0], reps[0], stats


def time_batch(sb, torch, probs, k, block, steps, warmup, tune_cache, workload=None):
    """ms per certified solve of all meshes in one context (every launch
    covers every mesh) and of the same meshes one context each."""
    dev = [{x: torch.from_numpy(p[x]).cuda() for x in ("rowptr", "col", "val", "W")} for p in probs]
    ntot = sum(p["n"] for p in probs)

    def run(groups):
        ctxs, outs = [], []
        for g in groups:
            ps = [sb.Problem.from_arrays(dev[i]["rowptr"], dev[i]["col"], dev[i]["val"], dev[i]["W"]) for i in g]
            ctxs.append(sb.Context(ps, k=k, block=block, prec=sb.FP32, tune_cache=tune_cache))
            outs.append(torch.empty((sum(probs[i]["n"] for i in g), k), dtype=torch.float32, device="cuda"))
        for _ in range(warmup):
            for c, z in zip(ctxs, outs):
                c.embed(Z_out=z)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for c, z in zip(ctxs, outs):
                _, _, reps, rc = c.embed(Z_out=z)
                if rc != 0:
                    raise RuntimeError("a batched mesh did not certify")
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        for c in ctxs:
            c.close()
        return ms

    ms_batch = run([list(range(len(probs)))])
    ms_single = run([[i] for i in range(len(probs))])
    return {"meshes": len(probs), "vertices": ntot, "ms": round(ms_batch, 3),
            "meshes_per_s": round(len(probs) / (ms_batch * 1e-3), 1),
            "vertices_per_s": round(ntot / (ms_batch * 1e-3), 1),
            "ms_one_context_per_mesh": round(ms_single, 3), "dtype": "f32",
            "workload": workload or "16 meshes, n ~ U[2000, 20000] (bumpy tori and deformed geodesic spheres), "
                                    "l = n/50, p_row = 10, k = 3, fp32 -> f64 certify"}


FORM_NAMES = {
    "fp32": "fp32 -> f64 certify, random start",
    "bf16_fp32": "bf16 -> fp32 -> f64 certify, random start",
    "fp32_lmds": "fp32 -> f64 certify, landmark-MDS start",
    "fp32_learned": "fp32 -> f64 certify, learned start",
}


def train_start_net(sb, torch, configs, k, block, family="sphere6"):
    """Train the warm-start network on 12 smaller meshes of the workload's
    family (level-6 icospheres with sphere7's kind of deformation, or the
    small bumpy tori), other seeds, on targets the solver produces; returns
    the weights file."""
    from paper_1705_10887_amd import mlp

    t0 = time.perf_counter()
    if family.startswith("sphere"):
        meshes = configs.sphere_family(level=int(family[len("sphere"):]), log=log)
    else:
        meshes = configs.torus_family(size=family[len("torus"):] or "small", log=log)
    for m in meshes:
        m["landmarks"] = m["landmarks"].astype("int32")
        m["xyz"] = m["V"].astype("float32")
    targets = mlp.solve_targets(meshes, k=k, block=block)
    feats = [mlp.features(m["xyz"], m["landmarks"], m["W"]) for m in meshes]
    net, losses = mlp.train(feats, targets, k=k, steps=600, lr=3e-3, seed=0)
    path = os.path.join(configs.cache_dir(), f"mlp_{family}_k{k}.bin")
    net.save(path)
    net.close()
    torch.cuda.synchronize()
    log(f"trained start network: loss {losses[0]:.3e} -> {losses[-1]:.3e} "
        f"({len(meshes)} meshes, {1e3 * (time.perf_counter() - t0):.0f} ms incl. target solves)")
    return path


def spmm_at_scale(sb, torch, steps, pattern, n=2_000_000, l=2000, per_row=10, block=8, seed=7):
    """SpMM bandwidth where HBM, not latency, bounds it: a synthetic operator
    of n rows with per_row entries each over l landmarks, a symmetric l x l
    W, fp32, block 8; a few uncertified iterations with per-kernel timing.
    pattern "random": increasing random columns anywhere (no locality, the
    worst case for the transposed product's gathers of Y); "banded": a row's
    columns lie within ~3 per_row landmarks of a position that follows the
    row index, as on a mesh whose vertices and landmarks are both in spatial
    order (W then comes from landmarks along a helix in column order).  Launch
    shapes from the autotuner.  Not the headline workload: it shows what the
    kernels reach once a launch moves ~250 MB."""
    import numpy as np

    rng = np.random.default_rng(seed)
    if pattern == "random":
        gaps = rng.integers(1, l // (per_row + 1), size=(n, per_row))
        cols = np.cumsum(gaps, axis=1)
        cols += rng.integers(0, l - cols[:, -1:], dtype=np.int64)
    else:
        gaps = rng.integers(1, 4, size=(n, per_row))
        cols = np.cumsum(gaps, axis=1)
        span = int(cols[:, -1].max())
        cols += (np.arange(n, dtype=np.int64) * (l - 1 - span) // n)[:, None]
    col = cols.astype(np.int32).ravel()
    rowptr = np.arange(0, n * per_row + 1, per_row, dtype=np.int32)
    val = rng.random(n * per_row, dtype=np.float32)
    if pattern == "random":
        pts = rng.standard_normal((l, 3))
    else:
        # landmarks along a helix in column order, so that W (the squared
        # distances) agrees with the band: landmarks close in W share rows
        t = np.arange(l) / l
        pts = np.stack([np.cos(16 * np.pi * t), np.sin(16 * np.pi * t), 8 * t], axis=1)
    W = ((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1).astype(np.float32)
    p = sb.Problem.from_arrays(*(torch.from_numpy(a).cuda() for a in (rowptr, col, val, W)))
    from synth import configs
    tune = os.path.join(configs.cache_dir(), f"tune_scale_{pattern}_n{n}_l{l}_b{block}.txt")
    ctx = sb.Context([p], k=3, block=block, prec=sb.FP32, max_iter=4,
                     flags=sb.FLAG_KERNEL_TIMING | sb.FLAG_NO_CERTIFY, tune_cache=tune)
    Z = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    ctx.embed(Z_out=Z)
    ctx.reset_kernel_stats()
    for _ in range(max(1, steps // 4)):
        ctx.embed(Z_out=Z)
    torch.cuda.synchronize()
    stats = {s["name"]: s for s in ctx.kernel_stats()}
    ctx.close()
    out = {"workload": f"{pattern} operator, n={n}, {per_row} entries per row, l={l}, block {block}, fp32"}
    for name in ("spmm_rr.fp32", "spmm_t.fp32", "gemm.fp32"):
        s_ = stats.get(name)
        if s_ and s_["launches"]:
            us = 1e3 * s_["ms_total"] / s_["launches"]
            gbs = s_["bytes_total"] / (s_["ms_total"] * 1e-3) / 1e9
            out[name] = {"avg_us": round(us, 2), "GB/s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    return out


def precision_workload(sb, torch, configs, steps, warmup, k, blocks, learned=True):
    """The bumpy torus of 1024 x 512 vertices with 10,000 landmarks (W 400 MB
    in float32, the dense product's bytes dominate): plain fp32 against the
    bf16 bulk form, from the random start and (unless learned is False) from
    the learned start of a network trained on 12 tori of 192 x 96, with the
    per-kernel rates of the fastest.  Uses only an input already generated
    (about an hour of host time); None otherwise."""
    import numpy as np
    prob = configs.bumpy_torus(1024, 512, l=10000, generate=False)
    if prob is None:
        log("precision workload skipped: the 1024 x 512 torus input is not generated")
        return None
    weights = train_start_net(sb, torch, configs, k, blocks[0], family="torus192") if learned else None
    forms = {}
    for block in blocks:
        tune = os.path.join(configs.cache_dir(), f"tune_torus1024x512_k{k}_b{block}.txt")
        kinds = [("fp32", sb.FP32, None), ("bf16_fp32", sb.BF16_FP32, None)]
        if weights:
            kinds += [("fp32_learned", sb.FP32, sb.START_LEARNED), ("bf16_fp32_learned", sb.BF16_FP32, sb.START_LEARNED)]
        for name, prec, start in kinds:
            ms, eig, rep, _ = time_form(sb, torch, prob, prec, steps, warmup, k, block, start=start, tune_cache=tune,
                                        mlp_weights=weights if start else None)
            forms[f"{name}/b{block}"] = (ms, eig, rep, prec, block, tune, start)
            log(f"torus {name}/b{block} {ms:.3f} ms  iters {rep['iters_bf16']}+{rep['iters_fp32']}+"
                f"{rep['iters_fp64']}  start iters {rep['start_iters']}")
    chosen = min(forms, key=lambda f: forms[f][0])
    ms, eig, rep, prec, block, tune, start = forms[chosen]
    plain = forms[f"fp32/b{blocks[0]}"][0]
    _, _, _, stats = time_form(sb, torch, prob, prec, steps, 1, k, block, flags=sb.FLAG_KERNEL_TIMING, start=start,
                               tune_cache=tune, mlp_weights=weights if start else None)
    out = {
        "workload": "bumpy torus 1024 x 512 (n=524288), l=10000 FPS landmarks, p_row=10 "
                    f"(nnz={len(prob['col'])}), W=D^2_ll float32, k={k}",
        "forms_ms": {f: round(v[0], 4) for f, v in forms.items()},
        "chosen": chosen, "ms": round(ms, 4), "plain_fp32_ms": round(plain, 4),
        "chosen_over_plain": round(plain / ms, 3),
        "iters": {"bf16": rep["iters_bf16"], "fp32": rep["iters_fp32"], "fp64": rep["iters_fp64"],
                  "start": rep["start_iters"]},
        "err_bound": max(rep["err_bound"][:k]),
        "kernels": {s["name"]: {"avg_us": round(1e3 * s["ms_total"] / max(s["launches"], 1), 2),
                                **({"GB/s": round(s["bytes_total"] / (s["ms_total"] * 1e-3) / 1e9, 1),
                                    "frac": round(s["bytes_total"] / (s["ms_total"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                                  4)}
                                   if s["bytes_total"] > 0 else {})} for s in stats},
    }
    gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                        "bumpy_torus1024x512_l10000.npz")
    if os.path.exists(gold):
        g = np.load(gold, allow_pickle=False)
        if json.loads(str(g["meta"]))["input_sha1"] == configs.input_digest(prob):
            lam = g["lam"][:k]
            out["rel_eig_err_vs_stored_oracle"] = float(np.max(np.abs(np.asarray(eig) - lam) / np.abs(lam)))
    return out


def largest_workload(sb, torch, steps, warmup, k, block=16):
    """The shape of the paper-scale workload with the most landmarks: a
    1,800 x 1,000 torus grid (n = 1.8M) with 50,000 landmarks, W 10 GB in
    float32, on the seeded synthetic operator of synth.large (its biharmonic
    and geodesic inputs would take many hours on the host).  Plain fp32
    against the bf16 bulk form, random start, with the per-kernel rates of
    the faster; a few steps each (a solve streams W once per iteration)."""
    from synth import large

    t0 = time.perf_counter()
    prob = large.grid_torus_operator()
    log(f"largest workload generated in {time.perf_counter() - t0:.1f} s")
    steps = max(1, min(steps, 5))
    forms = {}
    for name, prec in (("fp32", sb.FP32), ("bf16_fp32", sb.BF16_FP32)):
        ms, eig, rep, _ = time_form(sb, torch, prob, prec, steps, 1, k, block)
        forms[f"{name}/b{block}"] = (ms, rep, prec)
        log(f"largest {name}/b{block} {ms:.3f} ms  iters {rep['iters_bf16']}+{rep['iters_fp32']}+{rep['iters_fp64']}")
    chosen = min(forms, key=lambda f: forms[f][0])
    ms, rep, prec = forms[chosen]
    _, _, _, stats = time_form(sb, torch, prob, prec, 1, 1, k, block, flags=sb.FLAG_KERNEL_TIMING)
    return {
        "workload": "synthetic torus grid 1800 x 1000 (n=1800000), l=50000 grid landmarks, 10 nearest landmarks "
                    f"per row (nnz={len(prob['col'])}), W=D^2+0.3D float32 (10 GB), k={k}, block {block}",
        "forms_ms": {f: round(v[0], 3) for f, v in forms.items()},
        "chosen": chosen, "ms": round(ms, 3), "plain_fp32_ms": round(forms[f"fp32/b{block}"][0], 3),
        "iters": {"bf16": rep["iters_bf16"], "fp32": rep["iters_fp32"], "fp64": rep["iters_fp64"]},
        "err_bound": max(rep["err_bound"][:k]),
        "kernels": {s["name"]: {"avg_us": round(1e3 * s["ms_total"] / max(s["launches"], 1), 1),
                                **({"GB/s": round(s["bytes_total"] / (s["ms_total"] * 1e-3) / 1e9, 1),
                                    "frac": round(s["bytes_total"] / (s["ms_total"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                                  4)}
                                   if s["bytes_total"] > 0 else {})} for s in stats},
    }


def cpu_baseline(prob, k, budget_s=20.0):
    """The float64 oracle (l x l reduction route) on the host cores."""
    import numpy as np

    from oracle import eig as oeig
    from synth import configs

    threads = int(os.environ.get("OPENBLAS_NUM_THREADS", os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    P = configs.operator_rounded(prob)
    W = prob["W"].astype(np.float64)
    times = []
    t_start = time.perf_counter()
    lam = None
    while time.perf_counter() - t_start < budget_s and len(times) < 10:
        t0 = time.perf_counter()
        lam, _, _ = oeig.top_k(P, W, k, route="reduction")
        times.append(time.perf_counter() - t0)
    times.sort()
    return {"value": round(times[len(times) // 2] * 1e3, 1), "unit": "ms", "cores": threads, "kind": "oracle",
            "sample": f"full solve (float64 l x l reduction route, k={k}), median of {len(times)} runs"}, lam


def traffic_from_profiles(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel source changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"{kernel}_sphere7_traffic.md")
    if not os.path.exists(path):
        return None
    want, value = None, None
    for line in open(path):
        if line.startswith("kernel_source_sha1:"):
            parts = line.split()
            want = (parts[1], parts[2])
        elif line.startswith("traffic_bytes_per_launch:"):
            try:
                value = float(line.split(":", 1)[1])
            except ValueError:
                return None
    if want is None or value is None:
        return None
    src = os.path.join(ROOT, "paper_1705_10887_amd", "csrc", want[0])
    if not os.path.exists(src):
        return None
    have = hashlib.sha1(open(src, "rb").read()).hexdigest()[:12]
    return value if have == want[1] else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3, help=">= 1; the first call learns the phase schedule")
    ap.add_argument("--k", type=int, default=3)
    ap.add_argument("--blocks", type=str, default="16,8",
                    help="comma-separated block widths; every form is timed at each")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-scale", action="store_true", help="skip the bandwidth-bound SpMM measurement")
    ap.add_argument("--no-learned", action="store_true", help="skip the landmark-MDS and learned-start forms")
    ap.add_argument("--no-torus", action="store_true", help="skip the 1024 x 512 torus, 10,000-landmark workload")
    ap.add_argument("--no-largest", action="store_true", help="skip the 1.8M-vertex, 50,000-landmark workload")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.empty(args.calibrate_copy << 18, dtype=torch.float32, device="cuda")
        a.fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the solve runs on a single MI355X and --gpus {args.gpus} "
              f"is not supported", file=sys.stderr)
        sys.exit(2)

    from synth import configs

    log("loading inputs")
    prob = configs.sphere7(log=log)
    import numpy as np
    import torch

    import paper_1705_10887_amd as sb

    torch.cuda.set_device(0)
    k = args.k
    blocks = [int(x) for x in args.blocks.split(",") if x]
    forms = {}

    def tune_for(block):
        return os.path.join(configs.cache_dir(), f"tune_sphere7_k{k}_b{block}.txt")

    def run_form(name, block, prec, start=None, weights=None):
        key = f"{name}/b{block}"
        log(f"timing {key}")
        ms, eig, rep, _ = time_form(sb, torch, prob, prec, args.steps, args.warmup, k, block, start=start,
                                    tune_cache=tune_for(block), mlp_weights=weights)
        forms[key] = {"ms": ms, "eig": eig, "rep": rep, "prec": prec, "start": start, "weights": weights,
                      "block": block, "form": name}
        log(f"{key} {ms:.3f} ms  iters {rep['iters_bf16']}+{rep['iters_fp32']}+{rep['iters_fp64']}"
            f"  start iters {rep['start_iters']}")

    weights = None
    if not args.no_learned:
        weights = train_start_net(sb, torch, configs, k, blocks[0], family="sphere6")
    for block in blocks:
        run_form("fp32", block, sb.FP32)
        run_form("bf16_fp32", block, sb.BF16_FP32)
        if weights is not None:
            run_form("fp32_lmds", block, sb.FP32, sb.START_LMDS)
            run_form("fp32_learned", block, sb.FP32, sb.START_LEARNED, weights)
    # the form that certifies fastest is the chosen one; the plain form is
    # fp32 from the random start at the first (reference) block width
    chosen = min(forms, key=lambda f: forms[f]["ms"])
    ch = forms[chosen]
    value, eigc, repc, chosen_prec, block = ch["ms"], ch["eig"], ch["rep"], ch["prec"], ch["block"]
    plain = f"fp32/b{blocks[0]}"
    ms_fp32 = forms[plain]["ms"]
    log("kernel timing pass")
    _, _, _, stats = time_form(sb, torch, prob, chosen_prec, args.steps, 1, k, block, flags=sb.FLAG_KERNEL_TIMING,
                               start=ch["start"], tune_cache=tune_for(block), mlp_weights=ch["weights"])
    # dominant bandwidth kernel of the timed form (per kernel and arithmetic)
    dom = max((s for s in stats if s["bytes_total"] > 0), key=lambda s: s["ms_total"])
    avg_ms = dom["ms_total"] / dom["launches"]
    bytes_per = dom["bytes_total"] / dom["launches"]
    achieved = bytes_per / (avg_ms * 1e-3) / 1e9
    spmm = [s for s in stats if s["name"].startswith(("spmm.", "spmm_rr."))]
    spmm_gbs = (sum(s["bytes_total"] for s in spmm) / (sum(s["ms_total"] for s in spmm) * 1e-3) / 1e9) if spmm else None
    traffic = traffic_from_profiles(dom["name"].replace(".", "_"))

    # batched workload (reduced scale, not the headline): 16 meshes of uneven
    # size in one context against the same meshes solved one context each
    batched = None
    if not args.no_batch:
        log("batched workload")
        batched = time_batch(sb, torch, configs.mesh_batch(log=log), k, blocks[0], args.steps, args.warmup,
                             os.path.join(configs.cache_dir(), f"tune_batch16_k{k}_b{blocks[0]}.txt"))
        log(f"batched {batched}")

    batched_full = None
    if not args.no_batch:
        from synth import large
        log("batched workload at full scale: 256 synthetic grid tori")
        probs256 = large.grid_torus_batch()
        batched_full = time_batch(sb, torch, probs256, k, blocks[0], max(1, min(args.steps, 3)), 1, None,
                                  workload="256 synthetic grid-torus meshes, n ~ U[2000, 200000] "
                                           f"({sum(p['n'] for p in probs256)} vertices, "
                                           f"{sum(p['l'] for p in probs256)} landmarks, "
                                           f"{sum(len(p['col']) for p in probs256)} stored entries), l ~ n/50, "
                                           "10 entries per row, k = 3, fp32 -> f64 certify, default launch shapes")
        del probs256
        log(f"batched full {batched_full}")

    at_scale = None
    if not args.no_scale:
        log("SpMM at a bandwidth-bound size")
        at_scale = {pat: spmm_at_scale(sb, torch, args.steps, pat) for pat in ("banded", "random")}
        log(f"at scale {at_scale}")

    torus = None
    if not args.no_torus:
        log("precision workload: 1024 x 512 torus, 10,000 landmarks")
        torus = precision_workload(sb, torch, configs, args.steps, args.warmup, k, blocks,
                                   learned=not args.no_learned)
        log(f"torus {torus}")

    largest = None
    if not args.no_largest:
        log("largest workload: n = 1.8M, 50,000 landmarks")
        largest = largest_workload(sb, torch, args.steps, args.warmup, k)
        log(f"largest {largest}")

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        cpu, lam_cpu = cpu_baseline(prob, k)
        err = float(np.max(np.abs(eigc - lam_cpu[:k]) / np.abs(lam_cpu[:k])))
        log(f"chosen vs oracle rel eig err {err:.2e}")
        if err > 1e-6:
            raise RuntimeError(f"eigenvalues off the oracle by {err:.2e}")

    out = {
        "metric": "ms to k-embedding at 1e-6 rel eig err (chosen vs plain FP32); SpMM % HBM peak",
        "value": round(value, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(value, 4),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "bf16+f32" if chosen_prec == sb.BF16_FP32 else "f32",
        "data": "synthetic",
        "config": {
            "workload": "sphere7: icosphere level 7 (n=163842) deformed by 8 seeded spherical harmonics, "
                        "l=2000 FPS landmarks, p_row=10 (nnz=1620000), W=D^2_ll float32",
            "n": int(prob["n"]), "l": int(prob["l"]), "nnz": int(len(prob["col"])), "k": k, "block": block,
            "chosen": f"{FORM_NAMES[ch['form']]}, block {block}",
        },
        "plain_fp32_ms": round(ms_fp32, 4),
        "plain_fp32_form": f"{FORM_NAMES['fp32']}, block {blocks[0]}",
        "chosen_over_plain": round(ms_fp32 / value, 3),
        "forms_ms": {f: round(v["ms"], 4) for f, v in forms.items()},
        "iters": {"bf16": repc["iters_bf16"], "fp32": repc["iters_fp32"], "fp64": repc["iters_fp64"],
                  "start": repc["start_iters"]},
        "err_bound": max(repc["err_bound"][:k]),
        "spmm_hbm_frac": round(spmm_gbs / HBM_PEAK_GBS, 4) if spmm_gbs else None,
        "kernels": {s["name"]: {"avg_us": round(1e3 * s["ms_total"] / max(s["launches"], 1), 2),
                                "launches_per_step": round(s["launches"] / args.steps, 2),
                                **({"GB/s": round(s["bytes_total"] / (s["ms_total"] * 1e-3) / 1e9, 1)}
                                   if s["bytes_total"] > 0 else {})} for s in stats},
        "roofline": {
            "kernel": dom["name"],
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "bytes_per_launch": bytes_per,
            **({"note": "the launch also runs the b x b Rayleigh-Ritz step in the block that completes the Gram "
                        "reduction; its time is in the duration, its bytes are not"}
               if dom["name"].startswith("spmm_rr.") else {}),
        },
        "cpu_baseline": cpu,
        "batched": batched,
        "batched_full_scale": batched_full,
        "spmm_at_scale": at_scale,
        "precision_workload": torus,
        "largest_workload": largest,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
