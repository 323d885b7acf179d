"""Benchmark: particles/s for build + neighbours + gravity of the RCB tree on
one MI355X, 4,194,304-particle Plummer sphere in a 10% uniform background
(density contrast ~1e4), N_ll = 12, theta = 0.7, mixed form (FP32
leaf-relative interactions, FP64 moments and Taylor shift), next to the FP64
form and the FP64 CPU oracle.

One step = rcb_build + rcb_walk + rcb_neighbours_count + rcb_neighbours_fill
+ rcb_gravity on inputs already resident in HBM, tree destroyed at the end.

Prints ONE JSON line (rank 0). Extra fields: the FP64-form throughput, the
mixed form's error against the FP64 form, per-phase times (HIP events on the
library's stream inside the timed region), the roofline of the dominant
kernel (k_gravity, one launch per step), the per-leaf HBM model of walk +
gravity, and the oracle's CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks and the derived vector peak available to these kernels
# (packed FP32 is disabled, so FP32 issues at the FP64 rate):
# 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz = 78.6 TFLOP/s.
PEAK_HBM_GBS = 8000.0
PEAK_VALU_TFLOPS = 78.6

# Algorithmic operation counts of one interaction, frozen from one count of
# the straightforward formulas (an FMA counts as 2, a reciprocal or
# reciprocal square root as 1); kernel rewrites that need fewer instructions
# do not change them.
FLOP_P2P = 38          # near pair: offset, r^2, rsqrt, rcp, q, both spline branches, m F v
FLOP_M2L = 226         # far pair: D1..D5, Q x, x.Q.x, 3 f + 6 J + 10 H coefficients
FLOP_L2P = 66          # per sink: f + J d + H[d, d]/2


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--theta", type=float, default=0.7)
    ap.add_argument("--n-ll", type=int, default=12)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--pure-mac", action="store_true",
                    help="gravity lists from the geometric MAC alone (reachable cells may be accepted)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-leaves", type=int, default=2048)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration for profiles)")
    return ap.parse_args()


def main():
    a = _args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: runs on one GPU only (no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import workloads as W
    from paper_1108_0028_amd import Tree

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    cloud = W.plummer_background()
    n = cloud.n
    arrs = [torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in cloud.arrays()]
    torch.cuda.synchronize()

    def step(prec, ev=None):
        """One step: build, walk, neighbour search, gravity; events (if given)
        bracket each phase on the stream the library launches on."""
        rec = (lambda i: ev[i].record()) if ev is not None else (lambda i: None)
        rec(0)
        t = Tree(*arrs, n_ll=a.n_ll, theta=a.theta, precision=prec, pure_mac=a.pure_mac)
        rec(1)
        t.walk()
        rec(2)
        off, ids = t.neighbours()
        rec(3)
        acc = t.gravity()
        rec(4)
        t.destroy()
        return acc, off

    def timed(prec, steps, warmup):
        for _ in range(warmup):
            step(prec)
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            step(prec, evs[i])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ph = [sum(e[j].elapsed_time(e[j + 1]) for e in evs) / steps for j in range(4)]
        return (t1 - t0) / steps, dict(zip(("build", "walk", "neighbours", "gravity"), ph))

    if a.calib_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    sec, phases = timed(a.precision, a.steps, a.warmup)
    value = n / sec
    grav_ms = phases["gravity"]   # one launch of k_gravity per step

    # work counts of this tree for the roofline (outside the timed region)
    t = Tree(*arrs, n_ll=a.n_ll, theta=a.theta, precision=a.precision, pure_mac=a.pure_mac)
    cnt = t.export("count").to(torch.int64)
    near = t.export("near").to(torch.int64)
    in_field = (near & (1 << 30)) == 0     # entries of the gravity near field
    near = near & 0x3FFFFFFF
    noff = t.export("near_off")
    foff = t.export("far_off")
    inf = t.info()              # list totals are known once the lists exist
    nleaf = 1 << inf["k"]
    leaf = torch.arange(nleaf, device=dev)
    L_A = noff[1:] - noff[:-1]
    F_A = foff[1:] - foff[:-1]
    n_A = cnt[nleaf:2 * nleaf]
    P_A = torch.zeros(nleaf, dtype=torch.int64, device=dev).index_add_(
        0, torch.repeat_interleave(leaf, L_A), cnt[near] * in_field)
    pairs = int((P_A * n_A).sum())
    t.destroy()
    far_total = inf["far_total"]
    near_total = inf["near_total"]

    flops = FLOP_P2P * pairs + FLOP_M2L * far_total + FLOP_L2P * n
    achieved_tf = flops / (grav_ms * 1e-3) / 1e12
    traffic = _profiled_traffic("k_gravity_mixed") if a.precision == "mixed" else None
    roofline = {"kernel": f"k_gravity<{a.precision}>", "bound": "alu", "achieved": achieved_tf,
                "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s", "frac": achieved_tf / PEAK_VALU_TFLOPS,
                "traffic": traffic, "kernel_ms": grav_ms, "pairs": pairs, "far_pairs": far_total,
                "near_cells": near_total, "walk_requeued_groups": inf["walk_requeued"]}
    # the per-leaf streaming model of the walk + gravity (bytes each lowest-level
    # cell would read on its own): nodes tested V ~ 2 (F + L) in a binary walk
    V_A = 2 * (F_A + L_A)
    if a.precision == "mixed":
        model_b = int((32 * V_A + 8 * L_A + 80 * F_A + 20 * P_A + 32 * n_A).sum())
    else:
        model_b = int((64 * V_A + 8 * L_A + 80 * F_A + 40 * P_A + 64 * n_A).sum())
    wg_ms = phases["walk"] + phases["gravity"]
    walk_model = {"bytes": model_b, "ms": wg_ms, "floor_ms": model_b / (PEAK_HBM_GBS * 1e9) * 1e3,
                  "frac": model_b / (PEAK_HBM_GBS * 1e9) / (wg_ms * 1e-3)}

    # the other form and the mixed-vs-FP64 error
    other = "fp64" if a.precision == "mixed" else "mixed"
    sec_o, _ = timed(other, max(2, a.steps // 3), 1)
    acc_m, off = step("mixed")
    acc_d, _ = step("fp64")
    am = torch.stack([v.double() for v in acc_m], 1)
    ad = torch.stack([v.double() for v in acc_d], 1)
    da = (am - ad).norm(dim=1)
    na = ad.norm(dim=1)
    rms = float(na.pow(2).mean().sqrt())
    rel = da / na.clamp_min(1e-300)
    err = {"gate_max": float((da / na.clamp_min(1e-3 * rms)).max()),
           "mean": float(rel.mean()), "p99": float(torch.quantile(rel.float(), 0.99))}

    out = {
        "metric": "particles/sec (build+neighbours+gravity), 4M Plummer: mixed FP32 vs FP64 at stated err",
        "value": value,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64 (mixed)" if a.precision == "mixed" else "f64",
        "data": "synthetic (seeded Plummer + uniform background)",
        "config": {"workload": "plummer_background N=4194304: 90% Plummer (b=1, r<=20) + 10% uniform "
                               "sphere R=10.357, equal masses, analytic h for ~50 neighbours",
                   "n": n, "n_ll": a.n_ll, "theta": a.theta, "precision": a.precision,
                   "walk": "pure MAC" if a.pure_mac else "reachability overrides MAC (paper)"},
        "phases_ms": phases,
        "other_form": {"precision": other, "value": n / sec_o, "ms_per_step": sec_o * 1e3},
        "mixed_vs_fp64_error": err,
        "neighbours_total": int(off[-1]),
        "roofline": roofline,
        "walk_gravity_hbm_model": walk_model,
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cloud, a)
    print(json.dumps(out), flush=True)


def _profiled_traffic(name):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    profiles/<name>_counters.md, if the kernel's sources are unchanged since
    the counters were taken (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{name}_counters.md")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            rec[k.strip()] = v.strip().strip("`")
    try:
        h = hashlib.sha256()
        for f in rec["sources"].split(", "):
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() != rec["sources_sha256"]:
            return None
        return int(rec["hbm_bytes_per_launch"])
    except (KeyError, OSError, ValueError):
        return None


def cpu_baseline(cloud, a):
    """The FP64 oracle (unchanged) on the host: full tree build (serial), then
    walk, neighbours and gravity for a random sample of leaves (OpenMP over
    leaves), with all threads and again with one; throughput scaled to
    particles/s of build + neighbours + gravity."""
    import numpy as np

    from oracle import oracle as O
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    threads = O.threads()
    t0 = time.perf_counter()
    ot = O.OracleTree(*cloud.arrays(), n_ll=a.n_ll)
    t1 = time.perf_counter()
    rng = np.random.default_rng(0)
    leaves = np.sort(rng.choice(ot.n_leaves, min(a.cpu_leaves, ot.n_leaves), replace=False)) + ot.n_leaves

    def sampled():
        s0 = time.perf_counter()
        ot.walk(a.theta, leaves, pure_mac=a.pure_mac)
        s1 = time.perf_counter()
        _, _, valid = ot.neighbours()
        s2 = time.perf_counter()
        ot.gravity()
        s3 = time.perf_counter()
        return int(valid.sum()), (s1 - s0, s2 - s1, s3 - s2)

    n_s, ph = sampled()
    O.set_threads(1)
    _, ph1 = sampled()
    O.set_threads(threads)
    build = t1 - t0
    rate = lambda p: 1.0 / (build / cloud.n + sum(p) / max(1, n_s))
    return {"value": rate(ph), "unit": "particles/s", "cores": threads, "kind": "oracle",
            "single_thread_value": rate(ph1), "cpu": model,
            "phases_s": {"build_all": build, "walk": ph[0], "neighbours": ph[1], "gravity": ph[2],
                         "walk_1thread": ph1[0], "neighbours_1thread": ph1[1], "gravity_1thread": ph1[2]},
            "sample": f"oracle build of all {cloud.n} particles (serial, {build:.1f} s) + walk, "
                      f"neighbours and gravity of {len(leaves)} random leaves ({n_s} particles, "
                      f"{sum(ph):.1f} s on {threads} OpenMP threads, {sum(ph1):.1f} s on 1)"}


if __name__ == "__main__":
    main()
