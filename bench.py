"""Benchmark: particles/s for build + neighbours + gravity of the RCB tree on
one MI355X, 4,194,304-particle Plummer sphere in a 10% uniform background
(density contrast ~1e4), N_ll = 12, theta = 0.7, mixed form (FP32
leaf-relative interactions, FP64 moments and Taylor shift), next to the FP64
form and the FP64 CPU oracle.

One step = rcb_build + rcb_walk + rcb_neighbours_count + rcb_neighbours_fill
+ rcb_gravity on inputs already resident in HBM, tree destroyed at the end.

Prints ONE JSON line. Besides the contract fields: the FP64 form's
throughput, the mixed form's error against the FP64 form, per-phase times
(HIP events on the library's stream inside the timed region) with each
phase's algorithmic work against its own bound, the roofline of the dominant
kernel (k_gravity, one launch per step), the VJP's time against the
forward's, the device memory a step holds, the force error against the
direct sum on sampled particles, and the oracle's CPU baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6        # vector FP64
PEAK_FP32_TFLOPS = 157.3       # vector FP32

# Algorithmic operation weights per unit of work (fixed; kernel rewrites do
# not change them): a near pair ~27 flop (FP32 in the mixed form), a far
# (leaf, node) pair ~400 flop (FP64 M2L of reading A), a sink ~40 flop (L2P),
# a (node, leaf) walk test ~20 flop (FP64: reachability and MAC), a candidate
# pair of the neighbour cull ~8 flop (FP64 squared distance and compare).
FLOP_P2P = 27
FLOP_M2L = 400
FLOP_L2P = 40
FLOP_TEST = 20
FLOP_CULL = 8


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
    ap.add_argument("--no-extras", action="store_true",
                    help="time the steps only (for profiler runs): no counts, VJP, other form or errors")
    ap.add_argument("--cpu-leaves", type=int, default=2048)
    ap.add_argument("--direct-leaves", type=int, default=160,
                    help="lowest-level cells whose particles get the exact direct sum (cpu_baseline leg)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration for profiles)")
    return ap.parse_args()


def main():
    a = _args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1",
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

    def step(prec, ev=None, keep=False):
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
        if keep:
            t.kept_ids = ids   # the CSR stays alive with the tree
            return t, acc, off
        t.destroy()
        return None, acc, off

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

    # device memory one step holds (library pool + neighbour CSR), before any
    # other tree has been made
    mem = None
    if not a.no_extras:
        from paper_1108_0028_amd import release_cache
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        t_keep, acc_keep, off_keep = step(a.precision, keep=True)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        # the same with the caches emptied: what the live tree, its lists and
        # the step's outputs hold (the library's scratch of the step went back)
        release_cache()
        torch.cuda.empty_cache()
        free2 = torch.cuda.mem_get_info()[0]
        mem = {"bytes": int(free0 - free1), "bytes_per_particle": (free0 - free1) / n,
               "live_bytes_per_particle": (free0 - free2) / n,
               "basis": "device memory taken by one step, from hipMemGetInfo: bytes = held after the step "
                        "(the live tree with its lists and neighbour search state, the accelerations and "
                        "offsets, and the scratch the library and torch keep for the next step); "
                        "live_bytes_per_particle = the same once their kept scratch is released"}
        t_keep.destroy()
        del off_keep, acc_keep
        # the neighbour search alone: its scratch (slab, overflow pool, queues)
        # and the CSR it returns, on a walked tree, with the library's and
        # torch's caches emptied first
        torch.cuda.synchronize()
        release_cache()
        torch.cuda.empty_cache()
        t_nb = Tree(*arrs, n_ll=a.n_ll, theta=a.theta, precision=a.precision, pure_mac=a.pure_mac)
        t_nb.walk()
        torch.cuda.synchronize()
        f0 = torch.cuda.mem_get_info()[0]
        off_nb, ids_nb = t_nb.neighbours()
        torch.cuda.synchronize()
        f1 = torch.cuda.mem_get_info()[0]
        csr = off_nb.numel() * off_nb.element_size() + ids_nb.numel() * ids_nb.element_size()
        mem["neighbours"] = {"bytes_per_particle": (f0 - f1) / n, "csr_bytes_per_particle": csr / n,
                             "scratch_bytes_per_particle": (f0 - f1 - csr) / n,
                             "basis": "hipMemGetInfo around the count + fill calls on a walked tree: the "
                                      "library's scratch (64-slot slab, overflow chunks, queues) plus the "
                                      "returned CSR (int64 offsets, int32 ids); allocations round up to "
                                      "2 MiB"}
        t_nb.destroy()
        del off_nb, ids_nb

    sec, phases = timed(a.precision, a.steps, a.warmup)
    value = n / sec
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
    }
    if a.no_extras:
        print(json.dumps(out), flush=True)
        return

    # work counts of this tree (outside the timed region)
    t, acc_m, off = step(a.precision, keep=True)
    counts = _work_counts(t, off, n)
    roof, phase_roof = _rooflines(counts, phases, a.precision, n, t.info()["k"])
    out["roofline"] = roof
    out["phases_roofline"] = phase_roof
    out["neighbours_total"] = counts["neighbours"]
    out["memory"] = mem
    # VJP on the same tree after gravity (the far coefficients are kept)
    out["vjp"] = _vjp_timing(t, n, phases, a.precision)
    t.destroy()
    # the deterministic form (no atomics) on a tree of the same inputs
    td = Tree(*arrs, n_ll=a.n_ll, theta=a.theta, precision=a.precision, pure_mac=a.pure_mac,
              deterministic=True)
    td.gravity()
    vd = _vjp_timing(td, n, phases, a.precision)
    out["vjp_deterministic"] = {"ms": vd["ms"], "vjp_over_forward": vd["vjp_over_forward"],
                                "basis": "rcb_params.deterministic = 1: node adjoints and source-side "
                                         "near terms summed per node / per cell in a fixed order "
                                         "(label sort of the group lists on each call)"}
    td.destroy()

    # the other form and the mixed-vs-FP64 error
    other = "fp64" if a.precision == "mixed" else "mixed"
    sec_o, _ = timed(other, max(2, a.steps // 3), 1)
    _, acc_o, _ = step(other)
    acc = {a.precision: torch.stack([v.double() for v in acc_m], 1),
           other: torch.stack([v.double() for v in acc_o], 1)}
    da = (acc["mixed"] - acc["fp64"]).norm(dim=1)
    na = acc["fp64"].norm(dim=1)
    rms = float(na.pow(2).mean().sqrt())
    rel = da / na.clamp_min(1e-300)
    out["other_form"] = {"precision": other, "value": n / sec_o, "ms_per_step": sec_o * 1e3}
    out["mixed_vs_fp64_error"] = {"gate_max": float((da / na.clamp_min(1e-3 * rms)).max()),
                                  "mean": float(rel.mean()), "p99": float(torch.quantile(rel.float(), 0.99))}
    if not a.no_cpu_baseline:
        base, direct = cpu_baseline(cloud, a)
        out["cpu_baseline"] = base
        out["force_error_vs_direct_sum"] = _direct_errors(direct, acc, a.theta)
    print(json.dumps(out), flush=True)


def _work_counts(t, off, n):
    """Units of work of one step, counted from the tree's own lists."""
    import torch
    dev = off.device
    cnt = t.export("count").to(torch.int64)
    near = t.export("near").to(torch.int64)
    noff = t.export("near_off")
    inf = t.info()              # list totals are known once the per-cell lists exist
    nleaf = 1 << inf["k"]
    in_field = (near & (1 << 30)) == 0      # entries of the gravity near field
    cand = (near & (1 << 31)) != 0          # entries holding neighbour candidates
    lab = near & 0x3FFFFFFF
    L_A = noff[1:] - noff[:-1]
    n_A = cnt[nleaf:2 * nleaf]
    leaf = torch.repeat_interleave(torch.arange(nleaf, device=dev), L_A)
    P_A = torch.zeros(nleaf, dtype=torch.int64, device=dev).index_add_(0, leaf, cnt[lab] * in_field)
    C_A = torch.zeros(nleaf, dtype=torch.int64, device=dev).index_add_(0, leaf, cnt[lab] * cand)
    return {"pairs": int((P_A * n_A).sum()), "far_pairs": inf["far_total"], "near_cells": inf["near_total"],
            "cand_particles": int(C_A.sum()), "cand_pairs": int((C_A * n_A).sum()),
            "neighbours": int(off[-1]), "walk_nodes": inf["walk_nodes"], "walk_tests": inf["walk_tests"],
            "walk_requeued_groups": inf["walk_requeued"], "n": n}


def _profiled(kernel):
    """FETCH_SIZE + WRITE_SIZE bytes per launch of `kernel` from a committed
    rocprofv3 counter summary (profiles/*_counters.md), while the sources it
    lists are unchanged (else None)."""
    pdir = os.path.join(ROOT, "profiles")
    for fn in sorted(os.listdir(pdir)):
        if not fn.endswith("_counters.md"):
            continue
        rec, cur = {}, None
        for line in open(os.path.join(pdir, fn)):
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                rec[k.strip()] = v.strip().strip("`")
        try:
            h = hashlib.sha256()
            for f in rec["sources"].split(", "):
                h.update(open(os.path.join(ROOT, f), "rb").read())
            if h.hexdigest() != rec["sources_sha256"]:
                continue
            for item in rec["hbm_bytes_per_launch"].split("; "):
                name, val = item.rsplit("=", 1)
                if name.strip() == kernel:
                    cur = int(val)
        except (KeyError, OSError, ValueError):
            continue
        if cur is not None:
            return cur
    return None


def _rooflines(c, phases, prec, n, k):
    """The dominant kernel's roofline and each phase's algorithmic work against
    its own bound (HBM bytes against 8 TB/s; flops against the vector peak of
    their type; a mixed FP32/FP64 phase against the time both parts would need
    at their peaks)."""
    mixed = prec == "mixed"

    def alu(f32, f64, ms):
        floor_s = f32 / (PEAK_FP32_TFLOPS * 1e12) + f64 / (PEAK_FP64_TFLOPS * 1e12)
        tot = f32 + f64
        ach = tot / (ms * 1e-3) / 1e12
        peak = tot / floor_s / 1e12 if floor_s > 0 else PEAK_FP64_TFLOPS
        return {"bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
                "flops_fp32": f32, "flops_fp64": f64}

    def hbm(nbytes, ms):
        ach = nbytes / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": ach / PEAK_HBM_GBS, "bytes": nbytes}

    # gravity: near pairs (FP32 in the mixed form), far pairs (FP64 M2L), L2P per sink
    near_f = FLOP_P2P * c["pairs"] + FLOP_L2P * n
    far_f = FLOP_M2L * c["far_pairs"]
    g = alu(near_f if mixed else 0, far_f + (0 if mixed else near_f), phases["gravity"])
    kname = "k_gravity<true, false>" if mixed else "k_gravity<false, false>"
    g.update({"kernel": kname, "kernel_ms": phases["gravity"], "traffic": _profiled(kname),
              "basis": f"{FLOP_P2P} flop per near pair ({c['pairs']}), {FLOP_M2L} per far pair "
                       f"({c['far_pairs']}), {FLOP_L2P} per sink ({n}); one launch per step, timed by "
                       "HIP events on its stream"})
    # build: compulsory HBM bytes N (48 k + 100) (each of the k levels reads
    # and writes the node's particle data and order; the leaf level, bounds,
    # gather and records the rest)
    b = hbm(n * (48 * k + 100), phases["build"])
    b["basis"] = f"N (48 k + 100) bytes, k = {k}"
    b["traffic"] = {k_: _profiled(k_) for k_ in ("k_subtree", "k_scatter_classify", "k_chunk_reduce<0>",
                                                 "k_part_count<false>", "k_part_count<true>")}
    # walk: FP64 tests of (node, visiting cell) pairs; also the node records it loads
    w = alu(0, FLOP_TEST * c["walk_tests"], phases["walk"])
    w["hbm_bytes"] = 64 * c["walk_nodes"]
    w["hbm_frac"] = w["hbm_bytes"] / (phases["walk"] * 1e-3) / (PEAK_HBM_GBS * 1e9)
    w["basis"] = (f"{FLOP_TEST} FP64 flop per (node, cell) test ({c['walk_tests']}); 64 B per node record "
                  f"loaded per group of 8 cells ({c['walk_nodes']})")
    w["traffic"] = _profiled("k_walk_wide<false, 1024, 4>")
    # neighbours: FP64 distance test of every candidate pair; bytes: candidates
    # (position + id), ids written and compacted, offsets
    nb = alu(0, FLOP_CULL * c["cand_pairs"], phases["neighbours"])
    nbytes = 28 * c["cand_particles"] + 12 * c["neighbours"] + 16 * n
    nb["hbm_bytes"] = nbytes
    nb["hbm_frac"] = nbytes / (phases["neighbours"] * 1e-3) / (PEAK_HBM_GBS * 1e9)
    nb["basis"] = (f"{FLOP_CULL} FP64 flop per candidate pair ({c['cand_pairs']}); 28 B per candidate "
                   f"particle of a cell ({c['cand_particles']}), 12 B per neighbour id, 16 B per particle")
    nb["traffic"] = {k_: _profiled(k_) for k_ in ("k_neigh<true>", "k_nb_compact", "k_nb_compact_long")}
    g["counts"] = c
    return g, {"build": b, "walk": w, "neighbours": nb, "gravity": {k_: v for k_, v in g.items()
                                                                     if k_ != "counts"}}


def _vjp_timing(t, n, phases, prec):
    """rcb_gravity_vjp on the step's tree (after its gravity call), N(0,1)
    cotangents; HIP events on the library's stream."""
    import torch
    import workloads as W
    dt = torch.float32 if prec == "mixed" else torch.float64
    g = [torch.from_numpy(v).to("cuda:0", dt) for v in W.cotangents(n)]
    t.vjp(*g)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    reps = 3
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        t.vjp(*g)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    fwd = phases["build"] + phases["walk"] + phases["gravity"]
    far = "k_vjp_far<float, 0>" if prec == "mixed" else "k_vjp_far<double, 0>"
    near = "k_vjp_near<true, true>" if prec == "mixed" else "k_vjp_near<false, true>"
    return {"ms": ms, "forward_ms": fwd, "vjp_over_forward": ms / fwd,
            "basis": "forward = build + walk + gravity of the timed steps; the VJP reuses the tree, its "
                     "lists and the far coefficients kept by the gravity call",
            "traffic": {far: _profiled(far), near: _profiled(near)}}


def _direct_errors(direct, acc, theta):
    """Relative force errors (Sec. 3.1) of both forms at the bench's theta on
    the sampled particles against the exact FP64 direct sum."""
    import numpy as np
    idx, ref = direct
    out = {"theta": theta, "sinks": int(idx.size),
           "reference": "oracle at theta = 0 (every cell near: the kernel-softened direct sum over all "
                        "particles, FP64) on the particles of randomly sampled lowest-level cells"}
    na = np.linalg.norm(ref, axis=1)
    rms = float(np.sqrt(np.mean(na * na)))
    for prec, a in acc.items():
        got = a.cpu().numpy()[idx]
        da = np.linalg.norm(got - ref, axis=1)
        eps = da / np.maximum(na, 1e-300)
        out[prec] = {"mean": float(eps.mean()), "p99": float(np.quantile(eps, 0.99)),
                     "max": float(eps.max()), "frac_below_1pct": float((eps < 0.01).mean()),
                     "gate_max": float((da / np.maximum(na, 1e-3 * rms)).max())}
    return out


def cpu_baseline(cloud, a):
    """The FP64 oracle (unchanged) on the host: full tree build, then walk,
    neighbours and gravity for a random sample of leaves (OpenMP over
    leaves), with all threads and again with one; throughput scaled to
    particles/s of build + neighbours + gravity. Afterwards, untimed, the
    oracle at theta = 0 on another sample of leaves: the exact direct sum for
    their particles."""
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

    def near_far():
        """Table 1's NG and FG: the near and the far field alone, same leaves."""
        s0 = time.perf_counter()
        ot.gravity(parts=1)
        s1 = time.perf_counter()
        ot.gravity(parts=2)
        s2 = time.perf_counter()
        return s1 - s0, s2 - s1

    n_s, ph = sampled()
    ng, fg = near_far()
    O.set_threads(1)
    _, ph1 = sampled()
    O.set_threads(threads)
    build = t1 - t0
    rate = lambda p: 1.0 / (build / cloud.n + sum(p) / max(1, n_s))
    per = lambda sec: sec / max(1, n_s) * cloud.n   # seconds for all particles at the sampled rate
    base = {"value": rate(ph), "unit": "particles/s", "cores": threads, "kind": "oracle",
            "single_thread_value": rate(ph1), "cpu": model,
            "phases_s": {"build_all": build, "walk": ph[0], "neighbours": ph[1], "gravity": ph[2],
                         "walk_1thread": ph1[0], "neighbours_1thread": ph1[1], "gravity_1thread": ph1[2]},
            "table1_s": {"TB": build, "N": per(ph[1]), "NG": per(ng), "FG": per(fg), "G": per(ph[2]),
                         "walk": per(ph[0]),
                         "basis": f"Table 1's columns for all {cloud.n} particles on {threads} threads: the "
                                  "build as measured, the rest scaled from the sampled leaves (NG: near field "
                                  "alone, FG: far field and its Taylor evaluation alone, G: both)"},
            "sample": f"oracle build of all {cloud.n} particles ({build:.1f} s, levels split in parallel) + "
                      f"walk, neighbours and gravity of {len(leaves)} random leaves ({n_s} particles, "
                      f"{sum(ph):.1f} s on {threads} OpenMP threads, {sum(ph1):.1f} s on 1)"}
    # exact direct sums for the error report (not timed)
    rng = np.random.default_rng(1)
    dl = np.sort(rng.choice(ot.n_leaves, min(a.direct_leaves, ot.n_leaves), replace=False)) + ot.n_leaves
    ot.walk(0.0, dl)
    topo = ot.topology()
    pos = np.concatenate([np.arange(topo["first"][l], topo["first"][l] + topo["count"][l]) for l in dl])
    idx = topo["perm"][pos]
    ref = np.stack(ot.gravity(), 1)[idx]
    return base, (idx, ref)


if __name__ == "__main__":
    main()
