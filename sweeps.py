"""Paper-shaped sweeps of the RCB tree on one GPU (Sec. 3).

* ``table1``: the N_ll sweep of Table 1 -- depth L, fraction of particles with
  a relative force error below 1%, and the time of the build (TB), the walk,
  the neighbour search (N) and the gravity (G, near and far field fused in one
  kernel), with the near-pair and far-pair counts that split G.
* ``accuracy``: the cumulative distribution of relative errors
  eps_i = |da_i| / |a_i| for theta from 0.4 to 1.0 (Fig. accuracy).
* ``scaling``: build + walk + neighbours + gravity on the clumpy unit cube
  (50% uniform, 64 Gaussian clumps) from 2^20 to 10^8 particles, mixed and
  FP64 forms: particles/s per size (the O(N) claim of Sec. 3.2.3), with the
  neighbour lists of sampled particles checked against an all-pairs search
  and their accelerations against the direct sum over all particles.
* ``splits``: the three ways to cut a cell (centre of mass, centre of number,
  median position; Sec. 2.1 "Load balancing") on the Sobol sphere and on an
  unequal binary, where the median split creates "renegades": error
  statistics and build time of each.

Workload: a quasi-random Sobol sphere (500,000 particles, smoothing lengths
for ~105 neighbours, as in Table 1). The reference accelerations are the FP64
tree at theta = 0, which is the direct kernel-smoothed sum (no cell is
accepted, so every pair is summed directly; Sec. 2.4.1). Prints a markdown
table and one JSON line per row.

    python sweeps.py table1 [--n 500000] [--precision fp64]
    python sweeps.py accuracy [--pure-mac]
    python sweeps.py splits
    python sweeps.py scaling [--sizes 1048576,...]
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


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["table1", "accuracy", "splits", "scaling"])
    ap.add_argument("--sizes", default="1048576,4194304,16777216,67108864,100000000")
    ap.add_argument("--samples", type=int, default=256)
    ap.add_argument("--n", type=int, default=500_000)
    ap.add_argument("--neighbours", type=int, default=105)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--theta", type=float, default=0.7, help="theta of the table1 sweep")
    ap.add_argument("--n-ll", type=int, default=12, help="N_ll of the accuracy sweep")
    ap.add_argument("--nll-list", default="1,3,6,12,24,48,64,128")
    ap.add_argument("--theta-list", default="0.4,0.5,0.6,0.7,0.8,0.9,1.0")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--pure-mac", action="store_true")
    return ap.parse_args()


def main():
    a = _args()
    import numpy as np
    import torch

    import workloads as W
    from paper_1108_0028_amd import Tree

    assert torch.cuda.is_available(), "sweeps.py needs a GPU"
    dev = torch.device("cuda:0")
    if a.what == "scaling":
        return scaling(a, np, torch, W, Tree, dev)
    cloud = W.sobol_sphere(a.n, a.neighbours)
    arrs = [torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in cloud.arrays()]

    if a.what == "splits":
        return splits(a, np, torch, W, Tree, dev)

    def run(n_ll, theta, prec, ev=None):
        rec = (lambda i: ev[i].record()) if ev is not None else (lambda i: None)
        rec(0)
        t = Tree(*arrs, n_ll=n_ll, theta=theta, precision=prec, pure_mac=a.pure_mac)
        rec(1)
        t.walk()
        rec(2)
        off, _ = t.neighbours()
        rec(3)
        acc = t.gravity()
        rec(4)
        return t, off, acc

    def timed(n_ll, theta, prec):
        run(n_ll, theta, prec)[0].destroy()                      # warm-up
        rows = []
        for _ in range(a.reps):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
            t, off, acc = run(n_ll, theta, prec, ev)
            torch.cuda.synchronize()
            rows.append([ev[j].elapsed_time(ev[j + 1]) for j in range(4)])
            t.destroy()
        med = np.median(np.array(rows), 0)
        return dict(zip(("TB", "walk", "N", "G"), (float(v) for v in med)))

    def pairs(t):
        cnt = t.export("count").to(torch.int64)
        near = t.export("near").to(torch.int64)
        in_field = (near & (1 << 30)) == 0
        near = near & 0x3FFFFFFF
        noff, foff = t.export("near_off"), t.export("far_off")
        nleaf = 1 << t.info()["k"]
        L_A = noff[1:] - noff[:-1]
        P_A = torch.zeros(nleaf, dtype=torch.int64, device=dev).index_add_(
            0, torch.repeat_interleave(torch.arange(nleaf, device=dev), L_A), cnt[near] * in_field)
        n_A = cnt[nleaf:2 * nleaf]
        return int((P_A * n_A).sum()), int(foff[-1])

    def errors(acc, ref):
        am = torch.stack([v.double() for v in acc], 1)
        da = (am - ref).norm(dim=1)
        na = ref.norm(dim=1)
        eps = (da / na).cpu().numpy()
        return {"mean": float(eps.mean()), "p99": float(np.quantile(eps, 0.99)),
                "max": float(eps.max()),
                "P<1e-4": float((eps < 1e-4).mean()), "P<1e-3": float((eps < 1e-3).mean()),
                "P<2e-3": float((eps < 2e-3).mean()), "P<1e-2": float((eps < 1e-2).mean())}

    t0 = time.perf_counter()
    rt, _, racc = run(12, 0.0, "fp64")
    ref = torch.stack(racc, 1)
    torch.cuda.synchronize()
    ref_s = time.perf_counter() - t0
    rt.destroy()
    head = {"workload": f"sobol_sphere N={a.n}, ~{a.neighbours} neighbours", "precision": a.precision,
            "walk": "pure MAC" if a.pure_mac else "reachability overrides MAC",
            "reference": f"FP64 tree at theta = 0 (direct sum), {ref_s:.1f} s"}
    print(json.dumps(head), flush=True)

    if a.what == "table1":
        print(f"\n| N_ll | L | P<1% | mean eps | TB ms | walk ms | N ms | G ms | near pairs | far pairs | "
              f"neighbours/particle |\n|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|", flush=True)
        for nll in [int(v) for v in a.nll_list.split(",")]:
            ph = timed(nll, a.theta, a.precision)
            t, off, acc = run(nll, a.theta, a.precision)
            e = errors(acc, ref)
            npair, nfar = pairs(t)
            k = t.info()["k"]
            nb = float(off[-1]) / a.n
            t.destroy()
            row = {"n_ll": nll, "L": k, **ph, "near_pairs": npair, "far_pairs": nfar,
                   "neighbours_per_particle": nb, **e}
            print(f"| {nll} | {k} | {e['P<1e-2']:.4f} | {e['mean']:.2e} | {ph['TB']:.2f} | {ph['walk']:.2f} | "
                  f"{ph['N']:.2f} | {ph['G']:.2f} | {npair:.3e} | {nfar:.3e} | {nb:.1f} |", flush=True)
            print(json.dumps(row), flush=True)
    else:
        print(f"\n| theta | P<1e-4 | P<1e-3 | P<2e-3 | P<1e-2 | mean | p99 | max | G ms |\n"
              f"|---:|---:|---:|---:|---:|---:|---:|---:|---:|", flush=True)
        for th in [float(v) for v in a.theta_list.split(",")]:
            ph = timed(a.n_ll, th, a.precision)
            t, _, acc = run(a.n_ll, th, a.precision)
            e = errors(acc, ref)
            t.destroy()
            print(f"| {th} | {e['P<1e-4']:.4f} | {e['P<1e-3']:.4f} | {e['P<2e-3']:.4f} | {e['P<1e-2']:.4f} | "
                  f"{e['mean']:.2e} | {e['p99']:.2e} | {e['max']:.2e} | {ph['G']:.2f} |", flush=True)
            print(json.dumps({"theta": th, "n_ll": a.n_ll, **ph, **e}), flush=True)


def splits(a, np, torch, W, Tree, dev):
    """Error against the direct sum (FP64 tree at theta = 0) and build time
    for each split rule, FP64 form, theta = 0.7."""
    print(f"| workload | split | build ms | mean eps | p99 | max | P<1e-2 |\n"
          f"|---|---|---:|---:|---:|---:|---:|", flush=True)
    for name, cloud, n_ll in (("sobol_sphere 500k", W.sobol_sphere(a.n, a.neighbours), 12),
                              ("binary 3000 + 1000", W.binary_clumps(), 8)):
        arrs = [torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in cloud.arrays()]
        rt = Tree(*arrs, n_ll=n_ll, theta=0.0, precision="fp64")
        ref = torch.stack(rt.gravity(), 1)
        rt.destroy()
        na = ref.norm(dim=1)
        for split in ("mass", "number", "median"):
            Tree(*arrs, n_ll=n_ll, theta=0.7, split=split).destroy()          # warm-up
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            t = Tree(*arrs, n_ll=n_ll, theta=0.7, split=split)
            e1.record()
            acc = torch.stack(t.gravity(), 1)
            torch.cuda.synchronize()
            eps = ((acc - ref).norm(dim=1) / na).cpu().numpy()
            row = {"workload": name, "split": split, "build_ms": e0.elapsed_time(e1),
                   "mean": float(eps.mean()), "p99": float(np.quantile(eps, 0.99)),
                   "max": float(eps.max()), "P<1e-2": float((eps < 1e-2).mean())}
            t.destroy()
            print(f"| {name} | {split} | {row['build_ms']:.2f} | {row['mean']:.2e} | {row['p99']:.2e} | "
                  f"{row['max']:.2e} | {row['P<1e-2']:.4f} |", flush=True)
            print(json.dumps(row), flush=True)


def _direct(torch, P, m, h, sel, chunk=1 << 17):
    """Direct kernel-smoothed sum (Sec. 2.4.3: a -= m_b S(q)/r (r_a - r_b),
    h_ab = (h_a + h_b)/2, q = r/h_ab) for the sinks `sel`, FP64, by chunks of
    sources."""
    out = torch.zeros(len(sel), 3, dtype=torch.float64, device=P.device)
    pa, ha = P[sel], h[sel]
    for s0 in range(0, P.shape[0], chunk):
        pb, mb, hb = P[s0:s0 + chunk], m[s0:s0 + chunk], h[s0:s0 + chunk]
        v = pa[:, None, :] - pb[None, :, :]
        r2 = (v * v).sum(2)
        r = r2.sqrt()
        hab = 0.5 * (ha[:, None] + hb[None, :])
        q = r / hab
        inner = (4.0 / 3.0 - 1.2 * q * q + 0.5 * q ** 3) / hab ** 3
        outer = (8.0 / 3.0 - 3.0 * q + 1.2 * q * q - q ** 3 / 6.0) / hab ** 3 - 1.0 / (15.0 * r2 * r)
        newton = 1.0 / (r2 * r)
        F = torch.where(q < 1.0, inner, torch.where(q < 2.0, outer, newton))
        F = torch.where(r2 > 0.0, F, torch.zeros_like(F))
        out -= ((mb[None, :] * F)[:, :, None] * v).sum(1)
    return out


def scaling(a, np, torch, W, Tree, dev):
    print(f"| N | L | form | ms/step | build | walk | neighbours | gravity | particles/s | "
          f"nb check | mean eps | max eps | B/particle |\n|---:|---:|---|---:|---:|---:|---:|---:|---:|---|---:|---:|---:|",
          flush=True)
    rng = np.random.default_rng(7)
    for n in [int(v) for v in a.sizes.split(",")]:
        t0 = time.perf_counter()
        cloud = W.clumpy_cube(n)
        print(f"[progress] generated N={n} in {time.perf_counter() - t0:.0f} s", flush=True)
        arrs = [torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in cloud.arrays()]
        del cloud
        P = torch.stack(arrs[:3], 1)
        sel = torch.from_numpy(np.sort(rng.choice(n, a.samples, replace=False))).to(dev)
        ref = _direct(torch, P, arrs[3], arrs[4], sel)
        torch.cuda.synchronize()
        print(f"[progress] direct sum of {a.samples} sinks done", flush=True)
        for prec in ("mixed", "fp64"):
            def step(ev=None):
                rec = (lambda i: ev[i].record()) if ev is not None else (lambda i: None)
                rec(0)
                t = Tree(*arrs, n_ll=12, theta=0.7, precision=prec)
                rec(1)
                t.walk()
                rec(2)
                off, ids = t.neighbours()
                rec(3)
                acc = t.gravity()
                rec(4)
                return t, off, ids, acc
            from paper_1108_0028_amd import release_cache
            torch.cuda.synchronize()
            release_cache()
            torch.cuda.empty_cache()
            free0 = torch.cuda.mem_get_info()[0]
            t, off, ids, acc = step()            # warm-up; its outputs are checked
            torch.cuda.synchronize()
            mem = (free0 - torch.cuda.mem_get_info()[0]) / n   # device bytes per particle of a live step
            k = t.info()["k"]
            # neighbours of 32 sampled particles against an all-pairs search
            ok = True
            for i in sel[:32].tolist():
                dx, dy, dz = P[:, 0] - P[i, 0], P[:, 1] - P[i, 1], P[:, 2] - P[i, 2]
                d2 = (dx * dx + dy * dy) + dz * dz          # the kernels' order, no fused multiply-add
                lim = (2.0 * arrs[4][i]) ** 2
                exact = torch.nonzero((d2 < lim) & (torch.arange(n, device=dev) != i)).flatten()
                got = ids[off[i]:off[i + 1]].long()
                ok &= bool(torch.equal(got, exact))   # lists ascending by index
            am = torch.stack([v.double() for v in acc], 1)[sel]
            eps = ((am - ref).norm(dim=1) / ref.norm(dim=1)).cpu().numpy()
            t.destroy()
            del off, ids, acc
            rows = []
            for _ in range(3):
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
                torch.cuda.synchronize()
                w0 = time.perf_counter()
                t, _, _, _ = step(ev)
                torch.cuda.synchronize()
                rows.append([time.perf_counter() - w0] + [ev[j].elapsed_time(ev[j + 1]) for j in range(4)])
                t.destroy()
            med = np.median(np.array(rows), 0)
            row = {"n": n, "L": k, "form": prec, "ms_per_step": med[0] * 1e3, "build": med[1], "walk": med[2],
                   "neighbours": med[3], "gravity": med[4], "particles_per_s": n / med[0],
                   "neighbours_match": ok, "mean_eps": float(eps.mean()), "max_eps": float(eps.max()),
                   "bytes_per_particle": mem}
            print(f"| {n} | {k} | {prec} | {row['ms_per_step']:.1f} | {med[1]:.1f} | {med[2]:.1f} | {med[3]:.1f} | "
                  f"{med[4]:.1f} | {row['particles_per_s']:.3g} | {'identical' if ok else 'DIFFER'} | "
                  f"{row['mean_eps']:.2e} | {row['max_eps']:.2e} | {mem:.0f} |", flush=True)
            print(json.dumps(row), flush=True)
        del arrs, P, ref
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
