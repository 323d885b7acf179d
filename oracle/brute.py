"""Brute-force O(N^2) referees for the oracle (NumPy / PyTorch CPU, FP64).

TEST INFRASTRUCTURE ONLY. These are the plain definitions the tree method
approximates: the all-pairs neighbour sets within the kernel support and the
direct kernel-softened sum of Sec. 2.4.3 (Eq. for f_ng with S(q)), which the
paper's accuracy test compares against. They are written from S(q) and the unit
vector e_ab (not from the division-safe F = S/r form the oracle uses), so that
the two formulations check each other.
"""
from __future__ import annotations

import math

import numpy as np


def cubic_spline_W(r, h):
    """Monaghan & Lattanzio (1985) cubic spline in 3-D, support 2h, sigma = 1/pi."""
    q = np.asarray(r) / h
    w = np.where(q < 1.0, 1.0 - 1.5 * q ** 2 + 0.75 * q ** 3,
                 np.where(q < 2.0, 0.25 * (2.0 - q) ** 3, 0.0))
    return w / (math.pi * h ** 3)


def S_of_q(r, h):
    """S of Sec. 2.4.3 (the softened 1/r^2), as printed: piecewise in q = r/h."""
    r = np.asarray(r, dtype=np.float64)
    q = r / h
    inner = (4.0 / 3.0 * q - 6.0 / 5.0 * q ** 3 + 0.5 * q ** 4) / h ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        mid = (8.0 / 3.0 * q - 3.0 * q ** 2 + 6.0 / 5.0 * q ** 3 - q ** 4 / 6.0 - 1.0 / (15.0 * q ** 2)) / h ** 2
        outer = 1.0 / r ** 2
    return np.where(q < 1.0, inner, np.where(q < 2.0, mid, outer))


def neighbours(x, y, z, h, block: int = 2048):
    """All-pairs gather neighbours: b != a with |r_a - r_b|^2 < (2 h_a)^2.

    Returns CSR (offsets, ids) with each list ascending by id. The squared
    distance is formed as (dx*dx + dy*dy) + dz*dz in FP64, like the oracle.
    """
    n = x.shape[0]
    counts = np.zeros(n, np.int64)
    chunks = []
    for s in range(0, n, block):
        e = min(n, s + block)
        dx = x[s:e, None] - x[None, :]
        dy = y[s:e, None] - y[None, :]
        dz = z[s:e, None] - z[None, :]
        d2 = (dx * dx + dy * dy) + dz * dz
        lim = (2.0 * h[s:e]) * (2.0 * h[s:e])
        hit = d2 < lim[:, None]
        hit[np.arange(e - s), np.arange(s, e)] = False
        rows, cols = np.nonzero(hit)
        counts[s:e] = np.bincount(rows, minlength=e - s)
        chunks.append(cols.astype(np.int32))
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(counts)
    return off, np.concatenate(chunks) if chunks else np.zeros(0, np.int32)


def direct_accel(x, y, z, m, h, sinks=None, block: int = 512):
    """f_ng(r_a) = -sum_{b != a} m_b S(r_ab, h_ab) e_ab, h_ab = (h_a + h_b)/2."""
    n = x.shape[0]
    sinks = np.arange(n) if sinks is None else np.asarray(sinks)
    out = np.zeros((sinks.shape[0], 3))
    for s in range(0, sinks.shape[0], block):
        idx = sinks[s:s + block]
        dx = x[idx, None] - x[None, :]
        dy = y[idx, None] - y[None, :]
        dz = z[idx, None] - z[None, :]
        r = np.sqrt(dx * dx + dy * dy + dz * dz)
        hab = 0.5 * (h[idx, None] + h[None, :])
        Sv = S_of_q(r, hab)
        with np.errstate(divide="ignore", invalid="ignore"):
            w = np.where(r > 0.0, m[None, :] * Sv / r, 0.0)
        out[s:s + block, 0] = -(w * dx).sum(1)
        out[s:s + block, 1] = -(w * dy).sum(1)
        out[s:s + block, 2] = -(w * dz).sum(1)
    return out


def direct_accel_torch_grad(x, y, z, m, h, gx, gy, gz):
    """Gradient of L = sum_a g_a . f_ng(r_a) w.r.t. positions and masses, by
    PyTorch autograd (CPU, FP64) through the brute-force direct sum."""
    import torch

    X = torch.tensor(np.stack([x, y, z], 1), dtype=torch.float64, requires_grad=True)
    Mt = torch.tensor(m, dtype=torch.float64, requires_grad=True)
    Ht = torch.tensor(h, dtype=torch.float64)
    G = torch.tensor(np.stack([gx, gy, gz], 1), dtype=torch.float64)
    n = X.shape[0]
    eye = torch.eye(n, dtype=torch.bool)
    v = X[:, None, :] - X[None, :, :]
    r2 = (v * v).sum(-1)
    r2s = torch.where(eye, torch.ones_like(r2), r2)
    r = torch.sqrt(r2s)
    hab = 0.5 * (Ht[:, None] + Ht[None, :])
    q = r / hab
    inner = (4.0 / 3.0 * q - 6.0 / 5.0 * q ** 3 + 0.5 * q ** 4) / hab ** 2
    mid = (8.0 / 3.0 * q - 3.0 * q ** 2 + 6.0 / 5.0 * q ** 3 - q ** 4 / 6.0 - 1.0 / (15.0 * q ** 2)) / hab ** 2
    outer = 1.0 / r ** 2
    S = torch.where(q < 1.0, inner, torch.where(q < 2.0, mid, outer))
    w = torch.where(eye, torch.zeros_like(S), Mt[None, :] * S / r)
    acc = -(w[:, :, None] * v).sum(1)
    L = (acc * G).sum()
    L.backward()
    gX = X.grad.numpy()
    return gX[:, 0].copy(), gX[:, 1].copy(), gX[:, 2].copy(), Mt.grad.numpy().copy(), float(L.detach())


def error_stats(a_test, a_ref):
    """Relative force errors eps_i = |da_i| / |a_i| (Sec. 3.1) and the
    floor-normalised maximum used as the gate:
        max_i |da_i| / max(|a_i|, 1e-3 * rms|a|)."""
    da = np.linalg.norm(a_test - a_ref, axis=1)
    na = np.linalg.norm(a_ref, axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        eps = np.where(na > 0, da / na, np.where(da > 0, np.inf, 0.0))
    rms = math.sqrt(float(np.mean(na * na))) if na.size else 0.0
    gate = float(np.max(da / np.maximum(na, 1e-3 * rms))) if na.size else 0.0
    return dict(mean=float(np.mean(eps)), p99=float(np.quantile(eps, 0.99)),
                p999=float(np.quantile(eps, 0.999)), max=float(np.max(eps)), gate=gate,
                frac_below_1pct=float(np.mean(eps < 0.01)))
