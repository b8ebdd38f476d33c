"""Helpers shared by the GPU tests (no method arithmetic here)."""

import sys

import numpy as np


def announce(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def sigma_gate(s_gpu, s_ref, rel=1e-10, floor=1e-13):
    """FP64 gate: |ds_j| <= rel * s_j + floor * s_1. Returns (ok, worst ratio)."""
    s_gpu = np.asarray(s_gpu)
    s_ref = np.asarray(s_ref)
    bound = rel * s_ref + floor * s_ref[0]
    ratio = np.abs(s_gpu - s_ref) / bound
    return bool(np.all(ratio <= 1.0)), float(ratio.max())


def match_columns_up_to_sign(X, Xref, tol):
    """max_j || X_j - sign_j Xref_j ||_inf with sign_j chosen per column."""
    worst = 0.0
    for j in range(Xref.shape[1]):
        d1 = np.abs(X[:, j] - Xref[:, j]).max()
        d2 = np.abs(X[:, j] + Xref[:, j]).max()
        worst = max(worst, min(d1, d2))
    return worst <= tol, worst


def bf16_round(x):
    """Round to BF16 as the planes do: FP64 -> FP32 (nearest even), then the
    upper 16 bits of the FP32 word, nearest even on the dropped half."""
    f = np.ascontiguousarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
