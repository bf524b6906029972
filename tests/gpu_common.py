"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
import numpy as np


def rel_fro(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def announce(*parts):
    print("[case]", *parts, flush=True)


def to_np(t):
    return t.detach().cpu().numpy()
