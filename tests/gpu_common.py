"""Shared helpers for the GPU parity tests (imported by tests marked `gpu`)."""

import json
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SPECTRA = os.path.join(ROOT, "tests", "golden", "spectra.json")


def load_spectra():
    with open(SPECTRA) as f:
        return json.load(f)


def to_gpu_block(X: np.ndarray, dtype=None):
    """(n, N) column-major numpy block -> torch tensor (N, n) on cuda:0."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(X.T))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def from_gpu_block(T) -> np.ndarray:
    return T.detach().cpu().numpy().T


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def announce(msg: str):
    print("[gpu-test]", msg, flush=True)
