"""Helpers shared by the GPU tests: build fields on both sides from one config."""
import math
import sys

import numpy as np

from paper_2504_07090_amd import workload as w


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def chan_rel_err(gpu: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Per-channel normwise relative error ||gpu - ref|| / ||ref|| over (t, bl); arrays [t][nu][bl]."""
    num = np.sqrt(np.sum(np.abs(gpu - ref) ** 2, axis=(0, 2)))
    den = np.sqrt(np.sum(np.abs(ref) ** 2, axis=(0, 2)))
    return num / den


def rel_norm(a, b) -> float:
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def to_dev(torch, x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype).cuda()
