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


def chan_max_err(gpu: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Per-channel element-wise error max_{t,bl} |gpu - ref| / rms_{t,bl}(ref); arrays
    [t][nu][bl].  A localised error that a normwise measure would average away
    shows up here; rms in the denominator keeps it defined where |ref| ~ 0."""
    num = np.max(np.abs(gpu - ref), axis=(0, 2))
    den = np.sqrt(np.mean(np.abs(ref) ** 2, axis=(0, 2)))
    return num / den


def max_rel(a, b) -> float:
    """max |a - b| / rms(b) over all elements."""
    d = np.abs(np.ravel(a) - np.ravel(b))
    return float(np.max(d) / np.sqrt(np.mean(np.abs(np.ravel(b)) ** 2)))


# element-wise bars (max |error| / rms): ten times the normwise ones
VIS_ELEM_FP32, VIS_ELEM_SPLIT = 1e-4, 1e-3
GRAD_ELEM_FP32, GRAD_ELEM_SPLIT = 2e-3, 2e-2
