"""Shared helpers of the GPU tests (they call the library through the C-ABI)."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


def say(msg):
    """Name the case before each GPU step (flushed), so a fault is attributable."""
    sys.stdout.write(f"[gpu-case] {msg}\n")
    sys.stdout.flush()


def golden(i):
    """Golden trajectory of workload i (an int) or of a named one ("metal")."""
    tag = i if isinstance(i, str) else f"config{i}"
    path = os.path.join(GOLDEN, f"dbs_{tag}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
