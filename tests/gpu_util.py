"""Shared helpers for the GPU parity tests (no method arithmetic here)."""
import sys

import numpy as np
import torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def report(workload, dtype, quantity, value, tol=None):
    """Prints one measured error against the FP64 oracle as a JSON line
    (the table of errors per result is collected from these lines)."""
    import json
    say("ERROR-REPORT " + json.dumps({"workload": workload, "dtype": dtype,
                                      "quantity": quantity, "value": float(value),
                                      "tolerance": tol}))


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def dev(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype).cuda().contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)
