"""Shared helpers of the test suite (test code only)."""
import math

import numpy as np
import torch

G = 9.8


def rel_maxnorm(got, ref, g=G):
    """Relative max-norm over the interior of (h, hu, hv): each field's
    max |difference| divided by a scale of that field: ||h_ref||_inf for h and
    the momentum scale ||h_ref||_inf * sqrt(g ||h_ref||_inf) for hu and hv (a
    plain per-field ratio would divide by near-zero momenta).  Returns the
    largest of the three."""
    gh, gu, gv = (np.asarray(a, dtype=np.float64) for a in got)
    rh, ru, rv = (np.asarray(a, dtype=np.float64) for a in ref)
    sh = np.max(np.abs(rh))
    sm = sh * math.sqrt(g * sh)
    return max(np.max(np.abs(gh - rh)) / sh, np.max(np.abs(gu - ru)) / sm, np.max(np.abs(gv - rv)) / sm)


def gpu_available():
    return torch.cuda.is_available()


def announce(msg: str):
    """Print (and flush) what a GPU step is about to run."""
    print(f"[gpu-case] {msg}", flush=True)
