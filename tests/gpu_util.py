"""Helpers shared by the GPU parity tests (no GPU work at import)."""
import numpy as np

import oracle
from oracle import tt_ref


def dense_of_cores(cores):
    """Oracle densification of a TT list (per component tt_full)."""
    return np.stack([tt_ref.tt_full(comp) for comp in cores])


def oracle_problem(flow):
    bcs = tuple(oracle.BC_PERIODIC if b == 0 else oracle.BC_TRANSMISSIVE for b in flow.bc)
    return oracle.Problem(flow.n, flow.lo, flow.hi, bcs, gamma=flow.gamma)


def rel_err(a, b):
    """max_c ||a_c - b_c||_F / max_c ||b_c||_F"""
    num = max(np.linalg.norm(a[c] - b[c]) for c in range(a.shape[0]))
    den = max(np.linalg.norm(b[c]) for c in range(b.shape[0]))
    return num / den
