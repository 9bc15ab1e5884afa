"""Helpers shared by the GPU parity tests (no GPU work at import)."""
import numpy as np

import oracle
from oracle import tt_ref


def dense_of_cores(cores):
    """Oracle densification of a TT list (per component tt_full)."""
    return np.stack([tt_ref.tt_full(comp) for comp in cores])


def oracle_problem(flow):
    # the library's wenott_bc values and the oracle's boundary codes are both written out here
    code = {0: oracle.BC_PERIODIC, 1: oracle.BC_TRANSMISSIVE, 2: oracle.BC_SYMMETRY, 3: oracle.BC_INFLOW}
    bcs = tuple((code[b], code[b]) if np.ndim(b) == 0 else (code[b[0]], code[b[1]]) for b in flow.bc)
    model = {0: oracle.EULER, 1: oracle.LINADV, 2: oracle.BURGERS}[getattr(flow, "law", 0)]
    return oracle.Problem(flow.n, flow.lo, flow.hi, bcs, gamma=flow.gamma, model=model,
                          inflow=getattr(flow, "inflow", None))


def rel_err(a, b):
    """max_c ||a_c - b_c||_F / max_c ||b_c||_F"""
    num = max(np.linalg.norm(a[c] - b[c]) for c in range(a.shape[0]))
    den = max(np.linalg.norm(b[c]) for c in range(b.shape[0]))
    return num / den


def eps_formula(flow, u, c_eps):
    """eq. eps-tt-formula in d dimensions, computed here from the densified state u:
    eps = C_eps V^{1/2} h^{5 - d/2} / max_q ||q||_F with V the domain volume, h the geometric mean
    of the cell sizes and ||q||_F over the interior cells (the d = 3 case is the paper's h^{7/2})."""
    d = len(flow.n)
    vol = float(np.prod([b - a for a, b in zip(flow.lo, flow.hi)]))
    h = float(np.prod(flow.h)) ** (1.0 / d)
    qmax = max(np.linalg.norm(u[c]) for c in range(u.shape[0]))
    return c_eps * vol ** 0.5 * h ** (5.0 - 0.5 * d) / qmax


class EpsTracker:
    """The dynamic eps_TT of a run, computed independently of the library: C_eps is fixed so
    that the formula gives eps0 on the initial state (the "dynamic from eps0" reading), or
    given; eps(u) then follows eq. eps-tt-formula on each densified state."""

    def __init__(self, flow, u0, eps0=None, c_eps=None):
        self.flow = flow
        if c_eps is None:
            c_eps = eps0 / eps_formula(flow, u0, 1.0)
        self.c_eps = c_eps

    def __call__(self, u):
        return eps_formula(self.flow, u, self.c_eps)
