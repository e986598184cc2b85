"""Preconditioned conjugate gradients (oracle).

Test infrastructure only (see the package header).

Section 2.2, Algorithm 2, from U0 = 0 (so r0 = F and res0 = ||F||), with the
stopping rule of Section 5 (3): ||F - A U_k|| / ||F|| < eps, evaluated on the
recurrence residual. The iteration count is the number of products A p. The
preconditioner is applied only when the loop continues (Algorithm 2 applies it
before its test; the extra application does not change U). beta is
rho_new / rho_old as printed. The true residual is recomputed at exit.

Pins (tests/test_oracle_solver.py, test_pcg_error_bound, test_plain_cg_within_n_iterations,
test_coarsest_is_fine_level_gives_exact_inverse): on tiny systems the solution
error is bounded by kappa(A) * rtol against a dense direct solve; with B = I,
CG reaches rtol in at most n iterations; with B = A^{-1} it converges in one
iteration. The flexible beta r_new^T (z_new - z_old) / rho_old
(tests/test_oracle_precision.py): identical iterates to the printed beta under
a fixed SPD preconditioner, different (and still converging) under one that
varies between applications.
"""
from __future__ import annotations

import numpy as np


def pcg(A, F: np.ndarray, precond, rtol: float = 1e-6, max_iters: int = 10000,
        x0: np.ndarray | None = None, flexible: bool = False):
    """Returns (x, info) with info = dict(iterations, rel_res, rel_res_true, converged,
    history, breakdown)."""
    F = np.asarray(F, dtype=np.float64)
    n = F.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    r = F - A @ x
    normF = float(np.linalg.norm(F))
    info = dict(iterations=0, rel_res=0.0, rel_res_true=0.0, converged=True,
                history=[], breakdown=False)
    if normF == 0.0:
        return np.zeros(n), info
    res = float(np.linalg.norm(r))
    info["history"].append(res / normF)
    if res / normF < rtol:
        info["rel_res"] = res / normF
        info["rel_res_true"] = float(np.linalg.norm(F - A @ x)) / normF
        return x, info
    z = np.asarray(precond(r), dtype=np.float64)
    p = z.copy()
    rho = float(r @ z)
    k = 0
    converged = False
    while k < max_iters:
        q = A @ p
        pq = float(p @ q)
        if not np.isfinite(pq) or pq <= 0.0:
            info["breakdown"] = True
            break
        alpha = rho / pq
        x = x + alpha * p
        r = r - alpha * q
        k += 1
        res = float(np.linalg.norm(r))
        info["history"].append(res / normF)
        if res / normF < rtol:
            converged = True
            break
        z_new = np.asarray(precond(r), dtype=np.float64)
        rho_new = float(r @ z_new)
        if flexible:
            beta = float(r @ (z_new - z)) / rho
        else:
            beta = rho_new / rho
        p = z_new + beta * p
        z = z_new
        rho = rho_new
    info["iterations"] = k
    info["rel_res"] = res / normF
    info["rel_res_true"] = float(np.linalg.norm(F - A @ x)) / normF
    info["converged"] = converged
    return x, info
