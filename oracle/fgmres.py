"""Right-preconditioned flexible GMRES(m) in the Euclidean inner product.

Test infrastructure only (see the package docstring).

The paper solves the preconditioned system (eq. 2.24) with GMRES and analyses it with the Elman
theory (Sec. 1; Theorem 3.1).  This is Saad's flexible variant (it stores the preconditioned
directions z_j, so the preconditioner may change between applications, which the mixed-precision
path needs): modified Gram-Schmidt Arnoldi, Givens rotations for the Hessenberg least-squares
problem, restart after m inner steps, x_0 = 0.  Stopping: the recurrence residual |g_{j+1}| <=
tol ||f||, then the true residual ||f - B x|| <= tol ||f|| is checked explicitly and the method
restarts if it is not met.  The iteration count is the number of preconditioner applications.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def fgmres(matvec, precond, f, restart=50, tol=1e-8, max_iter=1000, breakdown_tol=1e-14):
    n = f.shape[0]
    x = np.zeros(n)
    fnorm = float(np.linalg.norm(f))
    info = {"iters": 0, "converged": False, "relres_est": 0.0, "relres_true": 0.0,
            "history": [], "cycles": 0}
    if fnorm == 0.0:
        info["converged"] = True
        return x, info
    r = f.copy()
    iters = 0
    while True:
        beta = float(np.linalg.norm(r))
        if beta <= tol * fnorm:
            info["converged"] = True
            break
        if iters >= max_iter:
            break
        info["cycles"] += 1
        V = np.zeros((n, restart + 1))
        Zk = np.zeros((n, restart))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[:, 0] = r / beta
        jd = 0
        for j in range(restart):
            Zk[:, j] = precond(V[:, j])
            w = matvec(Zk[:, j])
            w0 = float(np.linalg.norm(w))
            for i in range(j + 1):                      # modified Gram-Schmidt
                H[i, j] = float(V[:, i] @ w)
                w = w - H[i, j] * V[:, i]
            hn = float(np.linalg.norm(w))
            H[j + 1, j] = hn
            iters += 1
            for i in range(j):                          # previous rotations on column j
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            d = float(np.hypot(H[j, j], H[j + 1, j]))
            if d == 0.0:
                raise FloatingPointError("singular Hessenberg column")
            cs[j] = H[j, j] / d
            sn[j] = H[j + 1, j] / d
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            info["history"].append(abs(g[j + 1]) / fnorm)
            jd = j + 1
            if abs(g[j + 1]) <= tol * fnorm or hn <= breakdown_tol * w0 or iters >= max_iter:
                break
            V[:, j + 1] = w / hn
        y = sla.solve_triangular(H[:jd, :jd], g[:jd], lower=False)
        x = x + Zk[:, :jd] @ y
        info["relres_est"] = abs(g[jd]) / fnorm
        r = f - matvec(x)
    info["iters"] = iters
    info["relres_true"] = float(np.linalg.norm(f - matvec(x))) / fnorm
    info["converged"] = info["relres_true"] <= tol
    return x, info


def solve(problem, precond_obj, f=None, restart=50, tol=1e-8, max_iter=1000):
    """FGMRES on B u = f with the given preconditioner object (``.B`` and ``.apply``)."""
    B = precond_obj.B
    f = problem.f[0] if f is None else f
    return fgmres(lambda v: B @ v, precond_obj.apply, f, restart=restart, tol=tol, max_iter=max_iter)


def gmres_left_dk(matvec, precond, dk_matvec, f, restart=50, tol=1e-8, max_iter=1000, breakdown_tol=1e-14):
    """GMRES(m) on the left-preconditioned system M^{-1} B u = M^{-1} f (eq. 2.24) in the inner product
    <x, y>_{D_k} = y^T D_k x (Prop 2.11, D_k = A + k^2 S): the setting of Theorem 3.1.

    Arnoldi with modified Gram-Schmidt in the D_k inner product (v_1 = r_0 / ||r_0||_{D_k} with
    r_0 = M^{-1}(f - B x_0), w = M^{-1} B v_j, h_ij = <w, v_i>_{D_k}), Givens rotations on the Hessenberg
    matrix, so that the iterate x_0 + V_m y minimises ||M^{-1}(f - B x)||_{D_k} over the Krylov space.
    Stopping: the recurrence residual |g_{j+1}| <= tol ||M^{-1} f||_{D_k}, then the preconditioned
    residual ||M^{-1}(f - B x)||_{D_k} is recomputed at the cycle end and the method restarts if it is
    above the bar; x_0 = 0.  info: iterations (preconditioner applications), the preconditioned
    D_k-norm residuals (recurrence per step, and the recomputed one) and the Euclidean true residual
    ||f - B x|| / ||f||.
    """
    n = f.shape[0]
    x = np.zeros(n)

    def dnorm(v):
        return float(np.sqrt(max(float(v @ dk_matvec(v)), 0.0)))

    info = {"iters": 0, "converged": False, "relres_est": 0.0, "relres_prec": 0.0, "relres_true": 0.0,
            "history": [], "cycles": 0}
    fnorm = float(np.linalg.norm(f))
    if fnorm == 0.0:
        info["converged"] = True
        return x, info
    ref = dnorm(precond(f))
    iters = 0
    while True:
        r = precond(f - matvec(x))
        beta = dnorm(r)
        info["relres_prec"] = beta / ref
        if beta <= tol * ref:
            info["converged"] = True
            break
        if iters >= max_iter:
            break
        info["cycles"] += 1
        V = np.zeros((n, restart + 1))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[:, 0] = r / beta
        jd = 0
        for j in range(restart):
            w = precond(matvec(V[:, j]))
            w0 = dnorm(w)
            for i in range(j + 1):                      # modified Gram-Schmidt in <.,.>_{D_k}
                H[i, j] = float(V[:, i] @ dk_matvec(w))
                w = w - H[i, j] * V[:, i]
            hn = dnorm(w)
            H[j + 1, j] = hn
            iters += 1
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            d = float(np.hypot(H[j, j], H[j + 1, j]))
            if d == 0.0:
                raise FloatingPointError("singular Hessenberg column")
            cs[j] = H[j, j] / d
            sn[j] = H[j + 1, j] / d
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            info["history"].append(abs(g[j + 1]) / ref)
            jd = j + 1
            if abs(g[j + 1]) <= tol * ref or hn <= breakdown_tol * w0 or iters >= max_iter:
                break
            V[:, j + 1] = w / hn
        y = sla.solve_triangular(H[:jd, :jd], g[:jd], lower=False)
        x = x + V[:, :jd] @ y
        info["relres_est"] = abs(g[jd]) / ref
    info["iters"] = iters
    info["relres_true"] = float(np.linalg.norm(f - matvec(x))) / fnorm
    return x, info


def solve_left_dk(problem, precond_obj, f=None, restart=50, tol=1e-8, max_iter=1000):
    """gmres_left_dk on B u = f with the preconditioner object (``.B``, ``.apply``) and D_k = A + k^2 S."""
    B = precond_obj.B
    Dk = (problem.A + (problem.k ** 2) * problem.S).tocsr()
    f = problem.f[0] if f is None else f
    return gmres_left_dk(lambda v: B @ v, precond_obj.apply, lambda v: Dk @ v, f, restart=restart, tol=tol,
                         max_iter=max_iter)
