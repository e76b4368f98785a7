"""Pins of the two LM scalars of alg:lm_inexact that no other oracle pin reaches.

* The damping rule lambda = mu ||grad_zeta ell||^nu (D = I): the norm is the 2-norm of the
  derivative of f with respect to the K x M magnitudes zeta, built here by central finite
  differences of the per-measurement metric alone, and lambda is read back from an LM attempt.
* The forcing term of the inner stop, eq:lma_termination_eta (read as eta = min(beta, sqrt(||g||)),
  the gradient norm in parameter space): the iteration at which the oracle's PCG stops is compared
  with the residual history of a textbook CG on the dense system (G + lambda I) x = -g, with g from
  finite differences of f and G = J^T J from a finite-difference Jacobian.  The two cases put
  sqrt(||g||) below and above beta, and each asserts that the plausible misreadings (||g|| in
  place of its root, max in place of min, beta alone) stop at other iterations, so a slip in the
  forcing term changes the count.
"""
import math

import numpy as np
import pytest

import synth
from oracle import ptycho, solver

from test_oracle_pins import _fd_jacobian, tiny_problem


def _fd_zeta_gradient(zeta, y, metric, h=1e-6):
    """d f / d zeta_j for every measurement j, by central differences of ell alone."""
    return (ptycho.ell(zeta + h, y, metric) - ptycho.ell(zeta - h, y, metric)) / (2.0 * h)


@pytest.mark.parametrize("metric", ["gauss", "poisson"])
def test_zeta_residual_norm_is_norm_of_fd_zeta_gradient(metric):
    O, P, pos, y = tiny_problem(seed=11, obj=(8, 9), probe=(4, 3), joint=True, metric=metric)
    b = 1e-3
    lin = ptycho.linearize(O, P, pos, y, b, metric, True)
    fd = _fd_zeta_gradient(lin.zeta, y, metric)
    ref = float(np.linalg.norm(fd.ravel()))
    assert ptycho.zeta_residual_norm(lin) == pytest.approx(ref, rel=1e-8)
    # the norm is not that of the parameter-space gradient, nor its square
    g = np.linalg.norm(solver.pack(*ptycho.gradient(lin)))
    assert abs(g - ref) > 1e-3 * ref and abs(ref ** 2 - ref) > 1e-3 * ref


@pytest.mark.parametrize("nu", [1.0, 2.0])
@pytest.mark.parametrize("metric", ["gauss", "poisson"])
def test_lambda_rule_uses_fd_zeta_gradient_norm(metric, nu):
    O, P, pos, y = tiny_problem(seed=13, obj=(8, 8), probe=(4, 4), joint=False, metric=metric)
    b = 1e-3
    rng = np.random.default_rng(13)
    O0 = O + 0.1 * synth.random_complex(rng, O.shape)
    p = solver.LMParams(nu=nu, scaling=0, precond=0, beta=0.1 if metric == "gauss" else 0.9)
    res = solver.lm_solve(O0, P, pos, y, b, metric, False, p, 1)
    zeta = ptycho.magnitude(O0, P, pos, b)
    norm = float(np.linalg.norm(_fd_zeta_gradient(zeta, y, metric).ravel()))
    assert res.history[0].lam == pytest.approx(p.mu0 * norm ** nu, rel=1e-7)
    # with D = Dg(G) the rule is lambda = mu (no norm)
    p1 = solver.LMParams(nu=nu, scaling=1, precond=1, beta=p.beta)
    res1 = solver.lm_solve(O0, P, pos, y, b, metric, False, p1, 1)
    assert res1.history[0].lam == p1.mu0


def _dense_cg_history(A, g, iters):
    """Unpreconditioned residual norms ||r_i|| of textbook CG on A x = -g from x = 0."""
    x = np.zeros_like(g)
    r = -g.copy()
    p = r.copy()
    rr = float(r @ r)
    norms = [math.sqrt(rr)]
    for _ in range(iters):
        Ap = A @ p
        a = rr / float(p @ Ap)
        x += a * p
        r -= a * Ap
        rn = float(r @ r)
        p = r + (rn / rr) * p
        rr = rn
        norms.append(math.sqrt(rr))
    return norms


def _stop_iteration(norms, eta, gnorm):
    """First i with ||r_i|| <= eta ||g||, the products CG has taken by then; None if none."""
    for i, nr in enumerate(norms):
        if nr <= eta * gnorm:
            return i
    return None


@pytest.mark.parametrize("eps,beta,root_below_beta", [(1e-4, 0.1, True), (1.0, 0.1, False)])
def test_forcing_term_stop_iteration_matches_dense_cg(eps, beta, root_below_beta):
    # noise-free Gaussian data, start eps away from the truth: ||g|| scales with eps
    O, P, pos, _ = tiny_problem(seed=5, obj=(8, 8), probe=(4, 4), joint=False, noisy=False)
    b = 1e-3
    y = ptycho.intensity(O, P, pos, b)
    rng = np.random.default_rng(5)
    O0 = O + eps * synth.random_complex(rng, O.shape)
    cg_max = 60
    p = solver.LMParams(beta=beta, cg_max=cg_max, scaling=0, precond=0)
    att = solver.lm_solve(O0, P, pos, y, b, "gauss", False, p, 1).history[0]

    # g by central differences of f; G = J^T diag(ell'') J with ell'' = 1 (Gaussian) and J by
    # central differences of the magnitudes; lambda = mu0 ||d f / d zeta|| (pinned above)
    n = O.size
    f = lambda O_: ptycho.loss(O_, P, pos, y, b, "gauss")
    h = 1e-6
    g = np.empty(2 * n)
    for i in range(2 * n):
        d = np.zeros(n, complex)
        d[i % n] = h if i < n else 1j * h
        d = d.reshape(O.shape)
        g[i] = (f(O0 + d) - f(O0 - d)) / (2 * h)
    gnorm = float(np.linalg.norm(g))
    assert (math.sqrt(gnorm) < beta) == root_below_beta
    J = _fd_jacobian(O0, P, pos, b, False)
    zeta = ptycho.magnitude(O0, P, pos, b)
    lam = p.mu0 * float(np.linalg.norm(_fd_zeta_gradient(zeta, y, "gauss").ravel()))
    A = J.T @ J + lam * np.eye(2 * n)
    norms = _dense_cg_history(A, g, cg_max)

    eta = min(beta, math.sqrt(gnorm))
    want = _stop_iteration(norms, eta, gnorm)
    assert want is not None and 0 < want < cg_max
    # the stop is decided with room to spare against the finite-difference error
    assert norms[want] < 0.95 * eta * gnorm and norms[want - 1] > 1.05 * eta * gnorm
    assert att.eta == pytest.approx(eta, rel=1e-6)
    assert att.cg_iters == want
    # the misreadings of the forcing term stop elsewhere on this problem
    slips = {"min(beta, ||g||)": min(beta, gnorm), "max(beta, sqrt||g||)": max(beta, math.sqrt(gnorm))}
    slips["beta" if root_below_beta else "sqrt||g||"] = beta if root_below_beta else math.sqrt(gnorm)
    distinct = [name for name, e in slips.items() if _stop_iteration(norms, e, gnorm) != want]
    assert len(distinct) >= (2 if root_below_beta else 1), distinct
