"""FP64 oracle: truncated PCG inner solve and the LM outer loop (alg:lm_inexact).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Vectors of R^(2n) are flat complex arrays (object entries, then probe entries
for joint problems); a diagonal of R^(2n) is a real array of shape (n, 2)
holding the (Re, Im) weights of each complex entry.

Readings of points the paper leaves open (each used identically by the GPU
library):
* rejection (rho <= rho_min): mu <- kappa mu, z unchanged, the linearisation
  (G, J, grad ell, D) of the outer iteration is reused and the inner solve is
  repeated with the new lambda, at most ``retry_max`` times;
* rho is reset to 0 at the start of every outer iteration;
* eta = min(beta, sqrt(||J^T grad ell||)) (the printed J grad ell is ill-typed);
* predicted reduction = 1/2 Delta^T (lambda D Delta - g) (the printed formula
  has an unbalanced bracket);
* a non-positive predicted reduction or a non-finite ratio counts as a reject;
* warm start: the inner solve starts from the last accepted step (zero at
  t = 0 and after a reject);
* the inner stopping test uses the unpreconditioned residual norm;
* zero diagonal entries (unilluminated pixels) are floored at
  ``diag_floor`` times the largest entry of their block.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import ptycho


# ----------------------------------------------------------------------------
# vector helpers
# ----------------------------------------------------------------------------
def rdot(u: np.ndarray, v: np.ndarray) -> float:
    """Real inner product <u, v> = Re sum conj(u) v of the real coordinates."""
    return float(np.sum(u.real * v.real + u.imag * v.imag))


def rnorm(u: np.ndarray) -> float:
    return math.sqrt(rdot(u, u))


def apply_diag(d: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Multiply a real-coordinate diagonal (n, 2) into a complex vector (n,)."""
    return d[:, 0] * v.real + 1j * d[:, 1] * v.imag


def pack(O_part, P_part=None) -> np.ndarray:
    if P_part is None:
        return O_part.ravel().copy()
    return np.concatenate([O_part.ravel(), P_part.ravel()])


def unpack(v: np.ndarray, obj_shape, probe_shape, joint: bool):
    N = obj_shape[0] * obj_shape[1]
    O_part = v[:N].reshape(obj_shape)
    P_part = v[N:].reshape(probe_shape) if joint else None
    return O_part, P_part


def pack_diag(dO, dP=None) -> np.ndarray:
    if dP is None:
        return dO.reshape(-1, 2).copy()
    return np.concatenate([dO.reshape(-1, 2), dP.reshape(-1, 2)], axis=0)


def floor_block(d: np.ndarray, frac: float) -> np.ndarray:
    """Raise entries below frac * max(d) to that value (unilluminated pixels)."""
    return np.maximum(d, frac * float(d.max()))


# ----------------------------------------------------------------------------
# truncated PCG (eq:lma_termination_magnitude)
# ----------------------------------------------------------------------------
@dataclass
class PCGResult:
    x: np.ndarray
    r: np.ndarray
    iters: int
    res_norms: list


def pcg(apply_A, g: np.ndarray, x0: np.ndarray, precond_inv, eta: float, cg_max: int) -> PCGResult:
    """Solve A x = -g by preconditioned CG until ||A x + g|| <= eta ||g||.

    ``precond_inv`` maps a residual r to z = M^{-1} r (None: identity).  The
    iteration is the textbook PCG recurrence; all inner products are real and
    in FP64.  Stops after ``cg_max`` products with A, or on a non-positive
    curvature p^T A p (impossible for the SPD systems here, kept as a guard).
    """
    pc = precond_inv if precond_inv is not None else (lambda r: r.copy())
    x = x0.copy()
    r = -g - apply_A(x) if np.any(x0) else -g.copy()
    z = pc(r)
    p = z.copy()
    rz = rdot(r, z)
    gn = rnorm(g)
    norms = [rnorm(r)]
    it = 0
    while it < cg_max:
        if norms[-1] <= eta * gn:
            break
        Ap = apply_A(p)
        pAp = rdot(p, Ap)
        if not pAp > 0.0:
            break
        alpha = rz / pAp
        x = x + alpha * p
        r = r - alpha * Ap
        z = pc(r)
        rz_new = rdot(r, z)
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
        it += 1
        norms.append(rnorm(r))
    return PCGResult(x=x, r=r, iters=it, res_norms=norms)


# ----------------------------------------------------------------------------
# LM step control (alg:lm_inexact)
# ----------------------------------------------------------------------------
@dataclass
class LMParams:
    mu0: float = 1e-5        # Sec. 5 hyperparameters
    mu_min: float = 1e-8
    kappa: float = 4.0
    nu: float = 1.0
    rho_min: float = 1e-4
    beta: float = 0.1        # 0.1 Gaussian, 0.9 Poisson (Sec. 4.2)
    cg_max: int = 10
    retry_max: int = 10
    scaling: int = 0         # 0: D = I, 1: D = Dg(G) (App. B diagonal)
    precond: int = 0         # 0: none, 1: Jacobi Dg(G + lambda D), 2: learned + lambda D,
                             # 3: exact diagonal of G + lambda D, 4: stochastic estimate + lambda D
    diag_floor: float = 1e-6
    warm_start: bool = True
    surrogate_T: int = 0     # App. E surrogate Poisson metric: iterations with sigma_t > 0 (0: off)
    surrogate_s0: float = 1.0
    project: bool = False    # alg:projected_LM plug-in (constrained BPR), constants of Sec. 5
    o_max: float = 1.0       # eq:constraints: |O| <= 1
    p_max: float = 1e8       #                 |P| <= 1e8
    sigma_ls: float = 1e-4   # eq:armijo_criterion
    gamma: float = 1e-6
    tau_s: float = 1e-8
    p_s: float = 2.1
    ls_max: int = 30         # backtracking halvings before the iterate is kept
    alternate: bool = False  # alg:alt_LM_ptycho: object sub-step, then probe sub-step (joint only)
    ggn: str = "magnitude"   # GGN of the LM model: "magnitude" (eq:ggn_magnitude) or "intensity"
                             # (eq:ggn_intensity, the App. C ablation)
    stoch_samples: int = 8   # precond 4: sign-field draws of the stochastic diagonal per linearisation
    stoch_seed: int = 0      # precond 4: SplitMix64 seed; outer iteration t uses draws t S .. t S + S - 1


def surrogate_sigma(t: int, p: "LMParams") -> float:
    """sigma_t of the surrogate metric (App. E, eq:expected_count_surrogate): added to the
    background, decreasing on a logarithmic grid from s0 and then 0.  The paper's grid "from
    s0 to 0" cannot be logarithmic; read as s0 down to 1e-6 s0 over T iterations, then 0."""
    if p.surrogate_T <= 0 or t >= p.surrogate_T:
        return 0.0
    if p.surrogate_T == 1:
        return p.surrogate_s0
    return p.surrogate_s0 * 1e-6 ** (t / (p.surrogate_T - 1))


def project(O, P, p: LMParams):
    """Pi_Z of eq:projection for the separable sets of eq:constraints: the closest point with
    |O| <= o_max and |P| <= p_max is a clamp of each entry's magnitude (phase kept)."""
    def clamp(x, m):
        a = np.abs(x)
        return np.where(a > m, x * (m / np.where(a > 0, a, 1.0)), x)
    return clamp(O, p.o_max), (clamp(P, p.p_max) if P is not None else None)


def projected_update(O, P, step, g, f_t, loss, p: LMParams, joint, block="all"):
    """alg:projected_LM applied to an accepted LM step from the feasible point (O, P).

    Reading of the garbled points: the first branch accepts the projected point
    Pi_Z(z + Delta); otherwise a backtracking (halving) Armijo line search along
    s = Pi_Z(z + Delta) - z when s is a sufficient descent direction (z + alpha s stays in Z
    by convexity), else along -grad f with projection.  Returns (O, P, branch, alpha); when
    no step size passes eq:armijo_criterion the iterate is kept (alpha = 0).  ``step`` and
    ``g`` are full vectors; with ``block`` "O" or "P" (a sub-step of the alternating update)
    they vanish outside that block, and only that block is projected (the other is fixed).
    """
    shapes = (O.shape, P.shape)

    def proj(On, Pn):
        Oc, Pc = project(On, Pn, p)
        return (Oc if block != "P" else On), (Pc if block != "O" else Pn)

    sO, sP = unpack(step, *shapes, joint)
    Oc, Pc = proj(O + sO, (P + sP) if joint else P)
    if loss(Oc, Pc) < p.gamma * f_t:
        return Oc, Pc, "lm", 1.0
    s = pack(Oc - O, (Pc - P) if joint else None)
    if rdot(g, s) <= -p.tau_s * rnorm(s) ** p.p_s:
        d, use_proj, branch = s, False, "direction"
    else:
        d, use_proj, branch = -g, True, "gradient"
    dn2 = rdot(d, d)
    alpha = 1.0
    for _ in range(p.ls_max):
        dO, dP = unpack(alpha * d, *shapes, joint)
        On, Pn = O + dO, (P + dP) if joint else P
        if use_proj:
            On, Pn = proj(On, Pn)
        if loss(On, Pn) <= f_t - p.sigma_ls * alpha * dn2:
            return On, Pn, branch, alpha
        alpha *= 0.5
    return O, P, branch, 0.0


def gain_ratio(dfa: float, dfp: float) -> float:
    """rho = actual / predicted reduction; -inf when undefined (reject)."""
    if not (dfp > 0.0) or not math.isfinite(dfa) or not math.isfinite(dfp):
        return -math.inf
    rho = dfa / dfp
    return rho if math.isfinite(rho) else -math.inf


def mu_update(rho: float, mu: float, p: LMParams):
    """Damping update and acceptance of alg:lm_inexact (thresholds strict).

    Returns (new mu, accepted).
    """
    if rho > 0.75:
        return max(mu / p.kappa, p.mu_min), True
    if rho > 0.25:
        return mu, True
    if rho > p.rho_min:
        return p.kappa * mu, True
    return p.kappa * mu, False


def damping(mu: float, resid_norm: float, scaled: bool, p: LMParams) -> float:
    """lambda = mu ||grad_zeta ell||^nu when D = I, else lambda = mu."""
    return mu if scaled else mu * resid_norm ** p.nu


@dataclass
class Attempt:
    t: int
    f: float
    f_trial: float
    mu: float
    lam: float
    eta: float
    rho: float
    cg_iters: int
    accepted: bool
    ls: tuple = None          # (branch, step size) of the projected plug-in, when used
    block: str = "all"        # variables of the attempt: "all", or "O" / "P" (alternating update)


@dataclass
class LMResult:
    O: np.ndarray
    P: np.ndarray
    f: float
    history: list = field(default_factory=list)
    f_per_iter: list = field(default_factory=list)


def lm_solve(O0, P0, pos, y, b, metric, joint, params: LMParams, T: int,
             learned_diag=None, loss_fn=None, progress=None) -> LMResult:
    """Truncated matrix-free LM, alg:lm_inexact, step by step.

    ``learned_diag`` is a real-coordinate diagonal (n, 2) that replaces Dg(G) in
    the Jacobi preconditioner Dg(G + lambda D) when ``params.precond == 2``; precond 3 uses the
    exact diagonal of G there.  With ``surrogate_T`` > 0 outer iteration t works on the
    surrogate metric of App. E (background b + sigma_t), its trial loss included.  ``loss_fn``
    overrides the trial-loss evaluation (used to force branches in tests).
    ``progress(t, f_t)`` is called at the start of every outer iteration.

    With ``params.alternate`` (joint problems only) an outer iteration is the alternating
    update of alg:alt_LM_ptycho: the inner loop of alg:lm_inexact (its while loop) on the
    object with the probe fixed, then on the probe with the new object fixed.  Each sub-step
    linearises at its own starting point and solves with the object-object (probe-probe)
    block of G, the block's part of g, D and the preconditioner.  Readings: each block keeps
    its own damping mu and its own warm-start step; both sub-steps of outer iteration t use
    the metric of that iteration (surrogate term included); a sub-step whose retries are all
    rejected leaves its block unchanged and the other sub-step still runs.
    """
    p = params
    O = np.array(O0, dtype=np.complex128)
    P = np.array(P0, dtype=np.complex128)
    if p.alternate and not joint:
        raise ValueError("the alternating update needs a joint (object and probe) problem")
    blocks = ("O", "P") if p.alternate else ("all",)
    mu = {k: p.mu0 for k in blocks}
    prev_step = {k: None for k in blocks}
    res = LMResult(O=O, P=P, f=float("nan"))
    for t in range(T):
        # App. E: the surrogate metric of outer iteration t adds sigma_t to the background
        b_t = b + surrogate_sigma(t, p)
        trial_loss = loss_fn or (lambda O_, P_, b_t=b_t: ptycho.loss(O_, P_, pos, y, b_t, metric))
        for k in blocks:
            # line "Calculate G, J, grad ell and D_t" -- once per outer iteration (per sub-step)
            lin = ptycho.linearize(O, P, pos, y, b_t, metric, joint, p.ggn)
            if k == blocks[0]:
                res.f_per_iter.append(lin.f)
                if progress is not None:
                    progress(t, lin.f)
            O, P, mu[k], prev_step[k] = _inner_loop(t, k, lin, O, P, mu[k], prev_step[k], joint, p,
                                                    learned_diag, trial_loss, res.history)

    res.O, res.P = O, P
    res.f = ptycho.loss(O, P, pos, y, b, metric)
    return res


def _inner_loop(t, block, lin, O, P, mu, prev_step, joint, p: LMParams, learned_diag, trial_loss, history):
    """The while loop of alg:lm_inexact at the linearisation ``lin`` of (O, P), over the
    variables of ``block``: "all" (the object, and the probe for joint problems), "O" or "P"
    (the other block fixed, alg:alt_LM_ptycho).  Vectors here hold the block's entries only.
    Returns (O, P, mu, last accepted step of the block or the previous one)."""
    obj_shape, probe_shape = O.shape, P.shape
    N = O.size
    n = N + (P.size if joint else 0)
    sel = {"all": slice(0, n), "O": slice(0, N), "P": slice(N, n)}[block]

    def embed(v):  # block vector -> full vector, zero outside the block
        full = np.zeros(n, dtype=np.complex128)
        full[sel] = v
        return full

    f_t = lin.f
    gO, gP = ptycho.gradient(lin)
    g = pack(gO, gP)[sel]
    gnorm = rnorm(g)
    zres = ptycho.zeta_residual_norm(lin)
    dg = None
    if p.scaling == 1 or p.precond == 1:
        dO, dP = ptycho.ggn_diag_paper(lin)
        blocks = [floor_block(dO.reshape(-1, 2), p.diag_floor)]
        if joint:
            blocks.append(floor_block(dP.reshape(-1, 2), p.diag_floor))
        dg = np.concatenate(blocks, axis=0)[sel]
    scaled = p.scaling == 1
    dx = None
    if p.precond in (3, 4):
        # the exact diagonal of G, or its stochastic estimate, in place of the App. B one, floored alike
        if p.precond == 3:
            eO, eP = ptycho.ggn_diag_exact(lin)
        else:
            S = p.stoch_samples
            r = np.stack([ptycho.rademacher_field(lin, p.stoch_seed, t * S + s) for s in range(S)])
            eO, eP = ptycho.ggn_diag_stochastic(lin, r)
        blocks = [floor_block(eO.reshape(-1, 2), p.diag_floor)]
        if joint:
            blocks.append(floor_block(eP.reshape(-1, 2), p.diag_floor))
        dx = np.concatenate(blocks, axis=0)[sel]
    ld = learned_diag[sel] if learned_diag is not None else None

    def apply_G(v):  # the block of G acting on the block's variables
        vO, vP = unpack(embed(v), obj_shape, probe_shape, joint)
        return pack(*ptycho.ggn_vp(lin, vO, vP))[sel]

    retries = 0
    while True:  # the "while rho < rho_min" loop with its reject branch
        lam = damping(mu, zres, scaled, p)
        if scaled:
            A = lambda v, lam=lam: apply_G(v) + lam * apply_diag(dg, v)
        else:
            A = lambda v, lam=lam: apply_G(v) + lam * v
        if p.precond == 1:
            m = dg * (1.0 + lam) if scaled else dg + lam      # Dg(G + lambda D)
            pc = lambda r, m=m: r.real / m[:, 0] + 1j * r.imag / m[:, 1]
        elif p.precond in (2, 3, 4):
            # learned, exact or estimated diagonal in place of Dg(G) inside Dg(G + lambda D)
            m = (ld if p.precond == 2 else dx) + lam * (dg if scaled else 1.0)
            pc = lambda r, m=m: r.real / m[:, 0] + 1j * r.imag / m[:, 1]
        else:
            pc = None
        eta = min(p.beta, math.sqrt(gnorm))
        x0 = prev_step if (p.warm_start and retries == 0 and prev_step is not None) \
            else np.zeros_like(g)
        sol = pcg(A, g, x0, pc, eta, p.cg_max)
        step = sol.x
        sO, sP = unpack(embed(step), obj_shape, probe_shape, joint)
        O_t = O + sO
        P_t = P + sP if joint else P
        f_trial = trial_loss(O_t, P_t)
        dfa = f_t - f_trial
        Dstep = lam * (apply_diag(dg, step) if scaled else step)
        dfp = 0.5 * rdot(step, Dstep - g)
        rho = gain_ratio(dfa, dfp)
        mu_new, accepted = mu_update(rho, mu, p)
        history.append(Attempt(t, f_t, f_trial, mu, lam, eta, rho, sol.iters, accepted, block=block))
        mu = mu_new
        if accepted:
            if p.project:
                O, P, branch, alpha = projected_update(O, P, embed(step), embed(g), f_t, trial_loss, p,
                                                       joint, block)
                history[-1].ls = (branch, alpha)
            else:
                O, P = O_t, P_t
            return O, P, mu, step
        retries += 1
        if retries >= p.retry_max:
            return O, P, mu, prev_step
