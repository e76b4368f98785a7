"""GPU LM runs against the FP64 oracle's LM on the same problem.

Bar: final loss f_gpu <= 1.01 f_oracle + f_floor, where f_floor is twice the
FP32 GPU loss at the ground truth (noise-free data drive f to ~0, where an FP32
evaluation cannot reproduce an FP64 ratio).  LM trajectories are not compared
iterate by iterate: FP32 vs FP64 rounding legitimately changes accept/reject
decisions near convergence.
"""
import math

import numpy as np
import pytest

import synth
from oracle import ptycho, solver

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)
import paper_2103_01767_amd as pt  # noqa: E402

DEV = torch.device("cuda:0")


def to_dev(x, dt):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=dt))).to(DEV)


def test_c0_plain_lm_matches_oracle_final_loss():
    print("case c0 lm", flush=True)
    pr = synth.make_c0()
    O0 = pr.O_init.astype(np.complex64)
    P = pr.P_true.astype(np.complex64)
    Ot = pr.O_true.astype(np.complex64)
    y = ptycho.intensity(Ot.astype(np.complex128), P.astype(np.complex128), pr.pos, pr.background)
    y32 = y.astype(np.float32)
    ref = solver.lm_solve(O0.astype(np.complex128), P.astype(np.complex128), pr.pos, y32.astype(np.float64),
                          pr.background, "gauss", False, solver.LMParams(), 20)
    prob = pt.Problem(pr.O_true.shape, P.shape, pr.pos, mode="object", background=pr.background, device=DEV)
    O = to_dev(O0, np.complex64)
    Pd = to_dev(P, np.complex64)
    yd = to_dev(y32, np.float32)
    params = pt.default_params()
    st = prob.new_state()
    prob.lm_init(params, st)
    prob.lm_solve(O, Pd, yd, params, 20, st)
    torch.cuda.synchronize()
    s = pt.state_from_tensor(st)
    f_gpu = float(prob.loss(O, Pd, yd).cpu()[0])
    f_floor = 2.0 * float(prob.loss(to_dev(Ot, np.complex64), Pd, yd).cpu()[0])
    print("c0 oracle f=%.3e gpu f=%.3e floor=%.3e t=%d cg=%d" % (ref.f, f_gpu, f_floor, s.t, s.cg_total))
    assert s.t == 20
    assert f_gpu <= 1.01 * ref.f + f_floor
    assert f_gpu < 1e-4 * ref.f_per_iter[0]
    # the reconstruction matches the truth up to the global phase on illuminated pixels
    Og = O.cpu().numpy().astype(np.complex128)
    ov = ptycho.illumination_overlap(P.astype(np.complex128), pr.pos, pr.O_true.shape)
    m = ov > 0.05 * ov.max()
    c = np.vdot(Og[m], pr.O_true[m])
    err = np.linalg.norm(Og[m] * c / abs(c) - pr.O_true[m]) / np.linalg.norm(pr.O_true[m])
    assert err < 1e-2


def test_joint_scaled_jacobi_lm_matches_oracle():
    print("case joint lm", flush=True)
    pr = synth.make_small(5, obj_side=48, probe=(16, 16), n=6, step=5, photons=1e3, mode="joint")
    rng = np.random.default_rng(5)
    O0 = pr.O_init.astype(np.complex64)
    P0 = pr.P_init.astype(np.complex64)
    h = ptycho.intensity(pr.O_true, pr.P_true, pr.pos, pr.background)
    y = synth.poisson_counts(rng, h).astype(np.float32)
    p_or = solver.LMParams(scaling=1, precond=1)
    ref = solver.lm_solve(O0.astype(np.complex128), P0.astype(np.complex128), pr.pos, y.astype(np.float64),
                          pr.background, "gauss", True, p_or, 10)
    prob = pt.Problem(pr.O_true.shape, pr.P_true.shape, pr.pos, mode="joint", background=pr.background, device=DEV)
    O, P, yd = to_dev(O0, np.complex64), to_dev(P0, np.complex64), to_dev(y, np.float32)
    params = pt.default_params(scaling=1, precond=1)
    st = prob.new_state()
    prob.lm_init(params, st)
    prob.lm_solve(O, P, yd, params, 10, st)
    f_gpu = float(prob.loss(O, P, yd).cpu()[0])
    print("joint oracle f=%.6e gpu f=%.6e (start %.3e)" % (ref.f, f_gpu, ref.f_per_iter[0]))
    assert f_gpu <= 1.01 * ref.f
    assert f_gpu < 0.5 * ref.f_per_iter[0]


def test_first_attempt_matches_oracle_step():
    """One LM attempt from the same point: same lambda, eta, PCG iterations and rho."""
    pr = synth.make_small(7, obj_side=40, probe=(16, 16), n=5, step=5, photons=1e3, mode="joint")
    rng = np.random.default_rng(7)
    O0 = pr.O_init.astype(np.complex64)
    P0 = pr.P_init.astype(np.complex64)
    y = synth.poisson_counts(rng, ptycho.intensity(pr.O_true, pr.P_true, pr.pos, pr.background)).astype(np.float32)
    for scaling, precond in ((0, 0), (1, 1), (0, 1)):
        p_or = solver.LMParams(scaling=scaling, precond=precond)
        ref = solver.lm_solve(O0.astype(np.complex128), P0.astype(np.complex128), pr.pos, y.astype(np.float64),
                              pr.background, "gauss", True, p_or, 1)
        attempts = [h for h in ref.history if h.t == 0]
        h0 = attempts[-1]                      # the state reflects the last attempt of the iteration
        prob = pt.Problem(pr.O_true.shape, pr.P_true.shape, pr.pos, mode="joint", background=pr.background,
                          device=DEV)
        O, P, yd = to_dev(O0, np.complex64), to_dev(P0, np.complex64), to_dev(y, np.float32)
        params = pt.default_params(scaling=scaling, precond=precond)
        st = prob.new_state()
        prob.lm_init(params, st)
        prob.lm_step(O, P, yd, params, st)
        s = pt.state_from_tensor(st)
        print(scaling, precond, "oracle", h0.lam, h0.eta, h0.cg_iters, h0.rho, "gpu", s.lambda_, s.eta, s.cg_iters,
              s.rho)
        assert s.f == pytest.approx(h0.f, rel=1e-5)
        assert s.eta == pytest.approx(h0.eta, rel=1e-5)
        assert s.lambda_ == pytest.approx(h0.lam, rel=1e-5)
        assert s.retries == len(attempts) - 1 if h0.accepted else s.retries == len(attempts)
        assert abs(s.cg_iters - h0.cg_iters) <= 1
        if s.cg_iters == h0.cg_iters:
            assert s.rho == pytest.approx(h0.rho, rel=1e-3, abs=1e-3)


@pytest.mark.parametrize("mode,alternate", [("joint", 0), ("object", 0), ("joint", 1)])
def test_first_pcg_curvature_matches_oracle(mode, alternate):
    """p^T (G + lambda I) p of a PCG iteration, which the object and probe sums finishing the
    product accumulate block by block (alg:lm_inexact), against the oracle: at t = 0, with D = I,
    no preconditioner and one PCG iteration, PCG starts from zero and p = r = -g, so the state
    holds g^T G g + lambda g^T g at the linearisation point.  Under the alternating update the
    state is that of the probe sub-step: p is -g on the probe block and zero on the object, at
    the object the first sub-step left."""
    pr = synth.make_small(11, obj_side=40, probe=(16, 16), n=5, step=5, photons=1e3, mode=mode)
    rng = np.random.default_rng(11)
    joint = mode == "joint"
    y = synth.poisson_counts(rng, ptycho.intensity(pr.O_true, pr.P_true, pr.pos, pr.background)).astype(np.float32)
    O0, P0 = pr.O_init.astype(np.complex64), pr.P_init.astype(np.complex64)
    prob = pt.Problem(pr.O_true.shape, pr.P_true.shape, pr.pos, mode=mode, background=pr.background, device=DEV)
    O, P, yd = to_dev(O0, np.complex64), to_dev(P0, np.complex64), to_dev(y, np.float32)
    params = pt.default_params(scaling=0, precond=0, cg_max=1, alternate=alternate)
    st = prob.new_state()
    prob.lm_init(params, st)
    prob.lm_step(O, P, yd, params, st)
    s = pt.state_from_tensor(st)
    # the probe sub-step linearises at the object the object sub-step left (read back)
    Olin = O.cpu().numpy() if alternate else O0
    lin = ptycho.linearize(Olin.astype(np.complex128), P0.astype(np.complex128), pr.pos, y.astype(np.float64),
                           pr.background, "gauss", joint)
    gO, gP = ptycho.gradient(lin)
    if alternate:
        GO, GP = ptycho.ggn_vp(lin, np.zeros_like(gO), gP)
        ref = solver.rdot(gP, GP) + s.lambda_ * solver.rdot(gP, gP)
    else:
        GO, GP = ptycho.ggn_vp(lin, gO, gP)
        ref = solver.rdot(gO, GO) + s.lambda_ * solver.rdot(gO, gO)
        if joint:
            ref += solver.rdot(gP, GP) + s.lambda_ * solver.rdot(gP, gP)
    print(mode, alternate, "pap gpu", s.pap, "oracle", ref, "cg_iters", s.cg_iters)
    assert s.cg_iters == 1
    assert s.pap == pytest.approx(ref, rel=1e-5)


@pytest.mark.parametrize("shape,metric", [((32, 32), "gauss"), ((48, 48), "gauss"), ((64, 64), "gauss"),
                                          ((96, 96), "gauss"), ((256, 256), "gauss"), ((32, 64), "gauss"),
                                          ((128, 32), "gauss"), ((48, 48), "poisson"), ((96, 96), "poisson")])
def test_joint_lm_other_probe_sides_matches_oracle(shape, metric):
    """The joint scaled-Jacobi LM (alg:lm_inexact) through the tile kernels of other probe shapes:
    32 x 32 in its wide workgroup grouping, 48 x 48 and 96 x 96 with their 16 x 3 and 16 x 6
    transforms (the linearisation keeping the probe partial in the segment slot), 64 x 64,
    256 x 256 with its three stages through the transform tile, and the rectangular 32 x 64 and
    128 x 32.

    Gaussian metric: ten outer iterations end within 1 % of the oracle's loss.  Poisson metric
    (about 0.4 photons per pixel, damping down to 1e-8): the first outer iteration (linearisation,
    App. B diagonal, ten PCG products, trial loss) matches the oracle's loss and gain ratio;
    later iterations are not compared, since from the second one the truncated PCG in single
    precision and the FP64 oracle take visibly different steps on this ill-conditioned system
    (48 x 48: after ten iterations the GPU ends 16 % higher above the metric's minimum, and the
    oracle itself ends 13-21 % higher when its start is perturbed by 1e-7 or 1e-6 relative)."""
    print("case lm shape", shape, metric, flush=True)
    side = max(shape)
    seed = 40 + shape[0] + (shape[1] if shape[1] != shape[0] else 0)
    n, step = (3, 64) if side == 256 else (4, side // 4)
    pr = synth.make_small(seed, obj_side=(n - 1) * step + side + 8, probe=shape, n=n, step=step, photons=1e3,
                          mode="joint")
    rng = np.random.default_rng(seed)
    O0 = pr.O_init.astype(np.complex64)
    P0 = pr.P_init.astype(np.complex64)
    y = synth.poisson_counts(rng, ptycho.intensity(pr.O_true, pr.P_true, pr.pos, pr.background)).astype(np.float32)
    T = 10 if metric == "gauss" else 1
    p_or = solver.LMParams(scaling=1, precond=1)
    ref = solver.lm_solve(O0.astype(np.complex128), P0.astype(np.complex128), pr.pos, y.astype(np.float64),
                          pr.background, metric, True, p_or, T)
    prob = pt.Problem(pr.O_true.shape, pr.P_true.shape, pr.pos, metric=metric, mode="joint",
                      background=pr.background, device=DEV)
    O, P, yd = to_dev(O0, np.complex64), to_dev(P0, np.complex64), to_dev(y, np.float32)
    params = pt.default_params(scaling=1, precond=1)
    st = prob.new_state()
    prob.lm_init(params, st)
    prob.lm_solve(O, P, yd, params, T, st)
    f_gpu = float(prob.loss(O, P, yd).cpu()[0])
    f0 = ref.f_per_iter[0]
    print("shape %s %s: oracle f=%.6e gpu f=%.6e (start %.3e)" % (shape, metric, ref.f, f_gpu, f0))
    assert f_gpu < f0
    if metric == "gauss":
        assert f_gpu <= 1.01 * ref.f
    else:
        s = pt.state_from_tensor(st)
        h0 = [h for h in ref.history if h.t == 0][-1]
        assert h0.accepted and s.retries == 0
        assert f_gpu == pytest.approx(ref.f, rel=1e-4)
        assert s.rho == pytest.approx(h0.rho, rel=1e-3)


def _small_joint(seed=9):
    pr = synth.make_small(seed, obj_side=40, probe=(16, 16), n=5, step=5, photons=1e3, mode="joint")
    rng = np.random.default_rng(seed)
    y = synth.poisson_counts(rng, ptycho.intensity(pr.O_true, pr.P_true, pr.pos, pr.background)).astype(np.float32)
    prob = pt.Problem(pr.O_true.shape, pr.P_true.shape, pr.pos, mode="joint", background=pr.background, device=DEV)
    return pr, prob, to_dev(pr.O_init, np.complex64), to_dev(pr.P_init, np.complex64), to_dev(y, np.float32)


def test_all_rejected_outer_iteration_keeps_iterate():
    """Forced rejection: with no PCG iterations (and no accepted step to warm-start from) the
    step is zero, its predicted reduction is not positive and every retry is rejected (the gain
    ratio is taken as -inf when the predicted reduction is not positive); the step reports
    PTLM_ENOTACCEPTED, the iterate is unchanged and t advances (a retry budget spent ends the
    outer iteration without a step)."""
    pr, prob, O, P, y = _small_joint()
    O0, P0 = O.clone(), P.clone()
    params = pt.default_params(scaling=1, precond=1, cg_max=0, retry_max=3)
    st = prob.new_state()
    prob.lm_init(params, st)
    assert prob.lm_step(O, P, y, params, st) == pt.PTLM_ENOTACCEPTED
    s = pt.state_from_tensor(st)
    assert s.t == 1 and s.attempts == 3 and s.retries == 3 and s.status == pt.PTLM_ENOTACCEPTED
    assert torch.equal(O, O0) and torch.equal(P, P0)
    assert s.mu == pytest.approx(1e-5 * 4.0 ** 3)
    # the next outer iteration starts over (retries reset, same linearisation reused)
    assert prob.lm_step(O, P, y, params, st) == pt.PTLM_ENOTACCEPTED
    s = pt.state_from_tensor(st)
    assert s.t == 2 and s.attempts == 6 and torch.equal(O, O0)


def test_nonfinite_data_reports_enumeric_and_keeps_iterate():
    pr, prob, O, P, y = _small_joint()
    y[0, 3, 4] = float("nan")
    O0, P0 = O.clone(), P.clone()
    params = pt.default_params(scaling=1, precond=1)
    st = prob.new_state()
    prob.lm_init(params, st)
    with pytest.raises(pt.PtlmError) as e:
        prob.lm_step(O, P, y, params, st)
    assert e.value.status == pt.PTLM_ENUMERIC
    s = pt.state_from_tensor(st)
    assert s.nonfinite == 1 and s.status == pt.PTLM_ENUMERIC and s.t == 0
    assert torch.equal(O, O0) and torch.equal(P, P0)
    with pytest.raises(pt.PtlmError):  # the state stays failed
        prob.lm_step(O, P, y, params, st)


def test_batch_with_one_failing_problem_finishes_the_others():
    pr, prob, O, P, y = _small_joint(9)
    pr2, prob2, O2, P2, y2 = _small_joint(10)
    y2[1, 2, 2] = float("inf")
    specs = [dict(obj_shape=p.O_true.shape, probe_shape=p.P_true.shape, positions=p.pos, mode="joint",
                  background=p.background) for p in (pr, pr2)]
    b = pt.Batch(specs, device=DEV)
    params = pt.default_params(scaling=1, precond=1)
    b.bind([O, O2], [P, P2], [y, y2], params, 3, use_graph=True)
    status, attempts = b.solve(60, check_every=1)
    assert status == pt.PTLM_ENUMERIC
    s0, s1 = b.all_states()
    assert s0.t == 3 and s0.status in (pt.PTLM_OK, pt.PTLM_ENOTACCEPTED)
    assert s1.status == pt.PTLM_ENUMERIC and s1.t == 0
    assert torch.equal(O2, to_dev(pr2.O_init, np.complex64))


@pytest.mark.parametrize("variant", ["surrogate_poisson", "exact_jacobi"])
def test_lm_variants_match_oracle_final_loss(variant):
    """The surrogate Poisson metric of App. E (PLM-S, beta = 0.9) and the exact-diagonal
    Jacobi preconditioner: final loss within 1.01x of the oracle's LM on the same problem."""
    print("case lm variant", variant, flush=True)
    pr = synth.make_small(11, obj_side=48, probe=(16, 16), n=6, step=5, photons=1e3, mode="joint")
    rng = np.random.default_rng(11)
    y = synth.poisson_counts(rng, ptycho.intensity(pr.O_true, pr.P_true, pr.pos, pr.background)).astype(np.float32)
    if variant == "surrogate_poisson":
        metric, T = "poisson", 8
        kw = dict(scaling=1, precond=1, beta=0.9, surrogate_T=5, surrogate_s0=1.0)
    else:
        metric, T = "gauss", 8
        kw = dict(scaling=1, precond=3)
    ref = solver.lm_solve(pr.O_init, pr.P_init, pr.pos, y.astype(np.float64), pr.background, metric, True,
                          solver.LMParams(**kw), T)
    prob = pt.Problem(pr.O_true.shape, pr.P_true.shape, pr.pos, metric=metric, mode="joint",
                      background=pr.background, device=DEV)
    O, P, yd = to_dev(pr.O_init, np.complex64), to_dev(pr.P_init, np.complex64), to_dev(y, np.float32)
    params = pt.default_params(**kw)
    st = prob.new_state()
    prob.lm_init(params, st)
    s0 = pt.state_from_tensor(st)
    if variant == "surrogate_poisson":
        assert s0.sigma == 1.0
    prob.lm_solve(O, P, yd, params, T, st)
    s = pt.state_from_tensor(st)
    f_gpu = float(prob.loss(O, P, yd).cpu()[0])
    print("%s oracle f=%.6e gpu f=%.6e sigma=%g" % (variant, ref.f, f_gpu, s.sigma))
    assert s.t == T
    # the Poisson metric is negative in general: the 1.01x bar applies above its per-pixel
    # minimum sum(y - y log y), reached at zeta^2 = y (0 log 0 = 0)
    yy = y.astype(np.float64)
    f_min = float(np.sum(yy - yy * np.log(np.where(yy > 0, yy, 1.0)))) if metric == "poisson" else 0.0
    assert f_gpu - f_min <= 1.01 * (ref.f - f_min)
    if variant == "surrogate_poisson":
        assert s.sigma == 0.0   # after T_s iterations the metric is the true Poisson one


@pytest.mark.parametrize("mode,gamma", [("joint", 1e-6), ("joint", 0.0), ("object", 0.0)])
def test_projected_lm_matches_oracle(mode, gamma):
    """alg:projected_LM (|O| <= 1): feasible iterates, same plug-in branch and step size as the
    oracle on the first iteration, final loss within 1.01x of the oracle's.  gamma = 0 never
    takes the projected point, so every accepted step goes through the line search."""
    print("case projected lm", mode, "gamma", gamma, flush=True)
    joint = mode == "joint"
    pr = synth.make_small(6, obj_side=48, probe=(16, 16), n=6, step=5, photons=1e3, mode=mode)
    rng = np.random.default_rng(6)
    O_true = pr.O_true / np.abs(pr.O_true).max()
    y = synth.poisson_counts(rng, ptycho.intensity(O_true, pr.P_true, pr.pos, pr.background)).astype(np.float32)
    T = 8
    P0 = pr.P_init if joint else pr.P_true
    ref = solver.lm_solve(pr.O_init, P0, pr.pos, y.astype(np.float64), pr.background, "gauss", joint,
                          solver.LMParams(scaling=1, precond=1, project=True, gamma=gamma), T)
    first = [h for h in ref.history if h.t == 0 and h.accepted][0]
    if gamma == 0.0:
        assert first.ls[0] != "lm"
    prob = pt.Problem(pr.O_true.shape, pr.P_true.shape, pr.pos, mode=mode, background=pr.background, device=DEV)
    O, P, yd = to_dev(pr.O_init, np.complex64), to_dev(P0, np.complex64), to_dev(y, np.float32)
    params = pt.default_params(scaling=1, precond=1, project=1, gamma=gamma)
    st = prob.new_state()
    prob.lm_init(params, st)
    prob.lm_step(O, P, yd, params, st)
    s = pt.state_from_tensor(st)
    names = {0: "lm", 1: "direction", 2: "gradient", -1: "none"}
    assert names[s.ls_branch] == first.ls[0]
    assert s.ls_alpha == pytest.approx(first.ls[1])
    fs = [float(prob.loss(O, P, yd).cpu()[0])]
    for _ in range(T - 1):
        prob.lm_step(O, P, yd, params, st)
        fs.append(float(prob.loss(O, P, yd).cpu()[0]))
        assert float(torch.abs(O).max()) <= 1.0 + 1e-6
    print("projected oracle f=%.6e gpu f=%.6e" % (ref.f, fs[-1]))
    assert all(fs[i + 1] <= fs[i] * (1 + 1e-6) for i in range(len(fs) - 1))
    assert fs[-1] <= 1.01 * ref.f


# ---------------------------------------------------------------- alternating update (alg:alt_LM_ptycho)
@pytest.mark.parametrize("scaling,precond", [(0, 0), (1, 1)])
def test_alternating_step_matches_oracle_substeps(scaling, precond):
    """One outer iteration of the alternating update from the same point: the state after it
    holds the probe sub-step's last attempt (lambda, eta, PCG products, rho) and both blocks'
    damping values as the oracle's."""
    print("case alternating step", scaling, precond, flush=True)
    pr = synth.make_small(7, obj_side=40, probe=(16, 16), n=5, step=5, photons=1e3, mode="joint")
    rng = np.random.default_rng(7)
    y = synth.poisson_counts(rng, ptycho.intensity(pr.O_true, pr.P_true, pr.pos, pr.background)).astype(np.float32)
    p_or = solver.LMParams(scaling=scaling, precond=precond, alternate=True)
    ref = solver.lm_solve(pr.O_init, pr.P_init, pr.pos, y.astype(np.float64), pr.background, "gauss", True, p_or, 1)
    hO = [h for h in ref.history if h.block == "O"]
    hP = [h for h in ref.history if h.block == "P"]
    prob = pt.Problem(pr.O_true.shape, pr.P_true.shape, pr.pos, mode="joint", background=pr.background, device=DEV)
    O, P, yd = to_dev(pr.O_init, np.complex64), to_dev(pr.P_init, np.complex64), to_dev(y, np.float32)
    params = pt.default_params(scaling=scaling, precond=precond, alternate=1)
    st = prob.new_state()
    prob.lm_init(params, st)
    prob.lm_step(O, P, yd, params, st)
    s = pt.state_from_tensor(st)
    h0 = hP[-1]
    print("oracle P", h0.lam, h0.eta, h0.cg_iters, h0.rho, h0.f, "gpu", s.lambda_, s.eta, s.cg_iters, s.rho, s.f)
    assert s.t == 1 and s.block == 1
    assert s.f == pytest.approx(h0.f, rel=1e-5)               # f at (O_{t+1}, P_t)
    assert s.eta == pytest.approx(h0.eta, rel=1e-5)
    assert s.lambda_ == pytest.approx(h0.lam, rel=1e-5)
    assert abs(s.cg_iters - h0.cg_iters) <= 1
    if s.cg_iters == h0.cg_iters:
        assert s.rho == pytest.approx(h0.rho, rel=1e-3, abs=1e-3)
    mu_o = solver.mu_update(hO[-1].rho, hO[-1].mu, p_or)[0]
    mu_p = solver.mu_update(hP[-1].rho, hP[-1].mu, p_or)[0]
    assert s.mu_alt == pytest.approx(mu_o, rel=1e-12) and s.mu == pytest.approx(mu_p, rel=1e-12)
    # the object is the oracle's after its sub-step (the probe sub-step leaves it as it is)
    Og = O.cpu().numpy().astype(np.complex128)
    assert np.linalg.norm(Og - ref.O) <= 1e-3 * np.linalg.norm(ref.O)


@pytest.mark.parametrize("variant", ["plain", "scaled_jacobi", "projected"])
def test_alternating_lm_matches_oracle(variant):
    """LM-A and PLM-A: final loss within 1.01x of the oracle's alternating LM."""
    print("case alternating lm", variant, flush=True)
    pr = synth.make_small(5, obj_side=48, probe=(16, 16), n=6, step=5, photons=1e3, mode="joint")
    rng = np.random.default_rng(5)
    O_true = pr.O_true / np.abs(pr.O_true).max() if variant == "projected" else pr.O_true
    y = synth.poisson_counts(rng, ptycho.intensity(O_true, pr.P_true, pr.pos, pr.background)).astype(np.float32)
    kw = {"plain": {}, "scaled_jacobi": dict(scaling=1, precond=1),
          "projected": dict(scaling=1, precond=1, project=True)}[variant]
    T = 10
    ref = solver.lm_solve(pr.O_init, pr.P_init, pr.pos, y.astype(np.float64), pr.background, "gauss", True,
                          solver.LMParams(alternate=True, **kw), T)
    prob = pt.Problem(pr.O_true.shape, pr.P_true.shape, pr.pos, mode="joint", background=pr.background, device=DEV)
    O, P, yd = to_dev(pr.O_init, np.complex64), to_dev(pr.P_init, np.complex64), to_dev(y, np.float32)
    params = pt.default_params(alternate=1, **{k: int(v) for k, v in kw.items()})
    st = prob.new_state()
    prob.lm_init(params, st)
    prob.lm_solve(O, P, yd, params, T, st)
    s = pt.state_from_tensor(st)
    f_gpu = float(prob.loss(O, P, yd).cpu()[0])
    print("alternating %s oracle f=%.6e gpu f=%.6e (start %.3e)" % (variant, ref.f, f_gpu, ref.f_per_iter[0]))
    assert s.t == T
    assert f_gpu <= 1.01 * ref.f
    assert f_gpu < 0.5 * ref.f_per_iter[0]
    if variant == "projected":
        assert float(torch.abs(O).max()) <= 1.0 + 1e-6


def test_alternating_needs_joint_problem():
    pr = synth.make_small(3, obj_side=40, probe=(16, 16), n=4, step=6, photons=1e3, mode="object")
    prob = pt.Problem(pr.O_true.shape, pr.P_true.shape, pr.pos, mode="object", background=pr.background, device=DEV)
    st = prob.new_state()
    with pytest.raises(pt.PtlmError) as e:
        prob.lm_init(pt.default_params(alternate=1), st)
    assert e.value.status == pt.PTLM_EINVAL


# ---------------------------------------------------------------- intensity-based GGN (App. C ablation)
@pytest.mark.parametrize("mode", ["object", "joint"])
def test_intensity_ggn_lm_matches_oracle(mode):
    """LM on the intensity-based GGN (eq:ggn_intensity): final loss within 1.01x of the oracle's
    LM on the same GGN; on the object problem it ends above the magnitude-based LM (Fig. 1)."""
    print("case intensity lm", mode, flush=True)
    joint = mode == "joint"
    pr = synth.make_small(5, obj_side=48, probe=(16, 16), n=6, step=5, photons=1e3, mode=mode)
    rng = np.random.default_rng(5)
    y = synth.poisson_counts(rng, ptycho.intensity(pr.O_true, pr.P_true, pr.pos, pr.background)).astype(np.float32)
    P0 = pr.P_init if joint else pr.P_true
    kw = dict(scaling=1, precond=1) if joint else {}
    T = 10
    ref = solver.lm_solve(pr.O_init, P0, pr.pos, y.astype(np.float64), pr.background, "gauss", joint,
                          solver.LMParams(ggn="intensity", **kw), T)
    f_gpu = {}
    for ggn in ("intensity", "magnitude"):
        prob = pt.Problem(pr.O_true.shape, pr.P_true.shape, pr.pos, mode=mode, background=pr.background,
                          device=DEV, ggn=ggn)
        O, P, yd = to_dev(pr.O_init, np.complex64), to_dev(P0, np.complex64), to_dev(y, np.float32)
        params = pt.default_params(**kw)
        st = prob.new_state()
        prob.lm_init(params, st)
        prob.lm_solve(O, P, yd, params, T, st)
        assert pt.state_from_tensor(st).t == T
        f_gpu[ggn] = float(prob.loss(O, P, yd).cpu()[0])
    print("intensity %s oracle f=%.6e gpu f=%.6e magnitude gpu f=%.6e" % (mode, ref.f, f_gpu["intensity"],
                                                                        f_gpu["magnitude"]))
    assert f_gpu["intensity"] <= 1.01 * ref.f
    if not joint:
        assert f_gpu["magnitude"] < f_gpu["intensity"]


def test_stochastic_jacobi_lm_matches_oracle():
    """precond 4: the PCG preconditioner built from the stochastic diagonal estimate, drawn per
    outer iteration from the same counter-based signs as the oracle: final loss within 1.01x."""
    print("case stochastic lm", flush=True)
    pr = synth.make_small(11, obj_side=48, probe=(16, 16), n=6, step=5, photons=1e3, mode="joint")
    rng = np.random.default_rng(11)
    y = synth.poisson_counts(rng, ptycho.intensity(pr.O_true, pr.P_true, pr.pos, pr.background)).astype(np.float32)
    kw = dict(scaling=1, precond=4, stoch_samples=6, stoch_seed=99)
    T = 8
    ref = solver.lm_solve(pr.O_init, pr.P_init, pr.pos, y.astype(np.float64), pr.background, "gauss", True,
                          solver.LMParams(**kw), T)
    prob = pt.Problem(pr.O_true.shape, pr.P_true.shape, pr.pos, mode="joint", background=pr.background, device=DEV)
    O, P, yd = to_dev(pr.O_init, np.complex64), to_dev(pr.P_init, np.complex64), to_dev(y, np.float32)
    params = pt.default_params(**kw)
    st = prob.new_state()
    prob.lm_init(params, st)
    prob.lm_solve(O, P, yd, params, T, st)
    s = pt.state_from_tensor(st)
    f_gpu = float(prob.loss(O, P, yd).cpu()[0])
    print("stochastic oracle f=%.6e gpu f=%.6e (start %.3e)" % (ref.f, f_gpu, ref.f_per_iter[0]))
    assert s.t == T
    assert f_gpu <= 1.01 * ref.f


# ---------------------------------------------------------------- trial-point linearisation kept
def test_kept_trial_linearisation_is_adopted_only_at_the_same_point():
    """An accepted trial point's linearisation is adopted by the next outer iteration (no
    linearisation launch); after the caller moves O, or linearises the handle elsewhere, the
    next step linearises afresh: its f is the loss at the caller's current iterate."""
    print("case kept linearisation", flush=True)
    pr, prob, O, P, yd = _small_joint(13)
    params = pt.default_params(scaling=1, precond=1)
    st = prob.new_state()
    prob.lm_init(params, st)
    prob.lm_step(O, P, yd, params, st)
    s1 = pt.state_from_tensor(st)
    prob.lm_step(O, P, yd, params, st)
    s2 = pt.state_from_tensor(st)
    assert s1.accepted and s2.tile_now == 0          # adopted: f_t of step 2 is step 1's trial value
    assert s2.f == pytest.approx(s1.f_trial, rel=1e-12)
    # the caller moves the object: the next step must linearise at the moved point
    O.mul_(0.97)
    f_moved = float(prob.loss(O, P, yd).cpu()[0])
    prob.lm_step(O, P, yd, params, st)
    s3 = pt.state_from_tensor(st)
    assert s3.f == pytest.approx(f_moved, rel=1e-5)
    # a linearisation of the handle at another point between steps is not adopted either
    f_here = float(prob.loss(O, P, yd).cpu()[0])
    prob.linearize(O * 0.9, P, yd)
    prob.lm_step(O, P, yd, params, st)
    s4 = pt.state_from_tensor(st)
    assert s4.f == pytest.approx(f_here, rel=1e-5)


def test_lm_at_the_solution_stays_put():
    """Degenerate case: noise-free data and the iterate at the ground truth (f and g vanish up to
    single-precision rounding).  No value turns non-finite, the state stays usable and the
    iterate stays at the truth to rounding, whether the attempts are accepted or all rejected."""
    print("case at solution", flush=True)
    pr = synth.make_small(17, obj_side=40, probe=(16, 16), n=5, step=5, photons=1e3, mode="joint")
    y = ptycho.intensity(pr.O_true, pr.P_true, pr.pos, pr.background).astype(np.float32)
    prob = pt.Problem(pr.O_true.shape, pr.P_true.shape, pr.pos, mode="joint", background=pr.background, device=DEV)
    O, P, yd = to_dev(pr.O_true, np.complex64), to_dev(pr.P_true, np.complex64), to_dev(y, np.float32)
    O0, P0 = O.clone(), P.clone()
    for kw in (dict(scaling=1, precond=1), dict()):
        params = pt.default_params(**kw)
        st = prob.new_state()
        prob.lm_init(params, st)
        for _ in range(3):
            prob.lm_step(O, P, yd, params, st)
        s = pt.state_from_tensor(st)
        assert s.t == 3 and s.status != pt.PTLM_ENUMERIC and s.nonfinite == 0
        assert math.isfinite(s.f) and math.isfinite(s.mu) and math.isfinite(s.lambda_)
        assert bool(torch.isfinite(torch.view_as_real(O)).all()) and bool(torch.isfinite(torch.view_as_real(P)).all())
        assert float(torch.linalg.norm(O - O0) / torch.linalg.norm(O0)) < 1e-4
        assert float(torch.linalg.norm(P - P0) / torch.linalg.norm(P0)) < 1e-4


def test_projected_line_search_limits():
    """The projected plug-in's line-search bounds: with no step size to try (ls_max = 0) every
    accepted step keeps z_t (branch -1, step size 0), and a bound past the host look-ahead's
    slots (all step sizes enqueued at once) gives the same iterates as the default bound."""
    print("case projected limits", flush=True)
    pr = synth.make_small(6, obj_side=48, probe=(16, 16), n=6, step=5, photons=1e3, mode="joint")
    rng = np.random.default_rng(6)
    O_true = pr.O_true / np.abs(pr.O_true).max()
    y = to_dev(synth.poisson_counts(rng, ptycho.intensity(O_true, pr.P_true, pr.pos, pr.background))
               .astype(np.float32), np.float32)
    prob = pt.Problem(pr.O_true.shape, pr.P_true.shape, pr.pos, mode="joint", background=pr.background, device=DEV)
    runs = {}
    for ls_max in (0, 30, 200):
        O, P = to_dev(pr.O_init, np.complex64), to_dev(pr.P_init, np.complex64)
        params = pt.default_params(scaling=1, precond=1, project=1, gamma=0.0, ls_max=ls_max)
        st = prob.new_state()
        prob.lm_init(params, st)
        for _ in range(3):
            prob.lm_step(O, P, y, params, st)
        runs[ls_max] = (O, P, pt.state_from_tensor(st))
    O0, P0, s0 = runs[0]
    assert torch.equal(O0, to_dev(pr.O_init, np.complex64)) and torch.equal(P0, to_dev(pr.P_init, np.complex64))
    assert s0.ls_branch == -1 and s0.ls_alpha == 0.0
    (O1, P1, s1), (O2, P2, s2) = runs[30], runs[200]
    assert s1.ls_branch in (1, 2) and s1.ls_alpha > 0
    assert torch.equal(O1, O2) and torch.equal(P1, P2) and s1.f == s2.f and s1.ls_alpha == s2.ls_alpha
