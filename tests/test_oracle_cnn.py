"""Pins of the FP64 CNN oracle: convolution against SciPy's correlation, the backward pass
against central finite differences, Adam's first step against its closed form."""
import numpy as np
import pytest
from scipy import signal

from oracle import cnn

RNG = np.random.default_rng(4)


def test_conv3x3_is_zero_padded_correlation():
    x = RNG.standard_normal((2, 3, 7, 9))
    W = RNG.standard_normal((4, 3, 3, 3))
    b = RNG.standard_normal(4)
    y = cnn.conv3x3(x, W, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(signal.correlate2d(x[n, c], W[o, c], mode="same", boundary="fill")
                             for c in range(3))
            np.testing.assert_allclose(y[n, o], ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("layers", [1, 2, 3])
def test_gradient_matches_finite_differences(layers):
    cin, cmid, cout = 3, 4, 2
    x = RNG.standard_normal((2, cin, 6, 5))
    t = RNG.standard_normal((2, cout, 6, 5))
    mask = (RNG.uniform(size=t.shape) > 0.3).astype(float)
    p = cnn.init_params(RNG, cin, cmid, cout, layers) + 0.1 * RNG.standard_normal(cnn.param_count(cin, cmid, cout, layers))
    L, g = cnn.grad(p, x, t, mask, cin, cmid, cout, layers)
    assert L == pytest.approx(cnn.loss(p, x, t, mask, cin, cmid, cout, layers))
    h = 1e-6
    idx = RNG.choice(len(p), size=min(40, len(p)), replace=False)
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (cnn.loss(p + e, x, t, mask, cin, cmid, cout, layers) -
              cnn.loss(p - e, x, t, mask, cin, cmid, cout, layers)) / (2 * h)
        assert abs(g[i] - fd) <= 1e-6 * max(1.0, abs(fd)), (i, g[i], fd)


def test_adam_first_step_is_signed_learning_rate():
    p = RNG.standard_normal(10)
    g = RNG.standard_normal(10)
    p1, m, v = cnn.adam(p, g, np.zeros(10), np.zeros(10), 1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(p1, p - 0.01 * np.sign(g), rtol=1e-12)


def test_features_and_learned_diag_shapes():
    P = RNG.standard_normal((4, 4)) + 1j * RNG.standard_normal((4, 4))
    pos = np.array([[0, 0], [2, 3], [4, 4]])
    f = cnn.features(P, pos, (9, 9))
    assert f.shape == (3, 9, 9) and f[0].max() == pytest.approx(1.0)
    assert np.all(f[0][8, 0:3] == 0.0) and np.all(np.abs(f[2]) <= 1.0 + 1e-12)
    dO = RNG.uniform(0.5, 2.0, (9, 9, 2))
    d = cnn.learned_diag(dO, np.ones((4, 4, 2)), np.zeros((2, 9, 9)))
    # an untrained network (r = 0) gives the constant s = largest App. B object entry
    assert d.shape == (81 + 16, 2) and np.all(d[:81] == dO.max()) and np.all(d[81:] == 1.0)


def _small_object_problem():
    from oracle import ptycho
    import synth
    pr = synth.make_c3(2001)
    y = ptycho.intensity(pr.O_true, pr.P_true, pr.pos, pr.background)
    return pr, y


def test_network_predicting_the_app_b_shape_gives_back_jacobi():
    """r = target(App. B diagonal) makes the learned diagonal the floored App. B diagonal, so the
    LM with the learned preconditioner takes the Jacobi LM's steps exactly (D = I)."""
    from oracle import ptycho, solver
    pr, y = _small_object_problem()
    lin = ptycho.linearize(pr.O_init, pr.P_true, pr.pos, y, pr.background, "gauss", False)
    dO, _ = ptycho.ggn_diag_paper(lin)
    r = cnn.target(dO, dO)
    ld = cnn.learned_diag(dO, None, r)
    np.testing.assert_allclose(ld, np.maximum(dO, 1e-6 * dO.max()).reshape(-1, 2), rtol=1e-12)
    # the LM's Jacobi path recomputes App. B at every iterate; a fixed learned diagonal equals it
    # only at the first linearisation, so compare one outer iteration
    a = solver.lm_solve(pr.O_init, pr.P_true, pr.pos, y, pr.background, "gauss", False,
                        solver.LMParams(precond=1), 1)
    b = solver.lm_solve(pr.O_init, pr.P_true, pr.pos, y, pr.background, "gauss", False,
                        solver.LMParams(precond=2), 1, learned_diag=ld)
    assert [(h.cg_iters, h.accepted) for h in a.history] == [(h.cg_iters, h.accepted) for h in b.history]
    np.testing.assert_allclose(b.O, a.O, rtol=1e-10, atol=1e-12)


def test_untrained_network_is_unpreconditioned_cg():
    """A constant diagonal preconditioner (the untrained network, r = 0) leaves the CG iterates of
    the unpreconditioned solve unchanged: scaling the preconditioner by a constant does not move
    them (textbook property of PCG)."""
    from oracle import ptycho, solver
    pr, y = _small_object_problem()
    lin = ptycho.linearize(pr.O_init, pr.P_true, pr.pos, y, pr.background, "gauss", False)
    dO, _ = ptycho.ggn_diag_paper(lin)
    ld = cnn.learned_diag(dO, None, np.zeros((2,) + pr.O_true.shape))
    lam = 0.05
    A = lambda v: ptycho.ggn_vp(lin, v.reshape(pr.O_true.shape))[0].ravel() + lam * v
    g = ptycho.gradient(lin)[0].ravel()
    m = ld + lam
    pc = lambda rr: rr.real / m[:, 0] + 1j * rr.imag / m[:, 1]
    for it in (1, 3, 6):
        x0 = np.zeros_like(g)
        xa = solver.pcg(A, g, x0, None, 0.0, it).x
        xb = solver.pcg(A, g, x0, pc, 0.0, it).x
        assert np.linalg.norm(xa - xb) <= 1e-10 * np.linalg.norm(xa)


def test_target_is_log_of_floored_exact_diagonal_over_scale():
    d = RNG.uniform(1e-9, 3.0, (5, 6, 2))
    d[0, 0] = [0.0, 0.0]
    dO = RNG.uniform(0.5, 2.0, (5, 6, 2))
    t = cnn.target(d, dO)
    assert t.shape == (2, 5, 6)
    assert t[0, 0, 0] == pytest.approx(np.log(1e-6 * d.max() / dO.max()))
    assert t[1, 2, 3] == pytest.approx(np.log(max(d[2, 3, 1], 1e-6 * d.max()) / dO.max()))


def _coverage_count(pos, probe_shape, obj_shape):
    """Number of scan windows covering each object pixel, by direct counting."""
    cnt = np.zeros(obj_shape)
    for r, c in pos:
        for i in range(probe_shape[0]):
            for j in range(probe_shape[1]):
                cnt[r + i, c + j] += 1
    return cnt


def test_features_of_a_flat_probe_are_coverage_count_ones_and_zero_phase():
    pos = np.array([[0, 0], [1, 2], [3, 3], [3, 0]])
    P = np.ones((4, 5), complex)
    f = cnn.features(P, pos, (9, 10))
    cnt = _coverage_count(pos, P.shape, (9, 10))
    np.testing.assert_allclose(f[0], cnt / cnt.max(), rtol=1e-14)
    np.testing.assert_allclose(f[1], (cnt > 0).astype(float), rtol=1e-14)
    np.testing.assert_array_equal(f[2], 0.0)


def test_features_of_a_constant_phase_probe_carry_that_phase():
    pos = np.array([[0, 0], [2, 1], [1, 4]])
    amp = RNG.uniform(0.2, 1.0, (4, 4))
    phi = 0.7
    f = cnn.features(amp * np.exp(1j * phi), pos, (8, 9))
    cov = _coverage_count(pos, (4, 4), (8, 9)) > 0
    np.testing.assert_allclose(f[2][cov], phi / np.pi, rtol=1e-13)
    np.testing.assert_array_equal(f[2][~cov], 0.0)


def test_features_of_one_position_are_the_probe_maps():
    P = RNG.standard_normal((5, 4)) + 1j * RNG.standard_normal((5, 4))
    r, c = 2, 3
    f = cnn.features(P, np.array([[r, c]]), (9, 10))
    q = np.abs(P) ** 2
    win = (slice(r, r + 5), slice(c, c + 4))
    np.testing.assert_allclose(f[0][win], q / q.max(), rtol=1e-13)
    np.testing.assert_allclose(f[1][win], q / q.max(), rtol=1e-13)
    np.testing.assert_allclose(f[2][win], np.angle(P) / np.pi, rtol=1e-13)
    outside = np.ones((9, 10), bool)
    outside[win] = False
    assert np.all(f[:, outside] == 0.0)
