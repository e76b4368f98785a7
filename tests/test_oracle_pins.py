"""Pins of the FP64 oracle against facts fixed outside the oracle itself.

Each test checks an oracle function against something it cannot agree with by
construction: the DFT written from its definition, Parseval, finite
differences of the forward model alone, the adjoint identity, a dense Jacobian
built by finite differences, null vectors that follow from the model's
symmetries, a dense linear solve, and zero-loss convergence on noise-free
data.  A dropped term, a wrong sign or index, or a transposed operand anywhere
in ``oracle.ptycho`` / ``oracle.solver`` fails at least one of them.
"""
import math

import numpy as np
import pytest

import synth
from oracle import ptycho, solver

RNG = np.random.default_rng(12345)


def dft_matrix(n):
    """Unitary DFT matrix from the definition exp(-2 pi i j k / n) / sqrt(n)."""
    j = np.arange(n)
    return np.exp(-2j * math.pi * np.outer(j, j) / n) / math.sqrt(n)


def brute_dft2(x):
    My, Mx = x.shape[-2:]
    return dft_matrix(My) @ x @ dft_matrix(Mx).T


def tiny_problem(seed=7, obj=(9, 10), probe=(4, 3), joint=True, metric="gauss", noisy=True):
    rng = np.random.default_rng(seed)
    O = synth.random_complex(rng, obj) * 0.5 + 0.8
    P = synth.random_complex(rng, probe)
    pos = np.array([[r, c] for r in range(0, obj[0] - probe[0] + 1, 2)
                    for c in range(0, obj[1] - probe[1] + 1, 3)], dtype=np.int32)
    h = ptycho.intensity(O, P, pos, 1e-3)
    y = synth.poisson_counts(rng, 20 * h) / 20 if noisy else h
    if metric == "poisson":
        y = synth.poisson_counts(rng, h * 5.0)
        O = O * math.sqrt(5.0)
    return O, P, pos, y


# ---------------------------------------------------------------- forward model
@pytest.mark.parametrize("shape", [(4, 4), (6, 6), (8, 4), (3, 5)])
def test_dft_matches_definition(shape):
    x = synth.random_complex(RNG, (2,) + shape)
    np.testing.assert_allclose(ptycho.F(x), brute_dft2(x), atol=1e-13)
    np.testing.assert_allclose(ptycho.FH(ptycho.F(x)), x, atol=1e-13)


def test_parseval():
    x = synth.random_complex(RNG, (3, 16, 8))
    np.testing.assert_allclose(np.sum(np.abs(ptycho.F(x)) ** 2, axis=(1, 2)),
                               np.sum(np.abs(x) ** 2, axis=(1, 2)), rtol=1e-13)


def test_exit_wave_by_indexing():
    O = synth.random_complex(RNG, (7, 9))
    P = synth.random_complex(RNG, (3, 4))
    pos = np.array([[0, 0], [4, 5], [2, 3]], dtype=np.int32)
    psi = ptycho.exit_waves(O, P, pos)
    for k, (r, c) in enumerate(pos):
        for i in range(3):
            for j in range(4):
                assert abs(psi[k, i, j] - P[i, j] * O[r + i, c + j]) <= 1e-15 * abs(psi[k, i, j])


def test_single_position_full_probe_is_textbook_magnitude():
    O = synth.random_complex(RNG, (6, 6))
    P = np.ones((6, 6), complex)
    pos = np.zeros((1, 2), np.int32)
    b = 0.25
    zeta = ptycho.magnitude(O, P, pos, b)[0]
    np.testing.assert_allclose(zeta, np.sqrt(np.abs(brute_dft2(O)) ** 2 + b), rtol=1e-13)


def test_adjoint_extract():
    O = synth.random_complex(RNG, (8, 7))
    pos = np.array([[0, 1], [3, 2], [5, 4]], dtype=np.int32)
    w = synth.random_complex(RNG, (3, 3, 3))
    lhs = np.vdot(w, ptycho.extract(O, pos, (3, 3)))
    rhs = np.vdot(ptycho.extract_adjoint(w, pos, O.shape), O)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_metric_values_and_derivatives_by_fd():
    z = np.linspace(0.3, 3.0, 11)
    y = np.linspace(0.0, 4.0, 11)
    np.testing.assert_allclose(ptycho.ell(z, y, "gauss"), 0.5 * (z - np.sqrt(y)) ** 2)
    np.testing.assert_allclose(ptycho.ell(z, y, "poisson"), z ** 2 - y * np.log(z ** 2))
    h = 1e-5
    for m in ("gauss", "poisson"):
        fd1 = (ptycho.ell(z + h, y, m) - ptycho.ell(z - h, y, m)) / (2 * h)
        np.testing.assert_allclose(ptycho.ell_d1(z, y, m), fd1, rtol=1e-8, atol=1e-9)
        fd2 = (ptycho.ell_d1(z + h, y, m) - ptycho.ell_d1(z - h, y, m)) / (2 * h)
        np.testing.assert_allclose(ptycho.ell_d2(z, y, m), fd2, rtol=1e-8)


# ---------------------------------------------------------------- derivatives
def _fd_jacobian(O, P, pos, b, joint):
    """Dense J by central differences of the forward model only."""
    h = 1e-6
    cols = []
    targets = [("O", O.shape)] + ([("P", P.shape)] if joint else [])
    for name, shp in targets:
        n = shp[0] * shp[1]
        for part in (1.0, 1j):
            for i in range(n):
                d = np.zeros(n, complex)
                d[i] = part * h
                d = d.reshape(shp)
                if name == "O":
                    zp = ptycho.magnitude(O + d, P, pos, b)
                    zm = ptycho.magnitude(O - d, P, pos, b)
                else:
                    zp = ptycho.magnitude(O, P + d, pos, b)
                    zm = ptycho.magnitude(O, P - d, pos, b)
                cols.append(((zp - zm) / (2 * h)).ravel())
    # column order: [Re O, Im O, Re P, Im P]
    return np.stack(cols, axis=1)


def _to_real(vO, vP=None):
    parts = [vO.real.ravel(), vO.imag.ravel()]
    if vP is not None:
        parts += [vP.real.ravel(), vP.imag.ravel()]
    return np.concatenate(parts)


@pytest.mark.parametrize("joint", [False, True])
def test_jvp_matches_finite_differences(joint):
    O, P, pos, y = tiny_problem(joint=joint)
    b = 1e-3
    lin = ptycho.linearize(O, P, pos, y, b, "gauss", joint)
    vO = synth.random_complex(RNG, O.shape)
    vP = synth.random_complex(RNG, P.shape) if joint else None
    h = 1e-6
    zp = ptycho.magnitude(O + h * vO, P + (h * vP if joint else 0), pos, b)
    zm = ptycho.magnitude(O - h * vO, P - (h * vP if joint else 0), pos, b)
    fd = (zp - zm) / (2 * h)
    np.testing.assert_allclose(ptycho.jvp(lin, vO, vP), fd, rtol=1e-7, atol=1e-8)


@pytest.mark.parametrize("metric", ["gauss", "poisson"])
@pytest.mark.parametrize("joint", [False, True])
def test_gradient_matches_finite_differences(metric, joint):
    O, P, pos, y = tiny_problem(joint=joint, metric=metric)
    b = 1e-3
    lin = ptycho.linearize(O, P, pos, y, b, metric, joint)
    gO, gP = ptycho.gradient(lin)
    h = 1e-6
    f = lambda O_, P_: ptycho.loss(O_, P_, pos, y, b, metric)
    for idx in [(0, 0), (3, 4), (O.shape[0] - 1, O.shape[1] - 1), (2, 1)]:
        for part in (1.0, 1j):
            d = np.zeros(O.shape, complex)
            d[idx] = part * h
            fd = (f(O + d, P) - f(O - d, P)) / (2 * h)
            an = gO[idx].real if part == 1.0 else gO[idx].imag
            assert abs(an - fd) <= 1e-6 * max(1.0, abs(fd)), (idx, part, an, fd)
    if joint:
        for idx in [(0, 0), (1, 2), (3, 1)]:
            for part in (1.0, 1j):
                d = np.zeros(P.shape, complex)
                d[idx] = part * h
                fd = (f(O, P + d) - f(O, P - d)) / (2 * h)
                an = gP[idx].real if part == 1.0 else gP[idx].imag
                assert abs(an - fd) <= 1e-6 * max(1.0, abs(fd)), (idx, part, an, fd)


@pytest.mark.parametrize("joint", [False, True])
def test_adjoint_identity(joint):
    O, P, pos, y = tiny_problem(joint=joint)
    lin = ptycho.linearize(O, P, pos, y, 1e-3, "gauss", joint)
    vO = synth.random_complex(RNG, O.shape)
    vP = synth.random_complex(RNG, P.shape) if joint else None
    w = RNG.standard_normal(lin.zeta.shape)
    lhs = float(np.sum(ptycho.jvp(lin, vO, vP) * w))
    gO, gP = ptycho.vjp(lin, w)
    rhs = solver.rdot(vO, gO) + (solver.rdot(vP, gP) if joint else 0.0)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


@pytest.mark.parametrize("metric", ["gauss", "poisson"])
@pytest.mark.parametrize("joint", [False, True])
def test_ggn_matches_dense_fd_jacobian(metric, joint):
    O, P, pos, y = tiny_problem(obj=(7, 7), probe=(3, 3), joint=joint, metric=metric)
    b = 1e-3
    lin = ptycho.linearize(O, P, pos, y, b, metric, joint)
    J = _fd_jacobian(O, P, pos, b, joint)
    G = J.T @ (lin.l2.ravel()[:, None] * J)
    vO = synth.random_complex(RNG, O.shape)
    vP = synth.random_complex(RNG, P.shape) if joint else None
    gO, gP = ptycho.ggn_vp(lin, vO, vP)
    dense = G @ _to_real(vO, vP)
    mf = _to_real(gO, gP)
    assert np.linalg.norm(mf - dense) <= 1e-7 * np.linalg.norm(dense)
    # symmetric and PSD
    assert np.allclose(G, G.T, atol=1e-7 * np.abs(G).max())
    ev = np.linalg.eigvalsh(0.5 * (G + G.T))
    assert ev.min() >= -1e-7 * ev.max()
    # exact diagonal equals diag(J^T diag(l'') J)
    dO, dP = ptycho.ggn_diag_exact(lin)
    n = O.size
    dg = np.diag(G)
    np.testing.assert_allclose(dO[..., 0].ravel(), dg[:n], rtol=1e-6, atol=1e-8 * dg.max())
    np.testing.assert_allclose(dO[..., 1].ravel(), dg[n:2 * n], rtol=1e-6, atol=1e-8 * dg.max())
    if joint:
        m = P.size
        np.testing.assert_allclose(dP[..., 0].ravel(), dg[2 * n:2 * n + m], rtol=1e-6, atol=1e-8 * dg.max())
        np.testing.assert_allclose(dP[..., 1].ravel(), dg[2 * n + m:], rtol=1e-6, atol=1e-8 * dg.max())


def test_ggn_symmetry_matrix_free():
    O, P, pos, y = tiny_problem(obj=(12, 11), probe=(4, 4))
    lin = ptycho.linearize(O, P, pos, y, 1e-3, "gauss", True)
    u = (synth.random_complex(RNG, O.shape), synth.random_complex(RNG, P.shape))
    v = (synth.random_complex(RNG, O.shape), synth.random_complex(RNG, P.shape))
    Gu, Gv = ptycho.ggn_vp(lin, *u), ptycho.ggn_vp(lin, *v)
    a = solver.rdot(v[0], Gu[0]) + solver.rdot(v[1], Gu[1])
    c = solver.rdot(u[0], Gv[0]) + solver.rdot(u[1], Gv[1])
    assert abs(a - c) <= 1e-11 * abs(a)


def test_null_vectors():
    O, P, pos, y = tiny_problem(obj=(12, 13), probe=(4, 5))
    lin = ptycho.linearize(O, P, pos, y, 1e-3, "gauss", True)
    scale = np.linalg.norm(ptycho.jvp(lin, synth.random_complex(RNG, O.shape), None))
    # global phase (SPR and BPR)
    assert np.linalg.norm(ptycho.jvp(lin, 1j * O, None)) < 1e-12 * scale
    assert np.linalg.norm(ptycho.jvp(lin, 1j * O, -1j * P)) < 1e-12 * scale
    # scale ambiguity O -> sO, P -> P/s
    assert np.linalg.norm(ptycho.jvp(lin, O, -P)) < 1e-12 * scale
    # linear phase ramps in x and y
    yy, xx = np.mgrid[0:O.shape[0], 0:O.shape[1]]
    my, mx = np.mgrid[0:P.shape[0], 0:P.shape[1]]
    assert np.linalg.norm(ptycho.jvp(lin, 1j * xx * O, -1j * mx * P)) < 1e-12 * scale
    assert np.linalg.norm(ptycho.jvp(lin, 1j * yy * O, -1j * my * P)) < 1e-12 * scale
    # the GGN annihilates them too
    gO, gP = ptycho.ggn_vp(lin, 1j * O, -1j * P)
    ref = ptycho.ggn_vp(lin, synth.random_complex(RNG, O.shape), None)[0]
    assert np.linalg.norm(gO) < 1e-11 * np.linalg.norm(ref)


def test_unilluminated_pixels_have_zero_products():
    O, P, pos, y = tiny_problem(obj=(12, 12), probe=(4, 4))
    pos = pos[pos[:, 0] < 6]
    y = y[: len(pos)]
    lin = ptycho.linearize(O, P, pos, y, 1e-3, "gauss", False)
    gO, _ = ptycho.gradient(lin)
    assert np.all(gO[11, :] == 0)


def test_ggn_equals_hessian_at_zero_residual():
    """Gaussian metric, noise-free data, at the truth: grad^2 f v = G v (eq:ggn_approximation)."""
    O, P, pos, _ = tiny_problem(obj=(10, 10), probe=(4, 4), noisy=False)
    b = 1e-3
    y = ptycho.intensity(O, P, pos, b)
    lin = ptycho.linearize(O, P, pos, y, b, "gauss", True)
    vO, vP = synth.random_complex(RNG, O.shape), synth.random_complex(RNG, P.shape)
    h = 1e-5
    gp = ptycho.gradient(ptycho.linearize(O + h * vO, P + h * vP, pos, y, b, "gauss", True))
    gm = ptycho.gradient(ptycho.linearize(O - h * vO, P - h * vP, pos, y, b, "gauss", True))
    HvO, HvP = (gp[0] - gm[0]) / (2 * h), (gp[1] - gm[1]) / (2 * h)
    GvO, GvP = ptycho.ggn_vp(lin, vO, vP)
    assert np.linalg.norm(GvO - HvO) <= 1e-6 * np.linalg.norm(GvO)
    assert np.linalg.norm(GvP - HvP) <= 1e-6 * np.linalg.norm(GvP)
    # and away from zero residual the two differ (the dropped term is real)
    yn = y * 1.5
    lin2 = ptycho.linearize(O, P, pos, yn, b, "gauss", True)
    gp = ptycho.gradient(ptycho.linearize(O + h * vO, P + h * vP, pos, yn, b, "gauss", True))
    gm = ptycho.gradient(ptycho.linearize(O - h * vO, P - h * vP, pos, yn, b, "gauss", True))
    G2 = ptycho.ggn_vp(lin2, vO, vP)[0]
    assert np.linalg.norm(G2 - (gp[0] - gm[0]) / (2 * h)) > 1e-3 * np.linalg.norm(G2)


# ---------------------------------------------------------------- diagonals
def test_paper_diagonal_follows_appendix_b_dense_route():
    """App. B under h ~ |psi_hat|^2: D = 1/4 sum_k S_k^T diag(P) C_k diag(P*) S_k with
    C_k = F^T diag(l'') F^*, built densely; its diagonal, doubled by the change to
    (Re, Im) coordinates, is the oracle's ``ggn_diag_paper``."""
    O, P, pos, y = tiny_problem(obj=(8, 9), probe=(3, 4), joint=True)
    lin = ptycho.linearize(O, P, pos, y, 1e-3, "gauss", True)
    My, Mx = P.shape
    Fm = np.kron(dft_matrix(My), dft_matrix(Mx))  # acts on row-major vectors
    N = O.size
    Dw = np.zeros((N, N), complex)
    for k, (r, c) in enumerate(pos):
        S = np.zeros((My * Mx, N))
        for i in range(My):
            for j in range(Mx):
                S[i * Mx + j, (r + i) * O.shape[1] + (c + j)] = 1.0
        C = Fm.T @ np.diag(lin.l2[k].ravel()) @ Fm.conj()
        assert np.allclose(np.diag(C), lin.l2[k].sum() / (My * Mx))  # circulant diagonal = trace/M
        Dw += 0.25 * S.T @ np.diag(P.ravel()) @ C @ np.diag(P.conj().ravel()) @ S
    dO, _ = ptycho.ggn_diag_paper(lin)
    np.testing.assert_allclose(dO[..., 0].ravel(), 2 * np.diag(Dw).real, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(dO[..., 1].ravel(), 2 * np.diag(Dw).real, rtol=1e-12, atol=1e-14)


def test_paper_diagonal_gaussian_is_half_overlap_map():
    O, P, pos, y = tiny_problem(obj=(10, 9), probe=(4, 3))
    lin = ptycho.linearize(O, P, pos, y, 1e-3, "gauss", False)
    dO, _ = ptycho.ggn_diag_paper(lin)
    ov = ptycho.illumination_overlap(P, pos, O.shape)
    np.testing.assert_allclose(dO[..., 0], 0.5 * ov, rtol=1e-12)


def test_paper_diagonal_is_exact_without_dropped_terms():
    """With |e| = 1 (b -> 0) the paper's diagonal equals the exact one minus the B-term."""
    O, P, pos, y = tiny_problem(obj=(9, 9), probe=(4, 4), joint=True)
    lin = ptycho.linearize(O, P, pos, y, 1e-14, "gauss", True)
    dO_a, dP_a = ptycho.ggn_diag_paper(lin)
    dO_e, dP_e = ptycho.ggn_diag_exact(lin)
    # the B-term has opposite signs in the Re and Im coordinates: their mean drops it
    np.testing.assert_allclose(dO_a[..., 0], 0.5 * (dO_e[..., 0] + dO_e[..., 1]), rtol=1e-9)
    np.testing.assert_allclose(dP_a[..., 0], 0.5 * (dP_e[..., 0] + dP_e[..., 1]), rtol=1e-9)


# ---------------------------------------------------------------- PCG and LM
def test_pcg_matches_dense_solve():
    O, P, pos, y = tiny_problem(obj=(6, 6), probe=(3, 3), joint=False)
    lin = ptycho.linearize(O, P, pos, y, 1e-3, "gauss", False)
    n = O.size
    lam = 0.3
    A = lambda v: ptycho.ggn_vp(lin, v.reshape(O.shape))[0].ravel() + lam * v
    cols = []
    for i in range(2 * n):
        e = np.zeros(n, complex)
        e[i % n] = 1.0 if i < n else 1j
        Ae = A(e)
        cols.append(np.concatenate([Ae.real, Ae.imag]))
    Ad = np.stack(cols, axis=1)
    g = ptycho.gradient(lin)[0].ravel()
    xd = np.linalg.solve(Ad, -np.concatenate([g.real, g.imag]))
    dg = solver.pack_diag(ptycho.ggn_diag_paper(lin)[0]) + lam
    pc = lambda r: r.real / dg[:, 0] + 1j * r.imag / dg[:, 1]
    for precond in (None, pc):
        res = solver.pcg(A, g, np.zeros(n, complex), precond, 1e-13, 4 * n)
        x = np.concatenate([res.x.real, res.x.imag])
        np.testing.assert_allclose(x, xd, rtol=1e-7, atol=1e-9 * np.abs(xd).max())
    # warm start from the solution: zero iterations needed
    res = solver.pcg(A, g, xd[:n] + 1j * xd[n:], None, 1e-6, 10)
    assert res.iters == 0


def test_pcg_energy_norm_error_decreases():
    O, P, pos, y = tiny_problem(obj=(8, 8), probe=(3, 3), joint=False)
    lin = ptycho.linearize(O, P, pos, y, 1e-3, "gauss", False)
    lam = 0.1
    A = lambda v: ptycho.ggn_vp(lin, v.reshape(O.shape))[0].ravel() + lam * v
    g = ptycho.gradient(lin)[0].ravel()
    xs = solver.pcg(A, g, np.zeros_like(g), None, 1e-14, 400).x
    errs = []
    for k in range(1, 12):
        x = solver.pcg(A, g, np.zeros_like(g), None, 0.0, k).x
        e = x - xs
        errs.append(solver.rdot(e, A(e)))
    assert all(b <= a * (1 + 1e-9) for a, b in zip(errs, errs[1:]))


@pytest.mark.parametrize("rho,mu_f,acc", [
    (0.9, 0.25, True), (0.76, 0.25, True), (0.75, 1.0, True), (0.5, 1.0, True),
    (0.25, 4.0, True), (0.2, 4.0, True), (1e-3, 4.0, True), (1e-4, 4.0, False),
    (-5.0, 4.0, False), (-math.inf, 4.0, False)])
def test_mu_update_branches(rho, mu_f, acc):
    p = solver.LMParams()
    mu, a = solver.mu_update(rho, 1.0, p)
    assert a == acc and mu == pytest.approx(mu_f)
    # floor
    mu, _ = solver.mu_update(0.9, 2e-8, p)
    assert mu == p.mu_min


def test_gain_ratio_degenerate():
    assert solver.gain_ratio(1.0, 0.0) == -math.inf
    assert solver.gain_ratio(1.0, -1.0) == -math.inf
    assert solver.gain_ratio(math.nan, 1.0) == -math.inf
    assert solver.gain_ratio(2.0, 4.0) == 0.5


def test_lm_all_rejects_keeps_iterate():
    pr = synth.make_small(3, obj_side=24, probe=(8, 8), n=3, step=5, photons=None, mode="object")
    y = ptycho.intensity(pr.O_true, pr.P_true, pr.pos, pr.background)
    p = solver.LMParams(retry_max=3)
    res = solver.lm_solve(pr.O_init, pr.P_true, pr.pos, y, pr.background, "gauss", False, p, 1,
                          loss_fn=lambda O_, P_: math.inf)
    assert len(res.history) == 3 and not any(h.accepted for h in res.history)
    assert np.array_equal(res.O, pr.O_init)
    assert res.history[-1].mu == pytest.approx(p.mu0 * p.kappa ** 2)
    # lambda follows mu ||grad ell|| on every retry
    lams = [h.lam for h in res.history]
    assert lams[1] == pytest.approx(4 * lams[0]) and lams[2] == pytest.approx(16 * lams[0])


def _aligned_error(O, O_true, mask):
    c = np.vdot(O[mask], O_true[mask])
    ph = c / abs(c)
    return np.linalg.norm(O[mask] * ph - O_true[mask]) / np.linalg.norm(O_true[mask])


def test_lm_noise_free_c0_converges_to_truth():
    pr = synth.make_c0()
    y = ptycho.intensity(pr.O_true, pr.P_true, pr.pos, pr.background)
    res = solver.lm_solve(pr.O_init, pr.P_true, pr.pos, y, pr.background, "gauss", False,
                          solver.LMParams(), 20)
    fs = res.f_per_iter + [res.f]
    assert all(b <= a for a, b in zip(fs, fs[1:]))       # accepted steps never increase f
    assert res.f < 1e-6 * fs[0]
    ov = ptycho.illumination_overlap(pr.P_true, pr.pos, pr.O_true.shape)
    mask = ov > 0.05 * ov.max()
    assert _aligned_error(res.O, pr.O_true, mask) < 1e-3
    # gain ratio tends to 1 near the zero-residual solution
    assert abs(res.history[-1].rho - 1.0) < 0.3


def test_lm_joint_with_scaling_and_jacobi_decreases():
    pr = synth.make_small(5, obj_side=32, probe=(8, 8), n=4, step=4, photons=1e3, mode="joint")
    rng = np.random.default_rng(5)
    h = ptycho.intensity(pr.O_true, pr.P_true, pr.pos, pr.background)
    y = synth.poisson_counts(rng, h)
    p = solver.LMParams(scaling=1, precond=1)
    res = solver.lm_solve(pr.O_init, pr.P_init, pr.pos, y, pr.background, "gauss", True, p, 8)
    assert res.f < 0.2 * res.f_per_iter[0]
    assert all(h.lam == h.mu for h in res.history)        # lambda = mu when D = Dg(G)


# ---------------------------------------------------------------- NEXT: surrogate metric, exact Jacobi
def test_surrogate_schedule_is_logarithmic_then_zero():
    p = solver.LMParams(surrogate_T=5, surrogate_s0=1.0)
    s = [solver.surrogate_sigma(t, p) for t in range(8)]
    assert s[0] == 1.0 and s[4] == pytest.approx(1e-6) and s[5:] == [0.0, 0.0, 0.0]
    ratios = [s[t + 1] / s[t] for t in range(4)]
    np.testing.assert_allclose(ratios, ratios[0], rtol=1e-12)        # evenly spaced in log
    assert solver.surrogate_sigma(0, solver.LMParams()) == 0.0          # off by default


def test_surrogate_iterations_work_on_shifted_background():
    """Outer iteration t linearises and judges its trial point on the metric with b + sigma_t
    (eq:expected_count_surrogate); the loss values are recomputed here from the forward model."""
    O, P, pos, y = tiny_problem(obj=(8, 8), probe=(4, 4), joint=False, metric="poisson")
    b = 1e-3
    p = solver.LMParams(surrogate_T=3, surrogate_s0=0.5, beta=0.9)
    res = solver.lm_solve(O * 0.9, P, pos, y, b, "poisson", False, p, 4)
    first = [h for h in res.history if h.t == 0][0]
    h0 = ptycho.intensity(O * 0.9, P, pos, b + 0.5)
    f0 = float(np.sum(h0 - y * np.log(h0)))                             # ell_p = zeta^2 - y log zeta^2
    assert first.f == pytest.approx(f0, rel=1e-12)
    assert res.f == pytest.approx(ptycho.loss(res.O, P, pos, y, b, "poisson"), rel=1e-12)
    plain = solver.lm_solve(O * 0.9, P, pos, y, b, "poisson", False, solver.LMParams(beta=0.9), 4)
    off = solver.lm_solve(O * 0.9, P, pos, y, b, "poisson", False, solver.LMParams(beta=0.9, surrogate_T=0), 4)
    assert [h.f_trial for h in plain.history] == [h.f_trial for h in off.history]


def test_exact_jacobi_first_step_matches_dense_construction():
    """precond 3: one PCG iteration from zero with M = diag(G) + lambda (D = I); the step and
    its trial loss are rebuilt here from the dense G of the JVP definition."""
    O, P, pos, y = tiny_problem(obj=(6, 6), probe=(3, 3), joint=False)
    b = 1e-3
    p = solver.LMParams(precond=3, cg_max=1, scaling=0)
    res = solver.lm_solve(O * 0.95, P, pos, y, b, "gauss", False, p, 1)
    a0 = res.history[0]
    lin = ptycho.linearize(O * 0.95, P, pos, y, b, "gauss", False)
    n = O.size
    # dense J from JVPs of the real unit vectors, G = J^T diag(l'') J
    cols = []
    for j in range(2 * n):
        e = np.zeros(2 * n)
        e[j] = 1.0
        cols.append(ptycho.jvp(lin, (e[:n] + 1j * e[n:]).reshape(O.shape), None).ravel())
    Jcols = np.stack(cols, axis=1)
    G = Jcols.T @ (lin.l2.ravel()[:, None] * Jcols)
    gO, _ = ptycho.gradient(lin)
    g = np.concatenate([gO.real.ravel(), gO.imag.ravel()])
    lam = a0.lam
    d = np.maximum(np.diag(G), 1e-6 * np.diag(G).max())
    m = d + lam
    r0 = -g
    z = r0 / m
    Az = G @ z + lam * z
    alpha = (r0 @ z) / (z @ Az)
    step = alpha * z
    Ot = O * 0.95 + (step[:n] + 1j * step[n:]).reshape(O.shape)
    assert a0.f_trial == pytest.approx(ptycho.loss(Ot, P, pos, y, b, "gauss"), rel=1e-9)


# ---------------------------------------------------------------- NEXT: projected LM (constrained BPR)
def test_projection_satisfies_the_variational_inequality():
    """Pi_Z(x) is the Euclidean projection on {|z| <= m} iff Re(conj(x - Pi x)(y - Pi x)) <= 0
    for every feasible y; checked on random points inside and outside and random feasible y."""
    rng = np.random.default_rng(3)
    p = solver.LMParams(o_max=1.0, p_max=2.5)
    O = synth.random_complex(rng, (40,)) * 1.2
    P = synth.random_complex(rng, (40,)) * 3.0
    Oc, Pc = solver.project(O, P, p)
    assert np.all(np.abs(Oc) <= 1.0 + 1e-15) and np.all(np.abs(Pc) <= 2.5 + 1e-15)
    inside = np.abs(O) <= 1.0
    assert np.array_equal(Oc[inside], O[inside])
    for x, px, m in ((O, Oc, 1.0), (P, Pc, 2.5)):
        for _ in range(50):
            yv = m * np.sqrt(rng.uniform(size=x.shape)) * np.exp(2j * np.pi * rng.uniform(size=x.shape))
            assert np.all(np.real(np.conj(x - px) * (yv - px)) <= 1e-12)


def test_projected_lm_with_inactive_constraints_is_plain_lm():
    O, P, pos, y = tiny_problem(obj=(9, 9), probe=(4, 4), joint=True)
    b = 1e-3
    base = dict(scaling=1, precond=1)
    plain = solver.lm_solve(O * 0.9, P * 1.1, pos, y, b, "gauss", True, solver.LMParams(**base), 4)
    proj = solver.lm_solve(O * 0.9, P * 1.1, pos, y, b, "gauss", True,
                           solver.LMParams(project=True, o_max=1e30, p_max=1e30, **base), 4)
    steps = [h.ls for h in proj.history if h.accepted]
    assert steps and all(br == "direction" and a == 1.0 for br, a in steps)
    np.testing.assert_allclose(proj.O, plain.O, rtol=0, atol=1e-14)
    np.testing.assert_allclose(proj.P, plain.P, rtol=0, atol=1e-14)


def test_projected_lm_stays_feasible_and_descends():
    """BPR with |O| <= 1: every accepted iterate of the plug-in is feasible and satisfies the
    Armijo decrease, so the loss never increases (eq:armijo_criterion)."""
    pr = synth.make_small(6, obj_side=32, probe=(8, 8), n=5, step=4, photons=1e3, mode="joint")
    rng = np.random.default_rng(6)
    O_true = pr.O_true / np.abs(pr.O_true).max()          # truth on the boundary of Z
    y = synth.poisson_counts(rng, ptycho.intensity(O_true, pr.P_true, pr.pos, pr.background))
    p = solver.LMParams(scaling=1, precond=1, project=True)
    res = solver.lm_solve(pr.O_init, pr.P_init, pr.pos, y, pr.background, "gauss", True, p, 8)
    assert np.abs(res.O).max() <= 1.0 + 1e-12
    f = res.f_per_iter + [res.f]
    assert all(f[i + 1] <= f[i] for i in range(len(f) - 1))
    assert res.f < 0.5 * f[0]


# ---------------------------------------------------------------- NEXT: alternating LM (BPR)
def _accepted_of(history, block, t=0):
    acc = [h for h in history if h.block == block and h.t == t and h.accepted]
    return acc[0] if acc else None


def _dense_block_step(O, P, pos, y, b, block, lam):
    """-(J_B^T diag(l'') J_B + lam I)^{-1} J_B^T l' for one block B of the variables, with J_B
    from central differences of the forward model and l', l'' of the Gaussian metric (pinned
    by their own finite-difference test)."""
    J = _fd_jacobian(O, P, pos, b, True)
    n_o = 2 * O.size
    JB = J[:, :n_o] if block == "O" else J[:, n_o:]
    zeta = ptycho.magnitude(O, P, pos, b).ravel()
    l1 = ptycho.ell_d1(zeta, y.ravel(), "gauss")
    l2 = ptycho.ell_d2(zeta, y.ravel(), "gauss")
    G = JB.T @ (l2[:, None] * JB)
    step = np.linalg.solve(G + lam * np.eye(G.shape[0]), -(JB.T @ l1))
    m = step.size // 2
    shape = O.shape if block == "O" else P.shape
    return (step[:m] + 1j * step[m:]).reshape(shape)


def test_alternating_substeps_match_dense_block_solves():
    """alg:alt_LM_ptycho: the object update solves with the object block of G at (O_t, P_t), the
    probe update with the probe block at (O_{t+1}, P_t).  PCG is run to convergence and each
    accepted step is rebuilt from a dense finite-difference Jacobian of that block alone."""
    O, P, pos, y = tiny_problem(joint=True)
    b = 1e-3
    O0, P0 = O * 0.95, P * 1.05
    p = solver.LMParams(alternate=True, beta=1e-13, cg_max=400, warm_start=False)
    res = solver.lm_solve(O0, P0, pos, y, b, "gauss", True, p, 1)
    assert [h.block for h in res.history][0] == "O" and res.history[-1].block == "P"
    aO, aP = _accepted_of(res.history, "O"), _accepted_of(res.history, "P")
    assert aO is not None and aP is not None
    O1 = O0 + _dense_block_step(O0, P0, pos, y, b, "O", aO.lam)
    assert aO.f_trial == pytest.approx(ptycho.loss(O1, P0, pos, y, b, "gauss"), rel=1e-7)
    np.testing.assert_allclose(res.O, O1, rtol=0, atol=1e-6 * np.abs(O1).max())
    P1 = P0 + _dense_block_step(res.O, P0, pos, y, b, "P", aP.lam)
    assert aP.f_trial == pytest.approx(ptycho.loss(res.O, P1, pos, y, b, "gauss"), rel=1e-7)
    np.testing.assert_allclose(res.P, P1, rtol=0, atol=1e-6 * np.abs(P1).max())
    # the probe update starts at f(O_{t+1}, P_t), the object's trial value
    assert aP.f == pytest.approx(aO.f_trial, rel=1e-12)


def test_alternating_object_substep_is_the_object_only_step():
    """With the probe fixed, the object sub-step of a joint problem is the LM step of the
    object-only problem (SPR form of eq:cdp): same damping, diagonal D, Jacobi preconditioner,
    PCG iterations and trial values."""
    O, P, pos, y = tiny_problem(seed=11, joint=True)
    b = 1e-3
    kw = dict(scaling=1, precond=1)
    alt = solver.lm_solve(O * 0.9, P, pos, y, b, "gauss", True, solver.LMParams(alternate=True, **kw), 1)
    obj = solver.lm_solve(O * 0.9, P, pos, y, b, "gauss", False, solver.LMParams(**kw), 1)
    a = [h for h in alt.history if h.block == "O"]
    assert len(a) == len(obj.history)
    for u, v in zip(a, obj.history):
        assert (u.cg_iters, u.accepted) == (v.cg_iters, v.accepted)
        for name in ("f", "f_trial", "mu", "lam", "eta", "rho"):
            assert getattr(u, name) == pytest.approx(getattr(v, name), rel=1e-10, abs=1e-300), name
    np.testing.assert_allclose(alt.O, obj.O, rtol=0, atol=1e-12)


def test_alternating_probe_substep_mirrors_object_step():
    """With one scan position and equal object and probe shapes the exit wave P S O = P O is
    symmetric in O and P, so the probe sub-step (object fixed) is the object-only LM step of the
    problem with the two swapped -- with D = Dg(G) and the Jacobi preconditioner, whose probe
    part (eq:ggn_joint_diag) then mirrors the object part."""
    rng = np.random.default_rng(21)
    O = synth.random_complex(rng, (6, 6)) * 0.5 + 0.8
    P = synth.random_complex(rng, (6, 6))
    pos = np.zeros((1, 2), dtype=np.int32)
    b = 1e-3
    y = synth.poisson_counts(rng, 50 * ptycho.intensity(O, P, pos, b)) / 50
    kw = dict(scaling=1, precond=1)
    alt = solver.lm_solve(O * 0.9, P * 1.1, pos, y, b, "gauss", True, solver.LMParams(alternate=True, **kw), 1)
    O1 = alt.O                                      # the probe sub-step leaves the object as it is
    swapped = solver.lm_solve(P * 1.1, O1, pos, y, b, "gauss", False, solver.LMParams(**kw), 1)
    a = [h for h in alt.history if h.block == "P"]
    assert len(a) == len(swapped.history) and any(h.accepted for h in a)
    for u, v in zip(a, swapped.history):
        assert u.cg_iters == v.cg_iters
        for name in ("f", "f_trial", "lam", "rho"):
            assert getattr(u, name) == pytest.approx(getattr(v, name), rel=1e-9), name
    np.testing.assert_allclose(alt.P, swapped.O, rtol=0, atol=1e-12)


def test_alternating_blocks_keep_their_own_damping_and_descend():
    """Reading: each block carries its own mu from one outer iteration to the next, and every
    accepted sub-step lowers f (rho > rho_min > 0 with a positive predicted reduction)."""
    pr = synth.make_small(8, obj_side=32, probe=(8, 8), n=4, step=4, photons=1e3, mode="joint")
    rng = np.random.default_rng(8)
    y = synth.poisson_counts(rng, ptycho.intensity(pr.O_true, pr.P_true, pr.pos, pr.background))
    p = solver.LMParams(alternate=True, scaling=1, precond=1)
    res = solver.lm_solve(pr.O_init, pr.P_init, pr.pos, y, pr.background, "gauss", True, p, 5)
    for blk in ("O", "P"):
        seq = [h for h in res.history if h.block == blk]
        assert {h.t for h in seq} == set(range(5))
        assert seq[0].mu == p.mu0
        for u, v in zip(seq, seq[1:]):
            assert v.mu == solver.mu_update(u.rho, u.mu, p)[0]
    for h in res.history:
        if h.accepted:
            assert h.f_trial < h.f
    f = res.f_per_iter + [res.f]
    assert all(f[i + 1] <= f[i] for i in range(len(f) - 1))
    assert res.f < 0.5 * f[0]


def test_alternating_needs_joint_problem():
    O, P, pos, y = tiny_problem(joint=False)
    with pytest.raises(ValueError):
        solver.lm_solve(O, P, pos, y, 1e-3, "gauss", False, solver.LMParams(alternate=True), 1)


# ---------------------------------------------------------------- NEXT: intensity-based GGN (App. C)
def _fd_jacobian_h(O, P, pos, b, joint):
    """Dense J_h = d h / d z by central differences of the intensity forward model alone."""
    h = 1e-6
    cols = []
    targets = [("O", O.shape)] + ([("P", P.shape)] if joint else [])
    for name, shp in targets:
        n = shp[0] * shp[1]
        for part in (1.0, 1j):
            for i in range(n):
                d = np.zeros(n, complex)
                d[i] = part * h
                d = d.reshape(shp)
                if name == "O":
                    hp, hm = ptycho.intensity(O + d, P, pos, b), ptycho.intensity(O - d, P, pos, b)
                else:
                    hp, hm = ptycho.intensity(O, P + d, pos, b), ptycho.intensity(O, P - d, pos, b)
                cols.append(((hp - hm) / (2 * h)).ravel())
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("metric", ["gauss", "poisson"])
def test_intensity_metric_matches_magnitude_metric_and_its_fd_hessian(metric):
    rng = np.random.default_rng(3)
    h = rng.uniform(0.2, 3.0, 50)
    y = rng.uniform(0.1, 4.0, 50)
    # the same metric in h and in zeta = sqrt(h) (eq:error_metric_magnitude)
    np.testing.assert_allclose(ptycho.big_ell(h, y, metric), ptycho.ell(np.sqrt(h), y, metric), rtol=1e-12)
    e = 1e-4
    fd2 = (ptycho.big_ell(h + e, y, metric) - 2 * ptycho.big_ell(h, y, metric) + ptycho.big_ell(h - e, y, metric)) / e**2
    np.testing.assert_allclose(ptycho.big_ell_d2(h, y, metric), fd2, rtol=1e-5)


@pytest.mark.parametrize("metric", ["gauss", "poisson"])
@pytest.mark.parametrize("joint", [False, True])
def test_intensity_ggn_matches_dense_fd_construction(metric, joint):
    """G^L v (eq:ggn_intensity) against J_h^T diag(L''(h)) J_h with J_h by finite differences of
    the intensity model and L'' by finite differences of the metric in h; the gradient is that
    of the magnitude-based linearisation."""
    O, P, pos, y = tiny_problem(joint=joint, metric=metric)
    b = 1e-3
    lin = ptycho.linearize(O, P, pos, y, b, metric, joint, ggn="intensity")
    Jh = _fd_jacobian_h(O, P, pos, b, joint)
    hh = ptycho.intensity(O, P, pos, b).ravel()
    e = 1e-5 * hh
    yy = y.ravel()
    d2 = (ptycho.big_ell(hh + e, yy, metric) - 2 * ptycho.big_ell(hh, yy, metric)
          + ptycho.big_ell(hh - e, yy, metric)) / e**2
    G = Jh.T @ (d2[:, None] * Jh)
    vO = synth.random_complex(RNG, O.shape)
    vP = synth.random_complex(RNG, P.shape) if joint else None
    gO, gP = ptycho.ggn_vp(lin, vO, vP)
    mf = _to_real(gO, gP)
    dense = G @ _to_real(vO, vP)
    assert np.linalg.norm(mf - dense) <= 1e-5 * np.linalg.norm(dense)
    mag = ptycho.linearize(O, P, pos, y, b, metric, joint)
    for a, c in zip(ptycho.gradient(lin), ptycho.gradient(mag)):
        if a is not None:
            np.testing.assert_array_equal(a, c)


def test_intensity_ggn_equals_magnitude_ggn_at_zero_gaussian_residual():
    """With y = h the Gaussian weights coincide: 4 h L''(h) = sqrt(y) / zeta = 1 = ell''."""
    O, P, pos, _ = tiny_problem(joint=True, noisy=False)
    b = 1e-3
    y = ptycho.intensity(O, P, pos, b)
    li = ptycho.linearize(O, P, pos, y, b, "gauss", True, ggn="intensity")
    lm = ptycho.linearize(O, P, pos, y, b, "gauss", True)
    vO, vP = synth.random_complex(RNG, O.shape), synth.random_complex(RNG, P.shape)
    for a, c in zip(ptycho.ggn_vp(li, vO, vP), ptycho.ggn_vp(lm, vO, vP)):
        np.testing.assert_allclose(a, c, rtol=1e-12, atol=1e-12)


def test_magnitude_ggn_lm_converges_faster_than_intensity_ggn_lm():
    """The qualitative claim of Fig. 1 (SPR, known probe, Gaussian metric): LM built on the
    magnitude-based GGN reaches a lower loss in the same number of iterations than LM built on
    the intensity-based GGN, on noise-free and on Poisson data."""
    pr = synth.make_small(5, obj_side=32, probe=(8, 8), n=4, step=4, photons=1e3, mode="object")
    rng = np.random.default_rng(5)
    h = ptycho.intensity(pr.O_true, pr.P_true, pr.pos, pr.background)
    for y in (h, synth.poisson_counts(rng, h)):
        f = {}
        for ggn in ("magnitude", "intensity"):
            res = solver.lm_solve(pr.O_init, pr.P_true, pr.pos, y, pr.background, "gauss", False,
                                  solver.LMParams(ggn=ggn), 15)
            f[ggn] = res.f
        assert f["magnitude"] < 0.8 * f["intensity"], f


# ---------------------------------------------------------------- NEXT: stochastic diagonal
def test_splitmix64_first_outputs():
    """The first three outputs of SplitMix64 seeded with 0, as published with the generator."""
    out = ptycho.splitmix64(0, np.arange(1, 4, dtype=np.uint64))
    assert [int(x) for x in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_rademacher_signs_are_balanced_and_uncorrelated():
    n = np.arange(1, 1_000_001, dtype=np.uint64)
    r = ptycho.rademacher(12345, n)
    assert set(np.unique(r)) == {-1.0, 1.0}
    assert abs(r.mean()) < 4e-3                       # 4 sigma of a fair coin over 1e6 draws
    assert abs(np.mean(r[1:] * r[:-1])) < 4e-3        # neighbouring counters independent


def _tiny_joint(metric="gauss"):
    rng = np.random.default_rng(31)
    O = synth.random_complex(rng, (4, 4)) * 0.5 + 0.8
    P = synth.random_complex(rng, (2, 2))
    pos = np.array([[0, 0], [0, 2], [2, 1]], dtype=np.int32)
    y = synth.poisson_counts(rng, 30 * ptycho.intensity(O, P, pos, 1e-3)) / 30
    return ptycho.linearize(O * 0.9, P, pos, y, 1e-3, metric, True)


@pytest.mark.parametrize("metric", ["gauss", "poisson"])
def test_stochastic_diagonal_over_every_sign_pattern_is_exact(metric):
    """E over the uniform distribution on {+-1}^m is the average over all 2^m patterns, so the
    estimator averaged over every pattern must equal the diagonal of G exactly."""
    lin = _tiny_joint(metric)
    m = lin.zeta.size
    assert m <= 14
    bits = (np.arange(2 ** m)[:, None] >> np.arange(m)[None, :]) & 1
    r = (1.0 - 2.0 * bits).reshape((2 ** m,) + lin.zeta.shape)
    sO, sP = ptycho.ggn_diag_stochastic(lin, r)
    eO, eP = ptycho.ggn_diag_exact(lin)
    np.testing.assert_allclose(sO, eO, rtol=1e-10, atol=1e-12 * np.abs(eO).max())
    np.testing.assert_allclose(sP, eP, rtol=1e-10, atol=1e-12 * np.abs(eP).max())


def test_stochastic_diagonal_converges_with_generated_draws():
    """With the generator's sign fields the estimate approaches the exact diagonal as the draws
    grow (relative L2 error shrinking like 1/sqrt(S))."""
    O, P, pos, y = tiny_problem(joint=True)
    lin = ptycho.linearize(O, P, pos, y, 1e-3, "gauss", True)
    eO, eP = ptycho.ggn_diag_exact(lin)
    exact = np.concatenate([eO.ravel(), eP.ravel()])
    errs = []
    for S in (16, 1024):
        r = np.stack([ptycho.rademacher_field(lin, 7, d) for d in range(S)])
        sO, sP = ptycho.ggn_diag_stochastic(lin, r)
        est = np.concatenate([sO.ravel(), sP.ravel()])
        errs.append(np.linalg.norm(est - exact) / np.linalg.norm(exact))
    assert errs[1] < 0.06 and errs[1] < 0.25 * errs[0], errs


def test_lm_with_stochastic_jacobi_decreases():
    pr = synth.make_small(5, obj_side=32, probe=(8, 8), n=4, step=4, photons=1e3, mode="joint")
    rng = np.random.default_rng(5)
    y = synth.poisson_counts(rng, ptycho.intensity(pr.O_true, pr.P_true, pr.pos, pr.background))
    p = solver.LMParams(scaling=1, precond=4, stoch_samples=16, stoch_seed=3)
    res = solver.lm_solve(pr.O_init, pr.P_init, pr.pos, y, pr.background, "gauss", True, p, 6)
    assert res.f < 0.3 * res.f_per_iter[0]
