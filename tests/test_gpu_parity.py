"""GPU parity: every C-ABI product against the FP64 oracle on identical inputs.

Inputs come from ``synth``; both sides see the same complex64 / float32
values (the oracle upcasts them to FP64).  Error measure: relative L2 norm over
the whole output array, ||x_gpu - x_oracle|| / ||x_oracle||; bar 1e-5 for the
forward model and the GGN-vector product (and the other linear products).
Sizes span several tiles per workgroup, multi-position segments and ragged
segment tails; rectangular probes are included.
"""
import math

import numpy as np
import pytest

import synth
from oracle import ptycho, solver

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - collected on CPU hosts
    pytest.skip("no GPU", allow_module_level=True)
import paper_2103_01767_amd as pt  # noqa: E402

DEV = torch.device("cuda:0")
TOL = 1e-5


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128 if np.iscomplexobj(a) else np.float64)
    b = np.asarray(b, dtype=a.dtype)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def c64(x):
    return np.asarray(x, dtype=np.complex64)


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def raster(n_y, n_x, step, probe, jitter, seed):
    rng = np.random.default_rng(seed)
    my, mx = probe
    base_y = 1 + step * np.arange(n_y)
    base_x = 1 + step * np.arange(n_x)
    ry, rx = np.meshgrid(base_y, base_x, indexing="ij")
    pos = np.stack([ry.ravel(), rx.ravel()], 1)
    pos = pos + rng.integers(-jitter, jitter + 1, size=pos.shape)
    pos = np.maximum(pos, 0)
    ny = int(pos[:, 0].max()) + my + 3
    nx = int(pos[:, 1].max()) + mx + 2
    return pos.astype(np.int32), (ny, nx)


def make_case(probe, n_y, n_x, step, metric="gauss", joint=True, seed=0, photons=2e3):
    rng = np.random.default_rng(seed)
    pos, (ny, nx) = raster(n_y, n_x, step, probe, 1, seed)
    O = c64(synth.make_object(rng, max(ny, nx), amp=(0.7, 1.0), phase=(-math.pi, math.pi),
                              phase_sigma=2.0, phase_source="gaussian")[:ny, :nx])
    side = max(probe)
    P = synth.make_probe_fresnel(rng, side, side * 0.35, 3.0)[:probe[0], :probe[1]]
    P = c64(synth.scale_probe_to_photons(P, O, photons))
    O64, P64 = O.astype(np.complex128), P.astype(np.complex128)
    h = ptycho.intensity(O64, P64, pos, 1e-8)
    y = synth.poisson_counts(rng, h).astype(np.float32)
    return dict(O=O, P=P, pos=pos, y=y, O64=O64, P64=P64, y64=y.astype(np.float64), metric=metric,
                joint=joint, rng=rng)


def problem(case):
    return pt.Problem(case["O"].shape, case["P"].shape, case["pos"], metric=case["metric"],
                      mode="joint" if case["joint"] else "object", background=1e-8, device=DEV)


SHAPES = [(16, 16), (32, 32), (64, 64), (128, 128), (16, 64), (64, 32), (128, 32), (32, 128), (256, 256),
          (48, 48), (96, 96)]


@pytest.mark.parametrize("probe", SHAPES, ids=lambda p: "%dx%d" % p)
def test_forward_and_loss(probe):
    print("case forward", probe, flush=True)
    n = 6 if probe[0] * probe[1] >= 4096 else 7
    case = make_case(probe, n, n + 1, max(probe) // 4, seed=sum(probe))
    prob = problem(case)
    O, P, y = to_dev(case["O"]), to_dev(case["P"]), to_dev(case["y"])
    zeta = host(prob.forward(O, P))
    ref = ptycho.magnitude(case["O64"], case["P64"], case["pos"], 1e-8)
    assert rel(zeta, ref) < TOL
    for metric in ("gauss", "poisson"):
        case["metric"] = metric
        prob = problem(case)
        f, r = prob.loss(O, P, y, residual=True)
        lin = ptycho.linearize(case["O64"], case["P64"], case["pos"], case["y64"], 1e-8, metric, True)
        assert abs(float(host(f)[0]) - lin.f) <= 1e-5 * abs(lin.f)
        assert rel(host(r), lin.l1) < 1e-5


@pytest.mark.parametrize("metric", ["gauss", "poisson"])
@pytest.mark.parametrize("joint", [False, True])
@pytest.mark.parametrize("probe", [(16, 16), (64, 64), (128, 128), (32, 64), (256, 256), (48, 48), (96, 96)],
                         ids=lambda p: "%dx%d" % p)
def test_linear_products(probe, joint, metric):
    print("case products", probe, joint, metric, flush=True)
    case = make_case(probe, 5, 6, max(probe) // 4, metric=metric, joint=joint, seed=3 + probe[0])
    prob = problem(case)
    O, P, y = to_dev(case["O"]), to_dev(case["P"]), to_dev(case["y"])
    lin = ptycho.linearize(case["O64"], case["P64"], case["pos"], case["y64"], 1e-8, metric, joint)
    f, gO, gP = prob.linearize(O, P, y)
    f = host(f)
    assert abs(f[0] - lin.f) <= 1e-5 * abs(lin.f)
    assert abs(f[1] - np.sum(lin.l1 ** 2)) <= 1e-5 * np.sum(lin.l1 ** 2)
    rgO, rgP = ptycho.gradient(lin)
    assert rel(host(gO), rgO) < TOL
    if joint:
        assert rel(host(gP), rgP) < TOL
    rng = np.random.default_rng(11)
    vO = c64(synth.random_complex(rng, case["O"].shape))
    vP = c64(synth.random_complex(rng, case["P"].shape)) if joint else None
    vOd, vPd = to_dev(vO), (to_dev(vP) if joint else None)
    vO64 = vO.astype(np.complex128)
    vP64 = vP.astype(np.complex128) if joint else None
    # JVP
    assert rel(host(prob.jvp(vOd, vPd)), ptycho.jvp(lin, vO64, vP64)) < TOL
    # VJP
    w = rng.standard_normal(prob.meas_shape).astype(np.float32)
    oO, oP = prob.vjp(to_dev(w))
    rO, rP = ptycho.vjp(lin, w.astype(np.float64))
    assert rel(host(oO), rO) < TOL
    if joint:
        assert rel(host(oP), rP) < TOL
    # GGN-vector product, plain and damped with a diagonal.  Poisson weights l'' = 2 + 2y/h at
    # pixels with y >= 1 and h << 1 multiply the single-precision error of the far field; the
    # linearisation refines the few pixels of weight above 1e4 in FP64, which holds the 256 x 256
    # case at 0.03 photons per pixel to the bar like every other.
    GO, GP = ptycho.ggn_vp(lin, vO64, vP64)
    oO, oP = prob.ggn_vp(vOd, vPd)
    assert rel(host(oO), GO) < TOL
    if joint:
        assert rel(host(oP), GP) < TOL
    lam = 0.37
    dO = rng.uniform(0.5, 2.0, case["O"].shape + (2,)).astype(np.float32)
    dP = rng.uniform(0.5, 2.0, case["P"].shape + (2,)).astype(np.float32) if joint else None
    oO, oP = prob.ggn_vp(vOd, vPd, lam=lam, dO=to_dev(dO), dP=to_dev(dP) if joint else None)
    refO = GO + lam * solver.apply_diag(dO.reshape(-1, 2).astype(np.float64), vO64.ravel()).reshape(GO.shape)
    assert rel(host(oO), refO) < TOL
    if joint:
        refP = GP + lam * solver.apply_diag(dP.reshape(-1, 2).astype(np.float64), vP64.ravel()).reshape(GP.shape)
        assert rel(host(oP), refP) < TOL
    oO, _ = prob.ggn_vp(vOd, vPd, lam=lam)
    assert rel(host(oO), GO + lam * vO64) < TOL
    # diagonals
    dOg, dPg = prob.diag(exact=False)
    aO, aP = ptycho.ggn_diag_paper(lin)
    assert rel(host(dOg), aO) < TOL
    if joint:
        assert rel(host(dPg), aP) < TOL
    dOg, dPg = prob.diag(exact=True)
    eO, eP = ptycho.ggn_diag_exact(lin)
    assert rel(host(dOg), eO) < 2 * TOL
    if joint:
        assert rel(host(dPg), eP) < 2 * TOL


def test_ggn_null_vector_and_determinism():
    case = make_case((64, 64), 5, 5, 16, joint=True, seed=21)
    prob = problem(case)
    O, P, y = to_dev(case["O"]), to_dev(case["P"]), to_dev(case["y"])
    prob.linearize(O, P, y)
    rng = np.random.default_rng(2)
    vO = to_dev(c64(synth.random_complex(rng, case["O"].shape)))
    vP = to_dev(c64(synth.random_complex(rng, case["P"].shape)))
    a = prob.ggn_vp(vO, vP)
    b = prob.ggn_vp(vO, vP)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])       # fixed-order sums
    nO, nP = prob.ggn_vp(1j * O, -1j * P)                             # global phase
    scale = float(torch.linalg.vector_norm(a[0])) / float(torch.linalg.vector_norm(vO))
    assert float(torch.linalg.vector_norm(nO)) < 1e-5 * scale * float(torch.linalg.vector_norm(O))


@pytest.mark.parametrize("probe,n,step", [((128, 128), 17, 8), ((256, 256), 17, 8), ((48, 48), 48, 4),
                                          ((96, 96), 23, 8)], ids=lambda p: "%dx%d" % p if isinstance(p, tuple) else str(p))
def test_segments_longer_than_one_position(probe, n, step):
    """K > segments: each segment walks several positions (strip read-modify-write)."""
    print("case segments", probe, n, step, flush=True)
    case = make_case(probe, n, n + 2, step, joint=True, seed=5)
    prob = problem(case)
    O, P, y = to_dev(case["O"]), to_dev(case["P"]), to_dev(case["y"])
    lin = ptycho.linearize(case["O64"], case["P64"], case["pos"], case["y64"], 1e-8, "gauss", True)
    prob.linearize(O, P, y)
    rng = np.random.default_rng(8)
    vO = c64(synth.random_complex(rng, case["O"].shape))
    vP = c64(synth.random_complex(rng, case["P"].shape))
    oO, oP = prob.ggn_vp(to_dev(vO), to_dev(vP))
    GO, GP = ptycho.ggn_vp(lin, vO.astype(np.complex128), vP.astype(np.complex128))
    assert rel(host(oO), GO) < TOL and rel(host(oP), GP) < TOL


def test_invalid_arguments():
    case = make_case((16, 16), 3, 3, 4, seed=9)
    bad = case["pos"].copy()
    bad[1, 0] = case["O"].shape[0]
    with pytest.raises(pt.PtlmError) as e:
        pt.Problem(case["O"].shape, case["P"].shape, bad, device=DEV)
    assert e.value.status == pt.PTLM_EINVAL
    with pytest.raises(pt.PtlmError):
        pt.Problem(case["O"].shape, (48, 16), case["pos"], device=DEV)
    with pytest.raises(pt.PtlmError):  # 256 only as a square probe
        pt.Problem((300, 300), (256, 128), np.zeros((1, 2), np.int32), device=DEV)
    prob = problem(case)
    with pytest.raises(TypeError):
        prob.forward(to_dev(case["O"]).to(torch.complex128), to_dev(case["P"]))


@pytest.mark.parametrize("probe,n,step", [((64, 64), 20, 6), ((32, 32), 30, 4)], ids=["64x64", "32x32"])
def test_autotuned_segmentation_keeps_products(probe, n, step):
    """The autotuner only changes how positions are cut into segments and which transform and
    tile grouping the product uses: products stay at parity."""
    print("case autotune", probe, flush=True)
    case = make_case(probe, n, n, step, joint=True, seed=31)
    prob = problem(case)
    O, P, y = to_dev(case["O"]), to_dev(case["P"]), to_dev(case["y"])
    lin = ptycho.linearize(case["O64"], case["P64"], case["pos"], case["y64"], 1e-8, "gauss", True)
    prob.linearize(O, P, y)
    scale, ms, xf = prob.autotune(reps=3)
    print("autotune scale", scale, "transform", xf, "ms", ms)
    assert scale in (0.5, 1.0, 2.0) and len(ms) == 9
    fft, mfma, wide = ms[0:3], ms[3:6], ms[6:9]
    assert all(m > 0 for m in fft) and all(m > 0 for m in wide)  # both shapes have the wide grouping
    assert all(m > 0 for m in mfma) if probe == (32, 32) else all(m == -1 for m in mfma)
    best = min((m, name) for name, row in zip(pt.TRANSFORMS, (fft, mfma, wide)) for m in row if m > 0)
    assert xf == best[1] and min(ms[3 * pt.TRANSFORMS.index(xf):][:3]) == best[0]
    rng = np.random.default_rng(4)
    vO = c64(synth.random_complex(rng, case["O"].shape))
    vP = c64(synth.random_complex(rng, case["P"].shape))
    oO, oP = prob.ggn_vp(to_dev(vO), to_dev(vP))
    GO, GP = ptycho.ggn_vp(lin, vO.astype(np.complex128), vP.astype(np.complex128))
    assert rel(host(oO), GO) < TOL and rel(host(oP), GP) < TOL
    f, gO, gP = prob.linearize(O, P, y)
    rgO, rgP = ptycho.gradient(lin)
    assert rel(host(gO), rgO) < TOL and rel(host(gP), rgP) < TOL


@pytest.mark.parametrize("metric", ["gauss", "poisson"])
@pytest.mark.parametrize("probe,joint", [((16, 16), True), ((64, 64), False), ((128, 128), True), ((48, 48), True),
                                         ((256, 256), True)], ids=lambda p: "%dx%d" % p if isinstance(p, tuple) else str(p))
def test_intensity_ggn_products(probe, joint, metric):
    """Intensity-based GGN (eq:ggn_intensity, App. C): the same f, gradient, JVP and VJP as the
    magnitude-based problem, the GGN-vector product and both diagonals with the weight
    4 zeta^2 L''(zeta^2) (zero-count pixels included: their weight vanishes)."""
    print("case intensity ggn", probe, joint, metric, flush=True)
    case = make_case(probe, 5, 6, max(probe) // 4, metric=metric, joint=joint, seed=5 + probe[0])
    prob = pt.Problem(case["O"].shape, case["P"].shape, case["pos"], metric=metric,
                      mode="joint" if joint else "object", background=1e-8, device=DEV, ggn="intensity")
    O, P, y = to_dev(case["O"]), to_dev(case["P"]), to_dev(case["y"])
    assert np.any(case["y"] == 0)
    lin = ptycho.linearize(case["O64"], case["P64"], case["pos"], case["y64"], 1e-8, metric, joint, ggn="intensity")
    f, gO, gP = prob.linearize(O, P, y)
    f = host(f)
    assert abs(f[0] - lin.f) <= 1e-5 * abs(lin.f)
    rgO, rgP = ptycho.gradient(lin)
    assert rel(host(gO), rgO) < TOL
    if joint:
        assert rel(host(gP), rgP) < TOL
    rng = np.random.default_rng(12)
    vO = c64(synth.random_complex(rng, case["O"].shape))
    vP = c64(synth.random_complex(rng, case["P"].shape)) if joint else None
    vOd, vPd = to_dev(vO), (to_dev(vP) if joint else None)
    vO64 = vO.astype(np.complex128)
    vP64 = vP.astype(np.complex128) if joint else None
    assert rel(host(prob.jvp(vOd, vPd)), ptycho.jvp(lin, vO64, vP64)) < TOL
    w = rng.standard_normal(prob.meas_shape).astype(np.float32)
    oO, oP = prob.vjp(to_dev(w))
    rO, rP = ptycho.vjp(lin, w.astype(np.float64))
    assert rel(host(oO), rO) < TOL
    if joint:
        assert rel(host(oP), rP) < TOL
    GO, GP = ptycho.ggn_vp(lin, vO64, vP64)
    oO, oP = prob.ggn_vp(vOd, vPd)
    print("ggn rel", rel(host(oO), GO), rel(host(oP), GP) if joint else 0.0)
    assert rel(host(oO), GO) < TOL
    if joint:
        assert rel(host(oP), GP) < TOL
    dOg, dPg = prob.diag(exact=False)
    aO, aP = ptycho.ggn_diag_paper(lin)
    assert rel(host(dOg), aO) < TOL
    if joint:
        assert rel(host(dPg), aP) < TOL
    dOg, dPg = prob.diag(exact=True)
    eO, eP = ptycho.ggn_diag_exact(lin)
    assert rel(host(dOg), eO) < 2 * TOL
    if joint:
        assert rel(host(dPg), eP) < 2 * TOL


@pytest.mark.parametrize("metric", ["gauss", "poisson"])
@pytest.mark.parametrize("probe", [(16, 16), (128, 128), (48, 48), (256, 256), (32, 64)], ids=lambda p: "%dx%d" % p)
def test_stochastic_diagonal(probe, metric):
    """ptlm_diag_stochastic against the oracle's estimator on the oracle's own sign fields (the
    SplitMix64 draws agree bit for bit, so any sign slip would show as an O(1) error)."""
    print("case stochastic diag", probe, metric, flush=True)
    case = make_case(probe, 4, 5, max(probe) // 4, metric=metric, joint=True, seed=9 + probe[0])
    prob = problem(case)
    O, P, y = to_dev(case["O"]), to_dev(case["P"]), to_dev(case["y"])
    prob.linearize(O, P, y)
    lin = ptycho.linearize(case["O64"], case["P64"], case["pos"], case["y64"], 1e-8, metric, True)
    S, seed, draw0 = 3, 0x5EED1234ABCD, 7
    dO, dP = prob.diag_stochastic(S, seed, draw0)
    r = np.stack([ptycho.rademacher_field(lin, seed, draw0 + s) for s in range(S)])
    sO, sP = ptycho.ggn_diag_stochastic(lin, r)
    print("stoch rel", rel(host(dO), sO), rel(host(dP), sP))
    assert rel(host(dO), sO) < 2 * TOL
    assert rel(host(dP), sP) < 2 * TOL


def _check_products(probe, O, P, pos, metric, joint, seed, tol=TOL):
    rng = np.random.default_rng(seed)
    O64, P64 = O.astype(np.complex128), P.astype(np.complex128)
    y = synth.poisson_counts(rng, ptycho.intensity(O64, P64, pos, 1e-8)).astype(np.float32)
    case = dict(O=O, P=P, pos=pos, y=y, metric=metric, joint=joint)
    prob = problem(case)
    Od, Pd, yd = to_dev(O), to_dev(P), to_dev(y)
    assert rel(host(prob.forward(Od, Pd)), ptycho.magnitude(O64, P64, pos, 1e-8)) < TOL
    lin = ptycho.linearize(O64, P64, pos, y.astype(np.float64), 1e-8, metric, joint)
    f, gO, gP = prob.linearize(Od, Pd, yd)
    assert abs(float(host(f)[0]) - lin.f) <= 1e-5 * abs(lin.f)
    rgO, rgP = ptycho.gradient(lin)
    assert rel(host(gO), rgO) < tol
    vO = c64(synth.random_complex(rng, O.shape))
    vP = c64(synth.random_complex(rng, P.shape)) if joint else None
    GO, GP = ptycho.ggn_vp(lin, vO.astype(np.complex128), vP.astype(np.complex128) if joint else None)
    oO, oP = prob.ggn_vp(to_dev(vO), to_dev(vP) if joint else None)
    assert rel(host(oO), GO) < tol
    if joint:
        assert rel(host(gP), rgP) < tol
        assert rel(host(oP), GP) < tol
    dO, dP = prob.diag(exact=True)
    eO, eP = ptycho.ggn_diag_exact(lin)
    assert rel(host(dO), eO) < 2 * tol
    if joint:
        assert rel(host(dP), eP) < 2 * tol


@pytest.mark.parametrize("probe", [(16, 16), (128, 128), (48, 48), (256, 256), (32, 64)], ids=lambda p: "%dx%d" % p)
def test_single_position_covering_the_object(probe):
    """K = 1 with the object exactly the probe's size: one segment, every other workgroup empty,
    every object pixel covered once."""
    print("case single position", probe, flush=True)
    rng = np.random.default_rng(40 + probe[0])
    O = c64(synth.random_complex(rng, probe) * 0.3 + 0.8)
    P = c64(synth.scale_probe_to_photons(synth.make_probe_fresnel(rng, max(probe), 0.35 * max(probe), 3.0)
                                         [:probe[0], :probe[1]], O, 2e3))
    _check_products(probe, O, P, np.zeros((1, 2), np.int32), "gauss", True, seed=probe[0])


@pytest.mark.parametrize("probe", [(16, 16), (128, 128), (96, 96)], ids=lambda p: "%dx%d" % p)
def test_corner_and_repeated_positions(probe):
    """Positions at all four extreme corners of the object, the same position repeated, and a
    prime number of positions (ragged segments, most workgroups of a 128 x 128 launch empty);
    Poisson metric, joint."""
    print("case corners", probe, flush=True)
    rng = np.random.default_rng(50 + probe[0])
    ny, nx = probe[0] * 2 + 5, probe[1] * 2 + 3
    O = c64(synth.make_object(rng, max(ny, nx), amp=(0.7, 1.0), phase=(-math.pi, math.pi), phase_sigma=2.0,
                              phase_source="gaussian")[:ny, :nx])
    P = c64(synth.scale_probe_to_photons(synth.make_probe_fresnel(rng, max(probe), 0.35 * max(probe), 3.0)
                                         [:probe[0], :probe[1]], O, 2e3))
    ry, rx = ny - probe[0], nx - probe[1]
    pos = np.array([[0, 0], [0, rx], [ry, 0], [ry, rx], [ry // 2, rx // 3], [ry // 2, rx // 3], [1, rx - 1]],
                   np.int32)
    _check_products(probe, O, P, pos, "poisson", True, seed=probe[0] + 1)


@pytest.mark.parametrize("ggn", ["magnitude", "intensity"])
@pytest.mark.parametrize("probe,photons", [((48, 48), 20.0), ((64, 64), 30.0), ((128, 128), 100.0)],
                         ids=lambda p: "%dx%d" % p if isinstance(p, tuple) else "%g" % p)
def test_poisson_low_counts_extreme_weights(probe, photons, ggn):
    """Poisson data at a few hundredths of a photon per pixel: many counts y >= 1 fall where the
    model intensity h is far below 1, so the GGN weights 2 + 2y/h (or 4y/h) reach 2e4-3e5 and the
    FP64 refinement of the linearisation rewrites those pixels.  The linearisation's loss and
    gradient and the plain and damped GGN-vector products stay within 1e-5 of the FP64 oracle."""
    print("case poisson low counts", probe, photons, ggn, flush=True)
    case = make_case(probe, 5, 6, max(probe) // 4, metric="poisson", joint=True, seed=17 + probe[0],
                     photons=photons)
    prob = pt.Problem(case["O"].shape, case["P"].shape, case["pos"], metric="poisson", mode="joint",
                      background=1e-8, device=DEV, ggn=ggn)
    O, P, y = to_dev(case["O"]), to_dev(case["P"]), to_dev(case["y"])
    lin = ptycho.linearize(case["O64"], case["P64"], case["pos"], case["y64"], 1e-8, "poisson", True, ggn=ggn)
    w = lin.l2 if hasattr(lin, "l2") else None
    if w is not None:
        print("largest GGN weight %.3e, pixels above 1e4: %d" % (float(np.max(w)), int(np.sum(w > 1e4))))
        assert np.sum(w > 1e4) > 0
    f, gO, gP = prob.linearize(O, P, y)
    f = host(f)
    assert abs(f[0] - lin.f) <= 1e-5 * abs(lin.f)
    rgO, rgP = ptycho.gradient(lin)
    assert rel(host(gO), rgO) < TOL and rel(host(gP), rgP) < TOL
    rng = np.random.default_rng(29)
    vO = c64(synth.random_complex(rng, case["O"].shape))
    vP = c64(synth.random_complex(rng, case["P"].shape))
    GO, GP = ptycho.ggn_vp(lin, vO.astype(np.complex128), vP.astype(np.complex128))
    oO, oP = prob.ggn_vp(to_dev(vO), to_dev(vP))
    print("ggn rel", rel(host(oO), GO), rel(host(oP), GP))
    assert rel(host(oO), GO) < TOL and rel(host(oP), GP) < TOL
    dO = np.abs(rng.standard_normal(case["O"].shape + (2,))).astype(np.float32) + 0.1
    dP = np.abs(rng.standard_normal(case["P"].shape + (2,))).astype(np.float32) + 0.1
    lam = 0.21
    oO, oP = prob.ggn_vp(to_dev(vO), to_dev(vP), lam=lam, dO=to_dev(dO), dP=to_dev(dP))
    rO = GO + lam * (dO[..., 0] * vO.real + 1j * dO[..., 1] * vO.imag)
    rP = GP + lam * (dP[..., 0] * vP.real + 1j * dP[..., 1] * vP.imag)
    assert rel(host(oO), rO) < TOL and rel(host(oP), rP) < TOL


@pytest.mark.parametrize("metric", ["gauss", "poisson"])
@pytest.mark.parametrize("joint", [False, True])
@pytest.mark.parametrize("L", [16, 32])
def test_ggn_vp_mfma_matches_oracle(L, joint, metric):
    """The GGN-vector product with the DFT as matrix products on the matrix cores (16 x 16 and
    32 x 32 probes) and with the FFT tile kernel, against the FP64 oracle and each other, on a
    raster with multi-position segments; the damped product too."""
    print("case ggn mfma", L, joint, metric, flush=True)
    case = make_case((L, L), 9, 10, L // 4, metric=metric, joint=joint, seed=91 + L)
    prob = problem(case)
    O, P, y = to_dev(case["O"]), to_dev(case["P"]), to_dev(case["y"])
    lin = ptycho.linearize(case["O64"], case["P64"], case["pos"], case["y64"], 1e-8, metric, joint)
    prob.linearize(O, P, y)
    rng = np.random.default_rng(12)
    vO = c64(synth.random_complex(rng, case["O"].shape))
    vP = c64(synth.random_complex(rng, case["P"].shape)) if joint else None
    GO, GP = ptycho.ggn_vp(lin, vO.astype(np.complex128), vP.astype(np.complex128) if joint else None)
    out = {}
    for xf in ("mfma", "fft"):
        prob.set_transform(xf)
        out[xf] = prob.ggn_vp(to_dev(vO), to_dev(vP) if joint else None)
    (mO, mP), (fO, fP) = out["mfma"], out["fft"]
    assert rel(host(mO), GO) < TOL
    assert rel(host(mO), host(fO)) < TOL
    if joint:
        assert rel(host(mP), GP) < TOL
        assert rel(host(mP), host(fP)) < TOL
    # damped with a diagonal: lam D v added by the same reductions
    dO = np.abs(rng.standard_normal(case["O"].shape + (2,))).astype(np.float32) + 0.1
    dP = np.abs(rng.standard_normal(case["P"].shape + (2,))).astype(np.float32) + 0.1 if joint else None
    prob.set_transform("mfma")
    lam = 0.37
    oO, oP = prob.ggn_vp(to_dev(vO), to_dev(vP) if joint else None, lam=lam, dO=to_dev(dO),
                         dP=to_dev(dP) if joint else None)
    rO = GO + lam * (dO[..., 0] * vO.real + 1j * dO[..., 1] * vO.imag)
    assert rel(host(oO), rO) < TOL
    if joint:
        rP = GP + lam * (dP[..., 0] * vP.real + 1j * dP[..., 1] * vP.imag)
        assert rel(host(oP), rP) < TOL


def test_transform_choice_rejected_for_other_shapes():
    prob = problem(make_case((64, 64), 3, 3, 8, seed=92))
    with pytest.raises(pt.PtlmError):
        prob.set_transform("mfma")
    prob.set_transform("fft")
    prob.set_transform("fft_wide")
    for shape in ((128, 128), (64, 128), (96, 96)):  # more than 4096 pixels or not the generic kernel
        big = problem(make_case(shape, 2, 2, 8, seed=93))
        with pytest.raises(pt.PtlmError):
            big.set_transform("fft_wide")
        big.set_transform("fft")


@pytest.mark.parametrize("joint", [False, True], ids=["object", "joint"])
@pytest.mark.parametrize("probe,ny,nx", [((16, 16), 9, 9), ((16, 32), 9, 9), ((32, 32), 9, 9), ((32, 64), 9, 9),
                                         ((64, 64), 9, 9), ((128, 32), 9, 9), ((32, 32), 1, 1), ((64, 64), 1, 2)],
                         ids=lambda p: "%dx%d" % p if isinstance(p, tuple) else str(p))
def test_ggn_vp_wide_grouping_equals_fft(probe, ny, nx, joint):
    """The wide grouping (twice the tiles per workgroup over the same segments) runs the FFT tile
    kernel's arithmetic unchanged: its GGN-vector product equals the standard grouping's bit for
    bit and the FP64 oracle to the bar.  A 9 x 9 raster gives an odd standard grid for every
    shape here but 16 x 16, so the last wide workgroup has slots past the last segment; one and
    two positions leave a single wide workgroup with one or two real slots."""
    print("case ggn wide", probe, ny, nx, joint, flush=True)
    case = make_case(probe, ny, nx, 6, joint=joint, seed=95 + probe[0] + probe[1])
    prob = problem(case)
    O, P, y = to_dev(case["O"]), to_dev(case["P"]), to_dev(case["y"])
    lin = ptycho.linearize(case["O64"], case["P64"], case["pos"], case["y64"], 1e-8, "gauss", joint)
    prob.linearize(O, P, y)
    rng = np.random.default_rng(13)
    vO = c64(synth.random_complex(rng, case["O"].shape))
    vP = c64(synth.random_complex(rng, case["P"].shape)) if joint else None
    GO, GP = ptycho.ggn_vp(lin, vO.astype(np.complex128), vP.astype(np.complex128) if joint else None)
    out = {}
    for xf in ("fft", "fft_wide", "fft"):
        prob.set_transform(xf)
        out[xf] = [host(t) for t in prob.ggn_vp(to_dev(vO), to_dev(vP) if joint else None) if t is not None]
    assert all(np.array_equal(a, b) for a, b in zip(out["fft_wide"], out["fft"]))
    assert rel(out["fft_wide"][0], GO) < TOL
    if joint:
        assert rel(out["fft_wide"][1], GP) < TOL
