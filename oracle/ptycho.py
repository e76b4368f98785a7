"""FP64 oracle: far-field ptychography model and its matrix-free derivatives.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy in
complex128; one position at a time where that keeps the definition readable.

Notation (paper Sec. 2 and Sec. 4.1)
------------------------------------
O  (Ny, Nx)   object,  P (My, Mx) probe,  M = My*Mx
pos (K, 2)    integer top-left offsets r_k = (row, col); S_k extracts the
              M object pixels O[r_k + m]                (Sec. 2, eq:exit_wave)
psi_k       = P * S_k O                                 (eq:exit_wave)
psi_hat_k   = F psi_k, F the unitary 2D DFT, no shift   (eq:expected_count)
h           = |psi_hat|^2 + b                           (eq:expected_count)
zeta        = h^(1/2)                                   (eq:magnitude)
ell         = Gaussian 1/2 (zeta - sqrt y)^2  or  Poisson zeta^2 - y log zeta^2
                                                        (eq:ell_magnitude)
f           = sum_k sum_m ell(zeta_km, y_km)            (eq:error_metric_magnitude)

Real coordinates (Sec. 3): a complex array v stands for the real vector
[Re v; Im v]; the real inner product is Re sum conj(u) v.  All derivatives
below are in these real coordinates, so the gradient is twice the Wirtinger
gradient of the paper's App. B (reading of eq:wirtinger).

Reading of F (the paper calls it "the 2D discrete Fourier transform"): the
unitary DFT in FFT order.  It is the only normalisation for which the
diagonal of App. B's circulant C_k is trace/M as the paper states.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

GAUSS = "gauss"
POISSON = "poisson"


# ----------------------------------------------------------------------------
# shift operator S_k and its adjoint (Sec. 2; S_k is binary, App. B)
# ----------------------------------------------------------------------------
def extract(O: np.ndarray, pos: np.ndarray, shape) -> np.ndarray:
    """S_k O for every k -> (K, My, Mx).  Pinned by direct indexing tests."""
    My, Mx = shape
    out = np.empty((len(pos), My, Mx), dtype=np.result_type(O, np.complex128))
    for k, (r, c) in enumerate(pos):
        out[k] = O[r:r + My, c:c + Mx]
    return out


def extract_adjoint(patches: np.ndarray, pos: np.ndarray, obj_shape) -> np.ndarray:
    """sum_k S_k^T patches_k (overlap-add) -> obj_shape."""
    acc = np.zeros(obj_shape, dtype=np.result_type(patches, np.float64))
    My, Mx = patches.shape[1:]
    for k, (r, c) in enumerate(pos):
        acc[r:r + My, c:c + Mx] += patches[k]
    return acc


# ----------------------------------------------------------------------------
# forward model
# ----------------------------------------------------------------------------
def F(x: np.ndarray) -> np.ndarray:
    """Unitary 2D DFT over the last two axes, FFT order (reading of eq:expected_count)."""
    return np.fft.fft2(x, norm="ortho")


def FH(x: np.ndarray) -> np.ndarray:
    """Adjoint (= inverse) of ``F``."""
    return np.fft.ifft2(x, norm="ortho")


def exit_waves(O, P, pos) -> np.ndarray:
    """psi_k = diag(P) S_k O  (eq:exit_wave)."""
    return P[None, :, :] * extract(O, pos, P.shape)


def far_field(O, P, pos) -> np.ndarray:
    """psi_hat_k = F psi_k  (eq:expected_count)."""
    return F(exit_waves(O, P, pos))


def intensity(O, P, pos, b) -> np.ndarray:
    """Expected intensity h_k = |psi_hat_k|^2 + b_k  (eq:expected_count)."""
    return np.abs(far_field(O, P, pos)) ** 2 + b


def magnitude(O, P, pos, b) -> np.ndarray:
    """zeta = h^(1/2)  (eq:magnitude)."""
    return np.sqrt(intensity(O, P, pos, b))


# ----------------------------------------------------------------------------
# error metrics (eq:ell_magnitude) and their derivatives in zeta
# ----------------------------------------------------------------------------
def ell(zeta, y, metric=GAUSS):
    """Per-measurement magnitude-based metric ell(zeta, y)  (eq:ell_magnitude)."""
    if metric == GAUSS:
        return 0.5 * (zeta - np.sqrt(y)) ** 2
    if metric == POISSON:
        z2 = zeta ** 2
        return z2 - y * np.log(z2)
    raise ValueError(metric)


def ell_d1(zeta, y, metric=GAUSS):
    """d ell / d zeta (the "residual" of the metric)."""
    if metric == GAUSS:
        return zeta - np.sqrt(y)
    if metric == POISSON:
        return 2.0 * zeta - 2.0 * y / zeta
    raise ValueError(metric)


def ell_d2(zeta, y, metric=GAUSS):
    """d^2 ell / d zeta^2: the diagonal Hessian of the metric (App. A step 3)."""
    if metric == GAUSS:
        return np.ones_like(zeta)
    if metric == POISSON:
        return 2.0 + 2.0 * y / zeta ** 2
    raise ValueError(metric)


def big_ell(h, y, metric=GAUSS):
    """Intensity-based form L(h, y) of the same metric (eq:error_metric_magnitude): L(zeta^2, y)
    equals ell(zeta, y)."""
    if metric == GAUSS:
        return 0.5 * (np.sqrt(h) - np.sqrt(y)) ** 2
    if metric == POISSON:
        return h - y * np.log(h)
    raise ValueError(metric)


def big_ell_d2(h, y, metric=GAUSS):
    """d^2 L / d h^2, the Hessian of the intensity-based metric in eq:ggn_intensity."""
    if metric == GAUSS:
        return np.sqrt(y) / (4.0 * h ** 1.5)
    if metric == POISSON:
        return y / h ** 2
    raise ValueError(metric)


def loss(O, P, pos, y, b, metric=GAUSS) -> float:
    """f = sum_k sum_m ell(zeta_km, y_km)  (eq:error_metric_magnitude)."""
    return float(np.sum(ell(magnitude(O, P, pos, b), y, metric)))


# ----------------------------------------------------------------------------
# linearisation and matrix-free products
# ----------------------------------------------------------------------------
@dataclass
class Linearization:
    """State of the model at one point z = O (SPR) or z = (O, P) (BPR)."""
    O: np.ndarray
    P: np.ndarray
    pos: np.ndarray
    y: np.ndarray
    b: float
    metric: str
    joint: bool
    psi_hat: np.ndarray   # (K, My, Mx)
    zeta: np.ndarray
    e: np.ndarray         # psi_hat / zeta: d zeta = Re(conj(e) d psi_hat)
    l1: np.ndarray        # ell'(zeta)
    l2: np.ndarray        # GGN weight in zeta: ell''(zeta) (magnitude-based GGN, eq:ggn_magnitude)
                          # or 4 zeta^2 L''(zeta^2) (intensity-based GGN, eq:ggn_intensity)
    ggn: str = "magnitude"

    @property
    def f(self) -> float:
        return float(np.sum(ell(self.zeta, self.y, self.metric)))

    @property
    def M(self) -> int:
        return self.P.size


def linearize(O, P, pos, y, b, metric=GAUSS, joint=False, ggn="magnitude") -> Linearization:
    """Evaluate the forward model and the metric derivatives at (O, P).

    ``ggn`` chooses the GGN matrix of the LM model: "magnitude" (eq:ggn_magnitude, the paper's
    choice) or "intensity" (eq:ggn_intensity, the ablation of App. C).  Since h = zeta^2,
    J_h = diag(2 zeta) J_zeta, so G^L = J_zeta^T diag(4 zeta^2 L''(h)) J_zeta: only the weight
    between the two Jacobians differs; f and the gradient are the same.
    """
    psi_hat = far_field(O, P, pos)
    zeta = np.sqrt(np.abs(psi_hat) ** 2 + b)
    if ggn == "magnitude":
        l2 = ell_d2(zeta, y, metric)
    elif ggn == "intensity":
        l2 = 4.0 * zeta ** 2 * big_ell_d2(zeta ** 2, y, metric)
    else:
        raise ValueError(ggn)
    return Linearization(O=O, P=P, pos=pos, y=y, b=b, metric=metric, joint=joint,
                         psi_hat=psi_hat, zeta=zeta, e=psi_hat / zeta,
                         l1=ell_d1(zeta, y, metric), l2=l2, ggn=ggn)


def jvp(lin: Linearization, vO, vP=None) -> np.ndarray:
    """J v: the directional derivative of zeta along v = (vO, vP).

    d psi_k = P * S_k vO + vP * S_k O (product rule on eq:exit_wave), then
    d zeta = Re(conj(psi_hat) d psi_hat) / zeta.  Pinned by central finite
    differences of ``magnitude``.
    """
    dpsi = lin.P[None] * extract(vO, lin.pos, lin.P.shape)
    if vP is not None:
        dpsi = dpsi + vP[None] * extract(lin.O, lin.pos, lin.P.shape)
    return np.real(np.conj(lin.e) * F(dpsi))


def vjp(lin: Linearization, w):
    """J^T w for w in R^(K x M): the adjoint chain of eq:arbitrary_jtvp_sequence.

    Returns (object part, probe part or None), each a complex array standing
    for its real coordinates.  Pinned by the adjoint identity <Jv,w> = <v,J^T w>.
    """
    u = FH(w * lin.e)
    gO = extract_adjoint(np.conj(lin.P)[None] * u, lin.pos, lin.O.shape)
    gP = None
    if lin.joint:
        gP = np.sum(np.conj(extract(lin.O, lin.pos, lin.P.shape)) * u, axis=0)
    return gO, gP


def gradient(lin: Linearization):
    """g = J^T grad_zeta ell = grad f  (App. A step 1; eq:grad_f_obj times 2)."""
    return vjp(lin, lin.l1)


def ggn_vp(lin: Linearization, vO, vP=None):
    """G v = J^T (grad^2_zeta ell) J v  (eq:ggn_magnitude; App. A steps 2-4).

    The metric Hessian is diagonal for both metrics, so the HVP is the
    elementwise product with ell''.  Pinned by the dense J^T diag(ell'') J on tiny
    inputs, symmetry, PSD-ness and null vectors.
    """
    return vjp(lin, lin.l2 * jvp(lin, vO, vP))


def zeta_residual_norm(lin: Linearization) -> float:
    """||grad_zeta ell|| (the norm in the lambda rule of alg:lm_inexact)."""
    return float(np.sqrt(np.sum(lin.l1 ** 2)))


# ----------------------------------------------------------------------------
# GGN diagonals
# ----------------------------------------------------------------------------
def ggn_diag_paper(lin: Linearization):
    """The paper's analytic diagonal of G, App. B, in real coordinates.

    Steps as in App. B: with h ~ |psi_hat|^2 the circulant C_k has the constant
    diagonal trace(grad^2_k ell)/M, so each Wirtinger diagonal block is
    (1/4M) sum_k trace_k S_k^T |P|^2 (eq:ggn_diag_mat); both blocks are equal.
    The change to (Re, Im) coordinates (eq:ggn_coord_trans) adds the two
    diagonal blocks; the off-diagonal blocks are dropped (reading: the paper
    states only the diagonal blocks).  The same recipe with |S_k O|^2 gives
    the probe part (eq:ggn_joint_diag).

    Returns (dO, dP) with a trailing axis of 2 = (Re, Im) weights; dP is None
    for object-only problems.  Pinned by closed forms: half the
    illumination-overlap map for the Gaussian metric (trace = M), and the
    exact diagonal when the dropped terms vanish; the paper prints no values
    of it to compare with.
    """
    M = lin.M
    trace = lin.l2.reshape(len(lin.pos), -1).sum(axis=1)                  # trace(grad^2_k ell)
    wirt_O = extract_adjoint(trace[:, None, None] * (np.abs(lin.P) ** 2)[None],
                             lin.pos, lin.O.shape) / (4.0 * M)              # eq:ggn_diag_mat
    dO = np.stack([2.0 * wirt_O, 2.0 * wirt_O], axis=-1)                    # eq:ggn_coord_trans
    dP = None
    if lin.joint:
        SO = extract(lin.O, lin.pos, lin.P.shape)
        wirt_P = np.sum(trace[:, None, None] * np.abs(SO) ** 2, axis=0) / (4.0 * M)
        dP = np.stack([2.0 * wirt_P, 2.0 * wirt_P], axis=-1)
    return dO, dP


def ggn_diag_exact(lin: Linearization):
    """Exact diagonal of G in real coordinates (closed form, not in the paper).

    diag(G)_i = sum_j ell''_j J_ji^2.  For an object coordinate at probe pixel
    m' of position k, J's column is Re(conj(a) P_m' phi) with a = sqrt(ell'') e
    and phi = F delta_m'; Re(z)^2 = (|z|^2 + Re z^2)/2 splits the sum into
    |P_m'|^2 A_k/(2M) and Re(P_m'^2 B_k[2m'])/2 with A_k = sum |a|^2 and
    B_k = DFT_unnorm(conj(a)^2)/M read at frequency 2m' (mod the probe shape).
    The imaginary coordinate flips the sign of the second term.  Probe
    coordinates use S_k O in place of P.  Pinned by the dense diagonal.
    """
    K = len(lin.pos)
    My, Mx = lin.P.shape
    M = My * Mx
    a = np.sqrt(lin.l2) * lin.e
    A = np.sum(np.abs(a) ** 2, axis=(1, 2))
    B = np.fft.fft2(np.conj(a) ** 2) / M
    iy = (2 * np.arange(My)) % My
    ix = (2 * np.arange(Mx)) % Mx
    B2 = B[:, iy[:, None], ix[None, :]]

    def terms(Q):
        base = np.abs(Q) ** 2 * A[:, None, None] / (2.0 * M)
        cross = 0.5 * np.real(Q ** 2 * B2)
        return base + cross, base - cross

    re, im = terms(np.broadcast_to(lin.P[None], (K, My, Mx)))
    dO = np.stack([extract_adjoint(re, lin.pos, lin.O.shape),
                   extract_adjoint(im, lin.pos, lin.O.shape)], axis=-1)
    dP = None
    if lin.joint:
        re, im = terms(extract(lin.O, lin.pos, lin.P.shape))
        dP = np.stack([re.sum(axis=0), im.sum(axis=0)], axis=-1)
    return dO, dP


def illumination_overlap(P, pos, obj_shape) -> np.ndarray:
    """sum_k S_k^T |P|^2: the illumination-overlap map."""
    K = len(pos)
    return extract_adjoint(np.broadcast_to(np.abs(P)[None] ** 2, (K,) + P.shape), pos, obj_shape)


# ----------------------------------------------------------------------------
# stochastic diagonal estimate (the matrix-free route the paper points to when
# no analytic diagonal is available)
# ----------------------------------------------------------------------------
_U64 = np.uint64
_GOLDEN_GAMMA = _U64(0x9E3779B97F4A7C15)


def splitmix64(seed: int, n: np.ndarray) -> np.ndarray:
    """Output number n >= 1 of the SplitMix64 generator seeded with ``seed`` (Steele, Lea and
    Flood, OOPSLA 2014): the state after n steps is seed + n * gamma (mod 2^64) and the output
    is Stafford's 64-bit finaliser ("Mix13") of it.  Counter-based: any output is computed on
    its own.  Pinned by the generator's first outputs from seed 0."""
    with np.errstate(over="ignore"):
        z = _U64(seed) + np.asarray(n, dtype=_U64) * _GOLDEN_GAMMA
        z = (z ^ (z >> _U64(30))) * _U64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> _U64(27))) * _U64(0x94D049BB133111EB)
        return z ^ (z >> _U64(31))


def rademacher(seed: int, n: np.ndarray) -> np.ndarray:
    """+1 or -1 from the top bit of SplitMix64 output n (n >= 1)."""
    return np.where(splitmix64(seed, n) >> _U64(63), -1.0, 1.0)


def rademacher_field(lin: "Linearization", seed: int, draw: int) -> np.ndarray:
    """The sign field r of draw ``draw`` over all K x M measurements: measurement j (position k,
    detector pixel m in row-major order, j = k M + m) takes output draw K M + j + 1."""
    KM = lin.zeta.size
    n = np.uint64(draw) * np.uint64(KM) + np.arange(KM, dtype=np.uint64) + np.uint64(1)
    return rademacher(seed, n).reshape(lin.zeta.shape)


def ggn_diag_stochastic(lin: Linearization, r: np.ndarray):
    """Unbiased estimate of diag(G) from vector-Jacobian products alone (Chapelle and Erhan
    2011; Martens 2016): for a sign vector r over the measurements, u = J^T diag(sqrt(W)) r has
    E[u u^T] = J^T diag(W) J = G, so the mean of u_i^2 over draws estimates G_ii.  W is the GGN
    weight of the linearisation (ell'' or its intensity-based form).  ``r`` has shape
    (S, K, My, Mx), entries +-1.  Returns (dO, dP) in the layout of ggn_diag_exact.  Pinned:
    averaged over every sign pattern it is the exact diagonal; over many draws it converges
    to it."""
    w = np.sqrt(lin.l2)
    accO = np.zeros(lin.O.shape + (2,))
    accP = np.zeros(lin.P.shape + (2,)) if lin.joint else None
    for rs in r:
        uO, uP = vjp(lin, w * rs)
        accO += np.stack([uO.real ** 2, uO.imag ** 2], axis=-1)
        if lin.joint:
            accP += np.stack([uP.real ** 2, uP.imag ** 2], axis=-1)
    S = len(r)
    return accO / S, (accP / S if lin.joint else None)
