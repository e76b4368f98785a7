"""Seeded synthetic inputs for the ptychography workloads.

This module produces the *inputs* of a reconstruction problem -- true object,
true probe, scan offsets, initial guesses, random direction vectors and
Poisson draws of given intensities.  It holds none of the reconstruction
method's arithmetic (no exit wave, no far-field transform of an exit wave, no
error metric, no derivative).  Both the FP64 CPU oracle and the GPU path are
fed from here; neither is imported by this module.

Every generator takes a ``numpy.random.Generator`` (or a seed) so that each
workload is reproducible bit for bit.  Arrays are complex128 / float64; the GPU
side casts them to complex64 / float32.

Workload recipes (sizes and distributions follow the experiment descriptions
of the paper's Sec. 5 and the five benchmark configurations):

* ``c0``  64x64 object, 16x16 fixed probe, 8x8 raster (step 4), noise-free,
           object-only plain LM.
* ``c1``  512x512 object, 128x128 probe, 40x40 raster (step 8, +-1 jitter),
           Poisson data at 1e4 photons per pattern, joint object+probe.
* ``c2``  64 problems of uneven size (object side 128..384, probe side in
           {32,48,64,96}, n x n raster with n in 10..30, step = probe/4).
* ``c4``  2048x2048 object, 256x256 probe, 100x100 raster (step 16, +-2),
           Poisson at 1e3 photons per pattern.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy import ndimage

BACKGROUND = 1e-8  # Sec. 5: constant incoherent background, strictly positive


def rng_for(seed) -> np.random.Generator:
    return seed if isinstance(seed, np.random.Generator) else np.random.default_rng(seed)


# ----------------------------------------------------------------------------
# field helpers
# ----------------------------------------------------------------------------
def _rescale(x: np.ndarray, lo: float, hi: float) -> np.ndarray:
    """Min-max rescale of a real field into [lo, hi]."""
    mn, mx = float(x.min()), float(x.max())
    if mx - mn == 0.0:
        return np.full_like(x, 0.5 * (lo + hi))
    return lo + (hi - lo) * (x - mn) / (mx - mn)


def smooth_wrap(x: np.ndarray, sigma: float) -> np.ndarray:
    """Periodic Gaussian smoothing (a texture filter, not part of the method)."""
    return ndimage.gaussian_filter(x, sigma=sigma, mode="wrap")


def make_object(rng, side: int, amp=(0.8, 1.0), phase=(-math.pi / 2, math.pi / 2),
                phase_sigma: float = 2.0, phase_source: str = "uniform") -> np.ndarray:
    """Complex transmission function: iid uniform amplitude, smoothed phase.

    ``phase_source='uniform'`` smooths iid U[phase] noise; ``'gaussian'`` smooths
    white Gaussian noise.  Either way the smoothed field is min-max rescaled to
    the stated phase range.
    """
    a = rng.uniform(amp[0], amp[1], size=(side, side))
    if phase_source == "uniform":
        raw = rng.uniform(phase[0], phase[1], size=(side, side))
    else:
        raw = rng.standard_normal((side, side))
    ph = _rescale(smooth_wrap(raw, phase_sigma), phase[0], phase[1])
    return a * np.exp(1j * ph)


def _radius_grid(side: int, center=None) -> np.ndarray:
    c = (side - 1) / 2.0 if center is None else center
    yy, xx = np.mgrid[0:side, 0:side].astype(np.float64)
    return np.hypot(yy - c, xx - c)


def make_probe_gauss_aperture(side: int = 16, radius: float = 6.0, sigma: float = 4.0) -> np.ndarray:
    """Real probe: circular aperture times a Gaussian, centred on the array."""
    r = _radius_grid(side)
    return ((r <= radius) * np.exp(-r ** 2 / (2 * sigma ** 2))).astype(np.complex128)


def make_probe_fresnel(rng, side: int, radius: float, fresnel_px: float = 10.0) -> np.ndarray:
    """Aperture with a random quadratic phase, Fresnel-propagated.

    The quadratic curvature is c ~ U[-pi/R^2, pi/R^2] (at most pi of phase at the
    aperture edge); the propagator is the paraxial transfer function
    exp(-i pi lambda z |f|^2) with sqrt(lambda z) = ``fresnel_px`` pixels and f in
    cycles per pixel.  This only shapes a realistic probe; it is not the
    far-field model of the reconstruction.
    """
    r = _radius_grid(side)
    c = rng.uniform(-math.pi / radius ** 2, math.pi / radius ** 2)
    ap = (r <= radius) * np.exp(1j * c * r ** 2)
    f = np.fft.fftfreq(side)
    f2 = f[:, None] ** 2 + f[None, :] ** 2
    lz = fresnel_px ** 2
    return np.fft.ifft2(np.fft.fft2(ap) * np.exp(-1j * math.pi * lz * f2))


def scale_probe_to_photons(P: np.ndarray, O: np.ndarray, photons: float) -> np.ndarray:
    """Scale P so that sum|P|^2 * mean|O|^2 equals ``photons``.

    With a unitary transform the photons in a pattern equal the energy of the
    exit wave, which this product estimates without forming any exit wave.
    """
    e = float(np.sum(np.abs(P) ** 2)) * float(np.mean(np.abs(O) ** 2))
    return P * math.sqrt(photons / e)


def raster_positions(rng, n: int, step: int, offset: int, jitter: int,
                     obj_side: int, probe_side: int) -> np.ndarray:
    """n x n raster of integer top-left offsets (row, col), int32 (K, 2).

    Centred raster with integer jitter U{-j..j} per axis, clipped so that every
    probe window lies inside the object.
    """
    base = offset + step * np.arange(n)
    ry, rx = np.meshgrid(base, base, indexing="ij")
    pos = np.stack([ry.ravel(), rx.ravel()], axis=1).astype(np.int64)
    if jitter > 0:
        pos = pos + rng.integers(-jitter, jitter + 1, size=pos.shape)
    pos = np.clip(pos, 0, obj_side - probe_side)
    return pos.astype(np.int32)


def random_object_guess(rng, side: int) -> np.ndarray:
    """Uniformly random complex array with magnitude <= 1 (Sec. 5 initial guess)."""
    return rng.uniform(0.0, 1.0, (side, side)) * np.exp(1j * rng.uniform(-math.pi, math.pi, (side, side)))


def phaseless_aperture_guess(P_true: np.ndarray, radius: float) -> np.ndarray:
    """Phaseless circular aperture with the true probe's integrated intensity."""
    side = P_true.shape[0]
    ap = (_radius_grid(side) <= radius).astype(np.complex128)
    return ap * math.sqrt(np.sum(np.abs(P_true) ** 2) / np.sum(np.abs(ap) ** 2))


def random_complex(rng, shape) -> np.ndarray:
    """Standard complex Gaussian direction vector (for products with J, J^T, G)."""
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def poisson_counts(rng, intensity: np.ndarray) -> np.ndarray:
    """Poisson draws of a given expected-count array (photon noise)."""
    return rng.poisson(np.maximum(intensity, 0.0)).astype(np.float64)


def surrogate_counts(rng, K: int, shape, photons: float) -> np.ndarray:
    """Seeded stand-in detector counts (float32, K x My x Mx) for tests that only need
    data of the right size, scale and layout, not data consistent with an object: a
    radially decaying mean in detector (FFT) order holding ``photons`` per pattern, times
    independent U[0, 2) factors.  Generated in chunks of positions to bound memory."""
    my, mx = shape
    fy = np.fft.fftfreq(my)[:, None]
    fx = np.fft.fftfreq(mx)[None, :]
    prof = 1.0 / (1.0 + ((fy ** 2 + fx ** 2) / 0.02 ** 2) ** 2)
    prof = (photons * prof / prof.sum()).astype(np.float32)
    out = np.empty((K, my, mx), dtype=np.float32)
    step = max(1, (1 << 24) // (my * mx))
    for k0 in range(0, K, step):
        k1 = min(K, k0 + step)
        u = rng.random((k1 - k0, my, mx), dtype=np.float32)
        np.multiply(u, 2.0 * prof, out=out[k0:k1])
    return out


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
@dataclass
class Problem:
    name: str
    seed: int
    O_true: np.ndarray
    P_true: np.ndarray
    pos: np.ndarray            # int32 (K, 2): (row, col) top-left offsets
    O_init: np.ndarray
    P_init: np.ndarray
    background: float
    photons: float | None      # None: noise-free data
    mode: str                  # "object" or "joint"
    metric: str = "gauss"
    solver: dict = field(default_factory=dict)

    @property
    def K(self):
        return int(self.pos.shape[0])

    @property
    def obj_shape(self):
        return self.O_true.shape

    @property
    def probe_shape(self):
        return self.P_true.shape


def make_c0(seed: int = 1000) -> Problem:
    rng = rng_for(seed)
    O = make_object(rng, 64, amp=(0.8, 1.0), phase=(-math.pi / 2, math.pi / 2),
                    phase_sigma=2.0, phase_source="uniform")
    P = make_probe_gauss_aperture(16, 6.0, 4.0)
    pos = raster_positions(rng, 8, 4, 10, 0, 64, 16)
    O0 = random_object_guess(rng, 64)
    return Problem("c0", seed, O, P, pos, O0, P.copy(), BACKGROUND, None, "object",
                   solver=dict(T=20, cg_max=10, scaling=0, precond=0, beta=0.1))


def make_c3(seed: int) -> Problem:
    """Training / evaluation problem of the preconditioner network: the small object-only
    recipe (64 x 64 object, 8 x 8 raster at step 4, noise-free) with a random quadratic phase
    exp(i c r^2), c ~ U[-pi/R^2, pi/R^2] (R = 6 px, at most pi at the aperture edge), on the
    Gaussian-aperture probe, so that the phase input of the network carries information."""
    rng = rng_for(seed)
    O = make_object(rng, 64, amp=(0.8, 1.0), phase=(-math.pi / 2, math.pi / 2),
                    phase_sigma=2.0, phase_source="uniform")
    R = 6.0
    c = rng.uniform(-math.pi / R ** 2, math.pi / R ** 2)
    P = make_probe_gauss_aperture(16, R, 4.0) * np.exp(1j * c * _radius_grid(16) ** 2)
    pos = raster_positions(rng, 8, 4, 10, 0, 64, 16)
    O0 = random_object_guess(rng, 64)
    return Problem("c3_%d" % seed, seed, O, P, pos, O0, P.copy(), BACKGROUND, None, "object",
                   solver=dict(T=20, cg_max=10, scaling=0, precond=0, beta=0.1))


def make_scaled(name: str, seed: int, obj_side: int, probe_side: int, n: int, step: int,
                offset: int, jitter: int, radius: float, photons: float,
                phase_sigma: float, amp=(0.7, 1.0), fresnel_px: float = 10.0,
                T: int = 50) -> Problem:
    rng = rng_for(seed)
    O = make_object(rng, obj_side, amp=amp, phase=(-math.pi, math.pi),
                    phase_sigma=phase_sigma, phase_source="gaussian")
    P = make_probe_fresnel(rng, probe_side, radius, fresnel_px)
    P = scale_probe_to_photons(P, O, photons)
    pos = raster_positions(rng, n, step, offset, jitter, obj_side, probe_side)
    O0 = random_object_guess(rng, obj_side)
    P0 = phaseless_aperture_guess(P, radius)
    return Problem(name, seed, O, P, pos, O0, P0, BACKGROUND, photons, "joint",
                   solver=dict(T=T, cg_max=10, scaling=1, precond=1, beta=0.1))


def make_c1(seed: int = 1001) -> Problem:
    return make_scaled("c1", seed, 512, 128, 40, 8, 36, 1, 40.0, 1e4, 8.0)


def make_c4(seed: int = 1004) -> Problem:
    return make_scaled("c4", seed, 2048, 256, 100, 16, 104, 2, 80.0, 1e3, 32.0)


def make_c2_problem(p: int) -> Problem:
    """Problem p (0..63) of the uneven batch.

    Draws object side U{128..384}, probe side from {32,48,64,96}, raster n from
    U{10..30} with step = probe/4 and +-1 jitter, photons log-uniform in
    [1e3, 1e5].  When the drawn raster would not fit, the object side is
    enlarged to (n-1)*step + probe + 2 so that the drawn K*M work is kept.
    """
    rng = rng_for(1002 * 1000 + p)
    side = int(rng.integers(128, 385))
    ps = int(rng.choice([32, 48, 64, 96]))
    n = int(rng.integers(10, 31))
    step = ps // 4
    photons = float(10 ** rng.uniform(3, 5))
    need = (n - 1) * step + ps + 2
    side = max(side, need)
    offset = (side - ((n - 1) * step + ps)) // 2
    return make_scaled("c2_%02d" % p, rng, side, ps, n, step, offset, 1, ps * 40.0 / 128.0,
                       photons, side / 64.0)


def make_small(seed: int, obj_side: int = 40, probe: tuple = (16, 16), n: int = 4,
               step: int = 6, jitter: int = 1, photons: float | None = 1e3,
               mode: str = "joint") -> Problem:
    """Small generic problem used by unit tests (rectangular probes allowed)."""
    rng = rng_for(seed)
    O = make_object(rng, obj_side, amp=(0.7, 1.0), phase=(-math.pi, math.pi),
                    phase_sigma=2.0, phase_source="gaussian")
    my, mx = probe
    side = max(my, mx)
    Pfull = make_probe_fresnel(rng, side, side * 0.3, 2.0)
    P = Pfull[:my, :mx].copy()
    if photons is not None:
        P = scale_probe_to_photons(P, O, photons)
    base = 1 + step * np.arange(n)
    ry, rx = np.meshgrid(base, base, indexing="ij")
    pos = np.stack([ry.ravel(), rx.ravel()], axis=1)
    if jitter:
        pos = pos + rng.integers(-jitter, jitter + 1, size=pos.shape)
    pos[:, 0] = np.clip(pos[:, 0], 0, obj_side - my)
    pos[:, 1] = np.clip(pos[:, 1], 0, obj_side - mx)
    O0 = random_object_guess(rng, obj_side)
    P0 = P * 0.9 + 0.05 * random_complex(rng, P.shape) * np.abs(P).max()
    return Problem("small", seed, O, P, pos.astype(np.int32), O0, P0, BACKGROUND, photons, mode)


CONFIGS = {"c0": make_c0, "c1": make_c1, "c4": make_c4}
