"""ptlm_loss_noalloc, the entry point whose scratch (the loss kernel's FP64 partial sums) is a
static device array, against ptlm_loss, whose partial sums live in the handle's workspace.

Both run the same kernels in the same order, so the loss and the residual must agree bit for
bit; the loss is also held to the FP64 oracle's at the parity bar.  Two calls in a row, the
second on a smaller problem (fewer workgroups, so the static array still holds entries of
the first call beyond the second one's range), then the same two again in the other order;
and the documented refusal for a 256 x 256 probe."""
import numpy as np
import pytest

import synth
from oracle import ptycho

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - collected on CPU hosts
    pytest.skip("no GPU", allow_module_level=True)
import paper_2103_01767_amd as pt  # noqa: E402

DEV = torch.device("cuda:0")
TOL = 1e-5


def _problem(seed, obj_side, probe, n, step, metric):
    pr = synth.make_small(seed, obj_side=obj_side, probe=(probe, probe), n=n, step=step, photons=1e3, mode="joint")
    rng = np.random.default_rng(seed)
    O = pr.O_init.astype(np.complex64)
    P = pr.P_init.astype(np.complex64)
    y = synth.poisson_counts(rng, ptycho.intensity(pr.O_true, pr.P_true, pr.pos, pr.background)).astype(np.float32)
    prob = pt.Problem(O.shape, P.shape, pr.pos, metric=metric, mode="joint", background=pr.background, device=DEV)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    f_ref = ptycho.loss(O.astype(np.complex128), P.astype(np.complex128), pr.pos, y.astype(np.float64),
                        pr.background, metric)
    return prob, d(O), d(P), d(y), f_ref


def _check(prob, O, P, y, f_ref):
    f_ws, r_ws = prob.loss(O, P, y, residual=True)
    f_st = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
    r_st = torch.full(prob.meas_shape, float("nan"), dtype=torch.float32, device=DEV)
    prob.loss_noalloc(O, P, y, f_st, r_st)
    torch.cuda.synchronize()
    assert float(f_st.cpu()[0]) == float(f_ws.cpu()[0])
    assert torch.equal(r_st, r_ws)
    assert abs(float(f_st.cpu()[0]) - f_ref) <= TOL * abs(f_ref)


@pytest.mark.parametrize("metric", ["gauss", "poisson"])
def test_loss_noalloc_matches_loss_on_two_calls_in_a_row(metric):
    big = _problem(71, 120, 32, 12, 7, metric)     # 144 positions, 32 x 32: 36 workgroups of 4 tiles
    small = _problem(72, 48, 16, 3, 9, metric)     # 9 positions, 16 x 16: one workgroup of 16 tiles
    print("case loss_noalloc", metric, flush=True)
    _check(*big)
    _check(*small)
    _check(*small)
    _check(*big)


def test_loss_noalloc_covers_the_128_tile_kernel():
    case = _problem(73, 200, 128, 3, 30, "gauss")
    print("case loss_noalloc 128", flush=True)
    _check(*case)


def test_loss_noalloc_refuses_a_256_probe():
    pos = np.array([[0, 0], [4, 4]], np.int32)
    prob = pt.Problem((264, 264), (256, 256), pos, mode="joint", device=DEV)
    O = torch.ones((264, 264), dtype=torch.complex64, device=DEV)
    P = torch.ones((256, 256), dtype=torch.complex64, device=DEV)
    y = torch.ones(prob.meas_shape, dtype=torch.float32, device=DEV)
    with pytest.raises(pt.PtlmError) as e:
        prob.loss_noalloc(O, P, y)
    assert e.value.status == pt.PTLM_EINVAL and "256" in str(e.value)
