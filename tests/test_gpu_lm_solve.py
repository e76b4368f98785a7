"""ptlm_lm_solve(T) against T calls of ptlm_lm_step on the same problem, start and data.

ptlm_lm_solve keeps the state it reads at the end of one outer iteration for the start of
the next, where ptlm_lm_step reads it afresh; the iterates and the device LM state (FP64
scalars and counters) must come out bit for bit the same either way.  Cases: the joint
scaled-Jacobi LM, the alternating update, the projected plug-in (|O| <= 1 active, with
rejected attempts), and a 128 x 128 probe."""
import numpy as np
import pytest

import synth
from oracle import ptycho

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)
import paper_2103_01767_amd as pt  # noqa: E402

DEV = torch.device("cuda:0")


def _inputs(seed, obj_side, probe, n, step):
    pr = synth.make_small(seed, obj_side=obj_side, probe=(probe, probe), n=n, step=step, photons=1e3, mode="joint")
    rng = np.random.default_rng(seed)
    y = synth.poisson_counts(rng, ptycho.intensity(pr.O_true, pr.P_true, pr.pos, pr.background)).astype(np.float32)
    return pr, y


def _run(pr, y, params, T, use_solve):
    prob = pt.Problem(pr.O_true.shape, pr.P_true.shape, pr.pos, mode="joint", background=pr.background, device=DEV)
    d = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a.astype(dt))).to(DEV)
    O, P, yd = d(pr.O_init, np.complex64), d(pr.P_init, np.complex64), d(y, np.float32)
    st = prob.new_state()
    prob.lm_init(params, st)
    if use_solve:
        prob.lm_solve(O, P, yd, params, T, st)
    else:
        for _ in range(T):
            prob.lm_step(O, P, yd, params, st)
    torch.cuda.synchronize()
    return O, P, st


CASES = {
    "joint_jacobi": dict(scaling=1, precond=1),
    "alternating": dict(scaling=1, precond=1, alternate=1),
    "projected": dict(scaling=1, precond=1, project=1, o_max=0.8, retry_max=4, mu0=1e-9),
}


@pytest.mark.parametrize("name", list(CASES))
def test_lm_solve_equals_repeated_lm_step(name):
    print("case lm_solve vs lm_step", name, flush=True)
    pr, y = _inputs(31, 48, 16, 6, 5)
    params = pt.default_params(**CASES[name])
    T = 8
    O1, P1, s1 = _run(pr, y, params, T, True)
    O2, P2, s2 = _run(pr, y, params, T, False)
    st = pt.state_from_tensor(s1)
    print("%s: t=%d products=%d f=%.6e" % (name, st.t, st.products, st.f))
    assert st.t == T
    assert torch.equal(O1, O2) and torch.equal(P1, P2)
    assert torch.equal(s1, s2)


def test_lm_solve_equals_repeated_lm_step_128_probe():
    print("case lm_solve vs lm_step 128", flush=True)
    pr, y = _inputs(32, 180, 128, 3, 20)
    params = pt.default_params(scaling=1, precond=1)
    O1, P1, s1 = _run(pr, y, params, 4, True)
    O2, P2, s2 = _run(pr, y, params, 4, False)
    assert pt.state_from_tensor(s1).t == 4
    assert torch.equal(O1, O2) and torch.equal(P1, P2)
    assert torch.equal(s1, s2)
