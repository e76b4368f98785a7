"""Batched LM over problems of uneven sizes (probe sides 16-96, square and rectangular).

* Each problem of a batch ends with exactly the iterate, loss and counters it reaches when
  solved alone with ptlm_lm_step (same kernels, same blocks, same reduction order).
* Attempts replayed from the captured HIP graph equal eager attempts, checked after every
  replay, with eager work and synchronisations in between.
* The batch reproduces the single-problem LM, which is itself checked against the FP64
  oracle's LM (test_gpu_lm.py); the data here are Poisson draws of the oracle's intensities.
"""
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

# (object side, probe shape, raster n, step, seed)
SPECS = [(72, (32, 32), 6, 8, 11), (100, (48, 48), 6, 10, 12), (120, (64, 64), 5, 12, 13),
         (150, (96, 96), 4, 16, 14), (40, (16, 16), 5, 5, 15), (90, (32, 64), 4, 8, 16)]


def c64(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.complex64))).to(DEV)


# launch shape of some problems: segments of about this many positions (the rest: default cut)
SEG_LEN = {12: 3, 14: 2, 16: 5}


def make_problems():
    out = []
    for side, probe, n, step, seed in SPECS:
        rng = np.random.default_rng(seed)
        O = synth.make_object(rng, side, amp=(0.7, 1.0), phase=(-np.pi, np.pi), phase_sigma=3.0,
                              phase_source="gaussian")
        P = synth.make_probe_fresnel(rng, max(probe), 0.3 * max(probe), 5.0)[:probe[0], :probe[1]]
        P = synth.scale_probe_to_photons(P, O, 3e3)
        base_y = 2 + step * np.arange(n)
        base_x = 2 + step * np.arange(n)
        ry, rx = np.meshgrid(base_y, base_x, indexing="ij")
        pos = np.stack([ry.ravel(), rx.ravel()], 1) + rng.integers(-1, 2, size=(n * n, 2))
        pos = np.clip(pos, 0, [side - probe[0], side - probe[1]]).astype(np.int32)
        y = synth.poisson_counts(rng, ptycho.intensity(O, P, pos, 1e-8)).astype(np.float32)
        O0 = synth.random_object_guess(rng, side)
        P0 = np.abs(P)  # phaseless start with the true intensity
        out.append(dict(obj_shape=(side, side), probe_shape=probe, positions=pos, mode="joint", y=y, O0=O0, P0=P0,
                        seg_len=SEG_LEN.get(seed, 0)))
    return out


def run_single(p, params, T):
    prob = pt.Problem(p["obj_shape"], p["probe_shape"], p["positions"], mode="joint", device=DEV,
                      seg_len=p.get("seg_len", 0))
    O, P = c64(p["O0"]), c64(p["P0"])
    y = torch.from_numpy(p["y"]).to(DEV)
    st = prob.new_state()
    prob.lm_init(params, st)
    for _ in range(T):
        prob.lm_step(O, P, y, params, st)
    torch.cuda.synchronize()
    return O, P, pt.state_from_tensor(st)


@pytest.mark.parametrize("precond", [1, 0])
def test_batch_equals_problems_alone(precond):
    print("case batch vs single precond", precond, flush=True)
    probs = make_problems()
    params = pt.default_params(scaling=1 if precond else 0, precond=precond, cg_max=6)
    T = 4
    alone = [run_single(p, params, T) for p in probs]
    batch = pt.Batch(probs, device=DEV)
    Os = [c64(p["O0"]) for p in probs]
    Ps = [c64(p["P0"]) for p in probs]
    ys = [torch.from_numpy(p["y"]).to(DEV) for p in probs]
    batch.bind(Os, Ps, ys, params, T, use_graph=True)
    status, attempts = batch.solve(200, check_every=2)
    torch.cuda.synchronize()
    assert status in (pt.PTLM_OK,)
    for i, (O1, P1, s1) in enumerate(alone):
        s2 = batch.state(i)
        print("problem %d: t %d/%d f %.6e / %.6e products %d / %d" % (i, s1.t, s2.t, s1.f, s2.f, s1.products,
                                                                     s2.products))
        assert s2.t == T and s1.t == T
        assert s2.f == s1.f and s2.products == s1.products and s2.attempts == s1.attempts
        assert torch.equal(Os[i], O1) and torch.equal(Ps[i], P1)


def test_graph_replays_equal_eager_attempts():
    print("case graph vs eager", flush=True)
    probs = make_problems()[:4]
    params = pt.default_params(scaling=1, precond=1, cg_max=5)
    runs = []
    for use_graph in (False, True):
        b = pt.Batch(probs, device=DEV)
        Os = [c64(p["O0"]) for p in probs]
        Ps = [c64(p["P0"]) for p in probs]
        ys = [torch.from_numpy(p["y"]).to(DEV) for p in probs]
        b.bind(Os, Ps, ys, params, 100, use_graph=use_graph)
        runs.append((b, Os, Ps, ys))
    for a in range(6):
        for b, *_ in runs:
            b.attempt()
        torch.cuda.synchronize()
        # eager work between replays: a loss of every problem through its handle
        (b0, O0s, P0s, y0s), (b1, O1s, P1s, y1s) = runs
        for i in range(len(probs)):
            f0 = b0.problem(i).loss(O0s[i], P0s[i], y0s[i])
            f1 = b1.problem(i).loss(O1s[i], P1s[i], y1s[i])
            assert torch.equal(f0, f1), (a, i)
            assert torch.equal(O0s[i], O1s[i]) and torch.equal(P0s[i], P1s[i]), (a, i)
        torch.cuda.synchronize()
    for i in range(len(probs)):
        s0, s1 = runs[0][0].state(i), runs[1][0].state(i)
        assert (s0.t, s0.attempts, s0.products, s0.f) == (s1.t, s1.attempts, s1.products, s1.f)
        assert s0.attempts == 6


def test_batch_problem_handles_serve_single_calls():
    probs = make_problems()[:3]
    batch = pt.Batch(probs, device=DEV)
    for i, p in enumerate(probs):
        alone = pt.Problem(p["obj_shape"], p["probe_shape"], p["positions"], mode="joint", device=DEV,
                           seg_len=p.get("seg_len", 0))
        O, P = c64(p["O0"]), c64(p["P0"])
        z1 = batch.problem(i).forward(O, P)
        z2 = alone.forward(O, P)
        assert torch.equal(z1, z2)
    # the batch's tables fix each problem's launch shape: no re-segmentation or transform change
    with pytest.raises(pt.PtlmError, match="batch"):
        batch.problem(0).autotune(reps=1)
    with pytest.raises(pt.PtlmError, match="batch"):
        batch.problem(0).set_transform("fft")


def test_batch_learned_preconditioner_equals_alone():
    """precond 2: every problem's network runs once from its starting probe (in the batch at
    bind, alone at the first linearisation with refresh period 0); iterates agree bit for bit."""
    print("case batch learned", flush=True)
    from paper_2103_01767_amd import learned
    probs = make_problems()[:4]
    params = pt.default_params(scaling=1, precond=2, cg_max=5)
    T = 3
    net_params = learned.he_params(3, DEV)
    net_params[-2:] = 0.05  # a non-zero output bias: the learned diagonal differs from App. B
    alone = []
    for p in probs:
        prob = pt.Problem(p["obj_shape"], p["probe_shape"], p["positions"], mode="joint", device=DEV,
                          seg_len=p.get("seg_len", 0))
        net = learned.lm_net(net_params, p["obj_shape"], DEV)
        pt.lm_set_cnn(prob, net)
        pt.lm_set_cnn_refresh(prob, 0)
        O, P = c64(p["O0"]), c64(p["P0"])
        y = torch.from_numpy(p["y"]).to(DEV)
        st = prob.new_state()
        prob.lm_init(params, st)
        for _ in range(T):
            prob.lm_step(O, P, y, params, st)
        torch.cuda.synchronize()
        alone.append((O, P, pt.state_from_tensor(st)))
    batch = pt.Batch(probs, device=DEV)
    nets = [learned.lm_net(net_params, p["obj_shape"], DEV) for p in probs]
    for i in range(len(probs)):
        pt.lm_set_cnn(batch.problem(i), nets[i])
    Os = [c64(p["O0"]) for p in probs]
    Ps = [c64(p["P0"]) for p in probs]
    ys = [torch.from_numpy(p["y"]).to(DEV) for p in probs]
    batch.bind(Os, Ps, ys, params, T, use_graph=True)
    status, _ = batch.solve(100, check_every=1)
    torch.cuda.synchronize()
    assert status == pt.PTLM_OK
    for i, (O1, P1, s1) in enumerate(alone):
        s2 = batch.state(i)
        assert s2.t == T and s2.f == s1.f and s2.products == s1.products
        assert torch.equal(Os[i], O1) and torch.equal(Ps[i], P1)


def test_batch_learned_refresh_equals_alone_every_linearisation():
    """ptlm_batch_cnn_refresh after every attempt re-runs each network from the probe its next
    linearisation starts from (the new iterate after an accepted step, the unchanged one after
    a reject), so the batch equals each problem solved alone with the network re-run at every
    linearisation, bit for bit."""
    print("case batch learned refresh", flush=True)
    from paper_2103_01767_amd import learned
    probs = make_problems()[:4]
    params = pt.default_params(scaling=1, precond=2, cg_max=5)
    T = 3
    net_params = learned.he_params(5, DEV)
    net_params[-2:] = -0.05
    alone = []
    for p in probs:
        prob = pt.Problem(p["obj_shape"], p["probe_shape"], p["positions"], mode="joint", device=DEV,
                          seg_len=p.get("seg_len", 0))
        pt.lm_set_cnn(prob, learned.lm_net(net_params, p["obj_shape"], DEV))
        pt.lm_set_cnn_refresh(prob, 1)
        O, P = c64(p["O0"]), c64(p["P0"])
        y = torch.from_numpy(p["y"]).to(DEV)
        st = prob.new_state()
        prob.lm_init(params, st)
        for _ in range(T):
            prob.lm_step(O, P, y, params, st)
        torch.cuda.synchronize()
        alone.append((O, P, pt.state_from_tensor(st)))
    batch = pt.Batch(probs, device=DEV)
    nets = [learned.lm_net(net_params, p["obj_shape"], DEV) for p in probs]
    for i in range(len(probs)):
        pt.lm_set_cnn(batch.problem(i), nets[i])
    Os = [c64(p["O0"]) for p in probs]
    Ps = [c64(p["P0"]) for p in probs]
    ys = [torch.from_numpy(p["y"]).to(DEV) for p in probs]
    batch.bind(Os, Ps, ys, params, T, use_graph=True)
    for _ in range(100):
        status, _ = batch.solve(1, check_every=1)
        if all(s.t >= T for s in batch.all_states()):
            break
        batch.cnn_refresh()
    torch.cuda.synchronize()
    for i, (O1, P1, s1) in enumerate(alone):
        s2 = batch.state(i)
        print("problem %d: f %.6e / %.6e products %d / %d" % (i, s1.f, s2.f, s1.products, s2.products))
        assert s2.t == T and s2.f == s1.f and s2.products == s1.products
        assert torch.equal(Os[i], O1) and torch.equal(Ps[i], P1)


def test_batch_surrogate_equals_alone():
    """The surrogate term of App. E is read from each problem's device state by the batched
    kernels: a Poisson batch with the schedule equals its problems solved alone (probe sides 32,
    48, 64 and 96)."""
    probs = make_problems()[:4]
    for p in probs:
        p["metric"] = "poisson"
    params = pt.default_params(scaling=1, precond=1, beta=0.9, cg_max=5, surrogate_T=3, surrogate_s0=1.0)
    T = 4
    alone = []
    for p in probs:
        prob = pt.Problem(p["obj_shape"], p["probe_shape"], p["positions"], metric="poisson", mode="joint",
                          device=DEV, seg_len=p.get("seg_len", 0))
        O, P = c64(p["O0"]), c64(p["P0"])
        y = torch.from_numpy(p["y"]).to(DEV)
        st = prob.new_state()
        prob.lm_init(params, st)
        for _ in range(T):
            prob.lm_step(O, P, y, params, st)
        alone.append((O, P, pt.state_from_tensor(st)))
    batch = pt.Batch(probs, device=DEV)
    Os = [c64(p["O0"]) for p in probs]
    Ps = [c64(p["P0"]) for p in probs]
    ys = [torch.from_numpy(p["y"]).to(DEV) for p in probs]
    batch.bind(Os, Ps, ys, params, T, use_graph=True)
    status, _ = batch.solve(100, check_every=1)
    assert status == pt.PTLM_OK
    for i, (O1, P1, s1) in enumerate(alone):
        s2 = batch.state(i)
        assert s2.t == T and s2.f == s1.f and s2.sigma == s1.sigma == 0.0
        assert torch.equal(Os[i], O1) and torch.equal(Ps[i], P1)


def test_batch_alternating_equals_alone():
    """The alternating update (alg:alt_LM_ptycho) in a batch: each problem's active block,
    damping pair and per-block warm starts live in its own device state, so the batch equals
    its problems solved alone."""
    print("case batch alternating", flush=True)
    probs = make_problems()[:4]
    params = pt.default_params(scaling=1, precond=1, cg_max=6, alternate=1)
    T = 3
    alone = [run_single(p, params, T) for p in probs]
    batch = pt.Batch(probs, device=DEV)
    Os = [c64(p["O0"]) for p in probs]
    Ps = [c64(p["P0"]) for p in probs]
    ys = [torch.from_numpy(p["y"]).to(DEV) for p in probs]
    batch.bind(Os, Ps, ys, params, T, use_graph=True)
    status, _ = batch.solve(200, check_every=2)
    torch.cuda.synchronize()
    assert status == pt.PTLM_OK
    for i, (O1, P1, s1) in enumerate(alone):
        s2 = batch.state(i)
        assert s2.t == T and s1.t == T and s2.block == s1.block == 1
        assert s2.f == s1.f and s2.mu == s1.mu and s2.mu_alt == s1.mu_alt and s2.products == s1.products
        assert torch.equal(Os[i], O1) and torch.equal(Ps[i], P1)


def test_batch_mixed_ggn_equals_alone():
    """Problems with the intensity-based GGN (App. C) and the magnitude-based one in one batch:
    the batched kernels read each problem's GGN kind, so the batch equals them solved alone."""
    print("case batch mixed ggn", flush=True)
    probs = make_problems()[:4]
    for i, p in enumerate(probs):
        p["ggn"] = "intensity" if i % 2 == 0 else "magnitude"
    params = pt.default_params(scaling=1, precond=1, cg_max=6)
    T = 3
    alone = []
    for p in probs:
        prob = pt.Problem(p["obj_shape"], p["probe_shape"], p["positions"], mode="joint", device=DEV, ggn=p["ggn"],
                          seg_len=p.get("seg_len", 0))
        O, P = c64(p["O0"]), c64(p["P0"])
        y = torch.from_numpy(p["y"]).to(DEV)
        st = prob.new_state()
        prob.lm_init(params, st)
        for _ in range(T):
            prob.lm_step(O, P, y, params, st)
        alone.append((O, P, pt.state_from_tensor(st)))
    batch = pt.Batch(probs, device=DEV)
    Os = [c64(p["O0"]) for p in probs]
    Ps = [c64(p["P0"]) for p in probs]
    ys = [torch.from_numpy(p["y"]).to(DEV) for p in probs]
    batch.bind(Os, Ps, ys, params, T, use_graph=True)
    status, _ = batch.solve(100, check_every=1)
    assert status == pt.PTLM_OK
    for i, (O1, P1, s1) in enumerate(alone):
        s2 = batch.state(i)
        assert s2.t == T and s2.f == s1.f and s2.products == s1.products
        assert torch.equal(Os[i], O1) and torch.equal(Ps[i], P1)


@pytest.mark.parametrize("precond", [3, 4])
def test_batch_exact_and_stochastic_diagonal_equal_alone(precond):
    """The exact GGN diagonal (precond 3) and its stochastic estimate (precond 4, the sign
    fields drawn from the outer iteration) as Jacobi diagonals in a batch: every problem's
    diagonal comes from its own launches, so the batch equals its problems solved alone."""
    print("case batch diagonal precond", precond, flush=True)
    probs = make_problems()[:4]
    params = pt.default_params(scaling=1, precond=precond, cg_max=5, stoch_samples=3, stoch_seed=5)
    T = 3
    alone = [run_single(p, params, T) for p in probs]
    batch = pt.Batch(probs, device=DEV)
    Os = [c64(p["O0"]) for p in probs]
    Ps = [c64(p["P0"]) for p in probs]
    ys = [torch.from_numpy(p["y"]).to(DEV) for p in probs]
    batch.bind(Os, Ps, ys, params, T, use_graph=True)
    status, _ = batch.solve(100, check_every=2)
    torch.cuda.synchronize()
    assert status == pt.PTLM_OK
    for i, (O1, P1, s1) in enumerate(alone):
        s2 = batch.state(i)
        print("problem %d: f %.6e / %.6e products %d / %d" % (i, s1.f, s2.f, s1.products, s2.products))
        assert s2.t == T and s1.t == T
        assert s2.f == s1.f and s2.products == s1.products and s2.attempts == s1.attempts
        assert torch.equal(Os[i], O1) and torch.equal(Ps[i], P1)


@pytest.mark.parametrize("gamma", [1e-6, 0.0])
def test_batch_projected_equals_alone(gamma):
    """alg:projected_LM in a batch: the plug-in (projection, Armijo line search, choice of the
    iterate) is decided on the device per problem, so the batch equals its problems alone,
    and every object stays in |O| <= 1.  gamma = 0 sends every accepted step through the
    line search."""
    print("case batch projected gamma", gamma, flush=True)
    probs = make_problems()[:4]
    params = pt.default_params(scaling=1, precond=1, cg_max=6, project=1, gamma=gamma)
    T = 4
    alone = [run_single(p, params, T) for p in probs]
    batch = pt.Batch(probs, device=DEV)
    Os = [c64(p["O0"]) for p in probs]
    Ps = [c64(p["P0"]) for p in probs]
    ys = [torch.from_numpy(p["y"]).to(DEV) for p in probs]
    batch.bind(Os, Ps, ys, params, T, use_graph=True)
    status, _ = batch.solve(200, check_every=2)
    torch.cuda.synchronize()
    assert status == pt.PTLM_OK
    for i, (O1, P1, s1) in enumerate(alone):
        s2 = batch.state(i)
        print("problem %d: f %.6e / %.6e branch %d / %d alpha %g / %g" % (i, s1.f, s2.f, s1.ls_branch, s2.ls_branch,
                                                                          s1.ls_alpha, s2.ls_alpha))
        assert s2.t == T and s1.t == T
        assert s2.f == s1.f and s2.products == s1.products and s2.ls_branch == s1.ls_branch
        assert s2.ls_alpha == s1.ls_alpha
        assert torch.equal(Os[i], O1) and torch.equal(Ps[i], P1)
        assert float(torch.abs(Os[i]).max()) <= 1.0 + 1e-6
        if gamma == 0.0:
            assert s2.ls_branch != 0


def test_batch_with_large_probes_equals_alone():
    """128 x 128 and 256 x 256 probes in a batch (their batched kernels read the metric per
    pixel and, at 256 x 256, stage through per-workgroup transform tiles) next to a small
    problem: every problem equals its solve alone, bit for bit."""
    print("case batch large probes", flush=True)
    out = []
    for side, probe, n, step, seed in ((200, (128, 128), 3, 32, 21), (320, (256, 256), 2, 48, 22), (72, (32, 32), 5, 8, 23)):
        rng = np.random.default_rng(seed)
        O = synth.make_object(rng, side, amp=(0.7, 1.0), phase=(-np.pi, np.pi), phase_sigma=3.0,
                              phase_source="gaussian")
        P = synth.make_probe_fresnel(rng, probe[0], 0.3 * probe[0], 5.0)
        P = synth.scale_probe_to_photons(P, O, 3e3)
        base = 2 + step * np.arange(n)
        ry, rx = np.meshgrid(base, base, indexing="ij")
        pos = np.stack([ry.ravel(), rx.ravel()], 1) + rng.integers(-1, 2, size=(n * n, 2))
        pos = np.clip(pos, 0, [side - probe[0], side - probe[1]]).astype(np.int32)
        y = synth.poisson_counts(rng, ptycho.intensity(O, P, pos, 1e-8)).astype(np.float32)
        out.append(dict(obj_shape=(side, side), probe_shape=probe, positions=pos, mode="joint", y=y,
                        O0=synth.random_object_guess(rng, side), P0=np.abs(P)))
    params = pt.default_params(scaling=1, precond=1, cg_max=5)
    T = 2
    alone = [run_single(p, params, T) for p in out]
    batch = pt.Batch(out, device=DEV)
    Os = [c64(p["O0"]) for p in out]
    Ps = [c64(p["P0"]) for p in out]
    ys = [torch.from_numpy(p["y"]).to(DEV) for p in out]
    batch.bind(Os, Ps, ys, params, T, use_graph=True)
    status, _ = batch.solve(100, check_every=1)
    torch.cuda.synchronize()
    assert status == pt.PTLM_OK
    for i, (O1, P1, s1) in enumerate(alone):
        s2 = batch.state(i)
        print("problem %d (probe %s): f %.6e / %.6e" % (i, out[i]["probe_shape"], s1.f, s2.f))
        assert s2.t == T and s1.t == T
        assert s2.f == s1.f and s2.products == s1.products and s2.attempts == s1.attempts
        assert torch.equal(Os[i], O1) and torch.equal(Ps[i], P1)
