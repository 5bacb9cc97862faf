"""Pins of the oracle's GCP-Adam epoch driver (CPU): the safeguard of the
paper's experiments (Sec. 5) -- an epoch that does not lower the objective on
the fixed sample set is undone and the rate is multiplied by the decay; the run
stops after max_fails such epochs -- checked through properties that hold
whatever the arithmetic: a zero rate can never lower the objective, an
exploding rate is undone bit for bit, and small steps on a smooth objective are
accepted with a strictly decreasing objective."""
import numpy as np

import oracle
from paper_2605_20353_amd import synth


def _problem(seed=3):
    dims, R = [9, 8, 7], 3
    data = synth.count_tensor(dims, R, 120, seed=seed)
    t = oracle.SparseTensor(dims, data.coords.numpy(), data.vals.numpy())
    A0 = synth.init_model(dims, R, seed + 1).numpy()
    return t, dims, R, A0


def _run(t, R, A0, lr, decay=0.1, max_epochs=6, iters=5):
    return oracle.gcp_adam_epochs(t, R, A0, "poisson", 40, 40, 200, 200, iters, max_epochs, lr, decay, 3,
                                  seed=11, obj_client=1 << 62, ap=oracle.AdamParams(lower=0.0))


def test_zero_rate_is_undone_three_times_then_stops():
    t, dims, R, A0 = _problem()
    A, objs, rates, fails = _run(t, R, A0, lr=0.0)
    assert fails == 3 and rates == [0.0, 0.0, 0.0]
    assert len(objs) == 1                          # only the initial objective
    np.testing.assert_array_equal(A, A0.reshape(-1))


def test_exploding_rate_is_undone_exactly_and_decayed():
    t, dims, R, A0 = _problem(seed=5)
    A, objs, rates, fails = _run(t, R, A0, lr=50.0, decay=0.5, max_epochs=2)
    # both epochs move the factors far from the data: undone, rate halved
    assert rates == [50.0, 25.0] and fails == 2 and len(objs) == 1
    np.testing.assert_array_equal(A, A0.reshape(-1))


def test_small_steps_are_accepted_and_lower_the_objective():
    t, dims, R, A0 = _problem(seed=7)
    A, objs, rates, fails = _run(t, R, A0, lr=1e-3, max_epochs=3)
    assert fails == 0 and rates == [1e-3] * 3 and len(objs) == 4
    assert all(b < a for a, b in zip(objs, objs[1:]))
    assert np.abs(A - A0.reshape(-1)).max() > 0


def test_epochs_equal_an_independent_implementation():
    """The whole trajectory -- objectives of the accepted epochs, the rate of
    every epoch, the undone epochs and the final model -- equals a separate
    implementation that shares only the (separately pinned) sampler with the
    oracle: gradients by torch.autograd of the weighted Gaussian objective,
    torch.optim.Adam with eps = 0 (where its update is Alg. adam-update's;
    every factor row is sampled in every iteration on this 3 x 3 x 3 tensor,
    so no second moment is zero), and the restore-and-decay loop of the
    paper's experiments written out here with optimizer state snapshots."""
    import copy

    import torch

    dims, R = [3, 3, 3], 2
    data = synth.count_tensor(dims, R, 10, seed=21)
    t = oracle.SparseTensor(dims, data.coords.numpy(), data.vals.numpy())
    A0 = (0.3 + synth.init_model(dims, R, 22)).numpy()
    p = q = 30
    obj_p = obj_q = 100
    iters, max_epochs, lr, decay, max_fails, seed, oc = 4, 8, 4.0, 0.5, 3, 13, 1 << 62
    ap = oracle.AdamParams(eps=0.0, lower=-np.inf)
    A_o, objs_o, rates_o, fails_o = oracle.gcp_adam_epochs(t, R, A0, "gaussian", p, q, obj_p, obj_q, iters,
                                                           max_epochs, lr, decay, max_fails, seed=seed,
                                                           obj_client=oc, ap=ap)

    offs = np.cumsum([0] + dims)
    A = torch.tensor(A0.reshape(-1), dtype=torch.float64, requires_grad=True)

    def F(c, x, w):
        M = A.view(sum(dims), R)
        prod = torch.ones(len(x), R, dtype=torch.float64)
        for k in range(len(dims)):
            prod = prod * M[torch.as_tensor(offs[k] + c[:, k])]
        m = prod.sum(1)
        return (torch.as_tensor(w) * 0.5 * (m - torch.as_tensor(x)) ** 2).sum()

    def objective():
        c, x, w = oracle.sample_stratified(t, obj_p, obj_q, seed, 0, oc)
        with torch.no_grad():
            return float(F(c, x, w))

    opt = torch.optim.Adam([A], lr=lr, betas=(ap.beta1, ap.beta2), eps=0.0)
    f_prev = objective()
    objs, rates, fails, it, rate = [f_prev], [], 0, 0, lr
    for _ in range(max_epochs):
        saved = (A.detach().clone(), copy.deepcopy(opt.state_dict()))
        for _ in range(iters):
            c, x, w = oracle.sample_stratified(t, p, q, seed, it, 0)
            it += 1
            opt.zero_grad()
            F(c, x, w).backward()
            assert torch.count_nonzero(A.grad).item() == A.numel()
            opt.step()
        f = objective()
        rates.append(rate)
        if f < f_prev:
            f_prev = f
            objs.append(f)
        else:
            with torch.no_grad():
                A.copy_(saved[0])
            opt.load_state_dict(saved[1])
            rate *= decay
            for g in opt.param_groups:
                g["lr"] = rate
            fails += 1
            if fails >= max_fails:
                break
    assert fails == fails_o and rates == rates_o
    assert 0 < fails < max_fails and len(rates) == max_epochs   # epochs undone, decayed, then accepted again
    assert len(objs) == len(objs_o) > 1
    np.testing.assert_allclose(objs, objs_o, rtol=1e-10)
    np.testing.assert_allclose(A.detach().numpy(), A_o, rtol=1e-9, atol=1e-12)
