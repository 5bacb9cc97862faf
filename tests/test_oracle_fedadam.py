"""Pins for the oracle's GCP-FedAdam round (Alg. gcp-fed-iter) on the CPU.

With epsilon negligible, one local step and the first round, both Adam
updates reduce to sign steps, which gives the round in closed form:
U_new[row] = U[row] - meta_rate * sign(mean over covering clients of
sign(G_c[row])).  A zero local rate leaves every client model equal to the
server model, so D = 0 and the server model does not move.
"""
import numpy as np

import oracle

TINY_EPS = 1e-300      # Adam's step becomes sign(G) where G != 0, and 0 where G = 0


def _client_tensor(dims, nnz, seed):
    rng = np.random.default_rng(seed)
    lin = rng.choice(int(np.prod(dims)), nnz, replace=False)
    coords = np.stack(np.unravel_index(lin, dims), axis=1).astype(np.int64)
    vals = rng.integers(1, 5, nnz).astype(np.float64)
    return oracle.SparseTensor(dims, coords, vals)


def _setup(gdims, grid, R, seed=0):
    d = len(gdims)
    bsz = [gdims[k] // grid[k] for k in range(d)]
    clients = []
    for c in range(int(np.prod(grid))):
        pos = np.unravel_index(c, grid)
        base = np.array([pos[k] * bsz[k] for k in range(d)], dtype=np.int64)
        t = _client_tensor(bsz, 6 + c, seed + c)
        rows = int(sum(bsz)) * R
        clients.append(oracle.FedClient(t, base, np.zeros(rows), np.zeros(rows), np.zeros(rows)))
    rng = np.random.default_rng(seed + 99)
    U = rng.uniform(0.5, 1.5, int(sum(gdims)) * R)
    return clients, U


def _client_rows(gdims, cl, R):
    goff = np.concatenate([[0], np.cumsum(gdims)])
    return np.concatenate([np.arange(goff[k] + cl.row_base[k], goff[k] + cl.row_base[k] + n)
                           for k, n in enumerate(cl.tensor.dims)])


def test_first_round_closed_form_sign_of_mean_sign():
    gdims, grid, R = [6, 4, 5], (2, 1, 1), 2
    clients, U = _setup(gdims, grid, R)
    U0 = U.copy()
    p = q = 8
    seed = 17
    lr, meta = 1e-3, 1e-2
    # expected: each client's first-step gradient at M_c = U restricted
    sgn_sum = np.zeros((int(sum(gdims)), R))
    for c, cl in enumerate(clients):
        rows = _client_rows(gdims, cl, R)
        Mc = U0.reshape(-1, R)[rows].reshape(-1)
        sc, sx, sw = oracle.sample_stratified(cl.tensor, p, q, seed, step=0, client=c)
        G, _ = oracle.loss_grad(cl.tensor.dims, R, Mc, sc, sx, sw, "poisson")
        sgn_sum[rows] += np.sign(G.reshape(-1, R))
    want = U0.reshape(-1, R) - meta * np.sign(sgn_sum)

    Bs = np.zeros_like(U)
    Cs = np.zeros_like(U)
    ap_c = oracle.AdamParams(lr=lr, eps=TINY_EPS)
    ap_s = oracle.AdamParams(lr=meta, eps=TINY_EPS)
    t = oracle.fedadam_round(clients, gdims, R, U, Bs, Cs, 0, 0, 1, "poisson", p, q, seed,
                             ap_c, ap_s)
    assert t == 1
    np.testing.assert_allclose(U.reshape(-1, R), want, rtol=0, atol=1e-15)
    # the averaging really mattered somewhere: a shared row with opposite signs
    assert (np.sign(sgn_sum) == 0).any() or (np.abs(sgn_sum) == 2).any()


def test_zero_local_rate_leaves_server_model_fixed():
    gdims, grid, R = [4, 6, 4], (2, 2, 1), 3
    clients, U = _setup(gdims, grid, R, seed=5)
    U0 = U.copy()
    Bs, Cs = np.zeros_like(U), np.zeros_like(U)
    oracle.fedadam_round(clients, gdims, R, U, Bs, Cs, 0, 0, 3, "poisson", 5, 5, 3,
                         oracle.AdamParams(lr=0.0), oracle.AdamParams(lr=0.1))
    np.testing.assert_array_equal(U, U0)
    for cl in clients:
        assert cl.t == 3                      # the local counters still advanced
        assert np.abs(cl.B).max() > 0         # and the local moments were updated


def test_round_resets_clients_and_keeps_their_moments():
    gdims, grid, R = [4, 4, 4], (2, 1, 2), 2
    clients, U = _setup(gdims, grid, R, seed=8)
    Bs, Cs = np.zeros_like(U), np.zeros_like(U)
    ap = oracle.AdamParams(lr=1e-2)
    st = 0
    for rnd in range(2):
        B_before = [cl.B.copy() for cl in clients]
        st = oracle.fedadam_round(clients, gdims, R, U, Bs, Cs, st, rnd, 2, "poisson", 4, 4, 1,
                                  ap, ap)
        for cl, b in zip(clients, B_before):
            assert not np.array_equal(cl.B, b)
    assert st == 2
    assert all(cl.t == 4 for cl in clients)


def test_rounds_equal_an_independent_implementation():
    """Two rounds of three local steps equal a separate implementation that
    shares only the (separately pinned) sampler with the oracle: each client
    a torch tensor with its own torch.optim.Adam (state kept across rounds,
    the model reset to the server rows each round), gradients by
    torch.autograd of the client's weighted Gaussian objective in block
    coordinates, the per-row mean of U - M_c over the covering clients, and a
    server torch.optim.Adam at the meta-rate; eps = 0 on both sides (every
    row of every block is sampled in every step here, so no second moment is
    zero).  U, every M_c and the client moments must agree."""
    import torch

    gdims, grid, R = [6, 4, 6], (2, 1, 2), 2
    clients, U = _setup(gdims, grid, R, seed=5)
    U0 = U.copy()
    p = q = 20
    seed, tau, rounds, lr, meta = 23, 3, 2, 0.05, 0.1
    cap = oracle.AdamParams(lr=lr, eps=0.0, lower=-np.inf)
    sap = oracle.AdamParams(lr=meta, eps=0.0, lower=-np.inf)
    Bs, Cs = np.zeros_like(U), np.zeros_like(U)
    st = 0
    for r in range(rounds):
        st = oracle.fedadam_round(clients, gdims, R, U, Bs, Cs, st, r, tau, "gaussian", p, q, seed, cap, sap)

    goff = np.concatenate([[0], np.cumsum(gdims)])
    Ut = torch.tensor(U0, dtype=torch.float64, requires_grad=True)
    sopt = torch.optim.Adam([Ut], lr=meta, betas=(sap.beta1, sap.beta2), eps=0.0)
    Ms, opts = [], []
    for cl in clients:
        Mc = torch.zeros(int(sum(cl.tensor.dims)) * R, dtype=torch.float64, requires_grad=True)
        Ms.append(Mc)
        opts.append(torch.optim.Adam([Mc], lr=lr, betas=(cap.beta1, cap.beta2), eps=0.0))

    def F(Mc, dims, c, x, w):
        loff = np.concatenate([[0], np.cumsum(dims)])
        M2 = Mc.view(-1, R)
        prod = torch.ones(len(x), R, dtype=torch.float64)
        for k in range(len(dims)):
            prod = prod * M2[torch.as_tensor(loff[k] + c[:, k])]
        return (torch.as_tensor(w) * 0.5 * (prod.sum(1) - torch.as_tensor(x)) ** 2).sum()

    for r in range(rounds):
        Dsum = torch.zeros(int(sum(gdims)), R, dtype=torch.float64)
        count = torch.zeros(int(sum(gdims)), dtype=torch.float64)
        for c, cl in enumerate(clients):
            rows = torch.as_tensor(_client_rows(gdims, cl, R))
            with torch.no_grad():
                Ms[c].copy_(Ut.view(-1, R)[rows].reshape(-1))
            for j in range(tau):
                sc, sx, sw = oracle.sample_stratified(cl.tensor, p, q, seed, step=r * tau + j, client=c)
                opts[c].zero_grad()
                F(Ms[c], cl.tensor.dims, sc, sx, sw).backward()
                assert torch.count_nonzero(Ms[c].grad).item() == Ms[c].numel()
                opts[c].step()
            with torch.no_grad():
                Dsum[rows] += Ut.view(-1, R)[rows] - Ms[c].view(-1, R)
                count[rows] += 1
        Ut.grad = (Dsum / count[:, None]).reshape(-1)
        sopt.step()

    np.testing.assert_allclose(Ut.detach().numpy(), U, rtol=1e-10, atol=1e-13)
    for c, cl in enumerate(clients):
        np.testing.assert_allclose(Ms[c].detach().numpy(), cl.M, rtol=1e-10, atol=1e-13)
        state = opts[c].state[Ms[c]]
        np.testing.assert_allclose(state["exp_avg"].numpy(), cl.B, rtol=1e-10, atol=1e-15)
        np.testing.assert_allclose(state["exp_avg_sq"].numpy(), cl.C, rtol=1e-10, atol=1e-15)
    assert st == rounds and all(cl.t == rounds * tau for cl in clients)
    assert np.abs(U - U0).max() > 1e-3                     # the server model moved
