"""The learned selector's network on the device against the FP64 oracle MLP
(forward, loss, gradients; the oracle itself is pinned to central finite
differences in the CPU tests), plus the Adam step and the host inference."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

NI, NH, NO = 10, 32, 2


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build()
    from paper_2010_10131_amd import api as a
    return a


def unpack(p):
    o = 0
    W1 = p[o:o + NH * NI].reshape(NI, NH).T; o += NH * NI
    b1 = p[o:o + NH]; o += NH
    W2 = p[o:o + NH * NH].reshape(NH, NH).T; o += NH * NH
    b2 = p[o:o + NH]; o += NH
    W3 = p[o:o + NO * NH].reshape(NH, NO).T; o += NO * NH
    b3 = p[o:o + NO]; o += NO
    mu = p[o:o + NI]; o += NI
    isd = p[o:o + NI]
    return [W1, W2, W3], [b1, b2, b3], mu, isd


def rand_params(seed):
    rng = np.random.default_rng(seed)
    n = NH * NI + NH + NH * NH + NH + NO * NH + NO + 2 * NI
    p = (rng.standard_normal(n) * 0.3).astype(np.float32)
    p[-2 * NI:-NI] = rng.standard_normal(NI).astype(np.float32)            # mu
    p[-NI:] = (0.5 + rng.random(NI)).astype(np.float32)                    # inverse std
    return p


def test_param_count(api):
    assert api.selector_num_params() == NH * NI + NH + NH * NH + NH + NO * NH + NO + 2 * NI
    assert api.selector_num_trainable() == api.selector_num_params() - 2 * NI


@pytest.mark.parametrize("B", [1, 7, 300, 2049])
def test_forward_and_gradients_match_oracle(api, B):
    import torch
    p = rand_params(B)
    rng = np.random.default_rng(100 + B)
    X = rng.standard_normal((NI, B)).astype(np.float32)
    T = rng.standard_normal((NO, B)).astype(np.float32)
    pd = torch.from_numpy(p).cuda()
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).cuda().t()     # 10 x B column-major
    Td = torch.from_numpy(np.ascontiguousarray(T.T)).cuda().t()
    Y = api.mlp_forward(pd, Xd).cpu().numpy()
    loss, grad = api.mlp_loss_grad(pd, Xd, Td)
    loss, grad = float(loss.item()), grad.cpu().numpy()
    Ws, bs, mu, isd = unpack(p.astype(np.float64))
    Xn = (X.astype(np.float64) - mu[:, None]) * isd[:, None]
    Yo = oracle.mlp_forward(Ws, bs, Xn)
    np.testing.assert_allclose(Y, Yo, rtol=1e-5, atol=1e-5 * np.abs(Yo).max())
    lo, dW, db = oracle.mlp_loss_grad(Ws, bs, Xn, T.astype(np.float64))
    assert abs(loss - lo) <= 1e-5 * lo
    go = np.concatenate([dW[0].T.ravel(), db[0], dW[1].T.ravel(), db[1], dW[2].T.ravel(), db[2],
                         np.zeros(2 * NI)])
    scale = np.abs(go).max()
    np.testing.assert_allclose(grad, go, rtol=0, atol=2e-5 * scale)


def test_adam_step(api):
    import torch
    rng = np.random.default_rng(1)
    n = 64
    w = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    wd, gd, md, vd = (torch.from_numpy(a.copy()).cuda() for a in (w, g, m, v))
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    for step in (1, 2, 3):
        api.mlp_adam(wd, gd, md, vd, n, lr, step, b1, b2, eps)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        w = w - lr * (m / (1 - b1 ** step)) / (np.sqrt(v / (1 - b2 ** step)) + eps)
    np.testing.assert_allclose(wd.cpu().numpy(), w, rtol=1e-6, atol=1e-6)


def test_host_inference_matches_device(api):
    import torch
    p = rand_params(9)
    shapes = [(64, 8, 4096), (512, 64, 262144), (160, 16, 4096000), (48, 8, 110592)]
    feats = np.stack([api.selector_features(*s) for s in shapes], axis=1)
    ref = np.log(np.array([[I, R, J, I * I, R * R, I * R, R * R / I, R * R / J, I / J, R / J]
                           for I, R, J in shapes], dtype=np.float64)).T
    np.testing.assert_allclose(feats, ref, rtol=1e-6, atol=1e-6)
    Xd = torch.from_numpy(np.ascontiguousarray(feats.T)).cuda().t()
    Yd = api.mlp_forward(torch.from_numpy(p).cuda(), Xd).cpu().numpy()
    for k, s in enumerate(shapes):
        np.testing.assert_allclose(api.selector_predict(*s, weights=p), Yd[:, k], rtol=1e-5, atol=1e-5)


def test_auto_takes_eig_above_the_rank_bound(api):
    """(64, 2, 2) with ranks (5, 2, 2) under either selector: mode 1 runs EIG
    (ALS would meet singular normal equations) and matches the oracle."""
    import torch
    X = wl.lowrank_plus_noise((64, 2, 2), (4, 2, 2), "none", 1e-3, 3, "float64")
    for solver in ("auto", "auto_tree"):
        G, U, _ = api.sthosvd(api.to_device(X), (5, 2, 2), "fp64", "fp64", solver=solver)
        Go, Uo, _ = oracle.sthosvd(X, (5, 2, 2))
        Xh = oracle.reconstruct(api.to_numpy(G), [api.to_numpy(u) for u in U])
        assert np.linalg.norm(Xh - oracle.reconstruct(Go, Uo)) <= 1e-12 * np.linalg.norm(X)
