"""Pins of the surrogate-network oracle: GELU identities and the library GELU,
finite-difference gradients, the first Adam step, and the POD projection."""
import numpy as np
import torch

from oracle import mlp
from workloads import mlp_init


def test_gelu_identities_and_library_value():
    z = np.linspace(-6, 6, 97)
    assert np.allclose(mlp.gelu(z) - mlp.gelu(-z), z, atol=1e-15)
    assert np.isclose(mlp.gelu_grad(np.array([0.0]))[0], 0.5)
    ref = torch.nn.functional.gelu(torch.tensor(z, dtype=torch.float64), approximate="none")
    assert np.allclose(mlp.gelu(z), ref.numpy(), rtol=1e-14, atol=1e-15)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), fd, atol=1e-8)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    params = mlp_init(3, sizes=(2, 6, 5, 4))
    params = [p + 0.1 * rng.standard_normal(p.shape) for p in params]
    X = rng.uniform(-1, 1, (7, 2))
    T = rng.standard_normal((7, 4))
    Y, cache = mlp.forward(params, X)
    grads = mlp.backward(params, cache, Y, T)
    h = 1e-6
    for k, p in enumerate(params):
        for idx in np.ndindex(p.shape):
            pp = [q.copy() for q in params]
            pm = [q.copy() for q in params]
            pp[k][idx] += h
            pm[k][idx] -= h
            fd = (mlp.loss(mlp.forward(pp, X)[0], T) - mlp.loss(mlp.forward(pm, X)[0], T)) / (2 * h)
            assert abs(fd - grads[k][idx]) < 1e-8 + 1e-6 * abs(fd)


def test_backward_matches_torch_autograd():
    rng = np.random.default_rng(1)
    params = mlp_init(5)
    X = rng.uniform(-1, 1, (16, 2))
    T = rng.standard_normal((16, 30))
    Y, cache = mlp.forward(params, X)
    grads = mlp.backward(params, cache, Y, T)
    tp = [torch.tensor(p, requires_grad=True) for p in params]
    x = torch.tensor(X)
    h = torch.nn.functional.gelu(x @ tp[0].T + tp[1])
    h = torch.nn.functional.gelu(h @ tp[2].T + tp[3])
    y = h @ tp[4].T + tp[5]
    torch.mean((y - torch.tensor(T)) ** 2).backward()
    for g, t in zip(grads, tp):
        assert np.allclose(g, t.grad.numpy(), rtol=1e-10, atol=1e-14)


def test_first_adam_step_is_signed_lr():
    rng = np.random.default_rng(2)
    params = [rng.standard_normal((3, 2)), rng.standard_normal(3)]
    grads = [rng.standard_normal((3, 2)), rng.standard_normal(3)]
    opt = mlp.Adam(params, lr=1e-3, eps=1e-8)
    new = opt.step(params, grads)
    for p, g, q in zip(params, grads, new):
        assert np.allclose(q, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_training_reduces_loss():
    rng = np.random.default_rng(3)
    X = rng.uniform(-1, 1, (64, 2))
    T = np.column_stack([np.sin(X[:, 0]), X[:, 1] ** 2, X[:, 0] * X[:, 1]])
    params = mlp_init(7, sizes=(2, 16, 16, 3))
    _, hist = mlp.train(params, X, T, epochs=300, lr=1e-2)
    assert hist[-1] < 0.1 * hist[0]


def test_pod_basis_projection_error_is_svd_tail():
    rng = np.random.default_rng(4)
    S = rng.standard_normal((50, 12)) @ np.diag(np.logspace(0, -4, 12)) @ rng.standard_normal((12, 20))
    U0, s = mlp.pod_basis(S, 5)
    assert np.allclose(U0.T @ U0, np.eye(5), atol=1e-12)
    err = np.linalg.norm(S - U0 @ (U0.T @ S))
    assert np.isclose(err, np.sqrt(np.sum(s[5:] ** 2)), rtol=1e-8)


def test_normalise_inputs_hand_values():
    """The affine map sends each range's ends to -1 and +1 and its midpoint to 0
    (values worked out by hand)."""
    mu = np.array([0.5e4, 1.25e4, 2.0e4, 0.875e4])
    lam = np.array([4.0e4, 2.5e4, 1.0e4, 1.75e4])
    X = mlp.normalise_inputs(mu, lam, (0.5e4, 2.0e4), (1.0e4, 4.0e4))
    assert X.shape == (4, 2)
    assert np.allclose(X[:, 0], [-1.0, 0.0, 1.0, -0.5], rtol=0, atol=1e-15)
    assert np.allclose(X[:, 1], [1.0, 0.0, -1.0, -0.5], rtol=0, atol=1e-15)


def test_standardise_population_deviation_and_zero_spread():
    """Per-column mean and population (ddof = 0) deviation; a constant column
    gets deviation 1 so that it maps to zeros.  Hand-computed: column 0 of
    [1, 3, 5, 7] has mean 4 and deviation sqrt(5); column 1 is constant 2."""
    C = np.array([[1.0, 2.0], [3.0, 2.0], [5.0, 2.0], [7.0, 2.0]])
    Z, mu, sd = mlp.standardise(C)
    assert np.allclose(mu, [4.0, 2.0], rtol=0, atol=1e-15)
    assert np.allclose(sd, [np.sqrt(5.0), 1.0], rtol=1e-15)
    assert np.allclose(Z[:, 0], np.array([-3.0, -1.0, 1.0, 3.0]) / np.sqrt(5.0), rtol=1e-15)
    assert np.all(Z[:, 1] == 0.0)
    # a sample (ddof = 1) deviation would give sqrt(20 / 3) instead
    assert not np.isclose(sd[0], np.sqrt(20.0 / 3.0))


def test_adam_sequence_matches_torch_optimizer():
    """Five bias-corrected Adam steps against torch.optim.Adam (a library
    implementation of the same update) on changing gradients: a wrong second
    moment or bias correction at t >= 2 shows up here, not at t = 1."""
    rng = np.random.default_rng(8)
    params = [rng.standard_normal((3, 2)), rng.standard_normal(3)]
    grads_seq = [[rng.standard_normal((3, 2)) * (t + 1), rng.standard_normal(3) / (t + 1)]
                 for t in range(5)]
    opt = mlp.Adam(params, lr=1e-2, beta1=0.8, beta2=0.95, eps=1e-6)
    tp = [torch.tensor(p, requires_grad=True) for p in params]
    topt = torch.optim.Adam(tp, lr=1e-2, betas=(0.8, 0.95), eps=1e-6)
    cur = params
    for g in grads_seq:
        cur = opt.step(cur, g)
        topt.zero_grad()
        for t, gg in zip(tp, g):
            t.grad = torch.tensor(gg)
        topt.step()
        for a, t in zip(cur, tp):
            assert np.allclose(a, t.detach().numpy(), rtol=1e-12, atol=1e-15)
