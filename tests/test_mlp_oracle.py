"""Pins of the learned-guess oracle (oracle/mlp.py) against things it does not
compute itself: central finite differences of its own forward pass, closed
forms, and the features recomputed from the full ERI tensor and NumPy norms."""
import dataclasses

import numpy as np
import pytest
from scipy.special import expit

from oracle import ccsd as occ
from oracle import integrals
from oracle import mlp
from synth import make_fragment


def _random_model(H, rng, scale=0.5):
    F = mlp.NFEAT
    return mlp.Model(mu=rng.normal(size=F), inv_sigma=rng.uniform(0.5, 2.0, F),
                     y_mu=0.1, y_sigma=0.7,
                     W1=rng.normal(scale=scale, size=(H, F)), b1=rng.normal(scale=scale, size=H),
                     W2=rng.normal(scale=scale, size=(H, H)), b2=rng.normal(scale=scale, size=H),
                     W3=rng.normal(scale=scale, size=(H, H)), b3=rng.normal(scale=scale, size=H),
                     w4=rng.normal(scale=scale, size=H), b4=0.3)


def test_silu_and_derivative():
    z = np.linspace(-8, 8, 101)
    np.testing.assert_allclose(mlp.silu(z), z * expit(z), rtol=1e-14, atol=1e-15)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.dsilu(z), fd, rtol=1e-8, atol=1e-9)
    assert mlp.silu(0.0) == 0.0 and mlp.dsilu(0.0) == 0.5


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(7)
    m = _random_model(6, rng)
    X = rng.normal(size=(11, mlp.NFEAT))
    t = rng.normal(size=11)
    L0, g = mlp.loss_and_grad(m, X, t)
    h = 1e-6
    for name in mlp.Model.PARAMS:
        val = getattr(m, name)
        if np.isscalar(val):
            mp = dataclasses.replace(m, **{name: val + h})
            mm = dataclasses.replace(m, **{name: val - h})
            fd = (mlp.loss_and_grad(mp, X, t)[0] - mlp.loss_and_grad(mm, X, t)[0]) / (2 * h)
            assert abs(getattr(g, name) - fd) < 1e-7 * max(1.0, abs(fd)), name
            continue
        gv = getattr(g, name)
        for idx in list(np.ndindex(val.shape))[:: max(1, val.size // 17)]:
            vp, vm = val.copy(), val.copy()
            vp[idx] += h
            vm[idx] -= h
            Lp = mlp.loss_and_grad(dataclasses.replace(m, **{name: vp}), X, t)[0]
            Lm = mlp.loss_and_grad(dataclasses.replace(m, **{name: vm}), X, t)[0]
            fd = (Lp - Lm) / (2 * h)
            assert abs(gv[idx] - fd) < 1e-7 * max(1.0, abs(fd)), (name, idx)
    assert L0 > 0


def test_zero_network_outputs_its_last_bias():
    rng = np.random.default_rng(1)
    m = _random_model(5, rng)
    for k in ("W1", "W2", "W3", "w4"):
        setattr(m, k, np.zeros_like(getattr(m, k)))
    X = rng.normal(size=(4, mlp.NFEAT))
    y, _ = mlp.forward(m, X)
    np.testing.assert_array_equal(y, np.full(4, m.b4))
    np.testing.assert_allclose(mlp.predict_correction(m, X), m.y_mu + m.y_sigma * m.b4)


def test_blob_layout_round_trip():
    rng = np.random.default_rng(2)
    m = _random_model(256, rng, scale=0.01)
    blob = mlp.pack(m)
    assert blob.size == mlp.HEADER + mlp.n_params(256) == 64 + 136256
    m2 = mlp.unpack(blob.astype(np.float32), 256)
    np.testing.assert_allclose(m2.W2, m.W2, rtol=1e-6, atol=1e-9)
    assert abs(m2.b4 - m.b4) < 1e-7
    # W1 sits right after the header, b4 right after w4
    assert blob[64] == m.W1[0, 0] and blob[64 + 4096] == m.b1[0]
    assert blob[64 + 136192] == m.b4


def test_adam_first_step_is_lr_times_sign():
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    m1, m2 = np.zeros(3), np.zeros(3)
    mlp.adam_step(p, g, m1, m2, step=1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(p, [0.99, -1.99, 2.99], rtol=0, atol=1e-15)


def test_adam_constant_gradient_moves_lr_per_step():
    """With the same gradient at every step the bias-corrected moments are
    exactly g and g^2, so each Adam step moves every parameter by lr against
    the sign of its gradient (eps = 0), whatever the gradient's size.  A wrong
    bias-correction exponent or decay rate breaks this from step 2 on."""
    p0 = np.array([1.0, -2.0, 3.0, 0.5, -0.25])
    g = np.array([0.5, -4.0, 1e-3, 7e2, -3e-5])
    p = p0.copy()
    m1, m2 = np.zeros(5), np.zeros(5)
    lr = 0.01
    for t in range(1, 8):
        mlp.adam_step(p, g, m1, m2, step=t, lr=lr, eps=0.0)
        np.testing.assert_allclose(p, p0 - t * lr * np.sign(g), rtol=0, atol=1e-13)
        np.testing.assert_allclose(m1 / (1 - 0.9 ** t), g, rtol=1e-13)
        np.testing.assert_allclose(m2 / (1 - 0.999 ** t), g * g, rtol=1e-12)


def test_adam_alternating_gradient_closed_form():
    """Gradient +g, -g, +g, ...: m1_t = (1 - b1) g sum_s b1^(t-s) (-1)^(s-1)
    = (1 - b1) g (b1^t - (-1)^t) / (b1 + 1) (geometric series) and m2_t = g^2 (1 - b2^t)."""
    b1, b2, lr, eps = 0.9, 0.999, 1e-3, 1e-8
    g0 = np.array([0.3, -2.0, 5e-4])
    p = np.zeros(3)
    m1, m2 = np.zeros(3), np.zeros(3)
    expect = np.zeros(3)
    for t in range(1, 7):
        mlp.adam_step(p, g0 * (-1) ** (t - 1), m1, m2, step=t, lr=lr)
        m1t = (1 - b1) * g0 * (b1 ** t - (-1) ** t) / (b1 + 1)
        m2t = g0 * g0 * (1 - b2 ** t)
        expect -= lr * (m1t / (1 - b1 ** t)) / (np.sqrt(m2t / (1 - b2 ** t)) + eps)
        np.testing.assert_allclose(p, expect, rtol=1e-12, atol=1e-18)


def test_splitmix64_reference_outputs():
    """First outputs of the splitmix64 generator started from state 0 (the
    published reference sequence): the state advances by the golden gamma
    0x9E3779B97F4A7C15 and each output is the mixing function of the state."""
    gamma = 0x9E3779B97F4A7C15
    out = [mlp.splitmix64((k * gamma) & mlp.MASK64) for k in range(4)]
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F,
                   0xF88BB8A8724C81EC]
    rows = mlp.minibatch_rows(seed=7, step=3, batch=1000, n=37)
    assert rows.min() >= 0 and rows.max() < 37 and len(set(rows.tolist())) == 37


def test_first_training_step_is_lr_times_gradient_sign():
    """Step 1 of the oracle's training loop moves each parameter by
    -lr g / (|g| + eps), with g the gradient on the rows minibatch_rows draws."""
    rng = np.random.default_rng(8)
    m = _random_model(256, rng, scale=0.05)
    blob = mlp.pack(m)
    X = rng.normal(size=(300, 16))
    Y = rng.normal(size=300) * 0.1
    b1, _, _, losses = mlp.train(blob, X, Y, step0=0, nsteps=1, batch=64, lr=1e-3, seed=5)
    rows = mlp.minibatch_rows(5, 1, 64, 300)
    L, g = mlp.loss_and_grad(m, X[rows], Y[rows])
    gv = mlp.gradient_vector(m, g)
    np.testing.assert_allclose(b1[mlp.HEADER:] - blob[mlp.HEADER:], -1e-3 * gv / (np.abs(gv) + 1e-8),
                               rtol=1e-9, atol=1e-15)
    assert abs(losses[0] - L) < 1e-15
    np.testing.assert_array_equal(b1[:mlp.HEADER], blob[:mlp.HEADER])


def test_features_from_their_definitions():
    f = make_fragment(3, 7, 20, 11)
    o, v = 3, 7
    X = mlp.pair_features(f.B, f.eps_occ, f.eps_vir)
    eri = integrals.full_eri(f.B)
    t_mp2, _ = occ.mp2(f.B, f.eps_occ, f.eps_vir)
    np.testing.assert_allclose(X[..., 0], t_mp2, rtol=1e-13, atol=1e-16)
    for (i, j, a, b) in [(0, 1, 2, 5), (2, 2, 6, 6), (1, 0, 0, 3)]:
        A, Bv = o + a, o + b
        D = f.eps_occ[i] + f.eps_occ[j] - f.eps_vir[a] - f.eps_vir[b]
        x = X[i, j, a, b]
        assert abs(x[2] - eri[i, A, j, Bv]) < 1e-13 and abs(x[3] - eri[i, Bv, j, A]) < 1e-13
        assert abs(x[1] - eri[i, Bv, j, A] / D) < 1e-12 and abs(x[5] - D) < 1e-14
        assert abs(x[4] * D - 1) < 1e-14
        ei, ej, ea, eb = f.eps_occ[i], f.eps_occ[j], f.eps_vir[a], f.eps_vir[b]
        assert tuple(x[6:10]) == (ei + ej, abs(ei - ej), ea + eb, abs(ea - eb))
        nia = np.linalg.norm(f.B[:, i, A])
        njb = np.linalg.norm(f.B[:, j, Bv])
        nib, nja = np.linalg.norm(f.B[:, i, Bv]), np.linalg.norm(f.B[:, j, A])
        assert abs(x[10] - nia * njb) < 1e-13 and abs(x[11] - nib * nja) < 1e-13
        assert x[12] == (i == j) and x[13] == (a == b)
        assert abs(x[14] - (eri[i, i, A, A] + eri[j, j, Bv, Bv])) < 1e-13
        assert abs(x[15] - (eri[i, i, Bv, Bv] + eri[j, j, A, A])) < 1e-13


def test_amplitude_symmetry_of_features():
    """t_ij^ab = t_ji^ba: the features of (i,j,a,b) and (j,i,b,a) are equal, so
    any model predicts a guess with that symmetry."""
    f = make_fragment(2, 5, 12, 3)
    X = mlp.pair_features(f.B, f.eps_occ, f.eps_vir)
    Xs = X.transpose(1, 0, 3, 2, 4)
    np.testing.assert_allclose(X, Xs, rtol=1e-13, atol=1e-15)


@pytest.mark.slow
def test_exact_t2_start_saves_no_iterations():
    """What a T2-only starting guess can gain here: with T1 = 0, even the exact
    converged T2 takes as many iterations as the MP2 start (the T1 build-up and
    its coupling set the pace), while the exact pair (T1, T2) converges at
    once.  Bounds the learned start's iteration gain on these inputs."""
    f = make_fragment(6, 45, 120, 8000)
    ref = occ.ccsd(f.B, f.eps_occ, f.eps_vir, conv_tol=1e-10)
    assert ref.converged
    exact_t2 = occ.ccsd(f.B, f.eps_occ, f.eps_vir, conv_tol=1e-10, t1=np.zeros_like(ref.t1),
                        t2=ref.t2)
    both = occ.ccsd(f.B, f.eps_occ, f.eps_vir, conv_tol=1e-10, t1=ref.t1, t2=ref.t2)
    assert exact_t2.n_iter >= ref.n_iter - 1
    assert both.n_iter <= 2
    assert abs(exact_t2.e_ccsd - ref.e_ccsd) < 1e-9
