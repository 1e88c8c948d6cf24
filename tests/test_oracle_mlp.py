"""Pins for the learned-preconditioner oracle: finite differences, special cases, Adam."""
import numpy as np

from oracle import davidson as dav, mlp


def _data(seed=0, nb=3, npw=40):
    rng = np.random.default_rng(seed)
    kin = rng.uniform(0, 4, npw)
    r = rng.standard_normal((nb, npw)) + 1j * rng.standard_normal((nb, npw))
    delta = rng.standard_normal((nb, npw)) + 1j * rng.standard_normal((nb, npw))
    theta = rng.uniform(-0.5, 0.5, nb)
    tkin = rng.uniform(0.5, 1.5, nb)
    f = mlp.features(kin, r, theta, tkin).reshape(-1, 5)
    ptr = np.arange(nb + 1) * npw
    return f, r.reshape(-1), delta.reshape(-1), ptr


def test_features_hand_example(golden):
    """The five input features on a 3-G, 2-band example evaluated by hand
    (tests/golden/mlp_features_hand.txt): x = T(G)/T_n, log(1 + x), (theta_n - T_n)/T_n,
    |r_n(G)| sqrt(npw)/||r_n|| and T(G).  A log written for log1p, a missing sqrt(npw), a
    residual normalised by its square norm or x inverted each fail."""
    g = golden("mlp_features_hand.txt")
    kin = np.array(g["kin"])
    r = np.array([np.array(g["r0_re"]) + 1j * np.array(g["r0_im"]),
                  np.array(g["r1_re"]) + 1j * np.array(g["r1_im"])])
    f = mlp.features(kin, r, np.array(g["theta"]), np.array(g["tkin"]))
    assert f.shape == (2, 3, 5)
    for n in range(2):
        for q in range(3):
            np.testing.assert_allclose(f[n, q], g[f"f{n}_{q}"], rtol=1e-15, atol=1e-15)
    # the teter factor of the network's gain uses the same x as the Davidson's Teter step
    np.testing.assert_allclose(mlp.teter_factor(f[..., 0]), dav.teter(f[..., 0]), rtol=1e-15)


def test_gradient_matches_finite_differences():
    f, r, d, ptr = _data()
    w = mlp.init_weights(3)
    w[-256 - 2:] = np.random.default_rng(1).standard_normal(258) * 0.3   # non-trivial W2, b2
    L, g = mlp.loss_grad(w, f, r, d, ptr)
    assert abs(L - mlp.loss(w, f, r, d, ptr)) < 1e-14
    rng = np.random.default_rng(2)
    idx = rng.choice(mlp.NPARAM, 40, replace=False)
    for i in idx:
        h = 1e-6
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (mlp.loss(wp, f, r, d, ptr) - mlp.loss(wm, f, r, d, ptr)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_zero_output_layer_is_teter():
    """W2 = 0, b2 = 0: g = K(x) (Teter, Payne and Allan), so t = K(x) r; the loss is the
    cosine loss of the Teter correction, written out with np.vdot."""
    f, r, d, ptr = _data(4)
    w = mlp.init_weights(0)
    x = f[:, 0]
    num = 27 + 18 * x + 12 * x ** 2 + 8 * x ** 3
    kx = num / (num + 16 * x ** 4)
    np.testing.assert_allclose(mlp.forward(w, f), np.stack([kx, np.zeros_like(kx)], -1), rtol=1e-15)
    exp = 0.0
    for b in range(len(ptr) - 1):
        s = slice(ptr[b], ptr[b + 1])
        t = kx[s] * r[s]
        exp += 1 - abs(np.vdot(t, d[s])) ** 2 / (np.linalg.norm(t) ** 2 * np.linalg.norm(d[s]) ** 2)
    assert abs(mlp.loss(w, f, r, d, ptr) - exp / (len(ptr) - 1)) < 1e-14


def test_gain_is_bounded_around_teter():
    """Whatever the weights, e^-2 K(x) <= Re g <= e^2 K(x) and |Im g| <= K(x)/2."""
    f, r, d, ptr = _data(8)
    w = np.random.default_rng(9).standard_normal(mlp.NPARAM) * 3.0
    g = mlp.forward(w, f)
    kx = mlp.teter_factor(f[:, 0])
    assert np.all(g[:, 0] >= np.exp(-2) * kx * (1 - 1e-12)) and np.all(g[:, 0] <= np.exp(2) * kx * (1 + 1e-12))
    assert np.all(np.abs(g[:, 1]) <= 0.5 * kx * (1 + 1e-12))


def test_loss_is_phase_and_scale_free():
    f, r, d, ptr = _data(5)
    w = mlp.init_weights(1)
    L0 = mlp.loss(w, f, r, d, ptr)
    assert abs(mlp.loss(w, f, r, d * (2.5 * np.exp(0.7j)), ptr) - L0) < 1e-13
    # a gain proportional to delta/r gives zero loss
    assert abs(mlp.loss(w, f, r, r * 3j, ptr) - mlp.loss(w, f, r, r, ptr)) < 1e-13
    # the loss is invariant under a common phase of r and delta
    assert abs(mlp.loss(w, f, r * np.exp(0.3j), d * np.exp(0.3j), ptr) - L0) < 1e-13


def test_adam_first_step():
    """After one step the bias-corrected update is lr * g / (|g| + eps)."""
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    w1, m, v = mlp.adam_step(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    np.testing.assert_allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_correction_target():
    rng = np.random.default_rng(6)
    q, _ = np.linalg.qr(rng.standard_normal((30, 6)) + 1j * rng.standard_normal((30, 6)))
    xs = q.T                                  # 6 orthonormal rows
    eig = np.array([0.0, 1.0, 1.0, 2.0, 3.0, 4.0])  # rows 1, 2 degenerate
    assert np.abs(mlp.correction_target(xs[:3], xs, eig)).max() < 1e-14
    # x_1 tilted into the degenerate partner only: still exact (no correction needed)
    x = np.cos(0.3) * xs[1] + np.sin(0.3) * xs[2]
    assert np.abs(mlp.correction_target(np.stack([xs[0], x]), xs, eig)[1]).max() < 1e-14
    # tilted toward a non-degenerate level: target points back to the level
    y = np.cos(0.2) * xs[3] + np.sin(0.2) * xs[4]
    dlt = mlp.correction_target(np.stack([xs[0], xs[1], xs[2], y]), xs, eig)[3]
    np.testing.assert_allclose(dlt, xs[3] - y, atol=1e-14)
