"""Pins of the learned-preconditioner oracle (oracle/net.py) and of flexible
CG against things other than themselves: a site-by-site convolution, the
adjoint (dot-product) identities of the backward pass, central finite
differences of the loss, exact shift and identity kernels, the closed form of
the first Adam step, and flexible CG reducing to CG / one step / PCG for the
identity, the exact inverse and a fixed HPD preconditioner."""
import numpy as np
import pytest

import oracle as O
from oracle import net as NN
from oracle import precond as PC
from paper_2508_16298_amd import inputs


def _rand(shape, seed):
    return np.random.default_rng(seed).normal(size=shape)


@pytest.mark.parametrize("anti", [None, [False, True, False]])
def test_conv_matches_site_by_site(anti):
    X = _rand((3, 3, 4, 4), 1)
    W = _rand((2, 3, 27), 2)
    b = _rand(2, 3)
    a = None if anti is None else np.array(anti)
    assert np.allclose(NN.conv(X, W, b, a), NN.conv_bruteforce(X, W, b, a), atol=1e-12, rtol=0)


def test_single_tap_kernels_shift_the_input():
    """A kernel that is 1 on one tap and channel copies the input shifted by
    that tap, with the sign flip on wrapped antiperiodic channels."""
    Nt, L = 4, 4
    X = _rand((2, Nt, L, L), 4)
    anti = np.array([False, True])
    for k, (dt, dy, dx) in enumerate(NN.TAPS):
        W = np.zeros((2, 2, 27))
        W[0, 0, k] = 1.0
        W[1, 1, k] = 1.0
        out = NN.conv(X, W, np.zeros(2), anti)
        for t in range(Nt):
            ts = t + dt
            wrap = ts < 0 or ts >= Nt
            for y in range(L):
                for x in range(L):
                    src = X[:, ts % Nt, (y + dy) % L, (x + dx) % L]
                    assert out[0, t, y, x] == src[0]
                    assert out[1, t, y, x] == (-src[1] if wrap else src[1])
    assert NN.TAPS[13] == (0, 0, 0)


def test_conv_backward_adjoint_identities():
    """<dOut, conv(X, W, 0)> = <dX, X> = <dW, W> (the convolution is bilinear)."""
    X = _rand((3, 5, 4, 4), 5)
    W = _rand((4, 3, 27), 6)
    G = _rand((4, 5, 4, 4), 7)
    anti = np.array([True, False, True])
    y = np.sum(G * NN.conv(X, W, np.zeros(4), anti))
    dX, dW, db = NN.conv_backward(X, W, G, anti)
    assert abs(np.sum(dX * X) - y) <= 1e-11 * abs(y)
    assert abs(np.sum(dW * W) - y) <= 1e-11 * abs(y)
    assert np.allclose(db, G.sum(axis=(1, 2, 3)))


def test_silu_derivative():
    a = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (NN.silu(a + h) - NN.silu(a - h)) / (2 * h)
    assert np.abs(fd - NN.dsilu(a)).max() < 1e-9


def _small_net(seed):
    return inputs.net_init_weights(seed, ch=(6, 4, 4, 2))


def test_loss_gradients_match_finite_differences():
    L, Nt = 4, 4
    th = inputs.hot_start_theta(L, Nt, 11)
    r = inputs.gauss_cvec(L, Nt, 12)
    e = inputs.gauss_cvec(L, Nt, 13)
    params = _small_net(14)
    params = [(W, _rand(W.shape[0], 15 + l) * 0.1) for l, (W, _) in enumerate(params)]
    loss, grads = NN.loss_and_grads(params, th, r, e)
    rng = np.random.default_rng(16)
    h = 1e-6
    for l in range(len(params)):
        W, b = params[l]
        for _ in range(4):
            idx = tuple(rng.integers(0, n) for n in W.shape)
            Wp, Wm = W.copy(), W.copy()
            Wp[idx] += h
            Wm[idx] -= h
            pp = list(params); pp[l] = (Wp, b)
            pm = list(params); pm[l] = (Wm, b)
            fd = (NN.loss_and_grads(pp, th, r, e)[0] - NN.loss_and_grads(pm, th, r, e)[0]) / (2 * h)
            assert abs(fd - grads[l][0][idx]) <= 1e-6 * max(1.0, abs(fd)), (l, idx, fd, grads[l][0][idx])
        j = rng.integers(0, b.size)
        bp, bm = b.copy(), b.copy()
        bp[j] += h
        bm[j] -= h
        pp = list(params); pp[l] = (W, bp)
        pm = list(params); pm[l] = (W, bm)
        fd = (NN.loss_and_grads(pp, th, r, e)[0] - NN.loss_and_grads(pm, th, r, e)[0]) / (2 * h)
        assert abs(fd - grads[l][1][j]) <= 1e-6 * max(1.0, abs(fd))


def test_residual_loss_gradients_match_finite_differences():
    """The residual-form loss |O z - r|^2 / |r|^2 (O = M^dag M from the
    plain C oracle) against central finite differences of the same loss, and
    its value against the triple form's error measured through O: for e with
    O e = r it is |O (z - e)|^2 / |O e|^2."""
    L, Nt = 4, 4
    p = O.lat(L, Nt)
    th = inputs.hot_start_theta(L, Nt, 21)
    r = inputs.gauss_cvec(L, Nt, 22)
    apply_O = lambda v: O.apply_MdagM(p, th, v).reshape(Nt, L, L)
    params = _small_net(24)
    params = [(W, _rand(W.shape[0], 25 + l) * 0.1) for l, (W, _) in enumerate(params)]
    loss, grads = NN.loss_and_grads_residual(params, th, r, apply_O)
    e = np.linalg.solve(O.dense_MdagM(p, th), r.reshape(-1)).reshape(Nt, L, L)
    z = NN.forward(params, th, r)
    Oe = apply_O(e)
    assert abs(loss - np.linalg.norm(apply_O(z - e)) ** 2 / np.linalg.norm(Oe) ** 2) <= 1e-10 * loss
    f = lambda q: NN.loss_and_grads_residual(q, th, r, apply_O)[0]
    rng = np.random.default_rng(26)
    h = 1e-6
    for l in range(len(params)):
        W, b = params[l]
        for _ in range(3):
            idx = tuple(rng.integers(0, n) for n in W.shape)
            Wp, Wm = W.copy(), W.copy()
            Wp[idx] += h
            Wm[idx] -= h
            pp = list(params); pp[l] = (Wp, b)
            pm = list(params); pm[l] = (Wm, b)
            fd = (f(pp) - f(pm)) / (2 * h)
            assert abs(fd - grads[l][0][idx]) <= 1e-6 * max(1.0, abs(fd)), (l, idx, fd, grads[l][0][idx])
        j = rng.integers(0, b.size)
        bp, bm = b.copy(), b.copy()
        bp[j] += h
        bm[j] -= h
        pp = list(params); pp[l] = (W, bp)
        pm = list(params); pm[l] = (W, bm)
        fd = (f(pp) - f(pm)) / (2 * h)
        assert abs(fd - grads[l][1][j]) <= 1e-6 * max(1.0, abs(fd))


def test_network_translation_covariance():
    """Spatial translations commute with the network.  A shift by one slice
    in tau (theta periodic, r antiperiodic) shifts the output exactly on the
    slices whose receptive field (+-1 slice per layer) does not cross the
    wrap, for either configuration."""
    L, Nt = 4, 16
    th = inputs.hot_start_theta(L, Nt, 21)
    r = inputs.gauss_cvec(L, Nt, 22)
    params = inputs.net_init_weights(23, ch=(6, 4, 4, 4, 4, 4, 2))
    z = NN.forward(params, th, r)
    z3 = NN.forward(params, np.roll(th, (1, 2), axis=(2, 3)), np.roll(r, (1, 2), axis=(1, 2)))
    assert np.allclose(z3, np.roll(z, (1, 2), axis=(1, 2)), atol=1e-12)
    th2 = np.roll(th, 1, axis=1)
    r2 = np.roll(r, 1, axis=0)
    r2[0] *= -1
    z2 = NN.forward(params, th2, r2)
    depth = len(params)
    for t in range(Nt):
        inside = t - depth >= 1 and t + depth <= Nt - 1
        if inside:
            assert np.allclose(z2[t], z[t - 1], atol=1e-12), t


def test_network_scale_equivariance():
    """z(theta, c r) = c z(theta, r) for c > 0 (input normalised by |r|)."""
    L, Nt = 4, 3
    th = inputs.hot_start_theta(L, Nt, 31)
    r = inputs.gauss_cvec(L, Nt, 32)
    params = _small_net(33)
    assert np.allclose(NN.forward(params, th, 7.5 * r), 7.5 * NN.forward(params, th, r), rtol=1e-12)


def test_first_adam_step_closed_form():
    W = _rand((3, 2, 27), 41)
    b = _rand(3, 42)
    gW = _rand(W.shape, 43)
    gb = _rand(b.shape, 44)
    params, grads = [(W, b)], [(gW, gb)]
    newp, st = NN.adam_step(params, grads, NN.adam_init(params), lr=1e-2)
    # t = 1: m_hat = g, v_hat = g^2  =>  step = -lr g / (|g| + eps)
    assert np.allclose(newp[0][0], W - 1e-2 * gW / (np.abs(gW) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(newp[0][1], b - 1e-2 * gb / (np.abs(gb) + 1e-8), rtol=0, atol=1e-15)
    assert st[0] == 1


def _system(L, Nt, seed):
    p = O.lat(L, Nt)
    th = inputs.noisy_pi_flux_theta(L, Nt, 0.3, seed)
    R = inputs.gauss_cvec(L, Nt, seed + 1)
    eta = O.apply_M(p, th, R, dagger=True).reshape(Nt, L, L)
    Ofn = lambda v: O.apply_MdagM(p, th, v).reshape(Nt, L, L)
    return p, th, eta, Ofn


def test_fcg_identity_preconditioner_is_cg():
    p, th, eta, Ofn = _system(4, 8, 51)
    x, ok, it, rel, sw = NN.fcg_solve(Ofn, lambda r: r.copy(), eta, tol=1e-10)
    xo, sto, ito, relo = O.cg_solve(p, th, eta, tol=1e-10)
    assert ok and rel <= 1e-10 and sw == -1
    assert abs(it - ito) <= 1
    xd = np.linalg.solve(O.dense_MdagM(p, th), eta.reshape(-1))
    assert np.linalg.norm(x.reshape(-1) - xd) <= 1e-8 * np.linalg.norm(xd)


def test_fcg_exact_inverse_converges_in_one_step():
    p, th, eta, Ofn = _system(4, 6, 61)
    A = O.dense_MdagM(p, th)
    inv = lambda r: np.linalg.solve(A, r.reshape(-1)).reshape(r.shape)
    x, ok, it, rel, sw = NN.fcg_solve(Ofn, inv, eta, tol=1e-10)
    assert ok and it == 1


def test_fcg_with_fixed_hpd_preconditioner_matches_pcg():
    """With the paper's (linear, HPD) preconditioner flexible CG is PCG."""
    p, th, eta, Ofn = _system(8, 16, 71)
    taps, _ = PC.build_stencil(L0=8, Nt0=16, cap=4)
    P = lambda r: PC.apply_P(taps, r)
    x, ok, it, rel, sw = NN.fcg_solve(Ofn, P, eta, tol=1e-10)
    xo, sto, ito, relo = O.cg_solve(p, th, eta, tol=1e-10, maxit=2000,
                                    precond=lambda r: P(r.reshape(eta.shape)).reshape(-1))
    assert ok and abs(it - ito) <= 2, (it, ito)


def test_fcg_judge_falls_back_from_an_untrained_network():
    """A random (untrained) network is a useless preconditioner: the
    residual judge hands the solve to the fallback after the window, and the
    solve still reaches the tolerance and the dense solution."""
    p, th, eta, Ofn = _system(4, 6, 81)
    params = _small_net(82)
    x, ok, it, rel, sw = NN.fcg_solve(Ofn, lambda r: NN.forward(params, th, r), eta, tol=1e-10, maxit=2000)
    assert ok and rel <= 1e-10
    assert sw >= NN.JUDGE_WINDOW + 1
    xd = np.linalg.solve(O.dense_MdagM(p, th), eta.reshape(-1))
    assert np.linalg.norm(x.reshape(-1) - xd) <= 1e-7 * np.linalg.norm(xd)
