"""Oracle of the learned preconditioner and of flexible CG.  TEST
INFRASTRUCTURE ONLY: nothing in the product imports this module.

What is computed (FP64, numpy, plain loops over the 27 taps):

Network N(theta, r) -> z, a stack of six 3x3x3 convolutions over the
(tau, y, x) lattice with channel counts 6 -> 32 -> 32 -> 32 -> 32 -> 32 -> 2
and the SiLU activation a * sigmoid(a) after every layer but the last.
  input channels  cos th_x, sin th_x, cos th_y, sin th_y (th_d = theta[d] at
                  the site: the bond leaving the site along +d), Re rh, Im rh
                  with rh = r / s, s = |r| / sqrt(N)
  padding         periodic in x and y; in tau periodic for every channel
                  except the two residual channels of the first layer, which
                  change sign when they wrap (the fermion vectors are
                  antiperiodic in tau)
  output          z = s * (o_0 + i o_1), o the last layer's two channels
Layer l: out[co, n] = b[co] + sum_{ci, k} W[co, ci, k] in~[ci, n + d_k],
k = (dt + 1) * 9 + (dy + 1) * 3 + (dx + 1) over dt, dy, dx in {-1, 0, 1}.

Training loss for one triple (theta, r, e) with e the solution of
O e = r (O = M^dag M): |z - e|^2 / |e|^2; or in residual form
|O z - r|^2 / |r|^2 = |O (z - e)|^2 / |O e|^2, which needs no e; Adam
(Kingma and Ba 2015).

Flexible CG (Golub and Ye 1999; Notay 2000) with a nonlinear preconditioner:
  r0 = rhs, z0 = N(r0), p0 = z0
  alpha = <p, r> / <p, O p>;  x += alpha p;  r' = r - alpha O p
  z' = N(r');  beta = -<O p, z'> / <p, O p>;  p = z' + beta p
with <a, b> = a^dag b.  alpha minimises the O-norm of the error along p and
beta makes consecutive directions O-orthogonal, so the error norm falls
monotonically whatever N does.  In exact arithmetic this beta equals the
Polak-Ribiere form <r' - r, z'> / <r, z> (with r' - r = -alpha O p and
<p, r> = <z, r>), and with a fixed Hermitian positive definite N the
iteration is preconditioned CG.  It stops on the recursion's residual and
confirms with the true residual |rhs - O x| / |rhs| <= tol (restarting from
the true residual if it is not met).

The residual judges the network: when |r| has not at least halved over the
last 10 iterations (a decade per about 33 iterations: a network slower than
that loses to the paper's preconditioner as fallback), or the network's direction is not one of
descent (<p, O p> <= 0), the solve continues with the fallback preconditioner
(the paper's, or none), restarting its directions from the current residual.
"""
import numpy as np

CH = (6, 32, 32, 32, 32, 32, 2)
TAPS = [(dt, dy, dx) for dt in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def silu(a):
    return a / (1.0 + np.exp(-a))


def dsilu(a):
    s = 1.0 / (1.0 + np.exp(-a))
    return s * (1.0 + a * (1.0 - s))


def shifted(X, dt, dy, dx, anti):
    """Y[c, tau, y, x] = X~[c, tau + dt, y + dy, x + dx] with periodic x, y
    and tau periodic, times -1 on the channels flagged in ``anti`` where
    tau + dt leaves [0, Nt)."""
    Nt = X.shape[1]
    Y = np.roll(X, shift=(-dt, -dy, -dx), axis=(1, 2, 3))
    if dt != 0 and anti is not None and np.any(anti):
        tau = np.arange(Nt)
        wrap = (tau + dt < 0) | (tau + dt >= Nt)
        sign = np.where(wrap, -1.0, 1.0)[None, :, None, None]
        Y = np.where(np.asarray(anti)[:, None, None, None], Y * sign, Y)
    return Y


def unshifted(Y, dt, dy, dx, anti):
    """Adjoint of ``shifted``."""
    Nt = Y.shape[1]
    if dt != 0 and anti is not None and np.any(anti):
        tau = np.arange(Nt)
        wrap = (tau + dt < 0) | (tau + dt >= Nt)
        sign = np.where(wrap, -1.0, 1.0)[None, :, None, None]
        Y = np.where(np.asarray(anti)[:, None, None, None], Y * sign, Y)
    return np.roll(Y, shift=(dt, dy, dx), axis=(1, 2, 3))


def conv(X, W, b, anti=None):
    """X (Cin, Nt, L, L), W (Cout, Cin, 27), b (Cout,) -> (Cout, Nt, L, L)."""
    out = np.zeros((W.shape[0],) + X.shape[1:])
    for k, (dt, dy, dx) in enumerate(TAPS):
        Xs = shifted(X, dt, dy, dx, anti)
        out += np.tensordot(W[:, :, k], Xs, axes=(1, 0))
    return out + b[:, None, None, None]


def conv_backward(X, W, dOut, anti=None, need_dx=True):
    """Gradients of sum(dOut * conv(X, W, b)) w.r.t. X, W and b."""
    dW = np.zeros_like(W)
    dX = np.zeros_like(X) if need_dx else None
    for k, (dt, dy, dx) in enumerate(TAPS):
        Xs = shifted(X, dt, dy, dx, anti)
        dW[:, :, k] = np.tensordot(dOut, Xs, axes=((1, 2, 3), (1, 2, 3)))
        if need_dx:
            dX += unshifted(np.tensordot(W[:, :, k], dOut, axes=(0, 0)), dt, dy, dx, anti)
    db = dOut.sum(axis=(1, 2, 3))
    return dX, dW, db


def conv_bruteforce(X, W, b, anti=None):
    """The same convolution written site by site (tiny inputs only)."""
    Cin, Nt, L, _ = X.shape
    out = np.zeros((W.shape[0], Nt, L, L))
    for co in range(W.shape[0]):
        for t in range(Nt):
            for y in range(L):
                for x in range(L):
                    acc = b[co]
                    for k, (dt, dy, dx) in enumerate(TAPS):
                        ts = t + dt
                        sg = 1.0
                        if ts < 0 or ts >= Nt:
                            ts %= Nt
                            sg = -1.0
                        for ci in range(Cin):
                            s = sg if (anti is not None and anti[ci]) else 1.0
                            acc += W[co, ci, k] * s * X[ci, ts, (y + dy) % L, (x + dx) % L]
                    out[co, t, y, x] = acc
    return out


def features(theta, r):
    """Input channels (6, Nt, L, L) and the residual scale s."""
    N = r.size
    s = np.linalg.norm(r) / np.sqrt(N)
    rh = r / s if s > 0 else r * 0.0
    F = np.stack([np.cos(theta[0]), np.sin(theta[0]), np.cos(theta[1]), np.sin(theta[1]),
                  rh.real, rh.imag])
    return F, s


ANTI0 = np.array([False, False, False, False, True, True])


def forward(params, theta, r, keep=False):
    """z = N(theta, r); with keep, also the per-layer inputs and
    pre-activations for the backward pass."""
    F, s = features(theta, r)
    h = F
    acts, pres = [], []
    n = len(params)
    for l, (W, b) in enumerate(params):
        acts.append(h)
        a = conv(h, W, b, ANTI0 if l == 0 else None)
        pres.append(a)
        h = silu(a) if l < n - 1 else a
    z = s * (h[0] + 1j * h[1])
    if keep:
        return z, (acts, pres, s)
    return z


def loss_and_grads(params, theta, r, e):
    """Loss |z - e|^2 / |e|^2 and its gradients w.r.t. every (W, b)."""
    z, (acts, pres, s) = forward(params, theta, r, keep=True)
    ne2 = np.vdot(e, e).real
    d = z - e
    loss = np.vdot(d, d).real / ne2
    dz = 2.0 * d / ne2
    g = s * np.stack([dz.real, dz.imag])  # d loss / d o
    grads = [None] * len(params)
    n = len(params)
    for l in range(n - 1, -1, -1):
        W, _ = params[l]
        if l < n - 1:
            g = g * dsilu(pres[l])
        dX, dW, db = conv_backward(acts[l], W, g, ANTI0 if l == 0 else None, need_dx=l > 0)
        grads[l] = (dW, db)
        g = dX
    return loss, grads


def loss_and_grads_residual(params, theta, r, apply_O):
    """Residual form: loss |O z - r|^2 / |r|^2 (O = M^dag M, apply_O on arrays
    of r's shape) and its gradients; d loss / d z = 2 O (O z - r) / |r|^2
    since O is Hermitian."""
    z, (acts, pres, s) = forward(params, theta, r, keep=True)
    nr2 = np.vdot(r, r).real
    d = apply_O(z) - r
    loss = np.vdot(d, d).real / nr2
    dz = 2.0 * apply_O(d) / nr2
    return loss, _backward(params, acts, pres, s * np.stack([dz.real, dz.imag]))


def _backward(params, acts, pres, g):
    """Gradients w.r.t. every (W, b) given d loss / d (last layer's outputs)."""
    grads = [None] * len(params)
    n = len(params)
    for l in range(n - 1, -1, -1):
        W, _ = params[l]
        if l < n - 1:
            g = g * dsilu(pres[l])
        dX, dW, db = conv_backward(acts[l], W, g, ANTI0 if l == 0 else None, need_dx=l > 0)
        grads[l] = (dW, db)
        g = dX
    return grads


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (in place on new lists); state = (t, m, v)."""
    t, m, v = state
    t += 1
    newp, newm, newv = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        out = []
        for p, gp, mp, vp in ((W, gW, mW, vW), (b, gb, mb, vb)):
            mp = b1 * mp + (1 - b1) * gp
            vp = b2 * vp + (1 - b2) * gp * gp
            mh = mp / (1 - b1 ** t)
            vh = vp / (1 - b2 ** t)
            out.append((p - lr * mh / (np.sqrt(vh) + eps), mp, vp))
        newp.append((out[0][0], out[1][0]))
        newm.append((out[0][1], out[1][1]))
        newv.append((out[0][2], out[1][2]))
    return newp, (t, newm, newv)


def adam_init(params):
    z = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    return (0, z, [(np.zeros_like(W), np.zeros_like(b)) for W, b in params])


JUDGE_WINDOW = 10
JUDGE_FACTOR = 0.5


def fcg_solve(apply_O, precond, rhs, tol=1e-10, maxit=10000, fallback=None):
    """Flexible CG as in the module docstring.  apply_O, precond, fallback:
    callables on complex arrays of rhs's shape (fallback None: the identity).
    Returns (x, converged, iterations, true relative residual, iteration at
    which the fallback took over or -1)."""
    fallback = fallback if fallback is not None else (lambda v: v.copy())
    x = np.zeros_like(rhs)
    nb = np.linalg.norm(rhs)
    if nb == 0:
        return x, True, 0, 0.0, -1
    r = rhs.copy()
    it = 0
    stalls, last = 0, -1
    switched = -1
    hist = []
    while True:
        pc = precond if switched < 0 else fallback
        p = pc(r)
        just_switched = False
        while it < maxit and np.linalg.norm(r) > tol * nb:
            s = apply_O(p)
            ps = np.vdot(p, s).real
            if not ps > 0:
                if switched < 0:  # no descent direction: the network is unusable here
                    switched, just_switched = it, True
                break
            alpha = np.vdot(p, r) / ps
            x = x + alpha * p
            r = r - alpha * s
            it += 1
            hist.append(np.linalg.norm(r))
            if (switched < 0 and len(hist) > JUDGE_WINDOW
                    and hist[-1] > JUDGE_FACTOR * hist[-1 - JUDGE_WINDOW]):
                switched, just_switched = it, True
                break
            zn = pc(r)
            beta = -np.vdot(s, zn) / ps
            p = zn + beta * p
        if just_switched:
            continue
        true = np.linalg.norm(rhs - apply_O(x)) / nb
        stalls = stalls + 1 if it == last else 0
        last = it
        if true <= tol or it >= maxit or stalls >= 3:
            return x, true <= tol, it, true, switched
        r = rhs - apply_O(x)  # restart from the true residual
