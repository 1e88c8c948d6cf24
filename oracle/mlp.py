"""Learned residual -> correction preconditioner, FP64 reference (test infrastructure).

Not in the paper: the learned preconditioner is this project's extension of the
paper's Davidson (Sec. 5, 'dft' module).  The network acts per plane wave G
and band n with shared weights, so it does not depend on the basis size:

    f(G, n) = [x, log(1 + x), (theta_n - T_n) / T_n, |r_n(G)| sqrt(npw) / ||r_n||, 1/2|k+G|^2]
              x = (1/2|k+G|^2) / T_n,  T_n = <x_n|T|x_n> the band kinetic energy
    h = silu(W1 f + b1)             W1 [128, 5], b1 [128]
    o = W2 h + b2                   W2 [2, 128], b2 [2]
    g = K(x) [exp(2 tanh o_0) + 0.5 i tanh o_1]      K = Teter-Payne-Allan factor
    t_n(G) = g(G, n) r_n(G)

The network only reshapes the Teter preconditioner, by a real factor within
[e^-2, e^2] and a small imaginary part; with a zero output layer it is Teter
exactly, which is both its starting point and its fallback.

t is invariant in form under a global phase of r (g depends on phase-free inputs).
Training target: the direction delta_n the Ritz vector still has to move, with
the per-band scale- and phase-free loss

    L = (1 / nbands) sum_n [1 - |<t_n, delta_n>|^2 / (||t_n||^2 ||delta_n||^2)].

Parameter vector layout (float64 here, float32 on the GPU): W1 (row-major),
b1, W2 (row-major), b2 -> 128*5 + 128 + 2*128 + 2 = 1026 numbers.
Parity pins: finite differences of the loss, the zero-output-layer case (g = Teter's
K(x), loss written out with np.vdot), the bounds on g, Adam's published update rule.
"""
import numpy as np

NIN, NHID = 5, 128
NPARAM = NHID * NIN + NHID + 2 * NHID + 2


def unpack(w):
    w = np.asarray(w, np.float64)
    o = 0
    W1 = w[o:o + NHID * NIN].reshape(NHID, NIN); o += NHID * NIN
    b1 = w[o:o + NHID]; o += NHID
    W2 = w[o:o + 2 * NHID].reshape(2, NHID); o += 2 * NHID
    b2 = w[o:o + 2]
    return W1, b1, W2, b2


def pack(W1, b1, W2, b2):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2])


def init_weights(seed=0):
    """Random hidden layer, zero output layer: the untrained network is the Teter gain."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W1 = rng.standard_normal((NHID, NIN)) * np.sqrt(1.0 / NIN)
    b1 = np.zeros(NHID)
    return pack(W1, b1, np.zeros((2, NHID)), np.zeros(2))


def teter_factor(x):
    num = 27.0 + x * (18.0 + x * (12.0 + 8.0 * x))
    return num / (num + 16.0 * x ** 4)


def features(kin, r, theta, tkin):
    """kin [npw]; r [nb, npw] complex; theta, tkin [nb] -> [nb, npw, 5]."""
    kin = np.asarray(kin, np.float64)
    x = kin[None, :] / tkin[:, None]
    rn = np.linalg.norm(r, axis=1)
    amp = np.abs(r) * np.sqrt(r.shape[1]) / rn[:, None]
    f = np.stack([x, np.log1p(x), np.broadcast_to(((theta - tkin) / tkin)[:, None], x.shape), amp,
                  np.broadcast_to(kin[None, :], x.shape)], -1)
    return f


def silu(z):
    return z / (1.0 + np.exp(-z))


def forward(w, f):
    """f [..., 5] -> gain [..., 2] (re, im)."""
    W1, b1, W2, b2 = unpack(w)
    h = silu(f @ W1.T + b1)
    o = h @ W2.T + b2
    k = teter_factor(f[..., 0])
    return np.stack([k * np.exp(2.0 * np.tanh(o[..., 0])), k * 0.5 * np.tanh(o[..., 1])], -1)


def loss(w, f, r, delta, band_ptr):
    """Mean over bands of 1 - cos^2(t, delta); rows grouped by band_ptr (row offsets)."""
    g = forward(w, f)
    t = (g[:, 0] + 1j * g[:, 1]) * r
    tot = 0.0
    nb = len(band_ptr) - 1
    for b in range(nb):
        s = slice(band_ptr[b], band_ptr[b + 1])
        a = np.vdot(t[s], delta[s])
        tot += 1.0 - abs(a) ** 2 / (np.vdot(t[s], t[s]).real * np.vdot(delta[s], delta[s]).real)
    return tot / nb


def loss_grad(w, f, r, delta, band_ptr):
    """Loss and its gradient with respect to the 1026 parameters (explicit backprop)."""
    W1, b1, W2, b2 = unpack(w)
    z = f @ W1.T + b1
    sg = 1.0 / (1.0 + np.exp(-z))
    h = z * sg
    o = h @ W2.T + b2
    k = teter_factor(f[:, 0])
    th0, th1 = np.tanh(o[:, 0]), np.tanh(o[:, 1])
    e0 = np.exp(2.0 * th0)
    g = np.stack([k * e0, k * 0.5 * th1], -1)
    t = (g[:, 0] + 1j * g[:, 1]) * r
    nb = len(band_ptr) - 1
    dt = np.zeros_like(t)
    tot = 0.0
    for b in range(nb):
        s = slice(band_ptr[b], band_ptr[b + 1])
        a = np.vdot(t[s], delta[s])              # sum conj(t) delta
        tt = np.vdot(t[s], t[s]).real
        dd = np.vdot(delta[s], delta[s]).real
        c = abs(a) ** 2 / (tt * dd)
        tot += 1.0 - c
        # d|a|^2/dt (as d/du + i d/dv) = 2 conj(a) delta ; d tt/dt = 2 t
        dc = 2.0 * np.conj(a) * delta[s] / (tt * dd) - abs(a) ** 2 * 2.0 * t[s] / (tt * tt * dd)
        dt[s] = -dc / nb
    # t = g r:  dL/dg_re = Re(conj(dt) r), dL/dg_im = -Im(conj(dt) r)
    q = np.conj(dt) * r
    dgain = np.stack([q.real, -q.imag], -1)
    # through g_re = k exp(2 tanh o0), g_im = 0.5 k tanh o1
    dg = np.stack([dgain[:, 0] * k * e0 * 2.0 * (1.0 - th0 ** 2),
                   dgain[:, 1] * k * 0.5 * (1.0 - th1 ** 2)], -1)
    dW2 = dg.T @ h
    db2 = dg.sum(0)
    dh = dg @ W2
    dz = dh * (sg * (1.0 + z * (1.0 - sg)))
    dW1 = dz.T @ f
    db1 = dz.sum(0)
    return tot / nb, pack(dW1, db1, dW2, db2)


def adam_step(w, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma and Ba 2015): biased moments, bias-corrected step."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def correction_target(x, xstar, eig_star, cluster_tol=1e-6):
    """delta_n = P_n x_n / ||P_n x_n|| - x_n, P_n the projector on the converged eigenvectors
    whose eigenvalues lie within cluster_tol of eig_star[n] (degenerate levels)."""
    nb = x.shape[0]
    out = np.empty_like(x)
    c = xstar.conj() @ x.T                         # c[m, n] = <x*_m | x_n>
    for n in range(nb):
        sel = np.abs(eig_star - eig_star[n]) <= cluster_tol
        p = (c[sel, n][:, None] * xstar[sel]).sum(0)
        out[n] = p / np.linalg.norm(p) - x[n]
    return out
