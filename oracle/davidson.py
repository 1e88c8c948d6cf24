"""Block Davidson eigensolver for the lowest bands of H(k), FP64.

The paper's solver is "Davidson with overlap", modelled on Quantum ESPRESSO's,
which needs only repeated products H|psi> on trial blocks and treats H as a
Hermitian black box (Sec. 5, 'dft' module).  The paper gives no further
steps; this is the standard block Davidson (Davidson 1975; Liu 1978) in the
reading used throughout this project:

  1. V = orthonormalised start block (two CholQR passes); HV = H V.
  2. Rayleigh-Ritz: H_s = V^H H V (Hermitian part), eigenpairs (theta, Y),
     lowest nbnd kept.
  3. X = V Y, HX = HV Y, residuals r_n = HX_n - theta_n X_n.  With lazy (the default, as
     the GPU solve does it) only the rows of the bands being corrected in this iteration are
     formed; the others keep their earlier X, HX and residual norm until a restart or a
     convergence verdict needs them, when they are formed from the same V, HV and Y.
  4. Converged when max_n ||r_n||_2 <= tol (Ha), with every band's residual formed from
     the current Ritz vectors.
  5. Unconverged bands give corrections t_n(G) = K(x_G) r_n(G) (Teter, Payne and
     Allan 1989), x_G = (1/2|k+G|^2) / T_n with T_n = <X_n|T|X_n> the band's
     kinetic energy, normalised to unit length.
  6. If the basis would exceed max_basis columns (default 4 nbnd): restart with
     V = X, HV = HX.
  7. Orthogonalise t against V (two block classical Gram-Schmidt passes), then
     CholQR twice; append to V, append H t to HV; go to 2.

Every call returns eigenvalues (ascending), Ritz vectors, residual norms and the
iteration count; the basis is kept orthonormal, so the projected problem is a
standard Hermitian one (S_s = I to rounding).
"""
import numpy as np


def teter(x):
    """Teter-Payne-Allan preconditioning factor K(x)."""
    x = np.asarray(x, np.float64)
    num = 27.0 + x * (18.0 + x * (12.0 + 8.0 * x))
    return num / (num + 16.0 * x ** 4)


def cholqr(t):
    """Rows of t -> orthonormal rows spanning the same space (one CholQR pass)."""
    g = t.conj() @ t.T                    # g[a,b] = <t_a|t_b>
    g = 0.5 * (g + g.conj().T)
    l = np.linalg.cholesky(g)             # g = L L^H
    linv = np.linalg.inv(l)
    return linv.conj() @ t


def orthonormalise(t, v=None):
    """Two CGS passes against the rows of v, then two CholQR passes."""
    t = np.array(t, np.complex128)
    if v is not None and v.shape[0]:
        for _ in range(2):
            c = v.conj() @ t.T            # c[i,n] = <v_i|t_n>
            t = t - c.T @ v
    for _ in range(2):
        t = cholqr(t)
    return t


def rayleigh_ritz(v, hv, nbnd):
    theta, y = ritz_pairs(v, hv, nbnd)
    return theta, y.T @ v, y.T @ hv


def ritz_pairs(v, hv, nbnd):
    """Lowest nbnd eigenpairs (theta, Y) of the projected matrix V^H H V."""
    hs = v.conj() @ hv.T                  # hs[i,j] = <v_i|H v_j>
    hs = 0.5 * (hs + hs.conj().T)
    theta, y = np.linalg.eigh(hs)
    return theta[:nbnd], y[:, :nbnd]


def band_kinetic(x, kin):
    """<x|T|x> / <x|x> per row."""
    p = np.abs(x) ** 2
    return (p * kin[None, :]).sum(1) / p.sum(1)


def teter_precondition(r, x, kin):
    """t_n = K(T(G)/T_n) r_n, normalised; T_n the kinetic energy of Ritz vector x_n."""
    tn = band_kinetic(x, kin)
    t = teter(kin[None, :] / tn[:, None]) * r
    return t / np.linalg.norm(t, axis=1, keepdims=True)


def davidson_ref(apply_h, x0, kin, tol=1e-8, max_iter=200, max_basis=None,
                 precond=None, history=None, lazy=True):
    """Lowest x0.shape[0] eigenpairs of the Hermitian operator ``apply_h``.

    apply_h  callable [m, npw] -> [m, npw]
    x0       start block [nbnd, npw]
    kin      1/2|k+G|^2 [npw] (for the Teter preconditioner)
    precond  optional callable (r [n, npw], theta [n], x [n, npw]) -> t [n, npw];
             default Teter with the band kinetic energy
    history  optional list; receives (iteration, max residual, n_unconverged)
    lazy     form X, HX and residuals only for the bands being corrected (step 3)
    Returns dict(eig, x, resnorm, iterations, n_hpsi, converged).
    """
    nb = x0.shape[0]
    mb = 4 * nb if max_basis is None else int(max_basis)
    v = orthonormalise(x0)
    hv = apply_h(v)
    n_hpsi = v.shape[0]
    it = 0
    theta, y = ritz_pairs(v, hv, nb)
    x, hx = y.T @ v, y.T @ hv
    r = hx - theta[:, None] * x
    rn = np.linalg.norm(r, axis=1)
    stale = np.zeros(nb, bool)            # rows of x, hx, r, rn older than (theta, y)

    def complete(resid):
        x[stale] = y[:, stale].T @ v
        hx[stale] = y[:, stale].T @ hv
        if resid:
            r[stale] = hx[stale] - theta[stale, None] * x[stale]
            rn[stale] = np.linalg.norm(r[stale], axis=1)
        stale[:] = False

    while True:
        unconv = np.nonzero(rn > tol)[0]
        if unconv.size == 0 and stale.any():   # a verdict needs every band's residual
            complete(True)
            unconv = np.nonzero(rn > tol)[0]
        if history is not None:
            history.append((it, float(rn.max()), int(unconv.size)))
        if unconv.size == 0 or it >= max_iter:
            if stale.any():
                complete(True)
            return dict(eig=theta, x=x, resnorm=rn, iterations=it, n_hpsi=n_hpsi,
                        converged=bool((rn <= tol).all()))
        if precond is None:
            t = teter_precondition(r[unconv], x[unconv], kin)
        else:
            t = precond(r[unconv], theta[unconv], x[unconv])
        if v.shape[0] + unconv.size > mb:
            if stale.any():
                complete(False)
            v, hv = x.copy(), hx.copy()
        t = orthonormalise(t, v)
        ht = apply_h(t)
        n_hpsi += t.shape[0]
        v = np.concatenate([v, t])
        hv = np.concatenate([hv, ht])
        it += 1
        theta, y = ritz_pairs(v, hv, nb)
        upd = unconv if lazy else np.arange(nb)
        x[upd] = y[:, upd].T @ v
        hx[upd] = y[:, upd].T @ hv
        r[upd] = hx[upd] - theta[upd, None] * x[upd]
        rn[upd] = np.linalg.norm(r[upd], axis=1)
        stale[:] = True
        stale[upd] = False
