"""Data generation for the inverse problem (oracle; test infrastructure only).

The paper makes its model data with Algorithm 1 (Section 3): the fixed point
U_{n+1} = U_0 + omega^2 int G~ F[xi F^-1 U_n] dz' of eq. (6), followed by
eq. (7) for W. The fixed point converges for small omega only (Section 3,
closing remark); this oracle solves the same second-kind equation,
u - omega^2 K(xi u) = u0 in X (the first line of system (2)), with BiCGSTAB
(van der Vorst's stabilized biconjugate gradients) and then applies the data
operator to v = xi u (eq. 3, second line of eq. 7). A plain fixed-point
variant is kept for comparison with the paper's Algorithm 1.

Parity: pinned by tests/test_oracle_forward.py (dense direct solve on tiny
grids, residual invariants, agreement of the fixed point where it converges).
"""
from __future__ import annotations

import numpy as np

from . import model


def ls_operator(p, f, xi):
    """u -> u - omega^2 K(xi u) on X's grid (flattened)."""
    shape = (p.nz, p.ny, p.nx)

    def apply(u):
        u3 = u.reshape(shape)
        return (u3 - model.volume_potential(p, f, xi * u3)).ravel()

    return apply


def bicgstab(apply, b, tol=1e-12, maxit=500):
    """Solve apply(x) = b; stop when ||b - apply(x)|| <= tol ||b||.
    Returns (x, iterations, relative residual)."""
    x = np.zeros_like(b)
    r = b - apply(x)
    bn = np.linalg.norm(b)
    if bn == 0:
        return x, 0, 0.0
    rhat = r.copy()
    rho_old = alpha = omega = 1.0 + 0j
    vv = np.zeros_like(b)
    pp = np.zeros_like(b)
    for it in range(1, maxit + 1):
        rho = np.vdot(rhat, r)
        beta = (rho / rho_old) * (alpha / omega)
        pp = r + beta * (pp - omega * vv)
        vv = apply(pp)
        alpha = rho / np.vdot(rhat, vv)
        s = r - alpha * vv
        if np.linalg.norm(s) <= tol * bn:
            x = x + alpha * pp
            return x, it, np.linalg.norm(b - apply(x)) / bn
        t = apply(s)
        omega = np.vdot(t, s) / np.vdot(t, t)
        x = x + alpha * pp + omega * s
        r = s - omega * t
        rho_old = rho
        if np.linalg.norm(r) <= tol * bn:
            return x, it, np.linalg.norm(b - apply(x)) / bn
    return x, maxit, np.linalg.norm(b - apply(x)) / bn


def total_field(p, f, xi, u0_f, tol=1e-12, maxit=500):
    """u in X solving u = u0 + omega^2 K(xi u) (system (2), first line)."""
    x, it, res = bicgstab(ls_operator(p, f, xi), u0_f.ravel(), tol, maxit)
    return x.reshape(u0_f.shape), it, res


def fixed_point_field(p, f, xi, u0_f, tol=1e-13, maxit=500):
    """The paper's Algorithm 1 iteration in the space domain: u_{n+1} =
    u0 + omega^2 K(xi u_n), stopped when ||u_n - u_{n-1}|| <= tol ||u0||."""
    u = u0_f.copy()
    n0 = np.linalg.norm(u0_f)
    for it in range(1, maxit + 1):
        un = u0_f + model.volume_potential(p, f, xi * u)
        if np.linalg.norm(un - u) <= tol * n0:
            return un, it
        u = un
    return u, maxit


def synthesize(p, xi, u0, born=False, tol=1e-12, maxit=500, zconv=False):
    """Noise-free data W (n_omega, nd, py, px) and the fields (u, v) in X.

    born=True replaces the total field by the incident field (u = u0);
    zconv=True applies the data operator by the z-convolution route
    (model.data_operator_zconv; data planes on X's z-lattice only)."""
    nf = p.n_omega
    W = np.empty((nf, p.nd, p.py, p.px), np.complex128)
    U = np.empty((nf, p.nz, p.ny, p.nx), np.complex128)
    info = []
    for f in range(nf):
        if born:
            u, it, res = u0[f], 0, 0.0
        else:
            u, it, res = total_field(p, f, xi, u0[f], tol, maxit)
        U[f] = u
        op = model.data_operator_zconv if zconv else model.data_operator
        W[f] = op(p, f, xi * u)
        info.append((it, res))
    return W, U, xi[None] * U, info
